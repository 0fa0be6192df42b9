"""Pins of the oracle's discrete microscopic entropy H(f) = sum_j h_j(f_j)
(Sec. 1: h_j is the Legendre dual of the Perthame-Bouchut potential h_j^*;
potentials of Sec. 2 / Sec. 3 at a = 0).  Each pin is a fact of the
mathematics, not a retyped formula:

* at equilibrium, sum_j h_j(f^eq_j(W)) is the macroscopic entropy
  eta(W) = h |u|^2 / 2 + g h^2 / 2, and the dual variables are the entropy
  variables (g h - |u|^2 / 2, u, v) (Legendre duality of eta and eta^*);
* d h_j / d f_j = phi (Legendre duality), checked by central differences;
* at fixed conserved moments the equilibrium minimises H (Gibbs principle);
* the entropy variables of W lie in the convexity domain of the potentials
  exactly under the subcharacteristic condition (1D: lambda > |u| + sqrt(g h);
  2D: lambda > 2 (max(|u|, |v|) + sqrt(g h))), so only then is the dual of
  f^eq(W) attained at them;
* discrete H-theorem: with periodic faces and s <= 1 the relaxation is a
  convex combination and the streaming a permutation, so H never increases.
"""
import math

import numpy as np
import pytest

import oracle
from paper_1401_0427_amd import workloads as W


def _pops(P, f, dim):
    """Per-population component vectors of one node's distribution f."""
    if dim == 1:
        return [np.array([f[1 + j], f[3 + j]]) for j in range(2)]
    return [np.array([f[1 + j], f[5 + j], f[9 + j]]) for j in range(4)]


def _random_states(rng, dim, n, lam, margin=0.9):
    """Random (h, u, v) that satisfy the subcharacteristic condition with room."""
    out = []
    while len(out) < n:
        h = rng.uniform(0.3, 3.0)
        u, v = rng.uniform(-1.0, 1.0, 2)
        if dim == 1:
            v = 0.0
            if abs(u) + math.sqrt(h) < margin * lam:
                out.append((h, u, v))
        elif 2.0 * (max(abs(u), abs(v)) + math.sqrt(h)) < margin * lam:
            out.append((h, u, v))
    return out


@pytest.mark.parametrize("dim,lam", [(1, 3.0), (2, 6.0)])
def test_entropy_of_equilibrium_is_the_macroscopic_entropy(dim, lam):
    P = oracle.params(dim, 4, 4 if dim == 2 else 1, lam=lam)
    rng = np.random.default_rng(5)
    for h, u, v in _random_states(rng, dim, 40, lam):
        fe = oracle.feq(P, h, h * u, h * v)
        total = 0.0
        for j, F in enumerate(_pops(P, fe, dim)):
            ok, hj, phi = oracle.entropy_pop(P, j, F)
            assert ok
            want = [h - 0.5 * (u * u + v * v), u] + ([v] if dim == 2 else [])
            assert np.allclose(phi, want, rtol=0, atol=1e-12)
            total += hj
        eta = 0.5 * h * (u * u + v * v) + 0.5 * h * h
        assert abs(total - eta) <= 1e-13 * eta


@pytest.mark.parametrize("dim,lam", [(1, 3.0), (2, 6.0)])
def test_entropy_gradient_is_the_dual_variable(dim, lam):
    """Away from equilibrium: d h_j / d F = phi(F) (central differences)."""
    P = oracle.params(dim, 4, 4 if dim == 2 else 1, lam=lam)
    rng = np.random.default_rng(6)
    for h, u, v in _random_states(rng, dim, 8, lam):
        W0 = (h, h * u, h * v)
        fe = oracle.feq(P, *W0)
        for j, F0 in enumerate(_pops(P, fe, dim)):
            F = F0 * (1.0 + 0.05 * rng.standard_normal(F0.size))
            ok, hj, phi = oracle.entropy_pop(P, j, F)
            assert ok
            eps = 1e-6
            for k in range(F.size):
                Fp, Fm = F.copy(), F.copy()
                Fp[k] += eps
                Fm[k] -= eps
                _, hp, _ = oracle.entropy_pop(P, j, Fp)
                _, hm, _ = oracle.entropy_pop(P, j, Fm)
                assert abs((hp - hm) / (2 * eps) - phi[k]) <= 1e-6 * (1.0 + abs(phi[k]))


@pytest.mark.parametrize("dim,lam", [(1, 3.0), (2, 6.0)])
def test_equilibrium_minimises_entropy_at_fixed_moments(dim, lam):
    nx, ny = 4, (4 if dim == 2 else 1)
    P = oracle.params(dim, nx, ny, lam=lam)
    rng = np.random.default_rng(7)
    np_ = oracle.npop(dim)
    for h, u, v in _random_states(rng, dim, 10, lam):
        fe = oracle.feq(P, h, h * u, h * v)
        H0 = _node_entropy(P, fe, dim)
        comps = [[1, 2], [3, 4]] if dim == 1 else [[1, 2, 3, 4], [5, 6, 7, 8], [9, 10, 11, 12]]
        d = np.zeros(np_)
        for idx in comps:  # a perturbation with zero sum in every component
            r = rng.standard_normal(len(idx))
            d[idx] = r - r.mean()
        gains = []
        for eps in (1e-2, 5e-3):
            Hp = _node_entropy(P, fe + eps * d * h, dim)
            assert Hp > H0
            gains.append(Hp - H0)
        # second order: halving the perturbation quarters the gain
        assert 3.5 < gains[0] / gains[1] < 4.5


def _node_entropy(P, f, dim):
    """Entropy of a single-node distribution through orc_entropy on a 1-node grid."""
    P1 = oracle.params(dim, 1, 1, lam=P.lam, s=P.s, g=P.g)
    _, tot, bad = oracle.entropy(P1, np.asarray(f).reshape(-1, 1))
    assert bad == 0
    return tot


@pytest.mark.parametrize("dim", [1, 2])
def test_equilibrium_duality_holds_exactly_under_the_subcharacteristic_condition(dim):
    """The entropy variables of W lie in the convexity domain of every h_j^*
    exactly when lambda satisfies the subcharacteristic condition (1D:
    lambda > |u| + sqrt(g h); 2D: lambda > 2 (max(|u|, |v|) + sqrt(g h))).
    Inside, the dual of f^eq(W) is attained at them and H = eta(W); just
    outside, the maximiser in the domain is another point and H != eta(W)."""
    rng = np.random.default_rng(8)
    for _ in range(20):
        h = rng.uniform(0.3, 3.0)
        u, v = rng.uniform(-1.0, 1.0, 2)
        if dim == 1:
            v = 0.0
            crit = abs(u) + math.sqrt(h)
        else:
            crit = 2.0 * (max(abs(u), abs(v)) + math.sqrt(h))
        eta = 0.5 * h * (u * u + v * v) + 0.5 * h * h
        want = np.array([h - 0.5 * (u * u + v * v), u, v][: (2 if dim == 1 else 3)])
        for factor, inside in ((1.002, True), (0.998, False)):
            P = oracle.params(dim, 1, 1, lam=factor * crit)
            fe = oracle.feq(P, h, h * u, h * v)
            total, far = 0.0, 0.0
            for j, F in enumerate(_pops(P, fe, dim)):
                ok, hj, phi = oracle.entropy_pop(P, j, F)
                assert ok
                total += hj
                far = max(far, float(np.abs(phi - want).max()))
            if inside:
                assert far <= 1e-10 and abs(total - eta) <= 1e-12 * eta
            else:
                assert far > 1e-3 and abs(total - eta) > 1e-9 * eta


@pytest.mark.parametrize("s", [0.5, 1.0])
def test_discrete_h_theorem_periodic_2d(s):
    c = W.radial_dam_break_2d(48, lam=6.0, s=s)
    P = oracle.params(2, c.nx, c.ny, lam=c.lam, s=s)
    f = oracle.run(P, c.h0, c.qx0, c.qy0, 0)
    _, H, bad = oracle.entropy(P, f)
    eta0 = math.fsum((0.5 * c.h0 ** 2).ravel())
    assert bad == 0 and abs(H - eta0) <= 1e-12 * eta0
    Hs = [H]
    for _ in range(60):
        f = oracle.advance(P, f, 1)
        _, H, bad = oracle.entropy(P, f)
        assert bad == 0
        Hs.append(H)
    d = np.diff(Hs)
    assert (d <= 1e-12 * Hs[0]).all()
    assert Hs[-1] < Hs[0] - 1e-6  # the dam break does dissipate


def test_discrete_h_theorem_periodic_1d():
    n = 400
    x = W.cell_centres(n)
    h0 = np.where((x > 0.25) & (x < 0.75), 2.0, 1.0)
    P = oracle.params(1, n, lam=3.0, s=1.0)
    f = oracle.run(P, h0, np.zeros(n), None, 0)
    Hs = [oracle.entropy(P, f)[1]]
    for _ in range(150):
        f = oracle.advance(P, f, 1)
        _, H, bad = oracle.entropy(P, f)
        assert bad == 0
        Hs.append(H)
    assert (np.diff(Hs) <= 1e-12 * Hs[0]).all()
    assert Hs[-1] < Hs[0] - 1e-6


@pytest.mark.parametrize("dim,lam", [(1, 3.0), (2, 6.0)])
def test_entropy_is_convex_in_the_populations(dim, lam):
    """h_j is a Legendre dual, hence convex (Sec. 1): Jensen on random pairs of
    near-equilibrium populations, h((F1 + F2)/2) <= (h(F1) + h(F2))/2."""
    P = oracle.params(dim, 1, 1, lam=lam)
    rng = np.random.default_rng(9)
    states = _random_states(rng, dim, 30, lam)
    for (h1, u1, v1), (h2, u2, v2) in zip(states[::2], states[1::2]):
        f1 = oracle.feq(P, h1, h1 * u1, h1 * v1)
        f2 = oracle.feq(P, h2, h2 * u2, h2 * v2)
        for j, (F1, F2) in enumerate(zip(_pops(P, f1, dim), _pops(P, f2, dim))):
            F1 = F1 * (1.0 + 0.05 * rng.standard_normal(F1.size))
            F2 = F2 * (1.0 + 0.05 * rng.standard_normal(F2.size))
            ok1, a, _ = oracle.entropy_pop(P, j, F1)
            ok2, b, _ = oracle.entropy_pop(P, j, F2)
            okm, m, _ = oracle.entropy_pop(P, j, 0.5 * (F1 + F2))
            assert ok1 and ok2 and okm
            assert m <= 0.5 * (a + b) + 1e-13 * (abs(a) + abs(b))


@pytest.mark.parametrize("dim", [1, 2])
def test_nonzero_rest_population_is_outside_the_domain(dim):
    """At a = 0 the rest potential h_0^* vanishes, so the dual of f_0 is finite
    only at f_0 = 0 (sup_theta theta f_0 = +inf otherwise)."""
    P = oracle.params(dim, 1, 1, lam=6.0)
    fe = oracle.feq(P, 1.3, 0.2, -0.1)
    _, tot, bad = oracle.entropy(P, fe.reshape(-1, 1))
    assert bad == 0 and math.isfinite(tot)
    fe[0] = 1e-3
    _, tot, bad = oracle.entropy(P, fe.reshape(-1, 1))
    assert bad == 1 and tot == math.inf
