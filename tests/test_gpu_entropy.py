"""GPU entropy diagnostic (lbm_entropy) against the oracle's H(f).

The kernel solves one scalar equation per population (the stationarity
conditions reduced in closed form); the oracle maximises phi . F - h_j^*(phi)
over the convexity domain with a Newton ascent in all the entropy variables.
Same definition, different algorithms.  Tolerances: FP64 storage -- per-node
entropies normwise <= 1e-12 and totals relative <= 1e-12 (the FP64 states
agree bit for bit, so this measures the two solvers); FP32 storage -- total
relative <= 1e-5 against the FP64 oracle run (the state itself differs by
storage rounding)."""
import math

import numpy as np
import pytest

import oracle
from gpu_helpers import gpu_solver, normwise_rel, orc_params, say, smooth_random_2d, to_np
from paper_1401_0427_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL64 = 1e-12


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1401_0427_amd import lbm

    lbm.load()


def _oracle_entropy(case, steps):
    P = orc_params(case)
    f = oracle.run(P, case.h0, case.qx0, case.qy0 if case.dim == 2 else None, steps)
    return oracle.entropy(P, f)


def _check(case, steps, storage="f64"):
    say(f"[entropy] {case.name} steps={steps} storage={storage}")
    S = gpu_solver(case, storage=storage)
    S.step(steps)
    tot, bad, hn = S.entropy(per_node=True)
    hn = to_np(hn)
    ref_n, ref_tot, ref_bad = _oracle_entropy(case, steps)
    say(f"  total {tot!r} vs oracle {ref_tot!r}; invalid {bad} vs {ref_bad}")
    return tot, bad, hn, ref_tot, ref_bad, ref_n


@pytest.mark.parametrize("steps", [0, 1, 40])
def test_entropy_2d_periodic_fp64_matches_oracle(steps):
    case = W.radial_dam_break_2d(96, lam=6.0)
    tot, bad, hn, rt, rb, rn = _check(case, steps)
    assert bad == rb == 0
    err = normwise_rel(hn, rn)
    say(f"  per-node rel err {err:.3e}")
    assert err <= TOL64
    assert abs(tot - rt) <= TOL64 * abs(rt)
    if steps == 0:  # the equilibrium of a fluid at rest: H = sum g h^2 / 2
        eta = math.fsum((0.5 * case.h0 ** 2).ravel())
        assert abs(tot - eta) <= TOL64 * eta


def test_entropy_2d_moving_fluid_ragged_fp64():
    case = smooth_random_2d(300, 37, seed=3)  # 300 x 37 = 11100 nodes: 43 blocks + a ragged tail
    tot, bad, hn, rt, rb, rn = _check(case, 25)
    assert bad == rb == 0
    assert normwise_rel(hn, rn) <= TOL64
    assert abs(tot - rt) <= TOL64 * abs(rt)


def test_entropy_1d_fp64_matches_oracle():
    case = W.dam_break_1d(1000)
    tot, bad, hn, rt, rb, rn = _check(case, 100)
    assert bad == rb == 0
    assert normwise_rel(hn, rn) <= TOL64
    assert abs(tot - rt) <= TOL64 * abs(rt)


def test_entropy_walls_and_inflow_fp64():
    case = W.oblique_shock_2d(20, steps=300)
    tot, bad, hn, rt, rb, rn = _check(case, case.steps)
    assert bad == rb == 0
    assert normwise_rel(hn, rn) <= TOL64
    assert abs(tot - rt) <= TOL64 * abs(rt)


def test_entropy_invalid_populations_match_oracle():
    """lambda = 2.9 < 2 (|u| + sqrt(g h)) inside the disk (h = 2): after a few
    steps some populations have no stationary point in the convexity domain."""
    case = W.radial_dam_break_2d(64, lam=2.9)
    tot, bad, hn, rt, rb, rn = _check(case, 5)
    assert rb > 0 and bad == rb
    assert tot == math.inf and rt == math.inf
    fin = np.isfinite(rn)
    assert np.array_equal(np.isfinite(hn), fin)
    assert normwise_rel(hn[fin], rn[fin]) <= TOL64


def test_entropy_fp32_storage():
    case = W.radial_dam_break_2d(96, lam=6.0)
    tot, bad, hn, rt, rb, rn = _check(case, 40, storage="f32")
    assert bad == rb == 0
    assert abs(tot - rt) <= 1e-5 * abs(rt)


def test_discrete_h_theorem_on_the_gpu():
    """s = 1: the relaxation is a convex combination and the periodic streaming a
    permutation, so H never increases; the last value equals the oracle's."""
    case = W.radial_dam_break_2d(96, lam=6.0, s=1.0)
    S = gpu_solver(case)
    Hs = [S.entropy()[0]]
    for _ in range(50):
        S.step(1)
        H, bad = S.entropy()
        assert bad == 0
        Hs.append(H)
    d = np.diff(Hs)
    say(f"[entropy] H from {Hs[0]!r} to {Hs[-1]!r}, max step change {d.max():.3e}")
    assert (d <= 1e-12 * Hs[0]).all() and Hs[-1] < Hs[0]
    _, rt, _ = _oracle_entropy(case, 50)
    assert abs(Hs[-1] - rt) <= TOL64 * rt


def test_entropy_full_4096_equilibrium():
    """Headline grid at level 0 (equilibrium of the radial dam break at rest):
    total = sum g h0^2 / 2 and every node = g h0^2 / 2 (closed form)."""
    import torch

    case = W.radial_dam_break_2d(4096, lam=6.0)
    S = gpu_solver(case)
    tot, bad, hn = S.entropy(per_node=True)
    want = 0.5 * case.h0 ** 2
    eta = math.fsum(want.ravel())
    err = float((hn - torch.as_tensor(want, device=hn.device)).abs().max().item())
    say(f"[entropy 4096^2] total {tot!r} vs {eta!r}, max node err {err:.3e}")
    assert bad == 0 and abs(tot - eta) <= TOL64 * eta and err <= 1e-14
    del S, hn
    torch.cuda.empty_cache()
