"""Pins of the oracle's hand-derived discrete adjoint.

The adjoint (gradient of L = sum (h(T) - hhat)^2 with respect to the initial
height and the relaxation rate s) is checked against:

* complex-step directional derivatives of the same forward program (analytic
  in (h0, s): one division, no branches on the state) -- exact to ~1e-15;
* central finite differences (a check of the complex-step path itself);
* checkpoint-interval invariance (bitwise);
* the one-step transpose identity <J v, w> = <v, J^T w> with J v by complex step.
"""
import numpy as np
import pytest

from paper_1401_0427_amd import workloads as W


def _case(n=16, T=30, lam=3.0, s=1.8, sigma=0.1, seed=0):
    c, h_target0 = W.adjoint_case(n=n, lam=lam, s=s, steps=T, sigma=sigma, seed=seed, width2=0.05)
    return c, h_target0


def _hhat(orc, P, h_target0, T):
    f = orc.run(P, h_target0, None, None, T)
    return orc.moments(P, f)[0]


@pytest.mark.parametrize("n,T", [(16, 30), (12, 47)])
def test_adjoint_gradient_matches_complex_step(orc, n, T):
    c, ht0 = _case(n, T)
    P = orc.params(2, n, n, lam=c.lam, s=c.s)
    hhat = _hhat(orc, P, ht0, T)
    loss, gh, gs = orc.loss_grad_2d(P, c.h0, hhat, T, K=7)
    rng = np.random.default_rng(11)
    for _ in range(3):
        dh = rng.standard_normal((n, n))
        ds = float(rng.standard_normal())
        l_cs, d_cs = orc.loss_complex_step_2d(P, c.h0, hhat, T, dh0=dh, ds=ds)
        d_adj = float((gh * dh).sum()) + gs * ds
        assert abs(l_cs - loss) <= 1e-12 * loss
        assert abs(d_adj - d_cs) <= 1e-11 * (abs(d_cs) + 1e-300)
    # the s-gradient alone
    _, d_s = orc.loss_complex_step_2d(P, c.h0, hhat, T, dh0=None, ds=1.0)
    assert abs(gs - d_s) <= 1e-11 * abs(d_s)


def test_complex_step_agrees_with_central_differences(orc):
    n, T = 12, 25
    c, ht0 = _case(n, T)
    P = orc.params(2, n, n, lam=c.lam, s=c.s)
    hhat = _hhat(orc, P, ht0, T)
    rng = np.random.default_rng(3)
    dh = rng.standard_normal((n, n))
    _, d_cs = orc.loss_complex_step_2d(P, c.h0, hhat, T, dh0=dh, ds=0.0)
    eps = 1e-6
    lp = orc.loss_grad_2d(P, c.h0 + eps * dh, hhat, T, K=5)[0]
    lm = orc.loss_grad_2d(P, c.h0 - eps * dh, hhat, T, K=5)[0]
    assert abs((lp - lm) / (2 * eps) - d_cs) <= 1e-6 * abs(d_cs)


def test_checkpoint_interval_does_not_change_gradient(orc):
    n, T = 10, 40
    c, ht0 = _case(n, T)
    P = orc.params(2, n, n, lam=c.lam, s=c.s)
    hhat = _hhat(orc, P, ht0, T)
    ref = orc.loss_grad_2d(P, c.h0, hhat, T, K=1)
    for K in (3, 7, 40, 64):
        got = orc.loss_grad_2d(P, c.h0, hhat, T, K=K)
        assert got[0] == ref[0] and np.array_equal(got[1], ref[1]) and got[2] == ref[2]


def test_single_adjoint_step_is_transpose(orc):
    """<d u^{n+1}, w> = <d u^n, J^T w> for one step, with the forward
    directional derivative J d u^n taken by complex step of one step of the
    forward (through the complex-valued loss L(u) = sum h(u)^2 is not needed:
    linearity of the pull-stream lets us test via finite differences of
    orc.advance in double with a tiny, well-conditioned step)."""
    n = 8
    c, _ = _case(n, 1)
    P = orc.params(2, n, n, lam=c.lam, s=c.s)
    rng = np.random.default_rng(5)
    u = orc.run(P, c.h0 + 0.05 * rng.random((n, n)), 0.05 * rng.standard_normal((n, n)),
                0.05 * rng.standard_normal((n, n)), 3)
    u[0] = 0.0
    du = rng.standard_normal(u.shape)
    du[0] = 0.0
    w = rng.standard_normal(u.shape)
    w[0] = 0.0
    eps = 1e-6
    Jdu = (orc.advance(P, u + eps * du, 1) - orc.advance(P, u - eps * du, 1)) / (2 * eps)
    lam_n, _ = orc.adjoint_step(P, u, w)
    lhs = float((Jdu[1:] * w[1:]).sum())
    rhs = float((du[1:] * lam_n[1:]).sum())
    assert abs(lhs - rhs) <= 1e-7 * (abs(lhs) + 1.0)


FACE_SETS_1D = [("periodic", "periodic"), ("neumann", "neumann"), ("wall", "wall"),
                ("inflow", "wall"), ("neumann", "inflow"), ("wall", "neumann")]
FACE_SETS_2D = [("periodic",) * 4, ("wall", "wall", "wall", "wall"),
                ("neumann", "neumann", "neumann", "neumann"),
                ("inflow", "neumann", "wall", "inflow"), ("periodic", "periodic", "wall", "neumann"),
                ("wall", "inflow", "periodic", "periodic")]


def _faced(orc, dim, faces, n=(9, 7), lam=4.0, s=1.7):
    bc = tuple(faces) + (("periodic", "periodic") if dim == 1 else ())
    inflow = {f: (1.1, 0.15 * (1 - 2 * (f % 2)), 0.05) for f in range(4) if bc[f] == "inflow"}
    nx, ny = (n[0] * 3, 1) if dim == 1 else n
    return orc.params(dim, nx, ny, lam=lam, s=s, bc=bc, inflow=inflow)


def _state(orc, P, rng, steps=4):
    shape = (P.nx,) if P.dim == 1 else (P.ny, P.nx)
    h0 = 1.0 + 0.2 * rng.random(shape)
    qx0 = 0.1 * rng.standard_normal(shape)
    qy0 = 0.1 * rng.standard_normal(shape) if P.dim == 2 else None
    return orc.run(P, h0, qx0, qy0, steps)


@pytest.mark.parametrize("dim,faces", [(1, f) for f in FACE_SETS_1D] + [(2, f) for f in FACE_SETS_2D])
def test_adjoint_step_is_the_exact_transpose_with_faces(orc, dim, faces):
    """For one step u -> C(S(u)) with every face rule: <w, J du> = <J^T w, du> and
    <w, d/ds C(S(u))> = the step's dL/ds term, where J du and the s-derivative
    come from a complex step of the forward code (its pull and collision), not
    from the hand-derived transpose.  A wrong target, face, sign or opposite
    population in the transpose breaks the first identity."""
    P = _faced(orc, dim, faces)
    rng = np.random.default_rng(17 + dim)
    u = _state(orc, P, rng)
    du = rng.standard_normal(u.shape)  # the rest population included
    w = rng.standard_normal(u.shape)
    Jdu = orc.step_directional(P, u, du=du)
    lam_n, gs = orc.adjoint_step(P, u, w)
    lhs, rhs = float((w * Jdu).sum()), float((lam_n * du).sum())
    scale = float(np.abs(w * Jdu).sum())
    assert abs(lhs - rhs) <= 1e-13 * scale
    ds_dir = orc.step_directional(P, u, du=None, ds=1.0)
    assert abs(float((w * ds_dir).sum()) - gs) <= 1e-13 * float(np.abs(w * ds_dir).sum())


@pytest.mark.parametrize("dim,faces", [(1, FACE_SETS_1D[3]), (1, FACE_SETS_1D[4]),
                                       (2, FACE_SETS_2D[3]), (2, FACE_SETS_2D[4])])
def test_gradient_with_faces_matches_complex_step(orc, dim, faces):
    """The checkpointed gradient of L = sum (h(T) - hhat)^2 with respect to h0 and s
    on grids with inflow / wall / Neumann faces equals the complex-step
    directional derivative of the forward program."""
    P = _faced(orc, dim, faces, n=(12, 10))
    rng = np.random.default_rng(23)
    shape = (P.nx,) if dim == 1 else (P.ny, P.nx)
    h0 = 1.0 + 0.15 * rng.random(shape)
    T = 23
    hhat = orc.moments(P, orc.run(P, h0 + 0.05 * rng.standard_normal(shape), None, None, T))[0]
    loss, gh, gs = orc.loss_grad(P, h0, hhat, T, K=5)
    for _ in range(3):
        dh = rng.standard_normal(shape)
        ds = float(rng.standard_normal())
        l_cs, d_cs = orc.loss_complex_step_2d(P, h0, hhat, T, dh0=dh, ds=ds)
        assert abs(l_cs - loss) <= 1e-12 * loss
        d_adj = float((gh * dh).sum()) + gs * ds
        assert abs(d_adj - d_cs) <= 1e-10 * (abs(d_cs) + abs(gs * ds))
