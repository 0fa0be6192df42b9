"""GPU kernels of the paper's rest-population schemes (D1Q3Q2, D2Q5Q4Q4) with
moment-space MRT, against the oracle's literal moment-space relaxation.
Tolerance: FP64 storage 1e-12 normwise per plane (the two sides evaluate the
same formulas in different operation orders); FP32 storage L1 of h 1e-5."""
import numpy as np
import pytest

import oracle
from gpu_helpers import l1_rel, per_plane_rel, say, smooth_random_2d, to_np
from paper_1401_0427_amd import workloads as W

pytestmark = pytest.mark.gpu

RATES2D = [1.7, 1.6, 1.2, 1.9, 1.5, 1.3, 1.1, 1.45, 1.55, 1.8]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1401_0427_amd import lbm

    lbm.load()


def _gpu_rest(case, a, rates, steps, storage="f64"):
    from paper_1401_0427_amd.lbm import Solver

    S = Solver(case.dim, case.nx, case.ny, lam=case.lam, s=case.s, g=case.g, bc=case.bc,
               inflow=case.inflow, h0=case.h0, qx0=case.qx0,
               qy0=case.qy0 if case.dim == 2 else None, storage=storage, rest=True, a=a,
               rates=rates)
    S.step(steps)
    return S


def _orc_rest(case, a, rates, steps):
    P = oracle.params(case.dim, case.nx, case.ny, lam=case.lam, s=case.s, g=case.g, bc=case.bc,
                      inflow=case.inflow, a=a, mrt=True, rates=rates)
    return oracle.run(P, case.h0, case.qx0, case.qy0 if case.dim == 2 else None, steps), P


@pytest.mark.parametrize("bc,inflow", [
    (("periodic",) * 4, {}),
    (("inflow", "neumann", "wall", "wall"), {0: (1.2, 0.3, 0.0)}),
    (("wall", "wall", "periodic", "periodic"), {}),
])
def test_d2q5q4q4_mrt_matches_oracle(bc, inflow):
    case = smooth_random_2d(300, 34, seed=11, lam=6.0, s=1.7, bc=bc, inflow=inflow)
    say(f"[mrt 2D] {bc} a=0.05 rates={RATES2D}")
    S = _gpu_rest(case, 0.05, RATES2D, 120)
    got = to_np(S.planes())
    ref, _ = _orc_rest(case, 0.05, RATES2D, 120)
    err = per_plane_rel(got, ref)
    say(f"  max plane rel err {err:.3e}")
    assert got.shape == ref.shape == (13, 34, 300)
    assert err <= 1e-12


def test_d1q3q2_fig1_setup_matches_oracle():
    """Sec. 2 experiment on the GPU: 80 points, a = 0.15, lambda = 8, s = 1.8."""
    n = 80
    x = W.cell_centres(n)
    case = W.Case(1, n, 1, 8.0, 1.8, 96, bc=("neumann", "neumann", "periodic", "periodic"),
                  h0=np.where(x < 0.5, 2.0, 0.5), qx0=np.zeros(n))
    S = _gpu_rest(case, 0.15, [1.8, 1.8, 1.8], 96)
    ref, P = _orc_rest(case, 0.15, [1.8, 1.8, 1.8], 96)
    err = per_plane_rel(to_np(S.planes()), ref)
    say(f"[mrt 1D fig1] max plane rel err {err:.3e}")
    assert err <= 1e-12


def test_d1q3q2_distinct_rates_walls_inflow():
    case = W.wall_reflection_1d(4096, s=1.7, steps=2500)
    rates = [1.7, 1.3, 1.9]
    S = _gpu_rest(case, 0.1, rates, 2500)
    ref, _ = _orc_rest(case, 0.1, rates, 2500)
    err = per_plane_rel(to_np(S.planes()), ref)
    say(f"[mrt 1D wall/inflow] max plane rel err {err:.3e}")
    assert err <= 1e-12


def test_rest_scheme_at_a0_equal_rates_is_the_hot_path():
    """a = 0 with every rate equal to s reproduces the D2Q4x3 BGK kernel (the
    rest population stays at rounding level)."""
    from gpu_helpers import gpu_solver

    case = smooth_random_2d(128, 96, seed=12)
    R = _gpu_rest(case, 0.0, [case.s] * 10, 150)
    H = gpu_solver(case)
    H.step(150)
    a, b = to_np(R.planes()), to_np(H.planes())
    assert np.abs(a[0]).max() < 1e-14
    assert per_plane_rel(a[1:], b) <= 1e-13


def test_d2q5q4q4_fp32_storage_l1():
    case = W.radial_dam_break_2d(192, lam=6.0)
    S = _gpu_rest(case, 0.05, RATES2D, 300, storage="f32")
    ref, P = _orc_rest(case, 0.05, RATES2D, 300)
    e = l1_rel(to_np(S.moments()[0]), oracle.moments(P, ref)[0])
    say(f"[mrt fp32] L1 rel of h {e:.3e}")
    assert e <= 1e-5


def test_adjoint_rejects_rest_lattice():
    from paper_1401_0427_amd.lbm import LbmError

    case = smooth_random_2d(40, 40, seed=1)
    S = _gpu_rest(case, 0.05, RATES2D, 1)
    with pytest.raises(LbmError, match="D2Q4x3"):
        S.adjoint_step(S.current()[0], S.new_state(), S.new_state(), S.adjoint_partials())


def _rest_solver(case, storage, fuse, a=0.05, rates=RATES2D):
    from paper_1401_0427_amd.lbm import Solver

    return Solver(2, case.nx, case.ny, lam=case.lam, s=case.s, g=case.g, bc=case.bc,
                  h0=case.h0, qx0=case.qx0, qy0=case.qy0, storage=storage, rest=True, a=a,
                  rates=rates, fuse_steps=fuse)


@pytest.mark.parametrize("storage", ["f64", "f32"])
@pytest.mark.parametrize("nx,ny", [(300, 70), (130, 41), (40, 37)])
def test_d2q5q4q4_multistep_launch_equals_single_steps(storage, nx, ny):
    """K = 2 .. 6 steps per launch of the rest-population scheme on periodic grids
    (strips of 64 - 2 (K - 1) output columns: several strips with a ragged last
    one, and a grid narrower than one strip) equal single steps bit for bit, over
    runs whose plans mix launch depths."""
    import torch

    case = smooth_random_2d(nx, ny, seed=5, lam=6.0, s=1.7)
    steps = 23
    A = _rest_solver(case, storage, 1)
    assert A.launch_info()["steps_per_launch"] == 1
    A.step(steps)
    ref = A.planes()
    for K in range(2, 7):
        B = _rest_solver(case, storage, K)
        info = B.launch_info()
        plan = B.launch_plan(steps)
        say(f"[mrt multistep] {storage} {nx}x{ny} K={K} info={info} plan={plan}")
        assert info["steps_per_launch"] == K and info["segment_rows"] > 0
        assert sum(plan) == steps and max(plan) == K
        B.step(steps)
        torch.cuda.synchronize()
        assert torch.equal(B.planes(), ref), f"K={K}"


def test_d2q5q4q4_multistep_matches_oracle():
    """4 steps per launch against the oracle's literal moment-space MRT (FP64,
    1e-12 per plane), 120 steps on a periodic grid."""
    case = smooth_random_2d(300, 34, seed=11, lam=6.0, s=1.7)
    S = _rest_solver(case, "f64", 4)
    assert S.launch_info()["steps_per_launch"] == 4
    S.step(120)
    ref, _ = _orc_rest(case, 0.05, RATES2D, 120)
    err = per_plane_rel(to_np(S.planes()), ref)
    say(f"[mrt multistep oracle] max plane rel err {err:.3e}")
    assert err <= 1e-12


def test_d2q5q4q4_default_launch_on_a_large_periodic_grid():
    """On a grid large enough to fill the device the rest-population scheme runs 5
    steps per launch by default, bitwise equal to single steps; with a non-periodic
    face it keeps one step per launch."""
    import torch

    case = smooth_random_2d(1024, 1024, seed=2, lam=6.0, s=1.8)
    A = _rest_solver(case, "f64", 1)
    B = _rest_solver(case, "f64", 0)
    assert B.launch_info()["steps_per_launch"] == 5
    A.step(18)
    B.step(18)
    torch.cuda.synchronize()
    assert torch.equal(A.planes(), B.planes())
    walls = smooth_random_2d(1024, 1024, seed=2, lam=6.0, s=1.8,
                             bc=("wall", "wall", "periodic", "periodic"))
    assert _rest_solver(walls, "f64", 0).launch_info()["steps_per_launch"] == 1


def _rest1d_solver(case, storage, fuse, a=0.1, rates=(1.7, 1.3, 1.9)):
    from paper_1401_0427_amd.lbm import Solver

    return Solver(1, case.nx, 1, lam=case.lam, s=case.s, g=case.g, bc=case.bc, inflow=case.inflow,
                  h0=case.h0, qx0=case.qx0, storage=storage, rest=True, a=a, rates=list(rates),
                  fuse_steps=fuse)


def _riemann_1d(n, bc, inflow=None, lam=4.0):
    x = W.cell_centres(n)
    rng = np.random.default_rng(n)
    h0 = np.where(x < 0.5, 1.6, 0.7) + 0.01 * rng.random(n)
    q0 = 0.1 * np.sin(2 * np.pi * x)
    return W.Case(1, n, 1, lam, 1.7, 0, bc=bc, inflow=inflow or {}, h0=h0, qx0=q0)


@pytest.mark.parametrize("storage", ["f64", "f32"])
@pytest.mark.parametrize("n,bc,inflow,ks", [
    (3000, ("periodic",) * 4, None, (2, 5, 16)),
    (2500, ("inflow", "wall", "periodic", "periodic"), {0: (1.4, 0.35, 0.0)}, (3, 16)),
    (900, ("wall", "inflow", "periodic", "periodic"), {1: (1.1, -0.2, 0.0)}, (7, 64, 300)),
    (80, ("neumann", "neumann", "periodic", "periodic"), None, (96,)),
])
def test_d1q3q2_multistep_launch_equals_single_steps(storage, n, bc, inflow, ks):
    """K steps per launch of D1Q3Q2 with distinct rates equal single steps bit for bit:
    periodic tiles with a ragged last one, wall and inflow ends across tiles, and
    domains that fit one tile (any K, the whole run in few launches)."""
    import torch

    case = _riemann_1d(n, bc, inflow)
    steps = 300 if n > 100 else 96
    A = _rest1d_solver(case, storage, 1)
    A.step(steps)
    ref = A.planes()
    for K in ks:
        B = _rest1d_solver(case, storage, K)
        assert B.launch_info()["steps_per_launch"] == K
        B.step(steps)
        torch.cuda.synchronize()
        say(f"[mrt 1D multistep] {storage} n={n} {bc[:2]} K={K} launches={len(B.launch_plan(steps))}")
        assert torch.equal(B.planes(), ref), f"K={K}"


def test_d1q3q2_default_launches():
    """By default D1Q3Q2 takes the 1D launch plan of the hot path: 16 steps per launch,
    and the whole run in one launch for a domain with non-periodic ends that fits one
    tile (the Fig. 1 setup: 80 points, 96 steps)."""
    big = _rest1d_solver(_riemann_1d(5000, ("periodic",) * 4), "f64", 0)
    assert big.launch_info()["steps_per_launch"] == 16
    n = 80
    x = W.cell_centres(n)
    case = W.Case(1, n, 1, 8.0, 1.8, 96, bc=("neumann", "neumann", "periodic", "periodic"),
                  h0=np.where(x < 0.5, 2.0, 0.5), qx0=np.zeros(n))
    S = _rest1d_solver(case, "f64", 0, a=0.15, rates=(1.8, 1.8, 1.8))
    assert S.launch_plan(96) == [96]


@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_rest_multistep_launches_on_degenerate_grids(storage):
    """Tiny grids where a launch's strips and halo rows wrap the grid several times
    (D2Q5Q4Q4 5 x 3 and 2 x 2 periodic, K = 2 .. 6) and a two-node D1Q3Q2 domain with
    wall / Neumann ends (one tile, 40 steps per launch) equal single steps bit for bit."""
    import torch

    for nx, ny in ((5, 3), (2, 2)):
        case = smooth_random_2d(nx, ny, seed=13, lam=6.0, s=1.7)
        A = _rest_solver(case, storage, 1)
        A.step(17)
        for K in range(2, 7):
            B = _rest_solver(case, storage, K)
            assert B.launch_info()["steps_per_launch"] == K
            B.step(17)
            torch.cuda.synchronize()
            assert torch.equal(B.planes(), A.planes()), (nx, ny, K)
    case = _riemann_1d(2, ("wall", "neumann", "periodic", "periodic"))
    A = _rest1d_solver(case, storage, 1)
    A.step(80)
    B = _rest1d_solver(case, storage, 40)
    assert B.launch_plan(80) == [40, 40]
    B.step(80)
    torch.cuda.synchronize()
    assert torch.equal(B.planes(), A.planes())
