"""GPU (gfx950) parity of the HIP path against the CPU FP64 oracle, through the
C ABI.  Tolerances: FP64 storage -- normwise max relative error <= 1e-12 per
plane (the arithmetic order is the same on both sides, so the results are
expected to agree bit for bit); FP32 storage -- L1 relative error of h <= 1e-5
against the FP64 oracle."""
import math

import numpy as np
import pytest

import oracle
from gpu_helpers import (gpu_solver, l1_rel, normwise_rel, orc_params, orc_state,
                         per_plane_rel, say, smooth_random_2d, to_np)
from paper_1401_0427_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
TOL32_L1 = 1e-5


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1401_0427_amd import lbm

    lbm.load()


def _compare(case, steps, storage="f64", **kw):
    say(f"[parity] {case.name} steps={steps} storage={storage} {kw}")
    S = gpu_solver(case, storage=storage, **kw)
    S.step(steps)
    got = to_np(S.planes())
    ref, P = orc_state(case, steps)
    return got, ref, S, P


@pytest.mark.parametrize("launch", [dict(block=256, npt=1), dict(block=64, npt=4),
                                    dict(block=512, npt=2), dict(block=128, npt=2)])
def test_2d_periodic_fp64_matches_oracle(launch):
    case = smooth_random_2d(300, 40, seed=1)  # 300 = 256 + ragged 44
    got, ref, S, _ = _compare(case, 150, **launch)
    err = per_plane_rel(got, ref)
    say(f"  max plane rel err {err:.3e}, bitwise equal: {np.array_equal(got, ref)}")
    assert err <= TOL64


@pytest.mark.parametrize("bc,inflow", [
    (("inflow", "neumann", "wall", "wall"), {0: (1.2, 0.3, 0.0)}),
    (("wall", "wall", "periodic", "periodic"), {}),
    (("periodic", "periodic", "neumann", "inflow"), {3: (0.9, 0.05, -0.2)}),
])
def test_2d_boundaries_fp64_matches_oracle(bc, inflow):
    case = smooth_random_2d(70, 50, seed=2, bc=bc, inflow=inflow)
    got, ref, _, _ = _compare(case, 120)
    err = per_plane_rel(got, ref)
    say(f"  {bc}: max plane rel err {err:.3e}")
    assert err <= TOL64


def test_1d_dam_break_fp64_matches_oracle():
    case = W.dam_break_1d(1000)  # 1D Riemann workload: 1000 nodes, 400 steps, Neumann ends
    got, ref, _, _ = _compare(case, case.steps)
    err = per_plane_rel(got, ref)
    say(f"  max plane rel err {err:.3e}")
    assert err <= TOL64


@pytest.mark.parametrize("s", [1.5, 1.9])
def test_1d_wall_reflection_fp64_matches_oracle(s):
    case = W.wall_reflection_1d(8192, s=s, steps=3000)
    got, ref, _, _ = _compare(case, 3000, npt=2)
    err = per_plane_rel(got, ref)
    say(f"  s={s}: max plane rel err {err:.3e}")
    assert err <= TOL64


def test_1d_periodic_ragged_fp64():
    rng = np.random.default_rng(3)
    n = 777
    h = 1 + 0.2 * rng.random(n)
    case = W.Case(1, n, 1, 3.0, 1.7, 0, bc=("periodic",) * 4, h0=h, qx0=0.1 * rng.standard_normal(n))
    got, ref, S, P = _compare(case, 250, block=64, npt=4)
    assert per_plane_rel(got, ref) <= TOL64
    (hh, qq), tot = S.moments(totals=True)
    assert abs(tot[0] - math.fsum(h)) <= 1e-13 * math.fsum(h)


def test_moments_and_totals_match_oracle():
    case = smooth_random_2d(300, 40, seed=4)
    S = gpu_solver(case)
    S.step(77)
    (h, qx, qy), tot = S.moments(totals=True)
    ref, P = orc_state(case, 77)
    full = np.concatenate([np.zeros((1,) + ref.shape[1:]), ref])
    oh, oqx, oqy = oracle.moments(P, full)
    for a, b in ((h, oh), (qx, oqx), (qy, oqy)):
        assert normwise_rel(to_np(a), b) <= TOL64
    for k, (t, b) in enumerate(zip(tot, (case.h0, case.qx0, case.qy0))):
        assert abs(t - math.fsum(b.ravel())) <= 1e-12 * (math.fsum(np.abs(b).ravel()) + 1)


def test_graph_chunks_equal_single_launches():
    """lbm_step(70) (two captured 32-step graphs + 6 launches) = 70 x lbm_step(1)."""
    case = smooth_random_2d(128, 36, seed=5)
    A = gpu_solver(case)
    B = gpu_solver(case)
    A.step(70)
    for _ in range(70):
        B.step(1)
    assert np.array_equal(to_np(A.planes()), to_np(B.planes()))
    A.step(3)  # odd offset: the graph for the other starting buffer
    A.step(64)
    B.step(67)
    assert np.array_equal(to_np(A.planes()), to_np(B.planes()))


def test_step_buffers_export_import_roundtrip():
    case = smooth_random_2d(64, 64, seed=6)
    S = gpu_solver(case)
    a = S.new_state()
    b = S.new_state()
    S.export(a)
    S.step_buffers(a, b)
    S.step(1)
    assert np.array_equal(to_np(S.planes()), to_np(S.planes(b)))
    S.import_(a)
    S.step(1)
    assert np.array_equal(to_np(S.planes()), to_np(S.planes(b)))


def test_fp32_storage_l1_error_2d():
    case = W.radial_dam_break_2d(256, lam=6.0, steps=500)
    got, ref, S, P = _compare(case, 500, storage="f32")
    (h, _, _) = S.moments()
    full = np.concatenate([np.zeros((1,) + ref.shape[1:]), ref])
    oh = oracle.moments(P, full)[0]
    e = l1_rel(to_np(h), oh)
    say(f"  FP32 storage 256^2 x 500: L1 rel error of h = {e:.3e}")
    assert e <= TOL32_L1


def test_fp32_storage_l1_error_1d_wall():
    case = W.wall_reflection_1d(8192, s=1.9, steps=20000)
    got, ref, S, P = _compare(case, 20000, storage="f32")
    h = to_np(S.moments()[0])
    full = np.concatenate([np.zeros((1,) + ref.shape[1:]), ref])
    oh = oracle.moments(P, full)[0]
    e = l1_rel(h, oh)
    say(f"  FP32 storage 1D wall reflection 8192 x 20000: L1 rel error of h = {e:.3e}")
    assert e <= TOL32_L1


def test_divergence_detected():
    """The radial dam break at the stated lambda = 3 satisfies the D2Q4 bound at
    rest (2 sqrt(2) < 3) but the flow it develops does not, and it blows up; the
    periodic check reports it."""
    from paper_1401_0427_amd.lbm import LbmError

    case = W.radial_dam_break_2d(256, lam=3.0)
    S = gpu_solver(case, check_every=25)
    with pytest.raises(LbmError, match="diverged"):
        S.step(2000)


def test_subchar_warning():
    """lambda below 2 max(|u| + sqrt(g h)) at t = 0 warns (context still usable)."""
    case = W.radial_dam_break_2d(64, lam=2.5)
    with pytest.warns(RuntimeWarning, match="monotonicity bound"):
        S = gpu_solver(case)
    S.step(1)


@pytest.mark.parametrize("bad", [0.0, -1.0, 1e-200, 1e200, float("nan")])
def test_init_rejects_depth_outside_range(bad):
    """Initial heights must be positive and within (2^-500, 2^500), the range in
    which the library's reciprocal is the IEEE quotient."""
    from paper_1401_0427_amd.lbm import LbmError

    case = smooth_random_2d(40, 40, seed=7)
    case.h0[3, 5] = bad
    with pytest.raises(LbmError, match="2\\^-500 < h"):
        gpu_solver(case)


@pytest.mark.parametrize("ny", [20, 40, 80])
def test_oblique_shock_reflection_fp64_matches_oracle(ny):
    """Sec. 4 stationary reflection on the paper's meshes (35 x 20, 70 x 40,
    140 x 80): inflow faces (left, top), wall (bottom), outflow (right), run to
    steady state -- the GPU state equals the oracle's."""
    case = W.oblique_shock_2d(ny)
    got, ref, S, P = _compare(case, case.steps)
    err = per_plane_rel(got, ref)
    say(f"  {case.name} {case.steps} steps: max plane rel err {err:.3e}")
    assert err <= TOL64


@pytest.mark.parametrize("storage", ["f64", "f32"])
@pytest.mark.parametrize("fuse", [2, 3, 4, 5, 8])
@pytest.mark.parametrize("shape,steps", [((300, 70), 6), ((600, 130), 7), ((17, 5), 9),
                                         ((96, 80), 37), ((254, 64), 2), ((1100, 50), 4),
                                         ((3, 2), 11), ((58, 97), 8), ((2, 300), 13),
                                         ((233, 211), 70)])
def test_fused_launch_equals_single_steps(storage, fuse, shape, steps):
    """fuse_steps = 2 .. 8 (steps per launch, all-periodic 2D) gives bit for bit
    the state of single steps: one strip, several strips with a ragged last one,
    ragged row segments, grids smaller than one strip or than the halo, step
    counts that are not multiples of the launch depth (shorter last launches) and
    runs long enough for the captured graph chunks."""
    nx, ny = shape
    case = smooth_random_2d(nx, ny, seed=5)
    say(f"[fused] {nx}x{ny} steps={steps} fuse={fuse} storage={storage}")
    A = gpu_solver(case, storage=storage, fuse_steps=1)
    B = gpu_solver(case, storage=storage, fuse_steps=fuse)
    A.step(steps)
    B.step(steps)
    a, b = to_np(A.planes()), to_np(B.planes())
    assert np.array_equal(a, b)
    if storage == "f64":
        ref, _ = orc_state(case, steps)
        assert per_plane_rel(b, ref) <= TOL64


_IN = {0: (1.2, 0.3, 0.05), 1: (0.9, -0.2, 0.1), 2: (1.1, 0.05, 0.25), 3: (0.95, 0.1, -0.15)}


def _bounded(nx, ny, bc, seed):
    inflow = {f: _IN[f] for f in range(4) if bc[f] == "inflow"}
    return smooth_random_2d(nx, ny, seed=seed, bc=bc, inflow=inflow)


BOUNDED = [  # face rules (x-, x+, y-, y+), grid, steps
    (("inflow", "neumann", "wall", "inflow"), (300, 70), 13),   # the oblique shock's faces
    (("wall", "wall", "wall", "wall"), (233, 211), 70),          # closed box, many segments
    (("neumann", "neumann", "neumann", "neumann"), (17, 5), 9),  # one strip
    (("periodic", "periodic", "wall", "neumann"), (130, 97), 11),  # y faces only
    (("inflow", "wall", "periodic", "periodic"), (600, 40), 7),   # x faces only
    (("wall", "inflow", "neumann", "wall"), (2, 60), 21),         # narrower than the halo
    (("neumann", "inflow", "inflow", "neumann"), (70, 2), 10),    # two rows (the minimum)
    (("wall", "neumann", "inflow", "wall"), (3, 33), 12),         # three columns
]


@pytest.mark.parametrize("storage", ["f64", "f32"])
@pytest.mark.parametrize("fuse", [2, 3, 4, 5, 6, 7, 8])
@pytest.mark.parametrize("bc,shape,steps", BOUNDED)
def test_fused_bounded_launch_equals_single_steps(storage, fuse, bc, shape, steps):
    """fuse_steps = K (2 .. 8) on 2D grids with Neumann, wall and inflow faces
    (alone, in every corner combination, with the other axis periodic, on grids
    of two rows, three columns or narrower than the halo) gives bit for bit the
    state of single steps; FP64 also matches the oracle.  At least two whole
    launches and a remainder run."""
    nx, ny = shape
    steps = max(steps, 2 * fuse + 3)
    case = _bounded(nx, ny, bc, seed=nx + ny)
    say(f"[fused bounded] {nx}x{ny} bc={bc} steps={steps} fuse={fuse} storage={storage}")
    A = gpu_solver(case, storage=storage, fuse_steps=1)
    B = gpu_solver(case, storage=storage, fuse_steps=fuse)
    assert B.launch_info()["steps_per_launch"] == fuse
    A.step(steps)
    B.step(steps)
    a, b = to_np(A.planes()), to_np(B.planes())
    assert np.array_equal(a, b)
    if storage == "f64":
        ref, _ = orc_state(case, steps)
        assert per_plane_rel(b, ref) <= TOL64


@pytest.mark.parametrize("fuse", [3, 4, 6, 8])
def test_fused_oblique_shock_matches_oracle(fuse):
    """The oblique shock reflection (inflow left and top, wall bottom, outflow
    right) run to steady state with fuse_steps = K equals the oracle."""
    case = W.oblique_shock_2d(40)
    got, ref, S, _ = _compare(case, case.steps, fuse_steps=fuse)
    assert S.launch_info()["steps_per_launch"] == fuse
    err = per_plane_rel(got, ref)
    say(f"  {case.name} {case.steps} steps, fuse {fuse}: max plane rel err {err:.3e}")
    assert err <= TOL64


def _case_1d(n, bc, inflow, seed):
    rng = np.random.default_rng(seed)
    x = W.cell_centres(n)
    h = 1.0 + 0.5 * (x < 0.5) + 0.05 * rng.random(n)
    q = 0.1 * np.sin(2 * np.pi * x) + 0.02 * rng.standard_normal(n)
    return W.Case(1, n, 1, 3.0, 1.9, 0, bc=bc + ("periodic", "periodic"), h0=h, qx0=q,
                  inflow=inflow, name=f"fused1d_{n}")


@pytest.mark.parametrize("storage", ["f64", "f32"])
@pytest.mark.parametrize("fuse", [2, 4, 16])
@pytest.mark.parametrize("n,bc,inflow,steps", [
    (777, ("periodic", "periodic"), {}, 37),        # one tile, wraps onto itself
    (5000, ("periodic", "periodic"), {}, 70),       # several tiles, ragged last one
    (2000, ("neumann", "neumann"), {}, 45),
    (3000, ("inflow", "wall"), {0: (1.5, 0.75, 0.0)}, 101),
    (1500, ("wall", "inflow"), {1: (1.2, -0.3, 0.0)}, 33),
    (40, ("wall", "wall"), {}, 19),                 # grid smaller than the halo
])
def test_fused_1d_launch_equals_single_steps(storage, fuse, n, bc, inflow, steps):
    """fuse_steps = K on the 1D path (K steps per launch through LDS) gives bit for
    bit the state of single steps, for every face rule, one or several tiles,
    ragged tails, grids smaller than one tile, step counts that are not multiples
    of K (a shorter last launch) and runs long enough for the captured graphs."""
    case = _case_1d(n, bc, inflow, seed=n + fuse)
    say(f"[fused1d] n={n} bc={bc} fuse={fuse} steps={steps} storage={storage}")
    A = gpu_solver(case, storage=storage, fuse_steps=1)
    B = gpu_solver(case, storage=storage, fuse_steps=fuse)
    A.step(steps)
    B.step(steps)
    a, b = to_np(A.planes()), to_np(B.planes())
    assert np.array_equal(a, b)
    if storage == "f64":
        ref, _ = orc_state(case, steps)
        assert per_plane_rel(b, ref) <= TOL64


@pytest.mark.parametrize("storage", ["f64", "f32"])
@pytest.mark.parametrize("n,bc,inflow", [
    (1000, ("neumann", "neumann"), {}),
    (1024, ("inflow", "wall"), {0: (1.5, 0.75, 0.0)}),
    (333, ("wall", "inflow"), {1: (1.2, -0.3, 0.0)}),
])
def test_whole_domain_1d_launch_equals_single_steps(storage, n, bc, inflow):
    """A 1D domain with non-periodic ends that fits one LDS tile (at most 1024 nodes)
    loses nothing at the tile's ends, so it takes up to 1024 steps per launch by
    default (400 steps: one launch; 1500: 1024 + 476); the state equals single steps
    bit for bit and, in FP64, the oracle.  1025 nodes fall back to 16 steps."""
    case = _case_1d(n, bc, inflow, seed=n)
    A = gpu_solver(case, storage=storage, fuse_steps=1)
    B = gpu_solver(case, storage=storage)
    assert B.launch_info()["steps_per_launch"] == 1024
    assert B.launch_plan(400) == [400] and B.launch_plan(1500) == [1024, 476]
    for steps in (400, 1500):
        A.step(steps)
        B.step(steps)
        a, b = to_np(A.planes()), to_np(B.planes())
        assert np.array_equal(a, b), steps
    if storage == "f64":
        ref, _ = orc_state(case, 1900)
        assert per_plane_rel(b, ref) <= TOL64
    big = gpu_solver(_case_1d(1025, bc, inflow, seed=3), storage=storage)
    assert big.launch_info()["steps_per_launch"] == 16


def test_default_launch_plans():
    """lbm_launch_info reports the plan chosen at init: the wave-strip multi-step
    launch on grids it can fill (8 steps per launch; FP32 6 on grids below about
    three workgroups per resident slot, such as 1024^2), with a segment length and
    the resident workgroups it was chosen against; one step per launch on a
    small FP32 grid; 16 steps per launch in 1D (1024 on a domain with non-periodic ends that
    fits one tile); with non-periodic 2D faces 7
    (FP64) / 8 (FP32) steps, or fewer where that launch cannot fill the device;
    an explicit request is honoured up to 8 steps."""
    big64 = gpu_solver(smooth_random_2d(1024, 1024, seed=8), storage="f64").launch_info()
    assert big64["steps_per_launch"] == 8 and big64["segment_rows"] >= 16
    assert big64["resident_blocks"] > 0
    big32 = gpu_solver(smooth_random_2d(1024, 1024, seed=8), storage="f32").launch_info()
    assert big32["steps_per_launch"] == 6 and big32["segment_rows"] >= 16
    huge32 = gpu_solver(smooth_random_2d(4096, 4096, seed=8), storage="f32").launch_info()
    assert huge32["steps_per_launch"] == 8
    small32 = gpu_solver(smooth_random_2d(256, 256, seed=8), storage="f32").launch_info()
    assert small32["steps_per_launch"] == 1
    one_d = gpu_solver(W.dam_break_1d(5000)).launch_info()
    assert one_d["steps_per_launch"] == 16 and one_d["segment_rows"] == 0
    small_1d = gpu_solver(W.dam_break_1d(1000)).launch_info()
    assert small_1d["steps_per_launch"] == 1024
    walls = gpu_solver(W.oblique_shock_2d(20, steps=10), fuse_steps=4).launch_info()
    assert walls["steps_per_launch"] == 4 and walls["segment_rows"] >= 16
    walls8 = gpu_solver(W.oblique_shock_2d(20, steps=10), fuse_steps=8).launch_info()
    assert walls8["steps_per_launch"] == 8
    box = gpu_solver(smooth_random_2d(1024, 1024, seed=8, bc=("wall",) * 4)).launch_info()
    assert box["steps_per_launch"] == 7 and box["segment_rows"] >= 16
    box32 = gpu_solver(smooth_random_2d(1024, 1024, seed=8, bc=("wall",) * 4),
                       storage="f32").launch_info()
    assert 2 <= box32["steps_per_launch"] <= 8
    small_box = gpu_solver(smooth_random_2d(64, 64, seed=8, bc=("wall",) * 4)).launch_info()
    assert small_box["steps_per_launch"] == 1
    asked = gpu_solver(smooth_random_2d(300, 70, seed=8), fuse_steps=16).launch_info()
    assert asked["steps_per_launch"] == 8
    say(f"[plans] 1024^2 f64 {big64}, f32 {big32}, 256^2 f32 {small32}")


def test_launch_plan_spreads_the_remainder_and_keeps_the_state():
    """lbm_launch_plan lists the launches lbm_step issues.  2D at 8 steps per
    launch: a remainder of two or more steps is spread evenly over the last
    launches (20 -> 7, 7, 6; 10 -> 5, 5; 26 -> 7, 7, 6, 6), a remainder of one is a
    one-step launch (17 -> 8, 8, 1), captured chunks count launch by launch (64 ->
    eight launches of 8); 1D keeps the plain split (20 at 16 per launch -> 16, 4).
    The state after step(n) is bitwise the state after n single steps, on a ragged
    periodic grid in both storages and on a grid with faces (6 per launch: 20 ->
    5, 5, 5, 5)."""
    import torch

    per = smooth_random_2d(300, 70, seed=12)
    S = gpu_solver(per, fuse_steps=8)
    assert S.launch_plan(20) == [7, 7, 6]
    assert S.launch_plan(10) == [5, 5]
    assert S.launch_plan(26) == [7, 7, 6, 6]
    assert S.launch_plan(17) == [8, 8, 1]
    assert S.launch_plan(64) == [8] * 8
    assert S.launch_plan(42) == [7] * 6  # not a chunk of four 8s then 5 + 5
    long_plan = S.launch_plan(2002)
    assert (len(long_plan) == 251 and sum(long_plan) == 2002
            and set(long_plan) == {7, 8} and long_plan[:200] == [8] * 200)
    assert S.launch_plan(0) == [] and S.launch_plan(1) == [1] and S.launch_plan(8) == [8]
    assert gpu_solver(W.dam_break_1d(5000)).launch_plan(20) == [16, 4]
    assert gpu_solver(W.dam_break_1d(1000)).launch_plan(400) == [400]
    # state checks every 9 steps split a run into windows, each planned on its own
    # (a 9-step window: 8 + 1, the remainder of one step in the one-step kernel)
    Sc = gpu_solver(per, fuse_steps=8, check_every=9)
    assert Sc.launch_plan(20) == [8, 1, 8, 1, 2]
    Sc.step(3)
    assert Sc.launch_plan(20) == [6, 8, 1, 5]
    walls = W.oblique_shock_2d(20, steps=10)
    Sw = gpu_solver(walls, fuse_steps=6)
    assert Sw.launch_plan(20) == [5, 5, 5, 5]
    for case, storage, fuse, n in ((per, "f64", 8, 20), (per, "f32", 8, 26), (per, "f64", 8, 17),
                                   (walls, "f64", 6, 20)):
        A = gpu_solver(case, storage=storage, fuse_steps=fuse)
        B = gpu_solver(case, storage=storage, fuse_steps=1)
        A.step(n)
        B.step(n)
        torch.cuda.synchronize()
        assert torch.equal(A.planes(), B.planes()), (storage, fuse, n)
