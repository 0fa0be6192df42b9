"""The benchmark workload at its stated length against one full-grid oracle run.

2D radial dam break on 4096 x 4096 periodic nodes (lambda = 6, s = 1.8,
Sec. 3 scheme at a = 0, BGK relaxation of eq. 2-relaxation), 2000 steps, in
the launch plan the library picks by default and the benchmark times (FP64:
8 steps per launch).  The oracle advances the same initial state on the host
cores, and at eight checkpoints (every 256 steps, then 2000) every one of the
12 distribution planes of the FP64 run is compared element by element
(normwise relative error per plane <= 1e-12), and the L1 error of h of the
FP32-storage run is stated and bounded (<= 1e-5).

The tests share one oracle state and one pair of GPU solvers and must run in
file order; each advances them to its own checkpoint, so a single test run
alone still compares at its step count."""
import time

import numpy as np
import pytest

import oracle
from gpu_helpers import l1_rel, say
from paper_1401_0427_amd import workloads as W

pytestmark = pytest.mark.gpu

N = 4096
CHECKPOINTS = [256, 512, 768, 1024, 1280, 1536, 1792, 2000]


@pytest.fixture(scope="module")
def run():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1401_0427_amd.lbm import Solver

    case = W.radial_dam_break_2d(N, lam=6.0)
    P = oracle.params(2, N, N, lam=case.lam, s=case.s, g=case.g)
    t0 = time.time()
    f = oracle.run(P, case.h0, case.qx0, case.qy0, 0)
    say(f"[headline] oracle level 0 in {time.time() - t0:.1f} s")
    kw = dict(lam=case.lam, s=case.s, g=case.g, h0=case.h0, qx0=case.qx0, qy0=case.qy0)
    S64 = Solver(2, N, N, storage="f64", **kw)
    S32 = Solver(2, N, N, storage="f32", **kw)
    say(f"[headline] GPU launch plans: FP64 {S64.launch_info()}, FP32 {S32.launch_info()}")
    st = dict(P=P, f=f, step=0, S64=S64, S32=S32, l1=[])
    yield st
    del st["S64"], st["S32"]
    torch.cuda.empty_cache()


@pytest.mark.parametrize("target", CHECKPOINTS)
def test_radial_4096_matches_full_grid_oracle(run, target):
    import torch

    n = target - run["step"]
    assert n > 0, "checkpoints run in increasing order"
    t0 = time.time()
    run["S64"].step(n)
    run["S32"].step(n)
    torch.cuda.synchronize()
    t1 = time.time()
    run["f"] = oracle.advance(run["P"], run["f"], n)
    run["step"] = target
    t2 = time.time()
    ref = run["f"]
    assert np.all(ref[0] == 0.0)  # a = 0: the rest population stays zero
    got = run["S64"].planes().cpu().numpy()
    worst, worst_pl = 0.0, -1
    for pl in range(12):
        b = ref[pl + 1]
        d = np.abs(got[pl] - b).max()
        e = 0.0 if d == 0 else d / np.abs(b).max()
        if e > worst:
            worst, worst_pl = e, pl
    del got
    h_ref = oracle.moments(run["P"], ref)[0]
    h32 = run["S32"].moments()[0].cpu().numpy()
    e32 = l1_rel(h32, h_ref)
    run["l1"].append((target, e32))
    say(f"[headline] step {target}: GPU {t1 - t0:.1f} s, oracle {t2 - t1:.1f} s; FP64 max plane "
        f"rel err {worst:.3e} (plane {worst_pl}); FP32 L1 rel of h {e32:.3e}")
    assert worst <= 1e-12
    assert e32 <= 1e-5
