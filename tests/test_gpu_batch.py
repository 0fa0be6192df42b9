"""Batched persistent launch vs the oracle, instance by instance."""
import numpy as np
import pytest

import oracle
from gpu_helpers import l1_rel, normwise_rel, say, to_np
from paper_1401_0427_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1401_0427_amd import lbm

    lbm.load()


def instance_dicts(manifest):
    out = []
    for m in manifest:
        h, qx, qy = m.initial()
        bc = ("neumann", "neumann", "periodic", "periodic") if m.dim == 1 else ("periodic",) * 4
        out.append(dict(dim=m.dim, nx=m.nx, ny=m.ny, lam=m.lam, s=m.s, g=W.G, bc=bc, h0=h,
                        qx0=qx, qy0=qy))
    return out


def oracle_moments(d, steps):
    P = oracle.params(d["dim"], d["nx"], d["ny"], lam=d["lam"], s=d["s"], g=d["g"], bc=d["bc"])
    f = oracle.run(P, d["h0"], d["qx0"], d["qy0"] if d["dim"] == 2 else None, steps)
    return oracle.moments(P, f)


@pytest.mark.parametrize("tune", [dict(block=256, tile_nodes=256), dict(block=64, tile_nodes=100),
                                  dict(block=512, tile_nodes=4096, grid=7)])
def test_batch_small_manifest_fp64_matches_oracle(tune):
    from paper_1401_0427_amd.lbm import Batch

    insts = instance_dicts(W.small_manifest(seed=1))
    steps = 157
    say(f"[batch] {len(insts)} instances, {steps} steps, {tune}")
    B = Batch(insts, storage="f64", **tune)
    nt, grid = B.info()
    say(f"  tiles {nt}, grid {grid}")
    B.run(steps)
    h, qx, qy = (to_np(t) for t in B.moments())
    worst = 0.0
    for i, d in enumerate(insts):
        ref = oracle_moments(d, steps)
        got = [to_np(B.instance_view(i, t)) for t in B.moments()[: 2 if d["dim"] == 1 else 3]]
        e = max(normwise_rel(a, b) for a, b in zip(got, ref))
        worst = max(worst, e)
    say(f"  worst instance rel err {worst:.3e}")
    assert worst <= 1e-12


def test_batch_run_twice_equals_one_long_run():
    from paper_1401_0427_amd.lbm import Batch

    insts = instance_dicts(W.small_manifest(seed=2))
    A = Batch(insts, storage="f64", tile_nodes=256)
    B = Batch(insts, storage="f64", tile_nodes=256)
    A.run(51)
    A.run(50)
    B.run(101)
    for a, b in zip(A.moments(), B.moments()):
        assert np.array_equal(to_np(a), to_np(b))


def test_batch_fp32_l1():
    from paper_1401_0427_amd.lbm import Batch

    insts = instance_dicts(W.small_manifest(seed=3))
    steps = 300
    B = Batch(insts, storage="f32", tile_nodes=512)
    B.run(steps)
    worst = 0.0
    hs = B.moments()[0]
    for i, d in enumerate(insts):
        ref = oracle_moments(d, steps)[0]
        worst = max(worst, l1_rel(to_np(B.instance_view(i, hs)), ref))
    say(f"[batch fp32] worst L1 rel of h {worst:.3e}")
    assert worst <= 1e-5
