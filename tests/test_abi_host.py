"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every symbol include/lbm.h declares, computes layouts and rejects bad
arguments before touching device memory."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _header_symbols():
    src = open(os.path.join(ROOT, "include", "lbm.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(lbm_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def L():
    from paper_1401_0427_amd import lbm

    return lbm


def test_every_declared_symbol_is_exported(L):
    lib = L.load()
    syms = _header_symbols()
    assert len(syms) >= 20
    for s in syms:
        assert hasattr(lib, s), s
    assert set(syms) == set(L.EXPORTS)


def test_layout_pads_planes(L):
    p = L.make_params(2, 4096, 4096, 6.0, 1.8)
    ps, npl, nb = L.layout(p)
    assert npl == 12 and ps >= 4096 * 4096 and ps % 64 == 0
    assert ps != 4096 * 4096  # padded: no power-of-two plane stride
    assert nb == ps * 12 * 8
    p = L.make_params(1, 1 << 20, 1, 3.0, 1.8, storage="f32", plane_pad=0)
    ps, npl, nb = L.layout(p)
    assert (ps, npl, nb) == (1 << 20, 4, (1 << 20) * 4 * 4)


@pytest.mark.parametrize("bad", [dict(s=2.0), dict(s=0.0), dict(lam=-1.0), dict(g=0.0),
                                 dict(nx=1), dict(bc=("periodic", "wall", "periodic", "periodic")),
                                 dict(block=100), dict(npt=3), dict(fuse_steps=1025),
                                 dict(fuse_steps=4096), dict(fuse_steps=-1),
                                 dict(bc=("inflow", "wall", "periodic", "periodic"), inflow={0: (0.0, 0, 0)}),
                                 dict(adjoint_storage="f32"), dict(adjoint_storage=16)])
def test_init_rejects_bad_parameters_without_touching_memory(L, bad):
    kw = dict(dim=2, nx=64, ny=64, lam=6.0, s=1.8)
    kw.update(bad)
    p = L.make_params(kw.pop("dim"), kw.pop("nx"), kw.pop("ny"), kw.pop("lam"), kw.pop("s"), **kw)
    # non-null dummy pointers: validation must fail before any device access
    p.f_a, p.f_b = 0x1000, 0x2000
    ctx = ctypes.c_void_p()
    rc = L.load().lbm_init(ctypes.byref(p), ctypes.c_void_p(0x3000), None, None, ctypes.byref(ctx))
    assert rc == L.LBM_EINVAL, L.last_error()
    assert not ctx.value
    assert L.last_error()


def test_init_rejects_null_pointers(L):
    p = L.make_params(2, 64, 64, 6.0, 1.8)
    ctx = ctypes.c_void_p()
    assert L.load().lbm_init(ctypes.byref(p), ctypes.c_void_p(0x3000), None, None,
                             ctypes.byref(ctx)) == L.LBM_EINVAL
    p.f_a, p.f_b = 0x1000, 0x1000
    assert L.load().lbm_init(ctypes.byref(p), ctypes.c_void_p(0x3000), None, None,
                             ctypes.byref(ctx)) == L.LBM_EINVAL


def test_null_context_is_an_error(L):
    lib = L.load()
    assert lib.lbm_step(None, 1) == L.LBM_ESTATE
    lib.lbm_destroy(None)  # NULL-safe
    lib.lbm_batch_destroy(None)


def test_batch_layout_offsets(L):
    arr = (L.LbmInstance * 3)()
    for i, (d, nx, ny) in enumerate([(1, 1000, 1), (2, 130, 129), (1, 7, 1)]):
        arr[i].lattice = L.D1Q2x2 if d == 1 else L.D2Q4x3
        arr[i].nx, arr[i].ny = nx, ny
    nb, nodes = ctypes.c_size_t(), ctypes.c_long()
    assert L.load().lbm_batch_layout(arr, 3, L.F32, ctypes.byref(nb), ctypes.byref(nodes)) == 0
    assert nodes.value == 1000 + 130 * 129 + 7
    assert arr[0].state_offset == 0 and arr[1].state_offset == 1024 * 4
    assert arr[2].state_offset == 1024 * 4 + 16832 * 12
    assert [a.node_offset for a in arr] == [0, 1000, 1000 + 130 * 129]
    assert nb.value == (1024 * 4 + 16832 * 12 + 64 * 4) * 4


def test_batch_create_rejects_bad_step_synchronous_tuning(L):
    """Mode 1 (one grid barrier per step) needs a workgroup size that is a
    multiple of 64 in [64, 512]; a bad one is rejected before any device call."""
    arr = (L.LbmInstance * 1)()
    arr[0].lattice, arr[0].nx, arr[0].ny = L.D2Q4x3, 64, 64
    arr[0].lam, arr[0].s, arr[0].g = 6.0, 1.8, 1.0
    nb, nodes = ctypes.c_size_t(), ctypes.c_long()
    lib = L.load()
    assert lib.lbm_batch_layout(arr, 1, L.F32, ctypes.byref(nb), ctypes.byref(nodes)) == 0
    tune = L.LbmBatchTuning(100, 16384, 0, 1, 1, 0)
    b = ctypes.c_void_p()
    rc = lib.lbm_batch_create(arr, 1, L.F32, ctypes.c_void_p(0x1000), ctypes.c_void_p(0x2000),
                              None, ctypes.byref(tune), ctypes.byref(b))
    assert rc == L.LBM_EINVAL and not b.value
    assert "block" in L.last_error()


@pytest.mark.parametrize("bad", [dict(mode=3, fuse=1), dict(mode=3, fuse=9), dict(mode=4, fuse=1),
                                 dict(mode=4, fuse=9), dict(mode=5), dict(mode=-1)])
def test_batch_create_rejects_bad_fused_mode(L, bad):
    """Modes 3 and 4 take 2 .. 8 steps per launch / pass (0: the default);
    unknown modes are rejected."""
    arr = (L.LbmInstance * 1)()
    arr[0].lattice, arr[0].nx, arr[0].ny = L.D2Q4x3, 64, 64
    arr[0].lam, arr[0].s, arr[0].g = 6.0, 1.8, 1.0
    nb, nodes = ctypes.c_size_t(), ctypes.c_long()
    lib = L.load()
    assert lib.lbm_batch_layout(arr, 1, L.F32, ctypes.byref(nb), ctypes.byref(nodes)) == 0
    tune = L.LbmBatchTuning(256, 16384, 0, 1, bad["mode"], bad.get("fuse", 0))
    b = ctypes.c_void_p()
    rc = lib.lbm_batch_create(arr, 1, L.F32, ctypes.c_void_p(0x1000), ctypes.c_void_p(0x2000),
                              None, ctypes.byref(tune), ctypes.byref(b))
    assert rc == L.LBM_EINVAL and not b.value
    assert L.last_error()
