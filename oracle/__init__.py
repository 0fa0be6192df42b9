"""CPU FP64 oracle of the vectorial lattice Boltzmann shallow-water scheme.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by ``__graft_entry__.smoke``
and by the CPU-baseline leg of ``bench.py``.  The GPU package never imports it.

The numerical work happens in ``lbm_oracle.c`` (built into ``liboracle.so`` by
``oracle/build.py``); this module only marshals numpy arrays through ctypes.
Exact solutions of the shallow-water Riemann problems are in ``oracle.exact``.

Population layout returned by :func:`run` (population-major, ``npop`` planes of
``ny*nx`` values, row-major ``[y][x]``):

* 1D (``npop = 5``): ``f0, f+, f-, g+, g-``  (Sec. 2, D1Q3Q2)
* 2D (``npop = 13``): ``f0, f1..f4, gx1..gx4, gy1..gy4`` with
  e1 = +x, e2 = +y, e3 = -x, e4 = -y (Sec. 3, eq. 3-stencil-d2q5, D2Q5Q4Q4)

At ``a = 0`` the rest population ``f0`` is identically zero and the remaining
planes are the D1Q2 / D2Q4 per-component distributions.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

BC = {"periodic": 0, "neumann": 1, "wall": 2, "inflow": 3}


class OrcParams(ctypes.Structure):
    _fields_ = [
        ("dim", ctypes.c_int),
        ("nx", ctypes.c_int),
        ("ny", ctypes.c_int),
        ("lam", ctypes.c_double),
        ("s", ctypes.c_double),
        ("g", ctypes.c_double),
        ("a", ctypes.c_double),
        ("bc", ctypes.c_int * 4),
        ("inflow", (ctypes.c_double * 3) * 4),
        ("mrt", ctypes.c_int),
        ("rates", ctypes.c_double * 10),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from . import build as _b

            _b.build()
        _lib = ctypes.CDLL(_LIB_PATH)
        dp = ctypes.POINTER(ctypes.c_double)
        pp = ctypes.POINTER(OrcParams)
        _lib.orc_feq.argtypes = [pp, ctypes.c_double, ctypes.c_double, ctypes.c_double, dp]
        _lib.orc_collide.argtypes = [pp, dp, dp]
        _lib.orc_run.argtypes = [pp, dp, dp, dp, ctypes.c_long, dp, dp]
        _lib.orc_advance.argtypes = [pp, dp, ctypes.c_long]
        _lib.orc_moments.argtypes = [pp, dp, dp, dp, dp]
        _lib.orc_adjoint_step.argtypes = [pp, dp, dp, dp, dp]
        _lib.orc_loss_grad_2d.argtypes = [pp, dp, dp, ctypes.c_long, ctypes.c_int, dp, dp, dp]
        _lib.orc_loss_grad.argtypes = [pp, dp, dp, ctypes.c_long, ctypes.c_int, dp, dp, dp]
        _lib.orc_step_cs.argtypes = [pp, dp, dp, ctypes.c_double, ctypes.c_double, dp]
        _lib.orc_loss_cs_2d.argtypes = [pp, dp, dp, ctypes.c_double, dp, ctypes.c_long,
                                        ctypes.c_double, dp, dp]
        _lib.orc_entropy.argtypes = [pp, dp, dp, dp, ctypes.POINTER(ctypes.c_long)]
        _lib.orc_entropy_pop.argtypes = [pp, ctypes.c_int, dp, dp, dp]
        _lib.orc_set_threads.argtypes = [ctypes.c_int]
        _lib.orc_set_threads.restype = None
        _lib.orc_get_threads.argtypes = []
        _lib.orc_get_threads.restype = ctypes.c_int
        for name in ("orc_feq", "orc_collide", "orc_run", "orc_advance", "orc_moments",
                     "orc_adjoint_step", "orc_loss_grad_2d", "orc_loss_grad", "orc_step_cs",
                     "orc_loss_cs_2d", "orc_entropy", "orc_entropy_pop"):
            getattr(_lib, name).restype = ctypes.c_int
    return _lib


def _dp(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


def params(dim, nx, ny=1, lam=3.0, s=1.8, g=1.0, a=0.0, bc=("periodic",) * 4,
           inflow=None, mrt=False, rates=None) -> OrcParams:
    """Build an oracle parameter block.  ``bc`` = faces (x-, x+, y-, y+) by name
    or code; ``inflow`` = {face_index: (h, qx, qy)}; ``rates`` = MRT rates."""
    P = OrcParams()
    P.dim, P.nx, P.ny = dim, nx, (ny if dim == 2 else 1)
    P.lam, P.s, P.g, P.a = lam, s, g, a
    for i, b in enumerate(bc):
        P.bc[i] = BC[b] if isinstance(b, str) else int(b)
    for face, w in (inflow or {}).items():
        for k in range(3):
            P.inflow[face][k] = w[k] if k < len(w) else 0.0
    P.mrt = 1 if mrt else 0
    rr = rates if rates is not None else [s] * 10
    for i in range(10):
        P.rates[i] = rr[i] if i < len(rr) else s
    return P


def set_threads(n):
    """Host threads of the oracle's parallel loops (results are independent of it)."""
    lib().orc_set_threads(int(n))


def get_threads():
    return int(lib().orc_get_threads())


def npop(dim):
    return 5 if dim == 1 else 13


def feq(P: OrcParams, h, qx=0.0, qy=0.0) -> np.ndarray:
    out = np.zeros(npop(P.dim))
    rc = lib().orc_feq(ctypes.byref(P), float(h), float(qx), float(qy), _dp(out))
    assert rc == 0
    return out


def collide(P: OrcParams, f) -> np.ndarray:
    f = _f64(f)
    out = np.zeros_like(f)
    assert lib().orc_collide(ctypes.byref(P), _dp(f), _dp(out)) == 0
    return out


def run(P: OrcParams, h0, qx0=None, qy0=None, nsteps=0, want_pre=False):
    """Post-collision state f*(nsteps) as an array (npop, ny, nx) (1D: (npop, nx));
    with ``want_pre`` also the pre-collision state f(nsteps)."""
    n = P.nx * P.ny
    h0 = _f64(h0).reshape(-1)
    qx0 = None if qx0 is None else _f64(qx0).reshape(-1)
    qy0 = None if qy0 is None else _f64(qy0).reshape(-1)
    assert h0.size == n
    out = np.zeros(npop(P.dim) * n)
    pre = np.zeros(npop(P.dim) * n) if want_pre else None
    rc = lib().orc_run(ctypes.byref(P), _dp(h0), _dp(qx0), _dp(qy0), int(nsteps), _dp(out), _dp(pre))
    if rc != 0:
        raise ValueError(f"orc_run failed ({rc})")
    shape = (npop(P.dim), P.nx) if P.dim == 1 else (npop(P.dim), P.ny, P.nx)
    if want_pre:
        return out.reshape(shape), pre.reshape(shape)
    return out.reshape(shape)


def advance(P: OrcParams, fstar, nsteps):
    """Advance a post-collision state (npop planes) by nsteps; returns a new array."""
    f = np.array(fstar, dtype=np.float64, order="C", copy=True)
    rc = lib().orc_advance(ctypes.byref(P), _dp(f.reshape(-1)), int(nsteps))
    if rc != 0:
        raise ValueError(f"orc_advance failed ({rc})")
    return f


def moments(P: OrcParams, f):
    """Conserved fields (h, qx[, qy]) of a distribution array."""
    f = _f64(f)
    n = P.nx * P.ny
    h, qx, qy = np.zeros(n), np.zeros(n), np.zeros(n)
    assert lib().orc_moments(ctypes.byref(P), _dp(f.reshape(-1)), _dp(h), _dp(qx), _dp(qy)) == 0
    if P.dim == 1:
        return h, qx
    return h.reshape(P.ny, P.nx), qx.reshape(P.ny, P.nx), qy.reshape(P.ny, P.nx)


def _field_shape(P):
    np_ = 5 if P.dim == 1 else 13
    return (np_, P.nx) if P.dim == 1 else (np_, P.ny, P.nx)


def adjoint_step(P: OrcParams, un, lam_np1):
    """One adjoint step (population-major layout: 5 populations in 1D, 13 in 2D),
    any face rules: returns (lam_n, dL/ds contribution)."""
    un = _f64(un).reshape(-1)
    lam_np1 = _f64(lam_np1).reshape(-1)
    lam_n = np.zeros_like(lam_np1)
    gs = ctypes.c_double(0.0)
    rc = lib().orc_adjoint_step(ctypes.byref(P), _dp(un), _dp(lam_np1), _dp(lam_n),
                                ctypes.byref(gs))
    if rc != 0:
        raise ValueError(f"orc_adjoint_step failed ({rc})")
    return lam_n.reshape(_field_shape(P)), gs.value


def step_directional(P: OrcParams, u, du=None, ds=0.0, eps=1e-30):
    """Directional derivative of one step between post-collision levels along
    (du, ds), by complex step of the forward code."""
    u = _f64(u).reshape(-1)
    du = None if du is None else _f64(du).reshape(-1)
    out = np.zeros_like(u)
    rc = lib().orc_step_cs(ctypes.byref(P), _dp(u), _dp(du), float(ds), float(eps), _dp(out))
    if rc != 0:
        raise ValueError(f"orc_step_cs failed ({rc})")
    return out.reshape(_field_shape(P))


def loss_grad(P: OrcParams, h0, hhat, T, K=23):
    """(loss, dL/dh0, dL/ds) for L = sum (h(T) - hhat)^2 from W0 = (h0, 0, 0), 1D or
    2D, any face rules."""
    h0 = _f64(h0).reshape(-1)
    hhat = _f64(hhat).reshape(-1)
    g = np.zeros_like(h0)
    loss, gs = ctypes.c_double(0.0), ctypes.c_double(0.0)
    rc = lib().orc_loss_grad(ctypes.byref(P), _dp(h0), _dp(hhat), int(T), int(K),
                             ctypes.byref(loss), _dp(g), ctypes.byref(gs))
    if rc != 0:
        raise ValueError(f"orc_loss_grad failed ({rc})")
    return loss.value, (g if P.dim == 1 else g.reshape(P.ny, P.nx)), gs.value


def loss_grad_2d(P: OrcParams, h0, hhat, T, K=23):
    """(loss, dL/dh0, dL/ds) for L = sum (h(T) - hhat)^2 from W0 = (h0, 0, 0)."""
    h0 = _f64(h0).reshape(-1)
    hhat = _f64(hhat).reshape(-1)
    g = np.zeros_like(h0)
    loss, gs = ctypes.c_double(0.0), ctypes.c_double(0.0)
    rc = lib().orc_loss_grad_2d(ctypes.byref(P), _dp(h0), _dp(hhat), int(T), int(K),
                                ctypes.byref(loss), _dp(g), ctypes.byref(gs))
    if rc != 0:
        raise ValueError(f"orc_loss_grad_2d failed ({rc})")
    return loss.value, g.reshape(P.ny, P.nx), gs.value


def loss_complex_step_2d(P: OrcParams, h0, hhat, T, dh0=None, ds=0.0, eps=1e-30):
    """(loss, directional derivative) by complex step along (dh0, ds); 1D or 2D,
    any face rules (the name predates the 1D case)."""
    h0 = _f64(h0).reshape(-1)
    hhat = _f64(hhat).reshape(-1)
    dh0 = None if dh0 is None else _f64(dh0).reshape(-1)
    loss, dl = ctypes.c_double(0.0), ctypes.c_double(0.0)
    rc = lib().orc_loss_cs_2d(ctypes.byref(P), _dp(h0), _dp(dh0), float(ds), _dp(hhat), int(T),
                              float(eps), ctypes.byref(loss), ctypes.byref(dl))
    if rc != 0:
        raise ValueError(f"orc_loss_cs_2d failed ({rc})")
    return loss.value, dl.value


def entropy(P: OrcParams, f):
    """Discrete microscopic entropy of a distribution (a = 0): returns
    (per-node H, total H, number of populations outside the convexity domain)."""
    f = _f64(f).reshape(-1)
    n = P.nx * P.ny
    hn = np.zeros(n)
    tot = ctypes.c_double(0.0)
    bad = ctypes.c_long(0)
    rc = lib().orc_entropy(ctypes.byref(P), _dp(f), _dp(hn), ctypes.byref(tot), ctypes.byref(bad))
    if rc != 0:
        raise ValueError(f"orc_entropy failed ({rc})")
    return (hn if P.dim == 1 else hn.reshape(P.ny, P.nx)), tot.value, bad.value


def entropy_pop(P: OrcParams, j, F):
    """Entropy of one population j (1D: 0 = +, 1 = -; 2D: 0..3 = e_1..e_4) with
    components F.  Returns (valid, h, phi)."""
    F = _f64(F)
    h = ctypes.c_double(0.0)
    phi = np.zeros(3)
    rc = lib().orc_entropy_pop(ctypes.byref(P), int(j), _dp(F), ctypes.byref(h), _dp(phi))
    if rc < 0:
        raise ValueError(f"orc_entropy_pop failed ({rc})")
    return rc == 0, h.value, phi[: (2 if P.dim == 1 else 3)]


def to_hotpath_planes(f):
    """Drop the rest population: the 4 (1D) or 12 (2D) moving-population planes,
    in the order (h: e1..e4, qx: e1..e4, qy: e1..e4) / (h: +, -; q: +, -)."""
    return np.ascontiguousarray(f[1:])
