"""ctypes binding of liblbm.so (declared in include/lbm.h).

Argument marshalling only: every step of the path runs in the library's HIP
kernels.  PyTorch provides device memory (tensors own every state, field and
adjoint buffer) and the stream (the current torch stream at construction).

The library is loaded on first use.  If it is missing, or no GPU is visible,
calls raise instead of falling back to anything else.
"""
from __future__ import annotations

import ctypes
import os
import warnings

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblbm.so")

LBM_OK, LBM_WARN_SUBCHAR = 0, 1
LBM_EINVAL, LBM_EDEVICE, LBM_ESTATE, LBM_EDIVERGED = -1, -2, -3, -4
D1Q2x2, D2Q4x3, D1Q3Q2, D2Q5Q4Q4 = 1, 2, 3, 4
F64, F32 = 64, 32
BC = {"periodic": 0, "neumann": 1, "wall": 2, "inflow": 3}


class LbmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"liblbm error {code}: {msg}")
        self.code = code


class LbmParams(ctypes.Structure):
    _fields_ = [
        ("lattice", ctypes.c_int),
        ("storage", ctypes.c_int),
        ("nx", ctypes.c_int),
        ("ny", ctypes.c_int),
        ("lam", ctypes.c_double),
        ("s", ctypes.c_double),
        ("g", ctypes.c_double),
        ("a", ctypes.c_double),
        ("rates", ctypes.c_double * 10),
        ("bc", ctypes.c_int * 4),
        ("inflow", (ctypes.c_double * 3) * 4),
        ("check_every", ctypes.c_int),
        ("block", ctypes.c_int),
        ("nodes_per_thread", ctypes.c_int),
        ("plane_pad", ctypes.c_long),
        ("mem_hints", ctypes.c_int),
        ("fuse_steps", ctypes.c_int),
        ("f_a", ctypes.c_void_p),
        ("f_b", ctypes.c_void_p),
        ("stream", ctypes.c_void_p),
        ("adjoint_storage", ctypes.c_int),
    ]


class LbmInstance(ctypes.Structure):
    _fields_ = [
        ("lattice", ctypes.c_int),
        ("nx", ctypes.c_int),
        ("ny", ctypes.c_int),
        ("lam", ctypes.c_double),
        ("s", ctypes.c_double),
        ("g", ctypes.c_double),
        ("bc", ctypes.c_int * 4),
        ("inflow", (ctypes.c_double * 3) * 4),
        ("state_offset", ctypes.c_long),
        ("node_offset", ctypes.c_long),
    ]


class LbmBatchTuning(ctypes.Structure):
    _fields_ = [("block", ctypes.c_int), ("tile_nodes", ctypes.c_int), ("grid", ctypes.c_int),
                ("pass_nodes", ctypes.c_int), ("mode", ctypes.c_int), ("fuse_steps", ctypes.c_int),
                ("direct", ctypes.c_int)]


EXPORTS = [
    "lbm_layout", "lbm_init", "lbm_step", "lbm_step_buffers", "lbm_current",
    "lbm_launch_info", "lbm_launch_plan", "lbm_export", "lbm_adjoint_segment",
    "lbm_step_levels", "lbm_adjoint_levels",
    "lbm_import", "lbm_moments", "lbm_moments_noalloc", "lbm_entropy", "lbm_adjoint_step", "lbm_adjoint_partials",
    "lbm_adjoint_terminal", "lbm_adjoint_grad_w0", "lbm_sum", "lbm_destroy",
    "lbm_batch_layout", "lbm_batch_create", "lbm_batch_init", "lbm_batch_run",
    "lbm_batch_moments", "lbm_batch_current", "lbm_batch_info", "lbm_batch_check",
    "lbm_batch_destroy",
    "lbm_last_error", "lbm_version",
]

_lib = None


def load(path: str = LIB_PATH):
    """Load liblbm.so and declare the signatures of include/lbm.h."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"liblbm.so not found at {path}; build it with "
                           "`python -m paper_1401_0427_amd.build` (there is no fallback)")
    L = ctypes.CDLL(path)
    vp, dp, ip, lp = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.c_int, ctypes.c_long
    P = ctypes.POINTER(LbmParams)
    sig = {
        "lbm_layout": (ip, [P, ctypes.POINTER(ctypes.c_long), ctypes.POINTER(ctypes.c_int),
                            ctypes.POINTER(ctypes.c_size_t)]),
        "lbm_init": (ip, [P, vp, vp, vp, ctypes.POINTER(vp)]),
        "lbm_step": (ip, [vp, lp]),
        "lbm_step_buffers": (ip, [vp, vp, vp]),
        "lbm_current": (ip, [vp, ctypes.POINTER(vp), ctypes.POINTER(ctypes.c_long)]),
        "lbm_launch_info": (ip, [vp, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int),
                                 ctypes.POINTER(ctypes.c_long)]),
        "lbm_launch_plan": (ip, [vp, lp, ctypes.POINTER(ctypes.c_int), ip,
                                 ctypes.POINTER(ctypes.c_long)]),
        "lbm_export": (ip, [vp, vp]),
        "lbm_step_levels": (ip, [vp, vp, ip, vp]),
        "lbm_adjoint_levels": (ip, [vp, vp, ip, vp, vp, vp, ctypes.POINTER(ctypes.c_int)]),
        "lbm_import": (ip, [vp, vp]),
        "lbm_moments": (ip, [vp, vp, vp, vp, vp, dp]),
        "lbm_moments_noalloc": (ip, [P, vp, vp, vp, vp, vp]),
        "lbm_entropy": (ip, [vp, vp, vp, dp, ctypes.POINTER(ctypes.c_long)]),
        "lbm_adjoint_step": (ip, [vp, vp, vp, vp, vp]),
        "lbm_adjoint_partials": (lp, [vp]),
        "lbm_adjoint_segment": (ip, [vp, vp, ip, vp, vp, vp, vp, ctypes.POINTER(ctypes.c_int)]),
        "lbm_adjoint_terminal": (ip, [vp, vp, vp]),
        "lbm_adjoint_grad_w0": (ip, [vp, vp, vp, vp, vp, vp, vp, vp]),
        "lbm_sum": (ip, [vp, vp, lp, dp]),
        "lbm_destroy": (None, [vp]),
        "lbm_batch_layout": (ip, [ctypes.POINTER(LbmInstance), ip, ip,
                                  ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(ctypes.c_long)]),
        "lbm_batch_create": (ip, [ctypes.POINTER(LbmInstance), ip, ip, vp, vp, vp,
                                  ctypes.POINTER(LbmBatchTuning), ctypes.POINTER(vp)]),
        "lbm_batch_init": (ip, [vp, vp, vp, vp]),
        "lbm_batch_run": (ip, [vp, lp]),
        "lbm_batch_moments": (ip, [vp, vp, vp, vp]),
        "lbm_batch_current": (ip, [vp, ctypes.POINTER(vp), ctypes.POINTER(ctypes.c_long)]),
        "lbm_batch_info": (ip, [vp, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)]),
        "lbm_batch_check": (ip, [vp]),
        "lbm_batch_destroy": (None, [vp]),
        "lbm_last_error": (ctypes.c_char_p, []),
        "lbm_version": (ctypes.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


def last_error() -> str:
    return load().lbm_last_error().decode()


def check(rc: int, what: str = ""):
    if rc < 0:
        raise LbmError(rc, (what + ": " if what else "") + last_error())
    if rc > 0:
        warnings.warn(f"liblbm warning {rc}: {last_error()}", RuntimeWarning, stacklevel=3)
    return rc


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream_handle(torch):
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _require_gpu(torch):
    if not torch.cuda.is_available():
        raise RuntimeError("liblbm needs a visible GPU (no CPU fallback exists)")


def _field(torch, a, device):
    """Flat contiguous float64 device copy of a field (numpy array or tensor)."""
    if a is None:
        return None
    if isinstance(a, torch.Tensor):
        t = a.detach().to(device=device, dtype=torch.float64)
    else:
        t = torch.as_tensor(np.asarray(a, dtype=np.float64), device=device)
    return t.reshape(-1).contiguous()


def _bc_codes(bc):
    return [BC[b] if isinstance(b, str) else int(b) for b in bc]


def make_params(dim, nx, ny, lam, s, g=1.0, bc=("periodic",) * 4, inflow=None, storage="f64",
                check_every=0, block=256, npt=1, plane_pad=-1, mem_hints=-1, rest=False, a=0.0,
                rates=None, fuse_steps=0, adjoint_storage=None) -> LbmParams:
    """Parameter block; ``rest`` selects the rest-population schemes D1Q3Q2 /
    D2Q5Q4Q4 (weight ``a``, MRT ``rates``; 0 / missing rates take ``s``)."""
    p = LbmParams()
    if rest:
        p.lattice = D1Q3Q2 if dim == 1 else D2Q5Q4Q4
    else:
        p.lattice = D1Q2x2 if dim == 1 else D2Q4x3
    p.a = a
    for i, r in enumerate(rates or []):
        p.rates[i] = r
    p.storage = F32 if storage in ("f32", F32) else F64
    p.nx, p.ny = nx, (ny if dim == 2 else 1)
    p.lam, p.s, p.g = lam, s, g
    codes = _bc_codes(bc)
    for i in range(4):
        p.bc[i] = codes[i] if i < len(codes) else 0
    for face, w in (inflow or {}).items():
        for k in range(3):
            p.inflow[face][k] = w[k] if k < len(w) else 0.0
    p.check_every = check_every
    p.block = block
    p.nodes_per_thread = npt
    p.plane_pad = plane_pad
    p.mem_hints = mem_hints
    p.fuse_steps = fuse_steps
    p.adjoint_storage = {None: 0, "f64": F64, "f32": F32}.get(adjoint_storage, adjoint_storage)
    return p


def moments_noalloc(p: LbmParams, state, h=None, qx=None, qy=None, totals=None):
    """lbm_moments_noalloc: conserved fields and FP64 totals of a state in the
    layout of ``p``, enqueued on ``p.stream`` with no allocation and no
    synchronisation.  ``state``, ``h``, ``qx``, ``qy``, ``totals`` are device
    tensors (float64 for the outputs; ``totals`` holds 3 values)."""
    check(load().lbm_moments_noalloc(ctypes.byref(p), _ptr(state), _ptr(h), _ptr(qx), _ptr(qy),
                                     _ptr(totals)), "lbm_moments_noalloc")


def layout(p: LbmParams):
    ps, npl, nb = ctypes.c_long(), ctypes.c_int(), ctypes.c_size_t()
    check(load().lbm_layout(ctypes.byref(p), ctypes.byref(ps), ctypes.byref(npl), ctypes.byref(nb)),
          "lbm_layout")
    return ps.value, npl.value, nb.value


class Solver:
    """One problem on the GPU: owns (via torch) two state buffers."""

    def __init__(self, dim, nx, ny=1, lam=3.0, s=1.8, g=1.0, bc=("periodic",) * 4, inflow=None,
                 h0=None, qx0=None, qy0=None, storage="f64", check_every=0, block=256, npt=1,
                 plane_pad=-1, mem_hints=-1, rest=False, a=0.0, rates=None, fuse_steps=0,
                 adjoint_storage=None, device="cuda"):
        import torch

        _require_gpu(torch)
        L = load()
        self.torch = torch
        self.dim = dim
        self.nx, self.ny = nx, (ny if dim == 2 else 1)
        self.params = make_params(dim, nx, ny, lam, s, g, bc, inflow, storage, check_every, block,
                                  npt, plane_pad, mem_hints, rest, a, rates, fuse_steps,
                                  adjoint_storage)
        self.ps, self.nplanes, self.nbytes = layout(self.params)
        self.dtype = torch.float32 if self.params.storage == F32 else torch.float64
        a32 = self.params.adjoint_storage == F32 or (self.params.adjoint_storage == 0
                                                     and self.params.storage == F32)
        self.adj_dtype = torch.float32 if a32 else torch.float64
        self.device = torch.device(device)
        self.fa = torch.empty(self.nplanes * self.ps, dtype=self.dtype, device=self.device)
        self.fb = torch.empty_like(self.fa)
        self.params.f_a = self.fa.data_ptr()
        self.params.f_b = self.fb.data_ptr()
        self.params.stream = _stream_handle(torch).value
        n = self.nx * self.ny
        self.h0 = _field(torch, h0, self.device)
        self.qx0 = _field(torch, qx0, self.device)
        self.qy0 = None if dim == 1 else _field(torch, qy0, self.device)
        for t in (self.h0, self.qx0, self.qy0):
            if t is not None and t.numel() != n:
                raise ValueError("initial field size does not match the grid")
        ctx = ctypes.c_void_p()
        rc = L.lbm_init(ctypes.byref(self.params), _ptr(self.h0), _ptr(self.qx0), _ptr(self.qy0),
                        ctypes.byref(ctx))
        self.init_status = rc
        self.ctx = ctx
        check(rc, "lbm_init")

    # -- stepping ------------------------------------------------------------------
    def step(self, n=1):
        check(load().lbm_step(self.ctx, int(n)), "lbm_step")

    def step_buffers(self, src, dst):
        check(load().lbm_step_buffers(self.ctx, _ptr(src), _ptr(dst)), "lbm_step_buffers")

    def current(self):
        """(flat tensor holding the current state, steps done)."""
        ptr, steps = ctypes.c_void_p(), ctypes.c_long()
        check(load().lbm_current(self.ctx, ctypes.byref(ptr), ctypes.byref(steps)))
        buf = self.fa if ptr.value == self.fa.data_ptr() else self.fb
        return buf, steps.value

    def launch_info(self):
        """dict(steps_per_launch, segment_rows, resident_blocks) chosen at init."""
        k, seg, res = ctypes.c_int(), ctypes.c_int(), ctypes.c_long()
        check(load().lbm_launch_info(self.ctx, ctypes.byref(k), ctypes.byref(seg),
                                     ctypes.byref(res)), "lbm_launch_info")
        return dict(steps_per_launch=k.value, segment_rows=seg.value,
                    resident_blocks=res.value)

    def launch_plan(self, nsteps):
        """Steps of each launch that step(nsteps) issues from the current step count."""
        n = ctypes.c_long()
        check(load().lbm_launch_plan(self.ctx, nsteps, None, 0, ctypes.byref(n)),
              "lbm_launch_plan")
        ks = (ctypes.c_int * max(n.value, 1))()
        check(load().lbm_launch_plan(self.ctx, nsteps, ks, n.value, ctypes.byref(n)),
              "lbm_launch_plan")
        return list(ks[:n.value])

    def planes(self, buf=None):
        """(nplanes, ny, nx) view (1D: (nplanes, nx)) of a state buffer."""
        if buf is None:
            buf = self.current()[0]
        if self.dim == 1:
            return buf.as_strided((self.nplanes, self.nx), (self.ps, 1))
        return buf.as_strided((self.nplanes, self.ny, self.nx), (self.ps, self.nx, 1))

    def new_state(self, count=1):
        """Zeroed buffer of ``count`` consecutive states in this layout."""
        return self.torch.zeros(count * self.nplanes * self.ps, dtype=self.dtype,
                                device=self.device)

    def new_adjoint(self):
        """Zeroed adjoint buffer (state layout, the context's adjoint storage)."""
        return self.torch.zeros(self.nplanes * self.ps, dtype=self.adj_dtype, device=self.device)

    def export(self, dst):
        check(load().lbm_export(self.ctx, _ptr(dst)), "lbm_export")

    def import_(self, src):
        check(load().lbm_import(self.ctx, _ptr(src)), "lbm_import")

    def moments(self, state=None, totals=False):
        """Conserved fields (h, qx[, qy]) as device float64 tensors; with
        ``totals`` also their sums (host floats)."""
        torch = self.torch
        shape = (self.nx,) if self.dim == 1 else (self.ny, self.nx)
        h = torch.empty(shape, dtype=torch.float64, device=self.device)
        qx = torch.empty_like(h)
        qy = torch.empty_like(h) if self.dim == 2 else None
        tot = (ctypes.c_double * 3)() if totals else None
        check(load().lbm_moments(self.ctx, _ptr(state), _ptr(h), _ptr(qx), _ptr(qy), tot),
              "lbm_moments")
        out = (h, qx) if self.dim == 1 else (h, qx, qy)
        if totals:
            return out, (tot[0], tot[1], tot[2])
        return out

    def entropy(self, state=None, per_node=False):
        """Discrete microscopic entropy of a state (default: the current one):
        returns (total, number of populations outside the convexity domain) and,
        with ``per_node``, the per-node entropies as a device float64 tensor."""
        torch = self.torch
        hn = None
        if per_node:
            shape = (self.nx,) if self.dim == 1 else (self.ny, self.nx)
            hn = torch.empty(shape, dtype=torch.float64, device=self.device)
        tot = ctypes.c_double(0.0)
        bad = ctypes.c_long(0)
        check(load().lbm_entropy(self.ctx, _ptr(state), _ptr(hn), ctypes.byref(tot),
                                 ctypes.byref(bad)), "lbm_entropy")
        if per_node:
            return tot.value, bad.value, hn
        return tot.value, bad.value

    # -- adjoint -------------------------------------------------------------------------
    def adjoint_partials(self):
        n = load().lbm_adjoint_partials(self.ctx)
        return self.torch.zeros(n, dtype=self.torch.float64, device=self.device)

    def adjoint_step(self, f_n, lam_np1, lam_n, partials):
        check(load().lbm_adjoint_step(self.ctx, _ptr(f_n), _ptr(lam_np1), _ptr(lam_n),
                                      _ptr(partials)), "lbm_adjoint_step")

    def adjoint_segment(self, ck, nsteps, work, lam_a, lam_b, partials):
        """lbm_adjoint_segment: recompute a checkpoint segment into ``work`` and run
        its ``nsteps`` adjoint steps; returns 0 / 1 = lam_a / lam_b holds the result."""
        out = ctypes.c_int(-1)
        check(load().lbm_adjoint_segment(self.ctx, _ptr(ck), int(nsteps), _ptr(work), _ptr(lam_a),
                                         _ptr(lam_b), _ptr(partials), ctypes.byref(out)),
              "lbm_adjoint_segment")
        return out.value

    def step_levels(self, src, nsteps, levels):
        """lbm_step_levels: ``nsteps`` single steps from ``src``, level i into slot
        i - 1 of ``levels``."""
        check(load().lbm_step_levels(self.ctx, _ptr(src), int(nsteps), _ptr(levels)),
              "lbm_step_levels")

    def adjoint_levels(self, levels, nsteps, lam_a, lam_b, partials):
        """lbm_adjoint_levels: ``nsteps`` adjoint steps over stored levels; returns
        0 / 1 = lam_a / lam_b holds the result."""
        out = ctypes.c_int(-1)
        check(load().lbm_adjoint_levels(self.ctx, _ptr(levels), int(nsteps), _ptr(lam_a),
                                        _ptr(lam_b), _ptr(partials), ctypes.byref(out)),
              "lbm_adjoint_levels")
        return out.value

    def adjoint_terminal(self, dLdh, lam_T):
        dLdh = dLdh.to(dtype=self.torch.float64).contiguous()
        check(load().lbm_adjoint_terminal(self.ctx, _ptr(dLdh), _ptr(lam_T)), "lbm_adjoint_terminal")

    def adjoint_grad_w0(self, lam0, h0=None, qx0=None, qy0=None):
        torch = self.torch
        h0 = self.h0 if h0 is None else h0
        qx0 = self.qx0 if qx0 is None else qx0
        qy0 = self.qy0 if qy0 is None else qy0
        shape = (self.nx,) if self.dim == 1 else (self.ny, self.nx)
        gh = torch.empty(shape, dtype=torch.float64, device=self.device)
        gx = torch.empty_like(gh)
        gy = torch.empty_like(gh) if self.dim == 2 else None
        check(load().lbm_adjoint_grad_w0(self.ctx, _ptr(lam0), _ptr(h0), _ptr(qx0), _ptr(qy0),
                                         _ptr(gh), _ptr(gx), _ptr(gy)), "lbm_adjoint_grad_w0")
        return gh, gx, gy

    def sum(self, partials):
        out = ctypes.c_double()
        check(load().lbm_sum(self.ctx, _ptr(partials), int(partials.numel()), ctypes.byref(out)),
              "lbm_sum")
        return out.value

    def close(self):
        if getattr(self, "ctx", None) and self.ctx.value:
            load().lbm_destroy(self.ctx)
            self.ctx = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Many independent problems advanced in one persistent launch."""

    def __init__(self, instances, storage="f32", block=256, tile_nodes=16384, grid=0, pass_nodes=1,
                 mode=4, fuse_steps=0, direct=0, device="cuda"):
        """``instances``: iterable of dicts with keys dim, nx, ny, lam, s, g, bc,
        inflow, h0, qx0, qy0 (numpy arrays of the instance's nodes).  ``mode`` 0 is
        the dataflow persistent launch, 1 the step-synchronous persistent launch
        (one grid barrier per step), 2 one flat launch per step, 3 ``fuse_steps``
        steps per launch (0 = library default), 4 the tiles of mode 3 in one
        persistent launch (``fuse_steps`` steps per pass, one grid barrier per
        pass).  The default is mode 4, the fastest on the 256-instance manifest
        (mode 3 is within 1-2 %; modes 0 and 1 are several times slower but need no
        multi-step kernel).  ``direct`` launches every kernel directly instead of
        replaying captured graphs (e.g. under a profiler)."""
        import torch

        _require_gpu(torch)
        L = load()
        self.torch = torch
        insts = list(instances)
        n = len(insts)
        arr = (LbmInstance * n)()
        for i, d in enumerate(insts):
            I = arr[i]
            I.lattice = D1Q2x2 if d["dim"] == 1 else D2Q4x3
            I.nx, I.ny = d["nx"], (d.get("ny", 1) if d["dim"] == 2 else 1)
            I.lam, I.s, I.g = d["lam"], d["s"], d.get("g", 1.0)
            codes = _bc_codes(d.get("bc", ("periodic",) * 4))
            for f in range(4):
                I.bc[f] = codes[f] if f < len(codes) else 0
            for face, w in (d.get("inflow") or {}).items():
                for k in range(3):
                    I.inflow[face][k] = w[k] if k < len(w) else 0.0
        self.storage = F32 if storage in ("f32", F32) else F64
        nbytes, nodes = ctypes.c_size_t(), ctypes.c_long()
        check(L.lbm_batch_layout(arr, n, self.storage, ctypes.byref(nbytes), ctypes.byref(nodes)),
              "lbm_batch_layout")
        self.inst = arr
        self.meta = insts
        self.nodes = nodes.value
        self.dtype = torch.float32 if self.storage == F32 else torch.float64
        es = 4 if self.storage == F32 else 8
        self.device = torch.device(device)
        self.fa = torch.empty(nbytes.value // es, dtype=self.dtype, device=self.device)
        self.fb = torch.empty_like(self.fa)
        h0 = np.zeros(self.nodes)
        qx0 = np.zeros(self.nodes)
        qy0 = np.zeros(self.nodes)
        for i, d in enumerate(insts):
            o, m = arr[i].node_offset, arr[i].nx * arr[i].ny
            h0[o:o + m] = np.asarray(d["h0"]).reshape(-1)
            if d.get("qx0") is not None:
                qx0[o:o + m] = np.asarray(d["qx0"]).reshape(-1)
            if d.get("qy0") is not None and d["dim"] == 2:
                qy0[o:o + m] = np.asarray(d["qy0"]).reshape(-1)
        f64 = dict(dtype=torch.float64, device=self.device)
        self.h0, self.qx0, self.qy0 = (torch.as_tensor(a, **f64) for a in (h0, qx0, qy0))
        tune = LbmBatchTuning(block, tile_nodes, grid, pass_nodes, mode, fuse_steps, direct)
        b = ctypes.c_void_p()
        check(L.lbm_batch_create(arr, n, self.storage, _ptr(self.fa), _ptr(self.fb),
                                 _stream_handle(torch), ctypes.byref(tune), ctypes.byref(b)),
              "lbm_batch_create")
        self.b = b
        check(L.lbm_batch_init(b, _ptr(self.h0), _ptr(self.qx0), _ptr(self.qy0)), "lbm_batch_init")

    def run(self, nsteps, check_done=False):
        check(load().lbm_batch_run(self.b, int(nsteps)), "lbm_batch_run")
        if check_done:
            self.check()

    def check(self):
        """Synchronise and raise if the last run was aborted by the scheduler."""
        check(load().lbm_batch_check(self.b), "lbm_batch_check")

    def info(self):
        nt, gr = ctypes.c_int(), ctypes.c_int()
        check(load().lbm_batch_info(self.b, ctypes.byref(nt), ctypes.byref(gr)))
        return nt.value, gr.value

    def moments(self):
        """Packed (h, qx, qy) float64 device tensors over all instances' nodes."""
        torch = self.torch
        h = torch.zeros(self.nodes, dtype=torch.float64, device=self.device)
        qx, qy = torch.zeros_like(h), torch.zeros_like(h)
        check(load().lbm_batch_moments(self.b, _ptr(h), _ptr(qx), _ptr(qy)), "lbm_batch_moments")
        self.check()
        return h, qx, qy

    def instance_planes(self, i):
        """(nplanes, ny, nx) view (1D: (nplanes, nx)) of instance i's planes in the
        current state buffer."""
        ptr, steps = ctypes.c_void_p(), ctypes.c_long()
        check(load().lbm_batch_current(self.b, ctypes.byref(ptr), ctypes.byref(steps)),
              "lbm_batch_current")
        buf = self.fa if ptr.value == self.fa.data_ptr() else self.fb
        I = self.inst[i]
        m = I.nx * I.ny
        ps = (m + 63) // 64 * 64
        npl = 4 if I.lattice == D1Q2x2 else 12
        v = buf[I.state_offset:I.state_offset + npl * ps].view(npl, ps)[:, :m]
        return v if I.lattice == D1Q2x2 else v.reshape(npl, I.ny, I.nx)

    def instance_view(self, i, packed):
        I = self.inst[i]
        o, m = I.node_offset, I.nx * I.ny
        v = packed[o:o + m]
        return v if I.lattice == D1Q2x2 else v.reshape(I.ny, I.nx)

    def close(self):
        if getattr(self, "b", None) and self.b.value:
            load().lbm_batch_destroy(self.b)
            self.b = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
