"""Gradients of a final-height misfit through the lattice Boltzmann rollout.

``rollout(h0, s, T, ...)`` returns h(T) as a differentiable function of the
initial height field h0 and the relaxation rate s.  The forward keeps a copy of
the state every K steps (by default K is about sqrt(T)) and the backward, for
each K-step segment in reverse, recomputes its states from the checkpoint (one
extra forward step per adjoint step) and applies the hand-written adjoint kernel
step by step -- one library call per segment (``lbm_adjoint_segment``).  With K =
1 the forward keeps every level instead (single steps written level by level,
``lbm_step_levels``) and the backward applies the adjoint over them in one
library call (``lbm_adjoint_levels``), with no recomputation: the faster form
whenever the T + 1 states fit in device memory (``every_level_fits``; 1024^2 FP32
x 500 steps: 24 GB of an MI355X's 288).  Either way dL/ds
accumulates in FP64 per workgroup, and finally dL/dh0 = J(W0)^T lam^0.  Every
level is bitwise the same in both forms (multi-step launches equal single steps),
so are the gradients.

The 2D (D2Q4 x 3) and 1D (D1Q2 x 2) lattices have an adjoint, with any face rules
(periodic, Neumann, wall, inflow).  Initial momentum is zero (the adjoint
workload); the state storage may be FP64 or FP32.  The adjoint is stored like
the state unless asked otherwise (``adjoint_storage="f64"`` keeps it in FP64 for
an FP32 state); arithmetic and the s-gradient are FP64.
"""
from __future__ import annotations

import math

import torch

from .lbm import Solver


class _Rollout(torch.autograd.Function):
    @staticmethod
    def forward(ctx, h0, s, T, K, lam, g, storage, block, adjoint_storage, bc, inflow):
        n = h0.shape
        dim = h0.dim()
        solver = Solver(dim, n[-1], n[0] if dim == 2 else 1, lam=lam, s=float(s), g=g,
                        bc=bc, inflow=inflow, h0=h0.detach(), storage=storage, block=block,
                        adjoint_storage=adjoint_storage)
        ctx.levels, cks = None, None
        if K == 1:
            # every level: slot t holds level t, t = 0 .. T
            nb = solver.nplanes * solver.ps
            levels = torch.empty((T + 1) * nb, dtype=solver.dtype, device=solver.device)
            levels[:nb].copy_(solver.current()[0])
            solver.step_levels(levels[:nb], T, levels[nb:])
            hT = solver.moments(levels[T * nb:])[0]
            ctx.levels = levels
        else:
            cks = {0: solver.current()[0].clone()}
            t = 0
            while t < T:
                k = min(K, T - t)
                solver.step(k)
                t += k
                if t < T:
                    cks[t] = solver.current()[0].clone()
            hT = solver.moments()[0]
        ctx.solver = solver
        ctx.cks = cks
        ctx.T, ctx.K = T, K
        ctx.save_for_backward(h0)
        return hT

    @staticmethod
    def backward(ctx, grad_hT):
        solver, cks, T, K = ctx.solver, ctx.cks, ctx.T, ctx.K
        lam = [solver.new_adjoint(), solver.new_adjoint()]
        solver.adjoint_terminal(grad_hT.contiguous(), lam[0])
        partials = solver.adjoint_partials()
        if ctx.levels is not None:
            cur = solver.adjoint_levels(ctx.levels, T, lam[0], lam[1], partials)
        else:
            work = solver.new_state(max(1, K - 1))
            cur = 0
            for s0 in reversed(sorted(cks)):
                n = min(s0 + K, T) - s0
                out = solver.adjoint_segment(cks[s0], n, work, lam[cur], lam[1 - cur], partials)
                cur = cur if out == 0 else 1 - cur
        gh0 = solver.adjoint_grad_w0(lam[cur])[0]
        gs = solver.sum(partials)
        ctx.solver = None
        ctx.cks = None
        ctx.levels = None
        grad_s = torch.tensor(gs, dtype=torch.float64, device=gh0.device)
        return gh0, grad_s, None, None, None, None, None, None, None, None, None


def rollout(h0: torch.Tensor, s: torch.Tensor, T: int, K: int | None = None, lam: float = 3.0,
            g: float = 1.0, storage: str = "f64", block: int = 256,
            adjoint_storage: str | None = None, bc=("periodic",) * 4,
            inflow=None) -> torch.Tensor:
    """h(T) from W0 = (h0, 0, 0) (1D: (h0, 0)); differentiable in h0 (a 2D
    (ny, nx) or 1D (nx,) float64 CUDA tensor) and s (0-dim float64 tensor).  K =
    steps between checkpoints (default about sqrt(T)); K = 1 keeps every level (no
    recomputation in the backward).  ``bc`` = faces (x-, x+, y-, y+) by name,
    ``inflow`` = {face: (h, qx, qy)} as for Solver.  ``adjoint_storage``: element
    type of the adjoint buffers (None = the state's, "f64", or "f32" with FP32
    state storage)."""
    if K is None:
        K = max(1, int(round(math.sqrt(T))))
    return _Rollout.apply(h0, s, int(T), int(K), float(lam), float(g), storage, int(block),
                          adjoint_storage, tuple(bc), inflow)


def every_level_fits(shape, T: int, storage: str = "f64", device=None) -> bool:
    """Whether the T + 1 states of a rollout over a field of ``shape`` ((ny, nx) or
    (nx,)) fit in half the free device memory, so that K = 1 (every level kept, no
    recomputation) can be used."""
    nx = shape[-1]
    ny = shape[0] if len(shape) == 2 else 1
    planes = 12 if len(shape) == 2 else 4
    state_bytes = planes * nx * ny * (4 if storage == "f32" else 8)
    free = torch.cuda.mem_get_info(device)[0]
    return (T + 1) * state_bytes <= free // 2
