"""Shared helpers of the GPU parity tests (host logic only)."""
import sys

import numpy as np

import oracle
from paper_1401_0427_amd import workloads as W


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def to_np(t):
    return t.detach().cpu().numpy()


def orc_params(case, **kw):
    return oracle.params(case.dim, case.nx, case.ny, lam=case.lam, s=case.s, g=case.g,
                         bc=case.bc, inflow=case.inflow, **kw)


def orc_state(case, steps):
    """Oracle post-collision state after `steps`, hot-path planes only."""
    P = orc_params(case)
    f = oracle.run(P, case.h0, case.qx0, case.qy0 if case.dim == 2 else None, steps)
    assert np.all(f[0] == 0.0)
    return oracle.to_hotpath_planes(f), P


def gpu_solver(case, storage="f64", **kw):
    from paper_1401_0427_amd.lbm import Solver

    return Solver(case.dim, case.nx, case.ny, lam=case.lam, s=case.s, g=case.g, bc=case.bc,
                  inflow=case.inflow, h0=case.h0, qx0=case.qx0,
                  qy0=case.qy0 if case.dim == 2 else None, storage=storage, **kw)


def normwise_rel(a, b):
    """max |a - b| / max |b| (0 when both vanish)."""
    d = np.abs(np.asarray(a, dtype=np.float64) - np.asarray(b, dtype=np.float64)).max()
    s = np.abs(np.asarray(b, dtype=np.float64)).max()
    return 0.0 if d == 0 else d / (s if s > 0 else 1.0)


def per_plane_rel(A, B):
    return max(normwise_rel(a, b) for a, b in zip(A, B))


def l1_rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return np.abs(a - b).sum() / np.abs(b).sum()


def smooth_random_2d(nx, ny, seed=0, lam=6.0, s=1.8, bc=("periodic",) * 4, inflow=None):
    rng = np.random.default_rng(seed)
    x = W.cell_centres(nx)
    y = W.cell_centres(ny)
    X, Y = np.meshgrid(x, y)
    h = 1.0 + 0.3 * np.exp(-((X - 0.4) ** 2 + (Y - 0.55) ** 2) / 0.03) + 0.02 * rng.random((ny, nx))
    qx = 0.2 * np.sin(2 * np.pi * Y) + 0.02 * rng.standard_normal((ny, nx))
    qy = 0.15 * np.cos(2 * np.pi * X) + 0.02 * rng.standard_normal((ny, nx))
    return W.Case(2, nx, ny, lam, s, 0, bc=bc, inflow=inflow or {}, h0=h, qx0=qx, qy0=qy,
                  name=f"smooth2d_{nx}x{ny}")


def cone_window_1d(case, x, steps):
    """Sub-problem whose centre node reproduces node x after `steps` steps:
    nodes within `steps` of x, real boundary rules at real domain ends, a
    zero-gradient rule at cut ends (their errors travel one node per step and
    cannot reach x)."""
    a, b = max(0, x - steps), min(case.nx - 1, x + steps)
    bc = (case.bc[0] if a == 0 else "neumann", case.bc[1] if b == case.nx - 1 else "neumann",
          "periodic", "periodic")
    inflow = {f: w for f, w in case.inflow.items() if (f == 0 and a == 0) or (f == 1 and b == case.nx - 1)}
    sub = W.Case(1, b - a + 1, 1, case.lam, case.s, steps, g=case.g, bc=bc, inflow=inflow,
                 h0=case.h0[a:b + 1], qx0=case.qx0[a:b + 1], name="cone1d")
    return sub, x - a


def cone_window_2d_periodic(case, x, y, steps):
    """Periodic 2D analogue: the (2 steps + 1)^2 window centred on (x, y),
    wrapped around the torus."""
    r = steps
    xs = np.arange(x - r, x + r + 1) % case.nx
    ys = np.arange(y - r, y + r + 1) % case.ny
    sel = np.ix_(ys, xs)
    m = 2 * r + 1
    sub = W.Case(2, m, m, case.lam, case.s, steps, g=case.g, bc=("neumann",) * 4,
                 h0=case.h0[sel], qx0=case.qx0[sel], qy0=case.qy0[sel], name="cone2d")
    return sub, r, r
