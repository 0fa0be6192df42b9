"""Seeded synthetic workloads (initial conserved fields and run parameters).

This module holds no arithmetic of the lattice Boltzmann method: it only builds
initial states (h, qx, qy), physical/lattice parameters and the batched
manifest.  Both the GPU path and the CPU oracle consume its outputs; neither
side's arithmetic lives here.

Grid convention: cell-centred nodes x_i = (i + 1/2) dx on the unit interval /
unit square, dx = 1/N; lattice velocity lambda = dx/dt, so t_n = n dx / lambda.

Workloads (the paper's own runs use analytic initial states; these stand in for
them with the shapes of the paper's experiments, Sec. 2 Fig. 1 and Sec. 4):

* ``dam_break_1d``      1D Riemann problem, h = 2 | 1, u = 0 (Stoker)
* ``wall_reflection_1d`` 1D inflow (h = 1.5, u = 0.5) into still water (h = 1)
                         toward a solid wall on the right
* ``radial_dam_break_2d`` 2D periodic square, h = 2 inside a disk of radius 0.2,
                         h = 1 outside, at rest
* ``batched_manifest``  256 mixed 1D / 2D Riemann problems of uneven sizes
* ``adjoint_case``      2D Gaussian hump and a seeded perturbation of it
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

G = 1.0  # gravity in every workload


def cell_centres(n: int) -> np.ndarray:
    return (np.arange(n, dtype=np.float64) + 0.5) / n


@dataclass
class Case:
    """One run: dimension, grid, lattice parameters, boundary codes and W0."""

    dim: int
    nx: int
    ny: int
    lam: float
    s: float
    steps: int
    g: float = G
    bc: tuple = ("periodic", "periodic", "periodic", "periodic")  # x-, x+, y-, y+
    inflow: dict = field(default_factory=dict)  # face -> (h, qx, qy)
    h0: np.ndarray | None = None
    qx0: np.ndarray | None = None
    qy0: np.ndarray | None = None
    name: str = ""

    @property
    def nodes(self) -> int:
        return self.nx * self.ny


def dam_break_1d(n=1000, lam=3.0, s=1.8, steps=400) -> Case:
    """h = 2 for x < 1/2, h = 1 for x > 1/2, u = 0, Neumann ends."""
    x = cell_centres(n)
    h0 = np.where(x < 0.5, 2.0, 1.0)
    return Case(1, n, 1, lam, s, steps, bc=("neumann", "neumann", "periodic", "periodic"),
                h0=h0, qx0=np.zeros(n), name=f"dam_break_1d_n{n}")


def wall_reflection_1d(n=1 << 20, lam=3.0, s=1.9, steps=20000, h_in=1.5, u_in=0.5) -> Case:
    """Still water h = 1 with an inflow ghost state (1.5, 0.75) on the left and a
    solid wall on the right."""
    h0 = np.ones(n)
    return Case(1, n, 1, lam, s, steps, bc=("inflow", "wall", "periodic", "periodic"),
                inflow={0: (h_in, h_in * u_in, 0.0)}, h0=h0, qx0=np.zeros(n),
                name=f"wall_reflection_1d_n{n}_s{s}")


def radial_dam_break_2d(n=4096, lam=6.0, s=1.8, steps=2000, radius=0.2) -> Case:
    """h = 2 inside the centred disk r < radius (unit square), else 1; at rest;
    periodic in both directions.  No node lies on the circle for even n."""
    x = cell_centres(n)
    X, Y = np.meshgrid(x, x, indexing="xy")
    r2 = (X - 0.5) ** 2 + (Y - 0.5) ** 2
    h0 = np.where(r2 < radius * radius, 2.0, 1.0)
    z = np.zeros((n, n))
    return Case(2, n, n, lam, s, steps, h0=h0, qx0=z, qy0=z.copy(),
                name=f"radial_dam_break_2d_n{n}_lam{lam:g}")


# --- batched manifest -------------------------------------------------------------

@dataclass
class Instance:
    dim: int
    nx: int
    ny: int
    lam: float
    s: float
    hl: float
    ul: float
    vl: float
    hr: float
    ur: float
    vr: float
    lam_stated: float

    def initial(self):
        """W0 = (h, qx, qy) of the planar Riemann problem: left state on the
        first half of the x-nodes, right state on the second half (2D: the same
        for every row; periodic, so there are two interfaces)."""
        n = self.nx
        left = np.arange(n) < n // 2
        h = np.where(left, self.hl, self.hr)
        u = np.where(left, self.ul, self.ur)
        v = np.where(left, self.vl, self.vr)
        if self.dim == 1:
            return h, h * u, None
        H = np.broadcast_to(h, (self.ny, n)).copy()
        return H, H * np.broadcast_to(u, (self.ny, n)), H * np.broadcast_to(v, (self.ny, n))


def batched_manifest(seed=0, n1d=128, n2d=128, n1_range=(1024, 65536), side_range=(128, 1024),
                     lam_factor_1d=1.2, lam_factor_2d=2.4, stated_factor=1.2):
    """256 instances drawn with numpy default_rng(seed) in a fixed order:
    for each 1D instance N, hl, hr, ul, ur, s; for each 2D instance side, hl, hr,
    ul, ur, vl, vr, s.  h ~ U[0.5, 3], u, v ~ U[-1, 1], s ~ U[1.2, 1.95].
    lambda = factor * (max|u| + sqrt(g max h)); the stated factor is 1.2 for
    both; D2Q4 needs about twice the 1D margin, so 2D instances run at 2.4 by
    default (the stated value is kept in ``lam_stated``)."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n1d):
        n = int(rng.integers(n1_range[0], n1_range[1] + 1))
        hl, hr = rng.uniform(0.5, 3.0, 2)
        ul, ur = rng.uniform(-1.0, 1.0, 2)
        s = float(rng.uniform(1.2, 1.95))
        vmax = max(abs(ul), abs(ur)) + math.sqrt(G * max(hl, hr))
        out.append(Instance(1, n, 1, lam_factor_1d * vmax, s, hl, ul, 0.0, hr, ur, 0.0,
                            stated_factor * vmax))
    for _ in range(n2d):
        side = int(rng.integers(side_range[0], side_range[1] + 1))
        hl, hr = rng.uniform(0.5, 3.0, 2)
        ul, ur, vl, vr = rng.uniform(-1.0, 1.0, 4)
        s = float(rng.uniform(1.2, 1.95))
        vmax = max(abs(ul), abs(ur), abs(vl), abs(vr)) + math.sqrt(G * max(hl, hr))
        out.append(Instance(2, side, side, lam_factor_2d * vmax, s, hl, ul, vl, hr, ur, vr,
                            stated_factor * vmax))
    return out


def small_manifest(seed=1, n1d=6, n2d=6):
    """A few small instances of every kind (parity tests with the oracle)."""
    return batched_manifest(seed, n1d, n2d, n1_range=(37, 700), side_range=(9, 70))


# --- adjoint workload --------------------------------------------------------------

def adjoint_case(n=1024, lam=3.0, s=1.8, steps=500, sigma=0.1, seed=0, amp=0.3, width2=0.01):
    """Initial height 1 + amp exp(-r^2/width2) about the centre of the periodic unit
    square, and the initial height of the target run: the same plus seeded
    Gaussian noise N(0, sigma^2) drawn with default_rng(seed) in C order."""
    x = cell_centres(n)
    X, Y = np.meshgrid(x, x, indexing="xy")
    r2 = (X - 0.5) ** 2 + (Y - 0.5) ** 2
    h0 = 1.0 + amp * np.exp(-r2 / width2)
    noise = np.random.default_rng(seed).standard_normal((n, n)) * sigma
    return Case(2, n, n, lam, s, steps, h0=h0, qx0=np.zeros((n, n)), qy0=np.zeros((n, n)),
                name=f"adjoint_2d_n{n}"), h0 + noise


# --- stationary oblique shock reflection (Sec. 4, first test case) -------------------

OBLIQUE_STATES = {  # (h, u, v) printed in Sec. 4 (g = 1)
    "left": (1.0, 1.59497132403753, 0.0),
    "top": (1.17150636388320, 1.47822089880855, -0.116750425228984),
    "right": (1.38196199044604, 1.33228286727232, 0.0),
}


def oblique_shock_2d(ny=20, lam=8.0, s=1.8, steps=None, aspect=1.75) -> Case:
    """Domain [0, aspect] x [0, 1] with ny rows (the Sec. 4 meshes are 35 x 20,
    70 x 40, 140 x 80).  The left state enters through the left face and the top
    state through the top face (equilibrium inflow ghosts), the bottom face is a
    wall, the right face a zero-gradient outflow.  Starts from the left state
    everywhere; `steps` defaults to about ten crossings of the domain."""
    nx = int(round(aspect * ny))
    hl, ul, vl = OBLIQUE_STATES["left"]
    ht, ut, vt = OBLIQUE_STATES["top"]
    if steps is None:
        steps = 120 * ny
    h0 = np.full((ny, nx), hl)
    return Case(2, nx, ny, lam, s, steps, bc=("inflow", "neumann", "wall", "inflow"),
                inflow={0: (hl, hl * ul, hl * vl), 3: (ht, ht * ut, ht * vt)},
                h0=h0, qx0=np.full((ny, nx), hl * ul), qy0=np.zeros((ny, nx)),
                name=f"oblique_shock_{nx}x{ny}")
