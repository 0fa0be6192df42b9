"""Exact solutions of the shallow-water equations used to pin the oracle.

TEST INFRASTRUCTURE ONLY.

The paper compares its D1Q3Q2 results with the exact Riemann solution (Sec. 2,
Fig. 1) and its oblique shock reflection with the Rankine-Hugoniot solution
(Sec. 4, Fig. 2).  Shallow water here is rho = h, p = (g/2) h^2, c^2 = g h
(Sec. 2 with gamma = 2 and p0/rho0^2 = g/2).  Everything below is written from
the textbook theory of the shallow-water Riemann problem: a 1-wave and a
2-wave, each a shock (Rankine-Hugoniot) or a rarefaction (Riemann invariant
u +- 2c constant across it).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
from scipy.optimize import brentq


def _wave_fn(h, hk, g):
    """Velocity change across a 1- or 2-wave connecting depth hk to depth h."""
    if h > hk:  # shock: Rankine-Hugoniot
        return (h - hk) * math.sqrt(0.5 * g * (h + hk) / (h * hk))
    return 2.0 * (math.sqrt(g * h) - math.sqrt(g * hk))  # rarefaction: Riemann invariant


@dataclass
class RiemannSolution:
    hl: float
    ul: float
    hr: float
    ur: float
    g: float
    hs: float  # star (middle) state depth
    us: float  # star state velocity
    left_shock: bool
    right_shock: bool
    sl: float  # left shock speed (if shock)
    sr: float  # right shock speed (if shock)

    def wave_speeds(self):
        """Dict of characteristic / shock speeds bounding each wave."""
        g = self.g
        cl, cr, cs = (math.sqrt(g * self.hl), math.sqrt(g * self.hr), math.sqrt(g * self.hs))
        out = {}
        if self.left_shock:
            out["left_shock"] = self.sl
        else:
            out["left_head"] = self.ul - cl
            out["left_tail"] = self.us - cs
        if self.right_shock:
            out["right_shock"] = self.sr
        else:
            out["right_tail"] = self.us + cs
            out["right_head"] = self.ur + cr
        return out

    def sample(self, xi):
        """(h, u) at similarity variable xi = (x - x0)/t (array or scalar)."""
        xi = np.asarray(xi, dtype=np.float64)
        g = self.g
        cl, cr, cs = (math.sqrt(g * self.hl), math.sqrt(g * self.hr), math.sqrt(g * self.hs))
        h = np.empty_like(xi)
        u = np.empty_like(xi)
        left = xi < self.us
        # left of the contact-like middle line
        if self.left_shock:
            m = left & (xi < self.sl)
            h[m], u[m] = self.hl, self.ul
            m = left & (xi >= self.sl)
            h[m], u[m] = self.hs, self.us
        else:
            head, tail = self.ul - cl, self.us - cs
            m = left & (xi < head)
            h[m], u[m] = self.hl, self.ul
            m = left & (xi >= head) & (xi <= tail)
            c = (self.ul + 2.0 * cl - xi[m]) / 3.0
            u[m] = (self.ul + 2.0 * cl + 2.0 * xi[m]) / 3.0
            h[m] = c * c / g
            m = left & (xi > tail)
            h[m], u[m] = self.hs, self.us
        right = ~left
        if self.right_shock:
            m = right & (xi > self.sr)
            h[m], u[m] = self.hr, self.ur
            m = right & (xi <= self.sr)
            h[m], u[m] = self.hs, self.us
        else:
            tail, head = self.us + cs, self.ur + cr
            m = right & (xi > head)
            h[m], u[m] = self.hr, self.ur
            m = right & (xi >= tail) & (xi <= head)
            c = (-self.ur + 2.0 * cr + xi[m]) / 3.0
            u[m] = (self.ur - 2.0 * cr + 2.0 * xi[m]) / 3.0
            h[m] = c * c / g
            m = right & (xi < tail)
            h[m], u[m] = self.hs, self.us
        return h, u


def riemann(hl, ul, hr, ur, g=1.0) -> RiemannSolution:
    """Exact solution of the shallow-water Riemann problem (no dry bed)."""
    def phi(h):
        return _wave_fn(h, hl, g) + _wave_fn(h, hr, g) + ur - ul

    lo, hi = 1e-12, max(hl, hr)
    while phi(hi) < 0:
        hi *= 2.0
    hs = brentq(phi, lo, hi, xtol=1e-15, rtol=1e-15, maxiter=500)
    us = 0.5 * (ul + ur) + 0.5 * (_wave_fn(hs, hr, g) - _wave_fn(hs, hl, g))
    left_shock, right_shock = hs > hl, hs > hr
    # shock speeds from mass conservation across the jump
    sl = (hs * us - hl * ul) / (hs - hl) if left_shock else float("nan")
    sr = (hs * us - hr * ur) / (hs - hr) if right_shock else float("nan")
    return RiemannSolution(hl, ul, hr, ur, g, hs, us, left_shock, right_shock, sl, sr)


def wall_reflection(h, u, g=1.0):
    """State (h, u), u > 0, hitting a solid wall on its right: returns
    (h_wall, reflected shock speed).  Wall state has u = 0; by symmetry it is the
    middle state of the Riemann problem between (h, u) and its mirror (h, -u)."""
    sol = riemann(h, u, h, -u, g)
    hw = sol.hs
    s = (0.0 - h * u) / (hw - h)
    return hw, s


def rh_residual_2d(A, B, g=1.0):
    """Stationary oblique shock between states A and B = (h, u, v).  The shock
    normal n is along the velocity jump (tangential velocity is continuous when
    the mass flux is).  Returns (n, residual vector of [h u_n] and
    [h u_n u + p n]) -- zero for an exact Rankine-Hugoniot pair."""
    hA, uA, vA = A
    hB, uB, vB = B
    d = np.array([uA - uB, vA - vB])
    n = d / np.linalg.norm(d)
    unA = uA * n[0] + vA * n[1]
    unB = uB * n[0] + vB * n[1]
    pA, pB = 0.5 * g * hA * hA, 0.5 * g * hB * hB
    r_mass = hA * unA - hB * unB
    r_mom = (hA * unA * np.array([uA, vA]) + pA * n) - (hB * unB * np.array([uB, vB]) + pB * n)
    return n, np.array([r_mass, r_mom[0], r_mom[1]])


def oblique_shock_reflection(x, y, left, top, right, g=1.0):
    """Exact stationary solution of the Sec. 4 reflection on [0, L] x [0, 1]
    with the wall at y = 0: the incident shock runs from (0, 1) at angle -pi/4
    (line y = 1 - x), the reflected shock leaves the wall at (1, 0) along the
    normal computed from the top and right states (rh_residual_2d).  Returns the
    depth h at the points (x, y)."""
    n2, _ = rh_residual_2d(top, right, g)
    slope = -n2[0] / n2[1]
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    h = np.where(y > 1.0 - x, top[0], left[0])
    return np.where((x > 1.0) & (y < slope * (x - 1.0)), right[0], h)
