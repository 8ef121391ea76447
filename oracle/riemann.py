"""Exact solution of the one-dimensional Riemann problem for two stiffened gases.

TEST INFRASTRUCTURE ONLY.  It pins the oracle solver (Sec. 2.2 of
arXiv:1705.04374: Godunov-type scheme with HLLC fluxes) to something other than
itself: shock tubes of an ideal gas, of a single stiffened gas and of water
against air.

Textbook construction (Toro, "Riemann Solvers and Numerical Methods for Fluid
Dynamics", ch. 4), written for a stiffened gas p = (gamma - 1) rho e - gamma p_c
by the substitution pbar = p + p_c, under which each material behaves as an
ideal gas in pbar.  The two materials meet at the contact, so the left and
right waves use their own (gamma, p_c).
"""
from __future__ import annotations

import math

import numpy as np
from scipy.optimize import brentq


class Side:
    def __init__(self, rho, u, p, gamma, pc):
        self.rho, self.u, self.p, self.g, self.pc = float(rho), float(u), float(p), float(gamma), float(pc)
        self.pb = self.p + self.pc
        self.c = math.sqrt(self.g * self.pb / self.rho)

    def f(self, p):
        """Velocity jump across the wave connecting this side to pressure p."""
        g, pb = self.g, p + self.pc
        if p > self.p:
            A = 2.0 / ((g + 1.0) * self.rho)
            B = (g - 1.0) / (g + 1.0) * self.pb
            return (p - self.p) * math.sqrt(A / (pb + B))
        return 2.0 * self.c / (g - 1.0) * ((pb / self.pb) ** ((g - 1.0) / (2.0 * g)) - 1.0)


class ExactRiemann:
    def __init__(self, left: Side, right: Side):
        self.L, self.R = left, right
        du = right.u - left.u
        lo = max(-left.pc, -right.pc) + 1e-12 * max(left.pb, right.pb, 1.0)
        hi = 10.0 * max(left.p + left.pc, right.p + right.pc) + 1.0
        fun = lambda p: left.f(p) + right.f(p) + du
        while fun(hi) < 0:
            hi *= 10.0
        if fun(lo) > 0:
            raise ValueError("vacuum generated")
        self.ps = brentq(fun, lo, hi, xtol=1e-14 * hi, rtol=1e-15, maxiter=500)
        self.us = 0.5 * (left.u + right.u) + 0.5 * (right.f(self.ps) - left.f(self.ps))

    def _side(self, S: Side, xi: float, sign: float):
        """Sample on side S (sign -1 for left, +1 for right) at xi = x/t."""
        g, ps, us = S.g, self.ps, self.us
        psb = ps + S.pc
        ratio = psb / S.pb
        # mirror the right side onto the left-side formulas
        u_in, xi_m, us_m = sign * -1.0 * S.u, -sign * xi, -sign * us
        if ps > S.p:
            ss = u_in - S.c * math.sqrt((g + 1.0) / (2.0 * g) * ratio + (g - 1.0) / (2.0 * g))
            if xi_m < ss:
                return S.rho, S.u, S.p
            gm = (g - 1.0) / (g + 1.0)
            return S.rho * (ratio + gm) / (gm * ratio + 1.0), us, ps
        cs = S.c * ratio ** ((g - 1.0) / (2.0 * g))
        head, tail = u_in - S.c, us_m - cs
        if xi_m < head:
            return S.rho, S.u, S.p
        if xi_m > tail:
            return S.rho * ratio ** (1.0 / g), us, ps
        u = 2.0 / (g + 1.0) * (S.c + 0.5 * (g - 1.0) * u_in + xi_m)
        c = 2.0 / (g + 1.0) * (S.c + 0.5 * (g - 1.0) * (u_in - xi_m))
        rho = S.rho * (c / S.c) ** (2.0 / (g - 1.0))
        pb = S.pb * (c / S.c) ** (2.0 * g / (g - 1.0))
        return rho, -sign * u, pb - S.pc

    def sample(self, xi: float):
        """(rho, u, p, side) at xi = (x - x0)/t; side 0 = left material."""
        if xi < self.us:
            r, u, p = self._side(self.L, xi, -1.0)
            return r, u, p, 0
        r, u, p = self._side(self.R, xi, +1.0)
        return r, u, p, 1

    def profile(self, x: np.ndarray, x0: float, t: float):
        out = np.array([self.sample((xx - x0) / t) for xx in x])
        return out[:, 0], out[:, 1], out[:, 2], out[:, 3]
