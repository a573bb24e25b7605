"""Exact solution of the 1-D Riemann problem for an ideal gas.

Textbook construction (Toro, "Riemann Solvers and Numerical Methods for Fluid
Dynamics", ch. 4): the star pressure is the root of f_L(p) + f_R(p) + du = 0,
with f_K the shock (Rankine-Hugoniot) or rarefaction (isentropic) branch, and
the solution is sampled on the similarity variable (x - x0)/t.  Used as an
independent pin of the oracle's Sod-tube result.
"""
import math

from scipy.optimize import brentq


class ExactRiemann:
    def __init__(self, left, right, gamma):
        (self.rl, self.ul, self.pl), (self.rr, self.ur, self.pr) = left, right
        self.g = g = gamma
        self.cl = math.sqrt(g * self.pl / self.rl)
        self.cr = math.sqrt(g * self.pr / self.rr)
        fun = lambda p: self._f(p, self.rl, self.pl, self.cl) + \
            self._f(p, self.rr, self.pr, self.cr) + (self.ur - self.ul)
        self.p_star = brentq(fun, 1e-12, 100.0 * max(self.pl, self.pr), xtol=1e-15, rtol=1e-15)
        ps = self.p_star
        self.u_star = 0.5 * (self.ul + self.ur) + 0.5 * (
            self._f(ps, self.rr, self.pr, self.cr) - self._f(ps, self.rl, self.pl, self.cl))
        self.rho_star_l = self._rho_star(ps, self.rl, self.pl)
        self.rho_star_r = self._rho_star(ps, self.rr, self.pr)

    def _f(self, p, r, pk, c):
        g = self.g
        if p > pk:
            A = 2.0 / ((g + 1.0) * r)
            B = (g - 1.0) / (g + 1.0) * pk
            return (p - pk) * math.sqrt(A / (p + B))
        return 2.0 * c / (g - 1.0) * ((p / pk) ** ((g - 1.0) / (2.0 * g)) - 1.0)

    def _rho_star(self, p, r, pk):
        g = self.g
        if p > pk:
            k = (g - 1.0) / (g + 1.0)
            return r * (p / pk + k) / (k * p / pk + 1.0)
        return r * (p / pk) ** (1.0 / g)

    # Wave speeds for the configuration with a left rarefaction and a right
    # shock (the Sod case).
    def head_speed(self):
        return self.ul - self.cl

    def tail_speed(self):
        return self.u_star - self.cl * (self.p_star / self.pl) ** ((self.g - 1.0) / (2.0 * self.g))

    def shock_speed(self):
        g = self.g
        return self.ur + self.cr * math.sqrt((g + 1.0) / (2.0 * g) * self.p_star / self.pr +
                                             (g - 1.0) / (2.0 * g))

    def sample(self, xi):
        """(rho, u, p) at similarity coordinate xi = (x - x0)/t (Sod layout)."""
        g = self.g
        if xi < self.head_speed():
            return self.rl, self.ul, self.pl
        if xi < self.tail_speed():
            c = 2.0 / (g + 1.0) * (self.cl + 0.5 * (g - 1.0) * (self.ul - xi))
            u = 2.0 / (g + 1.0) * (self.cl + 0.5 * (g - 1.0) * self.ul + xi)
            return (self.rl * (c / self.cl) ** (2.0 / (g - 1.0)), u,
                    self.pl * (c / self.cl) ** (2.0 * g / (g - 1.0)))
        if xi < self.u_star:
            return self.rho_star_l, self.u_star, self.p_star
        if xi < self.shock_speed():
            return self.rho_star_r, self.u_star, self.p_star
        return self.rr, self.ur, self.pr
