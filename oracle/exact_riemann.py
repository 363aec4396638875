"""Exact solution of the Riemann problem for the 1D ideal-gas Euler equations.

TEST INFRASTRUCTURE ONLY (part of the oracle package).

Follows Toro 2009, "Riemann Solvers and Numerical Methods for Fluid
Dynamics", 3rd ed., chapter 4: the star pressure is the root of
f(p) = f_L(p) + f_R(p) + (u_R - u_L), where f_K is the shock branch
(Rankine-Hugoniot, p > p_K) or the rarefaction branch (isentropic,
p <= p_K); the star velocity follows from f_R - f_L; the solution at
(x, t) depends only on x/t.  The root is found by Newton iteration kept
inside a bisection bracket.  Cell averages integrate the self-similar
solution over each cell, split at every wave so that each piece is smooth,
with Gauss-Legendre quadrature on the pieces.
"""
import math

import numpy as np


class RiemannState:
    def __init__(self, rho, u, p):
        self.rho, self.u, self.p = float(rho), float(u), float(p)


def _sound(g, rho, p):
    return math.sqrt(g * p / rho)


def _f_branch(p, K, g):
    """Pressure function f_K(p) and its derivative for one side."""
    cK = _sound(g, K.rho, K.p)
    if p > K.p:  # shock
        A = 2.0 / ((g + 1.0) * K.rho)
        B = (g - 1.0) / (g + 1.0) * K.p
        q = math.sqrt(A / (p + B))
        f = (p - K.p) * q
        df = q * (1.0 - 0.5 * (p - K.p) / (B + p))
    else:  # rarefaction
        e = (g - 1.0) / (2.0 * g)
        f = 2.0 * cK / (g - 1.0) * ((p / K.p) ** e - 1.0)
        df = 1.0 / (K.rho * cK) * (p / K.p) ** (-(g + 1.0) / (2.0 * g))
    return f, df


def star_state(L, R, g, tol=1e-15, maxit=200):
    """Return (p_star, u_star) for left state L and right state R."""
    du = R.u - L.u
    cL, cR = _sound(g, L.rho, L.p), _sound(g, R.rho, R.p)
    if 2.0 * (cL + cR) / (g - 1.0) <= du:
        raise ValueError("vacuum is generated; not handled")

    def f(p):
        fl, dl = _f_branch(p, L, g)
        fr, dr = _f_branch(p, R, g)
        return fl + fr + du, dl + dr

    # bracket: f is increasing in p; f(tiny) < 0 by the no-vacuum condition
    lo = 1e-14 * min(L.p, R.p)
    hi = max(L.p, R.p)
    while f(hi)[0] < 0.0:
        hi *= 2.0
    p = 0.5 * (L.p + R.p)
    for _ in range(maxit):
        val, der = f(p)
        if val > 0.0:
            hi = min(hi, p)
        else:
            lo = max(lo, p)
        step = val / der
        pn = p - step
        if not (lo < pn < hi):
            pn = 0.5 * (lo + hi)
        if abs(pn - p) <= tol * 0.5 * (pn + p):
            p = pn
            break
        p = pn
    fl, _ = _f_branch(p, L, g)
    fr, _ = _f_branch(p, R, g)
    u = 0.5 * (L.u + R.u) + 0.5 * (fr - fl)
    return p, u


class ExactRiemann:
    """Self-similar exact solution; sample(xi) gives (rho, u, p) at x/t = xi."""

    def __init__(self, L, R, g):
        self.L, self.R, self.g = L, R, g
        self.p_star, self.u_star = star_state(L, R, g)
        ps, us = self.p_star, self.u_star
        cL, cR = _sound(g, L.rho, L.p), _sound(g, R.rho, R.p)
        self.cL, self.cR = cL, cR
        gm = (g - 1.0) / (g + 1.0)
        # left wave
        if ps > L.p:
            r = ps / L.p
            self.rho_star_L = L.rho * (r + gm) / (gm * r + 1.0)
            self.SL = L.u - cL * math.sqrt((g + 1.0) / (2.0 * g) * r +
                                           (g - 1.0) / (2.0 * g))
            self.left_shock = True
            self.left_head = self.left_tail = self.SL
        else:
            self.rho_star_L = L.rho * (ps / L.p) ** (1.0 / g)
            c_star = cL * (ps / L.p) ** ((g - 1.0) / (2.0 * g))
            self.left_shock = False
            self.left_head = L.u - cL
            self.left_tail = us - c_star
        # right wave
        if ps > R.p:
            r = ps / R.p
            self.rho_star_R = R.rho * (r + gm) / (gm * r + 1.0)
            self.SR = R.u + cR * math.sqrt((g + 1.0) / (2.0 * g) * r +
                                           (g - 1.0) / (2.0 * g))
            self.right_shock = True
            self.right_head = self.right_tail = self.SR
        else:
            self.rho_star_R = R.rho * (ps / R.p) ** (1.0 / g)
            c_star = cR * (ps / R.p) ** ((g - 1.0) / (2.0 * g))
            self.right_shock = False
            self.right_head = R.u + cR
            self.right_tail = us + c_star

    def wave_speeds(self):
        """Speeds bounding every region: sorted list of x/t breakpoints."""
        return sorted({self.left_head, self.left_tail, self.u_star,
                       self.right_tail, self.right_head})

    def sample(self, xi):
        L, R, g = self.L, self.R, self.g
        ps, us = self.p_star, self.u_star
        if xi <= us:
            if self.left_shock:
                if xi < self.SL:
                    return L.rho, L.u, L.p
                return self.rho_star_L, us, ps
            if xi < self.left_head:
                return L.rho, L.u, L.p
            if xi > self.left_tail:
                return self.rho_star_L, us, ps
            c = 2.0 / (g + 1.0) + (g - 1.0) / ((g + 1.0) * self.cL) * (L.u - xi)
            rho = L.rho * c ** (2.0 / (g - 1.0))
            u = 2.0 / (g + 1.0) * (self.cL + 0.5 * (g - 1.0) * L.u + xi)
            p = L.p * c ** (2.0 * g / (g - 1.0))
            return rho, u, p
        if self.right_shock:
            if xi > self.SR:
                return R.rho, R.u, R.p
            return self.rho_star_R, us, ps
        if xi > self.right_head:
            return R.rho, R.u, R.p
        if xi < self.right_tail:
            return self.rho_star_R, us, ps
        c = 2.0 / (g + 1.0) - (g - 1.0) / ((g + 1.0) * self.cR) * (R.u - xi)
        rho = R.rho * c ** (2.0 / (g - 1.0))
        u = 2.0 / (g + 1.0) * (-self.cR + 0.5 * (g - 1.0) * R.u + xi)
        p = R.p * c ** (2.0 * g / (g - 1.0))
        return rho, u, p

    def conserved(self, xi):
        rho, u, p = self.sample(xi)
        return np.array([rho, rho * u, p / (self.g - 1.0) + 0.5 * rho * u * u])

    def cell_averages(self, edges, t, x0, order=12):
        """Average of (rho, rho u, E) over cells [edges[i], edges[i+1]] at time
        t, for a problem whose initial discontinuity sits at x0."""
        gx, gw = np.polynomial.legendre.leggauss(order)
        breaks = [x0 + s * t for s in self.wave_speeds()]
        out = np.zeros((len(edges) - 1, 3))
        for i in range(len(edges) - 1):
            a, b = float(edges[i]), float(edges[i + 1])
            cuts = [a] + [x for x in breaks if a < x < b] + [b]
            acc = np.zeros(3)
            for lo, hi in zip(cuts[:-1], cuts[1:]):
                mid, half = 0.5 * (lo + hi), 0.5 * (hi - lo)
                for xg, wg in zip(gx, gw):
                    x = mid + half * xg
                    acc += wg * half * self.conserved((x - x0) / t)
            out[i] = acc / (b - a)
        return out
