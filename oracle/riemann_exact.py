"""Exact solution of the 1D Riemann problem for an ideal gamma-law gas.

TEST INFRASTRUCTURE ONLY (used to check the planar shock tube).

The release paper's method is a mesh-free finite-volume Godunov scheme (its
abstract names the family); the reference solution for its shock tube is
the classical exact Riemann solution: a pressure function per side (shock
branch from the Rankine-Hugoniot conditions, rarefaction branch from the
isentropic Riemann invariants), whose root is the star pressure, then
self-similar sampling in x/t.  Written from those conditions directly.
"""
from __future__ import annotations

import math

import numpy as np


def _side(p, rho, P, gamma):
    """Velocity jump f_K(p) across the wave of side K and its derivative."""
    c = math.sqrt(gamma * P / rho)
    if p > P:  # shock: Rankine-Hugoniot
        A = 2.0 / ((gamma + 1.0) * rho)
        Bc = (gamma - 1.0) / (gamma + 1.0) * P
        q = math.sqrt(A / (p + Bc))
        return (p - P) * q, q * (1.0 - 0.5 * (p - P) / (p + Bc))
    # rarefaction: isentropic
    e = (gamma - 1.0) / (2.0 * gamma)
    f = 2.0 * c / (gamma - 1.0) * ((p / P) ** e - 1.0)
    df = 1.0 / (rho * c) * (p / P) ** (-(gamma + 1.0) / (2.0 * gamma))
    return f, df


def star_state(left, right, gamma, tol=1e-15, maxit=200):
    """Star-region pressure and velocity for states (rho, u, P)."""
    rl, ul, pl = left
    rr, ur, pr = right
    cl = math.sqrt(gamma * pl / rl)
    cr = math.sqrt(gamma * pr / rr)
    if 2.0 * (cl + cr) / (gamma - 1.0) <= ur - ul:
        raise ValueError("vacuum is generated")
    # two-rarefaction guess, then Newton on f_L(p) + f_R(p) + (u_R - u_L) = 0
    e = (gamma - 1.0) / (2.0 * gamma)
    p = ((cl + cr - 0.5 * (gamma - 1.0) * (ur - ul)) / (cl / pl ** e + cr / pr ** e)) ** (1.0 / e)
    for _ in range(maxit):
        fl, dfl = _side(p, rl, pl, gamma)
        fr, dfr = _side(p, rr, pr, gamma)
        pn = p - (fl + fr + ur - ul) / (dfl + dfr)
        if pn <= 0.0:
            pn = 0.5 * p
        done = abs(pn - p) <= tol * 0.5 * (pn + p)
        p = pn
        if done:
            break
    fl, _ = _side(p, rl, pl, gamma)
    fr, _ = _side(p, rr, pr, gamma)
    u = 0.5 * (ul + ur) + 0.5 * (fr - fl)
    return p, u


def star_densities(left, right, gamma):
    rl, ul, pl = left
    rr, ur, pr = right
    p, u = star_state(left, right, gamma)
    g = (gamma - 1.0) / (gamma + 1.0)

    def rho_star(rk, pk):
        if p > pk:
            return rk * (p / pk + g) / (g * p / pk + 1.0)
        return rk * (p / pk) ** (1.0 / gamma)

    return rho_star(rl, pl), rho_star(rr, pr)


def wave_speeds(left, right, gamma):
    """dict of the wave speeds (shock or rarefaction head/tail per side, contact)."""
    rl, ul, pl = left
    rr, ur, pr = right
    p, u = star_state(left, right, gamma)
    rsl, rsr = star_densities(left, right, gamma)
    cl = math.sqrt(gamma * pl / rl)
    cr = math.sqrt(gamma * pr / rr)
    out = {"contact": u}
    if p > pl:
        out["left_shock"] = ul - cl * math.sqrt((gamma + 1) / (2 * gamma) * p / pl + (gamma - 1) / (2 * gamma))
    else:
        out["left_head"] = ul - cl
        out["left_tail"] = u - math.sqrt(gamma * p / rsl)
    if p > pr:
        out["right_shock"] = ur + cr * math.sqrt((gamma + 1) / (2 * gamma) * p / pr + (gamma - 1) / (2 * gamma))
    else:
        out["right_head"] = ur + cr
        out["right_tail"] = u + math.sqrt(gamma * p / rsr)
    return out


def sample(left, right, gamma, xi):
    """(rho, u, P) at similarity coordinates xi = (x - x0)/t (array)."""
    rl, ul, pl = left
    rr, ur, pr = right
    p, u = star_state(left, right, gamma)
    rsl, rsr = star_densities(left, right, gamma)
    ws = wave_speeds(left, right, gamma)
    cl = math.sqrt(gamma * pl / rl)
    cr = math.sqrt(gamma * pr / rr)
    xi = np.asarray(xi, dtype=np.float64)
    rho = np.empty_like(xi)
    vel = np.empty_like(xi)
    pres = np.empty_like(xi)
    g1 = gamma - 1.0
    g2 = gamma + 1.0
    for k, s in enumerate(xi.ravel()):
        if s <= u:  # left of contact
            if p > pl:
                if s <= ws["left_shock"]:
                    r, v, q = rl, ul, pl
                else:
                    r, v, q = rsl, u, p
            else:
                if s <= ws["left_head"]:
                    r, v, q = rl, ul, pl
                elif s >= ws["left_tail"]:
                    r, v, q = rsl, u, p
                else:  # inside the left fan
                    v = 2.0 / g2 * (cl + 0.5 * g1 * ul + s)
                    c = 2.0 / g2 * (cl + 0.5 * g1 * (ul - s))
                    r = rl * (c / cl) ** (2.0 / g1)
                    q = pl * (c / cl) ** (2.0 * gamma / g1)
        else:
            if p > pr:
                if s >= ws["right_shock"]:
                    r, v, q = rr, ur, pr
                else:
                    r, v, q = rsr, u, p
            else:
                if s >= ws["right_head"]:
                    r, v, q = rr, ur, pr
                elif s <= ws["right_tail"]:
                    r, v, q = rsr, u, p
                else:
                    v = 2.0 / g2 * (-cr + 0.5 * g1 * ur + s)
                    c = 2.0 / g2 * (cr - 0.5 * g1 * (ur - s))
                    r = rr * (c / cr) ** (2.0 / g1)
                    q = pr * (c / cr) ** (2.0 * gamma / g1)
        rho.flat[k] = r
        vel.flat[k] = v
        pres.flat[k] = q
    return rho, vel, pres
