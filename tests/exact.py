"""Closed-form and exact solutions used to pin the CPU reference solver.

Nothing here calls the reference solver or the GPU path. The exact Riemann
solver follows the standard construction (Toro's textbook, Ch. 4): the star
pressure is the root of f_L(p) + f_R(p) + (u_R - u_L) = 0, where each f_K is
the shock (Rankine-Hugoniot) or rarefaction (isentropic) relation for that
side; the self-similar solution is then sampled at x/t.
"""
from __future__ import annotations

import numpy as np
from scipy.optimize import brentq


def _fk(p, rho, pk, gamma):
    a = np.sqrt(gamma * pk / rho)
    if p > pk:  # shock
        A = 2.0 / ((gamma + 1.0) * rho)
        B = (gamma - 1.0) / (gamma + 1.0) * pk
        return (p - pk) * np.sqrt(A / (p + B))
    return 2.0 * a / (gamma - 1.0) * ((p / pk) ** ((gamma - 1.0) / (2.0 * gamma)) - 1.0)


def star_state(WL, WR, gamma):
    """Exact star pressure and velocity for primitive states (rho, u, p)."""
    rl, ul, pl = WL
    rr, ur, pr = WR
    f = lambda p: _fk(p, rl, pl, gamma) + _fk(p, rr, pr, gamma) + (ur - ul)
    hi = max(pl, pr)
    while f(hi) < 0.0:
        hi *= 2.0
    ps = brentq(f, 1e-14 * hi, hi, xtol=1e-15, rtol=1e-15, maxiter=500)
    us = 0.5 * (ul + ur) + 0.5 * (_fk(ps, rr, pr, gamma) - _fk(ps, rl, pl, gamma))
    return ps, us


def star_densities(WL, WR, gamma):
    rl, ul, pl = WL
    rr, ur, pr = WR
    ps, us = star_state(WL, WR, gamma)
    g = (gamma - 1.0) / (gamma + 1.0)

    def rho_star(rk, pk):
        if ps > pk:
            return rk * (ps / pk + g) / (g * ps / pk + 1.0)
        return rk * (ps / pk) ** (1.0 / gamma)

    return rho_star(rl, pl), rho_star(rr, pr)


def sample(WL, WR, gamma, xi):
    """Exact solution (rho, u, p) at similarity coordinates xi = (x - x0)/t."""
    rl, ul, pl = WL
    rr, ur, pr = WR
    ps, us = star_state(WL, WR, gamma)
    rsl, rsr = star_densities(WL, WR, gamma)
    al = np.sqrt(gamma * pl / rl)
    ar = np.sqrt(gamma * pr / rr)
    xi = np.atleast_1d(np.asarray(xi, dtype=np.float64))
    rho = np.empty_like(xi)
    u = np.empty_like(xi)
    p = np.empty_like(xi)
    gm1, gp1 = gamma - 1.0, gamma + 1.0
    for n, s in enumerate(xi):
        if s <= us:  # left of the contact
            if ps > pl:  # left shock
                sl = ul - al * np.sqrt(gp1 / (2 * gamma) * ps / pl + gm1 / (2 * gamma))
                st = (rl, ul, pl) if s <= sl else (rsl, us, ps)
            else:  # left rarefaction
                ash = al * (ps / pl) ** (gm1 / (2 * gamma))
                head, tail = ul - al, us - ash
                if s <= head:
                    st = (rl, ul, pl)
                elif s >= tail:
                    st = (rsl, us, ps)
                else:
                    c = 2.0 / gp1 + gm1 / (gp1 * al) * (ul - s)
                    st = (rl * c ** (2.0 / gm1), 2.0 / gp1 * (al + gm1 / 2 * ul + s),
                          pl * c ** (2 * gamma / gm1))
        else:  # right of the contact
            if ps > pr:
                sr = ur + ar * np.sqrt(gp1 / (2 * gamma) * ps / pr + gm1 / (2 * gamma))
                st = (rr, ur, pr) if s >= sr else (rsr, us, ps)
            else:
                ash = ar * (ps / pr) ** (gm1 / (2 * gamma))
                head, tail = ur + ar, us + ash
                if s >= head:
                    st = (rr, ur, pr)
                elif s <= tail:
                    st = (rsr, us, ps)
                else:
                    c = 2.0 / gp1 - gm1 / (gp1 * ar) * (ur - s)
                    st = (rr * c ** (2.0 / gm1), 2.0 / gp1 * (-ar + gm1 / 2 * ur + s),
                          pr * c ** (2 * gamma / gm1))
        rho[n], u[n], p[n] = st
    return rho, u, p


def cell_average_sod(N, t, gamma, WL=(1.0, 0.0, 1.0), WR=(0.125, 0.0, 0.1), x0=0.5, sub=64):
    """Exact Sod density averaged over each of N cells on [0, 1] at time t."""
    x = (np.arange(N * sub) + 0.5) / (N * sub)
    rho, _, _ = sample(WL, WR, gamma, (x - x0) / t)
    return rho.reshape(N, sub).mean(axis=1)


def euler_flux(W, gamma):
    """Physical x-flux of the Euler equations (Sec. 3.1, Eq. 4) for primitive
    (rho, u, v, w, p): [rho u, rho u^2 + p, rho u v, rho u w, u (E + p)]."""
    r, u, v, w, p = W
    E = p / (gamma - 1.0) + 0.5 * r * (u * u + v * v + w * w)
    return np.array([r * u, r * u * u + p, r * u * v, r * u * w, u * (E + p)])


def sedov_radius(t, E, rho0, xi0):
    """Sedov-Taylor shock radius xi0 (E t^2 / rho0)^(1/5)."""
    return xi0 * (E * t * t / rho0) ** 0.2


def read_golden(name):
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", name)
    rows = []
    with open(path) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            rows.append(line.split())
    return rows
