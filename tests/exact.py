"""Closed-form reference solutions used to pin the oracle (test infrastructure).

* Exact solution of the Riemann problem for the Euler equations of an ideal gas
  (the reference of the Sod tube, Sec. 3.2): the star pressure solves
  f_L(p) + f_R(p) + (u_R - u_L) = 0, where f_K is the shock (Rankine-Hugoniot)
  or rarefaction (isentropic) velocity jump across the wave on side K; Newton
  iteration in FP64, then the self-similar solution is sampled at x/t.
* Linearised Navier-Stokes-Fourier dispersion relation of a plane wave around a
  uniform state (for the viscous and conductive decay pins): the exact
  eigenvalues of the linear operator of eq. 2 for one Fourier mode.
"""
import math

import numpy as np


def _wave_jump(p, rho_k, p_k, gamma):
    """Velocity jump f_K(p) across a shock (p > p_k) or rarefaction (p <= p_k)."""
    c_k = math.sqrt(gamma * p_k / rho_k)
    if p > p_k:
        A = 2.0 / ((gamma + 1.0) * rho_k)
        B = (gamma - 1.0) / (gamma + 1.0) * p_k
        f = (p - p_k) * math.sqrt(A / (p + B))
        df = math.sqrt(A / (B + p)) * (1.0 - (p - p_k) / (2.0 * (B + p)))
    else:
        e = (gamma - 1.0) / (2.0 * gamma)
        f = 2.0 * c_k / (gamma - 1.0) * ((p / p_k) ** e - 1.0)
        df = 1.0 / (rho_k * c_k) * (p / p_k) ** (-(gamma + 1.0) / (2.0 * gamma))
    return f, df


def riemann_star(left, right, gamma=1.4):
    """left/right = (rho, u, p) -> (p_star, u_star)."""
    rl, ul, pl = left
    rr, ur, pr = right
    p = 0.5 * (pl + pr)
    for _ in range(100):
        fl, dfl = _wave_jump(p, rl, pl, gamma)
        fr, dfr = _wave_jump(p, rr, pr, gamma)
        g = fl + fr + (ur - ul)
        dp = g / (dfl + dfr)
        p_new = max(p - dp, 1e-14)
        if abs(p_new - p) < 1e-15 * p:
            p = p_new
            break
        p = p_new
    fl, _ = _wave_jump(p, rl, pl, gamma)
    fr, _ = _wave_jump(p, rr, pr, gamma)
    u = 0.5 * (ul + ur) + 0.5 * (fr - fl)
    return p, u


def riemann_sample(xi, left, right, gamma=1.4):
    """Self-similar exact solution at xi = (x - x0)/t; returns (rho, u, p) arrays."""
    rl, ul, pl = left
    rr, ur, pr = right
    ps, us = riemann_star(left, right, gamma)
    cl = math.sqrt(gamma * pl / rl)
    cr = math.sqrt(gamma * pr / rr)
    g1 = (gamma - 1.0) / (gamma + 1.0)
    xi = np.asarray(xi, dtype=np.float64)
    rho = np.empty_like(xi)
    u = np.empty_like(xi)
    p = np.empty_like(xi)
    for n, s in enumerate(xi.flat):
        if s <= us:  # left of contact
            if ps > pl:  # left shock
                rs = rl * ((ps / pl + g1) / (g1 * ps / pl + 1.0))
                S = ul - cl * math.sqrt((gamma + 1.0) / (2 * gamma) * ps / pl + (gamma - 1.0) / (2 * gamma))
                st = (rl, ul, pl) if s < S else (rs, us, ps)
            else:  # left rarefaction
                rs = rl * (ps / pl) ** (1.0 / gamma)
                cs = cl * (ps / pl) ** ((gamma - 1.0) / (2 * gamma))
                head, tail = ul - cl, us - cs
                if s < head:
                    st = (rl, ul, pl)
                elif s > tail:
                    st = (rs, us, ps)
                else:
                    uu = 2.0 / (gamma + 1.0) * (cl + (gamma - 1.0) / 2.0 * ul + s)
                    cc = 2.0 / (gamma + 1.0) * (cl + (gamma - 1.0) / 2.0 * (ul - s))
                    rr_ = rl * (cc / cl) ** (2.0 / (gamma - 1.0))
                    st = (rr_, uu, pl * (cc / cl) ** (2.0 * gamma / (gamma - 1.0)))
        else:  # right of contact
            if ps > pr:  # right shock
                rs = rr * ((ps / pr + g1) / (g1 * ps / pr + 1.0))
                S = ur + cr * math.sqrt((gamma + 1.0) / (2 * gamma) * ps / pr + (gamma - 1.0) / (2 * gamma))
                st = (rr, ur, pr) if s > S else (rs, us, ps)
            else:  # right rarefaction
                rs = rr * (ps / pr) ** (1.0 / gamma)
                cs = cr * (ps / pr) ** ((gamma - 1.0) / (2 * gamma))
                head, tail = ur + cr, us + cs
                if s > head:
                    st = (rr, ur, pr)
                elif s < tail:
                    st = (rs, us, ps)
                else:
                    uu = 2.0 / (gamma + 1.0) * (-cr + (gamma - 1.0) / 2.0 * ur + s)
                    cc = 2.0 / (gamma + 1.0) * (cr - (gamma - 1.0) / 2.0 * (ur - s))
                    rr_ = rr * (cc / cr) ** (2.0 / (gamma - 1.0))
                    st = (rr_, uu, pr * (cc / cr) ** (2.0 * gamma / (gamma - 1.0)))
        rho.flat[n], u.flat[n], p.flat[n] = st
    return rho, u, p


def linear_nsf_modes(k, rho0, T0, mu, kappa, gamma, transverse=False):
    """Eigenvalues lambda of a plane wave exp(i k x + lambda t) of eq. 2 linearised
    about rest (rho0, T0), p = rho T, c_v = 1/(gamma-1).

    Longitudinal variables (rho', u', T'):
      rho0 u' ...  d rho'/dt = -i k rho0 u'
      rho0 du'/dt = -i k (T0 rho' + rho0 T') - (4/3) mu k^2 u'
      rho0 c_v dT'/dt = -p0 i k u' - kappa k^2 T'
    Transverse (shear) mode: lambda = -mu k^2 / rho0."""
    if transverse:
        return np.array([-mu * k * k / rho0])
    cv = 1.0 / (gamma - 1.0)
    p0 = rho0 * T0
    A = np.array([
        [0.0, -1j * k * rho0, 0.0],
        [-1j * k * T0 / rho0, -(4.0 / 3.0) * mu * k * k / rho0, -1j * k],
        [0.0, -1j * k * p0 / (rho0 * cv), -kappa * k * k / (rho0 * cv)],
    ], dtype=complex)
    return np.linalg.eigvals(A)
