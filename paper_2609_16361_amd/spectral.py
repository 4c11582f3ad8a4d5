"""Spectral dissipation channels of a periodic state (post-processing, Sec. 3.3).

Sec. 3.3 evaluates the solenoidal and dilatational dissipation with Fourier
derivatives, like the solvers it compares with; a difference stencil would smear
the weak embedded shocks and bias the dilatational channel low.  The step kernels report the same channels from the gradients they
reconstruct in the collision; this module recomputes them from the conserved
fields alone (the output of lbm_moments), with exact Fourier derivatives on the
periodic lattice:

    E_k   = < rho |u|^2 / 2 >
    eps_s = < mu(T) |curl u|^2 >
    eps_d = < (4/3) mu(T) (div u)^2 >

in lattice units, averages over the cells (divide by rho0 and convert with the
case's scales for the paper's units).  mu(T) follows the case's viscosity law
(Sutherland with T_S, or constant), with T = p / rho from the equation of state.
It runs on the host with NumPy, off the step path.
"""
import numpy as np


def _mu(params, T):
    mu_ref = params["mu_ref"]
    if int(params["mu_law"]) == 0:
        return np.full_like(T, mu_ref)
    t = T / params["T_ref"]
    ts = params["T_S"]
    return mu_ref * (1.0 + ts) * t ** 1.5 / (t + ts)


def velocity_gradients(u):
    """Exact Fourier derivatives of a periodic vector field u[3][nz][ny][nx] (one
    cell = unit length): returns grad[j][c] = d u_j / d x_c, same shape."""
    nz, ny, nx = u[0].shape
    kx = 2.0 * np.pi * np.fft.fftfreq(nx)
    ky = 2.0 * np.pi * np.fft.fftfreq(ny)
    kz = 2.0 * np.pi * np.fft.fftfreq(nz)
    # the Nyquist mode of an even length has no odd derivative
    for k, n in ((kx, nx), (ky, ny), (kz, nz)):
        if n % 2 == 0:
            k[n // 2] = 0.0
    K = (kx[None, None, :], ky[None, :, None], kz[:, None, None])
    grad = np.empty((3, 3, nz, ny, nx))
    for j in range(3):
        uh = np.fft.fftn(u[j])
        for c in range(3):
            grad[j, c] = np.real(np.fft.ifftn(1j * K[c] * uh))
    return grad


def channels(Q, params):
    """(E_k, eps_s, eps_d) of the conserved fields Q[5][nz][ny][nx] (lattice units,
    cell averages)."""
    gamma = params["gamma"]
    rho = Q[0]
    u = Q[1:4] / rho[None]
    k2 = (u * u).sum(axis=0)
    p = (gamma - 1.0) * (Q[4] - 0.5 * rho * k2)
    mu = _mu(params, p / rho)
    g = velocity_gradients(u)
    wx = g[2, 1] - g[1, 2]
    wy = g[0, 2] - g[2, 0]
    wz = g[1, 0] - g[0, 1]
    theta = g[0, 0] + g[1, 1] + g[2, 2]
    ek = float(np.mean(0.5 * rho * k2))
    eps_s = float(np.mean(mu * (wx * wx + wy * wy + wz * wz)))
    eps_d = float(np.mean(4.0 / 3.0 * mu * theta * theta))
    return ek, eps_s, eps_d
