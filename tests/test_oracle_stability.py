"""Linear stability of the oracle's update about a uniform state (von Neumann).

The Jacobian of one cell's collision (central differences of the oracle) composed
with exact streaming, exp(-i k.c_i) per direction, gives the amplification matrix
of a Fourier mode; its spectral radius is the growth per step.  This documents
the reading of the time step used for the near-omega = 2 workloads:
  * BGK at rest is neutrally stable (|lambda| = 1, the conserved modes)
  * the regularized collision at omega -> 2 with a nearly inviscid closure grows at
    grid-scale wavenumbers, faster for larger lattice sound and flow speeds
  * enough physical viscosity (reconstructed stress) damps that growth
"""
import math

import numpy as np
import pytest

import oracle
from paper_2609_16361_amd import inputs

C = np.array([[0, 0, 0], [1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1]])


def spectral_radius(u, c, omega, coll, mu, nk=10):
    gamma = 1.4
    p = c * c / gamma
    prm = inputs.base_params(1, 1, 1, (0, 0, 0), mu=mu, omega=omega, collision=coll,
                             sensor_gain=40, J_min=1e-2, omega_min=1.987, p_min=1e-12,
                             rho_min=1e-6)
    one = np.ones((1, 1, 1))
    Q = inputs.conserved(one, [v * one for v in u], p * one, gamma)
    f0 = oracle.init(prm, Q)[:, 0]
    fo, _ = oracle.collide(prm, f0)
    np.testing.assert_allclose(fo, f0, rtol=1e-12, atol=1e-15)   # equilibrium is fixed
    h = 1e-7
    Jc = np.zeros((35, 35))
    for j in range(35):
        e = np.zeros(35)
        e[j] = h
        a, _ = oracle.collide(prm, f0 + e)
        b, _ = oracle.collide(prm, f0 - e)
        Jc[:, j] = (a - b) / (2 * h)
    best = 0.0
    for kx in np.linspace(0, math.pi, nk):
        for ky in np.linspace(0, math.pi, nk // 2 + 1):
            S = np.diag(np.tile(np.exp(-1j * (C @ np.array([kx, ky, 0.0]))), 5))
            best = max(best, np.abs(np.linalg.eigvals(S @ Jc)).max())
    return best


def test_bgk_at_rest_is_neutral():
    assert spectral_radius((0, 0, 0), 0.05, 1.9999, inputs.BGK, 1e-4) == pytest.approx(1.0, abs=1e-6)


def test_regularized_near_two_grows_with_lattice_speed():
    g_slow = spectral_radius((0, 0, 0), 0.03, 1.9999, inputs.RLB_SENSOR, 1e-4)
    g_fast = spectral_radius((0.1, 0, 0), 0.08, 1.9999, inputs.RLB_SENSOR, 1e-4)
    assert 1.0 < g_slow < g_fast
    assert g_fast > 1.05


def test_viscosity_damps_the_grid_scale_growth():
    assert spectral_radius((0, 0, 0), 0.05, 1.9999, inputs.RLB_SENSOR, 1e-3) <= 1.0 + 1e-9
