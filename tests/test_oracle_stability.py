"""Linear stability of the oracle's update about a uniform state (von Neumann).

The Jacobian of one cell's collision (central differences of the oracle) composed
with exact streaming, exp(-i k.c_i) per direction, gives the amplification matrix
of a Fourier mode; its spectral radius is the growth per step.

Pin.  For a mode along x and an inviscid closure, the regularized update of the
collision of Algorithm 1 (Sec. 2.5: the equilibrium with the flux in its first
moment, plus (1 - omega) times the first-moment part of the non-equilibrium)
touches only the zeroth and first moments of each field; streaming a mode
exp(i k x) then gives, per field, with a = the linearised flux dPhi_x/dQ:
    Q' = (3 + cos k)/4 Q - i sin k J*,    J' = -(i sin k)/4 Q + cos k J*,
    J* = omega a Q + (1 - omega) J
(D3Q7 weights 1/4 and 1/8).  The Euler flux Jacobian has the eigenvalues u - c,
u (three times) and u + c, so the 35x35 spectrum is the union of this 2x2
spectrum at those speeds, 1 - omega (the transverse first moments) and 0 (the
second moments the regularization discards).  test_regularized_linearisation_
closed_form checks the oracle's linearisation against that union.

Consequences for the reading of the time step:
  * the regularized update is stable for advection speeds up to a_crit(omega), with
    a_crit(1) = 1/2 exactly and a_crit ~ 0.41 sqrt(2 - omega) as omega -> 2
  * the Sod point of Table 1 (omega 1.4, fastest characteristic 0.35 cells per step)
    lies inside; the vortex point (omega -> 2, 0.1 cells per step) lies outside
  * BGK at rest is neutrally stable; enough physical viscosity damps the growth
"""
import math

import numpy as np
import pytest

import oracle
from paper_2609_16361_amd import inputs

C = np.array([[0, 0, 0], [1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1]])


def collision_jacobian(u, c, omega, coll, mu, gamma=1.4):
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
    return Jc


def amplification(Jc, k):
    """Collision Jacobian followed by exact streaming of the mode exp(i k.x)."""
    S = np.tile(np.exp(-1j * (C @ np.asarray(k, dtype=float))), 5)
    return S[:, None] * Jc


def spectral_radius(u, c, omega, coll, mu, nk=10):
    Jc = collision_jacobian(u, c, omega, coll, mu)
    best = 0.0
    for kx in np.linspace(0, math.pi, nk):
        for ky in np.linspace(0, math.pi, nk // 2 + 1):
            best = max(best, np.abs(np.linalg.eigvals(amplification(Jc, (kx, ky, 0.0)))).max())
    return best


def closed_form(a, omega, k):
    """The 2x2 (Q, J_x) amplification of one field with linear flux a Q."""
    cs, sn = math.cos(k), math.sin(k)
    return np.array([[(3 + cs) / 4 - 1j * sn * omega * a, -1j * sn * (1 - omega)],
                     [-1j * sn / 4 + omega * a * cs, (1 - omega) * cs]])


def closed_form_radius(a, omega, nk=721):
    return max(np.abs(np.linalg.eigvals(closed_form(a, omega, k))).max()
               for k in np.linspace(1e-4, math.pi, nk))


def critical_speed(omega):
    lo, hi = 0.0, 1.0
    for _ in range(40):
        mid = 0.5 * (lo + hi)
        if closed_form_radius(mid, omega) <= 1.0 + 1e-12:
            lo = mid
        else:
            hi = mid
    return lo


@pytest.mark.parametrize("u,c,omega", [(0.1, 0.08, 1.99996), (0.03, 0.05, 1.4), (0.0, 0.08, 1.9),
                                       (-0.2, 0.1, 1.2)])
def test_regularized_linearisation_closed_form(u, c, omega):
    Jc = collision_jacobian((u, 0, 0), c, omega, inputs.RLB_SENSOR, 0.0)
    for k in (0.3, 1.1, 2.0, 2.9):
        got = np.linalg.eigvals(amplification(Jc, (k, 0.0, 0.0)))
        want = [0.0] * 15 + [1.0 - omega] * 10
        for a in (u - c, u, u, u, u + c):
            want += list(np.linalg.eigvals(closed_form(a, omega, k)))
        want = np.array(want)
        # every predicted eigenvalue is matched by a distinct oracle eigenvalue
        left = list(got)
        for w in sorted(want, key=lambda z: -abs(z)):
            j = int(np.argmin([abs(g - w) for g in left]))
            assert abs(left[j] - w) < 1e-6, (k, w, left[j])
            left.pop(j)
        assert np.abs(got).max() == pytest.approx(np.abs(want).max(), abs=1e-7)


def test_critical_speed_of_the_regularized_update():
    # omega = 1 is the plain equilibrium update: |(3 + cos k)/4 - i a sin k| <= 1 for
    # every k exactly when a^2 <= (7 + cos k)/(16 (1 + cos k)), smallest (1/4) at k -> 0
    assert critical_speed(1.0) == pytest.approx(0.5, abs=1e-4)
    for om in (1.99, 1.9999, 1.99996):
        assert critical_speed(om) == pytest.approx(0.408 * math.sqrt(2.0 - om), rel=0.02)
    # Table 1: Sod (omega 1.4, fastest characteristic 0.35 cells per step) is inside
    assert critical_speed(1.4) > 0.35
    assert closed_form_radius(0.35, 1.4) <= 1.0 + 1e-9
    # the vortex (omega from f_mu = 0.001 at 256^3, 0.1 cells per step) is outside
    assert closed_form_radius(0.1, 1.99996) > 1.03


def test_bgk_at_rest_is_neutral():
    assert spectral_radius((0, 0, 0), 0.05, 1.9999, inputs.BGK, 1e-4) == pytest.approx(1.0, abs=1e-6)


def test_regularized_near_two_grows_with_lattice_speed():
    g_slow = spectral_radius((0, 0, 0), 0.03, 1.9999, inputs.RLB_SENSOR, 1e-4)
    g_fast = spectral_radius((0.1, 0, 0), 0.08, 1.9999, inputs.RLB_SENSOR, 1e-4)
    assert 1.0 < g_slow < g_fast
    assert g_fast > 1.05


def test_viscosity_damps_the_grid_scale_growth():
    assert spectral_radius((0, 0, 0), 0.05, 1.9999, inputs.RLB_SENSOR, 1e-3) <= 1.0 + 1e-9
