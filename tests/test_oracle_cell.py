"""Pins of the oracle's per-cell update (Algorithm 1) against closed forms.

Each test checks one step of the oracle against something the paper or the
mathematics fixes independently of the oracle's own code:
  * equilibrium moments of the linear D3Q7 equilibrium (Sec. 2.2, c_s^2 = 1/4)
  * the diffusive-flux Jacobian of eq. 5 against derivatives of the flux of eq. 2
  * exact recovery of a prescribed gradient through eqs. 3-4
  * the chain rule to grad u and grad T (complex-step derivatives of u(Q), T(Q))
  * moments of the regularized and BGK post-collision populations (Sec. 2.5)
  * the compression sensor's gate and clamp (Sec. 2.5, Listing 2)
  * Sutherland law limits and positivity floors (Listing 1, Table 1)
"""
import math

import numpy as np
import pytest

import oracle

C = np.array([[0, 0, 0], [1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1]], float)
CS2 = 0.25
# weights w_0 = 1/4, w_i = 1/8 -- the nearest-neighbour set with c_s^2 = 1/4
W = np.array([0.25] + [0.125] * 6)

GAMMA = 1.4


def params(**kw):
    p = dict(nx=1, ny=1, nz=1, bc=[0, 0, 0], collision=0, mu_law=1, gamma=GAMMA,
             mu_ref=0.03, kappa_ref=0.03 * GAMMA / (GAMMA - 1) / 0.71, T_ref=0.004,
             T_S=0.4042, omega=[1.9] * 5, sensor_gain=20.0, J_min=3e-3, omega_min=1.0,
             rho_min=1e-4, p_min=1e-9)
    p.update(kw)
    return p


def state(seed=0):
    rng = np.random.default_rng(seed)
    rho = 1.0 + 0.2 * rng.uniform(-1, 1)
    u = 0.03 * rng.uniform(-1, 1, 3)
    p = 0.005 * (1 + 0.2 * rng.uniform(-1, 1))
    Q = np.array([rho, *(rho * u), p / (GAMMA - 1) + 0.5 * rho * u @ u])
    return Q


def prim(Q):
    """Primitives of eq. 2 (no floors); works with complex input for complex-step."""
    rho = Q[0]
    u = Q[1:4] / rho
    p = (GAMMA - 1) * (Q[4] - 0.5 * rho * (u[0] * u[0] + u[1] * u[1] + u[2] * u[2]))
    return rho, u, p, p / rho


def sutherland(prm, T):
    t = T / prm["T_ref"]
    return prm["mu_ref"] * (1 + prm["T_S"]) * t ** 1.5 / (t + prm["T_S"])


def grad_prims(Q, gradQ):
    """grad u [j][c] and grad T [c] by complex-step differentiation of u(Q), T(Q)
    along each spatial column of gradQ[5][3]."""
    h = 1e-30
    gu = np.zeros((3, 3))
    gT = np.zeros(3)
    for c in range(3):
        _, u, _, T = prim(Q.astype(complex) + 1j * h * gradQ[:, c])
        gu[:, c] = u.imag / h
        gT[c] = T.imag / h
    return gu, gT


def flux_adv(Q):
    rho, u, p, _ = prim(Q)
    F = np.zeros((5, 3))
    F[0] = Q[1:4]
    for j in range(3):
        F[1 + j] = Q[1 + j] * u
        F[1 + j, j] += p
    F[4] = (Q[4] + p) * u
    return F


def flux_diff(prm, Q, gradQ):
    """Diffusive part of the flux of eq. 2: (0, -tau, -tau.u + q), from the
    Newtonian stress and Fourier flux evaluated on grad u and grad T."""
    rho, u, p, T = prim(Q)
    mu = sutherland(prm, T) if prm["mu_law"] == 1 else prm["mu_ref"]
    kappa = prm["kappa_ref"] * mu / prm["mu_ref"]
    gu, gT = grad_prims(Q, gradQ)
    th = np.trace(gu)
    tau = mu * (gu + gu.T - 2.0 / 3.0 * th * np.eye(3))
    q = -kappa * gT
    F = np.zeros((5, 3))
    F[1:4] = -tau
    F[4] = -tau @ u + q
    return F


def pops_from_moments(Q, J):
    """Any population set with zeroth moments Q[5] and first moments J[5][3]."""
    f = np.zeros(35)
    for k in range(5):
        for i in range(7):
            f[7 * k + i] = W[i] * (Q[k] + (C[i] @ J[k]) / CS2)
    return f


def moments(f):
    f = f.reshape(5, 7)
    return f.sum(1), f @ C, np.einsum("ki,ia,ib->kab", f, C, C)


# ----------------------------------------------------------------------------
def test_lattice_and_equilibrium_moments():
    """P1/P2: the equilibrium carries Q in the zeroth moment, the advective flux in
    the first and c_s^2 Q I in the second (the start of a uniform state is its
    equilibrium; each cell of a 1x1x1 periodic grid is a uniform state)."""
    prm = params(nx=1, ny=1, nz=1)
    rng = np.random.default_rng(1)
    Q = np.stack([state(s) for s in range(12)], axis=1)
    Q += 1e-3 * rng.standard_normal(Q.shape)
    for n in range(12):
        q = Q[:, n]
        f = oracle.init(prm, q.reshape(5, 1, 1, 1))
        m0, m1, m2 = moments(f[:, 0])
        np.testing.assert_allclose(m0, q, rtol=1e-14, atol=1e-16)
        np.testing.assert_allclose(m1, flux_adv(q), rtol=1e-13, atol=1e-17)
        for k in range(5):
            np.testing.assert_allclose(m2[k], CS2 * q[k] * np.eye(3), rtol=1e-13, atol=1e-17)


def test_jacobian_matches_flux_derivative():
    """P6: the dense M of eq. 5 equals d Phi_diff / d(grad Q) of the flux of eq. 2
    (Phi_diff is linear in grad Q, so each column is Phi_diff of a unit gradient)."""
    for mu_law in (0, 1):
        prm = params(mu_law=mu_law)
        Q = state(3)
        f = pops_from_moments(Q, flux_adv(Q))
        _, info = oracle.collide(prm, f)
        M = info["M"]
        Mt = np.zeros((15, 15))
        for col in range(15):
            g = np.zeros((5, 3))
            g[col // 3, col % 3] = 1.0
            Mt[:, col] = flux_diff(prm, Q, g).reshape(15)
        scale = np.abs(Mt).max()
        np.testing.assert_allclose(M, Mt, atol=1e-12 * scale)
        # structure stated with eq. 5: mass row zero, block lower triangular
        assert np.all(M[0:3] == 0)
        assert np.all(M[3:12, 12:15] == 0)


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
@pytest.mark.parametrize("omega", [1.2, 1.9, 1.9999])
def test_exact_gradient_recovery(seed, omega):
    """eqs. 3-4: if the first moment carries J = Phi_adv + Phi_diff(grad Q)
    - c_s^2 tau grad Q, the reconstruction returns grad Q exactly, and the chain
    rule returns the derivatives of u(Q) and T(Q) along it."""
    rng = np.random.default_rng(100 + seed)
    prm = params(omega=[omega] * 5, mu_ref=0.05 * rng.uniform(0.2, 1.0))
    Q = state(seed)
    gradQ = 1e-3 * rng.standard_normal((5, 3)) * np.abs(Q)[:, None].clip(1e-2)
    tau = 1.0 / np.array(prm["omega"])
    J = flux_adv(Q) + flux_diff(prm, Q, gradQ) - CS2 * tau[:, None] * gradQ
    f = pops_from_moments(Q, J)
    _, info = oracle.collide(prm, f)
    np.testing.assert_allclose(info["gradQ"], gradQ, rtol=1e-9, atol=1e-12 * np.abs(gradQ).max())
    gu, gT = grad_prims(Q, gradQ)
    np.testing.assert_allclose(info["grad_u"], gu, rtol=1e-9, atol=1e-12 * np.abs(gu).max())
    np.testing.assert_allclose(info["grad_T"], gT, rtol=1e-9, atol=1e-12 * np.abs(gT).max())
    # the closures enter the equilibrium flux (Algorithm 1)
    np.testing.assert_allclose(info["Phi"], flux_adv(Q) + flux_diff(prm, Q, gradQ),
                               rtol=1e-10, atol=1e-14)


def test_momentum_block_damps_only_sym_dev():
    """Sec. 2.4, eq. 6: with rho uniform and u = 0 the momentum block leaves the
    antisymmetric part (rotation) and the trace (expansion) of the direct gradient as
    they are and divides its traceless symmetric part by 1 + beta,
    beta = 2 nu omega / c_s^2."""
    omega = 1.95
    prm = params(mu_law=0, mu_ref=0.04, omega=[omega] * 5)
    Q = np.array([1.0, 0.0, 0.0, 0.0, 0.005 / (GAMMA - 1)])
    rng = np.random.default_rng(7)
    G = 1e-3 * rng.standard_normal((3, 3))           # grad(rho u) tilde
    gradQt = np.zeros((5, 3))
    gradQt[1:4] = G
    J = flux_adv(Q) - CS2 / omega * gradQt
    _, info = oracle.collide(prm, pops_from_moments(Q, J))
    beta = 2 * 0.04 * omega / CS2
    sym = 0.5 * (G + G.T)
    dev = sym - np.trace(G) / 3 * np.eye(3)
    expect = (G - dev) + dev / (1 + beta)
    np.testing.assert_allclose(info["grad_u"], expect, rtol=1e-10, atol=1e-16)


def test_energy_row_ratio_gamma_over_2Pr():
    """eq. 7: at rest the conduction damping of grad E is 1/(1 + c_s^-2 omega gamma
    alpha) with alpha = kappa/(rho c_p); its coefficient stands to the shear one
    (2 nu) in the ratio gamma/(2 Pr)."""
    omega, mu, Pr = 1.9, 0.02, 0.71
    kappa = mu * GAMMA / (GAMMA - 1) / Pr
    prm = params(mu_law=0, mu_ref=mu, kappa_ref=kappa, omega=[omega] * 5)
    Q = np.array([1.0, 0.0, 0.0, 0.0, 0.005 / (GAMMA - 1)])
    gE = np.array([1e-4, -2e-4, 3e-5])
    gradQt = np.zeros((5, 3))
    gradQt[4] = gE
    J = flux_adv(Q) - CS2 / omega * gradQt
    _, info = oracle.collide(prm, pops_from_moments(Q, J))
    cp = GAMMA / (GAMMA - 1)
    galpha = GAMMA * kappa / (1.0 * cp)
    np.testing.assert_allclose(info["gradQ"][4], gE / (1 + omega / CS2 * galpha), rtol=1e-12)
    assert math.isclose(galpha / (2 * mu), GAMMA / (2 * Pr), rel_tol=1e-12)


def _random_cell(seed, amp=1e-4):
    rng = np.random.default_rng(seed)
    Q = state(seed)
    J = flux_adv(Q) + amp * rng.standard_normal((5, 3))
    f = pops_from_moments(Q, J) + amp * 0.1 * rng.standard_normal(35)
    return f


@pytest.mark.parametrize("seed", range(5))
def test_regularized_collision_moments(seed):
    """Sec. 2.5: the regularized collision conserves Q, relaxes the first moment to
    omega_h Phi + (1-omega_h) J and discards every higher moment, leaving the
    second moment at its equilibrium value c_s^2 Q I."""
    prm = params(collision=0)
    f = _random_cell(seed)
    fo, info = oracle.collide(prm, f)
    Q, J, _ = moments(f)
    Qo, Jo, M2o = moments(fo)
    np.testing.assert_allclose(Qo, Q, rtol=1e-14, atol=1e-18)
    oh = info["omega_h"][:, None]
    np.testing.assert_allclose(Jo, oh * info["Phi"] + (1 - oh) * J, rtol=1e-12, atol=1e-18)
    for k in range(5):
        np.testing.assert_allclose(M2o[k], CS2 * Q[k] * np.eye(3), rtol=1e-12, atol=1e-18)


@pytest.mark.parametrize("seed", range(3))
def test_bgk_collision_moments(seed):
    """Sec. 2.2: BGK relaxes every moment towards the equilibrium at rate omega."""
    prm = params(collision=1, omega=[1.7, 1.8, 1.8, 1.8, 1.6])
    f = _random_cell(seed)
    fo, info = oracle.collide(prm, f)
    Q, J, M2 = moments(f)
    Qo, Jo, M2o = moments(fo)
    om = np.array(prm["omega"])
    np.testing.assert_allclose(Qo, Q, rtol=1e-14, atol=1e-18)
    np.testing.assert_allclose(Jo, J + om[:, None] * (info["Phi"] - J), rtol=1e-12, atol=1e-18)
    for k in range(5):
        np.testing.assert_allclose(M2o[k], M2[k] + om[k] * (CS2 * Q[k] * np.eye(3) - M2[k]),
                                   rtol=1e-12, atol=1e-18)


@pytest.mark.parametrize("s_target,expect", [
    (-0.01, 0.0),          # expansion: never fires
    (1.5e-3, 0.0),         # compression below the dead band J_min = 3e-3
    (4e-3, 20.0 * 4e-3),   # linear in the gain
    (0.2, 1.0),            # clamped at 1
])
def test_sensor_gate(s_target, expect):
    """Sec. 2.5: s = -div(u)/c_s; chi = clamp(g s) only in compression with s > J_min."""
    omega = 1.9
    prm = params(mu_law=0, mu_ref=0.01, omega=[omega] * 5, sensor_gain=20.0, J_min=3e-3,
                 omega_min=1.0)
    Q = state(11)
    rho, u, _, _ = prim(Q)
    theta = -s_target * math.sqrt(CS2)
    gu = np.diag([theta, 0.0, 0.0]) + 1e-5 * np.array([[0, 1, 0], [-1, 0, 0], [0, 0, 0]])
    grho = np.array([1e-4, 0, 0])
    gradQ = np.zeros((5, 3))
    gradQ[0] = grho
    gradQ[1:4] = rho * gu + np.outer(u, grho)
    gradQ[4] = 1e-6
    tau = 1.0 / omega
    J = flux_adv(Q) + flux_diff(prm, Q, gradQ) - CS2 * tau * gradQ
    f = pops_from_moments(Q, J)
    fo, info = oracle.collide(prm, f)
    assert info["theta"] == pytest.approx(theta, rel=1e-9)
    assert info["chi"] == pytest.approx(expect, rel=1e-9, abs=1e-15)
    oh = omega - expect * (omega - 1.0)
    np.testing.assert_allclose(info["omega_h"], oh, rtol=1e-12)
    # the reduced rate is the one the regularized collision applies
    _, Jo, _ = moments(fo)
    np.testing.assert_allclose(Jo, oh * info["Phi"] + (1 - oh) * J, rtol=1e-9, atol=1e-16)


def test_sutherland_limits():
    """Listing 1: mu(T_ref) = mu_ref; mu ~ T^(1/2) for T >> T_S T_ref and
    ~ T^(3/2) for T << T_S T_ref."""
    prm = params(mu_law=1, mu_ref=0.02, T_ref=0.01)

    def mu_at(T):
        rho = 1.0
        Q = np.array([rho, 0, 0, 0, rho * T / (GAMMA - 1)])
        _, info = oracle.collide(prm, pops_from_moments(Q, flux_adv(Q)))
        assert info["T"] == pytest.approx(T, rel=1e-12)
        return info["mu"]

    assert mu_at(0.01) == pytest.approx(0.02, rel=1e-13)
    hi1, hi2 = mu_at(0.01 * 1e6), mu_at(0.01 * 4e6)
    assert hi2 / hi1 == pytest.approx(2.0, rel=1e-6)
    lo1, lo2 = mu_at(0.01 * 1e-7), mu_at(0.01 * 4e-7)
    assert lo2 / lo1 == pytest.approx(8.0, rel=1e-5)
    prm0 = params(mu_law=0, mu_ref=0.02)
    Q = np.array([1.0, 0, 0, 0, 0.3])
    _, info = oracle.collide(prm0, pops_from_moments(Q, flux_adv(Q)))
    assert info["mu"] == 0.02
    assert info["kappa"] == pytest.approx(prm0["kappa_ref"], rel=1e-15)


def test_positivity_floors():
    """Algorithm 1 (primitives) and Table 1: rho and p are floored; conservation of the
    (unfloored) zeroth moment is kept."""
    prm = params(rho_min=1e-4, p_min=1e-7)
    Q = np.array([1e-6, 1e-8, 0.0, 0.0, 1e-12])
    f = pops_from_moments(Q, np.zeros((5, 3)))
    fo, info = oracle.collide(prm, f)
    assert info["rho_f"] == 1e-4
    assert info["p"] == 1e-7
    assert info["T"] == pytest.approx(1e-7 / 1e-4)
    np.testing.assert_allclose(moments(fo)[0], Q, rtol=1e-12, atol=1e-20)
