"""Seeded synthetic inputs shared by the GPU path, its tests and the oracle tests.

This module holds no lattice Boltzmann arithmetic.  It builds, for each workload,
the initial conserved fields Q = (rho, rho u, E) in lattice units and the lattice
parameter set, from the physical set-ups the paper evaluates (Sec. 3: Sod and
Becker shock tubes, compressible Taylor-Green vortex; Table 1 for the numerical
parameters), and it draws the seeded instance mixes of the batched and served
workloads.  Both the HIP path and the FP64 oracle start from what is built here.

Units (the paper leaves the mapping implicit).  With cell size dx and
r = dt/dx (the paper's Courant number, Sec. 2.6), density is unscaled and
    u_lat = r u,  p_lat = r^2 p,  E_lat = r^2 E,  T_lat = r^2 T,
    mu_lat = mu r / dx,  kappa_lat = kappa r / dx,
    E_k(phys) = E_k(lat) / r^2,  eps(phys) = eps(lat) / (r^3 dx).
The conductivity follows Pr = mu c_p / kappa with c_p = gamma/(gamma-1) (Sec. 2.4).

Parameter dict keys (lattice units): nx, ny, nz, bc (per axis, 0 periodic, 1 zero
gradient), collision (0 regularized with sensor, 1 BGK), mu_law (0 constant,
1 Sutherland), gamma, mu_ref, kappa_ref, T_ref, T_S, omega[5], sensor_gain, J_min,
omega_min, rho_min, p_min, rho_ref, E_ref (the uniform reference state whose
equilibrium the stored populations are shifted by, Sec. 2.2), and optionally start
(0 first-order start from the initial gradients, 1 equilibrium start for data with
jumps; the Sod tubes use 1).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

T_SUTHERLAND = 0.4042  # Listing 1
PERIODIC, ZERO_GRADIENT = 0, 1
RLB_SENSOR, BGK = 0, 1
START_FIRST_ORDER, START_EQUILIBRIUM = 0, 1
MU_CONSTANT, MU_SUTHERLAND = 0, 1


@dataclass
class Case:
    name: str
    params: dict
    Q0: np.ndarray            # [5, nz, ny, nx] float64, lattice units
    steps: int
    diag_every: int = 0
    meta: dict = field(default_factory=dict)

    @property
    def shape(self):
        return (self.params["nz"], self.params["ny"], self.params["nx"])

    @property
    def cells(self) -> int:
        return int(self.params["nx"]) * int(self.params["ny"]) * int(self.params["nz"])


def base_params(nx, ny, nz, bc, *, gamma=1.4, mu=0.0, Pr=0.71, mu_law=MU_CONSTANT,
                T_ref=1.0, omega=1.9, collision=RLB_SENSOR, sensor_gain=20.0, J_min=3e-3,
                omega_min=1.0, rho_min=1e-4, p_min=1e-4, rho_ref=1.0, E_ref=0.0) -> dict:
    """Lattice parameter dict; mu and the floors are already in lattice units."""
    cp = gamma / (gamma - 1.0)
    om = [float(omega)] * 5 if np.isscalar(omega) else [float(w) for w in omega]
    return dict(nx=int(nx), ny=int(ny), nz=int(nz), bc=[int(b) for b in bc],
                collision=int(collision), mu_law=int(mu_law), gamma=float(gamma),
                mu_ref=float(mu), kappa_ref=float(mu * cp / Pr) if Pr else 0.0,
                T_ref=float(T_ref), T_S=T_SUTHERLAND, omega=om,
                sensor_gain=float(sensor_gain), J_min=float(J_min),
                omega_min=float(omega_min), rho_min=float(rho_min), p_min=float(p_min),
                rho_ref=float(rho_ref), E_ref=float(E_ref), Pr=float(Pr))


def conserved(rho, u, p, gamma):
    """Primitive -> conserved state of eq. 2 (equation of state only)."""
    rho = np.asarray(rho, dtype=np.float64)
    Q = np.empty((5,) + rho.shape)
    Q[0] = rho
    for d in range(3):
        Q[1 + d] = rho * u[d]
    Q[4] = p / (gamma - 1.0) + 0.5 * rho * (u[0] ** 2 + u[1] ** 2 + u[2] ** 2)
    return Q


# ---------------------------------------------------------- manufactured solution
MMS_CFL = 0.05          # dt/dx, the acoustic time-step factor of the MMS row of Table 1
MMS_OMEGA_FINEST = 1.86  # omega at the finest grid (n = 256) of the dt-tied relaxation
MMS_N_FINEST = 256
MMS_BETA_MAX = 4.0       # largest beta = 2 nu omega / c_s^2 on the finest grid (Sec. 2.4)


def mms_fields(n, t, rho0=1.0, cs=0.5, mach=2.0, gamma=1.4, r=MMS_CFL):
    """Primitive fields of eq. 8 in lattice units on the n^3 lattice (x = i / n, one
    period per n cells) at lattice time t (steps; physical time t r / n).  Returns
    (rho, (u_x, u_y, u_z), p) arrays [nz][ny][nx]."""
    a = 0.30 / math.sqrt(3.0)
    p0 = rho0 * cs * cs * (0.30 / mach) ** 2 / gamma
    k = 2.0 * math.pi / n          # per cell
    w = 2.0 * math.pi * r / n      # per step (unit period)
    i = np.arange(n, dtype=np.float64)
    Z, Y, X = np.meshgrid(i, i, i, indexing="ij")
    U = r * cs                     # lattice velocity scale
    P0 = r * r * p0                # lattice pressure scale
    rho = rho0 * (1.0 + 0.05 * np.sin(k * X) + 0.03 * np.cos(k * Y) + 0.02 * np.cos(k * Z + w * t))
    ux = U * (a + 0.035 * np.cos(k * X + 0.4) + 0.025 * np.sin(k * Y))
    uy = U * (a + 0.035 * np.sin(k * Y + 0.9) + 0.025 * np.cos(k * Z))
    uz = U * (a + 0.025 * np.cos(k * Z + 1.7) + 0.015 * np.sin(k * X + w * t))
    p = P0 * (1.0 + 0.05 * np.cos(k * X + 1.2) + 0.03 * np.sin(k * Y + w * t) + 0.02 * np.sin(k * Z + 0.6))
    return rho, (ux, uy, uz), p


def mms(n=64, rho0=1.0, cs=0.5, mach=2.0, gamma=1.4, Pr=0.71, r=MMS_CFL, t_end=1.0,
        omega_finest=MMS_OMEGA_FINEST, n_finest=MMS_N_FINEST, beta_max=MMS_BETA_MAX,
        mu_phys=None) -> Case:
    """Manufactured solution of Sec. 3.1 (eq. 8) on the unit periodic cube at n^3,
    BGK, refined acoustically (dt/dx = r fixed) to physical time t_end.

    Readings (the paper leaves them open): the fields of eq. 8 are physical with
    c_s = 1/2 and dx = 1/n; the relaxation is tied to the time step as
    1/omega - 1/2 proportional to dt, equal to omega_finest at n_finest; the physical
    viscosity and conductivity are constant, with mu chosen so that beta reaches
    beta_max on the finest grid (at the lowest density, 0.9 rho0) and kappa from Pr.
    meta["mms"] holds the lattice constants the source needs: rho0, U, P0, a, K, W,
    gamma, mu, kappa.  The viscosity follows from the paper-level reading (beta_max at
    omega 1.86 on 256^3) unless mu_phys is given, whatever omega_finest/n_finest."""
    a = 0.30 / math.sqrt(3.0)
    p0 = rho0 * cs * cs * (0.30 / mach) ** 2 / gamma
    steps = int(round(t_end * n / r))
    nu_om = (1.0 / omega_finest - 0.5) * n_finest / n
    omega = 1.0 / (0.5 + nu_om)
    # beta = 8 nu_lat omega; nu_lat = mu_phys r n / rho on the lattice
    if mu_phys is None:
        mu_phys = (beta_max * 0.9 * rho0 /
                   (8.0 * MMS_OMEGA_FINEST * r * MMS_N_FINEST))
    mu_lat = mu_phys * r * n
    rho, u, p = mms_fields(n, 0.0, rho0, cs, mach, gamma, r)
    Q = conserved(rho, u, p, gamma)
    U, P0 = r * cs, r * r * p0
    prm = base_params(n, n, n, (PERIODIC, PERIODIC, PERIODIC), gamma=gamma, mu=mu_lat, Pr=Pr,
                      mu_law=MU_CONSTANT, omega=omega, collision=BGK, p_min=1e-4 * r * r,
                      rho_ref=rho0, E_ref=P0 / (gamma - 1.0) + 1.5 * rho0 * (U * a) ** 2)
    meta = dict(r=r, steps=steps, t_end=t_end, mu_phys=mu_phys, omega=omega,
                mms=dict(rho0=rho0, U=U, P0=P0, a=a, K=2.0 * math.pi / n, W=2.0 * math.pi * r / n,
                         gamma=gamma, mu=mu_lat, kappa=prm["kappa_ref"]),
                field_args=dict(rho0=rho0, cs=cs, mach=mach, gamma=gamma, r=r))
    return Case("mms", prm, Q, steps, 0, meta)


def mms_exact(case: Case, t) -> np.ndarray:
    """Conserved fields of the manufactured solution at lattice time t."""
    rho, u, p = mms_fields(case.params["nx"], t, **case.meta["field_args"])
    return conserved(rho, u, p, case.meta["field_args"]["gamma"])


# --------------------------------------------------------------------------- Sod
# --------------------------------------------------------------- time step (CFL)
# Sec. 2.6 and Table 1 state a Courant number and write it as dt/dx.  Taken
# literally, the Becker ceiling of about 0.7 would move the Mach 2 upstream flow 1.4
# cells per step.  The reading used throughout: the Courant number of the fastest
# characteristic, CFL = lambda_max dt/dx with lambda_max the largest |u| + c of the
# flow (of the exact solution where the case has one, else of the initial state).
# With Table 1's Sod value 0.35 the oracle then lands within 10% of every error of
# Table 3 (N = 750 to 6000), while the literal dt/dx = 0.35 diverges.
# Near omega = 2 this reading puts Table 1's vortex point (0.1) outside the linear
# stability limit of the regularized collision, about 0.41 sqrt(2 - omega) cells per
# step (0.003 at omega = 1.99996), and that run diverges within a few hundred steps;
# the cases run near omega = 2 (vortex, Becker, whose Table 1 entry is only the
# stability map) take 0.05, at which the 256^3 vortex stays finite to t_c = 10.
CFL_SOD = 0.35
CFL_NEAR_TWO = 0.05


def sod(n=256, ny=4, nz=4, r=None, t_end=0.2, steps=None, left=(1.0, 1.0), right=(0.125, 0.1),
        gamma=1.4, Pr=0.71, mu=1e-6, omega=1.40, sensor_gain=20.0, J_min=3e-3,
        omega_min=1.0, cfl=None) -> Case:
    """Sod shock tube on [0,1] (Sec. 3.2): left/right = (rho, p), u = 0, cell
    centres x = (i + 1/2)/n, zero gradient at both x ends, periodic in y and z.
    Unless r = dt/dx is given, r = cfl / lambda_max with lambda_max the fastest
    characteristic speed of the exact Riemann solution (2.19 for Sod) and cfl the
    Table 1 value 0.35 (CFL_SOD), so r = 0.160.  The run ends at t_end unless a step
    count is given (at n = 256, t = 0.2 takes 321 steps)."""
    dx = 1.0 / n
    if r is None:
        smax = riemann_max_speed((left[0], 0.0, left[1]), (right[0], 0.0, right[1]), gamma)
        r = (CFL_SOD if cfl is None else cfl) / smax
    x = (np.arange(n) + 0.5) * dx
    rho1 = np.where(x < 0.5, left[0], right[0])
    p1 = np.where(x < 0.5, left[1], right[1])
    rho = np.broadcast_to(rho1, (nz, ny, n)).copy()
    p = np.broadcast_to(p1, (nz, ny, n)).copy() * r * r
    zero = np.zeros_like(rho)
    Q = conserved(rho, (zero, zero, zero), p, gamma)
    prm = base_params(n, ny, nz, (ZERO_GRADIENT, PERIODIC, PERIODIC), gamma=gamma,
                      mu=mu * r / dx, Pr=Pr, omega=omega, sensor_gain=sensor_gain,
                      J_min=J_min, omega_min=omega_min, p_min=1e-4 * r * r,
                      rho_ref=right[0], E_ref=right[1] * r * r / (gamma - 1.0))
    prm["start"] = START_EQUILIBRIUM  # Riemann data: no gradient across the jump
    if steps is None:
        steps = int(round(t_end / (r * dx)))
    return Case("sod", prm, Q, int(steps), 0,
                dict(dx=dx, r=r, x=x, t_end=steps * r * dx, left=left, right=right, gamma=gamma))


# ------------------------------------------------------------ Taylor-Green vortex
F_MU = {64: 1.8, 128: 0.9, 256: 0.001, 512: 0.01}  # background damping per resolution


def f_mu_for(n: int) -> float:
    """Background damping of the cTGV section; nearest tabulated resolution in log2."""
    keys = sorted(F_MU)
    best = min(keys, key=lambda k: abs(math.log2(k) - math.log2(n)))
    return F_MU[best]


def tgv(n=256, mach=1.25, Re=1600.0, Pr=0.71, gamma=1.4, r=None, f_mu=None,
        sensor_gain=40.0, J_min=1e-2, omega_min=1.987, steps=2000, diag_every=50,
        collision=RLB_SENSOR, dims=None, cfl=CFL_NEAR_TWO, z_extruded=False) -> Case:
    """Compressible Taylor-Green vortex on [0, 2pi)^3 (Sec. 3.3): V0 = rho0 = L0 = 1,
    u = (sin x cos y cos z, -cos x sin y cos z, 0), pressure of the incompressible
    solution p = p0 + (1/16)(cos 2x + cos 2y)(cos 2z + 2) with p0 = c0^2/gamma,
    c0 = 1/M, uniform temperature so rho = p/T0, Sutherland viscosity with
    mu_ref = 1/Re at T_ref = T0.  Nodes x_i = i dx, dx = 2 pi / n.  The relaxation
    time follows the background damping rule tau = 1/2 + 4 f_mu nu dt/dx^2.

    Time step: unless r = dt/dx is given, r = cfl / (V0 + c0), i.e. the fastest
    initial characteristic moves cfl cells per step (CFL_NEAR_TWO: Table 1's 0.1
    diverges under the regularized collision near omega = 2).

    dims = (nx, ny, nz) samples a part of the n^3 field at its own spacing.  With
    z_extruded every z-plane is the plane z = 0, so a thin periodic slab of full
    x-y planes stays smooth across its z wrap (a two-dimensional vortex).  The time
    step, transport and relaxation keep the n^3 recipe either way."""
    nx, ny, nz = dims if dims is not None else (n, n, n)
    dx = 2.0 * math.pi / n
    c0 = 1.0 / mach
    if r is None:
        r = cfl / (1.0 + c0)
    p0 = c0 * c0 / gamma
    T0 = p0
    x = np.arange(nx) * dx
    y = np.arange(ny) * dx
    z = np.zeros(nz) if z_extruded else np.arange(nz) * dx
    Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
    ux = np.sin(X) * np.cos(Y) * np.cos(Z)
    uy = -np.cos(X) * np.sin(Y) * np.cos(Z)
    uz = np.zeros_like(ux)
    p = p0 + (1.0 / 16.0) * (np.cos(2 * X) + np.cos(2 * Y)) * (np.cos(2 * Z) + 2.0)
    rho = p / T0
    Q = conserved(rho, (r * ux, r * uy, r * uz), r * r * p, gamma)
    mu_lat = (1.0 / Re) * r / dx
    if f_mu is None:
        f_mu = f_mu_for(n)
    tau = 0.5 + 4.0 * f_mu * mu_lat  # nu = mu/rho0 with rho0 = 1
    omega = 1.0 / tau
    prm = base_params(nx, ny, nz, (PERIODIC, PERIODIC, PERIODIC), gamma=gamma, mu=mu_lat,
                      Pr=Pr, mu_law=MU_SUTHERLAND, T_ref=r * r * T0, omega=omega,
                      collision=collision, sensor_gain=sensor_gain, J_min=J_min,
                      omega_min=omega_min, p_min=1e-4 * r * r, rho_ref=1.0,
                      E_ref=r * r * p0 / (gamma - 1.0))
    return Case("tgv", prm, Q, steps, diag_every,
                dict(dx=dx, r=r, mach=mach, Re=Re, f_mu=f_mu, tc_per_step=r * dx,
                     ek_scale=1.0 / (r * r), eps_scale=1.0 / (r ** 3 * dx)))


def tgv2d(n=32, u0=0.005, c0=0.05, nu=0.02, Pr=0.71, gamma=1.4, omega=2.0,
          collision=BGK, nz=1) -> Case:
    """Two-dimensional low-Mach Taylor-Green vortex, directly in lattice units:
    u = u0 (sin kx cos ky, -cos kx sin ky, 0), k = 2 pi / n, incompressible pressure
    p = p0 + rho0 u0^2/4 (cos 2kx + cos 2ky), uniform temperature, constant mu."""
    k = 2.0 * math.pi / n
    p0 = c0 * c0 / gamma
    T0 = p0
    i = np.arange(n)
    Z, Y, X = np.meshgrid(np.arange(nz), i, i, indexing="ij")
    ux = u0 * np.sin(k * X) * np.cos(k * Y)
    uy = -u0 * np.cos(k * X) * np.sin(k * Y)
    p = p0 + 0.25 * u0 * u0 * (np.cos(2 * k * X) + np.cos(2 * k * Y))
    rho = p / T0
    Q = conserved(rho, (ux, uy, np.zeros_like(ux)), p, gamma)
    prm = base_params(n, n, nz, (PERIODIC, PERIODIC, PERIODIC), gamma=gamma, mu=nu, Pr=Pr,
                      omega=omega, collision=collision, p_min=1e-12, rho_min=1e-6,
                      rho_ref=1.0, E_ref=p0 / (gamma - 1.0))
    return Case("tgv2d", prm, Q, 0, 0, dict(k=k, u0=u0, c0=c0, nu=nu))


# ------------------------------------------------------------- Becker viscous shock
def becker_states(mach, gamma=1.4, rho1=1.0, c1=1.0):
    """Upstream/downstream states of a normal shock in its own frame."""
    u1 = mach * c1
    p1 = rho1 * c1 * c1 / gamma
    u2 = u1 * ((gamma - 1.0) * mach * mach + 2.0) / ((gamma + 1.0) * mach * mach)
    m = rho1 * u1
    cp = gamma / (gamma - 1.0)
    H = cp * p1 / rho1 + 0.5 * u1 * u1
    return dict(u1=u1, u2=u2, m=m, H=H, p1=p1, rho1=rho1, cp=cp)


def becker_K(mach, mu, gamma=1.4, rho1=1.0, c1=1.0):
    s = becker_states(mach, gamma, rho1, c1)
    return 3.0 * s["m"] * (gamma + 1.0) / (8.0 * gamma * mu)


def becker_thickness(mach, mu, gamma=1.4, rho1=1.0, c1=1.0):
    """Maximum-slope thickness (u1 - u2)/max|u'| of the Becker profile."""
    s = becker_states(mach, gamma, rho1, c1)
    K = becker_K(mach, mu, gamma, rho1, c1)
    a, b = math.sqrt(s["u1"]), math.sqrt(s["u2"])
    return (a + b) / (K * (a - b))


def becker_mu_for_thickness(mach, delta, gamma=1.4, rho1=1.0, c1=1.0):
    s = becker_states(mach, gamma, rho1, c1)
    a, b = math.sqrt(s["u1"]), math.sqrt(s["u2"])
    K = (a + b) / (delta * (a - b))
    return 3.0 * s["m"] * (gamma + 1.0) / (8.0 * gamma * K)


def becker_profile(x, mach, mu, x_shock=0.0, gamma=1.4, rho1=1.0, c1=1.0):
    """Closed-form Becker shock (Pr = 3/4, constant mu, Stokes hypothesis) in its own
    frame.  With Pr = 3/4 the total enthalpy H = c_p T + u^2/2 is constant, and
    momentum reduces to (4/3) mu u u' = m (gamma+1)/(2 gamma) (u - u1)(u - u2),
    whose solution is explicit in x(u):
        x(u) = [u1 ln((u1-u)/(u1-u2)) - u2 ln((u-u2)/(u1-u2))] / (K (u1-u2)) + C,
    K = 3 m (gamma+1)/(8 gamma mu).  C places the steepest point u = sqrt(u1 u2) at
    x_shock.  Inverted by bisection in FP64.  Returns (rho, u, p, T) arrays."""
    s = becker_states(mach, gamma, rho1, c1)
    u1, u2, m, H, cp = s["u1"], s["u2"], s["m"], s["H"], s["cp"]
    K = becker_K(mach, mu, gamma, rho1, c1)
    d = u1 - u2

    def xof(u):
        return (u1 * np.log((u1 - u) / d) - u2 * np.log((u - u2) / d)) / (K * d)

    x0 = xof(math.sqrt(u1 * u2))
    xs = np.asarray(x, dtype=np.float64) - x_shock + x0
    lo = np.full(xs.shape, u2)   # x(u) decreases with u: x(lo) = +inf
    hi = np.full(xs.shape, u1)   # x(hi) = -inf
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        with np.errstate(divide="ignore", invalid="ignore"):
            xm = xof(mid)
        go_up = xm > xs          # need larger u to reduce x
        lo = np.where(go_up, mid, lo)
        hi = np.where(go_up, hi, mid)
    u = 0.5 * (lo + hi)
    rho = m / u
    T = (H - 0.5 * u * u) / cp
    p = rho * T
    return rho, u, p, T


def becker(L=1024, mach=2.0, cells_per_front=16.0, ny=4, nz=4, gamma=1.4, omega=1.99,
           beta_max=4.0, sensor_gain=20.0, J_min=3e-3, omega_min=1.0, cfl=CFL_NEAR_TWO) -> Case:
    """Stationary Becker shock in lattice units, shock frame, centred in an L-cell tube
    with zero-gradient ends (Sec. 3.2 configuration, Pr = 3/4, constant mu).
    The upstream sound speed is set so that |u1| + c1 = cfl (the fastest
    characteristic moves cfl cells per step); mu is chosen for the
    requested maximum-slope thickness, capped so that the lattice viscous number
    beta = 2 nu omega / c_s^2 upstream stays <= beta_max (eq. 6)."""
    c1 = cfl / (mach + 1.0)
    mu = becker_mu_for_thickness(mach, cells_per_front, gamma, 1.0, c1)
    beta = 8.0 * mu * omega
    if beta > beta_max:
        mu = beta_max / (8.0 * omega)
    delta = becker_thickness(mach, mu, gamma, 1.0, c1)
    x = np.arange(L) + 0.5
    xs = 0.5 * L
    rho1d, u1d, p1d, _ = becker_profile(x, mach, mu, xs, gamma, 1.0, c1)
    rho = np.broadcast_to(rho1d, (nz, ny, L)).copy()
    ux = np.broadcast_to(u1d, (nz, ny, L)).copy()
    p = np.broadcast_to(p1d, (nz, ny, L)).copy()
    zero = np.zeros_like(rho)
    Q = conserved(rho, (ux, zero, zero), p, gamma)
    s = becker_states(mach, gamma, 1.0, c1)
    prm = base_params(L, ny, nz, (ZERO_GRADIENT, PERIODIC, PERIODIC), gamma=gamma, mu=mu,
                      Pr=0.75, omega=omega, sensor_gain=sensor_gain, J_min=J_min,
                      omega_min=omega_min, p_min=1e-4 * c1 * c1, rho_ref=1.0,
                      E_ref=s["p1"] / (gamma - 1.0) + 0.5 * s["u1"] ** 2)
    return Case("becker", prm, Q, 5000, 0,
                dict(mach=mach, mu=mu, c1=c1, x_shock=xs, cells_per_front=delta,
                     gamma=gamma, x=x))


def becker_batch(count=64, seed=0, L_range=(512, 8192), mach_range=(1.5, 5.0), **kw):
    """Seeded mix of Becker instances: tube lengths uniform on L_range (integers),
    upstream Mach uniform on mach_range."""
    rng = np.random.default_rng(seed)
    Ls = rng.integers(L_range[0], L_range[1] + 1, size=count)
    Ms = rng.uniform(mach_range[0], mach_range[1], size=count)
    return [becker(int(L), float(M), **kw) for L, M in zip(Ls, Ms)]


# ------------------------------------------------------------- random smooth states
def random_smooth(nx, ny, nz, seed=0, amp=0.05, bc=(PERIODIC, PERIODIC, PERIODIC),
                  c0=0.08, mach=1.0, collision=RLB_SENSOR, mu=2e-3, omega=1.95,
                  mu_law=MU_SUTHERLAND, sensor_gain=40.0, J_min=1e-2, omega_min=1.987,
                  modes=3) -> Case:
    """Smooth random state for parity tests: a few random Fourier modes on top of a
    uniform state with sound speed c0 and velocity amplitude mach*c0 (lattice)."""
    rng = np.random.default_rng(seed)
    gamma = 1.4
    Z, Y, X = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")

    def field_():
        out = np.zeros((nz, ny, nx))
        for _ in range(modes):
            k = rng.integers(0, 3, size=3)
            ph = rng.uniform(0, 2 * math.pi)
            a = rng.standard_normal()
            out += a * np.cos(2 * math.pi * (k[0] * X / nx + k[1] * Y / ny + k[2] * Z / nz) + ph)
        return out / modes

    p0 = c0 * c0 / gamma
    rho = 1.0 + amp * field_()
    p = p0 * (1.0 + amp * field_())
    u = [mach * c0 * field_() for _ in range(3)]
    Q = conserved(rho, u, p, gamma)
    prm = base_params(nx, ny, nz, bc, gamma=gamma, mu=mu, mu_law=mu_law, T_ref=p0,
                      omega=omega, collision=collision, sensor_gain=sensor_gain, J_min=J_min,
                      omega_min=omega_min, p_min=1e-4 * p0, rho_ref=1.0,
                      E_ref=p0 / (gamma - 1.0))
    return Case("random", prm, Q, 0, 0, dict(seed=seed))


# ------------------------------------------------------------------ served requests
def riemann_max_speed(left, right, gamma=1.4):
    """Fastest signal speed of a Riemann problem from left/right = (rho, u, p): star
    pressure by Newton iteration on the wave-jump function (shock branch from
    Rankine-Hugoniot, rarefaction branch isentropic), then the largest of the outer
    wave speeds and |u*| + c* on either side.  Used only to choose the time step."""
    def jump(p, rho, pk):
        c = math.sqrt(gamma * pk / rho)
        if p > pk:
            A = 2.0 / ((gamma + 1.0) * rho)
            B = (gamma - 1.0) / (gamma + 1.0) * pk
            return (p - pk) * math.sqrt(A / (p + B)), math.sqrt(A / (B + p)) * (1 - (p - pk) / (2 * (B + p)))
        e = (gamma - 1.0) / (2.0 * gamma)
        return (2 * c / (gamma - 1.0) * ((p / pk) ** e - 1.0),
                (p / pk) ** (-(gamma + 1.0) / (2 * gamma)) / (rho * c))
    rl, ul, pl = left
    rr, ur, pr = right
    p = 0.5 * (pl + pr)
    for _ in range(60):
        fl, dl = jump(p, rl, pl)
        fr, dr = jump(p, rr, pr)
        p = max(p - (fl + fr + ur - ul) / (dl + dr), 1e-12 * (pl + pr))
    fl, _ = jump(p, rl, pl)
    fr, _ = jump(p, rr, pr)
    us = 0.5 * (ul + ur) + 0.5 * (fr - fl)
    speeds = []
    for rho, u, pk, sgn in ((rl, ul, pl, -1.0), (rr, ur, pr, 1.0)):
        c = math.sqrt(gamma * pk / rho)
        if p > pk:
            speeds.append(abs(u + sgn * c * math.sqrt((gamma + 1) / (2 * gamma) * p / pk + (gamma - 1) / (2 * gamma))))
            rs = rho * ((p / pk + (gamma - 1) / (gamma + 1)) / ((gamma - 1) / (gamma + 1) * p / pk + 1))
        else:
            speeds.append(abs(u) + c)
            rs = rho * (p / pk) ** (1.0 / gamma)
        speeds.append(abs(us) + math.sqrt(gamma * p / rs))
    return max(speeds)


def sod_variant(n, rho_ratio, p_ratio, ny=4, nz=4, cfl=CFL_SOD, **kw):
    """Sod-type tube with left/right density and pressure ratios (right state 0.125,
    0.1 scaled by the ratios); r = dt/dx from the Courant number of the fastest
    wave of its exact solution."""
    left = (0.125 * rho_ratio, 0.1 * p_ratio)
    right = (0.125, 0.1)
    return sod(n=n, ny=ny, nz=nz, left=left, right=right, cfl=cfl, **kw)


@dataclass
class Request:
    rid: int
    arrival: float     # seconds after the trace starts
    kind: str
    case: Case
    steps: int
    storage: int       # 0 FP32, 1 FP16


def serving_trace(count=1000, rate=50.0, seed=1, steps_range=(1000, 20000), mix=(0.4, 0.4, 0.2),
                  sod_n=(256, 4096), tgv_n=(32, 128), tgv_mach=(0.5, 1.5), becker_mach=(1.5, 5.0),
                  becker_L=(512, 8192), fp16_share=0.5, tgv_tc_max=20.0):
    """Seeded Poisson request stream: 40% Sod variants (n x 4 x 4, left/right density
    and pressure ratios log-uniform on [1, 100]), 40% Taylor-Green vortices (n^3,
    Mach uniform, time step such that the request ends by t_c = tgv_tc_max), 20%
    Becker shocks (Mach uniform); steps uniform; FP32 or FP16 storage per request."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for rid in range(count):
        t += rng.exponential(1.0 / rate)
        u = rng.uniform()
        steps = int(rng.integers(steps_range[0], steps_range[1] + 1))
        storage = 1 if rng.uniform() < fp16_share else 0
        if u < mix[0]:
            n = int(rng.integers(sod_n[0], sod_n[1] + 1))
            rr = float(np.exp(rng.uniform(0, math.log(100))))
            pr = float(np.exp(rng.uniform(0, math.log(100))))
            case, kind = sod_variant(n, rr, pr), "sod"
        elif u < mix[0] + mix[1]:
            n = int(rng.integers(tgv_n[0], tgv_n[1] + 1))
            m = float(rng.uniform(*tgv_mach))
            # the requested steps cover at most t_c = 20 (the horizon of Sec. 3.3)
            r = min(CFL_NEAR_TWO / (1.0 + 1.0 / m), tgv_tc_max / (steps * 2.0 * math.pi / n))
            case, kind = tgv(n=n, mach=m, steps=steps, diag_every=0, r=r), "tgv"
        else:
            L = int(rng.integers(becker_L[0], becker_L[1] + 1))
            m = float(rng.uniform(*becker_mach))
            case, kind = becker(L=L, mach=m), "becker"
        out.append(Request(rid, t, kind, case, steps, storage))
    return out
