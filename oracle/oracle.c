/*
 * oracle.c -- plain FP64 CPU reference of the five-field gradient-reconstruction
 * lattice Boltzmann update (Kummerlaender, Bukreev, Krause, "A Gradient-Reconstruction
 * Lattice Boltzmann Method for Compressible Navier-Stokes-Fourier Equations").
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the oracle that the GPU path is checked
 * against.  Only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark may load it.  It shares no code, header, table or helper with the HIP
 * library and must never be linked into it.
 *
 * What it computes, step for step in the paper's order (Algorithm 1, Sec. 2.2-2.5):
 *   1. conserved moments Q_k = sum_i f_ki and first moments J_k = sum_i c_i f_ki
 *   2. primitives with positivity floors on rho and p, T = p/rho
 *   3. Sutherland (or constant) viscosity, conductivity kappa(T) = kappa_ref mu(T)/mu_ref
 *   4. advective flux Phi_adv = Phi at grad Q = 0 (eq. 2), non-equilibrium first
 *      moment Pi = J - Phi_adv and the direct gradient  gradQ~ = -Pi/(cs^2 tau) (eq. 3)
 *   5. gradQ = R gradQ~ with R = (I - cs^-2 diag(omega) M)^-1 (eq. 4).  Here M is the
 *      15x15 diffusive-flux Jacobian of eq. 5, assembled densely, and the linear
 *      system is solved by Gaussian elimination with partial pivoting -- the plain
 *      definition of R, not the closed-form block solve of eqs. 6-7.
 *   6. chain rule to grad u and grad T (Sec. 2.4)
 *   7. compression sensor chi (Sec. 2.5, Listing 2)
 *   8. Newtonian stress and Fourier flux (eq. 2), full flux Phi in the equilibrium
 *   9. regularized collision with reduced rate omega_h, or BGK (Sec. 2.2, 2.5)
 *  10. exact on-lattice push streaming into a second buffer
 * Initial state (ora_init): populations with the first-order non-equilibrium first
 * moment of the initial fields' central-difference gradients (see ora_init).
 * With a source S of eq. 1 (ora_step_src) the post-collision populations gain
 * w_i S_k before streaming (the collision of Algorithm 1).  ora_mms_source writes the
 * source of the manufactured solution of Sec. 3.1 (eq. 8), derived by hand from
 * eq. 2 with constant mu and kappa.
 *
 * Lattice: D3Q7 with c_s^2 = 1/4 (Sec. 2.2).  The paper gives only c_s^2; the weights
 * w_0 = 1/4, w_1..6 = 1/8 are the unique nearest-neighbour isotropic set with that
 * speed of sound (reading listed in the design notes).
 *
 * Storage: unshifted populations f[35][N] in FP64, slot = 7*field + direction, field
 * order (rho, rho u_x, rho u_y, rho u_z, E), direction order
 * (0, +x, -x, +y, -y, +z, -z), cell index x + nx*(y + ny*z).
 *
 * Boundaries (the paper states none): periodic wrap, or zero gradient where the
 * ghost cell beyond a face holds a copy of the adjacent cell's post-collision
 * populations.
 *
 * Pins: tests/test_oracle_*.py check this file against closed forms, invariants and
 * exact solutions (lattice moment identities, finite-difference Jacobian of the
 * diffusive flux, exact recovery of prescribed gradients, conservation, exact Sod
 * Riemann solution, Becker closed form, viscous decay of a Taylor-Green vortex,
 * second-order convergence to the manufactured solution of eq. 8, whose source is
 * checked against a symbolic differentiation of eq. 2).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORA_Q 7
#define ORA_NF 5
#define ORA_NPOP 35

static const int ORA_C[ORA_Q][3] = {
    {0, 0, 0}, {1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}, {0, 0, 1}, {0, 0, -1}};
static const double ORA_W[ORA_Q] = {0.25, 0.125, 0.125, 0.125, 0.125, 0.125, 0.125};
static const double ORA_CS2 = 0.25;

typedef struct {
  int32_t nx, ny, nz;
  int32_t bc[3];       /* 0 = periodic, 1 = zero gradient                         */
  int32_t collision;   /* 0 = regularized with compression sensor, 1 = BGK        */
  int32_t mu_law;      /* 0 = constant mu, 1 = Sutherland                         */
  int32_t start;       /* 0 = first-order start, 1 = equilibrium start (ora_init)  */
  double gamma;
  double mu_ref, kappa_ref, T_ref, T_S;
  double omega[ORA_NF];
  double sensor_gain, J_min, omega_min;
  double rho_min, p_min;
} ora_params;

/* Every intermediate of one cell update, exposed so that tests can check each step. */
typedef struct {
  double Q[ORA_NF], J[ORA_NF][3];
  double rho_f, u[3], k2, p, T, mu, kappa, nu;
  double Phi_adv[ORA_NF][3], Pi[ORA_NF][3], gradQ_tilde[ORA_NF][3];
  double M[15][15];          /* diffusive-flux Jacobian, row (k,c), column (l,d)     */
  double gradQ[ORA_NF][3];   /* reconstructed conserved gradients, [field][d]         */
  double grad_u[3][3];       /* grad_u[j][c] = d u_j / d x_c                          */
  double grad_T[3];
  double theta, s, chi;
  double omega_h[ORA_NF];
  double tau[3][3], q[3];
  double Phi[ORA_NF][3];
  double ek, eps_s, eps_d;
  int32_t nonfinite;
} ora_cell_info;

/* ---------------------------------------------------------------- viscosity law */
/* Temperature factor mu(T)/mu_ref of the Sutherland law of Listing 1 (T_S = 0.4042),
 * equal to 1 at T_ref; 1 for the constant law.  Listing 1 scales the conductivity by
 * the same factor, so it stays defined for an inviscid set-up (mu_ref = 0). */
static double ora_mu_ratio(const ora_params* P, double T) {
  if (P->mu_law == 0) return 1.0;
  double t = T / P->T_ref;
  return (1.0 + P->T_S) * pow(t, 1.5) / (t + P->T_S);
}

/* ------------------------------------------------ dense diffusive-flux Jacobian */
/* M = d Phi_diff / d(grad Q) of eq. 5, acting on the column
 * (grad rho, grad(rho u), grad E).  Index (k, c) -> 3k + c for field k and spatial
 * component c; a column (l, d) is the derivative along x_d of field l.
 *   momentum row:  Phi_diff_{m_j, c} = -tau_jc
 *   energy row:    Phi_diff_{E, c}   = -(tau u)_c + q_c
 * with S(X) = X + X^T - 2/3 tr(X) I the symmetric-deviatoric map and
 * (grad a)_{jc} = d_c a_j.  All of rho, mu, kappa are the cell's floored values. */
static void ora_assemble_M(const ora_params* P, double rho, const double u[3], double T,
                           double mu, double kappa, double M[15][15]) {
  const double g1 = P->gamma - 1.0;
  const double nu = mu / rho;
  const double k2 = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
  memset(M, 0, sizeof(double) * 225);
  for (int j = 0; j < 3; ++j) {
    for (int c = 0; c < 3; ++c) {
      const int row = 3 * (1 + j) + c;
      for (int d = 0; d < 3; ++d) {
        /* (mu/rho) S(u (x) grad rho)_jc, derivative with respect to d_d rho */
        double v = (u[j] * (c == d) + u[c] * (j == d) - (2.0 / 3.0) * (j == c) * u[d]);
        M[row][d] += nu * v;
        /* -(mu/rho) S(grad m)_jc, derivative with respect to d_d m_l */
        for (int l = 0; l < 3; ++l) {
          double s = (j == l) * (c == d) + (c == l) * (j == d) - (2.0 / 3.0) * (j == c) * (l == d);
          M[row][3 * (1 + l) + d] += -nu * s;
        }
      }
    }
  }
  for (int c = 0; c < 3; ++c) {
    const int row = 12 + c;
    for (int d = 0; d < 3; ++d) {
      /* (mu/rho)(|u|^2 I + 1/3 u u) + (kappa/rho)(T - (gamma-1)/2 |u|^2) I on grad rho */
      M[row][d] += nu * (k2 * (c == d) + u[c] * u[d] / 3.0) +
                   (kappa / rho) * (T - 0.5 * g1 * k2) * (c == d);
      for (int l = 0; l < 3; ++l) {
        /* -(mu/rho) (S(grad m) u)_c + ((gamma-1) kappa/rho) ((grad m)^T u)_c */
        double Su = (c == l) * u[d] + u[l] * (c == d) - (2.0 / 3.0) * u[c] * (l == d);
        double Tu = (c == d) * u[l];
        M[row][3 * (1 + l) + d] += -nu * Su + (g1 * kappa / rho) * Tu;
      }
      /* -((gamma-1) kappa/rho) I on grad E */
      M[row][12 + d] += -(g1 * kappa / rho) * (c == d);
    }
  }
}

/* Gaussian elimination with partial pivoting: solve A x = b (n <= 15), A and b
 * are overwritten.  Returns 0 on success, -1 on a zero pivot. */
static int ora_solve(int n, double A[15][15], double b[15], double x[15]) {
  for (int col = 0; col < n; ++col) {
    int piv = col;
    for (int r = col + 1; r < n; ++r)
      if (fabs(A[r][col]) > fabs(A[piv][col])) piv = r;
    if (A[piv][col] == 0.0) return -1;
    if (piv != col) {
      for (int cc = 0; cc < n; ++cc) {
        double t = A[col][cc];
        A[col][cc] = A[piv][cc];
        A[piv][cc] = t;
      }
      double t = b[col];
      b[col] = b[piv];
      b[piv] = t;
    }
    for (int r = col + 1; r < n; ++r) {
      double f = A[r][col] / A[col][col];
      if (f == 0.0) continue;
      for (int cc = col; cc < n; ++cc) A[r][cc] -= f * A[col][cc];
      b[r] -= f * b[col];
    }
  }
  for (int r = n - 1; r >= 0; --r) {
    double s = b[r];
    for (int cc = r + 1; cc < n; ++cc) s -= A[r][cc] * x[cc];
    x[r] = s / A[r][r];
  }
  return 0;
}

/* ------------------------------------------------------- primitives and fluxes */
/* Algorithm 1, primitives: rho and p floored; u = rho u / rho_floored, T = p/rho. */
static void ora_primitives(const ora_params* P, const double Q[5], double* rho_f, double u[3],
                           double* k2, double* p, double* T) {
  double r = Q[0] > P->rho_min ? Q[0] : P->rho_min;
  for (int d = 0; d < 3; ++d) u[d] = Q[1 + d] / r;
  double kk = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
  double pp = (P->gamma - 1.0) * (Q[4] - 0.5 * r * kk);
  if (!(pp > P->p_min)) pp = (pp != pp) ? pp : P->p_min; /* keep NaN visible */
  *rho_f = r;
  *k2 = kk;
  *p = pp;
  *T = pp / r;
}

/* Advective flux = flux of eq. 2 with the diffusive parts (tau, q) set to zero. */
static void ora_flux_adv(const double Q[5], const double u[3], double p, double F[5][3]) {
  for (int c = 0; c < 3; ++c) {
    F[0][c] = Q[1 + c];
    for (int j = 0; j < 3; ++j) F[1 + j][c] = Q[1 + j] * u[c] + (j == c ? p : 0.0);
    F[4][c] = (Q[4] + p) * u[c];
  }
}

/* Linear equilibrium (Sec. 2.2): f_eq_i = w_i (Q + c_i . Phi / c_s^2). */
static double ora_feq(int i, double Q, const double Phi[3]) {
  double cf = ORA_C[i][0] * Phi[0] + ORA_C[i][1] * Phi[1] + ORA_C[i][2] * Phi[2];
  return ORA_W[i] * (Q + cf / ORA_CS2);
}

/* ------------------------------------------------------------- one cell update */
/* Algorithm 1 for one cell: f_in[35] (post-stream, pre-collision) ->
 * f_out[35] (post-collision).  info may be NULL. */
void ora_collide(const ora_params* P, const double* f_in, double* f_out, ora_cell_info* info) {
  ora_cell_info L;
  ora_cell_info* I = info ? info : &L;
  memset(I, 0, sizeof(*I));
  const double g1 = P->gamma - 1.0;

  /* conserved moments and first moments */
  for (int k = 0; k < 5; ++k) {
    double q = 0.0, j0 = 0.0, j1 = 0.0, j2 = 0.0;
    for (int i = 0; i < 7; ++i) {
      double f = f_in[7 * k + i];
      q += f;
      j0 += ORA_C[i][0] * f;
      j1 += ORA_C[i][1] * f;
      j2 += ORA_C[i][2] * f;
    }
    I->Q[k] = q;
    I->J[k][0] = j0;
    I->J[k][1] = j1;
    I->J[k][2] = j2;
  }
  /* primitives with positivity floors */
  ora_primitives(P, I->Q, &I->rho_f, I->u, &I->k2, &I->p, &I->T);
  const double rho = I->rho_f;
  const double ratio = ora_mu_ratio(P, I->T);
  I->mu = P->mu_ref * ratio;
  I->kappa = P->kappa_ref * ratio;
  I->nu = I->mu / rho;

  /* non-equilibrium first moment against the advective flux (eq. 3) */
  ora_flux_adv(I->Q, I->u, I->p, I->Phi_adv);
  for (int k = 0; k < 5; ++k)
    for (int c = 0; c < 3; ++c) {
      I->Pi[k][c] = I->J[k][c] - I->Phi_adv[k][c];
      I->gradQ_tilde[k][c] = -I->Pi[k][c] * P->omega[k] / ORA_CS2; /* 1/tau = omega */
    }

  /* reconstruction: grad Q = R grad Q~ with R = (I - cs^-2 diag(omega) M)^-1 (eq. 4) */
  ora_assemble_M(P, rho, I->u, I->T, I->mu, I->kappa, I->M);
  {
    double A[15][15], b[15], x[15];
    for (int r = 0; r < 15; ++r) {
      const int k = r / 3;
      for (int cc = 0; cc < 15; ++cc)
        A[r][cc] = (r == cc ? 1.0 : 0.0) - P->omega[k] / ORA_CS2 * I->M[r][cc];
      b[r] = I->gradQ_tilde[k][r % 3];
    }
    if (ora_solve(15, A, b, x) != 0) {
      for (int r = 0; r < 15; ++r) x[r] = NAN;
    }
    for (int r = 0; r < 15; ++r) I->gradQ[r / 3][r % 3] = x[r];
  }
  /* chain rule: grad u = (grad(rho u) - u (x) grad rho)/rho */
  for (int j = 0; j < 3; ++j)
    for (int c = 0; c < 3; ++c)
      I->grad_u[j][c] = (I->gradQ[1 + j][c] - I->u[j] * I->gradQ[0][c]) / rho;
  /* grad T = (g-1)/rho (grad E - sum_j u_j grad(rho u_j)) + 1/rho ((g-1)/2 |u|^2 - T) grad rho */
  for (int c = 0; c < 3; ++c) {
    double um = 0.0;
    for (int j = 0; j < 3; ++j) um += I->u[j] * I->gradQ[1 + j][c];
    I->grad_T[c] = g1 / rho * (I->gradQ[4][c] - um) +
                   (0.5 * g1 * I->k2 - I->T) / rho * I->gradQ[0][c];
  }

  /* compression sensor (Sec. 2.5), s = -div(u)/c_s */
  I->theta = I->grad_u[0][0] + I->grad_u[1][1] + I->grad_u[2][2];
  I->s = -I->theta / sqrt(ORA_CS2);
  if (I->theta < 0.0 && I->s > P->J_min) {
    double v = P->sensor_gain * I->s;
    I->chi = v < 0.0 ? 0.0 : (v > 1.0 ? 1.0 : v);
  } else {
    I->chi = 0.0;
  }

  /* closures: Newtonian stress and Fourier flux */
  for (int j = 0; j < 3; ++j)
    for (int c = 0; c < 3; ++c)
      I->tau[j][c] = I->mu * (I->grad_u[j][c] + I->grad_u[c][j] - (j == c ? 2.0 / 3.0 * I->theta : 0.0));
  for (int c = 0; c < 3; ++c) I->q[c] = -I->kappa * I->grad_T[c];

  /* the closures enter the flux moment of the equilibrium (eq. 2) */
  for (int c = 0; c < 3; ++c) {
    I->Phi[0][c] = I->Q[1 + c];
    for (int j = 0; j < 3; ++j)
      I->Phi[1 + j][c] = I->Q[1 + j] * I->u[c] + (j == c ? I->p : 0.0) - I->tau[j][c];
    double tu = I->tau[c][0] * I->u[0] + I->tau[c][1] * I->u[1] + I->tau[c][2] * I->u[2];
    I->Phi[4][c] = (I->Q[4] + I->p) * I->u[c] - tu + I->q[c];
  }

  /* collision */
  for (int k = 0; k < 5; ++k) {
    const double om = P->omega[k];
    if (P->collision == 1) {
      /* BGK: f <- f + omega (f_eq - f) */
      I->omega_h[k] = om;
      for (int i = 0; i < 7; ++i) {
        double fe = ora_feq(i, I->Q[k], I->Phi[k]);
        f_out[7 * k + i] = f_in[7 * k + i] + om * (fe - f_in[7 * k + i]);
      }
    } else {
      /* regularized: keep only the first-moment part r of f - f_eq, relaxed at the
       * reduced rate omega_h = omega - chi (omega - omega_min) */
      const double oh = om - I->chi * (om - P->omega_min);
      I->omega_h[k] = oh;
      double dJ[3];
      for (int c = 0; c < 3; ++c) dJ[c] = I->J[k][c] - I->Phi[k][c];
      for (int i = 0; i < 7; ++i) {
        double fe = ora_feq(i, I->Q[k], I->Phi[k]);
        double cdj = ORA_C[i][0] * dJ[0] + ORA_C[i][1] * dJ[1] + ORA_C[i][2] * dJ[2];
        double r = ORA_W[i] * cdj / ORA_CS2;
        f_out[7 * k + i] = fe + (1.0 - oh) * r;
      }
    }
  }

  /* per-cell diagnostic densities: kinetic energy, solenoidal and dilatational
   * dissipation from the reconstructed velocity gradient */
  {
    double wx = I->grad_u[2][1] - I->grad_u[1][2];
    double wy = I->grad_u[0][2] - I->grad_u[2][0];
    double wz = I->grad_u[1][0] - I->grad_u[0][1];
    I->ek = 0.5 * rho * I->k2;
    I->eps_s = I->mu * (wx * wx + wy * wy + wz * wz);
    I->eps_d = (4.0 / 3.0) * I->mu * I->theta * I->theta;
  }
  I->nonfinite = 0;
  for (int s = 0; s < 35; ++s)
    if (!isfinite(f_out[s])) I->nonfinite = 1;
}

/* ------------------------------------------------------------------- lattice */
static int64_t ora_cells(const ora_params* P) { return (int64_t)P->nx * P->ny * P->nz; }

/* Neighbour coordinate along one axis; returns -1 when it lies outside a
 * zero-gradient axis. */
static int ora_shift(int x, int dx, int n, int bc) {
  int y = x + dx;
  if (y >= 0 && y < n) return y;
  if (bc == 0) return (y % n + n) % n;
  return -1;
}

/* coordinate of the neighbour along an axis for a central difference: periodic
 * wrap, or the cell itself beyond a zero-gradient face (the ghost copy) */
static int ora_fd_nb(int x, int d, int n, int bc) {
  int y = x + d;
  if (y >= 0 && y < n) return y;
  if (bc == 0) return (y % n + n) % n;
  return x;
}

/* Initial populations (the paper states no initialisation): the populations whose
 * first moment is the one the update holds a smooth field at to first order,
 *   J_k = Phi_k - (c_s^2 / omega_k) grad Q_k,   Phi = Phi_adv + M grad Q
 * (the non-equilibrium first moment of a collide-and-stream cycle: with
 * J* = Phi + (1 - omega)(J - Phi) and streaming J = J* - c_s^2 grad Q), with grad Q
 * from central differences of the initial fields (periodic wrap, or the cell itself
 * as the ghost beyond a zero-gradient face) and the second moment at equilibrium:
 * f_i = w_i (Q + c_i . J / c_s^2).  The reconstruction of eq. 4 then returns that
 * grad Q at step 0, and no odd-even start-up oscillation of the non-equilibrium is
 * excited (at omega -> 2 it would not decay).  A uniform state gets f = f_eq.
 * With P->start = 1 (initial data with jumps, where a difference across the jump is
 * no gradient: a Riemann problem) the start is the equilibrium of Q with the
 * advective flux.  Q[5][N] -> f[35][N]. */
void ora_init(const ora_params* P, const double* Q, double* f) {
  const int nx = P->nx, ny = P->ny, nz = P->nz;
  const int64_t N = ora_cells(P);
  for (int z = 0; z < nz; ++z)
    for (int y = 0; y < ny; ++y)
      for (int x = 0; x < nx; ++x) {
        const int64_t n = x + (int64_t)nx * (y + (int64_t)ny * z);
        double q[5], u[3], rf, k2, p, T, F[5][3], G[5][3], M[15][15], J[5][3];
        for (int k = 0; k < 5; ++k) q[k] = Q[k * N + n];
        ora_primitives(P, q, &rf, u, &k2, &p, &T);
        ora_flux_adv(q, u, p, F);
        /* central differences of the initial fields */
        const int64_t xm = ora_fd_nb(x, -1, nx, P->bc[0]) + (int64_t)nx * (y + (int64_t)ny * z);
        const int64_t xp = ora_fd_nb(x, 1, nx, P->bc[0]) + (int64_t)nx * (y + (int64_t)ny * z);
        const int64_t ym = x + (int64_t)nx * (ora_fd_nb(y, -1, ny, P->bc[1]) + (int64_t)ny * z);
        const int64_t yp = x + (int64_t)nx * (ora_fd_nb(y, 1, ny, P->bc[1]) + (int64_t)ny * z);
        const int64_t zm = x + (int64_t)nx * (y + (int64_t)ny * ora_fd_nb(z, -1, nz, P->bc[2]));
        const int64_t zp = x + (int64_t)nx * (y + (int64_t)ny * ora_fd_nb(z, 1, nz, P->bc[2]));
        for (int k = 0; k < 5; ++k) {
          G[k][0] = 0.5 * (Q[k * N + xp] - Q[k * N + xm]);
          G[k][1] = 0.5 * (Q[k * N + yp] - Q[k * N + ym]);
          G[k][2] = 0.5 * (Q[k * N + zp] - Q[k * N + zm]);
          if (P->start == 1) G[k][0] = G[k][1] = G[k][2] = 0.0;
        }
        const double ratio = ora_mu_ratio(P, T);
        ora_assemble_M(P, rf, u, T, P->mu_ref * ratio, P->kappa_ref * ratio, M);
        for (int r = 0; r < 15; ++r) {
          double d = 0.0;
          for (int cc = 0; cc < 15; ++cc) d += M[r][cc] * G[cc / 3][cc % 3];
          const int k = r / 3, c = r % 3;
          J[k][c] = F[k][c] + d - ORA_CS2 / P->omega[k] * G[k][c];
        }
        for (int k = 0; k < 5; ++k)
          for (int i = 0; i < 7; ++i) f[(7 * k + i) * N + n] = ora_feq(i, q[k], J[k]);
      }
}

/* Zeroth moments of every field: f[35][N] -> Q[5][N]. */
void ora_moments(const ora_params* P, const double* f, double* Q) {
  const int64_t N = ora_cells(P);
  for (int64_t n = 0; n < N; ++n)
    for (int k = 0; k < 5; ++k) {
      double s = 0.0;
      for (int i = 0; i < 7; ++i) s += f[(7 * k + i) * N + n];
      Q[k * N + n] = s;
    }
}

/* One collide-and-stream step with a source, as ora_step below; S (may be NULL) is
 * the source of eq. 1 for this step in lattice units, S[5][N], projected onto the
 * lattice weights and added to the post-collision populations (Algorithm 1, last
 * line): f*_ki += w_i S_k. */
void ora_step_src(const ora_params* P, const double* f_in, double* f_out, double* diag, const double* S);

/* One collide-and-stream step, two buffers, push streaming:
 *   f_out(x + c_i, i) <- f*(x, i)
 * On a zero-gradient axis the population leaving the domain is dropped and the one
 * entering from the ghost is the cell's own post-collision value.
 * diag (may be NULL) receives 9 sums over all cells of the pre-collision state:
 * kinetic energy, solenoidal and dilatational dissipation densities, the five
 * conserved totals, and the count of cells with non-finite output. */
void ora_step(const ora_params* P, const double* f_in, double* f_out, double* diag) {
  ora_step_src(P, f_in, f_out, diag, NULL);
}

void ora_step_src(const ora_params* P, const double* f_in, double* f_out, double* diag, const double* S) {
  const int nx = P->nx, ny = P->ny, nz = P->nz;
  const int64_t N = ora_cells(P);
  double ek = 0, es = 0, ed = 0, tot[5] = {0, 0, 0, 0, 0}, nonf = 0;
#pragma omp parallel for collapse(2) schedule(static) reduction(+ : ek, es, ed, nonf) reduction(+ : tot[:5])
  for (int z = 0; z < nz; ++z) {
    for (int y = 0; y < ny; ++y) {
      for (int x = 0; x < nx; ++x) {
        const int64_t n = x + (int64_t)nx * (y + (int64_t)ny * z);
        double fi[35], fo[35];
        ora_cell_info info;
        for (int s = 0; s < 35; ++s) fi[s] = f_in[s * N + n];
        ora_collide(P, fi, fo, &info);
        if (S) {
          for (int k = 0; k < 5; ++k)
            for (int i = 0; i < 7; ++i) fo[7 * k + i] += ORA_W[i] * S[k * N + n];
        }
        ek += info.ek;
        es += info.eps_s;
        ed += info.eps_d;
        for (int k = 0; k < 5; ++k) tot[k] += info.Q[k];
        nonf += info.nonfinite;
        for (int i = 0; i < 7; ++i) {
          const int xd = ora_shift(x, ORA_C[i][0], nx, P->bc[0]);
          const int yd = ora_shift(y, ORA_C[i][1], ny, P->bc[1]);
          const int zd = ora_shift(z, ORA_C[i][2], nz, P->bc[2]);
          if (xd >= 0 && yd >= 0 && zd >= 0) {
            const int64_t m = xd + (int64_t)nx * (yd + (int64_t)ny * zd);
            for (int k = 0; k < 5; ++k) f_out[(7 * k + i) * N + m] = fo[7 * k + i];
          }
          /* ghost upstream of this cell along c_i: its post-collision copy enters */
          const int xs = ora_shift(x, -ORA_C[i][0], nx, P->bc[0]);
          const int ys = ora_shift(y, -ORA_C[i][1], ny, P->bc[1]);
          const int zs = ora_shift(z, -ORA_C[i][2], nz, P->bc[2]);
          if (xs < 0 || ys < 0 || zs < 0) {
            for (int k = 0; k < 5; ++k) f_out[(7 * k + i) * N + n] = fo[7 * k + i];
          }
        }
      }
    }
  }
  if (diag) {
    diag[0] = ek;
    diag[1] = es;
    diag[2] = ed;
    for (int k = 0; k < 5; ++k) diag[3 + k] = tot[k];
    diag[8] = nonf;
  }
}

/* n steps from f (in place on return): alternates between f and work.  diag, when
 * not NULL, receives 9 values per step whose index t satisfies t % diag_every == 0
 * (rows written in order; the return value is the number of rows). */
int64_t ora_run(const ora_params* P, double* f, double* work, int64_t nsteps, int64_t diag_every,
                double* diag) {
  const int64_t N = ora_cells(P);
  double* a = f;
  double* b = work;
  int64_t rows = 0;
  for (int64_t t = 0; t < nsteps; ++t) {
    double* d = NULL;
    if (diag && diag_every > 0 && (t % diag_every) == 0) d = diag + 9 * rows++;
    ora_step(P, a, b, d);
    double* tmp = a;
    a = b;
    b = tmp;
  }
  if (a != f) memcpy(f, a, sizeof(double) * 35 * N);
  return rows;
}

/* Threads an OpenMP parallel region of the step uses. */
int32_t ora_num_threads(void) {
  int32_t n = 1;
#ifdef _OPENMP
#pragma omp parallel
  {
#pragma omp single
    n = (int32_t)omp_get_num_threads();
  }
#endif
  return n;
}

/* Threads for the following parallel regions (n >= 1; a no-op without OpenMP). */
void ora_set_num_threads(int32_t n) {
#ifdef _OPENMP
  if (n >= 1) omp_set_num_threads((int)n);
#else
  (void)n;
#endif
}

/* Size of the per-cell info record (lets the Python side check its mirror). */
int32_t ora_cell_info_size(void) { return (int32_t)sizeof(ora_cell_info); }
int32_t ora_params_size(void) { return (int32_t)sizeof(ora_params); }

/* ------------------------------------------------- manufactured solution (eq. 8) */
/* The manufactured field of Sec. 3.1 in lattice units on an n^3 periodic lattice
 * (cell (i, j, l) at x = (i, j, l), one period per n cells): every primitive is a
 * constant plus a sum of terms  A f(K x_axis + phase + s W t)  with f = sin or cos,
 * K = 2 pi / n per cell and W the angular frequency per step.  The amplitudes and
 * phases are those of eq. 8; the velocity scale U, pressure scale P0 and background
 * density rho0 come in lattice units. */
typedef struct {
  double rho0, U, P0, a;  /* background density, velocity scale (c_s of eq. 8), p0, a */
  double K, W;            /* 2 pi / n per cell, 2 pi per period in steps              */
  double gamma, mu, kappa;/* constant viscosity and conductivity, lattice units       */
} ora_mms;

typedef struct {
  double v, t, g[3], h[3][3]; /* value, d/dt, gradient, Hessian                        */
} ora_jet;

/* adds A f(K x_axis + ph + s W t), f = sin (is_sin) or cos, and its derivatives */
static void ora_jet_term(ora_jet* J, const ora_mms* M, double A, int axis, double ph, double s,
                         int is_sin, const double x[3], double t) {
  const double arg = M->K * x[axis] + ph + s * M->W * t;
  const double sn = sin(arg), cs = cos(arg);
  const double f = is_sin ? sn : cs;
  const double df = is_sin ? cs : -sn;  /* derivative of f with respect to its argument */
  J->v += A * f;
  J->g[axis] += A * M->K * df;
  J->t += A * s * M->W * df;
  J->h[axis][axis] += -A * M->K * M->K * f;
}

/* rho, u_x, u_y, u_z, p of eq. 8 with their derivatives at lattice point x, time t */
static void ora_mms_primitives(const ora_mms* M, const double x[3], double t, ora_jet J[5]) {
  memset(J, 0, 5 * sizeof(ora_jet));
  const double r0 = M->rho0, U = M->U, P0 = M->P0;
  J[0].v = r0;
  ora_jet_term(&J[0], M, 0.05 * r0, 0, 0.0, 0.0, 1, x, t);
  ora_jet_term(&J[0], M, 0.03 * r0, 1, 0.0, 0.0, 0, x, t);
  ora_jet_term(&J[0], M, 0.02 * r0, 2, 0.0, 1.0, 0, x, t);
  J[1].v = U * M->a;
  ora_jet_term(&J[1], M, 0.035 * U, 0, 0.4, 0.0, 0, x, t);
  ora_jet_term(&J[1], M, 0.025 * U, 1, 0.0, 0.0, 1, x, t);
  J[2].v = U * M->a;
  ora_jet_term(&J[2], M, 0.035 * U, 1, 0.9, 0.0, 1, x, t);
  ora_jet_term(&J[2], M, 0.025 * U, 2, 0.0, 0.0, 0, x, t);
  J[3].v = U * M->a;
  ora_jet_term(&J[3], M, 0.025 * U, 2, 1.7, 0.0, 0, x, t);
  ora_jet_term(&J[3], M, 0.015 * U, 0, 0.0, 1.0, 1, x, t);
  J[4].v = P0;
  ora_jet_term(&J[4], M, 0.05 * P0, 0, 1.2, 0.0, 0, x, t);
  ora_jet_term(&J[4], M, 0.03 * P0, 1, 0.0, 1.0, 1, x, t);
  ora_jet_term(&J[4], M, 0.02 * P0, 2, 0.6, 0.0, 1, x, t);
}

/* The source S = dQ/dt + div Phi of eq. 1 that makes the manufactured field an exact
 * solution of eq. 2 (constant mu and kappa, T = p/rho), written out by hand with
 * the product and chain rules from the primitive jets. */
static void ora_mms_source_point(const ora_mms* M, const double x[3], double t, double S[5]) {
  ora_jet J[5];
  ora_mms_primitives(M, x, t, J);
  const double g1 = M->gamma - 1.0;
  const double rho = J[0].v, p = J[4].v;
  const double* drho = J[0].g;
  const double* dp = J[4].g;
  double u[3], du[3][3], ut[3];  /* du[j][c] = d u_j / d x_c */
  for (int j = 0; j < 3; ++j) {
    u[j] = J[1 + j].v;
    ut[j] = J[1 + j].t;
    for (int c = 0; c < 3; ++c) du[j][c] = J[1 + j].g[c];
  }
  const double u2 = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
  const double E = p / g1 + 0.5 * rho * u2;
  double theta = du[0][0] + du[1][1] + du[2][2];
  /* d(theta)/dx_j = sum_c d^2 u_c / dx_j dx_c, and the Laplacian of u_j */
  double dtheta[3], lap_u[3];
  for (int j = 0; j < 3; ++j) {
    dtheta[j] = 0.0;
    lap_u[j] = 0.0;
    for (int c = 0; c < 3; ++c) {
      dtheta[j] += J[1 + c].h[j][c];
      lap_u[j] += J[1 + j].h[c][c];
    }
  }
  /* Newtonian stress and its divergence (constant mu) */
  double tau[3][3], div_tau[3];
  for (int j = 0; j < 3; ++j) {
    for (int c = 0; c < 3; ++c) tau[j][c] = M->mu * (du[j][c] + du[c][j] - (j == c ? 2.0 / 3.0 * theta : 0.0));
    div_tau[j] = M->mu * (lap_u[j] + dtheta[j] / 3.0);
  }
  /* time derivatives of the conserved fields */
  const double rho_t = J[0].t, p_t = J[4].t;
  double udut = 0.0;
  for (int j = 0; j < 3; ++j) udut += u[j] * ut[j];
  const double E_t = p_t / g1 + 0.5 * rho_t * u2 + rho * udut;
  /* gradient of E */
  double dE[3];
  for (int c = 0; c < 3; ++c) {
    double udu = 0.0;
    for (int j = 0; j < 3; ++j) udu += u[j] * du[j][c];
    dE[c] = dp[c] / g1 + 0.5 * drho[c] * u2 + rho * udu;
  }
  /* mass */
  double div_m = 0.0;
  for (int c = 0; c < 3; ++c) div_m += drho[c] * u[c] + rho * du[c][c];
  S[0] = rho_t + div_m;
  /* momentum: d_t(rho u_j) + d_c(rho u_j u_c) + d_j p - d_c tau_jc */
  for (int j = 0; j < 3; ++j) {
    double adv = 0.0;
    for (int c = 0; c < 3; ++c) adv += drho[c] * u[j] * u[c] + rho * du[j][c] * u[c] + rho * u[j] * du[c][c];
    S[1 + j] = rho_t * u[j] + rho * ut[j] + adv + dp[j] - div_tau[j];
  }
  /* energy: d_t E + d_c((E + p) u_c) - d_c(tau_cj u_j) + d_c q_c, q = -kappa grad(p/rho) */
  double adv = 0.0, work = 0.0;
  for (int c = 0; c < 3; ++c) adv += (dE[c] + dp[c]) * u[c] + (E + p) * du[c][c];
  for (int j = 0; j < 3; ++j) {
    work += div_tau[j] * u[j];
    for (int c = 0; c < 3; ++c) work += tau[c][j] * du[j][c];
  }
  double lap_T = 0.0;
  for (int c = 0; c < 3; ++c)
    lap_T += J[4].h[c][c] / rho - 2.0 * dp[c] * drho[c] / (rho * rho) - p * J[0].h[c][c] / (rho * rho) +
             2.0 * p * drho[c] * drho[c] / (rho * rho * rho);
  S[4] = E_t + adv - work - M->kappa * lap_T;
}

/* S[5][N] at every cell of P's lattice at lattice time t. */
void ora_mms_source(const ora_params* P, const ora_mms* M, double t, double* S) {
  const int64_t N = ora_cells(P);
#pragma omp parallel for collapse(2) schedule(static)
  for (int z = 0; z < P->nz; ++z)
    for (int y = 0; y < P->ny; ++y)
      for (int x = 0; x < P->nx; ++x) {
        const int64_t n = x + (int64_t)P->nx * (y + (int64_t)P->ny * z);
        const double xx[3] = {(double)x, (double)y, (double)z};
        double s[5];
        ora_mms_source_point(M, xx, t, s);
        for (int k = 0; k < 5; ++k) S[k * N + n] = s[k];
      }
}

/* n steps with the manufactured source, the source of step t0 + s evaluated at
 * lattice time t0 + s + t_frac (in place on return, work as in ora_run; S is scratch
 * of 5N doubles). */
void ora_run_mms(const ora_params* P, const ora_mms* M, double* f, double* work, double* S, int64_t nsteps,
                 double t0, double t_frac) {
  const int64_t N = ora_cells(P);
  double* a = f;
  double* b = work;
  for (int64_t s = 0; s < nsteps; ++s) {
    ora_mms_source(P, M, t0 + (double)s + t_frac, S);
    ora_step_src(P, a, b, NULL, S);
    double* tmp = a;
    a = b;
    b = tmp;
  }
  if (a != f) memcpy(f, a, sizeof(double) * 35 * N);
}

int32_t ora_mms_size(void) { return (int32_t)sizeof(ora_mms); }
