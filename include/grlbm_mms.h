/* grlbm_mms.h -- source of the manufactured solution of Sec. 3.1 (eq. 8), for
 * verification runs of the source term (lbm_set_source) on the GPU.
 *
 * The manufactured field is an exact solution of eq. 1 with the source
 * S = dQ/dt + div Phi of eq. 2 (constant mu and kappa, T = p/rho).  In lattice units
 * on an nx * ny * nz lattice, cell (i, j, l) at x = (i, j, l):
 *   rho = rho0 (1 + 0.05 sin(K x) + 0.03 cos(K y) + 0.02 cos(K z + W t))
 *   u_x = U (a + 0.035 cos(K x + 0.4) + 0.025 sin(K y))
 *   u_y = U (a + 0.035 sin(K y + 0.9) + 0.025 cos(K z))
 *   u_z = U (a + 0.025 cos(K z + 1.7) + 0.015 sin(K x + W t))
 *   p   = P0 (1 + 0.05 cos(K x + 1.2) + 0.03 sin(K y + W t) + 0.02 sin(K z + 0.6))
 *   E   = p / (gamma - 1) + rho |u|^2 / 2
 */
#ifndef GRLBM_MMS_H
#define GRLBM_MMS_H

#include <stdint.h>

#include "grlbm.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  double rho0, U, P0, a; /* background density, velocity scale, pressure scale, a = 0.3/sqrt(3) */
  double K, W;           /* wavenumber per cell (2 pi / n), angular frequency per step     */
  double gamma, mu, kappa;
} lbm_mms;

/* Writes S[5][nz][ny][nx] (FP32, device memory owned by the caller, lattice units per
 * step, field order rho, rho u_x, rho u_y, rho u_z, E) at lattice time t, evaluated in
 * FP64.  Asynchronous on hip_stream (NULL = the null stream).  EINVAL for NULL
 * pointers, empty or oversized (> 2^31 cells) lattices; EDEVICE if the launch fails. */
lbm_status lbm_mms_source(const lbm_mms* m, int32_t nx, int32_t ny, int32_t nz, double t, float* S_dev,
                          void* hip_stream);

#ifdef __cplusplus
}
#endif

#endif
