// grlbm_device.hpp -- device-side building blocks of the five-field update for
// gfx950: lattice addressing of the in-place AA pattern and the register-resident
// collision of Algorithm 1.
//
// Layout.  Populations are 35 arrays ("slots"), slot s = 7 k + i for field k
// (rho, rho u_x, rho u_y, rho u_z, E) and D3Q7 direction i (0, +x, -x, +y, -y, +z,
// -z); array s starts at element s * S, and cell (x, y, z) sits at element
// x + px (y + ny z) of every array, where the row pitch px >= nx pads each x-row to
// a whole number of 128-byte lines when that costs at most a sixteenth of the row
// (so the +-y and +-z neighbours of an aligned run of cells are aligned runs too);
// elements x in [nx, px) are padding that no update reads or writes.  Each stored
// value is g = f - w_i Q_ref,k.
//
// AA pattern (one buffer, updated in place).  At even parity slot i of cell x holds
// f_i(x).  An even step reads the cell's own slots and writes f*_i to its own slot
// opposite(i).  The odd step reads f_i(x) = f*_i(x - c_i) from slot opposite(i) of
// x - c_i and writes f*_i(x) to slot i of x + c_i, which restores even parity.  In
// both steps every memory location is read and written by the same lane only.
//
// Zero-gradient faces (the ghost beyond the face holds the adjacent cell's own
// post-collision populations).  For a direction i whose upstream neighbour x - c_i
// lies beyond such a face:
//   even step: slot i of x receives f*_i(x) (the ghost copy) instead of
//              f*_opposite(i)(x), which leaves the domain and is dropped;
//   odd step:  f_i(x) is read from slot i of x, f*_i(x) is also written to slot i
//              of x (the ghost copy entering at the next even step), and the
//              population leaving through the face is dropped.
// No other lane touches those locations in that step, so the scheme stays
// race-free; it needs at least two cells along a zero-gradient axis.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace grlbm {

constexpr int kQ = 7;
constexpr int kFields = 5;
constexpr int kPop = 35;

// Physics constants of one launch, FP32, lattice units.
struct Coll {
  float om[3];       // omega of rho, momentum, energy
  float gm1;         // gamma - 1
  float mu_ref;      // viscosity at T_ref
  float kappa_ref;   // conductivity at T_ref
  float suth_c;      // 1 + T_S, Sutherland prefactor
  float inv_T_ref, T_S;
  float gain, J_min, om_min;
  float rho_min, p_min;
  float rho_ref, E_ref;
  int32_t sutherland;
  float sc[5], isc[5];  // FP16 storage: stored value = g * sc[field] (powers of two)
};

struct Grid {
  int32_t nx, ny, nz;
  int32_t zg_x, zg_y, zg_z;  // zero-gradient flags per axis
  int64_t S;                 // elements between consecutive slot arrays
  int32_t px;                // row pitch: elements between consecutive x-rows (>= nx)
  int32_t pad_;
};

// Elements of one slot array that the grid's rows span (padding included).
__host__ __device__ __forceinline__ int64_t row_cells(const Grid& g) { return (int64_t)g.px * g.ny * g.nz; }

// Per-lane neighbourhood: the cell index and, for each of the six moving
// directions, where an odd step reads f_i (slot and cell) and whether the lane sits
// on a zero-gradient face upstream (lo) or downstream (hi) of that axis.
struct Nbr {
  int32_t n;
  int32_t xm, xp, ym, yp, zm, zp;  // periodic-wrapped neighbour cells
  bool lo_x, hi_x, lo_y, hi_y, lo_z, hi_z;
};

__device__ __forceinline__ Nbr make_nbr(const Grid& g, int x, int y, int z) {
  Nbr b;
  const int32_t plane = g.px * g.ny;
  b.n = x + g.px * (y + g.ny * z);
  b.xm = (x == 0) ? b.n + (g.nx - 1) : b.n - 1;
  b.xp = (x == g.nx - 1) ? b.n - (g.nx - 1) : b.n + 1;
  b.ym = (y == 0) ? b.n + g.px * (g.ny - 1) : b.n - g.px;
  b.yp = (y == g.ny - 1) ? b.n - g.px * (g.ny - 1) : b.n + g.px;
  b.zm = (z == 0) ? b.n + plane * (g.nz - 1) : b.n - plane;
  b.zp = (z == g.nz - 1) ? b.n - plane * (g.nz - 1) : b.n + plane;
  b.lo_x = g.zg_x && x == 0;
  b.hi_x = g.zg_x && x == g.nx - 1;
  b.lo_y = g.zg_y && y == 0;
  b.hi_y = g.zg_y && y == g.ny - 1;
  b.lo_z = g.zg_z && z == 0;
  b.hi_z = g.zg_z && z == g.nz - 1;
  return b;
}

// Element offset (within field k's block of 7 arrays) of f_i(x) for the read of an
// odd step, or equally the location of f_i(x) in the state after an odd number of
// completed steps.  Returns slot * S + cell relative to the field's first array.
template <bool ZG>
__device__ __forceinline__ int64_t odd_src(const Grid& g, const Nbr& b, int i) {
  const int64_t S = g.S;
  switch (i) {
    case 1: return (ZG && b.lo_x) ? 1 * S + b.n : 2 * S + b.xm;
    case 2: return (ZG && b.hi_x) ? 2 * S + b.n : 1 * S + b.xp;
    case 3: return (ZG && b.lo_y) ? 3 * S + b.n : 4 * S + b.ym;
    case 4: return (ZG && b.hi_y) ? 4 * S + b.n : 3 * S + b.yp;
    case 5: return (ZG && b.lo_z) ? 5 * S + b.n : 6 * S + b.zm;
    case 6: return (ZG && b.hi_z) ? 6 * S + b.n : 5 * S + b.zp;
    default: return b.n;
  }
}

// Element `cell` of the array at `base`; `base` must hold the same value in every
// lane of the wave (every caller passes a slot array of the kernel's state or of
// the block's batch instance).  FP16: the byte offset is formed in 32 bits (a cell
// index below 2^31 gives one below 2^32) and added to the base held in scalar
// registers, so each access is one global load or store with a scalar base and a
// per-lane offset, with no 64-bit address arithmetic per access.  The base goes
// through readfirstlane because otherwise the compiler folds the slot offset into
// a shared per-lane address and rebuilds a 64-bit address for every access (about
// 100 more VALU instructions per cell update); the integer round trip is cast back
// to the global address space, or the accesses would become flat ones.  With the
// 24-bit dither below, the FP16 kernels issue about 15% fewer VALU instructions
// and the even-pair kernel needs 130 registers instead of 198.  FP32 keeps plain
// pointer arithmetic: its byte offsets reach 2^33, and the step is bound by HBM
// rather than by issue.
__device__ __forceinline__ uint64_t wave_uniform(uint64_t v) {
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
  return ((uint64_t)hi << 32) | lo;
}
template <typename T>
__device__ __forceinline__ T* at(T* base, int32_t cell) {
  if constexpr (sizeof(T) == 2) {
    typedef __attribute__((address_space(1))) char gchar;
    gchar* b = (gchar*)wave_uniform(reinterpret_cast<uint64_t>(base));
    return (T*)(b + ((uint32_t)cell << 1));
  } else {
    return base + cell;
  }
}
template <typename T>
__device__ __forceinline__ const T* at(const T* base, int32_t cell) {
  return at(const_cast<T*>(base), cell);
}

// Address of f_i(x) for the read of an odd step (the location odd_src names).
template <bool ZG, typename T>
__device__ __forceinline__ const T* odd_at(const T* Fk, int64_t S, const Nbr& b, int i) {
  switch (i) {
    case 1: return (ZG && b.lo_x) ? at(Fk + 1 * S, b.n) : at(Fk + 2 * S, b.xm);
    case 2: return (ZG && b.hi_x) ? at(Fk + 2 * S, b.n) : at(Fk + 1 * S, b.xp);
    case 3: return (ZG && b.lo_y) ? at(Fk + 3 * S, b.n) : at(Fk + 4 * S, b.ym);
    case 4: return (ZG && b.hi_y) ? at(Fk + 4 * S, b.n) : at(Fk + 3 * S, b.yp);
    case 5: return (ZG && b.lo_z) ? at(Fk + 5 * S, b.n) : at(Fk + 6 * S, b.zm);
    case 6: return (ZG && b.hi_z) ? at(Fk + 6 * S, b.n) : at(Fk + 5 * S, b.zp);
    default: return at(Fk, b.n);
  }
}

// ---------------------------------------------------------------- storage types
template <typename T, bool NT>
__device__ __forceinline__ float ld(const T* p) {
  if constexpr (NT) {
    return static_cast<float>(__builtin_nontemporal_load(p));
  } else {
    return static_cast<float>(*p);
  }
}

// The stored value itself, unconverted.
template <typename T, bool NT>
__device__ __forceinline__ T ldraw(const T* p) {
  if constexpr (NT) {
    return __builtin_nontemporal_load(p);
  } else {
    return *p;
  }
}

// A stored population is the FP32 result rounded to the storage type.  For FP16
// the empty asm pins v as an FP32 register value first: otherwise the compiler may
// fold the last multiply-add into the conversion (one rounding straight to FP16)
// in one kernel and not in another, and kernels sharing the collision would store
// different bits.
template <typename T, bool NT>
__device__ __forceinline__ void st(T* p, float v) {
  if constexpr (sizeof(T) == 2) asm volatile("" : "+v"(v));
  if constexpr (NT) {
    __builtin_nontemporal_store(static_cast<T>(v), p);
  } else {
    *p = static_cast<T>(v);
  }
}

// ----------------------------------------------- FP16 stochastic rounding
// Round-to-nearest storage of a quasi-steady population rounds it the same way at
// every step, and the conserved fields drift by a fraction of an FP16 ulp per step.
// FP16 populations are therefore rounded stochastically: the 13 FP32 mantissa bits
// below FP16's 10 receive a uniform dither before they are cut off, so a value
// rounds up with probability equal to its distance from the lower FP16 neighbour
// and the rounding error has zero mean.  The dither of a stored element is a
// counter-based hash of its destination cell, its slot and the step, so every path
// that writes the element (even or odd step, direct or LDS-staged, single context
// or batch) stores the same bits.

// 32-bit integer finaliser (xor-shift and multiply rounds, "lowbias32").
__host__ __device__ __forceinline__ uint32_t mix32(uint32_t x) {
  x ^= x >> 16;
  x *= 0x7feb352du;
  x ^= x >> 15;
  x *= 0x846ca68bu;
  x ^= x >> 16;
  return x;
}

// Key of one step (the index of the step being taken, counted per instance).
__host__ __device__ __forceinline__ uint32_t step_key(int64_t step) {
  return mix32((uint32_t)step * 0x9e3779b9u + 0x632be5abu);
}

// Hash of a destination cell under a step key.
__device__ __forceinline__ uint32_t cell_key(int64_t cell, uint32_t skey) { return mix32((uint32_t)cell ^ skey); }

// The 13 dither bits of slot `slot` of a cell keyed hc: bits 11..23 of the cell
// key's low 24 bits times an odd 24-bit multiplier per slot.  Multiplication by an
// odd number is a bijection modulo 2^24, so over all keys every 13-bit value occurs
// equally often (exactly uniform).  The 24-bit multiply runs at full rate, where a
// 32-bit one is a quarter-rate instruction; it is written as the instruction
// because in C the compiler sees that the kept bits do not depend on the factors'
// top 8 bits, drops the 24-bit masks and emits the 32-bit multiply.  The
// multiplier goes in a scalar register, so `slot` must be the same in every lane
// (every caller passes a constant of an unrolled loop).
__device__ __forceinline__ uint32_t dither13(uint32_t hc, int slot) {
  const uint32_t m = ((0x9e3779u + 2u * (uint32_t)slot * 0x6c8e9du) & 0xffffffu) | 1u;
  uint32_t p;
  asm("v_mul_u32_u24 %0, %1, %2" : "=v"(p) : "s"(m), "v"(hc));
  return (p >> 11) & 0x1fffu;
}

// Stores population slot `slot` (7 k + i) of a cell whose key is hc.  FP32: plain
// store.  FP16: stochastic rounding as above (the rounded value is exact in FP16,
// so the conversion itself no longer rounds).
template <typename T, bool NT>
__device__ __forceinline__ void st_pop(T* p, float v, uint32_t hc, int slot) {
  if constexpr (sizeof(T) == 2) {
    const uint32_t dither = dither13(hc, slot);
    v = __uint_as_float((__float_as_uint(v) + dither) & 0xffffe000u);
  }
  st<T, NT>(p, v);
}

__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }

// Per-cell diagnostic densities (Sec. 3.3 channels) of the pre-collision state.
struct CellDiag {
  float ek, eps_s, eps_d;
  float dq[5];
  float nonfinite;
};

// --------------------------------------------------------------- the collision
// Algorithm 1 for one cell on the shifted populations g[35] (post-stream,
// pre-collision); overwrites g with the post-collision values.
//   COLL = 0: regularized collision with the compression sensor (Sec. 2.5)
//   COLL = 1: BGK
// The reconstruction R of eq. 4 is applied in closed form:
//   mass:      grad rho = grad~ rho                     (mass row of M is zero)
//   momentum:  X~ = grad~(rho u) - u (x) grad rho, and only the symmetric-
//              deviatoric part of X~ is scaled by 1/(1+beta), beta = 2 nu omega/c_s^2
//              (eq. 6); grad u = X / rho, grad(rho u) = X + u (x) grad rho
//   energy:    the scalar inversion of eq. 7 with the energy-row blocks of eq. 5
// followed by the chain rule to grad T.
// SCALED (FP16 storage): g holds the stored values g * sc[field]; the moments are
// brought back with isc and the post-collision values leave multiplied by sc, so
// the arithmetic in between is the same FP32 arithmetic as without scaling.
template <int COLL, bool DIAG, bool SCALED = false>
__device__ __forceinline__ void collide(float g[kPop], const Coll& c, CellDiag* d) {
  // moments (Algorithm 1; the shift cancels in the first moments)
  float dq[5], J[5][3];
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    const float* f = g + 7 * k;
    dq[k] = ((f[0] + f[1]) + (f[2] + f[3])) + ((f[4] + f[5]) + f[6]);
    J[k][0] = f[1] - f[2];
    J[k][1] = f[3] - f[4];
    J[k][2] = f[5] - f[6];
    if constexpr (SCALED) {
      dq[k] *= c.isc[k];
      J[k][0] *= c.isc[k];
      J[k][1] *= c.isc[k];
      J[k][2] *= c.isc[k];
    }
  }
  const float rho = c.rho_ref + dq[0];
  const float m0 = dq[1], m1 = dq[2], m2 = dq[3];
  const float E = c.E_ref + dq[4];

  // primitives with positivity floors
  const float rf = fmaxf(rho, c.rho_min);
  const float ir = rcp(rf);
  const float u0 = m0 * ir, u1 = m1 * ir, u2 = m2 * ir;
  const float k2 = u0 * u0 + u1 * u1 + u2 * u2;
  const float p = fmaxf(c.gm1 * (E - 0.5f * rf * k2), c.p_min);
  const float T = p * ir;
  // Sutherland factor mu(T)/mu_ref; the conductivity scales with the same factor
  float ratio = 1.0f;
  if (c.sutherland) {
    const float t = T * c.inv_T_ref;
    ratio = c.suth_c * t * __builtin_amdgcn_sqrtf(t) * rcp(t + c.T_S);
  }
  const float mu = c.mu_ref * ratio;
  const float kap = c.kappa_ref * ratio;
  const float nu = mu * ir;

  // direct gradients -Pi / (c_s^2 tau) = -4 omega (J - Phi_adv)  (eq. 3)
  const float a_r = -4.0f * c.om[0], a_m = -4.0f * c.om[1], a_e = -4.0f * c.om[2];
  const float gr0 = a_r * (J[0][0] - m0);
  const float gr1 = a_r * (J[0][1] - m1);
  const float gr2 = a_r * (J[0][2] - m2);
  const float u[3] = {u0, u1, u2};
  const float m[3] = {m0, m1, m2};
  const float gr[3] = {gr0, gr1, gr2};
  float X[3][3];  // X~ = grad~(rho u) - u (x) grad rho
#pragma unroll
  for (int j = 0; j < 3; ++j)
#pragma unroll
    for (int cc = 0; cc < 3; ++cc) {
      const float adv = m[j] * u[cc] + (j == cc ? p : 0.0f);
      X[j][cc] = a_m * (J[1 + j][cc] - adv) - u[j] * gr[cc];
    }
  const float H = E + p;
  float gE[3];
#pragma unroll
  for (int cc = 0; cc < 3; ++cc) gE[cc] = a_e * (J[4][cc] - H * u[cc]);

  // reconstruction (eq. 4).  Momentum block: scale the symmetric-deviatoric part.
  const float tr = X[0][0] + X[1][1] + X[2][2];
  const float beta = 8.0f * nu * c.om[1];
  const float fb = beta * rcp(1.0f + beta);
  const float tr3 = tr * (1.0f / 3.0f);
  float Xs[3][3];  // corrected rho grad u
#pragma unroll
  for (int j = 0; j < 3; ++j)
#pragma unroll
    for (int cc = 0; cc < 3; ++cc) {
      const float dev = 0.5f * (X[j][cc] + X[cc][j]) - (j == cc ? tr3 : 0.0f);
      Xs[j][cc] = X[j][cc] - fb * dev;
    }
  // grad(rho u) = Xs + u (x) grad rho
  float Gm[3][3];
#pragma unroll
  for (int j = 0; j < 3; ++j)
#pragma unroll
    for (int cc = 0; cc < 3; ++cc) Gm[j][cc] = Xs[j][cc] + u[j] * gr[cc];
  // energy row (eq. 7): grad E = (grad~E + 4 omega_E (M_Erho grad rho + M_Em grad m))
  //                               / (1 + 4 omega_E (gamma-1) kappa/rho)
  const float kr = kap * ir;
  const float ug = u0 * gr0 + u1 * gr1 + u2 * gr2;
  const float cr = nu * k2 + kr * (T - 0.5f * c.gm1 * k2);
  const float trm = Gm[0][0] + Gm[1][1] + Gm[2][2];
  const float ae4 = 4.0f * c.om[2];
  const float den = rcp(1.0f + ae4 * c.gm1 * kr);
  float Bt[3], gradE[3];
#pragma unroll
  for (int cc = 0; cc < 3; ++cc) {
    const float bm = Gm[cc][0] * u0 + Gm[cc][1] * u1 + Gm[cc][2] * u2;  // (grad m) u
    const float bt = Gm[0][cc] * u0 + Gm[1][cc] * u1 + Gm[2][cc] * u2;  // (grad m)^T u
    Bt[cc] = bt;
    const float MEr = cr * gr[cc] + nu * (1.0f / 3.0f) * u[cc] * ug;
    const float MEm = -nu * (bm + bt - (2.0f / 3.0f) * trm * u[cc]) + c.gm1 * kr * bt;
    gradE[cc] = (gE[cc] + ae4 * (MEr + MEm)) * den;
  }
  // chain rule: grad T = (gamma-1)/rho (grad E - (grad m)^T u) + (1/rho)((gamma-1)/2 |u|^2 - T) grad rho
  const float cT = ir * (0.5f * c.gm1 * k2 - T);
  const float gTf = c.gm1 * ir;
  float gT[3];
#pragma unroll
  for (int cc = 0; cc < 3; ++cc) gT[cc] = gTf * (gradE[cc] - Bt[cc]) + cT * gr[cc];

  // compression sensor (Sec. 2.5), s = -div(u)/c_s with c_s = 1/2
  const float theta = tr * ir;  // the deviatoric correction is traceless
  const float s = -2.0f * theta;
  float chi = 0.0f;
  if (COLL == 0) {
    chi = (theta < 0.0f && s > c.J_min) ? fminf(1.0f, fmaxf(0.0f, c.gain * s)) : 0.0f;
  }

  // closures: Newtonian stress tau = mu (grad u + grad u^T - 2/3 div u I), q = -kappa grad T
  const float mir = mu * ir;
  float tau[3][3];
#pragma unroll
  for (int j = 0; j < 3; ++j)
#pragma unroll
    for (int cc = 0; cc < 3; ++cc)
      tau[j][cc] = mir * (Xs[j][cc] + Xs[cc][j]) - (j == cc ? (2.0f / 3.0f) * mu * theta : 0.0f);

  // full flux of eq. 2 in the equilibrium
  float Phi[5][3];
#pragma unroll
  for (int cc = 0; cc < 3; ++cc) {
    Phi[0][cc] = m[cc];
#pragma unroll
    for (int j = 0; j < 3; ++j) Phi[1 + j][cc] = m[j] * u[cc] + (j == cc ? p : 0.0f) - tau[j][cc];
    const float tu = tau[cc][0] * u0 + tau[cc][1] * u1 + tau[cc][2] * u2;
    Phi[4][cc] = H * u[cc] - tu - kap * gT[cc];
  }

  if constexpr (DIAG) {
    const float wx = (X[2][1] - X[1][2]) * ir;  // curl from the antisymmetric part
    const float wy = (X[0][2] - X[2][0]) * ir;
    const float wz = (X[1][0] - X[0][1]) * ir;
    d->ek = 0.5f * rf * k2;
    d->eps_s = mu * (wx * wx + wy * wy + wz * wz);
    d->eps_d = (4.0f / 3.0f) * mu * theta * theta;
#pragma unroll
    for (int k = 0; k < 5; ++k) d->dq[k] = dq[k];
  }

  // collision
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    const float om = c.om[k == 0 ? 0 : (k == 4 ? 2 : 1)];
    float* f = g + 7 * k;
    // output scale (exactly 1 without SCALED)
    const float s = SCALED ? c.sc[k] : 1.0f;
    const float q8 = (SCALED ? 0.125f * s : 0.125f) * dq[k];
    const float h2 = SCALED ? 0.5f * s : 0.5f;
    if (COLL == 0) {
      // regularized: J* = omega_h Phi + (1 - omega_h) J
      const float oh = om - chi * (om - c.om_min);
      const float jx = J[k][0] + oh * (Phi[k][0] - J[k][0]);
      const float jy = J[k][1] + oh * (Phi[k][1] - J[k][1]);
      const float jz = J[k][2] + oh * (Phi[k][2] - J[k][2]);
      f[0] = (SCALED ? 0.25f * s : 0.25f) * dq[k];
      f[1] = q8 + h2 * jx;
      f[2] = q8 - h2 * jx;
      f[3] = q8 + h2 * jy;
      f[4] = q8 - h2 * jy;
      f[5] = q8 + h2 * jz;
      f[6] = q8 - h2 * jz;
    } else {
      // BGK: f <- f + omega (f_eq - f)
      const float e0 = (SCALED ? 0.25f * s : 0.25f) * dq[k];
      f[0] += om * (e0 - f[0]);
      f[1] += om * ((q8 + h2 * Phi[k][0]) - f[1]);
      f[2] += om * ((q8 - h2 * Phi[k][0]) - f[2]);
      f[3] += om * ((q8 + h2 * Phi[k][1]) - f[3]);
      f[4] += om * ((q8 - h2 * Phi[k][1]) - f[4]);
      f[5] += om * ((q8 + h2 * Phi[k][2]) - f[5]);
      f[6] += om * ((q8 - h2 * Phi[k][2]) - f[6]);
    }
  }
  if constexpr (DIAG) {
    bool bad = false;
#pragma unroll
    for (int s2 = 0; s2 < kPop; ++s2) bad |= !__builtin_isfinite(g[s2]);
    d->nonfinite = bad ? 1.0f : 0.0f;
  }
}

// ---------------------------------------------------------------- source term
// The source S of eq. 1 projected onto the lattice weights and added to the
// post-collision populations (the collision of Algorithm 1): f*_ki += w_i S_k.  src holds
// the step's source per cell, src[5][nz][ny][nx] (no row padding), lattice units.
__device__ __forceinline__ void add_source(float f[kPop], const float* __restrict__ src, const Grid& g, int x,
                                           int y, int z) {
  const int64_t N = (int64_t)g.nx * g.ny * g.nz;
  const int64_t n = x + (int64_t)g.nx * (y + (int64_t)g.ny * z);
#pragma unroll
  for (int k = 0; k < kFields; ++k) {
    const float s = src[k * N + n];
    f[7 * k] += 0.25f * s;
#pragma unroll
    for (int i = 1; i < kQ; ++i) f[7 * k + i] += 0.125f * s;
  }
}

// ----------------------------------------------------------------- one cell
// One cell's AA half step: gather the post-stream populations, run the collision of
// Algorithm 1 in registers, scatter the post-collision ones.  F points at slot 0 of
// the instance's arrays.  With DIAG, vals[9] receives the cell's diagnostic densities.
template <bool ODD, int COLL, typename T, bool ZG, bool DIAG, bool NT, bool SRC = false>
__device__ __forceinline__ void cell_update(T* __restrict__ F, const Grid& g, const Coll& c, int x,
                                            int y, int z, float* vals, uint32_t skey,
                                            const float* __restrict__ src = nullptr) {
  const Nbr b = make_nbr(g, x, y, z);
  const int64_t S = g.S;
  float f[kPop];
  // stream half of AA: gather the post-stream populations of this cell
#pragma unroll
  for (int k = 0; k < kFields; ++k) {
    const T* Fk = F + (int64_t)(7 * k) * S;
#pragma unroll
    for (int i = 0; i < kQ; ++i) {
      if constexpr (ODD) {
        f[7 * k + i] = ld<T, NT>(odd_at<ZG>(Fk, S, b, i));
      } else {
        f[7 * k + i] = ld<T, NT>(at(Fk + (int64_t)i * S, b.n));
      }
    }
  }
  CellDiag d;
  collide<COLL, DIAG, sizeof(T) == 2>(f, c, &d);
  if constexpr (DIAG) {
    vals[0] = d.ek;
    vals[1] = d.eps_s;
    vals[2] = d.eps_d;
#pragma unroll
    for (int k = 0; k < 5; ++k) vals[3 + k] = d.dq[k];
    vals[8] = d.nonfinite;
  }
  if constexpr (SRC) add_source(f, src, g, x, y, z);
  // store half of AA; FP16 dither keys of the destination cells
  const bool f16 = sizeof(T) == 2;
  const uint32_t hn = f16 ? cell_key(b.n, skey) : 0u;
  uint32_t hxp = 0u, hxm = 0u, hyp = 0u, hym = 0u, hzp = 0u, hzm = 0u;
  if constexpr (ODD && sizeof(T) == 2) {
    hxp = cell_key(b.xp, skey);
    hxm = cell_key(b.xm, skey);
    hyp = cell_key(b.yp, skey);
    hym = cell_key(b.ym, skey);
    hzp = cell_key(b.zp, skey);
    hzm = cell_key(b.zm, skey);
  }
#pragma unroll
  for (int k = 0; k < kFields; ++k) {
    T* Fk = F + (int64_t)(7 * k) * S;
    const float* fo = f + 7 * k;
    const int s0 = 7 * k;
    if constexpr (!ODD) {
      // own cell, opposite slot; on a zero-gradient face the ghost copy replaces
      // the population that leaves the domain
      st_pop<T, NT>(at(Fk, b.n), fo[0], hn, s0);
      st_pop<T, NT>(at(Fk + 1 * S, b.n), (ZG && b.lo_x) ? fo[1] : fo[2], hn, s0 + 1);
      st_pop<T, NT>(at(Fk + 2 * S, b.n), (ZG && b.hi_x) ? fo[2] : fo[1], hn, s0 + 2);
      st_pop<T, NT>(at(Fk + 3 * S, b.n), (ZG && b.lo_y) ? fo[3] : fo[4], hn, s0 + 3);
      st_pop<T, NT>(at(Fk + 4 * S, b.n), (ZG && b.hi_y) ? fo[4] : fo[3], hn, s0 + 4);
      st_pop<T, NT>(at(Fk + 5 * S, b.n), (ZG && b.lo_z) ? fo[5] : fo[6], hn, s0 + 5);
      st_pop<T, NT>(at(Fk + 6 * S, b.n), (ZG && b.hi_z) ? fo[6] : fo[5], hn, s0 + 6);
    } else {
      // slot i of the downstream cell x + c_i
      st_pop<T, NT>(at(Fk, b.n), fo[0], hn, s0);
      if (!(ZG && b.hi_x)) st_pop<T, NT>(at(Fk + 1 * S, b.xp), fo[1], hxp, s0 + 1);
      if (!(ZG && b.lo_x)) st_pop<T, NT>(at(Fk + 2 * S, b.xm), fo[2], hxm, s0 + 2);
      if (!(ZG && b.hi_y)) st_pop<T, NT>(at(Fk + 3 * S, b.yp), fo[3], hyp, s0 + 3);
      if (!(ZG && b.lo_y)) st_pop<T, NT>(at(Fk + 4 * S, b.ym), fo[4], hym, s0 + 4);
      if (!(ZG && b.hi_z)) st_pop<T, NT>(at(Fk + 5 * S, b.zp), fo[5], hzp, s0 + 5);
      if (!(ZG && b.lo_z)) st_pop<T, NT>(at(Fk + 6 * S, b.zm), fo[6], hzm, s0 + 6);
      if constexpr (ZG) {
        // ghost copy entering through a zero-gradient face
        if (b.lo_x) st_pop<T, NT>(at(Fk + 1 * S, b.n), fo[1], hn, s0 + 1);
        if (b.hi_x) st_pop<T, NT>(at(Fk + 2 * S, b.n), fo[2], hn, s0 + 2);
        if (b.lo_y) st_pop<T, NT>(at(Fk + 3 * S, b.n), fo[3], hn, s0 + 3);
        if (b.hi_y) st_pop<T, NT>(at(Fk + 4 * S, b.n), fo[4], hn, s0 + 4);
        if (b.lo_z) st_pop<T, NT>(at(Fk + 5 * S, b.n), fo[5], hn, s0 + 5);
        if (b.hi_z) st_pop<T, NT>(at(Fk + 6 * S, b.n), fo[6], hn, s0 + 6);
      }
    }
  }
}

// The even AA step for FP16 storage with two consecutive cells per lane.  The
// even step only touches the cell's own slots, so cells n and n + 1 (n even)
// share every access: each of the 35 slots moves as one 4-byte pair (low half
// cell n, high half cell n + 1), and a wave moves 256 bytes per array instead of
// 128.  The two cells are collided one after the other with the same call and
// rounded with the same per-cell dither as st_pop, so the stored bits are those
// of cell_update<false, COLL, _Float16, ...>.  Both cells must be cells of the grid
// (with nx even a pair never reaches into the row padding).
template <bool NT>
__device__ __forceinline__ uint32_t ld_pair(const _Float16* p) {
  const uint32_t* q = reinterpret_cast<const uint32_t*>(p);
  if constexpr (NT) return __builtin_nontemporal_load(q);
  return *q;
}
template <bool NT>
__device__ __forceinline__ void st_pair(_Float16* p, uint32_t v) {
  uint32_t* q = reinterpret_cast<uint32_t*>(p);
  if constexpr (NT) {
    __builtin_nontemporal_store(v, q);
  } else {
    *q = v;
  }
}
__device__ __forceinline__ float half_lo(uint32_t w) {
  return static_cast<float>(__builtin_bit_cast(_Float16, (uint16_t)(w & 0xffffu)));
}
__device__ __forceinline__ float half_hi(uint32_t w) {
  return static_cast<float>(__builtin_bit_cast(_Float16, (uint16_t)(w >> 16)));
}
// The FP16 bits st_pop<_Float16> stores for v.
__device__ __forceinline__ uint32_t half_bits(float v, uint32_t hc, int slot) {
  const uint32_t dither = dither13(hc, slot);
  v = __uint_as_float((__float_as_uint(v) + dither) & 0xffffe000u);
  asm volatile("" : "+v"(v));
  return (uint32_t)__builtin_bit_cast(uint16_t, static_cast<_Float16>(v));
}

template <int COLL, bool ZG, bool DIAG, bool NT>
__device__ __forceinline__ void pair_update_even(_Float16* __restrict__ F, const Grid& g, const Coll& c, int n,
                                                 float* vals, uint32_t skey) {
  const int64_t S = g.S;
  uint32_t w[kPop];  // slot pairs: inputs, overwritten half by half with the outputs
#pragma unroll
  for (int s = 0; s < kPop; ++s) w[s] = ld_pair<NT>(at(F + (int64_t)s * S, n));
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    // one cell at a time: the second cell's inputs stay packed until its turn
    // (otherwise they are unpacked early, next to the first cell's, and the
    // registers double)
    if (h == 1) {
#pragma unroll
      for (int s = 0; s < kPop; ++s) asm volatile("" : "+v"(w[s]));
    }
    const int cell = n + h;
    bool lo_x = false, hi_x = false, lo_y = false, hi_y = false, lo_z = false, hi_z = false;
    if constexpr (ZG) {
      const int row = cell / g.px;
      const int x = cell - row * g.px;
      const int z = row / g.ny;
      const int y = row - z * g.ny;
      lo_x = g.zg_x && x == 0;
      hi_x = g.zg_x && x == g.nx - 1;
      lo_y = g.zg_y && y == 0;
      hi_y = g.zg_y && y == g.ny - 1;
      lo_z = g.zg_z && z == 0;
      hi_z = g.zg_z && z == g.nz - 1;
    }
    float f[kPop];
#pragma unroll
    for (int s = 0; s < kPop; ++s) f[s] = h ? half_hi(w[s]) : half_lo(w[s]);
    CellDiag d;
    collide<COLL, DIAG, true>(f, c, &d);
    if constexpr (DIAG) {
      vals[0] += d.ek;
      vals[1] += d.eps_s;
      vals[2] += d.eps_d;
#pragma unroll
      for (int k = 0; k < 5; ++k) vals[3 + k] += d.dq[k];
      vals[8] += d.nonfinite;
    }
    const uint32_t hn = cell_key(cell, skey);
#pragma unroll
    for (int k = 0; k < kFields; ++k) {
      const float* fo = f + 7 * k;
      const int s0 = 7 * k;
      // own cell, opposite slot; the ghost copy on a zero-gradient face
      const float v[kQ] = {fo[0],
                           (ZG && lo_x) ? fo[1] : fo[2], (ZG && hi_x) ? fo[2] : fo[1],
                           (ZG && lo_y) ? fo[3] : fo[4], (ZG && hi_y) ? fo[4] : fo[3],
                           (ZG && lo_z) ? fo[5] : fo[6], (ZG && hi_z) ? fo[6] : fo[5]};
#pragma unroll
      for (int i = 0; i < kQ; ++i) {
        const uint32_t bits = half_bits(v[i], hn, s0 + i);
        w[s0 + i] = h ? (w[s0 + i] & 0xffffu) | (bits << 16) : (w[s0 + i] & 0xffff0000u) | bits;
      }
    }
  }
#pragma unroll
  for (int s = 0; s < kPop; ++s) st_pair<NT>(at(F + (int64_t)s * S, n), w[s]);
}

// ----------------------------------------------------- odd update of one tile
// The odd half step of a tile of B = blockDim.x consecutive cells [n0, n0 + B) of
// one grid (the tile may start mid-row and span rows), with the +-x populations
// moved through LDS.  Read directly, the x populations sit one element off the
// 64-lane chunks, so every wave would touch one more cache line than it moves and
// leave partial lines behind.  Here the two x slots of the tile's own cells are
// loaded aligned into LDS, the shifted reads and writes happen in LDS, and the
// slots go back to HBM aligned; the y, z and rest populations are accessed
// directly as in cell_update.
//
// In the AA scheme every slot location is read and then written by one and the
// same cell: slot 1 of cell m by its left neighbour (by m itself when m sits on a
// zero-gradient x = 0 face), slot 2 of m by its right neighbour (by m itself on an
// x = nx - 1 face).  A location whose cell lies in the tile is staged; the few
// whose cell lies in another tile (the tile's ends, periodic wraps to a row end
// outside the tile) are accessed directly by that cell, and the tile does not write
// them back.  So tiles never touch each other's locations and need no ordering.
//
// Every lane of the block must call this (it holds two barriers); lanes with
// act = false (past the grid's last cell) only take part in the barriers.  xs has
// room for 15 * B floats: the two slots and a per-lane column that absorbs the LDS
// writes a cell does not make, so that no LDS access needs a branch.  EDGES =
// false asserts that the tile holds whole x-rows (then every x location is in the
// tile and the edge handling compiles away).  HF > 0 loads the y slots without the
// nontemporal hint, HF = 2 the z slots as well.  Where rows are not whole 128-byte
// lines, a wave's y neighbours start part of a line off, and the adjacent wave
// reads the rest of that line: the hinted loads ran 10-12% slower there (FP32
// 100^3-176^3; FP16 5-9%), while the stores, the z slots of single grids and
// aligned rows gained nothing from dropping it.  Batches of tubes a few cells
// across, whose planes are a fraction of a line, gained from the z slots as well.
// The collision is the same call as in cell_update, so the results are bitwise
// those of cell_update<true, ...>.
template <int COLL, typename T, bool ZG, bool DIAG, bool NT, bool EDGES = true, bool SRC = false, int HF = 0>
__device__ __forceinline__ void tile_update_odd(T* __restrict__ F, const Grid& g, const Coll& c, int n0,
                                                bool act, int x, int y, int z, float* xs, float* vals,
                                                uint32_t skey, const float* __restrict__ src = nullptr) {
  const int B = blockDim.x;
  const int lane = threadIdx.x;
  const Nbr b = make_nbr(g, x, y, z);
  const int64_t S = g.S;
  float* s1 = xs;              // slot 1 of the tile's cells, [field][B]
  float* s2 = xs + 5 * B;      // slot 2
  float* sink = xs + 10 * B;   // [field][B], written and never read
  float f[kPop];
  T raw[kPop];  // FP16: the rest, y and z slots as loaded, converted after the barrier
  if (act) {
    if constexpr (sizeof(T) == 2) {
      // FP16: the ten x slots first, so that their LDS writes, and with them the
      // barrier, wait for those loads only while the other 25 are in flight (the
      // odd step took 422.8 against 427.2 us at 256^3, two alternating runs).  In
      // FP32 the same order ran 4.5% slower, so FP32 keeps the per-field order.
      float x1[kFields], x2[kFields];
#pragma unroll
      for (int k = 0; k < kFields; ++k) {
        const T* Fk = F + (int64_t)(7 * k) * S;
        x1[k] = ld<T, NT>(at(Fk + 1 * S, b.n));
        x2[k] = ld<T, NT>(at(Fk + 2 * S, b.n));
      }
#pragma unroll
      for (int k = 0; k < kFields; ++k) {
        const T* Fk = F + (int64_t)(7 * k) * S;
        raw[7 * k + 0] = ldraw<T, NT>(at(Fk, b.n));
        if constexpr (HF > 0) {
          raw[7 * k + 3] = ldraw<T, false>(odd_at<ZG>(Fk, S, b, 3));
          raw[7 * k + 4] = ldraw<T, false>(odd_at<ZG>(Fk, S, b, 4));
          raw[7 * k + 5] = ldraw<T, NT && HF < 2>(odd_at<ZG>(Fk, S, b, 5));
          raw[7 * k + 6] = ldraw<T, NT && HF < 2>(odd_at<ZG>(Fk, S, b, 6));
        } else {
#pragma unroll
          for (int i = 3; i < kQ; ++i) raw[7 * k + i] = ldraw<T, NT>(odd_at<ZG>(Fk, S, b, i));
        }
      }
#pragma unroll
      for (int k = 0; k < kFields; ++k) {
        s1[k * B + lane] = x1[k];
        s2[k * B + lane] = x2[k];
      }
    } else {
#pragma unroll
      for (int k = 0; k < kFields; ++k) {
        const T* Fk = F + (int64_t)(7 * k) * S;
        s1[k * B + lane] = ld<T, NT>(at(Fk + 1 * S, b.n));
        s2[k * B + lane] = ld<T, NT>(at(Fk + 2 * S, b.n));
        f[7 * k + 0] = ld<T, NT>(at(Fk, b.n));
        if constexpr (HF > 0) {
          f[7 * k + 3] = ld<T, false>(odd_at<ZG>(Fk, S, b, 3));
          f[7 * k + 4] = ld<T, false>(odd_at<ZG>(Fk, S, b, 4));
          f[7 * k + 5] = ld<T, NT && HF < 2>(odd_at<ZG>(Fk, S, b, 5));
          f[7 * k + 6] = ld<T, NT && HF < 2>(odd_at<ZG>(Fk, S, b, 6));
        } else {
#pragma unroll
          for (int i = 3; i < kQ; ++i) f[7 * k + i] = ld<T, NT>(odd_at<ZG>(Fk, S, b, i));
        }
      }
    }
  }
  const bool lo = ZG && b.lo_x;
  const bool hi = ZG && b.hi_x;
  // f_{+x} lives in slot 1 of the cell itself (zero-gradient face) or in slot 2 of
  // the left neighbour; f_{-x} in slot 2 of the cell itself or slot 1 of the right one
  const int m1 = lo ? b.n : b.xm;
  const int m2 = hi ? b.n : b.xp;
  const bool in1 = !EDGES || (unsigned)(m1 - n0) < (unsigned)B;  // always true when lo
  const bool in2 = !EDGES || (unsigned)(m2 - n0) < (unsigned)B;  // always true when hi
  // outside the tile (so neither lo nor hi): slot 2 of m1, slot 1 of m2, directly
  float d1[kFields], d2[kFields];
  if (act && !in1) {
#pragma unroll
    for (int k = 0; k < kFields; ++k) d1[k] = ld<T, NT>(at(F + (int64_t)(7 * k + 2) * S, m1));
  }
  if (act && !in2) {
#pragma unroll
    for (int k = 0; k < kFields; ++k) d2[k] = ld<T, NT>(at(F + (int64_t)(7 * k + 1) * S, m2));
  }
  __syncthreads();
  const float* r1 = (lo ? s1 : s2) + (in1 ? m1 - n0 : lane);
  const float* r2 = (hi ? s2 : s1) + (in2 ? m2 - n0 : lane);
  // LDS targets of the post-collision f_{+x}: slot 1 of the right neighbour, and
  // (ghost copy) slot 1 of the cell itself on an x = 0 face; f_{-x} mirrored
  float* w1 = (!hi && in2) ? s1 + (b.xp - n0) : sink + lane;
  float* w1g = lo ? s1 + lane : sink + lane;
  float* w2 = (!lo && in1) ? s2 + (b.xm - n0) : sink + lane;
  float* w2g = hi ? s2 + lane : sink + lane;
  if (act) {
#pragma unroll
    for (int k = 0; k < kFields; ++k) {
      const float v1 = r1[k * B];
      const float v2 = r2[k * B];
      f[7 * k + 1] = in1 ? v1 : d1[k];
      f[7 * k + 2] = in2 ? v2 : d2[k];
      if constexpr (sizeof(T) == 2) {
        // the empty asm keeps the conversions, and the waits for these loads,
        // after the barrier (the compiler would otherwise hoist them before it)
        asm volatile("" : "+v"(raw[7 * k + 0]));
#pragma unroll
        for (int i = 3; i < kQ; ++i) asm volatile("" : "+v"(raw[7 * k + i]));
        f[7 * k + 0] = static_cast<float>(raw[7 * k + 0]);
#pragma unroll
        for (int i = 3; i < kQ; ++i) f[7 * k + i] = static_cast<float>(raw[7 * k + i]);
      }
    }
    CellDiag d;
    collide<COLL, DIAG, sizeof(T) == 2>(f, c, &d);
    if constexpr (DIAG) {
      vals[0] = d.ek;
      vals[1] = d.eps_s;
      vals[2] = d.eps_d;
#pragma unroll
      for (int k = 0; k < 5; ++k) vals[3 + k] = d.dq[k];
      vals[8] = d.nonfinite;
    }
    if constexpr (SRC) add_source(f, src, g, x, y, z);
    // FP16 dither keys of the destination cells (the x slots are keyed by the cell
    // that finally stores them, which is their destination as well)
    uint32_t hn = 0u, hyp = 0u, hym = 0u, hzp = 0u, hzm = 0u;
    if constexpr (sizeof(T) == 2) {
      hn = cell_key(b.n, skey);
      hyp = cell_key(b.yp, skey);
      hym = cell_key(b.ym, skey);
      hzp = cell_key(b.zp, skey);
      hzm = cell_key(b.zm, skey);
    }
#pragma unroll
    for (int k = 0; k < kFields; ++k) {
      T* Fk = F + (int64_t)(7 * k) * S;
      const float* fo = f + 7 * k;
      const int s0 = 7 * k;
      st_pop<T, NT>(at(Fk, b.n), fo[0], hn, s0);
      if (!(ZG && b.hi_y)) st_pop<T, NT>(at(Fk + 3 * S, b.yp), fo[3], hyp, s0 + 3);
      if (!(ZG && b.lo_y)) st_pop<T, NT>(at(Fk + 4 * S, b.ym), fo[4], hym, s0 + 4);
      if (!(ZG && b.hi_z)) st_pop<T, NT>(at(Fk + 5 * S, b.zp), fo[5], hzp, s0 + 5);
      if (!(ZG && b.lo_z)) st_pop<T, NT>(at(Fk + 6 * S, b.zm), fo[6], hzm, s0 + 6);
      if constexpr (ZG) {
        if (b.lo_y) st_pop<T, NT>(at(Fk + 3 * S, b.n), fo[3], hn, s0 + 3);
        if (b.hi_y) st_pop<T, NT>(at(Fk + 4 * S, b.n), fo[4], hn, s0 + 4);
        if (b.lo_z) st_pop<T, NT>(at(Fk + 5 * S, b.n), fo[5], hn, s0 + 5);
        if (b.hi_z) st_pop<T, NT>(at(Fk + 6 * S, b.n), fo[6], hn, s0 + 6);
      }
      w1[k * B] = fo[1];
      w2[k * B] = fo[2];
      if constexpr (ZG) {
        w1g[k * B] = fo[1];
        w2g[k * B] = fo[2];
      }
    }
    if (!hi && !in2) {
      const uint32_t h = sizeof(T) == 2 ? cell_key(b.xp, skey) : 0u;
#pragma unroll
      for (int k = 0; k < kFields; ++k) st_pop<T, NT>(at(F + (int64_t)(7 * k + 1) * S, b.xp), f[7 * k + 1], h, 7 * k + 1);
    }
    if (!lo && !in1) {
      const uint32_t h = sizeof(T) == 2 ? cell_key(b.xm, skey) : 0u;
#pragma unroll
      for (int k = 0; k < kFields; ++k) st_pop<T, NT>(at(F + (int64_t)(7 * k + 2) * S, b.xm), f[7 * k + 2], h, 7 * k + 2);
    }
  }
  __syncthreads();
  // write back the slots of this tile's cells whose reader/writer is in the tile
  const uint32_t hown = (sizeof(T) == 2 && act) ? cell_key(b.n, skey) : 0u;
  if (act && in1) {
#pragma unroll
    for (int k = 0; k < kFields; ++k) st_pop<T, NT>(at(F + (int64_t)(7 * k + 1) * S, b.n), s1[k * B + lane], hown, 7 * k + 1);
  }
  if (act && in2) {
#pragma unroll
    for (int k = 0; k < kFields; ++k) st_pop<T, NT>(at(F + (int64_t)(7 * k + 2) * S, b.n), s2[k * B + lane], hown, 7 * k + 2);
  }
}

// ------------------------------------- FP16 odd update of one row, two cells a lane
// The odd half step of one x-row (y, z) with FP16 storage and two consecutive cells
// per lane: lane l (0 <= l < nx / 2) holds cells x = 2l and 2l + 1 (nx even).  The +-x populations move through LDS as in tile_update_odd
// (xs holds 15 nx floats: slot 1, slot 2, sink).  The rest, y and z populations of
// the two cells sit at consecutive elements of one array, 4-byte aligned because
// every row starts at an even cell, and both cells share the row and therefore the
// neighbour rows and the y and z zero-gradient flags: each of those accesses moves
// one half pair, as in pair_update_even.  On each of the y and z axes a cell stores
// exactly two populations, to the neighbour rows or, on a zero-gradient face, one of
// them to its own cell (the ghost copy); the pair words are named for those two
// stores.  The cells are collided one after the other with the same call, and every
// value is rounded with the dither of its destination cell and slot, so the bits
// are those of tile_update_odd<COLL, _Float16, ...>.  The block is the row's nx / 2
// lanes, and every one must call this (two barriers).
template <int COLL, bool ZG, bool DIAG, bool NT>
__device__ __forceinline__ void pair_row_update_odd(_Float16* __restrict__ F, const Grid& g, const Coll& c,
                                                    int lane, int y, int z, float* xs, float* vals,
                                                    uint32_t skey) {
  const int nx = g.nx;
  const int x0 = 2 * lane;
  const Nbr b = make_nbr(g, x0, y, z);  // of the first cell; the second is b.n + 1
  const int64_t S = g.S;
  float* s1 = xs;              // slot 1 of the row's cells, [field][nx]
  float* s2 = xs + 5 * nx;     // slot 2
  float* sink = xs + 10 * nx;  // [field][nx], written and never read
  // w[7k]: slot 0; w[7k + 3], w[7k + 4]: the two y stores (below); w[7k + 5],
  // w[7k + 6]: the two z stores.  Inputs first, then overwritten half by half.
  uint32_t w[kPop];
#pragma unroll
  for (int k = 0; k < kFields; ++k) {
    const _Float16* Fk = F + (int64_t)(7 * k) * S;
    const uint32_t p1 = ld_pair<NT>(at(Fk + 1 * S, b.n));
    const uint32_t p2 = ld_pair<NT>(at(Fk + 2 * S, b.n));
    s1[k * nx + x0] = half_lo(p1);
    s1[k * nx + x0 + 1] = half_hi(p1);
    s2[k * nx + x0] = half_lo(p2);
    s2[k * nx + x0 + 1] = half_hi(p2);
    w[7 * k] = ld_pair<NT>(at(Fk, b.n));
#pragma unroll
    for (int i = 3; i < kQ; ++i) w[7 * k + i] = ld_pair<NT>(odd_at<ZG>(Fk, S, b, i));
  }
  __syncthreads();
  const bool ylo = ZG && b.lo_y, yhi = ZG && b.hi_y, zlo = ZG && b.lo_z, zhi = ZG && b.hi_z;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    if (h == 1) {
#pragma unroll
      for (int s = 0; s < kPop; ++s) asm volatile("" : "+v"(w[s]));
    }
    const int x = x0 + h;
    const bool lo = ZG && g.zg_x && x == 0;
    const bool hi = ZG && g.zg_x && x == nx - 1;
    const int xm = (x == 0) ? nx - 1 : x - 1;
    const int xp = (x == nx - 1) ? 0 : x + 1;
    // f_{+x}: slot 1 of the cell itself (zero-gradient face) or slot 2 of the left
    // neighbour; f_{-x}: slot 2 of the cell itself or slot 1 of the right neighbour
    const float* r1 = lo ? s1 + x : s2 + xm;
    const float* r2 = hi ? s2 + x : s1 + xp;
    float* w1 = hi ? sink + x : s1 + xp;
    float* w1g = lo ? s1 + x : sink + x;
    float* w2 = lo ? sink + x : s2 + xm;
    float* w2g = hi ? s2 + x : sink + x;
    float f[kPop];
#pragma unroll
    for (int k = 0; k < kFields; ++k) {
      f[7 * k] = h ? half_hi(w[7 * k]) : half_lo(w[7 * k]);
      f[7 * k + 1] = r1[k * nx];
      f[7 * k + 2] = r2[k * nx];
#pragma unroll
      for (int i = 3; i < kQ; ++i) f[7 * k + i] = h ? half_hi(w[7 * k + i]) : half_lo(w[7 * k + i]);
    }
    CellDiag d;
    collide<COLL, DIAG, true>(f, c, &d);
    if constexpr (DIAG) {
      vals[0] += d.ek;
      vals[1] += d.eps_s;
      vals[2] += d.eps_d;
#pragma unroll
      for (int k = 0; k < 5; ++k) vals[3 + k] += d.dq[k];
      vals[8] += d.nonfinite;
    }
    const int n = b.n + h;
    const uint32_t hn = cell_key(n, skey);
    const uint32_t hy0 = yhi ? hn : cell_key(b.yp + h, skey);
    const uint32_t hy1 = ylo ? hn : cell_key(b.ym + h, skey);
    const uint32_t hz0 = zhi ? hn : cell_key(b.zp + h, skey);
    const uint32_t hz1 = zlo ? hn : cell_key(b.zm + h, skey);
#pragma unroll
    for (int k = 0; k < kFields; ++k) {
      const float* fo = f + 7 * k;
      const int s0 = 7 * k;
      const uint32_t bits[5] = {half_bits(fo[0], hn, s0),
                                yhi ? half_bits(fo[4], hy0, s0 + 4) : half_bits(fo[3], hy0, s0 + 3),
                                ylo ? half_bits(fo[3], hy1, s0 + 3) : half_bits(fo[4], hy1, s0 + 4),
                                zhi ? half_bits(fo[6], hz0, s0 + 6) : half_bits(fo[5], hz0, s0 + 5),
                                zlo ? half_bits(fo[5], hz1, s0 + 5) : half_bits(fo[6], hz1, s0 + 6)};
      const int ws[5] = {s0, s0 + 3, s0 + 4, s0 + 5, s0 + 6};
#pragma unroll
      for (int j = 0; j < 5; ++j)
        w[ws[j]] = h ? (w[ws[j]] & 0xffffu) | (bits[j] << 16) : (w[ws[j]] & 0xffff0000u) | bits[j];
      w1[k * nx] = fo[1];
      w2[k * nx] = fo[2];
      if constexpr (ZG) {
        w1g[k * nx] = fo[1];
        w2g[k * nx] = fo[2];
      }
    }
  }
#pragma unroll
  for (int k = 0; k < kFields; ++k) {
    _Float16* Fk = F + (int64_t)(7 * k) * S;
    // where the two stores of each axis go: (slot, cell) of the first and the second
    _Float16* const dst[4] = {yhi ? at(Fk + 4 * S, b.n) : at(Fk + 3 * S, b.yp),
                              ylo ? at(Fk + 3 * S, b.n) : at(Fk + 4 * S, b.ym),
                              zhi ? at(Fk + 6 * S, b.n) : at(Fk + 5 * S, b.zp),
                              zlo ? at(Fk + 5 * S, b.n) : at(Fk + 6 * S, b.zm)};
    st_pair<NT>(at(Fk, b.n), w[7 * k]);
#pragma unroll
    for (int j = 0; j < 4; ++j) st_pair<NT>(dst[j], w[7 * k + 3 + j]);
  }
  __syncthreads();
  // write back both cells' x slots, rounded with their own keys
  const uint32_t ha = cell_key(b.n, skey), hb = cell_key(b.n + 1, skey);
#pragma unroll
  for (int k = 0; k < kFields; ++k) {
    _Float16* Fk = F + (int64_t)(7 * k) * S;
    st_pair<NT>(at(Fk + 1 * S, b.n), half_bits(s1[k * nx + x0], ha, 7 * k + 1) |
                                      (half_bits(s1[k * nx + x0 + 1], hb, 7 * k + 1) << 16));
    st_pair<NT>(at(Fk + 2 * S, b.n), half_bits(s2[k * nx + x0], ha, 7 * k + 2) |
                                      (half_bits(s2[k * nx + x0 + 1], hb, 7 * k + 2) << 16));
  }
}

}  // namespace grlbm
