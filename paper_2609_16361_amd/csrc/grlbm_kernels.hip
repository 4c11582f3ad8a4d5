// grlbm_kernels.hip -- HIP kernels for gfx950 and their host-side launchers.
//
//   k_step      fused collide-and-stream update of one AA half step (even or odd
//               parity): 35 loads, the collision of Algorithm 1 in registers, 35
//               stores; optional fused diagnostics (wavefront shuffle + LDS
//               reduction to one partial per block) and an optional source term
//   k_step_odd_tiles  the odd half step over linear tiles of cells with the +-x
//               populations shifted in LDS, so every HBM access stays aligned
//   k_step_even_pairs, k_step_odd_row_pairs  FP16 even and odd half steps with
//               two consecutive cells per lane (4-byte accesses) on large grids
//   k_finalize  deterministic reduction of the per-block partials into one record
//   k_init      initial populations from the conserved fields (first-order start)
//   k_gather    parity-aware readout: canonical populations or conserved moments
//   k_scatter   parity-aware write of canonical populations (checkpoint restore)
//   k_copy      streaming copy used to measure achievable HBM bandwidth
//
// One lane owns one cell (two in the pair kernels); a block covers `blockDim.x`
// consecutive cells, so every wave reads and writes 64 consecutive elements of each
// of the 35 arrays (coalesced).  The update is memory-bound (no contraction, no
// MFMA).
#include <hip/hip_runtime.h>

#include "grlbm_device.hpp"
#include "grlbm_internal.h"

namespace grlbm {


// ----------------------------------------------------------------- block mapping
struct CellPos {
  int x, y, z;
  bool active;
};

// Block b holds the consecutive elements [b * blockDim.x, (b + 1) * blockDim.x) of
// the arrays, so a wave reads and writes 64 consecutive elements of each array;
// lanes past the last row or in a row's padding (x >= nx) have no cell.  (Blocks
// that stopped at row ends left lanes idle and waves straddling cache lines
// whenever nx was not a multiple of the block: 144-cell rows kept 144 of 256 lanes
// busy and cost a fifth of the rate.)  When whole blocks fit a row the position
// comes from the block index alone; otherwise each lane divides its element index.
__device__ __forceinline__ CellPos block_cell(const Grid& g) {
  const int bx = blockDim.x;
  const int b = blockIdx.x;
  CellPos p;
  if (g.px % bx == 0) {
    const int nxb = g.px / bx;
    const int row = b / nxb;
    p.x = (b - row * nxb) * bx + threadIdx.x;
    p.y = row % g.ny;
    p.z = row / g.ny;
    p.active = row < g.ny * g.nz && p.x < g.nx;
  } else {
    const int n = b * bx + (int)threadIdx.x;  // below 2^31: the element count is capped
    const bool in = n < g.px * g.ny * g.nz;
    const int row = in ? n / g.px : 0;
    p.x = in ? n - row * g.px : 0;
    p.z = row / g.ny;
    p.y = row - p.z * g.ny;
    p.active = in && p.x < g.nx;
  }
  return p;
}

// -------------------------------------------------------- diagnostics reduction
constexpr int kDiagVals = 9;  // ek, eps_s, eps_d, dq[5], nonfinite

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__device__ void block_reduce_store(float vals[kDiagVals], float* __restrict__ out) {
  __shared__ float sm[16][kDiagVals];  // up to 1024 threads = 16 waves
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
#pragma unroll
  for (int j = 0; j < kDiagVals; ++j) vals[j] = wave_sum(vals[j]);
  if (lane == 0) {
#pragma unroll
    for (int j = 0; j < kDiagVals; ++j) sm[wave][j] = vals[j];
  }
  __syncthreads();
  if (threadIdx.x < kDiagVals) {
    const int nw = (blockDim.x + 63) >> 6;
    float s = 0.0f;
    for (int w = 0; w < nw; ++w) s += sm[w][threadIdx.x];
    out[(int64_t)blockIdx.x * kDiagVals + threadIdx.x] = s;
  }
}

// ------------------------------------------------------------------ the update
template <bool ODD, int COLL, typename T, bool ZG, bool DIAG, bool NT, bool SRC = false>
__global__ void __launch_bounds__(1024) k_step(T* __restrict__ F, Grid g, Coll c, float* __restrict__ partials,
                                                const float* __restrict__ src, uint32_t skey) {
  const CellPos pos = block_cell(g);
  float vals[kDiagVals];
  if constexpr (DIAG) {
#pragma unroll
    for (int j = 0; j < kDiagVals; ++j) vals[j] = 0.0f;
  }
  if (pos.active) cell_update<ODD, COLL, T, ZG, DIAG, NT, SRC>(F, g, c, pos.x, pos.y, pos.z, vals, skey, src);
  if constexpr (DIAG) block_reduce_store(vals, partials);
}

// Even AA step for FP16 storage with two consecutive cells per lane
// (pair_update_even); needs an even cell count and blocks of at most 256 threads
// (two cells' populations in registers), and runs on grids of kPairMinCells and
// more.  Bitwise the same result as k_step's even step.
template <int COLL, bool ZG, bool DIAG, bool NT>
__global__ void __launch_bounds__(256) k_step_even_pairs(_Float16* __restrict__ F, Grid g, Coll c,
                                                           float* __restrict__ partials, uint32_t skey) {
  const int n = 2 * ((int)blockIdx.x * (int)blockDim.x + (int)threadIdx.x);
  float vals[kDiagVals];
  if constexpr (DIAG) {
#pragma unroll
    for (int j = 0; j < kDiagVals; ++j) vals[j] = 0.0f;
  }
  // nx and px even: a pair lies wholly in a row or wholly in its padding
  if (n < g.px * g.ny * g.nz && n % g.px < g.nx) pair_update_even<COLL, ZG, DIAG, NT>(F, g, c, n, vals, skey);
  if constexpr (DIAG) block_reduce_store(vals, partials);
}

// Odd AA step over tiles of consecutive cells with the +-x populations shifted in
// LDS (tile_update_odd): every HBM access of the x slots is aligned.  MAP selects
// the tiles: kOddRow, one block per x-row (nx <= 1024, blockDim.x = nx rounded up to
// 64); kOddRowGroup, `tl` consecutive cells that are whole rows (tl = R * px, R >= 1,
// tl <= blockDim.x, the lanes past tl idle), so that every x neighbour lies in the
// tile; kOddLinear, tiles of blockDim.x cells that may start mid-row.  HF: the y
// slots (HF = 1) are loaded without the nontemporal hint (tile_update_odd).
// Bitwise the same result as k_step's odd step.
template <int COLL, typename T, bool ZG, bool DIAG, bool NT, int MAP, bool SRC = false, int HF = 0>
__global__ void __launch_bounds__(1024) k_step_odd_tiles(T* __restrict__ F, Grid g, Coll c,
                                                          float* __restrict__ partials,
                                                          const float* __restrict__ src, uint32_t skey, int tl) {
  extern __shared__ float xs[];
  int n0, x = 0, y = 0, z = 0;
  bool act;
  if constexpr (MAP == kOddRow) {
    const int row = (int)blockIdx.x;
    n0 = row * g.px;
    act = (int)threadIdx.x < g.nx;
    z = row / g.ny;
    y = row - z * g.ny;
    if (act) x = (int)threadIdx.x;
  } else {
    n0 = (int)blockIdx.x * (MAP == kOddRowGroup ? tl : (int)blockDim.x);
    const int n = n0 + (int)threadIdx.x;
    act = n < g.px * g.ny * g.nz && (MAP != kOddRowGroup || (int)threadIdx.x < tl);
    if (act) {
      const int row = n / g.px;
      x = n - row * g.px;
      z = row / g.ny;
      y = row - z * g.ny;
      act = x < g.nx;  // the row's padding holds no cell
    }
  }
  float vals[kDiagVals];
  if constexpr (DIAG) {
#pragma unroll
    for (int j = 0; j < kDiagVals; ++j) vals[j] = 0.0f;
  }
  tile_update_odd<COLL, T, ZG, DIAG, NT, MAP == kOddLinear, SRC, HF>(F, g, c, n0, act, x, y, z, xs, vals, skey,
                                                                     src);
  if constexpr (DIAG) block_reduce_store(vals, partials);
}

// Odd AA step for FP16 storage with two consecutive cells per lane, one x-row per
// block (pair_row_update_odd, blockDim.x = nx / 2 <= 256); the rows for which
// odd_pairs holds.  Bitwise the same result as k_step_odd_tiles.
template <int COLL, bool ZG, bool DIAG, bool NT>
__global__ void __launch_bounds__(256) k_step_odd_row_pairs(_Float16* __restrict__ F, Grid g, Coll c,
                                                             float* __restrict__ partials, uint32_t skey) {
  extern __shared__ float xs[];
  const int row = (int)blockIdx.x;
  const int z = row / g.ny;
  const int y = row - z * g.ny;
  float vals[kDiagVals];
  if constexpr (DIAG) {
#pragma unroll
    for (int j = 0; j < kDiagVals; ++j) vals[j] = 0.0f;
  }
  pair_row_update_odd<COLL, ZG, DIAG, NT>(F, g, c, (int)threadIdx.x, y, z, xs, vals, skey);
  if constexpr (DIAG) block_reduce_store(vals, partials);
}

// One block of 1024 threads per value j: partials[nblocks][9] -> rec[j].  Each
// thread sums a fixed strided subset with compensated (Kahan) summation, then a
// fixed-order tree in LDS; the result does not depend on timing.
__global__ void __launch_bounds__(1024) k_finalize(const float* __restrict__ partials,
                                                    int64_t nblocks, float* __restrict__ rec) {
  __shared__ float sm[1024];
  const int j = blockIdx.x;
  float s = 0.0f, comp = 0.0f;
  for (int64_t b = threadIdx.x; b < nblocks; b += blockDim.x) {
    const float y = partials[b * kDiagVals + j] - comp;
    const float t = s + y;
    comp = (t - s) - y;
    s = t;
  }
  sm[threadIdx.x] = s;
  __syncthreads();
  for (int w = blockDim.x >> 1; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sm[threadIdx.x] += sm[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) rec[j] = sm[0];
}

// Largest |v| per field, as the bit pattern of a non-negative float (which orders
// like the value); the result does not depend on the order of the atomics.  The
// wave reduces first and issues one atomic per field: one atomic per cell on the
// same five words serialised and took 15 ms at 256^3.  Every lane of the wave must
// call it; lanes without a cell pass 0.  A NaN does not win the maximum.
__device__ __forceinline__ void wave_field_max(unsigned* maxabs, int k, float v) {
  float m = fabsf(v);
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off, 64));
  if ((threadIdx.x & 63) == 0) atomicMax(maxabs + k, __float_as_uint(m));
}

// Neighbour index along one axis for a central difference: periodic wrap, or the
// cell itself beyond a zero-gradient face (the ghost holds a copy of the cell).
__device__ __forceinline__ int64_t fd_neighbour(int64_t n, int x, int d, int len, int zg, int64_t stride) {
  int xx = x + d;
  if (xx < 0 || xx >= len) xx = zg ? x : (xx + len) % len;
  return n + (int64_t)(xx - x) * stride;
}

// Initial populations (the paper gives no initialisation): what a smooth field holds
// between two steps of the update, to first order.  Zeroth moment Q, second moment
// at equilibrium, first moment
//   J_k = Phi_adv,k + Phi_diff,k - (c_s^2 / omega_k) grad Q_k,
// the fixed point of the relaxation J* = Phi + (1 - omega)(J - Phi) followed by
// streaming, J = J* - c_s^2 grad Q.  grad Q comes from central differences of the
// initial fields, Phi_diff = (0, -tau, -tau u + q) from the Newtonian stress and
// Fourier flux of eq. 2 at that gradient (chain rule to grad u and grad T).  Without
// the non-equilibrium part the first streaming leaves J - Phi = -c_s^2 grad Q, omega
// times too large, and the difference oscillates from step to step undamped as
// omega -> 2.  Computed in FP64, stored as g_i = w_i (Q - Q_ref + 4 c_i . J) times
// the field's storage scale.  With ic.equilibrium (initial data with jumps, where a
// difference across a jump is no gradient) grad Q is taken as zero, which leaves
// the equilibrium of Q with the advective flux.  With mx set, nothing is stored and
// mx[k] receives the cell's largest |g| of field k (used to pick the FP16 scales).
template <typename T>
__device__ __forceinline__ void init_cell(T* __restrict__ F, const Grid& g, const Coll& c, const InitCoef& ic,
                                          const double* __restrict__ Q, int64_t N, int64_t n, float* mx) {
  const int64_t row = n / g.nx;
  const int x = (int)(n - row * g.nx);
  const int y = (int)(row % g.ny);
  const int z = (int)(row / g.ny);
  const int64_t plane = (int64_t)g.nx * g.ny;
  const int64_t ns = x + (int64_t)g.px * row;  // the cell's element in the padded rows
  const int64_t xm = fd_neighbour(n, x, -1, g.nx, g.zg_x, 1), xp = fd_neighbour(n, x, 1, g.nx, g.zg_x, 1);
  const int64_t ym = fd_neighbour(n, y, -1, g.ny, g.zg_y, g.nx), yp = fd_neighbour(n, y, 1, g.ny, g.zg_y, g.nx);
  const int64_t zm = fd_neighbour(n, z, -1, g.nz, g.zg_z, plane), zp = fd_neighbour(n, z, 1, g.nz, g.zg_z, plane);
  double q[5], G[5][3];
  for (int k = 0; k < 5; ++k) {
    const double* Qk = Q + k * N;
    q[k] = Qk[n];
    // the equilibrium start (data with jumps) takes no gradient
    G[k][0] = ic.equilibrium ? 0.0 : 0.5 * (Qk[xp] - Qk[xm]);
    G[k][1] = ic.equilibrium ? 0.0 : 0.5 * (Qk[yp] - Qk[ym]);
    G[k][2] = ic.equilibrium ? 0.0 : 0.5 * (Qk[zp] - Qk[zm]);
  }
  const double rf = fmax(q[0], ic.rho_min);
  const double u[3] = {q[1] / rf, q[2] / rf, q[3] / rf};
  const double k2 = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
  const double p = fmax(ic.gm1 * (q[4] - 0.5 * rf * k2), ic.p_min);
  const double Tc = p / rf;
  double ratio = 1.0;
  if (ic.sutherland) {
    const double t = Tc / ic.T_ref;
    ratio = (1.0 + ic.T_S) * t * sqrt(t) / (t + ic.T_S);
  }
  const double mu = ic.mu_ref * ratio, kap = ic.kappa_ref * ratio;
  // grad u = (grad(rho u) - u (x) grad rho)/rho and the chain rule for grad T
  double du[3][3], dT[3];
  for (int cc = 0; cc < 3; ++cc) {
    double um = 0.0;
    for (int j = 0; j < 3; ++j) {
      du[j][cc] = (G[1 + j][cc] - u[j] * G[0][cc]) / rf;
      um += u[j] * G[1 + j][cc];
    }
    dT[cc] = ic.gm1 / rf * (G[4][cc] - um) + (0.5 * ic.gm1 * k2 - Tc) / rf * G[0][cc];
  }
  const double theta = du[0][0] + du[1][1] + du[2][2];
  double tau[3][3];
  for (int j = 0; j < 3; ++j)
    for (int cc = 0; cc < 3; ++cc)
      tau[j][cc] = mu * (du[j][cc] + du[cc][j] - (j == cc ? 2.0 / 3.0 * theta : 0.0));
  double J[5][3];
  for (int cc = 0; cc < 3; ++cc) {
    J[0][cc] = q[1 + cc] - 0.25 * ic.inv_omega[0] * G[0][cc];
    for (int j = 0; j < 3; ++j)
      J[1 + j][cc] = q[1 + j] * u[cc] + (j == cc ? p : 0.0) - tau[j][cc] -
                     0.25 * ic.inv_omega[1 + j] * G[1 + j][cc];
    const double tu = tau[cc][0] * u[0] + tau[cc][1] * u[1] + tau[cc][2] * u[2];
    J[4][cc] = (q[4] + p) * u[cc] - tu - kap * dT[cc] - 0.25 * ic.inv_omega[4] * G[4][cc];
  }
  const double ref[5] = {ic.rho_ref, 0.0, 0.0, 0.0, ic.E_ref};
  for (int k = 0; k < 5; ++k) {
    const double dq = q[k] - ref[k];
    const double q8 = 0.125 * dq;
    const float v[7] = {(float)(0.25 * dq),           (float)(q8 + 0.5 * J[k][0]), (float)(q8 - 0.5 * J[k][0]),
                        (float)(q8 + 0.5 * J[k][1]), (float)(q8 - 0.5 * J[k][1]), (float)(q8 + 0.5 * J[k][2]),
                        (float)(q8 - 0.5 * J[k][2])};
    if (mx) {
      float m = 0.0f;
      for (int i = 0; i < kQ; ++i) m = fmaxf(m, fabsf(v[i]));
      mx[k] = m;
    } else {
      T* Fk = F + (int64_t)(7 * k) * g.S + ns;
      for (int i = 0; i < kQ; ++i) Fk[(int64_t)i * g.S] = static_cast<T>(v[i] * c.sc[k]);
    }
  }
}

// Largest |f| per field of a canonical population array f[35][N].
template <typename T>
__global__ void __launch_bounds__(256) k_init(T* __restrict__ F, Grid g, Coll c, InitCoef ic,
                                               const double* __restrict__ Q, int64_t N) {
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n < N) init_cell<T>(F, g, c, ic, Q, N, n, nullptr);
}

// The largest |g| of each field over the initial populations k_init would store,
// without storing them (picks the FP16 scales).  A fixed grid of at most 2048
// blocks strides over the cells, so the atomics number a few per wave and not
// one per wave of cells.
__global__ void __launch_bounds__(256) k_init_maxabs(Grid g, Coll c, InitCoef ic, const double* __restrict__ Q,
                                                      int64_t N, unsigned* __restrict__ maxabs) {
  float mx[kFields] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
  for (int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; n < N; n += (int64_t)gridDim.x * blockDim.x) {
    float m[kFields];
    init_cell<float>(nullptr, g, c, ic, Q, N, n, m);
#pragma unroll
    for (int k = 0; k < kFields; ++k) mx[k] = fmaxf(mx[k], m[k]);
  }
#pragma unroll
  for (int k = 0; k < kFields; ++k) wave_field_max(maxabs, k, mx[k]);
}

// The same over populations handed in by the caller (canonical layout, N cells).
__global__ void __launch_bounds__(256) k_maxabs_pops(const float* __restrict__ f, int64_t N,
                                                      unsigned* __restrict__ maxabs) {
  float mx[kFields] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
  for (int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; n < N; n += (int64_t)gridDim.x * blockDim.x) {
#pragma unroll
    for (int k = 0; k < kFields; ++k)
      for (int i = 0; i < kQ; ++i) mx[k] = fmaxf(mx[k], fabsf(f[(int64_t)(7 * k + i) * N + n]));
  }
#pragma unroll
  for (int k = 0; k < kFields; ++k) wave_field_max(maxabs, k, mx[k]);
}

// Element offset of canonical f_i of field k at the lane's cell for a state of
// the given parity.
template <typename T>
__device__ __forceinline__ int64_t canon_off(const Grid& g, const Nbr& b, int k, int i, bool odd) {
  const int64_t base = (int64_t)(7 * k) * g.S;
  if (!odd) return base + (int64_t)i * g.S + b.n;
  return base + odd_src<true>(g, b, i);
}

__device__ __forceinline__ void cell_of(const Grid& g, int64_t n, int& x, int& y, int& z) {
  x = (int)(n % g.nx);
  const int64_t r = n / g.nx;
  y = (int)(r % g.ny);
  z = (int)(r / g.ny);
}

// mode 0: canonical populations -> out_f[35][N] (float)
// mode 1: conserved moments Q_ref + sum_i g -> out_q[5][N] (double)
template <typename T>
__global__ void __launch_bounds__(256) k_gather(const T* __restrict__ F, Grid g, Coll c,
                                                 int64_t N, int odd, int mode,
                                                 float* __restrict__ out_f,
                                                 double* __restrict__ out_q) {
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  int x, y, z;
  cell_of(g, n, x, y, z);
  const Nbr b = make_nbr(g, x, y, z);
  for (int k = 0; k < 5; ++k) {
    float s = 0.0f;
    for (int i = 0; i < kQ; ++i) {
      const float v = static_cast<float>(F[canon_off<T>(g, b, k, i, odd != 0)]) * c.isc[k];
      if (mode == 0) out_f[(int64_t)(7 * k + i) * N + n] = v;
      s += v;
    }
    if (mode == 1) {
      const double ref = (k == 0) ? (double)c.rho_ref : (k == 4 ? (double)c.E_ref : 0.0);
      out_q[(int64_t)k * N + n] = ref + (double)s;
    }
  }
}

template <typename T>
__global__ void __launch_bounds__(256) k_scatter(T* __restrict__ F, Grid g, Coll c, int64_t N, int odd,
                                                  const float* __restrict__ in_f) {
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  int x, y, z;
  cell_of(g, n, x, y, z);
  const Nbr b = make_nbr(g, x, y, z);
  for (int k = 0; k < 5; ++k)
    for (int i = 0; i < kQ; ++i)
      F[canon_off<T>(g, b, k, i, odd != 0)] =
          static_cast<T>(in_f[(int64_t)(7 * k + i) * N + n] * c.sc[k]);
}

typedef float v4f __attribute__((ext_vector_type(4)));

// One 16-byte vector per lane, nontemporal in and out.
__global__ void __launch_bounds__(256) k_copy(const v4f* __restrict__ a, v4f* __restrict__ b,
                                               int64_t n4) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n4) __builtin_nontemporal_store(__builtin_nontemporal_load(&a[i]), &b[i]);
}

// ------------------------------------------------------------------ launchers
// `lds` bytes of dynamic LDS are reserved per block (and never touched): with 160 KB
// of LDS per CU this caps the resident blocks per CU, which the 35-stream access
// pattern prefers low (about 16 waves per CU).
template <int COLL, typename T, bool ZG, bool DIAG, bool NT, bool SRC, int HF>
static hipError_t launch_odd_tiles(const StepLaunch& L, const OddTiles& ot, hipStream_t s) {
  T* F = (T*)L.F;
  const dim3 grid((unsigned)ot.blocks), block(ot.block);
  if (ot.map == kOddRow)
    hipLaunchKernelGGL((k_step_odd_tiles<COLL, T, ZG, DIAG, NT, kOddRow, SRC, HF>), grid, block, ot.lds, s, F, L.g,
                       L.c, L.partials, L.src, L.skey, ot.tile);
  else if (ot.map == kOddRowGroup)
    hipLaunchKernelGGL((k_step_odd_tiles<COLL, T, ZG, DIAG, NT, kOddRowGroup, SRC, HF>), grid, block, ot.lds, s, F,
                       L.g, L.c, L.partials, L.src, L.skey, ot.tile);
  else
    hipLaunchKernelGGL((k_step_odd_tiles<COLL, T, ZG, DIAG, NT, kOddLinear, SRC, HF>), grid, block, ot.lds, s, F,
                       L.g, L.c, L.partials, L.src, L.skey, ot.tile);
  return hipGetLastError();
}

template <bool ODD, int COLL, typename T, bool ZG, bool DIAG, bool NT, bool SRC>
static hipError_t launch_step_nt(const StepLaunch& L, hipStream_t s) {
  const Grid& g = L.g;
  T* F = (T*)L.F;
  if constexpr (ODD && sizeof(T) == 2 && !SRC) {
    if (odd_pairs(L)) {
      hipLaunchKernelGGL((k_step_odd_row_pairs<COLL, ZG, DIAG, NT>), dim3((unsigned)((int64_t)g.ny * g.nz)),
                         dim3(g.nx / 2), odd_pair_lds(g), s, F, g, L.c, L.partials, L.skey);
      return hipGetLastError();
    }
  }
  if (ODD && L.odd_lds) {
    const OddTiles ot = odd_tiles(g, L.f16);
    if constexpr (NT) {
      if (ot.y_temporal) return launch_odd_tiles<COLL, T, ZG, DIAG, NT, SRC, 1>(L, ot, s);
    }
    return launch_odd_tiles<COLL, T, ZG, DIAG, NT, SRC, 0>(L, ot, s);
  }
  if constexpr (!ODD && sizeof(T) == 2 && !SRC) {
    if (even_pairs(L)) {
      hipLaunchKernelGGL((k_step_even_pairs<COLL, ZG, DIAG, NT>), dim3((unsigned)pair_blocks(L)), dim3(L.block),
                         L.lds, s, F, g, L.c, L.partials, L.skey);
      return hipGetLastError();
    }
  }
  const int64_t blocks = step_blocks(g, L.block);
  hipLaunchKernelGGL((k_step<ODD, COLL, T, ZG, DIAG, NT, SRC>), dim3((unsigned)blocks), dim3(L.block), L.lds, s,
                     F, g, L.c, L.partials, L.src, L.skey);
  return hipGetLastError();
}

// With a source only FP32 storage and nontemporal access are instantiated (the
// access mode never changes results; lbm_set_source rejects FP16 storage).
template <bool ODD, int COLL, typename T, bool ZG, bool DIAG, bool SRC>
static hipError_t launch_step_t(const StepLaunch& L, hipStream_t s) {
  if constexpr (SRC) {
    return launch_step_nt<ODD, COLL, T, ZG, DIAG, true, true>(L, s);
  } else {
    return L.nt ? launch_step_nt<ODD, COLL, T, ZG, DIAG, true, false>(L, s)
                : launch_step_nt<ODD, COLL, T, ZG, DIAG, false, false>(L, s);
  }
}

template <typename T, bool ZG, bool DIAG, bool SRC>
static hipError_t dispatch_odd_coll(const StepLaunch& L, hipStream_t s) {
  const bool odd = L.odd;
  if (L.coll == 0)
    return odd ? launch_step_t<true, 0, T, ZG, DIAG, SRC>(L, s) : launch_step_t<false, 0, T, ZG, DIAG, SRC>(L, s);
  return odd ? launch_step_t<true, 1, T, ZG, DIAG, SRC>(L, s) : launch_step_t<false, 1, T, ZG, DIAG, SRC>(L, s);
}

template <typename T, bool SRC>
static hipError_t dispatch_t(const StepLaunch& L, hipStream_t s) {
  const bool zg = L.g.zg_x || L.g.zg_y || L.g.zg_z;
  if (zg)
    return L.diag ? dispatch_odd_coll<T, true, true, SRC>(L, s) : dispatch_odd_coll<T, true, false, SRC>(L, s);
  return L.diag ? dispatch_odd_coll<T, false, true, SRC>(L, s) : dispatch_odd_coll<T, false, false, SRC>(L, s);
}

hipError_t launch_step(const StepLaunch& L, hipStream_t s) {
  if (L.f16) {
    if (L.src) return hipErrorInvalidValue;  // rejected earlier by lbm_set_source
    return dispatch_t<_Float16, false>(L, s);
  }
  return L.src ? dispatch_t<float, true>(L, s) : dispatch_t<float, false>(L, s);
}

int64_t step_blocks(const Grid& g, int block) { return (row_cells(g) + block - 1) / block; }

// Whole x-rows per k_step_odd_tiles block where rows of nx cells (no padding) leave
// the last wave of a one-row block partly idle: the fewest rows R whose R * nx cells
// fill whole waves, up to kMaxGroupTile cells (FP16: only R = 2); 0 if there is none.
int odd_group_rows(const Grid& g, bool f16) {
  if (g.nx % 64 == 0 || g.px != g.nx || g.nx > kMaxGroupTile) return 0;
  for (int r = 2; r * g.nx <= kMaxGroupTile && (r == 2 || !f16); ++r)
    if (r * g.nx % 64 == 0) return r;
  return 0;
}

// Launch shape of k_step_odd_tiles, from continuous-run A/B timing on MI355X (two
// alternating runs, cubes of 48-288).  Rows that a few whole rows fill exactly
// (odd_group_rows) take blocks of whole rows: FP32 48-160 cells +1% to +5%, FP16
// 96-224 cells (two rows) +3.5% to +6%, against the mappings below; FP16 blocks of
// four rows of 48 or 80 cells lost 3-14%.  Other rows of a multiple of 32 cells
// (FP16: 64) up to 1024 take one block per row, with no index division and no tile
// edge; the rest take linear tiles, which also beat larger blocks of whole rows (4
// or 5 rows of 144-200 cells: FP32 -4% to +2.4%, FP16 -5% to -15%).  The dynamic
// LDS holds the two x slots of a tile and a sink column (15 floats per cell), padded
// to cap the resident waves per CU where the odd step's sustained bandwidth peaked:
// FP32 row blocks at 8 waves per CU, the rest at 16 (FP16 keeps fewer bytes in
// flight per wave).
OddTiles odd_tiles(const Grid& g, bool f16) {
  OddTiles t;
  const int rows = odd_group_rows(g, f16);
  if (rows > 0) {
    t.map = kOddRowGroup;
    t.tile = rows * g.px;
    t.block = t.tile;
    t.blocks = ((int64_t)g.ny * g.nz + rows - 1) / rows;
  } else if (g.nx <= kMaxRowTile && g.nx % (f16 ? kRowMultipleF16 : kRowMultipleF32) == 0) {
    t.map = kOddRow;
    t.tile = g.px;
    t.block = (g.nx + 63) / 64 * 64;
    t.blocks = (int64_t)g.ny * g.nz;
  } else {
    t.map = kOddLinear;
    t.tile = f16 ? kOddTileF16 : kOddTileF32;
    t.block = t.tile;
    t.blocks = (row_cells(g) + t.tile - 1) / t.tile;
  }
  t.y_temporal = (int64_t)g.px * (f16 ? 2 : 4) % 128 != 0;
  const int waves = (t.map == kOddRow && !f16) ? 8 : 16;
  const int need = 15 * (int)sizeof(float) * t.block;
  const int per_cu = waves * 64 / t.block > 1 ? waves * 64 / t.block : 1;
  int lds = (int)(kLdsPerCU / (per_cu + 1)) + 256;
  if (lds > 65536) lds = 65536;
  t.lds = lds > need ? lds : need;
  return t;
}

bool even_pairs(const StepLaunch& L) {
  // measured: +3% at 256^3 and +4% at 384^3, but -8% at 128^3 (its two cells per
  // lane take about 190 registers, so fewer waves hide the latency)
  const int64_t N = (int64_t)L.g.nx * L.g.ny * L.g.nz;
  return !L.odd && L.f16 && !L.src && L.block <= 256 && L.g.nx % 2 == 0 && L.g.px % 2 == 0 &&
         N >= kPairMinCells;
}

bool odd_pairs(const StepLaunch& L) {
  // measured against k_step_odd_tiles: +6-9% at 384^3 and +5% at 512^3; -3% at 256^3
  // (one 128-lane block per row; two rows per block did worse), and nothing at 768^3
  // or 1024^3 (512-lane blocks)
  const int64_t N = (int64_t)L.g.nx * L.g.ny * L.g.nz;
  const int nx = L.g.nx;
  return L.odd && L.odd_lds && L.f16 && !L.src && nx % kRowMultipleOddPairs == 0 && nx >= kMinRowPairs &&
         nx <= kMaxRowPairs && N >= kPairMinCells;
}

int odd_pair_lds(const Grid& g) { return 15 * (int)sizeof(float) * g.nx; }

int64_t pair_blocks(const StepLaunch& L) {
  const int64_t pairs = row_cells(L.g) / 2;
  return (pairs + L.block - 1) / L.block;
}

int64_t launch_blocks(const StepLaunch& L) {
  if (odd_pairs(L)) return (int64_t)L.g.ny * L.g.nz;
  if (L.odd && L.odd_lds) return odd_tiles(L.g, L.f16).blocks;
  return even_pairs(L) ? pair_blocks(L) : step_blocks(L.g, L.block);
}

hipError_t launch_finalize(const float* partials, int64_t nblocks, float* rec, hipStream_t s) {
  hipLaunchKernelGGL(k_finalize, dim3(kDiagVals), dim3(1024), 0, s, partials, nblocks, rec);
  return hipGetLastError();
}

hipError_t launch_init(void* F, bool f16, const Grid& g, const Coll& c, const InitCoef& ic, const double* Q,
                       int64_t N, hipStream_t s) {
  const unsigned blocks = (unsigned)((N + 255) / 256);
  if (f16)
    hipLaunchKernelGGL(k_init<_Float16>, dim3(blocks), dim3(256), 0, s, (_Float16*)F, g, c, ic, Q, N);
  else
    hipLaunchKernelGGL(k_init<float>, dim3(blocks), dim3(256), 0, s, (float*)F, g, c, ic, Q, N);
  return hipGetLastError();
}

// Blocks of the striding max-abs reductions: 8 per CU, a few thousand atomics.
static unsigned maxabs_blocks(int64_t N) {
  const int64_t b = (N + 255) / 256;
  return (unsigned)(b < 2048 ? (b > 0 ? b : 1) : 2048);
}

hipError_t launch_init_maxabs(const Grid& g, const Coll& c, const InitCoef& ic, const double* Q, int64_t N,
                              unsigned* maxabs, hipStream_t s) {
  hipLaunchKernelGGL(k_init_maxabs, dim3(maxabs_blocks(N)), dim3(256), 0, s, g, c, ic, Q, N, maxabs);
  return hipGetLastError();
}

hipError_t launch_maxabs_pops(const float* f, int64_t N, unsigned* maxabs, hipStream_t s) {
  hipLaunchKernelGGL(k_maxabs_pops, dim3(maxabs_blocks(N)), dim3(256), 0, s, f, N, maxabs);
  return hipGetLastError();
}

hipError_t launch_gather(const void* F, bool f16, const Grid& g, const Coll& c, int64_t N, bool odd,
                         int mode, float* out_f, double* out_q, hipStream_t s) {
  const unsigned blocks = (unsigned)((N + 255) / 256);
  if (f16)
    hipLaunchKernelGGL(k_gather<_Float16>, dim3(blocks), dim3(256), 0, s, (const _Float16*)F, g, c, N,
                       (int)odd, mode, out_f, out_q);
  else
    hipLaunchKernelGGL(k_gather<float>, dim3(blocks), dim3(256), 0, s, (const float*)F, g, c, N,
                       (int)odd, mode, out_f, out_q);
  return hipGetLastError();
}

hipError_t launch_scatter(void* F, bool f16, const Grid& g, const Coll& c, int64_t N, bool odd,
                          const float* in_f, hipStream_t s) {
  const unsigned blocks = (unsigned)((N + 255) / 256);
  if (f16)
    hipLaunchKernelGGL(k_scatter<_Float16>, dim3(blocks), dim3(256), 0, s, (_Float16*)F, g, c, N, (int)odd,
                       in_f);
  else
    hipLaunchKernelGGL(k_scatter<float>, dim3(blocks), dim3(256), 0, s, (float*)F, g, c, N, (int)odd, in_f);
  return hipGetLastError();
}

hipError_t launch_copy(const void* a, void* b, int64_t bytes, hipStream_t s) {
  const int64_t n4 = bytes / 16;
  const unsigned blocks = (unsigned)((n4 + 255) / 256);
  hipLaunchKernelGGL(k_copy, dim3(blocks), dim3(256), 0, s, (const v4f*)a, (v4f*)b, n4);
  return hipGetLastError();
}

}  // namespace grlbm
