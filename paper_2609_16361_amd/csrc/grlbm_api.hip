// grlbm_api.hip -- the C ABI of include/grlbm.h: validation, device memory,
// stream binding, step scheduling and the diagnostic record queue.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <deque>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/grlbm.h"
#include "grlbm_internal.h"

using grlbm::Coll;
using grlbm::Grid;
using grlbm::fail;

namespace grlbm {

thread_local std::string g_err;

lbm_status fail(lbm_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return st;
}

static bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

lbm_status validate(const lbm_params* p) {
  if (!p) return fail(LBM_EINVAL, "params is NULL");
  if (p->nx < 1 || p->ny < 1 || p->nz < 1)
    return fail(LBM_EINVAL, "dims must be >= 1 (got %d x %d x %d)", p->nx, p->ny, p->nz);
  const int32_t dims[3] = {p->nx, p->ny, p->nz};
  for (int a = 0; a < 3; ++a) {
    if (p->bc[a] != LBM_BC_PERIODIC && p->bc[a] != LBM_BC_ZERO_GRADIENT)
      return fail(LBM_EINVAL, "bc[%d] = %d is not an lbm_bc", a, p->bc[a]);
    if (p->bc[a] == LBM_BC_ZERO_GRADIENT && dims[a] < 2)
      return fail(LBM_EINVAL, "zero-gradient axis %d needs >= 2 cells (got %d)", a, dims[a]);
  }
  if (p->collision != LBM_COLL_RLB_SENSOR && p->collision != LBM_COLL_BGK)
    return fail(LBM_EINVAL, "collision = %d is not an lbm_collision", p->collision);
  if (p->storage != LBM_STORE_F32 && p->storage != LBM_STORE_F16)
    return fail(LBM_EINVAL, "storage = %d is not an lbm_storage", p->storage);
  // the step kernels index array elements in 32 bits, and a tile's end (its first
  // element plus up to 1024) must stay representable: grids whose padded rows span
  // up to 2^31 - 2^16 elements (about 1290^3)
  const int64_t NE = row_pitch(p) * p->ny * p->nz;
  if (NE > (int64_t)INT32_MAX - 65535)
    return fail(LBM_EINVAL, "grid of %lld elements exceeds the 32-bit index range", (long long)NE);
  if (p->mu_law != LBM_MU_CONSTANT && p->mu_law != LBM_MU_SUTHERLAND)
    return fail(LBM_EINVAL, "mu_law = %d is not an lbm_mu_law", p->mu_law);
  if (p->layout_pad < 0) return fail(LBM_EINVAL, "layout_pad must be >= 0");
  if (p->start != LBM_START_FIRST_ORDER && p->start != LBM_START_EQUILIBRIUM)
    return fail(LBM_EINVAL, "start = %d is not an lbm_start", p->start);
  if (!finite_pos(p->gamma - 1.0)) return fail(LBM_EINVAL, "gamma must be finite and > 1");
  if (!(std::isfinite(p->mu_ref) && p->mu_ref >= 0.0)) return fail(LBM_EINVAL, "mu_ref must be >= 0");
  if (!(std::isfinite(p->kappa_ref) && p->kappa_ref >= 0.0))
    return fail(LBM_EINVAL, "kappa_ref must be >= 0");
  if (p->mu_law == LBM_MU_SUTHERLAND) {
    if (!finite_pos(p->T_ref)) return fail(LBM_EINVAL, "T_ref must be > 0");
    if (!(std::isfinite(p->T_S) && p->T_S >= 0.0)) return fail(LBM_EINVAL, "T_S must be >= 0");
  }
  for (int k = 0; k < 5; ++k)
    if (!(std::isfinite(p->omega[k]) && p->omega[k] > 0.0 && p->omega[k] <= 2.0))
      return fail(LBM_EINVAL, "omega[%d] = %g outside (0, 2]", k, p->omega[k]);
  if (p->omega[1] != p->omega[2] || p->omega[1] != p->omega[3])
    return fail(LBM_EINVAL, "the three momentum relaxation frequencies must be equal");
  if (!(std::isfinite(p->sensor_gain) && p->sensor_gain >= 0.0))
    return fail(LBM_EINVAL, "sensor_gain must be >= 0");
  if (!std::isfinite(p->J_min)) return fail(LBM_EINVAL, "J_min must be finite");
  if (!(std::isfinite(p->omega_min) && p->omega_min > 0.0 && p->omega_min <= 2.0))
    return fail(LBM_EINVAL, "omega_min outside (0, 2]");
  if (!finite_pos(p->rho_min)) return fail(LBM_EINVAL, "rho_min must be > 0");
  if (!(std::isfinite(p->p_min) && p->p_min >= 0.0)) return fail(LBM_EINVAL, "p_min must be >= 0");
  if (!std::isfinite(p->rho_ref) || !std::isfinite(p->E_ref))
    return fail(LBM_EINVAL, "rho_ref and E_ref must be finite");
  return LBM_OK;
}

lbm_status check_fields(const lbm_params* p, const double* Q) {
  const int64_t N = (int64_t)p->nx * p->ny * p->nz;
  const double g1 = p->gamma - 1.0;
  for (int64_t n = 0; n < N; ++n) {
    const double rho = Q[n], m0 = Q[N + n], m1 = Q[2 * N + n], m2 = Q[3 * N + n], E = Q[4 * N + n];
    if (!(std::isfinite(rho) && std::isfinite(m0) && std::isfinite(m1) && std::isfinite(m2) && std::isfinite(E)))
      return fail(LBM_EINVAL, "initial fields are not finite at cell %lld", (long long)n);
    if (!(rho > 0.0)) return fail(LBM_EINVAL, "initial density %g at cell %lld is not positive", rho, (long long)n);
    const double pr = g1 * (E - 0.5 * (m0 * m0 + m1 * m1 + m2 * m2) / rho);
    if (!(pr > 0.0)) return fail(LBM_EINVAL, "initial pressure %g at cell %lld is not positive", pr, (long long)n);
  }
  return LBM_OK;
}

int64_t row_pitch(const lbm_params* p) {
  // rows padded to whole 128-byte lines when the padding is at most a sixteenth of
  // the row (a grid of one row has no +-y or +-z neighbours to align) ...
  const int64_t nx = p->nx;
  if ((int64_t)p->ny * p->nz == 1) return nx;
  const int64_t line = p->storage == LBM_STORE_F16 ? 64 : 32;
  const int64_t px = (nx + line - 1) / line * line;
  // ... and never where the padding alone would leave the 32-bit index range
  if (16 * (px - nx) > nx || px * p->ny * p->nz > (int64_t)INT32_MAX - 65535) return nx;
  return px;
}

int64_t slot_stride(const lbm_params* p) {
  const int64_t N = row_pitch(p) * p->ny * p->nz;
  const int64_t el = p->storage == LBM_STORE_F16 ? 2 : 4;
  const int64_t align = 256 / el;  // arrays start on 256-byte boundaries
  const int64_t s = N + p->layout_pad;
  return (s + align - 1) / align * align;
}

size_t state_bytes(const lbm_params* p) {
  const int64_t el = p->storage == LBM_STORE_F16 ? 2 : 4;
  return (size_t)(slot_stride(p) * 35 * el);
}

Coll make_coll(const lbm_params* p) {
  Coll c;
  c.om[0] = (float)p->omega[0];
  c.om[1] = (float)p->omega[1];
  c.om[2] = (float)p->omega[4];
  c.gm1 = (float)(p->gamma - 1.0);
  c.mu_ref = (float)p->mu_ref;
  c.kappa_ref = (float)p->kappa_ref;
  c.suth_c = (float)(1.0 + p->T_S);
  c.inv_T_ref = p->T_ref > 0.0 ? (float)(1.0 / p->T_ref) : 0.0f;
  c.T_S = (float)p->T_S;
  c.gain = (float)p->sensor_gain;
  c.J_min = (float)p->J_min;
  c.om_min = (float)p->omega_min;
  c.rho_min = (float)p->rho_min;
  c.p_min = (float)p->p_min;
  c.rho_ref = (float)p->rho_ref;
  c.E_ref = (float)p->E_ref;
  c.sutherland = p->mu_law == LBM_MU_SUTHERLAND ? 1 : 0;
  for (int k = 0; k < 5; ++k) c.sc[k] = c.isc[k] = 1.0f;
  return c;
}

void set_storage_scales(Coll& c, const unsigned maxabs_bits[5]) {
  float mx[5], top = 0.0f;
  for (int k = 0; k < 5; ++k) {
    std::memcpy(&mx[k], &maxabs_bits[k], sizeof(float));
    if (!(mx[k] < 3.0e38f)) mx[k] = 0.0f;  // non-finite input: leave it unscaled
    top = std::max(top, mx[k]);
  }
  for (int k = 0; k < 5; ++k) {
    // a field that is identically zero takes its scale from the largest field
    const float m = std::max(mx[k], 1e-3f * top);
    int e = 0;
    if (m > 0.0f) {
      std::frexp(m, &e);  // m = f * 2^e, f in [0.5, 1)
      e = 6 - e;          // m * 2^e in [32, 64)
      e = std::min(std::max(e, -100), 100);
    }
    c.sc[k] = std::ldexp(1.0f, e);
    c.isc[k] = std::ldexp(1.0f, -e);
  }
}

static lbm_status read_maxabs(Coll& c, unsigned* d, hipStream_t s) {
  unsigned h[5];
  HIP_TRY(hipMemcpyAsync(h, d, sizeof h, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  set_storage_scales(c, h);
  return LBM_OK;
}

InitCoef make_init_coef(const lbm_params* p) {
  InitCoef ic;
  ic.gm1 = p->gamma - 1.0;
  ic.mu_ref = p->mu_ref;
  ic.kappa_ref = p->kappa_ref;
  ic.T_ref = p->T_ref;
  ic.T_S = p->T_S;
  ic.rho_min = p->rho_min;
  ic.p_min = p->p_min;
  ic.rho_ref = p->rho_ref;
  ic.E_ref = p->E_ref;
  for (int k = 0; k < 5; ++k) ic.inv_omega[k] = 1.0 / p->omega[k];
  ic.sutherland = p->mu_law == LBM_MU_SUTHERLAND ? 1 : 0;
  ic.equilibrium = p->start == LBM_START_EQUILIBRIUM ? 1 : 0;
  return ic;
}

lbm_status scales_from_fields(Coll& c, const Grid& g, const InitCoef& ic, const double* Q_dev, int64_t N,
                              hipStream_t s) {
  unsigned* d = nullptr;
  if (hipMalloc((void**)&d, 5 * sizeof(unsigned)) != hipSuccess) return fail(LBM_ENOMEM, "hipMalloc failed");
  lbm_status st = LBM_OK;
  if (hipMemsetAsync(d, 0, 5 * sizeof(unsigned), s) != hipSuccess ||
      launch_init_maxabs(g, c, ic, Q_dev, N, d, s) != hipSuccess)
    st = fail(LBM_EDEVICE, "storage-scale reduction failed");
  if (st == LBM_OK) st = read_maxabs(c, d, s);
  (void)hipFree(d);
  return st;
}

lbm_status scales_from_pops(Coll& c, const float* f_dev, int64_t N, hipStream_t s) {
  unsigned* d = nullptr;
  if (hipMalloc((void**)&d, 5 * sizeof(unsigned)) != hipSuccess) return fail(LBM_ENOMEM, "hipMalloc failed");
  lbm_status st = LBM_OK;
  if (hipMemsetAsync(d, 0, 5 * sizeof(unsigned), s) != hipSuccess || launch_maxabs_pops(f_dev, N, d, s) != hipSuccess)
    st = fail(LBM_EDEVICE, "storage-scale reduction failed");
  if (st == LBM_OK) st = read_maxabs(c, d, s);
  (void)hipFree(d);
  return st;
}

Grid make_grid(const lbm_params* p) {
  Grid g;
  g.nx = p->nx;
  g.ny = p->ny;
  g.nz = p->nz;
  g.zg_x = p->bc[0] == LBM_BC_ZERO_GRADIENT;
  g.zg_y = p->bc[1] == LBM_BC_ZERO_GRADIENT;
  g.zg_z = p->bc[2] == LBM_BC_ZERO_GRADIENT;
  g.S = slot_stride(p);
  g.px = (int32_t)row_pitch(p);
  g.pad_ = 0;
  return g;
}

}  // namespace grlbm

using grlbm::make_coll;
using grlbm::make_grid;
using grlbm::slot_stride;
using grlbm::state_bytes;
using grlbm::validate;

namespace {

constexpr int kDiagVals = 9;
constexpr int32_t kRingCap = 1024;
constexpr int kDefaultBlocksPerCuF32 = 4;

// Nontemporal access is the default except for states of kNtOffMin up to kNtOffMax
// bytes, about the size of the 256 MB Infinity Cache, which keeps part of such a
// state between steps unless the hint evicts it.  Measured on MI355X over cubes
// (GLUP/s without / with the hint, each storage's default occupancy cap): FP32 64^3
// (37 MB) 18.7 / 16.0, 96^3 (124 MB) 23.5 / 18.2, 128^3 (294 MB) 21.1 / 20.1, but
// 136^3 (352 MB) 19.0 / 20.1 and 48^3 (15 MB) 9.9 / 10.6; FP16 72^3 (26 MB) 29.1 /
// 26.7, 128^3 (147 MB) 44.8 / 37.7, 144^3 (209 MB) 41.2 / 35.6, 160^3 (287 MB) 37.1
// / 37.3, but 192^3 (495 MB) 37.1 / 39.8 and 64^3 (18 MB) 19.0 / 23.2.
constexpr int64_t kNtOffMin = 24ll << 20;
constexpr int64_t kNtOffMax = 320ll << 20;
bool default_nontemporal(int64_t state_bytes) { return state_bytes < kNtOffMin || state_bytes >= kNtOffMax; }

}  // namespace

struct lbm_ctx {
  lbm_params p{};
  Grid g{};
  Coll c{};
  int64_t N = 0;
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  void* F = nullptr;
  size_t F_bytes = 0;
  bool own_F = false;
  int64_t step = 0;
  bool ready = false;
  int block = 256;
  bool nt = true;
  int bpc = 0;  // occupancy cap of the even step (0 = none), enforced through lds
  int lds = 0;
  bool odd_lds = true;
  const float* src = nullptr;  // caller-owned source of eq. 1, [5][N] FP32, or nullptr
  float* partials = nullptr;
  int64_t partials_blocks = 0;
  float* ring = nullptr;
  int32_t ring_used = 0;
  std::vector<int64_t> ring_steps;
  std::deque<lbm_diag> done;
};

namespace {

// LDS reserved per block so that at most blocks_per_cu blocks are resident per CU:
// just over 1/(blocks_per_cu + 1) of the 160 KB of a CU (0 = no cap).
int lds_for_blocks_per_cu(int blocks_per_cu) {
  if (blocks_per_cu <= 0) return 0;
  const int lds = (int)(grlbm::kLdsPerCU / (blocks_per_cu + 1)) + 256;
  return lds > 65536 ? 65536 : lds;
}

lbm_status ensure_partials(lbm_ctx* c) {
  // partials for the larger of the two launch shapes (even step, LDS odd step)
  const int64_t nb = std::max(grlbm::step_blocks(c->g, c->block),
                              grlbm::odd_tiles(c->g, c->p.storage == LBM_STORE_F16).blocks);
  if (nb <= c->partials_blocks) return LBM_OK;
  if (c->partials) HIP_TRY(hipFree(c->partials));
  c->partials = nullptr;
  c->partials_blocks = 0;
  if (hipMalloc(&c->partials, (size_t)nb * kDiagVals * sizeof(float)) != hipSuccess)
    return fail(LBM_ENOMEM, "hipMalloc of %lld diagnostic partials failed", (long long)nb);
  c->partials_blocks = nb;
  return LBM_OK;
}

lbm_status drain_ring(lbm_ctx* c) {
  if (c->ring_used == 0) return LBM_OK;
  std::vector<float> h((size_t)c->ring_used * kDiagVals);
  HIP_TRY(hipMemcpyAsync(h.data(), c->ring, h.size() * sizeof(float), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  for (int32_t r = 0; r < c->ring_used; ++r) {
    const float* v = &h[(size_t)r * kDiagVals];
    lbm_diag d{};
    d.step = c->ring_steps[r];
    d.Ek = v[0];
    d.eps_s = v[1];
    d.eps_d = v[2];
    for (int k = 0; k < 5; ++k) d.dtotal[k] = v[3 + k];
    d.nonfinite = (int64_t)std::llround((double)v[8]);
    c->done.push_back(d);
  }
  c->ring_used = 0;
  c->ring_steps.clear();
  return LBM_OK;
}

lbm_status create_common(const lbm_params* p, void* buf, size_t bytes, void* stream, lbm_ctx** out) {
  if (!out) return fail(LBM_EINVAL, "out is NULL");
  *out = nullptr;
  lbm_status st = validate(p);
  if (st != LBM_OK) return st;
  lbm_ctx* c = new (std::nothrow) lbm_ctx();
  if (!c) return fail(LBM_ENOMEM, "host allocation of the context failed");
  c->p = *p;
  c->N = (int64_t)p->nx * p->ny * p->nz;
  c->g = make_grid(p);
  c->c = make_coll(p);
  c->F_bytes = state_bytes(p);
  // Default launch of the even step: 256-thread blocks; FP32 capped at 4 resident
  // blocks (16 waves) per CU, FP16 (two-byte loads keep fewer bytes in flight per
  // wave) uncapped -- the fastest shapes in continuous-run A/B timing on MI355X for
  // both short (256-cell) and long (1024- and 4096-cell) rows.
  c->block = 256;
  c->nt = default_nontemporal((int64_t)c->F_bytes);
  c->bpc = p->storage == LBM_STORE_F16 ? 0 : kDefaultBlocksPerCuF32;
  c->lds = lds_for_blocks_per_cu(c->bpc);
  auto bail = [&](lbm_status s) {
    lbm_destroy(c);
    return s;
  };
  if (hipGetDevice(&c->device) != hipSuccess) return bail(fail(LBM_EDEVICE, "no HIP device"));
  if (stream) {
    c->stream = (hipStream_t)stream;
  } else {
    if (hipStreamCreate(&c->stream) != hipSuccess) return bail(fail(LBM_EDEVICE, "hipStreamCreate failed"));
    c->own_stream = true;
  }
  if (buf) {
    if (bytes < c->F_bytes)
      return bail(fail(LBM_EINVAL, "buffer of %zu bytes is smaller than the %zu the state needs", bytes,
                       c->F_bytes));
    if (((uintptr_t)buf) % 256 != 0) return bail(fail(LBM_EINVAL, "buffer is not 256-byte aligned"));
    c->F = buf;
  } else {
    if (hipMalloc(&c->F, c->F_bytes) != hipSuccess)
      return bail(fail(LBM_ENOMEM, "hipMalloc of %zu population bytes failed", c->F_bytes));
    c->own_F = true;
  }
  if (hipMalloc(&c->ring, (size_t)kRingCap * kDiagVals * sizeof(float)) != hipSuccess)
    return bail(fail(LBM_ENOMEM, "hipMalloc of the diagnostic ring failed"));
  c->ring_steps.reserve(kRingCap);
  *out = c;
  return LBM_OK;
}

template <typename T>
lbm_status dev_alloc(T** p, size_t count, const char* what) {
  if (hipMalloc((void**)p, count * sizeof(T)) != hipSuccess)
    return fail(LBM_ENOMEM, "hipMalloc of %zu bytes (%s) failed", count * sizeof(T), what);
  return LBM_OK;
}

}  // namespace

extern "C" {

size_t lbm_state_bytes(const lbm_params* p) {
  if (validate(p) != LBM_OK) return 0;
  return state_bytes(p);
}

lbm_status lbm_create(const lbm_params* p, void* hip_stream, lbm_ctx** out) {
  return create_common(p, nullptr, 0, hip_stream, out);
}

lbm_status lbm_create_in(const lbm_params* p, void* dev_buf, size_t bytes, void* hip_stream,
                         lbm_ctx** out) {
  if (!dev_buf) {
    if (out) *out = nullptr;
    return fail(LBM_EINVAL, "dev_buf is NULL");
  }
  return create_common(p, dev_buf, bytes, hip_stream, out);
}

lbm_status lbm_set_launch(lbm_ctx* c, int32_t block, int32_t nontemporal, int32_t blocks_per_cu,
                          int32_t odd_lds) {
  if (!c) return fail(LBM_EINVAL, "ctx is NULL");
  if (odd_lds != 0 && odd_lds != 1) return fail(LBM_EINVAL, "odd_lds = %d must be 0 or 1", odd_lds);
  if (block < 64 || block > 1024 || block % 64 != 0)
    return fail(LBM_EINVAL, "block = %d must be a multiple of 64 in [64, 1024]", block);
  if (blocks_per_cu < 0 || blocks_per_cu > 32)
    return fail(LBM_EINVAL, "blocks_per_cu = %d outside [0, 32]", blocks_per_cu);
  c->block = block;
  c->nt = nontemporal != 0;
  c->odd_lds = odd_lds != 0;
  c->bpc = blocks_per_cu;
  c->lds = lds_for_blocks_per_cu(blocks_per_cu);
  return LBM_OK;
}

lbm_status lbm_get_launch(lbm_ctx* c, lbm_launch* out) {
  if (!c || !out) return fail(LBM_EINVAL, "NULL argument");
  out->block = c->block;
  out->nontemporal = c->nt ? 1 : 0;
  out->blocks_per_cu = c->bpc;
  out->odd_lds = c->odd_lds ? 1 : 0;
  return LBM_OK;
}

lbm_status lbm_autotune(lbm_ctx* c, int32_t trial_steps, lbm_launch* best, float* best_us, lbm_launch* tried,
                        float* tried_us, int32_t max_tried, int32_t* ntried) {
  if (!c || !best) return fail(LBM_EINVAL, "NULL argument");
  if (trial_steps < 2) return fail(LBM_EINVAL, "trial_steps must be >= 2");
  if (!c->ready) return fail(LBM_ESTATE, "lbm_autotune before lbm_init_fields or lbm_set_populations");
  if (ntried) *ntried = 0;
  trial_steps += trial_steps & 1;  // whole even/odd pairs
  // the trials advance the state; a device copy puts it back after each
  void* snap = nullptr;
  if (hipMalloc(&snap, c->F_bytes) != hipSuccess) {
    (void)hipGetLastError();
    return fail(LBM_ENOMEM, "snapshot of %zu bytes for autotuning failed", c->F_bytes);
  }
  HIP_TRY(hipMemcpyAsync(snap, c->F, c->F_bytes, hipMemcpyDeviceToDevice, c->stream));
  lbm_launch orig{};
  (void)lbm_get_launch(c, &orig);
  const int64_t step0 = c->step;
  // (threads per block, blocks per CU) of the even step, each with and without
  // nontemporal access; the odd step keeps its own shape
  static const int shapes[][2] = {{256, 4}, {256, 2}, {256, 0}, {512, 2}, {512, 0}, {1024, 0}};
  std::vector<lbm_launch> cands;
  for (int nt : {1, 0})
    for (const auto& sh : shapes) {
      lbm_launch t{};
      t.block = sh[0];
      t.nontemporal = nt;
      t.blocks_per_cu = sh[1];
      t.odd_lds = 1;
      cands.push_back(t);
    }
  hipEvent_t e0 = nullptr, e1 = nullptr;
  lbm_status st = LBM_OK;
  float best_time = 1e30f;
  lbm_launch best_t = orig;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
    st = fail(LBM_EDEVICE, "event creation failed");
  for (size_t ci = 0; st == LBM_OK && ci < cands.size(); ++ci) {
    const lbm_launch& t = cands[ci];
    st = lbm_set_launch(c, t.block, t.nontemporal, t.blocks_per_cu, t.odd_lds);
    if (st == LBM_OK) st = lbm_step(c, 2, 0);  // warm-up pair
    if (st != LBM_OK) break;
    float ms = 0.0f;
    if (hipEventRecord(e0, c->stream) != hipSuccess) {
      st = fail(LBM_EDEVICE, "event record failed");
      break;
    }
    st = lbm_step(c, trial_steps, 0);
    if (st != LBM_OK) break;
    if (hipEventRecord(e1, c->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
        hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
      st = fail(LBM_EDEVICE, "trial timing failed");
      break;
    }
    const float us = ms * 1000.0f / trial_steps;
    if (tried && ntried && *ntried < max_tried) {
      tried[*ntried] = t;
      if (tried_us) tried_us[*ntried] = us;
      ++*ntried;
    }
    if (us < best_time) {
      best_time = us;
      best_t = t;
    }
    if (hipMemcpyAsync(c->F, snap, c->F_bytes, hipMemcpyDeviceToDevice, c->stream) != hipSuccess) {
      st = fail(LBM_EDEVICE, "snapshot restore failed");
      break;
    }
    c->step = step0;
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  // the state must be back before the snapshot goes, whatever happened above
  if (hipMemcpyAsync(c->F, snap, c->F_bytes, hipMemcpyDeviceToDevice, c->stream) != hipSuccess ||
      hipStreamSynchronize(c->stream) != hipSuccess) {
    if (st == LBM_OK) st = fail(LBM_EDEVICE, "snapshot restore failed");
  }
  c->step = step0;
  (void)hipFree(snap);
  if (st != LBM_OK) {
    (void)lbm_set_launch(c, orig.block, orig.nontemporal, orig.blocks_per_cu, orig.odd_lds);
    return st;
  }
  st = lbm_set_launch(c, best_t.block, best_t.nontemporal, best_t.blocks_per_cu, best_t.odd_lds);
  if (st != LBM_OK) return st;
  *best = best_t;
  if (best_us) *best_us = best_time;
  return LBM_OK;
}

lbm_status lbm_set_source(lbm_ctx* c, const float* S_dev) {
  if (!c) return fail(LBM_EINVAL, "ctx is NULL");
  if (S_dev && c->p.storage != LBM_STORE_F32)
    return fail(LBM_EINVAL, "a source term needs FP32 population storage");
  if (S_dev && ((uintptr_t)S_dev) % sizeof(float) != 0) return fail(LBM_EINVAL, "source is not 4-byte aligned");
  c->src = S_dev;
  return LBM_OK;
}

lbm_status lbm_init_fields_device(lbm_ctx* c, const double* Q_dev) {
  if (!c || !Q_dev) return fail(LBM_EINVAL, "ctx or Q is NULL");
  if (c->p.storage == LBM_STORE_F16) {
    lbm_status st = grlbm::scales_from_fields(c->c, c->g, grlbm::make_init_coef(&c->p), Q_dev, c->N, c->stream);
    if (st != LBM_OK) return st;
  }
  HIP_TRY(grlbm::launch_init(c->F, c->p.storage == LBM_STORE_F16, c->g, c->c, grlbm::make_init_coef(&c->p), Q_dev,
                             c->N, c->stream));
  c->step = 0;
  c->ready = true;
  c->ring_used = 0;
  c->ring_steps.clear();
  c->done.clear();
  return LBM_OK;
}

lbm_status lbm_init_fields(lbm_ctx* c, const double* Q) {
  if (!c || !Q) return fail(LBM_EINVAL, "ctx or Q is NULL");
  lbm_status st0 = grlbm::check_fields(&c->p, Q);
  if (st0 != LBM_OK) return st0;
  double* d = nullptr;
  lbm_status st = dev_alloc(&d, (size_t)5 * c->N, "initial fields");
  if (st != LBM_OK) return st;
  hipError_t e = hipMemcpyAsync(d, Q, (size_t)5 * c->N * sizeof(double), hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess) {
    st = lbm_init_fields_device(c, d);
    e = hipStreamSynchronize(c->stream);
  }
  (void)hipFree(d);
  if (e != hipSuccess) return fail(LBM_EDEVICE, "initialisation failed: %s", hipGetErrorString(e));
  return st;
}

lbm_status lbm_step(lbm_ctx* c, int64_t n, int32_t diag_every) {
  if (!c) return fail(LBM_EINVAL, "ctx is NULL");
  if (n < 0) return fail(LBM_EINVAL, "n = %lld < 0", (long long)n);
  if (diag_every < 0) return fail(LBM_EINVAL, "diag_every < 0");
  if (!c->ready) return fail(LBM_ESTATE, "lbm_step before lbm_init_fields or lbm_set_populations");
  grlbm::StepLaunch L;
  L.F = c->F;
  L.g = c->g;
  L.c = c->c;
  L.block = c->block;
  L.coll = c->p.collision;
  L.f16 = c->p.storage == LBM_STORE_F16;
  L.nt = c->nt;
  L.lds = c->lds;
  L.odd_lds = c->odd_lds;
  L.src = c->src;
  L.partials = nullptr;
  if (diag_every > 0) {
    lbm_status st = ensure_partials(c);
    if (st != LBM_OK) return st;
  }
  for (int64_t s = 0; s < n; ++s) {
    const int64_t t = c->step;
    const bool diag = diag_every > 0 && (t % diag_every) == 0;
    L.odd = (t & 1) != 0;
    L.diag = diag;
    L.skey = grlbm::step_key(t);
    if (diag) {
      if (c->ring_used == kRingCap) {
        lbm_status st = drain_ring(c);
        if (st != LBM_OK) return st;
      }
      L.partials = c->partials;
    }
    HIP_TRY(grlbm::launch_step(L, c->stream));
    if (diag) {
      HIP_TRY(grlbm::launch_finalize(c->partials, grlbm::launch_blocks(L), c->ring + (size_t)c->ring_used * kDiagVals, c->stream));
      c->ring_steps.push_back(t);
      ++c->ring_used;
    }
    ++c->step;
  }
  return LBM_OK;
}

lbm_status lbm_moments_device(lbm_ctx* c, double* Q_dev) {
  if (!c || !Q_dev) return fail(LBM_EINVAL, "ctx or Q is NULL");
  if (!c->ready) return fail(LBM_ESTATE, "no state yet");
  HIP_TRY(grlbm::launch_gather(c->F, c->p.storage == LBM_STORE_F16, c->g, c->c, c->N, (c->step & 1) != 0, 1,
                               nullptr, Q_dev, c->stream));
  return LBM_OK;
}

lbm_status lbm_moments(lbm_ctx* c, double* Q_out) {
  if (!c || !Q_out) return fail(LBM_EINVAL, "ctx or Q_out is NULL");
  if (!c->ready) return fail(LBM_ESTATE, "no state yet");
  double* d = nullptr;
  lbm_status st = dev_alloc(&d, (size_t)5 * c->N, "moments");
  if (st != LBM_OK) return st;
  st = lbm_moments_device(c, d);
  hipError_t e = hipSuccess;
  if (st == LBM_OK) {
    e = hipMemcpyAsync(Q_out, d, (size_t)5 * c->N * sizeof(double), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  }
  (void)hipFree(d);
  if (e != hipSuccess) return fail(LBM_EDEVICE, "moments readout failed: %s", hipGetErrorString(e));
  return st;
}

lbm_status lbm_diagnostics(lbm_ctx* c, lbm_diag* out, int32_t max, int32_t* count) {
  if (!c || !count || (max > 0 && !out)) return fail(LBM_EINVAL, "NULL argument");
  *count = 0;
  lbm_status st = drain_ring(c);
  if (st != LBM_OK) return st;
  bool bad = false;
  while (*count < max && !c->done.empty()) {
    out[*count] = c->done.front();
    bad |= out[*count].nonfinite > 0;
    c->done.pop_front();
    ++*count;
  }
  if (bad) return fail(LBM_EDIVERGED, "non-finite populations in a diagnostic record");
  return LBM_OK;
}

lbm_status lbm_get_populations(lbm_ctx* c, float* f, int64_t* step) {
  if (!c || !f) return fail(LBM_EINVAL, "ctx or f is NULL");
  if (!c->ready) return fail(LBM_ESTATE, "no state yet");
  float* d = nullptr;
  lbm_status st = dev_alloc(&d, (size_t)35 * c->N, "populations");
  if (st != LBM_OK) return st;
  hipError_t e = grlbm::launch_gather(c->F, c->p.storage == LBM_STORE_F16, c->g, c->c, c->N,
                                      (c->step & 1) != 0, 0, d, nullptr, c->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(f, d, (size_t)35 * c->N * sizeof(float), hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  (void)hipFree(d);
  if (e != hipSuccess) return fail(LBM_EDEVICE, "population readout failed: %s", hipGetErrorString(e));
  if (step) *step = c->step;
  return LBM_OK;
}

lbm_status lbm_set_populations(lbm_ctx* c, const float* f, int64_t step) {
  if (!c || !f) return fail(LBM_EINVAL, "ctx or f is NULL");
  if (step < 0) return fail(LBM_EINVAL, "step < 0");
  float* d = nullptr;
  lbm_status st = dev_alloc(&d, (size_t)35 * c->N, "populations");
  if (st != LBM_OK) return st;
  hipError_t e = hipMemcpyAsync(d, f, (size_t)35 * c->N * sizeof(float), hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess && c->p.storage == LBM_STORE_F16) {
    st = grlbm::scales_from_pops(c->c, d, c->N, c->stream);
    if (st != LBM_OK) {
      (void)hipFree(d);
      return st;
    }
  }
  if (e == hipSuccess)
    e = grlbm::launch_scatter(c->F, c->p.storage == LBM_STORE_F16, c->g, c->c, c->N, (step & 1) != 0, d,
                              c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  (void)hipFree(d);
  if (e != hipSuccess) return fail(LBM_EDEVICE, "population restore failed: %s", hipGetErrorString(e));
  c->step = step;
  c->ready = true;
  c->ring_used = 0;
  c->ring_steps.clear();
  c->done.clear();
  return LBM_OK;
}

lbm_status lbm_get_step(lbm_ctx* c, int64_t* step) {
  if (!c || !step) return fail(LBM_EINVAL, "NULL argument");
  *step = c->step;
  return LBM_OK;
}

lbm_status lbm_destroy(lbm_ctx* c) {
  if (!c) return LBM_OK;
  lbm_status st = LBM_OK;
  if (c->stream && hipStreamSynchronize(c->stream) != hipSuccess)
    st = fail(LBM_EDEVICE, "stream synchronisation failed during destroy");
  if (c->own_F && c->F) (void)hipFree(c->F);
  if (c->partials) (void)hipFree(c->partials);
  if (c->ring) (void)hipFree(c->ring);
  if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
  delete c;
  return st;
}

lbm_status lbm_bw_probe(size_t bytes, int32_t iters, double* gbps) {
  if (!gbps || bytes < 16 || iters < 1 || bytes > ((size_t)1 << 40))
    return fail(LBM_EINVAL, "bad bw_probe arguments");
  bytes = bytes / 16 * 16;
  void *a = nullptr, *b = nullptr;
  hipStream_t s = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  lbm_status st = LBM_OK;
  float best = 1e30f;
  if (hipMalloc(&a, bytes) != hipSuccess || hipMalloc(&b, bytes) != hipSuccess) {
    st = fail(LBM_ENOMEM, "hipMalloc of 2 x %zu bytes failed", bytes);
    goto done;
  }
  if (hipStreamCreate(&s) != hipSuccess || hipEventCreate(&e0) != hipSuccess ||
      hipEventCreate(&e1) != hipSuccess) {
    st = fail(LBM_EDEVICE, "stream/event creation failed");
    goto done;
  }
  if (hipMemsetAsync(a, 0, bytes, s) != hipSuccess || grlbm::launch_copy(a, b, (int64_t)bytes, s) != hipSuccess) {
    st = fail(LBM_EDEVICE, "copy kernel failed");
    goto done;
  }
  for (int32_t it = 0; it < iters; ++it) {
    float ms = 0.0f;
    if (hipEventRecord(e0, s) != hipSuccess || grlbm::launch_copy(a, b, (int64_t)bytes, s) != hipSuccess ||
        hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
        hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
      st = fail(LBM_EDEVICE, "timed copy failed");
      goto done;
    }
    if (ms < best) best = ms;
  }
  *gbps = 2.0 * (double)bytes / (best * 1e-3) / 1e9;
done:
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (s) {
    (void)hipStreamSynchronize(s);
    (void)hipStreamDestroy(s);
  }
  if (a) (void)hipFree(a);
  if (b) (void)hipFree(b);
  return st;
}

}  // extern "C"

// Device memory for lbm_step_noalloc: the per-block diagnostic partials of one
// launch (kDiagVals floats per block), for grids whose launches have at most
// kNoAllocBlocks blocks.  Every launch writes each partial that its finalize then
// reads, so nothing here has to start at zero.  Each GPU holds its own copy at its
// own address, found once per device with hipGetSymbolAddress; host code uses only
// that address (the array's name is a host-side stand-in).
constexpr int64_t kNoAllocBlocks = int64_t(1) << 18;
static __device__ __align__(256) float scratch[kNoAllocBlocks * 9];

namespace {

static_assert(kDiagVals == 9, "scratch holds 9 diagnostic values per block");
constexpr int kNoAllocMaxDevices = 64;
std::mutex g_scratch_mu;
float* g_scratch_ptr[kNoAllocMaxDevices] = {};

lbm_status scratch_address(int dev, float** out) {
  if (dev < 0 || dev >= kNoAllocMaxDevices) return fail(LBM_EDEVICE, "device %d out of range", dev);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return fail(LBM_EDEVICE, "hipGetSymbolAddress of the scratch array failed: %s", hipGetErrorString(e));
    g_scratch_ptr[dev] = (float*)ptr;
  }
  *out = g_scratch_ptr[dev];
  return LBM_OK;
}

// Steps t in [step, step + n) with t % every == 0.
int64_t diag_count(int64_t step, int64_t n, int64_t every) {
  if (every <= 0 || n <= 0) return 0;
  const int64_t first = (step + every - 1) / every * every;
  return first < step + n ? (step + n - 1 - first) / every + 1 : 0;
}

}  // namespace

extern "C" {

lbm_status lbm_step_noalloc(const lbm_params* p, void* F_dev, int64_t step, int64_t n, int32_t diag_every,
                            float* rec_dev, int32_t rec_max, void* hip_stream) {
  lbm_status st = validate(p);
  if (st != LBM_OK) return st;
  if (!F_dev) return fail(LBM_EINVAL, "population buffer is NULL");
  if (((uintptr_t)F_dev) % 256 != 0) return fail(LBM_EINVAL, "population buffer is not 256-byte aligned");
  if (p->storage != LBM_STORE_F32)
    return fail(LBM_EINVAL, "lbm_step_noalloc takes FP32 storage only (FP16 scales are set at initialisation)");
  if (step < 0 || n < 0 || diag_every < 0) return fail(LBM_EINVAL, "step, n and diag_every must be >= 0");
  const int64_t records = diag_count(step, n, diag_every);
  if (records > 0 && (!rec_dev || rec_max < records))
    return fail(LBM_EINVAL, "%lld diagnostic records need room in rec_dev (rec_max = %d)", (long long)records,
                rec_max);
  grlbm::StepLaunch L;
  L.F = F_dev;
  L.g = make_grid(p);
  L.c = make_coll(p);
  L.block = 256;  // the launch shape of a new context
  L.coll = p->collision;
  L.f16 = false;
  L.nt = default_nontemporal((int64_t)state_bytes(p));
  L.lds = lds_for_blocks_per_cu(kDefaultBlocksPerCuF32);
  L.odd_lds = true;
  L.src = nullptr;
  L.partials = nullptr;
  float* partials = nullptr;
  if (records > 0) {
    const int64_t nb = std::max(grlbm::step_blocks(L.g, L.block), grlbm::odd_tiles(L.g, false).blocks);
    if (nb > kNoAllocBlocks)
      return fail(LBM_EINVAL, "the grid's launches need %lld diagnostic partial blocks; the fixed scratch holds %lld",
                  (long long)nb, (long long)kNoAllocBlocks);
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return fail(LBM_EDEVICE, "no HIP device");
    st = scratch_address(dev, &partials);
    if (st != LBM_OK) return st;
  }
  hipStream_t s = (hipStream_t)hip_stream;
  int64_t r = 0;
  for (int64_t k = 0; k < n; ++k) {
    const int64_t t = step + k;
    const bool diag = diag_every > 0 && (t % diag_every) == 0;
    L.odd = (t & 1) != 0;
    L.diag = diag;
    L.skey = grlbm::step_key(t);
    L.partials = diag ? partials : nullptr;
    HIP_TRY(grlbm::launch_step(L, s));
    if (diag) {
      HIP_TRY(grlbm::launch_finalize(partials, grlbm::launch_blocks(L), rec_dev + r * kDiagVals, s));
      ++r;
    }
  }
  return LBM_OK;
}

const char* lbm_last_error(void) { return grlbm::g_err.c_str(); }

}  // extern "C"
