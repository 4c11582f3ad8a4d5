// grlbm_internal.h -- launchers shared between the kernels and the C ABI runtime.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/grlbm.h"
#include "grlbm_device.hpp"

// Failure with a message for lbm_last_error (returns st).
#define HIP_TRY(expr)                                                                  \
  do {                                                                                 \
    hipError_t e_ = (expr);                                                            \
    if (e_ != hipSuccess)                                                              \
      return grlbm::fail(LBM_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));  \
  } while (0)

namespace grlbm {

lbm_status fail(lbm_status st, const char* fmt, ...);
lbm_status validate(const lbm_params* p);
// Initial conserved fields Q[5][N] (host) describe a physical state: every value
// finite, density and pressure positive in every cell; EINVAL names the first cell
// that is not.
lbm_status check_fields(const lbm_params* p, const double* Q);
// Elements between consecutive x-rows: nx, or nx rounded up to whole 128-byte
// lines when that adds at most a sixteenth of the row (grids of more than one row).
int64_t row_pitch(const lbm_params* p);
int64_t slot_stride(const lbm_params* p);
size_t state_bytes(const lbm_params* p);
Coll make_coll(const lbm_params* p);
Grid make_grid(const lbm_params* p);

// Coefficients of the initial state (k_init), FP64: it is computed once per solve.
struct InitCoef {
  double gm1, mu_ref, kappa_ref, T_ref, T_S;
  double rho_min, p_min, rho_ref, E_ref;
  double inv_omega[5];
  int32_t sutherland;
  int32_t equilibrium;  // 1: the equilibrium with the advective flux (LBM_START_EQUILIBRIUM)
};
InitCoef make_init_coef(const lbm_params* p);

struct StepLaunch {
  void* F;           // population buffer
  Grid g;
  Coll c;
  float* partials;   // per-block diagnostic partials (diag only)
  int block;         // threads per block (multiple of 64, <= 1024)
  int coll;          // 0 regularized with sensor, 1 BGK
  bool odd;          // AA parity of this step
  bool f16;          // FP16 storage
  bool diag;         // fused diagnostics
  bool nt;           // nontemporal loads and stores
  int lds;           // dynamic LDS bytes reserved per block (occupancy cap), 0 = none
  bool odd_lds;      // odd steps use k_step_odd_tiles (x populations shifted in LDS)
  const float* src;  // source of eq. 1, [5][N] per step, or nullptr (FP32 storage only)
  uint32_t skey;     // step_key of the step (FP16 stochastic rounding)
};

constexpr int64_t kLdsPerCU = 160 * 1024;  // LDS of one gfx950 compute unit
constexpr int kOddTileF32 = 512;           // cells per linear tile of k_step_odd_tiles, FP32
constexpr int kOddTileF16 = 256;           // the same for FP16 storage
constexpr int kMaxRowTile = 1024;          // longest x-row k_step_odd_tiles maps to one block
constexpr int kMaxGroupTile = 512;         // most cells in a k_step_odd_tiles block of whole rows
constexpr int64_t kPairMinCells = 1 << 23;  // FP16 even steps take two cells per lane from here on
// rows map to blocks only when nx is a multiple of this (FP32 / FP16): a partly
// filled last wave costs more than the tile edges
constexpr int kRowMultipleF32 = 32;
constexpr int kRowMultipleF16 = 64;
// FP16 odd steps take two cells per lane, one row per block, on grids of
// kPairMinCells and more whose nx is a multiple of kRowMultipleOddPairs (whole
// waves of pairs) from kMinRowPairs to kMaxRowPairs
constexpr int kRowMultipleOddPairs = 128;
constexpr int kMinRowPairs = 384;
constexpr int kMaxRowPairs = 512;

hipError_t launch_step(const StepLaunch& L, hipStream_t s);
int64_t step_blocks(const Grid& g, int block);
constexpr int kOddLinear = 0;    // k_step_odd_tiles: linear tiles of kOddTileF32/F16 cells
constexpr int kOddRow = 1;       // one block per x-row
constexpr int kOddRowGroup = 2;  // blocks of whole x-rows
struct OddTiles {
  int map;         // kOddLinear, kOddRow or kOddRowGroup
  int tile;        // cells per tile (kOddRowGroup: R * px)
  int block;       // threads per block
  int64_t blocks;  // blocks (= diagnostic partials)
  int lds;         // dynamic LDS bytes per block
  bool y_temporal; // rows not whole 128-byte lines: y slots loaded without the nontemporal hint
};
OddTiles odd_tiles(const Grid& g, bool f16);  // launch shape of k_step_odd_tiles
int odd_group_rows(const Grid& g, bool f16);  // x-rows per kOddRowGroup block, 0 if none
int64_t launch_blocks(const StepLaunch& L);  // blocks (= diagnostic partials) of a launch
bool even_pairs(const StepLaunch& L);        // the even step runs k_step_even_pairs
int64_t pair_blocks(const StepLaunch& L);    // its blocks
bool odd_pairs(const StepLaunch& L);         // the odd step runs k_step_odd_row_pairs
int odd_pair_lds(const Grid& g);             // its dynamic LDS bytes per block
hipError_t launch_finalize(const float* partials, int64_t nblocks, float* rec, hipStream_t s);
hipError_t launch_init(void* F, bool f16, const Grid& g, const Coll& c, const InitCoef& ic, const double* Q,
                       int64_t N, hipStream_t s);
hipError_t launch_gather(const void* F, bool f16, const Grid& g, const Coll& c, int64_t N, bool odd,
                         int mode, float* out_f, double* out_q, hipStream_t s);
hipError_t launch_scatter(void* F, bool f16, const Grid& g, const Coll& c, int64_t N, bool odd,
                          const float* in_f, hipStream_t s);
hipError_t launch_init_maxabs(const Grid& g, const Coll& c, const InitCoef& ic, const double* Q, int64_t N,
                              unsigned* maxabs, hipStream_t s);
hipError_t launch_maxabs_pops(const float* f, int64_t N, unsigned* maxabs, hipStream_t s);
// FP16 storage: pick power-of-two scales so that each field's largest initial |g|
// maps into [32, 64): 1024x headroom below the FP16 maximum for populations that
// grow during the run (a nearly uniform initial field gets a large scale, and a
// shock can raise its populations almost a hundredfold), and 2^-19 of it before
// subnormals.  A power-of-two scale leaves the mantissa bits, hence the stochastic
// rounding of every normal value, unchanged.
void set_storage_scales(Coll& c, const unsigned maxabs_bits[5]);
// Scales from the initial fields Q (device) or from canonical populations f
// (device); synchronises the stream to read the maxima back.
lbm_status scales_from_fields(Coll& c, const Grid& g, const InitCoef& ic, const double* Q_dev, int64_t N,
                              hipStream_t s);
lbm_status scales_from_pops(Coll& c, const float* f_dev, int64_t N, hipStream_t s);
hipError_t launch_copy(const void* a, void* b, int64_t bytes, hipStream_t s);

}  // namespace grlbm
