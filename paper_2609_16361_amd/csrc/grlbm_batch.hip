// grlbm_batch.hip -- many uneven instances stepped together (C ABI lbm_batch_*).
//
// One device arena holds the populations of every instance (the same SoA, AA
// in-place layout as a single context).  A descriptor table and a tile work-list
// live in device memory: a tile is one block-width range of consecutive cells of
// one instance.  k_batch_step loops over the tile list with a fixed grid
// (persistent) or takes one tile per block (grid 0 in the tuning), and each block
// derives its instance's AA parity and whether it is active from a device-resident
// clock, so one launch advances every active instance by one step whatever its
// size, boundaries, parameters or age.  Consecutive launches on one stream order
// the steps (no grid-wide barrier is needed).  Time loops of K steps are captured
// once in a hipGraph: K step nodes per (collision, storage) group followed by a
// one-lane kernel that advances the clock (no memset nodes), and replayed; the tile
// list, descriptors and tile count can change between replays because the graph
// only holds their addresses (with one block per tile, a change of the rounded
// grid captures the graph again).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <map>
#include <new>
#include <vector>

#include "../../include/grlbm.h"
#include "grlbm_device.hpp"
#include "grlbm_internal.h"

namespace grlbm {

struct BatchInst {
  Coll c;
  Grid g;
  int64_t off;      // element offset of the instance's slot 0 in the arena
  int64_t t_start;  // clock value at which the instance was at its step 0
  int64_t t_end;    // clock value at which it has completed all its steps
  double inv_px;    // 1/px and 1/ny for the element-index decomposition
  double inv_ny;
  int32_t cells;    // px * ny * nz: the elements the instance's rows span
  int32_t pad_;
};

// A tile is `blockDim.x` consecutive element indices of one instance (it may span
// several x-rows; lanes on a row's padding have no cell).
struct BatchTile {
  int32_t inst;
  int32_t tile;  // tile index within the instance: cells [tile * blockDim.x, ...)
};

// q = n / d and r = n % d for 0 <= n < 2^31: the FP64 product is within one of the
// quotient, one correction step makes it exact.
__device__ __forceinline__ int div_exact(int n, int d, double inv_d, int& r) {
  int q = (int)((double)n * inv_d);
  r = n - q * d;
  if (r < 0) {
    --q;
    r += d;
  } else if (r >= d) {
    ++q;
    r -= d;
  }
  return q;
}

template <int COLL, typename T, bool NT>
__global__ void __launch_bounds__(1024) k_batch_step(T* __restrict__ arena, const BatchInst* __restrict__ insts,
                                                      const BatchTile* __restrict__ tiles,
                                                      const int32_t* __restrict__ ntiles,
                                                      const int64_t* __restrict__ clock, int32_t j) {
  extern __shared__ float xs[];  // x slots of an odd-step tile (tile_update_odd)
  const int32_t nt = *ntiles;
  const int64_t t = *clock + j;
  for (int32_t tile = blockIdx.x; tile < nt; tile += gridDim.x) {
    const BatchTile bt = tiles[tile];
    const BatchInst* I = insts + bt.inst;
    const int64_t ts = I->t_start;
    if (t < ts || t >= I->t_end) continue;  // the same for the whole block
    const int n0 = bt.tile * (int)blockDim.x;
    const int n = n0 + (int)threadIdx.x;
    bool act = n < I->cells;
    const Grid g = I->g;
    int x = 0, y = 0, z = 0;
    if (act) {
      const int row = div_exact(n, g.px, I->inv_px, x);
      z = div_exact(row, g.ny, I->inv_ny, y);
      act = x < g.nx;  // the row's padding holds no cell
    }
    const Coll c = I->c;
    T* F = arena + I->off;
    // the same arithmetic as a single context uses for this instance, so the
    // results are bitwise the same.  Every instance takes the zero-gradient form
    // of the update: on a periodic axis its face flags are false and it reads and
    // writes exactly what the periodic form does.  A kernel holding both forms
    // compiled to 113-128 registers (94-99 with one) and ran FP16 batches of
    // periodic cubes at 21 GLUP/s against 33 with the single form.
    const bool odd = ((t - ts) & 1) != 0;
    const uint32_t skey = step_key(t - ts);  // the instance's own step index
    if (odd) {
      // every lane takes part (barriers inside).  With the nontemporal hint, the y
      // and z slots are loaded without it: on the batch of 64 Becker tubes (4 x 4
      // cells across, so rows and planes are fractions of a line) 62.35 against
      // 58.09 solves/s at the fastest launch shape, 62.00 with the y slots alone;
      // dropping it on the y and z stores as well gained nothing.
      tile_update_odd<COLL, T, true, false, NT, true, false, NT ? 2 : 0>(F, g, c, n0, act, x, y, z, xs, nullptr,
                                                                         skey);
    } else if (act) {
      cell_update<false, COLL, T, true, false, NT>(F, g, c, x, y, z, nullptr, skey);
    }
  }
}

__global__ void k_batch_advance(int64_t* clock, int32_t n) {
  if (blockIdx.x == 0 && threadIdx.x == 0) *clock += n;
}

// A run of cells [c0, c1) of one instance for the divergence check: element offset
// of the instance's slot 0 in the arena, elements between its slot arrays, storage,
// and the index of the instance's flag.
struct CheckItem {
  int64_t off;
  int64_t S;
  int32_t c0, c1;
  int32_t f16;
  int32_t flag;
  int32_t nx, px;  // row length and pitch: elements with (e mod px) >= nx are padding
};
constexpr int32_t kCheckRun = 16384;   // cells per item
constexpr int32_t kCheckBlocks = 16;   // blocks per item (256 lanes, 4 cells each)

// flags[item.flag] = 1 when the rest population (slot 0) of some field holds a
// non-finite value in the item's cells (exponent bits all ones: an infinity or a
// NaN, FP32 or FP16).  Slot 0 of field k after a step is a sum over all of the
// cell's field-k populations before it (Q_k / 4 in the regularized update, f_0 +
// omega (f_0^eq - f_0) with f_0^eq = Q_k / 4 in BGK), so a non-finite population of
// any field shows up there one step after it appears.  blockIdx.y picks the item;
// its kCheckBlocks blocks stride over the run.  Reads 5 of the 35 arrays.
__global__ void __launch_bounds__(256) k_batch_nonfinite(const char* __restrict__ arena,
                                                          const CheckItem* __restrict__ items,
                                                          int32_t* __restrict__ flags) {
  const CheckItem it = items[blockIdx.y];
  bool bad = false;
  for (int32_t c = it.c0 + (int32_t)(blockIdx.x * blockDim.x + threadIdx.x); c < it.c1;
       c += (int32_t)(gridDim.x * blockDim.x)) {
    if (c % it.px >= it.nx) continue;
#pragma unroll
    for (int k = 0; k < kFields; ++k) {
      const int64_t e = it.off + (int64_t)(7 * k) * it.S + c;
      if (it.f16) {
        bad |= (reinterpret_cast<const uint16_t*>(arena)[e] & 0x7c00u) == 0x7c00u;
      } else {
        bad |= (reinterpret_cast<const uint32_t*>(arena)[e] & 0x7f800000u) == 0x7f800000u;
      }
    }
  }
  if (bad) flags[it.flag] = 1;  // every writer stores the same value
}

}  // namespace grlbm

using grlbm::BatchInst;
using grlbm::BatchTile;
using grlbm::fail;

namespace {

constexpr int kGroups = 4;  // (collision, storage) pairs

int group_of(const lbm_params* p) { return p->collision * 2 + (p->storage == LBM_STORE_F16 ? 1 : 0); }

struct HostInst {
  bool live = false;
  lbm_params p{};
  BatchInst d{};
  size_t bytes = 0;
  int group = 0;
};

}  // namespace

struct lbm_batch {
  hipStream_t stream = nullptr;
  bool own_stream = false;
  int num_cus = 256;
  char* arena = nullptr;
  size_t arena_bytes = 0;
  std::map<size_t, size_t> free_list;  // offset -> bytes
  int32_t max_inst = 0;
  int32_t max_tiles = 0;
  BatchInst* d_insts = nullptr;
  BatchTile* d_tiles = nullptr;      // kGroups segments of max_tiles
  int32_t* d_ntiles = nullptr;       // kGroups counts
  int64_t* d_clock = nullptr;
  grlbm::CheckItem* d_check = nullptr;  // items of the divergence check (grown on demand)
  size_t check_cap = 0;
  int32_t* d_flags = nullptr;           // one flag per live instance (max_inst)
  std::vector<HostInst> insts;
  int64_t clock = 0;
  int32_t graph_steps = 16;
  lbm_batch_tuning tune{};
  bool dirty = true;
  int32_t ntiles_host[kGroups] = {0, 0, 0, 0};
  hipGraphExec_t graph = nullptr;
  unsigned graph_groups = 0;  // bitmask of groups captured
  int32_t graph_grid[kGroups] = {0, 0, 0, 0};  // launch grids baked into the graph
};

namespace {

int64_t inst_tiles(const lbm_params* p, int block) {
  const int64_t n = grlbm::row_pitch(p) * p->ny * p->nz;
  return (n + block - 1) / block;
}

lbm_status upload(lbm_batch* b) {
  if (!b->dirty) return LBM_OK;
  std::vector<BatchTile> tiles[kGroups];
  for (int32_t id = 0; id < (int32_t)b->insts.size(); ++id) {
    HostInst& h = b->insts[id];
    if (!h.live) continue;
    // an instance that has completed its steps keeps its slot but no tiles
    if (h.d.t_end <= b->clock) continue;
    const int64_t n = inst_tiles(&h.p, b->tune.block);
    for (int64_t t = 0; t < n; ++t) tiles[h.group].push_back({id, (int32_t)t});
  }
  for (int g = 0; g < kGroups; ++g)
    if ((int64_t)tiles[g].size() > b->max_tiles)
      return fail(LBM_ENOMEM, "tile list of %zu exceeds the batch capacity %d", tiles[g].size(), b->max_tiles);
  std::vector<BatchInst> desc(b->insts.size());
  for (size_t i = 0; i < b->insts.size(); ++i) desc[i] = b->insts[i].d;
  if (!desc.empty())
    HIP_TRY(hipMemcpyAsync(b->d_insts, desc.data(), desc.size() * sizeof(BatchInst), hipMemcpyHostToDevice,
                           b->stream));
  for (int g = 0; g < kGroups; ++g) {
    b->ntiles_host[g] = (int32_t)tiles[g].size();
    if (!tiles[g].empty())
      HIP_TRY(hipMemcpyAsync(b->d_tiles + (size_t)g * b->max_tiles, tiles[g].data(),
                             tiles[g].size() * sizeof(BatchTile), hipMemcpyHostToDevice, b->stream));
  }
  HIP_TRY(hipMemcpyAsync(b->d_ntiles, b->ntiles_host, sizeof(b->ntiles_host), hipMemcpyHostToDevice, b->stream));
  // the host arrays above must outlive the copies
  HIP_TRY(hipStreamSynchronize(b->stream));
  b->dirty = false;
  return LBM_OK;
}

unsigned active_groups(const lbm_batch* b) {
  unsigned m = 0;
  for (int g = 0; g < kGroups; ++g)
    if (b->ntiles_host[g] > 0) m |= 1u << g;
  return m;
}

// Blocks launched for group g.  A fixed grid loops over the tiles (persistent); grid
// 0 gives every tile its own block, rounded up to a multiple of kGridQuantum so
// that small changes of the tile count keep a captured graph (the extra blocks
// find no tile and exit).
constexpr int32_t kGridQuantum = 256;

int32_t launch_grid(const lbm_batch* b, int g) {
  if (b->tune.grid > 0) return b->tune.grid;
  const int32_t n = std::max<int32_t>(b->ntiles_host[g], 1);
  return (n + kGridQuantum - 1) / kGridQuantum * kGridQuantum;
}

template <int COLL, typename T>
hipError_t launch_group_t(lbm_batch* b, int g, int32_t j) {
  const dim3 grid((unsigned)launch_grid(b, g)), block((unsigned)b->tune.block);
  T* arena = reinterpret_cast<T*>(b->arena);
  const BatchTile* tiles = b->d_tiles + (size_t)g * b->max_tiles;
  const int32_t* nt = b->d_ntiles + g;
  int lds = b->tune.blocks_per_cu > 0 ? (int)(grlbm::kLdsPerCU / (b->tune.blocks_per_cu + 1)) + 256 : 0;
  if (lds > 65536) lds = 65536;
  const int need = 15 * (int)sizeof(float) * b->tune.block;  // odd-step x slots of one tile
  if (lds < need) lds = need;
  if (b->tune.nontemporal)
    hipLaunchKernelGGL((grlbm::k_batch_step<COLL, T, true>), grid, block, lds, b->stream, arena, b->d_insts, tiles,
                       nt, b->d_clock, j);
  else
    hipLaunchKernelGGL((grlbm::k_batch_step<COLL, T, false>), grid, block, lds, b->stream, arena, b->d_insts, tiles,
                       nt, b->d_clock, j);
  return hipGetLastError();
}

hipError_t launch_group(lbm_batch* b, int g, int32_t j) {
  switch (g) {
    case 0: return launch_group_t<0, float>(b, g, j);
    case 1: return launch_group_t<0, _Float16>(b, g, j);
    case 2: return launch_group_t<1, float>(b, g, j);
    default: return launch_group_t<1, _Float16>(b, g, j);
  }
}

// Enqueue n steps directly (no graph).
lbm_status enqueue_steps(lbm_batch* b, int32_t n, unsigned groups) {
  for (int32_t j = 0; j < n; ++j)
    for (int g = 0; g < kGroups; ++g)
      if (groups & (1u << g)) HIP_TRY(launch_group(b, g, j));
  hipLaunchKernelGGL(grlbm::k_batch_advance, dim3(1), dim3(64), 0, b->stream, b->d_clock, n);
  HIP_TRY(hipGetLastError());
  return LBM_OK;
}

void drop_graph(lbm_batch* b) {
  if (b->graph) (void)hipGraphExecDestroy(b->graph);
  b->graph = nullptr;
  b->graph_groups = 0;
}

lbm_status capture_graph(lbm_batch* b, unsigned groups) {
  drop_graph(b);
  hipGraph_t g = nullptr;
  HIP_TRY(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
  lbm_status st = enqueue_steps(b, b->graph_steps, groups);
  hipError_t e = hipStreamEndCapture(b->stream, &g);
  if (st != LBM_OK) {
    if (g) (void)hipGraphDestroy(g);
    return st;
  }
  if (e != hipSuccess) return fail(LBM_EDEVICE, "hipStreamEndCapture failed: %s", hipGetErrorString(e));
  e = hipGraphInstantiate(&b->graph, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) {
    b->graph = nullptr;
    return fail(LBM_EDEVICE, "hipGraphInstantiate failed: %s", hipGetErrorString(e));
  }
  b->graph_groups = groups;
  for (int k = 0; k < kGroups; ++k) b->graph_grid[k] = launch_grid(b, k);
  return LBM_OK;
}

// The captured graph no longer matches the groups to step or their launch grids.
bool graph_stale(const lbm_batch* b, unsigned groups) {
  if (!b->graph || b->graph_groups != groups) return true;
  for (int k = 0; k < kGroups; ++k)
    if ((groups & (1u << k)) && b->graph_grid[k] != launch_grid(b, k)) return true;
  return false;
}

lbm_status run_steps(lbm_batch* b, int64_t n) {
  lbm_status st = upload(b);
  if (st != LBM_OK) return st;
  const unsigned groups = active_groups(b);
  if (groups == 0 || n == 0) {
    // nothing to update: the clock still moves so instance windows stay consistent
    if (n > 0) {
      hipLaunchKernelGGL(grlbm::k_batch_advance, dim3(1), dim3(64), 0, b->stream, b->d_clock, (int32_t)n);
      HIP_TRY(hipGetLastError());
    }
    b->clock += n;
    return LBM_OK;
  }
  int64_t left = n;
  if (b->graph_steps > 1 && left >= b->graph_steps) {
    if (graph_stale(b, groups)) {
      st = capture_graph(b, groups);
      if (st != LBM_OK) return st;
    }
    while (left >= b->graph_steps) {
      HIP_TRY(hipGraphLaunch(b->graph, b->stream));
      left -= b->graph_steps;
    }
  }
  while (left > 0) {
    const int32_t chunk = (int32_t)std::min<int64_t>(left, 1 << 20);
    st = enqueue_steps(b, chunk, groups);
    if (st != LBM_OK) return st;
    left -= chunk;
  }
  b->clock += n;
  // instances finished inside this run drop out of the tile list next time
  for (const HostInst& h : b->insts)
    if (h.live && h.d.t_end <= b->clock && h.d.t_end > b->clock - n) b->dirty = true;
  return LBM_OK;
}

bool arena_alloc(lbm_batch* b, size_t bytes, size_t* off) {
  for (auto it = b->free_list.begin(); it != b->free_list.end(); ++it) {
    if (it->second >= bytes) {
      *off = it->first;
      const size_t rest = it->second - bytes;
      const size_t at = it->first + bytes;
      b->free_list.erase(it);
      if (rest) b->free_list[at] = rest;
      return true;
    }
  }
  return false;
}

void arena_free(lbm_batch* b, size_t off, size_t bytes) {
  auto it = b->free_list.emplace(off, bytes).first;
  auto nx = std::next(it);
  if (nx != b->free_list.end() && it->first + it->second == nx->first) {
    it->second += nx->second;
    b->free_list.erase(nx);
  }
  if (it != b->free_list.begin()) {
    auto pv = std::prev(it);
    if (pv->first + pv->second == it->first) {
      pv->second += it->second;
      b->free_list.erase(it);
    }
  }
}

lbm_status check_id(lbm_batch* b, int32_t id) {
  if (!b) return fail(LBM_EINVAL, "batch is NULL");
  if (id < 0 || id >= (int32_t)b->insts.size() || !b->insts[id].live)
    return fail(LBM_EINVAL, "no live instance with id %d", id);
  return LBM_OK;
}

int64_t completed_steps(const lbm_batch* b, const HostInst& h) {
  const int64_t t = std::min(b->clock, h.d.t_end);
  return std::max<int64_t>(0, t - h.d.t_start);
}

size_t used_extent(const lbm_batch* b) {
  size_t hi = 0;
  for (const HostInst& h : b->insts)
    if (h.live) hi = std::max(hi, (size_t)(h.d.off * (h.p.storage == LBM_STORE_F16 ? 2 : 4)) + h.bytes);
  return hi;
}

}  // namespace

extern "C" {

lbm_status lbm_batch_create(size_t arena_bytes, int32_t max_instances, int32_t max_tiles, int32_t graph_steps,
                            void* hip_stream, lbm_batch** out) {
  if (!out) return fail(LBM_EINVAL, "out is NULL");
  *out = nullptr;
  if (arena_bytes < 256 || max_instances < 1 || max_tiles < 1 || graph_steps < 1 || graph_steps > 4096)
    return fail(LBM_EINVAL, "bad batch sizes (arena %zu, instances %d, tiles %d, graph steps %d)", arena_bytes,
                max_instances, max_tiles, graph_steps);
  lbm_batch* b = new (std::nothrow) lbm_batch();
  if (!b) return fail(LBM_ENOMEM, "host allocation failed");
  auto bail = [&](lbm_status s) {
    lbm_batch_destroy(b);
    return s;
  };
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return bail(fail(LBM_EDEVICE, "no HIP device"));
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && cus > 0)
    b->num_cus = cus;
  if (hip_stream) {
    b->stream = (hipStream_t)hip_stream;
  } else {
    if (hipStreamCreate(&b->stream) != hipSuccess) return bail(fail(LBM_EDEVICE, "hipStreamCreate failed"));
    b->own_stream = true;
  }
  b->arena_bytes = arena_bytes / 256 * 256;
  if (hipMalloc((void**)&b->arena, b->arena_bytes) != hipSuccess)
    return bail(fail(LBM_ENOMEM, "hipMalloc of a %zu-byte arena failed", b->arena_bytes));
  b->free_list[0] = b->arena_bytes;
  b->max_inst = max_instances;
  b->max_tiles = max_tiles;
  if (hipMalloc((void**)&b->d_insts, sizeof(BatchInst) * (size_t)max_instances) != hipSuccess ||
      hipMalloc((void**)&b->d_tiles, sizeof(BatchTile) * (size_t)max_tiles * kGroups) != hipSuccess ||
      hipMalloc((void**)&b->d_ntiles, sizeof(int32_t) * kGroups) != hipSuccess ||
      hipMalloc((void**)&b->d_clock, sizeof(int64_t)) != hipSuccess ||
      hipMalloc((void**)&b->d_flags, sizeof(int32_t) * (size_t)max_instances) != hipSuccess)
    return bail(fail(LBM_ENOMEM, "hipMalloc of the batch tables failed"));
  const int64_t zero = 0;
  const int32_t zeros[kGroups] = {0, 0, 0, 0};
  if (hipMemcpyAsync(b->d_clock, &zero, sizeof zero, hipMemcpyHostToDevice, b->stream) != hipSuccess ||
      hipMemcpyAsync(b->d_ntiles, zeros, sizeof zeros, hipMemcpyHostToDevice, b->stream) != hipSuccess ||
      hipStreamSynchronize(b->stream) != hipSuccess)
    return bail(fail(LBM_EDEVICE, "batch table initialisation failed"));
  b->graph_steps = graph_steps;
  // one 256-cell tile per block with plain loads and stores, at most 2 blocks per
  // CU: the fastest shape on a mixed FP32/FP16 serving load (persistent grids
  // trail it by 6-9%, the nontemporal hint by 5%; uncapped blocks by 1-2% in
  // solves/s, 4.5% on the 64 requests resident at once); lbm_batch_autotune picks
  // per workload
  b->tune.block = 256;
  b->tune.nontemporal = 0;
  b->tune.blocks_per_cu = 2;
  b->tune.grid = 0;
  *out = b;
  return LBM_OK;
}

lbm_status lbm_batch_add(lbm_batch* b, const lbm_params* p, const double* Q, int64_t steps, int32_t* id) {
  if (!b || !p || !Q || !id) return fail(LBM_EINVAL, "NULL argument");
  if (steps < 0) return fail(LBM_EINVAL, "steps < 0");
  lbm_status st = grlbm::validate(p);
  if (st != LBM_OK) return st;
  st = grlbm::check_fields(p, Q);
  if (st != LBM_OK) return st;
  int32_t slot = -1;
  for (int32_t i = 0; i < (int32_t)b->insts.size(); ++i)
    if (!b->insts[i].live) {
      slot = i;
      break;
    }
  if (slot < 0) {
    if ((int32_t)b->insts.size() >= b->max_inst) return fail(LBM_ENOMEM, "batch holds %d instances already", b->max_inst);
    slot = (int32_t)b->insts.size();
    b->insts.emplace_back();
  }
  const int g = group_of(p);
  int64_t tiles_in_group = inst_tiles(p, b->tune.block);
  for (const HostInst& h : b->insts)
    if (h.live && h.group == g && h.d.t_end > b->clock) tiles_in_group += inst_tiles(&h.p, b->tune.block);
  if (tiles_in_group > b->max_tiles)
    return fail(LBM_ENOMEM, "instance needs %lld tiles beyond the capacity %d",
                (long long)inst_tiles(p, b->tune.block), b->max_tiles);
  const size_t bytes = grlbm::state_bytes(p);
  size_t off = 0;
  if (!arena_alloc(b, bytes, &off))
    return fail(LBM_ENOMEM, "arena has no free run of %zu bytes", bytes);
  HostInst& h = b->insts[slot];
  h.p = *p;
  h.bytes = bytes;
  h.group = g;
  h.d.c = grlbm::make_coll(p);
  h.d.g = grlbm::make_grid(p);
  const int el = p->storage == LBM_STORE_F16 ? 2 : 4;
  h.d.off = (int64_t)(off / el);
  h.d.t_start = b->clock;
  h.d.t_end = b->clock + steps;
  const int64_t N = (int64_t)p->nx * p->ny * p->nz;
  h.d.cells = (int32_t)grlbm::row_cells(h.d.g);
  h.d.inv_px = 1.0 / h.d.g.px;
  h.d.inv_ny = 1.0 / p->ny;
  double* dq = nullptr;
  if (hipMalloc((void**)&dq, sizeof(double) * 5 * (size_t)N) != hipSuccess) {
    arena_free(b, off, bytes);
    return fail(LBM_ENOMEM, "staging allocation for the initial fields failed");
  }
  hipError_t e = hipMemcpyAsync(dq, Q, sizeof(double) * 5 * (size_t)N, hipMemcpyHostToDevice, b->stream);
  if (e == hipSuccess && p->storage == LBM_STORE_F16) {
    st = grlbm::scales_from_fields(h.d.c, h.d.g, grlbm::make_init_coef(p), dq, N, b->stream);
    if (st != LBM_OK) {
      (void)hipFree(dq);
      arena_free(b, off, bytes);
      return st;
    }
  }
  if (e == hipSuccess)
    e = grlbm::launch_init(b->arena + off, p->storage == LBM_STORE_F16, h.d.g, h.d.c, grlbm::make_init_coef(p), dq,
                           N, b->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
  (void)hipFree(dq);
  if (e != hipSuccess) {
    arena_free(b, off, bytes);
    return fail(LBM_EDEVICE, "instance initialisation failed: %s", hipGetErrorString(e));
  }
  h.live = true;
  b->dirty = true;
  *id = slot;
  return LBM_OK;
}

lbm_status lbm_batch_run(lbm_batch* b, int64_t n) {
  if (!b) return fail(LBM_EINVAL, "batch is NULL");
  if (n < 0) return fail(LBM_EINVAL, "n < 0");
  return run_steps(b, n);
}

lbm_status lbm_batch_query(lbm_batch* b, int32_t id, int64_t* done_steps, int32_t* finished) {
  lbm_status st = check_id(b, id);
  if (st != LBM_OK) return st;
  const HostInst& h = b->insts[id];
  if (done_steps) *done_steps = completed_steps(b, h);
  if (finished) *finished = h.d.t_end <= b->clock ? 1 : 0;
  return LBM_OK;
}

lbm_status lbm_batch_moments(lbm_batch* b, int32_t id, double* Q_out) {
  lbm_status st = check_id(b, id);
  if (st != LBM_OK) return st;
  if (!Q_out) return fail(LBM_EINVAL, "Q_out is NULL");
  const HostInst& h = b->insts[id];
  const int64_t N = (int64_t)h.p.nx * h.p.ny * h.p.nz;
  const int el = h.p.storage == LBM_STORE_F16 ? 2 : 4;
  double* d = nullptr;
  if (hipMalloc((void**)&d, sizeof(double) * 5 * (size_t)N) != hipSuccess)
    return fail(LBM_ENOMEM, "staging allocation for the moments failed");
  hipError_t e = grlbm::launch_gather(b->arena + (size_t)h.d.off * el, h.p.storage == LBM_STORE_F16, h.d.g, h.d.c, N,
                                      (completed_steps(b, h) & 1) != 0, 1, nullptr, d, b->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(Q_out, d, sizeof(double) * 5 * (size_t)N, hipMemcpyDeviceToHost, b->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
  (void)hipFree(d);
  if (e != hipSuccess) return fail(LBM_EDEVICE, "moments readout failed: %s", hipGetErrorString(e));
  return LBM_OK;
}

lbm_status lbm_batch_populations(lbm_batch* b, int32_t id, float* f_out, int64_t* step) {
  lbm_status st = check_id(b, id);
  if (st != LBM_OK) return st;
  if (!f_out) return fail(LBM_EINVAL, "f_out is NULL");
  const HostInst& h = b->insts[id];
  const int64_t N = (int64_t)h.p.nx * h.p.ny * h.p.nz;
  const int el = h.p.storage == LBM_STORE_F16 ? 2 : 4;
  float* d = nullptr;
  if (hipMalloc((void**)&d, sizeof(float) * 35 * (size_t)N) != hipSuccess)
    return fail(LBM_ENOMEM, "staging allocation for the populations failed");
  const int64_t done = completed_steps(b, h);
  hipError_t e = grlbm::launch_gather(b->arena + (size_t)h.d.off * el, h.p.storage == LBM_STORE_F16, h.d.g, h.d.c, N,
                                      (done & 1) != 0, 0, d, nullptr, b->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(f_out, d, sizeof(float) * 35 * (size_t)N, hipMemcpyDeviceToHost, b->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
  (void)hipFree(d);
  if (e != hipSuccess) return fail(LBM_EDEVICE, "population readout failed: %s", hipGetErrorString(e));
  if (step) *step = done;
  return LBM_OK;
}

lbm_status lbm_batch_nonfinite(lbm_batch* b, int32_t* ids, int32_t max, int32_t* count) {
  if (!b || !count) return fail(LBM_EINVAL, "NULL argument");
  if (max < 0 || (max > 0 && !ids)) return fail(LBM_EINVAL, "bad id buffer (max %d)", max);
  *count = 0;
  std::vector<grlbm::CheckItem> items;
  std::vector<int32_t> which;  // flag index -> instance id
  for (int32_t id = 0; id < (int32_t)b->insts.size(); ++id) {
    const HostInst& h = b->insts[id];
    if (!h.live) continue;
    const int32_t f16 = h.p.storage == LBM_STORE_F16 ? 1 : 0;
    for (int32_t c0 = 0; c0 < h.d.cells; c0 += grlbm::kCheckRun)
      items.push_back({h.d.off, h.d.g.S, c0, c0 + std::min(grlbm::kCheckRun, h.d.cells - c0), f16,
                       (int32_t)which.size(), h.d.g.nx, h.d.g.px});
    which.push_back(id);
  }
  const int32_t n = (int32_t)which.size();  // at most max_inst flags
  if (n == 0) return LBM_OK;
  if (items.size() > b->check_cap) {
    // no check kernel is in flight: every call ends synchronised
    const size_t want = std::max(items.size(), 2 * b->check_cap);
    if (b->d_check) (void)hipFree(b->d_check);
    b->d_check = nullptr;
    b->check_cap = 0;
    if (hipMalloc((void**)&b->d_check, sizeof(grlbm::CheckItem) * want) != hipSuccess)
      return fail(LBM_ENOMEM, "hipMalloc of %zu check items failed", want);
    b->check_cap = want;
  }
  std::vector<int32_t> flags(n, 0);
  HIP_TRY(hipMemcpyAsync(b->d_check, items.data(), sizeof(grlbm::CheckItem) * items.size(), hipMemcpyHostToDevice,
                         b->stream));
  HIP_TRY(hipMemcpyAsync(b->d_flags, flags.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice, b->stream));
  constexpr size_t kMaxGridY = 65535;
  for (size_t i0 = 0; i0 < items.size(); i0 += kMaxGridY) {
    const size_t m = std::min(kMaxGridY, items.size() - i0);
    hipLaunchKernelGGL(grlbm::k_batch_nonfinite, dim3(grlbm::kCheckBlocks, (unsigned)m), dim3(256), 0, b->stream,
                       (const char*)b->arena, b->d_check + i0, b->d_flags);
    HIP_TRY(hipGetLastError());
  }
  HIP_TRY(hipMemcpyAsync(flags.data(), b->d_flags, sizeof(int32_t) * n, hipMemcpyDeviceToHost, b->stream));
  // the host vectors above must outlive the copies
  HIP_TRY(hipStreamSynchronize(b->stream));
  for (int32_t i = 0; i < n; ++i) {
    if (!flags[i]) continue;
    if (*count < max) ids[*count] = which[i];
    ++*count;
  }
  return LBM_OK;
}

lbm_status lbm_batch_remove(lbm_batch* b, int32_t id) {
  lbm_status st = check_id(b, id);
  if (st != LBM_OK) return st;
  // work already enqueued may still touch the instance's memory
  HIP_TRY(hipStreamSynchronize(b->stream));
  HostInst& h = b->insts[id];
  const int el = h.p.storage == LBM_STORE_F16 ? 2 : 4;
  arena_free(b, (size_t)h.d.off * el, h.bytes);
  h.live = false;
  h.d.t_start = h.d.t_end = 0;  // stale tiles of a later run skip it
  b->dirty = true;
  return LBM_OK;
}

lbm_status lbm_batch_info(lbm_batch* b, lbm_batch_stats* out) {
  if (!b || !out) return fail(LBM_EINVAL, "NULL argument");
  std::memset(out, 0, sizeof *out);
  out->clock = b->clock;
  out->arena_bytes = b->arena_bytes;
  size_t freeb = 0, largest = 0;
  for (auto& kv : b->free_list) {
    freeb += kv.second;
    largest = std::max(largest, kv.second);
  }
  out->arena_free_bytes = freeb;
  out->arena_largest_free = largest;
  for (const HostInst& h : b->insts) {
    if (!h.live) continue;
    ++out->live_instances;
    if (h.d.t_end > b->clock) {
      ++out->active_instances;
      out->active_cells += (int64_t)h.p.nx * h.p.ny * h.p.nz;
    }
  }
  out->tuning = b->tune;
  out->graph_steps = b->graph_steps;
  return LBM_OK;
}

lbm_status lbm_batch_set_tuning(lbm_batch* b, const lbm_batch_tuning* t) {
  if (!b || !t) return fail(LBM_EINVAL, "NULL argument");
  if (t->block < 64 || t->block > 1024 || t->block % 64 != 0)
    return fail(LBM_EINVAL, "block = %d must be a multiple of 64 in [64, 1024]", t->block);
  if (t->grid < 0 || t->grid > (1 << 24)) return fail(LBM_EINVAL, "grid = %d outside [0, 2^24]", t->grid);
  if (t->blocks_per_cu < 0 || t->blocks_per_cu > 32) return fail(LBM_EINVAL, "blocks_per_cu outside [0, 32]");
  if (t->block != b->tune.block) {
    // the tile width is the block width: check the capacity before switching
    int64_t per_group[kGroups] = {0, 0, 0, 0};
    for (const HostInst& h : b->insts)
      if (h.live && h.d.t_end > b->clock) per_group[h.group] += inst_tiles(&h.p, t->block);
    for (int g = 0; g < kGroups; ++g)
      if (per_group[g] > b->max_tiles) return fail(LBM_ENOMEM, "block %d needs more tiles than the capacity", t->block);
  }
  b->tune = *t;
  b->tune.nontemporal = t->nontemporal ? 1 : 0;
  b->dirty = true;
  drop_graph(b);
  return LBM_OK;
}

lbm_status lbm_batch_autotune(lbm_batch* b, int32_t trial_steps, lbm_batch_tuning* best, float* best_us,
                              lbm_batch_tuning* tried, float* tried_us, int32_t max_tried, int32_t* ntried) {
  if (!b || !best) return fail(LBM_EINVAL, "NULL argument");
  if (trial_steps < 2) return fail(LBM_EINVAL, "trial_steps must be >= 2");
  if (ntried) *ntried = 0;
  HIP_TRY(hipStreamSynchronize(b->stream));
  // snapshot of the live state: trials advance the instances, the snapshot puts
  // them back (results never depend on the launch shape)
  const size_t extent = used_extent(b);
  char* snap = nullptr;
  if (extent > 0) {
    if (hipMalloc((void**)&snap, extent) != hipSuccess) return fail(LBM_ENOMEM, "snapshot of %zu bytes failed", extent);
    HIP_TRY(hipMemcpyAsync(snap, b->arena, extent, hipMemcpyDeviceToDevice, b->stream));
  }
  const lbm_batch_tuning orig = b->tune;
  const int64_t clock0 = b->clock;
  std::vector<lbm_batch_tuning> cands;
  for (int block : {128, 256, 512, 1024})
    for (int waves_per_cu : {8, 16, 32}) {
      const int bpc = std::max(1, waves_per_cu / (block / 64));
      if (bpc * (block / 64) != waves_per_cu) continue;
      for (int nt : {0, 1}) {
        lbm_batch_tuning t{};
        t.block = block;
        t.nontemporal = nt;
        t.blocks_per_cu = bpc;
        t.grid = b->num_cus * bpc;
        cands.push_back(t);
      }
    }
  // one block per tile, occupancy set by the registers alone, and for 256- and
  // 512-thread blocks capped at 8 or 16 waves per CU as well (the default shape
  // is one of these; nontemporal access with 4 blocks of 256 per CU runs large
  // cubes at the single-context rate)
  for (int block : {128, 256, 512, 1024})
    for (int bpc : {0, 2, 4})
      for (int nt : {0, 1}) {
        if (bpc > 0 && (block < 256 || block > 512 || bpc * (block / 64) > 16)) continue;
        lbm_batch_tuning t{};
        t.block = block;
        t.nontemporal = nt;
        t.blocks_per_cu = bpc;
        t.grid = 0;
        cands.push_back(t);
      }
  hipEvent_t e0 = nullptr, e1 = nullptr;
  lbm_status st = LBM_OK;
  float best_time = 1e30f;
  lbm_batch_tuning best_t = orig;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    st = fail(LBM_EDEVICE, "event creation failed");
  }
  for (size_t ci = 0; st == LBM_OK && ci < cands.size(); ++ci) {
    st = lbm_batch_set_tuning(b, &cands[ci]);
    if (st == LBM_ENOMEM) {  // this block width does not fit the tile capacity
      st = LBM_OK;
      continue;
    }
    if (st != LBM_OK) break;
    // warm-up: uploads the tiles for this width and captures the graph, so the timed
    // run replays it without host work in between
    st = run_steps(b, std::max(2, b->graph_steps));
    if (st != LBM_OK) break;
    float ms = 0.0f;
    if (hipEventRecord(e0, b->stream) != hipSuccess) { st = fail(LBM_EDEVICE, "event record failed"); break; }
    st = run_steps(b, trial_steps);
    if (st != LBM_OK) break;
    if (hipEventRecord(e1, b->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
        hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
      st = fail(LBM_EDEVICE, "trial timing failed");
      break;
    }
    const float us = ms * 1000.0f / trial_steps;
    if (tried && ntried && *ntried < max_tried) {
      tried[*ntried] = cands[ci];
      if (tried_us) tried_us[*ntried] = us;
      ++*ntried;
    }
    if (us < best_time) {
      best_time = us;
      best_t = cands[ci];
    }
    // restore the state and the clock
    if (extent > 0 && hipMemcpyAsync(b->arena, snap, extent, hipMemcpyDeviceToDevice, b->stream) != hipSuccess) {
      st = fail(LBM_EDEVICE, "snapshot restore failed");
      break;
    }
    b->clock = clock0;
    if (hipMemcpyAsync(b->d_clock, &b->clock, sizeof(int64_t), hipMemcpyHostToDevice, b->stream) != hipSuccess ||
        hipStreamSynchronize(b->stream) != hipSuccess) {
      st = fail(LBM_EDEVICE, "clock restore failed");
      break;
    }
    b->dirty = true;
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (snap) {
    (void)hipStreamSynchronize(b->stream);
    (void)hipFree(snap);
  }
  if (st != LBM_OK) return st;
  st = lbm_batch_set_tuning(b, &best_t);
  if (st != LBM_OK) return st;
  *best = best_t;
  if (best_us) *best_us = best_time;
  return LBM_OK;
}

lbm_status lbm_batch_destroy(lbm_batch* b) {
  if (!b) return LBM_OK;
  lbm_status st = LBM_OK;
  if (b->stream && hipStreamSynchronize(b->stream) != hipSuccess)
    st = fail(LBM_EDEVICE, "stream synchronisation failed during destroy");
  drop_graph(b);
  if (b->arena) (void)hipFree(b->arena);
  if (b->d_insts) (void)hipFree(b->d_insts);
  if (b->d_tiles) (void)hipFree(b->d_tiles);
  if (b->d_ntiles) (void)hipFree(b->d_ntiles);
  if (b->d_clock) (void)hipFree(b->d_clock);
  if (b->d_check) (void)hipFree(b->d_check);
  if (b->d_flags) (void)hipFree(b->d_flags);
  if (b->own_stream && b->stream) (void)hipStreamDestroy(b->stream);
  delete b;
  return st;
}

}  // extern "C"
