// Host runtime and C interface of the batched MLS-MPM library.
//
// A batch holds E environments whose particles are concatenated (CSR by env)
// in structure-of-arrays FP32 state buffers of 24 components, and whose dense
// grids are concatenated tile by tile (4^3 nodes, 8 channels). A forward of S
// substeps runs in segments of K: each segment sorts the particles by
// (env, tile, cell) -- the sorted state is the segment's checkpoint -- and
// then runs its substeps (P2G, grid update, G2P). With recording on, the last
// segment also keeps every substep's state and grid (its tape). The backward
// walks the segments in reverse: it re-runs each segment from its checkpoint
// into the tape (gradient checkpointing with recomputation), runs the adjoint
// substeps in reverse, and undoes the segment's sort permutation.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <map>
#include <tuple>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/mpm.h"
#include "mpm_internal.h"
#include "mpm_kernels.h"

using namespace mpmx;

namespace {

enum KernelClass { KC_P2G = 0, KC_GRID, KC_G2P, KC_SORT, KC_G2P_ADJ, KC_GRID_ADJ, KC_P2G_ADJ, KC_G2P2G, KC_ADJ_PAIR, KC_COUNT };

struct TimedSpan {
  int kc;
  hipEvent_t a, b;
};

}  // namespace

struct mpm_batch {
  // configuration
  int E = 0;
  std::vector<mpm_env_desc> desc;
  int max_substeps = 0, K = 1, mode = MPM_MODE_BATCHED;
  mpm_allocator alloc{};
  bool has_alloc = false;
  hipStream_t stream = nullptr;
  std::string err;

  // layout
  std::vector<EnvDev> envs_h;
  int64_t N = 0, n_tiles = 0;   // particle positions (sum of capacities), tiles
  int64_t rows = 0;             // live particles = rows of the caller's concatenated arrays
  std::vector<int> cap_n;       // grid capacity per env (nodes per axis)
  int cell_bits = 0, key_bits = 0;
  std::vector<WorkItem> items_h;
  std::vector<int> item_off;  // [E+1]
  // the work items again for the LDS-staged kernels: [0, n) grouped by
  // material (one launch per (material, first, count) range), [n, 2n) all
  // items for the generic launch; each range in launch order (see xcd)
  struct MatRange { int mat, first, count; };
  std::vector<WorkItem> items_mat_h;
  std::vector<MatRange> mat_ranges;
  std::vector<MatRange> generic_range;
  int n_seg_max = 0;

  // device buffers
  std::vector<std::pair<void*, size_t>> allocations;
  int64_t bytes = 0;
  EnvDev* envs_d = nullptr;
  WorkItem* items_d = nullptr;
  WorkItem* items_mat_d = nullptr;
  int32_t* tile_env_d = nullptr;
  float* W[2] = {nullptr, nullptr};
  std::vector<float*> ckpt;        // [n_seg_max]
  std::vector<float*> seg;         // [K + 1], seg[0] unused
  std::vector<uint32_t*> perm;     // [n_seg_max]
  int32_t *ids_cur = nullptr, *ids_tmp = nullptr, *ids_start = nullptr;
  uint32_t *keys0 = nullptr, *vals0 = nullptr, *keys1 = nullptr, *vals1 = nullptr, *counts = nullptr;
  std::vector<float*> grid;        // [K + 1]: 0 = scratch grid, 1..K = tape grids
  std::vector<uint32_t*> flags;    // [K + 1]
  std::vector<bool> grid_dirty;    // tape grid holds a substep not yet consumed
  float* gcot = nullptr;
  float* cot[2] = {nullptr, nullptr};
  float* part = nullptr;
  double* pacc = nullptr;
  int32_t* errs = nullptr;
  int32_t* clock = nullptr;       // [E] per-env substep clocks (collider motion time)
  int32_t* clock_rec = nullptr;   // [E] the clocks at the start of the recorded forward
  float* motion_d = nullptr;     // prescribed collider motions: [E][kMaxColliders][max_substeps] rows of kMotionRow
                                 // floats
  double* gmotion_d = nullptr;   // their cotangents, same layout, FP64
  std::vector<float> motion_h;

  // state
  float* cur = nullptr;
  std::vector<int64_t> env_steps;   // host mirror of the clocks: substeps each env took since its particles were set
  bool recorded = false;
  int rec_S = 0;
  bool last_seg_taped = false;
  std::vector<int32_t> env_err_h;

  // kernel variants of the batched mode (0: one thread per particle with
  // global atomics, 1: LDS-staged), chosen by mpm_autotune
  // P2G / G2P adjoint: 2 = LDS-staged with segment reduction for blocks whose
  // particles average at least min_run per stencil base
  int var_p2g = 2, var_g2p = 1, var_g2p_adj = 2, var_p2g_adj = 1;
  int min_run = 3;
  int max_run = 8;    // runs of one stencil base are split every max_run particles
  int grid_cap = 0;   // 0: one block per work item; > 0: persistent grid of this many blocks
  int box = 0;        // LDS box budget of the LDS-staged kernels: 0 = 1024 nodes, 1 = 384 nodes
  int specialize = 1; // LDS-staged kernels: 1 = one launch per material, compiled for it; 0 = one generic launch
  int fuse = 0;       // 1: G2P of substep k and P2G of substep k + 1 in one kernel (with the segment P2G)
  int fuse_adj = 0;   // 1: P2G adjoint of substep k and G2P adjoint of substep k - 1 in one kernel
  int xcd = 0;        // 1: order each launch's items so that the blocks one XCD receives take a contiguous run
  int grid_list = 0;  // 1 / 2: the grid passes take 64 / 16 tiles per block and run only the flagged ones
  int max_col = 0;     // most colliders an env holds (slots in use): picks the grid passes' compiled variant

  // hipGraph replay of whole segments (batched mode): captured on a private
  // stream, replayed on the caller's stream, keyed by what the launches depend on
  bool use_graphs = true;
  hipStream_t cap = nullptr;
  std::map<std::tuple<int, int, int, int, int, const void*>, hipGraphExec_t> graphs;

  // timing
  bool timing = false;
  std::vector<TimedSpan> spans;
  std::vector<hipEvent_t> event_pool;
  size_t event_next = 0;
};

namespace {

const char* kVersion = "mpmx 0.1 (gfx950)";

int fail(mpm_batch* b, int code, const std::string& msg) {
  if (b) b->err = msg;
  return code;
}

#define HIPC(b, expr)                                                                     \
  do {                                                                                    \
    hipError_t _e = (expr);                                                               \
    if (_e != hipSuccess)                                                                 \
      return fail((b), MPM_DEVICE_ERROR, std::string(#expr) + ": " + hipGetErrorString(_e)); \
  } while (0)

void* dalloc(mpm_batch* b, size_t bytes) {
  if (bytes == 0) bytes = 256;
  bytes = (bytes + 255) & ~size_t(255);
  void* p = nullptr;
  if (b->has_alloc) {
    p = b->alloc.alloc(bytes, b->alloc.ctx);
  } else if (hipMalloc(&p, bytes) != hipSuccess) {
    p = nullptr;
  }
  if (p) {
    b->allocations.push_back({p, bytes});
    b->bytes += (int64_t)bytes;
  }
  return p;
}

void free_all(mpm_batch* b) {
  for (auto& a : b->allocations) {
    if (b->has_alloc)
      b->alloc.free(a.first, b->alloc.ctx);
    else
      (void)hipFree(a.first);
  }
  b->allocations.clear();
  b->bytes = 0;
  for (auto e : b->event_pool) (void)hipEventDestroy(e);
  b->event_pool.clear();
  for (auto& g : b->graphs) (void)hipGraphExecDestroy(g.second);
  b->graphs.clear();
  if (b->cap) (void)hipStreamDestroy(b->cap);
  b->cap = nullptr;
}

int ceil_log2(uint64_t v) {
  int b = 0;
  while ((uint64_t(1) << b) < v) ++b;
  return b;
}

// ---------------------------------------------------------------- timing
hipEvent_t next_event(mpm_batch* b) {
  if (b->event_next == b->event_pool.size()) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    b->event_pool.push_back(e);
  }
  return b->event_pool[b->event_next++];
}

struct Span {
  mpm_batch* b;
  int kc;
  hipEvent_t a = nullptr;
  Span(mpm_batch* b_, int kc_) : b(b_), kc(kc_) {
    if (b->timing) {
      a = next_event(b);
      if (a) (void)hipEventRecord(a, b->stream);
    }
  }
  ~Span() {
    if (b->timing && a) {
      hipEvent_t z = next_event(b);
      if (z) {
        (void)hipEventRecord(z, b->stream);
        b->spans.push_back({kc, a, z});
      }
    }
  }
};

// the (material, first, count) ranges the LDS-staged kernels launch over:
// one per material, or one generic range (material -1) over all items in env order
const std::vector<mpm_batch::MatRange>& launch_ranges(mpm_batch* b) {
  if (b->specialize) return b->mat_ranges;
  const int n = (int)b->items_h.size();
  b->generic_range.assign(1, {-1, n, n});
  return b->generic_range;
}

// ---------------------------------------------------------------- one substep
// batched-mode pieces of a substep
void batched_p2g(mpm_batch* b, const float* in, int gi, int kc) {
  const hipStream_t s = b->stream;
  const int ni = (int)b->items_h.size();
  const int runs = b->min_run | (b->max_run << 16);
  Span sp(b, KC_P2G);
  if (b->var_p2g == 0) launch_p2g_direct(in, b->N, b->envs_d, b->items_d, ni, b->grid[gi], b->flags[gi], b->errs, kc, s);
  for (const auto& r : launch_ranges(b)) {
    const WorkItem* it = b->items_mat_d + r.first;
    if (b->var_p2g == 2) launch_p2g_seg(in, b->N, b->envs_d, it, r.count, b->grid[gi], b->flags[gi], b->errs, runs, kc, b->grid_cap, b->box, r.mat, s);
    else if (b->var_p2g == 1) launch_p2g_lds(in, b->N, b->envs_d, it, r.count, b->grid[gi], b->flags[gi], b->errs, kc, b->grid_cap, b->box, r.mat, s);
    else if (b->var_p2g == 3) launch_p2g_pull(in, b->N, b->envs_d, it, r.count, b->grid[gi], b->flags[gi], b->errs, kc, b->grid_cap, b->box, r.mat, s);
  }
}

void batched_grid(mpm_batch* b, int gi, int clear, int k_rel) {
  Span sp(b, KC_GRID);
  if (b->grid_list)
    launch_grid_update_chunked(b->envs_d, b->tile_env_d, b->n_tiles, b->grid[gi], b->flags[gi], b->clock, 0.0,
                               k_rel, clear, b->motion_d, b->grid_list == 2 ? 16 : 64, b->stream, b->max_col);
  else
    launch_grid_update(b->envs_d, b->tile_env_d, 0, b->n_tiles, b->grid[gi], b->flags[gi], b->clock, 0.0, k_rel,
                       clear, b->motion_d, b->stream, b->max_col);
}

void batched_g2p(mpm_batch* b, const float* in, float* out, int gi, int kc) {
  const hipStream_t s = b->stream;
  const int ni = (int)b->items_h.size();
  Span sp(b, KC_G2P);
  if (b->var_g2p == 0) launch_g2p_direct(in, out, b->N, b->envs_d, b->items_d, ni, b->grid[gi], b->errs, kc, s);
  else
    for (const auto& r : launch_ranges(b))
      launch_g2p_lds(in, out, b->N, b->envs_d, b->items_mat_d + r.first, r.count, b->grid[gi],
                     b->errs, kc, b->grid_cap, b->box, r.mat, s);
}

// G2P of substep kc from grid gi_in fused with P2G of substep kc + 1 into grid gi_out
void batched_g2p2g(mpm_batch* b, const float* in, float* out, int gi_in, int gi_out, int kc) {
  const hipStream_t s = b->stream;
  const int runs = b->min_run | (b->max_run << 16);
  Span sp(b, KC_G2P2G);
  for (const auto& r : launch_ranges(b)) {
    if (b->var_p2g == 3)
      launch_g2p2g_pull(in, out, b->N, b->envs_d, b->items_mat_d + r.first, r.count, b->grid[gi_in],
                        b->grid[gi_out], b->flags[gi_out], b->errs, kc, b->box, r.mat, s);
    else
      launch_g2p2g(in, out, b->N, b->envs_d, b->items_mat_d + r.first, r.count, b->grid[gi_in],
                   b->grid[gi_out], b->flags[gi_out], b->errs, runs, kc, b->box, r.mat, s);
  }
}

// the forward fusion pairs the G2P with the per-cell-run or the pull scatter
bool fused(const mpm_batch* b) {
  return b->mode != MPM_MODE_PLAIN && b->fuse && (b->var_p2g == 2 || b->var_p2g == 3);
}

void substep(mpm_batch* b, const float* in, float* out, int gi, int clear, int k_rel, int kc) {
  float* g = b->grid[gi];
  uint32_t* fl = b->flags[gi];
  const hipStream_t s = b->stream;
  if (b->mode == MPM_MODE_PLAIN) {
    for (int e = 0; e < b->E; ++e) {
      const int i0 = b->item_off[e], ni = b->item_off[e + 1] - i0;
      const EnvDev& eh = b->envs_h[e];
      const int64_t nt = (int64_t)eh.T * eh.T * eh.T;
      { Span sp(b, KC_P2G); launch_p2g_direct(in, b->N, b->envs_d, b->items_d + i0, ni, g, fl, b->errs, kc, s); }
      { Span sp(b, KC_GRID); launch_grid_update(b->envs_d, b->tile_env_d, eh.tile_off, nt, g, fl, b->clock, 0.0, k_rel, clear, b->motion_d, s, b->max_col); }
      { Span sp(b, KC_G2P); launch_g2p_direct(in, out, b->N, b->envs_d, b->items_d + i0, ni, g, b->errs, kc, s); }
    }
  } else {
    batched_p2g(b, in, gi, kc);
    batched_grid(b, gi, clear, k_rel);
    batched_g2p(b, in, out, gi, kc);
  }
}

// batched-mode pieces of a substep's adjoint
void batched_g2p_adj(mpm_batch* b, const float* st, const float* st_next, const float* cot_in, int gi, int kc) {
  const hipStream_t s = b->stream;
  const int ni = (int)b->items_h.size();
  const int runs = b->min_run | (b->max_run << 16);
  float* g = b->grid[gi];
  Span sp(b, KC_G2P_ADJ);
  if (b->var_g2p_adj == 0) launch_g2p_adjoint_direct(st, st_next, cot_in, b->part, b->N, b->envs_d, b->items_d, ni, g, b->gcot, b->pacc, kc, s);
  for (const auto& r : launch_ranges(b)) {
    const WorkItem* it = b->items_mat_d + r.first;
    if (b->var_g2p_adj == 2) launch_g2p_adjoint_seg(st, st_next, cot_in, b->part, b->N, b->envs_d, it, r.count, g, b->gcot, b->pacc, runs, kc, b->grid_cap, b->box, r.mat, s);
    else if (b->var_g2p_adj == 1) launch_g2p_adjoint_lds(st, st_next, cot_in, b->part, b->N, b->envs_d, it, r.count, g, b->gcot, b->pacc, kc, b->grid_cap, b->box, r.mat, s);
    else if (b->var_g2p_adj == 3) launch_g2p_adjoint_pull(st, st_next, cot_in, b->part, b->N, b->envs_d, it, r.count, g, b->gcot, b->pacc, kc, b->grid_cap, b->box, r.mat, s);
  }
}

void batched_grid_adj(mpm_batch* b, int gi, int k_rel) {
  Span sp(b, KC_GRID_ADJ);
  if (b->grid_list)
    launch_grid_adjoint_chunked(b->envs_d, b->tile_env_d, b->n_tiles, b->grid[gi], b->flags[gi], b->gcot, b->clock,
                                0.0, k_rel, b->motion_d, b->gmotion_d, b->grid_list == 2 ? 16 : 64, b->stream,
                                b->max_col);
  else
    launch_grid_adjoint(b->envs_d, b->tile_env_d, 0, b->n_tiles, b->grid[gi], b->flags[gi], b->gcot, b->clock, 0.0,
                        k_rel, b->motion_d, b->gmotion_d, b->stream, b->max_col);
}

void batched_p2g_adj(mpm_batch* b, const float* st, const float* cot_in, float* cot_out, int kc) {
  const hipStream_t s = b->stream;
  const int ni = (int)b->items_h.size();
  Span sp(b, KC_P2G_ADJ);
  if (b->var_p2g_adj == 0) launch_p2g_adjoint_direct(st, b->part, cot_out, b->N, b->envs_d, b->items_d, ni, b->gcot, b->pacc, kc, cot_in, s);
  else
    for (const auto& r : launch_ranges(b))
      launch_p2g_adjoint_lds(st, b->part, cot_out, b->N, b->envs_d, b->items_mat_d + r.first, r.count, b->gcot, b->pacc, kc, cot_in, b->grid_cap, b->box, r.mat, s);
}

// P2G adjoint of substep kc (state st) fused with the G2P adjoint of substep
// kc - 1 (state st_prev, grid gi_prev); cot_end: the segment's incoming cotangent
void batched_adj_pair(mpm_batch* b, const float* st_prev, const float* st, const float* cot_end, int gi_prev, int kc) {
  const hipStream_t s = b->stream;
  const int runs = b->min_run | (b->max_run << 16);
  Span sp(b, KC_ADJ_PAIR);
  for (const auto& r : launch_ranges(b)) {
    if (b->var_g2p_adj == 3)
      launch_adj_pair_pull(st_prev, st, b->part, cot_end, b->N, b->envs_d, b->items_mat_d + r.first, r.count,
                           b->grid[gi_prev], b->gcot, b->pacc, kc, b->box, r.mat, s);
    else
      launch_adj_pair(st_prev, st, b->part, cot_end, b->N, b->envs_d, b->items_mat_d + r.first,
                      r.count, b->grid[gi_prev], b->gcot, b->pacc, runs, kc, b->box, r.mat, s);
  }
}

bool fused_adj(const mpm_batch* b) { return b->mode != MPM_MODE_PLAIN && b->fuse_adj; }

void adjoint_substep(mpm_batch* b, const float* st, const float* st_next, const float* cot_in, float* cot_out, int gi,
                     int k_rel, int kc) {
  if (b->mode == MPM_MODE_PLAIN) {
    float* g = b->grid[gi];
    uint32_t* fl = b->flags[gi];
    const hipStream_t s = b->stream;
    for (int e = 0; e < b->E; ++e) {
      const int i0 = b->item_off[e], ni = b->item_off[e + 1] - i0;
      const EnvDev& eh = b->envs_h[e];
      const int64_t nt = (int64_t)eh.T * eh.T * eh.T;
      { Span sp(b, KC_G2P_ADJ); launch_g2p_adjoint_direct(st, st_next, cot_in, b->part, b->N, b->envs_d, b->items_d + i0, ni, g, b->gcot, b->pacc, kc, s); }
      { Span sp(b, KC_GRID_ADJ); launch_grid_adjoint(b->envs_d, b->tile_env_d, eh.tile_off, nt, g, fl, b->gcot, b->clock, 0.0, k_rel, b->motion_d, b->gmotion_d, s, b->max_col); }
      { Span sp(b, KC_P2G_ADJ); launch_p2g_adjoint_direct(st, b->part, cot_out, b->N, b->envs_d, b->items_d + i0, ni, b->gcot, b->pacc, kc, cot_in, s); }
    }
  } else {
    batched_g2p_adj(b, st, st_next, cot_in, gi, kc);
    batched_grid_adj(b, gi, k_rel);
    batched_p2g_adj(b, st, cot_in, cot_out, kc);
  }
}

// sorts `src` by (env, tile, cell); writes the permuted state to `dst`, the
// permutation to `perm_out` (if not null) and updates ids_cur
void sort_into(mpm_batch* b, const float* src, float* dst, uint32_t* perm_out) {
  Span sp(b, KC_SORT);
  const hipStream_t s = b->stream;
  launch_keys(src, b->N, b->envs_d, b->items_d, (int)b->items_h.size(), b->keys0, b->vals0, b->cell_bits, s);
  const int which = launch_radix_sort(b->keys0, b->vals0, b->keys1, b->vals1, b->counts, b->N, b->key_bits, s);
  const uint32_t* pv = which ? b->vals1 : b->vals0;
  if (perm_out) {
    (void)hipMemcpyAsync(perm_out, pv, sizeof(uint32_t) * b->N, hipMemcpyDeviceToDevice, s);
    pv = perm_out;
  }
  launch_permute_state(src, dst, b->N, pv, b->ids_cur, b->ids_tmp, s);
  launch_copy_i32(b->ids_tmp, b->ids_cur, b->N, s);
}

void clear_dirty_tapes(mpm_batch* b) {
  for (int k = 1; k <= b->K; ++k)
    if (b->grid_dirty[k]) {
      launch_grid_clear_flagged(b->n_tiles, b->grid[k], b->flags[k], b->stream);
      b->grid_dirty[k] = false;
    }
}

float* other_work(mpm_batch* b, const float* in) { return in == b->W[0] ? b->W[1] : b->W[0]; }

bool graphs_on(const mpm_batch* b) { return b->mode == MPM_MODE_BATCHED && b->use_graphs && !b->timing; }

// Forward segment j: sort `src` into the segment's first buffer (its
// checkpoint when recording), run Kj substeps, advance the device clock.
// With dry = true nothing is launched; the return value (the buffer that
// holds the segment's last state) depends only on the arguments.
const float* fwd_segment(mpm_batch* b, int j, int Kj, bool record, bool tape, const float* src, bool dry) {
  float* dst0 = record ? b->ckpt[j] : other_work(b, src);
  if (!dry && b->N > 0) sort_into(b, src, dst0, record ? b->perm[j] : nullptr);
  const float* in = dst0;
  const bool run = !dry && b->N > 0;
  if (fused(b)) {
    // P2G(0), grid(0), then G2P(k) + P2G(k+1) in one kernel and grid(k+1), then G2P(K-1)
    auto gi = [&](int k) { return tape ? k + 1 : 0; };
    const int clear = tape ? 0 : 1;
    if (run && Kj > 0) {
      batched_p2g(b, in, gi(0), j * b->K);
      batched_grid(b, gi(0), clear, 0);
    }
    for (int k = 0; k < Kj; ++k) {
      float* out = tape ? b->seg[k + 1] : other_work(b, in);
      if (run) {
        if (k + 1 < Kj) {
          batched_g2p2g(b, in, out, gi(k), gi(k + 1), j * b->K + k);
          batched_grid(b, gi(k + 1), clear, k + 1);
        } else {
          batched_g2p(b, in, out, gi(k), j * b->K + k);
        }
      }
      in = out;
    }
  } else {
    for (int k = 0; k < Kj; ++k) {
      float* out = tape ? b->seg[k + 1] : other_work(b, in);
      if (run) substep(b, in, out, tape ? k + 1 : 0, tape ? 0 : 1, k, j * b->K + k);
      in = out;
    }
  }
  if (!dry) launch_advance_clocks(b->clock, b->envs_d, b->E, j * b->K, Kj, b->stream);
  return in;
}

// Backward segment j: recompute it into the tape (unless taped), run the
// adjoint substeps in reverse from cot[c], undo the segment's sort.
// Returns the index of the cotangent buffer that holds the result.
int bwd_segment(mpm_batch* b, int j, int Kj, bool have_tape, int c) {
  if (!have_tape) {   // recompute the segment's tape from its checkpoint (grid k + 1 holds substep k)
    const float* in = b->ckpt[j];
    if (fused(b) && Kj > 0) {
      batched_p2g(b, in, 1, j * b->K);
      batched_grid(b, 1, 0, 0);
      for (int k = 0; k < Kj; ++k) {
        if (k + 1 < Kj) {
          batched_g2p2g(b, in, b->seg[k + 1], k + 1, k + 2, j * b->K + k);
          batched_grid(b, k + 2, 0, k + 1);
        } else {
          batched_g2p(b, in, b->seg[k + 1], k + 1, j * b->K + k);
        }
        in = b->seg[k + 1];
      }
    } else {
      for (int k = 0; k < Kj; ++k) {
        substep(b, in, b->seg[k + 1], k + 1, 0, k, j * b->K + k);
        in = b->seg[k + 1];
      }
    }
  }
  auto state = [&](int k) -> const float* { return k == 0 ? b->ckpt[j] : b->seg[k]; };
  if (fused_adj(b) && Kj > 1) {
    // G2P adjoint of the last substep, then [P2G adjoint k + G2P adjoint k - 1,
    // grid adjoint k - 1] down to k = 1, then the P2G adjoint of substep 0. Only
    // the segment's incoming cotangent and the result live in HBM; the result
    // goes where the one-substep-at-a-time schedule leaves it
    const float* cot_end = b->cot[c];
    float* cot_res = b->cot[c ^ (Kj & 1)];
    batched_g2p_adj(b, state(Kj - 1), b->seg[Kj], cot_end, Kj, j * b->K + Kj - 1);
    batched_grid_adj(b, Kj, Kj - 1);
    for (int k = Kj - 1; k >= 1; --k) {
      batched_adj_pair(b, state(k - 1), state(k), cot_end, k, j * b->K + k);
      batched_grid_adj(b, k, k - 1);
    }
    batched_p2g_adj(b, state(0), cot_end, cot_res, j * b->K);
    c ^= Kj & 1;
  } else {
    for (int k = Kj - 1; k >= 0; --k) {
      adjoint_substep(b, state(k), b->seg[k + 1], b->cot[c], b->cot[c ^ 1], k + 1, k, j * b->K + k);
      c ^= 1;
    }
  }
  launch_unpermute(b->cot[c], b->cot[c ^ 1], b->N, b->perm[j], b->stream);
  return c ^ 1;
}

// runs `issue` directly, or as a cached graph replayed on the caller's stream
template <class Fn>
int run_maybe_graph(mpm_batch* b, std::tuple<int, int, int, int, int, const void*> key, Fn&& issue) {
  if (!graphs_on(b)) {
    issue();
    return MPM_OK;
  }
  auto it = b->graphs.find(key);
  if (it == b->graphs.end()) {
    if (!b->cap) HIPC(b, hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking));
    const hipStream_t user = b->stream;
    b->stream = b->cap;
    hipError_t e0 = hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal);
    if (e0 != hipSuccess) { b->stream = user; return fail(b, MPM_DEVICE_ERROR, std::string("hipStreamBeginCapture: ") + hipGetErrorString(e0)); }
    issue();
    hipGraph_t g = nullptr;
    hipError_t e1 = hipStreamEndCapture(b->cap, &g);
    b->stream = user;
    if (e1 != hipSuccess) return fail(b, MPM_DEVICE_ERROR, std::string("hipStreamEndCapture: ") + hipGetErrorString(e1));
    hipGraphExec_t ex = nullptr;
    hipError_t e2 = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e2 != hipSuccess) return fail(b, MPM_DEVICE_ERROR, std::string("hipGraphInstantiate: ") + hipGetErrorString(e2));
    it = b->graphs.emplace(key, ex).first;
  }
  HIPC(b, hipGraphLaunch(it->second, b->stream));
  return MPM_OK;
}

void drop_graphs(mpm_batch* b) {
  for (auto& g : b->graphs) (void)hipGraphExecDestroy(g.second);
  b->graphs.clear();
}

// Workgroups of a launch go to the eight XCDs in turn (block i to XCD i mod
// 8), and each XCD has its own L2. Reordering a range so that block i takes
// item start(i mod 8) + i / 8 gives every XCD one contiguous run of items:
// the same few envs' grid lines then stay in one L2. A bijection for any n.
void xcd_order(std::vector<WorkItem>& v, size_t first) {
  constexpr size_t kXcd = 8;
  const size_t n = v.size() - first, q = n / kXcd, r = n % kXcd;
  const std::vector<WorkItem> src(v.begin() + first, v.end());
  for (size_t i = 0; i < n; ++i) {
    const size_t x = i % kXcd, j = i / kXcd;
    v[first + i] = src[x * q + std::min(x, r) + j];
  }
}

int upload_items(mpm_batch* b) {
  // items grouped by material (env order kept inside a group), then all items
  std::vector<mpm_batch::MatRange> ranges;
  b->items_mat_h.clear();
  for (int m = 0; m < MAT_COUNT; ++m) {
    const int first = (int)b->items_mat_h.size();
    for (const WorkItem& it : b->items_h)
      if (b->envs_h[it.env].material == m) b->items_mat_h.push_back(it);
    const int count = (int)b->items_mat_h.size() - first;
    if (count > 0) ranges.push_back({m, first, count});
    if (b->xcd) xcd_order(b->items_mat_h, first);
  }
  const size_t gen = b->items_mat_h.size();
  b->items_mat_h.insert(b->items_mat_h.end(), b->items_h.begin(), b->items_h.end());
  if (b->xcd) xcd_order(b->items_mat_h, gen);
  if (!b->items_mat_h.empty())
    HIPC(b, hipMemcpyAsync(b->items_mat_d, b->items_mat_h.data(), sizeof(WorkItem) * b->items_mat_h.size(),
                           hipMemcpyHostToDevice, b->stream));
  bool same = ranges.size() == b->mat_ranges.size();
  for (size_t i = 0; same && i < ranges.size(); ++i)
    same = ranges[i].mat == b->mat_ranges[i].mat && ranges[i].first == b->mat_ranges[i].first &&
           ranges[i].count == b->mat_ranges[i].count;
  if (!same) {
    b->mat_ranges = ranges;
    drop_graphs(b);   // captured launches name the ranges
  }
  return MPM_OK;
}

int upload_envs(mpm_batch* b) {
  int most = 0;
  for (const EnvDev& e : b->envs_h) most = std::max(most, (int)e.n_col);
  if (most != b->max_col) {
    b->max_col = most;
    drop_graphs(b);   // captured grid passes name their kernel variant
  }
  HIPC(b, hipMemcpyAsync(b->envs_d, b->envs_h.data(), sizeof(EnvDev) * b->E, hipMemcpyHostToDevice, b->stream));
  const int rc = upload_items(b);
  if (rc != MPM_OK) return rc;
  launch_prep_params(b->envs_d, b->E, b->stream);
  HIPC(b, hipGetLastError());
  return MPM_OK;
}

// recomputes item counts, compact row offsets and the live total from envs_h
void refresh_layout(mpm_batch* b) {
  int64_t row = 0;
  for (int e = 0; e < b->E; ++e) {
    EnvDev& h = b->envs_h[e];
    h.row_off = row;
    row += h.p_cnt;
    for (int i = b->item_off[e]; i < b->item_off[e + 1]; ++i) {
      WorkItem& it = b->items_h[i];
      const int64_t s0 = it.start - h.p_off;
      it.count = (int32_t)std::max<int64_t>(0, std::min<int64_t>(it.cap, h.p_cnt - s0));
    }
  }
  b->rows = row;
}

int check_env(mpm_batch* b, int32_t env, bool allow_all) {
  if (env == -1 && allow_all) return MPM_OK;
  if (env < 0 || env >= b->E) return fail(b, MPM_INVALID_ARG, "env index out of range");
  return MPM_OK;
}

}  // namespace

namespace mpmx {

int64_t env_snapshot_floats(const mpm_batch* b, int env) {
  return env < 0 || env >= b->E ? 0 : 25 * b->envs_h[env].p_cnt;
}

int env_snapshot(mpm_batch* b, int env, float* dst, int64_t* steps) {
  if (env < 0 || env >= b->E || !dst) return fail(b, MPM_INVALID_ARG, "snapshot: bad env or buffer");
  const EnvDev& h = b->envs_h[env];
  launch_env_rows(b->cur, b->ids_cur, b->N, h.p_off, h.p_cnt, dst, 1, b->stream);
  HIPC(b, hipGetLastError());
  if (steps) *steps = b->env_steps[env];
  return MPM_OK;
}

int env_restore(mpm_batch* b, int env, const float* src, int64_t steps) {
  if (env < 0 || env >= b->E || !src) return fail(b, MPM_INVALID_ARG, "restore: bad env or buffer");
  const EnvDev& h = b->envs_h[env];
  clear_dirty_tapes(b);
  launch_env_rows(b->cur, b->ids_cur, b->N, h.p_off, h.p_cnt, const_cast<float*>(src), 0, b->stream);
  launch_set_clock(b->clock, env, b->E, (int32_t)steps, b->stream);
  HIPC(b, hipGetLastError());
  b->env_steps[env] = steps;
  b->recorded = false;
  b->last_seg_taped = false;
  return MPM_OK;
}

int64_t env_row_offset(const mpm_batch* b, int env) { return env < 0 || env >= b->E ? 0 : b->envs_h[env].row_off; }

void* batch_stream(const mpm_batch* b) { return (void*)b->stream; }

}  // namespace mpmx

namespace {

struct TuneChoice {
  int p2g, g2p, g2p_adj, p2g_adj, min_run, grid_cap, max_run, box, specialize, fuse, fuse_adj, xcd, grid_list;
};

// shape signature -> choice, shared by batches of the same shape in the process
std::map<std::string, TuneChoice>& tune_cache() {
  static std::map<std::string, TuneChoice> c;
  return c;
}

std::string shape_signature(const mpm_batch* b) {
  std::string sig = std::to_string(b->K) + ":";
  for (const EnvDev& e : b->envs_h)
    sig += std::to_string(e.n) + "," + std::to_string(e.material) + "," + std::to_string(e.p_cnt) + ";";
  return sig;
}

void apply_choice(mpm_batch* b, const TuneChoice& c) {
  b->var_p2g = c.p2g; b->var_g2p = c.g2p; b->var_g2p_adj = c.g2p_adj; b->var_p2g_adj = c.p2g_adj;
  b->min_run = c.min_run;
  b->grid_cap = c.grid_cap;
  b->max_run = c.max_run;
  b->box = c.box;
  b->specialize = c.specialize;
  b->fuse = c.fuse;
  b->fuse_adj = c.fuse_adj;
  b->grid_list = c.grid_list;
  if (b->xcd != c.xcd) {
    b->xcd = c.xcd;
    (void)upload_items(b);
  }
  drop_graphs(b);
}

}  // namespace

extern "C" {

const char* mpm_version(void) { return kVersion; }

const char* mpm_last_error(const mpm_batch* b) {
  if (!b) return "null batch";
  return b->err.c_str();
}

int64_t mpm_memory_bytes(const mpm_batch* b) { return b ? b->bytes : 0; }

int mpm_batch_create(const mpm_batch_desc* d, const mpm_allocator* a, void* stream, mpm_batch** out) {
  if (!d || !out || !d->envs) return MPM_INVALID_ARG;
  *out = nullptr;
  if (d->n_envs < 1 || d->ckpt_every < 1 || d->max_substeps < 0) return MPM_INVALID_ARG;
  if (d->mode != MPM_MODE_PLAIN && d->mode != MPM_MODE_BATCHED) return MPM_INVALID_ARG;
  if (a && (!a->alloc || !a->free)) return MPM_INVALID_ARG;
  int64_t N = 0, tiles = 0;
  uint64_t max_cells = 1;
  for (int e = 0; e < d->n_envs; ++e) {
    const mpm_env_desc& v = d->envs[e];
    if (v.n < 12 || v.n % 4 != 0 || v.n > 1024) return MPM_INVALID_ARG;
    if (v.material < 0 || v.material > MPM_FLUID_PAPER) return MPM_INVALID_ARG;
    if (v.n_particles < 0 || !(v.dt > 0.f) || v.wall < 0 || 2 * v.wall + 3 > v.n) return MPM_INVALID_ARG;
    N += v.n_particles;
    tiles += (int64_t)(v.n / 4) * (v.n / 4) * (v.n / 4);
    max_cells = std::max<uint64_t>(max_cells, (uint64_t)v.n * v.n * v.n);
  }
  if (N >= (int64_t(1) << 31)) return MPM_INVALID_ARG;
  const int cell_bits = ceil_log2(max_cells);
  const int env_bits = ceil_log2((uint64_t)d->n_envs);
  if (cell_bits + env_bits > 32) return MPM_INVALID_ARG;

  mpm_batch* b = new mpm_batch();
  b->E = d->n_envs;
  b->desc.assign(d->envs, d->envs + d->n_envs);
  b->max_substeps = d->max_substeps;
  b->K = d->ckpt_every;
  b->mode = d->mode;
  if (a) { b->alloc = *a; b->has_alloc = true; }
  b->stream = (hipStream_t)stream;
  b->N = N;
  b->n_tiles = tiles;
  b->cell_bits = cell_bits;
  b->key_bits = std::max(1, cell_bits + env_bits);
  b->n_seg_max = std::max(1, (b->max_substeps + b->K - 1) / b->K);

  // env table and work items
  b->envs_h.resize(b->E);
  b->item_off.assign(b->E + 1, 0);
  int64_t p_off = 0, t_off = 0;
  std::vector<int32_t> tile_env(std::max<int64_t>(tiles, 1), 0);
  for (int e = 0; e < b->E; ++e) {
    const mpm_env_desc& v = d->envs[e];
    EnvDev h;
    std::memset(&h, 0, sizeof(h));
    h.n = v.n; h.T = v.n / 4; h.material = v.material; h.wall = v.wall;
    h.p_off = p_off; h.p_cnt = v.n_particles; h.p_cap = v.n_particles; h.tile_off = t_off;
    h.row_off = p_off; h.nsub = 0;
    for (int ci = 0; ci < kMaxColliders; ++ci) h.col[ci].motion_off = (e * kMaxColliders + ci) * b->max_substeps;
    h.dt = v.dt; h.fn = (float)v.n; h.dx = 1.f / (float)v.n;
    h.gx = v.gravity[0]; h.gy = v.gravity[1]; h.gz = v.gravity[2];
    h.rho = 1.0; h.nu = 0.0;  // inert until mpm_set_material
    b->envs_h[e] = h;
    b->item_off[e] = (int)b->items_h.size();
    for (int64_t s0 = 0; s0 < v.n_particles; s0 += kItemSize) {
      WorkItem it;
      it.env = e;
      it.start = p_off + s0;
      it.count = (int32_t)std::min<int64_t>(kItemSize, v.n_particles - s0);
      it.cap = it.count;
      it.pad = 0;
      b->items_h.push_back(it);
    }
    const int64_t nt = (int64_t)h.T * h.T * h.T;
    for (int64_t t = 0; t < nt; ++t) tile_env[t_off + t] = e;
    p_off += v.n_particles;
    t_off += nt;
  }
  b->item_off[b->E] = (int)b->items_h.size();
  b->rows = N;
  for (int e = 0; e < b->E; ++e) b->cap_n.push_back(d->envs[e].n);
  b->env_err_h.assign(b->E, 0);
  b->env_steps.assign(b->E, 0);

  const size_t state_bytes = sizeof(float) * 24 * (size_t)std::max<int64_t>(N, 1);
  const size_t grid_bytes = sizeof(float) * 512 * (size_t)std::max<int64_t>(tiles, 1);
  const size_t flag_bytes = sizeof(uint32_t) * (size_t)std::max<int64_t>(tiles, 1);
  const size_t nbytes_i = sizeof(int32_t) * (size_t)std::max<int64_t>(N, 1);
  bool ok = true;
  auto A = [&](size_t bytes) -> void* {
    void* p = ok ? dalloc(b, bytes) : nullptr;
    if (!p) ok = false;
    return p;
  };
  b->envs_d = (EnvDev*)A(sizeof(EnvDev) * b->E);
  b->items_d = (WorkItem*)A(sizeof(WorkItem) * std::max<size_t>(b->items_h.size(), 1));
  b->items_mat_d = (WorkItem*)A(sizeof(WorkItem) * std::max<size_t>(2 * b->items_h.size(), 1));
  b->tile_env_d = (int32_t*)A(sizeof(int32_t) * tile_env.size());
  b->W[0] = (float*)A(state_bytes);
  b->W[1] = (float*)A(state_bytes);
  for (int j = 0; j < b->n_seg_max; ++j) b->ckpt.push_back((float*)A(state_bytes));
  b->seg.push_back(nullptr);
  for (int k = 1; k <= b->K; ++k) b->seg.push_back((float*)A(state_bytes));
  for (int j = 0; j < b->n_seg_max; ++j) b->perm.push_back((uint32_t*)A(nbytes_i));
  b->ids_cur = (int32_t*)A(nbytes_i);
  b->ids_tmp = (int32_t*)A(nbytes_i);
  b->ids_start = (int32_t*)A(nbytes_i);
  b->keys0 = (uint32_t*)A(nbytes_i);
  b->vals0 = (uint32_t*)A(nbytes_i);
  b->keys1 = (uint32_t*)A(nbytes_i);
  b->vals1 = (uint32_t*)A(nbytes_i);
  const int64_t rs_blocks = (std::max<int64_t>(N, 1) + RS_TILE - 1) / RS_TILE;
  b->counts = (uint32_t*)A(sizeof(uint32_t) * 256 * (rs_blocks + 1));   // per-block digit counts + digit totals
  for (int k = 0; k <= b->K; ++k) {
    b->grid.push_back((float*)A(grid_bytes));
    b->flags.push_back((uint32_t*)A(flag_bytes));
  }
  b->grid_dirty.assign(b->K + 1, false);
  b->gcot = (float*)A(grid_bytes);
  b->cot[0] = (float*)A(state_bytes);
  b->cot[1] = (float*)A(state_bytes);
  b->part = (float*)A(sizeof(float) * 12 * (size_t)std::max<int64_t>(N, 1));
  b->pacc = (double*)A(sizeof(double) * 8 * b->E);
  b->errs = (int32_t*)A(sizeof(int32_t) * b->E);
  b->clock = (int32_t*)A(sizeof(int32_t) * b->E);
  b->clock_rec = (int32_t*)A(sizeof(int32_t) * b->E);
  const size_t motion_rows = (size_t)kMaxColliders * b->E * b->max_substeps;
  b->motion_d = (float*)A(sizeof(float) * kMotionRow * motion_rows);
  b->gmotion_d = (double*)A(sizeof(double) * kMotionRow * motion_rows);
  if (!ok) {
    free_all(b);
    delete b;
    return MPM_OUT_OF_MEMORY;
  }
  const hipStream_t s = b->stream;
  auto zero = [&](void* p, size_t bytes) { launch_fill_u32(p, 0u, (int64_t)(bytes / 4), s); };
  int rc = MPM_OK;
  do {
    if (hipMemcpyAsync(b->items_d, b->items_h.data(), sizeof(WorkItem) * b->items_h.size(), hipMemcpyHostToDevice, s) != hipSuccess ||
        hipMemcpyAsync(b->tile_env_d, tile_env.data(), sizeof(int32_t) * tile_env.size(), hipMemcpyHostToDevice, s) != hipSuccess) {
      rc = MPM_DEVICE_ERROR;
      break;
    }
    for (int k = 0; k <= b->K; ++k) { zero(b->grid[k], grid_bytes); zero(b->flags[k], flag_bytes); }
    zero(b->gcot, grid_bytes);
    zero(b->W[0], state_bytes);
    zero(b->errs, sizeof(int32_t) * b->E);
    zero(b->clock, sizeof(int32_t) * b->E);
    zero(b->clock_rec, sizeof(int32_t) * b->E);
    zero(b->motion_d, sizeof(float) * kMotionRow * motion_rows);
    zero(b->gmotion_d, sizeof(double) * kMotionRow * motion_rows);
    // identity ids and an F = I rest state until particles are set
    rc = upload_envs(b);
  } while (0);
  if (rc == MPM_OK && hipStreamSynchronize(s) != hipSuccess) rc = MPM_DEVICE_ERROR;
  if (rc != MPM_OK) {
    free_all(b);
    delete b;
    return rc;
  }
  b->cur = b->W[0];
  *out = b;
  return MPM_OK;
}

int mpm_batch_destroy(mpm_batch* b) {
  if (!b) return MPM_INVALID_ARG;
  (void)hipStreamSynchronize(b->stream);
  free_all(b);
  delete b;
  return MPM_OK;
}

int mpm_set_particles(mpm_batch* b, int32_t env, const float* x, const float* v, const float* C, const float* F,
                      int64_t n) {
  if (!b) return MPM_INVALID_ARG;
  int rc = check_env(b, env, true);
  if (rc) return rc;
  const int64_t want = env < 0 ? b->rows : b->envs_h[env].p_cnt;
  if (n != want) return fail(b, MPM_INVALID_ARG, "particle count does not match the env description");
  if (n > 0 && (!x || !v || !C || !F)) return fail(b, MPM_INVALID_ARG, "null particle array");
  clear_dirty_tapes(b);
  const int i0 = env < 0 ? 0 : b->item_off[env];
  const int ni = env < 0 ? (int)b->items_h.size() : b->item_off[env + 1] - b->item_off[env];
  launch_load_aos(b->items_d + i0, ni, b->envs_d, env < 0 ? 1 : 0, x, v, C, F, b->cur, b->N, b->ids_cur, b->stream);
  launch_set_clock(b->clock, env, b->E, 0, b->stream);
  HIPC(b, hipGetLastError());
  for (int e = 0; e < b->E; ++e)
    if (env < 0 || e == env) b->env_steps[e] = 0;
  b->recorded = false;
  b->last_seg_taped = false;
  return MPM_OK;
}

int mpm_get_particles(mpm_batch* b, int32_t env, float* x, float* v, float* C, float* F) {
  if (!b) return MPM_INVALID_ARG;
  int rc = check_env(b, env, true);
  if (rc) return rc;
  const int i0 = env < 0 ? 0 : b->item_off[env];
  const int ni = env < 0 ? (int)b->items_h.size() : b->item_off[env + 1] - b->item_off[env];
  launch_store_aos(b->items_d + i0, ni, b->envs_d, env < 0 ? 1 : 0, b->cur, b->N, b->ids_cur, x, v, C, F, true, b->stream);
  HIPC(b, hipGetLastError());
  return MPM_OK;
}

int mpm_configure_env(mpm_batch* b, int32_t env, const mpm_env_desc* d) {
  if (!b || !d) return MPM_INVALID_ARG;
  int rc = check_env(b, env, false);
  if (rc) return rc;
  EnvDev& h = b->envs_h[env];
  if (d->n < 12 || d->n % 4 != 0 || d->n > b->cap_n[env]) return fail(b, MPM_INVALID_ARG, "grid n above the env's capacity");
  if (d->n_particles < 0 || d->n_particles > h.p_cap) return fail(b, MPM_INVALID_ARG, "particles above the env's capacity");
  if (d->material < 0 || d->material > MPM_FLUID_PAPER) return fail(b, MPM_INVALID_ARG, "unknown material");
  if (!(d->dt > 0.f) || d->wall < 0 || 2 * d->wall + 3 > d->n) return fail(b, MPM_INVALID_ARG, "bad dt or wall");
  clear_dirty_tapes(b);
  h.n = d->n; h.T = d->n / 4; h.material = d->material; h.wall = d->wall;
  h.dt = d->dt; h.fn = (float)d->n; h.dx = 1.f / (float)d->n;
  h.gx = d->gravity[0]; h.gy = d->gravity[1]; h.gz = d->gravity[2];
  h.p_cnt = d->n_particles;
  h.n_col = 0;
  for (int ci = 0; ci < kMaxColliders; ++ci) { h.col[ci].has_collider = 0; h.col[ci].motion_len = 0; }
  refresh_layout(b);
  HIPC(b, hipMemcpyAsync(b->items_d, b->items_h.data(), sizeof(WorkItem) * b->items_h.size(), hipMemcpyHostToDevice, b->stream));
  b->recorded = false;
  b->last_seg_taped = false;
  return upload_envs(b);
}

int mpm_set_material(mpm_batch* b, int32_t env, int32_t material, const double p[8]) {
  if (!b || !p) return MPM_INVALID_ARG;
  int rc = check_env(b, env, true);
  if (rc) return rc;
  if (material < 0 || material > MPM_FLUID_PAPER) return fail(b, MPM_INVALID_ARG, "unknown material");
  const double E = p[0], nu = p[1], rho = p[2], Vp = p[3], sy = p[4], K = p[5], gam = p[6];
  if (!(nu > -1.0 && nu < 0.5)) return fail(b, MPM_INVALID_ARG, "nu must lie in (-1, 0.5)");
  if (!(E >= 0.0) || !(rho >= 0.0) || !(Vp >= 0.0) || !(sy >= 0.0) || !(K >= 0.0))
    return fail(b, MPM_INVALID_ARG, "E, rho, Vp, sigma_y and K must be finite and >= 0");
  if (material == MPM_FLUID_TAIT && !(gam > 0.0)) return fail(b, MPM_INVALID_ARG, "Tait gamma must be > 0");
  if (material == MPM_VONMISES && !(E > 0.0)) return fail(b, MPM_INVALID_ARG, "von Mises needs E > 0");
  const int e0 = env < 0 ? 0 : env, e1 = env < 0 ? b->E : env + 1;
  for (int e = e0; e < e1; ++e) {
    EnvDev& h = b->envs_h[e];
    h.material = material;
    h.E = E; h.nu = nu; h.rho = rho; h.Vp = Vp; h.sigma_y = sy; h.K = K; h.gamma = gam;
  }
  b->recorded = false;
  return upload_envs(b);
}

static void count_colliders(EnvDev& d) {
  d.n_col = 0;
  for (int ci = 0; ci < kMaxColliders; ++ci)
    if (d.col[ci].has_collider) d.n_col = ci + 1;
}

static int check_collider_index(mpm_batch* b, int32_t index) {
  if (index < 0 || index >= kMaxColliders) return fail(b, MPM_INVALID_ARG, "collider index outside [0, MPM_MAX_COLLIDERS)");
  return MPM_OK;
}

static int set_collider(mpm_batch* b, int32_t env, int32_t shape, const float c[3], const float h[3], const float v[3],
                        float alpha, float mu_b, float rounding = 0.f, int32_t index = 0) {
  if (!b) return MPM_INVALID_ARG;
  int rc = check_env(b, env, true);
  if (rc) return rc;
  if ((rc = check_collider_index(b, index))) return rc;
  if (alpha > 0.f && (!c || !h || !v)) return fail(b, MPM_INVALID_ARG, "null collider array");
  if (alpha > 0.f && !(mu_b >= 0.f)) return fail(b, MPM_INVALID_ARG, "mu_b must be >= 0");
  if (alpha > 0.f && shape == kColliderSphere && !(h[0] >= 0.f && std::isfinite(h[0])))
    return fail(b, MPM_INVALID_ARG, "the sphere radius must be finite and >= 0");
  if (!(rounding >= 0.f) || !std::isfinite(rounding))
    return fail(b, MPM_INVALID_ARG, "the rounding radius must be finite and >= 0");
  const int e0 = env < 0 ? 0 : env, e1 = env < 0 ? b->E : env + 1;
  for (int e = e0; e < e1; ++e) {
    ColDev& d = b->envs_h[e].col[index];
    d.has_collider = alpha > 0.f ? shape : 0;
    if (d.has_collider) {
      for (int a = 0; a < 3; ++a) { d.cc[a] = c[a]; d.ch[a] = h[a]; d.cv[a] = v[a]; }
      d.c_alpha = alpha;
      d.c_mu = mu_b;
    }
    d.c_round = d.has_collider == kColliderBox ? rounding : 0.f;
    d.c_axis[0] = d.c_axis[1] = 0.f;   // no rotation until mpm_set_box_rotation
    d.c_axis[2] = 1.f;
    d.c_angle = d.c_omega = 0.f;
    d.motion_len = 0;   // a prescribed motion starts from the collider it was set for
    count_colliders(b->envs_h[e]);
  }
  b->recorded = false;
  return upload_envs(b);
}

int mpm_set_box_collider(mpm_batch* b, int32_t env, const float c[3], const float h[3], const float v[3], float alpha,
                         float mu_b) {
  return set_collider(b, env, kColliderBox, c, h, v, alpha, mu_b);
}

int mpm_set_sphere_collider(mpm_batch* b, int32_t env, const float c[3], float radius, const float v[3], float alpha,
                            float mu_b) {
  const float h[3] = {radius, radius, radius};
  return set_collider(b, env, kColliderSphere, c, h, v, alpha, mu_b);
}

int mpm_set_rounded_box_collider(mpm_batch* b, int32_t env, const float c[3], const float h[3], float radius,
                                 const float v[3], float alpha, float mu_b) {
  return set_collider(b, env, kColliderBox, c, h, v, alpha, mu_b, radius);
}

int mpm_set_collider(mpm_batch* b, int32_t env, int32_t index, int32_t shape, const float center[3],
                     const float half[3], float radius, const float vel[3], float alpha, float mu_b) {
  if (!b) return MPM_INVALID_ARG;
  if (alpha > 0.f && shape == MPM_COLLIDER_SPHERE) {
    const float h[3] = {radius, radius, radius};
    return set_collider(b, env, kColliderSphere, center, h, vel, alpha, mu_b, 0.f, index);
  }
  if (alpha > 0.f && shape != MPM_COLLIDER_BOX && shape != MPM_COLLIDER_ROUNDED_BOX)
    return fail(b, MPM_INVALID_ARG, "unknown collider shape");
  return set_collider(b, env, kColliderBox, center, half, vel, alpha, mu_b,
                      shape == MPM_COLLIDER_ROUNDED_BOX ? radius : 0.f, index);
}

int mpm_set_box_rotation(mpm_batch* b, int32_t env, const float axis[3], float angle, float omega) {
  return mpm_set_collider_rotation(b, env, 0, axis, angle, omega);
}

int mpm_set_collider_rotation(mpm_batch* b, int32_t env, int32_t index, const float axis[3], float angle,
                              float omega) {
  if (!b) return MPM_INVALID_ARG;
  int rc = check_env(b, env, true);
  if (rc) return rc;
  if ((rc = check_collider_index(b, index))) return rc;
  if (!axis) return fail(b, MPM_INVALID_ARG, "null axis");
  const double len = std::sqrt((double)axis[0] * axis[0] + (double)axis[1] * axis[1] + (double)axis[2] * axis[2]);
  if (!(len > 0.0) || !std::isfinite(len) || !std::isfinite(angle) || !std::isfinite(omega))
    return fail(b, MPM_INVALID_ARG, "the axis must be nonzero and the values finite");
  const int e0 = env < 0 ? 0 : env, e1 = env < 0 ? b->E : env + 1;
  for (int e = e0; e < e1; ++e)
    if (!b->envs_h[e].col[index].has_collider) return fail(b, MPM_INVALID_ARG, "the environment has no such collider");
  for (int e = e0; e < e1; ++e) {
    ColDev& d = b->envs_h[e].col[index];
    for (int a = 0; a < 3; ++a) d.c_axis[a] = (float)(axis[a] / len);
    d.c_angle = angle;
    d.c_omega = omega;
    d.motion_len = 0;
  }
  b->recorded = false;
  return upload_envs(b);
}

int mpm_set_collider_motion(mpm_batch* b, int32_t env, const float* vel, const float* omega, int32_t n) {
  return mpm_set_collider_motion_at(b, env, 0, vel, omega, n);
}

int mpm_set_collider_motion_at(mpm_batch* b, int32_t env, int32_t index, const float* vel, const float* omega,
                               int32_t n) {
  if (!b) return MPM_INVALID_ARG;
  int rc = check_env(b, env, false);
  if (rc) return rc;
  if ((rc = check_collider_index(b, index))) return rc;
  ColDev& d = b->envs_h[env].col[index];
  const float dt = b->envs_h[env].dt;
  if (n < 0 || n > b->max_substeps) return fail(b, MPM_INVALID_ARG, "motion length outside [0, max_substeps]");
  if (n > 0 && !vel) return fail(b, MPM_INVALID_ARG, "null velocity array");
  if (n > 0 && !d.has_collider) return fail(b, MPM_INVALID_ARG, "the environment has no such collider");
  for (int64_t i = 0; i < 3 * (int64_t)n; ++i)
    if (!std::isfinite(vel[i])) return fail(b, MPM_NONFINITE, "non-finite collider velocity");
  for (int64_t i = 0; omega && i < (int64_t)n; ++i)
    if (!std::isfinite(omega[i])) return fail(b, MPM_NONFINITE, "non-finite collider angular speed");
  if (n > 0) {
    // during substep k: center c0 + dt sum_{j<k} vel_j, angle angle0 + dt sum_{j<k}
    // omega_j, both accumulated in FP64
    constexpr int W = kMotionRow;
    b->motion_h.assign(W * (size_t)n, 0.f);
    double c[3] = {d.cc[0], d.cc[1], d.cc[2]}, th = d.c_angle;
    for (int k = 0; k < n; ++k) {
      const double om = omega ? (double)omega[k] : (double)d.c_omega;
      for (int a = 0; a < 3; ++a) {
        b->motion_h[W * k + a] = (float)c[a];
        b->motion_h[W * k + 3 + a] = vel[3 * k + a];
      }
      b->motion_h[W * k + 6] = (float)th;
      b->motion_h[W * k + 7] = (float)om;
      for (int a = 0; a < 3; ++a) c[a] += (double)dt * (double)vel[3 * k + a];
      th += (double)dt * om;
    }
    HIPC(b, hipMemcpyAsync(b->motion_d + W * (size_t)d.motion_off, b->motion_h.data(), sizeof(float) * W * (size_t)n,
                           hipMemcpyHostToDevice, b->stream));
    HIPC(b, hipStreamSynchronize(b->stream));   // the host rows are reused by the next call
  }
  d.motion_len = n;
  b->recorded = false;
  return upload_envs(b);
}

int mpm_get_collider_grad(mpm_batch* b, int32_t env, double* dvel, double* dc0, double* domega, double* dangle0,
                          int32_t n) {
  return mpm_get_collider_grad_at(b, env, 0, dvel, dc0, domega, dangle0, n);
}

int mpm_get_collider_grad_at(mpm_batch* b, int32_t env, int32_t index, double* dvel, double* dc0, double* domega,
                             double* dangle0, int32_t n) {
  if (!b) return MPM_INVALID_ARG;
  int rc = check_env(b, env, false);
  if (rc) return rc;
  if ((rc = check_collider_index(b, index))) return rc;
  const ColDev& d = b->envs_h[env].col[index];
  const float dt = b->envs_h[env].dt;
  if (d.motion_len == 0) return fail(b, MPM_BAD_STATE, "the collider has no prescribed motion");
  if (n < 0 || n > d.motion_len) return fail(b, MPM_INVALID_ARG, "n outside [0, motion length]");
  const int L = d.motion_len;
  constexpr int W = kMotionRow;
  std::vector<double> g(W * (size_t)L);
  HIPC(b, hipMemcpyAsync(g.data(), b->gmotion_d + W * (size_t)d.motion_off, sizeof(double) * g.size(),
                         hipMemcpyDeviceToHost, b->stream));
  HIPC(b, hipStreamSynchronize(b->stream));
  // row k holds the cotangents of (center_k, velocity_k, angle_k, omega_k);
  // center_k depends on every earlier velocity (dt each) and on c0, angle_k on
  // every earlier angular speed and on the starting angle
  double later[3] = {0.0, 0.0, 0.0}, later_th = 0.0;   // sums over k > j of the center / angle cotangents
  for (int j = L - 1; j >= 0; --j) {
    if (j < n && dvel)
      for (int a = 0; a < 3; ++a) dvel[3 * j + a] = g[W * j + 3 + a] + (double)dt * later[a];
    if (j < n && domega) domega[j] = g[W * j + 7] + (double)dt * later_th;
    for (int a = 0; a < 3; ++a) later[a] += g[W * j + a];
    later_th += g[W * j + 6];
  }
  if (dc0)
    for (int a = 0; a < 3; ++a) dc0[a] = later[a];
  if (dangle0) *dangle0 = later_th;
  return MPM_OK;
}

int mpm_moments(mpm_batch* b, const float* x, const float* v, const float* w, double* out) {
  if (!b) return MPM_INVALID_ARG;
  if (!x || !v || !out) return fail(b, MPM_INVALID_ARG, "null array");
  launch_moments(b->items_d, (int)b->items_h.size(), b->envs_d, x, v, w, out, b->E, b->stream);
  HIPC(b, hipGetLastError());
  return MPM_OK;
}

int mpm_moments_vjp(mpm_batch* b, const float* x, const float* v, const float* w, const double* gout, float* gx,
                    float* gv) {
  if (!b) return MPM_INVALID_ARG;
  if (!x || !v || !gout) return fail(b, MPM_INVALID_ARG, "null array");
  launch_moments_vjp(b->items_d, (int)b->items_h.size(), b->envs_d, x, v, w, gout, gx, gv, b->stream);
  HIPC(b, hipGetLastError());
  return MPM_OK;
}

int mpm_pair_distance(mpm_batch* b, const float* x, const int32_t* pairs, int64_t n_pairs, double* out) {
  if (!b) return MPM_INVALID_ARG;
  if (!x || !out || n_pairs < 0 || (n_pairs > 0 && !pairs)) return fail(b, MPM_INVALID_ARG, "null array or negative count");
  launch_pair_distance(b->envs_d, b->E, x, pairs, n_pairs, out, b->stream);
  HIPC(b, hipGetLastError());
  return MPM_OK;
}

int mpm_pair_distance_vjp(mpm_batch* b, const float* x, const int32_t* pairs, int64_t n_pairs, const double* out,
                          const double* gout, float* gx) {
  if (!b) return MPM_INVALID_ARG;
  if (!x || !out || !gout || !gx || n_pairs < 0 || (n_pairs > 0 && !pairs))
    return fail(b, MPM_INVALID_ARG, "null array or negative count");
  launch_pair_distance_vjp(b->envs_d, b->E, x, pairs, n_pairs, out, gout, gx, b->rows, b->stream);
  HIPC(b, hipGetLastError());
  return MPM_OK;
}

int mpm_forward_envs(mpm_batch* b, const int32_t* n_substeps, int32_t flags) {
  if (!b || !n_substeps) return MPM_INVALID_ARG;
  int32_t S = 0;
  for (int e = 0; e < b->E; ++e) {
    if (n_substeps[e] < 0 || n_substeps[e] > b->max_substeps)
      return fail(b, MPM_BAD_STATE, "n_substeps outside [0, max_substeps]");
    S = std::max(S, n_substeps[e]);
  }
  for (int e = 0; e < b->E; ++e)
    for (const ColDev& cd : b->envs_h[e].col)
      if (cd.has_collider && cd.motion_len > 0 && n_substeps[e] > 0 && b->env_steps[e] + n_substeps[e] > cd.motion_len)
        return fail(b, MPM_INVALID_ARG, "the collider motion of an environment is shorter than the rollout");
  bool changed = false;
  for (int e = 0; e < b->E; ++e) {
    changed |= b->envs_h[e].nsub != n_substeps[e];
    b->envs_h[e].nsub = n_substeps[e];
  }
  if (changed) {
    const int rc = upload_envs(b);
    if (rc != MPM_OK) return rc;
  }
  const bool record = (flags & MPM_FWD_RECORD) != 0;
  const hipStream_t s = b->stream;
  if (b->timing) { b->spans.clear(); b->event_next = 0; }
  clear_dirty_tapes(b);
  b->recorded = false;
  b->last_seg_taped = false;
  if (record) {
    launch_copy_i32(b->ids_cur, b->ids_start, b->N, s);
    launch_copy_i32(b->clock, b->clock_rec, b->E, s);
  }
  const int nseg = (S + b->K - 1) / b->K;
  const float* src = b->cur;
  for (int j = 0; j < nseg; ++j) {
    const int Kj = std::min(b->K, S - j * b->K);
    const bool tape = record && j == nseg - 1;
    const int rc = run_maybe_graph(b, std::make_tuple(0, j, Kj, (int)record, (int)tape, (const void*)src),
                                   [&] { fwd_segment(b, j, Kj, record, tape, src, false); });
    if (rc != MPM_OK) return rc;
    if (tape)
      for (int k = 1; k <= Kj; ++k) b->grid_dirty[k] = true;
    src = fwd_segment(b, j, Kj, record, tape, src, true);
  }
  b->cur = (float*)src;
  HIPC(b, hipGetLastError());
  if (record) {
    b->recorded = true;
    b->rec_S = S;
    b->last_seg_taped = nseg > 0;
  }
  for (int e = 0; e < b->E; ++e) b->env_steps[e] += n_substeps[e];
  return MPM_OK;
}

int mpm_forward(mpm_batch* b, int32_t S, int32_t flags) {
  if (!b) return MPM_INVALID_ARG;
  if (S < 0 || S > b->max_substeps) return fail(b, MPM_BAD_STATE, "n_substeps outside [0, max_substeps]");
  std::vector<int32_t> n(b->E, S);
  return mpm_forward_envs(b, n.data(), flags);
}

int mpm_backward(mpm_batch* b, const float* gx, const float* gv, const float* gC, const float* gF, float* dx0,
                 float* dv0, float* dC0, float* dF0, double* dparams) {
  if (!b) return MPM_INVALID_ARG;
  if (!b->recorded) return fail(b, MPM_BAD_STATE, "backward needs a preceding recorded forward");
  const hipStream_t s = b->stream;
  if (b->timing) { b->spans.clear(); b->event_next = 0; }
  launch_fill_u32(b->pacc, 0u, 2 * 8 * (int64_t)b->E, s);
  launch_fill_u32(b->gmotion_d, 0u, 2 * kMotionRow * (int64_t)kMaxColliders * b->E * b->max_substeps, s);
  const int S = b->rec_S;
  const int nseg = (S + b->K - 1) / b->K;
  int c = 0;
  launch_gather_aos(b->items_d, (int)b->items_h.size(), b->envs_d, gx, gv, gC, gF, b->ids_cur, b->cot[c], b->N, s);
  for (int j = nseg - 1; j >= 0; --j) {
    const int Kj = std::min(b->K, S - j * b->K);
    launch_clocks_from(b->clock, b->clock_rec, b->E, j * b->K, s);
    const bool have_tape = (j == nseg - 1) && b->last_seg_taped;
    if (!have_tape) clear_dirty_tapes(b);
    int c_out = c;
    const int rc = run_maybe_graph(b, std::make_tuple(1, j, Kj, (int)have_tape, c, (const void*)nullptr),
                                   [&] { c_out = bwd_segment(b, j, Kj, have_tape, c); });
    if (rc != MPM_OK) return rc;
    c = (c + Kj + 1) & 1;   // the adjoint substeps and the unpermute each switch buffers
    (void)c_out;
    for (int k = 1; k <= Kj; ++k) b->grid_dirty[k] = false;
  }
  b->last_seg_taped = false;
  launch_store_aos(b->items_d, (int)b->items_h.size(), b->envs_d, 1, b->cot[c], b->N, b->ids_start, dx0, dv0, dC0, dF0, false, s);
  if (dparams) launch_finalize_params(b->envs_d, b->pacc, dparams, b->E, s);
  HIPC(b, hipGetLastError());
  return MPM_OK;
}

int mpm_sort_keys(mpm_batch* b, uint32_t* keys, uint32_t* perm, int32_t* ids, int32_t* cell_bits) {
  if (!b) return MPM_INVALID_ARG;
  if (cell_bits) *cell_bits = b->cell_bits;
  if (b->N == 0) return MPM_OK;
  const hipStream_t s = b->stream;
  launch_keys(b->cur, b->N, b->envs_d, b->items_d, (int)b->items_h.size(), b->keys0, b->vals0, b->cell_bits, s);
  if (keys) HIPC(b, hipMemcpyAsync(keys, b->keys0, sizeof(uint32_t) * b->N, hipMemcpyDeviceToDevice, s));
  const int which = launch_radix_sort(b->keys0, b->vals0, b->keys1, b->vals1, b->counts, b->N, b->key_bits, s);
  if (perm) HIPC(b, hipMemcpyAsync(perm, which ? b->vals1 : b->vals0, sizeof(uint32_t) * b->N, hipMemcpyDeviceToDevice, s));
  if (ids) HIPC(b, hipMemcpyAsync(ids, b->ids_cur, sizeof(int32_t) * b->N, hipMemcpyDeviceToDevice, s));
  HIPC(b, hipGetLastError());
  return MPM_OK;
}

int mpm_sync(mpm_batch* b) {
  if (!b) return MPM_INVALID_ARG;
  HIPC(b, hipStreamSynchronize(b->stream));
  HIPC(b, hipMemcpy(b->env_err_h.data(), b->errs, sizeof(int32_t) * b->E, hipMemcpyDeviceToHost));
  int agg = 0;
  for (int v : b->env_err_h) agg |= v;
  launch_fill_u32(b->errs, 0u, b->E, b->stream);
  HIPC(b, hipStreamSynchronize(b->stream));
  if (agg & ERR_NONFINITE) return fail(b, MPM_NONFINITE, "non-finite particle state");
  if (agg & ERR_OUT_OF_DOMAIN) return fail(b, MPM_OUT_OF_DOMAIN, "particle left the stencil band (clamped)");
  return MPM_OK;
}

int mpm_env_errors(mpm_batch* b, int32_t* errs) {
  if (!b || !errs) return MPM_INVALID_ARG;
  std::memcpy(errs, b->env_err_h.data(), sizeof(int32_t) * b->E);
  return MPM_OK;
}

int mpm_set_timing(mpm_batch* b, int32_t enabled) {
  if (!b) return MPM_INVALID_ARG;
  b->timing = enabled != 0;
  b->spans.clear();
  b->event_next = 0;
  return MPM_OK;
}

int mpm_kernel_time(mpm_batch* b, int32_t kernel, double* mean_ms) {
  if (!b || !mean_ms || kernel < 0 || kernel >= KC_COUNT) return MPM_INVALID_ARG;
  HIPC(b, hipStreamSynchronize(b->stream));
  double tot = 0.0;
  int n = 0;
  for (auto& sp : b->spans) {
    if (sp.kc != kernel) continue;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, sp.a, sp.b) == hipSuccess) { tot += ms; ++n; }
  }
  *mean_ms = n ? tot / n : 0.0;
  return n;
}

int mpm_set_option(mpm_batch* b, int32_t option, int32_t value) {
  if (!b) return MPM_INVALID_ARG;
  switch (option) {
    case MPM_OPT_GRAPHS: b->use_graphs = value != 0; return MPM_OK;
    case MPM_OPT_P2G: if (value < 0 || value > 3) break; b->var_p2g = value; drop_graphs(b); return MPM_OK;
    case MPM_OPT_G2P: if (value < 0 || value > 1) break; b->var_g2p = value; drop_graphs(b); return MPM_OK;
    case MPM_OPT_G2P_ADJ: if (value < 0 || value > 3) break; b->var_g2p_adj = value; drop_graphs(b); return MPM_OK;
    case MPM_OPT_P2G_ADJ: if (value < 0 || value > 1) break; b->var_p2g_adj = value; drop_graphs(b); return MPM_OK;
    case MPM_OPT_MIN_RUN: if (value < 1 || value > 256) break; b->min_run = value; drop_graphs(b); return MPM_OK;
    case MPM_OPT_GRID_CAP: if (value < 0) break; b->grid_cap = value; drop_graphs(b); return MPM_OK;
    case MPM_OPT_MAX_RUN: if (value < 1 || value > 256) break; b->max_run = value; drop_graphs(b); return MPM_OK;
    case MPM_OPT_BOX: if (value < 0 || value > 1) break; b->box = value; drop_graphs(b); return MPM_OK;
    case MPM_OPT_SPECIALIZE: if (value < 0 || value > 1) break; b->specialize = value; drop_graphs(b); return MPM_OK;
    case MPM_OPT_FUSE: if (value < 0 || value > 1) break; b->fuse = value; drop_graphs(b); return MPM_OK;
    case MPM_OPT_FUSE_ADJ: if (value < 0 || value > 1) break; b->fuse_adj = value; drop_graphs(b); return MPM_OK;
    case MPM_OPT_GRID_LIST: if (value < 0 || value > 2) break; b->grid_list = value; drop_graphs(b); return MPM_OK;
    case MPM_OPT_XCD: {
      if (value < 0 || value > 1) break;
      b->xcd = value;
      const int rc = upload_items(b);
      drop_graphs(b);
      return rc;
    }
    default: break;
  }
  return fail(b, MPM_INVALID_ARG, "unknown option or value");
}

int mpm_get_option(mpm_batch* b, int32_t option, int32_t* value) {
  if (!b || !value) return MPM_INVALID_ARG;
  switch (option) {
    case MPM_OPT_GRAPHS: *value = b->use_graphs ? 1 : 0; return MPM_OK;
    case MPM_OPT_P2G: *value = b->var_p2g; return MPM_OK;
    case MPM_OPT_G2P: *value = b->var_g2p; return MPM_OK;
    case MPM_OPT_G2P_ADJ: *value = b->var_g2p_adj; return MPM_OK;
    case MPM_OPT_P2G_ADJ: *value = b->var_p2g_adj; return MPM_OK;
    case MPM_OPT_MIN_RUN: *value = b->min_run; return MPM_OK;
    case MPM_OPT_GRID_CAP: *value = b->grid_cap; return MPM_OK;
    case MPM_OPT_MAX_RUN: *value = b->max_run; return MPM_OK;
    case MPM_OPT_BOX: *value = b->box; return MPM_OK;
    case MPM_OPT_SPECIALIZE: *value = b->specialize; return MPM_OK;
    case MPM_OPT_FUSE: *value = b->fuse; return MPM_OK;
    case MPM_OPT_FUSE_ADJ: *value = b->fuse_adj; return MPM_OK;
    case MPM_OPT_XCD: *value = b->xcd; return MPM_OK;
    case MPM_OPT_GRID_LIST: *value = b->grid_list; return MPM_OK;
    default: return fail(b, MPM_INVALID_ARG, "unknown option");
  }
}


int mpm_autotune(mpm_batch* b, int32_t budget_ms) {
  if (!b) return MPM_INVALID_ARG;
  if (b->mode != MPM_MODE_BATCHED || b->N == 0 || b->max_substeps == 0) return MPM_OK;
  const std::string sig = shape_signature(b);
  auto hit = tune_cache().find(sig);
  if (hit != tune_cache().end()) { apply_choice(b, hit->second); return MPM_OK; }
  const hipStream_t s = b->stream;
  HIPC(b, hipStreamSynchronize(s));
  const int64_t NS = 24 * b->N;                // floats of one state buffer
  const int64_t R = std::max<int64_t>(b->rows, 1);
  float* saved = (float*)dalloc(b, sizeof(float) * NS);
  float* ref = (float*)dalloc(b, sizeof(float) * NS);
  float* cot_in = (float*)dalloc(b, sizeof(float) * 24 * R);
  float* gref = (float*)dalloc(b, sizeof(float) * 24 * R);
  float* gout = (float*)dalloc(b, sizeof(float) * 24 * R);
  int32_t* ids_saved = (int32_t*)dalloc(b, sizeof(int32_t) * b->N);
  int32_t* clock_saved = (int32_t*)dalloc(b, sizeof(int32_t) * b->E);
  double* acc = (double*)dalloc(b, 256);
  if (!saved || !ref || !cot_in || !gref || !gout || !ids_saved || !clock_saved || !acc)
    return fail(b, MPM_OUT_OF_MEMORY, "autotune scratch");
  float* cur0 = b->cur;
  const std::vector<int64_t> steps0 = b->env_steps;
  const bool graphs0 = b->use_graphs;
  b->use_graphs = false;
  b->recorded = false;
  launch_copy_f32(cur0, saved, NS, s);
  launch_copy_i32(b->ids_cur, ids_saved, b->N, s);
  launch_copy_i32(b->clock, clock_saved, b->E, s);
  launch_fill_u32(cot_in, 0x3f800000u, 24 * R, s);   // all-ones cotangent
  const int St = std::min(b->K, b->max_substeps);
  std::vector<int32_t> n_all(b->E, St);

  auto restore = [&]() {
    b->cur = cur0;
    launch_copy_f32(saved, cur0, NS, s);
    launch_copy_i32(ids_saved, b->ids_cur, b->N, s);
    launch_copy_i32(clock_saved, b->clock, b->E, s);
    b->env_steps = steps0;
    b->recorded = false;
  };
  float* g = gout;
  auto run_fwd = [&](float* dst) -> int {
    restore();
    int rc = mpm_forward_envs(b, n_all.data(), 0);
    if (rc) return rc;
    launch_copy_f32(b->cur, dst, NS, s);
    return MPM_OK;
  };
  auto run_bwd = [&](float* dst) -> int {
    restore();
    int rc = mpm_forward_envs(b, n_all.data(), MPM_FWD_RECORD);
    if (rc) return rc;
    return mpm_backward(b, cot_in, cot_in + 3 * R, cot_in + 6 * R, cot_in + 15 * R, dst, dst + 3 * R, dst + 6 * R,
                        dst + 15 * R, nullptr);
  };
  auto rel_err = [&](const float* a, const float* bb, int64_t n, double& out) -> int {
    launch_fill_u32(acc, 0u, 4, s);
    launch_sq_diff(a, bb, n, acc, s);
    double h[2];
    HIPC(b, hipMemcpyAsync(h, acc, sizeof(h), hipMemcpyDeviceToHost, s));
    HIPC(b, hipStreamSynchronize(s));
    out = h[1] > 0 ? std::sqrt(h[0] / h[1]) : std::sqrt(h[0]);
    return MPM_OK;
  };
  hipEvent_t e0, e1;
  HIPC(b, hipEventCreate(&e0));
  HIPC(b, hipEventCreate(&e1));
  const auto t_start = std::chrono::steady_clock::now();
  auto over_budget = [&]() {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count() > budget_ms;
  };
  // reference results: one thread per particle, global atomics
  TuneChoice best{0, 0, 0, 0, b->min_run, 0, b->max_run, 0, 1, 0, 0, 0, 0};
  apply_choice(b, best);
  int rc = run_fwd(ref);
  if (!rc) rc = run_bwd(gref);
  if (!rc) HIPC(b, hipStreamSynchronize(s));
  auto time_it = [&](bool bwd, double& ms) -> int {
    int r = bwd ? run_bwd(g) : run_fwd(g);     // warm-up (and first-use costs)
    if (r) return r;
    HIPC(b, hipEventRecord(e0, s));
    r = bwd ? run_bwd(g) : run_fwd(g);
    if (r) return r;
    HIPC(b, hipEventRecord(e1, s));
    HIPC(b, hipEventSynchronize(e1));
    float f = 0.f;
    HIPC(b, hipEventElapsedTime(&f, e0, e1));
    ms = f;
    return MPM_OK;
  };
  // one candidate: a field of TuneChoice, its value, optional min_run, timed with the backward
  struct Cand { int* slot; int value; int min_run; bool bwd; };
  std::vector<std::vector<Cand>> groups = {
      {{&best.p2g, 0, 0, false}, {&best.p2g, 1, 0, false}, {&best.p2g, 2, 2, false}, {&best.p2g, 2, 3, false},
       {&best.p2g, 2, 4, false}, {&best.p2g, 2, 8, false}, {&best.p2g, 3, 0, false}},
      {{&best.g2p, 0, 0, false}, {&best.g2p, 1, 0, false}},
      {{&best.g2p_adj, 0, 0, true}, {&best.g2p_adj, 1, 0, true}, {&best.g2p_adj, 2, 0, true},
       {&best.g2p_adj, 3, 0, true}},
      {{&best.p2g_adj, 0, 0, true}, {&best.p2g_adj, 1, 0, true}},
      {{&best.box, 0, 0, true}, {&best.box, 1, 0, true}},
      {{&best.specialize, 1, 0, true}, {&best.specialize, 0, 0, true}},
      {{&best.fuse, 0, 0, true}, {&best.fuse, 1, 0, true}},
      {{&best.fuse_adj, 0, 0, true}, {&best.fuse_adj, 1, 0, true}},
      {{&best.xcd, 0, 0, true}, {&best.xcd, 1, 0, true}},
      {{&best.grid_list, 0, 0, true}, {&best.grid_list, 1, 0, true}, {&best.grid_list, 2, 0, true}},
      {{&best.grid_cap, 0, 0, true}, {&best.grid_cap, 512, 0, true}, {&best.grid_cap, 1024, 0, true},
       {&best.grid_cap, 2048, 0, true}},
      {{&best.max_run, 4, 0, true}, {&best.max_run, 8, 0, true}, {&best.max_run, 16, 0, true},
       {&best.max_run, 256, 0, true}},
  };
  for (auto& grp : groups) {
    if (rc) break;
    double best_ms = 1e30;
    TuneChoice keep = best;
    for (auto& c : grp) {
      if (rc) break;
      if (over_budget() && best_ms < 1e30) break;
      TuneChoice trial = keep;
      *(&trial.p2g + (c.slot - &best.p2g)) = c.value;
      if (c.min_run > 0) trial.min_run = c.min_run;
      apply_choice(b, trial);
      double ms = 0.0, err = 0.0;
      rc = time_it(c.bwd, ms);
      if (rc) break;
      if (c.bwd) {
        rc = rel_err(g, gref, 6 * R, err);   // x and v cotangents of the initial state
      } else {
        rc = rel_err(g, ref, 6 * b->N, err);   // x and v of the end state
      }
      if (rc) break;
      // a later candidate must win by more than 1%: a tie keeps the earlier (default)
      // choice, so timing noise does not flip between equivalent variants
      if (err <= (c.bwd ? 1e-4 : 1e-5) && ms < best_ms * 0.99) {
        best_ms = ms;
        best = trial;
      }
    }
    if (best_ms >= 1e30) best = keep;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  restore();
  apply_choice(b, best);
  b->use_graphs = graphs0;
  if (hipStreamSynchronize(s) != hipSuccess && !rc) rc = MPM_DEVICE_ERROR;
  // scratch goes back to the allocator
  for (void* p : {(void*)saved, (void*)ref, (void*)cot_in, (void*)gref, (void*)gout, (void*)ids_saved,
                  (void*)clock_saved, (void*)acc}) {
    for (size_t i = 0; i < b->allocations.size(); ++i)
      if (b->allocations[i].first == p) {
        if (b->has_alloc) b->alloc.free(p, b->alloc.ctx); else (void)hipFree(p);
        b->bytes -= (int64_t)b->allocations[i].second;
        b->allocations.erase(b->allocations.begin() + i);
        break;
      }
  }
  if (rc) return rc;
  tune_cache()[sig] = best;
  return MPM_OK;
}

}  // extern "C"
