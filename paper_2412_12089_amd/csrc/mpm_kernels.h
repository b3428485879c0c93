// Host-visible launchers of the MLS-MPM kernels (internal to the library).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mpm_device.h"

namespace mpmx {

// A block's share of one environment's particles: [start, start + count).
// Positions [start, start + cap) belong to the env's capacity; the first
// `count` of them hold live particles (count may be 0).
struct WorkItem {
  int32_t env;
  int32_t count;
  int64_t start;
  int32_t cap;
  int32_t pad;
};
constexpr int kItemSize = 256;

// radix sort geometry: 256 threads x 4 keys per block
constexpr int RS_THREADS = 256;
constexpr int RS_ITEMS = 4;
constexpr int RS_TILE = RS_THREADS * RS_ITEMS;

void launch_prep_params(EnvDev* envs, int n_envs, hipStream_t s);
void launch_finalize_params(const EnvDev* envs, const double* acc, double* out, int n_envs, hipStream_t s);
void launch_load_aos(const WorkItem* items, int n_items, const EnvDev* envs, int all, const float* x, const float* v,
                     const float* C, const float* F, float* st, int64_t N, int32_t* ids, hipStream_t s);
void launch_store_aos(const WorkItem* items, int n_items, const EnvDev* envs, int all, const float* st, int64_t N,
                      const int32_t* ids, float* x, float* v, float* C, float* F, bool state, hipStream_t s);
void launch_gather_aos(const WorkItem* items, int n_items, const EnvDev* envs, const float* x, const float* v,
                       const float* C, const float* F, const int32_t* ids, float* st, int64_t N, hipStream_t s);
void launch_copy_i32(const int32_t* a, int32_t* b, int64_t n, hipStream_t s);
void launch_fill_u32(void* p, uint32_t v, int64_t n_words, hipStream_t s);
// copies one env's state rows [p0, p0 + cnt) and ids to (to_buf = 1) or from a compact [25][cnt] buffer
void launch_env_rows(float* st, int32_t* ids, int64_t N, int64_t p0, int64_t cnt, float* buf, int to_buf,
                     hipStream_t s);
// per-env substep clocks: set (env < 0: all), advance over a forward segment, or rebase for a backward segment
void launch_set_clock(int32_t* clock, int env, int n_envs, int32_t value, hipStream_t s);
void launch_advance_clocks(int32_t* clock, const EnvDev* envs, int n_envs, int k0, int Kj, hipStream_t s);
void launch_clocks_from(int32_t* clock, const int32_t* base, int n_envs, int k, hipStream_t s);
void launch_sq_diff(const float* a, const float* b, int64_t n, double* acc, hipStream_t s);
void launch_copy_f32(const float* a, float* b, int64_t n, hipStream_t s);
void launch_keys(const float* st, int64_t N, const EnvDev* envs, const WorkItem* items, int n_items, uint32_t* keys,
                 uint32_t* vals, int cell_bits, hipStream_t s);
int launch_radix_sort(uint32_t* k0, uint32_t* v0, uint32_t* k1, uint32_t* v1, uint32_t* counts, int64_t N,
                      int key_bits, hipStream_t s);
void launch_permute_state(const float* src, float* dst, int64_t N, const uint32_t* perm, const int32_t* ids_in,
                          int32_t* ids_out, hipStream_t s);
void launch_unpermute(const float* src, float* dst, int64_t N, const uint32_t* perm, hipStream_t s);
void launch_p2g_direct(const float* st, int64_t N, const EnvDev* envs, const WorkItem* items, int n_items, float* grid,
                       uint32_t* flags, int32_t* errs, int k_call, hipStream_t s);
// motion: per-substep (center, velocity) rows of prescribed collider motions;
// gmotion: FP64 cotangents of those rows, accumulated by the grid adjoint
void launch_grid_update(const EnvDev* envs, const int32_t* tile_env, int64_t tile0, int64_t ntiles, float* grid,
                        uint32_t* flags, const int32_t* clock, double t0, int k_rel, int clear, const float* motion,
                        hipStream_t s, int cols = kMaxColliders);
// the grid passes with `tiles` (16 or 64) tiles per block, the flagged ones found by one ballot; cols = the
// most colliders an env of the launch holds (0 and 1 launch variants compiled for them)
void launch_grid_update_chunked(const EnvDev* envs, const int32_t* tile_env, int64_t ntiles, float* grid,
                                uint32_t* flags, const int32_t* clock, double t0, int k_rel, int clear,
                                const float* motion, int tiles, hipStream_t s, int cols = kMaxColliders);
void launch_grid_adjoint_chunked(const EnvDev* envs, const int32_t* tile_env, int64_t ntiles, float* grid,
                                 uint32_t* flags, float* gcot, const int32_t* clock, double t0, int k_rel,
                                 const float* motion, double* gmotion, int tiles, hipStream_t s, int cols = kMaxColliders);
void launch_grid_adjoint(const EnvDev* envs, const int32_t* tile_env, int64_t tile0, int64_t ntiles, float* grid,
                         uint32_t* flags, float* gcot, const int32_t* clock, double t0, int k_rel, const float* motion,
                         double* gmotion, hipStream_t s, int cols = kMaxColliders);
void launch_grid_clear_flagged(int64_t ntiles, float* grid, uint32_t* flags, hipStream_t s);
void launch_g2p_direct(const float* st, float* out, int64_t N, const EnvDev* envs, const WorkItem* items, int n_items,
                       const float* grid, int32_t* errs, int k_call, hipStream_t s);
void launch_g2p_adjoint_direct(const float* st, const float* st_next, const float* cot, float* part, int64_t N, const EnvDev* envs,
                               const WorkItem* items, int n_items, const float* grid, float* gcot, double* pacc,
                               int k_call, hipStream_t s);
void launch_p2g_adjoint_direct(const float* st, const float* part, float* cot_out, int64_t N, const EnvDev* envs,
                               const WorkItem* items, int n_items, const float* gcot, double* pacc, int k_call, const float* cot_in, hipStream_t s);

// LDS-staged variants of the particle kernels (batched mode). Each launch
// covers work items of one material `mat`, compiled for that material; `box`
// picks the LDS box budget (0: 1024 nodes, 1: 384 nodes).
void launch_p2g_lds(const float* st, int64_t N, const EnvDev* envs, const WorkItem* items, int n_items, float* grid,
                    uint32_t* flags, int32_t* errs, int k_call, int grid_cap, int box, int mat, hipStream_t s);
void launch_g2p_lds(const float* st, float* out, int64_t N, const EnvDev* envs, const WorkItem* items, int n_items,
                    const float* grid, int32_t* errs, int k_call, int grid_cap, int box, int mat, hipStream_t s);
void launch_g2p_adjoint_lds(const float* st, const float* st_next, const float* cot, float* part, int64_t N, const EnvDev* envs,
                            const WorkItem* items, int n_items, const float* grid, float* gcot, double* pacc,
                            int k_call, int grid_cap, int box, int mat, hipStream_t s);
void launch_p2g_adjoint_lds(const float* st, const float* part, float* cot_out, int64_t N, const EnvDev* envs,
                            const WorkItem* items, int n_items, const float* gcot, double* pacc, int k_call, const float* cot_in, int grid_cap, int box, int mat, hipStream_t s);

// pull scatters: the LDS-staged kernels' boxes, but each box node is summed by
// its owner thread from LDS payloads of the block's particles (counting-sorted
// by stencil base) instead of LDS float atomics
void launch_p2g_pull(const float* st, int64_t N, const EnvDev* envs, const WorkItem* items, int n_items, float* grid,
                     uint32_t* flags, int32_t* errs, int k_call, int grid_cap, int box, int mat, hipStream_t s);
void launch_g2p_adjoint_pull(const float* st, const float* st_next, const float* cot, float* part, int64_t N,
                             const EnvDev* envs, const WorkItem* items, int n_items, const float* grid, float* gcot,
                             double* pacc, int k_call, int grid_cap, int box, int mat, hipStream_t s);

// segment-reduced scatters: runs = min_run | max_run << 16. Blocks whose
// particles average at least min_run per run sum each run (cut at max_run
// particles) in registers before the LDS atomics
void launch_p2g_seg(const float* st, int64_t N, const EnvDev* envs, const WorkItem* items, int n_items, float* grid,
                    uint32_t* flags, int32_t* errs, int runs, int k_call, int grid_cap, int box, int mat, hipStream_t s);
void launch_g2p_adjoint_seg(const float* st, const float* st_next, const float* cot, float* part, int64_t N, const EnvDev* envs,
                            const WorkItem* items, int n_items, const float* grid, float* gcot, double* pacc,
                            int runs, int k_call, int grid_cap, int box, int mat, hipStream_t s);

// G2P of substep k fused with the segment-reduced P2G of substep k + 1
// (grid_in: substep k's grid, read; grid_out / flags_out: substep k + 1's)
// G2P of substep k fused with the pull P2G of substep k + 1 (the low particles-per-cell form of launch_g2p2g)
void launch_g2p2g_pull(const float* st, float* out, int64_t N, const EnvDev* envs, const WorkItem* items, int n_items,
                       const float* grid_in, float* grid_out, uint32_t* flags_out, int32_t* errs, int k_call, int box,
                       int mat, hipStream_t s);
void launch_g2p2g(const float* st, float* out, int64_t N, const EnvDev* envs, const WorkItem* items, int n_items,
                  const float* grid_in, float* grid_out, uint32_t* flags_out, int32_t* errs, int runs, int k_call,
                  int box, int mat, hipStream_t s);

// P2G adjoint of substep k fused with the G2P adjoint of substep k - 1 (k_call:
// substep k's call index; st_prev / st: states k - 1 and k; grid_prev: substep
// k - 1's grid; gcot: channels 3-6 read, 0-2 scattered into; part: substep k's
// partials in, substep k - 1's out; cot_end: state-k cotangent of envs frozen at k)
// P2G adjoint of substep k fused with the pull G2P adjoint of substep k - 1
void launch_adj_pair_pull(const float* st_prev, const float* st, float* part, const float* cot_end, int64_t N,
                          const EnvDev* envs, const WorkItem* items, int n_items, const float* grid_prev, float* gcot,
                          double* pacc, int k_call, int box, int mat, hipStream_t s);
void launch_adj_pair(const float* st_prev, const float* st, float* part, const float* cot_end, int64_t N,
                     const EnvDev* envs, const WorkItem* items, int n_items, const float* grid_prev, float* gcot,
                     double* pacc, int runs, int k_call, int box, int mat, hipStream_t s);

// per-env weighted moments of caller-order x, v (see mpm_observe.hip) and their VJP
void launch_moments(const WorkItem* items, int n_items, const EnvDev* envs, const float* x, const float* v,
                    const float* w, double* out, int n_envs, hipStream_t s);
void launch_moments_vjp(const WorkItem* items, int n_items, const EnvDev* envs, const float* x, const float* v,
                        const float* w, const double* g, float* gx, float* gv, hipStream_t s);
// the flip reward term: per-env mean distance of paired particles [E][2] (mean, count), and its VJP (gx written)
void launch_pair_distance(const EnvDev* envs, int n_envs, const float* x, const int32_t* pairs, int64_t n_pairs,
                          double* out, hipStream_t s);
void launch_pair_distance_vjp(const EnvDev* envs, int n_envs, const float* x, const int32_t* pairs, int64_t n_pairs,
                              const double* out, const double* gout, float* gx, int64_t rows, hipStream_t s);

}  // namespace mpmx
