// LDS-staged particle kernels of the batched mode.
//
// A block takes one work item: up to 256 particles of one environment that
// are contiguous in (tile, cell) order, so their 3x3x3 stencils cover a few
// small boxes of grid nodes, one per tile row (tile x, tile y) the item
// crosses. The block finds those boxes, and
//  * scatters (P2G, G2P adjoint) accumulate into the box in LDS with LDS
//    atomics, then flush each touched node once to HBM with global atomics;
//  * gathers (G2P, P2G adjoint) first copy the box's grid channels into LDS
//    with coalesced loads and then read the stencil from LDS.
// Thread t works on particle (t % 64) * 4 + t / 64 of the item: the 64 lanes
// of a wave hold particles four apart in cell order, so lanes that update the
// same node in the same instruction (same cell) are rare.
// If the boxes exceed the LDS budget, or the item crosses more than four tile
// rows, the block falls back to global memory.
#include "mpm_kernels.h"

namespace mpmx {

constexpr int kBoxNodes = 1024;   // LDS budget in nodes per block (large-box variant)
constexpr int kBoxSmall = 384;    // small-box variant: less LDS per block, more blocks per CU
constexpr int kMaxRuns = 4;       // tile-row runs per block that get their own box

// A block's particles are contiguous in (tile, cell) order, so they fall into a
// few runs that share a tile row (tile x, tile y); each run's stencils cover a
// compact box of at most 6 x 6 x (z extent) nodes. The runs' boxes are packed
// one after another in LDS.
struct BoxShared {
  int rk[256];            // tile-row key of particle i (natural order), -1 if none
  int run[256];           // run index of particle i
  int wsum[4];
  int wlo[4][kMaxRuns][3], whi[4][kMaxRuns][3];   // per-wave bounds of each run
  int lo[kMaxRuns][3];
  int off[kMaxRuns + 1];  // first LDS node of each run's box; off[nruns] = total
  int ext[kMaxRuns][3];
  float inv_yz[kMaxRuns], inv_z[kMaxRuns];   // 1 / (ext y * ext z), 1 / ext z
  int nruns;
};

MD int lane_particle(int t) { return ((t & 63) << 2) | (t >> 6); }

// what one thread needs for its own particle's run
struct Box {
  int lo[3];
  int ey, ez;
  int off;
  int nodes;    // total over all runs
  bool fits;
  int run;
};

// whole-wavefront min / max (DPP reductions of the device library)
extern "C" __device__ __attribute__((const)) int __ockl_wfred_min_i32(int);
extern "C" __device__ __attribute__((const)) int __ockl_wfred_max_i32(int);
extern "C" __device__ __attribute__((const)) float __ockl_wfred_add_f32(float);

// every thread must call it (uniform control flow); lp = this thread's particle index in the item
template <int BOXN>
MD Box block_box(const EnvDev& e, const int b[3], bool valid, int lp, int count, BoxShared& bs) {
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  bs.rk[lp] = valid ? ((b[0] >> 2) * e.T + (b[1] >> 2)) : -1;
  __syncthreads();
  // runs of equal tile-row key in natural particle order (thread t looks at particle t)
  const bool in = t < count;
  const bool start = in && (t == 0 || bs.rk[t] != bs.rk[t - 1]);
  const uint64_t bal = __ballot(start);
  const uint64_t lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));
  const int before = __popcll(bal & lt) + (start ? 1 : 0);   // starts up to and including t
  if (lane == 63) bs.wsum[wave] = __popcll(bal);
  __syncthreads();
  int off = 0;
  for (int w = 0; w < wave; ++w) off += bs.wsum[w];
  if (in) bs.run[t] = off + before - 1;
  if (t == 0) {
    int tot = 0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) tot += bs.wsum[w];
    bs.nruns = tot;
  }
  __syncthreads();
  const int nruns = bs.nruns;
  const int nr = nruns < kMaxRuns ? nruns : kMaxRuns;
  const int r = valid ? bs.run[lp] : -1;
  // bounds of each run's stencils [min base, max base + 2]: a reduction in
  // registers per wave, then one value per wave (contended LDS atomics on a
  // handful of addresses would serialize 256 x 6 updates)
  for (int k = 0; k < nr; ++k) {
    const bool mine = r == k;
    if (__ballot(mine) == 0ull) {   // no particle of run k in this wave (uniform): identities only
      if (lane == 0)
        for (int a = 0; a < 3; ++a) {
          bs.wlo[wave][k][a] = 0x3fffffff;
          bs.whi[wave][k][a] = -0x3fffffff;
        }
      continue;
    }
    for (int a = 0; a < 3; ++a) {
      const int mn = __ockl_wfred_min_i32(mine ? b[a] : 0x3fffffff);
      const int mx = __ockl_wfred_max_i32(mine ? b[a] + 2 : -0x3fffffff);
      if (lane == 0) {
        bs.wlo[wave][k][a] = mn;
        bs.whi[wave][k][a] = mx;
      }
    }
  }
  __syncthreads();
  if (t == 0) {
    const int nw = (int)(blockDim.x >> 6);
    int acc = 0;
    for (int k = 0; k < nr; ++k) {
      bs.off[k] = acc;
      int n = 1;
      for (int a = 0; a < 3; ++a) {
        int lo = 0x3fffffff, hi = -0x3fffffff;
        for (int w = 0; w < nw; ++w) {
          lo = min(lo, bs.wlo[w][k][a]);
          hi = max(hi, bs.whi[w][k][a]);
        }
        bs.lo[k][a] = lo;
        bs.ext[k][a] = hi - lo + 1;
        n *= bs.ext[k][a];
      }
      bs.inv_yz[k] = 1.f / (float)(bs.ext[k][1] * bs.ext[k][2]);
      bs.inv_z[k] = 1.f / (float)bs.ext[k][2];
      acc += n;
    }
    bs.off[nr] = acc;
  }
  __syncthreads();
  Box bx;
  bx.nodes = bs.off[nr];
  bx.fits = nruns >= 1 && nruns <= kMaxRuns && bx.nodes <= BOXN;
  bx.run = r < 0 ? 0 : r;
  const int rr = (r >= 0 && r < kMaxRuns) ? r : 0;
  for (int a = 0; a < 3; ++a) bx.lo[a] = bs.lo[rr][a];
  bx.ey = bs.ext[rr][1];
  bx.ez = bs.ext[rr][2];
  bx.off = bs.off[rr];
  return bx;
}

// LDS node of (i, j, k) in this thread's run box
MD int box_index(const Box& bx, int i, int j, int k) {
  return bx.off + ((i - bx.lo[0]) * bx.ey + (j - bx.lo[1])) * bx.ez + (k - bx.lo[2]);
}
// LDS node of (i, j, k) in run r's box
MD int box_index_run(const BoxShared& bs, int r, int i, int j, int k) {
  return bs.off[r] + ((i - bs.lo[r][0]) * bs.ext[r][1] + (j - bs.lo[r][1])) * bs.ext[r][2] + (k - bs.lo[r][2]);
}
// quotient of 0 <= a < 2^21 by d >= 1 from a float reciprocal of d: (a + 1/2) / d
// lies at least 1/(2d) inside (q, q + 1), and the two roundings (of 1/d and of
// the product) move it by less than (a + 1/2) / d * 2^-23 < 1/(2d)
MD int small_div(int a, float inv_d) { return (int)(((float)a + 0.5f) * inv_d); }

MD void box_node(const BoxShared& bs, int idx, int& i, int& j, int& k) {
  int r = 0;
  while (r + 1 < kMaxRuns && r + 1 < bs.nruns && bs.off[r + 1] <= idx) ++r;
  const int loc = idx - bs.off[r];
  const int qi = small_div(loc, bs.inv_yz[r]);
  const int rem = loc - qi * bs.ext[r][1] * bs.ext[r][2];
  const int qj = small_div(rem, bs.inv_z[r]);
  i = bs.lo[r][0] + qi;
  j = bs.lo[r][1] + qj;
  k = bs.lo[r][2] + rem - qj * bs.ext[r][2];
}

// copies channels [c0, c0+nc) of every box node from a grid buffer into LDS
MD void box_load(const EnvDev& e, const Box& bx, const BoxShared& bs, const float* __restrict__ g, int c0, int nc,
                 float* lds) {
  for (int idx = threadIdx.x; idx < bx.nodes; idx += blockDim.x) {
    int i, j, k;
    box_node(bs, idx, i, j, k);
    const float* src = g + node_base(e, i, j, k) + c0 * CH;
    for (int c = 0; c < nc; ++c) lds[c * bx.nodes + idx] = src[c * CH];
  }
}

// adds the box's LDS channels to grid channels [c0, c0+nc); a node whose
// first channel is zero (no particle weight reached it) is skipped when
// skip_zero_first is set
MD void box_flush(const EnvDev& e, const Box& bx, const BoxShared& bs, float* __restrict__ g, int c0, int nc,
                  const float* lds, bool skip_zero_first) {
  for (int idx = threadIdx.x; idx < bx.nodes; idx += blockDim.x) {
    if (skip_zero_first && lds[idx] == 0.f) continue;
    int i, j, k;
    box_node(bs, idx, i, j, k);
    float* dst = g + node_base(e, i, j, k) + c0 * CH;
    for (int c = 0; c < nc; ++c) {
      const float v = lds[c * bx.nodes + idx];
      if (v != 0.f) atomicAdd(dst + c * CH, v);
    }
  }
}

MD void box_mark_tiles(const EnvDev& e, const BoxShared& bs, uint32_t* __restrict__ flags) {
  const int nr = bs.nruns < kMaxRuns ? bs.nruns : kMaxRuns;
  for (int r = 0; r < nr; ++r) {
    int tlo[3], tn[3];
    for (int a = 0; a < 3; ++a) {
      tlo[a] = bs.lo[r][a] >> 2;
      tn[a] = ((bs.lo[r][a] + bs.ext[r][a] - 1) >> 2) - tlo[a] + 1;
    }
    const int cnt = tn[0] * tn[1] * tn[2];
    for (int idx = threadIdx.x; idx < cnt; idx += blockDim.x) {
      const int tx = tlo[0] + idx / (tn[1] * tn[2]);
      const int ty = tlo[1] + (idx / tn[2]) % tn[1];
      const int tz = tlo[2] + idx % tn[2];
      flags[e.tile_off + (tx * e.T + ty) * e.T + tz] = 1u;
    }
  }
}

MD void mark_particle_tiles(const EnvDev& e, const int b[3], uint32_t* __restrict__ flags) {
  for (int a = 0; a < 2; ++a)
    for (int c = 0; c < 2; ++c)
      for (int d = 0; d < 2; ++d) {
        const int tx = (b[0] + 2 * a) >> 2, ty = (b[1] + 2 * c) >> 2, tz = (b[2] + 2 * d) >> 2;
        flags[e.tile_off + (tx * e.T + ty) * e.T + tz] = 1u;
      }
}

MD void load_x3(const float* __restrict__ st, int64_t N, int64_t p, float x[3]) {
  x[0] = st[p]; x[1] = st[N + p]; x[2] = st[2 * N + p];
}
MD M3 ld_m3(const float* __restrict__ st, int64_t N, int64_t p, int c0);
MD M3 load_cnext(const float* __restrict__ st, int64_t N, int64_t p) { return ld_m3(st, N, p, 6); }
MD M3 ld_m3(const float* __restrict__ st, int64_t N, int64_t p, int c0) {
  M3 m;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) m.m[i][j] = st[(c0 + 3 * i + j) * N + p];
  return m;
}
MD void st_m3(float* __restrict__ st, int64_t N, int64_t p, int c0, const M3& m) {
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) st[(c0 + 3 * i + j) * N + p] = m.m[i][j];
}

// a[i] for a runtime i in {0,1,2} without indexing a register array
MD float sel3(const float a[3], int i) { return i == 0 ? a[0] : (i == 1 ? a[1] : a[2]); }

// quadratic B-spline weight of node offset o (0, 1, 2) at f = x n - base, and
// its f-derivative: each piece is w = k (f - s)^2 + m, dw/df = 2 k (f - s). For
// a wave-uniform o the constants are scalars and the weight costs three
// instructions, so loops can recompute it instead of holding a table
MD void spline_piece(int o, float f, float& w, float& dw) {
  const float k = o == 1 ? -1.f : 0.5f, sft = o == 0 ? 1.5f : (o == 1 ? 1.f : 0.5f), m = o == 1 ? 0.75f : 0.f;
  const float u = f - sft;
  w = fmaf(k * u, u, m);
  dw = 2.f * k * u;
}

MD void stencil_offsets(const Stencil& sc, const EnvDev& e, int ox, int oy, int oz, float& W, float d[3]) {
  W = sel3(sc.w[0], ox) * sc.w[1][oy] * sc.w[2][oz];
  d[0] = ((float)ox - sc.f[0]) * e.dx;
  d[1] = ((float)oy - sc.f[1]) * e.dx;
  d[2] = ((float)oz - sc.f[2]) * e.dx;
}

// per-env parameter cotangents of a block: each wave sums its 64 FP32 terms
// with a DPP reduction (a parameter none of its lanes touched costs one
// ballot), the block and the grid accumulate in FP64
MD void block_reduce_params_lds(float pb[PB_COUNT], double* __restrict__ acc) {
  __shared__ double red[PB_COUNT][4];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < PB_COUNT; ++k) {
    float v = 0.f;
    if (__ballot(pb[k] != 0.f) != 0ull) v = __ockl_wfred_add_f32(pb[k]);
    if (lane == 0) red[k][wave] = (double)v;
  }
  __syncthreads();
  if (threadIdx.x < PB_COUNT) {
    const int nw = blockDim.x >> 6;
    double s = 0.0;
    for (int w = 0; w < nw; ++w) s += red[threadIdx.x][w];
    if (s != 0.0) atomicAdd(&acc[threadIdx.x], s);
  }
}

// ----------------------------------------------------------------------------
// Owner-computes ("pull") scatter through LDS. Float atomics into LDS run at a
// small fraction of the LDS read rate, so at a few particles per cell the
// push scatter (27 nodes x channels atomics per particle) is bound by them.
// Instead each particle writes its scatter payload once to LDS, the block
// counting-sorts its particles by their current stencil base (one integer LDS
// atomic per particle) and stores its payload at its sorted position, and the
// thread that owns a box node sums the contributions of the particles whose
// stencil holds it: for each of the node's 9 (x, y) base columns the three z
// bases are adjacent cells, so their particles are one contiguous range of
// the sorted payloads. A particle's
// contribution to node base + o is W(o) (g + A (o - f)) per channel (the
// affine form of both scatters), plus W(o) * mass for the mass channel.
// ----------------------------------------------------------------------------
constexpr int kPayload = 16;   // floats per particle: f (3), base z (int bits), g (3), A (9, row-major)
// box budgets (grid nodes per block) of the pull scatters: their LDS holds one
// int per base cell, not the box's channels, so a block covers more of the
// grid before it falls back to global atomics (at ~1 particle per cell a
// block's boxes average ~850 nodes and a few percent exceed 1024)
constexpr int kPullNodes = 2048;
constexpr int kPullSmall = 1024;
// room for base cells in a pull box: half its node budget. A run is one tile
// row, at most 4 x 4 base cells across and so at most 6 x 6 nodes, so its
// cells are under 16/36 of its nodes and the limit never binds; a block past
// it would fall back like one whose box does not fit. The smaller cell index
// lets six blocks share a CU.
template <int BOXN>
constexpr int pull_cells() { return BOXN / 2; }

// block-wide inclusive prefix sum of a[0, n) in place (every thread calls it)
MD void block_scan_inclusive(int* a, int n, int* wtot) {
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int per = (n + (int)blockDim.x - 1) / (int)blockDim.x;
  const int i0 = min(t * per, n), i1 = min(i0 + per, n);
  int s = 0;
  for (int i = i0; i < i1; ++i) { s += a[i]; a[i] = s; }
  int x = s;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int y = __shfl_up(x, d);
    if (lane >= d) x += y;
  }
  if (lane == 63) wtot[wave] = x;
  __syncthreads();
  int off = x - s;
  for (int w = 0; w < wave; ++w) off += wtot[w];
  for (int i = i0; i < i1; ++i) a[i] += off;
  __syncthreads();
}

// LDS of the pull scatter: the cell index and the payload rows
template <int BOXN>
struct PullShared {
  int start[pull_cells<BOXN>() + 1];     // first sorted position of each base cell (cells of all runs concatenated)
  int coff[kMaxRuns + 1];  // first cell of each run
  int cext[kMaxRuns][3];   // base-cell extents of each run (its box extents - 2)
  int wtot[4];
  float4 pay[(kPayload / 4) * 256];   // payload row r of sorted position q at pay[r * 256 + q]
};

// rows are strided by 256 particles, not packed per particle: lanes reading
// different particles' rows then spread over the LDS banks
MD void pull_store_payload(float4* pay, int q, const float f[3], int bz, const float g[3], const float A[3][3]) {
  pay[q] = make_float4(f[0], f[1], f[2], __int_as_float(bz));
  pay[256 + q] = make_float4(g[0], g[1], g[2], A[0][0]);
  pay[512 + q] = make_float4(A[0][1], A[0][2], A[1][0], A[1][1]);
  pay[768 + q] = make_float4(A[1][2], A[2][0], A[2][1], A[2][2]);
}

// counting sort of the block's particles by current stencil base within their
// run's box (every thread calls it; the box must fit): false, for every
// thread, if the boxes hold more base cells than the index has room for;
// else pos = the particle's sorted position (0 for an invalid lane)
template <int BOXN>
MD bool pull_index(const BoxShared& bs, PullShared<BOXN>& ps, const Box& bx, const int b[3], bool valid, int& pos) {
  const int nr = bs.nruns < kMaxRuns ? bs.nruns : kMaxRuns;
  if (threadIdx.x == 0) {
    int acc = 0;
    for (int r = 0; r < nr; ++r) {
      ps.coff[r] = acc;
      int n = 1;
      for (int a = 0; a < 3; ++a) {
        ps.cext[r][a] = bs.ext[r][a] - 2;
        n *= ps.cext[r][a];
      }
      acc += n;
    }
    ps.coff[nr] = acc;
  }
  __syncthreads();
  const int ncell = ps.coff[nr];
  if (ncell > pull_cells<BOXN>()) return false;
  for (int i = threadIdx.x; i <= ncell; i += blockDim.x) ps.start[i] = 0;
  __syncthreads();
  int cid = 0, rank = 0;
  if (valid) {
    const int r = bx.run;
    cid = ps.coff[r] + ((b[0] - bs.lo[r][0]) * ps.cext[r][1] + (b[1] - bs.lo[r][1])) * ps.cext[r][2] +
          (b[2] - bs.lo[r][2]);
    rank = atomicAdd(&ps.start[cid + 1], 1);   // counts one cell up: the inclusive scan makes start[] exclusive
  }
  __syncthreads();
  block_scan_inclusive(ps.start, ncell + 1, ps.wtot);
  pos = valid ? ps.start[cid] + rank : 0;
  return true;
}

// contribution of the payload at sorted position q to box node (ox, oy, k - base z) of its stencil
MD void pull_add(const float4* pay, int q, int ox, int oy, int k, float acc[3], float& wsum) {
  const float4 r0 = pay[q], r1 = pay[256 + q], r2 = pay[512 + q], r3 = pay[768 + q];
  const int oz = k - __float_as_int(r0.w);
  float wx, wy, wz, dw;
  spline_piece(ox, r0.x, wx, dw);
  spline_piece(oy, r0.y, wy, dw);
  spline_piece(oz, r0.z, wz, dw);
  const float W = wx * wy * wz;
  const float d0 = (float)ox - r0.x, d1 = (float)oy - r0.y, d2 = (float)oz - r0.z;
  const float g0 = fmaf(r1.w, d0, fmaf(r2.x, d1, fmaf(r2.y, d2, r1.x)));
  const float g1 = fmaf(r2.z, d0, fmaf(r2.w, d1, fmaf(r3.x, d2, r1.y)));
  const float g2 = fmaf(r3.y, d0, fmaf(r3.z, d1, fmaf(r3.w, d2, r1.z)));
  acc[0] = fmaf(W, g0, acc[0]);
  acc[1] = fmaf(W, g1, acc[1]);
  acc[2] = fmaf(W, g2, acc[2]);
  wsum += W;
}

// sum for box node idx (run r, node (i, j, k)) over the run's particles whose
// stencil holds it: acc[c] += W (g_c + A_c . (o - f)), wsum += W. The nine
// column ranges are read up front (one LDS round trip, not nine), and each
// column's loop is its own code with constant (x, y) offsets.
MD void pull_node(const BoxShared& bs, const int* start, const int* coff, const int (*cext)[3],
                  const float4* pay, int r, int i, int j, int k, float acc[3], float& wsum) {
  const int c0 = i - bs.lo[r][0], c1 = j - bs.lo[r][1], c2 = k - bs.lo[r][2];
  const int e0 = cext[r][0], e1 = cext[r][1], e2 = cext[r][2];
  const int z_lo = max(c2 - 2, 0), z_hi = min(c2, e2 - 1);
  if (z_lo > z_hi) return;
  int qa[9], qb[9];
#pragma unroll
  for (int c = 0; c < 9; ++c) {
    const int cx = c0 - c / 3, cy = c1 - c % 3;
    const bool ok = cx >= 0 && cx < e0 && cy >= 0 && cy < e1;
    const int cb = coff[r] + (cx * e1 + cy) * e2;
    qa[c] = start[ok ? cb + z_lo : 0];
    qb[c] = ok ? start[cb + z_hi + 1] : qa[c];
  }
#pragma unroll
  for (int c = 0; c < 9; ++c) {
#pragma unroll 1
    for (int q = qa[c]; q < qb[c]; ++q) pull_add(pay, q, c / 3, c % 3, k, acc, wsum);
  }
}

// run index and node of box node idx
MD void box_node_run(const BoxShared& bs, int idx, int& r, int& i, int& j, int& k) {
  r = 0;
  while (r + 1 < kMaxRuns && r + 1 < bs.nruns && bs.off[r + 1] <= idx) ++r;
  box_node(bs, idx, i, j, k);
}

// ----------------------------------------------------------------------------
// P2G
// ----------------------------------------------------------------------------
template <int BOXN, int MAT>
MD void p2g_lds_item(int item_idx, const float* __restrict__ st, int64_t N,
                                                 const EnvDev* __restrict__ envs, const WorkItem* __restrict__ items,
                                                 float* __restrict__ grid, uint32_t* __restrict__ flags,
                                                 int32_t* __restrict__ errs, int k_call) {
  __shared__ float lds[4 * BOXN];
  __shared__ BoxShared bsh;
  const WorkItem it = items[item_idx];
  const EnvDev& e = envs[it.env];
  const int mat = MAT >= 0 ? MAT : e.material;   // MAT < 0: the generic kernel
  if (k_call >= e.nsub) return;   // frozen env: nothing to scatter
  const int lp = lane_particle(threadIdx.x);
  const bool valid = lp < it.count;
  const int64_t p = it.start + (valid ? lp : 0);
  float x[3];
  load_x3(st, N, p, x);
  const Stencil sc = make_stencil(x, e.n, e.fn);
  if (valid && sc.oob) atomicOr(&errs[it.env], ERR_OUT_OF_DOMAIN);
  const Box bx = block_box<BOXN>(e, sc.b, valid, lp, it.count, bsh);
  if (bx.fits)
    for (int i = threadIdx.x; i < 4 * bx.nodes; i += blockDim.x) lds[i] = 0.f;
  __syncthreads();
  if (valid) {
    float v[3] = {st[3 * N + p], st[4 * N + p], st[5 * N + p]};
    const M3 Cm = ld_m3(st, N, p, 6);
    const M3 H = ld_m3(st, N, p, 15);
    const M3 tau = stress(e, H, mat);
    const float kf = -e.dt * e.vp * 4.f * e.fn * e.fn;
    const M3 A = m3_axpy(m3_scale(Cm, e.mp), kf, tau);
    float mv0[3];
    for (int a = 0; a < 3; ++a) mv0[a] = e.mp * v[a];
#pragma unroll 1
    for (int ox = 0; ox < 3; ++ox)
#pragma unroll
      for (int oy = 0; oy < 3; ++oy)
#pragma unroll
        for (int oz = 0; oz < 3; ++oz) {
          float W, d[3];
          stencil_offsets(sc, e, ox, oy, oz, W, d);
          float q[4];
          q[0] = W * e.mp;
          for (int a = 0; a < 3; ++a) q[1 + a] = W * (mv0[a] + A.m[a][0] * d[0] + A.m[a][1] * d[1] + A.m[a][2] * d[2]);
          if (bx.fits) {
            const int idx = box_index(bx, sc.b[0] + ox, sc.b[1] + oy, sc.b[2] + oz);
            for (int c = 0; c < 4; ++c) atomicAdd(&lds[c * bx.nodes + idx], q[c]);
          } else {
            float* g = grid + node_base(e, sc.b[0] + ox, sc.b[1] + oy, sc.b[2] + oz);
            for (int c = 0; c < 4; ++c) atomicAdd(g + c * CH, q[c]);
          }
        }
  }
  if (!bx.fits) {
    if (valid) mark_particle_tiles(e, sc.b, flags);
    return;
  }
  __syncthreads();
  box_flush(e, bx, bsh, grid, 0, 4, lds, true);
  box_mark_tiles(e, bsh, flags);
}

// one block per work item, or (PERSIST) a grid that strides over the items
template <bool PERSIST, int BOXN, int MAT>
__global__ void __launch_bounds__(256) k_p2g_lds(const float* __restrict__ st, int64_t N,
                                                 const EnvDev* __restrict__ envs, const WorkItem* __restrict__ items,
                                                 float* __restrict__ grid, uint32_t* __restrict__ flags,
                                                 int32_t* __restrict__ errs, int k_call, int n_items) {
  if (PERSIST) {
    for (int i = blockIdx.x; i < n_items; i += gridDim.x) {
      p2g_lds_item<BOXN, MAT>(i, st, N, envs, items, grid, flags, errs, k_call);
      __syncthreads();
    }
  } else {
    p2g_lds_item<BOXN, MAT>(blockIdx.x, st, N, envs, items, grid, flags, errs, k_call);
  }
}

// one particle's share of the pull P2G: its payload (m_p v, (m_p C - dt V_p
// 4 n^2 tau) dx, f, base z) at its sorted position when the block's boxes
// fit, else its 27 nodes added to the grid with global atomics
MD void p2g_pull_particle(const EnvDev& e, int mat, const Stencil& sc, bool fits, int pos, const float v[3],
                          const M3& Cm, const M3& H, float4* pay, float* __restrict__ grid) {
  const M3 tau = stress(e, H, mat);
  const float kf = -e.dt * e.vp * 4.f * e.fn * e.fn;
  const M3 A = m3_axpy(m3_scale(Cm, e.mp), kf, tau);
  float mv0[3];
  for (int a = 0; a < 3; ++a) mv0[a] = e.mp * v[a];
  if (fits) {
    float Ad[3][3];
    for (int a = 0; a < 3; ++a)
      for (int c = 0; c < 3; ++c) Ad[a][c] = A.m[a][c] * e.dx;
    pull_store_payload(pay, pos, sc.f, sc.b[2], mv0, Ad);
  } else {
#pragma unroll 1
    for (int ox = 0; ox < 3; ++ox)
#pragma unroll
      for (int oy = 0; oy < 3; ++oy)
#pragma unroll
        for (int oz = 0; oz < 3; ++oz) {
          float W, d[3];
          stencil_offsets(sc, e, ox, oy, oz, W, d);
          float* g = grid + node_base(e, sc.b[0] + ox, sc.b[1] + oy, sc.b[2] + oz);
          atomicAdd(g, W * e.mp);
          for (int a = 0; a < 3; ++a)
            atomicAdd(g + (1 + a) * CH, W * (mv0[a] + A.m[a][0] * d[0] + A.m[a][1] * d[1] + A.m[a][2] * d[2]));
        }
  }
}

// the owners' sums of a block whose payloads are stored (after a barrier):
// each box node's (m, m v) added to the grid once, the box's tiles flagged
template <int BOXN>
MD void p2g_pull_owners(const EnvDev& e, const BoxShared& bsh, const PullShared<BOXN>& ps, int nodes,
                        float* __restrict__ grid, uint32_t* __restrict__ flags) {
  for (int idx = threadIdx.x; idx < nodes; idx += blockDim.x) {
    int r, i, j, k;
    box_node_run(bsh, idx, r, i, j, k);
    float acc[3] = {0.f, 0.f, 0.f}, wsum = 0.f;
    pull_node(bsh, ps.start, ps.coff, ps.cext, ps.pay, r, i, j, k, acc, wsum);
    if (wsum == 0.f) continue;   // no particle weight reached the node
    float* dst = grid + node_base(e, i, j, k);
    atomicAdd(dst, wsum * e.mp);
    for (int a = 0; a < 3; ++a)
      if (acc[a] != 0.f) atomicAdd(dst + (1 + a) * CH, acc[a]);
  }
  box_mark_tiles(e, bsh, flags);
}

// P2G through the pull scatter: the block's particles write (m_p v, A dx, f)
// to LDS, each box node is summed by its owner thread and added to the grid
// once; a block whose boxes do not fit scatters with global atomics
template <int BOXN, int MAT>
MD void p2g_pull_item(int item_idx, const float* __restrict__ st, int64_t N, const EnvDev* __restrict__ envs,
                      const WorkItem* __restrict__ items, float* __restrict__ grid, uint32_t* __restrict__ flags,
                      int32_t* __restrict__ errs, int k_call) {
  __shared__ BoxShared bsh;
  __shared__ PullShared<BOXN> ps;
  const WorkItem it = items[item_idx];
  const EnvDev& e = envs[it.env];
  const int mat = MAT >= 0 ? MAT : e.material;   // MAT < 0: the generic kernel
  if (k_call >= e.nsub) return;   // frozen env: nothing to scatter
  const int lp = lane_particle(threadIdx.x);
  const bool valid = lp < it.count;
  const int64_t p = it.start + (valid ? lp : 0);
  float x[3];
  load_x3(st, N, p, x);
  const Stencil sc = make_stencil(x, e.n, e.fn);
  if (valid && sc.oob) atomicOr(&errs[it.env], ERR_OUT_OF_DOMAIN);
  const Box bx = block_box<BOXN>(e, sc.b, valid, lp, it.count, bsh);
  int pos = 0;
  const bool fits = bx.fits && pull_index<BOXN>(bsh, ps, bx, sc.b, valid, pos);
  if (valid) {
    const float v[3] = {st[3 * N + p], st[4 * N + p], st[5 * N + p]};
    p2g_pull_particle(e, mat, sc, fits, pos, v, ld_m3(st, N, p, 6), ld_m3(st, N, p, 15), ps.pay, grid);
  }
  if (!fits) {
    if (valid) mark_particle_tiles(e, sc.b, flags);
    return;
  }
  __syncthreads();
  p2g_pull_owners<BOXN>(e, bsh, ps, bx.nodes, grid, flags);
}

// six waves per SIMD: the LDS of six blocks fits a CU, and the registers fit six waves without spills
template <bool PERSIST, int BOXN, int MAT>
__global__ void __launch_bounds__(256, 6) k_p2g_pull(const float* __restrict__ st, int64_t N,
                                                  const EnvDev* __restrict__ envs, const WorkItem* __restrict__ items,
                                                  float* __restrict__ grid, uint32_t* __restrict__ flags,
                                                  int32_t* __restrict__ errs, int k_call, int n_items) {
  if (PERSIST) {
    for (int i = blockIdx.x; i < n_items; i += gridDim.x) {
      p2g_pull_item<BOXN, MAT>(i, st, N, envs, items, grid, flags, errs, k_call);
      __syncthreads();
    }
  } else {
    p2g_pull_item<BOXN, MAT>(blockIdx.x, st, N, envs, items, grid, flags, errs, k_call);
  }
}

// ----------------------------------------------------------------------------
// G2P
// ----------------------------------------------------------------------------
template <int BOXN, int MAT>
MD void g2p_lds_item(int item_idx, const float* __restrict__ st, float* __restrict__ out, int64_t N,
                                                 const EnvDev* __restrict__ envs, const WorkItem* __restrict__ items,
                                                 const float* __restrict__ grid, int32_t* __restrict__ errs, int k_call) {
  __shared__ float lds[3 * BOXN];
  __shared__ BoxShared bsh;
  const WorkItem it = items[item_idx];
  const EnvDev& e = envs[it.env];
  const int mat = MAT >= 0 ? MAT : e.material;   // MAT < 0: the generic kernel
  if (k_call >= e.nsub) {   // frozen env: the substep is the identity
    if ((int)threadIdx.x < it.count) {
      const int64_t q = it.start + threadIdx.x;
      for (int c = 0; c < 24; ++c) out[c * N + q] = st[c * N + q];
    }
    return;
  }
  const int lp = lane_particle(threadIdx.x);
  const bool valid = lp < it.count;
  const int64_t p = it.start + (valid ? lp : 0);
  float x[3];
  load_x3(st, N, p, x);
  const Stencil sc = make_stencil(x, e.n, e.fn);
  const Box bx = block_box<BOXN>(e, sc.b, valid, lp, it.count, bsh);
  if (bx.fits) box_load(e, bx, bsh, grid, 4, 3, lds);
  __syncthreads();
  if (!valid) return;
  const M3 H = ld_m3(st, N, p, 15);
  float vn[3] = {0.f, 0.f, 0.f};
  M3 Cn = m3_zero();
#pragma unroll 1
  for (int ox = 0; ox < 3; ++ox)
#pragma unroll
    for (int oy = 0; oy < 3; ++oy)
#pragma unroll
      for (int oz = 0; oz < 3; ++oz) {
        float W, d[3];
        stencil_offsets(sc, e, ox, oy, oz, W, d);
        float vi[3];
        if (bx.fits) {
          const int idx = box_index(bx, sc.b[0] + ox, sc.b[1] + oy, sc.b[2] + oz);
          for (int a = 0; a < 3; ++a) vi[a] = lds[a * bx.nodes + idx];
        } else {
          const float* g = grid + node_base(e, sc.b[0] + ox, sc.b[1] + oy, sc.b[2] + oz);
          for (int a = 0; a < 3; ++a) vi[a] = g[(4 + a) * CH];
        }
        for (int a = 0; a < 3; ++a) {
          vn[a] = fmaf(W, vi[a], vn[a]);
          const float wv = W * vi[a];
          Cn.m[a][0] = fmaf(wv, d[0], Cn.m[a][0]);
          Cn.m[a][1] = fmaf(wv, d[1], Cn.m[a][1]);
          Cn.m[a][2] = fmaf(wv, d[2], Cn.m[a][2]);
        }
      }
  Cn = m3_scale(Cn, 4.f * e.fn * e.fn);
  float xn[3];
  for (int a = 0; a < 3; ++a) xn[a] = fmaf(e.dt, vn[a], x[a]);
  const M3 Hn = project(e, trial_h(e, Cn, H), mat);
  for (int a = 0; a < 3; ++a) { out[a * N + p] = xn[a]; out[(3 + a) * N + p] = vn[a]; }
  st_m3(out, N, p, 6, Cn);
  st_m3(out, N, p, 15, Hn);
  bool fin = true;
  for (int a = 0; a < 3; ++a) fin = fin && isfinite(xn[a]) && isfinite(vn[a]);
  for (int i = 0; i < 3; ++i) for (int j = 0; j < 3; ++j) fin = fin && isfinite(Hn.m[i][j]);
  if (!fin) atomicOr(&errs[it.env], ERR_NONFINITE);
}

// one block per work item, or (PERSIST) a grid that strides over the items
template <bool PERSIST, int BOXN, int MAT>
__global__ void __launch_bounds__(256) k_g2p_lds(const float* __restrict__ st, float* __restrict__ out, int64_t N,
                                                 const EnvDev* __restrict__ envs, const WorkItem* __restrict__ items,
                                                 const float* __restrict__ grid, int32_t* __restrict__ errs, int k_call, int n_items) {
  if (PERSIST) {
    for (int i = blockIdx.x; i < n_items; i += gridDim.x) {
      g2p_lds_item<BOXN, MAT>(i, st, out, N, envs, items, grid, errs, k_call);
      __syncthreads();
    }
  } else {
    g2p_lds_item<BOXN, MAT>(blockIdx.x, st, out, N, envs, items, grid, errs, k_call);
  }
}

// ----------------------------------------------------------------------------
// G2P adjoint: gather v from an LDS copy, scatter vbar into LDS, flush
// ----------------------------------------------------------------------------
template <int BOXN, int MAT>
MD void g2p_adjoint_lds_item(int item_idx, const float* __restrict__ st, const float* __restrict__ st_next,
    const float* __restrict__ cot,
                                                         float* __restrict__ part, int64_t N,
                                                         const EnvDev* __restrict__ envs,
                                                         const WorkItem* __restrict__ items,
                                                         const float* __restrict__ grid, float* __restrict__ gcot,
                                                         double* __restrict__ pacc, int k_call) {
  __shared__ float lv[3 * BOXN];
  __shared__ float lg[3 * BOXN];
  __shared__ BoxShared bsh;
  const WorkItem it = items[item_idx];
  const EnvDev& e = envs[it.env];
  const int mat = MAT >= 0 ? MAT : e.material;   // MAT < 0: the generic kernel
  if (k_call >= e.nsub) return;   // frozen env: nothing to scatter
  const int lp = lane_particle(threadIdx.x);
  const bool valid = lp < it.count;
  const int64_t p = it.start + (valid ? lp : 0);
  float x[3];
  load_x3(st, N, p, x);
  const Stencil sc = make_stencil(x, e.n, e.fn);
  const Box bx = block_box<BOXN>(e, sc.b, valid, lp, it.count, bsh);
  if (bx.fits) {
    box_load(e, bx, bsh, grid, 4, 3, lv);
    for (int i = threadIdx.x; i < 3 * bx.nodes; i += blockDim.x) lg[i] = 0.f;
  }
  __syncthreads();
  float pb[PB_COUNT] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  if (valid) {
    const M3 H = ld_m3(st, N, p, 15);
    const M3 F = f_of(H);
    const float D4 = 4.f * e.fn * e.fn;
    // C' of the substep's output state, read from the tape (the forward's own value)
    const M3 Cn = load_cnext(st_next, N, p);
    const M3 G = m3_axpy(m3_eye(), e.dt, Cn);
    const M3 Htr = trial_h(e, Cn, H);
    float xb[3], vb[3];
    for (int a = 0; a < 3; ++a) { xb[a] = cot[a * N + p]; vb[a] = cot[(3 + a) * N + p] + e.dt * xb[a]; }
    const M3 Cb_in = ld_m3(cot, N, p, 6);
    const M3 Fb_in = ld_m3(cot, N, p, 15);
    const M3 Ftrb = project_vjp(e, Htr, Fb_in, pb, mat);
    const M3 Cb = m3_axpy(Cb_in, e.dt, m3_mul_abt(Ftrb, F));
    const M3 Fb = m3_mul_atb(G, Ftrb);
    st_m3(part, N, p, 3, Fb);   // stored before the stencil loop: fewer live registers in it
    float sv[3] = {0.f, 0.f, 0.f};   // sum of W v_i
    // per particle: the z factors of gW and of the affine cotangent
    float gz[3], cz[3];
    for (int o = 0; o < 3; ++o) gz[o] = e.fn * sc.dw[2][o];
    for (int a = 0; a < 3; ++a) cz[a] = D4 * Cb.m[a][2];
#pragma unroll 1
    for (int ox = 0; ox < 3; ++ox)
#pragma unroll 1
      for (int oy = 0; oy < 3; ++oy) {
        // column invariants: the x/y weight factors and vbar + D4 Cbar d at d_z = 0
        const float wx = sel3(sc.w[0], ox), wy = sel3(sc.w[1], oy);
        const float wxy = wx * wy, gx = e.fn * sel3(sc.dw[0], ox) * wy, gy = e.fn * wx * sel3(sc.dw[1], oy);
        const float d0 = ((float)ox - sc.f[0]) * e.dx, d1 = ((float)oy - sc.f[1]) * e.dx;
        float gc[3];
        for (int a = 0; a < 3; ++a) gc[a] = fmaf(D4, fmaf(Cb.m[a][0], d0, Cb.m[a][1] * d1), vb[a]);
#pragma unroll
        for (int oz = 0; oz < 3; ++oz) {
          const float wz = sc.w[2][oz];
          const float W = wxy * wz;
          const float gW[3] = {gx * wz, gy * wz, wxy * gz[oz]};
          const float d2 = ((float)oz - sc.f[2]) * e.dx;
          float vi[3], gv[3];
          for (int a = 0; a < 3; ++a) gv[a] = fmaf(cz[a], d2, gc[a]);
          if (bx.fits) {
            const int idx = box_index(bx, sc.b[0] + ox, sc.b[1] + oy, sc.b[2] + oz);
            for (int a = 0; a < 3; ++a) {
              vi[a] = lv[a * bx.nodes + idx];
              atomicAdd(&lg[a * bx.nodes + idx], W * gv[a]);
            }
          } else {
            const int64_t nb = node_base(e, sc.b[0] + ox, sc.b[1] + oy, sc.b[2] + oz);
            for (int a = 0; a < 3; ++a) {
              vi[a] = grid[nb + (4 + a) * CH];
              atomicAdd(gcot + nb + a * CH, W * gv[a]);
            }
          }
          const float vg = vi[0] * gv[0] + vi[1] * gv[1] + vi[2] * gv[2];
          for (int a = 0; a < 3; ++a) {
            xb[a] = fmaf(gW[a], vg, xb[a]);
            sv[a] = fmaf(W, vi[a], sv[a]);
          }
        }
      }
    // the stencil sum of -D4 W Cbar^T v_i is -D4 Cbar^T sv
    for (int a = 0; a < 3; ++a) xb[a] -= D4 * (Cb.m[0][a] * sv[0] + Cb.m[1][a] * sv[1] + Cb.m[2][a] * sv[2]);
    for (int a = 0; a < 3; ++a) part[a * N + p] = xb[a];
  }
  if (bx.fits) {
    __syncthreads();
    box_flush(e, bx, bsh, gcot, 0, 3, lg, false);
  }
  block_reduce_params_lds(pb, pacc + (int64_t)it.env * 8);
}

// one block per work item, or (PERSIST) a grid that strides over the items
template <bool PERSIST, int BOXN, int MAT>
__global__ void __launch_bounds__(256) k_g2p_adjoint_lds(const float* __restrict__ st, const float* __restrict__ st_next,
    const float* __restrict__ cot,
                                                         float* __restrict__ part, int64_t N,
                                                         const EnvDev* __restrict__ envs,
                                                         const WorkItem* __restrict__ items,
                                                         const float* __restrict__ grid, float* __restrict__ gcot,
                                                         double* __restrict__ pacc, int k_call, int n_items) {
  if (PERSIST) {
    for (int i = blockIdx.x; i < n_items; i += gridDim.x) {
      g2p_adjoint_lds_item<BOXN, MAT>(i, st, st_next, cot, part, N, envs, items, grid, gcot, pacc, k_call);
      __syncthreads();
    }
  } else {
    g2p_adjoint_lds_item<BOXN, MAT>(blockIdx.x, st, st_next, cot, part, N, envs, items, grid, gcot, pacc, k_call);
  }
}

// G2P adjoint through the pull scatter: v is gathered from the grid directly
// (the LDS holds the payloads and the cell index, whose box budget is larger
// than the staged kernels'); each particle writes (vbar', D4 dx Cbar, f) to
// LDS and the owner of each box node sums its cotangent W (vbar' + D4 Cbar d)
// and adds it to the grid once
template <int BOXN, int MAT>
MD void g2p_adjoint_pull_item(int item_idx, const float* __restrict__ st, const float* __restrict__ st_next,
                              const float* __restrict__ cot, float* __restrict__ part, int64_t N,
                              const EnvDev* __restrict__ envs, const WorkItem* __restrict__ items,
                              const float* __restrict__ grid, float* __restrict__ gcot, double* __restrict__ pacc,
                              int k_call) {
  __shared__ BoxShared bsh;
  __shared__ PullShared<BOXN> ps;
  const WorkItem it = items[item_idx];
  const EnvDev& e = envs[it.env];
  const int mat = MAT >= 0 ? MAT : e.material;   // MAT < 0: the generic kernel
  if (k_call >= e.nsub) return;   // frozen env: nothing to scatter
  const int lp = lane_particle(threadIdx.x);
  const bool valid = lp < it.count;
  const int64_t p = it.start + (valid ? lp : 0);
  float x[3];
  load_x3(st, N, p, x);
  const Stencil sc = make_stencil(x, e.n, e.fn);
  const Box bx = block_box<BOXN>(e, sc.b, valid, lp, it.count, bsh);
  int pos = 0;
  const bool fits = bx.fits && pull_index<BOXN>(bsh, ps, bx, sc.b, valid, pos);
  float pb[PB_COUNT] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  if (valid) {
    const M3 H = ld_m3(st, N, p, 15);
    const M3 F = f_of(H);
    const float D4 = 4.f * e.fn * e.fn;
    // C' of the substep's output state, read from the tape (the forward's own value)
    const M3 Cn = load_cnext(st_next, N, p);
    const M3 G = m3_axpy(m3_eye(), e.dt, Cn);
    const M3 Htr = trial_h(e, Cn, H);
    float xb[3], vb[3];
    for (int a = 0; a < 3; ++a) { xb[a] = cot[a * N + p]; vb[a] = cot[(3 + a) * N + p] + e.dt * xb[a]; }
    const M3 Cb_in = ld_m3(cot, N, p, 6);
    const M3 Fb_in = ld_m3(cot, N, p, 15);
    const M3 Ftrb = project_vjp(e, Htr, Fb_in, pb, mat);
    const M3 Cb = m3_axpy(Cb_in, e.dt, m3_mul_abt(Ftrb, F));
    const M3 Fb = m3_mul_atb(G, Ftrb);
    st_m3(part, N, p, 3, Fb);
    if (fits) {
      float Ad[3][3];
      for (int a = 0; a < 3; ++a)
        for (int c = 0; c < 3; ++c) Ad[a][c] = D4 * e.dx * Cb.m[a][c];
      pull_store_payload(ps.pay, pos, sc.f, sc.b[2], vb, Ad);
    }
    float sv[3] = {0.f, 0.f, 0.f};   // sum of W v_i
    float gz[3], cz[3];
    for (int o = 0; o < 3; ++o) gz[o] = e.fn * sc.dw[2][o];
    for (int a = 0; a < 3; ++a) cz[a] = D4 * Cb.m[a][2];
#pragma unroll 1
    for (int ox = 0; ox < 3; ++ox)
#pragma unroll 1
      for (int oy = 0; oy < 3; ++oy) {
        const float wx = sel3(sc.w[0], ox), wy = sel3(sc.w[1], oy);
        const float wxy = wx * wy, gx = e.fn * sel3(sc.dw[0], ox) * wy, gy = e.fn * wx * sel3(sc.dw[1], oy);
        const float d0 = ((float)ox - sc.f[0]) * e.dx, d1 = ((float)oy - sc.f[1]) * e.dx;
        float gc[3];
        for (int a = 0; a < 3; ++a) gc[a] = fmaf(D4, fmaf(Cb.m[a][0], d0, Cb.m[a][1] * d1), vb[a]);
#pragma unroll
        for (int oz = 0; oz < 3; ++oz) {
          const float wz = sc.w[2][oz];
          const float W = wxy * wz;
          const float gW[3] = {gx * wz, gy * wz, wxy * gz[oz]};
          const float d2 = ((float)oz - sc.f[2]) * e.dx;
          float vi[3], gv[3];
          for (int a = 0; a < 3; ++a) gv[a] = fmaf(cz[a], d2, gc[a]);
          const int64_t nb = node_base(e, sc.b[0] + ox, sc.b[1] + oy, sc.b[2] + oz);
          for (int a = 0; a < 3; ++a) vi[a] = grid[nb + (4 + a) * CH];
          if (!fits)
            for (int a = 0; a < 3; ++a) atomicAdd(gcot + nb + a * CH, W * gv[a]);
          const float vg = vi[0] * gv[0] + vi[1] * gv[1] + vi[2] * gv[2];
          for (int a = 0; a < 3; ++a) {
            xb[a] = fmaf(gW[a], vg, xb[a]);
            sv[a] = fmaf(W, vi[a], sv[a]);
          }
        }
      }
    for (int a = 0; a < 3; ++a) xb[a] -= D4 * (Cb.m[0][a] * sv[0] + Cb.m[1][a] * sv[1] + Cb.m[2][a] * sv[2]);
    for (int a = 0; a < 3; ++a) part[a * N + p] = xb[a];
  }
  if (fits) {
    __syncthreads();
    for (int idx = threadIdx.x; idx < bx.nodes; idx += blockDim.x) {
      int r, i, j, k;
      box_node_run(bsh, idx, r, i, j, k);
      float acc[3] = {0.f, 0.f, 0.f}, wsum = 0.f;
      pull_node(bsh, ps.start, ps.coff, ps.cext, ps.pay, r, i, j, k, acc, wsum);
      if (wsum == 0.f) continue;
      float* dst = gcot + node_base(e, i, j, k);
      for (int a = 0; a < 3; ++a)
        if (acc[a] != 0.f) atomicAdd(dst + a * CH, acc[a]);
    }
  }
  block_reduce_params_lds(pb, pacc + (int64_t)it.env * 8);
}

template <bool PERSIST, int BOXN, int MAT>
__global__ void __launch_bounds__(256) k_g2p_adjoint_pull(const float* __restrict__ st,
                                                          const float* __restrict__ st_next,
                                                          const float* __restrict__ cot, float* __restrict__ part,
                                                          int64_t N, const EnvDev* __restrict__ envs,
                                                          const WorkItem* __restrict__ items,
                                                          const float* __restrict__ grid, float* __restrict__ gcot,
                                                          double* __restrict__ pacc, int k_call, int n_items) {
  if (PERSIST) {
    for (int i = blockIdx.x; i < n_items; i += gridDim.x) {
      g2p_adjoint_pull_item<BOXN, MAT>(i, st, st_next, cot, part, N, envs, items, grid, gcot, pacc, k_call);
      __syncthreads();
    }
  } else {
    g2p_adjoint_pull_item<BOXN, MAT>(blockIdx.x, st, st_next, cot, part, N, envs, items, grid, gcot, pacc, k_call);
  }
}

// ----------------------------------------------------------------------------
// P2G adjoint: gather (mbar, Pbar) from an LDS copy
// ----------------------------------------------------------------------------
template <int BOXN, int MAT>
MD void p2g_adjoint_lds_item(int item_idx, const float* __restrict__ st,
                                                         const float* __restrict__ part,
                                                         float* __restrict__ cot_out, int64_t N,
                                                         const EnvDev* __restrict__ envs,
                                                         const WorkItem* __restrict__ items,
                                                         const float* __restrict__ gcot,
                                                         double* __restrict__ pacc, int k_call, const float* __restrict__ cot_in) {
  constexpr bool kEig = MAT == MAT_COROTATED || MAT == MAT_VONMISES || MAT < 0;
  __shared__ float lds[4 * BOXN];
  __shared__ BoxShared bsh;
  __shared__ float eig_keep[kEig ? 12 : 1][256];   // U and the eigenvalues of B, per thread
  const WorkItem it = items[item_idx];
  const EnvDev& e = envs[it.env];
  const int mat = MAT >= 0 ? MAT : e.material;   // MAT < 0: the generic kernel
  if (k_call >= e.nsub) {   // frozen env: the cotangent passes through
    if ((int)threadIdx.x < it.count) {
      const int64_t q = it.start + threadIdx.x;
      for (int c = 0; c < 24; ++c) cot_out[c * N + q] = cot_in[c * N + q];
    }
    return;
  }
  const int t = threadIdx.x;
  const int lp = lane_particle(t);
  const bool valid = lp < it.count;
  const int64_t p = it.start + (valid ? lp : 0);
  float x[3];
  load_x3(st, N, p, x);
  const Stencil sc = make_stencil(x, e.n, e.fn);
  const Box bx = block_box<BOXN>(e, sc.b, valid, lp, it.count, bsh);
  if (bx.fits) box_load(e, bx, bsh, gcot, 3, 4, lds);
  __syncthreads();
  float pb[PB_COUNT] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  if (valid) {
    const float kf = -e.dt * e.vp * 4.f * e.fn * e.fn;
    const float v[3] = {st[3 * N + p], st[4 * N + p], st[5 * N + p]};
    // only A and v stay live through the stencil loop; C, H and the stress
    // are read or rebuilt after it
    M3 A;
    {
      const M3 Cm = ld_m3(st, N, p, 6);
      const M3 H = ld_m3(st, N, p, 15);
      const StressPrep spr = stress_prep(e, H, mat);
      A = m3_axpy(m3_scale(Cm, e.mp), kf, stress_from(e, spr, mat));
      if (kEig && (mat == MAT_COROTATED || mat == MAT_VONMISES)) {
        for (int i = 0; i < 3; ++i) {
          eig_keep[9 + i][t] = spr.l[i];
          for (int j = 0; j < 3; ++j) eig_keep[3 * i + j][t] = spr.U.m[i][j];
        }
      }
    }
    float xb[3] = {part[p], part[N + p], part[2 * N + p]};
    float sP[3] = {0.f, 0.f, 0.f};   // sum of W Pbar
    float sm = 0.f;                  // sum of W mbar
    M3 Ab = m3_zero();               // sum of W Pbar d^T
#pragma unroll 1
    for (int ox = 0; ox < 3; ++ox)
#pragma unroll 1
      for (int oy = 0; oy < 3; ++oy) {
        // the column's three z-nodes are loaded together, then summed
        float mb[3], Pb[3][3];
#pragma unroll
        for (int oz = 0; oz < 3; ++oz) {
          if (bx.fits) {
            const int idx = box_index(bx, sc.b[0] + ox, sc.b[1] + oy, sc.b[2] + oz);
            mb[oz] = lds[idx];
            for (int a = 0; a < 3; ++a) Pb[oz][a] = lds[(1 + a) * bx.nodes + idx];
          } else {
            const float* gc = gcot + node_base(e, sc.b[0] + ox, sc.b[1] + oy, sc.b[2] + oz);
            mb[oz] = gc[3 * CH];
            for (int a = 0; a < 3; ++a) Pb[oz][a] = gc[(4 + a) * CH];
          }
        }
        float wx, wy, dwx, dwy;
        spline_piece(ox, sc.f[0], wx, dwx);
        spline_piece(oy, sc.f[1], wy, dwy);
        const float wxy = wx * wy, gxw = e.fn * dwx * wy, gyw = e.fn * wx * dwy;
        const float d0 = ((float)ox - sc.f[0]) * e.dx, d1 = ((float)oy - sc.f[1]) * e.dx;
        // column invariant m_p v + A d at d_z = 0; column sums of W Pbar and W Pbar d_z
        float uc[3], cP[3] = {0.f, 0.f, 0.f}, cPz[3] = {0.f, 0.f, 0.f};
        for (int a = 0; a < 3; ++a) uc[a] = fmaf(A.m[a][0], d0, fmaf(A.m[a][1], d1, e.mp * v[a]));
#pragma unroll
        for (int oz = 0; oz < 3; ++oz) {
          const float wz = sc.w[2][oz], dz = ((float)oz - sc.f[2]) * e.dx;
          const float W = wxy * wz, Wd = W * dz;
          const float gW[3] = {gxw * wz, gyw * wz, wxy * e.fn * sc.dw[2][oz]};
          float gw = e.mp * mb[oz];
          for (int a = 0; a < 3; ++a) gw = fmaf(Pb[oz][a], fmaf(A.m[a][2], dz, uc[a]), gw);
          sm = fmaf(W, mb[oz], sm);
          for (int a = 0; a < 3; ++a) {
            cP[a] = fmaf(W, Pb[oz][a], cP[a]);
            cPz[a] = fmaf(Wd, Pb[oz][a], cPz[a]);
            xb[a] = fmaf(gW[a], gw, xb[a]);
          }
        }
        for (int a = 0; a < 3; ++a) {
          sP[a] += cP[a];
          Ab.m[a][0] = fmaf(cP[a], d0, Ab.m[a][0]);
          Ab.m[a][1] = fmaf(cP[a], d1, Ab.m[a][1]);
          Ab.m[a][2] += cPz[a];
        }
      }
    // the stencil sum of -W A^T Pbar is -A^T sP
    for (int a = 0; a < 3; ++a) xb[a] -= A.m[0][a] * sP[0] + A.m[1][a] * sP[1] + A.m[2][a] * sP[2];
    const M3 Cm = ld_m3(st, N, p, 6);
    const M3 H = ld_m3(st, N, p, 15);
    StressPrep spr;
    if (kEig && (mat == MAT_COROTATED || mat == MAT_VONMISES)) {
      M3 U;
      float l[3];
      for (int i = 0; i < 3; ++i) {
        l[i] = eig_keep[9 + i][t];
        for (int j = 0; j < 3; ++j) U.m[i][j] = eig_keep[3 * i + j][t];
      }
      spr = stress_prep_with_eig(H, U, l, mat);
    } else {
      spr = stress_prep(e, H, mat);
    }
    const M3 tau = stress_from(e, spr, mat);
    // m_p enters m_i (weight W) and P_i through m_p (v + C d): the C d part
    // summed over the nodes is <C, sum W Pbar d^T>
    const float mpb = sm + v[0] * sP[0] + v[1] * sP[1] + v[2] * sP[2] + m3_ddot(Cm, Ab);
    for (int a = 0; a < 3; ++a) { cot_out[a * N + p] = xb[a]; cot_out[(3 + a) * N + p] = e.mp * sP[a]; }
    st_m3(cot_out, N, p, 6, m3_scale(Ab, e.mp));
    const M3 taub = m3_scale(Ab, kf);
    pb[PB_VP] += (-e.dt * 4.f * e.fn * e.fn) * m3_ddot(Ab, tau);
    pb[PB_MP] += mpb;
    M3 Fb = ld_m3(part, N, p, 3);
    stress_vjp_from(e, H, spr, taub, Fb, pb, mat);
    st_m3(cot_out, N, p, 15, Fb);
  }
  block_reduce_params_lds(pb, pacc + (int64_t)it.env * 8);
}

// one block per work item, or (PERSIST) a grid that strides over the items
template <bool PERSIST, int BOXN, int MAT>
// four waves per SIMD: the stress VJP would otherwise hold ~150 VGPRs and
// leave three; the compiler spills a few registers instead
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4, 8))) k_p2g_adjoint_lds(const float* __restrict__ st,
                                                         const float* __restrict__ part,
                                                         float* __restrict__ cot_out, int64_t N,
                                                         const EnvDev* __restrict__ envs,
                                                         const WorkItem* __restrict__ items,
                                                         const float* __restrict__ gcot,
                                                         double* __restrict__ pacc, int k_call, const float* __restrict__ cot_in, int n_items) {
  if (PERSIST) {
    for (int i = blockIdx.x; i < n_items; i += gridDim.x) {
      p2g_adjoint_lds_item<BOXN, MAT>(i, st, part, cot_out, N, envs, items, gcot, pacc, k_call, cot_in);
      __syncthreads();
    }
  } else {
    p2g_adjoint_lds_item<BOXN, MAT>(blockIdx.x, st, part, cot_out, N, envs, items, gcot, pacc, k_call, cot_in);
  }
}

// ----------------------------------------------------------------------------
// Segment-reduced scatter. Sorted particles of the same stencil base (a
// "segment") add to the same 27 nodes. A particle's contribution to node
// base + o is W(o) (q + Abar o) with per-particle q (3) and Abar (3x3), so a
// lane that owns (segment, ox, oy) sums the three z-nodes over the segment's
// particles in registers and then issues one atomic per node and channel.
// ----------------------------------------------------------------------------
constexpr int kItem = 256;

struct SegShared {
  // per particle, four 16-byte rows read with one 128-bit LDS load each:
  // (q0 q1 q2 fx) (A00 A01 A02 fy) (A10 A11 A12 wz0) (A20 A21 A22 wz1), where q
  // is the value at the base node offset o = 0 (before the weight), Abar
  // (row-major) its change per unit node offset, f = x n - base on x and y
  // (each lane evaluates its own x and y weight from it) and wz the first two
  // z weights (the third is 1 - wz0 - wz1)
  float4 pd[kItem][4];
  int key[kItem];        // packed base (10 bits per axis)
  int first[kItem + 1];  // first particle of each segment, then the count
  int wave_sum[4];
  int n_seg;
};

// quadratic B-spline weights of the three nodes from f = x n - base (the
// same expressions as the stencil's)
MD void bspline3(float f, float w[3]) {
  const float f0 = 1.5f - f, f1 = f - 1.f, f2 = f - 0.5f;
  w[0] = 0.5f * f0 * f0;
  w[1] = 0.75f - f1 * f1;
  w[2] = 0.5f * f2 * f2;
}

MD int pack_base(const int b[3]) { return (b[0] << 20) | (b[1] << 10) | b[2]; }

// stores particle t's scatter data: q (3), Abar (3x3, row-major), f (3)
MD void seg_store(SegShared& sh, int t, const float q[3], const float ab[3][3], const float f[3]) {
  float wz[3];
  bspline3(f[2], wz);
  sh.pd[t][0] = make_float4(q[0], q[1], q[2], f[0]);
  sh.pd[t][1] = make_float4(ab[0][0], ab[0][1], ab[0][2], f[1]);
  sh.pd[t][2] = make_float4(ab[1][0], ab[1][1], ab[1][2], wz[0]);
  sh.pd[t][3] = make_float4(ab[2][0], ab[2][1], ab[2][2], wz[1]);
}

// marks segment starts among the item's particles (thread t <-> particle t)
// and fills first[] / n_seg; a run of one stencil base is cut at every
// max_run-th item position so that long runs spread over more lanes. Every
// thread must call it.
MD void find_segments(SegShared& sh, int count, int max_run) {
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const bool valid = t < count;
  const bool start = valid && (t == 0 || sh.key[t] != sh.key[t - 1] || (t % max_run) == 0);
  const uint64_t bal = __ballot(start);
  const uint64_t lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));
  const int before = __popcll(bal & lt);
  if (lane == 0) sh.wave_sum[wave] = __popcll(bal);
  __syncthreads();
  int off = 0;
  for (int w = 0; w < wave; ++w) off += sh.wave_sum[w];
  if (start) sh.first[off + before] = t;
  if (t == 0) {
    int tot = 0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) tot += sh.wave_sum[w];
    sh.n_seg = tot;
    sh.first[tot] = count;
  }
  __syncthreads();
}

// phase 2: NCH channels; channel 0 is the weight sum times `mass` when
// WITH_MASS, the remaining three the affine value. Writes into the LDS box
// (fits) or straight to grid channels c0.. with global atomics. A lane owns
// (segment, ox, oy) and sums the segment's particles for the three z-nodes of
// that column in registers: nine lanes per segment, which read the same
// particle data (LDS broadcast), so a segment of k particles costs a chain of
// k short iterations rather than k long ones.
template <bool WITH_MASS>
MD void segment_scatter(const EnvDev& e, const Box& bx, const BoxShared& bs, const SegShared& sh, float mass, float* lds_box,
                        float* __restrict__ g, int c0) {
  constexpr int NCH = WITH_MASS ? 4 : 3;
  const int units = 9 * sh.n_seg;
  for (int u = threadIdx.x; u < units; u += blockDim.x) {
    const int seg = u / 9, r = u - 9 * seg, ox = r / 3, oy = r - 3 * ox;
    const int p0 = sh.first[seg], p1 = sh.first[seg + 1];
    float am[3], ap[3][3];
#pragma unroll
    for (int z = 0; z < 3; ++z) {
      am[z] = 0.f;
      ap[z][0] = ap[z][1] = ap[z][2] = 0.f;
    }
    // the lane's x and y weights, each B-spline piece as k (f - s)^2 + m with
    // (k, s, m) fixed per lane: no per-particle select (which the compiler
    // turns into divergent branches that stall the LDS loads)
    const float kx = ox == 1 ? -1.f : 0.5f, sx = ox == 0 ? 1.5f : (ox == 1 ? 1.f : 0.5f), mx = ox == 1 ? 0.75f : 0.f;
    const float ky = oy == 1 ? -1.f : 0.5f, sy = oy == 0 ? 1.5f : (oy == 1 ? 1.f : 0.5f), my = oy == 1 ? 0.75f : 0.f;
    // one particle's contribution to the lane's three z-nodes
    auto add = [&](int p) {
      const float4 P0 = sh.pd[p][0], P1 = sh.pd[p][1], P2 = sh.pd[p][2], P3 = sh.pd[p][3];
      const float w2[3] = {P2.w, P3.w, 1.f - P2.w - P3.w};
      const float dx0 = P0.w - sx, dy0 = P1.w - sy;
      const float wxy = fmaf(kx * dx0, dx0, mx) * fmaf(ky * dy0, dy0, my);
      const float fx = (float)ox, fy = (float)oy;
      const float r0[3] = {P0.x + P1.x * fx + P1.y * fy, P0.y + P2.x * fx + P2.y * fy, P0.z + P3.x * fx + P3.y * fy};
      const float az[3] = {P1.z, P2.z, P3.z};
      // r0 + az z for z = 0, 1, 2, written out (0 * az would not fold away)
      const float W0 = wxy * w2[0], W1 = wxy * w2[1], W2 = wxy * w2[2];
      am[0] += W0;
      am[1] += W1;
      am[2] += W2;
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        ap[0][a] = fmaf(W0, r0[a], ap[0][a]);
        ap[1][a] = fmaf(W1, r0[a] + az[a], ap[1][a]);
        ap[2][a] = fmaf(W2, fmaf(2.f, az[a], r0[a]), ap[2][a]);
      }
    };
    int p = p0;
    for (; p + 1 < p1; p += 2) {   // two at a time so that their LDS loads overlap
      add(p);
      add(p + 1);
    }
    if (p < p1) add(p);
    const int key = sh.key[p0];
    const int bx0 = (key >> 20) + ox, by0 = ((key >> 10) & 1023) + oy, bz0 = key & 1023;
#pragma unroll
    for (int z = 0; z < 3; ++z) {
      float v[4];
      int k = 0;
      if (WITH_MASS) v[k++] = am[z] * mass;
      for (int a = 0; a < 3; ++a) v[k++] = ap[z][a];
      if (bx.fits) {
        const int idx = box_index_run(bs, bs.run[p0], bx0, by0, bz0 + z);
        for (int c = 0; c < NCH; ++c) atomicAdd(&lds_box[c * bx.nodes + idx], v[c]);
      } else {
        float* dst = g + node_base(e, bx0, by0, bz0 + z) + c0 * CH;
        for (int c = 0; c < NCH; ++c) atomicAdd(dst + c * CH, v[c]);
      }
    }
  }
}

// P2G with segment reduction for the item's particles at positions x (thread
// t <-> particle t of the item); load_rest(v, C, H) supplies the rest of the
// particle's state once the block has set up its boxes. Every thread calls it.
template <int BOXN, typename LoadRest>
MD void p2g_seg_body(const EnvDev& e, int mat, const WorkItem& it, const float x[3], LoadRest load_rest,
                     float* __restrict__ grid, uint32_t* __restrict__ flags, int32_t* __restrict__ errs, int min_run,
                     int max_run, float* lds, BoxShared& bsh, SegShared& sh) {
  const int t = threadIdx.x;
  const bool valid = t < it.count;
  const Stencil sc = make_stencil(x, e.n, e.fn);
  if (valid && sc.oob) atomicOr(&errs[it.env], ERR_OUT_OF_DOMAIN);
  sh.key[t] = pack_base(sc.b);
  const Box bx = block_box<BOXN>(e, sc.b, valid, t, it.count, bsh);   // synchronizes
  find_segments(sh, it.count, max_run);        // synchronizes
  const bool seg_mode = it.count >= min_run * sh.n_seg;   // uniform across the block
  if (bx.fits)
    for (int i = t; i < 4 * bx.nodes; i += blockDim.x) lds[i] = 0.f;
  __syncthreads();   // the LDS box is clear before any lane adds to it
  if (valid) {
    float v[3];
    M3 Cm, H;
    load_rest(v, Cm, H);
    const M3 tau = stress(e, H, mat);
    const float kf = -e.dt * e.vp * 4.f * e.fn * e.fn;
    const M3 A = m3_axpy(m3_scale(Cm, e.mp), kf, tau);
    if (seg_mode) {
      float q[3], ab[3][3];
      for (int a = 0; a < 3; ++a) {
        q[a] = e.mp * v[a];
        for (int b = 0; b < 3; ++b) {
          ab[a][b] = A.m[a][b] * e.dx;
          q[a] = fmaf(-ab[a][b], sc.f[b], q[a]);
        }
      }
      seg_store(sh, t, q, ab, sc.f);
    } else {
      for (int ox = 0; ox < 3; ++ox)
#pragma unroll
        for (int oy = 0; oy < 3; ++oy)
#pragma unroll
          for (int oz = 0; oz < 3; ++oz) {
            float W, d[3];
            stencil_offsets(sc, e, ox, oy, oz, W, d);
            float q[4];
            q[0] = W * e.mp;
            for (int a = 0; a < 3; ++a) q[1 + a] = W * (e.mp * v[a] + A.m[a][0] * d[0] + A.m[a][1] * d[1] + A.m[a][2] * d[2]);
            if (bx.fits) {
              const int idx = box_index(bx, sc.b[0] + ox, sc.b[1] + oy, sc.b[2] + oz);
              for (int c = 0; c < 4; ++c) atomicAdd(&lds[c * bx.nodes + idx], q[c]);
            } else {
              float* g = grid + node_base(e, sc.b[0] + ox, sc.b[1] + oy, sc.b[2] + oz);
              for (int c = 0; c < 4; ++c) atomicAdd(g + c * CH, q[c]);
            }
          }
    }
  }
  __syncthreads();
  if (seg_mode) {
    segment_scatter<true>(e, bx, bsh, sh, e.mp, lds, grid, 0);
    __syncthreads();
  }
  if (bx.fits) {
    box_flush(e, bx, bsh, grid, 0, 4, lds, true);
    box_mark_tiles(e, bsh, flags);
  } else if (valid) {
    mark_particle_tiles(e, sc.b, flags);
  }
}

template <int BOXN, int MAT>
MD void p2g_seg_item(int item_idx, const float* __restrict__ st, int64_t N,
                                                 const EnvDev* __restrict__ envs, const WorkItem* __restrict__ items,
                                                 float* __restrict__ grid, uint32_t* __restrict__ flags,
                                                 int32_t* __restrict__ errs, int runs, int k_call) {
  const int min_run = runs & 0xffff, max_run = runs >> 16;   // seg-mode threshold, run split length
  __shared__ float lds[4 * BOXN];
  __shared__ BoxShared bsh;
  __shared__ SegShared sh;
  const WorkItem it = items[item_idx];
  const EnvDev& e = envs[it.env];
  const int mat = MAT >= 0 ? MAT : e.material;   // MAT < 0: the generic kernel
  if (k_call >= e.nsub) return;   // frozen env: nothing to scatter
  const int t = threadIdx.x;
  const int64_t p = it.start + (t < it.count ? t : 0);
  float x[3];
  load_x3(st, N, p, x);
  p2g_seg_body<BOXN>(e, mat, it, x, [&](float v[3], M3& Cm, M3& H) {
    for (int a = 0; a < 3; ++a) v[a] = st[(3 + a) * N + p];
    Cm = ld_m3(st, N, p, 6);
    H = ld_m3(st, N, p, 15);
  }, grid, flags, errs, min_run, max_run, lds, bsh, sh);
}

// G2P of substep k fused with P2G of substep k + 1: the particle's new state
// stays in registers between the gather from grid k and the scatter into grid
// k + 1 (thread t <-> particle t). k_call is substep k's call index; an env
// frozen at k copies its state, one frozen at k + 1 only takes the G2P.
template <int BOXN, int MAT>
MD void g2p2g_item(int item_idx, const float* __restrict__ st, float* __restrict__ out, int64_t N,
                   const EnvDev* __restrict__ envs, const WorkItem* __restrict__ items,
                   const float* __restrict__ grid_in, float* __restrict__ grid_out, uint32_t* __restrict__ flags_out,
                   int32_t* __restrict__ errs, int runs, int k_call) {
  const int min_run = runs & 0xffff, max_run = runs >> 16;
  __shared__ float lds[4 * BOXN];
  __shared__ BoxShared bsh;
  __shared__ SegShared sh;
  const WorkItem it = items[item_idx];
  const EnvDev& e = envs[it.env];
  const int mat = MAT >= 0 ? MAT : e.material;
  const int t = threadIdx.x;
  const bool valid = t < it.count;
  const int64_t p = it.start + (valid ? t : 0);
  if (k_call >= e.nsub) {   // frozen env: the substep is the identity
    if (valid)
      for (int c = 0; c < 24; ++c) out[c * N + p] = st[c * N + p];
    return;
  }
  // G2P (substep k), gathering straight from grid k
  float x[3];
  load_x3(st, N, p, x);
  const M3 H = ld_m3(st, N, p, 15);
  float vn[3] = {0.f, 0.f, 0.f};
  M3 Cn = m3_zero();
  if (valid) {
    const Stencil sc = make_stencil(x, e.n, e.fn);
    const StencilAddr sa = stencil_addr(e, sc.b);
    const float* genv = grid_in + (int64_t)e.tile_off * 512;
    // z offsets and their weighted copies, per particle
    float dz[3], wdz[3];
    for (int o = 0; o < 3; ++o) {
      dz[o] = ((float)o - sc.f[2]) * e.dx;
      wdz[o] = sc.w[2][o] * dz[o];
    }
#pragma unroll 1
    for (int ox = 0; ox < 3; ++ox) {
      const uint32_t ax = ox == 0 ? sa.x[0] : (ox == 1 ? sa.x[1] : sa.x[2]);
      const float wx = sel3(sc.w[0], ox), d0 = ((float)ox - sc.f[0]) * e.dx;
#pragma unroll
      for (int oy = 0; oy < 3; ++oy) {
        // a z-column shares d_x and d_y: sum W v_i and W v_i d_z over it,
        // then add the column into v and C
        const float wxy = wx * sc.w[1][oy], d1 = ((float)oy - sc.f[1]) * e.dx;
        float col[3] = {0.f, 0.f, 0.f}, colz[3] = {0.f, 0.f, 0.f};
#pragma unroll
        for (int oz = 0; oz < 3; ++oz) {
          const float* g = genv + (ax + sa.y[oy] + sa.z[oz]);
          const float vi[3] = {g[4 * CH], g[5 * CH], g[6 * CH]};
          const float W = wxy * sc.w[2][oz], Wd = wxy * wdz[oz];
#pragma unroll
          for (int a = 0; a < 3; ++a) {
            col[a] = fmaf(W, vi[a], col[a]);
            colz[a] = fmaf(Wd, vi[a], colz[a]);
          }
        }
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          vn[a] += col[a];
          Cn.m[a][0] = fmaf(col[a], d0, Cn.m[a][0]);
          Cn.m[a][1] = fmaf(col[a], d1, Cn.m[a][1]);
          Cn.m[a][2] += colz[a];
        }
      }
    }
  }
  Cn = m3_scale(Cn, 4.f * e.fn * e.fn);
  float xn[3];
  for (int a = 0; a < 3; ++a) xn[a] = fmaf(e.dt, vn[a], x[a]);
  const M3 Hn = project(e, trial_h(e, Cn, H), mat);
  if (valid) {
    for (int a = 0; a < 3; ++a) { out[a * N + p] = xn[a]; out[(3 + a) * N + p] = vn[a]; }
    st_m3(out, N, p, 6, Cn);
    st_m3(out, N, p, 15, Hn);
    bool fin = true;
    for (int a = 0; a < 3; ++a) fin = fin && isfinite(xn[a]) && isfinite(vn[a]);
    for (int i = 0; i < 3; ++i) for (int j = 0; j < 3; ++j) fin = fin && isfinite(Hn.m[i][j]);
    if (!fin) atomicOr(&errs[it.env], ERR_NONFINITE);
  }
  if (k_call + 1 >= e.nsub) return;   // the env stops after this substep (uniform over the block)
  // P2G (substep k + 1) of the state just computed
  p2g_seg_body<BOXN>(e, mat, it, xn, [&](float v[3], M3& Cm, M3& Hh) {
    for (int a = 0; a < 3; ++a) v[a] = vn[a];
    Cm = Cn;
    Hh = Hn;
  }, grid_out, flags_out, errs, min_run, max_run, lds, bsh, sh);
}

template <int BOXN, int MAT>
__global__ void __launch_bounds__(256) k_g2p2g(const float* __restrict__ st, float* __restrict__ out, int64_t N,
                                               const EnvDev* __restrict__ envs, const WorkItem* __restrict__ items,
                                               const float* __restrict__ grid_in, float* __restrict__ grid_out,
                                               uint32_t* __restrict__ flags_out, int32_t* __restrict__ errs, int runs,
                                               int k_call) {
  g2p2g_item<BOXN, MAT>(blockIdx.x, st, out, N, envs, items, grid_in, grid_out, flags_out, errs, runs, k_call);
}

template <int BOXN>
static void launch_g2p2g_m(const float* st, float* out, int64_t N, const EnvDev* envs, const WorkItem* items,
                           int n_items, const float* grid_in, float* grid_out, uint32_t* flags_out, int32_t* errs,
                           int runs, int k_call, hipStream_t s, int mat) {
  const dim3 g(n_items), blk(256);
  switch (mat) {
    case MAT_NEOHOOKEAN: hipLaunchKernelGGL((k_g2p2g<BOXN, MAT_NEOHOOKEAN>), g, blk, 0, s, st, out, N, envs, items, grid_in, grid_out, flags_out, errs, runs, k_call); break;
    case MAT_COROTATED: hipLaunchKernelGGL((k_g2p2g<BOXN, MAT_COROTATED>), g, blk, 0, s, st, out, N, envs, items, grid_in, grid_out, flags_out, errs, runs, k_call); break;
    case MAT_VONMISES: hipLaunchKernelGGL((k_g2p2g<BOXN, MAT_VONMISES>), g, blk, 0, s, st, out, N, envs, items, grid_in, grid_out, flags_out, errs, runs, k_call); break;
    case MAT_FLUID_TAIT: hipLaunchKernelGGL((k_g2p2g<BOXN, MAT_FLUID_TAIT>), g, blk, 0, s, st, out, N, envs, items, grid_in, grid_out, flags_out, errs, runs, k_call); break;
    case MAT_FLUID_PAPER: hipLaunchKernelGGL((k_g2p2g<BOXN, MAT_FLUID_PAPER>), g, blk, 0, s, st, out, N, envs, items, grid_in, grid_out, flags_out, errs, runs, k_call); break;
    case -1: hipLaunchKernelGGL((k_g2p2g<BOXN, -1>), g, blk, 0, s, st, out, N, envs, items, grid_in, grid_out, flags_out, errs, runs, k_call); break;
    default: break;
  }
}

void launch_g2p2g(const float* st, float* out, int64_t N, const EnvDev* envs, const WorkItem* items, int n_items,
                  const float* grid_in, float* grid_out, uint32_t* flags_out, int32_t* errs, int runs, int k_call,
                  int box, int mat, hipStream_t s) {
  if (n_items == 0) return;
  if (box)
    launch_g2p2g_m<kBoxSmall>(st, out, N, envs, items, n_items, grid_in, grid_out, flags_out, errs, runs, k_call, s, mat);
  else
    launch_g2p2g_m<kBoxNodes>(st, out, N, envs, items, n_items, grid_in, grid_out, flags_out, errs, runs, k_call, s, mat);
}

// G2P of substep k fused with the pull P2G of substep k + 1: the new state
// goes to the tape once and is scattered from registers. The G2P gathers
// straight from grid k; the P2G boxes come from the new positions.
template <int BOXN, int MAT>
MD void g2p2g_pull_item(int item_idx, const float* __restrict__ st, float* __restrict__ out, int64_t N,
                        const EnvDev* __restrict__ envs, const WorkItem* __restrict__ items,
                        const float* __restrict__ grid_in, float* __restrict__ grid_out,
                        uint32_t* __restrict__ flags_out, int32_t* __restrict__ errs, int k_call) {
  __shared__ BoxShared bsh;
  __shared__ PullShared<BOXN> ps;
  const WorkItem it = items[item_idx];
  const EnvDev& e = envs[it.env];
  const int mat = MAT >= 0 ? MAT : e.material;
  const int lp = lane_particle(threadIdx.x);
  const bool valid = lp < it.count;
  const int64_t p = it.start + (valid ? lp : 0);
  if (k_call >= e.nsub) {   // frozen env: the substep is the identity
    if (valid)
      for (int c = 0; c < 24; ++c) out[c * N + p] = st[c * N + p];
    return;
  }
  // G2P (substep k)
  float x[3];
  load_x3(st, N, p, x);
  const M3 H = ld_m3(st, N, p, 15);
  float vn[3] = {0.f, 0.f, 0.f};
  M3 Cn = m3_zero();
  if (valid) {
    const Stencil sc = make_stencil(x, e.n, e.fn);
    const StencilAddr sa = stencil_addr(e, sc.b);
    const float* genv = grid_in + (int64_t)e.tile_off * 512;
    float wdz[3];
    for (int o = 0; o < 3; ++o) wdz[o] = sc.w[2][o] * (((float)o - sc.f[2]) * e.dx);
#pragma unroll 1
    for (int ox = 0; ox < 3; ++ox) {
      const uint32_t ax = ox == 0 ? sa.x[0] : (ox == 1 ? sa.x[1] : sa.x[2]);
      const float wx = sel3(sc.w[0], ox), d0 = ((float)ox - sc.f[0]) * e.dx;
#pragma unroll
      for (int oy = 0; oy < 3; ++oy) {
        const float wxy = wx * sc.w[1][oy], d1 = ((float)oy - sc.f[1]) * e.dx;
        float col[3] = {0.f, 0.f, 0.f}, colz[3] = {0.f, 0.f, 0.f};
#pragma unroll
        for (int oz = 0; oz < 3; ++oz) {
          const float* g = genv + (ax + sa.y[oy] + sa.z[oz]);
          const float vi[3] = {g[4 * CH], g[5 * CH], g[6 * CH]};
          const float W = wxy * sc.w[2][oz], Wd = wxy * wdz[oz];
#pragma unroll
          for (int a = 0; a < 3; ++a) {
            col[a] = fmaf(W, vi[a], col[a]);
            colz[a] = fmaf(Wd, vi[a], colz[a]);
          }
        }
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          vn[a] += col[a];
          Cn.m[a][0] = fmaf(col[a], d0, Cn.m[a][0]);
          Cn.m[a][1] = fmaf(col[a], d1, Cn.m[a][1]);
          Cn.m[a][2] += colz[a];
        }
      }
    }
  }
  Cn = m3_scale(Cn, 4.f * e.fn * e.fn);
  float xn[3];
  for (int a = 0; a < 3; ++a) xn[a] = fmaf(e.dt, vn[a], x[a]);
  const M3 Hn = project(e, trial_h(e, Cn, H), mat);
  if (valid) {
    for (int a = 0; a < 3; ++a) { out[a * N + p] = xn[a]; out[(3 + a) * N + p] = vn[a]; }
    st_m3(out, N, p, 6, Cn);
    st_m3(out, N, p, 15, Hn);
    bool fin = true;
    for (int a = 0; a < 3; ++a) fin = fin && isfinite(xn[a]) && isfinite(vn[a]);
    for (int i = 0; i < 3; ++i) for (int j = 0; j < 3; ++j) fin = fin && isfinite(Hn.m[i][j]);
    if (!fin) atomicOr(&errs[it.env], ERR_NONFINITE);
  }
  if (k_call + 1 >= e.nsub) return;   // the env stops after this substep (uniform over the block)
  // pull P2G (substep k + 1) of the state just computed
  const Stencil sc = make_stencil(xn, e.n, e.fn);
  if (valid && sc.oob) atomicOr(&errs[it.env], ERR_OUT_OF_DOMAIN);
  const Box bx = block_box<BOXN>(e, sc.b, valid, lp, it.count, bsh);
  int pos = 0;
  const bool fits = bx.fits && pull_index<BOXN>(bsh, ps, bx, sc.b, valid, pos);
  if (valid) p2g_pull_particle(e, mat, sc, fits, pos, vn, Cn, Hn, ps.pay, grid_out);
  if (!fits) {
    if (valid) mark_particle_tiles(e, sc.b, flags_out);
    return;
  }
  __syncthreads();
  p2g_pull_owners<BOXN>(e, bsh, ps, bx.nodes, grid_out, flags_out);
}

template <int BOXN, int MAT>
__global__ void __launch_bounds__(256) k_g2p2g_pull(const float* __restrict__ st, float* __restrict__ out, int64_t N,
                                                    const EnvDev* __restrict__ envs,
                                                    const WorkItem* __restrict__ items,
                                                    const float* __restrict__ grid_in, float* __restrict__ grid_out,
                                                    uint32_t* __restrict__ flags_out, int32_t* __restrict__ errs,
                                                    int k_call) {
  g2p2g_pull_item<BOXN, MAT>(blockIdx.x, st, out, N, envs, items, grid_in, grid_out, flags_out, errs, k_call);
}

template <int BOXN>
static void launch_g2p2g_pull_m(const float* st, float* out, int64_t N, const EnvDev* envs, const WorkItem* items,
                                int n_items, const float* grid_in, float* grid_out, uint32_t* flags_out,
                                int32_t* errs, int k_call, hipStream_t s, int mat) {
  const dim3 g(n_items), blk(256);
#define G2P2G_PULL(M) \
  hipLaunchKernelGGL((k_g2p2g_pull<BOXN, M>), g, blk, 0, s, st, out, N, envs, items, grid_in, grid_out, flags_out, errs, k_call)
  switch (mat) {
    case MAT_NEOHOOKEAN: G2P2G_PULL(MAT_NEOHOOKEAN); break;
    case MAT_COROTATED: G2P2G_PULL(MAT_COROTATED); break;
    case MAT_VONMISES: G2P2G_PULL(MAT_VONMISES); break;
    case MAT_FLUID_TAIT: G2P2G_PULL(MAT_FLUID_TAIT); break;
    case MAT_FLUID_PAPER: G2P2G_PULL(MAT_FLUID_PAPER); break;
    case -1: G2P2G_PULL(-1); break;
    default: break;
  }
#undef G2P2G_PULL
}

void launch_g2p2g_pull(const float* st, float* out, int64_t N, const EnvDev* envs, const WorkItem* items, int n_items,
                       const float* grid_in, float* grid_out, uint32_t* flags_out, int32_t* errs, int k_call, int box,
                       int mat, hipStream_t s) {
  if (n_items == 0) return;
  if (box)
    launch_g2p2g_pull_m<kPullSmall>(st, out, N, envs, items, n_items, grid_in, grid_out, flags_out, errs, k_call, s, mat);
  else
    launch_g2p2g_pull_m<kPullNodes>(st, out, N, envs, items, n_items, grid_in, grid_out, flags_out, errs, k_call, s, mat);
}

// one block per work item, or (PERSIST) a grid that strides over the items
template <bool PERSIST, int BOXN, int MAT>
__global__ void __launch_bounds__(256) k_p2g_seg(const float* __restrict__ st, int64_t N,
                                                 const EnvDev* __restrict__ envs, const WorkItem* __restrict__ items,
                                                 float* __restrict__ grid, uint32_t* __restrict__ flags,
                                                 int32_t* __restrict__ errs, int runs, int k_call, int n_items) {
  if (PERSIST) {
    for (int i = blockIdx.x; i < n_items; i += gridDim.x) {
      p2g_seg_item<BOXN, MAT>(i, st, N, envs, items, grid, flags, errs, runs, k_call);
      __syncthreads();
    }
  } else {
    p2g_seg_item<BOXN, MAT>(blockIdx.x, st, N, envs, items, grid, flags, errs, runs, k_call);
  }
}

template <int BOXN, int MAT>
static void launch_p2g_seg_t(const float* st, int64_t N, const EnvDev* envs, const WorkItem* items, int n_items, float* grid,
                    uint32_t* flags, int32_t* errs, int runs, int k_call, int grid_cap, hipStream_t s) {
  if (grid_cap > 0 && grid_cap < n_items)
    hipLaunchKernelGGL((k_p2g_seg<true, BOXN, MAT>), dim3(grid_cap), dim3(256), 0, s, st, N, envs, items, grid, flags, errs, runs, k_call, n_items);
  else
    hipLaunchKernelGGL((k_p2g_seg<false, BOXN, MAT>), dim3(n_items), dim3(256), 0, s, st, N, envs, items, grid, flags, errs, runs, k_call, n_items);
}
template <int BOXN>
static void launch_p2g_seg_m(const float* st, int64_t N, const EnvDev* envs, const WorkItem* items, int n_items, float* grid,
                    uint32_t* flags, int32_t* errs, int runs, int k_call, int grid_cap, hipStream_t s, int mat) {
  switch (mat) {
    case MAT_NEOHOOKEAN: launch_p2g_seg_t<BOXN, MAT_NEOHOOKEAN>(st, N, envs, items, n_items, grid, flags, errs, runs, k_call, grid_cap, s); break;
    case MAT_COROTATED: launch_p2g_seg_t<BOXN, MAT_COROTATED>(st, N, envs, items, n_items, grid, flags, errs, runs, k_call, grid_cap, s); break;
    case MAT_VONMISES: launch_p2g_seg_t<BOXN, MAT_VONMISES>(st, N, envs, items, n_items, grid, flags, errs, runs, k_call, grid_cap, s); break;
    case MAT_FLUID_TAIT: launch_p2g_seg_t<BOXN, MAT_FLUID_TAIT>(st, N, envs, items, n_items, grid, flags, errs, runs, k_call, grid_cap, s); break;
    case MAT_FLUID_PAPER: launch_p2g_seg_t<BOXN, MAT_FLUID_PAPER>(st, N, envs, items, n_items, grid, flags, errs, runs, k_call, grid_cap, s); break;
    case -1: launch_p2g_seg_t<BOXN, -1>(st, N, envs, items, n_items, grid, flags, errs, runs, k_call, grid_cap, s); break;
    default: break;
  }
}
void launch_p2g_seg(const float* st, int64_t N, const EnvDev* envs, const WorkItem* items, int n_items, float* grid,
                    uint32_t* flags, int32_t* errs, int runs, int k_call, int grid_cap, int box, int mat, hipStream_t s) {
  if (n_items == 0) return;
  if (box)
    launch_p2g_seg_m<kBoxSmall>(st, N, envs, items, n_items, grid, flags, errs, runs, k_call, grid_cap, s, mat);
  else
    launch_p2g_seg_m<kBoxNodes>(st, N, envs, items, n_items, grid, flags, errs, runs, k_call, grid_cap, s, mat);
}

// G2P adjoint with segment-reduced scatter: thread t <-> particle t
template <int BOXN, int MAT>
MD void g2p_adjoint_seg_item(int item_idx, const float* __restrict__ st, const float* __restrict__ st_next,
    const float* __restrict__ cot,
                                                         float* __restrict__ part, int64_t N,
                                                         const EnvDev* __restrict__ envs,
                                                         const WorkItem* __restrict__ items,
                                                         const float* __restrict__ grid, float* __restrict__ gcot,
                                                         double* __restrict__ pacc, int runs, int k_call) {
  const int min_run = runs & 0xffff, max_run = runs >> 16;   // seg-mode threshold, run split length
  __shared__ float lv[3 * BOXN];
  __shared__ float lg[3 * BOXN];
  __shared__ BoxShared bsh;
  __shared__ SegShared sh;
  const WorkItem it = items[item_idx];
  const EnvDev& e = envs[it.env];
  const int mat = MAT >= 0 ? MAT : e.material;   // MAT < 0: the generic kernel
  if (k_call >= e.nsub) return;   // frozen env: nothing to scatter
  const int t = threadIdx.x;
  const bool valid = t < it.count;
  const int64_t p = it.start + (valid ? t : 0);
  float x[3];
  load_x3(st, N, p, x);
  const Stencil sc = make_stencil(x, e.n, e.fn);
  sh.key[t] = pack_base(sc.b);
  const Box bx = block_box<BOXN>(e, sc.b, valid, t, it.count, bsh);   // synchronizes
  find_segments(sh, it.count, max_run);
  const bool seg_mode = it.count >= min_run * sh.n_seg;
  if (bx.fits) {
    box_load(e, bx, bsh, grid, 4, 3, lv);
    for (int i = t; i < 3 * bx.nodes; i += blockDim.x) lg[i] = 0.f;
  }
  __syncthreads();
  float pb[PB_COUNT] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  if (valid) {
    const M3 H = ld_m3(st, N, p, 15);
    const M3 F = f_of(H);
    const float D4 = 4.f * e.fn * e.fn;
    // C' of the substep's output state, read from the tape (the forward's own value)
    const M3 Cn = load_cnext(st_next, N, p);
    const M3 G = m3_axpy(m3_eye(), e.dt, Cn);
    const M3 Htr = trial_h(e, Cn, H);
    float xb[3], vb[3];
    for (int a = 0; a < 3; ++a) { xb[a] = cot[a * N + p]; vb[a] = cot[(3 + a) * N + p] + e.dt * xb[a]; }
    const M3 Cb_in = ld_m3(cot, N, p, 6);
    const M3 Fb_in = ld_m3(cot, N, p, 15);
    const M3 Ftrb = project_vjp(e, Htr, Fb_in, pb, mat);
    const M3 Cb = m3_axpy(Cb_in, e.dt, m3_mul_abt(Ftrb, F));
    const M3 Fb = m3_mul_atb(G, Ftrb);
    if (seg_mode) {
      // gv(o) = vbar + D4 Cbar (o - f) dx = q + Abar o
      float q[3], ab[3][3];
      for (int a = 0; a < 3; ++a) {
        q[a] = vb[a];
        for (int b = 0; b < 3; ++b) {
          ab[a][b] = D4 * e.dx * Cb.m[a][b];
          q[a] = fmaf(-ab[a][b], sc.f[b], q[a]);
        }
      }
      seg_store(sh, t, q, ab, sc.f);
    }
    st_m3(part, N, p, 3, Fb);   // stored before the stencil loop: fewer live registers in it
    float sv[3] = {0.f, 0.f, 0.f};   // sum of W v_i
    // per particle: the z factors of gW and of the affine cotangent
    float gz[3], cz[3];
    for (int o = 0; o < 3; ++o) gz[o] = e.fn * sc.dw[2][o];
    for (int a = 0; a < 3; ++a) cz[a] = D4 * Cb.m[a][2];
#pragma unroll 1
    for (int ox = 0; ox < 3; ++ox)
#pragma unroll 1
      for (int oy = 0; oy < 3; ++oy) {
        // column invariants: the x/y weight factors and vbar + D4 Cbar d at d_z = 0
        const float wx = sel3(sc.w[0], ox), wy = sel3(sc.w[1], oy);
        const float wxy = wx * wy, gx = e.fn * sel3(sc.dw[0], ox) * wy, gy = e.fn * wx * sel3(sc.dw[1], oy);
        const float d0 = ((float)ox - sc.f[0]) * e.dx, d1 = ((float)oy - sc.f[1]) * e.dx;
        float gc[3];
        for (int a = 0; a < 3; ++a) gc[a] = fmaf(D4, fmaf(Cb.m[a][0], d0, Cb.m[a][1] * d1), vb[a]);
#pragma unroll
        for (int oz = 0; oz < 3; ++oz) {
          const float wz = sc.w[2][oz];
          const float W = wxy * wz;
          const float gW[3] = {gx * wz, gy * wz, wxy * gz[oz]};
          const float d2 = ((float)oz - sc.f[2]) * e.dx;
          float vi[3], gv[3];
          for (int a = 0; a < 3; ++a) gv[a] = fmaf(cz[a], d2, gc[a]);
          if (bx.fits) {
            const int idx = box_index(bx, sc.b[0] + ox, sc.b[1] + oy, sc.b[2] + oz);
            for (int a = 0; a < 3; ++a) {
              vi[a] = lv[a * bx.nodes + idx];
              if (!seg_mode) atomicAdd(&lg[a * bx.nodes + idx], W * gv[a]);
            }
          } else {
            const int64_t nb = node_base(e, sc.b[0] + ox, sc.b[1] + oy, sc.b[2] + oz);
            for (int a = 0; a < 3; ++a) {
              vi[a] = grid[nb + (4 + a) * CH];
              if (!seg_mode) atomicAdd(gcot + nb + a * CH, W * gv[a]);
            }
          }
          const float vg = vi[0] * gv[0] + vi[1] * gv[1] + vi[2] * gv[2];
          for (int a = 0; a < 3; ++a) {
            xb[a] = fmaf(gW[a], vg, xb[a]);
            sv[a] = fmaf(W, vi[a], sv[a]);
          }
        }
      }
    // the stencil sum of -D4 W Cbar^T v_i is -D4 Cbar^T sv
    for (int a = 0; a < 3; ++a) xb[a] -= D4 * (Cb.m[0][a] * sv[0] + Cb.m[1][a] * sv[1] + Cb.m[2][a] * sv[2]);
    for (int a = 0; a < 3; ++a) part[a * N + p] = xb[a];
  }
  __syncthreads();
  if (seg_mode) {
    segment_scatter<false>(e, bx, bsh, sh, 0.f, lg, gcot, 0);
    __syncthreads();
  }
  if (bx.fits) box_flush(e, bx, bsh, gcot, 0, 3, lg, false);
  block_reduce_params_lds(pb, pacc + (int64_t)it.env * 8);
}

// one block per work item, or (PERSIST) a grid that strides over the items;
// five waves per SIMD for the materials whose VJP is light (2-3 registers
// spill), the von Mises and generic variants keep their own allocation
template <bool PERSIST, int BOXN, int MAT>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(BOXN > 512 || MAT < 0 || MAT == MAT_VONMISES ? 3 : 5, 8))) k_g2p_adjoint_seg(const float* __restrict__ st, const float* __restrict__ st_next,
    const float* __restrict__ cot,
                                                         float* __restrict__ part, int64_t N,
                                                         const EnvDev* __restrict__ envs,
                                                         const WorkItem* __restrict__ items,
                                                         const float* __restrict__ grid, float* __restrict__ gcot,
                                                         double* __restrict__ pacc, int runs, int k_call, int n_items) {
  if (PERSIST) {
    for (int i = blockIdx.x; i < n_items; i += gridDim.x) {
      g2p_adjoint_seg_item<BOXN, MAT>(i, st, st_next, cot, part, N, envs, items, grid, gcot, pacc, runs, k_call);
      __syncthreads();
    }
  } else {
    g2p_adjoint_seg_item<BOXN, MAT>(blockIdx.x, st, st_next, cot, part, N, envs, items, grid, gcot, pacc, runs, k_call);
  }
}

template <int BOXN, int MAT>
static void launch_g2p_adjoint_seg_t(const float* st, const float* st_next, const float* cot, float* part, int64_t N, const EnvDev* envs,
                            const WorkItem* items, int n_items, const float* grid, float* gcot, double* pacc,
                            int runs, int k_call, int grid_cap, hipStream_t s) {
  if (grid_cap > 0 && grid_cap < n_items)
    hipLaunchKernelGGL((k_g2p_adjoint_seg<true, BOXN, MAT>), dim3(grid_cap), dim3(256), 0, s, st, st_next, cot, part, N, envs, items, grid, gcot,
                     pacc, runs, k_call, n_items);
  else
    hipLaunchKernelGGL((k_g2p_adjoint_seg<false, BOXN, MAT>), dim3(n_items), dim3(256), 0, s, st, st_next, cot, part, N, envs, items, grid, gcot,
                     pacc, runs, k_call, n_items);
}
template <int BOXN>
static void launch_g2p_adjoint_seg_m(const float* st, const float* st_next, const float* cot, float* part, int64_t N, const EnvDev* envs,
                            const WorkItem* items, int n_items, const float* grid, float* gcot, double* pacc,
                            int runs, int k_call, int grid_cap, hipStream_t s, int mat) {
  switch (mat) {
    case MAT_NEOHOOKEAN: launch_g2p_adjoint_seg_t<BOXN, MAT_NEOHOOKEAN>(st, st_next, cot, part, N, envs, items, n_items, grid, gcot, pacc, runs, k_call, grid_cap, s); break;
    case MAT_COROTATED: launch_g2p_adjoint_seg_t<BOXN, MAT_COROTATED>(st, st_next, cot, part, N, envs, items, n_items, grid, gcot, pacc, runs, k_call, grid_cap, s); break;
    case MAT_VONMISES: launch_g2p_adjoint_seg_t<BOXN, MAT_VONMISES>(st, st_next, cot, part, N, envs, items, n_items, grid, gcot, pacc, runs, k_call, grid_cap, s); break;
    case MAT_FLUID_TAIT: launch_g2p_adjoint_seg_t<BOXN, MAT_FLUID_TAIT>(st, st_next, cot, part, N, envs, items, n_items, grid, gcot, pacc, runs, k_call, grid_cap, s); break;
    case MAT_FLUID_PAPER: launch_g2p_adjoint_seg_t<BOXN, MAT_FLUID_PAPER>(st, st_next, cot, part, N, envs, items, n_items, grid, gcot, pacc, runs, k_call, grid_cap, s); break;
    case -1: launch_g2p_adjoint_seg_t<BOXN, -1>(st, st_next, cot, part, N, envs, items, n_items, grid, gcot, pacc, runs, k_call, grid_cap, s); break;
    default: break;
  }
}
void launch_g2p_adjoint_seg(const float* st, const float* st_next, const float* cot, float* part, int64_t N, const EnvDev* envs,
                            const WorkItem* items, int n_items, const float* grid, float* gcot, double* pacc,
                            int runs, int k_call, int grid_cap, int box, int mat, hipStream_t s) {
  if (n_items == 0) return;
  if (box)
    launch_g2p_adjoint_seg_m<kBoxSmall>(st, st_next, cot, part, N, envs, items, n_items, grid, gcot, pacc, runs, k_call, grid_cap, s, mat);
  else
    launch_g2p_adjoint_seg_m<kBoxNodes>(st, st_next, cot, part, N, envs, items, n_items, grid, gcot, pacc, runs, k_call, grid_cap, s, mat);
}

// ----------------------------------------------------------------------------
// P2G adjoint of substep k fused with the G2P adjoint of substep k - 1. The
// cotangent of the particle's state k stays in registers between phase A (a
// gather of substep k's (mbar, Pbar), grid-cotangent channels 3-6 written by
// its grid adjoint) and phase B (the segment-reduced scatter of substep k - 1's
// node-velocity cotangents into channels 0-2, which that grid adjoint cleared).
// Thread t <-> particle t of the item in both phases; k_call is substep k's
// call index. An env frozen at k takes its state-k cotangent from cot_end, the
// cotangent that entered the segment (every later substep is the identity for
// it); one frozen at k - 1 as well has nothing to do. `part` holds substep k's
// partials on entry and substep k - 1's on exit (each thread reads its own
// particle's before it writes them).
// ----------------------------------------------------------------------------
template <int BOXN, int MAT>
MD void adj_pair_item(int item_idx, const float* __restrict__ st_prev, const float* __restrict__ st, float* part,
                      const float* __restrict__ cot_end, int64_t N, const EnvDev* __restrict__ envs,
                      const WorkItem* __restrict__ items, const float* __restrict__ grid_prev, float* gcot,
                      double* __restrict__ pacc, int runs, int k_call) {
  constexpr bool kEig = MAT == MAT_COROTATED || MAT == MAT_VONMISES || MAT < 0;
  const int min_run = runs & 0xffff, max_run = runs >> 16;
  __shared__ float buf[6 * BOXN];   // phase A: the (mbar, Pbar) box; phase B: node velocities, then their cotangents
  __shared__ BoxShared bsh;
  __shared__ SegShared sh;
  // phase A keeps U and the eigenvalues of B per thread in the first 12 KB of
  // the segment rows, which phase B fills only after block_box's barriers
  float(*eig_keep)[256] = reinterpret_cast<float(*)[256]>(&sh.pd[0][0]);
  static_assert(sizeof(sh.pd) >= 12 * 256 * sizeof(float), "eigen stash exceeds the segment rows");
  const WorkItem it = items[item_idx];
  const EnvDev& e = envs[it.env];
  const int mat = MAT >= 0 ? MAT : e.material;
  if (k_call - 1 >= e.nsub) return;   // frozen at k - 1 and k
  const int t = threadIdx.x;
  const bool valid = t < it.count;
  const int64_t p = it.start + (valid ? t : 0);
  float pb[PB_COUNT] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  // cotangent of state k: x, v, C, F
  float cx[3] = {0.f, 0.f, 0.f}, cv[3] = {0.f, 0.f, 0.f};
  M3 cC = m3_zero(), cF = m3_zero();
  if (k_call >= e.nsub) {   // frozen at k (uniform over the block)
    if (valid) {
      for (int a = 0; a < 3; ++a) { cx[a] = cot_end[a * N + p]; cv[a] = cot_end[(3 + a) * N + p]; }
      cC = ld_m3(cot_end, N, p, 6);
      cF = ld_m3(cot_end, N, p, 15);
    }
  } else {
    // ---- phase A: P2G adjoint of substep k ----
    float x[3];
    load_x3(st, N, p, x);
    const Stencil sc = make_stencil(x, e.n, e.fn);
    const Box bx = block_box<BOXN>(e, sc.b, valid, t, it.count, bsh);
    if (bx.fits) box_load(e, bx, bsh, gcot, 3, 4, buf);
    __syncthreads();
    if (valid) {
      const float kf = -e.dt * e.vp * 4.f * e.fn * e.fn;
      const float v[3] = {st[3 * N + p], st[4 * N + p], st[5 * N + p]};
      M3 A;
      {
        const M3 Cm = ld_m3(st, N, p, 6);
        const M3 H = ld_m3(st, N, p, 15);
        const StressPrep spr = stress_prep(e, H, mat);
        A = m3_axpy(m3_scale(Cm, e.mp), kf, stress_from(e, spr, mat));
        if (kEig && (mat == MAT_COROTATED || mat == MAT_VONMISES)) {
          for (int i = 0; i < 3; ++i) {
            eig_keep[9 + i][t] = spr.l[i];
            for (int j = 0; j < 3; ++j) eig_keep[3 * i + j][t] = spr.U.m[i][j];
          }
        }
      }
      float xb[3] = {part[p], part[N + p], part[2 * N + p]};
      float sP[3] = {0.f, 0.f, 0.f};   // sum of W Pbar
      float sm = 0.f;                  // sum of W mbar
      M3 Ab = m3_zero();               // sum of W Pbar d^T
#pragma unroll 1
      for (int ox = 0; ox < 3; ++ox)
#pragma unroll 1
        for (int oy = 0; oy < 3; ++oy) {
          // the column's three z-nodes are loaded together, then summed
          float mb[3], Pb[3][3];
#pragma unroll
          for (int oz = 0; oz < 3; ++oz) {
            if (bx.fits) {
              const int idx = box_index(bx, sc.b[0] + ox, sc.b[1] + oy, sc.b[2] + oz);
              mb[oz] = buf[idx];
              for (int a = 0; a < 3; ++a) Pb[oz][a] = buf[(1 + a) * bx.nodes + idx];
            } else {
              const float* gc = gcot + node_base(e, sc.b[0] + ox, sc.b[1] + oy, sc.b[2] + oz);
              mb[oz] = gc[3 * CH];
              for (int a = 0; a < 3; ++a) Pb[oz][a] = gc[(4 + a) * CH];
            }
          }
          float wx, wy, dwx, dwy;
          spline_piece(ox, sc.f[0], wx, dwx);
          spline_piece(oy, sc.f[1], wy, dwy);
          const float wxy = wx * wy, gxw = e.fn * dwx * wy, gyw = e.fn * wx * dwy;
          const float d0 = ((float)ox - sc.f[0]) * e.dx, d1 = ((float)oy - sc.f[1]) * e.dx;
          // column invariant m_p v + A d at d_z = 0; column sums of W Pbar and W Pbar d_z
          float uc[3], cP[3] = {0.f, 0.f, 0.f}, cPz[3] = {0.f, 0.f, 0.f};
          for (int a = 0; a < 3; ++a) uc[a] = fmaf(A.m[a][0], d0, fmaf(A.m[a][1], d1, e.mp * v[a]));
#pragma unroll
          for (int oz = 0; oz < 3; ++oz) {
            const float wz = sc.w[2][oz], dz = ((float)oz - sc.f[2]) * e.dx;
            const float W = wxy * wz, Wd = W * dz;
            const float gW[3] = {gxw * wz, gyw * wz, wxy * e.fn * sc.dw[2][oz]};
            float gw = e.mp * mb[oz];
            for (int a = 0; a < 3; ++a) gw = fmaf(Pb[oz][a], fmaf(A.m[a][2], dz, uc[a]), gw);
            sm = fmaf(W, mb[oz], sm);
            for (int a = 0; a < 3; ++a) {
              cP[a] = fmaf(W, Pb[oz][a], cP[a]);
              cPz[a] = fmaf(Wd, Pb[oz][a], cPz[a]);
              xb[a] = fmaf(gW[a], gw, xb[a]);
            }
          }
          for (int a = 0; a < 3; ++a) {
            sP[a] += cP[a];
            Ab.m[a][0] = fmaf(cP[a], d0, Ab.m[a][0]);
            Ab.m[a][1] = fmaf(cP[a], d1, Ab.m[a][1]);
            Ab.m[a][2] += cPz[a];
          }
        }
      // the stencil sum of -W A^T Pbar is -A^T sP
      for (int a = 0; a < 3; ++a) xb[a] -= A.m[0][a] * sP[0] + A.m[1][a] * sP[1] + A.m[2][a] * sP[2];
      const M3 Cm = ld_m3(st, N, p, 6);
      const M3 H = ld_m3(st, N, p, 15);
      StressPrep spr;
      if (kEig && (mat == MAT_COROTATED || mat == MAT_VONMISES)) {
        M3 U;
        float l[3];
        for (int i = 0; i < 3; ++i) {
          l[i] = eig_keep[9 + i][t];
          for (int j = 0; j < 3; ++j) U.m[i][j] = eig_keep[3 * i + j][t];
        }
        spr = stress_prep_with_eig(H, U, l, mat);
      } else {
        spr = stress_prep(e, H, mat);
      }
      const M3 tau = stress_from(e, spr, mat);
      const float mpb = sm + v[0] * sP[0] + v[1] * sP[1] + v[2] * sP[2] + m3_ddot(Cm, Ab);
      for (int a = 0; a < 3; ++a) { cx[a] = xb[a]; cv[a] = e.mp * sP[a]; }
      cC = m3_scale(Ab, e.mp);
      const M3 taub = m3_scale(Ab, kf);
      pb[PB_VP] += (-e.dt * 4.f * e.fn * e.fn) * m3_ddot(Ab, tau);
      pb[PB_MP] += mpb;
      cF = ld_m3(part, N, p, 3);
      stress_vjp_from(e, H, spr, taub, cF, pb, mat);
    }
  }
  // ---- phase B: G2P adjoint of substep k - 1 (state k - 1 -> state k) ----
  float x[3];
  load_x3(st_prev, N, p, x);
  const Stencil sc = make_stencil(x, e.n, e.fn);
  sh.key[t] = pack_base(sc.b);
  const Box bx = block_box<BOXN>(e, sc.b, valid, t, it.count, bsh);   // synchronizes: phase A is done
  find_segments(sh, it.count, max_run);
  const bool seg_mode = it.count >= min_run * sh.n_seg;
  float* lv = buf;
  float* lg = buf + 3 * BOXN;
  if (bx.fits) {
    box_load(e, bx, bsh, grid_prev, 4, 3, lv);
    for (int i = t; i < 3 * bx.nodes; i += blockDim.x) lg[i] = 0.f;
  }
  __syncthreads();
  if (valid) {
    const M3 H = ld_m3(st_prev, N, p, 15);
    const M3 F = f_of(H);
    const float D4 = 4.f * e.fn * e.fn;
    const M3 Cn = load_cnext(st, N, p);   // C of state k, the substep's own output
    const M3 G = m3_axpy(m3_eye(), e.dt, Cn);
    const M3 Htr = trial_h(e, Cn, H);
    float xb[3], vb[3];
    for (int a = 0; a < 3; ++a) { xb[a] = cx[a]; vb[a] = cv[a] + e.dt * cx[a]; }
    const M3 Ftrb = project_vjp(e, Htr, cF, pb, mat);
    const M3 Cb = m3_axpy(cC, e.dt, m3_mul_abt(Ftrb, F));
    const M3 Fb = m3_mul_atb(G, Ftrb);
    if (seg_mode) {
      float q[3], ab[3][3];
      for (int a = 0; a < 3; ++a) {
        q[a] = vb[a];
        for (int b = 0; b < 3; ++b) {
          ab[a][b] = D4 * e.dx * Cb.m[a][b];
          q[a] = fmaf(-ab[a][b], sc.f[b], q[a]);
        }
      }
      seg_store(sh, t, q, ab, sc.f);
    }
    st_m3(part, N, p, 3, Fb);
    float sv[3] = {0.f, 0.f, 0.f};   // sum of W v_i
    // per particle: the z factors of gW and of the affine cotangent
    float gz[3], cz[3];
    for (int o = 0; o < 3; ++o) gz[o] = e.fn * sc.dw[2][o];
    for (int a = 0; a < 3; ++a) cz[a] = D4 * Cb.m[a][2];
#pragma unroll 1
    for (int ox = 0; ox < 3; ++ox)
#pragma unroll 1
      for (int oy = 0; oy < 3; ++oy) {
        // column invariants: the x/y weight factors and vbar + D4 Cbar d at d_z = 0
        const float wx = sel3(sc.w[0], ox), wy = sel3(sc.w[1], oy);
        const float wxy = wx * wy, gx = e.fn * sel3(sc.dw[0], ox) * wy, gy = e.fn * wx * sel3(sc.dw[1], oy);
        const float d0 = ((float)ox - sc.f[0]) * e.dx, d1 = ((float)oy - sc.f[1]) * e.dx;
        float gc[3];
        for (int a = 0; a < 3; ++a) gc[a] = fmaf(D4, fmaf(Cb.m[a][0], d0, Cb.m[a][1] * d1), vb[a]);
#pragma unroll
        for (int oz = 0; oz < 3; ++oz) {
          const float wz = sc.w[2][oz];
          const float W = wxy * wz;
          const float gW[3] = {gx * wz, gy * wz, wxy * gz[oz]};
          const float d2 = ((float)oz - sc.f[2]) * e.dx;
          float vi[3], gv[3];
          for (int a = 0; a < 3; ++a) gv[a] = fmaf(cz[a], d2, gc[a]);
          if (bx.fits) {
            const int idx = box_index(bx, sc.b[0] + ox, sc.b[1] + oy, sc.b[2] + oz);
            for (int a = 0; a < 3; ++a) {
              vi[a] = lv[a * bx.nodes + idx];
              if (!seg_mode) atomicAdd(&lg[a * bx.nodes + idx], W * gv[a]);
            }
          } else {
            const int64_t nb = node_base(e, sc.b[0] + ox, sc.b[1] + oy, sc.b[2] + oz);
            for (int a = 0; a < 3; ++a) {
              vi[a] = grid_prev[nb + (4 + a) * CH];
              if (!seg_mode) atomicAdd(gcot + nb + a * CH, W * gv[a]);
            }
          }
          const float vg = vi[0] * gv[0] + vi[1] * gv[1] + vi[2] * gv[2];
          for (int a = 0; a < 3; ++a) {
            xb[a] = fmaf(gW[a], vg, xb[a]);
            sv[a] = fmaf(W, vi[a], sv[a]);
          }
        }
      }
    // the stencil sum of -D4 W Cbar^T v_i is -D4 Cbar^T sv
    for (int a = 0; a < 3; ++a) xb[a] -= D4 * (Cb.m[0][a] * sv[0] + Cb.m[1][a] * sv[1] + Cb.m[2][a] * sv[2]);
    for (int a = 0; a < 3; ++a) part[a * N + p] = xb[a];
  }
  __syncthreads();
  if (seg_mode) {
    segment_scatter<false>(e, bx, bsh, sh, 0.f, lg, gcot, 0);
    __syncthreads();
  }
  if (bx.fits) box_flush(e, bx, bsh, gcot, 0, 3, lg, false);
  block_reduce_params_lds(pb, pacc + (int64_t)it.env * 8);
}

// four waves per SIMD, as for the P2G adjoint alone (three with the large box,
// whose LDS allows no more)
template <int BOXN, int MAT>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(BOXN > 512 ? 3 : 4, 8)))
k_adj_pair(const float* __restrict__ st_prev, const float* __restrict__ st, float* part,
           const float* __restrict__ cot_end, int64_t N, const EnvDev* __restrict__ envs,
           const WorkItem* __restrict__ items, const float* __restrict__ grid_prev, float* gcot,
           double* __restrict__ pacc, int runs, int k_call) {
  adj_pair_item<BOXN, MAT>(blockIdx.x, st_prev, st, part, cot_end, N, envs, items, grid_prev, gcot, pacc, runs, k_call);
}

template <int BOXN>
static void launch_adj_pair_m(const float* st_prev, const float* st, float* part, const float* cot_end, int64_t N,
                              const EnvDev* envs, const WorkItem* items, int n_items, const float* grid_prev,
                              float* gcot, double* pacc, int runs, int k_call, hipStream_t s, int mat) {
  const dim3 g(n_items), blk(256);
  switch (mat) {
    case MAT_NEOHOOKEAN: hipLaunchKernelGGL((k_adj_pair<BOXN, MAT_NEOHOOKEAN>), g, blk, 0, s, st_prev, st, part, cot_end, N, envs, items, grid_prev, gcot, pacc, runs, k_call); break;
    case MAT_COROTATED: hipLaunchKernelGGL((k_adj_pair<BOXN, MAT_COROTATED>), g, blk, 0, s, st_prev, st, part, cot_end, N, envs, items, grid_prev, gcot, pacc, runs, k_call); break;
    case MAT_VONMISES: hipLaunchKernelGGL((k_adj_pair<BOXN, MAT_VONMISES>), g, blk, 0, s, st_prev, st, part, cot_end, N, envs, items, grid_prev, gcot, pacc, runs, k_call); break;
    case MAT_FLUID_TAIT: hipLaunchKernelGGL((k_adj_pair<BOXN, MAT_FLUID_TAIT>), g, blk, 0, s, st_prev, st, part, cot_end, N, envs, items, grid_prev, gcot, pacc, runs, k_call); break;
    case MAT_FLUID_PAPER: hipLaunchKernelGGL((k_adj_pair<BOXN, MAT_FLUID_PAPER>), g, blk, 0, s, st_prev, st, part, cot_end, N, envs, items, grid_prev, gcot, pacc, runs, k_call); break;
    case -1: hipLaunchKernelGGL((k_adj_pair<BOXN, -1>), g, blk, 0, s, st_prev, st, part, cot_end, N, envs, items, grid_prev, gcot, pacc, runs, k_call); break;
    default: break;
  }
}

void launch_adj_pair(const float* st_prev, const float* st, float* part, const float* cot_end, int64_t N,
                     const EnvDev* envs, const WorkItem* items, int n_items, const float* grid_prev, float* gcot,
                     double* pacc, int runs, int k_call, int box, int mat, hipStream_t s) {
  if (n_items == 0) return;
  if (box)
    launch_adj_pair_m<kBoxSmall>(st_prev, st, part, cot_end, N, envs, items, n_items, grid_prev, gcot, pacc, runs, k_call, s, mat);
  else
    launch_adj_pair_m<kBoxNodes>(st_prev, st, part, cot_end, N, envs, items, n_items, grid_prev, gcot, pacc, runs, k_call, s, mat);
}

// P2G adjoint of substep k fused with the pull G2P adjoint of substep k - 1
// (the low particles-per-cell form of the pair above). Phase A gathers (mbar,
// Pbar) through an LDS box of half the pull budget; phase B scatters the
// grid-velocity cotangent through the owner-computes boxes. The two phases
// use the same LDS: phase B's index is built only after block_box's barriers.
template <int BOXN>
union PairPullShared {
  float box[4 * (BOXN / 2)];
  PullShared<BOXN> ps;
};

template <int BOXN, int MAT>
MD void adj_pair_pull_item(int item_idx, const float* __restrict__ st_prev, const float* __restrict__ st, float* part,
                           const float* __restrict__ cot_end, int64_t N, const EnvDev* __restrict__ envs,
                           const WorkItem* __restrict__ items, const float* __restrict__ grid_prev, float* gcot,
                           double* __restrict__ pacc, int k_call) {
  __shared__ BoxShared bsh;
  __shared__ PairPullShared<BOXN> u;
  const WorkItem it = items[item_idx];
  const EnvDev& e = envs[it.env];
  const int mat = MAT >= 0 ? MAT : e.material;
  if (k_call - 1 >= e.nsub) return;   // frozen at k - 1 and k
  const int lp = lane_particle(threadIdx.x);
  const bool valid = lp < it.count;
  const int64_t p = it.start + (valid ? lp : 0);
  float pb[PB_COUNT] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  // cotangent of state k: x, v, C, F
  float cx[3] = {0.f, 0.f, 0.f}, cv[3] = {0.f, 0.f, 0.f};
  M3 cC = m3_zero(), cF = m3_zero();
  if (k_call >= e.nsub) {   // frozen at k (uniform over the block)
    if (valid) {
      for (int a = 0; a < 3; ++a) { cx[a] = cot_end[a * N + p]; cv[a] = cot_end[(3 + a) * N + p]; }
      cC = ld_m3(cot_end, N, p, 6);
      cF = ld_m3(cot_end, N, p, 15);
    }
  } else {
    // ---- phase A: P2G adjoint of substep k ----
    float x[3];
    load_x3(st, N, p, x);
    const Stencil sc = make_stencil(x, e.n, e.fn);
    const Box bx = block_box<BOXN / 2>(e, sc.b, valid, lp, it.count, bsh);
    if (bx.fits) box_load(e, bx, bsh, gcot, 3, 4, u.box);
    __syncthreads();
    if (valid) {
      const float kf = -e.dt * e.vp * 4.f * e.fn * e.fn;
      const float v[3] = {st[3 * N + p], st[4 * N + p], st[5 * N + p]};
      const M3 Cm = ld_m3(st, N, p, 6);
      const M3 H = ld_m3(st, N, p, 15);
      const M3 A = m3_axpy(m3_scale(Cm, e.mp), kf, stress(e, H, mat));
      float xb[3] = {part[p], part[N + p], part[2 * N + p]};
      float sP[3] = {0.f, 0.f, 0.f};   // sum of W Pbar
      float sm = 0.f;                  // sum of W mbar
      M3 Ab = m3_zero();               // sum of W Pbar d^T
#pragma unroll 1
      for (int ox = 0; ox < 3; ++ox)
#pragma unroll 1
        for (int oy = 0; oy < 3; ++oy) {
          float mb[3], Pb[3][3];
#pragma unroll
          for (int oz = 0; oz < 3; ++oz) {
            if (bx.fits) {
              const int idx = box_index(bx, sc.b[0] + ox, sc.b[1] + oy, sc.b[2] + oz);
              mb[oz] = u.box[idx];
              for (int a = 0; a < 3; ++a) Pb[oz][a] = u.box[(1 + a) * bx.nodes + idx];
            } else {
              const float* gc = gcot + node_base(e, sc.b[0] + ox, sc.b[1] + oy, sc.b[2] + oz);
              mb[oz] = gc[3 * CH];
              for (int a = 0; a < 3; ++a) Pb[oz][a] = gc[(4 + a) * CH];
            }
          }
          float wx, wy, dwx, dwy;
          spline_piece(ox, sc.f[0], wx, dwx);
          spline_piece(oy, sc.f[1], wy, dwy);
          const float wxy = wx * wy, gxw = e.fn * dwx * wy, gyw = e.fn * wx * dwy;
          const float d0 = ((float)ox - sc.f[0]) * e.dx, d1 = ((float)oy - sc.f[1]) * e.dx;
          float uc[3], cP[3] = {0.f, 0.f, 0.f}, cPz[3] = {0.f, 0.f, 0.f};
          for (int a = 0; a < 3; ++a) uc[a] = fmaf(A.m[a][0], d0, fmaf(A.m[a][1], d1, e.mp * v[a]));
#pragma unroll
          for (int oz = 0; oz < 3; ++oz) {
            const float wz = sc.w[2][oz], dz = ((float)oz - sc.f[2]) * e.dx;
            const float W = wxy * wz, Wd = W * dz;
            const float gW[3] = {gxw * wz, gyw * wz, wxy * e.fn * sc.dw[2][oz]};
            float gw = e.mp * mb[oz];
            for (int a = 0; a < 3; ++a) gw = fmaf(Pb[oz][a], fmaf(A.m[a][2], dz, uc[a]), gw);
            sm = fmaf(W, mb[oz], sm);
            for (int a = 0; a < 3; ++a) {
              cP[a] = fmaf(W, Pb[oz][a], cP[a]);
              cPz[a] = fmaf(Wd, Pb[oz][a], cPz[a]);
              xb[a] = fmaf(gW[a], gw, xb[a]);
            }
          }
          for (int a = 0; a < 3; ++a) {
            sP[a] += cP[a];
            Ab.m[a][0] = fmaf(cP[a], d0, Ab.m[a][0]);
            Ab.m[a][1] = fmaf(cP[a], d1, Ab.m[a][1]);
            Ab.m[a][2] += cPz[a];
          }
        }
      // the stencil sum of -W A^T Pbar is -A^T sP
      for (int a = 0; a < 3; ++a) xb[a] -= A.m[0][a] * sP[0] + A.m[1][a] * sP[1] + A.m[2][a] * sP[2];
      const StressPrep spr = stress_prep(e, H, mat);
      const M3 tau = stress_from(e, spr, mat);
      const float mpb = sm + v[0] * sP[0] + v[1] * sP[1] + v[2] * sP[2] + m3_ddot(Cm, Ab);
      for (int a = 0; a < 3; ++a) { cx[a] = xb[a]; cv[a] = e.mp * sP[a]; }
      cC = m3_scale(Ab, e.mp);
      const M3 taub = m3_scale(Ab, kf);
      pb[PB_VP] += (-e.dt * 4.f * e.fn * e.fn) * m3_ddot(Ab, tau);
      pb[PB_MP] += mpb;
      cF = ld_m3(part, N, p, 3);
      stress_vjp_from(e, H, spr, taub, cF, pb, mat);
    }
  }
  // ---- phase B: G2P adjoint of substep k - 1 (state k - 1 -> state k) through the pull scatter ----
  float x[3];
  load_x3(st_prev, N, p, x);
  const Stencil sc = make_stencil(x, e.n, e.fn);
  const Box bx = block_box<BOXN>(e, sc.b, valid, lp, it.count, bsh);   // synchronizes: phase A is done
  int pos = 0;
  const bool fits = bx.fits && pull_index<BOXN>(bsh, u.ps, bx, sc.b, valid, pos);
  if (valid) {
    const M3 H = ld_m3(st_prev, N, p, 15);
    const M3 F = f_of(H);
    const float D4 = 4.f * e.fn * e.fn;
    const M3 Cn = load_cnext(st, N, p);   // C of state k, the substep's own output
    const M3 G = m3_axpy(m3_eye(), e.dt, Cn);
    const M3 Htr = trial_h(e, Cn, H);
    float xb[3], vb[3];
    for (int a = 0; a < 3; ++a) { xb[a] = cx[a]; vb[a] = cv[a] + e.dt * cx[a]; }
    const M3 Ftrb = project_vjp(e, Htr, cF, pb, mat);
    const M3 Cb = m3_axpy(cC, e.dt, m3_mul_abt(Ftrb, F));
    const M3 Fb = m3_mul_atb(G, Ftrb);
    st_m3(part, N, p, 3, Fb);
    if (fits) {
      float Ad[3][3];
      for (int a = 0; a < 3; ++a)
        for (int c = 0; c < 3; ++c) Ad[a][c] = D4 * e.dx * Cb.m[a][c];
      pull_store_payload(u.ps.pay, pos, sc.f, sc.b[2], vb, Ad);
    }
    float sv[3] = {0.f, 0.f, 0.f};   // sum of W v_i
    float gz[3], cz[3];
    for (int o = 0; o < 3; ++o) gz[o] = e.fn * sc.dw[2][o];
    for (int a = 0; a < 3; ++a) cz[a] = D4 * Cb.m[a][2];
#pragma unroll 1
    for (int ox = 0; ox < 3; ++ox)
#pragma unroll 1
      for (int oy = 0; oy < 3; ++oy) {
        const float wx = sel3(sc.w[0], ox), wy = sel3(sc.w[1], oy);
        const float wxy = wx * wy, gx = e.fn * sel3(sc.dw[0], ox) * wy, gy = e.fn * wx * sel3(sc.dw[1], oy);
        const float d0 = ((float)ox - sc.f[0]) * e.dx, d1 = ((float)oy - sc.f[1]) * e.dx;
        float gc[3];
        for (int a = 0; a < 3; ++a) gc[a] = fmaf(D4, fmaf(Cb.m[a][0], d0, Cb.m[a][1] * d1), vb[a]);
#pragma unroll
        for (int oz = 0; oz < 3; ++oz) {
          const float wz = sc.w[2][oz];
          const float W = wxy * wz;
          const float gW[3] = {gx * wz, gy * wz, wxy * gz[oz]};
          const float d2 = ((float)oz - sc.f[2]) * e.dx;
          float vi[3], gv[3];
          for (int a = 0; a < 3; ++a) gv[a] = fmaf(cz[a], d2, gc[a]);
          const int64_t nb = node_base(e, sc.b[0] + ox, sc.b[1] + oy, sc.b[2] + oz);
          for (int a = 0; a < 3; ++a) vi[a] = grid_prev[nb + (4 + a) * CH];
          if (!fits)
            for (int a = 0; a < 3; ++a) atomicAdd(gcot + nb + a * CH, W * gv[a]);
          const float vg = vi[0] * gv[0] + vi[1] * gv[1] + vi[2] * gv[2];
          for (int a = 0; a < 3; ++a) {
            xb[a] = fmaf(gW[a], vg, xb[a]);
            sv[a] = fmaf(W, vi[a], sv[a]);
          }
        }
      }
    for (int a = 0; a < 3; ++a) xb[a] -= D4 * (Cb.m[0][a] * sv[0] + Cb.m[1][a] * sv[1] + Cb.m[2][a] * sv[2]);
    for (int a = 0; a < 3; ++a) part[a * N + p] = xb[a];
  }
  if (fits) {
    __syncthreads();
    for (int idx = threadIdx.x; idx < bx.nodes; idx += blockDim.x) {
      int r, i, j, k;
      box_node_run(bsh, idx, r, i, j, k);
      float acc[3] = {0.f, 0.f, 0.f}, wsum = 0.f;
      pull_node(bsh, u.ps.start, u.ps.coff, u.ps.cext, u.ps.pay, r, i, j, k, acc, wsum);
      if (wsum == 0.f) continue;
      float* dst = gcot + node_base(e, i, j, k);
      for (int a = 0; a < 3; ++a)
        if (acc[a] != 0.f) atomicAdd(dst + a * CH, acc[a]);
    }
  }
  block_reduce_params_lds(pb, pacc + (int64_t)it.env * 8);
}

template <int BOXN, int MAT>
__global__ void __launch_bounds__(256)
k_adj_pair_pull(const float* __restrict__ st_prev, const float* __restrict__ st, float* part,
                const float* __restrict__ cot_end, int64_t N, const EnvDev* __restrict__ envs,
                const WorkItem* __restrict__ items, const float* __restrict__ grid_prev, float* gcot,
                double* __restrict__ pacc, int k_call) {
  adj_pair_pull_item<BOXN, MAT>(blockIdx.x, st_prev, st, part, cot_end, N, envs, items, grid_prev, gcot, pacc, k_call);
}

template <int BOXN>
static void launch_adj_pair_pull_m(const float* st_prev, const float* st, float* part, const float* cot_end, int64_t N,
                                   const EnvDev* envs, const WorkItem* items, int n_items, const float* grid_prev,
                                   float* gcot, double* pacc, int k_call, hipStream_t s, int mat) {
  const dim3 g(n_items), blk(256);
#define ADJ_PAIR_PULL(M) \
  hipLaunchKernelGGL((k_adj_pair_pull<BOXN, M>), g, blk, 0, s, st_prev, st, part, cot_end, N, envs, items, grid_prev, \
                     gcot, pacc, k_call)
  switch (mat) {
    case MAT_NEOHOOKEAN: ADJ_PAIR_PULL(MAT_NEOHOOKEAN); break;
    case MAT_COROTATED: ADJ_PAIR_PULL(MAT_COROTATED); break;
    case MAT_VONMISES: ADJ_PAIR_PULL(MAT_VONMISES); break;
    case MAT_FLUID_TAIT: ADJ_PAIR_PULL(MAT_FLUID_TAIT); break;
    case MAT_FLUID_PAPER: ADJ_PAIR_PULL(MAT_FLUID_PAPER); break;
    case -1: ADJ_PAIR_PULL(-1); break;
    default: break;
  }
#undef ADJ_PAIR_PULL
}

void launch_adj_pair_pull(const float* st_prev, const float* st, float* part, const float* cot_end, int64_t N,
                          const EnvDev* envs, const WorkItem* items, int n_items, const float* grid_prev, float* gcot,
                          double* pacc, int k_call, int box, int mat, hipStream_t s) {
  if (n_items == 0) return;
  if (box)
    launch_adj_pair_pull_m<kPullSmall>(st_prev, st, part, cot_end, N, envs, items, n_items, grid_prev, gcot, pacc,
                                       k_call, s, mat);
  else
    launch_adj_pair_pull_m<kPullNodes>(st_prev, st, part, cot_end, N, envs, items, n_items, grid_prev, gcot, pacc,
                                       k_call, s, mat);
}

template <int BOXN, int MAT>
static void launch_p2g_lds_t(const float* st, int64_t N, const EnvDev* envs, const WorkItem* items, int n_items, float* grid,
                    uint32_t* flags, int32_t* errs, int k_call, int grid_cap, hipStream_t s) {
  if (grid_cap > 0 && grid_cap < n_items)
    hipLaunchKernelGGL((k_p2g_lds<true, BOXN, MAT>), dim3(grid_cap), dim3(256), 0, s, st, N, envs, items, grid, flags, errs, k_call, n_items);
  else
    hipLaunchKernelGGL((k_p2g_lds<false, BOXN, MAT>), dim3(n_items), dim3(256), 0, s, st, N, envs, items, grid, flags, errs, k_call, n_items);
}
template <int BOXN>
static void launch_p2g_lds_m(const float* st, int64_t N, const EnvDev* envs, const WorkItem* items, int n_items, float* grid,
                    uint32_t* flags, int32_t* errs, int k_call, int grid_cap, hipStream_t s, int mat) {
  switch (mat) {
    case MAT_NEOHOOKEAN: launch_p2g_lds_t<BOXN, MAT_NEOHOOKEAN>(st, N, envs, items, n_items, grid, flags, errs, k_call, grid_cap, s); break;
    case MAT_COROTATED: launch_p2g_lds_t<BOXN, MAT_COROTATED>(st, N, envs, items, n_items, grid, flags, errs, k_call, grid_cap, s); break;
    case MAT_VONMISES: launch_p2g_lds_t<BOXN, MAT_VONMISES>(st, N, envs, items, n_items, grid, flags, errs, k_call, grid_cap, s); break;
    case MAT_FLUID_TAIT: launch_p2g_lds_t<BOXN, MAT_FLUID_TAIT>(st, N, envs, items, n_items, grid, flags, errs, k_call, grid_cap, s); break;
    case MAT_FLUID_PAPER: launch_p2g_lds_t<BOXN, MAT_FLUID_PAPER>(st, N, envs, items, n_items, grid, flags, errs, k_call, grid_cap, s); break;
    case -1: launch_p2g_lds_t<BOXN, -1>(st, N, envs, items, n_items, grid, flags, errs, k_call, grid_cap, s); break;
    default: break;
  }
}
void launch_p2g_lds(const float* st, int64_t N, const EnvDev* envs, const WorkItem* items, int n_items, float* grid,
                    uint32_t* flags, int32_t* errs, int k_call, int grid_cap, int box, int mat, hipStream_t s) {
  if (n_items == 0) return;
  if (box)
    launch_p2g_lds_m<kBoxSmall>(st, N, envs, items, n_items, grid, flags, errs, k_call, grid_cap, s, mat);
  else
    launch_p2g_lds_m<kBoxNodes>(st, N, envs, items, n_items, grid, flags, errs, k_call, grid_cap, s, mat);
}
template <int BOXN, int MAT>
static void launch_g2p_lds_t(const float* st, float* out, int64_t N, const EnvDev* envs, const WorkItem* items, int n_items,
                    const float* grid, int32_t* errs, int k_call, int grid_cap, hipStream_t s) {
  if (grid_cap > 0 && grid_cap < n_items)
    hipLaunchKernelGGL((k_g2p_lds<true, BOXN, MAT>), dim3(grid_cap), dim3(256), 0, s, st, out, N, envs, items, grid, errs, k_call, n_items);
  else
    hipLaunchKernelGGL((k_g2p_lds<false, BOXN, MAT>), dim3(n_items), dim3(256), 0, s, st, out, N, envs, items, grid, errs, k_call, n_items);
}
template <int BOXN>
static void launch_g2p_lds_m(const float* st, float* out, int64_t N, const EnvDev* envs, const WorkItem* items, int n_items,
                    const float* grid, int32_t* errs, int k_call, int grid_cap, hipStream_t s, int mat) {
  switch (mat) {
    case MAT_NEOHOOKEAN: launch_g2p_lds_t<BOXN, MAT_NEOHOOKEAN>(st, out, N, envs, items, n_items, grid, errs, k_call, grid_cap, s); break;
    case MAT_COROTATED: launch_g2p_lds_t<BOXN, MAT_COROTATED>(st, out, N, envs, items, n_items, grid, errs, k_call, grid_cap, s); break;
    case MAT_VONMISES: launch_g2p_lds_t<BOXN, MAT_VONMISES>(st, out, N, envs, items, n_items, grid, errs, k_call, grid_cap, s); break;
    case MAT_FLUID_TAIT: launch_g2p_lds_t<BOXN, MAT_FLUID_TAIT>(st, out, N, envs, items, n_items, grid, errs, k_call, grid_cap, s); break;
    case MAT_FLUID_PAPER: launch_g2p_lds_t<BOXN, MAT_FLUID_PAPER>(st, out, N, envs, items, n_items, grid, errs, k_call, grid_cap, s); break;
    case -1: launch_g2p_lds_t<BOXN, -1>(st, out, N, envs, items, n_items, grid, errs, k_call, grid_cap, s); break;
    default: break;
  }
}
void launch_g2p_lds(const float* st, float* out, int64_t N, const EnvDev* envs, const WorkItem* items, int n_items,
                    const float* grid, int32_t* errs, int k_call, int grid_cap, int box, int mat, hipStream_t s) {
  if (n_items == 0) return;
  if (box)
    launch_g2p_lds_m<kBoxSmall>(st, out, N, envs, items, n_items, grid, errs, k_call, grid_cap, s, mat);
  else
    launch_g2p_lds_m<kBoxNodes>(st, out, N, envs, items, n_items, grid, errs, k_call, grid_cap, s, mat);
}
template <int BOXN, int MAT>
static void launch_g2p_adjoint_lds_t(const float* st, const float* st_next, const float* cot, float* part, int64_t N, const EnvDev* envs,
                            const WorkItem* items, int n_items, const float* grid, float* gcot, double* pacc,
                            int k_call, int grid_cap, hipStream_t s) {
  if (grid_cap > 0 && grid_cap < n_items)
    hipLaunchKernelGGL((k_g2p_adjoint_lds<true, BOXN, MAT>), dim3(grid_cap), dim3(256), 0, s, st, st_next, cot, part, N, envs, items, grid, gcot,
                     pacc, k_call, n_items);
  else
    hipLaunchKernelGGL((k_g2p_adjoint_lds<false, BOXN, MAT>), dim3(n_items), dim3(256), 0, s, st, st_next, cot, part, N, envs, items, grid, gcot,
                     pacc, k_call, n_items);
}
template <int BOXN>
static void launch_g2p_adjoint_lds_m(const float* st, const float* st_next, const float* cot, float* part, int64_t N, const EnvDev* envs,
                            const WorkItem* items, int n_items, const float* grid, float* gcot, double* pacc,
                            int k_call, int grid_cap, hipStream_t s, int mat) {
  switch (mat) {
    case MAT_NEOHOOKEAN: launch_g2p_adjoint_lds_t<BOXN, MAT_NEOHOOKEAN>(st, st_next, cot, part, N, envs, items, n_items, grid, gcot, pacc, k_call, grid_cap, s); break;
    case MAT_COROTATED: launch_g2p_adjoint_lds_t<BOXN, MAT_COROTATED>(st, st_next, cot, part, N, envs, items, n_items, grid, gcot, pacc, k_call, grid_cap, s); break;
    case MAT_VONMISES: launch_g2p_adjoint_lds_t<BOXN, MAT_VONMISES>(st, st_next, cot, part, N, envs, items, n_items, grid, gcot, pacc, k_call, grid_cap, s); break;
    case MAT_FLUID_TAIT: launch_g2p_adjoint_lds_t<BOXN, MAT_FLUID_TAIT>(st, st_next, cot, part, N, envs, items, n_items, grid, gcot, pacc, k_call, grid_cap, s); break;
    case MAT_FLUID_PAPER: launch_g2p_adjoint_lds_t<BOXN, MAT_FLUID_PAPER>(st, st_next, cot, part, N, envs, items, n_items, grid, gcot, pacc, k_call, grid_cap, s); break;
    case -1: launch_g2p_adjoint_lds_t<BOXN, -1>(st, st_next, cot, part, N, envs, items, n_items, grid, gcot, pacc, k_call, grid_cap, s); break;
    default: break;
  }
}
void launch_g2p_adjoint_lds(const float* st, const float* st_next, const float* cot, float* part, int64_t N, const EnvDev* envs,
                            const WorkItem* items, int n_items, const float* grid, float* gcot, double* pacc,
                            int k_call, int grid_cap, int box, int mat, hipStream_t s) {
  if (n_items == 0) return;
  if (box)
    launch_g2p_adjoint_lds_m<kBoxSmall>(st, st_next, cot, part, N, envs, items, n_items, grid, gcot, pacc, k_call, grid_cap, s, mat);
  else
    launch_g2p_adjoint_lds_m<kBoxNodes>(st, st_next, cot, part, N, envs, items, n_items, grid, gcot, pacc, k_call, grid_cap, s, mat);
}
// pull-scatter variants: the same launch shapes as the LDS-staged kernels
template <int BOXN, int MAT>
static void launch_p2g_pull_t(const float* st, int64_t N, const EnvDev* envs, const WorkItem* items, int n_items,
                              float* grid, uint32_t* flags, int32_t* errs, int k_call, int grid_cap, hipStream_t s) {
  if (grid_cap > 0 && grid_cap < n_items)
    hipLaunchKernelGGL((k_p2g_pull<true, BOXN, MAT>), dim3(grid_cap), dim3(256), 0, s, st, N, envs, items, grid, flags,
                       errs, k_call, n_items);
  else
    hipLaunchKernelGGL((k_p2g_pull<false, BOXN, MAT>), dim3(n_items), dim3(256), 0, s, st, N, envs, items, grid, flags,
                       errs, k_call, n_items);
}
template <int BOXN, int MAT>
static void launch_g2p_adjoint_pull_t(const float* st, const float* st_next, const float* cot, float* part, int64_t N,
                                      const EnvDev* envs, const WorkItem* items, int n_items, const float* grid,
                                      float* gcot, double* pacc, int k_call, int grid_cap, hipStream_t s) {
  if (grid_cap > 0 && grid_cap < n_items)
    hipLaunchKernelGGL((k_g2p_adjoint_pull<true, BOXN, MAT>), dim3(grid_cap), dim3(256), 0, s, st, st_next, cot, part,
                       N, envs, items, grid, gcot, pacc, k_call, n_items);
  else
    hipLaunchKernelGGL((k_g2p_adjoint_pull<false, BOXN, MAT>), dim3(n_items), dim3(256), 0, s, st, st_next, cot, part,
                       N, envs, items, grid, gcot, pacc, k_call, n_items);
}
template <int BOXN>
static void launch_p2g_pull_m(const float* st, int64_t N, const EnvDev* envs, const WorkItem* items, int n_items,
                              float* grid, uint32_t* flags, int32_t* errs, int k_call, int grid_cap, hipStream_t s,
                              int mat) {
  switch (mat) {
    case MAT_NEOHOOKEAN: launch_p2g_pull_t<BOXN, MAT_NEOHOOKEAN>(st, N, envs, items, n_items, grid, flags, errs, k_call, grid_cap, s); break;
    case MAT_COROTATED: launch_p2g_pull_t<BOXN, MAT_COROTATED>(st, N, envs, items, n_items, grid, flags, errs, k_call, grid_cap, s); break;
    case MAT_VONMISES: launch_p2g_pull_t<BOXN, MAT_VONMISES>(st, N, envs, items, n_items, grid, flags, errs, k_call, grid_cap, s); break;
    case MAT_FLUID_TAIT: launch_p2g_pull_t<BOXN, MAT_FLUID_TAIT>(st, N, envs, items, n_items, grid, flags, errs, k_call, grid_cap, s); break;
    case MAT_FLUID_PAPER: launch_p2g_pull_t<BOXN, MAT_FLUID_PAPER>(st, N, envs, items, n_items, grid, flags, errs, k_call, grid_cap, s); break;
    case -1: launch_p2g_pull_t<BOXN, -1>(st, N, envs, items, n_items, grid, flags, errs, k_call, grid_cap, s); break;
    default: break;
  }
}
template <int BOXN>
static void launch_g2p_adjoint_pull_m(const float* st, const float* st_next, const float* cot, float* part, int64_t N,
                                      const EnvDev* envs, const WorkItem* items, int n_items, const float* grid,
                                      float* gcot, double* pacc, int k_call, int grid_cap, hipStream_t s, int mat) {
  switch (mat) {
    case MAT_NEOHOOKEAN: launch_g2p_adjoint_pull_t<BOXN, MAT_NEOHOOKEAN>(st, st_next, cot, part, N, envs, items, n_items, grid, gcot, pacc, k_call, grid_cap, s); break;
    case MAT_COROTATED: launch_g2p_adjoint_pull_t<BOXN, MAT_COROTATED>(st, st_next, cot, part, N, envs, items, n_items, grid, gcot, pacc, k_call, grid_cap, s); break;
    case MAT_VONMISES: launch_g2p_adjoint_pull_t<BOXN, MAT_VONMISES>(st, st_next, cot, part, N, envs, items, n_items, grid, gcot, pacc, k_call, grid_cap, s); break;
    case MAT_FLUID_TAIT: launch_g2p_adjoint_pull_t<BOXN, MAT_FLUID_TAIT>(st, st_next, cot, part, N, envs, items, n_items, grid, gcot, pacc, k_call, grid_cap, s); break;
    case MAT_FLUID_PAPER: launch_g2p_adjoint_pull_t<BOXN, MAT_FLUID_PAPER>(st, st_next, cot, part, N, envs, items, n_items, grid, gcot, pacc, k_call, grid_cap, s); break;
    case -1: launch_g2p_adjoint_pull_t<BOXN, -1>(st, st_next, cot, part, N, envs, items, n_items, grid, gcot, pacc, k_call, grid_cap, s); break;
    default: break;
  }
}
void launch_p2g_pull(const float* st, int64_t N, const EnvDev* envs, const WorkItem* items, int n_items, float* grid,
                     uint32_t* flags, int32_t* errs, int k_call, int grid_cap, int box, int mat, hipStream_t s) {
  if (n_items == 0) return;
  if (box)
    launch_p2g_pull_m<kPullSmall>(st, N, envs, items, n_items, grid, flags, errs, k_call, grid_cap, s, mat);
  else
    launch_p2g_pull_m<kPullNodes>(st, N, envs, items, n_items, grid, flags, errs, k_call, grid_cap, s, mat);
}
void launch_g2p_adjoint_pull(const float* st, const float* st_next, const float* cot, float* part, int64_t N,
                             const EnvDev* envs, const WorkItem* items, int n_items, const float* grid, float* gcot,
                             double* pacc, int k_call, int grid_cap, int box, int mat, hipStream_t s) {
  if (n_items == 0) return;
  if (box)
    launch_g2p_adjoint_pull_m<kPullSmall>(st, st_next, cot, part, N, envs, items, n_items, grid, gcot, pacc, k_call, grid_cap, s, mat);
  else
    launch_g2p_adjoint_pull_m<kPullNodes>(st, st_next, cot, part, N, envs, items, n_items, grid, gcot, pacc, k_call, grid_cap, s, mat);
}
template <int BOXN, int MAT>
static void launch_p2g_adjoint_lds_t(const float* st, const float* part, float* cot_out, int64_t N, const EnvDev* envs,
                            const WorkItem* items, int n_items, const float* gcot, double* pacc, int k_call, const float* cot_in, int grid_cap, hipStream_t s) {
  if (grid_cap > 0 && grid_cap < n_items)
    hipLaunchKernelGGL((k_p2g_adjoint_lds<true, BOXN, MAT>), dim3(grid_cap), dim3(256), 0, s, st, part, cot_out, N, envs, items, gcot,
                     pacc, k_call, cot_in, n_items);
  else
    hipLaunchKernelGGL((k_p2g_adjoint_lds<false, BOXN, MAT>), dim3(n_items), dim3(256), 0, s, st, part, cot_out, N, envs, items, gcot,
                     pacc, k_call, cot_in, n_items);
}
template <int BOXN>
static void launch_p2g_adjoint_lds_m(const float* st, const float* part, float* cot_out, int64_t N, const EnvDev* envs,
                            const WorkItem* items, int n_items, const float* gcot, double* pacc, int k_call, const float* cot_in, int grid_cap, hipStream_t s, int mat) {
  switch (mat) {
    case MAT_NEOHOOKEAN: launch_p2g_adjoint_lds_t<BOXN, MAT_NEOHOOKEAN>(st, part, cot_out, N, envs, items, n_items, gcot, pacc, k_call, cot_in, grid_cap, s); break;
    case MAT_COROTATED: launch_p2g_adjoint_lds_t<BOXN, MAT_COROTATED>(st, part, cot_out, N, envs, items, n_items, gcot, pacc, k_call, cot_in, grid_cap, s); break;
    case MAT_VONMISES: launch_p2g_adjoint_lds_t<BOXN, MAT_VONMISES>(st, part, cot_out, N, envs, items, n_items, gcot, pacc, k_call, cot_in, grid_cap, s); break;
    case MAT_FLUID_TAIT: launch_p2g_adjoint_lds_t<BOXN, MAT_FLUID_TAIT>(st, part, cot_out, N, envs, items, n_items, gcot, pacc, k_call, cot_in, grid_cap, s); break;
    case MAT_FLUID_PAPER: launch_p2g_adjoint_lds_t<BOXN, MAT_FLUID_PAPER>(st, part, cot_out, N, envs, items, n_items, gcot, pacc, k_call, cot_in, grid_cap, s); break;
    case -1: launch_p2g_adjoint_lds_t<BOXN, -1>(st, part, cot_out, N, envs, items, n_items, gcot, pacc, k_call, cot_in, grid_cap, s); break;
    default: break;
  }
}
void launch_p2g_adjoint_lds(const float* st, const float* part, float* cot_out, int64_t N, const EnvDev* envs,
                            const WorkItem* items, int n_items, const float* gcot, double* pacc, int k_call, const float* cot_in, int grid_cap, int box, int mat, hipStream_t s) {
  if (n_items == 0) return;
  if (box)
    launch_p2g_adjoint_lds_m<kBoxSmall>(st, part, cot_out, N, envs, items, n_items, gcot, pacc, k_call, cot_in, grid_cap, s, mat);
  else
    launch_p2g_adjoint_lds_m<kBoxNodes>(st, part, cot_out, N, envs, items, n_items, gcot, pacc, k_call, cot_in, grid_cap, s, mat);
}

}  // namespace mpmx
