// LDS-staged particle kernels of the batched mode.
//
// A block takes one work item: up to 256 particles of one environment that
// are contiguous in (tile, cell) order, so their 3x3x3 stencils cover a small
// box of grid nodes. The block finds that box, and
//  * scatters (P2G, G2P adjoint) accumulate into the box in LDS with LDS
//    atomics, then flush each touched node once to HBM with global atomics;
//  * gathers (G2P, P2G adjoint) first copy the box's grid channels into LDS
//    with coalesced loads and then read the stencil from LDS.
// Thread t works on particle (t % 64) * 4 + t / 64 of the item: the 64 lanes
// of a wave hold particles four apart in cell order, so lanes that update the
// same node in the same instruction (same cell) are rare.
// If the box exceeds the LDS budget the block falls back to global memory.
#include "mpm_kernels.h"

namespace mpmx {

constexpr int kBoxNodes = 1024;   // LDS budget in nodes per block

struct Box {
  int lo[3], ext[3];
  int nodes;
  bool fits;
};

MD int lane_particle(int t) { return ((t & 63) << 2) | (t >> 6); }

// bounding box of the block's stencils: [min base, max base + 2] per axis
MD Box block_box(const int b[3], bool valid, int (*wb)[6]) {
  int mn[3], mx[3];
  for (int a = 0; a < 3; ++a) {
    mn[a] = valid ? b[a] : 0x3fffffff;
    mx[a] = valid ? b[a] : -0x3fffffff;
  }
  for (int off = 32; off > 0; off >>= 1)
    for (int a = 0; a < 3; ++a) {
      mn[a] = min(mn[a], __shfl_xor(mn[a], off, 64));
      mx[a] = max(mx[a], __shfl_xor(mx[a], off, 64));
    }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0)
    for (int a = 0; a < 3; ++a) { wb[wave][a] = mn[a]; wb[wave][3 + a] = mx[a]; }
  __syncthreads();
  Box bx;
  const int nw = blockDim.x >> 6;
  for (int a = 0; a < 3; ++a) {
    int lo = wb[0][a], hi = wb[0][3 + a];
    for (int w = 1; w < nw; ++w) { lo = min(lo, wb[w][a]); hi = max(hi, wb[w][3 + a]); }
    bx.lo[a] = lo;
    bx.ext[a] = hi - lo + 3;
  }
  const bool any = bx.ext[0] > 0;
  bx.nodes = any ? bx.ext[0] * bx.ext[1] * bx.ext[2] : 0;
  bx.fits = any && bx.ext[0] <= kBoxNodes && bx.ext[1] <= kBoxNodes && bx.ext[2] <= kBoxNodes &&
            bx.nodes <= kBoxNodes;
  return bx;
}

MD int box_index(const Box& bx, int i, int j, int k) {
  return ((i - bx.lo[0]) * bx.ext[1] + (j - bx.lo[1])) * bx.ext[2] + (k - bx.lo[2]);
}
MD void box_node(const Box& bx, int idx, int& i, int& j, int& k) {
  const int yz = bx.ext[1] * bx.ext[2];
  i = bx.lo[0] + idx / yz;
  j = bx.lo[1] + (idx / bx.ext[2]) % bx.ext[1];
  k = bx.lo[2] + idx % bx.ext[2];
}

// copies channels [c0, c0+nc) of the box's nodes from a grid buffer into LDS
MD void box_load(const EnvDev& e, const Box& bx, const float* __restrict__ g, int c0, int nc, float* lds) {
  for (int idx = threadIdx.x; idx < bx.nodes; idx += blockDim.x) {
    int i, j, k;
    box_node(bx, idx, i, j, k);
    const float* src = g + node_base(e, i, j, k) + c0 * CH;
    for (int c = 0; c < nc; ++c) lds[c * bx.nodes + idx] = src[c * CH];
  }
}

// adds the box's LDS channels to grid channels [c0, c0+nc); a node whose
// first channel is zero (no particle weight reached it) is skipped when
// skip_zero_first is set
MD void box_flush(const EnvDev& e, const Box& bx, float* __restrict__ g, int c0, int nc, const float* lds,
                  bool skip_zero_first) {
  for (int idx = threadIdx.x; idx < bx.nodes; idx += blockDim.x) {
    if (skip_zero_first && lds[idx] == 0.f) continue;
    int i, j, k;
    box_node(bx, idx, i, j, k);
    float* dst = g + node_base(e, i, j, k) + c0 * CH;
    for (int c = 0; c < nc; ++c) {
      const float v = lds[c * bx.nodes + idx];
      if (v != 0.f) atomicAdd(dst + c * CH, v);
    }
  }
}

MD void box_mark_tiles(const EnvDev& e, const Box& bx, uint32_t* __restrict__ flags) {
  int tlo[3], tn[3];
  for (int a = 0; a < 3; ++a) {
    tlo[a] = bx.lo[a] >> 2;
    tn[a] = ((bx.lo[a] + bx.ext[a] - 1) >> 2) - tlo[a] + 1;
  }
  const int cnt = tn[0] * tn[1] * tn[2];
  for (int idx = threadIdx.x; idx < cnt; idx += blockDim.x) {
    const int tx = tlo[0] + idx / (tn[1] * tn[2]);
    const int ty = tlo[1] + (idx / tn[2]) % tn[1];
    const int tz = tlo[2] + idx % tn[2];
    flags[e.tile_off + (tx * e.T + ty) * e.T + tz] = 1u;
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

MD void stencil_offsets(const Stencil& sc, const EnvDev& e, int ox, int oy, int oz, float& W, float d[3]) {
  W = sel3(sc.w[0], ox) * sc.w[1][oy] * sc.w[2][oz];
  d[0] = ((float)ox - sc.f[0]) * e.dx;
  d[1] = ((float)oy - sc.f[1]) * e.dx;
  d[2] = ((float)oz - sc.f[2]) * e.dx;
}

MD void block_reduce_params_lds(float pb[PB_COUNT], double* __restrict__ acc) {
  __shared__ double red[PB_COUNT][4];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < PB_COUNT; ++k) {
    double v = (double)pb[k];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    if (lane == 0) red[k][wave] = v;
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
// P2G
// ----------------------------------------------------------------------------
MD void p2g_lds_item(int item_idx, const float* __restrict__ st, int64_t N,
                                                 const EnvDev* __restrict__ envs, const WorkItem* __restrict__ items,
                                                 float* __restrict__ grid, uint32_t* __restrict__ flags,
                                                 int32_t* __restrict__ errs, int k_call) {
  __shared__ float lds[4 * kBoxNodes];
  __shared__ int wb[4][6];
  const WorkItem it = items[item_idx];
  const EnvDev& e = envs[it.env];
  if (k_call >= e.nsub) return;   // frozen env: nothing to scatter
  const int lp = lane_particle(threadIdx.x);
  const bool valid = lp < it.count;
  const int64_t p = it.start + (valid ? lp : 0);
  float x[3];
  load_x3(st, N, p, x);
  const Stencil sc = make_stencil(x, e.n, e.fn);
  if (valid && sc.oob) atomicOr(&errs[it.env], ERR_OUT_OF_DOMAIN);
  const Box bx = block_box(sc.b, valid, wb);
  if (bx.fits)
    for (int i = threadIdx.x; i < 4 * bx.nodes; i += blockDim.x) lds[i] = 0.f;
  __syncthreads();
  if (valid) {
    float v[3] = {st[3 * N + p], st[4 * N + p], st[5 * N + p]};
    const M3 Cm = ld_m3(st, N, p, 6);
    const M3 F = ld_m3(st, N, p, 15);
    const M3 tau = stress(e, F);
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
  box_flush(e, bx, grid, 0, 4, lds, true);
  box_mark_tiles(e, bx, flags);
}

// one block per work item, or a persistent grid that strides over the items
__global__ void __launch_bounds__(256) k_p2g_lds(const float* __restrict__ st, int64_t N,
                                                 const EnvDev* __restrict__ envs, const WorkItem* __restrict__ items,
                                                 float* __restrict__ grid, uint32_t* __restrict__ flags,
                                                 int32_t* __restrict__ errs, int k_call, int n_items) {
  for (int i = blockIdx.x; i < n_items; i += gridDim.x) {
    p2g_lds_item(i, st, N, envs, items, grid, flags, errs, k_call);
    __syncthreads();
  }
}

// ----------------------------------------------------------------------------
// G2P
// ----------------------------------------------------------------------------
MD void g2p_lds_item(int item_idx, const float* __restrict__ st, float* __restrict__ out, int64_t N,
                                                 const EnvDev* __restrict__ envs, const WorkItem* __restrict__ items,
                                                 const float* __restrict__ grid, int32_t* __restrict__ errs, int k_call) {
  __shared__ float lds[3 * kBoxNodes];
  __shared__ int wb[4][6];
  const WorkItem it = items[item_idx];
  const EnvDev& e = envs[it.env];
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
  const Box bx = block_box(sc.b, valid, wb);
  if (bx.fits) box_load(e, bx, grid, 4, 3, lds);
  __syncthreads();
  if (!valid) return;
  const M3 F = ld_m3(st, N, p, 15);
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
  const M3 Fn = project(e, m3_mul(m3_axpy(m3_eye(), e.dt, Cn), F));
  for (int a = 0; a < 3; ++a) { out[a * N + p] = xn[a]; out[(3 + a) * N + p] = vn[a]; }
  st_m3(out, N, p, 6, Cn);
  st_m3(out, N, p, 15, Fn);
  bool fin = true;
  for (int a = 0; a < 3; ++a) fin = fin && isfinite(xn[a]) && isfinite(vn[a]);
  for (int i = 0; i < 3; ++i) for (int j = 0; j < 3; ++j) fin = fin && isfinite(Fn.m[i][j]);
  if (!fin) atomicOr(&errs[it.env], ERR_NONFINITE);
}

// one block per work item, or a persistent grid that strides over the items
__global__ void __launch_bounds__(256) k_g2p_lds(const float* __restrict__ st, float* __restrict__ out, int64_t N,
                                                 const EnvDev* __restrict__ envs, const WorkItem* __restrict__ items,
                                                 const float* __restrict__ grid, int32_t* __restrict__ errs, int k_call, int n_items) {
  for (int i = blockIdx.x; i < n_items; i += gridDim.x) {
    g2p_lds_item(i, st, out, N, envs, items, grid, errs, k_call);
    __syncthreads();
  }
}

// ----------------------------------------------------------------------------
// G2P adjoint: gather v from an LDS copy, scatter vbar into LDS, flush
// ----------------------------------------------------------------------------
MD void g2p_adjoint_lds_item(int item_idx, const float* __restrict__ st, const float* __restrict__ cot,
                                                         float* __restrict__ part, int64_t N,
                                                         const EnvDev* __restrict__ envs,
                                                         const WorkItem* __restrict__ items,
                                                         const float* __restrict__ grid, float* __restrict__ gcot,
                                                         double* __restrict__ pacc, int k_call) {
  __shared__ float lv[3 * kBoxNodes];
  __shared__ float lg[3 * kBoxNodes];
  __shared__ int wb[4][6];
  const WorkItem it = items[item_idx];
  const EnvDev& e = envs[it.env];
  if (k_call >= e.nsub) return;   // frozen env: nothing to scatter
  const int lp = lane_particle(threadIdx.x);
  const bool valid = lp < it.count;
  const int64_t p = it.start + (valid ? lp : 0);
  float x[3];
  load_x3(st, N, p, x);
  const Stencil sc = make_stencil(x, e.n, e.fn);
  const Box bx = block_box(sc.b, valid, wb);
  if (bx.fits) {
    box_load(e, bx, grid, 4, 3, lv);
    for (int i = threadIdx.x; i < 3 * bx.nodes; i += blockDim.x) lg[i] = 0.f;
  }
  __syncthreads();
  float pb[PB_COUNT] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  if (valid) {
    const M3 F = ld_m3(st, N, p, 15);
    const float D4 = 4.f * e.fn * e.fn;
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
            for (int a = 0; a < 3; ++a) vi[a] = lv[a * bx.nodes + idx];
          } else {
            const float* g = grid + node_base(e, sc.b[0] + ox, sc.b[1] + oy, sc.b[2] + oz);
            for (int a = 0; a < 3; ++a) vi[a] = g[(4 + a) * CH];
          }
          for (int a = 0; a < 3; ++a) {
            const float wv = W * vi[a];
            Cn.m[a][0] = fmaf(wv, d[0], Cn.m[a][0]);
            Cn.m[a][1] = fmaf(wv, d[1], Cn.m[a][1]);
            Cn.m[a][2] = fmaf(wv, d[2], Cn.m[a][2]);
          }
        }
    Cn = m3_scale(Cn, D4);
    const M3 G = m3_axpy(m3_eye(), e.dt, Cn);
    const M3 Ftr = m3_mul(G, F);
    float xb[3], vb[3];
    for (int a = 0; a < 3; ++a) { xb[a] = cot[a * N + p]; vb[a] = cot[(3 + a) * N + p] + e.dt * xb[a]; }
    const M3 Cb_in = ld_m3(cot, N, p, 6);
    const M3 Fb_in = ld_m3(cot, N, p, 15);
    const M3 Ftrb = project_vjp(e, Ftr, Fb_in, pb);
    const M3 Cb = m3_axpy(Cb_in, e.dt, m3_mul_abt(Ftrb, F));
    const M3 Fb = m3_mul_atb(G, Ftrb);
#pragma unroll 1
    for (int ox = 0; ox < 3; ++ox)
#pragma unroll
      for (int oy = 0; oy < 3; ++oy)
#pragma unroll
        for (int oz = 0; oz < 3; ++oz) {
          const float wx = sel3(sc.w[0], ox), wy = sc.w[1][oy], wz = sc.w[2][oz];
          const float W = wx * wy * wz;
          const float gW[3] = {e.fn * sel3(sc.dw[0], ox) * wy * wz, e.fn * wx * sc.dw[1][oy] * wz, e.fn * wx * wy * sc.dw[2][oz]};
          const float d[3] = {((float)ox - sc.f[0]) * e.dx, ((float)oy - sc.f[1]) * e.dx, ((float)oz - sc.f[2]) * e.dx};
          float vi[3], gv[3];
          for (int a = 0; a < 3; ++a)
            gv[a] = vb[a] + D4 * (Cb.m[a][0] * d[0] + Cb.m[a][1] * d[1] + Cb.m[a][2] * d[2]);
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
            const float ctv = Cb.m[0][a] * vi[0] + Cb.m[1][a] * vi[1] + Cb.m[2][a] * vi[2];
            xb[a] += gW[a] * vg - D4 * W * ctv;
          }
        }
    for (int a = 0; a < 3; ++a) part[a * N + p] = xb[a];
    st_m3(part, N, p, 3, Fb);
  }
  if (bx.fits) {
    __syncthreads();
    box_flush(e, bx, gcot, 0, 3, lg, false);
  }
  block_reduce_params_lds(pb, pacc + (int64_t)it.env * 8);
}

// one block per work item, or a persistent grid that strides over the items
__global__ void __launch_bounds__(256) k_g2p_adjoint_lds(const float* __restrict__ st, const float* __restrict__ cot,
                                                         float* __restrict__ part, int64_t N,
                                                         const EnvDev* __restrict__ envs,
                                                         const WorkItem* __restrict__ items,
                                                         const float* __restrict__ grid, float* __restrict__ gcot,
                                                         double* __restrict__ pacc, int k_call, int n_items) {
  for (int i = blockIdx.x; i < n_items; i += gridDim.x) {
    g2p_adjoint_lds_item(i, st, cot, part, N, envs, items, grid, gcot, pacc, k_call);
    __syncthreads();
  }
}

// ----------------------------------------------------------------------------
// P2G adjoint: gather (mbar, Pbar) from an LDS copy
// ----------------------------------------------------------------------------
MD void p2g_adjoint_lds_item(int item_idx, const float* __restrict__ st,
                                                         const float* __restrict__ part,
                                                         float* __restrict__ cot_out, int64_t N,
                                                         const EnvDev* __restrict__ envs,
                                                         const WorkItem* __restrict__ items,
                                                         const float* __restrict__ gcot,
                                                         double* __restrict__ pacc, int k_call, const float* __restrict__ cot_in) {
  __shared__ float lds[4 * kBoxNodes];
  __shared__ int wb[4][6];
  const WorkItem it = items[item_idx];
  const EnvDev& e = envs[it.env];
  if (k_call >= e.nsub) {   // frozen env: the cotangent passes through
    if ((int)threadIdx.x < it.count) {
      const int64_t q = it.start + threadIdx.x;
      for (int c = 0; c < 24; ++c) cot_out[c * N + q] = cot_in[c * N + q];
    }
    return;
  }
  const int lp = lane_particle(threadIdx.x);
  const bool valid = lp < it.count;
  const int64_t p = it.start + (valid ? lp : 0);
  float x[3];
  load_x3(st, N, p, x);
  const Stencil sc = make_stencil(x, e.n, e.fn);
  const Box bx = block_box(sc.b, valid, wb);
  if (bx.fits) box_load(e, bx, gcot, 3, 4, lds);
  __syncthreads();
  float pb[PB_COUNT] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  if (valid) {
    float v[3] = {st[3 * N + p], st[4 * N + p], st[5 * N + p]};
    const M3 Cm = ld_m3(st, N, p, 6);
    const M3 F = ld_m3(st, N, p, 15);
    const M3 tau = stress(e, F);
    const float kf = -e.dt * e.vp * 4.f * e.fn * e.fn;
    const M3 A = m3_axpy(m3_scale(Cm, e.mp), kf, tau);
    float xb[3] = {part[p], part[N + p], part[2 * N + p]};
    float vb[3] = {0.f, 0.f, 0.f};
    M3 Ab = m3_zero();
    float mpb = 0.f;
#pragma unroll 1
    for (int ox = 0; ox < 3; ++ox)
#pragma unroll 1
      for (int oy = 0; oy < 3; ++oy)
#pragma unroll
        for (int oz = 0; oz < 3; ++oz) {
          const float wx = sel3(sc.w[0], ox), wy = sel3(sc.w[1], oy), wz = sc.w[2][oz];
          const float W = wx * wy * wz;
          const float gW[3] = {e.fn * sel3(sc.dw[0], ox) * wy * wz, e.fn * wx * sel3(sc.dw[1], oy) * wz, e.fn * wx * wy * sc.dw[2][oz]};
          const float d[3] = {((float)ox - sc.f[0]) * e.dx, ((float)oy - sc.f[1]) * e.dx, ((float)oz - sc.f[2]) * e.dx};
          float mb, Pb[3];
          if (bx.fits) {
            const int idx = box_index(bx, sc.b[0] + ox, sc.b[1] + oy, sc.b[2] + oz);
            mb = lds[idx];
            for (int a = 0; a < 3; ++a) Pb[a] = lds[(1 + a) * bx.nodes + idx];
          } else {
            const float* gc = gcot + node_base(e, sc.b[0] + ox, sc.b[1] + oy, sc.b[2] + oz);
            mb = gc[3 * CH];
            for (int a = 0; a < 3; ++a) Pb[a] = gc[(4 + a) * CH];
          }
          float mom[3], vcd[3];
          for (int a = 0; a < 3; ++a) {
            const float Ad = A.m[a][0] * d[0] + A.m[a][1] * d[1] + A.m[a][2] * d[2];
            mom[a] = e.mp * v[a] + Ad;
            vcd[a] = v[a] + Cm.m[a][0] * d[0] + Cm.m[a][1] * d[1] + Cm.m[a][2] * d[2];
          }
          const float gw = e.mp * mb + Pb[0] * mom[0] + Pb[1] * mom[1] + Pb[2] * mom[2];
          for (int a = 0; a < 3; ++a) {
            vb[a] = fmaf(e.mp * W, Pb[a], vb[a]);
            const float wp = W * Pb[a];
            Ab.m[a][0] = fmaf(wp, d[0], Ab.m[a][0]);
            Ab.m[a][1] = fmaf(wp, d[1], Ab.m[a][1]);
            Ab.m[a][2] = fmaf(wp, d[2], Ab.m[a][2]);
            const float atp = A.m[0][a] * Pb[0] + A.m[1][a] * Pb[1] + A.m[2][a] * Pb[2];
            xb[a] += gW[a] * gw - W * atp;
          }
          mpb += W * (mb + Pb[0] * vcd[0] + Pb[1] * vcd[1] + Pb[2] * vcd[2]);
        }
    const M3 Cb = m3_scale(Ab, e.mp);
    const M3 taub = m3_scale(Ab, kf);
    pb[PB_VP] += (-e.dt * 4.f * e.fn * e.fn) * m3_ddot(Ab, tau);
    pb[PB_MP] += mpb;
    M3 Fb = ld_m3(part, N, p, 3);
    stress_vjp(e, F, taub, Fb, pb);
    for (int a = 0; a < 3; ++a) { cot_out[a * N + p] = xb[a]; cot_out[(3 + a) * N + p] = vb[a]; }
    st_m3(cot_out, N, p, 6, Cb);
    st_m3(cot_out, N, p, 15, Fb);
  }
  block_reduce_params_lds(pb, pacc + (int64_t)it.env * 8);
}

// one block per work item, or a persistent grid that strides over the items
__global__ void __launch_bounds__(256) k_p2g_adjoint_lds(const float* __restrict__ st,
                                                         const float* __restrict__ part,
                                                         float* __restrict__ cot_out, int64_t N,
                                                         const EnvDev* __restrict__ envs,
                                                         const WorkItem* __restrict__ items,
                                                         const float* __restrict__ gcot,
                                                         double* __restrict__ pacc, int k_call, const float* __restrict__ cot_in, int n_items) {
  for (int i = blockIdx.x; i < n_items; i += gridDim.x) {
    p2g_adjoint_lds_item(i, st, part, cot_out, N, envs, items, gcot, pacc, k_call, cot_in);
    __syncthreads();
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
  float w[9][kItem];     // per-axis weights: x 0-2, y 3-5, z 6-8
  float q[3][kItem];     // value at the base node offset o = 0 (before the weight)
  float a[9][kItem];     // Abar, row-major: the value's change per unit node offset
  int key[kItem];        // packed base (10 bits per axis)
  int first[kItem + 1];  // first particle of each segment, then the count
  int wave_sum[4];
  int n_seg;
};

MD int pack_base(const int b[3]) { return (b[0] << 20) | (b[1] << 10) | b[2]; }

// marks segment starts among the item's particles (thread t <-> particle t)
// and fills first[] / n_seg; every thread must call it
MD void find_segments(SegShared& sh, int count) {
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const bool valid = t < count;
  const bool start = valid && (t == 0 || sh.key[t] != sh.key[t - 1]);
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
// (fits) or straight to grid channels c0.. with global atomics.
template <bool WITH_MASS>
MD void segment_scatter(const EnvDev& e, const Box& bx, const SegShared& sh, float mass, float* lds_box,
                        float* __restrict__ g, int c0) {
  constexpr int NCH = WITH_MASS ? 4 : 3;
  const int units = 9 * sh.n_seg;
  for (int u = threadIdx.x; u < units; u += blockDim.x) {
    const int seg = u / 9, r = u - 9 * seg;
    const int ox = r / 3, oy = r - 3 * ox;
    const int p0 = sh.first[seg], p1 = sh.first[seg + 1];
    float am[3] = {0.f, 0.f, 0.f};
    float ap[3][3] = {{0.f, 0.f, 0.f}, {0.f, 0.f, 0.f}, {0.f, 0.f, 0.f}};
    for (int p = p0; p < p1; ++p) {
      const float wxy = sh.w[ox][p] * sh.w[3 + oy][p];
      float rr[3], az[3];
      for (int a = 0; a < 3; ++a) {
        rr[a] = sh.q[a][p] + sh.a[3 * a][p] * (float)ox + sh.a[3 * a + 1][p] * (float)oy;
        az[a] = sh.a[3 * a + 2][p];
      }
#pragma unroll
      for (int oz = 0; oz < 3; ++oz) {
        const float W = wxy * sh.w[6 + oz][p];
        am[oz] += W;
        for (int a = 0; a < 3; ++a) ap[oz][a] = fmaf(W, rr[a] + az[a] * (float)oz, ap[oz][a]);
      }
    }
    const int key = sh.key[p0];
    const int bx0 = (key >> 20) + ox, by0 = ((key >> 10) & 1023) + oy, bz0 = key & 1023;
#pragma unroll
    for (int oz = 0; oz < 3; ++oz) {
      float v[4];
      int k = 0;
      if (WITH_MASS) v[k++] = am[oz] * mass;
      for (int a = 0; a < 3; ++a) v[k++] = ap[oz][a];
      if (bx.fits) {
        const int idx = box_index(bx, bx0, by0, bz0 + oz);
        for (int c = 0; c < NCH; ++c) atomicAdd(&lds_box[c * bx.nodes + idx], v[c]);
      } else {
        float* dst = g + node_base(e, bx0, by0, bz0 + oz) + c0 * CH;
        for (int c = 0; c < NCH; ++c) atomicAdd(dst + c * CH, v[c]);
      }
    }
  }
}

// P2G with segment reduction: thread t <-> particle t of the item
MD void p2g_seg_item(int item_idx, const float* __restrict__ st, int64_t N,
                                                 const EnvDev* __restrict__ envs, const WorkItem* __restrict__ items,
                                                 float* __restrict__ grid, uint32_t* __restrict__ flags,
                                                 int32_t* __restrict__ errs, int min_run, int k_call) {
  __shared__ float lds[4 * kBoxNodes];
  __shared__ int wb[4][6];
  __shared__ SegShared sh;
  const WorkItem it = items[item_idx];
  const EnvDev& e = envs[it.env];
  if (k_call >= e.nsub) return;   // frozen env: nothing to scatter
  const int t = threadIdx.x;
  const bool valid = t < it.count;
  const int64_t p = it.start + (valid ? t : 0);
  float x[3];
  load_x3(st, N, p, x);
  const Stencil sc = make_stencil(x, e.n, e.fn);
  if (valid && sc.oob) atomicOr(&errs[it.env], ERR_OUT_OF_DOMAIN);
  sh.key[t] = pack_base(sc.b);
  const Box bx = block_box(sc.b, valid, wb);   // synchronizes
  find_segments(sh, it.count);                 // synchronizes
  const bool seg_mode = it.count >= min_run * sh.n_seg;   // uniform across the block
  if (bx.fits)
    for (int i = t; i < 4 * bx.nodes; i += blockDim.x) lds[i] = 0.f;
  __syncthreads();   // the LDS box is clear before any lane adds to it
  if (valid) {
    float v[3] = {st[3 * N + p], st[4 * N + p], st[5 * N + p]};
    const M3 Cm = ld_m3(st, N, p, 6);
    const M3 F = ld_m3(st, N, p, 15);
    const M3 tau = stress(e, F);
    const float kf = -e.dt * e.vp * 4.f * e.fn * e.fn;
    const M3 A = m3_axpy(m3_scale(Cm, e.mp), kf, tau);
    if (seg_mode) {
      for (int a = 0; a < 3; ++a)
        for (int o = 0; o < 3; ++o) sh.w[3 * a + o][t] = sc.w[a][o];
      for (int a = 0; a < 3; ++a) {
        float q = e.mp * v[a];
        for (int b = 0; b < 3; ++b) {
          const float ab = A.m[a][b] * e.dx;
          sh.a[3 * a + b][t] = ab;
          q = fmaf(-ab, sc.f[b], q);
        }
        sh.q[a][t] = q;
      }
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
    segment_scatter<true>(e, bx, sh, e.mp, lds, grid, 0);
    __syncthreads();
  }
  if (bx.fits) {
    box_flush(e, bx, grid, 0, 4, lds, true);
    box_mark_tiles(e, bx, flags);
  } else if (valid) {
    mark_particle_tiles(e, sc.b, flags);
  }
}

// one block per work item, or a persistent grid that strides over the items
__global__ void __launch_bounds__(256) k_p2g_seg(const float* __restrict__ st, int64_t N,
                                                 const EnvDev* __restrict__ envs, const WorkItem* __restrict__ items,
                                                 float* __restrict__ grid, uint32_t* __restrict__ flags,
                                                 int32_t* __restrict__ errs, int min_run, int k_call, int n_items) {
  for (int i = blockIdx.x; i < n_items; i += gridDim.x) {
    p2g_seg_item(i, st, N, envs, items, grid, flags, errs, min_run, k_call);
    __syncthreads();
  }
}

void launch_p2g_seg(const float* st, int64_t N, const EnvDev* envs, const WorkItem* items, int n_items, float* grid,
                    uint32_t* flags, int32_t* errs, int min_run, int k_call, int grid_cap, hipStream_t s) {
  if (n_items == 0) return;
  hipLaunchKernelGGL(k_p2g_seg, dim3(grid_cap > 0 && grid_cap < n_items ? grid_cap : n_items), dim3(256), 0, s, st, N, envs, items, grid, flags, errs, min_run, k_call, n_items);
}

// G2P adjoint with segment-reduced scatter: thread t <-> particle t
MD void g2p_adjoint_seg_item(int item_idx, const float* __restrict__ st, const float* __restrict__ cot,
                                                         float* __restrict__ part, int64_t N,
                                                         const EnvDev* __restrict__ envs,
                                                         const WorkItem* __restrict__ items,
                                                         const float* __restrict__ grid, float* __restrict__ gcot,
                                                         double* __restrict__ pacc, int min_run, int k_call) {
  __shared__ float lv[3 * kBoxNodes];
  __shared__ float lg[3 * kBoxNodes];
  __shared__ int wb[4][6];
  __shared__ SegShared sh;
  const WorkItem it = items[item_idx];
  const EnvDev& e = envs[it.env];
  if (k_call >= e.nsub) return;   // frozen env: nothing to scatter
  const int t = threadIdx.x;
  const bool valid = t < it.count;
  const int64_t p = it.start + (valid ? t : 0);
  float x[3];
  load_x3(st, N, p, x);
  const Stencil sc = make_stencil(x, e.n, e.fn);
  sh.key[t] = pack_base(sc.b);
  const Box bx = block_box(sc.b, valid, wb);
  find_segments(sh, it.count);
  const bool seg_mode = it.count >= min_run * sh.n_seg;
  if (bx.fits) {
    box_load(e, bx, grid, 4, 3, lv);
    for (int i = t; i < 3 * bx.nodes; i += blockDim.x) lg[i] = 0.f;
  }
  __syncthreads();
  float pb[PB_COUNT] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  if (valid) {
    const M3 F = ld_m3(st, N, p, 15);
    const float D4 = 4.f * e.fn * e.fn;
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
            for (int a = 0; a < 3; ++a) vi[a] = lv[a * bx.nodes + idx];
          } else {
            const float* g = grid + node_base(e, sc.b[0] + ox, sc.b[1] + oy, sc.b[2] + oz);
            for (int a = 0; a < 3; ++a) vi[a] = g[(4 + a) * CH];
          }
          for (int a = 0; a < 3; ++a) {
            const float wv = W * vi[a];
            Cn.m[a][0] = fmaf(wv, d[0], Cn.m[a][0]);
            Cn.m[a][1] = fmaf(wv, d[1], Cn.m[a][1]);
            Cn.m[a][2] = fmaf(wv, d[2], Cn.m[a][2]);
          }
        }
    Cn = m3_scale(Cn, D4);
    const M3 G = m3_axpy(m3_eye(), e.dt, Cn);
    const M3 Ftr = m3_mul(G, F);
    float xb[3], vb[3];
    for (int a = 0; a < 3; ++a) { xb[a] = cot[a * N + p]; vb[a] = cot[(3 + a) * N + p] + e.dt * xb[a]; }
    const M3 Cb_in = ld_m3(cot, N, p, 6);
    const M3 Fb_in = ld_m3(cot, N, p, 15);
    const M3 Ftrb = project_vjp(e, Ftr, Fb_in, pb);
    const M3 Cb = m3_axpy(Cb_in, e.dt, m3_mul_abt(Ftrb, F));
    const M3 Fb = m3_mul_atb(G, Ftrb);
    if (seg_mode) {
      // gv(o) = vbar + D4 Cbar (o - f) dx = q + Abar o
      for (int a = 0; a < 3; ++a)
        for (int o = 0; o < 3; ++o) sh.w[3 * a + o][t] = sc.w[a][o];
      for (int a = 0; a < 3; ++a) {
        float q = vb[a];
        for (int b = 0; b < 3; ++b) {
          const float ab = D4 * e.dx * Cb.m[a][b];
          sh.a[3 * a + b][t] = ab;
          q = fmaf(-ab, sc.f[b], q);
        }
        sh.q[a][t] = q;
      }
    }
#pragma unroll 1
    for (int ox = 0; ox < 3; ++ox)
#pragma unroll
      for (int oy = 0; oy < 3; ++oy)
#pragma unroll
        for (int oz = 0; oz < 3; ++oz) {
          const float wx = sel3(sc.w[0], ox), wy = sc.w[1][oy], wz = sc.w[2][oz];
          const float W = wx * wy * wz;
          const float gW[3] = {e.fn * sel3(sc.dw[0], ox) * wy * wz, e.fn * wx * sc.dw[1][oy] * wz, e.fn * wx * wy * sc.dw[2][oz]};
          const float d[3] = {((float)ox - sc.f[0]) * e.dx, ((float)oy - sc.f[1]) * e.dx, ((float)oz - sc.f[2]) * e.dx};
          float vi[3], gv[3];
          for (int a = 0; a < 3; ++a)
            gv[a] = vb[a] + D4 * (Cb.m[a][0] * d[0] + Cb.m[a][1] * d[1] + Cb.m[a][2] * d[2]);
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
            const float ctv = Cb.m[0][a] * vi[0] + Cb.m[1][a] * vi[1] + Cb.m[2][a] * vi[2];
            xb[a] += gW[a] * vg - D4 * W * ctv;
          }
        }
    for (int a = 0; a < 3; ++a) part[a * N + p] = xb[a];
    st_m3(part, N, p, 3, Fb);
  }
  __syncthreads();
  if (seg_mode) {
    segment_scatter<false>(e, bx, sh, 0.f, lg, gcot, 0);
    __syncthreads();
  }
  if (bx.fits) box_flush(e, bx, gcot, 0, 3, lg, false);
  block_reduce_params_lds(pb, pacc + (int64_t)it.env * 8);
}

// one block per work item, or a persistent grid that strides over the items
__global__ void __launch_bounds__(256) k_g2p_adjoint_seg(const float* __restrict__ st, const float* __restrict__ cot,
                                                         float* __restrict__ part, int64_t N,
                                                         const EnvDev* __restrict__ envs,
                                                         const WorkItem* __restrict__ items,
                                                         const float* __restrict__ grid, float* __restrict__ gcot,
                                                         double* __restrict__ pacc, int min_run, int k_call, int n_items) {
  for (int i = blockIdx.x; i < n_items; i += gridDim.x) {
    g2p_adjoint_seg_item(i, st, cot, part, N, envs, items, grid, gcot, pacc, min_run, k_call);
    __syncthreads();
  }
}

void launch_g2p_adjoint_seg(const float* st, const float* cot, float* part, int64_t N, const EnvDev* envs,
                            const WorkItem* items, int n_items, const float* grid, float* gcot, double* pacc,
                            int min_run, int k_call, int grid_cap, hipStream_t s) {
  if (n_items == 0) return;
  hipLaunchKernelGGL(k_g2p_adjoint_seg, dim3(grid_cap > 0 && grid_cap < n_items ? grid_cap : n_items), dim3(256), 0, s, st, cot, part, N, envs, items, grid, gcot,
                     pacc, min_run, k_call, n_items);
}

void launch_p2g_lds(const float* st, int64_t N, const EnvDev* envs, const WorkItem* items, int n_items, float* grid,
                    uint32_t* flags, int32_t* errs, int k_call, int grid_cap, hipStream_t s) {
  if (n_items == 0) return;
  hipLaunchKernelGGL(k_p2g_lds, dim3(grid_cap > 0 && grid_cap < n_items ? grid_cap : n_items), dim3(256), 0, s, st, N, envs, items, grid, flags, errs, k_call, n_items);
}
void launch_g2p_lds(const float* st, float* out, int64_t N, const EnvDev* envs, const WorkItem* items, int n_items,
                    const float* grid, int32_t* errs, int k_call, int grid_cap, hipStream_t s) {
  if (n_items == 0) return;
  hipLaunchKernelGGL(k_g2p_lds, dim3(grid_cap > 0 && grid_cap < n_items ? grid_cap : n_items), dim3(256), 0, s, st, out, N, envs, items, grid, errs, k_call, n_items);
}
void launch_g2p_adjoint_lds(const float* st, const float* cot, float* part, int64_t N, const EnvDev* envs,
                            const WorkItem* items, int n_items, const float* grid, float* gcot, double* pacc,
                            int k_call, int grid_cap, hipStream_t s) {
  if (n_items == 0) return;
  hipLaunchKernelGGL(k_g2p_adjoint_lds, dim3(grid_cap > 0 && grid_cap < n_items ? grid_cap : n_items), dim3(256), 0, s, st, cot, part, N, envs, items, grid, gcot,
                     pacc, k_call, n_items);
}
void launch_p2g_adjoint_lds(const float* st, const float* part, float* cot_out, int64_t N, const EnvDev* envs,
                            const WorkItem* items, int n_items, const float* gcot, double* pacc, int k_call, const float* cot_in, int grid_cap, hipStream_t s) {
  if (n_items == 0) return;
  hipLaunchKernelGGL(k_p2g_adjoint_lds, dim3(grid_cap > 0 && grid_cap < n_items ? grid_cap : n_items), dim3(256), 0, s, st, part, cot_out, N, envs, items, gcot,
                     pacc, k_call, cot_in, n_items);
}

}  // namespace mpmx
