// HIP kernels of the batched MLS-MPM substep (forward and adjoint) for gfx950.
//
// Particle kernels take a list of work items: (env, first particle, count),
// count <= 256, so a block never straddles two environments and its material
// branch is uniform. The per-environment ("plain") mode launches the items of
// one env at a time; the batched mode launches every item at once.
#include "mpm_kernels.h"

namespace mpmx {

// ----------------------------------------------------------------------------
// state access: SoA, component c of particle p at st[c * N + p]
// components: x 0-2, v 3-5, C 6-14 (row-major), H = F - I 15-23 (F at the
// boundary; the conversion happens in the AoS load/store kernels)
// ----------------------------------------------------------------------------
struct PState { float x[3], v[3]; M3 C, H; };

MD void load_x(const float* __restrict__ st, int64_t N, int64_t p, float x[3]) {
  x[0] = st[p]; x[1] = st[N + p]; x[2] = st[2 * N + p];
}
MD M3 load_m3(const float* __restrict__ st, int64_t N, int64_t p, int c0) {
  M3 m;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) m.m[i][j] = st[(c0 + 3 * i + j) * N + p];
  return m;
}
MD void store_m3(float* __restrict__ st, int64_t N, int64_t p, int c0, const M3& m) {
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) st[(c0 + 3 * i + j) * N + p] = m.m[i][j];
}
MD M3 load_cnext(const float* __restrict__ st, int64_t N, int64_t p) { return load_m3(st, N, p, 6); }
MD PState load_state(const float* __restrict__ st, int64_t N, int64_t p) {
  PState s;
  for (int a = 0; a < 3; ++a) { s.x[a] = st[a * N + p]; s.v[a] = st[(3 + a) * N + p]; }
  s.C = load_m3(st, N, p, 6);
  s.H = load_m3(st, N, p, 15);
  return s;
}
MD void store_state(float* __restrict__ st, int64_t N, int64_t p, const PState& s) {
  for (int a = 0; a < 3; ++a) { st[a * N + p] = s.x[a]; st[(3 + a) * N + p] = s.v[a]; }
  store_m3(st, N, p, 6, s.C);
  store_m3(st, N, p, 15, s.H);
}

// ----------------------------------------------------------------------------
// a1: parameter preparation
// ----------------------------------------------------------------------------
__global__ void k_prep_params(EnvDev* envs, int n_envs) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_envs) return;
  EnvDev& e = envs[i];
  const double mu = e.E / (2.0 * (1.0 + e.nu));
  const double lam = e.E * e.nu / ((1.0 + e.nu) * (1.0 - 2.0 * e.nu));
  e.mu = (float)mu;
  e.lam = (float)lam;
  e.alpha_nh = (float)(lam != 0.0 ? 1.0 + 3.0 * mu / (4.0 * lam) : 1.0);
  e.mp = (float)(e.rho * e.Vp);
  e.vp = (float)e.Vp;
  e.sy = (float)e.sigma_y;
  e.bulk = (float)e.K;
  e.gam = (float)e.gamma;
  e.yieldY = (float)(mu > 0.0 ? (double)kYieldScale * e.sigma_y / (2.0 * mu) : 0.0);
}

// accumulated (mu, lam, sigma_y, K, gamma, m_p, V_p) cotangents -> the 8-entry
// parameter row (E, nu, rho, Vp, sigma_y, K, gamma, 0)
__global__ void k_finalize_params(const EnvDev* envs, const double* acc, double* out, int n_envs) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_envs) return;
  const EnvDev& e = envs[i];
  const double* a = acc + i * 8;
  const double E = e.E, nu = e.nu;
  const double D = (1.0 + nu) * (1.0 - 2.0 * nu);
  const double dmu_dE = 1.0 / (2.0 * (1.0 + nu));
  const double dlam_dE = nu / D;
  const double dmu_dnu = -E / (2.0 * (1.0 + nu) * (1.0 + nu));
  const double dlam_dnu = E * (1.0 + 2.0 * nu * nu) / (D * D);
  double* o = out + i * 8;
  o[0] = a[PB_MU] * dmu_dE + a[PB_LAM] * dlam_dE;
  o[1] = a[PB_MU] * dmu_dnu + a[PB_LAM] * dlam_dnu;
  o[4] = a[PB_SY];
  o[5] = a[PB_K];
  // With one particle mass m_p = rho Vp per environment the substep depends on
  // the parameters only through tau / rho (Vp cancels between the mass and the
  // force, and every stress law is homogeneous of degree one in (E, sigma_y, K)
  // at fixed nu, gamma). Scaling (E, sigma_y, K, rho) together leaves the
  // trajectory unchanged, so rho dL/drho = -(E dL/dE + sigma_y dL/dsigma_y +
  // K dL/dK) and dL/dVp = 0 exactly. The rho cotangent is formed that way: its
  // mass-path and stress-path parts cancel to about 1e-3 of each, which the
  // FP32 per-particle sums (a[PB_MP], a[PB_VP]) cannot resolve.
  o[2] = e.rho > 0.0 ? -(E * o[0] + e.sigma_y * o[4] + e.K * o[5]) / e.rho : 0.0;
  o[3] = 0.0;
  o[6] = a[PB_GAMMA];
  o[7] = 0.0;
}

// ----------------------------------------------------------------------------
// layout conversion between the caller's AoS arrays and the internal SoA.
// States cross as F and are held as H = F - I; cotangents are the same for F
// and H and cross unchanged.
// Launched over work items; `all` selects rows in the concatenation of every
// env (row_off + local index) or the env's own rows (local index). ids[p]
// holds the env-local caller index of the particle at position p (-1: none).
// ----------------------------------------------------------------------------
__global__ void k_load_aos(const WorkItem* __restrict__ items, const EnvDev* __restrict__ envs, int all,
                           const float* __restrict__ x, const float* __restrict__ v, const float* __restrict__ C,
                           const float* __restrict__ F, float* __restrict__ st, int64_t N, int32_t* __restrict__ ids) {
  const WorkItem it = items[blockIdx.x];
  const int t = threadIdx.x;
  if (t >= it.cap) return;
  const EnvDev& e = envs[it.env];
  const int64_t p = it.start + t;
  const int64_t local = p - e.p_off;
  if (t >= it.count) { ids[p] = -1; return; }
  const int64_t i = (all ? e.row_off : 0) + local;
  for (int a = 0; a < 3; ++a) {
    st[a * N + p] = x[3 * i + a];
    st[(3 + a) * N + p] = v[3 * i + a];
  }
  for (int k = 0; k < 9; ++k) {
    st[(6 + k) * N + p] = C[9 * i + k];
    st[(15 + k) * N + p] = F[9 * i + k] - ((k & 3) == 0 ? 1.f : 0.f);   // exact for diagonals in [0.5, 2]
  }
  ids[p] = (int32_t)local;
}

__global__ void k_store_aos(const WorkItem* __restrict__ items, const EnvDev* __restrict__ envs, int all,
                            const float* __restrict__ st, int64_t N, const int32_t* __restrict__ ids,
                            float* __restrict__ x, float* __restrict__ v, float* __restrict__ C,
                            float* __restrict__ F, float f_shift) {
  const WorkItem it = items[blockIdx.x];
  const int t = threadIdx.x;
  if (t >= it.count) return;
  const EnvDev& e = envs[it.env];
  const int64_t p = it.start + t;
  const int64_t id = ids[p];
  if (id < 0) return;
  const int64_t r = (all ? e.row_off : 0) + id;
  for (int a = 0; a < 3; ++a) {
    if (x) x[3 * r + a] = st[a * N + p];
    if (v) v[3 * r + a] = st[(3 + a) * N + p];
  }
  for (int k = 0; k < 9; ++k) {
    if (C) C[9 * r + k] = st[(6 + k) * N + p];
    if (F) F[9 * r + k] = st[(15 + k) * N + p] + ((k & 3) == 0 ? f_shift : 0.f);
  }
}

// internal cot[p] = caller cotangent row (null arrays and empty positions count as zero)
__global__ void k_gather_aos(const WorkItem* __restrict__ items, const EnvDev* __restrict__ envs,
                             const float* __restrict__ x, const float* __restrict__ v, const float* __restrict__ C,
                             const float* __restrict__ F, const int32_t* __restrict__ ids, float* __restrict__ st,
                             int64_t N) {
  const WorkItem it = items[blockIdx.x];
  const int t = threadIdx.x;
  if (t >= it.cap) return;
  const EnvDev& e = envs[it.env];
  const int64_t p = it.start + t;
  const bool live = t < it.count && ids[p] >= 0;
  const int64_t u = live ? e.row_off + ids[p] : 0;
  for (int a = 0; a < 3; ++a) {
    st[a * N + p] = (live && x) ? x[3 * u + a] : 0.f;
    st[(3 + a) * N + p] = (live && v) ? v[3 * u + a] : 0.f;
  }
  for (int k = 0; k < 9; ++k) {
    st[(6 + k) * N + p] = (live && C) ? C[9 * u + k] : 0.f;
    st[(15 + k) * N + p] = (live && F) ? F[9 * u + k] : 0.f;
  }
}

__global__ void k_copy_i32(const int32_t* __restrict__ a, int32_t* __restrict__ b, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = a[i];
}

// one env's internal state rows [p0, p0 + cnt) (24 SoA components, then the
// caller ids) to or from a compact buffer [25][cnt]; to_buf = 1: state -> buf
__global__ void k_env_rows(float* __restrict__ st, int32_t* __restrict__ ids, int64_t N, int64_t p0, int64_t cnt,
                           float* __restrict__ buf, int to_buf) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= cnt) return;
  int32_t* bi = reinterpret_cast<int32_t*>(buf + 24 * cnt);
  if (to_buf) {
#pragma unroll
    for (int c = 0; c < 24; ++c) buf[c * cnt + i] = st[c * N + p0 + i];
    bi[i] = ids[p0 + i];
  } else {
#pragma unroll
    for (int c = 0; c < 24; ++c) st[c * N + p0 + i] = buf[c * cnt + i];
    ids[p0 + i] = bi[i];
  }
}

__global__ void k_fill_u32(uint32_t* __restrict__ p, uint32_t v, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = v;
}

// per-environment substep clocks (substeps since the env's particles were
// set); they place a prescribed collider motion in time
__global__ void k_set_clock(int32_t* clock, int env, int n_envs, int32_t value) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n_envs && (env < 0 || i == env)) clock[i] = value;
}

// a forward segment of Kj substeps starting at call substep k0: each env
// advances by the substeps it takes in it (frozen envs stop at nsub)
__global__ void k_advance_clocks(int32_t* clock, const EnvDev* envs, int n_envs, int k0, int Kj) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_envs) return;
  const int r = envs[i].nsub - k0;
  clock[i] += r < 0 ? 0 : (r < Kj ? r : Kj);
}

// clock[e] = base[e] + k: a backward segment starts k substeps after the recorded forward's start
__global__ void k_clocks_from(int32_t* clock, const int32_t* base, int n_envs, int k) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n_envs) clock[i] = base[i] + k;
}


// sum over i of (a_i - b_i)^2 and b_i^2 in FP64 (two accumulators), for the
// autotuner's parity check of a candidate against the reference kernels
__global__ void k_sq_diff(const float* __restrict__ a, const float* __restrict__ b, int64_t n, double* __restrict__ acc) {
  double d2 = 0.0, b2 = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const double d = (double)a[i] - (double)b[i];
    d2 += d * d;
    b2 += (double)b[i] * (double)b[i];
  }
  for (int off = 32; off > 0; off >>= 1) {
    d2 += __shfl_xor(d2, off, 64);
    b2 += __shfl_xor(b2, off, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    atomicAdd(&acc[0], d2);
    atomicAdd(&acc[1], b2);
  }
}

__global__ void k_copy_f32(const float* __restrict__ a, float* __restrict__ b, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) b[i] = a[i];
}

// ----------------------------------------------------------------------------
// a2: binning keys and a stable LSD radix sort (8-bit digits)
// ----------------------------------------------------------------------------

__global__ void __launch_bounds__(256) k_keys(const float* __restrict__ st, int64_t N, const EnvDev* __restrict__ envs,
                                              const WorkItem* __restrict__ items, uint32_t* __restrict__ keys,
                                              uint32_t* __restrict__ vals, int cell_bits) {
  const WorkItem it = items[blockIdx.x];
  if ((int)threadIdx.x >= it.cap) return;
  const EnvDev& e = envs[it.env];
  const int64_t p = it.start + threadIdx.x;
  uint32_t local = (1u << cell_bits) - 1u;   // empty positions sort last within their env
  if ((int)threadIdx.x < it.count) {
    int b[3];
    for (int a = 0; a < 3; ++a) {
      int q = base_floor(st[a * N + p], e.n);
      b[a] = q < 0 ? 0 : (q > e.n - 3 ? e.n - 3 : q);
    }
    const uint32_t tile = (uint32_t)(((b[0] >> 2) * e.T + (b[1] >> 2)) * e.T + (b[2] >> 2));
    const uint32_t cell = (uint32_t)((((b[0] & 3) << 4) | ((b[1] & 3) << 2) | (b[2] & 3)));
    local = tile * 64u + cell;
  }
  keys[p] = ((uint32_t)it.env << cell_bits) | local;
  vals[p] = (uint32_t)p;
}

__global__ void __launch_bounds__(RS_THREADS) k_radix_hist(const uint32_t* __restrict__ keys, int64_t N, int shift,
                                                           uint32_t* __restrict__ counts, int nblocks) {
  __shared__ uint32_t h[256];
  h[threadIdx.x] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * RS_TILE;
  for (int r = 0; r < RS_ITEMS; ++r) {
    const int64_t i = base + r * RS_THREADS + threadIdx.x;
    if (i < N) atomicAdd(&h[(keys[i] >> shift) & 255u], 1u);
  }
  __syncthreads();
  counts[(int64_t)threadIdx.x * nblocks + blockIdx.x] = h[threadIdx.x];
}

// per digit d (one block each): exclusive scan of counts[d][0..nblocks) in
// place, digit total into totals[d]
__global__ void __launch_bounds__(256) k_scan_digit(uint32_t* __restrict__ counts, uint32_t* __restrict__ totals,
                                                    int nblocks) {
  __shared__ uint32_t wsum[4];
  __shared__ uint32_t carry;
  uint32_t* row = counts + (int64_t)blockIdx.x * nblocks;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  if (t == 0) carry = 0;
  __syncthreads();
  for (int base = 0; base < nblocks; base += 256) {
    const int i = base + t;
    const uint32_t v = i < nblocks ? row[i] : 0u;
    uint32_t x = v;   // inclusive wave scan
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const uint32_t y = __shfl_up(x, off, 64);
      if (lane >= off) x += y;
    }
    if (lane == 63) wsum[wave] = x;
    __syncthreads();
    uint32_t pre = carry;
    for (int w = 0; w < wave; ++w) pre += wsum[w];
    if (i < nblocks) row[i] = pre + x - v;
    __syncthreads();
    if (t == 255) carry = pre + x;
    __syncthreads();
  }
  if (t == 0) totals[blockIdx.x] = carry;
}

// stable scatter of one 8-bit digit pass; positions = digit base + this
// block's offset within the digit + rank among equal digits (in index order)
__global__ void __launch_bounds__(RS_THREADS) k_radix_scatter(const uint32_t* __restrict__ kin,
                                                              const uint32_t* __restrict__ vin,
                                                              uint32_t* __restrict__ kout, uint32_t* __restrict__ vout,
                                                              int64_t N, int shift, const uint32_t* __restrict__ offs,
                                                              const uint32_t* __restrict__ totals, int nblocks) {
  __shared__ uint32_t run[256];
  __shared__ uint32_t wcnt[RS_THREADS / 64][256];
  __shared__ uint32_t dsum[RS_THREADS / 64];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  {
    const uint32_t v = totals[tid];
    uint32_t x = v;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const uint32_t y = __shfl_up(x, off, 64);
      if (lane >= off) x += y;
    }
    if (lane == 63) dsum[wave] = x;
    for (int w = 0; w < RS_THREADS / 64; ++w) wcnt[w][tid] = 0;
    __syncthreads();
    uint32_t pre = 0;
    for (int w = 0; w < wave; ++w) pre += dsum[w];
    run[tid] = pre + x - v + offs[(int64_t)tid * nblocks + blockIdx.x];
  }
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * RS_TILE;
  const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  for (int r = 0; r < RS_ITEMS; ++r) {
    const int64_t i = base + r * RS_THREADS + tid;
    const bool valid = i < N;
    const uint32_t key = valid ? kin[i] : 0u;
    const uint32_t val = valid ? vin[i] : 0u;
    const uint32_t digit = (key >> shift) & 255u;
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const int bit = (digit >> b) & 1u;
      const uint64_t bal = __ballot(bit);
      peers &= bit ? bal : ~bal;
    }
    const uint32_t rank = __popcll(peers & lt_mask);
    if (valid && rank == 0) wcnt[wave][digit] = __popcll(peers);
    __syncthreads();
    if (valid) {
      uint32_t pos = run[digit] + rank;
      for (int w = 0; w < wave; ++w) pos += wcnt[w][digit];
      kout[pos] = key;
      vout[pos] = val;
    }
    __syncthreads();
    uint32_t add = 0;
    for (int w = 0; w < RS_THREADS / 64; ++w) { add += wcnt[w][tid]; wcnt[w][tid] = 0; }
    run[tid] += add;
    __syncthreads();
  }
}

// dst[j] = src[perm[j]] for all 24 components; ids_out[j] = ids_in[perm[j]]
__global__ void k_permute_state(const float* __restrict__ src, float* __restrict__ dst, int64_t N,
                                const uint32_t* __restrict__ perm, const int32_t* __restrict__ ids_in,
                                int32_t* __restrict__ ids_out) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= N) return;
  const int64_t q = perm[j];
#pragma unroll
  for (int c = 0; c < 24; ++c) dst[c * N + j] = src[c * N + q];
  ids_out[j] = ids_in[q];
}

// adjoint of k_permute_state: dst[perm[j]] = src[j]
__global__ void k_unpermute(const float* __restrict__ src, float* __restrict__ dst, int64_t N,
                            const uint32_t* __restrict__ perm) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= N) return;
  const int64_t q = perm[j];
#pragma unroll
  for (int c = 0; c < 24; ++c) dst[c * N + q] = src[c * N + j];
}

// ----------------------------------------------------------------------------
// a3 + a4: P2G, one thread per particle, direct global atomics
// ----------------------------------------------------------------------------
MD void mark_tiles(const EnvDev& e, const int b[3], uint32_t* __restrict__ flags) {
  const int t0[3] = {b[0] >> 2, b[1] >> 2, b[2] >> 2};
  const int t1[3] = {(b[0] + 2) >> 2, (b[1] + 2) >> 2, (b[2] + 2) >> 2};
  for (int a = 0; a < 2; ++a)
    for (int c = 0; c < 2; ++c)
      for (int d = 0; d < 2; ++d) {
        const int tx = a ? t1[0] : t0[0], ty = c ? t1[1] : t0[1], tz = d ? t1[2] : t0[2];
        flags[e.tile_off + (tx * e.T + ty) * e.T + tz] = 1u;
      }
}

__global__ void __launch_bounds__(256) k_p2g_direct(const float* __restrict__ st, int64_t N,
                                                    const EnvDev* __restrict__ envs,
                                                    const WorkItem* __restrict__ items, float* __restrict__ grid,
                                                    uint32_t* __restrict__ flags, int32_t* __restrict__ errs, int k_call) {
  const WorkItem it = items[blockIdx.x];
  if ((int)threadIdx.x >= it.count) return;
  const EnvDev& e = envs[it.env];
  if (k_call >= e.nsub) return;   // frozen env: nothing to scatter
  const int64_t p = it.start + threadIdx.x;
  const PState s = load_state(st, N, p);
  const Stencil sc = make_stencil(s.x, e.n, e.fn);
  if (sc.oob) atomicOr(&errs[it.env], ERR_OUT_OF_DOMAIN);
  const M3 tau = stress(e, s.H, e.material);
  const float kf = -e.dt * e.vp * 4.f * e.fn * e.fn;
  const M3 A = m3_axpy(m3_scale(s.C, e.mp), kf, tau);
  mark_tiles(e, sc.b, flags);
#pragma unroll
  for (int ox = 0; ox < 3; ++ox)
#pragma unroll
    for (int oy = 0; oy < 3; ++oy)
#pragma unroll
      for (int oz = 0; oz < 3; ++oz) {
        const float W = sc.w[0][ox] * sc.w[1][oy] * sc.w[2][oz];
        const float d[3] = {((float)ox - sc.f[0]) * e.dx, ((float)oy - sc.f[1]) * e.dx, ((float)oz - sc.f[2]) * e.dx};
        float* g = grid + node_base(e, sc.b[0] + ox, sc.b[1] + oy, sc.b[2] + oz);
        atomicAdd(g, W * e.mp);
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          const float mv = e.mp * s.v[a] + A.m[a][0] * d[0] + A.m[a][1] * d[1] + A.m[a][2] * d[2];
          atomicAdd(g + (1 + a) * CH, W * mv);
        }
      }
}

// ----------------------------------------------------------------------------
// a5: grid update (and its adjoint) on touched 4^3 tiles, one wave per tile
// ----------------------------------------------------------------------------
MD void node_coords(const EnvDev& e, int64_t tile, int l, int& i, int& j, int& k) {
  const int lt = (int)(tile - e.tile_off);
  const int tx = lt / (e.T * e.T), ty = (lt / e.T) % e.T, tz = lt % e.T;
  i = 4 * tx + (l >> 4);
  j = 4 * ty + ((l >> 2) & 3);
  k = 4 * tz + (l & 3);
}

struct Contact {
  float n[3];     // outward unit normal (gradient of the distance), world frame
  float nb[3];    // the same in the box's frame
  float rb[3];    // node position relative to the center, box frame (R^T w)
  float w[3];     // node position relative to the center, world frame
  float s;        // blend weight min(exp(-alpha d), 1)
  float d;        // signed distance
  float L;        // length of the outside part of (|rel| - half), 0 inside
  int pos;        // bit a set when component a of (|rel| - half) is positive
};

// rotation by th about the box's unit axis a (Rodrigues): I + sin th K + (1 - cos th) K^2,
// K = [a]x; exactly I at th = 0
MD void box_rotation(const ColDev& e, float th, float R[3][3]) {
  float sn, cs;
  sincosf(th, &sn, &cs);
  const float oc = 1.f - cs;
  const float* a = e.c_axis;
  const float K[3][3] = {{0.f, -a[2], a[1]}, {a[2], 0.f, -a[0]}, {-a[1], a[0], 0.f}};
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) {
      const float kk = K[r][0] * K[0][c] + K[r][1] * K[1][c] + K[r][2] * K[2][c];
      R[r][c] = (r == c ? 1.f : 0.f) + sn * K[r][c] + oc * kk;
    }
}

MD void cross3(const float a[3], const float b[3], float out[3]) {
  out[0] = a[1] * b[2] - a[2] * b[1];
  out[1] = a[2] * b[0] - a[0] * b[2];
  out[2] = a[0] * b[1] - a[1] * b[0];
}

MD Contact contact_geometry(const ColDev& e, float dx, const float c[3], const float R[3][3], int i, int j, int k) {
  const float p[3] = {i * dx, j * dx, k * dx};
  float rel[3], q[3], qp[3];
  Contact ct;
  ct.pos = 0;
  for (int a = 0; a < 3; ++a) ct.w[a] = p[a] - c[a];
  if (e.has_collider == kColliderSphere) {
    // a ball of radius ch[0]: d = |w| - r, n = w / |w| (+z at the center). In the turned frame nb = r / |r| with
    // every axis "outside" and L = |r|, so the adjoint's terms for a normal that turns with r (the box's edges
    // and corners) give the ball's dn/dc = -(I - n n^T) / |w| and cancel its rigid turn with the angle.
    for (int a = 0; a < 3; ++a) ct.rb[a] = R[0][a] * ct.w[0] + R[1][a] * ct.w[1] + R[2][a] * ct.w[2];
    const float L = sqrtf(ct.w[0] * ct.w[0] + ct.w[1] * ct.w[1] + ct.w[2] * ct.w[2]);
    ct.d = L - e.ch[0];
    ct.L = L;
    if (L > 0.f) {
      const float il = 1.f / L;
      for (int a = 0; a < 3; ++a) {
        ct.nb[a] = ct.rb[a] * il;
        ct.n[a] = ct.w[a] * il;
      }
      ct.pos = 7;
    } else {   // the normal is taken fixed (+z) at the center: no derivative through it
      for (int a = 0; a < 3; ++a) {
        ct.n[a] = a == 2 ? 1.f : 0.f;
        ct.nb[a] = R[2][a];
      }
    }
    ct.s = fminf(expf(-e.c_alpha * ct.d), 1.f);
    return ct;
  }
  for (int a = 0; a < 3; ++a) {
    rel[a] = R[0][a] * ct.w[0] + R[1][a] * ct.w[1] + R[2][a] * ct.w[2];
    ct.rb[a] = rel[a];
    q[a] = fabsf(rel[a]) - e.ch[a];
    qp[a] = fmaxf(q[a], 0.f);
    if (q[a] > 0.f) ct.pos |= 1 << a;
  }
  const float out_len = sqrtf(qp[0] * qp[0] + qp[1] * qp[1] + qp[2] * qp[2]);
  const float inside = fmaxf(q[0], fmaxf(q[1], q[2]));
  ct.d = out_len + fminf(inside, 0.f) - e.c_round;   // a rounded box (a capsule with half (h, 0, 0)): same normal
  ct.L = out_len;
  if (out_len > 0.f) {
    for (int a = 0; a < 3; ++a) ct.nb[a] = (rel[a] >= 0.f ? 1.f : -1.f) * qp[a] / out_len;
  } else {
    const int ax = (q[0] >= q[1] && q[0] >= q[2]) ? 0 : (q[1] >= q[2] ? 1 : 2);
    for (int a = 0; a < 3; ++a) ct.nb[a] = (a == ax) ? (rel[a] >= 0.f ? 1.f : -1.f) : 0.f;
  }
  for (int a = 0; a < 3; ++a) ct.n[a] = R[a][0] * ct.nb[0] + R[a][1] * ct.nb[1] + R[a][2] * ct.nb[2];
  ct.s = fminf(expf(-e.c_alpha * ct.d), 1.f);
  return ct;
}

// the box's center and velocity during substep clock[0] + k_rel (clock: this
// env's substep clock): a row of the prescribed motion table, or the constant
// velocity from the center at t = 0
MD void box_motion(const ColDev& e, float dt, const float* __restrict__ motion, double t0, const int32_t* clock,
                   int k_rel, float c[3], float vb[3], float& th, float& om, int& row) {
  row = -1;
  if (e.motion_len > 0) {
    int k = clock[0] + k_rel;
    k = k < 0 ? 0 : (k >= e.motion_len ? e.motion_len - 1 : k);
    row = e.motion_off + k;
    const float* m = motion + kMotionRow * (int64_t)row;
    for (int a = 0; a < 3; ++a) { c[a] = m[a]; vb[a] = m[3 + a]; }
    th = m[6];
    om = m[7];
    return;
  }
  const float t = (float)(t0 + (double)(clock[0] + k_rel) * (double)dt);
  for (int a = 0; a < 3; ++a) { vb[a] = e.cv[a]; c[a] = fmaf(t, e.cv[a], e.cc[a]); }
  th = fmaf(t, e.c_omega, e.c_angle);
  om = e.c_omega;
}

// friction projection of the velocity relative to the box; returns the case (0 free, 1 stick, 2 slide)
MD int contact_project(const ColDev& e, const Contact& c, const float u[3], float up[3], float& un, float ut[3],
                       float& utn) {
  un = u[0] * c.n[0] + u[1] * c.n[1] + u[2] * c.n[2];
  for (int a = 0; a < 3; ++a) ut[a] = u[a] - un * c.n[a];
  utn = sqrtf(ut[0] * ut[0] + ut[1] * ut[1] + ut[2] * ut[2]);
  if (!(un < 0.f)) { for (int a = 0; a < 3; ++a) up[a] = u[a]; return 0; }
  if (utn <= -e.c_mu * un) { for (int a = 0; a < 3; ++a) up[a] = 0.f; return 1; }
  const float k = 1.f + e.c_mu * un / utn;
  for (int a = 0; a < 3; ++a) up[a] = ut[a] * k;
  return 2;
}

MD bool is_wall(const EnvDev& e, int i, int j, int k) {
  const int lo = e.wall, hi = e.n - 1 - e.wall;
  return i < lo || j < lo || k < lo || i > hi || j > hi || k > hi;
}


// one collider's contact blend of the velocity v of node (i, j, k), in place: the velocity relative to the
// collider's surface is projected (free, stick or slide) and blended with the free one by s(d)
MD void collider_blend(const EnvDev& e, const ColDev& cd, const float* __restrict__ motion, double t0,
                       const int32_t* clock, int k_rel, int i, int j, int k, float v[3]) {
  float bc[3], bv[3], th, om, R[3][3], spin[3];
  int row;
  box_motion(cd, e.dt, motion, t0, clock, k_rel, bc, bv, th, om, row);
  box_rotation(cd, th, R);
  const Contact c = contact_geometry(cd, e.dx, bc, R, i, j, k);
  cross3(cd.c_axis, c.w, spin);
  float vs[3], u[3], up[3], ut[3], un, utn;   // vs: the collider surface's velocity at the node
  for (int a = 0; a < 3; ++a) { vs[a] = fmaf(om, spin[a], bv[a]); u[a] = v[a] - vs[a]; }
  contact_project(cd, c, u, up, un, ut, utn);
  for (int a = 0; a < 3; ++a) v[a] = c.s * (vs[a] + up[a]) + (1.f - c.s) * v[a];
}

// one flagged tile (one wave, lane l = node) of the grid update. COLS bounds the colliders an env of the
// launch holds: 0 compiles them out, 1 takes slot 0 alone, kMaxColliders any number
template <int COLS>
MD void grid_update_tile(const EnvDev* __restrict__ envs, const int32_t* __restrict__ tile_env, int64_t tile, int l,
                         float* __restrict__ grid, uint32_t* __restrict__ flags, const int32_t* __restrict__ clock,
                         double t0, int k_rel, int clear, const float* __restrict__ motion) {
  const int ei = tile_env[tile];
  const EnvDev& e = envs[ei];
  int i, j, k;
  node_coords(e, tile, l, i, j, k);
  float* g = grid + tile * 512 + l;
  const float m = g[0];
  float v[3] = {0.f, 0.f, 0.f};
  if (m > 0.f) {
    const float inv = 1.f / m;
    v[0] = fmaf(g[CH], inv, e.dt * e.gx);
    v[1] = fmaf(g[2 * CH], inv, e.dt * e.gy);
    v[2] = fmaf(g[3 * CH], inv, e.dt * e.gz);
    const int nc = COLS == 0 ? 0 : COLS == 1 ? min(e.n_col, 1) : e.n_col;
#pragma unroll 1
    for (int ci = 0; ci < nc; ++ci)
      if (e.col[ci].has_collider) collider_blend(e, e.col[ci], motion, t0, clock + ei, k_rel, i, j, k, v);
  }
  if (is_wall(e, i, j, k)) v[0] = v[1] = v[2] = 0.f;
  g[4 * CH] = v[0];
  g[5 * CH] = v[1];
  g[6 * CH] = v[2];
  if (clear) {
    g[0] = 0.f; g[CH] = 0.f; g[2 * CH] = 0.f; g[3 * CH] = 0.f;
    if (l == 0) flags[tile] = 0u;
  }
}

template <int COLS>
__global__ void __launch_bounds__(256) k_grid_update(const EnvDev* __restrict__ envs,
                                                     const int32_t* __restrict__ tile_env, int64_t tile0,
                                                     int64_t ntiles, float* __restrict__ grid,
                                                     uint32_t* __restrict__ flags, const int32_t* __restrict__ clock,
                                                     double t0, int k_rel, int clear, const float* __restrict__ motion) {
  const int64_t tile = tile0 + (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (tile >= tile0 + ntiles) return;
  if (flags[tile] == 0u) return;
  grid_update_tile<COLS>(envs, tile_env, tile, threadIdx.x & 63, grid, flags, clock, t0, k_rel, clear, motion);
}

// the same, TILES (at most 64) tiles per block: one wave's ballot finds the flagged ones and the block's
// four waves take them in turn (far fewer blocks than one per 4 tiles when few tiles are flagged)
template <int TILES, int COLS>
__global__ void __launch_bounds__(256) k_grid_update_chunk(const EnvDev* __restrict__ envs,
                                                           const int32_t* __restrict__ tile_env, int64_t ntiles,
                                                           float* __restrict__ grid, uint32_t* __restrict__ flags,
                                                           const int32_t* __restrict__ clock, double t0, int k_rel,
                                                           int clear, const float* __restrict__ motion) {
  __shared__ uint64_t mask_s;
  const int wave = threadIdx.x >> 6;
  const int64_t base = (int64_t)blockIdx.x * TILES;
  if (wave == 0) {
    const int64_t tile = base + threadIdx.x;
    const uint64_t m = __ballot((int)threadIdx.x < TILES && tile < ntiles && flags[tile] != 0u);
    if (threadIdx.x == 0) mask_s = m;
  }
  __syncthreads();
  int rank = 0;
  for (uint64_t m = mask_s; m != 0ull; ++rank) {
    const int bit = __ffsll((unsigned long long)m) - 1;
    m &= m - 1ull;
    if ((rank & 3) == wave)
      grid_update_tile<COLS>(envs, tile_env, base + bit, threadIdx.x & 63, grid, flags, clock, t0, k_rel, clear,
                            motion);
  }
}

// reverse of collider_blend at node (i, j, k) with input velocity vpre: maps the cotangent vb of the blended
// velocity to that of vpre (in place), and puts the cotangents of the collider's motion row of this substep
// (center 0-2, velocity 3-5, angle 6, angular speed 7) in gmo and the row in row (-1: no prescribed motion)
MD void collider_blend_adjoint(const EnvDev& e, const ColDev& cd, const float* __restrict__ motion, double t0,
                               const int32_t* clock, int k_rel, int i, int j, int k, const float vpre[3], float vb[3],
                               float gmo[kMotionRow], int& row) {
  float bc[3], bv[3], th, om, R[3][3], spin[3];
  box_motion(cd, e.dt, motion, t0, clock, k_rel, bc, bv, th, om, row);
  box_rotation(cd, th, R);
  const Contact c = contact_geometry(cd, e.dx, bc, R, i, j, k);
  cross3(cd.c_axis, c.w, spin);
  float vs[3], u[3], up[3], ut[3], un, utn;
  for (int a = 0; a < 3; ++a) { vs[a] = fmaf(om, spin[a], bv[a]); u[a] = vpre[a] - vs[a]; }
  const int kase = contact_project(cd, c, u, up, un, ut, utn);
  float ub[3];
  float uh[3] = {0.f, 0.f, 0.f};
  if (kase == 0) {
    for (int a = 0; a < 3; ++a) ub[a] = vb[a];
  } else if (kase == 1) {
    ub[0] = ub[1] = ub[2] = 0.f;
  } else {
    for (int a = 0; a < 3; ++a) uh[a] = ut[a] / utn;
    const float nd = c.n[0] * vb[0] + c.n[1] * vb[1] + c.n[2] * vb[2];
    const float ud = uh[0] * vb[0] + uh[1] * vb[1] + uh[2] * vb[2];
    const float r = un / utn;
    for (int a = 0; a < 3; ++a) {
      const float pv = vb[a] - c.n[a] * nd;  // (I - n n^T) vbar
      ub[a] = pv + cd.c_mu * (c.n[a] * ud + r * (pv - uh[a] * ud));
    }
  }
  if (row >= 0) {
    // v' = s (v_s + u') + (1 - s) v with u = v - v_s and the surface velocity
    // v_s = v_b + omega a x w, w = x - c: v_b and omega enter through v_s; the
    // center through s(d), through n and through w; the angle through s(d)
    // and n, both functions of the box-frame position r = R^T w
    float sbar = 0.f, vsb[3];
    for (int a = 0; a < 3; ++a) {
      vsb[a] = c.s * (vb[a] - ub[a]);   // cotangent of v_s
      gmo[3 + a] = vsb[a];
      sbar += vb[a] * (vs[a] + up[a] - vpre[a]);
    }
    float axr[3], axv[3];
    cross3(cd.c_axis, c.rb, axr);        // d r / d angle = -a x r (a is fixed by the rotation)
    cross3(cd.c_axis, vsb, axv);
    gmo[7] = vsb[0] * spin[0] + vsb[1] * spin[1] + vsb[2] * spin[2];
    for (int a = 0; a < 3; ++a) gmo[a] += om * axv[a];
    if (c.d > 0.f) {   // s = exp(-alpha d) below its cap; d(d)/d(center) = -n, d(d)/d(angle) = -nb . (a x r)
      const float sa = sbar * cd.c_alpha * c.s;
      for (int a = 0; a < 3; ++a) gmo[a] += sa * c.n[a];
      gmo[6] += sa * (c.nb[0] * axr[0] + c.nb[1] * axr[1] + c.nb[2] * axr[2]);
    }
    if (kase == 2) {
      // sliding: u' depends on n = R nb(r). n turns rigidly with the angle
      // (d n = a x n d angle), and nb = sgn (|r| - h)^+ / L turns with r near
      // edges and corners: d nb / d r = (I_A - nb nb^T) / L
      float w[3], Pw[3];
      for (int a = 0; a < 3; ++a) w[a] = c.s * vb[a];
      const float wu = w[0] * uh[0] + w[1] * uh[1] + w[2] * uh[2];
      const float wn = w[0] * c.n[0] + w[1] * c.n[1] + w[2] * c.n[2];
      const float r = un / utn;
      for (int a = 0; a < 3; ++a) Pw[a] = w[a] - wu * uh[a];
      float nbar[3], axn[3];
      for (int a = 0; a < 3; ++a)
        nbar[a] = -(1.f + cd.c_mu * r) * wn * u[a] - un * (w[a] + cd.c_mu * r * Pw[a]) + cd.c_mu * wu * u[a];
      cross3(cd.c_axis, c.n, axn);
      gmo[6] += nbar[0] * axn[0] + nbar[1] * axn[1] + nbar[2] * axn[2];
      if (__popc(c.pos) >= 2) {
        float nbb[3], mm[3];
        for (int a = 0; a < 3; ++a) nbb[a] = R[0][a] * nbar[0] + R[1][a] * nbar[1] + R[2][a] * nbar[2];
        const float nn = c.nb[0] * nbb[0] + c.nb[1] * nbb[1] + c.nb[2] * nbb[2];
        for (int a = 0; a < 3; ++a) mm[a] = (c.pos & (1 << a)) ? (nbb[a] - c.nb[a] * nn) / c.L : 0.f;
        for (int a = 0; a < 3; ++a) gmo[a] -= R[a][0] * mm[0] + R[a][1] * mm[1] + R[a][2] * mm[2];
        gmo[6] -= mm[0] * axr[0] + mm[1] * axr[1] + mm[2] * axr[2];
      }
    }
  }
  for (int a = 0; a < 3; ++a) vb[a] = (1.f - c.s) * vb[a] + c.s * ub[a];
}

// reads vbar (channels 0-2 of gcot), writes mbar (3) and Pbar (4-6), clears
// vbar and the tape grid of this substep (and its flag)
// one flagged tile (one wave, lane l = node) of the grid adjoint (COLS as for the update)
template <int COLS>
MD void grid_adjoint_tile(const EnvDev* __restrict__ envs, const int32_t* __restrict__ tile_env, int64_t tile, int l,
                          float* __restrict__ grid, uint32_t* __restrict__ flags, float* __restrict__ gcot,
                          const int32_t* __restrict__ clock, double t0, int k_rel, const float* __restrict__ motion,
                          double* __restrict__ gmotion) {
  const int ei = tile_env[tile];
  const EnvDev& e = envs[ei];
  int i, j, k;
  node_coords(e, tile, l, i, j, k);
  float* g = grid + tile * 512 + l;
  float* gc = gcot + tile * 512 + l;
  const float m = g[0];
  const float P[3] = {g[CH], g[2 * CH], g[3 * CH]};
  float vb[3] = {gc[0], gc[CH], gc[2 * CH]};   // cotangent of the node velocity
  float mb = 0.f, Pb[3] = {0.f, 0.f, 0.f};
  const bool act = !is_wall(e, i, j, k) && m > 0.f;
  const float inv = act ? 1.f / m : 0.f;
  const float vpre[3] = {fmaf(P[0], inv, e.dt * e.gx), fmaf(P[1], inv, e.dt * e.gy), fmaf(P[2], inv, e.dt * e.gz)};
  // the colliders in reverse order (the loop is uniform over the wave, one tile of one env); each one's input
  // velocity comes from the forward chain of the ones before it, recomputed
  const int nc = COLS == 0 ? 0 : COLS == 1 ? min(e.n_col, 1) : e.n_col;
#pragma unroll 1
  for (int ci = nc - 1; ci >= 0; --ci) {
    const ColDev& cd = e.col[ci];
    if (!cd.has_collider) continue;
    // cotangents of the collider's center (0-2), velocity (3-5), angle (6) and angular speed (7) at this node
    float gmo[kMotionRow] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    int row = -1;
    if (act) {
      float vin[3] = {vpre[0], vpre[1], vpre[2]};
      if (COLS > 1) {
#pragma unroll 1
        for (int cj = 0; cj < ci; ++cj)
          if (e.col[cj].has_collider) collider_blend(e, e.col[cj], motion, t0, clock + ei, k_rel, i, j, k, vin);
      }
      collider_blend_adjoint(e, cd, motion, t0, clock + ei, k_rel, i, j, k, vin, vb, gmo, row);
    }
    // sum the wave's (one tile of one env) cotangents and add them to the collider's row of this substep in FP64
    if (cd.motion_len > 0) {
      bool nz = false;
      for (int c = 0; c < kMotionRow; ++c) nz |= gmo[c] != 0.f;
      const bool any = __ballot(row >= 0 && nz) != 0ull;
      if (any) {
        int rw = row;
        for (int off = 32; off > 0; off >>= 1) rw = max(rw, __shfl_xor(rw, off, 64));
        for (int c = 0; c < kMotionRow; ++c) {
          double x = (double)gmo[c];
          for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
          if (l == 0 && x != 0.0) atomicAdd(&gmotion[kMotionRow * (int64_t)rw + c], x);
        }
      }
    }
  }
  if (act) {
    for (int a = 0; a < 3; ++a) Pb[a] = vb[a] * inv;
    mb = -(vb[0] * P[0] + vb[1] * P[1] + vb[2] * P[2]) * inv * inv;
  }
  gc[3 * CH] = mb;
  gc[4 * CH] = Pb[0];
  gc[5 * CH] = Pb[1];
  gc[6 * CH] = Pb[2];
  gc[0] = 0.f; gc[CH] = 0.f; gc[2 * CH] = 0.f;
#pragma unroll
  for (int c = 0; c < 7; ++c) g[c * CH] = 0.f;
  if (l == 0) flags[tile] = 0u;
}

template <int COLS>
__global__ void __launch_bounds__(256) k_grid_adjoint(const EnvDev* __restrict__ envs,
                                                      const int32_t* __restrict__ tile_env, int64_t tile0,
                                                      int64_t ntiles, float* __restrict__ grid,
                                                      uint32_t* __restrict__ flags, float* __restrict__ gcot,
                                                      const int32_t* __restrict__ clock, double t0, int k_rel,
                                                      const float* __restrict__ motion, double* __restrict__ gmotion) {
  const int64_t tile = tile0 + (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (tile >= tile0 + ntiles) return;
  if (flags[tile] == 0u) return;
  grid_adjoint_tile<COLS>(envs, tile_env, tile, threadIdx.x & 63, grid, flags, gcot, clock, t0, k_rel, motion,
                         gmotion);
}

template <int TILES, int COLS>
__global__ void __launch_bounds__(256) k_grid_adjoint_chunk(const EnvDev* __restrict__ envs,
                                                            const int32_t* __restrict__ tile_env, int64_t ntiles,
                                                            float* __restrict__ grid, uint32_t* __restrict__ flags,
                                                            float* __restrict__ gcot, const int32_t* __restrict__ clock,
                                                            double t0, int k_rel, const float* __restrict__ motion,
                                                            double* __restrict__ gmotion) {
  __shared__ uint64_t mask_s;
  const int wave = threadIdx.x >> 6;
  const int64_t base = (int64_t)blockIdx.x * TILES;
  if (wave == 0) {
    const int64_t tile = base + threadIdx.x;
    const uint64_t m = __ballot((int)threadIdx.x < TILES && tile < ntiles && flags[tile] != 0u);
    if (threadIdx.x == 0) mask_s = m;
  }
  __syncthreads();
  int rank = 0;
  for (uint64_t m = mask_s; m != 0ull; ++rank) {
    const int bit = __ffsll((unsigned long long)m) - 1;
    m &= m - 1ull;
    if ((rank & 3) == wave)
      grid_adjoint_tile<COLS>(envs, tile_env, base + bit, threadIdx.x & 63, grid, flags, gcot, clock, t0, k_rel,
                             motion, gmotion);
  }
}

// clears every flagged tile of a grid buffer and its flag (for an abandoned tape)
__global__ void __launch_bounds__(256) k_grid_clear_flagged(int64_t ntiles, float* __restrict__ grid,
                                                            uint32_t* __restrict__ flags) {
  const int64_t tile = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int l = threadIdx.x & 63;
  if (tile >= ntiles) return;
  if (flags[tile] == 0u) return;
  float* g = grid + tile * 512 + l;
#pragma unroll
  for (int c = 0; c < 8; ++c) g[c * CH] = 0.f;
  if (l == 0) flags[tile] = 0u;
}

// ----------------------------------------------------------------------------
// a6: G2P gather, F update and return mapping, one thread per particle
// ----------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_g2p_direct(const float* __restrict__ st, float* __restrict__ out, int64_t N,
                                                    const EnvDev* __restrict__ envs,
                                                    const WorkItem* __restrict__ items,
                                                    const float* __restrict__ grid, int32_t* __restrict__ errs, int k_call) {
  const WorkItem it = items[blockIdx.x];
  if ((int)threadIdx.x >= it.count) return;
  const EnvDev& e = envs[it.env];
  if (k_call >= e.nsub) {   // frozen env: the substep is the identity
    if ((int)threadIdx.x < it.count) {
      const int64_t q = it.start + threadIdx.x;
      for (int c = 0; c < 24; ++c) out[c * N + q] = st[c * N + q];
    }
    return;
  }
  const int64_t p = it.start + threadIdx.x;
  float x[3];
  load_x(st, N, p, x);
  const M3 H = load_m3(st, N, p, 15);
  const Stencil sc = make_stencil(x, e.n, e.fn);
  float vn[3] = {0.f, 0.f, 0.f};
  M3 Cn = m3_zero();
  const StencilAddr sa = stencil_addr(e, sc.b);
  const float* genv = grid + (int64_t)e.tile_off * 512;
  float wdz[3];
  for (int o = 0; o < 3; ++o) wdz[o] = sc.w[2][o] * ((float)o - sc.f[2]) * e.dx;
#pragma unroll
  for (int ox = 0; ox < 3; ++ox)
#pragma unroll
    for (int oy = 0; oy < 3; ++oy) {
      // a z-column shares d_x and d_y: sum W v_i and W v_i d_z over it, then
      // add the column into v and C
      const float wxy = sc.w[0][ox] * sc.w[1][oy];
      const float d0 = ((float)ox - sc.f[0]) * e.dx, d1 = ((float)oy - sc.f[1]) * e.dx;
      float col[3] = {0.f, 0.f, 0.f}, colz[3] = {0.f, 0.f, 0.f};
#pragma unroll
      for (int oz = 0; oz < 3; ++oz) {
        const float* g = genv + (sa.x[ox] + sa.y[oy] + sa.z[oz]);
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
  Cn = m3_scale(Cn, 4.f * e.fn * e.fn);
  PState s;
  for (int a = 0; a < 3; ++a) { s.x[a] = fmaf(e.dt, vn[a], x[a]); s.v[a] = vn[a]; }
  s.C = Cn;
  s.H = project(e, trial_h(e, Cn, H), e.material);
  store_state(out, N, p, s);
  bool fin = true;
  for (int a = 0; a < 3; ++a) fin = fin && isfinite(s.x[a]) && isfinite(s.v[a]);
  for (int i = 0; i < 3; ++i) for (int j = 0; j < 3; ++j) fin = fin && isfinite(s.H.m[i][j]);
  if (!fin) atomicOr(&errs[it.env], ERR_NONFINITE);
}

// ----------------------------------------------------------------------------
// a7: adjoint kernels
// ----------------------------------------------------------------------------
// block sum of PB_COUNT floats in FP64, one atomic per slot per block
MD void block_reduce_params(float pb[PB_COUNT], double* __restrict__ acc) {
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
    const int nw = (blockDim.x + 63) >> 6;
    double s = 0.0;
    for (int w = 0; w < nw; ++w) s += red[threadIdx.x][w];
    if (s != 0.0) atomicAdd(&acc[threadIdx.x], s);
  }
}

// G2P adjoint: scatters grid-velocity cotangents (channels 0-2 of gcot) and
// writes the particle's direct x and F cotangents into `part` (12 comps)
__global__ void __launch_bounds__(256) k_g2p_adjoint_direct(const float* __restrict__ st,
                                                            const float* __restrict__ st_next, const float* __restrict__ cot,
                                                            float* __restrict__ part, int64_t N,
                                                            const EnvDev* __restrict__ envs,
                                                            const WorkItem* __restrict__ items,
                                                            const float* __restrict__ grid, float* __restrict__ gcot,
                                                            double* __restrict__ pacc, int k_call) {
  const WorkItem it = items[blockIdx.x];
  const bool valid = (int)threadIdx.x < it.count;
  const EnvDev& e = envs[it.env];
  if (k_call >= e.nsub) return;   // frozen env: nothing to scatter
  float pb[PB_COUNT] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  if (valid) {
    const int64_t p = it.start + threadIdx.x;
    float x[3];
    load_x(st, N, p, x);
    const M3 H = load_m3(st, N, p, 15);
    const M3 F = f_of(H);
    const Stencil sc = make_stencil(x, e.n, e.fn);
    const float D4 = 4.f * e.fn * e.fn;
    // C' of the substep's output state, read from the tape (the forward's own value)
    const M3 Cn = load_cnext(st_next, N, p);
    const M3 G = m3_axpy(m3_eye(), e.dt, Cn);
    const M3 Htr = trial_h(e, Cn, H);
    // incoming cotangents of (x', v', C', F')
    float xb[3], vb[3];
    for (int a = 0; a < 3; ++a) { xb[a] = cot[a * N + p]; vb[a] = cot[(3 + a) * N + p] + e.dt * xb[a]; }
    const M3 Cb_in = load_m3(cot, N, p, 6);
    const M3 Fb_in = load_m3(cot, N, p, 15);
    const M3 Ftrb = project_vjp(e, Htr, Fb_in, pb, e.material);
    const M3 Cb = m3_axpy(Cb_in, e.dt, m3_mul_abt(Ftrb, F));  // C' enters F_tr = (I + dt C') F
    const M3 Fb = m3_mul_atb(G, Ftrb);
    // pass 2: scatter to grid, accumulate dx
    for (int ox = 0; ox < 3; ++ox)
      for (int oy = 0; oy < 3; ++oy)
#pragma unroll
        for (int oz = 0; oz < 3; ++oz) {
          const float wx = sc.w[0][ox], wy = sc.w[1][oy], wz = sc.w[2][oz];
          const float W = wx * wy * wz;
          const float gW[3] = {e.fn * sc.dw[0][ox] * wy * wz, e.fn * wx * sc.dw[1][oy] * wz, e.fn * wx * wy * sc.dw[2][oz]};
          const float d[3] = {((float)ox - sc.f[0]) * e.dx, ((float)oy - sc.f[1]) * e.dx, ((float)oz - sc.f[2]) * e.dx};
          const int64_t nb = node_base(e, sc.b[0] + ox, sc.b[1] + oy, sc.b[2] + oz);
          const float* g = grid + nb;
          const float vi[3] = {g[4 * CH], g[5 * CH], g[6 * CH]};
          float gv[3];
          for (int a = 0; a < 3; ++a)
            gv[a] = vb[a] + D4 * (Cb.m[a][0] * d[0] + Cb.m[a][1] * d[1] + Cb.m[a][2] * d[2]);
          float* gc = gcot + nb;
          atomicAdd(gc, W * gv[0]);
          atomicAdd(gc + CH, W * gv[1]);
          atomicAdd(gc + 2 * CH, W * gv[2]);
          const float vg = vi[0] * gv[0] + vi[1] * gv[1] + vi[2] * gv[2];
          for (int a = 0; a < 3; ++a) {
            const float ctv = Cb.m[0][a] * vi[0] + Cb.m[1][a] * vi[1] + Cb.m[2][a] * vi[2];
            xb[a] += gW[a] * vg - D4 * W * ctv;
          }
        }
    for (int a = 0; a < 3; ++a) part[a * N + p] = xb[a];
    store_m3(part, N, p, 3, Fb);
  }
  block_reduce_params(pb, pacc + (int64_t)it.env * 8);
}

// P2G adjoint: gathers (mbar, Pbar), adds the G2P part, writes the full
// cotangent of the substep's input state
__global__ void __launch_bounds__(256) k_p2g_adjoint_direct(const float* __restrict__ st,
                                                            const float* __restrict__ part,
                                                            float* __restrict__ cot_out, int64_t N,
                                                            const EnvDev* __restrict__ envs,
                                                            const WorkItem* __restrict__ items,
                                                            const float* __restrict__ gcot,
                                                            double* __restrict__ pacc, int k_call, const float* __restrict__ cot_in) {
  const WorkItem it = items[blockIdx.x];
  const bool valid = (int)threadIdx.x < it.count;
  const EnvDev& e = envs[it.env];
  if (k_call >= e.nsub) {   // frozen env: the cotangent passes through
    if ((int)threadIdx.x < it.count) {
      const int64_t q = it.start + threadIdx.x;
      for (int c = 0; c < 24; ++c) cot_out[c * N + q] = cot_in[c * N + q];
    }
    return;
  }
  float pb[PB_COUNT] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  if (valid) {
    const int64_t p = it.start + threadIdx.x;
    const PState s = load_state(st, N, p);
    const Stencil sc = make_stencil(s.x, e.n, e.fn);
    const StressPrep spr = stress_prep(e, s.H, e.material);
    const M3 tau = stress_from(e, spr, e.material);
    const float kf = -e.dt * e.vp * 4.f * e.fn * e.fn;
    const M3 A = m3_axpy(m3_scale(s.C, e.mp), kf, tau);
    float xb[3] = {part[p], part[N + p], part[2 * N + p]};
    float vb[3] = {0.f, 0.f, 0.f};
    M3 Ab = m3_zero();
    float mpb = 0.f;
    for (int ox = 0; ox < 3; ++ox)
      for (int oy = 0; oy < 3; ++oy)
#pragma unroll
        for (int oz = 0; oz < 3; ++oz) {
          const float wx = sc.w[0][ox], wy = sc.w[1][oy], wz = sc.w[2][oz];
          const float W = wx * wy * wz;
          const float gW[3] = {e.fn * sc.dw[0][ox] * wy * wz, e.fn * wx * sc.dw[1][oy] * wz, e.fn * wx * wy * sc.dw[2][oz]};
          const float d[3] = {((float)ox - sc.f[0]) * e.dx, ((float)oy - sc.f[1]) * e.dx, ((float)oz - sc.f[2]) * e.dx};
          const float* gc = gcot + node_base(e, sc.b[0] + ox, sc.b[1] + oy, sc.b[2] + oz);
          const float mb = gc[3 * CH];
          const float Pb[3] = {gc[4 * CH], gc[5 * CH], gc[6 * CH]};
          float mom[3], vcd[3];
          for (int a = 0; a < 3; ++a) {
            const float Ad = A.m[a][0] * d[0] + A.m[a][1] * d[1] + A.m[a][2] * d[2];
            mom[a] = e.mp * s.v[a] + Ad;
            vcd[a] = s.v[a] + s.C.m[a][0] * d[0] + s.C.m[a][1] * d[1] + s.C.m[a][2] * d[2];
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
    M3 Fb = load_m3(part, N, p, 3);
    stress_vjp_from(e, s.H, spr, taub, Fb, pb, e.material);
    for (int a = 0; a < 3; ++a) { cot_out[a * N + p] = xb[a]; cot_out[(3 + a) * N + p] = vb[a]; }
    store_m3(cot_out, N, p, 6, Cb);
    store_m3(cot_out, N, p, 15, Fb);
  }
  block_reduce_params(pb, pacc + (int64_t)it.env * 8);
}

// ----------------------------------------------------------------------------
// host launchers
// ----------------------------------------------------------------------------
static inline unsigned nblk(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

void launch_prep_params(EnvDev* envs, int n_envs, hipStream_t s) {
  hipLaunchKernelGGL(k_prep_params, dim3(nblk(n_envs, 64)), dim3(64), 0, s, envs, n_envs);
}
void launch_finalize_params(const EnvDev* envs, const double* acc, double* out, int n_envs, hipStream_t s) {
  hipLaunchKernelGGL(k_finalize_params, dim3(nblk(n_envs, 64)), dim3(64), 0, s, envs, acc, out, n_envs);
}
void launch_load_aos(const WorkItem* items, int n_items, const EnvDev* envs, int all, const float* x, const float* v,
                     const float* C, const float* F, float* st, int64_t N, int32_t* ids, hipStream_t s) {
  if (n_items == 0) return;
  hipLaunchKernelGGL(k_load_aos, dim3(n_items), dim3(kItemSize), 0, s, items, envs, all, x, v, C, F, st, N, ids);
}
void launch_store_aos(const WorkItem* items, int n_items, const EnvDev* envs, int all, const float* st, int64_t N,
                      const int32_t* ids, float* x, float* v, float* C, float* F, bool state, hipStream_t s) {
  if (n_items == 0) return;
  hipLaunchKernelGGL(k_store_aos, dim3(n_items), dim3(kItemSize), 0, s, items, envs, all, st, N, ids, x, v, C, F,
                     state ? 1.f : 0.f);
}
void launch_gather_aos(const WorkItem* items, int n_items, const EnvDev* envs, const float* x, const float* v,
                       const float* C, const float* F, const int32_t* ids, float* st, int64_t N, hipStream_t s) {
  if (n_items == 0) return;
  hipLaunchKernelGGL(k_gather_aos, dim3(n_items), dim3(kItemSize), 0, s, items, envs, x, v, C, F, ids, st, N);
}
void launch_copy_i32(const int32_t* a, int32_t* b, int64_t n, hipStream_t s) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_copy_i32, dim3(nblk(n, 256)), dim3(256), 0, s, a, b, n);
}
void launch_env_rows(float* st, int32_t* ids, int64_t N, int64_t p0, int64_t cnt, float* buf, int to_buf,
                     hipStream_t s) {
  if (cnt == 0) return;
  hipLaunchKernelGGL(k_env_rows, dim3(nblk(cnt, 256)), dim3(256), 0, s, st, ids, N, p0, cnt, buf, to_buf);
}
void launch_fill_u32(void* p, uint32_t v, int64_t n_words, hipStream_t s) {
  if (n_words == 0) return;
  int64_t b = nblk(n_words, 256);
  if (b > 65536) b = 65536;
  hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)b), dim3(256), 0, s, (uint32_t*)p, v, n_words);
}
void launch_sq_diff(const float* a, const float* b, int64_t n, double* acc, hipStream_t s) {
  if (n == 0) return;
  int64_t blocks = nblk(n, 256);
  if (blocks > 2048) blocks = 2048;
  hipLaunchKernelGGL(k_sq_diff, dim3((unsigned)blocks), dim3(256), 0, s, a, b, n, acc);
}
void launch_copy_f32(const float* a, float* b, int64_t n, hipStream_t s) {
  if (n == 0) return;
  int64_t blocks = nblk(n, 256);
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(k_copy_f32, dim3((unsigned)blocks), dim3(256), 0, s, a, b, n);
}
void launch_set_clock(int32_t* clock, int env, int n_envs, int32_t value, hipStream_t s) {
  hipLaunchKernelGGL(k_set_clock, dim3((n_envs + 255) / 256), dim3(256), 0, s, clock, env, n_envs, value);
}
void launch_advance_clocks(int32_t* clock, const EnvDev* envs, int n_envs, int k0, int Kj, hipStream_t s) {
  hipLaunchKernelGGL(k_advance_clocks, dim3((n_envs + 255) / 256), dim3(256), 0, s, clock, envs, n_envs, k0, Kj);
}
void launch_clocks_from(int32_t* clock, const int32_t* base, int n_envs, int k, hipStream_t s) {
  hipLaunchKernelGGL(k_clocks_from, dim3((n_envs + 255) / 256), dim3(256), 0, s, clock, base, n_envs, k);
}
void launch_keys(const float* st, int64_t N, const EnvDev* envs, const WorkItem* items, int n_items, uint32_t* keys,
                 uint32_t* vals, int cell_bits, hipStream_t s) {
  if (n_items == 0) return;
  hipLaunchKernelGGL(k_keys, dim3(n_items), dim3(256), 0, s, st, N, envs, items, keys, vals, cell_bits);
}
// returns which buffer (0: k0/v0, 1: k1/v1) holds the sorted result
int launch_radix_sort(uint32_t* k0, uint32_t* v0, uint32_t* k1, uint32_t* v1, uint32_t* counts, int64_t N,
                      int key_bits, hipStream_t s) {
  if (N == 0) return 0;
  const int nblocks = (int)nblk(N, RS_TILE);
  int cur = 0;
  for (int shift = 0; shift < key_bits; shift += 8) {
    uint32_t* kin = cur ? k1 : k0;
    uint32_t* vin = cur ? v1 : v0;
    uint32_t* kout = cur ? k0 : k1;
    uint32_t* vout = cur ? v0 : v1;
    uint32_t* totals = counts + (int64_t)256 * nblocks;
    hipLaunchKernelGGL(k_radix_hist, dim3(nblocks), dim3(RS_THREADS), 0, s, kin, N, shift, counts, nblocks);
    hipLaunchKernelGGL(k_scan_digit, dim3(256), dim3(256), 0, s, counts, totals, nblocks);
    hipLaunchKernelGGL(k_radix_scatter, dim3(nblocks), dim3(RS_THREADS), 0, s, kin, vin, kout, vout, N, shift, counts,
                       totals, nblocks);
    cur ^= 1;
  }
  return cur;
}
void launch_permute_state(const float* src, float* dst, int64_t N, const uint32_t* perm, const int32_t* ids_in,
                          int32_t* ids_out, hipStream_t s) {
  if (N == 0) return;
  hipLaunchKernelGGL(k_permute_state, dim3(nblk(N, 256)), dim3(256), 0, s, src, dst, N, perm, ids_in, ids_out);
}
void launch_unpermute(const float* src, float* dst, int64_t N, const uint32_t* perm, hipStream_t s) {
  if (N == 0) return;
  hipLaunchKernelGGL(k_unpermute, dim3(nblk(N, 256)), dim3(256), 0, s, src, dst, N, perm);
}
void launch_p2g_direct(const float* st, int64_t N, const EnvDev* envs, const WorkItem* items, int n_items, float* grid,
                       uint32_t* flags, int32_t* errs, int k_call, hipStream_t s) {
  if (n_items == 0) return;
  hipLaunchKernelGGL(k_p2g_direct, dim3(n_items), dim3(256), 0, s, st, N, envs, items, grid, flags, errs, k_call);
}
#define MPMX_BY_COLS(cols, LAUNCH) \
  do {                                \
    if ((cols) == 0) LAUNCH(0);       \
    else if ((cols) == 1) LAUNCH(1);  \
    else LAUNCH(kMaxColliders);       \
  } while (0)
void launch_grid_update(const EnvDev* envs, const int32_t* tile_env, int64_t tile0, int64_t ntiles, float* grid,
                        uint32_t* flags, const int32_t* clock, double t0, int k_rel, int clear, const float* motion,
                        hipStream_t s, int cols) {
  if (ntiles == 0) return;
  const dim3 g(nblk(ntiles, 4));
#define MPMX_L(C) hipLaunchKernelGGL(k_grid_update<C>, g, dim3(256), 0, s, envs, tile_env, tile0, ntiles, grid, flags, \
                                     clock, t0, k_rel, clear, motion)
  MPMX_BY_COLS(cols, MPMX_L);
#undef MPMX_L
}
void launch_grid_adjoint(const EnvDev* envs, const int32_t* tile_env, int64_t tile0, int64_t ntiles, float* grid,
                         uint32_t* flags, float* gcot, const int32_t* clock, double t0, int k_rel, const float* motion,
                         double* gmotion, hipStream_t s, int cols) {
  if (ntiles == 0) return;
  const dim3 g(nblk(ntiles, 4));
#define MPMX_L(C) hipLaunchKernelGGL(k_grid_adjoint<C>, g, dim3(256), 0, s, envs, tile_env, tile0, ntiles, grid, flags, \
                                     gcot, clock, t0, k_rel, motion, gmotion)
  MPMX_BY_COLS(cols, MPMX_L);
#undef MPMX_L
}
void launch_grid_update_chunked(const EnvDev* envs, const int32_t* tile_env, int64_t ntiles, float* grid,
                                uint32_t* flags, const int32_t* clock, double t0, int k_rel, int clear,
                                const float* motion, int tiles, hipStream_t s, int cols) {
  if (ntiles == 0) return;
  const dim3 g((unsigned)((ntiles + tiles - 1) / tiles));
#define MPMX_L16(C) hipLaunchKernelGGL((k_grid_update_chunk<16, C>), g, dim3(256), 0, s, envs, tile_env, ntiles, grid, \
                                       flags, clock, t0, k_rel, clear, motion)
#define MPMX_L64(C) hipLaunchKernelGGL((k_grid_update_chunk<64, C>), g, dim3(256), 0, s, envs, tile_env, ntiles, grid, \
                                       flags, clock, t0, k_rel, clear, motion)
  if (tiles == 16) MPMX_BY_COLS(cols, MPMX_L16);
  else MPMX_BY_COLS(cols, MPMX_L64);
#undef MPMX_L16
#undef MPMX_L64
}
void launch_grid_adjoint_chunked(const EnvDev* envs, const int32_t* tile_env, int64_t ntiles, float* grid,
                                 uint32_t* flags, float* gcot, const int32_t* clock, double t0, int k_rel,
                                 const float* motion, double* gmotion, int tiles, hipStream_t s, int cols) {
  if (ntiles == 0) return;
  const dim3 g((unsigned)((ntiles + tiles - 1) / tiles));
#define MPMX_L16(C) hipLaunchKernelGGL((k_grid_adjoint_chunk<16, C>), g, dim3(256), 0, s, envs, tile_env, ntiles, grid, \
                                       flags, gcot, clock, t0, k_rel, motion, gmotion)
#define MPMX_L64(C) hipLaunchKernelGGL((k_grid_adjoint_chunk<64, C>), g, dim3(256), 0, s, envs, tile_env, ntiles, grid, \
                                       flags, gcot, clock, t0, k_rel, motion, gmotion)
  if (tiles == 16) MPMX_BY_COLS(cols, MPMX_L16);
  else MPMX_BY_COLS(cols, MPMX_L64);
#undef MPMX_L16
#undef MPMX_L64
}
#undef MPMX_BY_COLS
void launch_grid_clear_flagged(int64_t ntiles, float* grid, uint32_t* flags, hipStream_t s) {
  if (ntiles == 0) return;
  hipLaunchKernelGGL(k_grid_clear_flagged, dim3(nblk(ntiles, 4)), dim3(256), 0, s, ntiles, grid, flags);
}
void launch_g2p_direct(const float* st, float* out, int64_t N, const EnvDev* envs, const WorkItem* items, int n_items,
                       const float* grid, int32_t* errs, int k_call, hipStream_t s) {
  if (n_items == 0) return;
  hipLaunchKernelGGL(k_g2p_direct, dim3(n_items), dim3(256), 0, s, st, out, N, envs, items, grid, errs, k_call);
}
void launch_g2p_adjoint_direct(const float* st, const float* st_next, const float* cot, float* part, int64_t N, const EnvDev* envs,
                               const WorkItem* items, int n_items, const float* grid, float* gcot, double* pacc,
                               int k_call, hipStream_t s) {
  if (n_items == 0) return;
  hipLaunchKernelGGL(k_g2p_adjoint_direct, dim3(n_items), dim3(256), 0, s, st, st_next, cot, part, N, envs, items, grid, gcot,
                     pacc, k_call);
}
void launch_p2g_adjoint_direct(const float* st, const float* part, float* cot_out, int64_t N, const EnvDev* envs,
                               const WorkItem* items, int n_items, const float* gcot, double* pacc, int k_call, const float* cot_in, hipStream_t s) {
  if (n_items == 0) return;
  hipLaunchKernelGGL(k_p2g_adjoint_direct, dim3(n_items), dim3(256), 0, s, st, part, cot_out, N, envs, items, gcot,
                     pacc, k_call, cot_in);
}

}  // namespace mpmx
