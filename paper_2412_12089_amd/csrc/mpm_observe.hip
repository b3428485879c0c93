// Per-env weighted moments of particle positions and velocities, and their
// VJP: the statistics the manipulation tasks observe and reward (centre of
// mass of a subsampled particle set, variance of its heights, mean velocity;
// paper Appendix E task definitions). They read caller-order AoS arrays
// (x, v [rows][3]), so they apply to any state the boundary hands out.
//
// Moments of env e, 19 values (stride kMoments = 20 in the output):
//   0 sum w | 1-3 sum w x | 4-9 sum w (xx, yy, zz, xy, xz, yz) |
//   10-12 sum w v | 13-18 sum w (vx vx, vy vy, vz vz, vx vy, vx vz, vy vz)
#include "mpm_kernels.h"

namespace mpmx {

constexpr int kMoments = 20;

MD void second_moments(const float a[3], float w, float* out) {
  out[0] = w * a[0] * a[0];
  out[1] = w * a[1] * a[1];
  out[2] = w * a[2] * a[2];
  out[3] = w * a[0] * a[1];
  out[4] = w * a[0] * a[2];
  out[5] = w * a[1] * a[2];
}

// rows of work item `it`: its env's local indices [start - p_off, + count), read as caller rows
MD int64_t item_row(const EnvDev& e, const WorkItem& it, int t) { return e.row_off + (it.start - e.p_off) + t; }

__global__ void __launch_bounds__(256) k_moments(const WorkItem* __restrict__ items, const EnvDev* __restrict__ envs,
                                                 const float* __restrict__ x, const float* __restrict__ v,
                                                 const float* __restrict__ w, double* __restrict__ out) {
  __shared__ double red[19][4];
  const WorkItem it = items[blockIdx.x];
  const EnvDev& e = envs[it.env];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  float m[19];
  for (int c = 0; c < 19; ++c) m[c] = 0.f;
  if (t < it.count) {
    const int64_t r = item_row(e, it, t);
    const float wt = w ? w[r] : 1.f;
    const float xp[3] = {x[3 * r], x[3 * r + 1], x[3 * r + 2]};
    const float vp[3] = {v[3 * r], v[3 * r + 1], v[3 * r + 2]};
    m[0] = wt;
    for (int a = 0; a < 3; ++a) { m[1 + a] = wt * xp[a]; m[10 + a] = wt * vp[a]; }
    second_moments(xp, wt, m + 4);
    second_moments(vp, wt, m + 13);
  }
  for (int c = 0; c < 19; ++c) {
    double s = (double)m[c];
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    if (lane == 0) red[c][wave] = s;
  }
  __syncthreads();
  if (t < 19) {
    const double s = red[t][0] + red[t][1] + red[t][2] + red[t][3];
    if (s != 0.0) atomicAdd(&out[(int64_t)it.env * kMoments + t], s);
  }
}

// d/dx_p of sum_c g_c m_c = w (g1 + M x_p) with M the symmetric matrix of the
// second-moment cotangents (diagonal doubled); the same for v
__global__ void __launch_bounds__(256) k_moments_vjp(const WorkItem* __restrict__ items, const EnvDev* __restrict__ envs,
                                                     const float* __restrict__ x, const float* __restrict__ v,
                                                     const float* __restrict__ w, const double* __restrict__ g,
                                                     float* __restrict__ gx, float* __restrict__ gv) {
  const WorkItem it = items[blockIdx.x];
  const int t = threadIdx.x;
  if (t >= it.count) return;
  const EnvDev& e = envs[it.env];
  const int64_t r = item_row(e, it, t);
  const double* ge = g + (int64_t)it.env * kMoments;
  const float wt = w ? w[r] : 1.f;
  for (int pass = 0; pass < 2; ++pass) {
    const float* a = pass == 0 ? x : v;
    float* ga = pass == 0 ? gx : gv;
    if (!ga) continue;
    const int o1 = pass == 0 ? 1 : 10, o2 = pass == 0 ? 4 : 13;
    const float p[3] = {a[3 * r], a[3 * r + 1], a[3 * r + 2]};
    const float M[3][3] = {{(float)(2.0 * ge[o2]), (float)ge[o2 + 3], (float)ge[o2 + 4]},
                           {(float)ge[o2 + 3], (float)(2.0 * ge[o2 + 1]), (float)ge[o2 + 5]},
                           {(float)ge[o2 + 4], (float)ge[o2 + 5], (float)(2.0 * ge[o2 + 2])}};
    for (int i = 0; i < 3; ++i)
      ga[3 * r + i] = wt * ((float)ge[o1 + i] + M[i][0] * p[0] + M[i][1] * p[1] + M[i][2] * p[2]);
  }
}

// ----------------------------------------------------------------------------
// The flip reward term of the HandFlip task (paper Appendix E): per env, the
// mean Euclidean distance between paired particles, R = (1/P) sum_k
// ||x_a - x_b||, and its VJP. A pair is (env, a, b) with env-local caller
// indices; pairs naming an env or a particle out of range are skipped.
// ----------------------------------------------------------------------------
MD bool pair_rows(const EnvDev* __restrict__ envs, int n_envs, const int32_t* __restrict__ pr, int64_t& ra,
                  int64_t& rb, int& env) {
  env = pr[0];
  if (env < 0 || env >= n_envs) return false;
  const EnvDev& e = envs[env];
  const int32_t a = pr[1], b = pr[2];
  if (a < 0 || b < 0 || a >= e.p_cnt || b >= e.p_cnt) return false;
  ra = e.row_off + a;
  rb = e.row_off + b;
  return true;
}

__global__ void __launch_bounds__(256) k_pair_distance(const EnvDev* __restrict__ envs, int n_envs,
                                                       const float* __restrict__ x, const int32_t* __restrict__ pairs,
                                                       int64_t n_pairs, double* __restrict__ out) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n_pairs) return;
  int64_t ra, rb;
  int env;
  if (!pair_rows(envs, n_envs, pairs + 3 * k, ra, rb, env)) return;
  const float d0 = x[3 * ra] - x[3 * rb], d1 = x[3 * ra + 1] - x[3 * rb + 1], d2 = x[3 * ra + 2] - x[3 * rb + 2];
  atomicAdd(&out[2 * env], (double)sqrtf(d0 * d0 + d1 * d1 + d2 * d2));
  atomicAdd(&out[2 * env + 1], 1.0);
}

__global__ void k_pair_mean(double* __restrict__ out, int n_envs) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n_envs && out[2 * e + 1] > 0.0) out[2 * e] /= out[2 * e + 1];
}

// d R_e / d x_a = (x_a - x_b) / (P_e ||x_a - x_b||), the opposite for x_b; 0 at
// zero distance (the norm's subgradient there is taken as 0)
__global__ void __launch_bounds__(256) k_pair_distance_vjp(const EnvDev* __restrict__ envs, int n_envs,
                                                           const float* __restrict__ x,
                                                           const int32_t* __restrict__ pairs, int64_t n_pairs,
                                                           const double* __restrict__ out,
                                                           const double* __restrict__ gout, float* __restrict__ gx) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n_pairs) return;
  int64_t ra, rb;
  int env;
  if (!pair_rows(envs, n_envs, pairs + 3 * k, ra, rb, env)) return;
  const double P = out[2 * env + 1];
  const float d[3] = {x[3 * ra] - x[3 * rb], x[3 * ra + 1] - x[3 * rb + 1], x[3 * ra + 2] - x[3 * rb + 2]};
  const float len = sqrtf(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
  if (!(len > 0.f) || !(P > 0.0)) return;
  const float s = (float)(gout[env] / P) / len;
  for (int a = 0; a < 3; ++a) {
    atomicAdd(&gx[3 * ra + a], s * d[a]);
    atomicAdd(&gx[3 * rb + a], -s * d[a]);
  }
}

void launch_moments(const WorkItem* items, int n_items, const EnvDev* envs, const float* x, const float* v,
                    const float* w, double* out, int n_envs, hipStream_t s) {
  launch_fill_u32(out, 0u, 2 * (int64_t)kMoments * n_envs, s);
  if (n_items == 0) return;
  hipLaunchKernelGGL(k_moments, dim3(n_items), dim3(256), 0, s, items, envs, x, v, w, out);
}

void launch_moments_vjp(const WorkItem* items, int n_items, const EnvDev* envs, const float* x, const float* v,
                        const float* w, const double* g, float* gx, float* gv, hipStream_t s) {
  if (n_items == 0) return;
  hipLaunchKernelGGL(k_moments_vjp, dim3(n_items), dim3(256), 0, s, items, envs, x, v, w, g, gx, gv);
}

void launch_pair_distance(const EnvDev* envs, int n_envs, const float* x, const int32_t* pairs, int64_t n_pairs,
                          double* out, hipStream_t s) {
  launch_fill_u32(out, 0u, 2 * 2 * (int64_t)n_envs, s);
  if (n_pairs > 0)
    hipLaunchKernelGGL(k_pair_distance, dim3((unsigned)((n_pairs + 255) / 256)), dim3(256), 0, s, envs, n_envs, x,
                       pairs, n_pairs, out);
  hipLaunchKernelGGL(k_pair_mean, dim3((n_envs + 63) / 64), dim3(64), 0, s, out, n_envs);
}

void launch_pair_distance_vjp(const EnvDev* envs, int n_envs, const float* x, const int32_t* pairs, int64_t n_pairs,
                              const double* out, const double* gout, float* gx, int64_t rows, hipStream_t s) {
  launch_fill_u32(gx, 0u, 3 * rows, s);
  if (n_pairs > 0)
    hipLaunchKernelGGL(k_pair_distance_vjp, dim3((unsigned)((n_pairs + 255) / 256)), dim3(256), 0, s, envs, n_envs,
                       x, pairs, n_pairs, out, gout, gx);
}

}  // namespace mpmx
