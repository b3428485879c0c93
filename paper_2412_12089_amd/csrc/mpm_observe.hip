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

}  // namespace mpmx
