// Tetrahedral FEM with activations (Appendix D.2): rest data, the batched
// forward substeps and their reverse-mode adjoint.
//
// One block per environment. The env's nodes (positions, velocities, lumped
// volumes) and the node -> element incidences sit in LDS for the whole launch;
// a thread keeps its elements' indices, B_m and W in registers, so a substep
// touches HBM only for the activations and the tape. Each substep is an
// element pass (stress and the element's node forces, written to LDS) and a
// node pass that gathers them through the incidences -- no atomics, so the
// result does not depend on the schedule.
#include <hip/hip_runtime.h>

#include "fem_kernels.h"
#include "mpm_device.h"

namespace mpmx {

namespace fem {

MD float3 ld3(const float* p) { return make_float3(p[0], p[1], p[2]); }
MD float3 sub3(float3 a, float3 b) { return make_float3(a.x - b.x, a.y - b.y, a.z - b.z); }
MD float3 cross3f(float3 a, float3 b) {
  return make_float3(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}
MD float dot3f(float3 a, float3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }

// matrix with columns a, b, c
MD M3 from_cols(float3 a, float3 b, float3 c) {
  M3 r;
  r.m[0][0] = a.x; r.m[1][0] = a.y; r.m[2][0] = a.z;
  r.m[0][1] = b.x; r.m[1][1] = b.y; r.m[2][1] = b.z;
  r.m[0][2] = c.x; r.m[1][2] = c.y; r.m[2][2] = c.z;
  return r;
}
MD float3 col(const M3& A, int j) { return make_float3(A.m[0][j], A.m[1][j], A.m[2][j]); }
MD float ddot(const M3& A, const M3& B) {
  float s = 0.f;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) s = fmaf(A.m[i][j], B.m[i][j], s);
  return s;
}
// cof(F) = dJ/dF: column j is the cross product of the next two columns of F (cyclically)
MD M3 cofactor(const M3& F) {
  const float3 f0 = col(F, 0), f1 = col(F, 1), f2 = col(F, 2);
  return from_cols(cross3f(f1, f2), cross3f(f2, f0), cross3f(f0, f1));
}
// directional derivative of cof at F along G
MD M3 dcofactor(const M3& F, const M3& G) {
  const float3 f0 = col(F, 0), f1 = col(F, 1), f2 = col(F, 2);
  const float3 g0 = col(G, 0), g1 = col(G, 1), g2 = col(G, 2);
  const float3 a = cross3f(g1, f2), b = cross3f(f1, g2);
  const float3 c = cross3f(g2, f0), d = cross3f(f2, g0);
  const float3 p = cross3f(g0, f1), q = cross3f(f0, g1);
  return from_cols(make_float3(a.x + b.x, a.y + b.y, a.z + b.z), make_float3(c.x + d.x, c.y + d.y, c.z + d.z),
                   make_float3(p.x + q.x, p.y + q.y, p.z + q.z));
}

struct Prm {
  float mu, lam, rho, damp, ke, kd, kf, zg, alpha;
};
MD Prm load_prm(const float* p) {
  Prm r;
  r.mu = p[0]; r.lam = p[1]; r.rho = p[2]; r.damp = p[3];
  r.ke = p[4]; r.kd = p[5]; r.kf = p[6]; r.zg = p[7];
  r.alpha = 1.f + 0.75f * r.mu / r.lam;
  return r;
}

// LDS layout of the forward block (floats): x [3n], v [3n], per-element force columns [9T], lumped volume [n],
// then ints: incidence offsets [n + 1], incidences [4T]
struct FwdLds {
  float *xs, *vs, *tf, *ws;
  int *ioff, *inc;
};
MD FwdLds fwd_lds(float* base, int n, int T) {
  FwdLds L;
  L.xs = base;
  L.vs = L.xs + 3 * n;
  L.tf = L.vs + 3 * n;
  L.ws = L.tf + 9 * T;
  L.ioff = reinterpret_cast<int*>(L.ws + n);
  L.inc = L.ioff + n + 1;
  return L;
}

// the backward block: x, v of state k [3n each], their cotangents [3n each], u = dt/m vbar_tot [3n], per-element
// cotangent columns [9T] (those of D_s, then of D_v, gathered one after the other), lumped volume [n], incidence
// offsets [n + 1], incidences [4T]
struct BwdLds {
  float *xs, *vs, *xb, *vb, *us, *tb, *ws;
  int *ioff, *inc;
};
MD BwdLds bwd_lds(float* base, int n, int T) {
  BwdLds L;
  L.xs = base;
  L.vs = L.xs + 3 * n;
  L.xb = L.vs + 3 * n;
  L.vb = L.xb + 3 * n;
  L.us = L.vb + 3 * n;
  L.tb = L.us + 3 * n;
  L.ws = L.tb + 9 * T;
  L.ioff = reinterpret_cast<int*>(L.ws + n);
  L.inc = L.ioff + n + 1;
  return L;
}

MD void load_topology(const FemMesh& m, int e, float* ws, int* ioff, int* inc) {
  for (int i = threadIdx.x; i < m.n; i += blockDim.x) ws[i] = m.wm[(int64_t)e * m.n + i];
  for (int i = threadIdx.x; i <= m.n; i += blockDim.x) ioff[i] = m.inc_off[i];
  for (int i = threadIdx.x; i < 4 * m.T; i += blockDim.x) inc[i] = m.inc[i];
}

// element data a thread keeps for the whole launch
template <int TPT>
struct OwnTets {
  int4 t[TPT];
  M3 B[TPT];
  float W[TPT];
};
template <int TPT>
MD void load_own_tets(const FemMesh& m, int e, OwnTets<TPT>& o) {
#pragma unroll
  for (int q = 0; q < TPT; ++q) {
    const int t = threadIdx.x + q * kFemThreads;
    if (t < m.T) {
      o.t[q] = m.tets[t];
      const float* b = m.Bm + ((int64_t)e * m.T + t) * 9;
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) o.B[q].m[i][j] = b[3 * i + j];
      o.W[q] = m.W[(int64_t)e * m.T + t];
    } else {
      o.t[q] = make_int4(0, 0, 0, 0);
      o.B[q] = m3_zero();
      o.W[q] = 0.f;
    }
  }
}

// D of an element from a node array: columns p[i1] - p[i0], p[i2] - p[i0], p[i3] - p[i0]
MD M3 edge_matrix(const float* p, int4 t) {
  const float3 p0 = ld3(p + 3 * t.x);
  return from_cols(sub3(ld3(p + 3 * t.y), p0), sub3(ld3(p + 3 * t.z), p0), sub3(ld3(p + 3 * t.w), p0));
}

// one incidence's term: the element's column of the node's corner (corners 1..3), or minus the sum of its three
// columns (corner 0); `code` is tet * 4 + corner
MD float3 column_term(const float* cols, int stride, int code) {
  const float* h = cols + (int64_t)(code >> 2) * stride;
  const int c = code & 3;
  if (c > 0) return make_float3(h[3 * (c - 1)], h[3 * (c - 1) + 1], h[3 * (c - 1) + 2]);
  return make_float3(-(h[0] + h[3] + h[6]), -(h[1] + h[4] + h[7]), -(h[2] + h[5] + h[8]));
}

// sum over node i's incidences of the per-element columns cols[(tet * stride + c) * 3 ..] for corners c = 1..3,
// corner 0 taking minus the sum of its element's three columns; two incidences per iteration, so that their
// index and column reads overlap (the sum is taken in incidence order all the same)
MD float3 gather_columns(const float* cols, int stride, const int* ioff, const int* inc, int i) {
  float3 s = make_float3(0.f, 0.f, 0.f);
  int q = ioff[i];
  const int qe = ioff[i + 1];
  for (; q + 1 < qe; q += 2) {
    const int c0 = inc[q], c1 = inc[q + 1];
    const float3 a = column_term(cols, stride, c0), b = column_term(cols, stride, c1);
    s.x += a.x; s.y += a.y; s.z += a.z;
    s.x += b.x; s.y += b.y; s.z += b.z;
  }
  if (q < qe) {
    const float3 a = column_term(cols, stride, inc[q]);
    s.x += a.x; s.y += a.y; s.z += a.z;
  }
  return s;
}

// ----------------------------------------------------------------------------
// rest data
// ----------------------------------------------------------------------------
__global__ void k_fem_rest(FemMesh m, const float* __restrict__ X, float* __restrict__ Bm, float* __restrict__ W,
                           int32_t* __restrict__ bad) {
  const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= (int64_t)m.E * m.T) return;
  const int e = (int)(id / m.T), t = (int)(id - (int64_t)e * m.T);
  const int4 tt = m.tets[t];
  const M3 D = edge_matrix(X + (int64_t)e * m.n * 3, tt);
  const float3 d0 = col(D, 0), d1 = col(D, 1), d2 = col(D, 2);
  const float3 c12 = cross3f(d1, d2), c20 = cross3f(d2, d0), c01 = cross3f(d0, d1);
  const float det = dot3f(d0, c12);
  // longest edge: the three from node 0 and the three between the others
  float L2 = fmaxf(fmaxf(dot3f(d0, d0), dot3f(d1, d1)), dot3f(d2, d2));
  const float3 e01 = sub3(d1, d0), e02 = sub3(d2, d0), e12 = sub3(d2, d1);
  L2 = fmaxf(L2, fmaxf(fmaxf(dot3f(e01, e01), dot3f(e02, e02)), dot3f(e12, e12)));
  const float L3 = L2 * sqrtf(L2);
  if (!(fabsf(det) >= 1e-9f * L3) || !isfinite(det)) {
    atomicOr(bad, 1);
    return;
  }
  // rows of D^-1 are the cross products of the other two columns over det
  const float inv = 1.f / det;
  float* b = Bm + id * 9;
  b[0] = c12.x * inv; b[1] = c12.y * inv; b[2] = c12.z * inv;
  b[3] = c20.x * inv; b[4] = c20.y * inv; b[5] = c20.z * inv;
  b[6] = c01.x * inv; b[7] = c01.y * inv; b[8] = c01.z * inv;
  W[id] = fabsf(det) * (1.f / 6.f);
}

__global__ void k_fem_lumped(FemMesh m, const float* __restrict__ W, float* __restrict__ wm) {
  const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= (int64_t)m.E * m.n) return;
  const int e = (int)(id / m.n), i = (int)(id - (int64_t)e * m.n);
  float s = 0.f;
  for (int q = m.inc_off[i]; q < m.inc_off[i + 1]; ++q) s += W[(int64_t)e * m.T + (m.inc[q] >> 2)];
  wm[id] = 0.25f * s;
}

// ----------------------------------------------------------------------------
// forward
// ----------------------------------------------------------------------------
template <int TPT>
__global__ void __launch_bounds__(kFemThreads) k_fem_forward(FemMesh m, int S, float* __restrict__ x,
                                                             float* __restrict__ v, const float* __restrict__ act,
                                                             float* __restrict__ tape,
                                                             float* __restrict__ tape_act, int32_t* __restrict__ errs) {
  extern __shared__ float fem_lds[];
  const int e = blockIdx.x, n = m.n, T = m.T, E = m.E;
  const FwdLds L = fwd_lds(fem_lds, n, T);
  const int64_t node0 = (int64_t)e * n * 3;
  for (int i = threadIdx.x; i < 3 * n; i += blockDim.x) {
    L.xs[i] = x[node0 + i];
    L.vs[i] = v[node0 + i];
  }
  load_topology(m, e, L.ws, L.ioff, L.inc);
  const Prm p = load_prm(m.prm + (int64_t)e * kFemPrm);
  OwnTets<TPT> own;
  load_own_tets<TPT>(m, e, own);
  if (tape)
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
      float* o = tape + ((int64_t)e * n + i) * 6;
      for (int c = 0; c < 3; ++c) {
        o[c] = x[node0 + 3 * i + c];
        o[3 + c] = v[node0 + 3 * i + c];
      }
    }
  __syncthreads();
  for (int k = 0; k < S; ++k) {
    // element pass: P, and the forces -W P B_m^T on corners 1..3
#pragma unroll
    for (int q = 0; q < TPT; ++q) {
      const int t = threadIdx.x + q * kFemThreads;
      if (t >= T) continue;
      const int64_t ai = ((int64_t)k * E + e) * T + t;
      const float a = act ? act[ai] : 0.f;
      if (tape_act) tape_act[ai] = a;
      const M3 F = m3_mul(edge_matrix(L.xs, own.t[q]), own.B[q]);
      const M3 Fd = m3_mul(edge_matrix(L.vs, own.t[q]), own.B[q]);
      const float Ic = ddot(F, F);
      const float J = m3_det(F);
      const float s = p.mu * (1.f - 1.f / (Ic + 1.f));
      const float r = p.lam * (J - p.alpha - a);
      const M3 cof = cofactor(F);
      M3 P;
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) P.m[i][j] = fmaf(s, F.m[i][j], fmaf(r, cof.m[i][j], p.damp * Fd.m[i][j]));
      const M3 H = m3_mul_abt(P, own.B[q]);   // P B_m^T
      float* h = L.tf + t * 9;
      for (int c = 0; c < 3; ++c)
        for (int rr = 0; rr < 3; ++rr) h[3 * c + rr] = -own.W[q] * H.m[rr][c];
    }
    __syncthreads();
    // node pass: gather, ground contact, semi-implicit Euler
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
      float3 f = gather_columns(L.tf, 9, L.ioff, L.inc, i);
      const float3 xi = ld3(L.xs + 3 * i), vi = ld3(L.vs + 3 * i);
      if (xi.z < p.zg) {
        f.x -= p.kf * vi.x;
        f.y -= p.kf * vi.y;
        f.z += p.ke * (p.zg - xi.z) - p.kd * vi.z;
      }
      const float im = 1.f / (p.rho * L.ws[i]);
      const float3 vn = make_float3(vi.x + m.dt * (f.x * im + m.g[0]), vi.y + m.dt * (f.y * im + m.g[1]),
                                    vi.z + m.dt * (f.z * im + m.g[2]));
      const float3 xn = make_float3(xi.x + m.dt * vn.x, xi.y + m.dt * vn.y, xi.z + m.dt * vn.z);
      L.xs[3 * i] = xn.x; L.xs[3 * i + 1] = xn.y; L.xs[3 * i + 2] = xn.z;
      L.vs[3 * i] = vn.x; L.vs[3 * i + 1] = vn.y; L.vs[3 * i + 2] = vn.z;
      if (tape) {
        float* o = tape + (((int64_t)(k + 1) * E + e) * n + i) * 6;
        o[0] = xn.x; o[1] = xn.y; o[2] = xn.z;
        o[3] = vn.x; o[4] = vn.y; o[5] = vn.z;
      }
    }
    __syncthreads();
  }
  bool finite = true;
  for (int i = threadIdx.x; i < 3 * n; i += blockDim.x) {
    const float a = L.xs[i], b = L.vs[i];
    x[node0 + i] = a;
    v[node0 + i] = b;
    finite = finite && isfinite(a) && isfinite(b);
  }
  if (!finite) atomicOr(&errs[e], 1);
}

// ----------------------------------------------------------------------------
// backward
// ----------------------------------------------------------------------------
template <int TPT>
__global__ void __launch_bounds__(kFemThreads) k_fem_backward(FemMesh m, int S, const float* __restrict__ tape,
                                                              const float* __restrict__ tape_act,
                                                              const float* __restrict__ gx,
                                                              const float* __restrict__ gv, float* __restrict__ dx0,
                                                              float* __restrict__ dv0, float* __restrict__ dact,
                                                              double* __restrict__ dprm) {
  extern __shared__ float fem_lds[];
  __shared__ double red[kFemThreads / 64][8];
  const int e = blockIdx.x, n = m.n, T = m.T, E = m.E;
  const BwdLds L = bwd_lds(fem_lds, n, T);
  const int64_t node0 = (int64_t)e * n * 3;
  for (int i = threadIdx.x; i < 3 * n; i += blockDim.x) {
    L.xb[i] = gx ? gx[node0 + i] : 0.f;
    L.vb[i] = gv ? gv[node0 + i] : 0.f;
  }
  load_topology(m, e, L.ws, L.ioff, L.inc);
  const Prm p = load_prm(m.prm + (int64_t)e * kFemPrm);
  OwnTets<TPT> own;
  load_own_tets<TPT>(m, e, own);
  // per-thread parameter cotangents: mu, lam, damp, k_e, k_d, k_f, z_g
  float pmu = 0.f, plam = 0.f, pdamp = 0.f, pke = 0.f, pkd = 0.f, pkf = 0.f, pzg = 0.f;
  // the tape rows of this thread's nodes (n <= 2 * kFemThreads) for the next substep, read one substep ahead
  float pf[2][6];
  auto prefetch = [&](int k) {
#pragma unroll
    for (int jn = 0; jn < 2; ++jn) {
      const int i = threadIdx.x + jn * kFemThreads;
      if (k >= 0 && i < n) {
        const float* st = tape + (((int64_t)k * E + e) * n + i) * 6;
        for (int c = 0; c < 6; ++c) pf[jn][c] = st[c];
      }
    }
  };
  prefetch(S - 1);
  __syncthreads();
  for (int k = S - 1; k >= 0; --k) {
    // node pass 1: state k from the tape; vbar_tot = vbar' + dt xbar'; u = dt/m vbar_tot (the force
    // cotangent); ground-contact terms
#pragma unroll
    for (int jn = 0; jn < 2; ++jn) {
      const int i = threadIdx.x + jn * kFemThreads;
      if (i >= n) continue;
      const float3 xi = make_float3(pf[jn][0], pf[jn][1], pf[jn][2]);
      const float3 vi = make_float3(pf[jn][3], pf[jn][4], pf[jn][5]);
      L.xs[3 * i] = xi.x; L.xs[3 * i + 1] = xi.y; L.xs[3 * i + 2] = xi.z;
      L.vs[3 * i] = vi.x; L.vs[3 * i + 1] = vi.y; L.vs[3 * i + 2] = vi.z;
      float3 xb = ld3(L.xb + 3 * i), vb = ld3(L.vb + 3 * i);
      vb = make_float3(fmaf(m.dt, xb.x, vb.x), fmaf(m.dt, xb.y, vb.y), fmaf(m.dt, xb.z, vb.z));
      const float c = m.dt / (p.rho * L.ws[i]);
      const float3 u = make_float3(c * vb.x, c * vb.y, c * vb.z);
      L.us[3 * i] = u.x; L.us[3 * i + 1] = u.y; L.us[3 * i + 2] = u.z;
      if (xi.z < p.zg) {
        xb.z -= p.ke * u.z;
        vb.z -= p.kd * u.z;
        vb.x -= p.kf * u.x;
        vb.y -= p.kf * u.y;
        pke = fmaf(p.zg - xi.z, u.z, pke);
        pkd = fmaf(-vi.z, u.z, pkd);
        pkf -= vi.x * u.x + vi.y * u.y;
        pzg = fmaf(p.ke, u.z, pzg);
      }
      L.xb[3 * i] = xb.x; L.xb[3 * i + 1] = xb.y; L.xb[3 * i + 2] = xb.z;
      L.vb[3 * i] = vb.x; L.vb[3 * i + 1] = vb.y; L.vb[3 * i + 2] = vb.z;
    }
    prefetch(k - 1);   // in flight during the element pass
    __syncthreads();
    // element pass: with G = Ubar B_m (Ubar the edge differences of u), the element's share of the
    // loss is -W P : G; its cotangents are Fbar = -W dP[G] (the energy Hessian is symmetric),
    // Fdot_bar = -W damp G, and the activation's W lam cof(F) : G
    M3 dvb[TPT];   // the D_v cotangent columns wait in registers for the second gather
#pragma unroll
    for (int q = 0; q < TPT; ++q) {
      const int t = threadIdx.x + q * kFemThreads;
      dvb[q] = m3_zero();
      if (t >= T) continue;
      const int64_t ai = ((int64_t)k * E + e) * T + t;
      const float a = tape_act[ai];
      const M3 B = own.B[q];
      const float Wt = own.W[q];
      const M3 F = m3_mul(edge_matrix(L.xs, own.t[q]), B);
      const M3 Fd = m3_mul(edge_matrix(L.vs, own.t[q]), B);
      const M3 G = m3_mul(edge_matrix(L.us, own.t[q]), B);
      const float Ic = ddot(F, F);
      const float J = m3_det(F);
      const float ic1 = 1.f / (Ic + 1.f);
      const float s = p.mu * (1.f - ic1);
      const float r = p.lam * (J - p.alpha - a);
      const M3 cof = cofactor(F);
      const M3 dcof = dcofactor(F, G);
      const float FG = ddot(F, G), cG = ddot(cof, G);
      const float c2 = 2.f * p.mu * ic1 * ic1 * FG;
      M3 Fb, Fdb;
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
          const float dP = fmaf(s, G.m[i][j], fmaf(c2, F.m[i][j], fmaf(p.lam * cG, cof.m[i][j], r * dcof.m[i][j])));
          Fb.m[i][j] = -Wt * dP;
          Fdb.m[i][j] = -Wt * p.damp * G.m[i][j];
        }
      const M3 Dsb = m3_mul_abt(Fb, B);
      dvb[q] = m3_mul_abt(Fdb, B);
      float* h = L.tb + t * 9;
      for (int c = 0; c < 3; ++c)
        for (int rr = 0; rr < 3; ++rr) h[3 * c + rr] = Dsb.m[rr][c];
      if (dact) dact[ai] = Wt * p.lam * cG;
      pmu -= Wt * ((1.f - ic1) * FG - 0.75f * cG);
      plam -= Wt * (J - p.alpha - a + 0.75f * p.mu / p.lam) * cG;
      pdamp -= Wt * ddot(Fd, G);
    }
    __syncthreads();
    // node pass 2: the element cotangents gathered onto the nodes give the cotangent of state k, the
    // D_s columns first, then (through the same LDS) the D_v columns
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
      const float3 sx = gather_columns(L.tb, 9, L.ioff, L.inc, i);
      L.xb[3 * i] += sx.x; L.xb[3 * i + 1] += sx.y; L.xb[3 * i + 2] += sx.z;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < TPT; ++q) {
      const int t = threadIdx.x + q * kFemThreads;
      if (t >= T) continue;
      float* h = L.tb + t * 9;
      for (int c = 0; c < 3; ++c)
        for (int rr = 0; rr < 3; ++rr) h[3 * c + rr] = dvb[q].m[rr][c];
    }
    __syncthreads();
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
      const float3 sv = gather_columns(L.tb, 9, L.ioff, L.inc, i);
      L.vb[3 * i] += sv.x; L.vb[3 * i + 1] += sv.y; L.vb[3 * i + 2] += sv.z;
    }
    // the next iteration's node pass 1 touches only this thread's own nodes, and its element pass
    // starts after a barrier, so no barrier is needed here
  }
  __syncthreads();
  for (int i = threadIdx.x; i < 3 * n; i += blockDim.x) {
    dx0[node0 + i] = L.xb[i];
    dv0[node0 + i] = L.vb[i];
  }
  if (!dprm) return;
  // block sums of the parameter cotangents in FP64
  double part[7] = {pmu, plam, pdamp, pke, pkd, pkf, pzg};
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int c = 0; c < 7; ++c) {
    double vsum = part[c];
    for (int off = 32; off > 0; off >>= 1) vsum += __shfl_down(vsum, off);
    if (lane == 0) red[wave][c] = vsum;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double tot[7];
    for (int c = 0; c < 7; ++c) {
      tot[c] = 0.0;
      for (int w = 0; w < kFemThreads / 64; ++w) tot[c] += red[w][c];
    }
    const float* pr = m.prm + (int64_t)e * kFemPrm;
    // rho dL/drho = -(mu dL/dmu + lam dL/dlam + damp dL/ddamp + k_e dL/dk_e + k_d dL/dk_d + k_f dL/dk_f)
    const double scaled = (double)pr[0] * tot[0] + (double)pr[1] * tot[1] + (double)pr[3] * tot[2] +
                          (double)pr[4] * tot[3] + (double)pr[5] * tot[4] + (double)pr[6] * tot[5];
    double* o = dprm + (int64_t)e * kFemPrm;
    o[0] = tot[0];
    o[1] = tot[1];
    o[2] = -scaled / (double)pr[2];
    o[3] = tot[2];
    o[4] = tot[3];
    o[5] = tot[4];
    o[6] = tot[5];
    o[7] = tot[6];
  }
}

// dynamic LDS above 64 KiB has to be allowed per kernel
template <typename K>
void allow_lds(K kernel, size_t bytes) {
  if (bytes > 65536) (void)hipFuncSetAttribute((const void*)kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

int tets_per_thread(int T) {
  const int q = (T + kFemThreads - 1) / kFemThreads;
  return q <= 1 ? 1 : (q <= 2 ? 2 : 4);
}

}  // namespace fem

using namespace fem;

size_t fem_forward_lds(int n, int T) { return sizeof(float) * (size_t)(8 * n + 13 * T + 1); }
size_t fem_backward_lds(int n, int T) { return sizeof(float) * (size_t)(17 * n + 13 * T + 1); }

void launch_fem_rest(const FemMesh& m, const float* X, float* Bm, float* W, float* wm, int32_t* bad,
                     hipStream_t s) {
  const int64_t nt = (int64_t)m.E * m.T, nn = (int64_t)m.E * m.n;
  hipLaunchKernelGGL(k_fem_rest, dim3((unsigned)((nt + 255) / 256)), dim3(256), 0, s, m, X, Bm, W, bad);
  hipLaunchKernelGGL(k_fem_lumped, dim3((unsigned)((nn + 255) / 256)), dim3(256), 0, s, m, W, wm);
}

void launch_fem_forward(const FemMesh& m, int S, float* x, float* v, const float* act, float* tape,
                        float* tape_act, int32_t* errs, hipStream_t s) {
  const size_t lds = fem_forward_lds(m.n, m.T);
  switch (tets_per_thread(m.T)) {
    case 1:
      allow_lds(k_fem_forward<1>, lds);
      hipLaunchKernelGGL(k_fem_forward<1>, dim3(m.E), dim3(kFemThreads), lds, s, m, S, x, v, act, tape, tape_act, errs);
      break;
    case 2:
      allow_lds(k_fem_forward<2>, lds);
      hipLaunchKernelGGL(k_fem_forward<2>, dim3(m.E), dim3(kFemThreads), lds, s, m, S, x, v, act, tape, tape_act, errs);
      break;
    default:
      allow_lds(k_fem_forward<4>, lds);
      hipLaunchKernelGGL(k_fem_forward<4>, dim3(m.E), dim3(kFemThreads), lds, s, m, S, x, v, act, tape, tape_act, errs);
  }
}

void launch_fem_backward(const FemMesh& m, int S, const float* tape, const float* tape_act, const float* gx,
                         const float* gv, float* dx0, float* dv0, float* dact, double* dprm, hipStream_t s) {
  const size_t lds = fem_backward_lds(m.n, m.T);
  switch (tets_per_thread(m.T)) {
    case 1:
      allow_lds(k_fem_backward<1>, lds);
      hipLaunchKernelGGL(k_fem_backward<1>, dim3(m.E), dim3(kFemThreads), lds, s, m, S, tape, tape_act, gx, gv, dx0,
                         dv0, dact, dprm);
      break;
    case 2:
      allow_lds(k_fem_backward<2>, lds);
      hipLaunchKernelGGL(k_fem_backward<2>, dim3(m.E), dim3(kFemThreads), lds, s, m, S, tape, tape_act, gx, gv, dx0,
                         dv0, dact, dprm);
      break;
    default:
      allow_lds(k_fem_backward<4>, lds);
      hipLaunchKernelGGL(k_fem_backward<4>, dim3(m.E), dim3(kFemThreads), lds, s, m, S, tape, tape_act, gx, gv, dx0,
                         dv0, dact, dprm);
  }
}

}  // namespace mpmx
