// Device-side pieces of one MLS-MPM substep and its adjoint, all in registers.
//
// Physics: the paper's Appendix D.3 (MLS-MPM with APIC transfer, von Mises
// elastoplasticity with Hencky strain, weakly compressible fluid with the
// J^(1/3) projection, softened one-way contact) and the stable neo-Hookean
// energy of Appendix D.2 applied per particle.
//
// The isotropic 3x3 functions (corotated stress, Hencky stress, von Mises
// return mapping) are written through the left Cauchy-Green tensor
// b = F F^T = U diag(s) U^T (s = sigma^2), whose eigen-decomposition is the
// left half of F's SVD. Their adjoints use divided differences that stay
// finite when eigenvalues coincide (F = I at rest), never 1/(s_i - s_j).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mpmx {

#define MD __device__ __forceinline__

enum : int { MAT_NEOHOOKEAN = 0, MAT_COROTATED = 1, MAT_VONMISES = 2, MAT_FLUID_TAIT = 3, MAT_FLUID_PAPER = 4, MAT_COUNT = 5 };
enum : int { ERR_NONFINITE = 1, ERR_OUT_OF_DOMAIN = 2 };
// slots of the per-env parameter-cotangent accumulator (FP64)
enum : int { PB_MU = 0, PB_LAM, PB_SY, PB_K, PB_GAMMA, PB_MP, PB_VP, PB_COUNT };

constexpr float kSigmaMin = 1e-4f;   // singular values are clamped below this before the log
constexpr float kYieldScale = 2.0f;  // numerator of the printed yield offset kYieldScale*sigma_y/(2 mu)

constexpr int32_t kColliderBox = 1;      // box of half extents ch, axis-aligned in its own frame
constexpr int32_t kColliderSphere = 2;   // ball of radius ch[0]

// One kinematic collider of an environment (its grid update applies them in turn).
struct ColDev {
  int32_t has_collider;                  // 0 none, kColliderBox, kColliderSphere
  int32_t motion_off, motion_len;        // prescribed motion: rows [motion_off, + motion_len) of the motion
                                         // table, one per substep (len 0: constant velocity cv)
  float cc[3], ch[3], cv[3], c_alpha, c_mu;   // centre at t=0, half extents, velocity, contact softness, friction
  float c_axis[3];                       // rotation: unit axis (world), angle at t = 0, constant angular speed
  float c_angle, c_omega, c_round;       // (the box is axis-aligned in its own frame); the box's rounding radius
                                         // (its distance less c_round)
};
constexpr int kMaxColliders = 4;         // colliders per environment

// Per-environment settings as the kernels see them. The first block is
// written by the host; the derived block by the parameter-preparation kernel.
struct EnvDev {
  int32_t n, T, material, wall;          // nodes per axis, 4^3 tiles per axis
  int32_t n_col, nsub;                   // colliders in use (col[0, n_col), some may be off); nsub: substeps this
                                         // env takes in the current forward call
  int64_t p_off, p_cnt;                  // particle range in the batch arrays
  int64_t tile_off;                      // first tile of this env in the grid buffers
  float dt, fn, dx, gx, gy, gz;
  double E, nu, rho, Vp, sigma_y, K, gamma;   // user parameters (FP64 as given)
  // derived (a1): Lame parameters and constants in FP32
  float mu, lam, alpha_nh, mp, vp, sy, bulk, gam, yieldY;
  float pad1[3];
  int64_t row_off;                       // first row of this env in the caller's concatenated arrays
  int64_t p_cap;                         // particle capacity (positions [p_off, p_off + p_cap))
  ColDev col[kMaxColliders];
};


// a row of the prescribed collider motion table: center (3), velocity (3),
// angle about the box's axis, angular speed
constexpr int kMotionRow = 8;

// --------------------------------------------------------------------------
// small vector / matrix helpers
// --------------------------------------------------------------------------
struct M3 { float m[3][3]; };

MD M3 m3_zero() { M3 r; for (int i = 0; i < 3; ++i) for (int j = 0; j < 3; ++j) r.m[i][j] = 0.f; return r; }
MD M3 m3_eye() { M3 r = m3_zero(); r.m[0][0] = r.m[1][1] = r.m[2][2] = 1.f; return r; }
MD M3 m3_mul(const M3& a, const M3& b) {
  M3 r;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) r.m[i][j] = a.m[i][0] * b.m[0][j] + a.m[i][1] * b.m[1][j] + a.m[i][2] * b.m[2][j];
  return r;
}
MD M3 m3_mul_abt(const M3& a, const M3& b) {  // a b^T
  M3 r;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) r.m[i][j] = a.m[i][0] * b.m[j][0] + a.m[i][1] * b.m[j][1] + a.m[i][2] * b.m[j][2];
  return r;
}
MD M3 m3_mul_atb(const M3& a, const M3& b) {  // a^T b
  M3 r;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) r.m[i][j] = a.m[0][i] * b.m[0][j] + a.m[1][i] * b.m[1][j] + a.m[2][i] * b.m[2][j];
  return r;
}
MD M3 m3_add(const M3& a, const M3& b) { M3 r; for (int i = 0; i < 3; ++i) for (int j = 0; j < 3; ++j) r.m[i][j] = a.m[i][j] + b.m[i][j]; return r; }
MD M3 m3_scale(const M3& a, float s) { M3 r; for (int i = 0; i < 3; ++i) for (int j = 0; j < 3; ++j) r.m[i][j] = a.m[i][j] * s; return r; }
MD M3 m3_axpy(const M3& y, float s, const M3& x) { M3 r; for (int i = 0; i < 3; ++i) for (int j = 0; j < 3; ++j) r.m[i][j] = fmaf(s, x.m[i][j], y.m[i][j]); return r; }
MD M3 m3_sym(const M3& a) { M3 r; for (int i = 0; i < 3; ++i) for (int j = 0; j < 3; ++j) r.m[i][j] = 0.5f * (a.m[i][j] + a.m[j][i]); return r; }
MD M3 m3_transpose(const M3& a) { M3 r; for (int i = 0; i < 3; ++i) for (int j = 0; j < 3; ++j) r.m[i][j] = a.m[j][i]; return r; }
MD float m3_trace(const M3& a) { return a.m[0][0] + a.m[1][1] + a.m[2][2]; }
MD float m3_ddot(const M3& a, const M3& b) {
  float s = 0.f;
  for (int i = 0; i < 3; ++i) for (int j = 0; j < 3; ++j) s = fmaf(a.m[i][j], b.m[i][j], s);
  return s;
}
MD float m3_det(const M3& a) {
  return a.m[0][0] * (a.m[1][1] * a.m[2][2] - a.m[1][2] * a.m[2][1])
       - a.m[0][1] * (a.m[1][0] * a.m[2][2] - a.m[1][2] * a.m[2][0])
       + a.m[0][2] * (a.m[1][0] * a.m[2][1] - a.m[1][1] * a.m[2][0]);
}
// cofactor matrix: d det(A) / dA = det(A) A^-T
MD M3 m3_cof(const M3& a) {
  M3 c;
  c.m[0][0] = a.m[1][1] * a.m[2][2] - a.m[1][2] * a.m[2][1];
  c.m[0][1] = a.m[1][2] * a.m[2][0] - a.m[1][0] * a.m[2][2];
  c.m[0][2] = a.m[1][0] * a.m[2][1] - a.m[1][1] * a.m[2][0];
  c.m[1][0] = a.m[0][2] * a.m[2][1] - a.m[0][1] * a.m[2][2];
  c.m[1][1] = a.m[0][0] * a.m[2][2] - a.m[0][2] * a.m[2][0];
  c.m[1][2] = a.m[0][1] * a.m[2][0] - a.m[0][0] * a.m[2][1];
  c.m[2][0] = a.m[0][1] * a.m[1][2] - a.m[0][2] * a.m[1][1];
  c.m[2][1] = a.m[0][2] * a.m[1][0] - a.m[0][0] * a.m[1][2];
  c.m[2][2] = a.m[0][0] * a.m[1][1] - a.m[0][1] * a.m[1][0];
  return c;
}
// U diag(d) U^T (symmetric: the upper triangle is computed and mirrored)
MD M3 m3_spectral(const M3& U, const float d[3]) {
  M3 r;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const float ud[3] = {U.m[i][0] * d[0], U.m[i][1] * d[1], U.m[i][2] * d[2]};
#pragma unroll
    for (int j = i; j < 3; ++j) {
      r.m[i][j] = ud[0] * U.m[j][0] + ud[1] * U.m[j][1] + ud[2] * U.m[j][2];
      r.m[j][i] = r.m[i][j];
    }
  }
  return r;
}
// H + H^T + H H^T = F F^T - I (symmetric: upper triangle, mirrored)
MD M3 m3_left_strain(const M3& H) {
  M3 r;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = i; j < 3; ++j) {
      r.m[i][j] = H.m[i][j] + H.m[j][i] + H.m[i][0] * H.m[j][0] + H.m[i][1] * H.m[j][1] + H.m[i][2] * H.m[j][2];
      r.m[j][i] = r.m[i][j];
    }
  return r;
}
// U^T A U
MD M3 m3_rotate_in(const M3& U, const M3& A) { return m3_mul(m3_mul_atb(U, A), U); }
// U A U^T
MD M3 m3_rotate_out(const M3& U, const M3& A) { return m3_mul_abt(m3_mul(U, A), U); }

// --------------------------------------------------------------------------
// symmetric 3x3 eigen-decomposition by cyclic Jacobi rotations (fixed sweeps,
// no data-dependent loop): A = U diag(s) U^T
// --------------------------------------------------------------------------
// Each rotation is the classical Jacobi step in Rutishauser's numerically
// stable form (the tangent t of the smaller rotation angle from theta, then
// c = 1/sqrt(1 + t^2), s = t c, tau = s/(1 + c) and updates a - s (b + tau a);
// Rutishauser 1971, Handbook for Automatic Computation II, contribution II/1).
// The rotation uses the hardware reciprocal and square root (about 1 ulp) and
// no branch: c and s are built from t so that the rotation is orthogonal for
// any t, and an inexact t only leaves a slightly larger off-diagonal entry for
// the next sweep. A pair below 1e-30 counts as diagonal (that also keeps the
// reciprocal of 2 apq finite).
template <int p, int q, int r>
MD void jacobi_rotate(M3& A, M3& V) {
  const float apq = A.m[p][q];
  const float theta = (A.m[q][q] - A.m[p][p]) * __builtin_amdgcn_rcpf(2.f * apq);
  const float at = fabsf(theta);
  const float tm = __builtin_amdgcn_rcpf(at + __builtin_amdgcn_sqrtf(fmaf(at, at, 1.f)));
  const float t = fabsf(apq) > 1e-30f ? copysignf(tm, theta) : 0.f;
  const float c = __builtin_amdgcn_rsqf(fmaf(t, t, 1.f));   // argument >= 1: no denormal handling needed
  const float s = t * c;
  const float tau = s * __builtin_amdgcn_rcpf(1.f + c);
  A.m[p][p] -= t * apq;
  A.m[q][q] += t * apq;
  A.m[p][q] = A.m[q][p] = 0.f;
  const float arp = A.m[r][p], arq = A.m[r][q];
  A.m[r][p] = A.m[p][r] = arp - s * (arq + tau * arp);
  A.m[r][q] = A.m[q][r] = arq + s * (arp - tau * arq);
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const float vkp = V.m[k][p], vkq = V.m[k][q];
    V.m[k][p] = vkp - s * (vkq + tau * vkp);
    V.m[k][q] = vkq + s * (vkp - tau * vkq);
  }
}

// Four cyclic sweeps: in an FP32 emulation of this solver on strains 1e-4..0.3,
// including near-repeated eigenvalues, the corotated stress from four sweeps
// matched five to the last bit of its error vs FP64 (p99 3e-7); three left
// tails of 1e-5.
MD void eig_sym(M3 A, float s[3], M3& U) {
  U = m3_eye();
#pragma unroll
  for (int sweep = 0; sweep < 4; ++sweep) {
    jacobi_rotate<0, 1, 2>(A, U);
    jacobi_rotate<0, 2, 1>(A, U);
    jacobi_rotate<1, 2, 0>(A, U);
  }
  s[0] = A.m[0][0];
  s[1] = A.m[1][1];
  s[2] = A.m[2][2];
}

// expm1(z) / z, finite at 0
MD float expm1_over(float z) {
  if (fabsf(z) < 1e-3f) return 1.f + z * (0.5f + z * (1.f / 6.f));
  return expm1f(z) / z;
}

// --------------------------------------------------------------------------
// quadratic B-spline stencil of one particle
// --------------------------------------------------------------------------
struct Stencil {
  int b[3];        // base node
  float f[3];      // x n - base, in [0.5, 1.5) inside the band
  float w[3][3];   // w[axis][offset]
  float dw[3][3];  // dw/df
  bool oob;
};

// base = floor(x n - 1/2), bit-exact for FP32 x and n < 2^22 in FP32 alone: the
// fma rounds x n - 1/2 once, which can only carry it up onto the next integer;
// the residual x n - (b + 1/2), also one fma, has the exact sign and undoes
// that case
MD int base_floor(float x, int n) {
  const float fn = (float)n;
  float b = floorf(fmaf(x, fn, -0.5f));
  if (fmaf(x, fn, -(b + 0.5f)) < 0.f) b -= 1.f;
  return (int)b;
}

MD Stencil make_stencil(const float x[3], int n, float fn) {
  Stencil st;
  st.oob = false;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    int b = base_floor(x[a], n);
    if (b < 0 || b > n - 3) { st.oob = true; b = b < 0 ? 0 : n - 3; }
    st.b[a] = b;
    const float f = fmaf(x[a], fn, -(float)b);
    st.f[a] = f;
    const float f0 = 1.5f - f, f1 = f - 1.f, f2 = f - 0.5f;
    st.w[a][0] = 0.5f * f0 * f0;
    st.w[a][1] = 0.75f - f1 * f1;
    st.w[a][2] = 0.5f * f2 * f2;
    st.dw[a][0] = -f0;
    st.dw[a][1] = -2.f * f1;
    st.dw[a][2] = f2;
  }
  return st;
}

// storage index of node (i,j,k) of an env in a grid buffer laid out as
// [tile][channel(8)][64 nodes], tile = 4^3 nodes in raster order
MD int64_t node_base(const EnvDev& e, int i, int j, int k) {
  const int tile = ((i >> 2) * e.T + (j >> 2)) * e.T + (k >> 2);
  const int local = ((i & 3) << 4) | ((j & 3) << 2) | (k & 3);
  return (e.tile_off + tile) * 512 + local;
}
constexpr int CH = 64;  // channel stride inside a tile

// node_base is separable per axis: node_base(e, i, j, k) = e.tile_off * 512 +
// ax(i) + ay(j) + az(k). A gather precomputes the three offsets of each axis
// for its stencil once (element offsets within the env's grid block, below
// 2^32 for any grid this library allocates) and then addresses each of the 27
// nodes with two additions.
struct StencilAddr {
  uint32_t x[3], y[3], z[3];
};
MD StencilAddr stencil_addr(const EnvDev& e, const int b[3]) {
  StencilAddr s;
  const uint32_t T = (uint32_t)e.T;
#pragma unroll
  for (int o = 0; o < 3; ++o) {
    const uint32_t i = (uint32_t)(b[0] + o), j = (uint32_t)(b[1] + o), k = (uint32_t)(b[2] + o);
    s.x[o] = (i >> 2) * T * T * 512u + ((i & 3u) << 4);
    s.y[o] = (j >> 2) * T * 512u + ((j & 3u) << 2);
    s.z[o] = (k >> 2) * 512u + (k & 3u);
  }
  return s;
}

// --------------------------------------------------------------------------
// Deformation gradients are carried as H = F - I. Strains of 1e-4..1e-2 then
// keep FP32 precision relative to themselves (F rounds them relative to 1),
// and every quantity that vanishes at the rest state (J - 1, F F^T - I, the
// stresses) is formed from H without cancellation.
// --------------------------------------------------------------------------
MD M3 f_of(const M3& H) {
  M3 F = H;
  F.m[0][0] += 1.f; F.m[1][1] += 1.f; F.m[2][2] += 1.f;
  return F;
}
// det(I + H) - 1 = tr H + (principal 2x2 minors of H) + det H
MD float det_minus_one(const M3& H) {
  const float m2 = (H.m[0][0] * H.m[1][1] - H.m[0][1] * H.m[1][0]) + (H.m[0][0] * H.m[2][2] - H.m[0][2] * H.m[2][0]) +
                   (H.m[1][1] * H.m[2][2] - H.m[1][2] * H.m[2][1]);
  return m3_trace(H) + (m2 + m3_det(H));
}
// a6: F_tr = (I + dt C') F, as H_tr = H + dt C' (I + H)
MD M3 trial_h(const EnvDev& e, const M3& Cn, const M3& H) { return m3_axpy(H, e.dt, m3_add(Cn, m3_mul(Cn, H))); }

// (log1p(a) - log1p(b)) / (a - b) for a, b > -1, finite as a -> b (limit 1/(1+b))
MD float log1p_divdiff(float a, float b) {
  const float d = a - b;
  const float z = d / (1.f + b);
  if (fabsf(z) < 1e-3f) return (1.f - z * (0.5f - z * (1.f / 3.f))) / (1.f + b);
  return log1pf(z) / d;
}

// --------------------------------------------------------------------------
// a3: Kirchhoff stress tau = P F^T
// --------------------------------------------------------------------------
// `mat` is the material (a compile-time constant in the specialized
// kernels, e.material elsewhere).
// Quantities of F shared by the stress and its VJP (one eigen-decomposition
// of B = F F^T - I serves both in the P2G adjoint).
struct StressPrep {
  M3 B, U;      // B = F F^T - I = H + H^T + H H^T; U its eigenvectors
  float l[3];   // eigenvalues of B (those of F F^T minus one)
  float J, Jm1; // det F and det F - 1
};

MD StressPrep stress_prep(const EnvDev& e, const M3& H, int mat) {
  StressPrep p;
  p.Jm1 = det_minus_one(H);
  p.J = 1.f + p.Jm1;
  if (mat == MAT_NEOHOOKEAN || mat == MAT_COROTATED || mat == MAT_VONMISES)
    p.B = m3_left_strain(H);
  if (mat == MAT_COROTATED || mat == MAT_VONMISES) eig_sym(p.B, p.l, p.U);
  return p;
}

// the same quantities with the eigen-decomposition of B supplied (U, l kept
// from an earlier stress_prep of the same H)
MD StressPrep stress_prep_with_eig(const M3& H, const M3& U, const float l[3], int mat) {
  StressPrep p;
  p.Jm1 = det_minus_one(H);
  p.J = 1.f + p.Jm1;
  if (mat == MAT_NEOHOOKEAN || mat == MAT_COROTATED || mat == MAT_VONMISES)
    p.B = m3_left_strain(H);
  p.U = U;
  for (int i = 0; i < 3; ++i) p.l[i] = l[i];
  return p;
}

// singular value of F from an eigenvalue l of B: sqrt(1 + l), and sqrt(1 + l) - 1
MD void sv_of(float l, float& s, float& sm1) {
  const float lc = fmaxf(l, -1.f);
  s = __builtin_amdgcn_sqrtf(1.f + lc);   // about 1 ulp, like the reciprocal below
  sm1 = lc * __builtin_amdgcn_rcpf(1.f + s);
}
// log strain of an eigenvalue of B, with the singular value clamped at kSigmaMin
MD float log_strain(float l) { return 0.5f * log1pf(fmaxf(l, kSigmaMin * kSigmaMin - 1.f)); }
MD float clamp_l(float l) { return fmaxf(l, kSigmaMin * kSigmaMin - 1.f); }

MD M3 stress_from(const EnvDev& e, const StressPrep& p, int mat) {
  const float J = p.J, Jm1 = p.Jm1;
  switch (mat) {
    case MAT_NEOHOOKEAN: {
      // mu (1 - 1/(I_C + 1)) b + lam J (J - alpha) I with b = I + B, I_C = 3 + tr B and
      // alpha = 1 + 3 mu / (4 lam): the identity parts cancel at rest, so their sum is
      // mu (t / (4 (4 + t)) - 3/4 (J - 1)) + lam J (J - 1), t = tr B
      const float t = m3_trace(p.B);
      const float c1 = e.mu * (3.f + t) / (4.f + t);
      const float c0 = e.mu * (t / (4.f * (4.f + t)) - 0.75f * Jm1) + e.lam * J * Jm1;
      M3 r = m3_scale(p.B, c1);
      r.m[0][0] += c0; r.m[1][1] += c0; r.m[2][2] += c0;
      return r;
    }
    case MAT_COROTATED: {
      // 2 mu (F - R) F^T = 2 mu (b - b^(1/2)): eigenvalues s (s - 1), s = sqrt(1 + l)
      float h[3];
      for (int i = 0; i < 3; ++i) {
        float sg, sm1;
        sv_of(p.l[i], sg, sm1);
        h[i] = 2.f * e.mu * sg * sm1;
      }
      M3 r = m3_spectral(p.U, h);
      const float c2 = e.lam * J * Jm1;
      r.m[0][0] += c2; r.m[1][1] += c2; r.m[2][2] += c2;
      return r;
    }
    case MAT_VONMISES: {
      // U (2 mu eps + lam tr(eps) I) U^T, eps = log Sigma
      float eps[3];
      for (int i = 0; i < 3; ++i) eps[i] = log_strain(p.l[i]);
      const float tre = eps[0] + eps[1] + eps[2];
      float d[3];
      for (int i = 0; i < 3; ++i) d[i] = 2.f * e.mu * eps[i] + e.lam * tre;
      return m3_spectral(p.U, d);
    }
    case MAT_FLUID_TAIT: {
      // -J K (J^-gamma - 1)
      const float c = -e.bulk * J * expm1f(-e.gam * log1pf(Jm1));
      M3 r = m3_zero(); r.m[0][0] = r.m[1][1] = r.m[2][2] = c;
      return r;
    }
    default: {  // MAT_FLUID_PAPER: lam J (J - 1) I
      const float c = e.lam * J * Jm1;
      M3 r = m3_zero(); r.m[0][0] = r.m[1][1] = r.m[2][2] = c;
      return r;
    }
  }
}

// a3: Kirchhoff stress from H = F - I
MD M3 stress(const EnvDev& e, const M3& H, int mat) { return stress_from(e, stress_prep(e, H, mat), mat); }

// VJP of stress(): Fbar += d<taubar, tau>/dF, pb[] += d<taubar, tau>/d(params)
MD void stress_vjp_from(const EnvDev& e, const M3& H, const StressPrep& p, const M3& tb, M3& Fbar,
                        float pb[PB_COUNT], int mat) {
  const float J = p.J, Jm1 = p.Jm1;
  const float trtb = m3_trace(tb);
  const M3 F = f_of(H);
  switch (mat) {
    case MAT_NEOHOOKEAN: {
      const float t = m3_trace(p.B);
      const float inv = 1.f / (4.f + t);
      const float c1 = e.mu * (3.f + t) * inv;
      const M3 tbs = m3_sym(tb);
      const float c1b = m3_ddot(tb, p.B) + trtb;   // <taubar, b>
      const float Icb = c1b * e.mu * inv * inv;
      // b = F F^T: dF <- 2 bbar F with bbar = c1 sym(taubar); I_C: dF <- 2 Icbar F
      Fbar = m3_add(Fbar, m3_mul(m3_scale(tbs, 2.f * c1), F));
      Fbar = m3_axpy(Fbar, 2.f * Icb, F);
      // d/dJ of lam J (J - 1) - 3/4 mu J
      const float Jb = trtb * (e.lam * (2.f * J - 1.f) - 0.75f * e.mu);
      Fbar = m3_axpy(Fbar, Jb, m3_cof(F));
      // d/dmu: (1 - 1/(I_C+1)) <taubar, b> - 3/4 J tr(taubar), the identity part regrouped as in the stress
      pb[PB_MU] += m3_ddot(tb, p.B) * (3.f + t) * inv + trtb * (t * 0.25f * inv - 0.75f * Jm1);
      pb[PB_LAM] += trtb * J * Jm1;
      return;
    }
    case MAT_COROTATED: {
      float sg[3], hm = 0.f;
      const M3 G = m3_rotate_in(p.U, m3_sym(tb));
      for (int i = 0; i < 3; ++i) {
        float sm1;
        sv_of(p.l[i], sg[i], sm1);
        hm += G.m[i][i] * sg[i] * sm1;
      }
      // h(s) = s - sqrt(s): divided difference 1 - 1/(sigma_i + sigma_j)
      M3 Hd;
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) Hd.m[i][j] = 2.f * e.mu * G.m[i][j] * (1.f - __builtin_amdgcn_rcpf(sg[i] + sg[j]));
      const M3 bbar = m3_rotate_out(p.U, Hd);
      Fbar = m3_add(Fbar, m3_mul(m3_scale(bbar, 2.f), F));
      Fbar = m3_axpy(Fbar, trtb * e.lam * (2.f * J - 1.f), m3_cof(F));
      pb[PB_MU] += 2.f * hm;
      pb[PB_LAM] += trtb * J * Jm1;
      return;
    }
    case MAT_VONMISES: {
      float lc[3], ls[3];
      for (int i = 0; i < 3; ++i) { lc[i] = clamp_l(p.l[i]); ls[i] = log1pf(lc[i]); }
      const M3 G = m3_rotate_in(p.U, m3_sym(tb));
      M3 Bu;
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) Bu.m[i][j] = e.mu * G.m[i][j] * log1p_divdiff(lc[i], lc[j]);
      for (int i = 0; i < 3; ++i) Bu.m[i][i] += e.lam * trtb * 0.5f / (1.f + lc[i]);
      const M3 bbar = m3_rotate_out(p.U, Bu);
      Fbar = m3_add(Fbar, m3_mul(m3_scale(bbar, 2.f), F));
      float gl = 0.f;
      for (int i = 0; i < 3; ++i) gl += G.m[i][i] * ls[i];
      pb[PB_MU] += gl;
      pb[PB_LAM] += trtb * 0.5f * (ls[0] + ls[1] + ls[2]);
      return;
    }
    case MAT_FLUID_TAIT: {
      const float lJ = log1pf(Jm1);
      const float Jg = J * expf(-e.gam * lJ);  // J^(1-gamma)
      const float dc = e.bulk * (1.f - (1.f - e.gam) * Jg / J);
      Fbar = m3_axpy(Fbar, trtb * dc, m3_cof(F));
      pb[PB_K] += trtb * (-J * expm1f(-e.gam * lJ));   // J - J^(1-gamma)
      pb[PB_GAMMA] += trtb * e.bulk * Jg * lJ;
      return;
    }
    default: {
      Fbar = m3_axpy(Fbar, trtb * e.lam * (2.f * J - 1.f), m3_cof(F));
      pb[PB_LAM] += trtb * J * Jm1;
      return;
    }
  }
}

MD void stress_vjp(const EnvDev& e, const M3& H, const M3& tb, M3& Fbar, float pb[PB_COUNT], int mat) {
  stress_vjp_from(e, H, stress_prep(e, H, mat), tb, Fbar, pb, mat);
}

// --------------------------------------------------------------------------
// a6: return mapping P(F_tr), on H_tr = F_tr - I
// --------------------------------------------------------------------------
struct VMDecomp {   // shared by the projection and its VJP
  M3 U;
  float l[3];       // eigenvalues of F_tr F_tr^T - I, clamped at kSigmaMin^2 - 1
  float eh[3], g[3];
  float nrm, beta;
  bool plastic;
};

MD VMDecomp vm_decompose(const EnvDev& e, const M3& Htr) {
  VMDecomp d;
  const M3 B = m3_add(m3_add(Htr, m3_transpose(Htr)), m3_mul_abt(Htr, Htr));
  eig_sym(B, d.l, d.U);
  float eps[3];
  for (int i = 0; i < 3; ++i) {
    d.l[i] = clamp_l(d.l[i]);
    eps[i] = 0.5f * log1pf(d.l[i]);
  }
  const float mean = (eps[0] + eps[1] + eps[2]) * (1.f / 3.f);
  for (int i = 0; i < 3; ++i) d.eh[i] = eps[i] - mean;
  d.nrm = sqrtf(d.eh[0] * d.eh[0] + d.eh[1] * d.eh[1] + d.eh[2] * d.eh[2]);
  const float dgam = d.nrm - e.yieldY;
  d.plastic = dgam > 0.f;
  d.beta = d.plastic ? dgam / d.nrm : 0.f;
  for (int i = 0; i < 3; ++i) d.g[i] = expf(-d.beta * d.eh[i]);
  return d;
}

// returns H' = P(F_tr) - I
MD M3 project(const EnvDev& e, const M3& Htr, int mat) {
  if (mat == MAT_VONMISES) {
    const VMDecomp d = vm_decompose(e, Htr);
    if (!d.plastic) return Htr;
    // U exp(eps - dgam eps_hat/|eps_hat|) V^T = U diag(g) U^T F_tr, g = exp(-beta eps_hat):
    // H' = H_tr + U diag(g - 1) U^T F_tr
    float gm1[3];
    for (int i = 0; i < 3; ++i) gm1[i] = expm1f(-d.beta * d.eh[i]);
    return m3_add(Htr, m3_mul(m3_spectral(d.U, gm1), f_of(Htr)));
  }
  if (mat == MAT_FLUID_TAIT || mat == MAT_FLUID_PAPER) {
    const float c = expm1f(log1pf(det_minus_one(Htr)) * (1.f / 3.f));   // J^(1/3) - 1
    M3 r = m3_zero(); r.m[0][0] = r.m[1][1] = r.m[2][2] = c;
    return r;
  }
  return Htr;
}

// VJP of project(): returns Ftr_bar; pb[] += parameter cotangents
MD M3 project_vjp(const EnvDev& e, const M3& Htr, const M3& Fb, float pb[PB_COUNT], int mat) {
  if (mat == MAT_VONMISES) {
    const VMDecomp d = vm_decompose(e, Htr);
    if (!d.plastic) return Fb;
    const M3 Ftr = f_of(Htr);
    const M3 Mm = m3_spectral(d.U, d.g);
    M3 Ftb = m3_mul(Mm, Fb);                             // M symmetric: M^T Fbar'
    const M3 G = m3_rotate_in(d.U, m3_sym(m3_mul_abt(Fb, Ftr)));   // U^T sym(Mbar) U
    const float Y = e.yieldY, N = d.nrm, beta = d.beta;
    // diagonal: dg_i/ds_k with g_i = exp(-beta eh_i), beta = 1 - Y/N, s_k = 1 + l_k
    float S1 = 0.f, S2 = 0.f;
    for (int i = 0; i < 3; ++i) { S1 += G.m[i][i] * d.g[i] * d.eh[i]; S2 += G.m[i][i] * d.g[i]; }
    M3 Bu;
    for (int k = 0; k < 3; ++k)
      Bu.m[k][k] = -(0.5f / (1.f + d.l[k])) * (Y * d.eh[k] / (N * N * N) * S1 + beta * (G.m[k][k] * d.g[k] - S2 * (1.f / 3.f)));
    // off-diagonal: (g_i - g_j)/(s_i - s_j) = [-beta e^{-beta eh_j} phi(-beta (eh_i - eh_j))] * (1/2) L(s_i, s_j)
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        if (i == j) continue;
        const float dd = -beta * d.g[j] * expm1_over(-beta * (d.eh[i] - d.eh[j])) * 0.5f * log1p_divdiff(d.l[i], d.l[j]);
        Bu.m[i][j] = G.m[i][j] * dd;
      }
    const M3 bbar = m3_rotate_out(d.U, Bu);
    Ftb = m3_add(Ftb, m3_mul(m3_scale(bbar, 2.f), Ftr));
    // parameters: beta = 1 - Y/N, Y = kYieldScale sigma_y / (2 mu)
    const float betab = -S1;
    const float Yb = -betab / N;
    pb[PB_MU] += Yb * (-Y / e.mu);
    pb[PB_SY] += Yb * (kYieldScale / (2.f * e.mu));
    return Ftb;
  }
  if (mat == MAT_FLUID_TAIT || mat == MAT_FLUID_PAPER) {
    const float Jm1 = det_minus_one(Htr);
    const float J = 1.f + Jm1;
    const float c = expf(log1pf(Jm1) * (1.f / 3.f));
    const float k = m3_trace(Fb) * c / (3.f * J);   // d J^(1/3)/dJ = J^(1/3)/(3J)
    return m3_scale(m3_cof(f_of(Htr)), k);
  }
  return Fb;
}

}  // namespace mpmx
