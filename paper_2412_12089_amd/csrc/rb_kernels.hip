// Articulated rigid bodies on a fixed base (Appendix D.1): the batched forward
// substeps (composite rigid body algorithm for the mass matrix, recursive
// Newton-Euler for the bias forces, a sparse Cholesky solve, semi-implicit Euler) and
// their reverse-mode adjoint.
//
// One environment per group of G lanes of a wave (G: the link count rounded up
// to 8, 16, 32 or 64), lane i working on link i; a block is one wave, so its
// barriers are cheap. Every spatial quantity is a world-frame Plucker vector
// about one fixed origin (motion: angular velocity, velocity of the body point
// at the origin; force: moment about the origin, force). In that frame the
// tree recursions need no coordinate transforms: a link's velocity and
// acceleration are sums over the joints on its root path, its subtree force
// and composite inertia are sums over its subtree, and each lane takes those
// sums from LDS (through the link's ancestor bit mask, and children first over
// the tree's height levels). The
// joint-space mass matrix is M_ij = S_j . (Ic_i S_i) for j on i's root path
// and zero between different branches. Factorised leaves first, M = L^T L
// keeps that sparsity (no fill-in: eliminating a link touches only its root
// path), so the factorisation and the solve with L^T run one tree height level
// at a time and the solve with L one depth level at a time: a barrier per
// level instead of one per joint. A substep touches HBM only for the torques
// and the tape.
#include <hip/hip_runtime.h>

#include <cmath>

#include "mpm_device.h"
#include "rb_kernels.h"

namespace mpmx {

namespace rb {

constexpr int kBlock = 64;   // one wave per block

struct V6 {
  float c[6];   // [0..2] angular part (or moment), [3..5] linear part (or force)
};

MD V6 zero6() {
  V6 r;
#pragma unroll
  for (int k = 0; k < 6; ++k) r.c[k] = 0.f;
  return r;
}
MD V6 add6(const V6& a, const V6& b) {
  V6 r;
#pragma unroll
  for (int k = 0; k < 6; ++k) r.c[k] = a.c[k] + b.c[k];
  return r;
}
MD V6 sub6(const V6& a, const V6& b) {
  V6 r;
#pragma unroll
  for (int k = 0; k < 6; ++k) r.c[k] = a.c[k] - b.c[k];
  return r;
}
MD V6 scale6(const V6& a, float s) {
  V6 r;
#pragma unroll
  for (int k = 0; k < 6; ++k) r.c[k] = a.c[k] * s;
  return r;
}
MD float dot6(const V6& a, const V6& b) {
  float s = 0.f;
#pragma unroll
  for (int k = 0; k < 6; ++k) s = fmaf(a.c[k], b.c[k], s);
  return s;
}
MD void cross3(const float* a, const float* b, float* r) {
  r[0] = a[1] * b[2] - a[2] * b[1];
  r[1] = a[2] * b[0] - a[0] * b[2];
  r[2] = a[0] * b[1] - a[1] * b[0];
}
// motion x motion: (w_a x w_b, w_a x v_b + v_a x w_b)
MD V6 crm(const V6& a, const V6& b) {
  V6 r;
  float t[3];
  cross3(a.c, b.c, r.c);
  cross3(a.c, b.c + 3, r.c + 3);
  cross3(a.c + 3, b.c, t);
  r.c[3] += t[0]; r.c[4] += t[1]; r.c[5] += t[2];
  return r;
}
// motion x* force: (w x n + v x f, w x f)
MD V6 crf(const V6& a, const V6& f) {
  V6 r;
  float t[3];
  cross3(a.c, f.c, r.c);
  cross3(a.c + 3, f.c + 3, t);
  r.c[0] += t[0]; r.c[1] += t[1]; r.c[2] += t[2];
  cross3(a.c, f.c + 3, r.c + 3);
  return r;
}

// spatial inertia about the origin: mass, first moment h = m c, rotational inertia J about the origin
// (symmetric: xx yy zz xy xz yz)
struct Inertia {
  float m, h[3], J[6];
};
MD V6 iapply(const Inertia& I, const V6& a) {
  const float* w = a.c;
  const float* v = a.c + 3;
  V6 r;
  float t[3];
  cross3(I.h, v, t);
  r.c[0] = I.J[0] * w[0] + I.J[3] * w[1] + I.J[4] * w[2] + t[0];
  r.c[1] = I.J[3] * w[0] + I.J[1] * w[1] + I.J[5] * w[2] + t[1];
  r.c[2] = I.J[4] * w[0] + I.J[5] * w[1] + I.J[2] * w[2] + t[2];
  cross3(I.h, w, t);
  r.c[3] = I.m * v[0] - t[0];
  r.c[4] = I.m * v[1] - t[1];
  r.c[5] = I.m * v[2] - t[2];
  return r;
}

// a lane's own link
struct Link {
  float Rt[9], pt[3], ax[3], m, com[3], In[6];
  uint64_t anc, desc, kids;
  int cb, ce;
  int height, depth;   // levels: longest path down to a leaf, joints above
  bool prism;          // the joint slides along its axis instead of turning about it
};
MD Link load_link(const RbModel& M, int i, bool live) {
  Link l;
  const float* s = M.link + (size_t)(live ? i : 0) * kRbLinkF;
#pragma unroll
  for (int k = 0; k < 9; ++k) l.Rt[k] = s[k];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    l.pt[k] = s[9 + k];
    l.ax[k] = s[12 + k];
    l.com[k] = s[16 + k];
  }
  l.m = s[15];
#pragma unroll
  for (int k = 0; k < 6; ++k) l.In[k] = s[19 + k];
  l.anc = live ? M.anc[i] : 0ull;
  l.desc = live ? M.desc[i] : 0ull;
  l.kids = live ? M.kids[i] : 0ull;
  l.cb = live ? M.cbeg[i] : 0;
  l.ce = live ? M.cbeg[i + 1] : 0;
  l.height = live ? (M.level[i] & 0xffff) : -1;
  l.depth = live ? (M.level[i] >> 16) : -1;
  l.prism = s[25] != 0.f;
  return l;
}

struct Prm {
  float damp, ke, kd, kf, zg;   // zg relative to the spatial origin
};
MD Prm load_prm(const RbModel& M, int e) {
  Prm p{0.f, 0.f, 0.f, 0.f, -INFINITY};
  if (e < M.E) {
    const float* r = M.prm + (size_t)e * kRbPrm;
    p.damp = r[0]; p.ke = r[1]; p.kd = r[2]; p.kf = r[3]; p.zg = r[4] - M.zref;
  }
  return p;
}

// LDS of a block. The environments' columns are interleaved (column
// env * G + link of each row), so the four environments of a wave use
// different banks when their lanes touch the same link. The joint blocks live
// only while the lanes compose their poses; the inertias and the mass matrix
// are written after the next barriers, so the two share their space.
template <int G>
struct BlockLds {
  float X[6][kBlock];   // exchange of 6-vectors (and the final parameter-cotangent reduction)
  float Y[6][kBlock];
  float dinv[kBlock];   // 1 / L_kk
  float y[kBlock];      // substitution values
  float x[kBlock];
  union {
    float B[12][kBlock];   // per joint: joint_rot Rot(axis, q) (9), joint_pos (3)
    struct {
      float Ic[10][kBlock];                // body inertias, summed over subtrees
      float M[kBlock / G][G][G + 1];       // per env, row i, entries j on i's root path: the mass matrix, then L
    } cm;
  } u;
};

// one environment's view of the block's LDS: row pointers offset to its columns
template <int G>
struct EnvLds {
  float (*X)[kBlock];
  float (*Y)[kBlock];
  float (*B)[kBlock];
  float (*Ic)[kBlock];
  float (*M)[G + 1];
  float *dinv, *y, *x;
};
template <int G>
MD EnvLds<G> env_lds(BlockLds<G>& s, int grp) {
  const int c0 = grp * G;
  EnvLds<G> e;
  e.X = reinterpret_cast<float(*)[kBlock]>(&s.X[0][c0]);
  e.Y = reinterpret_cast<float(*)[kBlock]>(&s.Y[0][c0]);
  e.B = reinterpret_cast<float(*)[kBlock]>(&s.u.B[0][c0]);
  e.Ic = reinterpret_cast<float(*)[kBlock]>(&s.u.cm.Ic[0][c0]);
  e.M = s.u.cm.M[grp];
  e.dinv = s.dinv + c0;
  e.y = s.y + c0;
  e.x = s.x + c0;
  return e;
}

// sum of the 6-vectors of the links in a bit mask (a root path or a subtree), in ascending link order
MD V6 mask_sum(const float (*A)[kBlock], uint64_t mk) {
  V6 r = zero6();
  while (mk) {
    const int j = __builtin_ctzll(mk);
    mk &= mk - 1;
#pragma unroll
    for (int k = 0; k < 6; ++k) r.c[k] += A[k][j];
  }
  return r;
}
MD void put6(float (*A)[kBlock], int lane, const V6& v) {
#pragma unroll
  for (int k = 0; k < 6; ++k) A[k][lane] = v.c[k];
}
MD V6 get6(const float (*A)[kBlock], int j) {
  V6 r;
#pragma unroll
  for (int k = 0; k < 6; ++k) r.c[k] = A[k][j];
  return r;
}

// Subtree sums in place: every lane's column of the NA rows of A and the NB
// rows of B holds its link's own values on entry (visible after a barrier) and
// the sum over its subtree on return. One height level at a time, a link adds
// its children's finished sums, so a level costs the most children of any of
// its links (not the size of the largest subtree).
template <int NA, int NB>
MD void subtree_sums(const RbModel& M, const Link& l, int lane, bool live, float (*A)[kBlock], float (*B)[kBlock]) {
  for (int h = 1; h < M.H; ++h) {
    if (live && l.height == h) {
      float a[NA], b[NB > 0 ? NB : 1];
#pragma unroll
      for (int k = 0; k < NA; ++k) a[k] = A[k][lane];
#pragma unroll
      for (int k = 0; k < NB; ++k) b[k] = B[k][lane];
      uint64_t mk = l.kids;
      while (mk) {
        const int c = __builtin_ctzll(mk);
        mk &= mk - 1;
#pragma unroll
        for (int k = 0; k < NA; ++k) a[k] += A[k][c];
#pragma unroll
        for (int k = 0; k < NB; ++k) b[k] += B[k][c];
      }
#pragma unroll
      for (int k = 0; k < NA; ++k) A[k][lane] = a[k];
#pragma unroll
      for (int k = 0; k < NB; ++k) B[k][lane] = b[k];
    }
    __syncthreads();
  }
}

// what the adjoint needs of one substep's forward, per lane
struct Frame {
  float R[9], p[3];
  V6 S, V, u, Ab, fext;
  Inertia I;
};

MD void contact_point(const RbModel& M, const Frame& F, int c, float* cw, float* x) {
  const float* s = M.contact + (size_t)c * 4;
#pragma unroll
  for (int a = 0; a < 3; ++a) cw[a] = F.p[a] + F.R[3 * a] * s[0] + F.R[3 * a + 1] * s[1] + F.R[3 * a + 2] * s[2];
  x[0] = cw[0];
  x[1] = cw[1];
  x[2] = cw[2] - s[3];
}

// Solves M x = b with M = L^T L in E.M / E.dinv: L^T y = b over the height
// levels (y_k takes the subtree's y), then L x = y over the depth levels (x_k
// takes the root path's x); b and x are per lane (lane < N).
template <int G>
MD float tree_solve(const RbModel& M, const Link& l, EnvLds<G>& E, int lane, bool live, float b) {
  float y = 0.f;
  for (int h = 0; h < M.H; ++h) {
    if (live && l.height == h) {
      float t = b;
      uint64_t mk = l.desc & ~(1ull << lane);
      while (mk) {
        const int c = __builtin_ctzll(mk);
        mk &= mk - 1;
        t = fmaf(-E.M[c][lane], E.y[c], t);
      }
      y = t * E.dinv[lane];
      E.y[lane] = y;
    }
    __syncthreads();
  }
  float x = 0.f;
  for (int d = 0; d < M.D; ++d) {
    if (live && l.depth == d) {
      float t = y;
      uint64_t mk = l.anc & ~(1ull << lane);
      while (mk) {
        const int j = __builtin_ctzll(mk);
        mk &= mk - 1;
        t = fmaf(-E.M[lane][j], E.x[j], t);
      }
      x = t * E.dinv[lane];
      E.x[lane] = x;
    }
    __syncthreads();
  }
  return x;
}

// One substep's dynamics of an environment: fills F, leaves M's factor L in E and returns qdd of the
// lane's joint. Every lane of the block calls it (barriers inside).
template <int G>
MD float dynamics(const RbModel& M, const Link& l, EnvLds<G>& E, int lane, bool live, float q, float qd, float tau,
                  const Prm& P, Frame& F) {
  // joint blocks B = joint_rot Rot(axis, q) (Rodrigues: c I + s [a]x + (1 - c) a a^T) and joint_pos; a
  // prismatic joint turns nothing (Rot = I) and shifts joint_pos by q joint_rot axis
  {
    float sn = 0.f, cs = 1.f;
    if (!l.prism) sincosf(q, &sn, &cs);
    const float* a = l.ax;
    const float oc = 1.f - cs;
    float Rq[9] = {cs + oc * a[0] * a[0], oc * a[0] * a[1] - sn * a[2], oc * a[0] * a[2] + sn * a[1],
                   oc * a[1] * a[0] + sn * a[2], cs + oc * a[1] * a[1], oc * a[1] * a[2] - sn * a[0],
                   oc * a[2] * a[0] - sn * a[1], oc * a[2] * a[1] + sn * a[0], cs + oc * a[2] * a[2]};
    if (live) {
#pragma unroll
      for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c)
          E.B[3 * r + c][lane] = l.Rt[3 * r] * Rq[c] + l.Rt[3 * r + 1] * Rq[3 + c] + l.Rt[3 * r + 2] * Rq[6 + c];
      const float qs = l.prism ? q : 0.f;
#pragma unroll
      for (int k = 0; k < 3; ++k)
        E.B[9 + k][lane] = fmaf(qs, l.Rt[3 * k] * a[0] + l.Rt[3 * k + 1] * a[1] + l.Rt[3 * k + 2] * a[2], l.pt[k]);
    }
  }
  __syncthreads();
  // world pose: walk the root path (ascending joint index is root first)
  {
    float R[9] = {1.f, 0.f, 0.f, 0.f, 1.f, 0.f, 0.f, 0.f, 1.f};
    float p[3] = {0.f, 0.f, 0.f};
    uint64_t mk = l.anc;
    while (mk) {
      const int j = __builtin_ctzll(mk);
      mk &= mk - 1;
      const float t0 = E.B[9][j], t1 = E.B[10][j], t2 = E.B[11][j];
#pragma unroll
      for (int r = 0; r < 3; ++r) p[r] += R[3 * r] * t0 + R[3 * r + 1] * t1 + R[3 * r + 2] * t2;
      float Rn[9];
#pragma unroll
      for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c)
          Rn[3 * r + c] = R[3 * r] * E.B[c][j] + R[3 * r + 1] * E.B[3 + c][j] + R[3 * r + 2] * E.B[6 + c][j];
#pragma unroll
      for (int k = 0; k < 9; ++k) R[k] = Rn[k];
    }
#pragma unroll
    for (int k = 0; k < 9; ++k) F.R[k] = R[k];
#pragma unroll
    for (int k = 0; k < 3; ++k) F.p[k] = p[k];
  }
  // joint motion S = (s, p x s) for a revolute joint, (0, s) for a prismatic one, s = R axis; body inertia
  // about the origin
  {
    const float* R = F.R;
    float s[3];
#pragma unroll
    for (int r = 0; r < 3; ++r) s[r] = R[3 * r] * l.ax[0] + R[3 * r + 1] * l.ax[1] + R[3 * r + 2] * l.ax[2];
    if (l.prism) {
      F.S.c[0] = 0.f; F.S.c[1] = 0.f; F.S.c[2] = 0.f;
      F.S.c[3] = s[0]; F.S.c[4] = s[1]; F.S.c[5] = s[2];
    } else {
      F.S.c[0] = s[0]; F.S.c[1] = s[1]; F.S.c[2] = s[2];
      cross3(F.p, s, F.S.c + 3);
    }
    float c[3];
#pragma unroll
    for (int r = 0; r < 3; ++r) c[r] = F.p[r] + R[3 * r] * l.com[0] + R[3 * r + 1] * l.com[1] + R[3 * r + 2] * l.com[2];
    // R Ib R^T
    const float Ib[9] = {l.In[0], l.In[3], l.In[4], l.In[3], l.In[1], l.In[5], l.In[4], l.In[5], l.In[2]};
    float T[9];
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
      for (int k = 0; k < 3; ++k) T[3 * r + k] = R[3 * r] * Ib[k] + R[3 * r + 1] * Ib[3 + k] + R[3 * r + 2] * Ib[6 + k];
    float W[9];
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
      for (int k = 0; k < 3; ++k) W[3 * r + k] = T[3 * r] * R[3 * k] + T[3 * r + 1] * R[3 * k + 1] + T[3 * r + 2] * R[3 * k + 2];
    const float m = l.m;
    const float cc = c[0] * c[0] + c[1] * c[1] + c[2] * c[2];
    F.I.m = m;
    F.I.h[0] = m * c[0]; F.I.h[1] = m * c[1]; F.I.h[2] = m * c[2];
    F.I.J[0] = W[0] + m * (cc - c[0] * c[0]);
    F.I.J[1] = W[4] + m * (cc - c[1] * c[1]);
    F.I.J[2] = W[8] + m * (cc - c[2] * c[2]);
    F.I.J[3] = W[1] - m * c[0] * c[1];
    F.I.J[4] = W[2] - m * c[0] * c[2];
    F.I.J[5] = W[5] - m * c[1] * c[2];
  }
  // velocities: V_i = sum over the root path of S_j qd_j
  F.u = scale6(F.S, qd);
  if (live) put6(E.X, lane, F.u);
  __syncthreads();
  F.V = mask_sum(E.X, l.anc);
  // bias accelerations (qdd = 0): A_i = A_0 + sum over the root path of V_j x S_j qd_j, A_0 = -g
  if (live) put6(E.Y, lane, crm(F.V, F.u));
  __syncthreads();
  F.Ab = mask_sum(E.Y, l.anc);
  F.Ab.c[3] -= M.g[0];
  F.Ab.c[4] -= M.g[1];
  F.Ab.c[5] -= M.g[2];
  // ground contact on the link's spheres
  F.fext = zero6();
  for (int c = l.cb; c < l.ce; ++c) {
    float cw[3], x[3], xd[3];
    contact_point(M, F, c, cw, x);
    cross3(F.V.c, x, xd);
    xd[0] += F.V.c[3]; xd[1] += F.V.c[4]; xd[2] += F.V.c[5];
    const float depth = P.zg - x[2];
    if (depth > 0.f) {
      const float f[3] = {-P.kf * xd[0], -P.kf * xd[1], P.ke * depth - P.kd * xd[2]};
      float n[3];
      cross3(x, f, n);
      F.fext.c[0] += n[0]; F.fext.c[1] += n[1]; F.fext.c[2] += n[2];
      F.fext.c[3] += f[0]; F.fext.c[4] += f[1]; F.fext.c[5] += f[2];
    }
  }
  const V6 f = sub6(add6(iapply(F.I, F.Ab), crf(F.V, iapply(F.I, F.V))), F.fext);
  __syncthreads();
  if (live) {
    put6(E.X, lane, f);
    E.Ic[0][lane] = F.I.m;
#pragma unroll
    for (int k = 0; k < 3; ++k) E.Ic[1 + k][lane] = F.I.h[k];
#pragma unroll
    for (int k = 0; k < 6; ++k) E.Ic[4 + k][lane] = F.I.J[k];
    put6(E.Y, lane, F.S);
  }
  __syncthreads();
  // subtree sums: force (bias torque S_i . F_i) and composite inertia
  subtree_sums<6, 10>(M, l, lane, live, E.X, E.Ic);
  const V6 Ft = get6(E.X, lane);
  Inertia Ic;
  Ic.m = E.Ic[0][lane];
#pragma unroll
  for (int k = 0; k < 3; ++k) Ic.h[k] = E.Ic[1 + k][lane];
#pragma unroll
  for (int k = 0; k < 6; ++k) Ic.J[k] = E.Ic[4 + k][lane];
  const float rhs = tau - dot6(F.S, Ft) - P.damp * qd;
  // mass matrix row: M_ij = S_j . (Ic_i S_i) for j on the root path (the lane's own row only)
  if (live) {
    const V6 Fc = iapply(Ic, F.S);
    uint64_t mk = l.anc;
    while (mk) {
      const int j = __builtin_ctzll(mk);
      mk &= mk - 1;
      E.M[lane][j] = dot6(get6(E.Y, j), Fc);
    }
  }
  // M = L^T L, leaves first, one height level at a time: the level's links finish their rows (their
  // subtrees are eliminated), then every link updates its own row with the level's links below it,
  // M_ij -= L_ki L_kj for j on i's root path. Rows a level reads are never written in that level.
  for (int h = 0; h < M.H; ++h) {
    if (live && l.height == h) {
      const float d = sqrtf(E.M[lane][lane]);   // a non-positive pivot gives NaN: the env is flagged non-finite
      const float di = 1.f / d;
      E.M[lane][lane] = d;
      E.dinv[lane] = di;
      uint64_t mk = l.anc & ~(1ull << lane);
      while (mk) {
        const int j = __builtin_ctzll(mk);
        mk &= mk - 1;
        E.M[lane][j] *= di;
      }
    }
    __syncthreads();
    if (live) {
      uint64_t mk = l.desc & M.hmask[h] & ~(1ull << lane);
      while (mk) {
        const int k = __builtin_ctzll(mk);
        mk &= mk - 1;
        const float lki = E.M[k][lane];
        uint64_t aj = l.anc;
        while (aj) {
          const int j = __builtin_ctzll(aj);
          aj &= aj - 1;
          E.M[lane][j] = fmaf(-lki, E.M[k][j], E.M[lane][j]);
        }
      }
    }
  }
  __syncthreads();
  return tree_solve(M, l, E, lane, live, rhs);
}

template <int G>
__global__ __launch_bounds__(kBlock) void k_rb_forward(RbModel M, int S, float* __restrict__ q,
                                                       float* __restrict__ qd, const float* __restrict__ tau,
                                                       float* __restrict__ tape, float* __restrict__ tape_tau,
                                                       int32_t* __restrict__ errs) {
  constexpr int EPB = kBlock / G;
  __shared__ BlockLds<G> lds;
  const int lane = threadIdx.x % G, grp = threadIdx.x / G;
  const int e = blockIdx.x * EPB + grp;
  const int N = M.N, E = M.E;
  const bool live = e < E && lane < N;
  EnvLds<G> L = env_lds(lds, grp);
  const Link l = load_link(M, lane, live);
  const Prm P = load_prm(M, e);
  const size_t at = (size_t)e * N + lane;
  float qi = live ? q[at] : 0.f, qdi = live ? qd[at] : 0.f;
  if (tape && live) {
    tape[(size_t)e * 2 * N + lane] = qi;
    tape[(size_t)e * 2 * N + N + lane] = qdi;
  }
  for (int s = 0; s < S; ++s) {
    const float ti = (tau && live) ? tau[(size_t)s * E * N + at] : 0.f;
    if (tape_tau && live) tape_tau[(size_t)s * E * N + at] = ti;
    Frame F;
    const float qdd = dynamics<G>(M, l, L, lane, live, qi, qdi, ti, P, F);
    qdi = fmaf(M.dt, qdd, qdi);
    qi = fmaf(M.dt, qdi, qi);
    if (tape && live) {
      float* t = tape + ((size_t)(s + 1) * E + e) * 2 * N;
      t[lane] = qi;
      t[N + lane] = qdi;
    }
  }
  if (live) {
    q[at] = qi;
    qd[at] = qdi;
    if (!isfinite(qi) || !isfinite(qdi)) atomicOr(&errs[e], 1);
  }
}

// three waves per SIMD (168 VGPRs, three of them spilled): faster than two without spills once the chip is full
template <int G>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(3, 8))) void k_rb_backward(RbModel M, int S, const float* __restrict__ tape,
                                                        const float* __restrict__ tape_tau,
                                                        const float* __restrict__ gq, const float* __restrict__ gqd,
                                                        float* __restrict__ dq0, float* __restrict__ dqd0,
                                                        float* __restrict__ dtau, double* __restrict__ dprm) {
  constexpr int EPB = kBlock / G;
  __shared__ BlockLds<G> lds;
  const int lane = threadIdx.x % G, grp = threadIdx.x / G;
  const int e = blockIdx.x * EPB + grp;
  const int N = M.N, E = M.E;
  const bool live = e < E && lane < N;
  EnvLds<G> L = env_lds(lds, grp);
  const Link l = load_link(M, lane, live);
  const Prm P = load_prm(M, e);
  const size_t at = (size_t)e * N + lane;
  // cotangents of the current (q, qd)
  float a = (gq && live) ? gq[at] : 0.f;
  float b = (gqd && live) ? gqd[at] : 0.f;
  float acc[kRbPrm] = {0.f, 0.f, 0.f, 0.f, 0.f};
  for (int s = S - 1; s >= 0; --s) {
    const float* t = tape + ((size_t)s * E + e) * 2 * N;
    const float qi = live ? t[lane] : 0.f, qdi = live ? t[N + lane] : 0.f;
    const float ti = live ? tape_tau[(size_t)s * E * N + at] : 0.f;
    Frame F;
    const float qdd = dynamics<G>(M, l, L, lane, live, qi, qdi, ti, P, F);
    // qd' = qd + dt qdd, q' = q + dt qd': the cotangent of qd' is b + dt a, that of qdd dt (b + dt a)
    const float gtot = fmaf(M.dt, a, b);
    const float lam = tree_solve(M, l, L, lane, live, M.dt * gtot);   // torque cotangent M^-1 qdd_bar
    if (dtau && live) dtau[(size_t)s * E * N + at] = lam;
    acc[0] -= lam * qdi;
    // phi = lambda . ID(q, qd, qdd): accelerations with qdd, and Lambda_k = sum over k's root path of lambda_i S_i
    if (live) {
      put6(L.X, lane, scale6(F.S, qdd));
      put6(L.Y, lane, scale6(F.S, lam));
    }
    __syncthreads();
    const V6 A = add6(F.Ab, mask_sum(L.X, l.anc));
    const V6 Lam = mask_sum(L.Y, l.anc);
    const V6 IV = iapply(F.I, F.V);
    const V6 IA = iapply(F.I, A);
    const V6 f = sub6(add6(IA, crf(F.V, IV)), F.fext);
    // phi = sum_k Lambda_k . f_k: f_bar = Lambda; A_bar = I Lambda; V_bar from V x* (I V)
    const V6 Abar = iapply(F.I, Lam);
    const V6 VL = crm(F.V, Lam);
    const V6 IVL = iapply(F.I, VL);
    V6 Vbar = scale6(add6(crf(Lam, IV), IVL), -1.f);
    // geometric wrench of the body: the body's inertia turned with it, a . (I b) over the pairs
    // (Lambda, A) and (-V x Lambda, V) gives -(a x* I b + b x* I a)
    V6 W = sub6(add6(crf(VL, IV), crf(F.V, IVL)), add6(crf(Lam, IA), crf(A, Abar)));
    for (int c = l.cb; c < l.ce; ++c) {
      float cw[3], x[3], xd[3];
      contact_point(M, F, c, cw, x);
      cross3(F.V.c, x, xd);
      xd[0] += F.V.c[3]; xd[1] += F.V.c[4]; xd[2] += F.V.c[5];
      const float depth = P.zg - x[2];
      if (depth > 0.f) {
        const float fc[3] = {-P.kf * xd[0], -P.kf * xd[1], P.ke * depth - P.kd * xd[2]};
        // phi_c = -f . lh, lh = Lambda_v + Lambda_w x x (the point's velocity under Lambda)
        float lh[3];
        cross3(Lam.c, x, lh);
        lh[0] += Lam.c[3]; lh[1] += Lam.c[4]; lh[2] += Lam.c[5];
        const float xdb[3] = {P.kf * lh[0], P.kf * lh[1], P.kd * lh[2]};
        float xb[3], t1[3], t2[3];
        cross3(Lam.c, fc, t1);
        cross3(xdb, F.V.c, t2);
        xb[0] = t1[0] + t2[0];
        xb[1] = t1[1] + t2[1];
        xb[2] = t1[2] + t2[2] + P.ke * lh[2];
        // xd = v + w x x
        cross3(x, xdb, t1);
        Vbar.c[0] += t1[0]; Vbar.c[1] += t1[1]; Vbar.c[2] += t1[2];
        Vbar.c[3] += xdb[0]; Vbar.c[4] += xdb[1]; Vbar.c[5] += xdb[2];
        // the sphere centre moves with the body
        cross3(cw, xb, t1);
        W.c[0] += t1[0]; W.c[1] += t1[1]; W.c[2] += t1[2];
        W.c[3] += xb[0]; W.c[4] += xb[1]; W.c[5] += xb[2];
        // parameters (cotangent -dphi/dp)
        acc[1] += lh[2] * depth;
        acc[2] -= lh[2] * xd[2];
        acc[3] -= lh[0] * xd[0] + lh[1] * xd[1];
        acc[4] += P.ke * lh[2];
      }
    }
    __syncthreads();
    if (live) {
      put6(L.X, lane, f);
      put6(L.Y, lane, Abar);
    }
    __syncthreads();
    // phi = sum_i lambda_i S_i . F_i (F_i the subtree force) and A_i = A_0 + sum over the root path of
    // (S_j qdd_j + V_j x S_j qd_j): subtree sums of f and of A_bar
    subtree_sums<6, 6>(M, l, lane, live, L.X, L.Y);
    const V6 Ft = get6(L.X, lane), DA = get6(L.Y, lane);
    V6 Sbar = add6(scale6(Ft, lam), scale6(DA, qdd));
    Vbar = add6(Vbar, crf(F.u, DA));
    __syncthreads();
    if (live) put6(L.X, lane, Vbar);
    __syncthreads();
    // V_i = sum over the root path of u_j, u_j = S_j qd_j
    subtree_sums<6, 0>(M, l, lane, live, L.X, nullptr);
    const V6 ubar = sub6(get6(L.X, lane), crf(F.V, DA));
    Sbar = add6(Sbar, scale6(ubar, qdi));
    const float dphi_qd = dot6(F.S, ubar);
    W = add6(W, crf(F.S, Sbar));
    if (live) put6(L.Y, lane, W);
    __syncthreads();
    // turning joint j moves its whole subtree: dphi/dq_j = S_j . (subtree sum of the wrenches)
    subtree_sums<6, 0>(M, l, lane, live, L.Y, nullptr);
    const float dphi_q = dot6(F.S, get6(L.Y, lane));
    a = a - dphi_q;
    b = gtot - P.damp * lam - dphi_qd;
  }
  if (live) {
    dq0[at] = a;
    dqd0[at] = b;
  }
  if (dprm) {
    __syncthreads();
#pragma unroll
    for (int c = 0; c < kRbPrm; ++c) L.X[c][lane] = live ? acc[c] : 0.f;
    __syncthreads();
    if (lane < kRbPrm && e < E) {
      double s = 0.0;
      for (int k = 0; k < N; ++k) s += (double)L.X[lane][k];
      dprm[(size_t)e * kRbPrm + lane] = s;
    }
  }
}

}  // namespace rb

int rb_group(int N) { return N <= 8 ? 8 : N <= 16 ? 16 : N <= 32 ? 32 : 64; }

void launch_rb_forward(const RbModel& m, int S, float* q, float* qd, const float* tau, float* tape, float* tape_tau,
                       int32_t* errs, hipStream_t s) {
  const int G = rb_group(m.N), epb = rb::kBlock / G;
  const dim3 grid((m.E + epb - 1) / epb), block(rb::kBlock);
  switch (G) {
    case 8: rb::k_rb_forward<8><<<grid, block, 0, s>>>(m, S, q, qd, tau, tape, tape_tau, errs); break;
    case 16: rb::k_rb_forward<16><<<grid, block, 0, s>>>(m, S, q, qd, tau, tape, tape_tau, errs); break;
    case 32: rb::k_rb_forward<32><<<grid, block, 0, s>>>(m, S, q, qd, tau, tape, tape_tau, errs); break;
    default: rb::k_rb_forward<64><<<grid, block, 0, s>>>(m, S, q, qd, tau, tape, tape_tau, errs); break;
  }
}

void launch_rb_backward(const RbModel& m, int S, const float* tape, const float* tape_tau, const float* gq,
                        const float* gqd, float* dq0, float* dqd0, float* dtau, double* dprm, hipStream_t s) {
  const int G = rb_group(m.N), epb = rb::kBlock / G;
  const dim3 grid((m.E + epb - 1) / epb), block(rb::kBlock);
  switch (G) {
    case 8: rb::k_rb_backward<8><<<grid, block, 0, s>>>(m, S, tape, tape_tau, gq, gqd, dq0, dqd0, dtau, dprm); break;
    case 16: rb::k_rb_backward<16><<<grid, block, 0, s>>>(m, S, tape, tape_tau, gq, gqd, dq0, dqd0, dtau, dprm); break;
    case 32: rb::k_rb_backward<32><<<grid, block, 0, s>>>(m, S, tape, tape_tau, gq, gqd, dq0, dqd0, dtau, dprm); break;
    default: rb::k_rb_backward<64><<<grid, block, 0, s>>>(m, S, tape, tape_tau, gq, gqd, dq0, dqd0, dtau, dprm); break;
  }
}

}  // namespace mpmx
