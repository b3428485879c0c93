// Host-visible launchers of the articulated rigid-body kernels (internal to the library).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mpmx {

constexpr int kRbPrm = 5;      // damp, k_e, k_d, k_f, z_g
constexpr int kRbLinkF = 26;   // per link: joint_rot (9), joint_pos (3), axis (3), mass, com (3), inertia (6),
                               // prismatic (1) or revolute (0)

// shared links of a rigid-body batch and its per-env parameters
struct RbModel {
  int E, N, C;
  const float* link;        // [N][kRbLinkF]; root joint_pos already relative to the spatial origin
  const uint64_t* anc;      // [N] bit j: joint j is on the path from the root to link i (i included)
  const uint64_t* desc;     // [N] bit k: link k is in the subtree of link i (i included)
  const uint64_t* kids;     // [N] bit k: link k's parent is link i
  const int32_t* level;     // [N] height (longest path down to a leaf) | depth (joints above) << 16
  const uint64_t* hmask;    // [H] bit k: link k has height h
  int H, D;                 // height and depth levels
  const int32_t* cbeg;      // [N + 1] contact range of each link
  const float* contact;     // [C][4] sphere centre (link frame), radius
  const float* prm;         // [E][kRbPrm]
  float dt;
  float g[3];
  float zref;               // height of the spatial origin (subtracted from z_g)
};

// lanes of a wave that one environment uses (links rounded up to 8, 16, 32 or 64)
int rb_group(int N);

// S substeps of every env from (q, qd) [E][N] in place; tau [S][E][N] or null; with tape non-null, the states
// [S + 1][E][2][N] (q then qd) and the torques [S][E][N] are kept
void launch_rb_forward(const RbModel& m, int S, float* q, float* qd, const float* tau, float* tape, float* tape_tau,
                       int32_t* errs, hipStream_t s);

// reverse mode over the S recorded substeps: (gq, gqd) cotangents of the final state (null = 0), out:
// dq0, dqd0 [E][N], dtau [S][E][N] (or null), dprm [E][kRbPrm] doubles (or null)
void launch_rb_backward(const RbModel& m, int S, const float* tape, const float* tape_tau, const float* gq,
                        const float* gqd, float* dq0, float* dqd0, float* dtau, double* dprm, hipStream_t s);

}  // namespace mpmx
