// Host-visible launchers of the tetrahedral FEM kernels (internal to the library).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mpmx {

constexpr int kFemThreads = 256;   // one block per environment
constexpr int kFemPrm = 8;         // mu, lam, rho, damp, k_e, k_d, k_f, z_g

// shared topology and per-env rest data of a FEM batch
struct FemMesh {
  int E, n, T;
  const int4* tets;       // [T] node indices
  const int32_t* inc_off; // [n + 1] node -> incidence range
  const int32_t* inc;     // [4 T] incidences: tet * 4 + corner
  const float* Bm;        // [E][T][9] D_m^-1, row-major
  const float* W;         // [E][T] rest volumes
  const float* wm;        // [E][n] lumped rest volume per node
  const float* prm;       // [E][kFemPrm]
  float dt;
  float g[3];
};

// B_m, W per (env, tet) and the lumped volume per (env, node) of rest positions X [E][n][3];
// *bad is set to 1 if an element is degenerate
void launch_fem_rest(const FemMesh& m, const float* X, float* Bm, float* W, float* wm, int32_t* bad, hipStream_t s);

// S substeps of every env from (x, v) [E][n][3] in place; act [S][E][T] or null; with tape non-null, the
// states [S + 1][E][n][6] (x then v per node) and the activations [S][E][T] are kept
void launch_fem_forward(const FemMesh& m, int S, float* x, float* v, const float* act, float* tape,
                        float* tape_act, int32_t* errs, hipStream_t s);

// reverse mode over the S recorded substeps: (gx, gv) cotangents of the final state (null = 0), out:
// dx0, dv0 [E][n][3], dact [S][E][T] (or null), dprm [E][kFemPrm] doubles (or null)
void launch_fem_backward(const FemMesh& m, int S, const float* tape, const float* tape_act, const float* gx,
                         const float* gv, float* dx0, float* dv0, float* dact, double* dprm, hipStream_t s);

// LDS bytes of the forward / backward block of a mesh size
size_t fem_forward_lds(int n, int T);
size_t fem_backward_lds(int n, int T);

}  // namespace mpmx
