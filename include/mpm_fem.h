/*
 * mpm_fem.h -- C interface of the batched, differentiable tetrahedral FEM
 * step of the same library (libmpmx.so), for MI355X (gfx950).
 *
 * What it computes (paper: Appendix D.2 "Finite element method"). Every
 * environment of a batch is one soft body meshed with the same tetrahedra
 * (shared topology; rest shapes, parameters and states per environment).
 * One substep, per environment:
 *   F   = D_s B_m,  dF/dt = D_v B_m          (linear tet: D_s, D_v edge differences, B_m = D_m^-1 at rest)
 *   P   = mu (1 - 1/(I_C + 1)) F + lam (J - alpha - a_e) cof(F) + damp dF/dt
 *         (the gradient of the stable neo-Hookean energy
 *          mu/2 (I_C - 3) + lam/2 (J - alpha - a_e)^2 - mu/2 log(I_C + 1),
 *          alpha = 1 + 3 mu / (4 lam), with the element's activation a_e
 *          shifting its volume target, plus viscous damping)
 *   f   : nodes 1..3 of element e get the columns of -W_e P B_m^T, node 0 minus their sum;
 *         nodes below the ground z_g get (-k_f v_x, -k_f v_y, k_e (z_g - z) - k_d v_z)
 *   v' = v + dt (f / m + g),  x' = x + dt v'  (semi-implicit Euler; m lumped: a quarter of rho W_e per node)
 * The reverse-mode adjoint maps cotangents of the final (x, v) to cotangents
 * of the initial (x, v), of every substep's activations and of each
 * environment's parameters (Appendix D's simulation-gradient chain).
 *
 * Conventions are those of mpm.h: status codes, device pointers owned by the
 * caller and used only during the call's stream work, asynchronous calls on
 * the stream given at creation, one host thread per handle. Node arrays are
 * float32 [n_envs][n_nodes][3], row-major.
 */
#ifndef MPM_FEM_H_
#define MPM_FEM_H_

#include "mpm.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mpm_fem mpm_fem;

#define MPM_FEM_MAX_NODES 512    /* nodes per environment */
#define MPM_FEM_MAX_TETS 1024    /* tetrahedra per environment */
#define MPM_FEM_PARAMS 8         /* per-env parameter row: mu, lam, rho, damp, k_e, k_d, k_f, z_g */

typedef struct {
  int32_t n_envs;        /* >= 1 */
  int32_t n_nodes;       /* 4 .. MPM_FEM_MAX_NODES */
  int32_t n_tets;        /* 1 .. MPM_FEM_MAX_TETS */
  int32_t max_substeps;  /* >= 0: substeps a recorded forward can keep for the backward */
  float dt;              /* substep length, > 0 */
  float gravity[3];      /* body acceleration */
  int32_t reserved[4];
} mpm_fem_desc;

/* Creates a FEM batch on the current device: `tets` is a HOST array
 * [n_tets][4] of node indices (each in [0, n_nodes), four distinct per
 * element, every node in some element), read during the call. Allocates the states, the tape of
 * max_substeps + 1 states and activations, and the rest data (through `alloc`
 * if given; see mpm.h). `stream` is a hipStream_t. Parameters start as
 * mu = lam = rho = 1, no damping, no ground contact (z_g = -inf).
 * Errors: INVALID_ARG (sizes, an index out of range, a repeated node, a
 * node in no element), OUT_OF_MEMORY, DEVICE_ERROR. */
int mpm_fem_create(const mpm_fem_desc* desc, const int32_t* tets, const mpm_allocator* alloc, void* stream,
                   mpm_fem** out);

/* Waits for the stream, frees all memory, destroys the handle. */
int mpm_fem_destroy(mpm_fem* f);

/* Rest positions X [n_envs][n_nodes][3] (device): computes each element's
 * B_m = D_m^-1 and rest volume W_e = |det D_m| / 6, and each node's lumped
 * volume (Appendix D.2: the energy is integrated over each element). Drops
 * any record. Synchronizes the stream. Errors: INVALID_ARG (null),
 * BAD_STATE (a degenerate element, |det D_m| < 1e-9 L^3 with L its longest
 * rest edge; the previous rest data is kept). */
int mpm_fem_set_rest(mpm_fem* f, const float* X);

/* Per-env parameters, a HOST array [n_envs][MPM_FEM_PARAMS] of doubles:
 * mu, lam (Lame pair of the energy, lam > 0), rho (> 0), damp (>= 0), and
 * the ground's k_e, k_d, k_f (>= 0) and height z_g. Drops any record.
 * Errors: INVALID_ARG. */
int mpm_fem_set_params(mpm_fem* f, const double* params);

/* Copies the state in (x, v device [n_envs][n_nodes][3]; v NULL = zero).
 * Drops any record. */
int mpm_fem_set_state(mpm_fem* f, const float* x, const float* v);

/* Copies the current state out (either pointer may be NULL). */
int mpm_fem_get_state(mpm_fem* f, float* x, float* v);

/* Runs S substeps (0 <= S) on every environment. act: device
 * [S][n_envs][n_tets] activations a_e of each substep, or NULL (all zero).
 * flags & MPM_FWD_RECORD keeps every state and the activations for
 * mpm_fem_backward (S <= max_substeps); otherwise any record is dropped.
 * Asynchronous. Errors: INVALID_ARG, BAD_STATE (record longer than the tape,
 * no rest data). */
int mpm_fem_forward(mpm_fem* f, int32_t S, const float* act, int32_t flags);

/* Reverse mode through the recorded forward of S substeps: given the
 * cotangents gx, gv of its final (x, v) (device, NULL = zero), writes the
 * cotangents of its initial (x, v) to dx0, dv0 (device, required), of each
 * substep's activations to dact (device [S][n_envs][n_tets], or NULL), and of
 * the parameters to dparams (device [n_envs][MPM_FEM_PARAMS] doubles, or
 * NULL). d/d rho comes from the scale identity of the step: scaling mu, lam,
 * rho, damp, k_e, k_d and k_f together leaves f / m unchanged, so
 * rho dL/drho = -(mu dL/dmu + lam dL/dlam + damp dL/ddamp + k_e dL/dk_e +
 * k_d dL/dk_d + k_f dL/dk_f). The state after the call is unchanged; the
 * record is kept. Asynchronous. Errors: INVALID_ARG, BAD_STATE (no record). */
int mpm_fem_backward(mpm_fem* f, const float* gx, const float* gv, float* dx0, float* dv0, float* dact,
                     double* dparams);

/* Waits for the stream; returns NONFINITE if a forward since the last call
 * produced a non-finite state in some environment (mpm_fem_env_errors says
 * which). */
int mpm_fem_sync(mpm_fem* f);

/* Per-environment error bits of the last mpm_fem_sync (1: non-finite). */
int mpm_fem_env_errors(mpm_fem* f, int32_t* errs);

/* Text of the last error on this handle. */
const char* mpm_fem_last_error(const mpm_fem* f);

/* Device bytes held by the handle. */
int64_t mpm_fem_memory_bytes(const mpm_fem* f);

#ifdef __cplusplus
}
#endif

#endif /* MPM_FEM_H_ */
