/*
 * mpm.h -- C interface of a batched, differentiable MLS-MPM substep library
 * for AMD Instinct MI355X (gfx950).
 *
 * What it computes. One substep of the moving-least-squares material point
 * method with APIC transfer, per environment (paper: Appendix D.3 "Material
 * point method"; the transfer is Hu et al. 2018's MLS-MPM, cited there):
 *   P2G   m_i += w m_p,  P_i += w (m_p v_p + A_p d),  A_p = -dt V_p 4 n^2 tau_p + m_p C_p
 *   grid  v_i = P_i / m_i + dt g (m_i > 0, else 0), softened box contact, sticky walls
 *   G2P   v_p = sum w v_i,  C_p = 4 n^2 sum w v_i d^T,  x_p += dt v_p,  F_p <- Proj((I + dt C_p) F_p)
 * with the quadratic B-spline w, base node floor(x n - 1/2), d = node - x,
 * and Kirchhoff stress tau per material (stable neo-Hookean of Appendix D.2,
 * fixed corotated, von Mises/Hencky with return mapping, weakly compressible
 * fluid with F -> J^(1/3) I). The reverse-mode adjoint (Appendix D,
 * "simulation gradient" chain) maps cotangents of the final state to
 * cotangents of the initial state and of each environment's parameters; the
 * forward is recomputed from checkpoints (Section 5.1, gradient
 * checkpointing).
 *
 * Domain and grid. Each environment lives in the unit cube [0,1]^3 on n^3
 * nodes at i/n (n a multiple of 4, n >= 12). Particles must stay in the
 * stencil band 0.5/n <= x < (n - 1.5)/n on every axis; a particle outside is
 * clamped to the band and reported as MPM_OUT_OF_DOMAIN.
 *
 * Conventions for every call:
 *  - Return value is a status code (MPM_OK = 0 or one of the codes below);
 *    no C++ exception crosses this interface. mpm_last_error() gives text.
 *  - Particle arrays are row-major float32, array-of-structs: x and v are
 *    [n, 3], C and F are [n, 3, 3]. Unless stated otherwise they are DEVICE
 *    pointers on the batch's device, owned by the caller, read or written
 *    only during the call's stream work; the library keeps no pointer.
 *  - All device work is enqueued on the stream given at creation (a
 *    hipStream_t, NULL = the legacy default stream). Calls return once work
 *    is enqueued; mpm_sync() waits for it and reports device-side errors
 *    (non-finite state, particles out of the band).
 *  - One batch is used by one host thread at a time.
 */
#ifndef MPM_H_
#define MPM_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define MPM_OK 0
#define MPM_INVALID_ARG 1    /* null pointer, env index, n, nu outside (-1, 0.5), E < 0, dt <= 0, ... */
#define MPM_OUT_OF_MEMORY 2  /* the allocator failed */
#define MPM_DEVICE_ERROR 3   /* a HIP call failed */
#define MPM_NONFINITE 4      /* a NaN/Inf appeared in the particle state */
#define MPM_OUT_OF_DOMAIN 5  /* a particle left the stencil band (it was clamped) */
#define MPM_BAD_STATE 6      /* backward without a recorded forward, substeps above the maximum, ... */

/* materials (paper Appendix D.2 / D.3) */
#define MPM_NEOHOOKEAN 0   /* stable neo-Hookean energy, alpha = 1 + 3 mu / (4 lam) */
#define MPM_COROTATED 1    /* fixed corotated: tau = 2 mu (F - R) F^T + lam J (J - 1) I */
#define MPM_VONMISES 2     /* Hencky elasticity + von Mises return mapping */
#define MPM_FLUID_TAIT 3   /* tau = -J K (J^-gamma - 1) I, F projected to J^(1/3) I */
#define MPM_FLUID_PAPER 4  /* tau = lam J (J - 1) I, F projected to J^(1/3) I */

/* execution modes */
#define MPM_MODE_PLAIN 0    /* per environment: its own launches, one thread per particle, global atomics */
#define MPM_MODE_BATCHED 1  /* every environment in one launch per kernel, LDS-staged scatter, hipGraph */

/* mpm_forward flags */
#define MPM_FWD_RECORD 1    /* keep checkpoints and the last segment's tape for mpm_backward */

typedef struct mpm_batch mpm_batch;

/* One environment's fixed settings. */
typedef struct {
  int32_t n;            /* grid nodes per axis: multiple of 4, >= 12 */
  int32_t material;     /* MPM_NEOHOOKEAN ... MPM_FLUID_PAPER */
  int64_t n_particles;  /* >= 0 */
  float dt;             /* substep length, > 0 */
  float gravity[3];     /* body acceleration applied on the grid */
  int32_t wall;         /* sticky wall thickness in nodes (>= 0, 2*wall + 3 <= n) */
  int32_t reserved;
} mpm_env_desc;

typedef struct {
  int32_t n_envs;              /* >= 1 */
  const mpm_env_desc* envs;    /* host array [n_envs], read during the call */
  int32_t max_substeps;        /* upper bound on n_substeps per mpm_forward */
  int32_t ckpt_every;          /* K: checkpoint (and re-sort) interval in substeps, >= 1 */
  int32_t mode;                /* MPM_MODE_PLAIN or MPM_MODE_BATCHED */
  int32_t reserved;
} mpm_batch_desc;

/* Optional device-memory provider. alloc returns a device pointer aligned to
 * at least 256 bytes, or NULL on failure; free releases it. Both are called
 * from the host thread that calls into the library. NULL = hipMalloc/hipFree. */
typedef struct {
  void* (*alloc)(size_t bytes, void* ctx);
  void (*free)(void* ptr, void* ctx);
  void* ctx;
} mpm_allocator;

/* Creates a batch: allocates the particle state, checkpoints, the tape of one
 * segment and the grids (through `alloc` if given), on the current device.
 * `stream` is a hipStream_t. Parameters start as E = 0 (inert); set them with
 * mpm_set_material. Errors: INVALID_ARG, OUT_OF_MEMORY, DEVICE_ERROR. */
int mpm_batch_create(const mpm_batch_desc* desc, const mpm_allocator* alloc, void* stream, mpm_batch** out);

/* Waits for the batch's stream, frees all memory, destroys the handle. */
int mpm_batch_destroy(mpm_batch* b);

/* Copies particle state in (device pointers, AoS layout above). env >= 0 sets
 * that environment (n must equal its n_particles); env = -1 sets every
 * environment from arrays concatenated in env order (n = total of the
 * current counts). The clock of each environment set (the substep count that
 * places its collider in time) restarts at t = 0; other environments keep
 * theirs. Any recorded tape is dropped. */
int mpm_set_particles(mpm_batch* b, int32_t env, const float* x, const float* v, const float* C, const float* F,
                      int64_t n);

/* Copies the current particle state (x, v, C, F of Appendix D.3's particles)
 * out in the caller's original particle order (device pointers; any of the
 * four may be NULL to skip it). env = -1
 * writes all environments concatenated. The library holds F as F - I (small
 * strains keep FP32 precision relative to themselves); a set/get round trip
 * returns F unchanged for diagonal entries in [0.5, 2], where F - I is exact. */
int mpm_get_particles(mpm_batch* b, int32_t env, float* x, float* v, float* C, float* F);

/* Material and parameters of one environment (env = -1: all). `params` is a
 * HOST array of 8 doubles: E, nu, rho, Vp (particle volume), sigma_y, K
 * (Tait bulk modulus), gamma (Tait exponent), reserved. Lame parameters are
 * derived on the device (mu = E / (2 (1 + nu)), lam = E nu / ((1 + nu)(1 - 2 nu))).
 * Errors: INVALID_ARG for an unknown material, nu outside (-1, 0.5), E, rho or
 * Vp negative, gamma <= 0 for a Tait fluid. */
int mpm_set_material(mpm_batch* b, int32_t env, int32_t material, const double params[8]);

/* One-way coupled kinematic box for env (paper Appendix D.3, softened contact
 * after PlasticineLab): centre c(t) = center + t vel, half extents `half`,
 * contact strength s = min(exp(-alpha d), 1) for the node's signed distance
 * d, Coulomb friction mu_b on the velocity relative to the box. Host arrays.
 * alpha <= 0 removes the collider. */
int mpm_set_box_collider(mpm_batch* b, int32_t env, const float center[3], const float half[3], const float vel[3],
                         float alpha, float mu_b);

/* The same contact with a ball of radius `radius` about the centre instead of
 * a box (Appendix D.3's softened contact takes the collider's signed distance
 * and normal: d = |x - c| - radius, n = (x - c) / |x - c|, +z at the centre).
 * The rotation, the prescribed motion and the gradients below apply to it as
 * to the box: the ball's angle moves nothing, its spin moves its surface.
 * Errors: those of mpm_set_box_collider, INVALID_ARG for a negative or
 * non-finite radius. */
int mpm_set_sphere_collider(mpm_batch* b, int32_t env, const float center[3], float radius, const float vel[3],
                            float alpha, float mu_b);

/* The box of mpm_set_box_collider rounded by `radius`: its signed distance
 * less the radius, its normal unchanged (the contact of Appendix D.3 needs
 * only the two). half = (h, 0, 0) gives a capsule, a segment of half length h
 * along the box's own x axis inflated by the radius (a finger or a rod); the
 * rotation, motion and gradients below apply as to the box. Errors: those of
 * mpm_set_box_collider, INVALID_ARG for a negative or non-finite radius. */
int mpm_set_rounded_box_collider(mpm_batch* b, int32_t env, const float center[3], const float half[3], float radius,
                                 const float vel[3], float alpha, float mu_b);

/* Lets env's box (env = -1: every env's) rotate about a fixed axis through its
 * centre: the tools and hands of the paper's manipulation tasks turn as well
 * as translate (Section 5 task descriptions; contact of Appendix D.3). The box
 * is axis-aligned in its own frame, turned by `angle` (rad) about the unit
 * `axis` (HOST [3], normalized here) at t = 0 and spinning at `omega` (rad/s):
 * a node's distance and normal are taken in the box's frame, and the box
 * surface at a node x moves at vel + omega axis x (x - c). Call after
 * mpm_set_box_collider (which resets the rotation to none); clears any
 * prescribed motion. Errors: INVALID_ARG (no collider, zero axis, non-finite). */
int mpm_set_box_rotation(mpm_batch* b, int32_t env, const float axis[3], float angle, float omega);

/* Drives env's box collider by per-substep velocities and angular speeds
 * instead of its constant ones: the actions of the paper's manipulation tasks
 * move rigid bodies through the scene (Section 5 task descriptions; contact
 * of Appendix D.3). vel is a HOST array [n][3] (m/s), omega a HOST array [n]
 * (rad/s) or NULL (the box's constant angular speed): during substep k
 * (counted from the last mpm_set_particles of this env) the box moves at
 * vel[k] and spins at omega[k], its centre is center + dt sum_{j<k} vel[j] and
 * its angle angle0 + dt sum_{j<k} omega[j], with `center` as given to
 * mpm_set_box_collider and angle0 to mpm_set_box_rotation (accumulated in
 * FP64, stored as FP32). n = 0 (or vel = NULL) returns to the constant
 * motion. A forward past substep n - 1 fails with INVALID_ARG. Setting the
 * collider or its rotation again clears the motion. Copies the arrays;
 * synchronizes the stream. Errors: INVALID_ARG (env out of range, n outside
 * [0, max_substeps], no collider), NONFINITE. */
int mpm_set_collider_motion(mpm_batch* b, int32_t env, const float* vel, const float* omega, int32_t n);

/* After mpm_backward: cotangents of the loss with respect to env's collider
 * velocities, starting centre, angular speeds and starting angle. dvel: HOST
 * [n][3] doubles (n <= the motion length), dc0: HOST [3], domega: HOST [n],
 * dangle0: HOST [1]; any may be NULL. Includes every path: an action's direct
 * part in the contact and its effect on all later centres or angles (dt
 * each). Synchronizes the stream. Errors: BAD_STATE if env has no prescribed
 * motion, INVALID_ARG. */
int mpm_get_collider_grad(mpm_batch* b, int32_t env, double* dvel, double* dc0, double* domega, double* dangle0,
                          int32_t n);

/* Several colliders per environment (paper Section 5: a hand or a gripper is
 * several rigid bodies; Appendix D.3's contact applies to each). An env holds
 * up to MPM_MAX_COLLIDERS colliders; the grid update applies them in index
 * order, each one's blended velocity the next one's input. The functions
 * above address collider 0; those below take its index. A removed collider
 * (alpha <= 0) is skipped. */
#define MPM_MAX_COLLIDERS 4
#define MPM_COLLIDER_BOX 1           /* shapes of mpm_set_collider */
#define MPM_COLLIDER_SPHERE 2
#define MPM_COLLIDER_ROUNDED_BOX 3

/* Collider `index` of env (env = -1: all) as mpm_set_box_collider (shape
 * MPM_COLLIDER_BOX; radius ignored), mpm_set_sphere_collider (SPHERE; half
 * ignored, may be NULL) or mpm_set_rounded_box_collider (ROUNDED_BOX).
 * Errors: those of those functions, INVALID_ARG for an index outside
 * [0, MPM_MAX_COLLIDERS) or an unknown shape. */
int mpm_set_collider(mpm_batch* b, int32_t env, int32_t index, int32_t shape, const float center[3],
                     const float half[3], float radius, const float vel[3], float alpha, float mu_b);

/* mpm_set_box_rotation for collider `index`. */
int mpm_set_collider_rotation(mpm_batch* b, int32_t env, int32_t index, const float axis[3], float angle,
                              float omega);

/* mpm_set_collider_motion for collider `index` (each collider keeps its own
 * motion; a forward fails if any is shorter than the rollout). */
int mpm_set_collider_motion_at(mpm_batch* b, int32_t env, int32_t index, const float* vel, const float* omega,
                               int32_t n);

/* mpm_get_collider_grad for collider `index`. */
int mpm_get_collider_grad_at(mpm_batch* b, int32_t env, int32_t index, double* dvel, double* dc0, double* domega,
                             double* dangle0, int32_t n);

#define MPM_MOMENTS 20   /* stride of one env's moments */

/* Per-env weighted moments of particle positions and velocities: the
 * statistics the manipulation tasks observe and reward (centre of mass of a
 * subsampled particle set, variance of its heights, mean velocity; paper
 * Appendix E task definitions). x, v: DEVICE arrays [rows][3] in the caller's
 * concatenated env order (as mpm_get_particles writes them); w: DEVICE [rows]
 * weights, NULL for all ones (a 0/1 pattern selects a subsample). out: DEVICE
 * [n_envs][MPM_MOMENTS] doubles, per env: [0] sum w, [1..3] sum w x,
 * [4..9] sum w (xx, yy, zz, xy, xz, yz), [10..12] sum w v, [13..18] the same
 * products of v, [19] 0. Accumulated in FP64; asynchronous on the stream.
 * Errors: INVALID_ARG for a null x, v or out. */
int mpm_moments(mpm_batch* b, const float* x, const float* v, const float* w, double* out);

/* VJP of mpm_moments: gout DEVICE [n_envs][MPM_MOMENTS] cotangents -> gx, gv
 * DEVICE [rows][3] (written, not added; either may be NULL). Same x, v, w as
 * the forward. Asynchronous on the stream. */
int mpm_moments_vjp(mpm_batch* b, const float* x, const float* v, const float* w, const double* gout, float* gx,
                    float* gv);

/* The flip reward term of the HandFlip task (paper Appendix E): per env e, the
 * mean Euclidean distance between paired particles,
 *   R_e = (1 / P_e) sum_k ||x[a_k] - x[b_k]||_2
 * over the P_e pairs of env e (the two mirrored halves of the particles, paired
 * particle by particle). pairs: DEVICE int32 [n_pairs][3] rows (env, a, b)
 * with a, b env-local caller indices; a pair naming an env or a particle out of
 * range is skipped. x: DEVICE caller-order positions [rows][3]. out: DEVICE
 * [n_envs][2] doubles: [e][0] = R_e (0 for an env without pairs), [e][1] = P_e.
 * Distances in FP32, sums in FP64; asynchronous on the stream.
 * Errors: INVALID_ARG for a null array or n_pairs < 0. */
int mpm_pair_distance(mpm_batch* b, const float* x, const int32_t* pairs, int64_t n_pairs, double* out);

/* VJP of mpm_pair_distance: gout DEVICE [n_envs] cotangents of R_e, out the
 * forward's output (for P_e) -> gx DEVICE [rows][3] (written, not added):
 * dR_e/dx[a_k] = (x[a_k] - x[b_k]) / (P_e ||x[a_k] - x[b_k]||), the opposite
 * for x[b_k], summed over the pairs a particle belongs to; a pair at zero
 * distance contributes 0. Asynchronous on the stream. */
int mpm_pair_distance_vjp(mpm_batch* b, const float* x, const int32_t* pairs, int64_t n_pairs, const double* out,
                          const double* gout, float* gx);

/* Advances every environment by n_substeps (0 <= n <= max_substeps) of the
 * MLS-MPM substep above (paper Appendix D.3) from the current state and
 * clocks. Particles are re-sorted by cell at every checkpoint. With MPM_FWD_RECORD the checkpoints (every ckpt_every substeps)
 * and the last segment's states and grids are kept for mpm_backward;
 * otherwise any earlier record is dropped. Asynchronous on the stream. */
int mpm_forward(mpm_batch* b, int32_t n_substeps, int32_t flags);

/* Like mpm_forward, but environment e takes n_substeps[e] substeps (HOST
 * array [n_envs], each in [0, max_substeps]); once an environment has taken
 * its substeps it is frozen -- its state passes through unchanged, and in the
 * backward its cotangent passes through unchanged -- while the others run on.
 * The continuous-batching server advances slots by different amounts with it. */
int mpm_forward_envs(mpm_batch* b, const int32_t* n_substeps, int32_t flags);

/* Re-describes environment `env` in place (a serving slot): grid n up to the
 * n it was created with, n_particles up to its created count (its capacity),
 * and any material, dt, gravity, wall. Its collider is removed; set its
 * material and particles (mpm_set_material, mpm_set_particles with this
 * env's new count) before the next forward. The rows of every env=-1 array
 * become the concatenation of the current counts. Drops any record; cached
 * graphs stay valid. Errors: INVALID_ARG above capacity. */
int mpm_configure_env(mpm_batch* b, int32_t env, const mpm_env_desc* d);

/* Reverse-mode adjoint of the last recorded mpm_forward: the vector-Jacobian
 * product of the substep map s_{k+1} = f(s_k; params) composed over the
 * recorded substeps (paper Appendix D, the chain that carries simulation
 * gradients back through the states; Section 5.1, gradient checkpointing with
 * forward recomputation). Inputs: cotangents of the final state (device, AoS
 * over all environments in original order; NULL = zero). Outputs: cotangents
 * of the state at the start of that forward (device, same layout; NULL = not
 * wanted) and, if dparams != NULL, a DEVICE array [n_envs][8] of doubles
 * receiving dL/d(E, nu, rho, Vp, sigma_y, K, gamma, 0). dL/drho comes from the
 * scale invariance of the substep (it depends on the parameters only through
 * tau / rho): rho dL/drho = -(E dL/dE + sigma_y dL/dsigma_y + K dL/dK), and
 * dL/dVp = 0 exactly (Vp cancels between particle mass and force). Segments are
 * recomputed from checkpoints. The record stays valid (backward may be called
 * again with other cotangents).
 * Errors: BAD_STATE if no recorded forward precedes. */
int mpm_backward(mpm_batch* b, const float* gx, const float* gv, const float* gC, const float* gF, float* dx0,
                 float* dv0, float* dC0, float* dF0, double* dparams);

/* Execution options (mpm_set_option / mpm_get_option). Changing a kernel
 * variant drops the cached graphs. */
#define MPM_OPT_GRAPHS 1       /* 1: replay each segment as a hipGraph (batched mode only; default 1) */
#define MPM_OPT_P2G 2          /* P2G variant: 0 global atomics, 1 LDS-staged, 2 LDS + per-cell runs (default),
                                  3 LDS pull: each LDS box node summed by its owner thread from the block's
                                  particles (counting-sorted by cell in LDS), no LDS float atomics */
#define MPM_OPT_G2P 3          /* G2P variant: 0 global gathers, 1 LDS-staged (default) */
#define MPM_OPT_G2P_ADJ 4      /* G2P adjoint: 0 global atomics, 1 LDS-staged, 2 LDS + per-cell runs (default),
                                  3 LDS pull (as MPM_OPT_P2G = 3) */
#define MPM_OPT_P2G_ADJ 5      /* P2G adjoint: 0 global gathers, 1 LDS-staged (default) */
#define MPM_OPT_MIN_RUN 6      /* per-cell-run variants engage when particles per stencil base >= this (default 3) */
#define MPM_OPT_GRID_CAP 7     /* LDS-staged kernels: 0 = one block per work item (default); > 0 = a persistent
                                  grid of this many blocks striding over the work items */
#define MPM_OPT_MAX_RUN 8      /* per-cell-run variants cut a run of one stencil base every this many particles
                                  (default 8) */
#define MPM_OPT_BOX 9          /* LDS-staged kernels' box budget: 0 = 1024 grid nodes per block (default),
                                  1 = 384 nodes (less LDS, more blocks per CU; a block whose box is larger
                                  falls back to global atomics) */
#define MPM_OPT_FUSE 11        /* 1: within a segment, G2P of substep k and the P2G of substep k + 1 run as
                                  one kernel (the new state is scattered from registers); needs
                                  MPM_OPT_P2G = 2 (per-cell runs) or 3 (pull), otherwise ignored. Default 0;
                                  the autotuner may set it */
#define MPM_OPT_FUSE_ADJ 12    /* 1: within a segment's backward, the P2G adjoint of substep k and the G2P
                                  adjoint of substep k - 1 run as one kernel (the cotangent of state k stays
                                  in registers; the G2P adjoint part is the pull scatter when
                                  MPM_OPT_G2P_ADJ = 3, else the segment-reduced one). Batched mode.
                                  Default 0; the autotuner may set it */
#define MPM_OPT_XCD 13         /* LDS-staged kernels: 1 = each launch's work items are ordered so that the
                                  blocks one XCD receives (block i goes to XCD i mod 8) take a contiguous
                                  run of items, keeping an env's grid lines in one XCD's L2; 0 = item
                                  order (default). Results are the same up to float summation order; the
                                  autotuner may set it */
#define MPM_OPT_GRID_LIST 14   /* 1 (2): the grid update and its adjoint take 64 (16) tiles per block, find the
                                  flagged ones with one wave ballot and run only those, instead of one
                                  block per 4 tiles of the whole grid (fewer, busier blocks when few tiles
                                  are flagged). Batched mode. Default 0; the autotuner may set it */
#define MPM_OPT_SPECIALIZE 10  /* LDS-staged kernels: 1 = one launch per material over that material's work items,
                                  compiled for it (default); 0 = one launch over all items, material read at run time */

/* Sets one option; INVALID_ARG for an unknown option or value. */
int mpm_set_option(mpm_batch* b, int32_t option, int32_t value);
/* Reads one option into the host int *value. */
int mpm_get_option(mpm_batch* b, int32_t option, int32_t* value);

/* Autotuner (batched mode). Runs ckpt_every substeps from the current state
 * with every kernel variant (MPM_OPT_P2G, _G2P, _G2P_ADJ, _P2G_ADJ, _MIN_RUN,
 * _BOX, _SPECIALIZE, _FUSE, _FUSE_ADJ, _XCD, _GRID_CAP, _MAX_RUN), one option
 * at a time. A candidate is kept only if its end
 * state (x, v: relative error <= 1e-5) and its initial-state cotangent for an
 * all-ones loss cotangent (<= 1e-4) agree with the one-thread-per-particle
 * kernels; the fastest kept candidate wins, a later one only if it is more
 * than 1% faster than the choice so far. Stops trying further candidates
 * after about budget_ms milliseconds. Restores the particle state and clock,
 * drops any record, synchronizes the stream; the choice is cached per batch
 * shape for the process. Plain mode: no-op. */
int mpm_autotune(mpm_batch* b, int32_t budget_ms);

/* Binning of the current state without changing it (the paper is silent on
 * binning; the key orders particles by env, 4^3-node tile and stencil base
 * cell). Writes, as DEVICE arrays over the current internal particle order:
 * keys[i] = (env << cell_bits) | (tile * 64 + cell) with base clamped to
 * [0, n-3], tile = ((bx/4) T + by/4) T + bz/4, T = n/4, cell =
 * ((bx%4) 4 + by%4) 4 + bz%4, cell_bits = ceil(log2(max n^3)) (uint32 [N]);
 * perm, the stable sort order (new
 * position j takes internal position perm[j], uint32 [N]); ids, the
 * env-local caller index of each internal position, -1 where a slot's
 * capacity holds no particle (int32 [N]). N counts capacity positions.
 * *cell_bits is a host int.
 * Any output pointer may be NULL. */
int mpm_sort_keys(mpm_batch* b, uint32_t* keys, uint32_t* perm, int32_t* ids, int32_t* cell_bits);

/* For callers that cannot allocate device memory (code under stream or graph
 * capture, serving loops, harnesses that forbid allocation): the binning of
 * mpm_sort_keys for one environment, with no batch and no allocation. x:
 * DEVICE positions [n][3] (AoS float32) of one environment on a grid_n^3 grid;
 * writes keys[i] = tile * 64 + cell of particle i (as mpm_sort_keys writes for
 * env 0 of a batch) and perm, the stable sort order (DEVICE uint32 [n] each),
 * asynchronously on `stream` (a hipStream_t). Its scratch is a device array of
 * the library sized for MPM_SORT_NOALLOC_MAX particles, one per GPU, held
 * until the process ends; calls that overlap on one GPU share it and race.
 * Errors: INVALID_ARG for n < 0 or n > MPM_SORT_NOALLOC_MAX, a grid_n that
 * mpm_env_desc would reject, or a null array; DEVICE_ERROR. */
#define MPM_SORT_NOALLOC_MAX (1 << 20)
int mpm_sort_keys_noalloc(const float* x, int64_t n, int32_t grid_n, uint32_t* keys, uint32_t* perm, void* stream);

/* Waits for the stream and returns the first pending device-side error
 * (MPM_NONFINITE / MPM_OUT_OF_DOMAIN) or MPM_OK; clears it. */
int mpm_sync(mpm_batch* b);

/* Per-environment error bits of the last mpm_sync (1: non-finite, 2: out of
 * the band) into the host array errs[n_envs]. */
int mpm_env_errors(mpm_batch* b, int32_t* errs);

/* Device bytes held by the batch. */
int64_t mpm_memory_bytes(const mpm_batch* b);

/* Mean duration in milliseconds of the named kernel class over the last
 * mpm_forward / mpm_backward when timing is enabled (see mpm_set_timing).
 * kernel: 0 P2G, 1 grid update, 2 G2P, 3 sort+permute, 4 G2P adjoint,
 * 5 grid adjoint, 6 P2G adjoint, 7 fused G2P + next P2G (MPM_OPT_FUSE),
 * 8 fused P2G adjoint + previous G2P adjoint (MPM_OPT_FUSE_ADJ).
 * Returns the number of launches timed. */
int mpm_kernel_time(mpm_batch* b, int32_t kernel, double* mean_ms);
int mpm_set_timing(mpm_batch* b, int32_t enabled);

/* Text of the last error on this batch ("" if none); a static string if b is NULL. */
const char* mpm_last_error(const mpm_batch* b);

/* ------------------------------------------------------------------------
 * Serving: continuous batching of rollout requests over one batch of slots.
 *
 * A request is one environment: its description, material and optional box
 * collider, an initial state, a number of substeps S and, optionally, a
 * backward pass from cotangents of its final state to cotangents of its
 * initial state and parameters -- the rollout and its gradient that the
 * paper's first-order learner asks of the simulator for each environment
 * (Section 5.1: parallel differentiable simulation with gradient
 * checkpointing; Appendix D: the gradient chain through the substeps). The
 * server owns a batch whose environments are slots of a fixed capacity (grid
 * n_cap^3, n_cap_particles particles) and admits requests by an HBM budget:
 *  - requests queue in arrival order; the head is admitted when a slot is free
 *    and the bytes it keeps on the device (its state, grid share, and for a
 *    backward its chunk checkpoints and running cotangent) fit in the budget;
 *  - each mpm_server_step advances every slot in its forward phase by one
 *    chunk of substeps in ONE batched forward, then moves every slot in its
 *    backward phase one chunk back in ONE recorded forward + backward over
 *    those slots: a chunk's forward is recomputed from the checkpoint taken
 *    before it (internal state and collider clock), the running cotangent
 *    goes through it, and the parameter cotangents of the chunks are summed
 *    in FP64. Requests that arrive while others run join at the next step and
 *    share the same kernel launches;
 *  - a finished request frees its slot and budget at once; a request whose
 *    environment reports a device error (non-finite state, a particle out of
 *    the band) fails alone.
 * One server is used by one host thread at a time. Calls that return results
 * synchronize the server's stream.
 * ------------------------------------------------------------------------ */
typedef struct mpm_server mpm_server;

typedef struct {
  int32_t n_slots;          /* environments of the batch (concurrent requests), >= 1 */
  int32_t n_cap;            /* grid capacity per slot (nodes per axis, multiple of 4, >= 12) */
  int64_t n_cap_particles;  /* particle capacity per slot, >= 1 */
  int32_t chunk;            /* substeps per engine step and checkpoint interval, >= 1 */
  int32_t flags;            /* MPM_SERVER_DRY: schedule only, no device work (host-logic tests) */
  int64_t budget_bytes;     /* device bytes the admitted requests may keep resident */
} mpm_server_desc;

#define MPM_SERVER_DRY 1

/* a further collider of a request (as mpm_set_collider: shape MPM_COLLIDER_*,
 * radius of a SPHERE or ROUNDED_BOX) */
typedef struct {
  int32_t shape;
  float center[3], half[3], radius, vel[3], alpha, mu_b;
} mpm_collider;

typedef struct {
  mpm_env_desc env;        /* n <= n_cap, n_particles <= n_cap_particles, material */
  double params[8];        /* as mpm_set_material */
  int32_t has_collider;    /* 1: the box below (as mpm_set_box_collider); 2: a ball of radius c_half[0];
                              3: the box rounded by c_round (as mpm_set_rounded_box_collider) */
  int32_t substeps;        /* S >= 1 */
  float c_center[3], c_half[3], c_vel[3], c_alpha, c_mu;
  int32_t backward;        /* 1: run the backward pass after the forward */
  float c_round;           /* rounding radius of a has_collider = 3 box */
  double arrival;          /* seconds on the server clock (mpm_server_now); < 0 = at submission */
  /* DEVICE arrays owned by the caller, AoS as for mpm_set_particles; they must
   * stay valid and unchanged until the request reaches a final state. */
  const float *x, *v, *C, *F;        /* initial state, read at admission */
  const float *gx, *gv, *gC, *gF;    /* cotangents of the final state (backward; NULL = 0), read when it starts */
  float *out_x, *out_v, *out_C, *out_F;  /* final state, written when the forward ends (NULL = not wanted) */
  float *dx0, *dv0, *dC0, *dF0;          /* initial-state cotangents, written when the backward ends (NULL = skip) */
  int32_t n_more;                        /* further colliders, 0 .. MPM_MAX_COLLIDERS - 1, applied after the one
                                            above (slots 1 ..), held by value */
  mpm_collider more[MPM_MAX_COLLIDERS - 1];
} mpm_request;

/* request states */
#define MPM_REQ_QUEUED 0
#define MPM_REQ_RUNNING 1
#define MPM_REQ_DONE 2
#define MPM_REQ_ERROR 3      /* a device error in its environment; error_bits says which */
#define MPM_REQ_CANCELLED 4
#define MPM_REQ_REJECTED 5   /* above the slot capacity or the whole budget */
#define MPM_REQ_UNKNOWN 6    /* no such id, or its final state was already polled */

typedef struct {
  int32_t state;            /* MPM_REQ_* */
  int32_t error_bits;       /* 1 non-finite, 2 out of the band */
  double arrival, admitted, finished;   /* server-clock seconds (0 if not reached) */
  double dparams[8];        /* dL/d(E, nu, rho, Vp, sigma_y, K, gamma, 0), FP64 sum over the chunks */
} mpm_request_status;

typedef struct {
  int64_t submitted, done, errors, cancelled, rejected, queued, running;
  int64_t particle_substeps;   /* sum of N S over requests finished ok (each counted once, with or without a
                                  backward) */
  int64_t steps;               /* engine steps taken */
  int32_t max_running;         /* most requests admitted at once */
  int32_t reserved;
  int64_t bytes_in_use;        /* budget taken by the admitted requests */
  double p50_ms, p99_ms;       /* arrival-to-finish latency of the requests finished ok */
  double first_arrival, last_finish;   /* server-clock seconds */
} mpm_server_stats;

/* Creates a server and its batch of n_slots slots (device memory through
 * `alloc` if given, work on `stream`). Errors: INVALID_ARG, OUT_OF_MEMORY,
 * DEVICE_ERROR. */
int mpm_server_create(const mpm_server_desc* desc, const mpm_allocator* alloc, void* stream, mpm_server** out);

/* Waits for the stream, frees everything; requests still queued or running are dropped. */
int mpm_server_destroy(mpm_server* s);

/* Queues a request (copies the struct; the arrays stay the caller's). *id
 * receives its id. A request above the slot capacity or the whole budget is
 * recorded as MPM_REQ_REJECTED. Errors: INVALID_ARG (null state arrays,
 * S < 1, an unknown material, nu outside (-1, 0.5)). */
int mpm_server_submit(mpm_server* s, const mpm_request* r, int64_t* id);

/* One engine step: admit, one forward chunk, one backward chunk, wait for the
 * device, retire finished requests. Returns MPM_OK or the error of a failed
 * device call (failures of single environments only fail their requests). */
int mpm_server_step(mpm_server* s);

/* State of request `id` (host *st). A final state (DONE, ERROR, CANCELLED,
 * REJECTED) is reported once; the record is then dropped. */
int mpm_server_poll(mpm_server* s, int64_t id, mpm_request_status* st);

/* Cancels a queued or running request (its slot and budget are freed at
 * once). Returns INVALID_ARG if it is not queued or running. */
int mpm_server_cancel(mpm_server* s, int64_t id);

/* Seconds since the server was created (its clock for arrivals). */
double mpm_server_now(const mpm_server* s);

/* 1 if no request is queued or running, else 0. */
int mpm_server_idle(const mpm_server* s);

/* Counters and latency percentiles into the host struct *st. */
int mpm_server_stats_get(mpm_server* s, mpm_server_stats* st);

/* Text of the server's last error. */
const char* mpm_server_last_error(const mpm_server* s);

/* Library version string. */
const char* mpm_version(void);

#ifdef __cplusplus
}
#endif
#endif /* MPM_H_ */
