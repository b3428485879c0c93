/*
 * mpm_rb.h -- C interface of the batched, differentiable articulated
 * rigid-body step of the same library (libmpmx.so), for MI355X (gfx950).
 *
 * What it computes (paper: Appendix D.1 "Composite rigid body algorithm").
 * Every environment of a batch is one tree of rigid links joined by revolute
 * or prismatic joints on a fixed base (shared links; states, torques and parameters per
 * environment). One substep, per environment:
 *   M(q) qdd = tau - c(q, qd) - damp qd + J^T f_contact
 *   qd' = qd + dt qdd,  q' = q + dt qd'                  (semi-implicit Euler)
 * M is the joint-space mass matrix (composite rigid body algorithm), c the
 * Coriolis, centrifugal and gravity terms (recursive Newton-Euler with the
 * base accelerating against gravity), damp a viscous joint damping, and
 * f_contact the ground's penalty force on contact spheres fixed to the links:
 * at the lowest point x of a sphere while x_z < z_g,
 *   f = (-k_f v_x, -k_f v_y, k_e (z_g - x_z) - k_d v_z),
 * v the velocity of the link's material point at x. qdd comes from a Cholesky
 * factorisation of M ordered leaves first (M = L^T L, with no fill-in on a
 * tree). The reverse-mode adjoint maps cotangents of the final
 * (q, qd) to cotangents of the initial (q, qd), of every substep's torques and
 * of each environment's parameters (Appendix D's simulation-gradient chain):
 * per substep lambda = M^-1 qdd_bar is the torque cotangent, and the state
 * cotangents take -d/d(q, qd) of lambda . ID(q, qd, qdd) with qdd held, ID the
 * inverse dynamics (implicit-function rule).
 *
 * Kinematics: link i's frame is its joint frame, placed in the parent link's
 * frame (the world's for a root) by a fixed rotation joint_rot and offset
 * joint_pos, turned by q_i about the unit joint axis (joint-frame
 * coordinates): R_i = R_parent joint_rot_i Rot(axis_i, q_i),
 * p_i = p_parent + R_parent joint_pos_i; a prismatic joint slides the link
 * by q_i along the axis instead: R_i = R_parent joint_rot_i,
 * p_i = p_parent + R_parent (joint_pos_i + q_i joint_rot_i axis_i).
 *
 * Conventions are those of mpm.h: status codes, device pointers owned by the
 * caller and used only during the call's stream work, asynchronous calls on
 * the stream given at creation, one host thread per handle. Joint arrays are
 * float32 [n_envs][n_links], row-major.
 */
#ifndef MPM_RB_H_
#define MPM_RB_H_

#include "mpm.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mpm_rb mpm_rb;

#define MPM_RB_MAX_LINKS 64       /* links (joints) per environment */
#define MPM_RB_MAX_CONTACTS 256   /* contact spheres per environment */
#define MPM_RB_PARAMS 5           /* per-env parameter row: damp, k_e, k_d, k_f, z_g */

#define MPM_RB_REVOLUTE 0         /* joint kinds (mpm_rb_link.joint) */
#define MPM_RB_PRISMATIC 1

typedef struct {
  int32_t n_envs;        /* >= 1 */
  int32_t n_links;       /* 1 .. MPM_RB_MAX_LINKS */
  int32_t n_contacts;    /* 0 .. MPM_RB_MAX_CONTACTS */
  int32_t max_substeps;  /* >= 0: substeps a recorded forward can keep for the backward */
  float dt;              /* substep length, > 0 */
  float gravity[3];      /* acceleration of gravity */
  int32_t reserved[4];
} mpm_rb_desc;

typedef struct {
  int32_t parent;        /* -1 (the world) or a lower link index */
  float joint_rot[9];    /* joint frame in the parent frame, row-major, orthonormal, det +1 */
  float joint_pos[3];    /* joint origin in the parent frame */
  float axis[3];         /* joint axis in the joint frame, unit length */
  float mass;            /* >= 0 */
  float com[3];          /* centre of mass in the link frame */
  float inertia[6];      /* rotational inertia about the centre of mass, link frame: xx yy zz xy xz yz */
  int32_t joint;         /* MPM_RB_REVOLUTE (0: q is an angle) or MPM_RB_PRISMATIC (q is a length) */
} mpm_rb_link;

typedef struct {
  int32_t link;          /* link the sphere is fixed to */
  float centre[3];       /* in the link frame */
  float radius;          /* >= 0 */
} mpm_rb_contact;

/* Creates a rigid-body batch on the current device from HOST arrays of
 * n_links links (link 0 a root; every parent index lower than its child's)
 * and n_contacts contact spheres, read during the call. Allocates the states,
 * the tape of max_substeps + 1 states and max_substeps torques, and the model
 * (through `alloc` if given; see mpm.h). `stream` is a hipStream_t.
 * Parameters start with no damping and no ground (z_g = -inf); states at 0.
 * Errors: INVALID_ARG (sizes, a parent index out of order, a non-unit axis,
 * a joint_rot that is not a rotation to 1e-4, an unknown joint kind, a
 * negative mass or radius, a contact on no link), OUT_OF_MEMORY, DEVICE_ERROR. */
int mpm_rb_create(const mpm_rb_desc* desc, const mpm_rb_link* links, const mpm_rb_contact* contacts,
                  const mpm_allocator* alloc, void* stream, mpm_rb** out);

/* Waits for the stream, frees all memory, destroys the handle. */
int mpm_rb_destroy(mpm_rb* r);

/* Per-env parameters, a HOST array [n_envs][MPM_RB_PARAMS] of doubles: joint
 * damping damp (>= 0) and the ground's k_e, k_d, k_f (>= 0) and height z_g
 * (-inf: no ground). Drops any record. Errors: INVALID_ARG. */
int mpm_rb_set_params(mpm_rb* r, const double* params);

/* Copies the state in (q, qd device [n_envs][n_links]; qd NULL = zero).
 * Drops any record. */
int mpm_rb_set_state(mpm_rb* r, const float* q, const float* qd);

/* Copies the current state out (either pointer may be NULL). */
int mpm_rb_get_state(mpm_rb* r, float* q, float* qd);

/* Runs S substeps (0 <= S) on every environment. tau: device
 * [S][n_envs][n_links] joint torques of each substep, or NULL (all zero).
 * flags & MPM_FWD_RECORD keeps every state and the torques for
 * mpm_rb_backward (S <= max_substeps); otherwise any record is dropped.
 * Asynchronous. Errors: INVALID_ARG, BAD_STATE (record longer than the tape). */
int mpm_rb_forward(mpm_rb* r, int32_t S, const float* tau, int32_t flags);

/* Reverse mode through the recorded forward of S substeps: given the
 * cotangents gq, gqd of its final (q, qd) (device, NULL = zero), writes the
 * cotangents of its initial (q, qd) to dq0, dqd0 (device, required), of each
 * substep's torques to dtau (device [S][n_envs][n_links], or NULL), and of the
 * parameters to dparams (device [n_envs][MPM_RB_PARAMS] doubles, or NULL).
 * The state after the call is unchanged; the record is kept. Asynchronous.
 * Errors: INVALID_ARG, BAD_STATE (no record). */
int mpm_rb_backward(mpm_rb* r, const float* gq, const float* gqd, float* dq0, float* dqd0, float* dtau,
                    double* dparams);

/* Waits for the stream; returns NONFINITE if a forward since the last call
 * produced a non-finite state in some environment (a mass matrix that is not
 * positive definite does too; mpm_rb_env_errors says which). */
int mpm_rb_sync(mpm_rb* r);

/* Per-environment error bits of the last mpm_rb_sync (1: non-finite). */
int mpm_rb_env_errors(mpm_rb* r, int32_t* errs);

/* Text of the last error on this handle. */
const char* mpm_rb_last_error(const mpm_rb* r);

/* Device bytes held by the handle. */
int64_t mpm_rb_memory_bytes(const mpm_rb* r);

#ifdef __cplusplus
}
#endif

#endif /* MPM_RB_H_ */
