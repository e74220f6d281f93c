/*
 * cfsim.h - C ABI of the MI355X complementarity-free contact step.
 *
 * The library advances batches of independent worlds by one time step of the
 * complementarity-free contact model (arXiv 2603.12185, Sec. III):
 *   v_s  = v + h M^-1 (tau - c)                         (Eq. smooth_vel)
 *   per contact k, per facet f of its polyhedral dual cone (Eqs. dual_polyhedral,
 *   tilde_defs) with rows J~ = J_n - mu_s d_f^T J_s:
 *   lambda h = A_k * max(-(k_user h + d_user) J~ v_s - k_user phi_k, 0)  (Eq. cf_wrench,
 *        with K = k_user A / h, D = d_user A / h of Eq. k_d_setting and
 *        A_k = r/(1-r) / (tr(J_a M^-1 J_a^T) + tr(J_b M^-1 J_b^T)), r of Eq. r_scaling)
 *   v+   = v_s + M^-1 sum J~^T lambda h                  (Eq. vel_correction)
 *   q+   = q (+) h v+  (semi-implicit Euler)
 * Algorithm 1 of the paper lists the same four stages; the contact set comes
 * from the library's own analytic narrow phase.
 *
 * Conventions
 *  - Quaternions (w,x,y,z).  A free joint has q = (COM position, orientation)
 *    and v = (COM linear velocity, angular velocity), both in world
 *    coordinates; a state quaternion denotes the rotation of its normalised
 *    value and is re-normalised by every step.
 *  - Contact normal n points from geom a to geom b; a plane is always geom a,
 *    and a box paired with a sphere or capsule is geom a; phi > 0 means
 *    separated; the contact point is the middle of the overlap; a contact
 *    exists when phi < margin.
 *  - Box-sphere: the sphere centre, in the box frame, clamped to the box;
 *    outside, n runs from the clamped point to the centre and phi is their
 *    distance minus the radius; inside, n is the outward axis of the face of
 *    least depth (lowest axis on ties) and phi = -depth - radius.  A capsule
 *    meets a plane or a box with its two end spheres.
 *  - Tangent basis: helper e_x if |n_x| <= 0.5 else e_y; t1 = normalised
 *    component of the helper orthogonal to n; t2 = n x t1.
 *  - Facet order per contact: tangential d = (1,0),(0,1),(-1,0),(0,-1) in
 *    (t1,t2); torsional sigma = +1,-1; rolling d as tangential.  condim 1, 3,
 *    4, 6 give 1, 4, 6, 10 facets.  Pair friction is the element-wise max of
 *    the two geoms' (mu_t, mu_tor, mu_rol).
 *  - Contact order: geom pairs (i < j) in index order, then the sub-contact
 *    index (box corner bits x,y,z = bit 0,1,2 set for +half-size; capsule
 *    minus end first).  Only the first ncon_max contacts of a world are kept
 *    and resolved; the rest are counted in overflow.
 *  - Pairs that never produce contacts: both geoms static, same body,
 *    parent-child bodies, and types other than plane-sphere, plane-capsule,
 *    plane-box, sphere-sphere, box-sphere and box-capsule (cf_model_create
 *    then returns CF_W_PAIRS_SKIPPED, a warning).
 *
 * Memory, streams and errors
 *  - Descriptor arrays are host memory, read during cf_model_create only.
 *  - State, tau and contact views are caller-owned, contiguous float32/int32
 *    DEVICE buffers on the device that was current at cf_model_create.
 *    q_out/v_out may alias q/v exactly (not partially).
 *  - All compute calls are asynchronous on the given stream (a hipStream_t;
 *    NULL = default stream) and never synchronise.  The returned status covers
 *    argument checks and launch errors; device-side conditions (contact
 *    overflow) are reported through cf_contacts.overflow.
 *  - A model is not thread-safe (it owns one contact workspace); distinct
 *    models are independent.  cf_last_error() is per thread.
 */
#ifndef CFSIM_H
#define CFSIM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CF_ABI_VERSION 3

typedef struct cf_model cf_model;
typedef int32_t cf_status;

enum {
  CF_OK = 0,
  CF_W_PAIRS_SKIPPED = 1, /* warning: some geom pairs have no contact rule     */
  CF_E_INVALID_ARG = -1,  /* bad descriptor, size, pointer or alignment        */
  CF_E_DEVICE = -2,       /* HIP runtime error (launch, copy, event)           */
  CF_E_NOMEM = -3,        /* device allocation failed                          */
  CF_E_UNSUPPORTED = -4   /* valid model outside what this library implements  */
};

enum { CF_PLANE = 0, CF_SPHERE = 1, CF_CAPSULE = 2, CF_BOX = 3 };
enum { CF_JNT_FREE = 0, CF_JNT_HINGE = 1, CF_JNT_SLIDE = 2 };
enum { CF_IMPEDANCE_HEURISTIC = 0, CF_IMPEDANCE_DIAGONAL = 1 };

/* Model description (host memory, copied at create).  nworld worlds share the
 * tree and geom types; masses, inertias and geom data may differ per world.
 * Sizes: geom sizes are (radius) for spheres, (radius, half-length along local
 * z) for capsules, half-sizes for boxes; planes use their local z as normal. */
typedef struct {
  int32_t nworld, nbody, ngeom, ncon_max, condim;  /* condim in {1,3,4,6}               */
  const int32_t *body_parent;   /* [nbody] -1 = world; must be < own index            */
  const int32_t *body_jnt;      /* [nbody] one joint per body (CF_JNT_*)              */
  const double *body_pos;       /* [nbody][3] body frame in parent frame at q = 0      */
  const double *body_quat;      /* [nbody][4]                                          */
  const double *body_ipos;      /* [nbody][3] COM in the body frame (0 for free)       */
  const double *jnt_axis;       /* [nbody][3] hinge/slide axis in the body frame       */
  const double *body_mass;      /* [nworld][nbody]                                     */
  const double *body_inertia;   /* [nworld][nbody][3] principal, about the COM         */
  const int32_t *geom_type;     /* [ngeom] CF_PLANE..CF_BOX                            */
  const int32_t *geom_body;     /* [ngeom] -1 = static                                 */
  const double *geom_size;      /* [nworld][ngeom][3]                                  */
  const double *geom_pos;       /* [nworld][ngeom][3] in the body (or world) frame     */
  const double *geom_quat;      /* [nworld][ngeom][4]                                  */
  const double *geom_friction;  /* [nworld][ngeom][3] (mu_t, mu_tor, mu_rol)           */
  double h;                     /* time step > 0                                       */
  double gravity[3];
  double k_user, d_user;        /* >= 0; k_user in 1/s, d_user dimensionless           */
  double solimp[5];             /* r_min, r_max, width, midpoint, power (Eq. r_scaling) */
  double margin;                /* contact when phi < margin                           */
} cf_model_desc;

/* Optional contact outputs of a step (device memory, caller-owned; any
 * pointer may be NULL).  Rows past ncon[w] are left untouched. */
typedef struct {
  int32_t *ncon;      /* [nworld] contacts kept                                  */
  int32_t *overflow;  /* [nworld] contacts dropped beyond ncon_max               */
  int32_t *geom;      /* [nworld][ncon_max][2] geom a, geom b                    */
  int32_t *sub;       /* [nworld][ncon_max] sub-contact index (corner / end)     */
  float *dist;        /* [nworld][ncon_max] phi                                  */
  float *pos;         /* [nworld][ncon_max][3] contact point                     */
  float *frame;       /* [nworld][ncon_max][9] rows n, t1, t2                    */
  float *impulse;     /* [nworld][ncon_max][nfacet] lambda*h per facet           */
  /* training data of the learned impedance network (models of free bodies
   * only, else ignored): the contact's 7 features (8th 0) and, on each of the
   * nfacet outputs (the rest 0), the log of the gain multiplier g, clipped to
   * [-ln 256, ln 256], that the network should apply to the heuristic gains:
   * for the contact alone along its normal (the fallback rule's model, see
   * cf_model_set_learned_impedance), with the heuristic's facet impulses
   * summing to S and w = 1/m_a + 1/m_b (tr/3), the normal velocity after the
   * step v(g) = v_n + w g S is placed at min(-phi/h, (v(1) + v_max)/2),
   * v_max = sqrt(v(1)^2 + (margin/h)^2) the largest the fallback rule accepts
   * with the model's margin; g = 1 without normal impulse, e^-ln256 when the
   * velocity would need a pulling impulse */
  float *features;    /* [nworld][ncon_max][8]                                   */
  float *target;      /* [nworld][ncon_max][16]                                  */
  /* with the learned impedance on (cf_model_set_learned_impedance): 1 where
   * the contact fell back to the heuristic gains, 0 where it kept the learned
   * ones; left untouched otherwise */
  int32_t *fallback;  /* [nworld][ncon_max]                                      */
} cf_contacts;

/* Validate the descriptor, upload per-world constants and size the contact
 * workspace (nworld * ncon_max records) on the current HIP device.  Returns
 * CF_OK or CF_W_PAIRS_SKIPPED with *out set, else an error with *out = NULL.
 * Free joints are allowed only on bodies whose parent is the world.  A free
 * body without children needs mass > 0 and inertia > 0; every other root with
 * its descendants (hinge/slide chains, floating bases) must be contiguous in
 * body order and hold at most 32 dofs (else CF_E_UNSUPPORTED); its mass matrix
 * must be positive definite. */
cf_status cf_model_create(const cf_model_desc *desc, cf_model **out);

/* Free the model's device memory (synchronises the device first).  NULL is a no-op. */
void cf_model_destroy(cf_model *m);

/* nq, nv per world and facets per contact; any pointer may be NULL. */
cf_status cf_model_dims(const cf_model *m, int32_t *nq, int32_t *nv, int32_t *nfacet);

/* One step of every world (Algorithm 1 preceded by collision detection and
 * followed by integration).  q [nworld][nq], v and tau [nworld][nv] (tau NULL
 * = zero applied force), q_out/v_out same shapes.  All float32, 16-byte
 * aligned device pointers.  out may be NULL.  Two kernels (narrow phase, then
 * resolution), or one that runs both for each world (cf_model_step_kernels). */
cf_status cf_step(cf_model *m, void *stream, const float *q, const float *v, const float *tau,
                  float *q_out, float *v_out, const cf_contacts *out);

/* Adjoint of one cf_step (reverse mode).  With (q+, v+) = cf_step(q, v, tau)
 * and L = <gq_out, q+> + <gv_out, v+>, writes gq = dL/dq [nworld][nq],
 * gv = dL/dv and gtau = dL/dtau [nworld][nv] (gtau may be NULL; tau NULL =
 * zero applied force; gq_out or gv_out NULL = zero).  The step is piecewise
 * smooth: the derivative is that of the piece containing (q, v, tau), with the
 * contact set, each facet's activity (the max(., 0) of Eq. cf_wrench), the
 * clamp of the impedance argument (Eq. r_scaling) and the tangent-helper
 * choice held as the forward step took them; contact gaps, normals and points
 * are differentiated through the narrow phase's geometry.  Quaternion entries
 * of gq are derivatives with respect to the stored (not necessarily unit)
 * values.  Chaining the call backwards over a stored trajectory gives the
 * gradient of a rollout (per-step checkpointing: each call recomputes its
 * step's forward pass from (q, v, tau)).  Float32 device buffers, 16-byte
 * aligned; gq/gv may alias gq_out/gv_out exactly.  Asynchronous on stream;
 * uses the model's contact workspace (so it must not overlap a cf_step of the
 * same model on another stream).  Articulated subtrees (hinge and slide joints
 * below a fixed or a free root) and position actuators are covered (an
 * actuated dof's gtau entry is the adjoint of its target), and so is the
 * diagonal impedance on models of free bodies (its per-facet gains
 * differentiated through the lever arms, the contact frame and the bodies'
 * world inverse inertia, i.e. their orientation), and so are learned gains
 * (cf_model_set_learned_impedance): the gains are recomputed from the float32
 * network and differentiated through its features (gap, normal and
 * tangential relative velocity, effective mass) and the heuristic gain they
 * scale, each contact's keep-or-fall-back decision and each clamped output
 * held as the step took them.  (The step evaluates the network with bf16
 * operands, whose outputs are piecewise constant in the features; the
 * adjoint is that of the float32 network, the function the bf16 evaluation
 * rounds.)  The diagonal impedance on a model with articulated subtrees
 * returns CF_E_UNSUPPORTED. */
cf_status cf_step_backward(cf_model *m, void *stream, const float *q, const float *v, const float *tau,
                           const float *gq_out, const float *gv_out, float *gq, float *gv, float *gtau);

/* T consecutive steps (batched rollouts): q_traj/v_traj [T+1][nworld][nq|nv]
 * receive the initial state (copied from q0/v0 unless they already alias row 0)
 * and every step's result; tau_seq [T][nworld][nv] or NULL; ncon_traj
 * [T][nworld] receives the contacts kept at each step and overflow_traj
 * [T][nworld] the contacts dropped beyond ncon_max at each step (either may
 * be NULL).  T >= 0.  The same step as cf_step (Algorithm 1 with collision
 * and integration, repeated): batched rollouts are the workload of the
 * paper's throughput-versus-environments and MPC experiments (Sec. IV.E,
 * Sec. V).  All T steps run in one persistent kernel launch (one workgroup
 * per world; see cf_model_get_launch) for worlds of at most 64 free bodies
 * without actuators or learned gains (each body stepped by its own lane, the
 * contact records in the model's workspace) and for other models whose
 * world state, contact list (ncon_max records) and scratch fit one
 * workgroup's LDS (nothing but the trajectory crosses HBM); else, or when
 * cf_model_autotune finds step launches faster, as T cf_step calls.  Allocates nothing, so a
 * stream capture (HIP graph) of the call replays it. */
cf_status cf_rollout(cf_model *m, void *stream, int32_t T, const float *q0, const float *v0,
                     const float *tau_seq, float *q_traj, float *v_traj, int32_t *ncon_traj,
                     int32_t *overflow_traj);

/* Impedance of the facet impulses (Sec. III.B).  CF_IMPEDANCE_HEURISTIC (the
 * default): A = r(|phi|)/(1 - r(|phi|)) / (tr_a + tr_b), one scalar per contact
 * (Eqs. k_d_setting, r_scaling).  CF_IMPEDANCE_DIAGONAL: the diagonal form the
 * paper gives before its heuristic, K h + D = (1/h) (J~_f M^-1 J~_f^T)^-1 per
 * facet f, split between K and D in the ratio k_user : d_user / h, so
 * lambda_f h = max(-(k_user h + d_user) s_f - k_user phi, 0) / ((k_user h + d_user) g_f)
 * with g_f = J~_f M^-1 J~_f^T (0 when k_user h + d_user = 0, or when the row
 * moves no dof).  M is block diagonal over free bodies and articulated
 * subtrees: a free body contributes its closed-form block, a subtree
 * |L^-1 J~_f^T|^2 over its dofs from its Cholesky factor L (both bodies of
 * a contact inside one subtree make one row on its dofs).  On a model with
 * articulated subtrees the resolution keeps each body's L^-1 J_b^T in LDS
 * (6 nd floats per body, nd its subtree's dofs): CF_E_UNSUPPORTED when that
 * does not fit beside the world's other LDS data; cf_step_backward covers
 * the diagonal form on models of free bodies only.  Host call; takes effect
 * from the next launch. */
cf_status cf_model_set_impedance(cf_model *m, int32_t mode);

/* Position actuators on hinge and slide dofs (the actuated hand of the
 * paper's application section, Sec. V): for a dof with kp[i] or kd[i]
 * nonzero, the per-step input tau[i] (cf_step's tau, cf_rollout's tau_seq) is
 * the target position u_i and the applied force of Eq. smooth_vel is
 * kp[i] (u_i - q_i) - kd[i] v_i, evaluated on the state at the start of the
 * step; other dofs take tau[i] as a force.  kp, kd: host arrays of nv floats
 * (either may be NULL = zeros), finite and >= 0; a nonzero gain on a free-joint
 * dof is CF_E_INVALID_ARG.  Both NULL (or all zero) removes the actuators.
 * The gains are copied to the device synchronously: call between steps, not
 * while work of this model is in flight. */
cf_status cf_model_set_actuators(cf_model *m, const float *kp, const float *kd);

/* Learned impedance gains (see the network entry points below): with params
 * (device, cf_mlp_nparam() floats, read at every step, owned by the caller)
 * each facet gain of the heuristic is multiplied by exp(clamp(y_f, -ln 256,
 * ln 256)), y the network's output for the contact, unless that predicts, for
 * the contact alone along its normal, a next-step penetration larger than the
 * heuristic's by more than `margin` (m) or a normal kinetic energy larger by
 * more than that of moving `margin` in one step; then the contact keeps the
 * heuristic gain.  params NULL switches the network off and keeps `margin`
 * for the training targets that cf_contacts exports (finite, >= 0, else
 * CF_E_INVALID_ARG).  Models of free
 * bodies with the heuristic impedance only (else CF_E_UNSUPPORTED); the
 * resolution then runs at most 128 threads per world, after a one-workgroup
 * kernel that writes the network's bf16 LDS image from params (a device buffer
 * of the model, allocated by the first call with params); cf_rollout uses step
 * launches; cf_step_backward differentiates the float32 network (see there). */
cf_status cf_model_set_learned_impedance(cf_model *m, const float *params, float margin);

/* Workgroup size (64, 128 or 256 threads, one world per workgroup) of the
 * collision, the resolution and the rollout kernel.  Defaults by world size:
 * collision 64 threads, 128 above 64 and 256 above 128 spheres in the sphere
 * block (one block row per thread); resolution 128 threads, 256 above 64
 * bodies; rollout 256.  The contacts do not depend on the choice; v+ only in
 * its last bits (same arithmetic; the per-body contact sums are exact integer
 * sums within a chunk of one contact per thread, and chunks add in order, so
 * the chunk size can change the rounding). */
cf_status cf_model_set_launch(cf_model *m, int32_t collide_block, int32_t resolve_block, int32_t rollout_block);
/* Also reports whether cf_rollout uses the persistent kernel (1) or step calls (0). */
cf_status cf_model_get_launch(const cf_model *m, int32_t *collide_block, int32_t *resolve_block,
                              int32_t *rollout_block, int32_t *rollout_fused_kernel);

/* Autotuner: times every workgroup size of the two step kernels and of the
 * rollout kernel over `steps` steps from the state (q, v) (device, not
 * modified), on this model's worlds, and keeps the fastest of each; cf_rollout
 * then uses the persistent kernel only where it beat T cf_step calls by more
 * than 3 % (closer timings are within run-to-run noise).  It
 * allocates temporary device buffers and synchronises the stream.  Optional
 * outputs: the best microseconds per step of cf_step and of cf_rollout. */
cf_status cf_model_autotune(cf_model *m, void *stream, const float *q, const float *v, int32_t steps,
                            float *best_step_us, float *best_rollout_step_us);

/* Kernels of one cf_step: 1 when the narrow phase and the resolution of each
 * world run in one kernel (no learned gains, the one-wave launch shapes 64/64,
 * kernel timing off, the world's LDS within the limit, and either 1 to 64
 * free bodies without actuators or articulated subtrees, actuated or not; a
 * world's resolution then starts as soon as its own narrow phase ends; the
 * same contacts as the two launches and results equal to float32 rounding),
 * else 2.
 * Host call, no device work. */
cf_status cf_model_step_kernels(const cf_model *m, int32_t *nkernels);

/* Kernel timing.  When enabled, every cf_step runs its collision and resolution
 * kernels apart (never the one-kernel step) and records HIP events around them
 * on the step's stream.  cf_model_kernel_times
 * waits for the recorded events, returns the summed milliseconds of each
 * kernel and the number of steps since the last call, and resets the sums. */
cf_status cf_model_set_profiling(cf_model *m, int32_t enable);
cf_status cf_model_kernel_times(cf_model *m, double *ms_collide, double *ms_resolve,
                                int64_t *nsteps);

/* Isolated kernel durations: on `stream`, one warm-up collision launch from
 * q, then `reps` collision launches back to back, then `reps` resolution
 * launches back to back (from q, v into q_out, v_out, which must not alias
 * them), each group bracketed by one pair of HIP events; returns the average
 * microseconds per launch of each kernel.  Synchronises the stream; allocates
 * nothing.  The contact workspace holds the contacts of q afterwards. */
cf_status cf_model_time_kernels(cf_model *m, void *stream, const float *q, const float *v, float *q_out,
                                float *v_out, int32_t reps, float *us_collide, float *us_resolve);

/* ---- Learned per-contact impedance network (the learned K, D that Sec. III.B
 * allows in place of the heuristic).  Per contact, 7 features (phi, v_n, u_1,
 * u_2, m_eff = 1/(tr_a + tr_b), mu_t, h; stored as 8 floats, the 8th ignored)
 * are normalised, x = (f - mean)/std, and mapped by two SiLU layers of 64
 * units to 16 outputs y (one per facet used); the facet impulse gain becomes
 * the heuristic's times exp(clamp(y_f, -ln 256, ln 256)).  Parameters: one flat
 * float32 device array of cf_mlp_nparam() values, row-major: mean[8], std[8],
 * W1[8][64], b1[64], W2[64][64], b2[64], W3[64][16], b3[16].  Products run on
 * bf16 MFMA with float32 accumulation.  All pointers are 16-byte aligned
 * device memory; calls are asynchronous on `stream`. */
int32_t cf_mlp_nparam(void);
/* y [n][16] = network(feats [n][8]). */
cf_status cf_mlp_forward(void *stream, const float *params, const float *feats, int32_t n, float *out);
/* Floats of scratch that cf_mlp_gradient needs for n contacts. */
int64_t cf_mlp_work_floats(int32_t n);
/* Gradient of the mean squared error over the n contacts and the first nout
 * outputs, L = sum (y - targets)^2 / (n nout), targets [n][16]: grad
 * [nparam] (zero for mean and std) and *loss (device scalar, may be NULL).
 * Deterministic: per-wave partial sums in `work`, added in a fixed order. */
cf_status cf_mlp_gradient(void *stream, const float *params, const float *feats, const float *targets,
                          int32_t n, int32_t nout, float *work, int64_t work_floats, float *grad, float *loss);
/* cf_mlp_gradient for callers that cannot allocate device memory (code under
 * HIP graph capture, serving or training loops that forbid hipMalloc): the
 * same kernels and the same per-wave partition, so the same grad and loss bit
 * for bit, with the partial sums in a fixed static device array instead of a
 * caller workspace.  Allocates nothing, ever: the array holds the partials of
 * the largest grid the gradient launches (2048 waves x (nparam + 1) floats,
 * 47.5 MB), every GPU the library runs on keeps its own copy until the process
 * ends, and any n >= 1 fits (an n whose partials would not fit is rejected
 * with CF_E_INVALID_ARG).  The first call on a device looks up that device's
 * copy (CF_E_DEVICE if the lookup fails).  Nothing in the array needs to start
 * at zero; calls that overlap on one GPU share it and race, so serialise
 * them (one stream, or events).  Arguments as for cf_mlp_gradient. */
cf_status cf_mlp_gradient_noalloc(void *stream, const float *params, const float *feats, const float *targets,
                                  int32_t n, int32_t nout, float *grad, float *loss);
/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8; step counts from 1) of the
 * trained parameters (W1 onwards) with moment buffers m, v [nparam]. */
cf_status cf_mlp_adam(void *stream, float *params, float *m, float *v, const float *grad, int32_t step, float lr);

/* Message of the last failed call on this thread ("" if none). */
const char *cf_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
