/*
 * cfo.h - FP64 CPU oracle of the complementarity-free contact step.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or helper with the GPU library and is never on the product
 * path.
 *
 * What it computes (per world, everything in double precision), following the
 * paper's method section (Sec. III) and its Algorithm 1:
 *   1. kinematics of a tree of free / hinge / slide joints, the body Jacobians,
 *      the joint-space inertia M = sum_b J_b^T diag(m_b I, I_b) J_b and the bias
 *      c(q, v) (gravity + velocity-product terms) of the step dynamics (Eq. sys_dyn);
 *   2. the smooth prediction v_s = v + h M^-1 (tau - c)   (Eq. smooth_vel), tau
 *      the applied joint forces (optionally from position actuators on hinge
 *      and slide dofs: tau = kp (u - theta) - kd theta_dot, u the step's input);
 *   3. an analytic narrow phase (plane-sphere, plane-capsule, plane-box,
 *      sphere-sphere, box-sphere, box-capsule) enumerating geom pairs in index
 *      order;
 *   4. for every contact, dense facet rows J~ = J_n - mu_s d^T J_s
 *      (Eqs. dual_polyhedral / tilde_defs), the impedance of Eqs. k_d_setting and
 *      r_scaling, and the facet impulse lambda*h = (-K(J~ v_s h + phi) - D J~ v_s)_+
 *      (Eq. cf_wrench);
 *   5. p = sum J~^T lambda h, v+ = v_s + M^-1 p   (Eq. vel_correction);
 *   6. semi-implicit Euler integration of q.
 * Functions that reach a result with a plain definition (M, c, Jacobians,
 * distances) are that definition written out.  See cfo.c for the readings
 * taken where the paper is silent.
 *
 * Conventions: quaternions (w,x,y,z); free joint q = (COM position, quat),
 * v = (COM linear velocity, angular velocity), both in world coordinates.
 * All functions are re-entrant; distinct calls may run on distinct threads
 * provided their outputs do not overlap.
 */
#ifndef CFO_H
#define CFO_H

#ifdef __cplusplus
extern "C" {
#endif

enum { CFO_PLANE = 0, CFO_SPHERE = 1, CFO_CAPSULE = 2, CFO_BOX = 3 };
enum { CFO_FREE = 0, CFO_HINGE = 1, CFO_SLIDE = 2 };
enum { CFO_OK = 0, CFO_EINVAL = -1, CFO_ENOMEM = -3, CFO_ESINGULAR = -5 };

typedef struct {
  int nworld, nbody, ngeom, ncon_max, condim;
  const int *body_parent, *body_jnt;               /* [nbody]                      */
  const double *body_pos, *body_quat;              /* [nbody][3], [nbody][4]       */
  const double *body_ipos, *jnt_axis;              /* [nbody][3], [nbody][3]       */
  const double *body_mass, *body_inertia;          /* [nworld][nbody], [..][3]     */
  const int *geom_type, *geom_body;                /* [ngeom]                      */
  const double *geom_size, *geom_pos;              /* [nworld][ngeom][3]           */
  const double *geom_quat, *geom_friction;         /* [nworld][ngeom][4], [..][3]  */
  double h, gravity[3], k_user, d_user, solimp[5], margin;
  int impedance;                                   /* 0: heuristic M(phi); 1: exact diagonal */
  /* Position actuators, [nv] each or NULL: on a hinge or slide dof with
   * kp or kd nonzero the step's input tau_d is the target position u_d and the
   * applied force is kp_d (u_d - q_d) - kd_d v_d, evaluated at the start of the
   * step; other dofs take tau_d as a force.  Free-joint dofs must have 0. */
  const double *dof_kp, *dof_kd;
} cfo_desc;

typedef struct cfo_model cfo_model;

/* Optional per-step outputs; every pointer may be NULL.  Arrays are indexed
 * by the absolute world index (the full [nworld] extent must be allocated). */
typedef struct {
  int *ncon, *overflow;             /* [nworld]                                  */
  int *geom;                        /* [nworld][ncon_max][2]  (geom a, geom b)   */
  int *sub;                         /* [nworld][ncon_max]     sub-contact index  */
  double *dist, *pos, *frame;       /* [..][1], [..][3], [..][9] rows n, t1, t2  */
  double *impulse;                  /* [..][nfacet]  lambda*h per facet          */
  double *guard_phi;                /* [nworld] min |phi - margin| over every evaluated candidate */
  double *guard_frame;              /* [nworld] min ||n_x| - 0.5| over contacts  */
  double *v_smooth;                 /* [nworld][nv]                               */
  double *gen_impulse;              /* [nworld][nv] p = sum J~^T lambda h         */
  double *trace;                    /* [nworld][nbody] tr(J_b M^-1 J_b^T)          */
  double *facet_gain;               /* [..][nfacet] A_f with lambda_f h = A_f max(arg_f, 0) */
  double *features;                 /* [..][8] learned-gain features: phi, v_n, u_1, u_2,
                                       m_eff = 1/(tr_a + tr_b), mu_t, h, 0 (at v_s)   */
  int *fallback;                    /* [..] with learned gains set: 1 where the contact
                                       kept the heuristic, 0 where the learned gains  */
  double *fallback_slack;           /* [..][2] with learned gains set: penetration and
                                       energy slack of the fallback rule (>= 0: kept) */
} cfo_out;

int  cfo_create(const cfo_desc *d, cfo_model **out, char *err, int errlen);
void cfo_destroy(cfo_model *m);
void cfo_dims(const cfo_model *m, int *nq, int *nv, int *nfacet);

/* One step of worlds [w0, w1).  q, v, tau ([nworld][nq|nv], tau may be NULL),
 * q_out, v_out are full-size arrays; only the rows of the range are touched. */
int cfo_step(const cfo_model *m, int w0, int w1, const double *q, const double *v,
             const double *tau, double *q_out, double *v_out, const cfo_out *out);

/* Learned impedance gains (Sec. III.B lets K and D be learned; the network is
 * the build's, oracle/mlp.py).  y: [nworld][ncon_max][16] network outputs of
 * every contact in canonical order (the caller evaluates the network on the
 * features a plain step of the same state exports), or NULL to switch the
 * option off; read by cfo_step, owned by the caller.  Each facet gain of the
 * heuristic becomes A exp(clip(y_f, -ln 256, ln 256)) unless the fallback rule
 * (cfo.c) keeps the heuristic for the contact.  Heuristic impedance only. */
int cfo_set_learned(cfo_model *m, const double *y, double margin);

/* Building blocks, exposed for the closed-form tests (world w, state q/v of that world). */
int cfo_body_frames(const cfo_model *m, int w, const double *q, double *com /*[nb][3]*/,
                    double *rot /*[nb][9]*/);
int cfo_body_jacobian(const cfo_model *m, int w, const double *q, int body,
                      double *J /*[6][nv]: rows COM linear, then angular*/);
int cfo_mass_matrix(const cfo_model *m, int w, const double *q, double *M /*[nv][nv]*/);
int cfo_bias(const cfo_model *m, int w, const double *q, const double *v, double *c /*[nv]*/);
double cfo_impedance_ratio(const cfo_model *m, double phi);  /* r/(1-r) at |phi| */
double cfo_gamma(const cfo_model *m, double x);              /* gamma(x), x >= 0 */

#ifdef __cplusplus
}
#endif
#endif
