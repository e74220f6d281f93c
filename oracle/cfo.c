/*
 * cfo.c - FP64 CPU oracle of the complementarity-free contact step.
 *
 * TEST INFRASTRUCTURE ONLY (see cfo.h): a plain, slow, dense implementation
 * written from the paper's equations, used to check the GPU library.  Nothing
 * here is shared with the GPU sources.
 *
 * Readings taken where the paper is silent or ambiguous (each is also listed
 * in the design notes of the repository):
 *  - Impulse sign: the minus signs of Eq. cf_wrench are used (Algorithm 1's
 *    Kernel II omits them, which would attract on penetration).
 *  - Units: with lambda the step-averaged wrench (Eq. sys_dyn), the facet
 *    impulse is lambda*h = A * max(-(k_user*h + d_user) * s - k_user * phi, 0),
 *    where s = J~ v_s and A is the scalar of M(phi) (Eq. k_d_setting).
 *  - J_i in the trace of M(phi) is the 3 x nv Jacobian of body i's centre of
 *    mass (3/m for a free body); a static body contributes 0.  The identity in
 *    M(phi) spans every facet row of the contact, so A is one scalar per contact.
 *  - gamma(x) of Eq. r_scaling is evaluated with x clamped to [0, 1] (the
 *    printed branch turns negative for x > 1).
 *  - Facet directions: tangential and rolling use d = (1,0), (0,1), (-1,0),
 *    (0,-1) in the (t1, t2) basis; torsional uses sigma = +1, -1.  condim
 *    1 / 3 / 4 / 6 give 1 / 4 / 6 / 10 facets (normal only / +tangential /
 *    +torsional / +rolling).
 *  - Tangent basis: helper e_x if |n_x| <= 0.5 else e_y; t1 = normalised
 *    component of the helper orthogonal to n; t2 = n x t1.
 *  - Normal points from geom a to geom b, relative velocities are b minus a,
 *    a plane is always geom a; phi > 0 means separated.
 *  - Contact point: middle of the overlap.  Detection: phi < margin.
 *  - Pair friction: element-wise max of the two geoms' (mu_t, mu_tor, mu_rol).
 *  - Order: geom pairs (i < j) in index order, then sub-contact index (box
 *    corner bits x,y,z = bit 0,1,2 set for +half-size; capsule minus end first).
 *    Beyond ncon_max contacts are dropped and counted as overflow.
 *  - Excluded pairs: both geoms static, same body, parent-child bodies, and
 *    pair types outside {plane-sphere, plane-capsule, plane-box, sphere-sphere,
 *    box-sphere, box-capsule}.
 *  - Box-sphere: the box is geom a; the sphere centre c, in the box frame, is
 *    clamped to the box; outside (distance d > 1e-12 from the clamped point)
 *    the normal is the unit vector from the clamped point to c and phi = d - r;
 *    otherwise the normal is the outward axis of the face with the smallest
 *    depth s_k - |c_k| (lowest axis on ties, + side when c_k >= 0) and
 *    phi = -depth - r.  The point is c - n (r + phi / 2).  Box-capsule: as for
 *    the plane, the capsule meets the box with its two end spheres (minus end
 *    first); contact of the box with the capsule's side between the ends is
 *    not modelled.
 *  - Position actuators (the hand of the paper's application section): the
 *    applied force kp (u - theta) - kd theta_dot of an actuated hinge or slide
 *    dof is explicit (start-of-step state).
 *  - Degenerate sphere-sphere (centres closer than 1e-12) uses n = +z; a
 *    contact whose two traces sum to 0 is skipped.
 *  - Exact diagonal impedance (impedance = 1, the alternative the paper states
 *    before its heuristic, Sec. III.B): per facet f, K h + D equals
 *    (1/h) (J~_f M^-1 J~_f^T)^-1, split between K and D in the ratio
 *    k_user : d_user / h of Eq. k_d_setting, so the scalar A of the impulse
 *    becomes A_f = 1 / ((k_user h + d_user) g_f), g_f = J~_f M^-1 J~_f^T; r(|phi|)
 *    does not enter.  With k_user h + d_user = 0 or g_f = 0 the impulse is 0.
 *  - Learned gains (option; Sec. III.B allows a learned K, D, the network is
 *    this build's design): per contact the network's output y_f scales the
 *    heuristic gain, A_f = A exp(clip(y_f, -ln 256, ln 256)).  Fallback rule
 *    (also this build's design): the contact alone along its normal with
 *    inverse mass w = (tr_a + tr_b) / 3 (1/m_a + 1/m_b for free bodies); the
 *    normal velocity after the heuristic's impulses is v_h = v_n + w sum_f
 *    lambda_h,f, after the learned ones v_l likewise; the next-step
 *    penetration max(-(phi + h v_x), 0) and the normal kinetic energy
 *    v_x^2 / (2 w) of each; the learned impulses are kept iff the learned
 *    penetration is at most the heuristic's plus the margin delta, the
 *    learned energy at most the heuristic's plus (delta/h)^2 / (2 w), and v_l
 *    is finite; a contact with tr_a + tr_b = 0 keeps the heuristic.
 *  - Integration: semi-implicit Euler; free-joint orientation is updated by the
 *    exact exponential of h*omega (world frame, left-multiplied) then
 *    normalised; a state quaternion denotes the rotation of its normalised value.
 */
#include "cfo.h"

#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

struct cfo_model {
  cfo_desc d;
  int nq, nv, nf;
  int *qadr, *dadr;
  /* owned copies of every array of the descriptor */
  int *body_parent, *body_jnt, *geom_type, *geom_body;
  double *body_pos, *body_quat, *body_ipos, *jnt_axis, *body_mass, *body_inertia;
  double *geom_size, *geom_pos, *geom_quat, *geom_friction;
  double *dof_kp, *dof_kd; /* [nv], NULL without actuators */
  int *dof_q;              /* [nv] q index of an actuated dof, -1 otherwise */
  const double *learned_y; /* [nworld][ncon_max][16] network outputs, or NULL */
  double learned_margin;   /* fallback margin (m) */
};

/* ------------------------------------------------------------------ */
/* small vector / matrix helpers                                       */
/* ------------------------------------------------------------------ */
static double dot3(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
static void cross3(const double *a, const double *b, double *o) {
  double t[3] = {a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0]};
  o[0] = t[0]; o[1] = t[1]; o[2] = t[2];
}
static void sub3(const double *a, const double *b, double *o) { o[0] = a[0] - b[0]; o[1] = a[1] - b[1]; o[2] = a[2] - b[2]; }
/* o = A (3x3 row-major) * x */
static void mv3(const double *A, const double *x, double *o) {
  double t[3];
  for (int i = 0; i < 3; i++) t[i] = A[3 * i] * x[0] + A[3 * i + 1] * x[1] + A[3 * i + 2] * x[2];
  o[0] = t[0]; o[1] = t[1]; o[2] = t[2];
}
static void mm3(const double *A, const double *B, double *o) {
  double t[9];
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++) t[3 * i + j] = A[3 * i] * B[j] + A[3 * i + 1] * B[3 + j] + A[3 * i + 2] * B[6 + j];
  memcpy(o, t, sizeof t);
}
/* rotation matrix of the normalised quaternion (w,x,y,z) */
static void quat2mat(const double *q, double *R) {
  double n = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
  double w = q[0] / n, x = q[1] / n, y = q[2] / n, z = q[3] / n;
  R[0] = 1 - 2 * (y * y + z * z); R[1] = 2 * (x * y - z * w);     R[2] = 2 * (x * z + y * w);
  R[3] = 2 * (x * y + z * w);     R[4] = 1 - 2 * (x * x + z * z); R[5] = 2 * (y * z - x * w);
  R[6] = 2 * (x * z - y * w);     R[7] = 2 * (y * z + x * w);     R[8] = 1 - 2 * (x * x + y * y);
}
/* rotation by angle th about the unit axis a (Rodrigues) */
static void axis_angle(const double *a, double th, double *R) {
  double c = cos(th), s = sin(th), C = 1 - c;
  R[0] = c + a[0] * a[0] * C;        R[1] = a[0] * a[1] * C - a[2] * s; R[2] = a[0] * a[2] * C + a[1] * s;
  R[3] = a[1] * a[0] * C + a[2] * s; R[4] = c + a[1] * a[1] * C;        R[5] = a[1] * a[2] * C - a[0] * s;
  R[6] = a[2] * a[0] * C - a[1] * s; R[7] = a[2] * a[1] * C + a[0] * s; R[8] = c + a[2] * a[2] * C;
}
/* Hamilton product o = a (x) b */
static void quatmul(const double *a, const double *b, double *o) {
  double t[4] = {a[0] * b[0] - a[1] * b[1] - a[2] * b[2] - a[3] * b[3],
                 a[0] * b[1] + a[1] * b[0] + a[2] * b[3] - a[3] * b[2],
                 a[0] * b[2] - a[1] * b[3] + a[2] * b[0] + a[3] * b[1],
                 a[0] * b[3] + a[1] * b[2] - a[2] * b[1] + a[3] * b[0]};
  memcpy(o, t, sizeof t);
}

/* ------------------------------------------------------------------ */
/* model                                                               */
/* ------------------------------------------------------------------ */
static int jnt_nq(int t) { return t == CFO_FREE ? 7 : 1; }
static int jnt_nv(int t) { return t == CFO_FREE ? 6 : 1; }

static void *dupa(const void *src, size_t bytes) {
  if (bytes == 0) return calloc(1, 1);
  void *p = malloc(bytes);
  if (p && src) memcpy(p, src, bytes);
  return p;
}

static int fail(char *err, int errlen, const char *msg) {
  if (err && errlen > 0) snprintf(err, (size_t)errlen, "%s", msg);
  return CFO_EINVAL;
}

void cfo_destroy(cfo_model *m) {
  if (!m) return;
  free(m->qadr); free(m->dadr);
  free(m->body_parent); free(m->body_jnt); free(m->geom_type); free(m->geom_body);
  free(m->body_pos); free(m->body_quat); free(m->body_ipos); free(m->jnt_axis);
  free(m->body_mass); free(m->body_inertia);
  free(m->geom_size); free(m->geom_pos); free(m->geom_quat); free(m->geom_friction);
  free(m->dof_kp); free(m->dof_kd); free(m->dof_q);
  free(m);
}

int cfo_create(const cfo_desc *d, cfo_model **out, char *err, int errlen) {
  if (!d || !out) return fail(err, errlen, "null argument");
  *out = NULL;
  int nw = d->nworld, nb = d->nbody, ng = d->ngeom;
  if (nw < 1) return fail(err, errlen, "nworld must be >= 1");
  if (nb < 0 || ng < 0 || d->ncon_max < 0) return fail(err, errlen, "negative size");
  if (!(d->condim == 1 || d->condim == 3 || d->condim == 4 || d->condim == 6))
    return fail(err, errlen, "condim must be 1, 3, 4 or 6");
  if (!(d->h > 0)) return fail(err, errlen, "h must be > 0");
  if (d->impedance != 0 && d->impedance != 1) return fail(err, errlen, "impedance must be 0 or 1");
  if (!(d->k_user >= 0) || !(d->d_user >= 0)) return fail(err, errlen, "k_user, d_user must be >= 0");
  const double *si = d->solimp;
  if (!(si[0] > 0 && si[0] <= si[1] && si[1] < 1)) return fail(err, errlen, "need 0 < r_min <= r_max < 1");
  if (!(si[2] > 0)) return fail(err, errlen, "solimp width must be > 0");
  if (!(si[3] > 0 && si[3] < 1)) return fail(err, errlen, "solimp midpoint must be in (0, 1)");
  if (!(si[4] >= 1)) return fail(err, errlen, "solimp power must be >= 1");
  for (int b = 0; b < nb; b++) {
    int p = d->body_parent[b], t = d->body_jnt[b];
    if (p < -1 || p >= b) return fail(err, errlen, "body_parent must be -1 or a lower index");
    if (t != CFO_FREE && t != CFO_HINGE && t != CFO_SLIDE) return fail(err, errlen, "bad joint type");
    if (t == CFO_FREE) {
      if (p != -1) return fail(err, errlen, "free joints only on bodies whose parent is the world");
      const double *ip = d->body_ipos + 3 * b;
      if (ip[0] != 0 || ip[1] != 0 || ip[2] != 0) return fail(err, errlen, "free bodies need body_ipos = 0");
    } else {
      if (dot3(d->jnt_axis + 3 * b, d->jnt_axis + 3 * b) <= 0) return fail(err, errlen, "zero joint axis");
    }
    for (int w = 0; w < nw; w++) {
      if (!(d->body_mass[(size_t)w * nb + b] >= 0)) return fail(err, errlen, "negative mass");
      for (int k = 0; k < 3; k++)
        if (!(d->body_inertia[((size_t)w * nb + b) * 3 + k] >= 0)) return fail(err, errlen, "negative inertia");
    }
  }
  for (int g = 0; g < ng; g++) {
    int t = d->geom_type[g], b = d->geom_body[g];
    if (t < CFO_PLANE || t > CFO_BOX) return fail(err, errlen, "bad geom type");
    if (b < -1 || b >= nb) return fail(err, errlen, "bad geom_body");
  }

  cfo_model *m = (cfo_model *)calloc(1, sizeof *m);
  if (!m) return CFO_ENOMEM;
  m->d = *d;
  size_t W = (size_t)nw;
  m->body_parent = dupa(d->body_parent, sizeof(int) * nb);
  m->body_jnt = dupa(d->body_jnt, sizeof(int) * nb);
  m->geom_type = dupa(d->geom_type, sizeof(int) * ng);
  m->geom_body = dupa(d->geom_body, sizeof(int) * ng);
  m->body_pos = dupa(d->body_pos, sizeof(double) * 3 * nb);
  m->body_quat = dupa(d->body_quat, sizeof(double) * 4 * nb);
  m->body_ipos = dupa(d->body_ipos, sizeof(double) * 3 * nb);
  m->jnt_axis = dupa(d->jnt_axis, sizeof(double) * 3 * nb);
  m->body_mass = dupa(d->body_mass, sizeof(double) * W * nb);
  m->body_inertia = dupa(d->body_inertia, sizeof(double) * W * nb * 3);
  m->geom_size = dupa(d->geom_size, sizeof(double) * W * ng * 3);
  m->geom_pos = dupa(d->geom_pos, sizeof(double) * W * ng * 3);
  m->geom_quat = dupa(d->geom_quat, sizeof(double) * W * ng * 4);
  m->geom_friction = dupa(d->geom_friction, sizeof(double) * W * ng * 3);
  m->qadr = (int *)malloc(sizeof(int) * (nb + 1));
  m->dadr = (int *)malloc(sizeof(int) * (nb + 1));
  if (!m->body_parent || !m->body_jnt || !m->geom_type || !m->geom_body || !m->body_pos ||
      !m->body_quat || !m->body_ipos || !m->jnt_axis || !m->body_mass || !m->body_inertia ||
      !m->geom_size || !m->geom_pos || !m->geom_quat || !m->geom_friction || !m->qadr || !m->dadr) {
    cfo_destroy(m);
    return CFO_ENOMEM;
  }
  /* unit joint axes */
  for (int b = 0; b < nb; b++) {
    double *a = m->jnt_axis + 3 * b, n = sqrt(dot3(a, a));
    if (n > 0) { a[0] /= n; a[1] /= n; a[2] /= n; }
  }
  int qa = 0, da = 0;
  for (int b = 0; b < nb; b++) {
    m->qadr[b] = qa; m->dadr[b] = da;
    qa += jnt_nq(m->body_jnt[b]); da += jnt_nv(m->body_jnt[b]);
  }
  m->nq = qa; m->nv = da;
  m->nf = d->condim == 1 ? 1 : d->condim == 3 ? 4 : d->condim == 4 ? 6 : 10;
  m->d.dof_kp = m->d.dof_kd = NULL;
  if (d->dof_kp || d->dof_kd) {
    m->dof_kp = (double *)calloc(da ? da : 1, sizeof(double));
    m->dof_kd = (double *)calloc(da ? da : 1, sizeof(double));
    m->dof_q = (int *)malloc(sizeof(int) * (da ? da : 1));
    if (!m->dof_kp || !m->dof_kd || !m->dof_q) { cfo_destroy(m); return CFO_ENOMEM; }
    for (int b = 0; b < nb; b++) {
      int t = m->body_jnt[b];
      for (int k = 0; k < jnt_nv(t); k++) {
        int i = m->dadr[b] + k;
        double kp = d->dof_kp ? d->dof_kp[i] : 0.0, kd = d->dof_kd ? d->dof_kd[i] : 0.0;
        if (!(kp >= 0 && kd >= 0 && kp < 1e300 && kd < 1e300)) { cfo_destroy(m); return fail(err, errlen, "actuator gains must be finite and >= 0"); }
        if (t == CFO_FREE && (kp != 0 || kd != 0)) { cfo_destroy(m); return fail(err, errlen, "actuators only on hinge or slide dofs"); }
        m->dof_kp[i] = kp; m->dof_kd[i] = kd;
        m->dof_q[i] = (kp != 0 || kd != 0) ? m->qadr[b] : -1;
      }
    }
    m->d.dof_kp = m->dof_kp; m->d.dof_kd = m->dof_kd;
  }
  m->d.body_parent = m->body_parent; m->d.body_jnt = m->body_jnt;
  m->d.geom_type = m->geom_type; m->d.geom_body = m->geom_body;
  m->d.body_pos = m->body_pos; m->d.body_quat = m->body_quat; m->d.body_ipos = m->body_ipos;
  m->d.jnt_axis = m->jnt_axis; m->d.body_mass = m->body_mass; m->d.body_inertia = m->body_inertia;
  m->d.geom_size = m->geom_size; m->d.geom_pos = m->geom_pos; m->d.geom_quat = m->geom_quat;
  m->d.geom_friction = m->geom_friction;
  *out = m;
  return CFO_OK;
}

void cfo_dims(const cfo_model *m, int *nq, int *nv, int *nf) {
  if (nq) *nq = m->nq;
  if (nv) *nv = m->nv;
  if (nf) *nf = m->nf;
}

/* ------------------------------------------------------------------ */
/* kinematics: body frames and Jacobians                               */
/* ------------------------------------------------------------------ */
typedef struct {
  double org[3];  /* body frame origin (joint anchor), world */
  double rot[9];  /* body frame orientation, world            */
  double com[3];  /* centre of mass, world                    */
  double axis[3]; /* hinge / slide axis, world (unused for free) */
} frame_t;

static void body_frames(const cfo_model *m, const double *q, frame_t *f) {
  const cfo_desc *d = &m->d;
  for (int b = 0; b < d->nbody; b++) {
    int t = d->body_jnt[b], p = d->body_parent[b];
    const double *qb = q + m->qadr[b];
    frame_t *F = f + b;
    if (t == CFO_FREE) {
      memcpy(F->org, qb, 3 * sizeof(double));
      quat2mat(qb + 3, F->rot);
      memset(F->axis, 0, sizeof F->axis);
    } else {
      double porg[3] = {0, 0, 0}, prot[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};
      if (p >= 0) { memcpy(porg, f[p].org, sizeof porg); memcpy(prot, f[p].rot, sizeof prot); }
      double off[3], R0[9], Rb[9];
      mv3(prot, d->body_pos + 3 * b, off);
      quat2mat(d->body_quat + 4 * b, Rb);
      mm3(prot, Rb, R0);
      double org0[3] = {porg[0] + off[0], porg[1] + off[1], porg[2] + off[2]};
      mv3(R0, d->jnt_axis + 3 * b, F->axis);
      if (t == CFO_HINGE) {
        double Rj[9];
        axis_angle(d->jnt_axis + 3 * b, qb[0], Rj);
        mm3(R0, Rj, F->rot);
        memcpy(F->org, org0, sizeof org0);
      } else { /* slide */
        memcpy(F->rot, R0, sizeof R0);
        for (int k = 0; k < 3; k++) F->org[k] = org0[k] + F->axis[k] * qb[0];
      }
    }
    double ic[3];
    mv3(F->rot, d->body_ipos + 3 * b, ic);
    for (int k = 0; k < 3; k++) F->com[k] = F->org[k] + ic[k];
  }
}

/* J [6][nv]: rows 0-2 map v to the COM velocity of body b, rows 3-5 to its
 * angular velocity.  Column of each ancestor joint j (including b's own):
 *   free:  linear dof k -> (e_k, 0); angular dof k -> (e_k x (com_b - org_j), e_k)
 *   hinge: (a_j x (com_b - org_j), a_j)
 *   slide: (a_j, 0)                                                       */
static void jacobian(const cfo_model *m, const frame_t *f, int b, double *J) {
  const cfo_desc *d = &m->d;
  int nv = m->nv;
  memset(J, 0, sizeof(double) * 6 * nv);
  for (int j = b; j >= 0; j = d->body_parent[j]) {
    int t = d->body_jnt[j], da = m->dadr[j];
    double r[3];
    sub3(f[b].com, f[j].org, r);
    if (t == CFO_FREE) {
      for (int k = 0; k < 3; k++) {
        double e[3] = {0, 0, 0}, c[3];
        e[k] = 1;
        J[k * nv + da + k] = 1;
        cross3(e, r, c);
        for (int i = 0; i < 3; i++) J[i * nv + da + 3 + k] = c[i];
        J[(3 + k) * nv + da + 3 + k] = 1;
      }
    } else if (t == CFO_HINGE) {
      double c[3];
      cross3(f[j].axis, r, c);
      for (int i = 0; i < 3; i++) { J[i * nv + da] = c[i]; J[(3 + i) * nv + da] = f[j].axis[i]; }
    } else {
      for (int i = 0; i < 3; i++) J[i * nv + da] = f[j].axis[i];
    }
  }
}

/* world inertia about the COM: R diag(I) R^T */
static void world_inertia(const cfo_model *m, int w, int b, const frame_t *f, double *I) {
  const double *Id = m->d.body_inertia + ((size_t)w * m->d.nbody + b) * 3;
  const double *R = f[b].rot;
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++)
      I[3 * i + j] = R[3 * i] * Id[0] * R[3 * j] + R[3 * i + 1] * Id[1] * R[3 * j + 1] + R[3 * i + 2] * Id[2] * R[3 * j + 2];
}

/* M = sum_b J_b^T diag(m_b I3, I_b) J_b  (kinetic energy 1/2 v^T M v) */
static void mass_matrix(const cfo_model *m, int w, const frame_t *f, const double *Jall, double *M) {
  int nv = m->nv, nb = m->d.nbody;
  memset(M, 0, sizeof(double) * nv * nv);
  double *X = (double *)malloc(sizeof(double) * 6 * (nv ? nv : 1));
  for (int b = 0; b < nb; b++) {
    const double *J = Jall + (size_t)b * 6 * nv;
    double mb = m->d.body_mass[(size_t)w * nb + b], I[9];
    world_inertia(m, w, b, f, I);
    /* X = diag(m I3, I) J */
    for (int c = 0; c < nv; c++) {
      for (int r = 0; r < 3; r++) X[r * nv + c] = mb * J[r * nv + c];
      for (int r = 0; r < 3; r++)
        X[(3 + r) * nv + c] = I[3 * r] * J[3 * nv + c] + I[3 * r + 1] * J[4 * nv + c] + I[3 * r + 2] * J[5 * nv + c];
    }
    for (int i = 0; i < nv; i++) {
      int nz = 0;
      for (int r = 0; r < 6; r++) nz |= J[r * nv + i] != 0;
      if (!nz) continue; /* a zero column of J_b adds nothing */
      for (int j = 0; j < nv; j++) {
        double s = 0;
        for (int r = 0; r < 6; r++) s += J[r * nv + i] * X[r * nv + j];
        M[i * nv + j] += s;
      }
    }
  }
  free(X);
}

/* c(q,v) = sum_b J_b^T [ m_b (Jdot_b v)_lin - m_b g ;  I_b (Jdot_b v)_ang + w_b x I_b w_b ]
 * Jdot_b v differentiates each Jacobian column in time:
 *   free angular dof k: d/dt(e_k x (com_b - org_j)) = e_k x (vcom_b - vorg_j)
 *   hinge j: d/dt a_j = w_j x a_j;  d/dt(a_j x (com_b - org_j)) = (w_j x a_j) x (com_b - org_j) + a_j x (vcom_b - vorg_j)
 *   slide j: d/dt a_j = w_j x a_j                                                 */
static void bias(const cfo_model *m, int w, const frame_t *f, const double *Jall, const double *v, double *c) {
  const cfo_desc *d = &m->d;
  int nv = m->nv, nb = d->nbody;
  memset(c, 0, sizeof(double) * nv);
  double *vc = (double *)malloc(sizeof(double) * 3 * (nb ? nb : 1));
  double *om = (double *)malloc(sizeof(double) * 3 * (nb ? nb : 1));
  double *vo = (double *)malloc(sizeof(double) * 3 * (nb ? nb : 1));
  for (int b = 0; b < nb; b++) {
    const double *J = Jall + (size_t)b * 6 * nv;
    for (int r = 0; r < 3; r++) {
      double s1 = 0, s2 = 0;
      for (int i = 0; i < nv; i++) { s1 += J[r * nv + i] * v[i]; s2 += J[(3 + r) * nv + i] * v[i]; }
      vc[3 * b + r] = s1; om[3 * b + r] = s2;
    }
    double r[3], x[3];
    sub3(f[b].org, f[b].com, r);
    cross3(om + 3 * b, r, x);
    for (int k = 0; k < 3; k++) vo[3 * b + k] = vc[3 * b + k] + x[k];
  }
  for (int b = 0; b < nb; b++) {
    double jl[3] = {0, 0, 0}, ja[3] = {0, 0, 0};
    for (int j = b; j >= 0; j = d->body_parent[j]) {
      int t = d->body_jnt[j], da = m->dadr[j];
      double dv[3], rr[3], tmp[3], tmp2[3];
      sub3(vc + 3 * b, vo + 3 * j, dv);
      sub3(f[b].com, f[j].org, rr);
      if (t == CFO_FREE) {
        for (int k = 0; k < 3; k++) {
          double e[3] = {0, 0, 0};
          e[k] = 1;
          cross3(e, dv, tmp);
          for (int i = 0; i < 3; i++) jl[i] += tmp[i] * v[da + 3 + k];
        }
      } else if (t == CFO_HINGE) {
        double wa[3];
        cross3(om + 3 * j, f[j].axis, wa);
        cross3(wa, rr, tmp);
        cross3(f[j].axis, dv, tmp2);
        for (int i = 0; i < 3; i++) { jl[i] += (tmp[i] + tmp2[i]) * v[da]; ja[i] += wa[i] * v[da]; }
      } else {
        double wa[3];
        cross3(om + 3 * j, f[j].axis, wa);
        for (int i = 0; i < 3; i++) jl[i] += wa[i] * v[da];
      }
    }
    double mb = d->body_mass[(size_t)w * nb + b], I[9], Iw[3], gy[3], Ia[3];
    world_inertia(m, w, b, f, I);
    mv3(I, om + 3 * b, Iw);
    cross3(om + 3 * b, Iw, gy);
    mv3(I, ja, Ia);
    double F[6];
    for (int k = 0; k < 3; k++) { F[k] = mb * (jl[k] - d->gravity[k]); F[3 + k] = Ia[k] + gy[k]; }
    const double *J = Jall + (size_t)b * 6 * nv;
    for (int i = 0; i < nv; i++) {
      double s = 0;
      for (int r = 0; r < 6; r++) s += J[r * nv + i] * F[r];
      c[i] += s;
    }
  }
  free(vc); free(om); free(vo);
}

/* ------------------------------------------------------------------ */
/* dense linear algebra                                                */
/* ------------------------------------------------------------------ */
/* in-place lower Cholesky, A = L L^T; returns 0 on success */
static int cholesky(double *A, int n) {
  for (int j = 0; j < n; j++) {
    double s = A[j * n + j];
    for (int k = 0; k < j; k++) s -= A[j * n + k] * A[j * n + k];
    if (!(s > 0)) return -1;
    double l = sqrt(s);
    A[j * n + j] = l;
    for (int i = j + 1; i < n; i++) {
      double t = A[i * n + j];
      for (int k = 0; k < j; k++) t -= A[i * n + k] * A[j * n + k];
      A[i * n + j] = t / l;
    }
    for (int i = 0; i < j; i++) A[i * n + j] = 0;
  }
  return 0;
}
static void fwd_sub(const double *L, int n, double *x) { /* L y = x */
  for (int i = 0; i < n; i++) {
    double s = x[i];
    for (int k = 0; k < i; k++) s -= L[i * n + k] * x[k];
    x[i] = s / L[i * n + i];
  }
}
static void bwd_sub(const double *L, int n, double *x) { /* L^T y = x */
  for (int i = n - 1; i >= 0; i--) {
    double s = x[i];
    for (int k = i + 1; k < n; k++) s -= L[k * n + i] * x[k];
    x[i] = s / L[i * n + i];
  }
}
static void chol_solve(const double *L, int n, double *x) { fwd_sub(L, n, x); bwd_sub(L, n, x); }

/* ------------------------------------------------------------------ */
/* impedance, Eqs. k_d_setting and r_scaling                           */
/* ------------------------------------------------------------------ */
double cfo_gamma(const cfo_model *m, double x) {
  double mid = m->d.solimp[3], p = m->d.solimp[4];
  if (x > 1) x = 1;
  if (x < 0) x = 0;
  if (x < mid) return mid * pow(x / mid, p);
  return 1 - (1 - mid) * pow((1 - x) / (1 - mid), p);
}

double cfo_impedance_ratio(const cfo_model *m, double phi) {
  const double *si = m->d.solimp;
  double r = si[0] + (si[1] - si[0]) * cfo_gamma(m, fabs(phi) / si[2]);
  return r / (1 - r);
}

/* ------------------------------------------------------------------ */
/* narrow phase                                                        */
/* ------------------------------------------------------------------ */
typedef struct {
  int ga, gb, sub;
  double phi, n[3], p[3];
} contact_t;

typedef struct {
  double pos[3], rot[9];
} gpose_t;

static void geom_pose(const cfo_model *m, int w, int g, const frame_t *f, gpose_t *o) {
  const cfo_desc *d = &m->d;
  const double *gp = d->geom_pos + ((size_t)w * d->ngeom + g) * 3;
  const double *gq = d->geom_quat + ((size_t)w * d->ngeom + g) * 4;
  double Rg[9];
  quat2mat(gq, Rg);
  int b = d->geom_body[g];
  if (b < 0) {
    memcpy(o->pos, gp, 3 * sizeof(double));
    memcpy(o->rot, Rg, sizeof Rg);
  } else {
    double off[3];
    mv3(f[b].rot, gp, off);
    for (int k = 0; k < 3; k++) o->pos[k] = f[b].org[k] + off[k];
    mm3(f[b].rot, Rg, o->rot);
  }
}

static const double *gsize(const cfo_model *m, int w, int g) { return m->d.geom_size + ((size_t)w * m->d.ngeom + g) * 3; }

/* pair is handled (geoms are candidates for contact) */
static int pair_allowed(const cfo_model *m, int i, int j) {
  const cfo_desc *d = &m->d;
  int bi = d->geom_body[i], bj = d->geom_body[j];
  if (bi < 0 && bj < 0) return 0;
  if (bi == bj) return 0;
  if (bi >= 0 && bj >= 0 && (d->body_parent[bi] == bj || d->body_parent[bj] == bi)) return 0;
  int ti = d->geom_type[i], tj = d->geom_type[j];
  if (ti == CFO_PLANE && tj == CFO_PLANE) return 0;
  if (ti == CFO_PLANE || tj == CFO_PLANE) return 1;
  if (ti == CFO_BOX || tj == CFO_BOX) {
    int o = ti == CFO_BOX ? tj : ti;
    return o == CFO_SPHERE || o == CFO_CAPSULE;
  }
  return ti == CFO_SPHERE && tj == CFO_SPHERE;
}

/* candidate sub-contacts of pair (i<j); writes up to 8 entries, returns count */
static int pair_candidates(const cfo_model *m, int w, int i, int j, const frame_t *f, contact_t *c) {
  const cfo_desc *d = &m->d;
  int ga = i, gb = j;
  if (d->geom_type[j] == CFO_PLANE) { ga = j; gb = i; }
  else if (d->geom_type[j] == CFO_BOX && d->geom_type[i] != CFO_PLANE) { ga = j; gb = i; }
  gpose_t A, B;
  geom_pose(m, w, ga, f, &A);
  geom_pose(m, w, gb, f, &B);
  const double *sb = gsize(m, w, gb);
  int ta = d->geom_type[ga], tb = d->geom_type[gb];
  int n = 0;
  if (ta == CFO_PLANE) {
    double nrm[3] = {A.rot[2], A.rot[5], A.rot[8]}; /* plane normal: local z */
    if (tb == CFO_SPHERE || tb == CFO_CAPSULE) {
      int nend = tb == CFO_SPHERE ? 1 : 2;
      for (int e = 0; e < nend; e++) {
        double ctr[3];
        memcpy(ctr, B.pos, sizeof ctr);
        if (tb == CFO_CAPSULE) {
          double sgn = e == 0 ? -1.0 : 1.0;
          for (int k = 0; k < 3; k++) ctr[k] += sgn * sb[1] * B.rot[3 * k + 2];
        }
        double r[3];
        sub3(ctr, A.pos, r);
        double phi = dot3(nrm, r) - sb[0];
        contact_t *C = c + n++;
        C->ga = ga; C->gb = gb; C->sub = e; C->phi = phi;
        memcpy(C->n, nrm, sizeof nrm);
        for (int k = 0; k < 3; k++) C->p[k] = ctr[k] - nrm[k] * (sb[0] + 0.5 * phi);
      }
    } else if (tb == CFO_BOX) {
      for (int cb = 0; cb < 8; cb++) {
        double loc[3] = {(cb & 1) ? sb[0] : -sb[0], (cb & 2) ? sb[1] : -sb[1], (cb & 4) ? sb[2] : -sb[2]};
        double x[3], r[3];
        mv3(B.rot, loc, x);
        for (int k = 0; k < 3; k++) x[k] += B.pos[k];
        sub3(x, A.pos, r);
        double phi = dot3(nrm, r);
        contact_t *C = c + n++;
        C->ga = ga; C->gb = gb; C->sub = cb; C->phi = phi;
        memcpy(C->n, nrm, sizeof nrm);
        for (int k = 0; k < 3; k++) C->p[k] = x[k] - 0.5 * phi * nrm[k];
      }
    }
  } else if (ta == CFO_BOX) { /* box - sphere, box - capsule (end spheres) */
    const double *sa = gsize(m, w, ga);
    int nend = tb == CFO_SPHERE ? 1 : 2;
    for (int e = 0; e < nend; e++) {
      double ctr[3];
      memcpy(ctr, B.pos, sizeof ctr);
      if (tb == CFO_CAPSULE) {
        double sgn = e == 0 ? -1.0 : 1.0;
        for (int k = 0; k < 3; k++) ctr[k] += sgn * sb[1] * B.rot[3 * k + 2];
      }
      double r = sb[0], dw[3], l[3], diff[3], nl[3] = {0, 0, 0}, nrm[3], phi;
      sub3(ctr, A.pos, dw);
      for (int k = 0; k < 3; k++) l[k] = A.rot[k] * dw[0] + A.rot[3 + k] * dw[1] + A.rot[6 + k] * dw[2];
      for (int k = 0; k < 3; k++) {
        double cl = l[k] < -sa[k] ? -sa[k] : (l[k] > sa[k] ? sa[k] : l[k]);
        diff[k] = l[k] - cl;
      }
      double dist = sqrt(dot3(diff, diff));
      if (dist > 1e-12) {
        for (int k = 0; k < 3; k++) nl[k] = diff[k] / dist;
        phi = dist - r;
      } else {
        int kmin = 0;
        double dmin = sa[0] - fabs(l[0]);
        for (int k = 1; k < 3; k++) {
          double dk = sa[k] - fabs(l[k]);
          if (dk < dmin) { dmin = dk; kmin = k; }
        }
        nl[kmin] = l[kmin] >= 0 ? 1.0 : -1.0;
        phi = -dmin - r;
      }
      mv3(A.rot, nl, nrm);
      contact_t *C = c + n++;
      C->ga = ga; C->gb = gb; C->sub = e; C->phi = phi;
      memcpy(C->n, nrm, sizeof nrm);
      for (int k = 0; k < 3; k++) C->p[k] = ctr[k] - nrm[k] * (r + 0.5 * phi);
    }
  } else { /* sphere - sphere */
    const double *sa = gsize(m, w, ga);
    double dd[3];
    sub3(B.pos, A.pos, dd);
    double dist = sqrt(dot3(dd, dd));
    double nrm[3] = {0, 0, 1};
    if (dist >= 1e-12) for (int k = 0; k < 3; k++) nrm[k] = dd[k] / dist;
    double phi = dist - sa[0] - sb[0];
    contact_t *C = c + n++;
    C->ga = ga; C->gb = gb; C->sub = 0; C->phi = phi;
    memcpy(C->n, nrm, sizeof nrm);
    for (int k = 0; k < 3; k++) C->p[k] = A.pos[k] + nrm[k] * (sa[0] + 0.5 * phi);
  }
  return n;
}

/* tangent basis (reading above) */
static void tangent_basis(const double *n, double *t1, double *t2) {
  double a[3] = {0, 0, 0};
  if (fabs(n[0]) <= 0.5) a[0] = 1; else a[1] = 1;
  double an = dot3(a, n);
  for (int k = 0; k < 3; k++) t1[k] = a[k] - an * n[k];
  double l = sqrt(dot3(t1, t1));
  for (int k = 0; k < 3; k++) t1[k] /= l;
  cross3(n, t1, t2);
}

/* ------------------------------------------------------------------ */
/* public building blocks                                              */
/* ------------------------------------------------------------------ */
int cfo_body_frames(const cfo_model *m, int w, const double *q, double *com, double *rot) {
  if (w < 0 || w >= m->d.nworld) return CFO_EINVAL;
  int nb = m->d.nbody;
  frame_t *f = (frame_t *)malloc(sizeof(frame_t) * (nb ? nb : 1));
  if (!f) return CFO_ENOMEM;
  body_frames(m, q, f);
  for (int b = 0; b < nb; b++) {
    if (com) memcpy(com + 3 * b, f[b].com, 3 * sizeof(double));
    if (rot) memcpy(rot + 9 * b, f[b].rot, 9 * sizeof(double));
  }
  free(f);
  return CFO_OK;
}

int cfo_body_jacobian(const cfo_model *m, int w, const double *q, int body, double *J) {
  if (w < 0 || w >= m->d.nworld || body < 0 || body >= m->d.nbody) return CFO_EINVAL;
  frame_t *f = (frame_t *)malloc(sizeof(frame_t) * m->d.nbody);
  if (!f) return CFO_ENOMEM;
  body_frames(m, q, f);
  jacobian(m, f, body, J);
  free(f);
  return CFO_OK;
}

static int all_jacobians(const cfo_model *m, const double *q, frame_t **fo, double **Jo) {
  int nb = m->d.nbody, nv = m->nv;
  frame_t *f = (frame_t *)malloc(sizeof(frame_t) * (nb ? nb : 1));
  double *J = (double *)malloc(sizeof(double) * 6 * (size_t)(nv ? nv : 1) * (nb ? nb : 1));
  if (!f || !J) { free(f); free(J); return CFO_ENOMEM; }
  body_frames(m, q, f);
  for (int b = 0; b < nb; b++) jacobian(m, f, b, J + (size_t)b * 6 * nv);
  *fo = f; *Jo = J;
  return CFO_OK;
}

int cfo_mass_matrix(const cfo_model *m, int w, const double *q, double *M) {
  if (w < 0 || w >= m->d.nworld) return CFO_EINVAL;
  frame_t *f; double *J;
  int rc = all_jacobians(m, q, &f, &J);
  if (rc) return rc;
  mass_matrix(m, w, f, J, M);
  free(f); free(J);
  return CFO_OK;
}

int cfo_bias(const cfo_model *m, int w, const double *q, const double *v, double *c) {
  if (w < 0 || w >= m->d.nworld) return CFO_EINVAL;
  frame_t *f; double *J;
  int rc = all_jacobians(m, q, &f, &J);
  if (rc) return rc;
  bias(m, w, f, J, v, c);
  free(f); free(J);
  return CFO_OK;
}

/* ------------------------------------------------------------------ */
/* one step of one world (Algorithm 1 with collision and integration)  */
/* ------------------------------------------------------------------ */
static int step_world(const cfo_model *m, int w, const double *q, const double *v, const double *tau,
                      double *q_out, double *v_out, const cfo_out *out) {
  const cfo_desc *d = &m->d;
  int nb = d->nbody, ng = d->ngeom, nv = m->nv, nq = m->nq, nf = m->nf;
  double h = d->h;
  frame_t *f; double *Jall;
  int rc = all_jacobians(m, q, &f, &Jall);
  if (rc) return rc;
  double *M = (double *)malloc(sizeof(double) * (size_t)(nv ? nv * nv : 1));
  double *c = (double *)malloc(sizeof(double) * (nv ? nv : 1));
  double *vs = (double *)malloc(sizeof(double) * (nv ? nv : 1));
  double *p = (double *)calloc(nv ? nv : 1, sizeof(double));
  double *tr = (double *)calloc(nb ? nb : 1, sizeof(double));
  double *rows = (double *)malloc(sizeof(double) * 16 * (nv ? nv : 1)); /* Jn, Jt1, Jt2, Jtor, Jr1, Jr2, facet, scratch */
  double *Jp = (double *)malloc(sizeof(double) * 6 * (nv ? nv : 1));
  double *Jfs = (double *)malloc(sizeof(double) * 10 * (nv ? nv : 1)); /* the contact's facet rows */
  contact_t *con = (contact_t *)malloc(sizeof(contact_t) * (size_t)(d->ncon_max > 0 ? d->ncon_max : 1));
  if (!M || !c || !vs || !p || !tr || !rows || !Jp || !Jfs || !con) { rc = CFO_ENOMEM; goto done; }

  /* --- M(q), c(q,v), Cholesky --- */
  mass_matrix(m, w, f, Jall, M);
  bias(m, w, f, Jall, v, c);
  if (nv > 0 && cholesky(M, nv)) { rc = CFO_ESINGULAR; goto done; }

  /* --- smooth prediction, Eq. smooth_vel: v_s = v + h M^-1 (tau - c) --- */
  for (int i = 0; i < nv; i++) {
    double ti = tau ? tau[i] : 0.0;
    if (m->dof_q && m->dof_q[i] >= 0) ti = m->dof_kp[i] * (ti - q[m->dof_q[i]]) - m->dof_kd[i] * v[i];
    vs[i] = ti - c[i];
  }
  chol_solve(M, nv, vs);
  for (int i = 0; i < nv; i++) vs[i] = v[i] + h * vs[i];

  /* --- per-body trace tr(J_b M^-1 J_b^T) = || L^-1 J_b^T ||_F^2 over the COM rows --- */
  for (int b = 0; b < nb; b++) {
    const double *J = Jall + (size_t)b * 6 * nv;
    double s = 0;
    for (int r = 0; r < 3; r++) {
      double *y = rows + 15 * nv;
      memcpy(y, J + r * nv, sizeof(double) * nv);
      fwd_sub(M, nv, y);
      for (int i = 0; i < nv; i++) s += y[i] * y[i];
    }
    tr[b] = s;
  }

  /* --- narrow phase in canonical order --- */
  int ncon = 0, over = 0;
  double guard_phi = INFINITY, guard_frame = INFINITY;
  for (int i = 0; i < ng; i++)
    for (int j = i + 1; j < ng; j++) {
      if (!pair_allowed(m, i, j)) continue;
      contact_t cand[8];
      int nc = pair_candidates(m, w, i, j, f, cand);
      for (int k = 0; k < nc; k++) {
        double gphi = fabs(cand[k].phi - d->margin);
        if (gphi < guard_phi) guard_phi = gphi;
        if (cand[k].phi < d->margin) {
          if (ncon < d->ncon_max) con[ncon++] = cand[k];
          else over++;
        }
      }
    }

  /* --- per contact, per facet: Eqs. tilde_defs, cf_wrench; accumulate p --- */
  double kk = d->k_user, dd = d->d_user;
  size_t cbase = (size_t)w * d->ncon_max;
  for (int k = 0; k < ncon; k++) {
    contact_t *C = con + k;
    int ba = d->geom_body[C->ga], bb = d->geom_body[C->gb];
    double t1[3], t2[3];
    tangent_basis(C->n, t1, t2);
    double gf = fabs(fabs(C->n[0]) - 0.5);
    if (gf < guard_frame) guard_frame = gf;
    /* relative point Jacobian (b minus a) at the contact point: Jp rows 0-2 linear, 3-5 angular */
    memset(Jp, 0, sizeof(double) * 6 * nv);
    for (int side = 0; side < 2; side++) {
      int b = side ? bb : ba;
      if (b < 0) continue;
      double sg = side ? 1.0 : -1.0;
      const double *J = Jall + (size_t)b * 6 * nv;
      double r[3];
      sub3(C->p, f[b].com, r);
      for (int i = 0; i < nv; i++) {
        double wcol[3] = {J[3 * nv + i], J[4 * nv + i], J[5 * nv + i]}, x[3];
        cross3(wcol, r, x);
        for (int a = 0; a < 3; a++) {
          Jp[a * nv + i] += sg * (J[a * nv + i] + x[a]);
          Jp[(3 + a) * nv + i] += sg * wcol[a];
        }
      }
    }
    double *Jn = rows, *Jt1 = rows + nv, *Jt2 = rows + 2 * nv, *Jtor = rows + 3 * nv;
    double *Jr1 = rows + 4 * nv, *Jr2 = rows + 5 * nv;
    for (int i = 0; i < nv; i++) {
      double lv[3] = {Jp[i], Jp[nv + i], Jp[2 * nv + i]}, av[3] = {Jp[3 * nv + i], Jp[4 * nv + i], Jp[5 * nv + i]};
      Jn[i] = dot3(C->n, lv); Jt1[i] = dot3(t1, lv); Jt2[i] = dot3(t2, lv);
      Jtor[i] = dot3(C->n, av); Jr1[i] = dot3(t1, av); Jr2[i] = dot3(t2, av);
    }
    double trs = (ba >= 0 ? tr[ba] : 0) + (bb >= 0 ? tr[bb] : 0);
    const double *fa = d->geom_friction + ((size_t)w * ng + C->ga) * 3;
    const double *fb = d->geom_friction + ((size_t)w * ng + C->gb) * 3;
    double mu[3];
    for (int a = 0; a < 3; a++) mu[a] = fa[a] > fb[a] ? fa[a] : fb[a];
    /* M(phi) scalar: r/(1-r) / (tr_a + tr_b) */
    double A = trs > 0 ? cfo_impedance_ratio(m, C->phi) / trs : 0.0;
    static const double dir4[4][2] = {{1, 0}, {0, 1}, {-1, 0}, {0, -1}};
    double lam[10], gain[10], args[10];
    for (int fi = 0; fi < nf; fi++) {
      double *Jf = Jfs + (size_t)fi * nv;
      /* facet row J~ = J_n - mu_s d^T J_s */
      for (int i = 0; i < nv; i++) {
        double row = Jn[i];
        if (d->condim == 1) {
        } else if (fi < 4) {
          row -= mu[0] * (dir4[fi][0] * Jt1[i] + dir4[fi][1] * Jt2[i]);
        } else if (fi < 6) {
          double sigma = fi == 4 ? 1.0 : -1.0;
          row -= mu[1] * sigma * Jtor[i];
        } else {
          int j4 = fi - 6;
          row -= mu[2] * (dir4[j4][0] * Jr1[i] + dir4[j4][1] * Jr2[i]);
        }
        Jf[i] = row;
      }
      double s = 0;
      for (int i = 0; i < nv; i++) s += Jf[i] * vs[i];
      double arg = -(kk * h + dd) * s - kk * C->phi;
      double lh = trs > 0 && arg > 0 ? A * arg : 0.0;
      gain[fi] = trs > 0 ? A : 0.0;
      if (d->impedance == 1) {
        /* exact diagonal impedance: K h + D = (1/h) (J~_f M^-1 J~_f^T)^-1 per facet,
           split between K and D in the ratio k_user : d_user/h, so that
           A_f = 1 / ((k h + d) g_f) with g_f = J~_f M^-1 J~_f^T = |L^-1 J~_f^T|^2 */
        double *y = rows + 15 * nv;
        memcpy(y, Jf, sizeof(double) * nv);
        fwd_sub(M, nv, y);
        double g = 0;
        for (int i = 0; i < nv; i++) g += y[i] * y[i];
        double aa = kk * h + dd;
        gain[fi] = (g > 0 && aa > 0) ? 1.0 / (aa * g) : 0.0;
        lh = arg > 0 ? gain[fi] * arg : 0.0;
      }
      lam[fi] = lh;
      args[fi] = arg;
    }
    double vn = 0, u1 = 0, u2 = 0;
    for (int i = 0; i < nv; i++) { vn += Jn[i] * vs[i]; u1 += Jt1[i] * vs[i]; u2 += Jt2[i] * vs[i]; }
    int fell_back = 1;
    double slack[2] = {0, 0};
    if (m->learned_y && d->impedance == 0) {
      /* learned gains and the fallback rule (readings above) */
      const double *y = m->learned_y + (cbase + k) * 16;
      const double L256 = log(256.0);
      double ll[10], gl[10], Sh = 0, Sl = 0;
      for (int fi = 0; fi < nf; fi++) {
        double yf = y[fi] < -L256 ? -L256 : y[fi] > L256 ? L256 : y[fi];
        gl[fi] = trs > 0 ? A * exp(yf) : 0.0;
        ll[fi] = args[fi] > 0 ? gl[fi] * args[fi] : 0.0;
        Sh += lam[fi];
        Sl += ll[fi];
      }
      if (trs > 0) {
        double wi = trs / 3.0, delta = m->learned_margin;
        double v_h = vn + wi * Sh, v_l = vn + wi * Sl;
        double pen_h = -(C->phi + h * v_h), pen_l = -(C->phi + h * v_l);
        if (pen_h < 0) pen_h = 0;
        if (pen_l < 0) pen_l = 0;
        double e_h = 0.5 * v_h * v_h / wi, e_l = 0.5 * v_l * v_l / wi;
        double e_m = 0.5 * (delta / h) * (delta / h) / wi;
        slack[0] = pen_h + delta - pen_l;
        slack[1] = e_h + e_m - e_l;
        if (slack[0] >= 0 && slack[1] >= 0 && isfinite(v_l)) {
          fell_back = 0;
          for (int fi = 0; fi < nf; fi++) { lam[fi] = ll[fi]; gain[fi] = gl[fi]; }
        }
      }
    }
    for (int fi = 0; fi < nf; fi++)
      for (int i = 0; i < nv; i++) p[i] += Jfs[(size_t)fi * nv + i] * lam[fi];
    if (out) {
      size_t ci = cbase + k;
      if (out->geom) { out->geom[2 * ci] = C->ga; out->geom[2 * ci + 1] = C->gb; }
      if (out->sub) out->sub[ci] = C->sub;
      if (out->dist) out->dist[ci] = C->phi;
      if (out->pos) memcpy(out->pos + 3 * ci, C->p, 3 * sizeof(double));
      if (out->frame) {
        memcpy(out->frame + 9 * ci, C->n, 3 * sizeof(double));
        memcpy(out->frame + 9 * ci + 3, t1, 3 * sizeof(double));
        memcpy(out->frame + 9 * ci + 6, t2, 3 * sizeof(double));
      }
      if (out->impulse) memcpy(out->impulse + (size_t)nf * ci, lam, sizeof(double) * nf);
      if (out->facet_gain) memcpy(out->facet_gain + (size_t)nf * ci, gain, sizeof(double) * nf);
      if (out->features) {
        double *fe = out->features + 8 * ci;
        fe[0] = C->phi; fe[1] = vn; fe[2] = u1; fe[3] = u2;
        fe[4] = trs > 0 ? 1.0 / trs : 0.0; fe[5] = mu[0]; fe[6] = h; fe[7] = 0.0;
      }
      if (m->learned_y && d->impedance == 0) {
        if (out->fallback) out->fallback[ci] = fell_back;
        if (out->fallback_slack) { out->fallback_slack[2 * ci] = slack[0]; out->fallback_slack[2 * ci + 1] = slack[1]; }
      }
    }
  }

  /* --- velocity correction, Eq. vel_correction: v+ = v_s + M^-1 p --- */
  if (out && out->gen_impulse) memcpy(out->gen_impulse + (size_t)w * nv, p, sizeof(double) * nv);
  chol_solve(M, nv, p);
  for (int i = 0; i < nv; i++) v_out[i] = vs[i] + p[i];

  /* --- semi-implicit Euler --- */
  for (int b = 0; b < nb; b++) {
    int qa = m->qadr[b], da = m->dadr[b];
    if (d->body_jnt[b] == CFO_FREE) {
      const double *vb = v_out + da;
      for (int k = 0; k < 3; k++) q_out[qa + k] = q[qa + k] + h * vb[k];
      double th[3] = {h * vb[3], h * vb[4], h * vb[5]};
      double ang = sqrt(dot3(th, th)), e[4];
      if (ang < 1e-8) {
        e[0] = 1; e[1] = 0.5 * th[0]; e[2] = 0.5 * th[1]; e[3] = 0.5 * th[2];
      } else {
        double s = sin(0.5 * ang) / ang;
        e[0] = cos(0.5 * ang); e[1] = s * th[0]; e[2] = s * th[1]; e[3] = s * th[2];
      }
      double qn[4];
      quatmul(e, q + qa + 3, qn);
      double l = sqrt(qn[0] * qn[0] + qn[1] * qn[1] + qn[2] * qn[2] + qn[3] * qn[3]);
      for (int k = 0; k < 4; k++) q_out[qa + 3 + k] = qn[k] / l;
    } else {
      q_out[qa] = q[qa] + h * v_out[da];
    }
  }
  (void)nq;

  if (out) {
    if (out->ncon) out->ncon[w] = ncon;
    if (out->overflow) out->overflow[w] = over;
    if (out->guard_phi) out->guard_phi[w] = guard_phi;
    if (out->guard_frame) out->guard_frame[w] = guard_frame;
    if (out->v_smooth) memcpy(out->v_smooth + (size_t)w * nv, vs, sizeof(double) * nv);
    if (out->trace) memcpy(out->trace + (size_t)w * nb, tr, sizeof(double) * nb);
  }
  rc = CFO_OK;
done:
  free(f); free(Jall); free(M); free(c); free(vs); free(p); free(tr); free(rows); free(Jp); free(Jfs); free(con);
  return rc;
}

int cfo_set_learned(cfo_model *m, const double *y, double margin) {
  if (!m || !(margin >= 0)) return CFO_EINVAL;
  if (y && m->d.impedance != 0) return CFO_EINVAL;
  m->learned_y = y;
  m->learned_margin = margin;
  return CFO_OK;
}

int cfo_step(const cfo_model *m, int w0, int w1, const double *q, const double *v, const double *tau,
             double *q_out, double *v_out, const cfo_out *out) {
  if (!m || !q || !v || !q_out || !v_out) return CFO_EINVAL;
  if (w0 < 0 || w1 > m->d.nworld || w0 > w1) return CFO_EINVAL;
  int nq = m->nq, nv = m->nv;
  double *qtmp = (double *)malloc(sizeof(double) * (nq ? nq : 1));
  double *vtmp = (double *)malloc(sizeof(double) * (nv ? nv : 1));
  if (!qtmp || !vtmp) { free(qtmp); free(vtmp); return CFO_ENOMEM; }
  int rc = CFO_OK;
  for (int w = w0; w < w1 && rc == CFO_OK; w++) {
    rc = step_world(m, w, q + (size_t)w * nq, v + (size_t)w * nv, tau ? tau + (size_t)w * nv : NULL,
                    qtmp, vtmp, out);
    if (rc == CFO_OK) {
      memcpy(q_out + (size_t)w * nq, qtmp, sizeof(double) * nq);
      memcpy(v_out + (size_t)w * nv, vtmp, sizeof(double) * nv);
    }
  }
  free(qtmp); free(vtmp);
  return rc;
}
