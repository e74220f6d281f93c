// cf_adjoint.h - reverse-mode (vector-Jacobian) pieces of the contact step of
// free bodies, for any float type.  Host and device: the backward kernel runs
// them in float32; a host program checks each against central differences of
// the matching forward piece in float64.
//
// The step is piecewise smooth.  Its derivative is taken on the piece that
// contains the evaluation point: the contact set (which slots are in
// contact), which facets are active (max(., 0) of Eq. cf_wrench), the branch
// of the clamp x = min(|phi| / w, 1) and of gamma (Eq. r_scaling), and the
// tangent-helper choice stay as the forward step took them.
//
// Rotations: every quantity that depends on a body's orientation is
// differentiated with respect to a world-frame rotation increment dpsi
// (R -> exp([dpsi]x) R).  The adjoint psi_bar of such increments converts to
// the adjoint of the stored (not necessarily unit) quaternion q by
// quat_grad_from_psi().
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>

#include "cf_mlp.h"

namespace cf {
namespace adj {

#define CF_HD __host__ __device__ inline

template <class T>
struct Vec {
  T x, y, z;
};
template <class T> CF_HD Vec<T> vec(T x, T y, T z) { return {x, y, z}; }
template <class T> CF_HD Vec<T> operator+(Vec<T> a, Vec<T> b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
template <class T> CF_HD Vec<T> operator-(Vec<T> a, Vec<T> b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
template <class T> CF_HD Vec<T> operator-(Vec<T> a) { return {-a.x, -a.y, -a.z}; }
template <class T> CF_HD Vec<T> operator*(T s, Vec<T> a) { return {s * a.x, s * a.y, s * a.z}; }
template <class T> CF_HD T dot(Vec<T> a, Vec<T> b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
template <class T> CF_HD Vec<T> cross(Vec<T> a, Vec<T> b) {
  return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
// symmetric 3x3 stored (xx, yy, zz, xy, xz, yz)
template <class T> CF_HD Vec<T> sym_mul(const T *S, Vec<T> v) {
  return {S[0] * v.x + S[3] * v.y + S[4] * v.z, S[3] * v.x + S[1] * v.y + S[5] * v.z,
          S[4] * v.x + S[5] * v.y + S[2] * v.z};
}

// Rotation matrix (row-major) of the normalised quaternion (w, x, y, z).
template <class T>
CF_HD void rot_of_quat(const T *q, T *R) {
  const T inv = T(1) / sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
  const T w = q[0] * inv, x = q[1] * inv, y = q[2] * inv, z = q[3] * inv;
  R[0] = T(1) - T(2) * (y * y + z * z); R[1] = T(2) * (x * y - z * w); R[2] = T(2) * (x * z + y * w);
  R[3] = T(2) * (x * y + z * w); R[4] = T(1) - T(2) * (x * x + z * z); R[5] = T(2) * (y * z - x * w);
  R[6] = T(2) * (x * z - y * w); R[7] = T(2) * (y * z + x * w); R[8] = T(1) - T(2) * (x * x + y * y);
}

// R diag(d) R^T as (xx, yy, zz, xy, xz, yz).
template <class T>
CF_HD void rot_diag_rot(const T *R, const T *d, T *S) {
  const int ri[6] = {0, 1, 2, 0, 0, 1}, rj[6] = {0, 1, 2, 1, 2, 2};
  for (int k = 0; k < 6; ++k) {
    const T *u = R + 3 * ri[k], *v = R + 3 * rj[k];
    S[k] = u[0] * d[0] * v[0] + u[1] * d[1] * v[1] + u[2] * d[2] * v[2];
  }
}

// Adjoint of the stored quaternion q from the adjoint psi_bar of world-frame
// rotation increments of R(q / |q|): with (w, v) = q / |q|, the increment
// dq_hat gives dpsi = 2 vec(dq_hat (x) conj(q_hat)), so
// q_bar = (-2 v.psi_bar, 2 (w psi_bar + psi_bar x v)) / |q| (already
// orthogonal to q, as the normalisation requires).
template <class T>
CF_HD void quat_grad_from_psi(const T *q, Vec<T> pb, T *qbar) {
  const T l = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
  const T il = T(1) / l;
  const T w = q[0] * il;
  const Vec<T> v = vec(q[1] * il, q[2] * il, q[3] * il);
  const Vec<T> c = cross(pb, v);
  qbar[0] += T(-2) * dot(v, pb) * il;
  qbar[1] += T(2) * (w * pb.x + c.x) * il;
  qbar[2] += T(2) * (w * pb.y + c.y) * il;
  qbar[3] += T(2) * (w * pb.z + c.z) * il;
}

// ------------------------------------------------------------------ body: prediction
// v_s = v + h (f / m + g); w_s = w + h Iw^-1 (t - w x Iw w)  (Eq. smooth_vel for a
// free body: M = diag(m I3, Iw), c = (-m g, w x Iw w)).
template <class T>
struct BodyPredict {
  T m, d[3];        // mass, principal inertia
  T q[4];           // stored orientation
  Vec<T> v, w, f, t, g;
  T h;
};

template <class T>
CF_HD void predict_forward(const BodyPredict<T> &B, Vec<T> &vs, Vec<T> &ws) {
  T R[9], Iw[6], Ii[6];
  rot_of_quat(B.q, R);
  const T e[3] = {T(1) / B.d[0], T(1) / B.d[1], T(1) / B.d[2]};
  rot_diag_rot(R, B.d, Iw);
  rot_diag_rot(R, e, Ii);
  vs = B.v + B.h * ((T(1) / B.m) * B.f + B.g);
  const Vec<T> Io = sym_mul(Iw, B.w);
  const Vec<T> z = B.t - cross(B.w, Io);
  ws = B.w + B.h * sym_mul(Ii, z);
}

// Given the adjoints of v_s and w_s: adjoints of v, w, f, t (written) and of
// the rotation increment (added to psi).
template <class T>
CF_HD void predict_vjp(const BodyPredict<T> &B, Vec<T> vsb, Vec<T> wsb, Vec<T> &vb, Vec<T> &wb, Vec<T> &fb,
                       Vec<T> &tb, Vec<T> &psi) {
  T R[9], Iw[6], Ii[6];
  rot_of_quat(B.q, R);
  const T e[3] = {T(1) / B.d[0], T(1) / B.d[1], T(1) / B.d[2]};
  rot_diag_rot(R, B.d, Iw);
  rot_diag_rot(R, e, Ii);
  const Vec<T> Io = sym_mul(Iw, B.w);
  const Vec<T> z = B.t - cross(B.w, Io);
  const Vec<T> y = sym_mul(Ii, z);
  vb = vsb;
  fb = (B.h / B.m) * vsb;
  wb = wsb;
  // w_s = w + h y, y = Ii z: dy = dpsi x y + Ii (z x dpsi) + Ii dz
  const Vec<T> yb = B.h * wsb;
  const Vec<T> zb = sym_mul(Ii, yb);
  psi = psi + cross(y, yb) + cross(zb, z);
  tb = zb;
  // z = t - w x Io
  const Vec<T> gb = -zb;
  wb = wb + cross(Io, gb);
  const Vec<T> Iob = cross(gb, B.w);
  // Io = Iw w
  wb = wb + sym_mul(Iw, Iob);
  psi = psi + cross(Io, Iob) + cross(sym_mul(Iw, Iob), B.w);
}

// ------------------------------------------------------------------ body: correction + integration
// v+ = v_s + F / m, w+ = w_s + Ii T (Eq. vel_correction); x+ = x + h v+;
// q+ = normalise(exp(h w+) (x) q).
template <class T>
struct BodyUpdate {
  T m, d[3];
  T q[4];
  Vec<T> x, vs, ws, F, Tq;
  T h;
};

template <class T>
CF_HD void quat_exp(Vec<T> th, T *e) {
  const T ang = sqrt(dot(th, th));
  if (ang < T(1e-8)) {
    e[0] = T(1); e[1] = T(0.5) * th.x; e[2] = T(0.5) * th.y; e[3] = T(0.5) * th.z;
  } else {
    const T s = sin(T(0.5) * ang) / ang;
    e[0] = cos(T(0.5) * ang); e[1] = s * th.x; e[2] = s * th.y; e[3] = s * th.z;
  }
}

template <class T>
CF_HD void quat_mul(const T *a, const T *b, T *o) {
  o[0] = a[0] * b[0] - a[1] * b[1] - a[2] * b[2] - a[3] * b[3];
  o[1] = a[0] * b[1] + a[1] * b[0] + a[2] * b[3] - a[3] * b[2];
  o[2] = a[0] * b[2] - a[1] * b[3] + a[2] * b[0] + a[3] * b[1];
  o[3] = a[0] * b[3] + a[1] * b[2] - a[2] * b[1] + a[3] * b[0];
}

template <class T>
CF_HD void update_forward(const BodyUpdate<T> &B, Vec<T> &xp, T *qp, Vec<T> &vp, Vec<T> &wp) {
  T R[9], Ii[6];
  rot_of_quat(B.q, R);
  const T e[3] = {T(1) / B.d[0], T(1) / B.d[1], T(1) / B.d[2]};
  rot_diag_rot(R, e, Ii);
  vp = B.vs + (T(1) / B.m) * B.F;
  wp = B.ws + sym_mul(Ii, B.Tq);
  xp = B.x + B.h * vp;
  T ex[4], qn[4];
  quat_exp(B.h * wp, ex);
  quat_mul(ex, B.q, qn);
  const T il = T(1) / sqrt(qn[0] * qn[0] + qn[1] * qn[1] + qn[2] * qn[2] + qn[3] * qn[3]);
  for (int i = 0; i < 4; ++i) qp[i] = qn[i] * il;
}

// Adjoints of x+, q+, v+, w+ in; adjoints of x (written), of the stored
// quaternion through the exponential update (added to qb), of v_s, w_s, F,
// T (written) and of the rotation increment through Ii (added to psi).
template <class T>
CF_HD void update_vjp(const BodyUpdate<T> &B, Vec<T> xpb, const T *qpb, Vec<T> vpb, Vec<T> wpb, Vec<T> &xb,
                      T *qb, Vec<T> &vsb, Vec<T> &wsb, Vec<T> &Fb, Vec<T> &Tb, Vec<T> &psi) {
  T R[9], Ii[6];
  rot_of_quat(B.q, R);
  const T e3[3] = {T(1) / B.d[0], T(1) / B.d[1], T(1) / B.d[2]};
  rot_diag_rot(R, e3, Ii);
  const Vec<T> wp = B.ws + sym_mul(Ii, B.Tq);
  const Vec<T> th = B.h * wp;
  T e[4], qn[4];
  quat_exp(th, e);
  quat_mul(e, B.q, qn);
  const T l = sqrt(qn[0] * qn[0] + qn[1] * qn[1] + qn[2] * qn[2] + qn[3] * qn[3]);
  const T il = T(1) / l;
  // q+ = qn / |qn|
  const T qp[4] = {qn[0] * il, qn[1] * il, qn[2] * il, qn[3] * il};
  const T pr = qp[0] * qpb[0] + qp[1] * qpb[1] + qp[2] * qpb[2] + qp[3] * qpb[3];
  T g[4];
  for (int i = 0; i < 4; ++i) g[i] = (qpb[i] - qp[i] * pr) * il;
  // qn = e (x) q
  const T *q = B.q;
  const T eb[4] = {q[0] * g[0] + q[1] * g[1] + q[2] * g[2] + q[3] * g[3],
                   -q[1] * g[0] + q[0] * g[1] - q[3] * g[2] + q[2] * g[3],
                   -q[2] * g[0] + q[3] * g[1] + q[0] * g[2] - q[1] * g[3],
                   -q[3] * g[0] - q[2] * g[1] + q[1] * g[2] + q[0] * g[3]};
  qb[0] += e[0] * g[0] + e[1] * g[1] + e[2] * g[2] + e[3] * g[3];
  qb[1] += -e[1] * g[0] + e[0] * g[1] + e[3] * g[2] - e[2] * g[3];
  qb[2] += -e[2] * g[0] - e[3] * g[1] + e[0] * g[2] + e[1] * g[3];
  qb[3] += -e[3] * g[0] + e[2] * g[1] - e[1] * g[2] + e[0] * g[3];
  // e = exp(th): e_w = cos(a/2), e_v = s(a) th with s(a) = sin(a/2)/a
  const Vec<T> ev = vec(eb[1], eb[2], eb[3]);
  Vec<T> thb;
  const T a = sqrt(dot(th, th));
  if (a < T(1e-8)) {
    thb = T(0.5) * ev;
  } else {
    const T s = sin(T(0.5) * a) / a;
    // s'(a) / a, by its series where the closed form cancels
    const T a2 = a * a;
    const T ds_a = a < T(0.05) ? T(-1) / T(24) + a2 / T(960)
                               : (T(0.5) * a * cos(T(0.5) * a) - sin(T(0.5) * a)) / (a2 * a);
    thb = (-eb[0] * sin(T(0.5) * a) / (T(2) * a) + ds_a * dot(th, ev)) * th + s * ev;
  }
  const Vec<T> wpt = wpb + B.h * thb;
  const Vec<T> vpt = vpb + B.h * xpb;
  xb = xpb;
  vsb = vpt;
  Fb = (T(1) / B.m) * vpt;
  wsb = wpt;
  // w+ = w_s + Ii T
  Tb = sym_mul(Ii, wpt);
  psi = psi + cross(sym_mul(Ii, B.Tq), wpt) + cross(Tb, B.Tq);
}

// ------------------------------------------------------------------ impedance
template <class T>
struct Impedance {
  T r_min, r_max, width, mid, power;
};

// rho = r / (1 - r) of Eq. r_scaling at |phi| (x clamped to [0, 1]) and d rho / d phi.
template <class T>
CF_HD T impedance_rho(T phi, const Impedance<T> &P, T &drho) {
  const T x0 = fabs(phi) / P.width;
  const bool clamped = x0 >= T(1);
  const T x = clamped ? T(1) : x0;
  const bool lo = x < P.mid;
  const T u = lo ? x / P.mid : (T(1) - x) / (T(1) - P.mid);
  const T up = pow(u, P.power);
  const T gam = lo ? P.mid * up : T(1) - (T(1) - P.mid) * up;
  const T r = P.r_min + (P.r_max - P.r_min) * gam;
  const T dgam = P.power * pow(u, P.power - T(1));  // d gamma / dx on both branches
  const T dx = clamped ? T(0) : (phi > T(0) ? T(1) : phi < T(0) ? T(-1) : T(0)) / P.width;
  drho = (P.r_max - P.r_min) * dgam * dx / ((T(1) - r) * (T(1) - r));
  return r / (T(1) - r);
}

// ------------------------------------------------------------------ one contact
// Inputs of one contact's impulse and wrench (Eqs. dual_polyhedral, tilde_defs,
// cf_wrench): frame normal n, gap phi, point p; the two bodies' COM and smooth
// velocities (zero and has* = false for a static side); tr_a + tr_b; pair friction.
template <class T>
struct ContactIn {
  Vec<T> n, p;
  T phi;
  Vec<T> xa, va, wa, xb, vb, wb;
  bool has_a, has_b;
  T trs, mut, mutor, murol;
  T h, k, d;  // time step, k_user, d_user
  // exact diagonal impedance: per side 1/m and the world inverse inertia
  // (xx, yy, zz, xy, xz, yz); unused with the heuristic
  bool diag;
  T ima, imb, Sa[6], Sb[6];
  // learned gains (free bodies): the network's float32 parameters (cf_mlp.h
  // layout) or null, and the fallback margin (m)
  const float *net;
  T margin;
};

template <class T>
struct ContactBar {  // adjoints
  Vec<T> n, p;
  T phi;
  Vec<T> xa, va, wa, xb, vb, wb;
  T trs;  // of tr_a + tr_b (constant for free bodies, a function of the joints otherwise)
  Vec<T> psa, psb;  // of rotation increments of the sides through their inverse inertia (diagonal impedance)
};

template <class T>
CF_HD void tangent_basis(Vec<T> n, Vec<T> &u, T &ilen, bool &hx) {
  hx = fabs(n.x) <= T(0.5);
  u = hx ? vec(T(1) - n.x * n.x, -n.x * n.y, -n.x * n.z) : vec(-n.y * n.x, T(1) - n.y * n.y, -n.y * n.z);
  ilen = T(1) / sqrt(dot(u, u));
}

// Exact diagonal impedance of one contact (the form Sec. III.B gives before its
// heuristic): g_f = sum over the contact's bodies of im |u_f|^2 + a_f^T S a_f and
// A_f = 1 / (aa g_f), the facet row acting on a body at lever arm r as linear
// direction u_f and angular direction a_f: tangential d: u = n - mu_t d, a = r x u;
// torsional sigma: u = n, a = r x n - mu_tor sigma n; rolling d: u = n,
// a = r x n - mu_rol d (|u|^2 = 1 + mu_t^2 for the tangential facets).
template <int NF, class T>
CF_HD void diag_dirs(Vec<T> r, Vec<T> n, Vec<T> t1, Vec<T> t2, T mut, T mutor, T murol, Vec<T> *a, T *lin) {
  const Vec<T> rn = cross(r, n);
  if constexpr (NF == 1) {
    a[0] = rn; lin[0] = T(1);
  } else {
    const Vec<T> r1 = cross(r, t1), r2 = cross(r, t2);
    a[0] = rn - mut * r1; a[1] = rn - mut * r2; a[2] = rn + mut * r1; a[3] = rn + mut * r2;
    for (int i = 0; i < 4; ++i) lin[i] = T(1) + mut * mut;
    if constexpr (NF >= 6) {
      a[4] = rn - mutor * n; a[5] = rn + mutor * n;
      lin[4] = lin[5] = T(1);
    }
    if constexpr (NF == 10) {
      a[6] = rn - murol * t1; a[7] = rn - murol * t2; a[8] = rn + murol * t1; a[9] = rn + murol * t2;
      for (int i = 6; i < 10; ++i) lin[i] = T(1);
    }
  }
}

template <int NF, class T>
CF_HD void diag_gains(const ContactIn<T> &C, T *A) {
  T g[NF];
  for (int i = 0; i < NF; ++i) g[i] = T(0);
  for (int side = 0; side < 2; ++side) {
    if (!(side ? C.has_b : C.has_a)) continue;
    const Vec<T> r = C.p - (side ? C.xb : C.xa);
    const T im = side ? C.imb : C.ima;
    const T *S = side ? C.Sb : C.Sa;
    Vec<T> t1, t2;
    {
      Vec<T> u;
      T il;
      bool hx;
      tangent_basis(C.n, u, il, hx);
      t1 = il * u;
      t2 = cross(C.n, t1);
    }
    Vec<T> a[NF];
    T lin[NF];
    diag_dirs<NF>(r, C.n, t1, t2, C.mut, C.mutor, C.murol, a, lin);
    for (int i = 0; i < NF; ++i) g[i] += im * lin[i] + dot(a[i], sym_mul(S, a[i]));
  }
  const T aa = C.k * C.h + C.d;
  for (int i = 0; i < NF; ++i) A[i] = (g[i] > T(0) && aa > T(0)) ? T(1) / (aa * g[i]) : T(0);
}

// Reverse of diag_gains for one side: given gb[f] (the adjoints of g_f), adds
// the adjoints of the lever arm r, of n, t1, t2 and of the side's rotation
// increment (through S).
template <int NF, class T>
CF_HD void diag_side_vjp(Vec<T> r, Vec<T> n, Vec<T> t1, Vec<T> t2, T mut, T mutor, T murol, const T *S,
                         const T *gb, Vec<T> &rb, Vec<T> &nb, Vec<T> &t1b, Vec<T> &t2b, Vec<T> &psib) {
  Vec<T> a[NF];
  T lin[NF];
  diag_dirs<NF>(r, n, t1, t2, mut, mutor, murol, a, lin);
  Vec<T> ab[NF];
  for (int i = 0; i < NF; ++i) {
    const Vec<T> Sa = sym_mul(S, a[i]);
    ab[i] = (T(2) * gb[i]) * Sa;
    psib = psib + (T(2) * gb[i]) * cross(Sa, a[i]);  // d(a^T S a) = 2 dpsi . (S a x a)
  }
  // a = r x u (+ a term free of r): r_bar += u x a_bar, u_bar += a_bar x r
  auto lever = [&](Vec<T> u, Vec<T> abar) {
    rb = rb + cross(u, abar);
    return cross(abar, r);
  };
  if constexpr (NF == 1) {
    nb = nb + lever(n, ab[0]);
  } else {
    Vec<T> ub;
    ub = lever(n - mut * t1, ab[0]); nb = nb + ub; t1b = t1b - mut * ub;
    ub = lever(n - mut * t2, ab[1]); nb = nb + ub; t2b = t2b - mut * ub;
    ub = lever(n + mut * t1, ab[2]); nb = nb + ub; t1b = t1b + mut * ub;
    ub = lever(n + mut * t2, ab[3]); nb = nb + ub; t2b = t2b + mut * ub;
    if constexpr (NF >= 6) {
      nb = nb + lever(n, ab[4]) - mutor * ab[4];
      nb = nb + lever(n, ab[5]) + mutor * ab[5];
    }
    if constexpr (NF == 10) {
      nb = nb + lever(n, ab[6]); t1b = t1b - murol * ab[6];
      nb = nb + lever(n, ab[7]); t2b = t2b - murol * ab[7];
      nb = nb + lever(n, ab[8]); t1b = t1b + murol * ab[8];
      nb = nb + lever(n, ab[9]); t2b = t2b + murol * ab[9];
    }
  }
}

// ------------------------------------------------------------------ learned gains
// The learned gains of Sec. III.B (K and D scaled per facet by a network),
// evaluated in T from the float32 parameters: features (phi, v_n, u_1, u_2,
// 1/tr_s, mu_t, h) normalised, two SiLU layers of 64, one output y_f per
// facet; gain G_f = A exp(clamp(y_f, -ln 256, ln 256)) with A the heuristic
// gain; kept unless the fallback rule rejects the learned impulses (the same
// rule as the forward step: the contact alone along its normal, inverse mass
// tr_s / 3, must not predict more penetration or more normal kinetic energy
// than the heuristic impulses beyond the margin).  The derivative is that of
// this float network on the branch the step takes (kept or not, clamped or
// not); the forward step's bf16 evaluation of it is piecewise constant in its
// inputs and has no useful derivative of its own.
template <class T> CF_HD T silu_t(T z) { return z / (T(1) + exp(-z)); }
template <class T> CF_HD T dsilu_t(T z) {
  const T s = T(1) / (T(1) + exp(-z));
  return s * (T(1) + z * (T(1) - s));
}

template <int NF, class T>
struct LearnedEval {
  T fe[mlp::NIN], z1[mlp::NH], z2[mlp::NH], y[NF], G[NF];
  bool keep;
};

template <int NF, class T>
CF_HD void net_forward(const float *p, LearnedEval<NF, T> &L) {
  using namespace mlp;
  T x[NIN];
  for (int k = 0; k < NIN; ++k) x[k] = (L.fe[k] - T(p[OFF_MEAN + k])) / T(p[OFF_STD + k]);
  for (int j = 0; j < NH; ++j) {
    T s = T(p[OFF_B1 + j]);
    for (int k = 0; k < NIN; ++k) s += x[k] * T(p[OFF_W1 + k * NH + j]);
    L.z1[j] = s;
  }
  T a1[NH];
  for (int k = 0; k < NH; ++k) a1[k] = silu_t(L.z1[k]);
  for (int j = 0; j < NH; ++j) {
    T s = T(p[OFF_B2 + j]);
    for (int k = 0; k < NH; ++k) s += a1[k] * T(p[OFF_W2 + k * NH + j]);
    L.z2[j] = s;
  }
  for (int f = 0; f < NF; ++f) L.y[f] = T(p[OFF_B3 + f]);
  for (int j = 0; j < NH; ++j) {
    const T a = silu_t(L.z2[j]);
    for (int f = 0; f < NF; ++f) L.y[f] += a * T(p[OFF_W3 + j * NOUT + f]);
  }
}

// Adjoints of the features from the adjoints yb of the outputs.
template <int NF, class T>
CF_HD void net_vjp(const float *p, const LearnedEval<NF, T> &L, const T *yb, T *feb) {
  using namespace mlp;
  T z2b[NH], z1b[NH];
  for (int j = 0; j < NH; ++j) {
    T s = T(0);
    for (int f = 0; f < NF; ++f) s += yb[f] * T(p[OFF_W3 + j * NOUT + f]);
    z2b[j] = s * dsilu_t(L.z2[j]);
  }
  for (int k = 0; k < NH; ++k) {
    T s = T(0);
    for (int j = 0; j < NH; ++j) s += z2b[j] * T(p[OFF_W2 + k * NH + j]);
    z1b[k] = s * dsilu_t(L.z1[k]);
  }
  for (int k = 0; k < NIN; ++k) {
    T s = T(0);
    for (int j = 0; j < NH; ++j) s += z1b[j] * T(p[OFF_W1 + k * NH + j]);
    feb[k] = s / T(p[OFF_STD + k]);
  }
}

template <int NF, class T>
CF_HD bool learned_keep(const T *lh, const T *ll, T vn, T phi, T trs, T h, T margin) {
  if (!(trs > T(0))) return false;
  const T winv = trs / T(3);
  T Sh = T(0), Sl = T(0);
  for (int i = 0; i < NF; ++i) {
    Sh += lh[i];
    Sl += ll[i];
  }
  const T vh = vn + winv * Sh, vl = vn + winv * Sl;
  const T ph = fmax(-(phi + h * vh), T(0)), pl = fmax(-(phi + h * vl), T(0));
  const T eh = T(0.5) * vh * vh / winv, el = T(0.5) * vl * vl / winv;
  const T em = T(0.5) * (margin / h) * (margin / h) / winv;
  return pl <= ph + margin && el <= eh + em && isfinite(vl);
}

// Learned gains of one contact from its heuristic gain A0, its normal and
// tangential relative velocities and its facet arguments z_f = -aa s_f + c0.
template <int NF, class T>
CF_HD void learned_eval(const ContactIn<T> &C, T A0, T vn, T u1, T u2, const T *z, LearnedEval<NF, T> &L) {
  L.fe[0] = C.phi; L.fe[1] = vn; L.fe[2] = u1; L.fe[3] = u2;
  L.fe[4] = C.trs > T(0) ? T(1) / C.trs : T(0);
  L.fe[5] = C.mut; L.fe[6] = C.h;
  for (int k = mlp::NFEAT; k < mlp::NIN; ++k) L.fe[k] = T(0);
  net_forward<NF>(C.net, L);
  T lh[NF], ll[NF];
  const T clip = T(mlp::CLIP);
  for (int f = 0; f < NF; ++f) {
    L.G[f] = A0 * exp(fmin(fmax(L.y[f], -clip), clip));
    lh[f] = A0 * fmax(z[f], T(0));
    ll[f] = L.G[f] * fmax(z[f], T(0));
  }
  L.keep = learned_keep<NF>(lh, ll, vn, C.phi, C.trs, C.h, C.margin);
}

// Facet velocity terms s_f (the bracket of -aa s_f in Eq. cf_wrench) in facet order.
template <int NF, class T>
CF_HD void facet_s(const ContactIn<T> &C, Vec<T> n, Vec<T> t1, Vec<T> t2, Vec<T> vrel, Vec<T> wrel, T *s) {
  const T vn = dot(n, vrel);
  if constexpr (NF == 1) {
    s[0] = vn;
  } else {
    const T u1 = dot(t1, vrel), u2 = dot(t2, vrel);
    s[0] = vn - C.mut * u1; s[1] = vn - C.mut * u2; s[2] = vn + C.mut * u1; s[3] = vn + C.mut * u2;
    if constexpr (NF >= 6) {
      const T wt = dot(n, wrel);
      s[4] = vn - C.mutor * wt; s[5] = vn + C.mutor * wt;
    }
    if constexpr (NF == 10) {
      const T o1 = dot(t1, wrel), o2 = dot(t2, wrel);
      s[6] = vn - C.murol * o1; s[7] = vn - C.murol * o2; s[8] = vn + C.murol * o1; s[9] = vn + C.murol * o2;
    }
  }
}

// Facet impulses and the wrench on body b (f, tb) and on body a (-f, ta).
// NET: whether the learned gains can occur (C.net); a caller without them
// leaves the network's code out.
template <int NF, class T, bool NET = true>
CF_HD void contact_forward(const ContactIn<T> &C, const Impedance<T> &P, T *lam, Vec<T> &f, Vec<T> &ta,
                           Vec<T> &tb) {
  Vec<T> u;
  T il;
  bool hx;
  tangent_basis(C.n, u, il, hx);
  const Vec<T> t1 = il * u, t2 = cross(C.n, t1);
  const Vec<T> ra = C.p - C.xa, rb = C.p - C.xb;
  Vec<T> vrel = vec(T(0), T(0), T(0)), wrel = vrel;
  if (C.has_b) { vrel = C.vb + cross(C.wb, rb); wrel = C.wb; }
  if (C.has_a) { vrel = vrel - (C.va + cross(C.wa, ra)); wrel = wrel - C.wa; }
  T drho;
  const T A0 = C.trs > T(0) ? impedance_rho(C.phi, P, drho) / C.trs : T(0);
  T Af[NF];
  if (C.diag) diag_gains<NF>(C, Af);
  else for (int i = 0; i < NF; ++i) Af[i] = A0;
  const T aa = C.k * C.h + C.d, c0 = -C.k * C.phi;
  const T vn = dot(C.n, vrel);
  if (NET && C.net && !C.diag) {
    T s[NF], z[NF];
    facet_s<NF>(C, C.n, t1, t2, vrel, wrel, s);
    for (int i = 0; i < NF; ++i) z[i] = -aa * s[i] + c0;
    LearnedEval<NF, T> L;
    learned_eval<NF>(C, A0, vn, dot(t1, vrel), dot(t2, vrel), z, L);
    if (L.keep)
      for (int i = 0; i < NF; ++i) Af[i] = L.G[i];
  }
  Vec<T> tc = vec(T(0), T(0), T(0));
  if constexpr (NF == 1) {
    lam[0] = Af[0] * fmax(-aa * vn + c0, T(0));
    f = lam[0] * C.n;
  } else {
    const T u1 = dot(t1, vrel), u2 = dot(t2, vrel);
    lam[0] = Af[0] * fmax(-aa * (vn - C.mut * u1) + c0, T(0));
    lam[1] = Af[1] * fmax(-aa * (vn - C.mut * u2) + c0, T(0));
    lam[2] = Af[2] * fmax(-aa * (vn + C.mut * u1) + c0, T(0));
    lam[3] = Af[3] * fmax(-aa * (vn + C.mut * u2) + c0, T(0));
    T N = lam[0] + lam[1] + lam[2] + lam[3];
    const T e1 = -C.mut * (lam[0] - lam[2]), e2 = -C.mut * (lam[1] - lam[3]);
    if constexpr (NF >= 6) {
      const T wt = dot(C.n, wrel);
      lam[4] = Af[4] * fmax(-aa * (vn - C.mutor * wt) + c0, T(0));
      lam[5] = Af[5] * fmax(-aa * (vn + C.mutor * wt) + c0, T(0));
      N += lam[4] + lam[5];
      tc = (-C.mutor * (lam[4] - lam[5])) * C.n;
    }
    if constexpr (NF == 10) {
      const T o1 = dot(t1, wrel), o2 = dot(t2, wrel);
      lam[6] = Af[6] * fmax(-aa * (vn - C.murol * o1) + c0, T(0));
      lam[7] = Af[7] * fmax(-aa * (vn - C.murol * o2) + c0, T(0));
      lam[8] = Af[8] * fmax(-aa * (vn + C.murol * o1) + c0, T(0));
      lam[9] = Af[9] * fmax(-aa * (vn + C.murol * o2) + c0, T(0));
      N += lam[6] + lam[7] + lam[8] + lam[9];
      tc = tc + (-C.murol * (lam[6] - lam[8])) * t1 + (-C.murol * (lam[7] - lam[9])) * t2;
    }
    f = N * C.n + e1 * t1 + e2 * t2;
  }
  tb = cross(rb, f) + tc;
  ta = -(cross(ra, f) + tc);
}

// Given the adjoints of the wrenches the contact adds to body a (Fa, Ta) and
// body b (Fb, Tb): adjoints of n, phi, p and of both bodies' COM and smooth
// velocities.  NET as for contact_forward.
template <int NF, class T, bool NET = true>
CF_HD void contact_vjp(const ContactIn<T> &C, const Impedance<T> &P, Vec<T> Fa_b, Vec<T> Ta_b, Vec<T> Fb_b,
                       Vec<T> Tb_b, ContactBar<T> &o) {
  const Vec<T> Z = vec(T(0), T(0), T(0));
  Vec<T> u;
  T il;
  bool hx;
  tangent_basis(C.n, u, il, hx);
  const Vec<T> n = C.n, t1 = il * u, t2 = cross(n, t1);
  const Vec<T> ra = C.p - C.xa, rb = C.p - C.xb;
  Vec<T> vrel = Z, wrel = Z;
  if (C.has_b) { vrel = C.vb + cross(C.wb, rb); wrel = C.wb; }
  if (C.has_a) { vrel = vrel - (C.va + cross(C.wa, ra)); wrel = wrel - C.wa; }
  T drho = T(0);
  T Af[NF];
  if (C.diag) {
    diag_gains<NF>(C, Af);
  } else {
    const T rho = impedance_rho(C.phi, P, drho);
    for (int i = 0; i < NF; ++i) Af[i] = C.trs > T(0) ? rho / C.trs : T(0);
  }
  const T aa = C.k * C.h + C.d, c0 = -C.k * C.phi;
  const T vn = dot(n, vrel);
  const bool learned = NET && C.net && !C.diag;
  LearnedEval<NF, T> L;
  L.keep = false;
  if (learned) {
    T s0[NF], z0[NF];
    facet_s<NF>(C, n, t1, t2, vrel, wrel, s0);
    for (int i = 0; i < NF; ++i) z0[i] = -aa * s0[i] + c0;
    learned_eval<NF>(C, Af[0], vn, dot(t1, vrel), dot(t2, vrel), z0, L);
  }
  const T A0 = Af[0];
  if (L.keep)
    for (int i = 0; i < NF; ++i) Af[i] = L.G[i];
  T s[NF], z[NF], lam[NF];
  // facet velocity term s_f (the bracket of -aa * s_f) in facet order
  if constexpr (NF == 1) {
    s[0] = vn;
  } else {
    const T u1 = dot(t1, vrel), u2 = dot(t2, vrel);
    s[0] = vn - C.mut * u1; s[1] = vn - C.mut * u2; s[2] = vn + C.mut * u1; s[3] = vn + C.mut * u2;
    if constexpr (NF >= 6) {
      const T wt = dot(n, wrel);
      s[4] = vn - C.mutor * wt; s[5] = vn + C.mutor * wt;
    }
    if constexpr (NF == 10) {
      const T o1 = dot(t1, wrel), o2 = dot(t2, wrel);
      s[6] = vn - C.murol * o1; s[7] = vn - C.murol * o2; s[8] = vn + C.murol * o1; s[9] = vn + C.murol * o2;
    }
  }
  T N = T(0);
  for (int i = 0; i < NF; ++i) {
    z[i] = -aa * s[i] + c0;
    lam[i] = Af[i] * fmax(z[i], T(0));
    N += lam[i];
  }
  Vec<T> f;
  T e1 = T(0), e2 = T(0);
  if constexpr (NF == 1) {
    f = lam[0] * n;
  } else {
    e1 = -C.mut * (lam[0] - lam[2]);
    e2 = -C.mut * (lam[1] - lam[3]);
    f = N * n + e1 * t1 + e2 * t2;
  }
  // ---- reverse
  // wrenches: b gets (f, rb x f + tc), a gets (-f, -(ra x f + tc))
  const Vec<T> Tb = C.has_b ? Tb_b : Z, Ta = C.has_a ? -Ta_b : Z;
  Vec<T> fb = (C.has_b ? Fb_b : Z) - (C.has_a ? Fa_b : Z) + cross(Tb, rb) + cross(Ta, ra);
  Vec<T> rbb = cross(f, Tb), rab = cross(f, Ta);
  const Vec<T> tcb = Tb + Ta;
  Vec<T> nb = Z, t1b = Z, t2b = Z;
  T lb[NF];
  if constexpr (NF == 1) {
    lb[0] = dot(fb, n);
    nb = lam[0] * fb;
  } else {
    const T Nb = dot(fb, n), e1b = dot(fb, t1), e2b = dot(fb, t2);
    nb = N * fb;
    t1b = e1 * fb;
    t2b = e2 * fb;
    for (int i = 0; i < NF; ++i) lb[i] = Nb;
    lb[0] -= C.mut * e1b; lb[2] += C.mut * e1b;
    lb[1] -= C.mut * e2b; lb[3] += C.mut * e2b;
    if constexpr (NF >= 6) {  // tc = -mutor (l4 - l5) n - murol ((l6 - l8) t1 + (l7 - l9) t2)
      const T g = dot(n, tcb);
      nb = nb + (-C.mutor * (lam[4] - lam[5])) * tcb;
      lb[4] -= C.mutor * g; lb[5] += C.mutor * g;
    }
    if constexpr (NF == 10) {
      const T g1 = dot(t1, tcb), g2 = dot(t2, tcb);
      t1b = t1b + (-C.murol * (lam[6] - lam[8])) * tcb;
      t2b = t2b + (-C.murol * (lam[7] - lam[9])) * tcb;
      lb[6] -= C.murol * g1; lb[8] += C.murol * g1;
      lb[7] -= C.murol * g2; lb[9] += C.murol * g2;
    }
  }
  // lam_f = A_f max(z_f, 0), z_f = -aa s_f + c0
  T Ab = T(0), c0b = T(0);
  T sb[NF], Afb[NF];
  for (int i = 0; i < NF; ++i) {
    const T zb = z[i] > T(0) ? Af[i] * lb[i] : T(0);
    Afb[i] = z[i] > T(0) ? lb[i] * z[i] : T(0);
    Ab += Afb[i];
    sb[i] = -aa * zb;
    c0b += zb;
  }
  T phib = -C.k * c0b;
  T fvn = T(0), fu1 = T(0), fu2 = T(0);  // adjoints of the learned gains' features v_n, u_1, u_2
  o.trs = T(0);
  o.psa = o.psb = Z;
  Vec<T> rab_d = Z, rbb_d = Z;
  if (C.diag) {
    // A_f = 1 / (aa g_f): g_bar = -A_bar A_f / g_f = -A_bar aa A_f^2
    T gb[NF];
    for (int i = 0; i < NF; ++i) gb[i] = -Afb[i] * aa * Af[i] * Af[i];
    if (C.has_a) diag_side_vjp<NF>(ra, n, t1, t2, C.mut, C.mutor, C.murol, C.Sa, gb, rab_d, nb, t1b, t2b, o.psa);
    if (C.has_b) diag_side_vjp<NF>(rb, n, t1, t2, C.mut, C.mutor, C.murol, C.Sb, gb, rbb_d, nb, t1b, t2b, o.psb);
  } else if (L.keep) {
    // G_f = A exp(clamp(y_f)), A = rho(phi) / trs, y = net(phi, v_n, u_1, u_2, 1/trs, mu_t, h)
    T A0b = T(0), yb[NF], feb[mlp::NIN];
    const T clip = T(mlp::CLIP);
    for (int i = 0; i < NF; ++i) {
      A0b += Afb[i] * (L.G[i] / A0);
      yb[i] = fabs(L.y[i]) < clip ? Afb[i] * L.G[i] : T(0);
    }
    net_vjp<NF>(C.net, L, yb, feb);
    phib += A0b * drho / C.trs + feb[0];
    o.trs = -A0b * A0 / C.trs - feb[4] / (C.trs * C.trs);
    fvn = feb[1];
    fu1 = feb[2];
    fu2 = feb[3];
  } else if (C.trs > T(0)) {  // A = rho(phi) / trs
    phib += Ab * drho / C.trs;
    o.trs = -Ab * Af[0] / C.trs;
  }
  // s_f in terms of vn, u1, u2, wt, o1, o2 (and the learned gains' features)
  T vnb = fvn;
  for (int i = 0; i < NF; ++i) vnb += sb[i];
  Vec<T> vrelb = vnb * n + fu1 * t1 + fu2 * t2, wrelb = Z;
  nb = nb + vnb * vrel;
  t1b = t1b + fu1 * vrel;
  t2b = t2b + fu2 * vrel;
  if constexpr (NF > 1) {
    const T u1b = -C.mut * (sb[0] - sb[2]), u2b = -C.mut * (sb[1] - sb[3]);
    t1b = t1b + u1b * vrel;
    t2b = t2b + u2b * vrel;
    vrelb = vrelb + u1b * t1 + u2b * t2;
    if constexpr (NF >= 6) {
      const T wtb = -C.mutor * (sb[4] - sb[5]);
      nb = nb + wtb * wrel;
      wrelb = wrelb + wtb * n;
    }
    if constexpr (NF == 10) {
      const T o1b = -C.murol * (sb[6] - sb[8]), o2b = -C.murol * (sb[7] - sb[9]);
      t1b = t1b + o1b * wrel;
      t2b = t2b + o2b * wrel;
      wrelb = wrelb + o1b * t1 + o2b * t2;
    }
  }
  // vrel = vb + wb x rb - va - wa x ra ; wrel = wb - wa
  o.va = o.wa = o.vb = o.wb = Z;
  if (C.has_b) {
    o.vb = vrelb;
    o.wb = cross(rb, vrelb) + wrelb;
    rbb = rbb + cross(vrelb, C.wb);
  }
  if (C.has_a) {
    o.va = -vrelb;
    o.wa = -(cross(ra, vrelb) + wrelb);
    rab = rab - cross(vrelb, C.wa);
  }
  rab = rab + rab_d;
  rbb = rbb + rbb_d;
  // ra = p - xa, rb = p - xb
  o.p = rab + rbb;
  o.xa = -rab;
  o.xb = -rbb;
  // t2 = n x t1 ; t1 = u / |u|, u = hlp - (hlp . n) n
  nb = nb + cross(t1, t2b);
  t1b = t1b + cross(t2b, n);
  const Vec<T> ub = il * (t1b - dot(t1, t1b) * t1);
  const Vec<T> hlp = hx ? vec(T(1), T(0), T(0)) : vec(T(0), T(1), T(0));
  const T hn = hx ? n.x : n.y;
  nb = nb - dot(n, ub) * hlp - hn * ub;
  o.n = nb;
  o.phi = phib;
}

// ------------------------------------------------------------------ contact geometry
// Gap, normal and point from the geoms' world poses (narrow phase), and the
// adjoint of the poses given the adjoints of (n, phi, p).  The geometry is
// rebuilt from the contact's own (n, phi, p): sphere centres c = p -/+ (r +
// phi/2) n, the point of a plane contact c = p + (rad + phi/2) n.
//
// sphere-sphere: d = cb - ca, n = d / |d|, phi = |d| - ra - rb, p = ca + (ra + phi/2) n.
template <class T>
CF_HD void sphere_pair_forward(Vec<T> ca, Vec<T> cb, T ra, T rb, Vec<T> &n, T &phi, Vec<T> &p) {
  const Vec<T> d = cb - ca;
  const T dist = sqrt(dot(d, d));
  n = dist >= T(1e-12) ? (T(1) / dist) * d : vec(T(0), T(0), T(1));
  phi = dist - ra - rb;
  p = ca + (ra + T(0.5) * phi) * n;
}

template <class T>
CF_HD void sphere_pair_vjp(Vec<T> n, T phi, T ra, T rb, Vec<T> nb, T phib, Vec<T> pb, Vec<T> &cab, Vec<T> &cbb) {
  const T dist = phi + ra + rb;
  cab = pb;
  const Vec<T> n2 = nb + (ra + T(0.5) * phi) * pb;
  const T phi2 = phib + T(0.5) * dot(n, pb);
  Vec<T> db = phi2 * n;
  if (dist >= T(1e-12)) db = db + (T(1) / dist) * (n2 - dot(n, n2) * n);
  cbb = db;
  cab = cab - db;
}

// plane (point pp, unit normal n) against a point c with radius rad
// (sphere centre, capsule end, box corner with rad = 0):
// phi = n.(c - pp) - rad, p = c - (rad + phi/2) n.
template <class T>
CF_HD void plane_point_forward(Vec<T> pp, Vec<T> n, Vec<T> c, T rad, T &phi, Vec<T> &p) {
  phi = dot(n, c - pp) - rad;
  p = c - (rad + T(0.5) * phi) * n;
}

// Adjoints of c, of the plane point pp and of the plane normal n.
template <class T>
CF_HD void plane_point_vjp(Vec<T> pp, Vec<T> n, Vec<T> c, T rad, T phi, Vec<T> nb, T phib, Vec<T> pb, Vec<T> &cb,
                           Vec<T> &ppb, Vec<T> &nnb) {
  cb = pb;
  Vec<T> n2 = nb - (rad + T(0.5) * phi) * pb;
  const T phi2 = phib - T(0.5) * dot(n, pb);
  n2 = n2 + phi2 * (c - pp);
  cb = cb + phi2 * n;
  ppb = -phi2 * n;
  nnb = n2;
}

// line (point e0, unit direction u; a box edge) against a point c with radius
// rad: d = c - e0, d_perp = d - (u.d) u, n = d_perp / |d_perp|,
// phi = |d_perp| - rad, p = c - (rad + phi/2) n.
template <class T>
CF_HD void line_point_forward(Vec<T> e0, Vec<T> u, Vec<T> c, T rad, Vec<T> &n, T &phi, Vec<T> &p) {
  const Vec<T> d = c - e0;
  const Vec<T> dp = d - dot(u, d) * u;
  const T dist = sqrt(dot(dp, dp));
  n = (T(1) / dist) * dp;
  phi = dist - rad;
  p = c - (rad + T(0.5) * phi) * n;
}

// Adjoints of c, of the line point e0 and of the line direction u.
template <class T>
CF_HD void line_point_vjp(Vec<T> e0, Vec<T> u, Vec<T> c, T rad, Vec<T> n, T phi, Vec<T> nb, T phib, Vec<T> pb,
                          Vec<T> &cb, Vec<T> &e0b, Vec<T> &ub) {
  const Vec<T> d = c - e0;
  const T dist = phi + rad;
  const Vec<T> n2 = nb - (rad + T(0.5) * phi) * pb;
  const T phi2 = phib - T(0.5) * dot(n, pb);
  const Vec<T> dpb = phi2 * n + (T(1) / dist) * (n2 - dot(n, n2) * n);
  const Vec<T> db = dpb - dot(u, dpb) * u;
  ub = -dot(u, d) * dpb - dot(u, dpb) * d;
  cb = pb + db;
  e0b = -db;
}

#undef CF_HD

}  // namespace adj
}  // namespace cf
