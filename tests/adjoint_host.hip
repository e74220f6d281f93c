// Host-side check of the reverse-mode pieces in cf_adjoint.h: each vector-
// Jacobian product, instantiated in float64, against central differences of
// the matching forward piece.  Built by tests/test_adjoint_host.py with hipcc
// and run on the CPU (no device code is launched).
#include <cstdio>
#include <cstdlib>
#include <cmath>
#include <random>
#include <vector>

#include "../paper_2603_12185_amd/csrc/cf_adjoint.h"
#include "../paper_2603_12185_amd/csrc/cf_artadj.h"

using namespace cf::adj;
typedef double D;
typedef Vec<D> V;

static std::mt19937_64 rng(12345);
static D U(D a, D b) { return std::uniform_real_distribution<D>(a, b)(rng); }
static V rv(D s) { return vec(U(-s, s), U(-s, s), U(-s, s)); }
static D nrm(const std::vector<D> &x) {
  D s = 0;
  for (D v : x) s += v * v;
  return std::sqrt(s);
}

static int failures = 0;
static void report(const char *name, const std::vector<D> &an, const std::vector<D> &fd, D tol) {
  std::vector<D> d(an.size());
  for (size_t i = 0; i < an.size(); ++i) d[i] = an[i] - fd[i];
  const D rel = nrm(d) / (nrm(fd) + 1e-300);
  const bool ok = rel < tol;
  if (!ok) ++failures;
  printf("%-34s n=%2zu |g|=%.3e rel=%.2e %s\n", name, an.size(), nrm(fd), rel, ok ? "ok" : "FAIL");
  if (!ok)
    for (size_t i = 0; i < an.size(); ++i) printf("   %2zu  an %+.9e  fd %+.9e\n", i, an[i], fd[i]);
}

// central differences of scalar L(x) over every component of x
template <class F>
static std::vector<D> fd_grad(std::vector<D> x, F L, D eps = 1e-6) {
  std::vector<D> g(x.size());
  for (size_t i = 0; i < x.size(); ++i) {
    const D x0 = x[i];
    x[i] = x0 + eps;
    const D lp = L(x);
    x[i] = x0 - eps;
    const D lm = L(x);
    x[i] = x0;
    g[i] = (lp - lm) / (2 * eps);
  }
  return g;
}

static void put(std::vector<D> &x, V v) { x.push_back(v.x); x.push_back(v.y); x.push_back(v.z); }
static V get(const std::vector<D> &x, size_t i) { return vec(x[i], x[i + 1], x[i + 2]); }
static D vdot(V a, V b) { return dot(a, b); }

// ----------------------------------------------------------------------------
static void check_predict(int trial) {
  BodyPredict<D> B;
  B.m = U(0.05, 2.0);
  for (int i = 0; i < 3; ++i) B.d[i] = U(1e-4, 1e-2);
  for (int i = 0; i < 4; ++i) B.q[i] = U(-1, 1);
  B.v = rv(1.0); B.w = rv(20.0); B.f = rv(5.0); B.t = rv(0.05); B.g = vec(0.0, 0.0, -9.81); B.h = 0.002;
  const V vsb = rv(1.0), wsb = rv(1.0);
  // pack inputs: q(4) v w f t
  std::vector<D> x(B.q, B.q + 4);
  put(x, B.v); put(x, B.w); put(x, B.f); put(x, B.t);
  auto L = [&](const std::vector<D> &y) {
    BodyPredict<D> C = B;
    for (int i = 0; i < 4; ++i) C.q[i] = y[i];
    C.v = get(y, 4); C.w = get(y, 7); C.f = get(y, 10); C.t = get(y, 13);
    V vs, ws;
    predict_forward(C, vs, ws);
    return vdot(vs, vsb) + vdot(ws, wsb);
  };
  V vb, wb, fb, tb, psi = vec(0.0, 0.0, 0.0);
  predict_vjp(B, vsb, wsb, vb, wb, fb, tb, psi);
  D qb[4] = {0, 0, 0, 0};
  quat_grad_from_psi(B.q, psi, qb);
  std::vector<D> an(qb, qb + 4);
  put(an, vb); put(an, wb); put(an, fb); put(an, tb);
  char name[64];
  snprintf(name, sizeof name, "predict #%d", trial);
  report(name, an, fd_grad(x, L), 1e-7);
}

static void check_update(int trial, D wscale) {
  BodyUpdate<D> B;
  B.m = U(0.05, 2.0);
  for (int i = 0; i < 3; ++i) B.d[i] = U(1e-4, 1e-2);
  for (int i = 0; i < 4; ++i) B.q[i] = U(-1, 1);
  B.x = rv(0.3); B.vs = rv(1.0); B.ws = rv(wscale); B.F = rv(0.01); B.Tq = rv(1e-4); B.h = 0.002;
  const V xpb = rv(1.0), vpb = rv(1.0), wpb = rv(1.0);
  const D qpb[4] = {U(-1, 1), U(-1, 1), U(-1, 1), U(-1, 1)};
  std::vector<D> x(B.q, B.q + 4);
  put(x, B.x); put(x, B.vs); put(x, B.ws); put(x, B.F); put(x, B.Tq);
  auto L = [&](const std::vector<D> &y) {
    BodyUpdate<D> C = B;
    for (int i = 0; i < 4; ++i) C.q[i] = y[i];
    C.x = get(y, 4); C.vs = get(y, 7); C.ws = get(y, 10); C.F = get(y, 13); C.Tq = get(y, 16);
    V xp, vp, wp;
    D qp[4];
    update_forward(C, xp, qp, vp, wp);
    return vdot(xp, xpb) + vdot(vp, vpb) + vdot(wp, wpb) + qp[0] * qpb[0] + qp[1] * qpb[1] + qp[2] * qpb[2] +
           qp[3] * qpb[3];
  };
  V xb, vsb, wsb, Fb, Tb, psi = vec(0.0, 0.0, 0.0);
  D qb[4] = {0, 0, 0, 0};
  update_vjp(B, xpb, qpb, vpb, wpb, xb, qb, vsb, wsb, Fb, Tb, psi);
  quat_grad_from_psi(B.q, psi, qb);
  std::vector<D> an(qb, qb + 4);
  put(an, xb); put(an, vsb); put(an, wsb); put(an, Fb); put(an, Tb);
  char name[64];
  snprintf(name, sizeof name, "update |w|~%g #%d", wscale, trial);
  report(name, an, fd_grad(x, L), 1e-6);
}

static Impedance<D> imp() { return {0.9, 0.95, 0.001, 0.5, 2.0}; }

// Learned gains: whether the fallback rule keeps them and which outputs are
// clamped (recomputed here from the same pieces contact_forward uses).
template <int NF>
static unsigned learned_pattern(const ContactIn<D> &C) {
  if (!C.net) return 0;
  V u;
  D il;
  bool hx;
  tangent_basis(C.n, u, il, hx);
  const V t1 = il * u, t2 = cross(C.n, t1);
  const V ra = C.p - C.xa, rb = C.p - C.xb;
  V vrel = vec(0.0, 0.0, 0.0), wrel = vrel;
  if (C.has_b) { vrel = C.vb + cross(C.wb, rb); wrel = C.wb; }
  if (C.has_a) { vrel = vrel - (C.va + cross(C.wa, ra)); wrel = wrel - C.wa; }
  D drho;
  const D A0 = impedance_rho(C.phi, imp(), drho) / C.trs;
  D s[NF], z[NF];
  facet_s<NF>(C, C.n, t1, t2, vrel, wrel, s);
  for (int i = 0; i < NF; ++i) z[i] = -(C.k * C.h + C.d) * s[i] - C.k * C.phi;
  LearnedEval<NF, D> L;
  learned_eval<NF>(C, A0, dot(C.n, vrel), dot(t1, vrel), dot(t2, vrel), z, L);
  unsigned m = L.keep ? 1u : 0u;
  for (int f = 0; f < NF; ++f) m |= (std::fabs(L.y[f]) >= cf::mlp::CLIP ? 1u : 0u) << (1 + f);
  return m;
}

// Which branch each non-smooth operation of the contact takes: facet
// activity, the clamp of x, the sign of phi, the tangent helper, and for
// learned gains the fallback decision and the output clamps.
template <int NF>
static unsigned pattern(const ContactIn<D> &C) {
  D lam[NF];
  V f, ta, tb;
  contact_forward<NF>(C, imp(), lam, f, ta, tb);
  unsigned m = 0;
  for (int i = 0; i < NF; ++i) m |= (lam[i] > 0.0 ? 1u : 0u) << i;
  m |= (std::fabs(C.phi) >= imp().width ? 1u : 0u) << 12;
  m |= (C.phi > 0.0 ? 1u : 0u) << 13;
  m |= (std::fabs(C.n.x) <= 0.5 ? 1u : 0u) << 14;
  m |= learned_pattern<NF>(C) << 16;
  return m;
}

// World inverse inertia R(q) diag(d) R(q)^T of a body with quaternion q.
static void inv_inertia(const D *q, const D *d, D *S) {
  D R[9];
  rot_of_quat(q, R);
  rot_diag_rot(R, d, S);
}

template <int NF>
static void make_contact(ContactIn<D> &C, bool has_a, bool has_b, D phi_scale, const float *net = nullptr,
                         D margin = 0) {
  C.diag = false;
  C.net = net;
  C.margin = margin;
  C.ima = C.imb = 0;
  for (int i = 0; i < 6; ++i) C.Sa[i] = C.Sb[i] = 0;
  for (;;) {
    C.n = rv(1.0);
    const D l = std::sqrt(dot(C.n, C.n));
    C.n = (1.0 / l) * C.n;
    C.phi = U(-phi_scale, phi_scale * 0.2);
    C.p = rv(0.3);
    C.xa = C.p + rv(0.05); C.xb = C.p + rv(0.05);
    C.va = rv(0.05); C.vb = rv(0.05); C.wa = rv(2.0); C.wb = rv(2.0);
    C.has_a = has_a; C.has_b = has_b;
    C.trs = (has_a ? 3.0 / U(0.05, 1) : 0.0) + (has_b ? 3.0 / U(0.05, 1) : 0.0);
    C.mut = U(0.3, 1.0); C.mutor = U(0.001, 0.005); C.murol = U(1e-4, 5e-4);
    C.h = 0.002; C.k = 0.1; C.d = 0.001;
    // keep it only if no branch changes within 1e-5 of any input
    const unsigned p0 = pattern<NF>(C);
    bool same = true;
    D *fields[] = {&C.n.x, &C.n.y, &C.n.z, &C.phi, &C.p.x, &C.p.y, &C.p.z, &C.xa.x, &C.xa.y, &C.xa.z,
                   &C.va.x, &C.va.y, &C.va.z, &C.wa.x, &C.wa.y, &C.wa.z, &C.xb.x, &C.xb.y, &C.xb.z,
                   &C.vb.x, &C.vb.y, &C.vb.z, &C.wb.x, &C.wb.y, &C.wb.z};
    for (D *f : fields)
      for (D e : {-1e-5, 1e-5}) {
        const D f0 = *f;
        *f = f0 + e;
        same = same && pattern<NF>(C) == p0;
        *f = f0;
      }
    if (same && (p0 & ((1u << NF) - 1))) return;  // at least one facet active
  }
}

// diag: the exact diagonal impedance, the sides' inverse inertias rotated by
// quaternions that are inputs of the check too (their adjoints reach them
// through the rotation increments psa, psb).
template <int NF>
static void check_contact(int trial, bool has_a, bool has_b, D phi_scale, bool diag = false,
                          const float *net = nullptr, D margin = 0) {
  ContactIn<D> C;
  make_contact<NF>(C, has_a, has_b, phi_scale, net, margin);
  D qa[4], qb[4], da[3], db[3];
  for (int i = 0; i < 4; ++i) { qa[i] = U(-1, 1); qb[i] = U(-1, 1); }
  for (int i = 0; i < 3; ++i) { da[i] = 1.0 / U(1e-4, 1e-3); db[i] = 1.0 / U(1e-4, 1e-3); }
  if (diag) {
    C.diag = true;
    C.ima = 1.0 / U(0.1, 1.0);
    C.imb = 1.0 / U(0.1, 1.0);
    inv_inertia(qa, da, C.Sa);
    inv_inertia(qb, db, C.Sb);
  }
  const V Fab = rv(1.0), Tab = rv(1.0), Fbb = rv(1.0), Tbb = rv(1.0);
  std::vector<D> x;
  put(x, C.n); x.push_back(C.phi); put(x, C.p);
  put(x, C.xa); put(x, C.va); put(x, C.wa); put(x, C.xb); put(x, C.vb); put(x, C.wb);
  x.push_back(C.trs);
  for (int i = 0; i < 4; ++i) x.push_back(qa[i]);
  for (int i = 0; i < 4; ++i) x.push_back(qb[i]);
  auto L = [&](const std::vector<D> &y) {
    ContactIn<D> K = C;
    K.n = get(y, 0); K.phi = y[3]; K.p = get(y, 4);
    K.xa = get(y, 7); K.va = get(y, 10); K.wa = get(y, 13); K.xb = get(y, 16); K.vb = get(y, 19); K.wb = get(y, 22);
    K.trs = y[25];
    if (diag) {
      inv_inertia(&y[26], da, K.Sa);
      inv_inertia(&y[30], db, K.Sb);
    }
    D lam[NF];
    V f, ta, tb;
    contact_forward<NF>(K, imp(), lam, f, ta, tb);
    D s = 0;
    if (K.has_a) s += -vdot(f, Fab) + vdot(ta, Tab);
    if (K.has_b) s += vdot(f, Fbb) + vdot(tb, Tbb);
    return s;
  };
  ContactBar<D> o;
  contact_vjp<NF>(C, imp(), Fab, Tab, Fbb, Tbb, o);
  std::vector<D> an;
  put(an, o.n); an.push_back(o.phi); put(an, o.p);
  put(an, o.xa); put(an, o.va); put(an, o.wa); put(an, o.xb); put(an, o.vb); put(an, o.wb);
  an.push_back(o.trs);
  D gqa[4] = {0, 0, 0, 0}, gqb[4] = {0, 0, 0, 0};
  quat_grad_from_psi(qa, o.psa, gqa);
  quat_grad_from_psi(qb, o.psb, gqb);
  for (int i = 0; i < 4; ++i) an.push_back(gqa[i]);
  for (int i = 0; i < 4; ++i) an.push_back(gqb[i]);
  char name[80];
  snprintf(name, sizeof name, "contact nf=%d a=%d b=%d phi~%g%s%s #%d", NF, has_a, has_b, phi_scale,
           diag ? " diag" : "", net ? (learned_pattern<NF>(C) & 1u ? " learned" : " learned-fallback") : "",
           trial);
  report(name, an, fd_grad(x, L, 1e-7), 2e-6);
}

// A random learned-gain network (cf_mlp.h layout) with feature scales of a
// contact: outputs of order one, so the gains vary by factors of e.
static std::vector<float> random_net() {
  using namespace cf::mlp;
  std::vector<float> p(NPARAM, 0.f);
  const float mean[NFEAT] = {-0.002f, -0.02f, 0.f, 0.f, 0.1f, 0.6f, 0.002f};
  const float sd[NFEAT] = {0.005f, 0.05f, 0.05f, 0.05f, 0.1f, 0.2f, 1.f};
  for (int k = 0; k < NIN; ++k) {
    p[OFF_MEAN + k] = k < NFEAT ? mean[k] : 0.f;
    p[OFF_STD + k] = k < NFEAT ? sd[k] : 1.f;
  }
  for (int i = 0; i < NIN * NH; ++i) p[OFF_W1 + i] = (float)U(-0.6, 0.6);
  for (int i = 0; i < NH; ++i) p[OFF_B1 + i] = (float)U(-0.3, 0.3);
  for (int i = 0; i < NH * NH; ++i) p[OFF_W2 + i] = (float)U(-0.25, 0.25);
  for (int i = 0; i < NH; ++i) p[OFF_B2 + i] = (float)U(-0.3, 0.3);
  for (int i = 0; i < NH * NOUT; ++i) p[OFF_W3 + i] = (float)U(-0.3, 0.3);
  for (int i = 0; i < NOUT; ++i) p[OFF_B3 + i] = (float)U(-0.5, 0.5);
  return p;
}

static void check_sphere_pair(int trial) {
  const V ca = rv(0.3), cb = ca + rv(0.06);
  const D ra = U(0.02, 0.05), rb = U(0.02, 0.05);
  const V nb = rv(1.0), pb = rv(1.0);
  const D phib = U(-1, 1);
  std::vector<D> x;
  put(x, ca); put(x, cb);
  auto L = [&](const std::vector<D> &y) {
    V n, p;
    D phi;
    sphere_pair_forward(get(y, 0), get(y, 3), ra, rb, n, phi, p);
    return vdot(n, nb) + phi * phib + vdot(p, pb);
  };
  V n, p;
  D phi;
  sphere_pair_forward(ca, cb, ra, rb, n, phi, p);
  V cab, cbb;
  sphere_pair_vjp(n, phi, ra, rb, nb, phib, pb, cab, cbb);
  std::vector<D> an;
  put(an, cab); put(an, cbb);
  char name[64];
  snprintf(name, sizeof name, "sphere pair #%d", trial);
  report(name, an, fd_grad(x, L), 1e-7);
}

// plane attached to a rotating body: pp = x + R(q) o, n = R(q) R0 e_z; the
// point c = y + R(qc) oc on another body.  Checks plane_point_vjp and the
// conversion of point and direction adjoints to body pose adjoints.
static void check_plane_point(int trial) {
  D q[4], qc[4];
  for (int i = 0; i < 4; ++i) { q[i] = U(-1, 1); qc[i] = U(-1, 1); }
  const V x = rv(0.3), o = rv(0.1), y = rv(0.3), oc = rv(0.05);
  const D rad = U(0.0, 0.05);
  const V nb = rv(1.0), pb = rv(1.0);
  const D phib = U(-1, 1);
  auto geom = [&](const D *qq, V xx, const D *qqc, V yy, V &pp, V &n, V &c) {
    D R[9], Rc[9];
    rot_of_quat(qq, R);
    rot_of_quat(qqc, Rc);
    pp = xx + vec(R[0] * o.x + R[1] * o.y + R[2] * o.z, R[3] * o.x + R[4] * o.y + R[5] * o.z,
                  R[6] * o.x + R[7] * o.y + R[8] * o.z);
    n = vec(R[2], R[5], R[8]);
    c = yy + vec(Rc[0] * oc.x + Rc[1] * oc.y + Rc[2] * oc.z, Rc[3] * oc.x + Rc[4] * oc.y + Rc[5] * oc.z,
                 Rc[6] * oc.x + Rc[7] * oc.y + Rc[8] * oc.z);
  };
  std::vector<D> X(q, q + 4);
  put(X, x);
  for (int i = 0; i < 4; ++i) X.push_back(qc[i]);
  put(X, y);
  auto L = [&](const std::vector<D> &z) {
    V pp, n, c, p;
    D phi;
    geom(&z[0], get(z, 4), &z[7], get(z, 11), pp, n, c);
    plane_point_forward(pp, n, c, rad, phi, p);
    return vdot(n, nb) + phi * phib + vdot(p, pb);
  };
  V pp, n, c, p;
  D phi;
  geom(q, x, qc, y, pp, n, c);
  plane_point_forward(pp, n, c, rad, phi, p);
  V cb, ppb, nnb;
  plane_point_vjp(pp, n, c, rad, phi, nb, phib, pb, cb, ppb, nnb);
  // point on a body: x_bar += c_bar, psi += (c - x) x c_bar; direction: psi += n x n_bar
  const V psi_a = cross(pp - x, ppb) + cross(n, nnb);
  const V psi_b = cross(c - y, cb);
  D qa[4] = {0, 0, 0, 0}, qbb[4] = {0, 0, 0, 0};
  quat_grad_from_psi(q, psi_a, qa);
  quat_grad_from_psi(qc, psi_b, qbb);
  std::vector<D> an(qa, qa + 4);
  put(an, ppb);
  for (int i = 0; i < 4; ++i) an.push_back(qbb[i]);
  put(an, cb);
  char name[64];
  snprintf(name, sizeof name, "plane-point on bodies #%d", trial);
  report(name, an, fd_grad(X, L), 1e-7);
}

// box edge on a rotating body: e0 = x + R(q) o, u = R(q) a (unit); the point
// c = y + R(qc) oc on another body.  Checks line_point_vjp and the body
// conversion (e0 a point of the body, u a direction of the body).
static void check_line_point(int trial) {
  D q[4], qc[4];
  for (int i = 0; i < 4; ++i) { q[i] = U(-1, 1); qc[i] = U(-1, 1); }
  const V x = rv(0.3), o = rv(0.1), y = rv(0.3), oc = rv(0.05);
  V a = rv(1.0);
  a = (D(1) / sqrt(vdot(a, a))) * a;
  const D rad = U(0.0, 0.05);
  const V nb = rv(1.0), pb = rv(1.0);
  const D phib = U(-1, 1);
  auto rot = [](const D *R, V v) {
    return vec(R[0] * v.x + R[1] * v.y + R[2] * v.z, R[3] * v.x + R[4] * v.y + R[5] * v.z,
               R[6] * v.x + R[7] * v.y + R[8] * v.z);
  };
  auto geom = [&](const D *qq, V xx, const D *qqc, V yy, V &e0, V &u, V &c) {
    D R[9], Rc[9];
    rot_of_quat(qq, R);
    rot_of_quat(qqc, Rc);
    e0 = xx + rot(R, o);
    u = rot(R, a);
    c = yy + rot(Rc, oc);
  };
  // keep c off the line: shift the other body's origin sideways once
  const V side = rv(0.2);
  std::vector<D> X(q, q + 4);
  put(X, x);
  for (int i = 0; i < 4; ++i) X.push_back(qc[i]);
  put(X, y + side);
  auto L = [&](const std::vector<D> &z) {
    V e0, u, c, n, p;
    D phi;
    geom(&z[0], get(z, 4), &z[7], get(z, 11), e0, u, c);
    line_point_forward(e0, u, c, rad, n, phi, p);
    return vdot(n, nb) + phi * phib + vdot(p, pb);
  };
  V e0, u, c, n, p;
  D phi;
  geom(q, x, qc, y + side, e0, u, c);
  line_point_forward(e0, u, c, rad, n, phi, p);
  V cb, e0b, ub;
  line_point_vjp(e0, u, c, rad, n, phi, nb, phib, pb, cb, e0b, ub);
  const V psi_a = cross(e0 - x, e0b) + cross(u, ub);
  const V psi_b = cross(c - (y + side), cb);
  D qa[4] = {0, 0, 0, 0}, qbb[4] = {0, 0, 0, 0};
  quat_grad_from_psi(q, psi_a, qa);
  quat_grad_from_psi(qc, psi_b, qbb);
  std::vector<D> an(qa, qa + 4);
  put(an, e0b);
  for (int i = 0; i < 4; ++i) an.push_back(qbb[i]);
  put(an, cb);
  char name[64];
  snprintf(name, sizeof name, "line-point on bodies #%d", trial);
  report(name, an, fd_grad(X, L), 1e-7);
}

// Phi of an articulated subtree (cf_artadj.h): its derivatives along every
// joint angle and rate by the dual-number pass (float32) against central
// differences of the float64 pass.  A chain of four bodies under a fixed base
// (hinge, hinge, slide, hinge) with random frames, axes, COM offsets and
// inertias; random Mbar, cbar, Jbar.
static void check_subtree_phi(int trial) {
  using cf::BodyC;
  using namespace cf::artadj;
  const int nbs = 4, nd = 4;
  BodyC B[4] = {};
  const int jt[4] = {cf::kHinge, cf::kHinge, cf::kSlide, cf::kHinge};
  for (int k = 0; k < nbs; ++k) {
    BodyC &c = B[k];
    c.parent = k - 1;
    c.jnt = jt[k];
    c.qadr = k;
    c.dadr = k;
    c.fast = 0;
    const V p = rv(0.1), ip = rv(0.05);
    V ax = rv(1.0);
    ax = (D(1) / sqrt(vdot(ax, ax))) * ax;
    c.pos = make_float4((float)p.x, (float)p.y, (float)p.z, 0.f);
    c.quat = make_float4((float)U(-1, 1), (float)U(-1, 1), (float)U(-1, 1), (float)U(-1, 1));
    c.axis = make_float4((float)ax.x, (float)ax.y, (float)ax.z, 0.f);
    c.ipos = make_float4((float)ip.x, (float)ip.y, (float)ip.z, 0.f);
  }
  float4 bmi[4];
  for (int k = 0; k < nbs; ++k) bmi[k] = make_float4((float)U(0.1, 1), (float)U(1e-3, 1e-2), (float)U(1e-3, 1e-2), (float)U(1e-3, 1e-2));
  std::vector<float> Mb(nd * nd), cb(nd), Jb(6 * nd * nbs);
  for (auto &x : Mb) x = (float)U(-1, 1);
  for (auto &x : cb) x = (float)U(-1, 1);
  for (auto &x : Jb) x = (float)U(-1, 1);
  std::vector<D> th(nd), thd(nd);
  for (int i = 0; i < nd; ++i) { th[i] = (float)U(-1, 1); thd[i] = (float)U(-3, 3); }
  const float g[3] = {0.1f, -0.2f, -9.81f};
  std::vector<D> x(th);
  x.insert(x.end(), thd.begin(), thd.end());
  std::vector<D> wk(phi_work(nbs, nd));
  auto L = [&](const std::vector<D> &y) {
    return subtree_phi<D>(B, 0, nbs, 0, nd, bmi, y.data(), y.data() + nd, nullptr, nullptr, g[0], g[1], g[2],
                          Mb.data(), cb.data(), Jb.data(), wk.data());
  };
  std::vector<Du<float>> a(nd), ad(nd), wd(phi_work(nbs, nd));
  std::vector<D> an(2 * nd);
  for (int k = 0; k < 2 * nd; ++k) {
    for (int i = 0; i < nd; ++i) {
      a[i] = du<float>((float)th[i], k == i ? 1.f : 0.f);
      ad[i] = du<float>((float)thd[i], k == nd + i ? 1.f : 0.f);
    }
    an[k] = subtree_phi<Du<float>>(B, 0, nbs, 0, nd, bmi, a.data(), ad.data(), nullptr, nullptr, g[0], g[1], g[2],
                                   Mb.data(), cb.data(), Jb.data(), wd.data()).d;
  }
  char name[64];
  snprintf(name, sizeof name, "subtree phi (dual) #%d", trial);
  report(name, an, fd_grad(x, L), 2e-4);
}

// The same with a free root (6 dofs: translation of its frame origin and a
// world-frame rotation increment) carrying three hinge / slide children.
static void check_subtree_phi_free(int trial) {
  using cf::BodyC;
  using namespace cf::artadj;
  const int nbs = 4, nd = 9;
  BodyC B[4] = {};
  const int jt[4] = {cf::kFree, cf::kHinge, cf::kSlide, cf::kHinge};
  const int par[4] = {-1, 0, 1, 0};  // a branch: bodies 1 and 3 both hang from the root
  for (int k = 0; k < nbs; ++k) {
    BodyC &c = B[k];
    c.parent = par[k];
    c.jnt = jt[k];
    c.dadr = k == 0 ? 0 : 5 + k;
    c.qadr = k == 0 ? 0 : 6 + k;
    const V p = rv(0.1), ip = rv(0.05);
    V ax = rv(1.0);
    ax = (D(1) / sqrt(vdot(ax, ax))) * ax;
    c.pos = make_float4((float)p.x, (float)p.y, (float)p.z, 0.f);
    c.quat = make_float4((float)U(-1, 1), (float)U(-1, 1), (float)U(-1, 1), (float)U(-1, 1));
    c.axis = make_float4((float)ax.x, (float)ax.y, (float)ax.z, 0.f);
    c.ipos = k == 0 ? make_float4(0.f, 0.f, 0.f, 0.f) : make_float4((float)ip.x, (float)ip.y, (float)ip.z, 0.f);
  }
  float4 bmi[4];
  for (int k = 0; k < nbs; ++k) bmi[k] = make_float4((float)U(0.1, 1), (float)U(1e-3, 1e-2), (float)U(1e-3, 1e-2), (float)U(1e-3, 1e-2));
  std::vector<float> Mb(nd * nd), cb(nd), Jb(6 * nd * nbs);
  for (auto &x : Mb) x = (float)U(-1, 1);
  for (auto &x : cb) x = (float)U(-1, 1);
  for (auto &x : Jb) x = (float)U(-1, 1);
  D q[4] = {U(-1, 1), U(-1, 1), U(-1, 1), U(-1, 1)}, R0[9];
  rot_of_quat(q, R0);
  const V p0 = rv(0.3);
  std::vector<D> th(nd, 0.0), thd(nd);
  for (int i = 6; i < nd; ++i) th[i] = (float)U(-1, 1);
  for (int i = 0; i < nd; ++i) thd[i] = (float)U(-3, 3);
  const float g[3] = {0.1f, -0.2f, -9.81f};
  // x: translation (3), rotation increment (3), child joints (3), rates (9)
  std::vector<D> x(6, 0.0);
  for (int i = 6; i < nd; ++i) x.push_back(th[i]);
  x.insert(x.end(), thd.begin(), thd.end());
  std::vector<D> wk(phi_work(nbs, nd));
  auto L = [&](const std::vector<D> &y) {
    const V w = vec(y[3], y[4], y[5]);
    const D a = sqrt(vdot(w, w));
    D Rr[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1}, Rn[9];
    if (a > 0) {
      const D c = cos(a), s_ = sin(a), t = 1 - c, ux = w.x / a, uy = w.y / a, uz = w.z / a;
      const D K[9] = {c + ux * ux * t, ux * uy * t - uz * s_, ux * uz * t + uy * s_,
                      uy * ux * t + uz * s_, c + uy * uy * t, uy * uz * t - ux * s_,
                      uz * ux * t - uy * s_, uz * uy * t + ux * s_, c + uz * uz * t};
      for (int i = 0; i < 9; ++i) Rr[i] = K[i];
    }
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) Rn[3 * i + j] = Rr[3 * i] * R0[j] + Rr[3 * i + 1] * R0[3 + j] + Rr[3 * i + 2] * R0[6 + j];
    const D rp[3] = {p0.x + y[0], p0.y + y[1], p0.z + y[2]};
    std::vector<D> t(nd, 0.0);
    for (int i = 6; i < nd; ++i) t[i] = y[i];
    return subtree_phi<D>(B, 0, nbs, 0, nd, bmi, t.data(), y.data() + nd, rp, Rn, g[0], g[1], g[2], Mb.data(),
                          cb.data(), Jb.data(), wk.data());
  };
  std::vector<Du<float>> a(nd), ad(nd), rp(3), rr(9), wd(phi_work(nbs, nd));
  std::vector<D> an(2 * nd);
  for (int k = 0; k < 2 * nd; ++k) {
    for (int i = 0; i < nd; ++i) {
      a[i] = du<float>((float)th[i], (i >= 6 && k == i) ? 1.f : 0.f);
      ad[i] = du<float>((float)thd[i], k == nd + i ? 1.f : 0.f);
    }
    const D pp[3] = {p0.x, p0.y, p0.z};
    for (int i = 0; i < 3; ++i) rp[i] = du<float>((float)pp[i], k == i ? 1.f : 0.f);
    const int e = (k >= 3 && k < 6) ? k - 3 : -1;
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        float d = 0.f;
        if (e >= 0) {
          const int i1 = (e + 1) % 3, i2 = (e + 2) % 3;
          d = (float)(i == i1 ? -R0[3 * i2 + j] : i == i2 ? R0[3 * i1 + j] : 0.0);
        }
        rr[3 * i + j] = du<float>((float)R0[3 * i + j], d);
      }
    an[k] = subtree_phi<Du<float>>(B, 0, nbs, 0, nd, bmi, a.data(), ad.data(), rp.data(), rr.data(), g[0], g[1],
                                   g[2], Mb.data(), cb.data(), Jb.data(), wd.data()).d;
  }
  char name[64];
  snprintf(name, sizeof name, "subtree phi, free root (dual) #%d", trial);
  report(name, an, fd_grad(x, L), 5e-4);
}

int main() {
  for (int t = 0; t < 4; ++t) check_predict(t);
  for (int t = 0; t < 3; ++t) check_update(t, 20.0);
  for (int t = 0; t < 2; ++t) check_update(t, 1e-4);  // series branch of exp
  for (int t = 0; t < 2; ++t) check_update(t, 1e-9);  // small-angle branch
  for (int t = 0; t < 3; ++t) {
    check_contact<1>(t, true, true, 0.01);
    check_contact<4>(t, true, true, 0.01);
    check_contact<6>(t, true, true, 0.01);
    check_contact<10>(t, true, true, 0.01);
    check_contact<4>(t, false, true, 0.01);
    check_contact<10>(t, false, true, 0.0005);  // x below the clamp: rho varies with phi
    check_contact<4>(t, true, false, 0.0005);
    check_contact<1>(t, true, true, 0.01, true);
    check_contact<4>(t, true, true, 0.01, true);
    check_contact<6>(t, true, true, 0.01, true);
    check_contact<10>(t, true, true, 0.01, true);
    check_contact<4>(t, false, true, 0.01, true);
    check_contact<6>(t, true, false, 0.0005, true);
  }
  const std::vector<float> net = random_net();
  for (int t = 0; t < 3; ++t) {  // learned gains: kept (large margin) and under the tight rule
    check_contact<1>(t, true, true, 0.01, false, net.data(), 1.0);
    check_contact<4>(t, true, true, 0.01, false, net.data(), 1.0);
    check_contact<6>(t, true, true, 0.01, false, net.data(), 1.0);
    check_contact<10>(t, true, true, 0.01, false, net.data(), 1.0);
    check_contact<4>(t, false, true, 0.0005, false, net.data(), 1.0);
    check_contact<4>(t, true, true, 0.01, false, net.data(), 0.0);
    check_contact<6>(t, true, false, 0.01, false, net.data(), 1e-4);
  }
  for (int t = 0; t < 3; ++t) check_sphere_pair(t);
  for (int t = 0; t < 3; ++t) check_plane_point(t);
  for (int t = 0; t < 3; ++t) check_line_point(t);
  for (int t = 0; t < 3; ++t) check_subtree_phi(t);
  for (int t = 0; t < 3; ++t) check_subtree_phi_free(t);
  printf("%s (%d failures)\n", failures ? "FAILED" : "ALL OK", failures);
  return failures ? 1 : 0;
}
