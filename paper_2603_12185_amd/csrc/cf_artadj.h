// cf_artadj.h - pieces of the reverse pass of an articulated subtree (hinge and
// slide joints below a fixed or free root) for cf_step_backward.
//
// The subtree's prediction uses M(th), the bias c(th, thd) and the body
// Jacobians J_b(th) (Eq. smooth_vel and the J~^T lambda scatter of Eq.
// vel_correction).  Once the reverse pass has formed the adjoints Mbar, cbar and
// Jbar_b of those matrices (from the Cholesky solves, the contacts and the body
// velocities), the joint adjoints they contribute are the gradient of the scalar
//   Phi(th, thd) = <Mbar, M(th)> + <cbar, c(th, thd)> + sum_b <Jbar_b, J_b(th)>
// with Mbar, cbar, Jbar held fixed.  subtree_phi evaluates Phi over any scalar
// type; with the dual numbers below it gives one directional derivative per
// call (forward mode, one call per joint angle and one per joint rate; a free
// root's pose is varied along a translation or a world-frame rotation increment).
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>

#include "cf_internal.h"

namespace cf {
namespace artadj {

#define CF_HD __host__ __device__ inline

// Dual number: value and one directional derivative.
template <class T>
struct Du {
  T v, d;
};
template <class T> CF_HD Du<T> du(T v, T d = T(0)) { return {v, d}; }
template <class T> CF_HD Du<T> operator+(Du<T> a, Du<T> b) { return {a.v + b.v, a.d + b.d}; }
template <class T> CF_HD Du<T> operator-(Du<T> a, Du<T> b) { return {a.v - b.v, a.d - b.d}; }
template <class T> CF_HD Du<T> operator-(Du<T> a) { return {-a.v, -a.d}; }
template <class T> CF_HD Du<T> operator*(Du<T> a, Du<T> b) { return {a.v * b.v, a.d * b.v + a.v * b.d}; }
template <class T> CF_HD Du<T> operator*(T s, Du<T> a) { return {s * a.v, s * a.d}; }
template <class T> CF_HD Du<T> operator*(Du<T> a, T s) { return {s * a.v, s * a.d}; }
template <class T> CF_HD Du<T> operator+(Du<T> a, T s) { return {a.v + s, a.d}; }
template <class T> CF_HD Du<T> operator+(T s, Du<T> a) { return {a.v + s, a.d}; }
template <class T> CF_HD Du<T> operator-(Du<T> a, T s) { return {a.v - s, a.d}; }
template <class T> CF_HD Du<T> operator-(T s, Du<T> a) { return {s - a.v, -a.d}; }
template <class T> CF_HD Du<T> &operator+=(Du<T> &a, Du<T> b) { a = a + b; return a; }
template <class T> CF_HD Du<T> sin_(Du<T> a) { return {sin(a.v), cos(a.v) * a.d}; }
template <class T> CF_HD Du<T> cos_(Du<T> a) { return {cos(a.v), -sin(a.v) * a.d}; }
CF_HD float sin_(float a) { return sinf(a); }
CF_HD float cos_(float a) { return cosf(a); }
CF_HD double sin_(double a) { return sin(a); }
CF_HD double cos_(double a) { return cos(a); }

// Scalar promoted from a constant of the model.
template <class S> struct Lift { CF_HD static S of(float x) { return S(x); } };
template <class T> struct Lift<Du<T>> { CF_HD static Du<T> of(float x) { return {T(x), T(0)}; } };
template <class S> CF_HD S lift(float x) { return Lift<S>::of(x); }

// Rotation matrix (row-major) of the unit quaternion (w, x, y, z), constants.
CF_HD void quat_rot_f(float w, float x, float y, float z, float *R) {
  const float n = sqrtf(w * w + x * x + y * y + z * z);
  w /= n; x /= n; y /= n; z /= n;
  R[0] = 1 - 2 * (y * y + z * z); R[1] = 2 * (x * y - z * w);     R[2] = 2 * (x * z + y * w);
  R[3] = 2 * (x * y + z * w);     R[4] = 1 - 2 * (x * x + z * z); R[5] = 2 * (y * z - x * w);
  R[6] = 2 * (x * z - y * w);     R[7] = 2 * (y * z + x * w);     R[8] = 1 - 2 * (x * x + y * y);
}

// Workspace of subtree_phi, in scalars: 24 per body and 6 per dof.
CF_HD int phi_work(int nbs, int nd) { return 24 * nbs + 6 * nd; }

// Phi over one subtree: hinge / slide joints below a root that hangs from the
// world by a hinge, a slide or a free joint.  B: the model's bodies; the subtree
// is bodies [b0, b0 + nbs) with dofs [d0, d0 + nd) (a free root's 6 first, then
// one per body); bmi: (m, Ixx, Iyy, Izz) per body of the world (indexed by
// body); th, thd: joint values and rates [nd] (th unused for a free root's
// dofs, whose pose is rpos / rrot: frame origin and row-major rotation, so a
// caller can vary it along a translation or a world-frame rotation increment);
// g: gravity.  Mbar [nd][nd], cbar [nd], Jbar [nbs][6][nd] (rows: COM linear
// x y z, angular x y z).  wk: phi_work(nbs, nd) scalars.
template <class S>
CF_HD S subtree_phi(const BodyC *B, int b0, int nbs, int d0, int nd, const float4 *bmi, const S *th, const S *thd,
                    const S *rpos, const S *rrot, float gx, float gy, float gz, const float *Mbar,
                    const float *cbar, const float *Jbar, S *wk) {
  S *org = wk, *rot = org + 3 * nbs, *ax = rot + 9 * nbs, *com = ax + 3 * nbs, *om = com + 3 * nbs,
    *vo = om + 3 * nbs, *J = vo + 3 * nbs;
  const S zero = lift<S>(0.f);
  // forward kinematics (parents precede children)
  for (int k = 0; k < nbs; ++k) {
    const BodyC c = B[b0 + k];
    const int pk = c.parent - b0;
    if (c.jnt == kFree) {  // the root's pose as given
      const float ip[3] = {c.ipos.x, c.ipos.y, c.ipos.z};
      for (int i = 0; i < 3; ++i) {
        org[3 * k + i] = rpos[i];
        ax[3 * k + i] = zero;
        com[3 * k + i] = rpos[i] + rrot[3 * i] * ip[0] + rrot[3 * i + 1] * ip[1] + rrot[3 * i + 2] * ip[2];
        for (int j = 0; j < 3; ++j) rot[9 * k + 3 * i + j] = rrot[3 * i + j];
      }
      continue;
    }
    S po[3], pR[9];
    for (int i = 0; i < 3; ++i) {
      po[i] = pk >= 0 ? org[3 * pk + i] : zero;
      for (int j = 0; j < 3; ++j) pR[3 * i + j] = pk >= 0 ? rot[9 * pk + 3 * i + j] : lift<S>(i == j ? 1.f : 0.f);
    }
    float bq[9];
    quat_rot_f(c.quat.x, c.quat.y, c.quat.z, c.quat.w, bq);
    S R0[9];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) R0[3 * i + j] = pR[3 * i] * bq[j] + pR[3 * i + 1] * bq[3 + j] + pR[3 * i + 2] * bq[6 + j];
    const float lp[3] = {c.pos.x, c.pos.y, c.pos.z}, la[3] = {c.axis.x, c.axis.y, c.axis.z};
    S o[3], aw[3], R[9];
    for (int i = 0; i < 3; ++i) {
      o[i] = po[i] + pR[3 * i] * lp[0] + pR[3 * i + 1] * lp[1] + pR[3 * i + 2] * lp[2];
      aw[i] = R0[3 * i] * la[0] + R0[3 * i + 1] * la[1] + R0[3 * i + 2] * la[2];
    }
    const S t = th[c.dadr - d0];
    if (c.jnt == kHinge) {
      // R = R0 Rot(la, t), Rot = cos t I + sin t [la]x + (1 - cos t) la la^T
      const S ct = cos_(t), st = sin_(t), vt = lift<S>(1.f) - ct;
      S Rj[9];
      const float K[9] = {0.f, -la[2], la[1], la[2], 0.f, -la[0], -la[1], la[0], 0.f};
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
          Rj[3 * i + j] = (i == j ? ct : zero) + st * K[3 * i + j] + vt * (la[i] * la[j]);
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) R[3 * i + j] = R0[3 * i] * Rj[j] + R0[3 * i + 1] * Rj[3 + j] + R0[3 * i + 2] * Rj[6 + j];
    } else {
      for (int i = 0; i < 9; ++i) R[i] = R0[i];
      for (int i = 0; i < 3; ++i) o[i] = o[i] + aw[i] * t;
    }
    const float ip[3] = {c.ipos.x, c.ipos.y, c.ipos.z};
    for (int i = 0; i < 3; ++i) {
      org[3 * k + i] = o[i];
      ax[3 * k + i] = aw[i];
      com[3 * k + i] = o[i] + R[3 * i] * ip[0] + R[3 * i + 1] * ip[1] + R[3 * i + 2] * ip[2];
      for (int j = 0; j < 3; ++j) rot[9 * k + 3 * i + j] = R[3 * i + j];
    }
  }
  S phi = zero;
  for (int k = 0; k < nbs; ++k) {
    const int b = b0 + k;
    const float4 mi = bmi[b];
    const S cb[3] = {com[3 * k], com[3 * k + 1], com[3 * k + 2]};
    // Jacobian columns of the COM (zero off the chain)
    for (int i = 0; i < 6 * nd; ++i) J[i] = zero;
    for (int j = b; j >= b0; j = B[j].parent) {
      const int jk = j - b0, x = B[j].dadr - d0;
      const S a[3] = {ax[3 * jk], ax[3 * jk + 1], ax[3 * jk + 2]};
      if (B[j].jnt == kFree) {  // (e_k, 0) and (e_k x (c_b - o), e_k)
        const S r[3] = {cb[0] - org[3 * jk], cb[1] - org[3 * jk + 1], cb[2] - org[3 * jk + 2]};
        for (int e = 0; e < 3; ++e) {
          J[e * nd + x + e] = lift<S>(1.f);
          J[(3 + e) * nd + x + 3 + e] = lift<S>(1.f);
        }
        J[1 * nd + x + 3] = -r[2]; J[2 * nd + x + 3] = r[1];   // e_x x r = (0, -r_z, r_y)
        J[0 * nd + x + 4] = r[2];  J[2 * nd + x + 4] = -r[0];  // e_y x r = (r_z, 0, -r_x)
        J[0 * nd + x + 5] = -r[1]; J[1 * nd + x + 5] = r[0];   // e_z x r = (-r_y, r_x, 0)
      } else if (B[j].jnt == kHinge) {
        const S r[3] = {cb[0] - org[3 * jk], cb[1] - org[3 * jk + 1], cb[2] - org[3 * jk + 2]};
        J[0 * nd + x] = a[1] * r[2] - a[2] * r[1];
        J[1 * nd + x] = a[2] * r[0] - a[0] * r[2];
        J[2 * nd + x] = a[0] * r[1] - a[1] * r[0];
        J[3 * nd + x] = a[0]; J[4 * nd + x] = a[1]; J[5 * nd + x] = a[2];
      } else {
        J[0 * nd + x] = a[0]; J[1 * nd + x] = a[1]; J[2 * nd + x] = a[2];
      }
      if (B[j].parent < b0) break;
    }
    // velocities at thd: COM linear vc, angular om, frame origin vo
    S vc[3], w[3];
    for (int r = 0; r < 3; ++r) {
      vc[r] = zero; w[r] = zero;
      for (int i = 0; i < nd; ++i) { vc[r] = vc[r] + J[r * nd + i] * thd[i]; w[r] = w[r] + J[(3 + r) * nd + i] * thd[i]; }
    }
    const S ob[3] = {org[3 * k], org[3 * k + 1], org[3 * k + 2]};
    const S d_[3] = {ob[0] - cb[0], ob[1] - cb[1], ob[2] - cb[2]};
    for (int r = 0; r < 3; ++r) om[3 * k + r] = w[r];
    vo[3 * k + 0] = vc[0] + (w[1] * d_[2] - w[2] * d_[1]);
    vo[3 * k + 1] = vc[1] + (w[2] * d_[0] - w[0] * d_[2]);
    vo[3 * k + 2] = vc[2] + (w[0] * d_[1] - w[1] * d_[0]);
    // velocity-product accelerations Jdot_b thd over the chain
    S jl[3] = {zero, zero, zero}, ja[3] = {zero, zero, zero};
    for (int j = b; j >= b0; j = B[j].parent) {
      const int jk = j - b0;
      const S a[3] = {ax[3 * jk], ax[3 * jk + 1], ax[3 * jk + 2]};
      const S wj[3] = {om[3 * jk], om[3 * jk + 1], om[3 * jk + 2]};
      const S wa[3] = {wj[1] * a[2] - wj[2] * a[1], wj[2] * a[0] - wj[0] * a[2], wj[0] * a[1] - wj[1] * a[0]};
      if (B[j].jnt == kFree) {  // the root's angular rates act on c_b - origin velocity
        const int x = B[j].dadr - d0;
        const S wr[3] = {thd[x + 3], thd[x + 4], thd[x + 5]};
        const S dv[3] = {vc[0] - vo[3 * jk], vc[1] - vo[3 * jk + 1], vc[2] - vo[3 * jk + 2]};
        jl[0] = jl[0] + (wr[1] * dv[2] - wr[2] * dv[1]);
        jl[1] = jl[1] + (wr[2] * dv[0] - wr[0] * dv[2]);
        jl[2] = jl[2] + (wr[0] * dv[1] - wr[1] * dv[0]);
        if (B[j].parent < b0) break;
        continue;
      }
      const S td = thd[B[j].dadr - d0];
      if (B[j].jnt == kHinge) {
        const S rc[3] = {cb[0] - org[3 * jk], cb[1] - org[3 * jk + 1], cb[2] - org[3 * jk + 2]};
        const S dv[3] = {vc[0] - vo[3 * jk], vc[1] - vo[3 * jk + 1], vc[2] - vo[3 * jk + 2]};
        const S t1[3] = {wa[1] * rc[2] - wa[2] * rc[1], wa[2] * rc[0] - wa[0] * rc[2], wa[0] * rc[1] - wa[1] * rc[0]};
        const S t2[3] = {a[1] * dv[2] - a[2] * dv[1], a[2] * dv[0] - a[0] * dv[2], a[0] * dv[1] - a[1] * dv[0]};
        for (int r = 0; r < 3; ++r) { jl[r] = jl[r] + td * (t1[r] + t2[r]); ja[r] = ja[r] + td * wa[r]; }
      } else {
        for (int r = 0; r < 3; ++r) jl[r] = jl[r] + td * wa[r];
      }
      if (B[j].parent < b0) break;
    }
    // world inertia I = R diag(d) R^T
    const float dd[3] = {mi.y, mi.z, mi.w};
    S Iw[9];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j)
        Iw[3 * i + j] = rot[9 * k + 3 * i] * rot[9 * k + 3 * j] * dd[0] + rot[9 * k + 3 * i + 1] * rot[9 * k + 3 * j + 1] * dd[1] +
                        rot[9 * k + 3 * i + 2] * rot[9 * k + 3 * j + 2] * dd[2];
    const float g[3] = {gx, gy, gz};
    S Fl[3], Fa[3], Iw_w[3];
    for (int r = 0; r < 3; ++r) {
      Fl[r] = mi.x * (jl[r] - g[r]);
      Fa[r] = Iw[3 * r] * ja[0] + Iw[3 * r + 1] * ja[1] + Iw[3 * r + 2] * ja[2];
      Iw_w[r] = Iw[3 * r] * w[0] + Iw[3 * r + 1] * w[1] + Iw[3 * r + 2] * w[2];
    }
    Fa[0] = Fa[0] + (w[1] * Iw_w[2] - w[2] * Iw_w[1]);
    Fa[1] = Fa[1] + (w[2] * Iw_w[0] - w[0] * Iw_w[2]);
    Fa[2] = Fa[2] + (w[0] * Iw_w[1] - w[1] * Iw_w[0]);
    // <cbar, J^T F>, <Mbar, J^T diag(m, I) J>, <Jbar_b, J>
    for (int i = 0; i < nd; ++i) {
      S ci = zero;
      for (int r = 0; r < 3; ++r) ci = ci + J[r * nd + i] * Fl[r] + J[(3 + r) * nd + i] * Fa[r];
      phi = phi + cbar[i] * ci;
      S IJ[3];
      for (int r = 0; r < 3; ++r)
        IJ[r] = Iw[3 * r] * J[3 * nd + i] + Iw[3 * r + 1] * J[4 * nd + i] + Iw[3 * r + 2] * J[5 * nd + i];
      for (int j = 0; j < nd; ++j) {
        const float mb = Mbar[i * nd + j];
        if (mb == 0.f) continue;
        S mij = zero;
        for (int r = 0; r < 3; ++r) mij = mij + mi.x * (J[r * nd + i] * J[r * nd + j]) + IJ[r] * J[(3 + r) * nd + j];
        phi = phi + mb * mij;
      }
    }
    const float *Jb = Jbar + 6 * nd * k;
    for (int i = 0; i < 6 * nd; ++i)
      if (Jb[i] != 0.f) phi = phi + Jb[i] * J[i];
  }
  return phi;
}

#undef CF_HD

}  // namespace artadj
}  // namespace cf
