// cf_api.hip - host side of the C ABI declared in include/cfsim.h.
//
// Validates the model description, builds the canonical candidate-slot table,
// uploads per-world constants as float32 and owns the contact workspace.
// cf_step enqueues the collision kernel then the resolution kernel on the
// caller's stream; nothing here synchronises except create/destroy and the
// explicit timing query.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <algorithm>
#include <vector>

#include "../../include/cfsim.h"
#include "cf_internal.h"

namespace {

thread_local std::string g_err;

cf_status set_err(cf_status st, const std::string &msg) {
  g_err = msg;
  return st;
}

struct EventSet {
  hipEvent_t e[3];
};


}  // namespace

struct cf_model {
  int dev = 0;
  int nw = 0, nb = 0, ng = 0, nq = 0, nv = 0, ncon_max = 0, condim = 3, nf = 4, nbits = 1;
  int nslot = 0;
  int nslot_pre = 0, sph0 = 0, nsph = 0;  // sphere block of the narrow phase (see below)
  int npl = 0;                            // static planes tested as rows against the block
  int sph_mfma = 0;                       // block masks from an MFMA Gram matrix (see collide_args)
  cf::Params p{};
  // device constants
  uint32_t *d_slots = nullptr;
  int *d_gbody = nullptr, *d_gorient = nullptr;
  cf::BodyC *d_body = nullptr;
  cf::SubTree *d_sub = nullptr;
  int norient = 0, nsub = 0, art_floats = 0, artb_floats = 0;
  int ydiag_floats = 0;  // the bodies' L^-1 J^T columns (exact diagonal impedance), after the work blocks
  int block_collide = 64, block_resolve = 128, block_rollout = 256;
  size_t lds_rollout = 0;
  size_t lds_rollout_free = 0;  // persistent rollout of free bodies (0: not applicable)
  int ncu = 256;                // compute units of the model's device
  int block_backward = 0;  // 0: the adjoint's LDS does not fit any workgroup size
  size_t lds_backward = 0;
  bool rollout_steps = false;  // autotuner found T cf_step calls faster than the persistent kernel
  float4 *d_bmi = nullptr, *d_gdat = nullptr, *d_gpos = nullptr, *d_gquat = nullptr;
  float *d_gmu = nullptr;  // [nworld][ngeom] tangential friction alone
  cf::JointK<double> *d_jk64 = nullptr;  // [nb] joint constants (narrow phase kinematics)
  float4 *d_frames = nullptr;  // [nworld][nb][5] small-subtree frames, narrow phase -> resolution
  float2 *d_gfr2 = nullptr;
  int gpos_ws = 0, gquat_ws = 0;
  // workspace
  float4 *d_cnp = nullptr, *d_cpos = nullptr;
  int *d_ncon = nullptr, *d_over = nullptr;
  size_t lds_collide = 0, lds_resolve = 0;
  size_t lds_resolve_free = 0;  // resolution with each free body's state in its lane
  const float *mlp = nullptr;  // learned-gain network parameters (caller-owned device memory)
  float4 *d_mlp_img = nullptr; // their LDS image, rewritten by every step that uses them
  bool box_pairs = false;      // box-sphere or box-capsule slots present
  std::vector<int> dof_jnt;    // joint type of each dof
  std::vector<int> dof_q;      // q index of each dof's joint (hinge / slide)
  float4 *d_act = nullptr;     // [nv] position actuators, or null
  // timing
  bool prof = false;
  std::vector<EventSet> events;
  size_t ev_used = 0;
  double ms_collide = 0, ms_resolve = 0;
  long long prof_steps = 0;
};

// Floats of the resolution's articulated LDS region: the subtrees' work
// blocks and, with the exact diagonal impedance, their bodies' L^-1 J^T columns.
static int art_region_floats(const cf_model *m) {
  return m->art_floats + (m->p.imp_diag && m->nsub > 0 ? m->ydiag_floats : 0);
}

static size_t rollout_lds(const cf_model *m) {
  return cf::rollout_lds_bytes(m->nq, m->nv, m->nb, m->ng, m->norient, m->nsub, m->nsph, art_region_floats(m),
                               m->ncon_max);
}

namespace {

template <class T>
hipError_t upload(T **dst, const std::vector<T> &src) {
  size_t bytes = sizeof(T) * (src.empty() ? 1 : src.size());
  hipError_t e = hipMalloc((void **)dst, bytes);
  if (e != hipSuccess) return e;
  if (!src.empty()) e = hipMemcpy(*dst, src.data(), sizeof(T) * src.size(), hipMemcpyHostToDevice);
  return e;
}

// Joint constants of a hinge (or slide) body from its frame quaternion bq
// (w, x, y, z, normalised here), offset lp in the parent and unit axis a.
cf::JointK<double> joint_constants(const double *bq, const double *lp, const double *a, bool hinge) {
  const double n = std::sqrt(bq[0] * bq[0] + bq[1] * bq[1] + bq[2] * bq[2] + bq[3] * bq[3]);
  const double w = bq[0] / n, x = bq[1] / n, y = bq[2] / n, z = bq[3] / n;
  const double B[9] = {1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w),
                       2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w),
                       2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)};
  const double ax[9] = {0, -a[2], a[1], a[2], 0, -a[0], -a[1], a[0], 0};  // [a]x
  cf::JointK<double> K{};
  for (int i = 0; i < 3; ++i) {
    K.lp[i] = lp[i];
    K.Ba[i] = B[3 * i] * a[0] + B[3 * i + 1] * a[1] + B[3 * i + 2] * a[2];
  }
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      if (hinge) {
        K.Mk[3 * i + j] = K.Ba[i] * a[j];
        K.Mc[3 * i + j] = B[3 * i + j] - K.Ba[i] * a[j];
        K.Ms[3 * i + j] = B[3 * i] * ax[j] + B[3 * i + 1] * ax[3 + j] + B[3 * i + 2] * ax[6 + j];
      } else {
        K.Mk[3 * i + j] = B[3 * i + j];
      }
    }
  if (!hinge)
    for (int i = 0; i < 3; ++i) K.s[i] = K.Ba[i];
  return K;
}

void free_model(cf_model *m) {
  if (!m) return;
  (void)hipFree(m->d_slots); (void)hipFree(m->d_gbody); (void)hipFree(m->d_gorient); (void)hipFree(m->d_act);
  (void)hipFree(m->d_mlp_img);
  (void)hipFree(m->d_body); (void)hipFree(m->d_sub); (void)hipFree(m->d_bmi); (void)hipFree(m->d_gdat);
  (void)hipFree(m->d_gpos); (void)hipFree(m->d_gquat); (void)hipFree(m->d_gfr2); (void)hipFree(m->d_gmu);
  (void)hipFree(m->d_jk64); (void)hipFree(m->d_frames);
  (void)hipFree(m->d_cnp); (void)hipFree(m->d_cpos); (void)hipFree(m->d_ncon); (void)hipFree(m->d_over);
  for (auto &s : m->events)
    for (auto e : s.e) (void)hipEventDestroy(e);
  delete m;
}

bool finite_all(const double *a, size_t n) {
  for (size_t i = 0; i < n; ++i)
    if (!std::isfinite(a[i])) return false;
  return true;
}

// Drain recorded events into the per-kernel sums.
cf_status drain_events(cf_model *m) {
  for (size_t i = 0; i < m->ev_used; ++i) {
    EventSet &s = m->events[i];
    if (hipEventSynchronize(s.e[2]) != hipSuccess) return set_err(CF_E_DEVICE, "hipEventSynchronize failed");
    float a = 0, b = 0;
    if (hipEventElapsedTime(&a, s.e[0], s.e[1]) != hipSuccess ||
        hipEventElapsedTime(&b, s.e[1], s.e[2]) != hipSuccess)
      return set_err(CF_E_DEVICE, "hipEventElapsedTime failed");
    m->ms_collide += a;
    m->ms_resolve += b;
  }
  m->prof_steps += (long long)m->ev_used;
  m->ev_used = 0;
  return CF_OK;
}

bool aligned16(const void *p) { return ((uintptr_t)p & 15u) == 0; }

constexpr size_t kLdsLimit = 64 * 1024;  // per workgroup

}  // namespace

extern "C" {

const char *cf_last_error(void) { return g_err.c_str(); }

cf_status cf_model_create(const cf_model_desc *d, cf_model **out) {
  g_err.clear();
  if (!out) return set_err(CF_E_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (!d) return set_err(CF_E_INVALID_ARG, "desc is NULL");
  const int nw = d->nworld, nb = d->nbody, ng = d->ngeom;
  if (nw < 1) return set_err(CF_E_INVALID_ARG, "nworld must be >= 1");
  if (nb < 0 || ng < 0 || d->ncon_max < 0) return set_err(CF_E_INVALID_ARG, "negative size");
  if (!(d->condim == 1 || d->condim == 3 || d->condim == 4 || d->condim == 6))
    return set_err(CF_E_INVALID_ARG, "condim must be 1, 3, 4 or 6");
  if (!(d->h > 0) || !std::isfinite(d->h)) return set_err(CF_E_INVALID_ARG, "h must be finite and > 0");
  if (!(d->k_user >= 0) || !(d->d_user >= 0) || !std::isfinite(d->k_user) || !std::isfinite(d->d_user))
    return set_err(CF_E_INVALID_ARG, "k_user and d_user must be finite and >= 0");
  const double *si = d->solimp;
  if (!(si[0] > 0 && si[0] <= si[1] && si[1] < 1)) return set_err(CF_E_INVALID_ARG, "need 0 < r_min <= r_max < 1");
  if (!(si[2] > 0)) return set_err(CF_E_INVALID_ARG, "solimp width must be > 0");
  if (!(si[3] > 0 && si[3] < 1)) return set_err(CF_E_INVALID_ARG, "solimp midpoint must be in (0, 1)");
  if (!(si[4] >= 1)) return set_err(CF_E_INVALID_ARG, "solimp power must be >= 1");
  if (!finite_all(d->gravity, 3) || !std::isfinite(d->margin)) return set_err(CF_E_INVALID_ARG, "non-finite gravity or margin");
  if (nb > 0 && (!d->body_parent || !d->body_jnt || !d->body_mass || !d->body_inertia || !d->body_ipos))
    return set_err(CF_E_INVALID_ARG, "missing body arrays");
  if (ng > 0 && (!d->geom_type || !d->geom_body || !d->geom_size || !d->geom_pos || !d->geom_quat ||
                 !d->geom_friction))
    return set_err(CF_E_INVALID_ARG, "missing geom arrays");
  for (int b = 0; b < nb; ++b) {
    const int par = d->body_parent[b], t = d->body_jnt[b];
    if (par < -1 || par >= b) return set_err(CF_E_INVALID_ARG, "body_parent must be -1 or a lower index");
    if (t != CF_JNT_FREE && t != CF_JNT_HINGE && t != CF_JNT_SLIDE) return set_err(CF_E_INVALID_ARG, "bad joint type");
    if (t == CF_JNT_FREE) {
      if (par != -1) return set_err(CF_E_INVALID_ARG, "free joints only on bodies whose parent is the world");
      const double *ip = d->body_ipos + 3 * b;
      if (ip[0] != 0 || ip[1] != 0 || ip[2] != 0) return set_err(CF_E_INVALID_ARG, "free bodies need body_ipos = 0");
    }
  }
  // Tree structure: a free body without children takes the closed-form path;
  // every other root with its descendants forms an articulated subtree, which
  // must be contiguous in body order and hold at most kMaxSubDof dofs.
  std::vector<int> nchild(nb, 0), root(nb), qadr(nb), dadr(nb);
  int nq = 0, nv = 0;
  for (int b = 0; b < nb; ++b) {
    if (d->body_parent[b] >= 0) nchild[d->body_parent[b]]++;
    root[b] = d->body_parent[b] < 0 ? b : root[d->body_parent[b]];
    qadr[b] = nq; dadr[b] = nv;
    nq += d->body_jnt[b] == CF_JNT_FREE ? 7 : 1;
    nv += d->body_jnt[b] == CF_JNT_FREE ? 6 : 1;
  }
  std::vector<cf::BodyC> bodyc(nb);
  std::vector<cf::JointK<double>> jk64(nb);
  bool any_small = false;
  std::vector<cf::SubTree> subs;
  int art_floats = 0, artb_floats = 0;
  for (int b = 0; b < nb;) {
    int e = b + 1;
    while (e < nb && root[e] == b) ++e;
    for (int k = e; k < nb; ++k)
      if (root[k] == b) return set_err(CF_E_UNSUPPORTED, "each subtree's bodies must be contiguous in body order");
    const bool fast = d->body_jnt[b] == CF_JNT_FREE && e == b + 1;
    if (!fast) {
      cf::SubTree st{};
      st.b0 = b; st.nb = e - b; st.d0 = dadr[b];
      st.nd = (e < nb ? dadr[e] : nv) - dadr[b];
      if (st.nd > cf::kMaxSubDof) return set_err(CF_E_UNSUPPORTED, "articulated subtree with more than 32 dofs");
      st.lofs = art_floats;
      art_floats += st.nd * st.nd + 9 * st.nd;
      st.bofs = artb_floats;
      artb_floats += cf::art_backward_floats(st.nd, st.nb);
      st.small = st.nb <= cf::kSmallSub ? 1 : 0;
      for (int k = b; k < e; ++k)
        if (d->body_jnt[k] == CF_JNT_FREE) st.small = 0;
      if (st.small) {
        int anc[cf::kSmallSub] = {};
        for (int k = 0; k < st.nb; ++k) {
          const int p = d->body_parent[b + k] - b;  // parents precede children; -1 - b for the root
          anc[k] = (p >= 0 ? anc[p] : 0) | (1 << k);
          st.chain |= anc[k] << (4 * k);
          if (d->body_jnt[b + k] == CF_JNT_HINGE) st.chain |= 1 << (16 + k);
        }
        st.q0 = qadr[b];
        any_small = true;
      }
      subs.push_back(st);
    }
    for (int k = b; k < e; ++k) {
      cf::BodyC &c = bodyc[k];
      const double *bp = d->body_pos + 3 * k, *bq = d->body_quat + 4 * k, *ax = d->jnt_axis + 3 * k;
      const double *ip = d->body_ipos + 3 * k;
      const double an = std::sqrt(ax[0] * ax[0] + ax[1] * ax[1] + ax[2] * ax[2]);
      c.pos = make_float4((float)bp[0], (float)bp[1], (float)bp[2], 0.f);
      c.quat = make_float4((float)bq[0], (float)bq[1], (float)bq[2], (float)bq[3]);
      c.axis = an > 0 ? make_float4((float)(ax[0] / an), (float)(ax[1] / an), (float)(ax[2] / an), 0.f)
                      : make_float4(0.f, 0.f, 0.f, 0.f);
      c.ipos = make_float4((float)ip[0], (float)ip[1], (float)ip[2], 0.f);
      c.parent = d->body_parent[k]; c.jnt = d->body_jnt[k]; c.qadr = qadr[k]; c.dadr = dadr[k];
      c.fast = fast ? 1 : 0;
      if (c.jnt != CF_JNT_FREE && !(an > 0)) return set_err(CF_E_INVALID_ARG, "zero joint axis");
      const double *q = d->body_quat + 4 * k;
      if (!(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3] > 0)) return set_err(CF_E_INVALID_ARG, "zero body_quat");
      if (c.jnt != CF_JNT_FREE) {
        const double a[3] = {ax[0] / an, ax[1] / an, ax[2] / an};
        jk64[k] = joint_constants(bq, bp, a, c.jnt == CF_JNT_HINGE);
      }
    }
    b = e;
  }
  for (int w = 0; w < nw; ++w)
    for (int b = 0; b < nb; ++b) {
      const double m = d->body_mass[(size_t)w * nb + b];
      const double *I = d->body_inertia + ((size_t)w * nb + b) * 3;
      if (!std::isfinite(m) || !finite_all(I, 3) || m < 0 || I[0] < 0 || I[1] < 0 || I[2] < 0)
        return set_err(CF_E_INVALID_ARG, "masses and inertias must be finite and >= 0");
      if (bodyc[b].fast && (!(m > 0) || !(I[0] > 0) || !(I[1] > 0) || !(I[2] > 0)))
        return set_err(CF_E_INVALID_ARG, "free bodies need mass > 0 and inertia > 0");
    }
  if (ng > cf::kMaxGeom) return set_err(CF_E_UNSUPPORTED, "ngeom exceeds 8191");
  for (int g = 0; g < ng; ++g) {
    const int t = d->geom_type[g], b = d->geom_body[g];
    if (t < CF_PLANE || t > CF_BOX) return set_err(CF_E_INVALID_ARG, "bad geom type");
    if (b < -1 || b >= nb) return set_err(CF_E_INVALID_ARG, "bad geom_body");
  }
  const size_t wg = (size_t)nw * ng;
  if (ng > 0 && (!finite_all(d->geom_size, 3 * wg) || !finite_all(d->geom_pos, 3 * wg) ||
                 !finite_all(d->geom_quat, 4 * wg) || !finite_all(d->geom_friction, 3 * wg)))
    return set_err(CF_E_INVALID_ARG, "non-finite geom data");
  for (size_t i = 0; i < wg; ++i) {
    const double *q = d->geom_quat + 4 * i;
    if (!(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3] > 0)) return set_err(CF_E_INVALID_ARG, "zero geom_quat");
  }
  for (size_t i = 0; i < 3 * wg; ++i)
    if (d->geom_friction[i] < 0) return set_err(CF_E_INVALID_ARG, "negative friction");

  // ---- candidate slots in canonical order
  std::vector<uint32_t> slots;
  bool skipped = false, box_pairs = false;
  for (int i = 0; i < ng; ++i)
    for (int j = i + 1; j < ng; ++j) {
      const int bi = d->geom_body[i], bj = d->geom_body[j];
      if (bi < 0 && bj < 0) continue;
      if (bi == bj) continue;
      if (bi >= 0 && bj >= 0 && (d->body_parent[bi] == bj || d->body_parent[bj] == bi)) continue;
      const int ti = d->geom_type[i], tj = d->geom_type[j];
      int ga = i, gb = j;
      if (tj == CF_PLANE && ti != CF_PLANE) { ga = j; gb = i; }
      else if (tj == CF_BOX && ti != CF_PLANE && ti != CF_BOX) { ga = j; gb = i; }
      const int ta = d->geom_type[ga], tb = d->geom_type[gb];
      if (ta == CF_PLANE && tb == CF_SPHERE) slots.push_back(cf::slot_pack(ga, gb, 0, cf::kPlaneSphere));
      else if (ta == CF_PLANE && tb == CF_CAPSULE)
        for (int e = 0; e < 2; ++e) slots.push_back(cf::slot_pack(ga, gb, e, cf::kPlaneCapsule));
      else if (ta == CF_PLANE && tb == CF_BOX)
        for (int c = 0; c < 8; ++c) slots.push_back(cf::slot_pack(ga, gb, c, cf::kPlaneBox));
      else if (ta == CF_SPHERE && tb == CF_SPHERE) slots.push_back(cf::slot_pack(ga, gb, 0, cf::kSphereSphere));
      else if (ta == CF_BOX && tb == CF_SPHERE) { slots.push_back(cf::slot_pack(ga, gb, 0, cf::kBoxSphere)); box_pairs = true; }
      else if (ta == CF_BOX && tb == CF_CAPSULE) {
        for (int e = 0; e < 2; ++e) slots.push_back(cf::slot_pack(ga, gb, e, cf::kBoxCapsule));
        box_pairs = true;
      }
      else skipped = true;
    }

  cf_model *m = new cf_model();
  m->nw = nw; m->nb = nb; m->ng = ng; m->ncon_max = d->ncon_max; m->condim = d->condim;
  m->nf = d->condim == 1 ? 1 : d->condim == 3 ? 4 : d->condim == 4 ? 6 : 10;
  m->nq = nq; m->nv = nv;
  m->nsub = (int)subs.size(); m->art_floats = art_floats;
  m->artb_floats = artb_floats;
  for (cf::SubTree &st : subs) {
    st.yofs = art_floats + m->ydiag_floats;
    m->ydiag_floats += 6 * st.nb * st.nd;
  }
  m->nslot = (int)slots.size();
  m->box_pairs = box_pairs;
  m->dof_jnt.resize(nv);
  m->dof_q.resize(nv);
  for (int b = 0; b < nb; ++b)
    for (int k = 0; k < (d->body_jnt[b] == CF_JNT_FREE ? 6 : 1); ++k) {
      m->dof_jnt[dadr[b] + k] = d->body_jnt[b];
      m->dof_q[dadr[b] + k] = qadr[b];
    }
  m->nbits = 1;
  while ((1 << m->nbits) <= nb) ++m->nbits;  // keys 0..nb (nb = no body)
  m->p.h = (float)d->h; m->p.k_user = (float)d->k_user; m->p.d_user = (float)d->d_user;
  m->p.margin = (float)d->margin;
  m->p.gx = (float)d->gravity[0]; m->p.gy = (float)d->gravity[1]; m->p.gz = (float)d->gravity[2];
  m->p.r_min = (float)si[0]; m->p.r_max = (float)si[1]; m->p.width = (float)si[2];
  m->p.mid = (float)si[3]; m->p.power = (float)si[4];
  m->p.inv_width = (float)(1.0 / si[2]); m->p.inv_mid = (float)(1.0 / si[3]);
  m->p.inv_1mmid = (float)(1.0 / (1.0 - si[3])); m->p.power2 = si[4] == 2.0 ? 1 : 0;
  // Oriented geoms (planes, capsules, boxes, spheres offset from their body
  // origin) carry a full pose record in the narrow phase.
  std::vector<int> gorient(ng, -1);
  for (int g = 0; g < ng; ++g) {
    bool oriented = d->geom_type[g] != CF_SPHERE || (d->geom_body[g] >= 0 && !bodyc[d->geom_body[g]].fast);
    if (!oriented && d->geom_body[g] >= 0)
      for (int w = 0; w < nw && !oriented; ++w) {
        const double *p = d->geom_pos + 3 * ((size_t)w * ng + g);
        oriented = p[0] != 0 || p[1] != 0 || p[2] != 0;
      }
    if (oriented) gorient[g] = m->norient++;
  }
  // Sphere block: the longest run of trailing geoms that are spheres centred on
  // free bodies (or static).  When the slot table ends with exactly their
  // pairs of different bodies in row-major order, the narrow phase tests those
  // rows in bulk instead of slot by slot.
  {
    m->nslot_pre = m->nslot;
    int g0 = ng;
    while (g0 > 0 && d->geom_type[g0 - 1] == CF_SPHERE && gorient[g0 - 1] < 0) --g0;
    const int S = ng - g0;
    if (S >= 2 && S <= 256) {
      std::vector<uint32_t> tail;
      for (int i = g0; i < ng; ++i)
        for (int j = i + 1; j < ng; ++j)
          if (d->geom_body[i] != d->geom_body[j]) tail.push_back(cf::slot_pack(i, j, 0, cf::kSphereSphere));
      if (tail.size() <= slots.size() && std::equal(tail.begin(), tail.end(), slots.end() - tail.size())) {
        m->sph0 = g0;
        m->nsph = S;
        m->nslot_pre = m->nslot - (int)tail.size();
      }
    }
    // Plane rows: every geom before the block is a static plane and the slots
    // before the block are exactly each plane's pairs with every block sphere,
    // plane-major.
    if (m->nsph > 0 && m->sph0 > 0) {
      bool rows = true;
      for (int g = 0; g < m->sph0 && rows; ++g) rows = d->geom_type[g] == CF_PLANE && d->geom_body[g] < 0;
      if (rows && m->nslot_pre == m->sph0 * m->nsph) {
        for (int p = 0, k = 0; p < m->sph0 && rows; ++p)
          for (int i = 0; i < m->nsph && rows; ++i, ++k)
            rows = slots[k] == cf::slot_pack(p, m->sph0 + i, 0, cf::kPlaneSphere);
        if (rows) m->npl = m->sph0;
      }
    }
    // The block's hit masks come from an MFMA Gram matrix when it holds at most
    // 64 spheres on pairwise different bodies (so every pair is a slot) and the
    // margin is not negative (then r_i + r_j + margin > 0 for every pair).
    if (m->nsph > 0 && m->nsph <= 64 && m->p.margin >= 0.f) {
      std::vector<int> bodies;
      for (int g = m->sph0; g < ng; ++g) bodies.push_back(d->geom_body[g]);
      std::sort(bodies.begin(), bodies.end());
      m->sph_mfma = std::adjacent_find(bodies.begin(), bodies.end()) == bodies.end() ? 1 : 0;
    }
  }
  // Default launch shape by world size (cf_model_autotune measures instead):
  // one sphere-block row per collision thread; for free bodies one body per
  // resolution thread (the smallest workgroup that holds every body), else a
  // resolution workgroup of 256 threads once a world has more than 64 bodies
  // (fewer contact chunks).
  m->block_collide = m->nsph > 128 ? 256 : m->nsph > 64 ? 128 : 64;
  if (m->nsub == 0 && nb <= 256) m->block_resolve = nb > 128 ? 256 : nb > 64 ? 128 : 64;
  else m->block_resolve = nb > 64 ? 256 : 128;
  m->lds_collide = cf::collide_lds_bytes(m->nq, nb, ng, m->norient, m->nsub, m->nsph);
  m->lds_resolve = cf::resolve_lds_bytes(m->nq, m->nv, nb, ng, m->nsub, m->art_floats);
  m->lds_resolve_free = cf::resolve_free_lds_bytes(nb, ng);
  if (m->lds_collide > kLdsLimit || m->lds_resolve > kLdsLimit) {
    delete m;
    return set_err(CF_E_UNSUPPORTED, "world too large for one workgroup's LDS (reduce bodies or geoms)");
  }
  m->lds_rollout = rollout_lds(m);
  if (m->nsub == 0 && cf::rollout_free_fits(m->nq, nb))
    m->lds_rollout_free = cf::rollout_free_lds_bytes(nb, ng, m->norient, m->nsph);
  for (int bs : {256, 128, 64}) {
    const size_t l = cf::backward_lds_bytes(m->nq, m->nv, nb, ng, bs, m->nsub, m->art_floats, m->artb_floats);
    if (l <= kLdsLimit) { m->block_backward = bs; m->lds_backward = l; break; }
  }
  if (hipGetDevice(&m->dev) != hipSuccess) { delete m; return set_err(CF_E_DEVICE, "no HIP device"); }
  if (hipDeviceGetAttribute(&m->ncu, hipDeviceAttributeMultiprocessorCount, m->dev) != hipSuccess || m->ncu < 1)
    m->ncu = 256;

  // ---- per-world constants (float32); shared arrays get world stride 0
  std::vector<float4> bmi((size_t)nw * nb), gdat(wg), gpos, gquat;
  std::vector<float2> gfr2;
  for (size_t i = 0; i < (size_t)nw * nb; ++i) {
    const double *I = d->body_inertia + 3 * i;
    bmi[i] = make_float4((float)d->body_mass[i], (float)I[0], (float)I[1], (float)I[2]);
  }
  std::vector<float> gmu(wg);
  for (size_t i = 0; i < wg; ++i) {
    const double *s = d->geom_size + 3 * i, *f = d->geom_friction + 3 * i;
    gdat[i] = make_float4((float)s[0], (float)s[1], (float)s[2], (float)f[0]);
    gmu[i] = (float)f[0];
  }
  auto uniform = [&](const double *a, int width) {
    for (int w = 1; w < nw; ++w)
      if (std::memcmp(a, a + (size_t)w * ng * width, sizeof(double) * ng * width) != 0) return false;
    return true;
  };
  m->gpos_ws = (ng > 0 && uniform(d->geom_pos, 3)) ? 0 : ng;
  m->gquat_ws = (ng > 0 && uniform(d->geom_quat, 4)) ? 0 : ng;
  const size_t npw = m->gpos_ws ? wg : (size_t)ng, nqw = m->gquat_ws ? wg : (size_t)ng;
  gpos.resize(npw);
  gquat.resize(nqw);
  for (size_t i = 0; i < npw; ++i) {
    const double *p = d->geom_pos + 3 * i;
    gpos[i] = make_float4((float)p[0], (float)p[1], (float)p[2], 0.f);
  }
  for (size_t i = 0; i < nqw; ++i) {
    const double *q = d->geom_quat + 4 * i;
    gquat[i] = make_float4((float)q[0], (float)q[1], (float)q[2], (float)q[3]);  // (w,x,y,z) in (x,y,z,w)
  }
  if (m->condim >= 4) {
    gfr2.resize(wg);
    for (size_t i = 0; i < wg; ++i)
      gfr2[i] = make_float2((float)d->geom_friction[3 * i + 1], (float)d->geom_friction[3 * i + 2]);
  }
  std::vector<int> gbody(ng);
  for (int g = 0; g < ng; ++g) gbody[g] = d->geom_body[g];

  hipError_t e = hipSuccess;
  auto chk = [&](hipError_t r) { if (e == hipSuccess) e = r; };
  chk(upload(&m->d_slots, slots));
  chk(upload(&m->d_gbody, gbody));
  chk(upload(&m->d_gorient, gorient));
  chk(upload(&m->d_body, bodyc));
  chk(upload(&m->d_sub, subs));
  chk(upload(&m->d_jk64, jk64));
  if (any_small) {
    chk(hipMalloc((void **)&m->d_frames, sizeof(float4) * 5 * (size_t)nw * nb));
    if (e == hipSuccess) chk(hipMemset(m->d_frames, 0, sizeof(float4) * 5 * (size_t)nw * nb));
  }
  chk(upload(&m->d_bmi, bmi));
  chk(upload(&m->d_gdat, gdat));
  chk(upload(&m->d_gmu, gmu));
  chk(upload(&m->d_gpos, gpos));
  chk(upload(&m->d_gquat, gquat));
  if (m->condim >= 4) chk(upload(&m->d_gfr2, gfr2));
  const size_t ncap = (size_t)nw * (m->ncon_max > 0 ? m->ncon_max : 1);
  chk(hipMalloc((void **)&m->d_cnp, sizeof(float4) * ncap));
  chk(hipMalloc((void **)&m->d_cpos, sizeof(float4) * ncap));
  chk(hipMalloc((void **)&m->d_ncon, sizeof(int) * nw));
  chk(hipMalloc((void **)&m->d_over, sizeof(int) * nw));
  if (e == hipSuccess) chk(hipMemset(m->d_ncon, 0, sizeof(int) * nw));
  if (e != hipSuccess) {
    const bool oom = e == hipErrorOutOfMemory;
    std::string msg = std::string("device setup failed: ") + hipGetErrorString(e);
    free_model(m);
    return set_err(oom ? CF_E_NOMEM : CF_E_DEVICE, msg);
  }
  *out = m;
  if (skipped) {
    g_err = "some geom pairs have no contact rule and never collide";
    return CF_W_PAIRS_SKIPPED;
  }
  return CF_OK;
}

void cf_model_destroy(cf_model *m) {
  if (!m) return;
  (void)hipDeviceSynchronize();
  free_model(m);
}

cf_status cf_model_dims(const cf_model *m, int32_t *nq, int32_t *nv, int32_t *nf) {
  if (!m) return set_err(CF_E_INVALID_ARG, "model is NULL");
  if (nq) *nq = m->nq;
  if (nv) *nv = m->nv;
  if (nf) *nf = m->nf;
  return CF_OK;
}

static cf::CollideArgs collide_args(const cf_model *m) {
  cf::CollideArgs ca{};
  ca.gpos = m->d_gpos; ca.gquat = m->d_gquat; ca.gdat = m->d_gdat; ca.gbody = m->d_gbody;
  ca.gorient = m->d_gorient; ca.norient = m->norient;
  ca.body = m->d_body; ca.sub = m->d_sub; ca.nsub = m->nsub; ca.jk = m->d_jk64;
  ca.frames = m->d_frames;
  ca.slots = m->d_slots; ca.cnp = m->d_cnp; ca.cpos = m->d_cpos; ca.ncon = m->d_ncon; ca.overflow = m->d_over;
  ca.nq = m->nq; ca.nb = m->nb; ca.ng = m->ng; ca.nslot = m->nslot; ca.ncon_max = m->ncon_max;
  ca.gpos_ws = m->gpos_ws; ca.gquat_ws = m->gquat_ws; ca.margin = m->p.margin;
  ca.nslot_pre = m->nslot_pre; ca.sph0 = m->sph0; ca.nsph = m->nsph; ca.npl = m->npl; ca.sph_mfma = m->sph_mfma;
  return ca;
}

static cf::ResolveArgs resolve_args(const cf_model *m) {
  cf::ResolveArgs ra{};
  ra.bmi = m->d_bmi; ra.gdat = m->d_gdat; ra.gmu = m->d_gmu; ra.gfr2 = m->d_gfr2; ra.gbody = m->d_gbody;
  ra.body = m->d_body; ra.sub = m->d_sub; ra.nsub = m->nsub; ra.art_floats = art_region_floats(m);
  ra.frames = m->d_frames;
  ra.cnp = m->d_cnp; ra.cpos = m->d_cpos; ra.ncon = m->d_ncon;
  ra.nq = m->nq; ra.nv = m->nv; ra.nb = m->nb; ra.ng = m->ng; ra.ncon_max = m->ncon_max;
  ra.condim = m->condim; ra.nfacet = m->nf; ra.nbits = m->nbits; ra.p = m->p; ra.act = m->d_act;
  ra.nworld = m->nw;
  return ra;
}

// Worlds of free bodies (no actuators, no learned gains) take the persistent
// free-body rollout kernel (one wave per world, contacts in the global
// workspace); other models the general one when a world fits its LDS.
static bool rollout_free(const cf_model *m) {
  return m->lds_rollout_free > 0 && m->lds_rollout_free <= kLdsLimit && !m->d_act && !m->mlp;
}

// Worlds of at most 64 free bodies (no actuators, no learned gains) at the
// one-wave launch shapes: cf_step runs the narrow phase and the resolution of
// each world in one kernel (not while kernel timing is on, which times the two
// kernels apart).
static bool step_fused(const cf_model *m) {
  return !m->prof && !m->mlp && !m->d_act && m->nsub == 0 && m->nb >= 1 && m->nb <= 64 &&
         m->block_collide == 64 && m->block_resolve == 64 &&
         std::max(m->lds_collide, m->lds_resolve_free) <= kLdsLimit;
}

// Models with articulated subtrees (no learned gains) at the one-wave launch
// shapes: the same, the narrow phase and the general resolution in one kernel.
static bool step_fused_art(const cf_model *m) {
  return !m->prof && !m->mlp && m->nsub > 0 && m->nb >= 1 && m->block_collide == 64 && m->block_resolve == 64 &&
         std::max(m->lds_collide, m->lds_resolve) <= kLdsLimit;
}

static bool rollout_fused(const cf_model *m) {
  return !m->rollout_steps && !m->mlp && (rollout_free(m) || m->lds_rollout <= kLdsLimit);
}

// Learned gains on the register-resident resolution (several worlds per
// workgroup sharing the network's K = 32 image): free bodies, at most 128.
static bool learned_k32(const cf_model *m) {
  return m->nsub == 0 && !m->d_act && m->nb <= 128 &&
         cf::resolve_learned_k32_lds_bytes(m->nb, m->ng) <= kLdsLimit;
}

// The resolution launch of a step: worlds of free bodies that fit the
// workgroup one body per lane take the register-resident kernel; with learned
// gains the network's LDS image is first written from the current parameters
// (one small kernel), then the resolution copies it to LDS and runs at most
// 128 threads per world.
static hipError_t launch_resolve_model(const cf_model *m, cf::ResolveArgs ra, hipStream_t s) {
  if (!m->mlp && !m->d_act && m->nsub == 0 && m->nb <= m->block_resolve)
    return cf::launch_resolve_free(ra, m->nw, m->block_resolve, m->lds_resolve_free, s);
  if (!m->mlp) return cf::launch_resolve(ra, m->nw, m->block_resolve, m->lds_resolve, s);
  if (learned_k32(m)) {
    ra.mlp = m->mlp;
    ra.mlp_img = m->d_mlp_img;
    const hipError_t e = cf::launch_mlp_pack_k32(m->mlp, m->d_mlp_img, s);
    if (e != hipSuccess) return e;
    return cf::launch_resolve_learned(ra, m->nw, cf::resolve_learned_k32_lds_bytes(m->nb, m->ng), s);
  }
  const int block = m->block_resolve > 128 ? 128 : m->block_resolve;
  ra.mlp = m->mlp;
  ra.mlp_img = m->d_mlp_img;
  const hipError_t e = cf::launch_mlp_pack(m->mlp, m->d_mlp_img, s);
  if (e != hipSuccess) return e;
  const size_t lds = cf::resolve_lds_bytes(m->nq, m->nv, m->nb, m->ng, 0, 0) + cf::resolve_learned_lds_bytes(block);
  return cf::launch_resolve(ra, m->nw, block, lds, s);
}

cf_status cf_step(cf_model *m, void *stream, const float *q, const float *v, const float *tau,
                  float *q_out, float *v_out, const cf_contacts *out) {
  if (!m) return set_err(CF_E_INVALID_ARG, "model is NULL");
  if (!q || !v || !q_out || !v_out) return set_err(CF_E_INVALID_ARG, "q, v, q_out, v_out must be non-NULL");
  if (!aligned16(q) || !aligned16(v) || !aligned16(q_out) || !aligned16(v_out) || (tau && !aligned16(tau)))
    return set_err(CF_E_INVALID_ARG, "state buffers must be 16-byte aligned");
  if ((q_out != q && q_out < q + (size_t)m->nw * m->nq && q < q_out + (size_t)m->nw * m->nq) ||
      (v_out != v && v_out < v + (size_t)m->nw * m->nv && v < v_out + (size_t)m->nw * m->nv))
    return set_err(CF_E_INVALID_ARG, "outputs may alias inputs only exactly");
  hipStream_t s = (hipStream_t)stream;
  EventSet *ev = nullptr;
  if (m->prof) {
    if (m->ev_used == m->events.size()) {
      if (m->events.size() >= 4096) {
        cf_status st = drain_events(m);
        if (st != CF_OK) return st;
      } else {
        EventSet es;
        for (auto &x : es.e)
          if (hipEventCreate(&x) != hipSuccess) return set_err(CF_E_DEVICE, "hipEventCreate failed");
        m->events.push_back(es);
      }
    }
    ev = &m->events[m->ev_used++];
    if (hipEventRecord(ev->e[0], s) != hipSuccess) return set_err(CF_E_DEVICE, "hipEventRecord failed");
  }
  cf::CollideArgs ca = collide_args(m);
  ca.q = q;
  ca.ncon_out = out ? out->ncon : nullptr;
  ca.overflow_out = out ? out->overflow : nullptr;
  if (step_fused(m)) {
    cf::ResolveArgs ra = resolve_args(m);
    ra.q = q; ra.v = v; ra.tau = tau; ra.q_out = q_out; ra.v_out = v_out;
    if (out) {
      ra.x_geom = out->geom; ra.x_sub = out->sub; ra.x_dist = out->dist; ra.x_pos = out->pos;
      ra.x_frame = out->frame; ra.x_imp = out->impulse;
      ra.x_feat = out->features; ra.x_target = out->target;
      ra.x_fallback = out->fallback;
    }
    const hipError_t e = cf::launch_step_free(ca, ra, m->nw, std::max(m->lds_collide, m->lds_resolve_free), s);
    if (e != hipSuccess) return set_err(CF_E_DEVICE, std::string("step launch: ") + hipGetErrorString(e));
    return CF_OK;
  }
  if (step_fused_art(m)) {
    cf::ResolveArgs ra = resolve_args(m);
    ra.q = q; ra.v = v; ra.tau = tau; ra.q_out = q_out; ra.v_out = v_out;
    if (out) {
      ra.x_geom = out->geom; ra.x_sub = out->sub; ra.x_dist = out->dist; ra.x_pos = out->pos;
      ra.x_frame = out->frame; ra.x_imp = out->impulse;
      ra.x_fallback = out->fallback;
    }
    const hipError_t e = cf::launch_step_art(ca, ra, m->nw, std::max(m->lds_collide, m->lds_resolve), s);
    if (e != hipSuccess) return set_err(CF_E_DEVICE, std::string("step launch: ") + hipGetErrorString(e));
    return CF_OK;
  }
  hipError_t e = cf::launch_collide(ca, m->nw, m->block_collide, m->lds_collide, s);
  if (e != hipSuccess) return set_err(CF_E_DEVICE, std::string("collide launch: ") + hipGetErrorString(e));
  if (ev && hipEventRecord(ev->e[1], s) != hipSuccess) return set_err(CF_E_DEVICE, "hipEventRecord failed");

  cf::ResolveArgs ra = resolve_args(m);
  ra.q = q; ra.v = v; ra.tau = tau; ra.q_out = q_out; ra.v_out = v_out;
  if (out) {
    ra.x_geom = out->geom; ra.x_sub = out->sub; ra.x_dist = out->dist; ra.x_pos = out->pos;
    ra.x_frame = out->frame; ra.x_imp = out->impulse;
    if (m->nsub == 0) { ra.x_feat = out->features; ra.x_target = out->target; }
    ra.x_fallback = out->fallback;
  }
  e = launch_resolve_model(m, ra, s);
  if (e != hipSuccess) return set_err(CF_E_DEVICE, std::string("resolve launch: ") + hipGetErrorString(e));
  if (ev && hipEventRecord(ev->e[2], s) != hipSuccess) return set_err(CF_E_DEVICE, "hipEventRecord failed");
  return CF_OK;
}

cf_status cf_step_backward(cf_model *m, void *stream, const float *q, const float *v, const float *tau,
                           const float *gq_out, const float *gv_out, float *gq, float *gv, float *gtau) {
  if (!m) return set_err(CF_E_INVALID_ARG, "model is NULL");
  if (!q || !v || !gq || !gv) return set_err(CF_E_INVALID_ARG, "q, v, gq, gv must be non-NULL");
  const float *ptrs[] = {q, v, tau, gq_out, gv_out, gq, gv, gtau};
  for (const float *p : ptrs)
    if (p && !aligned16(p)) return set_err(CF_E_INVALID_ARG, "buffers must be 16-byte aligned");
  const size_t sq = (size_t)m->nw * m->nq, sv = (size_t)m->nw * m->nv;
  auto overlap = [](const float *x, size_t nx, const float *y, size_t ny) {
    return x && y && x < y + ny && y < x + nx;
  };
  // outputs may alias the incoming adjoints exactly, nothing else
  if (overlap(gq, sq, q, sq) || overlap(gq, sq, v, sv) || overlap(gq, sq, tau, sv) ||
      (gq != gq_out && overlap(gq, sq, gq_out, sq)) || overlap(gq, sq, gv_out, sv) ||
      overlap(gv, sv, q, sq) || overlap(gv, sv, v, sv) || overlap(gv, sv, tau, sv) ||
      overlap(gv, sv, gq_out, sq) || (gv != gv_out && overlap(gv, sv, gv_out, sv)) ||
      overlap(gv, sv, gq, sq) || overlap(gtau, sv, gq, sq) || overlap(gtau, sv, gv, sv) ||
      overlap(gtau, sv, q, sq) || overlap(gtau, sv, v, sv) || overlap(gtau, sv, tau, sv) ||
      overlap(gtau, sv, gq_out, sq) || overlap(gtau, sv, gv_out, sv))
    return set_err(CF_E_INVALID_ARG, "gq/gv may alias gq_out/gv_out only exactly; no other overlap");
  if (m->p.imp_diag && m->nsub > 0)
    return set_err(CF_E_UNSUPPORTED, "cf_step_backward covers the diagonal impedance on models of free bodies only");
  if (!m->block_backward) return set_err(CF_E_UNSUPPORTED, "world too large for the adjoint's LDS");
  hipStream_t s = (hipStream_t)stream;
  cf::CollideArgs ca = collide_args(m);
  ca.q = q;
  hipError_t e = cf::launch_collide(ca, m->nw, m->block_collide, m->lds_collide, s);
  if (e != hipSuccess) return set_err(CF_E_DEVICE, std::string("collide launch: ") + hipGetErrorString(e));
  cf::BackwardArgs b{};
  b.s = resolve_args(m);
  b.s.mlp = m->mlp;  // learned gains: the adjoint recomputes them from the float32 parameters
  b.s.q = q; b.s.v = v; b.s.tau = tau;
  b.gpos = m->d_gpos; b.gpos_ws = m->gpos_ws;
  b.gquat = m->d_gquat; b.gquat_ws = m->gquat_ws;
  b.gq_out = gq_out; b.gv_out = gv_out; b.gq = gq; b.gv = gv; b.gtau = gtau;
  e = cf::launch_backward(b, m->nw, m->block_backward, m->lds_backward, s);
  if (e != hipSuccess) return set_err(CF_E_DEVICE, std::string("backward launch: ") + hipGetErrorString(e));
  return CF_OK;
}

cf_status cf_rollout(cf_model *m, void *stream, int32_t T, const float *q0, const float *v0,
                     const float *tau_seq, float *q_traj, float *v_traj, int32_t *ncon_traj,
                     int32_t *overflow_traj) {
  if (!m) return set_err(CF_E_INVALID_ARG, "model is NULL");
  if (T < 0) return set_err(CF_E_INVALID_ARG, "T must be >= 0");
  if (!q0 || !v0 || !q_traj || !v_traj) return set_err(CF_E_INVALID_ARG, "NULL state pointer");
  if (!aligned16(q0) || !aligned16(v0) || !aligned16(q_traj) || !aligned16(v_traj) ||
      (tau_seq && !aligned16(tau_seq)))
    return set_err(CF_E_INVALID_ARG, "state buffers must be 16-byte aligned");
  const size_t sq = (size_t)m->nw * m->nq, sv = (size_t)m->nw * m->nv;
  hipStream_t s = (hipStream_t)stream;
  if (q0 != q_traj && hipMemcpyAsync(q_traj, q0, sizeof(float) * sq, hipMemcpyDeviceToDevice, s) != hipSuccess)
    return set_err(CF_E_DEVICE, "hipMemcpyAsync failed");
  if (v0 != v_traj && hipMemcpyAsync(v_traj, v0, sizeof(float) * sv, hipMemcpyDeviceToDevice, s) != hipSuccess)
    return set_err(CF_E_DEVICE, "hipMemcpyAsync failed");
  if (T == 0) return CF_OK;
  if (rollout_fused(m)) {
    cf::RolloutArgs r{};
    r.c = collide_args(m);
    r.s = resolve_args(m);
    r.q0 = q_traj; r.v0 = v_traj; r.tau_seq = tau_seq; r.q_traj = q_traj; r.v_traj = v_traj;
    r.ncon_traj = ncon_traj; r.over_traj = overflow_traj; r.T = T; r.nworld = m->nw; r.cap = m->ncon_max;
    // the free-body kernel sized for three resident waves per SIMD (twelve
    // one-wave worlds per CU, no register spills) while the batch fits the
    // device at that occupancy, else for four
    hipError_t e = rollout_free(m)
                       ? cf::launch_rollout_free(r, m->lds_rollout_free, m->nw <= 12 * m->ncu ? 3 : 4, s)
                       : cf::launch_rollout(r, m->block_rollout, m->lds_rollout, s);
    if (e != hipSuccess) return set_err(CF_E_DEVICE, std::string("rollout launch: ") + hipGetErrorString(e));
    return CF_OK;
  }
  for (int t = 0; t < T; ++t) {
    cf_contacts c{};
    c.ncon = ncon_traj ? ncon_traj + (size_t)t * m->nw : nullptr;
    c.overflow = overflow_traj ? overflow_traj + (size_t)t * m->nw : nullptr;
    cf_status st = cf_step(m, stream, q_traj + t * sq, v_traj + t * sv, tau_seq ? tau_seq + t * sv : nullptr,
                           q_traj + (t + 1) * sq, v_traj + (t + 1) * sv,
                           (ncon_traj || overflow_traj) ? &c : nullptr);
    if (st != CF_OK) return st;
  }
  return CF_OK;
}

cf_status cf_model_set_learned_impedance(cf_model *m, const float *params, float margin) {
  if (!m) return set_err(CF_E_INVALID_ARG, "model is NULL");
  if (!(margin >= 0.f) || !std::isfinite(margin)) return set_err(CF_E_INVALID_ARG, "margin must be finite and >= 0");
  if (!params) {
    m->mlp = nullptr;
    m->p.mlp_margin = margin;  // still sets the exported training targets
    return CF_OK;
  }
  if (!aligned16(params)) return set_err(CF_E_INVALID_ARG, "params must be 16-byte aligned");
  if (m->nsub > 0) return set_err(CF_E_UNSUPPORTED, "learned impedance covers models of free bodies only");
  if (m->p.imp_diag) return set_err(CF_E_UNSUPPORTED, "learned impedance scales the heuristic, not the diagonal form");
  const int block = m->block_resolve > 128 ? 128 : m->block_resolve;
  if (!learned_k32(m) &&
      cf::resolve_lds_bytes(m->nq, m->nv, m->nb, m->ng, 0, 0) + cf::resolve_learned_lds_bytes(block) > kLdsLimit)
    return set_err(CF_E_UNSUPPORTED, "world too large for the learned resolution's LDS");
  const size_t img = std::max(cf::mlp_image_bytes(), cf::mlp_image_k32_bytes());
  if (!m->d_mlp_img && hipMalloc((void **)&m->d_mlp_img, img) != hipSuccess) {
    m->d_mlp_img = nullptr;
    return set_err(CF_E_NOMEM, "learned-gain network image");
  }
  m->mlp = params;
  m->p.mlp_margin = margin;
  return CF_OK;
}

cf_status cf_model_set_impedance(cf_model *m, int32_t mode) {
  if (!m) return set_err(CF_E_INVALID_ARG, "model is NULL");
  if (mode == CF_IMPEDANCE_DIAGONAL && m->mlp)
    return set_err(CF_E_UNSUPPORTED, "switch the learned impedance off first");
  if (mode != CF_IMPEDANCE_HEURISTIC && mode != CF_IMPEDANCE_DIAGONAL)
    return set_err(CF_E_INVALID_ARG, "impedance mode must be CF_IMPEDANCE_HEURISTIC or CF_IMPEDANCE_DIAGONAL");
  if (mode == CF_IMPEDANCE_DIAGONAL && m->nsub > 0 &&
      cf::resolve_lds_bytes(m->nq, m->nv, m->nb, m->ng, m->nsub, m->art_floats + m->ydiag_floats) > kLdsLimit)
    return set_err(CF_E_UNSUPPORTED, "world too large for the diagonal impedance's LDS (L^-1 J^T per body)");
  m->p.imp_diag = mode == CF_IMPEDANCE_DIAGONAL ? 1 : 0;
  m->lds_resolve = cf::resolve_lds_bytes(m->nq, m->nv, m->nb, m->ng, m->nsub, art_region_floats(m));
  m->lds_rollout = rollout_lds(m);
  return CF_OK;
}

cf_status cf_model_set_actuators(cf_model *m, const float *kp, const float *kd) {
  if (!m) return set_err(CF_E_INVALID_ARG, "model is NULL");
  if (!kp && !kd) {
    if (m->d_act) (void)hipFree(m->d_act);
    m->d_act = nullptr;
    return CF_OK;
  }
  std::vector<float4> act(m->nv);
  bool any = false;
  for (int i = 0; i < m->nv; ++i) {
    const float p = kp ? kp[i] : 0.f, dd = kd ? kd[i] : 0.f;
    if (!(p >= 0.f && dd >= 0.f && std::isfinite(p) && std::isfinite(dd)))
      return set_err(CF_E_INVALID_ARG, "actuator gains must be finite and >= 0");
    const bool on = p != 0.f || dd != 0.f;
    if (on && m->dof_jnt[i] == CF_JNT_FREE) return set_err(CF_E_INVALID_ARG, "actuators only on hinge or slide dofs");
    any = any || on;
    int qi = on ? m->dof_q[i] : -1;
    float qf;
    memcpy(&qf, &qi, sizeof qf);
    act[i] = make_float4(p, dd, qf, 0.f);
  }
  if (!any) return cf_model_set_actuators(m, nullptr, nullptr);
  if (!m->d_act && hipMalloc((void **)&m->d_act, sizeof(float4) * (m->nv ? m->nv : 1)) != hipSuccess) {
    m->d_act = nullptr;
    return set_err(CF_E_NOMEM, "actuator table");
  }
  if (hipMemcpy(m->d_act, act.data(), sizeof(float4) * m->nv, hipMemcpyHostToDevice) != hipSuccess)
    return set_err(CF_E_DEVICE, "actuator table upload");
  return CF_OK;
}

cf_status cf_model_set_launch(cf_model *m, int32_t collide_block, int32_t resolve_block, int32_t rollout_block) {
  if (!m) return set_err(CF_E_INVALID_ARG, "model is NULL");
  auto ok = [](int b) { return b == 64 || b == 128 || b == 256; };
  if (!ok(collide_block) || !ok(resolve_block) || !ok(rollout_block))
    return set_err(CF_E_INVALID_ARG, "workgroup sizes must be 64, 128 or 256");
  m->block_collide = collide_block;
  m->block_resolve = resolve_block;
  m->block_rollout = rollout_block;
  m->rollout_steps = false;
  m->lds_rollout = rollout_lds(m);
  return CF_OK;
}

cf_status cf_model_get_launch(const cf_model *m, int32_t *collide_block, int32_t *resolve_block,
                              int32_t *rollout_block, int32_t *rollout_fused_kernel) {
  if (!m) return set_err(CF_E_INVALID_ARG, "model is NULL");
  if (collide_block) *collide_block = m->block_collide;
  if (resolve_block) *resolve_block = m->block_resolve;
  if (rollout_block) *rollout_block = m->block_rollout;
  if (rollout_fused_kernel) *rollout_fused_kernel = rollout_fused(m) ? 1 : 0;
  return CF_OK;
}

cf_status cf_model_autotune(cf_model *m, void *stream, const float *q, const float *v, int32_t steps,
                            float *best_step_us, float *best_rollout_step_us) {
  if (!m) return set_err(CF_E_INVALID_ARG, "model is NULL");
  if (!q || !v || steps < 1) return set_err(CF_E_INVALID_ARG, "need q, v and steps >= 1");
  hipStream_t s = (hipStream_t)stream;
  const size_t sq = (size_t)m->nw * m->nq, sv = (size_t)m->nw * m->nv;
  float *buf = nullptr;
  const size_t nbuf = 2 * (sq + sv) + (size_t)(steps + 1) * (sq + sv);
  if (hipMalloc((void **)&buf, sizeof(float) * nbuf) != hipSuccess) return set_err(CF_E_NOMEM, "autotune buffers");
  float *qa = buf, *va = qa + sq, *qb = va + sv, *vb = qb + sq, *qt = vb + sv, *vt = qt + (steps + 1) * sq;
  hipEvent_t e0, e1;
  (void)hipEventCreate(&e0);
  (void)hipEventCreate(&e1);
  const bool prof = m->prof;
  m->prof = false;
  const int sizes[3] = {64, 128, 256};
  float best = 1e30f, best_r = 1e30f;
  int bc = m->block_collide, br = m->block_resolve, bo = m->block_rollout;
  cf_status st = CF_OK;
  for (int ic = 0; ic < 3 && st == CF_OK; ++ic)
    for (int ir = 0; ir < 3 && st == CF_OK; ++ir) {
      m->block_collide = sizes[ic];
      m->block_resolve = sizes[ir];
      (void)hipMemcpyAsync(qa, q, sizeof(float) * sq, hipMemcpyDeviceToDevice, s);
      (void)hipMemcpyAsync(va, v, sizeof(float) * sv, hipMemcpyDeviceToDevice, s);
      st = cf_step(m, stream, qa, va, nullptr, qb, vb, nullptr);  // warm-up
      (void)hipEventRecord(e0, s);
      for (int t = 0; t < steps && st == CF_OK; ++t)
        st = (t & 1) ? cf_step(m, stream, qb, vb, nullptr, qa, va, nullptr)
                     : cf_step(m, stream, qa, va, nullptr, qb, vb, nullptr);
      (void)hipEventRecord(e1, s);
      (void)hipEventSynchronize(e1);
      float ms = 0;
      (void)hipEventElapsedTime(&ms, e0, e1);
      if (ms < best) { best = ms; bc = sizes[ic]; br = sizes[ir]; }
    }
  m->rollout_steps = false;
  for (int io = 0; io < 3 && st == CF_OK; ++io) {
    const size_t lds = rollout_lds(m);
    if (rollout_free(m) ? io > 0 : lds > kLdsLimit) continue;  // the free-body kernel has one shape
    m->block_rollout = sizes[io];
    m->lds_rollout = lds;
    st = cf_rollout(m, stream, 1, q, v, nullptr, qt, vt, nullptr, nullptr);  // warm-up
    (void)hipEventRecord(e0, s);
    if (st == CF_OK) st = cf_rollout(m, stream, steps, q, v, nullptr, qt, vt, nullptr, nullptr);
    (void)hipEventRecord(e1, s);
    (void)hipEventSynchronize(e1);
    float ms = 0;
    (void)hipEventElapsedTime(&ms, e0, e1);
    if (ms < best_r) { best_r = ms; bo = sizes[io]; }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipFree(buf);
  m->prof = prof;
  cf_status st2 = cf_model_set_launch(m, bc, br, bo);
  // the persistent kernel only when it beats T step calls of the chosen shape
  // by more than the run-to-run noise of these timings
  m->rollout_steps = !(best_r < 0.97f * best);
  if (st != CF_OK) return st;
  if (best_step_us) *best_step_us = best * 1e3f / steps;
  if (best_rollout_step_us) *best_rollout_step_us = best_r < 1e29f ? best_r * 1e3f / steps : -1.f;
  return st2;
}

cf_status cf_model_step_kernels(const cf_model *m, int32_t *nkernels) {
  if (!m || !nkernels) return set_err(CF_E_INVALID_ARG, "model and nkernels must be non-NULL");
  *nkernels = step_fused(m) || step_fused_art(m) ? 1 : 2;
  return CF_OK;
}

cf_status cf_model_set_profiling(cf_model *m, int32_t enable) {
  if (!m) return set_err(CF_E_INVALID_ARG, "model is NULL");
  if (!enable && m->prof) {
    cf_status st = drain_events(m);
    if (st != CF_OK) return st;
  }
  m->prof = enable != 0;
  return CF_OK;
}

cf_status cf_model_time_kernels(cf_model *m, void *stream, const float *q, const float *v, float *q_out,
                                float *v_out, int32_t reps, float *us_collide, float *us_resolve) {
  if (!m) return set_err(CF_E_INVALID_ARG, "model is NULL");
  if (!q || !v || !q_out || !v_out || reps < 1) return set_err(CF_E_INVALID_ARG, "need q, v, q_out, v_out and reps >= 1");
  if (!aligned16(q) || !aligned16(v) || !aligned16(q_out) || !aligned16(v_out))
    return set_err(CF_E_INVALID_ARG, "state buffers must be 16-byte aligned");
  if (q_out == q || v_out == v) return set_err(CF_E_INVALID_ARG, "q_out/v_out must not alias q/v here");
  hipStream_t s = (hipStream_t)stream;
  cf::CollideArgs ca = collide_args(m);
  ca.q = q;
  cf::ResolveArgs ra = resolve_args(m);
  ra.q = q; ra.v = v; ra.tau = nullptr; ra.q_out = q_out; ra.v_out = v_out;
  hipEvent_t e[3];
  for (auto &x : e)
    if (hipEventCreate(&x) != hipSuccess) return set_err(CF_E_DEVICE, "hipEventCreate failed");
  hipError_t err = cf::launch_collide(ca, m->nw, m->block_collide, m->lds_collide, s);
  if (err == hipSuccess) err = hipEventRecord(e[0], s);
  for (int i = 0; i < reps && err == hipSuccess; ++i)
    err = cf::launch_collide(ca, m->nw, m->block_collide, m->lds_collide, s);
  if (err == hipSuccess) err = hipEventRecord(e[1], s);
  for (int i = 0; i < reps && err == hipSuccess; ++i)
    err = launch_resolve_model(m, ra, s);
  if (err == hipSuccess) err = hipEventRecord(e[2], s);
  if (err == hipSuccess) err = hipEventSynchronize(e[2]);
  float t0 = 0.f, t1 = 0.f;
  if (err == hipSuccess) err = hipEventElapsedTime(&t0, e[0], e[1]);
  if (err == hipSuccess) err = hipEventElapsedTime(&t1, e[1], e[2]);
  for (auto &x : e) (void)hipEventDestroy(x);
  if (err != hipSuccess) return set_err(CF_E_DEVICE, std::string("kernel timing: ") + hipGetErrorString(err));
  if (us_collide) *us_collide = t0 * 1e3f / reps;
  if (us_resolve) *us_resolve = t1 * 1e3f / reps;
  return CF_OK;
}

cf_status cf_model_kernel_times(cf_model *m, double *ms_collide, double *ms_resolve, int64_t *nsteps) {
  if (!m) return set_err(CF_E_INVALID_ARG, "model is NULL");
  cf_status st = drain_events(m);
  if (st != CF_OK) return st;
  if (ms_collide) *ms_collide = m->ms_collide;
  if (ms_resolve) *ms_resolve = m->ms_resolve;
  if (nsteps) *nsteps = m->prof_steps;
  m->ms_collide = m->ms_resolve = 0;
  m->prof_steps = 0;
  return CF_OK;
}

}  // extern "C"

namespace cf {
// Error reporting for the other translation units of the library (the
// network kernels): records the message for cf_last_error().
cf_status api_error(cf_status st, const std::string &msg) { return set_err(st, msg); }
}  // namespace cf
