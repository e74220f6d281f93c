// cf_kernels.hip - gfx950 kernels of the complementarity-free contact step.
//
// Two kernels per step, each one workgroup (4 x wave64) per world:
//
//  collide_kernel  analytic narrow phase over the model's candidate slots
//                  (plane-sphere, plane-capsule, plane-box corner, sphere-sphere),
//                  in canonical order: float32 test of every slot, float64
//                  re-evaluation of the slots near contact (decision, gap,
//                  normal, point); an order-preserving block compaction (wave
//                  ballots + per-wave counts) writes the contact set to a flat
//                  structure-of-arrays buffer [world][ncon_max] in HBM.
//
//  resolve_kernel  smooth prediction v_s = v + h M^-1 (tau - c) (Eq. smooth_vel),
//                  one lane per contact: tangent basis, relative velocity at v_s,
//                  impedance A = r/(1-r)/(tr_a + tr_b) (Eqs. k_d_setting, r_scaling),
//                  facet impulses lambda*h = A max(-(k h + d) J~ v_s - k phi, 0)
//                  (Eq. cf_wrench) and the contact wrench J~^T lambda h; a
//                  deterministic per-body segmented reduction of the wrenches
//                  (wave64 ballot key matching, fixed summation order, no
//                  atomics); velocity correction v+ = v_s + M^-1 p
//                  (Eq. vel_correction) and semi-implicit Euler integration.
//
// Free bodies: M is block diagonal (m I3, R diag(I) R^T) and the COM trace of
// a body is 3/m, so the factorisation of M reduces to the per-body inverse
// inertia.  Apart from the float64 contact geometry, the step runs in float32.
#include "cf_internal.h"

namespace cf {

static __host__ __device__ inline int pad4(int n) { return (n + 3) & ~3; }

// ---------------------------------------------------------------- helpers
struct V3 { float x, y, z; };
__device__ inline V3 v3(float x, float y, float z) { return {x, y, z}; }
__device__ inline V3 operator+(V3 a, V3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
__device__ inline V3 operator-(V3 a, V3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
__device__ inline V3 operator*(float s, V3 a) { return {s * a.x, s * a.y, s * a.z}; }
__device__ inline float dot(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ inline V3 cross(V3 a, V3 b) {
  return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}

// Rotation matrix rows of the normalised quaternion (w, x, y, z).
__device__ inline void quat_rows(float qw, float qx, float qy, float qz, V3 &r0, V3 &r1, V3 &r2) {
  float inv = 1.0f / sqrtf(qw * qw + qx * qx + qy * qy + qz * qz);
  float w = qw * inv, x = qx * inv, y = qy * inv, z = qz * inv;
  r0 = v3(1.f - 2.f * (y * y + z * z), 2.f * (x * y - z * w), 2.f * (x * z + y * w));
  r1 = v3(2.f * (x * y + z * w), 1.f - 2.f * (x * x + z * z), 2.f * (y * z - x * w));
  r2 = v3(2.f * (x * z - y * w), 2.f * (y * z + x * w), 1.f - 2.f * (x * x + y * y));
}

// ====================================================================
// collision
// ====================================================================
// Every candidate slot is tested in float32; slots within a small band of
// contact are re-evaluated from float64 geometry, which decides the contact
// and supplies its gap, normal and point (rounded to float32 on store).  The
// gap enters the impulse multiplied by the contact stiffness, so its
// accuracy, not the dynamics', bounds the step's float32 error.
template <class T>
struct GeomRec {
  T p[3];   // world position
  T r[9];   // world rotation, row-major
  T s[3];   // size
  T pad;
};

size_t collide_lds_bytes(int nq, int ng) {
  return sizeof(float) * pad4(nq) + (sizeof(GeomRec<float>) + sizeof(GeomRec<double>)) * (size_t)ng;
}

// Geom pose from (world position, rotation rows) of its body and its local offset.
template <class T>
__device__ inline void geom_pose(const T *bp, const T *br, const float4 gp, const float4 gq, GeomRec<T> &o) {
  // rotation of the geom quaternion (w,x,y,z stored in x,y,z,w)
  const T qw = gq.x, qx = gq.y, qy = gq.z, qz = gq.w;
  const T inv = T(1) / sqrt(qw * qw + qx * qx + qy * qy + qz * qz);
  const T w = qw * inv, x = qx * inv, y = qy * inv, z = qz * inv;
  const T g[9] = {T(1) - T(2) * (y * y + z * z), T(2) * (x * y - z * w), T(2) * (x * z + y * w),
                  T(2) * (x * y + z * w), T(1) - T(2) * (x * x + z * z), T(2) * (y * z - x * w),
                  T(2) * (x * z - y * w), T(2) * (y * z + x * w), T(1) - T(2) * (x * x + y * y)};
  const T off[3] = {T(gp.x), T(gp.y), T(gp.z)};
  for (int i = 0; i < 3; ++i) {
    o.p[i] = bp[i] + br[3 * i] * off[0] + br[3 * i + 1] * off[1] + br[3 * i + 2] * off[2];
    for (int j = 0; j < 3; ++j)
      o.r[3 * i + j] = br[3 * i] * g[j] + br[3 * i + 1] * g[3 + j] + br[3 * i + 2] * g[6 + j];
  }
}

template <class T>
__device__ inline void quat_to_rot(T qw, T qx, T qy, T qz, T *R) {
  const T inv = T(1) / sqrt(qw * qw + qx * qx + qy * qy + qz * qz);
  const T w = qw * inv, x = qx * inv, y = qy * inv, z = qz * inv;
  R[0] = T(1) - T(2) * (y * y + z * z); R[1] = T(2) * (x * y - z * w); R[2] = T(2) * (x * z + y * w);
  R[3] = T(2) * (x * y + z * w); R[4] = T(1) - T(2) * (x * x + z * z); R[5] = T(2) * (y * z - x * w);
  R[6] = T(2) * (x * z - y * w); R[7] = T(2) * (y * z + x * w); R[8] = T(1) - T(2) * (x * x + y * y);
}

// Gap, normal (a -> b) and point of one candidate slot.
template <class T>
__device__ inline T eval_slot(uint32_t s, const GeomRec<T> *G, T n[3], T p[3]) {
  const GeomRec<T> &A = G[slot_ga(s)];
  const GeomRec<T> &B = G[slot_gb(s)];
  const uint32_t t = slot_type(s);
  const int sub = slot_sub(s);
  T phi;
  if (t == kSphereSphere) {
    const T d[3] = {B.p[0] - A.p[0], B.p[1] - A.p[1], B.p[2] - A.p[2]};
    const T dist = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    if (dist >= T(1e-12)) {
      n[0] = d[0] / dist; n[1] = d[1] / dist; n[2] = d[2] / dist;
    } else {
      n[0] = T(0); n[1] = T(0); n[2] = T(1);
    }
    phi = dist - A.s[0] - B.s[0];
    const T ra = A.s[0] + T(0.5) * phi;
    for (int i = 0; i < 3; ++i) p[i] = A.p[i] + ra * n[i];
    return phi;
  }
  n[0] = A.r[2]; n[1] = A.r[5]; n[2] = A.r[8];  // plane normal: local z
  T c[3] = {B.p[0], B.p[1], B.p[2]};
  if (t == kPlaneBox) {
    const T l0 = (sub & 1) ? B.s[0] : -B.s[0];
    const T l1 = (sub & 2) ? B.s[1] : -B.s[1];
    const T l2 = (sub & 4) ? B.s[2] : -B.s[2];
    for (int i = 0; i < 3; ++i) c[i] += B.r[3 * i] * l0 + B.r[3 * i + 1] * l1 + B.r[3 * i + 2] * l2;
    phi = n[0] * (c[0] - A.p[0]) + n[1] * (c[1] - A.p[1]) + n[2] * (c[2] - A.p[2]);
    for (int i = 0; i < 3; ++i) p[i] = c[i] - T(0.5) * phi * n[i];
    return phi;
  }
  if (t == kPlaneCapsule) {
    const T half = sub == 0 ? -B.s[1] : B.s[1];
    for (int i = 0; i < 3; ++i) c[i] += half * B.r[3 * i + 2];
  }
  phi = n[0] * (c[0] - A.p[0]) + n[1] * (c[1] - A.p[1]) + n[2] * (c[2] - A.p[2]) - B.s[0];
  const T rr = B.s[0] + T(0.5) * phi;
  for (int i = 0; i < 3; ++i) p[i] = c[i] - rr * n[i];
  return phi;
}

__global__ __launch_bounds__(kBlock) void collide_kernel(CollideArgs a) {
  extern __shared__ float4 lds[];
  const int w = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  float *sq = reinterpret_cast<float *>(lds);
  GeomRec<double> *Gd = reinterpret_cast<GeomRec<double> *>(lds + pad4(a.nq) / 4);
  GeomRec<float> *Gf = reinterpret_cast<GeomRec<float> *>(Gd + a.ng);
  __shared__ int wave_count[2][kWaves];

  const float *qw = a.q + (size_t)w * a.nq;
  for (int i = tid; i < a.nq; i += kBlock) sq[i] = qw[i];
  __syncthreads();

  // geom world poses in float64 (free bodies: body origin = COM, q = (x, quat))
  for (int g = tid; g < a.ng; g += kBlock) {
    const int b = a.gbody[g];
    const float4 gp = a.gpos[(size_t)w * a.gpos_ws + g];
    const float4 gq = a.gquat[(size_t)w * a.gquat_ws + g];
    const float4 gd = a.gdat[(size_t)w * a.ng + g];
    double bp[3] = {0.0, 0.0, 0.0}, br[9] = {1.0, 0.0, 0.0, 0.0, 1.0, 0.0, 0.0, 0.0, 1.0};
    if (b >= 0) {
      const float *qb = sq + 7 * b;
      bp[0] = qb[0]; bp[1] = qb[1]; bp[2] = qb[2];
      quat_to_rot<double>(qb[3], qb[4], qb[5], qb[6], br);
    }
    GeomRec<double> rd;
    geom_pose<double>(bp, br, gp, gq, rd);
    rd.s[0] = gd.x; rd.s[1] = gd.y; rd.s[2] = gd.z; rd.pad = 0.0;
    Gd[g] = rd;
    GeomRec<float> rf;
    for (int i = 0; i < 3; ++i) { rf.p[i] = (float)rd.p[i]; rf.s[i] = (float)rd.s[i]; }
    for (int i = 0; i < 9; ++i) rf.r[i] = (float)rd.r[i];
    rf.pad = 0.f;
    Gf[g] = rf;
  }
  __syncthreads();

  // candidate slots in canonical order; order-preserving compaction
  const size_t cbase = (size_t)w * a.ncon_max;
  const unsigned long long below = lane ? (~0ull >> (64 - lane)) : 0ull;
  int running = 0;
  for (int base = 0, it = 0; base < a.nslot; base += kBlock, ++it) {
    const int s = base + tid;
    bool hit = false;
    float4 cn, cp;
    if (s < a.nslot) {
      const uint32_t sl = a.slots[s];
      float nf[3], pf[3];
      const float phi32 = eval_slot<float>(sl, Gf, nf, pf);
      const GeomRec<float> &B = Gf[slot_gb(sl)];
      // float32 gap error is a few ulp of the coordinates involved
      const float band = 1e-4f + 1e-6f * (fabsf(B.p[0]) + fabsf(B.p[1]) + fabsf(B.p[2]) + B.s[0] + B.s[1] + B.s[2]);
      if (phi32 < a.margin + band) {
        double nd[3], pd[3];
        const double phi = eval_slot<double>(sl, Gd, nd, pd);
        hit = phi < (double)a.margin;
        cn = make_float4((float)nd[0], (float)nd[1], (float)nd[2], (float)phi);
        cp = make_float4((float)pd[0], (float)pd[1], (float)pd[2], __uint_as_float(sl));
      }
    }
    const unsigned long long m = __ballot(hit);
    if (lane == 0) wave_count[it & 1][wave] = __popcll(m);
    __syncthreads();
    int off = running, tot = 0;
#pragma unroll
    for (int i = 0; i < kWaves; ++i) {
      const int c = wave_count[it & 1][i];
      off += i < wave ? c : 0;
      tot += c;
    }
    if (hit) {
      const int idx = off + __popcll(m & below);
      if (idx < a.ncon_max) {
        a.cnp[cbase + idx] = cn;
        a.cpos[cbase + idx] = cp;
      }
    }
    running += tot;
  }
  if (tid == 0) {
    const int kept = running < a.ncon_max ? running : a.ncon_max;
    a.ncon[w] = kept;
    a.overflow[w] = running - kept;
    if (a.ncon_out) a.ncon_out[w] = kept;
    if (a.overflow_out) a.overflow_out[w] = running - kept;
  }
}

hipError_t launch_collide(const CollideArgs &a, int nworld, size_t lds, hipStream_t s) {
  hipLaunchKernelGGL(collide_kernel, dim3(nworld), dim3(kBlock), lds, s, a);
  return hipGetLastError();
}

// ====================================================================
// resolution
// ====================================================================
// LDS: q, v, tau rows; per body 7 float4 (com|invm, vs|tr, ws, Iinv a, Iinv b,
// accumulated force, accumulated torque); per geom float4 friction + int body;
// per lane the two wrench entries of its contact (float4 + float2 each).
size_t resolve_lds_bytes(int nq, int nv, int nb, int ng) {
  return sizeof(float) * (pad4(nq) + 2 * (size_t)pad4(nv)) + sizeof(float4) * 7 * (size_t)nb +
         sizeof(float4) * (size_t)ng + (sizeof(float4) + sizeof(float2)) * 2 * kBlock +
         sizeof(int) * (size_t)pad4(ng);
}

template <int CONDIM>
__global__ __launch_bounds__(kBlock) void resolve_kernel(ResolveArgs a) {
  constexpr int NF = CONDIM == 1 ? 1 : CONDIM == 3 ? 4 : CONDIM == 4 ? 6 : 10;
  extern __shared__ float4 lds[];
  const int w = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int nq = a.nq, nv = a.nv, nb = a.nb, ng = a.ng;
  float *sq = reinterpret_cast<float *>(lds);
  float *sv = sq + pad4(nq);
  float *st = sv + pad4(nv);
  float4 *bC = reinterpret_cast<float4 *>(st + pad4(nv));
  float4 *bV = bC + nb, *bW = bV + nb, *bI0 = bW + nb, *bI1 = bI0 + nb;
  float4 *accF = bI1 + nb, *accT = accF + nb;
  float4 *gM = accT + nb;
  float4 *vA = gM + ng, *vB = vA + kBlock;
  float2 *vA2 = reinterpret_cast<float2 *>(vB + kBlock), *vB2 = vA2 + kBlock;
  int *gB = reinterpret_cast<int *>(vB2 + kBlock);
  const Params P = a.p;

  // ---- stage the world's rows (coalesced) and per-geom constants
  {
    const float *qw = a.q + (size_t)w * nq, *vw = a.v + (size_t)w * nv;
    for (int i = tid; i < nq; i += kBlock) sq[i] = qw[i];
    for (int i = tid; i < nv; i += kBlock) sv[i] = vw[i];
    if (a.tau) {
      const float *tw = a.tau + (size_t)w * nv;
      for (int i = tid; i < nv; i += kBlock) st[i] = tw[i];
    } else {
      for (int i = tid; i < nv; i += kBlock) st[i] = 0.f;
    }
    for (int g = tid; g < ng; g += kBlock) {
      gB[g] = a.gbody[g];
      const float mu_t = a.gdat[(size_t)w * ng + g].w;
      float2 fr = make_float2(0.f, 0.f);
      if (CONDIM >= 4) fr = a.gfr2[(size_t)w * ng + g];
      gM[g] = make_float4(mu_t, fr.x, fr.y, 0.f);
    }
  }
  __syncthreads();

  // ---- per body: M blocks, bias, smooth prediction (Eq. smooth_vel), trace 3/m
  for (int b = tid; b < nb; b += kBlock) {
    const float4 mi = a.bmi[(size_t)w * nb + b];
    const float *qb = sq + 7 * b, *vb = sv + 6 * b, *tb = st + 6 * b;
    V3 r0, r1, r2;
    quat_rows(qb[3], qb[4], qb[5], qb[6], r0, r1, r2);
    const float invm = 1.0f / mi.x;
    const float i0 = mi.y, i1 = mi.z, i2 = mi.w;
    const float j0 = 1.0f / i0, j1 = 1.0f / i1, j2 = 1.0f / i2;
    // world inertia Iw = R diag(I) R^T and its inverse R diag(1/I) R^T (symmetric)
    const V3 c0 = v3(r0.x, r1.x, r2.x), c1 = v3(r0.y, r1.y, r2.y), c2 = v3(r0.z, r1.z, r2.z);
    (void)c0; (void)c1; (void)c2;
    auto sym = [&](float d0, float d1, float d2, float *o) {
      o[0] = r0.x * d0 * r0.x + r0.y * d1 * r0.y + r0.z * d2 * r0.z;  // xx
      o[1] = r1.x * d0 * r1.x + r1.y * d1 * r1.y + r1.z * d2 * r1.z;  // yy
      o[2] = r2.x * d0 * r2.x + r2.y * d1 * r2.y + r2.z * d2 * r2.z;  // zz
      o[3] = r0.x * d0 * r1.x + r0.y * d1 * r1.y + r0.z * d2 * r1.z;  // xy
      o[4] = r0.x * d0 * r2.x + r0.y * d1 * r2.y + r0.z * d2 * r2.z;  // xz
      o[5] = r1.x * d0 * r2.x + r1.y * d1 * r2.y + r1.z * d2 * r2.z;  // yz
    };
    float Iw[6], Ii[6];
    sym(i0, i1, i2, Iw);
    sym(j0, j1, j2, Ii);
    const V3 om = v3(vb[3], vb[4], vb[5]);
    const V3 Io = v3(Iw[0] * om.x + Iw[3] * om.y + Iw[4] * om.z,
                     Iw[3] * om.x + Iw[1] * om.y + Iw[5] * om.z,
                     Iw[4] * om.x + Iw[5] * om.y + Iw[2] * om.z);
    const V3 gyro = cross(om, Io);  // velocity-product part of c
    const V3 ta = v3(tb[3] - gyro.x, tb[4] - gyro.y, tb[5] - gyro.z);
    const V3 dw = v3(Ii[0] * ta.x + Ii[3] * ta.y + Ii[4] * ta.z,
                     Ii[3] * ta.x + Ii[1] * ta.y + Ii[5] * ta.z,
                     Ii[4] * ta.x + Ii[5] * ta.y + Ii[2] * ta.z);
    // c_lin = -m g, so M^-1 (tau - c) = tau/m + g for the linear block
    const V3 vs = v3(vb[0] + P.h * (tb[0] * invm + P.gx), vb[1] + P.h * (tb[1] * invm + P.gy),
                     vb[2] + P.h * (tb[2] * invm + P.gz));
    const V3 ws = om + P.h * dw;
    bC[b] = make_float4(qb[0], qb[1], qb[2], invm);
    bV[b] = make_float4(vs.x, vs.y, vs.z, 3.0f * invm);
    bW[b] = make_float4(ws.x, ws.y, ws.z, 0.f);
    bI0[b] = make_float4(Ii[0], Ii[1], Ii[2], Ii[3]);
    bI1[b] = make_float4(Ii[4], Ii[5], 0.f, 0.f);
    accF[b] = make_float4(0.f, 0.f, 0.f, 0.f);
    accT[b] = make_float4(0.f, 0.f, 0.f, 0.f);
  }
  __syncthreads();

  // ---- contacts: facet impulses, wrenches, deterministic per-body reduction
  const int nc = a.ncon[w];
  const size_t cbase = (size_t)w * a.ncon_max;
  const unsigned long long below = lane ? (~0ull >> (64 - lane)) : 0ull;
  const float aa = P.k_user * P.h + P.d_user;
  for (int base = 0; base < nc; base += kBlock) {
    const int k = base + tid;
    int kA = nb, kB = nb;  // key nb = no body (static geom or idle lane)
    float4 WA = make_float4(0.f, 0.f, 0.f, 0.f), WB = WA;
    float2 WA2 = make_float2(0.f, 0.f), WB2 = WA2;
    if (k < nc) {
      const float4 cn = a.cnp[cbase + k], cp = a.cpos[cbase + k];
      const uint32_t sl = __float_as_uint(cp.w);
      const int ga = slot_ga(sl), gb = slot_gb(sl);
      const int ba = gB[ga], bb = gB[gb];
      const V3 n = v3(cn.x, cn.y, cn.z), p = v3(cp.x, cp.y, cp.z);
      const float phi = cn.w;
      // tangent basis
      V3 t1 = fabsf(n.x) <= 0.5f ? v3(1.f - n.x * n.x, -n.x * n.y, -n.x * n.z)
                                 : v3(-n.y * n.x, 1.f - n.y * n.y, -n.y * n.z);
      t1 = (1.0f / sqrtf(dot(t1, t1))) * t1;
      const V3 t2 = cross(n, t1);
      // relative velocity at v_s (b minus a)
      V3 vrel = v3(0.f, 0.f, 0.f), wrel = vrel;
      float trs = 0.f;
      V3 ra = vrel, rb = vrel;
      if (bb >= 0) {
        const float4 C = bC[bb], Vb = bV[bb], Wb = bW[bb];
        rb = p - v3(C.x, C.y, C.z);
        const V3 wb = v3(Wb.x, Wb.y, Wb.z);
        vrel = v3(Vb.x, Vb.y, Vb.z) + cross(wb, rb);
        wrel = wb;
        trs += Vb.w;
      }
      if (ba >= 0) {
        const float4 C = bC[ba], Va = bV[ba], Wa = bW[ba];
        ra = p - v3(C.x, C.y, C.z);
        const V3 wa = v3(Wa.x, Wa.y, Wa.z);
        vrel = vrel - (v3(Va.x, Va.y, Va.z) + cross(wa, ra));
        wrel = wrel - wa;
        trs += Va.w;
      }
      const float4 ma = gM[ga], mb = gM[gb];
      const float mut = fmaxf(ma.x, mb.x), mutor = fmaxf(ma.y, mb.y), murol = fmaxf(ma.z, mb.z);
      // impedance (Eqs. k_d_setting, r_scaling), x clamped to [0, 1]
      const float x = fminf(fabsf(phi) / P.width, 1.0f);
      const float gam = x < P.mid ? P.mid * powf(x / P.mid, P.power)
                                  : 1.0f - (1.0f - P.mid) * powf((1.0f - x) / (1.0f - P.mid), P.power);
      const float r = P.r_min + (P.r_max - P.r_min) * gam;
      const float A = trs > 0.f ? (r / (1.0f - r)) / trs : 0.f;
      const float c0 = -P.k_user * phi;
      const float vn = dot(n, vrel);
      float lam[NF];
      V3 f, tc = v3(0.f, 0.f, 0.f);
      if (CONDIM == 1) {
        lam[0] = A * fmaxf(-aa * vn + c0, 0.f);
        f = lam[0] * n;
      } else {
        const float u1 = dot(t1, vrel), u2 = dot(t2, vrel);
        lam[0] = A * fmaxf(-aa * (vn - mut * u1) + c0, 0.f);
        lam[1] = A * fmaxf(-aa * (vn - mut * u2) + c0, 0.f);
        lam[2] = A * fmaxf(-aa * (vn + mut * u1) + c0, 0.f);
        lam[3] = A * fmaxf(-aa * (vn + mut * u2) + c0, 0.f);
        float N = lam[0] + lam[1] + lam[2] + lam[3];
        const float e1 = -mut * (lam[0] - lam[2]), e2 = -mut * (lam[1] - lam[3]);
        if (CONDIM >= 4) {
          const float wt = dot(n, wrel);
          lam[4] = A * fmaxf(-aa * (vn - mutor * wt) + c0, 0.f);
          lam[5] = A * fmaxf(-aa * (vn + mutor * wt) + c0, 0.f);
          N += lam[4] + lam[5];
          tc = (-mutor * (lam[4] - lam[5])) * n;
        }
        if (CONDIM == 6) {
          const float o1 = dot(t1, wrel), o2 = dot(t2, wrel);
          lam[6] = A * fmaxf(-aa * (vn - murol * o1) + c0, 0.f);
          lam[7] = A * fmaxf(-aa * (vn - murol * o2) + c0, 0.f);
          lam[8] = A * fmaxf(-aa * (vn + murol * o1) + c0, 0.f);
          lam[9] = A * fmaxf(-aa * (vn + murol * o2) + c0, 0.f);
          N += lam[6] + lam[7] + lam[8] + lam[9];
          tc = tc + (-murol * (lam[6] - lam[8])) * t1 + (-murol * (lam[7] - lam[9])) * t2;
        }
        f = N * n + e1 * t1 + e2 * t2;
      }
      if (bb >= 0) {
        const V3 T = cross(rb, f) + tc;
        kB = bb;
        WB = make_float4(f.x, f.y, f.z, T.x);
        WB2 = make_float2(T.y, T.z);
      }
      if (ba >= 0) {
        const V3 T = cross(ra, f) + tc;
        kA = ba;
        WA = make_float4(-f.x, -f.y, -f.z, -T.x);
        WA2 = make_float2(-T.y, -T.z);
      }
      // optional exports
      const size_t ci = cbase + k;
      if (a.x_geom) { a.x_geom[2 * ci] = ga; a.x_geom[2 * ci + 1] = gb; }
      if (a.x_sub) a.x_sub[ci] = slot_sub(sl);
      if (a.x_dist) a.x_dist[ci] = phi;
      if (a.x_pos) { a.x_pos[3 * ci] = p.x; a.x_pos[3 * ci + 1] = p.y; a.x_pos[3 * ci + 2] = p.z; }
      if (a.x_frame) {
        float *fr = a.x_frame + 9 * ci;
        fr[0] = n.x; fr[1] = n.y; fr[2] = n.z;
        fr[3] = t1.x; fr[4] = t1.y; fr[5] = t1.z;
        fr[6] = t2.x; fr[7] = t2.y; fr[8] = t2.z;
      }
      if (a.x_imp) {
#pragma unroll
        for (int i = 0; i < NF; ++i) a.x_imp[(size_t)NF * ci + i] = lam[i];
      }
    }
    vA[tid] = WA; vA2[tid] = WA2;
    vB[tid] = WB; vB2[tid] = WB2;
    __syncthreads();

    // Key matching inside the wave: each lane learns which lanes carry the
    // same body on side a and on side b (one ballot per key bit and side).
    unsigned long long eAA = ~0ull, eAB = ~0ull, eBA = ~0ull, eBB = ~0ull;
    for (int i = 0; i < a.nbits; ++i) {
      const bool a1 = (kA >> i) & 1, b1 = (kB >> i) & 1;
      const unsigned long long bA = __ballot(a1), bBv = __ballot(b1);
      eAA &= a1 ? bA : ~bA;
      eAB &= a1 ? bBv : ~bBv;
      eBA &= b1 ? bA : ~bA;
      eBB &= b1 ? bBv : ~bBv;
    }
    // Leader of a key: its first side-a lane, else its first side-b lane.
    // It sums the key's entries in lane order, side a before side b.
    const bool leadA = kA < nb && !(eAA & below);
    const bool leadB = kB < nb && !eBA && !(eBB & below);
    const int wb0 = wave * 64;
    float4 SA = make_float4(0.f, 0.f, 0.f, 0.f), SB = SA;
    float2 SA2 = make_float2(0.f, 0.f), SB2 = SA2;
    if (leadA) {
      for (unsigned long long m = eAA; m; m &= m - 1) {
        const int l = wb0 + __ffsll((unsigned long long)m) - 1;
        const float4 u = vA[l]; const float2 u2 = vA2[l];
        SA.x += u.x; SA.y += u.y; SA.z += u.z; SA.w += u.w; SA2.x += u2.x; SA2.y += u2.y;
      }
      for (unsigned long long m = eAB; m; m &= m - 1) {
        const int l = wb0 + __ffsll((unsigned long long)m) - 1;
        const float4 u = vB[l]; const float2 u2 = vB2[l];
        SA.x += u.x; SA.y += u.y; SA.z += u.z; SA.w += u.w; SA2.x += u2.x; SA2.y += u2.y;
      }
    }
    if (leadB) {
      for (unsigned long long m = eBB; m; m &= m - 1) {
        const int l = wb0 + __ffsll((unsigned long long)m) - 1;
        const float4 u = vB[l]; const float2 u2 = vB2[l];
        SB.x += u.x; SB.y += u.y; SB.z += u.z; SB.w += u.w; SB2.x += u2.x; SB2.y += u2.y;
      }
    }
    // waves add their partial sums in wave order (keys are distinct within a wave)
#pragma unroll
    for (int wv = 0; wv < kWaves; ++wv) {
      if (wave == wv) {
        if (leadA) {
          float4 F = accF[kA], T = accT[kA];
          F.x += SA.x; F.y += SA.y; F.z += SA.z;
          T.x += SA.w; T.y += SA2.x; T.z += SA2.y;
          accF[kA] = F; accT[kA] = T;
        }
        if (leadB) {
          float4 F = accF[kB], T = accT[kB];
          F.x += SB.x; F.y += SB.y; F.z += SB.z;
          T.x += SB.w; T.y += SB2.x; T.z += SB2.y;
          accF[kB] = F; accT[kB] = T;
        }
      }
      __syncthreads();
    }
  }

  // ---- velocity correction (Eq. vel_correction) and semi-implicit Euler
  for (int b = tid; b < nb; b += kBlock) {
    const float4 C = bC[b], Vs = bV[b], Ws = bW[b], I0 = bI0[b], I1 = bI1[b];
    const float4 F = accF[b], T = accT[b];
    const V3 vp = v3(Vs.x + C.w * F.x, Vs.y + C.w * F.y, Vs.z + C.w * F.z);
    const V3 wp = v3(Ws.x + I0.x * T.x + I0.w * T.y + I1.x * T.z,
                     Ws.y + I0.w * T.x + I0.y * T.y + I1.y * T.z,
                     Ws.z + I1.x * T.x + I1.y * T.y + I0.z * T.z);
    float *qb = sq + 7 * b, *vb = sv + 6 * b;
    vb[0] = vp.x; vb[1] = vp.y; vb[2] = vp.z; vb[3] = wp.x; vb[4] = wp.y; vb[5] = wp.z;
    qb[0] = C.x + P.h * vp.x;
    qb[1] = C.y + P.h * vp.y;
    qb[2] = C.z + P.h * vp.z;
    // quat <- normalize(exp(h w) (x) quat), world-frame angular velocity
    const V3 th = P.h * wp;
    const float ang = sqrtf(dot(th, th));
    float ew, ex, ey, ez;
    if (ang < 1e-8f) {
      ew = 1.f; ex = 0.5f * th.x; ey = 0.5f * th.y; ez = 0.5f * th.z;
    } else {
      const float s = sinf(0.5f * ang) / ang;
      ew = cosf(0.5f * ang); ex = s * th.x; ey = s * th.y; ez = s * th.z;
    }
    const float qw0 = qb[3], qx0 = qb[4], qy0 = qb[5], qz0 = qb[6];
    const float nw_ = ew * qw0 - ex * qx0 - ey * qy0 - ez * qz0;
    const float nx_ = ew * qx0 + ex * qw0 + ey * qz0 - ez * qy0;
    const float ny_ = ew * qy0 - ex * qz0 + ey * qw0 + ez * qx0;
    const float nz_ = ew * qz0 + ex * qy0 - ey * qx0 + ez * qw0;
    const float inv = 1.0f / sqrtf(nw_ * nw_ + nx_ * nx_ + ny_ * ny_ + nz_ * nz_);
    qb[3] = nw_ * inv; qb[4] = nx_ * inv; qb[5] = ny_ * inv; qb[6] = nz_ * inv;
  }
  __syncthreads();
  {
    float *qo = a.q_out + (size_t)w * nq, *vo = a.v_out + (size_t)w * nv;
    for (int i = tid; i < nq; i += kBlock) qo[i] = sq[i];
    for (int i = tid; i < nv; i += kBlock) vo[i] = sv[i];
  }
}

hipError_t launch_resolve(const ResolveArgs &a, int nworld, size_t lds, hipStream_t s) {
  switch (a.condim) {
    case 1: hipLaunchKernelGGL(resolve_kernel<1>, dim3(nworld), dim3(kBlock), lds, s, a); break;
    case 3: hipLaunchKernelGGL(resolve_kernel<3>, dim3(nworld), dim3(kBlock), lds, s, a); break;
    case 4: hipLaunchKernelGGL(resolve_kernel<4>, dim3(nworld), dim3(kBlock), lds, s, a); break;
    case 6: hipLaunchKernelGGL(resolve_kernel<6>, dim3(nworld), dim3(kBlock), lds, s, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace cf
