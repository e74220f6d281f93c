// cf_kernels.hip - gfx950 kernels of the complementarity-free contact step.
//
// Two kernels per step, one workgroup per world (64, 128 or 256 threads):
//
//  collide_kernel  analytic narrow phase over the model's candidate slots
//                  (plane-sphere, plane-capsule, plane-box corner, sphere-sphere,
//                  box-sphere, box-capsule) in canonical order.  Pass 1 tests
//                  every slot in float32 on 16-byte LDS records and keeps, in
//                  order, the slots within a small band of contact; pass 2
//                  evaluates only those candidates (decision, gap, normal,
//                  point) from float64 geometry, except sphere pairs centred on
//                  their bodies (float32).  Static planes against a trailing
//                  block of spheres are tested as rows, and the block's pairs
//                  through hit masks (an MFMA Gram matrix for up to 64 spheres
//                  in one wave).  Compaction is in order with wave ballots plus
//                  per-wave counts, so contacts land in the flat
//                  structure-of-arrays buffer [world][ncon_max] without atomics.
//
//  resolve_kernel  smooth prediction v_s = v + h M^-1 (tau - c) (Eq. smooth_vel);
//                  one lane per contact: tangent basis, relative velocity at v_s,
//                  impedance A = r/(1-r)/(tr_a + tr_b) (Eqs. k_d_setting, r_scaling),
//                  facet impulses lambda*h = A max(-(k h + d) J~ v_s - k phi, 0)
//                  (Eq. cf_wrench) and the contact wrench J~^T lambda h; per-body
//                  sums of the wrenches in fixed point with LDS integer atomics
//                  (order-free, so bitwise reproducible; no global atomics);
//                  velocity correction v+ = v_s + M^-1 p (Eq. vel_correction)
//                  and semi-implicit Euler integration.  Worlds of free bodies
//                  take resolve_free_kernel: the same steps with each body's
//                  state held in its own lane.
//
// Free bodies: M is block diagonal (m I3, R diag(I) R^T) and the COM trace of
// a body is 3/m, so the factorisation of M reduces to the per-body inverse
// inertia.  Apart from the float64 contact geometry the step runs in float32.
#include "cf_internal.h"
#include "cf_adjoint.h"
#include "cf_artadj.h"
#include "cf_mlp.h"

namespace cf {

static __host__ __device__ inline int pad4(int n) { return (n + 3) & ~3; }

__device__ inline unsigned long long lanes_below(int lane) {
  return lane ? (~0ull >> (64 - lane)) : 0ull;
}

// Wave64 inclusive prefix sum and maximum over lanes by DPP row shifts and
// row broadcasts (no LDS round trips); the last lane holds the total.
__device__ inline int wave_incl_sum(int x) {
  int v = x;
  v += __builtin_amdgcn_update_dpp(0, v, 0x111, 0xF, 0xF, false);  // row_shr:1
  v += __builtin_amdgcn_update_dpp(0, v, 0x112, 0xF, 0xF, false);  // row_shr:2
  v += __builtin_amdgcn_update_dpp(0, v, 0x114, 0xF, 0xF, false);  // row_shr:4
  v += __builtin_amdgcn_update_dpp(0, v, 0x118, 0xF, 0xF, false);  // row_shr:8
  v += __builtin_amdgcn_update_dpp(0, v, 0x142, 0xA, 0xF, false);  // row_bcast:15 into rows 1, 3
  v += __builtin_amdgcn_update_dpp(0, v, 0x143, 0xC, 0xF, false);  // row_bcast:31 into rows 2, 3
  return v;
}
__device__ inline float wave_incl_sum(float x) {
  float v = x;
  const int z = 0;
  v += __int_as_float(__builtin_amdgcn_update_dpp(z, __float_as_int(v), 0x111, 0xF, 0xF, false));
  v += __int_as_float(__builtin_amdgcn_update_dpp(z, __float_as_int(v), 0x112, 0xF, 0xF, false));
  v += __int_as_float(__builtin_amdgcn_update_dpp(z, __float_as_int(v), 0x114, 0xF, 0xF, false));
  v += __int_as_float(__builtin_amdgcn_update_dpp(z, __float_as_int(v), 0x118, 0xF, 0xF, false));
  v += __int_as_float(__builtin_amdgcn_update_dpp(z, __float_as_int(v), 0x142, 0xA, 0xF, false));
  v += __int_as_float(__builtin_amdgcn_update_dpp(z, __float_as_int(v), 0x143, 0xC, 0xF, false));
  return v;
}
__device__ inline float wave_incl_max(float x) {
  float v = x;
  // lanes without a source keep their own value
  v = fmaxf(v, __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(v), __float_as_int(v), 0x111, 0xF, 0xF, false)));
  v = fmaxf(v, __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(v), __float_as_int(v), 0x112, 0xF, 0xF, false)));
  v = fmaxf(v, __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(v), __float_as_int(v), 0x114, 0xF, 0xF, false)));
  v = fmaxf(v, __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(v), __float_as_int(v), 0x118, 0xF, 0xF, false)));
  v = fmaxf(v, __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(v), __float_as_int(v), 0x142, 0xA, 0xF, false)));
  v = fmaxf(v, __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(v), __float_as_int(v), 0x143, 0xC, 0xF, false)));
  return v;
}
// Value of lane 63 (the total of an inclusive scan), wave-uniform.
__device__ inline int wave_last(int v) { return __builtin_amdgcn_readlane(v, 63); }
__device__ inline float wave_last(float v) { return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63)); }

// Exclusive prefix of `flag` over the workgroup in thread order; *total gets
// the workgroup count.  wcnt: shared [2][BS/64]; callers alternate `parity`
// so that consecutive calls need a single barrier each.
template <int BS>
__device__ inline int block_scan(bool flag, int *total, int *wcnt, int parity) {
  constexpr int NW = BS / 64;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const unsigned long long m = __ballot(flag);
  const int pre = __popcll(m & lanes_below(lane));
  if (NW == 1) {
    *total = __popcll(m);
    return pre;
  }
  if (lane == 0) wcnt[parity * NW + wave] = __popcll(m);
  __syncthreads();
  int off = 0, tot = 0;
#pragma unroll
  for (int i = 0; i < NW; ++i) {
    const int c = wcnt[parity * NW + i];
    off += i < wave ? c : 0;
    tot += c;
  }
  *total = tot;
  return off + pre;
}

// Exclusive prefix of the integers x over the workgroup in thread order;
// *total gets their sum.  wsum: shared [BS/64].  Ends with a barrier when
// BS > 64 (wsum may be reused at once).
template <int BS>
__device__ inline int block_scan_int(int x, int *total, int *wsum) {
  constexpr int NW = BS / 64;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int inc = wave_incl_sum(x);
  if (NW == 1) {
    *total = wave_last(inc);
    return inc - x;
  }
  if (lane == 63) wsum[wave] = inc;
  __syncthreads();
  int base = 0, tot = 0;
#pragma unroll
  for (int i = 0; i < NW; ++i) {
    const int c = wsum[i];
    base += i < wave ? c : 0;
    tot += c;
  }
  __syncthreads();
  *total = tot;
  return base + inc - x;
}

// Maximum over the workgroup (every thread gets it); wmax: shared [BS/64].
template <int BS>
__device__ inline float block_max(float x, float *wmax) {
  x = wave_last(wave_incl_max(x));
  if (BS == 64) return x;
  if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = x;
  __syncthreads();
  float m = wmax[0];
  for (int i = 1; i < BS / 64; ++i) m = fmaxf(m, wmax[i]);
  return m;
}

// Copy of a row of n floats from global memory to LDS with every load of the
// first K * BS elements issued before any is waited for (a plain strided loop
// would wait for each load before issuing the next).
template <int BS, int K>
struct RowStage {
  float r[K];
  // every lane issues all K loads (indices clamped to the row, values past
  // its end unused), so no wait sits between them and later loads
  __device__ inline void load(const float *src, int n) {
    if (n <= 0) return;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int i = threadIdx.x + k * BS;
      r[k] = src[i < n ? i : n - 1];
    }
  }
  __device__ inline void store(float *dst, const float *src, int n) const {
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int i = threadIdx.x + k * BS;
      if (i < n) dst[i] = r[k];
    }
    for (int i = threadIdx.x + K * BS; i < n; i += BS) dst[i] = src[i];
  }
};

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

template <class T>
__device__ inline void quat_to_rot(T qw, T qx, T qy, T qz, T *R) {
  const T inv = T(1) / sqrt(qw * qw + qx * qx + qy * qy + qz * qz);
  const T w = qw * inv, x = qx * inv, y = qy * inv, z = qz * inv;
  R[0] = T(1) - T(2) * (y * y + z * z); R[1] = T(2) * (x * y - z * w); R[2] = T(2) * (x * z + y * w);
  R[3] = T(2) * (x * y + z * w); R[4] = T(1) - T(2) * (x * x + z * z); R[5] = T(2) * (y * z - x * w);
  R[6] = T(2) * (x * z - y * w); R[7] = T(2) * (y * z + x * w); R[8] = T(1) - T(2) * (x * x + y * y);
}

// Rotation by angle th about the unit axis (ax, ay, az) (Rodrigues).
template <class T>
__device__ inline void axis_angle_rot(T ax, T ay, T az, T th, T *R) {
  const T c = cos(th), s = sin(th), C = T(1) - c;
  R[0] = c + ax * ax * C; R[1] = ax * ay * C - az * s; R[2] = ax * az * C + ay * s;
  R[3] = ay * ax * C + az * s; R[4] = c + ay * ay * C; R[5] = ay * az * C - ax * s;
  R[6] = az * ax * C - ay * s; R[7] = az * ay * C + ax * s; R[8] = c + az * az * C;
}

template <class T>
__device__ inline void mul33(const T *A, const T *B, T *O) {
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) O[3 * i + j] = A[3 * i] * B[j] + A[3 * i + 1] * B[3 + j] + A[3 * i + 2] * B[6 + j];
}

// Forward kinematics of bodies [b0, b0+n) (parents precede children).  Writes
// each body's frame origin org[4b..], rotation rows rot[12b..] (3 rows of 4)
// and, when given, its world joint axis ax[4b..] and centre of mass com[4b..].
template <class T>
__device__ void fk_range(int b0, int n, const BodyC *B, const float *q, T *org, T *rot, T *ax, T *com) {
  for (int b = b0; b < b0 + n; ++b) {
    const BodyC c = B[b];
    const float *qb = q + c.qadr;
    T o[3], R[9], aw[3] = {T(0), T(0), T(0)};
    if (c.jnt == kFree) {
      o[0] = qb[0]; o[1] = qb[1]; o[2] = qb[2];
      quat_to_rot<T>(qb[3], qb[4], qb[5], qb[6], R);
    } else {
      T po[3] = {T(0), T(0), T(0)}, pR[9] = {T(1), T(0), T(0), T(0), T(1), T(0), T(0), T(0), T(1)};
      if (c.parent >= 0) {
        for (int i = 0; i < 3; ++i) {
          po[i] = org[4 * c.parent + i];
          for (int j = 0; j < 3; ++j) pR[3 * i + j] = rot[12 * c.parent + 4 * i + j];
        }
      }
      T bq[9], R0[9];
      quat_to_rot<T>(c.quat.x, c.quat.y, c.quat.z, c.quat.w, bq);
      mul33<T>(pR, bq, R0);
      const T lp[3] = {c.pos.x, c.pos.y, c.pos.z}, la[3] = {c.axis.x, c.axis.y, c.axis.z};
      for (int i = 0; i < 3; ++i) {
        o[i] = po[i] + pR[3 * i] * lp[0] + pR[3 * i + 1] * lp[1] + pR[3 * i + 2] * lp[2];
        aw[i] = R0[3 * i] * la[0] + R0[3 * i + 1] * la[1] + R0[3 * i + 2] * la[2];
      }
      const T th = qb[0];
      if (c.jnt == kHinge) {
        T Rj[9];
        axis_angle_rot<T>(la[0], la[1], la[2], th, Rj);
        mul33<T>(R0, Rj, R);
      } else {
        for (int i = 0; i < 9; ++i) R[i] = R0[i];
        for (int i = 0; i < 3; ++i) o[i] += aw[i] * th;
      }
    }
    for (int i = 0; i < 3; ++i) {
      org[4 * b + i] = o[i];
      for (int j = 0; j < 3; ++j) rot[12 * b + 4 * i + j] = R[3 * i + j];
      if (ax) ax[4 * b + i] = aw[i];
    }
    if (com) {
      const T ip[3] = {c.ipos.x, c.ipos.y, c.ipos.z};
      for (int i = 0; i < 3; ++i) com[4 * b + i] = o[i] + R[3 * i] * ip[0] + R[3 * i + 1] * ip[1] + R[3 * i + 2] * ip[2];
    }
  }
}

// ====================================================================
// articulated subtrees (one lane per subtree, float32, LDS work block)
// ====================================================================
// Jacobian columns of body b's COM for every dof on its chain to the root:
// cols[6x] = (linear, angular) of chain entry x, idx[x] = dof index within the
// subtree.  free joint dof k: (e_k, 0) for k < 3, (e x (com_b - org_j), e) with
// e = e_{k-3}; hinge: (a x (com_b - org_j), a); slide: (a, 0).
__device__ inline int chain_cols(int b, int d0, const BodyC *B, const float4 *bO, const float4 *bAx,
                                 const float4 *bC, float *cols, int *idx) {
  int n = 0;
  const V3 cb = v3(bC[b].x, bC[b].y, bC[b].z);
  for (int j = b; j >= 0; j = B[j].parent) {
    const int jt = B[j].jnt, da = B[j].dadr;
    const V3 r = cb - v3(bO[j].x, bO[j].y, bO[j].z);
    const V3 aj = v3(bAx[j].x, bAx[j].y, bAx[j].z);
    if (jt == kFree) {
      for (int k = 0; k < 6; ++k) {
        float *c = cols + 6 * n;
        const V3 e = v3(k % 3 == 0 ? 1.f : 0.f, k % 3 == 1 ? 1.f : 0.f, k % 3 == 2 ? 1.f : 0.f);
        const V3 lin = k < 3 ? e : cross(e, r), ang = k < 3 ? v3(0.f, 0.f, 0.f) : e;
        c[0] = lin.x; c[1] = lin.y; c[2] = lin.z; c[3] = ang.x; c[4] = ang.y; c[5] = ang.z;
        idx[n++] = da + k - d0;
      }
    } else {
      float *c = cols + 6 * n;
      const V3 lin = jt == kHinge ? cross(aj, r) : aj, ang = jt == kHinge ? aj : v3(0.f, 0.f, 0.f);
      c[0] = lin.x; c[1] = lin.y; c[2] = lin.z; c[3] = ang.x; c[4] = ang.y; c[5] = ang.z;
      idx[n++] = da - d0;
    }
  }
  return n;
}

// World inertia R diag(I) R^T of a body from its rotation rows.
__device__ inline void world_inertia(const float4 *Rr, float4 mi, float *I /*xx yy zz xy xz yz*/) {
  const float d[3] = {mi.y, mi.z, mi.w};
  const float R[9] = {Rr[0].x, Rr[0].y, Rr[0].z, Rr[1].x, Rr[1].y, Rr[1].z, Rr[2].x, Rr[2].y, Rr[2].z};
  const int ri[6] = {0, 1, 2, 0, 0, 1}, rj[6] = {0, 1, 2, 1, 2, 2};
  for (int k = 0; k < 6; ++k) {
    const float *u = R + 3 * ri[k], *v = R + 3 * rj[k];
    I[k] = u[0] * d[0] * v[0] + u[1] * d[1] * v[1] + u[2] * d[2] * v[2];
  }
}
__device__ inline V3 sym_mul(const float *I, V3 x) {
  return v3(I[0] * x.x + I[3] * x.y + I[4] * x.z, I[3] * x.x + I[1] * x.y + I[5] * x.z,
            I[4] * x.x + I[5] * x.y + I[2] * x.z);
}

__device__ inline void chol_lower(float *M, int n) {
  for (int j = 0; j < n; ++j) {
    float s = M[j * n + j];
    for (int k = 0; k < j; ++k) s -= M[j * n + k] * M[j * n + k];
    const float l = sqrtf(fmaxf(s, 1e-30f));
    M[j * n + j] = l;
    const float il = 1.0f / l;
    for (int i = j + 1; i < n; ++i) {
      float t = M[i * n + j];
      for (int k = 0; k < j; ++k) t -= M[i * n + k] * M[j * n + k];
      M[i * n + j] = t * il;
    }
  }
}
__device__ inline void fwd_solve(const float *L, int n, float *x) {
  for (int i = 0; i < n; ++i) {
    float s = x[i];
    for (int k = 0; k < i; ++k) s -= L[i * n + k] * x[k];
    x[i] = s / L[i * n + i];
  }
}
__device__ inline void bwd_solve(const float *L, int n, float *x) {
  for (int i = n - 1; i >= 0; --i) {
    float s = x[i];
    for (int k = i + 1; k < n; ++k) s -= L[k * n + i] * x[k];
    x[i] = s / L[i * n + i];
  }
}

// Smooth prediction of one articulated subtree: FK, M = sum_b J_b^T diag(m, I_b) J_b,
// bias c = sum_b J_b^T [m (Jdot_b v - g); I_b (Jdot_b v)_ang + w_b x I_b w_b],
// Cholesky, v_s = v + h M^-1 (tau - c), body velocities at v_s and COM traces.
// Work block: M/L [nd*nd] | c [nd] | v_s [nd] | cols [6 nd] | idx [nd].
// yd (or null): each body's L^-1 J_b^T, the six columns (linear, angular)
// of body b0 + k at yd + (6 k + r) nd, for the exact diagonal impedance.
__device__ __attribute__((noinline)) void art_predict(const SubTree S, const BodyC *B, const float4 *bmi,
                                                      const float *sq, const float *sv,
                            const float *st, float4 *bC, float4 *bV, float4 *bW, float4 *bO, float4 *bAx,
                            float4 *bR, float *blk, const Params &P, float *yd) {
  const int nd = S.nd, d0 = S.d0;
  float *M = blk, *cv = M + nd * nd, *vs = cv + nd, *cols = vs + nd;
  int *idx = reinterpret_cast<int *>(cols + 6 * nd);
  fk_range<float>(S.b0, S.nb, B, sq, reinterpret_cast<float *>(bO), reinterpret_cast<float *>(bR),
                  reinterpret_cast<float *>(bAx), reinterpret_cast<float *>(bC));
  for (int i = 0; i < nd * nd; ++i) M[i] = 0.f;
  for (int i = 0; i < nd; ++i) cv[i] = 0.f;
  const float *v = sv + d0;
  const V3 g = v3(P.gx, P.gy, P.gz);
  for (int b = S.b0; b < S.b0 + S.nb; ++b) {
    const int n = chain_cols(b, d0, B, bO, bAx, bC, cols, idx);
    const float4 mi = bmi[b];
    float Ib[6];
    world_inertia(bR + 3 * b, mi, Ib);
    V3 vc = v3(0.f, 0.f, 0.f), om = vc;
    for (int x = 0; x < n; ++x) {
      const float *c = cols + 6 * x, vx = v[idx[x]];
      vc = vc + vx * v3(c[0], c[1], c[2]);
      om = om + vx * v3(c[3], c[4], c[5]);
    }
    const V3 cb = v3(bC[b].x, bC[b].y, bC[b].z), ob = v3(bO[b].x, bO[b].y, bO[b].z);
    const V3 vo = vc + cross(om, ob - cb);
    bW[b] = make_float4(om.x, om.y, om.z, 0.f);  // velocities at v (ancestors first)
    bV[b] = make_float4(vo.x, vo.y, vo.z, 0.f);
    // velocity-product accelerations Jdot_b v
    V3 jl = v3(0.f, 0.f, 0.f), ja = jl;
    for (int j = b; j >= 0; j = B[j].parent) {
      const int jt = B[j].jnt, da = B[j].dadr - d0;
      const V3 wj = v3(bW[j].x, bW[j].y, bW[j].z), voj = v3(bV[j].x, bV[j].y, bV[j].z);
      const V3 aj = v3(bAx[j].x, bAx[j].y, bAx[j].z), oj = v3(bO[j].x, bO[j].y, bO[j].z);
      if (jt == kFree) {
        jl = jl + cross(v3(v[da + 3], v[da + 4], v[da + 5]), vc - voj);
      } else {
        const V3 wa = cross(wj, aj);
        const float td = v[da];
        if (jt == kHinge) {
          jl = jl + td * (cross(wa, cb - oj) + cross(aj, vc - voj));
          ja = ja + td * wa;
        } else {
          jl = jl + td * wa;
        }
      }
    }
    const V3 Flin = mi.x * (jl - g);
    const V3 Fang = sym_mul(Ib, ja) + cross(om, sym_mul(Ib, om));
    for (int x = 0; x < n; ++x) {
      const float *c = cols + 6 * x;
      const V3 lx = v3(c[0], c[1], c[2]), ax_ = v3(c[3], c[4], c[5]);
      cv[idx[x]] += dot(lx, Flin) + dot(ax_, Fang);
      const V3 Ia = sym_mul(Ib, ax_);
      for (int y = 0; y < n; ++y) {
        if (idx[y] > idx[x]) continue;
        const float *e = cols + 6 * y;
        M[idx[x] * nd + idx[y]] += mi.x * (lx.x * e[0] + lx.y * e[1] + lx.z * e[2]) +
                                   Ia.x * e[3] + Ia.y * e[4] + Ia.z * e[5];
      }
    }
  }
  chol_lower(M, nd);
  for (int i = 0; i < nd; ++i) vs[i] = st[d0 + i] - cv[i];
  fwd_solve(M, nd, vs);
  bwd_solve(M, nd, vs);
  for (int i = 0; i < nd; ++i) vs[i] = v[i] + P.h * vs[i];
  // body velocities at v_s and traces ||L^-1 J_lin^T||_F^2 (cv is scratch from here on)
  for (int b = S.b0; b < S.b0 + S.nb; ++b) {
    const int n = chain_cols(b, d0, B, bO, bAx, bC, cols, idx);
    V3 vc = v3(0.f, 0.f, 0.f), om = vc;
    for (int x = 0; x < n; ++x) {
      const float *c = cols + 6 * x, vx = vs[idx[x]];
      vc = vc + vx * v3(c[0], c[1], c[2]);
      om = om + vx * v3(c[3], c[4], c[5]);
    }
    float tr = 0.f;
    float *yb = yd ? yd + 6 * nd * (b - S.b0) : nullptr;
    for (int r = 0; r < (yb ? 6 : 3); ++r) {
      float *y = yb ? yb + r * nd : cv;
      for (int i = 0; i < nd; ++i) y[i] = 0.f;
      for (int x = 0; x < n; ++x) y[idx[x]] = cols[6 * x + r];
      fwd_solve(M, nd, y);
      if (r < 3)
        for (int i = 0; i < nd; ++i) tr += y[i] * y[i];
    }
    bV[b] = make_float4(vc.x, vc.y, vc.z, tr);
    bW[b] = make_float4(om.x, om.y, om.z, 0.f);
    bC[b].w = 0.f;
  }
}

// ---- small subtrees: one quad of lanes per subtree, one lane per body
// A subtree of at most kSmallSub bodies, each with one hinge or slide dof
// (body k of the subtree owns dof k), is computed by the four lanes of a quad:
// lane k forms body k's frame (walking its own ancestor chain in registers),
// its Jacobian columns, velocities, velocity-product and gravity forces and
// its terms of M and of the bias; quad sums (DPP) give every lane the whole
// M and bias, each lane factors the 4 x 4 matrix itself and lane k finishes
// body k (velocities at v_s, COM trace).  The chain structure is held as
// ancestor bit masks (anc[k] bit j: body j is body k or one of its
// ancestors).  Same equations as art_predict / art_correct; the work block
// holds what the other passes read: the Cholesky factor L (nd x nd), M^-1 p
// after the correction (at nd^2) and v_s (at nd^2 + nd).
struct SmallChain {
  int n, anc[kSmallSub], jnt[kSmallSub], qadr[kSmallSub], dadr[kSmallSub];
  uint32_t chain;
  int q0, d0;
};

// Entry k of the chain's tables for a lane-dependent k, computed from the
// subtree record (no indexed access to the tables, which would put them on
// the stack).
__device__ inline int chain_anc(const SmallChain &C, int k) { return k < C.n ? (int)((C.chain >> (4 * k)) & 15) : 0; }
__device__ inline int chain_qadr(const SmallChain &C, int k) { return k < C.n ? C.q0 + k : 0; }
__device__ inline int chain_dadr(const SmallChain &C, int k) { return k < C.n ? C.d0 + k : 0; }

// x[k] for a lane-dependent k, as selects (no indexed register access).
template <class T>
__device__ inline T pick(const T (&x)[kSmallSub], int k) {
  T r = x[0];
#pragma unroll
  for (int j = 1; j < kSmallSub; ++j) r = j == k ? x[j] : r;
  return r;
}

__device__ inline SmallChain small_chain(const SubTree S) {
  SmallChain C;
  C.n = S.nb;
  C.chain = (uint32_t)S.chain;
  C.q0 = S.q0;
  C.d0 = S.d0;
#pragma unroll
  for (int k = 0; k < kSmallSub; ++k) {
    const bool in = k < C.n;
    C.anc[k] = in ? (S.chain >> (4 * k)) & 15 : 0;
    C.jnt[k] = ((S.chain >> (16 + k)) & 1) ? kHinge : kSlide;
    C.qadr[k] = in ? S.q0 + k : 0;
    C.dadr[k] = in ? S.d0 + k : 0;
  }
  return C;
}

// Sum over the four lanes of a quad (every lane gets the same value).
__device__ inline float quad_sum(float x) {
  x += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0xB1, 0xF, 0xF, false));  // [1,0,3,2]
  x += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x4E, 0xF, 0xF, false));  // [2,3,0,1]
  return x;
}

// Broadcast of lane J of each quad to the quad's four lanes.
template <int J>
__device__ inline int quad_bcast_i(int x) {
  return __builtin_amdgcn_update_dpp(0, x, J * 0x55, 0xF, 0xF, false);
}
template <int J>
__device__ inline double quad_bcast(double x) {
  return __hiloint2double(quad_bcast_i<J>(__double2hiint(x)), quad_bcast_i<J>(__double2loint(x)));
}
__device__ inline void sin_cos(double x, double *s, double *c) { sincos(x, s, c); }

// Lane k of the quad: frames along the chain of body k of a small subtree
// from the joint constants (JointK).  Each lane takes the sine and cosine of
// its own body's joint angle once and the quad shares them; walking the
// ancestors root first, R_j = R_p (Mk + cos Mc + sin Ms), o_j = o_p +
// R_p (lp + th s), world axis a_j = R_p Ba (p: the previous ancestor, the
// world frame for the root).  o[j], a[j]: zero where j is not an ancestor of
// k (nor k); R, ok: body k's rotation and origin (identity and zero for a
// lane beyond the subtree).
template <class T>
struct QuadChain {
  T o[kSmallSub][3], a[kSmallSub][3], R[9], ok[3];
};

template <class T>
__device__ inline void quad_chain(const SubTree S, const SmallChain &C, int k, const JointK<T> *JK,
                                  const float *sq, QuadChain<T> &Q) {
  constexpr int N = kSmallSub;
  const bool own = k < C.n;
  const T th = own ? (T)sq[chain_qadr(C, k)] : T(0);
  T sn, cs;
  sin_cos(th, &sn, &cs);
  const T tj[N] = {quad_bcast<0>(th), quad_bcast<1>(th), quad_bcast<2>(th), quad_bcast<3>(th)};
  const T sj[N] = {quad_bcast<0>(sn), quad_bcast<1>(sn), quad_bcast<2>(sn), quad_bcast<3>(sn)};
  const T cj[N] = {quad_bcast<0>(cs), quad_bcast<1>(cs), quad_bcast<2>(cs), quad_bcast<3>(cs)};
  const int anc = own ? chain_anc(C, k) : 0;
  T pR[9] = {T(1), T(0), T(0), T(0), T(1), T(0), T(0), T(0), T(1)}, po[3] = {T(0), T(0), T(0)};
#pragma unroll
  for (int j = 0; j < N; ++j) {
#pragma unroll
    for (int i = 0; i < 3; ++i) Q.o[j][i] = Q.a[j][i] = T(0);
    if (!((anc >> j) & 1)) continue;
    const JointK<T> &K = JK[S.b0 + j];
    T l[3], Rl[9], R[9];
#pragma unroll
    for (int i = 0; i < 3; ++i) l[i] = K.lp[i] + tj[j] * K.s[i];
#pragma unroll
    for (int i = 0; i < 9; ++i) Rl[i] = K.Mk[i] + cj[j] * K.Mc[i] + sj[j] * K.Ms[i];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      Q.o[j][i] = po[i] + pR[3 * i] * l[0] + pR[3 * i + 1] * l[1] + pR[3 * i + 2] * l[2];
      Q.a[j][i] = pR[3 * i] * K.Ba[0] + pR[3 * i + 1] * K.Ba[1] + pR[3 * i + 2] * K.Ba[2];
#pragma unroll
      for (int c = 0; c < 3; ++c) R[3 * i + c] = pR[3 * i] * Rl[c] + pR[3 * i + 1] * Rl[3 + c] + pR[3 * i + 2] * Rl[6 + c];
    }
#pragma unroll
    for (int i = 0; i < 9; ++i) pR[i] = R[i];
#pragma unroll
    for (int i = 0; i < 3; ++i) po[i] = Q.o[j][i];
  }
#pragma unroll
  for (int i = 0; i < 9; ++i) Q.R[i] = pR[i];
#pragma unroll
  for (int i = 0; i < 3; ++i) Q.ok[i] = po[i];
}

// Float64 forward kinematics of a small subtree for the narrow phase (the
// frames fk_range writes), lane k of the quad writing body k's; `fr` (the
// world's frame rows, or null) receives body k's origin, world joint axis
// and rotation rows in float32 for the resolution of the same step.
__device__ __attribute__((always_inline)) inline void fk_small(const SubTree S, int k, const JointK<double> *JK,
                                                               const float *sq, double *org, double *rot,
                                                               float4 *fr) {
  const SmallChain C = small_chain(S);
  QuadChain<double> Q;
  quad_chain<double>(S, C, k, JK, sq, Q);
  if (k < C.n) {
    const int b = S.b0 + k;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      org[4 * b + i] = Q.ok[i];
#pragma unroll
      for (int j = 0; j < 3; ++j) rot[12 * b + 4 * i + j] = Q.R[3 * i + j];
    }
    if (fr) {
      double ak[3] = {Q.a[0][0], Q.a[0][1], Q.a[0][2]};
#pragma unroll
      for (int j = 1; j < kSmallSub; ++j)
        if (j == k) {
          ak[0] = Q.a[j][0]; ak[1] = Q.a[j][1]; ak[2] = Q.a[j][2];
        }
      fr += 5 * b;
      fr[0] = make_float4((float)Q.ok[0], (float)Q.ok[1], (float)Q.ok[2], 0.f);
      fr[1] = make_float4((float)ak[0], (float)ak[1], (float)ak[2], 0.f);
#pragma unroll
      for (int i = 0; i < 3; ++i)
        fr[2 + i] = make_float4((float)Q.R[3 * i], (float)Q.R[3 * i + 1], (float)Q.R[3 * i + 2], 0.f);
    }
  }
}

// The frames of the subtree's bodies (bO, bAx, bR: origin, world joint axis,
// rotation) are in LDS already (the narrow phase's float64 kinematics of the
// same q, staged by resolve_world), and so are body k's inertia in bW[b] and
// COM offset in bC[b], which this call replaces with its velocity and COM.
__device__ void art_predict_small(const SubTree S, int k, const float *sv, const float *st, float4 *bC,
                                  float4 *bV, float4 *bW, const float4 *bO, const float4 *bAx, const float4 *bR,
                                  float *blk, const Params &P, float *yd) {
  constexpr int N = kSmallSub;
  const SmallChain C = small_chain(S);
  const int n = C.n;
  const bool own = k < n;
  const int b = S.b0 + k;
  const int anck = own ? chain_anc(C, k) : 0;
  const float4 mi = own ? bW[b] : make_float4(0.f, 1.f, 1.f, 1.f);
  const float4 ip = own ? bC[b] : make_float4(0.f, 0.f, 0.f, 0.f);
  struct {
    V3 o[N], a[N], c;
    float R[9];
  } Fr;
#pragma unroll
  for (int j = 0; j < N; ++j) {
    Fr.o[j] = Fr.a[j] = v3(0.f, 0.f, 0.f);
    if ((anck >> j) & 1) {
      const float4 o = bO[S.b0 + j], x = bAx[S.b0 + j];
      Fr.o[j] = v3(o.x, o.y, o.z);
      Fr.a[j] = v3(x.x, x.y, x.z);
    }
  }
  V3 ok = v3(0.f, 0.f, 0.f);
  const float4 r0 = own ? bR[3 * b] : make_float4(1.f, 0.f, 0.f, 0.f);
  const float4 r1 = own ? bR[3 * b + 1] : make_float4(0.f, 1.f, 0.f, 0.f);
  const float4 r2 = own ? bR[3 * b + 2] : make_float4(0.f, 0.f, 1.f, 0.f);
  Fr.R[0] = r0.x; Fr.R[1] = r0.y; Fr.R[2] = r0.z;
  Fr.R[3] = r1.x; Fr.R[4] = r1.y; Fr.R[5] = r1.z;
  Fr.R[6] = r2.x; Fr.R[7] = r2.y; Fr.R[8] = r2.z;
  if (own) {
    const float4 o = bO[b];
    ok = v3(o.x, o.y, o.z);
  }
  Fr.c = v3(ok.x + Fr.R[0] * ip.x + Fr.R[1] * ip.y + Fr.R[2] * ip.z,
            ok.y + Fr.R[3] * ip.x + Fr.R[4] * ip.y + Fr.R[5] * ip.z,
            ok.z + Fr.R[6] * ip.x + Fr.R[7] * ip.y + Fr.R[8] * ip.z);
  // body k's Jacobian columns: lin[j] = a_j x (c_k - o_j) (hinge) or a_j
  // (slide) where dof j moves body k, ang[j] = a_j (hinge); else 0
  float mk[N], v[N];
  V3 lin[N], ang[N];
#pragma unroll
  for (int j = 0; j < N; ++j) {
    mk[j] = ((anck >> j) & 1) ? 1.f : 0.f;
    const float hj = C.jnt[j] == kHinge ? 1.f : 0.f;
    lin[j] = mk[j] * (hj * cross(Fr.a[j], Fr.c - Fr.o[j]) + (1.f - hj) * Fr.a[j]);
    ang[j] = (mk[j] * hj) * Fr.a[j];
    v[j] = j < n ? sv[C.dadr[j]] : 0.f;
  }
  // velocities at v of body k (the quad shares them through LDS)
  V3 vc = v3(0.f, 0.f, 0.f), om = vc;
#pragma unroll
  for (int j = 0; j < N; ++j) {
    vc = vc + v[j] * lin[j];
    om = om + v[j] * ang[j];
  }
  const V3 vo = vc + cross(om, ok - Fr.c);
  if (own) {
    bV[b] = make_float4(vo.x, vo.y, vo.z, 0.f);
    bW[b] = make_float4(om.x, om.y, om.z, 0.f);
  }
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
  // velocity-product accelerations Jdot_k v over the chain
  V3 jl = v3(0.f, 0.f, 0.f), ja = jl;
#pragma unroll
  for (int j = 0; j < N; ++j) {
    if (mk[j] == 0.f) continue;
    const float4 Wj = bW[S.b0 + j], Vj = bV[S.b0 + j];
    const V3 wa = cross(v3(Wj.x, Wj.y, Wj.z), Fr.a[j]);
    if (C.jnt[j] == kHinge) {
      jl = jl + v[j] * (cross(wa, Fr.c - Fr.o[j]) + cross(Fr.a[j], vc - v3(Vj.x, Vj.y, Vj.z)));
      ja = ja + v[j] * wa;
    } else {
      jl = jl + v[j] * wa;
    }
  }
  float Ib[6];
  {
    const float d[3] = {mi.y, mi.z, mi.w};
    const int ri[6] = {0, 1, 2, 0, 0, 1}, rj[6] = {0, 1, 2, 1, 2, 2};
#pragma unroll
    for (int q = 0; q < 6; ++q) {
      const float *u = Fr.R + 3 * ri[q], *w = Fr.R + 3 * rj[q];
      Ib[q] = u[0] * d[0] * w[0] + u[1] * d[1] * w[1] + u[2] * d[2] * w[2];
    }
  }
  const V3 g = v3(P.gx, P.gy, P.gz);
  const V3 Flin = mi.x * (jl - g);
  const V3 Fang = sym_mul(Ib, ja) + cross(om, sym_mul(Ib, om));
  // body k's terms of the bias and of M (lower triangle), summed over the quad
  float cv[N], M[N][N];
#pragma unroll
  for (int i = 0; i < N; ++i) {
    cv[i] = quad_sum(dot(lin[i], Flin) + dot(ang[i], Fang));
    const V3 Ia = sym_mul(Ib, ang[i]);
#pragma unroll
    for (int j = 0; j < N; ++j) M[i][j] = j <= i ? quad_sum(mi.x * dot(lin[i], lin[j]) + dot(Ia, ang[j])) : 0.f;
  }
  // Cholesky factor (lower, reciprocal diagonal kept) and v_s = v + h M^-1 (tau - c),
  // the same in every lane of the quad
  float dinv[N];
#pragma unroll
  for (int j = 0; j < N; ++j) {
    dinv[j] = 0.f;
    if (j >= n) continue;
    float sj = M[j][j];
#pragma unroll
    for (int q = 0; q < j; ++q) sj -= M[j][q] * M[j][q];
    const float l = sqrtf(fmaxf(sj, 1e-30f));
    M[j][j] = l;
    dinv[j] = 1.0f / l;
#pragma unroll
    for (int i = j + 1; i < N; ++i) {
      if (i >= n) continue;
      float t = M[i][j];
#pragma unroll
      for (int q = 0; q < j; ++q) t -= M[i][q] * M[j][q];
      M[i][j] = t * dinv[j];
    }
  }
  auto solve_fwd = [&](float *x) {
#pragma unroll
    for (int i = 0; i < N; ++i) {
      float t = x[i];
#pragma unroll
      for (int q = 0; q < i; ++q) t -= M[i][q] * x[q];
      x[i] = t * dinv[i];
    }
  };
  float vs[N];
#pragma unroll
  for (int i = 0; i < N; ++i) vs[i] = i < n ? st[C.dadr[i]] - cv[i] : 0.f;
  solve_fwd(vs);
#pragma unroll
  for (int i = N - 1; i >= 0; --i) {
    float t = vs[i];
#pragma unroll
    for (int q = i + 1; q < N; ++q) t -= M[q][i] * vs[q];
    vs[i] = t * dinv[i];
  }
#pragma unroll
  for (int i = 0; i < N; ++i) vs[i] = v[i] + P.h * vs[i];
  // body k at v_s: velocities and COM trace ||L^-1 J_lin^T||_F^2
  V3 vk = v3(0.f, 0.f, 0.f), wk = vk;
  float e0[N], e1[N], e2[N];
#pragma unroll
  for (int j = 0; j < N; ++j) {
    vk = vk + vs[j] * lin[j];
    wk = wk + vs[j] * ang[j];
    e0[j] = lin[j].x; e1[j] = lin[j].y; e2[j] = lin[j].z;
  }
  solve_fwd(e0);
  solve_fwd(e1);
  solve_fwd(e2);
  float tr = 0.f;
#pragma unroll
  for (int j = 0; j < N; ++j) tr += e0[j] * e0[j] + e1[j] * e1[j] + e2[j] * e2[j];
  if (yd && own) {  // body k's L^-1 J_k^T (art_predict's layout) for the exact diagonal impedance
    float e3[N], e4[N], e5[N];
#pragma unroll
    for (int j = 0; j < N; ++j) {
      e3[j] = ang[j].x; e4[j] = ang[j].y; e5[j] = ang[j].z;
    }
    solve_fwd(e3);
    solve_fwd(e4);
    solve_fwd(e5);
    float *yk = yd + 6 * n * k;
#pragma unroll
    for (int j = 0; j < N; ++j) {
      if (j >= n) continue;
      yk[j] = e0[j]; yk[n + j] = e1[j]; yk[2 * n + j] = e2[j];
      yk[3 * n + j] = e3[j]; yk[4 * n + j] = e4[j]; yk[5 * n + j] = e5[j];
    }
  }
  // the Jdot reads of the quad precede these writes (one wave, program order)
  if (own) {
    bC[b] = make_float4(Fr.c.x, Fr.c.y, Fr.c.z, 0.f);
    bV[b] = make_float4(vk.x, vk.y, vk.z, tr);
    bW[b] = make_float4(wk.x, wk.y, wk.z, 0.f);
  }
  if (k == 0) {  // work block: L row-major (nd x nd), v_s at nd^2 + nd
    float *Lb = blk, *vsb = blk + n * n + n;
#pragma unroll
    for (int i = 0; i < N; ++i) {
      if (i >= n) continue;
      vsb[i] = vs[i];
#pragma unroll
      for (int j = 0; j < N; ++j)
        if (j < n) Lb[i * n + j] = j <= i ? M[i][j] : 0.f;
    }
  }
}

// Velocity correction and integration of a small subtree (art_correct), lane
// k of the quad: body k's terms of p = sum_k J_k^T (F_k, T_k), quad sums,
// v+ = v_s + M^-1 p in every lane, then lane k updates dof k; the work block
// keeps M^-1 p after L (as art_correct leaves it).
__device__ void art_correct_small(const SubTree S, int k, const BodyC *B, const float4 *bC, const float4 *bO,
                                  const float4 *bAx, const float4 *accF, const float4 *accT, float *sq, float *sv,
                                  float *blk, const Params &P) {
  constexpr int N = kSmallSub;
  const SmallChain C = small_chain(S);
  const int n = C.n;
  const bool own = k < n;
  const int b = S.b0 + k;
  const int anck = own ? chain_anc(C, k) : 0;
  V3 cb = v3(0.f, 0.f, 0.f), F = cb, T = cb;
  if (own) {
    cb = v3(bC[b].x, bC[b].y, bC[b].z);
    F = v3(accF[b].x, accF[b].y, accF[b].z);
    T = v3(accT[b].x, accT[b].y, accT[b].z);
  }
  float p[N], L[N][N], dinv[N];
#pragma unroll
  for (int j = 0; j < N; ++j) {
    const float mk = ((anck >> j) & 1) ? 1.f : 0.f;
    float t = 0.f;
    if (j < n) {
      const V3 oj = v3(bO[S.b0 + j].x, bO[S.b0 + j].y, bO[S.b0 + j].z);
      const V3 aj = v3(bAx[S.b0 + j].x, bAx[S.b0 + j].y, bAx[S.b0 + j].z);
      const bool hinge = C.jnt[j] == kHinge;
      const V3 lin = hinge ? cross(aj, cb - oj) : aj;
      t = mk * (dot(lin, F) + (hinge ? dot(aj, T) : 0.f));
    }
    p[j] = quad_sum(t);
  }
#pragma unroll
  for (int i = 0; i < N; ++i) {
#pragma unroll
    for (int j = 0; j < N; ++j) L[i][j] = (i < n && j <= i) ? blk[i * n + j] : 0.f;
    dinv[i] = i < n ? 1.0f / L[i][i] : 0.f;
  }
#pragma unroll
  for (int i = 0; i < N; ++i) {
    float t = p[i];
#pragma unroll
    for (int q = 0; q < i; ++q) t -= L[i][q] * p[q];
    p[i] = t * dinv[i];
  }
#pragma unroll
  for (int i = N - 1; i >= 0; --i) {
    float t = p[i];
#pragma unroll
    for (int q = i + 1; q < N; ++q) t -= L[q][i] * p[q];
    p[i] = t * dinv[i];
  }
  if (own) {
    const float pk = pick(p, k);
    blk[n * n + k] = pk;  // z = M^-1 p, read by the adjoint
    const float vp = blk[n * n + n + k] + pk;
    sv[chain_dadr(C, k)] = vp;
    sq[chain_qadr(C, k)] += P.h * vp;
  }
}

// Unit quaternion exp(th/2) = (cos x, sin(x) th/|th|), x = |th|/2, of a rotation
// vector: below x = 1/4 from the Taylor series of cos x and of sin(x)/x (the
// first omitted terms are below 1e-13 relative, so the float32 result is that
// of the exact functions), else from sinf, cosf.
__device__ inline void quat_of_rotvec(V3 th, float &ew, float &ex, float &ey, float &ez) {
  const float ang = sqrtf(dot(th, th)), x = 0.5f * ang;
  float s;  // sin(x) / ang
  if (x < 0.25f) {
    const float x2 = x * x;
    s = 0.5f * (1.f - x2 * (1.f / 6.f - x2 * (1.f / 120.f - x2 * (1.f / 5040.f - x2 * (1.f / 362880.f)))));
    ew = 1.f - x2 * (0.5f - x2 * (1.f / 24.f - x2 * (1.f / 720.f - x2 * (1.f / 40320.f - x2 * (1.f / 3628800.f)))));
  } else {
    s = sinf(x) / ang;
    ew = cosf(x);
  }
  ex = s * th.x; ey = s * th.y; ez = s * th.z;
}

// Velocity correction and integration of one articulated subtree:
// p = sum_b J_b^T (F_b, T_b), v+ = v_s + M^-1 p, q+ = q (+) h v+.
__device__ __attribute__((noinline)) void art_correct(const SubTree S, const BodyC *B, const float4 *bC,
                                                      const float4 *bO,
                            const float4 *bAx, const float4 *accF, const float4 *accT, float *sq, float *sv,
                            float *blk, const Params &P) {
  const int nd = S.nd, d0 = S.d0;
  float *M = blk, *p = M + nd * nd, *vs = p + nd, *cols = vs + nd;
  int *idx = reinterpret_cast<int *>(cols + 6 * nd);
  for (int i = 0; i < nd; ++i) p[i] = 0.f;
  for (int b = S.b0; b < S.b0 + S.nb; ++b) {
    const int n = chain_cols(b, d0, B, bO, bAx, bC, cols, idx);
    const V3 F = v3(accF[b].x, accF[b].y, accF[b].z), T = v3(accT[b].x, accT[b].y, accT[b].z);
    for (int x = 0; x < n; ++x) {
      const float *c = cols + 6 * x;
      p[idx[x]] += c[0] * F.x + c[1] * F.y + c[2] * F.z + c[3] * T.x + c[4] * T.y + c[5] * T.z;
    }
  }
  fwd_solve(M, nd, p);
  bwd_solve(M, nd, p);
  for (int i = 0; i < nd; ++i) sv[d0 + i] = vs[i] + p[i];
  for (int b = S.b0; b < S.b0 + S.nb; ++b) {
    const BodyC c = B[b];
    float *qb = sq + c.qadr;
    const float *vb = sv + c.dadr;
    if (c.jnt != kFree) {
      qb[0] += P.h * vb[0];
      continue;
    }
    for (int k = 0; k < 3; ++k) qb[k] += P.h * vb[k];
    const V3 th = P.h * v3(vb[3], vb[4], vb[5]);
    float ew, ex, ey, ez;
    quat_of_rotvec(th, ew, ex, ey, ez);
    const float qw0 = qb[3], qx0 = qb[4], qy0 = qb[5], qz0 = qb[6];
    const float nw_ = ew * qw0 - ex * qx0 - ey * qy0 - ez * qz0;
    const float nx_ = ew * qx0 + ex * qw0 + ey * qz0 - ez * qy0;
    const float ny_ = ew * qy0 - ex * qz0 + ey * qw0 + ez * qx0;
    const float nz_ = ew * qz0 + ex * qy0 - ey * qx0 + ez * qw0;
    const float inv = rsqrtf(nw_ * nw_ + nx_ * nx_ + ny_ * ny_ + nz_ * nz_);
    qb[3] = nw_ * inv; qb[4] = nx_ * inv; qb[5] = ny_ * inv; qb[6] = nz_ * inv;
  }
}

// ====================================================================
// collision
// ====================================================================
// LDS: q row; per geom a float4 (position, size0) and its oriented index;
// per oriented geom (planes, capsules, boxes, offset spheres) a float32 and a
// float64 pose record; the ordered candidate list.
template <class T>
struct Pose {
  T p[3];   // world position
  T r[9];   // world rotation, row-major
  T s[3];   // size
  T pad;
};


// float32 test: is the slot's gap below `thr` (margin plus the float32 band)?
__device__ inline bool slot_candidate(uint32_t s, const float4 *Gs, const int *go, const Pose<float> *Of,
                                      float thr) {
  const int ga = slot_ga(s), gb = slot_gb(s);
  const uint32_t t = slot_type(s);
  if (t == kSphereSphere) {
    const float4 A = Gs[ga], B = Gs[gb];
    const float dx = B.x - A.x, dy = B.y - A.y, dz = B.z - A.z;
    const float R = A.w + B.w + thr;
    return R > 0.f && dx * dx + dy * dy + dz * dz < R * R;
  }
  if (t == kBoxSphere || t == kBoxCapsule) {
    // sphere centre (or capsule end) against the box: squared distance outside
    const Pose<float> &X = Of[go[ga]];
    float cx, cy, cz, rad;
    if (t == kBoxSphere) {
      const float4 S = Gs[gb];
      cx = S.x; cy = S.y; cz = S.z; rad = S.w;
    } else {
      const Pose<float> &C = Of[go[gb]];
      const float hl = slot_sub(s) == 0 ? -C.s[1] : C.s[1];
      cx = C.p[0] + hl * C.r[2]; cy = C.p[1] + hl * C.r[5]; cz = C.p[2] + hl * C.r[8];
      rad = C.s[0];
    }
    const float dx = cx - X.p[0], dy = cy - X.p[1], dz = cz - X.p[2];
    float d2 = 0.f;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const float e = fabsf(X.r[k] * dx + X.r[3 + k] * dy + X.r[6 + k] * dz) - X.s[k];
      if (e > 0.f) d2 += e * e;
    }
    const float R = rad + thr;
    return R > 0.f && d2 < R * R;
  }
  const Pose<float> &P = Of[go[ga]];
  const float nx = P.r[2], ny = P.r[5], nz = P.r[8];
  float cx, cy, cz, rad = 0.f;
  if (t == kPlaneSphere) {
    const float4 B = Gs[gb];
    cx = B.x; cy = B.y; cz = B.z; rad = B.w;
  } else {
    const Pose<float> &B = Of[go[gb]];
    cx = B.p[0]; cy = B.p[1]; cz = B.p[2];
    const int sub = slot_sub(s);
    if (t == kPlaneCapsule) {
      const float hl = sub == 0 ? -B.s[1] : B.s[1];
      cx += hl * B.r[2]; cy += hl * B.r[5]; cz += hl * B.r[8];
      rad = B.s[0];
    } else {
      const float l0 = (sub & 1) ? B.s[0] : -B.s[0];
      const float l1 = (sub & 2) ? B.s[1] : -B.s[1];
      const float l2 = (sub & 4) ? B.s[2] : -B.s[2];
      cx += B.r[0] * l0 + B.r[1] * l1 + B.r[2] * l2;
      cy += B.r[3] * l0 + B.r[4] * l1 + B.r[5] * l2;
      cz += B.r[6] * l0 + B.r[7] * l1 + B.r[8] * l2;
    }
  }
  const float phi = nx * (cx - P.p[0]) + ny * (cy - P.p[1]) + nz * (cz - P.p[2]) - rad;
  return phi < thr;
}

// float64 centre and radius of a sphere geom.
__device__ inline void sphere_of(int g, const float4 *Gs, const int *go, const Pose<double> *Od, double c[3],
                                 double &r) {
  const int o = go[g];
  if (o < 0) {
    const float4 G = Gs[g];
    c[0] = G.x; c[1] = G.y; c[2] = G.z; r = G.w;
  } else {
    c[0] = Od[o].p[0]; c[1] = Od[o].p[1]; c[2] = Od[o].p[2]; r = Od[o].s[0];
  }
}

// float64 gap, normal (a -> b) and point of one candidate slot.
__device__ inline double slot_eval(uint32_t s, const float4 *Gs, const int *go, const Pose<double> *Od,
                                   double n[3], double p[3]) {
  const int ga = slot_ga(s), gb = slot_gb(s);
  const uint32_t t = slot_type(s);
  const int sub = slot_sub(s);
  if (t == kSphereSphere) {
    double ca[3], cb[3], ra, rb;
    sphere_of(ga, Gs, go, Od, ca, ra);
    sphere_of(gb, Gs, go, Od, cb, rb);
    const double d[3] = {cb[0] - ca[0], cb[1] - ca[1], cb[2] - ca[2]};
    const double dist = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    if (dist >= 1e-12) {
      n[0] = d[0] / dist; n[1] = d[1] / dist; n[2] = d[2] / dist;
    } else {
      n[0] = 0.0; n[1] = 0.0; n[2] = 1.0;
    }
    const double phi = dist - ra - rb;
    const double k = ra + 0.5 * phi;
    for (int i = 0; i < 3; ++i) p[i] = ca[i] + k * n[i];
    return phi;
  }
  if (t == kBoxSphere || t == kBoxCapsule) {
    // sphere centre c (or capsule end) against the box X: c in the box frame,
    // clamped to the box; outside, n from the clamped point to c; inside, the
    // outward axis of the face of least depth (lowest axis on ties)
    const Pose<double> &X = Od[go[ga]];
    double c[3], rad;
    if (t == kBoxSphere) {
      sphere_of(gb, Gs, go, Od, c, rad);
    } else {
      const Pose<double> &C = Od[go[gb]];
      const double hl = sub == 0 ? -C.s[1] : C.s[1];
      for (int i = 0; i < 3; ++i) c[i] = C.p[i] + hl * C.r[3 * i + 2];
      rad = C.s[0];
    }
    const double d[3] = {c[0] - X.p[0], c[1] - X.p[1], c[2] - X.p[2]};
    double l[3], e[3], d2 = 0.0;
    for (int k = 0; k < 3; ++k) {
      l[k] = X.r[k] * d[0] + X.r[3 + k] * d[1] + X.r[6 + k] * d[2];
      e[k] = l[k] - fmin(fmax(l[k], -X.s[k]), X.s[k]);
      d2 += e[k] * e[k];
    }
    const double dist = sqrt(d2);
    double nl[3] = {0.0, 0.0, 0.0}, phi;
    if (dist > 1e-12) {
      for (int k = 0; k < 3; ++k) nl[k] = e[k] / dist;
      phi = dist - rad;
    } else {
      int kmin = 0;
      double dmin = X.s[0] - fabs(l[0]);
      for (int k = 1; k < 3; ++k) {
        const double dk = X.s[k] - fabs(l[k]);
        if (dk < dmin) { dmin = dk; kmin = k; }
      }
      nl[kmin] = l[kmin] >= 0.0 ? 1.0 : -1.0;
      phi = -dmin - rad;
    }
    const double k = rad + 0.5 * phi;
    for (int i = 0; i < 3; ++i) {
      n[i] = X.r[3 * i] * nl[0] + X.r[3 * i + 1] * nl[1] + X.r[3 * i + 2] * nl[2];
      p[i] = c[i] - k * n[i];
    }
    return phi;
  }
  const Pose<double> &P = Od[go[ga]];
  n[0] = P.r[2]; n[1] = P.r[5]; n[2] = P.r[8];  // plane normal: local z
  double c[3], rad = 0.0;
  if (t == kPlaneSphere) {
    sphere_of(gb, Gs, go, Od, c, rad);
  } else {
    const Pose<double> &B = Od[go[gb]];
    c[0] = B.p[0]; c[1] = B.p[1]; c[2] = B.p[2];
    if (t == kPlaneCapsule) {
      const double hl = sub == 0 ? -B.s[1] : B.s[1];
      for (int i = 0; i < 3; ++i) c[i] += hl * B.r[3 * i + 2];
      rad = B.s[0];
    } else {
      const double l0 = (sub & 1) ? B.s[0] : -B.s[0];
      const double l1 = (sub & 2) ? B.s[1] : -B.s[1];
      const double l2 = (sub & 4) ? B.s[2] : -B.s[2];
      for (int i = 0; i < 3; ++i) c[i] += B.r[3 * i] * l0 + B.r[3 * i + 1] * l1 + B.r[3 * i + 2] * l2;
    }
  }
  const double phi = n[0] * (c[0] - P.p[0]) + n[1] * (c[1] - P.p[1]) + n[2] * (c[2] - P.p[2]) - rad;
  const double k = rad + 0.5 * phi;
  for (int i = 0; i < 3; ++i) p[i] = c[i] - k * n[i];
  return phi;
}

// LDS scratch of the narrow phase of one world (after its q row); the sphere
// block's hit masks (nsph rows of ceil(nsph / 64) words) come last.
size_t collide_region_bytes(int nb, int ng, int norient, int nsub, int nsph) {
  return sizeof(float4) * (size_t)ng + 2 * sizeof(int) * (size_t)pad4(ng) +
         (sizeof(Pose<float>) + sizeof(Pose<double>)) * (size_t)norient + sizeof(uint32_t) * kCandCap +
         (nsub > 0 ? sizeof(double) * 16 * (size_t)nb : 0) +
         sizeof(unsigned long long) * (size_t)nsph * (size_t)((nsph + 63) / 64);
}

// Per-geom inputs of the narrow phase (loaded ahead of the q row's barrier).
struct GeomIn {
  int b, o;          // body (-1 static), index among oriented geoms (-1: plain sphere)
  float4 gp, gd, gq; // offset in the body frame, (size, mu_t), orientation in the body frame
};

__device__ inline GeomIn geom_in(const CollideArgs &a, int w, int g) {
  GeomIn x;
  x.b = a.gbody[g];
  x.o = a.gorient[g];
  x.gp = a.gpos[(size_t)w * a.gpos_ws + g];
  x.gd = a.gdat[(size_t)w * a.ng + g];
  x.gq = a.gquat[(size_t)w * a.gquat_ws + g];
  return x;
}

// Hit masks of a sphere block of S <= 64 NWD spheres (rows of NWD words in rm,
// zero on entry).  The lane of sphere i tests its partners j = i + d mod S,
// d = 1 ... S/2 (d = S/2 once per pair), branch-free, collecting the hit bits in
// NWD registers; the bits above i are ORed into row i and each bit j below i (a
// pair reached by wrapping round) into row j at bit i (integer OR: the order of
// the atomics does not matter).  A pair is a hit when |c_j - c_i|^2 <
// (r_i + r_j + margin)^2 in float32, the same value from either end.
// Contact test of a sphere pair from its LDS records (centre, radius):
// |c_j - c_i|^2 < (r_i + r_j + margin)^2 in float32 with a fixed operation
// order, so every path that decides a pair gets the same answer from either end.
__device__ inline bool sphere_pair_hit(float4 Gi, float4 Gj, float margin) {
  const float dx = Gj.x - Gi.x, dy = Gj.y - Gi.y, dz = Gj.z - Gi.z;
  const float R = (Gi.w + Gj.w) + margin;
  return (R > 0.f) & (fmaf(dz, dz, fmaf(dy, dy, dx * dx)) < R * R);
}

// Contact record of a sphere pair (a's centre and radius in A, b's in B):
// n = (c_b - c_a)/|c_b - c_a| (+z for coincident centres), phi = |c_b - c_a| -
// r_a - r_b, point c_a + (r_a + phi/2) n, the slot word in the last lane.  The
// distance and the normal come from one hardware reciprocal square root.
__device__ inline void sphere_pair_record(float4 A, float4 B, uint32_t sl, float4 &cn, float4 &cp) {
  const V3 d = v3(B.x - A.x, B.y - A.y, B.z - A.z);
  const float d2 = dot(d, d);
  const bool apart = d2 >= 1e-24f;
  const float inv = apart ? __builtin_amdgcn_rsqf(d2) : 0.f;
  const V3 n = apart ? inv * d : v3(0.f, 0.f, 1.f);
  const float phi = d2 * inv - A.w - B.w;
  const float k = A.w + 0.5f * phi;
  cn = make_float4(n.x, n.y, n.z, phi);
  cp = make_float4(A.x + k * n.x, A.y + k * n.y, A.z + k * n.z, __uint_as_float(sl));
}

template <int BS, int NWD>
__device__ inline void sphere_masks(const float4 *Gs, const int *gbd, int g0, int S, float margin,
                                    unsigned long long *rm) {
  const int half = S >> 1;
  for (int r0 = 0; r0 < S; r0 += BS) {
    const int i = r0 + (int)threadIdx.x;
    if (i >= S) continue;
    const float4 Gi = Gs[g0 + i];
    const int bi = gbd[g0 + i];
    const int dmax = (S & 1) ? half : (i < half ? half : half - 1);
    unsigned long long h[NWD];
#pragma unroll
    for (int w = 0; w < NWD; ++w) h[w] = 0ull;
    int j = i;
    for (int d = 1; d <= dmax; ++d) {
      j = j + 1 == S ? 0 : j + 1;
      const float4 Gj = Gs[g0 + j];
      const bool hit = (bi != gbd[g0 + j]) & sphere_pair_hit(Gi, Gj, margin);
      const unsigned long long bit = (unsigned long long)hit << (j & 63);
      if constexpr (NWD == 1) {
        h[0] |= bit;
      } else {
        h[0] |= j < 64 ? bit : 0ull;
        h[1] |= j < 64 ? 0ull : bit;
      }
    }
#pragma unroll
    for (int w = 0; w < NWD; ++w) {
      const int lo = i + 1 - 64 * w;  // first bit of word w above i
      const unsigned long long above = lo <= 0 ? ~0ull : lo >= 64 ? 0ull : ~0ull << lo;
      const unsigned long long own = h[w] & above;
      if (own) atomicOr(rm + i * NWD + w, own);
      for (unsigned long long b = h[w] & ~above; b; b &= b - 1ull)
        atomicOr(rm + (64 * w + __ffsll(b) - 1) * NWD + (i >> 6), 1ull << (i & 63));
    }
  }
}

// Hit masks of a sphere block of S <= 64 spheres on pairwise different
// bodies (at most one static) with margin >= 0, from a Gram matrix on bf16
// MFMA, one wave.  With centres c taken relative to the block's mean and
// rho = r + margin / 2, the test quantity g_ij = |c_i - c_j|^2 - (rho_i +
// rho_j)^2 is the product a_i . b_j of the 6-vectors a = (x, y, z, rho, s, 1)
// and b = (-2x, -2y, -2z, -2rho, 1, s), s = |c|^2 - rho^2.  Each float32
// component is split into bf16 parts, a = ah + al (+ a rest below 2^-18 |a|),
// and a . b is taken as ah . bh + ah . bl + al . bh: 18 exact bf16 products
// summed in float32, one v_mfma_f32_16x16x32_bf16 per 16 x 16 tile (K groups
// of eight: 0 ah.bh, 1 ah.bl, 2 al.bh, 3 zero), ten tiles for the upper
// triangle of 64 spheres.  Every product is at most M = max(|c|^2 + rho^2)
// in magnitude (their sum at most 4 M), so the dropped parts and the float32
// sums put g within 6e-5 M of the float32 test of sphere_pair_hit: outside
// the band |g| <= eps = M 2^-13 the sign of g is that test's answer, and the
// pairs inside it are decided by sphere_pair_hit itself.  The masks are
// therefore the ones sphere_masks builds.  The tiles are formed transposed,
// so lane l holds row i = 16 I + l % 16 at columns 16 J + 4 (l / 16) + r and
// sets its own bits; the four lanes of a row OR their parts at the end.
// `ab`: 4 x 64 x 16 bytes of LDS scratch.
__device__ __attribute__((always_inline)) inline void sphere_masks_mfma(const float4 *Gs, int g0, int S,
                                                                        float margin, unsigned long long *rm,
                                                                        void *ab) {
  typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
  typedef float f32x4 __attribute__((ext_vector_type(4)));
  const int l = threadIdx.x;  // the workgroup is one wave
  const bool real = l < S;
  const float4 G = real ? Gs[g0 + l] : make_float4(0.f, 0.f, 0.f, 0.f);
  const float invS = 1.0f / (float)S;
  const float cx = wave_last(wave_incl_sum(real ? G.x : 0.f)) * invS,
              cy = wave_last(wave_incl_sum(real ? G.y : 0.f)) * invS,
              cz = wave_last(wave_incl_sum(real ? G.z : 0.f)) * invS;
  const float x = G.x - cx, y = G.y - cy, z = G.z - cz;
  const float rho = G.w + 0.5f * margin;
  const float c2 = fmaf(z, z, fmaf(y, y, x * x)), r2 = rho * rho;
  const float M = wave_last(wave_incl_max(real ? c2 + r2 : 0.f));
  const float eps = M * (1.0f / 8192.0f);
  // padding rows and columns sit at g >= 4 M + 1 > eps from everything
  const float sa = real ? c2 - r2 : 4.0f * M + 1.0f;
  const float av[6] = {real ? x : 0.f, real ? y : 0.f, real ? z : 0.f, real ? rho : 0.f, sa, 1.f};
  const float bv[6] = {-2.f * av[0], -2.f * av[1], -2.f * av[2], -2.f * av[3], 1.f, sa};
  bf16x8 ah, al, bh, bl;
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const float a = k < 6 ? av[k] : 0.f, b = k < 6 ? bv[k] : 0.f;
    ah[k] = (__bf16)a;
    al[k] = (__bf16)(a - (float)ah[k]);
    bh[k] = (__bf16)b;
    bl[k] = (__bf16)(b - (float)bh[k]);
  }
  bf16x8 *tab = reinterpret_cast<bf16x8 *>(ab);  // [AH | AL | BH | BL][64]
  tab[l] = ah;
  tab[64 + l] = al;
  tab[128 + l] = bh;
  tab[192 + l] = bl;
  __syncthreads();
  const int c = l & 15, kg = l >> 4;
  // K group of this lane: the row operand (a) is ah, ah, al, 0 and the column
  // operand (b) bh, bl, bh, 0 for groups 0..3
  const bf16x8 zero8 = {};
  const bf16x8 *arow = tab + (kg == 2 ? 64 : 0), *bcol = tab + (kg == 1 ? 192 : 128);
  const int nt = (S + 15) >> 4;
  // the lane's bits of row 16 I + c (columns 16 J + 4 kg + r), per row block I
  uint32_t part[4][4] = {};
  uint32_t bit[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) bit[r] = 1u << (4 * kg + r);
#pragma unroll
  for (int I = 0; I < 4; ++I) {
    if (I >= nt) break;
    const bf16x8 bop = kg < 3 ? arow[16 * I + c] : zero8;  // rows i of this block (the product's N side)
#pragma unroll
    for (int J = 0; J < 4; ++J) {
      if (J < I || J >= nt) continue;
      const bf16x8 aop = kg < 3 ? bcol[16 * J + c] : zero8;  // columns j (the product's M side)
      f32x4 g = {0.f, 0.f, 0.f, 0.f};
      g = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aop, bop, g, 0, 0, 0);
      // lane l: g[r] = g_ij, i = 16 I + c, j = 16 J + 4 kg + r; a diagonal
      // tile keeps the columns above the row
      bool amb = false;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const bool above = I < J || 4 * kg + r > c;
        part[I][J] |= (above && g[r] < -eps) ? bit[r] : 0u;
        amb |= above && fabsf(g[r]) <= eps;
      }
      if (__builtin_amdgcn_ballot_w64(amb)) {  // pairs in the band (rare): the float32 test itself
        if (amb) {
          const float4 Gi = Gs[g0 + 16 * I + c];
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const bool above = I < J || 4 * kg + r > c;
            if (above && fabsf(g[r]) <= eps && sphere_pair_hit(Gi, Gs[g0 + 16 * J + 4 * kg + r], margin))
              part[I][J] |= bit[r];
          }
        }
      }
    }
  }
  // the four lanes of a row (equal l % 16) OR their parts into its mask
  // (zero on entry; integer OR is order-free)
#pragma unroll
  for (int I = 0; I < 4; ++I) {
    if (I >= nt) break;
    const unsigned long long m = (unsigned long long)(part[I][0] | (part[I][1] << 16)) |
                                 ((unsigned long long)(part[I][2] | (part[I][3] << 16)) << 32);
    if (m && 16 * I + c < S) atomicOr(rm + 16 * I + c, m);
  }
  __syncthreads();
}

// Narrow phase of world w from its q row `sq` (LDS).  Writes the first `cap`
// contacts of the canonical order to outn/outp (global or LDS) and returns the
// number found.  `reg` is LDS scratch of collide_region_bytes(); `nxt` is the
// caller's prefetch of slots[threadIdx.x]; `pre`, when given, the caller's
// prefetch of geoms threadIdx.x and threadIdx.x + BS (each valid where below
// ng).  Ends with a workgroup barrier.
template <int BS, bool ART>
__device__ int collide_world(const CollideArgs &a, int w, const float *sq, float4 *reg, float4 *outn,
                             float4 *outp, int cap, uint32_t nxt, const GeomIn *pre = nullptr, int tid_in = -1) {
  constexpr int NW = BS / 64;
  const int tid = tid_in >= 0 ? tid_in : (int)threadIdx.x;
  Pose<double> *Od = reinterpret_cast<Pose<double> *>(reg);
  Pose<float> *Of = reinterpret_cast<Pose<float> *>(Od + a.norient);
  float4 *Gs = reinterpret_cast<float4 *>(Of + a.norient);
  int *go = reinterpret_cast<int *>(Gs + a.ng);
  int *gbd = go + pad4(a.ng);  // body of each geom (-1 static)
  uint32_t *cand = reinterpret_cast<uint32_t *>(gbd + pad4(a.ng));
  double *borg = reinterpret_cast<double *>(cand + kCandCap);  // [nb][4] articulated bodies
  double *brot = borg + 4 * a.nb;                              // [nb][12]
  __shared__ int wcnt[2 * NW];
  __shared__ float wmax[NW];

  // slot words of the next three chunks, in flight during the set-up below
  // (loaded by every lane, index clamped into the table; a word past the
  // slots before the sphere block is never used)
  const int npre = a.npl > 0 ? 0 : a.nslot_pre, spl = npre > 0 ? npre - 1 : 0;
  uint32_t nxt2 = a.slots[tid + BS < npre ? tid + BS : spl];
  uint32_t nxt3 = a.slots[tid + 2 * BS < npre ? tid + 2 * BS : spl];
  uint32_t nxt4 = a.slots[tid + 3 * BS < npre ? tid + 3 * BS : spl];
  // articulated models: the lane's subtree record and the body record of
  // geom tid, also in flight before the kinematics
  SubTree sub0{};
  int gfast0 = 1, gqadr0 = 0;
  if (ART) {
    sub0 = a.sub[tid < 4 * a.nsub ? tid >> 2 : a.nsub - 1];  // (a lane past the subtrees: unused)
    if (pre && tid < a.ng && pre->b >= 0) {
      const BodyC &bc = a.body[pre->b];
      gfast0 = bc.fast;
      gqadr0 = bc.qadr;
    }
  }

  if (ART) {  // forward kinematics of articulated subtrees, float64
    // (lanes 4 si .. 4 si + 3 take subtree si: a quad for a small one, its
    // first lane for any other)
    for (int t = tid; t < 4 * a.nsub; t += BS) {
      const SubTree S = t == tid ? sub0 : a.sub[t >> 2];
      if (S.small)
        fk_small(S, t & 3, a.jk, sq, borg, brot, a.frames ? a.frames + (size_t)w * a.nb * 5 : nullptr);
      else if ((t & 3) == 0)
        fk_range<double>(S.b0, S.nb, a.body, sq, borg, brot, nullptr, nullptr);
    }
    __syncthreads();
  }

  // geom world poses; oriented geoms also get float64 and float32 pose records
  // (geoms tid and tid + BS from the caller's prefetch when given)
  auto geom_pose = [&](int g, const GeomIn &gi, bool own /* body record prefetched */) {
    const int b = gi.b, o = gi.o;
    const float4 gp = gi.gp, gd = gi.gd, gq = gi.gq;
    go[g] = o;
    gbd[g] = b;
    if (o < 0) {  // sphere at the origin of a free body (or static)
      const float *qb = b >= 0 ? sq + (ART ? (own ? gqadr0 : a.body[b].qadr) : 7 * b) : nullptr;
      Gs[g] = b >= 0 ? make_float4(qb[0], qb[1], qb[2], gd.x) : make_float4(gp.x, gp.y, gp.z, gd.x);
      return;
    }
    double bp[3] = {0.0, 0.0, 0.0}, br[9] = {1.0, 0.0, 0.0, 0.0, 1.0, 0.0, 0.0, 0.0, 1.0}, gr[9];
    if (b >= 0) {
      int fast = 1, qadr = 7 * b;
      if (ART) {
        if (own) {
          fast = gfast0;
          qadr = gqadr0;
        } else {
          const BodyC &bc = a.body[b];
          fast = bc.fast;
          qadr = bc.qadr;
        }
      }
      if (fast) {
        const float *qb = sq + qadr;
        bp[0] = qb[0]; bp[1] = qb[1]; bp[2] = qb[2];
        quat_to_rot<double>(qb[3], qb[4], qb[5], qb[6], br);
      } else {
        for (int i = 0; i < 3; ++i) {
          bp[i] = borg[4 * b + i];
          for (int j = 0; j < 3; ++j) br[3 * i + j] = brot[12 * b + 4 * i + j];
        }
      }
    }
    quat_to_rot<double>(gq.x, gq.y, gq.z, gq.w, gr);
    Pose<double> pd;
    Pose<float> pf;
    const double off[3] = {gp.x, gp.y, gp.z};
    if (b < 0) {  // static: the body frame is the world frame
      for (int i = 0; i < 3; ++i) pd.p[i] = off[i];
      for (int k = 0; k < 9; ++k) pd.r[k] = gr[k];
    } else {
      for (int i = 0; i < 3; ++i) {
        pd.p[i] = bp[i] + br[3 * i] * off[0] + br[3 * i + 1] * off[1] + br[3 * i + 2] * off[2];
        for (int j = 0; j < 3; ++j)
          pd.r[3 * i + j] = br[3 * i] * gr[j] + br[3 * i + 1] * gr[3 + j] + br[3 * i + 2] * gr[6 + j];
      }
    }
    pd.s[0] = gd.x; pd.s[1] = gd.y; pd.s[2] = gd.z; pd.pad = 0.0;
    for (int i = 0; i < 3; ++i) { pf.p[i] = (float)pd.p[i]; pf.s[i] = (float)pd.s[i]; }
    for (int i = 0; i < 9; ++i) pf.r[i] = (float)pd.r[i];
    pf.pad = 0.f;
    Od[o] = pd;
    Of[o] = pf;
    Gs[g] = make_float4(pf.p[0], pf.p[1], pf.p[2], gd.x);
  };
  int g0 = tid;
  if (pre) {
    if (tid < a.ng) geom_pose(tid, pre[0], true);
    if (tid + BS < a.ng) geom_pose(tid + BS, pre[1], false);
    g0 = tid + 2 * BS;
  }
  for (int g = g0; g < a.ng; g += BS) geom_pose(g, geom_in(a, w, g), false);
  __syncthreads();

  // Pass-1 band: float32 gaps are accurate to a few ulp of the coordinates and
  // sizes involved; one band per world, from the largest of them.
  float band, pband;
  {
    float ext = 0.f;
    for (int g = tid; g < a.ng; g += BS) {
      const float4 G = Gs[g];
      ext = fmaxf(ext, fmaxf(fmaxf(fabsf(G.x), fabsf(G.y)), fmaxf(fabsf(G.z), G.w)));
    }
    for (int o = tid; o < a.norient; o += BS)
      ext = fmaxf(ext, fmaxf(fmaxf(Of[o].s[0], Of[o].s[1]), Of[o].s[2]));
    ext = block_max<BS>(ext, wmax);
    band = 1e-4f + 8e-6f * ext;
    // plane rows: a float32 gap within pband of the margin is decided in
    // float64 (float32 rounding of a gap is a few 1e-8 of the extent)
    pband = 1e-6f + 1e-6f * ext;
  }
  int running = 0, ncand = 0, par = 0;
  // Pass 2 over the candidate list: float64 decision, ordered store.
  auto flush = [&]() {
    __syncthreads();
    for (int cb = 0; cb < ncand; cb += BS) {
      const int i = cb + tid;
      bool hit = false;
      float4 cn = make_float4(0.f, 0.f, 0.f, 0.f), cp = cn;
      if (i < ncand) {
        const uint32_t sl = cand[i];
        const int ga = slot_ga(sl), gb = slot_gb(sl);
        if (slot_type(sl) == kSphereSphere && go[ga] < 0 && go[gb] < 0) {
          // two spheres centred on their bodies: the centres are exact float32
          // state values and the gap needs no rotation, float32 suffices
          sphere_pair_record(Gs[ga], Gs[gb], sl, cn, cp);
          hit = cn.w < a.margin;
        } else {
          double nd[3], pd[3];
          const double phi = slot_eval(sl, Gs, go, Od, nd, pd);
          hit = phi < (double)a.margin;
          cn = make_float4((float)nd[0], (float)nd[1], (float)nd[2], (float)phi);
          cp = make_float4((float)pd[0], (float)pd[1], (float)pd[2], __uint_as_float(sl));
        }
      }
      int tot;
      const int idx = running + block_scan<BS>(hit, &tot, wcnt, par);
      par ^= 1;
      if (hit && idx < cap) {
        outn[idx] = cn;
        outp[idx] = cp;
      }
      running += tot;
    }
    __syncthreads();
    ncand = 0;
  };

  // Plane rows: when the slots before the sphere block are exactly every
  // (static plane p, sphere i) pair, plane-major, each lane takes a sphere and
  // decides every plane's pair directly (without slot words, type dispatch
  // and candidate list): in float32, or, when the float32 gap lies within
  // pband of the margin, by the per-slot path's float64 decision and record;
  // hits are stored in slot order by a workgroup scan.
  if (a.npl > 0) {
    const int g0 = a.sph0, S = a.nsph;
    for (int pl = 0; pl < a.npl; ++pl) {
      const Pose<float> &Pf = Of[go[pl]];
      const float px = Pf.p[0], py = Pf.p[1], pz = Pf.p[2];
      const float nx = Pf.r[2], ny = Pf.r[5], nz = Pf.r[8];  // plane normal: local z
      for (int r0 = 0; r0 < S; r0 += BS) {
        const int i = r0 + tid;
        bool hit = false;
        float4 cn = make_float4(0.f, 0.f, 0.f, 0.f), cp = cn;
        if (i < S) {
          const float4 G = Gs[g0 + i];
          const uint32_t sl = slot_pack(pl, g0 + i, 0, kPlaneSphere);
          const float phi = fmaf(nx, G.x - px, fmaf(ny, G.y - py, nz * (G.z - pz))) - G.w;
          if (fabsf(phi - a.margin) > pband) {
            const float k = G.w + 0.5f * phi;
            hit = phi < a.margin;
            cn = make_float4(nx, ny, nz, phi);
            cp = make_float4(G.x - k * nx, G.y - k * ny, G.z - k * nz, __uint_as_float(sl));
          } else {  // near the margin: the float64 decision and record
            const Pose<double> &Pd = Od[go[pl]];
            const double dx = Pd.r[2], dy = Pd.r[5], dz = Pd.r[8];
            const double cx = G.x, cy = G.y, cz = G.z, rad = G.w;
            const double phd = dx * (cx - Pd.p[0]) + dy * (cy - Pd.p[1]) + dz * (cz - Pd.p[2]) - rad;
            const double k = rad + 0.5 * phd;
            hit = phd < (double)a.margin;
            cn = make_float4((float)dx, (float)dy, (float)dz, (float)phd);
            cp = make_float4((float)(cx - k * dx), (float)(cy - k * dy), (float)(cz - k * dz), __uint_as_float(sl));
          }
        }
        int tot;
        const int idx = running + block_scan<BS>(hit, &tot, wcnt, par);
        par ^= 1;
        if (hit && idx < cap) {
          outn[idx] = cn;
          outp[idx] = cp;
        }
        running += tot;
      }
    }
  }

  // Pass 1 over the slots before the sphere block: float32 test, ordered
  // candidate list; slot words are loaded four chunks ahead.
  for (int base = 0; base < npre; base += BS) {
    if (ncand + BS > kCandCap) flush();
    const int s = base + tid;
    const uint32_t sl = nxt;
    nxt = nxt2;
    nxt2 = nxt3;
    nxt3 = nxt4;
    nxt4 = a.slots[s + 4 * BS < npre ? s + 4 * BS : spl];
    const bool c = s < npre && slot_candidate(sl, Gs, go, Of, a.margin + band);
    int tot;
    const int idx = block_scan<BS>(c, &tot, wcnt, par);
    par ^= 1;
    if (c) cand[ncand + idx] = sl;
    ncand += tot;
  }
  if (ncand > 0) flush();
  else __syncthreads();

  // Sphere block: the last nsph geoms are spheres centred on free bodies (or
  // static), and every pair of them on different bodies is a slot, in row-major
  // order after all other slots.  The pairs are tested cyclically: the lane of
  // sphere i tests (i, i + d mod S) for d = 1 .. S/2 (d = S/2 once per pair), so
  // every lane makes about S/2 tests against LDS records of consecutive
  // spheres; a hit sets bit max(i, j) of row min(i, j) in an LDS mask (integer
  // OR, order-free).  Rows are then placed in canonical order by a prefix sum
  // of their popcounts, and the hits are evaluated densely (float32: the centres
  // are exact state values) and stored in order.  A pair is a contact when
  // |c_b - c_a|^2 < (r_a + r_b + margin)^2 (the same float32 value from either
  // end of the pair).
  if (a.nsph > 0) {
    __shared__ int wsum[NW];
    const int g0 = a.sph0, S = a.nsph, nwd = (S + 63) >> 6;
    unsigned long long *rm = reinterpret_cast<unsigned long long *>(
        a.nsub > 0 ? reinterpret_cast<char *>(brot + 12 * a.nb) : reinterpret_cast<char *>(borg));
    for (int x = tid; x < S * nwd; x += BS) rm[x] = 0ull;
    __syncthreads();
    if (BS == 64 && a.sph_mfma) {
      sphere_masks_mfma(Gs, g0, S, a.margin, rm, cand);
    } else if (S <= 64) {
      sphere_masks<BS, 1>(Gs, gbd, g0, S, a.margin, rm);
    } else if (S <= 128) {
      sphere_masks<BS, 2>(Gs, gbd, g0, S, a.margin, rm);
    } else {
    const int half = S >> 1;
    for (int r0 = 0; r0 < S; r0 += BS) {
      const int i = r0 + tid;
      if (i < S) {
        const float4 Gi = Gs[g0 + i];
        const int bi = gbd[g0 + i];
        const int dmax = (S & 1) ? half : (i < half ? half : half - 1);
        for (int d = 1; d <= dmax; ++d) {
          const int j = i + d < S ? i + d : i + d - S;
          const float4 Gj = Gs[g0 + j];
          const int bj = gbd[g0 + j];
          if (bi != bj && sphere_pair_hit(Gi, Gj, a.margin)) {
            const int lo = min(i, j), hi = max(i, j);
            atomicOr(rm + lo * nwd + (hi >> 6), 1ull << (hi & 63));
          }
        }
      }
    }
    }
    __syncthreads();
    for (int r0 = 0; r0 < S; r0 += BS) {
      const int i = r0 + tid;
      const bool row = i < S;
      unsigned long long m[4] = {0ull, 0ull, 0ull, 0ull};
      int cnt = 0;
#pragma unroll
      for (int cw = 0; cw < 4; ++cw) {
        if (cw >= nwd) break;
        m[cw] = row ? rm[i * nwd + cw] : 0ull;
        cnt += __popcll(m[cw]);
      }
      int tot;
      const int pre = block_scan_int<BS>(cnt, &tot, wsum);
      for (int lo = 0; lo < tot; lo += kCandCap) {
        int k = pre;
#pragma unroll
        for (int cw = 0; cw < 4; ++cw) {
          if (cw >= nwd) break;
          for (unsigned long long mw = m[cw]; mw; mw &= mw - 1, ++k) {
            if (k >= lo && k < lo + kCandCap) {
              const int j = cw * 64 + __ffsll((unsigned long long)mw) - 1;
              cand[k - lo] = slot_pack(g0 + i, g0 + j, 0, kSphereSphere);
            }
          }
        }
        __syncthreads();
        const int nwin = min(kCandCap, tot - lo);
        for (int cb = 0; cb < nwin; cb += BS) {
          const int idx = cb + tid;
          const int pos = running + lo + idx;
          if (idx < nwin && pos < cap) {
            const uint32_t sl = cand[idx];
            float4 cn, cp;
            sphere_pair_record(Gs[slot_ga(sl)], Gs[slot_gb(sl)], sl, cn, cp);
            outn[pos] = cn;
            outp[pos] = cp;
          }
        }
        __syncthreads();
      }
      running += tot;
    }
  }
  (void)NW;
  return running;
}

template <int BS, bool ART>
__global__ __launch_bounds__(BS) void collide_kernel(CollideArgs a) {
  extern __shared__ float4 lds[];
  const int w = blockIdx.x, tid = threadIdx.x;
  float *sq = reinterpret_cast<float *>(lds);
  constexpr int K = 512 / BS;
  // issue the independent global loads (slots, geoms tid and tid + BS, q row)
  // before the first wait, every lane all of them (indices clamped into the
  // arrays, which hold at least one entry; values past their ends unused)
  const uint32_t nxt = a.slots[tid < a.nslot_pre ? tid : (a.nslot_pre > 0 ? a.nslot_pre - 1 : 0)];
  const int gl = a.ng > 0 ? a.ng - 1 : 0;
  const GeomIn pre[2] = {geom_in(a, w, tid < a.ng ? tid : gl), geom_in(a, w, tid + BS < a.ng ? tid + BS : gl)};
  const float *qw = a.q + (size_t)w * a.nq;
  RowStage<BS, K> rq;
  rq.load(qw, a.nq);
  rq.store(sq, qw, a.nq);
  __syncthreads();
  const size_t cbase = (size_t)w * a.ncon_max;
  const int found = collide_world<BS, ART>(a, w, sq, lds + pad4(a.nq) / 4, a.cnp + cbase, a.cpos + cbase,
                                           a.ncon_max, nxt, pre);
  if (tid == 0) {
    const int kept = found < a.ncon_max ? found : a.ncon_max;
    a.ncon[w] = kept;
    a.overflow[w] = found - kept;
    if (a.ncon_out) a.ncon_out[w] = kept;
    if (a.overflow_out) a.overflow_out[w] = found - kept;
  }
}

size_t collide_lds_bytes(int nq, int nb, int ng, int norient, int nsub, int nsph) {
  return sizeof(float) * pad4(nq) + collide_region_bytes(nb, ng, norient, nsub, nsph);
}

template <bool ART>
static hipError_t launch_collide_a(const CollideArgs &a, int nworld, int block, size_t lds, hipStream_t s) {
  switch (block) {
    case 64: hipLaunchKernelGGL((collide_kernel<64, ART>), dim3(nworld), dim3(64), lds, s, a); break;
    case 128: hipLaunchKernelGGL((collide_kernel<128, ART>), dim3(nworld), dim3(128), lds, s, a); break;
    case 256: hipLaunchKernelGGL((collide_kernel<256, ART>), dim3(nworld), dim3(256), lds, s, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_collide(const CollideArgs &a, int nworld, int block, size_t lds, hipStream_t s) {
  return a.nsub > 0 ? launch_collide_a<true>(a, nworld, block, lds, s)
                    : launch_collide_a<false>(a, nworld, block, lds, s);
}

// ====================================================================
// resolution
// ====================================================================
// LDS: q, v, tau rows; per body 7 float4 (com|invm, vs|tr, ws, Iinv a, Iinv b,
// accumulated force, accumulated torque) and 8 ints (the fixed-point wrench
// sums of the current contact chunk as three packed 64-bit words, the
// exponents of its force and its torque part, stored component-major); per
// geom float4 friction + int body.
// LDS scratch of the resolution of one world (after its q, v and tau rows).
__host__ __device__ size_t resolve_region_bytes(int nb, int ng, int nsub, int art_floats) {
  return sizeof(float4) * 7 * (size_t)nb + sizeof(float4) * (size_t)ng + sizeof(int) * 8 * (size_t)pad4(nb) +
         sizeof(int) * (size_t)pad4(ng) +
         (nsub > 0 ? sizeof(float4) * 5 * (size_t)nb + sizeof(float) * (size_t)pad4(art_floats) : 0);
}

size_t resolve_lds_bytes(int nq, int nv, int nb, int ng, int nsub, int art_floats) {
  return sizeof(float) * (pad4(nq) + 2 * (size_t)pad4(nv)) + resolve_region_bytes(nb, ng, nsub, art_floats);
}

// Arrays of the resolution's LDS scratch (layout of resolve_region_bytes()).
struct ResolveRegion {
  float4 *bC;            // per body: COM position, 1/m
  float4 *bV, *bW;       // v_s | trace, w_s
  float4 *bI0, *bI1;     // inverse world inertia (xx yy zz xy | xz yz)
  float4 *accF, *accT;   // accumulated contact force and torque
  float4 *gM;            // per geom (mu_t, mu_tor, mu_rol)
  int *fx;               // fixed-point chunk sums: 3 packed 64-bit words (6 ints), 2 exponents (pad4(nb) each)
  int *gB;               // per geom body
  float4 *bO, *bAx, *bR; // articulated bodies: origin, joint axis, rotation rows
  float *art;            // articulated subtree work blocks
};

__device__ inline ResolveRegion resolve_region(float4 *reg, int nb, int ng) {
  ResolveRegion r;
  r.bC = reg;
  r.bV = r.bC + nb; r.bW = r.bV + nb; r.bI0 = r.bW + nb; r.bI1 = r.bI0 + nb;
  r.accF = r.bI1 + nb; r.accT = r.accF + nb;
  r.gM = r.accT + nb;
  r.fx = reinterpret_cast<int *>(r.gM + ng);
  r.gB = r.fx + 8 * pad4(nb);
  r.bO = reinterpret_cast<float4 *>(r.gB + pad4(ng));
  r.bAx = r.bO + nb; r.bR = r.bAx + nb;
  r.art = reinterpret_cast<float *>(r.bR + 3 * nb);
  return r;
}

// x^T S y for the symmetric inverse world inertia S stored as (xx yy zz xy | xz yz).
__device__ inline float inv_inertia_form(float4 I0, float4 I1, V3 x, V3 y) {
  const V3 Sy = v3(I0.x * y.x + I0.w * y.y + I1.x * y.z, I0.w * y.x + I0.y * y.y + I1.y * y.z,
                   I1.x * y.x + I1.y * y.y + I0.z * y.z);
  return dot(x, Sy);
}

// Projections on dof i of a subtree of the facet rows' share on one of its
// bodies, y_f = (L^-1 J_b^T w_f)_i with w_f = (u_f, a_f) as in diag_impedance,
// from the body's columns Y = L^-1 J_b^T (column r at Y + r nd; linear 0-2,
// angular 3-5): u . yl + (r x u + e) . ya = u . (yl + ya x r) + e . ya, with
// e the torsional or rolling term of the angular direction.
template <int NF>
__device__ inline void art_facet_rows(const float *Y, int nd, int i, V3 r, V3 n, V3 t1, V3 t2, float mut,
                                      float mutor, float murol, float *y) {
  const V3 yl = v3(Y[i], Y[nd + i], Y[2 * nd + i]), ya = v3(Y[3 * nd + i], Y[4 * nd + i], Y[5 * nd + i]);
  const V3 ye = yl + cross(ya, r);
  const float pn = dot(n, ye);
  if constexpr (NF == 1) {
    y[0] = pn;
  } else {
    const float p1 = dot(t1, ye), p2 = dot(t2, ye);
    y[0] = pn - mut * p1; y[1] = pn - mut * p2; y[2] = pn + mut * p1; y[3] = pn + mut * p2;
    if constexpr (NF >= 6) {
      const float qn = dot(n, ya);
      y[4] = pn - mutor * qn; y[5] = pn + mutor * qn;
    }
    if constexpr (NF == 10) {
      const float q1 = dot(t1, ya), q2 = dot(t2, ya);
      y[6] = pn - murol * q1; y[7] = pn - murol * q2; y[8] = pn + murol * q1; y[9] = pn + murol * q2;
    }
  }
}

// Exact diagonal impedance of one contact (Sec. III.B, K h + D =
// (1/h) (J~_f M^-1 J~_f^T)^-1 per facet, split between K and D in the ratio
// k_user : d_user / h): A_f = 1 / ((k h + d) g_f), g_f = J~_f M^-1 J~_f^T.  The
// facet row acts on a body as linear direction u_f and angular direction a_f:
// tangential d: u = n - mu_t d, a = r x u; torsional sigma: u = n,
// a = r x n - mu_tor sigma n; rolling d: u = n, a = r x n - mu_rol d.  M is
// block diagonal over free bodies and subtrees, so g_f sums one term per
// block the row touches: a free body's |u_f|^2 / m + a_f^T Iw^-1 a_f; a
// subtree's |L^-1 J~_f^T|^2 over its dofs (ART: bodies of subtrees carry
// bI1.w = 1 as an integer and bI0 = (offset of their L^-1 J^T columns in
// `art`, nd, subtree root) as integers), with the row J_b^T w_b - J_a^T w_a
// when both bodies are in one subtree.
template <int NF, bool ART = false>
__device__ inline void diag_impedance(V3 n, V3 t1, V3 t2, int ba, int bb, V3 ra, V3 rb, const float4 *bC,
                                      const float4 *bI0, const float4 *bI1, float mut, float mutor, float murol,
                                      float aa, float *Af, const float *art = nullptr) {
  float g[NF];
#pragma unroll
  for (int i = 0; i < NF; ++i) g[i] = 0.f;
  // each facet's angular direction is formed as a vector before its quadratic
  // form (expanding the form into cross terms would cancel in float32)
#pragma unroll
  for (int side = 0; side < 2; ++side) {
    const int b = side ? bb : ba;
    if (b < 0) continue;
    const V3 r = side ? rb : ra;
    if constexpr (ART) {
      if (__float_as_int(bI1[b].w) != 0) {
        const float4 D = bI0[b];
        const int root = __float_as_int(D.z);
        auto in_sub = [&](int o) { return o >= 0 && __float_as_int(bI1[o].w) != 0 && __float_as_int(bI0[o].z) == root; };
        if (side == 1 && in_sub(ba)) continue;  // one row with body a's share, below
        const bool both = side == 0 && in_sub(bb);
        const int nd = __float_as_int(D.y);
        const float *Ya = art + __float_as_int(D.x), *Yb = both ? art + __float_as_int(bI0[bb].x) : Ya;
        for (int i = 0; i < nd; ++i) {
          float y[NF];
          art_facet_rows<NF>(Ya, nd, i, r, n, t1, t2, mut, mutor, murol, y);
          if (both) {
            float yb[NF];
            art_facet_rows<NF>(Yb, nd, i, rb, n, t1, t2, mut, mutor, murol, yb);
#pragma unroll
            for (int f = 0; f < NF; ++f) y[f] = yb[f] - y[f];
          }
#pragma unroll
          for (int f = 0; f < NF; ++f) g[f] += y[f] * y[f];
        }
        continue;
      }
    }
    const float4 I0 = bI0[b], I1 = bI1[b];
    const float im = bC[b].w;
    const V3 rn = cross(r, n);
    if constexpr (NF == 1) {
      g[0] += im + inv_inertia_form(I0, I1, rn, rn);
    } else {
      const V3 r1 = cross(r, t1), r2 = cross(r, t2);
      const float lin = im * (1.f + mut * mut);
      const V3 a0 = rn - mut * r1, a1 = rn - mut * r2, a2 = rn + mut * r1, a3 = rn + mut * r2;
      g[0] += lin + inv_inertia_form(I0, I1, a0, a0);
      g[1] += lin + inv_inertia_form(I0, I1, a1, a1);
      g[2] += lin + inv_inertia_form(I0, I1, a2, a2);
      g[3] += lin + inv_inertia_form(I0, I1, a3, a3);
      if constexpr (NF >= 6) {
        const V3 a4 = rn - mutor * n, a5 = rn + mutor * n;
        g[4] += im + inv_inertia_form(I0, I1, a4, a4);
        g[5] += im + inv_inertia_form(I0, I1, a5, a5);
      }
      if constexpr (NF == 10) {
        const V3 a6 = rn - murol * t1, a7 = rn - murol * t2, a8 = rn + murol * t1, a9 = rn + murol * t2;
        g[6] += im + inv_inertia_form(I0, I1, a6, a6);
        g[7] += im + inv_inertia_form(I0, I1, a7, a7);
        g[8] += im + inv_inertia_form(I0, I1, a8, a8);
        g[9] += im + inv_inertia_form(I0, I1, a9, a9);
      }
    }
  }
#pragma unroll
  for (int i = 0; i < NF; ++i) Af[i] = (g[i] > 0.f && aa > 0.f) ? 1.0f / (aa * g[i]) : 0.f;
}

// Kinematics of one contact record at the smooth velocities: frame, lever
// arms, relative velocity (b minus a), trace sum and pair friction.
struct ContactKin {
  V3 n, p, t1, t2, vrel, wrel, ra, rb;
  float phi, trs, mut, mutor, murol;
  int ga, gb, ba, bb;
  uint32_t sl;
};

__device__ inline ContactKin contact_kin(float4 cn, float4 cp, const int *gB, const float4 *gM, const float4 *bC,
                                         const float4 *bV, const float4 *bW) {
  ContactKin K;
  K.sl = __float_as_uint(cp.w);
  K.ga = slot_ga(K.sl);
  K.gb = slot_gb(K.sl);
  K.ba = gB[K.ga];
  K.bb = gB[K.gb];
  K.n = v3(cn.x, cn.y, cn.z);
  K.p = v3(cp.x, cp.y, cp.z);
  K.phi = cn.w;
  const V3 n = K.n;
  V3 t1 = fabsf(n.x) <= 0.5f ? v3(1.f - n.x * n.x, -n.x * n.y, -n.x * n.z) : v3(-n.y * n.x, 1.f - n.y * n.y, -n.y * n.z);
  K.t1 = rsqrtf(dot(t1, t1)) * t1;
  K.t2 = cross(n, K.t1);
  K.vrel = v3(0.f, 0.f, 0.f);
  K.wrel = K.vrel;
  K.ra = K.vrel;
  K.rb = K.vrel;
  K.trs = 0.f;
  if (K.bb >= 0) {
    const float4 C = bC[K.bb], Vb = bV[K.bb], Wb = bW[K.bb];
    K.rb = K.p - v3(C.x, C.y, C.z);
    const V3 wb = v3(Wb.x, Wb.y, Wb.z);
    K.vrel = v3(Vb.x, Vb.y, Vb.z) + cross(wb, K.rb);
    K.wrel = wb;
    K.trs += Vb.w;
  }
  if (K.ba >= 0) {
    const float4 C = bC[K.ba], Va = bV[K.ba], Wa = bW[K.ba];
    K.ra = K.p - v3(C.x, C.y, C.z);
    const V3 wa = v3(Wa.x, Wa.y, Wa.z);
    K.vrel = K.vrel - (v3(Va.x, Va.y, Va.z) + cross(wa, K.ra));
    K.wrel = K.wrel - wa;
    K.trs += Va.w;
  }
  const float4 ma = gM[K.ga], mb = gM[K.gb];
  K.mut = fmaxf(ma.x, mb.x);
  K.mutor = fmaxf(ma.y, mb.y);
  K.murol = fmaxf(ma.z, mb.z);
  return K;
}

// The network's 7 features (8th zero): phi, v_n, u_1, u_2, m_eff = 1/(tr_a + tr_b), mu_t, h.
__device__ inline void contact_features(const ContactKin &K, float h, float *fe) {
  fe[0] = K.phi;
  fe[1] = dot(K.n, K.vrel);
  fe[2] = dot(K.t1, K.vrel);
  fe[3] = dot(K.t2, K.vrel);
  fe[4] = K.trs > 0.f ? 1.0f / K.trs : 0.f;
  fe[5] = K.mut;
  fe[6] = h;
  fe[7] = 0.f;
}

// Fallback rule of the learned gains: with the contact alone along its normal
// (inverse mass tr_s / 3 = 1/m_a + 1/m_b for free bodies), the facet impulses
// change the normal velocity by (tr_s / 3) sum_f lambda_f; the learned
// impulses are kept unless they predict a next-step penetration larger than
// the heuristic's by more than `margin`, or a normal kinetic energy larger by
// more than that of moving `margin` in one step.
template <int NF>
__device__ inline bool learned_ok(const float *lh, const float *ll, float vn, float phi, float trs, float h,
                                  float margin) {
  if (!(trs > 0.f)) return false;
  const float winv = trs * (1.0f / 3.0f);
  float Sh = 0.f, Sl = 0.f;
#pragma unroll
  for (int i = 0; i < NF; ++i) {
    Sh += lh[i];
    Sl += ll[i];
  }
  const float vh = vn + winv * Sh, vl = vn + winv * Sl;
  const float ph = fmaxf(-(phi + h * vh), 0.f), pl = fmaxf(-(phi + h * vl), 0.f);
  const float eh = 0.5f * vh * vh / winv, el = 0.5f * vl * vl / winv;
  const float em = 0.5f * (margin / h) * (margin / h) / winv;
  return pl <= ph + margin && el <= eh + em && isfinite(vl);
}

// Smooth prediction of one free body (Eq. smooth_vel with the block-diagonal
// M = diag(m I3, R diag(I) R^T) and c = (-m g, w x I_w w)) from its q (7), v (6)
// and applied force (6) entries and its (m, Ixx, Iyy, Izz): (COM | 1/m),
// (v_s | trace 3/m), (w_s | 0) and the inverse world inertia (xx yy zz xy | xz yz).
__device__ inline void free_body_predict(const float *qb, const float *vb, const float *tb, float4 mi,
                                         const Params &P, float4 &C, float4 &Vs, float4 &Ws, float4 &I0,
                                         float4 &I1) {
  // hardware reciprocals (1 ulp) for the per-body inverses
  const float invm = __builtin_amdgcn_rcpf(mi.x);
  if (mi.y == mi.z && mi.y == mi.w) {
    // isotropic inertia (spheres, cubes): I_w = I 1 in every orientation, so
    // the gyroscopic bias w x I_w w vanishes and I_w^-1 = (1/I) 1
    const float ei = __builtin_amdgcn_rcpf(mi.y);
    C = make_float4(qb[0], qb[1], qb[2], invm);
    Vs = make_float4(vb[0] + P.h * (tb[0] * invm + P.gx), vb[1] + P.h * (tb[1] * invm + P.gy),
                     vb[2] + P.h * (tb[2] * invm + P.gz), 3.0f * invm);
    Ws = make_float4(vb[3] + P.h * (ei * tb[3]), vb[4] + P.h * (ei * tb[4]), vb[5] + P.h * (ei * tb[5]), 0.f);
    I0 = make_float4(ei, ei, ei, 0.f);
    I1 = make_float4(0.f, 0.f, 0.f, 0.f);
    return;
  }
  float R[9];
  quat_to_rot<float>(qb[3], qb[4], qb[5], qb[6], R);
  const float d[3] = {mi.y, mi.z, mi.w},
              e[3] = {__builtin_amdgcn_rcpf(mi.y), __builtin_amdgcn_rcpf(mi.z), __builtin_amdgcn_rcpf(mi.w)};
  // world inertia R diag(I) R^T and its inverse R diag(1/I) R^T (xx, yy, zz, xy, xz, yz)
  float Iw[6], Ii[6];
  const int ri[6] = {0, 1, 2, 0, 0, 1}, rj[6] = {0, 1, 2, 1, 2, 2};
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    const float *u = R + 3 * ri[k], *v = R + 3 * rj[k];
    Iw[k] = u[0] * d[0] * v[0] + u[1] * d[1] * v[1] + u[2] * d[2] * v[2];
    Ii[k] = u[0] * e[0] * v[0] + u[1] * e[1] * v[1] + u[2] * e[2] * v[2];
  }
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
  C = make_float4(qb[0], qb[1], qb[2], invm);
  Vs = make_float4(vs.x, vs.y, vs.z, 3.0f * invm);
  Ws = make_float4(ws.x, ws.y, ws.z, 0.f);
  I0 = make_float4(Ii[0], Ii[1], Ii[2], Ii[3]);
  I1 = make_float4(Ii[4], Ii[5], 0.f, 0.f);
}

// Velocity correction (Eq. vel_correction) and semi-implicit Euler step of one
// free body: v+ = v_s + (F/m, I_w^-1 T), x+ = x + h v+, quat+ = normalize(
// exp(h w+) (x) quat) with the world-frame angular velocity.  qb: the body's q
// entries (quaternion read from [3..6]); writes q+ (7) and v+ (6).
__device__ inline void free_body_correct(float4 C, float4 Vs, float4 Ws, float4 I0, float4 I1, float4 F, float4 T,
                                         const float *qb, const Params &P, float *qo, float *vo) {
  const V3 vp = v3(Vs.x + C.w * F.x, Vs.y + C.w * F.y, Vs.z + C.w * F.z);
  const V3 wp = v3(Ws.x + I0.x * T.x + I0.w * T.y + I1.x * T.z,
                   Ws.y + I0.w * T.x + I0.y * T.y + I1.y * T.z,
                   Ws.z + I1.x * T.x + I1.y * T.y + I0.z * T.z);
  const float qw0 = qb[3], qx0 = qb[4], qy0 = qb[5], qz0 = qb[6];
  vo[0] = vp.x; vo[1] = vp.y; vo[2] = vp.z; vo[3] = wp.x; vo[4] = wp.y; vo[5] = wp.z;
  qo[0] = C.x + P.h * vp.x;
  qo[1] = C.y + P.h * vp.y;
  qo[2] = C.z + P.h * vp.z;
  const V3 th = P.h * wp;
  float ew, ex, ey, ez;
  quat_of_rotvec(th, ew, ex, ey, ez);
  const float nw_ = ew * qw0 - ex * qx0 - ey * qy0 - ez * qz0;
  const float nx_ = ew * qx0 + ex * qw0 + ey * qz0 - ez * qy0;
  const float ny_ = ew * qy0 - ex * qz0 + ey * qw0 + ez * qx0;
  const float nz_ = ew * qz0 + ex * qy0 - ey * qx0 + ez * qw0;
  const float inv = rsqrtf(nw_ * nw_ + nx_ * nx_ + ny_ * ny_ + nz_ * nz_);
  qo[3] = nw_ * inv; qo[4] = nx_ * inv; qo[5] = ny_ * inv; qo[6] = nz_ * inv;
}

// Heuristic impedance of a contact (Eqs. k_d_setting, r_scaling): x = |phi|/w
// clamped to [0, 1], gamma(x) from the solimp power law, r between r_min and
// r_max, A = r / ((1 - r) (tr_a + tr_b)); 0 without a body trace.
__device__ inline float heuristic_gain(float phi, float trs, const Params &P) {
  const float x = fminf(fabsf(phi) * P.inv_width, 1.0f);
  const bool lo = x < P.mid;
  const float u = lo ? x * P.inv_mid : (1.0f - x) * P.inv_1mmid;
  const float up = P.power2 ? u * u : powf(u, P.power);
  const float gam = lo ? P.mid * up : 1.0f - (1.0f - P.mid) * up;
  const float r = P.r_min + (P.r_max - P.r_min) * gam;
  return trs > 0.f ? r * __builtin_amdgcn_rcpf((1.0f - r) * trs) : 0.f;
}

// Facet impulses lambda_f h = G_f max(-(k h + d) s_f - k phi, 0) (Eq. cf_wrench)
// with s_f = v_n - mu_s d_f . (subspace velocity), facets in the fixed order:
// tangential d = +t1, +t2, -t1, -t2, then torsional +, -, then rolling.
template <int CONDIM>
__device__ inline void facet_impulses(const float *G, const ContactKin &K, float aa, float c0, float *L) {
  const float vn = dot(K.n, K.vrel);
  if constexpr (CONDIM == 1) {
    L[0] = G[0] * fmaxf(-aa * vn + c0, 0.f);
  } else {
    const float u1 = dot(K.t1, K.vrel), u2 = dot(K.t2, K.vrel), mut = K.mut;
    L[0] = G[0] * fmaxf(-aa * (vn - mut * u1) + c0, 0.f);
    L[1] = G[1] * fmaxf(-aa * (vn - mut * u2) + c0, 0.f);
    L[2] = G[2] * fmaxf(-aa * (vn + mut * u1) + c0, 0.f);
    L[3] = G[3] * fmaxf(-aa * (vn + mut * u2) + c0, 0.f);
    if constexpr (CONDIM >= 4) {
      const float wt = dot(K.n, K.wrel);
      L[4] = G[4] * fmaxf(-aa * (vn - K.mutor * wt) + c0, 0.f);
      L[5] = G[5] * fmaxf(-aa * (vn + K.mutor * wt) + c0, 0.f);
    }
    if constexpr (CONDIM == 6) {
      const float o1 = dot(K.t1, K.wrel), o2 = dot(K.t2, K.wrel);
      L[6] = G[6] * fmaxf(-aa * (vn - K.murol * o1) + c0, 0.f);
      L[7] = G[7] * fmaxf(-aa * (vn - K.murol * o2) + c0, 0.f);
      L[8] = G[8] * fmaxf(-aa * (vn + K.murol * o1) + c0, 0.f);
      L[9] = G[9] * fmaxf(-aa * (vn + K.murol * o2) + c0, 0.f);
    }
  }
}

// Contact wrench of the facet impulses (J~^T lambda h in the contact frame):
// force f = sum_f lambda_f (n - mu_t d_f) over the tangential facets plus the
// normal part of the others, and the torsional / rolling torque tc.
template <int CONDIM>
__device__ inline void contact_wrench(const float *lam, const ContactKin &K, V3 &f, V3 &tc) {
  tc = v3(0.f, 0.f, 0.f);
  if constexpr (CONDIM == 1) {
    f = lam[0] * K.n;
  } else {
    float N = lam[0] + lam[1] + lam[2] + lam[3];
    const float e1 = -K.mut * (lam[0] - lam[2]), e2 = -K.mut * (lam[1] - lam[3]);
    if constexpr (CONDIM >= 4) {
      N += lam[4] + lam[5];
      tc = (-K.mutor * (lam[4] - lam[5])) * K.n;
    }
    if constexpr (CONDIM == 6) {
      N += lam[6] + lam[7] + lam[8] + lam[9];
      tc = tc + (-K.murol * (lam[6] - lam[8])) * K.t1 + (-K.murol * (lam[7] - lam[9])) * K.t2;
    }
    f = N * K.n + e1 * K.t1 + e2 * K.t2;
  }
}

// Optional per-contact exports of a step (row ci of the caller's arrays).
template <int NF>
__device__ inline void export_contact(const ResolveArgs &a, size_t ci, const ContactKin &K, const float *lam) {
  if (a.x_geom) { a.x_geom[2 * ci] = K.ga; a.x_geom[2 * ci + 1] = K.gb; }
  if (a.x_sub) a.x_sub[ci] = slot_sub(K.sl);
  if (a.x_dist) a.x_dist[ci] = K.phi;
  if (a.x_pos) { a.x_pos[3 * ci] = K.p.x; a.x_pos[3 * ci + 1] = K.p.y; a.x_pos[3 * ci + 2] = K.p.z; }
  if (a.x_frame) {
    float *fr = a.x_frame + 9 * ci;
    fr[0] = K.n.x; fr[1] = K.n.y; fr[2] = K.n.z;
    fr[3] = K.t1.x; fr[4] = K.t1.y; fr[5] = K.t1.z;
    fr[6] = K.t2.x; fr[7] = K.t2.y; fr[8] = K.t2.z;
  }
  if (a.x_imp) {
#pragma unroll
    for (int i = 0; i < NF; ++i) a.x_imp[(size_t)NF * ci + i] = lam[i];
  }
}

// Training data of the learned gains: the contact's features and, on every
// facet, the log of the gain multiplier g (clipped to [-ln 256, ln 256]) that
// the learned gains should apply to the heuristic's.  g is taken for the
// contact alone along its normal, the model of the fallback rule: with the
// heuristic's facet impulses lh (normal impulse S = sum lh) the normal
// velocity after the step is v(g) = v_n + w g S (w = trs / 3); g puts it at
// v* = min(-phi / h, (v_h + v_max) / 2), the velocity that closes the gap in
// this step, capped half-way between the heuristic's v_h = v(1) and the
// largest v_max = sqrt(v_h^2 + (margin / h)^2) the rule's energy test
// accepts (margin: the model's learned-gain margin).  No normal impulse: g = 1.
template <int CONDIM>
__device__ inline void export_training(const ResolveArgs &a, size_t ci, const ContactKin &K, float A, float aa,
                                       const Params &P) {
  constexpr int NF = CONDIM == 1 ? 1 : CONDIM == 3 ? 4 : CONDIM == 4 ? 6 : 10;
  if (a.x_feat) {
    float fe[mlp::NIN];
    contact_features(K, P.h, fe);
#pragma unroll
    for (int i = 0; i < mlp::NIN; ++i) a.x_feat[(size_t)mlp::NIN * ci + i] = fe[i];
  }
  if (a.x_target) {
    float Ah[NF], lh[NF], S = 0.f;
#pragma unroll
    for (int i = 0; i < NF; ++i) Ah[i] = A;
    facet_impulses<CONDIM>(Ah, K, aa, -P.k_user * K.phi, lh);
#pragma unroll
    for (int i = 0; i < NF; ++i) S += lh[i];
    float t = 0.f;
    const float wS = K.trs * (1.0f / 3.0f) * S;
    if (wS > 0.f) {
      const float vn = dot(K.n, K.vrel), vh = vn + wS, vm = P.mlp_margin / P.h;
      const float vmax = sqrtf(vh * vh + vm * vm);
      const float vs = fminf(-K.phi / P.h, 0.5f * (vh + vmax));
      const float g = (vs - vn) / wS;
      t = g > 0.f ? fminf(fmaxf(logf(g), -mlp::CLIP), mlp::CLIP) : -mlp::CLIP;
    }
#pragma unroll
    for (int i = 0; i < mlp::NOUT; ++i) a.x_target[(size_t)mlp::NOUT * ci + i] = i < NF ? t : 0.f;
  }
}

// Fixed-point wrench sums of the resolution: exponent slot of a body with no
// entry yet, exponent of a zero entry (below any float's), and the exponent
// that flags a non-finite entry.
constexpr int FX_EMPTY = -1024, FX_ZERO = -1000, FX_BAD = 1 << 20;

// e with |x|, |y|, |z| < 2^e: from the bit pattern of the largest magnitude
// (magnitudes of floats order as their bit patterns), e = biased exponent -
// 126 (the frexp exponent of a normal float; -126 bounds every subnormal);
// FX_ZERO when all are zero (zero fits any scale) and FX_BAD when one is
// infinite or NaN.
__device__ inline int fx_exp(float x, float y, float z) {
  const uint32_t m = max(max(__float_as_uint(x) & 0x7fffffffu, __float_as_uint(y) & 0x7fffffffu),
                         __float_as_uint(z) & 0x7fffffffu);
  return m == 0u ? FX_ZERO : m >= 0x7f800000u ? FX_BAD : (int)(m >> 23) - 126;
}

// Headroom bits of a chunk's sums: a body gets at most one entry per lane (a
// contact's two sides are different bodies), so at most BS entries per chunk.
template <int BS>
constexpr int fx_headroom() {
  return BS <= 64 ? 6 : BS <= 128 ? 7 : 8;
}

// Raises the force and torque exponents at e and e + stride to cover the
// wrench entry (a.xyz force, a.w b.xy torque).
__device__ inline void fx_exponents(int *e, int stride, float4 a, float2 b) {
  atomicMax(e, fx_exp(a.x, a.y, a.z));
  atomicMax(e + stride, fx_exp(a.w, b.x, b.y));
}

// Adds the entry (a, b) of body k, each part scaled by 2^s, s = 31 - e - L
// (L = headroom bits), and truncated, to the body's three packed words (Fx|Fy,
// Fz|Tx, Ty|Tz) at q[k], q[k + stride], q[k + 2 stride]; e: the body's force
// and torque exponents at e[k] and e[k + stride].  A word holds lo + 2^32 hi in
// two's complement: each half's sum stays below 2^31 in magnitude, so the
// 64-bit sum of the packed entries is exactly (sum of lo) + 2^32 (sum of hi).
template <int BS>
__device__ inline void fx_add(unsigned long long *q, const int *e, int k, int stride, float4 a, float2 b) {
  constexpr int L = fx_headroom<BS>();
  const int sf = 31 - e[k] - L, st = 31 - e[stride + k] - L;
  // the conversion truncates toward zero
  auto u = [&](float x, int sh) { return (unsigned long long)(long long)(int)ldexpf(x, sh); };
  atomicAdd(q + k, u(a.x, sf) + (u(a.y, sf) << 32));
  atomicAdd(q + stride + k, u(a.z, sf) + (u(a.w, st) << 32));
  atomicAdd(q + 2 * stride + k, u(b.x, st) + (u(b.y, st) << 32));
}

// The low and the high half's sums of a packed word.
__device__ inline int fx_lo(unsigned long long t) { return (int)(uint32_t)t; }
__device__ inline int fx_hi(unsigned long long t) {
  return (int)(uint32_t)((t - (unsigned long long)(long long)fx_lo(t)) >> 32);
}

// Float value of a fixed-point sum with exponent e (NaN when an entry was not
// finite).
template <int BS>
__device__ inline float fx_value(int sum, int e) {
  return e >= FX_BAD ? __builtin_nanf("") : ldexpf((float)sum, -(31 - e - fx_headroom<BS>()));
}

// Per geom: body and pair-friction inputs (mu_t, mu_tor, mu_rol) in LDS, for
// geoms g0, g0 + BS, ... (callers that prefetched geom threadIdx.x pass g0 = BS).
template <int CONDIM, int BS>
__device__ inline void resolve_geoms(const ResolveArgs &a, int w, int *gB, float4 *gM, int g0) {
  for (int g = g0 + (int)threadIdx.x; g < a.ng; g += BS) {
    gB[g] = a.gbody[g];
    const float mu_t = a.gmu[(size_t)w * a.ng + g];
    float2 fr = make_float2(0.f, 0.f);
    if (CONDIM >= 4) fr = a.gfr2[(size_t)w * a.ng + g];
    gM[g] = make_float4(mu_t, fr.x, fr.y, 0.f);
  }
}

// Per-lane records the resolution of world w reads after its first barrier:
// lane tid's actuator, body record (free-body flag, q and dof offsets),
// subtree (lanes 4 si .. 4 si + 3: subtree si) and, for a body of a small
// subtree, its frame rows and COM offset.
struct LanePre {
  float4 act;
  int fast, qadr, dadr;
  SubTree sub;
  float4 fr[5], ipos;
};

template <bool ART>
__device__ inline LanePre lane_prefetch(const ResolveArgs &a, int w, bool frames = true) {
  const int tid = threadIdx.x;
  // every lane loads (indices clamped into the tables; a lane past the dofs,
  // bodies or subtrees holds another entry's values, which it never uses), so
  // no wait separates these loads
  LanePre L;
  L.act = make_float4(0.f, 0.f, 0.f, __int_as_float(-1));
  if (a.act) L.act = a.act[tid < a.nv ? tid : a.nv - 1];
  L.fast = 1;
  L.qadr = 7 * tid;
  L.dadr = 6 * tid;
  L.sub = SubTree{};
#pragma unroll
  for (int i = 0; i < 5; ++i) L.fr[i] = make_float4(0.f, 0.f, 0.f, 0.f);
  L.ipos = L.fr[0];
  if (ART) {  // (at least one body and one subtree)
    const int b = tid < a.nb ? tid : a.nb - 1;
    const BodyC &bc = a.body[b];
    L.fast = bc.fast;
    L.qadr = bc.qadr;
    L.dadr = bc.dadr;
    L.ipos = bc.ipos;
    if (frames && a.frames) {
      const float4 *f = a.frames + ((size_t)w * a.nb + b) * 5;
#pragma unroll
      for (int i = 0; i < 5; ++i) L.fr[i] = f[i];
    }
    L.sub = a.sub[tid < 4 * a.nsub ? tid >> 2 : a.nsub - 1];
  }
  return L;
}

// Resolution of world w: its q and v rows (LDS sq, sv) become q+ and v+ in
// place; st holds the step input (applied forces; an actuated dof's target is
// replaced by its actuator force); the nc contacts are read from inn/inp
// (global or LDS), the first chunk already loaded by the caller into c0n/c0p
// (lane tid's record), and mi0 is body tid's mass/inertia.  `reg`: LDS scratch of
// resolve_region_bytes().  `xbase`: row of the world in the export arrays.
// NETREF (the adjoint's recomputation of a step with learned gains): the
// gains come from the float32 network of cf_adjoint.h, the function the
// adjoint differentiates, in place of the bf16 matrix evaluation.
// Ends with a workgroup barrier.
template <int CONDIM, int BS, bool ART, bool LEARN = false, bool NETREF = false>
__device__ void resolve_world(const ResolveArgs &a, int w, float *sq, float *sv, float *st,
                              const float4 *inn, const float4 *inp, int nc, float4 c0n, float4 c0p,
                              float4 mi0, float4 *reg, size_t xbase, bool geoms_ready = false,
                              const mlp::Weights *lnet = nullptr, float *lfeat = nullptr, float *lout = nullptr,
                              const LanePre *pre = nullptr) {
  constexpr int NF = CONDIM == 1 ? 1 : CONDIM == 3 ? 4 : CONDIM == 4 ? 6 : 10;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int nb = a.nb, ng = a.ng;
  const ResolveRegion RR = resolve_region(reg, nb, ng);
  float4 *bC = RR.bC, *bV = RR.bV, *bW = RR.bW, *bI0 = RR.bI0, *bI1 = RR.bI1;
  float4 *accF = RR.accF, *accT = RR.accT, *gM = RR.gM;
  int *gB = RR.gB, *fx = RR.fx;
  const int nbp = pad4(nb);
  int *fxE = fx + 6 * nbp;
  unsigned long long *fxQ = reinterpret_cast<unsigned long long *>(fx);  // [3][nbp] packed sums
  float4 *bO = RR.bO, *bAx = RR.bAx, *bR = RR.bR;  // articulated bodies only
  float *art = RR.art;
  const Params P = a.p;
  // the general subtree path's out-of-line calls take the parameters by
  // reference: their own copy, so that P's fields stay in registers here
  const Params Pcall = a.p;
  // what the lane reads below, loaded together up front unless the caller
  // has (its actuator, body record, subtree and body frame)
  const LanePre L = pre ? *pre : lane_prefetch<ART>(a, w);
  const float4 act0 = L.act;
  const int fast0 = L.fast, qadr0 = L.qadr, dadr0 = L.dadr;
  const SubTree sub0 = L.sub;
  if (!geoms_ready) resolve_geoms<CONDIM, BS>(a, w, gB, gM, 0);
  if (ART && a.frames) {
    // small subtrees: frames from the narrow phase, inertia in bW and COM
    // offset in bC until the prediction replaces them
    const float4 *fw = a.frames + (size_t)w * nb * 5;
    for (int b = tid; b < nb; b += BS) {
      const bool mine = b == tid;
      if (mine ? fast0 : a.body[b].fast) continue;
#pragma unroll
      for (int i = 0; i < 5; ++i) {
        const float4 f = mine ? L.fr[i] : fw[5 * b + i];
        if (i == 0) bO[b] = f;
        else if (i == 1) bAx[b] = f;
        else bR[3 * b + i - 2] = f;
      }
      bC[b] = mine ? L.ipos : a.body[b].ipos;
      bW[b] = mine ? mi0 : a.bmi[(size_t)w * nb + b];
    }
  }
  __syncthreads();
  if (a.act) {
    // position actuators: the input of an actuated dof is its target u, the
    // applied force kp (u - q) - kd v on the state at the start of the step
    for (int i = tid; i < a.nv; i += BS) {
      const float4 c = i == tid ? act0 : a.act[i];
      const int qi = __float_as_int(c.z);
      if (qi >= 0) st[i] = c.x * (st[i] - sq[qi]) - c.y * sv[i];
    }
    __syncthreads();
  }

  // ---- per free body: M blocks, bias, smooth prediction (Eq. smooth_vel), trace 3/m
  // (without articulated subtrees every body is a free root: q and v offsets 7b and 6b)
  for (int b = tid; b < nb; b += BS) {
    int qadr = 7 * b, dadr = 6 * b;
    if (ART) {
      if (b == tid) {
        if (!fast0) continue;
        qadr = qadr0;
        dadr = dadr0;
      } else {
        const BodyC &bc = a.body[b];
        if (!bc.fast) continue;
        qadr = bc.qadr;
        dadr = bc.dadr;
      }
    }
    const float4 mi = b == tid ? mi0 : a.bmi[(size_t)w * nb + b];
    free_body_predict(sq + qadr, sv + dadr, st + dadr, mi, P, bC[b], bV[b], bW[b], bI0[b], bI1[b]);
  }
  for (int b = tid; b < nb; b += BS) {
    accF[b] = make_float4(0.f, 0.f, 0.f, 0.f);
    accT[b] = make_float4(0.f, 0.f, 0.f, 0.f);
  }
  for (int i = tid; i < 8 * nbp; i += BS) fx[i] = i >= 6 * nbp ? FX_EMPTY : 0;
  // ---- articulated subtrees: one lane each (same equations, dense per-subtree M)
  // (lanes 4 si .. 4 si + 3 take subtree si: a quad for a small one, its first
  // lane for any other)
  if (ART)
  for (int t = tid; t < 4 * a.nsub; t += BS) {
    const SubTree S = t == tid ? sub0 : a.sub[t >> 2];
    float *yd = P.imp_diag ? art + S.yofs : nullptr;
    if (S.small)
      art_predict_small(S, t & 3, sv, st, bC, bV, bW, bO, bAx, bR, art + S.lofs, P, yd);
    else if ((t & 3) == 0)
      art_predict(S, a.body, a.bmi + (size_t)w * nb, sq, sv, st, bC, bV, bW, bO, bAx, bR, art + S.lofs, Pcall,
                  yd);
    if (yd && (t & 3) == 0)  // the subtree's bodies: where their L^-1 J^T columns are
      for (int k = 0; k < S.nb; ++k) {
        bI0[S.b0 + k] = make_float4(__int_as_float(S.yofs + 6 * S.nd * k), __int_as_float(S.nd),
                                    __int_as_float(S.b0), 0.f);
        bI1[S.b0 + k] = make_float4(0.f, 0.f, 0.f, __int_as_float(1));
      }
  }
  __syncthreads();

  // ---- contacts: facet impulses, wrenches, deterministic per-body reduction
  const float aa = P.k_user * P.h + P.d_user;
  for (int base = 0; base < nc; base += BS) {
    const int k = base + tid;
    int kA = nb, kB = nb;  // key nb = no body (static geom or idle lane)
    float4 WA = make_float4(0.f, 0.f, 0.f, 0.f), WB = WA;
    float2 WA2 = make_float2(0.f, 0.f), WB2 = WA2;
    if constexpr (LEARN) {
      // learned gains: features of the wave's contacts to LDS, the network on
      // MFMA (all lanes of the wave), outputs back to LDS
      float fe[mlp::NIN] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
      if (k < nc) {
        const ContactKin K = contact_kin(base == 0 ? c0n : inn[k], base == 0 ? c0p : inp[k], gB, gM, bC, bV, bW);
        contact_features(K, P.h, fe);
      }
#pragma unroll
      for (int i = 0; i < mlp::NIN; ++i) lfeat[tid * mlp::NIN + i] = fe[i];
      __builtin_amdgcn_wave_barrier();
      const int q = lane >> 4, cc = lane & 15;
#pragma unroll
      for (int tile = 0; tile < 4; ++tile) {
        const int row = wave * 64 + tile * 16 + cc;
        mlp::Tile T;
        mlp::forward_tile(lnet, [&](int t) { return lfeat[row * mlp::NIN + 4 * q + t]; }, T);
#pragma unroll
        for (int r = 0; r < 4; ++r) lout[row * mlp::NOUT + 4 * q + r] = T.y[r];
      }
      __builtin_amdgcn_wave_barrier();
    }
    if (k < nc) {
      const ContactKin K = contact_kin(base == 0 ? c0n : inn[k], base == 0 ? c0p : inp[k], gB, gM, bC, bV, bW);
      const int ba = K.ba, bb = K.bb;
      const V3 n = K.n, t1 = K.t1, t2 = K.t2, ra = K.ra, rb = K.rb;
      const float phi = K.phi, trs = K.trs, mut = K.mut, mutor = K.mutor, murol = K.murol;
      const float A = heuristic_gain(phi, trs, P);
      float Af[NF];
#pragma unroll
      for (int i = 0; i < NF; ++i) Af[i] = A;
      if (P.imp_diag)
        diag_impedance<NF, ART>(n, t1, t2, ba, bb, ra, rb, bC, bI0, bI1, mut, mutor, murol, aa, Af, art);
      const float c0 = -P.k_user * phi;
      float lam[NF];
      facet_impulses<CONDIM>(Af, K, aa, c0, lam);
      if constexpr (NETREF) {
        if (a.mlp) {
          // positive parts of the facet arguments (unit gains), then the
          // network's gains and the fallback rule on them
          float one[NF], pz[NF];
#pragma unroll
          for (int i = 0; i < NF; ++i) one[i] = 1.f;
          facet_impulses<CONDIM>(one, K, aa, c0, pz);
          adj::ContactIn<float> C{};
          C.phi = phi; C.trs = trs; C.mut = mut; C.h = P.h;
          C.net = a.mlp; C.margin = P.mlp_margin;
          adj::LearnedEval<NF, float> Le;
          adj::learned_eval<NF>(C, A, dot(n, K.vrel), dot(t1, K.vrel), dot(t2, K.vrel), pz, Le);
          if (Le.keep) {
#pragma unroll
            for (int i = 0; i < NF; ++i) lam[i] = Le.G[i] * pz[i];
          }
        }
      }
      if constexpr (LEARN) {
        // learned gains, kept unless they predict more penetration or more
        // kinetic energy along the normal than the heuristic's, beyond the margin
        float Gl[NF], ll[NF];
#pragma unroll
        for (int i = 0; i < NF; ++i) Gl[i] = A * __expf(fminf(fmaxf(lout[tid * mlp::NOUT + i], -mlp::CLIP), mlp::CLIP));
        facet_impulses<CONDIM>(Gl, K, aa, c0, ll);
        const bool keep = learned_ok<NF>(lam, ll, dot(n, K.vrel), phi, trs, P.h, P.mlp_margin);
        if (keep) {
#pragma unroll
          for (int i = 0; i < NF; ++i) lam[i] = ll[i];
        }
        if (a.x_fallback) a.x_fallback[xbase + k] = keep ? 0 : 1;
      }
      V3 f, tc;
      contact_wrench<CONDIM>(lam, K, f, tc);
      if (bb >= 0) {
        const V3 T = CONDIM >= 4 ? cross(rb, f) + tc : cross(rb, f);
        kB = bb;
        WB = make_float4(f.x, f.y, f.z, T.x);
        WB2 = make_float2(T.y, T.z);
      }
      if (ba >= 0) {
        const V3 T = CONDIM >= 4 ? cross(ra, f) + tc : cross(ra, f);
        kA = ba;
        WA = make_float4(-f.x, -f.y, -f.z, -T.x);
        WA2 = make_float2(-T.y, -T.z);
      }
      const size_t ci = xbase + k;
      export_contact<NF>(a, ci, K, lam);
      if (!ART) export_training<CONDIM>(a, ci, K, A, aa, P);
    }
    // Per-body sums of the chunk's wrench entries in fixed point: integer
    // additions commute, so the order of the LDS atomics does not change the
    // result.  The force and the torque part of body k are scaled by 2^s,
    // s = 31 - e - L, with every entry's components of that part below 2^e in
    // magnitude and at most 2^L entries, so no sum reaches 2^31; two
    // components share each 64-bit LDS word (three atomics per entry).
    if (kA < nb) fx_exponents(fxE + kA, nbp, WA, WA2);
    if (kB < nb) fx_exponents(fxE + kB, nbp, WB, WB2);
    __syncthreads();
    if (kA < nb) fx_add<BS>(fxQ, fxE, kA, nbp, WA, WA2);
    if (kB < nb) fx_add<BS>(fxQ, fxE, kB, nbp, WB, WB2);
    __syncthreads();
    // chunk sums into the float accumulators (chunks in order), slots cleared
    for (int b = tid; b < nb; b += BS) {
      const int ef = fxE[b], et = fxE[nbp + b];
      if (ef == FX_EMPTY) continue;  // no entry this chunk (an entry raises both exponents)
      float4 F = accF[b], T = accT[b];
      const unsigned long long q0 = fxQ[b], q1 = fxQ[nbp + b], q2 = fxQ[2 * nbp + b];
      F.x += fx_value<BS>(fx_lo(q0), ef);
      F.y += fx_value<BS>(fx_hi(q0), ef);
      F.z += fx_value<BS>(fx_lo(q1), ef);
      T.x += fx_value<BS>(fx_hi(q1), et);
      T.y += fx_value<BS>(fx_lo(q2), et);
      T.z += fx_value<BS>(fx_hi(q2), et);
      accF[b] = F; accT[b] = T;
      fxQ[b] = 0ull; fxQ[nbp + b] = 0ull; fxQ[2 * nbp + b] = 0ull;
      fxE[b] = FX_EMPTY;
      fxE[nbp + b] = FX_EMPTY;
    }
    __syncthreads();
  }

  // ---- velocity correction (Eq. vel_correction) and semi-implicit Euler
  if (ART)
  for (int t = tid; t < 4 * a.nsub; t += BS) {
    const SubTree S = t == tid ? sub0 : a.sub[t >> 2];
    if (S.small)
      art_correct_small(S, t & 3, a.body, bC, bO, bAx, accF, accT, sq, sv, art + S.lofs, P);
    else if ((t & 3) == 0)
      art_correct(S, a.body, bC, bO, bAx, accF, accT, sq, sv, art + S.lofs, Pcall);
  }
  for (int b = tid; b < nb; b += BS) {
    int qadr = 7 * b, dadr = 6 * b;
    if (ART) {
      const BodyC bc = a.body[b];
      if (!bc.fast) continue;
      qadr = bc.qadr;
      dadr = bc.dadr;
    }
    float *qb = sq + qadr;
    free_body_correct(bC[b], bV[b], bW[b], bI0[b], bI1[b], accF[b], accT[b], qb, P, qb, sv + dadr);
  }
  __syncthreads();
}

size_t resolve_learned_lds_bytes(int block) {
  return (sizeof(mlp::Weights) + 15) / 16 * 16 + sizeof(float) * (size_t)block * (mlp::NIN + mlp::NOUT);
}

template <int CONDIM, int BS, bool ART, bool LEARN>
__global__ __launch_bounds__(BS) void resolve_kernel(ResolveArgs a) {
  constexpr int K = 512 / BS;  // row elements per lane loaded up front
  extern __shared__ float4 lds[];
  const int w = blockIdx.x, tid = threadIdx.x;
  const int nq = a.nq, nv = a.nv, nb = a.nb, ng = a.ng;
  float *sq = reinterpret_cast<float *>(lds);
  float *sv = sq + pad4(nq);
  float *st = sv + pad4(nv);
  float4 *reg = reinterpret_cast<float4 *>(st + pad4(nv));
  const size_t cbase = (size_t)w * a.ncon_max;
  // issue every independent global load before the first wait, every lane
  // all of them (indices clamped into the arrays, which hold at least one
  // entry; a lane past the records, bodies or geoms never uses what it read)
  const int nc = a.ncon[w];
  const int r0 = tid < a.ncon_max ? tid : (a.ncon_max > 0 ? a.ncon_max - 1 : 0);
  const float4 c0n = a.cnp[cbase + r0], c0p = a.cpos[cbase + r0];  // the first chunk's records
  const float4 mi0 = a.bmi[(size_t)w * nb + (tid < nb ? tid : (nb > 0 ? nb - 1 : 0))];
  const LanePre pre = lane_prefetch<ART>(a, w);
  const int g0 = tid < ng ? tid : (ng > 0 ? ng - 1 : 0);
  const int gb0 = a.gbody[g0];
  const float mu0 = a.gmu[(size_t)w * ng + g0];
  float2 fr0 = make_float2(0.f, 0.f);
  if (CONDIM >= 4) fr0 = a.gfr2[(size_t)w * ng + g0];
  const float *qw = a.q + (size_t)w * nq, *vw = a.v + (size_t)w * nv;
  const float *tw = a.tau ? a.tau + (size_t)w * nv : nullptr;
  RowStage<BS, K> rq, rv, rt;
  rq.load(qw, nq);
  rv.load(vw, nv);
  if (tw) rt.load(tw, nv);
  rq.store(sq, qw, nq);
  rv.store(sv, vw, nv);
  if (tw) {
    rt.store(st, tw, nv);
  } else {
    for (int i = tid; i < nv; i += BS) st[i] = 0.f;
  }
  const ResolveRegion RR = resolve_region(reg, nb, ng);
  if (tid < ng) {
    RR.gB[tid] = gb0;
    RR.gM[tid] = make_float4(mu0, fr0.x, fr0.y, 0.f);
  }
  resolve_geoms<CONDIM, BS>(a, w, RR.gB, RR.gM, BS);
  mlp::Weights *lnet = nullptr;
  float *lfeat = nullptr, *lout = nullptr;
  if constexpr (LEARN) {
    char *base = reinterpret_cast<char *>(reg) + resolve_region_bytes(nb, ng, 0, 0);
    lnet = reinterpret_cast<mlp::Weights *>(base);
    lfeat = reinterpret_cast<float *>(base + (sizeof(mlp::Weights) + 15) / 16 * 16);
    lout = lfeat + BS * mlp::NIN;
    // copy of the network's image, written for this step by launch_mlp_pack
    static_assert(sizeof(mlp::Weights) % sizeof(float4) == 0, "image copied in float4");
    float4 *dst = reinterpret_cast<float4 *>(lnet);
    for (int i = tid; i < (int)(sizeof(mlp::Weights) / sizeof(float4)); i += BS) dst[i] = a.mlp_img[i];
    __syncthreads();
  }
  resolve_world<CONDIM, BS, ART, LEARN>(a, w, sq, sv, st, a.cnp + cbase, a.cpos + cbase, nc, c0n, c0p, mi0, reg,
                                        cbase, true, lnet, lfeat, lout, &pre);
  float *qo = a.q_out + (size_t)w * nq, *vo = a.v_out + (size_t)w * nv;
  for (int i = tid; i < nq; i += BS) qo[i] = sq[i];
  for (int i = tid; i < nv; i += BS) vo[i] = sv[i];
}

// ====================================================================
// resolution of worlds of free bodies, one body per lane
// ====================================================================
// When every body is a free body without children, a world has at most BS
// bodies and no actuators or learned gains are set, lane b owns body b: it
// reads the body's q, v and tau entries itself (no rows staged in LDS), keeps
// its accumulated contact wrench in registers through the contact chunks and
// writes q+ and v+.  LDS holds only what other lanes read: per body (COM |
// 1/m), (v_s | 3/m), (w_s | -) and the inverse world inertia, the fixed-point
// chunk sums, and per geom its body and friction (8.7 KB for 64 spheres and
// 69 geoms, against 15.5 KB with staged rows), so sixteen one-wave worlds fit
// a CU together.  The next chunk's contact records are loaded while the
// current chunk is resolved.  Arithmetic as in resolve_world.
__host__ __device__ size_t resolve_free_lds_bytes(int nb, int ng) {
  return sizeof(float4) * 5 * (size_t)nb + sizeof(int) * 8 * (size_t)pad4(nb) + sizeof(int) * (size_t)pad4(ng) +
         sizeof(float4) * (size_t)ng;
}

// The geom table of world w as the free-body resolution stages it: entries
// threadIdx.x and threadIdx.x + BS of the lane (body, tangential friction,
// torsional and rolling friction), loaded unconditionally with indices
// clamped into the arrays (which hold at least one entry); stored only where
// below ng.
struct FreeGeomPre {
  int b0, b1;
  float u0, u1;
  float2 f0, f1;
};

template <int CONDIM, int BS>
__device__ inline FreeGeomPre free_geom_prefetch(const ResolveArgs &a, int w, int tid) {
  const int ng = a.ng, gl = ng > 0 ? ng - 1 : 0, g0 = tid < ng ? tid : gl, g1 = tid + BS < ng ? tid + BS : gl;
  FreeGeomPre G;
  G.b0 = a.gbody[g0];
  G.b1 = a.gbody[g1];
  G.u0 = a.gmu[(size_t)w * ng + g0];
  G.u1 = a.gmu[(size_t)w * ng + g1];
  G.f0 = G.f1 = make_float2(0.f, 0.f);
  if (CONDIM >= 4) {
    G.f0 = a.gfr2[(size_t)w * ng + g0];
    G.f1 = a.gfr2[(size_t)w * ng + g1];
  }
  return G;
}

// Resolution of world w of free bodies, lane b owning body b: from the lane's
// q (7), v (6) and applied-force (6) entries and mass/inertia, the world's nc
// contacts (the first chunk's records cn, cp of lane threadIdx.x already
// loaded by the caller, the rest read from cnp/cpos), to the lane's q+ and v+
// (qo, vo; lanes beyond nb return zeros).  `lds`: resolve_free_lds_bytes();
// `xbase`: row of the world in the export arrays; `gpre`: the caller's
// free_geom_prefetch of world w, or null.  Ends with a workgroup barrier after
// the last read of the body arrays.
template <int CONDIM, int BS>
__device__ void resolve_free_world(const ResolveArgs &a, int w, const float *qb, const float *vb, const float *tb,
                                   float4 mi, int nc, float4 cn, float4 cp, const float4 *cnp, const float4 *cpos,
                                   size_t xbase, float4 *lds, float *qo, float *vo, int tid_in = -1,
                                   const FreeGeomPre *gpre = nullptr) {
  constexpr int NF = CONDIM == 1 ? 1 : CONDIM == 3 ? 4 : CONDIM == 4 ? 6 : 10;
  const int tid = tid_in >= 0 ? tid_in : (int)threadIdx.x;
  const int nb = a.nb, ng = a.ng, nbp = pad4(nb);
  float4 *bC = lds, *bV = bC + nb, *bW = bV + nb, *bI0 = bW + nb, *bI1 = bI0 + nb;
  int *fx = reinterpret_cast<int *>(bI1 + nb);
  int *fxE = fx + 6 * nbp;
  unsigned long long *fxQ = reinterpret_cast<unsigned long long *>(fx);  // [3][nbp] packed sums
  int *gB = fx + 8 * nbp;
  float4 *gM = reinterpret_cast<float4 *>(gB + pad4(ng));
  const Params P = a.p;
  const bool own = tid < nb;
  {
    // geom table: two entries per lane (free_geom_prefetch, or the caller's),
    // stored where they exist; any further entries in a loop
    const FreeGeomPre G = gpre ? *gpre : free_geom_prefetch<CONDIM, BS>(a, w, tid);
    if (tid < ng) {
      gB[tid] = G.b0;
      gM[tid] = make_float4(G.u0, G.f0.x, G.f0.y, 0.f);
    }
    if (tid + BS < ng) {
      gB[tid + BS] = G.b1;
      gM[tid + BS] = make_float4(G.u1, G.f1.x, G.f1.y, 0.f);
    }
    for (int g = tid + 2 * BS; g < ng; g += BS) {
      gB[g] = a.gbody[g];
      float2 fr = make_float2(0.f, 0.f);
      if (CONDIM >= 4) fr = a.gfr2[(size_t)w * ng + g];
      gM[g] = make_float4(a.gmu[(size_t)w * ng + g], fr.x, fr.y, 0.f);
    }
  }
  for (int i = tid; i < 8 * nbp; i += BS) fx[i] = i >= 6 * nbp ? FX_EMPTY : 0;
  if (own) free_body_predict(qb, vb, tb, mi, P, bC[tid], bV[tid], bW[tid], bI0[tid], bI1[tid]);
  float4 F = make_float4(0.f, 0.f, 0.f, 0.f), T = F;  // the lane's body: accumulated force and torque
  __syncthreads();

  const float aa = P.k_user * P.h + P.d_user;
  for (int base = 0; base < nc; base += BS) {
    const int k = base + tid;
    // next chunk, in flight during this one: loaded by every lane (a lane
    // past the count rereads the last record and ignores it), so the wait for
    // this chunk's records leaves these two loads outstanding
    const int kn = k + BS < nc ? k + BS : nc - 1;
    const float4 nn = cnp[kn], np = cpos[kn];
    int kA = nb, kB = nb;  // key nb = no body (static geom or idle lane)
    float4 WA = make_float4(0.f, 0.f, 0.f, 0.f), WB = WA;
    float2 WA2 = make_float2(0.f, 0.f), WB2 = WA2;
    int eF = FX_ZERO;  // force exponent of the contact (the same on both sides)
    if (k < nc) {
      const ContactKin K = contact_kin(cn, cp, gB, gM, bC, bV, bW);
      const float A = heuristic_gain(K.phi, K.trs, P);
      float Af[NF];
#pragma unroll
      for (int i = 0; i < NF; ++i) Af[i] = A;
      if (P.imp_diag)
        diag_impedance<NF>(K.n, K.t1, K.t2, K.ba, K.bb, K.ra, K.rb, bC, bI0, bI1, K.mut, K.mutor, K.murol, aa, Af);
      float lam[NF];
      facet_impulses<CONDIM>(Af, K, aa, -P.k_user * K.phi, lam);
      V3 f, tc;
      contact_wrench<CONDIM>(lam, K, f, tc);
      eF = fx_exp(f.x, f.y, f.z);
      if (K.bb >= 0) {
        const V3 Tb = CONDIM >= 4 ? cross(K.rb, f) + tc : cross(K.rb, f);
        kB = K.bb;
        WB = make_float4(f.x, f.y, f.z, Tb.x);
        WB2 = make_float2(Tb.y, Tb.z);
      }
      if (K.ba >= 0) {
        const V3 Ta = CONDIM >= 4 ? cross(K.ra, f) + tc : cross(K.ra, f);
        kA = K.ba;
        WA = make_float4(-f.x, -f.y, -f.z, -Ta.x);
        WA2 = make_float2(-Ta.y, -Ta.z);
      }
      export_contact<NF>(a, xbase + k, K, lam);
      export_training<CONDIM>(a, xbase + k, K, A, aa, P);
    }
    // per-body fixed-point sums of the chunk (as in resolve_world)
    if (kA < nb) {
      atomicMax(fxE + kA, eF);
      atomicMax(fxE + nbp + kA, fx_exp(WA.w, WA2.x, WA2.y));
    }
    if (kB < nb) {
      atomicMax(fxE + kB, eF);
      atomicMax(fxE + nbp + kB, fx_exp(WB.w, WB2.x, WB2.y));
    }
    __syncthreads();
    if (kA < nb) fx_add<BS>(fxQ, fxE, kA, nbp, WA, WA2);
    if (kB < nb) fx_add<BS>(fxQ, fxE, kB, nbp, WB, WB2);
    __syncthreads();
    if (own) {
      const int ef = fxE[tid], et = fxE[nbp + tid];
      if (ef != FX_EMPTY) {  // an entry raises both exponents
        const unsigned long long q0 = fxQ[tid], q1 = fxQ[nbp + tid], q2 = fxQ[2 * nbp + tid];
        F.x += fx_value<BS>(fx_lo(q0), ef);
        F.y += fx_value<BS>(fx_hi(q0), ef);
        F.z += fx_value<BS>(fx_lo(q1), ef);
        T.x += fx_value<BS>(fx_hi(q1), et);
        T.y += fx_value<BS>(fx_lo(q2), et);
        T.z += fx_value<BS>(fx_hi(q2), et);
        fxQ[tid] = 0ull; fxQ[nbp + tid] = 0ull; fxQ[2 * nbp + tid] = 0ull;
        fxE[tid] = FX_EMPTY;
        fxE[nbp + tid] = FX_EMPTY;
      }
    }
    __syncthreads();
    cn = nn;
    cp = np;
  }

  // velocity correction and integration of the lane's body
#pragma unroll
  for (int i = 0; i < 7; ++i) qo[i] = 0.f;
#pragma unroll
  for (int i = 0; i < 6; ++i) vo[i] = 0.f;
  if (own) free_body_correct(bC[tid], bV[tid], bW[tid], bI0[tid], bI1[tid], F, T, qb, P, qo, vo);
  __syncthreads();
}

template <int CONDIM, int BS>
__global__ __launch_bounds__(BS) void resolve_free_kernel(ResolveArgs a) {
  extern __shared__ float4 lds[];
  const int w = blockIdx.x, tid = threadIdx.x;
  const int nb = a.nb;
  if (nb == 0) return;
  const size_t cbase = (size_t)w * a.ncon_max;
  // every independent global load first and unconditionally (a lane without
  // a body rereads the last one, a lane beyond the capacity the last record;
  // both ignore what they read; the workspace holds at least one record per
  // world), so that no wait separates them: the lane's body, the count, the
  // first chunk of contact records
  const bool own = tid < nb;
  const int b = own ? tid : nb - 1;
  float qb[7], vb[6], tb[6];
  {
    const float *qs = a.q + (size_t)w * a.nq + 7 * b, *vs = a.v + (size_t)w * a.nv + 6 * b;
#pragma unroll
    for (int i = 0; i < 7; ++i) qb[i] = qs[i];
#pragma unroll
    for (int i = 0; i < 6; ++i) vb[i] = vs[i];
  }
  const float4 mi = a.bmi[(size_t)w * nb + b];
  const int nc = a.ncon[w];
  const int r0 = tid < a.ncon_max ? tid : (a.ncon_max > 0 ? a.ncon_max - 1 : 0);
  const float4 cn = a.cnp[cbase + r0], cp = a.cpos[cbase + r0];
#pragma unroll
  for (int i = 0; i < 6; ++i) tb[i] = 0.f;
  if (a.tau) {
    const float *ts = a.tau + (size_t)w * a.nv + 6 * b;
#pragma unroll
    for (int i = 0; i < 6; ++i) tb[i] = ts[i];
  }
  float qo[7], vo[6];
  resolve_free_world<CONDIM, BS>(a, w, qb, vb, tb, mi, nc, cn, cp, a.cnp + cbase, a.cpos + cbase, cbase, lds, qo, vo);
  // the lane's body, stored directly
  if (own) {
    float *qd = a.q_out + (size_t)w * a.nq + 7 * tid, *vd = a.v_out + (size_t)w * a.nv + 6 * tid;
#pragma unroll
    for (int i = 0; i < 7; ++i) qd[i] = qo[i];
#pragma unroll
    for (int i = 0; i < 6; ++i) vd[i] = vo[i];
  }
}

// One step of a world of at most 64 free bodies in one one-wave workgroup:
// the narrow phase (collide_kernel's) and then the free-body resolution
// (resolve_free_kernel's) of the same world, the contact records through the
// workspace as between the two kernels.  A world's resolution starts as soon
// as its own narrow phase ends, so worlds drift apart within the launch and
// one world's loads overlap others' arithmetic, where the resolution kernel
// starts every world on the same burst of loads.  Same device functions in
// the same order: the same contacts as the two launches and results equal to
// float32 rounding (the compiler may fuse a multiply and an add differently in
// the two compilations).
// Four resident worlds per SIMD, as each phase's own kernel holds: condim
// 1/3/4 need 95/111/123 VGPRs; condim 6, bounded to 128, spills 40 bytes.
template <int CONDIM>
__global__ __launch_bounds__(64, CONDIM == 6 ? 4 : 1) void step_free_kernel(CollideArgs ca, ResolveArgs ra) {
  constexpr int BS = 64, K = 512 / BS;
  extern __shared__ float4 lds[];
  const int w = blockIdx.x, tid = threadIdx.x;
  float *sq = reinterpret_cast<float *>(lds);
  const uint32_t nxt = ca.slots[tid < ca.nslot_pre ? tid : (ca.nslot_pre > 0 ? ca.nslot_pre - 1 : 0)];
  const int gl = ca.ng > 0 ? ca.ng - 1 : 0;
  const GeomIn pre[2] = {geom_in(ca, w, tid < ca.ng ? tid : gl), geom_in(ca, w, tid + BS < ca.ng ? tid + BS : gl)};
  const float *qw = ca.q + (size_t)w * ca.nq;
  RowStage<BS, K> rq;
  rq.load(qw, ca.nq);
  // the resolution's per-lane body state, in flight through the narrow phase
  const int nb = ra.nb;
  const bool own = tid < nb;
  const int b = own ? tid : nb - 1;
  float qb[7], vb[6], tb[6];
  {
    const float *qs = ra.q + (size_t)w * ra.nq + 7 * b, *vs = ra.v + (size_t)w * ra.nv + 6 * b;
#pragma unroll
    for (int i = 0; i < 7; ++i) qb[i] = qs[i];
#pragma unroll
    for (int i = 0; i < 6; ++i) vb[i] = vs[i];
  }
  const float4 mi = ra.bmi[(size_t)w * nb + b];
  const FreeGeomPre gpre = free_geom_prefetch<CONDIM, BS>(ra, w, tid);
  rq.store(sq, qw, ca.nq);
  __syncthreads();
  const size_t cbase = (size_t)w * ca.ncon_max;
  const int found = collide_world<BS, false>(ca, w, sq, lds + pad4(ca.nq) / 4, ca.cnp + cbase, ca.cpos + cbase,
                                             ca.ncon_max, nxt, pre);
  const int nc = found < ca.ncon_max ? found : ca.ncon_max;
  if (tid == 0) {
    ca.ncon[w] = nc;
    ca.overflow[w] = found - nc;
    if (ca.ncon_out) ca.ncon_out[w] = nc;
    if (ca.overflow_out) ca.overflow_out[w] = found - nc;
  }
  // the resolution: the first chunk of the records this workgroup wrote
  // (visible after collide_world's barrier)
  const int r0 = tid < nc ? tid : (nc > 0 ? nc - 1 : 0);
  const float4 cn = ra.cnp[cbase + r0], cp = ra.cpos[cbase + r0];
#pragma unroll
  for (int i = 0; i < 6; ++i) tb[i] = 0.f;
  if (ra.tau) {
    const float *ts = ra.tau + (size_t)w * ra.nv + 6 * b;
#pragma unroll
    for (int i = 0; i < 6; ++i) tb[i] = ts[i];
  }
  float qo[7], vo[6];
  resolve_free_world<CONDIM, BS>(ra, w, qb, vb, tb, mi, nc, cn, cp, ra.cnp + cbase, ra.cpos + cbase, cbase, lds, qo, vo,
                                 -1, &gpre);
  if (own) {
    float *qd = ra.q_out + (size_t)w * ra.nq + 7 * tid, *vd = ra.v_out + (size_t)w * ra.nv + 6 * tid;
#pragma unroll
    for (int i = 0; i < 7; ++i) qd[i] = qo[i];
#pragma unroll
    for (int i = 0; i < 6; ++i) vd[i] = vo[i];
  }
}

hipError_t launch_step_free(const CollideArgs &ca, const ResolveArgs &ra, int nworld, size_t lds, hipStream_t s) {
  if (ra.nsub > 0 || ra.mlp || ra.act || ra.nb > 64 || ra.nb < 1) return hipErrorInvalidValue;
  switch (ra.condim) {
    case 1: hipLaunchKernelGGL((step_free_kernel<1>), dim3(nworld), dim3(64), lds, s, ca, ra); break;
    case 3: hipLaunchKernelGGL((step_free_kernel<3>), dim3(nworld), dim3(64), lds, s, ca, ra); break;
    case 4: hipLaunchKernelGGL((step_free_kernel<4>), dim3(nworld), dim3(64), lds, s, ca, ra); break;
    case 6: hipLaunchKernelGGL((step_free_kernel<6>), dim3(nworld), dim3(64), lds, s, ca, ra); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// One step of a world with articulated subtrees in one one-wave workgroup:
// the narrow phase (collide_kernel's, float64 kinematics writing the small
// subtrees' frames) and then the resolution (resolve_kernel's), the contact
// records and frames through the model's buffers as between the two kernels
// (read back by the same workgroup after the narrow phase's barrier) and the
// q row kept in LDS between the phases.  The resolution's loads that do not
// depend on the narrow phase (v and tau rows, mass/inertia, actuator, body and
// subtree records, the geom table) are issued before it and stay in flight
// through it.  Same device functions in the same order as the two kernels.
template <int CONDIM>
__global__ __launch_bounds__(64) void step_art_kernel(CollideArgs ca, ResolveArgs ra) {
  constexpr int BS = 64, K = 512 / BS;
  extern __shared__ float4 lds[];
  const int w = blockIdx.x, tid = threadIdx.x;
  const int nq = ra.nq, nv = ra.nv, nb = ra.nb, ng = ra.ng;
  float *sq = reinterpret_cast<float *>(lds);
  const uint32_t nxt = ca.slots[tid < ca.nslot_pre ? tid : (ca.nslot_pre > 0 ? ca.nslot_pre - 1 : 0)];
  const int gl = ng > 0 ? ng - 1 : 0;
  const GeomIn pre[2] = {geom_in(ca, w, tid < ng ? tid : gl), geom_in(ca, w, tid + BS < ng ? tid + BS : gl)};
  const float *qw = ca.q + (size_t)w * nq, *vw = ra.v + (size_t)w * nv;
  const float *tw = ra.tau ? ra.tau + (size_t)w * nv : nullptr;
  RowStage<BS, K> rq, rv, rt;
  rq.load(qw, nq);
  // the resolution's loads, in flight through the narrow phase
  const float4 mi0 = ra.bmi[(size_t)w * nb + (tid < nb ? tid : (nb > 0 ? nb - 1 : 0))];
  LanePre L = lane_prefetch<true>(ra, w, false);
  const int gb0 = ra.gbody[tid < ng ? tid : gl];
  const float mu0 = ra.gmu[(size_t)w * ng + (tid < ng ? tid : gl)];
  float2 fr0 = make_float2(0.f, 0.f);
  if (CONDIM >= 4) fr0 = ra.gfr2[(size_t)w * ng + (tid < ng ? tid : gl)];
  rv.load(vw, nv);
  if (tw) rt.load(tw, nv);
  rq.store(sq, qw, nq);
  __syncthreads();
  const size_t cbase = (size_t)w * ca.ncon_max;
  const int found = collide_world<BS, true>(ca, w, sq, lds + pad4(nq) / 4, ca.cnp + cbase, ca.cpos + cbase,
                                            ca.ncon_max, nxt, pre);
  const int nc = found < ca.ncon_max ? found : ca.ncon_max;
  if (tid == 0) {
    ca.ncon[w] = nc;
    ca.overflow[w] = found - nc;
    if (ca.ncon_out) ca.ncon_out[w] = nc;
    if (ca.overflow_out) ca.overflow_out[w] = found - nc;
  }
  // the resolution: v and tau rows after the q row (over the narrow phase's
  // scratch), the first chunk of the records and the small subtrees' frames
  // this workgroup wrote (visible after collide_world's barrier)
  float *sv = sq + pad4(nq);
  float *st = sv + pad4(nv);
  float4 *reg = reinterpret_cast<float4 *>(st + pad4(nv));
  const int r0 = tid < nc ? tid : (nc > 0 ? nc - 1 : 0);
  const float4 c0n = ra.cnp[cbase + r0], c0p = ra.cpos[cbase + r0];
  if (ra.frames) {
    const int b = tid < nb ? tid : nb - 1;
    const float4 *f = ra.frames + ((size_t)w * nb + b) * 5;
#pragma unroll
    for (int i = 0; i < 5; ++i) L.fr[i] = f[i];
  }
  rv.store(sv, vw, nv);
  if (tw) {
    rt.store(st, tw, nv);
  } else {
    for (int i = tid; i < nv; i += BS) st[i] = 0.f;
  }
  const ResolveRegion RR = resolve_region(reg, nb, ng);
  if (tid < ng) {
    RR.gB[tid] = gb0;
    RR.gM[tid] = make_float4(mu0, fr0.x, fr0.y, 0.f);
  }
  resolve_geoms<CONDIM, BS>(ra, w, RR.gB, RR.gM, BS);
  resolve_world<CONDIM, BS, true>(ra, w, sq, sv, st, ra.cnp + cbase, ra.cpos + cbase, nc, c0n, c0p, mi0, reg, cbase,
                                  true, nullptr, nullptr, nullptr, &L);
  float *qo = ra.q_out + (size_t)w * nq, *vo = ra.v_out + (size_t)w * nv;
  for (int i = tid; i < nq; i += BS) qo[i] = sq[i];
  for (int i = tid; i < nv; i += BS) vo[i] = sv[i];
}

hipError_t launch_step_art(const CollideArgs &ca, const ResolveArgs &ra, int nworld, size_t lds, hipStream_t s) {
  if (ra.nsub < 1 || ra.mlp || ra.nb < 1) return hipErrorInvalidValue;
  switch (ra.condim) {
    case 1: hipLaunchKernelGGL((step_art_kernel<1>), dim3(nworld), dim3(64), lds, s, ca, ra); break;
    case 3: hipLaunchKernelGGL((step_art_kernel<3>), dim3(nworld), dim3(64), lds, s, ca, ra); break;
    case 4: hipLaunchKernelGGL((step_art_kernel<4>), dim3(nworld), dim3(64), lds, s, ca, ra); break;
    case 6: hipLaunchKernelGGL((step_art_kernel<6>), dim3(nworld), dim3(64), lds, s, ca, ra); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// ---- learned gains on worlds of free bodies (at most 128; lane b owns
// bodies b and b + 64): four one-wave worlds per workgroup share one LDS copy
// of the network (WeightsK32, written for the
// step by launch_mlp_pack_k32); each wave resolves its world as
// resolve_free_kernel does, with wave-local ordering in place of workgroup
// barriers (worlds differ in their number of contact chunks).  Per chunk each
// 16-contact tile of the wave runs the network on K = 32 bf16 MFMA (features
// moved to the tile's K-group-0 lanes and outputs back by lane permutes); the
// contact lane then keeps the learned facet impulses unless the fallback rule
// rejects them (learned_ok).
// Worlds (waves) per workgroup: four of up to 64 bodies, two of up to 128.
__host__ __device__ constexpr int learn_worlds(int nbl) { return nbl == 1 ? 4 : 2; }

size_t resolve_learned_k32_lds_bytes(int nb, int ng) {
  return (sizeof(mlp::WeightsK32) + 15) / 16 * 16 + learn_worlds(nb > 64 ? 2 : 1) * resolve_free_lds_bytes(nb, ng);
}

// Orders the wave's LDS accesses before and after (the wave's lanes exchange
// data through LDS without a workgroup barrier).
__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

template <int CONDIM, int NBL>
__global__ __launch_bounds__(64 * learn_worlds(NBL)) void resolve_learned_kernel(ResolveArgs a) {
  constexpr int NF = CONDIM == 1 ? 1 : CONDIM == 3 ? 4 : CONDIM == 4 ? 6 : 10;
  constexpr int kLearnWorlds = learn_worlds(NBL);
  extern __shared__ float4 lds[];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int w = blockIdx.x * kLearnWorlds + wv;
  mlp::WeightsK32 *W = reinterpret_cast<mlp::WeightsK32 *>(lds);
  {  // the network's image for this step, copied by the whole workgroup
    static_assert(sizeof(mlp::WeightsK32) % sizeof(float4) == 0, "image copied in float4");
    float4 *dst = reinterpret_cast<float4 *>(W);
    for (int i = threadIdx.x; i < (int)(sizeof(mlp::WeightsK32) / sizeof(float4)); i += 64 * kLearnWorlds)
      dst[i] = a.mlp_img[i];
  }
  __syncthreads();
  if (w >= a.nworld) return;
  const int nb = a.nb, ng = a.ng, nbp = pad4(nb);
  char *region = reinterpret_cast<char *>(lds) + (sizeof(mlp::WeightsK32) + 15) / 16 * 16 +
                 (size_t)wv * resolve_free_lds_bytes(nb, ng);
  float4 *bC = reinterpret_cast<float4 *>(region), *bV = bC + nb, *bW = bV + nb, *bI0 = bW + nb, *bI1 = bI0 + nb;
  int *fx = reinterpret_cast<int *>(bI1 + nb);
  int *fxE = fx + 6 * nbp;
  unsigned long long *fxQ = reinterpret_cast<unsigned long long *>(fx);
  int *gB = fx + 8 * nbp;
  float4 *gM = reinterpret_cast<float4 *>(gB + pad4(ng));
  const Params P = a.p;
  const size_t cbase = (size_t)w * a.ncon_max;

  const int nc = a.ncon[w];
  float4 cn = make_float4(0.f, 0.f, 0.f, 0.f), cp = cn;
  if (lane < a.ncon_max) {
    cn = a.cnp[cbase + lane];
    cp = a.cpos[cbase + lane];
  }
  // the lane's bodies: lane + 64 j, j < NBL
  float qb[NBL][7];
  float4 F[NBL], T[NBL];
#pragma unroll
  for (int j = 0; j < NBL; ++j) {
    const int b = lane + 64 * j;
    float vb[6], tb[6];
    float4 mi = make_float4(1.f, 1.f, 1.f, 1.f);
#pragma unroll
    for (int i = 0; i < 7; ++i) qb[j][i] = 0.f;
#pragma unroll
    for (int i = 0; i < 6; ++i) vb[i] = tb[i] = 0.f;
    if (b < nb) {
      const float *qs = a.q + (size_t)w * a.nq + 7 * b, *vs = a.v + (size_t)w * a.nv + 6 * b;
#pragma unroll
      for (int i = 0; i < 7; ++i) qb[j][i] = qs[i];
#pragma unroll
      for (int i = 0; i < 6; ++i) vb[i] = vs[i];
      if (a.tau) {
        const float *ts = a.tau + (size_t)w * a.nv + 6 * b;
#pragma unroll
        for (int i = 0; i < 6; ++i) tb[i] = ts[i];
      }
      mi = a.bmi[(size_t)w * nb + b];
      free_body_predict(qb[j], vb, tb, mi, P, bC[b], bV[b], bW[b], bI0[b], bI1[b]);
    }
    F[j] = make_float4(0.f, 0.f, 0.f, 0.f);
    T[j] = F[j];
  }
  for (int g = lane; g < ng; g += 64) {
    gB[g] = a.gbody[g];
    const float mu_t = a.gmu[(size_t)w * ng + g];
    float2 fr = make_float2(0.f, 0.f);
    if (CONDIM >= 4) fr = a.gfr2[(size_t)w * ng + g];
    gM[g] = make_float4(mu_t, fr.x, fr.y, 0.f);
  }
  for (int i = lane; i < 8 * nbp; i += 64) fx[i] = i >= 6 * nbp ? FX_EMPTY : 0;
  wave_sync();

  const float aa = P.k_user * P.h + P.d_user;
  const int kg = lane >> 4, c16 = lane & 15;
  for (int base = 0; base < nc; base += 64) {
    const int k = base + lane, kn = k + 64;
    float4 nn = make_float4(0.f, 0.f, 0.f, 0.f), np = nn;
    if (kn < nc) {
      nn = a.cnp[cbase + kn];
      np = a.cpos[cbase + kn];
    }
    const bool live = k < nc;
    // the lane's normalised features as bf16, four packed words (the contact's
    // kinematics are formed again after the network rather than held through it)
    int xw[4];
    {
      float fe[mlp::NIN] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
      if (live) contact_features(contact_kin(cn, cp, gB, gM, bC, bV, bW), P.h, fe);
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int f0 = 2 * i, f1 = 2 * i + 1;
        const float v0 = f0 < mlp::NFEAT ? (fe[f0] - W->mean[f0]) * W->istd[f0] : 0.f;
        const float v1 = f1 < mlp::NFEAT ? (fe[f1] - W->mean[f1]) * W->istd[f1] : 0.f;
        const __bf16 h0 = (__bf16)v0, h1 = (__bf16)v1;
        xw[i] = (int)((uint32_t)__builtin_bit_cast(uint16_t, h0) | ((uint32_t)__builtin_bit_cast(uint16_t, h1) << 16));
      }
    }
    float yo[NF];
#pragma unroll
    for (int i = 0; i < NF; ++i) yo[i] = 0.f;
    const int nlive = min(64, nc - base);
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      if (16 * t >= nlive) break;
      // K group 0 lanes take the features of the tile's contact c16
      mlp::bf16x8 x = {};
      const int src = (16 * t + c16) << 2;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int v = __builtin_amdgcn_ds_bpermute(src, xw[i]);
        if (kg == 0) {
          x[2 * i] = __builtin_bit_cast(__bf16, (uint16_t)(v & 0xFFFF));
          x[2 * i + 1] = __builtin_bit_cast(__bf16, (uint16_t)((uint32_t)v >> 16));
        }
      }
      const mlp::f32x4 y = mlp::forward_tile_k32(W, x);
      // outputs back to the contact lanes of the tile: output o of contact c16
      // sits in lane 16 (o / 4) + c16, register o % 4
#pragma unroll
      for (int q = 0; q < (NF + 3) / 4; ++q) {
        const int from = (16 * q + c16) << 2;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          if (4 * q + r >= NF) break;
          const float v = __int_as_float(__builtin_amdgcn_ds_bpermute(from, __float_as_int(y[r])));
          if ((lane >> 4) == t) yo[4 * q + r] = v;
        }
      }
    }
    int kA = nb, kB = nb;
    float4 WA = make_float4(0.f, 0.f, 0.f, 0.f), WB = WA;
    float2 WA2 = make_float2(0.f, 0.f), WB2 = WA2;
    int eF = FX_ZERO;
    if (live) {
      const ContactKin K = contact_kin(cn, cp, gB, gM, bC, bV, bW);
      const float A = heuristic_gain(K.phi, K.trs, P);
      float Af[NF];
#pragma unroll
      for (int i = 0; i < NF; ++i) Af[i] = A;
      const float c0 = -P.k_user * K.phi;
      float lam[NF], Gl[NF], ll[NF];
      facet_impulses<CONDIM>(Af, K, aa, c0, lam);
#pragma unroll
      for (int i = 0; i < NF; ++i) Gl[i] = A * __expf(fminf(fmaxf(yo[i], -mlp::CLIP), mlp::CLIP));
      facet_impulses<CONDIM>(Gl, K, aa, c0, ll);
      const bool keep = learned_ok<NF>(lam, ll, dot(K.n, K.vrel), K.phi, K.trs, P.h, P.mlp_margin);
      if (keep) {
#pragma unroll
        for (int i = 0; i < NF; ++i) lam[i] = ll[i];
      }
      if (a.x_fallback) a.x_fallback[cbase + k] = keep ? 0 : 1;
      V3 f, tc;
      contact_wrench<CONDIM>(lam, K, f, tc);
      eF = fx_exp(f.x, f.y, f.z);
      if (K.bb >= 0) {
        const V3 Tb = CONDIM >= 4 ? cross(K.rb, f) + tc : cross(K.rb, f);
        kB = K.bb;
        WB = make_float4(f.x, f.y, f.z, Tb.x);
        WB2 = make_float2(Tb.y, Tb.z);
      }
      if (K.ba >= 0) {
        const V3 Ta = CONDIM >= 4 ? cross(K.ra, f) + tc : cross(K.ra, f);
        kA = K.ba;
        WA = make_float4(-f.x, -f.y, -f.z, -Ta.x);
        WA2 = make_float2(-Ta.y, -Ta.z);
      }
      export_contact<NF>(a, cbase + k, K, lam);
      export_training<CONDIM>(a, cbase + k, K, A, aa, P);
    }
    if (kA < nb) {
      atomicMax(fxE + kA, eF);
      atomicMax(fxE + nbp + kA, fx_exp(WA.w, WA2.x, WA2.y));
    }
    if (kB < nb) {
      atomicMax(fxE + kB, eF);
      atomicMax(fxE + nbp + kB, fx_exp(WB.w, WB2.x, WB2.y));
    }
    wave_sync();
    if (kA < nb) fx_add<64>(fxQ, fxE, kA, nbp, WA, WA2);
    if (kB < nb) fx_add<64>(fxQ, fxE, kB, nbp, WB, WB2);
    wave_sync();
#pragma unroll
    for (int j = 0; j < NBL; ++j) {
      const int b = lane + 64 * j;
      const int ef = b < nb ? fxE[b] : FX_EMPTY, et = b < nb ? fxE[nbp + b] : FX_EMPTY;
      if (ef != FX_EMPTY) {
        const unsigned long long q0 = fxQ[b], q1 = fxQ[nbp + b], q2 = fxQ[2 * nbp + b];
        F[j].x += fx_value<64>(fx_lo(q0), ef);
        F[j].y += fx_value<64>(fx_hi(q0), ef);
        F[j].z += fx_value<64>(fx_lo(q1), ef);
        T[j].x += fx_value<64>(fx_hi(q1), et);
        T[j].y += fx_value<64>(fx_lo(q2), et);
        T[j].z += fx_value<64>(fx_hi(q2), et);
        fxQ[b] = 0ull; fxQ[nbp + b] = 0ull; fxQ[2 * nbp + b] = 0ull;
        fxE[b] = FX_EMPTY;
        fxE[nbp + b] = FX_EMPTY;
      }
    }
    wave_sync();
    cn = nn;
    cp = np;
  }

#pragma unroll
  for (int j = 0; j < NBL; ++j) {
    const int b = lane + 64 * j;
    if (b >= nb) continue;
    float qo[7], vo[6];
    free_body_correct(bC[b], bV[b], bW[b], bI0[b], bI1[b], F[j], T[j], qb[j], P, qo, vo);
    float *qd = a.q_out + (size_t)w * a.nq + 7 * b, *vd = a.v_out + (size_t)w * a.nv + 6 * b;
#pragma unroll
    for (int i = 0; i < 7; ++i) qd[i] = qo[i];
#pragma unroll
    for (int i = 0; i < 6; ++i) vd[i] = vo[i];
  }
}

template <int NBL>
static hipError_t launch_resolve_learned_n(const ResolveArgs &a, int nworld, size_t lds, hipStream_t s) {
  constexpr int kLearnWorlds = learn_worlds(NBL);
  const dim3 grid((nworld + kLearnWorlds - 1) / kLearnWorlds), block(64 * kLearnWorlds);
  switch (a.condim) {
    case 1: hipLaunchKernelGGL((resolve_learned_kernel<1, NBL>), grid, block, lds, s, a); break;
    case 3: hipLaunchKernelGGL((resolve_learned_kernel<3, NBL>), grid, block, lds, s, a); break;
    case 4: hipLaunchKernelGGL((resolve_learned_kernel<4, NBL>), grid, block, lds, s, a); break;
    case 6: hipLaunchKernelGGL((resolve_learned_kernel<6, NBL>), grid, block, lds, s, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_resolve_learned(const ResolveArgs &a, int nworld, size_t lds, hipStream_t s) {
  if (a.nsub > 0 || !a.mlp_img || a.act || a.nb > 128 || a.nworld != nworld) return hipErrorInvalidValue;
  return a.nb > 64 ? launch_resolve_learned_n<2>(a, nworld, lds, s) : launch_resolve_learned_n<1>(a, nworld, lds, s);
}

template <int CONDIM>
static hipError_t launch_resolve_free_c(const ResolveArgs &a, int nworld, int block, size_t lds, hipStream_t s) {
  switch (block) {
    case 64: hipLaunchKernelGGL((resolve_free_kernel<CONDIM, 64>), dim3(nworld), dim3(64), lds, s, a); break;
    case 128: hipLaunchKernelGGL((resolve_free_kernel<CONDIM, 128>), dim3(nworld), dim3(128), lds, s, a); break;
    case 256: hipLaunchKernelGGL((resolve_free_kernel<CONDIM, 256>), dim3(nworld), dim3(256), lds, s, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_resolve_free(const ResolveArgs &a, int nworld, int block, size_t lds, hipStream_t s) {
  if (a.nsub > 0 || a.mlp || a.act || a.nb > block) return hipErrorInvalidValue;
  switch (a.condim) {
    case 1: return launch_resolve_free_c<1>(a, nworld, block, lds, s);
    case 3: return launch_resolve_free_c<3>(a, nworld, block, lds, s);
    case 4: return launch_resolve_free_c<4>(a, nworld, block, lds, s);
    case 6: return launch_resolve_free_c<6>(a, nworld, block, lds, s);
    default: return hipErrorInvalidValue;
  }
}

// ====================================================================
// rollout: T steps of one world per workgroup, state and contacts in LDS
// ====================================================================
size_t rollout_lds_bytes(int nq, int nv, int nb, int ng, int norient, int nsub, int nsph, int art_floats, int cap) {
  const size_t c = collide_region_bytes(nb, ng, norient, nsub, nsph);
  const size_t r = resolve_region_bytes(nb, ng, nsub, art_floats);
  return sizeof(float) * (pad4(nq) + 2 * (size_t)pad4(nv)) + 2 * sizeof(float4) * (size_t)cap + (c > r ? c : r);
}

template <int CONDIM, int BS, bool ART>
__global__ __launch_bounds__(BS, 2) void rollout_kernel(RolloutArgs r) {
  extern __shared__ float4 lds[];
  const CollideArgs &ca = r.c;
  const ResolveArgs &ra = r.s;
  const int w = blockIdx.x, tid = threadIdx.x;
  const int nq = ra.nq, nv = ra.nv, nb = ra.nb, nw = r.nworld, cap = r.cap;
  float *sq = reinterpret_cast<float *>(lds);
  float *sv = sq + pad4(nq);
  float *st = sv + pad4(nv);
  float4 *cn = reinterpret_cast<float4 *>(st + pad4(nv));
  float4 *cp = cn + cap;
  float4 *reg = cp + cap;  // shared by the narrow phase and the resolution
  {
    const float *qw = r.q0 + (size_t)w * nq, *vw = r.v0 + (size_t)w * nv;
    for (int i = tid; i < nq; i += BS) sq[i] = qw[i];
    for (int i = tid; i < nv; i += BS) sv[i] = vw[i];
  }
  const uint32_t nxt = tid < ca.nslot_pre ? ca.slots[tid] : 0u;
  for (int t = 0; t < r.T; ++t) {
    if (r.tau_seq) {
      const float *tw = r.tau_seq + ((size_t)t * nw + w) * nv;
      for (int i = tid; i < nv; i += BS) st[i] = tw[i];
    } else {
      for (int i = tid; i < nv; i += BS) st[i] = 0.f;
    }
    float4 mi0 = make_float4(1.f, 1.f, 1.f, 1.f);
    if (tid < nb) mi0 = ra.bmi[(size_t)w * nb + tid];
    __syncthreads();
    const int found = collide_world<BS, ART>(ca, w, sq, reg, cn, cp, cap, nxt);
    const int nc = found < cap ? found : cap;
    float4 c0n = make_float4(0.f, 0.f, 0.f, 0.f), c0p = c0n;
    if (tid < nc) {
      c0n = cn[tid];
      c0p = cp[tid];
    }
    if (tid == 0 && r.ncon_traj) r.ncon_traj[(size_t)t * nw + w] = nc;
    if (tid == 0 && r.over_traj) r.over_traj[(size_t)t * nw + w] = found - nc;
    __syncthreads();
    resolve_world<CONDIM, BS, ART>(ra, w, sq, sv, st, cn, cp, nc, c0n, c0p, mi0, reg, 0);
    float *qo = r.q_traj + ((size_t)(t + 1) * nw + w) * nq, *vo = r.v_traj + ((size_t)(t + 1) * nw + w) * nv;
    for (int i = tid; i < nq; i += BS) qo[i] = sq[i];
    for (int i = tid; i < nv; i += BS) vo[i] = sv[i];
  }
}

// ---- rollout of worlds of free bodies: one persistent one-wave workgroup per
// world, lane b stepping body b.  Each step runs the narrow phase
// (collide_world, contacts to the model's global workspace, read back by the
// same workgroup) and the free-body resolution (resolve_free_world), whose
// per-body inputs the lane reads back from its own trajectory row (nothing
// held across the narrow phase, which keeps the kernel within 128 registers).  The q row the narrow phase reads
// lives in LDS inside the narrow phase's candidate list, which nothing uses
// between the end of a resolution and the geoms' world poses of the next
// step; the LDS footprint is then the larger of the two regions (8.6 KB for
// 64 spheres), so as many worlds share a CU as with step launches, and the
// worlds drift out of step with each other, overlapping one world's loads with
// another's arithmetic.  Same device functions, arithmetic and summation
// order as cf_step: the trajectories equal T steps to float32 rounding (bit
// for bit where the compilations fuse the same multiplies and adds).
__host__ __device__ inline size_t collide_cand_offset(int ng, int norient) {
  return (sizeof(Pose<double>) + sizeof(Pose<float>)) * (size_t)norient + sizeof(float4) * (size_t)ng +
         2 * sizeof(int) * (size_t)pad4(ng);
}

size_t rollout_free_lds_bytes(int nb, int ng, int norient, int nsph) {
  const size_t c = collide_region_bytes(nb, ng, norient, 0, nsph), r = resolve_free_lds_bytes(nb, ng);
  return c > r ? c : r;
}

bool rollout_free_fits(int nq, int nb) { return nb >= 1 && nb <= 64 && nq <= kCandCap; }

// WAVES: resident waves per SIMD the registers are sized for (3: no spills,
// twelve worlds per CU; 4: sixteen, a few spills).
template <int CONDIM, int WAVES>
__global__ __launch_bounds__(64, WAVES) void rollout_free_kernel(RolloutArgs r) {
  constexpr int BS = 64;
  extern __shared__ float4 lds[];
  const CollideArgs &ca = r.c;
  const ResolveArgs &ra = r.s;
  const int w = blockIdx.x, tid = threadIdx.x;
  const int nq = ra.nq, nv = ra.nv, nb = ra.nb, nw = r.nworld, cap = r.cap;
  const bool own = tid < nb;
  float *sq = reinterpret_cast<float *>(reinterpret_cast<char *>(lds) + collide_cand_offset(ca.ng, ca.norient));
  for (int i = tid; i < nq; i += BS) sq[i] = r.q_traj[(size_t)w * nq + i];  // row 0 = the initial state
  const uint32_t nxt = tid < ca.nslot_pre ? ca.slots[tid] : 0u;
  for (int t = 0; t < r.T; ++t) {
    // the world and lane index, opaque to the compiler in each step, so
    // addresses are formed where they are used instead of being hoisted out
    // of the step loop and held (and spilled) across it
    int wt = w, tl = tid;
    asm volatile("" : "+s"(wt), "+v"(tl));
    const size_t cbase = (size_t)wt * cap;
    __syncthreads();  // the q row is complete
    const int found = collide_world<BS, false>(ca, wt, sq, lds, ca.cnp + cbase, ca.cpos + cbase, cap, nxt, nullptr, tl);
    const int nc = found < cap ? found : cap;
    if (tid == 0 && r.ncon_traj) r.ncon_traj[(size_t)t * nw + wt] = nc;
    if (tid == 0 && r.over_traj) r.over_traj[(size_t)t * nw + wt] = found - nc;
    // the lane's body from trajectory row t (its own writes of the previous
    // step), and the contact records this workgroup wrote (visible after
    // collide_world's barrier); every lane loads (a lane without a body
    // rereads the last one, a lane past the count the last record or record
    // 0 of the world's capacity, and ignores it), so no wait separates them
    const int r0 = tid < nc ? tid : (nc > 0 ? nc - 1 : 0), bl = own ? tl : nb - 1;
    const float4 cn = ca.cnp[cbase + r0], cp = ca.cpos[cbase + r0];
    float qb[7], vb[6], tb[6];
    {
      const float *qs = r.q_traj + ((size_t)t * nw + wt) * nq + 7 * bl;
      const float *vs = r.v_traj + ((size_t)t * nw + wt) * nv + 6 * bl;
#pragma unroll
      for (int i = 0; i < 7; ++i) qb[i] = qs[i];
#pragma unroll
      for (int i = 0; i < 6; ++i) vb[i] = vs[i];
    }
    const float4 mi = ra.bmi[(size_t)wt * nb + bl];
#pragma unroll
    for (int i = 0; i < 6; ++i) tb[i] = 0.f;
    if (r.tau_seq) {
      const float *ts = r.tau_seq + ((size_t)t * nw + wt) * nv + 6 * bl;
#pragma unroll
      for (int i = 0; i < 6; ++i) tb[i] = ts[i];
    }
    float qo[7], vo[6];
    resolve_free_world<CONDIM, BS>(ra, wt, qb, vb, tb, mi, nc, cn, cp, ca.cnp + cbase, ca.cpos + cbase, 0, lds, qo, vo, tl);
    if (own) {
      float *qd = r.q_traj + ((size_t)(t + 1) * nw + wt) * nq + 7 * tid;
      float *vd = r.v_traj + ((size_t)(t + 1) * nw + wt) * nv + 6 * tid;
#pragma unroll
      for (int i = 0; i < 7; ++i) {
        qd[i] = qo[i];
        sq[7 * tid + i] = qo[i];
      }
#pragma unroll
      for (int i = 0; i < 6; ++i) vd[i] = vo[i];
    }
  }
}

template <int WAVES>
static hipError_t launch_rollout_free_w(const RolloutArgs &a, size_t lds, hipStream_t s) {
  switch (a.s.condim) {
    case 1: hipLaunchKernelGGL((rollout_free_kernel<1, WAVES>), dim3(a.nworld), dim3(64), lds, s, a); break;
    case 3: hipLaunchKernelGGL((rollout_free_kernel<3, WAVES>), dim3(a.nworld), dim3(64), lds, s, a); break;
    case 4: hipLaunchKernelGGL((rollout_free_kernel<4, WAVES>), dim3(a.nworld), dim3(64), lds, s, a); break;
    case 6: hipLaunchKernelGGL((rollout_free_kernel<6, WAVES>), dim3(a.nworld), dim3(64), lds, s, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_rollout_free(const RolloutArgs &a, size_t lds, int waves, hipStream_t s) {
  if (a.s.nsub > 0 || a.s.act || a.s.mlp || !rollout_free_fits(a.s.nq, a.s.nb) || a.cap != a.s.ncon_max)
    return hipErrorInvalidValue;
  return waves == 3 ? launch_rollout_free_w<3>(a, lds, s) : launch_rollout_free_w<4>(a, lds, s);
}

template <int CONDIM, bool ART>
static hipError_t launch_rollout_b(const RolloutArgs &a, int block, size_t lds, hipStream_t s) {
  switch (block) {
    case 64: hipLaunchKernelGGL((rollout_kernel<CONDIM, 64, ART>), dim3(a.nworld), dim3(64), lds, s, a); break;
    case 128: hipLaunchKernelGGL((rollout_kernel<CONDIM, 128, ART>), dim3(a.nworld), dim3(128), lds, s, a); break;
    case 256: hipLaunchKernelGGL((rollout_kernel<CONDIM, 256, ART>), dim3(a.nworld), dim3(256), lds, s, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int CONDIM>
static hipError_t launch_rollout_c(const RolloutArgs &a, int block, size_t lds, hipStream_t s) {
  return a.s.nsub > 0 ? launch_rollout_b<CONDIM, true>(a, block, lds, s)
                      : launch_rollout_b<CONDIM, false>(a, block, lds, s);
}

hipError_t launch_rollout(const RolloutArgs &a, int block, size_t lds, hipStream_t s) {
  switch (a.s.condim) {
    case 1: return launch_rollout_c<1>(a, block, lds, s);
    case 3: return launch_rollout_c<3>(a, block, lds, s);
    case 4: return launch_rollout_c<4>(a, block, lds, s);
    case 6: return launch_rollout_c<6>(a, block, lds, s);
    default: return hipErrorInvalidValue;
  }
}

template <int CONDIM, bool ART, bool LEARN>
static hipError_t launch_resolve_b(const ResolveArgs &a, int nworld, int block, size_t lds, hipStream_t s) {
  switch (block) {
    case 64: hipLaunchKernelGGL((resolve_kernel<CONDIM, 64, ART, LEARN>), dim3(nworld), dim3(64), lds, s, a); break;
    case 128: hipLaunchKernelGGL((resolve_kernel<CONDIM, 128, ART, LEARN>), dim3(nworld), dim3(128), lds, s, a); break;
    case 256: hipLaunchKernelGGL((resolve_kernel<CONDIM, 256, ART, LEARN>), dim3(nworld), dim3(256), lds, s, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int CONDIM>
static hipError_t launch_resolve_c(const ResolveArgs &a, int nworld, int block, size_t lds, hipStream_t s) {
  if (a.mlp) return a.nsub > 0 ? hipErrorInvalidValue : launch_resolve_b<CONDIM, false, true>(a, nworld, block, lds, s);
  return a.nsub > 0 ? launch_resolve_b<CONDIM, true, false>(a, nworld, block, lds, s)
                    : launch_resolve_b<CONDIM, false, false>(a, nworld, block, lds, s);
}

hipError_t launch_resolve(const ResolveArgs &a, int nworld, int block, size_t lds, hipStream_t s) {
  switch (a.condim) {
    case 1: return launch_resolve_c<1>(a, nworld, block, lds, s);
    case 3: return launch_resolve_c<3>(a, nworld, block, lds, s);
    case 4: return launch_resolve_c<4>(a, nworld, block, lds, s);
    case 6: return launch_resolve_c<6>(a, nworld, block, lds, s);
    default: return hipErrorInvalidValue;
  }
}

// ====================================================================
// adjoint of one step (free bodies)
// ====================================================================
// Segmented per-body sum of NV4 float4 per lane and side.  Lane tid holds
// keys kA, kB (nb = none) and payloads pa[i * BS + tid], pb[i * BS + tid] in
// LDS; each key's entries are summed by one leader lane in lane order (side a
// before side b) and the waves add their sums to acc[i * nb + key] in wave
// order: a fixed summation order, no atomics.  All threads call it; it ends
// with a barrier.
template <int BS, int NV4>
__device__ void body_segment_sum(int kA, int kB, const float4 *pa, const float4 *pb, float4 *acc, int nb,
                                 int nbits) {
  constexpr int NW = BS / 64;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const unsigned long long below = lanes_below(lane);
  unsigned long long eAA = ~0ull, eAB = ~0ull, eBA = ~0ull, eBB = ~0ull;
  for (int i = 0; i < nbits; ++i) {
    const bool a1 = (kA >> i) & 1, b1 = (kB >> i) & 1;
    const unsigned long long bA = __ballot(a1), bBv = __ballot(b1);
    eAA &= a1 ? bA : ~bA;
    eAB &= a1 ? bBv : ~bBv;
    eBA &= b1 ? bA : ~bA;
    eBB &= b1 ? bBv : ~bBv;
  }
  const bool leadA = kA < nb && !(eAA & below);
  const bool leadB = kB < nb && !eBA && !(eBB & below);
  const int wb0 = wave * 64;
  float4 SA[NV4], SB[NV4];
#pragma unroll
  for (int i = 0; i < NV4; ++i) SA[i] = SB[i] = make_float4(0.f, 0.f, 0.f, 0.f);
  auto add = [](float4 &x, float4 y) { x.x += y.x; x.y += y.y; x.z += y.z; x.w += y.w; };
  if (leadA) {
    for (unsigned long long m = eAA; m; m &= m - 1) {
      const int l = wb0 + __ffsll((unsigned long long)m) - 1;
#pragma unroll
      for (int i = 0; i < NV4; ++i) add(SA[i], pa[i * BS + l]);
    }
    for (unsigned long long m = eAB; m; m &= m - 1) {
      const int l = wb0 + __ffsll((unsigned long long)m) - 1;
#pragma unroll
      for (int i = 0; i < NV4; ++i) add(SA[i], pb[i * BS + l]);
    }
  }
  if (leadB) {
    for (unsigned long long m = eBB; m; m &= m - 1) {
      const int l = wb0 + __ffsll((unsigned long long)m) - 1;
#pragma unroll
      for (int i = 0; i < NV4; ++i) add(SB[i], pb[i * BS + l]);
    }
  }
#pragma unroll
  for (int wv = 0; wv < NW; ++wv) {
    if (wave == wv) {
#pragma unroll
      for (int i = 0; i < NV4; ++i) {
        if (leadA) add(acc[i * nb + kA], SA[i]);
        if (leadB) add(acc[i * nb + kB], SB[i]);
      }
    }
    __syncthreads();
  }
}

// LDS beyond the resolution's: the q row before the step; per body the
// accumulated adjoints (4 float4: x_bar | psi_bar | v_s bar | w_s bar | trace
// bar packed), the adjoints of the contact force and torque sums and the
// direct quaternion adjoint; per lane two packed 4-float4 payloads; the
// articulated subtrees' reverse-pass work blocks.
size_t backward_lds_bytes(int nq, int nv, int nb, int ng, int block, int nsub, int art_floats, int artb_floats) {
  return resolve_lds_bytes(nq, nv, nb, ng, nsub, art_floats) + sizeof(float) * pad4(nq) +
         sizeof(float4) * (7 * (size_t)nb + 8 * (size_t)block) + sizeof(float) * (size_t)pad4(artb_floats);
}

// Reverse-pass work block of a subtree (floats): theta bar, v_s bar, y, w,
// tau bar, theta-dot bar, c bar, u [nd each]; M bar [nd nd]; J bar [nbs][6][nd];
// a free root's direct quaternion adjoint [4]; dual joint values and rates
// [2 nd], dual root pose [12] and the dual workspace of subtree_phi.
int art_backward_floats(int nd, int nbs) {
  return nd * nd + 8 * nd + 6 * nd * nbs + 4 + 2 * (2 * nd + 12 + artadj::phi_work(nbs, nd));
}

// ---- articulated subtrees in the reverse pass (hinge and slide joints below a
// fixed or free root; one lane per subtree).  A free root's 6 dofs (linear and
// angular velocity, world frame) carry the adjoints of its frame origin and of
// a world-frame rotation increment.  Forward block (art_predict/art_correct):
// L [nd nd] | z = M^-1 p [nd] | v_s [nd] | cols [6 nd] | idx [nd].
struct ArtRev {
  float *thb, *vsb, *y, *wv, *tb, *thdb, *cb, *u, *Mb, *Jb, *qb;
  artadj::Du<float> *th, *thd, *rp, *rr, *wk;
};
__device__ inline ArtRev art_rev_block(float *bw, int nd, int nbs) {
  ArtRev r;
  r.thb = bw; r.vsb = r.thb + nd; r.y = r.vsb + nd; r.wv = r.y + nd; r.tb = r.wv + nd; r.thdb = r.tb + nd;
  r.cb = r.thdb + nd; r.u = r.cb + nd; r.Mb = r.u + nd; r.Jb = r.Mb + nd * nd; r.qb = r.Jb + 6 * nd * nbs;
  r.th = reinterpret_cast<artadj::Du<float> *>(r.qb + 4);
  r.thd = r.th + nd; r.rp = r.thd + nd; r.rr = r.rp + 3; r.wk = r.rr + 9;
  return r;
}

// Reverse of the subtree's integration theta+ = theta + h v+ and correction
// v+ = v_s + M^-1 p, p = sum_b J_b^T W_b: joint adjoints seeded from the
// outputs' adjoints, y = M^-1 (v+ bar), body wrench adjoints W_b bar = J_b y
// for the contact reverse, M bar = -y z^T, J_b bar = W_b y^T.
__device__ void art_rev_correct(const SubTree S, const BodyC *B, const float4 *bC, const float4 *bO,
                                const float4 *bAx, const float4 *accF, const float4 *accT, float *blk, float *bw,
                                const float *q0, const float *vp, const float *gqo, const float *gvo, float4 *bFb,
                                float4 *bTb, float4 *bQb, float4 *acc, int nb, float h) {
  const int nd = S.nd, d0 = S.d0;
  float *L = blk, *z = L + nd * nd, *cols = z + 2 * nd;
  int *idx = reinterpret_cast<int *>(cols + 6 * nd);
  const ArtRev R = art_rev_block(bw, nd, S.nb);
  for (int i = 0; i < 4; ++i) R.qb[i] = 0.f;
  for (int k = 0; k < S.nb; ++k) {
    const BodyC bc = B[S.b0 + k];
    const int x = bc.dadr - d0;
    if (bc.jnt == kFree) {
      // q+ = (o + h v+, normalise(exp(h w+) q)): the free-body update with no
      // wrench (the correction went through M^-1 p)
      adj::BodyUpdate<float> U;
      U.m = 1.f; U.d[0] = U.d[1] = U.d[2] = 1.f;
      for (int i = 0; i < 4; ++i) U.q[i] = q0[bc.qadr + 3 + i];
      U.x = adj::vec(q0[bc.qadr], q0[bc.qadr + 1], q0[bc.qadr + 2]);
      U.vs = adj::vec(vp[bc.dadr], vp[bc.dadr + 1], vp[bc.dadr + 2]);
      U.ws = adj::vec(vp[bc.dadr + 3], vp[bc.dadr + 4], vp[bc.dadr + 5]);
      U.F = U.Tq = adj::vec(0.f, 0.f, 0.f);
      U.h = h;
      adj::Vec<float> xpb = adj::vec(0.f, 0.f, 0.f), vpb = xpb, wpb = xpb;
      float qpb[4] = {0.f, 0.f, 0.f, 0.f};
      if (gqo) {
        xpb = adj::vec(gqo[bc.qadr], gqo[bc.qadr + 1], gqo[bc.qadr + 2]);
        for (int i = 0; i < 4; ++i) qpb[i] = gqo[bc.qadr + 3 + i];
      }
      if (gvo) {
        vpb = adj::vec(gvo[bc.dadr], gvo[bc.dadr + 1], gvo[bc.dadr + 2]);
        wpb = adj::vec(gvo[bc.dadr + 3], gvo[bc.dadr + 4], gvo[bc.dadr + 5]);
      }
      adj::Vec<float> xb, vsb, wsb, Fb, Tb, psi = adj::vec(0.f, 0.f, 0.f);
      adj::update_vjp(U, xpb, qpb, vpb, wpb, xb, R.qb, vsb, wsb, Fb, Tb, psi);
      const float tq[6] = {xb.x, xb.y, xb.z, 0.f, 0.f, 0.f}, tv[6] = {vsb.x, vsb.y, vsb.z, wsb.x, wsb.y, wsb.z};
      for (int e = 0; e < 6; ++e) {
        R.thb[x + e] = tq[e];
        R.vsb[x + e] = tv[e];
      }
    } else {
      const float tq = gqo ? gqo[bc.qadr] : 0.f;
      const float tv = gvo ? gvo[d0 + x] : 0.f;
      R.thb[x] = tq;
      R.vsb[x] = tv + h * tq;
    }
  }
  for (int i = 0; i < nd; ++i) {
    R.y[i] = R.vsb[i];
    R.thdb[i] = 0.f;
  }
  fwd_solve(L, nd, R.y);
  bwd_solve(L, nd, R.y);
  for (int i = 0; i < nd; ++i)
    for (int j = 0; j < nd; ++j) R.Mb[i * nd + j] = -R.y[i] * z[j];
  for (int i = 0; i < 6 * nd * S.nb; ++i) R.Jb[i] = 0.f;
  for (int k = 0; k < S.nb; ++k) {
    const int b = S.b0 + k;
    const int n = chain_cols(b, d0, B, bO, bAx, bC, cols, idx);
    const float W[6] = {accF[b].x, accF[b].y, accF[b].z, accT[b].x, accT[b].y, accT[b].z};
    float Wb[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    float *Jb = R.Jb + 6 * nd * k;
    for (int x = 0; x < n; ++x) {
      const int i = idx[x];
      for (int r = 0; r < 6; ++r) {
        Wb[r] += cols[6 * x + r] * R.y[i];
        Jb[r * nd + i] += W[r] * R.y[i];
      }
    }
    bFb[b] = make_float4(Wb[0], Wb[1], Wb[2], 0.f);
    bTb[b] = make_float4(Wb[3], Wb[4], Wb[5], 0.f);
    bQb[b] = make_float4(0.f, 0.f, 0.f, 0.f);
    for (int i = 0; i < 4; ++i) acc[i * nb + b] = make_float4(0.f, 0.f, 0.f, 0.f);
  }
}

// Reverse of the subtree's smooth prediction v_s = thd + h M^-1 (tau - c) and of
// its bodies' COM poses, velocities at v_s and traces, given the per-body
// adjoints from the contacts (acc: x bar, rotation-increment bar, v bar, w bar,
// trace bar).  Writes the joint adjoints to gq/gv/gt (the LDS rows of the
// outputs).  act: position actuators or null.
__device__ void art_rev_predict(const SubTree S, const BodyC *B, const float4 *bmi, const float4 *bC,
                                const float4 *bO, const float4 *bAx, float *blk, float *bw, const float4 *acc, int nb,
                                const float *q0, const float *v0, const float4 *act, const Params &P, float *gq,
                                float *gv, float *gt) {
  const int nd = S.nd, d0 = S.d0;
  float *L = blk, *vs = L + nd * nd + nd, *cols = vs + nd;
  int *idx = reinterpret_cast<int *>(cols + 6 * nd);
  const ArtRev R = art_rev_block(bw, nd, S.nb);
  for (int k = 0; k < S.nb; ++k) {
    const int b = S.b0 + k;
    const int n = chain_cols(b, d0, B, bO, bAx, bC, cols, idx);
    const float4 A0 = acc[b], A1 = acc[nb + b], A2 = acc[2 * nb + b], A3 = acc[3 * nb + b];
    const float xb[3] = {A0.x, A0.y, A0.z}, pb[3] = {A0.w, A1.x, A1.y};
    const float g6[6] = {A1.z, A1.w, A2.x, A2.y, A2.z, A2.w};  // v bar, w bar at v_s
    const float trb = A3.x;
    float *Jb = R.Jb + 6 * nd * k;
    for (int x = 0; x < n; ++x) {
      const int i = idx[x];
      const float *c = cols + 6 * x;
      R.thb[i] += c[0] * xb[0] + c[1] * xb[1] + c[2] * xb[2] + c[3] * pb[0] + c[4] * pb[1] + c[5] * pb[2];
      float sv = 0.f;
      for (int r = 0; r < 6; ++r) {
        sv += c[r] * g6[r];
        Jb[r * nd + idx[x]] += g6[r] * vs[idx[x]];
      }
      R.vsb[i] += sv;
    }
    if (trb != 0.f) {
      // tr_b = sum_r J_r M^-1 J_r^T over the COM rows r
      for (int r = 0; r < 3; ++r) {
        for (int i = 0; i < nd; ++i) R.u[i] = 0.f;
        for (int x = 0; x < n; ++x) R.u[idx[x]] = cols[6 * x + r];
        fwd_solve(L, nd, R.u);
        bwd_solve(L, nd, R.u);
        for (int x = 0; x < n; ++x) Jb[r * nd + idx[x]] += 2.f * trb * R.u[idx[x]];
        for (int i = 0; i < nd; ++i)
          for (int j = 0; j < nd; ++j) R.Mb[i * nd + j] -= trb * R.u[i] * R.u[j];
      }
    }
  }
  // v_s = thd + h s, s = M^-1 (tau - c): w = h M^-1 (v_s bar), M bar -= w s^T, c bar = -w, tau bar = w
  for (int i = 0; i < nd; ++i) R.wv[i] = P.h * R.vsb[i];
  fwd_solve(L, nd, R.wv);
  bwd_solve(L, nd, R.wv);
  for (int i = 0; i < nd; ++i) {
    const float si = (vs[i] - v0[d0 + i]) / P.h;
    for (int j = 0; j < nd; ++j) R.Mb[j * nd + i] -= R.wv[j] * si;
    R.cb[i] = -R.wv[i];
    R.thdb[i] += R.vsb[i];
    float tbar = R.wv[i];
    if (act) {  // tau = kp (u - theta) - kd theta-dot for an actuated dof
      const float4 c = act[d0 + i];
      if (__float_as_int(c.z) >= 0) {
        R.thb[i] -= c.x * tbar;
        R.thdb[i] -= c.y * tbar;
        tbar *= c.x;
      }
    }
    R.tb[i] = tbar;
  }
  // M, c and the J_b as functions of the joints: gradient of Phi by dual passes
  const BodyC rb = B[S.b0];
  const bool free_root = rb.jnt == kFree;
  float R0[9] = {1.f, 0.f, 0.f, 0.f, 1.f, 0.f, 0.f, 0.f, 1.f}, p0[3] = {0.f, 0.f, 0.f};
  if (free_root) {
    quat_to_rot<float>(q0[rb.qadr + 3], q0[rb.qadr + 4], q0[rb.qadr + 5], q0[rb.qadr + 6], R0);
    for (int i = 0; i < 3; ++i) p0[i] = q0[rb.qadr + i];
  }
  for (int k = 0; k < 2 * nd; ++k) {
    const int kd = k < nd ? k : -1;  // joint direction (a free root: translation, then rotation)
    for (int i = 0; i < nd; ++i) R.thd[i] = artadj::du<float>(v0[d0 + i], k == nd + i ? 1.f : 0.f);
    for (int b = S.b0; b < S.b0 + S.nb; ++b) {
      const BodyC bc = B[b];
      if (bc.jnt == kFree) continue;
      const int x = bc.dadr - d0;
      R.th[x] = artadj::du<float>(q0[bc.qadr], kd == x ? 1.f : 0.f);
    }
    for (int i = 0; i < 3; ++i) R.rp[i] = artadj::du<float>(p0[i], free_root && kd == i ? 1.f : 0.f);
    // rotation increment about world axis e: d R = [e]x R
    const int e = free_root && kd >= 3 && kd < 6 ? kd - 3 : -1;
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        float d = 0.f;
        if (e >= 0) {
          const int i1 = (e + 1) % 3, i2 = (e + 2) % 3;  // ([e]x R)_ij = e x (column j of R)
          d = i == i1 ? -R0[3 * i2 + j] : i == i2 ? R0[3 * i1 + j] : 0.f;
        }
        R.rr[3 * i + j] = artadj::du<float>(R0[3 * i + j], d);
      }
    const float d = artadj::subtree_phi<artadj::Du<float>>(B, S.b0, S.nb, d0, nd, bmi, R.th, R.thd, R.rp, R.rr, P.gx,
                                                          P.gy, P.gz, R.Mb, R.cb, R.Jb, R.wk).d;
    if (k < nd) R.thb[k] += d;
    else R.thdb[k - nd] += d;
  }
  for (int b = S.b0; b < S.b0 + S.nb; ++b) {
    const BodyC bc = B[b];
    const int x = bc.dadr - d0;
    if (bc.jnt == kFree) {
      float qb[4] = {R.qb[0], R.qb[1], R.qb[2], R.qb[3]};
      const float qq[4] = {q0[bc.qadr + 3], q0[bc.qadr + 4], q0[bc.qadr + 5], q0[bc.qadr + 6]};
      adj::quat_grad_from_psi(qq, adj::vec(R.thb[x + 3], R.thb[x + 4], R.thb[x + 5]), qb);
      for (int i = 0; i < 3; ++i) gq[bc.qadr + i] = R.thb[x + i];
      for (int i = 0; i < 4; ++i) gq[bc.qadr + 3 + i] = qb[i];
      for (int i = 0; i < 6; ++i) {
        gv[d0 + x + i] = R.thdb[x + i];
        gt[d0 + x + i] = R.tb[x + i];
      }
    } else {
      gq[bc.qadr] = R.thb[x];
      gv[d0 + x] = R.thdb[x];
      gt[d0 + x] = R.tb[x];
    }
  }
}

// Reverse of one step of world w: the forward step is recomputed in LDS
// (same code as the resolution kernel, so the same contact set, facet
// activity and branches), then the adjoints run backwards through
// integration and correction (per body), the contacts' impulses, wrenches and
// geometry (lane per contact, per-body segmented sums) and the smooth
// prediction (per body).  Contacts come from the collision kernel's workspace.
// NET: learned gains (models of free bodies), recomputed and differentiated
// through the float32 network.
template <int CONDIM, int BS, bool ART, bool NET>
__global__ __launch_bounds__(BS) void backward_kernel(BackwardArgs b) {
  using adj::Vec;
  using adj::vec;
  constexpr int NF = CONDIM == 1 ? 1 : CONDIM == 3 ? 4 : CONDIM == 4 ? 6 : 10;
  const ResolveArgs &a = b.s;
  extern __shared__ float4 lds[];
  const int w = blockIdx.x, tid = threadIdx.x;
  const int nq = a.nq, nv = a.nv, nb = a.nb, ng = a.ng;
  float *sq = reinterpret_cast<float *>(lds);
  float *sv = sq + pad4(nq);
  float *st = sv + pad4(nv);
  float4 *reg = reinterpret_cast<float4 *>(st + pad4(nv));
  float *sq0 = reinterpret_cast<float *>(reg + resolve_region_bytes(nb, ng, ART ? a.nsub : 0, ART ? a.art_floats : 0) /
                                                      sizeof(float4));
  float4 *acc = reinterpret_cast<float4 *>(sq0 + pad4(nq));  // [4][nb]
  float4 *bFb = acc + 4 * nb, *bTb = bFb + nb, *bQb = bTb + nb;
  float4 *pay = bQb + nb;  // [2][4][BS]
  float *artb = reinterpret_cast<float *>(pay + 8 * BS);  // subtree reverse blocks

  // ---- forward step, kept in LDS
  const size_t cbase = (size_t)w * a.ncon_max;
  const int nc = a.ncon[w];
  float4 c0n = make_float4(0.f, 0.f, 0.f, 0.f), c0p = c0n;
  if (tid < a.ncon_max) {
    c0n = a.cnp[cbase + tid];
    c0p = a.cpos[cbase + tid];
  }
  float4 mi0 = make_float4(1.f, 1.f, 1.f, 1.f);
  if (tid < nb) mi0 = a.bmi[(size_t)w * nb + tid];
  const float *qw = a.q + (size_t)w * nq, *vw = a.v + (size_t)w * nv;
  for (int i = tid; i < nq; i += BS) sq[i] = sq0[i] = qw[i];
  for (int i = tid; i < nv; i += BS) sv[i] = vw[i];
  if (a.tau) {
    const float *tw = a.tau + (size_t)w * nv;
    for (int i = tid; i < nv; i += BS) st[i] = tw[i];
  } else {
    for (int i = tid; i < nv; i += BS) st[i] = 0.f;
  }
  resolve_world<CONDIM, BS, ART, false, NET>(a, w, sq, sv, st, a.cnp + cbase, a.cpos + cbase, nc, c0n, c0p, mi0,
                                             reg, cbase);
  const ResolveRegion RR = resolve_region(reg, nb, ng);
  const Params P = a.p;
  auto xyz = [](float4 f) { return vec(f.x, f.y, f.z); };
  // Rotation and frame origin of body bi at the start of the step (a free body:
  // its quaternion and COM; an articulated body: the forward kinematics in LDS).
  auto body_frame = [&](int bi, float *R, Vec<float> &org) {
    if (ART && !a.body[bi].fast) {
      for (int r = 0; r < 3; ++r) {
        const float4 row = RR.bR[3 * bi + r];
        R[3 * r] = row.x; R[3 * r + 1] = row.y; R[3 * r + 2] = row.z;
      }
      org = xyz(RR.bO[bi]);
    } else {
      adj::rot_of_quat(sq0 + a.body[bi].qadr + 3, R);
      org = xyz(RR.bC[bi]);
    }
  };

  // ---- reverse of integration and correction, per free body and per subtree
  if (ART)
  for (int si = tid; si < a.nsub; si += BS) {
    const SubTree S = a.sub[si];
    art_rev_correct(S, a.body, RR.bC, RR.bO, RR.bAx, RR.accF, RR.accT, RR.art + S.lofs, artb + S.bofs, sq0, sv,
                    b.gq_out ? b.gq_out + (size_t)w * nq : nullptr, b.gv_out ? b.gv_out + (size_t)w * nv : nullptr,
                    bFb, bTb, bQb, acc, nb, P.h);
  }
  for (int bi = tid; bi < nb; bi += BS) {
    const BodyC bc = a.body[bi];
    if (ART && !bc.fast) continue;
    const float4 mi = a.bmi[(size_t)w * nb + bi];
    adj::BodyUpdate<float> U;
    U.m = mi.x; U.d[0] = mi.y; U.d[1] = mi.z; U.d[2] = mi.w;
    for (int i = 0; i < 4; ++i) U.q[i] = sq0[bc.qadr + 3 + i];
    U.x = xyz(RR.bC[bi]); U.vs = xyz(RR.bV[bi]); U.ws = xyz(RR.bW[bi]);
    U.F = xyz(RR.accF[bi]); U.Tq = xyz(RR.accT[bi]); U.h = P.h;
    Vec<float> xpb = vec(0.f, 0.f, 0.f), vpb = xpb, wpb = xpb;
    float qpb[4] = {0.f, 0.f, 0.f, 0.f};
    if (b.gq_out) {
      const float *g = b.gq_out + (size_t)w * nq + bc.qadr;
      xpb = vec(g[0], g[1], g[2]);
      for (int i = 0; i < 4; ++i) qpb[i] = g[3 + i];
    }
    if (b.gv_out) {
      const float *g = b.gv_out + (size_t)w * nv + bc.dadr;
      vpb = vec(g[0], g[1], g[2]);
      wpb = vec(g[3], g[4], g[5]);
    }
    Vec<float> xb, vsb, wsb, Fb, Tb, psi = vec(0.f, 0.f, 0.f);
    float qb[4] = {0.f, 0.f, 0.f, 0.f};
    adj::update_vjp(U, xpb, qpb, vpb, wpb, xb, qb, vsb, wsb, Fb, Tb, psi);
    acc[bi] = make_float4(xb.x, xb.y, xb.z, psi.x);
    acc[nb + bi] = make_float4(psi.y, psi.z, vsb.x, vsb.y);
    acc[2 * nb + bi] = make_float4(vsb.z, wsb.x, wsb.y, wsb.z);
    acc[3 * nb + bi] = make_float4(0.f, 0.f, 0.f, 0.f);
    bFb[bi] = make_float4(Fb.x, Fb.y, Fb.z, 0.f);
    bTb[bi] = make_float4(Tb.x, Tb.y, Tb.z, 0.f);
    bQb[bi] = make_float4(qb[0], qb[1], qb[2], qb[3]);
  }
  __syncthreads();

  // ---- reverse of the contacts: lane per contact, per-body sums
  const adj::Impedance<float> I{P.r_min, P.r_max, P.width, P.mid, P.power};
  for (int base = 0; base < nc; base += BS) {
    const int k = base + tid;
    int kA = nb, kB = nb;
    float4 pA[4], pB[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) pA[i] = pB[i] = make_float4(0.f, 0.f, 0.f, 0.f);
    if (k < nc) {
      const float4 cn = a.cnp[cbase + k], cp = a.cpos[cbase + k];
      const uint32_t sl = __float_as_uint(cp.w);
      const int ga = slot_ga(sl), gb = slot_gb(sl);
      const uint32_t type = slot_type(sl);
      const int ba = RR.gB[ga], bbd = RR.gB[gb];
      adj::ContactIn<float> C;
      const Vec<float> Z = vec(0.f, 0.f, 0.f);
      C.n = vec(cn.x, cn.y, cn.z); C.p = vec(cp.x, cp.y, cp.z); C.phi = cn.w;
      C.xa = C.va = C.wa = C.xb = C.vb = C.wb = Z;
      C.has_a = ba >= 0; C.has_b = bbd >= 0;
      C.trs = 0.f;
      if (ba >= 0) { C.xa = xyz(RR.bC[ba]); C.va = xyz(RR.bV[ba]); C.wa = xyz(RR.bW[ba]); C.trs += RR.bV[ba].w; }
      if (bbd >= 0) { C.xb = xyz(RR.bC[bbd]); C.vb = xyz(RR.bV[bbd]); C.wb = xyz(RR.bW[bbd]); C.trs += RR.bV[bbd].w; }
      const float4 ma = RR.gM[ga], mb = RR.gM[gb];
      C.mut = fmaxf(ma.x, mb.x); C.mutor = fmaxf(ma.y, mb.y); C.murol = fmaxf(ma.z, mb.z);
      C.h = P.h; C.k = P.k_user; C.d = P.d_user;
      C.diag = P.imp_diag != 0;
      C.net = NET ? a.mlp : nullptr;  // learned gains (free bodies): the float32 network
      C.margin = P.mlp_margin;
      C.ima = C.imb = 0.f;
      if (C.diag) {  // free bodies only: 1/m and the world inverse inertia at the step's start
        auto inertia = [&](int bi, float *S) {
          const float4 I0 = RR.bI0[bi], I1 = RR.bI1[bi];
          S[0] = I0.x; S[1] = I0.y; S[2] = I0.z; S[3] = I0.w; S[4] = I1.x; S[5] = I1.y;
        };
        if (ba >= 0) { C.ima = RR.bC[ba].w; inertia(ba, C.Sa); }
        if (bbd >= 0) { C.imb = RR.bC[bbd].w; inertia(bbd, C.Sb); }
      }
      const Vec<float> Fab = ba >= 0 ? xyz(bFb[ba]) : Z, Tab = ba >= 0 ? xyz(bTb[ba]) : Z;
      const Vec<float> Fbb = bbd >= 0 ? xyz(bFb[bbd]) : Z, Tbb = bbd >= 0 ? xyz(bTb[bbd]) : Z;
      adj::ContactBar<float> o;
      adj::contact_vjp<NF, float, NET>(C, I, Fab, Tab, Fbb, Tbb, o);
      // geometry: contact (n, phi, p) from the two geoms' poses
      Vec<float> xab = o.xa, xbb = o.xb, psa = Z, psb = Z;
      const float4 gda = a.gdat[(size_t)w * ng + ga], gdb = a.gdat[(size_t)w * ng + gb];
      const Vec<float> n = C.n, p = C.p;
      const float phi = C.phi;
      if (type == kSphereSphere) {
        const float ra = gda.x, rb = gdb.x;
        Vec<float> cab, cbb;
        adj::sphere_pair_vjp(n, phi, ra, rb, o.n, o.phi, o.p, cab, cbb);
        const Vec<float> ca = p - (ra + 0.5f * phi) * n;
        const Vec<float> cb = ca + (phi + ra + rb) * n;
        xab = xab + cab; psa = adj::cross(ca - C.xa, cab);
        xbb = xbb + cbb; psb = adj::cross(cb - C.xb, cbb);
      } else if (type == kBoxSphere || type == kBoxCapsule) {
        // box (geom a) against the sphere centre or capsule end c of geom b; the
        // region of c (axes outside the box) picks the face plane, the edge
        // line or the corner the forward gap was measured from
        const float rad = gdb.x;
        const Vec<float> c = p + (rad + 0.5f * phi) * n;
        float Rb[9] = {1.f, 0.f, 0.f, 0.f, 1.f, 0.f, 0.f, 0.f, 1.f}, Rg[9], RX[9];
        Vec<float> xo = Z;
        if (ba >= 0) body_frame(ba, Rb, xo);
        const float4 o4 = b.gpos[(size_t)w * b.gpos_ws + ga], g4 = b.gquat[(size_t)w * b.gquat_ws + ga];
        quat_to_rot<float>(g4.x, g4.y, g4.z, g4.w, Rg);
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
          for (int j = 0; j < 3; ++j) RX[3 * i + j] = Rb[3 * i] * Rg[j] + Rb[3 * i + 1] * Rg[3 + j] + Rb[3 * i + 2] * Rg[6 + j];
        const Vec<float> X = xo + vec(Rb[0] * o4.x + Rb[1] * o4.y + Rb[2] * o4.z, Rb[3] * o4.x + Rb[4] * o4.y + Rb[5] * o4.z,
                                      Rb[6] * o4.x + Rb[7] * o4.y + Rb[8] * o4.z);
        const float hs[3] = {gda.x, gda.y, gda.z};
        const Vec<float> dc = c - X;
        Vec<float> corner = X, e0 = X, u = Z;
        int nout = 0;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          const Vec<float> col = vec(RX[k], RX[3 + k], RX[6 + k]);
          const float l = adj::dot(col, dc);
          const float sh = (l >= 0.f ? hs[k] : -hs[k]);
          corner = corner + sh * col;
          if (fabsf(l) > hs[k]) {
            ++nout;
            e0 = e0 + sh * col;
          } else {
            u = col;
          }
        }
        Vec<float> cbar, abx, abp;
        if (nout <= 1) {  // face or inside: the plane of the face
          const Vec<float> pp = c - (phi + rad) * n;
          Vec<float> ppb, nnb;
          adj::plane_point_vjp(pp, n, c, rad, phi, o.n, o.phi, o.p, cbar, ppb, nnb);
          abx = ppb;
          abp = adj::cross(pp - C.xa, ppb) + adj::cross(n, nnb);
        } else if (nout == 2) {  // edge along the axis where c lies within the box
          Vec<float> e0b, ub;
          adj::line_point_vjp(e0, u, c, rad, n, phi, o.n, o.phi, o.p, cbar, e0b, ub);
          abx = e0b;
          abp = adj::cross(e0 - C.xa, e0b) + adj::cross(u, ub);
        } else {  // corner: a sphere of radius 0
          Vec<float> cab;
          adj::sphere_pair_vjp(n, phi, 0.f, rad, o.n, o.phi, o.p, cab, cbar);
          abx = cab;
          abp = adj::cross(corner - C.xa, cab);
        }
        xbb = xbb + cbar; psb = adj::cross(c - C.xb, cbar);
        if (ba >= 0) { xab = xab + abx; psa = abp; }
      } else {
        const float rad = type == kPlaneBox ? 0.f : gdb.x;
        const Vec<float> c = p + (rad + 0.5f * phi) * n;
        Vec<float> pp = c - (phi + rad) * n;  // a point of the plane (static plane: n is fixed)
        if (ba >= 0) {
          float R[9];
          Vec<float> xo;
          body_frame(ba, R, xo);
          const float4 o4 = b.gpos[(size_t)w * b.gpos_ws + ga];
          pp = xo + vec(R[0] * o4.x + R[1] * o4.y + R[2] * o4.z, R[3] * o4.x + R[4] * o4.y + R[5] * o4.z,
                        R[6] * o4.x + R[7] * o4.y + R[8] * o4.z);
        }
        Vec<float> cbar, ppb, nnb;
        adj::plane_point_vjp(pp, n, c, rad, phi, o.n, o.phi, o.p, cbar, ppb, nnb);
        xbb = xbb + cbar; psb = adj::cross(c - C.xb, cbar);
        if (ba >= 0) { xab = xab + ppb; psa = adj::cross(pp - C.xa, ppb) + adj::cross(n, nnb); }
      }
      psa = psa + o.psa;
      psb = psb + o.psb;
      if (ba >= 0) {
        kA = ba;
        pA[0] = make_float4(xab.x, xab.y, xab.z, psa.x);
        pA[1] = make_float4(psa.y, psa.z, o.va.x, o.va.y);
        pA[2] = make_float4(o.va.z, o.wa.x, o.wa.y, o.wa.z);
        pA[3] = make_float4(o.trs, 0.f, 0.f, 0.f);
      }
      if (bbd >= 0) {
        kB = bbd;
        pB[0] = make_float4(xbb.x, xbb.y, xbb.z, psb.x);
        pB[1] = make_float4(psb.y, psb.z, o.vb.x, o.vb.y);
        pB[2] = make_float4(o.vb.z, o.wb.x, o.wb.y, o.wb.z);
        pB[3] = make_float4(o.trs, 0.f, 0.f, 0.f);
      }
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      pay[i * BS + tid] = pA[i];
      pay[(4 + i) * BS + tid] = pB[i];
    }
    __syncthreads();
    body_segment_sum<BS, 4>(kA, kB, pay, pay + 4 * BS, acc, nb, a.nbits);
  }

  // ---- reverse of the smooth prediction, per free body and per subtree;
  // adjoint rows staged in LDS
  if (ART)
  for (int si = tid; si < a.nsub; si += BS) {
    const SubTree S = a.sub[si];
    art_rev_predict(S, a.body, a.bmi + (size_t)w * nb, RR.bC, RR.bO, RR.bAx, RR.art + S.lofs, artb + S.bofs, acc, nb,
                    sq0, vw, a.act, P, sq, sv, st);
  }
  for (int bi = tid; bi < nb; bi += BS) {
    const BodyC bc = a.body[bi];
    if (ART && !bc.fast) continue;
    const float4 mi = a.bmi[(size_t)w * nb + bi];
    adj::BodyPredict<float> B;
    B.m = mi.x; B.d[0] = mi.y; B.d[1] = mi.z; B.d[2] = mi.w;
    for (int i = 0; i < 4; ++i) B.q[i] = sq0[bc.qadr + 3 + i];
    const float *v0 = vw + bc.dadr, *t0 = st + bc.dadr;
    B.v = vec(v0[0], v0[1], v0[2]); B.w = vec(v0[3], v0[4], v0[5]);
    B.f = vec(t0[0], t0[1], t0[2]); B.t = vec(t0[3], t0[4], t0[5]);
    B.g = vec(P.gx, P.gy, P.gz); B.h = P.h;
    const float4 A0 = acc[bi], A1 = acc[nb + bi], A2 = acc[2 * nb + bi];
    const Vec<float> xb = vec(A0.x, A0.y, A0.z), vsb = vec(A1.z, A1.w, A2.x), wsb = vec(A2.y, A2.z, A2.w);
    Vec<float> psi = vec(A0.w, A1.x, A1.y);
    Vec<float> vb, wb, fb, tb;
    adj::predict_vjp(B, vsb, wsb, vb, wb, fb, tb, psi);
    const float4 Q = bQb[bi];
    float qb[4] = {Q.x, Q.y, Q.z, Q.w};
    adj::quat_grad_from_psi(B.q, psi, qb);
    float *gqr = sq + bc.qadr, *gvr = sv + bc.dadr, *gtr = st + bc.dadr;
    gqr[0] = xb.x; gqr[1] = xb.y; gqr[2] = xb.z;
    for (int i = 0; i < 4; ++i) gqr[3 + i] = qb[i];
    gvr[0] = vb.x; gvr[1] = vb.y; gvr[2] = vb.z; gvr[3] = wb.x; gvr[4] = wb.y; gvr[5] = wb.z;
    gtr[0] = fb.x; gtr[1] = fb.y; gtr[2] = fb.z; gtr[3] = tb.x; gtr[4] = tb.y; gtr[5] = tb.z;
  }
  __syncthreads();
  float *gqw = b.gq + (size_t)w * nq, *gvw = b.gv + (size_t)w * nv;
  for (int i = tid; i < nq; i += BS) gqw[i] = sq[i];
  for (int i = tid; i < nv; i += BS) gvw[i] = sv[i];
  if (b.gtau) {
    float *gtw = b.gtau + (size_t)w * nv;
    for (int i = tid; i < nv; i += BS) gtw[i] = st[i];
  }
}

template <int CONDIM, bool ART, bool NET>
static hipError_t launch_backward_c(const BackwardArgs &a, int nworld, int block, size_t lds, hipStream_t s) {
  switch (block) {
    case 64: hipLaunchKernelGGL((backward_kernel<CONDIM, 64, ART, NET>), dim3(nworld), dim3(64), lds, s, a); break;
    case 128: hipLaunchKernelGGL((backward_kernel<CONDIM, 128, ART, NET>), dim3(nworld), dim3(128), lds, s, a); break;
    case 256: hipLaunchKernelGGL((backward_kernel<CONDIM, 256, ART, NET>), dim3(nworld), dim3(256), lds, s, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <bool ART, bool NET>
static hipError_t launch_backward_a(const BackwardArgs &a, int nworld, int block, size_t lds, hipStream_t s) {
  switch (a.s.condim) {
    case 1: return launch_backward_c<1, ART, NET>(a, nworld, block, lds, s);
    case 3: return launch_backward_c<3, ART, NET>(a, nworld, block, lds, s);
    case 4: return launch_backward_c<4, ART, NET>(a, nworld, block, lds, s);
    case 6: return launch_backward_c<6, ART, NET>(a, nworld, block, lds, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_backward(const BackwardArgs &a, int nworld, int block, size_t lds, hipStream_t s) {
  if (a.s.nsub > 0) return a.s.mlp ? hipErrorInvalidValue : launch_backward_a<true, false>(a, nworld, block, lds, s);
  return a.s.mlp ? launch_backward_a<false, true>(a, nworld, block, lds, s)
                 : launch_backward_a<false, false>(a, nworld, block, lds, s);
}

}  // namespace cf
