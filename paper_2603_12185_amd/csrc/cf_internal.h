// cf_internal.h - kernel argument blocks shared by the host library and the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cf {

constexpr int kBlock = 256;            // threads per workgroup (4 wave64)
constexpr int kWaves = kBlock / 64;

// Candidate sub-contact ("slot"), packed in 32 bits:
//   bits  0..12 geom a, 13..25 geom b, 26..28 sub-contact index, 29..30 pair type.
enum PairType : uint32_t { kPlaneSphere = 0, kPlaneCapsule = 1, kPlaneBox = 2, kSphereSphere = 3 };
constexpr int kMaxGeom = 8191;

__host__ __device__ inline uint32_t slot_pack(int ga, int gb, int sub, uint32_t type) {
  return (uint32_t)ga | ((uint32_t)gb << 13) | ((uint32_t)sub << 26) | (type << 29);
}
__host__ __device__ inline int slot_ga(uint32_t s) { return (int)(s & 0x1FFFu); }
__host__ __device__ inline int slot_gb(uint32_t s) { return (int)((s >> 13) & 0x1FFFu); }
__host__ __device__ inline int slot_sub(uint32_t s) { return (int)((s >> 26) & 7u); }
__host__ __device__ inline uint32_t slot_type(uint32_t s) { return (s >> 29) & 3u; }

// Per-model solver constants (passed by value).
struct Params {
  float h, k_user, d_user, margin;
  float gx, gy, gz;
  float r_min, r_max, width, mid, power;
};

// Collision kernel: one workgroup per world.
struct CollideArgs {
  const float *q;               // [nw][nq]
  const float4 *gpos;           // [nw|1][ng] (x, y, z, -)
  const float4 *gquat;          // [nw|1][ng] (w, x, y, z)
  const float4 *gdat;           // [nw][ng] (size0, size1, size2, mu_t)
  const int *gbody;             // [ng]
  const uint32_t *slots;        // [nslot] canonical order
  float4 *cnp;                  // [nw][ncon_max] (n.x, n.y, n.z, phi)
  float4 *cpos;                 // [nw][ncon_max] (p.x, p.y, p.z, slot bits)
  int *ncon, *overflow;         // [nw] model workspace
  int *ncon_out, *overflow_out; // [nw] caller copies or null
  int nq, nb, ng, nslot, ncon_max;
  int gpos_ws, gquat_ws;        // world stride in elements (0 = shared by all worlds)
  float margin;
};

// Resolution kernel: one workgroup per world.
struct ResolveArgs {
  const float *q, *v, *tau;     // [nw][nq], [nw][nv], [nw][nv] or null
  float *q_out, *v_out;
  const float4 *bmi;            // [nw][nb] (m, Ixx, Iyy, Izz) principal inertia
  const float4 *gdat;           // [nw][ng] (size0, size1, size2, mu_t)
  const float2 *gfr2;           // [nw][ng] (mu_tor, mu_rol) or null when condim < 4
  const int *gbody;             // [ng]
  const float4 *cnp, *cpos;     // contact workspace
  const int *ncon;              // [nw]
  // optional exports (device, caller-owned), may be null
  int *x_geom, *x_sub;
  float *x_dist, *x_pos, *x_frame, *x_imp;
  int nq, nv, nb, ng, ncon_max, condim, nfacet, nbits;
  Params p;
};

size_t collide_lds_bytes(int nq, int ng);
size_t resolve_lds_bytes(int nq, int nv, int nb, int ng);
hipError_t launch_collide(const CollideArgs &a, int nworld, size_t lds, hipStream_t s);
hipError_t launch_resolve(const ResolveArgs &a, int nworld, size_t lds, hipStream_t s);

}  // namespace cf
