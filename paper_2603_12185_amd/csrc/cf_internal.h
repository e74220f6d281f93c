// cf_internal.h - kernel argument blocks shared by the host library and the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cf {

// Workgroup sizes the kernels are instantiated for (one world per workgroup).
constexpr int kBlockSizes[3] = {64, 128, 256};
constexpr int kCandCap = 1024;         // LDS candidate list of the narrow phase

// Candidate sub-contact ("slot"), packed in 32 bits:
//   bits  0..12 geom a, 13..25 geom b, 26..28 sub-contact index, 29..31 pair type.
// Geom a is the plane of a plane pair and the box of a box pair.
enum PairType : uint32_t {
  kPlaneSphere = 0, kPlaneCapsule = 1, kPlaneBox = 2, kSphereSphere = 3, kBoxSphere = 4, kBoxCapsule = 5
};
constexpr int kMaxGeom = 8191;

__host__ __device__ inline uint32_t slot_pack(int ga, int gb, int sub, uint32_t type) {
  return (uint32_t)ga | ((uint32_t)gb << 13) | ((uint32_t)sub << 26) | (type << 29);
}
__host__ __device__ inline int slot_ga(uint32_t s) { return (int)(s & 0x1FFFu); }
__host__ __device__ inline int slot_gb(uint32_t s) { return (int)((s >> 13) & 0x1FFFu); }
__host__ __device__ inline int slot_sub(uint32_t s) { return (int)((s >> 26) & 7u); }
__host__ __device__ inline uint32_t slot_type(uint32_t s) { return (s >> 29) & 7u; }

// Joint types (same values as the C ABI).
enum JointType : int { kFree = 0, kHinge = 1, kSlide = 2 };

// Per-body constants shared by all worlds.
struct BodyC {
  float4 pos;    // body frame origin in the parent frame at q = 0 (x, y, z, -)
  float4 quat;   // body frame orientation in the parent frame, (w,x,y,z) in (x,y,z,w)
  float4 axis;   // unit hinge/slide axis in the body frame
  float4 ipos;   // centre of mass in the body frame
  int parent, jnt, qadr, dadr;
  int fast;      // 1: free body without children (closed-form path), 0: articulated subtree member
  int pad[3];
};

// Articulated subtree (a root body with its descendants, contiguous in body
// and dof order): bodies [b0, b0+nb), dofs [d0, d0+nd), float offset of its
// LDS work block (nd*nd + 9*nd floats).
struct SubTree {
  int b0, nb, d0, nd, lofs;  // bodies [b0, b0+nb), dofs [d0, d0+nd), forward work block offset
  int bofs;                  // reverse-pass work block offset (cf_step_backward)
  int small;                 // 1: at most kSmallSub hinge/slide bodies (one dof each), registers path
  // small subtrees: body b0 + k has q index q0 + k and dof d0 + k; chain bits
  // 4k..4k+3 mark body k and its ancestors (bit j: body b0 + j), bit 16 + k a
  // hinge (else a slide)
  int chain, q0;
  // exact diagonal impedance only: float offset (in the same LDS region as
  // the work blocks, after all of them) of the bodies' L^-1 J_b^T blocks,
  // 6 nd floats per body, column r of body b0 + k at yofs + (6 k + r) nd
  int yofs;
};
constexpr int kSmallSub = 4;

// Joint constants of a hinge or slide body (model constants, computed on the
// host in float64): with B the body frame's rotation in its parent at q = 0
// and a its unit joint axis, the rotation in the parent at joint position th
// is Mk + cos(th) Mc + sin(th) Ms (hinge: B Rot(a, th) = B a a^T +
// cos(th) B (1 - a a^T) + sin(th) B [a]x; slide: Mk = B, Mc = Ms = 0), the
// origin in the parent frame is lp + th s (s = B a for a slide, 0 for a hinge)
// and the joint axis in the parent frame is Ba = B a.
template <class T>
struct JointK {
  T Mk[9], Mc[9], Ms[9], lp[3], s[3], Ba[3];
};
constexpr int kMaxSubDof = 32;

// Per-model solver constants (passed by value).
struct Params {
  float h, k_user, d_user, margin;
  float gx, gy, gz;
  float r_min, r_max, width, mid, power;
  float inv_width, inv_mid, inv_1mmid;  // 1/width, 1/mid, 1/(1 - mid)
  int power2;                           // power == 2: gamma uses squares
  int imp_diag;                         // 1: exact diagonal impedance per facet
  float mlp_margin;                     // fallback margin of the learned gains (m)
};

// Collision kernel: one workgroup per world.
struct CollideArgs {
  const float *q;               // [nw][nq]
  const float4 *gpos;           // [nw|1][ng] (x, y, z, -)
  const float4 *gquat;          // [nw|1][ng] (w, x, y, z)
  const float4 *gdat;           // [nw][ng] (size0, size1, size2, mu_t)
  const int *gbody;             // [ng]
  const int *gorient;           // [ng] index among oriented geoms, -1 for a plain sphere
  const BodyC *body;            // [nb]
  const SubTree *sub;           // [nsub]
  const uint32_t *slots;        // [nslot] canonical order
  float4 *cnp;                  // [nw][ncon_max] (n.x, n.y, n.z, phi)
  float4 *cpos;                 // [nw][ncon_max] (p.x, p.y, p.z, slot bits)
  int *ncon, *overflow;         // [nw] model workspace
  int *ncon_out, *overflow_out; // [nw] caller copies or null
  int nq, nb, ng, norient, nslot, ncon_max, nsub;
  int nslot_pre;                // slots tested one by one (all of them when nsph = 0)
  int sph0, nsph;               // sphere block: geoms [sph0, sph0 + nsph), pairs tested row-wise
  int npl;                      // > 0: geoms [0, npl) are static planes whose slots are their rows against the block
  int sph_mfma;                 // 1: block of <= 64 spheres on pairwise different bodies, margin >= 0 (MFMA masks)
  const JointK<double> *jk;     // [nb] joint constants (articulated models)
  float4 *frames;               // [nw][nb][5] frames of small-subtree bodies (origin, joint axis,
                                // rotation rows) for the resolution, or null
  int gpos_ws, gquat_ws;        // world stride in elements (0 = shared by all worlds)
  float margin;
};

// Resolution kernel: one workgroup per world.
struct ResolveArgs {
  const float *q, *v, *tau;     // [nw][nq], [nw][nv], [nw][nv] or null
  float *q_out, *v_out;
  const float4 *bmi;            // [nw][nb] (m, Ixx, Iyy, Izz) principal inertia
  const float4 *gdat;           // [nw][ng] (size0, size1, size2, mu_t)
  const float *gmu;             // [nw][ng] mu_t alone (what the resolution reads)
  const float2 *gfr2;           // [nw][ng] (mu_tor, mu_rol) or null when condim < 4
  const int *gbody;             // [ng]
  const BodyC *body;            // [nb]
  const SubTree *sub;           // [nsub]
  const float4 *cnp, *cpos;     // contact workspace
  const int *ncon;              // [nw]
  // optional exports (device, caller-owned), may be null
  int *x_geom, *x_sub;
  float *x_dist, *x_pos, *x_frame, *x_imp;
  float *x_feat, *x_target;     // learned-gain training data (free-body models)
  int *x_fallback;              // learned gains: 1 where a contact fell back to the heuristic
  const float *mlp;             // learned-gain network parameters, or null
  const float4 *mlp_img;        // their LDS image (launch_mlp_pack), with mlp
  const float4 *act;            // [nv] position actuators (kp, kd, q index bits, -), or null
  const float4 *frames;         // [nw][nb][5] frames of small-subtree bodies written by the
                                // narrow phase on the same q (CollideArgs::frames), or null
  int nq, nv, nb, ng, ncon_max, condim, nfacet, nbits, nsub, art_floats;
  int nworld;
  Params p;
};

// Fused rollout: T steps per launch, one workgroup per world.
struct RolloutArgs {
  CollideArgs c;                // q, contact workspace and counts unused
  ResolveArgs s;                // q, v, tau, outputs, contact inputs and exports unused
  const float *q0, *v0;         // [nw][nq], [nw][nv]
  const float *tau_seq;         // [T][nw][nv] or null
  float *q_traj, *v_traj;       // [T+1][nw][..]; row 0 written by the host
  int *ncon_traj;               // [T][nw] contacts kept per step, or null
  int *over_traj;               // [T][nw] contacts dropped beyond cap per step, or null
  int T, nworld, cap;           // cap: contacts held per world per step (= ncon_max)
};

// Adjoint of one step (free bodies): one workgroup per world.
struct BackwardArgs {
  ResolveArgs s;                // the step's inputs (q, v, tau), contacts; exports unused
  const float4 *gpos;           // [nw|1][ng] geom offsets in the body frame
  const float4 *gquat;          // [nw|1][ng] geom orientations in the body frame (x, y, z, w) = (w, x, y, z)
  int gpos_ws, gquat_ws;
  const float *gq_out, *gv_out; // [nw][nq], [nw][nv] adjoints of q+, v+ (null = 0)
  float *gq, *gv, *gtau;        // [nw][nq], [nw][nv], [nw][nv] (gtau may be null)
};

// Learned gains: bytes of the network's LDS image, and the kernel writing it
// from the float32 parameters (one workgroup).
size_t mlp_image_bytes();
hipError_t launch_mlp_pack(const float *params, void *img, hipStream_t s);

size_t backward_lds_bytes(int nq, int nv, int nb, int ng, int block, int nsub, int art_floats, int artb_floats);
// Floats of the reverse-pass work block of a subtree with nd dofs and nbs bodies.
int art_backward_floats(int nd, int nbs);
hipError_t launch_backward(const BackwardArgs &a, int nworld, int block, size_t lds, hipStream_t s);

size_t collide_lds_bytes(int nq, int nb, int ng, int norient, int nsub, int nsph);
size_t rollout_lds_bytes(int nq, int nv, int nb, int ng, int norient, int nsub, int nsph, int art_floats, int cap);
hipError_t launch_rollout(const RolloutArgs &a, int block, size_t lds, hipStream_t s);
size_t resolve_lds_bytes(int nq, int nv, int nb, int ng, int nsub, int art_floats);
size_t resolve_learned_lds_bytes(int block);  // extra LDS of the resolution with learned gains
hipError_t launch_collide(const CollideArgs &a, int nworld, int block, size_t lds, hipStream_t s);
hipError_t launch_resolve(const ResolveArgs &a, int nworld, int block, size_t lds, hipStream_t s);
// Resolution of worlds of free bodies (no subtrees, actuators or learned
// gains) with at most `block` bodies, each body's state in its lane.
__host__ __device__ size_t resolve_free_lds_bytes(int nb, int ng);
hipError_t launch_resolve_free(const ResolveArgs &a, int nworld, int block, size_t lds, hipStream_t s);
hipError_t launch_step_free(const CollideArgs &ca, const ResolveArgs &ra, int nworld, size_t lds, hipStream_t s);
hipError_t launch_step_art(const CollideArgs &ca, const ResolveArgs &ra, int nworld, size_t lds, hipStream_t s);
// The same with learned gains (network image of launch_mlp_pack_k32 in
// mlp_img), four worlds of at most 128 free bodies per workgroup.
size_t resolve_learned_k32_lds_bytes(int nb, int ng);
// Rollout of worlds of free bodies (at most 64, q row within the narrow
// phase's candidate list), one persistent one-wave workgroup per world;
// `waves`: 3 (registers for twelve resident worlds per CU, no spills) or 4
// (sixteen).
bool rollout_free_fits(int nq, int nb);
size_t rollout_free_lds_bytes(int nb, int ng, int norient, int nsph);
hipError_t launch_rollout_free(const RolloutArgs &a, size_t lds, int waves, hipStream_t s);
hipError_t launch_resolve_learned(const ResolveArgs &a, int nworld, size_t lds, hipStream_t s);
size_t mlp_image_k32_bytes();
hipError_t launch_mlp_pack_k32(const float *params, void *img, hipStream_t s);

}  // namespace cf
