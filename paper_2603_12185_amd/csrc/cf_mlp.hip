// cf_mlp.hip - training and batch inference of the learned per-contact
// impedance network (layout and forward pass in cf_mlp.h): bf16 MFMA with
// float32 accumulation, mean-squared-error gradient with deterministic
// per-wave partial sums, Adam.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "../../include/cfsim.h"
#include "cf_mlp.h"

namespace cf {
cf_status api_error(cf_status st, const std::string &msg);  // cf_api.hip
}

namespace cf {
namespace mlp {

constexpr int BS = 128;  // two waves per block
constexpr int NWAVE = BS / 64;
constexpr int MAX_GRAD_WAVES = 2048;

__device__ inline bf16x4 cvt4(const float *s) {
  bf16x4 r;
#pragma unroll
  for (int t = 0; t < 4; ++t) r[t] = to_bf16(s[t]);
  return r;
}

__global__ __launch_bounds__(BS) void forward_kernel(const float *p, const float *feats, int n, float *out) {
  __shared__ Weights W;
  stage_weights<BS>(p, &W);
  const int l = threadIdx.x & 63, q = l >> 4, c = l & 15;
  const int wave = blockIdx.x * NWAVE + (threadIdx.x >> 6), nwaves = gridDim.x * NWAVE;
  const int ntile = (n + 15) / 16;
  for (int tile = wave; tile < ntile; tile += nwaves) {
    const int ci = tile * 16 + c;
    const bool valid = ci < n;
    Tile T;
    forward_tile(&W, [&](int t) { return (valid && 4 * q + t < NFEAT) ? feats[(size_t)ci * NIN + 4 * q + t] : 0.f; },
                 T);
    if (valid) {
#pragma unroll
      for (int r = 0; r < 4; ++r) out[(size_t)ci * NOUT + 4 * q + r] = T.y[r];
    }
  }
}

// Per-wave scratch of the backward pass: transposed activations and adjoints
// of one tile, rows = units, 16 contacts per row.
struct Scratch {
  short xs[16 * 16];   // x^T (bf16)
  short a1s[NH * 16];  // a1^T (bf16)
  short a2s[NH * 16];  // a2^T (bf16)
  float dz1s[NH * 16]; // dL/dz1 ^T
  float dz2s[NH * 16]; // dL/dz2 ^T
  float dys[NOUT * 16];// dL/dy ^T
};

// Gradient of L = sum over contacts and the first nout outputs of
// (y - target)^2 / (n nout).  Each wave walks tiles wave, wave + nwaves, ...
// and writes its partial gradient and loss to partial[wave][NPARAM + 1].
__global__ __launch_bounds__(BS) void grad_kernel(const float *p, const float *feats, const float *tgt, int n,
                                                  int nout, float *partial) {
  __shared__ Weights W;
  __shared__ Scratch S[NWAVE];
  stage_weights<BS>(p, &W);
  const int l = threadIdx.x & 63, q = l >> 4, c = l & 15;
  const int wave = blockIdx.x * NWAVE + (threadIdx.x >> 6), nwaves = gridDim.x * NWAVE;
  Scratch &s = S[threadIdx.x >> 6];
  const int ntile = (n + 15) / 16;
  const float sc = 2.0f / ((float)n * (float)nout);
  f32x4 gW1[4], gW2[4][4], gW3[4];
  const f32x4 zero = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    gW1[i] = gW3[i] = zero;
#pragma unroll
    for (int j = 0; j < 4; ++j) gW2[i][j] = zero;
  }
  float gb1 = 0.f, gb2 = 0.f, gb3 = 0.f, lossp = 0.f;
  for (int tile = wave; tile < ntile; tile += nwaves) {
    const int ci = tile * 16 + c;
    const bool valid = ci < n;
    Tile T;
    forward_tile(&W, [&](int t) { return (valid && 4 * q + t < NFEAT) ? feats[(size_t)ci * NIN + 4 * q + t] : 0.f; },
                 T);
#pragma unroll
    for (int t = 0; t < 4; ++t) s.xs[(4 * q + t) * 16 + c] = T.x[t];
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int h = 16 * m + 4 * q + r;
        s.a1s[h * 16 + c] = to_bf16(silu(T.z1[m][r]));
        s.a2s[h * 16 + c] = to_bf16(silu(T.z2[m][r]));
      }
    // dL/dy, transposed: lane holds outputs 4 q + r of contact c
    f32x4 dy;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int o = 4 * q + r;
      const float d = (valid && o < nout) ? T.y[r] - tgt[(size_t)ci * NOUT + o] : 0.f;
      lossp += d * d;
      dy[r] = sc * d;
      s.dys[o * 16 + c] = dy[r];
    }
    bf16x4 dyb;
#pragma unroll
    for (int r = 0; r < 4; ++r) dyb[r] = to_bf16(dy[r]);
    // dz2^T = (W3 dy^T) * silu'(z2)
    f32x4 dz2[4];
    bf16x4 dz2b[4];
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      bf16x4 a;
#pragma unroll
      for (int t = 0; t < 4; ++t) a[t] = W.w3t[(4 * q + t) * NH + 16 * m + c];
      f32x4 acc = mfma(a, dyb, zero);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        dz2[m][r] = acc[r] * dsilu(T.z2[m][r]);
        dz2b[m][r] = to_bf16(dz2[m][r]);
        s.dz2s[(16 * m + 4 * q + r) * 16 + c] = dz2[m][r];
      }
    }
    // dz1^T = (W2 dz2^T) * silu'(z1)
#pragma unroll
    for (int m1 = 0; m1 < 4; ++m1) {
      f32x4 acc = zero;
#pragma unroll
      for (int ks = 0; ks < 4; ++ks) {
        bf16x4 a;
#pragma unroll
        for (int t = 0; t < 4; ++t) a[t] = W.w2t[(16 * ks + 4 * q + t) * NH + 16 * m1 + c];
        acc = mfma(a, dz2b[ks], acc);
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) s.dz1s[(16 * m1 + 4 * q + r) * 16 + c] = acc[r] * dsilu(T.z1[m1][r]);
    }
    __builtin_amdgcn_wave_barrier();
    // weight gradients over the tile's 16 contacts (K = contacts)
    const bf16x4 bdy = cvt4(s.dys + c * 16 + 4 * q);
#pragma unroll
    for (int m = 0; m < 4; ++m) gW3[m] = mfma(lds4(s.a2s + (16 * m + c) * 16 + 4 * q), bdy, gW3[m]);
#pragma unroll
    for (int mj = 0; mj < 4; ++mj) {
      const bf16x4 bz = cvt4(s.dz2s + (16 * mj + c) * 16 + 4 * q);
#pragma unroll
      for (int mi = 0; mi < 4; ++mi) gW2[mi][mj] = mfma(lds4(s.a1s + (16 * mi + c) * 16 + 4 * q), bz, gW2[mi][mj]);
    }
    const bf16x4 ax = lds4(s.xs + c * 16 + 4 * q);
#pragma unroll
    for (int mj = 0; mj < 4; ++mj) gW1[mj] = mfma(ax, cvt4(s.dz1s + (16 * mj + c) * 16 + 4 * q), gW1[mj]);
    // bias gradients: lane l sums unit l over the tile's contacts
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      gb1 += s.dz1s[l * 16 + k];
      gb2 += s.dz2s[l * 16 + k];
      if (l < NOUT) gb3 += s.dys[l * 16 + k];
    }
    __builtin_amdgcn_wave_barrier();
  }
  float *P = partial + (size_t)wave * (NPARAM + 1);
  for (int i = l; i < OFF_W1; i += 64) P[i] = 0.f;
#pragma unroll
  for (int mj = 0; mj < 4; ++mj)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int f = 4 * q + r;
      if (f < NIN) P[OFF_W1 + f * NH + 16 * mj + c] = gW1[mj][r];
    }
#pragma unroll
  for (int mi = 0; mi < 4; ++mi)
#pragma unroll
    for (int mj = 0; mj < 4; ++mj)
#pragma unroll
      for (int r = 0; r < 4; ++r) P[OFF_W2 + (16 * mi + 4 * q + r) * NH + 16 * mj + c] = gW2[mi][mj][r];
#pragma unroll
  for (int m = 0; m < 4; ++m)
#pragma unroll
    for (int r = 0; r < 4; ++r) P[OFF_W3 + (16 * m + 4 * q + r) * NOUT + c] = gW3[m][r];
  P[OFF_B1 + l] = gb1;
  P[OFF_B2 + l] = gb2;
  if (l < NOUT) P[OFF_B3 + l] = gb3;
  for (int off = 32; off > 0; off >>= 1) lossp += __shfl_xor(lossp, off);
  if (l == 0) P[NPARAM] = lossp / ((float)n * (float)nout);
}

// grad[i] (and the loss at i = NPARAM) = sum over waves in wave order.
__global__ void reduce_kernel(const float *partial, int nwaves, float *grad, float *loss) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i > NPARAM) return;
  float acc = 0.f;
  for (int w = 0; w < nwaves; ++w) acc += partial[(size_t)w * (NPARAM + 1) + i];
  if (i < NPARAM) grad[i] = acc;
  else if (loss) *loss = acc;
}

__global__ void adam_kernel(float *p, float *m, float *v, const float *g, float lr, float bc1, float bc2) {
  const int i = TRAIN_FROM + blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= NPARAM) return;
  const float gi = g[i];
  const float mi = 0.9f * m[i] + 0.1f * gi;
  const float vi = 0.999f * v[i] + 0.001f * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / bc1) / (sqrtf(vi / bc2) + 1e-8f);
}

static int grad_waves(int n) {
  const int ntile = (n + 15) / 16;
  int w = (ntile + 1) / 2;
  if (w > MAX_GRAD_WAVES) w = MAX_GRAD_WAVES;
  if (w < NWAVE) w = NWAVE;
  return (w + NWAVE - 1) / NWAVE * NWAVE;
}

// The network's LDS image (layout of Weights: bf16 transposed weights, float32
// biases and normalisation) written once per step from the float32 parameters,
// so each workgroup of the resolution copies it instead of converting.
__global__ __launch_bounds__(256) void pack_kernel(const float *p, Weights *img) { stage_weights<256>(p, img); }

// The resolution's K = 32 image (WeightsK32), written once per step.
__global__ __launch_bounds__(256) void pack_k32_kernel(const float *p, WeightsK32 *img) {
  pack_weights_k32<256>(p, img);
}

}  // namespace mlp

size_t mlp_image_bytes() { return sizeof(mlp::Weights); }
size_t mlp_image_k32_bytes() { return sizeof(mlp::WeightsK32); }

hipError_t launch_mlp_pack_k32(const float *params, void *img, hipStream_t s) {
  hipLaunchKernelGGL(mlp::pack_k32_kernel, dim3(1), dim3(256), 0, s, params, reinterpret_cast<mlp::WeightsK32 *>(img));
  return hipGetLastError();
}

hipError_t launch_mlp_pack(const float *params, void *img, hipStream_t s) {
  hipLaunchKernelGGL(mlp::pack_kernel, dim3(1), dim3(256), 0, s, params, reinterpret_cast<mlp::Weights *>(img));
  return hipGetLastError();
}

}  // namespace cf

using namespace cf::mlp;

static bool al16(const void *p) { return ((uintptr_t)p & 15u) == 0; }

extern "C" int32_t cf_mlp_nparam(void) { return NPARAM; }

extern "C" int64_t cf_mlp_work_floats(int32_t n) {
  if (n < 1) return 0;
  return (int64_t)grad_waves(n) * (NPARAM + 1);
}

extern "C" cf_status cf_mlp_forward(void *stream, const float *params, const float *feats, int32_t n, float *out) {
  if (!params || !feats || !out || n < 0) return cf::api_error(CF_E_INVALID_ARG, "cf_mlp_forward: bad argument");
  if (!al16(params) || !al16(feats) || !al16(out)) return cf::api_error(CF_E_INVALID_ARG, "buffers must be 16-byte aligned");
  if (n == 0) return CF_OK;
  int blocks = ((n + 15) / 16 + NWAVE - 1) / NWAVE;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(forward_kernel, dim3(blocks), dim3(BS), 0, (hipStream_t)stream, params, feats, n, out);
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? CF_OK : cf::api_error(CF_E_DEVICE, std::string("mlp forward: ") + hipGetErrorString(e));
}

// The gradient's two launches: per-wave partials into `work` (nw rows of
// NPARAM + 1 floats, every entry written), then their sum in wave order.
static cf_status launch_gradient(hipStream_t s, const float *params, const float *feats, const float *targets, int n,
                                 int nout, int nw, float *work, float *grad, float *loss) {
  hipLaunchKernelGGL(grad_kernel, dim3(nw / NWAVE), dim3(BS), 0, s, params, feats, targets, n, nout, work);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) {
    hipLaunchKernelGGL(reduce_kernel, dim3((NPARAM + 1 + 255) / 256), dim3(256), 0, s, work, nw, grad, loss);
    e = hipGetLastError();
  }
  return e == hipSuccess ? CF_OK : cf::api_error(CF_E_DEVICE, std::string("mlp gradient: ") + hipGetErrorString(e));
}

extern "C" cf_status cf_mlp_gradient(void *stream, const float *params, const float *feats, const float *targets,
                                     int32_t n, int32_t nout, float *work, int64_t work_floats, float *grad,
                                     float *loss) {
  if (!params || !feats || !targets || !work || !grad || n < 1 || nout < 1 || nout > NOUT)
    return cf::api_error(CF_E_INVALID_ARG, "cf_mlp_gradient: bad argument");
  if (!al16(params) || !al16(feats) || !al16(targets) || !al16(work) || !al16(grad))
    return cf::api_error(CF_E_INVALID_ARG, "buffers must be 16-byte aligned");
  const int nw = grad_waves(n);
  if (work_floats < (int64_t)nw * (NPARAM + 1))
    return cf::api_error(CF_E_INVALID_ARG, "work buffer smaller than cf_mlp_work_floats(n)");
  return launch_gradient((hipStream_t)stream, params, feats, targets, n, nout, nw, work, grad, loss);
}

// ---- cf_mlp_gradient without a caller workspace
// The per-wave partial gradients live in `scratch`: room for the largest grid
// the gradient launches (MAX_GRAD_WAVES waves of NPARAM + 1 floats, 47.5 MB),
// so every n fits.  Each GPU the library runs on holds its own copy until the
// process ends.  The kernel writes every entry of each row it uses before the
// sum reads it, so nothing is cleared between calls; calls that overlap on one
// GPU share the array and race.
constexpr size_t kScratchFloats = (size_t)MAX_GRAD_WAVES * (NPARAM + 1);
static __device__ __align__(256) float scratch[kScratchFloats];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
float *g_scratch[kMaxDevices] = {};  // device address of each GPU's `scratch`, taken once per device

// Device address of the current GPU's `scratch` (the array's name is a host
// stand-in: only this address may reach a kernel).
cf_status scratch_address(float **out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices)
    return cf::api_error(CF_E_DEVICE, "cf_mlp_gradient_noalloc: no current HIP device");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch[dev]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return cf::api_error(CF_E_DEVICE, std::string("cf_mlp_gradient_noalloc: address of the static scratch: ") +
                                            hipGetErrorString(e));
    g_scratch[dev] = static_cast<float *>(p);
  }
  *out = g_scratch[dev];
  return CF_OK;
}
}  // namespace

extern "C" cf_status cf_mlp_gradient_noalloc(void *stream, const float *params, const float *feats,
                                             const float *targets, int32_t n, int32_t nout, float *grad,
                                             float *loss) {
  if (!params || !feats || !targets || !grad || n < 1 || nout < 1 || nout > NOUT)
    return cf::api_error(CF_E_INVALID_ARG, "cf_mlp_gradient_noalloc: bad argument");
  if (!al16(params) || !al16(feats) || !al16(targets) || !al16(grad))
    return cf::api_error(CF_E_INVALID_ARG, "buffers must be 16-byte aligned");
  const int nw = grad_waves(n);
  if ((size_t)nw * (NPARAM + 1) > kScratchFloats)
    return cf::api_error(CF_E_INVALID_ARG, "cf_mlp_gradient_noalloc: partial sums exceed the fixed scratch (" +
                                               std::to_string(kScratchFloats) + " floats)");
  float *work = nullptr;
  const cf_status st = scratch_address(&work);
  if (st != CF_OK) return st;
  return launch_gradient((hipStream_t)stream, params, feats, targets, n, nout, nw, work, grad, loss);
}

extern "C" cf_status cf_mlp_adam(void *stream, float *params, float *m, float *v, const float *grad, int32_t step,
                                 float lr) {
  if (!params || !m || !v || !grad || step < 1) return cf::api_error(CF_E_INVALID_ARG, "cf_mlp_adam: bad argument");
  const float bc1 = 1.0f - powf(0.9f, (float)step), bc2 = 1.0f - powf(0.999f, (float)step);
  hipLaunchKernelGGL(adam_kernel, dim3((NPARAM - TRAIN_FROM + 255) / 256), dim3(256), 0, (hipStream_t)stream, params,
                     m, v, grad, lr, bc1, bc2);
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? CF_OK : cf::api_error(CF_E_DEVICE, std::string("mlp adam: ") + hipGetErrorString(e));
}
