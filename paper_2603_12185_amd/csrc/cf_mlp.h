// cf_mlp.h - the learned per-contact impedance network on MFMA (bf16 inputs,
// float32 accumulation): parameter layout and the per-wave forward pass shared
// by the training kernels and the resolution kernel.
//
// Network (per contact): 7 features (phi, v_n, u_1, u_2, m_eff, mu_t, h),
// normalised x = (f - mean) / std; z1 = W1^T x + b1, a1 = silu(z1) (64);
// z2 = W2^T a1 + b2, a2 = silu(z2) (64); y = W3^T a2 + b3 (16 outputs, one per
// facet used).  The facet impulse gain is the heuristic's times
// exp(clamp(y_f, -ln 256, ln 256)).
//
// Flat float32 parameters (row-major): mean[8], std[8], W1[8][64], b1[64],
// W2[64][64], b2[64], W3[64][16], b3[16].
//
// Products are formed transposed, Z^T = W^T A^T, with the 16x16x16 bf16 MFMA:
// the accumulator of one 16-unit block (lane l holds rows 4 (l / 16) + r,
// column l % 16) is exactly the B operand of the next layer's matching
// 16-wide K block, so activations never leave registers.  Weights are staged
// in LDS as bf16, transposed so each lane reads its four K values at once.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cf {
namespace mlp {

constexpr int NIN = 8, NH = 64, NOUT = 16, NFEAT = 7;
constexpr int OFF_MEAN = 0, OFF_STD = 8, OFF_W1 = 16, OFF_B1 = OFF_W1 + NIN * NH, OFF_W2 = OFF_B1 + NH,
              OFF_B2 = OFF_W2 + NH * NH, OFF_W3 = OFF_B2 + NH, OFF_B3 = OFF_W3 + NH * NOUT,
              NPARAM = OFF_B3 + NOUT, TRAIN_FROM = OFF_W1;
constexpr float CLIP = 5.5451774444795623f;  // ln 256

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// float -> bf16 bits, round to nearest even (finite inputs)
__device__ inline short to_bf16(float x) {
  uint32_t u = __float_as_uint(x);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (short)(u >> 16);
}

// SiLU and its derivative with the hardware exponential and reciprocal
// (v_exp_f32, v_rcp_f32: about 1 ulp each, far below the bf16 rounding of the
// activations); a large negative z gives exp = inf, rcp = 0, silu = -0.
__device__ inline float sigmoid(float z) { return __builtin_amdgcn_rcpf(1.0f + __expf(-z)); }
__device__ inline float silu(float z) { return z * sigmoid(z); }
__device__ inline float dsilu(float z) {
  const float s = sigmoid(z);
  return s * (1.0f + z * (1.0f - s));
}

__device__ inline f32x4 mfma(bf16x4 a, bf16x4 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

// Weights in LDS (bf16 bits): W1^T [64][16] (K padded with zeros), W2^T [64][64],
// W3^T [16][64]; biases and normalisation in float32.
struct Weights {
  short w1t[NH * 16];
  short w2t[NH * NH];
  short w3t[NOUT * NH];
  float b1[NH], b2[NH], b3[NOUT], mean[NIN], istd[NIN];
};

// Stage the parameters into LDS (all threads of the block; ends with a barrier).
template <int BS>
__device__ inline void stage_weights(const float *p, Weights *W) {
  for (int i = threadIdx.x; i < NH * 16; i += BS) {
    const int h = i >> 4, k = i & 15;
    W->w1t[i] = to_bf16(k < NIN ? p[OFF_W1 + k * NH + h] : 0.f);
  }
  for (int i = threadIdx.x; i < NH * NH; i += BS) {
    const int o = i >> 6, k = i & 63;
    W->w2t[i] = to_bf16(p[OFF_W2 + k * NH + o]);
  }
  for (int i = threadIdx.x; i < NOUT * NH; i += BS) {
    const int o = i >> 6, k = i & 63;
    W->w3t[i] = to_bf16(p[OFF_W3 + k * NOUT + o]);
  }
  for (int i = threadIdx.x; i < NH; i += BS) {
    W->b1[i] = p[OFF_B1 + i];
    W->b2[i] = p[OFF_B2 + i];
  }
  for (int i = threadIdx.x; i < NOUT; i += BS) W->b3[i] = p[OFF_B3 + i];
  for (int i = threadIdx.x; i < NIN; i += BS) {
    W->mean[i] = p[OFF_MEAN + i];
    W->istd[i] = 1.0f / p[OFF_STD + i];
  }
  __syncthreads();
}

__device__ inline bf16x4 lds4(const short *s) { return *reinterpret_cast<const bf16x4 *>(s); }

// Activations of one tile of 16 contacts, kept for the backward pass.
struct Tile {
  f32x4 z1[4], z2[4];  // pre-activations, block m: rows 16 m + 4 (l / 16) + r, column l % 16
  f32x4 y;             // outputs: rows 4 (l / 16) + r, column l % 16
  bf16x4 x;            // input operand: x[contact l % 16][4 (l / 16) + t]
};

// Forward pass of one wave over 16 contacts.  `f4(t)` returns raw feature
// 4 (l / 16) + t of the lane's contact l % 16 (features >= NFEAT are ignored).
template <class F>
__device__ inline void forward_tile(const Weights *W, F f4, Tile &T) {
  const int l = threadIdx.x & 63, q = l >> 4, c = l & 15;
  (void)c;
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int k = 4 * q + t;
    const float v = k < NFEAT ? (f4(t) - W->mean[k]) * W->istd[k] : 0.f;
    T.x[t] = to_bf16(v);
  }
  bf16x4 a1[4];
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    f32x4 z = {0.f, 0.f, 0.f, 0.f};
    z = mfma(lds4(W->w1t + (16 * m + c) * 16 + 4 * q), T.x, z);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      z[r] += W->b1[16 * m + 4 * q + r];
      a1[m][r] = to_bf16(silu(z[r]));
    }
    T.z1[m] = z;
  }
  bf16x4 a2[4];
#pragma unroll
  for (int m2 = 0; m2 < 4; ++m2) {
    f32x4 z = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int m = 0; m < 4; ++m) z = mfma(lds4(W->w2t + (16 * m2 + c) * NH + 16 * m + 4 * q), a1[m], z);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      z[r] += W->b2[16 * m2 + 4 * q + r];
      a2[m2][r] = to_bf16(silu(z[r]));
    }
    T.z2[m2] = z;
  }
  f32x4 y = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int m = 0; m < 4; ++m) y = mfma(lds4(W->w3t + c * NH + 16 * m + 4 * q), a2[m], y);
#pragma unroll
  for (int r = 0; r < 4; ++r) y[r] += W->b3[4 * q + r];
  T.y = y;
}

// ---- inference inside the resolution: v_mfma_f32_16x16x32_bf16 (K = 32)
//
// Per 16-contact tile the products are again formed transposed (outputs x
// contacts).  The 16 x 16 accumulator of an output block gives lane l the units
// 16 m + 4 (l / 16) + r of contact l % 16, and a K = 32 operand takes eight
// K values per lane (K = 8 (l / 16) + t).  Ordering the K index of input block
// b as pi_b(8 g + t) = 32 b + 4 g + t (t < 4), 32 b + 16 + 4 g + t - 4 (t >= 4)
// makes lane l's own activations of blocks m = 2 b and 2 b + 1 exactly its
// operand, so they never leave registers; the weights are stored in that
// order.  Layer 1 has 8 inputs (7 features and a zero), held by the lanes of
// K group 0.
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

struct WeightsK32 {
  bf16x8 w1[4][16];     // [output block][row]: W1^T rows, inputs 0..7 (K group 0 only)
  bf16x8 w2[4][2][64];  // [output block][input block][lane]: W2^T in pi order
  bf16x8 w3[2][64];     // [input block][lane]: W3^T in pi order
  float4 b1[16], b2[16], b3[4];  // biases by (output block, K group): units 16 m + 4 g + 0..3
  float mean[NIN], istd[NIN];
};

// Pack the float32 parameters into WeightsK32 (all threads of the block; ends
// with a barrier).
template <int BS>
__device__ inline void pack_weights_k32(const float *p, WeightsK32 *W) {
  auto in_of = [](int b, int k) {  // input unit of K index k of input block b
    const int g = k >> 3, t = k & 7;
    return 32 * b + (t < 4 ? 4 * g + t : 16 + 4 * g + t - 4);
  };
  for (int i = threadIdx.x; i < 4 * 16; i += BS) {
    const int m = i >> 4, row = i & 15;
    bf16x8 v;
#pragma unroll
    for (int t = 0; t < 8; ++t) v[t] = (__bf16)(t < NFEAT ? p[OFF_W1 + t * NH + 16 * m + row] : 0.f);
    W->w1[m][row] = v;
  }
  for (int i = threadIdx.x; i < 4 * 2 * 64; i += BS) {
    const int m = i >> 7, b = (i >> 6) & 1, lane = i & 63;
    const int out = 16 * m + (lane & 15), g = lane >> 4;
    bf16x8 v;
#pragma unroll
    for (int t = 0; t < 8; ++t) v[t] = (__bf16)p[OFF_W2 + in_of(b, 8 * g + t) * NH + out];
    W->w2[m][b][lane] = v;
  }
  for (int i = threadIdx.x; i < 2 * 64; i += BS) {
    const int b = i >> 6, lane = i & 63;
    const int out = lane & 15, g = lane >> 4;
    bf16x8 v;
#pragma unroll
    for (int t = 0; t < 8; ++t) v[t] = (__bf16)p[OFF_W3 + in_of(b, 8 * g + t) * NOUT + out];
    W->w3[b][lane] = v;
  }
  for (int i = threadIdx.x; i < 16; i += BS) {
    const int m = i >> 2, g = i & 3, u = 16 * m + 4 * g;
    W->b1[i] = make_float4(p[OFF_B1 + u], p[OFF_B1 + u + 1], p[OFF_B1 + u + 2], p[OFF_B1 + u + 3]);
    W->b2[i] = make_float4(p[OFF_B2 + u], p[OFF_B2 + u + 1], p[OFF_B2 + u + 2], p[OFF_B2 + u + 3]);
  }
  for (int i = threadIdx.x; i < 4; i += BS)
    W->b3[i] = make_float4(p[OFF_B3 + 4 * i], p[OFF_B3 + 4 * i + 1], p[OFF_B3 + 4 * i + 2], p[OFF_B3 + 4 * i + 3]);
  for (int i = threadIdx.x; i < NIN; i += BS) {
    W->mean[i] = p[OFF_MEAN + i];
    W->istd[i] = 1.0f / p[OFF_STD + i];
  }
  __syncthreads();
}

__device__ inline f32x4 mfma32(bf16x8 a, bf16x8 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// Outputs of one 16-contact tile: lane l gets outputs 4 (l / 16) + r of contact
// l % 16 of the tile.  `x` is the lane's input operand: the bf16 normalised
// features of contact l % 16 in the lanes of K group 0, zero elsewhere.
__device__ inline f32x4 forward_tile_k32(const WeightsK32 *W, bf16x8 x) {
  const int l = threadIdx.x & 63, g = l >> 4, c = l & 15;
  const bf16x8 zero8 = {};
  // each layer's bias is the accumulators' initial value
  auto bias = [](float4 b) {
    const f32x4 v = {b.x, b.y, b.z, b.w};
    return v;
  };
  bf16x8 a[2];  // layer-1 activations as the operands of input blocks 0, 1
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    const f32x4 z = mfma32(g == 0 ? W->w1[m][c] : zero8, x, bias(W->b1[4 * m + g]));
#pragma unroll
    for (int r = 0; r < 4; ++r) a[m >> 1][4 * (m & 1) + r] = (__bf16)silu(z[r]);
  }
  bf16x8 a2[2];
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    f32x4 z = mfma32(W->w2[m][0][l], a[0], bias(W->b2[4 * m + g]));
    z = mfma32(W->w2[m][1][l], a[1], z);
#pragma unroll
    for (int r = 0; r < 4; ++r) a2[m >> 1][4 * (m & 1) + r] = (__bf16)silu(z[r]);
  }
  f32x4 y = mfma32(W->w3[0][l], a2[0], bias(W->b3[g]));
  return mfma32(W->w3[1][l], a2[1], y);
}

}  // namespace mlp
}  // namespace cf
