// Device pieces of the surrogate network (10 -> 64 -> 64 -> 1, SiLU):
// bfloat16 rounding, the 16x16x32 BF16 MFMA tile and the per-block inference
// used inside the delayed-acceptance trial kernel.
#pragma once

#include "common.hpp"

namespace vc {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr int MLP_IN = 10;
constexpr int MLP_H = 64;
constexpr int MLP_KP = 32;  // first-layer K padded to one MFMA step
constexpr int MLP_NPARAM = 4929;

// Round a float to bfloat16 (nearest, ties to even) and return the bits.
__device__ __forceinline__ uint16_t bf16_bits(float v) {
  uint32_t b = __float_as_uint(v);
  b = b + 0x7FFFu + ((b >> 16) & 1u);
  return (uint16_t)(b >> 16);
}
__device__ __forceinline__ float bf16_round(float v) {
  return __uint_as_float(((uint32_t)bf16_bits(v)) << 16);
}
__device__ __forceinline__ __bf16 to_bf16(float v) {
  const uint16_t b = bf16_bits(v);
  return __builtin_bit_cast(__bf16, b);
}

// C[16x16] += A[16x32] * B[32x16] for one wave.  Lane l supplies
// A[l % 16][8 (l / 16) + 0..7] and B[8 (l / 16) + 0..7][l % 16] and receives
// C[4 (l / 16) + 0..3][l % 16].
__device__ __forceinline__ floatx4 mfma16(bf16x8 a, bf16x8 b, floatx4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// Parameters of the network on the device: bf16 copies for the products,
// FP32 biases, input / output normalization.
struct MlpDev {
  const __bf16 *w1;   // [64][32]: w1[n][k], k >= 10 zero
  const __bf16 *w2;   // [64][64]: w2[n][k]
  const float *b1, *b2, *w3, *b3;  // w3 holds bf16-rounded values
  float mu[MLP_IN], sd[MLP_IN];
  float out_mu, out_sd;
};

// Normalized, bf16-rounded input of one descriptor value.
__device__ __forceinline__ __bf16 mlp_input(const MlpDev &m, int k, double d) {
  const float z = (float)((d - (double)m.mu[k]) / (double)m.sd[k]);
  return to_bf16(z);
}

__device__ __forceinline__ float silu(float a) { return a / (1.0f + expf(-a)); }

// device view of a network handle (surrogate.hip)
MlpDev mlp_dev(const vcsgc_mlp *m);

// The weights a lane of a 256-thread block needs for the hidden layers:
// its B fragments of w1 and w2 (output neuron n = 16 wave + l % 16, rows
// 8 (l / 16) ..) and the two biases of neuron n.  Loading them ahead of the
// descriptors takes the weight reads off the inference's critical path.
struct MlpFrag {
  bf16x8 w1, w2a, w2b;
  float b1, b2;
};

__device__ __forceinline__ MlpFrag mlp_frag(const MlpDev &m) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int kb = (lane >> 4) * 8;
  const int n = wv * 16 + (lane & 15);
  MlpFrag f;
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    f.w1[q] = m.w1[n * MLP_KP + kb + q];
    f.w2a[q] = m.w2[n * MLP_H + kb + q];
    f.w2b[q] = m.w2[n * MLP_H + 32 + kb + q];
  }
  f.b1 = m.b1[n];
  f.b2 = m.b2[n];
  return f;
}

// Inference for the 16 rows of zs (LDS, [16][32] bf16, rows already filled)
// by the 4 waves of a 256-thread block; every wave computes one 16-neuron
// tile of each hidden layer.  Writes y[16] (normalized output) to LDS.
// w3 holds the 64 output weights (device or LDS).  Must be called by all
// 256 threads.
__device__ __forceinline__ void mlp_block16f(const MlpDev &m, const MlpFrag &f,
                                             const float *w3, const __bf16 *zs, __bf16 *h1,
                                             __bf16 *h2, float *y) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int r = lane & 15, kb = (lane >> 4) * 8;
  const int n = wv * 16 + r;  // output neuron of this lane's B column
  // layer 1
  {
    bf16x8 a;
#pragma unroll
    for (int q = 0; q < 8; ++q) a[q] = zs[r * MLP_KP + kb + q];
    floatx4 c = {0.f, 0.f, 0.f, 0.f};
    c = mfma16(a, f.w1, c);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int row = (lane >> 4) * 4 + q;
      h1[row * MLP_H + n] = to_bf16(silu(c[q] + f.b1));
    }
  }
  __syncthreads();
  // layer 2
  {
    floatx4 c = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ks = 0; ks < MLP_H; ks += 32) {
      bf16x8 a;
#pragma unroll
      for (int q = 0; q < 8; ++q) a[q] = h1[r * MLP_H + ks + kb + q];
      c = mfma16(a, ks == 0 ? f.w2a : f.w2b, c);
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int row = (lane >> 4) * 4 + q;
      h2[row * MLP_H + n] = to_bf16(silu(c[q] + f.b2));
    }
  }
  __syncthreads();
  // output layer: 16 dot products of length 64 in ascending k
  if (threadIdx.x < 16) {
    float acc = m.b3[0];
    for (int k = 0; k < MLP_H; ++k) acc += w3[k] * (float)h2[threadIdx.x * MLP_H + k];
    y[threadIdx.x] = acc;
  }
  __syncthreads();
}

// Inference for the 32 rows of zs ([32][32] bf16): two 16-row tiles that share
// every weight fragment.  The two tiles' products are independent, so their
// latencies overlap; each row's value is the one mlp_block16f gives it.
// h1, h2 hold [32][64]; writes y[32].  Must be called by all 256 threads.
__device__ __forceinline__ void mlp_block32f(const MlpDev &m, const MlpFrag &f,
                                             const float *w3, const __bf16 *zs, __bf16 *h1,
                                             __bf16 *h2, float *y) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int r = lane & 15, kb = (lane >> 4) * 8;
  const int n = wv * 16 + r;
  {
    bf16x8 a0, a1;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      a0[q] = zs[r * MLP_KP + kb + q];
      a1[q] = zs[(16 + r) * MLP_KP + kb + q];
    }
    floatx4 c0 = {0.f, 0.f, 0.f, 0.f}, c1 = {0.f, 0.f, 0.f, 0.f};
    c0 = mfma16(a0, f.w1, c0);
    c1 = mfma16(a1, f.w1, c1);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int row = (lane >> 4) * 4 + q;
      h1[row * MLP_H + n] = to_bf16(silu(c0[q] + f.b1));
      h1[(16 + row) * MLP_H + n] = to_bf16(silu(c1[q] + f.b1));
    }
  }
  __syncthreads();
  {
    floatx4 c0 = {0.f, 0.f, 0.f, 0.f}, c1 = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ks = 0; ks < MLP_H; ks += 32) {
      bf16x8 a0, a1;
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        a0[q] = h1[r * MLP_H + ks + kb + q];
        a1[q] = h1[(16 + r) * MLP_H + ks + kb + q];
      }
      c0 = mfma16(a0, ks == 0 ? f.w2a : f.w2b, c0);
      c1 = mfma16(a1, ks == 0 ? f.w2a : f.w2b, c1);
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int row = (lane >> 4) * 4 + q;
      h2[row * MLP_H + n] = to_bf16(silu(c0[q] + f.b2));
      h2[(16 + row) * MLP_H + n] = to_bf16(silu(c1[q] + f.b2));
    }
  }
  __syncthreads();
  if (threadIdx.x < 32) {
    float acc = m.b3[0];
    for (int k = 0; k < MLP_H; ++k) acc += w3[k] * (float)h2[threadIdx.x * MLP_H + k];
    y[threadIdx.x] = acc;
  }
  __syncthreads();
}

__device__ __forceinline__ void mlp_block16(const MlpDev &m, const __bf16 *zs, __bf16 *h1,
                                            __bf16 *h2, float *y) {
  mlp_block16f(m, mlp_frag(m), m.w3, zs, h1, h2, y);
}

}  // namespace vc
