// mlp_device.hpp - device pieces of the gradient-corrector network
// (85 -> 64 -> 64 -> 9, SiLU) on gfx950 matrix cores: BF16 operands, FP32
// accumulation with v_mfma_f32_16x16x32_bf16.
//
// Operand layout of one 16x16x32 product D = A B + C (64 lanes):
//   A(i, k): lane i + 16 (k / 8), element k % 8   (8 BF16 per lane)
//   B(k, j): lane j + 16 (k / 8), element k % 8
//   C/D(i, j): lane j + 16 (i / 4), element i % 4 (4 FP32 per lane)
// so a lane's A or B operand is 8 consecutive k of one row of a row-major
// [i][k] (A) or [j][k] (B, i.e. W[out][in]) matrix: one 16-byte load.
//
// Parameters are one FP32 vector in the order W1 (64x85, [out][in]), b1,
// W2 (64x64), b2, W3 (9x64), b3.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbm {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kMlpIn = 85, kMlpInPad = 96, kMlpHid = 64, kMlpOut = 9, kMlpOutPad = 16;
// Row stride of the multi-tile forward's activation rows: 144 bytes (16-byte
// aligned rows for the operand reads; the 16 rows a wavefront writes at once
// start 4 banks apart instead of all on one bank).
constexpr int kMlpHidRow = 72;
constexpr int kMlpParams = 10249;
constexpr int kOffW1 = 0, kOffB1 = 64 * 85, kOffW2 = kOffB1 + 64, kOffB2 = kOffW2 + 64 * 64, kOffW3 = kOffB2 + 64,
              kOffB3 = kOffW3 + 9 * 64;
static_assert(kOffB3 + 9 == kMlpParams, "parameter count");

__device__ __forceinline__ f32x4 mfma(const bf16x8& a, const bf16x8& b, const f32x4& c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ bf16x8 lds8(const __bf16* p) { return *(const bf16x8*)p; }

// The activations end up in BF16 (8 significant bits), so the logistic
// function takes the hardware exponential and reciprocal (about 1 ulp of
// FP32 each) instead of an IEEE division: the transcendental unit, not the
// matrix cores, bounds the forward pass.
__device__ __forceinline__ float sigmoid(float z) { return __builtin_amdgcn_rcpf(1.0f + __expf(-z)); }

__device__ __forceinline__ float silu(float z) { return z * sigmoid(z); }

// d/dz silu(z) = s + z s (1 - s), s = sigmoid(z)
__device__ __forceinline__ float silu_grad(float z) {
  const float s = sigmoid(z);
  return s + z * s * (1.0f - s);
}

// BF16 weights in the B-operand layout ([out][in], padded with zeros) and
// FP32 biases.
struct MlpWeights {
  __bf16 W1[kMlpHid][kMlpInPad];
  __bf16 W2[kMlpHid][kMlpHid];
  __bf16 W3[kMlpOutPad][kMlpHid];
  float b1[kMlpHid], b2[kMlpHid], b3[kMlpOutPad];
};

// Block-cooperative fill from the FP32 parameter vector (RNE to BF16).
template <int BLOCK>
__device__ void mlp_load_weights(const float* __restrict__ theta, MlpWeights& w) {
  for (int i = threadIdx.x; i < kMlpHid * kMlpInPad; i += BLOCK) {
    const int o = i / kMlpInPad, k = i % kMlpInPad;
    w.W1[o][k] = (__bf16)(k < kMlpIn ? theta[kOffW1 + o * kMlpIn + k] : 0.0f);
  }
  for (int i = threadIdx.x; i < kMlpHid * kMlpHid; i += BLOCK) w.W2[i / kMlpHid][i % kMlpHid] = (__bf16)theta[kOffW2 + i];
  for (int i = threadIdx.x; i < kMlpOutPad * kMlpHid; i += BLOCK) {
    const int o = i / kMlpHid, k = i % kMlpHid;
    w.W3[o][k] = (__bf16)(o < kMlpOut ? theta[kOffW3 + o * kMlpHid + k] : 0.0f);
  }
  for (int i = threadIdx.x; i < kMlpHid; i += BLOCK) {
    w.b1[i] = theta[kOffB1 + i];
    w.b2[i] = theta[kOffB2 + i];
  }
  for (int i = threadIdx.x; i < kMlpOutPad; i += BLOCK) w.b3[i] = i < kMlpOut ? theta[kOffB3 + i] : 0.0f;
}

// Forward pass of one 16-sample tile by one wavefront. a1: the tile's
// features as A operands of the three k-steps (features 0-31, 32-63,
// 64-95). h1, h2: this wave's [16][64] BF16 LDS rows for the hidden
// activations; d1, d2 (optional) receive silu'(z) in the same layout. Returns
// y (+ b3) in the C layout: lane j + 16 (i / 4) holds output j of samples
// 4 (lane / 16) + e, e = 0..3.
__device__ __forceinline__ f32x4 mlp_forward_tile(const bf16x8 (&a1)[3], const MlpWeights& w, __bf16* h1, __bf16* h2,
                                                   __bf16* d1, __bf16* d2) {
  const int lane = threadIdx.x & 63, col = lane & 15, grp = lane >> 4;
  // layer 1
#pragma unroll
  for (int n = 0; n < 4; ++n) {
    f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int ks = 0; ks < 3; ++ks) acc = mfma(a1[ks], lds8(&w.W1[n * 16 + col][ks * 32 + grp * 8]), acc);
    const int j = n * 16 + col;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const float z = acc[e] + w.b1[j];
      h1[(grp * 4 + e) * kMlpHid + j] = (__bf16)silu(z);
      if (d1) d1[(grp * 4 + e) * kMlpHid + j] = (__bf16)silu_grad(z);
    }
  }
  __builtin_amdgcn_s_waitcnt(0xc07f);  // lgkmcnt(0): this wave's LDS writes done
  __builtin_amdgcn_wave_barrier();
  // layer 2
  bf16x8 a2[2];
#pragma unroll
  for (int ks = 0; ks < 2; ++ks) a2[ks] = lds8(&h1[col * kMlpHid + ks * 32 + grp * 8]);
#pragma unroll
  for (int n = 0; n < 4; ++n) {
    f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int ks = 0; ks < 2; ++ks) acc = mfma(a2[ks], lds8(&w.W2[n * 16 + col][ks * 32 + grp * 8]), acc);
    const int j = n * 16 + col;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const float z = acc[e] + w.b2[j];
      h2[(grp * 4 + e) * kMlpHid + j] = (__bf16)silu(z);
      if (d2) d2[(grp * 4 + e) * kMlpHid + j] = (__bf16)silu_grad(z);
    }
  }
  __builtin_amdgcn_s_waitcnt(0xc07f);
  __builtin_amdgcn_wave_barrier();
  // layer 3
  bf16x8 a3[2];
#pragma unroll
  for (int ks = 0; ks < 2; ++ks) a3[ks] = lds8(&h2[col * kMlpHid + ks * 32 + grp * 8]);
  f32x4 y = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
  for (int ks = 0; ks < 2; ++ks) y = mfma(a3[ks], lds8(&w.W3[col][ks * 32 + grp * 8]), y);
#pragma unroll
  for (int e = 0; e < 4; ++e) y[e] += w.b3[col];
  return y;
}

// Inference on T 16-sample tiles at once by one wavefront: each weight
// operand is read from LDS once for the T tiles, and the T independent
// product chains hide one another's matrix-core and LDS latency. The
// products are taken transposed (the weights as the A operand, a tile's
// samples as the B operand, which is the same register content as the
// single-tile form's operands in the other roles), so a lane's four results
// are four consecutive neurons of one sample: one 8-byte LDS store per lane
// and neuron block instead of four 2-byte ones. h: this wave's [T][16][64]
// BF16 LDS rows, holding the first hidden layer and then, once every lane
// has read it, the second. y receives y + b3 per tile: lane l holds outputs
// 4 (l / 16) .. 4 (l / 16) + 3 of sample l % 16.
template <int T>
__device__ __forceinline__ void mlp_forward_tiles(const bf16x8 (&a1)[T][3], const MlpWeights& w, __bf16* h,
                                                  f32x4 (&y)[T]) {
  const int lane = threadIdx.x & 63, col = lane & 15, grp = lane >> 4;
  constexpr int kTile = 16 * kMlpHidRow;
  typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
  auto put = [&](int t, int j, const f32x4& z, const float* bias) {
    bf16x4 o;
#pragma unroll
    for (int e = 0; e < 4; ++e) o[e] = (__bf16)silu(z[e] + bias[j + e]);
    *(bf16x4*)&h[t * kTile + col * kMlpHidRow + j] = o;
  };
  // layer 1
#pragma unroll
  for (int n = 0; n < 4; ++n) {
    f32x4 acc[T];
#pragma unroll
    for (int t = 0; t < T; ++t) acc[t] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int ks = 0; ks < 3; ++ks) {
      const bf16x8 wop = lds8(&w.W1[n * 16 + col][ks * 32 + grp * 8]);
#pragma unroll
      for (int t = 0; t < T; ++t) acc[t] = mfma(wop, a1[t][ks], acc[t]);
    }
#pragma unroll
    for (int t = 0; t < T; ++t) put(t, n * 16 + grp * 4, acc[t], w.b1);
  }
  __builtin_amdgcn_s_waitcnt(0xc07f);  // lgkmcnt(0): this wave's LDS writes done
  __builtin_amdgcn_wave_barrier();
  // layer 2: every B operand read before the outputs overwrite h
  bf16x8 a2[T][2];
#pragma unroll
  for (int t = 0; t < T; ++t)
#pragma unroll
    for (int ks = 0; ks < 2; ++ks) a2[t][ks] = lds8(&h[t * kTile + col * kMlpHidRow + ks * 32 + grp * 8]);
  __builtin_amdgcn_s_waitcnt(0xc07f);
  __builtin_amdgcn_wave_barrier();
#pragma unroll
  for (int n = 0; n < 4; ++n) {
    f32x4 acc[T];
#pragma unroll
    for (int t = 0; t < T; ++t) acc[t] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int ks = 0; ks < 2; ++ks) {
      const bf16x8 wop = lds8(&w.W2[n * 16 + col][ks * 32 + grp * 8]);
#pragma unroll
      for (int t = 0; t < T; ++t) acc[t] = mfma(wop, a2[t][ks], acc[t]);
    }
#pragma unroll
    for (int t = 0; t < T; ++t) put(t, n * 16 + grp * 4, acc[t], w.b2);
  }
  __builtin_amdgcn_s_waitcnt(0xc07f);
  __builtin_amdgcn_wave_barrier();
  // layer 3
  bf16x8 a3[T][2];
#pragma unroll
  for (int t = 0; t < T; ++t)
#pragma unroll
    for (int ks = 0; ks < 2; ++ks) a3[t][ks] = lds8(&h[t * kTile + col * kMlpHidRow + ks * 32 + grp * 8]);
#pragma unroll
  for (int t = 0; t < T; ++t) y[t] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
  for (int ks = 0; ks < 2; ++ks) {
    const bf16x8 wop = lds8(&w.W3[col][ks * 32 + grp * 8]);
#pragma unroll
    for (int t = 0; t < T; ++t) y[t] = mfma(wop, a3[t][ks], y[t]);
  }
#pragma unroll
  for (int t = 0; t < T; ++t)
#pragma unroll
    for (int e = 0; e < 4; ++e) y[t][e] += w.b3[grp * 4 + e];
  // h is read again by the next call's first writes: keep this call's reads
  // ahead of them
  __builtin_amdgcn_s_waitcnt(0xc07f);
  __builtin_amdgcn_wave_barrier();
}

}  // namespace lbm
