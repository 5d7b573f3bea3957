// mlp.hip - forward pass, gradient and Adam update of the gradient-corrector
// network on matrix cores (BF16 operands, FP32 accumulation, FP32 master
// weights).
//
// Training: a workgroup takes 64 samples at a time (16 per wavefront). Each
// wave runs its tile forward, keeping h and silu'(z) in LDS row-major and
// transposed, then back-propagates dy = 2 (y - t) / (9 B) to dz2 and dz1 for
// its tile. The weight gradients dW = dz^T h contract over the 64 samples:
// the 16x16 output tiles are split over the waves and held in registers for
// the whole batch slice of the workgroup. Per-workgroup FP32 partials are
// added over workgroups in a fixed order, so the gradient is reproducible.
#include "device_util.hpp"
#include "internal.hpp"
#include "mlp_device.hpp"

namespace lbm {

namespace {

constexpr int kMBlock = 256;
constexpr int kChunk = 64;

struct TrainLds {
  MlpWeights w;
  __bf16 W2T[kMlpHid][kMlpHid];  // [in][out]
  __bf16 W3T[kMlpHid][32];       // [in][out], out padded to one k-step
  __bf16 XT[kMlpInPad][kChunk];
  __bf16 h1[kChunk][kMlpHid], h1T[kMlpHid][kChunk], d1[kChunk][kMlpHid];
  __bf16 h2[kChunk][kMlpHid], h2T[kMlpHid][kChunk], d2[kChunk][kMlpHid];
  __bf16 dy[kChunk][32], dyT[kMlpOutPad][kChunk];
  __bf16 dz2[kChunk][kMlpHid], dz2T[kMlpHid][kChunk], dz1T[kMlpHid][kChunk];
  float bred[kMBlock / 64][2 * kMlpHid + kMlpOutPad];
};

constexpr int kFwdTiles = 2;    // 16-sample tiles per wavefront in the forward kernel
constexpr int kFBlock = 768;    // forward workgroup: 12 wavefronts share one copy of the weights

struct FwdLds {
  MlpWeights w;
  __bf16 h[kFBlock / 64][kFwdTiles][16][kMlpHidRow];
};

__device__ __forceinline__ void load_tile(const __bf16* __restrict__ X, int64_t n, int64_t cell, bf16x8 (&a)[3]) {
  const int grp = (threadIdx.x & 63) >> 4;
#pragma unroll
  for (int ks = 0; ks < 3; ++ks) {
    if (cell < n) {
      a[ks] = *(const bf16x8*)(X + cell * kMlpInPad + ks * 32 + grp * 8);
    } else {
#pragma unroll
      for (int e = 0; e < 8; ++e) a[ks][e] = (__bf16)0.0f;
    }
  }
}

__global__ void __launch_bounds__(kFBlock)
k_mlp_forward(const float* __restrict__ theta, const __bf16* __restrict__ X, int64_t n, float* __restrict__ Y) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  FwdLds& s = *(FwdLds*)lds_raw;
  mlp_load_weights<kFBlock>(theta, s.w);
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, col = lane & 15, grp = lane >> 4;
  constexpr int64_t kFwdChunk = (kFBlock / 64) * kFwdTiles * 16;
  for (int64_t c0 = (int64_t)blockIdx.x * kFwdChunk; c0 < n; c0 += (int64_t)gridDim.x * kFwdChunk) {
    const int64_t base = c0 + wave * kFwdTiles * 16;
    bf16x8 a[kFwdTiles][3];
#pragma unroll
    for (int t = 0; t < kFwdTiles; ++t) load_tile(X, n, base + t * 16 + col, a[t]);
    f32x4 y[kFwdTiles];
    mlp_forward_tiles<kFwdTiles>(a, s.w, &s.h[wave][0][0][0], y);
#pragma unroll
    for (int t = 0; t < kFwdTiles; ++t) {
      const int64_t cell = base + t * 16 + col;
      if (cell < n) *(f32x4*)&Y[cell * kMlpOutPad + grp * 4] = y[t];
    }
  }
}

// Gradient of the mean squared error over a batch of n samples. part:
// [gridDim.x][kMlpParams] FP32 partial gradients; lpart: [gridDim.x] FP64
// partial sums of squared errors.
__global__ void __launch_bounds__(kMBlock)
k_mlp_train(const float* __restrict__ theta, const __bf16* __restrict__ X, const float* __restrict__ T, int64_t n,
            float* __restrict__ part, double* __restrict__ lpart) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  TrainLds& s = *(TrainLds*)lds_raw;
  mlp_load_weights<kMBlock>(theta, s.w);
  for (int i = threadIdx.x; i < kMlpHid * kMlpHid; i += kMBlock) {
    const int o = i / kMlpHid, k = i % kMlpHid;
    s.W2T[k][o] = (__bf16)theta[kOffW2 + i];
  }
  for (int i = threadIdx.x; i < kMlpHid * 32; i += kMBlock) {
    const int k = i / 32, o = i % 32;
    s.W3T[k][o] = (__bf16)(o < kMlpOut ? theta[kOffW3 + o * kMlpHid + k] : 0.0f);
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, col = lane & 15, grp = lane >> 4;
  const int r0 = wave * 16;  // this wave's rows of the chunk
  const float gscale = (float)(2.0 / (9.0 * (double)n));
  f32x4 gW1[6], gW2[4], gW3;
  float gb1[4], gb2[4], gb3 = 0.0f;
#pragma unroll
  for (int q = 0; q < 6; ++q) gW1[q] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    gW2[q] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    gb1[q] = gb2[q] = 0.0f;
  }
  gW3 = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
  double sq = 0.0;

  for (int64_t c0 = (int64_t)blockIdx.x * kChunk; c0 < n; c0 += (int64_t)gridDim.x * kChunk) {
    const int64_t base = c0 + r0;
    bf16x8 a[3];
    load_tile(X, n, base + col, a);
#pragma unroll
    for (int ks = 0; ks < 3; ++ks)
#pragma unroll
      for (int e = 0; e < 8; ++e) s.XT[ks * 32 + grp * 8 + e][r0 + col] = a[ks][e];
    const f32x4 y = mlp_forward_tile(a, s.w, &s.h1[r0][0], &s.h2[r0][0], &s.d1[r0][0], &s.d2[r0][0]);
    // transposed activations for the weight gradients
    for (int i = lane; i < 16 * kMlpHid; i += 64) {
      const int rr = i / kMlpHid, cc = i % kMlpHid;
      s.h1T[cc][r0 + rr] = s.h1[r0 + rr][cc];
      s.h2T[cc][r0 + rr] = s.h2[r0 + rr][cc];
    }
    // output error
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int row = r0 + grp * 4 + e;
      const int64_t cell = c0 + row;
      float dyv = 0.0f;
      if (cell < n && col < kMlpOut) {
        const float r = y[e] - T[cell * kMlpOutPad + col];
        sq += (double)r * (double)r;
        dyv = gscale * r;
      }
      gb3 += dyv;
      s.dy[row][col] = (__bf16)dyv;
      s.dy[row][col + 16] = (__bf16)0.0f;
      s.dyT[col][row] = (__bf16)dyv;
    }
    __builtin_amdgcn_s_waitcnt(0xc07f);
    __builtin_amdgcn_wave_barrier();
    // dz2 = (dy W3) * silu'(z2)
    {
      const bf16x8 A = lds8(&s.dy[r0 + col][grp * 8]);
#pragma unroll
      for (int nt = 0; nt < 4; ++nt) {
        f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
        acc = mfma(A, lds8(&s.W3T[nt * 16 + col][grp * 8]), acc);
        const int j = nt * 16 + col;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int row = r0 + grp * 4 + e;
          const float dz = acc[e] * (float)s.d2[row][j];
          gb2[nt] += dz;
          s.dz2[row][j] = (__bf16)dz;
          s.dz2T[j][row] = (__bf16)dz;
        }
      }
    }
    __builtin_amdgcn_s_waitcnt(0xc07f);
    __builtin_amdgcn_wave_barrier();
    // dz1 = (dz2 W2) * silu'(z1)
    {
      bf16x8 A[2];
#pragma unroll
      for (int ks = 0; ks < 2; ++ks) A[ks] = lds8(&s.dz2[r0 + col][ks * 32 + grp * 8]);
#pragma unroll
      for (int nt = 0; nt < 4; ++nt) {
        f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int ks = 0; ks < 2; ++ks) acc = mfma(A[ks], lds8(&s.W2T[nt * 16 + col][ks * 32 + grp * 8]), acc);
        const int j = nt * 16 + col;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int row = r0 + grp * 4 + e;
          const float dz = acc[e] * (float)s.d1[row][j];
          gb1[nt] += dz;
          s.dz1T[j][row] = (__bf16)dz;
        }
      }
    }
    __syncthreads();
    // weight gradients over the 64 samples: wave w owns output tile w of W1
    // and W2 (all input tiles) and input tile w of W3
#pragma unroll
    for (int ks = 0; ks < 2; ++ks) {
      const int k0 = ks * 32 + grp * 8;
      const bf16x8 A1 = lds8(&s.dz1T[wave * 16 + col][k0]);
      const bf16x8 A2 = lds8(&s.dz2T[wave * 16 + col][k0]);
#pragma unroll
      for (int q = 0; q < 6; ++q) gW1[q] = mfma(A1, lds8(&s.XT[q * 16 + col][k0]), gW1[q]);
#pragma unroll
      for (int q = 0; q < 4; ++q) gW2[q] = mfma(A2, lds8(&s.h1T[q * 16 + col][k0]), gW2[q]);
      gW3 = mfma(lds8(&s.dyT[col][k0]), lds8(&s.h2T[wave * 16 + col][k0]), gW3);
    }
    __syncthreads();
  }

  float* out = part + (size_t)blockIdx.x * kMlpParams;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int o = wave * 16 + grp * 4 + e;
#pragma unroll
    for (int q = 0; q < 6; ++q) {
      const int k = q * 16 + col;
      if (k < kMlpIn) out[kOffW1 + o * kMlpIn + k] = gW1[q][e];
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) out[kOffW2 + o * kMlpHid + q * 16 + col] = gW2[q][e];
    const int o3 = grp * 4 + e;
    if (o3 < kMlpOut) out[kOffW3 + o3 * kMlpHid + wave * 16 + col] = gW3[e];
  }
  // bias gradients: lanes col, col + 16, col + 32, col + 48 hold other samples
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    gb1[q] += __shfl_xor(gb1[q], 16, 64);
    gb1[q] += __shfl_xor(gb1[q], 32, 64);
    gb2[q] += __shfl_xor(gb2[q], 16, 64);
    gb2[q] += __shfl_xor(gb2[q], 32, 64);
  }
  gb3 += __shfl_xor(gb3, 16, 64);
  gb3 += __shfl_xor(gb3, 32, 64);
  if (grp == 0) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      s.bred[wave][q * 16 + col] = gb1[q];
      s.bred[wave][kMlpHid + q * 16 + col] = gb2[q];
    }
    s.bred[wave][2 * kMlpHid + col] = gb3;
  }
  __syncthreads();
  if (threadIdx.x < 2 * kMlpHid + kMlpOut) {
    float v = 0.0f;
    for (int w = 0; w < kMBlock / 64; ++w) v += s.bred[w][threadIdx.x];
    const int t = threadIdx.x;
    out[t < kMlpHid ? kOffB1 + t : (t < 2 * kMlpHid ? kOffB2 + t - kMlpHid : kOffB3 + t - 2 * kMlpHid)] = v;
  }
  double l[1] = {sq};
  block_sum_first<kMBlock, 1>(l);
  if (threadIdx.x == 0) lpart[blockIdx.x] = l[0];
}

__global__ void __launch_bounds__(256)
k_mlp_reduce(const float* __restrict__ part, const double* __restrict__ lpart, int nblocks, float* __restrict__ grad,
             double* __restrict__ loss) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < kMlpParams) {
    double s = 0.0;
    for (int b = 0; b < nblocks; ++b) s += (double)part[(size_t)b * kMlpParams + i];
    grad[i] = (float)s;
  }
  if (i == kMlpParams) {
    double s = 0.0;
    for (int b = 0; b < nblocks; ++b) s += lpart[b];
    *loss = s;
  }
}

__global__ void __launch_bounds__(256)
k_mlp_adam(float* __restrict__ theta, float* __restrict__ m, float* __restrict__ v, const float* __restrict__ g,
           float lr, float b1, float b2, float eps, float c1, float c2) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= kMlpParams) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.0f - b1) * gi;
  const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  theta[i] -= lr * (mi * c1) / (sqrtf(vi * c2) + eps);
}

}  // namespace

size_t mlp_train_lds_bytes() { return sizeof(TrainLds); }
size_t mlp_forward_lds_bytes() { return sizeof(FwdLds); }

hipError_t launch_mlp_forward(hipStream_t st, const float* theta, const uint16_t* X, int64_t n, float* Y) {
  if (n <= 0) return hipSuccess;
  const int64_t chunks = (n + (kFBlock / 64) * kFwdTiles * 16 - 1) / ((kFBlock / 64) * kFwdTiles * 16);
  const int grid = (int)std::min<int64_t>(chunks, 2048);
  hipLaunchKernelGGL(k_mlp_forward, dim3(grid), dim3(kFBlock), sizeof(FwdLds), st, theta, (const __bf16*)X, n, Y);
  return hipGetLastError();
}

hipError_t launch_mlp_gradient(hipStream_t st, const float* theta, const uint16_t* X, const float* T, int64_t n,
                               float* part, double* lpart, float* grad, double* loss) {
  const int64_t chunks = (n + kChunk - 1) / kChunk;
  const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(chunks, kMlpGrid));
  hipLaunchKernelGGL(k_mlp_train, dim3(grid), dim3(kMBlock), sizeof(TrainLds), st, theta, (const __bf16*)X, T, n,
                     part, lpart);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_mlp_reduce, dim3((kMlpParams + 1 + 255) / 256), dim3(256), 0, st, part, lpart, grid, grad,
                     loss);
  return hipGetLastError();
}

hipError_t launch_mlp_adam(hipStream_t st, float* theta, float* m, float* v, const float* g, float lr, float b1,
                           float b2, float eps, float c1, float c2) {
  hipLaunchKernelGGL(k_mlp_adam, dim3((kMlpParams + 255) / 256), dim3(256), 0, st, theta, m, v, g, lr, b1, b2, eps, c1,
                     c2);
  return hipGetLastError();
}

}  // namespace lbm
