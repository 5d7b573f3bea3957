// stats.hip - statistics of one snapshot (Sec. 3.2): kinetic energy and
// dissipation rate 2 nu <s_ij s_ij> (central differences), raw, masked by
// the rigid-body motion inside particles (zero in the pipe wall), and over
// fluid nodes; mass and momentum of the fluid; local profiles binned by the
// distance to the nearest surface (Sec. 3.2.1). Per-node arithmetic is FP64 on
// the FP32 velocity field and every sum is reduced in a fixed order, so the
// result does not change from run to run.
//
// Passes (u and rho extracted beforehand into idle population memory):
//   key      per node: 0 pipe wall, p + 1 inside sphere p (lowest index),
//            0x80000000 | bin for fluid within range, 0xFFFFFFFF otherwise;
//            the wall and its distance bins first, then one workgroup per
//            sphere lowers the keys of its box with atomicMin. The bin of
//            the nearest surface is the smallest bin over surfaces, since
//            floor is monotonic.
//   raw      fixed grid, grid-stride: raw sums and the fluid sums
//   masked   masked sums and the histograms; the velocity of a node inside a
//            sphere is U + Omega x (x - X) evaluated in FP64 where needed
//   reduce   one workgroup per column adds the per-block partials in order
#include "device_util.hpp"
#include "internal.hpp"
#include "stats_device.hpp"

namespace lbm {

namespace {

constexpr int kSBlock = 256;

__device__ __forceinline__ bool binned_bin(double d, double width, int nbins, uint32_t& b) {
  if (!(d < (double)nbins * width)) return false;
  const double q = floor(d / width);
  if (q >= (double)nbins) return false;
  b = (uint32_t)q;
  return true;
}

__global__ void __launch_bounds__(kSBlock)
k_stats_key(Dims d, int wall, double R, double cx, double cy, int nbins, double width, uint32_t* __restrict__ key) {
  const uint32_t n = blockIdx.x * kSBlock + threadIdx.x;
  if (n >= d.N) return;
  uint32_t k = kKeyFar;
  if (wall == LBM_WALL_PIPE_Z) {
    int x, y, z;
    node_coords(n, d.nx, d.ny, x, y, z);
    const double dx = (double)x - cx, dy = (double)y - cy;
    const double r2 = dy * dy + dx * dx;
    uint32_t b;
    if (r2 >= R * R)
      k = kKeyWall;
    else if (binned_bin(R - sqrt(r2), width, nbins, b))
      k = kKeyFluid | b;
  }
  key[n] = k;
}

__global__ void __launch_bounds__(kSBlock)
k_stats_spheres(const double* __restrict__ X, const double* __restrict__ rad, Dims d, int nbins, double width,
                uint32_t* __restrict__ key) {
  const int p = blockIdx.x;
  const double* Xp = X + 3 * p;
  const double r = rad[p];
  const double range = (double)nbins * width;
  const Box b = make_box(Xp, r + range);
  const uint32_t total = b.count();
  const uint32_t own = (uint32_t)p + 1u;
  for (uint32_t i = threadIdx.x; i < total; i += kSBlock) {
    int x, y, z;
    box_node(b, i, d.nx, d.ny, d.nz, x, y, z);
    const double D2 = dist2(min_image((double)x - Xp[0], d.nx), min_image((double)y - Xp[1], d.ny),
                            min_image((double)z - Xp[2], d.nz));
    const uint32_t n = node_index(x, y, z, d.nx, d.ny);
    if (D2 < r * r) {
      atomicMin(key + n, own);
    } else {
      uint32_t bin;
      if (binned_bin(sqrt(D2) - r, width, nbins, bin)) atomicMin(key + n, kKeyFluid | bin);
    }
  }
}

__global__ void __launch_bounds__(kSBlock)
k_stats_raw(const float* __restrict__ u, const float* __restrict__ rho, const uint32_t* __restrict__ key, Dims d,
            double nu, double* __restrict__ part, int stride) {
  const RawVel vel{u, d.N};
  double s[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};  // kNf .. kBulk
  double umax2 = 0.0;
  for (uint32_t n = blockIdx.x * kSBlock + threadIdx.x; n < d.N; n += gridDim.x * kSBlock) {
    const Neigh g = neighbours(n, d);
    double v[3];
    vel.at(n, v);
    const double v2 = (v[0] * v[0] + v[1] * v[1]) + v[2] * v[2];
    const double ke = 0.5 * v2;
    s[kStatKeRaw] += ke;
    s[kStatEpsRaw] += dissipation(vel, g, nu);
    if (key[n] >= kKeyFluid) {
      const double r = rho[n];
      s[kStatNf] += 1.0;
      s[kStatMass] += r;
      s[kStatMomX] += r * v[0];
      s[kStatMomY] += r * v[1];
      s[kStatMomZ] += r * v[2];
      s[kStatKeFluid] += ke;
      s[kStatBulk] += v[2];
      umax2 = fmax(umax2, v2);
    }
  }
  block_sum_first<kSBlock, 10>(s);
  // the maximum is order-independent: a plain LDS reduction
  __shared__ double mx[kSBlock];
  mx[threadIdx.x] = umax2;
  __syncthreads();
  for (int o = kSBlock / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) mx[threadIdx.x] = fmax(mx[threadIdx.x], mx[threadIdx.x + o]);
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    double* out = part + (size_t)blockIdx.x * stride;
    for (int k = 0; k < 10; ++k)
      if (k != kStatUmax2) out[k] = s[k];
    out[kStatUmax2] = mx[0];
  }
}

// Histograms: lane l of a wavefront owns bins l, l + 64, ...; the binned
// nodes of an iteration are broadcast one at a time in lane order, so every
// bin is summed in a fixed order without atomics.
template <int SLOTS>
__global__ void __launch_bounds__(kSBlock)
k_stats_masked(const float* __restrict__ u, const uint32_t* __restrict__ key, const double* __restrict__ X,
               const double* __restrict__ U, const double* __restrict__ Om, Dims d, double nu, int nbins,
               double* __restrict__ part, int stride) {
  const MaskedVel vel{u, key, X, U, Om, d};
  const RawVel raw{u, d.N};
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  double s[3] = {0, 0, 0};  // ke masked, eps masked, eps fluid
  double h[SLOTS][5];
#pragma unroll
  for (int j = 0; j < SLOTS; ++j)
    for (int k = 0; k < 5; ++k) h[j][k] = 0.0;
  for (uint32_t base = blockIdx.x * kSBlock; base < d.N; base += gridDim.x * kSBlock) {
    const uint32_t n = base + threadIdx.x;
    bool binned = false;
    uint32_t bin = 0;
    double val[5] = {0, 0, 0, 0, 0};
    if (n < d.N) {
      const Neigh g = neighbours(n, d);
      const uint32_t k = key[n];
      double v[3];
      vel.at(n, v);
      const double ke = 0.5 * ((v[0] * v[0] + v[1] * v[1]) + v[2] * v[2]);
      const double eps = dissipation(vel, g, nu);
      s[0] += ke;
      s[1] += eps;
      if (k >= kKeyFluid) {
        s[2] += eps;
        if (k != kKeyFar) {
          binned = true;
          bin = k & 0x7FFFFFFFu;
          raw.at(n, v);
          val[0] = 1.0;
          val[1] = ke;
          val[2] = eps;
          val[3] = v[2];
          val[4] = v[2] * v[2];
        }
      }
    }
    unsigned long long m = __ballot(binned);
    while (m) {
      const int src = __ffsll(m) - 1;
      m &= m - 1ull;
      const int b = __builtin_amdgcn_readlane((int)bin, src);
      double w[5];
      for (int k = 0; k < 5; ++k) w[k] = readlane_d(val[k], src);
#pragma unroll
      for (int j = 0; j < SLOTS; ++j)
        if ((b >> 6) == j && (b & 63) == lane)
          for (int k = 0; k < 5; ++k) h[j][k] += w[k];
    }
  }
  block_sum_first<kSBlock, 3>(s);
  __shared__ double hs[kSBlock / 64][5][64 * SLOTS];
#pragma unroll
  for (int j = 0; j < SLOTS; ++j)
    for (int k = 0; k < 5; ++k) hs[wave][k][j * 64 + lane] = h[j][k];
  __syncthreads();
  double* out = part + (size_t)blockIdx.x * stride;
  if (threadIdx.x == 0) {
    out[kStatKeMasked] = s[0];
    out[kStatEpsMasked] = s[1];
    out[kStatEpsFluid] = s[2];
  }
  for (int i = threadIdx.x; i < 5 * nbins; i += kSBlock) {
    const int k = i / nbins, b = i % nbins;
    double t = 0.0;
    for (int w = 0; w < kSBlock / 64; ++w) t += hs[w][k][b];
    out[kStatScalars + i] = t;
  }
}

__global__ void __launch_bounds__(kSBlock)
k_stats_reduce(const double* __restrict__ part, int nblocks, int stride, double* __restrict__ out) {
  const int col = blockIdx.x;
  const bool is_max = col == kStatUmax2;
  double s = 0.0;
  for (int b = threadIdx.x; b < nblocks; b += kSBlock) {
    const double v = part[(size_t)b * stride + col];
    s = is_max ? fmax(s, v) : s + v;
  }
  if (is_max) {
    __shared__ double mx[kSBlock];
    mx[threadIdx.x] = s;
    __syncthreads();
    for (int o = kSBlock / 2; o > 0; o >>= 1) {
      if ((int)threadIdx.x < o) mx[threadIdx.x] = fmax(mx[threadIdx.x], mx[threadIdx.x + o]);
      __syncthreads();
    }
    if (threadIdx.x == 0) out[col] = mx[0];
    return;
  }
  double v[1] = {s};
  block_sum_first<kSBlock, 1>(v);
  if (threadIdx.x == 0) out[col] = v[0];
}

}  // namespace

size_t stats_part_bytes() {
  // per-block partials, the statistics sums, the corrector sums
  return ((size_t)kStatGrid * kStatStride + 2 * kStatStride) * sizeof(double);
}

hipError_t launch_stats_keys(const Ctx& c, uint32_t* key, int nbins, double width, const double* X) {
  const Dims& d = c.dims;
  hipLaunchKernelGGL(k_stats_key, dim3((d.N + kSBlock - 1) / kSBlock), dim3(kSBlock), 0, c.stream, d, c.cfg.wall,
                     c.cfg.pipe_radius, c.cfg.pipe_cx, c.cfg.pipe_cy, nbins, width, key);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (c.np > 0) {
    hipLaunchKernelGGL(k_stats_spheres, dim3(c.np), dim3(kSBlock), 0, c.stream, X, c.P.r, d, nbins, width, key);
    e = hipGetLastError();
  }
  return e;
}

hipError_t launch_stats(const Ctx& c, const float* u, const float* rho, uint32_t* key, int nbins, double width,
                        const double* X, const double* U, const double* Om, double* part, double* out) {
  const Dims& d = c.dims;
  const double nu = (c.cfg.tau - 0.5) / 3.0;
  const int stride = kStatScalars + 5 * nbins;
  const int grid = (int)std::min<uint32_t>((uint32_t)kStatGrid, (d.N + kSBlock - 1) / kSBlock);
  hipError_t e = launch_stats_keys(c, key, nbins, width, X);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_stats_raw, dim3(grid), dim3(kSBlock), 0, c.stream, u, rho, key, d, nu, part, stride);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if (nbins <= 64)
    hipLaunchKernelGGL(k_stats_masked<1>, dim3(grid), dim3(kSBlock), 0, c.stream, u, key, X, U, Om, d, nu, nbins,
                       part, stride);
  else if (nbins <= 128)
    hipLaunchKernelGGL(k_stats_masked<2>, dim3(grid), dim3(kSBlock), 0, c.stream, u, key, X, U, Om, d, nu, nbins,
                       part, stride);
  else
    hipLaunchKernelGGL(k_stats_masked<4>, dim3(grid), dim3(kSBlock), 0, c.stream, u, key, X, U, Om, d, nu, nbins,
                       part, stride);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_stats_reduce, dim3(stride), dim3(kSBlock), 0, c.stream, part, grid, stride, out);
  return hipGetLastError();
}

}  // namespace lbm
