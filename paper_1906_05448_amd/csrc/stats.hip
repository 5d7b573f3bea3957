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
//   sums     one wavefront per 64-node row segment, segments dealt out to a
//            fixed grid: raw, masked and fluid sums and the histograms in one
//            pass. The x neighbours come from the lanes beside (loaded only
//            at the segment's ends), the y and z neighbours from coalesced
//            row loads; the velocity of a node inside a sphere is
//            U + Omega x (x - X) evaluated in FP64 where needed. Histogram
//            bins are summed per wavefront in LDS: the binned lanes are
//            ranked among the lanes of the same bin, and rank by rank each
//            adds its values with a plain read-modify-write, so a bin's sum
//            follows lane order and then segment order: reproducible.
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

// Velocity of node (x, y, z) with key k as the masked statistics see it:
// the lattice value v in fluid, zero in the wall, the rigid-body motion of
// the sphere inside it (FP64).
struct Vel3 {
  double v[3];
};

// Rigid-body velocity of sphere p at node (x, y, z).
__device__ __forceinline__ Vel3 rigid_at(uint32_t p, int x, int y, int z, const double* X, const double* U,
                                      const double* Om, int nx, int ny, int nz) {
  const double r[3] = {min_image((double)x - X[3 * p], nx), min_image((double)y - X[3 * p + 1], ny),
                       min_image((double)z - X[3 * p + 2], nz)};
  const double* w = Om + 3 * p;
  Vel3 m;
  m.v[0] = U[3 * p] + (w[1] * r[2] - w[2] * r[1]);
  m.v[1] = U[3 * p + 1] + (w[2] * r[0] - w[0] * r[2]);
  m.v[2] = U[3 * p + 2] + (w[0] * r[1] - w[1] * r[0]);
  return m;
}

__device__ __forceinline__ void masked_at(uint32_t k, const float* v, int x, int y, int z, const double* X,
                                          const double* U, const double* Om, const Dims& d, double m[3]) {
  if (k >= kKeyFluid) {
    m[0] = v[0];
    m[1] = v[1];
    m[2] = v[2];
    return;
  }
  if (k == kKeyWall) {
    m[0] = m[1] = m[2] = 0.0;
    return;
  }
  const Vel3 r = rigid_at(k - 1u, x, y, z, X, U, Om, d.nx, d.ny, d.nz);
  m[0] = r.v[0];
  m[1] = r.v[1];
  m[2] = r.v[2];
}

constexpr int kSegWaves = kSBlock / 64;

__global__ void __launch_bounds__(kSBlock)
k_stats_sums(const float* __restrict__ u, const float* __restrict__ rho, const uint32_t* __restrict__ key,
             const double* __restrict__ X, const double* __restrict__ U, const double* __restrict__ Om, Dims d,
             double nu, int nbins, double* __restrict__ part, int stride) {
  extern __shared__ double hist_lds[];  // [wave][5][nbins]
  const int lane = (int)(threadIdx.x & 63u), wv = (int)(threadIdx.x >> 6);
  double* hw = hist_lds + (size_t)wv * 5 * nbins;
  for (int i = lane; i < 5 * nbins; i += 64) hw[i] = 0.0;
  __builtin_amdgcn_wave_barrier();
  const int nx = d.nx, ny = d.ny, nz = d.nz;
  const uint32_t N = d.N;
  const uint32_t segs = (uint32_t)(nx + 63) / 64u;
  const uint32_t total = segs * (uint32_t)ny * (uint32_t)nz;
  double s[kStatScalars] = {};
  double umax2 = 0.0;
  const unsigned long long lt = (1ull << lane) - 1ull;
  for (uint32_t sg = blockIdx.x * kSegWaves + (uint32_t)wv; sg < total; sg += gridDim.x * kSegWaves) {
    const uint32_t row = sg / segs;
    const int x0 = (int)(sg - row * segs) * 64;
    const int y = (int)(row % (uint32_t)ny), z = (int)(row / (uint32_t)ny);
    const int x = x0 + lane;
    const bool live = x < nx;
    const int xc = live ? x : nx - 1;
    const int xl = xc == 0 ? nx - 1 : xc - 1, xr = xc == nx - 1 ? 0 : xc + 1;
    const int ym = y == 0 ? ny - 1 : y - 1, yp = y == ny - 1 ? 0 : y + 1;
    const int zm = z == 0 ? nz - 1 : z - 1, zp = z == nz - 1 ? 0 : z + 1;
    auto at = [&](int xx, int yy, int zz) {
      return ((uint32_t)zz * (uint32_t)ny + (uint32_t)yy) * (uint32_t)nx + (uint32_t)xx;
    };
    // nodes: centre, x+, x-, y+, y-, z+, z-; the x neighbours come from the
    // lanes beside except at the segment's ends
    const int nxs[7] = {xc, xr, xl, xc, xc, xc, xc}, nys[7] = {y, y, y, yp, ym, y, y},
              nzs[7] = {z, z, z, z, z, zp, zm};
    uint32_t kk[7];
    float vf[7][3];
#pragma unroll
    for (int j = 0; j < 7; ++j) {
      if (j == 1 || j == 2) continue;
      const uint32_t n = at(nxs[j], nys[j], nzs[j]);
      kk[j] = key[n];
      for (int c = 0; c < 3; ++c) vf[j][c] = u[(size_t)c * N + n];
    }
    const float r0 = rho[at(xc, y, z)];
    kk[1] = (uint32_t)__shfl_down((int)kk[0], 1, 64);
    kk[2] = (uint32_t)__shfl_up((int)kk[0], 1, 64);
    for (int c = 0; c < 3; ++c) {
      vf[1][c] = __shfl_down(vf[0][c], 1, 64);
      vf[2][c] = __shfl_up(vf[0][c], 1, 64);
    }
    if (lane == 63 || xc == nx - 1) {
      const uint32_t n = at(xr, y, z);
      kk[1] = key[n];
      for (int c = 0; c < 3; ++c) vf[1][c] = u[(size_t)c * N + n];
    }
    if (lane == 0) {
      const uint32_t n = at(xl, y, z);
      kk[2] = key[n];
      for (int c = 0; c < 3; ++c) vf[2][c] = u[(size_t)c * N + n];
    }
    // central-difference gradients in FP64, raw and (where a neighbour is
    // masked) masked
    bool any_masked = false;
#pragma unroll
    for (int j = 1; j < 7; ++j) any_masked = any_masked || kk[j] < kKeyFluid;
    double G[3][3];
#pragma unroll
    for (int ax = 0; ax < 3; ++ax)
      for (int c = 0; c < 3; ++c) G[c][ax] = 0.5 * ((double)vf[1 + 2 * ax][c] - (double)vf[2 + 2 * ax][c]);
    const double eps_raw = dissipation_of(G, nu);
    double eps_m = eps_raw;
    if (any_masked) {
#pragma unroll
      for (int ax = 0; ax < 3; ++ax) {
        double mp[3], mm[3];
        masked_at(kk[1 + 2 * ax], vf[1 + 2 * ax], nxs[1 + 2 * ax], nys[1 + 2 * ax], nzs[1 + 2 * ax], X, U, Om, d, mp);
        masked_at(kk[2 + 2 * ax], vf[2 + 2 * ax], nxs[2 + 2 * ax], nys[2 + 2 * ax], nzs[2 + 2 * ax], X, U, Om, d, mm);
        for (int c = 0; c < 3; ++c) G[c][ax] = 0.5 * (mp[c] - mm[c]);
      }
      eps_m = dissipation_of(G, nu);
    }
    const double vx = vf[0][0], vy = vf[0][1], vz = vf[0][2];
    const double ke = 0.5 * ((vx * vx + vy * vy) + vz * vz);
    if (live) {
      double vm[3];
      masked_at(kk[0], vf[0], xc, y, z, X, U, Om, d, vm);
      s[kStatKeRaw] += ke;
      s[kStatEpsRaw] += eps_raw;
      s[kStatKeMasked] += 0.5 * ((vm[0] * vm[0] + vm[1] * vm[1]) + vm[2] * vm[2]);
      s[kStatEpsMasked] += eps_m;
      if (kk[0] >= kKeyFluid) {
        const double r = r0;
        s[kStatNf] += 1.0;
        s[kStatMass] += r;
        s[kStatMomX] += r * vx;
        s[kStatMomY] += r * vy;
        s[kStatMomZ] += r * vz;
        s[kStatKeFluid] += ke;
        s[kStatBulk] += vz;
        s[kStatEpsFluid] += eps_m;
        umax2 = fmax(umax2, 2.0 * ke);
      }
    }
    // histograms: fluid nodes within the profile range
    const bool binned = live && kk[0] >= kKeyFluid && kk[0] != kKeyFar;
    const uint32_t bin = kk[0] & 0x7FFFFFFFu;
    unsigned long long todo = __ballot(binned);
    if (todo == 0ull) continue;
    uint32_t rank = 0, maxrank = 0;
    while (todo) {
      const int leader = __ffsll((long long)todo) - 1;
      const uint32_t b = (uint32_t)__builtin_amdgcn_readlane((int)bin, leader);
      const unsigned long long m = __ballot(binned && bin == b);
      if (binned && bin == b) rank = (uint32_t)__popcll(m & lt);
      maxrank = max(maxrank, (uint32_t)__popcll(m) - 1u);
      todo &= ~m;
    }
    const double val[5] = {1.0, ke, eps_m, vz, vz * vz};
    for (uint32_t t = 0; t <= maxrank; ++t) {
      if (binned && rank == t)
        for (int c = 0; c < 5; ++c) hw[(size_t)c * nbins + bin] += val[c];
      __builtin_amdgcn_wave_barrier();
    }
  }
  s[kStatUmax2] = 0.0;
  block_sum_first<kSBlock, kStatScalars>(s);
  // the maximum is order-independent: a plain LDS reduction
  __shared__ double mx[kSBlock];
  mx[threadIdx.x] = umax2;
  __syncthreads();
  for (int o = kSBlock / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) mx[threadIdx.x] = fmax(mx[threadIdx.x], mx[threadIdx.x + o]);
    __syncthreads();
  }
  double* out = part + (size_t)blockIdx.x * stride;
  if (threadIdx.x == 0) {
    for (int c = 0; c < kStatScalars; ++c) out[c] = s[c];
    out[kStatUmax2] = mx[0];
  }
  // wavefront histograms added in wavefront order
  for (int i = threadIdx.x; i < 5 * nbins; i += kSBlock) {
    double t = 0.0;
    for (int w = 0; w < kSegWaves; ++w) t += hist_lds[(size_t)w * 5 * nbins + i];
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
  hipLaunchKernelGGL(k_stats_sums, dim3(grid), dim3(kSBlock), (size_t)kSegWaves * 5 * std::max(nbins, 1) * sizeof(double),
                     c.stream, u, rho, key, X, U, Om, d, nu, nbins, part, stride);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_stats_reduce, dim3(stride), dim3(kSBlock), 0, c.stream, part, grid, stride, out);
  return hipGetLastError();
}

}  // namespace lbm
