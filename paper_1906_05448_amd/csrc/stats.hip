// stats.hip - statistics of one snapshot (Sec. 3.2): kinetic energy and
// dissipation rate 2 nu <s_ij s_ij> (central differences), raw, masked by
// the rigid-body motion inside particles (zero in the pipe wall), and over
// fluid nodes; mass and momentum of the fluid; local profiles binned by the
// distance to the nearest surface (Sec. 3.2.1). Per-node arithmetic is FP64 on
// the FP32 velocity field and every sum is reduced in a fixed order (fixed
// by the lattice and the device's size), so the result does not change from
// run to run.
//
// Passes (u and rho extracted beforehand into idle population memory):
//   key      per node: 0 pipe wall, p + 1 inside sphere p (lowest index),
//            0x80000000 | bin for fluid within range, 0xFFFFFFFF otherwise;
//            the wall and its distance bins first, then one workgroup per
//            sphere lowers the keys of its box with atomicMin. The bin of
//            the nearest surface is the smallest bin over surfaces, since
//            floor is monotonic.
//   sums     one wavefront walks a 64-node row segment along z (runs of z
//            dealt out to a grid the device holds at once): raw, masked and
//            fluid sums and the histograms in one pass. The rows at z - 1
//            and z stay in registers, the x neighbours come from the lanes
//            beside (loaded only at the segment's ends), the y neighbours
//            from coalesced row loads; the velocity of a node inside a sphere
//            is U + Omega x (x - X) evaluated in FP64 where needed. Histogram
//            bins are summed per wavefront in LDS as exact two-word fixed
//            point (integer atomics, whose order does not matter), added
//            over the workgroup's wavefronts and rounded once to FP64.
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

// Motion of one sphere: position, velocity, angular velocity.
struct Rigid {
  double X[3], U[3], W[3];
};

__device__ __forceinline__ Rigid rigid_load(uint32_t p, const double* X, const double* U, const double* Om) {
  Rigid s;
  for (int c = 0; c < 3; ++c) {
    s.X[c] = X[3 * p + c];
    s.U[c] = U[3 * p + c];
    s.W[c] = Om[3 * p + c];
  }
  return s;
}

// Rigid-body velocity U + Omega x (x - X) of sphere s at node (x, y, z).
__device__ __forceinline__ Vel3 rigid_vel(const Rigid& s, int x, int y, int z, int nx, int ny, int nz) {
  const double r[3] = {min_image((double)x - s.X[0], nx), min_image((double)y - s.X[1], ny),
                       min_image((double)z - s.X[2], nz)};
  const double* w = s.W;
  Vel3 m;
  m.v[0] = s.U[0] + (w[1] * r[2] - w[2] * r[1]);
  m.v[1] = s.U[1] + (w[2] * r[0] - w[0] * r[2]);
  m.v[2] = s.U[2] + (w[0] * r[1] - w[1] * r[0]);
  return m;
}

// Rigid-body velocity of sphere p at node (x, y, z).
__device__ __forceinline__ Vel3 rigid_at(uint32_t p, int x, int y, int z, const double* X, const double* U,
                                      const double* Om, int nx, int ny, int nz) {
  return rigid_vel(rigid_load(p, X, U, Om), x, y, z, nx, ny, nz);
}

// Masked velocity of a node with key k: sphere ps's motion (already loaded
// into s, ps = kNoSphere if none) serves the nodes inside ps; a node inside
// another sphere loads that sphere's motion.
constexpr uint32_t kNoSphere = 0xFFFFFFFFu;

__device__ __forceinline__ void masked_at(uint32_t k, const float* v, int x, int y, int z, uint32_t ps,
                                          const Rigid& s, const double* X, const double* U, const double* Om,
                                          const Dims& d, double m[3]) {
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
  const Vel3 r = k - 1u == ps ? rigid_vel(s, x, y, z, d.nx, d.ny, d.nz)
                              : rigid_at(k - 1u, x, y, z, X, U, Om, d.nx, d.ny, d.nz);
  m[0] = r.v[0];
  m[1] = r.v[1];
  m[2] = r.v[2];
}

__device__ __forceinline__ bool in_sphere_key(uint32_t k) { return k < kKeyFluid && k != kKeyWall; }

constexpr int kSegWaves = kSBlock / 64;

// Velocity and key of one node.
struct Node {
  float u[3];
  uint32_t k;
};

__device__ __forceinline__ Node load_node(const float* __restrict__ u, const uint32_t* __restrict__ key, uint32_t N,
                                          uint32_t n) {
  Node v;
  v.u[0] = u[n];
  v.u[1] = u[(size_t)N + n];
  v.u[2] = u[2 * (size_t)N + n];
  v.k = key[n];
  return v;
}

__device__ __forceinline__ Node shfl_node(const Node& v, int src) {
  Node o;
  for (int c = 0; c < 3; ++c) o.u[c] = __shfl(v.u[c], src, 64);
  o.k = (uint32_t)__shfl((int)v.k, src, 64);
  return o;
}

// Fixed-point form of a histogram value v: v = hi 2^-32 + lo 2^-72 with
// hi = floor(v 2^32) (two's complement) and 0 <= lo <= 2^40. Scaling by
// powers of two, the floor and the fraction are exact in FP64; lo rounds
// off the bits below 2^-72, at most 2^-73 per value, far below the FP64
// rounding of a workgroup's sums. The integer sums themselves are exact. A
// workgroup sums at most 2^23 values (2^31 nodes over at least 256
// workgroups), which fits both words for |v| < 2^8.
__device__ __forceinline__ void fixed_split(double v, unsigned long long& hi, unsigned long long& lo) {
  const double t = v * 4294967296.0;  // 2^32
  const double a = floor(t);
  hi = (unsigned long long)(long long)a;
  lo = (unsigned long long)rint((t - a) * 1099511627776.0);  // 2^40
}

__device__ __forceinline__ double fixed_join(unsigned long long hi, unsigned long long lo) {
  return (double)(long long)hi * (1.0 / 4294967296.0) + (double)lo * (1.0 / 4722366482869645213696.0);
}

// Work of the sums pass: (64-node row segment, y) columns, each cut into
// z runs so that there are about eight runs per wavefront (the runs are
// dealt out in a fixed order; eight or more keep the last round short).
struct ZPlan {
  uint32_t segs, cols, nzc, zlen, items;
};

__host__ __device__ inline ZPlan zplan(int nx, int ny, int nz, uint32_t waves) {
  ZPlan z;
  z.segs = (uint32_t)(nx + 63) / 64u;
  z.cols = z.segs * (uint32_t)ny;
  uint32_t k = (8u * waves + z.cols - 1) / z.cols;
  k = k < 1u ? 1u : (k > (uint32_t)nz ? (uint32_t)nz : k);
  z.zlen = ((uint32_t)nz + k - 1) / k;
  z.nzc = ((uint32_t)nz + z.zlen - 1) / z.zlen;
  z.items = z.cols * z.nzc;
  return z;
}

// One wavefront walks a 64-node row segment along z: the rows at z - 1 and
// z stay in registers from the previous steps, so each step loads the row
// at z + 1, the rows at y - 1 and y + 1 (which the wavefronts of the
// neighbouring columns, on the same XCD, load as well) and the density; the
// x neighbours come from the lanes beside, the nodes beyond the segment's
// ends from two lanes' extra loads.
// Held at three wavefronts per SIMD (168 VGPRs, 8 spilled): uncapped, the
// loaded sphere motion takes it to 180 and two wavefronts.
__global__ void __launch_bounds__(kSBlock, 3)
k_stats_sums(const float* __restrict__ u, const float* __restrict__ rho, const uint32_t* __restrict__ key,
             const double* __restrict__ X, const double* __restrict__ U, const double* __restrict__ Om, Dims d,
             double nu, int nbins, double* __restrict__ part, int stride, ZPlan zp, uint32_t per_xcd) {
  extern __shared__ unsigned long long hist_lds[];  // [wave][5][2][nbins]: fixed-point words
  const int lane = (int)(threadIdx.x & 63u), wv = (int)(threadIdx.x >> 6);
  unsigned long long* hw = hist_lds + (size_t)wv * 10 * nbins;
  for (int i = lane; i < 10 * nbins; i += 64) hw[i] = 0ull;
  __builtin_amdgcn_wave_barrier();
  const int nx = d.nx, ny = d.ny, nz = d.nz;
  const uint32_t N = d.N;
  // XCD-major block order: the blocks of one XCD take consecutive columns
  const uint32_t logical = (blockIdx.x & 7u) * per_xcd + (blockIdx.x >> 3);
  const uint32_t waves = gridDim.x * kSegWaves;
  double s[kStatScalars] = {};
  double umax2 = 0.0;
  for (uint32_t it = logical * kSegWaves + (uint32_t)wv; it < zp.items; it += waves) {
    const uint32_t zc = it / zp.cols, col = it - zc * zp.cols;
    const uint32_t yy = col / zp.segs;
    const int x0 = (int)(col - yy * zp.segs) * 64, y = (int)yy;
    const int z0 = (int)(zc * zp.zlen), z1 = min(nz, z0 + (int)zp.zlen);
    const int x = x0 + lane;
    const bool live = x < nx;
    const int xc = live ? x : nx - 1;
    const int xl = xc == 0 ? nx - 1 : xc - 1, xr = xc == nx - 1 ? 0 : xc + 1;
    const int ym = y == 0 ? ny - 1 : y - 1, yp = y == ny - 1 ? 0 : y + 1;
    const bool need_l = lane == 0, need_r = lane == 63 || xc == nx - 1;
    auto at = [&](int xx, int yv, int zz) {
      return ((uint32_t)zz * (uint32_t)ny + (uint32_t)yv) * (uint32_t)nx + (uint32_t)xx;
    };
    Node zm = load_node(u, key, N, at(xc, y, z0 == 0 ? nz - 1 : z0 - 1));
    Node c0 = load_node(u, key, N, at(xc, y, z0));
    for (int z = z0; z < z1; ++z) {
      const int zpl = z == nz - 1 ? 0 : z + 1, zmi = z == 0 ? nz - 1 : z - 1;
      // every load of the step before any use
      const Node cz = load_node(u, key, N, at(xc, y, zpl));
      const Node ymn = load_node(u, key, N, at(xc, ym, z));
      const Node ypn = load_node(u, key, N, at(xc, yp, z));
      const float r0 = rho[at(xc, y, z)];
      Node hl, hr;
      if (need_l) hl = load_node(u, key, N, at(xl, y, z));
      if (need_r) hr = load_node(u, key, N, at(xr, y, z));
      Node xpn = shfl_node(c0, min(lane + 1, 63));
      Node xmn = shfl_node(c0, max(lane - 1, 0));
      if (need_r) xpn = hr;
      if (need_l) xmn = hl;
      // neighbours: x+, x-, y+, y-, z+, z-
      const Node* nb[6] = {&xpn, &xmn, &ypn, &ymn, &cz, &zm};
      // central-difference gradients in FP64, raw and (where a neighbour is
      // masked) masked
      bool any_masked = false;
#pragma unroll
      for (int j = 0; j < 6; ++j) any_masked = any_masked || nb[j]->k < kKeyFluid;
      double G[3][3];
#pragma unroll
      for (int ax = 0; ax < 3; ++ax)
        for (int c = 0; c < 3; ++c) G[c][ax] = 0.5 * ((double)nb[2 * ax]->u[c] - (double)nb[2 * ax + 1]->u[c]);
      const double eps_raw = dissipation_of(G, nu);
      double eps_m = eps_raw;
      // the sphere of the node or of its first neighbour inside one, whose
      // motion is loaded once for the node and its neighbours
      uint32_t ps = in_sphere_key(c0.k) ? c0.k - 1u : kNoSphere;
#pragma unroll
      for (int j = 0; j < 6; ++j)
        if (ps == kNoSphere && in_sphere_key(nb[j]->k)) ps = nb[j]->k - 1u;
      Rigid rs{};
      if (ps != kNoSphere) rs = rigid_load(ps, X, U, Om);
      if (any_masked) {
        const int nxs[6] = {xr, xl, xc, xc, xc, xc}, nys[6] = {y, y, yp, ym, y, y}, nzs[6] = {z, z, z, z, zpl, zmi};
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) {
          double mp[3], mm[3];
          const int a = 2 * ax, b = 2 * ax + 1;
          masked_at(nb[a]->k, nb[a]->u, nxs[a], nys[a], nzs[a], ps, rs, X, U, Om, d, mp);
          masked_at(nb[b]->k, nb[b]->u, nxs[b], nys[b], nzs[b], ps, rs, X, U, Om, d, mm);
          for (int c = 0; c < 3; ++c) G[c][ax] = 0.5 * (mp[c] - mm[c]);
        }
        eps_m = dissipation_of(G, nu);
      }
      const double vx = c0.u[0], vy = c0.u[1], vz = c0.u[2];
      const double ke = 0.5 * ((vx * vx + vy * vy) + vz * vz);
      const uint32_t k0 = c0.k;
      if (live) {
        double vm[3];
        masked_at(k0, c0.u, xc, y, z, ps, rs, X, U, Om, d, vm);
        s[kStatKeRaw] += ke;
        s[kStatEpsRaw] += eps_raw;
        s[kStatKeMasked] += 0.5 * ((vm[0] * vm[0] + vm[1] * vm[1]) + vm[2] * vm[2]);
        s[kStatEpsMasked] += eps_m;
        if (k0 >= kKeyFluid) {
          const double rr = r0;
          s[kStatNf] += 1.0;
          s[kStatMass] += rr;
          s[kStatMomX] += rr * vx;
          s[kStatMomY] += rr * vy;
          s[kStatMomZ] += rr * vz;
          s[kStatKeFluid] += ke;
          s[kStatBulk] += vz;
          s[kStatEpsFluid] += eps_m;
          umax2 = fmax(umax2, 2.0 * ke);
        }
      }
      zm = c0;
      c0 = cz;
      // histograms: fluid nodes within the profile range, summed exactly
      // in fixed point (integer sums do not depend on the order)
      const bool binned = live && k0 >= kKeyFluid && k0 != kKeyFar;
      if (binned) {
        const uint32_t bin = k0 & 0x7FFFFFFFu;
        atomicAdd(&hw[bin], 1ull);  // the node count, an integer
        const double val[4] = {ke, eps_m, vz, vz * vz};
#pragma unroll
        for (int c = 1; c < 5; ++c) {
          unsigned long long hi, lo;
          fixed_split(val[c - 1], hi, lo);
          atomicAdd(&hw[(size_t)(2 * c) * nbins + bin], hi);
          atomicAdd(&hw[(size_t)(2 * c + 1) * nbins + bin], lo);
        }
      }
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
  // the wavefronts' fixed-point histograms added as integers, then one
  // rounding to FP64 per block and bin
  __syncthreads();
  for (int i = threadIdx.x; i < 5 * nbins; i += kSBlock) {
    const int c = i / nbins, bin = i - c * nbins;
    unsigned long long hi = 0ull, lo = 0ull;
    for (int w = 0; w < kSegWaves; ++w) {
      hi += hist_lds[((size_t)w * 10 + 2 * c) * nbins + bin];
      lo += hist_lds[((size_t)w * 10 + 2 * c + 1) * nbins + bin];
    }
    out[kStatScalars + i] = c == 0 ? (double)hi : fixed_join(hi, lo);
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
  // The work is dealt out statically, so the grid is what the device holds
  // at once (whole XCD groups, at most kStatGrid blocks): no block waits for
  // another to finish. The sums then depend on the device's size but not on
  // the run.
  const size_t lds = (size_t)kSegWaves * 10 * std::max(nbins, 1) * sizeof(unsigned long long);
  int dev = 0, cus = 0, per_cu = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_stats_sums, kSBlock, lds);
  if (e != hipSuccess) return e;
  const uint32_t hold = std::max<uint32_t>(8u, (uint32_t)std::max(cus, 1) * (uint32_t)std::max(per_cu, 1));
  const uint32_t per_xcd = std::min<uint32_t>((uint32_t)kStatGrid, hold) / 8u;
  const int grid = (int)(8u * per_xcd);
  const ZPlan zp = zplan(d.nx, d.ny, d.nz, (uint32_t)grid * kSegWaves);
  e = launch_stats_keys(c, key, nbins, width, X);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_stats_sums, dim3(grid), dim3(kSBlock), lds, c.stream, u, rho, key, X, U, Om, d, nu, nbins, part,
                     stride, zp, per_xcd);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_stats_reduce, dim3(stride), dim3(kSBlock), 0, c.stream, part, grid, stride, out);
  return hipGetLastError();
}

}  // namespace lbm
