// corrector.hip - interface cells, features and training labels of the
// learned gradient corrector, and its use in the statistics.
//
// Interface cells of sphere p: fluid nodes with r_p <= |x - X_p| <
// r_p - r_d + 2, d = |x - X_p| - r_p within [d_min, d_max], and no other
// sphere q with |x - X_q| < r_q - r_d + 2 + sqrt(3) (its band or interior
// within the 3x3x3 stencil; also a gap below two spacings). Every sphere
// marks its exclusion zone in two bitmasks (seen once / seen twice); a band
// node seen only once is a cell. The cell bitmask is compacted to an
// ascending node list.
//
// Features (85 per cell, BF16 rows of 96): for the 27 offsets o, z slowest
// and x fastest, and components c, (u_c(x + o) - [U_p + Omega_p x
// (x + o - X_p)]_c) / u_rms; then d; then (x - X_p) / |x - X_p|. Labels:
// central-difference G_ij = d_j u_i of the masked field, / u_rms, rows of 16
// (written, or subtracted from what the rows hold: the training target is
// the reference labels minus the plain immersed-boundary labels). The
// network output y corrects the plain gradient: G = G_plain + u_rms y.
// The statistics kernel gathers each wavefront's 16 cells' features into an
// LDS tile, runs the network on the matrix cores, and adds eps(predicted G)
// - eps(central difference) per cell, in a fixed order.
#include "device_util.hpp"
#include "internal.hpp"
#include "mlp_device.hpp"
#include "stats_device.hpp"

namespace lbm {

namespace {

constexpr int kCBlock = 256;
constexpr double kSqrt3 = 1.7320508075688772;

__device__ __forceinline__ double band_outer(double r, double rd) { return (r - rd) + 2.0; }
__device__ __forceinline__ double excl_radius(double r, double rd) { return ((r - rd) + 2.0) + kSqrt3; }

__device__ __forceinline__ double sphere_d2(const double* Xp, int x, int y, int z, const Dims& d) {
  return dist2(min_image((double)x - Xp[0], d.nx), min_image((double)y - Xp[1], d.ny),
               min_image((double)z - Xp[2], d.nz));
}

__global__ void __launch_bounds__(kCBlock)
k_corr_zone(const double* __restrict__ X, const double* __restrict__ rad, Dims d, double rd, uint32_t* __restrict__ once,
            uint32_t* __restrict__ twice) {
  const int p = blockIdx.x;
  const double* Xp = X + 3 * p;
  const double re = excl_radius(rad[p], rd);
  const Box b = make_box(Xp, re);
  // one thread per (row, run of 32 x positions): the nodes of a run that fall
  // into one bitmask word are marked with one atomic
  const int runs = (b.side[0] + 31) / 32;
  const int items = runs * b.side[1] * b.side[2];
  for (int it = threadIdx.x; it < items; it += kCBlock) {
    const int rowi = it / runs, run = it - rowi * runs;
    const int y = wrapi(b.lo[1] + rowi % b.side[1], d.ny), z = wrapi(b.lo[2] + rowi / b.side[1], d.nz);
    const int i0 = run * 32, i1 = min(b.side[0], i0 + 32);
    uint32_t word = 0xFFFFFFFFu, bits = 0u;
    auto flush = [&]() {
      if (bits) {
        const uint32_t old = atomicOr(once + word, bits);
        if (old & bits) atomicOr(twice + word, old & bits);
      }
    };
    for (int ix = i0; ix < i1; ++ix) {
      const int x = wrapi(b.lo[0] + ix, d.nx);
      if (!(sphere_d2(Xp, x, y, z, d) < re * re)) continue;
      const uint32_t n = node_index(x, y, z, d.nx, d.ny);
      if ((n >> 5) != word) {
        flush();
        word = n >> 5;
        bits = 0u;
      }
      bits |= 1u << (n & 31u);
    }
    flush();
  }
}

__global__ void __launch_bounds__(kCBlock)
k_corr_band(const double* __restrict__ X, const double* __restrict__ rad, Dims d, double rd, double dmin, double dmax,
            const uint32_t* __restrict__ twice, uint32_t* __restrict__ cellbits, uint32_t* __restrict__ cellp) {
  const int p = blockIdx.x;
  const double* Xp = X + 3 * p;
  const double r = rad[p], ro = band_outer(r, rd);
  const Box b = make_box(Xp, ro);
  const uint32_t total = b.count();
  for (uint32_t i = threadIdx.x; i < total; i += kCBlock) {
    int x, y, z;
    box_node(b, i, d.nx, d.ny, d.nz, x, y, z);
    const double D2 = sphere_d2(Xp, x, y, z, d);
    if (!(D2 >= r * r && D2 < ro * ro)) continue;
    const double dd = sqrt(D2) - r;
    if (!(dd >= dmin && dd <= dmax)) continue;
    const uint32_t n = node_index(x, y, z, d.nx, d.ny);
    const uint32_t bit = 1u << (n & 31u);
    if (twice[n >> 5] & bit) continue;
    atomicOr(cellbits + (n >> 5), bit);
    cellp[n] = (uint32_t)p;
  }
}

__global__ void __launch_bounds__(kCBlock)
k_corr_particles(const uint32_t* __restrict__ list, const uint32_t* __restrict__ count, uint32_t cap,
                 const uint32_t* __restrict__ cellp, uint32_t* __restrict__ plist) {
  const uint32_t i = blockIdx.x * kCBlock + threadIdx.x;
  if (i < cap && i < *count) plist[i] = cellp[list[i]];
}

// One interface cell: its node, sphere and the offset to the centre.
struct Cell {
  int x, y, z;
  const double *X, *U, *W;
  double r, rr[3], dist;
};

__device__ __forceinline__ Cell make_cell(uint32_t node, uint32_t p, const double* X, const double* U, const double* Om,
                                          const double* rad, const Dims& d) {
  Cell c;
  node_coords(node, d.nx, d.ny, c.x, c.y, c.z);
  c.X = X + 3 * p;
  c.U = U + 3 * p;
  c.W = Om + 3 * p;
  c.r = rad[p];
  c.rr[0] = min_image((double)c.x - c.X[0], d.nx);
  c.rr[1] = min_image((double)c.y - c.X[1], d.ny);
  c.rr[2] = min_image((double)c.z - c.X[2], d.nz);
  c.dist = sqrt(dist2(c.rr[0], c.rr[1], c.rr[2]));
  return c;
}

__device__ __forceinline__ float cell_feature(int f, const Cell& c, const float* __restrict__ u, const Dims& d,
                                              double u_rms) {
  if (f < 81) {
    const int o = f / 3, k = f - 3 * o;
    const int xn = wrap1(c.x + o % 3 - 1, d.nx), yn = wrap1(c.y + (o / 3) % 3 - 1, d.ny),
              zn = wrap1(c.z + o / 9 - 1, d.nz);
    const double r0 = min_image((double)xn - c.X[0], d.nx), r1 = min_image((double)yn - c.X[1], d.ny),
                 r2 = min_image((double)zn - c.X[2], d.nz);
    const double rig = k == 0 ? c.U[0] + (c.W[1] * r2 - c.W[2] * r1)
                              : (k == 1 ? c.U[1] + (c.W[2] * r0 - c.W[0] * r2) : c.U[2] + (c.W[0] * r1 - c.W[1] * r0));
    const uint32_t n = node_index(xn, yn, zn, d.nx, d.ny);
    return (float)(((double)u[(size_t)k * d.N + n] - rig) / u_rms);
  }
  if (f == 81) return (float)(c.dist - c.r);
  if (f == 82) return (float)(c.rr[0] / c.dist);
  if (f == 83) return (float)(c.rr[1] / c.dist);
  if (f == 84) return (float)(c.rr[2] / c.dist);
  return 0.0f;
}

// Feature f < 81 from its velocity value (feature_from), the others as
// cell_feature gives them.
__device__ __forceinline__ float cell_feature_from(int f, const Cell& c, float uval, const Dims& d, double u_rms) {
  if (f < 81) {
    const int o = f / 3, k = f - 3 * o;
    const int xn = wrap1(c.x + o % 3 - 1, d.nx), yn = wrap1(c.y + (o / 3) % 3 - 1, d.ny),
              zn = wrap1(c.z + o / 9 - 1, d.nz);
    const double r0 = min_image((double)xn - c.X[0], d.nx), r1 = min_image((double)yn - c.X[1], d.ny),
                 r2 = min_image((double)zn - c.X[2], d.nz);
    const double rig = k == 0 ? c.U[0] + (c.W[1] * r2 - c.W[2] * r1)
                              : (k == 1 ? c.U[1] + (c.W[2] * r0 - c.W[0] * r2) : c.U[2] + (c.W[0] * r1 - c.W[1] * r0));
    return (float)(((double)uval - rig) / u_rms);
  }
  return cell_feature(f, c, nullptr, d, u_rms);
}

// Thread per (cell, group of 8 features): one 16-byte store.
__global__ void __launch_bounds__(kCBlock)
k_corr_features(const uint32_t* __restrict__ list, const uint32_t* __restrict__ plist, const uint32_t* __restrict__ count,
                uint32_t cap, const float* __restrict__ u, const double* __restrict__ X, const double* __restrict__ U,
                const double* __restrict__ Om, const double* __restrict__ rad, Dims d, double u_rms,
                __bf16* __restrict__ out) {
  const uint64_t t = (uint64_t)blockIdx.x * kCBlock + threadIdx.x;
  const uint64_t i = t / 12;
  const int g = (int)(t % 12);
  const uint32_t n = min(*count, cap);
  if (i >= n) return;
  const Cell c = make_cell(list[i], plist[i], X, U, Om, rad, d);
  bf16x8 v;
#pragma unroll
  for (int e = 0; e < 8; ++e) v[e] = (__bf16)cell_feature(g * 8 + e, c, u, d, u_rms);
  *(bf16x8*)(out + i * kMlpInPad + g * 8) = v;
}

__global__ void __launch_bounds__(kCBlock)
k_corr_labels(const uint32_t* __restrict__ list, uint32_t n, const float* __restrict__ u,
              const uint32_t* __restrict__ key, const double* __restrict__ X, const double* __restrict__ U,
              const double* __restrict__ Om, Dims d, double u_rms, int subtract, float* __restrict__ out) {
  const uint32_t i = blockIdx.x * kCBlock + threadIdx.x;
  if (i >= n) return;
  const MaskedVel vel{u, key, X, U, Om, d};
  double G[3][3];
  velocity_gradient(vel, neighbours(list[i], d), G);
  float* o = out + (size_t)i * kMlpOutPad;
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) {
      const float g = (float)(G[a][b] / u_rms);
      o[3 * a + b] = subtract ? o[3 * a + b] - g : g;
    }
  for (int k = kMlpOut; k < kMlpOutPad; ++k) o[k] = 0.0f;
}

struct CorrLds {
  MlpWeights w;
  __bf16 h1[kCBlock / 64][16][kMlpHid], h2[kCBlock / 64][16][kMlpHid];
  float ys[kCBlock / 64][16][kMlpOutPad];
  __bf16 xs[kCBlock / 64][16][kMlpInPad];
  double hs[kCBlock / 64][4 * 64];
};

// Sum over corrected cells of eps(G_plain + u_rms y) - eps(G_plain), with
// G_plain the central difference of the masked field,
// their number and the per-bin sums. part: [gridDim.x][stride], columns
// (sum, count, bins...).
template <int SLOTS>
__global__ void __launch_bounds__(kCBlock)
k_corr_stats(const float* __restrict__ theta, const uint32_t* __restrict__ list, const uint32_t* __restrict__ plist,
             const uint32_t* __restrict__ count, uint32_t cap, const float* __restrict__ u,
             const uint32_t* __restrict__ key, const double* __restrict__ X, const double* __restrict__ U,
             const double* __restrict__ Om, const double* __restrict__ rad, Dims d, double u_rms, double nu, int nbins,
             double* __restrict__ part, int stride) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  CorrLds& s = *(CorrLds*)lds_raw;
  mlp_load_weights<kCBlock>(theta, s.w);
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, col = lane & 15, grp = lane >> 4;
  const uint32_t n = min(*count, cap);
  const MaskedVel vel{u, key, X, U, Om, d};
  double sum = 0.0, cnt = 0.0;
  double h[SLOTS];
#pragma unroll
  for (int j = 0; j < SLOTS; ++j) h[j] = 0.0;
  for (uint32_t c0 = blockIdx.x * 64u; c0 < n; c0 += gridDim.x * 64u) {
    const uint32_t ci = c0 + wave * 16 + col;
    const bool valid = ci < n;
    // features of the wave's 16 cells: lane group g fills entries 24g .. 24g + 23
    __bf16* xrow = &s.xs[wave][col][0];
    if (valid) {
      const Cell c = make_cell(list[ci], plist[ci], X, U, Om, rad, d);
      // lane group g takes the stencil offsets g, g + 4, ...: every velocity
      // load of the lane issued before the first is used
      float raw[7][3];
#pragma unroll
      for (int j = 0; j < 7; ++j) {
        const int o = grp + 4 * j;
        raw[j][0] = raw[j][1] = raw[j][2] = 0.0f;
        if (o < 27) {
          const uint32_t nn = node_index(wrap1(c.x + o % 3 - 1, d.nx), wrap1(c.y + (o / 3) % 3 - 1, d.ny),
                                         wrap1(c.z + o / 9 - 1, d.nz), d.nx, d.ny);
          for (int k = 0; k < 3; ++k) raw[j][k] = u[(size_t)k * d.N + nn];
        }
      }
#pragma unroll
      for (int j = 0; j < 7; ++j) {
        const int o = grp + 4 * j;
        if (o < 27)
          for (int k = 0; k < 3; ++k) xrow[3 * o + k] = (__bf16)cell_feature_from(3 * o + k, c, raw[j][k], d, u_rms);
      }
      if (grp == 3)
        for (int f = 81; f < kMlpInPad; ++f) xrow[f] = (__bf16)cell_feature(f, c, nullptr, d, u_rms);
    } else {
#pragma unroll 1
      for (int t = 0; t < 24; ++t) xrow[grp * 24 + t] = (__bf16)0.0f;
    }
    __builtin_amdgcn_s_waitcnt(0xc07f);
    __builtin_amdgcn_wave_barrier();
    bf16x8 a[3];
#pragma unroll
    for (int ks = 0; ks < 3; ++ks) a[ks] = lds8(&s.xs[wave][col][ks * 32 + grp * 8]);
    const f32x4 y = mlp_forward_tile(a, s.w, &s.h1[wave][0][0], &s.h2[wave][0][0], nullptr, nullptr);
#pragma unroll
    for (int e = 0; e < 4; ++e) s.ys[wave][grp * 4 + e][col] = y[e];
    __builtin_amdgcn_s_waitcnt(0xc07f);
    __builtin_amdgcn_wave_barrier();
    bool binned = false;
    uint32_t bin = 0;
    double delta = 0.0;
    if (grp == 0 && valid) {
      const uint32_t node = list[ci];
      double Gp[3][3], G[3][3];
      velocity_gradient(vel, neighbours(node, d), Gp);
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) G[i][j] = Gp[i][j] + (double)s.ys[wave][col][3 * i + j] * u_rms;
      delta = dissipation_of(G, nu) - dissipation_of(Gp, nu);
      sum += delta;
      cnt += 1.0;
      const uint32_t k = key[node];
      if (k >= kKeyFluid && k != kKeyFar) {
        binned = true;
        bin = k & 0x7FFFFFFFu;
      }
    }
    unsigned long long m = __ballot(binned);
    while (m) {
      const int src = __ffsll(m) - 1;
      m &= m - 1ull;
      const int b = __builtin_amdgcn_readlane((int)bin, src);
      const double w = readlane_d(delta, src);
#pragma unroll
      for (int j = 0; j < SLOTS; ++j)
        if ((b >> 6) == j && (b & 63) == lane) h[j] += w;
    }
  }
  double sc[2] = {sum, cnt};
  block_sum_first<kCBlock, 2>(sc);
#pragma unroll
  for (int j = 0; j < SLOTS; ++j) s.hs[wave][j * 64 + lane] = h[j];
  __syncthreads();
  double* out = part + (size_t)blockIdx.x * stride;
  if (threadIdx.x == 0) {
    out[0] = sc[0];
    out[1] = sc[1];
  }
  for (int b = threadIdx.x; b < nbins; b += kCBlock) {
    double t = 0.0;
    for (int w = 0; w < kCBlock / 64; ++w) t += s.hs[w][b];
    out[2 + b] = t;
  }
}

__global__ void __launch_bounds__(kCBlock)
k_corr_reduce(const double* __restrict__ part, int nblocks, int stride, double* __restrict__ out) {
  const int colm = blockIdx.x;
  double v[1] = {0.0};
  for (int b = threadIdx.x; b < nblocks; b += kCBlock) v[0] += part[(size_t)b * stride + colm];
  block_sum_first<kCBlock, 1>(v);
  if (threadIdx.x == 0) out[colm] = v[0];
}

}  // namespace

hipError_t launch_corrector_cells(const Ctx& c, const double* X, double dmin, double dmax, const CorrBufs& b,
                                  uint32_t* list, uint32_t* plist, uint32_t cap) {
  const Dims& d = c.dims;
  const uint32_t words = mask_words(d.N);
  hipError_t e = hipMemsetAsync(b.once, 0, (size_t)3 * words * 4, c.stream);  // once, twice, cellbits
  if (e != hipSuccess) return e;
  const double rd = c.cfg.ibm_retraction;
  if (c.np > 0) {
    hipLaunchKernelGGL(k_corr_zone, dim3(c.np), dim3(kCBlock), 0, c.stream, X, c.P.r, d, rd, b.once, b.twice);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_corr_band, dim3(c.np), dim3(kCBlock), 0, c.stream, X, c.P.r, d, rd, dmin, dmax, b.twice,
                       b.cellbits, b.cellp);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  if ((e = launch_bits_compact(c.stream, b.cellbits, words, b.rank, b.bsums, b.count, list, cap, b.err)) !=
      hipSuccess)
    return e;
  if (cap > 0) {
    hipLaunchKernelGGL(k_corr_particles, dim3((cap + kCBlock - 1) / kCBlock), dim3(kCBlock), 0, c.stream, list,
                       b.count, cap, b.cellp, plist);
    e = hipGetLastError();
  }
  return e;
}

hipError_t launch_corrector_features(const Ctx& c, const float* u, const uint32_t* list, const uint32_t* plist,
                                     const uint32_t* count, uint32_t cap, const double* X, const double* U,
                                     const double* Om, double u_rms, uint16_t* out) {
  if (cap == 0) return hipSuccess;
  const uint64_t threads = (uint64_t)cap * 12;
  hipLaunchKernelGGL(k_corr_features, dim3((unsigned)((threads + kCBlock - 1) / kCBlock)), dim3(kCBlock), 0, c.stream,
                     list, plist, count, cap, u, X, U, Om, c.P.r, c.dims, u_rms, (__bf16*)out);
  return hipGetLastError();
}

hipError_t launch_corrector_labels(const Ctx& c, const float* u, const uint32_t* key, const uint32_t* list, uint32_t n,
                                   const double* X, const double* U, const double* Om, double u_rms, int subtract,
                                   float* out) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_corr_labels, dim3((n + kCBlock - 1) / kCBlock), dim3(kCBlock), 0, c.stream, list, n, u, key, X,
                     U, Om, c.dims, u_rms, subtract, out);
  return hipGetLastError();
}

size_t corrector_stats_lds_bytes() { return sizeof(CorrLds); }

hipError_t launch_corrector_stats(const Ctx& c, const float* theta, const float* u, const uint32_t* key,
                                  const uint32_t* list, const uint32_t* plist, const uint32_t* count, uint32_t cap,
                                  const double* X, const double* U, const double* Om, double u_rms, int nbins,
                                  double* part, double* out) {
  const double nu = (c.cfg.tau - 0.5) / 3.0;
  const int stride = 2 + nbins;
  const int grid = (int)std::max<uint32_t>(1u, std::min<uint32_t>((uint32_t)kStatGrid, (cap + 63) / 64));
  const size_t lds = sizeof(CorrLds);
  if (nbins <= 64)
    hipLaunchKernelGGL(k_corr_stats<1>, dim3(grid), dim3(kCBlock), lds, c.stream, theta, list, plist, count, cap, u,
                       key, X, U, Om, c.P.r, c.dims, u_rms, nu, nbins, part, stride);
  else if (nbins <= 128)
    hipLaunchKernelGGL(k_corr_stats<2>, dim3(grid), dim3(kCBlock), lds, c.stream, theta, list, plist, count, cap, u,
                       key, X, U, Om, c.P.r, c.dims, u_rms, nu, nbins, part, stride);
  else
    hipLaunchKernelGGL(k_corr_stats<4>, dim3(grid), dim3(kCBlock), lds, c.stream, theta, list, plist, count, cap, u,
                       key, X, U, Om, c.P.r, c.dims, u_rms, nu, nbins, part, stride);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_corr_reduce, dim3(stride), dim3(kCBlock), 0, c.stream, part, grid, stride, out);
  return hipGetLastError();
}

}  // namespace lbm
