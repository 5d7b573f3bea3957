// spectrum.hip - three-dimensional spectra of the kinetic energy and of its
// dissipation rate for one snapshot (Sec. 3.2.1), with or without
// the rigid-body masking of the particle interiors.
//
// E(k) = 1/2 sum over the shell k - 1/2 <= |k| < k + 1/2 of |u^(k)|^2, with
// u^ = (1/N) sum_x u(x) exp(-2 pi i k.x / L) over the periodic box and k in
// integer wavenumbers (k_max = n/2 along an axis of n nodes), so that
// sum_k E(k) = 1/2 <|u|^2> (Parseval); D(k) = 2 nu k^2 E(k).
//
// Passes, all on the idle population buffer:
//   pack    Z1 = u_x + i u_y, Z2 = u_z (FP32 complex). Because every shell is
//           symmetric under k -> -k, sum_shell |Z1^|^2 = sum_shell
//           (|u_x^|^2 + |u_y^|^2), so two complex transforms carry all three
//           components.
//   fft     radix-2 decimation in time along x, then y: a workgroup
//           stages lines in LDS in bit-reversed order (several adjacent
//           lines, so every global access is coalesced; eight loads in
//           flight per thread) and transforms them in place; twiddles from
//           a per-workgroup table of sincospi of exact rationals.
//   z+bin   the z transform of both fields, line by line in LDS; then one
//           thread per (k_x, k_y) line walks |k_z| = 0 .. n_z/2 and sums
//           |Z1^|^2 + |Z2^|^2 per shell in that order, so the transformed
//           field never returns to memory. Shell s holds the integer k^2
//           with s(s-1) < k^2 <= s(s+1), which is round(|k|) exactly (k^2 is
//           an integer and (s + 1/2)^2 never is).
//   shells  a shell's line partials are added in line order over eight
//           fixed line ranges, and the eight sums in range order.
// Every sum has a fixed order, so the result does not change from run to
// run. Lattice sides must be powers of two.
#include <algorithm>

#include "device_util.hpp"
#include "internal.hpp"
#include "stats_device.hpp"

namespace lbm {

namespace {

constexpr int kSpBlock = 256;
constexpr int kFftLds = 32 * 1024;  // bytes of LDS per FFT workgroup for the lines

__global__ void __launch_bounds__(kSpBlock)
k_spec_pack(const float* __restrict__ u, const uint32_t* __restrict__ key, const double* __restrict__ X,
            const double* __restrict__ U, const double* __restrict__ Om, Dims d, int masked, float2* __restrict__ Z1,
            float2* __restrict__ Z2) {
  const uint32_t n = blockIdx.x * kSpBlock + threadIdx.x;
  if (n >= d.N) return;
  float v[3];
  if (masked) {
    const MaskedVel vel{u, key, X, U, Om, d};
    double w[3];
    vel.at(n, w);
    v[0] = (float)w[0];
    v[1] = (float)w[1];
    v[2] = (float)w[2];
  } else {
    v[0] = u[n];
    v[1] = u[(size_t)d.N + n];
    v[2] = u[2 * (size_t)d.N + n];
  }
  Z1[n] = make_float2(v[0], v[1]);
  Z2[n] = make_float2(v[2], 0.0f);
}

// In-place butterflies of `count` lines of n = 2^logn values in LDS (bit-
// reversed order in, natural order out); tw[k] = exp(-2 pi i k / n).
__device__ __forceinline__ void lds_fft(float2* buf, const float2* tw, uint32_t count, int logn) {
  const uint32_t n = 1u << logn, half_n = n >> 1;
  for (int s = 1; s <= logn; ++s) {
    const uint32_t hm = 1u << (s - 1);  // half the butterfly span
    const int tshift = logn - s;        // exp(-2 pi i pos / 2hm) = tw[pos << tshift]
    for (uint32_t b = threadIdx.x; b < count * half_n; b += kSpBlock) {
      const uint32_t w = b >> (logn - 1), k = b & (half_n - 1u);
      const uint32_t pos = k & (hm - 1u);
      const uint32_t i0 = w * n + ((k >> (s - 1)) << s) + pos, i1 = i0 + hm;
      const float2 t0 = tw[pos << tshift];
      const float2 a = buf[i0], c = buf[i1];
      const float2 t = make_float2(t0.x * c.x - t0.y * c.y, t0.x * c.y + t0.y * c.x);
      buf[i0] = make_float2(a.x + t.x, a.y + t.y);
      buf[i1] = make_float2(a.x - t.x, a.y - t.y);
    }
    __syncthreads();
  }
}

__device__ __forceinline__ void twiddles(float2* tw, uint32_t half_n) {
  for (uint32_t k = threadIdx.x; k < half_n; k += kSpBlock) {  // exp(-2 pi i k / n)
    float sn, cs;
    sincospif((float)k / (float)half_n, &sn, &cs);
    tw[k] = make_float2(cs, -sn);
  }
}

// Lines of one axis: line L starts at (L & (A - 1)) * sa + (L >> logA) * sb
// and steps by se. The W lines of a workgroup are L = W g .. W g + W - 1;
// `xfast` says whether a line's own elements are contiguous (the x axis), in
// which case the threads run along the line, else across the W lines.
struct LineMap {
  uint32_t logA, sa, sb, se;
  int xfast;
};

__device__ __forceinline__ size_t line_base(const LineMap& m, uint32_t L) {
  return (size_t)(L & ((1u << m.logA) - 1u)) * m.sa + (size_t)(L >> m.logA) * m.sb;
}

__global__ void __launch_bounds__(kSpBlock)
k_fft_lines(float2* __restrict__ Z, uint32_t lines, int logn, int W, LineMap m) {
  extern __shared__ float2 lds[];  // twiddles [n/2], then the lines [W][n]
  const uint32_t n = 1u << logn, half_n = n >> 1;
  float2* tw = lds;
  float2* buf = lds + half_n;
  twiddles(tw, half_n);
  const uint32_t L0 = blockIdx.x * (uint32_t)W;
  const uint32_t total = (uint32_t)W * n;
  constexpr int kU = 8;  // loads in flight per thread
  for (uint32_t i0 = 0; i0 < total; i0 += kU * kSpBlock) {
    float2 v[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const uint32_t i = i0 + (uint32_t)(u * kSpBlock) + threadIdx.x;
      const uint32_t w = m.xfast ? i >> logn : i % (uint32_t)W;
      const uint32_t j = m.xfast ? i & (n - 1u) : i / (uint32_t)W;
      const uint32_t L = L0 + w;
      v[u] = i < total && L < lines ? Z[line_base(m, L) + (size_t)j * m.se] : make_float2(0.0f, 0.0f);
    }
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const uint32_t i = i0 + (uint32_t)(u * kSpBlock) + threadIdx.x;
      const uint32_t w = m.xfast ? i >> logn : i % (uint32_t)W;
      const uint32_t j = m.xfast ? i & (n - 1u) : i / (uint32_t)W;
      if (i < total) buf[w * n + (__brev(j) >> (32 - logn))] = v[u];
    }
  }
  __syncthreads();
  lds_fft(buf, tw, (uint32_t)W, logn);
  for (uint32_t i = threadIdx.x; i < total; i += kSpBlock) {
    const uint32_t w = m.xfast ? i >> logn : i % (uint32_t)W;
    const uint32_t j = m.xfast ? i & (n - 1u) : i / (uint32_t)W;
    const uint32_t L = L0 + w;
    if (L < lines) Z[line_base(m, L) + (size_t)j * m.se] = buf[w * n + j];
  }
}

__device__ __forceinline__ int freq(int i, int n) { return i < n / 2 ? i : i - n; }

// Shell of an integer k^2: the s >= 0 with s(s-1) < k2 <= s(s+1).
__device__ __forceinline__ int shell_of(int64_t k2) {
  int s = (int)sqrt((double)k2);
  while ((int64_t)s * (s + 1) < k2) ++s;
  while (s > 0 && (int64_t)s * (s - 1) >= k2) --s;
  return s;
}

// Last pass: the z transform of Z1 and Z2 for W adjacent (x, y) lines, then
// one thread per line walks |k_z| = 0 .. nz/2 and sums |Z1^|^2 + |Z2^|^2 per
// shell in that order into the line's partials (P[line][s - smin]).
__global__ void __launch_bounds__(kSpBlock)
k_fft_z_bin(const float2* __restrict__ Z1, const float2* __restrict__ Z2, Dims d, int lx, int logn, int W,
            uint32_t rowlen, double* __restrict__ P, int* __restrict__ smin, int* __restrict__ cnt) {
  extern __shared__ float2 lds[];  // twiddles [n/2], then [2W][n]: Z1 lines, Z2 lines
  const uint32_t n = 1u << logn, half_n = n >> 1;
  float2* tw = lds;
  float2* buf = lds + half_n;
  twiddles(tw, half_n);
  const uint32_t lines = (uint32_t)d.nx * (uint32_t)d.ny, plane = (uint32_t)d.nx * (uint32_t)d.ny;
  const uint32_t L0 = blockIdx.x * (uint32_t)W;
  const uint32_t total = 2u * (uint32_t)W * n;
  constexpr int kU = 8;
  for (uint32_t i0 = 0; i0 < total; i0 += kU * kSpBlock) {
    float2 v[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const uint32_t i = i0 + (uint32_t)(u * kSpBlock) + threadIdx.x;
      const uint32_t w = i % (2u * (uint32_t)W), j = i / (2u * (uint32_t)W);  // w < W: Z1, else Z2
      const uint32_t L = L0 + (w % (uint32_t)W);
      const float2* src = w < (uint32_t)W ? Z1 : Z2;
      v[u] = i < total && L < lines ? src[(size_t)L + (size_t)j * plane] : make_float2(0.0f, 0.0f);
    }
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const uint32_t i = i0 + (uint32_t)(u * kSpBlock) + threadIdx.x;
      const uint32_t w = i % (2u * (uint32_t)W), j = i / (2u * (uint32_t)W);
      if (i < total) buf[w * n + (__brev(j) >> (32 - logn))] = v[u];
    }
  }
  __syncthreads();
  lds_fft(buf, tw, 2u * (uint32_t)W, logn);
  // One wavefront per line: lane l takes |k_z| = 64 c + l of chunk c. The
  // shell is non-decreasing along the lanes, so each shell of a chunk is a
  // run of lanes; a segmented shuffle scan sums every run in a fixed tree
  // order, the run's last lane writes it, and a shell running on into the
  // next chunk is carried. The lane where the shell skips one writes the
  // skipped shell's zero, so every partial of the line is written once.
  const uint32_t lane = threadIdx.x & 63u, w = threadIdx.x >> 6;
  const uint32_t L = L0 + w;
  if (w >= (uint32_t)W || L >= lines) return;  // the whole wavefront
  const int kx = freq((int)(L & ((1u << lx) - 1u)), d.nx), ky = freq((int)(L >> lx), d.ny);
  const int64_t r2 = (int64_t)kx * kx + (int64_t)ky * ky;
  const int s0 = shell_of(r2);
  double* out = P + (size_t)L * rowlen;
  const float2* z1 = buf + w * n;
  const float2* z2 = buf + ((uint32_t)W + w) * n;
  auto energy = [&](int j) {
    const float2 a = z1[j], b = z2[j];
    return (((double)a.x * a.x + (double)a.y * a.y) + (double)b.x * b.x) + (double)b.y * b.y;
  };
  const int amax = d.nz / 2;
  int prev_s = s0;     // shell of the last entry of the previous chunk
  double carry = 0.0;  // its run's sum, pending (0 before the first chunk)
  for (int c0 = 0; c0 <= amax; c0 += 64) {
    const bool final_chunk = c0 + 64 > amax;
    const int a = c0 + (int)lane;
    const bool live = a <= amax;
    const int s = live ? shell_of(r2 + (int64_t)a * a) : 0x7FFFFFFF;
    double v = 0.0;
    if (live) {
      v = energy(a);
      if (a > 0 && a < d.nz - a) v += energy(d.nz - a);  // k_z = -a
    }
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {  // segmented inclusive scan over runs
      const double t = __shfl_up(v, off, 64);
      const int ts = __shfl_up(s, off, 64);
      if ((int)lane >= off && ts == s) v += t;
    }
    // every shuffle at wavefront-uniform control flow, selections after
    const int s_first = __shfl(s, 0, 64);
    const int s_up = __shfl_up(s, 1, 64);
    const int s_down = __shfl_down(s, 1, 64);
    const int s63 = __shfl(s, 63, 64);
    if (s_first == prev_s) {
      if (s == prev_s) v += carry;  // the first run goes on from the previous chunk
    } else if (lane == 0) {
      out[prev_s - s0] = carry;  // the previous chunk's last run is complete
    }
    const double v63 = __shfl(v, 63, 64);
    const int s_before = lane == 0 ? prev_s : s_up;
    const int s_after = lane == 63u ? 0x7FFFFFFF : s_down;
    if (live) {
      for (int g = max(s_before + 1, s0); g < s; ++g) out[g - s0] = 0.0;  // shells no k_z of the line reaches
      if (s_after != s && (lane != 63u || final_chunk)) out[s - s0] = v;
    }
    if (!final_chunk) {  // lane 63 is live: its run may go on
      carry = v63;
      prev_s = s63;
    }
  }
  if (lane == 0) {
    smin[L] = s0;
    cnt[L] = shell_of(r2 + (int64_t)amax * amax) - s0 + 1;
  }
}

constexpr int kShellSplit = 8;  // workgroups per shell, each over a fixed range of lines

__global__ void __launch_bounds__(kSpBlock)
k_spec_shells(const double* __restrict__ P, const int* __restrict__ smin, const int* __restrict__ cnt,
              uint32_t lines, uint32_t rowlen, double* __restrict__ part) {
  const int s = (int)(blockIdx.x / kShellSplit), g = (int)(blockIdx.x % kShellSplit);
  const uint32_t lo = (uint32_t)((uint64_t)lines * g / kShellSplit);
  const uint32_t hi = (uint32_t)((uint64_t)lines * (g + 1) / kShellSplit);
  double acc = 0.0;
  for (uint32_t L = lo + threadIdx.x; L < hi; L += kSpBlock) {
    const int j = s - smin[L];
    if (j >= 0 && j < cnt[L]) acc += P[(size_t)L * rowlen + (uint32_t)j];
  }
  const double t = block_sum<kSpBlock>(acc);
  if (threadIdx.x == 0) part[blockIdx.x] = t;
}

__global__ void __launch_bounds__(kSpBlock)
k_spec_final(const double* __restrict__ part, int kmax, double scale, double nu, double* __restrict__ E,
             double* __restrict__ D) {
  const int s = (int)(blockIdx.x * kSpBlock + threadIdx.x);
  if (s > kmax) return;
  double t = 0.0;
  for (int g = 0; g < kShellSplit; ++g) t += part[s * kShellSplit + g];
  const double e = t * scale;
  E[s] = e;
  D[s] = 2.0 * nu * (double)s * (double)s * e;
}

int log2_exact(int n) {
  int l = 0;
  while ((1 << l) < n) ++l;
  return (1 << l) == n ? l : -1;
}

}  // namespace

size_t spectrum_row_len(const Ctx& c) { return (size_t)c.dims.nz / 2 + 2; }

size_t spectrum_lines(const Ctx& c) { return (size_t)c.dims.nx * (size_t)c.dims.ny; }

bool spectrum_supported(const Ctx& c) {
  const int lx = log2_exact(c.dims.nx), ly = log2_exact(c.dims.ny), lz = log2_exact(c.dims.nz);
  return lx > 0 && ly > 0 && lz > 0 && c.dims.nx <= 1024 && c.dims.ny <= 1024 && c.dims.nz <= 1024;
}

hipError_t launch_spec_pack(const Ctx& c, const float* u, const uint32_t* key, int masked, float2* Z1, float2* Z2) {
  const int pc = c.pcur;
  hipLaunchKernelGGL(k_spec_pack, dim3((c.dims.N + kSpBlock - 1) / kSpBlock), dim3(kSpBlock), 0, c.stream, u, key,
                     c.P.X[pc], c.P.U[pc], c.P.Om[pc], c.dims, masked, Z1, Z2);
  return hipGetLastError();
}

// In-place forward transform of a [nz][ny][nx] complex field along x and y.
hipError_t launch_fft_xy(const Ctx& c, float2* Z) {
  const Dims& d = c.dims;
  const int lx = log2_exact(d.nx), ly = log2_exact(d.ny);
  struct Axis {
    int logn;
    uint32_t lines;
    LineMap m;
  };
  const uint32_t nx = (uint32_t)d.nx, ny = (uint32_t)d.ny, nz = (uint32_t)d.nz;
  const Axis axes[2] = {{lx, ny * nz, LineMap{0, 0, nx, 1, 1}},                    // rows: line L at L nx
                        {ly, nx * nz, LineMap{(uint32_t)lx, 1, nx * ny, nx, 0}}};  // (x, z): x + z nx ny, step nx
  for (const Axis& a : axes) {
    const uint32_t n = 1u << a.logn;
    int W = (int)std::min<uint32_t>(16u, (uint32_t)(kFftLds / sizeof(float2)) / n);
    if (!a.m.xfast) W = (int)std::min<uint32_t>((uint32_t)W, nx);  // a group's lines share z
    W = std::max(W, 1);
    const uint32_t groups = (a.lines + (uint32_t)W - 1) / (uint32_t)W;
    hipLaunchKernelGGL(k_fft_lines, dim3(groups), dim3(kSpBlock), ((size_t)W + 1) * n * sizeof(float2), c.stream,
                       Z, a.lines, a.logn, W, a.m);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// z transform of both fields with the shell sums (line partials, then shells).
hipError_t launch_spec_zbins(const Ctx& c, const float2* Z1, const float2* Z2, double* P, int* smin, int* cnt,
                             int kmax, double nu, double* part, double* E, double* D) {
  const Dims& d = c.dims;
  const int lx = log2_exact(d.nx), lz = log2_exact(d.nz);
  const uint32_t n = 1u << lz;
  const uint32_t lines = (uint32_t)spectrum_lines(c), rowlen = (uint32_t)spectrum_row_len(c);
  int W = (int)std::min<uint32_t>(4u, (uint32_t)(kFftLds / sizeof(float2)) / (2u * n));  // a wavefront per line
  W = std::max(std::min(W, d.nx), 1);  // a group's lines share y
  hipLaunchKernelGGL(k_fft_z_bin, dim3((lines + (uint32_t)W - 1) / (uint32_t)W), dim3(kSpBlock),
                     (2 * (size_t)W * n + n / 2) * sizeof(float2), c.stream, Z1, Z2, d, lx, lz, W, rowlen, P, smin,
                     cnt);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_spec_shells, dim3(((uint32_t)kmax + 1) * kShellSplit), dim3(kSpBlock), 0, c.stream, P, smin,
                     cnt, lines, rowlen, part);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  const double Nd = (double)d.N;
  hipLaunchKernelGGL(k_spec_final, dim3(((uint32_t)kmax + kSpBlock) / kSpBlock), dim3(kSpBlock), 0, c.stream, part,
                     kmax, 0.5 / (Nd * Nd), nu, E, D);
  return hipGetLastError();
}

}  // namespace lbm
