// device_util.hpp - small device helpers: periodic wrap, per-sphere boxes,
// block-wide scans and FP64 reductions in a fixed order.
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

namespace lbm {

__device__ __forceinline__ int wrapi(int v, int n) {
  v %= n;
  return v < 0 ? v + n : v;
}

// Minimum image of an offset in (-L, L): one explicit branch per side, so
// any implementation following the same recipe rounds identically.
__device__ __forceinline__ double min_image(double d, double L) {
  if (d > 0.5 * L) d -= L;
  if (d < -0.5 * L) d += L;
  return d;
}

__device__ __forceinline__ double dist2(double dx, double dy, double dz) {
  return (dx * dx + dy * dy) + dz * dz;
}

// Axis-aligned periodic box floor(X - reach) .. ceil(X + reach) around a point.
struct Box {
  int lo[3];
  int side[3];
  __device__ uint32_t count() const { return (uint32_t)side[0] * (uint32_t)side[1] * (uint32_t)side[2]; }
};

__device__ __forceinline__ Box make_box(const double* X, double reach) {
  Box b;
  for (int k = 0; k < 3; ++k) {
    const int lo = (int)floor(X[k] - reach);
    const int hi = (int)ceil(X[k] + reach);
    b.lo[k] = lo;
    b.side[k] = hi - lo + 1;
  }
  return b;
}

// i-th node of a box in raster order (x fastest), wrapped into the lattice.
__device__ __forceinline__ void box_node(const Box& b, uint32_t i, int nx, int ny, int nz, int& x, int& y, int& z) {
  const uint32_t sx = (uint32_t)b.side[0], sy = (uint32_t)b.side[1];
  const int ix = (int)(i % sx);
  const int iy = (int)((i / sx) % sy);
  const int iz = (int)(i / (sx * sy));
  x = wrapi(b.lo[0] + ix, nx);
  y = wrapi(b.lo[1] + iy, ny);
  z = wrapi(b.lo[2] + iz, nz);
}

// Wrap for v in [-n, 2n): one conditional add or subtract, no division.
__device__ __forceinline__ int wrap1(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }

// Box traversal by x-rows: a 256-thread block covers 256/W rows of W lanes
// per iteration (W = 32 or 64 >= side_x), so a node's coordinates cost one
// division per row instead of two per node and wrapping needs no modulo.
struct BoxRows {
  int W, shift, rows_per_iter, nrows;
};

__device__ __forceinline__ BoxRows box_rows(const Box& b) {
  BoxRows r;
  r.W = b.side[0] <= 32 ? 32 : 64;
  r.shift = b.side[0] <= 32 ? 5 : 6;
  r.rows_per_iter = 256 >> r.shift;
  r.nrows = b.side[1] * b.side[2];
  return r;
}

// Node of lane t in iteration `base` (rows base .. base + rows_per_iter - 1).
// Returns false for lanes beyond the box.
__device__ __forceinline__ bool box_row_node(const Box& b, const BoxRows& br, int base, int t, int nx, int ny, int nz,
                                             int& x, int& y, int& z) {
  const int row = base + (t >> br.shift);
  const int ix = t & (br.W - 1);
  if (row >= br.nrows || ix >= b.side[0]) return false;
  const int iy = row % b.side[1];
  const int iz = row / b.side[1];
  x = wrap1(b.lo[0] + ix, nx);
  y = wrap1(b.lo[1] + iy, ny);
  z = wrap1(b.lo[2] + iz, nz);
  return true;
}

// Box traversal by linear raster index with every lane busy. i / s is a
// multiply-high by m = ceil(2^32 / s), exact while i * s < 2^32: box sides
// stay below 64 (radius <= 28) and indices below 64^3, so i * s < 2^30.
struct BoxLin {
  uint32_t sx, sxy, count, mx, mxy;
};

__device__ __forceinline__ BoxLin box_lin(const Box& b) {
  BoxLin L;
  L.sx = (uint32_t)b.side[0];
  L.sxy = L.sx * (uint32_t)b.side[1];
  L.count = L.sxy * (uint32_t)b.side[2];
  L.mx = (uint32_t)((0x100000000ull + L.sx - 1u) / L.sx);
  L.mxy = (uint32_t)((0x100000000ull + L.sxy - 1u) / L.sxy);
  return L;
}

// Node i (< L.count) of the box, wrapped into the lattice.
__device__ __forceinline__ void box_lin_node(const Box& b, const BoxLin& L, uint32_t i, int nx, int ny, int nz, int& x,
                                             int& y, int& z) {
  const uint32_t iz = __umulhi(i, L.mxy);
  const uint32_t rem = i - iz * L.sxy;
  const uint32_t iy = __umulhi(rem, L.mx);
  const uint32_t ix = rem - iy * L.sx;
  x = wrap1(b.lo[0] + (int)ix, nx);
  y = wrap1(b.lo[1] + (int)iy, ny);
  z = wrap1(b.lo[2] + (int)iz, nz);
}

// One row of a sphere: a row of nodes along x whose (y, z) lies at squared
// distance e2 from the centre X across the row, for a sphere of squared
// radius r2 with centre X0 along x. Nodes in [plo, phi] may be inside (none
// outside it is); nodes strictly between clo and chi certainly are. The
// margins (1e-6 (r2 + 1) on r2 - e2, 1e-9 on the roots) exceed any rounding
// of the exact FP64 test d2 < r2 of a node, so that test agrees wherever
// these bounds decide. `any` is false when no node of the row can be inside.
struct RowSpan {
  double plo, phi, clo, chi;
  bool any;
};

__device__ __forceinline__ RowSpan sphere_row(double X0, double e2, double r2) {
  RowSpan s;
  const double m = 1e-6 * (r2 + 1.0);
  s.any = r2 - e2 + m > 0.0;
  const double w = s.any ? sqrt(r2 - e2 + m) + 1e-9 : 0.0;
  s.plo = X0 - w;
  s.phi = X0 + w;
  const double v = r2 - e2 - m > 0.0 ? sqrt(r2 - e2 - m) - 1e-9 : 0.0;
  s.clo = X0 - v;
  s.chi = X0 + v;
  return s;
}

// Integers of [ceil(o_lo), floor(o_hi)] within [lo, hi], except those
// strictly between h_lo and h_hi, as up to two disjoint intervals [a0, a1],
// [b0, b1]; an empty interval has its end below its start.
__device__ __forceinline__ void row_band(double o_lo, double o_hi, double h_lo, double h_hi, int lo, int hi, int& a0,
                                         int& a1, int& b0, int& b1) {
  a0 = max((int)ceil(o_lo), lo);
  a1 = min((int)floor(o_hi), hi);
  b0 = 1;
  b1 = 0;
  if (a1 < a0) return;
  const int left_hi = (int)floor(h_lo), right_lo = (int)ceil(h_hi);
  if (left_hi + 1 > right_lo - 1) return;  // no integer strictly inside the hole
  const int o1 = a1;
  a1 = min(left_hi, o1);
  b0 = max(right_lo, max(a0, a1 + 1));
  b1 = o1;
}

// Pipe wall: root t in [0, 1) of |dxy + t cxy|^2 = R^2 for a point inside
// heading out.
__device__ __forceinline__ double pipe_q(double dx, double dy, int cx, int cy, double R) {
  const double a = (double)(cx * cx + cy * cy);
  const double b = dx * cx + dy * cy;
  const double cc = (dx * dx + dy * dy) - R * R;
  const double disc = sqrt(b * b - a * cc);
  return b >= 0.0 ? -cc / (b + disc) : (disc - b) / a;
}

// Link nodes are stored as packed coordinates x | y << 11 | z << 22.
__device__ __forceinline__ uint32_t pack_xyz(int x, int y, int z) {
  return (uint32_t)x | ((uint32_t)y << 11) | ((uint32_t)z << 22);
}
__device__ __forceinline__ void unpack_xyz(uint32_t v, int& x, int& y, int& z) {
  x = (int)(v & 2047u);
  y = (int)((v >> 11) & 2047u);
  z = (int)(v >> 22);
}

__device__ __forceinline__ uint32_t node_index(int x, int y, int z, int nx, int ny) {
  return ((uint32_t)z * (uint32_t)ny + (uint32_t)y) * (uint32_t)nx + (uint32_t)x;
}

__device__ __forceinline__ void node_coords(uint32_t n, int nx, int ny, int& x, int& y, int& z) {
  x = (int)(n % (uint32_t)nx);
  const uint32_t r = n / (uint32_t)nx;
  y = (int)(r % (uint32_t)ny);
  z = (int)(r / (uint32_t)ny);
}

// Kempe et al. solid fraction of the unit cell around a node at offset d
// from a sphere centre: sum over the 8 corners of (-phi) H(-phi) / sum |phi|,
// phi = |corner - X| - r (corners in the order (-,-,-), (-,-,+), ...).
__device__ __forceinline__ double kempe_alpha(double dx, double dy, double dz, double r) {
  // Away from the surface every corner is on one side: the formula gives
  // exactly 1 (num and den are the same sum) or exactly 0.
  const double d2 = dist2(dx, dy, dz);
  const double ri = r - 0.8661, ro = r + 0.8661;  // 0.8661 > sqrt(3)/2
  if (ri > 0.0 && d2 < ri * ri) return 1.0;
  if (d2 >= ro * ro) return 0.0;
  double num = 0.0, den = 0.0;
  // one corner at a time: the eight roots unrolled side by side hold about
  // forty more registers for little gain in a latency-bound caller
#pragma unroll 1
  for (int c = 0; c < 8; ++c) {
    const double sx = (c & 4) ? 0.5 : -0.5, sy = (c & 2) ? 0.5 : -0.5, sz = (c & 1) ? 0.5 : -0.5;
    const double phi = sqrt(dist2(dx + sx, dy + sy, dz + sz)) - r;
    num += phi < 0.0 ? -phi : 0.0;
    den += fabs(phi);
  }
  return den > 0.0 ? num / den : 0.0;
}

// Exclusive prefix sum over a block of BLOCK threads (multiple of 64).
// Every thread must call it. Returns the thread's offset; *total gets the sum.
template <int BLOCK>
__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t v, uint32_t* total) {
  __shared__ uint32_t wsum[BLOCK / 64];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  uint32_t incl = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t t = __shfl_up(incl, o, 64);
    if (lane >= o) incl += t;
  }
  if (lane == 63) wsum[wid] = incl;
  __syncthreads();
  uint32_t base = 0, all = 0;
#pragma unroll
  for (int w = 0; w < BLOCK / 64; ++w) {
    const uint32_t s = wsum[w];
    if (w < wid) base += s;
    all += s;
  }
  __syncthreads();
  *total = all;
  return base + incl - v;
}

// Sum of a double over the block in a fixed order (butterfly within each
// wavefront, then the wavefront partials in index order), so the result is
// deterministic for a given block size. Every thread must call it; all get
// the result.
template <int BLOCK>
__device__ __forceinline__ double block_sum(double v) {
  __shared__ double part[BLOCK / 64];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = v;
  __syncthreads();
  double r = 0.0;
#pragma unroll
  for (int w = 0; w < BLOCK / 64; ++w) r += part[w];
  __syncthreads();
  return r;
}

// N independent block sums at once (fewer barriers).
template <int BLOCK, int N>
__device__ __forceinline__ void block_sum_n(double (&v)[N]) {
  __shared__ double part[N][BLOCK / 64];
#pragma unroll
  for (int k = 0; k < N; ++k) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v[k] += __shfl_xor(v[k], o, 64);
  }
  if ((threadIdx.x & 63) == 0)
#pragma unroll
    for (int k = 0; k < N; ++k) part[k][threadIdx.x >> 6] = v[k];
  __syncthreads();
#pragma unroll
  for (int k = 0; k < N; ++k) {
    double r = 0.0;
#pragma unroll
    for (int w = 0; w < BLOCK / 64; ++w) r += part[k][w];
    v[k] = r;
  }
  __syncthreads();
}

// Value of a double in lane src (src uniform across the wavefront).
__device__ __forceinline__ double readlane_d(double v, int src) {
  const unsigned long long b = __double_as_longlong(v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)b, src);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), src);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// N block sums whose results only thread 0 needs: lanes 0 .. N-1 of the first
// wavefront add the wavefront partials in index order, so the result matches
// block_sum_n bit for bit. Every thread must call it.
template <int BLOCK, int N>
__device__ __forceinline__ void block_sum_first(double (&v)[N]) {
  static_assert(N <= 64, "one lane per sum");
  __shared__ double part[N][BLOCK / 64];
#pragma unroll
  for (int k = 0; k < N; ++k) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v[k] += __shfl_xor(v[k], o, 64);
  }
  if ((threadIdx.x & 63) == 0)
#pragma unroll
    for (int k = 0; k < N; ++k) part[k][threadIdx.x >> 6] = v[k];
  __syncthreads();
  if (threadIdx.x < 64) {
    const int k = threadIdx.x < N ? (int)threadIdx.x : 0;
    double r = 0.0;
#pragma unroll
    for (int w = 0; w < BLOCK / 64; ++w) r += part[k][w];
#pragma unroll
    for (int i = 0; i < N; ++i) v[i] = __shfl(r, i, 64);
  }
}

}  // namespace lbm
