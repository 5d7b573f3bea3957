// geometry.hip - solid/fluid classification and boundary links for
// interpolated bounce-back (Sec. 3.1, Sec. 2.1).
//
// Classification is exact FP64 with no contraction (this file is built with
// -ffp-contract=off): node x is inside sphere p iff the minimum-image
// squared distance ((dx*dx + dy*dy) + dz*dz) is below r_p^2. Overlaps go to
// the lowest particle index (atomicMin on the owner map). The pipe wall is
// solid where (x - cx)^2 + (y - cy)^2 >= R^2.
//
// Links are built per sphere by one workgroup. It first compacts the nodes
// of the shell r <= |x - X| < r + sqrt(2) (the only possible fluid ends of
// its links) into an LDS list in raster order, then examines the list with
// every lane busy; a block-wide prefix sum gives every link a deterministic
// slot, so the link order (and every FP64 sum over links) is reproducible.
#include "device_util.hpp"
#include "internal.hpp"

namespace lbm {

namespace {

constexpr int kBlock = 256;
constexpr int kCand = 2048;  // shell candidates buffered in LDS per flush

__device__ __forceinline__ bool inside_sphere(int x, int y, int z, const double* X, double r, double Lx, double Ly,
                                              double Lz) {
  const double dx = min_image((double)x - X[0], Lx);
  const double dy = min_image((double)y - X[1], Ly);
  const double dz = min_image((double)z - X[2], Lz);
  return dist2(dx, dy, dz) < r * r;
}

__global__ void __launch_bounds__(256) k_owner_fill(uint32_t* __restrict__ owner, const uint32_t* __restrict__ wall,
                                                    uint32_t N) {
  const uint32_t n = blockIdx.x * 256u + threadIdx.x;
  if (n >= N) return;
  owner[n] = ((wall[n >> 5] >> (n & 31u)) & 1u) ? kWall : kFluid;
}

// Resets the nodes inside every particle at its old position to fluid (every
// entry a set pass wrote lies inside some sphere at the positions it used).
__global__ void __launch_bounds__(kBlock) k_owner_clear(uint32_t* __restrict__ owner, const double* __restrict__ Xold,
                                                        const double* __restrict__ rad, Dims d) {
  const int p = blockIdx.x;
  const double r = rad[p];
  const double* Xp = Xold + 3 * p;
  const Box b = make_box(Xp, r + 1.0);
  const BoxLin L = box_lin(b);
  for (uint32_t i = threadIdx.x; i < L.count; i += kBlock) {
    int x, y, z;
    box_lin_node(b, L, i, d.nx, d.ny, d.nz, x, y, z);
    if (!inside_sphere(x, y, z, Xp, r, d.nx, d.ny, d.nz)) continue;
    const uint32_t n = node_index(x, y, z, d.nx, d.ny);
    if (owner[n] != kWall) owner[n] = kFluid;
  }
}

__global__ void __launch_bounds__(kBlock) k_owner_set(uint32_t* __restrict__ owner, const double* __restrict__ X,
                                                      const double* __restrict__ rad, Dims d) {
  const int p = blockIdx.x;
  const double r = rad[p];
  const double* Xp = X + 3 * p;
  const Box b = make_box(Xp, r + 1.0);
  const BoxLin L = box_lin(b);
  for (uint32_t i = threadIdx.x; i < L.count; i += kBlock) {
    int x, y, z;
    box_lin_node(b, L, i, d.nx, d.ny, d.nz, x, y, z);
    if (!inside_sphere(x, y, z, Xp, r, d.nx, d.ny, d.nz)) continue;
    atomicMin(owner + node_index(x, y, z, d.nx, d.ny), (uint32_t)p);
  }
}

// Nodes not owned by the fluid (spheres and wall), for reporting.
__global__ void __launch_bounds__(256) k_count_solid(const uint32_t* __restrict__ owner, uint32_t N,
                                                     unsigned long long* __restrict__ out) {
  __shared__ unsigned int part[4];
  const uint32_t n = blockIdx.x * 256u + threadIdx.x;
  const bool solid = n < N && owner[n] != kFluid;
  const unsigned long long b = __ballot(solid);
  if ((threadIdx.x & 63u) == 0) part[threadIdx.x >> 6] = (unsigned int)__popcll(b);
  __syncthreads();
  if (threadIdx.x == 0) {
    const unsigned int s = part[0] + part[1] + part[2] + part[3];
    if (s) atomicAdd(out, (unsigned long long)s);
  }
}

// q: smaller root t of |d + t c|^2 = r^2 for a fluid point heading into the
// sphere, in the cancellation-free form.
__device__ __forceinline__ double sphere_q(double dx, double dy, double dz, int cx, int cy, int cz, double r) {
  const double a = (double)((cx * cx + cy * cy) + cz * cz);
  const double b = (dx * cx + dy * cy) + dz * cz;
  const double cc = dist2(dx, dy, dz) - r * r;
  return cc / (-b + sqrt(b * b - a * cc));
}

// Fallback chain: quadratic needs x_f - c (and x_f - 2c when q < 1/2) fluid;
// linear needs x_f - c fluid when q < 1/2; otherwise the single-node scheme.
__device__ __forceinline__ uint32_t pick_scheme(double q, bool f1, bool f2, int max_order) {
  const bool lo = q < 0.5;
  const bool quad_ok = lo ? (f1 && f2) : f1;
  const bool lin_ok = lo ? f1 : true;
  if (max_order >= 2 && quad_ok) return kSchemeQuadratic;
  return lin_ok ? kSchemeLinear : kSchemeHalfway;
}

__device__ __forceinline__ uint32_t neighbour(int x, int y, int z, int k, int i, const Dims& d) {
  return node_index(wrap1(x + k * cx_of(i), d.nx), wrap1(y + k * cy_of(i), d.ny), wrap1(z + k * cz_of(i), d.nz),
                    d.nx, d.ny);
}

// Index offset of t steps (|t| <= 2 < n) from coordinate c along an axis of
// n nodes and index stride `stride`, with the periodic wrap.
__device__ __forceinline__ int step_offset(int c, int t, int n, int stride) {
  const int v = c + t;
  return (v < 0 ? t + n : (v >= n ? t - n : t)) * stride;
}

// Examines the buffered shell candidates and writes their links from slot
// `written` on. Every thread must call it. Per chunk of kBlock candidates the
// lanes first find each candidate's links (owner lookups, all issued before
// any is used), list them in LDS in candidate-then-direction order, and then
// evaluate q and the scheme with one link per lane, so the FP64 root is
// computed with every lane busy and the records are written contiguously.
__device__ void flush_candidates(const uint32_t* __restrict__ owner, const double* Xp, double r, const Dims& d,
                                 int max_order, uint32_t p, uint32_t cap, size_t base, const uint32_t* cand,
                                 int ncand, uint16_t* lbuf, uint32_t& written, uint32_t* __restrict__ link_node,
                                 float* __restrict__ link_q, uint8_t* __restrict__ link_meta) {
  for (int c0 = 0; c0 < ncand; c0 += kBlock) {
    const int k = c0 + (int)threadIdx.x;
    uint32_t hits = 0, fluid1 = 0, fluid2 = 0;
    if (k < ncand) {
      int x, y, z;
      unpack_xyz(cand[k], x, y, z);
      uint32_t own[kQ], own1[kQ], own2[kQ];
      const int n = (int)node_index(x, y, z, d.nx, d.ny);
      // index offsets of steps -2..2 along each axis, periodic wrap included;
      // neighbour k c_a of n is n plus one offset per axis
      const int sy = d.nx, sz = d.nx * d.ny;
      int ox[5], oy[5], oz[5];
#pragma unroll
      for (int t = -2; t <= 2; ++t) {
        ox[t + 2] = step_offset(x, t, d.nx, 1);
        oy[t + 2] = step_offset(y, t, d.ny, sy);
        oz[t + 2] = step_offset(z, t, d.nz, sz);
      }
      auto nb = [&](int kk, int a) -> uint32_t {
        return (uint32_t)(n + ox[kk * cx_of(a) + 2] + oy[kk * cy_of(a) + 2] + oz[kk * cz_of(a) + 2]);
      };
      own[0] = owner[n];
#pragma unroll
      for (int a = 1; a < kQ; ++a) own[a] = owner[nb(1, a)];
#pragma unroll
      for (int a = 1; a < kQ; ++a) own1[a] = owner[nb(-1, a)];
#pragma unroll
      for (int a = 1; a < kQ; ++a) own2[a] = owner[nb(-2, a)];
      if (own[0] == kFluid) {
#pragma unroll
        for (int a = 1; a < kQ; ++a) {
          hits |= (own[a] == p ? 1u : 0u) << a;
          fluid1 |= (own1[a] == kFluid ? 1u : 0u) << a;
          fluid2 |= (own2[a] == kFluid ? 1u : 0u) << a;
        }
      }
    }
    uint32_t total;
    uint32_t off = block_exclusive_scan<kBlock>(__popc(hits), &total);
    // entry: candidate within the chunk (8 bits), direction (5), x_f - c fluid, x_f - 2c fluid
    for (uint32_t h = hits; h; h &= h - 1u) {
      const uint32_t a = (uint32_t)__builtin_ctz(h);
      lbuf[off++] = (uint16_t)(threadIdx.x | (a << 8) | (((fluid1 >> a) & 1u) << 13) | (((fluid2 >> a) & 1u) << 14));
    }
    __syncthreads();
    for (uint32_t j = threadIdx.x; j < total; j += kBlock) {
      const uint32_t e = lbuf[j];
      const uint32_t xyz = cand[c0 + (int)(e & 0xFFu)];
      const int a = (int)((e >> 8) & 31u);
      int x, y, z;
      unpack_xyz(xyz, x, y, z);
      const double dx = min_image((double)x - Xp[0], d.nx);
      const double dy = min_image((double)y - Xp[1], d.ny);
      const double dz = min_image((double)z - Xp[2], d.nz);
      const double q = sphere_q(dx, dy, dz, cx_of(a), cy_of(a), cz_of(a), r);
      const uint32_t sch = pick_scheme(q, (e >> 13) & 1u, (e >> 14) & 1u, max_order);
      const uint32_t slot = written + j;
      if (slot < cap) {
        link_node[base + slot] = xyz;
        link_q[base + slot] = (float)q;
        link_meta[base + slot] = (uint8_t)(a | (sch << 5));
      }
    }
    written += total;
    __syncthreads();  // lbuf is refilled by the next chunk
  }
}

__global__ void __launch_bounds__(kBlock)
k_links_build(const uint32_t* __restrict__ owner, const double* __restrict__ X, const double* __restrict__ rad, Dims d,
              int max_order, uint32_t cap, uint32_t* __restrict__ link_node, float* __restrict__ link_q,
              uint8_t* __restrict__ link_meta, uint32_t* __restrict__ link_count, uint32_t* __restrict__ err) {
  __shared__ uint32_t cand[kCand];
  __shared__ uint16_t lbuf[kBlock * (kQ - 1)];  // a chunk's links, at most every direction of every candidate
  const uint32_t p = blockIdx.x;
  const double r = rad[p];
  const double* Xp = X + 3 * p;
  const Box b = make_box(Xp, r + 2.0);
  const BoxLin L = box_lin(b);
  const size_t base = (size_t)p * cap;
  // The outer bound only prunes, so it carries a margin.
  const double r_out = r + 1.4142135623730951 + 1e-6;
  const double r2 = r * r, ro2 = r_out * r_out;
  uint32_t written = 0;
  int ncand = 0;
  // kPer nodes per thread per iteration
  constexpr int kPer = 4;
  for (uint32_t i0 = 0; i0 < L.count; i0 += kPer * kBlock) {
    uint32_t packed[kPer];
    uint32_t mask = 0;
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      int x = 0, y = 0, z = 0;
      packed[k] = 0;
      const uint32_t i = i0 + (uint32_t)(k * kBlock) + threadIdx.x;
      if (i < L.count) {
        box_lin_node(b, L, i, d.nx, d.ny, d.nz, x, y, z);
        const double d2 = dist2(min_image((double)x - Xp[0], d.nx), min_image((double)y - Xp[1], d.ny),
                                min_image((double)z - Xp[2], d.nz));
        if (d2 >= r2 && d2 < ro2) {
          mask |= 1u << k;
          packed[k] = pack_xyz(x, y, z);
        }
      }
    }
    uint32_t total;
    uint32_t off = block_exclusive_scan<kBlock>(__popc(mask), &total);
    if (ncand + (int)total > kCand) {  // uniform: total is block-wide
      flush_candidates(owner, Xp, r, d, max_order, p, cap, base, cand, ncand, lbuf, written, link_node, link_q, link_meta);
      __syncthreads();
      ncand = 0;
    }
#pragma unroll
    for (int k = 0; k < kPer; ++k)
      if ((mask >> k) & 1u) cand[ncand + off++] = packed[k];
    ncand += (int)total;
    __syncthreads();
  }
  flush_candidates(owner, Xp, r, d, max_order, p, cap, base, cand, ncand, lbuf, written, link_node, link_q, link_meta);
  if (threadIdx.x == 0) {
    if (written > cap) {
      atomicOr(err, kErrCapacity);
      written = cap;
    }
    link_count[p] = written;
  }
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

__global__ void __launch_bounds__(256)
k_wall_links(const uint32_t* __restrict__ owner, Dims d, double R, double pcx, double pcy, uint32_t* __restrict__ counter,
             uint32_t cap, uint32_t* __restrict__ node_out, float* __restrict__ q_out, uint8_t* __restrict__ meta_out,
             int count_only) {
  const uint32_t n = blockIdx.x * 256u + threadIdx.x;
  if (n >= d.N) return;
  if (owner[n] != kFluid) return;
  int x, y, z;
  node_coords(n, d.nx, d.ny, x, y, z);
  for (int a = 1; a < kQ; ++a) {
    if (owner[neighbour(x, y, z, 1, a, d)] != kWall) continue;
    const uint32_t slot = atomicAdd(counter, 1u);
    if (count_only || slot >= cap) continue;
    const double q = pipe_q((double)x - pcx, (double)y - pcy, cx_of(a), cy_of(a), R);
    const bool f1 = owner[neighbour(x, y, z, -1, a, d)] == kFluid;
    const uint32_t s = pick_scheme(q, f1, false, 1);
    node_out[slot] = pack_xyz(x, y, z);
    q_out[slot] = (float)q;
    meta_out[slot] = (uint8_t)(a | (s << 5));
  }
}

}  // namespace

hipError_t launch_owner_fill(const Ctx& c, uint32_t* owner) {
  const uint32_t N = c.dims.N;
  hipLaunchKernelGGL(k_owner_fill, dim3((N + 255) / 256), dim3(256), 0, c.stream, owner, c.ibb.wall_bits, N);
  return hipGetLastError();
}

hipError_t launch_owner_clear(const Ctx& c, uint32_t* owner, const double* Xold, int32_t np_old) {
  if (np_old <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_owner_clear, dim3(np_old), dim3(kBlock), 0, c.stream, owner, Xold, c.P.r, c.dims);
  return hipGetLastError();
}

hipError_t launch_owner_set(const Ctx& c, uint32_t* owner, const double* X) {
  if (c.np <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_owner_set, dim3(c.np), dim3(kBlock), 0, c.stream, owner, X, c.P.r, c.dims);
  return hipGetLastError();
}

hipError_t launch_count_solid(const Ctx& c, const uint32_t* owner, unsigned long long* out) {
  const uint32_t N = c.dims.N;
  hipLaunchKernelGGL(k_count_solid, dim3((N + 255) / 256), dim3(256), 0, c.stream, owner, N, out);
  return hipGetLastError();
}

hipError_t launch_links_build(const Ctx& c, const uint32_t* owner, const double* X) {
  if (c.np <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_links_build, dim3(c.np), dim3(kBlock), 0, c.stream, owner, X, c.P.r, c.dims,
                     c.cfg.ibb_max_order, c.link_cap, c.ibb.link_node, c.ibb.link_q, c.ibb.link_meta,
                     c.ibb.link_count, c.err);
  return hipGetLastError();
}

hipError_t launch_wall_links(Ctx& c, const uint32_t* owner, uint32_t* counter, bool count_only) {
  const uint32_t N = c.dims.N;
  hipLaunchKernelGGL(k_wall_links, dim3((N + 255) / 256), dim3(256), 0, c.stream, owner, c.dims, c.cfg.pipe_radius,
                     c.cfg.pipe_cx, c.cfg.pipe_cy, counter, c.ibb.wl_count, c.ibb.wl_node, c.ibb.wl_q,
                     c.ibb.wl_meta, count_only ? 1 : 0);
  return hipGetLastError();
}

}  // namespace lbm
