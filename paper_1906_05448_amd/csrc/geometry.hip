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
constexpr int kCand = 4096;     // shell candidates buffered in LDS per round of rows
constexpr int kRowList = 4096;  // nodes listed per round of rows in the owner passes

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

// Calls f(n) for every node n inside the sphere (Xp, r) by the exact test.
// A round of rows of the sphere's box lists the nodes that may be inside in
// LDS (two square roots per row), flagging those certainly inside; the
// others take the exact test. Every thread of the block must call it.
template <class F>
__device__ void for_sphere_nodes(const double* Xp, double r, const Dims& d, uint32_t* list, F&& f) {
  const Box b = make_box(Xp, r + 1.0);
  const double r2 = r * r;
  const int rows = b.side[1] * b.side[2];
  const int R = min(kBlock, kRowList / b.side[0]);  // a round's nodes fit in the list
  const int xlo = b.lo[0], xhi = b.lo[0] + b.side[0] - 1;
  for (int r0 = 0; r0 < rows; r0 += R) {
    const int row = r0 + (int)threadIdx.x;
    int a0 = 1, a1 = 0, ly = 0, lz = 0;
    RowSpan sp{};
    if ((int)threadIdx.x < R && row < rows) {
      ly = row % b.side[1];
      lz = row / b.side[1];
      const double dy = (double)(b.lo[1] + ly) - Xp[1], dz = (double)(b.lo[2] + lz) - Xp[2];
      sp = sphere_row(Xp[0], dy * dy + dz * dz, r2);
      if (sp.any) {
        a0 = max((int)ceil(sp.plo), xlo);
        a1 = min((int)floor(sp.phi), xhi);
      }
    }
    uint32_t total;
    uint32_t off = block_exclusive_scan<kBlock>(a1 >= a0 ? (uint32_t)(a1 - a0 + 1) : 0u, &total);
    // entry: x, y, z offsets in the box (10 bits each), certainly inside (bit 31)
    for (int x = a0; x <= a1; ++x)
      list[off++] = (uint32_t)(x - xlo) | ((uint32_t)ly << 10) | ((uint32_t)lz << 20) |
                    (((double)x > sp.clo && (double)x < sp.chi) ? 0x80000000u : 0u);
    __syncthreads();
    for (uint32_t j = threadIdx.x; j < total; j += kBlock) {
      const uint32_t e = list[j];
      const int x = wrap1(xlo + (int)(e & 1023u), d.nx);
      const int y = wrap1(b.lo[1] + (int)((e >> 10) & 1023u), d.ny);
      const int z = wrap1(b.lo[2] + (int)((e >> 20) & 1023u), d.nz);
      if ((e >> 31) || inside_sphere(x, y, z, Xp, r, d.nx, d.ny, d.nz)) f(node_index(x, y, z, d.nx, d.ny));
    }
    __syncthreads();  // the list is refilled by the next round
  }
}

// Resets the nodes inside every particle at its old position to fluid (every
// entry a set pass wrote lies inside some sphere at the positions it used).
__global__ void __launch_bounds__(kBlock) k_owner_clear(uint32_t* __restrict__ owner, const double* __restrict__ Xold,
                                                        const double* __restrict__ rad, Dims d) {
  __shared__ uint32_t list[kRowList];
  const int p = blockIdx.x;
  for_sphere_nodes(Xold + 3 * p, rad[p], d, list, [&](uint32_t n) {
    if (owner[n] != kWall) owner[n] = kFluid;
  });
}

// Xown (optional) receives the positions the map was set with.
__global__ void __launch_bounds__(kBlock) k_owner_set(uint32_t* __restrict__ owner, const double* __restrict__ X,
                                                      const double* __restrict__ rad, Dims d,
                                                      double* __restrict__ Xown) {
  __shared__ uint32_t list[kRowList];
  const uint32_t p = blockIdx.x;
  if (Xown && threadIdx.x < 3) Xown[3 * p + threadIdx.x] = X[3 * p + threadIdx.x];
  for_sphere_nodes(X + 3 * p, rad[p], d, list, [&](uint32_t n) { atomicMin(owner + n, p); });
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

// Shell candidates of one row of a sphere's box. With e2 the squared
// distance of the row (y, z) from the centre, a link's fluid end x satisfies
// (x - X0)^2 < ro2 - e2 (it lies within r + |c| of the centre) and is not
// inside the sphere, (x - X0)^2 >= r2 - e2. Both bounds only prune (the owner
// map decides), so the intervals are taken slightly wide: the hole keeps a
// margin of 1e-6 (r2 + 1) below r2, so every node it drops is inside the
// sphere by the owner map's test as well. Returns up to two intervals
// [a0, a1], [b0, b1] of unwrapped x within [lo, hi]; empty ones have a1 < a0.
__device__ __forceinline__ void shell_row(double X0, double e2, double r2, double ro2, int lo, int hi, int& a0, int& a1,
                                          int& b0, int& b1) {
  a0 = b0 = 1;
  a1 = b1 = 0;
  if (!(e2 < ro2)) return;
  const double xo = sqrt(ro2 - e2) + 1e-9;
  const int o0 = max((int)ceil(X0 - xo), lo), o1 = min((int)floor(X0 + xo), hi);
  a0 = o0;
  a1 = o1;
  const double hole = r2 - e2 - 1e-6 * (r2 + 1.0);
  if (!(hole > 0.0)) return;
  // dropped: |x - X0| < xi, the integers strictly between X0 - xi and X0 + xi
  const double xi = sqrt(hole) - 1e-9;
  const int left_hi = (int)floor(X0 - xi), right_lo = (int)ceil(X0 + xi);
  if (left_hi + 1 > right_lo - 1) return;
  a1 = min(left_hi, o1);
  b0 = max(right_lo, max(o0, a1 + 1));
  b1 = o1;
}

__device__ __forceinline__ uint32_t plane_bit(const uint32_t* plane, int i) {
  return (plane[i >> 5] >> (i & 31)) & 1u;
}

// Examines the listed shell candidates (local coordinates in the staged box
// sb) and writes their links from slot `written` on. Every thread must call
// it. Per chunk of kBlock candidates the lanes find each candidate's links
// from the LDS bit planes (fluid, owned by p), list them in LDS in
// candidate-then-direction order, then evaluate q and the scheme with one
// link per lane, so the FP64 root is computed with every lane busy and the
// records are written contiguously.
__device__ void flush_candidates(const uint32_t* fl, const uint32_t* op, const Box& sb, const double* Xp, double r,
                                 const Dims& d, int max_order, uint32_t cap, size_t base, const uint32_t* cand,
                                 int ncand, uint16_t* lbuf, uint32_t& written, uint32_t* __restrict__ link_node,
                                 float* __restrict__ link_q, uint8_t* __restrict__ link_meta) {
  const int sx = sb.side[0], sxy = sb.side[0] * sb.side[1];
  for (int c0 = 0; c0 < ncand; c0 += kBlock) {
    const int k = c0 + (int)threadIdx.x;
    uint32_t hits = 0, fluid1 = 0, fluid2 = 0;
    if (k < ncand) {
      const uint32_t e = cand[k];
      const int i = (int)(e & 0xFFu) + sx * (int)((e >> 8) & 0xFFu) + sxy * (int)(e >> 16);
      if (plane_bit(fl, i)) {
#pragma unroll
        for (int a = 1; a < kQ; ++a) {
          const int o = cx_of(a) + sx * cy_of(a) + sxy * cz_of(a);
          hits |= plane_bit(op, i + o) << a;
          fluid1 |= plane_bit(fl, i - o) << a;
          fluid2 |= plane_bit(fl, i - 2 * o) << a;
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
      const uint32_t loc = cand[c0 + (int)(e & 0xFFu)];
      const int a = (int)((e >> 8) & 31u);
      const int x = wrap1(sb.lo[0] + (int)(loc & 0xFFu), d.nx);
      const int y = wrap1(sb.lo[1] + (int)((loc >> 8) & 0xFFu), d.ny);
      const int z = wrap1(sb.lo[2] + (int)(loc >> 16), d.nz);
      const double dx = min_image((double)x - Xp[0], d.nx);
      const double dy = min_image((double)y - Xp[1], d.ny);
      const double dz = min_image((double)z - Xp[2], d.nz);
      const double q = sphere_q(dx, dy, dz, cx_of(a), cy_of(a), cz_of(a), r);
      const uint32_t sch = pick_scheme(q, (e >> 13) & 1u, (e >> 14) & 1u, max_order);
      const uint32_t slot = written + j;
      if (slot < cap) {
        link_node[base + slot] = pack_xyz(x, y, z);
        link_q[base + slot] = (float)q;
        link_meta[base + slot] = (uint8_t)(a | (sch << 5));
      }
    }
    written += total;
    __syncthreads();  // lbuf is refilled by the next chunk
  }
}

// One workgroup per sphere. The owner map over the sphere's box plus two
// nodes (every entry a candidate's 55 tests read) is staged in LDS as two
// bit planes, built from coalesced row reads with wavefront ballots. The
// candidates are then listed row by row from the shell intervals, a round of
// rows at a time, and their links written in that order (deterministic).
__global__ void __launch_bounds__(kBlock)
k_links_build(const uint32_t* __restrict__ owner, const double* __restrict__ X, const double* __restrict__ rad, Dims d,
              int max_order, uint32_t cap, uint32_t* __restrict__ link_node, float* __restrict__ link_q,
              uint8_t* __restrict__ link_meta, uint32_t* __restrict__ link_count, uint32_t* __restrict__ err) {
  extern __shared__ uint32_t planes[];  // fluid bits, then owned-by-p bits, of the staged box
  __shared__ uint32_t cand[kCand];
  __shared__ uint16_t lbuf[kBlock * (kQ - 1)];  // a chunk's links, at most every direction of every candidate
  const uint32_t p = blockIdx.x;
  const double r = rad[p];
  const double* Xp = X + 3 * p;
  const size_t base = (size_t)p * cap;
  // The outer bound only prunes, so it carries a margin.
  const double r_out = r + 1.4142135623730951 + 1e-6;
  const double r2 = r * r, ro2 = r_out * r_out;
  const Box cb = make_box(Xp, r_out);  // every candidate, unwrapped coordinates
  Box sb;                               // staged: two more nodes on each side
  for (int k = 0; k < 3; ++k) {
    sb.lo[k] = cb.lo[k] - 2;
    sb.side[k] = cb.side[k] + 4;
  }
  const BoxLin SL = box_lin(sb);
  uint32_t* fl = planes;
  uint32_t* op = planes + (SL.count + 63u) / 64u * 2u;
  constexpr int kU = 8;  // owner reads in flight per thread
  for (uint32_t i0 = 0; i0 < SL.count; i0 += kU * kBlock) {
    uint32_t o[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const uint32_t i = i0 + (uint32_t)(u * kBlock) + threadIdx.x;
      o[u] = kFluid;
      if (i < SL.count) {
        int x, y, z;
        box_lin_node(sb, SL, i, d.nx, d.ny, d.nz, x, y, z);
        o[u] = owner[node_index(x, y, z, d.nx, d.ny)];
      }
    }
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const uint32_t i = i0 + (uint32_t)(u * kBlock) + threadIdx.x;
      const uint64_t bf = __ballot(i < SL.count && o[u] == kFluid);
      const uint64_t bp = __ballot(i < SL.count && o[u] == p);
      if ((threadIdx.x & 63u) == 0 && i < SL.count) {  // i is a multiple of 64 here
        fl[i >> 5] = (uint32_t)bf;
        fl[(i >> 5) + 1] = (uint32_t)(bf >> 32);
        op[i >> 5] = (uint32_t)bp;
        op[(i >> 5) + 1] = (uint32_t)(bp >> 32);
      }
    }
  }
  __syncthreads();
  const int rows = cb.side[1] * cb.side[2];
  const int R = min(kBlock, kCand / cb.side[0]);  // rows per round: a round's candidates fit in cand
  const int xlo = cb.lo[0], xhi = cb.lo[0] + cb.side[0] - 1;
  uint32_t written = 0;
  for (int r0 = 0; r0 < rows; r0 += R) {
    const int row = r0 + (int)threadIdx.x;
    int a0 = 1, a1 = 0, b0 = 1, b1 = 0, ly = 0, lz = 0;
    if ((int)threadIdx.x < R && row < rows) {
      ly = row % cb.side[1];
      lz = row / cb.side[1];
      const double dy = (double)(cb.lo[1] + ly) - Xp[1], dz = (double)(cb.lo[2] + lz) - Xp[2];
      shell_row(Xp[0], dy * dy + dz * dz, r2, ro2, xlo, xhi, a0, a1, b0, b1);
    }
    const int na = a1 >= a0 ? a1 - a0 + 1 : 0, nb = b1 >= b0 ? b1 - b0 + 1 : 0;
    uint32_t total;
    uint32_t off = block_exclusive_scan<kBlock>((uint32_t)(na + nb), &total);
    const uint32_t yz = ((uint32_t)(ly + 2) << 8) | ((uint32_t)(lz + 2) << 16);
    for (int x = a0; x <= a1; ++x) cand[off++] = (uint32_t)(x - sb.lo[0]) | yz;
    for (int x = b0; x <= b1; ++x) cand[off++] = (uint32_t)(x - sb.lo[0]) | yz;
    __syncthreads();
    flush_candidates(fl, op, sb, Xp, r, d, max_order, cap, base, cand, (int)total, lbuf, written, link_node, link_q,
                     link_meta);
  }
  if (threadIdx.x == 0) {
    if (written > cap) {
      atomicOr(err, kErrCapacity);
      written = cap;
    }
    link_count[p] = written;
  }
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

hipError_t launch_owner_set(const Ctx& c, uint32_t* owner, const double* X, double* Xown) {
  if (c.np <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_owner_set, dim3(c.np), dim3(kBlock), 0, c.stream, owner, X, c.P.r, c.dims, Xown);
  return hipGetLastError();
}

hipError_t launch_count_solid(const Ctx& c, const uint32_t* owner, unsigned long long* out) {
  const uint32_t N = c.dims.N;
  hipLaunchKernelGGL(k_count_solid, dim3((N + 255) / 256), dim3(256), 0, c.stream, owner, N, out);
  return hipGetLastError();
}

// Bit planes of the staged owner box: the candidate box of a sphere of the
// largest radius (at most floor(2 r_out) + 3 nodes a side) plus two nodes on
// each side.
size_t links_build_lds_bytes(double max_radius) {
  const size_t side = (size_t)std::floor(2.0 * (max_radius + 1.4142135623730951 + 1e-6)) + 7;
  return 2 * ((side * side * side + 63) / 64 * 2) * sizeof(uint32_t);
}

// Dynamic plus static LDS of one link-build workgroup.
size_t links_build_lds_total(double max_radius) {
  return links_build_lds_bytes(max_radius) + kCand * sizeof(uint32_t) + kBlock * (kQ - 1) * sizeof(uint16_t) + 64;
}

hipError_t launch_links_build(const Ctx& c, const uint32_t* owner, const double* X) {
  if (c.np <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_links_build, dim3(c.np), dim3(kBlock), links_build_lds_bytes(c.cfg.max_radius), c.stream,
                     owner, X, c.P.r, c.dims,
                     c.cfg.ibb_max_order, c.link_cap, c.ibb.link_node, c.ibb.link_q, c.ibb.link_meta,
                     c.ibb.link_count, c.err);
  return hipGetLastError();
}

hipError_t launch_wall_links(Ctx& c, const uint32_t* owner, uint32_t* counter, bool count_only) {
  if (lattice27(c)) return launch_wall_links27(c, owner, counter, count_only);
  const uint32_t N = c.dims.N;
  hipLaunchKernelGGL(k_wall_links, dim3((N + 255) / 256), dim3(256), 0, c.stream, owner, c.dims, c.cfg.pipe_radius,
                     c.cfg.pipe_cx, c.cfg.pipe_cy, counter, c.ibb.wl_count, c.ibb.wl_node, c.ibb.wl_q,
                     c.ibb.wl_meta, count_only ? 1 : 0);
  return hipGetLastError();
}

}  // namespace lbm
