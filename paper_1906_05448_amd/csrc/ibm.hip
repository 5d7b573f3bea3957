// ibm.hip - immersed boundary method on moving spheres (Sec. 2.1, Sec. 3.1):
// Peskin 4-point delta (Peskin 2002), multi-direct forcing with the
// prediction plus ibm_iters passes, and the Kempe et al. (2012) inner-fluid
// inertia, FP64 per-particle sums.
//
// Step structure (support of step n built at the end of step n-1):
//   prepass   pull the 19 populations at every support node: rho and
//             u* = (sum c f + F_body/2) / rho into the slot arrays
//   passes    one workgroup per sphere stages its forcing support (union
//             of its marker stencils) in LDS: u = u* + f_IB/(2 rho);
//             markers interpolate U_l, dF_l = 2 (U_d - U_l) (reference
//             density 1, half-force velocity), then spread dF_l delta dV
//             into LDS fixed-point sums. Nodes of this sphere alone get the
//             sum added to their slot force in place; at nodes another
//             sphere's support shares, the sums go to separate exact 64-bit
//             accumulators that a fold kernel adds to the slot forces after
//             the pass. So every marker of a pass reads the velocity of the
//             end of the previous pass, whatever the order the workgroups
//             run in, and the result does not depend on that order.
//   kempe     sum alpha u and sum alpha (x - X) x u over the cells with
//             solid fraction alpha > 0, per sphere, in FP64
//   dense     the fused stream + collide adds f_IB at support nodes
//   build     support of step n+1 from the new centres
// Marker positions are X + r_L n_k in FP64 with the box-local stencil base
// floor(X_l) - 1, so the stencil nodes match an FP64 reference.
#include "device_util.hpp"
#include "internal.hpp"

namespace lbm {

namespace {

constexpr int kBlock = 256;
constexpr double kAlphaReach = 0.8661;  // > sqrt(3)/2: cells with any corner inside

__device__ __forceinline__ float peskin(float r) {
  const float a = fabsf(r);
  if (a <= 1.0f) return (3.0f - 2.0f * a + sqrtf(1.0f + 4.0f * a - 4.0f * a * a)) * 0.125f;
  if (a < 2.0f) return (5.0f - 2.0f * a - sqrtf(fmaxf(-7.0f + 12.0f * a - 4.0f * a * a, 0.0f))) * 0.125f;
  return 0.0f;
}

// Box of a sphere: floor(X) - R_b .. floor(X) + R_b + 1 per axis.
__device__ __forceinline__ void ibm_box_lo(const double* X, int R_b, int lo[3]) {
  for (int k = 0; k < 3; ++k) lo[k] = (int)floor(X[k]) - R_b;
}

// A marker of a sphere: stencil base (box-local, packed 10 bits per axis)
// and the offsets t = x_l - floor(x_l) per axis.
struct MarkerPos {
  uint32_t base;
  float t[3];
};

__device__ __forceinline__ void marker_pos(const double* X, const double* dir, double r_l, const int lo[3],
                                           MarkerPos& m) {
  m.base = 0;
  for (int k = 0; k < 3; ++k) {
    const double xl = X[k] + r_l * dir[k];
    const double fl = floor(xl);
    m.t[k] = (float)(xl - fl);
    m.base |= (uint32_t)((int)fl - 1 - lo[k]) << (10 * k);
  }
}

// The four Peskin weights of the points floor(x) - 1 .. floor(x) + 2 for the
// offset t = x - floor(x) in [0, 1): their distances 1 + t, t, 1 - t, 2 - t
// all take the same square root sqrt(1 + 4t - 4t^2), so one root gives all
// four (they add up to one).
__device__ __forceinline__ void peskin4(float t, float (&w)[4]) {
  const float S = sqrtf(1.0f + 4.0f * t * (1.0f - t));
  const float a = 3.0f - 2.0f * t, b = 1.0f + 2.0f * t;
  w[0] = (a - S) * 0.125f;
  w[1] = (a + S) * 0.125f;
  w[2] = (b + S) * 0.125f;
  w[3] = (b - S) * 0.125f;
}

// ---------------------------------------------------------------- build --
// Per sphere: forcing rows (marker stencils) and the full support (stencils
// plus Kempe cells) in LDS, then the global support bits and the
// shared-node bits.
__global__ void __launch_bounds__(kBlock)
k_ibm_mark(const double* __restrict__ X, const double* __restrict__ rad, const double* __restrict__ dirs, int nmk,
           double r_l, int R_b, int side, Dims d, uint32_t* __restrict__ bits, uint32_t* __restrict__ shared,
           uint32_t* __restrict__ rowbits_out, uint32_t* __restrict__ fcount, uint32_t fcap,
           uint32_t* __restrict__ err) {
  extern __shared__ uint32_t lds[];
  const int rows = side * side;
  uint32_t* fb = lds;          // forcing rows
  uint32_t* ab = lds + rows;   // Kempe-cell rows
  const int p = blockIdx.x;
  const double* Xp = X + 3 * p;
  const double r = rad[p];
  int lo[3];
  ibm_box_lo(Xp, R_b, lo);
  for (int i = threadIdx.x; i < rows; i += kBlock) fb[i] = ab[i] = 0u;
  __syncthreads();
  for (int l = threadIdx.x; l < nmk; l += kBlock) {
    MarkerPos mp;
    marker_pos(Xp, dirs + 3 * l, r_l, lo, mp);
    const int bx = (int)(mp.base & 1023u), by = (int)((mp.base >> 10) & 1023u), bz = (int)(mp.base >> 20);
    const uint32_t m = 0xFu << bx;
    for (int jz = 0; jz < 4; ++jz)
      for (int jy = 0; jy < 4; ++jy) atomicOr(&fb[(by + jy) + side * (bz + jz)], m);
  }
  // Kempe cells, one thread per row: the candidates are the ball's x range
  // widened by one, the exact test (the Kempe kernel's) decides.
  const double ra = r + kAlphaReach;
  const double ra2 = ra * ra;
  for (int row = threadIdx.x; row < rows; row += kBlock) {
    const int ly = row % side, lz = row / side;
    const int y = wrap1(lo[1] + ly, d.ny), z = wrap1(lo[2] + lz, d.nz);
    const double dy = min_image((double)y - Xp[1], d.ny), dz = min_image((double)z - Xp[2], d.nz);
    const double e2 = dist2(0.0, dy, dz);
    uint32_t mrow = 0u;
    if (e2 < ra2) {
      const double hx = sqrt(ra2 - e2);
      const int c0 = max(0, (int)floor(Xp[0] - hx) - 1 - lo[0]);
      const int c1 = min(side - 1, (int)ceil(Xp[0] + hx) + 1 - lo[0]);
      for (int lx = c0; lx <= c1; ++lx) {
        const int x = wrap1(lo[0] + lx, d.nx);
        if (dist2(min_image((double)x - Xp[0], d.nx), dy, dz) < ra2) mrow |= 1u << lx;
      }
    }
    ab[row] = mrow;
  }
  __syncthreads();
  // The row's nodes are consecutive unless the box wraps around x: then the
  // mask goes out in two shifted words at most.
  const bool xwrap = lo[0] < 0 || lo[0] + side > d.nx;
  auto put = [&](uint32_t word, uint32_t wm) {
    if (!wm) return;
    const uint32_t old = atomicOr(bits + word, wm);
    if (old & wm) atomicOr(shared + word, old & wm);
  };
  uint32_t cnt = 0;
  for (int row = threadIdx.x; row < rows; row += kBlock) {
    const uint32_t f = fb[row];
    rowbits_out[(size_t)p * rows + row] = f;
    cnt += __popc(f);
    uint32_t m = f | ab[row];
    if (!m) continue;
    const int ly = row % side, lz = row / side;
    const int y = wrap1(lo[1] + ly, d.ny), z = wrap1(lo[2] + lz, d.nz);
    if (!xwrap) {
      const uint32_t n0 = node_index(lo[0], y, z, d.nx, d.ny);
      const uint64_t M = (uint64_t)m << (n0 & 31u);
      put(n0 >> 5, (uint32_t)M);
      put((n0 >> 5) + 1u, (uint32_t)(M >> 32));
      continue;
    }
    uint32_t word = 0xFFFFFFFFu, wm = 0u;
    while (m) {
      const int lx = __ffs(m) - 1;
      m &= m - 1u;
      const uint32_t n = node_index(wrap1(lo[0] + lx, d.nx), y, z, d.nx, d.ny);
      if ((n >> 5) != word) {
        put(word, wm);
        word = n >> 5;
        wm = 0u;
      }
      wm |= 1u << (n & 31u);
    }
    put(word, wm);
  }
  const double tot = block_sum<kBlock>((double)cnt);
  if (threadIdx.x == 0) {
    uint32_t t = (uint32_t)tot;
    if (t > fcap) {
      atomicOr(err, kErrCapacity);
      t = fcap;
    }
    fcount[p] = t;
  }
}

// Exclusive rank of the support words: per-block partial scans, a scan of
// the block sums, then the offsets plus the slot -> node list.
constexpr int kScanPer = 4;  // words per thread
constexpr int kScanWords = kBlock * kScanPer;

__global__ void __launch_bounds__(kBlock) k_scan_block(const uint32_t* __restrict__ bits, uint32_t nwords,
                                                      uint32_t* __restrict__ rank, uint32_t* __restrict__ block_sums) {
  const uint32_t w0 = blockIdx.x * kScanWords + threadIdx.x * kScanPer;
  uint32_t c[kScanPer], s = 0;
  for (int k = 0; k < kScanPer; ++k) {
    c[k] = (w0 + k < nwords) ? __popc(bits[w0 + k]) : 0u;
    s += c[k];
  }
  uint32_t total;
  uint32_t off = block_exclusive_scan<kBlock>(s, &total);
  for (int k = 0; k < kScanPer; ++k) {
    if (w0 + k < nwords) rank[w0 + k] = off;
    off += c[k];
  }
  if (threadIdx.x == 0) block_sums[blockIdx.x] = total;
}

__global__ void __launch_bounds__(1024) k_scan_top(uint32_t* __restrict__ block_sums, uint32_t nblocks,
                                                   uint32_t* __restrict__ count) {
  uint32_t carry = 0;
  for (uint32_t b0 = 0; b0 < nblocks; b0 += 1024) {
    const uint32_t i = b0 + threadIdx.x;
    const uint32_t v = i < nblocks ? block_sums[i] : 0u;
    uint32_t total;
    const uint32_t off = block_exclusive_scan<1024>(v, &total);
    if (i < nblocks) block_sums[i] = carry + off;
    carry += total;
  }
  if (threadIdx.x == 0) *count = carry;
}

// Adds the block offsets to the word ranks, then lists the set bits' nodes
// by slot: each wavefront expands two words per step with one lane per bit,
// so a dense word's 32 slots are written by 32 consecutive lanes.
__global__ void __launch_bounds__(kBlock) k_scan_add(const uint32_t* __restrict__ bits, uint32_t nwords,
                                                    uint32_t* __restrict__ rank,
                                                    const uint32_t* __restrict__ block_sums,
                                                    uint32_t* __restrict__ list, uint32_t s_cap,
                                                    uint32_t* __restrict__ err) {
  __shared__ uint32_t wb[kScanWords], wr[kScanWords];
  const uint32_t base = blockIdx.x * kScanWords;
  const uint32_t add = block_sums[blockIdx.x];
  for (int k = 0; k < kScanPer; ++k) {
    const uint32_t i = threadIdx.x + (uint32_t)(k * kBlock), w = base + i;
    uint32_t m = 0u, rk = 0u;
    if (w < nwords) {
      rk = rank[w] + add;
      rank[w] = rk;
      m = bits[w];
    }
    wb[i] = m;
    wr[i] = rk;
  }
  __syncthreads();
  const uint32_t lane = threadIdx.x & 63u, bit = lane & 31u;
  for (uint32_t i = (threadIdx.x >> 6) * 2u + (lane >> 5); i < (uint32_t)kScanWords; i += kBlock / 32) {
    const uint32_t m = wb[i];
    if (!((m >> bit) & 1u)) continue;
    const uint32_t slot = wr[i] + __popc(m & ((1u << bit) - 1u));
    if (slot < s_cap)
      list[slot] = (base + i) * 32u + bit;
    else
      atomicOr(err, kErrCapacity);
  }
}

__device__ __forceinline__ bool support_slot(const uint32_t* bits, const uint32_t* rank, uint32_t n, uint32_t& slot) {
  const uint32_t w = bits[n >> 5];
  const uint32_t b = n & 31u;
  if (!((w >> b) & 1u)) return false;
  slot = rank[n >> 5] + __popc(w & ((1u << b) - 1u));
  return true;
}

// Per sphere: global slot of every forcing-support node, in box raster order,
// or, where another support shares the node, bit 31 set and the node's index
// among the shared nodes (slots and indices stay below 2^31). A box row (side <= 32 nodes) touches at most two words of the
// support bitmask per contiguous x segment, and there are two segments when
// the row wraps around x. Those words, their ranks and their shared bits are
// loaded once per row, all together, and every slot of the row is formed
// from them.
constexpr uint32_t kSlotShared = 0x80000000u;

__global__ void __launch_bounds__(kBlock)
k_ibm_slots(const double* __restrict__ X, int R_b, int side, Dims d, const uint32_t* __restrict__ bits,
            const uint32_t* __restrict__ rank, const uint32_t* __restrict__ shared,
            const uint32_t* __restrict__ sh_rank, const uint32_t* __restrict__ rowbits,
            const uint32_t* __restrict__ fcount, uint32_t fcap, uint32_t* __restrict__ fslot) {
  const int rows = side * side;
  const int p = blockIdx.x;
  int lo[3];
  ibm_box_lo(X + 3 * p, R_b, lo);
  const uint32_t cap = fcount[p];
  uint32_t base = 0;
  for (int r0 = 0; r0 < rows; r0 += kBlock) {
    const int row = r0 + threadIdx.x;
    uint32_t m = row < rows ? rowbits[(size_t)p * rows + row] : 0u;
    uint32_t total;
    uint32_t j = base + block_exclusive_scan<kBlock>(__popc(m), &total);
    if (m) {
      const int ly = row % side, lz = row / side;
      const int y = wrap1(lo[1] + ly, d.ny), z = wrap1(lo[2] + lz, d.nz);
      const uint32_t rowbase = ((uint32_t)z * (uint32_t)d.ny + (uint32_t)y) * (uint32_t)d.nx;
      const int xa = wrap1(lo[0] + (__ffs(m) - 1), d.nx), xb = wrap1(lo[0] + (31 - __clz(m)), d.nx);
      // words of the first node of each segment and the one after it
      uint32_t w[4], wb[4], wr[4], ws[4], wq[4];
      w[0] = (rowbase + (uint32_t)xa) >> 5;
      w[2] = rowbase >> 5;  // wrapped segment starts at x = 0
      const uint32_t last1 = xa <= xb ? (rowbase + (uint32_t)xb) >> 5 : (rowbase + (uint32_t)d.nx - 1u) >> 5;
      const bool wrapped = xa > xb;
      const uint32_t last2 = wrapped ? (rowbase + (uint32_t)xb) >> 5 : 0u;
      w[1] = last1 > w[0] ? w[0] + 1u : w[0];
      w[3] = wrapped && last2 > w[2] ? w[2] + 1u : w[2];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const bool use = k < 2 || wrapped;
        wb[k] = use ? bits[w[k]] : 0u;
        wr[k] = use ? rank[w[k]] : 0u;
        ws[k] = use ? shared[w[k]] : 0u;
        wq[k] = use ? sh_rank[w[k]] : 0u;
      }
      while (m) {
        const int lx = __ffs(m) - 1;
        m &= m - 1u;
        const uint32_t n = rowbase + (uint32_t)wrap1(lo[0] + lx, d.nx);
        const uint32_t wn = n >> 5;
        const int k = wn == w[0] ? 0 : (wn == w[1] ? 1 : (wn == w[2] ? 2 : 3));
        const uint32_t word = k == 0 ? wb[0] : (k == 1 ? wb[1] : (k == 2 ? wb[2] : wb[3]));
        const uint32_t rk = k == 0 ? wr[0] : (k == 1 ? wr[1] : (k == 2 ? wr[2] : wr[3]));
        const uint32_t sw = k == 0 ? ws[0] : (k == 1 ? ws[1] : (k == 2 ? ws[2] : ws[3]));
        const uint32_t below = (1u << (n & 31u)) - 1u;
        uint32_t entry;
        if ((sw >> (n & 31u)) & 1u) {
          const uint32_t sq = k == 0 ? wq[0] : (k == 1 ? wq[1] : (k == 2 ? wq[2] : wq[3]));
          entry = kSlotShared | (sq + __popc(sw & below));
        } else {
          entry = rk + __popc(word & below);
        }
        if (j < cap) fslot[(size_t)p * fcap + j] = entry;
        ++j;
      }
    }
    base += total;
  }
}

// -------------------------------------------------------------- prepass --
template <int STORE>
__global__ void __launch_bounds__(256)
k_ibm_prepass(const typename Pop<STORE>::T* __restrict__ A, Dims d, float3 F0, const uint32_t* __restrict__ nobody,
              const uint32_t* __restrict__ list, const uint32_t* __restrict__ count, uint32_t s_cap,
              float4* __restrict__ us, float4* __restrict__ fib) {
  const uint32_t s = blockIdx.x * 256u + threadIdx.x;
  if (s >= *count || s >= s_cap) return;
  const uint32_t n = list[s];
  // no body force outside the pipe (the virtual fluid there is not driven)
  const float3 F = (nobody && ((nobody[n >> 5] >> (n & 31u)) & 1u)) ? make_float3(0.0f, 0.0f, 0.0f) : F0;
  int x, y, z;
  node_coords(n, d.nx, d.ny, x, y, z);
  float drho = 0.0f, jx = 0.0f, jy = 0.0f, jz = 0.0f;
#pragma unroll
  for (int i = 0; i < kQ; ++i) {
    const uint32_t src = node_index(wrap1(x - cx_of(i), d.nx), wrap1(y - cy_of(i), d.ny), wrap1(z - cz_of(i), d.nz),
                                    d.nx, d.ny);
    const float g = Pop<STORE>::load(A + (size_t)i * d.S + src);
    drho += g;
    jx += cx_of(i) * g;
    jy += cy_of(i) * g;
    jz += cz_of(i) * g;
  }
  const float rho = 1.0f + drho;
  us[s] = make_float4((jx + 0.5f * F.x) / rho, (jy + 0.5f * F.y) / rho, (jz + 0.5f * F.z) / rho, rho);
  fib[s] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
}

// --------------------------------------------------------------- passes --
// One 1024-thread workgroup per sphere, MPT markers per thread.
// LDS: rows x (u32 forcing row bits, u32 row prefix), then fcap x 12
// bytes holding first the staged velocities (float3 per node) and, once every
// marker has interpolated, the spread sums (per node the x and y sums packed
// in one 64-bit word, so one 64-bit LDS atomic adds both, and the z sum in
// a 32-bit word), then fcap u32 (the nodes' slot-list entries, kept for the
// write-back). About 74 KB for r = 8, so two spheres share a compute
// unit and one's memory trips overlap the other's LDS work.
//
// The spread sums are 32-bit fixed point in units of 2^-e with a scale
// exponent e per sphere and pass, chosen from the largest |dF| of the
// sphere's markers so that no node sum can reach 2^31: LDS integer atomics
// run at about the rate of plain LDS accesses (float atomics measured about
// 25 times slower on gfx950), integer sums are exact, so a node's total does
// not depend on the order in which markers land, and the per-sphere scale
// keeps the resolution relative to the forces of the pass (a few 1e-9 of the
// largest |dF|) however weak or strong the flow. A node's weights from one
// sphere's markers add up to about 1/2 (one marker per unit area of the
// surface, the delta integrating to one over the tangent plane and to at
// most phi(0) = 1/2 across it); kSpreadBound = 8 covers that with margin.
// At shared nodes the sums are rescaled to the common units 2^-50 and added
// with 64-bit atomics: exact, so the order of the spheres does not matter
// either.
constexpr int kPassBlock = 1024;
// A sphere of radius 8 has about 4 050 - 4 110 forcing-support nodes: one
// staging round (4 096) covers most, one write-back round (5 120) all.
constexpr int kStage = 4;  // support nodes per thread per staging round
constexpr int kWrite = 5;  // support nodes per thread per write-back round
constexpr float kSpreadBound = 8.0f;
constexpr int kShUnitExp = 50;  // shared accumulators: units of 2^-50

__device__ __forceinline__ int spread_exponent(float max_dF, float dV) {
  const float B = max_dF * dV * kSpreadBound;
  if (!(B > 0.0f)) return kShUnitExp;  // no force (or non-finite: the collision latches it)
  int ex;
  (void)frexpf(B, &ex);                // B < 2^ex
  return min(kShUnitExp, max(0, 30 - ex));
}

// A node's x, y, z spread sums from the packed word y 2^32 + x (both
// signed, |x|, |y| < 2^31, so the low word is x and the rest an exact
// multiple of 2^32) and the z word.
__device__ __forceinline__ void unpack_sums(unsigned long long xy, int z, int (&a)[3]) {
  a[0] = (int)(uint32_t)xy;
  a[1] = (int)(((long long)xy - (long long)a[0]) / 4294967296ll);
  a[2] = z;
}

// Slot-list entries j0 + threadIdx.x + i kPassBlock of a sphere and their
// slots (a shared node's from the shared-node table); 0xFFFFFFFF past the
// list.
__device__ __forceinline__ void stage_slots(const uint32_t* __restrict__ slots, const uint32_t* __restrict__ sh_slot,
                                            uint32_t sh_cap, uint32_t cnt, uint32_t fcap, uint32_t j0,
                                            uint32_t (&w)[kStage], uint32_t (&s)[kStage]) {
#pragma unroll
  for (int i = 0; i < kStage; ++i) {
    const uint32_t j = j0 + threadIdx.x + i * kPassBlock;
    w[i] = j < cnt && j < fcap ? slots[j] : 0xFFFFFFFFu;
  }
#pragma unroll
  for (int i = 0; i < kStage; ++i) {
    const uint32_t q = w[i] & ~kSlotShared;
    s[i] = !(w[i] & kSlotShared) ? w[i] : (w[i] != 0xFFFFFFFFu && q < sh_cap ? sh_slot[q] : 0xFFFFFFFFu);
  }
}

template <int MPT>
// One marker per thread: 8 waves per SIMD (<= 64 VGPRs), two workgroups per
// CU; two markers per thread keep one workgroup per CU.
__global__ void __launch_bounds__(kPassBlock, MPT == 1 ? 8 : 4)
k_ibm_pass(const double* __restrict__ X, const double* __restrict__ U, const double* __restrict__ Om,
           const double* __restrict__ dirs, int nmk, double r_l, double dV, int R_b, int side, Dims d,
           const uint32_t* __restrict__ rowbits, const uint32_t* __restrict__ fcount, uint32_t fcap,
           const uint32_t* __restrict__ fslot, const uint32_t* __restrict__ sh_slot, uint32_t sh_cap,
           const float4* __restrict__ us, float4* __restrict__ fib, uint32_t s_cap,
           unsigned long long* __restrict__ sh_acc, double* __restrict__ F_ib, double* __restrict__ T_ib,
           float4* __restrict__ pu, float4* __restrict__ pf, int first, int last) {
  extern __shared__ uint32_t lds[];
  __shared__ double red_f[kPassBlock / 64][6];  // per-wavefront force and torque sums
  __shared__ uint32_t red_m[kPassBlock / 64];   // per-wavefront largest |dF|
  const int rows = side * side;
  uint2* rbp = (uint2*)lds;  // per row: forcing bits, exclusive prefix
  float* uj = (float*)(rbp + rows);
  // The spread sums alias uj once every marker has interpolated: x and y of
  // a node packed in one 64-bit word (y * 2^32 + x, both signed), z apart.
  unsigned long long* acc_xy = (unsigned long long*)(rbp + rows);
  int* acc_z = (int*)(acc_xy + fcap);
  uint32_t* sl = (uint32_t*)(uj + 3 * (size_t)fcap);
  const int p = blockIdx.x;
  const double* Xp = X + 3 * p;
  const uint32_t* slots = fslot + (size_t)p * fcap;
  int lo[3];
  ibm_box_lo(Xp, R_b, lo);
  const uint32_t cnt = fcount[p];
  // The marker positions first: their loads and FP64 arithmetic overlap the
  // staging loads and the row scan below.
  MarkerPos mk[MPT];
#pragma unroll
  for (int m = 0; m < MPT; ++m) {
    const int l = threadIdx.x + m * kPassBlock;
    if (l < nmk) marker_pos(Xp, dirs + 3 * l, r_l, lo, mk[m]);
  }
  // Stage u = u* + f_IB / (2 rho) as the previous pass left it: all loads of
  // a round are issued before any is used, the first round's slot-list
  // entries before the row scan. A shared node's slot comes from the shared-node table. The spread
  // force is zero before the first pass (the pre-pass cleared it). With the
  // per-sphere copies (pu, pf non-null) the first pass gathers (u*, rho) once
  // and keeps it in fslot order; later passes read the unshared nodes from
  // the copies.
  float4* const pu_p = pu ? pu + (size_t)p * fcap : nullptr;
  float4* const pf_p = pf ? pf + (size_t)p * fcap : nullptr;
  uint32_t w[kStage], s[kStage];
  stage_slots(slots, sh_slot, sh_cap, cnt, fcap, 0, w, s);
  // row bits and their exclusive prefix (box raster order = slot list order)
  uint32_t base = 0;
  for (int r0 = 0; r0 < rows; r0 += kPassBlock) {
    const int row = r0 + threadIdx.x;
    const uint32_t m = row < rows ? rowbits[(size_t)p * rows + row] : 0u;
    uint32_t total;
    const uint32_t off = block_exclusive_scan<kPassBlock>(__popc(m), &total);
    if (row < rows) {
      rbp[row] = make_uint2(m, base + off);
    }
    base += total;
  }
  // A forcing support beyond the LDS capacity was latched as an error when it
  // was built; skip the sphere rather than index past the buffers.
  if (base > fcap || base != cnt) return;
  for (uint32_t j0 = 0; j0 < cnt; j0 += kStage * kPassBlock) {
    if (j0) stage_slots(slots, sh_slot, sh_cap, cnt, fcap, j0, w, s);
    float4 v[kStage], f[kStage];
#pragma unroll
    for (int i = 0; i < kStage; ++i) {
      const uint32_t j = j0 + threadIdx.x + i * kPassBlock;
      f[i] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
      if (s[i] >= s_cap) continue;
      if (pu_p && !first && !(w[i] & kSlotShared)) {
        v[i] = pu_p[j];
        f[i] = pf_p[j];
      } else {
        v[i] = us[s[i]];
        if (!first) f[i] = fib[s[i]];
      }
    }
#pragma unroll
    for (int i = 0; i < kStage; ++i) {
      const uint32_t j = j0 + threadIdx.x + i * kPassBlock;
      if (j >= cnt) continue;
      sl[j] = w[i];
      if (s[i] >= s_cap) {
        uj[3 * j] = uj[3 * j + 1] = uj[3 * j + 2] = 0.0f;
        continue;
      }
      if (pu_p && first && !(w[i] & kSlotShared)) pu_p[j] = v[i];
      const float h = 0.5f / v[i].w;
      uj[3 * j] = v[i].x + f[i].x * h;
      uj[3 * j + 1] = v[i].y + f[i].y * h;
      uj[3 * j + 2] = v[i].z + f[i].z * h;
    }
  }
  __syncthreads();
  // interpolate and form the marker forces
  const double Up[3] = {U[3 * p], U[3 * p + 1], U[3 * p + 2]};
  const double Wp[3] = {Om[3 * p], Om[3 * p + 1], Om[3 * p + 2]};
  const float dVf = (float)dV;
  double fsum[6] = {0, 0, 0, 0, 0, 0};  // force and torque on the particle
  float dF[MPT][3];
  float dmax = 0.0f;
#pragma unroll
  for (int m = 0; m < MPT; ++m) {
    const int l = threadIdx.x + m * kPassBlock;
    dF[m][0] = dF[m][1] = dF[m][2] = 0.0f;
    if (l >= nmk) continue;
    const int bx = (int)(mk[m].base & 1023u), by = (int)((mk[m].base >> 10) & 1023u), bz = (int)(mk[m].base >> 20);
    float wx[4], wy[4], wz[4];
    peskin4(mk[m].t[0], wx);
    peskin4(mk[m].t[1], wy);
    peskin4(mk[m].t[2], wz);
    const uint32_t below = (1u << bx) - 1u;
    float Ul[3] = {0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int jy = q & 3, jz = q >> 2;
      const int row = (by + jy) + side * (bz + jz);
      const uint2 rw = rbp[row];
      const uint32_t j0 = rw.y + __popc(rw.x & below);
      const float wyz = wy[jy] * wz[jz];
#pragma unroll
      for (int jx = 0; jx < 4; ++jx) {
        const float w = wx[jx] * wyz;
        const uint32_t j = j0 + jx;
        Ul[0] += w * uj[3 * j];
        Ul[1] += w * uj[3 * j + 1];
        Ul[2] += w * uj[3 * j + 2];
      }
    }
    const double arm[3] = {r_l * dirs[3 * l], r_l * dirs[3 * l + 1], r_l * dirs[3 * l + 2]};
    const double Ud[3] = {Up[0] + (Wp[1] * arm[2] - Wp[2] * arm[1]), Up[1] + (Wp[2] * arm[0] - Wp[0] * arm[2]),
                          Up[2] + (Wp[0] * arm[1] - Wp[1] * arm[0])};
    for (int k = 0; k < 3; ++k) {
      dF[m][k] = 2.0f * ((float)Ud[k] - Ul[k]);
      dmax = fmaxf(dmax, fabsf(dF[m][k]));
    }
    const double f[3] = {(double)dF[m][0] * dV, (double)dF[m][1] * dV, (double)dF[m][2] * dV};
    // the particle feels minus the force on the fluid
    for (int k = 0; k < 3; ++k) fsum[k] -= f[k];
    fsum[3] -= arm[1] * f[2] - arm[2] * f[1];
    fsum[4] -= arm[2] * f[0] - arm[0] * f[2];
    fsum[5] -= arm[0] * f[1] - arm[1] * f[0];
  }
  // Per wavefront: the six sums by a fixed butterfly that leaves sum k in
  // lanes 8k .. 8k+7 (each exchange step halves the values a lane carries),
  // and the largest |dF|.
  {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    double v4[4], v2[2];
    const bool h = lane & 32, g = lane & 16, o = lane & 8;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const double lo_v = fsum[i], hi_v = i < 2 ? fsum[4 + i] : 0.0;
      v4[i] = (h ? hi_v : lo_v) + __shfl_xor(h ? lo_v : hi_v, 32, 64);
    }
#pragma unroll
    for (int i = 0; i < 2; ++i) v2[i] = (g ? v4[2 + i] : v4[i]) + __shfl_xor(g ? v4[i] : v4[2 + i], 16, 64);
    double v1 = (o ? v2[1] : v2[0]) + __shfl_xor(o ? v2[0] : v2[1], 8, 64);
    v1 += __shfl_xor(v1, 4, 64);
    v1 += __shfl_xor(v1, 2, 64);
    v1 += __shfl_xor(v1, 1, 64);
    uint32_t mb = __float_as_uint(dmax);
#pragma unroll
    for (int sh = 32; sh > 0; sh >>= 1) mb = max(mb, (uint32_t)__shfl_xor((int)mb, sh, 64));
    if ((lane & 7) == 0 && (lane >> 3) < 6) red_f[wv][lane >> 3] = v1;
    if (lane == 0) red_m[wv] = mb;
  }
  __syncthreads();  // every marker has read uj; the partials are complete
  uint32_t mb = 0;
#pragma unroll
  for (int wv = 0; wv < kPassBlock / 64; ++wv) mb = max(mb, red_m[wv]);
  const int e = spread_exponent(__uint_as_float(mb), dVf);
  // the particle's force and torque: the wavefront partials in index order
  if (threadIdx.x < 6) {
    double t = 0.0;
#pragma unroll
    for (int wv = 0; wv < kPassBlock / 64; ++wv) t += red_f[wv][threadIdx.x];
    double* out = threadIdx.x < 3 ? F_ib + 3 * p + threadIdx.x : T_ib + 3 * p + (threadIdx.x - 3);
    *out = (first ? 0.0 : *out) + t;
  }
  for (uint32_t j = threadIdx.x; j < cnt; j += kPassBlock) {
    acc_xy[j] = 0ull;
    acc_z[j] = 0;
  }
  __syncthreads();
#pragma unroll
  for (int m = 0; m < MPT; ++m) {
    const int l = threadIdx.x + m * kPassBlock;
    if (l >= nmk) continue;
    // the weights again from the offsets (fewer registers held across the
    // barriers than keeping all twelve)
    const int bx = (int)(mk[m].base & 1023u), by = (int)((mk[m].base >> 10) & 1023u), bz = (int)(mk[m].base >> 20);
    float wx[4], wy[4], wz[4];
    peskin4(mk[m].t[0], wx);
    peskin4(mk[m].t[1], wy);
    peskin4(mk[m].t[2], wz);
    const uint32_t below = (1u << bx) - 1u;
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int jy = q & 3, jz = q >> 2;
      const int row = (by + jy) + side * (bz + jz);
      const uint2 rw = rbp[row];
      const uint32_t j0 = rw.y + __popc(rw.x & below);
      const float wyz = wy[jy] * wz[jz] * dVf;
#pragma unroll
      for (int jx = 0; jx < 4; ++jx) {
        const float w = wx[jx] * wyz;
        const uint32_t j = j0 + jx;
        const long long ax = __float2int_rn(ldexpf(dF[m][0] * w, e));
        const long long ay = __float2int_rn(ldexpf(dF[m][1] * w, e));
        atomicAdd(&acc_xy[j], (unsigned long long)(ay * 4294967296ll + ax));
        atomicAdd(&acc_z[j], __float2int_rn(ldexpf(dF[m][2] * w, e)));
      }
    }
  }
  __syncthreads();
  // Write back: nodes of this sphere alone in place (no other workgroup reads
  // or writes them; into the per-sphere copy until the last pass), shared
  // nodes into the exact accumulators.
  for (uint32_t j0 = 0; j0 < cnt; j0 += kWrite * kPassBlock) {
    uint32_t w[kWrite];
    float4 old[kWrite];
#pragma unroll
    for (int i = 0; i < kWrite; ++i) {
      const uint32_t j = j0 + threadIdx.x + i * kPassBlock;
      w[i] = j < cnt ? sl[j] : 0xFFFFFFFFu;
    }
#pragma unroll
    for (int i = 0; i < kWrite; ++i) {
      const uint32_t j = j0 + threadIdx.x + i * kPassBlock;
      old[i] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
      if (!first && !(w[i] & kSlotShared) && w[i] < s_cap) old[i] = pf_p ? pf_p[j] : fib[w[i]];
    }
#pragma unroll
    for (int i = 0; i < kWrite; ++i) {
      const uint32_t j = j0 + threadIdx.x + i * kPassBlock;
      if (j >= cnt) continue;
      if (!(w[i] & kSlotShared)) {
        if (w[i] >= s_cap) continue;
        int a3[3];
        unpack_sums(acc_xy[j], acc_z[j], a3);
        const float4 fn = make_float4(old[i].x + (float)ldexp((double)a3[0], -e),
                                      old[i].y + (float)ldexp((double)a3[1], -e),
                                      old[i].z + (float)ldexp((double)a3[2], -e), 0.0f);
        if (pf_p && !last)
          pf_p[j] = fn;
        else
          fib[w[i]] = fn;
      } else {
        const uint32_t q = w[i] & ~kSlotShared;
        if (q >= sh_cap) continue;
        int a3s[3];
        unpack_sums(acc_xy[j], acc_z[j], a3s);
        for (int k = 0; k < 3; ++k) {
          const int a = a3s[k];
          if (a)
            atomicAdd(sh_acc + (size_t)k * sh_cap + q,
                      (unsigned long long)((long long)a * (1ll << (kShUnitExp - e))));
        }
      }
    }
  }
}

// After a pass: the exact sums at shared nodes join the slot forces and the
// accumulators return to zero.
__global__ void __launch_bounds__(kBlock)
k_ibm_fold(const uint32_t* __restrict__ sh_count, uint32_t sh_cap, const uint32_t* __restrict__ sh_slot,
           unsigned long long* __restrict__ sh_acc, float4* __restrict__ fib, uint32_t s_cap) {
  const uint32_t n = min(*sh_count, sh_cap);
  for (uint32_t i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) {
    const uint32_t s = sh_slot[i];
    float add[3];
    for (int k = 0; k < 3; ++k) {
      unsigned long long* a = sh_acc + (size_t)k * sh_cap + i;
      const long long v = (long long)*a;
      add[k] = (float)((double)v * 0x1p-50);
      if (v) *a = 0ull;
    }
    if (s < s_cap && (add[0] != 0.0f || add[1] != 0.0f || add[2] != 0.0f)) {
      const float4 o = fib[s];
      fib[s] = make_float4(o.x + add[0], o.y + add[1], o.z + add[2], 0.0f);
    }
  }
}

// Shared-node table: node -> slot, in place.
__global__ void __launch_bounds__(kBlock)
k_ibm_shared_slots(const uint32_t* __restrict__ sh_count, uint32_t sh_cap, const uint32_t* __restrict__ bits,
                   const uint32_t* __restrict__ rank, uint32_t* __restrict__ sh_slot) {
  const uint32_t n = min(*sh_count, sh_cap);
  for (uint32_t i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) {
    uint32_t slot;
    sh_slot[i] = support_slot(bits, rank, sh_slot[i], slot) ? slot : 0xFFFFFFFFu;
  }
}

// ----------------------------------------------------------------- wall --
// Static pipe-wall markers (rings at every integer z, desired velocity 0),
// one thread per marker. A pass is split in launches so every marker
// interpolates the same velocity before any spread lands: interpolate and
// store dF = 2 (0 - U_l), spread dF delta dV into exact 64-bit fixed-point
// sums per slot (units 2^-50; a wall carries no spheres, so the shared-node
// accumulators are free for it), then fold the sums into the slot forces:
// the result does not depend on the order of the atomics.
__device__ __forceinline__ void wall_stencil(const double* __restrict__ xm, uint32_t l, int b[3], float w[3][4]) {
  for (int k = 0; k < 3; ++k) {
    const double X = xm[3 * l + k];
    b[k] = (int)floor(X) - 1;
    for (int j = 0; j < 4; ++j) w[k][j] = peskin((float)(X - (double)(b[k] + j)));
  }
}

__global__ void __launch_bounds__(kBlock)
k_ibm_wall_interp(const double* __restrict__ xm, uint32_t nm, Dims d, const uint32_t* __restrict__ bits,
                  const uint32_t* __restrict__ rank, const float4* __restrict__ us, const float4* __restrict__ fib,
                  uint32_t s_cap, float* __restrict__ dF) {
  const uint32_t l = blockIdx.x * kBlock + threadIdx.x;
  if (l >= nm) return;
  int b[3];
  float w[3][4];
  wall_stencil(xm, l, b, w);
  float U[3] = {0.0f, 0.0f, 0.0f};
  for (int jz = 0; jz < 4; ++jz)
    for (int jy = 0; jy < 4; ++jy) {
      const float wyz = w[1][jy] * w[2][jz];
      const int y = wrapi(b[1] + jy, d.ny), z = wrapi(b[2] + jz, d.nz);
      for (int jx = 0; jx < 4; ++jx) {
        uint32_t s;
        if (!support_slot(bits, rank, node_index(wrapi(b[0] + jx, d.nx), y, z, d.nx, d.ny), s) || s >= s_cap)
          continue;
        const float4 v = us[s];
        const float4 f = fib[s];
        const float h = 0.5f / v.w;
        const float wt = w[0][jx] * wyz;
        U[0] += wt * (v.x + f.x * h);
        U[1] += wt * (v.y + f.y * h);
        U[2] += wt * (v.z + f.z * h);
      }
    }
  for (int k = 0; k < 3; ++k) dF[3 * (size_t)l + k] = -2.0f * U[k];
}

__global__ void __launch_bounds__(kBlock)
k_ibm_wall_spread(const double* __restrict__ xm, uint32_t nm, float dV, Dims d, const uint32_t* __restrict__ bits,
                  const uint32_t* __restrict__ rank, unsigned long long* __restrict__ acc, uint32_t s_cap,
                  const float* __restrict__ dF) {
  const uint32_t l = blockIdx.x * kBlock + threadIdx.x;
  if (l >= nm) return;
  int b[3];
  float w[3][4];
  wall_stencil(xm, l, b, w);
  const float f[3] = {dF[3 * (size_t)l] * dV, dF[3 * (size_t)l + 1] * dV, dF[3 * (size_t)l + 2] * dV};
  for (int jz = 0; jz < 4; ++jz)
    for (int jy = 0; jy < 4; ++jy) {
      const float wyz = w[1][jy] * w[2][jz];
      const int y = wrapi(b[1] + jy, d.ny), z = wrapi(b[2] + jz, d.nz);
      for (int jx = 0; jx < 4; ++jx) {
        uint32_t s;
        if (!support_slot(bits, rank, node_index(wrapi(b[0] + jx, d.nx), y, z, d.nx, d.ny), s) || s >= s_cap)
          continue;
        const float wt = w[0][jx] * wyz;
        for (int k = 0; k < 3; ++k) {
          const long long v = llrint((double)(f[k] * wt) * 0x1p50);
          if (v) atomicAdd(acc + (size_t)k * s_cap + s, (unsigned long long)v);
        }
      }
    }
}

__global__ void __launch_bounds__(kBlock)
k_ibm_wall_fold(const uint32_t* __restrict__ count, unsigned long long* __restrict__ acc, float4* __restrict__ fib,
                uint32_t s_cap) {
  const uint32_t n = min(*count, s_cap);
  for (uint32_t s = blockIdx.x * kBlock + threadIdx.x; s < n; s += gridDim.x * kBlock) {
    float add[3];
    for (int k = 0; k < 3; ++k) {
      unsigned long long* a = acc + (size_t)k * s_cap + s;
      const long long v = (long long)*a;
      add[k] = (float)((double)v * 0x1p-50);
      if (v) *a = 0ull;
    }
    if (add[0] != 0.0f || add[1] != 0.0f || add[2] != 0.0f) {
      const float4 o = fib[s];
      fib[s] = make_float4(o.x + add[0], o.y + add[1], o.z + add[2], 0.0f);
    }
  }
}

// ---------------------------------------------------------------- kempe --
// Sum alpha u and sum alpha (x - X) x u per sphere; u from the support
// slots (u* + f_IB / (2 rho)) or, before the first step, a dense field.
//
// Only cells whose centre lies within r + sqrt(3)/2 of the centre have a
// fraction above zero; those deeper than sqrt(3)/2 inside the surface have
// fraction 1 from the centre distance alone, the rest (the surface cells)
// take the eight-corner fraction. Per round, one thread per box row counts
// the row's inner and surface cells (two intervals of the ball's x range),
// and the cells are listed in LDS, inner ones first, each group in box
// order. The list is then taken kKempeBatch cells per thread with
// consecutive lanes on consecutive cells: the slot loads of a row coalesce,
// and the wavefronts on surface cells evaluate the fraction with every lane
// busy. Rounds take as many rows as the list holds. Rows and cells are
// taken in a fixed order, so the sums are reproducible.
constexpr int kKempeBatch = 2;
constexpr int kKempeCells = 4096;  // listed cells per round
// u at K cells (a[k] > 0 only); a cell outside the support gets a[k] = 0.
template <bool DENSE, int K>
__device__ __forceinline__ void kempe_u(const uint32_t (&n)[K], double (&a)[K], float (&u)[K][3], const Dims& d,
                                        const uint32_t* __restrict__ bits, const uint32_t* __restrict__ rank,
                                        const float4* __restrict__ us, const float4* __restrict__ fib, uint32_t s_cap,
                                        const float* __restrict__ ufield) {
  if (DENSE) {
#pragma unroll
    for (int k = 0; k < K; ++k) {
      u[k][0] = u[k][1] = u[k][2] = 0.0f;
      if (!(a[k] > 0.0)) continue;
      u[k][0] = ufield[n[k]];
      u[k][1] = ufield[(size_t)d.N + n[k]];
      u[k][2] = ufield[2 * (size_t)d.N + n[k]];
    }
    return;
  }
  uint32_t wb[K], wr[K];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    wb[k] = wr[k] = 0u;
    if (!(a[k] > 0.0)) continue;
    wb[k] = bits[n[k] >> 5];
    wr[k] = rank[n[k] >> 5];
  }
  float4 v[K], f[K];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const uint32_t bit = n[k] & 31u;
    const uint32_t slot = wr[k] + __popc(wb[k] & ((1u << bit) - 1u));
    v[k] = make_float4(0.0f, 0.0f, 0.0f, 1.0f);
    f[k] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    if (!((wb[k] >> bit) & 1u) || slot >= s_cap) {
      a[k] = 0.0;
      continue;
    }
    v[k] = us[slot];
    f[k] = fib[slot];
  }
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const float h = 0.5f / v[k].w;
    u[k][0] = v[k].x + f[k].x * h;
    u[k][1] = v[k].y + f[k].y * h;
    u[k][2] = v[k].z + f[k].z * h;
  }
}

template <bool DENSE>
__global__ void __launch_bounds__(kBlock)
k_kempe(const double* __restrict__ X, const double* __restrict__ rad, Dims d, const uint32_t* __restrict__ bits,
        const uint32_t* __restrict__ rank, const float4* __restrict__ us, const float4* __restrict__ fib,
        uint32_t s_cap, const float* __restrict__ ufield, double* __restrict__ Iu, double* __restrict__ IL) {
  constexpr int K = kKempeBatch;
  __shared__ uint32_t cells[kKempeCells];  // box-local x | y << 8 | z << 16
  const int p = blockIdx.x;
  const double* Xp = X + 3 * p;
  const double r = rad[p];
  const Box b = make_box(Xp, r + 1.0);  // side <= 2 r + 4 < 256
  const double ri = r - 0.8661, ro = r + 0.8661;  // the fraction's own margins
  const double ri2 = ri > 0.0 ? ri * ri : -1.0, ro2 = ro * ro;
  const int rows = b.side[1] * b.side[2];
  double s[6] = {0, 0, 0, 0, 0, 0};
  int row0 = 0;
  while (row0 < rows) {  // uniform: every thread sees the same row0
    // this thread's row: the ball's x range [xa, xb] and inside it the inner
    // cells [ia, ib] (both box-local; empty ranges have b < a)
    const int row = row0 + (int)threadIdx.x;
    int xa = 0, xb = -1, ia = 0, ib = -1;
    if (row < rows) {
      const int y = wrap1(b.lo[1] + row % b.side[1], d.ny), z = wrap1(b.lo[2] + row / b.side[1], d.nz);
      const double dy = min_image((double)y - Xp[1], d.ny), dz = min_image((double)z - Xp[2], d.nz);
      if (dy * dy + dz * dz < ro2) {
        // widened by one around the root; the exact test below decides
        const double hx = sqrt(fmax(ro2 - (dy * dy + dz * dz), 0.0));
        const int lo = max(0, (int)floor(Xp[0] - hx) - 1 - b.lo[0]);
        const int hi = min(b.side[0] - 1, (int)ceil(Xp[0] + hx) + 1 - b.lo[0]);
        xa = hi + 1;
        for (int lx = lo; lx <= hi; ++lx) {
          const int x = wrap1(b.lo[0] + lx, d.nx);
          const double d2 = dist2(min_image((double)x - Xp[0], d.nx), dy, dz);
          if (d2 < ro2) {
            xa = min(xa, lx);
            xb = lx;
          }
          if (d2 < ri2) {
            if (ib < ia) ia = lx;
            ib = lx;
          }
        }
      }
    }
    const uint32_t ni = ib >= ia ? (uint32_t)(ib - ia + 1) : 0u;
    const uint32_t nall = xb >= xa ? (uint32_t)(xb - xa + 1) : 0u;
    // the rows of this round: as many as the list holds (at least one)
    uint32_t total;
    const uint32_t before = block_exclusive_scan<kBlock>(row < rows ? nall : 0u, &total);
    const bool take = row < rows && (before + nall <= (uint32_t)kKempeCells || threadIdx.x == 0);
    const uint32_t ti = take ? ni : 0u, ts = take ? nall - ni : 0u;
    uint32_t n_in, n_surf;
    const uint32_t oi = block_exclusive_scan<kBlock>(ti, &n_in);
    const uint32_t os = block_exclusive_scan<kBlock>(ts, &n_surf);
    uint32_t taken;
    (void)block_exclusive_scan<kBlock>(take ? 1u : 0u, &taken);
    if (take) {
      const uint32_t yz = (uint32_t)(row % b.side[1]) << 8 | (uint32_t)(row / b.side[1]) << 16;
      for (uint32_t k = 0; k < ni; ++k) cells[min(oi + k, (uint32_t)kKempeCells - 1u)] = (uint32_t)(ia + (int)k) | yz;
      uint32_t o = n_in + os;
      for (int lx = xa; lx <= xb; ++lx)
        if (lx < ia || lx > ib) cells[min(o++, (uint32_t)kKempeCells - 1u)] = (uint32_t)lx | yz;
    }
    __syncthreads();
    const uint32_t n_cells = min(n_in + n_surf, (uint32_t)kKempeCells);
    for (uint32_t f0 = 0; f0 < n_cells; f0 += K * kBlock) {
      uint32_t n[K];
      double a[K], dx[K], dy[K], dz[K];
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const uint32_t f = f0 + (uint32_t)(k * kBlock) + threadIdx.x;
        a[k] = dx[k] = dy[k] = dz[k] = 0.0;
        n[k] = 0u;
        if (f >= n_cells) continue;
        const uint32_t e = cells[f];
        const int x = wrap1(b.lo[0] + (int)(e & 0xFFu), d.nx), y = wrap1(b.lo[1] + (int)((e >> 8) & 0xFFu), d.ny),
                  z = wrap1(b.lo[2] + (int)(e >> 16), d.nz);
        dx[k] = min_image((double)x - Xp[0], d.nx);
        dy[k] = min_image((double)y - Xp[1], d.ny);
        dz[k] = min_image((double)z - Xp[2], d.nz);
        n[k] = node_index(x, y, z, d.nx, d.ny);
        a[k] = f < n_in ? 1.0 : kempe_alpha(dx[k], dy[k], dz[k], r);
      }
      float u[K][3];
      kempe_u<DENSE, K>(n, a, u, d, bits, rank, us, fib, s_cap, ufield);
#pragma unroll
      for (int k = 0; k < K; ++k) {
        if (!(a[k] > 0.0)) continue;
        const double ux = (double)u[k][0], uy = (double)u[k][1], uz = (double)u[k][2];
        s[0] += a[k] * ux;
        s[1] += a[k] * uy;
        s[2] += a[k] * uz;
        s[3] += a[k] * (dy[k] * uz - dz[k] * uy);
        s[4] += a[k] * (dz[k] * ux - dx[k] * uz);
        s[5] += a[k] * (dx[k] * uy - dy[k] * ux);
      }
    }
    __syncthreads();  // the list is refilled by the next round
    row0 += (int)taken;
  }
  block_sum_n<kBlock, 6>(s);
  if (threadIdx.x == 0)
    for (int k = 0; k < 3; ++k) {
      Iu[3 * p + k] = s[k];
      IL[3 * p + k] = s[3 + k];
    }
}

size_t pass_lds_bytes(const Ctx& c) {
  const size_t rows = (size_t)c.ibm.side * c.ibm.side;
  return rows * 8 + (size_t)c.ibm.fcap * 16;
}

}  // namespace

size_t ibm_pass_lds_bytes(const Ctx& c) { return pass_lds_bytes(c); }

size_t bits_compact_scratch_words(uint32_t nwords) { return (nwords + kScanWords - 1) / kScanWords + 2; }

hipError_t launch_bits_compact(hipStream_t st, const uint32_t* bits, uint32_t nwords, uint32_t* rank,
                               uint32_t* block_sums, uint32_t* count, uint32_t* list, uint32_t cap, uint32_t* err) {
  const uint32_t nblk = (nwords + kScanWords - 1) / kScanWords;
  hipLaunchKernelGGL(k_scan_block, dim3(nblk), dim3(kBlock), 0, st, bits, nwords, rank, block_sums);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(1024), 0, st, block_sums, nblk, count);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_scan_add, dim3(nblk), dim3(kBlock), 0, st, bits, nwords, rank, block_sums, list, cap, err);
  return hipGetLastError();
}

// Clears the support and shared bitmasks (16-byte stores; the runtime's
// fill took about 40 us for each 16.8 MB mask at 512^3). With a static wall
// the support starts as the wall's support instead.
__global__ void __launch_bounds__(kBlock)
k_masks_reset(uint32_t* __restrict__ bits, uint32_t* __restrict__ shared, const uint32_t* __restrict__ wall,
              uint32_t words) {
  const uint32_t n4 = words / 4u;
  for (uint32_t i = blockIdx.x * kBlock + threadIdx.x; i < n4; i += gridDim.x * kBlock) {
    ((uint4*)bits)[i] = wall ? ((const uint4*)wall)[i] : make_uint4(0u, 0u, 0u, 0u);
    ((uint4*)shared)[i] = make_uint4(0u, 0u, 0u, 0u);
  }
  if (blockIdx.x == 0 && threadIdx.x < words % 4u) {
    const uint32_t w = n4 * 4u + threadIdx.x;
    bits[w] = wall ? wall[w] : 0u;
    shared[w] = 0u;
  }
}

hipError_t launch_ibm_support_build(Ctx& c, int buf, const double* X) {
  const uint32_t words = mask_words(c.dims.N);
  IbmBufs& m = c.ibm;
  // the static wall support, if any, is part of every support set
  const uint32_t blocks = std::min<uint32_t>(std::max<uint32_t>((words / 4u + kBlock - 1) / kBlock, 1u), 2048u);
  hipLaunchKernelGGL(k_masks_reset, dim3(blocks), dim3(kBlock), 0, c.stream, m.bits[buf], m.shared,
                     m.n_wall ? (const uint32_t*)m.wsup : nullptr, words);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (c.np > 0) {
    const size_t lds = (size_t)m.side * m.side * 8;
    hipLaunchKernelGGL(k_ibm_mark, dim3(c.np), dim3(kBlock), lds, c.stream, X, c.P.r, m.dirs, m.n_markers, m.r_l,
                       m.R_b, m.side, c.dims, m.bits[buf], m.shared, m.rowbits, m.fcount, m.fcap, c.err);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  if ((e = launch_bits_compact(c.stream, m.bits[buf], words, m.rank[buf], m.block_sums, m.count[buf], m.list,
                               m.s_cap, c.err)) != hipSuccess)
    return e;
  if (c.np > 0) {
    // shared nodes: their rank, then their slots
    if ((e = launch_bits_compact(c.stream, m.shared, words, m.sh_rank, m.block_sums, m.sh_count, m.sh_slot,
                                 m.sh_cap, c.err)) != hipSuccess)
      return e;
    hipLaunchKernelGGL(k_ibm_shared_slots, dim3(1024), dim3(kBlock), 0, c.stream, m.sh_count, m.sh_cap,
                       m.bits[buf], m.rank[buf], m.sh_slot);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_ibm_slots, dim3(c.np), dim3(kBlock), 0, c.stream, X, m.R_b, m.side, c.dims, m.bits[buf],
                       m.rank[buf], m.shared, m.sh_rank, m.rowbits, m.fcount, m.fcap, m.fslot);
    e = hipGetLastError();
  }
  return e;
}

hipError_t launch_ibm_prepass(const Ctx& c, const void* A) {
  const IbmBufs& m = c.ibm;
  const dim3 grid((m.s_cap + 255) / 256);
  if (c.cfg.store == LBM_STORE_F32)
    hipLaunchKernelGGL(k_ibm_prepass<0>, grid, dim3(256), 0, c.stream, (const float*)A, c.dims, c.body_force,
                       ibm_body_force_mask(c), m.list, m.count[m.cur], m.s_cap, m.us, m.fib[m.cur]);
  else
    hipLaunchKernelGGL(k_ibm_prepass<1>, grid, dim3(256), 0, c.stream, (const _Float16*)A, c.dims, c.body_force,
                       ibm_body_force_mask(c), m.list, m.count[m.cur], m.s_cap, m.us, m.fib[m.cur]);
  return hipGetLastError();
}

hipError_t launch_ibm_forcing_pass(const Ctx& c, const double* X, const double* U, const double* Om) {
  const IbmBufs& m = c.ibm;
  if (c.np <= 0 && m.n_wall == 0) return hipSuccess;
  const size_t lds = pass_lds_bytes(c);
  const int passes = 1 + c.cfg.ibm_iters;
  const dim3 wgrid((m.n_wall + kBlock - 1) / kBlock);
  // Per-sphere copies between passes, unless a wall's markers also act on
  // the slot forces between the sphere passes.
  float4* const pu = m.n_wall ? nullptr : m.pu;
  float4* const pf = m.n_wall ? nullptr : m.pf;
  for (int k = 0; k < passes; ++k) {
    if (m.n_wall) {
      hipLaunchKernelGGL(k_ibm_wall_interp, wgrid, dim3(kBlock), 0, c.stream, m.wmark, m.n_wall, c.dims,
                         m.bits[m.cur], m.rank[m.cur], m.us, m.fib[m.cur], m.s_cap, m.wdF);
      hipError_t e = hipGetLastError();
      if (e != hipSuccess) return e;
    }
    if (c.np > 0) {
      if (m.n_markers <= kPassBlock)
        hipLaunchKernelGGL(k_ibm_pass<1>, dim3(c.np), dim3(kPassBlock), lds, c.stream, X, U, Om, m.dirs,
                           m.n_markers, m.r_l, m.dV, m.R_b, m.side, c.dims, m.rowbits, m.fcount, m.fcap, m.fslot,
                           m.sh_slot, m.sh_cap, m.us, m.fib[m.cur], m.s_cap, m.sh_acc, c.P.F_ib, c.P.T_ib, pu, pf,
                           k == 0 ? 1 : 0, k == passes - 1 ? 1 : 0);
      else
        hipLaunchKernelGGL(k_ibm_pass<2>, dim3(c.np), dim3(kPassBlock), lds, c.stream, X, U, Om, m.dirs,
                           m.n_markers, m.r_l, m.dV, m.R_b, m.side, c.dims, m.rowbits, m.fcount, m.fcap, m.fslot,
                           m.sh_slot, m.sh_cap, m.us, m.fib[m.cur], m.s_cap, m.sh_acc, c.P.F_ib, c.P.T_ib, pu, pf,
                           k == 0 ? 1 : 0, k == passes - 1 ? 1 : 0);
      hipError_t e = hipGetLastError();
      if (e != hipSuccess) return e;
      hipLaunchKernelGGL(k_ibm_fold, dim3(1024), dim3(kBlock), 0, c.stream, m.sh_count, m.sh_cap, m.sh_slot,
                         m.sh_acc, m.fib[m.cur], m.s_cap);
      if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    hipError_t e = hipSuccess;
    if (m.n_wall) {
      // the wall accumulators are indexed by slot: the shared-node table has
      // room for every slot (sh_cap = s_cap)
      hipLaunchKernelGGL(k_ibm_wall_spread, wgrid, dim3(kBlock), 0, c.stream, m.wmark, m.n_wall, (float)m.wdV, c.dims,
                         m.bits[m.cur], m.rank[m.cur], m.sh_acc, m.sh_cap, m.wdF);
      if ((e = hipGetLastError()) != hipSuccess) return e;
      hipLaunchKernelGGL(k_ibm_wall_fold, dim3(1024), dim3(kBlock), 0, c.stream, m.count[m.cur], m.sh_acc,
                         m.fib[m.cur], m.s_cap);
      if ((e = hipGetLastError()) != hipSuccess) return e;
    }
  }
  return hipSuccess;
}

hipError_t launch_ibm_kempe(const Ctx& c, const double* X, double* Iu, double* IL) {
  if (c.np <= 0) return hipSuccess;
  const IbmBufs& m = c.ibm;
  hipLaunchKernelGGL(k_kempe<false>, dim3(c.np), dim3(kBlock), 0, c.stream, X, c.P.r, c.dims, m.bits[m.cur],
                     m.rank[m.cur], m.us, m.fib[m.cur], m.s_cap, nullptr, Iu, IL);
  return hipGetLastError();
}

hipError_t launch_kempe_dense(const Ctx& c, const float* u, const double* X, double* Iu, double* IL) {
  if (c.np <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_kempe<true>, dim3(c.np), dim3(kBlock), 0, c.stream, X, c.P.r, c.dims, nullptr, nullptr,
                     nullptr, nullptr, c.ibm.s_cap, u, Iu, IL);
  return hipGetLastError();
}

}  // namespace lbm
