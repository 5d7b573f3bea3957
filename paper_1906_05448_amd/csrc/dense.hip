// dense.hip - the lattice-wide kernels: fused pull-stream + MRT collision,
// equilibrium initialisation and macroscopic-field extraction.
//
// Memory layout: structure of arrays, population i of node n at
// f[i * S + n], n = x + nx * (y + ny * z), with the array stride S the node
// count N plus a 1 KB pad (Dims::S). The pull form
//   f_i(x, t+1) = f~_i(x - c_i, t)
// reads each of the 19 arrays once, shifted by c_i, and writes each once,
// so one node update moves 19 * 2 * sizeof(store) bytes of HBM: 152 B in
// FP32, 76 B with FP16 shifted storage. Reads of a row shifted by one in x
// straddle cache lines shared with the neighbouring tile; the XCD-aware tile
// order keeps that neighbour in the same L2. The output is written with
// non-temporal stores (measured 3% faster at 512^3; non-temporal loads were
// slower).
#include "internal.hpp"

namespace lbm {

namespace {

// Immersed-boundary force lookup: node n is in the support iff its bit is
// set; its slot is the word rank plus the set bits below it.
struct IbView {
  const uint32_t* bits;
  const uint32_t* rank;
  const float4* fib;  // [s_cap] (x, y, z, unused)
  uint32_t s_cap;
  const uint32_t* nobody;  // nodes without body force (outside a pipe), or null
};

// Bounce-back patches of the current step for the row kernels (cnt null:
// none): per row of 512 nodes, cnt[row] records of a node x, an opposite
// direction and the stored value's bits, each replacing the staged value
// that node x pulls for that direction (its ghost slot).
struct PatchView {
  const uint32_t* cnt;
  const void* rec;  // FP16: one word per record, FP32: two (the link pass's layout)
};
static_assert(kPatchCap <= 256, "one patch record per thread of the row kernels");

// Body force at node n: none where the mask says so.
__device__ __forceinline__ float3 body_force_at(const IbView& v, uint32_t n, float3 F0) {
  if (v.nobody && ((v.nobody[n >> 5] >> (n & 31u)) & 1u)) return make_float3(0.0f, 0.0f, 0.0f);
  return F0;
}

__device__ __forceinline__ void add_ib_force(const IbView& v, uint32_t n, float3& F) {
  const uint32_t w = v.bits[n >> 5];
  const uint32_t b = n & 31u;
  if ((w >> b) & 1u) {
    const uint32_t s = v.rank[n >> 5] + __popc(w & ((1u << b) - 1u));
    if (s >= v.s_cap) return;  // capacity overflow is latched by the build
    const float4 f = v.fib[s];
    F.x += f.x;
    F.y += f.y;
    F.z += f.z;
  }
}

// MODE 0: uniform force. MODE 2: plus the immersed-boundary force at the
// support nodes. TW: tile width, 128 (128 x 2 tiles) or 64 (64 x 4) where
// that fills the rows better.
template <int STORE, int MODE, int TW>
__global__ void __launch_bounds__(256)
k_stream_collide(const typename Pop<STORE>::T* __restrict__ A, typename Pop<STORE>::T* __restrict__ B,
                 Dims d, Tiles tg, MrtRates r, float3 F0, IbView ib, uint32_t* __restrict__ err) {
  using P = Pop<STORE>;
  const Tile t = tile_of<TW>(d, tg);
  if (!t.live) return;
  // One wavefront covers 64 nodes of one row: y is uniform across it. With FP32
  // storage the kernel keeps the row offsets in scalar registers (measured
  // 1.3% faster at 512^3); with FP16 the per-lane offsets measured 1.7%
  // faster, so that form is kept there.
  const int x = t.x, z = t.z;
  const int y = STORE == 0 ? __builtin_amdgcn_readfirstlane(t.y) : t.y;
  float3 F = F0;
  if (MODE == 2) {
    const uint32_t n0 = ((uint32_t)z * (uint32_t)d.ny + (uint32_t)y) * (uint32_t)d.nx + (uint32_t)x;
    F = body_force_at(ib, n0, F0);
    add_ib_force(ib, n0, F);
  }
  const int nx = d.nx, ny = d.ny, nz = d.nz;
  const uint32_t S = d.S;  // population array stride
  const int xm = x == 0 ? nx - 1 : x - 1, xp = x == nx - 1 ? 0 : x + 1;
  const int ym = y == 0 ? ny - 1 : y - 1, yp = y == ny - 1 ? 0 : y + 1;
  const int zm = z == 0 ? nz - 1 : z - 1, zp = z == nz - 1 ? 0 : z + 1;
  auto row = [&](int yy, int zz) -> uint32_t { return ((uint32_t)zz * (uint32_t)ny + (uint32_t)yy) * (uint32_t)nx; };
  const uint32_t r00 = row(y, z), rm0 = row(ym, z), rp0 = row(yp, z);
  const uint32_t r0m = row(y, zm), r0p = row(y, zp);
  const uint32_t rmm = row(ym, zm), rmp = row(ym, zp), rpp = row(yp, zp), rpm = row(yp, zm);
  // Source row (y - c_iy, z - c_iz) of direction i; the source column is
  // x - c_ix.
  const uint32_t srow[kQ] = {r00, r00, rm0, r0m, rm0, rp0, r0m, r0p, rmm, rmp,
                             r00, rp0, r0p, rp0, rm0, r0p, r0m, rpp, rpm};

  using T = typename P::T;
  const uint32_t ox = (uint32_t)x * (uint32_t)sizeof(T), oxm = (uint32_t)xm * (uint32_t)sizeof(T),
                 oxp = (uint32_t)xp * (uint32_t)sizeof(T);
  float g[kQ];
#pragma unroll
  for (int i = 0; i < kQ; ++i) {
    const uint32_t o = cx_of(i) > 0 ? oxm : (cx_of(i) < 0 ? oxp : ox);
    if (STORE == 0) {
      // uniform row base (scalar) plus one of three column offsets
      g[i] = P::load((const T*)((const char*)(A + (size_t)i * S + srow[i]) + o));
    } else {
      // direction base plus one 32-bit byte offset per lane (N * sizeof(T)
      // <= 4 GiB is checked at init)
      const uint32_t src = srow[i] + (uint32_t)(cx_of(i) > 0 ? xm : (cx_of(i) < 0 ? xp : x));
      g[i] = P::load((const T*)((const char*)(A + (size_t)i * S) + src * (uint32_t)sizeof(T)));
    }
  }

  float rho, ux, uy, uz;
  mrt_collide(g, F.x, F.y, F.z, r, rho, ux, uy, uz);

  const uint32_t noff = (r00 + (uint32_t)x) * (uint32_t)sizeof(T);
#pragma unroll
  for (int i = 0; i < kQ; ++i) {
    if (STORE == 0)
      P::store_stream((T*)((char*)(B + (size_t)i * S + r00) + ox), g[i]);
    else
      P::store_stream((T*)((char*)(B + (size_t)i * S) + noff), g[i]);
  }

  const bool bad = !(rho > 0.0f) || !(ux * ux + uy * uy + uz * uz < 0.1225f);
  if (bad) atomicOr(err, kErrUnstable);
}

// FP16 storage with rows staged through LDS (nx even). A wavefront owns a
// 128-node row segment. It reads each population's source segment as aligned
// dwords (two nodes per lane: the access width the memory system serves
// best; 16-bit accesses measured slower) plus the node beyond each end, into
// its own LDS rows; each lane then takes its node's 19 shifted values from
// LDS as halves (any 2-byte offset), in two rounds of 64 nodes, and collides
// them exactly as the one-node kernel does. The results return through the
// same LDS rows and leave as dwords. Round 1 (nodes 64..127) reads one slot
// that round 0 writes: node 63's, for the directions with c_x = +1; those
// five results wait in a small tail area until round 1 has read.
constexpr int kSegW = 128;               // nodes per wavefront segment
constexpr int kSegRow = (kSegW + 4) / 2; // dwords per population row: 2 halves before, 2 after

__device__ __forceinline__ float half_to_g(uint16_t h) {
  return static_cast<float>(__builtin_bit_cast(_Float16, h)) * (1.0f / kHalfScale);
}
__device__ __forceinline__ uint16_t g_to_half(float g) {
  return __builtin_bit_cast(uint16_t, static_cast<_Float16>(g * kHalfScale));
}

template <int MODE>
__global__ void __launch_bounds__(256)
k_stream_collide_seg(const _Float16* __restrict__ A, _Float16* __restrict__ B, Dims d, MrtRates r, float3 F0,
                     IbView ib, uint32_t* __restrict__ err) {
  __shared__ uint32_t seg_all[4][kQ][kSegRow];
  __shared__ uint16_t tail_all[4][kQ];
  const uint32_t b = blockIdx.x;
  const uint32_t logical = (b & 7u) * d.per_xcd2 + (b >> 3);
  if (logical >= d.ntiles2) return;
  const uint32_t rest = fast_div(d.div_gx2, logical);
  const uint32_t bx = logical - rest * d.gx2;
  const uint32_t bz = fast_div(d.div_gy2, rest);
  const uint32_t by = rest - bz * d.gy2;
  const uint32_t lane = threadIdx.x & 63u;
  const int wv = (int)(threadIdx.x >> 6);
  const int y = __builtin_amdgcn_readfirstlane((int)(by * 4u) + wv);
  const int z = (int)bz;
  if (y >= d.ny) return;  // the whole wavefront
  uint32_t(*seg)[kSegRow] = seg_all[wv];
  uint16_t* tail = tail_all[wv];
  const int nx = d.nx, ny = d.ny, nz = d.nz;
  const uint32_t S = d.S;  // population array stride
  const int x0 = (int)bx * kSegW;
  const int w = min(kSegW, nx - x0);  // nodes in the segment, even
  auto row = [&](int yy, int zz) -> uint32_t { return ((uint32_t)zz * (uint32_t)ny + (uint32_t)yy) * (uint32_t)nx; };
  const int ym = y == 0 ? ny - 1 : y - 1, yp = y == ny - 1 ? 0 : y + 1;
  const int zm = z == 0 ? nz - 1 : z - 1, zp = z == nz - 1 ? 0 : z + 1;
  const uint32_t r00 = row(y, z), rm0 = row(ym, z), rp0 = row(yp, z);
  const uint32_t r0m = row(y, zm), r0p = row(y, zp);
  const uint32_t rmm = row(ym, zm), rmp = row(ym, zp), rpp = row(yp, zp), rpm = row(yp, zm);
  // source row (y - c_iy, z - c_iz) of direction i
  const uint32_t srow[kQ] = {r00, r00, rm0, r0m, rm0, rp0, r0m, r0p, rmm, rmp,
                             r00, rp0, r0p, rp0, rm0, r0p, r0m, rpp, rpm};
  // the node left of the segment and the one right of it (periodic)
  const uint32_t xl = (uint32_t)(x0 == 0 ? nx - 1 : x0 - 1);
  const uint32_t xr = (uint32_t)(x0 + w >= nx ? 0 : x0 + w);
  const bool pair_live = 2 * (int)lane < w;

  // stage: every load of the segment issued before the first LDS write
  uint32_t v[kQ];
  uint16_t e[kQ];
#pragma unroll
  for (int i = 0; i < kQ; ++i) {
    const _Float16* rowp = A + (size_t)i * S + srow[i];
    v[i] = pair_live ? __builtin_nontemporal_load((const uint32_t*)(rowp + x0 + 2 * (int)lane)) : 0u;
    // edge node: a vector load at a uniform address (scalar loads of the
    // same nodes measured 7.5% extra HBM reads: their lines are not served
    // from the copy the neighbouring segment's vector loads bring into L2)
    e[i] = cx_of(i) > 0 ? *(const uint16_t*)(rowp + xl) : (cx_of(i) < 0 ? *(const uint16_t*)(rowp + xr) : (uint16_t)0);
  }
#pragma unroll
  for (int i = 0; i < kQ; ++i) {
    uint16_t* h = (uint16_t*)seg[i];
    seg[i][1 + lane] = v[i];  // halves 2 + 2 lane, 3 + 2 lane
    if (lane == 0 && cx_of(i) > 0) h[1] = e[i];       // x0 - 1
    if (lane == 0 && cx_of(i) < 0) h[2 + w] = e[i];   // x0 + w
  }
  __builtin_amdgcn_wave_barrier();

  bool bad = false;
  // one round at a time (unrolled, the rounds' values would all be live)
#pragma unroll 1
  for (int rnd = 0; rnd < 2; ++rnd) {
    const int j = (int)lane + 64 * rnd;
    const bool live = j < w;
    const uint32_t n = r00 + (uint32_t)(x0 + j);
    float3 F = F0;
    if (MODE == 2 && live) {
      F = body_force_at(ib, n, F0);
      add_ib_force(ib, n, F);
    }
    float g[kQ];
#pragma unroll
    for (int i = 0; i < kQ; ++i) g[i] = half_to_g(((const uint16_t*)seg[i])[2 + j - cx_of(i)]);
    float rho, ux, uy, uz;
    mrt_collide(g, F.x, F.y, F.z, r, rho, ux, uy, uz);
    bad = bad || (live && (!(rho > 0.0f) || !(ux * ux + uy * uy + uz * uz < 0.1225f)));
    // every lane has read this round's inputs (same wavefront, in order)
#pragma unroll
    for (int i = 0; i < kQ; ++i) {
      uint16_t* h = (uint16_t*)seg[i];
      if (rnd == 0 && cx_of(i) > 0 && lane == 63u)
        tail[i] = g_to_half(g[i]);
      else
        h[2 + j] = g_to_half(g[i]);
    }
  }
  if (lane == 63u) {
#pragma unroll
    for (int i = 0; i < kQ; ++i)
      if (cx_of(i) > 0) ((uint16_t*)seg[i])[2 + 63] = tail[i];
  }
  __builtin_amdgcn_wave_barrier();
  if (pair_live) {
    const uint32_t off = (r00 + (uint32_t)(x0 + 2 * (int)lane)) * 2u;
#pragma unroll
    for (int i = 0; i < kQ; ++i)
      __builtin_nontemporal_store(seg[i][1 + lane], (uint32_t*)((char*)(B + (size_t)i * S) + off));
  }
  if (bad) atomicOr(err, kErrUnstable);
}

// The same update with a workgroup holding one whole row of 512 nodes: its
// four wavefronts take consecutive 128-node segments, and each hands its
// first and last node to its neighbours through LDS (periodic within the
// workgroup), so no segment end is loaded from memory. Consecutive
// workgroups of an XCD take consecutive rows, which share their source rows
// in L2. 1.926 -> 1.82-1.86 ms at 512^3 (5.5-5.6 TB/s).
template <int MODE>
__global__ void __launch_bounds__(256)
k_stream_collide_row(const _Float16* __restrict__ A, _Float16* __restrict__ B, Dims d, MrtRates r, float3 F0,
                     IbView ib, PatchView pv, uint32_t* __restrict__ err) {
  __shared__ uint32_t seg_all[4][kQ][kSegRow];
  __shared__ uint16_t tail_all[4][kQ];
  const uint32_t b = blockIdx.x;
  const uint32_t rowi = (b & 7u) * d.per_xcdr + (b >> 3);  // nx = 512: one workgroup per row
  if (rowi >= d.ntilesr) return;  // the whole workgroup
  const uint32_t bz = fast_div(d.div_ny, rowi);
  const uint32_t lane = threadIdx.x & 63u;
  const int wv = (int)(threadIdx.x >> 6);
  const int y = (int)(rowi - bz * (uint32_t)d.ny);
  const int z = (int)bz;
  uint32_t(*seg)[kSegRow] = seg_all[wv];
  uint16_t* tail = tail_all[wv];
  const int nx = d.nx, ny = d.ny, nz = d.nz;
  const uint32_t S = d.S;  // population array stride
  const int x0 = wv * kSegW;
  constexpr int w = kSegW;
  // the wavefronts of the left and right segments (periodic within the row)
  const int wl = (wv + 3) & 3, wr = (wv + 1) & 3;
  auto row = [&](int yy, int zz) -> uint32_t { return ((uint32_t)zz * (uint32_t)ny + (uint32_t)yy) * (uint32_t)nx; };
  const int ym = y == 0 ? ny - 1 : y - 1, yp = y == ny - 1 ? 0 : y + 1;
  const int zm = z == 0 ? nz - 1 : z - 1, zp = z == nz - 1 ? 0 : z + 1;
  const uint32_t r00 = row(y, z), rm0 = row(ym, z), rp0 = row(yp, z);
  const uint32_t r0m = row(y, zm), r0p = row(y, zp);
  const uint32_t rmm = row(ym, zm), rmp = row(ym, zp), rpp = row(yp, zp), rpm = row(yp, zm);
  // source row (y - c_iy, z - c_iz) of direction i
  const uint32_t srow[kQ] = {r00, r00, rm0, r0m, rm0, rp0, r0m, r0p, rmm, rmp,
                             r00, rp0, r0p, rp0, rm0, r0p, r0m, rpp, rpm};
  constexpr bool pair_live = true;

  // stage: every load of the segment issued before the first LDS write;
  // this thread's patch record (at most one: kPatchCap <= 256) with them
  uint32_t v[kQ];
#pragma unroll
  for (int i = 0; i < kQ; ++i)
    v[i] = __builtin_nontemporal_load((const uint32_t*)(A + (size_t)i * S + srow[i] + x0 + 2 * (int)lane));
  const uint32_t np = pv.cnt ? min(pv.cnt[rowi], kPatchCap) : 0u;
  uint32_t pr = 0u;
  if (threadIdx.x < np) pr = ((const uint32_t*)pv.rec)[(size_t)rowi * kPatchCap + threadIdx.x];
#pragma unroll
  for (int i = 0; i < kQ; ++i) {
    seg[i][1 + lane] = v[i];  // halves 2 + 2 lane, 3 + 2 lane
    // node x0 + 127 is the right neighbour's x0 - 1; node x0 the left
    // neighbour's x0 + w
    if (cx_of(i) > 0 && lane == 63u) ((uint16_t*)seg_all[wr][i])[1] = (uint16_t)(v[i] >> 16);
    if (cx_of(i) < 0 && lane == 0u) ((uint16_t*)seg_all[wl][i])[2 + w] = (uint16_t)(v[i] & 0xFFFFu);
  }
  __syncthreads();  // the neighbours' end nodes are in place
  if (np) {  // the same for the whole workgroup
    // the slot node x pulls direction i from: half 2 + (x mod 128) - c_ix of
    // wavefront x / 128's staged row i
    if (threadIdx.x < np) {
      const uint32_t x = pr & 511u, i = (pr >> 9) & 31u;
      ((uint16_t*)seg_all[x >> 7][i])[2 + (int)(x & 127u) - cx_of((int)i)] = (uint16_t)(pr >> 16);
    }
    __syncthreads();
  }

  bool bad = false;
  // one round at a time (unrolled, the rounds' values would all be live)
#pragma unroll 1
  for (int rnd = 0; rnd < 2; ++rnd) {
    const int j = (int)lane + 64 * rnd;
    const bool live = j < w;
    const uint32_t n = r00 + (uint32_t)(x0 + j);
    float3 F = F0;
    if (MODE == 2 && live) {
      F = body_force_at(ib, n, F0);
      add_ib_force(ib, n, F);
    }
    float g[kQ];
#pragma unroll
    for (int i = 0; i < kQ; ++i) g[i] = half_to_g(((const uint16_t*)seg[i])[2 + j - cx_of(i)]);
    float rho, ux, uy, uz;
    mrt_collide(g, F.x, F.y, F.z, r, rho, ux, uy, uz);
    bad = bad || (live && (!(rho > 0.0f) || !(ux * ux + uy * uy + uz * uz < 0.1225f)));
    // every lane has read this round's inputs (same wavefront, in order)
#pragma unroll
    for (int i = 0; i < kQ; ++i) {
      uint16_t* h = (uint16_t*)seg[i];
      if (rnd == 0 && cx_of(i) > 0 && lane == 63u)
        tail[i] = g_to_half(g[i]);
      else
        h[2 + j] = g_to_half(g[i]);
    }
  }
  if (lane == 63u) {
#pragma unroll
    for (int i = 0; i < kQ; ++i)
      if (cx_of(i) > 0) ((uint16_t*)seg[i])[2 + 63] = tail[i];
  }
  __builtin_amdgcn_wave_barrier();
  if (pair_live) {
    const uint32_t off = (r00 + (uint32_t)(x0 + 2 * (int)lane)) * 2u;
#pragma unroll
    for (int i = 0; i < kQ; ++i)
      __builtin_nontemporal_store(seg[i][1 + lane], (uint32_t*)((char*)(B + (size_t)i * S) + off));
  }
  if (bad) atomicOr(err, kErrUnstable);
}

// FP32 storage, nx a multiple of 512: a 512-thread workgroup holds 512 nodes
// of one row, one node per lane. Each wavefront stages its 64-node source
// segment of every population with aligned loads and passes its end nodes to
// its neighbours through LDS; the x-shifted values then come from LDS
// instead of unaligned global loads that straddle two cache lines. With
// non-temporal loads (which made the one-node kernel 7% slower) 3.77 ->
// 3.70 ms at 512^3 (5.51 TB/s).
template <int MODE>
__global__ void __launch_bounds__(512)
k_stream_collide_row32(const float* __restrict__ A, float* __restrict__ B, Dims d, MrtRates r, float3 F0, IbView ib,
                       PatchView pv, uint32_t* __restrict__ err) {
  constexpr int kW = 8, kRow = 66;  // wavefronts per workgroup; floats per staged row: x0 - 1 .. x0 + 64
  __shared__ float seg_all[kW][kQ][kRow];
  const uint32_t b = blockIdx.x;
  const uint32_t logical = (b & 7u) * d.per_xcdr + (b >> 3);
  if (logical >= d.ntilesr) return;  // the whole workgroup
  const uint32_t rowi = fast_div(d.div_gxr, logical);
  const uint32_t bx = logical - rowi * d.gxr;
  const uint32_t bz = fast_div(d.div_ny, rowi);
  const int lane = (int)(threadIdx.x & 63u);
  const int wv = (int)(threadIdx.x >> 6);
  const int y = (int)(rowi - bz * (uint32_t)d.ny);
  const int z = (int)bz;
  float(*seg)[kRow] = seg_all[wv];
  const int nx = d.nx, ny = d.ny, nz = d.nz;
  const uint32_t S = d.S;  // population array stride
  const int x0 = (int)bx * 512 + wv * 64;
  const int x = x0 + lane;
  const bool whole_row = d.gxr == 1u;
  const int wl = wv > 0 ? wv - 1 : (whole_row ? kW - 1 : -1);
  const int wr = wv < kW - 1 ? wv + 1 : (whole_row ? 0 : -1);
  auto row = [&](int yy, int zz) -> uint32_t { return ((uint32_t)zz * (uint32_t)ny + (uint32_t)yy) * (uint32_t)nx; };
  const int ym = y == 0 ? ny - 1 : y - 1, yp = y == ny - 1 ? 0 : y + 1;
  const int zm = z == 0 ? nz - 1 : z - 1, zp = z == nz - 1 ? 0 : z + 1;
  const uint32_t r00 = row(y, z), rm0 = row(ym, z), rp0 = row(yp, z);
  const uint32_t r0m = row(y, zm), r0p = row(y, zp);
  const uint32_t rmm = row(ym, zm), rmp = row(ym, zp), rpp = row(yp, zp), rpm = row(yp, zm);
  const uint32_t srow[kQ] = {r00, r00, rm0, r0m, rm0, rp0, r0m, r0p, rmm, rmp,
                             r00, rp0, r0p, rp0, rm0, r0p, r0m, rpp, rpm};
  const uint32_t xl = (uint32_t)(x0 == 0 ? nx - 1 : x0 - 1);
  const uint32_t xr = (uint32_t)(x0 + 64 >= nx ? 0 : x0 + 64);
  float v[kQ], e[kQ];
#pragma unroll
  for (int i = 0; i < kQ; ++i) {
    const float* rowp = A + (size_t)i * S + srow[i];
    v[i] = __builtin_nontemporal_load(rowp + x);
    e[i] = 0.0f;
    if (cx_of(i) > 0 && wl < 0) e[i] = rowp[xl];
    if (cx_of(i) < 0 && wr < 0) e[i] = rowp[xr];
  }
  // this thread's patch record (at most one: kPatchCap <= 512) with the
  // staging loads
  const uint32_t np = pv.cnt ? min(pv.cnt[rowi], kPatchCap) : 0u;
  uint2 pr = make_uint2(0u, 0u);
  if (threadIdx.x < np) pr = ((const uint2*)pv.rec)[(size_t)rowi * kPatchCap + threadIdx.x];
#pragma unroll
  for (int i = 0; i < kQ; ++i) {
    seg[i][1 + lane] = v[i];
    if (cx_of(i) > 0) {  // reads x - 1: slot 0 holds x0 - 1
      if (lane == 63 && wr >= 0) seg_all[wr][i][0] = v[i];
      if (lane == 0 && wl < 0) seg[i][0] = e[i];
    }
    if (cx_of(i) < 0) {  // reads x + 1: slot 65 holds x0 + 64
      if (lane == 0 && wl >= 0) seg_all[wl][i][kRow - 1] = v[i];
      if (lane == 0 && wr < 0) seg[i][kRow - 1] = e[i];
    }
  }
  __syncthreads();  // the neighbours' end nodes are in place
  if (np) {  // the same for the whole workgroup
    // the slot node x pulls direction i from: 1 + (x mod 64) - c_ix of
    // wavefront x / 64's staged row i (whole rows only: bx = 0)
    if (threadIdx.x < np) {
      const uint32_t xp = pr.x & 0xFFFFu, i = pr.x >> 16;
      seg_all[xp >> 6][i][1 + (int)(xp & 63u) - cx_of((int)i)] = __uint_as_float(pr.y);
    }
    __syncthreads();
  }
  const uint32_t n = r00 + (uint32_t)x;
  float3 F = F0;
  if (MODE == 2) {
    F = body_force_at(ib, n, F0);
    add_ib_force(ib, n, F);
  }
  float g[kQ];
#pragma unroll
  for (int i = 0; i < kQ; ++i) g[i] = seg[i][1 + lane - cx_of(i)];
  float rho, ux, uy, uz;
  mrt_collide(g, F.x, F.y, F.z, r, rho, ux, uy, uz);
#pragma unroll
  for (int i = 0; i < kQ; ++i) Pop<0>::store_stream(B + (size_t)i * S + n, g[i]);
  const bool bad = !(rho > 0.0f) || !(ux * ux + uy * uy + uz * uz < 0.1225f);
  if (bad) atomicOr(err, kErrUnstable);
}

template <int STORE>
__global__ void __launch_bounds__(256)
k_init_equilibrium(const float* __restrict__ u, const float* __restrict__ rho, typename Pop<STORE>::T* __restrict__ f,
                   uint32_t N, uint32_t S) {
  const uint32_t n = blockIdx.x * 256u + threadIdx.x;
  if (n >= N) return;
  const float r = rho ? rho[n] : 1.0f;
  const float ux = u[n], uy = u[(size_t)N + n], uz = u[2 * (size_t)N + n];
#pragma unroll
  for (int i = 0; i < kQ; ++i) Pop<STORE>::store(f + (size_t)i * S + n, geq(i, r, ux, uy, uz));
}

// rho and u from post-collision populations: the Guo collision adds F to the
// momentum, so sum_i c_i f~_i = rho u + F/2 and u = (sum_i c_i f~_i - F/2)/rho.
template <int STORE, int MODE>
__global__ void __launch_bounds__(256)
k_fields(const typename Pop<STORE>::T* __restrict__ f, uint32_t N, uint32_t S, float3 F0, IbView ib,
         float* __restrict__ u, float* __restrict__ rho) {
  const uint32_t n = blockIdx.x * 256u + threadIdx.x;
  if (n >= N) return;
  float3 F = F0;
  if (MODE == 2) {
    F = body_force_at(ib, n, F0);
    add_ib_force(ib, n, F);
  }
  float drho = 0.0f, jx = 0.0f, jy = 0.0f, jz = 0.0f;
#pragma unroll
  for (int i = 0; i < kQ; ++i) {
    const float g = Pop<STORE>::load(f + (size_t)i * S + n);
    drho += g;
    jx += cx_of(i) * g;
    jy += cy_of(i) * g;
    jz += cz_of(i) * g;
  }
  const float r = 1.0f + drho;
  if (rho) rho[n] = r;
  if (u) {
    u[n] = (jx - 0.5f * F.x) / r;
    u[(size_t)N + n] = (jy - 0.5f * F.y) / r;
    u[2 * (size_t)N + n] = (jz - 0.5f * F.z) / r;
  }
}

}  // namespace

hipError_t launch_init_equilibrium(const Ctx& c, const float* u, const float* rho, void* f) {
  if (lattice27(c)) return launch_init_equilibrium27(c, u, rho, f);
  const uint32_t N = c.dims.N;
  const dim3 grid((N + 255) / 256), block(256);
  if (c.cfg.store == LBM_STORE_F32)
    hipLaunchKernelGGL(k_init_equilibrium<0>, grid, block, 0, c.stream, u, rho, (float*)f, N, c.dims.S);
  else
    hipLaunchKernelGGL(k_init_equilibrium<1>, grid, block, 0, c.stream, u, rho, (_Float16*)f, N, c.dims.S);
  return hipGetLastError();
}

// Interpolated bounce-back runs this kernel over solid nodes too: a sphere
// of diameter 16 is narrower than one 64-node wavefront row, so skipping
// them saves no cache lines and only costs divergence. Their values are never
// read by a fluid node (those pull the ghost slots) and are refilled before
// the node turns fluid.
// FP16 storage with an even row length stages its rows through LDS.
static bool use_seg_kernel(const Ctx& c) { return c.cfg.store == LBM_STORE_F16S && c.dims.nx % 2 == 0; }
// The row kernels where one workgroup holds the whole row (nx = 512): at
// 1024-node rows (two workgroups per row) the FP16 one measured 7% slower
// than the 128 x 4 tiles, whose four rows per workgroup share their source
// rows.
static bool use_row_kernel(const Ctx& c) { return c.cfg.store == LBM_STORE_F16S && c.dims.nx == 512; }
static bool use_row32_kernel(const Ctx& c) { return c.cfg.store == LBM_STORE_F32 && c.dims.nx == 512; }

// One-node kernel in the tile width that fills the rows best.
template <int STORE, int MODE>
hipError_t launch_one_node(const Ctx& c, const void* A, void* B, const IbView& ib) {
  using T = typename Pop<STORE>::T;
  if (tile_width(c.dims.nx) == 64) {
    const Tiles tg = make_tiles(c.dims, 64);
    hipLaunchKernelGGL((k_stream_collide<STORE, MODE, 64>), dim3(tg.per_xcd * 8), dim3(256), 0, c.stream,
                       (const T*)A, (T*)B, c.dims, tg, c.rates, c.body_force, ib, c.err);
  } else {
    const Tiles tg = make_tiles(c.dims, 128);
    hipLaunchKernelGGL((k_stream_collide<STORE, MODE, 128>), dim3(tg.per_xcd * 8), dim3(256), 0, c.stream,
                       (const T*)A, (T*)B, c.dims, tg, c.rates, c.body_force, ib, c.err);
  }
  return hipGetLastError();
}

hipError_t launch_stream_collide(const Ctx& c, const void* A, void* B, bool patches) {
  if (lattice27(c)) return launch_stream_collide27(c, A, B);
  const dim3 block(256);
  const IbView none{nullptr, nullptr, nullptr, 0, nullptr};
  const PatchView pv{patches && c.ibb.patches ? c.ibb.patch_cnt : nullptr, c.ibb.patch};
  if (use_row32_kernel(c))
    hipLaunchKernelGGL((k_stream_collide_row32<0>), dim3(c.dims.per_xcdr * 8), dim3(512), 0, c.stream,
                       (const float*)A, (float*)B, c.dims, c.rates, c.body_force, none, pv, c.err);
  else if (use_row_kernel(c))
    hipLaunchKernelGGL((k_stream_collide_row<0>), dim3(c.dims.per_xcdr * 8), block, 0, c.stream,
                       (const _Float16*)A, (_Float16*)B, c.dims, c.rates, c.body_force, none, pv, c.err);
  else if (use_seg_kernel(c))
    hipLaunchKernelGGL((k_stream_collide_seg<0>), dim3(c.dims.per_xcd2 * 8), block, 0, c.stream,
                       (const _Float16*)A, (_Float16*)B, c.dims, c.rates, c.body_force, none, c.err);
  else if (c.cfg.store == LBM_STORE_F32)
    return launch_one_node<0, 0>(c, A, B, none);
  else
    return launch_one_node<1, 0>(c, A, B, none);
  return hipGetLastError();
}

hipError_t launch_stream_collide_ibm(const Ctx& c, const void* A, void* B) {
  const dim3 block(256);
  const int b = c.ibm.cur;
  const IbView ib{c.ibm.bits[b], c.ibm.rank[b], c.ibm.fib[b], c.ibm.s_cap, ibm_body_force_mask(c)};
  const PatchView nop{nullptr, nullptr};
  if (use_row32_kernel(c))
    hipLaunchKernelGGL((k_stream_collide_row32<2>), dim3(c.dims.per_xcdr * 8), dim3(512), 0, c.stream,
                       (const float*)A, (float*)B, c.dims, c.rates, c.body_force, ib, nop, c.err);
  else if (use_row_kernel(c))
    hipLaunchKernelGGL((k_stream_collide_row<2>), dim3(c.dims.per_xcdr * 8), block, 0, c.stream,
                       (const _Float16*)A, (_Float16*)B, c.dims, c.rates, c.body_force, ib, nop, c.err);
  else if (use_seg_kernel(c))
    hipLaunchKernelGGL((k_stream_collide_seg<2>), dim3(c.dims.per_xcd2 * 8), block, 0, c.stream,
                       (const _Float16*)A, (_Float16*)B, c.dims, c.rates, c.body_force, ib, c.err);
  else if (c.cfg.store == LBM_STORE_F32)
    return launch_one_node<0, 2>(c, A, B, ib);
  else
    return launch_one_node<1, 2>(c, A, B, ib);
  return hipGetLastError();
}

hipError_t launch_fields(const Ctx& c, const void* f, float3 F, float* u, float* rho) {
  if (lattice27(c)) return launch_fields27(c, f, F, u, rho);
  const uint32_t N = c.dims.N;
  const dim3 grid((N + 255) / 256), block(256);
  const IbView none{nullptr, nullptr, nullptr, 0, nullptr};
  if (c.cfg.store == LBM_STORE_F32)
    hipLaunchKernelGGL((k_fields<0, 0>), grid, block, 0, c.stream, (const float*)f, N, c.dims.S, F, none, u, rho);
  else
    hipLaunchKernelGGL((k_fields<1, 0>), grid, block, 0, c.stream, (const _Float16*)f, N, c.dims.S, F, none, u, rho);
  return hipGetLastError();
}

// Fields after an immersed-boundary step: the collision force was the body
// force plus the spread force of support buffer `buf`.
hipError_t launch_fields_ibm(const Ctx& c, const void* f, int buf, float* u, float* rho) {
  const uint32_t N = c.dims.N;
  const dim3 grid((N + 255) / 256), block(256);
  const IbView ib{c.ibm.bits[buf], c.ibm.rank[buf], c.ibm.fib[buf], c.ibm.s_cap, ibm_body_force_mask(c)};
  if (c.cfg.store == LBM_STORE_F32)
    hipLaunchKernelGGL((k_fields<0, 2>), grid, block, 0, c.stream, (const float*)f, N, c.dims.S, c.body_force, ib, u, rho);
  else
    hipLaunchKernelGGL((k_fields<1, 2>), grid, block, 0, c.stream, (const _Float16*)f, N, c.dims.S, c.body_force, ib, u, rho);
  return hipGetLastError();
}

}  // namespace lbm
