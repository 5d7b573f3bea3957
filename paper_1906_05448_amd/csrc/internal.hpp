// internal.hpp - context layout and kernel launchers shared by the library's
// translation units. Not part of the public ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <algorithm>
#include <vector>

#include "d3q19.hpp"
#include "lbm.h"

namespace lbm {

// Error bits latched on the device and reported by the next sync call.
enum : uint32_t { kErrUnstable = 1u, kErrOverlap = 2u, kErrCapacity = 4u };

// Owner map codes: a particle index, or one of these.
constexpr uint32_t kFluid = 0xFFFFFFFFu;
constexpr uint32_t kWall = 0xFFFFFFFEu;

// Link metadata byte: direction (bits 0..4), scheme (bits 5..6).
enum : uint32_t { kSchemeHalfway = 0, kSchemeLinear = 1, kSchemeQuadratic = 2 };

// Dense kernels remap the flat block id so that consecutive tiles land on the
// same XCD (the hardware deals workgroups round-robin over the 8 XCDs, each
// with its own L2).
// Unsigned division by an invariant divisor d >= 1 with one multiply-high
// (Granlund & Montgomery 1994, round-up method):
//   l = ceil(log2 d), m = floor(2^32 (2^l - d) / d) + 1,
//   q = (t + ((n - t) >> min(l, 1))) >> max(l - 1, 0), t = mulhi(m, n),
// exact for every 32-bit n.
struct FastDiv {
  uint32_t m, s1, s2;
};

inline FastDiv make_fastdiv(uint32_t d) {
  uint32_t l = 0;
  while ((1ull << l) < (unsigned long long)d) ++l;
  FastDiv f;
  f.m = (uint32_t)(((1ull << 32) * ((1ull << l) - d)) / d + 1);
  f.s1 = l < 1 ? l : 1;
  f.s2 = l > 0 ? l - 1 : 0;
  return f;
}

__device__ __forceinline__ uint32_t fast_div(const FastDiv& f, uint32_t n) {
  const uint32_t t = __umulhi(f.m, n);
  return (t + ((n - t) >> f.s1)) >> f.s2;
}

struct Dims {
  int nx, ny, nz;
  uint32_t N;       // nodes
  uint32_t S;       // elements from one population array to the next (N plus a pad)
  // Tiles of 128 x 4 nodes for the FP16 kernel that stages rows in LDS.
  uint32_t gx2, gy2, ntiles2, per_xcd2;
  FastDiv div_gx2, div_gy2;
  // Row tiles of 512 x 1 nodes (nx a multiple of 512) for the same kernel
  // with the segment edges passed between wavefronts.
  uint32_t gxr, ntilesr, per_xcdr;
  FastDiv div_gxr, div_ny;
};

// The population arrays are kPopPadBytes further apart than their length.
// With N a large power of two the arrays would otherwise start at the same
// offset modulo every interleave period of the memory, and the 19 read and
// 19 write streams of the stream-collide kernels would meet in the same
// channels at the same time. At 512^3, with the two population buffers
// adjacent as the workspace places them, a 1 KB pad took the FP16 row kernel
// from 5.60 to 5.68 TB/s and the FP32 one from 5.55 to 5.58 TB/s (pads of
// 256 B to 4 KB all measured within 0.4% of that; in separately allocated
// buffers the unpadded kernel varied between 5.47 and 5.59 TB/s and a
// 64-byte pad took it to 4.95). The pad is a multiple of 128 bytes, so every
// alignment of an array start is kept.
constexpr uint32_t kPopPadBytes = 1024;

inline Dims make_dims(int nx, int ny, int nz, uint32_t elem_bytes) {
  Dims d;
  d.nx = nx;
  d.ny = ny;
  d.nz = nz;
  d.N = (uint32_t)nx * (uint32_t)ny * (uint32_t)nz;
  d.S = d.N + kPopPadBytes / elem_bytes;
  d.gx2 = (uint32_t)(nx + 127) / 128;
  d.gy2 = (uint32_t)(ny + 3) / 4;
  d.ntiles2 = d.gx2 * d.gy2 * (uint32_t)nz;
  d.per_xcd2 = (d.ntiles2 + 7) / 8;
  d.div_gx2 = make_fastdiv(d.gx2);
  d.div_gy2 = make_fastdiv(d.gy2);
  d.gxr = (uint32_t)(nx + 511) / 512;
  d.ntilesr = d.gxr * (uint32_t)ny * (uint32_t)nz;
  d.per_xcdr = (d.ntilesr + 7) / 8;
  d.div_gxr = make_fastdiv(d.gxr);
  d.div_ny = make_fastdiv((uint32_t)ny);
  return d;
}

// Coordinates of a lane's node in its workgroup's tile.
struct Tile {
  int x, y, z;
  bool live;
};

// Tiles of TW x (256 / TW) nodes of the one-node FP32 kernels (D3Q19 and
// D3Q27) in XCD-contiguous order: 128 x 2 (measured 1.4% faster than 64 x 4
// where both fill the rows), or 64 x 4 where that leaves fewer idle lanes at
// the end of a row (a 160-node row fills 5 of 6 wavefronts instead of 5 of 8).
struct Tiles {
  uint32_t gx, gy, ntiles, per_xcd;
  FastDiv div_gx, div_gy;
};

inline Tiles make_tiles(const Dims& d, int tw) {
  Tiles g;
  g.gx = (uint32_t)(d.nx + tw - 1) / (uint32_t)tw;
  g.gy = (uint32_t)(d.ny + 256 / tw - 1) / (uint32_t)(256 / tw);
  g.ntiles = g.gx * g.gy * (uint32_t)d.nz;
  g.per_xcd = (g.ntiles + 7) / 8;
  g.div_gx = make_fastdiv(g.gx);
  g.div_gy = make_fastdiv(g.gy);
  return g;
}

template <int TW>
__device__ __forceinline__ Tile tile_of(const Dims& d, const Tiles& g) {
  const uint32_t b = blockIdx.x;
  const uint32_t logical = (b & 7u) * g.per_xcd + (b >> 3);
  const uint32_t rest = fast_div(g.div_gx, logical);
  const uint32_t bx = logical - rest * g.gx;
  const uint32_t bz = fast_div(g.div_gy, rest);
  const uint32_t by = rest - bz * g.gy;
  Tile t;
  t.x = (int)(bx * (uint32_t)TW + (threadIdx.x % (uint32_t)TW));
  t.y = (int)(by * (256u / TW) + threadIdx.x / (uint32_t)TW);
  t.z = (int)bz;
  t.live = logical < g.ntiles && t.x < d.nx && t.y < d.ny;
  return t;
}

// 64 where 64 x 4 tiles leave fewer idle lanes along x than 128 x 2.
inline int tile_width(int nx) {
  const int g128 = (nx + 127) / 128, g64 = (nx + 63) / 64;
  return 128 * g128 > 64 * g64 ? 64 : 128;
}

// Bitmask words covering N nodes.
inline uint32_t mask_words(uint32_t N) { return (N + 31u) / 32u; }

// Optional per-kernel timing with HIP events on the context's stream.
struct Profiler {
  struct Pair {
    hipEvent_t a, b;
    int cls;
  };
  bool on = false;
  std::vector<Pair> pending;
  std::vector<hipEvent_t> pool;
  double ms[LBM_NPROF] = {};
  int64_t launches[LBM_NPROF] = {};

  hipEvent_t take() {
    if (!pool.empty()) {
      hipEvent_t e = pool.back();
      pool.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
  }
  // Waits for every pending pair and folds it into the totals.
  hipError_t harvest() {
    hipError_t st = hipSuccess;
    for (auto& p : pending) {
      float t = 0.0f;
      hipError_t e = hipEventSynchronize(p.b);
      if (e == hipSuccess) e = hipEventElapsedTime(&t, p.a, p.b);
      if (e != hipSuccess) st = e;
      ms[p.cls] += t;
      launches[p.cls] += 1;
      pool.push_back(p.a);
      pool.push_back(p.b);
    }
    pending.clear();
    return st;
  }
  ~Profiler() {
    (void)harvest();
    for (auto e : pool) (void)hipEventDestroy(e);
  }
};

// FP64 particle state and per-particle accumulators, each [P][3] unless
// noted. X/U/Om are double-buffered: [cur] holds step n, [1-cur] receives n+1.
struct ParticleBufs {
  double* X[2];
  double* U[2];
  double* Om[2];
  double* r;       // [P]
  double* rho;     // [P]
  double* F_link;  // interpolated bounce-back: link forces of this step
  double* T_link;
  double* F_rc;    // momentum of covered/uncovered nodes, for the next step
  double* T_rc;
  double* F_h;     // hydrodynamic force/torque that entered the last update
  double* T_h;
  double* F_c;     // contact force of the last update
  double* F_ib;    // immersed boundary: -sum F_l dV of this step
  double* T_ib;
  double* Iu;      // Kempe inner momentum sum alpha u, previous and new
  double* IL;
  double* Iu_new;
  double* IL_new;
  double* Xown[2]; // positions owner map [b] was last built for
  uint32_t* cell_head;  // [cells] first particle of each contact cell
  uint32_t* cell_next;  // [P] next particle in the same cell
  int cells[3];         // contact cell grid
};

// The link kernel works on slices of a sphere's links, one workgroup of
// kLinkSliceThreads threads per slice.
constexpr int kLinkSliceThreads = 256;
constexpr uint32_t kLinkSlice = 1280;

// Interpolated bounce-back geometry.
struct IbbBufs {
  uint32_t* owner[2];    // [N] owner codes, [cur] at step n
  uint32_t* solid_bits;  // [mask_words] solid nodes of step n (dense kernel)
  uint32_t* wall_bits;   // [mask_words] static wall
  uint32_t* link_node;   // [P * link_cap] fluid node of each link
  float* link_q;         // wall fraction q
  uint8_t* link_meta;    // direction | scheme << 5
  uint32_t* link_count;  // [P]
  double* link_part;     // [P][link_slices][6] FP64 force/torque per slice of links
  uint32_t link_slices;  // slices of kLinkSlice links per sphere
  uint32_t* wl_node;     // static wall links
  float* wl_q;
  uint8_t* wl_meta;
  uint32_t wl_count;
  // Bounce-back patches (rows of 512 nodes, where the stream-collide
  // kernels stage whole rows in LDS): the link pass lists each interpolated
  // value under the row of its fluid node instead of storing it into the
  // ghost slot, and the kernel writes it over the staged slot in LDS. A
  // link beyond kPatchCap in its row falls back to the ghost slot.
  bool patches;          // this context uses them
  uint32_t* patch_cnt;   // [ny * nz] links listed per row this step
  // [ny * nz][kPatchCap] records of the node x, the opposite direction i and
  // the stored value's bits: FP16 one word, x | i << 9 | bits << 16; FP32
  // two words, x | i << 16 and the bits
  void* patch;
};

constexpr uint32_t kPatchCap = 256;

// Immersed boundary support. The support set S (marker stencils plus the
// cells of the Kempe integrals) is a bitmask with a per-word exclusive rank,
// so node n in S has slot rank[n >> 5] + popcount(bits[n >> 5] below n).
// Slot arrays hold the prepass density/velocity and the spread force. Bits,
// rank, count and force are double-buffered: [cur] is the support of step n,
// [1-cur] that of the last completed collision (field extraction).
struct IbmBufs {
  uint32_t* bits[2];     // [mask_words]
  uint32_t* rank[2];     // [mask_words]
  uint32_t* count[2];    // [1] support size
  float4* fib[2];        // [S_cap] spread force per slot (x, y, z; w unused)
  uint32_t* shared;      // [mask_words] nodes in more than one sphere's support
  // Shared nodes: their forcing contributions of a pass are summed exactly
  // (64-bit fixed point, units 2^-50) apart from the slot forces, which the
  // other spheres read during the same pass, and folded in after it.
  uint32_t* sh_rank;     // [mask_words] rank of the shared bitmask words
  uint32_t* sh_count;    // [1] shared nodes
  uint32_t* sh_slot;     // [sh_cap] node, then slot, of each shared node
  unsigned long long* sh_acc;  // [3][sh_cap] pass contributions, zero between passes
  uint32_t sh_cap;
  uint32_t* list;        // [S_cap] node of each slot (current support)
  float4* us;            // [S_cap] (u*, rho) from the prepass
  uint32_t* block_sums;  // scan scratch
  double* dirs;          // [n_markers][3] unit marker directions (Fibonacci)
  uint32_t* rowbits;     // [P][rows] per-sphere forcing-support rows (box-local)
  uint32_t* fcount;      // [P] forcing-support size per sphere
  uint32_t* fslot;       // [P][fcap] global slot of each forcing-support node,
                         // or kSlotShared | shared index at shared nodes
  // Per-sphere copies, in fslot order, of (u*, rho) and of the spread force
  // at the sphere's unshared forcing nodes between the passes of one step:
  // read contiguously instead of gathered through the slot list.
  float4* pu;            // [P][fcap]
  float4* pf;            // [P][fcap]
  uint32_t s_cap;        // slots reserved
  uint32_t fcap;         // forcing-support nodes reserved per sphere
  int n_markers;         // markers per sphere
  double r_l;            // marker radius r - r_d
  double dV;             // marker volume
  int R_b;               // box half-width: box is floor(X) - R_b .. + R_b + 1
  int side;              // 2 R_b + 2 (<= 32)
  int cur;               // support of the next collision
  int last;              // support used by the last collision
  // Static pipe-wall markers (rings at every integer z), if any.
  uint32_t n_wall;       // markers
  double wdV;            // marker volume
  double* wmark;         // [n_wall][3] positions
  float* wdF;            // [n_wall][3] force of the current pass
  uint32_t* wsup;        // [mask_words] support of the wall stencils
};

// A second stream, at the default priority, for the work of a step that
// can run beside the stream-collide kernel (the particle stage and the next
// step's geometry): forked from the caller's stream and joined back into it
// within the step, so every call that returns leaves all of its work ordered
// on the caller's stream.
struct SideStream {
  hipStream_t s = nullptr;
  hipEvent_t fork = nullptr, join = nullptr;
  SideStream() = default;
  SideStream(const SideStream&) = delete;
  SideStream& operator=(const SideStream&) = delete;
  hipError_t create() {
    hipError_t e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&fork, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&join, hipEventDisableTiming);
    return e;
  }
  ~SideStream() {
    if (join) (void)hipEventDestroy(join);
    if (fork) (void)hipEventDestroy(fork);
    if (s) (void)hipStreamDestroy(s);
  }
};

struct Ctx {
  lbm_config cfg;
  hipStream_t stream;
  int device;
  Dims dims;
  MrtRates rates;
  float3 body_force;
  // Workspace slices (device pointers).
  void* f_cur;      // post-collision shifted populations, [19][N]
  void* f_nxt;
  uint32_t* err;    // latched error bits (one word)
  double* scratch_d;  // small FP64 scratch for reductions
  double* stats_part; // [kStatGrid + 1][kStatStride] statistics partial sums
  int64_t step;
  Profiler prof;
  SideStream side;
  bool overlap = false;  // particle stage and next geometry beside the stream-collide kernel
  // Particles.
  int32_t np;            // particles set
  int32_t motion;        // LBM_MOTION_*
  int pcur;              // which X/U/Om buffer is current
  int ocur;              // which owner map is current
  uint32_t link_cap;     // links reserved per particle
  ParticleBufs P;
  IbbBufs ibb;
  IbmBufs ibm;
  double max_radius_set; // largest radius of the particles set
  // Gradient corrector attached for the statistics (lbm_corrector_set).
  const float* corr_theta;  // device FP32 network parameters, null: off
  double corr_dmin, corr_dmax, corr_urms;
  // Pipe TKE budget accumulator (lbm_pipe_budget_*).
  struct PipeBudget {
    double* acc;      // [LBM_PIPE_BUDGET_MOMENTS][nbins] moment sums
    uint32_t* list;   // fluid (x, y) of the cross-section by bin: x | y << 16
    uint32_t* off;    // [nbins + 1] bin offsets in list
    int nbins;        // 0 until reset
    double width;
    int64_t snapshots;
  } pb;
};

// Runs a launcher, bracketed by timing events when profiling is on.
template <class F>
hipError_t timed(Ctx& c, int cls, F&& launch) {
  if (!c.prof.on) return launch();
  hipEvent_t a = c.prof.take(), b = c.prof.take();
  if (!a || !b) return hipErrorOutOfMemory;
  hipError_t e = hipEventRecord(a, c.stream);
  if (e == hipSuccess) e = launch();
  if (e == hipSuccess) e = hipEventRecord(b, c.stream);
  if (e != hipSuccess) return e;
  c.prof.pending.push_back({a, b, cls});
  if (c.prof.pending.size() > 8192) e = c.prof.harvest();
  return e;
}

// The side stream waits for the caller's stream up to here.
inline hipError_t fork_side(Ctx& c) {
  hipError_t e = hipEventRecord(c.side.fork, c.stream);
  if (e == hipSuccess) e = hipStreamWaitEvent(c.side.s, c.side.fork, 0);
  return e;
}

// The caller's stream waits for everything launched on the side stream.
inline hipError_t join_side(Ctx& c) {
  hipError_t e = hipEventRecord(c.side.join, c.side.s);
  if (e == hipSuccess) e = hipStreamWaitEvent(c.stream, c.side.join, 0);
  return e;
}

// Runs launchers (and their timing events) on the side stream.
template <class F>
hipError_t on_side(Ctx& c, F&& launch) {
  const hipStream_t main = c.stream;
  c.stream = c.side.s;
  const hipError_t e = launch();
  c.stream = main;
  return e;
}

// Dense kernels (dense.hip).
hipError_t launch_init_equilibrium(const Ctx& c, const float* u, const float* rho, void* f);
// patches: apply the bounce-back patches the link pass listed this step.
hipError_t launch_stream_collide(const Ctx& c, const void* A, void* B, bool patches = false);
// D3Q27 pipe solver (d3q27.hip); the D3Q19 launchers dispatch to these
// when the configuration selects that lattice.
hipError_t launch_stream_collide27(const Ctx& c, const void* A, void* B);
hipError_t launch_init_equilibrium27(const Ctx& c, const float* u, const float* rho, void* f);
hipError_t launch_fields27(const Ctx& c, const void* f, float3 F, float* u, float* rho);
hipError_t launch_wall_links27(Ctx& c, const uint32_t* owner, uint32_t* counter, bool count_only);
hipError_t launch_wall_bounce27(const Ctx& c, void* A);
inline bool lattice27(const Ctx& c) { return c.cfg.lattice == LBM_LATTICE_D3Q27; }
// u, rho from post-collision populations; F is the force of the collision
// that produced them (zero before the first step).
hipError_t launch_fields(const Ctx& c, const void* f, float3 F, float* u, float* rho);

// Geometry (geometry.hip).
hipError_t launch_owner_fill(const Ctx& c, uint32_t* owner);
hipError_t launch_owner_clear(const Ctx& c, uint32_t* owner, const double* Xold, int32_t np_old);
// Xown (optional): receives X, the positions the map is set with.
hipError_t launch_owner_set(const Ctx& c, uint32_t* owner, const double* X, double* Xown = nullptr);
hipError_t launch_count_solid(const Ctx& c, const uint32_t* owner, unsigned long long* out);
size_t links_build_lds_bytes(double max_radius);  // dynamic LDS of the link build
size_t links_build_lds_total(double max_radius);  // its dynamic plus static LDS
hipError_t launch_links_build(const Ctx& c, const uint32_t* owner, const double* X);
hipError_t launch_wall_links(Ctx& c, const uint32_t* owner, uint32_t* counter, bool count_only);

// Interpolated bounce-back (ibb.hip).
hipError_t launch_ibb_links(const Ctx& c, void* A, const double* X, const double* U, const double* Om);
hipError_t launch_cover_refill(const Ctx& c, void* B, const uint32_t* owner_old, const uint32_t* owner_new,
                               const double* Xold, const double* Xnew, const double* Unew, const double* Omnew);

// Immersed boundary (ibm.hip).
size_t ibm_pass_lds_bytes(const Ctx& c);
hipError_t launch_ibm_support_build(Ctx& c, int buf, const double* X);
hipError_t launch_ibm_prepass(const Ctx& c, const void* A);
hipError_t launch_ibm_forcing_pass(const Ctx& c, const double* X, const double* U, const double* Om);
hipError_t launch_ibm_kempe(const Ctx& c, const double* X, double* Iu, double* IL);
hipError_t launch_kempe_dense(const Ctx& c, const float* u, const double* X, double* Iu, double* IL);
hipError_t launch_stream_collide_ibm(const Ctx& c, const void* A, void* B);
// Nodes without body force under the immersed boundary: outside the pipe
// (null without a wall).
inline const uint32_t* ibm_body_force_mask(const Ctx& c) {
  return c.cfg.wall == LBM_WALL_PIPE_Z ? c.ibb.wall_bits : nullptr;
}
// Set bits of a node bitmask -> ascending node list: rank[w] = set bits
// before word w, *count = total, list[i] = i-th set node (entries beyond cap
// dropped, *err |= capacity bit). block_sums: bits_compact_scratch_words().
size_t bits_compact_scratch_words(uint32_t nwords);
hipError_t launch_bits_compact(hipStream_t st, const uint32_t* bits, uint32_t nwords, uint32_t* rank,
                               uint32_t* block_sums, uint32_t* count, uint32_t* list, uint32_t cap, uint32_t* err);
hipError_t launch_fields_ibm(const Ctx& c, const void* f, int buf, float* u, float* rho);

// Particles (particles.hip).
hipError_t launch_particle_update(const Ctx& c);
hipError_t launch_release_average(const Ctx& c, const float* u, double* Uout);
// Interior populations of every sphere -> equilibrium of the local density
// and the rigid-body velocity U + Omega x (x - X).
hipError_t launch_release_overwrite(const Ctx& c, void* f, const uint32_t* owner, const double* U, const double* Om);
// Statistics (stats.hip). Columns of the per-block partial sums; the
// histograms follow as [5][nbins] (count, sum 1/2|u|^2, sum eps, sum u_z,
// sum u_z^2).
enum {
  kStatNf, kStatMass, kStatMomX, kStatMomY, kStatMomZ, kStatKeRaw, kStatKeFluid, kStatEpsRaw, kStatUmax2, kStatBulk,
  kStatKeMasked, kStatEpsMasked, kStatEpsFluid, kStatScalars
};
constexpr int kStatGrid = 1024;  // workgroups of the grid-stride passes
constexpr int kStatStride = kStatScalars + 5 * LBM_STATS_MAX_BINS;
size_t stats_part_bytes();
// u, rho: the extracted field; key: [N] scratch. Writes kStatScalars + 5 nbins
// sums to out (device).
// Corrector network (mlp.hip). part: [kMlpGrid][10249] FP32, lpart:
// [kMlpGrid] FP64.
constexpr int kMlpGrid = 256;
size_t mlp_train_lds_bytes();
size_t mlp_forward_lds_bytes();
hipError_t launch_mlp_forward(hipStream_t st, const float* theta, const uint16_t* X, int64_t n, float* Y);
hipError_t launch_mlp_gradient(hipStream_t st, const float* theta, const uint16_t* X, const float* T, int64_t n,
                               float* part, double* lpart, float* grad, double* loss);
hipError_t launch_mlp_adam(hipStream_t st, float* theta, float* m, float* v, const float* g, float lr, float b1,
                           float b2, float eps, float c1, float c2);
// Gradient corrector (corrector.hip). once, twice and cellbits are
// consecutive [mask_words] bitmasks.
struct CorrBufs {
  uint32_t *once, *twice, *cellbits, *rank, *bsums, *count, *err;
  uint32_t* cellp;  // [N] sphere of each cell node
};
hipError_t launch_corrector_cells(const Ctx& c, const double* X, double dmin, double dmax, const CorrBufs& b,
                                  uint32_t* list, uint32_t* plist, uint32_t cap);
hipError_t launch_corrector_features(const Ctx& c, const float* u, const uint32_t* list, const uint32_t* plist,
                                     const uint32_t* count, uint32_t cap, const double* X, const double* U,
                                     const double* Om, double u_rms, uint16_t* out);
hipError_t launch_corrector_labels(const Ctx& c, const float* u, const uint32_t* key, const uint32_t* list, uint32_t n,
                                   const double* X, const double* U, const double* Om, double u_rms, int subtract,
                                   float* out);
size_t corrector_stats_lds_bytes();
// Writes (sum of eps corrected - eps plain, cells, per-bin sums) to out.
hipError_t launch_corrector_stats(const Ctx& c, const float* theta, const float* u, const uint32_t* key,
                                  const uint32_t* list, const uint32_t* plist, const uint32_t* count, uint32_t cap,
                                  const double* X, const double* U, const double* Om, double u_rms, int nbins,
                                  double* part, double* out);
// Node keys only (see stats_device.hpp).
hipError_t launch_stats_keys(const Ctx& c, uint32_t* key, int nbins, double width, const double* X);
// Pipe TKE budget moments (budget.hip). part: nbins * nz * 38 doubles.
size_t pipe_budget_part_bytes(const Ctx& c, int nbins);
hipError_t launch_pipe_budget_add(const Ctx& c, const float* u, const float* rho, const uint32_t* key, double* part);
// Energy and dissipation spectra (spectrum.hip).
bool spectrum_supported(const Ctx& c);
size_t spectrum_row_len(const Ctx& c);  // partials per (x, y) line
size_t spectrum_lines(const Ctx& c);
hipError_t launch_spec_pack(const Ctx& c, const float* u, const uint32_t* key, int masked, float2* Z1, float2* Z2);
hipError_t launch_fft_xy(const Ctx& c, float2* Z);
hipError_t launch_spec_zbins(const Ctx& c, const float2* Z1, const float2* Z2, double* P, int* smin, int* cnt,
                             int kmax, double nu, double* part, double* E, double* D);
hipError_t launch_stats(const Ctx& c, const float* u, const float* rho, uint32_t* key, int nbins, double width,
                        const double* X, const double* U, const double* Om, double* part, double* out);

}  // namespace lbm

struct lbm_ctx {
  lbm::Ctx c;
};
