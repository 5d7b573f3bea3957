// api.hip - the extern "C" boundary: configuration checks, workspace
// carving, and the host-side sequencing of the kernels on the caller's
// stream. No kernel arithmetic lives here.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <vector>

#include "d3q27.hpp"
#include "internal.hpp"

using namespace lbm;

namespace {

constexpr size_t kAlign = 256;

size_t align_up(size_t v) { return (v + kAlign - 1) & ~(kAlign - 1); }

size_t n_nodes(const lbm_config& c) { return (size_t)c.nx * (size_t)c.ny * (size_t)c.nz; }

int lattice_q(const lbm_config& c) { return c.lattice == LBM_LATTICE_D3Q27 ? q27::kQ : kQ; }

size_t pop_elem_bytes(const lbm_config& c) { return c.store == LBM_STORE_F32 ? 4 : 2; }

// Elements from one population array to the next (the node count plus the
// pad of make_dims).
size_t pop_stride(const lbm_config& c) {
  return (size_t)make_dims(c.nx, c.ny, c.nz, (uint32_t)pop_elem_bytes(c)).S;
}

size_t pop_bytes(const lbm_config& c) { return align_up((size_t)lattice_q(c) * pop_stride(c) * pop_elem_bytes(c)); }

bool has_particles(const lbm_config& c) { return c.bc != LBM_BC_NONE && c.max_particles > 0; }

// Links of an isolated sphere of radius r centred at offset o from a node:
// an upper bound for the links any one particle can own (neighbours only
// remove links). Evaluated on a few sub-grid offsets.
uint32_t link_capacity(double r) {
  uint32_t best = 0;
  const int R = (int)ceil(r) + 2;
  const int cxv[18] = {1, 0, 0, 1, 1, 1, 1, 0, 0, -1, 0, 0, -1, -1, -1, -1, 0, 0};
  const int cyv[18] = {0, 1, 0, 1, -1, 0, 0, 1, 1, 0, -1, 0, -1, 1, 0, 0, -1, -1};
  const int czv[18] = {0, 0, 1, 0, 0, 1, -1, 1, -1, 0, 0, -1, 0, 0, -1, 1, -1, 1};
  for (int t = 0; t < 27; ++t) {
    const double o[3] = {0.5 * (t % 3) * 0.5 + 0.03, 0.5 * ((t / 3) % 3) * 0.5 + 0.07, 0.5 * (t / 9) * 0.5 + 0.11};
    auto inside = [&](int x, int y, int z) {
      const double dx = x - o[0], dy = y - o[1], dz = z - o[2];
      return (dx * dx + dy * dy) + dz * dz < r * r;
    };
    uint32_t n = 0;
    for (int z = -R; z <= R; ++z)
      for (int y = -R; y <= R; ++y)
        for (int x = -R; x <= R; ++x) {
          if (inside(x, y, z)) continue;
          for (int a = 0; a < 18; ++a)
            if (inside(x + cxv[a], y + cyv[a], z + czv[a])) ++n;
        }
    best = std::max(best, n);
  }
  return (uint32_t)(best * 1.25) + 64;
}

bool pipe_solid(const lbm_config& c, int x, int y) {
  const double dx = (double)x - c.pipe_cx, dy = (double)y - c.pipe_cy;
  return dx * dx + dy * dy >= c.pipe_radius * c.pipe_radius;
}

// Links into the static pipe wall (exact count; the pipe is z-invariant).
uint32_t wall_link_count(const lbm_config& c) {
  if (c.wall != LBM_WALL_PIPE_Z) return 0;
  const bool l27 = c.lattice == LBM_LATTICE_D3Q27;
  const int q = l27 ? q27::kQ : kQ;
  uint64_t n = 0;
  for (int y = 0; y < c.ny; ++y)
    for (int x = 0; x < c.nx; ++x) {
      if (pipe_solid(c, x, y)) continue;
      for (int a = 1; a < q; ++a) {
        const int dx = l27 ? q27::cx(a) : cx_of(a), dy = l27 ? q27::cy(a) : cy_of(a);
        const int xs = ((x + dx) % c.nx + c.nx) % c.nx, ys = ((y + dy) % c.ny + c.ny) % c.ny;
        if (pipe_solid(c, xs, ys)) ++n;
      }
    }
  return (uint32_t)(n * (uint64_t)c.nz);
}

// Immersed-boundary pipe wall (Sec. 2.1): rings at every integer z of
// N_theta = round(2 pi r_L) markers (ties to even), retracted into the wall,
// r_L = R + r_d; theta_k = 2 pi k / N_theta; volume 2 pi r_L / N_theta.
bool ibm_wall(const lbm_config& c) { return c.bc == LBM_BC_IBM && c.wall == LBM_WALL_PIPE_Z; }

int pipe_ring_count(const lbm_config& c) {
  return (int)std::nearbyint(2.0 * M_PI * (c.pipe_radius + c.ibm_retraction));
}

void pipe_markers(const lbm_config& c, std::vector<double>& xm, double& dV) {
  const double r_l = c.pipe_radius + c.ibm_retraction;
  const int n = pipe_ring_count(c);
  xm.clear();
  xm.reserve((size_t)3 * n * c.nz);
  for (int z = 0; z < c.nz; ++z)
    for (int k = 0; k < n; ++k) {
      const double th = (2.0 * M_PI) * (double)k / (double)n;
      xm.push_back(c.pipe_cx + r_l * cos(th));
      xm.push_back(c.pipe_cy + r_l * sin(th));
      xm.push_back((double)z);
    }
  dV = 2.0 * M_PI * r_l / (double)n;
}

// Union of the 4x4x4 delta stencils of the wall markers; returns its size.
uint32_t pipe_support(const lbm_config& c, const std::vector<double>& xm, std::vector<uint32_t>& bits) {
  const size_t N = (size_t)c.nx * c.ny * c.nz;
  bits.assign((N + 31) / 32, 0u);
  auto wrap = [](long v, int n) { return (int)(((v % n) + n) % n); };
  for (size_t l = 0; l < xm.size() / 3; ++l) {
    long b[3];
    for (int k = 0; k < 3; ++k) b[k] = (long)floor(xm[3 * l + k]) - 1;
    for (int jz = 0; jz < 4; ++jz)
      for (int jy = 0; jy < 4; ++jy)
        for (int jx = 0; jx < 4; ++jx) {
          const size_t n = ((size_t)wrap(b[2] + jz, c.nz) * c.ny + wrap(b[1] + jy, c.ny)) * c.nx + wrap(b[0] + jx, c.nx);
          bits[n >> 5] |= 1u << (n & 31);
        }
  }
  uint32_t cnt = 0;
  for (uint32_t w : bits) cnt += (uint32_t)__builtin_popcount(w);
  return cnt;
}

// Immersed boundary marker layout (Uhlmann/Breugem count and a Fibonacci
// lattice of directions; the paper only asks for a marker volume close to
// the cell volume, Sec. 2.1).
int marker_count(double r_l) { return (int)lround(M_PI * (12.0 * r_l * r_l + 1.0) / 3.0); }
double marker_volume(double r_l, int n) {
  return (4.0 / 3.0) * M_PI * ((r_l + 0.5) * (r_l + 0.5) * (r_l + 0.5) - (r_l - 0.5) * (r_l - 0.5) * (r_l - 0.5)) / n;
}
void fibonacci_dirs(int n, std::vector<double>& out) {
  out.resize(3 * (size_t)n);
  const double ga = M_PI * (3.0 - sqrt(5.0));
  for (int k = 0; k < n; ++k) {
    const double z = 1.0 - (2.0 * k + 1.0) / n;
    const double phi = k * ga;
    const double s = sqrt(1.0 - z * z);
    out[3 * k] = s * cos(phi);
    out[3 * k + 1] = s * sin(phi);
    out[3 * k + 2] = z;
  }
}
int ibm_half_width(double r, double r_d) {
  return std::max((int)ceil(r - r_d) + 3, (int)ceil(r) + 2);
}
int ibm_box_side(double r, double r_d) { return 2 * ibm_half_width(r, r_d) + 2; }

// Forcing support (union of marker stencils) and full support (plus the
// Kempe cells) of an isolated sphere, maximised over sub-grid offsets:
// capacity bounds (neighbours only merge supports).
void ibm_support_bounds(double r, double r_d, uint32_t& forcing, uint32_t& full) {
  const double r_l = r - r_d;
  const int n = marker_count(r_l);
  std::vector<double> dirs;
  fibonacci_dirs(n, dirs);
  const int R = ibm_half_width(r, r_d), side = 2 * R + 2;
  forcing = full = 0;
  std::vector<uint8_t> box((size_t)side * side * side);
  for (int t = 0; t < 27; ++t) {
    const double o[3] = {0.5 * (t % 3) * 0.5 + 0.03, 0.5 * ((t / 3) % 3) * 0.5 + 0.07, 0.5 * (t / 9) * 0.5 + 0.11};
    std::fill(box.begin(), box.end(), 0);
    const int lo = -R;  // floor(o) = 0
    for (int l = 0; l < n; ++l) {
      int b[3];
      for (int k = 0; k < 3; ++k) b[k] = (int)floor(o[k] + r_l * dirs[3 * l + k]) - 1 - lo;
      for (int jz = 0; jz < 4; ++jz)
        for (int jy = 0; jy < 4; ++jy)
          for (int jx = 0; jx < 4; ++jx) box[((size_t)(b[2] + jz) * side + b[1] + jy) * side + b[0] + jx] = 1;
    }
    uint32_t f = 0, a = 0;
    const double ra = r + 0.8661;
    for (int z = 0; z < side; ++z)
      for (int y = 0; y < side; ++y)
        for (int x = 0; x < side; ++x) {
          const size_t i = ((size_t)z * side + y) * side + x;
          const double dx = x + lo - o[0], dy = y + lo - o[1], dz = z + lo - o[2];
          const bool cell = (dx * dx + dy * dy) + dz * dz < ra * ra;
          f += box[i];
          a += (box[i] || cell) ? 1u : 0u;
        }
    forcing = std::max(forcing, f);
    full = std::max(full, a);
  }
  forcing = (uint32_t)(forcing * 1.05) + 32;
  full = (uint32_t)(full * 1.05) + 32;
}

// Workspace plan: offsets of every slice for a configuration.
struct Plan {
  size_t f_a, f_b, err, scratch, stats_part;
  size_t pdoubles;       // particle FP64 block
  size_t cell_head, cell_next;
  int cells[3];
  size_t owner[2], solid_bits, wall_bits;
  size_t pb_acc, pb_list, pb_off;  // pipe TKE budget
  size_t link_node, link_q, link_meta, link_count, link_part;
  size_t patch_cnt, patch;  // bounce-back patch lists (rows of 512 nodes)
  bool patches;
  uint32_t link_slices;
  size_t wl_node, wl_q, wl_meta;
  uint32_t link_cap, wl_count;
  // immersed boundary
  size_t ib_bits[2], ib_rank[2], ib_count, ib_fib[2], ib_shared, ib_list, ib_us, ib_bsum, ib_dirs, ib_rowbits,
      ib_fcount, ib_fslot, ib_pu, ib_pf, ib_wmark, ib_wdF, ib_wsup, ib_sh_rank, ib_sh_count, ib_sh_slot, ib_sh_acc;
  uint32_t s_cap, fcap, n_markers, n_wall, wall_support;
  int side;
  size_t total;
};

constexpr int kParticleVecs = 21;  // [P][3] FP64 arrays in ParticleBufs (plus r, rho, U0)

// Contact cell grid: cells at least 2 max_radius wide (plus a margin against
// rounding of the cell index), so spheres in contact sit in the same or
// adjacent cells. Coarsened, which keeps that property, until the grid holds
// at most 8 cells per particle.
void contact_cells(const lbm_config& c, size_t P, int n[3]) {
  const double h = 2.0 * c.max_radius + 0.01;
  const int L[3] = {c.nx, c.ny, c.nz};
  for (int a = 0; a < 3; ++a) n[a] = std::max(1, (int)std::floor((double)L[a] / h));
  const size_t cap = std::max<size_t>(8 * P, 4096);
  while ((size_t)n[0] * n[1] * n[2] > cap) {
    const int a = n[0] >= n[1] && n[0] >= n[2] ? 0 : (n[1] >= n[2] ? 1 : 2);
    n[a] = std::max(1, n[a] / 2);
  }
}

Plan plan(const lbm_config& c) {
  Plan p{};
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += align_up(bytes);
    return o;
  };
  const size_t N = n_nodes(c);
  const size_t words = mask_words((uint32_t)N);
  p.f_a = take(pop_bytes(c));
  p.f_b = take(pop_bytes(c));
  p.err = take(kAlign);
  p.scratch = take(64 * sizeof(double));
  p.stats_part = take(stats_part_bytes());
  const size_t P = has_particles(c) ? (size_t)c.max_particles : 0;
  p.pdoubles = take((size_t)(kParticleVecs * 3 + 2 + 3) * std::max<size_t>(P, 1) * sizeof(double));
  p.cells[0] = p.cells[1] = p.cells[2] = 1;
  if (P) contact_cells(c, P, p.cells);
  p.cell_head = take((size_t)p.cells[0] * p.cells[1] * p.cells[2] * 4);
  p.cell_next = take(std::max<size_t>(P, 1) * 4);
  p.wall_bits = take(words * 4);
  if (c.wall == LBM_WALL_PIPE_Z) {
    p.pb_acc = take((size_t)LBM_PIPE_BUDGET_MOMENTS * LBM_PIPE_BUDGET_MAX_BINS * sizeof(double));
    p.pb_list = take((size_t)c.nx * (size_t)c.ny * 4);
    p.pb_off = take((LBM_PIPE_BUDGET_MAX_BINS + 1) * 4);
  }
  p.solid_bits = take(words * 4);
  if (c.bc != LBM_BC_NONE) {
    p.owner[0] = take(N * 4);
    p.owner[1] = take(N * 4);
  }
  if (c.bc == LBM_BC_IBB) {
    p.link_cap = P ? link_capacity(c.max_radius) : 0;
    const size_t L = P * p.link_cap;
    p.link_node = take(L * 4 + 4);
    p.link_q = take(L * 4 + 4);
    p.link_meta = take(L + 4);
    p.link_count = take(P * 4 + 4);
    p.link_slices = std::max<uint32_t>((p.link_cap + kLinkSlice - 1) / kLinkSlice, 1);
    p.link_part = take(P * p.link_slices * 6 * sizeof(double) + 8);
    // The stream-collide kernels that stage whole rows of 512 nodes take the
    // interpolated values as per-row patches.
    p.patches = P > 0 && c.nx == 512 && c.lattice != LBM_LATTICE_D3Q27;
    if (p.patches) {
      const size_t rows = (size_t)c.ny * (size_t)c.nz;
      p.patch_cnt = take(rows * 4);
      p.patch = take(rows * kPatchCap * (c.store == LBM_STORE_F16S ? 4 : 8));
    }
    p.wl_count = wall_link_count(c);
    p.wl_node = take((size_t)p.wl_count * 4 + 4);
    p.wl_q = take((size_t)p.wl_count * 4 + 4);
    p.wl_meta = take((size_t)p.wl_count + 4);
  }
  if (c.bc == LBM_BC_IBM) {
    uint32_t forcing = 1, full = 1;
    if (P) ibm_support_bounds(c.max_radius, c.ibm_retraction, forcing, full);
    p.fcap = forcing;
    if (ibm_wall(c)) {
      std::vector<double> xm;
      std::vector<uint32_t> wb;
      double dV = 0.0;
      pipe_markers(c, xm, dV);
      p.n_wall = (uint32_t)(xm.size() / 3);
      p.wall_support = pipe_support(c, xm, wb);
    }
    // below 2^31: the forcing slot lists keep a shared-node flag in bit 31
    p.s_cap = (uint32_t)std::min<uint64_t>(std::min<uint64_t>((uint64_t)N, 0x7FFFFFFFull),
                                           (uint64_t)P * full + p.wall_support + 4096);
    p.n_markers = P ? (uint32_t)marker_count(c.max_radius - c.ibm_retraction) : 0;
    p.side = P ? ibm_box_side(c.max_radius, c.ibm_retraction) : 0;
    const size_t rows = (size_t)p.side * p.side;
    for (int b = 0; b < 2; ++b) {
      p.ib_bits[b] = take(words * 4);
      p.ib_rank[b] = take(words * 4);
      p.ib_fib[b] = take((size_t)p.s_cap * 16);
    }
    p.ib_count = take(2 * sizeof(uint32_t));
    p.ib_shared = take(words * 4);
    p.ib_sh_rank = take(words * 4);
    p.ib_sh_count = take(sizeof(uint32_t));
    p.ib_sh_slot = take((size_t)p.s_cap * 4);
    p.ib_sh_acc = take((size_t)3 * p.s_cap * 8);
    p.ib_list = take((size_t)p.s_cap * 4);
    p.ib_us = take((size_t)p.s_cap * 16);
    p.ib_bsum = take((words / 1024 + 2) * 4);
    p.ib_dirs = take((size_t)std::max<uint32_t>(p.n_markers, 1) * 3 * sizeof(double));
    p.ib_rowbits = take(P * rows * 4 + 4);
    p.ib_fcount = take(P * 4 + 4);
    p.ib_fslot = take(P * (size_t)p.fcap * 4 + 4);
    p.ib_pu = take(P * (size_t)p.fcap * 16 + 16);
    p.ib_pf = take(P * (size_t)p.fcap * 16 + 16);
    p.ib_wmark = take((size_t)p.n_wall * 3 * sizeof(double) + 8);
    p.ib_wdF = take((size_t)p.n_wall * 3 * sizeof(float) + 4);
    p.ib_wsup = take(p.n_wall ? words * 4 : 4);
  }
  p.total = off;
  return p;
}

bool rate_ok(double s) { return s > 0.0 && s < 2.0; }

int check_config(const lbm_config* c) {
  if (!c) return LBM_E_ARG;
  if (c->nx < 4 || c->ny < 4 || c->nz < 4) return LBM_E_ARG;
  const double N = (double)c->nx * (double)c->ny * (double)c->nz;
  if (N > 2147483647.0) return LBM_E_SIZE;
  // one direction array must be addressable with a 32-bit byte offset
  if (c->store == LBM_STORE_F32 && N > 1073741824.0) return LBM_E_SIZE;
  if (!(c->tau > 0.5) || !isfinite(c->tau)) return LBM_E_ARG;
  if (!rate_ok(c->s_e) || !rate_ok(c->s_eps) || !rate_ok(c->s_q) || !rate_ok(c->s_pi) || !rate_ok(c->s_m))
    return LBM_E_ARG;
  for (int k = 0; k < 3; ++k)
    if (!isfinite(c->body_force[k])) return LBM_E_ARG;
  if (c->store != LBM_STORE_F32 && c->store != LBM_STORE_F16S) return LBM_E_ARG;
  if (c->bc != LBM_BC_NONE && c->bc != LBM_BC_IBB && c->bc != LBM_BC_IBM) return LBM_E_ARG;
  if (c->bc == LBM_BC_IBM) {
    // A sphere's box (side 2 R_b + 2) must fit a 32-bit row mask.
    if (!(c->ibm_retraction >= 0.0) || c->ibm_retraction > 2.0) return LBM_E_ARG;
    if (c->max_particles > 0) {
      if (!(c->max_radius - c->ibm_retraction > 1.0)) return LBM_E_ARG;
      const int side = ibm_box_side(c->max_radius, c->ibm_retraction);
      // the box must not wrap onto itself
      if (side > 32 || side > std::min(c->nx, std::min(c->ny, c->nz))) return LBM_E_ARG;
    }
  }
  if (c->wall != LBM_WALL_NONE && c->wall != LBM_WALL_PIPE_Z) return LBM_E_ARG;
  if (c->wall == LBM_WALL_PIPE_Z) {
    if (c->bc == LBM_BC_NONE) return LBM_E_ARG;
    if (!(c->pipe_radius > 1.0) || !isfinite(c->pipe_cx) || !isfinite(c->pipe_cy)) return LBM_E_ARG;
  }
  if (c->max_particles < 0 || c->max_particles > (1 << 24)) return LBM_E_ARG;
  // Boundary nodes are stored as packed 11/11/10-bit coordinates.
  if ((c->max_particles > 0 || c->wall != LBM_WALL_NONE) && (c->nx > 2048 || c->ny > 2048 || c->nz > 1024))
    return LBM_E_SIZE;
  if (c->max_radius > 28.0) return LBM_E_ARG;
  if (c->max_particles > 0) {
    if (c->bc == LBM_BC_NONE) return LBM_E_ARG;
    if (!(c->max_radius > 0.0) || 2.0 * c->max_radius + 8.0 > (double)std::min(c->nx, std::min(c->ny, c->nz)))
      return LBM_E_ARG;
  }
  if (c->ibb_max_order != 1 && c->ibb_max_order != 2) return LBM_E_ARG;
  if (c->lattice != LBM_LATTICE_D3Q19 && c->lattice != LBM_LATTICE_D3Q27) return LBM_E_ARG;
  if (c->lattice == LBM_LATTICE_D3Q19 && c->tau_bulk != 0.0) return LBM_E_ARG;
  if (c->lattice == LBM_LATTICE_D3Q27) {
    // the pipe solver: FP32, periodic box or the linear bounce-back pipe wall
    if (c->store != LBM_STORE_F32 || c->max_particles != 0 || c->bc == LBM_BC_IBM) return LBM_E_ARG;
    if (c->bc == LBM_BC_IBB && (c->wall != LBM_WALL_PIPE_Z || c->ibb_max_order != 1)) return LBM_E_ARG;
    if (!(c->tau_bulk == 0.0 || (c->tau_bulk > 0.5 && isfinite(c->tau_bulk)))) return LBM_E_ARG;
  }
  if (c->ibm_iters < 0 || c->ibm_iters > 16) return LBM_E_ARG;
  if (!(c->coll_restitution > 0.0 && c->coll_restitution <= 1.0) || !(c->coll_tc_steps > 0.0)) return LBM_E_ARG;
  return LBM_OK;
}

int hip_status(hipError_t e) { return e == hipSuccess ? LBM_OK : LBM_E_HIP; }

// Reads and clears the latched device error word (waits for the stream).
int drain_errors(Ctx& c) {
  uint32_t bits = 0;
  if (hipMemcpyAsync(&bits, c.err, sizeof(bits), hipMemcpyDeviceToHost, c.stream) != hipSuccess) return LBM_E_HIP;
  if (hipStreamSynchronize(c.stream) != hipSuccess) return LBM_E_HIP;
  if (bits) {
    if (hipMemsetAsync(c.err, 0, sizeof(uint32_t), c.stream) != hipSuccess) return LBM_E_HIP;
    if (bits & kErrUnstable) return LBM_E_UNSTABLE;
    if (bits & kErrOverlap) return LBM_E_OVERLAP;
    if (bits & kErrCapacity) return LBM_E_SIZE;
  }
  return LBM_OK;
}

// Force of the last collision for field extraction: none before the first
// step, the body force afterwards.
float3 extraction_force(const Ctx& c) { return c.step > 0 ? c.body_force : make_float3(0.0f, 0.0f, 0.0f); }

size_t pvec_bytes(const Ctx& c) { return (size_t)std::max(c.np, 0) * 3 * sizeof(double); }

hipError_t zero_particle_accumulators(Ctx& c) {
  const size_t b = pvec_bytes(c);
  if (!b) return hipSuccess;
  double* v[] = {c.P.F_link, c.P.T_link, c.P.F_rc, c.P.T_rc, c.P.F_h, c.P.T_h, c.P.F_c,
                 c.P.F_ib,   c.P.T_ib,   c.P.Iu,   c.P.IL,   c.P.Iu_new, c.P.IL_new};
  for (double* p : v) {
    hipError_t e = hipMemsetAsync(p, 0, b, c.stream);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// Kempe inner momentum of the current fields (step 0: the extraction force is
// zero), the reference for the first step's inner-inertia term.
hipError_t ibm_inner_momentum_init(Ctx& c) {
  if (c.cfg.bc != LBM_BC_IBM || c.np <= 0) return hipSuccess;
  float* ufield = (float*)c.f_nxt;  // idle between steps
  hipError_t e = launch_fields(c, c.f_cur, extraction_force(c), ufield, nullptr);
  if (e == hipSuccess) e = launch_kempe_dense(c, ufield, c.P.X[c.pcur], c.P.Iu, c.P.IL);
  return e;
}

// One immersed-boundary step. The particle stage (Kempe integral and the
// update, which need the forcing result) and the next step's support build
// (which needs the new positions) read nothing the stream-collide kernel
// writes and write nothing it reads (it reads the current support and force
// slots; the build fills the other buffer). With overlap on they run on the
// side stream beside it and the step ends with both streams joined;
// otherwise the particle stage runs before it and the build after it.
hipError_t step_ibm(Ctx& c) {
  const int pc = c.pcur, pn = 1 - c.pcur;
  hipError_t e = timed(c, LBM_K_IBM_PREPASS, [&] { return launch_ibm_prepass(c, c.f_cur); });
  if (e != hipSuccess) return e;
  if (c.np > 0 || c.ibm.n_wall > 0) {
    e = timed(c, LBM_K_IBM_FORCING, [&] { return launch_ibm_forcing_pass(c, c.P.X[pc], c.P.U[pc], c.P.Om[pc]); });
    if (e != hipSuccess) return e;
  }
  const bool moving = c.np > 0 && c.motion != LBM_MOTION_FIXED;
  const bool ov = c.overlap && c.np > 0;
  const int nb = 1 - c.ibm.cur;
  auto particles = [&] {
    return timed(c, LBM_K_PARTICLE, [&] {
      hipError_t q = launch_ibm_kempe(c, c.P.X[pc], c.P.Iu_new, c.P.IL_new);
      if (q == hipSuccess) q = launch_particle_update(c);
      return q;
    });
  };
  auto geometry = [&] {
    return moving ? timed(c, LBM_K_GEOMETRY, [&] { return launch_ibm_support_build(c, nb, c.P.X[pn]); })
                  : hipSuccess;
  };
  if (ov) {
    if ((e = fork_side(c)) != hipSuccess) return e;
    e = on_side(c, [&] {
      hipError_t r = particles();
      return r == hipSuccess ? geometry() : r;
    });
  } else if (c.np > 0) {
    e = particles();
  }
  if (e != hipSuccess) return e;
  e = timed(c, LBM_K_STREAM_COLLIDE, [&] { return launch_stream_collide_ibm(c, c.f_cur, c.f_nxt); });
  if (e != hipSuccess) return e;
  e = ov ? join_side(c) : geometry();
  if (e != hipSuccess) return e;
  c.ibm.last = c.ibm.cur;
  if (c.np > 0) {
    if (moving) c.ibm.cur = nb;
    c.pcur = pn;
  }
  return hipSuccess;
}

// One bounce-back step. The particle update (it needs this step's link
// forces) and the next step's geometry (owner map and links from the new
// positions, into the other owner buffer and the link arrays, which the link
// pass has finished reading) do not touch what the stream-collide kernel
// reads or writes. With overlap on they run on the side stream beside it;
// otherwise after it. The refill needs the collision's output and the new
// geometry, so it comes after both.
hipError_t step_ibb(Ctx& c) {
  const int pc = c.pcur, pn = 1 - c.pcur;
  hipError_t e = timed(c, LBM_K_IBB_LINKS, [&] { return launch_ibb_links(c, c.f_cur, c.P.X[pc], c.P.U[pc], c.P.Om[pc]); });
  if (e != hipSuccess) return e;
  const bool moving = c.np > 0 && c.motion != LBM_MOTION_FIXED;
  const bool ov = c.overlap && c.np > 0;
  const int on = 1 - c.ocur;
  auto particles_and_geometry = [&] {
    hipError_t r = timed(c, LBM_K_PARTICLE, [&] { return launch_particle_update(c); });
    if (r == hipSuccess && moving)
      r = timed(c, LBM_K_GEOMETRY, [&] {
        hipError_t q = launch_owner_clear(c, c.ibb.owner[on], c.P.Xown[on], c.np);
        if (q == hipSuccess) q = launch_owner_set(c, c.ibb.owner[on], c.P.X[pn], c.P.Xown[on]);
        if (q == hipSuccess) q = launch_links_build(c, c.ibb.owner[on], c.P.X[pn]);
        return q;
      });
    return r;
  };
  if (ov) {
    if ((e = fork_side(c)) != hipSuccess) return e;
    if ((e = on_side(c, particles_and_geometry)) != hipSuccess) return e;
  }
  // the link pass listed this step's patches when there are particles
  e = timed(c, LBM_K_STREAM_COLLIDE, [&] { return launch_stream_collide(c, c.f_cur, c.f_nxt, c.np > 0); });
  if (e != hipSuccess) return e;
  if (c.np > 0) {
    e = ov ? join_side(c) : particles_and_geometry();
    if (e != hipSuccess) return e;
    if (moving) {
      e = timed(c, LBM_K_REFILL, [&] {
        return launch_cover_refill(c, c.f_nxt, c.ibb.owner[c.ocur], c.ibb.owner[on], c.P.X[pc], c.P.X[pn],
                                   c.P.U[pn], c.P.Om[pn]);
      });
      if (e != hipSuccess) return e;
      c.ocur = on;
    }
    c.pcur = pn;
  }
  return hipSuccess;
}

}  // namespace

extern "C" {

void lbm_config_default(lbm_config* cfg) {
  if (!cfg) return;
  memset(cfg, 0, sizeof(*cfg));
  cfg->nx = cfg->ny = cfg->nz = 32;
  cfg->tau = 0.6;
  cfg->s_e = 1.19;
  cfg->s_eps = 1.4;
  cfg->s_q = 1.2;
  cfg->s_pi = 1.4;
  cfg->s_m = 1.98;
  cfg->bc = LBM_BC_NONE;
  cfg->ibb_max_order = 2;
  cfg->ibm_retraction = 0.0;
  cfg->ibm_iters = 2;
  cfg->store = LBM_STORE_F32;
  cfg->wall = LBM_WALL_NONE;
  cfg->coll_restitution = 0.97;
  cfg->coll_tc_steps = 8.0;
}

int lbm_workspace_size(const lbm_config* cfg, size_t* bytes) {
  const int st = check_config(cfg);
  if (st != LBM_OK) return st;
  if (!bytes) return LBM_E_ARG;
  *bytes = plan(*cfg).total;
  return LBM_OK;
}

int lbm_init(const lbm_config* cfg, void* workspace, size_t bytes, void* stream, lbm_ctx** out) {
  if (!out) return LBM_E_ARG;
  *out = nullptr;
  const int st = check_config(cfg);
  if (st != LBM_OK) return st;
  if (!workspace || ((uintptr_t)workspace % kAlign) != 0) return LBM_E_ARG;
  const Plan p = plan(*cfg);
  if (bytes < p.total) return LBM_E_SIZE;

  lbm_ctx* h = new (std::nothrow) lbm_ctx();
  if (!h) return LBM_E_ARG;
  Ctx& c = h->c;
  c.cfg = *cfg;
  c.stream = (hipStream_t)stream;
  if (hipGetDevice(&c.device) != hipSuccess || c.side.create() != hipSuccess) {
    delete h;
    return LBM_E_HIP;
  }
  c.dims = make_dims(cfg->nx, cfg->ny, cfg->nz, (uint32_t)pop_elem_bytes(*cfg));
  c.rates.s_nu = (float)(1.0 / cfg->tau);
  c.rates.s_e = (float)cfg->s_e;
  c.rates.s_eps = (float)cfg->s_eps;
  c.rates.s_q = (float)cfg->s_q;
  c.rates.s_pi = (float)cfg->s_pi;
  c.rates.s_m = (float)cfg->s_m;
  c.body_force = make_float3((float)cfg->body_force[0], (float)cfg->body_force[1], (float)cfg->body_force[2]);
  char* base = (char*)workspace;
  c.f_cur = base + p.f_a;
  c.f_nxt = base + p.f_b;
  c.err = (uint32_t*)(base + p.err);
  c.scratch_d = (double*)(base + p.scratch);
  c.stats_part = (double*)(base + p.stats_part);
  c.step = 0;
  c.np = 0;
  c.motion = LBM_MOTION_FREE;
  c.pcur = 0;
  c.ocur = 0;
  c.link_cap = p.link_cap;
  {
    const size_t P = std::max(has_particles(*cfg) ? (size_t)cfg->max_particles : (size_t)0, (size_t)1);
    double* d = (double*)(base + p.pdoubles);
    auto vec = [&]() {
      double* r = d;
      d += 3 * P;
      return r;
    };
    ParticleBufs& B = c.P;
    B.X[0] = vec(); B.X[1] = vec(); B.U[0] = vec(); B.U[1] = vec(); B.Om[0] = vec(); B.Om[1] = vec();
    B.F_link = vec(); B.T_link = vec(); B.F_rc = vec(); B.T_rc = vec(); B.F_h = vec(); B.T_h = vec();
    B.F_c = vec(); B.F_ib = vec(); B.T_ib = vec(); B.Iu = vec(); B.IL = vec(); B.Iu_new = vec();
    B.IL_new = vec(); B.Xown[0] = vec(); B.Xown[1] = vec();
    B.r = d;
    d += P;
    B.rho = d;
    B.cell_head = (uint32_t*)(base + p.cell_head);
    B.cell_next = (uint32_t*)(base + p.cell_next);
    for (int a = 0; a < 3; ++a) B.cells[a] = p.cells[a];
  }
  c.pb = Ctx::PipeBudget{};
  if (cfg->wall == LBM_WALL_PIPE_Z) {
    c.pb.acc = (double*)(base + p.pb_acc);
    c.pb.list = (uint32_t*)(base + p.pb_list);
    c.pb.off = (uint32_t*)(base + p.pb_off);
  }
  c.ibb = IbbBufs{};
  c.ibb.wall_bits = (uint32_t*)(base + p.wall_bits);
  c.ibb.solid_bits = (uint32_t*)(base + p.solid_bits);
  if (cfg->bc != LBM_BC_NONE) {
    c.ibb.owner[0] = (uint32_t*)(base + p.owner[0]);
    c.ibb.owner[1] = (uint32_t*)(base + p.owner[1]);
  }
  c.ibb.patches = false;
  c.ibb.patch_cnt = nullptr;
  c.ibb.patch = nullptr;
  if (cfg->bc == LBM_BC_IBB) {
    if (p.patches) {
      c.ibb.patches = true;
      c.ibb.patch_cnt = (uint32_t*)(base + p.patch_cnt);
      c.ibb.patch = base + p.patch;
    }
    c.ibb.link_node = (uint32_t*)(base + p.link_node);
    c.ibb.link_q = (float*)(base + p.link_q);
    c.ibb.link_meta = (uint8_t*)(base + p.link_meta);
    c.ibb.link_count = (uint32_t*)(base + p.link_count);
    c.ibb.link_part = (double*)(base + p.link_part);
    c.ibb.link_slices = p.link_slices;
    c.ibb.wl_node = (uint32_t*)(base + p.wl_node);
    c.ibb.wl_q = (float*)(base + p.wl_q);
    c.ibb.wl_meta = (uint8_t*)(base + p.wl_meta);
    c.ibb.wl_count = p.wl_count;
  }
  c.ibm = IbmBufs{};
  if (cfg->bc == LBM_BC_IBM) {
    IbmBufs& m = c.ibm;
    for (int b = 0; b < 2; ++b) {
      m.bits[b] = (uint32_t*)(base + p.ib_bits[b]);
      m.rank[b] = (uint32_t*)(base + p.ib_rank[b]);
      m.fib[b] = (float4*)(base + p.ib_fib[b]);
      m.count[b] = (uint32_t*)(base + p.ib_count) + b;
    }
    m.shared = (uint32_t*)(base + p.ib_shared);
    m.sh_rank = (uint32_t*)(base + p.ib_sh_rank);
    m.sh_count = (uint32_t*)(base + p.ib_sh_count);
    m.sh_slot = (uint32_t*)(base + p.ib_sh_slot);
    m.sh_acc = (unsigned long long*)(base + p.ib_sh_acc);
    m.sh_cap = p.s_cap;
    m.list = (uint32_t*)(base + p.ib_list);
    m.us = (float4*)(base + p.ib_us);
    m.block_sums = (uint32_t*)(base + p.ib_bsum);
    m.dirs = (double*)(base + p.ib_dirs);
    m.rowbits = (uint32_t*)(base + p.ib_rowbits);
    m.fcount = (uint32_t*)(base + p.ib_fcount);
    m.fslot = (uint32_t*)(base + p.ib_fslot);
    m.pu = (float4*)(base + p.ib_pu);
    m.pf = (float4*)(base + p.ib_pf);
    m.s_cap = p.s_cap;
    m.fcap = p.fcap;
    m.side = p.side;
    m.R_b = (p.side - 2) / 2;
    m.cur = m.last = 0;
    m.n_wall = p.n_wall;
    m.wmark = (double*)(base + p.ib_wmark);
    m.wdF = (float*)(base + p.ib_wdF);
    m.wsup = (uint32_t*)(base + p.ib_wsup);
    if (has_particles(*cfg)) {
      int lds_max = 0;
      if (hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, c.device) != hipSuccess ||
          ibm_pass_lds_bytes(c) > (size_t)lds_max) {
        delete h;
        return LBM_E_SIZE;
      }
    }
  }

  if (cfg->bc == LBM_BC_IBB && has_particles(*cfg)) {
    int lds_max = 0;
    if (hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, c.device) != hipSuccess ||
        links_build_lds_total(cfg->max_radius) > (size_t)lds_max) {
      delete h;
      return LBM_E_SIZE;
    }
  }

  // Start at rest, density 1: shifted populations are all zero.
  hipError_t e = hipMemsetAsync(c.f_cur, 0, pop_bytes(*cfg), c.stream);
  if (e == hipSuccess) e = hipMemsetAsync(c.err, 0, sizeof(uint32_t), c.stream);
  // Static wall mask.
  const size_t words = mask_words(c.dims.N);
  if (e == hipSuccess) {
    std::vector<uint32_t> wall(words, 0u);
    if (cfg->wall == LBM_WALL_PIPE_Z) {
      for (int z = 0; z < cfg->nz; ++z)
        for (int y = 0; y < cfg->ny; ++y)
          for (int x = 0; x < cfg->nx; ++x)
            if (pipe_solid(*cfg, x, y)) {
              const size_t n = ((size_t)z * cfg->ny + y) * cfg->nx + x;
              wall[n >> 5] |= 1u << (n & 31);
            }
    }
    e = hipMemcpyAsync(c.ibb.wall_bits, wall.data(), words * 4, hipMemcpyHostToDevice, c.stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(c.ibb.solid_bits, wall.data(), words * 4, hipMemcpyHostToDevice, c.stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c.stream);
  }
  if (e == hipSuccess && cfg->bc != LBM_BC_NONE) {
    e = launch_owner_fill(c, c.ibb.owner[0]);
    if (e == hipSuccess) e = launch_owner_fill(c, c.ibb.owner[1]);
  }
  if (e == hipSuccess && cfg->bc == LBM_BC_IBB && c.ibb.wl_count) {
    // Static wall links, filled once.
    uint32_t* counter = (uint32_t*)c.scratch_d;
    e = hipMemsetAsync(counter, 0, sizeof(uint32_t), c.stream);
    if (e == hipSuccess) e = launch_wall_links(c, c.ibb.owner[0], counter, false);
    uint32_t got = 0;
    if (e == hipSuccess) e = hipMemcpyAsync(&got, counter, sizeof(got), hipMemcpyDeviceToHost, c.stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c.stream);
    if (e == hipSuccess && got != c.ibb.wl_count) e = hipErrorUnknown;
  }
  if (e == hipSuccess && has_particles(*cfg)) {
    c.np = 0;
    e = zero_particle_accumulators(c);
  }
  if (e == hipSuccess && cfg->bc == LBM_BC_IBM) {
    // the forcing passes keep these zero between passes
    e = hipMemsetAsync(c.ibm.sh_acc, 0, (size_t)3 * c.ibm.sh_cap * 8, c.stream);
    if (e == hipSuccess) e = hipMemsetAsync(c.ibm.sh_count, 0, sizeof(uint32_t), c.stream);
  }
  if (e == hipSuccess && cfg->bc == LBM_BC_IBM && c.ibm.n_wall == 0) {
    // empty support until particles are set
    for (int b = 0; b < 2 && e == hipSuccess; ++b) {
      e = hipMemsetAsync(c.ibm.bits[b], 0, words * 4, c.stream);
      if (e == hipSuccess) e = hipMemsetAsync(c.ibm.rank[b], 0, words * 4, c.stream);
      if (e == hipSuccess) e = hipMemsetAsync(c.ibm.count[b], 0, sizeof(uint32_t), c.stream);
    }
  }
  std::vector<double> wxm;
  std::vector<uint32_t> wbits;
  if (e == hipSuccess && c.ibm.n_wall) {
    // static pipe-wall markers and their support, in both support buffers
    pipe_markers(*cfg, wxm, c.ibm.wdV);
    (void)pipe_support(*cfg, wxm, wbits);
    e = hipMemcpyAsync(c.ibm.wmark, wxm.data(), wxm.size() * sizeof(double), hipMemcpyHostToDevice, c.stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(c.ibm.wsup, wbits.data(), wbits.size() * 4, hipMemcpyHostToDevice, c.stream);
    for (int b = 0; b < 2 && e == hipSuccess; ++b) e = launch_ibm_support_build(c, b, nullptr);
  }
  if (e == hipSuccess) e = hipStreamSynchronize(c.stream);
  if (e != hipSuccess) {
    delete h;
    return LBM_E_HIP;
  }
  *out = h;
  return LBM_OK;
}

int lbm_set_fields_device(lbm_ctx* h, const float* u_dev, const float* rho_dev) {
  if (!h || !u_dev) return LBM_E_ARG;
  Ctx& c = h->c;
  c.step = 0;
  hipError_t e = launch_init_equilibrium(c, u_dev, rho_dev, c.f_cur);
  if (e == hipSuccess) e = zero_particle_accumulators(c);
  if (e == hipSuccess) e = ibm_inner_momentum_init(c);
  return hip_status(e);
}

int lbm_set_fields(lbm_ctx* h, const float* u, const float* rho) {
  if (!h || !u) return LBM_E_ARG;
  Ctx& c = h->c;
  // Stage through the idle population buffer: it holds no state between
  // steps and is at least 16 bytes per node.
  const size_t N = c.dims.N;
  float* su = (float*)c.f_nxt;
  float* sr = rho ? su + 3 * N : nullptr;
  if (hipMemcpyAsync(su, u, 3 * N * sizeof(float), hipMemcpyHostToDevice, c.stream) != hipSuccess) return LBM_E_HIP;
  if (rho && hipMemcpyAsync(sr, rho, N * sizeof(float), hipMemcpyHostToDevice, c.stream) != hipSuccess)
    return LBM_E_HIP;
  int st = lbm_set_fields_device(h, su, sr);
  if (st != LBM_OK) return st;
  if (hipStreamSynchronize(c.stream) != hipSuccess) return LBM_E_HIP;
  return LBM_OK;
}

extern "C++" {
namespace {
hipError_t ibm_marker_setup(Ctx& c, double r);
}  // namespace
}  // extern "C++"

int lbm_set_particles(lbm_ctx* h, int32_t np, const double* x, const double* u, const double* omega,
                      const double* radius, const double* rho_p, int32_t mode, int32_t motion) {
  if (!h) return LBM_E_ARG;
  Ctx& c = h->c;
  const lbm_config& cfg = c.cfg;
  if (cfg.bc == LBM_BC_NONE || cfg.wall != LBM_WALL_NONE) return LBM_E_ARG;
  if (np < 0 || np > cfg.max_particles) return LBM_E_SIZE;
  if (np > 0 && (!x || !radius)) return LBM_E_ARG;
  if (mode != LBM_SET_STATE && mode != LBM_RELEASE && mode != LBM_SET_RIGID) return LBM_E_ARG;
  if (motion != LBM_MOTION_FREE && motion != LBM_MOTION_FIXED && motion != LBM_MOTION_PRESCRIBED) return LBM_E_ARG;
  const double L[3] = {(double)cfg.nx, (double)cfg.ny, (double)cfg.nz};
  std::vector<double> X(3 * (size_t)np), U(3 * (size_t)np, 0.0), W(3 * (size_t)np, 0.0), R(np), RHO(np, 1.0);
  for (int32_t i = 0; i < np; ++i) {
    const double r = radius[i];
    if (!(r > 0.0) || r > cfg.max_radius) return LBM_E_ARG;
    R[i] = r;
    if (rho_p) {
      if (!(rho_p[i] > 0.0) || !isfinite(rho_p[i])) return LBM_E_ARG;
      RHO[i] = rho_p[i];
    }
    for (int k = 0; k < 3; ++k) {
      double v = x[3 * i + k];
      if (!isfinite(v)) return LBM_E_ARG;
      v = fmod(v, L[k]);
      if (v < 0.0) v += L[k];
      if (v >= L[k]) v -= L[k];
      X[3 * i + k] = v;
      if (u) {
        if (!isfinite(u[3 * i + k])) return LBM_E_ARG;
        U[3 * i + k] = u[3 * i + k];
      }
      if (omega) {
        if (!isfinite(omega[3 * i + k])) return LBM_E_ARG;
        W[3 * i + k] = omega[3 * i + k];
      }
    }
  }
  // The immersed boundary lays out one marker set for all spheres; checked
  // before anything of the context changes, so a rejected call leaves it as
  // it was.
  if (cfg.bc == LBM_BC_IBM && np > 0) {
    for (int32_t i = 1; i < np; ++i)
      if (R[i] != R[0]) return LBM_E_ARG;
    if (!(R[0] - cfg.ibm_retraction > 1.0)) return LBM_E_ARG;
  }
  c.np = np;
  c.motion = motion;
  c.pcur = 0;
  const size_t vb = pvec_bytes(c);
  hipError_t e = hipSuccess;
  if (np > 0) {
    e = hipMemcpyAsync(c.P.X[0], X.data(), vb, hipMemcpyHostToDevice, c.stream);
    if (e == hipSuccess) e = hipMemcpyAsync(c.P.U[0], U.data(), vb, hipMemcpyHostToDevice, c.stream);
    if (e == hipSuccess) e = hipMemcpyAsync(c.P.Om[0], W.data(), vb, hipMemcpyHostToDevice, c.stream);
    if (e == hipSuccess) e = hipMemcpyAsync(c.P.r, R.data(), np * sizeof(double), hipMemcpyHostToDevice, c.stream);
    if (e == hipSuccess) e = hipMemcpyAsync(c.P.rho, RHO.data(), np * sizeof(double), hipMemcpyHostToDevice, c.stream);
  }
  if (e == hipSuccess) e = zero_particle_accumulators(c);
  // Owner map of the new positions (lowest index wins), needed by release
  // and by the bounce-back geometry.
  c.ocur = 0;
  if (e == hipSuccess) e = launch_owner_fill(c, c.ibb.owner[0]);
  if (e == hipSuccess) e = launch_owner_fill(c, c.ibb.owner[1]);
  if (e == hipSuccess) e = launch_owner_set(c, c.ibb.owner[0], c.P.X[0]);
  if (e == hipSuccess && mode == LBM_RELEASE && np > 0) {
    float* ufield = (float*)c.f_nxt;  // idle between steps
    double* U0 = c.P.F_h;             // scratch until the first step
    e = launch_fields(c, c.f_cur, extraction_force(c), ufield, nullptr);
    if (e == hipSuccess) e = launch_release_average(c, ufield, U0);
    if (e == hipSuccess) e = hipMemcpyAsync(c.P.U[0], U0, vb, hipMemcpyDeviceToDevice, c.stream);
    if (e == hipSuccess) e = hipMemsetAsync(c.P.Om[0], 0, vb, c.stream);
    if (e == hipSuccess) e = launch_release_overwrite(c, c.f_cur, c.ibb.owner[0], c.P.U[0], c.P.Om[0]);
    if (e == hipSuccess) e = hipMemsetAsync(c.P.F_h, 0, vb, c.stream);
  }
  if (e == hipSuccess && mode == LBM_SET_RIGID && np > 0)
    e = launch_release_overwrite(c, c.f_cur, c.ibb.owner[0], c.P.U[0], c.P.Om[0]);
  // Both owner maps now hold (at most) the current spheres, so the box
  // positions recorded for each must be valid centres before the first
  // clear: clearing around the current centres in the other map is a no-op.
  if (e == hipSuccess && np > 0) e = hipMemcpyAsync(c.P.Xown[0], c.P.X[0], vb, hipMemcpyDeviceToDevice, c.stream);
  if (e == hipSuccess && np > 0) e = hipMemcpyAsync(c.P.Xown[1], c.P.X[0], vb, hipMemcpyDeviceToDevice, c.stream);
  if (e == hipSuccess && cfg.bc == LBM_BC_IBB) e = launch_links_build(c, c.ibb.owner[0], c.P.X[0]);
  if (e == hipSuccess && cfg.bc == LBM_BC_IBM) {
    IbmBufs& m = c.ibm;
    m.cur = m.last = 0;
    m.n_markers = 0;
    if (np > 0) e = ibm_marker_setup(c, R[0]);
    if (e == hipSuccess) e = launch_ibm_support_build(c, 0, c.P.X[0]);
    if (e == hipSuccess) e = ibm_inner_momentum_init(c);
  }
  if (e != hipSuccess) return LBM_E_HIP;
  return drain_errors(c);
}

extern "C++" {
namespace {

// ---- checkpoint blob ------------------------------------------------------
// Layout (native byte order): StateHeader, the populations of the current
// step (exactly Q N element bytes), the particle block (X, U, Omega, F_rc,
// T_rc, F_h, T_h, F_c, I_u, I_L as [np][3] FP64, then r and rho_p as [np]),
// then, for the immersed boundary after the first step, the support of the
// last collision: bitmask and rank words, and the spread force of its
// slots component by component ([3][count] FP32).
constexpr char kStateMagic[8] = {'L', 'B', 'M', 'S', 'T', 'A', 'T', 'E'};
constexpr uint32_t kStateVersion = 2;
constexpr int kStateVec3 = 10;  // [np][3] arrays in the particle block

struct StateHeader {
  char magic[8];
  uint32_t version, header_bytes;
  lbm_config cfg;      // field by field, padding zeroed
  int64_t step;
  int32_t np, motion;
  uint64_t pop_bytes;  // Q N element bytes
  uint64_t ibm_words;  // support bitmask words saved (0: no support section)
  uint32_t ibm_count;  // slots of the saved support
  uint32_t reserved;
};

lbm_config normalized(const lbm_config& a) {
  lbm_config z;
  memset(&z, 0, sizeof(z));
  z.nx = a.nx; z.ny = a.ny; z.nz = a.nz;
  z.tau = a.tau;
  z.s_e = a.s_e; z.s_eps = a.s_eps; z.s_q = a.s_q; z.s_pi = a.s_pi; z.s_m = a.s_m;
  for (int k = 0; k < 3; ++k) z.body_force[k] = a.body_force[k];
  z.bc = a.bc; z.ibb_max_order = a.ibb_max_order;
  z.ibm_retraction = a.ibm_retraction; z.ibm_iters = a.ibm_iters;
  z.store = a.store; z.wall = a.wall;
  z.pipe_radius = a.pipe_radius; z.pipe_cx = a.pipe_cx; z.pipe_cy = a.pipe_cy;
  z.max_particles = a.max_particles; z.max_radius = a.max_radius;
  z.coll_restitution = a.coll_restitution; z.coll_tc_steps = a.coll_tc_steps;
  z.lattice = a.lattice; z.tau_bulk = a.tau_bulk;
  return z;
}

// The populations in a state blob: the Q arrays of N elements back to back
// (without the pad between the arrays in device memory).
size_t pop_exact_bytes(const lbm_config& c) { return (size_t)lattice_q(c) * n_nodes(c) * pop_elem_bytes(c); }

// Copies the populations between a blob (arrays back to back) and device
// memory (arrays pop_stride apart), one array per copy.
hipError_t copy_pops(const Ctx& c, char* blob, void* dev, bool to_host) {
  const size_t elem = pop_elem_bytes(c.cfg), n = n_nodes(c.cfg) * elem, s = pop_stride(c.cfg) * elem;
  hipError_t e = hipSuccess;
  for (int i = 0; i < lattice_q(c.cfg) && e == hipSuccess; ++i) {
    char* d = (char*)dev + (size_t)i * s;
    e = to_host ? hipMemcpyAsync(blob + (size_t)i * n, d, n, hipMemcpyDeviceToHost, c.stream)
                : hipMemcpyAsync(d, blob + (size_t)i * n, n, hipMemcpyHostToDevice, c.stream);
  }
  return e;
}

size_t particle_block_bytes(int32_t np) { return (size_t)np * (3 * kStateVec3 + 2) * sizeof(double); }

// The immersed boundary saves the support and spread force of the last
// collision, which the velocity extraction of the current step reads.
bool state_has_support(const Ctx& c) { return c.cfg.bc == LBM_BC_IBM && c.step > 0; }

size_t state_bytes(const StateHeader& h) {
  return sizeof(StateHeader) + h.pop_bytes + particle_block_bytes(h.np) + h.ibm_words * 8 +
         (size_t)h.ibm_count * sizeof(float4);
}

int state_header(Ctx& c, StateHeader& h) {
  memset(&h, 0, sizeof(h));
  memcpy(h.magic, kStateMagic, sizeof(h.magic));
  h.version = kStateVersion;
  h.header_bytes = (uint32_t)sizeof(StateHeader);
  h.cfg = normalized(c.cfg);
  h.step = c.step;
  h.np = std::max(c.np, 0);
  h.motion = c.motion;
  h.pop_bytes = pop_exact_bytes(c.cfg);
  if (state_has_support(c)) {
    uint32_t cnt = 0;
    if (hipMemcpyAsync(&cnt, c.ibm.count[c.ibm.last], 4, hipMemcpyDeviceToHost, c.stream) != hipSuccess)
      return LBM_E_HIP;
    const int st = drain_errors(c);
    if (st != LBM_OK) return st;
    h.ibm_words = mask_words(c.dims.N);
    h.ibm_count = std::min(cnt, c.ibm.s_cap);
    return LBM_OK;
  }
  return drain_errors(c);
}

// Particle block arrays in blob order.
void particle_arrays(Ctx& c, double* v[kStateVec3 + 2]) {
  const int pc = c.pcur;
  double* a[kStateVec3 + 2] = {c.P.X[pc], c.P.U[pc], c.P.Om[pc], c.P.F_rc, c.P.T_rc, c.P.F_h,
                               c.P.T_h,   c.P.F_c,   c.P.Iu,     c.P.IL,   c.P.r,    c.P.rho};
  for (int k = 0; k < kStateVec3 + 2; ++k) v[k] = a[k];
}

// Marker layout of the immersed boundary for spheres of radius r.
hipError_t ibm_marker_setup(Ctx& c, double r) {
  IbmBufs& m = c.ibm;
  m.r_l = r - c.cfg.ibm_retraction;
  m.n_markers = marker_count(m.r_l);
  m.dV = marker_volume(m.r_l, m.n_markers);
  std::vector<double> dirs;
  fibonacci_dirs(m.n_markers, dirs);
  hipError_t e =
      hipMemcpyAsync(m.dirs, dirs.data(), dirs.size() * sizeof(double), hipMemcpyHostToDevice, c.stream);
  // the host vector must outlive the copy
  if (e == hipSuccess) e = hipStreamSynchronize(c.stream);
  return e;
}

}  // namespace
}  // extern "C++"

int lbm_state_size(lbm_ctx* h, size_t* bytes) {
  if (!h || !bytes) return LBM_E_ARG;
  StateHeader hd;
  const int st = state_header(h->c, hd);
  if (st != LBM_OK) return st;
  *bytes = state_bytes(hd);
  return LBM_OK;
}

int lbm_get_state(lbm_ctx* h, void* host, size_t bytes) {
  if (!h || !host) return LBM_E_ARG;
  Ctx& c = h->c;
  StateHeader hd;
  int st = state_header(c, hd);
  if (st != LBM_OK) return st;
  if (bytes < state_bytes(hd)) return LBM_E_SIZE;
  char* out = (char*)host;
  memcpy(out, &hd, sizeof(hd));
  size_t off = sizeof(hd);
  hipError_t e = copy_pops(c, out + off, c.f_cur, true);
  off += hd.pop_bytes;
  double* v[kStateVec3 + 2];
  particle_arrays(c, v);
  const size_t vb = (size_t)hd.np * 3 * sizeof(double), sb = (size_t)hd.np * sizeof(double);
  for (int k = 0; k < kStateVec3 + 2 && e == hipSuccess; ++k) {
    const size_t b = k < kStateVec3 ? vb : sb;
    if (b) e = hipMemcpyAsync(out + off, v[k], b, hipMemcpyDeviceToHost, c.stream);
    off += b;
  }
  if (e == hipSuccess && hd.ibm_words) {
    const IbmBufs& m = c.ibm;
    const int b = m.last;
    e = hipMemcpyAsync(out + off, m.bits[b], hd.ibm_words * 4, hipMemcpyDeviceToHost, c.stream);
    off += hd.ibm_words * 4;
    if (e == hipSuccess) e = hipMemcpyAsync(out + off, m.rank[b], hd.ibm_words * 4, hipMemcpyDeviceToHost, c.stream);
    off += hd.ibm_words * 4;
    if (e == hipSuccess && hd.ibm_count)
      e = hipMemcpyAsync(out + off, m.fib[b], (size_t)hd.ibm_count * sizeof(float4), hipMemcpyDeviceToHost,
                         c.stream);
    off += (size_t)hd.ibm_count * sizeof(float4);
  }
  if (e != hipSuccess) return LBM_E_HIP;
  return drain_errors(c);
}

int lbm_set_state(lbm_ctx* h, const void* host, size_t bytes) {
  if (!h || !host || bytes < sizeof(StateHeader)) return LBM_E_ARG;
  Ctx& c = h->c;
  const lbm_config& cfg = c.cfg;
  StateHeader hd;
  memcpy(&hd, host, sizeof(hd));
  if (memcmp(hd.magic, kStateMagic, sizeof(hd.magic)) != 0 || hd.version != kStateVersion ||
      hd.header_bytes != sizeof(StateHeader))
    return LBM_E_ARG;
  const lbm_config want = normalized(cfg);
  if (memcmp(&hd.cfg, &want, sizeof(want)) != 0) return LBM_E_ARG;
  if (hd.step < 0 || hd.np < 0 || hd.np > (has_particles(cfg) ? cfg.max_particles : 0)) return LBM_E_ARG;
  if (hd.motion != LBM_MOTION_FREE && hd.motion != LBM_MOTION_FIXED && hd.motion != LBM_MOTION_PRESCRIBED)
    return LBM_E_ARG;
  if (hd.pop_bytes != pop_exact_bytes(cfg)) return LBM_E_ARG;
  const bool support = cfg.bc == LBM_BC_IBM && hd.step > 0;
  if (support ? (hd.ibm_words != mask_words(c.dims.N) || hd.ibm_count > c.ibm.s_cap)
              : (hd.ibm_words != 0 || hd.ibm_count != 0))
    return LBM_E_ARG;
  if (bytes < state_bytes(hd)) return LBM_E_SIZE;
  const char* in = (const char*)host;
  // the particle block is checked like lbm_set_particles' arguments
  const int32_t np = hd.np;
  const double* pb = (const double*)(in + sizeof(hd) + hd.pop_bytes);
  std::vector<double> blk((size_t)np * (3 * kStateVec3 + 2));
  if (np) memcpy(blk.data(), pb, blk.size() * sizeof(double));
  const double L[3] = {(double)cfg.nx, (double)cfg.ny, (double)cfg.nz};
  const double* Xb = blk.data();
  const double* Rb = blk.data() + (size_t)np * 3 * kStateVec3;
  for (size_t i = 0; i < (size_t)np * 3 * kStateVec3; ++i)
    if (!isfinite(blk[i])) return LBM_E_ARG;
  for (int32_t i = 0; i < np; ++i) {
    const double r = Rb[i], rho = Rb[np + i];
    if (!(r > 0.0) || r > cfg.max_radius || !(rho > 0.0) || !isfinite(rho)) return LBM_E_ARG;
    for (int k = 0; k < 3; ++k)
      if (!(Xb[3 * i + k] >= 0.0 && Xb[3 * i + k] < L[k])) return LBM_E_ARG;
    if (cfg.bc == LBM_BC_IBM && r != Rb[0]) return LBM_E_ARG;
  }
  if (cfg.bc == LBM_BC_IBM && np > 0 && !(Rb[0] - cfg.ibm_retraction > 1.0)) return LBM_E_ARG;

  // Restore: populations, particle state, then the geometry of the centres
  // (built as the step builds it) and the last collision's support.
  c.step = hd.step;
  c.np = np;
  c.motion = hd.motion;
  c.pcur = 0;
  c.ocur = 0;
  size_t off = sizeof(hd);
  hipError_t e = copy_pops(c, (char*)in + off, c.f_cur, false);
  off += hd.pop_bytes;
  if (e == hipSuccess && has_particles(cfg)) e = zero_particle_accumulators(c);
  double* v[kStateVec3 + 2];
  particle_arrays(c, v);
  const size_t vb = (size_t)np * 3 * sizeof(double), sb = (size_t)np * sizeof(double);
  for (int k = 0; k < kStateVec3 + 2 && e == hipSuccess; ++k) {
    const size_t b = k < kStateVec3 ? vb : sb;
    if (b) e = hipMemcpyAsync(v[k], in + off, b, hipMemcpyHostToDevice, c.stream);
    off += b;
  }
  if (cfg.bc != LBM_BC_NONE && cfg.wall == LBM_WALL_NONE) {
    if (e == hipSuccess) e = launch_owner_fill(c, c.ibb.owner[0]);
    if (e == hipSuccess) e = launch_owner_fill(c, c.ibb.owner[1]);
    if (e == hipSuccess) e = launch_owner_set(c, c.ibb.owner[0], c.P.X[0]);
    if (e == hipSuccess && np > 0) e = hipMemcpyAsync(c.P.Xown[0], c.P.X[0], vb, hipMemcpyDeviceToDevice, c.stream);
    if (e == hipSuccess && np > 0) e = hipMemcpyAsync(c.P.Xown[1], c.P.X[0], vb, hipMemcpyDeviceToDevice, c.stream);
    if (e == hipSuccess && cfg.bc == LBM_BC_IBB) e = launch_links_build(c, c.ibb.owner[0], c.P.X[0]);
  }
  if (e == hipSuccess && cfg.bc == LBM_BC_IBM) {
    IbmBufs& m = c.ibm;
    m.cur = m.last = 0;
    if (cfg.wall == LBM_WALL_NONE) {
      m.n_markers = 0;
      if (np > 0) e = ibm_marker_setup(c, Rb[0]);
      if (e == hipSuccess) e = launch_ibm_support_build(c, 0, c.P.X[0]);
    }
    if (e == hipSuccess && support) {
      const size_t wb = hd.ibm_words * 4;
      e = hipMemcpyAsync(m.bits[1], in + off, wb, hipMemcpyHostToDevice, c.stream);
      off += wb;
      if (e == hipSuccess) e = hipMemcpyAsync(m.rank[1], in + off, wb, hipMemcpyHostToDevice, c.stream);
      off += wb;
      if (e == hipSuccess) e = hipMemcpyAsync(m.count[1], &hd.ibm_count, 4, hipMemcpyHostToDevice, c.stream);
      if (e == hipSuccess && hd.ibm_count)
        e = hipMemcpyAsync(m.fib[1], in + off, (size_t)hd.ibm_count * sizeof(float4), hipMemcpyHostToDevice,
                           c.stream);
      off += (size_t)hd.ibm_count * sizeof(float4);
      m.last = 1;
    }
  }
  if (e == hipSuccess) e = hipStreamSynchronize(c.stream);
  if (e != hipSuccess) return LBM_E_HIP;
  return drain_errors(c);
}

int lbm_particle_count(const lbm_ctx* h, int32_t* np) {
  if (!h || !np) return LBM_E_ARG;
  *np = std::max(h->c.np, 0);
  return LBM_OK;
}

int lbm_get_particles(lbm_ctx* h, double* x, double* u, double* omega) {
  if (!h) return LBM_E_ARG;
  Ctx& c = h->c;
  const size_t vb = pvec_bytes(c);
  if (vb) {
    if (x && hipMemcpyAsync(x, c.P.X[c.pcur], vb, hipMemcpyDeviceToHost, c.stream) != hipSuccess) return LBM_E_HIP;
    if (u && hipMemcpyAsync(u, c.P.U[c.pcur], vb, hipMemcpyDeviceToHost, c.stream) != hipSuccess) return LBM_E_HIP;
    if (omega && hipMemcpyAsync(omega, c.P.Om[c.pcur], vb, hipMemcpyDeviceToHost, c.stream) != hipSuccess)
      return LBM_E_HIP;
  }
  return drain_errors(c);
}

int lbm_forces(lbm_ctx* h, double* F, double* T, double* F_contact) {
  if (!h) return LBM_E_ARG;
  Ctx& c = h->c;
  const size_t vb = pvec_bytes(c);
  if (vb) {
    if (F && hipMemcpyAsync(F, c.P.F_h, vb, hipMemcpyDeviceToHost, c.stream) != hipSuccess) return LBM_E_HIP;
    if (T && hipMemcpyAsync(T, c.P.T_h, vb, hipMemcpyDeviceToHost, c.stream) != hipSuccess) return LBM_E_HIP;
    if (F_contact && hipMemcpyAsync(F_contact, c.P.F_c, vb, hipMemcpyDeviceToHost, c.stream) != hipSuccess)
      return LBM_E_HIP;
  }
  return drain_errors(c);
}

int lbm_link_count(lbm_ctx* h, int64_t* n) {
  if (!h || !n) return LBM_E_ARG;
  Ctx& c = h->c;
  *n = 0;
  if (c.cfg.bc != LBM_BC_IBB) return drain_errors(c);
  std::vector<uint32_t> cnt(std::max(c.np, 0));
  if (c.np > 0 && hipMemcpyAsync(cnt.data(), c.ibb.link_count, c.np * sizeof(uint32_t), hipMemcpyDeviceToHost,
                                 c.stream) != hipSuccess)
    return LBM_E_HIP;
  const int st = drain_errors(c);
  int64_t t = c.ibb.wl_count;
  for (uint32_t v : cnt) t += v;
  *n = t;
  return st;
}

int lbm_get_links(lbm_ctx* h, int64_t cap, int32_t* node, int32_t* dir, int32_t* particle, float* q, int32_t* scheme,
                  int64_t* n) {
  if (!h || !n || cap < 0) return LBM_E_ARG;
  Ctx& c = h->c;
  *n = 0;
  if (c.cfg.bc != LBM_BC_IBB) return drain_errors(c);
  const size_t tot = (size_t)std::max(c.np, 0) * c.link_cap;
  std::vector<uint32_t> cnt(std::max(c.np, 0)), nd(tot), wn(c.ibb.wl_count);
  std::vector<float> qq(tot), wq(c.ibb.wl_count);
  std::vector<uint8_t> mm(tot), wm(c.ibb.wl_count);
  hipError_t e = hipSuccess;
  if (c.np > 0) {
    e = hipMemcpyAsync(cnt.data(), c.ibb.link_count, c.np * 4, hipMemcpyDeviceToHost, c.stream);
    if (e == hipSuccess) e = hipMemcpyAsync(nd.data(), c.ibb.link_node, tot * 4, hipMemcpyDeviceToHost, c.stream);
    if (e == hipSuccess) e = hipMemcpyAsync(qq.data(), c.ibb.link_q, tot * 4, hipMemcpyDeviceToHost, c.stream);
    if (e == hipSuccess) e = hipMemcpyAsync(mm.data(), c.ibb.link_meta, tot, hipMemcpyDeviceToHost, c.stream);
  }
  if (e == hipSuccess && c.ibb.wl_count) {
    e = hipMemcpyAsync(wn.data(), c.ibb.wl_node, wn.size() * 4, hipMemcpyDeviceToHost, c.stream);
    if (e == hipSuccess) e = hipMemcpyAsync(wq.data(), c.ibb.wl_q, wq.size() * 4, hipMemcpyDeviceToHost, c.stream);
    if (e == hipSuccess) e = hipMemcpyAsync(wm.data(), c.ibb.wl_meta, wm.size(), hipMemcpyDeviceToHost, c.stream);
  }
  if (e != hipSuccess) return LBM_E_HIP;
  const int st = drain_errors(c);
  if (st != LBM_OK) return st;
  int64_t k = 0;
  auto emit = [&](uint32_t nn, float qv, uint8_t meta, int32_t p) {
    if (k >= cap) return;
    const int a = meta & 31;
    // packed coordinates x | y << 11 | z << 22
    const int x = (int)(nn & 2047u), y = (int)((nn >> 11) & 2047u), z = (int)(nn >> 22);
    if (node) {
      node[3 * k] = x;
      node[3 * k + 1] = y;
      node[3 * k + 2] = z;
    }
    if (dir) {
      const bool l27 = lattice27(c);
      dir[3 * k] = l27 ? q27::cx(a) : cx_of(a);
      dir[3 * k + 1] = l27 ? q27::cy(a) : cy_of(a);
      dir[3 * k + 2] = l27 ? q27::cz(a) : cz_of(a);
    }
    if (particle) particle[k] = p;
    if (q) q[k] = qv;
    if (scheme) scheme[k] = meta >> 5;
    ++k;
  };
  for (int32_t p = 0; p < c.np; ++p)
    for (uint32_t j = 0; j < std::min(cnt[p], c.link_cap); ++j) {
      const size_t o = (size_t)p * c.link_cap + j;
      emit(nd[o], qq[o], mm[o], p);
    }
  for (uint32_t j = 0; j < c.ibb.wl_count; ++j) emit(wn[j], wq[j], wm[j], -1);
  *n = k;
  return LBM_OK;
}

int lbm_geometry_counts(lbm_ctx* h, int64_t* solid_nodes, int64_t* links) {
  if (!h) return LBM_E_ARG;
  Ctx& c = h->c;
  if (solid_nodes) {
    *solid_nodes = 0;
    if (c.cfg.bc == LBM_BC_IBB) {
      unsigned long long* cnt = (unsigned long long*)c.scratch_d;
      unsigned long long s = 0;
      hipError_t e = hipMemsetAsync(cnt, 0, sizeof(s), c.stream);
      if (e == hipSuccess) e = launch_count_solid(c, c.ibb.owner[c.ocur], cnt);
      if (e == hipSuccess) e = hipMemcpyAsync(&s, cnt, sizeof(s), hipMemcpyDeviceToHost, c.stream);
      if (e != hipSuccess) return LBM_E_HIP;
      const int st = drain_errors(c);
      if (st != LBM_OK) return st;
      *solid_nodes = (int64_t)s;
    }
  }
  if (links) return lbm_link_count(h, links);
  return drain_errors(c);
}

int lbm_ibm_support(lbm_ctx* h, int64_t* support_nodes, int64_t* shared_nodes) {
  if (!h) return LBM_E_ARG;
  Ctx& c = h->c;
  uint32_t v[2] = {0, 0};
  if (c.cfg.bc == LBM_BC_IBM) {
    if (hipMemcpyAsync(&v[0], c.ibm.count[c.ibm.cur], 4, hipMemcpyDeviceToHost, c.stream) != hipSuccess)
      return LBM_E_HIP;
    if (c.np > 0 && hipMemcpyAsync(&v[1], c.ibm.sh_count, 4, hipMemcpyDeviceToHost, c.stream) != hipSuccess)
      return LBM_E_HIP;
  }
  const int st = drain_errors(c);
  if (st != LBM_OK) return st;
  if (support_nodes) *support_nodes = v[0];
  if (shared_nodes) *shared_nodes = v[1];
  return LBM_OK;
}

int lbm_step(lbm_ctx* h, int32_t nsteps) {
  if (!h || nsteps < 0) return LBM_E_ARG;
  Ctx& c = h->c;
  for (int32_t s = 0; s < nsteps; ++s) {
    hipError_t e;
    if (c.cfg.bc == LBM_BC_IBB)
      e = step_ibb(c);
    else if (c.cfg.bc == LBM_BC_IBM)
      e = step_ibm(c);
    else
      e = timed(c, LBM_K_STREAM_COLLIDE, [&] { return launch_stream_collide(c, c.f_cur, c.f_nxt); });
    if (e != hipSuccess) return LBM_E_HIP;
    void* t = c.f_cur;
    c.f_cur = c.f_nxt;
    c.f_nxt = t;
    ++c.step;
  }
  return LBM_OK;
}

int lbm_get_fields_device(lbm_ctx* h, float* u_dev, float* rho_dev) {
  if (!h) return LBM_E_ARG;
  Ctx& c = h->c;
  if (c.cfg.bc == LBM_BC_IBM && c.step > 0)
    return hip_status(launch_fields_ibm(c, c.f_cur, c.ibm.last, u_dev, rho_dev));
  return hip_status(launch_fields(c, c.f_cur, extraction_force(c), u_dev, rho_dev));
}

int lbm_get_fields(lbm_ctx* h, float* u, float* rho) {
  if (!h) return LBM_E_ARG;
  Ctx& c = h->c;
  const size_t N = c.dims.N;
  float* su = (float*)c.f_nxt;
  float* sr = su + 3 * N;
  int st = lbm_get_fields_device(h, u ? su : nullptr, rho ? sr : nullptr);
  if (st != LBM_OK) return st;
  if (u && hipMemcpyAsync(u, su, 3 * N * sizeof(float), hipMemcpyDeviceToHost, c.stream) != hipSuccess)
    return LBM_E_HIP;
  if (rho && hipMemcpyAsync(rho, sr, N * sizeof(float), hipMemcpyDeviceToHost, c.stream) != hipSuccess)
    return LBM_E_HIP;
  return drain_errors(c);
}

extern "C++" {
namespace {

// Statistics and corrector scratch in the idle population buffer (at least
// 38 bytes per node): u [3][N], rho [N], node keys [N], three bitmasks, the
// bitmask rank and scan sums, counters, the sphere of each cell [N], then the
// cell and sphere lists.
struct Scratch {
  float* u;
  float* rho;
  uint32_t* key;
  CorrBufs cb;
  uint32_t* list;
  uint32_t* plist;
  uint32_t cap;
};

Scratch scratch_layout(const Ctx& c) {
  const size_t N = c.dims.N;
  const size_t words = mask_words(c.dims.N);
  char* base = (char*)c.f_nxt;
  size_t off = 0;
  auto take = [&](size_t b) {
    char* p = base + off;
    off += align_up(b);
    return p;
  };
  Scratch s{};
  s.u = (float*)take(3 * N * 4);
  s.rho = (float*)take(N * 4);
  s.key = (uint32_t*)take(N * 4);
  s.cb.once = (uint32_t*)take(3 * words * 4);
  s.cb.twice = s.cb.once + words;
  s.cb.cellbits = s.cb.twice + words;
  s.cb.rank = (uint32_t*)take(words * 4);
  s.cb.bsums = (uint32_t*)take(bits_compact_scratch_words((uint32_t)words) * 4);
  s.cb.count = (uint32_t*)take(4);
  s.cb.err = (uint32_t*)take(4);
  s.cb.cellp = (uint32_t*)take(N * 4);
  const size_t total = pop_bytes(c.cfg);
  const size_t left = total > off + 2 * kAlign ? total - off - 2 * kAlign : 0;
  s.cap = (uint32_t)std::min<size_t>(N, left / 8);
  s.list = (uint32_t*)take((size_t)s.cap * 4);
  s.plist = (uint32_t*)take((size_t)s.cap * 4);
  return s;
}

// The exclusion zone of every sphere must fit in the lattice once.
bool corrector_fits(const Ctx& c) {
  const double re = (c.cfg.max_radius - c.cfg.ibm_retraction) + 2.0 + 1.7320508075688772;
  const double side = 2.0 * re + 3.0;
  return side <= (double)c.dims.nx && side <= (double)c.dims.ny && side <= (double)c.dims.nz;
}

}  // namespace
}  // extern "C++"

int lbm_stats(lbm_ctx* h, int32_t nbins, double bin_width, lbm_stats_t* out, double* hist) {
  if (!h || !out || nbins < 0 || nbins > LBM_STATS_MAX_BINS || !(bin_width > 0.0)) return LBM_E_ARG;
  Ctx& c = h->c;
  const size_t N = c.dims.N;
  const Scratch sc = scratch_layout(c);
  float* su = sc.u;
  float* sr = sc.rho;
  uint32_t* key = sc.key;
  int st = lbm_get_fields_device(h, su, sr);
  if (st != LBM_OK) return st;
  const int pc = c.pcur;
  double* part = c.stats_part;
  double* dout = part + (size_t)kStatGrid * kStatStride;
  double* cout = dout + kStatStride;
  hipError_t e = timed(c, LBM_K_STATS, [&] {
    return launch_stats(c, su, sr, key, nbins, bin_width, c.P.X[pc], c.P.U[pc], c.P.Om[pc], part, dout);
  });
  if (e != hipSuccess) return LBM_E_HIP;
  const bool corr = c.corr_theta && c.np > 0;
  if (corr) {
    if (!corrector_fits(c)) return LBM_E_SIZE;
    e = timed(c, LBM_K_CORRECTOR, [&] {
      hipError_t r = launch_corrector_cells(c, c.P.X[pc], c.corr_dmin, c.corr_dmax, sc.cb, sc.list, sc.plist, sc.cap);
      if (r != hipSuccess) return r;
      return launch_corrector_stats(c, c.corr_theta, su, key, sc.list, sc.plist, sc.cb.count, sc.cap, c.P.X[pc],
                                    c.P.U[pc], c.P.Om[pc], c.corr_urms, nbins, part, cout);
    });
    if (e != hipSuccess) return LBM_E_HIP;
  }
  std::vector<double> v((size_t)kStatScalars + 5 * (size_t)nbins), cv(2 + (size_t)nbins, 0.0);
  uint32_t ncells = 0;
  if (hipMemcpyAsync(v.data(), dout, v.size() * sizeof(double), hipMemcpyDeviceToHost, c.stream) != hipSuccess)
    return LBM_E_HIP;
  if (corr && (hipMemcpyAsync(cv.data(), cout, cv.size() * sizeof(double), hipMemcpyDeviceToHost, c.stream) !=
                   hipSuccess ||
               hipMemcpyAsync(&ncells, sc.cb.count, 4, hipMemcpyDeviceToHost, c.stream) != hipSuccess))
    return LBM_E_HIP;
  const size_t np = (size_t)std::max(c.np, 0);
  std::vector<double> U(3 * np), Om(3 * np), r(np), rp(np);
  if (np) {
    if (hipMemcpyAsync(U.data(), c.P.U[pc], 3 * np * 8, hipMemcpyDeviceToHost, c.stream) != hipSuccess ||
        hipMemcpyAsync(Om.data(), c.P.Om[pc], 3 * np * 8, hipMemcpyDeviceToHost, c.stream) != hipSuccess ||
        hipMemcpyAsync(r.data(), c.P.r, np * 8, hipMemcpyDeviceToHost, c.stream) != hipSuccess ||
        hipMemcpyAsync(rp.data(), c.P.rho, np * 8, hipMemcpyDeviceToHost, c.stream) != hipSuccess)
      return LBM_E_HIP;
  }
  st = drain_errors(c);
  if (st != LBM_OK) return st;
  const double Nd = (double)N, nf = v[kStatNf], nfd = nf > 0.0 ? nf : 1.0;
  lbm_stats_t o{};
  o.step = c.step;
  o.n_nodes = (int64_t)N;
  o.n_fluid = (int64_t)nf;
  o.mass = v[kStatMass];
  o.momentum[0] = v[kStatMomX];
  o.momentum[1] = v[kStatMomY];
  o.momentum[2] = v[kStatMomZ];
  o.ke_raw = v[kStatKeRaw] / Nd;
  o.ke_masked = v[kStatKeMasked] / Nd;
  o.ke_fluid = v[kStatKeFluid] / nfd;
  o.eps_raw = v[kStatEpsRaw] / Nd;
  o.eps_masked = v[kStatEpsMasked] / Nd;
  o.eps_fluid = v[kStatEpsFluid] / nfd;
  o.umax = sqrt(v[kStatUmax2]);
  o.bulk_u = v[kStatBulk] / nfd;
  for (size_t p = 0; p < np; ++p) {
    const double m = rp[p] * (4.0 / 3.0) * M_PI * r[p] * r[p] * r[p];
    const double I = 0.4 * m * r[p] * r[p];
    double u2 = 0.0, w2 = 0.0;
    for (int k = 0; k < 3; ++k) {
      u2 += U[3 * p + k] * U[3 * p + k];
      w2 += Om[3 * p + k] * Om[3 * p + k];
    }
    o.particle_ke += 0.5 * m * u2;
    o.particle_ke_rot += 0.5 * I * w2;
  }
  if (corr && ncells > sc.cap) return LBM_E_SIZE;
  o.eps_fluid_corrected = (v[kStatEpsFluid] + cv[0]) / nfd;
  o.n_corrected = (int64_t)cv[1];
  *out = o;
  if (hist && nbins > 0) {
    std::copy(v.begin() + kStatScalars, v.end(), hist);
    for (int b = 0; b < nbins; ++b) hist[5 * (size_t)nbins + b] = hist[2 * (size_t)nbins + b] + cv[2 + b];
  }
  return LBM_OK;
}

int lbm_corrector_set(lbm_ctx* h, const float* params_dev, double d_min, double d_max, double u_rms) {
  if (!h) return LBM_E_ARG;
  Ctx& c = h->c;
  if (!params_dev) {
    c.corr_theta = nullptr;
    return LBM_OK;
  }
  if (!(u_rms > 0.0) || !(d_max >= d_min)) return LBM_E_ARG;
  if (!corrector_fits(c)) return LBM_E_SIZE;
  c.corr_theta = params_dev;
  c.corr_dmin = d_min;
  c.corr_dmax = d_max;
  c.corr_urms = u_rms;
  return LBM_OK;
}

int lbm_corrector_cells(lbm_ctx* h, double d_min, double d_max, double u_rms, int64_t cap, int32_t* node_dev,
                        int32_t* particle_dev, uint16_t* x_dev, int64_t* n) {
  if (!h || !n || cap < 0 || cap > (int64_t)UINT32_MAX || !(u_rms > 0.0) || !(d_max >= d_min)) return LBM_E_ARG;
  if (cap > 0 && (!node_dev || !particle_dev)) return LBM_E_ARG;
  if (x_dev && ((uintptr_t)x_dev % 16)) return LBM_E_ARG;
  Ctx& c = h->c;
  *n = 0;
  if (!corrector_fits(c)) return LBM_E_SIZE;
  const Scratch sc = scratch_layout(c);
  int st = lbm_get_fields_device(h, sc.u, nullptr);
  if (st != LBM_OK) return st;
  const int pc = c.pcur;
  const uint32_t ucap = (uint32_t)cap;
  hipError_t e = launch_corrector_cells(c, c.P.X[pc], d_min, d_max, sc.cb, (uint32_t*)node_dev,
                                        (uint32_t*)particle_dev, ucap);
  if (e == hipSuccess && x_dev)
    e = launch_corrector_features(c, sc.u, (const uint32_t*)node_dev, (const uint32_t*)particle_dev, sc.cb.count,
                                  ucap, c.P.X[pc], c.P.U[pc], c.P.Om[pc], u_rms, x_dev);
  if (e != hipSuccess) return LBM_E_HIP;
  uint32_t count = 0;
  if (hipMemcpyAsync(&count, sc.cb.count, 4, hipMemcpyDeviceToHost, c.stream) != hipSuccess) return LBM_E_HIP;
  st = drain_errors(c);
  if (st != LBM_OK) return st;
  *n = count;
  return count > ucap ? LBM_E_SIZE : LBM_OK;
}

int lbm_corrector_labels(lbm_ctx* h, const int32_t* node_dev, int64_t n, double u_rms, int32_t subtract,
                         float* t_dev) {
  if (!h || n < 0 || n > (int64_t)UINT32_MAX || !(u_rms > 0.0) || (n > 0 && (!node_dev || !t_dev))) return LBM_E_ARG;
  Ctx& c = h->c;
  const Scratch sc = scratch_layout(c);
  int st = lbm_get_fields_device(h, sc.u, nullptr);
  if (st != LBM_OK) return st;
  const int pc = c.pcur;
  hipError_t e = launch_stats_keys(c, sc.key, 0, 1.0, c.P.X[pc]);
  if (e == hipSuccess)
    e = launch_corrector_labels(c, sc.u, sc.key, (const uint32_t*)node_dev, (uint32_t)n, c.P.X[pc], c.P.U[pc],
                                c.P.Om[pc], u_rms, subtract != 0, t_dev);
  if (e != hipSuccess) return LBM_E_HIP;
  return drain_errors(c);
}

int lbm_spectrum(lbm_ctx* h, int32_t masked, int32_t kmax, double* E, double* D) {
  if (!h || !E || kmax < 0 || kmax > LBM_SPECTRUM_MAX_SHELL) return LBM_E_ARG;
  Ctx& c = h->c;
  if (!spectrum_supported(c)) return LBM_E_ARG;
  const size_t N = c.dims.N;
  const size_t rows = spectrum_lines(c), rowlen = spectrum_row_len(c);
  // Idle population buffer: [Z1 | Z2], then [u | key]; the per-line shell
  // partials overwrite u and key once the fields are packed.
  char* base = (char*)c.f_nxt;
  float2* Z1 = (float2*)base;
  float2* Z2 = Z1 + N;
  char* second = base + align_up(2 * N * sizeof(float2));
  float* u = (float*)second;
  uint32_t* key = (uint32_t*)(second + align_up(3 * N * sizeof(float)));
  double* P = (double*)second;
  int* smin = (int*)(second + align_up(rows * rowlen * sizeof(double)));
  int* cnt = (int*)((char*)smin + align_up(rows * sizeof(int)));
  const size_t need_a = align_up(3 * N * sizeof(float)) + align_up(N * sizeof(uint32_t));
  const size_t need_b = align_up(rows * rowlen * sizeof(double)) + 2 * align_up(rows * sizeof(int));
  if (align_up(2 * N * sizeof(float2)) + std::max(need_a, need_b) > pop_bytes(c.cfg)) return LBM_E_SIZE;
  // E, D and the per-shell partials on the device in the statistics partials
  double* Ed = c.stats_part;
  double* Dd = Ed + (kmax + 1);
  double* part = Dd + (kmax + 1);
  int st = lbm_get_fields_device(h, u, nullptr);
  if (st != LBM_OK) return st;
  const int pc = c.pcur;
  hipError_t e = timed(c, LBM_K_STATS, [&] {
    hipError_t r = masked ? launch_stats_keys(c, key, 0, 1.0, c.P.X[pc]) : hipSuccess;
    if (r == hipSuccess) r = launch_spec_pack(c, u, key, masked, Z1, Z2);
    if (r == hipSuccess) r = launch_fft_xy(c, Z1);
    if (r == hipSuccess) r = launch_fft_xy(c, Z2);
    if (r == hipSuccess)
      r = launch_spec_zbins(c, Z1, Z2, P, smin, cnt, kmax, (c.cfg.tau - 0.5) / 3.0, part, Ed, Dd);
    return r;
  });
  if (e != hipSuccess) return LBM_E_HIP;
  const size_t bytes = (size_t)(kmax + 1) * sizeof(double);
  if (hipMemcpyAsync(E, Ed, bytes, hipMemcpyDeviceToHost, c.stream) != hipSuccess) return LBM_E_HIP;
  if (D && hipMemcpyAsync(D, Dd, bytes, hipMemcpyDeviceToHost, c.stream) != hipSuccess) return LBM_E_HIP;
  return drain_errors(c);
}

int lbm_pipe_budget_reset(lbm_ctx* h, double bin_width) {
  if (!h) return LBM_E_ARG;
  Ctx& c = h->c;
  if (c.cfg.wall != LBM_WALL_PIPE_Z || !c.pb.acc) return LBM_E_STATE;
  const double R = c.cfg.pipe_radius;
  if (!(bin_width > 0.0) || !(std::ceil(R / bin_width) <= (double)LBM_PIPE_BUDGET_MAX_BINS)) return LBM_E_ARG;
  const int nbins = std::max(1, (int)std::ceil(R / bin_width));
  // fluid (x, y) of the cross-section by bin; r^2 and the bin exactly as
  // the device and the wall test evaluate them
  std::vector<std::vector<uint32_t>> by(nbins);
  for (int y = 0; y < c.dims.ny; ++y)
    for (int x = 0; x < c.dims.nx; ++x) {
      const double dx = (double)x - c.cfg.pipe_cx, dy = (double)y - c.cfg.pipe_cy;
      const double r2 = dy * dy + dx * dx;
      if (!(r2 < R * R)) continue;
      const int k = (int)std::floor(std::sqrt(r2) / bin_width);
      if (k < nbins) by[k].push_back((uint32_t)x | ((uint32_t)y << 16));
    }
  std::vector<uint32_t> list, off(nbins + 1, 0);
  for (int k = 0; k < nbins; ++k) {
    off[k] = (uint32_t)list.size();
    list.insert(list.end(), by[k].begin(), by[k].end());
  }
  off[nbins] = (uint32_t)list.size();
  if (!list.empty() &&
      hipMemcpyAsync(c.pb.list, list.data(), list.size() * 4, hipMemcpyHostToDevice, c.stream) != hipSuccess)
    return LBM_E_HIP;
  if (hipMemcpyAsync(c.pb.off, off.data(), off.size() * 4, hipMemcpyHostToDevice, c.stream) != hipSuccess ||
      hipMemsetAsync(c.pb.acc, 0, (size_t)LBM_PIPE_BUDGET_MOMENTS * nbins * sizeof(double), c.stream) != hipSuccess ||
      hipStreamSynchronize(c.stream) != hipSuccess)
    return LBM_E_HIP;
  c.pb.nbins = nbins;
  c.pb.width = bin_width;
  c.pb.snapshots = 0;
  return LBM_OK;
}

int lbm_pipe_budget_add(lbm_ctx* h) {
  if (!h) return LBM_E_ARG;
  Ctx& c = h->c;
  if (c.pb.nbins <= 0) return LBM_E_STATE;
  const size_t N = c.dims.N;
  const Scratch sc = scratch_layout(c);
  double* part = (double*)((char*)sc.key + align_up(N * sizeof(uint32_t)));
  const size_t used = (size_t)((char*)part - (char*)c.f_nxt);
  if (used + pipe_budget_part_bytes(c, c.pb.nbins) > pop_bytes(c.cfg)) return LBM_E_SIZE;
  int st = lbm_get_fields_device(h, sc.u, sc.rho);
  if (st != LBM_OK) return st;
  const int pc = c.pcur;
  hipError_t e = timed(c, LBM_K_STATS, [&] {
    hipError_t r = launch_stats_keys(c, sc.key, 0, 1.0, c.P.X[pc]);
    if (r == hipSuccess) r = launch_pipe_budget_add(c, sc.u, sc.rho, sc.key, part);
    return r;
  });
  if (e != hipSuccess) return LBM_E_HIP;
  st = drain_errors(c);
  if (st == LBM_OK) ++c.pb.snapshots;
  return st;
}

int lbm_pipe_budget_read(lbm_ctx* h, int32_t* nbins, int64_t* snapshots, double* moments, double* terms) {
  if (!h || !nbins || !snapshots) return LBM_E_ARG;
  Ctx& c = h->c;
  if (c.pb.nbins <= 0) return LBM_E_STATE;
  const int K = c.pb.nbins;
  const int NM = LBM_PIPE_BUDGET_MOMENTS;
  std::vector<double> M((size_t)NM * K);
  if (hipMemcpyAsync(M.data(), c.pb.acc, M.size() * sizeof(double), hipMemcpyDeviceToHost, c.stream) != hipSuccess)
    return LBM_E_HIP;
  const int st = drain_errors(c);
  if (st != LBM_OK) return st;
  *nbins = K;
  *snapshots = c.pb.snapshots;
  if (moments) std::copy(M.begin(), M.end(), moments);
  if (!terms) return LBM_OK;
  // bin means of the sums (moment order as documented in lbm.h)
  enum { kCnt, kUr, kUt, kUz, kP, kSrr, kSrt, kSrz, kStt, kStz, kSzz, kLzr, kLzt, kLzz, kLrr, kLrt, kLrz, kLtt,
         kLtr, kLtz, kUzUr, kUrUr, kUtUr, kUzUz, kUtUt, kPUr, kPLzz, kPLrr, kPLtt, kUzSzr, kUrSrr, kUtStr, kDz,
         kDr, kDt, kUzUzUr, kUrUrUr, kUtUtUr };
  const double w = c.pb.width, nu = (c.cfg.tau - 0.5) / 3.0;
  auto mean = [&](int m, int k) { return M[(size_t)m * K + k] / M[(size_t)kCnt * K + k]; };
  auto rk = [&](int k) { return ((double)k + 0.5) * w; };
  // d f/dr at bin k over the bin centres: central, one-sided at the ends
  auto ddr = [&](auto f, int k) {
    if (K == 1) return std::nan("");
    if (k == 0) return (f(1) - f(0)) / w;
    if (k == K - 1) return (f(K - 1) - f(K - 2)) / w;
    return (f(k + 1) - f(k - 1)) / (2.0 * w);
  };
  auto cov = [&](int ab, int a, int b, int k) { return mean(ab, k) - mean(a, k) * mean(b, k); };
  auto trip = [&](int aab, int ab, int aa, int a, int b, int k) {  // <a'a'b'>
    const double A = mean(a, k), B = mean(b, k);
    return mean(aab, k) - 2.0 * A * mean(ab, k) - B * mean(aa, k) + 2.0 * A * A * B;
  };
  for (int k = 0; k < K; ++k) {
    auto cyl_div = [&](auto f) { return ddr([&](int j) { return rk(j) * f(j); }, k) / rk(k); };
    double* T = terms;
    T[0 * K + k] = -cov(kUzUr, kUz, kUr, k) * ddr([&](int j) { return mean(kUz, j); }, k);
    T[1 * K + k] = -cyl_div([&](int j) { return 0.5 * trip(kUzUzUr, kUzUr, kUzUz, kUz, kUr, j); });
    T[2 * K + k] = cov(kPLzz, kP, kLzz, k);
    T[3 * K + k] = 2.0 * nu * cyl_div([&](int j) { return cov(kUzSzr, kUz, kSrz, j); });
    T[4 * K + k] = -2.0 * nu *
                   (mean(kDz, k) - (mean(kSrz, k) * mean(kLzr, k) + mean(kStz, k) * mean(kLzt, k) +
                                    mean(kSzz, k) * mean(kLzz, k)));
    T[5 * K + k] = -cyl_div([&](int j) {
      const double A = mean(kUr, j);
      return 0.5 * (mean(kUrUrUr, j) - 3.0 * A * mean(kUrUr, j) + 2.0 * A * A * A);
    });
    T[6 * K + k] = -ddr([&](int j) { return cov(kPUr, kUr, kP, j); }, k) + cov(kPLrr, kP, kLrr, k);
    T[7 * K + k] = 2.0 * nu * cyl_div([&](int j) { return cov(kUrSrr, kUr, kSrr, j); });
    T[8 * K + k] = -2.0 * nu *
                   (mean(kDr, k) - (mean(kSrr, k) * mean(kLrr, k) + mean(kSrt, k) * mean(kLrt, k) +
                                    mean(kSrz, k) * mean(kLrz, k)));
    T[9 * K + k] = -cyl_div([&](int j) { return 0.5 * trip(kUtUtUr, kUtUr, kUtUt, kUt, kUr, j); });
    T[10 * K + k] = cov(kPLtt, kP, kLtt, k);
    T[11 * K + k] = 2.0 * nu * cyl_div([&](int j) { return cov(kUtStr, kUt, kSrt, j); });
    T[12 * K + k] = -2.0 * nu *
                    (mean(kDt, k) - (mean(kStt, k) * mean(kLtt, k) + mean(kSrt, k) * mean(kLtr, k) +
                                     mean(kStz, k) * mean(kLtz, k)));
  }
  return LBM_OK;
}

int lbm_sync(lbm_ctx* h) {
  if (!h) return LBM_E_ARG;
  return drain_errors(h->c);
}

int lbm_step_count(const lbm_ctx* h, int64_t* step) {
  if (!h || !step) return LBM_E_ARG;
  *step = h->c.step;
  return LBM_OK;
}

int lbm_set_overlap(lbm_ctx* h, int32_t on) {
  if (!h) return LBM_E_ARG;
  h->c.overlap = on != 0;
  return LBM_OK;
}

int lbm_profile_enable(lbm_ctx* h, int32_t on) {
  if (!h) return LBM_E_ARG;
  h->c.prof.on = on != 0;
  return LBM_OK;
}

int lbm_profile_read(lbm_ctx* h, double* ms, int64_t* launches) {
  if (!h) return LBM_E_ARG;
  Profiler& p = h->c.prof;
  if (p.harvest() != hipSuccess) return LBM_E_HIP;
  for (int k = 0; k < LBM_NPROF; ++k) {
    if (ms) ms[k] = p.ms[k];
    if (launches) launches[k] = p.launches[k];
    p.ms[k] = 0.0;
    p.launches[k] = 0;
  }
  return LBM_OK;
}

void lbm_destroy(lbm_ctx* h) {
  if (!h) return;
  (void)hipStreamSynchronize(h->c.stream);
  delete h;
}

const char* lbm_strerror(int status) {
  switch (status) {
    case LBM_OK: return "ok";
    case LBM_E_ARG: return "invalid argument or configuration";
    case LBM_E_HIP: return "HIP runtime call failed";
    case LBM_E_SIZE: return "workspace too small or capacity exceeded";
    case LBM_E_STATE: return "call not valid in the current state";
    case LBM_E_UNSTABLE: return "numerical instability: non-finite or |u| > 0.35";
    case LBM_E_OVERLAP: return "particles overlap by more than half a radius";
    default: return "unknown status";
  }
}

}  // extern "C"
