// ibb.hip - interpolated bounce-back at boundary links, the link forces, and
// the refilling of uncovered nodes (Sec. 3.1, Sec. 2.1).
//
// Ghost-slot design: for a link (x_f, a) the unknown population f_abar(x_f)
// is pulled from slot (abar, x_s) of the source buffer, where x_s = x_f + c_a
// is the solid node. That slot is read by no other node, so this kernel
// writes the interpolated bounce-back value there before the dense kernel
// runs, and the dense kernel stays a branch-free pull over fluid nodes.
// Where the dense kernel stages whole 512-node rows in LDS, the value goes
// instead into a list per row of the fluid node (patches), which that
// kernel writes over the staged slot: one scattered 2- or 4-byte store per
// link into the population arrays cost about 0.5 ms per step at 512^3 with
// 28.8 M links (each a partial write of its own memory sector).
//
// Interpolation (Bouzidi, Firdaouss & Lallemand 2001) with the moving-wall
// term delta = -6 w_a (c_a . u_w); coefficients of every branch sum to one
// and w_a = w_abar, so the shifted populations g = f - w enter directly:
//   quadratic q < 1/2 : q(1+2q) g_a(x_f) + (1-4q^2) g_a(x_f-c) - q(1-2q) g_a(x_f-2c) + delta
//   quadratic q >= 1/2: [g_a(x_f) + delta]/(q(2q+1)) + (2q-1)/q g_abar(x_f)
//                       - (2q-1)/(2q+1) g_abar(x_f-c)
//   linear q < 1/2    : 2q g_a(x_f) + (1-2q) g_a(x_f-c) + delta
//   linear q >= 1/2   : [g_a(x_f) + delta]/(2q) + (2q-1)/(2q) g_abar(x_f)
//   single node       : g_a(x_f) + delta   (halfway bounce-back)
// Link force (Wen et al. 2014, Galilean invariant momentum exchange):
//   F = (c_a - u_w) f~_a(x_f) - (c_abar - u_w) f_abar(x_f, t+1), torque (x_w - X) x F.
#include "device_util.hpp"
#include "internal.hpp"

namespace lbm {

namespace {

constexpr int kBlock = 256;
constexpr int kLinkBlock = kLinkSliceThreads;  // a slice of a sphere's links per workgroup
constexpr int kRefillList = 4096; // nodes listed per round of rows in the refill

template <int STORE>
__device__ __forceinline__ float ld(const typename Pop<STORE>::T* f, int i, uint32_t S, uint32_t n) {
  return Pop<STORE>::load(f + (size_t)i * S + n);
}

// Interpolated value of the entering population for one link, from the
// values the scheme reads: ga0 = g_a(x_f) and, with q < 1/2, v1 = g_a(x_f - c),
// v2 = g_a(x_f - 2c); with q >= 1/2, v1 = g_ab(x_f), v2 = g_ab(x_f - c)
// (ab the opposite of a). The linear scheme uses v1 only, the single-node
// scheme neither.
__device__ __forceinline__ float bounce_from(float ga0, float v1, float v2, uint32_t scheme, float q, float delta) {
  if (scheme == kSchemeQuadratic) {
    if (q < 0.5f) return q * (1.0f + 2.0f * q) * ga0 + (1.0f - 4.0f * q * q) * v1 - q * (1.0f - 2.0f * q) * v2 + delta;
    const float t = 2.0f * q - 1.0f;
    return (ga0 + delta) / (q * (2.0f * q + 1.0f)) + t / q * v1 - t / (2.0f * q + 1.0f) * v2;
  }
  if (scheme == kSchemeLinear) {
    if (q < 0.5f) return 2.0f * q * ga0 + (1.0f - 2.0f * q) * v1 + delta;
    return (ga0 + delta) / (2.0f * q) + (2.0f * q - 1.0f) / (2.0f * q) * v1;
  }
  return ga0 + delta;
}

// Population array and node of the two extra values a link reads.
__device__ __forceinline__ void bounce_sources(int a, float q, uint32_t nf, uint32_t nm1, uint32_t nm2, int& i1,
                                               uint32_t& n1, int& i2, uint32_t& n2) {
  const bool lo = q < 0.5f;
  i1 = lo ? a : opp_of(a);
  n1 = lo ? nm1 : nf;
  i2 = i1;
  n2 = lo ? nm2 : nm1;
}

template <int STORE>
__device__ __forceinline__ float bounce_value(const typename Pop<STORE>::T* A, uint32_t S, uint32_t nf, uint32_t nm1,
                                              uint32_t nm2, int a, uint32_t scheme, float q, float delta) {
  int i1, i2;
  uint32_t n1, n2;
  bounce_sources(a, q, nf, nm1, nm2, i1, n1, i2, n2);
  const float ga0 = ld<STORE>(A, a, S, nf);
  const float v1 = scheme != kSchemeHalfway ? ld<STORE>(A, i1, S, n1) : 0.0f;
  const float v2 = scheme == kSchemeQuadratic ? ld<STORE>(A, i2, S, n2) : 0.0f;
  return bounce_from(ga0, v1, v2, scheme, q, delta);
}

// Rank of each live lane's link in the list of its row: the lanes of a
// wavefront hold consecutive links, so equal rows come in runs; the first
// lane of each run takes the run's places with one atomic add and the
// others count on from it (ranks per row stay distinct; their order does
// not matter). Every lane of the wavefront must call it.
__device__ __forceinline__ uint32_t row_rank(uint32_t* cnt, uint32_t row, bool live) {
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t prev = (uint32_t)__shfl_up((int)row, 1, 64);
  const bool head = live && (lane == 0u || prev != row);
  const unsigned long long heads = __ballot(head);
  const unsigned long long ends = __ballot(head || !live);
  const unsigned long long above = lane == 63u ? 0ull : (~0ull << (lane + 1u));
  const unsigned long long later = ends & above;
  const uint32_t next = later ? (uint32_t)__builtin_ctzll(later) : 64u;
  uint32_t base = 0u;
  if (head) base = atomicAdd(cnt + row, next - lane);
  const unsigned long long upto = lane == 63u ? ~0ull : ((2ull << lane) - 1ull);
  const unsigned long long mine = heads & upto;
  const uint32_t h = mine ? 63u - (uint32_t)__builtin_clzll(mine) : lane;
  const uint32_t b = (uint32_t)__shfl((int)base, (int)h, 64);
  return b + (lane - h);
}

// One workgroup per slice of kLinkSlice links of a sphere (slices of one
// sphere run side by side on different CUs): fill the ghost slots of its
// links and reduce the slice's link forces and torques in FP64 in a fixed
// order into part[p][g][6]; k_link_sum adds the slices in order.
template <int STORE>
__global__ void __launch_bounds__(kLinkBlock)
k_ibb_links(typename Pop<STORE>::T* A, Dims d, const double* __restrict__ X, const double* __restrict__ U,
            const double* __restrict__ Om, uint32_t cap, uint32_t slices, const uint32_t* __restrict__ link_node,
            const float* __restrict__ link_q, const uint8_t* __restrict__ link_meta,
            const uint32_t* __restrict__ link_count, double* __restrict__ part, uint32_t* __restrict__ patch_cnt,
            void* __restrict__ patch) {
  const int p = (int)(blockIdx.x / slices);
  const uint32_t g = blockIdx.x % slices;
  const uint32_t cnt = min(link_count[p], (g + 1u) * kLinkSlice);
  const size_t base = (size_t)p * cap;
  const double Xp[3] = {X[3 * p], X[3 * p + 1], X[3 * p + 2]};
  const double Up[3] = {U[3 * p], U[3 * p + 1], U[3 * p + 2]};
  const double Wp[3] = {Om[3 * p], Om[3 * p + 1], Om[3 * p + 2]};
  double F[3] = {0, 0, 0}, T[3] = {0, 0, 0};
  // kLinks links per thread: the records of the slice, then all the
  // population values its links read, are in flight together. The ghost
  // slots written here are at solid nodes, which no link reads.
  constexpr int kLinks = kLinkSlice / kLinkBlock;
  static_assert(kLinks * kLinkBlock == kLinkSlice, "a slice is one round");
  for (uint32_t k0 = g * kLinkSlice; k0 < cnt; k0 += kLinks * kLinkBlock) {
    uint32_t nf[kLinks], meta[kLinks];
    float q[kLinks];
#pragma unroll
    for (int i = 0; i < kLinks; ++i) {
      const uint32_t k = k0 + (uint32_t)(i * kLinkBlock) + threadIdx.x;
      const bool live = k < cnt;
      nf[i] = live ? link_node[base + k] : 0u;
      q[i] = live ? link_q[base + k] : 0.0f;
      meta[i] = live ? (uint32_t)link_meta[base + k] : 0xFFu;
    }
    uint32_t n0[kLinks], ns[kLinks];
    float g0[kLinks], g1[kLinks], g2[kLinks];
#pragma unroll
    for (int i = 0; i < kLinks; ++i) {
      g0[i] = g1[i] = g2[i] = 0.0f;
      n0[i] = ns[i] = 0u;
      if (meta[i] == 0xFFu) continue;
      const int a = (int)(meta[i] & 31u);
      const uint32_t scheme = meta[i] >> 5;
      int x, y, z;
      unpack_xyz(nf[i], x, y, z);
      const int cx = cx_of(a), cy = cy_of(a), cz = cz_of(a);
      n0[i] = node_index(x, y, z, d.nx, d.ny);
      const uint32_t nm1 = node_index(wrap1(x - cx, d.nx), wrap1(y - cy, d.ny), wrap1(z - cz, d.nz), d.nx, d.ny);
      const uint32_t nm2 =
          node_index(wrap1(x - 2 * cx, d.nx), wrap1(y - 2 * cy, d.ny), wrap1(z - 2 * cz, d.nz), d.nx, d.ny);
      ns[i] = node_index(wrap1(x + cx, d.nx), wrap1(y + cy, d.ny), wrap1(z + cz, d.nz), d.nx, d.ny);
      int i1, i2;
      uint32_t m1, m2;
      bounce_sources(a, q[i], n0[i], nm1, nm2, i1, m1, i2, m2);
      g0[i] = ld<STORE>(A, a, d.S, n0[i]);
      if (scheme != kSchemeHalfway) g1[i] = ld<STORE>(A, i1, d.S, m1);
      if (scheme == kSchemeQuadratic) g2[i] = ld<STORE>(A, i2, d.S, m2);
    }
#pragma unroll
    for (int i = 0; i < kLinks; ++i) {
      const bool live = meta[i] != 0xFFu;
      float gnew = 0.0f;
      uint32_t row = 0xFFFFFFFFu, px = 0u, pi = 0u;
      if (live) {
        const int a = (int)(meta[i] & 31u);
        const uint32_t scheme = meta[i] >> 5;
        int x, y, z;
        unpack_xyz(nf[i], x, y, z);
        const int cx = cx_of(a), cy = cy_of(a), cz = cz_of(a);
        // lever arm x_w - X and wall velocity U + Omega x arm
        const double arm[3] = {min_image((double)x - Xp[0], d.nx) + (double)q[i] * cx,
                               min_image((double)y - Xp[1], d.ny) + (double)q[i] * cy,
                               min_image((double)z - Xp[2], d.nz) + (double)q[i] * cz};
        const double uw[3] = {Up[0] + (Wp[1] * arm[2] - Wp[2] * arm[1]), Up[1] + (Wp[2] * arm[0] - Wp[0] * arm[2]),
                              Up[2] + (Wp[0] * arm[1] - Wp[1] * arm[0])};
        const float delta = (float)(-6.0 * (double)w_of(a) * (cx * uw[0] + cy * uw[1] + cz * uw[2]));
        gnew = bounce_from(g0[i], g1[i], g2[i], scheme, q[i], delta);
        row = (uint32_t)z * (uint32_t)d.ny + (uint32_t)y;
        px = (uint32_t)x;
        pi = (uint32_t)opp_of(a);
        const double fa = (double)g0[i] + (double)w_of(a);
        const double fb = (double)gnew + (double)w_of(a);
        const double c[3] = {(double)cx, (double)cy, (double)cz};
        double Fl[3];
        for (int k3 = 0; k3 < 3; ++k3) Fl[k3] = (c[k3] - uw[k3]) * fa + (c[k3] + uw[k3]) * fb;
        F[0] += Fl[0];
        F[1] += Fl[1];
        F[2] += Fl[2];
        T[0] += arm[1] * Fl[2] - arm[2] * Fl[1];
        T[1] += arm[2] * Fl[0] - arm[0] * Fl[2];
        T[2] += arm[0] * Fl[1] - arm[1] * Fl[0];
      }
      // the value listed under its fluid node's row, else (no lists, or the
      // row's list full) stored into the ghost slot; every lane takes part
      // in the ranking
      bool listed = false;
      if (patch_cnt) {
        const uint32_t rank = row_rank(patch_cnt, row, live);
        if (live && rank < kPatchCap) {
          const size_t at = (size_t)row * kPatchCap + rank;
          if (STORE == 1)
            ((uint32_t*)patch)[at] = px | (pi << 9) | (Pop<STORE>::bits(gnew) << 16);
          else
            ((uint2*)patch)[at] = make_uint2(px | (pi << 16), Pop<STORE>::bits(gnew));
          listed = true;
        }
      }
      if (live && !listed) Pop<STORE>::store(A + (size_t)opp_of((int)(meta[i] & 31u)) * d.S + ns[i], gnew);
    }
  }
  double* out = part + (size_t)blockIdx.x * 6;
  for (int k3 = 0; k3 < 3; ++k3) {
    const double fs = block_sum<kLinkBlock>(F[k3]);
    const double ts = block_sum<kLinkBlock>(T[k3]);
    if (threadIdx.x == 0) {
      out[k3] = fs;
      out[3 + k3] = ts;
    }
  }
}

// F, T of sphere p: its slice partials added in slice order.
__global__ void __launch_bounds__(64)
k_link_sum(int np, uint32_t slices, const double* __restrict__ part, double* __restrict__ F_out,
           double* __restrict__ T_out) {
  const int p = (int)(blockIdx.x * 64u + threadIdx.x);
  if (p >= np) return;
  double f[6] = {0, 0, 0, 0, 0, 0};
  for (uint32_t g = 0; g < slices; ++g)
    for (int k = 0; k < 6; ++k) f[k] += part[((size_t)p * slices + g) * 6 + k];
  for (int k = 0; k < 3; ++k) {
    F_out[3 * p + k] = f[k];
    T_out[3 * p + k] = f[3 + k];
  }
}

// Static wall links (pipe): zero wall velocity, no force needed.
template <int STORE>
__global__ void __launch_bounds__(256)
k_wall_bounce(typename Pop<STORE>::T* A, Dims d, uint32_t count, const uint32_t* __restrict__ node,
              const float* __restrict__ qv, const uint8_t* __restrict__ meta_v) {
  const uint32_t k = blockIdx.x * 256u + threadIdx.x;
  if (k >= count) return;
  const uint32_t nf = node[k];
  const float q = qv[k];
  const uint32_t meta = meta_v[k];
  const int a = (int)(meta & 31u);
  int x, y, z;
  unpack_xyz(nf, x, y, z);
  const int cx = cx_of(a), cy = cy_of(a), cz = cz_of(a);
  const uint32_t n0 = node_index(x, y, z, d.nx, d.ny);
  const uint32_t nm1 = node_index(wrap1(x - cx, d.nx), wrap1(y - cy, d.ny), wrap1(z - cz, d.nz), d.nx, d.ny);
  const uint32_t ns = node_index(wrap1(x + cx, d.nx), wrap1(y + cy, d.ny), wrap1(z + cz, d.nz), d.nx, d.ny);
  const float gnew = bounce_value<STORE>(A, d.S, n0, nm1, nm1, a, meta >> 5, q, 0.0f);
  Pop<STORE>::store(A + (size_t)opp_of(a) * d.S + ns, gnew);
}

__device__ __forceinline__ bool valid_node(const uint32_t* o_old, const uint32_t* o_new, uint32_t n) {
  return o_old[n] == kFluid && o_new[n] == kFluid;
}

// Refill of one uncovered node: extrapolation along the lattice direction
// closest to the outward normal, then the equilibrium part swapped for the
// wall velocity. Writes g into B and returns the node's momentum.
template <int STORE>
__device__ void refill_node(typename Pop<STORE>::T* B, const Dims& d, const uint32_t* o_old, const uint32_t* o_new,
                            int x, int y, int z, const double dd[3], const double uwd[3], double mom[3]) {
  // direction maximising c . d; ties to the lexicographically largest c
  int best = 1;
  double bv = -1e300;
  for (int k = 1; k < kQ; ++k) {
    const double v = (cx_of(k) * dd[0] + cy_of(k) * dd[1]) + cz_of(k) * dd[2];
    bool take = v > bv;
    if (v == bv) {
      const int b0 = cx_of(best), b1 = cy_of(best), b2 = cz_of(best);
      const int k0 = cx_of(k), k1 = cy_of(k), k2 = cz_of(k);
      take = (k0 > b0) || (k0 == b0 && (k1 > b1 || (k1 == b1 && k2 > b2)));
    }
    if (take) {
      bv = v;
      best = k;
    }
  }
  const int cx = cx_of(best), cy = cy_of(best), cz = cz_of(best);
  uint32_t nb[3];
  bool ok[3];
  for (int s = 0; s < 3; ++s) {
    nb[s] = node_index(wrapi(x + (s + 1) * cx, d.nx), wrapi(y + (s + 1) * cy, d.ny), wrapi(z + (s + 1) * cz, d.nz),
                       d.nx, d.ny);
    ok[s] = valid_node(o_old, o_new, nb[s]);
  }
  float ge[kQ];
  if (ok[0] && ok[1] && ok[2]) {
    for (int i = 0; i < kQ; ++i)
      ge[i] = 3.0f * ld<STORE>(B, i, d.S, nb[0]) - 3.0f * ld<STORE>(B, i, d.S, nb[1]) + ld<STORE>(B, i, d.S, nb[2]);
  } else if (ok[0] && ok[1]) {
    for (int i = 0; i < kQ; ++i) ge[i] = 2.0f * ld<STORE>(B, i, d.S, nb[0]) - ld<STORE>(B, i, d.S, nb[1]);
  } else {
    // equilibrium of the mean density and mean raw velocity of the valid
    // nearest neighbours, or of (1, u_w) if there are none
    float rs = 0.0f, us[3] = {0.0f, 0.0f, 0.0f};
    int cnt = 0;
    for (int k = 1; k < kQ; ++k) {
      const uint32_t m = node_index(wrapi(x + cx_of(k), d.nx), wrapi(y + cy_of(k), d.ny), wrapi(z + cz_of(k), d.nz),
                                    d.nx, d.ny);
      if (!valid_node(o_old, o_new, m)) continue;
      float dr = 0.0f, jx = 0.0f, jy = 0.0f, jz = 0.0f;
      for (int i = 0; i < kQ; ++i) {
        const float g = ld<STORE>(B, i, d.S, m);
        dr += g;
        jx += cx_of(i) * g;
        jy += cy_of(i) * g;
        jz += cz_of(i) * g;
      }
      const float rho = 1.0f + dr;
      rs += rho;
      us[0] += jx / rho;
      us[1] += jy / rho;
      us[2] += jz / rho;
      ++cnt;
    }
    float rho = 1.0f, ux = (float)uwd[0], uy = (float)uwd[1], uz = (float)uwd[2];
    if (cnt) {
      rho = rs / cnt;
      ux = us[0] / cnt;
      uy = us[1] / cnt;
      uz = us[2] / cnt;
    }
    for (int i = 0; i < kQ; ++i) ge[i] = geq(i, rho, ux, uy, uz);
  }
  float dr = 0.0f, jx = 0.0f, jy = 0.0f, jz = 0.0f;
  for (int i = 0; i < kQ; ++i) {
    dr += ge[i];
    jx += cx_of(i) * ge[i];
    jy += cy_of(i) * ge[i];
    jz += cz_of(i) * ge[i];
  }
  const float rho_e = 1.0f + dr;
  const float ux = jx / rho_e, uy = jy / rho_e, uz = jz / rho_e;
  const float wx = (float)uwd[0], wy = (float)uwd[1], wz = (float)uwd[2];
  mom[0] = mom[1] = mom[2] = 0.0;
  for (int i = 0; i < kQ; ++i) {
    const float g = ge[i] - geq(i, rho_e, ux, uy, uz) + geq(i, rho_e, wx, wy, wz);
    Pop<STORE>::store(B + (size_t)i * d.S + node_index(x, y, z, d.nx, d.ny), g);
    const double gd = (double)g;
    mom[0] += cx_of(i) * gd;
    mom[1] += cy_of(i) * gd;
    mom[2] += cz_of(i) * gd;
  }
}

// One workgroup per sphere: refill the nodes it uncovered and collect the
// momentum of the nodes it covered, both into F_rc/T_rc for the next step.
template <int STORE>
__global__ void __launch_bounds__(kBlock, 4)
k_cover_refill(typename Pop<STORE>::T* B, Dims d, const uint32_t* __restrict__ o_old,
               const uint32_t* __restrict__ o_new, const double* __restrict__ Xold, const double* __restrict__ Xnew,
               const double* __restrict__ Unew, const double* __restrict__ Omnew, const double* __restrict__ rad,
               double* __restrict__ F_rc, double* __restrict__ T_rc, uint32_t* __restrict__ err) {
  const uint32_t p = blockIdx.x;
  const double r = rad[p];
  const double* Xn = Xnew + 3 * p;
  const double Up[3] = {Unew[3 * p], Unew[3 * p + 1], Unew[3 * p + 2]};
  const double Wp[3] = {Omnew[3 * p], Omnew[3 * p + 1], Omnew[3 * p + 2]};
  double F[3] = {0, 0, 0}, T[3] = {0, 0, 0};
  const double* Xo = Xold + 3 * p;
  // A node p uncovers lies inside p's old sphere and outside its new one; a
  // node p covers lies inside the new sphere and outside the old one, by the
  // exact FP64 tests that built the owner maps.
  auto inside = [&](int x, int y, int z, const double* C) {
    const double dx = min_image((double)x - C[0], d.nx), dy = min_image((double)y - C[1], d.ny),
                 dz = min_image((double)z - C[2], d.nz);
    return dist2(dx, dy, dz) < r * r;
  };
  // One pass over the union of the old and new boxes: uncovered nodes are
  // inside the old sphere only, covered nodes inside the new one only. The
  // new box is placed at the old centre plus the minimum-image displacement,
  // so a sphere that crossed a periodic face still has a compact union.
  const double Xn_near[3] = {Xo[0] + min_image(Xn[0] - Xo[0], d.nx), Xo[1] + min_image(Xn[1] - Xo[1], d.ny),
                             Xo[2] + min_image(Xn[2] - Xo[2], d.nz)};
  Box b = make_box(Xo, r + 1.0);
  {
    const Box bn = make_box(Xn_near, r + 1.0);
    for (int k = 0; k < 3; ++k) {
      const int lo = min(b.lo[k], bn.lo[k]);
      const int hi = max(b.lo[k] + b.side[k], bn.lo[k] + bn.side[k]);
      b.lo[k] = lo;
      b.side[k] = hi - lo;
    }
  }
  // box offsets are packed in 10 bits; a sphere that moved that far in one
  // step comes only from a diverged flow
  if (b.side[0] > 1023 || b.side[1] > 1023 || b.side[2] > 1023) {
    if (threadIdx.x == 0) atomicOr(err, kErrUnstable);
    return;
  }
  // A node that changed side: uncovered (inside the old sphere) is refilled
  // and its new momentum leaves the sphere; covered (inside the new sphere)
  // hands its momentum to the sphere.
  __shared__ uint32_t changed_all[kBlock];
  uint32_t* changed = changed_all + (threadIdx.x & ~63u);
  const uint32_t lane = threadIdx.x & 63u;
  uint32_t nchanged = 0;
  // Processes the first `count` entries of the wavefront's list, one per lane.
  auto process = [&](uint32_t count) {
    __builtin_amdgcn_wave_barrier();  // the list entries other lanes wrote
    if (lane >= count) return;
    int x, y, z;
    unpack_xyz(changed[lane], x, y, z);
    const bool in_old = inside(x, y, z, Xo);
    const uint32_t n = node_index(x, y, z, d.nx, d.ny);
    const double dd[3] = {min_image((double)x - Xn[0], d.nx), min_image((double)y - Xn[1], d.ny),
                          min_image((double)z - Xn[2], d.nz)};
    if (in_old) {
      // uncovered: solid for p before, fluid now
      if (o_old[n] != p || o_new[n] != kFluid) return;
      const double uw[3] = {Up[0] + (Wp[1] * dd[2] - Wp[2] * dd[1]), Up[1] + (Wp[2] * dd[0] - Wp[0] * dd[2]),
                            Up[2] + (Wp[0] * dd[1] - Wp[1] * dd[0])};
      double mom[3];
      refill_node<STORE>(B, d, o_old, o_new, x, y, z, dd, uw, mom);
      for (int k = 0; k < 3; ++k) F[k] -= mom[k];
      T[0] -= dd[1] * mom[2] - dd[2] * mom[1];
      T[1] -= dd[2] * mom[0] - dd[0] * mom[2];
      T[2] -= dd[0] * mom[1] - dd[1] * mom[0];
    } else {
      // covered: fluid before, solid for p now
      if (o_new[n] != p || o_old[n] != kFluid) return;
      double mom[3] = {0, 0, 0};
      for (int k = 0; k < kQ; ++k) {
        const double g = (double)ld<STORE>(B, k, d.S, n);
        mom[0] += cx_of(k) * g;
        mom[1] += cy_of(k) * g;
        mom[2] += cz_of(k) * g;
      }
      for (int k = 0; k < 3; ++k) F[k] += mom[k];
      T[0] += dd[1] * mom[2] - dd[2] * mom[1];
      T[1] += dd[2] * mom[0] - dd[0] * mom[2];
      T[2] += dd[0] * mom[1] - dd[1] * mom[0];
    }
  };
  // Each row of the union box lists only the nodes that may have changed
  // side: those possibly inside one sphere and not certainly inside both
  // (two square roots per sphere and row, margins beyond any rounding of the
  // exact FP64 test); the exact tests then decide, one node per lane.
  // Refills read only nodes that are fluid in both maps, never another
  // refilled node, so the processing order does not matter.
  __shared__ uint32_t list[kRefillList];
  const double r2 = r * r;
  const int rows = b.side[1] * b.side[2];
  const int R = min(kBlock, kRefillList / b.side[0]);
  const int xlo = b.lo[0], xhi = b.lo[0] + b.side[0] - 1;
  for (int r0 = 0; r0 < rows; r0 += R) {
    const int row = r0 + (int)threadIdx.x;
    int a0 = 1, a1 = 0, b0 = 1, b1 = 0, ly = 0, lz = 0;
    if ((int)threadIdx.x < R && row < rows) {
      ly = row % b.side[1];
      lz = row / b.side[1];
      const double y = (double)(b.lo[1] + ly), z = (double)(b.lo[2] + lz);
      const double eo = (y - Xo[1]) * (y - Xo[1]) + (z - Xo[2]) * (z - Xo[2]);
      const double en = (y - Xn_near[1]) * (y - Xn_near[1]) + (z - Xn_near[2]) * (z - Xn_near[2]);
      const RowSpan so = sphere_row(Xo[0], eo, r2), sn = sphere_row(Xn_near[0], en, r2);
      if (so.any || sn.any) {
        const double olo = so.any ? (sn.any ? fmin(so.plo, sn.plo) : so.plo) : sn.plo;
        const double ohi = so.any ? (sn.any ? fmax(so.phi, sn.phi) : so.phi) : sn.phi;
        // certainly inside both: the intersection of the two certain spans
        const double hlo = fmax(so.clo, sn.clo), hhi = fmin(so.chi, sn.chi);
        row_band(olo, ohi, hlo, hhi, xlo, xhi, a0, a1, b0, b1);
      }
    }
    const uint32_t na = a1 >= a0 ? (uint32_t)(a1 - a0 + 1) : 0u, nb = b1 >= b0 ? (uint32_t)(b1 - b0 + 1) : 0u;
    uint32_t total;
    uint32_t off = block_exclusive_scan<kBlock>(na + nb, &total);
    const uint32_t yz = ((uint32_t)ly << 10) | ((uint32_t)lz << 20);
    for (int x = a0; x <= a1; ++x) list[off++] = (uint32_t)(x - xlo) | yz;
    for (int x = b0; x <= b1; ++x) list[off++] = (uint32_t)(x - xlo) | yz;
    __syncthreads();
    // every lane runs the same number of iterations, so the wavefront-wide
    // ballots see all 64 lanes; the changed nodes go to the wavefront's list,
    // processed whenever it would overflow and at the end
    for (uint32_t j0 = 0; j0 < total; j0 += kBlock) {
      const uint32_t j = j0 + threadIdx.x;
      bool hit = false;
      uint32_t packed = 0;
      if (j < total) {
        const uint32_t e = list[j];
        const int x = wrap1(xlo + (int)(e & 1023u), d.nx);
        const int y = wrap1(b.lo[1] + (int)((e >> 10) & 1023u), d.ny);
        const int z = wrap1(b.lo[2] + (int)((e >> 20) & 1023u), d.nz);
        hit = inside(x, y, z, Xo) != inside(x, y, z, Xn);
        packed = pack_xyz(x, y, z);
      }
      const unsigned long long m = __ballot(hit);
      const uint32_t nhit = (uint32_t)__popcll(m);
      if (nchanged + nhit > 64u) {  // uniform across the wavefront
        process(nchanged);
        nchanged = 0;
      }
      if (hit) changed[nchanged + (uint32_t)__popcll(m & ((1ull << lane) - 1ull))] = packed;
      nchanged += nhit;
    }
    __syncthreads();  // the list is refilled by the next round
  }
  process(nchanged);
  for (int k = 0; k < 3; ++k) {
    const double fs = block_sum<kBlock>(F[k]);
    const double ts = block_sum<kBlock>(T[k]);
    if (threadIdx.x == 0) {
      F_rc[3 * p + k] = fs;
      T_rc[3 * p + k] = ts;
    }
  }
}

// Empties the per-row patch lists.
__global__ void __launch_bounds__(256) k_patch_clear(uint32_t* __restrict__ cnt, uint32_t n) {
  const uint32_t i = blockIdx.x * 256u + threadIdx.x;
  if (i < n) cnt[i] = 0u;
}

}  // namespace

hipError_t launch_ibb_links(const Ctx& c, void* A, const double* X, const double* U, const double* Om) {
  if (lattice27(c)) return launch_wall_bounce27(c, A);  // no particles on that lattice
  if (c.ibb.wl_count) {
    const dim3 g((c.ibb.wl_count + 255) / 256);
    if (c.cfg.store == LBM_STORE_F32)
      hipLaunchKernelGGL(k_wall_bounce<0>, g, dim3(256), 0, c.stream, (float*)A, c.dims, c.ibb.wl_count,
                         c.ibb.wl_node, c.ibb.wl_q, c.ibb.wl_meta);
    else
      hipLaunchKernelGGL(k_wall_bounce<1>, g, dim3(256), 0, c.stream, (_Float16*)A, c.dims, c.ibb.wl_count,
                         c.ibb.wl_node, c.ibb.wl_q, c.ibb.wl_meta);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (c.np <= 0) return hipSuccess;
  uint32_t* pcnt = nullptr;
  if (c.ibb.patches) {
    const uint32_t rows = (uint32_t)c.dims.ny * (uint32_t)c.dims.nz;
    hipLaunchKernelGGL(k_patch_clear, dim3((rows + 255u) / 256u), dim3(256), 0, c.stream, c.ibb.patch_cnt, rows);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    pcnt = c.ibb.patch_cnt;
  }
  const uint32_t slices = c.ibb.link_slices;
  const dim3 grid((uint32_t)c.np * slices);
  if (c.cfg.store == LBM_STORE_F32)
    hipLaunchKernelGGL(k_ibb_links<0>, grid, dim3(kLinkBlock), 0, c.stream, (float*)A, c.dims, X, U, Om, c.link_cap,
                       slices, c.ibb.link_node, c.ibb.link_q, c.ibb.link_meta, c.ibb.link_count, c.ibb.link_part, pcnt,
                       c.ibb.patch);
  else
    hipLaunchKernelGGL(k_ibb_links<1>, grid, dim3(kLinkBlock), 0, c.stream, (_Float16*)A, c.dims, X, U, Om,
                       c.link_cap, slices, c.ibb.link_node, c.ibb.link_q, c.ibb.link_meta, c.ibb.link_count,
                       c.ibb.link_part, pcnt, c.ibb.patch);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_link_sum, dim3(((uint32_t)c.np + 63u) / 64u), dim3(64), 0, c.stream, c.np, slices,
                     c.ibb.link_part, c.P.F_link, c.P.T_link);
  return hipGetLastError();
}

hipError_t launch_cover_refill(const Ctx& c, void* B, const uint32_t* owner_old, const uint32_t* owner_new,
                               const double* Xold, const double* Xnew, const double* Unew, const double* Omnew) {
  if (c.np <= 0) return hipSuccess;
  if (c.cfg.store == LBM_STORE_F32)
    hipLaunchKernelGGL(k_cover_refill<0>, dim3(c.np), dim3(kBlock), 0, c.stream, (float*)B, c.dims, owner_old,
                       owner_new, Xold, Xnew, Unew, Omnew, c.P.r, c.P.F_rc, c.P.T_rc, c.err);
  else
    hipLaunchKernelGGL(k_cover_refill<1>, dim3(c.np), dim3(kBlock), 0, c.stream, (_Float16*)B, c.dims, owner_old,
                       owner_new, Xold, Xnew, Unew, Omnew, c.P.r, c.P.F_rc, c.P.T_rc, c.err);
  return hipGetLastError();
}

}  // namespace lbm
