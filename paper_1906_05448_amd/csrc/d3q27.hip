// d3q27.hip - the D3Q27 pipe solver (Sec. 2.2): fused pull-stream +
// single-parameter collision (optional energy-mode rate) + Guo forcing, FP32
// populations; equilibrium initialisation; fields; and the links and linear
// interpolated bounce-back of the static pipe wall (Sec. 2.1).
//
// Layout: 27 arrays of N FP32 shifted populations, x fastest, S apart. The fused
// kernel uses the D3Q19 kernel's 128 x 2 tiles in XCD-contiguous order, one
// node per lane, the nine source row offsets in scalar registers and
// non-temporal stores: 216 bytes of HBM traffic per node and step.
#include "d3q27.hpp"
#include "device_util.hpp"
#include "internal.hpp"

namespace lbm {

namespace {

using namespace q27;

template <int TW>
__global__ void __launch_bounds__(256)
k_sc27(const float* __restrict__ A, float* __restrict__ B, Dims d, Tiles tg, Rates r, float3 F,
       uint32_t* __restrict__ err) {
  const Tile t = tile_of<TW>(d, tg);
  if (!t.live) return;
  // a wavefront covers 64 nodes of one row: y and z are uniform across it
  const int x = t.x, z = t.z;
  const int y = __builtin_amdgcn_readfirstlane(t.y);
  const int nx = d.nx, ny = d.ny, nz = d.nz;
  const uint32_t S = d.S;  // population array stride
  const int xm = x == 0 ? nx - 1 : x - 1, xp = x == nx - 1 ? 0 : x + 1;
  const int ys[3] = {y == ny - 1 ? 0 : y + 1, y, y == 0 ? ny - 1 : y - 1};  // y - c_y for c_y = -1, 0, 1
  const int zs[3] = {z == nz - 1 ? 0 : z + 1, z, z == 0 ? nz - 1 : z - 1};
  auto row = [&](int yy, int zz) -> uint32_t { return ((uint32_t)zz * (uint32_t)ny + (uint32_t)yy) * (uint32_t)nx; };
  const uint32_t ox = (uint32_t)x * 4u, oxm = (uint32_t)xm * 4u, oxp = (uint32_t)xp * 4u;
  float g[q27::kQ];
#pragma unroll
  for (int i = 0; i < q27::kQ; ++i) {
    const uint32_t src = row(ys[cy(i) + 1], zs[cz(i) + 1]);
    const uint32_t o = cx(i) > 0 ? oxm : (cx(i) < 0 ? oxp : ox);
    g[i] = *(const float*)((const char*)(A + (size_t)i * S + src) + o);
  }
  float rho, ux, uy, uz;
  collide(g, F.x, F.y, F.z, r, rho, ux, uy, uz);
  const uint32_t r00 = row(y, z);
#pragma unroll
  for (int i = 0; i < q27::kQ; ++i) __builtin_nontemporal_store(g[i], (float*)((char*)(B + (size_t)i * S + r00) + ox));
  const bool bad = !(rho > 0.0f) || !(ux * ux + uy * uy + uz * uz < 0.1225f);
  if (bad) atomicOr(err, kErrUnstable);
}

__global__ void __launch_bounds__(256)
k_init27(const float* __restrict__ u, const float* __restrict__ rho, float* __restrict__ f, uint32_t N, uint32_t S) {
  const uint32_t n = blockIdx.x * 256u + threadIdx.x;
  if (n >= N) return;
  const float r = rho ? rho[n] : 1.0f;
  const float ux = u[n], uy = u[(size_t)N + n], uz = u[2 * (size_t)N + n];
#pragma unroll
  for (int i = 0; i < q27::kQ; ++i) f[(size_t)i * S + n] = q27::geq(i, r, ux, uy, uz);
}

// rho and u = (sum_i c_i f~_i - F/2) / rho from post-collision populations.
__global__ void __launch_bounds__(256)
k_fields27(const float* __restrict__ f, uint32_t N, uint32_t S, float3 F, float* __restrict__ u,
           float* __restrict__ rho) {
  const uint32_t n = blockIdx.x * 256u + threadIdx.x;
  if (n >= N) return;
  float drho = 0.0f, jx = 0.0f, jy = 0.0f, jz = 0.0f;
#pragma unroll
  for (int i = 0; i < q27::kQ; ++i) {
    const float g = f[(size_t)i * S + n];
    drho += g;
    jx += (float)cx(i) * g;
    jy += (float)cy(i) * g;
    jz += (float)cz(i) * g;
  }
  const float r = 1.0f + drho;
  if (rho) rho[n] = r;
  if (u) {
    u[n] = (jx - 0.5f * F.x) / r;
    u[(size_t)N + n] = (jy - 0.5f * F.y) / r;
    u[2 * (size_t)N + n] = (jz - 0.5f * F.z) / r;
  }
}

__device__ __forceinline__ uint32_t nb27(int x, int y, int z, int k, int a, const Dims& d) {
  return node_index(wrap1(x + k * cx(a), d.nx), wrap1(y + k * cy(a), d.ny), wrap1(z + k * cz(a), d.nz), d.nx, d.ny);
}

// Links from every fluid node towards the wall over the 26 moving
// directions, q in FP64; the linear scheme needs x_f - c fluid when q < 1/2,
// else the link takes the single-node fallback. Slots come from a counter
// (the wall carries no force, so the order does not matter).
__global__ void __launch_bounds__(256)
k_wall_links27(const uint32_t* __restrict__ owner, Dims d, double R, double pcx, double pcy,
               uint32_t* __restrict__ counter, uint32_t cap, uint32_t* __restrict__ node_out, float* __restrict__ q_out,
               uint8_t* __restrict__ meta_out, int count_only) {
  const uint32_t n = blockIdx.x * 256u + threadIdx.x;
  if (n >= d.N) return;
  if (owner[n] != kFluid) return;
  int x, y, z;
  node_coords(n, d.nx, d.ny, x, y, z);
  for (int a = 1; a < q27::kQ; ++a) {
    if (owner[nb27(x, y, z, 1, a, d)] != kWall) continue;
    const uint32_t slot = atomicAdd(counter, 1u);
    if (count_only || slot >= cap) continue;
    const double q = pipe_q((double)x - pcx, (double)y - pcy, cx(a), cy(a), R);
    const bool f1 = owner[nb27(x, y, z, -1, a, d)] == kFluid;
    const uint32_t s = (q >= 0.5 || f1) ? kSchemeLinear : kSchemeHalfway;
    node_out[slot] = pack_xyz(x, y, z);
    q_out[slot] = (float)q;
    meta_out[slot] = (uint8_t)(a | (s << 5));
  }
}

// Linear interpolated bounce-back (Bouzidi et al.) at the static wall: the
// value entering x_f in direction opp(a) is written into the ghost slot at
// the wall node x_f + c_a, which the fused kernel pulls. The coefficients
// sum to one and w_a = w_opp(a), so the formula holds for shifted values.
__global__ void __launch_bounds__(256)
k_wall_bounce27(float* __restrict__ A, Dims d, uint32_t count, const uint32_t* __restrict__ node,
                const float* __restrict__ qv, const uint8_t* __restrict__ meta_v) {
  const uint32_t k = blockIdx.x * 256u + threadIdx.x;
  if (k >= count) return;
  const uint32_t meta = meta_v[k];
  const int a = (int)(meta & 31u);
  const float q = qv[k];
  int x, y, z;
  unpack_xyz(node[k], x, y, z);
  const uint32_t n0 = node_index(x, y, z, d.nx, d.ny);
  const size_t S = d.S;
  const float fa0 = A[(size_t)a * S + n0];
  float v = fa0;
  if ((meta >> 5) == kSchemeLinear) {
    if (q < 0.5f)
      v = 2.0f * q * fa0 + (1.0f - 2.0f * q) * A[(size_t)a * S + nb27(x, y, z, -1, a, d)];
    else
      v = (fa0 + (2.0f * q - 1.0f) * A[(size_t)opp(a) * S + n0]) / (2.0f * q);
  }
  A[(size_t)opp(a) * S + nb27(x, y, z, 1, a, d)] = v;
}

Rates rates27(const Ctx& c) {
  const double tb = c.cfg.tau_bulk > 0.0 ? c.cfg.tau_bulk : c.cfg.tau;
  return Rates{(float)(1.0 / c.cfg.tau), (float)(1.0 / tb)};
}

}  // namespace

hipError_t launch_stream_collide27(const Ctx& c, const void* A, void* B) {
  if (tile_width(c.dims.nx) == 64) {
    const Tiles tg = make_tiles(c.dims, 64);
    hipLaunchKernelGGL(k_sc27<64>, dim3(tg.per_xcd * 8), dim3(256), 0, c.stream, (const float*)A, (float*)B, c.dims,
                       tg, rates27(c), c.body_force, c.err);
  } else {
    const Tiles tg = make_tiles(c.dims, 128);
    hipLaunchKernelGGL(k_sc27<128>, dim3(tg.per_xcd * 8), dim3(256), 0, c.stream, (const float*)A, (float*)B,
                       c.dims, tg, rates27(c), c.body_force, c.err);
  }
  return hipGetLastError();
}

hipError_t launch_init_equilibrium27(const Ctx& c, const float* u, const float* rho, void* f) {
  const uint32_t N = c.dims.N;
  hipLaunchKernelGGL(k_init27, dim3((N + 255) / 256), dim3(256), 0, c.stream, u, rho, (float*)f, N, c.dims.S);
  return hipGetLastError();
}

hipError_t launch_fields27(const Ctx& c, const void* f, float3 F, float* u, float* rho) {
  const uint32_t N = c.dims.N;
  hipLaunchKernelGGL(k_fields27, dim3((N + 255) / 256), dim3(256), 0, c.stream, (const float*)f, N, c.dims.S, F, u, rho);
  return hipGetLastError();
}

hipError_t launch_wall_links27(Ctx& c, const uint32_t* owner, uint32_t* counter, bool count_only) {
  const uint32_t N = c.dims.N;
  hipLaunchKernelGGL(k_wall_links27, dim3((N + 255) / 256), dim3(256), 0, c.stream, owner, c.dims, c.cfg.pipe_radius,
                     c.cfg.pipe_cx, c.cfg.pipe_cy, counter, c.ibb.wl_count, c.ibb.wl_node, c.ibb.wl_q, c.ibb.wl_meta,
                     count_only ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_wall_bounce27(const Ctx& c, void* A) {
  if (!c.ibb.wl_count) return hipSuccess;
  hipLaunchKernelGGL(k_wall_bounce27, dim3((c.ibb.wl_count + 255) / 256), dim3(256), 0, c.stream, (float*)A, c.dims,
                     c.ibb.wl_count, c.ibb.wl_node, c.ibb.wl_q, c.ibb.wl_meta);
  return hipGetLastError();
}

}  // namespace lbm
