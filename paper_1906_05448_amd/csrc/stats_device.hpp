// stats_device.hpp - node keys, neighbour indices, raw and masked velocity
// sources and the central-difference dissipation shared by the statistics
// and the gradient corrector.
//
// Node keys: 0 pipe wall, p + 1 inside sphere p (lowest index),
// 0x80000000 | bin for fluid within the profile range, 0xFFFFFFFF other
// fluid. Masked velocity: U_p + Omega_p x (x - X_p) (minimum image) inside
// sphere p, zero in the wall, the lattice field elsewhere; evaluated in FP64.
#pragma once
#include "device_util.hpp"
#include "internal.hpp"

namespace lbm {

constexpr uint32_t kKeyWall = 0u;
constexpr uint32_t kKeyFluid = 0x80000000u;
constexpr uint32_t kKeyFar = 0xFFFFFFFFu;

struct Neigh {
  uint32_t c, xm, xp, ym, yp, zm, zp;
  int x, y, z;
};

__device__ __forceinline__ Neigh neighbours(uint32_t n, const Dims& d) {
  Neigh g;
  node_coords(n, d.nx, d.ny, g.x, g.y, g.z);
  g.c = n;
  const int xm = g.x == 0 ? d.nx - 1 : g.x - 1, xp = g.x == d.nx - 1 ? 0 : g.x + 1;
  const int ym = g.y == 0 ? d.ny - 1 : g.y - 1, yp = g.y == d.ny - 1 ? 0 : g.y + 1;
  const int zm = g.z == 0 ? d.nz - 1 : g.z - 1, zp = g.z == d.nz - 1 ? 0 : g.z + 1;
  g.xm = node_index(xm, g.y, g.z, d.nx, d.ny);
  g.xp = node_index(xp, g.y, g.z, d.nx, d.ny);
  g.ym = node_index(g.x, ym, g.z, d.nx, d.ny);
  g.yp = node_index(g.x, yp, g.z, d.nx, d.ny);
  g.zm = node_index(g.x, g.y, zm, d.nx, d.ny);
  g.zp = node_index(g.x, g.y, zp, d.nx, d.ny);
  return g;
}

// Velocity source: the raw field, or the field masked by the key.
struct RawVel {
  const float* u;
  uint32_t N;
  __device__ void at(uint32_t n, double v[3]) const {
    v[0] = u[n];
    v[1] = u[(size_t)N + n];
    v[2] = u[2 * (size_t)N + n];
  }
};

struct MaskedVel {
  const float* u;
  const uint32_t* key;
  const double *X, *U, *Om;
  Dims d;
  __device__ void at(uint32_t n, double v[3]) const {
    const uint32_t k = key[n];
    if (k >= kKeyFluid) {
      v[0] = u[n];
      v[1] = u[(size_t)d.N + n];
      v[2] = u[2 * (size_t)d.N + n];
      return;
    }
    if (k == kKeyWall) {
      v[0] = v[1] = v[2] = 0.0;
      return;
    }
    const uint32_t p = k - 1u;
    int x, y, z;
    node_coords(n, d.nx, d.ny, x, y, z);
    const double r[3] = {min_image((double)x - X[3 * p], d.nx), min_image((double)y - X[3 * p + 1], d.ny),
                         min_image((double)z - X[3 * p + 2], d.nz)};
    const double* w = Om + 3 * p;
    v[0] = U[3 * p] + (w[1] * r[2] - w[2] * r[1]);
    v[1] = U[3 * p + 1] + (w[2] * r[0] - w[0] * r[2]);
    v[2] = U[3 * p + 2] + (w[0] * r[1] - w[1] * r[0]);
  }
};

// G_ij = d_j u_i by periodic central differences.
template <class V>
__device__ __forceinline__ void velocity_gradient(const V& vel, const Neigh& g, double (&G)[3][3]) {
  double a[3], b[3];
  vel.at(g.xp, a);
  vel.at(g.xm, b);
  for (int i = 0; i < 3; ++i) G[i][0] = 0.5 * (a[i] - b[i]);
  vel.at(g.yp, a);
  vel.at(g.ym, b);
  for (int i = 0; i < 3; ++i) G[i][1] = 0.5 * (a[i] - b[i]);
  vel.at(g.zp, a);
  vel.at(g.zm, b);
  for (int i = 0; i < 3; ++i) G[i][2] = 0.5 * (a[i] - b[i]);
}

// eps = 2 nu s_ij s_ij, s = (G + G^T) / 2.
__device__ __forceinline__ double dissipation_of(const double (&G)[3][3], double nu) {
  double ss = 0.0;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      const double s = 0.5 * (G[i][j] + G[j][i]);
      ss += s * s;
    }
  return 2.0 * nu * ss;
}

template <class V>
__device__ __forceinline__ double dissipation(const V& vel, const Neigh& g, double nu) {
  double G[3][3];
  velocity_gradient(vel, g, G);
  return dissipation_of(G, nu);
}

}  // namespace lbm
