// particles.hip - rigid-sphere motion, soft-sphere contact and particle
// release (Sec. 3.1), all in FP64.
//
// Equations of motion, one explicit step of length 1 with m = rho_p 4/3 pi r^3
// and I = 2/5 m r^2:
//   U' = U + (F_h + F_c)/m,  X' = X + (U + U')/2 (wrapped),  Omega' = Omega + T_h/I.
// Contact (normal only, no friction or lubrication): for an overlap
// delta = r_i + r_j - |X_i - X_j| > 0,
//   F_i = (k_n delta - eta_n (U_i - U_j).n) n,  k_n = m_eff (pi^2 + ln^2 e)/T_c^2,
//   eta_n = -2 m_eff ln e / T_c,
// summed over j in index order per particle (deterministic).
// Release: U = Kempe-weighted mean of the fluid velocity over the particle,
// Omega = 0, and the populations at the particle's nodes are reset once to the
// equilibrium of the local density and U.
#include "device_util.hpp"
#include "internal.hpp"

namespace lbm {

namespace {

constexpr double kPi = 3.14159265358979323846;

__global__ void __launch_bounds__(64)
k_particle_update(int np, int motion, int bc, Dims d, const double* __restrict__ X, const double* __restrict__ U,
                  const double* __restrict__ Om, double* __restrict__ Xn, double* __restrict__ Un,
                  double* __restrict__ Omn, const double* __restrict__ rad, const double* __restrict__ rho_p,
                  const double* __restrict__ F_a, const double* __restrict__ T_a, const double* __restrict__ F_b,
                  const double* __restrict__ T_b, double* __restrict__ Iu, double* __restrict__ IL,
                  const double* __restrict__ Iu_new, const double* __restrict__ IL_new, double* __restrict__ F_h,
                  double* __restrict__ T_h, double* __restrict__ F_c, double lne, double tc,
                  uint32_t* __restrict__ err) {
  // One wavefront per particle: lanes stride over the partners, a butterfly
  // reduction (fixed order) combines them, lane 0 applies the update.
  const int i = blockIdx.x;
  const int lane = threadIdx.x;
  const double L[3] = {(double)d.nx, (double)d.ny, (double)d.nz};
  const double ri = rad[i];
  const double mi = rho_p[i] * (4.0 / 3.0) * kPi * ri * ri * ri;
  const double Ii = 0.4 * mi * ri * ri;
  double Fh[3], Th[3];
  for (int k = 0; k < 3; ++k) {
    // bounce-back: link forces + cover/uncover momentum of the last step;
    // immersed boundary: -sum F_l dV + change of the inner momentum
    if (bc == LBM_BC_IBB) {
      Fh[k] = F_a[3 * i + k] + F_b[3 * i + k];
      Th[k] = T_a[3 * i + k] + T_b[3 * i + k];
    } else {
      Fh[k] = F_a[3 * i + k] + (Iu_new[3 * i + k] - Iu[3 * i + k]);
      Th[k] = T_a[3 * i + k] + (IL_new[3 * i + k] - IL[3 * i + k]);
    }
  }
  double Fc[3] = {0.0, 0.0, 0.0};
  if (motion == LBM_MOTION_FREE) {
    const double Xi[3] = {X[3 * i], X[3 * i + 1], X[3 * i + 2]};
    const double Ui[3] = {U[3 * i], U[3 * i + 1], U[3 * i + 2]};
    for (int j = lane; j < np; j += 64) {
      if (j == i) continue;
      const double dx = min_image(Xi[0] - X[3 * j], L[0]);
      const double dy = min_image(Xi[1] - X[3 * j + 1], L[1]);
      const double dz = min_image(Xi[2] - X[3 * j + 2], L[2]);
      const double dist = sqrt(dist2(dx, dy, dz));
      const double rj = rad[j];
      const double delta = ri + rj - dist;
      if (!(delta > 0.0)) continue;
      if (delta > 0.5 * fmin(ri, rj)) atomicOr(err, kErrOverlap);
      const double n[3] = {dx / dist, dy / dist, dz / dist};
      const double mj = rho_p[j] * (4.0 / 3.0) * kPi * rj * rj * rj;
      const double meff = mi * mj / (mi + mj);
      const double kn = meff * (kPi * kPi + lne * lne) / (tc * tc);
      const double eta = -2.0 * meff * lne / tc;
      const double vn = ((Ui[0] - U[3 * j]) * n[0] + (Ui[1] - U[3 * j + 1]) * n[1]) + (Ui[2] - U[3 * j + 2]) * n[2];
      const double mag = kn * delta - eta * vn;
      Fc[0] += mag * n[0];
      Fc[1] += mag * n[1];
      Fc[2] += mag * n[2];
    }
  }
  for (int k = 0; k < 3; ++k)
    for (int o = 32; o > 0; o >>= 1) Fc[k] += __shfl_xor(Fc[k], o, 64);
  if (lane != 0) return;
  for (int k = 0; k < 3; ++k) {
    double u1 = U[3 * i + k], w1 = Om[3 * i + k];
    if (motion == LBM_MOTION_FREE) {
      u1 = U[3 * i + k] + (Fh[k] + Fc[k]) / mi;
      w1 = Om[3 * i + k] + Th[k] / Ii;
    }
    double x1 = X[3 * i + k];
    if (motion != LBM_MOTION_FIXED) {
      x1 = X[3 * i + k] + 0.5 * (U[3 * i + k] + u1);
      if (x1 >= L[k]) x1 -= L[k];
      if (x1 < 0.0) x1 += L[k];
    }
    Xn[3 * i + k] = x1;
    Un[3 * i + k] = u1;
    Omn[3 * i + k] = w1;
    F_h[3 * i + k] = Fh[k];
    T_h[3 * i + k] = Th[k];
    F_c[3 * i + k] = Fc[k];
    if (bc == LBM_BC_IBM) {
      Iu[3 * i + k] = Iu_new[3 * i + k];
      IL[3 * i + k] = IL_new[3 * i + k];
    }
  }
}

}  // namespace

namespace {

__global__ void __launch_bounds__(256)
k_release_average(const float* __restrict__ u, Dims d, const double* __restrict__ X, const double* __restrict__ rad,
                  double* __restrict__ Uout) {
  const int p = blockIdx.x;
  const double* Xp = X + 3 * p;
  const double r = rad[p];
  const Box b = make_box(Xp, r + 1.0);
  const uint32_t cnt = b.count();
  double s[4] = {0, 0, 0, 0};
  for (uint32_t i = threadIdx.x; i < cnt; i += 256) {
    int x, y, z;
    box_node(b, i, d.nx, d.ny, d.nz, x, y, z);
    const double a = kempe_alpha(min_image((double)x - Xp[0], d.nx), min_image((double)y - Xp[1], d.ny),
                                 min_image((double)z - Xp[2], d.nz), r);
    if (a <= 0.0) continue;
    const uint32_t n = node_index(x, y, z, d.nx, d.ny);
    s[0] += a * (double)u[n];
    s[1] += a * (double)u[(size_t)d.N + n];
    s[2] += a * (double)u[2 * (size_t)d.N + n];
    s[3] += a;
  }
  double t[4];
  for (int k = 0; k < 4; ++k) t[k] = block_sum<256>(s[k]);
  if (threadIdx.x == 0)
    for (int k = 0; k < 3; ++k) Uout[3 * p + k] = t[k] / t[3];
}

template <int STORE>
__global__ void __launch_bounds__(256)
k_release_overwrite(typename Pop<STORE>::T* f, Dims d, const uint32_t* __restrict__ owner,
                    const double* __restrict__ X, const double* __restrict__ rad, const double* __restrict__ U,
                    const double* __restrict__ Om) {
  const uint32_t p = blockIdx.x;
  const double* Xp = X + 3 * p;
  const double* W = Om + 3 * p;
  const Box b = make_box(Xp, rad[p] + 1.0);
  const uint32_t cnt = b.count();
  for (uint32_t i = threadIdx.x; i < cnt; i += 256) {
    int x, y, z;
    box_node(b, i, d.nx, d.ny, d.nz, x, y, z);
    const uint32_t n = node_index(x, y, z, d.nx, d.ny);
    if (owner[n] != p) continue;
    // rigid-body velocity U + Omega x (x - X), minimum image
    const double r0 = min_image((double)x - Xp[0], d.nx), r1 = min_image((double)y - Xp[1], d.ny),
                 r2 = min_image((double)z - Xp[2], d.nz);
    const float ux = (float)(U[3 * p] + (W[1] * r2 - W[2] * r1));
    const float uy = (float)(U[3 * p + 1] + (W[2] * r0 - W[0] * r2));
    const float uz = (float)(U[3 * p + 2] + (W[0] * r1 - W[1] * r0));
    float dr = 0.0f;
    for (int k = 0; k < kQ; ++k) dr += Pop<STORE>::load(f + (size_t)k * d.N + n);
    const float rho = 1.0f + dr;
    for (int k = 0; k < kQ; ++k) Pop<STORE>::store(f + (size_t)k * d.N + n, geq(k, rho, ux, uy, uz));
  }
}

}  // namespace

hipError_t launch_particle_update(const Ctx& c) {
  if (c.np <= 0) return hipSuccess;
  const int pc = c.pcur, pn = 1 - c.pcur;
  const bool ibb = c.cfg.bc == LBM_BC_IBB;
  const double lne = log(c.cfg.coll_restitution);
  hipLaunchKernelGGL(k_particle_update, dim3(c.np), dim3(64), 0, c.stream, c.np, c.motion, c.cfg.bc,
                     c.dims, c.P.X[pc], c.P.U[pc], c.P.Om[pc], c.P.X[pn], c.P.U[pn], c.P.Om[pn], c.P.r, c.P.rho,
                     ibb ? c.P.F_link : c.P.F_ib, ibb ? c.P.T_link : c.P.T_ib, c.P.F_rc, c.P.T_rc, c.P.Iu, c.P.IL,
                     c.P.Iu_new, c.P.IL_new, c.P.F_h, c.P.T_h, c.P.F_c, lne, c.cfg.coll_tc_steps, c.err);
  return hipGetLastError();
}

hipError_t launch_release_average(const Ctx& c, const float* u, double* Uout) {
  if (c.np <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_release_average, dim3(c.np), dim3(256), 0, c.stream, u, c.dims, c.P.X[c.pcur], c.P.r, Uout);
  return hipGetLastError();
}

hipError_t launch_release_overwrite(const Ctx& c, void* f, const uint32_t* owner, const double* U, const double* Om) {
  if (c.np <= 0) return hipSuccess;
  if (c.cfg.store == LBM_STORE_F32)
    hipLaunchKernelGGL(k_release_overwrite<0>, dim3(c.np), dim3(256), 0, c.stream, (float*)f, c.dims, owner,
                       c.P.X[c.pcur], c.P.r, U, Om);
  else
    hipLaunchKernelGGL(k_release_overwrite<1>, dim3(c.np), dim3(256), 0, c.stream, (_Float16*)f, c.dims, owner,
                       c.P.X[c.pcur], c.P.r, U, Om);
  return hipGetLastError();
}

}  // namespace lbm
