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
// Partners are found through a uniform cell grid whose cells are wider than
// 2 max_radius, so a sphere in contact lies in one of the 27 cells around a
// particle's own (periodic); the partners found are then summed in index order.
// Release: U = Kempe-weighted mean of the fluid velocity over the particle,
// Omega = 0, and the populations at the particle's nodes are reset once to the
// equilibrium of the local density and U.
#include "device_util.hpp"
#include "internal.hpp"

namespace lbm {

namespace {

constexpr double kPi = 3.14159265358979323846;

constexpr uint32_t kNoParticle = 0xFFFFFFFFu;
constexpr int kMaxPartners = 64;  // partners collected per particle before the all-pairs fallback

__device__ __forceinline__ int contact_cell_axis(double x, double L, int n) {
  const int c = (int)floor(x * ((double)n / L));
  return c < 0 ? 0 : (c >= n ? n - 1 : c);
}

__device__ __forceinline__ uint32_t contact_cell(const double* Xp, Dims d, int3 cn) {
  const int cx = contact_cell_axis(Xp[0], (double)d.nx, cn.x);
  const int cy = contact_cell_axis(Xp[1], (double)d.ny, cn.y);
  const int cz = contact_cell_axis(Xp[2], (double)d.nz, cn.z);
  return ((uint32_t)cz * (uint32_t)cn.y + (uint32_t)cy) * (uint32_t)cn.x + (uint32_t)cx;
}

__global__ void __launch_bounds__(256) k_cells_clear(uint32_t* __restrict__ head, uint32_t n) {
  const uint32_t i = blockIdx.x * 256u + threadIdx.x;
  if (i < n) head[i] = kNoParticle;
}

// Each particle pushes itself onto its cell's list; the order within a list
// is arbitrary, only the set matters.
__global__ void __launch_bounds__(256)
k_cells_link(int np, Dims d, int3 cn, const double* __restrict__ X, uint32_t* __restrict__ head,
             uint32_t* __restrict__ next) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= np) return;
  next[i] = atomicExch(&head[contact_cell(X + 3 * i, d, cn)], (uint32_t)i);
}

// Overlap of spheres i and j under the minimum image; dx..dz is X_i - X_j.
__device__ __forceinline__ double contact_overlap(const double* Xi, double ri, const double* __restrict__ X,
                                                  const double* __restrict__ rad, int j, const double L[3],
                                                  double& dx, double& dy, double& dz, double& dist) {
  dx = min_image(Xi[0] - X[3 * j], L[0]);
  dy = min_image(Xi[1] - X[3 * j + 1], L[1]);
  dz = min_image(Xi[2] - X[3 * j + 2], L[2]);
  dist = sqrt(dist2(dx, dy, dz));
  return ri + rad[j] - dist;
}

// Adds the contact force of partner j on particle i to Fc.
__device__ __forceinline__ void add_contact(const double* Xi, const double* Ui, double ri, double mi, int j,
                                            const double* __restrict__ X, const double* __restrict__ U,
                                            const double* __restrict__ rad, const double* __restrict__ rho_p,
                                            const double L[3], double lne, double tc, double Fc[3],
                                            uint32_t* __restrict__ err) {
  double dx, dy, dz, dist;
  const double delta = contact_overlap(Xi, ri, X, rad, j, L, dx, dy, dz, dist);
  if (!(delta > 0.0)) return;
  const double rj = rad[j];
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

__global__ void __launch_bounds__(64)
k_particle_update(int np, int motion, int bc, Dims d, int3 cn, const uint32_t* __restrict__ cell_head,
                  const uint32_t* __restrict__ cell_next, const double* __restrict__ X,
                  const double* __restrict__ U, const double* __restrict__ Om, double* __restrict__ Xn,
                  double* __restrict__ Un, double* __restrict__ Omn, const double* __restrict__ rad,
                  const double* __restrict__ rho_p, const double* __restrict__ F_a, const double* __restrict__ T_a,
                  const double* __restrict__ F_b, const double* __restrict__ T_b, double* __restrict__ Iu,
                  double* __restrict__ IL, const double* __restrict__ Iu_new, const double* __restrict__ IL_new,
                  double* __restrict__ F_h, double* __restrict__ T_h, double* __restrict__ F_c, double lne,
                  double tc, uint32_t* __restrict__ err) {
  // One wavefront per particle: each lane walks one neighbouring cell and
  // collects the overlapping partners; lane 0 sorts them by index, sums their
  // forces in that order and applies the update.
  __shared__ int s_count;
  __shared__ int s_partner[kMaxPartners];
  const int i = blockIdx.x;
  const int lane = threadIdx.x;
  const double L[3] = {(double)d.nx, (double)d.ny, (double)d.nz};
  const double ri = rad[i];
  const double mi = rho_p[i] * (4.0 / 3.0) * kPi * ri * ri * ri;
  const double Ii = 0.4 * mi * ri * ri;
  const double Xi[3] = {X[3 * i], X[3 * i + 1], X[3 * i + 2]};
  const double Ui[3] = {U[3 * i], U[3 * i + 1], U[3 * i + 2]};
  double Fc[3] = {0.0, 0.0, 0.0};
  if (motion == LBM_MOTION_FREE) {
    if (lane == 0) s_count = 0;
    __syncthreads();
    // distinct neighbour offsets per axis: -1..1, or fewer when the grid has
    // fewer than three cells along that axis
    const int ax = cn.x < 3 ? cn.x : 3, ay = cn.y < 3 ? cn.y : 3, az = cn.z < 3 ? cn.z : 3;
    if (lane < ax * ay * az) {
      const int ox = lane % ax, oy = (lane / ax) % ay, oz = lane / (ax * ay);
      const int cx0 = contact_cell_axis(Xi[0], L[0], cn.x), cy0 = contact_cell_axis(Xi[1], L[1], cn.y),
                cz0 = contact_cell_axis(Xi[2], L[2], cn.z);
      const int cx = (cx0 + (cn.x >= 3 ? ox - 1 : ox) + cn.x) % cn.x;
      const int cy = (cy0 + (cn.y >= 3 ? oy - 1 : oy) + cn.y) % cn.y;
      const int cz = (cz0 + (cn.z >= 3 ? oz - 1 : oz) + cn.z) % cn.z;
      const uint32_t cell = ((uint32_t)cz * (uint32_t)cn.y + (uint32_t)cy) * (uint32_t)cn.x + (uint32_t)cx;
      for (uint32_t j = cell_head[cell]; j != kNoParticle; j = cell_next[j]) {
        if ((int)j == i) continue;
        double dx, dy, dz, dist;
        if (!(contact_overlap(Xi, ri, X, rad, (int)j, L, dx, dy, dz, dist) > 0.0)) continue;
        const int k = atomicAdd(&s_count, 1);
        if (k < kMaxPartners) s_partner[k] = (int)j;
      }
    }
    __syncthreads();
    if (lane == 0) {
      const int n = s_count;
      if (n <= kMaxPartners) {
        for (int a = 1; a < n; ++a) {
          const int v = s_partner[a];
          int b = a;
          for (; b > 0 && s_partner[b - 1] > v; --b) s_partner[b] = s_partner[b - 1];
          s_partner[b] = v;
        }
        for (int a = 0; a < n; ++a) add_contact(Xi, Ui, ri, mi, s_partner[a], X, U, rad, rho_p, L, lne, tc, Fc, err);
      } else {
        for (int j = 0; j < np; ++j)
          if (j != i) add_contact(Xi, Ui, ri, mi, j, X, U, rad, rho_p, L, lne, tc, Fc, err);
      }
    }
  }
  if (lane != 0) return;
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
      // a position more than one period out (or not finite) comes only from a
      // diverged flow: latch it and keep the geometry kernels in the lattice
      if (!(x1 >= 0.0 && x1 < L[k])) {
        atomicOr(err, kErrUnstable);
        x1 = 0.0;
      }
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
    for (int k = 0; k < kQ; ++k) dr += Pop<STORE>::load(f + (size_t)k * d.S + n);
    const float rho = 1.0f + dr;
    for (int k = 0; k < kQ; ++k) Pop<STORE>::store(f + (size_t)k * d.S + n, geq(k, rho, ux, uy, uz));
  }
}

}  // namespace

hipError_t launch_particle_update(const Ctx& c) {
  if (c.np <= 0) return hipSuccess;
  const int pc = c.pcur, pn = 1 - c.pcur;
  const bool ibb = c.cfg.bc == LBM_BC_IBB;
  const double lne = log(c.cfg.coll_restitution);
  const int3 cn = make_int3(c.P.cells[0], c.P.cells[1], c.P.cells[2]);
  if (c.motion == LBM_MOTION_FREE) {
    const uint32_t ncell = (uint32_t)cn.x * (uint32_t)cn.y * (uint32_t)cn.z;
    hipLaunchKernelGGL(k_cells_clear, dim3((ncell + 255) / 256), dim3(256), 0, c.stream, c.P.cell_head, ncell);
    hipLaunchKernelGGL(k_cells_link, dim3((c.np + 255) / 256), dim3(256), 0, c.stream, c.np, c.dims, cn, c.P.X[pc],
                       c.P.cell_head, c.P.cell_next);
  }
  hipLaunchKernelGGL(k_particle_update, dim3(c.np), dim3(64), 0, c.stream, c.np, c.motion, c.cfg.bc,
                     c.dims, cn, c.P.cell_head, c.P.cell_next, c.P.X[pc], c.P.U[pc], c.P.Om[pc], c.P.X[pn], c.P.U[pn], c.P.Om[pn], c.P.r, c.P.rho,
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
