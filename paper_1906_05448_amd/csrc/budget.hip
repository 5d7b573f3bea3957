// budget.hip - moment sums of the component-wise turbulent kinetic energy
// budget of the pipe in cylindrical coordinates (Sec. 2.2, Eq. (1a)-(1c)).
//
// Per fluid node (r^2 < R^2 about the axis (cx, cy)), from the masked
// velocity and its central-difference gradient G_ij = d_j u_i (the
// statistics' operator) and p = rho / 3: the cylindrical components
// (u_r, u_theta, u_z), the physical components of the velocity-gradient
// tensor L_ab = e_a . G . e_b and the strain s_ab = (L_ab + L_ba) / 2, with
// e_r = (x_perp - c) / r (e_x on the axis), e_theta = e_z x e_r. The 38
// sums of the products Eq. (1) needs (lbm.h lists them) are taken per
// radial bin [k w, (k + 1) w): one workgroup per (bin, chunk of kPbZ z
// planes) walks the bin's (x, y) list, which the host built once, over its
// planes, sums in FP64 and reduces in a fixed order; the chunks are then
// added in order into the accumulator. The budget terms follow from the
// accumulated sums on the host.
#include "device_util.hpp"
#include "internal.hpp"
#include "stats_device.hpp"

namespace lbm {

namespace {

constexpr int kPbBlock = 256;
constexpr int kPbZ = 4;  // z planes per workgroup
constexpr int kPbM = LBM_PIPE_BUDGET_MOMENTS;

int pb_chunks(int nz) { return (nz + kPbZ - 1) / kPbZ; }

__global__ void __launch_bounds__(kPbBlock)
k_pb_nodes(const float* __restrict__ u, const float* __restrict__ rho, const uint32_t* __restrict__ key,
           const double* __restrict__ X, const double* __restrict__ U, const double* __restrict__ Om, Dims d,
           double cx, double cy, const uint32_t* __restrict__ list, const uint32_t* __restrict__ off, int nbins,
           int nchunks, double* __restrict__ part) {
  const int k = (int)(blockIdx.x % (uint32_t)nbins);
  const int ch = (int)(blockIdx.x / (uint32_t)nbins);
  const int z0 = ch * kPbZ, nzc = min(kPbZ, d.nz - z0);
  const MaskedVel vel{u, key, X, U, Om, d};
  double s[kPbM];
#pragma unroll
  for (int i = 0; i < kPbM; ++i) s[i] = 0.0;
  // thread t takes the (list entry, plane) pairs t, t + kPbBlock, ... of the
  // chunk, entries fastest
  const uint32_t cnt = off[k + 1] - off[k], total = cnt * (uint32_t)nzc;
  for (uint32_t t = threadIdx.x; t < total; t += kPbBlock) {
    const uint32_t zq = t / cnt;
    const int z = z0 + (int)zq;
    const uint32_t xy = list[off[k] + (t - zq * cnt)];
    const int x = (int)(xy & 0xFFFFu), y = (int)(xy >> 16);
    const uint32_t n = node_index(x, y, z, d.nx, d.ny);
    const double dx = (double)x - cx, dy = (double)y - cy;
    const double r = sqrt(dy * dy + dx * dx);
    const double er0 = r > 0.0 ? dx / r : 1.0, er1 = r > 0.0 ? dy / r : 0.0;
    const double E[3][3] = {{er0, er1, 0.0}, {-er1, er0, 0.0}, {0.0, 0.0, 1.0}};  // rows e_r, e_theta, e_z
    double v[3], G[3][3];
    vel.at(n, v);
    velocity_gradient(vel, neighbours(n, d), G);
    const double p = (double)rho[n] / 3.0;
    double uc[3], L[3][3], S[3][3];
    for (int a = 0; a < 3; ++a) uc[a] = (E[a][0] * v[0] + E[a][1] * v[1]) + E[a][2] * v[2];
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) {
        double t = 0.0;
        for (int i = 0; i < 3; ++i)
          for (int jj = 0; jj < 3; ++jj) t += E[a][i] * G[i][jj] * E[b][jj];
        L[a][b] = t;
      }
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) S[a][b] = 0.5 * (L[a][b] + L[b][a]);
    const double ur = uc[0], ut = uc[1], uz = uc[2];
    const double q[kPbM] = {1.0, ur, ut, uz, p,
                            S[0][0], S[0][1], S[0][2], S[1][1], S[1][2], S[2][2],
                            L[2][0], L[2][1], L[2][2], L[0][0], L[0][1], L[0][2], L[1][1], L[1][0], L[1][2],
                            uz * ur, ur * ur, ut * ur, uz * uz, ut * ut,
                            p * ur, p * L[2][2], p * L[0][0], p * L[1][1],
                            uz * S[2][0], ur * S[0][0], ut * S[1][0],
                            (S[2][0] * L[2][0] + S[2][1] * L[2][1]) + S[2][2] * L[2][2],
                            (S[0][0] * L[0][0] + S[0][1] * L[0][1]) + S[0][2] * L[0][2],
                            (S[1][1] * L[1][1] + S[1][0] * L[1][0]) + S[1][2] * L[1][2],
                            uz * uz * ur, ur * ur * ur, ut * ut * ur};
#pragma unroll
    for (int i = 0; i < kPbM; ++i) s[i] += q[i];
  }
  // fixed-order reduction: butterfly within each wavefront, then the
  // wavefront sums in order
  __shared__ double ws[kPbBlock / 64][kPbM];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int i = 0; i < kPbM; ++i) {
    double t = s[i];
    for (int o = 32; o > 0; o >>= 1) t += __shfl_xor(t, o, 64);
    if (lane == 0) ws[wave][i] = t;
  }
  __syncthreads();
  if (threadIdx.x < kPbM) {
    double t = 0.0;
    for (int w = 0; w < kPbBlock / 64; ++w) t += ws[w][threadIdx.x];
    part[((size_t)k * nchunks + ch) * kPbM + threadIdx.x] = t;
  }
}

// acc[m][k] += sum over the chunks of part[k][chunk][m], in order.
__global__ void __launch_bounds__(256)
k_pb_reduce(const double* __restrict__ part, int nbins, int nchunks, double* __restrict__ acc) {
  const int i = (int)(blockIdx.x * 256u + threadIdx.x);
  if (i >= kPbM * nbins) return;
  const int m = i / nbins, k = i % nbins;
  double t = 0.0;
  for (int ch = 0; ch < nchunks; ++ch) t += part[((size_t)k * nchunks + ch) * kPbM + m];
  acc[(size_t)m * nbins + k] += t;
}

}  // namespace

size_t pipe_budget_part_bytes(const Ctx& c, int nbins) {
  return (size_t)nbins * (size_t)pb_chunks(c.dims.nz) * kPbM * sizeof(double);
}

hipError_t launch_pipe_budget_add(const Ctx& c, const float* u, const float* rho, const uint32_t* key,
                                  double* part) {
  const int nbins = c.pb.nbins;
  const int pc = c.pcur;
  const int nch = pb_chunks(c.dims.nz);
  hipLaunchKernelGGL(k_pb_nodes, dim3((uint32_t)nbins * (uint32_t)nch), dim3(kPbBlock), 0, c.stream, u, rho, key,
                     c.P.X[pc], c.P.U[pc], c.P.Om[pc], c.dims, c.cfg.pipe_cx, c.cfg.pipe_cy, c.pb.list, c.pb.off,
                     nbins, nch, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_pb_reduce, dim3((kPbM * nbins + 255) / 256), dim3(256), 0, c.stream, part, nbins, nch,
                     c.pb.acc);
  return hipGetLastError();
}

}  // namespace lbm
