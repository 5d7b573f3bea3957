// d3q27.hpp - D3Q27 lattice of the turbulent-pipe solver (Sec. 2.2) and its
// node update.
//
// The pipe runs use a D3Q27 MRT model with one relaxation parameter for all
// moments (bulk viscosity equal to shear viscosity), with the option of a
// longer relaxation time for the energy mode to damp acoustic noise. With one
// rate the moment-space collision is BGK; the energy mode |c|^2 - 1 is one row
// of a weight-orthogonal basis, so relaxing it at omega_e instead of omega
// adds to the BGK result the term
//   -(omega_e - omega) [(m_e - m_e^eq) + (u.F)] (3/2) w_i (|c_i|^2 - 1),
// m_e = sum_i (|c_i|^2 - 1) f_i, m_e^eq = rho u.u, where u.F is the energy
// moment of the Guo source, 3/2 = 1 / sum_i w_i (|c_i|^2 - 1)^2, and the
// Guo factor (1 - S/2) is applied per mode.
//
// Velocity order (this library's own): 0 rest; 1..13 one vector of each
// opposite pair
//   1 (1,0,0)  2 (0,1,0)  3 (0,0,1)  4 (1,1,0)  5 (1,-1,0)  6 (1,0,1)
//   7 (1,0,-1) 8 (0,1,1)  9 (0,1,-1) 10 (1,1,1) 11 (1,1,-1) 12 (1,-1,1)
//   13 (1,-1,-1)
// and 14..26 their negatives in the same order, so opposite(i) = i +- 13.
// Weights 8/27, 2/27, 1/54, 1/216 for |c|^2 = 0, 1, 2, 3. Populations are
// stored shifted, g_i = f_i - w_i, in FP32.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbm {
namespace q27 {

constexpr int kQ = 27;

__host__ __device__ constexpr int cx(int i) {
  constexpr int t[27] = {0,  1, 0, 0,  1, 1,  1,  1,  0,  0, 1,  1,  1,  1,
                         -1, 0, 0, -1, -1, -1, -1, 0, 0, -1, -1, -1, -1};
  return t[i];
}
__host__ __device__ constexpr int cy(int i) {
  constexpr int t[27] = {0, 0,  1, 0, 1,  -1, 0, 0, 1,  1,  1,  1, -1, -1,
                         0, -1, 0, -1, 1, 0,  0, -1, -1, -1, -1, 1, 1};
  return t[i];
}
__host__ __device__ constexpr int cz(int i) {
  constexpr int t[27] = {0, 0, 0, 1,  0, 0, 1,  -1, 1, -1, 1,  -1, 1, -1,
                         0, 0, -1, 0, 0, -1, 1, -1, 1, -1, 1,  -1, 1};
  return t[i];
}
__host__ __device__ constexpr int opp(int i) { return i == 0 ? 0 : (i <= 13 ? i + 13 : i - 13); }
__host__ __device__ constexpr int c2(int i) { return cx(i) * cx(i) + cy(i) * cy(i) + cz(i) * cz(i); }
__host__ __device__ constexpr float w(int i) {
  return c2(i) == 0 ? 8.0f / 27.0f : (c2(i) == 1 ? 2.0f / 27.0f : (c2(i) == 2 ? 1.0f / 54.0f : 1.0f / 216.0f));
}

struct Rates {
  float omega;    // 1 / tau: every non-conserved moment but the energy mode
  float omega_e;  // 1 / tau_bulk: the energy mode
};

// One collision in place on shifted populations g[27] under force density F;
// returns rho and the half-force velocity u = (sum c g + F/2) / rho.
__device__ __forceinline__ void collide(float (&g)[kQ], float Fx, float Fy, float Fz, const Rates& r, float& rho_out,
                                        float& ux_out, float& uy_out, float& uz_out) {
  float drho = g[0], jx = 0.0f, jy = 0.0f, jz = 0.0f, me = -g[0];
#pragma unroll
  for (int i = 1; i <= 13; ++i) {
    const float s = g[i] + g[i + 13], d = g[i] - g[i + 13];
    drho += s;
    jx += (float)cx(i) * d;
    jy += (float)cy(i) * d;
    jz += (float)cz(i) * d;
    me += (float)(c2(i) - 1) * s;
  }
  const float rho = 1.0f + drho;
  const float inv_rho = __builtin_amdgcn_rcpf(rho);  // hardware reciprocal, 1 ulp
  const float ux = (jx + 0.5f * Fx) * inv_rho;
  const float uy = (jy + 0.5f * Fy) * inv_rho;
  const float uz = (jz + 0.5f * Fz) * inv_rho;
  const float u2 = ux * ux + uy * uy + uz * uz;
  const float uF = ux * Fx + uy * Fy + uz * Fz;
  const float om = r.omega, keep = 1.0f - om, h = 1.0f - 0.5f * om;
  // energy-mode correction per unit w_i (|c_i|^2 - 1)
  const float de = -1.5f * (r.omega_e - om) * ((me - rho * u2) + uF);
  const float base = om * (drho - 1.5f * rho * u2) - 3.0f * h * uF;  // even part shared by every direction
  g[0] = keep * g[0] + w(0) * (base - de);
#pragma unroll
  for (int i = 1; i <= 13; ++i) {
    const float cu = (float)cx(i) * ux + (float)cy(i) * uy + (float)cz(i) * uz;
    const float cF = (float)cx(i) * Fx + (float)cy(i) * Fy + (float)cz(i) * Fz;
    const float even = w(i) * (base + cu * (4.5f * om * rho * cu + 9.0f * h * cF) + (float)(c2(i) - 1) * de);
    const float odd = w(i) * 3.0f * (om * rho * cu + h * cF);
    g[i] = keep * g[i] + (even + odd);
    g[i + 13] = keep * g[i + 13] + (even - odd);
  }
  rho_out = rho;
  ux_out = ux;
  uy_out = uy;
  uz_out = uz;
}

// Shifted equilibrium g_i^eq = f_i^eq(rho, u) - w_i.
__device__ __forceinline__ float geq(int i, float rho, float ux, float uy, float uz) {
  const float cu = (float)cx(i) * ux + (float)cy(i) * uy + (float)cz(i) * uz;
  const float u2 = ux * ux + uy * uy + uz * uz;
  return w(i) * ((rho - 1.0f) + rho * (3.0f * cu + 4.5f * cu * cu - 1.5f * u2));
}

}  // namespace q27
}  // namespace lbm
