// d3q19.hpp - D3Q19 lattice and the fused MRT + Guo node update for gfx950.
//
// Model: D3Q19 with the d'Humieres (2002) moment basis and relaxation rates,
// as used for the particle-laden case (Sec. 3.1); Guo forcing in moment
// space for the body force rho*g (Sec. 2.1) and the immersed-boundary force.
//
// Velocity order (this library's own): 0 rest; 1..9 the "positive" half
//   1 (1,0,0)  2 (0,1,0)  3 (0,0,1)  4 (1,1,0)  5 (1,-1,0)
//   6 (1,0,1)  7 (1,0,-1) 8 (0,1,1)  9 (0,1,-1)
// and 10..18 their negatives in the same order, so opposite(i) = i +- 9.
//
// Populations are handled as shifted values g_i = f_i - w_i. With that shift
// every moment below is a small quantity, which keeps FP32 collision and FP16
// storage accurate. The collision works on pair sums s = g_i + g_opp (even
// moments) and pair differences d = g_i - g_opp (odd moments), which halves
// the moment transform; the back-transform uses M^-1 = M^T diag(1/|row|^2)
// because the d'Humieres rows are mutually orthogonal.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbm {

constexpr int kQ = 19;

__host__ __device__ constexpr int cx_of(int i) {
  constexpr int t[19] = {0, 1, 0, 0, 1, 1, 1, 1, 0, 0, -1, 0, 0, -1, -1, -1, -1, 0, 0};
  return t[i];
}
__host__ __device__ constexpr int cy_of(int i) {
  constexpr int t[19] = {0, 0, 1, 0, 1, -1, 0, 0, 1, 1, 0, -1, 0, -1, 1, 0, 0, -1, -1};
  return t[i];
}
__host__ __device__ constexpr int cz_of(int i) {
  constexpr int t[19] = {0, 0, 0, 1, 0, 0, 1, -1, 1, -1, 0, 0, -1, 0, 0, -1, 1, -1, 1};
  return t[i];
}
__host__ __device__ constexpr int opp_of(int i) { return i == 0 ? 0 : (i <= 9 ? i + 9 : i - 9); }
__host__ __device__ constexpr float w_of(int i) {
  return i == 0 ? 1.0f / 3.0f : ((i <= 3 || (i >= 10 && i <= 12)) ? 1.0f / 18.0f : 1.0f / 36.0f);
}

// Relaxation rates for the non-conserved moments.
struct MrtRates {
  float s_nu;   // stress moments 3p_xx, p_ww, p_xy, p_yz, p_xz: 1/tau
  float s_e;    // energy
  float s_eps;  // energy square
  float s_q;    // energy flux
  float s_pi;   // 3pi_xx, pi_ww
  float s_m;    // third-order m_x, m_y, m_z
};

// One MRT + Guo collision in place on shifted populations g[19].
// F: total force density at the node. Returns rho and the half-force
// velocity u = (sum c g + F/2)/rho through the out parameters.
__device__ __forceinline__ void mrt_collide(float (&g)[kQ], float Fx, float Fy, float Fz,
                                            const MrtRates& r, float& rho_out, float& ux_out,
                                            float& uy_out, float& uz_out) {
  float s1 = g[1] + g[10], s2 = g[2] + g[11], s3 = g[3] + g[12];
  float s4 = g[4] + g[13], s5 = g[5] + g[14], s6 = g[6] + g[15];
  float s7 = g[7] + g[16], s8 = g[8] + g[17], s9 = g[9] + g[18];
  float d1 = g[1] - g[10], d2 = g[2] - g[11], d3 = g[3] - g[12];
  float d4 = g[4] - g[13], d5 = g[5] - g[14], d6 = g[6] - g[15];
  float d7 = g[7] - g[16], d8 = g[8] - g[17], d9 = g[9] - g[18];

  const float sf = s1 + s2 + s3;
  const float se = (s4 + s5) + (s6 + s7) + (s8 + s9);
  const float drho = g[0] + sf + se;
  const float rho = 1.0f + drho;
  const float jx = d1 + (d4 + d5) + (d6 + d7);
  const float jy = d2 + (d4 - d5) + (d8 + d9);
  const float jz = d3 + (d6 - d7) + (d8 - d9);
  const float inv_rho = __builtin_amdgcn_rcpf(rho);  // hardware reciprocal, 1 ulp
  const float ux = (jx + 0.5f * Fx) * inv_rho;
  const float uy = (jy + 0.5f * Fy) * inv_rho;
  const float uz = (jz + 0.5f * Fz) * inv_rho;
  const float u2 = ux * ux + uy * uy + uz * uz;
  const float ru2 = rho * u2;

  // Even moments of g (the constant parts of M w cancel against m^eq).
  const float m_e = -30.0f * g[0] - 11.0f * sf + 8.0f * se;
  const float m_eps = 12.0f * g[0] - 4.0f * sf + se;
  const float t47 = (s4 + s5) + (s6 + s7), t89 = s8 + s9;
  const float m_pxx = 2.0f * s1 - s2 - s3 + t47 - 2.0f * t89;
  const float m_Pxx = -4.0f * s1 + 2.0f * (s2 + s3) + t47 - 2.0f * t89;
  const float m_pww = s2 - s3 + (s4 + s5) - (s6 + s7);
  const float m_Pww = -2.0f * (s2 - s3) + (s4 + s5) - (s6 + s7);
  const float m_pxy = s4 - s5, m_pxz = s6 - s7, m_pyz = s8 - s9;
  // Odd non-conserved moments.
  const float m_qx = -4.0f * d1 + (d4 + d5) + (d6 + d7);
  const float m_qy = -4.0f * d2 + (d4 - d5) + (d8 + d9);
  const float m_qz = -4.0f * d3 + (d6 - d7) + (d8 - d9);
  const float m_mx = (d4 + d5) - (d6 + d7);
  const float m_my = (d5 - d4) + (d8 + d9);
  const float m_mz = (d6 - d7) - (d8 - d9);

  // Equilibrium parts and Guo source moments (M Fbar).
  const float uF = ux * Fx + uy * Fy + uz * Fz;
  const float A = 2.0f * ux * Fx - uy * Fy - uz * Fz;
  const float B = uy * Fy - uz * Fz;
  const float X = rho * (3.0f * ux * ux - u2);
  const float Y = rho * (uy * uy - uz * uz);
  const float hnu = 1.0f - 0.5f * r.s_nu, hpi = 1.0f - 0.5f * r.s_pi, hq = 1.0f - 0.5f * r.s_q;

  // a_k = (change of moment k) / |row k|^2.
  const float a_e = (-r.s_e * (m_e + 11.0f * drho - 19.0f * ru2) + (1.0f - 0.5f * r.s_e) * 38.0f * uF) *
                    (1.0f / 2394.0f);
  const float a_eps = (-r.s_eps * (m_eps - 3.0f * drho + 5.5f * ru2) - (1.0f - 0.5f * r.s_eps) * 11.0f * uF) *
                      (1.0f / 252.0f);
  const float a_jx = 0.1f * Fx, a_jy = 0.1f * Fy, a_jz = 0.1f * Fz;
  const float q23 = 2.0f / 3.0f;
  const float a_qx = (-r.s_q * (m_qx + q23 * rho * ux) - hq * q23 * Fx) * (1.0f / 40.0f);
  const float a_qy = (-r.s_q * (m_qy + q23 * rho * uy) - hq * q23 * Fy) * (1.0f / 40.0f);
  const float a_qz = (-r.s_q * (m_qz + q23 * rho * uz) - hq * q23 * Fz) * (1.0f / 40.0f);
  const float a_pxx = (-r.s_nu * (m_pxx - X) + hnu * 2.0f * A) * (1.0f / 36.0f);
  const float a_Pxx = (-r.s_pi * (m_Pxx + 0.5f * X) - hpi * A) * (1.0f / 72.0f);
  const float a_pww = (-r.s_nu * (m_pww - Y) + hnu * 2.0f * B) * (1.0f / 12.0f);
  const float a_Pww = (-r.s_pi * (m_Pww + 0.5f * Y) - hpi * B) * (1.0f / 24.0f);
  const float a_pxy = (-r.s_nu * (m_pxy - rho * ux * uy) + hnu * (ux * Fy + uy * Fx)) * 0.25f;
  const float a_pxz = (-r.s_nu * (m_pxz - rho * ux * uz) + hnu * (ux * Fz + uz * Fx)) * 0.25f;
  const float a_pyz = (-r.s_nu * (m_pyz - rho * uy * uz) + hnu * (uy * Fz + uz * Fy)) * 0.25f;
  const float a_mx = -r.s_m * m_mx * 0.125f;
  const float a_my = -r.s_m * m_my * 0.125f;
  const float a_mz = -r.s_m * m_mz * 0.125f;

  // Back-transform: g~_i = g_i + sum_k M_ki a_k, split into the part even
  // in c (shared by i and opp(i)) and the odd part (sign flips).
  const float ef = -11.0f * a_e - 4.0f * a_eps;
  const float ee = 8.0f * a_e + a_eps;
  const float E0 = -30.0f * a_e + 12.0f * a_eps;
  const float E1 = ef + 2.0f * a_pxx - 4.0f * a_Pxx;
  const float Eyz = ef - a_pxx + 2.0f * a_Pxx;
  const float E2 = Eyz + (a_pww - 2.0f * a_Pww);
  const float E3 = Eyz - (a_pww - 2.0f * a_Pww);
  const float bxe = ee + a_pxx + a_Pxx;
  const float E45 = bxe + a_pww + a_Pww;
  const float E67 = bxe - a_pww - a_Pww;
  const float E89 = ee - 2.0f * (a_pxx + a_Pxx);
  const float O1 = a_jx - 4.0f * a_qx, O2 = a_jy - 4.0f * a_qy, O3 = a_jz - 4.0f * a_qz;
  const float px = a_jx + a_qx, py = a_jy + a_qy, pz = a_jz + a_qz;
  const float O4 = px + py + a_mx - a_my;
  const float O5 = px - py + a_mx + a_my;
  const float O6 = px + pz - a_mx + a_mz;
  const float O7 = px - pz - a_mx - a_mz;
  const float O8 = py + pz + a_my - a_mz;
  const float O9 = py - pz + a_my + a_mz;

  g[0] += E0;
  g[1] += E1 + O1;  g[10] += E1 - O1;
  g[2] += E2 + O2;  g[11] += E2 - O2;
  g[3] += E3 + O3;  g[12] += E3 - O3;
  g[4] += (E45 + a_pxy) + O4;  g[13] += (E45 + a_pxy) - O4;
  g[5] += (E45 - a_pxy) + O5;  g[14] += (E45 - a_pxy) - O5;
  g[6] += (E67 + a_pxz) + O6;  g[15] += (E67 + a_pxz) - O6;
  g[7] += (E67 - a_pxz) + O7;  g[16] += (E67 - a_pxz) - O7;
  g[8] += (E89 + a_pyz) + O8;  g[17] += (E89 + a_pyz) - O8;
  g[9] += (E89 - a_pyz) + O9;  g[18] += (E89 - a_pyz) - O9;

  rho_out = rho;
  ux_out = ux;
  uy_out = uy;
  uz_out = uz;
}

// Shifted equilibrium g_i^eq = f_i^eq(rho, u) - w_i for the compressible
// second-order equilibrium.
__device__ __forceinline__ float geq(int i, float rho, float ux, float uy, float uz) {
  const float cu = cx_of(i) * ux + cy_of(i) * uy + cz_of(i) * uz;
  const float u2 = ux * ux + uy * uy + uz * uz;
  return w_of(i) * ((rho - 1.0f) + rho * (3.0f * cu + 4.5f * cu * cu - 1.5f * u2));
}

// Storage of shifted populations.
template <int STORE> struct Pop;
template <> struct Pop<0> {
  using T = float;
  __device__ static __forceinline__ float load(const T* p) { return *p; }
  __device__ static __forceinline__ void store(T* p, float v) { *p = v; }
  // the bits store() writes
  __device__ static __forceinline__ uint32_t bits(float v) { return __float_as_uint(v); }
  // Streaming store (non-temporal hint): for the fused kernel's output,
  // which no one reads before the next step.
  __device__ static __forceinline__ void store_stream(T* p, float v) { __builtin_nontemporal_store(v, p); }
};
// FP16 holds (f_i - w_i) * 2^14. The power-of-two scale is exact both ways;
// it moves the shifted populations of slow flows (|g| ~ 1e-7 near rest) out
// of the FP16 subnormal range while |g| up to 4 stays finite, so every value
// from ~4e-9 to 4 keeps the full 11-bit significand (round to nearest even).
constexpr float kHalfScale = 16384.0f;
template <> struct Pop<1> {
  using T = _Float16;
  __device__ static __forceinline__ float load(const T* p) { return static_cast<float>(*p) * (1.0f / kHalfScale); }
  __device__ static __forceinline__ void store(T* p, float v) { *p = static_cast<_Float16>(v * kHalfScale); }
  // the bits store() writes
  __device__ static __forceinline__ uint32_t bits(float v) {
    return (uint32_t)__builtin_bit_cast(uint16_t, static_cast<_Float16>(v * kHalfScale));
  }
  __device__ static __forceinline__ void store_stream(T* p, float v) {
    __builtin_nontemporal_store(static_cast<_Float16>(v * kHalfScale), p);
  }
};

}  // namespace lbm
