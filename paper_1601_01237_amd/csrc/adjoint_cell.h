// Cell-local part of the reverse (adjoint) step: the transpose of the
// collision of Eqs. (2)-(3) (BGK) or Eqs. (10)-(11) (regularized) with the
// exact-difference force term and the Shan-Chen force of Eq. (7), at one
// cell whose forward quantities (rho^a, u, g^a) are known.
#pragma once

#include "cell.h"
#include "launch.h"

namespace lbm {

// Transposed collision of one cell (reverse mode of Eqs. 2-3 and 7).
// With lam = dL/df* at this cell and K_i = (w-1) P_i(u) + P_i(v^a):
//   rho_bar^a = sum_i lam_i w_i K_i
//   u_bar     = sum_a rho^a sum_i lam_i w_i [(w-1) dP_i(u) + dP_i(v^a)]
//   g_bar^a   = rho^a sum_i lam_i w_i dP_i(v^a)
// where dP_i(v) = c_i (3 + 9 cv + 13.5 cv^2 - 4.5 vv) - v (3 + 9 cv).
// The local part of dL/df_k^a is (1-w) lam_k + a^a + b . c_k with
//   a^a = rho_bar^a - u_bar . u / rho,  b = u_bar / rho       (written to mo)
// and the transpose of the Eq. (7) gather needs Sbar^B = G^{AB} g_bar^A,
// Sbar^A = G^{BA} g_bar^B (written to sb).  acc += dL/dG (tied), dL/dtau_a.
// The populations f enter only through dot^a = sum_i lam_i f_i^a.
__device__ __forceinline__ constexpr int pair_cx(int k) { return (k == 0 || (k >= 3 && k <= 6)) ? 1 : 0; }
__device__ __forceinline__ constexpr int pair_cy(int k) {
  return (k == 1 || k == 3 || k == 7 || k == 8) ? 1 : (k == 4 ? -1 : 0);
}
__device__ __forceinline__ constexpr int pair_cz(int k) {
  return (k == 2 || k == 5 || k == 7) ? 1 : ((k == 6 || k == 8) ? -1 : 0);
}

// Species part of the transposed collision: rho_bar^a, g_bar^a and the
// species' share of u_bar and of dL/dtau_a, from lam^a (19 values) and dot^a.
struct AdjointSums {
  float ubar[3];
  float rbar[2];
  float gbar[2][3];
  float dtau[2];
};

//
// With REG (regularized collision) only the E(rho^a, v^a) part is summed
// here (om1 = 0 drops the E(rho^a, u) weights); adjoint_species_reg adds the
// pullback through the projected flux and dL/dtau_a.
template <bool REG = false>
__device__ __forceinline__ void adjoint_species(int s, float dot, const float lam[Q], const Local& L,
                                                const Phys& ph, AdjointSums& A) {
  const float* u = L.u;
  const float uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
  float cu[9];
  pair_dots(u[0], u[1], u[2], cu);
  const float v[3] = {u[0] + L.g[s][0], u[1] + L.g[s][1], u[2] + L.g[s][2]};
  const float vv = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
  float cv[9];
  pair_dots(v[0], v[1], v[2], cv);
  const float om = ph.omega[s];
  const float om1 = REG ? 0.0f : om - 1.0f;
  const float r = L.rho[s];
  const float l0 = lam[0] * W0;
  const float pu0 = 1.0f - 1.5f * uu;
  const float pv0 = 1.0f - 1.5f * vv;
  float rb = l0 * (om1 * pu0 + pv0);
  float bu = 3.0f * l0, bv = 3.0f * l0;
  float au[3] = {0.f, 0.f, 0.f}, av[3] = {0.f, 0.f, 0.f};
  float le = l0 * pu0;  // sum_i lam_i E_i(rho^a, u) / rho^a
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    const float w = pair_w(k);
    const float lp = lam[2 * k + 1] * w;
    const float lm = lam[2 * k + 2] * w;
    const float tu = cu[k] * cu[k];
    const float tv = cv[k] * cv[k];
    const float evu = pu0 + 4.5f * tu;
    const float odu = cu[k] * (3.0f - 4.5f * uu + 4.5f * tu);
    const float evv = pv0 + 4.5f * tv;
    const float odv = cv[k] * (3.0f - 4.5f * vv + 4.5f * tv);
    const float pup = evu + odu, pum = evu - odu;
    const float pvp = evv + odv, pvm = evv - odv;
    rb += lp * (om1 * pup + pvp) + lm * (om1 * pum + pvm);
    const float aue = 3.0f + 13.5f * tu - 4.5f * uu, auo = 9.0f * cu[k];
    const float ave = 3.0f + 13.5f * tv - 4.5f * vv, avo = 9.0f * cv[k];
    const float qu = lp * (aue + auo) - lm * (aue - auo);
    const float qv = lp * (ave + avo) - lm * (ave - avo);
    bu += lp * (3.0f + auo) + lm * (3.0f - auo);
    bv += lp * (3.0f + avo) + lm * (3.0f - avo);
    if (pair_cx(k)) { au[0] += pair_cx(k) * qu; av[0] += pair_cx(k) * qv; }
    if (pair_cy(k)) { au[1] += pair_cy(k) * qu; av[1] += pair_cy(k) * qv; }
    if (pair_cz(k)) { au[2] += pair_cz(k) * qu; av[2] += pair_cz(k) * qv; }
    le += lp * pup + lm * pum;
  }
  // dL/dtau_a = sum_i lam_i (f_i - E_i(rho^a, u)) / tau_a^2
  const float dt = dot - r * le;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    A.gbar[s][a] = r * (av[a] - v[a] * bv);
    A.ubar[a] += r * (om1 * (au[a] - u[a] * bu) + (av[a] - v[a] * bv));
  }
  A.rbar[s] = rb;
  A.dtau[s] = REG ? 0.0f : om * om * dt;
}

// Regularized collision (Sec. 3, Eqs. 10-11): f*_i = E_i(rho, v) + (1 - w)
// w_i (c_i c_i - T0 I) : Pi / (2 T0^2) with Pi = sum_j c_j c_j f_j - rho (T0 I
// + u u).  With B = sum_i lam_i w_i (c_i c_i - T0 I) / (2 T0^2) and
// Pbar = (1 - w) B, dL = Pbar : dPi adds
//   to dL/df_k   c_k c_k : Pbar        (pb, per pair of directions)
//   to rho_bar  -(T0 tr Pbar + u . Pbar u)
//   to u_bar    -2 rho Pbar u
// and dL/dtau_a = (Pi : B) / tau^2.  pb = (xx, yy, zz, xy, xz, yz) of Pbar.
__device__ __forceinline__ void adjoint_species_reg(int s, const float lam[Q], const float f[Q], const Local& L,
                                                    const Phys& ph, AdjointSums& A, float pb[6]) {
  const float ux = L.u[0], uy = L.u[1], uz = L.u[2];
  const float r = L.rho[s];
  float e[9], fe[9];
  float sl = lam[0] * W0;
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    e[k] = (lam[2 * k + 1] + lam[2 * k + 2]) * pair_w(k);
    fe[k] = f[2 * k + 1] + f[2 * k + 2];
    sl += e[k];
  }
  const float bxx = 4.5f * ((((e[0] + e[3]) + (e[4] + e[5])) + e[6]) - T0F * sl);
  const float byy = 4.5f * ((((e[1] + e[3]) + (e[4] + e[7])) + e[8]) - T0F * sl);
  const float bzz = 4.5f * ((((e[2] + e[5]) + (e[6] + e[7])) + e[8]) - T0F * sl);
  const float bxy = 4.5f * (e[3] - e[4]);
  const float bxz = 4.5f * (e[5] - e[6]);
  const float byz = 4.5f * (e[7] - e[8]);
  // Pi of the forward (pre-collision populations of the cell)
  const float rt = r * T0F;
  const float pxx = (((fe[0] + fe[3]) + (fe[4] + fe[5])) + fe[6]) - fmaf(r * ux, ux, rt);
  const float pyy = (((fe[1] + fe[3]) + (fe[4] + fe[7])) + fe[8]) - fmaf(r * uy, uy, rt);
  const float pzz = (((fe[2] + fe[5]) + (fe[6] + fe[7])) + fe[8]) - fmaf(r * uz, uz, rt);
  const float pxy = (fe[3] - fe[4]) - (r * ux) * uy;
  const float pxz = (fe[5] - fe[6]) - (r * ux) * uz;
  const float pyz = (fe[7] - fe[8]) - (r * uy) * uz;
  const float om = ph.omega[s];
  A.dtau[s] = om * om * (pxx * bxx + pyy * byy + pzz * bzz + 2.0f * (pxy * bxy + pxz * bxz + pyz * byz));
  const float keep = 1.0f - om;
  pb[0] = keep * bxx;
  pb[1] = keep * byy;
  pb[2] = keep * bzz;
  pb[3] = keep * bxy;
  pb[4] = keep * bxz;
  pb[5] = keep * byz;
  const float px = pb[0] * ux + pb[3] * uy + pb[4] * uz;  // Pbar u
  const float py = pb[3] * ux + pb[1] * uy + pb[5] * uz;
  const float pz = pb[4] * ux + pb[5] * uy + pb[2] * uz;
  A.rbar[s] -= T0F * (pb[0] + pb[1] + pb[2]) + (ux * px + uy * py + uz * pz);
  A.ubar[0] -= 2.0f * r * px;
  A.ubar[1] -= 2.0f * r * py;
  A.ubar[2] -= 2.0f * r * pz;
}

// Third-order reading of the filter (R22): N_i also holds w_i H_i . q / N
// with the energy-flux polynomials H_i = h_k c_i (h_k = -2 T0 on the faces,
// T0 on the edges; H_0 = 0), N = 2 T0^3 their norm and q = sum_j H_j (f_j -
// E_j(rho, u)), linear in f - E(rho, u) as Pi is.  With B_E = sum_i lam_i w_i
// H_i / N and qb = (1 - w) B_E, dL = qb . dq adds
//   to dL/df_k   H_k . qb               (odd: +- h_k c_k . qb per pair)
//   through the weights -H_j . qb of E_j(rho, u): to rho_bar and u_bar the
//   pullback of sum_j w_j (-H_j . qb) rho P_j(u) (only the odd part of P)
// and dL/dtau_a gains (q . B_E) / tau^2.
__device__ __forceinline__ constexpr float pair_h(int k) { return k < 3 ? -2.0f * T0F : T0F; }

__device__ __forceinline__ void adjoint_species_energy(int s, const float lam[Q], const float f[Q], const Local& L,
                                                       const Phys& ph, AdjointSums& A, float qb[3]) {
  const float* u = L.u;
  const float uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
  float cu[9];
  pair_dots(u[0], u[1], u[2], cu);
  const float r = L.rho[s];
  float be[3] = {0.f, 0.f, 0.f}, q[3] = {0.f, 0.f, 0.f}, odd[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    const float w = pair_w(k);
    odd[k] = cu[k] * (3.0f - 4.5f * uu + 4.5f * cu[k] * cu[k]);  // (P_k+ - P_k-) / 2 at u
    const float dl = (lam[2 * k + 1] - lam[2 * k + 2]) * (w * pair_h(k));
    const float dq = pair_h(k) * ((f[2 * k + 1] - f[2 * k + 2]) - 2.0f * w * r * odd[k]);
    if (pair_cx(k)) { be[0] += pair_cx(k) * dl; q[0] += pair_cx(k) * dq; }
    if (pair_cy(k)) { be[1] += pair_cy(k) * dl; q[1] += pair_cy(k) * dq; }
    if (pair_cz(k)) { be[2] += pair_cz(k) * dl; q[2] += pair_cz(k) * dq; }
  }
  constexpr float inv_norm = 1.0f / (2.0f * T0F * T0F * T0F);
  const float om = ph.omega[s];
  const float keep = 1.0f - om;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    be[a] *= inv_norm;
    qb[a] = keep * be[a];
  }
  A.dtau[s] += om * om * (q[0] * be[0] + q[1] * be[1] + q[2] * be[2]);
  float ub[3] = {0.f, 0.f, 0.f};
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    const float cq = pair_cx(k) * qb[0] + pair_cy(k) * qb[1] + pair_cz(k) * qb[2];
    const float m2w = -2.0f * pair_h(k) * cq * pair_w(k);  // 2 w_k times the weight of E_k+ (E_k- takes minus it)
    A.rbar[s] += m2w * odd[k];
    const float e = 3.0f - 4.5f * uu + 13.5f * cu[k] * cu[k];
    const float o = 9.0f * cu[k];
    if (pair_cx(k)) ub[0] += m2w * pair_cx(k) * e;
    if (pair_cy(k)) ub[1] += m2w * pair_cy(k) * e;
    if (pair_cz(k)) ub[2] += m2w * pair_cz(k) * e;
#pragma unroll
    for (int a = 0; a < 3; ++a) ub[a] -= m2w * o * u[a];
  }
#pragma unroll
  for (int a = 0; a < 3; ++a) A.ubar[a] += r * ub[a];
}

// H_k . qb for pair k's first direction (the second takes minus it).
__device__ __forceinline__ float pair_hq(int k, const float qb[3]) {
  return pair_h(k) * (pair_cx(k) * qb[0] + pair_cy(k) * qb[1] + pair_cz(k) * qb[2]);
}

// c_k c_k : Pbar for pair k (both of its directions).
__device__ __forceinline__ float pair_quad(int k, const float pb[6]) {
  switch (k) {
    case 0: return pb[0];
    case 1: return pb[1];
    case 2: return pb[2];
    case 3: return (pb[0] + pb[1]) + 2.0f * pb[3];
    case 4: return (pb[0] + pb[1]) - 2.0f * pb[3];
    case 5: return (pb[0] + pb[2]) + 2.0f * pb[4];
    case 6: return (pb[0] + pb[2]) - 2.0f * pb[4];
    case 7: return (pb[1] + pb[2]) + 2.0f * pb[5];
    default: return (pb[1] + pb[2]) - 2.0f * pb[5];
  }
}

// Cell outputs once both species are in: mo = (a^A, a^B, b), sb = Sbar, and
// the parameter sums.
__device__ __forceinline__ void adjoint_finish(const AdjointSums& A, const Local& L, const Phys& ph, float mo[5],
                                               float sb[6], double acc[3]) {
  const float* u = L.u;
  const float ubu = A.ubar[0] * u[0] + A.ubar[1] * u[1] + A.ubar[2] * u[2];
  mo[0] = A.rbar[0] - ubu * L.rinv;
  mo[1] = A.rbar[1] - ubu * L.rinv;
  mo[2] = A.ubar[0] * L.rinv;
  mo[3] = A.ubar[1] * L.rinv;
  mo[4] = A.ubar[2] * L.rinv;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    sb[a] = ph.g_ba * A.gbar[1][a];
    sb[3 + a] = ph.g_ab * A.gbar[0][a];
  }
  acc[0] += static_cast<double>(A.gbar[0][0] * L.S[1][0] + A.gbar[0][1] * L.S[1][1] + A.gbar[0][2] * L.S[1][2]) +
            static_cast<double>(A.gbar[1][0] * L.S[0][0] + A.gbar[1][1] * L.S[0][1] + A.gbar[1][2] * L.S[0][2]);
  acc[1] += A.dtau[0];
  acc[2] += A.dtau[1];
}

}  // namespace lbm
