// Cell-local algebra of the two-component step, shared by the z-marching
// kernels: densities from stored sums, the mixture velocity (Eqs. 4-6), the
// Shan-Chen neighbour sum (Eq. 7), the BGK collision with the exact-difference
// force term (Eqs. 2-3, Sec. 2), the regularized collision (Eqs. 10-11) and
// the rounding of post-collision populations into the 16-bit storage forms.
#pragma once

#include "launch.h"

namespace lbm {

// rho^a from a stored sum D (the sum of the 19 stored values of a species
// at a cell as read back by the pull).
template <Storage S>
__device__ __forceinline__ float density(float d, float shift) {
  if constexpr (StorageTraits<S>::shifted) {
    return d + shift;
  } else {
    return d;
  }
}

// Row of a row block that holds direction i of species s; i = Q stands for
// the residual of the rest population (16-bit forms only, launch.h).
__host__ __device__ constexpr int store_row(int s, int i) { return i < Q ? s * Q + i : RES_ROW + s; }

// Store of one species' post-collision populations f* in the 16-bit forms:
// the 18 moving populations are rounded as f*_i - w_i rho_shift, and the rest
// population takes the stored remainder e = D - sum_{i>0} decode(q_i), so
// that the stored values of the cell still sum to D and the density is not
// drifted by the rounding of the others.  The remainder is kept in two 16-bit
// values, q_0 = round(e) and the residual round((e - decode(q_0)) s) with s =
// res_scale, which read back as decode(q_0) + decode(residual) / s: the
// rounding left in the stored sum (and in the mass) is
// then that of the residual, 2^-11 (FP16) or 2^-8 (BF16) times that of a
// single value.  A single rounding of the rest population drifted the mass
// by 1e-2 (FP16) over 2000 steps of a droplet that persists, where the field
// keeps changing slowly and the roundings of successive steps are
// correlated.  `put(i, q)` receives the stored value of direction i, with
// i = Q for the residual.
template <Storage S, typename Put>
__device__ __forceinline__ void encode_species(const float f[Q], float d, const float ws[3], Put put) {
  using Tr = StorageTraits<S>;
  float dsum = 0.0f;
#pragma unroll
  for (int i = 1; i < Q; ++i) {
    const auto q = Tr::encode(f[i] - ws[i <= 6 ? 1 : 2]);
    const float back = Tr::decode(q);
    dsum = i == 1 ? back : dsum + back;
    put(i, q);
  }
  const float e = d - dsum;
  const auto q0 = Tr::encode(e);
  put(0, q0);
  put(Q, Tr::encode((e - Tr::decode(q0)) * Tr::res_scale));
}

// ---------------------------------------------------------------------------
// Cell-local algebra
// ---------------------------------------------------------------------------

// Pair k (0..8) holds directions 2k+1 (velocity p_k) and 2k+2 (-p_k):
// p = (1,0,0) (0,1,0) (0,0,1) (1,1,0) (1,-1,0) (1,0,1) (1,0,-1) (0,1,1) (0,1,-1).
__device__ __forceinline__ void pair_dots(float vx, float vy, float vz, float cv[9]) {
  cv[0] = vx; cv[1] = vy; cv[2] = vz;
  cv[3] = vx + vy; cv[4] = vx - vy;
  cv[5] = vx + vz; cv[6] = vx - vz;
  cv[7] = vy + vz; cv[8] = vy - vz;
}

__device__ __forceinline__ constexpr float pair_w(int k) { return k < 3 ? WF : WE; }

// Everything a cell needs from its neighbourhood and its populations.
struct Local {
  float rho[2];  // rho^A, rho^B (Eq. 4)
  float rinv;    // 1 / rho (Eq. 5)
  float u[3];    // mixture velocity (Eq. 6)
  float S[2][3]; // sum_i w_i c_i rho~^b(x + c_i) for b = A, B (Eq. 7)
  float g[2][3]; // g^a = sum_b G^{ab} S^b (force per unit mass, Sec. 2)
};

// Mixture velocity of Eq. (6) from the pulled populations: u = j / rho.
__device__ __forceinline__ void mixture_velocity(const float f[2][Q], float rho, float u[3]) {
  float d[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) d[k] = (f[0][2 * k + 1] + f[1][2 * k + 1]) - (f[0][2 * k + 2] + f[1][2 * k + 2]);
  const float rinv = 1.0f / rho;
  u[0] = (d[0] + d[3] + d[4] + d[5] + d[6]) * rinv;
  u[1] = (d[1] + d[3] - d[4] + d[7] + d[8]) * rinv;
  u[2] = (d[2] + d[5] - d[6] + d[7] - d[8]) * rinv;
}

// Shan-Chen neighbour sum S^b(x) = sum_i w_i c_i rho~^b(x + c_i) (Eq. 7) from
// the LDS density ring, in two parts.  `at` is the cell's position in a ring
// plane (row stride EX).  The partial sum takes the 13 neighbours in planes
// z-1 (pm) and z (p0); the finish adds the 5 in plane z+1 (pp).  The scalar
// forms do one component (one species at one cell); ring entries hold
// (rho~^A, rho~^B) of one cell (float2) or of the two cells of a folded word
// (float4), and every component goes through the same scalar form.
__device__ __forceinline__ void sc_partial_c(float a, float b, float c, float d, float e, float f, float g, float h,
                                             float m0, float mx, float mxm, float my, float mym, float S[3]) {
  // in plane: faces (w = 1/18) and xy edges (w = 1/36); plane below: c_z = -1
  S[0] = fmaf(WF, a - b, WE * (((e + f) - (g + h)) + (mx - mxm)));
  S[1] = fmaf(WF, c - d, WE * (((e + g) - (f + h)) + (my - mym)));
  S[2] = -fmaf(WF, m0, WE * ((mx + mxm) + (my + mym)));
}

__device__ __forceinline__ void sc_finish_c(float p0, float px, float pxm, float py, float pym, float S[3]) {
  S[0] = fmaf(WE, px - pxm, S[0]);
  S[1] = fmaf(WE, py - pym, S[1]);
  S[2] += fmaf(WF, p0, WE * ((px + pxm) + (py + pym)));
}

// Component k of a ring entry.
__device__ __forceinline__ float comp(const float2& v, int k) { return k == 0 ? v.x : v.y; }
__device__ __forceinline__ float comp(const float4& v, int k) {
  return k == 0 ? v.x : (k == 1 ? v.y : (k == 2 ? v.z : v.w));
}

// S[k][c]: component c of the ring entries, axis k.
template <int EX, int NC, typename V>
__device__ __forceinline__ void shan_chen_partial(const V* pm, const V* p0, int at, float S[NC][3]) {
  auto R = [&](const V* pl, int dy, int dx) { return pl[at + dy * EX + dx]; };
  const V a = R(p0, 0, 1), b = R(p0, 0, -1), c = R(p0, 1, 0), d = R(p0, -1, 0);
  const V e = R(p0, 1, 1), f = R(p0, -1, 1), g = R(p0, 1, -1), h = R(p0, -1, -1);
  const V m0 = R(pm, 0, 0), mx = R(pm, 0, 1), mxm = R(pm, 0, -1), my = R(pm, 1, 0), mym = R(pm, -1, 0);
#pragma unroll
  for (int k = 0; k < NC; ++k)
    sc_partial_c(comp(a, k), comp(b, k), comp(c, k), comp(d, k), comp(e, k), comp(f, k), comp(g, k), comp(h, k),
                 comp(m0, k), comp(mx, k), comp(mxm, k), comp(my, k), comp(mym, k), S[k]);
}

template <int EX, int NC, typename V>
__device__ __forceinline__ void shan_chen_finish(const V* pp, int at, float S[NC][3]) {
  auto R = [&](int dy, int dx) { return pp[at + dy * EX + dx]; };
  const V p0 = R(0, 0), px = R(0, 1), pxm = R(0, -1), py = R(1, 0), pym = R(-1, 0);
#pragma unroll
  for (int k = 0; k < NC; ++k) sc_finish_c(comp(p0, k), comp(px, k), comp(pxm, k), comp(py, k), comp(pym, k), S[k]);
}

__device__ __forceinline__ void make_local(const float rho_a, const float rho_b, const float u[3],
                                           const float S[2][3], const Phys& ph, Local& L) {
  L.rho[0] = rho_a;
  L.rho[1] = rho_b;
  L.rinv = 1.0f / (rho_a + rho_b);
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    L.u[k] = u[k];
    L.S[0][k] = S[0][k];
    L.S[1][k] = S[1][k];
    L.g[0][k] = ph.g_ab * S[1][k];  // g^A = G^{AB} S^B
    L.g[1][k] = ph.g_ba * S[0][k];  // g^B = G^{BA} S^A
  }
}

// BGK collision (Eq. 2) plus the exact-difference forcing term, in place:
//   f*_i = (1 - w) f_i + w_i rho^a [(w - 1) P_i(u) + P_i(u + g^a)],  w = 1/tau_a,
// with P the bracket of Eq. (3) at T0 = 1/3,
//   P(v) = 1 + 3 cv + 4.5 cv^2 - 1.5 vv + 4.5 cv^3 - 4.5 cv vv,
// evaluated per opposite pair as P(+-p_k) = even +- odd in cv.
__device__ __forceinline__ float pair_dot(int k, float vx, float vy, float vz) {
  switch (k) {
    case 0: return vx;
    case 1: return vy;
    case 2: return vz;
    case 3: return vx + vy;
    case 4: return vx - vy;
    case 5: return vx + vz;
    case 6: return vx - vz;
    case 7: return vy + vz;
    default: return vy - vz;
  }
}

__device__ __forceinline__ void collide(float f[2][Q], const Local& L, const Phys& ph) {
  const float ux = L.u[0], uy = L.u[1], uz = L.u[2];
  const float uu = fmaf(ux, ux, fmaf(uy, uy, uz * uz));
  const float au = fmaf(-1.5f, uu, 1.0f);
  const float bu = fmaf(-4.5f, uu, 3.0f);
  float vx[2], vy[2], vz[2], av[2], bv[2], om1[2], keep[2], r[2];
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    vx[s] = ux + L.g[s][0];
    vy[s] = uy + L.g[s][1];
    vz[s] = uz + L.g[s][2];
    const float vv = fmaf(vx[s], vx[s], fmaf(vy[s], vy[s], vz[s] * vz[s]));
    av[s] = fmaf(-1.5f, vv, 1.0f);
    bv[s] = fmaf(-4.5f, vv, 3.0f);
    om1[s] = ph.omega[s] - 1.0f;
    keep[s] = 1.0f - ph.omega[s];
    r[s] = L.rho[s];
  }
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    const float cu = pair_dot(k, ux, uy, uz);
    const float tu = cu * cu;
    const float eu = fmaf(4.5f, tu, au);
    const float ou = cu * fmaf(4.5f, tu, bu);
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      const float cv = pair_dot(k, vx[s], vy[s], vz[s]);
      const float tv = cv * cv;
      const float ke = fmaf(om1[s], eu, fmaf(4.5f, tv, av[s]));
      const float ko = fmaf(om1[s], ou, cv * fmaf(4.5f, tv, bv[s]));
      const float wr = pair_w(k) * r[s];
      f[s][2 * k + 1] = fmaf(keep[s], f[s][2 * k + 1], wr * (ke + ko));
      f[s][2 * k + 2] = fmaf(keep[s], f[s][2 * k + 2], wr * (ke - ko));
    }
  }
  // Collision and forcing leave rho^a unchanged (sum_i w_i P_i(v) = 1).  The
  // rest population is written as the remainder rho^a - sum_{i>0} f*_i, which
  // equals (1 - w) f_0 + w_0 rho^a [(w - 1) P_0(u) + P_0(v^a)] in exact
  // arithmetic; in FP32 it keeps the rounding of the weights 1/3, 1/18, 1/36
  // (their FP32 values sum to 1 + 3e-8) from creating mass every step.
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    float moving = f[s][1];
#pragma unroll
    for (int i = 2; i < Q; ++i) moving += f[s][i];
    f[s][0] = r[s] - moving;
  }
}

// Regularized collision, Eqs. (10)-(11): f* = E(rho^a, u + g^a) +
// (1 - w) f^neq with f^neq the Hermite projection of the non-equilibrium part
// f - E(rho^a, u):
//   momentum flux   w_i (c_i c_i - T0 I) : Pi^a / (2 T0^2), with
//                   Pi^a = sum_i c_i c_i f_i - rho^a (T0 I + u u) (the second
//                   moment of Eq. 3 is exactly rho (T0 I + u u) on D3Q19);
//                   even in c_i, so both members of a pair get it;
//   energy flux     (ENERGY only) w_i H_i . q / (2 T0^3) with the contracted
//                   third-order polynomials H_{i,a} = sum_{b != a} (c_a c_b^2
//                   - T0 c_a) and q_a = sum_i H_{i,a} (f_i - E_i(rho^a, u));
//                   odd in c_i.  2 T0^3 is the polynomials' norm on D3Q19.
// The rest population is again the remainder rho^a - sum_{i>0} f*_i.
template <bool ENERGY = false>
__device__ __forceinline__ void collide_regularized(float f[2][Q], const Local& L, const Phys& ph) {
  const float ux = L.u[0], uy = L.u[1], uz = L.u[2];
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    const float r = L.rho[s];
    float e[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) e[k] = f[s][2 * k + 1] + f[s][2 * k + 2];
    const float rt = r * T0F;
    const float pxx = (((e[0] + e[3]) + (e[4] + e[5])) + e[6]) - fmaf(r * ux, ux, rt);
    const float pyy = (((e[1] + e[3]) + (e[4] + e[7])) + e[8]) - fmaf(r * uy, uy, rt);
    const float pzz = (((e[2] + e[5]) + (e[6] + e[7])) + e[8]) - fmaf(r * uz, uz, rt);
    const float pxy = (e[3] - e[4]) - (r * ux) * uy;
    const float pxz = (e[5] - e[6]) - (r * ux) * uz;
    const float pyz = (e[7] - e[8]) - (r * uy) * uz;
    const float tt = T0F * ((pxx + pyy) + pzz);
    float h[9];  // c . Pi . c - T0 tr(Pi) for pair k
    h[0] = pxx - tt;
    h[1] = pyy - tt;
    h[2] = pzz - tt;
    h[3] = fmaf(2.0f, pxy, pxx + pyy) - tt;
    h[4] = fmaf(-2.0f, pxy, pxx + pyy) - tt;
    h[5] = fmaf(2.0f, pxz, pxx + pzz) - tt;
    h[6] = fmaf(-2.0f, pxz, pxx + pzz) - tt;
    h[7] = fmaf(2.0f, pyz, pyy + pzz) - tt;
    h[8] = fmaf(-2.0f, pyz, pyy + pzz) - tt;
    // Energy flux: odd part o_k = w_k H_k . q / (2 T0^3) of pair k, from the
    // pair differences of f - E(rho^a, u) (E's odd part is
    // 2 w rho cu (3 + 4.5 cu^2 - 4.5 uu)).  On D3Q19, H_k is -2/3 along the
    // axis of a face pair and 1/3 per non-zero component of an edge pair.
    float o[9];
    if constexpr (ENERGY) {
      const float uu = fmaf(ux, ux, fmaf(uy, uy, uz * uz));
      const float bu = fmaf(-4.5f, uu, 3.0f);
      float d[9];
#pragma unroll
      for (int k = 0; k < 9; ++k) {
        const float cu = pair_dot(k, ux, uy, uz);
        const float eo = (2.0f * pair_w(k) * r) * (cu * fmaf(4.5f, cu * cu, bu));
        d[k] = (f[s][2 * k + 1] - f[s][2 * k + 2]) - eo;
      }
      const float third = 1.0f / 3.0f;
      const float qx = fmaf(-2.0f * third, d[0], third * ((d[3] + d[4]) + (d[5] + d[6])));
      const float qy = fmaf(-2.0f * third, d[1], third * ((d[3] - d[4]) + (d[7] + d[8])));
      const float qz = fmaf(-2.0f * third, d[2], third * ((d[5] - d[6]) + (d[7] - d[8])));
      const float keep = 1.0f - ph.omega[s];
      // 13.5 w_k (H_k . q): -0.5 q_a for the face pairs, 0.125 (q_a +- q_b) for the edges
      o[0] = keep * (-0.5f * qx);
      o[1] = keep * (-0.5f * qy);
      o[2] = keep * (-0.5f * qz);
      o[3] = keep * (0.125f * (qx + qy));
      o[4] = keep * (0.125f * (qx - qy));
      o[5] = keep * (0.125f * (qx + qz));
      o[6] = keep * (0.125f * (qx - qz));
      o[7] = keep * (0.125f * (qy + qz));
      o[8] = keep * (0.125f * (qy - qz));
    }
    const float vx = ux + L.g[s][0], vy = uy + L.g[s][1], vz = uz + L.g[s][2];
    const float vv = fmaf(vx, vx, fmaf(vy, vy, vz * vz));
    const float av = fmaf(-1.5f, vv, 1.0f);
    const float bv = fmaf(-4.5f, vv, 3.0f);
    const float keep45 = 4.5f * (1.0f - ph.omega[s]);  // (1 - w) / (2 T0^2)
    float moving = 0.0f;
#pragma unroll
    for (int k = 0; k < 9; ++k) {
      const float cv = pair_dot(k, vx, vy, vz);
      const float tv = cv * cv;
      const float ev = fmaf(4.5f, tv, av);
      const float ov = cv * fmaf(4.5f, tv, bv);
      const float w = pair_w(k);
      const float neq = w * (keep45 * h[k]);
      if constexpr (ENERGY) {
        f[s][2 * k + 1] = fmaf(w * r, ev + ov, neq + o[k]);
        f[s][2 * k + 2] = fmaf(w * r, ev - ov, neq - o[k]);
      } else {
        f[s][2 * k + 1] = fmaf(w * r, ev + ov, neq);
        f[s][2 * k + 2] = fmaf(w * r, ev - ov, neq);
      }
      moving += f[s][2 * k + 1] + f[s][2 * k + 2];
    }
    f[s][0] = r - moving;
  }
}

}  // namespace lbm
