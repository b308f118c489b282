// Fused z-marching kernels of the two-component D3Q19 step (gfx950).
//
// One workgroup owns a tile of BX x ROWS cells in the x-y plane and marches
// up a chunk of z planes.  For each new plane it pulls the 38 populations of
// its cells (Eq. 1 in pull form, with halfway bounce-back at walls, Sec. 4)
// and reduces the species densities rho^A, rho^B (Eq. 4) into a 5-slot LDS
// ring that also holds a one-cell halo of the tile.  Separate halo waves
// recompute the halo densities from the populations around the tile, in
// step with the owner waves' pulls, so no density field ever travels through
// HBM.  Once plane z+1 is in the ring, plane z has every neighbour density the
// Shan-Chen sum of Eq. (7) needs, and the cell update (Eqs. 2-9) runs from the
// populations the owner thread kept in registers.
//
// The same march serves three bodies:
//   Step     collide and store X_{t+1}(x) = f*(x)  (post-collision state);
//   Moments  rho^a and u_F fields plus FP64 per-workgroup diagnostic sums;
//   Adjoint  per-cell transposed collision (see below) for one reverse step.
//
// Memory layout: row blocks of Grid::brows rows per z plane, each holding
// the rows of all 38 populations (launch.h; pos(x) = x except on folded
// 16-bit rows, see buffer.h), so each population load of a 64-wide row is
// one contiguous 256-byte run (FP32), the 38 population rows of a few y rows
// are one contiguous range and one z plane is one contiguous block;
// population blocks are padded (Grid::pstride) so that they are not a power
// of two apart.  Blocks are remapped
// so that the tiles dispatched to one XCD (block id mod 8) are contiguous in
// x and y and share that XCD's L2 for the halo re-reads.

#include "buffer.h"
#include "cell.h"
#include "launch.h"

namespace lbm {

// Pull of Eq. (1): f_i(x) = X_i(x - c_i), or X_opp(i)(x) when x - c_i is a
// wall cell (bit i of `links`).  rz[k] covers z plane z - 1 + k; `ppb` is the
// byte size of one population plane, so population (a, i) of a plane starts
// at (19 a + i) * pp.  Every load is scalar resource + scalar population
// offset + per-lane (y, x) offset.
//
// Returns the species' stored sum D: rho^a itself for FP32; for the shifted
// 16-bit forms the sum of the stored deviations X_i - w_i rho_shift, so that
// rho^a = D + rho_shift (the weights sum to one) and the store can keep the
// stored sum of a cell equal to D.  Both sums run in direction order.
template <Storage S, bool WALLS>
__device__ __forceinline__ float pull_species(const __amdgpu_buffer_rsrc_t rz[3], uint32_t ppb, const Column& c,
                                              uint32_t links, const float ws[3], int s, float f[Q]) {
  using Tr = StorageTraits<S>;
  using T = typename Tr::T;
  const uint32_t own = c.y[1] + c.x[1];
  float d = 0.0f;
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const uint32_t off = c.y[1 - CY[i]] + c.x[1 - CX[i]];
    T v;
    if constexpr (WALLS) {
      if ((i != 0) && ((links >> i) & 1u)) {
        v = buf_load<T, LOAD_BOUNCE>(rz[1], own, static_cast<uint32_t>(s * Q + opp(i)) * ppb);
      } else {
        v = buf_load<T>(rz[1 - CZ[i]], off, static_cast<uint32_t>(s * Q + i) * ppb);
      }
    } else {
      v = buf_load<T>(rz[1 - CZ[i]], off, static_cast<uint32_t>(s * Q + i) * ppb);
    }
    const float x = Tr::decode(v);
    d = i == 0 ? x : d + x;
    if constexpr (Tr::shifted) {
      f[i] = x + ws[i == 0 ? 0 : (i <= 6 ? 1 : 2)];
    } else {
      f[i] = x;
    }
  }
  return d;
}

template <Storage S, bool WALLS>
__device__ __forceinline__ void pull(const __amdgpu_buffer_rsrc_t rz[3], uint32_t ppb, const Column& c,
                                     uint32_t links, const float ws[2][3], float f[2][Q], float d[2]) {
#pragma unroll
  for (int s = 0; s < 2; ++s) d[s] = pull_species<S, WALLS>(rz, ppb, c, links, ws[s], s, f[s]);
}

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

// ---------------------------------------------------------------------------
// Wave / block reductions (fixed order, deterministic)
// ---------------------------------------------------------------------------
template <int NV>
__device__ __forceinline__ void block_reduce_store(double (&v)[NV], const bool (&is_max)[NV],
                                                   double* out, double* scratch) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int nwaves = blockDim.x >> 6;
#pragma unroll
  for (int k = 0; k < NV; ++k) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      const double w = __shfl_xor(v[k], o, 64);
      v[k] = is_max[k] ? fmax(v[k], w) : v[k] + w;
    }
  }
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) scratch[wave * NV + k] = v[k];
  }
  __syncthreads();
  if (threadIdx.x < NV) {
    const int k = threadIdx.x;
    double acc = scratch[k];
    for (int w = 1; w < nwaves; ++w) {
      const double x = scratch[w * NV + k];
      acc = is_max[k] ? fmax(acc, x) : acc + x;
    }
    out[k] = acc;
  }
}

__device__ __forceinline__ float min_image(float d, float n) { return d - n * rintf(d / n); }

// ---------------------------------------------------------------------------
// The march
// ---------------------------------------------------------------------------

// Workgroup shape: BXT x ROWS "own" lanes (one cell column each, a multiple of
// 64) followed by HW "halo" waves that compute the densities of the one-cell
// ring around the tile.  Own waves keep the pulled populations of planes z
// and z+1 in registers.  The density ring has 5 slots: plane p_k (the k-th
// plane a workgroup loads) lives in slot k % 5.  There is one barrier per
// plane (k >= 1): before barrier k the own waves have written their cells of
// p_k and the halo waves the ring of p_0 .. p_k; after it the own waves
// finish plane p_{k-1} (needs p_{k-2} .. p_k), start the Shan-Chen sum of p_k
// from p_{k-1} and p_k and pull p_{k+1}, while the halo waves fill p_{k+1}
// into slot (k+1) % 5, whose last reader finished before barrier k-2.  The
// halo waves thus read the rows around the tile in the same interval as the
// neighbouring tiles' own waves read them as their own rows, while those
// lines are still in L2 (two planes ahead, the FP32 step read 1.37-1.44x its
// algorithmic bytes; in step, 1.09-1.17x).
template <int BXT, int ROWS, int HW>
struct Shape {
  static constexpr int NOWN = BXT * ROWS;
  static constexpr int EX = BXT + 2;
  static constexpr int EY = ROWS + 2;
  static constexpr int NH = 2 * EX + 2 * ROWS;
  static constexpr int NT = NOWN + 64 * HW;
  static constexpr int HPL = (NH + 64 * HW - 1) / (64 * HW);  // halo cells per halo lane
  static constexpr int SLOTS = 5;
  static_assert(NOWN % 64 == 0, "own lanes fill whole waves");
};

// Ring position of halo cell h: bottom row, top row, left column, right column.
template <int BXT, int ROWS>
__device__ __forceinline__ void halo_pos(int h, int& hx, int& hy) {
  constexpr int EX = BXT + 2;
  if (h < EX) { hx = h - 1; hy = -1; }
  else if (h < 2 * EX) { hx = h - EX - 1; hy = ROWS; }
  else if (h < 2 * EX + ROWS) { hx = -1; hy = h - 2 * EX; }
  else { hx = BXT; hy = h - 2 * EX - ROWS; }
}

template <Storage S, bool WALLS, Mode M, int BXT, int ROWS, int HW, bool REG>
__global__ void __launch_bounds__(BXT * ROWS + 64 * HW)
march_kernel(const Grid g, const Phys ph, const Tiling tl, const MarchIO io) {
  using Sh = Shape<BXT, ROWS, HW>;
  using Tr = StorageTraits<S>;
  using T = typename Tr::T;
  constexpr int EX = Sh::EX;
  constexpr int PLANE = Sh::EX * Sh::EY;
  __shared__ float2 ring[Sh::SLOTS * PLANE];
  __shared__ double red[(Sh::NT / 64) * 16];

  const int tid = threadIdx.x;
  const int b = xcd_remap(blockIdx.x, gridDim.x);
  const int tiles_xy = tl.tiles_x * tl.tiles_y;
  // Block order: without walls, an XCD's blocks are whole x-y planes of tiles
  // of one z chunk (neighbouring tiles share their border rows in L2).  With
  // walls the work of a chunk depends on the geometry (solid cells are
  // skipped), so each XCD takes every chunk of its tiles instead, which keeps
  // the XCDs evenly loaded (measured: 5% on the inclined channel, 2% slower
  // on open boxes).
  const int bz = WALLS ? b % tl.tiles_z : b / tiles_xy;
  const int rem = WALLS ? b / tl.tiles_z : b - bz * tiles_xy;
  const int byy = rem / tl.tiles_x;
  const int bxx = rem - byy * tl.tiles_x;
  const int x0 = bxx * BXT, y0 = byy * ROWS, z0 = bz * tl.zchunk;
  const int z1 = min(z0 + tl.zchunk, g.nz);
  const int kmax = z1 - z0 + 1;  // planes p_k = z0 - 1 + k for k = 0..kmax

  const uint64_t n = g.n;
  const uint32_t ppb = g.pstride * static_cast<uint32_t>(sizeof(T));  // bytes between population planes

  float ws[2][3];
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    ws[s][0] = W0 * ph.shift[s];
    ws[s][1] = WF * ph.shift[s];
    ws[s][2] = WE * ph.shift[s];
  }

  constexpr int NV = (M == Mode::Moments) ? 16 : 3;
  double acc[NV];
#pragma unroll
  for (int k = 0; k < NV; ++k) acc[k] = 0.0;

  if (tid < Sh::NOWN) {
    // ------------------------------------------------------------ own waves
    const int tx = tid % BXT, ty = tid / BXT;
    const int ex = x0 + tx, ey = y0 + ty;
    const bool owner = ex < g.nx && ey < g.ny;  // ragged edge lanes only feed the ring
    const Column col = make_column<T>(ex, ey, g);
    const uint32_t col_b = col.y[1] + col.x[1];
    const uint32_t col_off = col.cell;
    const int at = (ty + 1) * EX + tx + 1;

    float cur[2][Q], nxt[2][Q];
    float cur_d[2] = {0.f, 0.f}, nxt_d[2] = {0.f, 0.f};  // stored sums D (pull_species)
    float cur_u[3] = {0.f, 0.f, 0.f}, nxt_u[3] = {0.f, 0.f, 0.f};
    float cur_S[2][3], nxt_S[2][3];  // Shan-Chen sums [species][axis] from planes z-1 and z
#pragma unroll
    for (int c = 0; c < 3; ++c) cur_S[0][c] = cur_S[1][c] = nxt_S[0][c] = nxt_S[1][c] = 0.f;
    uint32_t cur_links = 0, nxt_links = 0;
    int slot = 0;  // k % 5

    for (int k = 0; k <= kmax; ++k) {
      const int p = z0 - 1 + k;
      const int zw = wrap(p, g.nz);
      __amdgpu_buffer_rsrc_t rz[3];
      rz[0] = plane_rsrc<T>(io.src, wrap(p - 1, g.nz), g);
      rz[1] = plane_rsrc<T>(io.src, zw, g);
      rz[2] = plane_rsrc<T>(io.src, wrap(p + 1, g.nz), g);
      if constexpr (WALLS) nxt_links = io.links[static_cast<uint32_t>(zw) * g.nxy + col_off];
      const bool solid = WALLS && (nxt_links & 1u);
      if (!solid) {
        pull<S, WALLS>(rz, ppb, col, nxt_links, ws, nxt, nxt_d);
        const float ra = density<S>(nxt_d[0], ph.shift[0]);
        const float rb = density<S>(nxt_d[1], ph.shift[1]);
        ring[slot * PLANE + at] = make_float2(ra, rb);
        mixture_velocity(nxt, ra + rb, nxt_u);
      } else {
        ring[slot * PLANE + at] = make_float2(ph.rho_wall[0], ph.rho_wall[1]);
      }

      if constexpr (M == Mode::Adjoint) {
        // Finish u here: computed after the barrier it would keep all 38
        // pulled values alive through the adjoint body.
        asm volatile("" ::"v"(nxt_u[0]), "v"(nxt_u[1]), "v"(nxt_u[2]));
      }
      if (k >= 1) {
        __syncthreads();
        const int sm1 = slot >= 1 ? slot - 1 : slot + 4;  // (k-1) % 5
        if (k >= 2) {
          const int z = p - 1;
          const int zc = wrap(z, g.nz);
          const bool csolid = WALLS && (cur_links & 1u);
          const uint32_t cell = static_cast<uint32_t>(zc) * g.nxy + col_off;
          if (owner) {
            if constexpr (M == Mode::Step) {
              if (!csolid) {
                shan_chen_finish<EX, 2>(ring + slot * PLANE, at, cur_S);
                Local L;
                make_local(density<S>(cur_d[0], ph.shift[0]), density<S>(cur_d[1], ph.shift[1]), cur_u, cur_S,
                           ph, L);
                if constexpr (REG) {
                  collide_regularized(cur, L, ph);
                } else {
                  collide(cur, L, ph);
                }
                const __amdgpu_buffer_rsrc_t rd = plane_rsrc<T>(io.dst, zc, g);
#pragma unroll
                for (int s = 0; s < 2; ++s) {
                  if constexpr (Tr::shifted) {
                    encode_species<S>(cur[s], cur_d[s], ws[s], [&](int i, T q) {
                      buf_store<T>(q, rd, col_b, static_cast<uint32_t>(s * Q + i) * ppb);
                    });
                  } else {
#pragma unroll
                    for (int i = 0; i < Q; ++i)
                      buf_store<T>(Tr::encode(cur[s][i]), rd, col_b, static_cast<uint32_t>(s * Q + i) * ppb);
                  }
                }
              }
            } else if constexpr (M == Mode::Moments) {
              float ra = 0.f, rb = 0.f, uf[3] = {0.f, 0.f, 0.f};
              if (!csolid) {
                shan_chen_finish<EX, 2>(ring + slot * PLANE, at, cur_S);
                Local L;
                make_local(density<S>(cur_d[0], ph.shift[0]), density<S>(cur_d[1], ph.shift[1]), cur_u, cur_S,
                           ph, L);
                ra = L.rho[0];
                rb = L.rho[1];
                // u_F = u + g/2, g = sum_a rho^a g^a / rho  (Eqs. 8-9)
#pragma unroll
                for (int c = 0; c < 3; ++c)
                  uf[c] = L.u[c] + 0.5f * (ra * L.g[0][c] + rb * L.g[1][c]) * L.rinv;
                const double rho = static_cast<double>(ra) + static_cast<double>(rb);
                acc[0] += ra;
                acc[1] += rb;
                acc[2] += rho * uf[0];
                acc[3] += rho * uf[1];
                acc[4] += rho * uf[2];
                const double sp = sqrt(static_cast<double>(uf[0]) * uf[0] + static_cast<double>(uf[1]) * uf[1] +
                                       static_cast<double>(uf[2]) * uf[2]);
                const bool finite = isfinite(ra) && isfinite(rb) && isfinite(uf[0]) && isfinite(uf[1]) &&
                                    isfinite(uf[2]);
                acc[5] = fmax(acc[5], finite ? sp : 0.0);
                acc[6] += finite ? 0.0 : 1.0;
                acc[7] += 1.0;
                const Region& R = io.region;
                const float dx = min_image(static_cast<float>(col_off % g.nx) - R.cx, static_cast<float>(g.nx));
                const float dy = min_image(static_cast<float>(col_off / g.nx) - R.cy, static_cast<float>(g.ny));
                const float dz = min_image(static_cast<float>(zc) - R.cz, static_cast<float>(g.nz));
                const float r2 = dx * dx + dy * dy + dz * dz;
                const double pr = (1.0 / 3.0) * rho - static_cast<double>(R.p_g) * (1.0 / 3.0) *
                                                          static_cast<double>(ra) * static_cast<double>(rb);
                if (r2 < R.r_in2) { acc[8] += pr; acc[9] += 1.0; }
                if (r2 > R.r_out2) { acc[10] += pr; acc[11] += 1.0; }
                if (ra > R.thr) { acc[12] += 1.0; acc[13] += dx; acc[14] += dy; acc[15] += dz; }
              }
              if (io.rho_out) {
                io.rho_out[cell] = ra;
                io.rho_out[n + cell] = rb;
              }
              if (io.uf_out) {
                io.uf_out[cell] = uf[0];
                io.uf_out[n + cell] = uf[1];
                io.uf_out[2 * n + cell] = uf[2];
              }
            } else {  // Mode::Adjoint
              float mo[5] = {0.f, 0.f, 0.f, 0.f, 0.f};
              float sb[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
              if (!csolid) {
                shan_chen_finish<EX, 2>(ring + slot * PLANE, at, cur_S);
                Local L;
                make_local(density<S>(cur_d[0], ph.shift[0]), density<S>(cur_d[1], ph.shift[1]), cur_u, cur_S,
                           ph, L);
                // One species at a time: lam^a = dL/dX at the cell, and the
                // populations of plane z, pulled again (cache hits) rather
                // than held in registers since they were first read.
                const __amdgpu_buffer_rsrc_t rl = plane_rsrc<float>(io.lam, zc, g);
                __amdgpu_buffer_rsrc_t rc[3];
                rc[0] = plane_rsrc<T>(io.src, wrap(z - 1, g.nz), g);
                rc[1] = plane_rsrc<T>(io.src, zc, g);
                rc[2] = rz[1];
                AdjointSums A;
#pragma unroll
                for (int c = 0; c < 3; ++c) A.ubar[c] = 0.0f;
                float pb[2][6];
#pragma unroll
                for (int s = 0; s < 2; ++s) {
                  float lam[Q], fs[Q];
#pragma unroll
                  for (int i = 0; i < Q; ++i)
                    lam[i] = buf_load<float>(rl, col_b, static_cast<uint32_t>(s * Q + i) * ppb);
                  pull_species<S, WALLS>(rc, ppb, col, cur_links, ws[s], s, fs);
                  if constexpr (REG) {
                    adjoint_species<true>(s, 0.0f, lam, L, ph, A);
                    adjoint_species_reg(s, lam, fs, L, ph, A, pb[s]);
                  } else {
                    float dot = lam[0] * fs[0];
#pragma unroll
                    for (int i = 1; i < Q; ++i) dot = fmaf(lam[i], fs[i], dot);
                    adjoint_species(s, dot, lam, L, ph, A);
                  }
                  // keep the next species' loads below this one's arithmetic
                  __builtin_amdgcn_sched_barrier(0);
                }
                adjoint_finish(A, L, ph, mo, sb, acc);
                if constexpr (REG) {
                  // The direct term c_k c_k : Pbar^a of dL/df, one value per
                  // pair (both directions share it), in the rows of the
                  // pair's first direction; the stream pass pulls it in place
                  // of lam, and A, b stay in the m fields as for BGK.
                  const __amdgpu_buffer_rsrc_t rdb = plane_rsrc<float>(io.dbar, zc, g);
#pragma unroll
                  for (int s = 0; s < 2; ++s)
#pragma unroll
                    for (int k = 0; k < 9; ++k)
                      buf_store<float>(pair_quad(k, pb[s]), rdb, col_b, static_cast<uint32_t>(s * Q + 2 * k + 1) * ppb);
                }
              } else if constexpr (REG) {
                const __amdgpu_buffer_rsrc_t rdb = plane_rsrc<float>(io.dbar, zc, g);
#pragma unroll
                for (int s = 0; s < 2; ++s)
#pragma unroll
                  for (int k = 0; k < 9; ++k)
                    buf_store<float>(0.0f, rdb, col_b, static_cast<uint32_t>(s * Q + 2 * k + 1) * ppb);
              }
#pragma unroll
              for (int c = 0; c < 5; ++c) io.m[c * n + cell] = mo[c];
#pragma unroll
              for (int c = 0; c < 6; ++c) io.sbar[c * n + cell] = sb[c];
            }
          }
        }
        // Planes p_{k-1} and p_k are complete: the first part of S for plane p_k.
        if (k < kmax) shan_chen_partial<EX, 2>(ring + sm1 * PLANE, ring + slot * PLANE, at, nxt_S);
      }

#pragma unroll
      for (int s = 0; s < 2; ++s) {
        if constexpr (M != Mode::Adjoint) {
#pragma unroll
          for (int i = 0; i < Q; ++i) cur[s][i] = nxt[s][i];
        }
        cur_d[s] = nxt_d[s];
      }
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        cur_u[c] = nxt_u[c];
        cur_S[0][c] = nxt_S[0][c];
        cur_S[1][c] = nxt_S[1][c];
      }
      cur_links = nxt_links;
      slot = slot == 4 ? 0 : slot + 1;
    }
  } else {
    // ----------------------------------------------------------- halo waves
    // Halo lane l owns ring cells l, l + 64 HW, l + 128 HW, ... (HPL of them).
    const int hl = tid - Sh::NOWN;
    int hat[Sh::HPL];
    Column hcol[Sh::HPL];
    uint32_t hcol_off[Sh::HPL];
    bool has[Sh::HPL];
#pragma unroll
    for (int j = 0; j < Sh::HPL; ++j) {
      const int h = hl + j * 64 * HW;
      has[j] = h < Sh::NH;
      int hx = 0, hy = 0;
      halo_pos<BXT, ROWS>(has[j] ? h : 0, hx, hy);
      hcol[j] = make_column<T>(x0 + hx, y0 + hy, g);
      hcol_off[j] = hcol[j].cell;
      hat[j] = (hy + 1) * EX + hx + 1;
    }

    auto halo_plane = [&](int k) {
      const int p = z0 - 1 + k;
      const int zw = wrap(p, g.nz);
      __amdgpu_buffer_rsrc_t rz[3];
      rz[0] = plane_rsrc<T>(io.src, wrap(p - 1, g.nz), g);
      rz[1] = plane_rsrc<T>(io.src, zw, g);
      rz[2] = plane_rsrc<T>(io.src, wrap(p + 1, g.nz), g);
      const int sl = k % 5;
#pragma unroll
      for (int j = 0; j < Sh::HPL; ++j) {
        if (!has[j]) continue;
        uint32_t lk = 0;
        if constexpr (WALLS) lk = io.links[static_cast<uint32_t>(zw) * g.nxy + hcol_off[j]];
        float2 r;
        if (WALLS && (lk & 1u)) {
          r = make_float2(ph.rho_wall[0], ph.rho_wall[1]);
        } else {
          float hf[2][Q], hd[2];
          pull<S, WALLS>(rz, ppb, hcol[j], lk, ws, hf, hd);
          r = make_float2(density<S>(hd[0], ph.shift[0]), density<S>(hd[1], ph.shift[1]));
        }
        ring[sl * PLANE + hat[j]] = r;
      }
    };

    // Planes p_0 and p_1 before the first barrier (k = 1), then p_{k+1}
    // right after barrier k, in step with the own waves' pull of p_{k+1}.
    for (int k = 0; k <= min(1, kmax); ++k) halo_plane(k);
    for (int k = 1; k <= kmax; ++k) {
      __syncthreads();
      if (k + 1 <= kmax) halo_plane(k + 1);
    }
  }

  if constexpr (M != Mode::Step) {
    bool is_max[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) is_max[k] = (M == Mode::Moments) && (k == 5);
    __syncthreads();
    block_reduce_store<NV>(acc, is_max, io.partials + static_cast<uint64_t>(blockIdx.x) * NV, red);
  }
}

// ---------------------------------------------------------------------------
// Launch
// ---------------------------------------------------------------------------

// Tile shapes selectable at run time: (columns of cells, rows, halo waves);
// shapes 6..9 are the paired march over folded 16-bit rows (2 cells per lane).
struct TileShape {
  int bx, rows, hw;
};
constexpr TileShape TILES[] = {{64, 8, 3},  {64, 12, 3}, {32, 16, 2}, {128, 4, 3}, {64, 4, 3},
                               {256, 2, 3}, {128, 8, 3}, {64, 16, 2}, {64, 8, 2},  {64, 12, 2}};
static_assert(sizeof(TILES) / sizeof(TILES[0]) == TILE_SHAPES, "one entry per tile shape");
constexpr int NTILES = sizeof(TILES) / sizeof(TILES[0]);

// Default chunk length of an open box (no walls).  A step workgroup fills a
// CU, so the launch runs in ceil(blocks / 256) rounds, each as long as one
// chunk: zchunk + 2 plane iterations (two fill the pipeline).  Take the chunk
// length of at least 4 planes (or nz) and at most `cap` that minimises
// rounds x iterations; the first minimum is the shortest such chunk.
// Measured against the fixed rule below on open cubes: 64^3 47 -> 28 us,
// 112^3 154 -> 107 us, 160^3 332 -> 286 us, 192^3 596 -> 474 us; 128^3 and
// 512^3 keep their chunks.
static int round_chunk(long long txy, int nz, long long cap) {
  const int lo = nz < 4 ? nz : 4;
  const int hi = static_cast<int>(cap < nz ? cap : nz);
  int best = hi;
  long long best_cost = -1;
  for (int zc = lo; zc <= hi; ++zc) {
    const long long chunks = (nz + zc - 1) / zc;
    const long long rounds = (txy * chunks + 255) / 256;
    const long long cost = rounds * (zc + 2);
    if (best_cost < 0 || cost < best_cost) {
      best_cost = cost;
      best = zc;
    }
  }
  return best;
}

Tiling make_tiling(const Grid& g, int tile, int zchunk, bool open_box) {
  Tiling t{};
  if (tile < 0 || tile >= NTILES) {
    t.blocks = -1;
    return t;
  }
  t.tile = tile;
  const TileShape sh = TILES[tile];
  t.tiles_x = (g.nx + sh.bx - 1) / sh.bx;
  t.tiles_y = (g.ny + sh.rows - 1) / sh.rows;
  const long long txy = static_cast<long long>(t.tiles_x) * t.tiles_y;
  if (zchunk <= 0) {
    // One workgroup fills a CU; march as many planes as leave about two
    // workgroups per CU (256 CUs) over the launch, so that the planes each
    // workgroup re-reads at the ends of its column cost little (measured at
    // 512^3: 256 planes beat 64 by 1.5-2%; for the paired march 512 beat 256
    // by 1%, for the single-cell march 256 beat 512 by 1.5%).  Small grids
    // go down to 8 planes to keep one workgroup per CU.
    const long long cols = static_cast<long long>(g.nz) * txy;
    long long zc = (cols + 511) / 512;
    if (zc < 16) {
      zc = cols / 256;
      if (zc < 8) zc = 8;
      if (zc > 16) zc = 16;
    }
    const long long cap = pair_shape(tile) ? 512 : 256;
    if (zc > cap) zc = cap;
    if (open_box) zc = round_chunk(txy, g.nz, cap);
    if (zc > g.nz) zc = g.nz;
    zchunk = static_cast<int>(zc);
  }
  if (zchunk > g.nz) zchunk = g.nz;
  t.zchunk = zchunk;
  t.tiles_z = (g.nz + zchunk - 1) / zchunk;
  const long long nb = txy * t.tiles_z;
  t.blocks = nb > 0x7fffffffLL ? -1 : static_cast<int>(nb);
  return t;
}

int auto_tile(const Grid& g, bool walls, int elem_bytes) {
  // FP32 without walls: widest rows first (128-lane rows read whole 512-byte
  // population rows).  With walls (the 128 x 4 shape keeps too few registers
  // for the wall path) and for unfolded 16-bit rows (measured faster) 64 x 8
  // comes first.  Folded 16-bit rows without walls take the paired march in
  // 32 x 8 words (measured fastest of the pair shapes at 512^3: one 128-byte
  // line per population row and six waves per CU).
  // A later shape wins only by padding the x-y plane less (lanes past nx or
  // ny do no work).
  static constexpr int open_order[] = {3, 0, 2};
  static constexpr int tall_order[] = {0, 2};
  static constexpr int pair_order[] = {8};
  const bool paired = elem_bytes == 2 && g.half != 0 && !walls;
  const bool tall = walls || elem_bytes != 4;
  const int* order = paired ? pair_order : (tall ? tall_order : open_order);
  const int count = paired ? 1 : (tall ? 2 : 3);
  int best = order[0];
  long long best_cells = -1;
  for (int k = 0; k < count; ++k) {
    const TileShape sh = TILES[order[k]];
    const long long cells = static_cast<long long>((g.nx + sh.bx - 1) / sh.bx) * sh.bx *
                            (static_cast<long long>((g.ny + sh.rows - 1) / sh.rows) * sh.rows);
    if (best_cells < 0 || cells < best_cells) {
      best_cells = cells;
      best = order[k];
    }
  }
  return best;
}

template <Storage S, bool WALLS, Mode M, int BXT, int ROWS, int HW, bool REG = false>
static hipError_t launch_shape(const Grid& g, const Phys& ph, const Tiling& t, const MarchIO& io,
                               hipStream_t st) {
  using Sh = Shape<BXT, ROWS, HW>;
  hipLaunchKernelGGL((march_kernel<S, WALLS, M, BXT, ROWS, HW, REG>), dim3(t.blocks), dim3(Sh::NT), 0, st, g, ph,
                     t, io);
  return hipGetLastError();
}

template <Storage S, bool WALLS, bool REG>
static hipError_t launch_step(const Grid& g, const Phys& ph, const Tiling& t, const MarchIO& io, hipStream_t st) {
  constexpr Mode M = Mode::Step;
  switch (t.tile) {
    case 0: return launch_shape<S, WALLS, M, 64, 8, 3, REG>(g, ph, t, io, st);
    case 1: return launch_shape<S, WALLS, M, 64, 12, 3, REG>(g, ph, t, io, st);
    case 2: return launch_shape<S, WALLS, M, 32, 16, 2, REG>(g, ph, t, io, st);
    case 3: return launch_shape<S, WALLS, M, 128, 4, 3, REG>(g, ph, t, io, st);
    case 4: return launch_shape<S, WALLS, M, 64, 4, 3, REG>(g, ph, t, io, st);
    case 5: return launch_shape<S, WALLS, M, 256, 2, 3, REG>(g, ph, t, io, st);
    default: return hipErrorInvalidValue;
  }
}

template <Storage S, bool WALLS, Mode M>
static hipError_t launch_tile(const Grid& g, const Phys& ph, const Tiling& t, const MarchIO& io,
                              hipStream_t st) {
  if constexpr (M == Mode::Step) {
    return ph.regularized ? launch_step<S, WALLS, true>(g, ph, t, io, st)
                          : launch_step<S, WALLS, false>(g, ph, t, io, st);
  } else if constexpr (M == Mode::Moments) {
    // Diagnostics use one shape (tile 0).
    if (t.tile != 0) return hipErrorInvalidValue;
    return launch_shape<S, WALLS, M, 64, 8, 3>(g, ph, t, io, st);
  } else if (ph.regularized) {
    if (!io.dbar) return hipErrorInvalidValue;
    switch (t.tile) {
      case 0: return launch_shape<S, WALLS, M, 64, 8, 3, true>(g, ph, t, io, st);
      case 2: return launch_shape<S, WALLS, M, 32, 16, 2, true>(g, ph, t, io, st);
      case 4: return launch_shape<S, WALLS, M, 64, 4, 3, true>(g, ph, t, io, st);
      default: return hipErrorInvalidValue;
    }
  } else {
    switch (t.tile) {
      case 0: return launch_shape<S, WALLS, M, 64, 8, 3>(g, ph, t, io, st);
      case 2: return launch_shape<S, WALLS, M, 32, 16, 2>(g, ph, t, io, st);
      case 4: return launch_shape<S, WALLS, M, 64, 4, 3>(g, ph, t, io, st);
      default: return hipErrorInvalidValue;
    }
  }
}

template <Storage S, Mode M>
static hipError_t launch_walls(const Grid& g, const Phys& ph, const Tiling& t, const MarchIO& io,
                               hipStream_t st) {
  return io.links ? launch_tile<S, true, M>(g, ph, t, io, st) : launch_tile<S, false, M>(g, ph, t, io, st);
}

template <Storage S>
static hipError_t launch_mode(Mode mode, const Grid& g, const Phys& ph, const Tiling& t, const MarchIO& io,
                              hipStream_t st) {
  switch (mode) {
    case Mode::Step: return launch_walls<S, Mode::Step>(g, ph, t, io, st);
    case Mode::Moments: return launch_walls<S, Mode::Moments>(g, ph, t, io, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_march(Storage s, Mode mode, const Grid& g, const Phys& ph, const Tiling& t,
                        const MarchIO& io, hipStream_t st) {
  if (t.blocks <= 0) return hipErrorInvalidValue;
  if (pair_shape(t.tile)) {
    if (mode != Mode::Step) return hipErrorInvalidValue;
    return launch_pair_step(s, g, ph, t, io, st);
  }
  if (mode == Mode::Adjoint) {
    if (s != Storage::F32) return hipErrorInvalidValue;
    return launch_walls<Storage::F32, Mode::Adjoint>(g, ph, t, io, st);
  }
  switch (s) {
    case Storage::F32: return launch_mode<Storage::F32>(mode, g, ph, t, io, st);
    case Storage::F16: return launch_mode<Storage::F16>(mode, g, ph, t, io, st);
    case Storage::BF16: return launch_mode<Storage::BF16>(mode, g, ph, t, io, st);
  }
  return hipErrorInvalidValue;
}

}  // namespace lbm
