// Fused z-marching kernels of the two-component D3Q19 step (gfx950).
//
// One workgroup owns a tile of 64 x ROWS cells in the x-y plane and marches
// up a chunk of z planes.  For each new plane it pulls the 38 populations of
// its cells (Eq. 1 in pull form, with halfway bounce-back at walls, Sec. 4)
// and reduces the species densities rho^A, rho^B (Eq. 4) into a 4-slot LDS
// ring that also holds a one-cell halo of the tile.  The halo densities are
// recomputed from the populations around the tile, so no density field ever
// travels through HBM.  Once plane z+1 is in the ring, plane z has every
// neighbour density the Shan-Chen sum of Eq. (7) needs, and the cell update
// (Eqs. 2-9) runs from the populations the thread kept in registers.
//
// The same march serves three bodies:
//   Step     collide and store X_{t+1}(x) = f*(x)  (post-collision state);
//   Moments  rho^a and u_F fields plus FP64 per-workgroup diagnostic sums;
//   Adjoint  per-cell transposed collision (see below) for one reverse step.
//
// Memory layout: SoA X[a][i][z][y][x], x fastest, so each population load of
// a 64-wide row is one contiguous 256-byte run (FP32).  Blocks are remapped
// so that the tiles dispatched to one XCD (block id mod 8) are contiguous in
// x and y and share that XCD's L2 for the halo re-reads.

#include "launch.h"

namespace lbm {

constexpr int BX = 64;

// Tile index of a block: dispatch sends block b to XCD b % 8, so give each
// XCD a contiguous range of tiles.
__device__ __forceinline__ int xcd_remap(int b, int nb) {
  const int q = nb >> 3, r = nb & 7;
  const int k = b & 7, i = b >> 3;
  return (k < r ? k * (q + 1) : r * (q + 1) + (k - r) * q) + i;
}

__device__ __forceinline__ int wrap(int v, int n) {
  int r = v % n;
  return r < 0 ? r + n : r;
}

// Wrapped coordinates of one cell column (x, y) and of its x/y neighbours,
// as BYTE offsets inside one population plane (nx * ny elements).
struct Column {
  uint32_t x[3];  // (x-1, x, x+1) * sizeof(T)
  uint32_t y[3];  // ((y-1), y, (y+1)) * nx * sizeof(T)
};

template <typename T>
__device__ __forceinline__ Column make_column(int ex, int ey, const Grid& g) {
  const int gx = wrap(ex, g.nx), gy = wrap(ey, g.ny);
  const uint32_t sz = sizeof(T);
  Column c;
  c.x[0] = (gx == 0 ? g.nx - 1 : gx - 1) * sz;
  c.x[1] = gx * sz;
  c.x[2] = (gx == g.nx - 1 ? 0 : gx + 1) * sz;
  const int ym = gy == 0 ? g.ny - 1 : gy - 1;
  const int yp = gy == g.ny - 1 ? 0 : gy + 1;
  c.y[0] = static_cast<uint32_t>(ym) * g.nx * sz;
  c.y[1] = static_cast<uint32_t>(gy) * g.nx * sz;
  c.y[2] = static_cast<uint32_t>(yp) * g.nx * sz;
  return c;
}

// Buffer resource over the 38 population planes of z plane `zw`
// (plane-major layout X[z][a][i][y][x]).  Out-of-range offsets read as zero
// instead of faulting.
constexpr int RSRC_FLAGS = 0x00020000;  // 32-bit data format, gfx9 family

template <typename T>
__device__ __forceinline__ __amdgpu_buffer_rsrc_t plane_rsrc(const void* buf, int zw, const Grid& g) {
  const uint64_t block = static_cast<uint64_t>(2 * Q) * g.nxy * sizeof(T);
  const char* base = static_cast<const char*>(buf) + static_cast<uint64_t>(zw) * block;
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<char*>(base), static_cast<short>(0),
                                           static_cast<int>(block), RSRC_FLAGS);
}

template <typename T>
__device__ __forceinline__ T buf_load(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
  if constexpr (sizeof(T) == 4) {
    return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
  } else {
    return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b16(r, voff, soff, 0));
  }
}

template <typename T>
__device__ __forceinline__ void buf_store(T v, __amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
  if constexpr (sizeof(T) == 4) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, voff, soff, 0);
  } else {
    __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(unsigned short, v), r, voff, soff, 0);
  }
}

// Pull of Eq. (1): f_i(x) = X_i(x - c_i), or X_opp(i)(x) when x - c_i is a
// wall cell (bit i of `links`).  rz[k] covers z plane z - 1 + k; `ppb` is the
// byte size of one population plane, so population (a, i) of a plane starts
// at (19 a + i) * pp.  Every load is scalar resource + scalar population
// offset + per-lane (y, x) offset.
template <Storage S, bool WALLS>
__device__ __forceinline__ void pull(const __amdgpu_buffer_rsrc_t rz[3], uint32_t ppb, const Column& c,
                                     uint32_t links, const float ws[2][3], float f[2][Q]) {
  using Tr = StorageTraits<S>;
  using T = typename Tr::T;
  const uint32_t own = c.y[1] + c.x[1];
#pragma unroll
  for (int s = 0; s < 2; ++s) {
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      const uint32_t off = c.y[1 - CY[i]] + c.x[1 - CX[i]];
      T v;
      if constexpr (WALLS) {
        if ((i != 0) && ((links >> i) & 1u)) {
          v = buf_load<T>(rz[1], own, static_cast<uint32_t>(s * Q + opp(i)) * ppb);
        } else {
          v = buf_load<T>(rz[1 - CZ[i]], off, static_cast<uint32_t>(s * Q + i) * ppb);
        }
      } else {
        v = buf_load<T>(rz[1 - CZ[i]], off, static_cast<uint32_t>(s * Q + i) * ppb);
      }
      float x = Tr::decode(v);
      if constexpr (Tr::shifted) x += ws[s][i == 0 ? 0 : (i <= 6 ? 1 : 2)];
      f[s][i] = x;
    }
  }
}

__device__ __forceinline__ float sum19(const float f[Q]) {
  float r = f[0];
#pragma unroll
  for (int i = 1; i < Q; ++i) r += f[i];
  return r;
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

// Bracket of Eq. (3) at T0 = 1/3: P(v) = 1 + 3 cv + 4.5 cv^2 - 1.5 vv + 4.5 cv^3
// - 4.5 cv vv, split into the part even in cv and the part odd in cv so that
// P(+p_k) = ev + od and P(-p_k) = ev - od.
struct Bracket {
  float rest;
  float ev[9];
  float od[9];
};

__device__ __forceinline__ void bracket(float vx, float vy, float vz, Bracket& B) {
  const float vv = vx * vx + vy * vy + vz * vz;
  const float a = 1.0f - 1.5f * vv;
  const float b = 3.0f - 4.5f * vv;
  float cv[9];
  pair_dots(vx, vy, vz, cv);
  B.rest = a;
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    const float t = cv[k] * cv[k];
    B.ev[k] = a + 4.5f * t;
    B.od[k] = cv[k] * (b + 4.5f * t);
  }
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

// u from the populations; S from the LDS density ring.
__device__ __forceinline__ void make_local(const float f[2][Q], const float rho_a, const float rho_b,
                                           const float2 (*pm)[BX + 2], const float2 (*p0)[BX + 2],
                                           const float2 (*pp)[BX + 2], int ly, int lx,
                                           const Phys& ph, Local& L) {
  L.rho[0] = rho_a;
  L.rho[1] = rho_b;
  L.rinv = 1.0f / (rho_a + rho_b);
  float d[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) d[k] = (f[0][2 * k + 1] + f[1][2 * k + 1]) - (f[0][2 * k + 2] + f[1][2 * k + 2]);
  const float jx = d[0] + d[3] + d[4] + d[5] + d[6];
  const float jy = d[1] + d[3] - d[4] + d[7] + d[8];
  const float jz = d[2] + d[5] - d[6] + d[7] - d[8];
  L.u[0] = jx * L.rinv;
  L.u[1] = jy * L.rinv;
  L.u[2] = jz * L.rinv;

  // Neighbour densities rho~(x + p_k) - rho~(x - p_k) for each pair.
  // Ring rows are indexed [y + 1][x + 1] relative to the tile.
  float2 e[9];
  auto R = [&](const float2 (*pl)[BX + 2], int dy, int dx) { return pl[ly + dy][lx + dx]; };
  auto dif = [](float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); };
  e[0] = dif(R(p0, 0, 1), R(p0, 0, -1));
  e[1] = dif(R(p0, 1, 0), R(p0, -1, 0));
  e[2] = dif(R(pp, 0, 0), R(pm, 0, 0));
  e[3] = dif(R(p0, 1, 1), R(p0, -1, -1));
  e[4] = dif(R(p0, -1, 1), R(p0, 1, -1));
  e[5] = dif(R(pp, 0, 1), R(pm, 0, -1));
  e[6] = dif(R(pm, 0, 1), R(pp, 0, -1));
  e[7] = dif(R(pp, 1, 0), R(pm, -1, 0));
  e[8] = dif(R(pm, 1, 0), R(pp, -1, 0));
  const float2 sx = make_float2(WF * e[0].x + WE * (e[3].x + e[4].x + e[5].x + e[6].x),
                                WF * e[0].y + WE * (e[3].y + e[4].y + e[5].y + e[6].y));
  const float2 sy = make_float2(WF * e[1].x + WE * (e[3].x - e[4].x + e[7].x + e[8].x),
                                WF * e[1].y + WE * (e[3].y - e[4].y + e[7].y + e[8].y));
  const float2 sz = make_float2(WF * e[2].x + WE * (e[5].x - e[6].x + e[7].x - e[8].x),
                                WF * e[2].y + WE * (e[5].y - e[6].y + e[7].y - e[8].y));
  L.S[0][0] = sx.x; L.S[0][1] = sy.x; L.S[0][2] = sz.x;
  L.S[1][0] = sx.y; L.S[1][1] = sy.y; L.S[1][2] = sz.y;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    L.g[0][k] = ph.g_ab * L.S[1][k];
    L.g[1][k] = ph.g_ba * L.S[0][k];
  }
}

// BGK collision (Eq. 2) plus the exact-difference forcing term, in place:
//   f*_i = (1 - w) f_i + w_i rho^a [(w - 1) P_i(u) + P_i(u + g^a)],  w = 1/tau_a.
__device__ __forceinline__ void collide(float f[2][Q], const Local& L, const Phys& ph) {
  Bracket Bu;
  bracket(L.u[0], L.u[1], L.u[2], Bu);
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    Bracket Bv;
    bracket(L.u[0] + L.g[s][0], L.u[1] + L.g[s][1], L.u[2] + L.g[s][2], Bv);
    const float om = ph.omega[s];
    const float om1 = om - 1.0f;
    const float keep = 1.0f - om;
    const float r = L.rho[s];
    f[s][0] = keep * f[s][0] + (W0 * r) * (om1 * Bu.rest + Bv.rest);
#pragma unroll
    for (int k = 0; k < 9; ++k) {
      const float ke = om1 * Bu.ev[k] + Bv.ev[k];
      const float ko = om1 * Bu.od[k] + Bv.od[k];
      const float wr = pair_w(k) * r;
      f[s][2 * k + 1] = keep * f[s][2 * k + 1] + wr * (ke + ko);
      f[s][2 * k + 2] = keep * f[s][2 * k + 2] + wr * (ke - ko);
    }
  }
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
__device__ __forceinline__ constexpr int pair_cx(int k) { return (k == 0 || (k >= 3 && k <= 6)) ? 1 : 0; }
__device__ __forceinline__ constexpr int pair_cy(int k) {
  return (k == 1 || k == 3 || k == 7 || k == 8) ? 1 : (k == 4 ? -1 : 0);
}
__device__ __forceinline__ constexpr int pair_cz(int k) {
  return (k == 2 || k == 5 || k == 7) ? 1 : ((k == 6 || k == 8) ? -1 : 0);
}

__device__ __forceinline__ void adjoint_cell(const float f[2][Q], const float lam[2][Q], const Local& L,
                                             const Phys& ph, float mo[5], float sb[6], double acc[3]) {
  const float* u = L.u;
  const float uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
  float cu[9];
  pair_dots(u[0], u[1], u[2], cu);
  float ubar[3] = {0.f, 0.f, 0.f};
  float rbar[2], gbar[2][3];
  float dtau[2];
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    const float v[3] = {u[0] + L.g[s][0], u[1] + L.g[s][1], u[2] + L.g[s][2]};
    const float vv = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
    float cv[9];
    pair_dots(v[0], v[1], v[2], cv);
    const float om = ph.omega[s];
    const float om1 = om - 1.0f;
    const float r = L.rho[s];
    const float l0 = lam[s][0] * W0;
    const float pu0 = 1.0f - 1.5f * uu;
    const float pv0 = 1.0f - 1.5f * vv;
    float rb = l0 * (om1 * pu0 + pv0);
    float bu = 3.0f * l0, bv = 3.0f * l0;
    float au[3] = {0.f, 0.f, 0.f}, av[3] = {0.f, 0.f, 0.f};
    float dt = lam[s][0] * (f[s][0] - W0 * r * pu0);
#pragma unroll
    for (int k = 0; k < 9; ++k) {
      const float w = pair_w(k);
      const float lp = lam[s][2 * k + 1] * w;
      const float lm = lam[s][2 * k + 2] * w;
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
      dt += lam[s][2 * k + 1] * (f[s][2 * k + 1] - w * r * pup) +
            lam[s][2 * k + 2] * (f[s][2 * k + 2] - w * r * pum);
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      gbar[s][a] = r * (av[a] - v[a] * bv);
      ubar[a] += r * (om1 * (au[a] - u[a] * bu) + (av[a] - v[a] * bv));
    }
    rbar[s] = rb;
    dtau[s] = om * om * dt;
  }
  const float ubu = ubar[0] * u[0] + ubar[1] * u[1] + ubar[2] * u[2];
  mo[0] = rbar[0] - ubu * L.rinv;
  mo[1] = rbar[1] - ubu * L.rinv;
  mo[2] = ubar[0] * L.rinv;
  mo[3] = ubar[1] * L.rinv;
  mo[4] = ubar[2] * L.rinv;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    sb[a] = ph.g_ba * gbar[1][a];
    sb[3 + a] = ph.g_ab * gbar[0][a];
  }
  acc[0] += static_cast<double>(gbar[0][0] * L.S[1][0] + gbar[0][1] * L.S[1][1] + gbar[0][2] * L.S[1][2]) +
            static_cast<double>(gbar[1][0] * L.S[0][0] + gbar[1][1] * L.S[0][1] + gbar[1][2] * L.S[0][2]);
  acc[1] += dtau[0];
  acc[2] += dtau[1];
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
template <Storage S, bool WALLS, Mode M, int ROWS>
__global__ void __launch_bounds__(BX * ROWS)
march_kernel(const Grid g, const Phys ph, const Tiling tl, const MarchIO io) {
  using Tr = StorageTraits<S>;
  using T = typename Tr::T;
  constexpr int NT = BX * ROWS;
  constexpr int EX = BX + 2;
  constexpr int NH = 2 * EX + 2 * ROWS;  // halo cells around the tile
  static_assert(NH <= NT, "one halo cell per thread at most");
  __shared__ float2 ring[4][ROWS + 2][EX];
  __shared__ double red[(NT / 64) * 16];

  const int tid = threadIdx.x;
  const int tx = tid % BX, ty = tid / BX;
  const int b = xcd_remap(blockIdx.x, gridDim.x);
  const int tiles_xy = tl.tiles_x * tl.tiles_y;
  const int bz = b / tiles_xy;
  const int rem = b - bz * tiles_xy;
  const int byy = rem / tl.tiles_x;
  const int bxx = rem - byy * tl.tiles_x;
  const int x0 = bxx * BX, y0 = byy * ROWS, z0 = bz * tl.zchunk;
  const int z1 = min(z0 + tl.zchunk, g.nz);

  const uint64_t n = g.n;
  const uint32_t ppb = g.nxy * static_cast<uint32_t>(sizeof(T));  // bytes of one population plane

  // This thread's own column (always computed; only owners update cells).
  const int ex = x0 + tx, ey = y0 + ty;
  const bool owner = ex < g.nx && ey < g.ny;
  const Column col = make_column<T>(ex, ey, g);
  const uint32_t col_b = col.y[1] + col.x[1];             // byte offset in a plane
  const uint32_t col_off = col_b / static_cast<uint32_t>(sizeof(T));  // element offset

  // Halo column of this thread, if any: bottom row, top row, left, right.
  const bool has_halo = tid < NH;
  int hx = 0, hy = 0;
  if (tid < EX) { hx = tid - 1; hy = -1; }
  else if (tid < 2 * EX) { hx = tid - EX - 1; hy = ROWS; }
  else if (tid < 2 * EX + ROWS) { hx = -1; hy = tid - 2 * EX; }
  else { hx = BX; hy = tid - 2 * EX - ROWS; }
  const Column hcol = make_column<T>(x0 + hx, y0 + hy, g);
  const uint32_t hcol_off = (hcol.y[1] + hcol.x[1]) / static_cast<uint32_t>(sizeof(T));

  float ws[2][3];
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    ws[s][0] = W0 * ph.shift[s];
    ws[s][1] = WF * ph.shift[s];
    ws[s][2] = WE * ph.shift[s];
  }

  float cur[2][Q], nxt[2][Q];
  float cur_rho[2] = {0.f, 0.f}, nxt_rho[2] = {0.f, 0.f};
  uint32_t cur_links = 0, nxt_links = 0;

  // Per-thread diagnostic / gradient accumulators.
  constexpr int NV = (M == Mode::Moments) ? 16 : 3;
  double acc[NV];
#pragma unroll
  for (int k = 0; k < NV; ++k) acc[k] = 0.0;

  for (int p = z0 - 1; p <= z1; ++p) {
    const int zw = wrap(p, g.nz);
    __amdgpu_buffer_rsrc_t rz[3];
    rz[0] = plane_rsrc<T>(io.src, wrap(p - 1, g.nz), g);
    rz[1] = plane_rsrc<T>(io.src, zw, g);
    rz[2] = plane_rsrc<T>(io.src, wrap(p + 1, g.nz), g);
    const uint32_t zo1 = static_cast<uint32_t>(zw) * g.nxy;  // element offset of plane p in a cell field
    const int slot = (p + 4) & 3;

    // ---- phase A: pull plane p, reduce densities into the ring ----------
    {
      if constexpr (WALLS) nxt_links = io.links[zo1 + col_off];
      const bool solid = WALLS && (nxt_links & 1u);
      if (!solid) {
        pull<S, WALLS>(rz, ppb, col, nxt_links, ws, nxt);
        nxt_rho[0] = sum19(nxt[0]);
        nxt_rho[1] = sum19(nxt[1]);
        ring[slot][ty + 1][tx + 1] = make_float2(nxt_rho[0], nxt_rho[1]);
      } else {
        ring[slot][ty + 1][tx + 1] = make_float2(ph.rho_wall[0], ph.rho_wall[1]);
      }
    }
    if (has_halo) {
      uint32_t hl = 0;
      if constexpr (WALLS) hl = io.links[zo1 + hcol_off];
      float2 r;
      if (WALLS && (hl & 1u)) {
        r = make_float2(ph.rho_wall[0], ph.rho_wall[1]);
      } else {
        float hf[2][Q];
        pull<S, WALLS>(rz, ppb, hcol, hl, ws, hf);
        r = make_float2(sum19(hf[0]), sum19(hf[1]));
      }
      ring[slot][hy + 1][hx + 1] = r;
    }

    // ---- phase B: update plane p - 1 --------------------------------------
    if (p >= z0 + 1) {
      __syncthreads();
      const int z = p - 1;
      const bool solid = WALLS && (cur_links & 1u);
      const uint32_t cell = static_cast<uint32_t>(wrap(z, g.nz)) * g.nxy + col_off;
      if (owner) {
        const float2 (*pm)[EX] = ring[(z - 1 + 4) & 3];
        const float2 (*p0)[EX] = ring[(z + 4) & 3];
        const float2 (*pp)[EX] = ring[(z + 1 + 4) & 3];
        if constexpr (M == Mode::Step) {
          if (!solid) {
            Local L;
            make_local(cur, cur_rho[0], cur_rho[1], pm, p0, pp, ty + 1, tx + 1, ph, L);
            collide(cur, L, ph);
            const __amdgpu_buffer_rsrc_t rd = plane_rsrc<T>(io.dst, wrap(z, g.nz), g);
#pragma unroll
            for (int s = 0; s < 2; ++s) {
#pragma unroll
              for (int i = 0; i < Q; ++i) {
                float v = cur[s][i];
                if constexpr (Tr::shifted) v -= ws[s][i == 0 ? 0 : (i <= 6 ? 1 : 2)];
                buf_store<T>(Tr::encode(v), rd, col_b, static_cast<uint32_t>(s * Q + i) * ppb);
              }
            }
          }
        } else if constexpr (M == Mode::Moments) {
          float ra = 0.f, rb = 0.f, uf[3] = {0.f, 0.f, 0.f};
          if (!solid) {
            Local L;
            make_local(cur, cur_rho[0], cur_rho[1], pm, p0, pp, ty + 1, tx + 1, ph, L);
            ra = L.rho[0];
            rb = L.rho[1];
            // u_F = u + g/2, g = sum_a rho^a g^a / rho  (Eqs. 8-9)
#pragma unroll
            for (int k = 0; k < 3; ++k)
              uf[k] = L.u[k] + 0.5f * (ra * L.g[0][k] + rb * L.g[1][k]) * L.rinv;
            const double rho = static_cast<double>(ra) + static_cast<double>(rb);
            acc[0] += ra;
            acc[1] += rb;
            acc[2] += rho * uf[0];
            acc[3] += rho * uf[1];
            acc[4] += rho * uf[2];
            const double sp = sqrt(static_cast<double>(uf[0]) * uf[0] +
                                   static_cast<double>(uf[1]) * uf[1] +
                                   static_cast<double>(uf[2]) * uf[2]);
            const bool finite = isfinite(ra) && isfinite(rb) && isfinite(uf[0]) &&
                                isfinite(uf[1]) && isfinite(uf[2]);
            acc[5] = fmax(acc[5], finite ? sp : 0.0);
            acc[6] += finite ? 0.0 : 1.0;
            acc[7] += 1.0;
            const Region& R = io.region;
            const float dx = min_image(static_cast<float>(col_off % g.nx) - R.cx, static_cast<float>(g.nx));
            const float dy = min_image(static_cast<float>(col_off / g.nx) - R.cy, static_cast<float>(g.ny));
            const float dz = min_image(static_cast<float>(wrap(z, g.nz)) - R.cz, static_cast<float>(g.nz));
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
          if (!solid) {
            Local L;
            make_local(cur, cur_rho[0], cur_rho[1], pm, p0, pp, ty + 1, tx + 1, ph, L);
            float lam[2][Q];
            const __amdgpu_buffer_rsrc_t rl = plane_rsrc<float>(io.lam, wrap(z, g.nz), g);
#pragma unroll
            for (int s = 0; s < 2; ++s)
#pragma unroll
              for (int i = 0; i < Q; ++i) lam[s][i] = buf_load<float>(rl, col_b, static_cast<uint32_t>(s * Q + i) * ppb);
            adjoint_cell(cur, lam, L, ph, mo, sb, acc);
          }
#pragma unroll
          for (int k = 0; k < 5; ++k) io.m[k * n + cell] = mo[k];
#pragma unroll
          for (int k = 0; k < 6; ++k) io.sbar[k * n + cell] = sb[k];
        }
      }
    }

    // ---- rotate registers ---------------------------------------------------
#pragma unroll
    for (int s = 0; s < 2; ++s) {
#pragma unroll
      for (int i = 0; i < Q; ++i) cur[s][i] = nxt[s][i];
      cur_rho[s] = nxt_rho[s];
    }
    cur_links = nxt_links;
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
Tiling make_tiling(const Grid& g, int rows, int zchunk) {
  Tiling t{};
  t.rows = rows;
  t.tiles_x = (g.nx + BX - 1) / BX;
  t.tiles_y = (g.ny + rows - 1) / rows;
  const long long txy = static_cast<long long>(t.tiles_x) * t.tiles_y;
  if (zchunk <= 0) {
    // Aim for about 2048 workgroups (8 per CU) with the longest march.
    long long zc = (static_cast<long long>(g.nz) * txy + 2047) / 2048;
    if (zc < 4) zc = 4;
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

template <Storage S, bool WALLS, Mode M>
static hipError_t launch_rows(const Grid& g, const Phys& ph, const Tiling& t, const MarchIO& io,
                              hipStream_t st) {
  if (t.rows == 4) {
    hipLaunchKernelGGL((march_kernel<S, WALLS, M, 4>), dim3(t.blocks), dim3(BX * 4), 0, st, g, ph, t, io);
  } else {
    hipLaunchKernelGGL((march_kernel<S, WALLS, M, 8>), dim3(t.blocks), dim3(BX * 8), 0, st, g, ph, t, io);
  }
  return hipGetLastError();
}

template <Storage S, Mode M>
static hipError_t launch_walls(const Grid& g, const Phys& ph, const Tiling& t, const MarchIO& io,
                               hipStream_t st) {
  return io.links ? launch_rows<S, true, M>(g, ph, t, io, st) : launch_rows<S, false, M>(g, ph, t, io, st);
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
  if (t.blocks <= 0 || (t.rows != 4 && t.rows != 8)) return hipErrorInvalidValue;
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
