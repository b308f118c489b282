// Neighbour passes of the reverse (adjoint) step.  The march computes, per
// fluid cell, the local part of the transposed collision (a^a, b) and the
// transposed Shan-Chen sources Sbar; these kernels finish the step:
//
//   gather   A^a(x) = a^a(x) + sum_i w_i c_i . Sbar^a(x - c_i)  (transpose of
//            the Eq. 7 neighbour sum; wall neighbours are constants);
//   stream   lam_t,i(y) = (1 - w_a) lam_{t+1},i(x) + A^a(x) + b(x) . c_i with
//            x = y + c_i, or, when y + c_i is a wall, x = y read through
//            direction opp(i) with the sign of c_i flipped (transpose of the
//            pull with bounce-back, Eq. 1 and Sec. 4); with the regularized
//            collision (Sec. 3) the first term is c_i c_i : Pbar^a(x), which
//            the march stores per pair of directions;
//   seed     dL/dX_T from dL/drho(T).

#include "buffer.h"
#include "launch.h"

namespace lbm {

namespace {

// Lane of a 3-D launch (x fastest): block (bx, y, z), 64 lanes along x.  The
// wrapped coordinates of the +-1 neighbours come from compares, not division.
struct Cell3 {
  int x, y, z;
  int xm, xp, ym, yp, zm, zp;
  bool valid;
};

__device__ __forceinline__ Cell3 cell3(const Grid& g) {
  Cell3 c;
  c.x = blockIdx.x * blockDim.x + threadIdx.x;
  c.y = blockIdx.y;
  c.z = blockIdx.z;
  c.valid = c.x < g.nx;
  c.xm = c.x == 0 ? g.nx - 1 : c.x - 1;
  c.xp = c.x >= g.nx - 1 ? 0 : c.x + 1;
  c.ym = c.y == 0 ? g.ny - 1 : c.y - 1;
  c.yp = c.y == g.ny - 1 ? 0 : c.y + 1;
  c.zm = c.z == 0 ? g.nz - 1 : c.z - 1;
  c.zp = c.z == g.nz - 1 ? 0 : c.z + 1;
  return c;
}

__device__ __forceinline__ int pick(int d, int m, int o, int p) { return d < 0 ? m : (d > 0 ? p : o); }

// Cell index of (x + dx, y + dy, z + dz), |d| <= 1.
__device__ __forceinline__ uint64_t near(const Cell3& c, int dx, int dy, int dz, const Grid& g) {
  const uint64_t x = pick(dx, c.xm, c.x, c.xp), y = pick(dy, c.ym, c.y, c.yp), z = pick(dz, c.zm, c.z, c.zp);
  return (z * g.ny + y) * g.nx + x;
}

// Index of population (s, i) at (x + dx, y + dy, z + dz) in a state-layout array.
__device__ __forceinline__ uint64_t near_pm(const Cell3& c, int s, int i, int dx, int dy, int dz, const Grid& g) {
  const uint64_t x = pick(dx, c.xm, c.x, c.xp), z = pick(dz, c.zm, c.z, c.zp);
  const int y = pick(dy, c.ym, c.y, c.yp);
  return z * g.zstride + row_off(y, g) + static_cast<uint64_t>(s * Q + i) * g.pstride + x;
}

// Adjoint, pass 2: A^b(x) = a^b(x) + sum_i w_i c_i . Sbar^b(x - c_i) on fluid x.
// m holds (a^A, a^B, b_x, b_y, b_z) per cell; a^b is replaced by A^b in place.
// A workgroup owns BXT x ROWS columns and marches up a chunk of z planes; the
// six Sbar fields of planes z - 1 .. z + 1 with a one-cell x-y border sit in
// a 4-slot LDS ring, so each value is read from memory about once per
// workgroup instead of once per neighbour.  As in the stream pass, plane
// p_k = z0 - 1 + k lives in slot k % 4 and the loads of p_{k+2} are in
// flight while p_k is summed.
constexpr int SBAR_FIELDS = 6;

template <int BXT, int ROWS>
__global__ void __launch_bounds__(BXT * ROWS)
adjoint_gather_kernel(const Grid g, const Tiling tl, const uint32_t* __restrict__ links, float* __restrict__ m,
                      const float* __restrict__ sbar) {
  constexpr int NT = BXT * ROWS;
  constexpr int EX = BXT + 2, EY = ROWS + 2, PLANE = EX * EY;
  constexpr int LPT = (PLANE + NT - 1) / NT;
  constexpr int SLOTS = 4;
  __shared__ float ring[SLOTS * SBAR_FIELDS * PLANE];

  const int tid = threadIdx.x;
  const int b = xcd_remap(blockIdx.x, gridDim.x);
  const int tiles_xy = tl.tiles_x * tl.tiles_y;
  const int bz = b / tiles_xy;
  const int rem = b - bz * tiles_xy;
  const int byy = rem / tl.tiles_x;
  const int bxx = rem - byy * tl.tiles_x;
  const int x0 = bxx * BXT, y0 = byy * ROWS, z0 = bz * tl.zchunk;
  const int z1 = min(z0 + tl.zchunk, g.nz);
  const int kmax = z1 - z0 + 1;  // planes p_k = z0 - 1 + k, k = 0..kmax
  const uint32_t n = static_cast<uint32_t>(g.n);

  uint32_t loff[LPT];
  bool lhas[LPT];
#pragma unroll
  for (int j = 0; j < LPT; ++j) {
    const int l = tid + j * NT;
    lhas[j] = l < PLANE;
    const int ly = l / EX, lx = l - (l / EX) * EX;
    loff[j] = static_cast<uint32_t>(wrap(y0 + ly - 1, g.ny)) * g.nx + static_cast<uint32_t>(wrap(x0 + lx - 1, g.nx));
  }
  float fv[LPT][SBAR_FIELDS];
  auto fetch = [&](int p) {
    const uint32_t base = static_cast<uint32_t>(wrap(p, g.nz)) * g.nxy;
#pragma unroll
    for (int j = 0; j < LPT; ++j)
#pragma unroll
      for (int f = 0; f < SBAR_FIELDS; ++f) fv[j][f] = lhas[j] ? sbar[f * n + base + loff[j]] : 0.0f;
  };
  auto publish = [&](int slot) {
#pragma unroll
    for (int j = 0; j < LPT; ++j) {
      if (!lhas[j]) continue;
      const int l = tid + j * NT;
#pragma unroll
      for (int f = 0; f < SBAR_FIELDS; ++f) ring[(slot * SBAR_FIELDS + f) * PLANE + l] = fv[j][f];
    }
  };

  const int tx = tid % BXT, ty = tid / BXT;
  const int ex = x0 + tx, ey = y0 + ty;
  const bool owner = ex < g.nx && ey < g.ny;
  const uint32_t col = owner ? static_cast<uint32_t>(ey) * g.nx + static_cast<uint32_t>(ex) : 0u;
  const int at = (ty + 1) * EX + tx + 1;

  for (int k = 0; k <= 2; ++k) {
    fetch(z0 - 1 + k);
    publish(k);
  }
  __syncthreads();
  for (int k = 1; k < kmax; ++k) {
    if (k + 2 <= kmax) fetch(z0 + 1 + k);
    if (owner) {
      const uint32_t c = static_cast<uint32_t>(z0 - 1 + k) * g.nxy + col;
      if (!is_solid(links, c)) {
        float r[2] = {0.f, 0.f};
#pragma unroll
        for (int i = 1; i < Q; ++i) {
          // Sbar at x - c_i: plane p_{k - c_z} (slot (k - c_z) % 4), ring cell at - c_y EX - c_x
          const float* rs = ring + ((k - CZ[i] + SLOTS) % SLOTS) * SBAR_FIELDS * PLANE + at - CY[i] * EX - CX[i];
          const float w = weight(i);
#pragma unroll
          for (int s = 0; s < 2; ++s) {
            float dot = 0.0f;
            if (CX[i]) dot += CX[i] * rs[(3 * s) * PLANE];
            if (CY[i]) dot += CY[i] * rs[(3 * s + 1) * PLANE];
            if (CZ[i]) dot += CZ[i] * rs[(3 * s + 2) * PLANE];
            r[s] += w * dot;
          }
        }
        m[c] += r[0];
        m[n + c] += r[1];
      }
    }
    if (k + 2 <= kmax) publish((k + 2) % SLOTS);
    __syncthreads();
  }
}

// dL/dX_T for L(rho(T)): lam_i(y) = grad(y + c_i), or grad(y) if y + c_i is a wall.
__global__ void __launch_bounds__(64) adjoint_seed_kernel(const Grid g, const uint32_t* __restrict__ links,
                                                          const float* __restrict__ grad, float* __restrict__ lam) {
  const Cell3 p = cell3(g);
  if (!p.valid) return;
  const uint64_t c = near(p, 0, 0, 0, g);
  const bool solid = is_solid(links, c);
#pragma unroll
  for (int s = 0; s < 2; ++s) {
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      float v = 0.0f;
      if (!solid) {
        const uint64_t x = ahead_solid(links, c, i) ? c : near(p, CX[i], CY[i], CZ[i], g);
        v = grad[s * g.n + x];
      }
      lam[near_pm(p, s, i, 0, 0, 0, g)] = v;
    }
  }
}


// Stream pass.  A workgroup owns BXT x ROWS columns and marches up a chunk of
// z planes.  The five per-cell fields (A^A, A^B, b_x, b_y, b_z) of planes
// z - 1 .. z + 1 with a one-cell x-y border sit in a 4-slot LDS ring, so each
// field value is read from memory once per workgroup instead of once per
// neighbour; lam_{t+1} is pulled with the same buffer addressing as the
// forward step.  The march is software-pipelined: while plane p_k is
// finished from registers, the pulled lam of p_{k+1} and the fields of
// p_{k+2} are in flight.  Plane p_k = z0 - 1 + k lives in slot k % 4; one
// barrier ends each iteration, after which the slot written in it (p_{k+2},
// last read in iteration k - 1) is visible.
//
// PAIRS (regularized collision): lam_in holds, instead of lam_{t+1}, the
// direct term c_i c_i : Pbar of dL/df_i, the same for both directions of a
// pair, in the rows of the pair's first direction (2k + 1); the rest
// direction's term is zero.  The kernel then runs with weight 1 (omega = 0).
constexpr int FIELDS = 5;

// Row of lam_in read for direction i (PAIRS: the pair's first direction).
template <bool PAIRS>
__device__ __forceinline__ constexpr int direct_row(int i) { return PAIRS ? ((i - 1) | 1) : i; }

template <int BXT, int ROWS, bool WALLS, bool PAIRS>
__global__ void __launch_bounds__(BXT * ROWS)
adjoint_stream_kernel(const Grid g, const Phys ph, const Tiling tl, const uint32_t* __restrict__ links,
                      const float* __restrict__ lam_in, const float* __restrict__ m, float* __restrict__ lam_out,
                      double* __restrict__ drho0) {
  constexpr int NT = BXT * ROWS;
  constexpr int EX = BXT + 2, EY = ROWS + 2, PLANE = EX * EY;
  constexpr int LPT = (PLANE + NT - 1) / NT;  // ring cells loaded per thread
  constexpr int SLOTS = 4;
  __shared__ float ring[SLOTS * FIELDS * PLANE];

  const int tid = threadIdx.x;
  const int b = xcd_remap(blockIdx.x, gridDim.x);
  const int tiles_xy = tl.tiles_x * tl.tiles_y;
  const int bz = b / tiles_xy;
  const int rem = b - bz * tiles_xy;
  const int byy = rem / tl.tiles_x;
  const int bxx = rem - byy * tl.tiles_x;
  const int x0 = bxx * BXT, y0 = byy * ROWS, z0 = bz * tl.zchunk;
  const int z1 = min(z0 + tl.zchunk, g.nz);
  const int kmax = z1 - z0 + 1;  // planes p_k = z0 - 1 + k, k = 0..kmax
  const uint32_t n = static_cast<uint32_t>(g.n);

  // Ring cells of this thread: in-plane offsets of their (wrapped) columns.
  uint32_t loff[LPT];
  bool lhas[LPT];
#pragma unroll
  for (int j = 0; j < LPT; ++j) {
    const int l = tid + j * NT;
    lhas[j] = l < PLANE;
    const int ly = l / EX, lx = l - (l / EX) * EX;
    loff[j] = static_cast<uint32_t>(wrap(y0 + ly - 1, g.ny)) * g.nx + static_cast<uint32_t>(wrap(x0 + lx - 1, g.nx));
  }
  float fv[LPT][FIELDS];
  auto fetch = [&](int p) {
    const uint32_t base = static_cast<uint32_t>(wrap(p, g.nz)) * g.nxy;
#pragma unroll
    for (int j = 0; j < LPT; ++j)
#pragma unroll
      for (int f = 0; f < FIELDS; ++f) fv[j][f] = lhas[j] ? m[f * n + base + loff[j]] : 0.0f;
  };
  auto publish = [&](int slot) {
#pragma unroll
    for (int j = 0; j < LPT; ++j) {
      if (!lhas[j]) continue;
      const int l = tid + j * NT;
#pragma unroll
      for (int f = 0; f < FIELDS; ++f) ring[(slot * FIELDS + f) * PLANE + l] = fv[j][f];
    }
  };

  const int tx = tid % BXT, ty = tid / BXT;
  const int ex = x0 + tx, ey = y0 + ty;
  const bool owner = ex < g.nx && ey < g.ny;
  const Column col = make_column<float>(ex, ey, g);
  const uint32_t col_b = col.y[1] + col.x[1];
  const uint32_t col_off = col.cell;
  const int at = (ty + 1) * EX + tx + 1;
  const uint32_t ppb = g.pstride * 4u;
  const float keep[2] = {1.0f - ph.omega[0], 1.0f - ph.omega[1]};

  // lam_{t+1} as read by plane p: population i of cell y comes from y + c_i,
  // or from y itself through opp(i) when y + c_i is a wall.
  auto pull_lam = [&](int p, float (&dst)[2][Q], uint32_t& lk) {
    const int zw = wrap(p, g.nz);
    __amdgpu_buffer_rsrc_t rz[3];
    rz[0] = plane_rsrc<float>(lam_in, wrap(p - 1, g.nz), g);
    rz[1] = plane_rsrc<float>(lam_in, zw, g);
    rz[2] = plane_rsrc<float>(lam_in, wrap(p + 1, g.nz), g);
    lk = 0u;
    if constexpr (WALLS) lk = links[static_cast<uint32_t>(zw) * g.nxy + col_off];
#pragma unroll
    for (int s = 0; s < 2; ++s) {
#pragma unroll
      for (int i = 0; i < Q; ++i) {
        if (PAIRS && i == 0) {
          dst[s][0] = 0.0f;
          continue;
        }
        const uint32_t fwd_off = col.y[1 + CY[i]] + col.x[1 + CX[i]];
        const int row = direct_row<PAIRS>(i);
        // after a bounce the source is opp(i) at the cell itself (same pair)
        const int brow = PAIRS ? row : opp(i);
        if constexpr (WALLS) {
          if (i != 0 && ((lk >> opp(i)) & 1u))
            dst[s][i] = buf_load<float, LOAD_BOUNCE>(rz[1], col_b, static_cast<uint32_t>(s * Q + brow) * ppb);
          else
            dst[s][i] = buf_load<float>(rz[1 + CZ[i]], fwd_off, static_cast<uint32_t>(s * Q + row) * ppb);
        } else {
          dst[s][i] = buf_load<float>(rz[1 + CZ[i]], fwd_off, static_cast<uint32_t>(s * Q + row) * ppb);
        }
      }
    }
  };

  float cur[2][Q], nxt[2][Q];
  uint32_t cur_lk = 0u, nxt_lk = 0u;
  for (int k = 0; k <= 2; ++k) {
    fetch(z0 - 1 + k);
    publish(k);
  }
  pull_lam(z0, cur, cur_lk);
  __syncthreads();

  for (int k = 1; k < kmax; ++k) {
    if (k + 2 <= kmax) fetch(z0 + 1 + k);
    if (k + 1 < kmax) pull_lam(z0 + k, nxt, nxt_lk);
    if (owner) {
      const int zc = wrap(z0 - 1 + k, g.nz);
      const uint32_t cell = static_cast<uint32_t>(zc) * g.nxy + col_off;
      const bool solid = WALLS && (cur_lk & 1u);
      const __amdgpu_buffer_rsrc_t rd = plane_rsrc<float>(lam_out, zc, g);
      const float* rp[3];
      rp[0] = ring + ((k + SLOTS - 1) % SLOTS) * FIELDS * PLANE;
      rp[1] = ring + (k % SLOTS) * FIELDS * PLANE;
      rp[2] = ring + ((k + 1) % SLOTS) * FIELDS * PLANE;
#pragma unroll
      for (int s = 0; s < 2; ++s) {
#pragma unroll
        for (int i = 0; i < Q; ++i) {
          float v = 0.0f;
          if (!solid) {
            const bool back = WALLS && (i != 0) && ((cur_lk >> opp(i)) & 1u);
            // the cell x: y + c_i, or y itself after a bounce
            const float* fx = back ? rp[1] : rp[1 + CZ[i]];
            const int ax = back ? at : at + CY[i] * EX + CX[i];
            const float A = fx[s * PLANE + ax];
            float dot = 0.0f;
            if (CX[i]) dot += CX[i] * fx[2 * PLANE + ax];
            if (CY[i]) dot += CY[i] * fx[3 * PLANE + ax];
            if (CZ[i]) dot += CZ[i] * fx[4 * PLANE + ax];
            v = keep[s] * cur[s][i] + A + (back ? -dot : dot);
          }
          buf_store<float>(v, rd, col_b, static_cast<uint32_t>(s * Q + i) * ppb);
        }
        if (drho0) {
          // dL/drho0^a(x) = sum_i w_i dL/df_i^a(x, 0): the initial pull reads
          // w_i rho0 at every population of the cell.
          double d = 0.0;
          if (!solid) {
            const __amdgpu_buffer_rsrc_t rc = plane_rsrc<float>(lam_in, zc, g);
            float acc = 0.0f;
#pragma unroll
            for (int i = PAIRS ? 1 : 0; i < Q; ++i)
              acc += weight(i) * buf_load<float>(rc, col_b, static_cast<uint32_t>(s * Q + direct_row<PAIRS>(i)) * ppb);
            d = static_cast<double>(keep[s] * acc + rp[1][s * PLANE + at]);
          }
          drho0[s * g.n + cell] = d;
        }
      }
    }
    if (k + 2 <= kmax) publish((k + 2) % SLOTS);
    __syncthreads();
    if (k + 1 < kmax) {
#pragma unroll
      for (int s = 0; s < 2; ++s)
#pragma unroll
        for (int i = 0; i < Q; ++i) cur[s][i] = nxt[s][i];
      cur_lk = nxt_lk;
    }
  }
}

unsigned grid_for_3d(const Grid& g) { return static_cast<unsigned>((g.nx + 63) / 64); }

dim3 grid3(const Grid& g) {
  return dim3(grid_for_3d(g), static_cast<unsigned>(g.ny), static_cast<unsigned>(g.nz));
}

// Stream-pass tiling: 64 x 4 or 32 x 8 columns (whichever pads the x-y plane
// less), chunks of 8 to 32 planes with about two workgroups per CU.
struct StreamShape {
  int bx, rows;
};
constexpr StreamShape STREAM_SHAPES[2] = {{64, 4}, {32, 8}};

Tiling stream_tiling(const Grid& g, int& shape) {
  long long best = -1;
  shape = 0;
  for (int k = 0; k < 2; ++k) {
    const StreamShape sh = STREAM_SHAPES[k];
    const long long cells = static_cast<long long>((g.nx + sh.bx - 1) / sh.bx) * sh.bx *
                            (static_cast<long long>((g.ny + sh.rows - 1) / sh.rows) * sh.rows);
    if (best < 0 || cells < best) {
      best = cells;
      shape = k;
    }
  }
  const StreamShape sh = STREAM_SHAPES[shape];
  Tiling t{};
  t.tile = shape;
  t.tiles_x = (g.nx + sh.bx - 1) / sh.bx;
  t.tiles_y = (g.ny + sh.rows - 1) / sh.rows;
  const long long txy = static_cast<long long>(t.tiles_x) * t.tiles_y;
  long long zc = static_cast<long long>(g.nz) * txy / 512;
  if (zc < 8) zc = 8;
  if (zc > 32) zc = 32;
  if (zc > g.nz) zc = g.nz;
  t.zchunk = static_cast<int>(zc);
  t.tiles_z = (g.nz + t.zchunk - 1) / t.zchunk;
  const long long nb = txy * t.tiles_z;
  t.blocks = nb > 0x7fffffffLL ? -1 : static_cast<int>(nb);
  return t;
}

}  // namespace

hipError_t launch_adjoint_gather(const Grid& g, const uint32_t* links, float* m, const float* sbar,
                                 hipStream_t st) {
  // The six Sbar planes are indexed with 32-bit offsets.
  if (g.n * SBAR_FIELDS > 0xffffffffull) return hipErrorInvalidValue;
  // The stream pass's column tiles in shorter chunks (about eight workgroups
  // per CU): the pass is short and its chunks' first planes cost little.
  int shape = 0;
  Tiling t = stream_tiling(g, shape);
  if (t.blocks <= 0) return hipErrorInvalidValue;
  long long zc = static_cast<long long>(g.nz) * t.tiles_x * t.tiles_y / 2048;
  if (zc < 4) zc = 4;
  if (zc > 32) zc = 32;
  if (zc > g.nz) zc = g.nz;
  t.zchunk = static_cast<int>(zc);
  t.tiles_z = (g.nz + t.zchunk - 1) / t.zchunk;
  const long long nb = static_cast<long long>(t.tiles_x) * t.tiles_y * t.tiles_z;
  if (nb > 0x7fffffffLL) return hipErrorInvalidValue;
  t.blocks = static_cast<int>(nb);
  const dim3 gr(static_cast<unsigned>(t.blocks)), bl(256);
  if (shape == 0)
    hipLaunchKernelGGL((adjoint_gather_kernel<64, 4>), gr, bl, 0, st, g, t, links, m, sbar);
  else
    hipLaunchKernelGGL((adjoint_gather_kernel<32, 8>), gr, bl, 0, st, g, t, links, m, sbar);
  return hipGetLastError();
}

template <bool PAIRS>
static void launch_stream_variant(int shape, const dim3& gr, const Grid& g, const Phys& ph, const Tiling& t,
                                  const uint32_t* links, const float* lam_in, const float* m, float* lam_out,
                                  double* drho0, hipStream_t st) {
  const dim3 bl(256);
  if (shape == 0) {
    if (links)
      hipLaunchKernelGGL((adjoint_stream_kernel<64, 4, true, PAIRS>), gr, bl, 0, st, g, ph, t, links, lam_in, m,
                         lam_out, drho0);
    else
      hipLaunchKernelGGL((adjoint_stream_kernel<64, 4, false, PAIRS>), gr, bl, 0, st, g, ph, t, links, lam_in, m,
                         lam_out, drho0);
  } else {
    if (links)
      hipLaunchKernelGGL((adjoint_stream_kernel<32, 8, true, PAIRS>), gr, bl, 0, st, g, ph, t, links, lam_in, m,
                         lam_out, drho0);
    else
      hipLaunchKernelGGL((adjoint_stream_kernel<32, 8, false, PAIRS>), gr, bl, 0, st, g, ph, t, links, lam_in, m,
                         lam_out, drho0);
  }
}

hipError_t launch_adjoint_stream(const Grid& g, const Phys& ph, const uint32_t* links, const float* lam_in,
                                 const float* m, float* lam_out, double* drho0, bool pairs, hipStream_t st) {
  // The five field planes are indexed with 32-bit offsets.
  if (g.n * FIELDS > 0xffffffffull) return hipErrorInvalidValue;
  int shape = 0;
  const Tiling t = stream_tiling(g, shape);
  if (t.blocks <= 0) return hipErrorInvalidValue;
  const dim3 gr(static_cast<unsigned>(t.blocks));
  if (pairs)
    launch_stream_variant<true>(shape, gr, g, ph, t, links, lam_in, m, lam_out, drho0, st);
  else
    launch_stream_variant<false>(shape, gr, g, ph, t, links, lam_in, m, lam_out, drho0, st);
  return hipGetLastError();
}

hipError_t launch_adjoint_seed(const Grid& g, const uint32_t* links, const float* grad_rho, float* lam,
                               hipStream_t st) {
  if (g.ny > 65535 || g.nz > 65535) return hipErrorInvalidValue;
  hipLaunchKernelGGL(adjoint_seed_kernel, grid3(g), dim3(64), 0, st, g, links, grad_rho, lam);
  return hipGetLastError();
}

}  // namespace lbm
