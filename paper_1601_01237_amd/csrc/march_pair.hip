// Paired z-march of the 16-bit storage forms (gfx950).
//
// The 16-bit forms with even nx store each row folded: 32-bit word k holds
// cells k (low half) and k + nx/2 (high half).  One lane here owns one word,
// so every population read and write is one aligned 32-bit access covering
// two cells, half the memory instructions of a 16-bit access per cell (the
// per-lane instruction rate, not HBM bandwidth, bounds 16-bit loads on this
// part).  The x neighbours of both cells of word k sit in words k - 1 and
// k + 1; only where the fold is crossed (k = 0 going left, k = nx/2 - 1 going
// right) do the two halves of the neighbouring word trade places.
//
// Structure follows the single-cell march: a workgroup owns BK words x ROWS
// rows (2 BK x ROWS cells in two x segments) and marches up a chunk of z
// planes; densities go through a 5-slot LDS ring (float4 per word: rho~^A,
// rho~^B of the low cell, then of the high cell) that also holds the one-word
// halo computed by HW halo waves one plane ahead.  Each step pulls the 38
// words of its cells (Eq. 1), forms the stored sums, and, one plane behind,
// takes the full Shan-Chen sum (Eq. 7) and collides the low cell and then
// the high cell (Eqs. 2-9, or Eqs. 10-11), writing both halves back into the
// words before one 32-bit store per population.  The cell arithmetic is the
// same code as the single-cell march, so both give bit-identical states.
// Periodic boundaries only (no wall links); Step mode only.

#include "buffer.h"
#include "cell.h"
#include "launch.h"

namespace lbm {

namespace {

// Addressing of the word at unbounded row position d (cells d and d + H in
// an unfolded, periodically extended row, H = nx / 2) in row ey.
struct PairColumn {
  uint32_t x[3];  // byte offsets of the words holding the x-1, x, x+1 neighbours
  uint32_t y[3];  // byte offsets of rows y-1, y, y+1
  bool swap_p;    // c_x = +1 source crosses the fold: halves of word x[0] traded
  bool swap_m;    // c_x = -1 source crosses the fold: halves of word x[2] traded
  bool flip;      // position d maps to the word with its halves traded
};

__device__ __forceinline__ PairColumn make_pair_column(int d, int ey, const Grid& g) {
  const int H = static_cast<int>(g.half);
  const int m = wrap(d, H);
  PairColumn c;
  c.x[0] = static_cast<uint32_t>(m == 0 ? H - 1 : m - 1) * 4u;
  c.x[1] = static_cast<uint32_t>(m) * 4u;
  c.x[2] = static_cast<uint32_t>(m == H - 1 ? 0 : m + 1) * 4u;
  c.swap_p = m == 0;
  c.swap_m = m == H - 1;
  c.flip = wrap(d, 2 * H) >= H;
  const int gy = wrap(ey, g.ny);
  const int ym = gy == 0 ? g.ny - 1 : gy - 1;
  const int yp = gy == g.ny - 1 ? 0 : gy + 1;
  c.y[0] = row_off(ym, g) * 2u;
  c.y[1] = row_off(gy, g) * 2u;
  c.y[2] = row_off(yp, g) * 2u;
  return c;
}

__device__ __forceinline__ uint32_t trade_halves(uint32_t w) { return __builtin_amdgcn_alignbit(w, w, 16); }

// Words of one species per column: the 19 directions, then (index Q) the
// residual of the rest population (launch.h).
constexpr int QW = Q + 1;

// Pull (Eq. 1) of the words of species s for the two cells of column c: the
// loads, then (fold_fix, once the words are in) the trade of halves for the
// sources across the fold.  The rest population and its residual come from
// the column itself.
template <Storage S>
__device__ __forceinline__ void pull_words(const __amdgpu_buffer_rsrc_t rz[3], uint32_t ppb, const PairColumn& c,
                                           int s, uint32_t w[QW]) {
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const uint32_t off = c.y[1 - CY[i]] + c.x[1 - CX[i]];
    w[i] = __builtin_amdgcn_raw_buffer_load_b32(rz[1 - CZ[i]], off, static_cast<uint32_t>(s * Q + i) * ppb, 0);
  }
  w[Q] = __builtin_amdgcn_raw_buffer_load_b32(rz[1], c.y[1] + c.x[1], static_cast<uint32_t>(RES_ROW + s) * ppb, 0);
}

__device__ __forceinline__ void fold_fix(const PairColumn& c, uint32_t w[2][QW]) {
  if (c.swap_p) {
#pragma unroll
    for (int s = 0; s < 2; ++s) {
#pragma unroll
      for (int i = 0; i < Q; ++i)
        if (CX[i] == 1) w[s][i] = trade_halves(w[s][i]);
    }
  }
  if (c.swap_m) {
#pragma unroll
    for (int s = 0; s < 2; ++s) {
#pragma unroll
      for (int i = 0; i < Q; ++i)
        if (CX[i] == -1) w[s][i] = trade_halves(w[s][i]);
    }
  }
}

// Stored sums D (direction order, as pull_species) of the low and high cell.
template <Storage S>
__device__ __forceinline__ void word_sums(const uint32_t w[QW], float& dl, float& dh) {
  using Tr = StorageTraits<S>;
  dl = Tr::lo(w[0]) + Tr::lo(w[Q]) * (1.0f / Tr::res_scale);
  dh = Tr::hi(w[0]) + Tr::hi(w[Q]) * (1.0f / Tr::res_scale);
#pragma unroll
  for (int i = 1; i < Q; ++i) {
    dl += Tr::lo(w[i]);
    dh += Tr::hi(w[i]);
  }
}

template <Storage S>
__device__ __forceinline__ float4 ring_entry(const uint32_t w[2][QW], const Phys& ph, bool flip, float d[2][2]) {
  word_sums<S>(w[0], d[0][0], d[1][0]);
  word_sums<S>(w[1], d[0][1], d[1][1]);
  const float4 r = make_float4(density<S>(d[0][0], ph.shift[0]), density<S>(d[0][1], ph.shift[1]),
                               density<S>(d[1][0], ph.shift[0]), density<S>(d[1][1], ph.shift[1]));
  return flip ? make_float4(r.z, r.w, r.x, r.y) : r;
}

// Populations f_i = X_i of cell c (0 = low, 1 = high half) of both species,
// decoded exactly as the single-cell pull does.
template <Storage S>
__device__ __forceinline__ void decode_cell(const uint32_t w[2][QW], int c, const float ws[2][3], float f[2][Q]) {
  using Tr = StorageTraits<S>;
#pragma unroll
  for (int s = 0; s < 2; ++s) {
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      float x = c == 0 ? Tr::lo(w[s][i]) : Tr::hi(w[s][i]);
      if (i == 0) x += (c == 0 ? Tr::lo(w[s][Q]) : Tr::hi(w[s][Q])) * (1.0f / Tr::res_scale);
      f[s][i] = x + ws[s][i == 0 ? 0 : (i <= 6 ? 1 : 2)];
    }
  }
}

template <int BK, int ROWS, int HW>
struct PairShape {
  static constexpr int NOWN = BK * ROWS;
  static constexpr int EX = BK + 2;
  static constexpr int EY = ROWS + 2;
  static constexpr int NH = 2 * EX + 2 * ROWS;
  static constexpr int NT = NOWN + 64 * HW;
  static constexpr int HPL = (NH + 64 * HW - 1) / (64 * HW);
  static constexpr int SLOTS = 5;
  static_assert(NOWN % 64 == 0, "own lanes fill whole waves");
};

template <int BK, int ROWS>
__device__ __forceinline__ void pair_halo_pos(int h, int& hx, int& hy) {
  constexpr int EX = BK + 2;
  if (h < EX) { hx = h - 1; hy = -1; }
  else if (h < 2 * EX) { hx = h - EX - 1; hy = ROWS; }
  else if (h < 2 * EX + ROWS) { hx = -1; hy = h - 2 * EX; }
  else { hx = BK; hy = h - 2 * EX - ROWS; }
}

// Ring slots: plane p_k (the k-th plane a workgroup loads) lives in slot
// k % 5.  Before barrier k the own waves have written their words of p_k and
// the halo waves p_0 .. p_{k+1}; after it the own waves collide plane
// p_{k-1} from slots (k-2), (k-1), k while the halo waves fill p_{k+2} into
// slot (k+2) % 5, whose last readers finished before barrier k.
template <Storage S, int BK, int ROWS, int HW, int REG>
__global__ void __launch_bounds__(BK * ROWS + 64 * HW)
march_pair_kernel(const Grid g, const Phys ph, const Tiling tl, const MarchIO io) {
  using Sh = PairShape<BK, ROWS, HW>;
  using Tr = StorageTraits<S>;
  using T = typename Tr::T;
  constexpr int EX = Sh::EX;
  constexpr int PLANE = Sh::EX * Sh::EY;
  __shared__ float4 ring[Sh::SLOTS * PLANE];

  const int tid = threadIdx.x;
  const int b = xcd_remap(blockIdx.x, gridDim.x);
  const TileCoord tc = tile_of_block(b, tl);
  const int bxx = tc.x, byy = tc.y, bz = tc.z;
  const int k0 = bxx * BK, y0 = byy * ROWS, z0 = bz * tl.zchunk;
  const int z1 = min(z0 + tl.zchunk, g.nz);
  const int kmax = z1 - z0 + 1;  // planes p_k = z0 - 1 + k for k = 0..kmax
  const uint32_t ppb = g.pstride * static_cast<uint32_t>(sizeof(T));

  float ws[2][3];
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    ws[s][0] = W0 * ph.shift[s];
    ws[s][1] = WF * ph.shift[s];
    ws[s][2] = WE * ph.shift[s];
  }

  if (tid < Sh::NOWN) {
    // ------------------------------------------------------------ own waves
    const int tx = tid % BK, ty = tid / BK;
    const int d = k0 + tx, ey = y0 + ty;
    const bool owner = d < static_cast<int>(g.half) && ey < g.ny;  // others only feed the ring
    const PairColumn col = make_pair_column(d, ey, g);
    const uint32_t col_b = col.y[1] + col.x[1];
    const int at = (ty + 1) * EX + tx + 1;

    // Words of three planes: cur = p_{k-1} (collided after barrier k),
    // nxt = p_k (its densities go into the ring before barrier k) and ahead =
    // p_{k+1}, loaded one iteration early so that its latency overlaps the
    // barrier and the collision of p_{k-1}.
    uint32_t cur[2][QW], nxt[2][QW], ahead[2][QW];
    float cur_d[2][2] = {{0.f, 0.f}, {0.f, 0.f}}, nxt_d[2][2];  // stored sums [cell][species]
    int slot = 0;  // k % 5
    auto load_plane = [&](int k, uint32_t w[2][QW]) {
      const int p = z0 - 1 + k;
      __amdgpu_buffer_rsrc_t rz[3];
      rz[0] = plane_rsrc<T>(io.src, wrap(p - 1, g.nz), g);
      rz[1] = plane_rsrc<T>(io.src, wrap(p, g.nz), g);
      rz[2] = plane_rsrc<T>(io.src, wrap(p + 1, g.nz), g);
      pull_words<S>(rz, ppb, col, 0, w[0]);
      pull_words<S>(rz, ppb, col, 1, w[1]);
    };
    load_plane(0, nxt);

    for (int k = 0; k <= kmax; ++k) {
      const int p = z0 - 1 + k;
      if (k < kmax) load_plane(k + 1, ahead);
      fold_fix(col, nxt);
      ring[slot * PLANE + at] = ring_entry<S>(nxt, ph, col.flip, nxt_d);

      if (k >= 1) {
        __syncthreads();
        if (k >= 2 && owner) {
          const int zc = wrap(p - 1, g.nz);
          const int s2 = slot >= 2 ? slot - 2 : slot + 3;  // (k-2) % 5
          const int s1 = slot >= 1 ? slot - 1 : slot + 4;  // (k-1) % 5
          float SC[4][3];  // [component of the ring entry][axis]
          shan_chen_partial<EX, 4>(ring + s2 * PLANE, ring + s1 * PLANE, at, SC);
          shan_chen_finish<EX, 4>(ring + slot * PLANE, at, SC);
          const __amdgpu_buffer_rsrc_t rd = plane_rsrc<T>(io.dst, zc, g);
#pragma unroll
          for (int c = 0; c < 2; ++c) {
            float f[2][Q];
            decode_cell<S>(cur, c, ws, f);
            const float ra = density<S>(cur_d[c][0], ph.shift[0]);
            const float rb = density<S>(cur_d[c][1], ph.shift[1]);
            float u[3];
            mixture_velocity(f, ra + rb, u);
            const float Sc[2][3] = {{SC[2 * c][0], SC[2 * c][1], SC[2 * c][2]},
                                    {SC[2 * c + 1][0], SC[2 * c + 1][1], SC[2 * c + 1][2]}};
            Local L;
            make_local(ra, rb, u, Sc, ph, L);
            if constexpr (REG != 0) {
              collide_regularized<REG == 2>(f, L, ph);
            } else {
              collide(f, L, ph);
            }
#pragma unroll
            for (int s = 0; s < 2; ++s) {
              encode_species<S>(f[s], cur_d[c][s], ws[s], [&](int i, T q) {
                const uint32_t v = Tr::bits(q);
                cur[s][i] = c == 0 ? ((cur[s][i] & 0xffff0000u) | v) : ((cur[s][i] & 0xffffu) | (v << 16));
              });
            }
          }
#pragma unroll
          for (int s = 0; s < 2; ++s) {
#pragma unroll
            for (int i = 0; i < QW; ++i)
              __builtin_amdgcn_raw_buffer_store_b32(cur[s][i], rd, col_b,
                                                    static_cast<uint32_t>(store_row(s, i)) * ppb, STORE_NT);
          }
        }
      }

#pragma unroll
      for (int s = 0; s < 2; ++s) {
#pragma unroll
        for (int i = 0; i < QW; ++i) {
          cur[s][i] = nxt[s][i];
          nxt[s][i] = ahead[s][i];
        }
        cur_d[0][s] = nxt_d[0][s];
        cur_d[1][s] = nxt_d[1][s];
      }
      slot = slot == 4 ? 0 : slot + 1;
    }
  } else {
    // ----------------------------------------------------------- halo waves
    const int hl = tid - Sh::NOWN;
    int hat[Sh::HPL];
    PairColumn hcol[Sh::HPL];
    bool has[Sh::HPL];
#pragma unroll
    for (int j = 0; j < Sh::HPL; ++j) {
      const int h = hl + j * 64 * HW;
      has[j] = h < Sh::NH;
      int hx = 0, hy = 0;
      pair_halo_pos<BK, ROWS>(has[j] ? h : 0, hx, hy);
      hcol[j] = make_pair_column(k0 + hx, y0 + hy, g);
      hat[j] = (hy + 1) * EX + hx + 1;
    }

    auto halo_plane = [&](int k) {
      const int p = z0 - 1 + k;
      __amdgpu_buffer_rsrc_t rz[3];
      rz[0] = plane_rsrc<T>(io.src, wrap(p - 1, g.nz), g);
      rz[1] = plane_rsrc<T>(io.src, wrap(p, g.nz), g);
      rz[2] = plane_rsrc<T>(io.src, wrap(p + 1, g.nz), g);
      const int sl = k % 5;
#pragma unroll
      for (int j = 0; j < Sh::HPL; ++j) {
        if (!has[j]) continue;
        uint32_t w[2][QW];
        float hd[2][2];
        pull_words<S>(rz, ppb, hcol[j], 0, w[0]);
        pull_words<S>(rz, ppb, hcol[j], 1, w[1]);
        fold_fix(hcol[j], w);
        ring[sl * PLANE + hat[j]] = ring_entry<S>(w, ph, hcol[j].flip, hd);
      }
    };

    // Planes p_0 .. p_2 before the first barrier, then p_{k+2} after barrier
    // k.  (The single-cell march fills p_{k+1} there, in step with its own
    // pulls; with the own loads prefetched here, that put the halo loads on
    // the critical path: 6.3 against 4.7 ms at 512^3.)
    for (int k = 0; k <= min(2, kmax); ++k) halo_plane(k);
    for (int k = 1; k <= kmax; ++k) {
      __syncthreads();
      if (k + 2 <= kmax) halo_plane(k + 2);
    }
  }
}

template <Storage S, int BK, int ROWS, int HW, int REG>
hipError_t launch_pair_shape(const Grid& g, const Phys& ph, const Tiling& t, const MarchIO& io, hipStream_t st) {
  using Sh = PairShape<BK, ROWS, HW>;
  hipLaunchKernelGGL((march_pair_kernel<S, BK, ROWS, HW, REG>), dim3(t.blocks), dim3(Sh::NT), 0, st, g, ph, t, io);
  return hipGetLastError();
}

template <Storage S, int REG>
hipError_t launch_pair_reg(const Grid& g, const Phys& ph, const Tiling& t, const MarchIO& io, hipStream_t st) {
  switch (t.tile) {
    case 6: return launch_pair_shape<S, 64, 8, 3, REG>(g, ph, t, io, st);
    case 7: return launch_pair_shape<S, 32, 16, 2, REG>(g, ph, t, io, st);
    case 8: return launch_pair_shape<S, 32, 8, 2, REG>(g, ph, t, io, st);
    case 9: return launch_pair_shape<S, 32, 12, 2, REG>(g, ph, t, io, st);
    default: return hipErrorInvalidValue;
  }
}

template <Storage S>
hipError_t launch_pair_storage(const Grid& g, const Phys& ph, const Tiling& t, const MarchIO& io, hipStream_t st) {
  switch (ph.regularized) {
    case 0: return launch_pair_reg<S, 0>(g, ph, t, io, st);
    case 1: return launch_pair_reg<S, 1>(g, ph, t, io, st);
    case 2: return launch_pair_reg<S, 2>(g, ph, t, io, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

hipError_t launch_pair_step(Storage s, const Grid& g, const Phys& ph, const Tiling& t, const MarchIO& io,
                            hipStream_t st) {
  if (t.blocks <= 0 || g.half == 0 || io.links != nullptr) return hipErrorInvalidValue;
  switch (s) {
    case Storage::F16: return launch_pair_storage<Storage::F16>(g, ph, t, io, st);
    case Storage::BF16: return launch_pair_storage<Storage::BF16>(g, ph, t, io, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace lbm
