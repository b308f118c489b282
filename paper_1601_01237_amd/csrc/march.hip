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
// The same march serves two bodies:
//   Step     collide and store X_{t+1}(x) = f*(x)  (post-collision state);
//   Moments  rho^a and u_F fields plus FP64 per-workgroup diagnostic sums.
// (The reverse step has a march of its own, adjoint_march.hip.)
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

#include "pull.h"

namespace lbm {

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

template <Storage S, bool WALLS, Mode M, int BXT, int ROWS, int HW, int REG>
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
  // Link words of the wall classes (buffer.h).
  __shared__ uint32_t ltab[WALLS ? WALL_CLASSES : 1];
  if constexpr (WALLS) load_wall_classes(io.cls, io.ltab, ltab, tid, Sh::NT);
  const int b = xcd_remap(blockIdx.x, gridDim.x);
  // Which tile and z chunk: the launch's block order (launch.h).
  const TileCoord tc = tile_of_block(b, tl);
  const int bxx = tc.x, byy = tc.y, bz = tc.z;
  // The tile grid may be shifted in x by tl.xoff cells (wrapping): tile
  // column bxx covers x = bxx * BXT + xoff + tx (mod nx); the lane owns its
  // cell when the unshifted column bxx * BXT + tx lies inside the grid.
  const int lx0 = bxx * BXT;
  const int x0 = lx0 + tl.xoff, y0 = byy * ROWS, z0 = bz * tl.zchunk;
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

  constexpr int NV = 16;  // diagnostic sums (Moments)
  double acc[NV];
#pragma unroll
  for (int k = 0; k < NV; ++k) acc[k] = 0.0;

  if (tid < Sh::NOWN) {
    // ------------------------------------------------------------ own waves
    const int tx = tid % BXT, ty = tid / BXT;
    const int ex = x0 + tx, ey = y0 + ty;
    const bool owner = lx0 + tx < g.nx && ey < g.ny;  // ragged edge lanes only feed the ring
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
    // Wall data of the plane pulled next, loaded one plane ahead (the pull
    // addresses of a plane depend on its link words).
    uint32_t ahead = 0;
    if constexpr (WALLS) ahead = wall_raw(io.cls, io.links, static_cast<uint32_t>(wrap(z0 - 1, g.nz)) * g.nxy + col_off);
    int slot = 0;  // k % 5

    for (int k = 0; k <= kmax; ++k) {
      const int p = z0 - 1 + k;
      const int zw = wrap(p, g.nz);
      __amdgpu_buffer_rsrc_t rz[3];
      rz[0] = plane_rsrc<T>(io.src, wrap(p - 1, g.nz), g);
      rz[1] = plane_rsrc<T>(io.src, zw, g);
      rz[2] = plane_rsrc<T>(io.src, wrap(p + 1, g.nz), g);
      if constexpr (WALLS) {
        nxt_links = link_word(io.cls, ltab, ahead);
        if (k < kmax) ahead = wall_raw(io.cls, io.links, static_cast<uint32_t>(wrap(p + 1, g.nz)) * g.nxy + col_off);
      }
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
      if constexpr (M == Mode::StepFields) {
        // the chunk's own planes: rho~ (rho_s on wall cells) and u (0 there)
        // (non-temporal: read back by a reverse step much later, they should
        // not displace the lines neighbouring tiles still need)
        if (owner && k >= 1 && k < kmax) {
          const uint32_t c = static_cast<uint32_t>(zw) * g.nxy + col_off;
          const float2 rr = ring[slot * PLANE + at];
          __builtin_nontemporal_store(rr.x, io.fields + c);
          __builtin_nontemporal_store(rr.y, io.fields + n + c);
          __builtin_nontemporal_store(solid ? 0.0f : nxt_u[0], io.fields + 2 * n + c);
          __builtin_nontemporal_store(solid ? 0.0f : nxt_u[1], io.fields + 3 * n + c);
          __builtin_nontemporal_store(solid ? 0.0f : nxt_u[2], io.fields + 4 * n + c);
        }
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
            if constexpr (M == Mode::Step || M == Mode::StepFields) {
              if (!csolid) {
                shan_chen_finish<EX, 2>(ring + slot * PLANE, at, cur_S);
                Local L;
                make_local(density<S>(cur_d[0], ph.shift[0]), density<S>(cur_d[1], ph.shift[1]), cur_u, cur_S,
                           ph, L);
                if constexpr (REG != 0) {
                  collide_regularized<REG == 2>(cur, L, ph);
                } else {
                  collide(cur, L, ph);
                }
                const __amdgpu_buffer_rsrc_t rd = plane_rsrc<T>(io.dst, zc, g);
#pragma unroll
                for (int s = 0; s < 2; ++s) {
                  if constexpr (Tr::shifted) {
                    encode_species<S>(cur[s], cur_d[s], ws[s], [&](int i, T q) {
                      buf_store<T>(q, rd, col_b, static_cast<uint32_t>(store_row(s, i)) * ppb);
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
            }
          }
        }
        // Planes p_{k-1} and p_k are complete: the first part of S for plane p_k.
        if (k < kmax) shan_chen_partial<EX, 2>(ring + sm1 * PLANE, ring + slot * PLANE, at, nxt_S);
      }

#pragma unroll
      for (int s = 0; s < 2; ++s) {
#pragma unroll
        for (int i = 0; i < Q; ++i) cur[s][i] = nxt[s][i];
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
        if constexpr (WALLS) lk = cell_links(io.cls, ltab, io.links, static_cast<uint32_t>(zw) * g.nxy + hcol_off[j]);
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

  if constexpr (M == Mode::Moments) {
    bool is_max[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) is_max[k] = k == 5;
    __syncthreads();
    block_reduce_store<NV>(acc, is_max, io.partials + static_cast<uint64_t>(blockIdx.x) * NV, red);
  }
}

// ---------------------------------------------------------------------------
// Launch
// ---------------------------------------------------------------------------

// Tile shapes selectable at run time: (columns of cells, rows, halo waves);
// shapes 6..9 are the paired march over folded 16-bit rows (2 cells per lane).
// 64 x 12 takes two halo waves (some lanes fill two ring cells): against
// three, 3% faster on the inclined-channel walls case, the same on open boxes.
struct TileShape {
  int bx, rows, hw;
};
constexpr TileShape TILES[] = {{64, 8, 3},  {64, 12, 2}, {32, 16, 2}, {128, 4, 3}, {64, 4, 3},
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
  t.order = ORDER_PLANE_X;
  t.xoff = 0;
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
  // population rows), then 64 x 12; a shape is taken when it pads the x-y
  // plane (lanes past nx or ny do no work) by at most 30% more than the least
  // padded candidate, the first such in this order.  Measured (open cubes,
  // ms per step, against the least padded shape alone): 144^3 0.239 (64 x 12)
  // against 0.266, 192^3 0.444 (64 x 12) against 0.473, 224^3 0.749
  // (128 x 4, padded 14%) against 0.871.  With walls (the 128 x 4 shape
  // keeps too few registers for the wall path) and for unfolded 16-bit rows
  // 64 x 8 comes first, and the least padded shape wins (64 x 12 was 14%
  // faster on an inclined channel but 25% slower on a random porous medium).
  // Folded 16-bit rows without walls take the paired march in 32 x 8 words
  // (measured fastest of the pair shapes at 512^3: one 128-byte line per
  // population row and six waves per CU).
  static constexpr int open_order[] = {3, 1, 0, 2};
  static constexpr int tall_order[] = {0, 2};
  static constexpr int pair_order[] = {8};
  const bool paired = elem_bytes == 2 && g.half != 0 && !walls;
  const bool tall = walls || elem_bytes != 4;
  const int* order = paired ? pair_order : (tall ? tall_order : open_order);
  const int count = paired ? 1 : (tall ? 2 : 4);
  const long long slack = (paired || tall) ? 10 : 13;  // tenths of the least padded plane
  long long cells[4];
  long long least = -1;
  for (int k = 0; k < count; ++k) {
    const TileShape sh = TILES[order[k]];
    cells[k] = static_cast<long long>((g.nx + sh.bx - 1) / sh.bx) * sh.bx *
               (static_cast<long long>((g.ny + sh.rows - 1) / sh.rows) * sh.rows);
    if (least < 0 || cells[k] < least) least = cells[k];
  }
  for (int k = 0; k < count; ++k)
    if (cells[k] * 10 <= least * slack) return order[k];
  return order[0];
}

template <Storage S, bool WALLS, Mode M, int BXT, int ROWS, int HW, int REG = 0>
static hipError_t launch_shape(const Grid& g, const Phys& ph, const Tiling& t, const MarchIO& io,
                               hipStream_t st) {
  using Sh = Shape<BXT, ROWS, HW>;
  hipLaunchKernelGGL((march_kernel<S, WALLS, M, BXT, ROWS, HW, REG>), dim3(t.blocks), dim3(Sh::NT), 0, st, g, ph,
                     t, io);
  return hipGetLastError();
}

template <Storage S, bool WALLS, int REG, Mode M = Mode::Step>
static hipError_t launch_step(const Grid& g, const Phys& ph, const Tiling& t, const MarchIO& io, hipStream_t st) {
  switch (t.tile) {
    case 0: return launch_shape<S, WALLS, M, 64, 8, 3, REG>(g, ph, t, io, st);
    case 1: return launch_shape<S, WALLS, M, 64, 12, 2, REG>(g, ph, t, io, st);
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
    switch (ph.regularized) {
      case 0: return launch_step<S, WALLS, 0>(g, ph, t, io, st);
      case 1: return launch_step<S, WALLS, 1>(g, ph, t, io, st);
      case 2: return launch_step<S, WALLS, 2>(g, ph, t, io, st);
      default: return hipErrorInvalidValue;
    }
  } else if constexpr (M == Mode::Moments) {
    // Diagnostics use one shape (tile 0).
    if (t.tile != 0) return hipErrorInvalidValue;
    return launch_shape<S, WALLS, M, 64, 8, 3>(g, ph, t, io, st);
  } else if constexpr (M == Mode::StepFields && S == Storage::F32) {
    if (!io.fields) return hipErrorInvalidValue;
    switch (ph.regularized) {
      case 0: return launch_step<S, WALLS, 0, M>(g, ph, t, io, st);
      case 1: return launch_step<S, WALLS, 1, M>(g, ph, t, io, st);
      case 2: return launch_step<S, WALLS, 2, M>(g, ph, t, io, st);
      default: return hipErrorInvalidValue;
    }
  } else {
    return hipErrorInvalidValue;
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
    case Mode::StepFields: return launch_walls<S, Mode::StepFields>(g, ph, t, io, st);
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
  switch (s) {
    case Storage::F32: return launch_mode<Storage::F32>(mode, g, ph, t, io, st);
    case Storage::F16: return launch_mode<Storage::F16>(mode, g, ph, t, io, st);
    case Storage::BF16: return launch_mode<Storage::BF16>(mode, g, ph, t, io, st);
  }
  return hipErrorInvalidValue;
}

}  // namespace lbm
