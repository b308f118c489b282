// Fused reverse (adjoint) step of the two-component D3Q19 update (gfx950).
//
// One step maps the stored state X_t to X_{t+1} = stream(collide(pull(X_t)))
// (Eq. 1 with the collision of Eq. 2 or Eqs. 10-11, the Shan-Chen force of
// Eq. 7 and halfway bounce-back, Sec. 4).  Given lam_{t+1} = dL/dX_{t+1} this
// kernel writes lam_t = dL/dX_t in one z march, in the frame of the cell x
// whose collision is transposed:
//
//   dL/df_i(x) = mu_i(x) + A^a(x) + b(x) . c_i,   A^a = a^a + r^a,
//   r^a(x)     = sum_i w_i c_i . Sbar^a(x - c_i)   (transpose of the Eq. 7 sum),
//
// with mu_i = (1 - w) lam_i(x) (BGK) or c_i c_i : Pbar(x) (regularized), a, b
// and Sbar from the cell-local transpose (adjoint_cell.h).  The pull
// f_i(x) = X_i(x - c_i) is transposed by pushing dL/df_i(x) to lam_t at
// (x - c_i, i), or to (x, opp(i)) when x - c_i is a wall cell: every element
// of lam_t has exactly one such source, so the stores need no atomics, and
// lam_{t+1} is read only at the cell itself.
//
// The dependencies reach two cells: r at x needs Sbar at x - c_i, Sbar needs
// the force S at that cell, which needs rho one cell further.  A workgroup
// owns a BXT x ROWS tile and marches up a chunk of z planes with three stages
// one plane apart, one barrier per plane:
//
//   A  plane p:   pull X_t at the tile and a two-cell border; rho^A, rho^B
//                 into the density ring (4 slots of float2), u kept in
//                 registers;
//   B  plane p-1: the force from the ring, then the local transpose for the
//                 tile (a, b, Sbar, dL/dG, dL/dtau) and for its one-cell
//                 border (Sbar only); Sbar into the Sbar ring (4 slots);
//   C  plane p-3: r from the Sbar ring, dL/df of the tile's cells and the
//                 38 pushed stores (plus sum_i w_i dL/df_i when asked).
//
// "Own" waves carry the tile's cells through A, B and C; "halo" waves pull the
// border cells (stage A) and transpose the one-cell border (stage B).  Ragged
// lanes (past nx or ny) compute the wrapped cell so that the rings hold the
// right values, but store nothing.

#include "adjoint_cell.h"
#include "pull.h"

namespace lbm {

namespace {

template <int BXT, int ROWS, int HW>
struct AdjShape {
  static constexpr int NOWN = BXT * ROWS;
  static constexpr int HL = 64 * HW;                   // halo lanes
  static constexpr int NT = NOWN + HL;
  static constexpr int EX1 = BXT + 2, EY1 = ROWS + 2;  // Sbar ring plane: one-cell border
  static constexpr int EX2 = BXT + 4, EY2 = ROWS + 4;  // density ring plane: two-cell border
  static constexpr int P1 = EX1 * EY1, P2 = EX2 * EY2;
  static constexpr int NB1 = 2 * EX1 + 2 * ROWS;       // cells of the one-cell border
  static constexpr int NB2 = NB1 + 2 * EX2 + 2 * EY1;  // plus those of the second ring
  static constexpr int HPL = (NB2 + HL - 1) / HL;      // border cells per halo lane
  static constexpr int SLOTS = 4;
  static_assert(NOWN % 64 == 0, "own lanes fill whole waves");
  static_assert(NB1 <= HL, "each one-cell border cell is the first cell of one halo lane");
};

// Offset (hx, hy) from the tile origin of border cell h: the one-cell ring
// first (row below, row above, left column, right column), then the second
// ring in the same order.
template <int BXT, int ROWS>
__device__ __forceinline__ void border_pos(int h, int& hx, int& hy) {
  constexpr int EX1 = BXT + 2, EX2 = BXT + 4;
  constexpr int NB1 = 2 * EX1 + 2 * ROWS;
  if (h < NB1) {
    if (h < EX1) { hx = h - 1; hy = -1; }
    else if (h < 2 * EX1) { hx = h - EX1 - 1; hy = ROWS; }
    else if (h < 2 * EX1 + ROWS) { hx = -1; hy = h - 2 * EX1; }
    else { hx = BXT; hy = h - 2 * EX1 - ROWS; }
  } else {
    const int k = h - NB1;
    if (k < EX2) { hx = k - 2; hy = -2; }
    else if (k < 2 * EX2) { hx = k - EX2 - 2; hy = ROWS + 1; }
    else if (k < 2 * EX2 + ROWS + 2) { hx = -2; hy = k - 2 * EX2 - 1; }
    else { hx = BXT + 1; hy = k - 2 * EX2 - (ROWS + 2) - 1; }
  }
}

// Forward quantities of a cell from the density ring: S (Eq. 7) from the
// three planes around it, then rho, u and g (Local).
template <int EX2>
__device__ __forceinline__ void local_from_ring(const float2* rm, const float2* r0, const float2* rp, int at,
                                                const float u[3], const Phys& ph, Local& L) {
  float S[2][3];
  shan_chen_partial<EX2, 2>(rm, r0, at, S);
  shan_chen_finish<EX2, 2>(rp, at, S);
  const float2 rho = r0[at];
  make_local(rho.x, rho.y, u, S, ph, L);
}

// rho^a and the mixture velocity (Eqs. 4-6) of one cell, pulled from X_t.
template <bool WALLS>
__device__ __forceinline__ void pull_moments(const __amdgpu_buffer_rsrc_t rz[3], uint32_t ppb, const Column& col,
                                             uint32_t links, float rho[2], float u[3]) {
  const float ws[2][3] = {{0.f, 0.f, 0.f}, {0.f, 0.f, 0.f}};
  float f[2][Q], d[2];
  pull<Storage::F32, WALLS>(rz, ppb, col, links, ws, f, d);
  rho[0] = d[0];
  rho[1] = d[1];
  mixture_velocity(f, d[0] + d[1], u);
}

// Store of lambda_t, without the non-temporal hint of the forward step's
// stores: the reverse step writes to the cells its pull read from (one cell
// off in x, y or z), so neighbouring lanes and tiles write a population row
// in pieces, which merge into whole lines in the L2 before they reach HBM.
// With the hint the reverse step wrote 1.21x its algorithmic bytes (1.02x
// without) and was 9-14% slower at 96^3-192^3.
__device__ __forceinline__ void lam_store(float v, __amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, voff, soff, 0);
}

// The same quantities from the fields a forward step wrote (Mode::StepFields):
// bitwise what pull_moments gives for the cell.
__device__ __forceinline__ void read_fields(const float* __restrict__ fields, uint32_t c, uint64_t n, float2& r,
                                            float u[3]) {
  r = make_float2(fields[c], fields[n + c]);
  u[0] = fields[2 * n + c];
  u[1] = fields[3 * n + c];
  u[2] = fields[4 * n + c];
}

template <bool WALLS, int REG, bool FIELDS, int BXT, int ROWS, int HW>
__global__ void __launch_bounds__(BXT * ROWS + 64 * HW)
adjoint_march_kernel(const Grid g, const Phys ph, const Tiling tl, const AdjointIO io) {
  using Sh = AdjShape<BXT, ROWS, HW>;
  constexpr int EX1 = Sh::EX1, EX2 = Sh::EX2, P1 = Sh::P1, P2 = Sh::P2, SL = Sh::SLOTS;
  __shared__ float2 rring[SL * P2];      // rho~^A, rho~^B (wall cells: rho_s)
  __shared__ float sring[SL * 6 * P1];   // Sbar^A xyz, Sbar^B xyz: six planes per slot
  __shared__ double red[(Sh::NT / 64) * 3];
  // BGK keeps (1 - w) lam_{t+1} of each own cell from stage B to stage C (two
  // planes later) in LDS, one lane's values for its own use only, two plane
  // slots; read again from memory at stage C they mostly missed the L2.  The
  // 512-cell tiles do not have the LDS for it and read them again.
  constexpr bool STASH = REG == 0 && Sh::NOWN <= 256;
  __shared__ float stash[STASH ? 2 * 2 * Q * Sh::NOWN : 1];

  const int tid = threadIdx.x;
  // Link words of the wall classes (buffer.h).
  __shared__ uint32_t ltab[WALLS ? WALL_CLASSES : 1];
  if constexpr (WALLS) load_wall_classes(io.cls, io.ltab, ltab, tid, Sh::NT);
  const int b = xcd_remap(blockIdx.x, gridDim.x);
  // Block order of the tiling (launch.h): with walls every chunk of a run of
  // tiles per XCD (the work of a chunk depends on the geometry).
  const TileCoord tc = tile_of_block(b, tl);
  const int bxx = tc.x, byy = tc.y, bz = tc.z;
  const int x0 = bxx * BXT, y0 = byy * ROWS, z0 = bz * tl.zchunk;
  const int zc = min(z0 + tl.zchunk, g.nz) - z0;  // planes z0 .. z0 + zc - 1 are stored
  // Iteration k: A on plane z0 - 2 + k (k <= zc + 3), B on plane z0 - 3 + k
  // (2 <= k <= zc + 3), C on plane z0 - 5 + k (5 <= k <= zc + 4).
  const int kend = zc + 4;
  const uint32_t ppb = g.pstride * 4u;  // bytes between population rows
  const uint32_t n = static_cast<uint32_t>(g.n);

  double acc[3] = {0.0, 0.0, 0.0};

  if (tid < Sh::NOWN) {
    // ------------------------------------------------------------ own waves
    const int tx = tid % BXT, ty = tid / BXT;
    const int ex = x0 + tx, ey = y0 + ty;
    const bool owner = ex < g.nx && ey < g.ny;
    const Column col = make_column<float>(ex, ey, g);
    const uint32_t col_b = col.y[1] + col.x[1];
    const int at2 = (ty + 2) * EX2 + tx + 2;
    const int at1 = (ty + 1) * EX1 + tx + 1;

    // per plane in flight: links and u from A (used by B one plane later);
    // a, b (and Pbar) from B (used by C two planes later).
    uint32_t lk_a = 0u, lk_b = 0u, lk_c1 = 0u, lk_c2 = 0u;
    float u_a[3] = {0.f, 0.f, 0.f}, u_b[3] = {0.f, 0.f, 0.f};
    constexpr int NM = REG == 2 ? 23 : (REG ? 17 : 5);  // a^A, a^B, b xyz (+ Pbar^A, Pbar^B (+ qb^A, qb^B))
    // At the top of iteration k: m1 holds B's values of plane z0 - 4 + k,
    // m2 those of plane z0 - 5 + k (the plane of stage C).
    float m1[NM], m2[NM];
#pragma unroll
    for (int c = 0; c < NM; ++c) m1[c] = m2[c] = 0.f;

    for (int k = 0; k <= kend; ++k) {
      // ---- A: pull plane z0 - 2 + k
      if (k <= zc + 3) {
        const int p = z0 - 2 + k;
        const int zw = wrap(p, g.nz);
        lk_a = WALLS ? cell_links(io.cls, ltab, io.links, static_cast<uint32_t>(zw) * g.nxy + col.cell) : 0u;
        float2 r = make_float2(ph.rho_wall[0], ph.rho_wall[1]);
        if (!(WALLS && (lk_a & 1u))) {
          if constexpr (FIELDS) {
            read_fields(io.fields, static_cast<uint32_t>(zw) * g.nxy + col.cell, g.n, r, u_a);
          } else {
            __amdgpu_buffer_rsrc_t rz[3];
            rz[0] = plane_rsrc<float>(io.x_t, wrap(p - 1, g.nz), g);
            rz[1] = plane_rsrc<float>(io.x_t, zw, g);
            rz[2] = plane_rsrc<float>(io.x_t, wrap(p + 1, g.nz), g);
            float rho[2];
            pull_moments<WALLS>(rz, ppb, col, lk_a, rho, u_a);
            r = make_float2(rho[0], rho[1]);
          }
        }
        rring[(k % SL) * P2 + at2] = r;
      }
      __syncthreads();

      // BGK: stage B's loads for species A (lam_{t+1} and f of plane
      // z0 - 3 + k) go out before C, so that C's work overlaps them (species
      // B's follow in B: holding both would not fit the register budget).
      // Measured at 96^3 with the forward fields: 0.141 -> 0.132 ms.  The
      // regularized transpose has no registers to spare for it.
      constexpr bool PRE = REG == 0;
      float pre_lam[Q], pre_f[Q];
      if (PRE && k >= 2 && k <= zc + 3 && !(WALLS && (lk_b & 1u))) {
        const int zq = wrap(z0 - 3 + k, g.nz);
        const __amdgpu_buffer_rsrc_t rl = plane_rsrc<float>(io.lam_in, zq, g);
        __amdgpu_buffer_rsrc_t rc[3];
        rc[0] = plane_rsrc<float>(io.x_t, wrap(zq - 1, g.nz), g);
        rc[1] = plane_rsrc<float>(io.x_t, zq, g);
        rc[2] = plane_rsrc<float>(io.x_t, wrap(zq + 1, g.nz), g);
        const float ws0[3] = {0.f, 0.f, 0.f};
#pragma unroll
        for (int i = 0; i < Q; ++i) pre_lam[i] = buf_load<float>(rl, col_b, static_cast<uint32_t>(i) * ppb);
        pull_species<Storage::F32, WALLS>(rc, ppb, col, lk_b, ws0, 0, pre_f);
      }

      // ---- C: plane q3 = z0 - 5 + k (its Sbar neighbours are complete)
      if (k >= 5 && owner) {
        const int zq = wrap(z0 - 5 + k, g.nz);
        const uint32_t cell = static_cast<uint32_t>(zq) * g.nxy + col.cell;
        const bool solid = WALLS && (lk_c2 & 1u);
        __amdgpu_buffer_rsrc_t rd[3];
        rd[0] = plane_rsrc<float>(io.lam_out, wrap(zq - 1, g.nz), g);
        rd[1] = plane_rsrc<float>(io.lam_out, zq, g);
        rd[2] = plane_rsrc<float>(io.lam_out, wrap(zq + 1, g.nz), g);
        if (solid) {
          // no population lives here: zero this cell's own entries
#pragma unroll
          for (int i = 0; i < 2 * Q; ++i) lam_store(0.0f, rd[1], col_b, static_cast<uint32_t>(i) * ppb);
          if (io.drho0) {
            io.drho0[cell] = 0.0;
            io.drho0[static_cast<uint64_t>(n) + cell] = 0.0;
          }
        } else {
          // r^a = sum_i w_i c_i . Sbar^a(x - c_i); Sbar plane of x - c_i: z - c_z
          float r[2] = {0.f, 0.f};
#pragma unroll
          for (int i = 1; i < Q; ++i) {
            const int slot = (k - 3 - CZ[i] + SL) % SL;  // plane z0 - 5 + k - c_z was B's in iteration k - 2 - c_z
            const float* sp = sring + slot * 6 * P1 + at1 - CY[i] * EX1 - CX[i];
#pragma unroll
            for (int s = 0; s < 2; ++s) {
              float dot = 0.0f;
              if (CX[i]) dot += CX[i] * sp[(3 * s + 0) * P1];
              if (CY[i]) dot += CY[i] * sp[(3 * s + 1) * P1];
              if (CZ[i]) dot += CZ[i] * sp[(3 * s + 2) * P1];
              r[s] = fmaf(weight(i), dot, r[s]);
            }
          }
          const __amdgpu_buffer_rsrc_t rl = plane_rsrc<float>(io.lam_in, zq, g);
#pragma unroll
          for (int s = 0; s < 2; ++s) {
            const float A = m2[s] + r[s];
            const float keep = 1.0f - ph.omega[s];
            float dw = 0.0f;  // sum_i w_i dL/df_i
#pragma unroll
            for (int i = 0; i < Q; ++i) {
              float mu;
              if constexpr (REG != 0) {
                mu = i == 0 ? 0.0f : pair_quad((i - 1) >> 1, &m2[5 + 6 * s]);
                if constexpr (REG == 2) {
                  if (i != 0) {
                    const float hq = pair_hq((i - 1) >> 1, &m2[17 + 3 * s]);
                    mu += (i & 1) ? hq : -hq;
                  }
                }
              } else if constexpr (STASH) {
                mu = stash[(((k - 1) & 1) * 2 * Q + s * Q + i) * Sh::NOWN + tid];  // slot of plane z0 - 5 + k
              } else {
                mu = keep * buf_load<float>(rl, col_b, static_cast<uint32_t>(s * Q + i) * ppb);
              }
              float bc = 0.0f;
              if (CX[i]) bc += CX[i] * m2[2];
              if (CY[i]) bc += CY[i] * m2[3];
              if (CZ[i]) bc += CZ[i] * m2[4];
              const float v = (mu + A) + bc;
              dw = fmaf(weight(i), v, dw);
              if (WALLS && i != 0 && ((lk_c2 >> i) & 1u)) {
                // x - c_i is a wall: the pull read X_opp(i)(x) for f_i(x)
                lam_store(v, rd[1], col_b, static_cast<uint32_t>(s * Q + opp(i)) * ppb);
              } else {
                const uint32_t off = col.y[1 - CY[i]] + col.x[1 - CX[i]];
                lam_store(v, rd[1 - CZ[i]], off, static_cast<uint32_t>(s * Q + i) * ppb);
              }
            }
            if (io.drho0) io.drho0[static_cast<uint64_t>(s) * n + cell] = static_cast<double>(dw);
          }
        }
      }

      // ---- B: plane q = z0 - 3 + k (density planes q - 1 .. q + 1 are complete)
      if (k >= 2 && k <= zc + 3) {
        const int zq = wrap(z0 - 3 + k, g.nz);
        float sb[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        float mo[NM];
#pragma unroll
        for (int c = 0; c < NM; ++c) mo[c] = 0.f;
        if (!(WALLS && (lk_b & 1u))) {
          Local L;
          local_from_ring<EX2>(rring + ((k - 2) % SL) * P2, rring + ((k - 1) % SL) * P2, rring + (k % SL) * P2, at2,
                               u_b, ph, L);
          // lam_{t+1} at the cell and f of species B (species A came before C)
          const __amdgpu_buffer_rsrc_t rl = plane_rsrc<float>(io.lam_in, zq, g);
          __amdgpu_buffer_rsrc_t rc[3];
          rc[0] = plane_rsrc<float>(io.x_t, wrap(zq - 1, g.nz), g);
          rc[1] = plane_rsrc<float>(io.x_t, zq, g);
          rc[2] = plane_rsrc<float>(io.x_t, wrap(zq + 1, g.nz), g);
          const float ws0[3] = {0.f, 0.f, 0.f};
          AdjointSums S;
#pragma unroll
          for (int c = 0; c < 3; ++c) S.ubar[c] = 0.0f;
          float pb[2][6], qe[2][3];
#pragma unroll
          for (int s = 0; s < 2; ++s) {
            float lam[Q], fs[Q];
            if (PRE && s == 0) {
#pragma unroll
              for (int i = 0; i < Q; ++i) {
                lam[i] = pre_lam[i];
                fs[i] = pre_f[i];
              }
            } else {
#pragma unroll
              for (int i = 0; i < Q; ++i) lam[i] = buf_load<float>(rl, col_b, static_cast<uint32_t>(s * Q + i) * ppb);
              pull_species<Storage::F32, WALLS>(rc, ppb, col, lk_b, ws0, s, fs);
            }
            if constexpr (REG != 0) {
              adjoint_species<true>(s, 0.0f, lam, L, ph, S);
              adjoint_species_reg(s, lam, fs, L, ph, S, pb[s]);
              if constexpr (REG == 2) adjoint_species_energy(s, lam, fs, L, ph, S, qe[s]);
            } else {
              float dot = lam[0] * fs[0];
#pragma unroll
              for (int i = 1; i < Q; ++i) dot = fmaf(lam[i], fs[i], dot);
              adjoint_species(s, dot, lam, L, ph, S);
              if constexpr (STASH) {
                // plane z0 - 3 + k: its slot, (k - 1) & 1, last held plane
                // z0 - 5 + k, which stage C of this iteration has read
                const float keep = 1.0f - ph.omega[s];
#pragma unroll
                for (int i = 0; i < Q; ++i) stash[(((k - 1) & 1) * 2 * Q + s * Q + i) * Sh::NOWN + tid] = keep * lam[i];
              }
            }
            __builtin_amdgcn_sched_barrier(0);  // keep the next species' loads below this one's arithmetic
          }
          double a3[3] = {0.0, 0.0, 0.0};
          adjoint_finish(S, L, ph, mo, sb, a3);
          // parameter sums over the chunk's own planes (B also visits the
          // plane on either side of the chunk, which other chunks own)
          if (owner && k >= 3 && k <= zc + 2) {
            acc[0] += a3[0];
            acc[1] += a3[1];
            acc[2] += a3[2];
          }
          if constexpr (REG != 0) {
#pragma unroll
            for (int c = 0; c < 6; ++c) {
              mo[5 + c] = pb[0][c];
              mo[11 + c] = pb[1][c];
            }
          }
          if constexpr (REG == 2) {
#pragma unroll
            for (int c = 0; c < 3; ++c) {
              mo[17 + c] = qe[0][c];
              mo[20 + c] = qe[1][c];
            }
          }
        }
        float* sl = sring + ((k - 1) % SL) * 6 * P1 + at1;
#pragma unroll
        for (int c = 0; c < 6; ++c) sl[c * P1] = sb[c];
#pragma unroll
        for (int c = 0; c < NM; ++c) {
          m2[c] = m1[c];
          m1[c] = mo[c];
        }
      }
      lk_c2 = lk_c1;
      lk_c1 = lk_b;
      lk_b = lk_a;
#pragma unroll
      for (int c = 0; c < 3; ++c) u_b[c] = u_a[c];
    }
  } else {
    // ----------------------------------------------------------- halo waves
    const int hl = tid - Sh::NOWN;
    Column hcol[Sh::HPL];
    int hat2[Sh::HPL];
    bool has[Sh::HPL];
#pragma unroll
    for (int j = 0; j < Sh::HPL; ++j) {
      const int h = hl + j * Sh::HL;
      has[j] = h < Sh::NB2;
      int hx = 0, hy = 0;
      border_pos<BXT, ROWS>(has[j] ? h : 0, hx, hy);
      hcol[j] = make_column<float>(x0 + hx, y0 + hy, g);
      hat2[j] = (hy + 2) * EX2 + hx + 2;
    }
    // the lane's first cell lies on the one-cell border when hl < NB1
    const bool ring1 = hl < Sh::NB1;
    int hx1 = 0, hy1 = 0;
    border_pos<BXT, ROWS>(ring1 ? hl : 0, hx1, hy1);
    const int hat1 = (hy1 + 1) * EX1 + hx1 + 1;
    const uint32_t hcol_b = hcol[0].y[1] + hcol[0].x[1];
    uint32_t lk_a = 0u, lk_b = 0u;
    float u_a[3] = {0.f, 0.f, 0.f}, u_b[3] = {0.f, 0.f, 0.f};

    for (int k = 0; k <= kend; ++k) {
      if (k <= zc + 3) {
        const int p = z0 - 2 + k;
        const int zw = wrap(p, g.nz);
        __amdgpu_buffer_rsrc_t rz[3];
        rz[0] = plane_rsrc<float>(io.x_t, wrap(p - 1, g.nz), g);
        rz[1] = plane_rsrc<float>(io.x_t, zw, g);
        rz[2] = plane_rsrc<float>(io.x_t, wrap(p + 1, g.nz), g);
#pragma unroll
        for (int j = 0; j < Sh::HPL; ++j) {
          if (!has[j]) continue;
          const uint32_t lk = WALLS ? cell_links(io.cls, ltab, io.links, static_cast<uint32_t>(zw) * g.nxy + hcol[j].cell) : 0u;
          float2 r = make_float2(ph.rho_wall[0], ph.rho_wall[1]);
          float uu[3] = {0.f, 0.f, 0.f};
          if (!(WALLS && (lk & 1u))) {
            if constexpr (FIELDS) {
              read_fields(io.fields, static_cast<uint32_t>(zw) * g.nxy + hcol[j].cell, g.n, r, uu);
            } else {
              float rho[2];
              pull_moments<WALLS>(rz, ppb, hcol[j], lk, rho, uu);
              r = make_float2(rho[0], rho[1]);
            }
          }
          rring[(k % SL) * P2 + hat2[j]] = r;
          if (j == 0) {
            lk_a = lk;
#pragma unroll
            for (int c = 0; c < 3; ++c) u_a[c] = uu[c];
          }
        }
      }
      __syncthreads();
      // B on the one-cell border: Sbar only (gbar needs the E(rho, v) part alone)
      if (k >= 2 && k <= zc + 3 && ring1) {
        const int zq = wrap(z0 - 3 + k, g.nz);
        float sb[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        if (!(WALLS && (lk_b & 1u))) {
          Local L;
          const int at2 = (hy1 + 2) * EX2 + hx1 + 2;
          local_from_ring<EX2>(rring + ((k - 2) % SL) * P2, rring + ((k - 1) % SL) * P2, rring + (k % SL) * P2,
                               at2, u_b, ph, L);
          const __amdgpu_buffer_rsrc_t rl = plane_rsrc<float>(io.lam_in, zq, g);
          AdjointSums S;
#pragma unroll
          for (int c = 0; c < 3; ++c) S.ubar[c] = 0.0f;
#pragma unroll
          for (int s = 0; s < 2; ++s) {
            float lam[Q];
#pragma unroll
            for (int i = 0; i < Q; ++i) lam[i] = buf_load<float>(rl, hcol_b, static_cast<uint32_t>(s * Q + i) * ppb);
            adjoint_species<true>(s, 0.0f, lam, L, ph, S);
          }
#pragma unroll
          for (int a = 0; a < 3; ++a) {
            sb[a] = ph.g_ba * S.gbar[1][a];
            sb[3 + a] = ph.g_ab * S.gbar[0][a];
          }
        }
        float* sl = sring + ((k - 1) % SL) * 6 * P1 + hat1;
#pragma unroll
        for (int c = 0; c < 6; ++c) sl[c * P1] = sb[c];
      }
      lk_b = lk_a;
#pragma unroll
      for (int c = 0; c < 3; ++c) u_b[c] = u_a[c];
    }
  }

  bool is_max[3] = {false, false, false};
  __syncthreads();
  block_reduce_store<3>(acc, is_max, io.partials + static_cast<uint64_t>(blockIdx.x) * 3, red);
}

struct AdjTile {
  int bx, rows, hw;
};
constexpr AdjTile ADJ_TILES[ADJOINT_SHAPES] = {{64, 8, 3}, {32, 16, 2}, {32, 8, 2}, {64, 4, 3}};

template <bool WALLS, int REG, bool FIELDS, int BXT, int ROWS, int HW>
hipError_t launch_shape(const Grid& g, const Phys& ph, const Tiling& t, const AdjointIO& io, hipStream_t st) {
  using Sh = AdjShape<BXT, ROWS, HW>;
  hipLaunchKernelGGL((adjoint_march_kernel<WALLS, REG, FIELDS, BXT, ROWS, HW>), dim3(t.blocks), dim3(Sh::NT), 0, st,
                     g, ph, t, io);
  return hipGetLastError();
}

template <bool WALLS, int REG, bool FIELDS>
hipError_t launch_shapes(const Grid& g, const Phys& ph, const Tiling& t, const AdjointIO& io, hipStream_t st) {
  switch (t.tile) {
    case 0: return launch_shape<WALLS, REG, FIELDS, 64, 8, 3>(g, ph, t, io, st);
    case 1: return launch_shape<WALLS, REG, FIELDS, 32, 16, 2>(g, ph, t, io, st);
    case 2: return launch_shape<WALLS, REG, FIELDS, 32, 8, 2>(g, ph, t, io, st);
    case 3: return launch_shape<WALLS, REG, FIELDS, 64, 4, 3>(g, ph, t, io, st);
    default: return hipErrorInvalidValue;
  }
}

template <bool WALLS, int REG>
hipError_t launch_variant(const Grid& g, const Phys& ph, const Tiling& t, const AdjointIO& io, hipStream_t st) {
  return io.fields ? launch_shapes<WALLS, REG, true>(g, ph, t, io, st) : launch_shapes<WALLS, REG, false>(g, ph, t, io, st);
}

}  // namespace

Tiling adjoint_march_tiling(const Grid& g, int shape, int zchunk) {
  Tiling t{};
  t.order = ORDER_PLANE_X;
  t.xoff = 0;
  if (shape < 0 || shape >= ADJOINT_SHAPES) {
    t.blocks = -1;
    return t;
  }
  const AdjTile sh = ADJ_TILES[shape];
  t.tile = shape;
  t.tiles_x = (g.nx + sh.bx - 1) / sh.bx;
  t.tiles_y = (g.ny + sh.rows - 1) / sh.rows;
  const long long txy = static_cast<long long>(t.tiles_x) * t.tiles_y;
  if (zchunk <= 0) {
    // One workgroup per CU (its two rings take 50-90 KB of LDS): the
    // launch runs in ceil(blocks / 256) rounds of zchunk + 5 plane
    // iterations each (five fill and drain the three stages).  Take the
    // chunk of 4 to 256 planes (or nz) that minimises rounds x iterations.
    const int lo = g.nz < 4 ? g.nz : 4;
    const int hi = g.nz < 256 ? g.nz : 256;
    long long best_cost = -1;
    zchunk = hi;
    for (int z = lo; z <= hi; ++z) {
      const long long chunks = (g.nz + z - 1) / z;
      const long long rounds = (txy * chunks + 255) / 256;
      const long long cost = rounds * (z + 5);
      if (best_cost < 0 || cost < best_cost) {
        best_cost = cost;
        zchunk = z;
      }
    }
  }
  if (zchunk > g.nz) zchunk = g.nz;
  t.zchunk = zchunk;
  t.tiles_z = (g.nz + zchunk - 1) / zchunk;
  const long long nb = txy * t.tiles_z;
  t.blocks = nb > 0x7fffffffLL ? -1 : static_cast<int>(nb);
  return t;
}

int adjoint_auto_shape(const Grid& g, bool walls, int collision) {
  // The 256-cell tiles (32 x 8 and 64 x 4: six and seven waves, about 220
  // registers without spills, and the LDS to keep lam for BGK) measured
  // fastest; the 512-cell tiles spill with walls or the regularized
  // transpose.  The one that pads the x-y plane less, 64 x 4 on a tie: its
  // rows are two 128-byte lines wide (BGK reverse step 4% faster at 128^3
  // and 192^3, 16% at 256^3); at 96^3, where 64 x 4 pads x to 128, 32 x 8
  // is 17% faster.
  (void)walls;
  (void)collision;
  const int first = 3, second = 2;
  int best = first;
  long long best_cells = -1;
  for (int k : {first, second}) {
    const AdjTile sh = ADJ_TILES[k];
    const long long cells = static_cast<long long>((g.nx + sh.bx - 1) / sh.bx) * sh.bx *
                            (static_cast<long long>((g.ny + sh.rows - 1) / sh.rows) * sh.rows);
    if (best_cells < 0 || cells < best_cells) {
      best_cells = cells;
      best = k;
    }
  }
  return best;
}

hipError_t launch_adjoint_march(const Grid& g, const Phys& ph, const Tiling& t, const AdjointIO& io,
                                hipStream_t st) {
  if (t.blocks <= 0 || !io.x_t || !io.lam_in || !io.lam_out || !io.partials) return hipErrorInvalidValue;
  // ph.regularized: 0 BGK, 1 second-order, 2 third-order reading of the filter
  switch (ph.regularized + (io.links ? 3 : 0)) {
    case 0: return launch_variant<false, 0>(g, ph, t, io, st);
    case 1: return launch_variant<false, 1>(g, ph, t, io, st);
    case 2: return launch_variant<false, 2>(g, ph, t, io, st);
    case 3: return launch_variant<true, 0>(g, ph, t, io, st);
    case 4: return launch_variant<true, 1>(g, ph, t, io, st);
    case 5: return launch_variant<true, 2>(g, ph, t, io, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace lbm
