// Host-side launchers of the device kernels (C++ linkage, internal to liblbm).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lattice.h"

namespace lbm {

// Per-launch description of the grid and the physics, shared by every kernel.
// The stored state of one z plane is a sequence of row blocks of `brows` y
// rows each; a row block holds, population after population, the rows of
// all 38 populations (pstride elements apart).  Element (a, i, x, y, z) sits
// at z * zstride + (y / brows) * 38 * pstride + (a * 19 + i) * pstride +
// (y % brows) * nx + pos(x).
struct Grid {
  int nx, ny, nz;
  uint32_t nxy;      // nx * ny
  uint64_t n;        // nx * ny * nz
  uint32_t pstride;  // elements from one population's rows of a row block to the next
  uint32_t half;     // nx / 2 when rows of the 16-bit forms are folded (even nx), else 0
  uint32_t brows;    // y rows per row block
  uint32_t zstride;  // elements of one z plane: 38 * pstride * ceil(ny / brows)
};

// Layout of the stored state (and of the FP32 adjoint arrays) for a storage
// element size.  FP32 takes row blocks of 4 rows: the 38 population rows a
// workgroup of a few rows reads in one plane are then one contiguous range
// (measured 2-5% faster steps than whole population planes).  The 16-bit
// forms keep one block per plane (brows = ny): their paired march measured
// 1.5% slower on 4-row blocks.  pstride is brows * nx rounded up to 256
// bytes, plus 256 bytes when that is a multiple of 64 KiB (population blocks
// a large power of two apart put the rows a step reads together on the same
// DRAM channels: 4-5% of step time at 128^2 and 512^2 planes).
struct Layout {
  uint32_t brows;
  uint32_t pstride;
  uint64_t zstride;
};
Layout state_layout(int nx, int ny, int elem_bytes);

struct Phys {
  float omega[2];     // 1 / tau_a
  float g_ab, g_ba;   // G^{AB}, G^{BA}
  float rho_wall[2];  // rho_s^a
  float shift[2];     // rho_shift^a of the 16-bit storage forms (0 for FP32)
  int regularized;    // collision operator: 0 = BGK (Eq. 2), 1 = regularized (Eqs. 10-11)
};

struct Tiling {
  int tile;      // workgroup tile shape (index into the shapes of march.hip)
  int zchunk;    // z planes marched per workgroup
  int tiles_x, tiles_y, tiles_z;
  int blocks;
};

// Tile shapes: 0 = 64x8, 1 = 64x12, 2 = 32x16, 3 = 128x4, 4 = 64x4, 5 = 256x2 cells
// (one cell per lane); 6 = 64x8, 7 = 32x16, 8 = 32x8, 9 = 32x12 words of a
// folded 16-bit row (two cells per lane; 16-bit storage, even nx, no walls).
constexpr int TILE_SHAPES = 10;
constexpr bool pair_shape(int tile) { return tile >= 6 && tile < TILE_SHAPES; }
// Shapes the adjoint march is built for.
constexpr bool adjoint_shape(int tile) { return tile == 0 || tile == 2 || tile == 4; }
// zchunk <= 0 picks a default; open_box (a step without walls) takes the
// round-count rule of march.hip.
Tiling make_tiling(const Grid& g, int tile, int zchunk, bool open_box = false);
// Shape used when the caller asks for the automatic choice.
int auto_tile(const Grid& g, bool walls, int elem_bytes);

// Diagnostic region (device-side floats).
struct Region {
  float cx, cy, cz;
  float r_in2, r_out2, thr;
  float p_g;  // symmetric coupling used in the pressure
};

enum class Mode : int { Step = 0, Moments = 1, Adjoint = 2 };

struct MarchIO {
  const void* src = nullptr;       // stored state X_t
  void* dst = nullptr;             // Step: X_{t+1}
  const uint32_t* links = nullptr; // wall link bits or null
  float* rho_out = nullptr;        // Moments
  float* uf_out = nullptr;         // Moments
  double* partials = nullptr;      // Moments (16 per block) / Adjoint (3 per block)
  Region region{};
  const float* lam = nullptr;      // Adjoint: lam_{t+1}
  float* m = nullptr;              // Adjoint: 5 N  (a^A, a^B, b_x, b_y, b_z)
  float* sbar = nullptr;           // Adjoint: 6 N  (Sbar^A xyz, Sbar^B xyz)
  float* dbar = nullptr;           // Adjoint, regularized: per-pair direct term of dL/df (state layout)
};

hipError_t launch_march(Storage s, Mode mode, const Grid& g, const Phys& ph, const Tiling& t,
                        const MarchIO& io, hipStream_t st);
// Step of the 16-bit forms on folded rows (pair shapes 6..9, no walls).
hipError_t launch_pair_step(Storage s, const Grid& g, const Phys& ph, const Tiling& t, const MarchIO& io,
                            hipStream_t st);

hipError_t launch_init(Storage s, const Grid& g, const Phys& ph, const uint32_t* links,
                       const double* rho0, void* dst, hipStream_t st);
hipError_t launch_links(const Grid& g, const uint8_t* solid, uint32_t* links, hipStream_t st);
hipError_t launch_get_populations(Storage s, const Grid& g, const Phys& ph, const uint32_t* links,
                                  const void* src, float* f, hipStream_t st);
hipError_t launch_set_populations(Storage s, const Grid& g, const Phys& ph, const uint32_t* links,
                                  const float* f, void* dst, hipStream_t st);
// Sums the per-workgroup partials (blocks x nvals) into out[0..nvals); entry
// max_index (-1: none) takes the maximum instead of the sum.
hipError_t launch_finalize(const double* partials, int blocks, int nvals, int max_index, double* out,
                           bool accumulate, hipStream_t st);
hipError_t launch_adjoint_gather(const Grid& g, const uint32_t* links, float* m, const float* sbar,
                                 hipStream_t st);
// pairs: lam_in holds the regularized collision's per-pair direct term (see
// adjoint.hip) instead of lam_{t+1}.
hipError_t launch_adjoint_stream(const Grid& g, const Phys& ph, const uint32_t* links,
                                 const float* lam_in, const float* m, float* lam_out,
                                 double* drho0, bool pairs, hipStream_t st);
hipError_t launch_stream_copy(const void* src, void* dst, uint64_t bytes, hipStream_t st);
hipError_t launch_march_copy(Storage s, const Grid& g, const void* src, void* dst, hipStream_t st);
hipError_t launch_adjoint_seed(const Grid& g, const uint32_t* links, const float* grad_rho,
                               float* lam, hipStream_t st);

}  // namespace lbm
