// Host-side launchers of the device kernels (C++ linkage, internal to liblbm).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lattice.h"

namespace lbm {

// Per-launch description of the grid and the physics, shared by every kernel.
// The stored state of one z plane is a sequence of row blocks of `brows` y
// rows each; a row block holds, population after population, the rows of
// all 38 populations (pstride elements apart), and in the 16-bit forms two
// residual rows (Layout).  Element (a, i, x, y, z) sits at z * zstride +
// (y / brows) * 38 * pstride + (a * 19 + i) * pstride + (y % brows) * nx +
// pos(x); FP32 blocks hold 38 rows, while the 16-bit forms have one block per
// plane (brows = ny), so the block stride never applies to them.
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

// Rows of one row block: the 38 population rows, and for the 16-bit forms
// two more (row 38 + a): the residual of species a's rest population, the
// rounding error of its stored value, itself stored in the same 16-bit form
// (see encode_species).  Row r of a block starts r * pstride elements in.
constexpr int POP_ROWS = 2 * Q;
constexpr int RES_ROW = 2 * Q;
__host__ __device__ constexpr int block_rows(int elem_bytes) { return elem_bytes == 4 ? POP_ROWS : POP_ROWS + 2; }
Layout state_layout(int nx, int ny, int elem_bytes);

struct Phys {
  float omega[2];     // 1 / tau_a
  float g_ab, g_ba;   // G^{AB}, G^{BA}
  float rho_wall[2];  // rho_s^a
  float shift[2];     // rho_shift^a of the 16-bit storage forms (0 for FP32)
  int regularized;    // collision operator: 0 = BGK (Eq. 2); regularized (Eqs. 10-11) with the
                      // momentum flux (1) or the momentum and energy flux (2)
};

// Order of the workgroups over the (z chunk, tile) pairs.  The hardware
// hands consecutive workgroups to the 8 XCDs in turn; xcd_remap makes each
// XCD's share a contiguous range b0..b1 of the order, so the order decides
// which tiles share an XCD's L2 while they run: with PLANE orders an XCD
// takes whole rows (X: x fastest) or columns (Y: y fastest) of tiles of one
// z chunk, with TILE orders every chunk of a run of tiles.
enum BlockOrder : int { ORDER_PLANE_X = 1, ORDER_PLANE_Y = 2, ORDER_TILE_X = 3, ORDER_TILE_Y = 4 };
constexpr int BLOCK_ORDERS = 4;

struct Tiling {
  int tile;      // workgroup tile shape (index into the shapes of march.hip)
  int zchunk;    // z planes marched per workgroup
  int tiles_x, tiles_y, tiles_z;
  int blocks;
  int order;     // BlockOrder
  int xoff;      // x of the first tile's first column (the tile grid is shifted, wrapping in x)
};

struct TileCoord {
  int x, y, z;  // tile column, tile row, z chunk
};

__host__ __device__ inline TileCoord tile_of_block(int b, const Tiling& t) {
  const int txy = t.tiles_x * t.tiles_y;
  const bool chunk_fastest = t.order == ORDER_TILE_X || t.order == ORDER_TILE_Y;
  const int z = chunk_fastest ? b % t.tiles_z : b / txy;
  const int rem = chunk_fastest ? b / t.tiles_z : b - z * txy;
  if (t.order == ORDER_PLANE_Y || t.order == ORDER_TILE_Y) return {rem / t.tiles_y, rem % t.tiles_y, z};
  return {rem % t.tiles_x, rem / t.tiles_x, z};
}

// Tile shapes: 0 = 64x8, 1 = 64x12, 2 = 32x16, 3 = 128x4, 4 = 64x4, 5 = 256x2 cells
// (one cell per lane); 6 = 64x8, 7 = 32x16, 8 = 32x8, 9 = 32x12 words of a
// folded 16-bit row (two cells per lane; 16-bit storage, even nx, no walls).
constexpr int TILE_SHAPES = 10;
constexpr bool pair_shape(int tile) { return tile >= 6 && tile < TILE_SHAPES; }
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

// Step: one step.  Moments: diagnostics.  StepFields: one step that also
// writes, for every cell, rho^A, rho^B and u of the pull it collides (the
// forward quantities the reverse step needs at that time level; FP32).
enum class Mode : int { Step = 0, Moments = 1, StepFields = 2 };

// Entries of the wall class table (buffer.h).
constexpr int WALL_CLASSES = 256;

struct MarchIO {
  const void* src = nullptr;       // stored state X_t
  void* dst = nullptr;             // Step: X_{t+1}
  const uint32_t* links = nullptr; // wall link bits or null
  const uint8_t* cls = nullptr;    // wall class per cell, or null (buffer.h)
  const uint32_t* ltab = nullptr;  // link word of each class (WALL_CLASSES)
  float* rho_out = nullptr;        // Moments
  float* uf_out = nullptr;         // Moments
  double* partials = nullptr;      // Moments: 16 per block
  Region region{};
  float* fields = nullptr;         // StepFields: 5 N floats, rho^A, rho^B, u_x, u_y, u_z (cell order)
};

// One reverse step (adjoint_march.hip): lam_t = dL/dX_t from lam_{t+1} =
// dL/dX_{t+1} at the stored FP32 state X_t.
struct AdjointIO {
  const void* x_t = nullptr;        // stored state X_t (FP32, state layout)
  const uint32_t* links = nullptr;  // wall link bits or null
  const uint8_t* cls = nullptr;     // wall class per cell, or null (buffer.h)
  const uint32_t* ltab = nullptr;   // link word of each class (WALL_CLASSES)
  const float* lam_in = nullptr;    // lam_{t+1} (state layout)
  float* lam_out = nullptr;         // lam_t (state layout)
  double* partials = nullptr;       // 3 per block: dL/dG (tied), dL/dtau_A, dL/dtau_B
  double* drho0 = nullptr;          // 2 N, sum_i w_i dL/df_i^a, or null
  const float* fields = nullptr;    // rho^A, rho^B, u of X_t's pull (StepFields), or null: pull them
};

// Tile shapes of the reverse march: 0 = 64x8, 1 = 32x16, 2 = 32x8, 3 = 64x4
// cells.  zchunk <= 0 picks the default chunk.
constexpr int ADJOINT_SHAPES = 4;
Tiling adjoint_march_tiling(const Grid& g, int shape, int zchunk);
int adjoint_auto_shape(const Grid& g, bool walls, int collision);
hipError_t launch_adjoint_march(const Grid& g, const Phys& ph, const Tiling& t, const AdjointIO& io,
                                hipStream_t st);

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
// A 16-bit stored state (layout g) as an FP32 stored state (layout g32, the
// same lattice) of the populations its pull reads; 16-bit storage only.
hipError_t launch_widen_state(Storage s, const Grid& g, const Grid& g32, const Phys& ph, const uint32_t* links,
                              const void* src, float* dst, hipStream_t st);
// Sums the per-workgroup partials (blocks x nvals) into out[0..nvals); entry
// max_index (-1: none) takes the maximum instead of the sum.
hipError_t launch_finalize(const double* partials, int blocks, int nvals, int max_index, double* out,
                           bool accumulate, hipStream_t st);
hipError_t launch_stream_copy(const void* src, void* dst, uint64_t bytes, hipStream_t st);
hipError_t launch_march_copy(Storage s, const Grid& g, const void* src, void* dst, hipStream_t st);
hipError_t launch_adjoint_seed(const Grid& g, const uint32_t* links, const float* grad_rho,
                               float* lam, hipStream_t st);

}  // namespace lbm
