// Addressing helpers shared by the z-marching kernels: XCD-aware block
// order, periodic wrap, per-column byte offsets and buffer resources over one
// z plane of the row-blocked population layout (Grid).
#pragma once

#include "launch.h"

namespace lbm {

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

// Position of cell x inside a stored row.  The 16-bit forms with even nx
// fold each row: the 32-bit word k holds cells k and k + nx/2 (x < nx/2 at
// element 2x, x >= nx/2 at element 2(x - nx/2) + 1), so that one aligned
// 32-bit load brings two cells whose x neighbours sit in the neighbouring
// words.  FP32 rows and odd nx are stored in x order.
template <typename T>
__device__ __forceinline__ uint32_t row_pos(int gx, const Grid& g) {
  if constexpr (sizeof(T) == 2) {
    if (g.half) {
      const uint32_t x = static_cast<uint32_t>(gx);
      return x < g.half ? 2u * x : 2u * (x - g.half) + 1u;
    }
  }
  return static_cast<uint32_t>(gx);
}

// Element offset of row y inside one z plane, population (0, 0); the other
// populations of the row are pstride elements apart.  One division per
// column, outside the z march.
__device__ __forceinline__ uint32_t row_off(int y, const Grid& g) {
  const uint32_t yy = static_cast<uint32_t>(y);
  const uint32_t q = yy / g.brows;
  return q * (2u * Q) * g.pstride + (yy - q * g.brows) * static_cast<uint32_t>(g.nx);
}

// Wrapped coordinates of one cell column (x, y) and of its x/y neighbours,
// as BYTE offsets inside one z plane (population (0, 0)), and the column's
// cell index y * nx + x.
struct Column {
  uint32_t x[3];  // row positions of (x-1, x, x+1), times sizeof(T)
  uint32_t y[3];  // ((y-1), y, (y+1)) * nx * sizeof(T)
  uint32_t cell;  // y * nx + x
};

template <typename T>
__device__ __forceinline__ Column make_column(int ex, int ey, const Grid& g) {
  const int gx = wrap(ex, g.nx), gy = wrap(ey, g.ny);
  const uint32_t sz = sizeof(T);
  Column c;
  c.x[0] = row_pos<T>(gx == 0 ? g.nx - 1 : gx - 1, g) * sz;
  c.x[1] = row_pos<T>(gx, g) * sz;
  c.x[2] = row_pos<T>(gx == g.nx - 1 ? 0 : gx + 1, g) * sz;
  const int ym = gy == 0 ? g.ny - 1 : gy - 1;
  const int yp = gy == g.ny - 1 ? 0 : gy + 1;
  c.y[0] = row_off(ym, g) * sz;
  c.y[1] = row_off(gy, g) * sz;
  c.y[2] = row_off(yp, g) * sz;
  c.cell = static_cast<uint32_t>(gy) * g.nx + static_cast<uint32_t>(gx);
  return c;
}

// Buffer resource over z plane `zw` of a state (g.zstride elements).
// Out-of-range offsets read as zero instead of faulting.
constexpr int RSRC_FLAGS = 0x00020000;  // 32-bit data format, gfx9 family

template <typename T>
__device__ __forceinline__ __amdgpu_buffer_rsrc_t plane_rsrc(const void* buf, int zw, const Grid& g) {
  const uint64_t block = static_cast<uint64_t>(g.zstride) * sizeof(T);
  const char* base = static_cast<const char*>(buf) + static_cast<uint64_t>(zw) * block;
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<char*>(base), static_cast<short>(0),
                                           static_cast<int>(block), RSRC_FLAGS);
}

template <typename T, int AUX = 0>
__device__ __forceinline__ T buf_load(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
  if constexpr (sizeof(T) == 4) {
    return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, AUX));
  } else {
    return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b16(r, voff, soff, AUX));
  }
}

// Cache-policy bits of the bounce-back loads (sc0).  A load whose resource or
// scalar offset depends on a per-lane condition would need a loop over the
// distinct values; with a different policy than the ordinary pull, the two
// loads of a population stay separate instructions under a lane mask.
constexpr int LOAD_BOUNCE = 1;

// Stores carry the non-temporal hint: the new state is not read again in this
// step, so it should not displace the lines neighbouring workgroups still
// need for their halo.
constexpr int STORE_NT = 2;

template <typename T>
__device__ __forceinline__ void buf_store(T v, __amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
  if constexpr (sizeof(T) == 4) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, voff, soff, STORE_NT);
  } else {
    __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(unsigned short, v), r, voff, soff, STORE_NT);
  }
}

// Wall links (one 32-bit word per cell): bit i set when x - c_i is a wall
// cell, bit 0 when x itself is.  When the geometry's fluid cells show at
// most WALL_CLASSES distinct words, every cell also has a one-byte class,
// the index of its word in a table of those words (a wall cell takes the
// class of the word 1: the marches use only bit 0 of a wall cell).  The
// marches then hold the table in LDS and read one byte of wall data per
// cell; cls == nullptr means the geometry has no classes and they read the
// words.

// The wall data a march loads for cell c: its class byte, or its link word
// when the geometry has no classes.
__device__ __forceinline__ uint32_t wall_raw(const uint8_t* __restrict__ cls, const uint32_t* __restrict__ links,
                                             uint32_t c) {
  return cls ? static_cast<uint32_t>(cls[c]) : links[c];
}
// The link word of that data (ltab: the class table in LDS).
__device__ __forceinline__ uint32_t link_word(const uint8_t* cls, const uint32_t* ltab, uint32_t raw) {
  return cls ? ltab[raw] : raw;
}
__device__ __forceinline__ uint32_t cell_links(const uint8_t* __restrict__ cls, const uint32_t* ltab,
                                               const uint32_t* __restrict__ links, uint32_t c) {
  return link_word(cls, ltab, wall_raw(cls, links, c));
}

// Copies the class table into LDS (a workgroup barrier follows when there
// is one; all threads of the workgroup call this).
__device__ __forceinline__ void load_wall_classes(const uint8_t* cls, const uint32_t* __restrict__ table,
                                                  uint32_t* ltab, int tid, int nthreads) {
  if (!cls) return;
  for (int i = tid; i < WALL_CLASSES; i += nthreads) ltab[i] = table[i];
  __syncthreads();
}

__device__ __forceinline__ bool is_solid(const uint32_t* links, uint64_t c) { return links && (links[c] & 1u); }
// Neighbour x + c_i is a wall: bit opp(i) of x.
__device__ __forceinline__ bool ahead_solid(const uint32_t* links, uint64_t c, int i) {
  return links && ((links[c] >> opp(i)) & 1u);
}

}  // namespace lbm
