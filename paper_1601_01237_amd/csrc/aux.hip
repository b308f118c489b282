// One-thread-per-cell kernels around the fused march: initial state, wall
// link masks, conversion between stored and pre-collision populations,
// deterministic reduction of per-workgroup partial sums and the reference
// copy kernel.

#include "buffer.h"
#include "launch.h"

namespace lbm {

namespace {

constexpr int TPB = 256;

__device__ __forceinline__ uint64_t wrap_u(long long v, long long n) {
  long long r = v % n;
  return static_cast<uint64_t>(r < 0 ? r + n : r);
}

struct Coord {
  int x, y, z;
};

__device__ __forceinline__ Coord coord_of(uint64_t c, const Grid& g) {
  Coord r;
  r.z = static_cast<int>(c / g.nxy);
  const uint64_t rem = c - static_cast<uint64_t>(r.z) * g.nxy;
  r.y = static_cast<int>(rem / g.nx);
  r.x = static_cast<int>(rem - static_cast<uint64_t>(r.y) * g.nx);
  return r;
}

// Linear index of (x + dx, y + dy, z + dz) on the periodic box.
__device__ __forceinline__ uint64_t shifted(const Coord& p, int dx, int dy, int dz, const Grid& g) {
  const uint64_t x = wrap_u(p.x + dx, g.nx), y = wrap_u(p.y + dy, g.ny), z = wrap_u(p.z + dz, g.nz);
  return (z * g.ny + y) * g.nx + x;
}

// State-layout index of population (s, i) at cell (x, y, z) + (dx, dy, dz):
// z * zstride + (y / brows) * 38 * pstride + (s * 19 + i) * pstride +
// (y % brows) * nx + pos(x), with pos the row position of the storage form
// (folded 16-bit rows).
template <typename T>
__device__ __forceinline__ uint64_t pm_at(int s, int i, const Coord& p, int dx, int dy, int dz, const Grid& g) {
  const uint64_t x = wrap_u(p.x + dx, g.nx), y = wrap_u(p.y + dy, g.ny), z = wrap_u(p.z + dz, g.nz);
  return z * g.zstride + row_off(static_cast<int>(y), g) + static_cast<uint64_t>(s * Q + i) * g.pstride +
         row_pos<T>(static_cast<int>(x), g);
}

// State-layout index of the residual row of species s's rest population at
// cell p (16-bit forms, launch.h).
template <typename T>
__device__ __forceinline__ uint64_t res_at(int s, const Coord& p, const Grid& g) {
  return static_cast<uint64_t>(p.z) * g.zstride + row_off(p.y, g) + static_cast<uint64_t>(RES_ROW + s) * g.pstride +
         row_pos<T>(p.x, g);
}

// Canonical SoA index (s * 19 + i) * N + c of the FP32 population interface.
__device__ __forceinline__ uint64_t soa(int s, int i, uint64_t c, const Grid& g) {
  return static_cast<uint64_t>(s * Q + i) * g.n + c;
}

__device__ __forceinline__ float wshift(const Phys& ph, int s, int i) { return weight(i) * ph.shift[s]; }

// links bit i: cell x - c_i is solid (bit 0: x itself is solid).
__global__ void links_kernel(const Grid g, const uint8_t* __restrict__ solid, uint32_t* __restrict__ links) {
  for (uint64_t c = blockIdx.x * static_cast<uint64_t>(TPB) + threadIdx.x; c < g.n;
       c += static_cast<uint64_t>(gridDim.x) * TPB) {
    const Coord p = coord_of(c, g);
    uint32_t bits = 0;
#pragma unroll
    for (int i = 0; i < Q; ++i)
      if (solid[shifted(p, -CX[i], -CY[i], -CZ[i], g)]) bits |= 1u << i;
    links[c] = bits;
  }
}


// Stored state whose pull at every fluid cell is f_i = w_i rho0 (rest state).
template <Storage S>
__global__ void init_kernel(const Grid g, const Phys ph, const uint32_t* __restrict__ links,
                            const double* __restrict__ rho0, typename StorageTraits<S>::T* __restrict__ dst) {
  using Tr = StorageTraits<S>;
  for (uint64_t c = blockIdx.x * static_cast<uint64_t>(TPB) + threadIdx.x; c < g.n;
       c += static_cast<uint64_t>(gridDim.x) * TPB) {
    const Coord p = coord_of(c, g);
    const bool solid = is_solid(links, c);
#pragma unroll
    for (int s = 0; s < 2; ++s) {
#pragma unroll
      for (int i = 0; i < Q; ++i) {
        float v = 0.0f;
        if (!solid) {
          const uint64_t src = ahead_solid(links, c, i) ? c : shifted(p, CX[i], CY[i], CZ[i], g);
          v = static_cast<float>(weight_d(i) * rho0[s * g.n + src]);
        }
        if constexpr (Tr::shifted) v -= wshift(ph, s, i);
        const auto q = Tr::encode(v);
        dst[pm_at<typename Tr::T>(s, i, p, 0, 0, 0, g)] = q;
        // the rest population keeps its rounding error in the residual row
        if constexpr (Tr::shifted) {
          if (i == 0) dst[res_at<typename Tr::T>(s, p, g)] = Tr::encode((v - Tr::decode(q)) * Tr::res_scale);
        }
      }
    }
  }
}

template <Storage S>
__global__ void get_pop_kernel(const Grid g, const Phys ph, const uint32_t* __restrict__ links,
                               const typename StorageTraits<S>::T* __restrict__ src, float* __restrict__ f) {
  using Tr = StorageTraits<S>;
  for (uint64_t c = blockIdx.x * static_cast<uint64_t>(TPB) + threadIdx.x; c < g.n;
       c += static_cast<uint64_t>(gridDim.x) * TPB) {
    const Coord p = coord_of(c, g);
    const bool solid = is_solid(links, c);
    const uint32_t lk = links ? links[c] : 0u;
#pragma unroll
    for (int s = 0; s < 2; ++s) {
#pragma unroll
      for (int i = 0; i < Q; ++i) {
        float v = 0.0f;
        if (!solid) {
          const bool bb = (i != 0) && ((lk >> i) & 1u);
          const uint64_t at = bb ? pm_at<typename Tr::T>(s, opp(i), p, 0, 0, 0, g) : pm_at<typename Tr::T>(s, i, p, -CX[i], -CY[i], -CZ[i], g);
          v = Tr::decode(src[at]);
          if constexpr (Tr::shifted) {
            if (i == 0) v += Tr::decode(src[res_at<typename Tr::T>(s, p, g)]) * (1.0f / Tr::res_scale);
            v += wshift(ph, s, i);
          }
        }
        f[soa(s, i, c, g)] = v;
      }
    }
  }
}

// A 16-bit stored state rewritten as the FP32 stored state of the same
// populations, in the FP32 layout g32: each value decoded and shifted back
// (plus the rest population's residual), exactly as the 16-bit step's pull
// reads it.  Wall cells carry no populations and get 0.
template <Storage S>
__global__ void widen_kernel(const Grid g, const Grid g32, const Phys ph, const uint32_t* __restrict__ links,
                             const typename StorageTraits<S>::T* __restrict__ src, float* __restrict__ dst) {
  using Tr = StorageTraits<S>;
  using T = typename Tr::T;
  for (uint64_t c = blockIdx.x * static_cast<uint64_t>(TPB) + threadIdx.x; c < g.n;
       c += static_cast<uint64_t>(gridDim.x) * TPB) {
    const Coord p = coord_of(c, g);
    const bool solid = is_solid(links, c);
#pragma unroll
    for (int s = 0; s < 2; ++s) {
#pragma unroll
      for (int i = 0; i < Q; ++i) {
        float v = 0.0f;
        if (!solid) {
          v = Tr::decode(src[pm_at<T>(s, i, p, 0, 0, 0, g)]);
          if (i == 0) v += Tr::decode(src[res_at<T>(s, p, g)]) * (1.0f / Tr::res_scale);
          v += wshift(ph, s, i);
        }
        dst[pm_at<float>(s, i, p, 0, 0, 0, g32)] = v;
      }
    }
  }
}

template <Storage S>
__global__ void set_pop_kernel(const Grid g, const Phys ph, const uint32_t* __restrict__ links,
                               const float* __restrict__ f, typename StorageTraits<S>::T* __restrict__ dst) {
  using Tr = StorageTraits<S>;
  for (uint64_t c = blockIdx.x * static_cast<uint64_t>(TPB) + threadIdx.x; c < g.n;
       c += static_cast<uint64_t>(gridDim.x) * TPB) {
    const Coord p = coord_of(c, g);
    const bool solid = is_solid(links, c);
#pragma unroll
    for (int s = 0; s < 2; ++s) {
#pragma unroll
      for (int j = 0; j < Q; ++j) {
        float v = 0.0f;
        if (!solid) {
          // X_j(y) is read by f_j(y + c_j), or by f_opp(j)(y) if y + c_j is a wall.
          const bool back = ahead_solid(links, c, j);
          const uint64_t at = back ? c : shifted(p, CX[j], CY[j], CZ[j], g);
          const int pop = back ? opp(j) : j;
          v = f[soa(s, pop, at, g)];
        }
        if constexpr (Tr::shifted) v -= wshift(ph, s, j);
        const auto q = Tr::encode(v);
        dst[pm_at<typename Tr::T>(s, j, p, 0, 0, 0, g)] = q;
        if constexpr (Tr::shifted) {
          if (j == 0) dst[res_at<typename Tr::T>(s, p, g)] = Tr::encode((v - Tr::decode(q)) * Tr::res_scale);
        }
      }
    }
  }
}

// Sum (or max) of per-workgroup partials, one value per block of threads,
// in a fixed order so that results are bitwise reproducible.  Entry
// max_index takes the maximum (the partials it reduces are >= 0).
__global__ void finalize_kernel(const double* __restrict__ partials, int blocks, int nvals, int max_index,
                                double* out, int accumulate) {
  __shared__ double sh[TPB];
  const int k = blockIdx.x;
  const bool mx = (k == max_index);
  double acc = 0.0;
  for (int b = threadIdx.x; b < blocks; b += TPB) {
    const double v = partials[static_cast<uint64_t>(b) * nvals + k];
    acc = mx ? fmax(acc, v) : acc + v;
  }
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int o = TPB / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) sh[threadIdx.x] = mx ? fmax(sh[threadIdx.x], sh[threadIdx.x + o])
                                              : sh[threadIdx.x] + sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[k] = accumulate ? out[k] + sh[0] : sh[0];
}

// Plain streaming copy: the reference for how much read + write bandwidth
// the memory system delivers to a kernel.  One 16-byte element per lane and
// no loop (many short-lived waves keep the most requests in flight), with
// non-temporal stores.
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

__global__ void __launch_bounds__(256) stream_copy_kernel(const u32x4* __restrict__ src, u32x4* __restrict__ dst,
                                                          uint64_t n16) {
  const uint64_t i = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x;
  if (i < n16) __builtin_nontemporal_store(src[i], &dst[i]);
}

// The fused step's memory pattern without its arithmetic: one workgroup per
// 128 x 4 column tile marches its chunk of z planes (the step's automatic
// tiling for FP32), and per plane every lane loads the 38 population values
// of its cell, then stores them (non-temporal) at the same place in dst.  No
// halo and no re-read: it moves exactly the step's algorithmic bytes (with
// the residual rows of the 16-bit forms), so its rate is the ceiling of that
// access pattern on the device.
template <typename T>
__global__ void __launch_bounds__(512) march_copy_kernel(const Grid g, const Tiling tl, const T* __restrict__ src,
                                                         T* __restrict__ dst) {
  const int b = xcd_remap(blockIdx.x, gridDim.x);
  const TileCoord tc = tile_of_block(b, tl);
  const int bxx = tc.x, byy = tc.y, bz = tc.z;
  const int x = bxx * 128 + static_cast<int>(threadIdx.x & 127u);
  const int y = byy * 4 + static_cast<int>(threadIdx.x >> 7);
  if (x >= g.nx || y >= g.ny) return;  // no barriers below
  const uint64_t col = row_off(y, g) + static_cast<uint64_t>(x);
  const int z1 = min((bz + 1) * tl.zchunk, g.nz);
  for (int z = bz * tl.zchunk; z < z1; ++z) {
    const uint64_t base = static_cast<uint64_t>(z) * g.zstride + col;
    constexpr int R = block_rows(sizeof(T));
    T v[R];
#pragma unroll
    for (int i = 0; i < R; ++i) v[i] = src[base + static_cast<uint64_t>(i) * g.pstride];
#pragma unroll
    for (int i = 0; i < R; ++i) __builtin_nontemporal_store(v[i], &dst[base + static_cast<uint64_t>(i) * g.pstride]);
  }
}

unsigned grid_for(uint64_t n) {
  uint64_t b = (n + TPB - 1) / TPB;
  if (b > 65536ull * 16) b = 65536ull * 16;
  if (b == 0) b = 1;
  return static_cast<unsigned>(b);
}

}  // namespace

Layout state_layout(int nx, int ny, int elem_bytes) {
  Layout L;
  L.brows = static_cast<uint32_t>(elem_bytes == 4 ? (ny < 4 ? ny : 4) : ny);
  const uint64_t bytes = static_cast<uint64_t>(nx) * L.brows * elem_bytes;
  uint64_t padded = ((bytes + 255) / 256) * 256;
  if (padded % 65536 == 0) padded += 256;
  L.pstride = static_cast<uint32_t>(padded / elem_bytes);
  const uint64_t blocks = (static_cast<uint64_t>(ny) + L.brows - 1) / L.brows;
  L.zstride = static_cast<uint64_t>(block_rows(elem_bytes)) * L.pstride * blocks;
  return L;
}

hipError_t launch_links(const Grid& g, const uint8_t* solid, uint32_t* links, hipStream_t st) {
  hipLaunchKernelGGL(links_kernel, dim3(grid_for(g.n)), dim3(TPB), 0, st, g, solid, links);
  return hipGetLastError();
}

hipError_t launch_init(Storage s, const Grid& g, const Phys& ph, const uint32_t* links, const double* rho0,
                       void* dst, hipStream_t st) {
  const dim3 gr(grid_for(g.n)), bl(TPB);
  switch (s) {
    case Storage::F32:
      hipLaunchKernelGGL(init_kernel<Storage::F32>, gr, bl, 0, st, g, ph, links, rho0, static_cast<float*>(dst));
      break;
    case Storage::F16:
      hipLaunchKernelGGL(init_kernel<Storage::F16>, gr, bl, 0, st, g, ph, links, rho0, static_cast<_Float16*>(dst));
      break;
    case Storage::BF16:
      hipLaunchKernelGGL(init_kernel<Storage::BF16>, gr, bl, 0, st, g, ph, links, rho0, static_cast<uint16_t*>(dst));
      break;
  }
  return hipGetLastError();
}

hipError_t launch_get_populations(Storage s, const Grid& g, const Phys& ph, const uint32_t* links,
                                  const void* src, float* f, hipStream_t st) {
  const dim3 gr(grid_for(g.n)), bl(TPB);
  switch (s) {
    case Storage::F32:
      hipLaunchKernelGGL(get_pop_kernel<Storage::F32>, gr, bl, 0, st, g, ph, links, static_cast<const float*>(src), f);
      break;
    case Storage::F16:
      hipLaunchKernelGGL(get_pop_kernel<Storage::F16>, gr, bl, 0, st, g, ph, links, static_cast<const _Float16*>(src), f);
      break;
    case Storage::BF16:
      hipLaunchKernelGGL(get_pop_kernel<Storage::BF16>, gr, bl, 0, st, g, ph, links, static_cast<const uint16_t*>(src), f);
      break;
  }
  return hipGetLastError();
}

hipError_t launch_widen_state(Storage s, const Grid& g, const Grid& g32, const Phys& ph, const uint32_t* links,
                              const void* src, float* dst, hipStream_t st) {
  const dim3 gr(grid_for(g.n)), bl(TPB);
  switch (s) {
    case Storage::F16:
      hipLaunchKernelGGL(widen_kernel<Storage::F16>, gr, bl, 0, st, g, g32, ph, links,
                         static_cast<const _Float16*>(src), dst);
      break;
    case Storage::BF16:
      hipLaunchKernelGGL(widen_kernel<Storage::BF16>, gr, bl, 0, st, g, g32, ph, links,
                         static_cast<const uint16_t*>(src), dst);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_set_populations(Storage s, const Grid& g, const Phys& ph, const uint32_t* links,
                                  const float* f, void* dst, hipStream_t st) {
  const dim3 gr(grid_for(g.n)), bl(TPB);
  switch (s) {
    case Storage::F32:
      hipLaunchKernelGGL(set_pop_kernel<Storage::F32>, gr, bl, 0, st, g, ph, links, f, static_cast<float*>(dst));
      break;
    case Storage::F16:
      hipLaunchKernelGGL(set_pop_kernel<Storage::F16>, gr, bl, 0, st, g, ph, links, f, static_cast<_Float16*>(dst));
      break;
    case Storage::BF16:
      hipLaunchKernelGGL(set_pop_kernel<Storage::BF16>, gr, bl, 0, st, g, ph, links, f, static_cast<uint16_t*>(dst));
      break;
  }
  return hipGetLastError();
}

hipError_t launch_finalize(const double* partials, int blocks, int nvals, int max_index, double* out,
                           bool accumulate, hipStream_t st) {
  hipLaunchKernelGGL(finalize_kernel, dim3(nvals), dim3(TPB), 0, st, partials, blocks, nvals, max_index, out,
                     accumulate ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_march_copy(Storage s, const Grid& g, const void* src, void* dst, hipStream_t st) {
  const Tiling t = make_tiling(g, 3, 0, true);  // 128 x 4 tiles, the open-box default chunk of z planes
  if (t.blocks <= 0) return hipErrorInvalidValue;
  if (s == Storage::F32) {
    hipLaunchKernelGGL(march_copy_kernel<float>, dim3(t.blocks), dim3(512), 0, st, g, t,
                       static_cast<const float*>(src), static_cast<float*>(dst));
  } else {
    hipLaunchKernelGGL(march_copy_kernel<uint16_t>, dim3(t.blocks), dim3(512), 0, st, g, t,
                       static_cast<const uint16_t*>(src), static_cast<uint16_t*>(dst));
  }
  return hipGetLastError();
}

hipError_t launch_stream_copy(const void* src, void* dst, uint64_t bytes, hipStream_t st) {
  const uint64_t n16 = bytes / 16;
  if (n16 == 0) return hipSuccess;
  const uint64_t blocks = (n16 + TPB - 1) / TPB;
  if (blocks > 0x7fffffffull) return hipErrorInvalidValue;
  hipLaunchKernelGGL(stream_copy_kernel, dim3(static_cast<unsigned>(blocks)), dim3(TPB), 0, st,
                     static_cast<const u32x4*>(src), static_cast<u32x4*>(dst), n16);
  return hipGetLastError();
}

}  // namespace lbm
