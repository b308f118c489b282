// Pieces shared by the z-marching kernels (the fused step and the fused
// reverse step): the pull of Eq. (1) with halfway bounce-back (Sec. 4) from
// one z plane's buffer resources, and the fixed-order workgroup reduction of
// FP64 partial sums.
#pragma once

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
// 16-bit forms the sum of the stored deviations X_i - w_i rho_shift (the rest
// population's with its residual row added), so that rho^a = D + rho_shift
// (the weights sum to one) and the store can keep the stored sum of a cell
// equal to D.  Both sums run in direction order.
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
    float x = Tr::decode(v);
    if constexpr (Tr::shifted) {
      // the rest population reads back as its stored value plus its residual
      if (i == 0)
        x += Tr::decode(buf_load<T>(rz[1], own, static_cast<uint32_t>(RES_ROW + s) * ppb)) * (1.0f / Tr::res_scale);
    }
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

}  // namespace lbm
