// D3Q19 velocity set and the storage forms of the population buffers.
//
// Velocities follow the lattice of Sec. 2 of arXiv 1601.01237 (19 discrete
// velocities); the weights are the isotropic ones (1/3 rest, 1/18 faces,
// 1/36 edges).  Order: rest, then opposite pairs (1,2), (3,4), ..., (17,18),
// so that direction 2k-1 and 2k are negatives of each other.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbm {

constexpr int Q = 19;

// Component tables (x, y, z) of each direction.
constexpr int CX[Q] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
constexpr int CY[Q] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
constexpr int CZ[Q] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};

constexpr float T0F = 1.0f / 3.0f;  // lattice temperature T0 (Sec. 2)
constexpr float W0 = 1.0f / 3.0f;
constexpr float WF = 1.0f / 18.0f;
constexpr float WE = 1.0f / 36.0f;

__host__ __device__ constexpr float weight(int i) { return i == 0 ? W0 : (i <= 6 ? WF : WE); }
__host__ __device__ constexpr double weight_d(int i) {
  return i == 0 ? 1.0 / 3.0 : (i <= 6 ? 1.0 / 18.0 : 1.0 / 36.0);
}
__host__ __device__ constexpr int opp(int i) { return i == 0 ? 0 : ((i & 1) ? i + 1 : i - 1); }

// ---------------------------------------------------------------------------
// Storage forms.  Arithmetic is FP32; the 16-bit forms hold X - w_i rho_shift
// rounded to nearest even.
// ---------------------------------------------------------------------------
enum class Storage : int { F32 = 0, F16 = 1, BF16 = 2 };

template <Storage S> struct StorageTraits;

template <> struct StorageTraits<Storage::F32> {
  using T = float;
  static constexpr bool shifted = false;
  __device__ static inline float decode(float v) { return v; }
  __device__ static inline float encode(float v) { return v; }
};

// The 16-bit forms store X - w_shift: decode reads a stored value back as the
// deviation, encode rounds a deviation to the storage type (the kernels add
// and subtract w_shift).  (Mixed-precision FMAs would fuse a conversion and
// the shift into one instruction, but measured slower on gfx950 than convert
// plus add.)
// res_scale: the residual of a rest population (launch.h) is stored
// multiplied by this power of two, which keeps it clear of the FP16
// subnormals (the residual is at most 2^-11 of the value it corrects).
template <> struct StorageTraits<Storage::F16> {
  using T = _Float16;
  static constexpr bool shifted = true;
  static constexpr float res_scale = 2048.0f;
  __device__ static inline float decode(_Float16 v) { return static_cast<float>(v); }
  __device__ static inline _Float16 encode(float v) { return static_cast<_Float16>(v); }
  // Halves of a 32-bit word of a folded row, and the bits of one value.
  __device__ static inline float lo(uint32_t w) {
    return static_cast<float>(__builtin_bit_cast(_Float16, static_cast<uint16_t>(w & 0xffffu)));
  }
  __device__ static inline float hi(uint32_t w) {
    return static_cast<float>(__builtin_bit_cast(_Float16, static_cast<uint16_t>(w >> 16)));
  }
  __device__ static inline uint32_t bits(_Float16 q) { return __builtin_bit_cast(uint16_t, q); }
};

// bfloat16 kept as its bit pattern: the upper half of an IEEE binary32.
// Encoding rounds to nearest, ties to even (the native conversion).
template <> struct StorageTraits<Storage::BF16> {
  using T = uint16_t;
  static constexpr bool shifted = true;
  static constexpr float res_scale = 1.0f;
  __device__ static inline float decode(uint16_t v) {
    return __uint_as_float(static_cast<uint32_t>(v) << 16);
  }
  __device__ static inline uint16_t encode(float v) { return __builtin_bit_cast(uint16_t, static_cast<__bf16>(v)); }
  __device__ static inline float lo(uint32_t w) { return __uint_as_float(w << 16); }
  __device__ static inline float hi(uint32_t w) { return __uint_as_float(w & 0xffff0000u); }
  __device__ static inline uint32_t bits(uint16_t q) { return q; }
};

}  // namespace lbm
