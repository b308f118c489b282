// Seed of the reverse (adjoint) sweep: dL/dX_T from dL/drho(T), the
// transpose of the pull of Eq. (1) (with halfway bounce-back, Sec. 4) that
// forms the densities at the final time.  The reverse step itself is the
// march of adjoint_march.hip.

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


unsigned grid_for_3d(const Grid& g) { return static_cast<unsigned>((g.nx + 63) / 64); }

dim3 grid3(const Grid& g) {
  return dim3(grid_for_3d(g), static_cast<unsigned>(g.ny), static_cast<unsigned>(g.nz));
}

}  // namespace

hipError_t launch_adjoint_seed(const Grid& g, const uint32_t* links, const float* grad_rho, float* lam,
                               hipStream_t st) {
  if (g.ny > 65535 || g.nz > 65535) return hipErrorInvalidValue;
  hipLaunchKernelGGL(adjoint_seed_kernel, grid3(g), dim3(64), 0, st, g, links, grad_rho, lam);
  return hipGetLastError();
}

}  // namespace lbm
