/* Host-side calls of the C ABI that need no GPU, for a build of liblbm.so
 * whose host code carries AddressSanitizer: size queries, velocity set,
 * status strings, and every argument check that must reject a call before
 * any device work.  Exits non-zero on an unexpected status. */
#include <stdio.h>
#include <string.h>

#include "lbm.h"

static int fails = 0;
#define EXPECT(cond)                                              \
  do {                                                            \
    if (!(cond)) {                                                \
      fprintf(stderr, "expectation failed: %s (line %d)\n", #cond, __LINE__); \
      ++fails;                                                    \
    }                                                             \
  } while (0)

int main(void) {
  int32_t c[3 * LBM_Q];
  double w[LBM_Q];
  EXPECT(lbm_version() > 0);
  EXPECT(lbm_velocity_set(c, w) == LBM_OK);
  EXPECT(lbm_velocity_set(NULL, NULL) == LBM_OK);
  for (int s = -6; s <= 1; ++s) EXPECT(lbm_status_str((lbm_status)s) != NULL && strlen(lbm_status_str((lbm_status)s)) > 0);
  EXPECT(lbm_plane_stride(128, 128, LBM_FP32) >= 4 * 128);
  EXPECT(lbm_plane_stride(128, 128, LBM_FP16) >= 128 * 128);
  EXPECT(lbm_plane_stride(0, 4, LBM_FP32) == -1);
  EXPECT(lbm_row_block(128, 128, LBM_FP32) == 4);
  EXPECT(lbm_row_block(128, 128, LBM_FP16) == 128);
  EXPECT(lbm_state_elems(70, 19, 7, LBM_BF16) > 0);
  EXPECT(lbm_state_elems(4, 4, 0, LBM_FP32) == -1);
  EXPECT(lbm_row_half(64, LBM_FP16, 0) == 32);
  EXPECT(lbm_row_half(64, LBM_FP16, 1) == 0);
  EXPECT(lbm_row_half(0, LBM_FP16, 0) == -1);

  lbm_params p;
  memset(&p, 0, sizeof(p));
  p.nx = p.ny = p.nz = 8;
  p.storage = LBM_FP32;
  p.tau[0] = p.tau[1] = 1.0;
  p.G[0][1] = p.G[1][0] = -1.0;
  p.collision = LBM_BGK;
  char a[8], b[8];
  double rho0[2];
  lbm_ctx *ctx = (lbm_ctx *)&p; /* must be overwritten with NULL on failure */
  EXPECT(lbm_init(NULL, &p, a, b, NULL, rho0, NULL) == LBM_EINVAL);
  EXPECT(lbm_init(&ctx, NULL, a, b, NULL, rho0, NULL) == LBM_EINVAL);
  EXPECT(lbm_init(&ctx, &p, NULL, b, NULL, rho0, NULL) == LBM_EINVAL);
  EXPECT(lbm_init(&ctx, &p, a, a, NULL, rho0, NULL) == LBM_EINVAL);
  EXPECT(lbm_init(&ctx, &p, a, b, NULL, NULL, NULL) == LBM_EINVAL);
  lbm_params q = p;
  q.tau[1] = 0.5;
  EXPECT(lbm_init(&ctx, &q, a, b, NULL, rho0, NULL) == LBM_EINVAL);
  q = p;
  q.nx = 0;
  EXPECT(lbm_init(&ctx, &q, a, b, NULL, rho0, NULL) == LBM_EINVAL);
  q = p;
  q.storage = 7;
  EXPECT(lbm_init(&ctx, &q, a, b, NULL, rho0, NULL) == LBM_EINVAL);
  q = p;
  q.collision = 9;
  EXPECT(lbm_init(&ctx, &q, a, b, NULL, rho0, NULL) == LBM_EINVAL);
  EXPECT(ctx == NULL);

  float f[4];
  double diag[LBM_DIAG_LEN];
  EXPECT(lbm_step(NULL, 1) == LBM_EINVAL);
  EXPECT(lbm_moments(NULL, f, f, diag, NULL) == LBM_EINVAL);
  EXPECT(lbm_get_populations(NULL, f) == LBM_EINVAL);
  EXPECT(lbm_set_populations(NULL, f) == LBM_EINVAL);
  EXPECT(lbm_time(NULL) == -1);
  EXPECT(lbm_set_time(NULL, 3) == LBM_EINVAL);
  EXPECT(lbm_set_tiling(NULL, 0, 0) == LBM_EINVAL);
  EXPECT(lbm_adjoint_work_bytes(NULL) == 0);
  EXPECT(lbm_adjoint_step(NULL, a, f, f, a, 8, diag, NULL) == LBM_EINVAL);
  EXPECT(lbm_adjoint_seed(NULL, f, f) == LBM_EINVAL);
  EXPECT(lbm_stream_copy(a, a, 16, NULL) == LBM_EINVAL);
  EXPECT(lbm_stream_copy(a, b, 15, NULL) == LBM_EINVAL);
  EXPECT(lbm_march_copy(NULL, a, b) == LBM_EINVAL);
  EXPECT(lbm_destroy(NULL) == LBM_OK);

  if (fails) {
    fprintf(stderr, "%d expectation(s) failed\n", fails);
    return 1;
  }
  printf("asan driver: all host-side checks passed\n");
  return 0;
}
