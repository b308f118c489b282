/*
 * lbm.h -- C ABI of the MI355X (gfx950) two-component D3Q19 lattice
 * Boltzmann library liblbm.so.
 *
 * Method: Otomo et al., "Studies of accurate multi-component lattice Boltzmann
 * models on benchmark cases required for engineering applications"
 * (arXiv 1601.01237), Sec. 2 and Sec. 4:
 *   - Eq. (1)   per-species lattice Boltzmann equation, D3Q19, dt = dx = 1;
 *   - Eq. (2)   BGK collision with relaxation time tau_a;
 *   - Eq. (3)   third-order equilibrium, T0 = 1/3;
 *   - Eqs. (4)-(6) species density, mixture density and mixture velocity;
 *   - Eq. (7)   Shan-Chen inter-component force with G^{aa} = 0;
 *   - Eqs. (8)-(9) force velocity u_F = u + g/2;
 *   - Sec. 4    pointwise (halfway) bounce-back and wall potential rho_s^a.
 * The forcing term, which the paper takes from a citation, is the exact
 * difference f^eq(rho^a, u + g^a) - f^eq(rho^a, u) of Eq. (3).
 *
 * Conventions shared by every entry point
 *   Grid:     nx * ny * nz cells, x fastest; cell index c = (z*ny + y)*nx + x.
 *             Every axis is periodic; walls are solid cells inside the box.
 *   Species:  a = 0 (A) and a = 1 (B).
 *   Velocity set: LBM_Q = 19 directions in the order returned by
 *             lbm_velocity_set(): rest, then opposite pairs (1,2), (3,4), ...
 *   Populations (FP32 interface of lbm_get/set_populations): 2*19*N
 *             elements, element (a, i, c) at index (a*19 + i)*N + c.
 *   State:    the library keeps the post-collision, pre-streaming populations
 *             X (one buffer per time level, two buffers ping-pong).  At time t
 *             the current state lives in buf_a if t is even, buf_b if odd.
 *             Stored states and adjoint arrays use the row-blocked layout:
 *             each z plane is a sequence of blocks of B = lbm_row_block(nx,
 *             ny, storage) y rows, and a block holds the B rows of population
 *             (0, 0), then those of (0, 1), ..., (1, 18), S elements apart
 *             (S = lbm_plane_stride(nx, ny, storage) >= B*nx), then, in the
 *             16-bit forms only, two residual rows: row 38 + a holds the
 *             rounding residual r of species a's rest population, scaled by
 *             s = 2048 (FP16) or 1 (BF16), so that the rest population reads
 *             back as decode(X_0) + decode(r)/s.  With R = 38 rows per block
 *             (FP32) or 40 (16-bit), element (a, i, x, y, z) sits at index
 *               z*Z + (y / B)*R*S + (a*19 + i)*S + (y % B)*nx + pos(x),
 *             Z = R*S*ceil(ny / B) elements per z plane.  FP32 takes B = 4
 *             (or ny if smaller): the 38 population rows a workgroup reads
 *             from one plane are one contiguous range.  The 16-bit forms
 *             take B = ny (population planes).  pos(x) = x, except for the
 *             16-bit storage forms with even nx and no walls, whose rows
 *             are folded: with h = nx/2 (lbm_row_half), pos(x) = 2x for
 *             x < h and 2(x - h) + 1 for x >= h, so the 32-bit word k of a
 *             row holds cells k and k + h.  The S - B*nx elements after each
 *             population's rows, and the rows past ny in the last block,
 *             are padding (never read): population blocks a large power of
 *             two apart would map the rows a step reads together onto the
 *             same DRAM channels.  A state (or adjoint) buffer holds
 *             lbm_state_elems(nx, ny, nz, storage) = nz*Z elements.
 *             The pre-collision populations of Eq. (1) at time t are the pull
 *             f_i(x) = X_i(x - c_i), or X_opp(i)(x) if x - c_i is solid.
 *   Memory:   every array pointer is DEVICE memory owned by the caller unless
 *             stated otherwise; the library keeps non-owning pointers, so the
 *             arrays must outlive the context.  The library itself allocates
 *             only its context, a per-cell link mask when walls are given
 *             (4 bytes per cell) and a small reduction buffer.
 *   Streams:  every call is enqueued asynchronously on the stream given to
 *             lbm_init (a hipStream_t passed as void*; NULL = null stream).
 *             Argument checks are synchronous and return LBM_EINVAL /
 *             LBM_ENOTSUP before anything is enqueued; a failed launch
 *             returns LBM_EHIP.  No call synchronises the stream.
 *   Threads:  a context is not thread-safe; use one context per stream.
 *   Errors:   no exception, abort or exit crosses this interface.
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  LBM_OK = 0,
  LBM_EINVAL = -1,    /* bad argument (null pointer, size, tau <= 1/2, ...)  */
  LBM_EHIP = -2,      /* a HIP runtime call or kernel launch failed          */
  LBM_ESTATE = -3,    /* call not valid in the context's current state       */
  LBM_EUNSTABLE = -4, /* non-finite values found (reported by callers that   */
                      /* read the diagnostic vector)                         */
  LBM_ENOTSUP = -5    /* valid request outside what this build supports      */
} lbm_status;

/* Storage of the population buffers.  Arithmetic is always FP32.  The
 * 16-bit forms store X_i - w_i * rho_shift[a] rounded to nearest even; the
 * rest population (i = 0), which holds most of a cell's mass, also keeps the
 * rounding residual of that value (the residual rows of the layout). */
typedef enum { LBM_FP32 = 0, LBM_FP16 = 1, LBM_BF16 = 2 } lbm_storage;

/* Collision operator.
 *   LBM_BGK          Eq. (2): f* = f - (f - f^eq)/tau + F.
 *   LBM_REGULARIZED  Eqs. (10)-(11) of Sec. 3: f* = f^eq + (1 - 1/tau) f^neq
 *                    + F, where f^neq is the second-order Hermite projection
 *                    w_i (c_i c_i - T0 I) : Pi / (2 T0^2) of the
 *                    non-equilibrium part (Pi = sum_i c_i c_i (f_i - f^eq_i))
 *                    -- a reading: the paper names the filter and takes its
 *                    formula from citations.
 *   LBM_REGULARIZED3 the same filter also keeping the energy flux (Sec. 3:
 *                    the third order for the energy flux): f^neq adds
 *                    w_i H_i . q / (2 T0^3) with the contracted third-order
 *                    Hermite polynomials H_{i,a} = sum_{b != a} (c_a c_b^2 -
 *                    T0 c_a) and q_a = sum_i H_{i,a} (f_i - f^eq_i).
 * F is the exact-difference forcing term in all three. */
typedef enum { LBM_BGK = 0, LBM_REGULARIZED = 1, LBM_REGULARIZED3 = 2 } lbm_collision;

#define LBM_Q 19
#define LBM_DIAG_LEN 16

/* Indices into the diagnostic vector written by lbm_moments (FP64). */
enum {
  LBM_DIAG_MASS_A = 0,   /* sum over fluid cells of rho^A                       */
  LBM_DIAG_MASS_B = 1,   /* sum over fluid cells of rho^B                       */
  LBM_DIAG_MOM_X = 2,    /* sum of rho * u_F, x y z (Eqs. 8-9)                  */
  LBM_DIAG_MOM_Y = 3,
  LBM_DIAG_MOM_Z = 4,
  LBM_DIAG_MAX_UF = 5,   /* max |u_F| over fluid cells (spurious velocity)      */
  LBM_DIAG_NONFINITE = 6,/* fluid cells with a non-finite rho^A, rho^B or u_F   */
  LBM_DIAG_N_FLUID = 7,  /* number of fluid cells                               */
  LBM_DIAG_P_IN_SUM = 8, /* sum of p over fluid cells with |x - centre| < r_in  */
  LBM_DIAG_N_IN = 9,
  LBM_DIAG_P_OUT_SUM = 10,/* sum of p over fluid cells with |x - centre| > r_out */
  LBM_DIAG_N_OUT = 11,
  LBM_DIAG_N_THR = 12,   /* fluid cells with rho^A > thr                        */
  LBM_DIAG_SDX_THR = 13, /* sum over those cells of the minimum-image offset    */
  LBM_DIAG_SDY_THR = 14, /* from the centre, x y z                              */
  LBM_DIAG_SDZ_THR = 15
};

typedef struct {
  int32_t nx, ny, nz;  /* >= 1 each; sizes as lbm_state_elems accepts      */
  int32_t storage;     /* lbm_storage                                        */
  double tau[2];       /* relaxation times tau_A, tau_B (Eq. 2), > 1/2       */
  double G[2][2];      /* interaction matrix G^{ab} of Eq. (7), paper sign:  */
                       /* repulsion is G[0][1], G[1][0] < 0.  G[a][a] must   */
                       /* be 0 (Sec. 2), else LBM_ENOTSUP.                   */
  double rho_shift[2]; /* shift of the 16-bit storage forms (ignored in FP32)*/
  double rho_wall[2];  /* wall potential rho_s^a (Sec. 4): the density a     */
                       /* solid neighbour contributes to the Eq. (7) sum     */
  int32_t collision;   /* lbm_collision                                      */
} lbm_params;

/* Region parameters of the diagnostic vector (host struct). */
typedef struct {
  double center[3];    /* x, y, z; offsets use the periodic minimum image    */
  double r_in, r_out;  /* Laplace-pressure averaging radii                   */
  double thr;          /* droplet threshold on rho^A                         */
} lbm_diag_region;

typedef struct lbm_ctx lbm_ctx;

/* Library version (major*10000 + minor*100 + patch).  Pure host call. */
int32_t lbm_version(void);

/* Copies the D3Q19 velocity set in the library's order: c[3*i + k] is
 * component k (x, y, z) of c_i; w[i] its weight (1/3, 1/18, 1/36 -- the
 * isotropic weights of Sec. 2).  Either pointer may be NULL.  Host memory.
 * Pure host call, needs no GPU. */
lbm_status lbm_velocity_set(int32_t *c, double *w);

/* Human-readable name of a status code (static string). */
const char *lbm_status_str(lbm_status s);

/* S of the layout above: elements from one population's rows of a row
 * block to the next population's, for storage `storage` (lbm_storage): B*nx
 * elements rounded up to 256 bytes, plus 256 bytes when that is a multiple
 * of 64 KiB.  Adjoint arrays use the FP32 value.  Returns -1 for sizes the
 * library does not support: nx*ny times the element size, and one z plane
 * of the state (Z elements), must stay below 2 GiB.  Pure host call. */
int64_t lbm_plane_stride(int32_t nx, int32_t ny, int32_t storage);

/* B of the layout above: y rows per row block (4 or ny for FP32, ny for
 * the 16-bit forms); -1 where lbm_plane_stride is -1.  Pure host call. */
int32_t lbm_row_block(int32_t nx, int32_t ny, int32_t storage);

/* h = nx/2 when rows of storage `storage` are folded (16-bit forms, even
 * nx, walls == 0; see pos(x) above), 0 when rows are stored in x order, -1
 * for nx < 1 or an unknown storage.  `walls` is nonzero when the context is
 * created with a solid mask.  Pure host call. */
int32_t lbm_row_half(int32_t nx, int32_t storage, int32_t walls);

/* Elements of one state buffer (buf_a, buf_b, x_t) of storage `storage`, and
 * of one adjoint array (lam) with storage LBM_FP32: nz*Z (layout above).
 * Returns -1 for unsupported sizes: those of lbm_plane_stride, and N cells
 * with N >= 2^31 or N times the element size >= 4 GiB.  lbm_init answers
 * LBM_ENOTSUP for exactly these sizes (nx, ny, nz >= 1).  Pure host call. */
int64_t lbm_state_elems(int32_t nx, int32_t ny, int32_t nz, int32_t storage);

/* Creates a context and writes the rest state at t = 0 into buf_a.
 *   p      host; copied.
 *   buf_a, buf_b  device, lbm_state_elems(nx, ny, nz, storage) elements of
 *          the storage type each (the padding between planes is not written).
 *   solid  device, N bytes, nonzero = wall cell; NULL = no walls.
 *   rho0   device, 2*N doubles: rho0^a(c) at index a*N + c.  The initial
 *          pre-collision state is f_i^a = w_i rho0^a (Eq. 3 at u = 0) on fluid
 *          cells; solid cells carry no populations.
 *   stream hipStream_t as void*.
 * On success *ctx owns a host struct and (walls only) a device link mask:
 * the 4-byte link words and, when there are few distinct words, the class
 * bytes (lbm_wall_classes), 5 bytes per cell and 1 KiB.  With walls the
 * call waits for the stream: it reads the link words back to the host once
 * to number the classes (5 bytes per cell of pageable host memory, freed
 * before it returns).
 * Allocation failures return LBM_EHIP and leave *ctx NULL. */
lbm_status lbm_init(lbm_ctx **ctx, const lbm_params *p, void *buf_a, void *buf_b,
                    const uint8_t *solid, const double *rho0, void *stream);

/* Advances n >= 0 time steps of Eq. (1) (collide with Eqs. 2-3 and 7, then
 * stream with bounce-back); t += n.  One fused kernel launch per step. */
lbm_status lbm_step(lbm_ctx *ctx, int64_t n);

/* One step, as lbm_step(ctx, 1), that also writes the forward quantities
 * the reverse step at this time level needs (Eqs. 4-6 at the pull of X_t):
 * fields (device float, 5*N, caller-owned, index k*N + c) receives
 * rho~^A, rho~^B, u_x, u_y, u_z of every cell c, with rho~^a = rho_s^a and
 * u = 0 on wall cells.  Passed to lbm_adjoint_step_fields with the same X_t,
 * it replaces the reverse march's own pull of the tile border.  FP32
 * storage only (LBM_ENOTSUP otherwise); fields must not alias a state
 * buffer (LBM_EINVAL).  t += 1. */
lbm_status lbm_step_fields(lbm_ctx *ctx, float *fields);

/* Observables of the current time t (Eqs. 4-9).  Any output may be NULL.
 *   rho    device float, 2*N: rho^a(c) at a*N + c (0 on solid cells).
 *   u_f    device float, 3*N: component k of u_F at k*N + c (0 on solid).
 *   diag   device double, LBM_DIAG_LEN entries (see the index list above);
 *          pressure p = T0 (rho^A + rho^B) - G T0 rho^A rho^B with
 *          G = (G[0][1] + G[1][0]) / 2.
 *   region host, may be NULL (centre of the box, r_in = 0, r_out = inf,
 *          thr = 0.515). */
lbm_status lbm_moments(lbm_ctx *ctx, float *rho, float *u_f, double *diag,
                       const lbm_diag_region *region);

/* Workgroups of the diagnostics launch that lbm_moments_static can hold. */
#define LBM_STATIC_BLOCKS 8192

/* lbm_moments for callers that cannot allocate device memory: code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.
 * Same arguments, launch and outputs as lbm_moments (bitwise equal).  It
 * calls no allocating routine: its per-workgroup partial sums live in a
 * fixed device array of the library, LBM_STATIC_BLOCKS * LBM_DIAG_LEN
 * doubles (1 MiB) per GPU, held until the process ends; every workgroup
 * overwrites its own partials, so nothing needs clearing between calls.
 *   Limit: the diagnostics launch (64 x 8 column tiles, z chunks of up to
 *   256 planes) must have at most LBM_STATIC_BLOCKS workgroups, which holds
 *   for nx*ny up to about 4.2 million cells and nx*ny*nz up to about 10^9.
 *   Errors: LBM_EINVAL for a NULL ctx; LBM_ENOTSUP beyond the limit;
 *   LBM_EHIP if the array's device address could not be looked up at
 *   lbm_init or the launch fails.
 *   Concurrency: every call on one GPU shares that GPU's array, so calls
 *   that overlap in time on one GPU (other streams, other contexts, other
 *   host threads) race and must be ordered by the caller. */
lbm_status lbm_moments_static(lbm_ctx *ctx, float *rho, float *u_f, double *diag,
                              const lbm_diag_region *region);

/* Pre-collision populations f_i^a(x, t) of the current time as FP32
 * (device, 2*19*N, index (a*19 + i)*N + c); zero on solid cells. */
lbm_status lbm_get_populations(lbm_ctx *ctx, float *f);

/* Replaces the current state by the given pre-collision populations
 * (device FP32, 2*19*N, index (a*19 + i)*N + c).  Values on solid cells are
 * ignored. */
lbm_status lbm_set_populations(lbm_ctx *ctx, const float *f);

/* Current time level t. */
int64_t lbm_time(const lbm_ctx *ctx);

/* Sets t (e.g. after restoring a checkpoint into the matching buffer). */
lbm_status lbm_set_time(lbm_ctx *ctx, int64_t t);

/* Tiling of the fused step kernel: workgroup tile shape and the number of z
 * planes each workgroup marches through (>= 1; 0 picks a default from the
 * grid).  Shapes with one cell per lane (cells in x by y): 0 = 64x8,
 * 1 = 64x12, 2 = 32x16, 3 = 128x4, 4 = 64x4, 5 = 256x2.  Shapes with one
 * folded 32-bit word (two cells) per lane, for 16-bit storage with folded
 * rows and no walls only (else LBM_EINVAL), in words by rows: 6 = 64x8,
 * 7 = 32x16, 8 = 32x8, 9 = 32x12.  -1 (the default) picks 8 for folded
 * 16-bit rows without walls; with walls or 16-bit storage, of 64x8 and
 * 32x16 the one that pads the x-y plane least (64x8 on a tie); for FP32
 * without walls the first of 128x4, 64x12, 64x8 and 32x16 whose padded x-y
 * plane is at most 1.3 times the least padded one, and 64x4 when that
 * choice would launch at most 128 workgroups.  The default z chunk of a context
 * without walls minimises (rounds of 256 workgroups) x (chunk + 2) over
 * chunks of 4 to 256 planes (512 for the folded shapes); with walls it is
 * about nz * tiles / 512 planes, 8 to 256.  Results do not depend on this
 * choice (bitwise).
 * The reverse march has its own setting (lbm_set_adjoint_tiling);
 * diagnostics use 64x8.  Host-side setting. */
lbm_status lbm_set_tiling(lbm_ctx *ctx, int32_t tile, int32_t zchunk);

/* Placement of the step kernel's workgroups (results do not depend on it,
 * bitwise; host-side setting).
 *   order: the order in which workgroups cover the (z chunk, tile) pairs.
 *     The device deals consecutive workgroups to its 8 XCDs in turn and the
 *     kernel renumbers them so that each XCD (with its own L2 cache) runs a
 *     contiguous range of the order, so the order decides which tiles share
 *     an L2 while they run.  1 = chunk by chunk, tiles x fastest; 2 = chunk
 *     by chunk, tiles y fastest; 3 = tile by tile (x fastest), every chunk
 *     of a tile together; 4 = as 3 with tiles y fastest; 0 (the default) = 3
 *     with walls, 1 without.
 *   x_offset: the tile grid of the single-cell shapes (0..5) is shifted by
 *     this many cells in x, wrapping around the periodic x axis (the tile
 *     starting at x_offset); -1 (the default) takes 32 (128 bytes) for FP32
 *     rows of at least 64 cells and 0 otherwise.  The paired shapes ignore
 *     it.
 * LBM_EINVAL for order outside 0..4 or x_offset outside -1..nx-1. */
lbm_status lbm_set_placement(lbm_ctx *ctx, int32_t order, int32_t x_offset);

/* Wall classes of a context with walls.  Bit i of a fluid cell's link word
 * says whether x - c_i is a wall cell (the bounce-back of Eq. 1's
 * streaming).  When the geometry's fluid cells show at most 256 distinct
 * words, lbm_init also stores one class byte per cell, the index of its word
 * in a table of those words, and the step, diagnostics and reverse marches
 * read that byte instead of the 4-byte word.  Returns the number of classes
 * in use (at least 2: the fluid cells away from walls, and the wall cells),
 * 0 when the context has no walls or its geometry has more distinct words
 * (the marches then read the words), -1 for a NULL context.  Host call. */
int32_t lbm_wall_classes(const lbm_ctx *ctx);

/* ---- Adjoint (reverse mode) of one step ---------------------------------
 * BGK (Eq. 2) and the regularized operator (Eqs. 10-11) in both readings:
 * the projection of the non-equilibrium momentum flux (LBM_REGULARIZED) and
 * that plus the energy flux (LBM_REGULARIZED3).  With a 16-bit storage form the step
 * differentiated is the FP32 step at the populations X_t decodes to (the
 * values its own pull reads): the storage rounding is passed through as the
 * identity, and the adjoint arrays are FP32 as for FP32 storage.
 * Let X_t be the stored state at t and L a scalar objective.  With
 * lam_{t+1} = dL/dX_{t+1} (device float, lbm_state_elems(nx, ny, nz,
 * LBM_FP32), in the layout of an FP32 stored state) this computes
 * lam_t = dL/dX_t, the transpose of one step at X_t (collision with the
 * Eq. 7 gather, then pull streaming with bounce-back).  It also ADDS to
 * dparams (device double[3]): dL/dG (for tied G^{AB} = G^{BA}), dL/dtau_A,
 * dL/dtau_B.  If drho0 (device double, 2*N) is not NULL it receives
 * sum_i w_i dL/df_i^a(x, t): at t = 0 this is dL/drho0 of lbm_init.
 *   x_t    device, a state buffer: X_t (may be a saved copy).
 *   work   device scratch; work_bytes must be at least
 *          lbm_adjoint_work_bytes(ctx) for the current tiling (else
 *          LBM_EINVAL): 24 bytes (three FP64 partial sums) per workgroup of
 *          the reverse march, and for 16-bit storage, from the next
 *          multiple of 256 bytes on, an FP32 copy of X_t in the FP32 layout
 *          (lbm_state_elems(nx, ny, nz, LBM_FP32) floats).  0 when the
 *          lattice does not fit the FP32 layout (the calls answer
 *          LBM_ENOTSUP).
 * lam_in and lam_out must not alias each other, x_t or work. */
size_t lbm_adjoint_work_bytes(const lbm_ctx *ctx);

/* Tiling of the reverse march (results do not depend on it, up to the
 * summation order of dparams): shape 0 = 64x8, 1 = 32x16, 2 = 32x8, 3 = 64x4
 * cells, or -1 (the default) for the automatic choice -- 32x8 or 64x4,
 * whichever pads the x-y plane less, 64x4 on a tie; zchunk = z planes per
 * workgroup, 0 =
 * the default, which minimises (rounds of 256 workgroups) x (zchunk + 5).
 * lbm_adjoint_work_bytes follows this setting.  Host-side setting;
 * LBM_EINVAL outside these ranges. */
lbm_status lbm_set_adjoint_tiling(lbm_ctx *ctx, int32_t shape, int32_t zchunk);
lbm_status lbm_adjoint_step(lbm_ctx *ctx, const void *x_t, const float *lam_in,
                            float *lam_out, void *work, size_t work_bytes,
                            double *dparams, double *drho0);

/* lbm_adjoint_step with the forward quantities of X_t read from fields (5*N
 * floats written by the lbm_step_fields call that advanced X_t) instead of
 * pulled again from X_t for the tile and its two-cell border: the same
 * results, bitwise, with less traffic.  FP32 storage only (LBM_ENOTSUP
 * otherwise).  fields must not alias x_t, lam_in or lam_out (LBM_EINVAL);
 * NULL fields: LBM_EINVAL. */
lbm_status lbm_adjoint_step_fields(lbm_ctx *ctx, const void *x_t, const float *fields,
                                   const float *lam_in, float *lam_out, void *work,
                                   size_t work_bytes, double *dparams, double *drho0);

/* dL/dX_T for an objective of the densities at time T: given
 * grad_rho (device float, 2*N, index a*N + c) = dL/drho^a(x, T), writes lam
 * (device float, an adjoint array: the FP32 state layout, whatever the
 * storage) = dL/dX_T.  Solid cells get zero. */
lbm_status lbm_adjoint_seed(lbm_ctx *ctx, const float *grad_rho, float *lam);

/* Plain device-to-device copy of `bytes` bytes (a multiple of 16; both
 * pointers 16-byte aligned, not overlapping) on `stream` (hipStream_t as
 * void*).  Not part of the method: it is the reference for the read + write
 * bandwidth the memory system delivers to a streaming kernel, against which
 * the step kernel's bandwidth is compared. */
lbm_status lbm_stream_copy(const void *src, void *dst, size_t bytes, void *stream);

/* Copies the nx*ny cells of every population plane of a stored state `src`
 * to `dst` (device, lbm_state_elems(nx, ny, nz, storage) elements each,
 * distinct; padding not written) with the memory pattern of the step: one
 * workgroup per 128 x 4 column tile marching its chunk of z planes, 38 loads
 * then 38 stores per cell and plane, on the context's stream.  Not part of
 * the method: it moves exactly the step's algorithmic bytes with no
 * arithmetic, so its rate is the ceiling of the step's access pattern. */
lbm_status lbm_march_copy(lbm_ctx *ctx, const void *src, void *dst);

/* Frees the context and what the library allocated; NULL is a no-op.
 * Waits for the context's stream first. */
lbm_status lbm_destroy(lbm_ctx *ctx);

#ifdef __cplusplus
}
#endif

#endif /* LBM_H */
