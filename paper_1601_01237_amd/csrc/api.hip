// C ABI of liblbm.so (declared in include/lbm.h): argument checks, context
// bookkeeping and kernel launches on the caller's stream.

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdlib>
#include <mutex>
#include <new>
#include <unordered_map>
#include <vector>

#include "lbm.h"
#include "launch.h"

using namespace lbm;

struct lbm_ctx {
  lbm_params p;
  Grid g;
  Phys ph;
  Storage storage;
  void* buf[2];
  uint32_t* links;     // owned; null without walls
  const uint8_t* cls;  // wall classes (in the links allocation), or null
  const uint32_t* ltab;  // link word of each class (in the links allocation)
  int classes;         // classes in use (0: none)
  hipStream_t stream;
  int64_t t;
  int tile, zchunk;    // tiling of the step kernel
  double* partials;    // owned reduction scratch
  size_t partials_cap; // doubles
  int device;          // HIP device current at lbm_init
  int adj_shape, adj_zchunk;  // tiling of the reverse march (-1 / 0: automatic)
  int order;           // block order of the step kernel (0: automatic)
  int xoff;            // x shift of the step kernel's tile grid (-1: automatic)
};

// Partial sums of lbm_moments_static: a fixed array in device memory, one
// copy per GPU, held until the process ends.  Sized for LBM_STATIC_BLOCKS
// workgroups of 16 FP64 partials each (1 MiB).  Host code never passes the
// name itself to a kernel (on the host it only stands for the symbol): it
// uses the device address looked up once per device by static_partials().
static __device__ __align__(256) double scratch[LBM_STATIC_BLOCKS * LBM_DIAG_LEN];

namespace {

constexpr int MAX_DEVICES = 64;
std::mutex scratch_mu;
double* scratch_ptr[MAX_DEVICES] = {};
hipError_t scratch_err[MAX_DEVICES] = {};
bool scratch_done[MAX_DEVICES] = {};

// Device address of `scratch` on `dev`, which must be the current device.
// Looked up on the first call for a device (lbm_init makes that call) and
// kept; returns null if the lookup failed.
double* static_partials(int dev) {
  if (dev < 0 || dev >= MAX_DEVICES) return nullptr;
  std::lock_guard<std::mutex> lock(scratch_mu);
  if (!scratch_done[dev]) {
    void* ptr = nullptr;
    scratch_err[dev] = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    scratch_ptr[dev] = scratch_err[dev] == hipSuccess ? static_cast<double*>(ptr) : nullptr;
    scratch_done[dev] = true;
  }
  return scratch_ptr[dev];
}

}  // namespace

// Supported layouts and sizes (defined with the layout entry points below).
static bool layout_of(int32_t nx, int32_t ny, int32_t storage, Layout* L);
static bool cells_fit(uint64_t n, size_t es);

namespace {

size_t elem_size(Storage s) { return s == Storage::F32 ? 4 : 2; }

lbm_status from_hip(hipError_t e) { return e == hipSuccess ? LBM_OK : LBM_EHIP; }

// Automatic block order: without walls an XCD takes whole rows of tiles of
// one z chunk (neighbouring tiles share their border rows in L2).  With walls
// the work of a chunk depends on the geometry (solid cells are skipped), so
// each XCD takes every chunk of a run of tiles, which keeps the XCDs evenly
// loaded (measured: 5% on the inclined channel, 2% slower on open boxes).
int default_order(const lbm_ctx* c) { return c->links ? ORDER_TILE_X : ORDER_PLANE_X; }
// Automatic x shift of the tile grid: 32 cells (128 bytes) for FP32 rows of
// at least 64 cells, else none.  Measured with the automatic tiles: 128^3
// 131.2 -> 129.1 us, 512^3 8.06 -> 7.92 ms, and with the tuned 64 x 12 tiles
// on the 384 x 192 x 192 inclined channel 0.858 -> 0.798 ms; shifts of 8 or
// 16 cells (rows no longer 128-byte aligned) were slower than none.
int default_xoff(const lbm_ctx* c, const Tiling& t) {
  if (pair_shape(t.tile) || c->storage != Storage::F32 || c->g.nx < 64) return 0;
  return 32;
}

// Step kernel: the selected tile shape (automatic: 128x4 without walls, 64x8
// with walls, the faster of the shapes measured on each); diagnostics: shape 0.
Tiling step_tiling(const lbm_ctx* c) {
  const bool open_box = c->links == nullptr;
  const int tile = c->tile >= 0 ? c->tile : auto_tile(c->g, !open_box, static_cast<int>(elem_size(c->storage)));
  Tiling t = make_tiling(c->g, tile, c->zchunk, open_box);
  // A small open FP32 box that would leave half the CUs idle takes 64 x 4
  // tiles instead (twice the workgroups of 64 x 8): 18-30% faster steps
  // measured from 16^3 to 64^3; from 72^3 on the grid fills the device.
  if (c->tile < 0 && open_box && c->storage == Storage::F32 && t.blocks > 0 && t.blocks <= 128)
    t = make_tiling(c->g, 4, c->zchunk, open_box);
  t.order = c->order > 0 ? c->order : default_order(c);
  t.xoff = c->xoff >= 0 ? c->xoff : default_xoff(c, t);
  return t;
}
Tiling aux_tiling(const lbm_ctx* c) {
  Tiling t = make_tiling(c->g, 0, 0);
  t.order = default_order(c);
  return t;
}
// The lattice in the FP32 layout: that of the adjoint arrays, and of the
// state itself with FP32 storage.  nz = 0 when the lattice does not fit it.
Grid fp32_grid(const lbm_ctx* c) {
  if (c->storage == Storage::F32) return c->g;
  Grid g = c->g;
  Layout L;
  if (!cells_fit(g.n, sizeof(float)) || !layout_of(g.nx, g.ny, LBM_FP32, &L)) {
    g.nz = 0;
    return g;
  }
  g.pstride = L.pstride;
  g.half = 0;
  g.brows = L.brows;
  g.zstride = static_cast<uint32_t>(L.zstride);
  return g;
}
Tiling adjoint_tiling(const lbm_ctx* c) {
  const Grid g = fp32_grid(c);
  Tiling t{};
  if (g.nz < 1) {
    t.blocks = -1;
    return t;
  }
  const int shape = c->adj_shape >= 0 ? c->adj_shape : adjoint_auto_shape(g, c->links != nullptr, c->ph.regularized);
  t = adjoint_march_tiling(g, shape, c->adj_zchunk);
  t.order = default_order(c);
  return t;
}

lbm_status ensure_partials(lbm_ctx* c, size_t need) {
  if (need <= c->partials_cap) return LBM_OK;
  if (c->partials) {
    // The previous buffer may still be read by work queued on the stream.
    if (hipStreamSynchronize(c->stream) != hipSuccess) return LBM_EHIP;
    (void)hipFree(c->partials);
    c->partials = nullptr;
    c->partials_cap = 0;
  }
  if (hipMalloc(reinterpret_cast<void**>(&c->partials), need * sizeof(double)) != hipSuccess) {
    c->partials = nullptr;
    return LBM_EHIP;
  }
  c->partials_cap = need;
  return LBM_OK;
}

}  // namespace

extern "C" {

int32_t lbm_version(void) { return 10000; }

lbm_status lbm_velocity_set(int32_t* c, double* w) {
  for (int i = 0; i < Q; ++i) {
    if (c) {
      c[3 * i + 0] = CX[i];
      c[3 * i + 1] = CY[i];
      c[3 * i + 2] = CZ[i];
    }
    if (w) w[i] = weight_d(i);
  }
  return LBM_OK;
}

const char* lbm_status_str(lbm_status s) {
  switch (s) {
    case LBM_OK: return "ok";
    case LBM_EINVAL: return "invalid argument";
    case LBM_EHIP: return "HIP runtime error";
    case LBM_ESTATE: return "invalid state";
    case LBM_EUNSTABLE: return "non-finite values (unstable run)";
    case LBM_ENOTSUP: return "not supported";
  }
  return "unknown status";
}

// One z plane of all 38 populations is addressed by a single buffer
// resource with 32-bit offsets: it must stay below 2 GiB.
static bool plane_block_fits(const Layout& L, size_t es) { return L.zstride * es < (1ull << 31); }

// Layout of a supported plane size, else false.
static bool layout_of(int32_t nx, int32_t ny, int32_t storage, Layout* L) {
  if (nx < 1 || ny < 1 || storage < LBM_FP32 || storage > LBM_BF16) return false;
  const size_t es = elem_size(static_cast<Storage>(storage));
  if (static_cast<uint64_t>(nx) * ny * es >= (1ull << 31)) return false;
  *L = state_layout(nx, ny, static_cast<int>(es));
  return plane_block_fits(*L, es);
}

// Cell indices are 32-bit inside the kernels, and one population array of N
// cells is addressed with 32-bit offsets.
static bool cells_fit(uint64_t n, size_t es) { return n * es < (1ull << 32) && n < (1ull << 31); }

int64_t lbm_plane_stride(int32_t nx, int32_t ny, int32_t storage) {
  Layout L;
  return layout_of(nx, ny, storage, &L) ? static_cast<int64_t>(L.pstride) : -1;
}

int32_t lbm_row_block(int32_t nx, int32_t ny, int32_t storage) {
  Layout L;
  return layout_of(nx, ny, storage, &L) ? static_cast<int32_t>(L.brows) : -1;
}

int32_t lbm_row_half(int32_t nx, int32_t storage, int32_t walls) {
  if (nx < 1 || storage < LBM_FP32 || storage > LBM_BF16) return -1;
  return (storage != LBM_FP32 && nx % 2 == 0 && !walls) ? nx / 2 : 0;
}

int64_t lbm_state_elems(int32_t nx, int32_t ny, int32_t nz, int32_t storage) {
  Layout L;
  if (!layout_of(nx, ny, storage, &L) || nz < 1) return -1;
  const uint64_t n = static_cast<uint64_t>(nx) * ny * nz;
  if (!cells_fit(n, elem_size(static_cast<Storage>(storage)))) return -1;
  return static_cast<int64_t>(nz) * static_cast<int64_t>(L.zstride);
}

// Wall classes of the link words (buffer.h): each cell's word (1 for a wall
// cell) replaced by its index in a table of the distinct words, when there
// are at most WALL_CLASSES of them.  Otherwise, or when the host cannot hold
// the N words, the context keeps no classes and the marches read the words.
static hipError_t build_wall_classes(lbm_ctx* c) {
  const uint64_t n = c->g.n;
  std::vector<uint32_t> words;
  std::vector<uint8_t> cls;
  try {
    words.resize(n);
    cls.resize(n);
  } catch (const std::bad_alloc&) {
    return hipSuccess;
  }
  hipError_t e = hipMemcpyAsync(words.data(), c->links, n * sizeof(uint32_t), hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return e;
  uint32_t table[WALL_CLASSES] = {0u, 1u};
  int classes = 2;
  std::unordered_map<uint32_t, int> index;
  for (uint64_t i = 0; i < n; ++i) {
    const uint32_t w = (words[i] & 1u) ? 1u : words[i];
    int k = static_cast<int>(w);  // 0: fluid away from walls, 1: wall cell
    if (w > 1u) {
      const auto it = index.find(w);
      if (it != index.end()) {
        k = it->second;
      } else {
        if (classes == WALL_CLASSES) return hipSuccess;
        k = classes++;
        table[k] = w;
        index.emplace(w, k);
      }
    }
    cls[i] = static_cast<uint8_t>(k);
  }
  uint32_t* tab = c->links + n;
  uint8_t* dcls = reinterpret_cast<uint8_t*>(tab + WALL_CLASSES);
  e = hipMemcpyAsync(tab, table, sizeof(table), hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(dcls, cls.data(), n, hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);  // the host arrays end here
  if (e != hipSuccess) return e;
  c->ltab = tab;
  c->cls = dcls;
  c->classes = classes;
  return hipSuccess;
}

lbm_status lbm_init(lbm_ctx** out, const lbm_params* p, void* buf_a, void* buf_b, const uint8_t* solid,
                    const double* rho0, void* stream) {
  if (!out) return LBM_EINVAL;
  *out = nullptr;
  if (!p || !buf_a || !buf_b || !rho0 || buf_a == buf_b) return LBM_EINVAL;
  if (p->nx < 1 || p->ny < 1 || p->nz < 1) return LBM_EINVAL;
  if (p->storage < LBM_FP32 || p->storage > LBM_BF16) return LBM_EINVAL;
  for (int a = 0; a < 2; ++a) {
    if (!(p->tau[a] > 0.5) || !std::isfinite(p->tau[a])) return LBM_EINVAL;
    if (!std::isfinite(p->rho_shift[a]) || !std::isfinite(p->rho_wall[a])) return LBM_EINVAL;
    for (int b = 0; b < 2; ++b)
      if (!std::isfinite(p->G[a][b])) return LBM_EINVAL;
  }
  if (p->G[0][0] != 0.0 || p->G[1][1] != 0.0) return LBM_ENOTSUP;
  if (p->collision != LBM_BGK && p->collision != LBM_REGULARIZED && p->collision != LBM_REGULARIZED3)
    return LBM_EINVAL;
  const uint64_t nxy = static_cast<uint64_t>(p->nx) * p->ny;
  const uint64_t n = nxy * p->nz;
  const Storage st = static_cast<Storage>(p->storage);
  Layout L;
  if (!cells_fit(n, elem_size(st)) || !layout_of(p->nx, p->ny, p->storage, &L)) return LBM_ENOTSUP;

  lbm_ctx* c = new (std::nothrow) lbm_ctx();
  if (!c) return LBM_EHIP;
  c->p = *p;
  // 16-bit rows with even nx and no walls are stored folded (two cells per
  // 32-bit word, stepped by the paired march).
  const uint32_t half = static_cast<uint32_t>(lbm_row_half(p->nx, p->storage, solid != nullptr));
  c->g = Grid{p->nx, p->ny, p->nz, static_cast<uint32_t>(nxy), n, L.pstride, half, L.brows,
               static_cast<uint32_t>(L.zstride)};
  for (int a = 0; a < 2; ++a) {
    c->ph.omega[a] = static_cast<float>(1.0 / p->tau[a]);
    c->ph.rho_wall[a] = static_cast<float>(p->rho_wall[a]);
    c->ph.shift[a] = st == Storage::F32 ? 0.0f : static_cast<float>(p->rho_shift[a]);
  }
  c->ph.regularized = p->collision == LBM_REGULARIZED3 ? 2 : (p->collision == LBM_REGULARIZED ? 1 : 0);
  c->ph.g_ab = static_cast<float>(p->G[0][1]);
  c->ph.g_ba = static_cast<float>(p->G[1][0]);
  c->storage = st;
  c->buf[0] = buf_a;
  c->buf[1] = buf_b;
  c->links = nullptr;
  c->cls = nullptr;
  c->ltab = nullptr;
  c->classes = 0;
  c->stream = static_cast<hipStream_t>(stream);
  c->t = 0;
  c->tile = -1;
  c->zchunk = 0;
  c->partials = nullptr;
  c->partials_cap = 0;
  c->adj_shape = -1;
  c->adj_zchunk = 0;
  c->order = 0;
  c->xoff = -1;
  c->device = -1;
  if (hipGetDevice(&c->device) != hipSuccess) {
    delete c;
    return LBM_EHIP;
  }
  // Device address of the fixed partial-sum array of lbm_moments_static on
  // this device (looked up once per device; a failed lookup only disables
  // that entry point).
  (void)static_partials(c->device);

  hipError_t e = hipSuccess;
  if (solid) {
    // link words of every cell, the class table, one class byte per cell
    const size_t bytes = n * sizeof(uint32_t) + WALL_CLASSES * sizeof(uint32_t) + n;
    if (hipMalloc(reinterpret_cast<void**>(&c->links), bytes) != hipSuccess) {
      delete c;
      return LBM_EHIP;
    }
    e = launch_links(c->g, solid, c->links, c->stream);
    if (e == hipSuccess) e = build_wall_classes(c);
  }
  // Both buffers get the rest state, so wall cells (never written by a step)
  // hold the same defined values in either time level.
  if (e == hipSuccess) e = launch_init(st, c->g, c->ph, c->links, rho0, buf_a, c->stream);
  if (e == hipSuccess) e = launch_init(st, c->g, c->ph, c->links, rho0, buf_b, c->stream);
  if (e != hipSuccess) {
    (void)hipStreamSynchronize(c->stream);
    if (c->links) (void)hipFree(c->links);
    delete c;
    return LBM_EHIP;
  }
  *out = c;
  return LBM_OK;
}

lbm_status lbm_step(lbm_ctx* c, int64_t n) {
  if (!c || n < 0) return LBM_EINVAL;
  const Tiling t = step_tiling(c);
  if (t.blocks <= 0) return LBM_ENOTSUP;
  for (int64_t k = 0; k < n; ++k) {
    MarchIO io;
    io.src = c->buf[c->t & 1];
    io.dst = c->buf[(c->t + 1) & 1];
    io.links = c->links;
    io.cls = c->cls;
    io.ltab = c->ltab;
    const hipError_t e = launch_march(c->storage, Mode::Step, c->g, c->ph, t, io, c->stream);
    if (e != hipSuccess) return LBM_EHIP;
    ++c->t;
  }
  return LBM_OK;
}

lbm_status lbm_step_fields(lbm_ctx* c, float* fields) {
  if (!c || !fields) return LBM_EINVAL;
  if (static_cast<void*>(fields) == c->buf[0] || static_cast<void*>(fields) == c->buf[1]) return LBM_EINVAL;
  if (c->storage != Storage::F32) return LBM_ENOTSUP;
  const Tiling t = step_tiling(c);
  if (t.blocks <= 0) return LBM_ENOTSUP;
  MarchIO io;
  io.src = c->buf[c->t & 1];
  io.dst = c->buf[(c->t + 1) & 1];
  io.links = c->links;
  io.cls = c->cls;
  io.ltab = c->ltab;
  io.fields = fields;
  const hipError_t e = launch_march(c->storage, Mode::StepFields, c->g, c->ph, t, io, c->stream);
  if (e != hipSuccess) return LBM_EHIP;
  ++c->t;
  return LBM_OK;
}

// The diagnostics march (shape 64 x 8) and its fixed-order reduction, with
// the per-workgroup partial sums in `partials` (t.blocks * 16 doubles).
static lbm_status moments_launch(lbm_ctx* c, const Tiling& t, double* partials, float* rho, float* u_f,
                                 double* diag, const lbm_diag_region* region) {
  MarchIO io;
  io.src = c->buf[c->t & 1];
  io.links = c->links;
  io.cls = c->cls;
  io.ltab = c->ltab;
  io.rho_out = rho;
  io.uf_out = u_f;
  io.partials = partials;  // written even without diag
  Region R;
  if (region) {
    R.cx = static_cast<float>(region->center[0]);
    R.cy = static_cast<float>(region->center[1]);
    R.cz = static_cast<float>(region->center[2]);
    R.r_in2 = static_cast<float>(region->r_in * region->r_in);
    R.r_out2 = static_cast<float>(region->r_out * region->r_out);
    R.thr = static_cast<float>(region->thr);
  } else {
    R.cx = 0.5f * c->g.nx;
    R.cy = 0.5f * c->g.ny;
    R.cz = 0.5f * c->g.nz;
    R.r_in2 = 0.0f;
    R.r_out2 = INFINITY;
    R.thr = 0.515f;
  }
  R.p_g = static_cast<float>(0.5 * (c->p.G[0][1] + c->p.G[1][0]));
  io.region = R;
  hipError_t e = launch_march(c->storage, Mode::Moments, c->g, c->ph, t, io, c->stream);
  if (e == hipSuccess && diag) e = launch_finalize(partials, t.blocks, LBM_DIAG_LEN, LBM_DIAG_MAX_UF, diag, false, c->stream);
  return from_hip(e);
}

lbm_status lbm_moments(lbm_ctx* c, float* rho, float* u_f, double* diag, const lbm_diag_region* region) {
  if (!c) return LBM_EINVAL;
  const Tiling t = aux_tiling(c);
  if (t.blocks <= 0) return LBM_ENOTSUP;
  const lbm_status s = ensure_partials(c, static_cast<size_t>(t.blocks) * LBM_DIAG_LEN);
  if (s != LBM_OK) return s;
  return moments_launch(c, t, c->partials, rho, u_f, diag, region);
}

lbm_status lbm_moments_static(lbm_ctx* c, float* rho, float* u_f, double* diag, const lbm_diag_region* region) {
  if (!c) return LBM_EINVAL;
  // The tiling of lbm_moments, so the two give bitwise equal results.
  const Tiling t = aux_tiling(c);
  if (t.blocks <= 0 || t.blocks > LBM_STATIC_BLOCKS) return LBM_ENOTSUP;
  double* partials = static_partials(c->device);
  if (!partials) return LBM_EHIP;
  return moments_launch(c, t, partials, rho, u_f, diag, region);
}

lbm_status lbm_get_populations(lbm_ctx* c, float* f) {
  if (!c || !f) return LBM_EINVAL;
  return from_hip(launch_get_populations(c->storage, c->g, c->ph, c->links, c->buf[c->t & 1], f, c->stream));
}

lbm_status lbm_set_populations(lbm_ctx* c, const float* f) {
  if (!c || !f) return LBM_EINVAL;
  return from_hip(launch_set_populations(c->storage, c->g, c->ph, c->links, f, c->buf[c->t & 1], c->stream));
}

int64_t lbm_time(const lbm_ctx* c) { return c ? c->t : -1; }

lbm_status lbm_set_time(lbm_ctx* c, int64_t t) {
  if (!c || t < 0) return LBM_EINVAL;
  c->t = t;
  return LBM_OK;
}

lbm_status lbm_set_tiling(lbm_ctx* c, int32_t tile, int32_t zchunk) {
  if (!c || tile < -1 || tile >= TILE_SHAPES || zchunk < 0) return LBM_EINVAL;
  // The paired march needs folded 16-bit rows and no walls.
  if (pair_shape(tile) && (c->g.half == 0 || c->links != nullptr)) return LBM_EINVAL;
  c->tile = tile;
  c->zchunk = zchunk;
  return LBM_OK;
}

lbm_status lbm_set_placement(lbm_ctx* c, int32_t order, int32_t x_offset) {
  if (!c || order < 0 || order > BLOCK_ORDERS || x_offset < -1 || x_offset >= c->g.nx) return LBM_EINVAL;
  c->order = order;
  c->xoff = x_offset;
  return LBM_OK;
}

int32_t lbm_wall_classes(const lbm_ctx* c) { return c ? c->classes : -1; }

lbm_status lbm_set_adjoint_tiling(lbm_ctx* c, int32_t shape, int32_t zchunk) {
  if (!c || shape < -1 || shape >= ADJOINT_SHAPES || zchunk < 0) return LBM_EINVAL;
  c->adj_shape = shape;
  c->adj_zchunk = zchunk;
  return LBM_OK;
}

// Workspace of one reverse step: the FP64 partial sums (dL/dG, dL/dtau_A,
// dL/dtau_B) of each workgroup of the reverse march.
static size_t adjoint_work(const Tiling& t) {
  return static_cast<size_t>(t.blocks > 0 ? t.blocks : 0) * 3 * sizeof(double);
}

// Workspace bytes of the partial sums, rounded up to 256 bytes: for 16-bit
// storage the FP32 copy of X_t follows them.
static size_t adjoint_partials_span(const Tiling& t) { return (adjoint_work(t) + 255) / 256 * 256; }

size_t lbm_adjoint_work_bytes(const lbm_ctx* c) {
  if (!c) return 0;
  const Tiling t = adjoint_tiling(c);
  if (c->storage == Storage::F32) return adjoint_work(t);
  const Grid g = fp32_grid(c);
  if (g.nz < 1) return 0;
  return adjoint_partials_span(t) + static_cast<size_t>(g.nz) * g.zstride * sizeof(float);
}

static lbm_status adjoint_step(lbm_ctx* c, const void* x_t, const float* fields, const float* lam_in,
                               float* lam_out, void* work, size_t work_bytes, double* dparams, double* drho0) {
  if (!c || !x_t || !lam_in || !lam_out || !work || !dparams) return LBM_EINVAL;
  if (work_bytes < lbm_adjoint_work_bytes(c)) return LBM_EINVAL;
  if (lam_in == lam_out || static_cast<const void*>(lam_in) == x_t || static_cast<const void*>(lam_out) == x_t)
    return LBM_EINVAL;
  if (work == x_t || work == static_cast<const void*>(lam_in) || work == static_cast<void*>(lam_out))
    return LBM_EINVAL;
  if (fields && (static_cast<const void*>(fields) == x_t || fields == lam_in || fields == lam_out))
    return LBM_EINVAL;
  if (fields && c->storage != Storage::F32) return LBM_ENOTSUP;
  const Tiling t = adjoint_tiling(c);
  if (t.blocks <= 0) return LBM_ENOTSUP;
  const Grid g = fp32_grid(c);
  hipError_t e = hipSuccess;
  const void* xs = x_t;
  if (c->storage != Storage::F32) {
    // the reverse step of the FP32 step at the populations X_t decodes to
    float* wide = reinterpret_cast<float*>(static_cast<char*>(work) + adjoint_partials_span(t));
    e = launch_widen_state(c->storage, c->g, g, c->ph, c->links, x_t, wide, c->stream);
    if (e != hipSuccess) return from_hip(e);
    xs = wide;
  }
  AdjointIO io;
  io.x_t = xs;
  io.links = c->links;
  io.cls = c->cls;
  io.ltab = c->ltab;
  io.lam_in = lam_in;
  io.lam_out = lam_out;
  io.partials = static_cast<double*>(work);
  io.drho0 = drho0;
  io.fields = fields;
  e = launch_adjoint_march(g, c->ph, t, io, c->stream);
  if (e == hipSuccess) e = launch_finalize(io.partials, t.blocks, 3, -1, dparams, true, c->stream);
  return from_hip(e);
}

lbm_status lbm_adjoint_step(lbm_ctx* c, const void* x_t, const float* lam_in, float* lam_out, void* work,
                            size_t work_bytes, double* dparams, double* drho0) {
  return adjoint_step(c, x_t, nullptr, lam_in, lam_out, work, work_bytes, dparams, drho0);
}

lbm_status lbm_adjoint_step_fields(lbm_ctx* c, const void* x_t, const float* fields, const float* lam_in,
                                   float* lam_out, void* work, size_t work_bytes, double* dparams, double* drho0) {
  if (!fields) return LBM_EINVAL;
  return adjoint_step(c, x_t, fields, lam_in, lam_out, work, work_bytes, dparams, drho0);
}

lbm_status lbm_adjoint_seed(lbm_ctx* c, const float* grad_rho, float* lam) {
  if (!c || !grad_rho || !lam) return LBM_EINVAL;
  const Grid g = fp32_grid(c);  // the adjoint arrays' layout, whatever the storage
  if (g.nz < 1) return LBM_ENOTSUP;
  return from_hip(launch_adjoint_seed(g, c->links, grad_rho, lam, c->stream));
}

lbm_status lbm_stream_copy(const void* src, void* dst, size_t bytes, void* stream) {
  if (!src || !dst || src == dst || bytes == 0 || bytes % 16 != 0) return LBM_EINVAL;
  if ((reinterpret_cast<uintptr_t>(src) | reinterpret_cast<uintptr_t>(dst)) % 16 != 0) return LBM_EINVAL;
  return from_hip(launch_stream_copy(src, dst, bytes, static_cast<hipStream_t>(stream)));
}

lbm_status lbm_march_copy(lbm_ctx* c, const void* src, void* dst) {
  if (!c || !src || !dst || src == dst) return LBM_EINVAL;
  return from_hip(launch_march_copy(c->storage, c->g, src, dst, c->stream));
}

lbm_status lbm_destroy(lbm_ctx* c) {
  if (!c) return LBM_OK;
  const hipError_t e = hipStreamSynchronize(c->stream);
  if (c->links) (void)hipFree(c->links);
  if (c->partials) (void)hipFree(c->partials);
  delete c;
  return from_hip(e);
}

}  // extern "C"
