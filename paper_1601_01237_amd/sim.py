"""``Sim``: one two-component D3Q19 run on one GPU through the C ABI.

PyTorch only owns the device memory and supplies the stream; the step,
moments, population transfers and adjoint run in liblbm.so.
"""

from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import _lib

STORAGE = {"fp32": (_lib.FP32, torch.float32), "fp16": (_lib.FP16, torch.float16),
           "bf16": (_lib.BF16, torch.bfloat16)}

DIAG_NAMES = ["mass_a", "mass_b", "mom_x", "mom_y", "mom_z", "max_uf", "nonfinite", "n_fluid",
              "p_in_sum", "n_in", "p_out_sum", "n_out", "n_thr", "sdx_thr", "sdy_thr", "sdz_thr"]

Q = _lib.Q


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def layout_rows(storage):
    """Rows of one row block of the state layout (lbm.h): the 38 population
    rows, and for the 16-bit forms the residual rows of the two rest
    populations."""
    return 2 * Q + (0 if storage == "fp32" else 2)


def coupling_matrix(G):
    """G as a 2x2 matrix; a scalar means G^{AB} = G^{BA} = G and G^{aa} = 0."""
    if np.isscalar(G):
        return ((0.0, float(G)), (float(G), 0.0))
    return tuple(tuple(float(v) for v in row) for row in G)


class Sim:
    """A context of liblbm plus the two state buffers it ping-pongs between.

    Parameters
    ----------
    rho0 : array (2, nz, ny, nx)  initial species densities (float64).
    tau : (tau_A, tau_B) relaxation times (Eq. 2).
    G : scalar or 2x2 coupling of Eq. (7) (paper sign: repulsion < 0).
    storage : "fp32", "fp16" or "bf16" (16-bit forms store f - w rho_shift).
    rho_shift : per-species shift of the 16-bit forms; default: mean density.
    solid : optional bool array (nz, ny, nx) of wall cells.
    rho_wall : wall potential rho_s^a (Sec. 4).
    collision : "bgk" (Eq. 2), "regularized" (Eqs. 10-11 of Sec. 3, momentum
        flux) or "regularized3" (the same filter keeping the energy flux).
    tile, zchunk : tiling of the step kernel (results do not depend on it).
    """

    COLLISIONS = {"bgk": _lib.BGK, "regularized": _lib.REGULARIZED, "regularized3": _lib.REGULARIZED3}

    def __init__(self, rho0, tau=(1.0, 1.0), G=-1.0, storage="fp32", rho_shift=None,
                 solid=None, rho_wall=(0.0, 0.0), device="cuda:0", tile=None, zchunk=None,
                 collision="bgk"):
        self.lib = _lib.load()
        self.device = torch.device(device)
        rho0 = torch.as_tensor(np.asarray(rho0, dtype=np.float64))
        if rho0.ndim != 4 or rho0.shape[0] != 2:
            raise ValueError("rho0 must have shape (2, nz, ny, nx)")
        self.shape = tuple(int(v) for v in rho0.shape[1:])
        nz, ny, nx = self.shape
        self.n = nx * ny * nz
        self.storage = storage
        code, self.dtype = STORAGE[storage]
        fluid = np.ones(self.shape, bool) if solid is None else ~np.asarray(solid, bool)
        if rho_shift is None:
            r = rho0.numpy()
            if storage == "fp32" or not fluid.any():
                rho_shift = (0.0, 0.0)
            else:
                rho_shift = tuple(float(r[a][fluid].mean()) for a in range(2))
        self.rho_shift = tuple(float(v) for v in rho_shift)
        self.G = coupling_matrix(G)
        self.tau = tuple(float(t) for t in (tau if not np.isscalar(tau) else (tau, tau)))
        self.rho_wall = tuple(float(v) for v in rho_wall)

        p = _lib.Params()
        p.nx, p.ny, p.nz = nx, ny, nz
        p.storage = code
        p.tau[0], p.tau[1] = self.tau
        for a in range(2):
            for b in range(2):
                p.G[a][b] = self.G[a][b]
        p.rho_shift[0], p.rho_shift[1] = self.rho_shift
        p.rho_wall[0], p.rho_wall[1] = self.rho_wall
        if collision not in self.COLLISIONS:
            raise ValueError(f"collision must be one of {sorted(self.COLLISIONS)}")
        self.collision = collision
        p.collision = self.COLLISIONS[collision]
        self.params = p

        # Row-blocked state layout (lbm.h): (y rows per block, population
        # stride, rows of population data per block: 38, plus the two residual
        # rows of the rest populations in the 16-bit forms).
        self.pstride = int(self.lib.lbm_plane_stride(nx, ny, code))
        self.layout = (int(self.lib.lbm_row_block(nx, ny, code)), self.pstride, layout_rows(storage))
        self.state_elems = int(self.lib.lbm_state_elems(nx, ny, nz, code))
        self.lam_layout = (int(self.lib.lbm_row_block(nx, ny, _lib.FP32)),
                           int(self.lib.lbm_plane_stride(nx, ny, _lib.FP32)), layout_rows("fp32"))
        self.lam_elems = int(self.lib.lbm_state_elems(nx, ny, nz, _lib.FP32))
        self.row_half = int(self.lib.lbm_row_half(nx, code, int(solid is not None)))
        # (the adjoint arrays are FP32, in the FP32 layout whatever the storage)
        if min(self.pstride, *self.layout, self.state_elems, self.row_half) < 0:
            raise ValueError(f"grid {self.shape} is not supported")

        with torch.cuda.device(self.device):
            # Row position of cell x in the stored state (folded 16-bit rows, lbm.h).
            x = torch.arange(nx, device=self.device)
            h = self.row_half
            self.x_pos = torch.where(x < h, 2 * x, 2 * (x - h) + 1) if h else x
            self.stream = torch.cuda.current_stream(self.device)
            # zeroed so that the padding between planes holds defined values
            self.bufs = [torch.zeros(self.state_elems, dtype=self.dtype, device=self.device) for _ in range(2)]
            self.rho0_dev = rho0.to(self.device).contiguous()
            self.solid_dev = None
            if solid is not None:
                self.solid_dev = torch.as_tensor(np.asarray(solid, dtype=np.uint8)).to(self.device).contiguous()
            ctx = C.c_void_p()
            _lib.check("lbm_init", self.lib.lbm_init(
                C.byref(ctx), C.byref(p), _ptr(self.bufs[0]), _ptr(self.bufs[1]),
                _ptr(self.solid_dev), _ptr(self.rho0_dev), C.c_void_p(self.stream.cuda_stream)))
        self.ctx = ctx
        self.tiling = (-1, 0)
        if tile is not None or zchunk is not None:
            self.set_tiling(-1 if tile is None else tile, zchunk or 0)

    # -- lifetime --------------------------------------------------------------
    def close(self):
        if getattr(self, "ctx", None):
            _lib.check("lbm_destroy", self.lib.lbm_destroy(self.ctx))
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- stepping --------------------------------------------------------------
    @property
    def t(self):
        return int(self.lib.lbm_time(self.ctx))

    def set_time(self, t):
        _lib.check("lbm_set_time", self.lib.lbm_set_time(self.ctx, int(t)))

    def step(self, n=1):
        _lib.check("lbm_step", self.lib.lbm_step(self.ctx, int(n)))

    def step_fields(self, fields=None):
        """One step that also writes rho~^A, rho~^B, u_x, u_y, u_z of the pull
        it collides into ``fields`` (float32, 5 N, on the device; allocated
        when None) and returns it: what the reverse step at this time level
        reads instead of pulling the state again (lbm_step_fields)."""
        import torch
        if fields is None:
            fields = torch.empty(5 * self.n, dtype=torch.float32, device=self.device)
        _lib.check("lbm_step_fields", self.lib.lbm_step_fields(self.ctx, _ptr(fields)))
        return fields

    def run(self, n, check_every=0):
        """Advance n steps.  With check_every > 0, read the diagnostics every
        check_every steps and after the last one, and raise LBMError with
        code LBM_EUNSTABLE (-4) at the first time level that holds a
        non-finite density or velocity; the state of that time level is kept
        (restore a checkpoint to recover)."""
        n = int(n)
        if check_every <= 0:
            self.step(n)
            return
        done = 0
        while done < n:
            k = min(int(check_every), n - done)
            self.step(k)
            done += k
            self.check_finite()

    def check_finite(self):
        """Raise LBMError(LBM_EUNSTABLE) if the current state holds a
        non-finite density or velocity on any fluid cell."""
        _, _, d = self.moments(want_fields=False)
        if d["nonfinite"] > 0:
            raise _lib.LBMError(f"lbm_step (t = {self.t}, {int(d['nonfinite'])} cells)", _lib.EUNSTABLE)

    def set_tiling(self, tile=-1, zchunk=0):
        """Tile shape of the step kernel (-1 = automatic, 0..9, see lbm_set_tiling) and z planes per workgroup."""
        _lib.check("lbm_set_tiling", self.lib.lbm_set_tiling(self.ctx, int(tile), int(zchunk)))
        self.tiling = (int(tile), int(zchunk))

    def set_placement(self, order=0, x_offset=-1):
        """Placement of the step kernel's workgroups: their order over (z chunk, tile) (0 = automatic,
        1..4) and the x shift of the tile grid (-1 = automatic); see lbm_set_placement."""
        _lib.check("lbm_set_placement", self.lib.lbm_set_placement(self.ctx, int(order), int(x_offset)))

    def wall_classes(self):
        """Number of one-byte wall classes the marches read (0: they read the 4-byte link words;
        see lbm_wall_classes)."""
        return int(self.lib.lbm_wall_classes(self.ctx))

    def set_adjoint_tiling(self, shape=-1, zchunk=0):
        """Tile shape of the reverse march (-1 = automatic, 0..3, see
        lbm_set_adjoint_tiling) and z planes per workgroup (0 = default)."""
        _lib.check("lbm_set_adjoint_tiling", self.lib.lbm_set_adjoint_tiling(self.ctx, int(shape), int(zchunk)))

    def tune(self, zchunks=(0, 8, 12, 16, 24, 32, 48, 64), tiles=(-1,), steps=None, placements=((0, -1),)):
        """Time the step for every (tile shape, z chunk, placement) of
        ``tiles`` x ``zchunks`` x ``placements`` (tile -1 = the library's
        automatic shape, zchunk 0 = its default chunk, placement (0, -1) = its
        default order and x shift; see lbm_set_tiling and lbm_set_placement)
        and keep the fastest.  The state and time level are restored
        afterwards (bitwise: every tiling computes the same step), so tuning
        can precede any run.  Shapes the context cannot run (pair shapes on
        unfolded rows, for instance) are skipped.  Returns (tile, zchunk,
        {(tile, zchunk[, placement]): ms per step}); the keys carry the
        placement only when more than one is tried, and the chosen placement
        stays set."""
        import torch
        nz = self.shape[0]
        cands = [z for z in dict.fromkeys(int(z) for z in zchunks) if z <= nz]
        place_list = list(dict.fromkeys((int(o), int(x)) for o, x in placements))
        n = int(steps) if steps else max(2, min(20, int(4e8 // self.n)))
        ckpt = self.checkpoint()

        def timed(k):
            start = torch.cuda.Event(enable_timing=True)
            end = torch.cuda.Event(enable_timing=True)
            start.record(self.stream)
            self.step(k)
            end.record(self.stream)
            end.synchronize()
            return start.elapsed_time(end)

        # Bring the device to its working clocks first (about 50 ms of steps):
        # the first candidate would otherwise pay for the ramp.
        spent = 0.0
        while spent < 50.0:
            spent += timed(n)
        times = {}
        for place in place_list:
            self.set_placement(*place)
            for tile in dict.fromkeys(int(t) for t in tiles):
                for z in cands:
                    try:
                        self.set_tiling(tile, z)
                    except _lib.LBMError:
                        break
                    self.step(1)
                    key = (tile, z, place) if len(place_list) > 1 else (tile, z)
                    times[key] = min(timed(n), timed(n)) / n  # best of two
        self.restore(ckpt)
        if not times:
            raise ValueError("no tiling of the candidates runs on this grid")
        best = min(times, key=times.get)
        self.set_tiling(best[0], best[1])
        self.set_placement(*(best[2] if len(best) > 2 else place_list[0]))
        return best[0], best[1], times

    @property
    def state(self):
        """The stored (post-collision) buffer of the current time level."""
        return self.bufs[self.t & 1]

    def plane_view(self, flat, layout=None):
        """(nz, nyb, 2, 19, B, nx) view of the population rows of a flat
        state-layout buffer: z plane, row block, species, population, row in
        the block, row position (see :attr:`x_pos`).  Rows past ny in the last
        block are padding."""
        nz, ny, nx = self.shape
        b, ps, rows = self.layout if layout is None else layout
        nyb = -(-ny // b)
        v = flat.view(nz, nyb, rows, ps)[:, :, : 2 * Q]
        return v.unflatten(2, (2, Q))[..., : b * nx].unflatten(-1, (b, nx))

    def residual_view(self, flat, layout=None):
        """(nz, nyb, 2, B, nx) view of the residual rows of the rest
        populations (16-bit forms; lbm.h): the stored rest population of
        species a reads back as its value in the population row plus this."""
        nz, ny, nx = self.shape
        b, ps, rows = self.layout if layout is None else layout
        if rows == 2 * Q:
            raise ValueError("this layout has no residual rows")
        nyb = -(-ny // b)
        return flat.view(nz, nyb, rows, ps)[:, :, 2 * Q:][..., : b * nx].unflatten(-1, (b, nx))

    def live_mask(self, layout=None, dtype=None):
        """Boolean flat mask of the elements of a state-layout buffer that hold
        a population value or a residual (not padding)."""
        b, ps, rows = self.layout if layout is None else layout
        nz, ny, nx = self.shape
        nyb = -(-ny // b)
        m = torch.zeros(nz * nyb * rows * ps, dtype=torch.bool, device=self.device)
        v = m.view(nz, nyb, rows, ps)[..., : b * nx].unflatten(-1, (b, nx))
        for yb in range(nyb):
            v[:, yb, :, : min(b, ny - yb * b)] = True
        return m

    def _row_order(self, flat):
        # the stored state is folded for 16-bit rows; adjoint arrays (FP32) never are
        return self.row_half and flat.dtype != torch.float32

    def cells(self, flat, z, y, x, layout=None):
        """Values (..., 2, 19) of a state-layout buffer at integer cell
        coordinates z, y, x (tensors of one shape, on the buffer's device).
        In the 16-bit forms the rest population's residual is separate
        (:meth:`cells_residual`)."""
        b = (self.layout if layout is None else layout)[0]
        if self._row_order(flat):
            x = self.x_pos.to(flat.device)[x]
        v = self.plane_view(flat, layout)
        return v[z, torch.div(y, b, rounding_mode="floor"), :, :, y % b, x]

    def cells_residual(self, flat, z, y, x, layout=None):
        """Residuals (..., 2) of the rest populations at cells z, y, x (16-bit forms)."""
        b = (self.layout if layout is None else layout)[0]
        if self._row_order(flat):
            x = self.x_pos.to(flat.device)[x]
        v = self.residual_view(flat, layout)
        return v[z, torch.div(y, b, rounding_mode="floor"), :, y % b, x]

    def to_state_layout(self, f, layout=None, elems=None):
        """(2, 19, nz, ny, nx) array -> new flat state-layout buffer (zero padding
        and, in the 16-bit forms, zero residual rows)."""
        nz, ny, nx = self.shape
        lay = self.layout if layout is None else layout
        b = lay[0]
        nyb = -(-ny // b)
        n = self.state_elems if elems is None else elems
        out = torch.zeros(n, dtype=f.dtype, device=f.device)
        rows = torch.zeros((2, Q, nz, nyb * b, nx), dtype=f.dtype, device=f.device)
        src = f.reshape(2, Q, nz, ny, nx)
        if self._row_order(out):
            rows[:, :, :, :ny, self.x_pos.to(f.device)] = src
        else:
            rows[:, :, :, :ny] = src
        self.plane_view(out, lay).copy_(rows.view(2, Q, nz, nyb, b, nx).permute(2, 3, 0, 1, 4, 5))
        return out

    def from_state_layout(self, flat, layout=None):
        """Flat state-layout buffer -> (2, 19, nz, ny, nx) contiguous copy of the
        population rows (cell order; 16-bit residual rows not included)."""
        nz, ny, nx = self.shape
        v = self.plane_view(flat, layout)                   # (nz, nyb, 2, Q, b, nx)
        rows = v.permute(2, 3, 0, 1, 4, 5).reshape(2, Q, nz, -1, nx)[:, :, :, :ny]
        if self._row_order(flat):
            rows = rows[..., self.x_pos.to(flat.device)]
        return rows.contiguous()

    # -- observables -------------------------------------------------------------
    def moments(self, region=None, want_fields=True):
        """(rho (2,nz,ny,nx), u_F (3,nz,ny,nx), diag dict) at the current time."""
        nz, ny, nx = self.shape
        rho = uf = None
        if want_fields:
            rho = torch.empty(2 * self.n, dtype=torch.float32, device=self.device)
            uf = torch.empty(3 * self.n, dtype=torch.float32, device=self.device)
        diag = torch.empty(_lib.DIAG_LEN, dtype=torch.float64, device=self.device)
        reg = None
        if region is not None:
            reg = _lib.DiagRegion()
            c = region.get("center", (nx / 2.0, ny / 2.0, nz / 2.0))
            reg.center[0], reg.center[1], reg.center[2] = c
            reg.r_in = region.get("r_in", 0.0)
            reg.r_out = region.get("r_out", 1e30)
            reg.thr = region.get("thr", 0.515)
        _lib.check("lbm_moments", self.lib.lbm_moments(
            self.ctx, _ptr(rho), _ptr(uf), _ptr(diag), C.byref(reg) if reg is not None else None))
        d = diag.cpu().numpy()
        out = dict(zip(DIAG_NAMES, d.tolist()))
        out["vector"] = d
        if want_fields:
            return rho.view(2, nz, ny, nx), uf.view(3, nz, ny, nx), out
        return None, None, out

    def populations(self):
        """Pre-collision populations f_i^a(x, t) as FP32 (2, 19, nz, ny, nx)."""
        f = torch.empty(2 * Q * self.n, dtype=torch.float32, device=self.device)
        _lib.check("lbm_get_populations", self.lib.lbm_get_populations(self.ctx, _ptr(f)))
        return f.view(2, Q, *self.shape)

    def set_populations(self, f):
        f = torch.as_tensor(f, dtype=torch.float32).to(self.device).contiguous()
        if f.numel() != 2 * Q * self.n:
            raise ValueError("populations must have 2*19*N elements")
        _lib.check("lbm_set_populations", self.lib.lbm_set_populations(self.ctx, _ptr(f)))
        self.stream.synchronize()

    # -- checkpoint / resume -----------------------------------------------------
    def checkpoint(self):
        """Copy of (stored state, t) that :meth:`restore` can put back."""
        return self.state.clone(), self.t

    def restore(self, ckpt):
        buf, t = ckpt
        self.bufs[t & 1].copy_(buf)
        self.set_time(t)
