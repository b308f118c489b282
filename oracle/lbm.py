"""FP64 CPU oracle: two-component D3Q19 lattice Boltzmann step (test infrastructure).

This module is test infrastructure.  Only ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py`` may import it; the HIP library never
calls it and shares no code, table or helper with it.

It is a plain, slow, obviously correct NumPy restatement of Sec. 2 of
Otomo et al., "Studies of accurate multi-component lattice Boltzmann models on
benchmark cases required for engineering applications" (arXiv 1601.01237):

* Eq. (1)  per-species lattice Boltzmann equation (push form, dt = dx = 1);
* Eq. (2)  BGK collision with relaxation time tau_alpha;
* Eq. (3)  third-order equilibrium, lattice temperature T0 = 1/3;
* Eqs. (4)-(6) species density, mixture density, mixture velocity;
* Eq. (7)  Shan-Chen inter-component force, G^{aa} = 0 (Sec. 2);
* Eqs. (10)-(11) regularized collision of Sec. 3 (Hermite projection of the
  non-equilibrium part onto the momentum flux, optionally plus the energy
  flux; a reading: see regularized_neq);
* Eqs. (8)-(9) force velocity u_F = u + g/2 and g = sum_a g^a rho^a / rho,
  with g^a = sum_b F^{ab} / rho^a;
* Sec. 4 pointwise (halfway) bounce-back wall and the pointwise wall
  potential rho_s^a used in place of the density of a solid neighbour.

Readings where the paper is silent (each listed in the design notes):

* weights of D3Q19 (called "isotropic" in Sec. 2, values not printed): 1/3 for
  the rest particle, 1/18 for the 6 face and 1/36 for the 12 edge neighbours --
  the only choice with sum w = 1, sum w c c = T0 I and fourth-order isotropy;
* forcing term (Sec. 2 delegates it to a citation): exact-difference form
  F_i^a = f_i^eq(rho^a, u + g^a) - f_i^eq(rho^a, u), built from Eq. (3) only;
  it adds no mass and exactly rho^a g^a momentum, so the mean of the pre- and
  post-collision mixture velocity is u + g/2 as in Eq. (8);
* a solid neighbour contributes rho_s^b to the Eq. (7) sum (Sec. 4, pointwise
  wall potential); solid cells carry no populations.

State convention: ``f`` has shape ``(2, 19, nz, ny, nx)`` and holds the
pre-collision populations f_i^a(x, t) (left-hand side of Eq. (1) at integer
t).  Every function works for float64 and for complex128 (complex-step
derivatives), so nothing here takes abs, max or a branch on a value.
"""

from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

# Lattice temperature, Sec. 2 after Eq. (3).
T0 = 1.0 / 3.0

# D3Q19 velocities (c_x, c_y, c_z): rest, 6 faces, 12 edges; opposite
# directions sit next to each other (1<->2, 3<->4, ...).
C = np.array([
    [0, 0, 0],
    [1, 0, 0], [-1, 0, 0],
    [0, 1, 0], [0, -1, 0],
    [0, 0, 1], [0, 0, -1],
    [1, 1, 0], [-1, -1, 0],
    [1, -1, 0], [-1, 1, 0],
    [1, 0, 1], [-1, 0, -1],
    [1, 0, -1], [-1, 0, 1],
    [0, 1, 1], [0, -1, -1],
    [0, 1, -1], [0, -1, 1],
], dtype=np.int64)
Q = 19

W = np.array([1.0 / 3.0] + [1.0 / 18.0] * 6 + [1.0 / 36.0] * 12, dtype=np.float64)

OPP = np.array([int(np.nonzero((C == -C[i]).all(axis=1))[0][0]) for i in range(Q)],
               dtype=np.int64)


@dataclass
class Params:
    """Physical parameters of one run (lattice units)."""

    tau: tuple = (1.0, 1.0)                     # tau_A, tau_B  (Eq. 2)
    G: tuple = ((0.0, -1.0), (-1.0, 0.0))       # G^{ab}       (Eq. 7), G^{aa} = 0
    rho_wall: tuple = (0.0, 0.0)                # rho_s^a      (Sec. 4)
    collision: str = "bgk"                      # "bgk" (Eq. 2), "regularized" or "regularized3" (Eqs. 10-11)
    extra: dict = field(default_factory=dict)


def at_offset(a, c):
    """Value of a periodic field at x + c: ``out[..., z, y, x] = a[..., z+cz, y+cy, x+cx]``."""
    cx, cy, cz = (int(v) for v in c)
    return np.roll(a, shift=(-cz, -cy, -cx), axis=(-3, -2, -1))


def fluid_mask(shape, solid):
    if solid is None:
        return np.ones(shape, dtype=bool)
    return ~np.asarray(solid, dtype=bool)


# ---------------------------------------------------------------------------
# Eqs. (4)-(6): moments
# ---------------------------------------------------------------------------

def species_density(f):
    """rho^a = sum_i f_i^a, Eq. (4).  Returns (2, nz, ny, nx)."""
    return f.sum(axis=1)


def mixture_density(rho_s):
    """rho = sum_a rho^a, Eq. (5)."""
    return rho_s[0] + rho_s[1]


def mixture_velocity(f, rho, fluid):
    """u = sum_a sum_i c_i f_i^a / rho, Eq. (6).  Zero on solid cells."""
    j = np.zeros((3,) + f.shape[2:], dtype=f.dtype)
    for i in range(Q):
        for a in range(3):
            if C[i, a] != 0:
                j[a] = j[a] + C[i, a] * (f[0, i] + f[1, i])
    rho_safe = np.where(fluid, rho, 1.0)
    return np.where(fluid, j / rho_safe, 0.0)


# ---------------------------------------------------------------------------
# Eq. (7): Shan-Chen inter-component force
# ---------------------------------------------------------------------------

def neighbour_sum(rho_b, fluid, rho_wall_b):
    """sum_i w_i c_i rho^b(x + c_i) with rho_s^b substituted on solid neighbours."""
    rho_tilde = np.where(fluid, rho_b, rho_wall_b)
    s = np.zeros((3,) + rho_b.shape, dtype=np.result_type(rho_b, np.float64))
    for i in range(1, Q):
        nb = at_offset(rho_tilde, C[i])
        for a in range(3):
            if C[i, a] != 0:
                s[a] = s[a] + W[i] * C[i, a] * nb
    return s


def shan_chen_force(rho_s, G, fluid, rho_wall):
    """F^{ab}(x) = G^{ab} rho^a(x) sum_i w_i c_i rho^b(x + c_i), Eq. (7).

    Returns an array (2, 2, 3, nz, ny, nx): ``F[a, b]`` is the force on
    species a from species b.  Entries with G^{ab} = 0 are zero.
    """
    shape = rho_s.shape[1:]
    F = np.zeros((2, 2, 3) + shape, dtype=np.result_type(rho_s, np.asarray(G).dtype))
    sums = [neighbour_sum(rho_s[b], fluid, rho_wall[b]) for b in range(2)]
    for a in range(2):
        for b in range(2):
            if G[a][b] != 0:
                F[a, b] = G[a][b] * rho_s[a] * sums[b]
    return F


def acceleration(F, rho_s, fluid):
    """g^a = sum_b F^{ab} / rho^a (Sec. 2, after Eq. 9).  Zero on solid cells."""
    g = np.zeros((2, 3) + rho_s.shape[1:], dtype=F.dtype)
    for a in range(2):
        rho_safe = np.where(fluid, rho_s[a], 1.0)
        g[a] = np.where(fluid, (F[a, 0] + F[a, 1]) / rho_safe, 0.0)
    return g


# ---------------------------------------------------------------------------
# Eq. (3): third-order equilibrium
# ---------------------------------------------------------------------------

def equilibrium(rho_a, u):
    """f_i^eq(rho^a, u), Eq. (3) with T0 = 1/3.  Returns (19, nz, ny, nx)."""
    uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2]
    out = np.empty((Q,) + rho_a.shape, dtype=np.result_type(rho_a, u))
    for i in range(Q):
        cu = C[i, 0] * u[0] + C[i, 1] * u[1] + C[i, 2] * u[2]
        out[i] = rho_a * W[i] * (1.0
                                 + cu / T0
                                 + (cu * cu) / (2.0 * T0 * T0)
                                 - uu / (2.0 * T0)
                                 + (cu * cu * cu) / (6.0 * T0 * T0 * T0)
                                 - cu * uu / (2.0 * T0 * T0))
    return out


def forcing_term(rho_a, u, g_a):
    """Exact-difference forcing term f^eq(rho^a, u + g^a dt) - f^eq(rho^a, u) (dt = 1)."""
    return equilibrium(rho_a, u + g_a) - equilibrium(rho_a, u)


# ---------------------------------------------------------------------------
# Eqs. (1)-(2): collision and streaming
# ---------------------------------------------------------------------------

def macroscopic(f, p: Params, solid=None):
    """All cell-local quantities of one step: rho^a, rho, u, F^{ab}, g^a."""
    fluid = fluid_mask(f.shape[2:], solid)
    rho_s = species_density(f)
    rho = mixture_density(rho_s)
    u = mixture_velocity(f, rho, fluid)
    F = shan_chen_force(rho_s, p.G, fluid, p.rho_wall)
    g = acceleration(F, rho_s, fluid)
    return dict(fluid=fluid, rho_s=rho_s, rho=rho, u=u, F=F, g=g)


def momentum_flux_neq(f_a, rho_a, u):
    """Non-equilibrium momentum flux Pi^a = sum_i c_i c_i (f_i^a - f_i^eq(rho^a, u)).

    Returns (3, 3, nz, ny, nx) (symmetric)."""
    d = f_a - equilibrium(rho_a, u)
    out = np.empty((3, 3) + rho_a.shape, dtype=d.dtype)
    for a in range(3):
        for b in range(3):
            out[a, b] = np.einsum("i,izyx->zyx", C[:, a] * C[:, b], d)
    return out


def energy_flux_hermite():
    """Third-order Hermite polynomials of the contracted ("energy flux")
    third moment, H^E_{i,a} = c_{ia} (|c_i|^2 - c_{ia}^2) - 2 T0 c_{ia}, for a = x, y, z.

    On D3Q19 with T0 = 1/3 the diagonal polynomial c_a^3 - 3 T0 c_a vanishes
    identically (c_a^3 = c_a), so the full contraction of the third-order
    Hermite tensor, sum_b H_{abb}, reduces to this sum over b != a.  Returns
    (19, 3)."""
    c2 = (C * C).sum(axis=1)
    return C * (c2[:, None] - C * C) - 2.0 * T0 * C


def regularized_neq(f_a, rho_a, u, order=2):
    """Regularized non-equilibrium part, Eq. (11): f^neq_i = Phi_i : Pi^a.

    Reading of Phi (the paper delegates it to citations and states only that
    it keeps the non-equilibrium moments up to the wanted order, the second
    for the momentum flux and the third for the energy flux, and removes the
    rest in Hermite space): the orthogonal projection, in the w-weighted
    inner product of the lattice, of d = f - f^eq(rho^a, u) onto

    * order 2: the second-order Hermite polynomials c c - T0 I; the
      coefficients are Pi^a = sum_i c_i c_i d_i and the reconstruction is
      w_i (c_i c_i - T0 I) : Pi^a / (2 T0^2);
    * order 3: those plus the energy-flux polynomials H^E of
      :func:`energy_flux_hermite`, with coefficients q_a = sum_i H^E_{ia} d_i
      and the reconstruction w_i H^E_i . q / N, where N = sum_i w_i
      (H^E_{ix})^2 is the polynomials' norm on the lattice (so the
      projection returns q exactly).

    Returns (19, nz, ny, nx).
    """
    pi = momentum_flux_neq(f_a, rho_a, u)
    trace = pi[0, 0] + pi[1, 1] + pi[2, 2]
    out = np.empty((Q,) + rho_a.shape, dtype=pi.dtype)
    for i in range(Q):
        cpc = sum(C[i, a] * C[i, b] * pi[a, b] for a in range(3) for b in range(3))
        out[i] = W[i] * (cpc - T0 * trace) / (2.0 * T0 * T0)
    if order == 3:
        he = energy_flux_hermite()
        norm = float(np.sum(W * he[:, 0] ** 2))
        d = f_a - equilibrium(rho_a, u)
        q = [np.einsum("i,izyx->zyx", he[:, a], d) for a in range(3)]
        for i in range(Q):
            out[i] = out[i] + W[i] * sum(he[i, a] * q[a] for a in range(3)) / norm
    elif order != 2:
        raise ValueError(order)
    return out


def collide(f, p: Params, solid=None):
    """Right-hand side of Eq. (1): f* = f + C_i^a + F_i^a.

    BGK (Eq. 2): f* = f - (f - f^eq) / tau + F.
    Regularized (Eqs. 10-11): f* = f^eq + (1 - 1/tau) f^neq + F with the
    projected f^neq of :func:`regularized_neq` ("regularized": momentum flux
    only; "regularized3": momentum and energy flux).
    Solid cells keep zero populations.
    """
    m = macroscopic(f, p, solid)
    fluid, rho_s, u, g = m["fluid"], m["rho_s"], m["u"], m["g"]
    fstar = np.zeros_like(f, dtype=np.result_type(f, np.asarray(p.tau).dtype,
                                                  np.asarray(p.G).dtype))
    for a in range(2):
        feq = equilibrium(rho_s[a], u)
        force = forcing_term(rho_s[a], u, g[a])
        if p.collision == "bgk":
            coll = -(f[a] - feq) / p.tau[a]
            fstar[a] = np.where(fluid, f[a] + coll + force, 0.0)
        elif p.collision in ("regularized", "regularized3"):
            neq = regularized_neq(f[a], rho_s[a], u, order=3 if p.collision == "regularized3" else 2)
            fstar[a] = np.where(fluid, feq + (1.0 - 1.0 / p.tau[a]) * neq + force, 0.0)
        else:
            raise ValueError(p.collision)
    return fstar


def stream(fstar, solid=None):
    """Left-hand side of Eq. (1): f_i(x + c_i, t + 1) = f*_i(x, t).

    A population whose target x + c_i is a wall cell is reflected back to x
    in direction opp(i) (pointwise bounce-back, Sec. 4).
    """
    fluid = fluid_mask(fstar.shape[2:], solid)
    out = np.zeros_like(fstar)
    for i in range(Q):
        target_fluid = at_offset(fluid, C[i])
        go = fluid & target_fluid
        back = fluid & ~target_fluid
        moved = np.where(go, fstar[:, i], 0.0)
        # value computed at x lands on x + c_i
        cx, cy, cz = (int(v) for v in C[i])
        out[:, i] = out[:, i] + np.roll(moved, shift=(cz, cy, cx), axis=(-3, -2, -1))
        out[:, OPP[i]] = out[:, OPP[i]] + np.where(back, fstar[:, i], 0.0)
    return out


def step(f, p: Params, solid=None):
    """One time step of Eq. (1): collide, then stream."""
    return stream(collide(f, p, solid), solid)


def run(f, p: Params, steps, solid=None):
    for _ in range(steps):
        f = step(f, p, solid)
    return f


# ---------------------------------------------------------------------------
# Initial state and observables
# ---------------------------------------------------------------------------

def init_state(rho0, solid=None):
    """Rest state f_i^a = w_i rho0^a (Eq. 3 at u = 0); zero on solid cells."""
    fluid = fluid_mask(rho0.shape[1:], solid)
    f = np.zeros((2, Q) + rho0.shape[1:], dtype=rho0.dtype)
    for a in range(2):
        for i in range(Q):
            f[a, i] = np.where(fluid, W[i] * rho0[a], 0.0)
    return f


def force_velocity(f, p: Params, solid=None):
    """u_F = u + g dt / 2 with g = sum_a g^a rho^a / rho, Eqs. (8)-(9)."""
    m = macroscopic(f, p, solid)
    fluid, rho_s, rho, u, g = m["fluid"], m["rho_s"], m["rho"], m["u"], m["g"]
    rho_safe = np.where(fluid, rho, 1.0)
    gmix = (g[0] * rho_s[0] + g[1] * rho_s[1]) / rho_safe
    return np.where(fluid, u + 0.5 * gmix, 0.0)


def observables(f, p: Params, solid=None):
    """(rho^A, rho^B, u_F) at the current time: the fields the step reports."""
    rho_s = species_density(f)
    return rho_s, force_velocity(f, p, solid)


# ---------------------------------------------------------------------------
# Reduced-precision storage (emulation of the shifted FP16 / BF16 form)
# ---------------------------------------------------------------------------

def _round_bf16(x64):
    """Round to bfloat16 via float32, round-to-nearest-even on the 16 dropped bits."""
    x32 = np.asarray(x64, dtype=np.float32)
    bits = x32.view(np.uint32).astype(np.uint64)
    lsb = (bits >> 16) & 1
    bits = (bits + 0x7FFF + lsb) & 0xFFFF0000
    return bits.astype(np.uint32).view(np.float32).astype(np.float64)


def _round_to(dev, storage):
    if storage == "fp32":
        return dev.astype(np.float32).astype(np.float64)
    if storage == "fp16":
        return dev.astype(np.float16).astype(np.float64)
    if storage == "bf16":
        return _round_bf16(dev)
    raise ValueError(storage)


# The residual of the rest population is stored times this power of two: an
# FP16 residual (at most 2^-11 of the rest value) would otherwise fall among
# the FP16 subnormals.
RESIDUAL_SCALE = {"fp32": 1.0, "fp16": 2048.0, "bf16": 1.0}


def round_storage(fstar, storage, rho_shift):
    """Pass post-collision populations through the shifted 16-bit storage form.

    The storage rule of this build (not the paper's): each moving population
    is stored as round(f*_i^a - w_i rho_shift^a); the rest population keeps
    the remainder e = rho^a - sum_{i>0} decoded_i - w_0 rho_shift^a in two
    stored values, round(e) and round((e - round(e)) s) with s the residual
    scale, and reads back as round(e) + round(...) / s, so that the decoded
    populations of a cell sum to its density up to the rounding of that
    residual.  Returns the decoded values in FP64.
    """
    if storage == "fp64":
        return fstar
    out = np.empty_like(fstar)
    for a in range(2):
        shift = W[:, None, None, None] * rho_shift[a]
        moving = _round_to(fstar[a, 1:] - shift[1:], storage) + shift[1:]
        rho = fstar[a].sum(axis=0)
        e = rho - moving.sum(axis=0) - shift[0]
        high = _round_to(e, storage)
        rest = high + _round_to((e - high) * RESIDUAL_SCALE[storage], storage) / RESIDUAL_SCALE[storage] + shift[0]
        out[a, 1:] = moving
        out[a, 0] = rest
    return out


def step_stored(f, p: Params, storage, rho_shift, solid=None):
    """One step in which the post-collision populations pass through ``storage``."""
    fstar = collide(f, p, solid)
    fluid = fluid_mask(f.shape[2:], solid)
    fstar = np.where(fluid, round_storage(fstar, storage, rho_shift), 0.0)
    return stream(fstar, solid)
