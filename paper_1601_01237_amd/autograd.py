"""Reverse mode of the two-component step behind ``torch.autograd.Function``.

``LBMFunction.apply(rho0, G, tau, steps, every, solid, rho_wall, collision,
storage)`` runs ``steps`` fused steps from the rest state of ``rho0`` and
returns the species densities rho^a(x, T) as float32 (2, nz, ny, nx).  Its
backward pass gives dL/drho0 (float64, same shape), dL/dG (tied G^{AB} =
G^{BA}) and dL/dtau (tied tau_A = tau_B) for any scalar L of those densities.
With 16-bit storage each reverse step is that of the FP32 step at the
populations the stored state decodes to (the storage rounding is passed
through as the identity).

Backward is a checkpointed reverse sweep: the forward pass keeps the stored
state every ``every`` steps; for each segment, last first, the states of the
segment are recomputed from its checkpoint (with FP32 storage each
recomputed step also writes the densities and mixture velocity of the state
it starts from) and the
library's adjoint step (transposed collision with the Eq. (7) gather,
transposed pull streaming) carries dL/dX_{t+1} back to dL/dX_t.  All of it
runs in liblbm.so.
"""

from __future__ import annotations

import ctypes as C

import torch

from . import _lib
from .sim import Sim, _ptr


def to_adjoint_layout(f, sim):
    """(2, 19, nz, ny, nx) FP32 array -> adjoint array in the state layout of ``sim``."""
    return sim.to_state_layout(f, sim.lam_layout, sim.lam_elems)


def from_adjoint_layout(x, sim):
    """Adjoint array (state layout of ``sim``) -> (2, 19, nz, ny, nx)."""
    return sim.from_state_layout(x, sim.lam_layout)


class Reverse:
    """Adjoint machinery of one Sim.  The adjoint arrays are FP32 in the FP32
    state layout whatever the storage; with 16-bit storage the workspace also
    holds an FP32 copy of X_t and only the pulling reverse step exists."""

    def __init__(self, sim: Sim):
        self.sim = sim
        self.lib = sim.lib
        nbytes = int(self.lib.lbm_adjoint_work_bytes(sim.ctx))
        self.work = torch.empty(nbytes, dtype=torch.uint8, device=sim.device)
        self.dparams = torch.zeros(3, dtype=torch.float64, device=sim.device)

    def seed(self, grad_rho):
        """dL/dX_T from dL/drho(T) ((2, nz, ny, nx), any float dtype)."""
        g = grad_rho.to(device=self.sim.device, dtype=torch.float32).contiguous()
        lam = torch.zeros(self.sim.lam_elems, dtype=torch.float32, device=self.sim.device)
        _lib.check("lbm_adjoint_seed", self.lib.lbm_adjoint_seed(self.sim.ctx, _ptr(g), _ptr(lam)))
        return lam

    def step(self, x_t, lam_next, want_drho0=False, fields=None):
        """dL/dX_t from dL/dX_{t+1}; accumulates into self.dparams.  With
        ``fields`` (from ``Sim.step_fields`` at X_t) the reverse march reads
        the forward densities and velocity instead of pulling X_t again
        (same results, bitwise)."""
        lam = torch.empty_like(lam_next)
        drho0 = None
        if want_drho0:
            drho0 = torch.empty(2 * self.sim.n, dtype=torch.float64, device=self.sim.device)
        if fields is None:
            _lib.check("lbm_adjoint_step", self.lib.lbm_adjoint_step(
                self.sim.ctx, _ptr(x_t), _ptr(lam_next), _ptr(lam), _ptr(self.work),
                C.c_size_t(self.work.numel()), _ptr(self.dparams), _ptr(drho0)))
        else:
            _lib.check("lbm_adjoint_step_fields", self.lib.lbm_adjoint_step_fields(
                self.sim.ctx, _ptr(x_t), _ptr(fields), _ptr(lam_next), _ptr(lam), _ptr(self.work),
                C.c_size_t(self.work.numel()), _ptr(self.dparams), _ptr(drho0)))
        return lam, drho0


def forward_with_checkpoints(sim: Sim, steps: int, every: int):
    ckpts = {0: sim.state.clone()}
    for t0 in range(0, steps, every):
        n = min(every, steps - t0)
        sim.step(n)
        if sim.t < steps:
            ckpts[sim.t] = sim.state.clone()
    return ckpts


def reverse_sweep(sim: Sim, ckpts, steps: int, every: int, grad_rho):
    """Returns (dL/drho0 (2,nz,ny,nx) float64, dL/dG tied, dL/dtau_A, dL/dtau_B)."""
    rev = Reverse(sim)
    lam = rev.seed(grad_rho)
    drho0 = None
    starts = sorted(ckpts)
    for s in reversed(starts):
        e = min(s + every, steps)
        sim.restore((ckpts[s], s))
        # recompute the segment: X_s .. X_{e-1}, and with each step the
        # forward fields of the state it started from (the step to X_e
        # gives those of X_{e-1})
        states, fields = [], []
        for _ in range(s, e):
            states.append(sim.state.clone())
            if sim.storage == "fp32":
                fields.append(sim.step_fields())
            else:
                sim.step(1)
                fields.append(None)
        for t in range(e - 1, s - 1, -1):
            lam, d = rev.step(states[t - s], lam, want_drho0=(t == 0), fields=fields[t - s])
            if d is not None:
                drho0 = d
    d = rev.dparams.cpu()
    nz, ny, nx = sim.shape
    return drho0.view(2, nz, ny, nx), float(d[0]), float(d[1]), float(d[2])


class LBMFunction(torch.autograd.Function):
    """rho(T) = run(rho0; G, tau) with a hand-written adjoint (see module doc)."""

    @staticmethod
    def forward(ctx, rho0, G, tau, steps, every=50, solid=None, rho_wall=(0.0, 0.0), collision="bgk",
                storage="fp32"):
        g = float(G)
        t = float(tau)
        sim = Sim(rho0.detach().double().cpu().numpy(), tau=(t, t), G=g, solid=solid, storage=storage,
                  rho_wall=rho_wall, device=rho0.device if rho0.is_cuda else "cuda:0", collision=collision)
        ckpts = forward_with_checkpoints(sim, int(steps), int(every))
        rho, _, _ = sim.moments()
        ctx.sim = sim
        ctx.ckpts = ckpts
        ctx.steps = int(steps)
        ctx.every = int(every)
        ctx.rho0_device = rho0.device
        return rho.clone()

    @staticmethod
    def backward(ctx, grad_rho):
        drho0, dG, dtA, dtB = reverse_sweep(ctx.sim, ctx.ckpts, ctx.steps, ctx.every, grad_rho)
        ctx.sim.close()
        dev = ctx.rho0_device
        return (drho0.to(dev), torch.tensor(dG, dtype=torch.float64, device=dev),
                torch.tensor(dtA + dtB, dtype=torch.float64, device=dev), None, None, None, None, None, None)
