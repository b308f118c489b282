"""GPU adjoint against the FP64 oracle's hand-written transpose (through the C ABI).

The stored state of the library is the post-collision population X_t, so one
library adjoint step is dL/dX_t = S^T C^T dL/dX_{t+1} with C the collision at
f_t = pull(X_t) and S the pull streaming; in oracle terms that is
``stream_adjoint(collide_adjoint(f_t, lam))``.
"""

import ctypes

import numpy as np
import pytest
import torch

from oracle import adjoint as oadj
from oracle import lbm as olbm
from paper_1601_01237_amd import inputs

from ._gpu_util import rel_err, say

pytestmark = pytest.mark.gpu


def _random_state(shape, seed, solid=None):
    rng = np.random.default_rng(seed)
    rho = 0.3 + rng.uniform(0.0, 0.7, size=(2,) + shape)
    u = rng.uniform(-0.05, 0.05, size=(3,) + shape)
    f = np.stack([olbm.equilibrium(rho[a], u) for a in range(2)])
    f = f * (1.0 + 0.02 * rng.uniform(-1.0, 1.0, size=f.shape))
    if solid is not None:
        f[:, :, solid] = 0.0
    return f.astype(np.float32).astype(np.float64), rho


@pytest.mark.parametrize("collision", ["bgk", "regularized", "regularized3"])
@pytest.mark.parametrize("walls", [None, "obstacle", "porous"])
def test_one_adjoint_step_matches_oracle(lib, walls, collision):
    """The obstacle geometry takes the one-byte wall classes, the random
    porous one (more distinct link words than classes) the link words."""
    from paper_1601_01237_amd.autograd import Reverse, from_adjoint_layout, to_adjoint_layout
    from paper_1601_01237_amd.sim import Sim
    say(f"adjoint one step walls={walls} {collision}")
    shape = (7, 9, 70)
    solid = None
    if walls == "obstacle":
        solid = np.zeros(shape, bool)
        solid[0] = True
        solid[3, 2:6, 10:30] = True
    elif walls == "porous":
        solid = np.random.default_rng(23).uniform(size=shape) < 0.3
        solid[0] = True
    f, rho = _random_state(shape, 1, solid)
    p = olbm.Params(tau=(0.8, 1.3), G=((0.0, -1.4), (-0.6, 0.0)), rho_wall=(0.15, 0.35), collision=collision)
    if solid is not None:
        rho[:, solid] = 0.0
    sim = Sim(rho, tau=p.tau, G=p.G, rho_wall=p.rho_wall, solid=solid, collision=collision)
    if walls:
        assert (sim.wall_classes() > 0) == (walls == "obstacle")
    sim.set_populations(torch.from_numpy(f.astype(np.float32)))
    lam1 = np.random.default_rng(2).normal(size=f.shape)
    if solid is not None:
        lam1[:, :, solid] = 0.0
    lam1 = lam1.astype(np.float32)
    rev = Reverse(sim)
    x_t = sim.state
    lam_gpu, drho = rev.step(x_t, to_adjoint_layout(torch.from_numpy(lam1).cuda(), sim), want_drho0=True)
    got = from_adjoint_layout(lam_gpu, sim).cpu().numpy()

    mu, dG, dtau = oadj.collide_adjoint(f, lam1.astype(np.float64), p, solid)
    want = oadj.stream_adjoint(mu, solid)
    e = rel_err(got, want)
    assert e < 1e-5, e
    d = rev.dparams.cpu().numpy()
    # Parameter derivatives are sums over cells of terms with random signs
    # (lam is random here), so the sum is much smaller than its terms; each
    # FP32 term carries the rounding of f - f^eq.  Bound the error by the sum
    # of magnitudes of the terms.
    m = olbm.macroscopic(f, p, solid)
    if collision == "bgk":
        part = [f[a] - olbm.equilibrium(m["rho_s"][a], m["u"]) for a in range(2)]
    else:
        order = 3 if collision == "regularized3" else 2
        part = [olbm.regularized_neq(f[a], m["rho_s"][a], m["u"], order) for a in range(2)]
    scale_tau = [np.sum(np.abs(lam1[a] * part[a])) / p.tau[a] ** 2 for a in range(2)]
    assert abs(d[0] - (dG[0, 1] + dG[1, 0])) <= 1e-4 * abs(dG[0, 1] + dG[1, 0]), (d[0], dG)
    assert abs(d[1] - dtau[0]) <= 1e-6 * scale_tau[0], (d[1], dtau, scale_tau)
    assert abs(d[2] - dtau[1]) <= 1e-6 * scale_tau[1], (d[2], dtau, scale_tau)
    drho_want = np.einsum("i,aizyx->azyx", olbm.W, mu)
    e = rel_err(drho.view(2, *shape).cpu().numpy(), drho_want)
    assert e < 1e-5, e
    sim.close()


@pytest.mark.parametrize("collision", ["bgk", "regularized"])
@pytest.mark.parametrize("shape", [(3, 5, 9), (2, 3, 130), (5, 1, 4), (9, 13, 65)])
def test_adjoint_step_ragged_grids(lib, shape, collision):
    """Grids thinner than one chunk (nz < 4), a single row, and x-y planes
    that leave partial tiles in the reverse march."""
    from paper_1601_01237_amd.autograd import Reverse, from_adjoint_layout, to_adjoint_layout
    from paper_1601_01237_amd.sim import Sim
    say(f"adjoint ragged {shape} {collision}")
    f, rho = _random_state(shape, 11)
    p = olbm.Params(tau=(0.9, 1.2), G=((0.0, -1.1), (-0.8, 0.0)), collision=collision)
    sim = Sim(rho, tau=p.tau, G=p.G, collision=collision)
    sim.set_populations(torch.from_numpy(f.astype(np.float32)))
    lam1 = np.random.default_rng(12).normal(size=f.shape).astype(np.float32)
    rev = Reverse(sim)
    lam_gpu, drho = rev.step(sim.state, to_adjoint_layout(torch.from_numpy(lam1).cuda(), sim), want_drho0=True)
    got = from_adjoint_layout(lam_gpu, sim).cpu().numpy()
    sim.close()
    mu, _, _ = oadj.collide_adjoint(f, lam1.astype(np.float64), p)
    want = oadj.stream_adjoint(mu)
    assert rel_err(got, want) < 1e-5
    e = rel_err(drho.view(2, *shape).cpu().numpy(), np.einsum("i,aizyx->azyx", olbm.W, mu))
    assert e < 1e-5, e


def test_seed_matches_oracle(lib):
    from paper_1601_01237_amd.autograd import Reverse, from_adjoint_layout
    from paper_1601_01237_amd.sim import Sim
    say("adjoint seed")
    shape = (8, 6, 10)
    solid = np.zeros(shape, bool)
    solid[0] = True
    solid[4, 2, 3] = True
    rho0 = np.full((2,) + shape, 0.5)
    rho0[:, solid] = 0.0
    sim = Sim(rho0, solid=solid)
    g = np.random.default_rng(3).normal(size=(2,) + shape)
    g[:, solid] = 0.0
    lam = Reverse(sim).seed(torch.from_numpy(g))
    got = from_adjoint_layout(lam, sim).cpu().numpy()
    lam_f = np.repeat(g[:, None], 19, axis=1)
    want = oadj.stream_adjoint(lam_f, solid)
    assert rel_err(got, want) < 1e-6
    sim.close()


def _calibration_inputs(n):
    rho0 = inputs.sphere_droplet((n, n, n), radius=n * 20.0 / 96.0, seed=0)
    target = inputs.target_ellipsoid((n, n, n), radius=n * 20.0 / 96.0, seed=1)
    return rho0, target


def test_calibration_gradient_16cube_matches_fp64_oracle(lib):
    """Differentiation workload scaled to 16^3: 500 steps, checkpoints every 50."""
    from paper_1601_01237_amd.autograd import LBMFunction
    say("calibration gradient 16^3 x 500")
    n, steps, every = 16, 500, 50
    rho0, target = _calibration_inputs(n)
    G, tau = -1.0, 1.0
    r0 = torch.tensor(rho0, device="cuda", requires_grad=True)
    Gt = torch.tensor(G, dtype=torch.float64, requires_grad=True)
    Tt = torch.tensor(tau, dtype=torch.float64, requires_grad=True)
    rho = LBMFunction.apply(r0, Gt, Tt, steps, every)
    tgt = torch.tensor(target, dtype=torch.float32, device="cuda")
    L = 0.5 * ((rho[0].double() - tgt.double()) ** 2).sum()
    L.backward()

    p = olbm.Params(tau=(tau, tau), G=((0.0, G), (G, 0.0)))
    L_ref, dG_ref, dtau_ref, drho0_ref = oadj.loss_and_gradient(rho0, p, steps, target)
    e_G = abs(float(Gt.grad) - dG_ref) / abs(dG_ref)
    e_t = abs(float(Tt.grad) - dtau_ref) / abs(dtau_ref)
    e_r = rel_err(r0.grad.cpu().numpy(), drho0_ref)
    say(f"16^3 calibration: L {float(L.detach()):.6e} vs {L_ref:.6e}; dL/dG {float(Gt.grad):.6e} vs {dG_ref:.6e} "
        f"({e_G:.1e}); dL/dtau {float(Tt.grad):.6e} vs {dtau_ref:.6e} ({e_t:.1e}); dL/drho0 {e_r:.1e}")
    assert abs(float(L.detach()) - L_ref) <= 1e-5 * L_ref
    assert e_G < 1e-3 and e_t < 1e-3 and e_r < 1e-3, (e_G, e_t, e_r)


@pytest.mark.parametrize("collision", ["regularized", "regularized3"])
def test_regularized_calibration_gradient_16cube_matches_fp64_oracle(lib, collision):
    """The differentiation workload at 16^3 with the regularized collision
    (Sec. 3; second- and third-order readings) at tau = 0.8: 200 steps,
    checkpoints every 50."""
    from paper_1601_01237_amd.autograd import LBMFunction
    say(f"{collision} calibration gradient 16^3 x 200")
    n, steps, every = 16, 200, 50
    rho0, target = _calibration_inputs(n)
    G, tau = -1.0, 0.8
    r0 = torch.tensor(rho0, device="cuda", requires_grad=True)
    Gt = torch.tensor(G, dtype=torch.float64, requires_grad=True)
    Tt = torch.tensor(tau, dtype=torch.float64, requires_grad=True)
    rho = LBMFunction.apply(r0, Gt, Tt, steps, every, None, (0.0, 0.0), collision)
    tgt = torch.tensor(target, dtype=torch.float32, device="cuda")
    L = 0.5 * ((rho[0].double() - tgt.double()) ** 2).sum()
    L.backward()

    p = olbm.Params(tau=(tau, tau), G=((0.0, G), (G, 0.0)), collision=collision)
    L_ref, dG_ref, dtau_ref, drho0_ref = oadj.loss_and_gradient(rho0, p, steps, target)
    e_G = abs(float(Gt.grad) - dG_ref) / abs(dG_ref)
    e_t = abs(float(Tt.grad) - dtau_ref) / abs(dtau_ref)
    e_r = rel_err(r0.grad.cpu().numpy(), drho0_ref)
    say(f"16^3 {collision} calibration: L {float(L.detach()):.6e} vs {L_ref:.6e}; dL/dG {float(Gt.grad):.6e} vs "
        f"{dG_ref:.6e} ({e_G:.1e}); dL/dtau {float(Tt.grad):.6e} vs {dtau_ref:.6e} ({e_t:.1e}); dL/drho0 {e_r:.1e}")
    assert abs(float(L.detach()) - L_ref) <= 1e-5 * L_ref
    assert e_G < 1e-3 and e_t < 1e-3 and e_r < 1e-3, (e_G, e_t, e_r)


def test_calibration_gradient_against_central_differences(lib):
    from paper_1601_01237_amd.autograd import LBMFunction
    say("calibration gradient vs central differences 16^3 x 100")
    # The FP32 forward leaves ~1e-7 relative rounding noise in the loss; at
    # h = 1e-3 that is ~0.3% of the central difference, whose O(h^2)
    # truncation error stays far below it.
    n, steps, every, h = 16, 100, 25, 1e-3
    rho0, target = _calibration_inputs(n)
    tgt = torch.tensor(target, dtype=torch.float64, device="cuda")

    def loss(G, tau, r0=None):
        r = torch.tensor(rho0, device="cuda") if r0 is None else r0
        rho = LBMFunction.apply(r, torch.tensor(G), torch.tensor(tau), steps, every)
        return 0.5 * ((rho[0].double() - tgt) ** 2).sum()

    G, tau = -1.0, 1.0
    r0 = torch.tensor(rho0, device="cuda", requires_grad=True)
    Gt = torch.tensor(G, dtype=torch.float64, requires_grad=True)
    Tt = torch.tensor(tau, dtype=torch.float64, requires_grad=True)
    L = 0.5 * ((LBMFunction.apply(r0, Gt, Tt, steps, every)[0].double() - tgt) ** 2).sum()
    L.backward()
    with torch.no_grad():
        fd_G = (float(loss(G + h, tau)) - float(loss(G - h, tau))) / (2 * h)
        fd_t = (float(loss(G, tau + h)) - float(loss(G, tau - h))) / (2 * h)
        v = torch.tensor(inputs.uniform_noise(rho0.shape, seed=4), device="cuda")
        fd_r = (float(loss(G, tau, torch.tensor(rho0, device="cuda") + h * v))
                - float(loss(G, tau, torch.tensor(rho0, device="cuda") - h * v))) / (2 * h)
    assert abs(float(Gt.grad) - fd_G) <= 1e-2 * abs(fd_G), (float(Gt.grad), fd_G)
    assert abs(float(Tt.grad) - fd_t) <= 1e-2 * abs(fd_t), (float(Tt.grad), fd_t)
    ad_r = float((r0.grad * v).sum())
    assert abs(ad_r - fd_r) <= 1e-2 * abs(fd_r), (ad_r, fd_r)


@pytest.mark.parametrize("n,steps,every", [(96, 500, 50)])
def test_calibration_gradient_full_size_against_central_differences(lib, n, steps, every):
    """The differentiation workload at full size: 96^3, R = 20, 500 steps with
    a checkpoint every 50; dL/dG, dL/dtau and a random direction of dL/drho0
    against central differences of the FP32 forward (h = 1e-3, as on 16^3:
    the forward's rounding noise swamps h = 1e-4)."""
    from paper_1601_01237_amd.autograd import LBMFunction
    say(f"calibration gradient vs central differences {n}^3 x {steps}")
    h = 1e-3
    rho0, target = _calibration_inputs(n)
    tgt = torch.tensor(target, dtype=torch.float64, device="cuda")

    def loss(G, tau, r0=None):
        r = torch.tensor(rho0, device="cuda") if r0 is None else r0
        rho = LBMFunction.apply(r, torch.tensor(G), torch.tensor(tau), steps, every)
        return 0.5 * ((rho[0].double() - tgt) ** 2).sum()

    G, tau = -1.0, 1.0
    r0 = torch.tensor(rho0, device="cuda", requires_grad=True)
    Gt = torch.tensor(G, dtype=torch.float64, requires_grad=True)
    Tt = torch.tensor(tau, dtype=torch.float64, requires_grad=True)
    L = 0.5 * ((LBMFunction.apply(r0, Gt, Tt, steps, every)[0].double() - tgt) ** 2).sum()
    L.backward()
    with torch.no_grad():
        fd_G = (float(loss(G + h, tau)) - float(loss(G - h, tau))) / (2 * h)
        fd_t = (float(loss(G, tau + h)) - float(loss(G, tau - h))) / (2 * h)
        v = torch.tensor(inputs.uniform_noise(rho0.shape, seed=4), device="cuda")
        fd_r = (float(loss(G, tau, torch.tensor(rho0, device="cuda") + h * v))
                - float(loss(G, tau, torch.tensor(rho0, device="cuda") - h * v))) / (2 * h)
    ad_r = float((r0.grad * v).sum())
    say(f"{n}^3 gradient: dG {float(Gt.grad):.6e} (FD {fd_G:.6e}), dtau {float(Tt.grad):.6e} (FD {fd_t:.6e}), "
        f"drho0.v {ad_r:.6e} (FD {fd_r:.6e})")
    assert abs(float(Gt.grad) - fd_G) <= 1e-2 * abs(fd_G), (float(Gt.grad), fd_G)
    assert abs(float(Tt.grad) - fd_t) <= 1e-2 * abs(fd_t), (float(Tt.grad), fd_t)
    assert abs(ad_r - fd_r) <= 1e-2 * abs(fd_r), (ad_r, fd_r)


@pytest.mark.parametrize("fields", [False, True])
@pytest.mark.parametrize("collision,tau", [("bgk", 1.0), ("regularized", 0.8)])
def test_adjoint_step_96cube_all_cells(lib, collision, tau, fields):
    """One reverse step of the differentiation workload at its full size
    (96^3 droplet, R = 20, G = -1, automatic tiling as timed), every cell
    against the oracle; tau = 1 with BGK, 0.8 with the regularized collision.
    With ``fields`` the reverse step reads the densities and velocity a
    forward step wrote (the path the benchmark times) and must equal the
    pulling reverse step bitwise."""
    from paper_1601_01237_amd.autograd import Reverse, from_adjoint_layout, to_adjoint_layout
    from paper_1601_01237_amd.sim import Sim
    say(f"adjoint one step 96^3 {collision} fields={fields}")
    n = 96
    rho0 = inputs.sphere_droplet((n, n, n), radius=20.0, seed=0)
    p = olbm.Params(tau=(tau, tau), G=((0.0, -1.0), (-1.0, 0.0)), collision=collision)
    sim = Sim(rho0, tau=p.tau, G=p.G, collision=collision)
    sim.step(20)
    f = sim.populations().cpu().numpy().astype(np.float64)   # pre-collision f at t = 20
    lam1 = np.random.default_rng(9).normal(size=f.shape).astype(np.float32)
    rev = Reverse(sim)
    x_t = sim.state.clone()
    lam_in = to_adjoint_layout(torch.from_numpy(lam1).cuda(), sim)
    lam_gpu, drho = rev.step(x_t, lam_in, want_drho0=True)
    got = from_adjoint_layout(lam_gpu, sim).cpu().numpy()
    d = rev.dparams.cpu().numpy()
    if fields:
        fl = sim.step_fields()  # the forward step from x_t, with its fields
        rev_f = Reverse(sim)
        lam_f, drho_f = rev_f.step(x_t, lam_in, want_drho0=True, fields=fl)
        live = sim.live_mask(sim.lam_layout)
        assert torch.equal(lam_f[live], lam_gpu[live]) and torch.equal(drho_f, drho)
        np.testing.assert_allclose(rev_f.dparams.cpu().numpy(), d, rtol=1e-12, atol=0)
    sim.close()
    mu, dG, dtau = oadj.collide_adjoint(f, lam1.astype(np.float64), p)
    want = oadj.stream_adjoint(mu)
    e = rel_err(got, want)
    say(f"96^3 adjoint step: lam error {e:.2e}, dG {d[0]:.6e} vs {dG[0, 1] + dG[1, 0]:.6e}")
    assert e < 1e-5, e
    m = olbm.macroscopic(f, p)
    if collision == "bgk":
        part = [f[a] - olbm.equilibrium(m["rho_s"][a], m["u"]) for a in range(2)]
    else:
        part = [olbm.regularized_neq(f[a], m["rho_s"][a], m["u"]) for a in range(2)]
    scale_tau = [np.sum(np.abs(lam1[a] * part[a])) / p.tau[a] ** 2 for a in range(2)]
    assert abs(d[0] - (dG[0, 1] + dG[1, 0])) <= 1e-4 * abs(dG[0, 1] + dG[1, 0]), (d[0], dG)
    assert abs(d[1] - dtau[0]) <= 1e-6 * scale_tau[0]
    assert abs(d[2] - dtau[1]) <= 1e-6 * scale_tau[1]
    e = rel_err(drho.view(2, n, n, n).cpu().numpy(), np.einsum("i,aizyx->azyx", olbm.W, mu))
    assert e < 1e-5, e


def test_adjoint_workspace_size_and_checks(lib):
    """The workspace holds three FP64 partial sums per workgroup of the
    reverse march, whatever the collision, and for 16-bit storage an FP32
    copy of X_t after them; a workspace one byte short, aliased arrays and
    16-bit storage with the fields path are refused before anything is
    launched."""
    import ctypes
    from paper_1601_01237_amd.sim import Sim
    say("adjoint workspace checks")
    shape = (6, 9, 20)
    rho0 = inputs.sphere_droplet(shape, radius=2.5, seed=3)
    sims = {c: Sim(rho0, tau=(0.8, 0.8), G=-1.0, collision=c) for c in ("bgk", "regularized")}
    for s in sims.values():
        s.set_adjoint_tiling(2, 2)  # 32 x 8 tiles, 2-plane chunks: 1 x 2 x 3 workgroups
    wb = {c: int(lib.lbm_adjoint_work_bytes(s.ctx)) for c, s in sims.items()}
    assert wb["regularized"] == wb["bgk"] == 6 * 3 * 8
    s = sims["regularized"]
    lam_in = torch.zeros(s.lam_elems, dtype=torch.float32, device="cuda")
    lam_out = torch.zeros_like(lam_in)
    dparams = torch.zeros(3, dtype=torch.float64, device="cuda")
    work = torch.empty(wb["regularized"], dtype=torch.uint8, device="cuda")
    p = lambda t: ctypes.c_void_p(t.data_ptr())  # noqa: E731
    short = ctypes.c_size_t(wb["regularized"] - 1)
    assert lib.lbm_adjoint_step(s.ctx, p(s.state), p(lam_in), p(lam_out), p(work), short, p(dparams), None) == -1
    full = ctypes.c_size_t(wb["regularized"])
    assert lib.lbm_adjoint_step(s.ctx, p(s.state), p(lam_in), p(lam_in), p(work), full, p(dparams), None) == -1
    assert lib.lbm_adjoint_step(s.ctx, p(s.state), p(lam_in), p(lam_out), p(work), full, p(dparams), None) == 0
    torch.cuda.synchronize()
    assert bool(torch.isfinite(lam_out).all())
    for sim in sims.values():
        sim.close()
    h = Sim(rho0, storage="fp16")
    h.set_adjoint_tiling(2, 2)
    wb16 = int(lib.lbm_adjoint_work_bytes(h.ctx))
    assert wb16 == 256 + 4 * h.lam_elems  # 144 bytes of partial sums, rounded up, then X_t in FP32
    work16 = torch.empty(wb16, dtype=torch.uint8, device="cuda")
    assert lib.lbm_adjoint_step(h.ctx, p(h.state), p(lam_in), p(lam_out), p(work16),
                                ctypes.c_size_t(wb16 - 1), p(dparams), None) == -1
    assert lib.lbm_adjoint_step(h.ctx, p(h.state), p(lam_in), p(lam_out), p(work16),
                                ctypes.c_size_t(wb16), p(dparams), None) == 0
    torch.cuda.synchronize()
    assert bool(torch.isfinite(lam_out).all())
    h.close()
    r3 = Sim(rho0, collision="regularized3")
    r3.set_adjoint_tiling(2, 2)
    work3 = torch.empty(int(lib.lbm_adjoint_work_bytes(r3.ctx)), dtype=torch.uint8, device="cuda")
    assert work3.numel() == wb["bgk"]
    assert lib.lbm_adjoint_step(r3.ctx, p(r3.state), p(lam_in), p(lam_out), p(work3),
                                ctypes.c_size_t(work3.numel()), p(dparams), None) == 0
    torch.cuda.synchronize()
    assert bool(torch.isfinite(lam_out).all())
    r3.close()


@pytest.mark.parametrize("collision,walls", [("bgk", False), ("regularized", True), ("regularized3", True)])
def test_adjoint_tiling_invariance(lib, collision, walls):
    """Every shape and z chunk of the reverse march gives the same lam_t,
    bitwise (only the summation order of dL/dG and dL/dtau changes)."""
    from paper_1601_01237_amd.autograd import Reverse, to_adjoint_layout
    from paper_1601_01237_amd.sim import Sim
    shape = (11, 21, 70)
    say(f"adjoint tiling invariance {collision} walls={walls}")
    solid = None
    if walls:
        solid = np.zeros(shape, bool)
        solid[0] = True
        solid[5, 3:9, 20:41] = True
    f, rho = _random_state(shape, 21, solid)
    if solid is not None:
        rho[:, solid] = 0.0
    sim = Sim(rho, tau=(0.8, 1.2), G=((0.0, -1.3), (-0.7, 0.0)), rho_wall=(0.2, 0.1), solid=solid,
              collision=collision)
    sim.set_populations(torch.from_numpy(f.astype(np.float32)))
    lam1 = np.random.default_rng(22).normal(size=f.shape).astype(np.float32)
    if solid is not None:
        lam1[:, :, solid] = 0.0
    lam_in = to_adjoint_layout(torch.from_numpy(lam1).cuda(), sim)
    live = sim.live_mask(sim.lam_layout)
    outs, params = [], []
    for shp, zc in [(-1, 0), (0, 3), (1, 1), (2, 5), (3, 0), (3, 11)]:
        sim.set_adjoint_tiling(shp, zc)
        rev = Reverse(sim)
        lam, drho = rev.step(sim.state, lam_in, want_drho0=True)
        torch.cuda.synchronize()
        outs.append((lam[live].cpu(), drho.cpu()))
        params.append(rev.dparams.cpu().numpy())
    sim.close()
    for lam, drho in outs[1:]:
        assert torch.equal(lam, outs[0][0]) and torch.equal(drho, outs[0][1])
    for p in params[1:]:
        np.testing.assert_allclose(p, params[0], rtol=1e-9, atol=1e-12)


@pytest.mark.parametrize("collision", ["bgk", "regularized", "regularized3"])
@pytest.mark.parametrize("walls", [False, True])
def test_step_fields_and_reverse_with_fields(lib, walls, collision):
    """lbm_step_fields advances the state exactly as lbm_step and writes the
    densities and mixture velocity of the pull it collides (against the
    oracle's Eqs. 4-6; rho_s and 0 on wall cells); the reverse step that
    reads them is bitwise the reverse step that pulls them itself, for every
    reverse-march shape."""
    from paper_1601_01237_amd.autograd import Reverse, to_adjoint_layout
    from paper_1601_01237_amd.sim import Sim
    say(f"step fields and reverse with fields walls={walls} {collision}")
    shape = (11, 21, 70)
    solid = None
    if walls:
        solid = np.zeros(shape, bool)
        solid[0] = True
        solid[5, 3:9, 20:41] = True
    f, rho = _random_state(shape, 31, solid)
    if solid is not None:
        rho[:, solid] = 0.0
    p = olbm.Params(tau=(0.8, 1.2), G=((0.0, -1.3), (-0.7, 0.0)), rho_wall=(0.2, 0.1), collision=collision)
    sim = Sim(rho, tau=p.tau, G=p.G, rho_wall=p.rho_wall, solid=solid, collision=collision)
    sim.set_populations(torch.from_numpy(f.astype(np.float32)))
    x_t = sim.state.clone()
    ck = sim.checkpoint()
    sim.step(1)
    plain = sim.state.clone()
    sim.restore(ck)
    fields = sim.step_fields()
    assert torch.equal(sim.state, plain) and sim.t == ck[1] + 1
    # the fields against the oracle's moments of the same pre-collision f
    fl = fields.view(5, *shape).cpu().numpy().astype(np.float64)
    m = olbm.macroscopic(f, p, solid)
    fluid = olbm.fluid_mask(shape, solid)
    for a in range(2):
        assert np.max(np.abs(fl[a] - m["rho_s"][a])[fluid]) <= 1e-5 * np.max(m["rho_s"][a])
    assert np.max(np.abs(fl[2:] - m["u"])[:, fluid]) <= 1e-5 * max(1.0, np.max(np.abs(m["u"])))
    if solid is not None:
        assert np.all(fl[0][solid] == np.float32(0.2)) and np.all(fl[1][solid] == np.float32(0.1))
        assert np.all(fl[2:][:, solid] == 0.0)
    # reverse step with and without the fields
    lam1 = np.random.default_rng(32).normal(size=f.shape).astype(np.float32)
    if solid is not None:
        lam1[:, :, solid] = 0.0
    lam_in = to_adjoint_layout(torch.from_numpy(lam1).cuda(), sim)
    live = sim.live_mask(sim.lam_layout)
    for shp in (-1, 0, 1, 2, 3):
        sim.set_adjoint_tiling(shp, 0)
        r0, r1 = Reverse(sim), Reverse(sim)
        a, da = r0.step(x_t, lam_in, want_drho0=True)
        b, db = r1.step(x_t, lam_in, want_drho0=True, fields=fields)
        torch.cuda.synchronize()
        assert torch.equal(a[live], b[live]) and torch.equal(da, db), shp
        np.testing.assert_allclose(r1.dparams.cpu().numpy(), r0.dparams.cpu().numpy(), rtol=1e-12, atol=0)
    sim.close()


def test_step_fields_refusals(lib):
    """16-bit storage has no fields step (its reverse step reads an FP32 copy
    of X_t); null or aliased buffers are refused."""
    import ctypes
    from paper_1601_01237_amd.sim import Sim
    rho0 = inputs.sphere_droplet((8, 8, 8), radius=2.0, seed=1)
    buf = torch.empty(5 * 512, dtype=torch.float32, device="cuda")
    for kw in (dict(storage="fp16"), dict(storage="bf16")):
        s = Sim(rho0, **kw)
        assert s.lib.lbm_step_fields(s.ctx, ctypes.c_void_p(buf.data_ptr())) == -5
        s.close()
    s = Sim(rho0)
    assert s.lib.lbm_step_fields(s.ctx, None) == -1
    assert s.lib.lbm_step_fields(s.ctx, ctypes.c_void_p(s.state.data_ptr())) == -1
    assert s.t == 0
    s.close()


@pytest.mark.parametrize("collision", ["bgk", "regularized", "regularized3"])
@pytest.mark.parametrize("storage,walls", [("fp16", None), ("bf16", None), ("fp16", "obstacle"), ("bf16", "porous")])
def test_16bit_reverse_step(lib, storage, walls, collision):
    """The reverse step of a 16-bit context is the FP32 reverse step at the
    populations its stored state decodes to: bitwise that of an FP32 context
    holding those populations, and the oracle's transpose at them.  Folded
    rows (even nx, no walls) and unfolded rows, class bytes and link words."""
    from paper_1601_01237_amd.autograd import Reverse, from_adjoint_layout, to_adjoint_layout
    from paper_1601_01237_amd.sim import Sim
    say(f"16-bit reverse step {storage} walls={walls} {collision}")
    shape = (7, 9, 70)
    solid = None
    if walls == "obstacle":
        solid = np.zeros(shape, bool)
        solid[0] = True
        solid[3, 2:6, 10:30] = True
    elif walls == "porous":
        solid = np.random.default_rng(23).uniform(size=shape) < 0.3
        solid[0] = True
    f, rho = _random_state(shape, 5, solid)
    if solid is not None:
        rho[:, solid] = 0.0
    p = olbm.Params(tau=(0.8, 1.3), G=((0.0, -1.4), (-0.6, 0.0)), rho_wall=(0.15, 0.35), collision=collision)
    kw = dict(tau=p.tau, G=p.G, rho_wall=p.rho_wall, solid=solid, collision=collision)
    s16 = Sim(rho, storage=storage, **kw)
    assert (s16.row_half > 0) == (walls is None)
    s16.set_populations(torch.from_numpy(f.astype(np.float32)))
    f16 = s16.populations().cpu().numpy()          # what the 16-bit step pulls
    s32 = Sim(rho, storage="fp32", **kw)
    s32.set_populations(torch.from_numpy(f16))
    assert np.array_equal(s32.populations().cpu().numpy(), f16)
    lam1 = np.random.default_rng(6).normal(size=f.shape)
    if solid is not None:
        lam1[:, :, solid] = 0.0
    lam1 = lam1.astype(np.float32)
    lam_in = to_adjoint_layout(torch.from_numpy(lam1).cuda(), s32)
    r16, r32 = Reverse(s16), Reverse(s32)
    assert r16.work.numel() > r32.work.numel()     # the FP32 copy of X_t
    a, da = r16.step(s16.state, lam_in, want_drho0=True)
    b, db = r32.step(s32.state, lam_in, want_drho0=True)
    torch.cuda.synchronize()
    live = s32.live_mask(s32.lam_layout)
    assert torch.equal(a[live], b[live]) and torch.equal(da, db)
    np.testing.assert_array_equal(r16.dparams.cpu().numpy(), r32.dparams.cpu().numpy())
    got = from_adjoint_layout(a, s32).cpu().numpy()
    mu, _, _ = oadj.collide_adjoint(f16.astype(np.float64), lam1.astype(np.float64), p, solid)
    want = oadj.stream_adjoint(mu, solid)
    e = rel_err(got, want)
    assert e < 1e-5, e
    # the fields path stays FP32-only
    fl = torch.zeros(5 * s16.n, dtype=torch.float32, device="cuda")
    assert s16.lib.lbm_adjoint_step_fields(
        s16.ctx, ctypes.c_void_p(s16.state.data_ptr()), ctypes.c_void_p(fl.data_ptr()),
        ctypes.c_void_p(lam_in.data_ptr()), ctypes.c_void_p(a.data_ptr()), ctypes.c_void_p(r16.work.data_ptr()),
        ctypes.c_size_t(r16.work.numel()), ctypes.c_void_p(r16.dparams.data_ptr()), None) == -5
    s16.close()
    s32.close()


@pytest.mark.parametrize("storage,tol", [("fp16", 1e-3), ("bf16", 1e-2)])
def test_16bit_calibration_gradient_16cube(lib, storage, tol):
    """The calibration gradient of a 16-bit run (16^3, 200 steps, checkpoints
    every 50) against the FP64 oracle's gradient of the exact run: the
    forward's storage rounding (2^-11 of a stored deviation for FP16, 2^-8
    for BF16, per step) is all that separates them.  Measured: at most 6e-5
    (FP16) and 3e-4 (BF16); the bounds sit an order of magnitude above,
    the FP16 one ten times inside the 1e-2 the FP16 forward is held to."""
    from paper_1601_01237_amd.autograd import LBMFunction
    say(f"16-bit calibration gradient 16^3 x 200 {storage}")
    n, steps, every = 16, 200, 50
    rho0, target = _calibration_inputs(n)
    G, tau = -1.0, 1.0
    r0 = torch.tensor(rho0, device="cuda", requires_grad=True)
    Gt = torch.tensor(G, dtype=torch.float64, requires_grad=True)
    Tt = torch.tensor(tau, dtype=torch.float64, requires_grad=True)
    rho = LBMFunction.apply(r0, Gt, Tt, steps, every, None, (0.0, 0.0), "bgk", storage)
    tgt = torch.tensor(target, dtype=torch.float32, device="cuda")
    L = 0.5 * ((rho[0].double() - tgt.double()) ** 2).sum()
    L.backward()
    p = olbm.Params(tau=(tau, tau), G=((0.0, G), (G, 0.0)))
    L_ref, dG_ref, dtau_ref, drho0_ref = oadj.loss_and_gradient(rho0, p, steps, target)
    e_G = abs(float(Gt.grad) - dG_ref) / abs(dG_ref)
    e_t = abs(float(Tt.grad) - dtau_ref) / abs(dtau_ref)
    e_r = rel_err(r0.grad.cpu().numpy(), drho0_ref)
    say(f"16^3 {storage} calibration: dL/dG {e_G:.1e}, dL/dtau {e_t:.1e}, dL/drho0 {e_r:.1e}")
    assert e_G < tol and e_t < tol and e_r < tol, (e_G, e_t, e_r)
