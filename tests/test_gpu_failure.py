"""Failure detection: a run that turns non-finite raises LBM_EUNSTABLE.

The check reads the diagnostic vector of the fused moments kernel (count of
fluid cells with a non-finite density or velocity).  Forced from the host:
a NaN written into the initial density field, and parameters for which the
FP64 oracle itself diverges (tau = 0.51, G = -3, pinned on the CPU in
test_oracle_diagnostics).  Recovery is a restore of a checkpoint taken
before the failure.
"""

import numpy as np
import pytest
import torch

from paper_1601_01237_amd import inputs

from ._gpu_util import say

pytestmark = pytest.mark.gpu


def test_nan_in_initial_field_is_reported(lib):
    from paper_1601_01237_amd import _lib
    from paper_1601_01237_amd.sim import Sim
    say("NaN injected into rho0")
    rho0 = inputs.sphere_droplet((10, 12, 14), radius=3.0, seed=2)
    rho0[0, 4, 5, 6] = np.nan
    sim = Sim(rho0, tau=(1.0, 1.0), G=-1.0)
    with pytest.raises(_lib.LBMError) as e:
        sim.run(3, check_every=1)
    assert e.value.code == _lib.EUNSTABLE
    assert sim.t == 1
    sim.close()


@pytest.mark.parametrize("storage", ["fp32", "fp16"])
def test_divergent_parameters_raise_and_checkpoint_recovers(lib, storage):
    from paper_1601_01237_amd import _lib
    from paper_1601_01237_amd.sim import Sim
    say(f"divergent run {storage}")
    rho0 = inputs.sphere_droplet((12, 12, 12), radius=4.0, seed=0)
    sim = Sim(rho0, tau=(0.51, 0.51), G=-3.0, storage=storage)
    sim.run(2, check_every=1)
    ck = sim.checkpoint()
    with pytest.raises(_lib.LBMError) as e:
        sim.run(60, check_every=1)
    assert e.value.code == _lib.EUNSTABLE
    assert 2 < sim.t <= 62
    sim.restore(ck)
    assert sim.t == 2
    assert torch.equal(sim.state, ck[0])
    sim.check_finite()
    sim.close()


def test_stable_run_passes_the_check(lib):
    from paper_1601_01237_amd.sim import Sim
    say("stable run with checks")
    rho0 = inputs.sphere_droplet((12, 12, 12), radius=4.0, seed=0)
    sim = Sim(rho0, tau=(1.0, 1.0), G=-1.0)
    sim.run(20, check_every=7)
    assert sim.t == 20
    sim.close()
