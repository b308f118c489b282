"""The named workload presets run end to end and write their records."""

import json

import pytest

from ._gpu_util import say

pytestmark = pytest.mark.gpu


def test_c1_and_c5_presets_write_jsonl(lib, tmp_path):
    from paper_1601_01237_amd import configs
    say("presets C1, C5 (48^3)")
    out = tmp_path / "runs.jsonl"
    configs.main(["C1", "--jsonl", str(out)])
    rec = json.loads(out.read_text().splitlines()[0])
    assert rec["config"] == "C1" and rec["steps"] == 200 and rec["nonfinite"] == 0
    assert rec["mass_drift_a"] < 1e-6 and rec["mass_drift_b"] < 1e-6 and rec["mlups"] > 0
    r5 = configs.c5(n=48, steps=40, every=10)[0]
    assert r5["config"] == "C5" and r5["loss"] > 0 and r5["dL_drho0_norm"] > 0
    assert r5["dL_dG"] == r5["dL_dG"] and r5["dL_dtau"] == r5["dL_dtau"]  # finite, not NaN
