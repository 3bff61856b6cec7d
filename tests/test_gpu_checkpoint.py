"""Checkpoint and resume of a run (Simulation.save / Simulation.restore):
the resumed run continues bit for bit as the uninterrupted one, in FP64 and
in FP32 storage, with the moving cloud."""
import pytest
import torch

import paper_2408_02350_amd.bgk as bgk
from paper_2408_02350_amd.inputs import CONFIGS, CavityConfig

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


@pytest.mark.parametrize("cav,precision", [
    (CONFIGS["c1"], "fp64"),
    (CavityConfig("t3d_n7_v8", 3, 7, 8, 4.0, 2.2, 1.0, 0.1, 1, 1), "fp32"),
])
def test_resumed_run_matches_the_uninterrupted_one(cav, precision, tmp_path):
    a = bgk.Simulation(cav.replace(precision=precision), precision=precision, device=DEV)
    a.step(3)
    path = tmp_path / "ck.pt"
    a.save(path)
    a.step(4)
    bgk.bgk_check(a.ctx)
    b = bgk.Simulation.restore(path, device=DEV)
    assert b.steps == 3 and b.cfg.precision == a.cfg.precision
    b.step(4)
    bgk.bgk_check(b.ctx)
    assert b.steps == a.steps == 7
    for name in ("f", "x", "U", "rho", "T"):
        assert torch.equal(getattr(a, name), getattr(b, name)), name
