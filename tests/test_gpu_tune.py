"""The autotuner: every launch shape it may pick reproduces the default
shape's S bit for bit, later calls use its choice, and PREC_AUTO follows its
precision choice."""
import numpy as np
import pytest
import torch

import oracle
from paper_1607_00693_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sm():
    from paper_1607_00693_amd import stomsfem
    yield stomsfem
    stomsfem.tuning_reset()


@pytest.mark.parametrize("m,nc,N", [(8, 8, 300), (16, 8, 60), (32, 4, 40)])
def test_autotune_keeps_results(sm, m, nc, N):
    sm.tuning_reset()
    a = torch.from_numpy(W.lognormal_field((N, nc * m, nc * m), 1.0, 4000 + m)).cuda()
    S0 = sm.upscale(a, nc, nc, m)
    S1 = torch.empty_like(S0)
    rep = sm.autotune(a, nc, nc, m, S=S1, reps=2)
    assert rep["m"] == m and rep["candidates"] == (3 if m <= 8 else 2)
    assert rep["lane_block"] in (64, 128, 256) and rep["tiled_waves"] in (1, 2)
    assert 0 < rep["ms_best"] <= rep["ms_default"]
    assert rep["precision"] in (sm.PREC_F64, sm.PREC_F32_REFINE64)
    scale = S0.abs().amax(dim=2)
    if rep["precision"] == sm.PREC_F64:
        assert torch.equal(S1, S0)
    assert float(((S1 - S0).abs().amax(dim=2) / scale).max()) <= 1e-10
    # later calls run the tuned shape (FP64) and the tuned precision (AUTO)
    S2 = sm.upscale(a, nc, nc, m)
    assert torch.equal(S2, S0)
    S3 = sm.upscale(a, nc, nc, m, precision=sm.PREC_AUTO)
    assert float(((S3 - S0).abs().amax(dim=2) / scale).max()) <= 1e-10
    Sr, _, _ = oracle.upscale(a.cpu().numpy(), nc, nc, m)
    assert float((np.abs(S2.cpu().numpy() - Sr).max(-1) / np.abs(Sr).max(-1)).max()) <= 1e-10
    sm.tuning_reset()


def test_autotune_rejects_empty(sm):
    a = torch.zeros((0, 8, 8), dtype=torch.float64, device="cuda")
    with pytest.raises(sm.StomsfemError):
        sm.autotune(a, 1, 1, 8)
