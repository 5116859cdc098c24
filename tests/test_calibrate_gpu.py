"""The matrix-core calibration hook (a measurement aid, no part of the method): it runs, it is
deterministic, its accumulators grow linearly with the iteration count (so the MFMAs are executed,
not removed), and bad arguments raise."""
import pytest
import torch

import paper_2307_12041_amd as pp

pytestmark = pytest.mark.gpu


def test_calibration_runs_deterministically_and_accumulates():
    wg = 256
    out1 = torch.empty(wg * 256, dtype=torch.float32, device="cuda:0")
    out1b = torch.empty_like(out1)
    out2 = torch.empty_like(out1)
    pp.mfma_calibrate(out1, workgroups=wg, iters=1)
    pp.mfma_calibrate(out1b, workgroups=wg, iters=1)
    pp.mfma_calibrate(out2, workgroups=wg, iters=2)
    torch.cuda.synchronize()
    assert torch.isfinite(out1).all() and torch.isfinite(out2).all()
    assert torch.equal(out1, out1b)
    assert out1.abs().max() > 0
    # two iterations accumulate the same products twice: exactly twice the sums in exact arithmetic,
    # within fp32 rounding of the 16 x 16 accumulator sums here
    torch.testing.assert_close(out2, 2.0 * out1, rtol=1e-4, atol=1e-3 * float(out1.abs().max()))


def test_calibration_rejects_bad_arguments():
    out = torch.empty(256, dtype=torch.float32, device="cuda:0")
    with pytest.raises(ValueError):
        pp.mfma_calibrate(out, workgroups=2, iters=1)
    with pytest.raises(pp.PPError):
        pp.mfma_calibrate(out, workgroups=1, iters=0)
    with pytest.raises(TypeError):
        pp.mfma_calibrate(out.double(), workgroups=1, iters=1)
