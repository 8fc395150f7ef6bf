"""The allocation-free entry point pic_divergence_arrays against the entry
point it varies, pic_divergence, through the C ABI: the same electrons (a
run's state after a few steps of a strong pulse, copied to device arrays of
the run's precision) give the same divergence sums, to the reduction order
(1e-12 relative) with the count exact.  Two calls in a row on one GPU, the
second with fewer electrons, so that the second reuses the fixed scratch
the first left filled; in FP64 and FP32."""
import numpy as np
import pytest

import workloads
from test_gpu_parity import _pic, _say, energetic_cut

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("precision", [64, 32])
def test_allocation_free_divergence_matches_pic_divergence(precision):
    import torch

    pic = _pic()
    _say(f"[gpu] allocation-free divergence, fp{precision}")
    dev = torch.device("cuda:0")
    dtype = torch.float64 if precision == 64 else torch.float32
    for Nz, Nr in ((96, 16), (48, 8)):  # the second call takes fewer electrons
        run = workloads.small(M=1, Nz=Nz, Nr=Nr, ppc=3, a0=3.0, n_tracked=16)["runs"][0]
        run["pulses"] = [dict(a0=3.0, w0=2 * workloads.LAMBDA0, tau=2 * workloads.LAMBDA0,
                              zc=2 * workloads.LAMBDA0)]
        sim = pic.Simulation([workloads.to_rundesc(run)], precision=precision)
        sim.step(12)
        P = sim.particles()
        g = np.sqrt(1 + P["ux"] ** 2 + P["uy"] ** 2 + P["uz"] ** 2)
        cut, _ = energetic_cut(g, 0.05, 0.2)
        ref = sim.divergence(cut)
        arrs = [torch.tensor(P[k], dtype=dtype, device=dev) for k in ("ux", "uy", "uz", "w")]
        got = pic.divergence_arrays(*arrs, gamma_min=cut)
        _say(f"  {P['ux'].size} electrons, {got['count']} counted, rms_x {got['rms_x']:.4e}")
        assert got["count"] == ref["count"] > 0
        for k in ("w", "sum_wtx2", "sum_wty2", "rms_x", "rms_y"):
            assert abs(got[k] / ref[k] - 1.0) < 1e-12, (k, got[k], ref[k])
        sim.close()
