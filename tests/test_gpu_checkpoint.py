"""Checkpoint and restore through pic_checkpoint / pic_restore: a context
restored from a checkpoint continues like the checkpointed one.

The deposit's atomic additions make two runs of the same steps differ in the
order of their sums, so the continuation is compared to 1e-12 (FP64) and 1e-5
(FP32) of each array's largest value rather than bit for bit; the FP64
continuation must also still match the oracle at the 1e-10 parity bar.
"""
import numpy as np
import pytest

import workloads
from test_gpu_parity import TOL64, _pic, _say, _setup, compare_fields, oracle_of

pytestmark = pytest.mark.gpu

COMPS = (0, 1, 2, 6, 7, 8, 13, 14, 15)


def _max_rel(a, b):
    worst = 0.0
    for i in range(len(a.runs)):
        M = a.runs[i].M
        for comp in COMPS:
            for m in range(M + 1):
                x, y = a.fields(comp, m, i), b.fields(comp, m, i)
                worst = max(worst, np.abs(x - y).max() / max(np.abs(x).max(), 1e-300))
        pa, pb = a.particles(i), b.particles(i)
        assert np.array_equal(pa["id"], pb["id"])  # same order after the restore
        for k in ("z", "x", "y", "ux", "uy", "uz"):
            worst = max(worst, np.abs(pa[k] - pb[k]).max() / max(np.abs(pa[k]).max(), 1e-300))
    return worst


def test_fp64_restore_continues_the_run():
    _say("[gpu] checkpoint fp64")
    pic = _pic()
    run = workloads.small(M=2, Nz=64, Nr=12, ppc=2, n_tracked=40)["runs"][0]
    dt, CE, CB, _ = _setup(16, 2, run["dz"], run["dr"])
    mk = lambda: pic.Simulation([workloads.to_rundesc(run)], dt=dt, coef_E=CE, coef_B=CB, sort_interval=4)
    a = mk()
    a.step(13)
    blob = a.checkpoint()
    a.step(7)
    b = mk()
    b.step(3)  # a different state, overwritten by the restore
    b.restore(blob)
    assert b.info(0)["steps_done"] == 13
    b.step(7)
    assert _max_rel(a, b) < 1e-12
    wa, wb = a.mode_work(), b.mode_work()
    assert np.abs(wa["W"] - wb["W"]).max() <= 1e-12 * np.abs(wa["W"]).max()
    o = oracle_of(run, dt, CE, CB)
    o.step(20)
    worst = compare_fields(b, o, run["M"], TOL64)
    assert max(worst.values()) < TOL64, worst
    a.close()
    b.close()


def test_fp32_batched_restore_and_mismatch():
    _say("[gpu] checkpoint fp32 batched")
    pic = _pic()
    runs = [workloads.small(M=1, Nz=64, Nr=12, ppc=2, seed=900 + r)["runs"][0] for r in range(2)]
    descs = [workloads.to_rundesc(r) for r in runs]
    a = pic.Simulation(descs, precision=pic.PREC_FP32, sort_interval=3)
    a.step(10)
    blob = a.checkpoint()
    a.step(5)
    b = pic.Simulation(descs, precision=pic.PREC_FP32, sort_interval=3)
    b.restore(blob)
    b.step(5)
    assert _max_rel(a, b) < 1e-5
    # a context of other runs refuses the checkpoint and keeps its state
    other = [workloads.to_rundesc(dict(runs[0], seed=7)), descs[1]]
    c = pic.Simulation(other, precision=pic.PREC_FP32, sort_interval=3)
    before = c.fields(2, 0, 0).copy()
    with pytest.raises(pic.PicError):
        c.restore(blob)
    assert np.array_equal(c.fields(2, 0, 0), before)
    for s in (a, b, c):
        s.close()


def test_exact_jz_restore_and_mode_mismatch():
    """A context with the exact J_z correction restores its own checkpoint
    and continues like the original; a context that filters the current
    instead refuses it."""
    _say("[gpu] checkpoint exact J_z")
    pic = _pic()
    run = workloads.small(M=1, Nz=64, Nr=12, ppc=2, n_tracked=10)["runs"][0]
    dt, CE, CB, _ = _setup(16, 1, run["dz"], run["dr"])
    mk = lambda cur: pic.Simulation([workloads.to_rundesc(run)], dt=dt, coef_E=CE, coef_B=CB, sort_interval=4,
                                    current=cur)
    a = mk(pic.CURRENT_EXACT_JZ)
    a.step(9)
    blob = a.checkpoint()
    a.step(6)
    b = mk(pic.CURRENT_EXACT_JZ)
    b.restore(blob)
    b.step(6)
    assert _max_rel(a, b) < 1e-12
    c = mk(pic.CURRENT_FILTER)
    with pytest.raises(pic.PicError):
        c.restore(blob)
    for s in (a, b, c):
        s.close()
