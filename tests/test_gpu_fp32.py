"""FP32 form against the FP64 oracle.

The oracle starts from the same FP32-rounded initial state (particles as
int32 cell + FP32 offset, FP32 momenta/weights, FP32 E^0 and B^0), so only
the arithmetic of the FP32 path is measured.  Bounds, per quantity:
  * E and B error (L2 over the grid) per component and mode <= 1e-4 of that
    array's L2 norm;
  * current J <= 3e-4: an electron's current comes from the difference of
    its FP32 cell offsets before and after the move (that is what keeps the
    deposit exactly consistent with the stored positions), whose rounding is
    ~2^-24 absolute against moves of 1e-2..1e-1 cell per step -- about 1e-5
    to 1e-4 relative per electron, summed in an order the atomics choose;
    measured 6e-5..1e-4 on config 3, against a few 1e-5 for E and B, which
    integrate J;
  * tracked-electron energy gamma (FP64 accumulation): p99 error <= 1e-4 and
    max <= 1e-3 of max(gamma_oracle - 1, 1e-3);
  * per-mode work: |dW_m| <= 1e-3 max_p |W_m| + 1e-7.
"""
import numpy as np
import pytest

import workloads
from test_gpu_parity import FIELD_PAIRS, _pic, _say, _setup, oracle_of

pytestmark = pytest.mark.gpu


JTOL, EBTOL = 3e-4, 1e-4


def check_fields(field_err):
    """per-quantity field bounds: currents J, then E and B"""
    for (name, m), v in field_err.items():
        assert v <= (JTOL if name.startswith("J") else EBTOL), (name, m, v)


def fp32_errors(run, nsteps, sort_interval=0):
    pic = _pic()
    dt, CE, CB, _ = _setup(16, run["M"], run["dz"], run["dr"])
    sim = pic.Simulation([workloads.to_rundesc(run)], precision=pic.PREC_FP32, dt=dt, coef_E=CE, coef_B=CB,
                         sort_interval=sort_interval)
    o = oracle_of(run, dt, CE, CB, fp32_start=True)
    sim.step(nsteps)
    o.step(nsteps)
    field_err = {}
    for name, comp, ocomp in FIELD_PAIRS:
        for m in range(run["M"] + 1):
            g, r = sim.fields(comp, m), o.get_field(ocomp, m)
            nr = np.linalg.norm(r)
            field_err[(name, m)] = np.linalg.norm(g - r) / nr if nr > 0 else np.linalg.norm(g)
    wg, wo = sim.mode_work(), o.tracked()
    assert np.array_equal(wg["id"], wo["id"])
    scale = np.maximum(wo["gamma_acc"] - 1.0, 1e-3)
    gerr = np.abs(wg["gamma_acc"] - wo["gamma_acc"]) / scale
    werr = np.abs(wg["W"] - wo["W"])
    wtol = 1e-3 * np.abs(wo["W"]).max(axis=0) + 1e-7
    # the direction split (Eq. (17)) to the per-mode work's bar
    cg, co = sim.cartesian_work(corrected=False), o.cartesian_work()
    for k in ("Wz", "Wperp"):
        assert np.all(np.abs(cg[k] - co[k]) <= 1e-3 * np.abs(co[k]).max() + 1e-7), k
    # the FP32 instantiation of the divergence reduction on the run's own state
    from oracle import beam

    pg = sim.particles()
    dg, rs = sim.divergence(1.0), beam.divergence(pg, 1.0)
    assert dg["count"] == rs["count"]
    for k in ("w", "sum_wtx2", "sum_wty2"):
        if rs["count"] == 0:  # nothing selected (no laser: the cold plasma has no forward electron)
            assert dg[k] == 0.0 and rs[k] == 0.0, k
        else:
            assert abs(dg[k] / rs[k] - 1) < 1e-12, k
    sim.close()
    return field_err, gerr, werr, wtol


def test_fp32_config3_per_quantity_bounds():
    _say("[gpu] fp32 config c3 (256x64, modes 0..1), 100 steps")
    cfg = workloads.config("c3")
    run = cfg["runs"][0]
    field_err, gerr, werr, wtol = fp32_errors(run, cfg["steps"])
    worst = max(field_err.values())
    _say(f"  field L2 worst {worst:.3e}: " + ", ".join(f"{k[0]}/{k[1]} {v:.1e}" for k, v in field_err.items()))
    _say(f"  gamma p99 {np.percentile(gerr, 99):.3e} max {gerr.max():.3e}; work max/tol "
         f"{(werr / wtol).max():.3e}")
    check_fields(field_err)
    assert np.percentile(gerr, 99) <= 1e-4 and gerr.max() <= 1e-3
    assert np.all(werr <= wtol)


@pytest.mark.parametrize("M", [0, 2, 3])
def test_fp32_small_grid_bounds(M):
    _say(f"[gpu] fp32 small grid M={M}")
    run = workloads.small(M=M, Nz=64, Nr=12, ppc=2, n_tracked=40)["runs"][0]
    field_err, gerr, werr, wtol = fp32_errors(run, 20)
    worst = max(field_err.values())
    _say(f"  field L2 worst {worst:.3e}, gamma max {gerr.max():.3e}")
    check_fields(field_err)
    assert gerr.max() <= 1e-3
    assert np.all(werr <= wtol)


def test_fp32_smallest_grid_bounds():
    """The smallest grid accepted (32 x 4) in FP32, every electron tracked."""
    _say("[gpu] fp32 smallest grid")
    run = workloads.small(M=1, Nz=32, Nr=4, ppc=3, n_tracked=0)["runs"][0]
    run["n_tracked"] = 32 * 3 * 3
    field_err, gerr, werr, wtol = fp32_errors(run, 25)
    check_fields(field_err)
    assert gerr.max() <= 1e-3
    assert np.all(werr <= wtol)
