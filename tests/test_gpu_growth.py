"""Error growth past the parity horizon.

Within the first few hundred steps the FP64 library matches the FP64 oracle
to 1e-10; the deposit's atomics reorder sums at the 1e-16 level and the
plasma's dynamics (trapped and crossing electrons) amplify that difference,
so after the horizon the agreement is reported as a curve rather than held to
the parity bar.

* 256 x 64, modes 0..1, 4 ppc (the small benchmark config), FP64 library
  against the FP64 oracle for 1000 steps: max |difference| / max |oracle|
  over every E and B array and mode at steps 100, 200, 500, 1000; the 1e-10
  bar holds through step 200, and at step 1000 (the pulse has crossed the
  16-wavelength periodic box three times) the laser (E_r, m = 1) still agrees
  to 1e-2.
* 8192 x 512, modes 0..3, 16 ppc (67 M electrons), FP32 against the FP64
  library path (the FP64 oracle does not reach this size; the FP64 path is
  the one held to it at 1e-10 elsewhere) for 1000 steps: L2 difference /
  L2 norm of E per mode at steps 10, 100, 1000; at step 10 the laser and
  wake arrays meet the FP32 field bound (1e-4) and every array the current's
  (3e-4), and at step 1000 the laser (E_r, m = 1) agrees to 1e-2 and the wake
  (E_z, m = 0) to 1e-1.
Past the horizon only sanity bounds are asserted (the fields must still be the
same fields); the curves are printed.
"""
import numpy as np
import pytest

import workloads
from test_gpu_fp32 import EBTOL, JTOL
from test_gpu_parity import _pic, _say, _setup, oracle_of

pytestmark = pytest.mark.gpu

EB = ((0, 0), (1, 1), (2, 2), (10, 3), (11, 4), (12, 5), (13, 6), (14, 7), (15, 8))  # (library comp, oracle comp)


def test_fp64_against_oracle_growth_1000_steps():
    _say("[gpu] error growth, fp64 against the oracle, 256x64, 1000 steps")
    pic = _pic()
    run = workloads.config("c1")["runs"][0]
    dt, CE, CB, _ = _setup(16, run["M"], run["dz"], run["dr"])
    sim = pic.Simulation([workloads.to_rundesc(run)], dt=dt, coef_E=CE, coef_B=CB)
    o = oracle_of(run, dt, CE, CB)
    curve, done = {}, 0
    for n in (100, 200, 500, 1000):
        sim.step(n - done)
        o.step(n - done)
        done = n
        errs = {}
        for gc, oc in EB:
            for m in range(run["M"] + 1):
                g, r = sim.fields(gc, m), o.get_field(oc, m)
                errs[(gc, m)] = np.abs(g - r).max() / np.abs(r).max()
        curve[n] = errs
        _say(f"  step {n}: worst {max(errs.values()):.3e}; laser (E_r, m=1) {errs[(pic.ER, 1)]:.3e}, "
             f"wake (E_z, m=0) {errs[(pic.EZ, 0)]:.3e}")
    assert max(curve[100].values()) <= 1e-10 and max(curve[200].values()) <= 1e-10, curve[200]
    assert curve[1000][(pic.ER, 1)] <= 1e-2, curve[1000]
    sim.close()


def test_fp32_against_fp64_growth_1000_steps():
    _say("[gpu] error growth, fp32 against the fp64 path, 8192x512, 1000 steps")
    pic = _pic()
    run = workloads.config("c5")["runs"][0]
    kw = dict(tile_z=16, tile_r=4, sort_interval=16)
    s32 = pic.Simulation([workloads.to_rundesc(run)], precision=pic.PREC_FP32, **kw)
    CE, CB, _ = s32.coefficients()
    s64 = pic.Simulation([workloads.to_rundesc(run)], precision=pic.PREC_FP64, dt=s32.info()["dt"], coef_E=CE,
                         coef_B=CB, **kw)
    curve, done = {}, 0
    for n in (10, 100, 1000):
        s32.step(n - done)
        s64.step(n - done)
        done = n
        errs = {}
        for name, gc in (("E_r", pic.ER), ("E_phi", pic.EPHI), ("E_z", pic.EZ)):
            for m in range(run["M"] + 1):
                a, b = s32.fields(gc, m), s64.fields(gc, m)
                errs[(name, m)] = np.linalg.norm(a - b) / np.linalg.norm(b)
        curve[n] = errs
        wk = max(errs, key=errs.get)
        _say(f"  step {n}: worst {errs[wk]:.3e} ({wk[0]}, m={wk[1]}); laser (E_r, m=1) {errs[('E_r', 1)]:.3e}, "
             f"wake (E_z, m=0) {errs[('E_z', 0)]:.3e}")
    # the laser and wake arrays at the FP32 field bound; every array, including
    # those that hold only the field of the electrons' noise current (E_phi of
    # m = 0, the modes neither the laser nor the wake drive), at the current's
    # bound, since such a field is the integral of that current
    assert max(curve[10][k] for k in (("E_r", 1), ("E_phi", 1), ("E_r", 0), ("E_z", 0))) <= EBTOL, curve[10]
    assert max(curve[10].values()) <= JTOL, curve[10]
    assert curve[1000][("E_r", 1)] <= 1e-2 and curve[1000][("E_z", 0)] <= 1e-1, curve[1000]
    s32.close()
    s64.close()
