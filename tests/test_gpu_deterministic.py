"""The deterministic FP64 mode (pic_opts.deterministic): the deposit's sums
are integer pairs, so a run's results do not depend on the order the atomics
run in.

* Parity: against the oracle at the FP64 bar (1e-10), on a small grid and on
  the push's out-of-window path (electrons far from their sort tile).
* Bitwise reproducibility: the same run with different sort tiles and sort
  intervals (which change which workgroup deposits which electron, and in
  what order), eagerly and from captured graphs, and continued from a
  checkpoint, gives identical fields, electrons and tracked work, bit for
  bit.  The plain FP64 mode is compared too: there the atomics' order shows
  in the last bits, so the same pair of runs differs, which the test records
  (not asserts: equal bits by chance are possible on tiny runs).
"""
import numpy as np
import pytest

import workloads
from test_gpu_parity import FIELD_PAIRS, TOL64, _pic, _say, _setup, compare_fields, compare_particles, oracle_of

pytestmark = pytest.mark.gpu


def _run():
    run = workloads.small(M=2, Nz=64, Nr=12, ppc=3, a0=2.5, n_tracked=64)["runs"][0]
    run["pulses"] = [dict(a0=2.5, w0=3 * workloads.LAMBDA0, tau=4 * workloads.LAMBDA0, zc=2 * workloads.LAMBDA0)]
    return run


def _state(sim, run):
    """Every field array and mode, the electrons in id order, the tracked work."""
    out = {}
    for name, comp, _ in FIELD_PAIRS:
        for m in range(run["M"] + 1):
            out[f"{name}/{m}"] = sim.fields(comp, m)
    P = sim.particles()
    order = np.argsort(P["id"])
    for k in ("z", "x", "y", "ux", "uy", "uz"):
        out["p_" + k] = P[k][order]
    w = sim.mode_work()
    out["W"], out["gamma_acc"] = w["W"], w["gamma_acc"]
    return out


def _same_bits(a, b):
    return all(np.array_equal(a[k].view(np.uint8), b[k].view(np.uint8)) for k in a)


def _sim(pic, run, dt, CE, CB, **kw):
    return pic.Simulation([workloads.to_rundesc(run)], dt=dt, coef_E=CE, coef_B=CB, **kw)


def test_deterministic_matches_oracle():
    _say("[gpu] deterministic fp64 against the oracle")
    pic = _pic()
    run = _run()
    dt, CE, CB, _ = _setup(16, run["M"], run["dz"], run["dr"])
    for kw in (dict(), dict(tile_z=8, tile_r=1, sort_interval=1000)):  # the second: mostly out-of-window
        sim = _sim(pic, run, dt, CE, CB, deterministic=True, **kw)
        o = oracle_of(run, dt, CE, CB)
        sim.step(24)
        o.step(24)
        worst = compare_fields(sim, o, run["M"], TOL64)
        bad = {k: v for k, v in worst.items() if v > TOL64}
        assert not bad, (kw, bad)
        dzmax, dxy, du, _ = compare_particles(sim, o, run["Nz"])
        assert dzmax < TOL64 and dxy < TOL64 and du < TOL64, (kw, dzmax, dxy, du)
        wg, wo = sim.mode_work(), o.tracked()
        assert np.abs(wg["W"] - wo["W"]).max() <= TOL64 * max(np.abs(wo["W"]).max(), 1e-300)
        _say(f"  {kw or 'default tiles'}: worst array {max(worst.values()):.2e}")
        sim.close()


def test_deterministic_is_bitwise_reproducible():
    """Tiles, sort intervals, graphs and a checkpoint do not change a bit."""
    _say("[gpu] deterministic fp64, bitwise across tiles, sort intervals, graphs and a checkpoint")
    pic = _pic()
    run = _run()
    dt, CE, CB, _ = _setup(16, run["M"], run["dz"], run["dr"])
    n = 24
    settings = [dict(), dict(tile_z=8, tile_r=1, sort_interval=1000), dict(tile_z=16, tile_r=4, sort_interval=3),
                dict(tile_z=24, tile_r=2, sort_interval=5, use_graph=True)]
    ref = None
    for kw in settings:
        sim = _sim(pic, run, dt, CE, CB, deterministic=True, **kw)
        sim.step(n)
        st = _state(sim, run)
        sim.close()
        if ref is None:
            ref = st
        else:
            assert _same_bits(ref, st), kw
    # checkpoint after 10 steps, restore into a fresh context, continue
    a = _sim(pic, run, dt, CE, CB, deterministic=True, use_graph=True)
    a.step(10)
    blob = a.checkpoint()
    a.close()
    b = _sim(pic, run, dt, CE, CB, deterministic=True, use_graph=True)
    b.restore(blob)
    b.step(n - 10)
    assert _same_bits(ref, _state(b, run))
    b.close()
    # the plain FP64 mode, for the record: the same two tilings
    plain = []
    for kw in settings[:2]:
        sim = _sim(pic, run, dt, CE, CB, **kw)
        sim.step(n)
        plain.append(_state(sim, run))
        sim.close()
    diff = max(np.abs(plain[0][k] - plain[1][k]).max() for k in plain[0])
    _say(f"  plain FP64, two tilings: largest difference {diff:.3e} (deterministic: 0)")


def test_deterministic_quadratic_shapes():
    """The deterministic mode with quadratic shapes (the fold of row r_{-1}
    done on the integer pairs): against the oracle's quadratic shapes at the
    FP64 bar, and bitwise the same across sort tiles, sort intervals (8 x 1
    tiles never re-sorted: most electrons on the device-memory path), graph
    replay and a checkpoint."""
    _say("[gpu] deterministic fp64 with quadratic shapes")
    pic = _pic()
    run = _run()
    dt, CE, CB, _ = _setup(16, run["M"], run["dz"], run["dr"])
    n = 24
    sim = _sim(pic, run, dt, CE, CB, deterministic=True, shape=2)
    o = oracle_of(run, dt, CE, CB)
    o.set_shape(2)
    sim.step(n)
    o.step(n)
    worst = compare_fields(sim, o, run["M"], TOL64)
    bad = {k: v for k, v in worst.items() if v > TOL64}
    assert not bad, bad
    dzmax, dxy, du, _ = compare_particles(sim, o, run["Nz"])
    assert dzmax < TOL64 and dxy < TOL64 and du < TOL64, (dzmax, dxy, du)
    ref = _state(sim, run)
    sim.close()
    for kw in (dict(tile_z=8, tile_r=1, sort_interval=1000), dict(tile_z=16, tile_r=4, sort_interval=3),
               dict(tile_z=24, tile_r=2, sort_interval=5, use_graph=True)):
        sim = _sim(pic, run, dt, CE, CB, deterministic=True, shape=2, **kw)
        sim.step(n)
        assert _same_bits(ref, _state(sim, run)), kw
        sim.close()
    a = _sim(pic, run, dt, CE, CB, deterministic=True, shape=2)
    a.step(10)
    blob = a.checkpoint()
    a.close()
    b = _sim(pic, run, dt, CE, CB, deterministic=True, shape=2)
    b.restore(blob)
    b.step(n - 10)
    assert _same_bits(ref, _state(b, run))
    b.close()
