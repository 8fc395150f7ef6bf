"""GPU parity of the batched form: several runs of different grids, cell
sizes and step limits in one context (one launch per phase for all of them),
each against its own FP64 oracle, and captured-graph replay against eager
stepping.

Every run of a context shares the solver options, so the runs here share the
oracle's coefficients and dt fitted for the finest cell (the coarser runs are
then further below their Courant limit); each oracle gets the identical
inputs.  Bar as in the single-run FP64 parity tests: 1e-10 per field array
and mode, positions and momenta.
"""
import sys

import numpy as np
import pytest

import workloads
from test_gpu_parity import (TOL64, _pic, _say, _setup, compare_cartesian_work, compare_fields, compare_particles,
                             oracle_of)

pytestmark = pytest.mark.gpu


def _runs():
    """Three small runs: different dz (so different c dt/dz), grids, seeds."""
    out = []
    for r, (ppl, Nz, Nr, ppc) in enumerate(((16, 64, 12, 2), (20, 80, 14, 3), (24, 96, 16, 2))):
        run = workloads.small(M=2, Nz=Nz, Nr=Nr, ppc=ppc, seed=700 + r, n_tracked=30)["runs"][0]
        run["dz"] = workloads.LAMBDA0 / ppl
        run["dr"] = 4 * run["dz"]
        out.append(run)
    return out


def test_batched_runs_with_step_limits_match_oracles():
    """Runs stepped together stop at their own limits and each matches its
    oracle stepped the same number of times."""
    _say("[gpu] batched runs with step limits")
    pic = _pic()
    runs = _runs()
    dt, CE, CB, _ = _setup(16, 2, runs[-1]["dz"], runs[-1]["dr"])  # finest cell sets dt
    limits = [12, 20, 0]
    sim = pic.Simulation([workloads.to_rundesc(r, n_steps=n) for r, n in zip(runs, limits)], dt=dt, coef_E=CE,
                         coef_B=CB)
    sim.step(20)
    for i, (run, lim) in enumerate(zip(runs, limits)):
        steps = lim or 20
        assert sim.info(i)["steps_done"] == steps
        o = oracle_of(run, dt, CE, CB)
        o.step(steps)
        worst = compare_fields(sim, o, run["M"], TOL64, run=i)
        bad = {k: v for k, v in worst.items() if v > TOL64}
        assert not bad, (i, bad)
        dzmax, dxy, du, _ = compare_particles(sim, o, run["Nz"], run=i)
        assert dzmax < TOL64 and dxy < TOL64 and du < TOL64, (i, dzmax, dxy, du)
        wg, wo = sim.mode_work(i), o.tracked()
        assert np.array_equal(wg["id"], wo["id"])
        scale = max(np.abs(wo["W"]).max(), 1e-300)
        assert np.abs(wg["W"] - wo["W"]).max() / scale < TOL64, i
        cw = compare_cartesian_work(sim, o, run, TOL64, i)
        assert max(cw.values()) < TOL64, (i, cw)
    sim.close()


def test_graph_replay_matches_eager_and_oracle():
    """Two identical batched contexts, one stepping eagerly and one replaying
    captured graphs, advanced in chunks with reads and syncs in between (sorts
    every 4 steps, so the replays cross sorted and unsorted steps of both
    parities); every chunk agrees to 1e-12, and the end state matches the
    oracles to 1e-10."""
    _say("[gpu] graph replay vs eager")
    pic = _pic()
    runs = _runs()[:2]
    dt, CE, CB, _ = _setup(16, 2, runs[-1]["dz"], runs[-1]["dr"])
    descs = [workloads.to_rundesc(r) for r in runs]
    eager = pic.Simulation(descs, dt=dt, coef_E=CE, coef_B=CB, sort_interval=4)
    graph = pic.Simulation(descs, dt=dt, coef_E=CE, coef_B=CB, sort_interval=4, use_graph=True)
    done = 0
    for chunk in (3, 5, 6, 4):
        eager.step(chunk)
        graph.step(chunk)
        done += chunk
        for i, run in enumerate(runs):
            for comp in (0, 1, 2, 6, 7, 8, 13, 14, 15):
                for m in range(run["M"] + 1):
                    a, b = eager.fields(comp, m, i), graph.fields(comp, m, i)
                    scale = max(np.abs(a).max(), 1e-300)
                    assert np.abs(a - b).max() / scale < 1e-12, (done, i, comp, m)
        _say(f"  chunk to step {done} agrees")
    for i, run in enumerate(runs):
        o = oracle_of(run, dt, CE, CB)
        o.step(done)
        worst = compare_fields(graph, o, run["M"], TOL64, run=i)
        bad = {k: v for k, v in worst.items() if v > TOL64}
        assert not bad, (i, bad)
    eager.close()
    graph.close()


def test_autotune_reports_candidates_and_choice_keeps_parity():
    """The autotuner times every fitting candidate tile on the GPU, returns
    the cheapest (tile, interval), and a run with that choice still matches
    the oracle (the choice changes no physics)."""
    _say("[gpu] autotune")
    pic = _pic()
    runs = _runs()[:2]
    dt, CE, CB, _ = _setup(16, 2, runs[-1]["dz"], runs[-1]["dr"])
    descs = [workloads.to_rundesc(r) for r in runs]
    t = pic.autotune(descs, dt=dt, coef_E=CE, coef_B=CB, trial_steps=8)
    cands = t["candidates"]
    assert len(cands) >= 4
    assert all(ms > 0 and 1 <= k <= 8 for _, _, k, ms in cands)
    best = min(cands, key=lambda c: c[3])
    assert (t["tile_z"], t["tile_r"], t["sort_interval"]) == best[:3]
    _say(f"  chose {best}")
    sim = pic.Simulation(descs, dt=dt, coef_E=CE, coef_B=CB, tile_z=t["tile_z"], tile_r=t["tile_r"],
                         sort_interval=t["sort_interval"])
    sim.step(12)
    for i, run in enumerate(runs):
        o = oracle_of(run, dt, CE, CB)
        o.step(12)
        worst = compare_fields(sim, o, run["M"], TOL64, run=i)
        bad = {k: v for k, v in worst.items() if v > TOL64}
        assert not bad, (i, bad)
    sim.close()


def test_empty_run_beside_a_full_one():
    """A run with no electrons (ppc = 0: a laser in vacuum) in one context with
    a populated run: the empty run's fields match its oracle (the current
    stays zero), its diagnostics are empty or zero, and the populated run
    matches its own oracle."""
    _say("[gpu] empty run beside a full one")
    pic = _pic()
    empty = workloads.small(M=2, Nz=64, Nr=12, ppc=2, seed=11, n_tracked=0)["runs"][0]
    empty["ppc"] = 0
    full = workloads.small(M=2, Nz=80, Nr=10, ppc=2, seed=12, n_tracked=20)["runs"][0]
    dt, CE, CB, _ = _setup(16, 2, full["dz"], full["dr"])
    sim = pic.Simulation([workloads.to_rundesc(empty), workloads.to_rundesc(full)], dt=dt, coef_E=CE, coef_B=CB)
    assert sim.info(0)["n_particles"] == 0
    sim.step(15)
    o = oracle_of(empty, dt, CE, CB)
    o.step(15)
    worst = compare_fields(sim, o, 2, TOL64, run=0)
    bad = {k: v for k, v in worst.items() if v > TOL64}
    assert not bad, bad
    assert all(np.abs(sim.fields(c, m, 0)).max() == 0 for c in (pic.JR, pic.JPHI, pic.JZ, pic.RHO) for m in range(3))
    assert np.abs(sim.fields(pic.EPHI, 1, 0)).max() > 0.1  # the laser is there
    assert sim.particles(0)["z"].size == 0
    mw = sim.mode_work(0)
    assert mw["id"].size == 0 and mw["kinetic"] == 0.0
    assert sim.divergence(1.0, 0)["count"] == 0
    o = oracle_of(full, dt, CE, CB)
    o.step(15)
    worst = compare_fields(sim, o, 2, TOL64, run=1)
    bad = {k: v for k, v in worst.items() if v > TOL64}
    assert not bad, bad
    dzmax, dxy, du, _ = compare_particles(sim, o, full["Nz"], run=1)
    assert dzmax < TOL64 and dxy < TOL64 and du < TOL64, (dzmax, dxy, du)
    sim.close()
