"""GPU parity of the moving window (App. A) against the oracle's window.

Both sides take the same cadence (a move before every step whose count of
steps taken is a positive multiple of K, by the cells a light-speed front
crossed), shift the fields with fresh vacuum at the front and a cleared guard
band at the back, drop the electrons outside the box and load the new
columns' plasma from the same counter-based draws.  The library loads those
columns on the host with the formulas of its initial load, appends them to
the particle arrays and drops the electrons in the step's cell sort; the
electron count then varies.  Checked: every field array and mode, every
electron by id (positions unwrapped), the count, the cells moved, and the
tracked electrons (work, gamma, and NaN gamma once dropped) -- FP64 to the
1e-10 bar, FP32 to the per-quantity FP32 bounds, and the fresh plasma of a
run at rest bit for bit.
"""
import math

import numpy as np
import pytest

import workloads
from test_gpu_fp32 import EBTOL, JTOL
from test_gpu_parity import TOL64, _pic, _say, _setup, compare_fields, oracle_of

pytestmark = pytest.mark.gpu


def _window_pair(run, nsteps, K, guard, precision=64, sort_interval=0):
    pic = _pic()
    dt, CE, CB, _ = _setup(16, run["M"], run["dz"], run["dr"])
    sim = pic.Simulation([workloads.to_rundesc(run)], precision=precision, dt=dt, coef_E=CE, coef_B=CB,
                         sort_interval=sort_interval, window_interval=K, window_guard=guard)
    o = oracle_of(run, dt, CE, CB, fp32_start=(precision == 32))
    o.set_window(K, 1.0, guard)
    sim.step(nsteps)
    o.step(nsteps)
    return sim, o, dt


def _particles_by_id(sim, o):
    P, Q = sim.particles(), o.particles()
    a, b = np.argsort(P["id"]), np.argsort(Q["id"])
    assert P["id"].size == Q["id"].size == o.np, (P["id"].size, Q["id"].size)
    assert np.array_equal(P["id"][a], Q["id"][b])
    return {k: P[k][a] for k in P}, {k: Q[k][b] for k in Q}


def _window_run(M=2, Nz=128, Nr=12):
    run = workloads.small(M=M, Nz=Nz, Nr=Nr, ppc=2, n_tracked=40)["runs"][0]
    run["pulses"][0]["zc"] = 3.5 * workloads.LAMBDA0  # well inside the box
    L = Nz * run["dz"]
    run.update(ramp_start=0.2 * L, ramp_len=0.3 * L)  # the box moves into the plasma
    return run


def test_fp64_moving_window_matches_oracle():
    """128 x 12 grid, modes 0..2, 60 steps, a move every 4 steps (about 45
    cells in all), guard band 8, cell sort every 6 steps (moves force a
    sort), to the FP64 bar."""
    _say("[gpu] fp64 moving window, 60 steps")
    run = _window_run()
    sim, o, dt = _window_pair(run, 60, K=4, guard=8, sort_interval=6)
    S = sim.info()["window_cells"]
    assert S == o.window_cells == math.floor(56 * dt / run["dz"]) and S > 30
    assert sim.info()["n_particles"] == o.np
    worst = compare_fields(sim, o, run["M"], TOL64)
    bad = {k: v for k, v in worst.items() if v > TOL64}
    assert not bad, bad
    P, Q = _particles_by_id(sim, o)
    assert np.abs(P["z"] - Q["z"]).max() < TOL64  # unwrapped on both sides
    assert max(np.abs(P[k] - Q[k]).max() for k in ("x", "y")) < TOL64
    umax = max(np.abs(Q[k]).max() for k in ("ux", "uy", "uz"))
    assert max(np.abs(P[k] - Q[k]).max() for k in ("ux", "uy", "uz")) < TOL64 * umax
    assert np.array_equal(P["w"] == 0, Q["w"] == 0)
    wg, wo = sim.mode_work(), o.tracked()
    assert np.array_equal(wg["id"], wo["id"])
    gone = np.isnan(wo["gamma"])
    assert gone.any() and not gone.all()  # some tracked electrons were dropped at the back
    assert np.array_equal(np.isnan(wg["gamma"]), gone)
    assert np.abs(wg["gamma"][~gone] - wo["gamma"][~gone]).max() < TOL64 * wo["gamma"][~gone].max()
    scale = max(np.abs(wo["W"]).max(), 1e-300)
    assert np.abs(wg["W"] - wo["W"]).max() / scale < TOL64
    assert np.abs(wg["gamma_acc"] - wo["gamma_acc"]).max() < TOL64 * np.abs(wo["gamma_acc"]).max()
    sim.close()


def test_fp32_moving_window_within_fp32_bounds():
    """The same run in FP32 (int32 cell + FP32 offset, unwrapped), from the
    FP32-rounded start, to the per-quantity FP32 bounds."""
    _say("[gpu] fp32 moving window, 60 steps")
    run = _window_run(M=1)
    sim, o, _ = _window_pair(run, 60, K=4, guard=8, precision=32, sort_interval=8)
    assert sim.info()["window_cells"] == o.window_cells
    assert sim.info()["n_particles"] == o.np
    for (name, m), v in compare_fields(sim, o, run["M"], 0).items():
        assert v <= (JTOL if name.startswith("J") else EBTOL), (name, m, v)
    P, Q = _particles_by_id(sim, o)
    assert np.abs(P["z"] - Q["z"]).max() < 1e-3
    sim.close()


def test_fresh_plasma_is_bitwise_the_oracles():
    """A cold plasma with no laser never moves (zero fields, zero current), so
    after the moves every electron, the fresh columns' included, is the
    oracle's bit for bit and the fields stay exactly zero."""
    _say("[gpu] fp64 moving window, plasma at rest")
    run = _window_run(M=1, Nz=96, Nr=8)
    run["pulses"] = []
    sim, o, _ = _window_pair(run, 31, K=3, guard=4)
    assert sim.info()["window_cells"] == o.window_cells > 20
    P, Q = _particles_by_id(sim, o)
    for k in ("z", "x", "y", "ux", "uy", "uz", "w"):
        assert np.array_equal(P[k], Q[k]), k
    for comp in (0, 1, 2, 13, 14, 15):
        assert not np.any(sim.fields(comp, 0)), comp
    sim.close()
