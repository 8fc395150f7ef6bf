"""GPU parity of the quadratic particle shapes (pic_opts.shape = 2) against
the oracle's quadratic gather and deposit.

Both sides take the same reading of the order the paper leaves open
(Sec. III): quadratic B-spline weights on the 3 x 3 nodes round the nearest
node of each component's grid for the gather, the charge-conserving deposit
on the 4 x 4 nodes that hold both positions' supports, and rows below the
axis folded onto the rows above with each quantity's mirror sign.  The
library stages the mirrored rows in the tile's field window and folds row
r_{-1} of the tile's current window when it is flushed; an electron outside
its tile's windows gathers and deposits in device memory, folding at once.

Checked: every field and current array of every mode, every electron, the
per-mode work of the tracked electrons, the charge density diagnostic, and
Gauss's law of the dual solver on the library's own output -- FP64 to the
1e-10 bar, FP32 to the per-quantity FP32 bounds.
"""
import numpy as np
import pytest

import oracle
import workloads
from test_gpu_fp32 import EBTOL, JTOL
from test_gpu_parity import (TOL64, _pic, _say, _setup, compare_cartesian_work, compare_fields, compare_particles,
                             oracle_of)

pytestmark = pytest.mark.gpu


def _pair(run, nsteps, precision=64, N=16, **kw):
    pic = _pic()
    dt, CE, CB, _ = _setup(N, run["M"], run["dz"], run["dr"])
    solver = pic.SOLVER_YEE if N == 1 else pic.SOLVER_DUAL
    sim = pic.Simulation([workloads.to_rundesc(run)], precision=precision, solver=solver, n_coef=N, dt=dt, coef_E=CE,
                         coef_B=CB, shape=2, **kw)
    o = oracle_of(run, dt, CE, CB, fp32_start=(precision == 32))
    o.set_shape(2)
    if kw.get("window_interval"):
        o.set_window(kw["window_interval"], 1.0, kw.get("window_guard", 0))
    sim.step(nsteps)
    o.step(nsteps)
    return sim, o


def _check_fp64(sim, o, run):
    worst = compare_fields(sim, o, run["M"], TOL64)
    bad = {k: v for k, v in worst.items() if v > TOL64}
    assert not bad, bad
    dzmax, dxy, du, _ = compare_particles(sim, o, run["Nz"])
    assert dzmax < TOL64 and dxy < TOL64 and du < TOL64, (dzmax, dxy, du)
    wg, wo = sim.mode_work(), o.tracked()
    assert np.array_equal(wg["id"], wo["id"])
    scale = max(np.abs(wo["W"]).max(), 1e-300)
    assert np.abs(wg["W"] - wo["W"]).max() / scale < TOL64
    # Eq. (16) work identity on the GPU path: sum_m W_m = gamma - gamma_0
    assert np.abs(wg["gamma_acc"] - wg["gamma"]).max() < 1e-13 * max(1.0, wg["gamma"].max())


@pytest.mark.parametrize("M", [0, 1, 2, 3])
def test_fp64_quadratic_small_grid_parity(M):
    """64 x 12 grid, 2 electrons per cell from the axis out (so the folded
    rows take part), 20 steps, modes 0..M, to the FP64 bar."""
    _say(f"[gpu] fp64 quadratic shapes, small grid M={M}")
    run = workloads.small(M=M, Nz=64, Nr=12, ppc=2, n_tracked=40)["runs"][0]
    if M == 0:
        run["pulses"] = []
    sim, o = _pair(run, 20)
    _check_fp64(sim, o, run)
    cw = compare_cartesian_work(sim, o, run, TOL64)
    assert max(cw.values()) < TOL64, cw
    sim.close()


def test_fp64_quadratic_ragged_grid_and_density_ramps():
    """A grid that no tile divides (70 x 11 with 16 x 4 tiles), App. A's ramps,
    sorted every 3 steps, 24 steps, to the FP64 bar."""
    _say("[gpu] fp64 quadratic shapes, ragged grid and ramps")
    run = workloads.small(M=2, Nz=70, Nr=11, ppc=3, n_tracked=30)["runs"][0]
    L = run["Nz"] * run["dz"]
    run.update(ramp_start=0.1 * L, ramp_len=0.2 * L, down_start=0.6 * L, down_len=0.25 * L)
    sim, o = _pair(run, 24, tile_z=16, tile_r=4, sort_interval=3)
    _check_fp64(sim, o, run)
    sim.close()


def test_fp64_quadratic_electrons_outside_their_tile_windows():
    """The device-memory path of the quadratic gather and deposit (with the
    fold done at once): a strong pulse over the whole box, 8 x 1 tiles and no
    re-sort, so that most electron-steps leave their tile's windows."""
    _say("[gpu] fp64 quadratic shapes outside the tile windows")
    run = workloads.small(M=2, Nz=64, Nr=12, ppc=2, a0=4.0, n_tracked=64)["runs"][0]
    run["pulses"] = [dict(a0=4.0, w0=3 * workloads.LAMBDA0, tau=6 * workloads.LAMBDA0, zc=2 * workloads.LAMBDA0)]
    sim, o = _pair(run, 32, tile_z=8, tile_r=1, sort_interval=1000)
    _check_fp64(sim, o, run)
    sim.close()


def test_fp64_quadratic_smallest_grid_all_tracked_and_many_per_cell():
    """Edge cases with quadratic shapes: the smallest grid accepted (32 x 4:
    the stencils wrap the whole periodic line, every electron within reach of
    both the axis fold and the wall row) with every electron tracked, and 24
    electrons per cell (a wavefront's lanes share cells, so their LDS atomics
    collide), each against the oracle at the FP64 bar."""
    _say("[gpu] fp64 quadratic shapes, smallest grid and 24 ppc")
    run = workloads.small(M=1, Nz=32, Nr=4, ppc=3, n_tracked=0)["runs"][0]
    run["n_tracked"] = 32 * 3 * 3
    sim, o = _pair(run, 25)
    _check_fp64(sim, o, run)
    assert sim.mode_work()["id"].size == run["n_tracked"]
    sim.close()
    run = workloads.small(M=2, Nz=64, Nr=12, ppc=24, n_tracked=50)["runs"][0]
    sim, o = _pair(run, 10)
    _check_fp64(sim, o, run)
    sim.close()


def test_fp32_quadratic_within_fp32_bounds():
    """The FP32 form (int32 cell + FP32 offset) with quadratic shapes, from the
    FP32-rounded start, 20 steps, modes 0..3, to the FP32 bounds."""
    _say("[gpu] fp32 quadratic shapes")
    run = workloads.small(M=3, Nz=64, Nr=12, ppc=2, n_tracked=40)["runs"][0]
    sim, o = _pair(run, 20, precision=32)
    for (name, m), v in compare_fields(sim, o, run["M"], 0).items():
        assert v <= (JTOL if name.startswith("J") else EBTOL), (name, m, v)
    dzmax, dxy, du, _ = compare_particles(sim, o, run["Nz"])
    assert dzmax < 1e-3 and dxy < 1e-3 and du < 1e-3, (dzmax, dxy, du)
    sim.close()


def test_fp64_quadratic_yee_solver():
    """Quadratic shapes with the Yee solver (one coefficient per operator, no
    filter) through the same kernels, against the oracle run with
    C^E = C^B = (1), to the FP64 bar."""
    _say("[gpu] fp64 quadratic shapes, Yee solver")
    run = workloads.small(M=2, Nz=64, Nr=12, ppc=2, n_tracked=40)["runs"][0]
    sim, o = _pair(run, 30, N=1)
    _check_fp64(sim, o, run)
    sim.close()


def test_fp64_quadratic_charge_density_and_gauss_law():
    """The quadratic charge density diagnostic equals the oracle's, and
    div_B E - P rho stays constant through 15 steps on the library's own
    output (Eq. (10) with the filtered current)."""
    _say("[gpu] fp64 quadratic charge density and Gauss's law")
    pic = _pic()
    run = workloads.small(M=2, Nz=64, Nr=12, ppc=2)["runs"][0]
    dt, CE, CB, _ = _setup(16, run["M"], run["dz"], run["dr"])
    sim = pic.Simulation([workloads.to_rundesc(run)], dt=dt, coef_E=CE, coef_B=CB, shape=2)
    o = oracle_of(run, dt, CE, CB)
    o.set_shape(2)
    o.deposit_rho()
    for m in range(run["M"] + 1):
        g, r = sim.fields(pic.RHO, m), o.get_field(oracle.RHO, m)
        assert np.abs(g - r).max() < TOL64 * np.abs(r).max(), m
    _, _, taps = sim.coefficients()
    N = CB.size
    dz, dr, Nr = run["dz"], run["dr"], run["Nr"]

    def DB(g):  # half-z data (column k = z_{k+1/2}) -> integer z
        out = np.zeros_like(g)
        for l in range(1, N + 1):
            out += CB[l - 1] * (np.roll(g, -(l - 1), axis=1) - np.roll(g, l, axis=1))
        return out / dz

    def P(f):
        out = np.zeros_like(f)
        for l in range(-(N - 1), N):
            out += taps[l + N - 1] * np.roll(f, -l, axis=1)
        return out

    def gauss(m):
        Er, Ep, Ez, rho = (sim.fields(c, m) for c in (pic.ER, pic.EPHI, pic.EZ, pic.RHO))
        G = np.zeros_like(Er)
        j = np.arange(1, Nr)[:, None]
        G[1:Nr] = (DB(Ez)[1:Nr] + ((j + 0.5) * Er[1:Nr] - (j - 0.5) * Er[0:Nr - 1]) / (j * dr)
                   + 1j * m / (j * dr) * Ep[1:Nr] - P(rho)[1:Nr])
        if m == 0:
            G[0] = DB(Ez)[0] + 4 * Er[0] / dr - P(rho)[0]
        return G

    G0 = [gauss(m) for m in range(run["M"] + 1)]
    sim.step(15)
    for m in range(run["M"] + 1):
        G1 = gauss(m)
        scale = np.abs(G0[m]).max() + np.abs(G1).max()
        assert np.abs(G1 - G0[m]).max() < 1e-12 * scale, m
    sim.close()


def test_fp64_quadratic_moving_window():
    """Quadratic shapes with the moving window: 128 x 12 grid, a move every 4
    steps for 40 steps, guard band 8, to the FP64 bar by electron id."""
    _say("[gpu] fp64 quadratic shapes with the moving window")
    run = workloads.small(M=1, Nz=128, Nr=12, ppc=2, n_tracked=40)["runs"][0]
    run["pulses"][0]["zc"] = 3.5 * workloads.LAMBDA0
    L = run["Nz"] * run["dz"]
    run.update(ramp_start=0.2 * L, ramp_len=0.3 * L)
    sim, o = _pair(run, 40, window_interval=4, window_guard=8, sort_interval=6)
    assert sim.info()["window_cells"] == o.window_cells > 20
    assert sim.info()["n_particles"] == o.np
    worst = compare_fields(sim, o, run["M"], TOL64)
    bad = {k: v for k, v in worst.items() if v > TOL64}
    assert not bad, bad
    P, Q = sim.particles(), o.particles()
    a, b = np.argsort(P["id"]), np.argsort(Q["id"])
    assert np.array_equal(P["id"][a], Q["id"][b])
    assert max(np.abs(P[k][a] - Q[k][b]).max() for k in ("z", "x", "y")) < TOL64
    sim.close()


def test_fp32_quadratic_moving_window():
    """The FP32 form with quadratic shapes and the moving window (positions
    unwrapped, electrons dropped and fresh columns loaded), 40 steps, a move
    every 4, to the FP32 bounds by electron id."""
    _say("[gpu] fp32 quadratic shapes with the moving window")
    run = workloads.small(M=1, Nz=128, Nr=12, ppc=2, n_tracked=40)["runs"][0]
    run["pulses"][0]["zc"] = 3.5 * workloads.LAMBDA0
    L = run["Nz"] * run["dz"]
    run.update(ramp_start=0.2 * L, ramp_len=0.3 * L)
    sim, o = _pair(run, 40, precision=32, window_interval=4, window_guard=8, sort_interval=6)
    assert sim.info()["window_cells"] == o.window_cells > 20
    assert sim.info()["n_particles"] == o.np
    for (name, m), v in compare_fields(sim, o, run["M"], 0).items():
        assert v <= (JTOL if name.startswith("J") else EBTOL), (name, m, v)
    P, Q = sim.particles(), o.particles()
    a, b = np.argsort(P["id"]), np.argsort(Q["id"])
    assert np.array_equal(P["id"][a], Q["id"][b])
    assert np.abs(P["z"][a] - Q["z"][b]).max() < 1e-3
    sim.close()


def test_fp64_quadratic_batched_graph_exact_jz():
    """Two runs of different grids and cells in one context with quadratic
    shapes, the exact J_z correction and captured-graph steps (sorts every 4
    steps, advanced in chunks with reads in between), each run against its
    own oracle with the same switches at the FP64 bar."""
    _say("[gpu] fp64 quadratic shapes, batched runs, graph replay, exact J_z")
    from test_gpu_batch import _runs

    pic = _pic()
    runs = _runs()[:2]
    dt, CE, CB, _ = _setup(16, 2, runs[-1]["dz"], runs[-1]["dr"])
    sim = pic.Simulation([workloads.to_rundesc(r) for r in runs], dt=dt, coef_E=CE, coef_B=CB, sort_interval=4,
                         use_graph=True, current=pic.CURRENT_EXACT_JZ, shape=2)
    done = 0
    for chunk in (3, 5, 6):
        sim.step(chunk)
        done += chunk
        sim.fields(pic.EZ, 0, 0)  # a read between replays
    for i, run in enumerate(runs):
        o = oracle_of(run, dt, CE, CB)
        o.set_shape(2)
        o.set_exact_jz(True)
        o.step(done)
        worst = compare_fields(sim, o, run["M"], TOL64, run=i)
        bad = {k: v for k, v in worst.items() if v > TOL64}
        assert not bad, (i, bad)
        dzmax, dxy, du, _ = compare_particles(sim, o, run["Nz"], run=i)
        assert dzmax < TOL64 and dxy < TOL64 and du < TOL64, (i, dzmax, dxy, du)
    sim.close()


def test_quadratic_checkpoint_restore_and_shape_mismatch():
    """A quadratic-shape context restores its own checkpoint and continues like
    the original (to 1e-12); a linear-shape context of the same runs refuses
    it (the header records the shape order)."""
    _say("[gpu] quadratic shapes, checkpoint and restore")
    pic = _pic()
    run = workloads.small(M=2, Nz=64, Nr=12, ppc=2, n_tracked=10)["runs"][0]
    dt, CE, CB, _ = _setup(16, 2, run["dz"], run["dr"])

    def make(shape):
        return pic.Simulation([workloads.to_rundesc(run)], dt=dt, coef_E=CE, coef_B=CB, sort_interval=4, shape=shape)

    a = make(2)
    a.step(9)
    blob = a.checkpoint()
    a.step(6)
    b = make(2)
    b.restore(blob)
    b.step(6)
    for comp in (0, 1, 2, 6, 7, 8, 13, 14, 15):
        for m in range(run["M"] + 1):
            x, y = a.fields(comp, m), b.fields(comp, m)
            assert np.abs(x - y).max() <= 1e-12 * max(np.abs(x).max(), 1e-300), (comp, m)
    c = make(1)
    with pytest.raises(pic.PicError):
        c.restore(blob)
    for s in (a, b, c):
        s.close()
