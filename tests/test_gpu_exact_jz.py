"""GPU parity of the exact J_z correction: the current that conserves charge
with D_B by J_z <- P^{-1} J_z, with J_r and J_phi as deposited (Sec. III.A:
the solver conserves charge, Gauss's law written with [k]_B, Eq. (10)).

The library applies P^{-1} as a symmetric stencil cut below 2^-53 (FP64) or
2^-24 (FP32) of its centre tap, fused into the E update; the oracle applies
it exactly with a DFT on each periodic z line.  Bars: FP64 at 1e-10 as every
FP64 parity test; FP32 at the per-quantity bounds of the FP32 tests (the
FP32 cut adds at most ~2^-24 relative to J_z, far below the 3e-4 current
bound); Gauss's law with rho itself (no filter) from the library's output.
"""
import numpy as np
import pytest

import workloads
from test_gpu_fp32 import EBTOL, JTOL
from test_gpu_parity import (FIELD_PAIRS, TOL64, _pic, _say, _setup, compare_fields, compare_particles,
                             oracle_of)

pytestmark = pytest.mark.gpu


def _pair(run, nsteps, precision=64, N=16, **kw):
    pic = _pic()
    dt, CE, CB, _ = _setup(N, run["M"], run["dz"], run["dr"])
    solver = pic.SOLVER_YEE if N == 1 else pic.SOLVER_DUAL
    sim = pic.Simulation([workloads.to_rundesc(run)], precision=precision, solver=solver, n_coef=N, dt=dt,
                         coef_E=CE, coef_B=CB, current=pic.CURRENT_EXACT_JZ, **kw)
    o = oracle_of(run, dt, CE, CB, fp32_start=(precision == 32))
    o.set_exact_jz(True)
    sim.step(nsteps)
    o.step(nsteps)
    return sim, o


def _check64(sim, o, run, i=0):
    worst = compare_fields(sim, o, run["M"], TOL64, run=i)
    bad = {k: v for k, v in worst.items() if v > TOL64}
    assert not bad, bad
    dzmax, dxy, du, _ = compare_particles(sim, o, run["Nz"], run=i)
    assert dzmax < TOL64 and dxy < TOL64 and du < TOL64, (dzmax, dxy, du)
    wg, wo = sim.mode_work(i), o.tracked()
    assert np.array_equal(wg["id"], wo["id"])
    assert np.abs(wg["W"] - wo["W"]).max() <= TOL64 * max(np.abs(wo["W"]).max(), 1e-300)


@pytest.mark.parametrize("M", [0, 1, 2, 3])
def test_fp64_exact_jz_parity(M):
    """70 columns: not a multiple of the 128-column field tile, and shorter
    than the stencil (up to 2 x 83 - 1 taps), which wraps round the periodic
    line more than once."""
    _say(f"[gpu] exact J_z fp64 M={M}")
    run = workloads.small(M=M, Nz=70, Nr=12, ppc=2, n_tracked=40)["runs"][0]
    if M == 0:
        run["pulses"] = []
    sim, o = _pair(run, 12)
    _check64(sim, o, run)
    sim.close()


def test_fp64_exact_jz_yee_and_graph():
    """Yee (one tap, h = delta) and a graph-replayed step, to the same bar."""
    _say("[gpu] exact J_z fp64 Yee, graph")
    run = workloads.small(M=1, Nz=64, Nr=12, ppc=2, n_tracked=40)["runs"][0]
    sim, o = _pair(run, 10, N=1, use_graph=True)
    _check64(sim, o, run)
    sim.close()


def test_two_runs_with_their_own_stencils():
    """Two runs of one context at different resolutions fit their own
    coefficients, hence stencils of different lengths in one launch; each
    matches the oracle run with that run's coefficients and dt."""
    _say("[gpu] exact J_z, two runs")
    pic = _pic()
    from oracle import coef

    runs = [workloads.small(M=2, Nz=64, Nr=12, ppc=2, n_tracked=20)["runs"][0],
            workloads.small(M=2, Nz=96, Nr=10, ppc=2, n_tracked=20, seed=7)["runs"][0]]
    runs[1]["dz"] = runs[0]["dz"] * 0.75
    runs[1]["dr"] = runs[0]["dr"] * 0.9
    sim = pic.Simulation([workloads.to_rundesc(r) for r in runs], current=pic.CURRENT_EXACT_JZ)
    lens = []
    for i, r in enumerate(runs):
        _, cb, _ = sim.coefficients(i)
        lens.append(pic.jz_inverse_taps(cb).size)
    assert lens[0] != lens[1], lens
    sim.step(8)
    for i, r in enumerate(runs):
        ce, cb, _ = sim.coefficients(i)
        o = oracle_of(r, sim.info(i)["dt"], ce, cb)
        o.set_exact_jz(True)
        o.step(8)
        _check64(sim, o, r, i)
    sim.close()


def test_fp64_gauss_law_with_rho_on_gpu():
    """div_B E - rho (rho itself, not P rho) is constant in time on the GPU
    path, from the library's own output."""
    _say("[gpu] exact J_z fp64 Gauss invariant")
    pic = _pic()
    run = workloads.small(M=2, Nz=64, Nr=12, ppc=2)["runs"][0]
    dt, CE, CB, _ = _setup(16, run["M"], run["dz"], run["dr"])
    sim = pic.Simulation([workloads.to_rundesc(run)], dt=dt, coef_E=CE, coef_B=CB, current=pic.CURRENT_EXACT_JZ)
    N, dz, dr, Nr = CB.size, run["dz"], run["dr"], run["Nr"]

    def DB(g):  # half-z data (column k = z_{k+1/2}) -> integer z
        out = np.zeros_like(g)
        for l in range(1, N + 1):
            out += CB[l - 1] * (np.roll(g, -(l - 1), axis=1) - np.roll(g, l, axis=1))
        return out / dz

    def gauss(m):
        Er, Ep, Ez, rho = (sim.fields(c, m) for c in (pic.ER, pic.EPHI, pic.EZ, pic.RHO))
        G = np.zeros_like(Er)
        j = np.arange(1, Nr)[:, None]
        G[1:Nr] = (DB(Ez)[1:Nr] + ((j + 0.5) * Er[1:Nr] - (j - 0.5) * Er[0:Nr - 1]) / (j * dr)
                   + 1j * m / (j * dr) * Ep[1:Nr] - rho[1:Nr])
        if m == 0:
            G[0] = DB(Ez)[0] + 4 * Er[0] / dr - rho[0]
        return G

    G0 = [gauss(m) for m in range(run["M"] + 1)]
    sim.step(15)
    for m in range(run["M"] + 1):
        G1 = gauss(m)
        scale = np.abs(G0[m]).max() + np.abs(G1).max()
        assert np.abs(G1 - G0[m]).max() < 1e-12 * scale, m
    sim.close()


def test_fp32_exact_jz_per_quantity_bounds():
    """256 x 64, modes 0..1, 4 ppc, 100 steps in FP32 against the FP64 oracle
    from the same FP32-rounded start."""
    _say("[gpu] exact J_z fp32 256x64, 100 steps")
    pic = _pic()
    run = workloads.config("c3")["runs"][0]
    sim, o = _pair(run, 100, precision=pic.PREC_FP32)
    for name, comp, ocomp in FIELD_PAIRS:
        for m in range(run["M"] + 1):
            g, r = sim.fields(comp, m), o.get_field(ocomp, m)
            err = np.linalg.norm(g - r) / np.linalg.norm(r)
            assert err <= (JTOL if name.startswith("J") else EBTOL), (name, m, err)
    wg, wo = sim.mode_work(), o.tracked()
    scale = np.maximum(wo["gamma_acc"] - 1.0, 1e-3)
    gerr = np.abs(wg["gamma_acc"] - wo["gamma_acc"]) / scale
    assert np.percentile(gerr, 99) <= 1e-4 and gerr.max() <= 1e-3
    sim.close()


@pytest.mark.parametrize("M", [0, 2, 3])
def test_fp32_exact_jz_small_grid_bounds(M):
    """The FP32 instantiations of the other mode counts, 70 columns, 40 steps,
    at the FP32 per-quantity bounds."""
    _say(f"[gpu] exact J_z fp32 M={M}")
    pic = _pic()
    run = workloads.small(M=M, Nz=70, Nr=12, ppc=2, n_tracked=40)["runs"][0]
    sim, o = _pair(run, 40, precision=pic.PREC_FP32)
    for name, comp, ocomp in FIELD_PAIRS:
        for m in range(M + 1):
            g, r = sim.fields(comp, m), o.get_field(ocomp, m)
            nr = np.linalg.norm(r)
            err = np.linalg.norm(g - r) / nr if nr > 0 else np.linalg.norm(g)
            assert err <= (JTOL if name.startswith("J") else EBTOL), (name, m, err)
    wg, wo = sim.mode_work(), o.tracked()
    gerr = np.abs(wg["gamma_acc"] - wo["gamma_acc"]) / np.maximum(wo["gamma_acc"] - 1.0, 1e-3)
    assert gerr.max() <= 1e-3
    sim.close()
