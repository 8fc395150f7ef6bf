"""Parity at the benchmark sizes, in the launch configurations bench.py times.

* 4096 x 256, modes 0..2, 8 ppc, FP64 (8.4 M electrons, 30 x 4 tiles, sort
  every 8 steps): two full steps against the oracle, every field array and
  mode and every electron at the 1e-10 bar (the oracle takes a few seconds
  per step at this size).
* 8192 x 512, modes 0..3, 16 ppc, FP32 (67 M electrons, 16 x 4 tiles, sort
  every 16 steps): too large for the oracle in a test, so properties that
  hold at any size are checked on the library's own output: Gauss's law with
  the filtered current (Eq. (10)) stays constant to within a bound derived
  from the FP32 arithmetic of the E update and of the push's radius, and the
  tracked work sums over modes to the change of gamma (Eq. (16)).
"""
import numpy as np
import pytest

import workloads
from test_gpu_parity import TOL64, _pic, _say, _setup, compare_fields, compare_particles, oracle_of

pytestmark = pytest.mark.gpu


def _gauss(sim, pic, run, CB, taps, m):
    """div_B E - P rho of mode m from the library's arrays (interior rows)."""
    N = CB.size
    dz, dr, Nr = run["dz"], run["dr"], run["Nr"]
    Er, Ep, Ez, rho = (sim.fields(c, m) for c in (pic.ER, pic.EPHI, pic.EZ, pic.RHO))
    dbz = np.zeros_like(Ez)
    for l in range(1, N + 1):
        dbz += CB[l - 1] * (np.roll(Ez, -(l - 1), axis=1) - np.roll(Ez, l, axis=1))
    dbz /= dz
    prho = np.zeros_like(rho)
    for l in range(-(N - 1), N):
        prho += taps[l + N - 1] * np.roll(rho, -l, axis=1)
    G = np.zeros_like(Er)
    j = np.arange(1, Nr)[:, None]
    G[1:Nr] = (dbz[1:Nr] + ((j + 0.5) * Er[1:Nr] - (j - 0.5) * Er[0:Nr - 1]) / (j * dr)
               + 1j * m / (j * dr) * Ep[1:Nr] - prho[1:Nr])
    if m == 0:
        G[0] = dbz[0] + 4 * Er[0] / dr - prho[0]
    return G, max(np.abs(Er).max(), np.abs(Ep).max(), np.abs(Ez).max())


def test_fp64_4096x256_two_steps_match_oracle():
    _say("[gpu] full size 4096x256 fp64, 2 steps")
    pic = _pic()
    cfg = workloads.config("c2")
    run = cfg["runs"][0]
    dt, CE, CB, _ = _setup(16, run["M"], run["dz"], run["dr"])
    sim = pic.Simulation([workloads.to_rundesc(run)], dt=dt, coef_E=CE, coef_B=CB, tile_z=30, tile_r=4,
                         sort_interval=8)
    sim.step(2)
    o = oracle_of(run, dt, CE, CB)
    o.step(2)
    worst = compare_fields(sim, o, run["M"], TOL64)
    bad = {k: v for k, v in worst.items() if v > TOL64}
    assert not bad, bad
    dzmax, dxy, du, _ = compare_particles(sim, o, run["Nz"])
    assert dzmax < TOL64 and dxy < TOL64 and du < TOL64, (dzmax, dxy, du)
    wg, wo = sim.mode_work(), o.tracked()
    assert np.array_equal(wg["id"], wo["id"])
    assert np.abs(wg["W"] - wo["W"]).max() <= TOL64 * max(np.abs(wo["W"]).max(), 1e-300)
    sim.close()


def test_fp32_8192x512_invariants():
    """Three steps.  Bound on the change of the Gauss residual, per step, from
    the FP32 arithmetic (u = 2^-24, a factor 2 sqrt(2) for complex parts and
    margin):
      * each E update rounds E, and takes an FP32 J: errors u (|E| + dt |J|)
        per node, whose discrete divergence is at most that times
        S = 2 sum|C^B| / dz + 4 / dr + M / dr;
      * the push forms r from the FP32 x, y in FP32, absolute error u r
        cells, while rho is deposited in FP64 from the same stored x, y: the
        current's radial weights differ from rho's by u j at row j, so
        continuity holds to u max_j (j |rho_j|), times sum|P| after the
        filter."""
    _say("[gpu] full size 8192x512 fp32, invariants")
    pic = _pic()
    cfg = workloads.config("c5")
    run = cfg["runs"][0]
    sim = pic.Simulation([workloads.to_rundesc(run)], precision=pic.PREC_FP32, tile_z=16, tile_r=4,
                         sort_interval=16)
    CE, CB, taps = sim.coefficients()
    dt = sim.info(0)["dt"]
    M, dz, dr = run["M"], run["dz"], run["dr"]
    S = 2 * np.abs(CB).sum() / dz + 4 / dr + M / dr
    G0 = [_gauss(sim, pic, run, CB, taps, m) for m in range(M + 1)]
    nsteps = 3
    sim.step(nsteps)
    u = 2.0 ** -24
    rows = np.arange(run["Nr"] + 1)[:, None]
    for m in range(M + 1):
        G1, emax = _gauss(sim, pic, run, CB, taps, m)
        jmax = max(np.abs(sim.fields(c, m)).max() for c in (pic.JR, pic.JPHI, pic.JZ))
        rho_r = (rows * np.abs(sim.fields(pic.RHO, m))).max()
        bound = nsteps * 2 * np.sqrt(2) * u * ((max(emax, G0[m][1]) + dt * jmax) * S + rho_r * np.abs(taps).sum())
        dG = np.abs(G1 - G0[m][0]).max()
        _say(f"  m={m}: |dG| {dG:.3e}, bound {bound:.3e}")
        assert dG <= bound, (m, dG, bound)
    w = sim.mode_work()
    gmax = max(1.0, w["gamma"].max())
    assert np.abs(w["gamma_acc"] - w["gamma"]).max() <= 1e-6 * gmax
    sim.close()
