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
  Sampled outputs the oracle computes one by one: the gather and push of
  3600 electrons from the library's own field and electron state.  Both
  checks run with linear and with quadratic particle shapes.
* the six-run FP32 scan (34 M electrons, 24 x 8 tiles, sort every 16 steps,
  captured-graph steps): the smallest run against the oracle at the FP32
  bounds, every run against the same Gauss-law and work-identity checks.
"""
import numpy as np
import pytest

import workloads
from test_gpu_parity import TOL64, _pic, _say, _setup, compare_fields, compare_particles, oracle_of

pytestmark = pytest.mark.gpu


def _gauss(sim, pic, run, CB, taps, m):
    """div_B E - P rho of mode m from the library's arrays (interior rows)."""
    return _gauss_run(sim, pic, run, CB, taps, m, 0)


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


@pytest.mark.parametrize("shape", [1, 2])
def test_fp32_8192x512_invariants(shape):
    """Three steps, linear or quadratic shapes.  Bound on the change of the Gauss residual, per step, from
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
    _say(f"[gpu] full size 8192x512 fp32, invariants, shape order {shape}")
    pic = _pic()
    cfg = workloads.config("c5")
    run = cfg["runs"][0]
    sim = pic.Simulation([workloads.to_rundesc(run)], precision=pic.PREC_FP32, tile_z=16, tile_r=4,
                         sort_interval=16, shape=shape)
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


def test_fp32_six_run_scan_full_size_graph():
    """The six-run FP32 scan (12..64 points per wavelength, 34 M electrons) in
    the launch configuration of the benchmark (tile 24 x 8, sort every 16
    steps) with captured-graph steps: four steps, then
      * the smallest run (3072 x 48, 577 k electrons) against the FP64 oracle
        from the same FP32-rounded start, at the FP32 per-quantity bounds;
      * every run: Gauss's law with the filtered current drifts by no more
        than the FP32 bound of the 8192 x 512 test, and the tracked work sums
        over modes to the change of gamma."""
    _say("[gpu] full size six-run scan fp32, graph")
    from test_gpu_fp32 import EBTOL, JTOL
    from test_gpu_parity import FIELD_PAIRS

    pic = _pic()
    cfg = workloads.config("c4")
    runs = cfg["runs"]
    sim = pic.Simulation([workloads.to_rundesc(r) for r in runs], precision=pic.PREC_FP32, tile_z=24, tile_r=8,
                         sort_interval=16, use_graph=True)
    nsteps = 4
    G0 = []
    for i, run in enumerate(runs):
        CE, CB, taps = sim.coefficients(i)
        G0.append([_gauss_run(sim, pic, run, CB, taps, m, i) for m in range(run["M"] + 1)])
    sim.step(nsteps)
    u = 2.0 ** -24
    for i, run in enumerate(runs):
        CE, CB, taps = sim.coefficients(i)
        dt = sim.info(i)["dt"]
        M, dz, dr = run["M"], run["dz"], run["dr"]
        S = 2 * np.abs(CB).sum() / dz + 4 / dr + M / dr
        rows = np.arange(run["Nr"] + 1)[:, None]
        for m in range(M + 1):
            G1, emax = _gauss_run(sim, pic, run, CB, taps, m, i)
            jmax = max(np.abs(sim.fields(c, m, i)).max() for c in (pic.JR, pic.JPHI, pic.JZ))
            rho_r = (rows * np.abs(sim.fields(pic.RHO, m, i))).max()
            bound = nsteps * 2 * np.sqrt(2) * u * ((max(emax, G0[i][m][1]) + dt * jmax) * S
                                                    + rho_r * np.abs(taps).sum())
            dG = np.abs(G1 - G0[i][m][0]).max()
            assert dG <= bound, (i, m, dG, bound)
        w = sim.mode_work(i)
        assert np.abs(w["gamma_acc"] - w["gamma"]).max() <= 1e-6 * max(1.0, w["gamma"].max()), i
    # the smallest run against the oracle
    run = runs[0]
    CE, CB, _ = sim.coefficients(0)
    o = oracle_of(run, sim.info(0)["dt"], CE, CB, fp32_start=True)
    o.step(nsteps)
    for name, comp, ocomp in FIELD_PAIRS:
        for m in range(run["M"] + 1):
            g, r = sim.fields(comp, m, 0), o.get_field(ocomp, m)
            err = np.linalg.norm(g - r) / np.linalg.norm(r)
            assert err <= (JTOL if name.startswith("J") else EBTOL), (name, m, err)
    wg, wo = sim.mode_work(0), o.tracked()
    assert np.array_equal(wg["id"], wo["id"])
    gerr = np.abs(wg["gamma_acc"] - wo["gamma_acc"]) / np.maximum(wo["gamma_acc"] - 1.0, 1e-3)
    assert np.percentile(gerr, 99) <= 1e-4 and gerr.max() <= 1e-3
    sim.close()


def _gauss_run(sim, pic, run, CB, taps, m, i):
    """div_B E - P rho of mode m of run i from the library's arrays."""
    N = CB.size
    dz, dr, Nr = run["dz"], run["dr"], run["Nr"]
    Er, Ep, Ez, rho = (sim.fields(c, m, i) for c in (pic.ER, pic.EPHI, pic.EZ, pic.RHO))
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


@pytest.mark.parametrize("shape", [1, 2])
def test_fp32_8192x512_sampled_step_matches_oracle(shape):
    """Sampled parity at full size, gather + push and deposit, with linear or
    quadratic shapes (the oracle takes the same shape order): after two steps of the 8192 x 512 FP32 run
    (67 M electrons, the benchmark's 16 x 4 tiles), the library's E^n and
    time-averaged B^n are loaded into an FP64 oracle grid, and for 3600
    sampled electrons (random ones, the closest to the axis, the most
    energetic) the oracle's gather and Boris push (Eqs. (6), (12)) from the
    electron's stored state are compared with the library's next step.  Both
    start from the same FP32 values; the bounds are those of FP32 arithmetic
    with a 10x margin: momenta within 1e-5 (|u| + dt |E| + 1e-3), the
    transverse position within 1e-6 (|x| + 1) cells and z within 2e-6 cells
    (its FP32 offset).  The deposit of the same step is checked on node
    patches (below) within 1e-5 of the largest current there: each
    electron's FP32 offset difference is exact to ~2^-24 cells, and a node
    sums a few hundred of them."""
    _say(f"[gpu] full size 8192x512 fp32, sampled push against the oracle, shape order {shape}")
    import oracle

    pic = _pic()
    run = workloads.config("c5")["runs"][0]
    sim = pic.Simulation([workloads.to_rundesc(run)], precision=pic.PREC_FP32, tile_z=16, tile_r=4,
                         sort_interval=16, shape=shape)
    sim.step(2)  # the next step sorts nothing: the storage order is kept
    P0 = sim.particles()
    Nz, Nr, M, dz, dr = run["Nz"], run["Nr"], run["M"], run["dz"], run["dr"]
    CE, CB, _ = sim.coefficients()
    dt = sim.info()["dt"]
    o = oracle.Oracle(Nz, Nr, M, dz, dr, dt, CE, CB)
    o.set_shape(shape)
    for m in range(M + 1):
        for gc, oc in ((pic.ER, oracle.ER), (pic.EPHI, oracle.EP), (pic.EZ, oracle.EZ)):
            o.set_field(oc, m, sim.fields(gc, m))
        for gc, oo, on in ((pic.BR, oracle.BOR, oracle.BR), (pic.BPHI, oracle.BOP, oracle.BP),
                           (pic.BZ, oracle.BOZ, oracle.BZ)):
            b = sim.fields(gc, m)  # Bbar^n: both half steps set to it, so the oracle gathers it
            o.set_field(oo, m, b)
            o.set_field(on, m, b)
    sim.step(1)
    P1 = sim.particles()
    assert np.array_equal(P0["id"], P1["id"])
    rng = np.random.default_rng(2303)
    r0 = np.hypot(P0["x"], P0["y"])
    u0 = np.sqrt(P0["ux"] ** 2 + P0["uy"] ** 2 + P0["uz"] ** 2)
    pick = np.unique(np.concatenate([rng.choice(P0["z"].size, 3000, replace=False), np.argsort(r0)[:300],
                                     np.argsort(u0)[-300:]]))
    pick = pick[r0[pick] < Nr - 3]  # away from the reflecting wall
    lib = oracle.lib()
    worst = {"u": 0.0, "xy": 0.0, "z": 0.0}
    for p in pick:
        EB = o.gather(P0["z"][p], P0["x"][p], P0["y"][p])
        u = np.array([P0["ux"][p], P0["uy"][p], P0["uz"][p]])
        E, B = np.ascontiguousarray(EB[:3]), np.ascontiguousarray(EB[3:])
        lib.orc_boris(u.ctypes.data, E.ctypes.data, B.ctypes.data, dt)
        g = np.sqrt(1.0 + u @ u)
        x1, y1 = P0["x"][p] + dt * u[0] / g / dr, P0["y"][p] + dt * u[1] / g / dr
        z1 = (P0["z"][p] + dt * u[2] / g / dz) % Nz
        ug = np.array([P1["ux"][p], P1["uy"][p], P1["uz"][p]])
        du = np.abs(ug - u).max() / (1e-5 * (np.abs(u).max() + dt * np.abs(E).max() + 1e-3))
        dxy = max(abs(P1["x"][p] - x1), abs(P1["y"][p] - y1)) / (1e-6 * (max(abs(x1), abs(y1)) + 1))
        dzc = abs(P1["z"][p] - z1)
        dzc = min(dzc, Nz - dzc) / 2e-6
        worst = {"u": max(worst["u"], du), "xy": max(worst["xy"], dxy), "z": max(worst["z"], dzc)}
    _say(f"  {pick.size} electrons; worst error / bound: {worst}")
    assert max(worst.values()) <= 1.0, worst

    # the deposit of that step on 12 patches of 8 x 6 nodes (two on the axis):
    # every electron whose old cell is within reach of a patch (two cells
    # below and three above it with quadratic shapes, one and two with
    # linear ones, plus a cell of move) is deposited
    # by the oracle from the library's own old and new states, and the current
    # on the patch is compared with the library's J of the step
    z0, z1 = P0["z"], P1["z"].copy()
    z1 += np.where(z1 - z0 > Nz / 2, -Nz, 0.0) + np.where(z1 - z0 < -Nz / 2, Nz, 0.0)  # undo the periodic wrap
    i0, j0 = np.floor(z0).astype(np.int64), np.floor(r0).astype(np.int64)
    patches = [(300 + 650 * k, rs) for k, rs in enumerate((0, 0, 40, 120, 200, 300, 400, 480, 60, 250, 350, 10))]
    for zs, rs in patches:
        sel = np.nonzero((i0 >= zs - 3) & (i0 <= zs + 7 + 2) & (j0 >= rs - 3) & (j0 <= rs + 5 + 2))[0]
        for p in sel:
            xm, ym = 0.5 * (P0["x"][p] + P1["x"][p]), 0.5 * (P0["y"][p] + P1["y"][p])
            rm = np.hypot(xm, ym)
            u1 = np.array([P1["ux"][p], P1["uy"][p], P1["uz"][p]])
            vphi = (xm / rm * u1[1] - ym / rm * u1[0]) / np.sqrt(1.0 + u1 @ u1) if rm > 0 else 0.0
            o.deposit_add(-P0["w"][p], (z0[p], P0["x"][p], P0["y"][p]), (z1[p], P1["x"][p], P1["y"][p]), vphi)
    jworst = 0.0
    for gc, oc in ((pic.JR, oracle.JR), (pic.JPHI, oracle.JP), (pic.JZ, oracle.JZ)):
        for m in range(M + 1):
            g, r = sim.fields(gc, m), o.get_field(oc, m)
            if gc == pic.JZ and m >= 1:
                r[0] = 0.0  # the m >= 1 J_z vanishes on the axis
            gp = np.concatenate([g[rs:rs + 6, zs:zs + 8].ravel() for zs, rs in patches])
            rp = np.concatenate([r[rs:rs + 6, zs:zs + 8].ravel() for zs, rs in patches])
            jworst = max(jworst, np.abs(gp - rp).max() / (1e-5 * np.abs(rp).max()))
    _say(f"  deposit on {len(patches)} patches: worst error / (1e-5 max|J|) = {jworst:.3f}")
    assert jworst <= 1.0, jworst
    sim.close()
