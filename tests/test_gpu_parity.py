"""GPU parity: the HIP library against the FP64 oracle on the same seeded
inputs, element by element, through the C ABI.

Both sides are built from the same workload description; the solver
coefficients and dt come from the oracle's own fit and are passed to the
library (the fit is ill-conditioned, so two correct fits differ in the
last digits; the library's own fit is checked against the oracle's at the
symbol level on the CPU).  FP64 bar: max |gpu - oracle| / max |oracle| <= 1e-10
per field array and mode, positions within 1e-10 cells, momenta within
1e-10 of the largest momentum, tracked work within 1e-10 of the largest.
"""
import functools
import math
import sys

import numpy as np
import pytest

import oracle
import workloads
from oracle import coef

pytestmark = pytest.mark.gpu

TOL64 = 1e-10


def _pic():
    import torch

    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    import paper_2303_12874_amd as pic

    return pic


@functools.lru_cache(maxsize=None)
def _setup(N, M, dz, dr):
    return coef.solver_setup(N, M, dz, dr)


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


FIELD_PAIRS = [
    ("E_r", 0, oracle.ER), ("E_phi", 1, oracle.EP), ("E_z", 2, oracle.EZ),
    ("B_r(n-1/2)", 10, oracle.BOR), ("B_phi(n-1/2)", 11, oracle.BOP), ("B_z(n-1/2)", 12, oracle.BOZ),
    ("B_r(n+1/2)", 13, oracle.BR), ("B_phi(n+1/2)", 14, oracle.BP), ("B_z(n+1/2)", 15, oracle.BZ),
    ("J_r", 6, oracle.JR), ("J_phi", 7, oracle.JP), ("J_z", 8, oracle.JZ),
]


def compare_fields(sim, o, M, tol, run=0):
    worst = {}
    for name, comp, ocomp in FIELD_PAIRS:
        for m in range(M + 1):
            g = sim.fields(comp, m, run)
            r = o.get_field(ocomp, m)
            scale = np.abs(r).max()
            err = np.abs(g - r).max() / scale if scale > 0 else np.abs(g).max()
            worst[(name, m)] = err
    return worst


def compare_particles(sim, o, Nz, run=0):
    P = sim.particles(run)
    Q = o.particles()
    order = np.argsort(P["id"])
    assert np.array_equal(P["id"][order], Q["id"])
    dz = np.abs(P["z"][order] - Q["z"])
    dz = np.minimum(dz, Nz - dz)  # periodic
    umax = max(np.abs(Q[k]).max() for k in ("ux", "uy", "uz"))
    du = max(np.abs(P[k][order] - Q[k]).max() for k in ("ux", "uy", "uz"))
    dxy = max(np.abs(P[k][order] - Q[k]).max() for k in ("x", "y"))
    return dz.max(), dxy, du / max(umax, 1e-300), P


def oracle_of(run, dt, CE, CB, fp32_start=False):
    """The oracle of a run; with fp32_start its initial particles and E^0, B^0
    are first rounded as the FP32 library stores them."""
    o = oracle.Oracle(run["Nz"], run["Nr"], run["M"], run["dz"], run["dr"], dt, CE, CB)
    o.load_plasma(run["ppc"], run["n0"], run["ramp_start"], run["ramp_len"], run["seed"], run["n_tracked"],
                  run.get("down_start", 0.0), run.get("down_len", 0.0))
    for p in run["pulses"]:
        o.add_laser(p["a0"], p["w0"], p["tau"], p["zc"], run["taper"])
    if fp32_start:
        o.round_to_fp32()
    o.start_fields()
    return o


def compare_cartesian_work(sim, o, run, tol, i=0):
    """W_z, W_perp (Eq. (17)) against the oracle's accumulators, and f, W*
    (Eqs. (20)-(21)) against the oracle's formulas applied to the oracle's
    own W_z, W_perp and gamma.  Returns the worst relative differences."""
    from oracle import work

    cg = sim.cartesian_work(i, corrected=bool(run["pulses"]))
    co, to = o.cartesian_work(), o.tracked()
    scale = max(np.abs(co["Wz"]).max(), np.abs(co["Wperp"]).max(), 1e-300)
    out = {"Wz": np.abs(cg["Wz"] - co["Wz"]).max() / scale, "Wperp": np.abs(cg["Wperp"] - co["Wperp"]).max() / scale}
    if run["pulses"]:
        p = run["pulses"][0]
        f = work.pukhov_ratio(to["gamma"], run["n0"], p["w0"])
        lw, dl = work.corrected_work(co["Wz"], co["Wperp"], f)
        out["f"] = np.abs(cg["f"] / f - 1).max()
        ws = max(np.abs(lw).max(), np.abs(dl).max(), 1e-300)
        out["W*"] = max(np.abs(cg["W_lwfa"] - lw).max(), np.abs(cg["W_dla"] - dl).max()) / ws
    return out


def energetic_cut(gamma, lo=0.01, hi=0.03):
    """A Lorentz-factor cut that keeps the top 1-3 % of the electrons, placed
    in the middle of the widest gap between neighbouring values there, so that
    state differences far below the gap cannot move an electron across it."""
    g = np.sort(gamma)[::-1]
    a, b = max(1, int(lo * g.size)), max(2, int(hi * g.size))
    i = a + int(np.argmax(g[a - 1:b - 1] - g[a:b]))
    return 0.5 * (g[i - 1] + g[i]), g[i - 1] - g[i]


def compare_divergence(sim, o, i=0):
    """The library's divergence sums against the oracle's: on the oracle's own
    state (physics parity; count exact) and on the library's state (the
    reduction alone).  Returns (worst relative difference, count)."""
    from oracle import beam

    po, pg = o.particles(), sim.particles(i)
    go = np.sqrt(1 + po["ux"] ** 2 + po["uy"] ** 2 + po["uz"] ** 2)
    cut, gap = energetic_cut(go)
    dg, ro, rs = sim.divergence(cut, i), beam.divergence(po, cut), beam.divergence(pg, cut)
    assert dg["count"] == ro["count"] == rs["count"], (dg["count"], ro["count"], rs["count"], gap)
    worst = 0.0
    for k in ("w", "sum_wtx2", "sum_wty2", "rms_x", "rms_y"):  # the RMS angles come from the library itself
        worst = max(worst, abs(dg[k] / ro[k] - 1), abs(dg[k] / rs[k] - 1))
    return worst, dg["count"]


def run_pair(run, nsteps, precision=64, N=16):
    pic = _pic()
    dt, CE, CB, _ = _setup(N, run["M"], run["dz"], run["dr"])
    solver = pic.SOLVER_YEE if N == 1 else pic.SOLVER_DUAL
    sim = pic.Simulation([workloads.to_rundesc(run)], precision=precision, solver=solver, n_coef=N, dt=dt, coef_E=CE,
                         coef_B=CB)
    o = oracle_of(run, dt, CE, CB, fp32_start=(precision == 32))
    sim.step(nsteps)
    o.step(nsteps)
    return sim, o


@pytest.mark.parametrize("M", [0, 1, 2, 3])
def test_fp64_small_grid_parity(M):
    _say(f"[gpu] fp64 small grid M={M}")
    cfg = workloads.small(M=M, Nz=64, Nr=12, ppc=2, n_tracked=40)
    run = cfg["runs"][0]
    if M == 0:
        run["pulses"] = []
    sim, o = run_pair(run, 20)
    worst = compare_fields(sim, o, M, TOL64)
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
    cw = compare_cartesian_work(sim, o, run, TOL64)
    assert max(cw.values()) < TOL64, cw
    sim.close()


def test_fp64_density_ramps_parity():
    """App. A's density profile (up-ramp, plateau, down-ramp) in a short box:
    12 steps, modes 0..1, to the FP64 bar."""
    _say("[gpu] fp64 density ramps")
    run = workloads.small(M=1, Nz=96, Nr=12, ppc=2, n_tracked=40)["runs"][0]
    L = run["Nz"] * run["dz"]
    run.update(ramp_start=0.1 * L, ramp_len=0.2 * L, down_start=0.55 * L, down_len=0.3 * L)
    sim, o = run_pair(run, 12)
    worst = compare_fields(sim, o, run["M"], TOL64)
    bad = {k: v for k, v in worst.items() if v > TOL64}
    assert not bad, bad
    dzmax, dxy, du, _ = compare_particles(sim, o, run["Nz"])
    assert dzmax < TOL64 and dxy < TOL64 and du < TOL64, (dzmax, dxy, du)
    sim.close()


def test_fp64_config1_full_parity():
    """256 x 64 grid, modes 0..1, 4 ppc, 100 steps (the small benchmark config)."""
    _say("[gpu] fp64 config c1, 100 steps")
    cfg = workloads.config("c1")
    run = cfg["runs"][0]
    sim, o = run_pair(run, cfg["steps"])
    worst = compare_fields(sim, o, run["M"], TOL64)
    bad = {k: v for k, v in worst.items() if v > TOL64}
    assert not bad, bad
    dzmax, dxy, du, _ = compare_particles(sim, o, run["Nz"])
    assert dzmax < TOL64 and dxy < TOL64 and du < TOL64, (dzmax, dxy, du)
    wg, wo = sim.mode_work(), o.tracked()
    scale = np.abs(wo["W"]).max()
    assert np.abs(wg["W"] - wo["W"]).max() / scale < TOL64
    assert np.abs(wg["gamma"] - wo["gamma"]).max() < TOL64
    U = wg["field_energy"]
    Uo = np.array([o.field_energy(m) for m in range(run["M"] + 1)])
    assert np.abs(U / Uo - 1).max() < TOL64
    assert abs(wg["kinetic"] / o.kinetic() - 1) < 1e-9
    cw = compare_cartesian_work(sim, o, run, TOL64)
    assert max(cw.values()) < TOL64, cw
    dv, cnt = compare_divergence(sim, o)
    assert dv < TOL64 and cnt > 100, (dv, cnt)
    sim.close()


@pytest.mark.parametrize("M", [1, 2])
def test_yee_solver_parity(M):
    """The Yee solver (one coefficient per operator, no filter) through the
    same kernels: fields, particles, work and divergence against the oracle
    run with C^E = C^B = (1)."""
    _say(f"[gpu] yee M={M}")
    run = workloads.small(M=M, Nz=64, Nr=12, ppc=2, n_tracked=40)["runs"][0]
    sim, o = run_pair(run, 30, N=1)
    worst = compare_fields(sim, o, M, TOL64)
    bad = {k: v for k, v in worst.items() if v > TOL64}
    assert not bad, bad
    dzmax, dxy, du, _ = compare_particles(sim, o, run["Nz"])
    assert dzmax < TOL64 and dxy < TOL64 and du < TOL64, (dzmax, dxy, du)
    wg, wo = sim.mode_work(), o.tracked()
    assert np.abs(wg["W"] - wo["W"]).max() / np.abs(wo["W"]).max() < TOL64
    cw = compare_cartesian_work(sim, o, run, TOL64)
    assert max(cw.values()) < TOL64, cw
    dv, _ = compare_divergence(sim, o)
    assert dv < TOL64, dv
    sim.close()


def test_fp64_gauss_law_invariant_on_gpu():
    """div_B E - P rho is constant in time on the GPU path (Eq. (10) with the
    filtered current), computed here from the library's own output."""
    _say("[gpu] fp64 Gauss invariant")
    pic = _pic()
    cfg = workloads.small(M=2, Nz=64, Nr=12, ppc=2)
    run = cfg["runs"][0]
    dt, CE, CB, _ = _setup(16, run["M"], run["dz"], run["dr"])
    sim = pic.Simulation([workloads.to_rundesc(run)], dt=dt, coef_E=CE, coef_B=CB)
    _, _, taps = sim.coefficients()
    N = CB.size
    dz, dr, Nz, Nr = run["dz"], run["dr"], run["Nz"], run["Nr"]

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


def _oracle_order(o, Tz, Tr, threads=256):
    """ids in (tile, cell, id) order from the oracle's own positions, each
    tile's list then stored transposed as the library's workgroup reads it:
    with n electrons and chunk = ceil(n / threads), round `it` holds
    L[c chunk + it] for the columns c with c chunk + it < n, ordered by
    (c mod S, c div S), where S (1, 2 or 4) is the smallest with
    S chunk Tz Tr >= n, or 4."""
    P = o.particles()
    ords = o.cell_order(Tz, Tr)
    order = np.lexsort((P["id"], ords))
    ids, tiles = P["id"][order], ords[order] // (Tz * Tr)
    out = []
    for tile in np.unique(tiles):
        L = ids[tiles == tile]
        n = L.size
        chunk = -(-n // threads)
        S = 1
        while S < 4 and S * chunk * Tz * Tr < n:
            S *= 2
        for it in range(chunk):
            c = np.arange(threads)
            c = c[c * chunk + it < n]
            c = c[np.lexsort((c // S, c % S))]
            out.append(L[c * chunk + it])
    return np.concatenate(out)


@pytest.mark.parametrize("precision", [64, 32])
def test_initial_cell_sort_bit_exact(precision):
    """The cell sort after loading orders electrons exactly as the oracle's
    (tile, cell, id) key on the identical loaded state."""
    _say(f"[gpu] initial sort fp{precision}")
    pic = _pic()
    run = workloads.config("c1")["runs"][0]
    dt, CE, CB, _ = _setup(16, run["M"], run["dz"], run["dr"])
    sim = pic.Simulation([workloads.to_rundesc(run)], precision=precision, dt=dt, coef_E=CE, coef_B=CB,
                         tile_z=32, tile_r=8)
    o = oracle_of(run, dt, CE, CB, fp32_start=(precision == 32))
    assert np.array_equal(sim.particles()["id"], _oracle_order(o, 32, 8))
    sim.close()


@pytest.mark.parametrize("ppc", [2, 3, 10])
def test_cell_sort_after_steps_bit_exact(ppc):
    """FP64 run with a sort every 4 steps: after 9 steps the order is the one
    the oracle's key gives for its state after 8 steps (16 x 4 tiles: with 2
    electrons per cell most tiles store their rounds with S = 2, with 3 with
    S = 4, in partly filled rounds; with 10 the tiles' cells are ranked in
    parallel instead of sorted one per thread)."""
    _say(f"[gpu] sort after 8 steps, {ppc} ppc")
    pic = _pic()
    run = workloads.small(M=2, Nz=96, Nr=20, ppc=ppc, n_tracked=10)["runs"][0]
    dt, CE, CB, _ = _setup(16, run["M"], run["dz"], run["dr"])
    sim = pic.Simulation([workloads.to_rundesc(run)], dt=dt, coef_E=CE, coef_B=CB, sort_interval=4,
                         tile_z=16, tile_r=4)
    o = oracle_of(run, dt, CE, CB)
    sim.step(9)
    o.step(8)
    assert np.array_equal(sim.particles()["id"], _oracle_order(o, 16, 4))
    sim.close()


def test_dense_tile_sort_bit_exact():
    """Tiles too dense for the sort's LDS budget (64 x 8 cells at 10 electrons
    per cell: over 5000 entries a tile) are sorted in device memory instead:
    the same order as the oracle's key, at start-up and after 8 steps."""
    _say("[gpu] dense-tile sort (device-memory path)")
    pic = _pic()
    run = workloads.small(M=0, Nz=128, Nr=17, ppc=10, n_tracked=10)["runs"][0]
    dt, CE, CB, _ = _setup(16, run["M"], run["dz"], run["dr"])
    sim = pic.Simulation([workloads.to_rundesc(run)], dt=dt, coef_E=CE, coef_B=CB, sort_interval=4,
                         tile_z=64, tile_r=8)
    o = oracle_of(run, dt, CE, CB)
    assert np.array_equal(sim.particles()["id"], _oracle_order(o, 64, 8))
    sim.step(9)
    o.step(8)
    assert np.array_equal(sim.particles()["id"], _oracle_order(o, 64, 8))
    sim.close()


def test_fp64_edge_case_largest_operators_ragged_grid_no_tracking():
    """The extremes at once: 32 coefficients per operator (the most the ABI
    takes), modes 0..3 (the most), no tracked electrons, a 70 x 13 grid that
    neither tile dimension divides (16 x 8 tiles), and a sort every step."""
    _say("[gpu] fp64 edge case: N=32, M=3, 70x13, no tracking, sort every step")
    pic = _pic()
    run = workloads.small(M=3, Nz=70, Nr=13, ppc=2, n_tracked=0)["runs"][0]
    dt, CE, CB, _ = _setup(32, 3, run["dz"], run["dr"])
    sim = pic.Simulation([workloads.to_rundesc(run)], dt=dt, coef_E=CE, coef_B=CB, n_coef=32, tile_z=16, tile_r=8,
                         sort_interval=1)
    o = oracle_of(run, dt, CE, CB)
    sim.step(12)
    o.step(12)
    worst = compare_fields(sim, o, run["M"], TOL64)
    bad = {k: v for k, v in worst.items() if v > TOL64}
    assert not bad, bad
    dzmax, dxy, du, _ = compare_particles(sim, o, run["Nz"])
    assert dzmax < TOL64 and dxy < TOL64 and du < TOL64, (dzmax, dxy, du)
    w = sim.mode_work()
    assert w["W"].shape == (0, 4) and w["id"].size == 0
    assert all(v.size == 0 for v in sim.cartesian_work().values())
    sim.close()


def test_fp64_smallest_grid_and_all_electrons_tracked():
    """The smallest grid the library accepts (Nz = 2N = 32 columns, so the
    16-coefficient stencils reach round the whole periodic line; Nr = 4, one
    tile row, electrons loaded in the three cells below the reflecting
    radius) with every electron tracked: fields, electrons and every
    electron's work against the oracle at the FP64 bar."""
    _say("[gpu] fp64 smallest grid, all electrons tracked")
    run = workloads.small(M=1, Nz=32, Nr=4, ppc=3, n_tracked=0)["runs"][0]
    run["n_tracked"] = 32 * 3 * 3
    sim, o = run_pair(run, 25)
    worst = compare_fields(sim, o, run["M"], TOL64)
    bad = {k: v for k, v in worst.items() if v > TOL64}
    assert not bad, bad
    dzmax, dxy, du, _ = compare_particles(sim, o, run["Nz"])
    assert dzmax < TOL64 and dxy < TOL64 and du < TOL64, (dzmax, dxy, du)
    wg, wo = sim.mode_work(), o.tracked()
    assert wg["id"].size == run["n_tracked"] and np.array_equal(wg["id"], wo["id"])
    assert np.abs(wg["W"] - wo["W"]).max() <= TOL64 * max(np.abs(wo["W"]).max(), 1e-300)
    assert np.abs(wg["gamma_acc"] - wg["gamma"]).max() < 1e-13 * max(1.0, wg["gamma"].max())
    sim.close()


def test_fp64_many_electrons_per_cell():
    """24 electrons per cell: each tile holds more electrons than four list
    columns per cell can keep in distinct cells, so a wavefront's lanes share
    cells and their LDS atomics collide; the result is still the oracle's to
    the FP64 bar."""
    _say("[gpu] fp64 24 ppc")
    run = workloads.small(M=2, Nz=64, Nr=12, ppc=24, n_tracked=50)["runs"][0]
    sim, o = run_pair(run, 10)
    worst = compare_fields(sim, o, run["M"], TOL64)
    bad = {k: v for k, v in worst.items() if v > TOL64}
    assert not bad, bad
    dzmax, dxy, du, _ = compare_particles(sim, o, run["Nz"])
    assert dzmax < TOL64 and dxy < TOL64 and du < TOL64, (dzmax, dxy, du)
    sim.close()


def test_fp64_electrons_outside_their_tile_window():
    """The push's other path: an electron that has moved out of its sort
    tile's LDS windows since the last sort gathers from and deposits to
    device memory directly.  A strong, long pulse (a0 = 4) over the whole
    small box drives the electrons forward at nearly c, the tiles are 8 x 1
    cells (the field window reaches one column past the tile in z and no row
    past it in r) and nothing is re-sorted after the first sort: over 32
    steps more than half of the electron-steps (checked here from the
    oracle's own trajectories) take that path.  FP64 bar, every array and
    electron, and the tracked work."""
    _say("[gpu] fp64 electrons outside their tile windows")
    pic = _pic()
    run = workloads.small(M=2, Nz=64, Nr=12, ppc=2, a0=4.0, n_tracked=64)["runs"][0]
    run["pulses"] = [dict(a0=4.0, w0=3 * workloads.LAMBDA0, tau=6 * workloads.LAMBDA0, zc=2 * workloads.LAMBDA0)]
    Tz, Tr, nsteps = 8, 1, 32
    dt, CE, CB, _ = _setup(16, run["M"], run["dz"], run["dr"])
    sim = pic.Simulation([workloads.to_rundesc(run)], dt=dt, coef_E=CE, coef_B=CB, tile_z=Tz, tile_r=Tr,
                         sort_interval=1000)
    o = oracle_of(run, dt, CE, CB)
    Nz = run["Nz"]

    def cells(P):
        r = np.sqrt(P["x"] ** 2 + P["y"] ** 2)
        return np.floor(P["z"]).astype(np.int64) % Nz, np.floor(r).astype(np.int64)

    iz0, ir0 = cells(o.particles())
    tz0, tr0 = iz0 // Tz, ir0 // Tr
    outside = total = 0
    for _ in range(nsteps):
        iz, ir = cells(o.particles())
        dzc = (iz - tz0 * Tz) % Nz
        dzc = np.where(dzc > Nz // 2, dzc - Nz, dzc)
        inside = (dzc >= -1) & (dzc <= Tz) & (ir >= tr0 * Tr) & (ir < tr0 * Tr + Tr)
        outside += int((~inside).sum())
        total += inside.size
        o.step(1)
    _say(f"  {outside / total:.2f} of the electron-steps outside their tile's windows")
    assert outside > 0.5 * total
    sim.step(nsteps)
    worst = compare_fields(sim, o, run["M"], TOL64)
    bad = {k: v for k, v in worst.items() if v > TOL64}
    assert not bad, bad
    dzmax, dxy, du, _ = compare_particles(sim, o, Nz)
    assert dzmax < TOL64 and dxy < TOL64 and du < TOL64, (dzmax, dxy, du)
    wg, wo = sim.mode_work(), o.tracked()
    assert np.array_equal(wg["id"], wo["id"])
    assert np.abs(wg["W"] - wo["W"]).max() <= TOL64 * max(np.abs(wo["W"]).max(), 1e-300)
    sim.close()
