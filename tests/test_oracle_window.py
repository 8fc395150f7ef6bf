"""Pins of the oracle's moving window (App. A: the box follows the pulse
through a plasma longer than the box).

The reading (the paper gives no mechanism): before a step whose count of
steps taken is a positive multiple of K, the box advances by the whole cells
a front moving at c has crossed since the start; fields move back with zeros
entering at the front and a guard band at the back cleared; electrons move
back, those outside the box are dropped, and the plasma of the new absolute
columns is loaded exactly as the initial load would load it.  An electron
that leaves the box carries no charge from the next step on.

Each pin checks the window against something other than itself: a static
run of the same pulse, a fresh load of a longer box, Gauss's law of the
static solver, the cadence formula.
"""
import functools
import math

import numpy as np
import pytest

import oracle
from oracle import coef

LAMBDA0 = 2.0 * math.pi


@functools.lru_cache(maxsize=None)
def _setup(M, dz, dr):
    return coef.solver_setup(16, M, dz, dr)


def _grid(Nz=192, Nr=16, M=1):
    dz = LAMBDA0 / 16
    dr = 4 * dz
    dt, CE, CB, _ = _setup(M, dz, dr)
    return Nz, Nr, M, dz, dr, dt, CE, CB


def _oracle(Nz, Nr, M, dz, dr, dt, CE, CB):
    return oracle.Oracle(Nz, Nr, M, dz, dr, dt, CE, CB)


def _laser_energy_by_column(o):
    e = sum(np.abs(o.get_field(c, 1)) ** 2 for c in (oracle.ER, oracle.EP, oracle.EZ))
    return (e * (np.arange(o.Nr + 1) + 0.5)[:, None]).sum(axis=0)


def test_window_cadence_is_the_light_front():
    """S after n steps is floor(n' dt / dz) at the last move, n' the largest
    positive multiple of K with n' < n + 1 (moves happen before a step)."""
    g = _grid(Nz=64, Nr=8)
    o = _oracle(*g)
    dt, dz = g[5], g[3]
    K = 3
    o.set_window(K)
    for n in range(1, 40):
        o.step(1)
        last = (n // K) * K if n % K else n - K  # moves before steps whose count taken is a multiple of K
        last = max(last, 0)
        want = math.floor(last * dt / dz) if last > 0 else 0
        assert o.window_cells == want, (n, o.window_cells, want)


def test_window_vacuum_pulse_moves_with_the_box():
    """In vacuum the pulse travels at c (Eq. (10) with the fitted
    coefficients): in the static box its energy centroid advances by c t, in
    the moving box it stays within a cell of where it started, and the
    moving-box fields are the static fields shifted by the cells moved."""
    Nz, Nr, M, dz, dr, dt, CE, CB = _grid(Nz=256, Nr=24, M=1)
    stat = _oracle(Nz, Nr, M, dz, dr, dt, CE, CB)
    mov = _oracle(Nz, Nr, M, dz, dr, dt, CE, CB)
    for o in (stat, mov):
        o.add_laser(1.0, 4 * LAMBDA0, 2 * LAMBDA0, 6 * LAMBDA0, taper=LAMBDA0)
        o.start_fields()
    mov.set_window(4)
    col = np.arange(Nz)

    def centroid(o):
        w = _laser_energy_by_column(o)
        return (w * col).sum() / w.sum()

    c0 = centroid(mov)
    n = 81  # the last move comes before step 81: 80 steps of travel
    stat.step(n)
    mov.step(n)
    S = mov.window_cells
    assert S == math.floor(80 * dt / dz) and S > 40
    assert abs(centroid(mov) - c0) < 1.5 + n * dt / dz * 0.02
    assert abs(centroid(stat) - c0 - n * dt / dz) < 0.02 * n * dt / dz
    # away from the seam the moved fields are the static ones, shifted by S:
    # they differ only by what the static box carries round its periodic z
    # ends, which the window replaces by fresh vacuum (the pulse's small
    # non-local tail, 1e-4 of its peak); a shift one cell off would differ by
    # k0 dz = 0.4 of the peak
    inner = slice(24, Nz - S - 24)
    for comp in (oracle.ER, oracle.EP, oracle.EZ, oracle.BR, oracle.BP, oracle.BZ):
        a = mov.get_field(comp, 1)[:, inner]
        b = np.roll(stat.get_field(comp, 1), -S, axis=1)[:, inner]
        scale = np.abs(stat.get_field(comp, 1)).max()
        assert np.abs(a - b).max() <= 1e-3 * scale, comp
        b1 = np.roll(stat.get_field(comp, 1), -S - 1, axis=1)[:, inner]
        assert np.abs(a - b1).max() > 0.1 * scale, comp


def test_window_fresh_plasma_is_the_load_of_the_advanced_box():
    """With the fields frozen at zero nothing moves, so after the window has
    advanced by S cells the box holds exactly (bit for bit) the electrons a
    load of absolute columns [S, S + Nz) produces: those of a longer box's
    load with column >= S, shifted back by S."""
    Nz, Nr, M, dz, dr, dt, CE, CB = _grid(Nz=48, Nr=6, M=1)
    mov = _oracle(Nz, Nr, M, dz, dr, dt, CE, CB)
    mov.load_plasma(3, 0.02, ramp_start=10 * dz, ramp_len=30 * dz, seed=7)
    mov.set_flags(freeze_fields=True)
    mov.set_window(2)
    mov.step(31)
    S = mov.window_cells
    assert S == math.floor(30 * dt / dz) and S > 10
    ref = _oracle(Nz + S, Nr, M, dz, dr, dt, CE, CB)
    ref.load_plasma(3, 0.02, ramp_start=10 * dz, ramp_len=30 * dz, seed=7)
    P, Q = mov.particles(), ref.particles()
    keep = Q["z"] >= S
    order_p, order_q = np.argsort(P["id"]), np.argsort(Q["id"][keep])
    assert np.array_equal(P["id"][order_p], Q["id"][keep][order_q])
    for k in ("x", "y", "w", "ux", "uy", "uz"):
        assert np.array_equal(P[k][order_p], Q[k][keep][order_q]), k
    assert np.array_equal(P["z"][order_p] + S, Q["z"][keep][order_q])
    # the dropped electrons are exactly those of the columns left behind
    assert mov.np == (Nz) * (Nr - 1) * 3


def test_window_gauss_law_across_moves():
    """Gauss's law of the dual solver (div_B E - rho, Eq. (10)) is invariant
    in the static box; with the window it is the residual of the freshly
    loaded box at the same absolute position, away from the seam and the
    guard band, after the pulse and the plasma have moved through several
    window moves."""
    Nz, Nr, M, dz, dr, dt, CE, CB = _grid(Nz=160, Nr=12, M=2)
    guard = 8
    mov = _oracle(Nz, Nr, M, dz, dr, dt, CE, CB)
    mov.load_plasma(2, 0.03, ramp_start=0.0, ramp_len=20 * dz, seed=11, n_tracked=32)
    mov.add_laser(2.0, 3 * LAMBDA0, 2 * LAMBDA0, 5 * LAMBDA0, taper=LAMBDA0)
    mov.start_fields()
    mov.set_flags(deposit_rho=True)
    mov.set_window(4, guard=guard)
    mov.step(41)
    S = mov.window_cells
    assert S > 20
    ref = _oracle(Nz + S, Nr, M, dz, dr, dt, CE, CB)
    ref.load_plasma(2, 0.03, ramp_start=0.0, ramp_len=20 * dz, seed=11)
    ref.add_laser(2.0, 3 * LAMBDA0, 2 * LAMBDA0, 5 * LAMBDA0, taper=LAMBDA0)
    ref.start_fields()
    ref.deposit_rho()
    # Exact (round-off) from the guard band plus one stencil up to the part
    # of the box that entered at the front during the run (plus a stencil):
    # there each move replaced the pulse's small forward leak by fresh vacuum,
    # which changes div E by that leak (a few 1e-4 of the residual's scale).
    lo, hi = guard + 16, Nz - S - 40
    assert hi - lo > 50
    for m in range(M + 1):
        g = mov.gauss_residual(m)
        r = ref.gauss_residual(m)[:, S:S + Nz]
        scale = np.abs(r).max()
        assert np.abs(g - r)[:, lo:hi].max() < 1e-12 * scale, m
        assert np.abs(g - r)[:, lo:Nz - 24].max() < 3e-3 * scale, m
    # the plasma moved: the check is not of an unperturbed box
    assert np.abs(mov.particles()["uz"]).max() > 1e-3


def test_window_electron_leaving_carries_no_charge():
    """An electron that crosses z = 0 backwards keeps its position outside the
    box with zero weight and is dropped at the next move; one inside keeps
    its charge."""
    Nz, Nr, M, dz, dr, dt, CE, CB = _grid(Nz=64, Nr=8, M=1)
    o = _oracle(Nz, Nr, M, dz, dr, dt, CE, CB)
    z = np.array([0.3, 30.0])
    x = np.array([2.5, 2.5])
    y = np.zeros(2)
    ux = np.zeros(2)
    uz = np.array([-5.0, 0.0])
    w = np.array([1e-3, 1e-3])
    o.set_particles(z, x, y, ux, y, uz, w)
    o.set_flags(freeze_fields=True)
    o.set_window(8)
    o.step(1)
    P = o.particles()
    assert P["z"][0] < 0.0 and P["w"][0] == 0.0 and P["w"][1] == 1e-3
    o.step(8)  # the move before step 9 drops it
    P = o.particles()
    assert list(P["id"]) == [1]
    t = o.tracked()
    assert np.isnan(t["gamma"][0]) and t["gamma"][1] == 1.0
    assert list(t["id"]) == [0, 1]
