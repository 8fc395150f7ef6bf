"""Pins of the oracle's quadratic particle shapes (the order the paper leaves
open, Sec. III): the quadratic B-spline gather and the charge-conserving
deposit on 4 x 4 nodes, with the rows below the axis folded onto the rows
above it by each quantity's mirror sign.

Checked against what the mathematics fixes: a quadratic B-spline reproduces
linear fields exactly and adds its variance 1/4 cell^2 to a quadratic one;
the deposited charge has the particle's charge, dipole and (along z) second
moment plus that variance; the discrete Gauss law of the dual solver is
invariant through a step of one particle anywhere, the axis included, and
through a plasma run; the per-mode work still sums to the energy gain.
"""
import functools
import math

import numpy as np
import pytest

import oracle
from oracle import coef

LAMBDA0 = 2.0 * math.pi


@functools.lru_cache(maxsize=None)
def _setup(N, M, dz, dr):
    return coef.solver_setup(N, M, dz, dr)


def test_quadratic_gather_exact_for_linear_fields_and_adds_the_variance():
    Nz, Nr, M = 10, 7, 2
    dz, dr = 0.5, 0.7
    o = oracle.Oracle(Nz, Nr, M, dz, dr, 0.1, [1.0], [1.0])
    o.set_shape(2)
    zero = np.zeros((Nr + 1, Nz), dtype=complex)
    for c in range(9):
        for m in range(M + 1):
            o.set_field(c, m, zero)
    rows = np.arange(Nr + 1)[:, None] * np.ones((1, Nz))
    # E_x = 1.5, E_y = -0.4 (uniform, m = 1); E_z = 0.25 + 0.3 x; B_x = 0.2; B_z = -0.6 y
    o.set_field(oracle.ER, 1, (1.5 + 0.4j) + 0 * rows)
    o.set_field(oracle.EP, 1, (1.5j - 0.4) + 0 * rows)
    o.set_field(oracle.EZ, 0, 0.25 + 0 * rows)
    o.set_field(oracle.EZ, 1, 0.3 * rows * dr)
    for bc in (oracle.BOZ, oracle.BZ):
        o.set_field(bc, 1, 0.6j * (rows + 0.5) * dr)
    for bc, val in ((oracle.BOR, 0.2), (oracle.BR, 0.2), (oracle.BOP, 0.2j), (oracle.BP, 0.2j)):
        o.set_field(bc, 1, val + 0 * rows)
    rng = np.random.default_rng(5)
    for k in range(300):
        zc = rng.uniform(2, Nz - 2)
        r = rng.uniform(0, 0.6) if k % 3 == 0 else rng.uniform(0, Nr - 2.0)  # the axis rows mirrored
        ph = rng.uniform(0, 2 * np.pi)
        xc, yc = r * math.cos(ph), r * math.sin(ph)
        EB = o.gather(zc, xc, yc)
        X, Y = xc * dr, yc * dr
        assert np.allclose(EB, [1.5, -0.4, 0.25 + 0.3 * X, 0.2, 0.0, -0.6 * Y], rtol=0, atol=1e-13), (zc, xc, yc)
    # a quadratic field along z: E_z^0 at z_{i+1/2} = (i + 1/2)^2 cells^2 -> zc^2 + 1/4
    cols = (np.arange(Nz) + 0.5)[None, :] * np.ones((Nr + 1, 1))
    o.set_field(oracle.EZ, 0, cols ** 2)
    o.set_field(oracle.EZ, 1, zero)
    for _ in range(50):
        zc = rng.uniform(3, Nz - 3)
        r = rng.uniform(0, Nr - 2.0)
        EB = o.gather(zc, r, 0.0)
        assert abs(EB[2] - (zc ** 2 + 0.25)) < 1e-12


def _single_particle_run(p0, u, shape=2, Nz=12, Nr=8, M=3, dz=0.4, dr=1.2, dt=0.3, N=16, q=-1.0):
    CE, CB = coef.fit(N, dt / dz)
    o = oracle.Oracle(Nz, Nr, M, dz, dr, dt, CE, CB)
    o.set_shape(shape)
    z, x, y = p0
    o.set_particles([z], [x], [y], [u[0]], [u[1]], [u[2]], [-q])
    o.set_flags(deposit_rho=True)
    o.deposit_rho()
    G0 = [o.gauss_residual(m) for m in range(M + 1)]
    o.step(1)
    G1 = [o.gauss_residual(m) for m in range(M + 1)]
    return o, G0, G1


@pytest.mark.parametrize("seed", range(24))
def test_quadratic_single_particle_gauss_invariant(seed):
    """div_B E - P rho stays constant through a full step for one particle
    with quadratic shape, for every mode: within half a cell of the axis
    (rows folded), crossing r = dr/2 and cell faces, next to the wall, and
    across the seam."""
    rng = np.random.default_rng(100 + seed)
    Nz = 12
    z = rng.choice([rng.uniform(0, Nz), rng.uniform(Nz - 0.3, Nz), rng.uniform(0, 0.3)])
    r = rng.choice([rng.uniform(0, 0.5), rng.uniform(0.4, 0.6), rng.uniform(0.9, 1.6), rng.uniform(0, 5.0),
                    rng.uniform(5.5, 6.9)])  # the last: the stencil reaches the wall row r_8
    ph = rng.uniform(0, 2 * np.pi)
    u = rng.normal(size=3) * 3.0
    o, G0, G1 = _single_particle_run((z, r * math.cos(ph), r * math.sin(ph)), u, Nz=Nz)
    scale = max(np.abs(g).max() for g in G0)
    for m in range(o.M + 1):
        assert np.abs(G1[m] - G0[m]).max() < 1e-13 * scale, (m, np.abs(G1[m] - G0[m]).max(), scale)


def test_quadratic_deposit_moments():
    """Charge, dipole and the z second moment (plus the spline's variance
    1/4 cell^2) of rho, and the current's moments, equal a point particle's;
    the fold of the axis rows keeps the charge, the dipole and the magnetic
    moment exact."""
    Nz, Nr, M = 12, 8, 2
    dz, dr, dt = 0.4, 1.3, 0.35
    o = oracle.Oracle(Nz, Nr, M, dz, dr, dt, [1.0], [1.0])
    o.set_shape(2)
    V = np.array([math.pi * dr * dr * dz / 4] + [2 * math.pi * j * dr * dr * dz for j in range(1, Nr + 1)])
    rj = np.arange(Nr + 1) * dr
    zi = np.arange(Nz) * dz
    rng = np.random.default_rng(11)
    q = -0.7
    for k in range(24):
        z0 = rng.uniform(2, Nz - 3)
        r0 = rng.uniform(0, 0.5) if k % 3 == 0 else rng.uniform(0, Nr - 3.0)
        ph0 = rng.uniform(0, 2 * math.pi)
        x0, y0 = r0 * math.cos(ph0), r0 * math.sin(ph0)
        o.set_particles([z0], [x0], [y0], [0.0], [0.0], [0.0], [-q])
        o.deposit_rho()
        rho0, rho1 = o.get_field(oracle.RHO, 0), o.get_field(oracle.RHO, 1)
        Q0 = rho0.real * V[:, None]
        assert abs(np.sum(Q0) - q) < 1e-14
        assert abs(np.sum(Q0 * zi[None, :]) - q * z0 * dz) < 1e-13
        assert abs(np.sum(Q0 * zi[None, :] ** 2) - q * ((z0 * dz) ** 2 + dz * dz / 4)) < 1e-13
        d = np.sum(rho1 * (V * rj / 2.0)[:, None])
        assert abs(d - q * (x0 - 1j * y0) * dr) < 1e-13
        dzc, dxc, dyc = rng.uniform(-0.9, 0.9), rng.uniform(-0.2, 0.2), rng.uniform(-0.2, 0.2)
        z1, x1, y1 = z0 + dzc, x0 + dxc, y0 + dyc
        vphi = rng.normal()
        o.deposit_one(q, (z0, x0, y0), (z1, x1, y1), vphi)
        Jz0 = o.get_field(oracle.JZ, 0)
        Jp0 = o.get_field(oracle.JP, 0)
        r1 = math.hypot(x1, y1)
        assert abs(np.sum(Jz0.real * V[:, None]) - q * dzc * dz / dt) < 1e-13
        # the azimuthal current's magnetic moment (1/2) int r J_phi dV is the
        # particle's, q v_phi times the mean radius of the two positions, also
        # near the axis: the fold spreads the current as a vector (the row
        # r_{-1} seen from r_1 points the other way round the axis)
        mu = 0.5 * np.sum(Jp0.real * (V * rj)[:, None])
        assert abs(mu - 0.5 * q * vphi * 0.5 * (r0 + r1) * dr) < 1e-13
        if r0 > 1.6:  # away from the fold: the radial current's moment is the move's
            Jr0 = o.get_field(oracle.JR, 0)
            Ar = 2 * math.pi * (np.arange(Nr + 1) + 0.5) * dr * dz
            assert abs(np.sum(Jr0.real * (Ar * dr)[:, None]) - q * (r1 - r0) * dr / dt) < 1e-13
            assert abs(np.sum(Jp0.real * V[:, None]) - q * vphi) < 1e-13


@functools.lru_cache(maxsize=None)
def _plasma_run(shape, nsteps=20):
    Nz, Nr, M = 64, 12, 2
    dz = LAMBDA0 / 16
    dr = 4 * dz
    dt, CE, CB, _ = _setup(16, M, dz, dr)
    o = oracle.Oracle(Nz, Nr, M, dz, dr, dt, CE, CB)
    o.set_shape(shape)
    o.load_plasma(2, 0.02, seed=99, n_tracked=64)
    o.add_laser(1.5, 3 * LAMBDA0, 2 * LAMBDA0, 2 * LAMBDA0, taper=LAMBDA0)
    o.start_fields()
    o.set_flags(deposit_rho=True)
    o.deposit_rho()
    G0 = [o.gauss_residual(m) for m in range(M + 1)]
    o.step(nsteps)
    G1 = [o.gauss_residual(m) for m in range(M + 1)]
    return o, G0, G1


def test_quadratic_plasma_run_gauss_law_and_work_identity():
    o, G0, G1 = _plasma_run(2)
    for m in range(o.M + 1):
        scale = np.abs(G1[m]).max() + np.abs(G0[m]).max()
        assert np.abs(G1[m] - G0[m]).max() < 1e-13 * scale, m
    t = o.tracked()
    assert np.abs(t["gamma_acc"] - t["gamma"]).max() < 1e-12
    # the switch changes the physics: linear and quadratic runs differ
    o1, _, _ = _plasma_run(1)
    a, b = o.get_field(oracle.EZ, 0), o1.get_field(oracle.EZ, 0)
    assert np.abs(a - b).max() > 1e-6 * np.abs(b).max()
