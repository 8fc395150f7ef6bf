"""Pins of the reduced-model oracle (Sec. II, Eq. (8); App. A) against what
the mathematics and the physics fix: the order of the integrator, the two
constants of motion of the model's fields (bubble alone: gamma - p_z - psi;
laser alone: gamma - v_phi (p_z - A_z)), the betatron frequency of Eq. (1),
and the constraints of the injection recipe."""
import math

import numpy as np
import pytest

import workloads
from oracle import dla


def _electrons(n=8, seed=1):
    d = workloads.dla_injection(n, seed)
    y0 = np.stack([d["x"], d["zeta"], d["xd"], d["zetad"]])
    return d, y0


def test_dp5_is_fifth_order():
    """y'' = -y from (1, 0) to t = 2: the error falls by ~2^5 per halving of
    h, and at h = 0.01 it is below 1e-12 (cos and -sin exactly)."""
    f = lambda t, y: np.stack([y[1], -y[0]])

    def err(h):
        y = np.array([[1.0], [0.0]])
        n = int(round(2.0 / h))
        for k in range(n):
            y = dla.dp5_step(f, k * h, y, h)
        return max(abs(y[0, 0] - math.cos(2.0)), abs(y[1, 0] + math.sin(2.0)))

    e1, e2 = err(0.2), err(0.1)
    assert 25.0 < e1 / e2 < 40.0, e1 / e2
    assert err(0.01) < 1e-12


def _wake_invariant(p, t, y):
    g = dla.gamma(y)
    psi = (p["R"] ** 2 - y[1] ** 2 - y[0] ** 2) / 4.0
    return g - g * (y[3] + 1.0) - psi


def _laser_invariant(p, t, y):
    g = dla.gamma(y)
    xi = y[1] + (1.0 - p["vphi"]) * t
    az = p["a0"] * (p["kperp"] / p["kz"]) * dla.bessel(p["kperp"] * y[0])[1] * np.sin(p["kz"] * xi)
    return g - p["vphi"] * (g * (y[3] + 1.0) - az)


def test_bubble_alone_conserves_gamma_minus_pz_minus_psi():
    """With a0 = 0 the fields depend on z - t only, so gamma - p_z - psi is a
    constant of motion (psi of Eq. (6)); the integrated Eq. (8) keeps it."""
    p = dla.params(a0=0.0)
    d, y0 = _electrons()
    t0 = np.zeros(y0.shape[1])
    y = dla.integrate(p, t0, y0, 30.0, 0.01)
    drift = np.abs(_wake_invariant(p, 30.0, y) - _wake_invariant(p, t0, y0))
    assert drift.max() < 1e-11 * dla.gamma(y).max(), drift.max()
    assert np.abs(dla.gamma(y) - d["gamma"]).max() > 1.0  # the bubble does work


def test_laser_alone_conserves_gamma_minus_vphi_canonical_pz():
    """Without the bubble the fields depend on z - v_phi t only (Eqs. (4)-(5),
    Coulomb gauge, no scalar potential), so gamma - v_phi (p_z - A_z) is
    constant (charge -1: canonical p - A); Eq. (8)'s laser terms keep it."""
    p = dla.params(wake=0.0)
    d, y0 = _electrons()
    t0 = np.zeros(y0.shape[1])
    y = dla.integrate(p, t0, y0, 30.0, 0.005)
    drift = np.abs(_laser_invariant(p, 30.0, y) - _laser_invariant(p, t0, y0))
    assert drift.max() < 1e-10 * dla.gamma(y).max(), drift.max()
    assert np.abs(dla.gamma(y) - d["gamma"]).max() > 0.1  # the laser does work


def test_staggering_factor_acts_on_the_magnetic_terms():
    """cB != 1 unbalances the laser's electric and magnetic forces, so the
    laser-alone constant of motion drifts by far more than round-off; cB = 1
    restores it (previous test)."""
    p = dla.params(wake=0.0, cB=math.cos(0.1))
    _, y0 = _electrons()
    t0 = np.zeros(y0.shape[1])
    y = dla.integrate(p, t0, y0, 30.0, 0.005)
    drift = np.abs(_laser_invariant(p, 30.0, y) - _laser_invariant(p, t0, y0))
    assert drift.max() > 1e-3


@pytest.mark.parametrize("g", [200.0, 2000.0])
def test_betatron_frequency_in_the_bubble(g):
    """A fast electron at the bubble centre with a small offset oscillates at
    omega_beta = omega_p / sqrt(2 gamma) (Eq. (1)): the first zero of x comes
    after a quarter period, pi/2 sqrt(2 gamma), to 1 %."""
    p = dla.params(a0=0.0)
    A = 1e-3
    vz = math.sqrt(1.0 - 1.0 / g ** 2)
    y = np.array([[A], [0.0], [0.0], [vz - 1.0]])
    quarter = 0.5 * math.pi * math.sqrt(2.0 * g)
    h = quarter / 400.0
    t = 0.0
    while y[0, 0] > 0:
        yp, tp = y, t
        y = dla.dp5_step(lambda tt, yy: dla.rhs(p, tt, yy), t, y, h)
        t += h
    tz = tp + h * yp[0, 0] / (yp[0, 0] - y[0, 0])
    assert abs(tz / quarter - 1.0) < 0.01, tz / quarter


def test_injection_follows_the_recipe():
    """App. A: t0 in [0, 200]; zeta in [-2R + 0.286, -2R + 0.836]; |x| <=
    r_b(zeta); gamma in [gamma_g, 2 gamma_g] and equal to the gamma of the
    state; v_z >= v_g."""
    R, vg = 3.0, 0.993583
    d = workloads.dla_injection(20000, 7, R=R, vg=vg)
    assert np.all(np.diff(d["t0"]) >= 0) and d["t0"].min() >= 0 and d["t0"].max() <= 200.0
    assert d["zeta"].min() >= -2 * R + 0.286 and d["zeta"].max() <= -2 * R + 0.836
    assert np.all(np.abs(d["x"]) <= np.sqrt(R * R - (d["zeta"] + R) ** 2))
    gg = 1.0 / math.sqrt(1 - vg * vg)
    assert d["gamma"].min() >= gg and d["gamma"].max() <= 2 * gg
    y = np.stack([d["x"], d["zeta"], d["xd"], d["zetad"]])
    assert np.abs(dla.gamma(y) / d["gamma"] - 1).max() < 1e-9
    assert np.all(d["zetad"] + 1.0 >= vg - 1e-15)
