"""Cartesian work estimate with the Pukhov correction -- oracle side (numpy, FP64).

TEST INFRASTRUCTURE ONLY: used by the tests; the product library computes its
own with no code in common.

Sec. III.B of the paper.  Without an azimuthal decomposition, the work on an
electron is split by field direction (Eq. (17)): W_z from E_z v_z and W_perp
from E_perp . v_perp.  A focused linearly polarised pulse also has a
longitudinal field, so part of W_z is the laser's.  For a small-amplitude
betatron orbit in resonance with the pulse, the cycle-averaged longitudinal
and transverse laser work have the ratio of Eq. (20),

    f = <W_z> / <W_perp> = -2 c^2 sqrt(2 gamma) / (omega_0 omega_p w_0^2),

and Eq. (21) moves that share from W_z to the laser:

    W*_LWFA = W_z - f W_perp,        W*_DLA = (1 + f) W_perp.

Units here: c = omega_0 = 1, density n0 in units of the critical density, so
omega_p = sqrt(n0); w_0 is the pulse waist in c / omega_0.  The reading taken
for gamma is the electron's Lorentz factor at the time of the estimate (the
paper gives one f per electron and does not say at which time; the end of the
run is the time at which Sec. IV.C compares the estimates).
"""
from __future__ import annotations

import numpy as np


def pukhov_ratio(gamma, n0: float, w0: float):
    """f of Eq. (20) for Lorentz factor(s) gamma, density n0 (n_c), waist w0."""
    wp = np.sqrt(n0)
    return -2.0 * np.sqrt(2.0 * np.asarray(gamma, dtype=np.float64)) / (wp * w0 * w0)


def corrected_work(wz, wperp, f):
    """(W*_LWFA, W*_DLA) of Eq. (21) from W_z, W_perp and f."""
    wz = np.asarray(wz, dtype=np.float64)
    wperp = np.asarray(wperp, dtype=np.float64)
    return wz - f * wperp, (1.0 + f) * wperp
