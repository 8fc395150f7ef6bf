"""Reduced model of an electron in a bubble with a laser pulse -- oracle side
(numpy, FP64).

TEST INFRASTRUCTURE ONLY: used by the tests and the smoke check; the product
library integrates the same model with no code in common.

Sec. II of the paper.  Units c = omega_p = 1 (time 1/omega_p, length
c/omega_p), electron charge -1, motion in the x-z plane (y = 0).  The laser
(Eqs. (4)-(5)) is a Bessel mode of the bubble channel with longitudinal
wavenumber k_z, phase velocity v_phi, frequency omega_0 = k_z v_phi and
transverse wavenumber k_perp = (omega_0^2 - k_z^2)^(1/2); the bubble (Eq. (6))
is spherical with radius R and moves at c.  Eq. (8) gives the coordinate
accelerations in the form

    xdd    + (gdot/g) xd         + (w_b^2 / 2)(1 + zd) x        = RHS_x,
    zetadd + (gdot/g)(zetad + 1) + w_b^2 (zeta - x xd / 2)      = RHS_zeta,

with zd = zetad + 1, w_b^2 = 1 / (2 g) (Eq. (1)), xi = z - v_phi t =
zeta + (1 - v_phi) t, s = k_perp x and

    RHS_x    =  (a0/g) [ w0 J0(s) - cB k_z zd (J0(s) + (k_perp/k_z)^2 J1'(s)) ] sin(k_z xi),
    RHS_zeta = -(a0/g) [ (k_perp/k_z) w0 J1(s) cos(k_z xi)
                         - cB k_z xd (J0(s) + (k_perp/k_z)^2 J1'(s)) sin(k_z xi) ].

cB multiplies the laser's magnetic terms (those with a velocity times
sin(k_z xi)); cB = cos(omega_0 dt / 2) models the time-staggering error of a
Yee-type PIC step (Sec. IV.A), cB = 1 the exact fields.  `wake` multiplies the
bubble terms (1: the model; 0: the laser alone, used by the pins).

The left-hand sides are (d/dt)(g v) / g, so with G the right-hand side minus
the bubble terms (the force over g), energy balance gives gdot/g = G . v and
the system is explicit:  a = G - (G . v) v  (z component with zd = zetad + 1).

Integration (App. A): an explicit fifth-order Runge-Kutta method; the paper
does not name the scheme.  Reading: the fifth-order solution of the
Dormand-Prince 5(4) pair (six stages) at a fixed step.  Each electron starts
at its own injection time t0 and takes n = ceil((t_end - t0) / h) steps of
length (t_end - t0) / n.
"""
from __future__ import annotations

import math

import numpy as np
from scipy import special

# Dormand & Prince (1980), the fifth-order solution of their 5(4) pair
_C = (0.0, 1.0 / 5.0, 3.0 / 10.0, 4.0 / 5.0, 8.0 / 9.0, 1.0)
_A = ((),
      (1.0 / 5.0,),
      (3.0 / 40.0, 9.0 / 40.0),
      (44.0 / 45.0, -56.0 / 15.0, 32.0 / 9.0),
      (19372.0 / 6561.0, -25360.0 / 2187.0, 64448.0 / 6561.0, -212.0 / 729.0),
      (9017.0 / 3168.0, -355.0 / 33.0, 46732.0 / 5247.0, 49.0 / 176.0, -5103.0 / 18656.0))
_B = (35.0 / 384.0, 0.0, 500.0 / 1113.0, 125.0 / 192.0, -2187.0 / 6784.0, 11.0 / 84.0)


def params(a0=2.8, kz=12.14, vphi=1.002565, R=3.0, cB=1.0, wake=1.0) -> dict:
    """Model parameters; the defaults are the values App. A gives (c = omega_p = 1)."""
    w0 = kz * vphi
    return {"a0": a0, "kz": kz, "vphi": vphi, "w0": w0, "kperp": math.sqrt(w0 * w0 - kz * kz), "R": R, "cB": cB,
            "wake": wake}


def bessel(s):
    """J0(s), J1(s) and J1'(s) = J0(s) - J1(s)/s (1/2 at s = 0)."""
    s = np.asarray(s, dtype=np.float64)
    j0, j1 = special.j0(s), special.j1(s)
    small = np.abs(s) < 1e-4
    safe = np.where(small, 1.0, s)
    j1p = np.where(small, 0.5 - 3.0 * s * s / 16.0, j0 - j1 / safe)
    return j0, j1, j1p


def rhs(p: dict, t, y):
    """d/dt of the state y = (x, zeta, xd, zetad) (arrays of equal shape)."""
    x, zeta, u, w = y
    zd = w + 1.0
    g = 1.0 / np.sqrt(-w * (2.0 + w) - u * u)  # 1 - v^2 without the cancellation of 1 - zd^2
    wb2 = 1.0 / (2.0 * g)
    xi = zeta + (1.0 - p["vphi"]) * t
    j0, j1, j1p = bessel(p["kperp"] * x)
    kk = (p["kperp"] / p["kz"]) ** 2
    sn, cs = np.sin(p["kz"] * xi), np.cos(p["kz"] * xi)
    amp = p["a0"] / g
    rhs_x = amp * (p["w0"] * j0 - p["cB"] * p["kz"] * zd * (j0 + kk * j1p)) * sn
    rhs_z = -amp * ((p["kperp"] / p["kz"]) * p["w0"] * j1 * cs - p["cB"] * p["kz"] * u * (j0 + kk * j1p) * sn)
    gx = rhs_x - p["wake"] * 0.5 * wb2 * (1.0 + zd) * x
    gz = rhs_z - p["wake"] * wb2 * (zeta - 0.5 * x * u)
    gv = gx * u + gz * zd  # gdot / g
    return np.stack([u, w, gx - gv * u, gz - gv * zd])


def dp5_step(f, t, y, h):
    """One step of the fifth-order Dormand-Prince solution for y' = f(t, y)."""
    k = []
    for i in range(6):
        yi = y
        for j, a in enumerate(_A[i]):
            yi = yi + h * a * k[j]
        k.append(f(t + _C[i] * h, yi))
    out = y
    for b, kk in zip(_B, k):
        if b != 0.0:
            out = out + h * b * kk
    return out


def integrate(p: dict, t0, y0, t_end: float, h: float):
    """Each electron from its own t0 to t_end in n = ceil((t_end - t0)/h)
    equal steps.  y0: (4, n) array; returns the (4, n) state at t_end."""
    t0 = np.asarray(t0, dtype=np.float64)
    y = np.array(y0, dtype=np.float64, copy=True)
    nstep = np.maximum(0, np.ceil((t_end - t0) / h)).astype(np.int64)
    hs = np.where(nstep > 0, (t_end - t0) / np.maximum(nstep, 1), 0.0)
    for k in range(int(nstep.max(initial=0))):
        act = nstep > k
        t = t0[act] + k * hs[act]
        y[:, act] = dp5_step(lambda tt, yy: rhs(p, tt, yy), t, y[:, act], hs[act])
    return y


def gamma(y):
    """Lorentz factor of states y = (x, zeta, xd, zetad)."""
    u, w = y[2], y[3]
    return 1.0 / np.sqrt(-w * (2.0 + w) - u * u)
