"""Dual-solver z-stencil coefficients and Courant limit -- oracle side (numpy, FP64).

TEST INFRASTRUCTURE ONLY: used by the tests, the smoke check and the CPU
baseline of the benchmark; the product library computes its own with no code
in common.

Sec. III.A of the paper.  The finite-difference z-derivative applied to E
(operator D_E) and the one applied to B (operator D_B) are staggered central
differences with N coefficients each,

    (D f)_{i+1/2} = sum_{l=1..N} C_l (f_{i+l} - f_{i-l+1}) / dz,

whose Fourier symbols are [k] = sum_l C_l 2 sin((2l-1) k dz / 2) / dz.  Two
conditions fix the targets: Eq. (11), [k]_B [k]_E = (sin(c k dt/2)/(c dt/2))^2,
exact light dispersion; and Eq. (15), sqrt([k]_E/[k]_B) cos(c k dt/2) = 1, no
E/B time-staggering error in the Lorentz force.  Their product and quotient
give the two targets separately:

    [k]_E = tan(c k dt/2) / (c dt/2),     [k]_B = sin(c k dt) / (c dt).

The paper leaves the fitting procedure and its accuracy open; the reading used here is a least-squares fit of each operator on
k dz in (0, 2 pi/3] (4000 midpoint samples) under the consistency constraint
sum_l (2l-1) C_l = 1, solved in the null space of the constraint.

Stability (von Neumann, periodic z): with mu the largest eigenvalue of the
discrete curl_B curl_E, leapfrog is stable iff (dt/2)^2 mu <= 1.  The z part
contributes max_k [k]_B[k]_E and the radial part a mode-dependent lambda_r(m)/dr^2
(largest eigenvalue of the radial operator at k_z = 0, axis rules included);
the two add.  The radial eigenvalue is measured by running the oracle's own
field step as a black box on a one-cell-long periodic grid.
"""
from __future__ import annotations

import numpy as np

BAND = 2.0 * np.pi / 3.0
NSAMP = 4000
KAPPA_MAX_SAMPLES = 20001


def target_symbols(kappa, nu):
    """dz*[k]_E and dz*[k]_B targets at kappa = k dz, nu = c dt / dz (Eqs. (11), (15))."""
    x = np.asarray(kappa, dtype=np.float64) * nu
    return np.tan(0.5 * x) / (0.5 * nu), np.sin(x) / nu


def symbol(C, kappa):
    """dz * [k] of a staggered difference with coefficients C_1..C_N."""
    C = np.asarray(C, dtype=np.float64)
    l = np.arange(1, C.size + 1, dtype=np.float64)
    kap = np.asarray(kappa, dtype=np.float64)
    return (2.0 * np.sin(np.multiply.outer(kap, 2.0 * l - 1.0) * 0.5)) @ C


def fit(N: int, nu: float, band: float = BAND, nsamp: int = NSAMP):
    """Constrained least-squares fit of (C^E, C^B), N coefficients each."""
    if N == 1:
        return np.array([1.0]), np.array([1.0])
    kap = (np.arange(nsamp, dtype=np.float64) + 0.5) * (band / nsamp)
    l = np.arange(1, N + 1, dtype=np.float64)
    A = 2.0 * np.sin(np.multiply.outer(kap, 2.0 * l - 1.0) * 0.5)
    g = 2.0 * l - 1.0
    c_part = g / (g @ g)
    Q, _ = np.linalg.qr(g[:, None], mode="complete")
    Z = Q[:, 1:]
    AZ = A @ Z
    out = []
    for T in target_symbols(kap, nu):
        y, *_ = np.linalg.lstsq(AZ, T - A @ c_part, rcond=None)
        out.append(c_part + Z @ y)
    return out[0], out[1]


def filter_taps(CB):
    """Taps p_l (l = -(N-1)..N-1) of the z filter with D_B = D_Yee o P."""
    CB = np.asarray(CB, dtype=np.float64)
    N = CB.size
    p = np.array([CB[l:].sum() for l in range(1, N)] + [0.0])  # p_l, l = 1..N
    half = np.concatenate([[CB.sum()], p[:-1]])  # p_0 .. p_{N-1}
    return np.concatenate([half[:0:-1], half])


def zmax_product(CE, CB, samples: int = KAPPA_MAX_SAMPLES):
    """(max, min) of dz^2 [k]_B [k]_E over k dz in (0, pi]."""
    kap = np.linspace(0.0, np.pi, samples)[1:]
    prod = symbol(CB, kap) * symbol(CE, kap)
    return float(prod.max()), float(prod.min())


def radial_lambda(m: int, nr: int = 32) -> float:
    """dr^2 * largest eigenvalue of curl_B curl_E of mode m at k_z = 0.

    Built by applying the oracle's own field step to unit vectors of a
    one-cell-long periodic grid (every z difference then vanishes) and reading
    mu = (2 - 2 Re lambda) / dt^2 from the unit-modulus eigenvalues lambda of
    the step (entries held at zero by the axis and wall rules give lambda = 0)."""
    from . import Oracle  # local import: the C oracle

    dr = 1.0
    dt = 0.05
    o = Oracle(1, nr, m, 1.0, dr, dt, [1.0], [1.0])
    n = nr + 1
    comps = [0, 1, 2, 6, 7, 8]  # E_r, E_phi, E_z, B^{n+1/2} r, phi, z
    dim = len(comps) * n
    T = np.zeros((dim, dim), dtype=np.complex128)
    zero = np.zeros((n, 1), dtype=np.complex128)
    for col in range(dim):
        for c in comps:
            o.set_field(c, m, zero)
        ci, j = divmod(col, n)
        v = zero.copy()
        v[j, 0] = 1.0
        o.set_field(comps[ci], m, v)
        o.field_step(1)
        T[:, col] = np.concatenate([o.get_field(c, m)[:, 0] for c in comps])
    lam = np.linalg.eigvals(T)
    lam = lam[np.abs(lam) > 0.5]  # drop the null space of entries held at zero
    mu = (2.0 - 2.0 * lam.real) / dt**2
    return float(mu.max()) * dr**2


_RADIAL_CACHE: dict[int, float] = {}


def radial_lambda_max(M: int) -> float:
    out = 0.0
    for m in range(M + 1):
        if m not in _RADIAL_CACHE:
            _RADIAL_CACHE[m] = radial_lambda(m)
        out = max(out, _RADIAL_CACHE[m])
    return out


def stability_measure(nu, N, M, dz, dr):
    """(nu/2)^2 (max dz^2[k]_B[k]_E + Lambda_M (dz/dr)^2) with a refit at nu; and min product."""
    CE, CB = fit(N, nu)
    pmax, pmin = zmax_product(CE, CB)
    return 0.25 * nu * nu * (pmax + radial_lambda_max(M) * (dz / dr) ** 2), pmin


def courant_limit(N, M, dz, dr, iters: int = 60):
    """Largest c dt / dz that is stable, refitting the coefficients at each trial."""
    lo, hi = 0.0, 1.0
    for _ in range(iters):
        mid = 0.5 * (lo + hi)
        s, pmin = stability_measure(mid, N, M, dz, dr)
        if s <= 1.0 and pmin >= 0.0:
            lo = mid
        else:
            hi = mid
    return lo


def solver_setup(N, M, dz, dr, cfl_fraction=0.95):
    """(dt, CE, CB, nu_limit): dt = fraction * limit, coefficients refit at dt."""
    nu_lim = courant_limit(N, M, dz, dr)
    nu = cfl_fraction * nu_lim
    CE, CB = fit(N, nu)
    return nu * dz, CE, CB, nu_lim
