"""FP64 CPU oracle of the quasi-3D r-z PIC step with the dual Maxwell solver.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
baseline of the benchmark import this package.  It shares no code with the HIP
library (``paper_2303_12874_amd``) and neither imports the other.

``q3d_oracle.c`` holds the step (gather, Boris push, charge-conserving deposit,
z filter, dual-solver field update, diagnostics), compiled with gcc into
``liborc.so``; ``coef.py`` holds the coefficient fit and Courant limit (numpy).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "q3d_oracle.c")
_LIB = os.path.join(_HERE, "liborc.so")

GCC_FLAGS = ["-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off", "-fcx-fortran-rules",
             "-fno-builtin-sin", "-fno-builtin-cos", "-fno-builtin-sincos"]


def build(force: bool = False) -> str:
    """Compile liborc.so with gcc (no FMA contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", *GCC_FLAGS, "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = C.CDLL(build())
        d, i, l, p, u64 = C.c_double, C.c_int, C.c_long, C.c_void_p, C.c_uint64
        dp = C.POINTER(C.c_double)
        sig = {
            "orc_create": (p, [i, i, i, d, d, d, i, dp, dp]),
            "orc_destroy": (None, [p]),
            "orc_set_flags": (None, [p, i, i]),
            "orc_num_particles": (l, [p]),
            "orc_num_steps": (l, [p]),
            "orc_get_field": (i, [p, i, i, p]),
            "orc_set_field": (i, [p, i, i, p]),
            "orc_gauss_residual": (i, [p, i, p]),
            "orc_field_energy": (d, [p, i]),
            "orc_gather": (None, [p, d, d, d, p]),
            "orc_boris": (None, [p, p, p, d]),
            "orc_deposit_rho": (None, [p]),
            "orc_deposit_one": (None, [p, d, d, d, d, d, d, d, d]),
            "orc_deposit_add": (None, [p, d, d, d, d, d, d, d, d]),
            "orc_step": (None, [p, i]),
            "orc_field_step": (None, [p, i]),
            "orc_start_fields": (None, [p]),
            "orc_splitmix64": (u64, [u64, u64]),
            "orc_load_plasma": (i, [p, i, d, d, d, u64, i, d, d]),
            "orc_set_particles": (i, [p, l, p, p, p, p, p, p, p, i]),
            "orc_get_particles": (None, [p, p, p, p, p, p, p, p, p]),
            "orc_put_particles": (None, [p, p, p, p, p, p, p, p]),
            "orc_tracked": (i, [p, p, p, p, p]),
            "orc_cartesian_work": (i, [p, p, p]),
            "orc_kinetic": (d, [p]),
            "orc_add_laser": (i, [p, d, d, d, d, d]),
            "orc_round_to_fp32": (None, [p]),
            "orc_cell_order": (None, [p, i, i, p]),
            "orc_filter_taps": (dp, [p]),
            "orc_set_exact_jz": (None, [p, i]),
            "orc_inverse_filter": (i, [p, p, p]),
            "orc_set_window": (None, [p, i, d, i]),
            "orc_set_shape": (i, [p, i]),
            "orc_window_cells": (l, [p]),
        }
        for name, (res, args) in sig.items():
            f = getattr(_lib, name)
            f.restype = res
            f.argtypes = args
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


# field component numbers
ER, EP, EZ, BOR, BOP, BOZ, BR, BP, BZ, JR, JP, JZ, RHO = range(13)


class Oracle:
    """One run of the oracle.  Particle positions are in cell units."""

    def __init__(self, Nz, Nr, M, dz, dr, dt, CE, CB):
        L = lib()
        self.Nz, self.Nr, self.M = int(Nz), int(Nr), int(M)
        self.dz, self.dr, self.dt = float(dz), float(dr), float(dt)
        self.CE = np.ascontiguousarray(CE, dtype=np.float64)
        self.CB = np.ascontiguousarray(CB, dtype=np.float64)
        dp = C.POINTER(C.c_double)
        self._h = L.orc_create(self.Nz, self.Nr, self.M, self.dz, self.dr, self.dt, self.CE.size,
                               self.CE.ctypes.data_as(dp), self.CB.ctypes.data_as(dp))
        if not self._h:
            raise ValueError("invalid oracle grid")

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().orc_destroy(h)
            self._h = None

    # --- fields ---------------------------------------------------------
    def get_field(self, comp, m):
        out = np.zeros((self.Nr + 1, self.Nz), dtype=np.complex128)
        if lib().orc_get_field(self._h, comp, m, _ptr(out)) != 0:
            raise ValueError("bad component/mode")
        return out

    def set_field(self, comp, m, arr):
        a = np.ascontiguousarray(np.broadcast_to(arr, (self.Nr + 1, self.Nz)), dtype=np.complex128)
        if lib().orc_set_field(self._h, comp, m, _ptr(a)) != 0:
            raise ValueError("bad component/mode")

    def gauss_residual(self, m):
        out = np.zeros((self.Nr + 1, self.Nz), dtype=np.complex128)
        lib().orc_gauss_residual(self._h, m, _ptr(out))
        return out

    def field_energy(self, m):
        return lib().orc_field_energy(self._h, m)

    def gather(self, z, x, y):
        out = np.zeros(6)
        lib().orc_gather(self._h, z, x, y, _ptr(out))
        return out

    # --- stepping -------------------------------------------------------
    def set_flags(self, freeze_fields=False, deposit_rho=False):
        lib().orc_set_flags(self._h, int(freeze_fields), int(deposit_rho))

    def step(self, n=1):
        lib().orc_step(self._h, int(n))

    def field_step(self, n=1):
        lib().orc_field_step(self._h, int(n))

    def start_fields(self):
        lib().orc_start_fields(self._h)

    def deposit_rho(self):
        lib().orc_deposit_rho(self._h)

    def deposit_one(self, q, p0, p1, vphi=0.0):
        lib().orc_deposit_one(self._h, q, *map(float, p0), *map(float, p1), float(vphi))

    def deposit_add(self, q, p0, p1, vphi=0.0):
        """Add one particle's move from p0 to p1 (z, x, y in cell units) to J."""
        lib().orc_deposit_add(self._h, q, *map(float, p0), *map(float, p1), float(vphi))

    # --- particles ------------------------------------------------------
    @property
    def np(self):
        return lib().orc_num_particles(self._h)

    def load_plasma(self, ppc, n0, ramp_start=0.0, ramp_len=0.0, seed=0, n_tracked=0, down_start=0.0,
                    down_len=0.0):
        r = lib().orc_load_plasma(self._h, int(ppc), float(n0), float(ramp_start), float(ramp_len),
                                  int(seed) & (2**64 - 1), int(n_tracked), float(down_start), float(down_len))
        if r != 0:
            raise ValueError("bad plasma load")

    def set_particles(self, z, x, y, ux, uy, uz, w, track_all=True):
        arrs = [np.ascontiguousarray(a, dtype=np.float64) for a in (z, x, y, ux, uy, uz, w)]
        lib().orc_set_particles(self._h, arrs[0].size, *[_ptr(a) for a in arrs], int(track_all))

    def set_shape(self, order):
        """Particle shape order of the gather and the deposit: 1 linear (the
        default), 2 quadratic."""
        if lib().orc_set_shape(self._h, int(order)) != 0:
            raise ValueError("shape order must be 1 or 2")

    def set_window(self, interval, speed=1.0, guard=0):
        """Moving window (App. A): before a step whose count of steps taken is
        a positive multiple of `interval`, the box advances by the whole cells
        a front moving at `speed` c has crossed since the start; `guard`
        columns at the back are cleared at each move.  interval 0: off."""
        lib().orc_set_window(self._h, int(interval), float(speed), int(guard))

    @property
    def window_cells(self):
        """Cells the window has moved: box column i is absolute column i + this."""
        return int(lib().orc_window_cells(self._h))

    def particles(self):
        n = self.np
        out = {k: np.zeros(n) for k in ("z", "x", "y", "ux", "uy", "uz", "w")}
        ids = np.zeros(n, dtype=np.int64)
        lib().orc_get_particles(self._h, *[_ptr(out[k]) for k in ("z", "x", "y", "ux", "uy", "uz", "w")],
                                _ptr(ids))
        out["id"] = ids
        return out

    def put_particles(self, d):
        arrs = [np.ascontiguousarray(d[k], dtype=np.float64) for k in ("z", "x", "y", "ux", "uy", "uz", "w")]
        lib().orc_put_particles(self._h, *[_ptr(a) for a in arrs])

    def tracked(self):
        n = lib().orc_tracked(self._h, None, None, None, None)
        ids = np.zeros(n, dtype=np.int64)
        W = np.zeros((n, self.M + 1))
        g = np.zeros(n)
        ga = np.zeros(n)
        lib().orc_tracked(self._h, _ptr(ids), _ptr(W), _ptr(g), _ptr(ga))
        return {"id": ids, "W": W, "gamma": g, "gamma_acc": ga}

    def cartesian_work(self):
        """W_z and W_perp of the tracked particles (Eq. (17)), slot order."""
        n = lib().orc_cartesian_work(self._h, None, None)
        wz, wp = np.zeros(n), np.zeros(n)
        lib().orc_cartesian_work(self._h, _ptr(wz), _ptr(wp))
        return {"Wz": wz, "Wperp": wp}

    def kinetic(self):
        return lib().orc_kinetic(self._h)

    def add_laser(self, a0, w0, tau, zc, taper=0.0):
        if lib().orc_add_laser(self._h, a0, w0, tau, zc, taper) != 0:
            raise ValueError("laser needs M >= 1")

    def filter_taps(self):
        """Taps p_l, l = -(N-1)..N-1, of the z filter the oracle applies to J_r, J_phi."""
        ptr = lib().orc_filter_taps(self._h)
        return np.array([ptr[k] for k in range(2 * self.CB.size - 1)])

    def set_exact_jz(self, on=True):
        """Charge conservation by J_z <- P^{-1} J_z with J_r, J_phi unfiltered
        (Gauss's law then holds with rho itself) instead of filtering J_r, J_phi."""
        lib().orc_set_exact_jz(self._h, int(on))

    def inverse_filter(self, line):
        """P^{-1} of one periodic complex z line of Nz values (DFT)."""
        a = np.ascontiguousarray(line, dtype=np.complex128)
        if a.shape != (self.Nz,):
            raise ValueError("line of Nz values expected")
        out = np.zeros_like(a)
        if lib().orc_inverse_filter(self._h, _ptr(a), _ptr(out)) != 0:
            raise ValueError("P has a non-positive symbol on this grid")
        return out

    def round_to_fp32(self):
        lib().orc_round_to_fp32(self._h)

    def cell_order(self, Tz, Tr):
        out = np.zeros(self.np, dtype=np.int64)
        lib().orc_cell_order(self._h, int(Tz), int(Tr), _ptr(out))
        return out


def splitmix64(seed: int, k: int) -> int:
    """k-th output of the SplitMix64 stream seeded with `seed` (oracle's C)."""
    return int(lib().orc_splitmix64(seed & (2**64 - 1), k & (2**64 - 1)))
