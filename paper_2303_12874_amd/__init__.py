"""Python binding of libpic.so, the MI355X quasi-3D r-z PIC step with the dual solver.

Argument marshalling only: every computation runs in the C ABI declared in
include/pic.h (host set-up in C++, the step in HIP kernels for gfx950).
PyTorch provides the device workspace and the stream.  If the built library
is missing, importing this package raises: there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass, field
from typing import List, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpic.so")

PIC_OK, PIC_E_INVALID, PIC_E_CFL, PIC_E_NOMEM, PIC_E_STATE, PIC_E_DEVICE, PIC_E_NUMERIC = 0, -1, -2, -3, -4, -5, -6
PREC_FP64, PREC_FP32 = 64, 32
SOLVER_DUAL, SOLVER_YEE = 0, 1
CURRENT_FILTER, CURRENT_EXACT_JZ = 0, 1  # P on J_r, J_phi; or P^{-1} on J_z
MAX_JZ_TAPS = 128
(ER, EPHI, EZ, BR, BPHI, BZ, JR, JPHI, JZ, RHO, BR_OLD, BPHI_OLD, BZ_OLD, BR_NEW, BPHI_NEW,
 BZ_NEW) = range(16)
MAX_PULSES = 2


class PicError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"pic error {code}: {msg}")
        self.code = code


class _Pulse(C.Structure):
    _fields_ = [("a0", C.c_double), ("w0", C.c_double), ("tau", C.c_double), ("zc", C.c_double)]


class _RunDesc(C.Structure):
    _fields_ = [
        ("Nz", C.c_int32), ("Nr", C.c_int32), ("M", C.c_int32), ("ppc", C.c_int32),
        ("dz", C.c_double), ("dr", C.c_double), ("n0", C.c_double),
        ("ramp_start", C.c_double), ("ramp_len", C.c_double),
        ("down_start", C.c_double), ("down_len", C.c_double),
        ("n_pulses", C.c_int32), ("pulse", _Pulse * MAX_PULSES), ("taper", C.c_double),
        ("seed", C.c_uint64), ("n_tracked", C.c_int32), ("n_steps", C.c_int64),
    ]


class _Opts(C.Structure):
    _fields_ = [
        ("precision", C.c_int32), ("solver", C.c_int32), ("n_coef", C.c_int32),
        ("fit_band", C.c_double), ("cfl_fraction", C.c_double), ("dt", C.c_double),
        ("coef_E", C.POINTER(C.c_double)), ("coef_B", C.POINTER(C.c_double)),
        ("sort_interval", C.c_int32), ("tile_z", C.c_int32), ("tile_r", C.c_int32),
        ("use_graph", C.c_int32), ("current", C.c_int32),
        ("run_dt", C.POINTER(C.c_double)), ("run_coef_E", C.POINTER(C.c_double)),
        ("run_coef_B", C.POINTER(C.c_double)), ("deterministic", C.c_int32),
        ("window_interval", C.c_int32), ("window_guard", C.c_int32), ("window_speed", C.c_double),
        ("shape", C.c_int32),
    ]


class _RunInfo(C.Structure):
    _fields_ = [("dt", C.c_double), ("courant_limit", C.c_double), ("n_particles", C.c_int64),
                ("steps_done", C.c_int64), ("n_coef", C.c_int32), ("n_tracked", C.c_int32),
                ("tile_z", C.c_int32), ("tile_r", C.c_int32), ("window_cells", C.c_int64)]


MAX_TUNE = 16


class _DlaModel(C.Structure):
    _fields_ = [("a0", C.c_double), ("kz", C.c_double), ("vphi", C.c_double), ("cB", C.c_double),
                ("wake", C.c_double)]


class _TuneReport(C.Structure):
    _fields_ = [("n", C.c_int32), ("tile_z", C.c_int32 * MAX_TUNE), ("tile_r", C.c_int32 * MAX_TUNE),
                ("interval", C.c_int32 * MAX_TUNE), ("ms_per_step", C.c_double * MAX_TUNE), ("best", C.c_int32)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run python -m paper_2303_12874_amd.build")
    # The device memory and streams the library is handed come from torch, so
    # it must bind to the HIP runtime torch loads: load torch first, or the
    # dynamic linker picks the system runtime and the process holds two.
    import torch  # noqa: F401
    lib = C.CDLL(LIB_PATH)
    i32, i64, d, p, sz = C.c_int32, C.c_int64, C.c_double, C.c_void_p, C.c_size_t
    dp = C.POINTER(C.c_double)
    sigs = {
        "pic_solver_setup": [i32, i32, i32, d, d, d, d, dp, dp, dp, dp],
        "pic_courant_limit": [i32, dp, dp, i32, d, d, dp],
        "pic_jz_inverse_taps": [i32, dp, i32, dp, C.POINTER(C.c_int32)],
        "pic_load_host": [C.POINTER(_RunDesc), p, p, p, p, p, p, C.POINTER(C.c_int64)],
        "pic_init": [C.POINTER(_RunDesc), i32, C.POINTER(_Opts), p, C.POINTER(C.c_size_t), p, C.POINTER(p)],
        "pic_step": [p, i64],
        "pic_mode_work": [p, i32, p, p, p, p, p, p],
        "pic_cartesian_work": [p, i32, p, p, p, p, p],
        "pic_divergence": [p, i32, C.c_double, p],
        "pic_checkpoint": [p, p, C.POINTER(C.c_size_t)],
        "pic_restore": [p, p, sz],
        "pic_dla_integrate": [C.POINTER(_DlaModel), C.c_int64, p, p, p, p, p, C.c_double, C.c_double, p],
        "pic_fields": [p, i32, i32, i32, p, sz],
        "pic_particles": [p, i32, p, p, p, p, p, p, p, p, sz],
        "pic_coefficients": [p, i32, p, p, p],
        "pic_run_info_get": [p, i32, C.POINTER(_RunInfo)],
        "pic_destroy": [p],
        "pic_profile": [p, i32],
        "pic_profile_read": [p, p, p],
        "pic_autotune": [C.POINTER(_RunDesc), i32, C.POINTER(_Opts), p, C.POINTER(C.c_size_t), p, i32,
                         C.POINTER(_TuneReport)],
        "pic_divergence_arrays": [i32, i64, p, p, p, p, d, p, p],
    }
    for name, args in sigs.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = C.c_int
    lib.pic_last_error.argtypes = []
    lib.pic_last_error.restype = C.c_char_p
    return lib


_lib = _load()
EXPORTED = ("pic_solver_setup", "pic_courant_limit", "pic_jz_inverse_taps", "pic_load_host", "pic_init", "pic_step",
            "pic_mode_work", "pic_cartesian_work", "pic_divergence", "pic_dla_integrate", "pic_checkpoint",
            "pic_restore", "pic_fields", "pic_particles", "pic_coefficients", "pic_run_info_get", "pic_destroy",
            "pic_last_error", "pic_profile", "pic_profile_read", "pic_autotune", "pic_divergence_arrays")
PHASES = ("sort", "push", "efield", "bfield", "step")  # "step": a whole step replayed from a graph


def _check(rc):
    if rc != PIC_OK:
        raise PicError(rc, _lib.pic_last_error().decode())


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


@dataclass
class Pulse:
    a0: float
    w0: float
    tau: float
    zc: float


@dataclass
class RunDesc:
    """One run (grid, plasma, laser); lengths in c/omega_0."""
    Nz: int
    Nr: int
    M: int
    ppc: int
    dz: float
    dr: float
    n0: float = 0.0
    ramp_start: float = 0.0
    ramp_len: float = 0.0
    down_start: float = 0.0
    down_len: float = 0.0
    pulses: List[Pulse] = field(default_factory=list)
    taper: float = 0.0
    seed: int = 0
    n_tracked: int = 0
    n_steps: int = 0  # steps the run takes in total (0: no limit)

    def to_c(self) -> _RunDesc:
        r = _RunDesc()
        r.Nz, r.Nr, r.M, r.ppc = self.Nz, self.Nr, self.M, self.ppc
        r.dz, r.dr, r.n0, r.ramp_start, r.ramp_len = self.dz, self.dr, self.n0, self.ramp_start, self.ramp_len
        r.down_start, r.down_len = self.down_start, self.down_len
        if len(self.pulses) > MAX_PULSES:
            raise ValueError("at most %d pulses" % MAX_PULSES)
        r.n_pulses = len(self.pulses)
        for k, pl in enumerate(self.pulses):
            r.pulse[k] = _Pulse(pl.a0, pl.w0, pl.tau, pl.zc)
        r.taper = self.taper
        r.seed = self.seed & (2**64 - 1)
        r.n_tracked = self.n_tracked
        r.n_steps = self.n_steps
        return r


def solver_setup(M, dz, dr, solver=SOLVER_DUAL, n_coef=16, cfl_fraction=0.95, fit_band=0.0):
    """(dt, courant_limit, coef_E, coef_B) from the library's host set-up."""
    N = 1 if solver == SOLVER_YEE else n_coef
    dt, lim = C.c_double(), C.c_double()
    ce, cb = np.zeros(N), np.zeros(N)
    dp = C.POINTER(C.c_double)
    _check(_lib.pic_solver_setup(solver, n_coef, M, dz, dr, cfl_fraction, fit_band, C.byref(dt), C.byref(lim),
                                 ce.ctypes.data_as(dp), cb.ctypes.data_as(dp)))
    return dt.value, lim.value, ce, cb


def courant_limit(coef_E, coef_B, M, dz, dr):
    ce = np.ascontiguousarray(coef_E, dtype=np.float64)
    cb = np.ascontiguousarray(coef_B, dtype=np.float64)
    out = C.c_double()
    dp = C.POINTER(C.c_double)
    _check(_lib.pic_courant_limit(ce.size, ce.ctypes.data_as(dp), cb.ctypes.data_as(dp), M, dz, dr, C.byref(out)))
    return out.value


def jz_inverse_taps(coef_B, precision=PREC_FP64):
    """Taps h_0..h_{n-1} of the stencil the library uses for P^{-1} with the
    exact J_z correction (pic_jz_inverse_taps)."""
    cb = np.ascontiguousarray(coef_B, dtype=np.float64)
    h = np.zeros(MAX_JZ_TAPS)
    n = C.c_int32()
    dp = C.POINTER(C.c_double)
    _check(_lib.pic_jz_inverse_taps(cb.size, cb.ctypes.data_as(dp), precision, h.ctypes.data_as(dp), C.byref(n)))
    return h[:n.value].copy()


def load_host(run: RunDesc):
    """Electrons the library loads for `run` (host, FP64, cell units)."""
    rd = run.to_c()
    n = C.c_int64()
    _check(_lib.pic_load_host(C.byref(rd), None, None, None, None, None, None, C.byref(n)))
    z, x, y, w = (np.zeros(n.value) for _ in range(4))
    ids = np.zeros(n.value, dtype=np.int64)
    tr = np.zeros(max(run.n_tracked, 1), dtype=np.int64)
    _check(_lib.pic_load_host(C.byref(rd), _ptr(z), _ptr(x), _ptr(y), _ptr(w), _ptr(ids), _ptr(tr), C.byref(n)))
    return {"z": z, "x": x, "y": y, "w": w, "id": ids, "tracked": tr[: run.n_tracked]}


def workspace_bytes(runs: Sequence[RunDesc], precision=PREC_FP64, solver=SOLVER_DUAL, n_coef=16, **kw) -> int:
    arr = (_RunDesc * len(runs))(*[r.to_c() for r in runs])
    o = _make_opts(precision, solver, n_coef, **kw)[0]
    nbytes = C.c_size_t(0)
    _check(_lib.pic_init(arr, len(runs), C.byref(o), None, C.byref(nbytes), None, None))
    return nbytes.value


def _make_opts(precision, solver, n_coef, dt=0.0, coef_E=None, coef_B=None, cfl_fraction=0.0, fit_band=0.0,
               sort_interval=0, tile_z=0, tile_r=0, use_graph=False, current=CURRENT_FILTER, run_dt=None,
               run_coef_E=None, run_coef_B=None, deterministic=False, window_interval=0, window_guard=0,
               window_speed=0.0, shape=1):
    """pic_opts.  run_dt: one dt per run; run_coef_E / run_coef_B: one
    coefficient vector per run (sequences over the runs); window_*: the
    moving window (0: static box); shape: particle shape order (1 linear,
    2 quadratic)."""
    o = _Opts()
    o.precision, o.solver, o.n_coef = precision, solver, n_coef
    o.fit_band, o.cfl_fraction, o.dt = fit_band, cfl_fraction, dt
    keep = []
    for name, val in (("coef_E", coef_E), ("coef_B", coef_B), ("run_dt", run_dt), ("run_coef_E", run_coef_E),
                      ("run_coef_B", run_coef_B)):
        if val is not None:
            a = np.ascontiguousarray(np.concatenate([np.ravel(v) for v in val]) if name.startswith("run_coef")
                                     else val, dtype=np.float64)
            keep.append(a)
            setattr(o, name, a.ctypes.data_as(C.POINTER(C.c_double)))
    o.sort_interval, o.tile_z, o.tile_r, o.use_graph = sort_interval, tile_z, tile_r, int(use_graph)
    o.current = current
    o.deterministic = int(bool(deterministic))
    o.window_interval, o.window_guard, o.window_speed = int(window_interval), int(window_guard), float(window_speed)
    o.shape = int(shape)
    return o, keep


def dla_integrate(t0, x, zeta, xd, zetad, t_end: float, h: float, a0=2.8, kz=12.14, vphi=1.002565, cB=1.0,
                  wake=1.0):
    """Integrate electrons of the reduced model (Sec. II, Eq. (8)) in place with
    pic_dla_integrate, units c = omega_p = 1.  t0, x, zeta, xd, zetad: FP64
    contiguous device tensors (torch) of one length; asynchronous on torch's
    current stream of their device."""
    import torch  # device memory and streams only

    arrs = (t0, x, zeta, xd, zetad)
    n = t0.numel()
    for a in arrs:
        if not (isinstance(a, torch.Tensor) and a.is_cuda and a.dtype == torch.float64 and a.is_contiguous()
                and a.numel() == n and a.device == t0.device):
            raise ValueError("dla_integrate takes contiguous float64 device tensors of one length on one device")
    m = _DlaModel(a0, kz, vphi, cB, wake)
    stream = torch.cuda.current_stream(t0.device)
    _check(_lib.pic_dla_integrate(C.byref(m), n, *[C.c_void_p(a.data_ptr()) for a in arrs], float(t_end), float(h),
                                  C.c_void_p(stream.cuda_stream)))


def divergence_arrays(ux, uy, uz, w, gamma_min=1.0):
    """pic_divergence_arrays: the divergence sums of pic_divergence over
    electrons in caller device arrays (contiguous torch tensors of one length
    and dtype, float64 or float32, on one device), with no allocation (the
    library's fixed per-GPU scratch).  Synchronises torch's current stream of
    that device.  {"w", "rms_x", "rms_y", "count", "sum_wtx2", "sum_wty2"}."""
    import torch  # device memory and streams only

    arrs = (ux, uy, uz, w)
    n = ux.numel()
    dt = ux.dtype
    for a in arrs:
        if not (isinstance(a, torch.Tensor) and a.is_cuda and a.dtype == dt and a.is_contiguous()
                and a.numel() == n and a.device == ux.device and dt in (torch.float64, torch.float32)):
            raise ValueError("divergence_arrays takes contiguous float64 or float32 device tensors of one length")
    out = np.zeros(6)
    stream = torch.cuda.current_stream(ux.device)
    _check(_lib.pic_divergence_arrays(PREC_FP64 if dt == torch.float64 else PREC_FP32, n,
                                      *[C.c_void_p(a.data_ptr()) for a in arrs], float(gamma_min), _ptr(out),
                                      C.c_void_p(stream.cuda_stream)))
    return {"w": out[0], "rms_x": float(out[4]), "rms_y": float(out[5]), "count": int(out[3]), "sum_wtx2": out[1],
            "sum_wty2": out[2]}


def autotune(runs: Sequence[RunDesc], precision=PREC_FP64, solver=SOLVER_DUAL, n_coef=16, device="cuda:0",
             trial_steps=16, **kw) -> dict:
    """Sort tile and sort interval picked by pic_autotune for these runs and
    options: {"tile_z", "tile_r", "sort_interval", "candidates": [(tile_z,
    tile_r, interval, ms_per_step), ...]}.  Pass the first three to
    Simulation.  Trial contexts live in a temporary torch workspace."""
    import torch  # device memory and streams only

    arr = (_RunDesc * len(runs))(*[r.to_c() for r in runs])
    opts, keep = _make_opts(precision, solver, n_coef, **kw)
    nbytes = C.c_size_t(0)
    _check(_lib.pic_autotune(arr, len(runs), C.byref(opts), None, C.byref(nbytes), None, int(trial_steps), None))
    ws = torch.empty(nbytes.value, dtype=torch.uint8, device=torch.device(device))
    stream = torch.cuda.current_stream(torch.device(device))
    rep = _TuneReport()
    _check(_lib.pic_autotune(arr, len(runs), C.byref(opts), C.c_void_p(ws.data_ptr()), C.byref(nbytes),
                             C.c_void_p(stream.cuda_stream), int(trial_steps), C.byref(rep)))
    del ws, keep
    cands = [(rep.tile_z[i], rep.tile_r[i], rep.interval[i], rep.ms_per_step[i]) for i in range(rep.n)]
    return {"tile_z": opts.tile_z, "tile_r": opts.tile_r, "sort_interval": opts.sort_interval, "candidates": cands}


class Simulation:
    """Runs on one GPU.  `device` is a torch device string; the workspace is a
    torch uint8 tensor and the stream torch's current stream on that device."""

    def __init__(self, runs: Sequence[RunDesc], precision=PREC_FP64, solver=SOLVER_DUAL, n_coef=16,
                 device="cuda:0", **kw):
        import torch  # device memory and streams only

        self.runs = list(runs)
        self.precision = precision
        self._arr = (_RunDesc * len(self.runs))(*[r.to_c() for r in self.runs])
        self._opts, self._keep = _make_opts(precision, solver, n_coef, **kw)
        nbytes = C.c_size_t(0)
        _check(_lib.pic_init(self._arr, len(self.runs), C.byref(self._opts), None, C.byref(nbytes), None, None))
        self.device = torch.device(device)
        self.workspace = torch.empty(nbytes.value, dtype=torch.uint8, device=self.device)
        self.stream = torch.cuda.current_stream(self.device)
        h = C.c_void_p()
        _check(_lib.pic_init(self._arr, len(self.runs), C.byref(self._opts), C.c_void_p(self.workspace.data_ptr()),
                             C.byref(nbytes), C.c_void_p(self.stream.cuda_stream), C.byref(h)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            _check(_lib.pic_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self, n=1):
        _check(_lib.pic_step(self._h, int(n)))

    def profile(self, enable=True):
        """Start (restart) or stop per-phase HIP-event timing of pic_step."""
        _check(_lib.pic_profile(self._h, int(enable)))

    def profile_read(self):
        """{phase: (total ms, launches)} since profiling was enabled."""
        ms = np.zeros(len(PHASES))
        n = np.zeros(len(PHASES), dtype=np.int64)
        _check(_lib.pic_profile_read(self._h, _ptr(ms), _ptr(n)))
        return {ph: (float(ms[i]), int(n[i])) for i, ph in enumerate(PHASES)}

    def info(self, run=0):
        inf = _RunInfo()
        _check(_lib.pic_run_info_get(self._h, run, C.byref(inf)))
        return {"dt": inf.dt, "courant_limit": inf.courant_limit, "n_particles": inf.n_particles,
                "steps_done": inf.steps_done, "n_coef": inf.n_coef, "n_tracked": inf.n_tracked,
                "tile": (inf.tile_z, inf.tile_r), "window_cells": inf.window_cells}

    def coefficients(self, run=0):
        N = self.info(run)["n_coef"]
        ce, cb, p = np.zeros(N), np.zeros(N), np.zeros(2 * N - 1)
        _check(_lib.pic_coefficients(self._h, run, _ptr(ce), _ptr(cb), _ptr(p)))
        return ce, cb, p

    def fields(self, comp, m, run=0):
        r = self.runs[run]
        out = np.zeros((r.Nr + 1, r.Nz), dtype=np.complex128)
        _check(_lib.pic_fields(self._h, run, comp, m, _ptr(out), out.size * 2))
        return out

    def particles(self, run=0):
        n = self.info(run)["n_particles"]
        d = {k: np.zeros(n) for k in ("z", "x", "y", "ux", "uy", "uz", "w")}
        ids = np.zeros(n, dtype=np.int64)
        _check(_lib.pic_particles(self._h, run, *[_ptr(d[k]) for k in ("z", "x", "y", "ux", "uy", "uz", "w")],
                                  _ptr(ids), n))
        d["id"] = ids
        return d

    def mode_work(self, run=0):
        r = self.runs[run]
        nt = r.n_tracked
        W = np.zeros((max(nt, 1), r.M + 1))
        g, ga = np.zeros(max(nt, 1)), np.zeros(max(nt, 1))
        ids = np.zeros(max(nt, 1), dtype=np.int64)
        U = np.zeros(r.M + 1)
        K = np.zeros(1)
        _check(_lib.pic_mode_work(self._h, run, _ptr(W), _ptr(g), _ptr(ga), _ptr(ids), _ptr(U), _ptr(K)))
        return {"W": W[:nt], "gamma": g[:nt], "gamma_acc": ga[:nt], "id": ids[:nt], "field_energy": U,
                "kinetic": K[0]}

    def checkpoint(self) -> bytes:
        """The whole state of the context as bytes (pic_checkpoint)."""
        n = C.c_size_t(0)
        _check(_lib.pic_checkpoint(self._h, None, C.byref(n)))
        buf = (C.c_ubyte * n.value)()
        _check(_lib.pic_checkpoint(self._h, buf, C.byref(n)))
        return bytes(buf)

    def restore(self, blob: bytes):
        """Continue from a checkpoint of a context with the same runs and options."""
        buf = (C.c_ubyte * len(blob)).from_buffer_copy(blob)
        _check(_lib.pic_restore(self._h, buf, len(blob)))

    def divergence(self, gamma_min=1.0, run=0):
        """Charge-weighted RMS divergence theta_x = atan(u_x/u_z) (and theta_y)
        of the electrons with gamma >= gamma_min moving forward, with the raw
        sums: {"w", "rms_x", "rms_y", "count"}."""
        out = np.zeros(6)
        _check(_lib.pic_divergence(self._h, run, float(gamma_min), _ptr(out)))
        return {"w": out[0], "rms_x": float(out[4]), "rms_y": float(out[5]), "count": int(out[3]),
                "sum_wtx2": out[1], "sum_wty2": out[2]}

    def cartesian_work(self, run=0, corrected=True):
        """Work on the tracked electrons by field direction (Eq. (17)); with
        corrected=True also the Pukhov ratio f (Eq. (20)) and the corrected
        W*_LWFA, W*_DLA (Eq. (21)) -- the run needs a pulse for those."""
        nt = self.runs[run].n_tracked
        out = {k: np.zeros(max(nt, 1)) for k in ("Wz", "Wperp", "f", "W_lwfa", "W_dla")}
        keys = ("Wz", "Wperp", "f", "W_lwfa", "W_dla") if corrected else ("Wz", "Wperp")
        _check(_lib.pic_cartesian_work(self._h, run, *[_ptr(out[k]) if k in keys else None
                                                       for k in ("Wz", "Wperp", "f", "W_lwfa", "W_dla")]))
        return {k: out[k][:nt] for k in keys}
