"""CPU tests of the C ABI: the library loads and exports every declared
symbol, argument validation fails cleanly before any device call, and the
host-side set-up (coefficient fit, Courant limit, loading) agrees with the
oracle -- bit-exactly for the loading."""
import ctypes
import math
import os
import re

import numpy as np
import pytest

import oracle
import paper_2303_12874_amd as pic
import workloads
from oracle import coef

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_library_exports_every_declared_symbol():
    header = open(os.path.join(ROOT, "include", "pic.h")).read()
    declared = set(re.findall(r"^(?:int|const char \*)\s*\*?(pic_\w+)\s*\(", header, flags=re.M))
    assert declared == set(pic.EXPORTED)
    lib = ctypes.CDLL(pic.LIB_PATH)
    for name in declared:
        assert hasattr(lib, name), name


def _desc(**kw):
    base = dict(workloads.small()["runs"][0])
    base.update(kw)
    return workloads.to_rundesc(base)


@pytest.mark.parametrize("field,value", [("Nz", 4), ("Nr", 2), ("M", 4), ("dz", 0.0), ("dr", -1.0),
                                         ("n_tracked", 10**9), ("ppc", -1)])
def test_invalid_descriptor_is_rejected_without_device(field, value):
    d = _desc()
    setattr(d, field, value)
    with pytest.raises(pic.PicError) as e:
        pic.workspace_bytes([d])
    assert e.value.code == pic.PIC_E_INVALID


def test_plane_beyond_32_bit_offsets_is_rejected():
    """The largest plane the kernels address with 32-bit offsets is accepted
    (size query only), one node more is not."""
    Nz = 65536
    ok = _desc(Nz=Nz, Nr=(2**31 - 1) // Nz - 1, ppc=0, n_tracked=0)
    assert pic.workspace_bytes([ok]) > 0
    bad = _desc(Nz=Nz, Nr=(2**31 - 1) // Nz, ppc=0, n_tracked=0)
    assert (bad.Nr + 1) * bad.Nz > 2**31 - 1
    with pytest.raises(pic.PicError) as e:
        pic.workspace_bytes([bad])
    assert e.value.code == pic.PIC_E_INVALID


def test_bad_options_rejected():
    d = _desc()
    for kw in (dict(precision=16), dict(solver=7), dict(n_coef=0), dict(n_coef=99)):
        args = dict(precision=pic.PREC_FP64, solver=pic.SOLVER_DUAL, n_coef=16)
        args.update(kw)
        with pytest.raises(pic.PicError) as e:
            pic.workspace_bytes([d], **args)
        assert e.value.code == pic.PIC_E_INVALID
    with pytest.raises(pic.PicError):
        pic.workspace_bytes([d], coef_E=[1.0], coef_B=None)


def test_per_run_options_are_checked():
    """run_dt must be positive and finite for every run; run_coef_E and
    run_coef_B come together (checked before any device call)."""
    runs = [_desc(Nz=64), _desc(Nz=96)]
    assert pic.workspace_bytes(runs, run_dt=[0.2, 0.15]) > 0
    for bad in ([0.2, 0.0], [0.2, -1.0], [0.2, float("nan")]):
        with pytest.raises(pic.PicError) as e:
            pic.workspace_bytes(runs, run_dt=bad)
        assert e.value.code == pic.PIC_E_INVALID
    with pytest.raises(pic.PicError) as e:
        pic.workspace_bytes(runs, run_coef_E=[np.ones(16), np.ones(16)])
    assert e.value.code == pic.PIC_E_INVALID


def test_deterministic_mode_is_fp64_only():
    d = _desc()
    assert pic.workspace_bytes([d], deterministic=True) > pic.workspace_bytes([d])  # the integer sums of J
    with pytest.raises(pic.PicError) as e:
        pic.workspace_bytes([d], precision=pic.PREC_FP32, deterministic=True)
    assert e.value.code == pic.PIC_E_INVALID


def test_moving_window_options_are_checked():
    """The moving window sizes the particle arrays for four moves' worth of
    fresh columns and refuses bad values, captured graphs, the deterministic
    mode and a guard band as long as the box."""
    d = _desc()
    plain = pic.workspace_bytes([d])
    assert pic.workspace_bytes([d], window_interval=8) > plain
    assert pic.workspace_bytes([d], window_interval=8, window_speed=2.0) > pic.workspace_bytes([d], window_interval=8)
    for kw in (dict(window_interval=-1), dict(window_interval=4, window_guard=-2),
               dict(window_interval=4, window_speed=-1.0), dict(window_interval=4, use_graph=True),
               dict(window_interval=4, deterministic=True), dict(window_interval=4, window_guard=d.Nz)):
        with pytest.raises(pic.PicError) as e:
            pic.workspace_bytes([d], **kw)
        assert e.value.code == pic.PIC_E_INVALID, kw


def test_shape_order_option_is_checked():
    """Shape order 0 or 1 (linear) and 2 (quadratic) are taken, quadratic also
    with the deterministic mode; other values are refused."""
    d = _desc()
    for sh in (0, 1, 2):
        assert pic.workspace_bytes([d], shape=sh) > 0
    assert pic.workspace_bytes([d], shape=2, deterministic=True) > pic.workspace_bytes([d], shape=2)
    for kw in (dict(shape=3), dict(shape=-1)):
        with pytest.raises(pic.PicError) as e:
            pic.workspace_bytes([d], **kw)
        assert e.value.code == pic.PIC_E_INVALID, kw


def test_allocation_free_divergence_checks_its_arguments_first():
    """pic_divergence_arrays refuses bad arguments and counts beyond its fixed
    scratch (2048 x 256 x 64 electrons) before any device call."""
    out = np.zeros(6)
    dummy = ctypes.c_void_p(16)  # never dereferenced: the checks come first
    f = pic._lib.pic_divergence_arrays
    assert f(64, 2048 * 256 * 64 + 1, dummy, dummy, dummy, dummy, 1.0, pic._ptr(out), None) == pic.PIC_E_NOMEM
    assert "33554432" in pic._lib.pic_last_error().decode()
    assert f(16, 10, dummy, dummy, dummy, dummy, 1.0, pic._ptr(out), None) == pic.PIC_E_INVALID
    assert f(64, -1, dummy, dummy, dummy, dummy, 1.0, pic._ptr(out), None) == pic.PIC_E_INVALID
    assert f(64, 10, None, dummy, dummy, dummy, 1.0, pic._ptr(out), None) == pic.PIC_E_INVALID
    assert f(64, 10, dummy, dummy, dummy, dummy, 0.5, pic._ptr(out), None) == pic.PIC_E_INVALID
    out[:] = 7.0
    assert f(32, 0, None, None, None, None, 1.0, pic._ptr(out), None) == pic.PIC_OK  # nothing to reduce
    assert np.all(out == 0.0)


def test_runs_must_share_modes():
    with pytest.raises(pic.PicError) as e:
        pic.workspace_bytes([_desc(M=1), _desc(M=2)])
    assert e.value.code == pic.PIC_E_INVALID


def test_workspace_query_scales_with_problem():
    a = pic.workspace_bytes([_desc(Nz=64)])
    b = pic.workspace_bytes([_desc(Nz=128)])
    c = pic.workspace_bytes([_desc(Nz=64)], precision=pic.PREC_FP32)
    assert 1.8 < b / a < 2.2 and c < a
    assert a % 256 == 0


def test_null_and_destroyed_context():
    lib = pic._lib
    assert lib.pic_step(None, 1) == pic.PIC_E_STATE
    assert lib.pic_destroy(None) == pic.PIC_E_STATE
    bogus = ctypes.c_void_p(12345678)
    assert lib.pic_step(bogus, 1) == pic.PIC_E_STATE
    assert lib.pic_cartesian_work(None, 0, None, None, None, None, None) == pic.PIC_E_STATE
    n = ctypes.c_size_t(0)
    assert lib.pic_checkpoint(None, None, ctypes.byref(n)) == pic.PIC_E_STATE
    assert lib.pic_restore(None, None, 0) == pic.PIC_E_STATE
    assert lib.pic_mode_work(None, 0, None, None, None, None, None, None) == pic.PIC_E_STATE
    assert b"context" in lib.pic_last_error()


@pytest.mark.parametrize("M", [1, 2, 3])
def test_solver_setup_matches_oracle(M):
    dz = workloads.LAMBDA0 / 16
    dr = 4 * dz
    dt, lim, ce, cb = pic.solver_setup(M, dz, dr)
    dt_o, CE, CB, lim_o = coef.solver_setup(16, M, dz, dr)
    assert abs(lim / lim_o - 1) < 1e-8
    assert abs(dt / dt_o - 1) < 1e-8
    kap = np.linspace(1e-3, 2 * np.pi / 3, 2000)
    assert np.abs(coef.symbol(ce, kap) - coef.symbol(CE, kap)).max() < 1e-8
    assert np.abs(coef.symbol(cb, kap) - coef.symbol(CB, kap)).max() < 1e-8
    # limit of fixed coefficients: (dt/2)^2 (max [k]_B[k]_E + Lambda_M/dr^2) = 1
    pmax, _ = coef.zmax_product(CE, CB)
    nu_fixed = 2.0 / math.sqrt(pmax + coef.radial_lambda_max(M) * (dz / dr) ** 2)
    assert abs(pic.courant_limit(CE, CB, M, dz, dr) / nu_fixed - 1) < 1e-9


def test_yee_setup_is_textbook():
    dz = 0.3
    dr = 1.2
    dt, lim, ce, cb = pic.solver_setup(0, dz, dr, solver=pic.SOLVER_YEE)
    assert list(ce) == [1.0] and list(cb) == [1.0]
    lam0 = coef.radial_lambda(0)
    assert abs(lim - 1 / math.sqrt(1 + lam0 * (dz / dr) ** 2 / 4)) < 1e-9


@pytest.mark.parametrize("M", [0, 1, 2, 3])
def test_jz_inverse_taps_invert_the_filter(M):
    """The stencil of the exact J_z correction against the oracle's P^{-1} (a
    DFT on a periodic line, no cut) applied to a unit impulse, and against the
    forward filter by direct convolution; FP32 cuts it shorter."""
    dz = workloads.LAMBDA0 / 16
    _, _, _, cb = pic.solver_setup(M, dz, 4 * dz)
    h = pic.jz_inverse_taps(cb, pic.PREC_FP64)
    nh = h.size
    assert 1 < nh <= pic.MAX_JZ_TAPS
    Nz = 512
    o = oracle.Oracle(Nz, 4, 0, dz, 4 * dz, 0.5 * dz, cb, cb)
    delta = np.zeros(Nz, dtype=complex)
    delta[0] = 1.0
    ref = o.inverse_filter(delta).real  # periodic P^{-1}: ref[l] = h_l
    # both sides round: the oracle's 512-term DFT sums to a few units of 1e-15
    assert np.abs(ref[:nh] - h).max() < 1e-14 * abs(h[0])
    assert np.abs(ref[nh:Nz - nh + 1]).max() <= 2 * 2.0 ** -53 * abs(h[0])
    full = np.concatenate([h[:0:-1], h])  # h_{-(nh-1)} .. h_{nh-1}
    p = o.filter_taps()
    conv = np.convolve(full, p)
    centre = (conv.size - 1) // 2
    e = np.zeros(conv.size)
    e[centre] = 1.0
    assert np.abs(conv - e).max() < 1e-14
    h32 = pic.jz_inverse_taps(cb, pic.PREC_FP32)
    assert h32.size < nh and np.array_equal(h32, h[:h32.size])
    assert np.abs(ref[h32.size:Nz - h32.size + 1]).max() <= 2.0 ** -24 * abs(h[0])


def test_jz_inverse_taps_yee_and_refusal():
    assert list(pic.jz_inverse_taps([1.0])) == [1.0]
    # a 32-coefficient fit whose filter changes sign near k dz = 0.93 pi
    _, CB = coef.fit(32, 0.75)
    with pytest.raises(pic.PicError):
        pic.jz_inverse_taps(CB)
    with pytest.raises(pic.PicError):
        pic.jz_inverse_taps(np.ones(40))


@pytest.mark.parametrize("name", ["c1", "small"])
def test_loader_bit_exact_with_oracle(name):
    run = (workloads.config("c1") if name == "c1" else workloads.small(M=2, Nz=48, Nr=9, ppc=3))["runs"][0]
    L = pic.load_host(workloads.to_rundesc(run))
    o = oracle.Oracle(run["Nz"], run["Nr"], run["M"], run["dz"], run["dr"], 0.3, [1.0], [1.0])
    o.load_plasma(run["ppc"], run["n0"], run["ramp_start"], run["ramp_len"], run["seed"], run["n_tracked"])
    P = o.particles()
    for k in ("z", "x", "y", "w", "id"):
        assert np.array_equal(L[k], P[k]), k
    assert np.array_equal(L["tracked"], o.tracked()["id"])


def test_loader_ramps_bit_exact():
    """Up-ramp, plateau and down-ramp (App. A's profile)."""
    run = dict(workloads.small(M=1, Nz=40, Nr=6, ppc=2)["runs"][0])
    run.update(ramp_start=1.0, ramp_len=5.0, down_start=9.0, down_len=4.0)
    L = pic.load_host(workloads.to_rundesc(run))
    o = workloads.to_oracle(run, 0.3, [1.0], [1.0])
    assert np.array_equal(L["w"], o.particles()["w"])
    z = L["z"] * run["dz"]
    assert (L["w"][z < 1.0] == 0).all() and (L["w"][z > 13.0] == 0).all()
    assert (L["w"][(z > 6.0) & (z < 9.0)] > 0).all()


def _tune_query(runs, trial_steps=16, **kw):
    arr = (pic._RunDesc * len(runs))(*[r.to_c() for r in runs])
    opts, keep = pic._make_opts(kw.pop("precision", pic.PREC_FP64), pic.SOLVER_DUAL, 16, **kw)
    nbytes = ctypes.c_size_t(0)
    rc = pic._lib.pic_autotune(arr, len(runs), ctypes.byref(opts), None, ctypes.byref(nbytes), None, trial_steps,
                               None)
    return rc, nbytes.value, opts


def test_autotune_workspace_query_covers_every_candidate():
    """The autotuner's size query needs no device and covers its largest
    trial context: at least the context of any fitting candidate tile."""
    runs = [_desc(M=2, Nz=96, Nr=20), _desc(M=2, Nz=64, Nr=12)]
    rc, need, opts = _tune_query(runs)
    assert rc == pic.PIC_OK and need > 0
    for tz, tr in ((32, 8), (16, 4), (64, 2)):
        assert need >= pic.workspace_bytes(runs, tile_z=tz, tile_r=tr)
    # a fixed tile is the only candidate
    rc, need1, _ = _tune_query(runs, tile_z=16, tile_r=4)
    assert rc == pic.PIC_OK and need1 == pic.workspace_bytes(runs, tile_z=16, tile_r=4)


def test_autotune_rejects_bad_arguments():
    runs = [_desc(M=1)]
    assert _tune_query(runs, trial_steps=2)[0] == pic.PIC_E_INVALID
    assert _tune_query(runs, trial_steps=65)[0] == pic.PIC_E_INVALID
    assert _tune_query(runs, precision=16)[0] == pic.PIC_E_INVALID
    assert _tune_query([_desc(M=1), _desc(M=2)])[0] == pic.PIC_E_INVALID


def test_dla_integrate_rejects_bad_arguments_without_device():
    """Validation happens before any device call; n = 0 with valid arguments
    is a no-op that needs no GPU."""
    lib = pic._lib
    good = pic._DlaModel(2.8, 12.14, 1.002565, 1.0, 1.0)
    assert lib.pic_dla_integrate(ctypes.byref(good), 0, None, None, None, None, None, 100.0, 0.01, None) == pic.PIC_OK
    dummy = ctypes.c_void_p(4096)
    for model, n, h, t_end in ((pic._DlaModel(2.8, 12.14, 0.99, 1.0, 1.0), 4, 0.01, 10.0),  # vphi < 1
                               (pic._DlaModel(2.8, 0.0, 1.002, 1.0, 1.0), 4, 0.01, 10.0),  # kz <= 0
                               (good, -1, 0.01, 10.0), (good, 4, 0.0, 10.0), (good, 4, 0.01, float("inf"))):
        assert lib.pic_dla_integrate(ctypes.byref(model), n, dummy, dummy, dummy, dummy, dummy, t_end, h,
                                     None) == pic.PIC_E_INVALID
    assert lib.pic_dla_integrate(ctypes.byref(good), 4, None, dummy, dummy, dummy, dummy, 10.0, 0.01,
                                 None) == pic.PIC_E_INVALID
    assert lib.pic_dla_integrate(None, 0, None, None, None, None, None, 10.0, 0.01, None) == pic.PIC_E_INVALID


def test_library_binds_to_the_runtime_torch_loads():
    """Importing the package before torch must not bring a second HIP runtime
    into the process: the library receives torch's device memory and streams,
    so it has to bind to the runtime torch loads."""
    import subprocess
    import sys

    code = ("import paper_2303_12874_amd, torch\n"
            "maps = open('/proc/self/maps').read().splitlines()\n"
            "print(len({l.split()[-1] for l in maps if 'libamdhip64' in l}))\n")
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, cwd=ROOT, timeout=300)
    assert out.returncode == 0, out.stderr
    assert out.stdout.strip() == "1", out.stdout
