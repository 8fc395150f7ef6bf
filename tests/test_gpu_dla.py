"""GPU parity of the reduced-model ensemble (Sec. II, Eq. (8); App. A) against
the FP64 oracle, through pic_dla_integrate.

Electrons are injected by the App. A recipe (over a shortened window so that
the oracle finishes in seconds) and integrated to a common end time; the final
states must agree to 1e-10 of each component's largest value.  Perturbing the
initial states by 1e-15 moves the oracle's end states by about 1e-13 over
these horizons, so the bar leaves room only for rounding-order differences.
The laser-alone constant of motion is checked on the GPU path itself.
"""
import math

import numpy as np
import pytest

import workloads
from oracle import dla
from test_gpu_parity import _pic, _say

pytestmark = pytest.mark.gpu
TOL = 1e-10


def _run_gpu(pic, d, t_end, h, **model):
    import torch

    dev = torch.device("cuda:0")
    ts = {k: torch.tensor(np.ascontiguousarray(d[k]), dtype=torch.float64, device=dev)
          for k in ("t0", "x", "zeta", "xd", "zetad")}
    pic.dla_integrate(ts["t0"], ts["x"], ts["zeta"], ts["xd"], ts["zetad"], t_end, h, **model)
    torch.cuda.synchronize()
    return np.stack([ts[k].cpu().numpy() for k in ("x", "zeta", "xd", "zetad")])


def _oracle(d, t_end, h, **model):
    p = dla.params(**{k: v for k, v in model.items()})
    y0 = np.stack([d["x"], d["zeta"], d["xd"], d["zetad"]])
    return dla.integrate(p, d["t0"], y0, t_end, h)


def _worst(a, b):
    sc = np.maximum(np.abs(b).max(axis=1), 1e-300)
    return (np.abs(a - b).max(axis=1) / sc).max()


# cos(omega_0 dt / 2) of the 3D Yee run of App. A (dt = 0.01875 / omega_p): about 0.994
@pytest.mark.parametrize("cB", [1.0, math.cos(0.5 * 12.14 * 1.002565 * 0.01875)])
def test_dla_ensemble_matches_oracle(cB):
    """1000 electrons (a ragged last block of 256) injected over [0, 20],
    integrated to t = 40 with h = 0.01, with exact fields and with the
    magnetic terms scaled by cos(omega_0 dt / 2)."""
    _say(f"[gpu] dla ensemble cB={cB:.6f}")
    pic = _pic()
    d = workloads.dla_injection(1000, 11, t_inject=20.0)
    g = _run_gpu(pic, d, 40.0, 0.01, cB=cB)
    o = _oracle(d, 40.0, 0.01, cB=cB)
    assert np.isfinite(g).all()
    w = _worst(g, o)
    assert w < TOL, w
    assert dla.gamma(g).max() > 2 * d["gamma"].max()  # the electrons were accelerated


def test_dla_laser_alone_invariant_on_gpu():
    """Without the bubble, gamma - v_phi (p_z - A_z) stays constant along the
    GPU trajectories (all electrons start at t = 0)."""
    _say("[gpu] dla laser-alone invariant")
    pic = _pic()
    d = workloads.dla_injection(512, 12, t_inject=0.0)
    p = dla.params(wake=0.0)
    y0 = np.stack([d["x"], d["zeta"], d["xd"], d["zetad"]])
    g = _run_gpu(pic, d, 30.0, 0.005, wake=0.0)

    def inv(t, y):
        gm = dla.gamma(y)
        xi = y[1] + (1.0 - p["vphi"]) * t
        az = p["a0"] * (p["kperp"] / p["kz"]) * dla.bessel(p["kperp"] * y[0])[1] * np.sin(p["kz"] * xi)
        return gm - p["vphi"] * (gm * (y[3] + 1.0) - az)

    drift = np.abs(inv(30.0, g) - inv(0.0, y0))
    assert drift.max() < 1e-10 * dla.gamma(g).max(), drift.max()


def test_dla_edge_cases():
    """Electrons injected at or after t_end keep their state bit for bit; a
    single electron and an empty call work."""
    _say("[gpu] dla edge cases")
    pic = _pic()
    d = workloads.dla_injection(7, 13, t_inject=20.0)
    d["t0"][[1, 4]] = [25.0, 10.0]  # 10.0 is the end time itself
    g = _run_gpu(pic, d, 10.0, 0.01)
    o = _oracle(d, 10.0, 0.01)
    y0 = np.stack([d["x"], d["zeta"], d["xd"], d["zetad"]])
    late = d["t0"] >= 10.0
    assert np.array_equal(g[:, late], y0[:, late])
    assert _worst(g, o) < TOL
    one = {k: v[:1].copy() for k, v in d.items()}
    assert _worst(_run_gpu(pic, one, 10.0, 0.01), _oracle(one, 10.0, 0.01)) < TOL
    empty = {k: v[:0].copy() for k, v in d.items()}
    assert _run_gpu(pic, empty, 10.0, 0.01).shape == (4, 0)


def test_dla_outside_the_series_range():
    """Electrons at |k_perp x| from 2.5 to 6 (the kernel's Bessel functions
    switch from their power series to the library's at 3) match the oracle."""
    _say("[gpu] dla outside the series range")
    pic = _pic()
    d = workloads.dla_injection(256, 14, t_inject=5.0)
    kperp = dla.params()["kperp"]
    d["x"] = np.linspace(2.5, 6.0, 256) / kperp * np.where(np.arange(256) % 2 == 0, 1.0, -1.0)
    g = _run_gpu(pic, d, 8.0, 0.005)
    o = _oracle(d, 8.0, 0.005)
    assert np.isfinite(g).all()
    assert _worst(g, o) < TOL
