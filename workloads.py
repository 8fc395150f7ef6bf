"""Seeded synthetic workloads (LWFA-shaped plasmas and lasers).

Plain parameters only -- no arithmetic of the method -- shared by the tests
(both the HIP library and the oracle are built from the same description)
and by the benchmark.  Lengths are in c/omega_0 (laser wavelength 2 pi),
densities in units of the critical density.  The paper's own runs use a
1814 x 160 quasi-3D grid, ionisation injection into a He/N2 gas and a moving
window (Appendix A); none of that data is available, so these synthetic
plasmas and pulses stand in for it at the sizes of the benchmark configs.
"""
from __future__ import annotations

import math
import numpy as np

LAMBDA0 = 2.0 * math.pi
SEED_BASE = 2303128740


def _lp(n0):
    """plasma wavelength (c/omega_0) at density n0 (units of n_c)"""
    return LAMBDA0 / math.sqrt(n0)


def config(name: str) -> dict:
    """One named workload: a list of runs and the precision / step count."""
    if name in ("c1", "c3"):
        dz = LAMBDA0 / 16
        run = dict(Nz=256, Nr=64, M=1, ppc=4, dz=dz, dr=4 * dz, n0=0.01, ramp_start=0.0, ramp_len=0.0,
                   pulses=[dict(a0=1.0, w0=8 * LAMBDA0, tau=10 * LAMBDA0, zc=8 * LAMBDA0)], taper=2 * LAMBDA0,
                   seed=SEED_BASE + (10 if name == "c1" else 30), n_tracked=1000)
        return dict(name=name, runs=[run], precision=64 if name == "c1" else 32, steps=100,
                    desc="256x64 r-z grid, modes 0..1, 4 ppc (~65k electrons), n=0.01 n_c, a0=1 w0=8 lambda "
                         "10-period pulse")
    if name == "c2":
        dz = LAMBDA0 / 16
        tau = 2 * _lp(0.005)
        run = dict(Nz=4096, Nr=256, M=2, ppc=8, dz=dz, dr=4 * dz, n0=0.005, ramp_start=0.0,
                   ramp_len=200 * LAMBDA0,
                   pulses=[dict(a0=2.0, w0=10 * LAMBDA0, tau=tau, zc=1.5 * tau + 2 * LAMBDA0)], taper=2 * LAMBDA0,
                   seed=SEED_BASE + 20, n_tracked=10000)
        return dict(name=name, runs=[run], precision=64, steps=2000,
                    desc="4096x256 r-z grid, modes 0..2, 8 ppc (~8.4M electrons), n=0.005 n_c with a 200-lambda "
                         "up-ramp, a0=2 w0=10 lambda, 2-plasma-period pulse")
    if name == "c4":
        runs = []
        steps = []
        for r, ppl in enumerate((12, 16, 24, 32, 48, 64)):
            dz = LAMBDA0 / ppl
            runs.append(dict(Nz=256 * ppl, Nr=4 * ppl, M=2, ppc=4, dz=dz, dr=4 * dz, n0=0.01, ramp_start=0.0,
                             ramp_len=0.0,
                             pulses=[dict(a0=1.0, w0=8 * LAMBDA0, tau=10 * LAMBDA0, zc=22 * LAMBDA0)],
                             taper=2 * LAMBDA0, seed=SEED_BASE + 40 + r, n_tracked=1000))
            steps.append(100 * ppl // 16)
        return dict(name=name, runs=runs, precision=32, steps=steps,
                    desc="six runs at 12..64 points per lambda (Nz 3072..16384, Nr 48..256), modes 0..2, 4 ppc")
    if name == "c5":
        dz = LAMBDA0 / 16
        lp = _lp(0.003)
        run = dict(Nz=8192, Nr=512, M=3, ppc=16, dz=dz, dr=4 * dz, n0=0.003, ramp_start=0.0, ramp_len=0.0,
                   pulses=[dict(a0=3.0, w0=10 * LAMBDA0, tau=lp / 2, zc=60 * LAMBDA0),
                           dict(a0=1.5, w0=10 * LAMBDA0, tau=lp / 2, zc=60 * LAMBDA0 - lp)],
                   taper=2 * LAMBDA0, seed=SEED_BASE + 50, n_tracked=100000)
        return dict(name=name, runs=[run], precision=32, steps=5000,
                    desc="8192x512 r-z grid, modes 0..3, 16 ppc (~67M electrons), n=0.003 n_c, two pulses a0=3 "
                         "and 1.5 one plasma period apart")
    if name in ("cv32", "cv128"):
        # the cost comparison of converged runs (Sec. IV.B): the dual solver
        # at about 30 points per wavelength against Yee at about 120 with half
        # the electrons per cell; same box (256 x 16 lambda), same radial cell
        ppl = 32 if name == "cv32" else 128
        dz = LAMBDA0 / ppl
        run = dict(Nz=256 * ppl, Nr=128, M=2, ppc=4 if ppl == 32 else 2, dz=dz, dr=LAMBDA0 / 8, n0=0.01,
                   ramp_start=0.0, ramp_len=0.0,
                   pulses=[dict(a0=1.0, w0=8 * LAMBDA0, tau=10 * LAMBDA0, zc=22 * LAMBDA0)], taper=2 * LAMBDA0,
                   seed=SEED_BASE + 60, n_tracked=1000)
        return dict(name=name, runs=[run], precision=32, steps=200,
                    desc=f"{256 * ppl}x128 r-z grid ({ppl} points per lambda, dr = lambda/8), modes 0..2, "
                         f"{run['ppc']} ppc: the {'dual' if ppl == 32 else 'Yee'} side of the converged-run cost "
                         "comparison")
    raise KeyError(name)


def cpu_sample(name: str) -> dict:
    """The bounded sample of a workload that the CPU baseline times with the
    oracle: {"runs", "steps", "desc"}.  Whole steps of the workload's own runs,
    except for the 67 M-electron run, whose one step takes the serial oracle
    about 50 s and 8 GB: its sample is a slab of 512 of its 8192 columns (same
    radius, modes, electrons per cell, density and pulses, the leading pulse
    inside the slab), 4.2 M electrons."""
    cfg = config(name)
    if name != "c5":
        steps = {"c1": 200, "c3": 200, "c2": 3, "c4": 1, "cv32": 3, "cv128": 1}[name]
        return dict(runs=cfg["runs"], steps=steps, desc=f"{steps} full step(s) of the workload")
    run = dict(cfg["runs"][0])
    run["Nz"] = 512
    lp = _lp(run["n0"])
    run["pulses"] = [dict(p, zc=20 * LAMBDA0 - k * lp) for k, p in enumerate(run["pulses"])]
    return dict(runs=[run], steps=3,
                desc="3 steps of a 512-column slab of the workload (512x512, modes 0..3, 16 ppc, 4.2M electrons, "
                     "both pulses)")


def small(name="tiny", M=1, Nz=64, Nr=12, ppc=2, n0=0.02, a0=1.5, seed=99, n_tracked=64) -> dict:
    """Small grids that still span several sort tiles and a ragged radial tile."""
    dz = LAMBDA0 / 16
    run = dict(Nz=Nz, Nr=Nr, M=M, ppc=ppc, dz=dz, dr=4 * dz, n0=n0, ramp_start=0.0, ramp_len=0.0,
               pulses=[dict(a0=a0, w0=3 * LAMBDA0, tau=2 * LAMBDA0, zc=2 * LAMBDA0)] if M >= 1 else [],
               taper=LAMBDA0, seed=seed, n_tracked=n_tracked)
    return dict(name=name, runs=[run], precision=64, steps=20, desc="small test grid")


def to_rundesc(run: dict, n_steps: int = 0):
    """The HIP library's RunDesc of a run (imports the binding lazily)."""
    import paper_2303_12874_amd as pic

    return pic.RunDesc(Nz=run["Nz"], Nr=run["Nr"], M=run["M"], ppc=run["ppc"], dz=run["dz"], dr=run["dr"],
                       n0=run["n0"], ramp_start=run["ramp_start"], ramp_len=run["ramp_len"],
                       down_start=run.get("down_start", 0.0), down_len=run.get("down_len", 0.0),
                       pulses=[pic.Pulse(**p) for p in run["pulses"]], taper=run["taper"], seed=run["seed"],
                       n_tracked=run["n_tracked"], n_steps=n_steps)


def to_oracle(run: dict, dt, CE, CB):
    """The oracle run of the same description (imports the oracle lazily)."""
    import oracle

    o = oracle.Oracle(run["Nz"], run["Nr"], run["M"], run["dz"], run["dr"], dt, CE, CB)
    if run["ppc"] > 0:
        o.load_plasma(run["ppc"], run["n0"], run["ramp_start"], run["ramp_len"], run["seed"], run["n_tracked"],
                      run.get("down_start", 0.0), run.get("down_len", 0.0))
    for p in run["pulses"]:
        o.add_laser(p["a0"], p["w0"], p["tau"], p["zc"], run["taper"])
    o.start_fields()
    return o


# ---------------------------------------------------------------------------
# injected electrons for the reduced model of Sec. II (units c = omega_p = 1)

DLA_APP_A = {"a0": 2.8, "kz": 12.14, "vphi": 1.002565, "vg": 0.993583, "R": 3.0, "t_inject": 200.0}


def dla_injection(n: int, seed: int, R: float = 3.0, vg: float = 0.993583, t_inject: float = 200.0) -> dict:
    """Electrons injected into the bubble as App. A describes: injection time
    uniform over [0, t_inject]; on the y = 0 plane with zeta uniform in
    [-2R + 0.286, -2R + 0.836] and x uniform in [-r_b, r_b], r_b(zeta) =
    (R^2 - (zeta + R)^2)^(1/2); gamma uniform in [gamma_g, 2 gamma_g] with
    gamma_g = (1 - vg^2)^(-1/2); the velocity's angle to the x axis uniform
    over the angles with v_z >= vg.  Returns t0 and the state (x, zeta, xd,
    zetad = v_z - 1), FP64, sorted by t0 (so that neighbouring electrons take
    similar numbers of steps)."""
    rng = np.random.default_rng(seed)
    t0 = np.sort(rng.uniform(0.0, t_inject, n))
    zeta = rng.uniform(-2 * R + 0.286, -2 * R + 0.836, n)
    rb = np.sqrt(R * R - (zeta + R) ** 2)
    x = rng.uniform(-1.0, 1.0, n) * rb
    gg = 1.0 / np.sqrt(1.0 - vg * vg)
    g = rng.uniform(gg, 2 * gg, n)
    v = np.sqrt(1.0 - 1.0 / (g * g))
    amin = np.arcsin(np.minimum(vg / v, 1.0))
    ang = rng.uniform(amin, np.pi - amin)
    vz = v * np.sin(ang)
    return {"t0": t0, "x": x, "zeta": zeta, "xd": v * np.cos(ang), "zetad": vz - 1.0, "gamma": g}
