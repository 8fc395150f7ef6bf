"""Write the stored oracle results the full-size GPU tests compare against.

Runs only the FP64 oracle (``oracle/``) on the benchmark workloads, which are
too large for the serial oracle inside a test, and stores a sample of its
state after a prefix of steps (npz, a few MB each):

* ``oracle_c2_200.npz``: the 4096 x 256, modes 0..2, 8 ppc FP64 run over its
  first 200 steps (the FP64 parity horizon), from the loaded state;
* ``oracle_c5_20.npz``: the 8192 x 512, modes 0..3, 16 ppc run over 20 steps
  from the FP32-rounded loaded state (electrons as int32 cell + FP32
  offset, FP32 momenta and weights, FP32 E^0 and B^0), the start the FP32
  library takes;
* ``oracle_c4_r{k}_20.npz``, k = 0..5: each run of the six-run convergence
  scan over 20 steps from its FP32-rounded loaded state.

Each file holds: the run's description, the steps taken, dt and the
coefficients the oracle fitted (the GPU tests hand these to the library);
for every field array (E, B at both half steps, J) and mode the values at a
seeded sample of nodes (random nodes, the axis rows and the nodes where the
array is largest), each array's largest magnitude and L2 norm over the whole
grid; every tracked electron's id, per-mode work, gamma, initial gamma plus
the summed work, and its work by field direction; and (the FP64 run) the full
state of a sample of electrons chosen by id.

Usage: python tests/golden/make_oracle_fixtures.py [c2] [c5] [c4] (all three
by default, one process per run, in parallel).  The c2 and c5 runs take
about 15 minutes of one core each.
"""
from __future__ import annotations

import math
import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads  # noqa: E402
from oracle import coef  # noqa: E402

# the arrays compared, with the library's component number beside each
FIELDS = [("E_r", oracle.ER), ("E_phi", oracle.EP), ("E_z", oracle.EZ), ("B_r(n-1/2)", oracle.BOR),
          ("B_phi(n-1/2)", oracle.BOP), ("B_z(n-1/2)", oracle.BOZ), ("B_r(n+1/2)", oracle.BR),
          ("B_phi(n+1/2)", oracle.BP), ("B_z(n+1/2)", oracle.BZ), ("J_r", oracle.JR), ("J_phi", oracle.JP),
          ("J_z", oracle.JZ)]
N_RANDOM_NODES = 2048
N_AXIS_COLS = 256
N_TOP_NODES = 64
N_PARTICLES = 4096
MAX_TRACKED_STORED = 20000


def _node_sample(rng, Nz, Nr):
    """Flat indices (j * Nz + i) of the sampled nodes: random ones and a
    random set of columns on the two rows nearest the axis."""
    rnd = rng.choice((Nr + 1) * Nz, N_RANDOM_NODES, replace=False)
    cols = rng.choice(Nz, N_AXIS_COLS, replace=False)
    axis = np.concatenate([cols, Nz + cols])
    return np.unique(np.concatenate([rnd, axis]))


def run_one(job):
    name, run_index, steps, fp32_start = job
    cfg = workloads.config(name)
    run = cfg["runs"][run_index]
    tag = f"{name}" + (f"_r{run_index}" if len(cfg["runs"]) > 1 else "") + f"_{steps}"
    t0 = time.time()
    dt, CE, CB, lim = coef.solver_setup(16, run["M"], run["dz"], run["dr"])
    o = oracle.Oracle(run["Nz"], run["Nr"], run["M"], run["dz"], run["dr"], dt, CE, CB)
    o.load_plasma(run["ppc"], run["n0"], run["ramp_start"], run["ramp_len"], run["seed"], run["n_tracked"],
                  run.get("down_start", 0.0), run.get("down_len", 0.0))
    for p in run["pulses"]:
        o.add_laser(p["a0"], p["w0"], p["tau"], p["zc"], run["taper"])
    if fp32_start:
        o.round_to_fp32()
    o.start_fields()
    print(f"[{tag}] loaded {o.np} electrons in {time.time() - t0:.0f} s", flush=True)
    for k in range(steps):
        o.step(1)
        if (k + 1) % 10 == 0:
            print(f"[{tag}] step {k + 1}/{steps} at {time.time() - t0:.0f} s", flush=True)
    Nz, Nr, M = run["Nz"], run["Nr"], run["M"]
    rng = np.random.default_rng(20230322 + 97 * run_index + steps)
    base = _node_sample(rng, Nz, Nr)
    out = {"steps": steps, "dt": dt, "coef_E": CE, "coef_B": CB, "fp32_start": fp32_start, "np": o.np,
           "Nz": Nz, "Nr": Nr, "M": M, "field_names": np.array([f[0] for f in FIELDS])}
    for name_f, comp in FIELDS:
        for m in range(M + 1):
            a = o.get_field(comp, m).ravel()
            top = np.argsort(np.abs(a))[-N_TOP_NODES:]
            idx = np.unique(np.concatenate([base, top]))
            key = f"{name_f}/m{m}"
            out[f"idx:{key}"] = idx.astype(np.int64)
            out[f"val:{key}"] = a[idx]
            out[f"max:{key}"] = float(np.abs(a).max())
            out[f"l2:{key}"] = float(np.linalg.norm(a))
    tr = o.tracked()
    cw = o.cartesian_work()
    keep = np.arange(tr["id"].size)
    if keep.size > MAX_TRACKED_STORED:
        keep = np.sort(rng.choice(keep.size, MAX_TRACKED_STORED, replace=False))
    out["tracked_total"] = tr["id"].size
    out["tracked_W_absmax"] = np.abs(tr["W"]).max(axis=0) if tr["id"].size else np.zeros(M + 1)
    for k in ("id", "W", "gamma", "gamma_acc"):
        out[f"tracked_{k}"] = tr[k][keep]
    out["tracked_Wz"], out["tracked_Wperp"] = cw["Wz"][keep], cw["Wperp"][keep]
    if not fp32_start:  # the FP64 run: a sample of electrons, full state
        P = o.particles()
        u = np.sqrt(P["ux"] ** 2 + P["uy"] ** 2 + P["uz"] ** 2)
        r = np.hypot(P["x"], P["y"])
        pick = np.unique(np.concatenate([rng.choice(P["z"].size, N_PARTICLES, replace=False),
                                         np.argsort(u)[-256:], np.argsort(r)[:256]]))
        for k in ("z", "x", "y", "ux", "uy", "uz", "w", "id"):
            out[f"p_{k}"] = P[k][pick]
        out["p_umax"] = float(max(np.abs(P[k]).max() for k in ("ux", "uy", "uz")))
    path = os.path.join(HERE, f"oracle_{tag}.npz")
    np.savez_compressed(path, **out)
    print(f"[{tag}] wrote {path} ({os.path.getsize(path) / 1e6:.1f} MB) after {time.time() - t0:.0f} s",
          flush=True)
    return path


def jobs(which):
    out = []
    if "c2" in which:
        out.append(("c2", 0, 200, False))
    if "c5" in which:
        out.append(("c5", 0, 20, True))
    if "c4" in which:
        out += [("c4", k, 20, True) for k in range(6)]
    return out


if __name__ == "__main__":
    which = sys.argv[1:] or ["c2", "c5", "c4"]
    js = jobs(which)
    with ProcessPoolExecutor(max_workers=min(len(js), max(1, (os.cpu_count() or 1)))) as ex:
        for p in ex.map(run_one, js):
            print(p, flush=True)
