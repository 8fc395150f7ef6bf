"""Benchmark: particle-steps/s of the quasi-3D r-z PIC step with the dual solver.

One bench step = one time step of the whole hot path (cell sort when due,
gather + push + deposit, E update with the filtered current, B update) on a
synthetic LWFA-shaped plasma, with every input resident in HBM.  Prints one
JSON line.  The default workload is the largest single-GPU one: the 8192 x
512, modes 0..3, 16 ppc FP32 run (67 M electrons, tile and sort interval from
the library's autotuner); after its timed region the plain FP64 path is timed
on the same workload, and the FP32 state's difference from the FP64 state
after the same steps is reported beside the FP32 bounds the tests hold
against the FP64 oracle.  --workload c2 selects the 4096 x 256, modes 0..2,
8 ppc FP64 run, --workload c4 the six-run FP32 convergence scan (12..64
points per wavelength) stepped as one batch, each run for its own number of
steps.

Per-kernel durations come from HIP events the library records around each
launch on its own stream (pic_profile); the roofline object prices the
dominant kernel's algorithmic bytes against the MI355X HBM peak.  The CPU
baseline times the FP64 oracle (test infrastructure) on a bounded sample of
the same workload on the host, on one core and on every usable core.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import workloads  # noqa: E402

METRIC = "particle-steps/s (gather+push+deposit+solve), FP32 vs FP64 GPU at stated error"
HBM_PEAK_GBS = 8000.0


def algorithmic_bytes(run: dict, precision: int) -> dict:
    """Bytes each kernel must move per launch: particle state
    read and written once, field/current planes read or written once."""
    w = 8 if precision == 64 else 4
    NM = 2 * run["M"] + 1
    np_ = run["Nz"] * (run["Nr"] - 1) * run["ppc"]
    cells = (run["Nr"] + 1) * run["Nz"]
    # particle: read z (+fz), x, y, ux, uy, uz, w, id; write z (+fz), x, y, ux, uy, uz
    part_read = 7 * w + 4 + (4 if precision == 32 else 0)
    part_write = 6 * w + (4 if precision == 32 else 0)
    return {
        "push": np_ * (part_read + part_write) + cells * 9 * NM * w,  # E, Bbar read; J written
        "efield": cells * 15 * NM * w,  # B, J, E read; E and the next J written
        "bfield": cells * 12 * NM * w,  # E, B read; B and Bbar written
        "sort": np_ * 2 * (part_read + 4),  # read + permuted write of the particle state
    }


def measured_traffic(workload: str, kernel: str, tile: str, sort_interval: int, precision: int):
    """HBM bytes per launch of `kernel` from the committed FETCH_SIZE / WRITE_SIZE
    counter passes (copy-calibrated), or None when the kernels changed since or
    the run's tile, sort interval or precision differ from the profiled ones."""
    try:
        with open(os.path.join(ROOT, "profiles", "hbm_traffic.json")) as f:
            t = json.load(f)
        with open(os.path.join(ROOT, "paper_2303_12874_amd", "csrc", "kernels.hip"), "rb") as f:
            h = hashlib.sha256(f.read()).hexdigest()
    except (OSError, ValueError):
        return None
    if t.get("kernels_sha256") != h:
        return None
    w = t.get("workloads", {}).get(workload, {})
    if w.get("settings") != {"tile": tile, "sort_interval": sort_interval, "precision": precision}:
        return None
    e = w.get(kernel)
    return None if e is None else e["read_bytes"] + e["write_bytes"]


# kernel name -> bench phase of the rocprofv3 summaries
_PHASE_OF = (("push_kernel", "push"), ("efield_kernel", "efield"), ("bfield_kernel", "bfield"),
             ("sort_tile_kernel", "sort_tile"), ("sort_key_kernel", "sort_key"), ("sort_scatter_kernel", "sort_scatter"),
             ("scan_block_kernel", "scan_block"), ("scan_add_kernel", "scan_add"), ("copy_i32_kernel", "copy_i32"),
             ("window_shift_kernel", "window_shift"))


def _csv_rows(directory: str, suffix: str) -> list:
    import csv
    import glob

    rows = []
    for f in sorted(glob.glob(os.path.join(directory, "**", "*" + suffix), recursive=True)):
        with open(f) as fh:
            rows += list(csv.DictReader(fh))
    return rows


def summarize_counters(workload: str, fetch_dir: str, write_dir: str, tile: str, sort_interval: int,
                       precision: int) -> dict:
    """Per-launch HBM bytes of each kernel from a FETCH_SIZE pass and a
    WRITE_SIZE pass (rocprofv3 --pmc, csv) of the benchmark's command, scaled
    by what the same counters read for the benchmark's own 1 GiB device copy
    (the largest copyBuffer dispatch); written into profiles/hbm_traffic.json
    under the workload with the kernels' source hash, so that bench lines of
    the same settings report it as roofline.traffic."""
    vals = {}
    for counter, d in (("FETCH_SIZE", fetch_dir), ("WRITE_SIZE", write_dir)):
        for r in _csv_rows(d, "counter_collection.csv"):
            if r["Counter_Name"] == counter:
                vals.setdefault(counter, []).append((r["Kernel_Name"], float(r["Counter_Value"])))
    gib_kib = (1 << 30) / 1024.0
    copies = {c: max(v for n, v in vals[c] if "copyBuffer" in n) for c in ("FETCH_SIZE", "WRITE_SIZE")}
    ff, wf = gib_kib / copies["FETCH_SIZE"], gib_kib / copies["WRITE_SIZE"]
    entry = {"settings": {"tile": tile, "sort_interval": sort_interval, "precision": precision}}
    for key, phase in _PHASE_OF:
        f = [v for n, v in vals["FETCH_SIZE"] if key in n]
        w = [v for n, v in vals["WRITE_SIZE"] if key in n]
        if f and w:
            fk, wk = sum(f) / len(f), sum(w) / len(w)
            entry[phase] = {"read_bytes": fk * 1024 * ff, "write_bytes": wk * 1024 * wf, "fetch_kib": fk,
                            "write_kib": wk, "launches": len(f)}
    path = os.path.join(ROOT, "profiles", "hbm_traffic.json")
    try:
        with open(path) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        t = {}
    with open(os.path.join(ROOT, "paper_2303_12874_amd", "csrc", "kernels.hip"), "rb") as fh:
        h = hashlib.sha256(fh.read()).hexdigest()
    if t.get("kernels_sha256") != h:
        t = {"workloads": {}}
    t["kernels_sha256"] = h
    t["fetch_factor"], t["write_factor"] = ff, wf
    t["calibration"] = (f"1 GiB device copy: FETCH_SIZE {copies['FETCH_SIZE']:.0f} KiB, "
                        f"WRITE_SIZE {copies['WRITE_SIZE']:.0f} KiB")
    t.setdefault("workloads", {})[workload] = entry
    with open(path, "w") as fh:
        json.dump(t, fh, indent=1)
    return entry


def summarize_trace(trace_dir: str) -> str:
    """Markdown table of a rocprofv3 --kernel-trace --stats run (kernel_stats.csv)."""
    rows = _csv_rows(trace_dir, "kernel_stats.csv")
    tot = sum(float(r["TotalDurationNs"]) for r in rows) or 1.0
    out = ["| Kernel | Calls | Average (us) | Min (us) | Max (us) | Share |", "|---|---:|---:|---:|---:|---:|"]
    for r in sorted(rows, key=lambda r: -float(r["TotalDurationNs"])):
        name = r["Name"] if len(r["Name"]) < 72 else r["Name"][:69] + "..."
        out.append(f"| `{name}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | {float(r['MinNs']) / 1e3:.1f} | "
                   f"{float(r['MaxNs']) / 1e3:.1f} | {100 * float(r['TotalDurationNs']) / tot:.1f}% |")
    return "\n".join(out)


WORKLOADS = ("c1", "c2", "c3", "c4", "c5", "cv32", "cv128", "dla")


def _oracle_sample(workload: str, n_coef: int, shape: int = 1) -> tuple:
    """The serial FP64 oracle over the workload's bounded CPU sample
    (workloads.cpu_sample), with the given particle shape order:
    (particle-steps, seconds of stepping)."""
    import oracle  # noqa: F401  (test infrastructure: the CPU baseline only)
    from oracle import coef

    smp = workloads.cpu_sample(workload)
    tot, el = 0, 0.0
    for run in smp["runs"]:
        dt, CE, CB, _ = coef.solver_setup(n_coef, run["M"], run["dz"], run["dr"])
        o = workloads.to_oracle(run, dt, CE, CB)
        o.set_shape(shape)
        t0 = time.perf_counter()
        o.step(smp["steps"])
        el += time.perf_counter() - t0
        tot += o.np * smp["steps"]
        del o
    return tot, el


def host_cpu() -> tuple:
    """(usable host cores, CPU model name)"""
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count() or 1
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return cores, model


def cpu_baseline(workload: str, n_coef: int = 16, max_procs: int = 16, shape: int = 1) -> dict:
    """The FP64 oracle as it stands (serial C) on the workload's bounded
    sample: once on one core, then as one process per usable host core (at
    most max_procs), all running the same sample at once; the all-core value
    is their summed particle-steps over the wall time of the slowest."""
    cores, model = host_cpu()
    smp = workloads.cpu_sample(workload)
    tot1, el1 = _oracle_sample(workload, n_coef, shape)
    one = {"value": tot1 / el1, "unit": "particle-steps/s", "cores": 1, "kind": "oracle",
           "sample": f"{smp['desc']}: {tot1} particle-steps, serial C oracle, setup excluded, {el1:.1f} s",
           "cpu": model}
    nproc = max(1, min(cores, max_procs))
    if nproc == 1:
        return dict(one, all_cores=dict(one))
    import subprocess

    cmd = [sys.executable, os.path.abspath(__file__), "--oracle-sample", workload, "--n-coef", str(n_coef),
           "--shape", str(shape)]
    procs = [subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.DEVNULL, text=True,
                              env=dict(os.environ, OMP_NUM_THREADS="1")) for _ in range(nproc)]
    res = []
    for p in procs:
        out, _ = p.communicate()
        if p.returncode != 0:
            raise RuntimeError(f"oracle sample process failed ({p.returncode})")
        res.append(json.loads(out.strip().splitlines()[-1]))
    tot = sum(r["particle_steps"] for r in res)
    wall = max(r["seconds"] for r in res)
    one["all_cores"] = {"value": tot / wall, "unit": "particle-steps/s", "cores": nproc, "kind": "oracle",
                        "sample": f"{nproc} concurrent processes of the serial oracle, each on the same sample "
                                  f"({smp['desc']}); summed particle-steps over the slowest one's "
                                  f"{wall:.1f} s of stepping",
                        "cpu": model, "host_cores": cores}
    return one


# The FP32 form's error bounds against the FP64 oracle (started from the same
# FP32-rounded state), as the GPU tests hold them: per field array and mode
# (relative L2: E and B integrate the current and are held to its bound, the
# laser's and the wake's signature arrays tighter; largest node error over
# the array's largest value), per tracked electron (gamma, relative to max(gamma - 1, 1e-3)) and
# per mode (work).
FP32_BOUNDS = {"E_B_l2": 3e-4, "laser_E_r_m1_and_wake_E_z_m0_l2": 1e-4, "J_l2": 3e-4, "E_B_max": 1e-3,
               "J_max": 3e-3,
               "tracked_gamma_p99": 1e-4, "tracked_gamma_max": 1e-3,
               "mode_work": "1e-3 max_p |W_m| + 1e-7",
               "held_by": "tests/test_gpu_fp32.py (256x64, 100 steps), tests/test_gpu_fullsize.py (8192x512 prefix, "
                          "six-run scan), tests/test_gpu_vs_stored_oracle.py"}


def fp32_vs_fp64(pic, s32, s64, run: dict) -> dict:
    """Difference of the FP32 state from the FP64 state of the same workload
    after the same steps (run 0): relative L2 of every E, Bbar and J array
    and mode, and the tracked electrons' gamma and per-mode work."""
    import numpy as np

    comps = [("E_r", pic.ER), ("E_phi", pic.EPHI), ("E_z", pic.EZ), ("Bbar_r", pic.BR), ("Bbar_phi", pic.BPHI),
             ("Bbar_z", pic.BZ), ("J_r", pic.JR), ("J_phi", pic.JPHI), ("J_z", pic.JZ)]
    l2 = {}
    for name, c in comps:
        for m in range(run["M"] + 1):
            a, b = s32.fields(c, m), s64.fields(c, m)
            nb = np.linalg.norm(b)
            l2[f"{name}/m{m}"] = float(np.linalg.norm(a - b) / nb) if nb > 0 else float(np.linalg.norm(a))
    w32, w64 = s32.mode_work(0), s64.mode_work(0)
    ok = bool(np.array_equal(w32["id"], w64["id"]))
    g = np.abs(w32["gamma_acc"] - w64["gamma_acc"]) / np.maximum(w64["gamma_acc"] - 1.0, 1e-3)
    wtol = 1e-3 * np.abs(w64["W"]).max(axis=0) + 1e-7
    eb = {k: v for k, v in l2.items() if not k.startswith("J")}
    jj = {k: v for k, v in l2.items() if k.startswith("J")}
    return {"steps": int(s32.info(0)["steps_done"]), "field_l2": l2,
            "E_B_l2_worst": max(eb.values()), "J_l2_worst": max(jj.values()),
            "tracked_ids_equal": ok, "tracked_gamma_p99": float(np.percentile(g, 99)) if g.size else 0.0,
            "tracked_gamma_max": float(g.max()) if g.size else 0.0,
            "mode_work_max_over_tol": float((np.abs(w32["W"] - w64["W"]) / wtol).max()) if g.size else 0.0}


# FP64 operations of one Runge-Kutta step of Eq. (8), not counting the three
# special-function calls (J0, J1, sincos) and the reciprocal square root and
# division of each of the six right-hand-side evaluations: 48 per evaluation
# and 170 for the stage combinations and times
DLA_FLOPS_PER_STEP = 6 * 48 + 170
FP64_VECTOR_PEAK_TFLOPS = 78.6


def work_split(sim, M: int) -> dict:
    """Energy gain of the tracked electrons of run 0 split by azimuthal mode
    (Eq. (16)): m = 0 is the wake's work, m = 1 the laser's.  Sums over all
    tracked electrons and over the 1% with the largest gamma."""
    import numpy as np

    w = sim.mode_work(0)
    W, g = w["W"], w["gamma"]
    top = np.argsort(g)[-max(1, g.size // 100):]
    return {"tracked": int(g.size), "steps": int(sim.info(0)["steps_done"]),
            "gamma_max": float(g.max()), "gamma_mean": float(g.mean()),
            "W_sum_by_mode": [float(v) for v in W.sum(axis=0)],
            "top1pct": {"gamma_min": float(g[top].min()), "W_mean_by_mode": [float(v) for v in W[top].mean(axis=0)],
                        "laser_share": float(W[top, 1].sum() / max(W[top].sum(), 1e-300)) if M >= 1 else 0.0},
            "identity_max_err": float(np.abs(w["gamma_acc"] - g).max())}


def work_compare(sim, run: dict) -> dict:
    """The three estimates of the LWFA / DLA split that Sec. IV.C compares
    (Fig. 4), on the tracked electrons of run 0: the per-mode work of the
    quasi-3D decomposition (Eq. (16); m = 0 the wake, m = 1 the laser), the
    work of the longitudinal and transverse fields (Eq. (17)), and that work
    corrected for the laser's longitudinal field with the Pukhov ratio
    (Eqs. (20)-(21)).  Means over all tracked electrons and over the 1% with
    the largest gamma (the "highest-energy electrons" of the figure)."""
    import numpy as np

    mw = sim.mode_work(0)
    cw = sim.cartesian_work(0, corrected=True)
    g = mw["gamma"]
    top = np.argsort(g)[-max(1, g.size // 100):]

    def means(sel):
        return {"modal_lwfa_W0": float(mw["W"][sel, 0].mean()), "modal_dla_W1": float(mw["W"][sel, 1].mean()),
                "modal_other_modes": float(mw["W"][sel, 2:].sum(axis=1).mean()) if run["M"] >= 2 else 0.0,
                "component_lwfa_Wz": float(cw["Wz"][sel].mean()), "component_dla_Wperp": float(cw["Wperp"][sel].mean()),
                "corrected_lwfa_W*": float(cw["W_lwfa"][sel].mean()), "corrected_dla_W*": float(cw["W_dla"][sel].mean()),
                "pukhov_f": float(cw["f"][sel].mean()), "gamma_mean": float(g[sel].mean()),
                "gamma_minus_1": float((g[sel] - 1).mean())}
    return {"tracked": int(g.size), "steps": int(sim.info(0)["steps_done"]), "all": means(np.arange(g.size)),
            "top1pct": means(top), "top1pct_gamma_min": float(g[top].min())}


def convergence_scan(pic, torch, dev, args) -> dict:
    """The resolution scan of Sec. IV.B (Fig. 3) on the six-run workload
    (12..64 points per wavelength, equal physical time), once with the dual
    solver and once with Yee, each batch in one context: per run, the
    charge-weighted RMS divergence theta_x = atan(u_x / u_z) of the electrons
    above a Lorentz-factor cut (the 99th percentile of gamma in the finest
    dual run, the same cut for every run) and the cost (ms per step, steps
    taken, ms for the whole run)."""
    import numpy as np

    cfg = workloads.config("c4")
    runs = cfg["runs"]
    scale = max(1, args.convergence_scale)
    # equal physical time: the dual runs take the workload's steps (times the
    # scale), the Yee runs (whose Courant-limited dt is longer) as many as
    # cover the same time
    dts = {name: [pic.solver_setup(r["M"], r["dz"], r["dr"], solver=sv, n_coef=nc)[0] for r in runs]
           for name, sv, nc in (("dual", pic.SOLVER_DUAL, 16), ("yee", pic.SOLVER_YEE, 1))}
    nsteps = {"dual": [n * scale for n in cfg["steps"]]}
    nsteps["yee"] = [int(round(n * dd / dy)) for n, dd, dy in zip(nsteps["dual"], dts["dual"], dts["yee"])]
    out = {"runs": [f"{r['Nz']}x{r['Nr']} ({round(2 * np.pi / r['dz'])} points per wavelength)" for r in runs],
           "physical_time": [n * dd for n, dd in zip(nsteps["dual"], dts["dual"])], "scale": scale}
    sims = {}
    for name, solver, n_coef in (("dual", pic.SOLVER_DUAL, 16), ("yee", pic.SOLVER_YEE, 1)):
        steps = nsteps[name]
        sim = pic.Simulation([workloads.to_rundesc(r, n_steps=n) for r, n in zip(runs, steps)],
                             precision=cfg["precision"], solver=solver, n_coef=n_coef, tile_z=24, tile_r=8,
                             sort_interval=16, device="cuda:0")
        sim.profile(True)
        stream = torch.cuda.current_stream(dev)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        sim.step(max(steps))
        e1.record(stream)
        torch.cuda.synchronize()
        out[name] = {"ms_whole_scan": e0.elapsed_time(e1), "dt": [sim.info(i)["dt"] for i in range(len(runs))],
                     "steps": steps}
        sims[name] = sim
        print(f"# convergence: {name} scan {out[name]['ms_whole_scan']:.1f} ms", file=sys.stderr, flush=True)
    finest = sims["dual"].particles(len(runs) - 1)
    gam = np.sqrt(1 + finest["ux"] ** 2 + finest["uy"] ** 2 + finest["uz"] ** 2)
    cut = float(np.percentile(gam, 99))
    out["gamma_cut"] = cut
    for name, sim in sims.items():
        rows = []
        for i, r in enumerate(runs):
            d = sim.divergence(cut, i)
            # cost of the run alone: its share of the batch, by particle-steps
            rows.append({"rms_theta_x": d["rms_x"], "rms_theta_y": d["rms_y"], "count": d["count"],
                         "particle_steps": int(sim.info(i)["n_particles"]) * nsteps[name][i]})
        tot = sum(x["particle_steps"] for x in rows)
        for x in rows:
            x["ms_share"] = out[name]["ms_whole_scan"] * x["particle_steps"] / tot
        out[name]["per_run"] = rows
        sim.close()
    return out


def stream_bandwidth(torch, dev, nbytes: int = 1 << 30, reps: int = 10) -> dict:
    """Achievable HBM bandwidth on this device (GB/s, read + write counted)
    of two streaming operations on nbytes: a device-to-device copy and an
    in-place elementwise add, each timed with events over `reps` calls after
    two untimed ones.  Measured after the timed region, beside the published
    peak the roofline is priced against."""
    x = torch.empty(nbytes // 4, dtype=torch.float32, device=dev).fill_(1.0)
    y = torch.empty_like(x)
    s = torch.cuda.current_stream(dev)

    def timed(op):
        for _ in range(2):
            op()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(s)
        for _ in range(reps):
            op()
        e1.record(s)
        torch.cuda.synchronize()
        return 2.0 * nbytes * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9

    bw = {"device_copy": timed(lambda: y.copy_(x)), "elementwise_add": timed(lambda: x.add_(1.0))}
    del x, y
    torch.cuda.empty_cache()
    return bw


def bench_dla(args, torch, pic) -> int:
    """Electrons of the App. A recipe (injection over 200 / omega_p, model
    parameters of App. A) integrated to t = 400 / omega_p with h = 0.01 /
    omega_p; one bench step is one integration of the whole ensemble from the
    injected state; value = electron-steps/s (Runge-Kutta steps)."""
    import numpy as np

    A = workloads.DLA_APP_A
    n, t_end, h = args.electrons, 400.0, 0.01
    K = args.steps if args.steps is not None else 3
    W = args.warmup if args.warmup is not None else 1
    d = workloads.dla_injection(n, workloads.SEED_BASE + 90, R=A["R"], vg=A["vg"], t_inject=A["t_inject"])
    names = ("t0", "x", "zeta", "xd", "zetad")
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    pristine = {k: torch.tensor(d[k], dtype=torch.float64, device=dev) for k in names}
    work = {k: torch.empty_like(v) for k, v in pristine.items()}
    steps_per_electron = np.maximum(0.0, np.ceil((t_end - d["t0"]) / h))
    total_steps = float(steps_per_electron.sum())
    model = {k: A[k] for k in ("a0", "kz", "vphi")}
    stream = torch.cuda.current_stream(dev)

    def once(timed):
        for k in names:
            work[k].copy_(pristine[k])
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        pic.dla_integrate(*[work[k] for k in names], t_end, h, **model)
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1)

    for _ in range(W):
        once(False)
    print(f"# dla warmup {W} done", file=sys.stderr, flush=True)
    ms = [once(True) for _ in range(K)]
    avg = sum(ms) / K
    g = 1.0 / torch.sqrt(-work["zetad"] * (2.0 + work["zetad"]) - work["xd"] ** 2)
    finite = bool(torch.isfinite(g).all().item())
    ach = DLA_FLOPS_PER_STEP * total_steps / (avg * 1e-3) / 1e12
    out = {
        "metric": "electron-steps/s (reduced model of Eq. (8), fifth-order Runge-Kutta)",
        "value": total_steps / (avg * 1e-3), "unit": "electron-steps/s", "n_gpus": 1, "steps": K, "warmup": W,
        "ms_per_step": avg, "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"dla: {n} electrons injected as in App. A over 200/omega_p, integrated to "
                               f"t = {t_end:g}/omega_p with h = {h:g}/omega_p",
                   "model": "a0 2.8, k_z 12.14 omega_p/c, v_phi 1.002565 c, R 3 c/omega_p (App. A)",
                   "electrons": n, "rk_steps": total_steps},
        "roofline": {"bound": "alu", "kernel": "dla", "achieved": ach, "peak": FP64_VECTOR_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": ach / FP64_VECTOR_PEAK_TFLOPS, "traffic": None,
                     "flops_per_step": DLA_FLOPS_PER_STEP, "avg_launch_ms": avg},
        "state_finite": finite, "max_gamma": float(g.max().item()),
    }
    if args.cpu_baseline:
        from oracle import dla

        print("# cpu baseline (oracle) ...", file=sys.stderr, flush=True)
        m = 4096
        y0 = np.stack([d[k][:m] for k in ("x", "zeta", "xd", "zetad")])
        nst = 10000  # about 12 s of host time
        t0 = time.perf_counter()
        dla.integrate(dla.params(), np.zeros(m), y0, nst * h, h)
        el = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": m * nst / el, "unit": "electron-steps/s", "cores": 1, "kind": "oracle",
                               "sample": f"{nst} steps of {m} of the electrons (numpy, vectorised over electrons), "
                                         f"{el:.1f} s"}
    print(json.dumps(out), flush=True)
    return 0


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="timed steps (default 200; c4: each run its own count, at most --steps)")
    ap.add_argument("--warmup", type=int, default=None, help="untimed steps first (default 20; c4: 8)")
    ap.add_argument("--workload", default="c5", choices=WORKLOADS,
                    help="c1..c5: the PIC step; dla: the reduced-model ensemble of Eq. (8)")
    ap.add_argument("--electrons", type=int, default=262144, help="dla: electrons in the ensemble")
    ap.add_argument("--cpu-baseline", type=int, default=1,
                    help="1: time the oracle on the workload's bounded sample, on one core and on all host cores")
    ap.add_argument("--fp64-beside", type=int, default=None,
                    help="FP32 workloads: 1 also times the FP64 path on the same workload and reports the FP32 "
                         "result's difference from it (default on for FP32 runs)")
    ap.add_argument("--oracle-sample", default=None, help=argparse.SUPPRESS)
    ap.add_argument("--n-coef", type=int, default=16, help=argparse.SUPPRESS)
    ap.add_argument("--sort-interval", type=int, default=0)
    ap.add_argument("--tile-z", type=int, default=0, help="sort tile extent in z (0: library default)")
    ap.add_argument("--tile-r", type=int, default=0, help="sort tile extent in r (0: library default)")
    ap.add_argument("--graph", action="store_true", help="replay captured steps (per-phase timing then unavailable)")
    ap.add_argument("--window", type=int, default=0,
                    help="moving window (App. A): a move every K steps (0: the static box of the workload)")
    ap.add_argument("--window-guard", type=int, default=16, help="moving window: guard columns cleared at a move")
    ap.add_argument("--deterministic", action="store_true",
                    help="FP64 only: the deposit's sums in integers, bitwise independent of the atomics' order")
    ap.add_argument("--shape", type=int, default=1, choices=[1, 2],
                    help="particle shape order of the gather and deposit: 1 linear, 2 quadratic")
    ap.add_argument("--autotune", type=int, default=None,
                    help="1: tile and sort interval from the library's autotuner (default: on for c4 and c5)")
    ap.add_argument("--precision", type=int, default=0, choices=[0, 32, 64],
                    help="override the workload's precision (0: as defined)")
    ap.add_argument("--solver", default="dual", choices=["dual", "yee"],
                    help="field solver: dual (16 coefficients per operator) or Yee (one)")
    ap.add_argument("--current", default="filter", choices=["filter", "exact"],
                    help="charge conservation with D_B: z filter on J_r, J_phi (default) or P^-1 on J_z")
    ap.add_argument("--work-split", action="store_true",
                    help="after the timed steps, report the tracked electrons' energy gain split by mode (Eq. (16))")
    ap.add_argument("--work-compare", action="store_true",
                    help="after the timed steps, report the modal, component and corrected LWFA/DLA work estimates "
                         "of the tracked electrons (Eqs. (16), (17), (20)-(21); Sec. IV.C)")
    ap.add_argument("--convergence-scale", type=int, default=1,
                    help="--convergence: run each resolution this many times the workload's steps")
    ap.add_argument("--convergence", action="store_true",
                    help="the six-run resolution scan with the dual and the Yee solver: RMS divergence of the "
                         "energetic electrons and cost per run (Sec. IV.B); prints that table's JSON line only")
    ap.add_argument("--summarize-trace", default=None, metavar="DIR",
                    help="print the markdown table of a rocprofv3 --kernel-trace --stats csv run and exit")
    ap.add_argument("--summarize-counters", nargs=2, default=None, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="write the per-launch HBM bytes of a FETCH_SIZE and a WRITE_SIZE pass of this workload's "
                         "bench command into profiles/hbm_traffic.json (with --tile-z, --tile-r, --sort-interval, "
                         "--precision as the bench line ran) and exit")
    args = ap.parse_args(argv)
    if args.summarize_trace:
        print(summarize_trace(args.summarize_trace))
        return 0
    if args.summarize_counters:
        prec = args.precision or workloads.config(args.workload)["precision"]
        e = summarize_counters(args.workload, *args.summarize_counters, "%dx%d" % (args.tile_z, args.tile_r),
                               args.sort_interval, prec)
        print(json.dumps(e, indent=1))
        return 0
    if args.oracle_sample:  # a child process of the all-core CPU baseline: no GPU is touched
        tot, el = _oracle_sample(args.oracle_sample, args.n_coef, args.shape)
        print(json.dumps({"particle_steps": tot, "seconds": el}), flush=True)
        return 0
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only (--gpus 1); the multi-GPU sharding of "
                                   "the path is a design, not built"}), flush=True)
        return 2

    import torch

    import paper_2303_12874_amd as pic

    if args.workload == "dla":
        return bench_dla(args, torch, pic)
    if args.convergence:
        dev = torch.device("cuda:0")
        torch.cuda.set_device(dev)
        print(json.dumps({"convergence_scan": convergence_scan(pic, torch, dev, args)}), flush=True)
        return 0
    cfg = workloads.config(args.workload)
    runs = cfg["runs"]
    multi = len(runs) > 1
    K = args.steps if args.steps is not None else (max(cfg["steps"]) if multi else 200)
    W = args.warmup if args.warmup is not None else (8 if multi else 20)
    per_run = [min(n, K) for n in cfg["steps"]] if multi else [K]
    prec = args.precision or cfg["precision"]
    if args.deterministic and prec != 64:
        print("--deterministic needs FP64 (--precision 64 for an FP32 workload)", file=sys.stderr)
        return 2
    solver = pic.SOLVER_YEE if args.solver == "yee" else pic.SOLVER_DUAL
    n_coef = 1 if args.solver == "yee" else 16
    current = pic.CURRENT_EXACT_JZ if args.current == "exact" else pic.CURRENT_FILTER
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    tune = None
    if args.autotune if args.autotune is not None else args.workload in ("c4", "c5"):
        t0 = time.perf_counter()
        tune = pic.autotune([workloads.to_rundesc(r) for r in runs], precision=prec, solver=solver, n_coef=n_coef,
                            current=current, tile_z=args.tile_z,
                            tile_r=args.tile_r, shape=args.shape, deterministic=args.deterministic,
                            device="cuda:0")
        torch.cuda.empty_cache()
        args.tile_z, args.tile_r = tune["tile_z"], tune["tile_r"]
        args.sort_interval = args.sort_interval or tune["sort_interval"]
        tune["seconds"] = time.perf_counter() - t0
        print(f"# autotune {tune['seconds']:.1f} s: tile {args.tile_z}x{args.tile_r}, sort every "
              f"{args.sort_interval}; {tune['candidates']}", file=sys.stderr, flush=True)
    sort_k = args.sort_interval or 8

    def timed(prec_, tile_z, tile_r, sort_interval):
        """Build the job (multi-run jobs warm up on a context of their own, so
        that the timed job starts at step 0), take W untimed steps (single
        run), then time K steps with HIP events on the library's stream."""
        def make(limits):
            return pic.Simulation([workloads.to_rundesc(r, n_steps=n) for r, n in zip(runs, limits)],
                                  precision=prec_, solver=solver, n_coef=n_coef, sort_interval=sort_interval,
                                  tile_z=tile_z, tile_r=tile_r, use_graph=args.graph, current=current,
                                  window_interval=args.window, window_guard=args.window_guard if args.window else 0,
                                  shape=args.shape, deterministic=args.deterministic, device="cuda:0")

        if multi:
            warm = make([0] * len(runs))
            warm.step(W)
            torch.cuda.synchronize()
            warm.close()
            del warm
            torch.cuda.empty_cache()
        t_init = time.perf_counter()
        sim_ = make(per_run if multi else [0])
        torch.cuda.synchronize()
        t_init = time.perf_counter() - t_init
        infos_ = [sim_.info(i) for i in range(len(runs))]
        print(f"# fp{prec_} init {t_init:.1f} s, {sum(i['n_particles'] for i in infos_)} electrons in {len(runs)} "
              f"run(s), dt {[round(i['dt'], 5) for i in infos_]}", file=sys.stderr, flush=True)
        if not multi:
            sim_.step(W)
            torch.cuda.synchronize()
        print(f"# fp{prec_} warmup {W} steps done", file=sys.stderr, flush=True)
        sim_.profile(True)
        stream = torch.cuda.current_stream(dev)
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        ev0.record(stream)
        sim_.step(K)
        ev1.record(stream)
        torch.cuda.synchronize()
        ms_ = ev0.elapsed_time(ev1)
        phases_ = sim_.profile_read()
        sim_.profile(False)
        print(f"# fp{prec_} timed {K} steps: {ms_:.2f} ms", file=sys.stderr, flush=True)
        return sim_, ms_, phases_, infos_

    sim, elapsed_ms, phases, infos = timed(prec, args.tile_z, args.tile_r, args.sort_interval)
    nps = [inf["n_particles"] for inf in infos]

    # sanity of the state after the run (FP64 reductions)
    finite = True
    for i in range(len(runs)):
        mw = sim.mode_work(i)
        finite = finite and all(map(lambda v: v == v, list(mw["field_energy"]) + [mw["kinetic"]]))

    # algorithmic bytes of each phase over the timed region, summed over the runs
    first = 0 if multi else W

    def phase_bytes(ph):
        tot = 0
        for run, n in zip(runs, per_run):
            ab = algorithmic_bytes(run, prec)
            sorts = sum(1 for st in range(first, first + n) if st > 0 and st % sort_k == 0)
            if ph == "sort":
                tot += sorts * ab["sort"]
            elif ph == "step":
                tot += sorts * ab["sort"] + n * (ab["push"] + ab["efield"] + ab["bfield"])
            else:
                tot += n * ab[ph]
        return tot

    kernels = {}
    for ph, (ms, n) in phases.items():
        if n == 0:
            continue
        kernels[ph] = {"avg_ms": ms / n, "launches": n, "GBs": phase_bytes(ph) / (ms * 1e-3) / 1e9}
    dom = max(kernels, key=lambda k: kernels[k]["avg_ms"] * kernels[k]["launches"])
    ach = kernels[dom]["GBs"]
    traffic = (measured_traffic(args.workload, dom, "%dx%d" % infos[0]["tile"], sort_k, prec)
               if args.solver == "dual" and args.current == "filter" and not args.window and args.shape == 1
               and not args.deterministic else None)  # the counters' settings
    particle_steps = sum(n * s for n, s in zip(nps, per_run))
    value = particle_steps / (elapsed_ms * 1e-3)
    run = runs[0]
    config = {"workload": f"{args.workload}: {cfg['desc']}",
              "grid": ", ".join(f"{r['Nz']}x{r['Nr']}" for r in runs), "modes": run["M"] + 1,
              "ppc": run["ppc"], "electrons": sum(nps), "precision": f"fp{prec}",
              "solver": "Yee, one coefficient per operator" if args.solver == "yee"
              else "dual, 16 coefficients per operator",
              "current": "P^-1 on J_z" if args.current == "exact" else "z filter on J_r, J_phi",
              "dt": [i["dt"] for i in infos] if multi else infos[0]["dt"],
              "sort_interval": sort_k, "tile": "%dx%d" % infos[0]["tile"], "graph": bool(args.graph),
              "shape": "quadratic" if args.shape == 2 else "linear", "deterministic": bool(args.deterministic)}
    if multi:
        config["steps_per_run"] = per_run
    if args.window:
        # electrons counted at the start of the timed region (the count varies by the fresh columns' share)
        config["window"] = {"interval": args.window, "guard": args.window_guard,
                            "cells_moved": [sim.info(i)["window_cells"] for i in range(len(runs))],
                            "electrons_after": sum(sim.info(i)["n_particles"] for i in range(len(runs)))}
    if tune is not None:
        config["autotune"] = {"seconds": round(tune["seconds"], 1),
                              "candidates": [list(c[:3]) + [round(c[3], 4)] for c in tune["candidates"]]}
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": elapsed_ms / K,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec == 64 else "f32",
        "data": "synthetic",
        "config": config,
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": ach / HBM_PEAK_GBS, "traffic": traffic,
                     "bytes_per_launch": phase_bytes(dom) / kernels[dom]["launches"],
                     "avg_launch_ms": kernels[dom]["avg_ms"]},
        "kernels": kernels,
        "state_finite": finite,
    }
    if args.work_split:
        out["work_split"] = work_split(sim, run["M"])
    if args.work_compare:
        out["work_compare"] = work_compare(sim, run)
    if args.fp64_beside if args.fp64_beside is not None else prec == 32:
        # the plain FP64 path on the same workload (library default tile and
        # sort interval), timed the same way, after the FP32 timed region; then
        # the FP32 state's difference from the FP64 state after the same steps
        sim64, ms64, ph64, inf64 = timed(64, 0, 0, 0)
        v64 = particle_steps / (ms64 * 1e-3)
        out["fp64"] = {"value": v64, "unit": "particle-steps/s", "ms_per_step": ms64 / K,
                       "tile": "%dx%d" % inf64[0]["tile"], "sort_interval": 8,
                       "kernels": {ph: {"avg_ms": ms / n, "launches": n} for ph, (ms, n) in ph64.items() if n}}
        out["fp32_over_fp64"] = value / v64
        out["fp32_error"] = {"vs_fp64_gpu": fp32_vs_fp64(pic, sim, sim64, runs[0]),
                             "stated_bounds_vs_fp64_oracle": FP32_BOUNDS}
        sim64.close()
        del sim64
    sim.close()
    del sim
    torch.cuda.empty_cache()
    bw = stream_bandwidth(torch, dev)
    peak = max(bw.values())  # the faster of a 1 GiB device copy and an in-place add on this GPU
    out["roofline"]["measured_peak"] = peak
    out["roofline"]["measured_peak_by"] = bw
    out["roofline"]["frac_of_measured_peak"] = ach / peak
    if args.cpu_baseline:
        print("# cpu baseline (oracle) ...", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(args.workload, n_coef, shape=args.shape)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
