"""CPU checks of the benchmark's contract pieces (no GPU): the refusal of more
than one GPU, the algorithmic bytes the roofline is priced with, the lookup of
the measured HBM traffic, and the CPU-baseline sample sizes."""
import hashlib
import json
import os

import pytest

import bench
import workloads

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused(capsys):
    assert bench.main(["--gpus", "2"]) == 2
    out = json.loads(capsys.readouterr().out.strip().splitlines()[-1])
    assert "one GPU" in out["error"]


def test_algorithmic_bytes_of_the_headline_run():
    """4096 x 256, modes 0..2, 8 ppc, FP64: per electron 7 words + id read and
    6 words written; per node E and Bbar read and J written (9 NM words)."""
    run = workloads.config("c2")["runs"][0]
    ab = bench.algorithmic_bytes(run, 64)
    n_e = 4096 * 255 * 8
    nodes = 4096 * 257
    assert ab["push"] == n_e * (7 * 8 + 4 + 6 * 8) + nodes * 9 * 5 * 8
    assert ab["efield"] == nodes * 15 * 5 * 8 and ab["bfield"] == nodes * 12 * 5 * 8
    assert abs(ab["push"] / 1.2814e9 - 1) < 1e-3  # the figure the design notes quote
    ab32 = bench.algorithmic_bytes(workloads.config("c5")["runs"][0], 32)
    assert abs(ab32["push"] / 5.3456e9 - 1) < 1e-3


def test_measured_traffic_only_for_the_profiled_build_and_settings():
    t = json.load(open(os.path.join(ROOT, "profiles", "hbm_traffic.json")))
    sha = hashlib.sha256(open(os.path.join(ROOT, "paper_2303_12874_amd", "csrc", "kernels.hip"), "rb").read()).hexdigest()
    w = t["workloads"]["c2"]
    st = w["settings"]
    got = bench.measured_traffic("c2", "push", st["tile"], st["sort_interval"], st["precision"])
    if t["kernels_sha256"] == sha:
        assert got == pytest.approx(w["push"]["read_bytes"] + w["push"]["write_bytes"])
    else:
        assert got is None  # kernels changed since the counters were taken
    assert bench.measured_traffic("c2", "push", "8x2", st["sort_interval"], st["precision"]) is None
    assert bench.measured_traffic("c2", "push", st["tile"], st["sort_interval"], 32) is None


def test_cpu_baseline_sample_covers_every_pic_workload():
    """Every PIC workload has a bounded oracle sample; the 67 M-electron run's
    is a slab of the same physics (radius, modes, ppc, density, pulses)."""
    for name in bench.WORKLOADS:
        if name == "dla":
            continue
        smp = workloads.cpu_sample(name)
        assert smp["steps"] >= 1 and smp["runs"]
    full, slab = workloads.config("c5")["runs"][0], workloads.cpu_sample("c5")["runs"][0]
    assert slab["Nz"] == 512 and slab["Nz"] < full["Nz"]
    for k in ("Nr", "M", "ppc", "dz", "dr", "n0", "seed", "taper"):
        assert slab[k] == full[k], k
    assert len(slab["pulses"]) == 2
    for p in slab["pulses"]:
        assert 0 < p["zc"] < slab["Nz"] * slab["dz"]


def test_cpu_baseline_all_cores_leg():
    """The all-core leg runs one oracle process per core on the same sample
    and sums their particle-steps (here on the smallest workload)."""
    out = bench.cpu_baseline("c1", max_procs=2)
    assert out["cores"] == 1 and out["kind"] == "oracle" and out["value"] > 0
    ac = out["all_cores"]
    assert ac["kind"] == "oracle" and ac["value"] > 0 and 1 <= ac["cores"] <= 2
    assert out["cpu"] == ac["cpu"]

