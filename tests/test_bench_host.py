"""Host-side checks of bench.py and the committed measurement records (no GPU)."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def _run(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], capture_output=True, text=True,
                          timeout=600, cwd=ROOT)


def test_more_than_one_gpu_is_refused():
    r = _run("--gpus", "2")
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_rank_environment_is_refused():
    env = dict(os.environ, WORLD_SIZE="2")
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py")], capture_output=True, text=True,
                       timeout=600, cwd=ROOT, env=env)
    assert r.returncode == 2


def test_no_gpu_is_an_error_not_a_fallback():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    r = _run("--steps", "1", "--warmup", "0")
    assert r.returncode == 2
    assert "needs a GPU" in r.stderr


@pytest.mark.parametrize("wl", ["fan2d_512", "cone_helical_512x256"])
@pytest.mark.parametrize("cls", ["backproject", "project", "update"])
def test_traffic_records_are_complete(cls, wl):
    import bench
    path = os.path.join(ROOT, "profiles", "traffic_%s_%s.json" % (cls, wl))
    rec = json.load(open(path))
    assert rec["kernel_class"] == cls and rec["workload"] == wl
    assert abs(rec["hbm_bytes_per_launch"] - rec["hbm_read_bytes_per_launch"] - rec["hbm_write_bytes_per_launch"]) <= 1
    assert rec["hbm_bytes_per_launch"] > 0
    assert all("rocprofv3 --pmc" in c for c in rec["commands"])
    cp = rec["copy_probe"]
    # the scale factors come from a plain copy of known size: about 2 for
    # FETCH_SIZE (it counts half of the bytes read) and 1 for WRITE_SIZE
    assert 1.9 < cp["fetch_scale"] < 2.1 and 0.95 < cp["write_scale"] < 1.05
    assert len(rec["source_sha256_16"]) == 16
    assert rec["source"] == bench.KERNEL_SOURCES[cls]


def test_source_hash_tracks_every_listed_file():
    import bench
    h1 = bench.source_hash(bench.KERNEL_SOURCES["update"])
    h2 = bench.source_hash(bench.KERNEL_SOURCES["update"][:-1])
    assert h1 != h2 and len(h1) == 16


def test_oracle_timing_mode_runs_without_a_gpu():
    env = dict(os.environ, OMP_NUM_THREADS="2")
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--oracle-timing", "--workload", "fan2d_128"],
                       capture_output=True, text=True, timeout=600, cwd=ROOT, env=env)
    assert r.returncode == 0, r.stderr
    rec = json.loads(r.stdout.strip().splitlines()[-1])
    assert rec["workload"] == "fan2d_128" and rec["threads"] == 2 and rec["reps"] == 5
    assert rec["subset_views"] == 45
    assert 0 < rec["fp_subset_s"] and 0 < rec["bp_subset_s"]
    assert rec["iteration_s"] == pytest.approx(4 * rec["step_s"], rel=1e-3, abs=1e-4)


@pytest.mark.parametrize("cls", ["backproject", "project", "update"])
def test_counter_records_of_the_default_workload(cls):
    """The default workload's counter records carry the L2 hit rate and the
    VALU issue use the benchmark line reports, keyed on the kernel sources."""
    import bench
    rec = json.load(open(os.path.join(ROOT, "profiles", "counters_%s_%s.json" % (cls, bench.DEFAULT_WORKLOAD))))
    assert rec["kernel_class"] == cls and rec["workload"] == bench.DEFAULT_WORKLOAD
    assert 0.0 < rec["l2_hit_rate"] < 1.0 and 0.0 < rec["valu_issue"] < 1.0
    assert rec["l2_hits"] > 0 and rec["valu_insts_per_launch"] > 0
    assert "rocprofv3 --pmc" in rec["command"] and "TCC_HIT_sum" in rec["command"]
    assert rec["source"] == bench.KERNEL_SOURCES[cls] and len(rec["source_sha256_16"]) == 16
