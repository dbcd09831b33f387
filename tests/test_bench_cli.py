"""bench.py's command line on the CPU: the one-GPU rule, section names, and the
host-side helpers that need no GPU."""
import json
import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args],
                          capture_output=True, text=True, timeout=120)


def test_more_than_one_gpu_is_refused():
    r = _run("--gpus", "2")
    assert r.returncode == 2 and "one GPU" in r.stderr


def test_unknown_section_is_refused():
    r = _run("--sections", "headline,nonsense")
    assert r.returncode != 0 and "nonsense" in r.stderr


def test_algorithmic_flops_counts_each_unit():
    sys.path.insert(0, ROOT)
    import bench
    zero = {k: 0 for k in ("steps", "shortcuts", "dist_out", "dist_in", "inside", "voxel_nodes",
                           "tracks", "compton", "pe", "pair")}
    assert bench.algorithmic_flops(zero) == 0
    one_step = dict(zero, steps=1)
    # a geometry-limited step: bookkeeping, frame and mother safety
    assert bench.algorithmic_flops(one_step) == bench.FLOPS["step"] + bench.FLOPS["frame"] + bench.FLOPS["safety"]
    shortcut = dict(zero, steps=1, shortcuts=1)
    assert bench.algorithmic_flops(shortcut) == bench.FLOPS["step"]


def test_stored_traffic_is_tied_to_the_kernel_sources():
    sys.path.insert(0, ROOT)
    import bench
    path = os.path.join(ROOT, "profiles", "k_transport_calorimeter_1e6_traffic.json")
    with open(path) as f:
        t = json.load(f)
    assert t["bytes_per_launch"] > 0
    # another kernel name never picks up the stored figure
    assert bench.stored_traffic("gnav::pool128::k_transport<false, false, 0, 0>") is None
    if t["kernel_source_hash"] == bench.kernel_source_hash():
        assert np.isclose(bench.stored_traffic(t["kernel"]), t["bytes_per_launch"])
    else:
        assert bench.stored_traffic(t["kernel"]) is None


def test_oracle_rates_both_modes_on_a_small_sample():
    sys.path.insert(0, ROOT)
    import bench
    import workloads as W
    geoms, prim, _ = W.tiny(n=300)
    r = bench.oracle_rates(geoms[0], prim, 200)
    assert r["brute_force"] > 0 and r["voxel"] > 0 and "200" in r["sample"]
