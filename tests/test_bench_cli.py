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


def _zero():
    sys.path.insert(0, ROOT)
    import bench
    from paper_1209_5235_amd import gnav
    return bench, {k: 0 for k in gnav.COUNTERS}


def test_algorithmic_flops_counts_each_unit():
    bench, zero = _zero()
    assert bench.algorithmic_flops(zero) == (0.0, 0.0)
    u = bench.UNIT_FLOPS
    assert bench.algorithmic_flops(dict(zero, steps=1)) == (u["step"], 0.0)
    assert bench.algorithmic_flops(dict(zero, frame_maps=3)) == (3 * u["frame"], 0.0)
    assert bench.algorithmic_flops(dict(zero, voxel_nodes=2)) == (2 * u["node"], 0.0)
    assert bench.algorithmic_flops(dict(zero, compton=1, pe=1)) == (2 * u["interaction"], 0.0)
    for fam in bench.FAMILIES:
        assert bench.algorithmic_flops(dict(zero, **{"dist_in_" + fam: 1}))[0] == u["dist_in"][fam]
        assert bench.algorithmic_flops(dict(zero, **{"dist_out_" + fam: 1}))[0] == u["dist_out"][fam]
        assert bench.algorithmic_flops(dict(zero, **{"safety_" + fam: 1}))[0] == u["safety"][fam]
        assert bench.algorithmic_flops(dict(zero, **{"inside_" + fam: 1}))[0] == u["safety"][fam]
    # a calorimeter-like step in a cell (three placement levels, box exit and safety)
    cell = dict(zero, steps=1, frame_maps=3, dist_out_box=1, safety_box=1)
    assert sum(bench.algorithmic_flops(cell)) == 3 * 33 + 15 + 8 + 10
    # FP32 forms: the FP32 share of the entry distances (and, pure, exits and safeties)
    c = dict(zero, dist_in=2, dist_in_f32=2, dist_in_tubs=4, dist_out_tubs=1, safety_tubs=1)
    f64, f32 = bench.algorithmic_flops(c, precision=1)
    assert f32 == 2 * u["dist_in"]["tubs"] and f64 == 2 * u["dist_in"]["tubs"] + 90 + 20
    f64, f32 = bench.algorithmic_flops(c, precision=2)
    assert f32 == 2 * u["dist_in"]["tubs"] + 90 + 20 and f64 == 2 * u["dist_in"]["tubs"]


def test_roofline_mixes_peaks_by_work():
    bench, zero = _zero()
    c = dict(zero, steps=10 ** 9)
    r = bench.roofline(c, 1.0, "k")
    assert r["peak"] == bench.PEAK_FP64_TFLOPS and abs(r["achieved"] - 10.0) < 1e-9
    assert r["frac"] == r["fp64_frac"] and r["traffic"] is None
    c = dict(zero, dist_in=0, dist_in_f32=1, dist_in_box=10 ** 9)
    r = bench.roofline(c, 1.0, "k", precision=1, traffic=8e9)
    assert r["peak"] == bench.PEAK_FP32_TFLOPS and r["hbm_gbs"] == 8000.0 and r["hbm_frac"] == 1.0


def test_stored_traffic_is_tied_to_kernel_workload_and_sources():
    bench, _ = _zero()
    if not os.path.exists(bench.TRAFFIC_FILE):
        assert bench.stored_traffic("any", "any") is None
        return
    with open(bench.TRAFFIC_FILE) as f:
        t = json.load(f)
    e = t["entries"][0]
    assert e["bytes_per_launch"] > 0
    assert bench.stored_traffic(e["kernel"], "another workload") is None
    assert bench.stored_traffic("gnav::pool999::k_transport", e["workload"]) is None
    if t["kernel_source_hash"] == bench.kernel_source_hash():
        assert np.isclose(bench.stored_traffic(e["kernel"], e["workload"]), e["bytes_per_launch"])
    else:
        assert bench.stored_traffic(e["kernel"], e["workload"]) is None


def test_digest_comparison_counts_mismatches():
    bench, _ = _zero()
    from paper_1209_5235_amd import gnav
    ref = np.zeros(6, gnav.DIGEST_DTYPE)
    ref["fate"][:4] = 1
    ref["sum_step"][:4] = 10.0
    got = ref.copy()
    assert bench.compare_digests(got, ref) == (0, 4)
    got["sum_step"][1] = 10.0 * (1 + 1e-10)
    assert bench.compare_digests(got, ref) == (0, 4)
    got["sum_step"][1] = 10.0 * (1 + 1e-8)
    got["hash"][2] ^= 1
    assert bench.compare_digests(got, ref) == (2, 4)


def test_oracle_rates_both_modes_on_a_small_sample():
    sys.path.insert(0, ROOT)
    import bench
    import workloads as W
    geoms, prim, _ = W.tiny(n=300)
    r = bench.oracle_rates(geoms[0], prim, 200)
    assert r["brute_force"] > 0 and r["voxel"] > 0 and "200" in r["sample"]
