"""The oracle's per-track digests and decision margins, and the full-size
parity helpers built on them (oracle/parity.py)."""
import numpy as np

import workloads as W

FNV_BASIS = 14695981039346656037
FNV_PRIME = 1099511628211


def fnv1a_records(rec):
    """64-bit FNV-1a over the little-endian int32 bytes of (touchable, code) pairs."""
    h = FNV_BASIS
    for t, c in zip(rec["touchable"], rec["code"]):
        for x in (int(t), int(c)):
            for b in (x & 0xFFFFFFFF).to_bytes(4, "little"):
                h ^= b
                h = (h * FNV_PRIME) & 0xFFFFFFFFFFFFFFFF
    return h


def test_digest_matches_log(oracle_lib):
    geoms, prim, _ = W.barrel(n=300, seed=4)
    og = oracle_lib.Geometry(geoms[0])
    r = og.transport(prim, seed=2, log_cap=4096, want_digest=True)
    d = r["digest"]
    for s in range(3 * prim.n):
        n = int(r["log_n"][s])
        assert d["n"][s] == n and d["fate"][s] == r["log_fate"][s]
        if r["log_fate"][s] == 0:
            continue
        rec = r["log"][s, :n]
        assert int(d["hash"][s]) == fnv1a_records(rec)
        assert d["sum_step"][s] == np.sum(rec["step"]) or np.isclose(d["sum_step"][s], rec["step"].sum(),
                                                                     rtol=1e-15)
        assert np.isclose(d["sum_edep"][s], rec["edep"].sum(), rtol=1e-15, atol=0)


def test_fnv1a_known_answers():
    """Published FNV-1a 64 test values: the empty input and the single byte 'a'."""
    h = FNV_BASIS
    assert h == 0xcbf29ce484222325
    h ^= ord("a")
    h = (h * FNV_PRIME) & 0xFFFFFFFFFFFFFFFF
    assert h == 0xaf63dc4c8601ec8c


def test_margins_are_recorded_and_small_at_tolerance_edges(oracle_lib):
    desc = W.geometry.foil_stack()
    og = oracle_lib.Geometry(desc)
    n = 20
    pos = np.stack([np.zeros(n), np.linspace(-5, 5, n), np.full(n, -50.0)], 1)
    prim = W.primaries.one_per_event(pos, np.tile([0, 0, 1.0], (n, 1)), np.ones(n))
    r = og.transport(prim, seed=0, log_cap=64, want_margins=True)
    m = r["margin"]
    assert np.all(m[0::3, :26] >= 0)
    # every zero step compares a step shorter than 1e-9 mm with the tolerance 1e-9 mm,
    # so its margin is below 1e-9 / 100 mm (the world's extent)
    assert np.all(m[0::3, 1:26] <= 1e-11)
    plain = og.transport(prim, seed=0, log_cap=64)
    assert np.array_equal(plain["log"], r["log"])  # margins change nothing
    # a pencil beam entering a slab head-on: the first step (vacuum to the slab face,
    # 475 mm, against the world exit at 1500 mm) is decided far from any edge
    og = oracle_lib.Geometry(W.geometry.slab("water"))
    prim = W.primaries.one_per_event(np.tile([0, 0, -500.0], (n, 1)), np.tile([0, 0, 1.0], (n, 1)), np.ones(n))
    r = og.transport(prim, seed=0, log_cap=64, want_margins=True)
    assert np.all(r["log"][0::3, 0]["code"] == 0)
    assert np.all(r["margin"][0::3, 0] > 1e-3)


def test_first_divergence_and_classification(oracle_lib):
    from oracle import parity
    geoms, prim, _ = W.calorimeter(n=200, seed=1)
    og = oracle_lib.Geometry(geoms[0])
    r = og.transport(prim, seed=0, log_cap=256, want_margins=True)
    s = int(np.argmax(r["log_n"]))
    rec = r["log"][s].copy()
    n, f = int(r["log_n"][s]), int(r["log_fate"][s])
    assert parity.first_divergence(rec, n, f, r["log"][s], n, f) == -1
    bad = rec.copy()
    bad[3]["touchable"] += 1
    assert parity.first_divergence(bad, n, f, r["log"][s], n, f) == 3
    bad = rec.copy()
    bad[2]["step"] *= 1 + 1e-6
    assert parity.first_divergence(bad, n, f, r["log"][s], n, f) == 2
    assert parity.first_divergence(rec, n - 1, f, r["log"][s], n, f) == n - 1
    ora = {s: (r["log"][s], n, f, r["margin"][s], float(r["tail_margin"][s]))}
    out = parity.classify([s], {s: (bad, n, f)}, ora)
    want = "flip" if min(r["margin"][s][2], r["margin"][s][1]) < parity.FLIP_MARGIN else "bug"
    assert out[0][1] == 2 and out[0][3] == want


def test_worker_split_equals_one_process(oracle_lib):
    from oracle import parity
    geoms, prim, _ = W.calorimeter(n=3000, seed=2)
    a = parity.oracle_run(geoms[0], prim, workers=1)
    b = parity.oracle_run(geoms[0], prim, workers=3)
    assert np.array_equal(a["digest"], b["digest"])
    assert a["counters"] == b["counters"]
    assert np.allclose(a["edep_event"], b["edep_event"], rtol=1e-14, atol=0)
    assert np.allclose(a["edep_touchable"], b["edep_touchable"], rtol=1e-12, atol=1e-15)
    # the digests cover every primary's slot
    assert np.all(a["digest"]["fate"][0::3] > 0)
    mism = parity.digest_mismatches(a["digest"], b["digest"])
    assert len(mism) == 0
    c = a["digest"].copy()
    i, j = np.nonzero(c["sum_step"] > 1.0)[0][:2]
    c["sum_step"][i] *= 1 + 1e-8
    c["hash"][j] ^= 1
    assert list(parity.digest_mismatches(c, a["digest"])) == [i, j]


def test_full_check_voxel_mode_against_brute_force(oracle_lib):
    """The oracle's voxel mode reaches the brute-force answers, so full_check finds
    every track equal; with a planted shift of one daughter it finds differences."""
    from oracle import parity
    geoms, prim, _ = W.barrel(n=2000, seed=6)
    desc = geoms[0]
    vox = oracle_lib.Geometry(desc)
    vox.set_voxels(True)
    r = vox.transport(prim, seed=0, want_digest=True)

    def logs(idx):
        q = vox.transport(prim.subset(idx), seed=0, log_cap=4096, n_events=prim.n_events)
        return q["log"], q["log_n"], q["log_fate"]

    res = parity.full_check(desc, prim, r["digest"], logs, gpu_tally=r, workers=2)
    assert res["tracks"] > 2000 and res["mismatches"] == 0 and res["bugs"] == 0
    assert res["counters_equal"] and res["max_rel_event_deposit"] <= 1e-12
    # a layer moved sideways by 1 um (inside its vacuum gap): tracks crossing it differ
    # by far more than rounding
    moved = W.geometry.barrel()
    env = int(np.nonzero(moved.lv_dau_cnt == 64)[0][0])  # the envelope holds the 64 layers
    moved.pv_trans[int(moved.lv_dau_off[env]) + 31] += np.array([1e-3, 0.0, 0.0])
    other = oracle_lib.Geometry(moved)
    q = other.transport(prim, seed=0, want_digest=True)

    def logs2(idx):
        z = other.transport(prim.subset(idx), seed=0, log_cap=4096, n_events=prim.n_events)
        return z["log"], z["log_n"], z["log_fate"]

    res = parity.full_check(desc, prim, q["digest"], logs2, workers=2)
    assert res["mismatches"] > 0 and res["bugs"] > 0
