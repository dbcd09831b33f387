"""GPU: FP32-distance navigation against the FP64 oracle.

Screened form: every step, limiter and next touchable equals the FP64 result
(the FP32 arithmetic only ranks candidates and proves skips), so transports
match the oracle per track exactly as the FP64 path does.

Pure form: steps come from FP32 distances.  Per-query errors against the
oracle, the rate of identical per-track volume sequences and a chi-square
comparison of deposit histograms are measured and bounded.
"""
import numpy as np
import pytest

import workloads as W
from tests.gpu_common import (ATOL, EXACT, GEOMS, RTOL, compare_logs, ctx, geom,  # noqa: F401
                               print_case, run_transport, sample_points, surface_points, torch_dev)

pytestmark = pytest.mark.gpu

SCREENED, PURE = 1, 2


def step_queries(desc, og, seed):
    rng = np.random.Generator(np.random.Philox(key=seed))
    pts = sample_points(desc, rng, 20000)
    dirs = W.primaries.isotropic(rng, 20000)
    end, d2, nxt = surface_points(desc, og, rng, 6000)
    keep = nxt >= 0
    pts = np.concatenate([pts, end[keep]])
    dirs = np.concatenate([dirs, d2[keep]])
    T = og.locate(pts, dirs)
    ok = T >= 0
    return pts[ok], dirs[ok], T[ok]


@pytest.mark.parametrize("name", list(GEOMS))
def test_screened_step_equals_fp64(ctx, torch_dev, oracle_lib, name):
    torch = torch_dev
    desc, gid, nt, og = geom(ctx, name, oracle_lib)
    print_case("fp32_screened_step", name)
    pts, dirs, T = step_queries(desc, og, 2002)
    s_ref, l_ref, n_ref = og.compute_step(pts, dirs, T)
    args = (gid, torch.from_numpy(pts).cuda(), torch.from_numpy(dirs).cuda(),
            torch.from_numpy(T.astype(np.int32)).cuda())
    s, l, nx, saf = (a.cpu().numpy() for a in ctx.compute_step(*args, precision=SCREENED,
                                                                 with_safety=True))
    s64, l64, _, saf64 = (a.cpu().numpy() for a in ctx.compute_step(*args, precision=0,
                                                                       with_safety=True))
    assert np.array_equal(l, l_ref)
    assert np.array_equal(nx, n_ref)
    assert np.allclose(s, s_ref, rtol=RTOL, atol=ATOL)
    # bitwise equal to the library's own FP64 path
    assert np.array_equal(s.view(np.uint64), s64.view(np.uint64))
    assert np.array_equal(l, l64)
    # the screened safety is the FP64 one lowered by the FP32 rounding margin at most
    assert np.all(saf >= 0) and np.all(saf <= saf64 + 1e-12)
    # (the lowering is 2^-18 of the local coordinate and parameter magnitudes: < 0.1 mm here)
    assert np.all(saf >= saf64 - 0.1)


@pytest.mark.parametrize("name,n,cap", [("tiny", 10000, 64), ("calorimeter", 4000, 400),
                                        ("barrel", 3000, 512), ("endcap", 4000, 256)])
def test_screened_transport_matches_oracle(ctx, torch_dev, oracle_lib, name, n, cap):
    torch = torch_dev
    desc, gid, nt, og = geom(ctx, name, oracle_lib)
    print_case("fp32_screened_transport", name, n)
    _, prim, _ = W.WORKLOADS[name](n=n)
    got = run_transport(ctx, torch, gid, prim, cap, precision=SCREENED, count_work=True)
    ref = og.transport(prim, seed=0, log_cap=cap)
    bad = compare_logs(got["log"], got["log_n"], got["log_fate"], ref, cap)
    assert not bad, bad[:10]
    for k in EXACT:
        assert got["counters"][k] == ref["counters"][k], k
    assert np.allclose(got["edep_event"], ref["edep_event"], rtol=RTOL, atol=1e-15)
    assert np.allclose(got["edep_touchable"], ref["edep_touchable"], rtol=RTOL, atol=1e-12)
    # nodes with fewer than six candidates are walked in FP64 (every node of the
    # calorimeter and of the barrel's shape-aware grids); the tiny world's eight
    # daughters (no grid) are screened in FP32
    if name == "tiny":
        assert got["counters"]["dist_in_f32"] > 0


def test_screened_transport_bbox_lists_matches_oracle(ctx, torch_dev, oracle_lib):
    """Bounding-box node lists hold many candidates, so nearly every daughter
    search is screened in FP32: per-track parity with the oracle still holds."""
    torch = torch_dev
    desc = W.geometry.barrel(seed=1)
    gid, _ = ctx.upload_geometry(desc, voxel_lists=1)
    og = oracle_lib.Geometry(desc)
    print_case("fp32_screened_transport_bbox_lists")
    _, prim, _ = W.barrel(n=2000)
    got = run_transport(ctx, torch, gid, prim, 512, precision=SCREENED, count_work=True)
    ref = og.transport(prim, seed=0, log_cap=512)
    bad = compare_logs(got["log"], got["log_n"], got["log_fate"], ref, 512)
    assert not bad, bad[:10]
    for k in EXACT:
        assert got["counters"][k] == ref["counters"][k], k
    assert np.allclose(got["edep_event"], ref["edep_event"], rtol=RTOL, atol=1e-15)
    assert got["counters"]["dist_in_f32"] > 5 * got["counters"]["dist_in"]


def query_error_stats(s, l, s_ref, l_ref):
    fin = np.isfinite(s_ref) & np.isfinite(s)
    err = np.abs(s[fin] - s_ref[fin])
    rel = err / np.maximum(s_ref[fin], 1.0)
    return dict(limiter_agree=float(np.mean(l == l_ref)), n=int(fin.sum()),
                abs_median=float(np.median(err)), abs_p99=float(np.quantile(err, 0.99)),
                rel_p99=float(np.quantile(rel, 0.99)), rel_max=float(rel.max()))


@pytest.mark.parametrize("name", list(GEOMS))
def test_pure_per_query_error(ctx, torch_dev, oracle_lib, name):
    torch = torch_dev
    desc, gid, nt, og = geom(ctx, name, oracle_lib)
    print_case("fp32_pure_step", name)
    pts, dirs, T = step_queries(desc, og, 2003)
    s_ref, l_ref, _ = og.compute_step(pts, dirs, T)
    out = ctx.compute_step(gid, torch.from_numpy(pts).cuda(), torch.from_numpy(dirs).cuda(),
                           torch.from_numpy(T.astype(np.int32)).cuda(), precision=PURE)
    s, l = out[0].cpu().numpy(), out[1].cpu().numpy()
    st = query_error_stats(s, l, s_ref, l_ref)
    print("per-query FP32 error", name, st, flush=True)
    # FP32 carries ~7 significant digits of coordinates up to a few metres
    assert st["limiter_agree"] > 0.99
    assert st["abs_median"] < 1e-3
    assert st["rel_p99"] < 1e-3


def chi2_per_ndf(a, b):
    m = (a + b) > 0
    return float(np.sum((a[m] - b[m]) ** 2 / (a[m] + b[m])) / max(int(m.sum()) - 1, 1))


def test_pure_transport_barrel_deposits(ctx, torch_dev, oracle_lib):
    """Pure FP32 on the barrel: energy conserved per event, most tracks follow
    identical volume sequences, deposit histograms agree (chi-square)."""
    torch = torch_dev
    desc, gid, nt, og = geom(ctx, "barrel", oracle_lib)
    print_case("fp32_pure_transport")
    _, prim, _ = W.barrel(n=20000)
    cap = 512
    a = run_transport(ctx, torch, gid, prim, cap)
    b = run_transport(ctx, torch, gid, prim, cap, precision=PURE)
    tot = b["edep_event"] + b["escaped_event"]
    assert np.allclose(tot, prim.energy, rtol=1e-12, atol=0)
    used = a["log_fate"] != 0

    def sequences(r, slot, drop_zero):
        k = min(int(r["log_n"][slot]), cap)
        rec = r["log"][slot, :k]
        keep = np.ones(k, bool)
        if drop_zero:
            # geometry-limited steps shorter than the FP32 surface band
            keep = ~((rec["code"] >= -1) & (rec["step"] < 2e-3))
        return rec["touchable"][keep], rec["code"][keep], r["log_fate"][slot]

    def identity(drop_zero):
        same = 0
        for slot in np.nonzero(used)[0]:
            ta, ca, fa = sequences(a, slot, drop_zero)
            tb, cb, fb = sequences(b, slot, drop_zero)
            same += int(fa == fb and np.array_equal(ta, tb) and np.array_equal(ca, cb))
        return same / int(used.sum())

    ident_raw, ident = identity(False), identity(True)
    bins = np.logspace(-3, np.log10(25.0), 41)
    ha = np.histogram(a["edep_event"], bins)[0].astype(float)
    hb = np.histogram(b["edep_event"], bins)[0].astype(float)
    c_ev = chi2_per_ndf(ha, hb)
    # deposits per layer touchable class: sum over touchables of each LV
    t_parent, t_pv, t_lv, _ = ctx.touchables(gid)
    la = np.bincount(t_lv, weights=a["edep_touchable"], minlength=desc.n_lv)
    lb = np.bincount(t_lv, weights=b["edep_touchable"], minlength=desc.n_lv)
    rel_lv = np.abs(la - lb).sum() / la.sum()
    print("pure FP32 barrel: identical volume sequences", ident_raw, "without zero-length crossings",
          ident, "chi2/ndf(event deposits)", c_ev,
          "L1 rel diff of per-LV deposits", rel_lv, "pushes", b["counters"]["pushes"],
          "stuck", b["counters"]["stuck"], flush=True)
    # Pure FP32 can stop short of a face shared by two volumes by less than
    # the FP32 surface band; the FP64 relocation then leaves the track in the
    # mother for one zero-length step before it enters the neighbour.  Those
    # steps aside, volume sequences agree for nearly every track.
    assert ident > 0.95
    assert c_ev < 2.0
    assert rel_lv < 0.02
    assert b["counters"]["stuck"] <= 1e-4 * prim.n + 1


def test_pure_transport_calorimeter_conserves_energy(ctx, torch_dev, oracle_lib):
    """Pure FP32 on the calorimeter (the axis-aligned box build's FP32 instantiation):
    energy conserved per event, nearly every track follows the FP64 volume sequence."""
    torch = torch_dev
    desc, gid, nt, og = geom(ctx, "calorimeter", oracle_lib)
    print_case("fp32_pure_calorimeter")
    _, prim, _ = W.calorimeter(n=4000)
    cap = 400
    a = run_transport(ctx, torch, gid, prim, cap)
    b = run_transport(ctx, torch, gid, prim, cap, precision=PURE)
    tot = b["edep_event"] + b["escaped_event"]
    assert np.allclose(tot, prim.energy, rtol=1e-12, atol=0)
    assert b["counters"]["stuck"] == 0
    used = np.nonzero(a["log_fate"] != 0)[0]
    same = 0
    for slot in used:
        ka, kb = min(int(a["log_n"][slot]), cap), min(int(b["log_n"][slot]), cap)
        ta, tb = a["log"][slot, :ka], b["log"][slot, :kb]
        same += int(a["log_fate"][slot] == b["log_fate"][slot] and
                    np.array_equal(ta["touchable"], tb["touchable"]) and np.array_equal(ta["code"], tb["code"]))
    ident = same / len(used)
    print("pure FP32 calorimeter: identical volume sequences", ident, flush=True)
    assert ident > 0.95
