"""GPU parity: the HIP library (through the C ABI) against the CPU oracle.

Touchable ids, limiters, fates and step counts must match exactly; lengths and
deposits within 1e-9 relative (plus 1e-12 mm absolute for zero-length steps).
"""
import sys

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

from tests.gpu_common import (ATOL, EXACT, GEOMS, RTOL, compare_logs, ctx, geom,  # noqa: F401
                               print_case, run_transport, sample_points, surface_points,
                               torch_dev)


@pytest.mark.parametrize("name", list(GEOMS))
def test_locate_parity(ctx, torch_dev, oracle_lib, name):
    torch = torch_dev
    desc, gid, nt, og = geom(ctx, name, oracle_lib)
    print_case("locate", name)
    rng = np.random.Generator(np.random.Philox(key=1000))
    n = 20000
    pts = sample_points(desc, rng, n)
    dirs = W.primaries.isotropic(rng, n)
    ref = og.locate(pts)
    ref_d = og.locate(pts, dirs)
    p_t = torch.from_numpy(pts).cuda()
    d_t = torch.from_numpy(dirs).cuda()
    got = ctx.locate(gid, p_t).cpu().numpy()
    got_d = ctx.locate(gid, p_t, d_t).cpu().numpy()
    assert np.array_equal(got, ref)
    assert np.array_equal(got_d, ref_d)


@pytest.mark.parametrize("name", list(GEOMS))
def test_locate_parity_on_surfaces(ctx, torch_dev, oracle_lib, name):
    torch = torch_dev
    desc, gid, nt, og = geom(ctx, name, oracle_lib)
    print_case("locate_surface", name)
    rng = np.random.Generator(np.random.Philox(key=1001))
    end, dirs, nxt = surface_points(desc, og, rng, 8000)
    new_dirs = W.primaries.isotropic(rng, len(end))
    for d in (dirs, new_dirs):
        ref = og.locate(end, d)
        got = ctx.locate(gid, torch.from_numpy(end).cuda(), torch.from_numpy(d).cuda()).cpu().numpy()
        assert np.array_equal(got, ref)


@pytest.mark.parametrize("name", list(GEOMS))
def test_compute_step_parity(ctx, torch_dev, oracle_lib, name):
    torch = torch_dev
    desc, gid, nt, og = geom(ctx, name, oracle_lib)
    print_case("step", name)
    rng = np.random.Generator(np.random.Philox(key=1002))
    n = 20000
    pts = sample_points(desc, rng, n)
    dirs = W.primaries.isotropic(rng, n)
    # include starts on surfaces (the usual case inside transport)
    end, d2, nxt = surface_points(desc, og, rng, 6000)
    keep = nxt >= 0
    pts = np.concatenate([pts, end[keep]])
    dirs = np.concatenate([dirs, d2[keep]])
    T = og.locate(pts, dirs)
    ok = T >= 0
    pts, dirs, T = pts[ok], dirs[ok], T[ok]
    s_ref, l_ref, n_ref = og.compute_step(pts, dirs, T)
    s, l, nx = ctx.compute_step(gid, torch.from_numpy(pts).cuda(), torch.from_numpy(dirs).cuda(),
                                torch.from_numpy(T.astype(np.int32)).cuda())
    s, l, nx = s.cpu().numpy(), l.cpu().numpy(), nx.cpu().numpy()
    assert np.array_equal(l, l_ref)
    assert np.allclose(s, s_ref, rtol=RTOL, atol=ATOL)
    assert np.array_equal(nx, n_ref)
    # without a given touchable the library locates first
    s2, l2, _ = ctx.compute_step(gid, torch.from_numpy(pts).cuda(), torch.from_numpy(dirs).cuda())
    assert np.array_equal(l2.cpu().numpy(), l_ref)


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("name", ["tiny_rot", "zoo", "calorimeter", "barrel"])
def test_safety_is_lower_bound(ctx, torch_dev, oracle_lib, name, precision):
    """Every point strictly inside the sphere of the GPU safety lies in the same
    touchable (brute-force oracle locate), for 2000 points and 64 directions
    each.  (The voxel safety is not compared with the oracle's brute-force
    safety: both are lower bounds of the true distance and neither bounds the
    other, since an isotropic solid safety can fall below the distance to a
    voxel node face.)"""
    torch = torch_dev
    desc, gid, nt, og = geom(ctx, name, oracle_lib)
    print_case("safety", name, precision)
    rng = np.random.Generator(np.random.Philox(key=1003))
    pts = sample_points(desc, rng, 3000)
    T = og.locate(pts)
    ok = T >= 0
    pts, T = pts[ok][:2000], T[ok][:2000]
    saf = ctx.compute_safety(gid, torch.from_numpy(pts).cuda(), precision=precision).cpu().numpy()
    same = ctx.compute_safety(gid, torch.from_numpy(pts).cuda(), torch.from_numpy(T.astype(np.int32)).cuda(),
                              precision=precision).cpu().numpy()
    assert np.array_equal(saf, same)
    assert np.all(saf >= 0)
    sph = W.primaries.isotropic(rng, 64)
    q = (pts[:, None, :] + (saf * (1 - 1e-9))[:, None, None] * sph[None, :, :]).reshape(-1, 3)
    loc = og.locate(q).reshape(len(pts), 64)
    d = og.compute_safety(q, loc.reshape(-1)).reshape(len(pts), 64)
    # a sphere point may only leave the touchable within the surface band of
    # a boundary it just touches
    bad = (loc != T[:, None]) & (d > 1e-6)
    assert not bad.any(), np.argwhere(bad)[:5]
    # the safety is positive away from boundaries for most points
    assert np.mean(saf > 0) > 0.9


@pytest.mark.parametrize("name,n,cap", [("tiny", 10000, 64), ("calorimeter", 4000, 400),
                                        ("barrel", 3000, 512), ("endcap", 4000, 256)])
def test_transport_parity_per_track(ctx, torch_dev, oracle_lib, name, n, cap):
    torch = torch_dev
    desc, gid, nt, og = geom(ctx, name, oracle_lib)
    print_case("transport", name, n)
    _, prim, _ = W.WORKLOADS[name](n=n)
    got = run_transport(ctx, torch, gid, prim, cap)
    ref = og.transport(prim, seed=0, log_cap=cap)
    bad = compare_logs(got["log"], got["log_n"], got["log_fate"], ref, cap)
    assert not bad, bad[:10]
    for k in EXACT:
        assert got["counters"][k] == ref["counters"][k], k
    assert got["counters"]["invalid"] == 0
    assert np.allclose(got["edep_event"], ref["edep_event"], rtol=RTOL, atol=1e-15)
    assert np.allclose(got["escaped_event"], ref["escaped_event"], rtol=RTOL, atol=1e-15)
    assert np.allclose(got["edep_touchable"], ref["edep_touchable"], rtol=RTOL, atol=1e-12)


@pytest.mark.parametrize("name,n,prim_seed,seed", [("calorimeter", 3000, 5, 3), ("barrel", 2000, 9, 11),
                                                   ("tiny", 5000, 2, 7)])
def test_transport_parity_other_seeds(ctx, torch_dev, oracle_lib, name, n, prim_seed, seed):
    """Other primary sets and other transport streams: per-track parity."""
    torch = torch_dev
    desc, gid, nt, og = geom(ctx, name, oracle_lib)
    print_case("transport_seeds", name, prim_seed, seed)
    _, prim, _ = W.WORKLOADS[name](n=n, seed=prim_seed)
    cap = 512
    got = run_transport(ctx, torch, gid, prim, cap, seed=seed)
    ref = og.transport(prim, seed=seed, log_cap=cap)
    bad = compare_logs(got["log"], got["log_n"], got["log_fate"], ref, cap)
    assert not bad, bad[:10]
    for k in EXACT:
        assert got["counters"][k] == ref["counters"][k], k
    assert np.allclose(got["edep_event"], ref["edep_event"], rtol=RTOL, atol=1e-15)
    assert np.allclose(got["edep_touchable"], ref["edep_touchable"], rtol=RTOL, atol=1e-12)


def test_transport_parity_rotated_boxes(ctx, torch_dev, oracle_lib):
    """Boxes placed with rotations run the general kernel (the axis-aligned box
    build serves unrotated boxes only): per-track parity with the oracle."""
    torch = torch_dev
    desc, gid, nt, og = geom(ctx, "tiny_rot", oracle_lib)
    print_case("transport_rotated_boxes")
    prim = W.primaries.tiny_source(6000, 0)
    got = run_transport(ctx, torch, gid, prim, 64)
    ref = og.transport(prim, seed=0, log_cap=64)
    bad = compare_logs(got["log"], got["log_n"], got["log_fate"], ref, 64)
    assert not bad, bad[:10]
    for k in EXACT:
        assert got["counters"][k] == ref["counters"][k], k
    assert np.allclose(got["edep_event"], ref["edep_event"], rtol=RTOL, atol=1e-15)


def test_transport_parity_pair_heavy(ctx, torch_dev, oracle_lib):
    """20 MeV photons in the calorimeter convert often, so annihilation photons
    outrun the block stack and also take the per-slot pending path: per-track
    parity with the oracle."""
    torch = torch_dev
    desc, gid, nt, og = geom(ctx, "calorimeter", oracle_lib)
    print_case("transport_pair_heavy")
    _, prim, _ = W.calorimeter(n=3000)
    prim.energy[:] = 20.0
    got = run_transport(ctx, torch, gid, prim, 600)
    ref = og.transport(prim, seed=0, log_cap=600)
    assert ref["counters"]["pair"] > 1000
    bad = compare_logs(got["log"], got["log_n"], got["log_fate"], ref, 600)
    assert not bad, bad[:10]
    for k in EXACT:
        assert got["counters"][k] == ref["counters"][k], k
    assert np.allclose(got["edep_event"], ref["edep_event"], rtol=RTOL, atol=1e-15)


@pytest.mark.parametrize("block", [128, 256])
def test_transport_parity_sphere_builds(ctx, torch_dev, oracle_lib, block):
    """Geometries with sphere sections run the transport builds that dispatch
    them, at every pool size: per-track parity on the endcap workload."""
    torch = torch_dev
    desc, gid, nt, og = geom(ctx, "endcap", oracle_lib)
    print_case("transport_sphere_build", block)
    _, prim, _ = W.endcap(n=2000, seed=4)
    got = run_transport(ctx, torch, gid, prim, 256, block=block)
    ref = og.transport(prim, seed=0, log_cap=256)
    bad = compare_logs(got["log"], got["log_n"], got["log_fate"], ref, 256)
    assert not bad, bad[:10]
    for k in EXACT:
        assert got["counters"][k] == ref["counters"][k], k
    assert np.allclose(got["edep_touchable"], ref["edep_touchable"], rtol=RTOL, atol=1e-12)


def test_transport_launch_shape_independent(ctx, torch_dev, oracle_lib):
    """Counter-keyed random numbers: any block/grid gives the same tracks."""
    torch = torch_dev
    desc, gid, nt, og = geom(ctx, "calorimeter", oracle_lib)
    print_case("launch_shape")
    _, prim, _ = W.calorimeter(n=3000)
    a = run_transport(ctx, torch, gid, prim, 200, grid=3)
    b = run_transport(ctx, torch, gid, prim, 200, block=256, grid=97)
    assert np.array_equal(a["log_n"], b["log_n"])
    for f in ("touchable", "code", "step", "edep", "energy"):
        assert np.array_equal(a["log"][f], b["log"][f])


def test_transport_full_calorimeter_sampled(ctx, torch_dev, oracle_lib):
    """The bench workload (1e6 photons) at its launch shape: energy conservation
    per event on every track, and 1000 sampled tracks against the oracle."""
    torch = torch_dev
    desc, gid, nt, og = geom(ctx, "calorimeter", oracle_lib)
    print_case("calorimeter_full")
    _, prim, _ = W.calorimeter()
    got = run_transport(ctx, torch, gid, prim, 0)
    assert got["counters"]["truncated"] == 0 and got["counters"]["invalid"] == 0
    tot = got["edep_event"] + got["escaped_event"]
    assert np.allclose(tot, prim.energy, rtol=1e-12, atol=0)
    rng = np.random.Generator(np.random.Philox(key=5))
    idx = np.sort(rng.choice(prim.n, 1000, replace=False))
    sub = prim.subset(idx)
    ref = og.transport(sub, seed=0, log_cap=0, n_events=prim.n_events)
    assert np.allclose(got["edep_event"][idx], ref["edep_event"][idx], rtol=RTOL, atol=1e-15)
    assert np.allclose(got["escaped_event"][idx], ref["escaped_event"][idx], rtol=RTOL, atol=1e-15)


def test_invalid_primaries_are_skipped(ctx, torch_dev, oracle_lib):
    torch = torch_dev
    desc, gid, nt, og = geom(ctx, "tiny", oracle_lib)
    print_case("invalid")
    _, prim, _ = W.tiny(n=64)
    prim.energy[3] = np.nan
    prim.event[5] = 10_000  # outside the tally's events
    prim.energy[7] = -1.0
    got = run_transport(ctx, torch, gid, prim, 0)
    assert got["counters"]["invalid"] == 3
    assert got["counters"]["tracks"] + 3 >= 64
