"""GPU: the benchmark configurations at full size in the launch configuration
bench.py times, checked on properties that hold at any size (per-event energy
conservation) and on sampled events against the oracle; plus the degenerate
batches (empty, photons outside the world)."""
import numpy as np
import pytest

import workloads as W
from tests.gpu_common import RTOL, ctx, print_case, run_transport, torch_dev  # noqa: F401

pytestmark = pytest.mark.gpu


def _events_vs_oracle(oracle_lib, desc, prim, got, events):
    og = oracle_lib.Geometry(desc)
    idx = np.nonzero(np.isin(prim.event, events))[0]
    ref = og.transport(prim.subset(idx), seed=0, n_events=prim.n_events)
    assert np.allclose(got["edep_event"][events], ref["edep_event"][events], rtol=RTOL, atol=1e-15)
    assert np.allclose(got["escaped_event"][events], ref["escaped_event"][events], rtol=RTOL, atol=1e-15)


def test_barrel_full_size(ctx, torch_dev, oracle_lib):
    """1e7 photons, default launch: every event conserves energy; 2000 sampled
    photons (each its own event) match the oracle."""
    torch = torch_dev
    print_case("barrel_full")
    geoms, prim, _ = W.barrel()
    gid, _ = ctx.upload_geometry(geoms[0])
    got = run_transport(ctx, torch, gid, prim, 0)
    assert got["counters"]["truncated"] == 0 and got["counters"]["invalid"] == 0
    assert got["counters"]["stuck"] == 0
    tot = got["edep_event"] + got["escaped_event"]
    assert np.allclose(tot, prim.energy, rtol=1e-12, atol=0)
    rng = np.random.Generator(np.random.Philox(key=11))
    ev = np.sort(rng.choice(prim.n_events, 2000, replace=False))
    _events_vs_oracle(oracle_lib, geoms[0], prim, got, ev)


def test_batched_full_size_tuned_graph(ctx, torch_dev, oracle_lib):
    """4096 uneven events over 8 geometries, autotuned and graph-captured as in
    the benchmark: energy conserved per event; the smallest event of five
    geometries matches the oracle."""
    torch = torch_dev
    from paper_1209_5235_amd import gnav
    print_case("batched_full")
    geoms, prim, event_geom = W.batched()
    gids = [ctx.upload_geometry(g)[0] for g in geoms]
    dev = gnav.primaries_to_device(prim, "cuda")
    eg = torch.from_numpy(np.asarray(event_geom, np.int32) + gids[0]).cuda()
    tally = ctx.tally_create(prim.n_events)
    best = ctx.autotune(gids[0], dev, tally, trials=1, event_geom=eg)
    print("tuned", best, flush=True)
    g = ctx.graph_create(gids[0], dev, tally, tuned=True, event_geom=eg)
    for _ in range(2):
        tally.reset()
        ctx.graph_launch(g)
    torch.cuda.synchronize()
    got = tally.read()
    ctx.graph_free(g)
    tally.free()
    assert got["counters"]["invalid"] == 0 and got["counters"]["truncated"] == 0
    tot = got["edep_event"] + got["escaped_event"]
    e_ev = np.bincount(prim.event, weights=prim.energy, minlength=prim.n_events)
    assert np.allclose(tot, e_ev, rtol=1e-12, atol=0)
    counts = np.bincount(prim.event, minlength=prim.n_events)
    seen = {}
    for e in np.argsort(counts, kind="stable"):
        gi = int(event_geom[e])
        if gi not in seen:
            seen[gi] = int(e)
        if len(seen) == 5:
            break
    for gi, e in seen.items():
        sub_idx = np.nonzero(prim.event == e)[0]
        og = oracle_lib.Geometry(geoms[gi])
        ref = og.transport(prim.subset(sub_idx), seed=0, n_events=prim.n_events)
        assert np.isclose(got["edep_event"][e], ref["edep_event"][e], rtol=RTOL, atol=1e-15), (gi, e)
        assert np.isclose(got["escaped_event"][e], ref["escaped_event"][e], rtol=RTOL, atol=1e-15), (gi, e)


def test_empty_batch(ctx, torch_dev, oracle_lib):
    torch = torch_dev
    print_case("empty")
    _, prim, _ = W.tiny(n=8)
    gid, _ = ctx.upload_geometry(W.geometry.tiny())
    got = run_transport(ctx, torch, gid, prim.subset(np.arange(0)), 0)
    assert all(v == 0 for v in got["counters"].values())


def test_photons_outside_the_world_escape(ctx, torch_dev, oracle_lib):
    torch = torch_dev
    print_case("outside")
    _, prim, _ = W.tiny(n=256)
    prim.pos[:] = np.array([0.0, 0.0, 2000.0])  # beyond the 500 mm half-size world
    gid, _ = ctx.upload_geometry(W.geometry.tiny())
    got = run_transport(ctx, torch, gid, prim, 0)
    assert got["counters"]["escaped"] == 256 and got["counters"]["steps"] == 0
    assert np.array_equal(got["escaped_event"], prim.energy)
    ref = oracle_lib.Geometry(W.geometry.tiny()).transport(prim, seed=0)
    assert ref["counters"]["escaped"] == 256
