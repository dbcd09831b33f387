"""GPU: uneven events over several resident geometries in one launch, and
graph-captured repeated batches (through the C ABI)."""
import sys

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

RTOL = 1e-9


def print_case(*a):
    print("CASE", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible MI355X"
    return torch


def small_batched(seed=4):
    geoms = [W.geometry.tiny(), W.geometry.calorimeter(n_layers=10, n_cells=8),
             W.geometry.barrel_variant(104)]
    sources = [W.primaries.source_origin_iso, W.primaries.source_beam, W.primaries.source_axis_iso]
    prim, event_geom = W.primaries.batched_events(n_events=90, n_geoms=3, seed=seed, median=20,
                                                  lo=3, hi=200, sources=sources)
    return geoms, prim, event_geom


def test_batched_matches_oracle_per_geometry(torch_dev, oracle_lib):
    torch = torch_dev
    from paper_1209_5235_amd import gnav
    print_case("batched")
    geoms, prim, event_geom = small_batched()
    ctx = gnav.Context(0)
    gids = [ctx.upload_geometry(g)[0] for g in geoms]
    assert gids == [0, 1, 2]
    tally = ctx.tally_create(prim.n_events)
    cap = 256
    dev = gnav.primaries_to_device(prim, "cuda")
    log = gnav.make_log(prim.n, cap, "cuda")
    eg = torch.from_numpy(event_geom).cuda()
    ctx.transport_batch(0, dev, tally, seed=0, log=log, event_geom=eg)
    torch.cuda.synchronize()
    got = tally.read()
    rec, n, fate = gnav.log_to_numpy(log)
    for g, desc in enumerate(geoms):
        idx = np.nonzero(event_geom[prim.event] == g)[0]
        sub = prim.subset(idx)
        ref = oracle_lib.Geometry(desc).transport(sub, seed=0, log_cap=cap, n_events=prim.n_events)
        slots = (3 * idx[:, None] + np.arange(3)[None, :]).reshape(-1)
        assert np.array_equal(n[slots], ref["log_n"])
        assert np.array_equal(fate[slots], ref["log_fate"])
        for j, s in enumerate(slots):
            k = min(int(n[s]), cap)
            a, b = rec[s, :k], ref["log"][j, :k]
            assert np.array_equal(a["touchable"], b["touchable"])
            assert np.array_equal(a["code"], b["code"])
            assert np.allclose(a["step"], b["step"], rtol=RTOL, atol=1e-12)
        evs = np.unique(sub.event)
        assert np.allclose(got["edep_event"][evs], ref["edep_event"][evs], rtol=RTOL, atol=1e-15)
        off, _ = ctx.touchable_offset(g)
        nt = ctx.geoms[g][1]
        assert np.allclose(got["edep_touchable"][off:off + nt], ref["edep_touchable"], rtol=RTOL,
                           atol=1e-12)
    tot = got["edep_event"] + got["escaped_event"]
    per_event = np.bincount(prim.event, weights=prim.energy, minlength=prim.n_events)
    assert np.allclose(tot, per_event, rtol=1e-12, atol=0)
    tally.free()
    ctx.close()


def test_graph_replays_match_eager(torch_dev, oracle_lib):
    torch = torch_dev
    from paper_1209_5235_amd import gnav
    print_case("graph")
    geoms, prim, _ = W.calorimeter(n=20000)
    ctx = gnav.Context(0)
    gid, nt = ctx.upload_geometry(geoms[0])
    dev = gnav.primaries_to_device(prim, "cuda")
    eager_t = ctx.tally_create(prim.n_events)
    ctx.transport_batch(gid, dev, eager_t)
    torch.cuda.synchronize()
    eager = eager_t.read()
    gt = ctx.tally_create(prim.n_events)
    g = ctx.graph_create(gid, dev, gt)
    for rep in range(3):
        ctx.graph_launch(g)
        torch.cuda.synchronize()
        r = gt.read()
        assert r["counters"] == eager["counters"], rep
        assert np.allclose(r["edep_event"], eager["edep_event"], rtol=RTOL, atol=1e-15)
        assert np.allclose(r["edep_touchable"], eager["edep_touchable"], rtol=RTOL, atol=1e-12)
        # eager work between replays
        eager_t.reset()
        ctx.transport_batch(gid, dev, eager_t)
        torch.cuda.synchronize()
    ctx.graph_free(g)
    gt.free()
    eager_t.free()
    ctx.close()
