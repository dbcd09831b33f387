"""GPU: every track of the full-size workloads against the oracle.

For each workload the HIP library runs twice: in the launch configuration
bench.py times (no logging), whose per-event and per-touchable tallies and
counters are compared with the oracle's, and with per-track digests, which
are compared slot by slot.  Tracks whose digests differ are transported again
with full logs on both sides; the oracle's decision margins at the first
divergence classify each as a rounding-edge flip or a bug.  The bar: no bug,
flips below 1e-5 of the tracks (the oracle runs in 16 processes):

* calorimeter: all 1e6 photons;
* barrel: the first 1e5 of its 1e7 photons;
* endcap (trapezoids and sphere sections): 2e5 photons;
* batched events: every 64th of the 4096 events, over their geometries.
"""
import numpy as np
import pytest

import workloads as W
from tests.gpu_common import ctx, geom, print_case, run_transport, torch_dev  # noqa: F401

pytestmark = pytest.mark.gpu

FLIP_RATE = 1e-5


def _gpu_digests(ctx, torch, gid, prim, event_geom=None):
    from paper_1209_5235_amd import gnav
    dev = gnav.primaries_to_device(prim, "cuda")
    d = gnav.make_digests(prim.n, "cuda")
    tally = ctx.tally_create(prim.n_events)
    ctx.transport_batch(gid, dev, tally, digest=d, event_geom=event_geom)
    torch.cuda.synchronize()
    tally.free()
    return gnav.digests_to_numpy(d)


def _logs_fn(ctx, torch, gid, prim, cap, event_geom_np=None):
    def fn(idx):
        sub = prim.subset(idx)
        kw = {}
        if event_geom_np is not None:
            kw["event_geom"] = torch.from_numpy(np.ascontiguousarray(event_geom_np, np.int32)).cuda()
        got = run_transport(ctx, torch, gid, sub, cap, **kw)
        return got["log"], got["log_n"], got["log_fate"]
    return fn


def _report(name, res):
    print(name, {k: res[k] for k in ("tracks", "mismatches", "flips", "bugs")},
          {k: v for k, v in res.items() if k.startswith("max_rel") or k == "counters_equal"},
          res["classified"][:10], flush=True)


def _assert_bar(res, tally=True):
    assert res["bugs"] == 0, res["classified"][:20]
    assert res["flips"] <= FLIP_RATE * res["tracks"], (res["flips"], res["tracks"])
    if tally:
        assert res["counters_equal"]
        assert res["max_rel_event_deposit"] <= 1e-9 and res["max_rel_event_escape"] <= 1e-9
        assert res["max_rel_touchable_deposit"] <= 1e-9


def test_calorimeter_every_track(ctx, torch_dev, oracle_lib):
    from oracle import parity
    torch = torch_dev
    desc, gid, nt, og = geom(ctx, "calorimeter", oracle_lib)
    print_case("fullparity_calorimeter")
    _, prim, _ = W.calorimeter()
    tally = run_transport(ctx, torch, gid, prim, 0)  # the benchmark's launch
    dig = _gpu_digests(ctx, torch, gid, prim)
    res = parity.full_check(desc, prim, dig, _logs_fn(ctx, torch, gid, prim, 4096), gpu_tally=tally)
    _report("calorimeter", res)
    assert res["tracks"] > 1_000_000
    _assert_bar(res)


def test_barrel_first_1e5_tracks(ctx, torch_dev, oracle_lib):
    from oracle import parity
    torch = torch_dev
    desc, gid, nt, og = geom(ctx, "barrel", oracle_lib)
    print_case("fullparity_barrel")
    _, full, _ = W.barrel()
    prim = full.subset(np.arange(100_000))
    del full
    tally = run_transport(ctx, torch, gid, prim, 0)
    dig = _gpu_digests(ctx, torch, gid, prim)
    res = parity.full_check(desc, prim, dig, _logs_fn(ctx, torch, gid, prim, 4096), gpu_tally=tally)
    _report("barrel", res)
    assert res["tracks"] > 100_000
    _assert_bar(res)


def test_endcap_every_track(ctx, torch_dev, oracle_lib):
    """The trapezoid endcap with its sphere-section shell (the sphere builds run):
    every track of 2e5 photons from the origin."""
    from oracle import parity
    torch = torch_dev
    desc, gid, nt, og = geom(ctx, "endcap", oracle_lib)
    print_case("fullparity_endcap")
    _, prim, _ = W.endcap(n=200_000, seed=3)
    tally = run_transport(ctx, torch, gid, prim, 0)
    dig = _gpu_digests(ctx, torch, gid, prim)
    res = parity.full_check(desc, prim, dig, _logs_fn(ctx, torch, gid, prim, 4096), gpu_tally=tally)
    _report("endcap", res)
    assert res["tracks"] > 200_000
    _assert_bar(res)


def test_batched_every_64th_event(torch_dev, oracle_lib):
    from oracle import parity
    from paper_1209_5235_amd import gnav
    torch = torch_dev
    print_case("fullparity_batched")
    geoms, full, event_geom = W.batched()
    ctx = gnav.Context(0)
    gids = [ctx.upload_geometry(g)[0] for g in geoms]
    idx = np.nonzero(full.event % 64 == 0)[0]
    prim = full.subset(idx)
    del full
    eg_np = np.asarray(event_geom, np.int32) + gids[0]
    eg = torch.from_numpy(eg_np).cuda()
    dig = _gpu_digests(ctx, torch, gids[0], prim, event_geom=eg)
    total = dict(tracks=0, mismatches=0, flips=0, bugs=0)
    for g, desc in enumerate(geoms):
        sel = np.nonzero(np.asarray(event_geom)[prim.event] == g)[0]
        if len(sel) == 0:
            continue
        sub = prim.subset(sel)
        slots = (3 * sel[:, None] + np.arange(3)[None, :]).reshape(-1)
        res = parity.full_check(desc, sub, dig[slots], _logs_fn(ctx, torch, gids[0], sub, 4096, eg_np),
                                n_events=prim.n_events)
        _report(f"batched geometry {g}", res)
        for k in total:
            total[k] += res[k]
        _assert_bar(res, tally=False)
    print("batched total", total, flush=True)
    assert total["tracks"] > 100_000
    assert total["flips"] <= FLIP_RATE * total["tracks"]
    ctx.close()
