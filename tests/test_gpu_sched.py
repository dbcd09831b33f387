"""GPU: scheduling knobs (queue chunk, sort period, grid) and the autotuner.

Random numbers are keyed by (event, track, draw), so every setting must give
bitwise identical per-track logs and identical counters.
"""
import numpy as np
import pytest

import workloads as W
from tests.gpu_common import ctx, geom, print_case, run_transport, torch_dev  # noqa: F401

pytestmark = pytest.mark.gpu

SETTINGS = [dict(), dict(chunk=256), dict(chunk=4096, grid=7), dict(sort_period=1),
            dict(chunk=1024, sort_period=4, grid=300), dict(chunk=64, sort_period=16),
            dict(block=128), dict(block=64, chunk=256, sort_period=4), dict(block=64, grid=3),
            dict(block=128, grid=1000, sort_period=1)]


@pytest.mark.parametrize("name,n,cap", [("calorimeter", 3000, 200), ("barrel", 2000, 512)])
def test_schedule_settings_give_identical_tracks(ctx, torch_dev, oracle_lib, name, n, cap):
    torch = torch_dev
    desc, gid, nt, og = geom(ctx, name, oracle_lib)
    _, prim, _ = W.WORKLOADS[name](n=n)
    runs = []
    for kw in SETTINGS:
        print_case("schedule", name, kw)
        runs.append(run_transport(ctx, torch, gid, prim, cap, **kw))
    a = runs[0]
    for b in runs[1:]:
        assert np.array_equal(a["log_n"], b["log_n"])
        assert np.array_equal(a["log_fate"], b["log_fate"])
        for f in ("touchable", "code", "step", "edep", "energy"):
            assert np.array_equal(a["log"][f], b["log"][f]), f
        for k in ("steps", "pe", "compton", "pair", "crossings", "escaped", "tracks", "invalid"):
            assert a["counters"][k] == b["counters"][k], k


def test_invalid_runs_do_not_end_blocks_early(ctx, torch_dev, oracle_lib):
    """A long run of invalid primaries between valid ones: every valid one is
    still transported, with both refill schemes."""
    torch = torch_dev
    desc, gid, nt, og = geom(ctx, "tiny", oracle_lib)
    _, prim, _ = W.tiny(n=6000)
    prim.energy[100:5000] = -1.0
    for kw in (dict(grid=2), dict(grid=2, chunk=512)):
        print_case("invalid_run", kw)
        got = run_transport(ctx, torch, gid, prim, 0, **kw)
        assert got["counters"]["invalid"] == 4900
        ref = og.transport(prim.subset(np.nonzero(prim.energy > 0)[0]), seed=0, n_events=prim.n_events)
        assert got["counters"]["tracks"] == ref["counters"]["tracks"]
        assert got["counters"]["steps"] == ref["counters"]["steps"]


def test_autotune_picks_a_setting_and_tuned_runs_match(ctx, torch_dev, oracle_lib):
    torch = torch_dev
    from paper_1209_5235_amd import gnav
    desc, gid, nt, og = geom(ctx, "calorimeter", oracle_lib)
    print_case("autotune")
    _, prim, _ = W.calorimeter(n=200000)
    dev = gnav.primaries_to_device(prim, "cuda")
    tally = ctx.tally_create(prim.n_events)
    best = ctx.autotune(gid, dev, tally, trials=2)
    print("autotune", best, flush=True)
    assert best["block"] in (64, 128, 256) and best["grid"] >= 1 and best["chunk"] in (0, 256, 1024, 4096)
    assert best["sort_period"] in (0, 1, 4, 16) and best["ms"] > 0
    # the tally is left zeroed
    z = tally.read()
    assert z["counters"]["steps"] == 0 and not z["edep_event"].any()
    ctx.transport_batch(gid, dev, tally)
    torch.cuda.synchronize()
    a = tally.read()
    tally.reset()
    ctx.transport_batch(gid, dev, tally, tuned=True)
    torch.cuda.synchronize()
    b = tally.read()
    tally.free()
    assert a["counters"] == b["counters"]
    assert np.allclose(a["edep_event"], b["edep_event"], rtol=1e-12, atol=1e-15)


def test_bound_order_on_box_geometry_is_identical(ctx, torch_dev, oracle_lib):
    """The axis-aligned box build's ordered-walk instantiation: identical logs."""
    torch = torch_dev
    desc, gid, nt, og = geom(ctx, "calorimeter", oracle_lib)
    print_case("bound_order_boxes")
    _, prim, _ = W.calorimeter(n=3000)
    a = run_transport(ctx, torch, gid, prim, 200)
    b = run_transport(ctx, torch, gid, prim, 200, order=1)
    assert np.array_equal(a["log_n"], b["log_n"]) and np.array_equal(a["log_fate"], b["log_fate"])
    for f in ("touchable", "code", "step", "edep", "energy"):
        assert np.array_equal(a["log"][f], b["log"][f]), f
