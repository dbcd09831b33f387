"""GPU: crossing recorder, on-GPU training, and candidate orders that leave
every result unchanged (plain voxel walk vs lower-bound order vs learned order)."""
import sys

import numpy as np
import pytest

import workloads as W
from tests.gpu_common import EXACT, compare_logs

pytestmark = pytest.mark.gpu


def print_case(*a):
    print("CASE", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def barrel():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible MI355X"
    from paper_1209_5235_amd import gnav
    ctx = gnav.Context(0)
    desc = W.geometry.barrel()
    gid, nt = ctx.upload_geometry(desc)
    yield torch, gnav, ctx, gid, desc
    ctx.close()


def _run(torch, gnav, ctx, gid, prim, cap, **kw):
    tally = ctx.tally_create(prim.n_events)
    dev = gnav.primaries_to_device(prim, "cuda")
    log = gnav.make_log(prim.n, cap, "cuda")
    ctx.transport_batch(gid, dev, tally, log=log, count_work=True, **kw)
    torch.cuda.synchronize()
    out = tally.read()
    tally.free()
    out["log"], out["log_n"], out["log_fate"] = gnav.log_to_numpy(log)
    return out


def test_recorder_records_valid_crossings(barrel):
    torch, gnav, ctx, gid, desc = barrel
    print_case("recorder")
    from paper_1209_5235_amd import learned
    _, prim, _ = W.barrel(n=4000, seed=1)
    dev = gnav.primaries_to_device(prim, "cuda")
    rec = learned.record_crossings(ctx, gid, dev, prim.n_events, capacity=200000, seed=1)
    r = gnav.recorder_to_numpy(rec)
    n_class = ctx.ordering_classes(gid)
    assert n_class == 66  # world, envelope and 64 layers carry voxel grids
    assert len(r) > 1000
    assert np.all((r["label"] >= 0) & (r["label"] < 64))
    assert np.all((r["cls"] >= 0) & (r["cls"] < n_class))
    assert np.allclose(np.linalg.norm(r["v"], axis=1), 1, atol=1e-6)
    assert np.all(np.abs(r["x"]) <= 1.0 + 1e-5)


@pytest.mark.parametrize("voxel_lists", [0, 1])
def test_orders_give_identical_results(barrel, voxel_lists):
    """Plain, lower-bound and learned orders: bitwise identical per-track logs, with
    the shape-aware node lists (no mother holds enough candidates per node for the
    orders to engage) and with bounding-box lists (the envelope's nodes do)."""
    torch, gnav, ctx, gid, desc = barrel
    print_case("order_identity", voxel_lists)
    from paper_1209_5235_amd import learned
    if voxel_lists:
        gid, _ = ctx.upload_geometry(desc, voxel_lists=1)
    n_class = ctx.ordering_classes(gid)
    # train briefly on crossings recorded with other seeds
    _, tprim, _ = W.barrel(n=20000, seed=1)
    rec = learned.record_crossings(ctx, gid, gnav.primaries_to_device(tprim, "cuda"), tprim.n_events,
                                   capacity=400000, seed=1)
    x, cls, label = learned.records_to_tensors(rec)
    net, _ = learned.train(ctx, n_class, x, cls, label, epochs=1, batch=1024)
    ctx.set_mlp(gid, net)
    _, prim, _ = W.barrel(n=3000, seed=0)
    cap = 512
    plain = _run(torch, gnav, ctx, gid, prim, cap, order=0)
    bound = _run(torch, gnav, ctx, gid, prim, cap, order=1)
    learn = _run(torch, gnav, ctx, gid, prim, cap, order=2)
    for other in (bound, learn):
        assert np.array_equal(other["log_n"], plain["log_n"])
        assert np.array_equal(other["log_fate"], plain["log_fate"])
        for f in ("touchable", "code", "step", "edep", "energy"):
            assert np.array_equal(other["log"][f], plain["log"][f]), f
        assert np.array_equal(other["edep_event"], plain["edep_event"]) or np.allclose(
            other["edep_event"], plain["edep_event"], rtol=1e-12, atol=0)
        for k in ["steps", "pe", "compton", "pair", "crossings", "escaped"]:
            assert other["counters"][k] == plain["counters"][k]
    if voxel_lists:
        # where they engage, the orders examine fewer exact daughter distances
        assert bound["counters"]["dist_in"] < plain["counters"]["dist_in"]
        assert learn["counters"]["dist_in"] < plain["counters"]["dist_in"]
    else:
        assert bound["counters"]["dist_in"] == plain["counters"]["dist_in"]
    print("dist_in evaluations plain/bound/learned:", plain["counters"]["dist_in"],
          bound["counters"]["dist_in"], learn["counters"]["dist_in"], flush=True)
    ctx.set_mlp(gid, None)
    net.free()


def test_training_learns_the_limiting_candidate(barrel):
    torch, gnav, ctx, gid, desc = barrel
    print_case("train")
    from paper_1209_5235_amd import learned
    n_class = ctx.ordering_classes(gid)
    _, tprim, _ = W.barrel(n=40000, seed=1)
    rec = learned.record_crossings(ctx, gid, gnav.primaries_to_device(tprim, "cuda"), tprim.n_events,
                                   capacity=1_000_000, seed=1)
    x, cls, label = learned.records_to_tensors(rec)
    net, losses = learned.train(ctx, n_class, x, cls, label, epochs=2, batch=4096, log_every=10)
    # held-out crossings (other primaries, other transport seed)
    _, eprim, _ = W.barrel(n=10000, seed=7)
    erec = learned.record_crossings(ctx, gid, gnav.primaries_to_device(eprim, "cuda"), eprim.n_events,
                                    capacity=400000, seed=7)
    ex, ec, el = learned.records_to_tensors(erec)
    acc = learned.accuracy(net, ex, ec, el)
    base = np.bincount(el.cpu().numpy(), minlength=64).max() / el.shape[0]
    print("held-out accuracy", acc, "most-frequent-label baseline", base, "losses", losses[:3],
          losses[-3:], flush=True)
    assert losses[-1] < losses[0]
    assert acc > base
    net.free()


@pytest.mark.parametrize("trained", [True, False])
def test_learned_order_matches_oracle_per_track(barrel, oracle_lib, trained):
    """Learned-order transport (bounding-box node lists, where the network
    scores steps) against the oracle track by track: volume and limiter
    sequences exact, lengths and deposits within 1e-9.  With an untrained
    network the predictions are mostly wrong, which exercises the pruning of
    the candidates it did not pick."""
    torch, gnav, ctx, gid, desc = barrel
    print_case("learned_vs_oracle", trained)
    from oracle import mlp as omlp
    from paper_1209_5235_amd import learned
    gid_b, _ = ctx.upload_geometry(desc, voxel_lists=1)
    n_class = ctx.ordering_classes(gid_b)
    if trained:
        _, tprim, _ = W.barrel(n=20000, seed=1)
        rec = learned.record_crossings(ctx, gid_b, gnav.primaries_to_device(tprim, "cuda"), tprim.n_events,
                                       capacity=600000, seed=1)
        x, cls, label = learned.records_to_tensors(rec)
        net, _ = learned.train(ctx, n_class, x, cls, label, epochs=1, batch=1024)
    else:
        net = gnav.MLP(ctx, n_class, omlp.init(n_class, seed=21), max_batch=64)
    ctx.set_mlp(gid_b, net)
    _, prim, _ = W.barrel(n=3000, seed=0)
    cap = 512
    got = _run(torch, gnav, ctx, gid_b, prim, cap, order=2)
    ref = oracle_lib.Geometry(desc).transport(prim, seed=0, log_cap=cap)
    bad = compare_logs(got["log"], got["log_n"], got["log_fate"], ref, cap)
    assert not bad, bad[:10]
    for k in EXACT:
        assert got["counters"][k] == ref["counters"][k], k
    assert np.allclose(got["edep_event"], ref["edep_event"], rtol=1e-9, atol=1e-15)
    print("scored steps", got["counters"]["scored"], "of", got["counters"]["steps"], flush=True)
    assert got["counters"]["scored"] > 0
    ctx.set_mlp(gid_b, None)
    net.free()


def test_learned_order_scores_nothing_without_wide_mothers(barrel):
    """With shape-aware node lists no barrel mother holds three or more
    candidates per node on average: order 2 then runs the bound order's walk,
    and the scored-step counter says so."""
    torch, gnav, ctx, gid, desc = barrel
    print_case("learned_no_wide")
    from oracle import mlp as omlp
    n_class = ctx.ordering_classes(gid)
    net = gnav.MLP(ctx, n_class, omlp.init(n_class, seed=21), max_batch=64)
    ctx.set_mlp(gid, net)
    _, prim, _ = W.barrel(n=2000, seed=0)
    got = _run(torch, gnav, ctx, gid, prim, 64, order=2)
    plain = _run(torch, gnav, ctx, gid, prim, 64, order=0)
    assert got["counters"]["scored"] == 0
    assert plain["counters"]["scored"] == 0
    assert np.array_equal(got["log"]["touchable"], plain["log"]["touchable"])
    ctx.set_mlp(gid, None)
    net.free()
