"""GPU: gnav_transport_batch_noalloc (fixed per-device scratch, no allocation)
against gnav_transport_batch on the same inputs, through the C ABI.

Two calls in a row share the device's scratch array: the first a pair-heavy
calorimeter batch (annihilation photons overflow the block stack and take the
per-slot pending entries that live in the scratch), the second a smaller tiny
batch with a smaller grid.  Each must equal the allocating entry point's
result: per-track logs and counters exactly, tallies within 1e-9 relative
(atomic summation order)."""
import ctypes as C

import numpy as np
import pytest

import workloads as W
from tests.gpu_common import EXACT, RTOL, compare_logs, ctx, geom, print_case, torch_dev  # noqa: F401

pytestmark = pytest.mark.gpu


def _run(ctx, torch, gid, prim, cap, noalloc, **kw):
    from paper_1209_5235_amd import gnav
    tally = ctx.tally_create(prim.n_events)
    dev = gnav.primaries_to_device(prim, "cuda")
    log = gnav.make_log(prim.n, cap, "cuda")
    b = ctx._batch(gid, dev, log=log, **kw)
    fn = gnav.gnav_transport_batch_noalloc if noalloc else gnav.gnav_transport_batch
    st = fn(ctx.h, C.byref(b), tally.h, gnav._stream(None))
    assert st == gnav.GNAV_OK, gnav.gnav_last_error(ctx.h)
    torch.cuda.synchronize()
    got = tally.read()
    tally.free()
    got["log"], got["log_n"], got["log_fate"] = gnav.log_to_numpy(log)
    return got


def _same(a, b, cap):
    ref = dict(log=b["log"], log_n=b["log_n"], log_fate=b["log_fate"])
    bad = compare_logs(a["log"], a["log_n"], a["log_fate"], ref, cap)
    assert not bad, bad[:10]
    for f in ("touchable", "code", "step", "edep", "energy"):
        assert np.array_equal(a["log"][f], b["log"][f]), f
    for k in EXACT:
        assert a["counters"][k] == b["counters"][k], k
    for f in ("edep_event", "escaped_event", "edep_touchable"):
        assert np.allclose(a[f], b[f], rtol=RTOL, atol=1e-15), f


def test_noalloc_matches_transport_batch_two_calls(ctx, torch_dev, oracle_lib):
    torch = torch_dev
    _, gid_c, _, _ = geom(ctx, "calorimeter", oracle_lib)
    _, gid_t, _, _ = geom(ctx, "tiny", oracle_lib)
    print_case("noalloc call 1: calorimeter 3000 photons at 20 MeV, default grid")
    _, prim, _ = W.calorimeter(n=3000)
    prim.energy[:] = 20.0
    a = _run(ctx, torch, gid_c, prim, 600, True)
    b = _run(ctx, torch, gid_c, prim, 600, False)
    assert a["counters"]["pair"] > 1000
    _same(a, b, 600)
    print_case("noalloc call 2: tiny 1000 photons, grid 5, block 128")
    _, prim2, _ = W.tiny(n=1000)
    a2 = _run(ctx, torch, gid_t, prim2, 256, True, grid=5, block=128)
    b2 = _run(ctx, torch, gid_t, prim2, 256, False, grid=5, block=128)
    assert a2["counters"]["tracks"] >= 1000
    _same(a2, b2, 256)


def test_noalloc_rejects_too_many_slots(ctx, torch_dev, oracle_lib):
    from paper_1209_5235_amd import gnav
    _, gid, _, _ = geom(ctx, "tiny", oracle_lib)
    print_case("noalloc limit")
    _, prim, _ = W.tiny(n=100)
    tally = ctx.tally_create(prim.n_events)
    dev = gnav.primaries_to_device(prim, "cuda")
    b = ctx._batch(gid, dev, block=256, grid=gnav.NOALLOC_MAX_SLOTS // 256 + 1)
    st = gnav.gnav_transport_batch_noalloc(ctx.h, C.byref(b), tally.h, gnav._stream(None))
    assert st == -1  # GNAV_EINVAL, before any device work
    assert b"GNAV_NOALLOC_MAX_SLOTS" in gnav.gnav_last_error(ctx.h)
    b = ctx._batch(gid, dev, block=256, grid=gnav.NOALLOC_MAX_SLOTS // 256)
    st = gnav.gnav_transport_batch_noalloc(ctx.h, C.byref(b), tally.h, gnav._stream(None))
    assert st == gnav.GNAV_OK, gnav.gnav_last_error(ctx.h)
    torch_dev.cuda.synchronize()
    assert tally.read()["counters"]["tracks"] == 100
    tally.free()
