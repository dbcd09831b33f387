"""Run the transport of the host-emulation library on small cases and compare
with the oracle (run in a child process by tests/test_hostemu.py, so that a
trapped bounds check or a guard-page fault ends only the child).

Usage: python tests/hostemu/run_cases.py <emulation dir> <case>[,<case>...] [fork]
Prints one line per case and configuration, "OK" or "BAD <what>", and exits
with status 1 when any differs.
"""
from __future__ import annotations

import importlib.util
import os
import sys
import types

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads as W  # noqa: E402
from tests.gpu_common import EXACT, compare_logs  # noqa: E402

STREAM = types.SimpleNamespace(cuda_stream=0)


def _pair_heavy():
    _, prim, _ = W.calorimeter(n=800)
    prim.energy[:] = 20.0
    return W.geometry.calorimeter(), prim


CASES = {
    "tiny": lambda: (W.geometry.tiny(), W.tiny(n=1500)[1]),
    "tiny_rot": lambda: (W.geometry.tiny(rotated=True), W.primaries.tiny_source(1500, 0)),
    "calorimeter": lambda: (W.geometry.calorimeter(), W.calorimeter(n=1200)[1]),
    "pair_heavy": _pair_heavy,
    "barrel": lambda: (W.geometry.barrel(), W.barrel(n=800)[1]),
    "endcap": lambda: (W.geometry.endcap(), W.endcap(n=1000, seed=4)[1]),
}

# every launch shape and instantiation the library selects from batch fields
CONFIGS = [dict(cap=64), dict(block=128, cap=64), dict(block=256, chunk=64, sort_period=2, cap=64),
           dict(count_work=True, digests=True), dict(order=1, cap=64), dict(precision=1, cap=64),
           dict(precision=2, compare=False), dict(noalloc=True), dict(keep_order=True, cap=64)]
# blocks in concurrent processes: only tallies (device memory) come back
FORK_CONFIGS = [dict(), dict(block=256, chunk=32), dict(count_work=True, sort_period=3)]


def multi_case(gnav, ctx, fork):
    """Events over three geometries (per-event geometry ids): each geometry's
    events against the oracle run on that geometry alone."""
    import torch
    geoms = [W.geometry.tiny(), W.geometry.calorimeter(), W.geometry.barrel()]
    sources = [W.primaries.source_origin_iso, W.primaries.source_beam, W.primaries.source_axis_iso]
    prim, event_geom = W.primaries.batched_events(n_events=24, n_geoms=3, seed=5, median=60.0, lo=10, hi=200,
                                                  sources=sources)
    gids = [ctx.upload_geometry(g, stream=STREAM)[0] for g in geoms]
    eg = torch.from_numpy(np.asarray(event_geom, np.int32) + gids[0])
    refs = []
    for g, desc in enumerate(geoms):
        sel = np.nonzero(np.asarray(event_geom)[prim.event] == g)[0]
        refs.append((sel, oracle.Geometry(desc).transport(prim.subset(sel), seed=0, n_events=prim.n_events)))
    n_bad = 0
    for cfg in ([dict(), dict(block=128, chunk=32)] if fork else [dict(), dict(keep_order=True), dict(block=256)]):
        got = run(gnav, ctx, gids[0], prim, event_geom=eg, **cfg)
        bad = []
        for k in EXACT:
            if got["counters"][k] != sum(r["counters"][k] for _, r in refs):
                bad.append(k)
        for g, (sel, r) in enumerate(refs):
            evs = np.unique(prim.event[sel])
            if not np.allclose(got["edep_event"][evs], r["edep_event"][evs], rtol=1e-9, atol=1e-15):
                bad.append(f"edep_event geometry {g}")
        n_bad += bool(bad)
        print("multi", cfg, "steps", got["counters"]["steps"], "OK" if not bad else "BAD " + ",".join(bad), flush=True)
    return n_bad


def load(emu_dir):
    spec = importlib.util.spec_from_file_location("gnav_hostemu", os.path.join(emu_dir, "gnav.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def run(gnav, ctx, gid, prim, cap=0, digests=False, noalloc=False, compare=True, **kw):
    tally = ctx.tally_create(prim.n_events)
    dev = gnav.primaries_to_device(prim, "cpu")
    log = gnav.make_log(prim.n, cap, "cpu") if cap else None
    dg = gnav.make_digests(prim.n, "cpu") if digests else None
    f = ctx.transport_batch_noalloc if noalloc else ctx.transport_batch
    f(gid, dev, tally, stream=STREAM, log=log, digest=dg, **kw)
    got = tally.read(STREAM)
    tally.free()
    off, _ = ctx.touchable_offset(gid)
    got["edep_touchable"] = got["edep_touchable"][off:off + ctx.geoms[gid][1]]
    if cap:
        got["log"], got["log_n"], got["log_fate"] = gnav.log_to_numpy(log)
    if dg is not None:
        got["digests"] = gnav.digests_to_numpy(dg)
    return got


def differences(got, ref, cap):
    bad = [k for k in EXACT if got["counters"][k] != ref["counters"][k]]
    if not np.allclose(got["edep_event"], ref["edep_event"], rtol=1e-9, atol=1e-15):
        bad.append("edep_event")
    if not np.allclose(got["escaped_event"], ref["escaped_event"], rtol=1e-9, atol=1e-15):
        bad.append("escaped_event")
    if not np.allclose(got["edep_touchable"], ref["edep_touchable"], rtol=1e-9, atol=1e-12):
        bad.append("edep_touchable")
    if cap and compare_logs(got["log"], got["log_n"], got["log_fate"], ref, cap):
        bad.append("logs")
    return bad


def main():
    emu, names = sys.argv[1], sys.argv[2].split(",")
    fork = len(sys.argv) > 3 and sys.argv[3] == "fork"
    gnav = load(emu)
    ctx = gnav.Context(0)
    n_bad = 0
    for name in names:
        if name == "multi":
            n_bad += multi_case(gnav, ctx, fork)
            continue
        desc, prim = CASES[name]()
        gid, _ = ctx.upload_geometry(desc, stream=STREAM)
        ref = oracle.Geometry(desc).transport(prim, seed=0, log_cap=64)
        for cfg in (FORK_CONFIGS if fork else CONFIGS):
            cfg = dict(cfg)
            compare = cfg.pop("compare", True)
            got = run(gnav, ctx, gid, prim, **cfg)
            bad = differences(got, ref, cfg.get("cap", 0)) if compare else []
            if cfg.get("digests"):
                used = got["digests"]["fate"] != 0
                if int(used.sum()) != ref["counters"]["tracks"]:
                    bad.append("digest count")
            if not compare:
                tot = got["edep_event"] + got["escaped_event"]
                e_ev = np.bincount(prim.event, weights=prim.energy, minlength=prim.n_events)
                if not np.allclose(tot, e_ev, rtol=1e-12, atol=0):
                    bad.append("energy per event")
            n_bad += bool(bad)
            print(name, cfg, "steps", got["counters"]["steps"], "OK" if not bad else "BAD " + ",".join(bad),
                  flush=True)
    sys.exit(1 if n_bad else 0)


if __name__ == "__main__":
    main()
