#!/usr/bin/env python3
"""Benchmark: gamma navigation steps/s on one MI355X (FP64 transport).

One "step" of the benchmark is one transport_batch over the whole workload
(1e6 photons in the Pb/Si sampling calorimeter), i.e. one pass of the hot
path: locate, voxel ComputeStep/ComputeSafety, box distances, physics and
tallies.  The metric counts navigation steps (transport-loop iterations of
single tracks) per second.  Primaries are resident in HBM before timing
starts; geometry upload is excluded, as the paper times only the parallel
phase (Alg. 2, phase 5).

Prints one JSON line.  Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Algorithmic work per counted unit (add/mul = 1, fma = 2, div and sqrt = 1
# each), the method's own costs whatever the kernel does to save work: a
# frame map of a point and a direction (rotation + translation, per
# placement level of a touchable frame and per daughter candidate examined),
# entry / exit distances, isotropic distances (safeties, also charged for
# point-in-solid tests) by solid family, a voxel node visit, the physics and
# advance of a step, and an interaction (attenuation lookup, sampling,
# rotation).  The counts come from the kernel's work counters (a counting
# launch of the same batch).
FAMILIES = ("box", "tubs", "cons", "orb", "trd", "sphere")
UNIT_FLOPS = {
    "frame": 33,
    "dist_in": {"box": 30, "tubs": 110, "cons": 150, "orb": 20, "trd": 60, "sphere": 200},
    "dist_out": {"box": 15, "tubs": 90, "cons": 120, "orb": 15, "trd": 40, "sphere": 150},
    "safety": {"box": 8, "tubs": 20, "cons": 30, "orb": 7, "trd": 30, "sphere": 30},
    "node": 8,
    "step": 10,
    "interaction": 150,
}

PEAK_FP64_TFLOPS = 78.6   # MI355X vector FP64 (256 CUs x 2.4 GHz x 128 flop/clk)
PEAK_FP32_TFLOPS = 157.3  # MI355X vector FP32
PEAK_HBM_GBS = 8000.0     # MI355X HBM3E


def algorithmic_flops(c, precision=0):
    """(FP64 flops, FP32 flops) of one launch from its counters.  In the FP32
    forms the daughter entry distances evaluated in FP32 (their share of all
    entry distances) count as FP32 work, and in the pure form the mother exit
    distance and safeties too."""
    din = sum(UNIT_FLOPS["dist_in"][f] * c["dist_in_" + f] for f in FAMILIES)
    dout = sum(UNIT_FLOPS["dist_out"][f] * c["dist_out_" + f] for f in FAMILIES)
    saf = sum(UNIT_FLOPS["safety"][f] * (c["safety_" + f] + c["inside_" + f]) for f in FAMILIES)
    other = (UNIT_FLOPS["frame"] * c["frame_maps"] + UNIT_FLOPS["node"] * c["voxel_nodes"]
             + UNIT_FLOPS["step"] * c["steps"] + UNIT_FLOPS["interaction"] * (c["pe"] + c["compton"] + c["pair"]))
    f32_share = c["dist_in_f32"] / max(c["dist_in"] + c["dist_in_f32"], 1) if precision else 0.0
    f32 = din * f32_share + ((dout + saf) if precision == 2 else 0.0)
    f64 = din + dout + saf + other - f32
    return float(f64), float(f32)


def roofline(counters, kernel_ms, kernel, precision=0, traffic=None):
    """Roofline object of one launch: ALU bound, achieved = algorithmic flops /
    average launch time; with FP32 work the peak is the time-weighted mix of the
    FP64 and FP32 peaks (the rate the launch would reach at both peaks)."""
    f64, f32 = algorithmic_flops(counters, precision)
    t = kernel_ms / 1e3
    achieved = (f64 + f32) / t / 1e12
    peak = (f64 + f32) / (f64 / PEAK_FP64_TFLOPS + f32 / PEAK_FP32_TFLOPS) if f64 + f32 > 0 else PEAK_FP64_TFLOPS
    out = {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "TFLOP/s", "frac": achieved / peak,
           "traffic": traffic, "kernel": kernel, "kernel_ms": kernel_ms, "flops_fp64": f64, "flops_fp32": f32,
           "fp64_frac": f64 / t / 1e12 / PEAK_FP64_TFLOPS, "fp32_frac": f32 / t / 1e12 / PEAK_FP32_TFLOPS}
    if traffic:
        out["hbm_gbs"] = traffic / t / 1e9
        out["hbm_frac"] = traffic / t / 1e9 / PEAK_HBM_GBS
    return out


def kernel_name(block, axis_boxes, precision=0, order=0):
    return (f"gnav::pool{block}{'_axis_boxes' if axis_boxes else ''}::k_transport<false, false, "
            f"{order}, {precision}>")


def _oracle_slice(args):
    """Oracle transport of primaries [lo, hi) of the calorimeter workload (worker);
    `voxels` selects the oracle's cell-grid search instead of brute force."""
    n_sample, lo, hi, voxels = args
    import oracle
    import workloads as W
    geoms, prim, _ = W.calorimeter(n=n_sample, seed=0)
    og = oracle.Geometry(geoms[0])
    og.set_voxels(voxels)
    sub = prim.subset(np.arange(lo, hi))
    t0 = time.perf_counter()
    r = og.transport(sub, seed=0, n_events=prim.n_events)
    return r["counters"]["steps"], time.perf_counter() - t0


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(n_sample, workers, n_full=0):
    """Oracle steps/s on host cores: one thread over the sample, then `workers`
    processes over equal slices of it (each a plain single-threaded oracle);
    both with brute-force navigation and with the oracle's voxel mode.  With
    n_full, the oracle also transports the whole headline workload (n_full
    photons, `workers` processes, untimed) and keeps every track's digest and
    the tallies, which the GPU's launch is compared with."""
    out = {}
    if n_full > 0:
        import oracle
        from oracle import parity
        import workloads as W
        geoms, prim, _ = W.calorimeter(n=n_full, seed=0)
        oracle.build()
        out["reference"] = parity.oracle_run(geoms[0], prim, seed=0, workers=max(1, workers))
    for voxels in (False, True):
        tag = "voxel_" if voxels else ""
        steps1, dt1 = _oracle_slice((n_sample, 0, n_sample, voxels))
        out[tag + "single"] = (steps1 / dt1, dt1, steps1)
        if workers > 1:
            import multiprocessing as mp
            cuts = np.linspace(0, n_sample, workers + 1).astype(int)
            t0 = time.perf_counter()
            with mp.get_context("fork").Pool(workers) as pool:
                res = pool.map(_oracle_slice, [(n_sample, int(a), int(b), voxels)
                                               for a, b in zip(cuts[:-1], cuts[1:])])
            dt = time.perf_counter() - t0
            steps = sum(r[0] for r in res)
            out[tag + "all"] = (steps / dt, dt, steps)
    return out


def kernel_source_hash():
    """Hash of the transport kernel sources (ties stored counter readings to a build)."""
    import hashlib
    h = hashlib.sha256()
    for f in ("gnav_transport.hip", "gnav_physics.h", "gnav_device.h", "gnav_internal.h", "gnav_learned.h"):
        with open(os.path.join(ROOT, "paper_1209_5235_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_transport_traffic.json")


def stored_traffic(kernel, workload):
    """HBM bytes per launch of `kernel` on `workload` from the committed counter
    summary (FETCH_SIZE and WRITE_SIZE scaled by a device copy), or None when no
    reading was taken for that kernel and workload with the current sources."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    with open(TRAFFIC_FILE) as fh:
        t = json.load(fh)
    if t.get("kernel_source_hash") != kernel_source_hash():
        return None
    for e in t.get("entries", []):
        if e.get("kernel") == kernel and e.get("workload") == workload:
            return e.get("bytes_per_launch")
    return None


def compare_digests(got, ref, rtol=1e-9, atol=1e-12):
    """Track slots whose digests differ (hash, record count or fate unequal, or the
    sums of step lengths and deposits beyond the tolerance), and the used slots."""
    bad = (got["hash"] != ref["hash"]) | (got["n"] != ref["n"]) | (got["fate"] != ref["fate"])
    for f in ("sum_step", "sum_edep"):
        a, b = got[f], ref[f]
        bad |= ~(np.abs(a - b) <= rtol * np.maximum(np.abs(a), np.abs(b)) + atol)
    return int(bad.sum()), int((ref["fate"] != 0).sum())


def max_rel(a, b):
    d = np.abs(a - b) / np.maximum(np.maximum(np.abs(a), np.abs(b)), 1e-300)
    d[a == b] = 0.0
    return float(d.max()) if d.size else 0.0


def time_batches(ctx, gid, prim_d, tally, stream, reps, **kw):
    """Median kernel time (ms, HIP events on the launch stream) of `reps` batches
    after one warm-up, the tallies of the last one, and the counters of an extra
    counting batch (work counters by solid family)."""
    import torch
    tally.reset(stream)
    ctx.transport_batch(gid, prim_d, tally, stream=stream, **kw)
    ms = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        tally.reset(stream)
        a.record(stream)
        ctx.transport_batch(gid, prim_d, tally, stream=stream, **kw)
        b.record(stream)
        torch.cuda.synchronize()
        ms.append(a.elapsed_time(b))
    res = tally.read(stream)
    tally.reset(stream)
    ctx.transport_batch(gid, prim_d, tally, stream=stream, count_work=True, **kw)
    work = tally.read(stream)["counters"]
    return float(np.median(ms)), res, work


def oracle_rates(desc, prim, n_sample):
    """Oracle steps/s (one thread) on the first n_sample primaries, brute force and
    voxel mode; the same deterministic subset for both."""
    import oracle
    sub = prim.subset(np.arange(min(n_sample, prim.n)))
    out = {}
    for voxels in (False, True):
        og = oracle.Geometry(desc)
        og.set_voxels(voxels)
        t0 = time.perf_counter()
        r = og.transport(sub, seed=0, n_events=prim.n_events)
        dt = time.perf_counter() - t0
        out["voxel" if voxels else "brute_force"] = r["counters"]["steps"] / dt
    out["sample"] = f"first {sub.n} primaries, one thread"
    return out


def _progress(what):
    print(f"done: {what}", file=sys.stderr, flush=True)


def _same_counters(a, b):
    return all(a["counters"][k] == b["counters"][k]
               for k in ("steps", "pe", "compton", "pair", "crossings", "escaped", "tracks"))


def _deposit_chi2(a, b, bins):
    ha = np.histogram(a, bins)[0].astype(float)
    hb = np.histogram(b, bins)[0].astype(float)
    m = (ha + hb) > 0
    return float(np.sum((ha[m] - hb[m]) ** 2 / (ha[m] + hb[m])) / max(int(m.sum()) - 1, 1))


def barrel_variants(ctx, gnav, n, reps, oracle_sample=0):
    """Barrel workload: FP64 against the FP32-distance forms (pure and screened)
    and the bound candidate order, each with its roofline."""
    import torch
    import workloads as W
    geoms, prim, _ = W.barrel(n=n, seed=0)
    gid, _ = ctx.upload_geometry(geoms[0])
    stream = torch.cuda.current_stream()
    prim_d = gnav.primaries_to_device(prim, "cuda")
    tally = ctx.tally_create(prim.n_events)
    wl = f"barrel_{n:.0e}"
    out = {"workload": f"barrel: 64 tubs layers x 128 segments, 2x16 cons rings, 32 orbs; {n:.0e} "
                       "photons from the axis, log-uniform 0.05-20 MeV, seed 0"}
    base_ms, base, base_w = time_batches(ctx, gid, prim_d, tally, stream, reps)
    steps = base["counters"]["steps"]

    def entry(ms, res, work, precision=0, order=0):
        k = kernel_name(64, False, precision, order)
        e = {"ms": ms, "steps_per_s": res["counters"]["steps"] / ms * 1e3, "speedup": base_ms / ms,
             "dist_in_fp64": work["dist_in"], "dist_in_fp32": work["dist_in_f32"],
             "same_counters": _same_counters(res, base),
             "roofline": roofline(work, ms, k, precision, stored_traffic(k, wl))}
        d = np.abs(res["edep_event"] - base["edep_event"]) / np.maximum(base["edep_event"], 1e-300)
        e["max_rel_event_deposit_diff"] = float(d[base["edep_event"] > 0].max())
        return e

    out["fp64"] = {"ms": base_ms, "steps_per_s": steps / base_ms * 1e3, "steps": steps,
                   "dist_in_fp64": base_w["dist_in"],
                   "roofline": roofline(base_w, base_ms, kernel_name(64, False), 0,
                                        stored_traffic(kernel_name(64, False), wl))}
    if oracle_sample > 0:
        out["fp64"]["oracle_steps_per_s"] = oracle_rates(geoms[0], prim, oracle_sample)
    _progress("barrel fp64")
    out["fp64_bound_order"] = entry(*time_batches(ctx, gid, prim_d, tally, stream, reps, order=1), order=1)
    _progress("barrel bound order")
    out["fp32_screened"] = entry(*time_batches(ctx, gid, prim_d, tally, stream, reps, precision=1), precision=1)
    _progress("barrel fp32 screened")
    pure = entry(*time_batches(ctx, gid, prim_d, tally, stream, reps, precision=2), precision=2)
    # deposit histograms: pure FP32 (transport seed 0) against FP64 on an independent
    # transport stream (seed 1), next to FP64 seed 0 against FP64 seed 1 (the
    # statistical reference); chi-square per degree of freedom, 40 log bins
    tally.reset(stream)
    ctx.transport_batch(gid, prim_d, tally, stream=stream, precision=2)
    pr = tally.read(stream)
    tally.reset(stream)
    ctx.transport_batch(gid, prim_d, tally, stream=stream, seed=1)
    ind = tally.read(stream)
    bins = np.logspace(-3, np.log10(25.0), 41)
    pure["chi2_per_ndf_fp32_vs_fp64_independent_seed"] = _deposit_chi2(pr["edep_event"], ind["edep_event"], bins)
    pure["chi2_per_ndf_fp64_vs_fp64_independent_seed"] = _deposit_chi2(base["edep_event"], ind["edep_event"],
                                                                      bins)
    pure["pushes"] = pr["counters"]["pushes"]
    pure["stuck"] = pr["counters"]["stuck"]
    out["fp32_pure"] = pure
    _progress("barrel fp32 pure")
    # per-query FP32 error against FP64 (the FP64 query path equals the oracle per query)
    rng = np.random.Generator(np.random.Philox(key=77))
    q = 100_000
    pts = np.column_stack([rng.uniform(-1500, 1500, q), rng.uniform(-1500, 1500, q),
                           rng.uniform(-2900, 2900, q)])
    dirs = W.primaries.isotropic(rng, q)
    pt, dt = torch.from_numpy(pts).cuda(), torch.from_numpy(dirs).cuda()
    s64, l64, _ = ctx.compute_step(gid, pt, dt, with_next=False)
    s32, l32, _ = ctx.compute_step(gid, pt, dt, with_next=False, precision=2)
    s64, l64, s32, l32 = (x.cpu().numpy() for x in (s64, l64, s32, l32))
    fin = np.isfinite(s64) & np.isfinite(s32)
    err = np.abs(s32[fin] - s64[fin])
    out["fp32_pure"]["per_query"] = {
        "queries": q, "limiter_agreement": float(np.mean(l32 == l64)),
        "abs_err_median_mm": float(np.median(err)), "abs_err_p99_mm": float(np.quantile(err, 0.99)),
        "rel_err_p99": float(np.quantile(err / np.maximum(s64[fin], 1.0), 0.99))}
    tally.free()
    return out


def learned_config(ctx, gnav, n, reps, train_crossings, epochs=1):
    """Learned candidate ordering on the barrel: the network is trained on the GPU
    on crossings recorded from FP64 runs (primary and transport seed 1), then the
    n evaluation photons (seed 0) run with the plain voxel walk, the bound order
    (nearest enclosing cylinder first, no network) and the learned order, on
    bounding-box voxel node lists (the smart voxels of Geant4, whose nodes hold up
    to 64 candidates; the network's 64 outputs are the positions in such a node).
    The shape-aware node lists' plain walk, which leaves the network nothing to
    order, is timed beside them."""
    import torch
    import workloads as W
    from paper_1209_5235_amd import learned
    geoms, prim, _ = W.barrel(n=n, seed=0)
    desc = geoms[0]
    gid, _ = ctx.upload_geometry(desc, voxel_lists=1)
    n_class = ctx.ordering_classes(gid)
    stream = torch.cuda.current_stream()
    wl = f"barrel_bbox_{n:.0e}"
    out = {"workload": f"barrel with bounding-box voxel node lists; {n:.0e} photons, seed 0; network "
                       f"6 features + one-hot of {n_class} mothers, 128-128 ReLU, 64 logits, bf16 MFMA"}
    # training crossings: size the recording run from a small one's yield
    t0 = time.perf_counter()
    _, pprim, _ = W.barrel(n=100_000, seed=1)
    rec = learned.record_crossings(ctx, gid, gnav.primaries_to_device(pprim, "cuda"), pprim.n_events,
                                   capacity=16, seed=1)
    per_photon = float(rec["count"].cpu()[0]) / pprim.n
    n_train = int(min(4e7, max(1e5, np.ceil(train_crossings / max(per_photon, 1e-9) * 1.02))))
    del rec, pprim
    _, tprim, _ = W.barrel(n=n_train, seed=1)
    rec = learned.record_crossings(ctx, gid, gnav.primaries_to_device(tprim, "cuda"), tprim.n_events,
                                   capacity=int(train_crossings), seed=1)
    seen = int(rec["count"].cpu()[0])
    x, cls, label = learned.records_to_tensors(rec)
    del rec, tprim
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    net, losses = learned.train(ctx, n_class, x, cls, label, epochs=epochs, batch=4096, log_every=2000)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    n_records = int(x.shape[0])
    del x, cls, label
    _, eprim, _ = W.barrel(n=20_000, seed=7)
    erec = learned.record_crossings(ctx, gid, gnav.primaries_to_device(eprim, "cuda"), eprim.n_events,
                                    capacity=2_000_000, seed=7)
    ex, ec, el = learned.records_to_tensors(erec)
    acc = learned.accuracy(net, ex, ec, el)
    del erec, ex, ec, el
    out["training"] = {"crossings": n_records, "crossings_seen": seen, "photons": n_train,
                       "crossings_per_photon": per_photon, "epochs": epochs, "batch": 4096,
                       "record_s": t1 - t0, "train_s": t2 - t1, "loss_first_last": [losses[0], losses[-1]],
                       "heldout_accuracy_top1": acc}
    _progress("learned: training")
    ctx.set_mlp(gid, net)
    prim_d = gnav.primaries_to_device(prim, "cuda")
    tally = ctx.tally_create(prim.n_events)
    runs = {}
    for name, order in (("plain", 0), ("bound_order", 1), ("learned", 2)):
        ms, res, work = time_batches(ctx, gid, prim_d, tally, stream, reps, order=order)
        k = kernel_name(64, False, 0, order)
        runs[name] = {"ms": ms, "steps_per_s": res["counters"]["steps"] / ms * 1e3,
                      "dist_in": work["dist_in"], "scored_steps": work["scored"],
                      "roofline": roofline(work, ms, k, 0, stored_traffic(k, wl)), "_res": res}
        _progress(f"learned: {name}")
    # identical results: every track's digest of the learned and bound orders equals the plain walk's
    digs = {}
    for name, order in (("plain", 0), ("bound_order", 1), ("learned", 2)):
        d = gnav.make_digests(prim.n, "cuda")
        tally.reset(stream)
        ctx.transport_batch(gid, prim_d, tally, stream=stream, order=order, digest=d)
        torch.cuda.synchronize()
        digs[name] = gnav.digests_to_numpy(d)
        del d
    for name in ("bound_order", "learned"):
        mism, used = compare_digests(digs[name], digs["plain"], rtol=0.0, atol=0.0)
        runs[name]["identical_tracks"] = bool(mism == 0 and _same_counters(runs[name]["_res"], runs["plain"]["_res"]))
        runs[name]["tracks_compared"] = used
        runs[name]["speedup_vs_plain"] = runs["plain"]["ms"] / runs[name]["ms"]
    runs["learned"]["speedup_vs_bound_order"] = runs["bound_order"]["ms"] / runs["learned"]["ms"]
    for r in runs.values():
        r.pop("_res")
    out.update(runs)
    if runs["learned"]["scored_steps"] == 0:
        out["note"] = "the network scored no step: the learned line is the bound order's walk"
    ctx.set_mlp(gid, None)
    net.free()
    tally.free()
    # the shape-aware node lists (the library default) for context
    gid_s, _ = ctx.upload_geometry(desc)
    tally = ctx.tally_create(prim.n_events)
    ms, res, work = time_batches(ctx, gid_s, prim_d, tally, stream, reps)
    out["shape_aware_plain"] = {"ms": ms, "steps_per_s": res["counters"]["steps"] / ms * 1e3,
                                "dist_in": work["dist_in"]}
    tally.free()
    return out


# The paper's Table 1 (Spheres, N = 1e5, free path only), milliseconds, as context.
PAPER_TABLE1_MS = {"regular": {"gtx470": 33, "cpu_1_thread": 442, "cpu_12_threads": 54},
                   "random": {"gtx470": 114, "cpu_1_thread": 458, "cpu_12_threads": 56}}


def paper_free_path(ctx, gnav, reps, oracle_sample):
    """Alg. 1 free path alone on the paper's Spheres geometry with its Random and
    Regular particle sets (mu = rho x 0.06146 cm2/g, Eq. 9), N = 1e5."""
    import torch
    import workloads as W
    desc = W.geometry.spheres()
    gid, _ = ctx.upload_geometry(desc)
    stream = torch.cuda.current_stream()
    out = {"workload": "Spheres: 8000 Al orbs r = 100 mm on a 20^3 grid in a 5 m vacuum cube, "
                       "particles from the centre, mu = rho x 0.06146 cm2/g, N = 1e5, FP64"}
    for name, (pos, dirs, life) in (("random", W.primaries.paper_random(100_000, seed=0)),
                                    ("regular", W.primaries.paper_regular())):
        p, d, y = (torch.from_numpy(a).cuda() for a in (pos, dirs, life))
        ctx.free_path(gid, p, d, y, mu_mass=0.06146, stream=stream)
        ms = []
        for _ in range(reps):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            t, nb = ctx.free_path(gid, p, d, y, mu_mass=0.06146, stream=stream)
            b.record(stream)
            torch.cuda.synchronize()
            ms.append(a.elapsed_time(b))
        m = float(np.median(ms))
        e = {"gpu_ms": m, "particles_per_s": len(life) / m * 1e3,
             "boundaries_per_particle": float(nb.double().mean().cpu()),
             "paper_ms_context": PAPER_TABLE1_MS[name]}
        if oracle_sample > 0:
            import oracle
            og = oracle.Geometry(desc)
            og.set_paper_mode(True, 0.06146)
            t0 = time.perf_counter()
            for i in range(oracle_sample):
                og.free_path(pos[i], dirs[i], 1.0, float(life[i]))
            dt = time.perf_counter() - t0
            e["oracle_particles_per_s"] = oracle_sample / dt
            e["oracle_sample"] = f"first {oracle_sample} particles, one thread, brute-force navigation"
        out[name] = e
    return out


def tiny_config(ctx, gnav, reps, with_oracle):
    """The small configuration: eight boxes in a vacuum world, 1e4 photons of
    1 MeV from the origin (the parity case the oracle runs in seconds)."""
    import torch
    import workloads as W
    geoms, prim, _ = W.tiny(n=10_000, seed=0)
    gid, _ = ctx.upload_geometry(geoms[0])
    prim_d = gnav.primaries_to_device(prim, "cuda")
    tally = ctx.tally_create(prim.n_events)
    ms, res, _ = time_batches(ctx, gid, prim_d, tally, torch.cuda.current_stream(), reps)
    tally.free()
    steps = res["counters"]["steps"]
    out = {"workload": "tiny: 8 water/Pb boxes in a vacuum world, 1e4 photons of 1 MeV from the origin",
           "ms": ms, "steps": steps, "steps_per_s": steps / ms * 1e3}
    if with_oracle:
        out["oracle_steps_per_s"] = oracle_rates(geoms[0], prim, prim.n)
    return out


def batched_config(ctx, gnav, reps):
    """Uneven events over eight resident geometries in one launch: autotuned
    launch settings, then the tuned launch captured in a HIP graph."""
    import torch
    import workloads as W
    t0 = time.perf_counter()
    geoms, prim, event_geom = W.batched()
    gids = [ctx.upload_geometry(g)[0] for g in geoms]
    prim_d = gnav.primaries_to_device(prim, "cuda")
    eg = torch.from_numpy(np.asarray(event_geom, np.int32) + gids[0]).cuda()
    tally = ctx.tally_create(prim.n_events)
    stream = torch.cuda.current_stream()
    setup_s = time.perf_counter() - t0
    kw = dict(event_geom=eg)
    best = ctx.autotune(gids[0], prim_d, tally, trials=2, stream=stream, **kw)
    ms_e, res, work = time_batches(ctx, gid=gids[0], prim_d=prim_d, tally=tally, stream=stream, reps=reps,
                                   tuned=True, **kw)
    g = ctx.graph_create(gids[0], prim_d, tally, stream=stream, tuned=True, **kw)
    ms_g = []
    for _ in range(reps + 1):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        tally.reset(stream)
        a.record(stream)
        ctx.graph_launch(g, stream)
        b.record(stream)
        torch.cuda.synchronize()
        ms_g.append(a.elapsed_time(b))
    gr = tally.read(stream)
    ctx.graph_free(g)
    tally.free()
    steps = res["counters"]["steps"]
    same = gr["counters"] == res["counters"]
    return {"workload": f"batched: {prim.n_events} events, {prim.n} photons (lognormal sizes, median "
                        "2000, 10-50000) over 8 resident geometries (tiny, calorimeter, barrel, 5 barrel "
                        "variants), log-uniform 0.05-20 MeV",
            "photons": int(prim.n), "steps": steps, "tuned": best,
            "ms_eager_tuned": ms_e, "ms_graph_tuned": float(np.median(ms_g[1:])),
            "steps_per_s": steps / float(np.median(ms_g[1:])) * 1e3,
            "graph_same_counters": bool(same), "setup_s": setup_s,
            "roofline": roofline(work, ms_e, kernel_name(best["block"], False), 0,
                                 stored_traffic(kernel_name(best["block"], False), "batched_4096"))}


def headline(args, ctx, gnav, cpu, workers):
    """The calorimeter throughput line with its roofline and CPU baseline."""
    import torch
    import workloads as W
    dev = torch.device("cuda:0")
    geoms, prim, _ = W.calorimeter(n=args.n, seed=0)
    gid, nt = ctx.upload_geometry(geoms[0])
    prim_d = gnav.primaries_to_device(prim, dev)
    tally = ctx.tally_create(prim.n_events)
    stream = torch.cuda.current_stream()
    kw = dict(seed=0, block=args.block, grid=args.grid)

    for _ in range(args.warmup):
        tally.reset(stream)
        ctx.transport_batch(gid, prim_d, tally, stream=stream, **kw)
    torch.cuda.synchronize()
    # counters of one batch (identical every batch: counter-keyed random numbers);
    # the work counters (candidate evaluations etc.) come from a counting launch
    tally.reset(stream)
    ctx.transport_batch(gid, prim_d, tally, stream=stream, count_work=True, **kw)
    c = tally.read(stream)["counters"]
    steps_per_batch = c["steps"]

    # timed region: K batches; per-launch durations from events on the launch stream
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        tally.reset(stream)
        starts[i].record(stream)
        ctx.transport_batch(gid, prim_d, tally, stream=stream, **kw)
        ends[i].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    print(f"timed region done: {args.steps} batches in {wall:.3f} s", file=sys.stderr, flush=True)
    kern_ms = [s.elapsed_time(e) for s, e in zip(starts, ends)]
    avg_kern_s = float(np.mean(kern_ms)) / 1e3
    ms_per_step = wall * 1e3 / args.steps
    value = steps_per_batch * args.steps / wall

    # 64-slot blocks on a geometry of unrotated boxes run the axis-aligned box build
    block = args.block or 64
    d0 = geoms[0]
    axis_boxes = (block == 64 and bool(np.all(np.asarray(d0.solid_type) == 0)) and
                  bool(np.all(np.asarray(d0.pv_rot).reshape(-1, 9) == np.eye(3).ravel())))
    kernel = kernel_name(block, axis_boxes)
    roof = roofline(c, avg_kern_s * 1e3, kernel, 0, stored_traffic(kernel, f"calorimeter_{args.n:.0e}"))
    roof["kernel_source_hash"] = kernel_source_hash()
    out = {
        "metric": "gamma navigation steps/s on 1 GPU",
        "value": value,
        "unit": "steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": "sampling calorimeter: 50 Pb 5 mm / Si 10 mm layers x 20x20 cells "
                        "(3-level nesting, voxels), 1e6 photons along +z, log-uniform "
                        "0.1-10 MeV, Gaussian beam sigma 10 mm, FP64, Philox seed 0",
            "photons_per_batch": prim.n,
            "nav_steps_per_batch": steps_per_batch,
            "block": args.block or 64,
            "grid": args.grid or "default",
            "claim_order": "decreasing energy (library default)",
        },
        "roofline": roof,
        "counters": c,
    }
    # every track of the timed workload against the oracle's digests (computed by the
    # CPU-baseline leg over the same photons): a mismatch is a rounding-edge flip or a
    # bug (the GPU tests classify them by the oracle's decision margins); here each
    # counts against the bar of 1e-5 of the tracks
    ref = cpu.get("reference") if cpu is not None else None
    if ref is not None:
        d = gnav.make_digests(prim.n, dev)
        tally.reset(stream)
        ctx.transport_batch(gid, prim_d, tally, stream=stream, digest=d, **kw)
        torch.cuda.synchronize()
        mism, used = compare_digests(gnav.digests_to_numpy(d), ref["digest"])
        del d
        tally.reset(stream)
        ctx.transport_batch(gid, prim_d, tally, stream=stream, **kw)
        t = tally.read(stream)
        out["parity"] = {
            "tracks": used, "mismatching_tracks": mism, "mismatch_rate": mism / max(used, 1),
            "bar": "mismatching tracks (flips included) below 1e-5 of the tracks",
            "max_rel_event_deposit": max_rel(t["edep_event"], ref["edep_event"]),
            "max_rel_touchable_deposit": max_rel(t["edep_touchable"][:nt], ref["edep_touchable"]),
            "counters_equal": all(t["counters"][k] == ref["counters"][k]
                                  for k in ("steps", "pe", "compton", "pair", "crossings", "escaped",
                                            "cutoff", "pushes", "stuck", "truncated", "tracks"))}
    if cpu is not None:
        rate, dt, nsteps = cpu["single"]
        out["cpu_baseline"] = {
            "value": rate, "unit": "steps/s", "cores": 1, "kind": "oracle",
            "cpu": f"{cpu_model()}, {os.cpu_count()} logical CPUs visible",
            "sample": f"first {args.cpu_sample} primaries of the same calorimeter workload "
                      f"({nsteps} steps in {dt:.1f} s, one thread, brute-force navigation)",
        }
        if "all" in cpu:
            rate, dt, nsteps = cpu["all"]
            out["cpu_baseline_all_cores"] = {
                "value": rate, "unit": "steps/s", "cores": workers, "kind": "oracle",
                "sample": f"the same {args.cpu_sample} primaries in {workers} single-threaded "
                          f"oracle processes ({nsteps} steps in {dt:.1f} s wall)"}
        # the oracle's own cell-grid search: a faster CPU method, same answers
        rate, dt, nsteps = cpu["voxel_single"]
        out["cpu_baseline_voxel"] = {
            "value": rate, "unit": "steps/s", "cores": 1, "kind": "oracle, voxel mode",
            "sample": f"the same {args.cpu_sample} primaries, one thread, cell-grid navigation "
                      f"({nsteps} steps in {dt:.1f} s)"}
        if "voxel_all" in cpu:
            rate, dt, nsteps = cpu["voxel_all"]
            out["cpu_baseline_voxel_all_cores"] = {
                "value": rate, "unit": "steps/s", "cores": workers, "kind": "oracle, voxel mode",
                "sample": f"the same {args.cpu_sample} primaries in {workers} single-threaded "
                          f"processes, cell-grid navigation ({nsteps} steps in {dt:.1f} s wall)"}
    tally.free()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=1_000_000, help="photons per batch")
    ap.add_argument("--block", type=int, default=0)
    ap.add_argument("--grid", type=int, default=0)
    ap.add_argument("--cpu-sample", type=int, default=1_000_000,
                    help="primaries of the same workload for the oracle timing (0: skip)")
    ap.add_argument("--cpu-workers", type=int, default=0,
                    help="oracle processes for the all-cores figure (0: min(16, cpus))")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--barrel-n", type=int, default=10_000_000,
                    help="photons of the barrel variant comparison (0: skip)")
    ap.add_argument("--train-crossings", type=float, default=1e8,
                    help="recorded crossings that train the learned order (0: skip)")
    ap.add_argument("--learned-n", type=int, default=10_000_000,
                    help="evaluation photons of the learned-order comparison")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched-events config")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run one 256 MiB device-to-device copy (reference for HBM counters)")
    ap.add_argument("--sections", default="headline,tiny,barrel,learned,paper,batched",
                    help="comma-separated parts to run (profiling runs pick one); without "
                         "'headline' the line carries only the parts that ran")
    args = ap.parse_args()
    sections = set(args.sections.split(","))
    unknown = sections - {"headline", "tiny", "barrel", "learned", "paper", "batched"}
    if unknown:
        ap.error(f"unknown sections {sorted(unknown)}")

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: the library drives one GPU; --gpus must be 1 (events are independent: "
              "a multi-GPU run would split the event range and sum the tallies)",
              file=sys.stderr)
        sys.exit(2)

    # the CPU baseline runs first, in processes forked before any GPU use
    cpu, workers = None, 0
    if "headline" in sections and not args.no_cpu and args.cpu_sample > 0:
        workers = args.cpu_workers or min(16, os.cpu_count() or 1)
        cpu = cpu_baseline(args.cpu_sample, workers, n_full=args.n)
        print(f"cpu baseline done: { {k: v for k, v in cpu.items() if k != 'reference'} }", file=sys.stderr,
              flush=True)

    import torch
    from paper_1209_5235_amd import gnav

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    ctx = gnav.Context(0)
    if args.calibrate_copy:
        src = torch.ones(32 << 20, dtype=torch.float64, device="cuda:0")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    out = headline(args, ctx, gnav, cpu, workers) if "headline" in sections else {}
    if "tiny" in sections:
        out["tiny"] = tiny_config(ctx, gnav, 5, not args.no_cpu)
        _progress("tiny config")
    if "barrel" in sections and args.barrel_n > 0:
        out["variants"] = barrel_variants(ctx, gnav, args.barrel_n, 3, 0 if args.no_cpu else 20_000)
        print("barrel variants done", file=sys.stderr, flush=True)
    if "learned" in sections and args.train_crossings > 0:
        out["learned_order"] = learned_config(ctx, gnav, args.learned_n, 3, args.train_crossings)
        print("learned-order config done", file=sys.stderr, flush=True)
    if "paper" in sections:
        out["paper_free_path"] = paper_free_path(ctx, gnav, 5, 0 if args.no_cpu else 3000)
        print("paper free-path config done", file=sys.stderr, flush=True)
    if "batched" in sections and not args.no_batched:
        out["batched"] = batched_config(ctx, gnav, 3)
        print("batched config done", file=sys.stderr, flush=True)
    ctx.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
