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

# Algorithmic FP64 work per counted unit (add/mul/compare = 1, fma = 2,
# div and sqrt = 1 each), for box-only geometries such as the calorimeter.
# See the table of per-unit costs in the design notes.
FLOPS = {
    "step": 10,          # s_phys = n_lambda / mu, compare, advance (6), depth update (2)
    "frame": 3,          # touchable frame for an axis-aligned placement (3 sub)
    "dist_out": 12,      # box exit: 3 x (sub, |.|, div) + 3 min
    "dist_in": 33,       # translation (3) + box slab entry (30)
    "safety": 8,         # box signed distance: 3 x (|.|, sub) + 2 max
    "inside": 11,        # translation (3) + box classification (8)
    "node": 10,          # voxel index or exit-plane distance
    "mu": 12,            # log-interpolation of three tables
    "compton": 150,      # Butcher-Messel trial(s), rotation, renormalisation
    "pe": 4,
    "pair": 40,
}

PEAK_FP64_TFLOPS = 78.6  # MI355X vector FP64 (256 CUs x 2.4 GHz x 128 flop/clk)


def algorithmic_flops(c):
    geo = c["steps"] - c["shortcuts"]
    return (FLOPS["step"] * c["steps"] + (FLOPS["frame"] + FLOPS["safety"]) * geo
            + FLOPS["dist_out"] * c["dist_out"] + FLOPS["dist_in"] * c["dist_in"]
            + FLOPS["inside"] * c["inside"] + FLOPS["node"] * c["voxel_nodes"]
            + FLOPS["mu"] * (c["tracks"] + c["compton"])
            + FLOPS["compton"] * c["compton"] + FLOPS["pe"] * c["pe"] + FLOPS["pair"] * c["pair"])


def cpu_baseline(n_sample, seed=0):
    import oracle
    import workloads as W
    geoms, prim, _ = W.calorimeter(n=n_sample, seed=seed)
    og = oracle.Geometry(geoms[0])
    t0 = time.perf_counter()
    r = og.transport(prim, seed=0)
    dt = time.perf_counter() - t0
    return r["counters"]["steps"] / dt, dt, r["counters"]["steps"]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=1_000_000, help="photons per batch")
    ap.add_argument("--block", type=int, default=0)
    ap.add_argument("--grid", type=int, default=0)
    ap.add_argument("--cpu-sample", type=int, default=400_000,
                    help="primaries of the same workload for the oracle timing (0: skip)")
    ap.add_argument("--no-cpu", action="store_true")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: this build runs on one GPU only; --gpus must be 1 "
              "(events are independent, see the sharding notes in the design document)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import workloads as W
    from paper_1209_5235_amd import gnav

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    geoms, prim, _ = W.calorimeter(n=args.n, seed=0)
    ctx = gnav.Context(0)
    gid, nt = ctx.upload_geometry(geoms[0])
    prim_d = gnav.primaries_to_device(prim, dev)
    tally = ctx.tally_create(prim.n_events)
    stream = torch.cuda.current_stream()

    def one_batch():
        tally.reset(stream)
        ctx.transport_batch(gid, prim_d, tally, seed=0, block=args.block, grid=args.grid,
                            stream=stream)

    for _ in range(args.warmup):
        one_batch()
    torch.cuda.synchronize()
    # counters of one batch (identical every batch: counter-keyed random numbers)
    tally.reset(stream)
    ctx.transport_batch(gid, prim_d, tally, seed=0, block=args.block, grid=args.grid, stream=stream)
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
        ctx.transport_batch(gid, prim_d, tally, seed=0, block=args.block, grid=args.grid,
                            stream=stream)
        ends[i].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kern_ms = [s.elapsed_time(e) for s, e in zip(starts, ends)]
    avg_kern_s = float(np.mean(kern_ms)) / 1e3
    ms_per_step = wall * 1e3 / args.steps
    value = steps_per_batch * args.steps / wall

    flops = algorithmic_flops(c)
    achieved_tf = flops / avg_kern_s / 1e12
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
            "block": args.block or 256,
            "grid": args.grid or "default",
        },
        "roofline": {
            "bound": "alu",
            "achieved": achieved_tf,
            "peak": PEAK_FP64_TFLOPS,
            "unit": "TFLOP/s",
            "frac": achieved_tf / PEAK_FP64_TFLOPS,
            "traffic": None,
            "kernel": "k_transport<false>",
            "kernel_ms": avg_kern_s * 1e3,
            "flops_per_launch": flops,
        },
        "counters": c,
    }
    if not args.no_cpu and args.cpu_sample > 0:
        rate, dt, nsteps = cpu_baseline(args.cpu_sample)
        out["cpu_baseline"] = {
            "value": rate, "unit": "steps/s", "cores": 1, "kind": "oracle",
            "sample": f"first {args.cpu_sample} primaries of the same calorimeter workload "
                      f"({nsteps} steps in {dt:.1f} s, single thread, brute-force navigation)",
        }
    tally.free()
    ctx.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
