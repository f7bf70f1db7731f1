#!/usr/bin/env python
"""Throughput of one time-split Boltzmann step (stream + collide) on one MI355X.

Workload (default): the 64x64-cell driven cavity with a 20^3 velocity grid on
[-5, 5], Kn = 0.05, lid velocity 0.1, 20000 Monte Carlo pairs per cell per
step, CFL 0.5, second-order streaming, FP32 h with FP64 moment/correction sums.
The state starts at rest (h = 0) and evolves through the warm-up steps, so the
timed steps act on a developing cavity flow; all data stay resident in HBM.

One step = boltz_stream (wall densities + streaming kernels) followed by
boltz_collide in place (sampling, gain/loss, correction in one kernel):
exactly what boltz_step enqueues, with HIP events recorded between the two
calls on the launch stream to time each kernel group.

Prints one JSON line: node-updates/s (value), pairs/s, the roofline of the
dominant kernel, and the FP64 CPU oracle's throughput on a bounded sample of
the same workload (a baseline only).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# One vector operation per lane per clock on every SIMD: 256 CUs x 4 SIMD x
# 16 lanes x 2.4 GHz = 39.3e12 lane-ops/s (no FMA doubling).
ALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12
# Algorithmic operations of one Monte Carlo sample (two Philox4x32-10 calls,
# six inverse-CDF searches, direction map, kinematics, cell lookup, weight and
# the gain/loss update) and of one node of the update + correction; the count
# is itemised in the design notes.
OPS_PER_PAIR = 319
OPS_PER_NODE = 60
# Algorithmic HBM bytes per phase-space node: FP32 read + FP32 write.
BYTES_PER_NODE_KERNEL = 8


def _json_line(d):
    print(json.dumps(d), flush=True)


def cpu_baseline(preset, seconds_budget: float):
    """FP64 oracle on the host cores: full steps of the same workload."""
    import numpy as np

    import oracle

    threads = min(os.cpu_count() or 1, int(os.environ.get("OMP_NUM_THREADS", "16") or 16))
    oracle.set_threads(threads)
    used = oracle.get_threads()
    kw = preset.problem()
    o = oracle.Oracle(**kw)
    walls = oracle.Walls(lid_u=preset.lid(0.0))
    h = np.zeros(o.shape)
    steps, t0 = 0, time.perf_counter()
    while True:
        h = o.step(h, walls, steps)
        steps += 1
        if time.perf_counter() - t0 >= seconds_budget or steps >= 3:
            break
    dt = time.perf_counter() - t0
    ncells, nv = o.nx * o.ny, o.nv
    return {"value": ncells * nv * steps / dt, "unit": "node-updates/s", "cores": used, "kind": "oracle",
            "sample": "%d full step(s) of the same %dx%d-cell, %d-node, %d-pair workload from rest, "
                      "FP64, OpenMP over cells, %.1f s" % (steps, o.nx, o.ny, nv, kw["n_pairs"], dt),
            "pairs_per_s": ncells * kw["n_pairs"] * steps / dt}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=40)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--config", default="cavity64")
    ap.add_argument("--sample-group", type=int, default=None, help="cells sharing a pair stream (0 = all)")
    ap.add_argument("--order", type=int, default=None)
    ap.add_argument("--cpu-baseline", choices=["auto", "skip"], default="auto")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on exactly one GPU: this build has no multi-GPU path "
              "(requested --gpus %d, WORLD_SIZE %d)" % (args.gpus, world), file=sys.stderr, flush=True)
        sys.exit(2)

    import torch

    import paper_1005_5405_amd as pkg

    preset = pkg.PRESETS[args.config]
    over = {}
    if args.sample_group is not None:
        over["sample_group"] = args.sample_group
    if args.order is not None:
        over["order"] = args.order
    preset = preset.with_(**over) if over else preset
    kw = preset.problem()
    g = pkg.Boltz(**kw)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    a, b = g.empty(0.0), g.empty()
    walls = pkg.Walls(lid_u=preset.lid(0.0))
    n = 0
    print("[bench] %s: %d cells x %d nodes, %d pairs/cell, G=%d, order %d; warm-up %d steps" %
          (args.config, g.ncells, g.nv, g.n_pairs, kw["sample_group"], g.order, args.warmup), flush=True)
    for _ in range(args.warmup):
        walls.lid_u = preset.lid(n * g.dt)
        g.stream(a, b, walls)
        g.collide(b, b, n)
        a, b = b, a
        n += 1
    torch.cuda.synchronize()
    K = args.steps
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(K)]
    t0 = time.perf_counter()
    for k in range(K):
        walls.lid_u = preset.lid(n * g.dt)
        ev[k][0].record(stream)
        g.stream(a, b, walls)
        ev[k][1].record(stream)
        g.collide(b, b, n)
        ev[k][2].record(stream)
        a, b = b, a
        n += 1
    torch.cuda.synchronize()
    wall_s = time.perf_counter() - t0
    t_stream = sum(e[0].elapsed_time(e[1]) for e in ev) / K * 1e-3
    t_collide = sum(e[1].elapsed_time(e[2]) for e in ev) / K * 1e-3
    t_events = ev[0][0].elapsed_time(ev[-1][2]) * 1e-3
    status = g.read_status()
    if status:
        print("[bench] device status %d (numerical failure)" % status, file=sys.stderr, flush=True)
        sys.exit(3)
    ms_per_step = wall_s / K * 1e3
    nodes = g.ncells * g.nv
    value = nodes * K / wall_s
    pairs_per_s = g.ncells * g.n_pairs * K / wall_s
    hbm_step = 2 * BYTES_PER_NODE_KERNEL * nodes / (wall_s / K) / 1e9
    # dominant kernel: the collision (sampling + gain/loss + correction)
    ops = g.ncells * (g.n_pairs * OPS_PER_PAIR + g.nv * OPS_PER_NODE)
    coll_bytes = BYTES_PER_NODE_KERNEL * nodes
    roof = {"kernel": "collide_kernel", "bound": "alu", "achieved": ops / t_collide / 1e12,
            "peak": ALU_PEAK_TOPS, "unit": "TFLOP/s", "frac": ops / t_collide / 1e12 / ALU_PEAK_TOPS,
            "traffic": None, "avg_ms": t_collide * 1e3,
            "hbm_algorithmic_GBs": coll_bytes / t_collide / 1e9,
            "note": "lane operations per launch (OPS_PER_PAIR x pairs + OPS_PER_NODE x nodes) over the "
                    "HIP-event average of the launch; peak = one vector op per lane per clock"}
    stream_k = {"kernel": "wall_kernel + stream_kernel", "bound": "hbm", "avg_ms": t_stream * 1e3,
                "achieved": BYTES_PER_NODE_KERNEL * nodes / t_stream / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": BYTES_PER_NODE_KERNEL * nodes / t_stream / 1e9 / HBM_PEAK_GBS}
    line = {"metric": "phase-space node-updates/s (stream+collide), collision pairs/s, % HBM peak",
            "value": value, "unit": "node-updates/s", "n_gpus": 1, "steps": K, "warmup": args.warmup,
            "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": "f32", "data": "synthetic",
            "config": {"workload": preset.name, "cells": [g.nx, g.ny], "velocity_grid": list(g.nv3),
                       "pairs_per_cell": g.n_pairs, "sample_group": kw["sample_group"], "order": g.order,
                       "kn": preset.kn, "lid_u": preset.lid_u, "cfl": preset.cfl, "parallelism": "single GPU"},
            "pairs_per_s": pairs_per_s, "hbm_frac_step": hbm_step / HBM_PEAK_GBS,
            "event_ms_per_step": t_events / K * 1e3,
            "roofline": roof, "kernels": {"stream": stream_k}}
    if args.cpu_baseline == "auto":
        print("[bench] CPU oracle baseline ...", flush=True)
        line["cpu_baseline"] = cpu_baseline(preset, args.cpu_seconds)
    _json_line(line)


if __name__ == "__main__":
    main()
