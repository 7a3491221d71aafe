#!/usr/bin/env python3
"""Throughput of the whole LCS hot path on one MI355X.

One step = build every breakout matrix of the strip recursion (next-match
tables, base strips, combine levels), read the length and trace one witness,
for one synthetic pair that is already resident in HBM.  The default workload
is the 4096 x 4096 pair over an alphabet of 4 with 64-row base strips.

Prints ONE JSON line: cells/s (m*n per second of wall time over the timed
steps), the roofline position of the dominant kernel (algorithmic bytes per
launch over its HIP-event duration, against the 8 TB/s HBM peak), and the CPU
oracle timed on this host as a reported baseline.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
WORKLOADS = {
    "pair-256x256-s4": "config_small",
    "pair-4096x4096-s4": "config_4096",
    "pair-16384x16384-s20-mut20": "config_16384",
}
DEFAULT_WORKLOAD = "pair-4096x4096-s4"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in ("lcs_device.h", "lcs_kernels.hip", "lcs_geom.h"):
        with open(os.path.join(ROOT, "paper_2309_09072_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def read_traffic(workload: str, kernel: str):
    """HBM bytes per launch from the committed counter summary, if it was taken
    on the current kernel sources (else None)."""
    path = os.path.join(ROOT, "profiles", "traffic_%s_%s.md" % (kernel, workload))
    if not os.path.exists(path):
        return None
    txt = open(path).read()
    src = re.search(r"kernel_source_sha256_16:\s*([0-9a-f]+)", txt)
    val = re.search(r"hbm_bytes_per_launch:\s*([0-9.eE+]+)", txt)
    if not src or not val or src.group(1) != kernel_source_hash():
        return None
    return float(val.group(1))


def cpu_baseline(pair, seconds: float):
    """The oracle (textbook DP + canonical traceback, single thread) on this host."""
    import oracle
    t0 = time.perf_counter()
    reps = 0
    while True:
        oracle.lcs_witness(pair.a, pair.b)
        reps += 1
        el = time.perf_counter() - t0
        if el >= seconds:
            break
    cells = reps * pair.a.size * pair.b.size
    return {"value": cells / el, "unit": "cells/s", "cores": 1, "kind": "oracle",
            "sample": "%d x the full %dx%d pair (length + witness), %.1f s" % (
                reps, pair.a.size, pair.b.size, el)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default=DEFAULT_WORKLOAD, choices=sorted(WORKLOADS))
    ap.add_argument("--base-rows", type=int, default=64)
    ap.add_argument("--tile", type=int, default=32)
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="also launch one plain device copy of this many MiB (counter calibration)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: this engine has no multi-GPU path "
              "(each pair runs on one device); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2309_09072_amd.synth as synth
    from paper_2309_09072_amd import lcs

    pair = getattr(synth, WORKLOADS[args.workload])()
    m, n = int(pair.a.size), int(pair.b.size)
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream()
    ad, bd = lcs.device_bytes(pair.a), lcs.device_bytes(pair.b)
    plan = lcs.Plan(m, n, pair.sigma, args.base_rows, args.tile)
    pplan = lcs.Plan(m, n, pair.sigma, args.base_rows, args.tile, profile=True)
    ws = lcs.alloc_workspace(plan.workspace_for(m, n))
    cap = max(1, min(m, n))
    ai = torch.empty(cap, dtype=torch.int32, device=dev)
    bi = torch.empty(cap, dtype=torch.int32, device=dev)
    ld = torch.zeros(1, dtype=torch.int32, device=dev)

    def step(p):
        p.build(ad, bd, ws)
        p.trace_device(ai, bi, ld)

    log("workload %s: m=%d n=%d alphabet=%d, workspace %.2f GB" % (
        args.workload, m, n, pair.sigma, ws.numel() / 1e9))
    for _ in range(args.warmup):
        step(plan)
    torch.cuda.synchronize()

    # ---- timed region: K steps, events on the stream the kernels run on
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(stream)
    for _ in range(args.steps):
        step(plan)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = e0.elapsed_time(e1)
    ms_per_step = 1000.0 * wall / args.steps
    log("timed %d steps: %.3f ms/step wall, %.3f ms/step events" % (
        args.steps, ms_per_step, gpu_ms / args.steps))

    # ---- exactness of the timed result
    import oracle
    Lo, ao, bo = oracle.lcs_witness(pair.a, pair.b)
    Lg = int(ld.item())
    exact = (Lg == Lo and np.array_equal(ai[:Lg].cpu().numpy(), ao)
             and np.array_equal(bi[:Lg].cpu().numpy(), bo))
    log("length %d (oracle %d), exact=%s" % (Lg, Lo, exact))

    # ---- per-kernel durations: the same K steps again with HIP events around every launch
    step(pplan)
    pplan.profile()  # drop the warm-up records
    for _ in range(args.steps):
        step(pplan)
    recs = pplan.profile()
    by = {}
    for kind, level, ms, nbytes in recs:
        d = by.setdefault(kind, {"ms": 0.0, "bytes": 0, "launches": 0})
        d["ms"] += ms
        d["bytes"] += nbytes
        d["launches"] += 1
    breakdown = {}
    for kind, d in by.items():
        breakdown[kind] = {
            "ms_per_step": round(d["ms"] / args.steps, 4),
            "launches_per_step": d["launches"] // args.steps,
            "alg_GBps": round(d["bytes"] / (d["ms"] * 1e-3) / 1e9, 1) if d["ms"] > 0 else None,
        }
    dom = max(("base", "anchor", "bracket"), key=lambda k: by.get(k, {"ms": 0})["ms"])
    d = by[dom]
    per_launch_bytes = d["bytes"] / d["launches"]
    per_launch_s = d["ms"] * 1e-3 / d["launches"]
    achieved = per_launch_bytes / per_launch_s / 1e9
    kernel_name = {"base": "k_base", "anchor": "k_anchor", "bracket": "k_bracket"}[dom]
    traffic = read_traffic(args.workload, kernel_name)
    total_alg = sum(v["bytes"] for k, v in by.items() if k in ("nextmatch", "base", "anchor", "bracket", "length")) / args.steps
    log("breakdown: " + json.dumps(breakdown))

    if args.calib_copy_mib > 0:
        nb = args.calib_copy_mib << 20
        x = torch.ones(nb // 4, dtype=torch.int32, device=dev)
        y = torch.empty_like(x)
        torch.cuda.synchronize()
        y.copy_(x)
        torch.cuda.synchronize()
        log("calibration copy: %d bytes read, %d bytes written" % (nb, nb))

    cells = m * n
    out = {
        "metric": "LCS cells/s (m*n/s) + HBM GB/s; exact match",
        "value": cells / (ms_per_step * 1e-3) if exact else None,
        "unit": "cells/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": args.workload, "m": m, "n": n, "alphabet": pair.sigma,
                   "seed": pair.seed, "base_rows": args.base_rows, "tile": args.tile,
                   "parallelism": "single-gpu"},
        "exact_match": bool(exact),
        "lcs_length": Lg,
        "alg_GBps_whole_build": round(total_alg / (ms_per_step * 1e-3) / 1e9, 1),
        "roofline": {
            "kernel": kernel_name,
            "bound": "hbm",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic,
            "alg_bytes_per_launch": int(per_launch_bytes),
            "avg_launch_ms": round(per_launch_s * 1e3, 4),
        },
        "breakdown": breakdown,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(pair, args.cpu_seconds)
    print(json.dumps(out), flush=True)
    if not exact:
        sys.exit(1)


if __name__ == "__main__":
    main()
