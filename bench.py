#!/usr/bin/env python3
"""Throughput of the whole LCS hot path on one MI355X.

One step = build every breakout matrix of the strip recursion (next-match
tables, base strips, combine levels), read the length and trace one witness,
for one synthetic pair that is already resident in HBM.  The headline workload
is the largest single pair: 16384 x 16384 over an alphabet of 20, the second
string a mutated copy of the first, with 64-row base strips.

Prints ONE JSON line: cells/s (m*n per second of wall time over the timed
steps), the roofline position of the dominant kernel (algorithmic bytes per
launch over its HIP-event duration, against the 8 TB/s HBM peak), and the CPU
oracle timed on this host as a reported baseline (one core on the headline
pair; all cores on the batch).  Sub-blocks, each exact-checked: the 4096 x 4096
pair, the 4096-pair batch in every batch mode against one pair per launch,
the serving loop under Poisson arrivals, and the paper's own shapes.
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
DEFAULT_WORKLOAD = "pair-16384x16384-s20-mut20"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash(batch_sources: bool = False) -> str:
    """Hash of the device sources a counter summary was taken on (the batch kernels
    add their own file)."""
    h = hashlib.sha256()
    files = ["lcs_device.h", "lcs_kernels.hip", "lcs_geom.h"]
    if batch_sources:
        files += ["lcs_batch.hip", "lcs_sched.h"]
    for f in files:
        with open(os.path.join(ROOT, "paper_2309_09072_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


VALU_PEAK_LANE_OPS = 256 * 4 * 16 * 2.4e9  # CUs x SIMDs x lanes x clock: 39.3 T lane-ops/s


def read_valu(workload: str, kernel: str):
    """VALU wave-instructions per launch from the committed counter summary, if it
    was taken on the current kernel sources (else None)."""
    path = os.path.join(ROOT, "profiles", "valu_%s_%s.md" % (kernel, workload))
    if not os.path.exists(path):
        return None
    txt = open(path).read()
    src = re.search(r"kernel_source_sha256_16:\s*([0-9a-f]+)", txt)
    val = re.search(r"valu_insts_per_launch:\s*([0-9.eE+]+)", txt)
    if not src or not val or src.group(1) != kernel_source_hash():
        return None
    return float(val.group(1))


def read_traffic(workload: str, kernel: str, batch_sources: bool = False):
    """HBM bytes per launch (per batch for the batch summaries) from the committed
    counter summary, if it was taken on the current kernel sources (else None)."""
    path = os.path.join(ROOT, "profiles", "traffic_%s_%s.md" % (kernel, workload))
    if not os.path.exists(path):
        return None
    txt = open(path).read()
    src = re.search(r"kernel_source_sha256_16:\s*([0-9a-f]+)", txt)
    val = re.search(r"hbm_bytes_per_launch:\s*([0-9.eE+]+)", txt)
    if not src or not val or src.group(1) != kernel_source_hash(batch_sources):
        return None
    return float(val.group(1))


def host_info() -> dict:
    """Core count and CPU model of this host (the CPU baseline's machine)."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return {"nproc": os.cpu_count(), "usable_cores": usable, "cpu_model": model}


def cpu_threads() -> int:
    """Threads of the all-core baseline: the cores this process may use, at most
    16 (the host share of one GPU)."""
    return max(1, min(16, host_info()["usable_cores"] or 1))


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


def cpu_baseline_all_cores(batch, threads: int):
    """The oracle on every pair of a batch, one pair per task over `threads` host
    threads (the C oracle runs outside the interpreter lock)."""
    import concurrent.futures as cf
    import oracle
    oracle.lcs_witness(*batch.pair(0))  # load the library before timing
    t0 = time.perf_counter()
    with cf.ThreadPoolExecutor(threads) as ex:
        for _ in ex.map(lambda p: oracle.lcs_witness(*batch.pair(p)), range(batch.count), chunksize=8):
            pass
    el = time.perf_counter() - t0
    return {"value": batch.cells / el, "unit": "cells/s", "cores": threads, "kind": "oracle",
            "sample": "all %d pairs of %s (length + witness), one pair per task, %.1f s" % (
                batch.count, batch.name, el)}


def _oracle_check(args):
    import numpy as np
    import oracle
    a, b, L, ai, bi = args
    Lo, ao, bo = oracle.lcs_witness(a, b)
    return L == Lo and np.array_equal(ai, ao) and np.array_equal(bi, bo)


def oracle_check_many(items, procs=8):
    """Every (a, b, L, a_idx, b_idx) against the oracle, on `procs` host processes."""
    import multiprocessing as mp
    with mp.get_context("fork").Pool(procs) as pool:
        return all(pool.imap_unordered(_oracle_check, items, chunksize=16))


def alg_bytes(m: int, n: int, h0: int) -> int:
    """Algorithmic bytes of one build of an m x n pair with base strips of h0 rows:
    every base-strip matrix written once, and for every combine the rows of D_U
    and D_L read once and the rows of D_G written once (4-byte cells, n + 2 rows
    per matrix with the sentinel row), plus the row string read once."""
    if m <= 0 or n <= 0:
        return 0
    S = (m + h0 - 1) // h0
    hs = [h0] * (S - 1) + [m - (S - 1) * h0]
    tot = 4 * (n + 2) * (m + S) + m
    while len(hs) > 1:
        nxt = []
        for p in range(len(hs) // 2):
            hU, hL = hs[2 * p], hs[2 * p + 1]
            tot += 4 * (n + 2) * ((hU + 1) + (hL + 1) + (hU + hL + 1))
            nxt.append(hU + hL)
        if len(hs) % 2:
            nxt.append(hs[-1])
        hs = nxt
    return tot


BATCH_MODES = ("staged_graph", "pair_queue_graph", "persistent_graph", "one_pair_per_launch")


def bench_batched(reps: int, tune_shapes: bool = True, modes=BATCH_MODES, base_rows: int = 0):
    """Many pairs of uneven length: one launch per step across the pairs (staged),
    one persistent launch (pair queue, task queue), and one pair per launch."""
    import numpy as np
    import torch
    import paper_2309_09072_amd.synth as synth
    from paper_2309_09072_amd import lcs
    batch = synth.batch_mixed()
    maxlen = int(max(batch.m.max(), batch.n.max()))
    slots = 512
    tuning = None
    h0, tile = (base_rows or 64), 32
    if tune_shapes:  # the autotuner picks the shapes on a sample of the batch (staged mode)
        from paper_2309_09072_amd import tune
        tr = tune.tune_batch(batch, lcs.BATCH_STAGED | lcs.BATCH_GRAPH, base_rows=base_rows or None,
                             slots=slots, use_cache=False)
        h0, tile = tr.best
        tuning = tr.as_json()
        log("batch autotuner: base_rows %d tile %d (%s)" % (h0, tile, tuning["ms"]))
    plan = lcs.Batch(batch.count, maxlen, batch.sigma, h0, tile, slots=slots)
    # the persistent and pair-queue modes append rows: base strips of at most 64
    # rows; one pair per launch runs at 64 rows too (its best for pairs this short)
    h0_rows = min(h0, 64)
    plan_rows = plan if h0 <= 64 else lcs.Batch(batch.count, maxlen, batch.sigma, h0_rows, tile,
                                                  slots=slots)
    ws = lcs.alloc_workspace(max(plan.workspace_bytes, plan_rows.workspace_bytes))
    sym = lcs.device_bytes(batch.symbols)
    off = lcs.Batch.witness_offsets(batch.m, batch.n)
    lengths = torch.zeros(batch.count, dtype=torch.int32, device="cuda")
    ai = torch.zeros(int(off[-1]), dtype=torch.int32, device="cuda")
    bi = torch.zeros(int(off[-1]), dtype=torch.int32, device="cuda")
    nbytes = sum(alg_bytes(int(batch.m[p]), int(batch.n[p]), h0) for p in range(batch.count))
    nbytes_rows = nbytes if h0 <= 64 else sum(alg_bytes(int(batch.m[p]), int(batch.n[p]), h0_rows)
                                              for p in range(batch.count))
    out = {"workload": batch.name, "pairs": batch.count, "cells": batch.cells, "seed": batch.seed,
           "slots": slots, "base_rows": h0, "base_rows_other_modes": h0_rows, "tile": tile,
           "autotune": tuning,
           "workspace_GB": round(ws.numel() / 1e9, 2), "alg_bytes_per_batch": nbytes}
    mode_of = {"staged_graph": lcs.BATCH_STAGED | lcs.BATCH_GRAPH,
               "staged": lcs.BATCH_STAGED,
               "pair_queue_graph": lcs.BATCH_PAIR_QUEUE | lcs.BATCH_GRAPH,
               "persistent_graph": lcs.BATCH_PERSISTENT | lcs.BATCH_GRAPH,
               "one_pair_per_launch": lcs.BATCH_PER_PAIR}
    for name in modes:
        mode = mode_of[name]
        staged = bool(mode & lcs.BATCH_STAGED)
        pl, nb = (plan, nbytes) if staged else (plan_rows, nbytes_rows)
        pl.submit(sym, batch.a_off, batch.b_off, batch.m, batch.n, ws, lengths, ai, bi, mode)
        torch.cuda.synchronize()
        # poison the outputs, so that a mode which wrote nothing cannot pass on the
        # previous mode's results
        lengths.fill_(-99)
        ai.fill_(-1)
        bi.fill_(-1)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            pl.submit(sym, batch.a_off, batch.b_off, batch.m, batch.n, ws, lengths, ai, bi, mode)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / reps
        if not (mode & (lcs.BATCH_PER_PAIR | lcs.BATCH_STAGED | lcs.BATCH_PAIR_QUEUE)):
            pl.status(ws)
        L = lengths.cpu().numpy()
        A, B = ai.cpu().numpy(), bi.cpu().numpy()
        items = [(batch.pair(p)[0], batch.pair(p)[1], int(L[p]), A[off[p]:off[p] + max(L[p], 0)],
                  B[off[p]:off[p] + max(L[p], 0)]) for p in range(batch.count)]
        exact = oracle_check_many(items)
        out[name] = {"s_per_batch": round(dt, 4), "cells_per_s": batch.cells / dt,
                     "alg_GBps": round(nb / dt / 1e9, 1), "exact_match": exact,
                     "base_rows": pl.desc.base_rows}
        log("batched %s: %.3f s per batch, %.3g cells/s, exact=%s" % (name, dt, batch.cells / dt, exact))
    one_launch = [k for k in out if k in ("staged_graph", "staged", "pair_queue_graph", "persistent_graph")]
    if one_launch:
        best = min(one_launch, key=lambda k: out[k]["s_per_batch"])
        nbest = nbytes if best.startswith("staged") else nbytes_rows
        ach = nbest / out[best]["s_per_batch"] / 1e9
        out["roofline"] = {"kernel": "whole batch, %s (all step kernels)" % best, "bound": "hbm",
                           "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                           "frac": round(ach / HBM_PEAK_GBS, 4),
                           "traffic": read_traffic(batch.name, "staged", batch_sources=True),
                           "alg_bytes_per_batch": nbest}
        if "one_pair_per_launch" in out:
            for k in one_launch:
                out["speedup_%s_vs_per_pair" % k.replace("_graph", "")] = round(
                    out["one_pair_per_launch"]["s_per_batch"] / out[k]["s_per_batch"], 2)
    if plan_rows is not plan:
        plan_rows.close()
    plan.close()
    del ws
    torch.cuda.empty_cache()
    return out, batch


def bench_serving(count: int, budget_gb: float, slots: int):
    """Poisson arrivals (lengths log-uniform 128..8192, alphabet 4 or 20, 30% related
    pairs at a 10% edit rate), admission by arena memory; p50/p99 latency + cells/s."""
    import numpy as np
    import torch
    import paper_2309_09072_amd.synth as synth
    from paper_2309_09072_amd import lcs
    arena = lcs.alloc_workspace(int(budget_gb * (1 << 30)))

    def run(rate):
        reqs = synth.serving_requests(count, rate=rate)
        srv = lcs.Server(arena, 8192, 20, slots=slots, max_queue=count + 1)
        bufs = {}
        for r in reqs:
            cap = max(1, min(r.a.size, r.b.size))
            bufs[r.rid] = (torch.empty(cap, dtype=torch.int32, device="cuda"),
                           torch.empty(cap, dtype=torch.int32, device="cuda"))
        torch.cuda.synchronize()
        res = {}
        t0 = time.perf_counter()
        i = 0
        max_running = 0
        while len(res) < len(reqs):
            now = time.perf_counter() - t0
            while i < len(reqs) and (rate <= 0 or reqs[i].arrival <= now):
                r = reqs[i]
                st = srv.submit(r.rid, r.a, r.b, r.sigma, *bufs[r.rid])
                assert st == 0, st
                i += 1
            for tag, status, length, ts, tadm, tdone in srv.poll():
                res[tag] = (status, length, ts, tadm, tdone)
            max_running = max(max_running, srv.pending()[0])
            time.sleep(0.0002)
        wall = time.perf_counter() - t0
        peak = srv.pending()[3]
        srv.close()
        lat = np.array([res[r.rid][4] - res[r.rid][2] for r in reqs])
        cells = sum(int(r.a.size) * int(r.b.size) for r in reqs)
        return reqs, res, bufs, wall, lat, cells, peak, max_running

    reqs, res, bufs, wall, lat, cells, peak, _ = run(0.0)   # closed loop: saturation rate
    r_sat = count / wall
    out = {"workload": "serving-poisson-128..8192", "requests": count, "slots": slots,
           "budget_GB": budget_gb, "saturation_req_per_s": round(r_sat, 1),
           "saturation_cells_per_s": cells / wall}
    for frac in (0.5, 0.7, 0.9):
        reqs, res, bufs, wall, lat, cells, peak, max_running = run(frac * r_sat)
        items = []
        for r in reqs:
            st, L = res[r.rid][0], res[r.rid][1]
            ai, bi = bufs[r.rid]
            items.append((r.a, r.b, L if st == 0 else -1, ai[:L].cpu().numpy(), bi[:L].cpu().numpy()))
        exact = oracle_check_many(items)
        out["at_%d_pct" % int(frac * 100)] = {
            "rate_req_per_s": round(frac * r_sat, 1), "p50_ms": round(1e3 * float(np.percentile(lat, 50)), 3),
            "p99_ms": round(1e3 * float(np.percentile(lat, 99)), 3), "cells_per_s": cells / wall,
            "peak_arena_GB": round(peak / 1e9, 3), "max_running": max_running, "exact_match": exact}
        log("serving at %.0f%% of saturation: p50 %.2f ms p99 %.2f ms, exact=%s" % (
            frac * 100, 1e3 * np.percentile(lat, 50), 1e3 * np.percentile(lat, 99), exact))
    del arena
    torch.cuda.empty_cache()
    return out


# Table I of the paper: seconds per LCS of its Chapel implementation on Xeon
# Gold 6330 cores, for string lengths (s1, s2); {s1: (32-core row, 8-core row)}.
PAPER_TABLE_I = {
    1024: ((0.119569, 0.62156, 1.63747, 3.2784), (0.370135, 1.5887, 2.30283, 4.75351)),
    2048: ((0.890801, 2.4456, 4.51969, 12.2226), (1.37578, 6.31841, 8.03229, 19.2526)),
    4096: ((6.64456, 11.1501, 16.5999, 51.9423), (5.35454, 21.2137, 33.1638, 72.9992)),
    8192: ((29.5529, 53.5266, 67.5972, 190.575), (28.722, 88.2542, 145.517, 417.969)),
}
PAPER_S2 = (2, 4, 8, 16)


def paper_sweep(steps: int, warmup: int):
    """The paper's Table I shapes on one GPU (both orientations: the long string
    on the rows, then on the columns), exact-checked, beside the paper's seconds."""
    import numpy as np
    import torch
    import oracle
    import paper_2309_09072_amd.synth as synth
    from paper_2309_09072_amd import lcs
    g = np.random.default_rng(synth.SEED_BASE + 90)
    rows = []
    for s1, (t32, t8) in sorted(PAPER_TABLE_I.items()):
        for c, s2 in enumerate(PAPER_S2):
            x, y = synth.uniform(g, s1, 4), synth.uniform(g, s2, 4)
            want = oracle.lcs_witness(x, y)
            entry = {"s1": s1, "s2": s2, "paper_s_32_cores": t32[c], "paper_s_8_cores": t8[c]}
            for name, (a, b), orient in (("long_rows", (x, y), False), ("long_cols", (y, x), False),
                                         ("long_rows_oriented", (x, y), True)):
                m, n = a.size, b.size
                ad, bd = lcs.device_bytes(a), lcs.device_bytes(b)
                plan = lcs.Plan(m, n, 4, 64, 32, orient=orient)
                ws = lcs.alloc_workspace(plan.workspace_for(m, n))
                cap = max(1, min(m, n))
                ai = torch.empty(cap, dtype=torch.int32, device="cuda")
                bi = torch.empty(cap, dtype=torch.int32, device="cuda")
                ld = torch.zeros(1, dtype=torch.int32, device="cuda")

                def step():
                    plan.build(ad, bd, ws)
                    plan.trace_device(ai, bi, ld)

                for _ in range(warmup):
                    step()
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                torch.cuda.synchronize()
                e0.record()
                for _ in range(steps):
                    step()
                e1.record()
                torch.cuda.synchronize()
                us = e0.elapsed_time(e1) * 1e3 / steps
                L = int(ld.item())
                ref = oracle.lcs_witness(a, b)
                exact = (L == ref[0] and np.array_equal(ai[:L].cpu().numpy(), ref[1])
                         and np.array_equal(bi[:L].cpu().numpy(), ref[2]))
                assert L == want[0]
                entry[name] = {"us_per_lcs": round(us, 2), "exact_match": bool(exact),
                               "speedup_vs_paper_32_cores": round(t32[c] / (us * 1e-6), 1)}
                plan.close()
            rows.append(entry)
            log("paper shape %dx%d: %s us (long rows), %s us (long cols), %s us (long rows, oriented);"
                " paper 32 cores %.3g s" % (s1, s2, entry["long_rows"]["us_per_lcs"],
                                             entry["long_cols"]["us_per_lcs"],
                                             entry["long_rows_oriented"]["us_per_lcs"], t32[c]))
    return rows


# Figs. 3 and 4 of the paper: one string held at 2 or 4 symbols, the other
# grown from 2 to 8192 (powers of two); the paper prints only fitted curves.
PAPER_FIG_FIXED = (2, 4)
PAPER_FIG_SIZES = tuple(2 ** e for e in range(1, 14))


def paper_shapes(steps: int):
    """Compact block of the paper's shapes (Table I and Figs. 3/4): one uniform
    pair over 4 symbols per shape, the long string on the rows, built with the
    orientation choice (the recursion runs over the shorter string); build +
    witness per LCS, event-timed over `steps`, exact against the oracle."""
    import numpy as np
    import torch
    import oracle
    import paper_2309_09072_amd.synth as synth
    from paper_2309_09072_amd import lcs
    g = np.random.default_rng(synth.SEED_BASE + 91)
    shapes = []
    for s1, (t32, t8) in sorted(PAPER_TABLE_I.items()):
        for c, s2 in enumerate(PAPER_S2):
            shapes.append((s1, s2, "table1", t32[c], t8[c]))
    for fixed in PAPER_FIG_FIXED:
        for s1 in PAPER_FIG_SIZES:
            shapes.append((s1, fixed, "fig3_4", None, None))
    rows = []
    all_exact = True
    for s1, s2, src, t32, t8 in shapes:
        a, b = synth.uniform(g, s1, 4), synth.uniform(g, s2, 4)
        m, n = a.size, b.size
        ad, bd = lcs.device_bytes(a), lcs.device_bytes(b)
        plan = lcs.Plan(m, n, 4, 64, 32, orient=True)
        ws = lcs.alloc_workspace(plan.workspace_for(m, n))
        cap = max(1, min(m, n))
        ai = torch.empty(cap, dtype=torch.int32, device="cuda")
        bi = torch.empty(cap, dtype=torch.int32, device="cuda")
        ld = torch.zeros(1, dtype=torch.int32, device="cuda")
        for _ in range(3):  # warm-up: the first shape also pays first-use costs
            plan.build(ad, bd, ws)
            plan.trace_device(ai, bi, ld)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(steps):
            plan.build(ad, bd, ws)
            plan.trace_device(ai, bi, ld)
        e1.record()
        torch.cuda.synchronize()
        us = e0.elapsed_time(e1) * 1e3 / steps
        L = int(ld.item())
        ref = oracle.lcs_witness(a, b)
        exact = bool(L == ref[0] and np.array_equal(ai[:L].cpu().numpy(), ref[1])
                     and np.array_equal(bi[:L].cpu().numpy(), ref[2]))
        all_exact &= exact
        row = {"s1": s1, "s2": s2, "from": src, "us_per_lcs": round(us, 2), "exact_match": exact}
        if t32 is not None:
            row["paper_s_32_cores"] = t32
            row["paper_s_8_cores"] = t8
        rows.append(row)
        plan.close()
    log("paper shapes: %d shapes, %.1f..%.1f us per LCS, exact=%s" % (
        len(rows), min(r["us_per_lcs"] for r in rows), max(r["us_per_lcs"] for r in rows), all_exact))
    return {"note": "paper seconds: Chapel on Xeon Gold 6330 (Table I), context only",
            "exact_match": all_exact, "rows": rows}


def bench_pair(workload: str, steps: int, warmup: int, base_rows: int, tile: int):
    """One pair resident in HBM: K timed steps (build + witness), the oracle check
    of the timed result, then the same steps with events around every launch for
    the per-kernel breakdown and the dominant kernel's roofline position."""
    import numpy as np
    import torch
    import paper_2309_09072_amd.synth as synth
    from paper_2309_09072_amd import lcs
    pair = getattr(synth, WORKLOADS[workload])()
    m, n = int(pair.a.size), int(pair.b.size)
    dev = torch.device("cuda", 0)
    stream = torch.cuda.current_stream()
    ad, bd = lcs.device_bytes(pair.a), lcs.device_bytes(pair.b)
    tuning = None
    if base_rows == 0:  # the library's choice for this size
        probe = lcs.Plan(m, n, pair.sigma, 0, max(tile, 4))
        base_rows = probe.base_rows
        probe.close()
    if tile == 0:  # the autotuner picks the tile for this base-strip height
        from paper_2309_09072_amd import tune
        tr = tune.tune_pair(ad, bd, pair.sigma, base_rows=base_rows, use_cache=False)
        tile = tr.best[1]
        tuning = tr.as_json()
        log("%s autotuner: tile %d (%s)" % (workload, tile, tuning["ms"]))
    plan = lcs.Plan(m, n, pair.sigma, base_rows, tile)
    pplan = lcs.Plan(m, n, pair.sigma, base_rows, tile, profile=True)
    ws = lcs.alloc_workspace(plan.workspace_for(m, n))
    cap = max(1, min(m, n))
    ai = torch.empty(cap, dtype=torch.int32, device=dev)
    bi = torch.empty(cap, dtype=torch.int32, device=dev)
    ld = torch.zeros(1, dtype=torch.int32, device=dev)

    def step(p):
        p.build(ad, bd, ws)
        p.trace_device(ai, bi, ld)

    log("workload %s: m=%d n=%d alphabet=%d, workspace %.2f GB" % (
        workload, m, n, pair.sigma, ws.numel() / 1e9))
    for _ in range(warmup):
        step(plan)
    ai.fill_(-1)
    bi.fill_(-1)
    ld.fill_(-1)
    torch.cuda.synchronize()

    # ---- timed region: K steps, events on the stream the kernels run on
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(stream)
    for _ in range(steps):
        step(plan)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = e0.elapsed_time(e1)
    ms_per_step = 1000.0 * wall / steps
    log("timed %d steps: %.3f ms/step wall, %.3f ms/step events" % (steps, ms_per_step, gpu_ms / steps))

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
    for _ in range(steps):
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
            "ms_per_step": round(d["ms"] / steps, 4),
            "launches_per_step": d["launches"] // steps,
            "alg_GBps": round(d["bytes"] / (d["ms"] * 1e-3) / 1e9, 1) if d["ms"] > 0 else None,
        }
    dom = max(("base", "anchor", "bracket"), key=lambda k: by.get(k, {"ms": 0})["ms"])
    d = by[dom]
    per_launch_bytes = d["bytes"] / d["launches"]
    per_launch_s = d["ms"] * 1e-3 / d["launches"]
    achieved = per_launch_bytes / per_launch_s / 1e9
    kernel_name = {"base": "k_base", "anchor": "k_anchor", "bracket": "k_bracket"}[dom]
    traffic = read_traffic(workload, kernel_name)
    valu_insts = read_valu(workload, kernel_name)
    valu = None
    if valu_insts is not None:  # wave instructions x 64 lanes per launch / launch time
        lane_ops = valu_insts * 64 / per_launch_s
        valu = {"lane_ops_per_s": lane_ops, "peak": VALU_PEAK_LANE_OPS,
                "frac": round(lane_ops / VALU_PEAK_LANE_OPS, 4), "insts_per_launch": valu_insts}
    total_alg = alg_bytes(m, n, base_rows)
    log("breakdown: " + json.dumps(breakdown))
    res = {
        "value": m * n / (ms_per_step * 1e-3) if exact else None,
        "ms_per_step": round(ms_per_step, 4),
        "config": {"workload": workload, "m": m, "n": n, "alphabet": pair.sigma, "seed": pair.seed,
                   "base_rows": base_rows, "tile": tile},
        "autotune": tuning,
        "exact_match": bool(exact),
        "lcs_length": Lg,
        "alg_bytes_per_step": total_alg,
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
            "valu": valu,
        },
        "breakdown": breakdown,
    }
    plan.close()
    pplan.close()
    del ws
    torch.cuda.empty_cache()
    return res, pair


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default=DEFAULT_WORKLOAD, choices=sorted(WORKLOADS))
    ap.add_argument("--base-rows", type=int, default=0,
                    help="rows per base strip; 0: the library's choice for the size")
    ap.add_argument("--tile", type=int, default=0,
                    help="vertices between anchor searches; 0: chosen by the autotuner")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the 4096 x 4096 pair, the batched (4096 pairs), serving and "
                         "paper-shape workloads")
    ap.add_argument("--batch-base-rows", type=int, default=0,
                    help="rows per base strip of the batch; 0: the autotuner's choice "
                         "(64 with --only-batched)")
    ap.add_argument("--only-batched", action="store_true",
                    help="run the batched workload alone (its own JSON line; for profiling)")
    ap.add_argument("--batch-reps", type=int, default=3)
    ap.add_argument("--batch-modes", default=",".join(BATCH_MODES),
                    help="comma-separated batch modes (staged = the staged mode without a graph)")
    ap.add_argument("--serve-requests", type=int, default=2000)
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="also launch one plain device copy of this many MiB (counter calibration)")
    ap.add_argument("--paper-sweep", action="store_true",
                    help="instead: the paper's Table I shapes in both orientations (one JSON line)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: this engine has no multi-GPU path "
              "(each pair runs on one device); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch

    torch.cuda.set_device(0)
    if args.paper_sweep:
        rows = paper_sweep(max(args.steps, 5), max(args.warmup, 1))
        print(json.dumps({"metric": "microseconds per LCS, paper Table I shapes", "unit": "us",
                          "higher_is_better": False, "n_gpus": 1, "dtype": "int32",
                          "data": "synthetic", "rows": rows}))
        return

    def calib():
        if args.calib_copy_mib > 0:
            nb = args.calib_copy_mib << 20
            x = torch.ones(nb // 4, dtype=torch.int32, device="cuda")
            y = torch.empty_like(x)
            torch.cuda.synchronize()
            y.copy_(x)
            torch.cuda.synchronize()
            log("calibration copy: %d bytes read, %d bytes written" % (nb, nb))

    if args.only_batched:
        bres, _ = bench_batched(args.batch_reps, tune_shapes=False,
                                modes=tuple(args.batch_modes.split(",")), base_rows=args.batch_base_rows)
        calib()
        print(json.dumps({"metric": "batched LCS cells/s", "batched": bres}), flush=True)
        return

    head, pair = bench_pair(args.workload, args.steps, args.warmup, args.base_rows, args.tile)
    calib()
    out = {
        "metric": "LCS cells/s (m\u00b7n/s) + HBM GB/s; batched vs one-pair-per-launch, exact match",
        "value": head["value"],
        "unit": "cells/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": dict(head["config"], parallelism="single-gpu"),
    }
    for k in ("autotune", "exact_match", "lcs_length", "alg_bytes_per_step", "alg_GBps_whole_build",
              "roofline", "breakdown"):
        out[k] = head[k]
    batch = None
    if not args.no_extras:
        if args.workload != "pair-4096x4096-s4":
            sub, _ = bench_pair("pair-4096x4096-s4", args.steps, args.warmup, args.base_rows, 0)
            out["pair_4096"] = sub
        out["batched"], batch = bench_batched(args.batch_reps)
        out["serving"] = bench_serving(args.serve_requests, 64.0, 16)
        out["paper_shapes"] = paper_shapes(max(args.steps // 2, 5))
    if not args.no_cpu_baseline:
        cb = cpu_baseline(pair, args.cpu_seconds)
        cb["host"] = host_info()
        if batch is not None:
            cb["all_cores"] = cpu_baseline_all_cores(batch, cpu_threads())
        out["cpu_baseline"] = cb
        log("cpu baseline: %.3g cells/s on 1 core%s" % (
            cb["value"], "" if batch is None else ", %.3g cells/s on %d cores" % (
                cb["all_cores"]["value"], cb["all_cores"]["cores"])))
    print(json.dumps(out), flush=True)
    if not head["exact_match"]:
        sys.exit(1)


if __name__ == "__main__":
    main()
