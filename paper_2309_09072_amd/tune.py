"""Autotuner for the tile shapes of the strip recursion.

Two shape parameters change the speed but never the result (every choice is
exact): ``base_rows`` (rows per base strip: 16 to 1024 for single pairs and
staged batches, 16/32/64 for the persistent batch modes) and ``tile`` (vertices
between two anchor searches of a combine, a power of two 4..32).  The tuner
times each candidate on the GPU through the C ABI (one pair: the whole build
plus the witness trace; a batch: one submit of a sample of its pairs), keeps
the fastest, and caches the choice per device and size class in a JSON file,
so that later runs pick it up without timing again.

Cache file: ``$LCS_TUNE_CACHE`` or ``~/.cache/paper_2309_09072_amd/tune.json``.
"""
from __future__ import annotations

import json
import os
import time
from dataclasses import dataclass, field
from typing import Callable, Dict, List, Optional, Sequence, Tuple

BASE_ROWS = (16, 32, 64)                  # persistent batches (row-append base strips)
PAIR_BASE_ROWS = (16, 32, 64, 128, 256, 512, 1024)  # single pairs, staged batches (combed)
TILES = (8, 16, 32)
DEFAULT = (64, 32)

Config = Tuple[int, int]  # (base_rows, tile)


def candidates(base_rows: Optional[int] = None, tiles: Sequence[int] = TILES,
               rows: Sequence[int] = BASE_ROWS) -> List[Config]:
    """Candidate (base_rows, tile) pairs; base_rows fixed when given, else from `rows`."""
    hs = (int(base_rows),) if base_rows else tuple(rows)
    return [(h, int(t)) for h in hs for t in tiles]


def bucket(x: int) -> int:
    """Size class: the next power of two (at least 1)."""
    x = max(int(x), 1)
    return 1 << (x - 1).bit_length()


def cache_key(device: str, kind: str, m: int, n: int, sigma: int,
              base_rows: Optional[int] = None) -> str:
    return "%s|%s|m%d|n%d|s%d|h%s" % (device, kind, bucket(m), bucket(n), bucket(sigma),
                                      base_rows if base_rows else "any")


def default_cache_path() -> str:
    p = os.environ.get("LCS_TUNE_CACHE")
    if p:
        return p
    return os.path.join(os.path.expanduser("~"), ".cache", "paper_2309_09072_amd", "tune.json")


def load_cache(path: Optional[str] = None) -> Dict[str, dict]:
    path = path or default_cache_path()
    try:
        with open(path) as f:
            data = json.load(f)
        return data if isinstance(data, dict) else {}
    except (OSError, ValueError):
        return {}


def store_cache(key: str, entry: dict, path: Optional[str] = None) -> None:
    path = path or default_cache_path()
    data = load_cache(path)
    data[key] = entry
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    tmp = "%s.tmp%d" % (path, os.getpid())
    with open(tmp, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


@dataclass
class TuneResult:
    best: Config
    ms: Dict[Config, float] = field(default_factory=dict)
    cached: bool = False

    def as_json(self) -> dict:
        return {"base_rows": self.best[0], "tile": self.best[1], "cached": self.cached,
                "ms": {"%dx%d" % c: round(t, 4) for c, t in sorted(self.ms.items())}}


def pick(ms: Dict[Config, float], order: Sequence[Config]) -> Config:
    """Fastest candidate; ties go to the earlier entry of `order`."""
    best, best_t = None, float("inf")
    for c in order:
        t = ms.get(c)
        if t is not None and t < best_t:
            best, best_t = c, t
    if best is None:
        raise ValueError("no candidate was timed")
    return best


def device_name() -> str:
    import torch
    p = torch.cuda.get_device_properties(torch.cuda.current_device())
    return "%s:%s" % (getattr(p, "gcnArchName", "gpu").split(":")[0], p.multi_processor_count)


def _run(timer: Callable[[Config], float], cands: Sequence[Config], key: Optional[str],
         use_cache: bool, cache_path: Optional[str]) -> TuneResult:
    if use_cache and key is not None:
        hit = load_cache(cache_path).get(key)
        if hit and (hit["base_rows"], hit["tile"]) in set(cands):
            ms = {tuple(int(v) for v in c.split("x")): t for c, t in hit.get("ms", {}).items()}
            return TuneResult((hit["base_rows"], hit["tile"]), ms, cached=True)
    ms = {c: timer(c) for c in cands}
    res = TuneResult(pick(ms, cands), ms)
    if key is not None:
        try:
            store_cache(key, res.as_json(), cache_path)
        except OSError:  # the cache only saves time; an unwritable one is skipped
            pass
    return res


def tune_pair(a, b, alphabet: int, base_rows: Optional[int] = None,
              tiles: Sequence[int] = TILES, reps: int = 3, use_cache: bool = True,
              cache_path: Optional[str] = None,
              timer: Optional[Callable[[Config], float]] = None) -> TuneResult:
    """Best (base_rows, tile) for one pair of device byte tensors a, b.

    Each candidate runs one warm-up and `reps` timed steps (build + witness
    trace, HIP events on the current stream); the mean step time decides.
    `timer` replaces the GPU timing (host tests of the selection logic)."""
    m, n = int(a.numel()), int(b.numel())
    cands = candidates(base_rows, tiles, PAIR_BASE_ROWS)
    if timer is None:
        timer = _pair_timer(a, b, alphabet, reps, cands)
        key = cache_key(device_name(), "pair", m, n, alphabet, base_rows)
    else:
        key = cache_key("host", "pair", m, n, alphabet, base_rows)
    return _run(timer, cands, key, use_cache, cache_path)


def _pair_timer(a, b, alphabet: int, reps: int,
                cands: Sequence[Config]) -> Callable[[Config], float]:
    import torch

    from . import lcs
    m, n = int(a.numel()), int(b.numel())
    plans = {}
    need = 0
    for h, t in cands:
        p = lcs.Plan(m, n, alphabet, h, t)
        plans[(h, t)] = p
        need = max(need, p.workspace_for(m, n))
    ws = lcs.alloc_workspace(need)
    cap = max(1, min(m, n))
    ai = torch.empty(cap, dtype=torch.int32, device=ws.device)
    bi = torch.empty(cap, dtype=torch.int32, device=ws.device)
    ld = torch.zeros(1, dtype=torch.int32, device=ws.device)
    stream = torch.cuda.current_stream()

    def timer(c: Config) -> float:
        p = plans[c]
        p.build(a, b, ws)
        p.trace_device(ai, bi, ld)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(reps):
            p.build(a, b, ws)
            p.trace_device(ai, bi, ld)
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    return timer


def tune_batch(batch, mode: int, base_rows: Optional[int] = None, tiles: Sequence[int] = TILES,
               slots: int = 0, sample: int = 512, reps: int = 2, use_cache: bool = True,
               cache_path: Optional[str] = None,
               timer: Optional[Callable[[Config], float]] = None) -> TuneResult:
    """Best (base_rows, tile) for a synth.Batch run in `mode`, timed on its
    first `sample` pairs (wall time of one submit, after a warm-up)."""
    import numpy as np

    from . import lcs
    # the staged and per-pair modes comb their base strips (up to 256 rows);
    # the persistent ones append rows (up to 64)
    rows = PAIR_BASE_ROWS if mode & (lcs.BATCH_STAGED | lcs.BATCH_PER_PAIR) else BASE_ROWS
    cands = candidates(base_rows, tiles, rows)
    k = min(int(sample), batch.count)
    mm = int(np.median(batch.m[:k])) if k else 0
    nn = int(np.median(batch.n[:k])) if k else 0
    if timer is None:
        timer = _batch_timer(batch, k, mode, slots, reps)
        key = cache_key(device_name(), "batch%d" % mode, mm, nn, batch.sigma, base_rows)
    else:
        key = cache_key("host", "batch%d" % mode, mm, nn, batch.sigma, base_rows)
    return _run(timer, cands, key, use_cache, cache_path)


def _batch_timer(batch, k: int, mode: int, slots: int, reps: int) -> Callable[[Config], float]:
    import torch

    from . import lcs, synth
    sub = synth.batch_from_pairs([batch.pair(p) for p in range(k)], batch.sigma)

    def timer(c: Config) -> float:
        h, t = c
        planned = lcs.Batch(sub.count, int(max(sub.m.max(initial=1), sub.n.max(initial=1))),
                            sub.sigma, h, t, slots)
        ws = lcs.alloc_workspace(planned.workspace_bytes)
        lcs.run_batch(sub, mode, h, t, slots, planned=planned, ws=ws)
        best = float("inf")
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            lcs.run_batch(sub, mode, h, t, slots, planned=planned, ws=ws)
            best = min(best, (time.perf_counter() - t0) * 1e3)
        del ws
        planned.close()
        return best

    return timer


def best_pair_config(m: int, n: int, alphabet: int, base_rows: Optional[int] = None,
                     cache_path: Optional[str] = None) -> Config:
    """Cached choice for this size class on the current device, else the default."""
    try:
        key = cache_key(device_name(), "pair", m, n, alphabet, base_rows)
    except Exception:
        return (base_rows or DEFAULT[0], DEFAULT[1])
    hit = load_cache(cache_path).get(key)
    if hit:
        return (hit["base_rows"], hit["tile"])
    return (base_rows or DEFAULT[0], DEFAULT[1])
