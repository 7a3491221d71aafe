"""Seeded synthetic inputs shaped like the paper's workloads.

This module holds no LCS arithmetic: it only draws symbol strings, mutated
copies, batch descriptors and request arrival times.  Both the HIP path (via
tests and ``bench.py``) and the CPU oracle are fed the same bytes from here.

The paper states string lengths only (Table I, Figs. 3-4), not the content or
the alphabet, so every workload is synthetic: symbols are uint8 codes
0..sigma-1 drawn i.i.d. uniform from ``numpy.random.Generator(PCG64(seed))``.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

SEED_BASE = 230909072


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def uniform(g: np.random.Generator, length: int, sigma: int) -> np.ndarray:
    """i.i.d. uniform symbols 0..sigma-1."""
    return g.integers(0, sigma, size=int(length), dtype=np.uint8)


def mutate(g: np.random.Generator, x: np.ndarray, sigma: int,
           p_sub: float, p_ins: float, p_del: float) -> np.ndarray:
    """Edit-model copy of x.

    For each symbol: with probability p_del drop it; otherwise with p_sub
    replace it by a uniformly chosen different symbol; then with p_ins insert
    a uniform symbol after it.
    """
    x = np.asarray(x, dtype=np.uint8)
    k = x.size
    u_del = g.random(k)
    u_sub = g.random(k)
    shift = g.integers(1, max(sigma, 2), size=k)
    u_ins = g.random(k)
    ins_sym = g.integers(0, sigma, size=k, dtype=np.uint8)
    out = []
    for t in range(k):
        if u_del[t] < p_del:
            continue
        s = int(x[t])
        if sigma > 1 and u_sub[t] < p_sub:
            s = (s + int(shift[t])) % sigma
        out.append(s)
        if u_ins[t] < p_ins:
            out.append(int(ins_sym[t]))
    return np.asarray(out, dtype=np.uint8)


def fit_length(g: np.random.Generator, x: np.ndarray, n: int, sigma: int) -> np.ndarray:
    """Truncate x to n symbols or pad it with i.i.d. uniform symbols."""
    if x.size >= n:
        return x[:n].copy()
    return np.concatenate([x, uniform(g, n - x.size, sigma)])


# ----------------------------------------------------------------------------
# single pairs


@dataclass
class Pair:
    a: np.ndarray   # row string
    b: np.ndarray   # column string
    sigma: int
    seed: int
    name: str


def pair_uniform(m: int, n: int, sigma: int, seed: int, name: str = "uniform") -> Pair:
    g = rng(seed)
    return Pair(uniform(g, m, sigma), uniform(g, n, sigma), sigma, seed, name)


def pair_mutated(m: int, n: int, sigma: int, seed: int, p_sub: float, p_ins: float,
                 p_del: float, name: str = "mutated") -> Pair:
    g = rng(seed)
    a = uniform(g, m, sigma)
    b = fit_length(g, mutate(g, a, sigma, p_sub, p_ins, p_del), n, sigma)
    return Pair(a, b, sigma, seed, name)


def config_small() -> Pair:
    """256 x 256, alphabet 4 (ACGT as 0..3), i.i.d. uniform."""
    return pair_uniform(256, 256, 4, SEED_BASE + 1, "pair-256x256-s4")


def config_4096() -> Pair:
    """4096 x 4096, alphabet 4, i.i.d. uniform; 64-row base strips."""
    return pair_uniform(4096, 4096, 4, SEED_BASE + 2, "pair-4096x4096-s4")


def config_16384() -> Pair:
    """16384 x 16384, alphabet 20; b is a 10%/5%/5% (sub/ins/del) mutated copy of a."""
    return pair_mutated(16384, 16384, 20, SEED_BASE + 3, 0.10, 0.05, 0.05,
                        "pair-16384x16384-s20-mut20")


# ----------------------------------------------------------------------------
# batches


@dataclass
class Batch:
    symbols: np.ndarray        # all strings back to back
    a_off: np.ndarray          # int64 offsets into symbols
    b_off: np.ndarray
    m: np.ndarray              # int32 lengths
    n: np.ndarray
    sigma: int
    seed: int
    name: str

    @property
    def count(self) -> int:
        return int(self.m.size)

    def pair(self, p: int):
        a = self.symbols[self.a_off[p]:self.a_off[p] + self.m[p]]
        b = self.symbols[self.b_off[p]:self.b_off[p] + self.n[p]]
        return a, b

    @property
    def cells(self) -> int:
        return int(np.sum(self.m.astype(np.int64) * self.n.astype(np.int64)))


def _pack(pairs, sigma, seed, name) -> Batch:
    parts, a_off, b_off, ms, ns = [], [], [], [], []
    off = 0
    for a, b in pairs:
        a_off.append(off); parts.append(a); off += a.size
        b_off.append(off); parts.append(b); off += b.size
        ms.append(a.size); ns.append(b.size)
    sym = np.concatenate(parts) if parts else np.zeros(0, np.uint8)
    return Batch(sym, np.asarray(a_off, np.int64), np.asarray(b_off, np.int64),
                 np.asarray(ms, np.int32), np.asarray(ns, np.int32), sigma, seed, name)


def batch_mixed(count: int = 4096, lo: int = 64, hi: int = 2048, sigma: int = 4,
                seed: int = SEED_BASE + 4, edit: float = 0.15) -> Batch:
    """Even-indexed pairs: m, n independent U[lo, hi], i.i.d. symbols.  Odd-indexed:
    m ~ U[lo, hi], b a mutated copy of a at total edit rate ``edit`` split 2:1:1
    (sub/ins/del), its length clamped to [lo, hi] by truncation or padding."""
    g = rng(seed)
    pairs = []
    for p in range(count):
        m = int(g.integers(lo, hi + 1))
        a = uniform(g, m, sigma)
        if p % 2 == 0:
            b = uniform(g, int(g.integers(lo, hi + 1)), sigma)
        else:
            b = mutate(g, a, sigma, edit / 2, edit / 4, edit / 4)
            n = min(max(b.size, lo), hi)
            b = fit_length(g, b, n, sigma)
        pairs.append((a, b))
    return _pack(pairs, sigma, seed, "batch-%d-pairs-%d..%d-s%d" % (count, lo, hi, sigma))


def batch_from_pairs(pairs, sigma, seed=0, name="batch") -> Batch:
    return _pack([(np.asarray(a, np.uint8), np.asarray(b, np.uint8)) for a, b in pairs],
                 sigma, seed, name)


# ----------------------------------------------------------------------------
# serving


@dataclass
class Request:
    rid: int
    arrival: float       # seconds after the start of the run
    a: np.ndarray
    b: np.ndarray
    sigma: int


def serving_requests(count: int, rate: float, seed: int = SEED_BASE + 5,
                     lo: int = 128, hi: int = 8192, p_related: float = 0.30,
                     edit: float = 0.10):
    """Poisson arrivals at ``rate`` per second.  m log-uniform in [lo, hi];
    alphabet 4 or 20 with probability 1/2 each; a fraction ``p_related`` of the
    pairs are mutated copies at total edit rate ``edit`` (split 2:1:1), the rest
    have an independent log-uniform n."""
    g = rng(seed)
    t = 0.0
    out = []
    for r in range(count):
        t += float(g.exponential(1.0 / rate)) if rate > 0 else 0.0
        sigma = 4 if g.random() < 0.5 else 20
        m = int(round(np.exp(g.uniform(np.log(lo), np.log(hi)))))
        a = uniform(g, m, sigma)
        if g.random() < p_related:
            b = mutate(g, a, sigma, edit / 2, edit / 4, edit / 4)
            if b.size == 0:
                b = uniform(g, 1, sigma)
            b = b[:hi]  # insertions may carry a copy past the longest length
        else:
            n = int(round(np.exp(g.uniform(np.log(lo), np.log(hi)))))
            b = uniform(g, n, sigma)
        out.append(Request(r, t, a, b, sigma))
    return out
