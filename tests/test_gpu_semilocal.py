"""Semi-local queries LCS(a, b[i:k]) from the top breakout matrix, against the oracle."""
import json
import os

import numpy as np
import pytest
import torch

import oracle
from paper_2309_09072_amd import lcs, synth

pytestmark = pytest.mark.gpu


def run(a, b, sigma, qi, qk, base_rows=16, tile=8):
    ad, bd = lcs.device_bytes(a), lcs.device_bytes(b)
    plan = lcs.Plan(max(a.size, 1), max(b.size, 1), sigma, base_rows, tile)
    ws = lcs.alloc_workspace(plan.workspace_for(a.size, b.size))
    plan.build(ad, bd, ws)
    ti = torch.tensor(np.asarray(qi, np.int32), device="cuda")
    tk = torch.tensor(np.asarray(qk, np.int32), device="cuda")
    out = plan.semilocal(ti, tk)
    torch.cuda.synchronize()
    plan.close()
    return out.cpu().numpy()


def all_queries(n):
    qi, qk = zip(*[(i, k) for i in range(n + 1) for k in range(i, n + 1)])
    return list(qi), list(qk)


def test_every_substring_small():
    g = np.random.default_rng(synth.SEED_BASE + 80)
    a, b = synth.uniform(g, 37, 3), synth.uniform(g, 29, 3)   # 3 base strips of 16 rows
    qi, qk = all_queries(b.size)
    got = run(a, b, 3, qi, qk)
    want = [oracle.lcs_length(a, b[i:k]) for i, k in zip(qi, qk)]
    assert got.tolist() == want


def test_paper_grid_every_substring():
    ex = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_example.json")))
    grid = ex["grid"]
    codes = {c: x for x, c in enumerate("acgt")}
    a = np.array([codes[c] for c in grid["a_rows"]], np.uint8)
    b = np.array([codes[c] for c in grid["b_cols"]], np.uint8)
    qi, qk = all_queries(b.size)
    got = run(a, b, 4, qi, qk, base_rows=16, tile=4)
    want = [oracle.lcs_length(a, b[i:k]) for i, k in zip(qi, qk)]
    assert got.tolist() == want


def test_sampled_queries_several_levels_and_bad_queries():
    g = np.random.default_rng(synth.SEED_BASE + 81)
    a = synth.uniform(g, 300, 4)
    b = synth.mutate(g, a, 4, 0.1, 0.05, 0.05)[:260]
    n = b.size
    qi = g.integers(0, n + 1, 300)
    qk = np.array([g.integers(i, n + 1) for i in qi])
    bad_i = [-1, 5, n + 1, 0, 3]
    bad_k = [4, 4, n + 1, n + 1, -2]
    got = run(a, b, 4, list(qi) + bad_i, list(qk) + bad_k)
    want = [oracle.lcs_length(a, b[i:k]) for i, k in zip(qi, qk)]
    assert got[:300].tolist() == want
    assert got[300:].tolist() == [-1] * 5
    # whole-string query equals the length
    assert run(a, b, 4, [0], [n])[0] == oracle.lcs_length(a, b)


def test_empty_strings():
    b = np.array([0, 1, 2], np.uint8)
    assert run(np.zeros(0, np.uint8), b, 4, [0, 1, 0, 2], [3, 2, 0, 1]).tolist() == [0, 0, 0, -1]
    assert run(b, np.zeros(0, np.uint8), 4, [0, 0], [0, 1]).tolist() == [0, -1]
