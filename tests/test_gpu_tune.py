"""Autotuner on the GPU: the chosen shape is exact and is cached."""
import numpy as np
import pytest

import oracle
from paper_2309_09072_amd import lcs, synth, tune

pytestmark = pytest.mark.gpu


def test_tune_pair_exact_and_cached(tmp_path):
    path = str(tmp_path / "tune.json")
    g = np.random.default_rng(synth.SEED_BASE + 70)
    a = synth.uniform(g, 1000, 4)
    b = synth.uniform(g, 1300, 4)
    ad, bd = lcs.device_bytes(a), lcs.device_bytes(b)
    r = tune.tune_pair(ad, bd, 4, reps=1, cache_path=path)
    assert not r.cached and set(r.ms) == set(tune.candidates(rows=tune.PAIR_BASE_ROWS))
    assert all(t > 0 for t in r.ms.values())
    h, t = r.best
    length, ai, bi = lcs.lcs(a, b, 4, base_rows=h, tile=t)
    want_len, want_a, want_b = oracle.lcs_witness(a, b)
    assert length == want_len
    assert np.array_equal(ai, want_a) and np.array_equal(bi, want_b)
    r2 = tune.tune_pair(ad, bd, 4, reps=1, cache_path=path)
    assert r2.cached and r2.best == r.best
    assert tune.best_pair_config(1000, 1300, 4, cache_path=path) == r.best


def test_tune_batch_staged(tmp_path):
    path = str(tmp_path / "tune.json")
    batch = synth.batch_mixed(count=48, lo=64, hi=400, seed=synth.SEED_BASE + 71)
    r = tune.tune_batch(batch, lcs.BATCH_STAGED, base_rows=64, tiles=(16, 32), sample=48,
                        reps=1, cache_path=path)
    assert set(r.ms) == {(64, 16), (64, 32)}
    lengths, _, _, _ = lcs.run_batch(batch, lcs.BATCH_STAGED, *r.best)
    for p in range(batch.count):
        a, b = batch.pair(p)
        assert lengths[p] == oracle.lcs_length(a, b)
