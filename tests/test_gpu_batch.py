"""Batches on the GPU: every pair's length and witness equals the oracle's, for
the persistent single launch, its graph replay and the one-pair-per-launch
mode, including slot reuse, empty pairs and a bad symbol."""
import sys

import numpy as np
import pytest

import oracle
from paper_2309_09072_amd import lcs as L
from paper_2309_09072_amd import synth

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def mixed_small(count, seed, maxlen=300, sigma=4):
    r = np.random.default_rng(seed)
    pairs = []
    for p in range(count):
        m = int(r.integers(0, maxlen)) if p % 11 else 0
        n = int(r.integers(0, maxlen)) if p % 13 else 0
        a = r.integers(0, sigma, m).astype(np.uint8)
        if p % 3 == 1 and m > 0:
            b = synth.fit_length(r, synth.mutate(r, a, sigma, 0.1, 0.05, 0.05), max(n, 1), sigma)
        else:
            b = r.integers(0, sigma, n).astype(np.uint8)
        pairs.append((a, b))
    return synth.batch_from_pairs(pairs, sigma, seed, "mixed")


def check(batch, lengths, ai, bi, off, skip=()):
    for p in range(batch.count):
        if p in skip:
            continue
        a, b = batch.pair(p)
        Lo, ao, bo = oracle.lcs_witness(a, b)
        assert lengths[p] == Lo, "pair %d (%dx%d): %d vs oracle %d" % (p, a.size, b.size, lengths[p], Lo)
        assert np.array_equal(ai[off[p]:off[p] + Lo], ao), "pair %d a_idx" % p
        assert np.array_equal(bi[off[p]:off[p] + Lo], bo), "pair %d b_idx" % p


@pytest.mark.parametrize("base_rows,tile,slots", [(16, 8, 7), (32, 32, 0), (64, 16, 3)])
def test_persistent_matches_oracle(base_rows, tile, slots):
    batch = mixed_small(60, 40 + base_rows)
    say("persistent", base_rows, tile, slots)
    res = L.run_batch(batch, L.BATCH_PERSISTENT, base_rows, tile, slots)
    check(batch, *res)


@pytest.mark.parametrize("base_rows,tile,slots", [(16, 8, 2), (32, 32, 0), (64, 16, 1), (128, 16, 3),
                                                  (256, 32, 0), (512, 32, 5), (1024, 16, 0)])
def test_staged_matches_oracle(base_rows, tile, slots):
    """Staged launches; small slot areas force the pairs into several waves.
    Base strips of 128 to 1024 rows (staged mode only) get pairs long enough
    for several strips and combine levels."""
    batch = mixed_small(60, 50 + base_rows, maxlen=300 if base_rows <= 64 else 1100 if base_rows <= 256 else
                        1700 if base_rows <= 512 else 2400)
    say("staged", base_rows, tile, slots)
    res = L.run_batch(batch, L.BATCH_STAGED, base_rows, tile, slots)
    check(batch, *res)


def test_tall_base_strips_staged_or_per_pair_only():
    batch = mixed_small(4, 7)
    for mode in (L.BATCH_PERSISTENT, L.BATCH_PAIR_QUEUE):
        with pytest.raises(L.LcsError) as e:
            L.run_batch(batch, mode, 128, 32, 0)
        assert e.value.status == -1
    check(batch, *L.run_batch(batch, L.BATCH_PER_PAIR, 256, 32, 0))


@pytest.mark.parametrize("base_rows,tile,slots", [(16, 8, 3), (32, 32, 0), (64, 16, 1)])
def test_pair_queue_matches_oracle(base_rows, tile, slots):
    """Pair queue: one work-group per pair; fewer slots than pairs means a
    work-group runs many pairs in its slot."""
    batch = mixed_small(60, 60 + base_rows)
    say("pair queue", base_rows, tile, slots)
    res = L.run_batch(batch, L.BATCH_PAIR_QUEUE, base_rows, tile, slots)
    check(batch, *res)


def test_pair_queue_graph_replays():
    batch = mixed_small(40, 79)
    plan = L.Batch(batch.count, 300, 4, 32, 16, 6)
    ws = L.alloc_workspace(plan.workspace_bytes)
    r1 = L.run_batch(batch, L.BATCH_PER_PAIR, planned=plan, ws=ws)
    check(batch, *r1)
    for rep in range(3):
        r2 = L.run_batch(batch, L.BATCH_PAIR_QUEUE | L.BATCH_GRAPH, planned=plan, ws=ws)
        for x, y in zip(r1, r2):
            assert np.array_equal(x, y), "replay %d differs" % rep


def test_staged_graph_replays():
    batch = mixed_small(40, 78)
    plan = L.Batch(batch.count, 300, 4, 32, 16, 4)
    ws = L.alloc_workspace(plan.workspace_bytes)
    r1 = L.run_batch(batch, L.BATCH_PER_PAIR, planned=plan, ws=ws)
    check(batch, *r1)
    for rep in range(3):
        r2 = L.run_batch(batch, L.BATCH_STAGED | L.BATCH_GRAPH, planned=plan, ws=ws)
        for x, y in zip(r1, r2):
            assert np.array_equal(x, y), "replay %d differs" % rep


def test_per_pair_and_graph_agree():
    batch = mixed_small(40, 77)
    plan = L.Batch(batch.count, 300, 4, 32, 16, 5)
    ws = L.alloc_workspace(plan.workspace_bytes)
    r1 = L.run_batch(batch, L.BATCH_PER_PAIR, planned=plan, ws=ws)
    check(batch, *r1)
    for rep in range(3):   # graph capture, then replays with eager work in between
        r2 = L.run_batch(batch, L.BATCH_PERSISTENT | L.BATCH_GRAPH, planned=plan, ws=ws)
        for x, y in zip(r1, r2):
            assert np.array_equal(x, y), "replay %d differs" % rep
        r3 = L.run_batch(batch, L.BATCH_PERSISTENT, planned=plan, ws=ws)
        for x, y in zip(r1, r3):
            assert np.array_equal(x, y)


def test_bad_symbol_only_fails_its_pair():
    r = np.random.default_rng(5)
    pairs = [(r.integers(0, 4, 100).astype(np.uint8), r.integers(0, 4, 90).astype(np.uint8))
             for _ in range(6)]
    pairs[3] = (np.array([0, 1, 7, 2], np.uint8), np.array([0, 1, 2], np.uint8))
    pairs[4] = (np.array([0, 1, 3, 2], np.uint8), np.array([0, 5, 2], np.uint8))  # bad column symbol
    batch = synth.batch_from_pairs(pairs, 4)
    for mode in (L.BATCH_PERSISTENT, L.BATCH_PAIR_QUEUE, L.BATCH_STAGED, L.BATCH_PER_PAIR):
        lengths, ai, bi, off = L.run_batch(batch, mode, 16, 8, 2)
        assert lengths[3] == -5 and lengths[4] == -5, mode
        check(batch, lengths, ai, bi, off, skip=(3, 4))


def test_mixed_workload_sample():
    """512 pairs of the 64..2048 mixed workload (half unrelated, half mutated copies)."""
    batch = synth.batch_mixed(count=512, seed=synth.SEED_BASE + 40)
    say("mixed 512 pairs, cells", batch.cells)
    for mode in (L.BATCH_STAGED, L.BATCH_PERSISTENT, L.BATCH_PAIR_QUEUE):
        res = L.run_batch(batch, mode, 64, 32, 0)
        check(batch, *res)


def test_tall_pairs_every_bracket_shape():
    """Pairs tall enough for child strips of 512, 1024 and 2048 rows (the
    cooperative and wide-window bracket shapes) next to a short one, in every
    one-launch mode."""
    r = np.random.default_rng(4200)
    a0 = r.integers(0, 4, 4200).astype(np.uint8)
    b0 = synth.fit_length(r, synth.mutate(r, a0, 4, 0.1, 0.05, 0.05), 3000, 4)
    a1 = r.integers(0, 4, 2500).astype(np.uint8)
    b1 = r.integers(0, 4, 2600).astype(np.uint8)
    a2 = r.integers(0, 4, 100).astype(np.uint8)
    b2 = r.integers(0, 4, 90).astype(np.uint8)
    batch = synth.batch_from_pairs([(a0, b0), (a1, b1), (a2, b2)], 4, 4200, "tall")
    for mode in (L.BATCH_STAGED, L.BATCH_PERSISTENT, L.BATCH_PAIR_QUEUE):
        say("tall pairs, mode", mode)
        check(batch, *L.run_batch(batch, mode, 64, 32, 0))


@pytest.mark.parametrize("sigma", [20, 256])
def test_large_alphabets_every_mode(sigma):
    """Alphabets whose next-match stage spans several chunks of the persistent
    task queue (one task per symbol, 16 per chunk), and at 256 symbols base
    strips with the global next-match tables; fewer slots than pairs."""
    batch = mixed_small(30, 90 + sigma, maxlen=400, sigma=sigma)
    for mode in (L.BATCH_PERSISTENT, L.BATCH_STAGED, L.BATCH_PAIR_QUEUE):
        say("alphabet", sigma, "mode", mode)
        check(batch, *L.run_batch(batch, mode, 32, 16, 5))


@pytest.mark.parametrize("mode", [L.BATCH_STAGED, L.BATCH_PERSISTENT, L.BATCH_PAIR_QUEUE])
def test_graph_replay_follows_a_new_b_idx_buffer(mode):
    """A graph replay with only the b_idx buffer changed writes the new buffer
    (every device pointer the captured kernels take is part of the graph key)
    and leaves the old one alone."""
    import torch
    batch = mixed_small(24, 81)
    plan = L.Batch(batch.count, 300, 4, 32, 16, 5)
    ws = L.alloc_workspace(plan.workspace_bytes)
    sym = L.device_bytes(batch.symbols)
    off = L.Batch.witness_offsets(batch.m, batch.n)
    cap = max(int(off[-1]), 1)
    lengths = torch.full((batch.count,), -99, dtype=torch.int32, device="cuda")
    ai = torch.full((cap,), -1, dtype=torch.int32, device="cuda")
    b_old = torch.full((cap,), -1, dtype=torch.int32, device="cuda")
    b_new = torch.full((cap,), -1, dtype=torch.int32, device="cuda")
    plan.submit(sym, batch.a_off, batch.b_off, batch.m, batch.n, ws, lengths, ai, b_old,
                mode | L.BATCH_GRAPH)
    torch.cuda.synchronize()
    check(batch, lengths.cpu().numpy(), ai.cpu().numpy(), b_old.cpu().numpy(), off)
    b_old.fill_(-7)
    lengths.fill_(-99)
    ai.fill_(-1)
    torch.cuda.synchronize()
    plan.submit(sym, batch.a_off, batch.b_off, batch.m, batch.n, ws, lengths, ai, b_new,
                mode | L.BATCH_GRAPH)
    torch.cuda.synchronize()
    check(batch, lengths.cpu().numpy(), ai.cpu().numpy(), b_new.cpu().numpy(), off)
    assert bool((b_old == -7).all()), "the replay wrote into the old b_idx buffer"
    plan.close()
