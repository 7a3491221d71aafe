"""Serving on the GPU: results of requests admitted while others run are the
oracle's, identical alone and in the mix (integers: tolerance 0); the arena
budget is never exceeded; oversize requests are refused."""
import time

import numpy as np
import pytest

import oracle
from paper_2309_09072_amd import lcs as L
from paper_2309_09072_amd import synth

pytestmark = pytest.mark.gpu


def serve_all(server, reqs, gap=0.0):
    import torch
    outs, results = {}, {}
    bufs = {}
    for r in reqs:       # output buffers ready before any submit (the server uses its own streams)
        cap = max(1, min(r.a.size, r.b.size))
        bufs[r.rid] = (torch.full((cap,), -1, dtype=torch.int32, device="cuda"),
                       torch.full((cap,), -1, dtype=torch.int32, device="cuda"))
    torch.cuda.synchronize()
    pending = list(reqs)
    while pending or len(results) < len(reqs):
        if pending:
            r = pending[0]
            ai, bi = bufs[r.rid]
            st = server.submit(r.rid, r.a, r.b, r.sigma, ai, bi)
            if st == 0:
                outs[r.rid] = (ai, bi)
                pending.pop(0)
            else:
                assert st == -10        # queue full: poll and retry
        for tag, status, length, ts, tadm, tdone in server.poll():
            assert status == 0, status
            ai, bi = outs[tag]
            results[tag] = (length, ai[:length].cpu().numpy(), bi[:length].cpu().numpy(), ts, tadm, tdone)
        if gap:
            time.sleep(gap)
    return results


def test_alone_and_mixed_equal_oracle():
    import torch
    reqs = synth.serving_requests(60, rate=1000.0, seed=11, lo=16, hi=900)
    arena = L.alloc_workspace(256 << 20)
    server = L.Server(arena, 900, 20, slots=6, max_queue=16, base_rows=32, tile=16)
    mixed = serve_all(server, reqs)
    running, waiting, used, peak = server.pending()
    assert running == 0 and waiting == 0 and used == 0
    assert 0 < peak <= arena.numel()
    overlap = sum(1 for r in mixed.values() if r[4] < max(x[5] for x in mixed.values()))
    for r in reqs:
        L_, ai, bi = mixed[r.rid][:3]
        Lo, ao, bo = oracle.lcs_witness(r.a, r.b)
        assert L_ == Lo and np.array_equal(ai, ao) and np.array_equal(bi, bo), r.rid
    # the same requests one at a time through the same server
    for r in reqs[:12]:
        alone = serve_all(server, [r])
        assert alone[r.rid][0] == mixed[r.rid][0]
        assert np.array_equal(alone[r.rid][1], mixed[r.rid][1])
        assert np.array_equal(alone[r.rid][2], mixed[r.rid][2])
    server.close()


def test_budget_and_oversize():
    arena = L.alloc_workspace(8 << 20)
    server = L.Server(arena, 2048, 4, slots=4, max_queue=64, base_rows=64, tile=32)
    big = np.zeros(2048, np.uint8)
    assert server.footprint(2048, 2048) > arena.numel()
    assert server.submit(1, big, big, 4) == -9                  # can never fit
    reqs = synth.serving_requests(20, rate=1000.0, seed=3, lo=64, hi=300)
    for r in reqs:
        r.sigma = min(r.sigma, 4)
        r.a = (r.a % 4).astype(np.uint8)
        r.b = (r.b % 4).astype(np.uint8)
    res = serve_all(server, reqs)
    assert server.pending()[3] <= arena.numel()
    for r in reqs:
        assert res[r.rid][0] == oracle.lcs_length(r.a, r.b)
    server.close()
