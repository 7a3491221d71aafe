"""Oriented builds (LCS_PLAN_ORIENT): the shorter string on the rows, the same
length and canonical witness as the oracle for the caller's (a, b)."""
import numpy as np
import pytest
import torch

import oracle
from paper_2309_09072_amd import lcs, synth

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("m,n,sigma,h0,tile,seed", [
    (700, 300, 4, 16, 8, 1), (2000, 40, 4, 64, 32, 2), (513, 512, 2, 32, 16, 3),
    (3000, 700, 20, 64, 32, 4), (65, 1, 4, 16, 4, 5), (300, 300, 4, 16, 8, 6), (40, 900, 4, 16, 8, 7)])
def test_oriented_matches_oracle(m, n, sigma, h0, tile, seed):
    g = np.random.default_rng(synth.SEED_BASE + 100 + seed)
    a = synth.uniform(g, m, sigma)
    b = synth.mutate(g, a[:n], sigma, 0.1, 0.05, 0.05)[:n] if n <= m else synth.uniform(g, n, sigma)
    L, ai, bi = lcs.lcs(a, b, sigma, h0, tile, orient=True)
    want = oracle.lcs_witness(a, b)
    assert L == want[0]
    assert np.array_equal(ai, want[1]) and np.array_equal(bi, want[2])


def test_oriented_device_trace_and_semilocal_state():
    g = np.random.default_rng(synth.SEED_BASE + 120)
    a, b = synth.uniform(g, 900, 4), synth.uniform(g, 200, 4)
    ad, bd = lcs.device_bytes(a), lcs.device_bytes(b)
    plan = lcs.Plan(900, 200, 4, 16, 8, orient=True)
    ws = lcs.alloc_workspace(plan.workspace_for(900, 200))
    plan.build(ad, bd, ws)
    ai = torch.full((200,), -7, dtype=torch.int32, device="cuda")
    bi = torch.full((200,), -7, dtype=torch.int32, device="cuda")
    ld = torch.zeros(1, dtype=torch.int32, device="cuda")
    plan.trace_device(ai, bi, ld)
    torch.cuda.synchronize()
    L = int(ld.item())
    want = oracle.lcs_witness(a, b)
    assert L == want[0] == plan.length()
    assert np.array_equal(ai[:L].cpu().numpy(), want[1])
    assert np.array_equal(bi[:L].cpu().numpy(), want[2])
    with pytest.raises(lcs.LcsError):   # semi-local queries refer to substrings of b
        plan.semilocal(torch.zeros(1, dtype=torch.int32, device="cuda"),
                       torch.ones(1, dtype=torch.int32, device="cuda"))
    plan.close()
