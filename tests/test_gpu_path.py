"""Full path listing (lcs_path, Section II-E) against the oracle's path rows:
the first and last column the canonical (leftmost) path visits on every grid
row, from the textbook table's LEFT > DIAG > UP walk (pinned by brute force)."""
import numpy as np
import pytest
import torch

import oracle
from paper_2309_09072_amd import lcs, synth

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("m,n,sigma,seed", [(120, 150, 4, 1), (200, 90, 2, 2), (64, 64, 1, 3),
                                            (150, 150, 20, 4), (0, 40, 4, 5), (33, 0, 4, 6),
                                            (1, 70, 4, 7), (90, 1, 3, 8)])
def test_path_matches_oracle(m, n, sigma, seed):
    g = np.random.default_rng(synth.SEED_BASE + 130 + seed)
    a = synth.uniform(g, m, sigma)
    b = synth.mutate(g, a, sigma, 0.1, 0.05, 0.05)[:n] if seed % 2 else synth.uniform(g, n, sigma)
    b = np.concatenate([b, synth.uniform(g, n - b.size, sigma)]) if b.size < n else b
    plan = lcs.Plan(max(m, 1), max(n, 1), sigma, 16, 8)
    ws = lcs.alloc_workspace(plan.workspace_for(m, n))
    ad = lcs.device_bytes(a) if m else torch.zeros(1, dtype=torch.uint8, device="cuda")
    bd = lcs.device_bytes(b) if n else torch.zeros(1, dtype=torch.uint8, device="cuda")
    plan.build(ad[:m], bd[:n], ws)
    cap = max(1, min(m, n))
    ai = torch.empty(cap, dtype=torch.int32, device="cuda")
    bi = torch.empty(cap, dtype=torch.int32, device="cuda")
    ld = torch.zeros(1, dtype=torch.int32, device="cuda")
    plan.trace_device(ai, bi, ld)
    cin, cout = plan.path(ai, bi, ld, m)
    torch.cuda.synchronize()
    lo, hi = oracle.path_rows(a, b)
    assert cin.cpu().numpy().tolist() == lo.tolist()
    assert cout.cpu().numpy().tolist() == hi.tolist()
    plan.close()
