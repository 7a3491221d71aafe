"""The paper's own problem shapes (Section III) on the GPU, exact against the
oracle: every Table I shape (string lengths 1024..8192 against 2..16) with the
long string on the rows, on the columns, and on the rows with the orientation
choice; and the shapes of Figs. 3/4 (one string held at 2 or 4 symbols, the
other grown from 2 to 8192), in both orientations.  The paper does not say
which string is on the rows, nor what the strings contain; uniform strings over
four symbols stand in."""
import numpy as np
import pytest

import oracle
from paper_2309_09072_amd import lcs as L
from paper_2309_09072_amd import synth

pytestmark = pytest.mark.gpu

TABLE_I_S1 = (1024, 2048, 4096, 8192)
TABLE_I_S2 = (2, 4, 8, 16)
FIG_FIXED = (2, 4)
FIG_SIZES = tuple(2 ** e for e in range(1, 14))


def run(a, b, orient):
    import torch
    m, n = a.size, b.size
    plan = L.Plan(m, n, 4, 64, 32, orient=orient)
    ws = L.alloc_workspace(plan.workspace_for(m, n))
    plan.build(L.device_bytes(a), L.device_bytes(b), ws)
    cap = max(1, min(m, n))
    ai = torch.full((cap,), -1, dtype=torch.int32, device="cuda")
    bi = torch.full((cap,), -1, dtype=torch.int32, device="cuda")
    Lg = plan.trace(ai, bi)
    plan.close()
    return Lg, ai[:Lg].cpu().numpy(), bi[:Lg].cpu().numpy()


def check(a, b, orient):
    Lg, ai, bi = run(a, b, orient)
    Lo, ao, bo = oracle.lcs_witness(a, b)
    assert Lg == Lo, (a.size, b.size, orient, Lg, Lo)
    assert np.array_equal(ai, ao) and np.array_equal(bi, bo), (a.size, b.size, orient)


@pytest.mark.parametrize("s1", TABLE_I_S1)
def test_table_i_shapes(s1):
    g = np.random.default_rng(synth.SEED_BASE + 60 + s1)
    for s2 in TABLE_I_S2:
        x, y = synth.uniform(g, s1, 4), synth.uniform(g, s2, 4)
        print("table I shape", s1, s2, flush=True)
        check(x, y, False)   # long string on the rows
        check(y, x, False)   # long string on the columns
        check(x, y, True)    # long string on the rows, oriented build


@pytest.mark.parametrize("fixed", FIG_FIXED)
def test_figure_3_4_shapes(fixed):
    g = np.random.default_rng(synth.SEED_BASE + 70 + fixed)
    for size in FIG_SIZES:
        x, y = synth.uniform(g, size, 4), synth.uniform(g, fixed, 4)
        print("figure shape", size, fixed, flush=True)
        check(x, y, True)
        check(y, x, False)
