"""The persistent batch schedule, checked on the CPU by the library's own host
simulation (lcs_batch_selftest): waits only on earlier tasks, wait targets equal
the number of producers, every task leads to its pair's finish (so slot reuse
is ordered after ALL work of the previous occupant), layouts fit their slots."""
import numpy as np
import pytest

from paper_2309_09072_amd import lcs as L


@pytest.mark.parametrize("base_rows,tile", [(16, 4), (32, 8), (64, 32), (16, 32)])
def test_random_batches(base_rows, tile):
    r = np.random.default_rng(base_rows * 100 + tile)
    for case in range(25):
        count = int(r.integers(1, 40))
        m = [int(x) for x in r.integers(0, 700, count)]
        n = [int(x) for x in r.integers(0, 700, count)]
        for p in range(count):               # plenty of empty and tiny pairs
            if r.random() < 0.15:
                m[p] = 0
            if r.random() < 0.15:
                n[p] = 0
            if r.random() < 0.1:
                m[p] = int(r.integers(1, base_rows + 2))
        slots = int(r.integers(0, count + 1))
        assert L.batch_selftest(m, n, 4, base_rows, tile, slots) == 0, (m, n, slots)


def test_all_slot_counts_with_empties():
    m = [0, 5, 300, 0, 64, 65, 1, 200, 0, 129, 33, 0]
    n = [7, 0, 280, 0, 64, 1, 90, 200, 3, 130, 0, 40]
    for slots in range(0, len(m) + 1):
        assert L.batch_selftest(m, n, 4, 16, 8, slots) == 0, slots


def test_mixed_workload_shapes():
    from paper_2309_09072_amd import synth
    b = synth.batch_mixed(count=300, seed=3)
    assert L.batch_selftest(list(b.m), list(b.n), 4, 64, 32, 64) == 0


def test_rejects_bad_descriptors():
    assert L.batch_selftest([10], [10], 0) == -1
    assert L.batch_selftest([10], [10], 4, 48) == -1
    # base strips of more than 64 rows are for the combing modes only
    assert L.batch_selftest([10], [10], 4, 128) == -1
    assert L.batch_selftest([10], [10], 4, 256) == -1
    assert L.batch_selftest([100], [10], 4, max_len=50) == -2
