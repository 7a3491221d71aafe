"""GPU parity: the HIP path against the CPU oracle, through the C ABI.

Breakout matrices are compared cell for cell with the oracle's definition at
sizes that span several tiles and ragged tails; lengths and witnesses are
compared exactly (integer results, tolerance 0) up to the 16384 x 16384 pair.
"""
import sys

import numpy as np
import pytest

import oracle
from paper_2309_09072_amd import lcs as L
from paper_2309_09072_amd import synth

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def run_pair(a, b, sigma, base_rows=0, tile=0, check_levels=False, trace=True):
    import torch
    a = np.asarray(a, np.uint8)
    b = np.asarray(b, np.uint8)
    m, n = a.size, b.size
    ad, bd = L.device_bytes(a), L.device_bytes(b)
    plan = L.Plan(m, n, sigma, base_rows, tile)
    ws = L.alloc_workspace(plan.workspace_for(m, n))
    plan.build(ad, bd, ws)
    Lg = plan.length()
    if check_levels and m > 0 and n > 0:
        for lv, cnt in enumerate(plan.levels()):
            for s in range(cnt):
                D, row0 = plan.dist(lv, s, ws)
                Dh = D.cpu().numpy()
                h = Dh.shape[1] - 1
                want = oracle.dist_rows(a, row0, row0 + h, b)
                bad = np.argwhere(Dh[: n + 1] != want)
                assert bad.size == 0, "level %d strip %d (rows %d..%d): first mismatch %s got %d want %d" % (
                    lv, s, row0, row0 + h, bad[0], Dh[tuple(bad[0])], want[tuple(bad[0])])
                assert np.all(Dh[n + 1] == n + 1)
    wit = None
    if trace:
        cap = max(1, min(m, n))
        ai = torch.full((cap,), -1, dtype=torch.int32, device="cuda")
        bi = torch.full((cap,), -1, dtype=torch.int32, device="cuda")
        Lt = plan.trace(ai, bi)
        assert Lt == Lg
        wit = (ai[:Lt].cpu().numpy(), bi[:Lt].cpu().numpy())
    return Lg, wit, plan, ws


def check_against_oracle(a, b, sigma, **kw):
    Lg, wit, plan, ws = run_pair(a, b, sigma, **kw)
    Lo, ao, bo = oracle.lcs_witness(np.asarray(a, np.uint8), np.asarray(b, np.uint8))
    assert Lg == Lo, "length %d vs oracle %d" % (Lg, Lo)
    if wit is not None:
        assert np.array_equal(wit[0], ao), "a_idx differs from the oracle's canonical witness"
        assert np.array_equal(wit[1], bo), "b_idx differs from the oracle's canonical witness"
    return Lg, plan, ws


# ----------------------------------------------------------------- small, full D


@pytest.mark.parametrize("base_rows,tile", [(16, 4), (16, 8), (32, 16), (64, 32), (16, 32), (128, 8),
                                            (256, 32), (512, 16), (1024, 32)])
def test_levels_cell_for_cell(base_rows, tile):
    r = np.random.default_rng(100 + base_rows + tile)
    shapes = [(200, 150, 4), (129, 203, 2), (97, 64, 20), (65, 257, 4), (16, 31, 1), (250, 9, 3)]
    if base_rows >= 128:  # several strips of the tall shapes, a short last one
        shapes += [(700, 333, 4), (530, 260, 20), (257, 1100, 2)]
    if base_rows >= 512:
        shapes += [(1300, 700, 4), (1100, 900, 20)]
    if base_rows >= 1024:
        shapes += [(2300, 600, 4), (2100, 1500, 20)]
    for m, n, sig in shapes:
        a = r.integers(0, sig, m).astype(np.uint8)
        b = r.integers(0, sig, n).astype(np.uint8)
        say("levels", base_rows, tile, m, n, sig)
        check_against_oracle(a, b, sig, base_rows=base_rows, tile=tile, check_levels=True)


def _base_rows_check(a, b, plan, ws, verts):
    """Every base strip's rows for the sampled vertices against the oracle."""
    for s in range(plan.levels()[0]):
        D, row0 = plan.dist(0, s, ws)
        h = D.shape[1] - 1
        got = D[verts].cpu().numpy()
        want = oracle.dist_rows(a, row0, row0 + h, b, verts)
        bad = np.argwhere(got != want)
        assert bad.size == 0, "strip %d: vertex %d weight %d got %d want %d" % (
            s, verts[bad[0][0]], bad[0][1], got[tuple(bad[0])], want[tuple(bad[0])])


def test_base_table_window_and_fallback():
    """Matches that jump far ahead.  Case 1: i.i.d. strings.  Case 2: symbol 3
    is absent from b's first 4000 columns.  Single pairs (combed base
    strips): for the vertices left of ~4000 the later breakouts of strips
    holding symbol 3 lie thousands of columns away, so the row generation's
    first-vertex scans run long.  Batches (row-append base strips): those
    strips reach past the LDS window of the next-match tables for every
    vertex block left of ~1950 and take the fallback to the global tables;
    blocks further right see the whole table."""
    r = np.random.default_rng(4242)
    n = 5000
    verts = sorted(set(list(range(0, n + 1, 37)) + [1, 255, 256, 257, 1950, 2954, 2955, n - 1, n]))
    a1 = r.integers(0, 4, 256).astype(np.uint8)
    b1 = r.integers(0, 4, n).astype(np.uint8)
    b2 = np.concatenate([r.integers(0, 3, 4000), r.integers(0, 4, n - 4000)]).astype(np.uint8)
    for a, b in ((a1, b1), (a1, b2)):
        for h0 in (16, 64, 256):
            say("base window", h0, int(b[:4000].max()))
            Lg, plan, ws = check_against_oracle(a, b, 4, base_rows=h0)
            _base_rows_check(a, b, plan, ws, verts)
    batch = synth.batch_from_pairs([(a1, b1), (a1, b2)], 4, 4242, "window")
    for h0 in (16, 64):
        say("batch base window", h0)
        lengths, ai, bi, off = L.run_batch(batch, L.BATCH_STAGED, h0, 32, 0)
        for p in range(batch.count):
            a, b = batch.pair(p)
            Lo, ao, bo = oracle.lcs_witness(a, b)
            assert lengths[p] == Lo, "pair %d: %d vs oracle %d" % (p, lengths[p], Lo)
            assert np.array_equal(ai[off[p]:off[p] + Lo], ao), "pair %d a_idx" % p
            assert np.array_equal(bi[off[p]:off[p] + Lo], bo), "pair %d b_idx" % p


def test_base_strips_alphabet_20():
    """Alphabet 20 (the global next-match tables): base strips of every
    height against the oracle.  Case 1: i.i.d. strings.  Case 2: symbols 18
    and 19 are absent from b's first 3000 columns (matches jump far ahead).
    Case 3: a mutated copy (long matching runs)."""
    r = np.random.default_rng(2020)
    n = 5000
    verts = sorted(set(list(range(0, n + 1, 41)) + [1, 255, 256, 257, 2999, 3000, 3001, n - 1, n]))
    a1 = r.integers(0, 20, 192).astype(np.uint8)
    b1 = r.integers(0, 20, n).astype(np.uint8)
    b2 = np.concatenate([r.integers(0, 18, 3000), r.integers(0, 20, n - 3000)]).astype(np.uint8)
    p3 = synth.pair_mutated(192, 192, 20, 77, 0.10, 0.05, 0.05)
    b3 = np.concatenate([p3.b, r.integers(0, 20, n - p3.b.size)]).astype(np.uint8)
    for a, b in ((a1, b1), (a1, b2), (p3.a, b3)):
        for h0 in (16, 32, 64, 128, 256, 512, 1024):
            say("alphabet 20 base", h0, b.size)
            Lg, plan, ws = check_against_oracle(a, b, 20, base_rows=h0)
            _base_rows_check(a, b, plan, ws, verts)


def test_wide_strings_combed_in_32_bits():
    """More than 32767 columns: labels no longer fit 16 bits, so the base strips
    are combed in the 32-bit form (several column tiles per strip)."""
    r = np.random.default_rng(3232)
    n = 40000
    verts = sorted(set(list(range(0, n + 1, 997)) + [1, 16383, 16384, 32767, 32768, 32769, n - 1, n]))
    for sig, h0 in ((4, 64), (20, 256)):
        a = r.integers(0, sig, 700).astype(np.uint8)
        b = r.integers(0, sig, n).astype(np.uint8)
        say("wide comb", sig, h0)
        Lg, plan, ws = check_against_oracle(a, b, sig, base_rows=h0)
        _base_rows_check(a, b, plan, ws, verts)


def test_combing_in_column_segments():
    """Tall, few base strips are combed by several work-groups per strip (1024
    columns each), handing the row labels on through records: segment counts
    with a full last segment (4096 columns), a one-column last segment (4097)
    and a ragged one, alphabets 4 and 20, base strips of 256, 512 and 1024 rows."""
    r = np.random.default_rng(5150)
    for m, n, sig, h0 in ((1300, 4096, 4, 512), (2100, 4097, 20, 1024), (1100, 7000, 4, 1024),
                          (700, 5000, 4, 256)):
        a = r.integers(0, sig, m).astype(np.uint8)
        b = r.integers(0, sig, n).astype(np.uint8)
        verts = sorted(set(list(range(0, n + 1, 211)) + [1, 1023, 1024, 1025, 2047, 2048, n - 1, n]))
        say("segmented comb", m, n, sig, h0)
        Lg, plan, ws = check_against_oracle(a, b, sig, base_rows=h0)
        _base_rows_check(a, b, plan, ws, verts)


def test_many_short_anchor_rows():
    """Levels with many anchors and rows of at most 1024 weights run one
    anchor search per wave; 512 x 3000 with 16-row strips and tile 4 puts
    more than 3 x 256 anchors on levels 1-4.  Every level's rows for sampled
    vertices (anchors, their neighbours and tails) against the oracle."""
    r = np.random.default_rng(777)
    m, n = 512, 3000
    a = r.integers(0, 4, m).astype(np.uint8)
    b = r.integers(0, 4, n).astype(np.uint8)
    Lg, plan, ws = check_against_oracle(a, b, 4, base_rows=16, tile=4)
    verts = sorted(set(list(range(0, n + 1, 9)) + list(range(0, n + 1, 4)[::23]) + [1, 2, 3, n - 1, n]))
    for lv, cnt in enumerate(plan.levels()):
        if lv == 0 or lv > 4:
            continue
        for s_ in sorted({0, cnt // 2, cnt - 1}):
            D, row0 = plan.dist(lv, s_, ws)
            h = D.shape[1] - 1
            got = D[verts].cpu().numpy()
            want = oracle.dist_rows(a, row0, row0 + h, b, verts)
            bad = np.argwhere(got != want)
            assert bad.size == 0, "level %d strip %d: vertex %d weight %d got %d want %d" % (
                lv, s_, verts[bad[0][0]], bad[0][1], got[tuple(bad[0])], want[tuple(bad[0])])


def test_paper_grid_example():
    """Fig. 1 grid: rows tcaggatt, columns gatttatgcagg; breakouts of Section II-B-1."""
    a = np.frombuffer(b"tcaggatt", np.uint8) - ord("a")
    b = np.frombuffer(b"gatttatgcagg", np.uint8) - ord("a")
    Lg, wit, plan, ws = run_pair(a, b, 26, base_rows=16, tile=4, check_levels=True)
    assert Lg == 5
    top, _ = plan.dist(len(plan.levels()) - 1, 0, ws)
    top = top.cpu().numpy()
    assert list(top[0][:6]) == [0, 1, 2, 3, 4, 12]
    assert top[7][5] == 13
    assert bytes((a[wit[0]] + ord("a")).astype(np.uint8)) == b"tcagg"


def test_three_string_example_pairwise():
    a = np.frombuffer(b"abccb", np.uint8) - ord("a")
    b = np.frombuffer(b"abba", np.uint8) - ord("a")
    Lg, wit, _, _ = run_pair(a, b, 3, base_rows=16, tile=4)
    assert Lg == 3 and list(wit[0]) == [0, 1, 4] and list(wit[1]) == [0, 1, 2]


# ----------------------------------------------------------------- random shapes


def test_random_shapes_length_and_witness():
    r = np.random.default_rng(7)
    for case in range(40):
        sig = int(r.choice([1, 2, 4, 20, 256]))
        m = int(r.integers(0, 3000))
        n = int(r.integers(0, 3000))
        if case % 5 == 0:
            m = int(r.integers(0, 70))
        base_rows = int(r.choice([16, 32, 64, 128, 256, 512, 1024]))
        tile = int(r.choice([4, 8, 16, 32]))
        a = r.integers(0, sig, m).astype(np.uint8)
        if case % 3 == 0 and m > 0:
            b = synth.fit_length(r, synth.mutate(r, a, sig, 0.1, 0.05, 0.05), max(n, 1), sig)
        else:
            b = r.integers(0, sig, n).astype(np.uint8)
        say("random case", case, m, b.size, sig, base_rows, tile)
        check_against_oracle(a, b, sig, base_rows=base_rows, tile=tile)


def test_edge_cases():
    r = np.random.default_rng(9)
    x = r.integers(0, 4, 300).astype(np.uint8)
    cases = [
        (np.zeros(0, np.uint8), x, 4), (x, np.zeros(0, np.uint8), 4),
        (np.zeros(0, np.uint8), np.zeros(0, np.uint8), 4),
        (x[:1], x, 4), (x, x[:1], 4), (x[:1], x[:1], 4),
        (x, x, 4),                                            # LCS(x, x) = |x|
        (np.zeros(100, np.uint8), np.zeros(37, np.uint8), 1),  # unary alphabet
        (np.zeros(37, np.uint8), np.zeros(100, np.uint8), 1),
        (x, (x + 4).astype(np.uint8), 8),                     # disjoint alphabets
        (x[:64], x, 4), (x[:65], x, 4), (x[:63], x, 4),       # around one base strip
        (x, x[:64], 4), (x, x[:65], 4), (x, x[:63], 4),       # around one tile
    ]
    for a, b, sig in cases:
        say("edge", a.size, b.size, sig)
        Lg, _, _ = check_against_oracle(a, b, sig)
        if a is b or (a.size == b.size and np.array_equal(a, b)):
            assert Lg == a.size


def test_bad_symbol_reports_error():
    """A symbol outside the alphabet in either string is LCS_E_SYMBOL (row string:
    base strips; column string: the next-match scan), also with the orientation
    choice, which swaps the roles of the two strings."""
    good_a = np.array([0, 1, 2, 3, 1], np.uint8)
    good_b = np.array([0, 1, 2, 1], np.uint8)
    bad_a = good_a.copy()
    bad_a[3] = 9
    bad_b = good_b.copy()
    bad_b[2] = 4
    for a, b in ((bad_a, good_b), (good_a, bad_b), (bad_a, bad_b)):
        for orient in (False, True):
            plan = L.Plan(5, 4, 4, orient=orient)
            ws = L.alloc_workspace(plan.workspace_for(5, 4))
            plan.build(L.device_bytes(a), L.device_bytes(b), ws)
            with pytest.raises(L.LcsError) as e:
                plan.length()
            assert e.value.status == -5
            plan.close()
    plan = L.Plan(5, 4, 4)  # and a good pair in the same plan afterwards is fine
    ws = L.alloc_workspace(plan.workspace_for(5, 4))
    plan.build(L.device_bytes(good_a), L.device_bytes(good_b), ws)
    assert plan.length() == oracle.lcs_length(good_a, good_b)


def test_determinism_and_reuse():
    """Two builds into the same workspace give identical matrices; a plan is reusable."""
    import torch
    p = synth.pair_uniform(700, 900, 4, 31)
    plan = L.Plan(1000, 1000, 4, 16, 16)
    ws = L.alloc_workspace(plan.workspace_bytes)
    ad, bd = L.device_bytes(p.a), L.device_bytes(p.b)
    plan.build(ad, bd, ws)
    L1 = plan.length()
    top1 = plan.dist(len(plan.levels()) - 1, 0, ws)[0].clone()
    q = synth.pair_uniform(300, 200, 4, 32)          # something else in between
    plan.build(L.device_bytes(q.a), L.device_bytes(q.b), ws)
    assert plan.length() == oracle.lcs_length(q.a, q.b)
    plan.build(ad, bd, ws)
    assert plan.length() == L1 == oracle.lcs_length(p.a, p.b)
    top2 = plan.dist(len(plan.levels()) - 1, 0, ws)[0]
    assert torch.equal(top1, top2)


# ----------------------------------------------------------------- the named workloads


def _top_rows_check(a, b, plan, ws, verts):
    top, row0 = plan.dist(len(plan.levels()) - 1, 0, ws)
    assert row0 == 0
    got = top[list(verts)].cpu().numpy()
    want = oracle.dist_rows(a, 0, a.size, b, verts)
    assert np.array_equal(got[:, :], want)


def test_config_small_256():
    p = synth.config_small()
    say("pair 256x256")
    Lg, plan, ws = check_against_oracle(p.a, p.b, p.sigma, base_rows=64, check_levels=True)


def test_config_4096():
    p = synth.config_4096()
    say("pair 4096x4096")
    Lg, plan, ws = check_against_oracle(p.a, p.b, p.sigma, base_rows=64)
    # sampled rows of the top matrix (the oracle computes one row per dynamic program)
    _top_rows_check(p.a, p.b, plan, ws, [0, 1, 63, 64, 65, 2048, 4000, 4095, 4096])
    # sampled rows of every level's first and last strip; the top two levels
    # (the bracket shapes of 1024- and 2048-row child strips: 128- and 160-wide D_U
    # windows, cooperative pass 2) at vertices around tile boundaries and
    # spread over the row range
    rng = np.random.default_rng(4096)
    top_verts = sorted(set([1, 2, 15, 16, 17, 31, 32, 33, 63, 64, 65, 95, 2047, 2048, 2049, 4064, 4095]
                           + [int(v) for v in rng.integers(0, 4097, 24)]))
    nlev = len(plan.levels())
    for lv, cnt in enumerate(plan.levels()):
        for s in sorted({0, cnt - 1}):
            D, row0 = plan.dist(lv, s, ws)
            h = D.shape[1] - 1
            verts = [0, 777, 4033, 4096] + (top_verts if lv >= nlev - 2 else [])
            got = D[verts].cpu().numpy()
            want = oracle.dist_rows(p.a, row0, row0 + h, p.b, verts)
            bad = np.argwhere(got != want)
            assert bad.size == 0, "level %d strip %d vertex %d weight %d got %d want %d" % (
                lv, s, verts[bad[0][0]], bad[0][1], got[tuple(bad[0])], want[tuple(bad[0])])


def test_config_16384_mutated():
    p = synth.config_16384()
    say("pair 16384x16384 mutated, alphabet 20")
    Lg, plan, ws = check_against_oracle(p.a, p.b, p.sigma, base_rows=64)
    top, _ = plan.dist(len(plan.levels()) - 1, 0, ws)
    row = oracle.lcs_last_row(p.a, p.b)                 # C[m][k] for every k
    D0 = top[0].cpu().numpy()
    for k in range(0, p.b.size + 1, 97):
        assert int(np.sum(D0 <= k)) - 1 == row[k]
    _top_rows_check(p.a, p.b, plan, ws, [16300, 16383, 16384])


def test_wide_rows_across_16bit_limits():
    """Rows as wide as the 16-bit shapes allow and just beyond: the base strips
    keep their next-match window in 16-bit LDS entries while n + 2 <= 65535,
    and the bracketed combine keeps 16-bit state while n + 1 <= 65535; at
    n = 65535 and above both take their 32-bit forms.  Length, witness and
    sampled breakout rows of every level against the oracle."""
    r = np.random.default_rng(65535)
    m = 1000
    a = r.integers(0, 4, m).astype(np.uint8)
    for n in (65533, 65534, 65535, 70001):
        b = r.integers(0, 4, n).astype(np.uint8)
        b[n - 1500:n - 500] = a[r.permutation(m)]   # a shuffled copy of a near the end
        say("wide rows", m, n)
        Lg, plan, ws = check_against_oracle(a, b, 4, base_rows=64, tile=32)
        verts = [0, 1, 63, 64, 65, n // 2, n - 1600, n - 1000, n - 700, n - 65, n - 1, n]
        for lv, cnt in enumerate(plan.levels()):
            for s in sorted({0, cnt - 1}):
                D, row0 = plan.dist(lv, s, ws)
                h = D.shape[1] - 1
                got = D[verts].cpu().numpy()
                want = oracle.dist_rows(a, row0, row0 + h, b, verts)
                bad = np.argwhere(got != want)
                assert bad.size == 0, "n %d level %d strip %d vertex %d weight %d got %d want %d" % (
                    n, lv, s, verts[bad[0][0]], bad[0][1], got[tuple(bad[0])], want[tuple(bad[0])])


@pytest.mark.parametrize("m,n", [(20000, 3000), (20000, 10000), (17000, 25000)])
def test_tall_pairs_global_anchor_rows(m, n):
    """Row strings longer than 16384: the top combine merges child strips of
    16384 rows, whose anchor rows (2 * 16384 + 1 weights plus the D_U row) do
    not fit one work-group's LDS, so the anchor search keeps them in global
    memory; the three shapes reach its 1024-, 512- and 256-thread forms (at
    most one, three, or more anchor rows per compute unit).  Length, witness,
    sampled rows of the top matrix, and the top row against the textbook
    table's last row."""
    r = np.random.default_rng(m + n)
    a = r.integers(0, 4, m).astype(np.uint8)
    b = synth.fit_length(r, synth.mutate(r, a, 4, 0.1, 0.05, 0.05), n, 4) if n >= 10000 else \
        r.integers(0, 4, n).astype(np.uint8)
    say("tall pair", m, n)
    Lg, plan, ws = check_against_oracle(a, b, 4, base_rows=64, tile=32)
    levels = plan.levels()
    assert levels[-1] == 1 and levels[-2] == 2
    top, row0 = plan.dist(len(levels) - 1, 0, ws)
    D0 = top[0].cpu().numpy()
    row = oracle.lcs_last_row(a, b)
    for k in list(range(0, n + 1, 61)) + [n]:
        assert int(np.sum(D0 <= k)) - 1 == row[k], k
    verts = [1, 31, 32, 33, n // 2, n - 33, n - 1]
    got = top[verts].cpu().numpy()
    want = oracle.dist_rows(a, 0, m, b, verts)
    bad = np.argwhere(got != want)
    assert bad.size == 0, "vertex %d weight %d got %d want %d" % (
        verts[bad[0][0]], bad[0][1], got[tuple(bad[0])], want[tuple(bad[0])])
