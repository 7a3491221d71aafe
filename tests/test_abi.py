"""The C ABI on the CPU: the library loads, exports every declared symbol, and
validates arguments before touching the device."""
import ctypes
import math
import os
import re

import pytest

from paper_2309_09072_amd import lcs as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    hdr = open(os.path.join(ROOT, "include", "lcs.h")).read()
    hdr = re.sub(r"/\*.*?\*/", "", hdr, flags=re.S)
    return sorted(set(re.findall(r"\b(lcs_[a-z_]+)\s*\(", hdr)))


def test_library_exports_every_declared_symbol():
    lib = L.load()
    names = declared_symbols()
    assert len(names) >= 20
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, "declared in include/lcs.h but not exported: %s" % missing


def test_status_strings():
    lib = L.load()
    for s in range(0, -11, -1):
        txt = lib.lcs_status_string(s).decode()
        assert txt.startswith("LCS_"), txt
    assert lib.lcs_status_string(-999)


@pytest.mark.parametrize("kw", [
    dict(alphabet=0), dict(alphabet=257), dict(base_rows=8), dict(base_rows=48), dict(base_rows=96),
    dict(base_rows=2048),
    dict(tile=3), dict(tile=128), dict(tile=24), dict(max_m=-1), dict(max_n=-5),
])
def test_plan_rejects_bad_descriptors(kw):
    args = dict(max_m=100, max_n=100, alphabet=4, base_rows=0, tile=0)
    args.update(kw)
    with pytest.raises(L.LcsError) as e:
        L.Plan(args["max_m"], args["max_n"], args["alphabet"], args["base_rows"], args["tile"])
    assert e.value.status == -1


def test_plan_rejects_int32_overflow():
    with pytest.raises(L.LcsError) as e:
        L.Plan(70000, 70000, 4)
    assert e.value.status == -2


def test_workspace_sizes():
    p = L.Plan(16384, 16384, 20)
    assert p.base_rows == 1024  # the default for this many rows
    # all levels kept: about 4 (n+2) m (1 + log2(m / base_rows)) bytes
    est = 4 * 16386 * 16384 * (1 + math.log2(16384 / p.base_rows))
    assert est < p.workspace_bytes < 1.05 * est
    for m, n, h in ((100, 100, 64), (4095, 9000, 64), (4096, 4096, 256), (4096, 8191, 256),
                    (4096, 8192, 512), (8191, 100, 256), (8191, 9000, 512), (8192, 100, 1024)):
        assert L.Plan(m, n, 4).base_rows == h, (m, n)
    # oriented: rows = the shorter string, columns = the longer
    assert L.Plan(20000, 3000, 4, orient=True).base_rows == 64
    assert L.Plan(20000, 5000, 4, orient=True).base_rows == 512
    assert L.Plan(20000, 9000, 4, orient=True).base_rows == 1024
    assert L.Plan(5000, 6000, 4, orient=True).base_rows == 256
    assert L.Plan(100, 100, 4, 32).base_rows == 32
    assert p.workspace_for(16384, 16384) == p.workspace_bytes
    assert p.workspace_for(100, 100) < p.workspace_for(200, 100) < p.workspace_for(200, 200)
    assert p.workspace_for(0, 0) > 0
    with pytest.raises(L.LcsError) as e:
        p.workspace_for(16385, 10)
    assert e.value.status == -2


def test_calls_validate_before_device_work():
    lib = L.load()
    p = L.Plan(100, 100, 4)
    h = p._h
    null = ctypes.c_void_p(0)
    fake = ctypes.c_void_p(0x10000)            # never dereferenced: validation fails first
    # no workspace
    assert lib.lcs_dist_build(h, fake, 10, fake, 10, null, 1 << 20, null) == -1
    # sizes above the plan
    assert lib.lcs_dist_build(h, fake, 101, fake, 10, fake, 1 << 30, null) == -2
    # workspace too small
    assert lib.lcs_dist_build(h, fake, 10, fake, 10, fake, 16, null) == -3
    # misaligned workspace
    assert lib.lcs_dist_build(h, fake, 10, fake, 10, ctypes.c_void_p(0x10004), 1 << 30, null) == -1
    # null inputs with positive lengths
    assert lib.lcs_dist_build(h, null, 10, fake, 10, fake, 1 << 30, null) == -1
    # length / trace / views before any successful build
    out = ctypes.c_int32()
    assert lib.lcs_length(h, ctypes.byref(out), null) == -7
    assert lib.lcs_trace(h, fake, fake, 100, ctypes.byref(out), null) == -7
    assert lib.lcs_plan_levels(h, ctypes.byref(out), None) == -7
    # null plan / null outputs
    assert lib.lcs_length(null, ctypes.byref(out), null) == -1
    assert lib.lcs_plan_workspace(null, 1, 1, None) == -1


def test_orient_flag_and_workspace_bound():
    from paper_2309_09072_amd import lcs
    p = lcs.Plan(1000, 300, 4, 16, 8, orient=True)
    for m, n in [(1000, 300), (1000, 1), (301, 300), (300, 300), (5, 300), (0, 0), (1000, 0)]:
        assert p.workspace_for(m, n) <= p.workspace_bytes, (m, n)
    # oriented: layout of the transposed problem (fewer levels when m > n)
    q = lcs.Plan(1000, 300, 4, 16, 8)
    assert p.workspace_for(1000, 300) < q.workspace_for(1000, 300)
    assert p.workspace_for(200, 300) == q.workspace_for(200, 300)
    p.close()
    q.close()
    desc = lcs.PlanDesc(10, 10, 4, 16, 8, 4)   # unknown flag bit
    import ctypes
    h, ws = ctypes.c_void_p(), ctypes.c_size_t()
    assert lcs.load().lcs_plan(ctypes.byref(desc), ctypes.byref(h), ctypes.byref(ws)) == -1


def test_noalloc_build_rejects_pairs_beyond_its_array():
    """The no-allocation build refuses a pair whose workspace exceeds the
    library's own device array, before any device work (null strings are never
    read)."""
    lib = L.load()
    p = L.Plan(4096, 4096, 4)
    assert p.workspace_for(4096, 4096) > L.NOALLOC_WORKSPACE_BYTES
    st = lib.lcs_dist_build_noalloc(p._h, None, 4096, None, 4096, None)
    assert st == -3
    assert p.workspace_for(1450, 1450) <= L.NOALLOC_WORKSPACE_BYTES
