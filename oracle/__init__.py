"""CPU oracle for the LCS hot path (arXiv 2309.09072) -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The product library never loads it, and
it shares no code with the HIP path: the C functions live in ``lcs_oracle.c``
and are reached through ``ctypes`` here.

Functions and the passage each one follows:

* ``lcs_length``     -- textbook O(mn) dynamic program (Section I).
* ``lcs_last_row``   -- last row of that dynamic program.
* ``lcs_witness``    -- the same table plus a LEFT > DIAG > UP walk back from
  (m, n): the optimal path that enters every row as far left as possible
  (the cross vertices of Section II-C taken leftmost; the tie rule of Alg. 2).
* ``path_rows``      -- every vertex of that canonical path, row by row: the
  first and last column it visits on each grid row (Section II-E).
* ``dist_rows``      -- the breakout matrix D_G by its definition
  (Section II-B-1), one fresh dynamic program per vertex.
* ``base_row``       -- the two-row base case D_{G_h} by the steps of
  Section II-B-3 (positions, gaps, prefix sum, unreachable tail).
* ``combine``        -- the combine equation of Section II-B-1 by brute force
  over every admissible split.
* ``brute``          -- subsequence enumeration for strings of length <= 12.
* ``paper_search``   -- Alg. 1 (column minima by divide and conquer) and Alg. 2
  (parallel prefix minimum with index) in the paper's order.

Every function here is pinned by ``tests/test_oracle_*.py`` against values the
paper prints, closed forms, invariants and brute force.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lcs_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile ``lcs_oracle.c`` into ``liboracle.so`` with gcc (plain C, -O2)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-shared", "-fPIC", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


def _bind(path: str):
    lib = ctypes.CDLL(path)
    i64, p = ctypes.c_int64, ctypes.c_void_p
    lib.oracle_lcs_length.restype = i64
    lib.oracle_lcs_length.argtypes = [p, i64, p, i64]
    lib.oracle_lcs_last_row.restype = ctypes.c_int
    lib.oracle_lcs_last_row.argtypes = [p, i64, p, i64, p]
    lib.oracle_lcs_witness.restype = i64
    lib.oracle_lcs_witness.argtypes = [p, i64, p, i64, p, p]
    lib.oracle_path_rows.restype = i64
    lib.oracle_path_rows.argtypes = [p, i64, p, i64, p, p]
    lib.oracle_dist_rows.restype = ctypes.c_int
    lib.oracle_dist_rows.argtypes = [p, i64, i64, p, i64, p, i64, p]
    lib.oracle_base_row.restype = i64
    lib.oracle_base_row.argtypes = [ctypes.c_uint8, p, i64, p]
    lib.oracle_combine.restype = ctypes.c_int
    lib.oracle_combine.argtypes = [p, i64, p, i64, i64, p, p]
    return lib


def _load():
    global _lib
    if _lib is None:
        _lib = _bind(build())
    return _lib


def _u8(x) -> np.ndarray:
    if isinstance(x, (bytes, bytearray)):
        return np.frombuffer(bytes(x), dtype=np.uint8).copy()
    if isinstance(x, str):
        return np.frombuffer(x.encode("latin-1"), dtype=np.uint8).copy()
    return np.ascontiguousarray(np.asarray(x, dtype=np.uint8))


def _ptr(arr: np.ndarray):
    return arr.ctypes.data_as(ctypes.c_void_p)


def lcs_length(a, b, lib=None) -> int:
    """LCS length by the textbook dynamic program (Section I)."""
    a, b = _u8(a), _u8(b)
    r = (lib or _load()).oracle_lcs_length(_ptr(a), a.size, _ptr(b), b.size)
    if r < 0:
        raise MemoryError("oracle_lcs_length")
    return int(r)


def lcs_last_row(a, b, lib=None) -> np.ndarray:
    """row[c] = LCS(a, b[:c]) for c = 0..len(b)."""
    a, b = _u8(a), _u8(b)
    out = np.zeros(b.size + 1, dtype=np.int32)
    if (lib or _load()).oracle_lcs_last_row(_ptr(a), a.size, _ptr(b), b.size, _ptr(out)) != 0:
        raise MemoryError("oracle_lcs_last_row")
    return out


def lcs_witness(a, b, lib=None):
    """(L, a_idx, b_idx): the canonical (leftmost) optimal alignment."""
    a, b = _u8(a), _u8(b)
    cap = max(1, min(a.size, b.size))
    ai = np.zeros(cap, dtype=np.int32)
    bi = np.zeros(cap, dtype=np.int32)
    L = (lib or _load()).oracle_lcs_witness(_ptr(a), a.size, _ptr(b), b.size, _ptr(ai), _ptr(bi))
    if L < 0:
        raise MemoryError("oracle_lcs_witness: table does not fit in host memory")
    return int(L), ai[:L].copy(), bi[:L].copy()


def path_rows(a, b, lib=None):
    """(col_in, col_out), int32[m + 1] each: on grid row r the canonical path
    (the one lcs_witness's walk follows) enters at column col_in[r] and leaves
    at col_out[r] (Section II-E: the vertices between the cross vertices)."""
    a, b = _u8(a), _u8(b)
    cin = np.zeros(a.size + 1, dtype=np.int32)
    cout = np.zeros(a.size + 1, dtype=np.int32)
    if (lib or _load()).oracle_path_rows(_ptr(a), a.size, _ptr(b), b.size, _ptr(cin), _ptr(cout)) < 0:
        raise MemoryError("oracle_path_rows: table does not fit in host memory")
    return cin, cout


def dist_rows(a, r0: int, r1: int, b, verts=None, lib=None) -> np.ndarray:
    """Breakout matrix rows D(i, 0..h) of the strip a[r0:r1] for vertices ``verts``.

    Default: every vertex 0..n.  Entries above n mean "unreachable" (value n+1).
    """
    a, b = _u8(a), _u8(b)
    n = b.size
    if verts is None:
        verts = np.arange(n + 1, dtype=np.int32)
    verts = np.ascontiguousarray(np.asarray(verts, dtype=np.int32))
    h = r1 - r0
    out = np.zeros((verts.size, h + 1), dtype=np.int32)
    rc = (lib or _load()).oracle_dist_rows(_ptr(a), r0, r1, _ptr(b), n, _ptr(verts), verts.size, _ptr(out))
    if rc != 0:
        raise ValueError("oracle_dist_rows: bad arguments")
    return out


def base_row(ah: int, b, lib=None) -> np.ndarray:
    """First breakouts of every top vertex of the two-row grid for symbol ``ah``."""
    b = _u8(b)
    out = np.zeros(b.size + 1, dtype=np.int32)
    r = (lib or _load()).oracle_base_row(int(ah), _ptr(b), b.size, _ptr(out))
    if r < 0:
        raise MemoryError("oracle_base_row")
    return out


def combine(DU: np.ndarray, DL: np.ndarray, n: int, with_argk: bool = False, lib=None):
    """The combine equation by brute force; DU is (n+1)x(hU+1), DL is (n+1)x(hL+1)."""
    DU = np.ascontiguousarray(DU, dtype=np.int32)
    DL = np.ascontiguousarray(DL, dtype=np.int32)
    assert DU.shape[0] == n + 1 and DL.shape[0] == n + 1
    hU, hL = DU.shape[1] - 1, DL.shape[1] - 1
    DG = np.zeros((n + 1, hU + hL + 1), dtype=np.int32)
    K = np.zeros_like(DG) if with_argk else None
    (lib or _load()).oracle_combine(_ptr(DU), hU, _ptr(DL), hL, n, _ptr(DG),
                           _ptr(K) if with_argk else None)
    return (DG, K) if with_argk else DG
