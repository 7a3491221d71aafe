"""Thin ctypes binding of ``liblcs.so`` (the C ABI declared in include/lcs.h).

Argument marshalling only: torch tensors on the ROCm device are passed as raw
device pointers, streams as ``hipStream_t`` handles.  Every step of the method
runs in the library's HIP kernels; there is no CPU fallback, and loading fails
loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "liblcs.so")

LCS_OK = 0
STATUS = {
    0: "LCS_OK", -1: "LCS_E_INVAL", -2: "LCS_E_TOO_BIG", -3: "LCS_E_WORKSPACE", -4: "LCS_E_HIP",
    -5: "LCS_E_SYMBOL", -6: "LCS_E_CAPACITY", -7: "LCS_E_STATE", -8: "LCS_E_NOMEM",
    -9: "LCS_E_BUDGET", -10: "LCS_E_AGAIN",
}
BATCH_PERSISTENT, BATCH_PER_PAIR, BATCH_GRAPH, BATCH_STAGED, BATCH_PAIR_QUEUE = 0, 1, 2, 4, 8
NOALLOC_WORKSPACE_BYTES = 64 << 20  # LCS_NOALLOC_WORKSPACE_BYTES of include/lcs.h


class LcsError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__("%s: %s" % (where, _lib_status(status)))


class PlanDesc(ctypes.Structure):
    _fields_ = [("max_m", ctypes.c_int32), ("max_n", ctypes.c_int32), ("alphabet", ctypes.c_int32),
                ("base_rows", ctypes.c_int32), ("tile", ctypes.c_int32), ("flags", ctypes.c_uint32)]


class PairDesc(ctypes.Structure):
    _fields_ = [("a_off", ctypes.c_int64), ("b_off", ctypes.c_int64), ("m", ctypes.c_int32),
                ("n", ctypes.c_int32)]


class BatchDesc(ctypes.Structure):
    _fields_ = [("max_pairs", ctypes.c_int32), ("max_len", ctypes.c_int32),
                ("alphabet", ctypes.c_int32), ("base_rows", ctypes.c_int32),
                ("tile", ctypes.c_int32), ("slots", ctypes.c_int32), ("flags", ctypes.c_uint32)]


class ServerDesc(ctypes.Structure):
    _fields_ = [("max_len", ctypes.c_int32), ("alphabet", ctypes.c_int32),
                ("base_rows", ctypes.c_int32), ("tile", ctypes.c_int32),
                ("slots", ctypes.c_int32), ("max_queue", ctypes.c_int32),
                ("flags", ctypes.c_uint32)]


class PhaseTime(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("level", ctypes.c_int32), ("ms", ctypes.c_float),
                ("bytes", ctypes.c_int64)]


PHASES = {0: "nextmatch", 1: "base", 2: "anchor", 3: "bracket", 4: "length", 5: "trace_split",
          6: "trace_leaf"}
PLAN_PROFILE = 1
PLAN_ORIENT = 2


class Result(ctypes.Structure):
    _fields_ = [("tag", ctypes.c_int64), ("status", ctypes.c_int32), ("length", ctypes.c_int32),
                ("t_submit", ctypes.c_double), ("t_admit", ctypes.c_double),
                ("t_done", ctypes.c_double)]


_lib = None

_P = ctypes.c_void_p
_I32 = ctypes.c_int32
_I64 = ctypes.c_int64
_U32 = ctypes.c_uint32
_SZ = ctypes.c_size_t
_PI32 = ctypes.POINTER(ctypes.c_int32)
_PSZ = ctypes.POINTER(ctypes.c_size_t)

PROTOTYPES = {
    "lcs_status_string": (ctypes.c_char_p, [_I32]),
    "lcs_plan": (_I32, [ctypes.POINTER(PlanDesc), ctypes.POINTER(_P), _PSZ]),
    "lcs_plan_workspace": (_I32, [_P, _I32, _I32, _PSZ]),
    "lcs_plan_describe": (_I32, [_P, ctypes.POINTER(PlanDesc)]),
    "lcs_plan_destroy": (_I32, [_P]),
    "lcs_dist_build": (_I32, [_P, _P, _I32, _P, _I32, _P, _SZ, _P]),
    "lcs_dist_build_noalloc": (_I32, [_P, _P, _I32, _P, _I32, _P]),
    "lcs_length": (_I32, [_P, _PI32, _P]),
    "lcs_length_device": (_I32, [_P, _P, _P]),
    "lcs_trace": (_I32, [_P, _P, _P, _I32, _PI32, _P]),
    "lcs_trace_device": (_I32, [_P, _P, _P, _I32, _P, _P]),
    "lcs_plan_profile": (_I32, [_P, _P, _I32, _PI32]),
    "lcs_semilocal": (_I32, [_P, _P, _P, _I32, _P, _P]),
    "lcs_path": (_I32, [_P, _P, _P, _P, _P, _P, _P]),
    "lcs_plan_levels": (_I32, [_P, _PI32, _PI32]),
    "lcs_dist_view": (_I32, [_P, _I32, _I32, ctypes.POINTER(_P), _PI32, _PI32, _PI32]),
    "lcs_batch_plan": (_I32, [ctypes.POINTER(BatchDesc), ctypes.POINTER(_P), _PSZ]),
    "lcs_batch_destroy": (_I32, [_P]),
    "lcs_batch_status": (_I32, [_P, _P, _P]),
    "lcs_batch_selftest": (_I32, [ctypes.POINTER(BatchDesc), _P, _I32]),
    "lcs_batch_submit": (_I32, [_P, _P, _I32, _P, _I64, _P, _P, _P, _I64, _P, _SZ, _U32, _P]),
    "lcs_server_open": (_I32, [ctypes.POINTER(ServerDesc), _P, _SZ, ctypes.POINTER(_P)]),
    "lcs_server_footprint": (_I32, [_P, _I32, _I32, _PSZ]),
    "lcs_server_submit": (_I32, [_P, _I64, _P, _I32, _P, _I32, _I32, _P, _P]),
    "lcs_server_poll": (_I32, [_P, _P, _I32, _PI32]),
    "lcs_server_pending": (_I32, [_P, _PI32, _PI32, _PSZ, _PSZ]),
    "lcs_server_close": (_I32, [_P]),
    "lcs_server_simulate": (_I32, [_SZ, _I32, _I32, _P, _P, _P, _P, _P, _PSZ]),
}


def load():
    """Load liblcs.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("liblcs.so not found at %s; build it with "
                              "`python -c 'import __graft_entry__ as g; g.build()'`" % LIB_PATH)
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in PROTOTYPES.items():
            fn = getattr(lib, name, None)
            if fn is None:
                continue
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def _lib_status(s: int) -> str:
    try:
        return load().lcs_status_string(int(s)).decode()
    except Exception:
        return STATUS.get(int(s), str(s))


def check(status: int, where: str) -> None:
    if status != LCS_OK:
        raise LcsError(status, where)


def _torch():
    import torch
    return torch


def stream_handle(stream=None) -> ctypes.c_void_p:
    """hipStream_t of a torch stream (default: the current stream)."""
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(int(s.cuda_stream))


def _dptr(t) -> ctypes.c_void_p:
    if t is None:
        return ctypes.c_void_p(0)
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    return ctypes.c_void_p(int(t.data_ptr()))


def device_bytes(x, device="cuda"):
    """uint8 device tensor from a numpy array / bytes / str."""
    torch = _torch()
    if isinstance(x, str):
        x = x.encode("latin-1")
    arr = np.frombuffer(bytes(x), dtype=np.uint8) if isinstance(x, (bytes, bytearray)) else np.asarray(x, dtype=np.uint8)
    t = torch.from_numpy(np.ascontiguousarray(arr).copy())
    return t.to(device) if t.numel() else torch.zeros(0, dtype=torch.uint8, device=device)


def alloc_workspace(nbytes: int, device="cuda"):
    """A device byte buffer usable as a workspace (torch allocations are 512-byte aligned)."""
    torch = _torch()
    t = torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)
    if t.data_ptr() % 256:
        raise RuntimeError("workspace allocation is not 256-byte aligned")
    return t


class Plan:
    """One planned strip recursion (lcs_plan); reusable for any m <= max_m, n <= max_n."""

    def __init__(self, max_m: int, max_n: int, alphabet: int, base_rows: int = 0, tile: int = 0,
                 profile: bool = False, orient: bool = False):
        lib = load()
        self.desc = PlanDesc(int(max_m), int(max_n), int(alphabet), int(base_rows), int(tile),
                             (PLAN_PROFILE if profile else 0) | (PLAN_ORIENT if orient else 0))
        h = ctypes.c_void_p()
        ws = ctypes.c_size_t()
        check(lib.lcs_plan(ctypes.byref(self.desc), ctypes.byref(h), ctypes.byref(ws)), "lcs_plan")
        self._h = h
        self.workspace_bytes = int(ws.value)
        self._keep = None
        res = PlanDesc()
        check(lib.lcs_plan_describe(h, ctypes.byref(res)), "lcs_plan_describe")
        self.base_rows = int(res.base_rows)  # as resolved by the library
        self.tile = int(res.tile)

    def workspace_for(self, m: int, n: int) -> int:
        ws = ctypes.c_size_t()
        check(load().lcs_plan_workspace(self._h, int(m), int(n), ctypes.byref(ws)), "lcs_plan_workspace")
        return int(ws.value)

    def build(self, a, b, ws, stream=None) -> None:
        """lcs_dist_build on device tensors a (m bytes), b (n bytes), ws (workspace)."""
        self._keep = (a, b, ws)  # the library keeps raw pointers until the next build
        check(load().lcs_dist_build(self._h, _dptr(a), int(a.numel()), _dptr(b), int(b.numel()),
                                    _dptr(ws), int(ws.numel()), stream_handle(stream)),
              "lcs_dist_build")

    def build_noalloc(self, a, b, stream=None) -> None:
        """lcs_dist_build_noalloc: the build on the library's own device array
        (no workspace argument, nothing allocated)."""
        self._keep = (a, b)
        check(load().lcs_dist_build_noalloc(self._h, _dptr(a), int(a.numel()), _dptr(b),
                                            int(b.numel()), stream_handle(stream)),
              "lcs_dist_build_noalloc")

    def length(self, stream=None) -> int:
        out = ctypes.c_int32()
        check(load().lcs_length(self._h, ctypes.byref(out), stream_handle(stream)), "lcs_length")
        return int(out.value)

    def path(self, a_idx, b_idx, length_dev, m: int, stream=None):
        """(col_in, col_out) device int32[m + 1]: the canonical path row by row
        (lcs_path) from a device witness of trace_device."""
        torch = _torch()
        dev = length_dev.device
        cin = torch.empty(m + 1, dtype=torch.int32, device=dev)
        cout = torch.empty(m + 1, dtype=torch.int32, device=dev)
        check(load().lcs_path(self._h, _dptr(a_idx), _dptr(b_idx), _dptr(length_dev), _dptr(cin),
                              _dptr(cout), stream_handle(stream)), "lcs_path")
        return cin, cout

    def semilocal(self, qi, qk, out=None, stream=None):
        """LCS(a, b[i:k]) for device int32 query tensors qi, qk (lcs_semilocal);
        -1 for a query outside 0 <= i <= k <= n."""
        torch = _torch()
        if out is None:
            out = torch.empty(int(qi.numel()), dtype=torch.int32, device=qi.device)
        check(load().lcs_semilocal(self._h, _dptr(qi), _dptr(qk), int(qi.numel()), _dptr(out),
                                   stream_handle(stream)), "lcs_semilocal")
        return out

    def length_device(self, out, stream=None) -> None:
        check(load().lcs_length_device(self._h, _dptr(out), stream_handle(stream)), "lcs_length_device")

    def trace(self, a_idx, b_idx, stream=None) -> int:
        out = ctypes.c_int32()
        cap = min(int(a_idx.numel()), int(b_idx.numel()))
        check(load().lcs_trace(self._h, _dptr(a_idx), _dptr(b_idx), cap, ctypes.byref(out),
                               stream_handle(stream)), "lcs_trace")
        return int(out.value)

    def trace_device(self, a_idx, b_idx, length_dev, stream=None) -> None:
        """Enqueue the witness trace without synchronising; L goes to length_dev (int32[1])."""
        cap = min(int(a_idx.numel()), int(b_idx.numel()))
        check(load().lcs_trace_device(self._h, _dptr(a_idx), _dptr(b_idx), cap, _dptr(length_dev),
                                      stream_handle(stream)), "lcs_trace_device")

    def profile(self):
        """Per-launch records since the last read: list of (phase, level, ms, bytes)."""
        lib = load()
        cnt = ctypes.c_int32()
        check(lib.lcs_plan_profile(self._h, None, 0, ctypes.byref(cnt)), "lcs_plan_profile")
        arr = (PhaseTime * max(cnt.value, 1))()
        check(lib.lcs_plan_profile(self._h, ctypes.cast(arr, ctypes.c_void_p), cnt.value,
                                   ctypes.byref(cnt)), "lcs_plan_profile")
        return [(PHASES.get(arr[i].kind, str(arr[i].kind)), int(arr[i].level), float(arr[i].ms),
                 int(arr[i].bytes)) for i in range(cnt.value)]

    def levels(self):
        nl = ctypes.c_int32()
        check(load().lcs_plan_levels(self._h, ctypes.byref(nl), None), "lcs_plan_levels")
        arr = (ctypes.c_int32 * max(nl.value, 1))()
        check(load().lcs_plan_levels(self._h, ctypes.byref(nl), arr), "lcs_plan_levels")
        return [int(arr[i]) for i in range(nl.value)]

    def dist(self, level: int, strip: int, ws):
        """(matrix view (n+2) x (h+1) int32 on the device, first grid row of the strip)."""
        ptr = ctypes.c_void_p()
        rows, cols, row0 = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        check(load().lcs_dist_view(self._h, int(level), int(strip), ctypes.byref(ptr),
                                   ctypes.byref(rows), ctypes.byref(cols), ctypes.byref(row0)),
              "lcs_dist_view")
        off = int(ptr.value) - int(ws.data_ptr())
        nbytes = rows.value * cols.value * 4
        view = ws[off:off + nbytes].view(_torch().int32).view(rows.value, cols.value)
        return view, int(row0.value)

    def close(self) -> None:
        if getattr(self, "_h", None):
            load().lcs_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def lcs(a, b, alphabet: int, base_rows: int = 0, tile: int = 0, witness: bool = True,
        device="cuda", stream=None, orient: bool = False):
    """LCS of two symbol strings on the GPU: (L, a_idx, b_idx) as numpy arrays."""
    torch = _torch()
    ad, bd = device_bytes(a, device), device_bytes(b, device)
    m, n = int(ad.numel()), int(bd.numel())
    plan = Plan(m, n, alphabet, base_rows, tile, orient=orient)
    try:
        ws = alloc_workspace(plan.workspace_for(m, n), device)
        plan.build(ad, bd, ws, stream)
        if not witness:
            return plan.length(stream), None, None
        cap = max(1, min(m, n))
        ai = torch.empty(cap, dtype=torch.int32, device=device)
        bi = torch.empty(cap, dtype=torch.int32, device=device)
        L = plan.trace(ai, bi, stream)
        return L, ai[:L].cpu().numpy(), bi[:L].cpu().numpy()
    finally:
        plan.close()


class Batch:
    """A planned batch (lcs_batch_plan): many pairs per submit, one persistent launch."""

    def __init__(self, max_pairs: int, max_len: int, alphabet: int, base_rows: int = 0,
                 tile: int = 0, slots: int = 0):
        lib = load()
        self.desc = BatchDesc(int(max_pairs), int(max_len), int(alphabet), int(base_rows),
                              int(tile), int(slots), 0)
        h = ctypes.c_void_p()
        ws = ctypes.c_size_t()
        check(lib.lcs_batch_plan(ctypes.byref(self.desc), ctypes.byref(h), ctypes.byref(ws)),
              "lcs_batch_plan")
        self._h = h
        self.workspace_bytes = int(ws.value)

    @staticmethod
    def witness_offsets(m, n):
        mn = np.minimum(np.asarray(m, np.int64), np.asarray(n, np.int64))
        off = np.zeros(mn.size + 1, np.int64)
        np.cumsum(mn, out=off[1:])
        return off

    def submit(self, symbols, a_off, b_off, m, n, ws, lengths, a_idx, b_idx,
               mode: int = BATCH_PERSISTENT, stream=None) -> None:
        """Enqueue every pair; symbols is a device uint8 tensor, the rest host arrays /
        device output tensors (lengths int32[count], a_idx/b_idx int32[sum min(m,n)])."""
        count = int(len(m))
        descs = (PairDesc * max(count, 1))()
        for p in range(count):
            descs[p].a_off, descs[p].b_off = int(a_off[p]), int(b_off[p])
            descs[p].m, descs[p].n = int(m[p]), int(n[p])
        self._keep = (symbols, ws, lengths, a_idx, b_idx, descs)
        cap = 0 if a_idx is None else min(int(a_idx.numel()), int(b_idx.numel()))
        check(load().lcs_batch_submit(self._h, ctypes.cast(descs, ctypes.c_void_p), count,
                                      _dptr(symbols), int(symbols.numel()), _dptr(lengths),
                                      _dptr(a_idx), _dptr(b_idx), cap, _dptr(ws), int(ws.numel()),
                                      int(mode), stream_handle(stream)), "lcs_batch_submit")

    def status(self, ws, stream=None) -> None:
        check(load().lcs_batch_status(self._h, _dptr(ws), stream_handle(stream)), "lcs_batch_status")

    def close(self) -> None:
        if getattr(self, "_h", None):
            load().lcs_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def batch_selftest(m, n, alphabet: int, base_rows: int = 0, tile: int = 0, slots: int = 0,
                   max_len: int = 0) -> int:
    """Host simulation of the persistent schedule (lcs_batch_selftest); returns the status."""
    count = len(m)
    max_len = max_len or int(max(max(m, default=1), max(n, default=1), 1))
    desc = BatchDesc(max(count, 1), max_len, int(alphabet), int(base_rows), int(tile), int(slots), 0)
    descs = (PairDesc * max(count, 1))()
    off = 0
    for p in range(count):
        descs[p].a_off, descs[p].b_off, descs[p].m, descs[p].n = off, off + m[p], int(m[p]), int(n[p])
        off += m[p] + n[p]
    return int(load().lcs_batch_selftest(ctypes.byref(desc), ctypes.cast(descs, ctypes.c_void_p), count))


def run_batch(batch, mode: int = BATCH_PERSISTENT, base_rows: int = 0, tile: int = 0,
              slots: int = 0, device="cuda", planned=None, ws=None):
    """Lengths and witnesses of every pair of a synth.Batch on the GPU (numpy results)."""
    torch = _torch()
    b = planned or Batch(batch.count, int(max(batch.m.max(initial=1), batch.n.max(initial=1))),
                         batch.sigma, base_rows, tile, slots)
    if ws is None:
        ws = alloc_workspace(b.workspace_bytes, device)
    sym = device_bytes(batch.symbols, device) if batch.symbols.size else torch.zeros(1, dtype=torch.uint8, device=device)
    off = Batch.witness_offsets(batch.m, batch.n)
    lengths = torch.full((batch.count,), -99, dtype=torch.int32, device=device)
    ai = torch.full((max(int(off[-1]), 1),), -1, dtype=torch.int32, device=device)
    bi = torch.full((max(int(off[-1]), 1),), -1, dtype=torch.int32, device=device)
    b.submit(sym, batch.a_off, batch.b_off, batch.m, batch.n, ws, lengths, ai, bi, mode)
    torch.cuda.synchronize()
    if not (mode & (BATCH_PER_PAIR | BATCH_STAGED | BATCH_PAIR_QUEUE)):
        b.status(ws)
    return lengths.cpu().numpy(), ai.cpu().numpy(), bi.cpu().numpy(), off



class Server:
    """Continuous-batching server (lcs_server_*) over a device arena tensor."""

    def __init__(self, arena, max_len: int, alphabet: int, slots: int = 8, max_queue: int = 1 << 16,
                 base_rows: int = 0, tile: int = 0):
        self.desc = ServerDesc(int(max_len), int(alphabet), int(base_rows), int(tile), int(slots),
                               int(max_queue), 0)
        h = ctypes.c_void_p()
        self.arena = arena
        check(load().lcs_server_open(ctypes.byref(self.desc), _dptr(arena), int(arena.numel()),
                                     ctypes.byref(h)), "lcs_server_open")
        self._h = h
        self._buf = (Result * 256)()
        self._outs = {}

    def footprint(self, m: int, n: int) -> int:
        out = ctypes.c_size_t()
        check(load().lcs_server_footprint(self._h, int(m), int(n), ctypes.byref(out)), "lcs_server_footprint")
        return int(out.value)

    def submit(self, tag: int, a, b, alphabet: int, a_idx=None, b_idx=None) -> int:
        """Returns the status (LCS_E_AGAIN / LCS_E_BUDGET are not raised)."""
        a = np.ascontiguousarray(a, np.uint8)
        b = np.ascontiguousarray(b, np.uint8)
        self._outs[int(tag)] = (a_idx, b_idx)
        st = load().lcs_server_submit(self._h, int(tag), a.ctypes.data_as(ctypes.c_void_p), a.size,
                                      b.ctypes.data_as(ctypes.c_void_p), b.size, int(alphabet),
                                      _dptr(a_idx), _dptr(b_idx))
        if st not in (LCS_OK, -9, -10):
            check(st, "lcs_server_submit")
        if st != LCS_OK:
            self._outs.pop(int(tag), None)
        return int(st)

    def poll(self):
        """List of (tag, status, length, t_submit, t_admit, t_done) finished since the last poll."""
        out = []
        while True:
            cnt = ctypes.c_int32()
            check(load().lcs_server_poll(self._h, ctypes.cast(self._buf, ctypes.c_void_p), 256,
                                         ctypes.byref(cnt)), "lcs_server_poll")
            for i in range(cnt.value):
                r = self._buf[i]
                out.append((int(r.tag), int(r.status), int(r.length), r.t_submit, r.t_admit, r.t_done))
                self._outs.pop(int(r.tag), None)
            if cnt.value < 256:
                return out

    def pending(self):
        r, w = ctypes.c_int32(), ctypes.c_int32()
        u, p = ctypes.c_size_t(), ctypes.c_size_t()
        check(load().lcs_server_pending(self._h, ctypes.byref(r), ctypes.byref(w), ctypes.byref(u),
                                        ctypes.byref(p)), "lcs_server_pending")
        return int(r.value), int(w.value), int(u.value), int(p.value)

    def close(self) -> None:
        if getattr(self, "_h", None):
            load().lcs_server_close(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def server_simulate(arena_bytes: int, slots: int, arrival, footprint, service):
    """Admission policy under a virtual clock: (t_admit, t_done, peak) numpy arrays."""
    arrival = np.ascontiguousarray(arrival, np.float64)
    foot = np.ascontiguousarray(footprint, np.uint64)
    service = np.ascontiguousarray(service, np.float64)
    ta = np.zeros_like(arrival)
    td = np.zeros_like(arrival)
    peak = ctypes.c_size_t()
    st = load().lcs_server_simulate(int(arena_bytes), int(slots), int(arrival.size),
                                    arrival.ctypes.data_as(ctypes.c_void_p),
                                    foot.ctypes.data_as(ctypes.c_void_p),
                                    service.ctypes.data_as(ctypes.c_void_p),
                                    ta.ctypes.data_as(ctypes.c_void_p),
                                    td.ctypes.data_as(ctypes.c_void_p), ctypes.byref(peak))
    check(st, "lcs_server_simulate")
    return ta, td, int(peak.value)
