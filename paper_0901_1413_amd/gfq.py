"""ctypes binding of libgfq.so (C ABI in include/gfq.h).

Argument marshalling only: torch tensors provide device memory, torch's current stream
is handed to the library before every call, and every computation runs in the HIP
kernels of the library.  A missing library raises; nothing falls back to another path.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgfq.so")

GFQ_OK = 0
FIELDS = (3, 4, 5, 7, 8, 9)


class GfqError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(msg)
        self.status = status


class Config(ctypes.Structure):
    _fields_ = [("k", ctypes.c_int), ("rows", ctypes.c_int), ("split", ctypes.c_int),
                ("variant", ctypes.c_int)]

    def as_dict(self):
        return {"k": self.k, "rows": self.rows, "split": self.split, "variant": self.variant}


class Problem(ctypes.Structure):
    _fields_ = [("q", ctypes.c_int), ("m", ctypes.c_int64), ("l", ctypes.c_int64),
                ("n", ctypes.c_int64), ("A", ctypes.c_void_p), ("B", ctypes.c_void_p),
                ("C", ctypes.c_void_p)]


class ServerOpts(ctypes.Structure):
    _fields_ = [("budget_bytes", ctypes.c_size_t), ("slots", ctypes.c_int), ("max_batch", ctypes.c_int),
                ("max_items", ctypes.c_int), ("mode", ctypes.c_int), ("watchdog_s", ctypes.c_double)]


class Request(ctypes.Structure):
    _fields_ = [("q", ctypes.c_int), ("m", ctypes.c_int64), ("l", ctypes.c_int64), ("n", ctypes.c_int64),
                ("A", ctypes.c_void_p), ("lda", ctypes.c_int64), ("B", ctypes.c_void_p), ("ldb", ctypes.c_int64),
                ("C", ctypes.c_void_p), ("ldc", ctypes.c_int64), ("flags", ctypes.c_int),
                ("tag", ctypes.c_uint64), ("not_before_us", ctypes.c_double), ("C_host", ctypes.c_void_p)]


class Completion(ctypes.Structure):
    _fields_ = [("tag", ctypes.c_uint64), ("status", ctypes.c_int), ("batch_size", ctypes.c_int),
                ("arrival_us", ctypes.c_double), ("launch_us", ctypes.c_double), ("done_us", ctypes.c_double)]


class ServerStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("completed", ctypes.c_int64), ("batches", ctypes.c_int64),
                ("queued", ctypes.c_int64), ("max_batch_seen", ctypes.c_int64), ("arena_in_use", ctypes.c_size_t),
                ("arena_held", ctypes.c_size_t), ("arena_peak_in_use", ctypes.c_size_t)]


_lib = None
_I64 = ctypes.c_int64
_VP = ctypes.c_void_p
_SIGS = {
    "gfq_packed_bytes": (ctypes.c_size_t, [ctypes.c_int, _I64, _I64]),
    "gfq_pack": (ctypes.c_int, [ctypes.c_int, _I64, _I64, _VP, _I64, _VP]),
    "gfq_unpack": (ctypes.c_int, [ctypes.c_int, _I64, _I64, _VP, _VP, _I64]),
    "gfq_matmul": (ctypes.c_int, [ctypes.c_int, _I64, _I64, _I64, _VP, _VP, _VP]),
    "gfq_matmul_config": (ctypes.c_int, [ctypes.c_int, _I64, _I64, _I64, _VP, _VP, _VP,
                                         ctypes.POINTER(Config)]),
    "gfq_matmul_noalloc": (ctypes.c_int, [ctypes.c_int, _I64, _I64, _I64, _VP, _VP, _VP,
                                          ctypes.POINTER(Config)]),
    "gfq_choose_config": (ctypes.c_int, [ctypes.c_int, _I64, _I64, _I64, ctypes.POINTER(Config)]),
    "gfq_matmul_sw": (ctypes.c_int, [ctypes.c_int, _I64, _I64, _I64, _VP, _VP, _VP, ctypes.c_int,
                                     ctypes.POINTER(Config)]),
    "gfq_matmul_batched": (ctypes.c_int, [ctypes.c_int, ctypes.POINTER(Problem)]),
    "gfq_batch_create": (ctypes.c_int, [ctypes.c_int, ctypes.POINTER(Problem), ctypes.POINTER(_VP)]),
    "gfq_batch_launch": (ctypes.c_int, [_VP]),
    "gfq_batch_times": (ctypes.c_int, [_VP, ctypes.POINTER(ctypes.c_double)]),
    "gfq_batch_destroy": (ctypes.c_int, [_VP]),
    "gfq_batch_slab_widths": (ctypes.c_int, [_VP, ctypes.POINTER(ctypes.c_int)]),
    "gfq_batch_slices": (ctypes.c_int, [_VP, ctypes.POINTER(ctypes.c_int)]),
    "gfq_batch_launch_persistent": (ctypes.c_int, [_VP]),
    "gfq_tune": (ctypes.c_int, [ctypes.c_int, _I64, _I64, _I64, ctypes.c_int, ctypes.POINTER(Config)]),
    "gfq_tune_lookup": (ctypes.c_int, [ctypes.c_int, _I64, _I64, _I64, ctypes.c_int, ctypes.POINTER(Config)]),
    "gfq_tune_save": (ctypes.c_int, [ctypes.c_char_p]),
    "gfq_tune_load": (ctypes.c_int, [ctypes.c_char_p]),
    "gfq_tune_clear": (ctypes.c_int, []),
    "gfq_server_create": (ctypes.c_int, [ctypes.POINTER(ServerOpts), ctypes.POINTER(_VP)]),
    "gfq_server_submit": (ctypes.c_int, [_VP, ctypes.POINTER(Request), ctypes.c_int]),
    "gfq_server_poll": (ctypes.c_int, [_VP, ctypes.POINTER(Completion), ctypes.c_int, ctypes.POINTER(ctypes.c_int),
                                       ctypes.c_double]),
    "gfq_server_now_us": (ctypes.c_double, [_VP]),
    "gfq_server_stats_read": (ctypes.c_int, [_VP, ctypes.POINTER(ServerStats)]),
    "gfq_server_destroy": (ctypes.c_int, [_VP]),
    "gfq_set_stream": (ctypes.c_int, [_VP]),
    "gfq_sync": (ctypes.c_int, []),
    "gfq_set_timing": (ctypes.c_int, [ctypes.c_int]),
    "gfq_timing_read": (ctypes.c_int, [ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int),
                                       ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int)]),
    "gfq_probe_valu": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, _VP, ctypes.POINTER(ctypes.c_double),
                                      ctypes.POINTER(ctypes.c_float)]),
    "gfq_probe_lds": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, _VP, ctypes.POINTER(ctypes.c_double),
                                     ctypes.POINTER(ctypes.c_float)]),
    "gfq_probe_copy": (ctypes.c_int, [_VP, _VP, ctypes.c_size_t, ctypes.POINTER(ctypes.c_float)]),
    "gfq_strerror": (ctypes.c_char_p, [ctypes.c_int]),
    "gfq_last_hip_error": (ctypes.c_char_p, []),
}


def load():
    """Load libgfq.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def lib():
    return load()


def _check(status: int, what: str):
    if status != GFQ_OK:
        l = load()
        msg = l.gfq_strerror(status).decode()
        hip = l.gfq_last_hip_error().decode()
        raise GfqError(status, f"{what}: {msg}" + (f" ({hip})" if hip else ""))


def _bind_stream():
    import torch
    load().gfq_set_stream(ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))


def planes(q: int) -> int:
    return 2 if q in (3, 4) else (4 if q == 9 else 3)


def packed_bytes(q: int, rows: int, cols: int) -> int:
    return int(load().gfq_packed_bytes(q, rows, cols))


def empty_packed(q: int, rows: int, cols: int, device="cuda"):
    import torch
    return torch.empty(max(packed_bytes(q, rows, cols), 16), dtype=torch.uint8, device=device)


def pack(q: int, X, out=None):
    """Pack a device uint8 matrix X (rows x cols, row-major, any leading dimension)."""
    import torch
    assert X.dtype == torch.uint8 and X.dim() == 2 and X.is_cuda
    rows, cols = X.shape
    if X.stride(1) != 1:
        X = X.contiguous()
    if out is None:
        out = empty_packed(q, rows, cols, X.device)
    _bind_stream()
    _check(load().gfq_pack(q, rows, cols, _VP(X.data_ptr()), max(X.stride(0), cols), _VP(out.data_ptr())), "gfq_pack")
    return out


def unpack(q: int, Pk, rows: int, cols: int, out=None):
    import torch
    if out is None:
        out = torch.empty((rows, cols), dtype=torch.uint8, device=Pk.device)
    assert out.dim() == 2 and out.stride(1) == 1 and out.dtype == torch.uint8
    _bind_stream()
    _check(load().gfq_unpack(q, rows, cols, _VP(Pk.data_ptr()), _VP(out.data_ptr()), max(out.stride(0), cols)),
           "gfq_unpack")
    return out


def choose_config(q: int, m: int, l: int, n: int) -> dict:
    c = Config()
    _check(load().gfq_choose_config(q, m, l, n, ctypes.byref(c)), "gfq_choose_config")
    return c.as_dict()


VARIANT_ROWWISE, VARIANT_KARATSUBA = 0, 1


def matmul(q: int, A, B, m: int, l: int, n: int, out=None, k: int = 0, rows: int = 0, split: int = 0,
           variant=None):
    """C = A B on packed device operands; returns the packed product.  k, rows, split and
    variant (GF(4): VARIANT_ROWWISE or VARIANT_KARATSUBA) override the chosen configuration."""
    if out is None:
        out = empty_packed(q, m, n, A.device)
    _bind_stream()
    if k or rows or split or variant is not None:
        c = Config()
        _check(load().gfq_choose_config(q, m, l, n, ctypes.byref(c)), "gfq_choose_config")
        if k:
            c.k = k
        if rows:
            c.rows = rows
        if split:
            c.split = split
        if variant is not None:
            c.variant = variant
        _check(load().gfq_matmul_config(q, m, l, n, _VP(A.data_ptr()), _VP(B.data_ptr()), _VP(out.data_ptr()),
                                        ctypes.byref(c)), "gfq_matmul_config")
    else:
        _check(load().gfq_matmul(q, m, l, n, _VP(A.data_ptr()), _VP(B.data_ptr()), _VP(out.data_ptr())),
               "gfq_matmul")
    return out


NOALLOC_SCRATCH_BYTES = 64 << 20   # GFQ_NOALLOC_SCRATCH_BYTES


def matmul_noalloc(q: int, A, B, m: int, l: int, n: int, out, k: int = 0, rows: int = 0, split: int = 0,
                   variant=None):
    """gfq_matmul_noalloc: C = A B into the caller's packed `out` with no device allocation
    (split partial products in the library's fixed per-device array).  k, rows, split and
    variant give an explicit configuration (the others from gfq_choose_config); none of
    them: the library's choice with the split fitted to the array."""
    _bind_stream()
    cfg = None
    if k or rows or split or variant is not None:
        c = Config()
        _check(load().gfq_choose_config(q, m, l, n, ctypes.byref(c)), "gfq_choose_config")
        if k:
            c.k = k
        if rows:
            c.rows = rows
        if split:
            c.split = split
        if variant is not None:
            c.variant = variant
        cfg = ctypes.byref(c)
    _check(load().gfq_matmul_noalloc(q, m, l, n, _VP(A.data_ptr()), _VP(B.data_ptr()), _VP(out.data_ptr()), cfg),
           "gfq_matmul_noalloc")
    return out


SW_MAX_LEVELS = 4
SW_AUTO = -1          # levels from the tuner's cache (tune_sw), else 0
TUNE_SW = 2


def matmul_sw(q: int, A, B, m: int, l: int, n: int, levels: int, out=None, k: int = 0, rows: int = 0,
              variant=None, split: int = 0):
    """C = A B by `levels` levels of Strassen-Winograd over the Four-Russians product
    (gfq_matmul_sw); k, rows, variant and split override the leaf configuration (split
    defaults to 1 when any of them is given)."""
    if out is None:
        out = empty_packed(q, m, n, A.device)
    _bind_stream()
    cp = None
    if k or rows or variant is not None or split:
        c = Config()
        _check(load().gfq_choose_config(q, m, l, n, ctypes.byref(c)), "gfq_choose_config")
        if k:
            c.k = k
        if rows:
            c.rows = rows
        if variant is not None:
            c.variant = variant
        c.split = split or 1
        cp = ctypes.byref(c)
    _check(load().gfq_matmul_sw(q, m, l, n, _VP(A.data_ptr()), _VP(B.data_ptr()), _VP(out.data_ptr()), levels, cp),
           "gfq_matmul_sw")
    return out


def matmul_batched(problems: Sequence[tuple]):
    """problems: [(q, m, l, n, A, B, C)] with packed device tensors."""
    arr = (Problem * len(problems))()
    for i, (q, m, l, n, A, B, C) in enumerate(problems):
        arr[i] = Problem(q, m, l, n, A.data_ptr(), B.data_ptr(), C.data_ptr())
    _bind_stream()
    _check(load().gfq_matmul_batched(len(problems), arr), "gfq_matmul_batched")


class Batch:
    """A prepared batch of products (gfq_batch_create): launch it any number of times."""

    def __init__(self, problems: Sequence[tuple]):
        self.count = len(problems)
        arr = (Problem * max(1, len(problems)))()
        for i, (q, m, l, n, A, B, C) in enumerate(problems):
            arr[i] = Problem(q, m, l, n, A.data_ptr(), B.data_ptr(), C.data_ptr())
        self._keep = [(A, B, C) for (_, _, _, _, A, B, C) in problems]
        h = _VP()
        _bind_stream()
        _check(load().gfq_batch_create(len(problems), arr, ctypes.byref(h)), "gfq_batch_create")
        self.handle = h

    def launch(self):
        _bind_stream()
        _check(load().gfq_batch_launch(self.handle), "gfq_batch_launch")

    def launch_persistent(self):
        """The same items drained by persistent workgroups through a device queue head."""
        _bind_stream()
        _check(load().gfq_batch_launch_persistent(self.handle), "gfq_batch_launch_persistent")

    def times_us(self):
        """Per-product completion time of the last launch, microseconds from its start."""
        out = (ctypes.c_double * max(1, self.count))()
        _bind_stream()
        _check(load().gfq_batch_times(self.handle, out), "gfq_batch_times")
        return list(out)[: self.count]

    def slab_widths(self):
        """The slab width k the batch gives each product."""
        out = (ctypes.c_int * max(1, self.count))()
        _check(load().gfq_batch_slab_widths(self.handle, out), "gfq_batch_slab_widths")
        return list(out)[: self.count]

    def slices(self):
        """The number of slab slices the batch cut each product into (1: whole tiles)."""
        out = (ctypes.c_int * max(1, self.count))()
        _check(load().gfq_batch_slices(self.handle, out), "gfq_batch_slices")
        return list(out)[: self.count]

    def destroy(self):
        if self.handle:
            _check(load().gfq_batch_destroy(self.handle), "gfq_batch_destroy")
            self.handle = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


TUNE_BATCH = 1


def tune(q: int, m: int, l: int, n: int, batch: bool = False) -> dict:
    """Time candidate configurations for this shape's size class and cache the fastest."""
    c = Config()
    _bind_stream()
    _check(load().gfq_tune(q, m, l, n, TUNE_BATCH if batch else 0, ctypes.byref(c)), "gfq_tune")
    return c.as_dict()


def tune_lookup(q: int, m: int, l: int, n: int, batch: bool = False):
    c = Config()
    st = load().gfq_tune_lookup(q, m, l, n, TUNE_BATCH if batch else 0, ctypes.byref(c))
    return c.as_dict() if st == GFQ_OK else None


def tune_sw(q: int, m: int, l: int, n: int) -> int:
    """Time Strassen-Winograd levels 0 .. SW_MAX_LEVELS - 1 for this size class; cache and
    return the fastest (matmul_sw(..., SW_AUTO) then uses it)."""
    c = Config()
    _bind_stream()
    _check(load().gfq_tune(q, m, l, n, TUNE_SW, ctypes.byref(c)), "gfq_tune")
    return c.k


def tune_sw_lookup(q: int, m: int, l: int, n: int):
    c = Config()
    st = load().gfq_tune_lookup(q, m, l, n, TUNE_SW, ctypes.byref(c))
    return c.k if st == GFQ_OK else None


def tune_save(path: str):
    _check(load().gfq_tune_save(path.encode()), "gfq_tune_save")


def tune_load(path: str):
    _check(load().gfq_tune_load(path.encode()), "gfq_tune_load")


def tune_clear():
    load().gfq_tune_clear()


def set_timing(on: bool):
    load().gfq_set_timing(1 if on else 0)


def timing_read() -> dict:
    """Summed kernel milliseconds and launch counts since the last read (needs set_timing)."""
    pm, rm = ctypes.c_double(), ctypes.c_double()
    pc, rc = ctypes.c_int(), ctypes.c_int()
    _check(load().gfq_timing_read(ctypes.byref(pm), ctypes.byref(pc), ctypes.byref(rm), ctypes.byref(rc)),
           "gfq_timing_read")
    return {"product_ms": pm.value, "product_launches": pc.value, "reduce_ms": rm.value,
            "reduce_launches": rc.value}


def probe(kind: str, blocks: int = 2048, iters: int = 4096, nbytes: int = 1 << 30) -> dict:
    """Machine-rate microbenchmarks (gfq_probe_*): kind "valu" (lane operations per second of
    v_bitop3_b32), "lds" (128-bit LDS read bytes per second), "copy" (HBM bytes per second of
    a device copy, reads plus writes)."""
    import torch
    _bind_stream()
    ms = ctypes.c_float()
    amount = ctypes.c_double()
    if kind in ("valu", "lds"):
        sink = torch.empty(blocks * 512, dtype=torch.int32, device="cuda")
        fn = load().gfq_probe_valu if kind == "valu" else load().gfq_probe_lds
        _check(fn(blocks, iters, _VP(sink.data_ptr()), ctypes.byref(amount), ctypes.byref(ms)), f"gfq_probe_{kind}")
        return {"amount": amount.value, "ms": ms.value, "rate": amount.value / (ms.value * 1e-3)}
    if kind == "copy":
        src = torch.ones(nbytes, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        _check(load().gfq_probe_copy(_VP(src.data_ptr()), _VP(dst.data_ptr()), nbytes, ctypes.byref(ms)),
               "gfq_probe_copy")
        return {"amount": 2.0 * nbytes, "ms": ms.value, "rate": 2.0 * nbytes / (ms.value * 1e-3)}
    raise ValueError(kind)


def sync():
    _bind_stream()
    _check(load().gfq_sync(), "gfq_sync")


def matmul_unpacked(q: int, A_u8, B_u8, **kw):
    """Convenience: pack both operands, multiply, unpack (all on the GPU)."""
    m, l = A_u8.shape
    n = B_u8.shape[1]
    Ap = pack(q, A_u8)
    Bp = pack(q, B_u8)
    Cp = matmul(q, Ap, Bp, m, l, n, **kw)
    return unpack(q, Cp, m, n)


REQ_A_PACKED, REQ_B_PACKED, REQ_C_PACKED = 1, 2, 4


def _operand(X, rows: int, cols: int, packed: bool):
    """(pointer, leading dimension) of a device operand: a 2-D uint8 tensor (rows may be
    strided, columns contiguous) or, when packed, any tensor holding the packed matrix."""
    if X is None:
        return None, 0
    if packed:
        return X.data_ptr(), 0
    assert X.dim() == 2 and tuple(X.shape) == (rows, cols) and (cols <= 1 or X.stride(1) == 1), \
        (tuple(X.shape), (rows, cols))
    return X.data_ptr(), max(X.stride(0), cols)


class Server:
    """Continuous-batching product server (gfq_server_*).  submit() queues requests and
    keeps their tensors alive until poll() has returned their completions."""

    def __init__(self, budget_bytes: int = 0, slots: int = 0, max_batch: int = 0, max_items: int = 0,
                 serial: bool = False, watchdog_s: float = 0.0):
        o = ServerOpts(budget_bytes, slots, max_batch, max_items, 1 if serial else 0, watchdog_s)
        h = _VP()
        _check(load().gfq_server_create(ctypes.byref(o), ctypes.byref(h)), "gfq_server_create")
        self.handle = h
        self._keep = {}

    @staticmethod
    def request(q, m, l, n, A, B, C, tag, not_before_us=0.0, flags=0, C_host=None) -> Request:
        """C_host: optional (pinned) host tensor that receives a copy of the product before
        the completion is reported."""
        a, lda = _operand(A, m, l, flags & REQ_A_PACKED)
        b, ldb = _operand(B, l, n, flags & REQ_B_PACKED)
        c, ldc = _operand(C, m, n, flags & REQ_C_PACKED)
        h = C_host.data_ptr() if C_host is not None else None
        return Request(q, m, l, n, a, lda, b, ldb, c, ldc, flags, tag, not_before_us, h)

    def submit(self, reqs: Sequence[Request], keep: Sequence = ()):
        """Queue requests (Request structures); keep[i] (optional) is held until request i
        completes."""
        arr = (Request * len(reqs))(*reqs)
        _check(load().gfq_server_submit(self.handle, arr, len(reqs)), "gfq_server_submit")
        for i, r in enumerate(reqs):
            if i < len(keep):
                self._keep[r.tag] = keep[i]

    def poll(self, max_count: int = 4096, timeout_us: float = 0.0):
        buf = (Completion * max_count)()
        got = ctypes.c_int()
        _check(load().gfq_server_poll(self.handle, buf, max_count, ctypes.byref(got), timeout_us), "gfq_server_poll")
        out = []
        for i in range(got.value):
            c = buf[i]
            self._keep.pop(c.tag, None)
            out.append({"tag": c.tag, "status": c.status, "batch_size": c.batch_size,
                        "arrival_us": c.arrival_us, "launch_us": c.launch_us, "done_us": c.done_us})
        return out

    def wait_all(self, count: int, timeout_s: float = 60.0):
        """Poll until count completions have arrived (raises on timeout)."""
        import time
        out, t_end = [], time.monotonic() + timeout_s
        while len(out) < count:
            if time.monotonic() > t_end:
                raise TimeoutError(f"{len(out)} of {count} completions after {timeout_s} s")
            out += self.poll(timeout_us=20000.0)
        return out

    def now_us(self) -> float:
        return load().gfq_server_now_us(self.handle)

    def stats(self) -> dict:
        st = ServerStats()
        _check(load().gfq_server_stats_read(self.handle, ctypes.byref(st)), "gfq_server_stats_read")
        return {f: getattr(st, f) for f, _ in ServerStats._fields_}

    def destroy(self):
        if self.handle:
            _check(load().gfq_server_destroy(self.handle), "gfq_server_destroy")
            self.handle = None
            self._keep.clear()

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass
