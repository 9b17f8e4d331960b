"""CPU oracle for C = A B over F_3, F_5, F_7, GF(4), GF(8), F_9 -- TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check of the entry module and the CPU-baseline leg of the
benchmark may import this package.  The GPU library never uses it, and it shares no code
with the GPU library: the product is computed by the plain schoolbook loop in
``gfq_oracle.c``; the packed-plane encoder below is written from the element encodings
the paper fixes and from the packed layout documented in the library header, not from
the library's code.

Functions
---------
matmul(q, A, B)        schoolbook product of canonical uint8 matrices (C library).
encode_planes(q, X)    element -> bit-planes in the paper's encodings (Sections 4.1, 4.2, 4.3).
pack(q, X)             bit-planes laid out in the library's packed row format.
unpack(q, words, r, c) inverse of ``pack`` for canonical representatives.
packed_words(q, cols)  uint32 words per row of a packed matrix.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gfq_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
FIELDS = (3, 4, 5, 7, 8, 9)


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc (x86-64-v3 so the library runs on any recent host)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O3", "-march=x86-64-v3", "-fopenmp", "-fPIC", "-shared",
               "-Wall", "-Wextra", "-o", tmp, _SRC]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        lib.gfq_oracle_matmul.restype = ctypes.c_int
        lib.gfq_oracle_matmul.argtypes = [
            ctypes.c_int, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64,
            ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_int64,
            ctypes.c_void_p, ctypes.c_int64, ctypes.c_int]
        lib.gfq_oracle_max_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def max_threads() -> int:
    return _load().gfq_oracle_max_threads()


def planes(q: int) -> int:
    """Bit-planes per element: 2 for F_3 (unit, sign) and GF(4) (c0, c1); 3 for F_5, F_7
    and GF(8) (c0, c1, c2); 4 for F_9 (unit and sign of a0, then of a1)."""
    if q in (3, 4):
        return 2
    if q in (5, 7, 8):
        return 3
    if q == 9:
        return 4
    raise ValueError(f"unsupported field q={q}")


def matmul(q: int, A: np.ndarray, B: np.ndarray, threads: int = 0) -> np.ndarray:
    """C = A B over F_q (q = 4 means GF(4), q = 8 GF(8), q = 9 F_9 = F_3[i]/(i^2 + 1));
    A, B and C canonical uint8."""
    A = np.ascontiguousarray(A, dtype=np.uint8)
    B = np.ascontiguousarray(B, dtype=np.uint8)
    if A.ndim != 2 or B.ndim != 2 or A.shape[1] != B.shape[0]:
        raise ValueError(f"shape mismatch {A.shape} x {B.shape}")
    m, l = A.shape
    n = B.shape[1]
    C = np.zeros((m, n), dtype=np.uint8)
    rc = _load().gfq_oracle_matmul(q, m, l, n, A.ctypes.data, max(l, 1), B.ctypes.data,
                                   max(n, 1), C.ctypes.data, max(n, 1), int(threads))
    if rc != 0:
        raise ValueError(f"oracle rejected the problem (code {rc})")
    return C


def encode_planes(q: int, X: np.ndarray) -> list:
    """Return the list of 0/1 bit-planes of canonical elements X.

    F_3 (Section 4.1): 0 = (0,0), 1 = (1,0), -1 = (1,1) with the first bit x0 marking a
    unit and the second bit x1 the sign; the integer 2 stands for -1.
    F_5, F_7 (Section 4.2): the binary digits of the representative, plane d = bit d.
    GF(4) (Section 4.3, basis {1, x}): e = c0 + 2 c1, plane d = c_d.
    GF(8) (Section 4.3, power basis {1, x, x^2}): e = c0 + 2 c1 + 4 c2, plane d = c_d.
    F_9 (Section 4.3, F_3[i]/(i^2 + 1)): e = a0 + 3 a1; each coefficient in the F_3 code of
    Section 4.1, planes (unit a0, sign a0, unit a1, sign a1).
    """
    X = np.asarray(X, dtype=np.uint8)
    if q == 3:
        return [(X != 0).astype(np.uint8), (X == 2).astype(np.uint8)]
    if q == 9:
        return encode_planes(3, X % 3) + encode_planes(3, X // 3)
    return [((X >> d) & 1).astype(np.uint8) for d in range(planes(q))]


def decode_planes(q: int, bits: list) -> np.ndarray:
    """Inverse of encode_planes; for F_5/F_7 the representative is reduced mod q."""
    if q == 3:
        x0, x1 = bits
        return np.where(x0 == 0, 0, np.where(x1 == 0, 1, 2)).astype(np.uint8)
    if q == 9:
        return (decode_planes(3, bits[:2]) + 3 * decode_planes(3, bits[2:])).astype(np.uint8)
    v = np.zeros_like(bits[0], dtype=np.int64)
    for d, b in enumerate(bits):
        v |= b.astype(np.int64) << d
    if q in (5, 7):
        v %= q
    return v.astype(np.uint8)


def packed_words(q: int, cols: int) -> int:
    """uint32 words in one packed row: P planes of ceil(cols/128)*4 words each."""
    return planes(q) * (-(-cols // 128) * 4)


def pack(q: int, X: np.ndarray) -> np.ndarray:
    """Packed rows: row r holds plane 0, then plane 1, ... each of W = ceil(cols/128)*4
    little-endian uint32 words; element j is bit (j mod 32) of word (j div 32); pad bits 0."""
    X = np.asarray(X, dtype=np.uint8)
    rows, cols = X.shape
    W = -(-cols // 128) * 4
    out = np.zeros((rows, planes(q), W * 32), dtype=np.uint8)
    for d, bits in enumerate(encode_planes(q, X)):
        out[:, d, :cols] = bits
    packed = np.packbits(out, axis=2, bitorder="little")          # bytes, LSB first
    return packed.view("<u4").reshape(rows, planes(q) * W).copy()


def unpack(q: int, words: np.ndarray, rows: int, cols: int) -> np.ndarray:
    W = -(-cols // 128) * 4
    w = np.asarray(words).reshape(rows, planes(q), W).astype("<u4")
    bits = np.unpackbits(w.view(np.uint8), axis=2, bitorder="little")[:, :, :cols]
    return decode_planes(q, [bits[:, d, :] for d in range(planes(q))])
