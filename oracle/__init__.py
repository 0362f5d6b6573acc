"""The oracle: a plain scalar CPU base64 codec written from the paper.

TEST INFRASTRUCTURE. Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package. The GPU codec
neither imports nor links it, and it imports nothing from the GPU codec.

What it computes (Muła & Lemire, arXiv 1704.00605):

* ``encode``: Algorithm 1 (Section 2) with the map B of Table 1, or the
  base64url variant (Section 2: 62 -> '-', 63 -> '_').
* ``decode``: Algorithm 2 (Section 2) with A the inverse of B, plus the strict
  readings R1-R5 stated at the top of ``b64_oracle.c`` ('=' only as the last
  one or two characters of a length divisible by 4; length not divisible by 4
  is an error at offset n; the smallest offending index is reported).
* ``decode_strict``: Appendix A's extra checks on the final quad.
* ``encode_nopad`` / ``decode_nopad``: Section 2's remark that padding may be
  omitted when the size is known.
* ``strip_ws`` / ``decode_ws``: Appendix B's removal of space, LF and CR.

Pins: every function here is checked by ``tests/test_oracle.py`` against the
paper's worked examples, Tables 1/4/5/6, closed forms and brute force.
"""
import ctypes
import os

import numpy as np

from . import build as _build

STD = 0
URL = 1

_lib = None


def lib():
    """Load (building first if absent) the oracle shared library."""
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        L = ctypes.CDLL(_build.LIB)
        i64, p, i32 = ctypes.c_int64, ctypes.c_void_p, ctypes.c_int
        pi64 = ctypes.POINTER(ctypes.c_int64)
        sig = {
            "oracle_symbol": (i32, [i32, i32]),
            "oracle_value": (i32, [i32, i32]),
            "oracle_encoded_len": (i64, [i64]),
            "oracle_decoded_max": (i64, [i64]),
            "oracle_encode": (i64, [p, i64, p, i32]),
            "oracle_decode": (i64, [p, i64, p, i32, pi64]),
            "oracle_decode_strict": (i64, [p, i64, p, i32, pi64]),
            "oracle_encode_nopad": (i64, [p, i64, p, i32]),
            "oracle_decode_nopad": (i64, [p, i64, p, i32, pi64]),
            "oracle_strip_ws": (i64, [p, i64, p, p]),
            "oracle_decode_ws": (i64, [p, i64, p, i32, pi64]),
            "oracle_encode_batch": (None, [p, p, i64, p, p, p, p]),
            "oracle_decode_batch": (None, [p, p, i64, p, p, p, p, p]),
            "oracle_encode_batch_mt": (None, [p, p, i64, p, p, p, p, i32]),
            "oracle_decode_batch_mt": (None, [p, p, i64, p, p, p, p, p, i32]),
            "oracle_encode_gather_mt": (None, [p, p, p, i64, p, p, p, p, i32]),
            "oracle_decode_gather_mt": (None, [p, p, p, i64, p, p, p, p, p, i32]),
            "oracle_encode_mt": (i64, [p, i64, p, i32, i32]),
            "oracle_decode_mt": (i64, [p, i64, p, i32, i32, pi64]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _u8(x):
    if isinstance(x, (bytes, bytearray, memoryview)):
        return np.frombuffer(bytes(x), dtype=np.uint8)
    a = np.ascontiguousarray(x)
    if a.dtype != np.uint8:
        raise TypeError("expected uint8 data")
    return a


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a.size else None


def symbol(v, alphabet=STD):
    """B(v) as an int (Table 1), -1 outside [0, 64)."""
    return lib().oracle_symbol(alphabet, v)


def value(ch, alphabet=STD):
    """A(ch): the 6-bit value of byte ``ch``, or -1 if it is not a symbol."""
    return lib().oracle_value(alphabet, ch)


def encoded_len(n):
    return lib().oracle_encoded_len(n)


def decoded_max(m):
    return lib().oracle_decoded_max(m)


def encode(data, alphabet=STD, threads=1):
    """Algorithm 1. Returns the encoded characters as a uint8 array."""
    s = _u8(data)
    out = np.empty(max(encoded_len(s.size), 1), dtype=np.uint8)
    if threads > 1:
        n = lib().oracle_encode_mt(_ptr(s), s.size, _ptr(out), alphabet, threads)
    else:
        n = lib().oracle_encode(_ptr(s), s.size, _ptr(out), alphabet)
    return out[:n]


def _dec(fn, data, alphabet, extra=()):
    c = _u8(data)
    out = np.empty(max(decoded_max(c.size) + 3, 1), dtype=np.uint8)
    err = ctypes.c_int64(-1)
    n = fn(_ptr(c), c.size, _ptr(out), alphabet, *extra, ctypes.byref(err))
    return (n, err.value, out[:n] if n >= 0 else None)


def decode(data, alphabet=STD, threads=1):
    """Validating decode: returns ``(length | -1, err_off | -1, bytes | None)``."""
    if threads > 1:
        return _dec(lib().oracle_decode_mt, data, alphabet, (threads,))
    return _dec(lib().oracle_decode, data, alphabet)


def decode_strict(data, alphabet=STD):
    """Decode plus Appendix A's final-quad checks."""
    return _dec(lib().oracle_decode_strict, data, alphabet)


def encode_nopad(data, alphabet=STD):
    s = _u8(data)
    out = np.empty(max(encoded_len(s.size), 1), dtype=np.uint8)
    n = lib().oracle_encode_nopad(_ptr(s), s.size, _ptr(out), alphabet)
    return out[:n]


def decode_nopad(data, alphabet=STD):
    return _dec(lib().oracle_decode_nopad, data, alphabet)


def strip_ws(data):
    """Appendix B: drop space, LF, CR. Returns (kept bytes, original indexes)."""
    a = _u8(data)
    out = np.empty(max(a.size, 1), dtype=np.uint8)
    pos = np.empty(max(a.size, 1), dtype=np.int64)
    n = lib().oracle_strip_ws(_ptr(a), a.size, _ptr(out), _ptr(pos))
    return out[:n], pos[:n]


def decode_ws(data, alphabet=STD):
    """Whitespace-tolerant decode; error offsets in original coordinates."""
    return _dec(lib().oracle_decode_ws, data, alphabet)


def encode_batch(src, in_off, flags=None, threads=1):
    """Plain loop over messages (split over ``threads`` host threads by
    contiguous message ranges). Returns (dst, out_off, out_len)."""
    src = _u8(src)
    in_off = np.ascontiguousarray(in_off, dtype=np.int64)
    N = in_off.size - 1
    lens = np.diff(in_off)
    out_off = np.zeros(N + 1, dtype=np.int64)
    np.cumsum(4 * ((lens + 2) // 3), out=out_off[1:])
    dst = np.zeros(max(int(out_off[-1]), 1), dtype=np.uint8)
    out_len = np.empty(max(N, 1), dtype=np.int64)
    fl = None if flags is None else np.ascontiguousarray(flags, dtype=np.uint8)
    if threads > 1:
        lib().oracle_encode_batch_mt(_ptr(src), _ptr(in_off), N, _ptr(dst), _ptr(out_off),
                                     None if fl is None else _ptr(fl), _ptr(out_len), int(threads))
    else:
        lib().oracle_encode_batch(_ptr(src), _ptr(in_off), N, _ptr(dst), _ptr(out_off),
                                  None if fl is None else _ptr(fl), _ptr(out_len))
    return dst[: out_off[-1]], out_off, out_len[:N]


def decode_batch(src, in_off, flags=None, threads=1):
    """Plain loop over messages (split over ``threads`` host threads by
    contiguous message ranges). Returns (dst, out_off, out_len, err_off);
    out_off holds capacity slots of 3 * floor(len / 4) bytes."""
    src = _u8(src)
    in_off = np.ascontiguousarray(in_off, dtype=np.int64)
    N = in_off.size - 1
    lens = np.diff(in_off)
    out_off = np.zeros(N + 1, dtype=np.int64)
    np.cumsum(3 * (lens // 4), out=out_off[1:])
    dst = np.zeros(max(int(out_off[-1]) + 3, 1), dtype=np.uint8)
    out_len = np.empty(max(N, 1), dtype=np.int64)
    err = np.empty(max(N, 1), dtype=np.int64)
    fl = None if flags is None else np.ascontiguousarray(flags, dtype=np.uint8)
    if threads > 1:
        lib().oracle_decode_batch_mt(_ptr(src), _ptr(in_off), N, _ptr(dst), _ptr(out_off),
                                     None if fl is None else _ptr(fl), _ptr(out_len), _ptr(err),
                                     int(threads))
    else:
        lib().oracle_decode_batch(_ptr(src), _ptr(in_off), N, _ptr(dst), _ptr(out_off),
                                  None if fl is None else _ptr(fl), _ptr(out_len), _ptr(err))
    return dst[: out_off[-1]], out_off, out_len[:N], err[:N]


def encode_gather(src, in_begin, in_len, out_off, dst, flags=None, threads=1):
    """Message i is src[in_begin[i], in_begin[i] + in_len[i]); its characters
    are written to dst[out_off[i]:] (caller-sized host array). Returns the
    per-message lengths."""
    src = _u8(src)
    ib = np.ascontiguousarray(in_begin, dtype=np.int64)
    il = np.ascontiguousarray(in_len, dtype=np.int64)
    oo = np.ascontiguousarray(out_off, dtype=np.int64)
    N = ib.size
    if il.size != N or oo.size < N or np.any(il < 0) or np.any(ib < 0) or np.any(ib + il > src.size) \
            or np.any(oo + 4 * ((il + 2) // 3) > dst.size):
        raise ValueError("message spans or output slots out of range")
    out_len = np.empty(max(N, 1), dtype=np.int64)
    fl = None if flags is None else np.ascontiguousarray(flags, dtype=np.uint8)
    lib().oracle_encode_gather_mt(_ptr(src), _ptr(ib), _ptr(il), N, _ptr(dst), _ptr(oo),
                                  None if fl is None else _ptr(fl), _ptr(out_len), int(threads))
    return out_len[:N]


def decode_gather(src, in_begin, in_len, out_off, dst, flags=None, threads=1):
    """Validating decode of messages src[in_begin[i], in_begin[i] + in_len[i])
    into dst[out_off[i]:]. Returns (out_len, err_off) per message."""
    src = _u8(src)
    ib = np.ascontiguousarray(in_begin, dtype=np.int64)
    il = np.ascontiguousarray(in_len, dtype=np.int64)
    oo = np.ascontiguousarray(out_off, dtype=np.int64)
    N = ib.size
    if il.size != N or oo.size < N or np.any(il < 0) or np.any(ib < 0) or np.any(ib + il > src.size) \
            or np.any(oo + 3 * (il // 4) > dst.size):
        raise ValueError("message spans or output slots out of range")
    out_len = np.empty(max(N, 1), dtype=np.int64)
    err = np.empty(max(N, 1), dtype=np.int64)
    fl = None if flags is None else np.ascontiguousarray(flags, dtype=np.uint8)
    lib().oracle_decode_gather_mt(_ptr(src), _ptr(ib), _ptr(il), N, _ptr(dst), _ptr(oo),
                                  None if fl is None else _ptr(fl), _ptr(out_len), _ptr(err), int(threads))
    return out_len[:N], err[:N]


class using:
    """Context manager that points this module at another build of the oracle
    (used by the mutation tests to check that the pins catch planted bugs)."""

    def __init__(self, path):
        self.path = path

    def __enter__(self):
        global _lib
        self._saved = _lib
        _lib = None
        saved_path = _build.LIB
        _build.LIB = self.path
        try:
            lib()
        finally:
            _build.LIB = saved_path
        return self

    def __exit__(self, *exc):
        global _lib
        _lib = self._saved
        return False
