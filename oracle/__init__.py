"""CPU oracle for the bitmap sort (test infrastructure only).

Thin ctypes wrapper over ``bitsort_oracle.c``: a plain, single-threaded C
implementation written from the paper (Yordzhev, arXiv:1312.0138) -- the
bit helpers of Section III, the bitmap mark / scan / emit steps, the paper's
Algorithm 1 (BitwiseSort1 / BitwiseSort), counting sort (Section IV) and a
64-bit-key variant.  Every reading of the paper it takes is listed in the
header of the C file.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import this package.  The HIP library never calls it, and the two share no
code; they meet only through the seeded input generators.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from .build import LIB_PATH, build_oracle

FLAG_OUT_OF_RANGE = 1
FLAG_DUPLICATE = 2

_u32p = ctypes.POINTER(ctypes.c_uint32)
_u64p = ctypes.POINTER(ctypes.c_uint64)
_i32p = ctypes.POINTER(ctypes.c_int32)
_u8p = ctypes.POINTER(ctypes.c_uint8)


def _ptr(a: np.ndarray, typ):
    return a.ctypes.data_as(typ)


class OracleError(RuntimeError):
    pass


class Oracle:
    """One loaded copy of the oracle library (tests load planted-mistake
    copies through the same class)."""

    def __init__(self, path: str):
        lib = ctypes.CDLL(path)
        self._lib = lib
        self.path = path
        c = ctypes
        sig = {
            "oracle_bit_value": (c.c_uint32, [c.c_uint32, c.c_uint32]),
            "oracle_power2": (c.c_uint32, [c.c_uint32]),
            "oracle_count_ones": (c.c_uint32, [c.c_uint32]),
            "oracle_bin_repl_i16": (None, [c.c_int16, c.c_char_p]),
            "oracle_bitmap_words": (c.c_uint64, [c.c_uint32]),
            "oracle_bitmap_mark_u32": (c.c_int, [_u32p, c.c_uint64, c.c_uint32, _u32p, _u32p]),
            "oracle_bitmap_build_u32": (c.c_int, [_u32p, c.c_uint64, c.c_uint32, _u32p, _u32p]),
            "oracle_bitmap_scan_u32": (c.c_int, [_u32p, c.c_uint64, _u64p]),
            "oracle_bitmap_emit_u32": (c.c_uint64, [_u32p, c.c_uint64, _u32p]),
            "oracle_bitmap_sort_u32": (c.c_int, [_u32p, c.c_uint64, c.c_uint32, _u32p, _u64p, _u32p]),
            "oracle_bitmap_sort_u32_w64": (c.c_int, [_u32p, c.c_uint64, c.c_uint32, _u32p, _u64p]),
            "oracle_bitmap_sort_u32_w8": (c.c_int, [_u32p, c.c_uint64, c.c_uint32, _u32p, _u64p]),
            "oracle_bitmap_sort_segments_u32": (
                c.c_int, [_u32p, _u64p, c.c_uint32, _u8p, _u32p, _u64p, _u32p]),
            "oracle_bitwise_sort1_u32": (c.c_int, [_u32p, c.c_uint64, c.c_uint32]),
            "oracle_bitwise_sort1_u64": (c.c_int, [_u64p, c.c_uint64, c.c_uint32]),
            "oracle_bitwise_sort1_pairs_u32": (c.c_int, [_u32p, _u32p, c.c_uint64, c.c_uint32]),
            "oracle_bitwise_sort_i32": (c.c_int, [_i32p, c.c_uint64]),
            "oracle_counting_sort_u32": (c.c_int, [_u32p, c.c_uint64, c.c_uint32, _u32p, _u64p, _u32p]),
            "oracle_bitmap_sort_u64": (c.c_int, [_u64p, c.c_uint64, c.c_uint32, _u64p, _u64p, _u32p]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args

    # -- Section III helpers -------------------------------------------------
    def bit_value(self, x: int, i: int) -> int:
        return int(self._lib.oracle_bit_value(x, i))

    def power2(self, n: int) -> int:
        return int(self._lib.oracle_power2(n))

    def count_ones(self, x: int) -> int:
        return int(self._lib.oracle_count_ones(x))

    def bin_repl_i16(self, v: int) -> str:
        buf = ctypes.create_string_buffer(17)
        self._lib.oracle_bin_repl_i16(v, buf)
        return buf.value.decode()

    # -- bitmap steps -----------------------------------------------------------
    def bitmap_words(self, range_bits: int) -> int:
        return int(self._lib.oracle_bitmap_words(range_bits))

    def bitmap_build(self, keys, range_bits: int):
        """Mark step into a zeroed bitmap -> (uint32 words, flags)."""
        keys = np.ascontiguousarray(keys, dtype=np.uint32)
        words = np.zeros(max(self.bitmap_words(range_bits), 1), dtype=np.uint32)
        flags = np.zeros(1, dtype=np.uint32)
        rc = self._lib.oracle_bitmap_build_u32(_ptr(keys, _u32p), keys.size, range_bits,
                                               _ptr(words, _u32p), _ptr(flags, _u32p))
        if rc != 0:
            raise OracleError(f"oracle_bitmap_build_u32 -> {rc}")
        return words, int(flags[0])

    def bitmap_mark_into(self, words: np.ndarray, keys, range_bits: int) -> int:
        """Mark step OR-ed into an existing bitmap (modified in place) -> flags."""
        keys = np.ascontiguousarray(keys, dtype=np.uint32)
        assert words.dtype == np.uint32 and words.flags.c_contiguous
        flags = np.zeros(1, dtype=np.uint32)
        rc = self._lib.oracle_bitmap_mark_u32(_ptr(keys, _u32p), keys.size, range_bits,
                                              _ptr(words, _u32p), _ptr(flags, _u32p))
        if rc != 0:
            raise OracleError(f"oracle_bitmap_mark_u32 -> {rc}")
        return int(flags[0])

    def bitmap_scan(self, words) -> np.ndarray:
        """Scan step -> uint64 prefix of length words+1."""
        words = np.ascontiguousarray(words, dtype=np.uint32)
        prefix = np.zeros(words.size + 1, dtype=np.uint64)
        rc = self._lib.oracle_bitmap_scan_u32(_ptr(words, _u32p), words.size, _ptr(prefix, _u64p))
        if rc != 0:
            raise OracleError(f"oracle_bitmap_scan_u32 -> {rc}")
        return prefix

    def bitmap_emit(self, words) -> np.ndarray:
        words = np.ascontiguousarray(words, dtype=np.uint32)
        total = int(np.bitwise_count(words).sum()) if words.size else 0
        out = np.zeros(max(total, 1), dtype=np.uint32)
        j = self._lib.oracle_bitmap_emit_u32(_ptr(words, _u32p), words.size, _ptr(out, _u32p))
        return out[: int(j)]

    # -- whole sorts --------------------------------------------------------------
    def bitmap_sort(self, keys, range_bits: int, out_init=None):
        """Bitmap sort -> (out[:d], flags, out_full).  out_full holds all n slots,
        the slots past d keep out_init (default: zeros)."""
        keys = np.ascontiguousarray(keys, dtype=np.uint32)
        n = keys.size
        if out_init is None:
            out = np.zeros(max(n, 1), dtype=np.uint32)
        else:
            out = np.array(out_init, dtype=np.uint32, copy=True)
            if out.size == 0:
                out = np.zeros(1, dtype=np.uint32)
        n_out = np.zeros(1, dtype=np.uint64)
        flags = np.zeros(1, dtype=np.uint32)
        rc = self._lib.oracle_bitmap_sort_u32(_ptr(keys, _u32p), n, range_bits, _ptr(out, _u32p),
                                              _ptr(n_out, _u64p), _ptr(flags, _u32p))
        if rc != 0:
            raise OracleError(f"oracle_bitmap_sort_u32 -> {rc}")
        d = int(n_out[0])
        return out[:d].copy(), int(flags[0]), out[:n]

    def bitmap_sort_w64(self, keys, range_bits: int) -> np.ndarray:
        keys = np.ascontiguousarray(keys, dtype=np.uint32)
        out = np.zeros(max(keys.size, 1), dtype=np.uint32)
        n_out = np.zeros(1, dtype=np.uint64)
        rc = self._lib.oracle_bitmap_sort_u32_w64(_ptr(keys, _u32p), keys.size, range_bits,
                                                  _ptr(out, _u32p), _ptr(n_out, _u64p))
        if rc != 0:
            raise OracleError(f"oracle_bitmap_sort_u32_w64 -> {rc}")
        return out[: int(n_out[0])]

    def bitmap_sort_w8(self, keys, range_bits: int) -> np.ndarray:
        keys = np.ascontiguousarray(keys, dtype=np.uint32)
        out = np.zeros(max(keys.size, 1), dtype=np.uint32)
        n_out = np.zeros(1, dtype=np.uint64)
        rc = self._lib.oracle_bitmap_sort_u32_w8(_ptr(keys, _u32p), keys.size, range_bits,
                                                 _ptr(out, _u32p), _ptr(n_out, _u64p))
        if rc != 0:
            raise OracleError(f"oracle_bitmap_sort_u32_w8 -> {rc}")
        return out[: int(n_out[0])]

    def bitmap_sort_segments(self, keys, offsets, range_bits, out_init=None):
        """Segmented bitmap sort -> (out, n_out per segment, flags per segment)."""
        keys = np.ascontiguousarray(keys, dtype=np.uint32)
        offsets = np.ascontiguousarray(offsets, dtype=np.uint64)
        rbits = np.ascontiguousarray(range_bits, dtype=np.uint8)
        s = rbits.size
        assert offsets.size == s + 1
        if out_init is None:
            out = np.zeros(max(keys.size, 1), dtype=np.uint32)
        else:
            out = np.array(out_init, dtype=np.uint32, copy=True)
        n_out = np.zeros(max(s, 1), dtype=np.uint64)
        flags = np.zeros(max(s, 1), dtype=np.uint32)
        rc = self._lib.oracle_bitmap_sort_segments_u32(
            _ptr(keys, _u32p), _ptr(offsets, _u64p), s, _ptr(rbits, _u8p), _ptr(out, _u32p),
            _ptr(n_out, _u64p), _ptr(flags, _u32p))
        if rc != 0:
            raise OracleError(f"oracle_bitmap_sort_segments_u32 -> {rc}")
        return out[: keys.size], n_out[:s], flags[:s]

    def bitwise_sort1(self, keys, passes: int = 32) -> np.ndarray:
        """The paper's BitwiseSort1 on uint32 (a sorted copy)."""
        a = np.array(keys, dtype=np.uint32, copy=True)
        if a.size == 0:
            return a
        rc = self._lib.oracle_bitwise_sort1_u32(_ptr(a, _u32p), a.size, passes)
        if rc != 0:
            raise OracleError(f"oracle_bitwise_sort1_u32 -> {rc}")
        return a

    def bitwise_sort1_u64(self, keys, passes: int = 64) -> np.ndarray:
        """BitwiseSort1 for T = uint64 (a sorted copy)."""
        a = np.array(keys, dtype=np.uint64, copy=True)
        if a.size == 0:
            return a
        rc = self._lib.oracle_bitwise_sort1_u64(_ptr(a, _u64p), a.size, passes)
        if rc != 0:
            raise OracleError(f"oracle_bitwise_sort1_u64 -> {rc}")
        return a

    def bitwise_sort1_pairs(self, keys, values, passes: int = 32):
        """BitwiseSort1 on (key, value) records: (sorted keys, their values)."""
        k = np.array(keys, dtype=np.uint32, copy=True)
        v = np.array(values, dtype=np.uint32, copy=True)
        if k.size != v.size:
            raise ValueError("keys and values differ in length")
        if k.size == 0:
            return k, v
        rc = self._lib.oracle_bitwise_sort1_pairs_u32(_ptr(k, _u32p), _ptr(v, _u32p), k.size, passes)
        if rc != 0:
            raise OracleError(f"oracle_bitwise_sort1_pairs_u32 -> {rc}")
        return k, v

    def bitwise_sort_i32(self, keys) -> np.ndarray:
        """The paper's BitwiseSort (sign split) on int32 (a sorted copy)."""
        a = np.array(keys, dtype=np.int32, copy=True)
        if a.size == 0:
            return a
        rc = self._lib.oracle_bitwise_sort_i32(_ptr(a, _i32p), a.size)
        if rc != 0:
            raise OracleError(f"oracle_bitwise_sort_i32 -> {rc}")
        return a

    def counting_sort(self, keys, range_bits: int):
        keys = np.ascontiguousarray(keys, dtype=np.uint32)
        out = np.zeros(max(keys.size, 1), dtype=np.uint32)
        n_out = np.zeros(1, dtype=np.uint64)
        flags = np.zeros(1, dtype=np.uint32)
        rc = self._lib.oracle_counting_sort_u32(_ptr(keys, _u32p), keys.size, range_bits,
                                                _ptr(out, _u32p), _ptr(n_out, _u64p),
                                                _ptr(flags, _u32p))
        if rc != 0:
            raise OracleError(f"oracle_counting_sort_u32 -> {rc}")
        return out[: int(n_out[0])].copy(), int(flags[0])

    def bitmap_sort_u64(self, keys, range_bits: int):
        keys = np.ascontiguousarray(keys, dtype=np.uint64)
        out = np.zeros(max(keys.size, 1), dtype=np.uint64)
        n_out = np.zeros(1, dtype=np.uint64)
        flags = np.zeros(1, dtype=np.uint32)
        rc = self._lib.oracle_bitmap_sort_u64(_ptr(keys, _u64p), keys.size, range_bits,
                                              _ptr(out, _u64p), _ptr(n_out, _u64p),
                                              _ptr(flags, _u32p))
        if rc != 0:
            raise OracleError(f"oracle_bitmap_sort_u64 -> {rc}")
        return out[: int(n_out[0])].copy(), int(flags[0])


_default: Oracle | None = None


def default() -> Oracle:
    """The oracle built from ``bitsort_oracle.c`` (built with gcc if missing)."""
    global _default
    if _default is None:
        if not os.path.exists(LIB_PATH):
            build_oracle()
        _default = Oracle(LIB_PATH)
    return _default
