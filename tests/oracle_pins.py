"""Pins that tie the CPU oracle to facts outside itself.

Each ``pin_*`` takes an ``oracle.Oracle`` and raises AssertionError when the
oracle disagrees with the paper or with mathematics: the paper's printed
tables, brute force against Python's ``sorted`` on tiny inputs, closed forms,
invariants, an independent second method (the paper's Algorithm 1 against the
bitmap), and numpy routines.  ``run_all`` runs every pin; the planted-mistake
test runs it against mutated copies of the oracle and expects a failure.
"""
from __future__ import annotations

import os
import random

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")

FLAG_OOR = 1
FLAG_DUP = 2


def _rows(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append(line.split())
    return rows


def table1():
    """Section II, Table I: (x, y, and, or, xor, not x) bit rows."""
    return [tuple(int(v) for v in r) for r in _rows("table1_bitwise_ops.txt")]


def table2():
    """Section III, Table II: (value, 16-bit pattern) rows."""
    return [(int(r[0]), r[1]) for r in _rows("table2_short_repr.txt")]


def _to_i16(v: int) -> int:
    return ((v + 0x8000) & 0xFFFF) - 0x8000


# ---- the paper's tables ------------------------------------------------------

def pin_table1(o):
    """Bit test (Example 1) reads the bit of Table I's operands; marking is
    Table I's OR: it sets the bit whatever it held and touches no other."""
    rows = table1()
    assert len(rows) == 4
    for x, y, _and, orr, _xor, _notx in rows:
        for i in (0, 5, 31):
            assert o.bit_value(x << i, i) == x
            assert o.bit_value((x << i) ^ 0xFFFFFFFF, i) == 1 - x
        for bit in (0, 5, 31):
            words = np.array([x << bit], dtype=np.uint32)
            o.bitmap_mark_into(words, [bit] if y else [], 5)
            assert (int(words[0]) >> bit) & 1 == orr
            assert int(words[0]) & ~(1 << bit) == 0


def pin_table2(o):
    """Example 4's bit printer reproduces Table II (bit 0 rightmost)."""
    rows = table2()
    assert len(rows) == 15
    for v, bits in rows:
        assert o.bin_repl_i16(_to_i16(v)) == bits, (v, bits)


def pin_helpers(o):
    """Example 2's power of two and Example 6's count of ones, over all bits."""
    for n in range(32):
        assert o.power2(n) == 1 << n
    rng = random.Random(12)
    vals = [0, 1, 0x80000000, 0xFFFFFFFF, 0x7FFFFFFF, 0x55555555, 0xAAAAAAAA]
    vals += [rng.getrandbits(32) for _ in range(200)]
    for x in vals:
        assert o.count_ones(x) == bin(x).count("1")
        for i in (0, 1, 15, 30, 31):
            assert o.bit_value(x, i) == (x >> i) & 1


# ---- brute force on tiny inputs ---------------------------------------------------

def pin_all_subsets(o):
    """Every subset of [0, 16), shuffled, sorted at range_bits 4, 5 and 6,
    equals Python's sorted()."""
    rng = random.Random(3)
    subsets = []
    for mask in range(1 << 16):
        s = [i for i in range(16) if (mask >> i) & 1]
        rng.shuffle(s)
        subsets.append(s)
    sizes = np.array([len(s) for s in subsets], dtype=np.uint64)
    flat = np.array([v for s in subsets for v in s], dtype=np.uint32)
    expect = np.array([v for s in subsets for v in sorted(s)], dtype=np.uint32)
    offsets = np.zeros(len(subsets) + 1, dtype=np.uint64)
    offsets[1:] = np.cumsum(sizes)
    for rb in (4, 5, 6):
        out, n_out, flags = o.bitmap_sort_segments(flat, offsets, np.full(len(subsets), rb))
        assert np.array_equal(n_out, sizes)
        assert not flags.any()
        assert np.array_equal(out, expect), rb


def pin_random_tiny(o):
    """Random distinct keys, n <= 64, every range_bits in [0, 32]: the bitmap
    sort, the 8- and 64-bit-word variants and Algorithm 1 all equal sorted()."""
    rng = random.Random(5)
    for rb in range(33):
        for _ in range(12 if rb <= 24 else 2):
            n = rng.randint(0, min(64, 1 << rb))
            keys = rng.sample(range(1 << rb), n)
            expect = sorted(keys)
            out, flags, _ = o.bitmap_sort(keys, rb)
            assert flags == 0
            assert out.tolist() == expect, (rb, keys)
            assert o.bitmap_sort_w64(keys, rb).tolist() == expect
            assert o.bitmap_sort_w8(keys, rb).tolist() == expect
            assert o.bitwise_sort1(keys, 32).tolist() == expect


# ---- closed forms and invariants -----------------------------------------------

def pin_permutation_identity(o):
    """A permutation of [0, R) sorts to the identity 0, 1, ..., R-1."""
    rng = np.random.default_rng(7)
    for rb in list(range(0, 13)) + [16, 20]:
        keys = rng.permutation(1 << rb).astype(np.uint32)
        out, flags, _ = o.bitmap_sort(keys, rb)
        assert flags == 0
        assert np.array_equal(out, np.arange(1 << rb, dtype=np.uint32)), rb


def pin_invariants(o):
    """Medium random input: length n, strictly ascending, same set as the
    input (numpy's sort as the reference), independent of input order."""
    rng = np.random.default_rng(11)
    for rb, n in ((24, 100_000), (32, 50_000), (17, 1 << 17), (5, 20)):
        keys = rng.choice(1 << rb, size=n, replace=False).astype(np.uint32) if rb < 32 else \
            np.unique(rng.integers(0, 1 << 32, size=n, dtype=np.uint64)).astype(np.uint32)
        out, flags, _ = o.bitmap_sort(keys, rb)
        assert flags == 0
        assert out.size == keys.size
        assert np.all(out[1:] > out[:-1])
        assert np.array_equal(out, np.sort(keys))
        out2, _, _ = o.bitmap_sort(keys[rng.permutation(keys.size)], rb)
        assert np.array_equal(out, out2)


def pin_word_width(o):
    """The result does not depend on the word width (8, 32 or 64 bits)."""
    rng = np.random.default_rng(13)
    for rb in (3, 6, 7, 9, 20, 26):
        n = min(5000, 1 << rb)
        keys = rng.choice(1 << rb, size=n, replace=False).astype(np.uint32)
        a, _, _ = o.bitmap_sort(keys, rb)
        assert np.array_equal(a, o.bitmap_sort_w64(keys, rb))
        assert np.array_equal(a, o.bitmap_sort_w8(keys, rb))


def pin_scan(o):
    """Scan step: prefix[w] = set bits in words < w, against numpy's
    cumulative sum of numpy's bit count."""
    rng = np.random.default_rng(17)
    for words in (
        np.zeros(5, dtype=np.uint32),
        np.full(7, 0xFFFFFFFF, dtype=np.uint32),
        np.array([0x80000000, 1, 0x80000001, 0], dtype=np.uint32),
        rng.integers(0, 1 << 32, size=1000, dtype=np.uint64).astype(np.uint32),
    ):
        ref = np.concatenate([[0], np.cumsum(np.bitwise_count(words).astype(np.uint64))])
        assert np.array_equal(o.bitmap_scan(words), ref.astype(np.uint64))


def pin_mark_emit(o):
    """Mark sets exactly the bits numpy's bit arithmetic predicts; emit of that
    bitmap gives back the keys ascending."""
    rng = np.random.default_rng(19)
    for rb in (0, 4, 5, 6, 12, 21):
        n = min(3000, 1 << rb)
        keys = rng.choice(1 << rb, size=n, replace=False).astype(np.uint32)
        words, flags = o.bitmap_build(keys, rb)
        assert flags == 0
        ref = np.zeros(max(1, (1 << rb) // 32), dtype=np.uint32)
        np.bitwise_or.at(ref, (keys >> 5).astype(np.int64),
                         np.left_shift(np.uint32(1), keys & np.uint32(31)))
        assert np.array_equal(words, ref)
        assert np.array_equal(o.bitmap_emit(words), np.sort(keys))


# ---- the paper's Algorithm 1 ---------------------------------------------------------

def pin_algorithm1(o):
    """BitwiseSort1 with 32 passes equals numpy's sort on unsigned keys; the
    listing's 31 passes leave keys >= 2^31 out of order (reading O5)."""
    rng = np.random.default_rng(23)
    keys = rng.integers(0, 1 << 32, size=4000, dtype=np.uint64).astype(np.uint32)
    assert np.array_equal(o.bitwise_sort1(keys, 32), np.sort(keys))
    short = o.bitwise_sort1(keys, 31)
    assert not np.all(short[1:] >= short[:-1])
    assert np.array_equal(np.sort(short), np.sort(keys))


def pin_theorem1(o):
    """Theorem 1's induction: after p passes the array is ordered by its low p
    bits, and elements with equal low bits keep their input order (Python's
    stable sort by key is the reference)."""
    rng = random.Random(29)
    keys = [rng.getrandbits(32) for _ in range(600)] + [5, 5 + (1 << 7), 5 + (1 << 20)]
    rng.shuffle(keys)
    for p in (0, 1, 2, 3, 7, 8, 16, 31, 32):
        mask = (1 << p) - 1
        expect = sorted(keys, key=lambda v: v & mask)
        assert o.bitwise_sort1(keys, p).tolist() == expect, p


def pin_signed(o):
    """BitwiseSort (sign split, negatives first) equals numpy's sort on int32,
    including INT_MIN, -1, 0 and INT_MAX."""
    rng = np.random.default_rng(31)
    keys = rng.integers(-(1 << 31), 1 << 31, size=3000, dtype=np.int64).astype(np.int32)
    keys = np.concatenate([keys, np.array([-(1 << 31), -1, 0, (1 << 31) - 1, 0, -1], dtype=np.int32)])
    rng.shuffle(keys)
    assert np.array_equal(o.bitwise_sort_i32(keys), np.sort(keys))
    assert o.bitwise_sort_i32(np.array([3, -2, 0], dtype=np.int32)).tolist() == [-2, 0, 3]


def pin_algorithm1_u64(o):
    """Algorithm 1 for T = uint64: 64 passes equal numpy's sort (keys above
    2^32 and 2^63 included), and Theorem 1's induction holds at every pass
    count (Python's stable sort by the low p bits is the reference)."""
    rng = np.random.default_rng(47)
    keys = rng.integers(0, 1 << 64, size=3000, dtype=np.uint64)
    keys[:4] = [0, (1 << 64) - 1, 1 << 63, (1 << 32) + 1]
    assert np.array_equal(o.bitwise_sort1_u64(keys, 64), np.sort(keys))
    small = [int(v) for v in keys[:400]] + [7, 7 + (1 << 40), 7 + (1 << 63)]
    for p in (0, 1, 8, 32, 33, 40, 63, 64):
        mask = (1 << p) - 1
        expect = sorted(small, key=lambda v: v & mask)
        assert o.bitwise_sort1_u64(np.array(small, dtype=np.uint64), p).tolist() == expect, p


def pin_pairs(o):
    """Algorithm 1 on (key, value) records: the keys come out sorted and the
    values follow their keys in input order among equal keys -- numpy's
    stable argsort of the keys; after p passes, Python's stable sort by the
    low p bits."""
    rng = np.random.default_rng(53)
    keys = rng.integers(0, 300, size=5000, dtype=np.uint64).astype(np.uint32)
    keys[::7] = rng.integers(0, 1 << 32, size=keys[::7].size, dtype=np.uint64).astype(np.uint32)
    vals = np.arange(keys.size, dtype=np.uint32)
    k, v = o.bitwise_sort1_pairs(keys, vals, 32)
    order = np.argsort(keys, kind="stable")
    assert np.array_equal(k, keys[order]) and np.array_equal(v, vals[order])
    for p in (0, 3, 9, 31):
        mask = (1 << p) - 1
        idx = sorted(range(600), key=lambda i: int(keys[i]) & mask)
        k, v = o.bitwise_sort1_pairs(keys[:600], vals[:600], p)
        assert v.tolist() == idx and k.tolist() == [int(keys[i]) for i in idx], p


# ---- precondition violations and edges --------------------------------------------------

def pin_duplicates(o):
    """Reading O6: duplicates collapse to one copy, out[d..n) is untouched and
    the DUPLICATE flag is raised."""
    keys = [9, 3, 9, 0, 3, 31, 32, 9]
    init = [77] * len(keys)
    out, flags, full = o.bitmap_sort(keys, 6, out_init=init)
    assert out.tolist() == [0, 3, 9, 31, 32]
    assert full.tolist()[5:] == [77, 77, 77]
    assert flags & FLAG_DUP and not flags & FLAG_OOR
    _, f2, _ = o.bitmap_sort([1, 2, 3], 2)
    assert f2 == 0


def pin_out_of_range(o):
    """Reading O7: a key >= R is dropped and flagged; R-1 is kept."""
    for rb in (0, 1, 5, 6, 16):
        r = 1 << rb
        keys = [r - 1, r, r + 5, 0xFFFFFFFF]
        out, flags, _ = o.bitmap_sort(keys, rb)
        assert flags & FLAG_OOR
        assert out.tolist() == [r - 1]
    out, flags, _ = o.bitmap_sort([0xFFFFFFFF, 0], 32)
    assert flags == 0 and out.tolist() == [0, 0xFFFFFFFF]


def pin_edges(o):
    """n = 0; range_bits 0 (only key 0); word boundaries; a full word;
    range_bits < 5; range_bits 32 with the extreme keys."""
    out, flags, _ = o.bitmap_sort([], 10)
    assert out.size == 0 and flags == 0
    assert o.bitmap_sort([0], 0)[0].tolist() == [0]
    b = [64, 31, 63, 32, 0, 95, 96]
    assert o.bitmap_sort(b, 7)[0].tolist() == sorted(b)
    full = list(range(32, 64))
    random.Random(1).shuffle(full)
    assert o.bitmap_sort(full, 6)[0].tolist() == list(range(32, 64))
    for rb in range(5):
        ks = list(range(1 << rb))[::-1]
        assert o.bitmap_sort(ks, rb)[0].tolist() == list(range(1 << rb))
    ext = [0xFFFFFFFF, 0x80000000, 0x7FFFFFFF, 0, 1]
    assert o.bitmap_sort(ext, 32)[0].tolist() == sorted(ext)
    assert o.bitmap_words(0) == 1 and o.bitmap_words(5) == 1 and o.bitmap_words(6) == 2
    assert o.bitmap_words(32) == 1 << 27 and o.bitmap_words(33) == 0


def pin_segments(o):
    """Segmented form: each segment equals the single-array sort of its keys,
    empty segments included."""
    rng = np.random.default_rng(37)
    sizes = [0, 1, 5, 0, 300, 1024, 2]
    rbits = [3, 1, 4, 9, 12, 10, 2]
    parts = [rng.choice(1 << rb, size=n, replace=False).astype(np.uint32) for n, rb in zip(sizes, rbits)]
    keys = np.concatenate(parts)
    offsets = np.concatenate([[0], np.cumsum(sizes)]).astype(np.uint64)
    out, n_out, flags = o.bitmap_sort_segments(keys, offsets, rbits)
    assert n_out.tolist() == sizes and not flags.any()
    for i, p in enumerate(parts):
        assert np.array_equal(out[offsets[i]:offsets[i + 1]], np.sort(p))


def pin_counting(o):
    """Counting sort keeps duplicates: equals numpy's sort of the multiset."""
    rng = np.random.default_rng(41)
    for rb in (0, 3, 10, 16):
        keys = rng.integers(0, 1 << rb, size=2000, dtype=np.uint64).astype(np.uint32)
        out, flags = o.counting_sort(keys, rb)
        assert flags == 0 and np.array_equal(out, np.sort(keys))
    out, flags = o.counting_sort([7, 8, 7], 3)
    assert out.tolist() == [7, 7] and flags & FLAG_OOR


def pin_u64(o):
    """64-bit keys: equals numpy's sort for range_bits up to 36."""
    rng = np.random.default_rng(43)
    for rb in (1, 6, 7, 20, 33):
        n = min(3000, 1 << rb)
        keys = np.unique(rng.integers(0, 1 << rb, size=n, dtype=np.uint64))
        rng.shuffle(keys)
        out, flags = o.bitmap_sort_u64(keys, rb)
        assert flags == 0 and np.array_equal(out, np.sort(keys))
    out, flags = o.bitmap_sort_u64(np.array([5, 5, 1 << 40], dtype=np.uint64), 20)
    assert out.tolist() == [5] and flags & FLAG_DUP and flags & FLAG_OOR


ALL_PINS = [
    pin_table1, pin_table2, pin_helpers, pin_all_subsets, pin_random_tiny,
    pin_permutation_identity, pin_invariants, pin_word_width, pin_scan, pin_mark_emit,
    pin_algorithm1, pin_theorem1, pin_signed, pin_duplicates, pin_out_of_range, pin_edges,
    pin_segments, pin_counting, pin_u64, pin_algorithm1_u64, pin_pairs,
]


def run_all(o, stop_at_first: bool = False) -> list[str]:
    """Run every pin; return the names of the pins that failed (an exception
    of any kind counts as a failure)."""
    failed = []
    for pin in ALL_PINS:
        try:
            pin(o)
        except Exception:  # noqa: BLE001 - any error means the pin caught it
            failed.append(pin.__name__)
            if stop_at_first:
                break
    return failed
