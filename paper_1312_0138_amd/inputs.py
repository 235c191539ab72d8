"""Seeded synthetic inputs for the bitmap sort.

This module holds input generation only -- no step of the sort.  Both the
tests (which feed the oracle) and the benchmark use it; the HIP library has a
device twin of ``distinct_uniform`` (the keyed permutation below), and a test
checks the two bit for bit.

Generators
----------
* ``keyed_permutation`` -- a seeded bijection pi on [0, 2^bits): a 4-round
  Feistel network (Luby-Rackoff construction) whose halves have ceil(bits/2)
  and floor(bits/2) bits and trade places every round (an alternating
  unbalanced network; balanced when ``bits`` is even), so any ``bits`` maps
  onto itself without cycle walking.  Round keys come from SplitMix64
  (Steele, Lea, Flood 2014).  The round function is a multiply / xor-shift
  mix.
* ``distinct_uniform(n, bits, seed)`` = pi(0), ..., pi(n-1): n distinct keys in
  [0, 2^bits) in pseudo-random order ("uniform without replacement").
* ``dense_permutation(bits, seed)`` = pi over all of [0, 2^bits).
* ``clustered`` -- Gaussian clusters, rounded, clipped by redrawing,
  de-duplicated and shuffled.
* ``log_uniform_sizes`` and ``batch_segments`` -- uneven segment batches.
* ``poisson_arrivals`` -- exponential inter-arrival gaps.
"""
from __future__ import annotations

import math

import numpy as np

MASK32 = np.uint64(0xFFFFFFFF)
_GOLDEN64 = 0x9E3779B97F4A7C15
_M1 = np.uint64(0x9E3779B1)
_M2 = np.uint64(0x85EBCA77)
FEISTEL_ROUNDS = 4


def splitmix64(state: int):
    """One SplitMix64 step: returns (new_state, 64-bit output)."""
    state = (state + _GOLDEN64) & 0xFFFFFFFFFFFFFFFF
    z = state
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & 0xFFFFFFFFFFFFFFFF
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & 0xFFFFFFFFFFFFFFFF
    return state, z ^ (z >> 31)


def feistel_round_keys(seed: int) -> list[int]:
    """The four 32-bit round keys for ``seed`` (low halves of SplitMix64)."""
    st = seed & 0xFFFFFFFFFFFFFFFF
    keys = []
    for _ in range(FEISTEL_ROUNDS):
        st, z = splitmix64(st)
        keys.append(z & 0xFFFFFFFF)
    return keys


def _round_fn(r: np.ndarray, k: int) -> np.ndarray:
    x = (r ^ np.uint64(k)) & MASK32
    x = (x * _M1) & MASK32
    x ^= x >> np.uint64(15)
    x = (x * _M2) & MASK32
    x ^= x >> np.uint64(13)
    return x


def _feistel(x: np.ndarray, bits: int, rkeys) -> np.ndarray:
    """Feistel permutation of [0, 2^bits), 1 <= bits <= 32.

    The state is (left, right) with a = bits - bits//2 and b = bits//2 bits.
    A round maps (left, right) to (right, left ^ (F(right) mod 2^a)); the
    halves then hold b and a bits.  Each round is invertible, and after the
    (even) number of rounds the widths are back to (a, b)."""
    a, b = bits - bits // 2, bits // 2
    left = x >> np.uint64(b)
    right = x & np.uint64((1 << b) - 1)
    for k in rkeys:
        left, right = right, left ^ (_round_fn(right, k) & np.uint64((1 << a) - 1))
        a, b = b, a
    return (left << np.uint64(b)) | right


def keyed_permutation(idx, bits: int, seed: int) -> np.ndarray:
    """pi(idx) for the seeded bijection pi on [0, 2^bits); idx < 2^bits."""
    if not 0 <= bits <= 32:
        raise ValueError("bits must be in [0, 32]")
    idx = np.asarray(idx, dtype=np.uint64)
    if bits == 0:
        return np.zeros(idx.shape, dtype=np.uint32)
    return _feistel(idx, bits, feistel_round_keys(seed)).astype(np.uint32)


def distinct_uniform(n: int, bits: int, seed: int, chunk: int = 1 << 22) -> np.ndarray:
    """n distinct keys in [0, 2^bits), pseudo-random order: pi(0..n-1)."""
    if n > (1 << bits):
        raise ValueError("n exceeds the key range")
    out = np.empty(n, dtype=np.uint32)
    for lo in range(0, n, chunk):
        hi = min(n, lo + chunk)
        out[lo:hi] = keyed_permutation(np.arange(lo, hi, dtype=np.uint64), bits, seed)
    return out


def distinct_uniform_u64(n: int, bits: int, seed: int, chunk: int = 1 << 22) -> np.ndarray:
    """n distinct uint64 keys in [0, 2^bits), bits <= 64, pseudo-random order:
    the same Feistel network on wider halves (each at most 32 bits)."""
    if not 0 <= bits <= 64:
        raise ValueError("bits must be in [0, 64]")
    if n > (1 << bits):
        raise ValueError("n exceeds the key range")
    out = np.zeros(n, dtype=np.uint64)
    if bits == 0:
        return out
    rk = feistel_round_keys(seed)
    for lo in range(0, n, chunk):
        hi = min(n, lo + chunk)
        out[lo:hi] = _feistel(np.arange(lo, hi, dtype=np.uint64), bits, rk)
    return out


def dense_permutation(bits: int, seed: int) -> np.ndarray:
    """Every key of [0, 2^bits) once, in pseudo-random order."""
    return distinct_uniform(1 << bits, bits, seed)


def clustered(n_draws: int, bits: int, seed: int, clusters: int = 64,
              sigma: float = float(1 << 16)) -> np.ndarray:
    """Distinct keys from ``clusters`` Gaussian clusters in [0, 2^bits).

    Centres are uniform in [0, 2^bits).  Each of ``n_draws`` draws picks a
    cluster uniformly and adds sigma * N(0, 1); the value is rounded half up
    and redrawn while outside the range.  The draws are de-duplicated and the
    survivors shuffled, so the result has fewer than ``n_draws`` keys.
    """
    rng = np.random.default_rng(seed)
    r = 1 << bits
    centres = rng.integers(0, r, size=clusters, dtype=np.int64)
    vals = np.empty(n_draws, dtype=np.int64)
    todo = np.arange(n_draws)
    while todo.size:
        cid = rng.integers(0, clusters, size=todo.size)
        x = centres[cid] + sigma * rng.standard_normal(todo.size)
        k = np.floor(x + 0.5).astype(np.int64)
        ok = (k >= 0) & (k < r)
        vals[todo[ok]] = k[ok]
        todo = todo[~ok]
    keys = np.unique(vals).astype(np.uint32)
    return keys[rng.permutation(keys.size)]


def log_uniform_sizes(count: int, lo: int, hi: int, seed: int) -> np.ndarray:
    """``count`` sizes floor(exp(U(ln lo, ln hi))), clamped to [lo, hi]."""
    rng = np.random.default_rng(seed)
    u = rng.uniform(math.log(lo), math.log(hi), size=count)
    return np.clip(np.floor(np.exp(u)).astype(np.int64), lo, hi)


def range_bits_for(n: int, factor: int = 4) -> int:
    """Smallest b with 2^b >= factor * n (the power-of-two rounded range)."""
    need = max(1, factor * int(n))
    return int(need - 1).bit_length()


def segment_seed(seed: int, i: int) -> int:
    """Per-segment seed: SplitMix64 of (seed, i)."""
    _, z = splitmix64((seed * 0x100000001B3 + i) & 0xFFFFFFFFFFFFFFFF)
    return z


def batch_segments(count: int, lo: int, hi: int, seed: int, factor: int = 4):
    """A batch of ``count`` independent arrays, concatenated.

    Sizes are log-uniform in [lo, hi]; array i holds distinct_uniform(n_i,
    b_i, segment_seed(seed, i)) with 2^b_i the next power of two >= factor*n_i.
    Returns (keys uint32, offsets uint64[count+1], range_bits uint8[count]).
    """
    sizes = log_uniform_sizes(count, lo, hi, seed)
    rbits = np.array([range_bits_for(n, factor) for n in sizes], dtype=np.uint8)
    offsets = np.zeros(count + 1, dtype=np.uint64)
    offsets[1:] = np.cumsum(sizes, dtype=np.uint64)
    keys = np.empty(int(offsets[-1]), dtype=np.uint32)
    for i in range(count):
        keys[int(offsets[i]):int(offsets[i + 1])] = distinct_uniform(
            int(sizes[i]), int(rbits[i]), segment_seed(seed, i))
    return keys, offsets, rbits


def poisson_arrivals(count: int, rate_per_s: float, seed: int) -> np.ndarray:
    """Arrival times (s) of a Poisson process: cumulative exponential gaps."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate_per_s, size=count))


def config_seed(config_id: int, rep: int = 0) -> int:
    """Seed of a named workload and repetition."""
    return (0x13120138 ^ (config_id << 32) ^ rep) & 0xFFFFFFFFFFFFFFFF
