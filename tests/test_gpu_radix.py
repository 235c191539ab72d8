"""Parity of the GPU LSD radix sort (bitsort_radix_u32: the paper's
Algorithm 1 run as 8-bit digit passes) with the oracle's Algorithm 1 over
the same number of bit passes, element by element."""
import numpy as np
import pytest

import oracle
from gpu_util import require_gpu, to_dev, to_np

pytestmark = pytest.mark.gpu

TILE = 4096


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


@pytest.fixture(scope="module")
def o():
    return oracle.default()


def _radix(keys, key_bits, out_init=None):
    import paper_1312_0138_amd as bs
    k = to_dev(keys)
    out = bs.radix_sort(k, key_bits)
    st = bs.status()
    return to_np(out), st


def _rand(n, bits, seed):
    rng = np.random.default_rng(seed)
    hi = 1 << bits
    return rng.integers(0, hi, size=n, dtype=np.uint64).astype(np.uint32)


@pytest.mark.parametrize("n", [1, 2, 63, 64, 65, 1023, TILE - 1, TILE, TILE + 1, 3 * TILE + 17, 100_003, 1_000_000])
def test_random_full_width(o, n):
    keys = _rand(n, 32, n)
    got, st = _radix(keys, 32)
    np.testing.assert_array_equal(got, o.bitwise_sort1(keys, 32))
    assert st.flags == 0 and st.count == n


@pytest.mark.parametrize("n", [5, 4099, 100_003])
def test_unaligned_input(o, n):
    """Keys starting 4 bytes past a 16-byte boundary (the histogram's scalar path) and
    sizes with a ragged tail of the 16-byte loads."""
    import paper_1312_0138_amd as bs
    keys = _rand(n + 1, 32, 300 + n)
    base = to_dev(keys)
    view = base[1:]
    assert view.data_ptr() % 16 != 0
    got = to_np(bs.radix_sort(view, 32))
    np.testing.assert_array_equal(got, o.bitwise_sort1(keys[1:], 32))
    st = bs.status()
    assert st.flags == 0 and st.count == n


@pytest.mark.parametrize("key_bits", [0, 1, 5, 8, 9, 16, 17, 24, 31])
def test_key_bits(o, key_bits):
    n = 2 * TILE + 333
    keys = _rand(n, key_bits, 100 + key_bits)
    got, st = _radix(keys, key_bits)
    np.testing.assert_array_equal(got, o.bitwise_sort1(keys, key_bits))
    assert st.flags == 0 and st.count == n


@pytest.mark.parametrize("key_bits", [4, 12, 20, 27])
def test_out_of_range_keys_order_by_low_bits_stably(o, key_bits):
    # high bits above key_bits make equal low parts distinguishable: their
    # input order must survive (the stability Theorem 1's induction uses)
    n = 50_000
    keys = _rand(n, 32, 7 + key_bits)
    got, st = _radix(keys, key_bits)
    np.testing.assert_array_equal(got, o.bitwise_sort1(keys, key_bits))
    assert st.flags == 1 and st.count == n


@pytest.mark.parametrize("distinct", [1, 2, 16, 255, 256, 257, 70_000])
def test_duplicates_kept(o, distinct):
    n = 300_000
    rng = np.random.default_rng(distinct)
    pool = rng.integers(0, 1 << 32, size=distinct, dtype=np.uint64).astype(np.uint32)
    keys = pool[rng.integers(0, distinct, size=n)]
    got, st = _radix(keys, 32)
    np.testing.assert_array_equal(got, o.bitwise_sort1(keys, 32))
    assert st.flags == 0


def test_presorted_and_reversed(o):
    n = 5 * TILE + 1
    up = np.sort(_rand(n, 32, 3))
    for keys in (up, up[::-1].copy(), np.zeros(n, np.uint32), np.full(n, 0xFFFFFFFF, np.uint32)):
        got, _ = _radix(keys, 32)
        np.testing.assert_array_equal(got, o.bitwise_sort1(keys, 32))


@pytest.mark.parametrize("key_bits", [8, 24, 32])
def test_in_place(o, key_bits):
    import paper_1312_0138_amd as bs
    keys = _rand(3 * TILE + 5, key_bits, key_bits)
    k = to_dev(keys)
    bs.radix_sort(k, key_bits, out=k)
    np.testing.assert_array_equal(to_np(k), o.bitwise_sort1(keys, key_bits))


def test_workspace_variant_and_side_stream(o):
    import torch
    import paper_1312_0138_amd as bs
    keys = _rand(200_000, 32, 11)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        k = to_dev(keys)
        ws = torch.empty(bs.radix_workspace_bytes(keys.size, 32), dtype=torch.uint8, device="cuda")
        out = bs.radix_sort_ws(k, ws, 32, stream=s)
        st = bs.workspace_status(ws, stream=s)
    s.synchronize()
    np.testing.assert_array_equal(to_np(out), o.bitwise_sort1(keys, 32))
    assert st.flags == 0 and st.count == keys.size


def test_empty():
    import torch
    import paper_1312_0138_amd as bs
    k = torch.empty(0, dtype=torch.int32, device="cuda")
    assert bs.radix_sort(k, 32).numel() == 0
    st = bs.status()
    assert st.count == 0


def test_full_size_against_oracle(o):
    # 2^26 uniform keys (the bitmap sort's default size), full width
    from paper_1312_0138_amd import inputs
    n = 1 << 26
    keys = inputs.distinct_uniform(n, 28, inputs.config_seed(2, 0))
    got, st = _radix(keys, 32)
    np.testing.assert_array_equal(got, o.bitwise_sort1(keys, 32))
    assert st.flags == 0


def test_matches_bitmap_sort_on_distinct_keys():
    import paper_1312_0138_amd as bs
    k = bs.generate(1 << 22, 26, 99)
    a = bs.sort(k, 26)
    b = bs.radix_sort(k, 26)
    import torch
    assert torch.equal(a, b)


def test_repeatable():
    import torch
    import paper_1312_0138_amd as bs
    k = to_dev(_rand(1 << 20, 32, 5))
    first = bs.radix_sort(k, 32).clone()
    for _ in range(3):
        assert torch.equal(bs.radix_sort(k, 32), first)


# ---- 64-bit keys and key-value records ---------------------------------------------------

def _dev64(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.uint64).view(np.int64).copy()).cuda()


@pytest.mark.parametrize("n", [1, 63, 2047, 2048, 2049, 100_003, 1_000_000])
def test_u64_full_width(o, n):
    import paper_1312_0138_amd as bs
    rng = np.random.default_rng(n + 64)
    keys = rng.integers(0, 1 << 64, size=n, dtype=np.uint64)
    got = bs.radix_sort_u64(_dev64(keys), 64).cpu().numpy().view(np.uint64)
    np.testing.assert_array_equal(got, o.bitwise_sort1_u64(keys, 64))
    st = bs.status()
    assert st.flags == 0 and st.count == n


@pytest.mark.parametrize("key_bits", [0, 8, 33, 40, 57])
def test_u64_key_bits_and_out_of_range(o, key_bits):
    import paper_1312_0138_amd as bs
    rng = np.random.default_rng(key_bits)
    n = 30_000
    keys = rng.integers(0, 1 << 64, size=n, dtype=np.uint64)  # bits above key_bits set: placed by low bits, stably
    got = bs.radix_sort_u64(_dev64(keys), key_bits).cpu().numpy().view(np.uint64)
    np.testing.assert_array_equal(got, o.bitwise_sort1_u64(keys, key_bits))
    assert bs.status().flags == (1 if key_bits < 64 else 0)


def test_u64_unaligned_input(o):
    """64-bit keys starting 8 bytes past a 16-byte boundary."""
    import paper_1312_0138_amd as bs
    rng = np.random.default_rng(77)
    keys = rng.integers(0, 1 << 64, size=20_001, dtype=np.uint64)
    view = _dev64(keys)[1:]
    assert view.data_ptr() % 16 != 0
    got = bs.radix_sort_u64(view, 64).cpu().numpy().view(np.uint64)
    np.testing.assert_array_equal(got, o.bitwise_sort1_u64(keys[1:], 64))


def test_u64_in_place_and_duplicates(o):
    import paper_1312_0138_amd as bs
    rng = np.random.default_rng(9)
    pool = rng.integers(0, 1 << 64, size=100, dtype=np.uint64)
    keys = pool[rng.integers(0, 100, size=50_001)]
    k = _dev64(keys)
    bs.radix_sort_u64(k, 64, out=k)
    np.testing.assert_array_equal(k.cpu().numpy().view(np.uint64), o.bitwise_sort1_u64(keys, 64))


@pytest.mark.parametrize("n,key_bits", [(1, 32), (8191, 32), (8192, 32), (8193, 32), (300_001, 32), (200_000, 20),
                                        (50_000, 9), (1 << 22, 32)])
def test_pairs(o, n, key_bits):
    import paper_1312_0138_amd as bs
    rng = np.random.default_rng(n + key_bits)
    keys = rng.integers(0, 1 << 32, size=n, dtype=np.uint64).astype(np.uint32)
    keys[::3] = keys[0]  # many equal keys: their values must keep input order
    vals = rng.permutation(n).astype(np.uint32)
    ok, ov = bs.radix_sort_pairs(to_dev(keys), to_dev(vals), key_bits)
    wk, wv = o.bitwise_sort1_pairs(keys, vals, key_bits)
    np.testing.assert_array_equal(to_np(ok), wk)
    np.testing.assert_array_equal(to_np(ov), wv)
    assert bs.status().flags == (1 if key_bits < 32 and int(keys.max()) >> key_bits else 0)


@pytest.mark.parametrize("key_bits", [16, 24])
def test_pairs_in_place(o, key_bits):
    import paper_1312_0138_amd as bs
    rng = np.random.default_rng(key_bits)
    keys = rng.integers(0, 1 << key_bits, size=70_000, dtype=np.uint64).astype(np.uint32)
    vals = np.arange(keys.size, dtype=np.uint32)
    k, v = to_dev(keys), to_dev(vals)
    bs.radix_sort_pairs(k, v, key_bits, out_keys=k, out_values=v)
    wk, wv = o.bitwise_sort1_pairs(keys, vals, key_bits)
    np.testing.assert_array_equal(to_np(k), wk)
    np.testing.assert_array_equal(to_np(v), wv)
