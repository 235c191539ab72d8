"""Signed keys: the bitmap sort of distinct int32 keys (bitsort_i32) and the
radix sort of any int32 keys (bitsort_radix_i32) against the oracle's
version of the paper's BitwiseSort (negative keys first, each sign group
sorted by its low 31 bits)."""
import numpy as np
import pytest

import oracle
from gpu_util import require_gpu
from paper_1312_0138_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


@pytest.fixture(scope="module")
def o():
    return oracle.default()


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.int32).copy()).cuda()


def _signed_distinct(n, rb, seed):
    u = inputs.distinct_uniform(n, rb, seed).astype(np.int64)
    return (u - (1 << (rb - 1) if rb else 0)).astype(np.int32)


@pytest.mark.parametrize("rb,n", [(1, 2), (2, 3), (8, 200), (10, 1000), (16, 5000), (16, 40_000), (20, 8192),
                                  (20, 300_000), (24, 1_000_000), (28, 1 << 22), (32, 1 << 20), (32, 12_345)])
def test_bitmap_signed_matches_bitwise_sort(o, rb, n):
    import paper_1312_0138_amd as bs
    keys = _signed_distinct(n, rb, 1000 + rb + n)
    out = bs.sort_signed(_dev(keys), rb).cpu().numpy()
    np.testing.assert_array_equal(out, o.bitwise_sort_i32(keys))
    st = bs.status()
    assert st.flags == 0 and st.count == n


@pytest.mark.parametrize("emit_path", [1, 2])
def test_bitmap_signed_both_emit_paths(o, emit_path):
    import paper_1312_0138_amd as bs
    keys = _signed_distinct(1 << 21, 24, 77)
    try:
        bs.set_tuning(0, 0, emit_path)
        out = bs.sort_signed(_dev(keys), 24).cpu().numpy()
    finally:
        bs.set_tuning(0, 0, 0)
    np.testing.assert_array_equal(out, o.bitwise_sort_i32(keys))


def test_bitmap_signed_large_tiles(o):
    """Signed keys through the persistent partition (2^15-key tiles, several per workgroup)."""
    import paper_1312_0138_amd as bs
    keys = _signed_distinct((1 << 24) + 3, 28, 78)
    try:
        bs.set_tuning(0, 15, 0)
        out = bs.sort_signed(_dev(keys), 28).cpu().numpy()
    finally:
        bs.set_tuning(0, 0, 0)
    np.testing.assert_array_equal(out, o.bitwise_sort_i32(keys))


@pytest.mark.parametrize("rb,n", [(8, 250), (20, 100_000)])
def test_bitmap_signed_out_of_range_dropped(o, rb, n):
    import paper_1312_0138_amd as bs
    half = 1 << (rb - 1)
    rng = np.random.default_rng(rb)
    keys = rng.permutation(np.arange(-2 * half, 2 * half, dtype=np.int64))[:n].astype(np.int32)
    inside = keys[(keys >= -half) & (keys < half)]
    out = bs.sort_signed(_dev(keys), rb)
    st = bs.status()
    assert st.flags == 1 and st.count == inside.size
    np.testing.assert_array_equal(out.cpu().numpy()[: inside.size], o.bitwise_sort_i32(inside))


@pytest.mark.parametrize("n", [1, 64, 4097, 8192, 8193, 100_003, 1 << 22])
def test_radix_signed_matches_bitwise_sort(o, n):
    import paper_1312_0138_amd as bs
    rng = np.random.default_rng(n)
    keys = rng.integers(-(1 << 31), 1 << 31, size=n, dtype=np.int64).astype(np.int32)
    out = bs.radix_sort_signed(_dev(keys)).cpu().numpy()
    np.testing.assert_array_equal(out, o.bitwise_sort_i32(keys))
    st = bs.status()
    assert st.flags == 0 and st.count == n


def test_radix_signed_duplicates_and_extremes(o):
    import paper_1312_0138_amd as bs
    rng = np.random.default_rng(5)
    pool = np.array([-(1 << 31), -1, 0, 1, (1 << 31) - 1, -12345, 777], dtype=np.int32)
    keys = pool[rng.integers(0, pool.size, size=200_000)]
    out = bs.radix_sort_signed(_dev(keys)).cpu().numpy()
    np.testing.assert_array_equal(out, o.bitwise_sort_i32(keys))
    np.testing.assert_array_equal(out, np.sort(keys))


def test_signed_paths_agree_on_distinct_keys():
    import torch
    import paper_1312_0138_amd as bs
    keys = _dev(_signed_distinct(1 << 20, 32, 9))
    assert torch.equal(bs.sort_signed(keys, 32), bs.radix_sort_signed(keys))
