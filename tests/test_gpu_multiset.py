"""Multiset sort by counting (bitsort_count_u32) against the oracle's
counting sort: repeats kept, out-of-range keys dropped and flagged."""
import numpy as np
import pytest

import oracle
from gpu_util import require_gpu, to_dev, to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


@pytest.fixture(scope="module")
def o():
    return oracle.default()


def _count(keys, rb):
    import paper_1312_0138_amd as bs
    out = bs.sort_multiset(to_dev(keys), rb)
    st = bs.status()
    return to_np(out), st


@pytest.mark.parametrize("rb,n", [(0, 10), (1, 1000), (5, 64), (10, 4096), (12, 4097), (16, 100_000), (20, 1_000_000),
                                  (24, 1 << 22), (27, 1 << 20), (27, 12_345), (12, 131_072), (14, 655_360)])
def test_random_repeats(o, rb, n):
    rng = np.random.default_rng(rb * 1000 + n)
    keys = rng.integers(0, 1 << rb, size=n, dtype=np.uint64).astype(np.uint32)
    got, st = _count(keys, rb)
    want, flags = o.counting_sort(keys, rb)
    assert st.flags == flags == 0 and st.count == want.size == n
    np.testing.assert_array_equal(got, want)


@pytest.mark.parametrize("distinct", [1, 2, 3, 64, 1000])
def test_heavy_repeats(o, distinct):
    rng = np.random.default_rng(distinct)
    pool = rng.choice(1 << 20, size=distinct, replace=False).astype(np.uint32)
    keys = pool[rng.integers(0, distinct, size=2_000_000)]
    got, st = _count(keys, 20)
    want, _ = o.counting_sort(keys, 20)
    assert st.count == want.size
    np.testing.assert_array_equal(got, want)


def test_out_of_range_dropped(o):
    rng = np.random.default_rng(3)
    keys = rng.integers(0, 1 << 18, size=300_000, dtype=np.uint64).astype(np.uint32)
    got, st = _count(keys, 16)
    want, flags = o.counting_sort(keys, 16)
    assert flags == 1 and st.flags == 1 and st.count == want.size
    np.testing.assert_array_equal(got[: want.size], want)


def test_distinct_keys_match_bitmap_sort():
    import torch
    import paper_1312_0138_amd as bs
    k = bs.generate(1 << 21, 24, 5)
    assert torch.equal(bs.sort_multiset(k, 24), bs.sort(k, 24))


def test_matches_radix_sort():
    import torch
    import paper_1312_0138_amd as bs
    rng = np.random.default_rng(8)
    keys = to_dev(rng.integers(0, 1 << 22, size=3_000_000, dtype=np.uint64).astype(np.uint32))
    assert torch.equal(bs.sort_multiset(keys, 22), bs.radix_sort(keys, 22))


def test_in_place_and_empty(o):
    import torch
    import paper_1312_0138_amd as bs
    rng = np.random.default_rng(4)
    keys = rng.integers(0, 1 << 14, size=50_000, dtype=np.uint64).astype(np.uint32)
    k = to_dev(keys)
    bs.sort_multiset(k, 14, out=k)
    np.testing.assert_array_equal(to_np(k), o.counting_sort(keys, 14)[0])
    e = torch.empty(0, dtype=torch.int32, device="cuda")
    assert bs.sort_multiset(e, 10).numel() == 0
