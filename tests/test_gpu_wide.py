"""Parity of the 64-bit-key bitmap path (bitsort_u64: ranges up to 2^36, cut
into groups of 2^32 keys, each sorted by the plain path's kernels) with the
oracle's 64-bit bitmap sort, element by element."""
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


def _dev64(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.uint64).view(np.int64).copy()).cuda()


def _run(keys, rb, out_init=None):
    import torch
    import paper_1312_0138_amd as bs
    k = _dev64(keys)
    out = _dev64(out_init) if out_init is not None else torch.empty_like(k)
    bs.sort_u64(k, rb, out)
    st = bs.status()
    return out.cpu().numpy().view(np.uint64), st


@pytest.mark.parametrize("n,rb", [(1, 0), (2, 1), (100, 7), (5000, 20), (300_000, 32), (300_000, 33),
                                  ((1 << 20) + 5, 36), (70_000, 34)])
def test_sizes(o, n, rb):
    keys = inputs.distinct_uniform_u64(n, rb, 40 + rb)
    want, flags = o.bitmap_sort_u64(keys, rb)
    assert flags == 0
    got, st = _run(keys, rb)
    assert st.flags == 0 and st.count == n
    np.testing.assert_array_equal(got, want)


def test_full_size_2_25_over_2_36(o):
    """2^25 distinct keys over [0, 2^36): 16 groups of 2^32 keys, each a
    sparse array of about 2^21 keys."""
    keys = inputs.distinct_uniform_u64(1 << 25, 36, 0x36)
    want, flags = o.bitmap_sort_u64(keys, 36)
    got, st = _run(keys, 36)
    assert st.flags == 0 and st.count == keys.size
    np.testing.assert_array_equal(got, want)


def test_dense_2_26_over_2_33(o):
    keys = inputs.distinct_uniform_u64(1 << 26, 33, 0x33)
    want, flags = o.bitmap_sort_u64(keys, 33)
    got, st = _run(keys, 33)
    assert st.flags == 0 and st.count == keys.size
    np.testing.assert_array_equal(got, want)


def test_group_boundaries_duplicates_and_range(o):
    edge = []
    for g in range(16):
        b = g << 32
        edge += [b, b + 1, b + 31, b + 32, b + (1 << 20) - 1, b + (1 << 20), b + (1 << 32) - 1]
    edge = np.array(edge, dtype=np.uint64)
    rng = np.random.default_rng(2)
    keys = np.concatenate([edge, inputs.distinct_uniform_u64(50_000, 36, 3)])
    keys = np.unique(keys)
    keys = keys[rng.permutation(keys.size)]
    want, flags = o.bitmap_sort_u64(keys, 36)
    got, st = _run(keys, 36)
    assert flags == 0 and st.flags == 0 and st.count == keys.size
    np.testing.assert_array_equal(got, want)
    # repeats and keys past 2^36 (and past 2^63)
    bad = keys.copy()
    bad[rng.choice(bad.size, 500, replace=False)] = keys[rng.integers(0, keys.size, 500)]
    bad[rng.choice(bad.size, 50, replace=False)] |= np.uint64(1 << 40)
    bad[0] = np.uint64(0xFFFFFFFFFFFFFFFF)
    want, flags = o.bitmap_sort_u64(bad, 36)
    assert flags == 3
    got, st = _run(bad, 36)
    assert st.flags == 3 and st.count == want.size
    np.testing.assert_array_equal(got[: want.size], want)


def test_in_place_and_all_out_of_range(o):
    import paper_1312_0138_amd as bs
    keys = inputs.distinct_uniform_u64(100_000, 35, 5)
    k = _dev64(keys)
    bs.sort_u64(k, 35, k)
    assert bs.status().count == keys.size
    np.testing.assert_array_equal(k.cpu().numpy().view(np.uint64), np.sort(keys))
    far = (keys | np.uint64(1 << 35))[:1000]
    got, st = _run(far, 35, out_init=np.full(1000, 7, dtype=np.uint64))
    assert st.flags == 1 and st.count == 0
    assert np.all(got == 7)
