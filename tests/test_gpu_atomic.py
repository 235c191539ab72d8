"""Parity of the atomic-mark path (bitsort_u32_atomic: the bit-vector marked
in HBM with wave-combined atomic ORs, chunk counts, prefix, emission) with the
oracle, element by element."""
import numpy as np
import pytest

import oracle
from gpu_util import require_gpu, to_dev, to_np
from paper_1312_0138_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


@pytest.fixture(scope="module")
def o():
    return oracle.default()


def _run(keys_np, rb, out_init=None):
    import torch
    import paper_1312_0138_amd as bs
    k = to_dev(keys_np)
    out = to_dev(out_init) if out_init is not None else torch.empty_like(k)
    bs.sort_atomic(k, rb, out)
    st = bs.status()
    return to_np(out), st


@pytest.mark.parametrize("n,rb", [(1, 0), (2, 1), (33, 6), (700, 10), (5000, 16), (1 << 15, 15), (70_001, 20),
                                  ((1 << 20) + 3, 22)])
def test_sizes(o, n, rb):
    keys = inputs.distinct_uniform(n, rb, 31 + rb)
    want, _, _ = o.bitmap_sort(keys, rb)
    got, st = _run(keys, rb)
    assert st.flags == 0 and st.count == n
    np.testing.assert_array_equal(got, want)


@pytest.mark.parametrize("rep", [0, 1, 2])
def test_ten_to_the_six_keys(o, rep):
    keys = inputs.distinct_uniform(1_000_000, 24, inputs.config_seed(1, rep))
    want, _, _ = o.bitmap_sort(keys, 24)
    got, st = _run(keys, 24)
    assert st.flags == 0 and st.count == keys.size
    np.testing.assert_array_equal(got, want)


def test_full_size_2_26_over_2_28(o):
    keys = inputs.distinct_uniform(1 << 26, 28, inputs.config_seed(2, 0))
    want, _, _ = o.bitmap_sort(keys, 28)
    got, st = _run(keys, 28)
    assert st.flags == 0 and st.count == keys.size
    np.testing.assert_array_equal(got, want)


def test_sorted_and_runs_combine(o):
    """Ascending input: whole waves fall into a few words, so the lanes' masks
    combine before the atomic; blocks of consecutive keys in random order too."""
    keys = np.arange(1 << 20, dtype=np.uint32)
    got, st = _run(keys, 20)
    assert st.count == keys.size
    np.testing.assert_array_equal(got, keys)
    blocks = np.random.default_rng(3).permutation(1 << 12)
    keys2 = (blocks[:, None] * 64 + np.arange(64)[None, :]).astype(np.uint32).ravel()
    want, _, _ = o.bitmap_sort(keys2, 18)
    got, st = _run(keys2, 18)
    assert st.flags == 0 and st.count == keys2.size
    np.testing.assert_array_equal(got, want)


def test_duplicates_out_of_range_and_in_place(o):
    import paper_1312_0138_amd as bs
    base = inputs.distinct_uniform(200_000, 22, 8)
    rng = np.random.default_rng(9)
    keys = base.copy()
    keys[rng.choice(keys.size, 2000, replace=False)] = base[rng.integers(0, keys.size, 2000)]
    keys[rng.choice(keys.size, 100, replace=False)] |= np.uint32(1 << 30)
    want, flags, _ = o.bitmap_sort(keys, 22)
    assert flags == 3
    got, st = _run(keys, 22)
    assert st.flags == 3 and st.count == want.size
    np.testing.assert_array_equal(got[: want.size], want)
    k = to_dev(base)
    bs.sort_atomic(k, 22, k)
    assert bs.status().count == base.size
    np.testing.assert_array_equal(to_np(k), np.sort(base))


def test_bit_vector_stays_zero_between_calls(o):
    """Calls of different widths in a row on one stream: each starts from an
    all-zero bit-vector that the previous emission left behind."""
    for n, rb, seed in [(300_000, 24, 1), (1000, 12, 2), (300_000, 24, 3), (50_000, 17, 4), (1 << 21, 25, 5)]:
        keys = inputs.distinct_uniform(n, rb, seed)
        want, _, _ = o.bitmap_sort(keys, rb)
        got, st = _run(keys, rb)
        assert st.flags == 0 and st.count == n, (n, rb)
        np.testing.assert_array_equal(got, want)
