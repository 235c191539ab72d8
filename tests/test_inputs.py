"""The seeded input generators: bijectivity of the keyed permutation,
distinctness and range of the keys, and the shapes of the size and arrival
generators."""
import numpy as np
import pytest

from paper_1312_0138_amd import inputs


@pytest.mark.parametrize("bits", list(range(0, 17)))
def test_keyed_permutation_is_a_bijection(bits):
    for seed in (0, 1, 0x13120138):
        y = inputs.keyed_permutation(np.arange(1 << bits, dtype=np.uint64), bits, seed)
        assert y.dtype == np.uint32
        assert np.array_equal(np.sort(y), np.arange(1 << bits, dtype=np.uint32))


def test_keyed_permutation_depends_on_seed_and_mixes():
    a = inputs.keyed_permutation(np.arange(1 << 12), 12, 1)
    b = inputs.keyed_permutation(np.arange(1 << 12), 12, 2)
    assert not np.array_equal(a, b)
    assert not np.array_equal(a, np.arange(1 << 12))
    # no long identity runs: fewer than 1% fixed points
    assert np.count_nonzero(a == np.arange(1 << 12)) < 41


@pytest.mark.parametrize("bits", [17, 23, 32])
def test_distinct_uniform_large_ranges(bits):
    k = inputs.distinct_uniform(50_000, bits, 7)
    assert k.size == 50_000 and np.unique(k).size == 50_000
    assert int(k.max()) < (1 << bits)
    # roughly uniform over the range: each eighth holds about an eighth of the keys
    hist = np.bincount((k.astype(np.uint64) >> np.uint64(bits - 3)).astype(np.int64), minlength=8)
    assert hist.min() > 50_000 / 8 * 0.9


def test_distinct_uniform_rejects_overfull():
    with pytest.raises(ValueError):
        inputs.distinct_uniform(9, 3, 0)


def test_sizes_ranges_and_arrivals():
    s = inputs.log_uniform_sizes(10_000, 1 << 10, 1 << 24, 5)
    assert s.min() >= 1 << 10 and s.max() <= 1 << 24
    # log-uniform: the median is near the geometric mean 2^17
    assert 2 ** 16.5 < np.median(s) < 2 ** 17.5
    assert inputs.range_bits_for(1) == 2 and inputs.range_bits_for(1000) == 12
    assert inputs.range_bits_for(1 << 20) == 22
    t = inputs.poisson_arrivals(10_000, 1000.0, 3)
    assert np.all(np.diff(t) > 0)
    assert abs(t[-1] - 10.0) < 0.5


@pytest.mark.parametrize("bits", [1, 9, 16])
def test_distinct_uniform_u64_is_a_bijection_on_small_ranges(bits):
    k = inputs.distinct_uniform_u64(1 << bits, bits, 11)
    assert k.dtype == np.uint64
    assert np.array_equal(np.sort(k), np.arange(1 << bits, dtype=np.uint64))


@pytest.mark.parametrize("bits", [33, 36, 48])
def test_distinct_uniform_u64_wide_ranges(bits):
    k = inputs.distinct_uniform_u64(60_000, bits, 12)
    assert np.unique(k).size == 60_000 and int(k.max()) < (1 << bits)
    hist = np.bincount((k >> np.uint64(bits - 3)).astype(np.int64), minlength=8)
    assert hist.min() > 60_000 / 8 * 0.9
