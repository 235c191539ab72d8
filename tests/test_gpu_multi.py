"""The pointer-array batch (bitsort_batch_ptr_u32): many arrays through the
plain path's kernels in one launch each, every array checked against the
oracle's bitmap sort."""
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


def _run(arrays, rbits, outs=None):
    import paper_1312_0138_amd as bs
    dev = [to_dev(a) for a in arrays]
    res = bs.sort_many(dev, rbits, outs=outs)
    flags, counts = bs.batch_status(len(arrays))
    return [to_np(r) for r in res], flags, counts


def _check(o, arrays, rbits):
    got, flags, counts = _run(arrays, rbits)
    for i, (a, rb) in enumerate(zip(arrays, rbits)):
        want, wflags, _ = o.bitmap_sort(a, rb)
        assert flags[i] == wflags and counts[i] == want.size, i
        np.testing.assert_array_equal(got[i][: want.size], want, err_msg=f"array {i} n={a.size} rb={rb}")


def test_mixed_widths(o):
    spec = [(0, 10), (1, 0), (2, 1), (31, 5), (1000, 12), (4096, 16), (4097, 20), (100_000, 21), (300_001, 24),
            (1 << 20, 26), (1 << 22, 28), (12_345, 32), (1 << 21, 32), (5, 3)]
    arrays = [inputs.distinct_uniform(n, rb, 100 + i) for i, (n, rb) in enumerate(spec)]
    _check(o, arrays, [rb for _, rb in spec])


def test_many_small_arrays(o):
    sizes = inputs.log_uniform_sizes(700, 1, 1 << 16, 3)
    rbits = [inputs.range_bits_for(int(n)) for n in sizes]
    arrays = [inputs.distinct_uniform(int(n), rb, inputs.segment_seed(3, i)) for i, (n, rb) in
              enumerate(zip(sizes, rbits))]
    _check(o, arrays, rbits)


def test_duplicates_and_out_of_range(o):
    rng = np.random.default_rng(5)
    a = rng.integers(0, 1 << 12, size=3000, dtype=np.uint64).astype(np.uint32)   # repeats
    b = rng.integers(0, 1 << 18, size=5000, dtype=np.uint64).astype(np.uint32)   # keys >= 2^16
    c = inputs.distinct_uniform(70_000, 20, 9)                                     # clean
    _check(o, [a, b, c], [12, 16, 20])


def test_in_place_and_same_as_plain(o):
    import torch
    import paper_1312_0138_amd as bs
    arrays = [inputs.distinct_uniform(n, rb, n) for n, rb in ((50_000, 18), (1 << 21, 27), (777, 11))]
    dev = [to_dev(a) for a in arrays]
    plain = [bs.sort(d, rb) for d, rb in zip(dev, (18, 27, 11))]
    bs.sort_many(dev, [18, 27, 11], outs=dev)
    for d, p in zip(dev, plain):
        assert torch.equal(d, p)


def test_wide_segments_match_batch_kernel():
    # the segmented batch kernel (ranges up to 2^24) and the pointer-array form agree
    import torch
    import paper_1312_0138_amd as bs
    keys, offsets, rbits = inputs.batch_segments(64, 1 << 10, 1 << 22, 11)
    k = to_dev(keys)
    off = torch.from_numpy(offsets.astype(np.int64)).cuda()
    rb = torch.from_numpy(rbits).cuda()
    ref = bs.sort_batch(k, off, rb)
    views = [k[int(offsets[i]):int(offsets[i + 1])] for i in range(64)]
    outs = bs.sort_many(views, [int(r) for r in rbits])
    assert torch.equal(torch.cat(outs), ref)


def test_bitvector_route(o):
    # arrays with R/8 <= 2n and R >= 2^21 emit through the HBM bit-vector;
    # they sit between LDS-emitting arrays so that the chunk search skips
    # arrays without chunks
    spec = [(1 << 17, 21), (3000, 14), ((1 << 20) + 77, 24), (1 << 21, 21), (0, 22), ((1 << 22) - 3, 24),
            (100_000, 23), ((1 << 19) + 1, 23), (9, 4)]
    arrays = [inputs.distinct_uniform(n, rb, 500 + i) for i, (n, rb) in enumerate(spec)]
    _check(o, arrays, [rb for _, rb in spec])


def test_bitvector_route_duplicates_and_range(o):
    rng = np.random.default_rng(8)
    a = rng.integers(0, 1 << 21, size=1 << 18, dtype=np.uint64).astype(np.uint32)   # repeats
    b = inputs.distinct_uniform(1 << 19, 23, 4)
    b[12345] = np.uint32(1 << 23) + 7                                                # out of range
    c = inputs.dense_permutation(22, 6)
    c[777] = c[778]                                                                  # one repeat
    _check(o, [a, b, c], [21, 23, 22])


def test_bitvector_route_in_place_and_same_as_plain():
    # out[a] == keys[a] on the bit-vector route, next to an LDS-emitting array
    import torch
    import paper_1312_0138_amd as bs
    spec = ((1 << 20, 22), ((1 << 21) + 5, 23), (40_000, 20))
    dev = [to_dev(inputs.distinct_uniform(n, rb, 31 + n)) for n, rb in spec]
    plain = [bs.sort(d, rb) for d, (_, rb) in zip(dev, spec)]
    bs.sort_many(dev, [rb for _, rb in spec], outs=dev)
    for d, p in zip(dev, plain):
        assert torch.equal(d, p)


def test_batch_workload_shape_matches_segmented_kernel():
    # sizes log-uniform in [256, 2^20], range the power of two >= 4n: enough
    # arrays that each takes a single slice unless it is on the bit-vector
    # route; the segmented kernel sorts the same segments
    import torch
    import paper_1312_0138_amd as bs
    keys, offsets, rbits = inputs.batch_segments(256, 256, 1 << 20, 21)
    k = to_dev(keys)
    off = torch.from_numpy(offsets.astype(np.int64)).cuda()
    ref = bs.sort_batch(k, off, torch.from_numpy(rbits).cuda())
    views = [k[int(offsets[i]):int(offsets[i + 1])] for i in range(256)]
    outs = bs.sort_many(views, [int(r) for r in rbits])
    flags, counts = bs.batch_status(256)
    assert not flags.any() and np.array_equal(counts, np.diff(offsets).astype(np.uint64))
    assert torch.equal(torch.cat(outs), ref)
