"""Parity of the segmented batch path (bitsort_batch_u32) with the oracle."""
import os

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


def _run_batch(keys, offsets, rbits):
    import torch
    import paper_1312_0138_amd as bs
    k = to_dev(keys)
    off = torch.from_numpy(offsets.astype(np.int64)).cuda()
    rb = torch.from_numpy(rbits.astype(np.uint8)).cuda()
    out = torch.full_like(k, -1)
    bs.sort_batch(k, off, rb, out)
    flags, counts = bs.batch_status(rbits.size)
    return to_np(out), flags, counts


def _check(o, keys, offsets, rbits):
    want, n_out, wflags = o.bitmap_sort_segments(keys, offsets, rbits)
    got, flags, counts = _run_batch(keys, offsets, rbits)
    np.testing.assert_array_equal(counts, n_out)
    np.testing.assert_array_equal(flags, wflags)
    for s in range(rbits.size):
        lo, d = int(offsets[s]), int(n_out[s])
        np.testing.assert_array_equal(got[lo:lo + d], want[lo:lo + d], err_msg=f"segment {s}")


def test_small_segments(o):
    keys, offsets, rbits = inputs.batch_segments(300, 1, 5000, seed=21)
    _check(o, keys, offsets, rbits)


def test_multi_slice_segments(o):
    """Ranges above one LDS slice (2^21 .. 2^24 bits) split into slices."""
    sizes = [300_000, 1 << 19, 1 << 20, 5, 0, 4_000_000, 123_457]
    rbits = np.array([21, 21, 22, 3, 7, 24, 23], dtype=np.uint8)
    parts = [inputs.distinct_uniform(n, int(rb), 900 + i) for i, (n, rb) in enumerate(zip(sizes, rbits))]
    keys = np.concatenate(parts)
    offsets = np.concatenate([[0], np.cumsum(sizes)]).astype(np.uint64)
    _check(o, keys, offsets, rbits)


def test_empty_and_tiny(o):
    sizes = [0, 1, 0, 2, 1, 0]
    rbits = np.array([0, 0, 5, 1, 20, 24], dtype=np.uint8)
    parts = [inputs.distinct_uniform(n, int(rb), 31 + i) for i, (n, rb) in enumerate(zip(sizes, rbits))]
    keys = np.concatenate(parts).astype(np.uint32)
    offsets = np.concatenate([[0], np.cumsum(sizes)]).astype(np.uint64)
    _check(o, keys, offsets, rbits)


def test_out_of_range_and_bad_segment(o):
    import torch
    import paper_1312_0138_amd as bs
    sizes = [100, 50, 70]
    keys = np.concatenate([inputs.distinct_uniform(100, 8, 1), inputs.distinct_uniform(50, 6, 2),
                           inputs.distinct_uniform(70, 10, 3)])
    rbits = np.array([7, 6, 25], dtype=np.uint8)  # segment 0 has keys >= 2^7; segment 2 is over the limit
    offsets = np.concatenate([[0], np.cumsum(sizes)]).astype(np.uint64)
    k = to_dev(keys)
    out = torch.full_like(k, -1)
    bs.sort_batch(k, torch.from_numpy(offsets.astype(np.int64)).cuda(), torch.from_numpy(rbits).cuda(), out)
    flags, counts = bs.batch_status(3)
    want0, f0, _ = o.bitmap_sort(keys[:100], 7)
    assert flags[0] == bs.STATUS_OUT_OF_RANGE and f0 == oracle.FLAG_OUT_OF_RANGE
    assert counts[0] == want0.size
    np.testing.assert_array_equal(to_np(out)[: want0.size], want0)
    assert flags[1] == 0 and counts[1] == 50
    assert flags[2] == bs.STATUS_BAD_SEGMENT and counts[2] == 0


def test_batch_workload_every_segment(o):
    """4096 segments, sizes log-uniform in [256, 2^20], range 4n rounded up to
    a power of two: the full batch runs on the GPU, and every segment is
    regenerated on the host and checked element by element against the
    oracle's sort of it (its input as well)."""
    from concurrent.futures import ThreadPoolExecutor

    import torch
    import paper_1312_0138_amd as bs
    count, seed = 4096, inputs.config_seed(4, 0)
    sizes = inputs.log_uniform_sizes(count, 256, 1 << 20, seed)
    rbits = np.array([inputs.range_bits_for(n) for n in sizes], dtype=np.uint8)
    offsets = np.zeros(count + 1, dtype=np.uint64)
    offsets[1:] = np.cumsum(sizes)
    total = int(offsets[-1])
    k = torch.empty(total, dtype=torch.int32, device="cuda")
    for i in range(count):  # the device generator fills the batch; the host re-makes every segment
        lo, hi = int(offsets[i]), int(offsets[i + 1])
        bs.generate(hi - lo, int(rbits[i]), inputs.segment_seed(seed, i), out=k[lo:hi])
    out = torch.empty_like(k)
    bs.sort_batch(k, torch.from_numpy(offsets.astype(np.int64)).cuda(), torch.from_numpy(rbits).cuda(), out)
    flags, counts = bs.batch_status(count)
    assert not flags.any()
    np.testing.assert_array_equal(counts, sizes.astype(np.uint64))
    keys_all, got_all = to_np(k), to_np(out)

    def check(i):
        lo, hi = int(offsets[i]), int(offsets[i + 1])
        host_keys = inputs.distinct_uniform(hi - lo, int(rbits[i]), inputs.segment_seed(seed, i))
        want, _, _ = o.bitmap_sort(host_keys, int(rbits[i]))
        return (np.array_equal(keys_all[lo:hi], host_keys), np.array_equal(got_all[lo:hi], want))

    with ThreadPoolExecutor(max_workers=min(16, os.cpu_count() or 1)) as ex:
        res = list(ex.map(check, range(count)))
    bad_in = [i for i, (a, _) in enumerate(res) if not a]
    bad_out = [i for i, (_, b) in enumerate(res) if not b]
    assert not bad_in, f"device-generated input differs from the host's in segments {bad_in[:10]}"
    assert not bad_out, f"{len(bad_out)} segments differ from the oracle, first {bad_out[:10]}"