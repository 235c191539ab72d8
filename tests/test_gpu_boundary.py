"""The boundary's two-step batch (bitsort_batch_plan / bitsort_batch_run),
its capture into a HIP graph, and caller workspaces (bitsort_set_workspace),
all through the C ABI, against the oracle element by element."""
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


def _segments(count, seed, lo=1, hi=1 << 16):
    sizes = inputs.log_uniform_sizes(count, lo, hi, seed)
    rbits = np.array([inputs.range_bits_for(int(n)) for n in sizes], dtype=np.uint8)
    offsets = np.zeros(count + 1, dtype=np.uint64)
    offsets[1:] = np.cumsum(sizes)
    keys = np.concatenate([inputs.distinct_uniform(int(n), int(r), inputs.segment_seed(seed, i))
                           for i, (n, r) in enumerate(zip(sizes, rbits))]).astype(np.uint32)
    return keys, offsets, rbits


def test_batch_plan_and_run(o):
    import torch
    import paper_1312_0138_amd as bs
    keys, offsets, rbits = _segments(300, 77)
    keys[:3] = 0  # a duplicate in segment 0 when it has 3 keys or more
    want, n_out, flags = o.bitmap_sort_segments(keys, offsets, rbits)
    plan = bs.BatchPlan(offsets, rbits)
    k = to_dev(keys)
    off_d = torch.from_numpy(offsets.astype(np.int64)).cuda()
    rb_d = torch.from_numpy(rbits).cuda()
    out = torch.empty_like(k)
    plan.run(k, off_d, rb_d, out)
    f, c = plan.status()
    np.testing.assert_array_equal(c, n_out)
    assert np.array_equal(f != 0, flags != 0)
    got = to_np(out)
    for s in range(rbits.size):
        lo = int(offsets[s])
        np.testing.assert_array_equal(got[lo:lo + int(n_out[s])], want[lo:lo + int(n_out[s])], err_msg=f"segment {s}")
    # a second run of the same plan on other keys of the same shape
    keys2, _, _ = _segments(300, 78)
    keys2 = np.concatenate([inputs.distinct_uniform(int(offsets[s + 1] - offsets[s]), int(rbits[s]), 9000 + s)
                            for s in range(rbits.size)]).astype(np.uint32)
    want2, n2, _ = o.bitmap_sort_segments(keys2, offsets, rbits)
    k.copy_(to_dev(keys2))
    plan.run(k, off_d, rb_d, out)
    f, c = plan.status()
    assert not f.any()
    np.testing.assert_array_equal(c, n2)
    np.testing.assert_array_equal(to_np(out), want2)
    plan.close()


def test_batch_run_in_a_captured_graph(o):
    """bitsort_batch_run captured by torch into a HIP graph: every replay,
    with eager work and synchronisations in between, equals the eager run."""
    import torch
    import paper_1312_0138_amd as bs
    keys, offsets, rbits = _segments(200, 81, hi=1 << 18)
    want, n_out, _ = o.bitmap_sort_segments(keys, offsets, rbits)
    plan = bs.BatchPlan(offsets, rbits)
    k = to_dev(keys)
    off_d = torch.from_numpy(offsets.astype(np.int64)).cuda()
    rb_d = torch.from_numpy(rbits).cuda()
    out = torch.empty_like(k)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        plan.run(k, off_d, rb_d, out)  # warm-up outside the capture
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, capture_error_mode="thread_local"):
        plan.run(k, off_d, rb_d, out)
    for rep in range(4):
        out.fill_(-1)
        scratch = torch.arange(1 << 20, device="cuda", dtype=torch.int32).sum()  # eager work between replays
        g.replay()
        torch.cuda.synchronize()
        assert int(scratch) >= 0
        np.testing.assert_array_equal(to_np(out), want, err_msg=f"replay {rep}")
        f, c = plan.status()
        assert not f.any()
        np.testing.assert_array_equal(c, n_out)
    plan.close()


def test_caller_workspace(o):
    import torch
    import paper_1312_0138_amd as bs
    keys = inputs.distinct_uniform(600_000, 24, 5)
    want, _, _ = o.bitmap_sort(keys, 24)
    k = to_dev(keys)
    s = torch.cuda.Stream()
    need = bs.workspace_bytes(keys.size, 24)
    ws = torch.zeros(need, dtype=torch.uint8, device="cuda")
    with torch.cuda.stream(s):
        bs.set_workspace(ws, s)
        try:
            out = bs.sort(k, 24)
            st = bs.status(s)
            assert st.flags == 0 and st.count == keys.size
            np.testing.assert_array_equal(to_np(out), want)
            # a larger problem than the workspace holds: refused, nothing allocated
            big = to_dev(inputs.distinct_uniform(1 << 22, 26, 6))
            with pytest.raises(bs.BitsortError) as e:
                bs.sort(big, 26)
            assert e.value.code == bs._lib.BITSORT_ERR_NO_MEMORY
        finally:
            bs.set_workspace(None, s)
        out2 = bs.sort(k, 24)  # the library's own workspace again
        st = bs.status(s)
    assert st.count == keys.size
    np.testing.assert_array_equal(to_np(out2), want)
