"""bitsort_u32_noalloc, the entry point for callers that cannot allocate,
called through the C ABI: on consecutive calls (each smaller than the one
before, so stale contents of the shared device array would show) its output
and status equal bitsort_u32's on the same keys, element by element, and the
oracle's sort."""
import numpy as np
import pytest

import oracle
from gpu_util import require_gpu, to_dev, to_np
from paper_1312_0138_amd import _lib, inputs

pytestmark = pytest.mark.gpu


def _noalloc(keys_t, rb, out_t, status_t):
    import torch
    return _lib.bitsort_u32_noalloc(keys_t.data_ptr(), keys_t.numel(), rb, out_t.data_ptr(),
                                    0 if status_t is None else status_t.data_ptr(),
                                    int(torch.cuda.current_stream().cuda_stream))


def _status(st):
    v = st.cpu().numpy().view(np.uint64)
    return int(v[0]) & 0xFFFFFFFF, int(v[1])


def test_noalloc_equals_plain_on_shrinking_calls():
    require_gpu()
    import torch

    import paper_1312_0138_amd as bs
    o = oracle.default()
    st = torch.full((2,), -1, dtype=torch.int64, device="cuda")
    # HBM bit-vector emission, LDS emission (the 10^6-key workload), a
    # single-workgroup problem, then an empty call
    cases = ((1 << 22, 24), (1_000_000, 24), (300_001, 21), (5000, 16), (0, 10))
    for i, (n, rb) in enumerate(cases):
        print(f"noalloc case {i}: n={n} range_bits={rb}", flush=True)
        assert _lib.bitsort_workspace_bytes(max(n, 1), rb) <= _lib.NOALLOC_SCRATCH_BYTES
        keys = inputs.distinct_uniform(n, rb, inputs.config_seed(1, 40 + i))
        k = to_dev(keys) if n else torch.empty(0, dtype=torch.int32, device="cuda")
        want_t = bs.sort(k, rb) if n else k.clone()
        got = torch.full_like(k, -1)
        assert _noalloc(k, rb, got, st) == _lib.BITSORT_OK
        torch.cuda.synchronize()
        assert torch.equal(got, want_t), f"case {i}: differs from bitsort_u32"
        flags, count = _status(st)
        assert (flags, count) == (0, n), f"case {i}: status {flags}, {count}"
        want, wflags, _ = o.bitmap_sort(keys, rb)
        assert wflags == 0
        np.testing.assert_array_equal(to_np(got), want)


def test_noalloc_duplicates_and_null_status():
    require_gpu()
    import torch
    o = oracle.default()
    keys = inputs.distinct_uniform(200_000, 22, 77)
    keys[1000:1100] = keys[:100]  # 100 repeats
    k = to_dev(keys)
    got = torch.full_like(k, -1)
    st = torch.full((2,), -1, dtype=torch.int64, device="cuda")
    assert _noalloc(k, 22, got, st) == _lib.BITSORT_OK
    want, wflags, _ = o.bitmap_sort(keys, 22)
    d = want.size
    flags, count = _status(st)
    assert flags == _lib.STATUS_DUPLICATE and wflags == oracle.FLAG_DUPLICATE and count == d
    np.testing.assert_array_equal(to_np(got)[:d], want[:d])
    got2 = torch.full_like(k, -1)
    assert _noalloc(k, 22, got2, None) == _lib.BITSORT_OK  # status discarded
    torch.cuda.synchronize()
    np.testing.assert_array_equal(to_np(got2)[:d], want[:d])
