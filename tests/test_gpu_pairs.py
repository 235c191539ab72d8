"""Parity of the bitmap sort of (key, value) records (bitsort_pairs_u32) with
the oracle's Algorithm 1 on the same records over range_bits bit passes,
element by element.

With distinct keys the ascending arrangement of the records is unique
(Theorem 1), so every value must land beside its key.  Repeated keys keep one
of their values: those cases check the keys and flags against the oracle's
bitmap sort and each value against the set of values its key came with.

Two routes: the records route (records staged by slice, gathered with the
slice's bit-vector and placed by rank; a slice with more records than LDS
holds gathers them again and writes straight to HBM) for more than 8192 keys
at a density above 1/256, and the table route (a value table indexed by key)
for smaller or sparser inputs.  Each case states the route it takes, checked through the library's
kernel timings.
"""
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


RECORDS, TABLE = "k_slice_kv", "k_pairs_scatter"


def _pairs(keys, values, rb, route=None, **kw):
    """Sort on the device; with `route`, also check that the kernel naming
    that route ran."""
    import paper_1312_0138_amd as bs
    from paper_1312_0138_amd import _lib
    k, v = to_dev(keys), to_dev(values)
    _lib.check(_lib.bitsort_profile_reset(), "profile_reset")
    _lib.check(_lib.bitsort_profile_enable(True), "profile_enable")
    try:
        ok, ov = bs.sort_pairs(k, v, rb, **kw)
        st = bs.status()
    finally:
        _lib.check(_lib.bitsort_profile_enable(False), "profile_enable")
    rc, prof = _lib.bitsort_profile_read()
    _lib.check(rc, "profile_read")
    if route is not None and keys.size:
        assert route in prof, sorted(prof)
        assert ({RECORDS, TABLE} - {route}).isdisjoint(prof), sorted(prof)
    return to_np(ok), to_np(ov), st


# table route: one workgroup, sparse ranges (a 4 GiB table at 2^30, touched
# only where keys fall); records route: 2^18- to 2^14-bit slices, 2^12-,
# 2^14- and 2^15-key tiles, ragged tails, 16- and 64-key gather units, and a
# density of 1/128 at 2^29 and 2^30 (2048 and 4096 slices of 2^18 bits, about
# 2048 records each; the second with 8-record segments, on the register route)
@pytest.mark.parametrize("n,rb,route", [(1, 8, TABLE), (1000, 12, TABLE), (4097, 16, TABLE), (1000, 30, TABLE),
                                        (1_000_000, 30, TABLE), (2_000_000, 28, RECORDS), (100_003, 20, RECORDS),
                                        (1_000_000, 24, RECORDS), (3_000_000, 23, RECORDS), (3_000_001, 22, RECORDS),
                                        (5_000_000, 24, RECORDS), (4_200_000, 29, RECORDS), (8_400_000, 30, RECORDS)])
def test_distinct_keys(o, n, rb, route):
    keys = inputs.distinct_uniform(n, rb, 900 + rb)
    vals = np.random.default_rng(n).integers(0, 1 << 32, size=n, dtype=np.uint64).astype(np.uint32)
    got_k, got_v, st = _pairs(keys, vals, rb, route)
    want_k, want_v = o.bitwise_sort1_pairs(keys, vals, rb)
    assert st.flags == 0 and st.count == n
    np.testing.assert_array_equal(got_k, want_k)
    np.testing.assert_array_equal(got_v, want_v)


@pytest.mark.parametrize("path", [1, 2, 3, 4])
def test_table_route_over_every_emission_path(o, path):
    """Sparse records (about 2^-9 of the range) through the table route, with
    the plain sort's emission path forced each way in turn."""
    import paper_1312_0138_amd as bs
    rb, n = 28, 500_000
    keys = inputs.distinct_uniform(n, rb, 31 + path)
    vals = np.arange(n, dtype=np.uint32)[::-1].copy()
    want_k, want_v = o.bitwise_sort1_pairs(keys, vals, rb)
    bs.set_tuning(0, 0, path)
    try:
        got_k, got_v, st = _pairs(keys, vals, rb, TABLE)
    finally:
        bs.set_tuning(0, 0, 0)
    assert st.flags == 0 and st.count == n
    np.testing.assert_array_equal(got_k, want_k)
    np.testing.assert_array_equal(got_v, want_v)


@pytest.mark.parametrize("rb,n", [(22, 700_001), (28, 300_000)])  # records, table route
def test_in_place(o, rb, n):
    import paper_1312_0138_amd as bs
    keys = inputs.distinct_uniform(n, rb, 5)
    vals = (keys.astype(np.uint64) * 2654435761 % (1 << 32)).astype(np.uint32)
    k, v = to_dev(keys), to_dev(vals)
    ok, ov = bs.sort_pairs(k, v, rb, out_keys=k, out_values=v)
    assert ok.data_ptr() == k.data_ptr() and ov.data_ptr() == v.data_ptr()
    want_k, want_v = o.bitwise_sort1_pairs(keys, vals, rb)
    np.testing.assert_array_equal(to_np(k), want_k)
    np.testing.assert_array_equal(to_np(v), want_v)


@pytest.mark.parametrize("rb,n,route", [(12, 3000, TABLE), (24, 900_000, RECORDS), (22, 3_000_000, RECORDS)])
def test_repeated_and_out_of_range_keys(o, rb, n, route):
    """Flags and the compacted keys (and values) as the oracle's bitmap sort
    gives them; each value one of those its key arrived with."""
    import paper_1312_0138_amd as bs
    rng = np.random.default_rng(rb)
    base = inputs.distinct_uniform(n, rb, 70 + rb)
    dup = rng.choice(base, size=n // 10, replace=False)
    bad = ((1 << rb) + rng.integers(0, 1 << 8, size=37)).astype(np.uint32)
    keys = np.concatenate([base, dup, bad])
    keys = keys[rng.permutation(keys.size)]
    vals = rng.integers(0, 1 << 32, size=keys.size, dtype=np.uint64).astype(np.uint32)
    got_k, got_v, st = _pairs(keys, vals, rb, route)
    want_k, _, _ = o.bitmap_sort(keys, rb)
    assert st.flags == (bs.STATUS_OUT_OF_RANGE | bs.STATUS_DUPLICATE)
    assert st.count == want_k.size
    m = want_k.size
    np.testing.assert_array_equal(got_k[:m], want_k)
    # the values each key arrived with, as sorted (key, value) records
    order = np.lexsort((vals, keys))
    rk, rv = keys[order], vals[order]
    lo = np.searchsorted(rk, got_k[:m], side="left")
    hi = np.searchsorted(rk, got_k[:m], side="right")
    assert np.all(hi > lo)
    ok = np.array([got_v[j] in rv[lo[j]:hi[j]] for j in np.nonzero(hi - lo > 1)[0]], dtype=bool)
    assert ok.all()
    single = hi - lo == 1
    np.testing.assert_array_equal(got_v[:m][single], rv[lo[single]])


def test_headline_size_values_follow_keys(o):
    """2^26 distinct keys below 2^28 (the uniform workload's shape) with
    values a bijection of the keys: the keys as the oracle's bitmap sort
    gives them and every value equal to its key's image."""
    import paper_1312_0138_amd as bs
    rb, n = 28, 1 << 26
    keys = inputs.distinct_uniform(n, rb, inputs.config_seed(1, 0))
    img = lambda k: ((k.astype(np.uint64) * 0x9E3779B1) % (1 << 32)).astype(np.uint32) ^ np.uint32(0x5bd1e995)
    got_k, got_v, st = _pairs(keys, img(keys), rb, RECORDS)
    want_k, _, _ = o.bitmap_sort(keys, rb)
    assert st.flags == 0 and st.count == n
    np.testing.assert_array_equal(got_k, want_k)
    np.testing.assert_array_equal(got_v, img(want_k))


def test_empty_and_reuse(o):
    """n = 0 leaves the outputs alone and reads back an empty status; the next
    call on the same stream, smaller than an earlier one, is exact."""
    import torch
    import paper_1312_0138_amd as bs
    e = torch.empty(0, dtype=torch.int32, device="cuda")
    ok, ov = bs.sort_pairs(e, e.clone(), 20)
    st = bs.status()
    assert ok.numel() == 0 and ov.numel() == 0 and st.flags == 0 and st.count == 0
    for n, rb, route in ((200_000, 26, TABLE), (2_000_000, 22, RECORDS), (300_000, 20, RECORDS), (5000, 14, TABLE)):
        keys = inputs.distinct_uniform(n, rb, n)
        vals = np.arange(n, dtype=np.uint32)
        got_k, got_v, st = _pairs(keys, vals, rb, route)
        want_k, want_v = o.bitwise_sort1_pairs(keys, vals, rb)
        assert st.flags == 0 and st.count == n
        np.testing.assert_array_equal(got_k, want_k)
        np.testing.assert_array_equal(got_v, want_v)


def test_caller_workspace_too_small_is_an_error():
    """With a caller workspace that holds the plain sort but not the value
    table, the call returns BITSORT_ERR_NO_MEMORY and allocates nothing."""
    import torch
    import paper_1312_0138_amd as bs
    from paper_1312_0138_amd import _lib
    n, rb = 100_000, 24
    ws = torch.empty(bs.workspace_bytes(n, rb), dtype=torch.uint8, device="cuda")
    keys = to_dev(inputs.distinct_uniform(n, rb, 3))
    vals = to_dev(np.arange(n, dtype=np.uint32))
    ok, ov = torch.empty_like(keys), torch.empty_like(vals)
    s = torch.cuda.current_stream().cuda_stream
    assert _lib.bitsort_set_workspace(ws.data_ptr(), ws.numel(), s) == _lib.BITSORT_OK
    try:
        rc = _lib.bitsort_pairs_u32(keys.data_ptr(), vals.data_ptr(), n, rb, ok.data_ptr(), ov.data_ptr(), s)
        assert rc == _lib.BITSORT_ERR_NO_MEMORY
    finally:
        assert _lib.bitsort_set_workspace(0, 0, s) == _lib.BITSORT_OK


def test_slices_past_the_window(o):
    """Three slices holding more records than LDS has room for (2^16-bit
    slices at this density, room for 18,396 records) gather them again and
    write values and keys straight to HBM; the rest go through LDS."""
    rb, sb = 24, 16
    rng = np.random.default_rng(44)
    bg = inputs.distinct_uniform(3_000_000, rb, 45).astype(np.uint64)
    heavy = np.array([3, 100, 255], dtype=np.uint64)
    bg = bg[~np.isin(bg >> np.uint64(sb), heavy)]
    parts = [bg] + [(h << np.uint64(sb)) + rng.choice(1 << sb, size=c, replace=False).astype(np.uint64)
                    for h, c in zip(heavy, (40_000, 65_536, 50_000))]
    keys = np.concatenate(parts).astype(np.uint32)
    keys = keys[rng.permutation(keys.size)]
    assert 1 << 21 < keys.size <= 1 << 22  # 2^16-bit slices at range 2^24
    vals = rng.integers(0, 1 << 32, size=keys.size, dtype=np.uint64).astype(np.uint32)
    got_k, got_v, st = _pairs(keys, vals, rb, RECORDS)
    want_k, want_v = o.bitwise_sort1_pairs(keys, vals, rb)
    assert st.flags == 0 and st.count == keys.size
    np.testing.assert_array_equal(got_k, want_k)
    np.testing.assert_array_equal(got_v, want_v)


@pytest.mark.parametrize("rb,n,route", [(24, 1_000_003, RECORDS), (28, 300_001, TABLE)])
def test_unaligned_arrays(o, rb, n, route):
    """Keys and values starting 4 bytes past a 16-byte boundary (the
    partition's element-wise loads), outputs likewise."""
    import torch
    import paper_1312_0138_amd as bs
    keys = inputs.distinct_uniform(n, rb, 8)
    vals = np.arange(n, dtype=np.uint32) * np.uint32(3)
    k = to_dev(np.concatenate([[0], keys]).astype(np.uint32))[1:]
    v = to_dev(np.concatenate([[0], vals]).astype(np.uint32))[1:]
    ok = torch.empty(n + 1, dtype=torch.int32, device="cuda")[1:]
    ov = torch.empty(n + 1, dtype=torch.int32, device="cuda")[1:]
    assert k.data_ptr() % 16 and v.data_ptr() % 16 and ok.data_ptr() % 16
    bs.sort_pairs(k, v, rb, out_keys=ok, out_values=ov)
    st = bs.status()
    want_k, want_v = o.bitwise_sort1_pairs(keys, vals, rb)
    assert st.flags == 0 and st.count == n
    np.testing.assert_array_equal(to_np(ok), want_k)
    np.testing.assert_array_equal(to_np(ov), want_v)


def _dense_slice(keys_bg, rb, sb, slice_id, count, seed):
    """keys_bg without slice `slice_id`'s keys, plus `count` distinct keys of it."""
    k = keys_bg.astype(np.uint64)
    k = k[(k >> np.uint64(sb)) != np.uint64(slice_id)]
    rng = np.random.default_rng(seed)
    extra = (np.uint64(slice_id) << np.uint64(sb)) + rng.choice(1 << sb, size=count, replace=False).astype(np.uint64)
    out = np.concatenate([k, extra]).astype(np.uint32)
    return out[rng.permutation(out.size)]


# 4096 slices of 2^15 bits over 2^27 and 2^15-record tiles: a tile holds
# about 8 records of a slice, and each tile's first 16 are gathered into
# registers.  Slice 7 at 1.5 times the density leaves a few hundred records
# past their tile's 16th (kept in LDS beside the windows); slice 9 at 2.2
# times leaves thousands, more than that area keeps (the slice takes the
# general walk, its records in LDS); slice 11 at 3 times holds more records
# than LDS (the second gather).  The ragged case is compared with the
# oracle's Algorithm 1 on the records; the others, at the same size, with its
# bitmap sort for the keys and with values that are a bijection of the keys.
def _img(k):
    return ((k.astype(np.uint64) * 0x9E3779B1) % (1 << 32)).astype(np.uint32) ^ np.uint32(0x2545F491)


@pytest.mark.parametrize("case", ["ragged", "uniform", "spill", "general", "regather"])
def test_register_route(o, case):
    rb, sb = 27, 15
    n = (1 << 25) - {"ragged": 12345, "uniform": 0}.get(case, 60_000)  # room for the dense slices
    keys = inputs.distinct_uniform(n, rb, 61)
    dense = {"spill": [(7, 12288)], "general": [(7, 12288), (9, 18000)], "regather": [(9, 18000), (11, 24576)]}
    for slice_id, count in dense.get(case, []):
        keys = _dense_slice(keys, rb, sb, slice_id, count, 62 + slice_id)
    assert (1 << 24) < keys.size <= (1 << 25)
    if case == "ragged":
        vals = np.random.default_rng(64).integers(0, 1 << 32, size=keys.size, dtype=np.uint64).astype(np.uint32)
        got_k, got_v, st = _pairs(keys, vals, rb, RECORDS)
        want_k, want_v = o.bitwise_sort1_pairs(keys, vals, rb)
    else:
        got_k, got_v, st = _pairs(keys, _img(keys), rb, RECORDS)
        want_k, _, _ = o.bitmap_sort(keys, rb)
        want_v = _img(want_k)
    assert st.flags == 0 and st.count == keys.size
    np.testing.assert_array_equal(got_k, want_k)
    np.testing.assert_array_equal(got_v, want_v)


def test_register_route_repeated_and_out_of_range_keys(o):
    """The register route with repeated keys (their records share a rank) and
    keys past the range: flags, compacted keys as the oracle's bitmap sort,
    and each value one its key arrived with."""
    import paper_1312_0138_amd as bs
    rb = 27
    rng = np.random.default_rng(65)
    base = inputs.distinct_uniform((1 << 25) - 300_000, rb, 66)
    dup = rng.choice(base, size=250_000, replace=False)
    bad = ((1 << rb) + rng.integers(0, 1 << 10, size=500)).astype(np.uint32)
    keys = np.concatenate([base, dup, bad])
    keys = keys[rng.permutation(keys.size)]
    vals = rng.integers(0, 1 << 32, size=keys.size, dtype=np.uint64).astype(np.uint32)
    got_k, got_v, st = _pairs(keys, vals, rb, RECORDS)
    want_k, _, _ = o.bitmap_sort(keys, rb)
    assert st.flags == (bs.STATUS_OUT_OF_RANGE | bs.STATUS_DUPLICATE)
    m = want_k.size
    assert st.count == m
    np.testing.assert_array_equal(got_k[:m], want_k)
    order = np.lexsort((vals, keys))
    rk, rv = keys[order], vals[order]
    lo = np.searchsorted(rk, got_k[:m], side="left")
    hi = np.searchsorted(rk, got_k[:m], side="right")
    single = hi - lo == 1
    np.testing.assert_array_equal(got_v[:m][single], rv[lo[single]])
    multi = np.nonzero(~single)[0]
    assert multi.size > 1000
    assert all(got_v[j] in rv[lo[j]:hi[j]] for j in multi)


@pytest.mark.parametrize("n,rb,route", [(1_000_000, 24, RECORDS), (300_000, 28, TABLE)])
def test_side_stream_and_caller_workspace(o, n, rb, route):
    """On a side stream, first in the library's own workspace, then in a
    caller workspace large enough for the route (records: about 8n bytes and
    the tile table; table: the plain workspace and 4 * 2^range_bits bytes):
    both exact, statuses read on that stream."""
    import torch
    import paper_1312_0138_amd as bs
    keys = inputs.distinct_uniform(n, rb, 17)
    vals = np.random.default_rng(18).integers(0, 1 << 32, size=n, dtype=np.uint64).astype(np.uint32)
    want_k, want_v = o.bitwise_sort1_pairs(keys, vals, rb)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        k, v = to_dev(keys), to_dev(vals)
        ok, ov = bs.sort_pairs(k, v, rb, stream=s)
        st = bs.status(s)
        assert st.flags == 0 and st.count == n
        np.testing.assert_array_equal(to_np(ok), want_k)
        np.testing.assert_array_equal(to_np(ov), want_v)
        ws = torch.empty(16 * n + (4 << rb) + (64 << 20), dtype=torch.uint8, device="cuda")
        bs.set_workspace(ws, stream=s)
        try:
            ok2, ov2 = bs.sort_pairs(k, v, rb, stream=s)
            st = bs.status(s)
        finally:
            bs.set_workspace(None, stream=s)
        assert st.flags == 0 and st.count == n
        np.testing.assert_array_equal(to_np(ok2), want_k)
        np.testing.assert_array_equal(to_np(ov2), want_v)


@pytest.mark.parametrize("n,rb,route", [(1_000_000, 24, RECORDS), (300_000, 28, TABLE)])
def test_captured_graph_replays(o, n, rb, route):
    """bitsort_pairs_u32 captured by torch into a HIP graph on a stream whose
    workspace an eager call grew first: four replays over two inputs, with
    eager work and synchronisations between them, each equal to the oracle."""
    import torch
    import paper_1312_0138_amd as bs
    ka = inputs.distinct_uniform(n, rb, 23)
    kb = inputs.distinct_uniform(n, rb, 24)
    vals = np.random.default_rng(25).integers(0, 1 << 32, size=n, dtype=np.uint64).astype(np.uint32)
    wants = [o.bitwise_sort1_pairs(ka, vals, rb), o.bitwise_sort1_pairs(kb, vals, rb)]
    k, v = to_dev(ka), to_dev(vals)
    ok, ov = torch.empty_like(k), torch.empty_like(v)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        bs.sort_pairs(k, v, rb, out_keys=ok, out_values=ov, stream=s)  # warm-up outside the capture
    s.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s, capture_error_mode="thread_local"):
        bs.sort_pairs(k, v, rb, out_keys=ok, out_values=ov, stream=s)
    for rep in range(4):
        k.copy_(to_dev(ka if rep % 2 == 0 else kb))
        ok.fill_(-1)
        scratch = torch.arange(1 << 20, device="cuda", dtype=torch.int32).sum()  # eager work between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert int(scratch) >= 0
        want_k, want_v = wants[rep % 2]
        np.testing.assert_array_equal(to_np(ok), want_k, err_msg=f"replay {rep}")
        np.testing.assert_array_equal(to_np(ov), want_v, err_msg=f"replay {rep}")
        st = bs.status(s)
        assert st.flags == 0 and st.count == n
