"""Parity of the HIP plain path (bitsort_u32) with the CPU oracle.

Every comparison is element by element (integers: bit-exact).  Inputs come
from the seeded host generators in ``paper_1312_0138_amd.inputs``; the oracle
never sees a value produced by the HIP path.
"""
import numpy as np
import pytest

import oracle
from gpu_util import require_gpu, to_dev, to_np
from paper_1312_0138_amd import inputs

pytestmark = pytest.mark.gpu

SENTINEL = 0xDEADBEEF


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


@pytest.fixture(scope="module")
def o():
    return oracle.default()


def _gpu_sort(keys_np, rb, out_init=None):
    import torch
    import paper_1312_0138_amd as bs
    k = to_dev(keys_np)
    out = to_dev(out_init) if out_init is not None else torch.empty_like(k)
    bs.sort(k, rb, out)
    st = bs.status()
    return to_np(out), st


# (n, range_bits): both paths, word and tile boundaries, ragged tails.
SIZES = [
    (1, 0), (1, 1), (2, 1), (3, 2), (16, 4), (17, 5), (32, 5), (33, 6), (700, 10), (1024, 10),
    (5000, 13), (8192, 20), (8193, 20), (9000, 14), (16384, 14), (20000, 16), (65536, 16),
    (100_000, 20), (1 << 20, 20), (4097, 24), (16385, 24), (300_001, 24), (1_000_000, 24),
    (50_000, 32), (1 << 18, 28), (123_457, 31), ((1 << 22) + 1, 24), (3 << 20, 22),
]


@pytest.mark.parametrize("n,rb", SIZES)
def test_parity_sizes(o, n, rb):
    keys = inputs.distinct_uniform(n, rb, inputs.config_seed(100 + rb, n))
    want, flags, _ = o.bitmap_sort(keys, rb)
    assert flags == 0
    got, st = _gpu_sort(keys, rb)
    assert st.flags == 0 and st.count == n
    np.testing.assert_array_equal(got, want)


@pytest.mark.parametrize("rb", [0, 1, 4, 5, 6, 20, 21, 28, 32])
@pytest.mark.parametrize("path", [0, 1])
def test_edge_keys(o, rb, path):
    """Word, slice and range boundaries: 0, 31, 32, 63, 64, a fully set word (96..127),
    2^20 - 1 and 2^20 (a slice boundary), R - 1 (the last key, 0xFFFFFFFF at 32 bits),
    and every key of the range when it is below one word."""
    import paper_1312_0138_amd as bs
    R = 1 << rb
    if rb <= 5:
        keys = np.arange(R, dtype=np.uint64)
    else:
        cand = [0, 31, 32, 63, 64, *range(96, 128), (1 << 20) - 1, 1 << 20, R - 1, R - 2, R // 2]
        keys = np.array(sorted({c for c in cand if c < R}), dtype=np.uint64)
    keys = keys.astype(np.uint32)[np.random.default_rng(rb).permutation(keys.size)]
    want, _, _ = o.bitmap_sort(keys, rb)
    bs.set_tuning(0, 0, path)
    try:
        got, st = _gpu_sort(keys, rb)
    finally:
        bs.set_tuning(0, 0, 0)
    assert st.flags == 0 and st.count == keys.size
    np.testing.assert_array_equal(got, want)


@pytest.mark.parametrize("rep", [0, 1, 2])
def test_parity_config_small(o, rep):
    """10^6 distinct keys from [0, 2^24), three seeds."""
    keys = inputs.distinct_uniform(1_000_000, 24, inputs.config_seed(1, rep))
    want, _, _ = o.bitmap_sort(keys, 24)
    got, st = _gpu_sort(keys, 24)
    assert st.flags == 0 and st.count == keys.size
    np.testing.assert_array_equal(got, want)


@pytest.mark.parametrize("rep", [0, 1, 2])
def test_parity_config_large_uniform(o, rep):
    """2^26 distinct keys from [0, 2^28), full size, three seeds."""
    keys = inputs.distinct_uniform(1 << 26, 28, inputs.config_seed(2, rep))
    want, _, _ = o.bitmap_sort(keys, 28)
    got, st = _gpu_sort(keys, 28)
    assert st.flags == 0 and st.count == keys.size
    np.testing.assert_array_equal(got, want)


def test_parity_clustered(o):
    """Gaussian-cluster keys (64 clusters, sigma 2^16) in [0, 2^28)."""
    keys = inputs.clustered(1 << 22, 28, inputs.config_seed(2, 1))
    want, _, _ = o.bitmap_sort(keys, 28)
    got, st = _gpu_sort(keys, 28)
    assert st.flags == 0 and st.count == keys.size
    np.testing.assert_array_equal(got, want)


@pytest.mark.parametrize("rep", [1, 2, 3])
def test_parity_clustered_full_size(o, rep):
    """The clustered workload itself: 2^26 draws, de-duplicated (about 1.7 x 10^7 keys),
    three seeds."""
    keys = inputs.clustered(1 << 26, 28, inputs.config_seed(2, rep))
    want, _, _ = o.bitmap_sort(keys, 28)
    got, st = _gpu_sort(keys, 28)
    assert st.flags == 0 and st.count == keys.size
    np.testing.assert_array_equal(got, want)


@pytest.mark.parametrize("path", [0, 2])
@pytest.mark.parametrize("rb,density", [(24, 0.55), (24, 0.8), (24, 0.97), (26, 0.7), (22, 0.999)])
def test_parity_dense_groups(o, rb, density, path):
    """Dense but not full words (over 16 keys per word) on both emission routes, so
    that 64-word groups with more keys than one emission window occur."""
    import paper_1312_0138_amd as bs
    n = int(density * (1 << rb)) + 5
    keys = inputs.distinct_uniform(n, rb, 80 + rb)
    want, _, _ = o.bitmap_sort(keys, rb)
    bs.set_tuning(0, 0, path)
    try:
        got, st = _gpu_sort(keys, rb)
    finally:
        bs.set_tuning(0, 0, 0)
    assert st.flags == 0 and st.count == n
    np.testing.assert_array_equal(got, want)


@pytest.mark.parametrize("n,rb", [(1_000_000, 24), (1 << 24, 26), ((1 << 22) + 17, 32)])
def test_order_independence(o, n, rb):
    """Shuffling the input leaves the output unchanged (LDS, bit-vector and summary paths),
    and the output keeps the invariants: length n, strictly ascending, every key < 2^rb."""
    keys = inputs.distinct_uniform(n, rb, 101 + rb)
    got1, st1 = _gpu_sort(keys, rb)
    shuffled = keys[np.random.default_rng(5).permutation(n)]
    got2, st2 = _gpu_sort(shuffled, rb)
    assert st1.flags == st2.flags == 0 and st1.count == st2.count == n
    np.testing.assert_array_equal(got1, got2)
    assert got1.size == n and np.all(got1[1:] > got1[:-1]) and int(got1[-1]) < (1 << rb)
    np.testing.assert_array_equal(got1, o.bitmap_sort(keys, rb)[0])


def test_dense_permutation_is_identity():
    """A permutation of all of [0, 2^28) sorts to 0, 1, ..., 2^28-1."""
    import torch
    import paper_1312_0138_amd as bs
    g = torch.Generator(device="cuda")
    g.manual_seed(3)
    k = torch.randperm(1 << 28, device="cuda", dtype=torch.int64, generator=g).to(torch.int32)
    out = torch.empty_like(k)
    bs.sort(k, 28, out)
    st = bs.status()
    assert st.flags == 0 and st.count == 1 << 28
    ref = torch.arange(1 << 28, device="cuda", dtype=torch.int32)
    assert torch.equal(out, ref)


@pytest.mark.parametrize("rep", [0, 1, 2])
def test_parity_sparse_full_range(o, rep):
    """2^24 distinct keys over all of [0, 2^32), three seeds."""
    keys = inputs.distinct_uniform(1 << 24, 32, inputs.config_seed(3, rep))
    want, _, _ = o.bitmap_sort(keys, 32)
    got, st = _gpu_sort(keys, 32)
    assert st.flags == 0 and st.count == keys.size
    np.testing.assert_array_equal(got, want)


# (n, range_bits, emit path): 0 = library choice, 1 = from LDS, 2 = through the HBM bit-vector
STEP_CASES = [(3000, 12, 0), (1 << 20, 20, 0), (1_000_000, 24, 1), (1_000_000, 24, 2), (40_000, 27, 0),
              ((1 << 22) + 3, 24, 0), (1 << 22, 26, 2), ((1 << 21) + 5, 30, 0)]


@pytest.mark.parametrize("n,rb,path", STEP_CASES)
def test_mark_step_matches_oracle_bitmap(o, n, rb, path):
    import paper_1312_0138_amd as bs
    keys = inputs.distinct_uniform(n, rb, 77)
    want, _ = o.bitmap_build(keys, rb)
    bs.set_tuning(0, 0, path)
    try:
        got = to_np(bs.debug_bitmap(to_dev(keys), rb))
    finally:
        bs.set_tuning(0, 0, 0)
    np.testing.assert_array_equal(got, want)


@pytest.mark.parametrize("n,rb,path", STEP_CASES)
def test_scan_step_matches_oracle_prefix(o, n, rb, path):
    import paper_1312_0138_amd as bs
    keys = inputs.distinct_uniform(n, rb, 78)
    words, _ = o.bitmap_build(keys, rb)
    want = o.bitmap_scan(words)[:-1]
    bs.set_tuning(0, 0, path)
    try:
        got = bs.debug_prefix(to_dev(keys), rb).cpu().numpy().astype(np.uint64)
    finally:
        bs.set_tuning(0, 0, 0)
    np.testing.assert_array_equal(got, want)


@pytest.mark.parametrize("path", [1, 2])
@pytest.mark.parametrize("n,rb", [(1 << 20, 24), (3_000_001, 26), (1 << 24, 28)])
def test_both_emit_paths(o, n, rb, path):
    import paper_1312_0138_amd as bs
    keys = inputs.distinct_uniform(n, rb, 79)
    want, _, _ = o.bitmap_sort(keys, rb)
    bs.set_tuning(0, 0, path)
    try:
        assert bs.plan_info(n, rb)["emit_path"] == {1: "lds", 2: "hbm-bitvector"}[path]
        got, st = _gpu_sort(keys, rb)
    finally:
        bs.set_tuning(0, 0, 0)
    assert st.flags == 0 and st.count == n
    np.testing.assert_array_equal(got, want)


# (n, range_bits, forced emit path): 0 lets the library choose (the word summary
# for n <= R/32 with 2^20-bit slices), 1 forces the plain word scan, 3 the summary.
# Segments of 8 keys or fewer per tile and slice (2^14 << 20 <= 8 R, or 2^12 << 20
# <= 8 R) switch the gather to 16-key units: (2^22 + 17, 32), (2^22 + 9, 32, 1),
# (2^21, 30) and (5000, 32) take them, with and without the summary.
SPARSE_CASES = [(1 << 20, 28, 0), (1 << 20, 28, 1), (1_000_003, 30, 0), ((1 << 22) + 17, 32, 0), (5000, 32, 0),
                (70_001, 26, 3), (1 << 23, 28, 0), ((1 << 23) + 1, 28, 3), (1 << 24, 28, 3),
                ((1 << 22) + 9, 32, 1), (1 << 21, 30, 0)]


@pytest.mark.parametrize("n,rb,path", SPARSE_CASES)
def test_sparse_summary_path(o, n, rb, path):
    """Emission through the per-word summary (few keys per word) against the oracle,
    with the plan the test means to exercise."""
    import paper_1312_0138_amd as bs
    keys = inputs.distinct_uniform(n, rb, 90 + rb)
    want, _, _ = o.bitmap_sort(keys, rb)
    bs.set_tuning(20 if path == 3 else 0, 0, path)  # the summary needs 2^20-bit slices
    try:
        plan = bs.plan_info(n, rb)
        sparse = path == 3 or (path == 0 and 32 * n <= 1 << rb)
        assert plan["emit_path"] == ("lds-sparse" if sparse else "lds"), plan
        got, st = _gpu_sort(keys, rb)
    finally:
        bs.set_tuning(0, 0, 0)
    assert st.flags == 0 and st.count == n
    np.testing.assert_array_equal(got, want)


def test_sparse_slices_over_several_rounds_of_tiles(o):
    """Many sparse slices per workgroup with more than 1024 tiles, so that each slice's
    gather runs over several rounds of tiles after the prefetched first one."""
    import paper_1312_0138_amd as bs
    n, rb = (1 << 22) + 3, 32
    keys = inputs.distinct_uniform(n, rb, 99)
    want, _, _ = o.bitmap_sort(keys, rb)
    bs.set_tuning(0, 12, 0)
    try:
        plan = bs.plan_info(n, rb)
        assert plan["emit_path"] == "lds-sparse" and plan["tile_log2"] == 12 and plan["buckets"] == 4096
        got, st = _gpu_sort(keys, rb)
    finally:
        bs.set_tuning(0, 0, 0)
    assert st.flags == 0 and st.count == n
    np.testing.assert_array_equal(got, want)


def _emission_shape_keys(rb, seed):
    """Keys laid out for the summary emission's branches.  A 2^20-bit slice has
    32768 words; its wave v covers words [2048 v, 2048 v + 2048), lane l of it the
    32 words of summary word 64 v + l.  The emission keeps a lane's first eight
    nonzero words in registers and stages the wave's keys in a window of 440.
    Every wave of every fifth slice (every thirteenth at 2^30) gets one of these shapes:
    0: 0-4 nonzero words per lane, 1-3 keys each (registers, window);
    1: 440 keys, lanes 0-61 with seven one-key words, lane 62 with six (window full);
    2: 441 keys, lanes 0-62 with seven one-key words (one key over the window);
    3: eight one-key words in every lane (512 keys, over the window);
    4: eight full words in every lane (16384 keys);
    5: nine one-key words in lane 5, one in every other lane (a lane past eight);
    6: eight one-key words in lanes 0-54 (440 keys, every register in use)."""
    rng = np.random.default_rng(seed)
    parts = []
    slices = 1 << (rb - 20)

    def words_for(base, count, full=False, keys_each=None):
        offs = np.sort(rng.choice(32, size=count, replace=False)).astype(np.uint64)
        for w in base + offs:
            if full:
                bits = np.arange(32, dtype=np.uint64)
            else:
                k = keys_each if keys_each is not None else int(rng.integers(1, 4))
                bits = rng.choice(32, size=k, replace=False).astype(np.uint64)
            parts.append(w * np.uint64(32) + bits)

    step = 5 if rb <= 28 else 13
    for s in range(0, slices, step):
        for v in range(16):
            shape = (s // step + v) % 7
            for lane in range(64):
                base = np.uint64(s * 32768 + (v * 64 + lane) * 32)
                if shape == 0:
                    words_for(base, int(rng.integers(0, 5)))
                elif shape == 1:
                    words_for(base, 7 if lane < 62 else (6 if lane == 62 else 0), keys_each=1)
                elif shape == 2:
                    words_for(base, 7 if lane < 63 else 0, keys_each=1)
                elif shape == 3:
                    words_for(base, 8, keys_each=1)
                elif shape == 4:
                    words_for(base, 8, full=True)
                elif shape == 5:
                    words_for(base, 9 if lane == 5 else 1, keys_each=1)
                else:
                    words_for(base, 8 if lane < 55 else 0, keys_each=1)
    keys = np.concatenate(parts).astype(np.uint32)
    return keys[rng.permutation(keys.size)]


@pytest.mark.parametrize("rb", [28, 30])
def test_sparse_emission_shapes(o, rb):
    """The summary emission's register, window and fallback branches, each at its
    edge, against the oracle: 2^28 runs one workgroup per slice (k_slice), 2^30
    one workgroup walking many slices (k_slice_seq)."""
    import paper_1312_0138_amd as bs
    keys = _emission_shape_keys(rb, 40 + rb)
    want, _, _ = o.bitmap_sort(keys, rb)
    bs.set_tuning(20, 0, 3)
    try:
        plan = bs.plan_info(keys.size, rb)
        assert plan["emit_path"] == "lds-sparse" and plan["buckets"] == 1 << (rb - 20), plan
        got, st = _gpu_sort(keys, rb)
    finally:
        bs.set_tuning(0, 0, 0)
    assert st.flags == 0 and st.count == keys.size
    np.testing.assert_array_equal(got, want)


def test_sparse_summary_duplicates_and_range(o):
    """Duplicates and keys beyond the range on the summary path: flags, count and the
    compacted output as the oracle gives them."""
    import paper_1312_0138_amd as bs
    rb = 30
    base = inputs.distinct_uniform(300_000, rb, 97)
    rng = np.random.default_rng(5)
    dup = rng.choice(base, size=2000, replace=False)
    bad = (np.uint64(1) << np.uint64(rb)) + rng.integers(0, 1 << 20, size=300).astype(np.uint64)
    keys = np.concatenate([base, dup, bad.astype(np.uint32)])
    rng.shuffle(keys)
    want, _, _ = o.bitmap_sort(keys, rb)
    assert bs.plan_info(keys.size, rb)["emit_path"] == "lds-sparse"
    got, st = _gpu_sort(keys, rb)
    assert st.flags == (bs.STATUS_OUT_OF_RANGE | bs.STATUS_DUPLICATE)
    assert st.count == want.size
    np.testing.assert_array_equal(got[:want.size], want)


@pytest.mark.parametrize("path", [1, 2])
def test_duplicates_and_range_on_both_paths(o, path):
    import paper_1312_0138_amd as bs
    base = inputs.distinct_uniform(1 << 21, 25, 81)
    keys = base.copy()
    rng = np.random.default_rng(2)
    at = rng.choice(keys.size, size=5000, replace=False)
    keys[at] = base[rng.integers(0, keys.size, size=at.size)]       # duplicates
    keys[rng.choice(keys.size, size=300, replace=False)] |= np.uint32(1 << 31)  # out of range
    want, flags, _ = o.bitmap_sort(keys, 25)
    assert flags == 3
    bs.set_tuning(0, 0, path)
    try:
        got, st = _gpu_sort(keys, 25)
    finally:
        bs.set_tuning(0, 0, 0)
    assert st.flags == 3 and st.count == want.size
    np.testing.assert_array_equal(got[: want.size], want)


@pytest.mark.parametrize("n,rb", [(500, 12), (200_000, 24), (60_000, 32)])
def test_out_of_range_keys_dropped(o, n, rb):
    keys = inputs.distinct_uniform(n, rb + 1 if rb < 32 else 32, 5)
    want, flags, _ = o.bitmap_sort(keys, rb)
    init = np.full(n, SENTINEL, dtype=np.uint32)
    got, st = _gpu_sort(keys, rb, out_init=init)
    if rb < 32:
        assert flags & oracle.FLAG_OUT_OF_RANGE
        assert st.flags == 1
    else:
        assert st.flags == 0
    d = want.size
    assert st.count == d
    np.testing.assert_array_equal(got[:d], want)
    assert np.all(got[d:] == SENTINEL)


@pytest.mark.parametrize("n,rb", [(400, 12), (300_000, 24), (5000, 20)])
def test_duplicates_collapse(o, n, rb):
    base = inputs.distinct_uniform(n, rb, 9)
    rng = np.random.default_rng(1)
    keys = base.copy()
    dup_at = rng.choice(n, size=max(1, n // 10), replace=False)
    keys[dup_at] = base[rng.integers(0, n, size=dup_at.size)]
    want, flags, _ = o.bitmap_sort(keys, rb)
    assert flags & oracle.FLAG_DUPLICATE
    got, st = _gpu_sort(keys, rb)
    assert st.flags & 2 and st.count == want.size
    np.testing.assert_array_equal(got[: want.size], want)


def test_status_read_runs_the_pending_finish_once(o):
    """A two-kernel sort leaves its totals to the status read: reading the
    status after repeated keys compacts out[0..d) once, a second read (on the
    stream, or on the caller's workspace) returns the same status and leaves
    the output as it is."""
    import torch
    import paper_1312_0138_amd as bs
    base = inputs.distinct_uniform(300_000, 24, 44)
    rng = np.random.default_rng(4)
    keys = base.copy()
    at = rng.choice(keys.size, size=3000, replace=False)
    keys[at] = base[rng.integers(0, keys.size, size=at.size)]
    want, flags, _ = o.bitmap_sort(keys, 24)
    assert flags == oracle.FLAG_DUPLICATE
    k = to_dev(keys)
    out = bs.sort(k, 24)
    st1 = bs.status()
    first = to_np(out).copy()
    st2 = bs.status()
    assert (st1.flags, st1.count) == (st2.flags, st2.count) == (2, want.size)
    np.testing.assert_array_equal(first[: want.size], want)
    np.testing.assert_array_equal(to_np(out), first)
    ws = torch.empty(bs.workspace_bytes(keys.size, 24), dtype=torch.uint8, device="cuda")
    out2 = bs.sort_ws(k, 24, ws)
    a = bs.workspace_status(ws)
    b = bs.workspace_status(ws)
    assert (a.flags, a.count) == (b.flags, b.count) == (2, want.size)
    np.testing.assert_array_equal(to_np(out2)[: want.size], want)


def test_in_place_and_misaligned(o):
    import torch
    import paper_1312_0138_amd as bs
    keys = inputs.distinct_uniform(500_000, 24, 11)
    want, _, _ = o.bitmap_sort(keys, 24)
    k = to_dev(keys)
    bs.sort(k, 24, k)  # out == keys
    np.testing.assert_array_equal(to_np(k), want)
    buf = to_dev(np.concatenate([[7], keys]))
    view = buf[1:]  # 4-byte aligned, not 16-byte aligned
    out = torch.empty_like(view)
    bs.sort(view, 24, out)
    np.testing.assert_array_equal(to_np(out), want)


def test_rejects_partial_overlap_and_bad_sizes():
    import torch
    import paper_1312_0138_amd as bs
    buf = torch.zeros(101, dtype=torch.int32, device="cuda")
    with pytest.raises(bs.BitsortError):
        bs.sort(buf[:100], 10, buf[1:])
    with pytest.raises(bs.BitsortError):
        bs.sort(buf[:100], 6)  # 100 keys cannot be distinct below 64
    with pytest.raises(bs.BitsortError):
        bs.sort(buf[:100], 33)


def test_empty_input():
    import torch
    import paper_1312_0138_amd as bs
    k = torch.empty(0, dtype=torch.int32, device="cuda")
    bs.sort(k, 20)
    st = bs.status()
    assert st.flags == 0 and st.count == 0


def test_deterministic_repeats():
    import torch
    import paper_1312_0138_amd as bs
    keys = to_dev(inputs.distinct_uniform(1 << 22, 26, 13))
    ref = bs.sort(keys, 26).clone()
    for _ in range(10):
        assert torch.equal(bs.sort(keys, 26), ref)


def test_side_stream_and_workspace_variant(o):
    import torch
    import paper_1312_0138_amd as bs
    keys = inputs.distinct_uniform(2_000_000, 25, 17)
    want, _, _ = o.bitmap_sort(keys, 25)
    k = to_dev(keys)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        out = bs.sort(k, 25)
        st = bs.status(s)
    assert st.count == keys.size
    np.testing.assert_array_equal(to_np(out), want)
    ws = torch.empty(bs.workspace_bytes(keys.size, 25), dtype=torch.uint8, device="cuda")
    out2 = bs.sort_ws(k, 25, ws)
    st2 = bs.workspace_status(ws)
    assert st2.flags == 0 and st2.count == keys.size
    np.testing.assert_array_equal(to_np(out2), want)


# (range_bits, emit path): with 2^16-bit slices and 2^14-key tiles a tile's segment
# holds about 2^(30 - rb) keys -- 512, 256, 128 -- so the waves' choice between
# 64-key units and 256-key units (16-byte loads) falls on both sides.
@pytest.mark.parametrize("rb", [21, 22, 23])
@pytest.mark.parametrize("path", [1, 2])
@pytest.mark.parametrize("extra", [0, 3])
def test_long_gather_units(o, rb, path, extra):
    """The slice kernel's 256-key gather units around their switch point: full tiles
    (the last slice's last segment ends where the staging area ends), or a last
    tile of three keys."""
    import paper_1312_0138_amd as bs
    n = 37 * (1 << 14) + extra
    keys = inputs.distinct_uniform(n, rb, 60 + rb)
    want, _, _ = o.bitmap_sort(keys, rb)
    bs.set_tuning(16, 14, path)
    try:
        plan = bs.plan_info(n, rb)
        assert plan["slice_bits"] == 16 and plan["tile_log2"] == 14, plan
        got, st = _gpu_sort(keys, rb)
    finally:
        bs.set_tuning(0, 0, 0)
    assert st.flags == 0 and st.count == n
    np.testing.assert_array_equal(got, want)


@pytest.mark.parametrize("sb,tl,path", [(10, 12, 1), (14, 13, 1), (18, 14, 1), (20, 12, 1), (16, 14, 1),
                                        (15, 12, 2), (16, 13, 2), (18, 14, 2), (20, 14, 2), (0, 0, 2), (20, 15, 2), (16, 15, 1)])
def test_tuning_knobs_keep_results(o, sb, tl, path):
    import paper_1312_0138_amd as bs
    keys = inputs.distinct_uniform(700_001, 24, 19)
    want, _, _ = o.bitmap_sort(keys, 24)
    bs.set_tuning(sb, tl, path)
    try:
        got, st = _gpu_sort(keys, 24)
    finally:
        bs.set_tuning(0, 0, 0)
    assert st.count == keys.size
    np.testing.assert_array_equal(got, want)


@pytest.mark.parametrize("n,rb,path", [((1 << 24) + 12345, 28, 2), ((1 << 23) + 7, 30, 0), ((1 << 24) + 1, 26, 1)])
def test_partition_large_tiles(o, n, rb, path):
    """2^15-key tiles (1024 threads of 32 keys, one workgroup per tile): more
    than 256 tiles here, the last one ragged."""
    import paper_1312_0138_amd as bs
    keys = inputs.distinct_uniform(n, rb, 107 + rb)
    want, _, _ = o.bitmap_sort(keys, rb)
    bs.set_tuning(0, 15, path)
    try:
        assert bs.plan_info(n, rb)["tile_log2"] == 15
        got, st = _gpu_sort(keys, rb)
    finally:
        bs.set_tuning(0, 0, 0)
    assert st.flags == 0 and st.count == n
    np.testing.assert_array_equal(got, want)


@pytest.mark.parametrize("rb,first,count", [(0, 0, 1), (1, 0, 2), (5, 3, 20), (7, 0, 128), (16, 100, 5000),
                                            (24, 12345, 100_000), (31, 1 << 30, 70_000), (32, 0, 100_000)])
def test_device_generator_matches_host(rb, first, count):
    import paper_1312_0138_amd as bs
    seed = 0xABCDEF + rb
    got = to_np(bs.generate(count, rb, seed, first=first))
    want = inputs.keyed_permutation(np.arange(first, first + count, dtype=np.uint64), rb, seed)
    np.testing.assert_array_equal(got, want)
