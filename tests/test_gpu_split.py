"""Parity of the bit-vector route with heavy slices shared out among workgroups
(k_slice_split) against the CPU oracle, element by element.

With emit path 4 (the tuning knob), a slice holding more than four times the
mean keys (and 2^16 or more) is cut into tile chunks that several workgroups
mark into partial bit-vectors and then OR together.  The inputs here put
chosen slices far above that threshold, and every test checks through
``debug_split`` that the sort really published them, so the shared path is
the one under test.
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


@pytest.fixture(autouse=True)
def _shared_path():
    import paper_1312_0138_amd as bs
    bs.set_tuning(0, 0, 4)
    yield
    bs.set_tuning(0, 0, 0)


def _heavy_keys(n_background, rb, sb, heavy, seed):
    """Distinct keys below 2^rb: n_background uniform keys outside the heavy
    slices, plus, for each (slice, count) in heavy, `count` distinct keys of
    that 2^sb-key slice."""
    bg = inputs.distinct_uniform(n_background, rb, seed).astype(np.uint64)
    hs = np.array([s for s, _ in heavy], dtype=np.uint64)
    bg = bg[~np.isin(bg >> np.uint64(sb), hs)]
    rng = np.random.default_rng(seed + 1)
    parts = [bg]
    for s, count in heavy:
        offs = rng.choice(1 << sb, size=count, replace=False).astype(np.uint64)
        parts.append((np.uint64(s) << np.uint64(sb)) + offs)
    keys = np.concatenate(parts).astype(np.uint32)
    return keys[rng.permutation(keys.size)]


def _sort_ws(keys, rb):
    import torch
    import paper_1312_0138_amd as bs
    k = to_dev(keys)
    ws = torch.empty(bs.workspace_bytes(keys.size, rb), dtype=torch.uint8, device="cuda")
    out = bs.sort_ws(k, rb, ws)
    st = bs.workspace_status(ws)
    return to_np(out), st, bs.debug_split(ws, keys.size, rb)


# (range_bits, background keys, heavy slices (slice, keys)): the plan for 2^26
# uses 2^18-bit slices (256 of them) and 2^14-key tiles; 2^25 with about 2.2 x 10^6
# keys uses 2^17-bit slices and 2^12-key tiles (about 540 tiles, 9 tile chunks).
CASES = [
    (26, 4_500_000, [(77, 200_000)]),
    (26, 4_500_000, [(0, 150_000), (3, 240_000), (255, 180_000)]),
    (26, 4_200_000, [(s, 150_000) for s in range(10, 250, 20)]),  # 12 heavy slices
    (25, 2_000_000, [(5, 120_000), (127, 90_000)]),
]


@pytest.mark.parametrize("rb,nbg,heavy", CASES)
def test_shared_heavy_slices(o, rb, nbg, heavy):
    import paper_1312_0138_amd as bs
    sb = bs.plan_info(nbg, rb)["slice_bits"]
    keys = _heavy_keys(nbg, rb, sb, heavy, 500 + rb + len(heavy))
    plan = bs.plan_info(keys.size, rb)
    assert plan["emit_path"] == "hbm-bitvector-shared" and plan["slice_bits"] == sb, plan
    want, _, _ = o.bitmap_sort(keys, rb)
    got, st, published = _sort_ws(keys, rb)
    assert published == len(heavy), published
    assert st.flags == 0 and st.count == keys.size
    np.testing.assert_array_equal(got, want)


def test_shared_heavy_slices_with_duplicates_and_range(o):
    """Repeated keys inside heavy slices (so a key's two copies may land in two
    workgroups' partials) and keys past the range: flags, count and the
    compacted output as the oracle gives them."""
    import paper_1312_0138_amd as bs
    rb = 26
    sb = bs.plan_info(4_500_000, rb)["slice_bits"]
    base = _heavy_keys(4_500_000, rb, sb, [(40, 220_000), (41, 200_000)], 77)
    rng = np.random.default_rng(78)
    in_heavy = base[np.isin(base.astype(np.uint64) >> np.uint64(sb), np.array([40, 41], dtype=np.uint64))]
    dup = rng.choice(in_heavy, size=3000, replace=False)
    bad = (np.uint64(1) << np.uint64(rb)) + rng.integers(0, 1 << 20, size=500).astype(np.uint64)
    keys = np.concatenate([base, dup, bad.astype(np.uint32)])
    keys = keys[rng.permutation(keys.size)]
    want, _, _ = o.bitmap_sort(keys, rb)
    got, st, published = _sort_ws(keys, rb)
    assert published == 2
    assert st.flags == (bs.STATUS_OUT_OF_RANGE | bs.STATUS_DUPLICATE)
    assert st.count == want.size
    np.testing.assert_array_equal(got[:want.size], want)


def test_clustered_workload_shares_its_heavy_slices(o):
    """The clustered workload (64 Gaussian clusters, 2^26 draws, 2^28 range)
    publishes heavy slices and sorts exactly."""
    keys = inputs.clustered(1 << 26, 28, inputs.config_seed(2, 4))
    want, _, _ = o.bitmap_sort(keys, 28)
    got, st, published = _sort_ws(keys, 28)
    assert published >= 1
    assert st.flags == 0 and st.count == keys.size
    np.testing.assert_array_equal(got, want)


def test_shared_slices_in_a_caller_workspace_full_of_garbage(o):
    """The split's control words live in the workspace and are cleared by the
    partition step of every sort: a workspace filled with 0xFF before the first
    call, and reused for a second, different input, gives exact results."""
    import torch
    import paper_1312_0138_amd as bs
    rb = 26
    sb = bs.plan_info(4_500_000, rb)["slice_bits"]
    k1 = _heavy_keys(4_500_000, rb, sb, [(9, 230_000), (200, 160_000)], 91)
    k2 = _heavy_keys(4_500_000, rb, sb, [(100, 210_000)], 92)
    n = max(k1.size, k2.size)
    ws = torch.full((bs.workspace_bytes(n, rb),), 0xFF, dtype=torch.uint8, device="cuda")
    for keys, heavy in ((k1, 2), (k2, 1)):
        want, _, _ = o.bitmap_sort(keys, rb)
        out = bs.sort_ws(to_dev(keys), rb, ws)
        st = bs.workspace_status(ws)
        assert bs.debug_split(ws, keys.size, rb) == heavy
        assert st.flags == 0 and st.count == keys.size
        np.testing.assert_array_equal(to_np(out), want)


def test_graph_replays_with_shared_slices(o):
    """A captured plain sort replayed four times over two inputs with heavy
    slices (the control words are cleared on the device at every replay),
    with eager sorts between the replays; every replay checked."""
    import torch
    import paper_1312_0138_amd as bs
    rb = 26
    sb = bs.plan_info(4_500_000, rb)["slice_bits"]
    ka = _heavy_keys(4_500_000, rb, sb, [(60, 220_000)], 11)
    kb = _heavy_keys(4_500_000, rb, sb, [(61, 190_000), (62, 170_000)], 12)
    n = min(ka.size, kb.size)
    ka, kb = ka[:n], kb[:n]  # one graph, one size (both are in random order already)
    wants = [o.bitmap_sort(ka, rb)[0], o.bitmap_sort(kb, rb)[0]]
    keys = to_dev(ka)
    out = torch.empty_like(keys)
    g = bs.Graph.plain(keys, rb, out)
    for i in range(4):
        keys.copy_(to_dev(ka if i % 2 == 0 else kb))
        g.launch()
        (flags, count), = g.status()
        assert flags == 0 and count == n
        np.testing.assert_array_equal(to_np(out), wants[i % 2])
        eager = bs.sort(to_dev(kb), rb)
        np.testing.assert_array_equal(to_np(eager), wants[1])
