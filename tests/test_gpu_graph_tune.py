"""HIP-graph replays and the autotuner, checked against eager calls and the
oracle.  Each graph is replayed several times with eager work and
synchronisations in between, and every replay is compared."""
import numpy as np
import pytest

import oracle
from gpu_util import require_gpu, to_dev, to_np
from paper_1312_0138_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()
    import paper_1312_0138_amd as bs
    yield
    bs.tuning_clear()
    bs.set_tuning(0, 0, 0)


@pytest.fixture(scope="module")
def o():
    return oracle.default()


@pytest.mark.parametrize("n,rb", [(1_000_000, 24), ((1 << 22) + 5, 24), (5000, 16), ((1 << 21) + 3, 32)])
def test_plain_graph_replays(o, n, rb):
    import torch
    import paper_1312_0138_amd as bs
    keys = torch.empty(n, dtype=torch.int32, device="cuda")
    out = torch.empty_like(keys)
    eager = torch.empty_like(keys)
    g = bs.Graph.plain(keys, rb, out)
    try:
        for rep in range(4):
            seed = inputs.config_seed(7, rep)
            bs.generate(n, rb, seed, out=keys)          # new contents, same buffer
            bs.sort(keys, rb, eager)
            torch.cuda.synchronize()
            g.launch()
            (flags, count), = g.status()
            assert flags == 0 and count == n
            assert torch.equal(out, eager), f"replay {rep} differs from the eager sort"
            if rep == 0:
                host = inputs.distinct_uniform(n, rb, seed)
                np.testing.assert_array_equal(to_np(keys), host)
                want, _, _ = o.bitmap_sort(host, rb)
                np.testing.assert_array_equal(to_np(out), want)
    finally:
        g.close()


def test_batch_graph_replays(o):
    import torch
    import paper_1312_0138_amd as bs
    keys_np, offsets, rbits = inputs.batch_segments(200, 16, 300_000, seed=44)
    k = to_dev(keys_np)
    off = torch.from_numpy(offsets.astype(np.int64)).cuda()
    rb = torch.from_numpy(rbits).cuda()
    out = torch.empty_like(k)
    eager = torch.empty_like(k)
    want, n_out, _ = o.bitmap_sort_segments(keys_np, offsets, rbits)
    g = bs.Graph.batch(k, off, rb, out)
    try:
        for rep in range(3):
            out.fill_(-1)
            bs.sort_batch(k, off, rb, eager)
            torch.cuda.synchronize()
            g.launch()
            st = g.status()
            assert [c for _, c in st] == n_out.tolist() and not any(f for f, _ in st)
            assert torch.equal(out, eager)
            np.testing.assert_array_equal(to_np(out), want)
    finally:
        g.close()


def test_autotune_plain_and_cache(o, tmp_path):
    import paper_1312_0138_amd as bs
    n, rb = 1 << 22, 26
    best = bs.autotune(n, rb, reps=2)
    assert 10 <= best["slice_bits"] <= 20 and 12 <= best["tile_log2"] <= 15 and best["emit_path"] in (1, 2, 3)
    info = bs.plan_info(n, rb)
    assert info["slice_bits"] == best["slice_bits"] and info["tile_log2"] == best["tile_log2"]
    keys = inputs.distinct_uniform(n, rb, 45)
    want, _, _ = o.bitmap_sort(keys, rb)
    got = to_np(bs.sort(to_dev(keys), rb))
    np.testing.assert_array_equal(got, want)
    path = str(tmp_path / "tune.jsonl")
    bs.tuning_save(path)
    bs.tuning_clear()
    assert bs.tuning_load(path) >= 1
    assert bs.plan_info(n, rb)["slice_bits"] == best["slice_bits"]
    bs.tuning_clear()


def test_autotune_batch(o):
    import torch
    import paper_1312_0138_amd as bs
    keys_np, offsets, rbits = inputs.batch_segments(300, 64, 200_000, seed=46)
    k = to_dev(keys_np)
    off = torch.from_numpy(offsets.astype(np.int64)).cuda()
    rb = torch.from_numpy(rbits).cuda()
    out = torch.empty_like(k)
    best = bs.autotune_batch(k, off, rb, out, reps=2)
    assert best["block"] in (256, 512, 1024) and 16 <= best["slice_bits"] <= 20
    want, n_out, _ = o.bitmap_sort_segments(keys_np, offsets, rbits)
    out.fill_(-1)
    bs.sort_batch(k, off, rb, out)
    flags, counts = bs.batch_status(rbits.size)
    assert not flags.any() and np.array_equal(counts, n_out)
    np.testing.assert_array_equal(to_np(out), want)
    bs.tuning_clear()
