"""Serving loop on the virtual-clock executor (no GPU): admission order,
memory budget, batching, rejection and determinism of the scheduler."""
import numpy as np
import pytest

from paper_1312_0138_amd import _lib, serve


def _trace(count=300, lo=1000, hi=1 << 20, rate=2e4, seed=7):
    return serve.make_trace(count, lo, hi, rate, seed)


def _run(req, budget=1 << 30, **kw):
    kw.setdefault("simulate", True)
    return serve.run(req, budget, **kw)


def test_all_served_and_counted():
    req = _trace()
    res, st = _run(req)
    assert np.all(res["flags"] == 0)
    assert np.array_equal(res["count"], req["n"])
    assert st["keys"] == int(req["n"].sum())
    assert np.all(res["batch"] != np.iinfo(np.uint32).max)
    assert np.all(res["done_s"] >= res["launch_s"])
    assert np.all(res["launch_s"] >= req["arrival_s"])


def _kinds(req, thr=20):
    """0: segmented launch, 1: pointer-array launch, 2: alone (the loop's rule)."""
    wide = req["range_bits"] > thr
    return np.where(~wide, 0, np.where(req["n"] >= 1 << 23, 2, 1))


def test_fifo_admission_order():
    req = _trace(count=600, lo=1000, hi=1 << 24, rate=5e4, seed=11)
    res, _ = _run(req, budget=160 << 20, streams=3)
    kinds = _kinds(req)
    assert len(set(kinds.tolist())) == 3
    order = np.argsort(req["arrival_s"], kind="stable")
    order = order[res["flags"][order] == 0]  # rejected requests (larger than the budget) never launch
    for k in range(3):
        o = order[kinds[order] == k]  # requests of one kind launch in arrival order
        assert np.all(np.diff(res["launch_s"][o]) >= 0)
        assert np.all(np.diff(res["batch"][o].astype(np.int64)) >= 0)
    # no request is overtaken by a later one of its own kind, and a request
    # waits at most until every earlier request has been launched or is in
    # the same launch
    first_launch_after = np.maximum.accumulate(res["launch_s"][order][::-1])[::-1]
    assert np.all(res["launch_s"][order] <= first_launch_after + 1e-12)


def test_peak_within_budget_and_memory_wait():
    req = _trace(count=200, lo=1 << 18, hi=1 << 21, rate=1e6, seed=3)
    budget = 48 << 20
    res, st = _run(req, budget=budget, streams=4)
    assert st["peak_bytes"] <= budget
    assert np.all(res["flags"] == 0)
    # a tight budget keeps fewer requests in flight than an ample one
    _, st_big = _run(req, budget=8 << 30, streams=4)
    assert st["max_inflight_requests"] <= st_big["max_inflight_requests"]


def test_burst_is_batched():
    req = _trace(count=500, hi=1 << 18, rate=float("inf"))
    res, st = _run(req, streams=1)
    assert st["launches"] < 20
    res1, st1 = _run(req, streams=1, max_batch_requests=1)
    assert st1["launches"] == len(req)
    assert st["makespan_s"] < st1["makespan_s"]  # per-launch overhead is paid once per batch


def test_batch_key_cap():
    req = _trace(count=100, lo=1 << 16, hi=1 << 16, rate=float("inf"))
    res, st = _run(req, max_batch_keys=1 << 20)
    sizes = np.bincount(res["batch"].astype(np.int64))
    assert sizes.max() <= 16
    assert st["launches"] >= 100 // 16


def test_plain_range_bits_threshold():
    req = _trace(count=200, lo=1000, hi=1 << 24, rate=float("inf"), seed=13)
    for thr in (16, 20, 24):
        res, _ = _run(req, plain_range_bits=thr)
        ids, counts = np.unique(res["batch"], return_counts=True)
        size = dict(zip(ids.tolist(), counts.tolist()))
        wide = req["range_bits"] > thr
        big = wide & (req["n"] >= 1 << 23)
        # a launch never mixes narrow and wide requests; big wide ones run alone
        for b in np.unique(res["batch"]):
            members = res["batch"] == b
            assert wide[members].all() or not wide[members].any()
        assert all(size[b] == 1 for b in res["batch"][big].tolist())
        assert any(size[b] > 1 for b in res["batch"][~wide].tolist())
        if (wide & ~big).sum() > 1:
            assert any(size[b] > 1 for b in res["batch"][wide & ~big].tolist())


def test_wide_requests_run_alone():
    req = _trace(count=60, rate=float("inf"), seed=5)
    req["n"][::10] = 1 << 23
    req["range_bits"][::10] = 28
    res, _ = _run(req, budget=2 << 30)
    assert np.all(res["flags"] == 0)
    for i in range(0, 60, 10):
        assert np.count_nonzero(res["batch"] == res["batch"][i]) == 1


def test_rejection_and_invalid():
    req = _trace(count=40, rate=float("inf"), seed=9)
    req["n"][5] = 1 << 26          # 2 x 256 MiB of keys: larger than the budget
    req["range_bits"][5] = 28
    req["n"][7] = 100              # more keys than the range holds
    req["range_bits"][7] = 6
    req["range_bits"][8] = 33      # key range beyond 32 bits
    res, st = _run(req, budget=256 << 20)
    assert res["flags"][5] == _lib.REQ_REJECTED
    assert res["flags"][7] == _lib.REQ_INVALID and res["flags"][8] == _lib.REQ_INVALID
    ok = np.ones(len(req), bool)
    ok[[5, 7, 8]] = False
    assert np.all(res["flags"][ok] == 0)
    assert np.array_equal(res["count"][ok], req["n"][ok])
    s = serve.summarize(req, res, st)
    assert s["served"] == len(req) - 3 and s["rejected"] == 3


def test_simulated_latency_model():
    req = _trace(count=1, lo=1 << 20, hi=1 << 20, rate=1e3)
    res, st = _run(req, sim_overhead_s=1e-4, sim_keys_per_s=1e9)
    lat = res["done_s"][0] - req["arrival_s"][0]
    assert lat == pytest.approx(1e-4 + (1 << 20) / 1e9, rel=1e-9)
    assert st["makespan_s"] == pytest.approx(lat, rel=1e-9)


def test_deterministic():
    req = _trace(seed=21)
    a, sa = _run(req, budget=96 << 20, streams=2)
    b, sb = _run(req, budget=96 << 20, streams=2)
    assert a.tobytes() == b.tobytes() and sa == sb


def test_empty_trace_and_bad_config():
    res, st = _run(np.zeros(0, dtype=serve.REQUEST))
    assert res.size == 0 and st["launches"] == 0
    with pytest.raises(_lib.BitsortError):
        _run(_trace(count=2), streams=0)
    with pytest.raises(_lib.BitsortError):
        _run(_trace(count=2), budget=0)
    with pytest.raises(_lib.BitsortError):
        _run(_trace(count=2), sim_keys_per_s=0.0)


def test_host_digest_is_order_sensitive():
    v = np.arange(100, dtype=np.uint32) * 7
    d = serve.host_digest(v)
    assert d != serve.host_digest(v[::-1])
    w = v.copy()
    w[50] += 1
    assert d != serve.host_digest(w)
    assert serve.host_digest(np.zeros(0, np.uint32)) == 0
