"""Serving loop on the device: every request's sorted output, digested on
the device, equals the oracle's sort of the same keys and the result of
sorting that request alone, whatever batch it shared."""
import numpy as np
import pytest

import oracle
from gpu_util import require_gpu, to_np
from paper_1312_0138_amd import inputs, serve

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


@pytest.fixture(scope="module")
def o():
    return oracle.default()


SENTINEL = -559038737  # 0xDEADBEEF as int32


def _oracle_sorted(o, n, rb, seed):
    keys = inputs.distinct_uniform(int(n), int(rb), int(seed))
    want, flags, _ = o.bitmap_sort(keys, int(rb))
    assert flags == 0
    return want


def _oracle_digest(o, n, rb, seed):
    return serve.host_digest(_oracle_sorted(o, n, rb, seed))


def _mixed_trace(seed):
    req = serve.make_trace(160, 1, 1 << 19, float("inf"), seed)
    # a few requests wider than the batch kernel's range go through the pointer-array launches
    req["n"][17::40] = [1 << 20, 3 << 19, 1000, 1 << 21][: len(req["n"][17::40])]
    req["range_bits"][17::40] = [26, 28, 30, 25][: len(req["range_bits"][17::40])]
    req["n"][3] = 0  # an empty request
    return req


def _sentinel_outputs(req):
    import torch
    return [torch.full((max(int(n), 1),), SENTINEL, dtype=torch.int32, device="cuda") for n in req["n"]]


def _check_outputs(o, req, res, outs, verify=True):
    """Every request's output, element by element, against the oracle's sort
    of the same keys regenerated on the host (Theorem 1: one correct output)."""
    for i in range(len(req)):
        n, rb, seed = int(req["n"][i]), int(req["range_bits"][i]), int(req["seed"][i])
        want = _oracle_sorted(o, n, rb, seed)
        got = to_np(outs[i])
        assert int(res["count"][i]) == n and int(res["flags"][i]) == 0, f"request {i}"
        np.testing.assert_array_equal(got[:n], want, err_msg=f"request {i} n={n} rb={rb}")
        if n == 0:
            assert got[0] == np.uint32(SENTINEL & 0xFFFFFFFF)
        if verify:
            assert int(res["digest"][i]) == serve.host_digest(want), f"request {i}"


def test_mix_matches_oracle_and_alone(o):
    import torch
    import paper_1312_0138_amd as bs
    req = _mixed_trace(0x5E1)
    budget = 96 << 20  # tight: requests wait for memory
    outs = _sentinel_outputs(req)
    res, st = serve.run(req, budget, streams=3, max_batch_requests=64, max_batch_keys=1 << 21, verify=True,
                        outputs=outs)
    assert st["peak_bytes"] <= budget
    assert np.all(res["flags"] == 0)
    np.testing.assert_array_equal(res["count"], req["n"])
    assert st["launches"] < len(req)  # some requests shared a launch
    _check_outputs(o, req, res, outs)
    # alone through the plain API (a different kernel path for batched requests)
    for i in [0, 1, 3, 17, 57, 100, 159]:
        n, rb, seed = int(req["n"][i]), int(req["range_bits"][i]), int(req["seed"][i])
        keys = bs.generate(n, rb, seed)
        out = bs.sort(keys, rb)
        assert serve.digest(out) == int(res["digest"][i])
        np.testing.assert_array_equal(to_np(out), to_np(outs[i])[:n])
    # alone through the serving loop
    for i in [2, 17, 80]:
        one_out = _sentinel_outputs(req[i:i + 1])
        one, _ = serve.run(req[i:i + 1], budget, verify=True, outputs=one_out)
        assert int(one["digest"][0]) == int(res["digest"][i])
        np.testing.assert_array_equal(to_np(one_out[0]), to_np(outs[i]))
    torch.cuda.synchronize()


def test_alone_launches_in_the_mix(o):
    """Requests of 2^23 keys or more with ranges above 2^20 bits run alone
    through the plain path (with its HBM bit-vector emission); the others
    share segmented and pointer-array launches around them.  Every output is
    checked element by element, with and without digests, and the big
    requests equal the same sort run on its own."""
    import paper_1312_0138_amd as bs
    req = serve.make_trace(96, 1, 1 << 18, float("inf"), 0x5E3)
    req["n"][20], req["range_bits"][20] = 1 << 23, 25          # alone, bit-vector emission
    req["n"][45], req["range_bits"][45] = (1 << 24) - 3, 26    # alone, ragged length
    req["n"][46], req["range_bits"][46] = 1 << 23, 28          # alone, LDS emission (R/8 > 2n)
    req["n"][70], req["range_bits"][70] = 1 << 21, 24          # pointer-array launch
    budget = 512 << 20
    for verify in (True, False):
        outs = _sentinel_outputs(req)
        res, st = serve.run(req, budget, streams=3, verify=verify, outputs=outs)
        assert st["peak_bytes"] <= budget
        big = [20, 45, 46]
        assert len({int(res["batch"][i]) for i in big}) == 3
        for i in big:  # each ran in a launch of its own
            assert np.count_nonzero(res["batch"] == res["batch"][i]) == 1
        _check_outputs(o, req, res, outs, verify)
    for i in (20, 46):
        n, rb, seed = int(req["n"][i]), int(req["range_bits"][i]), int(req["seed"][i])
        alone = bs.sort(bs.generate(n, rb, seed), rb)
        np.testing.assert_array_equal(to_np(alone), to_np(outs[i])[:n])


def test_poisson_trace_and_rejection(o):
    req = serve.make_trace(120, 1000, 1 << 18, 4e4, 0x5E2)
    req["n"][10] = 1 << 24
    req["range_bits"][10] = 27  # 128 MiB of keys and output: over the budget
    budget = 64 << 20
    outs = _sentinel_outputs(req)
    outs[10] = None
    res, st = serve.run(req, budget, streams=2, verify=True, outputs=outs)
    assert res["flags"][10] == 8
    ok = np.arange(len(req)) != 10
    assert np.all(res["flags"][ok] == 0)
    assert st["peak_bytes"] <= budget
    assert np.all(res["done_s"][ok] >= res["launch_s"][ok])
    assert np.all(res["launch_s"][ok] + 1e-3 >= req["arrival_s"][ok])
    keep = np.nonzero(ok)[0]
    _check_outputs(o, req[keep], res[keep], [outs[i] for i in keep])


def test_device_digest_matches_host():
    import torch
    v = np.random.default_rng(3).integers(0, 1 << 32, size=300_001, dtype=np.uint64).astype(np.uint32)
    t = torch.from_numpy(v.view(np.int32)).cuda()
    assert serve.digest(t) == serve.host_digest(v)
    assert serve.digest(t[:0]) == 0
