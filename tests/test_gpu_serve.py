"""Serving loop on the device: every request's sorted output, digested on
the device, equals the oracle's sort of the same keys and the result of
sorting that request alone, whatever batch it shared."""
import numpy as np
import pytest

import oracle
from gpu_util import require_gpu
from paper_1312_0138_amd import inputs, serve

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    require_gpu()


@pytest.fixture(scope="module")
def o():
    return oracle.default()


def _oracle_digest(o, n, rb, seed):
    keys = inputs.distinct_uniform(int(n), int(rb), int(seed))
    want, flags, _ = o.bitmap_sort(keys, int(rb))
    assert flags == 0
    return serve.host_digest(want)


def _mixed_trace(seed):
    req = serve.make_trace(160, 1, 1 << 19, float("inf"), seed)
    # a few requests wider than the batch kernel's range go through the plain path
    req["n"][17::40] = [1 << 20, 3 << 19, 1000, 1 << 21][: len(req["n"][17::40])]
    req["range_bits"][17::40] = [26, 28, 30, 25][: len(req["range_bits"][17::40])]
    req["n"][3] = 0  # an empty request
    return req


def test_mix_matches_oracle_and_alone(o):
    import torch
    import paper_1312_0138_amd as bs
    req = _mixed_trace(0x5E1)
    budget = 96 << 20  # tight: requests wait for memory
    res, st = serve.run(req, budget, streams=3, max_batch_requests=64, max_batch_keys=1 << 21, verify=True)
    assert st["peak_bytes"] <= budget
    assert np.all(res["flags"] == 0)
    np.testing.assert_array_equal(res["count"], req["n"])
    assert st["launches"] < len(req)  # some requests shared a launch
    for i in range(len(req)):
        want = _oracle_digest(o, req["n"][i], req["range_bits"][i], req["seed"][i])
        assert int(res["digest"][i]) == want, f"request {i} n={req['n'][i]} rb={req['range_bits'][i]}"
    # alone through the plain API (a different kernel path for batched requests)
    for i in [0, 1, 3, 17, 57, 100, 159]:
        n, rb, seed = int(req["n"][i]), int(req["range_bits"][i]), int(req["seed"][i])
        keys = bs.generate(n, rb, seed)
        out = bs.sort(keys, rb)
        assert serve.digest(out) == int(res["digest"][i])
    # alone through the serving loop
    for i in [2, 17, 80]:
        one, _ = serve.run(req[i:i + 1], budget, verify=True)
        assert int(one["digest"][0]) == int(res["digest"][i])
    torch.cuda.synchronize()


def test_poisson_trace_and_rejection(o):
    req = serve.make_trace(120, 1000, 1 << 18, 4e4, 0x5E2)
    req["n"][10] = 1 << 24
    req["range_bits"][10] = 27  # 128 MiB of keys and output: over the budget
    budget = 64 << 20
    res, st = serve.run(req, budget, streams=2, verify=True)
    assert res["flags"][10] == 8
    ok = np.arange(len(req)) != 10
    assert np.all(res["flags"][ok] == 0)
    assert st["peak_bytes"] <= budget
    assert np.all(res["done_s"][ok] >= res["launch_s"][ok])
    assert np.all(res["launch_s"][ok] + 1e-3 >= req["arrival_s"][ok])
    for i in np.nonzero(ok)[0][::7]:
        assert int(res["digest"][i]) == _oracle_digest(o, req["n"][i], req["range_bits"][i], req["seed"][i])


def test_device_digest_matches_host():
    import torch
    v = np.random.default_rng(3).integers(0, 1 << 32, size=300_001, dtype=np.uint64).astype(np.uint32)
    t = torch.from_numpy(v.view(np.int32)).cuda()
    assert serve.digest(t) == serve.host_digest(v)
    assert serve.digest(t[:0]) == 0
