"""Serving-loop driver: build a request trace, run the library's
continuous-batching loop (``bitsort_serve_run``) and summarise latencies.

The loop itself -- admission, memory budget, batching, streams, completion
timing -- is C++ in the library; this module only lays out the request
arrays and reads the results back."""
from __future__ import annotations

import math

import numpy as np

from . import _lib, inputs

REQUEST = np.dtype([("n", "<u8"), ("range_bits", "<u4"), ("pad", "<u4"), ("seed", "<u8"),
                    ("arrival_s", "<f8")])
RESULT = np.dtype([("launch_s", "<f8"), ("ready_s", "<f8"), ("done_s", "<f8"), ("digest", "<u8"),
                   ("count", "<u8"), ("flags", "<u4"), ("batch", "<u4")])
CONFIG = np.dtype([("arena", "<u8"), ("budget_bytes", "<u8"), ("streams", "<u4"), ("max_batch_requests", "<u4"),
                   ("max_batch_keys", "<u8"), ("plain_range_bits", "<u4"), ("verify", "<u4"), ("simulate", "<u4"),
                   ("pad", "<u4"),
                   ("sim_overhead_s", "<f8"), ("sim_keys_per_s", "<f8"), ("outputs", "<u8")])
STATS = np.dtype([("makespan_s", "<f8"), ("keys", "<u8"), ("launches", "<u4"),
                  ("max_inflight_requests", "<u4"), ("peak_bytes", "<u8")])
assert REQUEST.itemsize == 32 and RESULT.itemsize == 48 and CONFIG.itemsize == 72 and STATS.itemsize == 32


def make_trace(count: int, lo: int, hi: int, rate_per_s: float, seed: int, factor: int = 4) -> np.ndarray:
    """``count`` requests: sizes log-uniform in [lo, hi], range the power of
    two >= factor * n, Poisson arrivals at ``rate_per_s``, per-request seeds."""
    sizes = inputs.log_uniform_sizes(count, lo, hi, seed)
    req = np.zeros(count, dtype=REQUEST)
    req["n"] = sizes
    req["range_bits"] = [inputs.range_bits_for(int(n), factor) for n in sizes]
    req["seed"] = [inputs.segment_seed(seed, i) for i in range(count)]
    req["arrival_s"] = inputs.poisson_arrivals(count, rate_per_s, seed + 1) if math.isfinite(rate_per_s) else 0.0
    return req


_ARENA = {}


def _arena(budget_bytes: int):
    """A torch-allocated arena, kept for later calls with the same budget."""
    import torch
    t = _ARENA.get(budget_bytes)
    if t is None:
        _ARENA.clear()
        t = _ARENA[budget_bytes] = torch.empty(budget_bytes, dtype=torch.uint8, device="cuda")
    return t


def release_arena() -> None:
    _ARENA.clear()


def run(requests: np.ndarray, budget_bytes: int, streams: int = 4, max_batch_requests: int = 4096,
        max_batch_keys: int = 1 << 26, plain_range_bits: int = 0, verify: bool = False, simulate: bool = False,
        sim_overhead_s: float = 20e-6, sim_keys_per_s: float = 2e11, arena=None, outputs=None):
    """Run the trace; returns (results array, stats dict).

    The arena is ``arena`` (a uint8 device tensor of at least budget_bytes)
    or a torch allocation cached across calls; nothing is allocated when
    ``simulate`` is set.  ``outputs``: None, or one device int32/uint32 tensor
    (or None) per request, at least n long, that receives the request's
    sorted keys."""
    requests = np.ascontiguousarray(requests, dtype=REQUEST)
    res = np.zeros(max(len(requests), 1), dtype=RESULT)
    cfg = np.zeros(1, dtype=CONFIG)
    if not simulate:
        if arena is None:
            arena = _arena(budget_bytes)
        if arena.numel() * arena.element_size() < budget_bytes:
            raise ValueError("arena is smaller than budget_bytes")
        cfg["arena"] = arena.data_ptr()
    cfg["budget_bytes"] = budget_bytes
    cfg["streams"] = streams
    cfg["max_batch_requests"] = max_batch_requests
    cfg["max_batch_keys"] = max_batch_keys
    cfg["plain_range_bits"] = plain_range_bits
    cfg["verify"] = int(verify)
    cfg["simulate"] = int(simulate)
    cfg["sim_overhead_s"] = sim_overhead_s
    cfg["sim_keys_per_s"] = sim_keys_per_s
    ptrs = None
    if outputs is not None:
        if len(outputs) != len(requests):
            raise ValueError("outputs needs one entry per request")
        ptrs = np.zeros(max(len(requests), 1), dtype=np.uint64)
        for i, t in enumerate(outputs):
            if t is None:
                continue
            if not t.is_cuda or not t.is_contiguous() or t.element_size() != 4 or t.numel() < int(requests["n"][i]):
                raise ValueError(f"outputs[{i}] must be a contiguous 4-byte device tensor of at least n elements")
            ptrs[i] = t.data_ptr()
        cfg["outputs"] = ptrs.ctypes.data
    st = np.zeros(1, dtype=STATS)
    _lib.check(_lib.bitsort_serve_run(requests.ctypes.data, len(requests), cfg.ctypes.data, res.ctypes.data,
                                      st.ctypes.data), "bitsort_serve_run")
    stats = {k: st[k][0].item() for k in STATS.names}
    return res[: len(requests)], stats


def summarize(requests: np.ndarray, results: np.ndarray, stats: dict) -> dict:
    ok = (results["flags"] & (_lib.REQ_REJECTED | _lib.REQ_INVALID)) == 0
    lat = (results["done_s"] - requests["arrival_s"])[ok]
    wait = (results["launch_s"] - requests["arrival_s"])[ok]
    gen = (results["ready_s"] - results["launch_s"])[ok]
    keys = int(results["count"][ok].sum())
    per_launch = np.bincount(results["batch"][ok].astype(np.int64)) if ok.any() else np.zeros(0, np.int64)
    per_launch = per_launch[per_launch > 0]
    return {
        "requests": int(len(requests)), "served": int(ok.sum()), "rejected": int((~ok).sum()),
        "keys": keys, "makespan_s": stats["makespan_s"],
        "gkeys_per_s": keys / stats["makespan_s"] / 1e9 if stats["makespan_s"] > 0 else None,
        "p50_ms": float(np.percentile(lat, 50) * 1e3) if lat.size else None,
        "p99_ms": float(np.percentile(lat, 99) * 1e3) if lat.size else None,
        "mean_queue_ms": float(wait.mean() * 1e3) if wait.size else None,
        "mean_launch_to_keys_ready_ms": float(gen.mean() * 1e3) if gen.size else None,
        "keys_ready_share_of_latency": float(gen.sum() / lat.sum()) if lat.size and lat.sum() > 0 else None,
        "launches": stats["launches"], "max_inflight_requests": stats["max_inflight_requests"],
        "requests_per_launch": ({"mean": float(per_launch.mean()), "max": int(per_launch.max()),
                                 "hist_pow2": np.bincount(np.log2(per_launch).astype(np.int64)).tolist()}
                                if per_launch.size else None),
        "peak_bytes": stats["peak_bytes"],
    }


def digest(t, stream=None) -> int:
    """Digest of a device uint32 tensor (the function the loop uses)."""
    from . import _stream
    rc, d = _lib.bitsort_digest_u32(t.data_ptr(), t.numel(), _stream(stream))
    _lib.check(rc, "bitsort_digest_u32")
    return d


def host_digest(values: np.ndarray) -> int:
    """The same digest computed on the host (tests)."""
    v = np.ascontiguousarray(values, dtype=np.uint32).astype(np.uint64)
    i = np.arange(v.size, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = (i << np.uint64(32)) ^ v
        z = z + np.uint64(0x9E3779B97F4A7C15)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
        return int(z.sum(dtype=np.uint64))
