#!/usr/bin/env python3
"""Benchmark of the bitmap sort on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]

A step is one bitsort_u32 call (partition + slice kernels) over one array
already resident in HBM; inputs rotate through a pool of device buffers whose
total exceeds the 256 MB Infinity Cache.  Prints one JSON line with the
whole-job throughput (Gkeys/s), the dominant kernel's roofline against the
8 TB/s HBM3E peak (its duration measured with HIP events on its own stream),
and the CPU oracle timed on this host's cores as a reported baseline.

With no --workload, the headline is plain-small (10^6 keys, the workload the
roofline target is set on) and the same JSON line carries, under "extras",
plain-uniform (value and roofline fractions), both through the atomic-OR
mark, bitmap-pairs (the 2^26 keys with a value each), the batch workload (one
batched launch against 4096 plain launches, identical results) and the
serving trace (throughput, p50/p99 latency); --no-extras leaves them out.

Workloads:
  plain-uniform   2^26 distinct keys uniform without replacement in [0, 2^28)
  plain-small     10^6 distinct keys in [0, 2^24)
  plain-clustered keys from 64 Gaussian clusters (sigma 2^16) in [0, 2^28)
  plain-dense     a permutation of all of [0, 2^28)
  plain-sparse    2^24 distinct keys in [0, 2^32)
  radix-uniform   2^26 uint32 keys uniform in [0, 2^32) with repeats, through
                  the LSD radix sort (the paper's Algorithm 1, 8-bit digits)
  radix-sparse    the plain-sparse input through the LSD radix sort
  radix-u64       2^25 uint64 keys through the 64-bit radix sort (8 passes)
  radix-pairs     2^26 uint32 keys with uint32 values (key-value radix sort)
  bitmap-pairs    2^26 distinct keys in [0, 2^28), each with a uint32 value,
                  through the bitmap sort of key-value records
  signed-uniform  2^26 distinct int32 keys in [-2^27, 2^27), signed bitmap sort
  count-uniform   2^26 keys in [0, 2^24) with repeats, counting (multiset) sort
  batch           4096 arrays, sizes log-uniform in [256, 2^20], range the
                  power of two >= 4n: one batched launch vs 4096 plain launches
  serve           20,000 sort requests, sizes log-uniform in [2^10, 2^24],
                  range the power of two >= 4n, Poisson arrivals at 70% of the
                  loop's measured burst throughput, 64 GiB device budget; one
                  step is the whole trace (keys/s, p50/p99 latency)
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "sorted Gkeys/s and % of HBM roofline at 1 GPU; batched vs per-array plain, p99"
HBM_PEAK_GBPS = 8000.0
MALL_BYTES = 256 << 20

PLAIN = {
    "plain-uniform": dict(n=1 << 26, rb=28, cfg=2, desc="2^26 distinct uint32 keys uniform in [0, 2^28), 32 MiB bit-vector"),
    "plain-small": dict(n=1_000_000, rb=24, cfg=1, desc="10^6 distinct uint32 keys uniform in [0, 2^24), 2 MiB bit-vector"),
    "plain-clustered": dict(n=None, rb=28, cfg=2, desc="64 Gaussian clusters (sigma 2^16) in [0, 2^28), 2^26 draws de-duplicated"),
    "plain-dense": dict(n=1 << 28, rb=28, cfg=3, desc="permutation of all of [0, 2^28)"),
    "plain-sparse": dict(n=1 << 24, rb=32, cfg=3, desc="2^24 distinct uint32 keys uniform in [0, 2^32), 512 MiB bit-vector"),
    "radix-uniform": dict(n=1 << 26, rb=32, cfg=6, sorter="radix",
                          desc="2^26 uint32 keys uniform in [0, 2^32) with repeats; LSD radix, 4 passes of 8-bit digits"),
    "radix-sparse": dict(n=1 << 24, rb=32, cfg=3, sorter="radix",
                         desc="the plain-sparse input (2^24 distinct keys in [0, 2^32)) through the LSD radix sort"),
    "radix-u64": dict(n=1 << 25, rb=64, cfg=7, sorter="radix64",
                      desc="2^25 uint64 keys uniform in [0, 2^64) with repeats; LSD radix, 8 passes"),
    "radix-pairs": dict(n=1 << 26, rb=32, cfg=8, sorter="pairs",
                        desc="2^26 uint32 keys uniform in [0, 2^32) with repeats, each with a uint32 value; 4 passes"),
    "bitmap-pairs": dict(n=1 << 26, rb=28, cfg=2, sorter="bitmap_pairs",
                         desc="2^26 distinct uint32 keys uniform in [0, 2^28), each with a uint32 value; bitmap sort "
                              "of the records"),
    "signed-uniform": dict(n=1 << 26, rb=28, cfg=9, sorter="signed",
                           desc="2^26 distinct int32 keys uniform in [-2^27, 2^27); bitmap sort with the signed shift"),
    "count-uniform": dict(n=1 << 26, rb=24, cfg=10, sorter="count",
                          desc="2^26 uint32 keys uniform in [0, 2^24), about 4 repeats per value; counting sort"),
}


KERNEL_SOURCES = {
    "plain": ["bitsort_device.h", "plain_kernels.inc"],
    "batch": ["bitsort_device.h", "plain_kernels.inc", "batch_kernels.inc"],
    "radix": ["bitsort_device.h", "radix_kernels.inc"],
    "count": ["bitsort_device.h", "plain_kernels.inc", "count_kernels.inc"],
    "pairs": ["bitsort_device.h", "plain_kernels.inc", "pairs_kernels.inc"],
}


def source_digest(which: str = "plain") -> str:
    """Digest of the device sources a workload's kernels are built from: a
    stored counter reading is used only while it matches."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1312_0138_amd", "csrc")
    for name in KERNEL_SOURCES[which]:
        with open(os.path.join(csrc, name), "rb") as f:
            h.update(name.encode())
            h.update(f.read())
    return h.hexdigest()[:16]


def algorithmic_bytes(n: int, rb: int, emit_path: str) -> dict:
    """The method's bytes: keys in (4n), one pass over the R-bit bit-vector
    (R/8), keys out (4n).  Per kernel, the bytes its step must move:
    k_partition reads the keys; on the LDS emit path k_slice owns the
    bit-vector pass and writes the keys; on the HBM bit-vector path k_slice
    writes the bit-vector once and k_emit reads it once and writes the keys."""
    r8 = (1 << rb) // 8
    ab = {"k_partition": 4 * n, "k_direct": 4 * n + r8 + 4 * n, "path": 4 * n + r8 + 4 * n, "k_finish": 0}
    if emit_path == "hbm-bitvector":
        ab.update({"k_slice": r8, "k_emit": r8 + 4 * n})
    else:
        ab.update({"k_slice": r8 + 4 * n})
    return ab


def atomic_algorithmic_bytes(n: int, rb: int) -> dict:
    """The same method's bytes on the atomic-mark path: the mark reads the
    keys (4n), the chunk counts make the bit-vector pass (R/8), the emission
    writes the keys (4n); its second read of the bit-vector is overhead."""
    r8 = max(1 << rb, 1 << 15) // 8
    return {"k_mark_atomic": 4 * n, "k_chunk_count": r8, "k_chunk_scan": 0, "k_emit": 4 * n,
            "path": 4 * n + (1 << rb) // 8 + 4 * n}


def radix_algorithmic_bytes(n: int, key_bits: int, elem_bytes: int = 4) -> dict:
    """The LSD radix sort's own bytes: every digit pass reads and writes the
    n elements once (2 x elem_bytes x n: 8n for uint32 keys, 16n for uint64
    keys or key-value records); the histogram pass and look-back state are
    overhead."""
    passes = (key_bits + 7) // 8
    e = elem_bytes
    return {"k_radix_pass": 2 * e * n, "k_radix_hist": 0, "k_radix_scan": 0, "path": passes * 2 * e * n}


def pairs_algorithmic_bytes(n: int, rb: int, emit_path: str) -> dict:
    """The bitmap sort of key-value records: keys and values in (8n), one pass
    over the bit-vector (R/8), keys and values out (8n).  Records route: the
    partition reads the records, the slice step makes the bit-vector pass and
    writes them.  Table route: the plain sort's kernels as for the keys alone,
    the scatter credited with the values in and the gather with the values out."""
    r8 = (1 << rb) // 8
    ab = algorithmic_bytes(n, rb, emit_path)
    ab.update({"k_partition_kv": 8 * n, "k_slice_kv": r8 + 8 * n, "k_pairs_finish": 0,
               "k_pairs_scatter": 4 * n, "k_pairs_gather": 4 * n, "path": ab["path"] + 8 * n})
    return ab


def count_algorithmic_bytes(n: int, rb: int) -> dict:
    """The counting sort credited like the bitmap: keys in, one pass over the
    key range's presence (R/8), keys out; the counters themselves stay in LDS."""
    r8 = (1 << rb) // 8
    return {"k_partition": 4 * n, "k_count_slice": r8 + 4 * n, "k_finish": 0, "path": 8 * n + r8}


def read_traffic(kernel: str, workload: str, digest: str):
    """HBM bytes per launch from the committed rocprofv3 counter summary, or
    None when there is none or the kernel sources changed since."""
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel}_{workload}.txt")
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get("source_digest") != digest:
        return None
    try:
        return int(float(vals["hbm_bytes_per_launch"]))
    except (KeyError, ValueError):
        return None


PAIRS = ("pairs", "bitmap_pairs")


def cpu_baseline(host, sorter: str, rb: int, budget_s: float = 12.0, max_reps: int = 5):
    """The oracle, single-threaded, timed on the host: (Gkeys/s, reps, median s, out)."""
    import oracle
    fn = oracle_fn(oracle.default(), sorter, rb)
    n = host[0].size if sorter in PAIRS else host.size
    times, out = [], None
    t_start = time.perf_counter()
    for _ in range(max_reps):
        t0 = time.perf_counter()
        out = fn(host)
        times.append(time.perf_counter() - t0)
        if time.perf_counter() - t_start > budget_s:
            break
    med = statistics.median(times)
    return n / med / 1e9, len(times), med, out


def make_plain_inputs(bs, torch, spec, workload, pool):
    """Device input buffers (a tuple of keys and values for the pairs sort)."""
    from paper_1312_0138_amd import inputs
    n, rb, cfg = spec["n"], spec["rb"], spec["cfg"]
    sorter = spec.get("sorter", "bitmap")
    bufs = []
    if sorter in ("radix64", "pairs", "count") or workload in ("radix-uniform", "plain-clustered"):
        reps = 1 if workload == "plain-clustered" else pool
        for rep in range(reps):
            host = host_input(spec, workload, n, rep)
            if sorter == "pairs":
                bufs.append(tuple(torch.from_numpy(h.view("int32")).cuda() for h in host))
            elif sorter == "radix64":
                bufs.append(torch.from_numpy(host.view("int64")).cuda())
            else:
                bufs.append(torch.from_numpy(host.view("int32")).cuda())
        n = host[0].size if sorter == "pairs" else host.size
        while len(bufs) < pool:
            bufs.append(bufs[0].clone())
        return bufs, n
    for rep in range(pool):
        t = torch.empty(n, dtype=torch.int32, device="cuda")
        bs.generate(n, rb, inputs.config_seed(cfg, rep), out=t)
        if sorter == "signed":
            t -= 1 << (rb - 1)  # onto [-2^(rb-1), 2^(rb-1))
        if sorter == "bitmap_pairs":  # value of record i: i + rep
            t = (t, torch.arange(rep, rep + n, dtype=torch.int32, device="cuda"))
        bufs.append(t)
    return bufs, n


def host_input(spec, workload, n, rep=0):
    """The same inputs on the host (numpy), for the oracle."""
    import numpy as np

    from paper_1312_0138_amd import inputs
    rb, cfg = spec["rb"], spec["cfg"]
    sorter = spec.get("sorter", "bitmap")
    rng = np.random.default_rng(inputs.config_seed(cfg, rep))
    if workload == "radix-uniform" or sorter == "pairs":
        keys = rng.integers(0, 1 << 32, size=n, dtype=np.uint64).astype(np.uint32)
        return (keys, np.arange(n, dtype=np.uint32)) if sorter == "pairs" else keys
    if sorter == "radix64":
        return rng.integers(0, 1 << 64, size=n, dtype=np.uint64)
    if sorter == "count":
        return rng.integers(0, 1 << rb, size=n, dtype=np.uint64).astype(np.uint32)
    if workload == "plain-clustered":
        return inputs.clustered(1 << 26, rb, inputs.config_seed(cfg, 1))
    keys = inputs.distinct_uniform(n, rb, inputs.config_seed(cfg, rep))
    if sorter == "bitmap_pairs":
        return keys, np.arange(rep, rep + n, dtype=np.uint32)
    if sorter == "signed":
        return (keys.astype(np.int64) - (1 << (rb - 1))).astype(np.int32)
    return keys


def sort_fn(bs, sorter):
    """The library call a step makes: fn(input buffer, rb, output buffer)."""
    return {
        "bitmap": lambda x, rb, out: bs.sort(x, rb, out),
        "atomic": lambda x, rb, out: bs.sort_atomic(x, rb, out),
        "signed": lambda x, rb, out: bs.sort_signed(x, rb, out),
        "count": lambda x, rb, out: bs.sort_multiset(x, rb, out),
        "radix": lambda x, rb, out: bs.radix_sort(x, rb, out),
        "radix64": lambda x, rb, out: bs.radix_sort_u64(x, rb, out),
        "pairs": lambda x, rb, out: bs.radix_sort_pairs(x[0], x[1], rb, out[0], out[1]),
        "bitmap_pairs": lambda x, rb, out: bs.sort_pairs(x[0], x[1], rb, out[0], out[1]),
    }[sorter]


def oracle_fn(o, sorter, rb):
    """The oracle's version of the same sort: fn(host input) -> expected output."""
    import numpy as np
    if sorter == "signed":
        def signed(keys):
            shift = 1 << (rb - 1)
            out, _, _ = o.bitmap_sort((keys.astype(np.int64) + shift).astype(np.uint32), rb)
            return (out.astype(np.int64) - shift).astype(np.int32)
        return signed
    return {
        "bitmap": lambda keys: o.bitmap_sort(keys, rb)[0],
        "atomic": lambda keys: o.bitmap_sort(keys, rb)[0],
        "count": lambda keys: o.counting_sort(keys, rb)[0],
        "radix": lambda keys: o.bitwise_sort1(keys, rb),
        "radix64": lambda keys: o.bitwise_sort1_u64(keys, rb),
        "pairs": lambda kv: o.bitwise_sort1_pairs(kv[0], kv[1], rb),
        "bitmap_pairs": lambda kv: o.bitwise_sort1_pairs(kv[0], kv[1], rb),
    }[sorter]


ORACLE_KIND = {
    "bitmap": "single-threaded C oracle (bitmap sort)",
    "atomic": "single-threaded C oracle (bitmap sort)",
    "signed": "single-threaded C oracle (bitmap sort of the shifted keys)",
    "count": "single-threaded C oracle (counting sort)",
    "radix": "single-threaded C oracle (Algorithm 1, one-bit passes)",
    "radix64": "single-threaded C oracle (Algorithm 1 for uint64, 64 one-bit passes)",
    "pairs": "single-threaded C oracle (Algorithm 1 on key-value records)",
    "bitmap_pairs": "single-threaded C oracle (Algorithm 1 on key-value records, range_bits passes)",
}


def bench_plain(args, workload):
    import numpy as np
    import torch

    import paper_1312_0138_amd as bs
    from paper_1312_0138_amd import _lib

    spec = PLAIN[workload]
    rb = spec["rb"]
    sorter = spec.get("sorter", "bitmap")
    if getattr(args, "mark", "partition") == "atomic":
        if sorter != "bitmap":
            raise SystemExit("--mark atomic applies to the unsigned bitmap workloads")
        sorter = "atomic"
    bitmap_like = sorter in ("bitmap", "signed", "atomic")
    radix = sorter in ("radix", "radix64", "pairs")
    sort = sort_fn(bs, sorter)
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    elem = {"radix64": 8, "pairs": 8, "bitmap_pairs": 8}.get(sorter, 4)
    pool = args.pool
    if pool == 0:
        per = elem * (spec["n"] or (1 << 26))
        pool = max(2, min(128, -(-2 * MALL_BYTES // per)))
    bufs, n = make_plain_inputs(bs, torch, spec, workload, pool)
    if sorter in PAIRS:
        out = (torch.empty(n, dtype=torch.int32, device="cuda"), torch.empty(n, dtype=torch.int32, device="cuda"))
    else:
        out = torch.empty_like(bufs[0])
    tuned = bs.autotune(n, rb, reps=3) if args.autotune and sorter == "bitmap" else None
    plan = bs.plan_info(n, rb) if bitmap_like else None

    graphs = None
    if args.graph and sorter == "bitmap":
        # one captured graph per input buffer: replays allocate and launch nothing else
        graphs = [bs.Graph.plain(b, rb, out) for b in bufs]

    def step(i):
        if graphs is not None:
            graphs[i % len(graphs)].launch()
        else:
            sort(bufs[i % len(bufs)], rb, out)

    for i in range(args.warmup):
        step(i)
    torch.cuda.synchronize()

    # Timed region 1 (the reported value): K back-to-back sorts, bracketed by
    # two events on the stream, nothing else in between.
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0.record(stream)
    for i in range(args.steps):
        step(i)
    t1.record(stream)
    torch.cuda.synchronize()
    total_ms = t0.elapsed_time(t1)
    if graphs is not None:
        (flags, count), = graphs[(args.steps - 1) % len(graphs)].status()
    else:
        st = bs.status()
        flags, count = st.flags, st.count
    assert flags == 0 and count == n, f"device status flags={flags} count={count}"

    # Timed region 2: the same K sorts with every kernel bracketed by HIP
    # events on its own stream (library profiling) and per-step events: the
    # kernels' average durations and the step-time distribution.
    _lib.check(_lib.bitsort_profile_reset(), "profile_reset")
    _lib.check(_lib.bitsort_profile_enable(True), "profile_enable")
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    torch.cuda.synchronize()
    for i in range(args.steps):
        starts[i].record(stream)
        sort(bufs[i % len(bufs)], rb, out)  # eager calls: kernels timed by library events
        ends[i].record(stream)
    torch.cuda.synchronize()
    _lib.check(_lib.bitsort_profile_enable(False), "profile_enable")
    rc, prof = _lib.bitsort_profile_read()
    _lib.check(rc, "profile_read")
    step_ms = sorted(s.elapsed_time(e) for s, e in zip(starts, ends))
    p50 = step_ms[len(step_ms) // 2]
    p99 = step_ms[min(len(step_ms) - 1, int(round(0.99 * (len(step_ms) - 1))))]

    ms_per_step = total_ms / args.steps
    value = n / (ms_per_step / 1e3) / 1e9
    if radix:
        ab = radix_algorithmic_bytes(n, rb, elem)
    elif sorter == "count":
        ab = count_algorithmic_bytes(n, rb)
    elif sorter == "bitmap_pairs":
        ab = pairs_algorithmic_bytes(n, rb, bs.plan_info(n, rb)["emit_path"])
    elif sorter == "atomic":
        ab = atomic_algorithmic_bytes(n, rb)
    else:
        ab = algorithmic_bytes(n, rb, plan["emit_path"])
    kernels = {k: {"launches": int(l), "avg_us": round(1e3 * ms / max(l, 1), 3)} for k, (l, ms) in prof.items()}
    dom = max(prof, key=lambda k: prof[k][1])
    dom_avg_s = prof[dom][1] / prof[dom][0] / 1e3
    digest = source_digest("radix" if radix else {"count": "count", "bitmap_pairs": "pairs"}.get(sorter, "plain"))
    achieved = ab[dom] / dom_avg_s / 1e9
    roofline = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBPS, 4),
                "traffic": read_traffic(dom, workload, digest), "algorithmic_bytes": ab[dom]}
    path_gbps = ab["path"] / (ms_per_step / 1e3) / 1e9
    if sorter == "atomic":
        config = {"workload": workload, "description": spec["desc"], "n": n, "range_bits": rb,
                  "input_pool": len(bufs), "mark": "atomic OR into the HBM bit-vector (bitsort_u32_atomic)"}
    elif bitmap_like:
        config = {"workload": workload, "description": spec["desc"], "n": n, "range_bits": rb,
                  "input_pool": len(bufs), "slice_bits": plan["slice_bits"], "tile_log2": plan["tile_log2"],
                  "slices": plan["buckets"], "emit_path": plan["emit_path"]}
    else:
        config = {"workload": workload, "description": spec["desc"], "n": n,
                  ("key_bits" if radix else "range_bits"): rb, "input_pool": len(bufs)}
        if radix:
            config["passes"] = (rb + 7) // 8
    result = {
        "metric": METRIC, "value": round(value, 3), "unit": "Gkeys/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_per_step, 5), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": {"signed": "i32", "radix64": "u64", "pairs": "u32+u32", "bitmap_pairs": "u32+u32"}.get(sorter, "u32"),
        "data": "synthetic",
        "config": config,
        "p50_ms": round(p50, 5), "p99_ms": round(p99, 5),
        "profiled_ms_per_step": round(sum(step_ms) / len(step_ms), 5),
        "roofline": roofline,
        "roofline_path": {"achieved": round(path_gbps, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                          "frac": round(path_gbps / HBM_PEAK_GBPS, 4), "algorithmic_bytes": ab["path"]},
        "kernels": kernels, "source_digest": digest, "tuning": args.tune or "default",
        "launch": "hip-graph replay" if graphs is not None else "eager calls",
        "autotuned": tuned,
    }
    if not args.no_cpu_baseline:
        host = host_input(spec, workload, n)
        gk, reps, med, want = cpu_baseline(host, sorter, rb)
        # the GPU result for the same input must equal the oracle's
        if sorter in PAIRS:
            dev = tuple(torch.from_numpy(h.view(np.int32)).cuda() for h in host)
            got_k, got_v = sort(dev, rb, (torch.empty_like(dev[0]), torch.empty_like(dev[1])))
            same = (np.array_equal(got_k.cpu().numpy().view(np.uint32), want[0])
                    and np.array_equal(got_v.cpu().numpy().view(np.uint32), want[1]))
        else:
            view = {"radix64": np.int64, "signed": np.int32}.get(sorter, np.int32)
            dev = torch.from_numpy(host.view(view)).cuda()
            got = sort(dev, rb, torch.empty_like(dev)).cpu().numpy().view(want.dtype)
            same = np.array_equal(got, want)
        if not same:
            print(json.dumps({"error": "GPU output differs from the CPU oracle", "workload": workload}))
            sys.exit(3)
        result["cpu_baseline"] = {"value": round(gk, 4), "unit": "Gkeys/s", "cores": 1, "kind": "oracle",
                                  "sample": f"full {workload} input (n={n}), {reps} repetition(s), "
                                            f"median {med:.3f} s per sort; {ORACLE_KIND[sorter]}",
                                  "host_cores": os.cpu_count()}
        result["verified_against_oracle"] = True
    return result


def bench_batch(args):
    import numpy as np
    import torch

    import paper_1312_0138_amd as bs
    from paper_1312_0138_amd import _lib, inputs

    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    count, seed = 4096, inputs.config_seed(4, 0)
    sizes = inputs.log_uniform_sizes(count, 256, 1 << 20, seed)
    rbits = np.array([inputs.range_bits_for(n) for n in sizes], dtype=np.uint8)
    offsets = np.zeros(count + 1, dtype=np.uint64)
    offsets[1:] = np.cumsum(sizes)
    total = int(offsets[-1])
    keys = torch.empty(total, dtype=torch.int32, device="cuda")
    for i in range(count):
        lo, hi = int(offsets[i]), int(offsets[i + 1])
        bs.generate(hi - lo, int(rbits[i]), inputs.segment_seed(seed, i), out=keys[lo:hi])
    off_d = torch.from_numpy(offsets.astype(np.int64)).cuda()
    rb_d = torch.from_numpy(rbits).cuda()
    out_b = torch.empty_like(keys)
    out_p = torch.empty_like(keys)
    views = [(keys[int(offsets[i]):int(offsets[i + 1])], out_p[int(offsets[i]):int(offsets[i + 1])], int(rbits[i]))
             for i in range(count)]

    def run_batch():
        bs.sort_batch(keys, off_d, rb_d, out_b)

    out_g = torch.empty_like(keys)
    graph = bs.Graph.batch(keys, off_d, rb_d, out_g)

    def run_graph():
        graph.launch()

    def run_plain():
        for k, o, rb in views:
            bs.sort(k, rb, o)

    # the same segments as separate arrays through the pointer-array batch
    # (bitsort_batch_ptr_u32), its pointer arrays built once on the host
    out_m = torch.empty_like(keys)
    kp = (keys.data_ptr() + 4 * offsets[:-1]).astype(np.uint64)
    op = (out_m.data_ptr() + 4 * offsets[:-1]).astype(np.uint64)
    nn = sizes.astype(np.uint64)
    sid = int(stream.cuda_stream)

    def run_pointer_array():
        _lib.check(_lib.bitsort_batch_ptr_u32(kp.ctypes.data, nn.ctypes.data, rbits.ctypes.data, op.ctypes.data,
                                              count, sid), "bitsort_batch_ptr_u32")

    if args.autotune:
        res_tune = bs.autotune_batch(keys, off_d, rb_d, out_b, reps=2)
    for _ in range(args.warmup):
        run_batch()
        run_graph()
        run_plain()
        run_pointer_array()
    torch.cuda.synchronize()
    res = {}
    for name, fn in (("batched", run_batch), ("batched_graph", run_graph), ("plain_loop", run_plain),
                     ("pointer_array", run_pointer_array)):
        times = []
        for _ in range(max(3, args.steps // 10)):
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record(stream)
            fn()
            b.record(stream)
            torch.cuda.synchronize()
            times.append(a.elapsed_time(b))
        times.sort()
        med = times[len(times) // 2]
        res[name] = {"median_ms": round(med, 4), "p99_ms": round(times[-1], 4),
                     "gkeys_per_s": round(total / (med / 1e3) / 1e9, 3)}
    flags, counts = bs.batch_status(count)  # of the last call: the pointer-array batch
    assert not flags.any() and np.array_equal(counts, sizes.astype(np.uint64))
    same = torch.equal(out_b, out_p) and torch.equal(out_g, out_p) and torch.equal(out_m, out_p)
    ab = sum(4 * int(n) + (1 << int(r)) // 8 + 4 * int(n) for n, r in zip(sizes, rbits))
    med_s = res["batched"]["median_ms"] / 1e3
    return {
        "metric": METRIC, "value": res["batched"]["gkeys_per_s"], "unit": "Gkeys/s", "n_gpus": 1,
        "steps": max(3, args.steps // 10), "warmup": args.warmup, "ms_per_step": res["batched"]["median_ms"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u32", "data": "synthetic",
        "config": {"workload": "batch", "segments": count, "total_keys": total,
                   "sizes": "log-uniform in [256, 2^20]", "range": "next power of two >= 4n"},
        "batched": res["batched"], "batched_graph": res["batched_graph"], "plain_loop": res["plain_loop"],
        "pointer_array": res["pointer_array"],
        "autotuned": res_tune if args.autotune else None,
        "batched_over_plain": round(res["plain_loop"]["median_ms"] / res["batched"]["median_ms"], 3),
        "identical_results": bool(same),
        "roofline_path": {"achieved": round(ab / med_s / 1e9, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                          "frac": round(ab / med_s / 1e9 / HBM_PEAK_GBPS, 4), "algorithmic_bytes": ab},
    }


def serve_cpu_baseline(trace, results, budget_s: float = 20.0, max_keys: int = 1 << 24):
    """The oracle sorts a seeded sample of the trace's requests (inputs
    regenerated on the host); its digests must equal the served ones."""
    import numpy as np

    import oracle
    from paper_1312_0138_amd import inputs, serve
    o = oracle.default()
    rng = np.random.default_rng(0xB5)
    keys_done, t_sort, checked, bad = 0, 0.0, 0, []
    t_start = time.perf_counter()
    for i in rng.permutation(len(trace)):
        n, rb, seed = int(trace["n"][i]), int(trace["range_bits"][i]), int(trace["seed"][i])
        if time.perf_counter() - t_start > budget_s:
            break
        if keys_done + n > max_keys:
            continue
        keys = inputs.distinct_uniform(n, rb, seed)
        t0 = time.perf_counter()
        want, flags, _ = o.bitmap_sort(keys, rb)
        t_sort += time.perf_counter() - t0
        keys_done += n
        checked += 1
        if flags != 0 or serve.host_digest(want) != int(results["digest"][i]):
            bad.append(int(i))
    return keys_done / t_sort / 1e9, checked, keys_done, t_sort, bad


def bench_serve(args, oracle_check_s: float = 20.0):
    import math

    import numpy as np
    import torch

    from paper_1312_0138_amd import inputs, serve

    torch.cuda.set_device(0)
    count, lo, hi, budget = args.serve_requests, 1 << 10, 1 << 24, 64 << 30
    streams = args.serve_streams
    seed = inputs.config_seed(5, 0)
    # burst calibration on a 512-request sample of the same size distribution
    cal = serve.make_trace(512, lo, hi, math.inf, inputs.config_seed(5, 1))
    serve.run(cal[:64], budget, streams=streams)
    _, st_cal = serve.run(cal, budget, streams=streams)
    t_burst = st_cal["keys"] / st_cal["makespan_s"]
    _, st_one = serve.run(cal, budget, streams=1, max_batch_requests=1)
    t_one = st_one["keys"] / st_one["makespan_s"]
    trace = serve.make_trace(count, lo, hi, 1.0, seed)
    rate = 0.7 * t_burst / float(trace["n"].mean())
    trace["arrival_s"] = inputs.poisson_arrivals(count, rate, seed + 1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res, st = serve.run(trace, budget, streams=streams)
    wall = time.perf_counter() - t0
    summ = serve.summarize(trace, res, st)
    # the same trace again with every request's output digested on the device
    res_v, st_v = serve.run(trace, budget, streams=streams, verify=True)
    ok = bool(np.all(res_v["flags"] == 0) and np.array_equal(res_v["count"], trace["n"]))
    out = {
        "metric": METRIC, "value": round(summ["gkeys_per_s"], 3), "unit": "Gkeys/s", "n_gpus": 1, "steps": 1,
        "warmup": 1, "ms_per_step": round(st["makespan_s"] * 1e3, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u32", "data": "synthetic",
        "config": {"workload": "serve", "requests": count, "sizes": "log-uniform in [2^10, 2^24]",
                   "range": "next power of two >= 4n", "arrivals": f"Poisson, {rate:.1f} requests/s",
                   "budget_bytes": budget, "streams": streams, "total_keys": int(trace["n"].sum())},
        "latency_ms": {"p50": round(summ["p50_ms"], 4), "p99": round(summ["p99_ms"], 4),
                       "mean_queue": round(summ["mean_queue_ms"], 4),
                       "mean_launch_to_keys_ready": round(summ["mean_launch_to_keys_ready_ms"], 4),
                       "keys_ready_share": round(summ["keys_ready_share_of_latency"], 4)},
        "launches": summ["launches"], "max_inflight_requests": summ["max_inflight_requests"],
        "requests_per_launch": summ["requests_per_launch"],
        "peak_bytes": summ["peak_bytes"], "host_wall_s": round(wall, 3),
        "calibration": {"burst_gkeys_per_s": round(t_burst / 1e9, 3),
                        "one_request_per_launch_gkeys_per_s": round(t_one / 1e9, 3),
                        "burst_over_one_by_one": round(t_burst / t_one, 3), "requests": 512},
        "verify_run": {"all_counts_and_flags_ok": ok, "gkeys_per_s": round(st_v["keys"] / st_v["makespan_s"] / 1e9, 3)},
    }
    gk, checked, keys_done, t_sort, bad = serve_cpu_baseline(trace, res_v, budget_s=oracle_check_s)
    sample = (f"{checked} requests of the trace ({keys_done} keys) sorted by the oracle, "
              f"{t_sort:.2f} s; inputs regenerated on the host")
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = {"value": round(gk, 4), "unit": "Gkeys/s", "cores": 1, "kind": "oracle",
                               "sample": sample}
    out["oracle_sample"] = sample
    out["oracle_digests_match"] = not bad
    if bad:
        out["oracle_mismatch_requests"] = bad[:20]
    return out


def copy_calibration(args):
    """A plain device copy of known size (1 GiB read + 1 GiB written per
    launch), for scaling rocprofv3's FETCH_SIZE / WRITE_SIZE counters and as
    the practical bandwidth ceiling."""
    import torch
    nbytes = 1 << 30
    src = torch.empty(nbytes // 4, dtype=torch.int32, device="cuda").fill_(7)
    dst = torch.empty_like(src)
    for _ in range(2):
        dst.copy_(src)
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    reps = max(3, args.steps // 10)
    a.record()
    for _ in range(reps):
        dst.copy_(src)
    b.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / reps
    return {"workload": "copy-calibration", "bytes_read_per_launch": nbytes, "bytes_written_per_launch": nbytes,
            "ms_per_copy": round(ms, 4), "copy_GBps": round(2 * nbytes / (ms / 1e3) / 1e9, 1), "launches": reps + 2}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default=None, choices=sorted(PLAIN) + ["batch", "serve", "copy-calibration"],
                    help="one workload only (default: plain-small plus the extras)")
    ap.add_argument("--no-extras", action="store_true", help="default run: the headline workload only")
    ap.add_argument("--serve-requests", type=int, default=20000)
    ap.add_argument("--serve-streams", type=int, default=4)
    ap.add_argument("--pool", type=int, default=0, help="input buffers to rotate through (0: auto)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--tune", default="", help="slice_bits,tile_log2,emit_path (0 = library choice)")
    ap.add_argument("--graph", action="store_true", help="time HIP-graph replays instead of eager calls")
    ap.add_argument("--mark", default="partition", choices=["partition", "atomic"],
                    help="bitmap workloads: the partitioned LDS mark (default) or the atomic-OR HBM mark")
    ap.add_argument("--autotune", action="store_true", help="run the autotuner for the workload first")
    args = ap.parse_args()
    if args.tune:
        import paper_1312_0138_amd as bs
        bs.set_tuning(*[int(v) for v in args.tune.split(",")])
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (run with --gpus 1)", file=sys.stderr)
        sys.exit(2)
    if args.workload is None:
        result = bench_plain(args, "plain-small")
        if not args.no_extras:
            result["extras"] = bench_extras(args)
    elif args.workload == "batch":
        result = bench_batch(args)
    elif args.workload == "serve":
        result = bench_serve(args)
    elif args.workload == "copy-calibration":
        result = copy_calibration(args)
    else:
        result = bench_plain(args, args.workload)
    print(json.dumps(result), flush=True)


def bench_extras(args):
    """The rest of the metric beside the headline: the 2^26-key workload (also
    through the atomic-OR mark, and as key-value records), the batch against
    per-array launches, and the serving trace (each its own run; CPU
    baselines left to the single-workload runs)."""
    import copy
    sub = copy.copy(args)
    sub.no_cpu_baseline = True
    sub.autotune = False
    sub.graph = False
    sub.steps = max(10, min(args.steps, 50))
    sub.warmup = max(2, min(args.warmup, 5))
    t0 = time.perf_counter()
    big = bench_plain(sub, "plain-uniform")
    print(f"extras: plain-uniform done in {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
    atomic = {}
    for wl in ("plain-small", "plain-uniform"):
        t0 = time.perf_counter()
        sub_a = copy.copy(sub)
        sub_a.mark = "atomic"
        r = bench_plain(sub_a, wl)
        atomic[wl] = {"value": r["value"], "unit": "Gkeys/s", "ms_per_step": r["ms_per_step"],
                      "roofline": r["roofline"], "roofline_path": r["roofline_path"], "kernels": r["kernels"]}
        print(f"extras: atomic {wl} done in {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    kv = bench_plain(sub, "bitmap-pairs")
    print(f"extras: bitmap-pairs done in {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    batch = bench_batch(sub)
    print(f"extras: batch done in {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    srv = bench_serve(sub, oracle_check_s=5.0)
    print(f"extras: serve done in {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
    return {
        "plain-uniform": {"value": big["value"], "unit": "Gkeys/s", "ms_per_step": big["ms_per_step"],
                          "steps": big["steps"], "config": big["config"], "roofline": big["roofline"],
                          "roofline_path": big["roofline_path"], "kernels": big["kernels"]},
        "atomic_mark": atomic,
        "bitmap-pairs": {"value": kv["value"], "unit": "Gkeys/s", "ms_per_step": kv["ms_per_step"],
                         "steps": kv["steps"], "config": kv["config"], "roofline": kv["roofline"],
                         "roofline_path": kv["roofline_path"], "kernels": kv["kernels"]},
        "batch": {"value": batch["value"], "unit": "Gkeys/s", "config": batch["config"],
                  "batched": batch["batched"], "batched_graph": batch["batched_graph"],
                  "plain_loop": batch["plain_loop"], "pointer_array": batch["pointer_array"],
                  "batched_over_plain": batch["batched_over_plain"],
                  "identical_results": batch["identical_results"], "roofline_path": batch["roofline_path"]},
        "serve": {"value": srv["value"], "unit": "Gkeys/s", "config": srv["config"],
                  "latency_ms": srv["latency_ms"], "launches": srv["launches"],
                  "calibration": srv["calibration"], "verify_run": srv["verify_run"],
                  "oracle_digests_match": srv.get("oracle_digests_match"),
                  "oracle_sample": srv.get("oracle_sample")},
    }


if __name__ == "__main__":
    main()
