"""ctypes binding of libbitsort.so: one Python function per C-ABI entry point,
same names, argument marshalling only.  Raises if the library is not built --
there is no fallback of any kind."""
from __future__ import annotations

import ctypes
import os
import re

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libbitsort.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "bitsort.h")

BITSORT_OK = 0
BITSORT_ERR_INVALID_ARG = 1
BITSORT_ERR_TOO_LARGE = 2
BITSORT_ERR_NO_MEMORY = 3
BITSORT_ERR_HIP = 4

STATUS_OUT_OF_RANGE = 1
STATUS_DUPLICATE = 2
STATUS_BAD_SEGMENT = 4
STATUS_TIMEOUT = 32
STATUS_BAD_STATE = 64
REQ_REJECTED = 8
REQ_INVALID = 16

BATCH_MAX_RANGE_BITS = 24


class BitsortError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        super().__init__(f"{where}: error {code} ({error_string(code) if _lib else '?'})")


class Status(ctypes.Structure):
    _fields_ = [("flags", ctypes.c_uint32), ("_pad", ctypes.c_uint32), ("count", ctypes.c_uint64)]


class Tuning(ctypes.Structure):
    _fields_ = [("slice_bits", ctypes.c_uint32), ("tile_log2", ctypes.c_uint32), ("emit_path", ctypes.c_uint32),
                ("batch_block", ctypes.c_uint32), ("ms", ctypes.c_float)]


class ProfileEntry(ctypes.Structure):
    _fields_ = [("kernel", ctypes.c_char * 32), ("launches", ctypes.c_uint64), ("total_ms", ctypes.c_double)]


_c = ctypes
_vp = ctypes.c_void_p
_u32 = ctypes.c_uint32
_u64 = ctypes.c_uint64
_SIGS = {
    "bitsort_version": (_c.c_int, []),
    "bitsort_error_string": (_c.c_char_p, [_c.c_int]),
    "bitsort_u32": (_c.c_int, [_vp, _u64, _u32, _vp, _vp]),
    "bitsort_workspace_bytes": (_c.c_size_t, [_u64, _u32]),
    "bitsort_u32_ws": (_c.c_int, [_vp, _u64, _u32, _vp, _vp, _c.c_size_t, _vp]),
    "bitsort_u32_noalloc": (_c.c_int, [_vp, _u64, _u32, _vp, _vp, _vp]),
    "bitsort_u32_atomic": (_c.c_int, [_vp, _u64, _u32, _vp, _vp]),
    "bitsort_u64": (_c.c_int, [_vp, _u64, _u32, _vp, _vp]),
    "bitsort_radix_u32": (_c.c_int, [_vp, _u64, _u32, _vp, _vp]),
    "bitsort_radix_i32": (_c.c_int, [_vp, _u64, _vp, _vp]),
    "bitsort_radix_u64": (_c.c_int, [_vp, _u64, _u32, _vp, _vp]),
    "bitsort_radix_pairs_u32": (_c.c_int, [_vp, _vp, _u64, _u32, _vp, _vp, _vp]),
    "bitsort_i32": (_c.c_int, [_vp, _u64, _u32, _vp, _vp]),
    "bitsort_count_u32": (_c.c_int, [_vp, _u64, _u32, _vp, _vp]),
    "bitsort_radix_workspace_bytes": (_c.c_size_t, [_u64, _u32]),
    "bitsort_radix_u32_ws": (_c.c_int, [_vp, _u64, _u32, _vp, _vp, _c.c_size_t, _vp]),
    "bitsort_get_status": (_c.c_int, [_vp, _c.POINTER(Status)]),
    "bitsort_workspace_status": (_c.c_int, [_vp, _vp, _c.POINTER(Status)]),
    "bitsort_batch_u32": (_c.c_int, [_vp, _vp, _u32, _vp, _vp, _u64, _vp]),
    "bitsort_batch_status": (_c.c_int, [_vp, _c.POINTER(Status), _u32]),
    "bitsort_batch_ptr_u32": (_c.c_int, [_vp, _vp, _vp, _vp, _u32, _vp]),
    "bitsort_batch_plan": (_c.c_int, [_vp, _vp, _u32, _c.POINTER(_vp)]),
    "bitsort_batch_run": (_c.c_int, [_vp, _vp, _vp, _vp, _vp, _vp]),
    "bitsort_batch_plan_status": (_c.c_int, [_vp, _vp, _c.POINTER(Status), _u32]),
    "bitsort_batch_plan_destroy": (_c.c_int, [_vp]),
    "bitsort_set_workspace": (_c.c_int, [_vp, _c.c_size_t, _vp]),
    "bitsort_generate_u32": (_c.c_int, [_vp, _u64, _u64, _u32, _u64, _vp]),
    "bitsort_debug_bitmap_u32": (_c.c_int, [_vp, _u64, _u32, _vp, _vp]),
    "bitsort_debug_prefix_u32": (_c.c_int, [_vp, _u64, _u32, _vp, _vp]),
    "bitsort_pairs_u32": (_c.c_int, [_vp, _vp, _u64, _u32, _vp, _vp, _vp]),
    "bitsort_debug_split_u32": (_c.c_int, [_vp, _u64, _u32, _c.POINTER(_u32), _vp]),
    "bitsort_set_tuning": (_c.c_int, [_u32, _u32, _u32]),
    "bitsort_plan_info": (_c.c_int, [_u64, _u32, _c.POINTER(_u32), _c.POINTER(_u32), _c.POINTER(_u32),
                                     _c.POINTER(_u32)]),
    "bitsort_graph_create_u32": (_c.c_int, [_vp, _u64, _u32, _vp, _c.POINTER(_vp)]),
    "bitsort_graph_create_batch_u32": (_c.c_int, [_vp, _vp, _u32, _vp, _vp, _u64, _c.POINTER(_vp)]),
    "bitsort_graph_launch": (_c.c_int, [_vp, _vp]),
    "bitsort_graph_status": (_c.c_int, [_vp, _vp, _c.POINTER(Status), _u32]),
    "bitsort_graph_destroy": (_c.c_int, [_vp]),
    "bitsort_autotune_u32": (_c.c_int, [_u64, _u32, _c.c_int, _vp, _c.POINTER(Tuning)]),
    "bitsort_autotune_batch_u32": (_c.c_int, [_vp, _vp, _u32, _vp, _vp, _u64, _c.c_int, _vp, _c.POINTER(Tuning)]),
    "bitsort_tuning_save": (_c.c_int, [_c.c_char_p]),
    "bitsort_tuning_load": (_c.c_int, [_c.c_char_p, _c.POINTER(_c.c_int)]),
    "bitsort_tuning_clear": (_c.c_int, []),
    "bitsort_serve_run": (_c.c_int, [_vp, _u32, _vp, _vp, _vp]),
    "bitsort_digest_u32": (_c.c_int, [_vp, _u64, _c.POINTER(_u64), _vp]),
    "bitsort_profile_enable": (_c.c_int, [_c.c_int]),
    "bitsort_profile_reset": (_c.c_int, []),
    "bitsort_profile_read": (_c.c_int, [_c.POINTER(ProfileEntry), _c.c_int, _c.POINTER(_c.c_int)]),
}

_lib = None


def lib():
    """The loaded library.  Raises FileNotFoundError when it is not built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise FileNotFoundError(
                f"{LIB_PATH} is not built: run `python -c 'import __graft_entry__ as g; g.build()'` "
                "(hipcc, --offload-arch=gfx950)")
        # torch ships its own libamdhip64 (same soname).  Loading it first makes
        # this library bind to that runtime, so device pointers and streams
        # from torch are valid here; loading this library first would map a
        # second HIP runtime into the process.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        handle = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(handle, name)
            fn.restype = res
            fn.argtypes = args
        _lib = handle
    return _lib


def header_symbols() -> list[str]:
    """Every function the public header declares."""
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(bitsort_[a-z0-9_]+)\s*\(", text)))


def check(code: int, where: str) -> None:
    if code != BITSORT_OK:
        raise BitsortError(code, where)


# ---- one wrapper per entry point (raw pointers / ints in, return code out) ----

def bitsort_version() -> int:
    return lib().bitsort_version()


def error_string(code: int) -> str:
    return lib().bitsort_error_string(code).decode()


def bitsort_u32(keys: int, n: int, range_bits: int, out: int, stream: int) -> int:
    return lib().bitsort_u32(keys, n, range_bits, out, stream)


def bitsort_u32_atomic(keys: int, n: int, range_bits: int, out: int, stream: int) -> int:
    return lib().bitsort_u32_atomic(keys, n, range_bits, out, stream)


def bitsort_u64(keys: int, n: int, range_bits: int, out: int, stream: int) -> int:
    return lib().bitsort_u64(keys, n, range_bits, out, stream)


def bitsort_workspace_bytes(n: int, range_bits: int) -> int:
    return lib().bitsort_workspace_bytes(n, range_bits)


def bitsort_u32_ws(keys: int, n: int, range_bits: int, out: int, ws: int, ws_bytes: int, stream: int) -> int:
    return lib().bitsort_u32_ws(keys, n, range_bits, out, ws, ws_bytes, stream)


def bitsort_u32_noalloc(keys: int, n: int, range_bits: int, out: int, status: int, stream: int) -> int:
    """status: device address of one bitsort_status_t, or 0."""
    return lib().bitsort_u32_noalloc(keys, n, range_bits, out, status, stream)


NOALLOC_SCRATCH_BYTES = 32 << 20


def bitsort_radix_u32(keys: int, n: int, key_bits: int, out: int, stream: int) -> int:
    return lib().bitsort_radix_u32(keys, n, key_bits, out, stream)


def bitsort_radix_i32(keys: int, n: int, out: int, stream: int) -> int:
    return lib().bitsort_radix_i32(keys, n, out, stream)


def bitsort_radix_u64(keys: int, n: int, key_bits: int, out: int, stream: int) -> int:
    return lib().bitsort_radix_u64(keys, n, key_bits, out, stream)


def bitsort_radix_pairs_u32(keys: int, values: int, n: int, key_bits: int, out_keys: int, out_values: int,
                            stream: int) -> int:
    return lib().bitsort_radix_pairs_u32(keys, values, n, key_bits, out_keys, out_values, stream)


def bitsort_count_u32(keys: int, n: int, range_bits: int, out: int, stream: int) -> int:
    return lib().bitsort_count_u32(keys, n, range_bits, out, stream)


def bitsort_i32(keys: int, n: int, range_bits: int, out: int, stream: int) -> int:
    return lib().bitsort_i32(keys, n, range_bits, out, stream)


def bitsort_radix_workspace_bytes(n: int, key_bits: int) -> int:
    return lib().bitsort_radix_workspace_bytes(n, key_bits)


def bitsort_radix_u32_ws(keys: int, n: int, key_bits: int, out: int, ws: int, ws_bytes: int, stream: int) -> int:
    return lib().bitsort_radix_u32_ws(keys, n, key_bits, out, ws, ws_bytes, stream)


def bitsort_batch_ptr_u32(keys: int, n: int, range_bits: int, out: int, count: int, stream: int) -> int:
    """keys/n/range_bits/out: addresses of host arrays (see the header)."""
    return lib().bitsort_batch_ptr_u32(keys, n, range_bits, out, count, stream)


def bitsort_batch_plan(offsets: int, range_bits: int, num_segments: int):
    """offsets / range_bits: addresses of HOST arrays; -> (rc, plan handle)."""
    p = _vp()
    rc = lib().bitsort_batch_plan(offsets, range_bits, num_segments, ctypes.byref(p))
    return rc, p.value


def bitsort_batch_run(plan: int, keys: int, offsets: int, range_bits: int, out: int, stream: int) -> int:
    return lib().bitsort_batch_run(plan, keys, offsets, range_bits, out, stream)


def bitsort_batch_plan_status(plan: int, stream: int, count: int):
    arr = (Status * max(count, 1))()
    rc = lib().bitsort_batch_plan_status(plan, stream, arr, count)
    return rc, arr


def bitsort_batch_plan_destroy(plan: int) -> int:
    return lib().bitsort_batch_plan_destroy(plan)


def bitsort_set_workspace(workspace: int, nbytes: int, stream: int) -> int:
    return lib().bitsort_set_workspace(workspace, nbytes, stream)


def bitsort_get_status(stream: int) -> tuple[int, Status]:
    st = Status()
    rc = lib().bitsort_get_status(stream, ctypes.byref(st))
    return rc, st


def bitsort_workspace_status(ws: int, stream: int) -> tuple[int, Status]:
    st = Status()
    rc = lib().bitsort_workspace_status(ws, stream, ctypes.byref(st))
    return rc, st


def bitsort_batch_u32(keys: int, offsets: int, num_segments: int, range_bits: int, out: int,
                      max_keys: int, stream: int) -> int:
    return lib().bitsort_batch_u32(keys, offsets, num_segments, range_bits, out, max_keys, stream)


def bitsort_batch_status(stream: int, num_segments: int):
    arr = (Status * max(num_segments, 1))()
    rc = lib().bitsort_batch_status(stream, arr, num_segments)
    return rc, arr


def bitsort_generate_u32(out: int, first: int, count: int, range_bits: int, seed: int, stream: int) -> int:
    return lib().bitsort_generate_u32(out, first, count, range_bits, seed & 0xFFFFFFFFFFFFFFFF, stream)


def bitsort_debug_bitmap_u32(keys: int, n: int, range_bits: int, bitmap: int, stream: int) -> int:
    return lib().bitsort_debug_bitmap_u32(keys, n, range_bits, bitmap, stream)


def bitsort_debug_prefix_u32(keys: int, n: int, range_bits: int, prefix: int, stream: int) -> int:
    return lib().bitsort_debug_prefix_u32(keys, n, range_bits, prefix, stream)


def bitsort_pairs_u32(keys: int, values: int, n: int, range_bits: int, out_keys: int, out_values: int,
                      stream: int) -> int:
    return lib().bitsort_pairs_u32(keys, values, n, range_bits, out_keys, out_values, stream)


def bitsort_debug_split_u32(workspace: int, n: int, range_bits: int, stream: int):
    published = _u32()
    rc = lib().bitsort_debug_split_u32(workspace, n, range_bits, ctypes.byref(published), stream)
    return rc, published.value


def bitsort_set_tuning(slice_bits: int, tile_log2: int, emit_path: int = 0) -> int:
    return lib().bitsort_set_tuning(slice_bits, tile_log2, emit_path)


def bitsort_plan_info(n: int, range_bits: int):
    sb, tl, nb, ep = _u32(), _u32(), _u32(), _u32()
    rc = lib().bitsort_plan_info(n, range_bits, ctypes.byref(sb), ctypes.byref(tl), ctypes.byref(nb),
                                 ctypes.byref(ep))
    return rc, sb.value, tl.value, nb.value, ep.value


def bitsort_profile_enable(on: bool) -> int:
    return lib().bitsort_profile_enable(1 if on else 0)


def bitsort_profile_reset() -> int:
    return lib().bitsort_profile_reset()


def bitsort_profile_read():
    """-> (rc, {kernel: (launches, total_ms)})."""
    arr = (ProfileEntry * 64)()
    n = ctypes.c_int()
    rc = lib().bitsort_profile_read(arr, 64, ctypes.byref(n))
    return rc, {arr[i].kernel.decode(): (arr[i].launches, arr[i].total_ms) for i in range(min(n.value, 64))}


def bitsort_graph_create_u32(keys: int, n: int, range_bits: int, out: int):
    g = _vp()
    rc = lib().bitsort_graph_create_u32(keys, n, range_bits, out, ctypes.byref(g))
    return rc, g.value


def bitsort_graph_create_batch_u32(keys: int, offsets: int, num_segments: int, range_bits: int, out: int,
                                   max_keys: int):
    g = _vp()
    rc = lib().bitsort_graph_create_batch_u32(keys, offsets, num_segments, range_bits, out, max_keys,
                                              ctypes.byref(g))
    return rc, g.value


def bitsort_graph_launch(graph: int, stream: int) -> int:
    return lib().bitsort_graph_launch(graph, stream)


def bitsort_graph_status(graph: int, stream: int, count: int):
    arr = (Status * max(count, 1))()
    rc = lib().bitsort_graph_status(graph, stream, arr, count)
    return rc, arr


def bitsort_graph_destroy(graph: int) -> int:
    return lib().bitsort_graph_destroy(graph)


def bitsort_autotune_u32(n: int, range_bits: int, reps: int, stream: int):
    t = Tuning()
    rc = lib().bitsort_autotune_u32(n, range_bits, reps, stream, ctypes.byref(t))
    return rc, t


def bitsort_autotune_batch_u32(keys: int, offsets: int, num_segments: int, range_bits: int, out: int,
                               max_keys: int, reps: int, stream: int):
    t = Tuning()
    rc = lib().bitsort_autotune_batch_u32(keys, offsets, num_segments, range_bits, out, max_keys, reps, stream,
                                          ctypes.byref(t))
    return rc, t


def bitsort_tuning_save(path: str) -> int:
    return lib().bitsort_tuning_save(path.encode())


def bitsort_tuning_load(path: str):
    n = ctypes.c_int()
    rc = lib().bitsort_tuning_load(path.encode(), ctypes.byref(n))
    return rc, n.value


def bitsort_tuning_clear() -> int:
    return lib().bitsort_tuning_clear()


def bitsort_serve_run(requests: int, count: int, config: int, results: int, stats: int) -> int:
    """Pointers to arrays laid out as bitsort_request_t / _config_t /
    _request_result_t / _serve_stats_t (see serve.py for the dtypes)."""
    return lib().bitsort_serve_run(requests, count, config, results, stats)


def bitsort_digest_u32(data: int, n: int, stream: int):
    d = _u64()
    rc = lib().bitsort_digest_u32(data, n, ctypes.byref(d), stream)
    return rc, d.value
