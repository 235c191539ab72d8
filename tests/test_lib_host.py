"""libbitsort.so loads, exports every symbol its header declares, and rejects
bad arguments on the host (no kernel launch, no GPU needed)."""
import ctypes

import pytest

from paper_1312_0138_amd import _lib


@pytest.fixture(scope="module")
def lib():
    return _lib.lib()


def test_exports_every_header_symbol(lib):
    names = _lib.header_symbols()
    assert "bitsort_u32" in names and "bitsort_batch_u32" in names
    handle = ctypes.CDLL(_lib.LIB_PATH)
    for name in names:
        assert hasattr(handle, name), f"{name} declared in bitsort.h but not exported"
    assert set(names) == set(_lib._SIGS), "binding and header disagree"


def test_version_and_errors(lib):
    assert _lib.bitsort_version() == 10000
    assert _lib.error_string(0) == "ok"
    for code in range(1, 5):
        assert _lib.error_string(code) != "unknown error"


def test_host_argument_checks(lib):
    E = _lib
    fake = 1 << 20  # never dereferenced: every call below fails its host checks
    assert E.bitsort_u32(fake, 10, 33, fake + 4096, 0) == E.BITSORT_ERR_INVALID_ARG
    assert E.bitsort_u32(0, 10, 10, fake, 0) == E.BITSORT_ERR_INVALID_ARG
    assert E.bitsort_u32(fake, 10, 3, fake + 4096, 0) == E.BITSORT_ERR_TOO_LARGE  # n > 2^range_bits
    assert E.bitsort_u32(fake, 1 << 32, 32, fake + (1 << 36), 0) == E.BITSORT_ERR_TOO_LARGE
    assert E.bitsort_u32(fake, 100, 10, fake + 4, 0) == E.BITSORT_ERR_INVALID_ARG  # partial overlap
    assert E.bitsort_workspace_bytes(10, 3) == 0
    assert E.bitsort_workspace_bytes(10, 33) == 0
    assert E.bitsort_set_tuning(9, 0) == E.BITSORT_ERR_INVALID_ARG
    assert E.bitsort_set_tuning(0, 15) == E.BITSORT_ERR_INVALID_ARG
    assert E.bitsort_batch_u32(fake, fake, 0, fake, fake, 0, 0) == E.BITSORT_ERR_INVALID_ARG
    assert E.bitsort_generate_u32(fake, 10, 1, 3, 0, 0) == E.BITSORT_ERR_TOO_LARGE


def test_plan_shapes(lib):
    rc, sb, tl, nb = _lib.bitsort_plan_info(1 << 26, 28)
    assert rc == 0 and nb == 1 << (28 - sb) and 10 <= sb <= 20
    rc, sb, tl, nb = _lib.bitsort_plan_info(1 << 24, 32)
    assert rc == 0 and sb == 20 and nb == 4096
    rc, sb, tl, nb = _lib.bitsort_plan_info(100, 10)
    assert rc == 0 and nb == 1 and tl == 0  # single-workgroup path
    ws = _lib.bitsort_workspace_bytes(1 << 26, 28)
    assert ws >= 4 * (1 << 26)
