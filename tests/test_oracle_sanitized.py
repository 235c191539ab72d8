"""The oracle built with AddressSanitizer and UndefinedBehaviorSanitizer (gcc,
host code only) and driven through every entry point by a small C program:
any out-of-bounds access, leak, signed overflow or out-of-range shift in the
oracle fails the run."""
import os
import shutil
import subprocess

import pytest

from oracle import build as obuild

HERE = os.path.dirname(os.path.abspath(__file__))
DRIVER = os.path.join(HERE, "native", "oracle_sanitize_driver.c")


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_under_asan_and_ubsan(tmp_path):
    exe = str(tmp_path / "oracle_sanitized")
    flags = ["-std=c99", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
             "-fno-sanitize-recover=all"]
    subprocess.run(["gcc", *flags, "-o", exe, obuild.SRC, DRIVER], check=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    env.pop("LD_PRELOAD", None)
    res = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    assert res.returncode == 0, res.stdout + res.stderr
