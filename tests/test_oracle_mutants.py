"""Planted mistakes in the oracle must be caught by its pins.

Each case copies ``oracle/bitsort_oracle.c``, plants one plausible mistake (a
wrong shift or mask, a dropped term, XOR for OR, reversed bit order, a lost
pass of Algorithm 1, ...), builds the copy with gcc and runs the pins against
it in a child process (a planted out-of-bounds write may crash it, which also
counts as caught).  The real oracle is never modified.
"""
import os
import subprocess
import sys

import pytest

from oracle import build as obuild

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
TESTS = os.path.join(ROOT, "tests")

MUTANTS = {
    "word_index_shift": ("uint64_t w = (uint64_t)(k >> 5);", "uint64_t w = (uint64_t)(k >> 6);"),
    "bit_mask": ("uint32_t m = oracle_power2(k & 31u);", "uint32_t m = oracle_power2(k & 15u);"),
    "xor_for_or": ("bitmap[w] = bitmap[w] | m;", "bitmap[w] = bitmap[w] ^ m;"),
    "count_ones_skips_bit31": (
        "    for (uint32_t i = 0; i < 32; i++)\n        if (oracle_bit_value(x, i))",
        "    for (uint32_t i = 0; i < 31; i++)\n        if (oracle_bit_value(x, i))"),
    "emit_msb_first": ("out[j++] = (uint32_t)(w * 32u + b);", "out[j++] = (uint32_t)(w * 32u + (31u - b));"),
    "bit_value_index": ("return ((x & (1u << i)) == 0) ? 0u : 1u;",
                        "return ((x & (1u << (i ^ 1u))) == 0) ? 0u : 1u;"),
    "bitmap_words_extra": ("return r < 32 ? 1 : r / 32;", "return r < 32 ? 1 : r / 32 + 1;"),
    "radix_ones_first": ("        split_by_bit_u32(from, to, n, k, 0u);", "        split_by_bit_u32(from, to, n, k, 1u);"),
    "radix_unstable": ("            dst[at_back++] = src[i];", "            dst[n - 1 - (at_back++ - first)] = src[i];"),
    "sign_split_order": ("split_by_bit_u32(bits, grouped, n, 31u, 1u);", "split_by_bit_u32(bits, grouped, n, 31u, 0u);"),
    "signed_lost_pass": ("rc = oracle_bitwise_sort1_u32(grouped + negatives, n - negatives, 31);",
                         "rc = oracle_bitwise_sort1_u32(grouped + negatives, n - negatives, 30);"),
    "scan_dropped_term": ("prefix[w + 1] = prefix[w] + oracle_count_ones(bitmap[w]);",
                          "prefix[w + 1] = oracle_count_ones(bitmap[w]);"),
    "counting_collapses": ("        count[keys[i]]++;", "        count[keys[i]] = 1;"),
    "u64_bit_mask": ("uint64_t m = (uint64_t)1 << (k & 63);", "uint64_t m = (uint64_t)1 << (k & 31);"),
    "out_of_range_unflagged": (
        "        if ((uint64_t)k >= r) {\n            *flags |= ORACLE_FLAG_OUT_OF_RANGE;\n            continue;\n        }\n        uint64_t w",
        "        if ((uint64_t)k >= r) {\n            continue;\n        }\n        uint64_t w"),
    "duplicate_unflagged": ("        if (bitmap[w] & m)\n            *flags |= ORACLE_FLAG_DUPLICATE;\n", ""),
    "w64_variant_mask": ("bitmap[k >> 6] = bitmap[k >> 6] | ((uint64_t)1 << (k & 63));",
                         "bitmap[k >> 6] = bitmap[k >> 6] | ((uint64_t)1 << (k & 31));"),
    "bin_repl_reversed": ("out[15 - d] = oracle_bit_value", "out[d] = oracle_bit_value"),
    "u64_radix_32bit_shift": ("const uint64_t mask = (uint64_t)1 << k;", "const uint64_t mask = (uint64_t)(1u << (k & 31));"),
    "pairs_value_left_behind": ("        dv[*slot] = sv[i];", "        dv[*slot] = sv[n - 1 - i];"),
}

_RUNNER = """
import sys
sys.path.insert(0, {root!r}); sys.path.insert(0, {tests!r})
import oracle, oracle_pins
failed = oracle_pins.run_all(oracle.Oracle({lib!r}), stop_at_first=True)
print("failed:", failed)
sys.exit(1 if failed else 0)
"""


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistake_is_caught(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(obuild.SRC).read()
    assert src.count(old) == 1, f"mutation anchor for {name} must occur exactly once"
    mutated = tmp_path / "mutant.c"
    mutated.write_text(src.replace(old, new))
    lib = str(tmp_path / "libmutant.so")
    obuild.build_from(str(mutated), lib, extra_flags=["-Wno-error"])
    code = _RUNNER.format(root=ROOT, tests=TESTS, lib=lib)
    res = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300)
    assert res.returncode != 0, f"planted mistake {name} passed every pin:\n{res.stdout}{res.stderr}"


def test_unmutated_copy_passes(tmp_path):
    lib = str(tmp_path / "libcopy.so")
    obuild.build_from(obuild.SRC, lib)
    code = _RUNNER.format(root=ROOT, tests=TESTS, lib=lib)
    res = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300)
    assert res.returncode == 0, res.stdout + res.stderr
