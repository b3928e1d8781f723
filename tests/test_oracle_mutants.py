"""Planted mistakes in the oracle (on the CPU) must be caught by its pins.

Each case copies the oracle's C++ source, plants one plausible mistake (a
dropped mask, a wrong width or padding, an unstable sort, a skipped run, a
reversed or prefix-blind comparator, a run split early, swapped UTF-16
forms), compiles the copy and runs the pin battery against it.  At least one
pin must fail for every mutant; the unmodified source must pass them all.
"""

import ctypes
import os
import subprocess

import numpy as np
import pytest

import oracle
from workloads import BYTES_FAMILIES, adversarial, adversarial_bytes, config2, from_strings

SRC = os.path.join(os.path.dirname(oracle.__file__), "husky_oracle.cpp")

MUTANTS = {
    "drop_ascii_mask": ("code |= ((uint64_t)s[j] & c.mask) << (c.w * (c.m - 1 - (int)j));",
                        "code |= ((uint64_t)s[j]) << (c.w * (c.m - 1 - (int)j));"),
    "padding_off_by_one": ("code |= ((uint64_t)s[j] & c.mask) << (c.w * (c.m - 1 - (int)j));",
                           "code |= ((uint64_t)s[j] & c.mask) << (c.w * (c.m - 1 - (int)j) "
                           "- (len < (uint64_t)c.m ? c.w : 0));"),
    "eight_ascii_chars": ("const Coder ASCII7 = {9, 7, 0x7F};", "const Coder ASCII7 = {8, 7, 0x7F};"),
    "unstable_pair_sort": ("std::stable_sort(v.begin(), v.end()", "std::sort(v.begin(), v.end()"),
    "skip_runs_of_two": ("if (end - start >= 2) {", "if (end - start >= 3) {"),
    "reversed_comparator": ("return std::lexicographical_compare(pa, pa + la, pb, pb + lb);",
                            "return std::lexicographical_compare(pb, pb + lb, pa, pa + la);"),
    "prefix_blind_comparator": (
        "return std::lexicographical_compare(pa, pa + la, pb, pb + lb);",
        "return std::lexicographical_compare(pa, pa + std::min(la, lb), pb, pb + std::min(la, lb));"),
    "run_split_early": ("while (end < n && codes[end] == codes[start]) ++end;",
                        "while (end < n && codes[end] == codes[start] && end - start < 4) ++end;"),
    "utf16_forms_swapped": ("codes[i] = coder == 2 ? (c >> 1) : c;",
                            "codes[i] = coder == 2 ? c : (c >> 1);"),
    "unicode_width_15": ("const Coder UTF16 = {4, 16, 0xFFFF};", "const Coder UTF16 = {4, 15, 0xFFFF};"),
    "bytes8_masked": ("const Coder BYTES8 = {8, 8, 0xFF};", "const Coder BYTES8 = {8, 8, 0x7F};"),
    "bytes8_nine_chars": ("const Coder BYTES8 = {8, 8, 0xFF};", "const Coder BYTES8 = {9, 7, 0xFF};"),
}


def _battery():
    """Return the list of failed pin names (empty = all pass)."""
    from test_oracle_pins import _bitstring_code, _brute, _golden_rows

    failed = []
    for coder, units, code in _golden_rows():
        byte_coder = coder in ("ascii7", "bytes8")
        b = from_strings([bytes(units)] if byte_coder else [tuple(units)],
                         coder if byte_coder else "utf16")
        if int(oracle.encode(b, coder)[0][0]) != code:
            failed.append("golden")
            break
    for fam in ("nul", "prefix9", "identical", "utf16_edges", "utf16_prefix4", "mixed"):
        b = adversarial(fam, seed=11, n=600)
        if not np.array_equal(oracle.sort(b)[0], _brute(b)):
            failed.append(f"brute:{fam}")
        coders = ["utf16", "utf16_paper"] if b.coder == "utf16" else ["ascii7"]
        for c in coders:
            if [int(x) for x in oracle.encode(b, c)[0]] != [_bitstring_code(s, c) for s in b.strings()]:
                failed.append(f"bitstring:{fam}:{c}")
    rng = np.random.default_rng(5)
    codes = rng.integers(0, 50, size=5000).astype(np.uint64) << np.uint64(57)
    _, i = oracle.sort_pairs(codes, np.arange(5000, dtype=np.uint32))
    if not np.array_equal(i, np.argsort(codes, kind="stable")):
        failed.append("stable_argsort")
    b = config2(n=3000)
    if not np.array_equal(oracle.sort(b)[0], _brute(b)):
        failed.append("brute:config2")
    for fam in BYTES_FAMILIES:
        b = adversarial_bytes(fam, seed=11, n=600)
        if not np.array_equal(oracle.sort(b)[0], _brute(b)):
            failed.append(f"brute:{fam}")
        if [int(x) for x in oracle.encode(b)[0]] != [_bitstring_code(s, "bytes8") for s in b.strings()]:
            failed.append(f"bitstring:{fam}")
    return failed


def _with_lib(path):
    saved = oracle._lib
    oracle._lib = None
    real = oracle._LIB_PATH
    try:
        oracle._LIB_PATH = path
        # load without the rebuild-if-stale check
        oracle._SRC_saved = oracle._SRC
        oracle._SRC = path
        oracle._load()
        return _battery()
    finally:
        oracle._lib = saved
        oracle._LIB_PATH = real
        oracle._SRC = oracle._SRC_saved


def test_unmodified_oracle_passes_battery():
    assert _battery() == []


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation site for {name} not unique"
    mut = tmp_path / "mut.cpp"
    mut.write_text(src.replace(old, new))
    so = tmp_path / f"liboracle_{name}.so"
    subprocess.check_call(["g++", "-O1", "-std=c++17", "-shared", "-fPIC", str(mut), "-o", str(so)])
    failed = _with_lib(str(so))
    assert failed, f"mutant {name} passed every pin"
