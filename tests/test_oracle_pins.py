"""Pins for the CPU oracle against what the paper and the mathematics fix.

* worked values of stringToLong (Algorithm 4) derived by hand (tests/golden);
* an independent bit-string derivation of the same codes on random inputs;
* the coder contract of Sec. 3.2 (equal strings -> equal codes; x > y never
  gives code(x) < code(y) inside the domain), checked exhaustively over small
  alphabets;
* the whole sort against a brute-force stable comparison sort (Python's
  ``sorted`` over ``bytes`` / unit tuples) and against invariants;
* coder independence: with any monotone coder (ASCII, the paper's shifted
  UTF-16 form, the null coder, the full-byte coder) the result is the same
  permutation, because Step 3 removes every inversion left inside equal-code
  runs (Sec. 3.4);
* the full-byte coder (eight 8-bit characters, the widest-alphabet member of
  Sec. 3.2's alphabet-dependent coders) the same ways, over every byte value.
"""

import itertools
import os

import numpy as np
import pytest

import oracle
from workloads import (ADVERSARIAL_FAMILIES, BYTES_FAMILIES, adversarial, adversarial_bytes,
                       config1, config2, config3, config4, config5, from_strings, utf8_words)

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "stringToLong_values.tsv")


def _golden_rows():
    rows = []
    with open(GOLDEN) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            coder, elems, code, _note = line.rstrip("\n").split("\t")
            units = [] if elems == "-" else [int(x, 16) for x in elems.split(":")]
            rows.append((coder, units, int(code, 16)))
    return rows


@pytest.mark.parametrize("row", _golden_rows(), ids=lambda r: f"{r[0]}:{r[1][:4]}")
def test_golden_stringToLong(row):
    coder, units, code = row
    if coder in ("ascii7", "bytes8"):
        b = from_strings([bytes(units)], coder)
    else:
        b = from_strings([tuple(units)], "utf16")
    codes, _ = oracle.encode(b, coder)
    assert int(codes[0]) == code


def _bitstring_code(s, coder):
    """Code as the concatenation of per-character bit groups (independent derivation)."""
    if coder == "ascii7":
        groups = [format(c & 0x7F, "07b") for c in s[:9]] + ["0" * 7] * (9 - min(len(s), 9))
        return int("".join(groups), 2)
    if coder == "bytes8":
        groups = [format(c, "08b") for c in s[:8]] + ["0" * 8] * (8 - min(len(s), 8))
        return int("".join(groups), 2)
    groups = [format(c, "016b") for c in s[:4]] + ["0" * 16] * (4 - min(len(s), 4))
    v = int("".join(groups), 2)
    return v >> 1 if coder == "utf16_paper" else v


@pytest.mark.parametrize("family", ADVERSARIAL_FAMILIES)
def test_encode_matches_bitstring(family):
    b = adversarial(family, seed=7, n=400)
    coders = ["utf16", "utf16_paper"] if b.coder == "utf16" else ["ascii7"]
    strs = b.strings()
    for coder in coders:
        codes, _ = oracle.encode(b, coder)
        expect = [_bitstring_code(s, coder) for s in strs]
        assert [int(c) for c in codes] == expect


def test_encode_matches_bitstring_configs():
    for b in (config1(n=3000), config2(n=3000), config3(n=3000)):
        codes, bad = oracle.encode(b)
        assert bad == 0
        assert [int(c) for c in codes] == [_bitstring_code(s, b.coder) for s in b.strings()]


def test_domain_violation_count():
    strs = [b"abc", b"\x80", b"abcdefgh\xff", b"abcdefghi\xff", b"a\xc3\xa9", b""]
    codes, bad = oracle.encode(from_strings(strs))
    # bytes >= 0x80 in the first nine positions: "\x80", "abcdefgh\xff", "a\xc3\xa9"
    assert bad == 3
    b = adversarial("high_after9", n=300)
    assert oracle.encode(b)[1] == 0


def _all_strings(alphabet, max_len):
    for L in range(max_len + 1):
        for t in itertools.product(alphabet, repeat=L):
            yield t


@pytest.mark.parametrize("alphabet,max_len", [((0x00, 0x61, 0x7F), 7), ((0x00, 0x7F), 11),
                                              ((0x01, 0x41, 0x7E), 7)])
def test_ascii_coder_monotone_exhaustive(alphabet, max_len):
    strs = [bytes(t) for t in _all_strings(alphabet, max_len)]
    strs.sort()
    codes, bad = oracle.encode(from_strings(strs))
    assert bad == 0
    # Sec. 3.2: equal strings give equal codes, and inside the domain x > y
    # never gives code(x) < code(y): codes are non-decreasing in string order.
    assert np.all(np.diff(codes.astype(object)) >= 0)


@pytest.mark.parametrize("coder", ["utf16", "utf16_paper"])
def test_utf16_coder_monotone_exhaustive(coder):
    strs = sorted(_all_strings((0x0000, 0x8000, 0xFFFF), 6))
    codes, _ = oracle.encode(from_strings(strs, "utf16"), coder)
    assert np.all(np.diff(codes.astype(object)) >= 0)


def test_paper_utf16_collision():
    # The printed unicodeToLong drops the fourth unit's low bit (3 15/16
    # characters, Sec. 3.4), so these two strings collide there but not in the
    # full 64-bit form; the sort result is the same either way.
    b = from_strings([(0x4E00,) * 4, (0x4E00, 0x4E00, 0x4E00, 0x4E01)], "utf16")
    full, _ = oracle.encode(b, "utf16")
    paper, _ = oracle.encode(b, "utf16_paper")
    assert full[0] != full[1] and paper[0] == paper[1]


def _brute(b):
    strs = b.strings()
    return np.array(sorted(range(b.n), key=lambda i: strs[i]), dtype=np.uint32)


@pytest.mark.parametrize("family", ADVERSARIAL_FAMILIES)
def test_sort_matches_bruteforce_adversarial(family):
    b = adversarial(family, seed=3, n=1500)
    perm, _ = oracle.sort(b)
    np.testing.assert_array_equal(perm, _brute(b))


@pytest.mark.parametrize("maker", [config1, config2, config3, lambda n: config5(n=n)])
def test_sort_matches_bruteforce_configs(maker):
    b = maker(n=20000)
    perm, bad = oracle.sort(b)
    assert bad == 0
    np.testing.assert_array_equal(perm, _brute(b))


def test_sort_pairs_is_stable_argsort():
    rng = np.random.default_rng(5)
    codes = rng.integers(0, 50, size=5000).astype(np.uint64) << np.uint64(57)
    idx = np.arange(5000, dtype=np.uint32)
    c, i = oracle.sort_pairs(codes, idx)
    ref = np.argsort(codes, kind="stable").astype(np.uint32)
    np.testing.assert_array_equal(i, ref)
    np.testing.assert_array_equal(c, codes[ref])


def test_fixup_only_touches_equal_code_runs():
    b = config2(n=5000)
    codes, _ = oracle.encode(b)
    c, i = oracle.sort_pairs(codes, np.arange(b.n, dtype=np.uint32))
    fixed = oracle.fixup(b, c, i)
    # each run of equal codes holds the same members before and after
    heads = np.flatnonzero(np.concatenate([[True], c[1:] != c[:-1], [True]]))
    for a, z in zip(heads[:-1], heads[1:]):
        assert sorted(i[a:z]) == sorted(fixed[a:z])


@pytest.mark.parametrize("coder", ["null"])
def test_coder_independence_ascii(coder):
    for b in (adversarial("nul", n=800), adversarial("prefix9", n=800), config2(n=4000)):
        ref, _ = oracle.sort(b, "ascii7")
        alt, _ = oracle.sort(b, coder)
        np.testing.assert_array_equal(ref, alt)


def test_coder_independence_utf16():
    for b in (adversarial("utf16_edges", n=800), adversarial("utf16_prefix4", n=800),
              config3(n=4000)):
        ref, _ = oracle.sort(b, "utf16")
        for alt in ("utf16_paper", "null"):
            np.testing.assert_array_equal(ref, oracle.sort(b, alt)[0])


def test_invariants_configs():
    for b in (config1(n=50000), config2(n=50000), config3(n=50000)):
        perm, _ = oracle.sort(b)
        assert np.array_equal(np.sort(perm), np.arange(b.n, dtype=np.uint32))
        strs = b.strings()
        for k in range(b.n - 1):
            x, y = strs[perm[k]], strs[perm[k + 1]]
            assert x < y or (x == y and perm[k] < perm[k + 1])
        codes, _ = oracle.encode(b)
        assert np.all(np.diff(codes[perm].astype(object)) >= 0)  # monotone along the order


def test_check_perm_detects_errors():
    b = config2(n=3000)
    perm, _ = oracle.sort(b)
    assert oracle.check_perm(b, perm) == (0, b.n)
    bad = perm.copy()
    bad[[10, 11]] = bad[[11, 10]]
    assert oracle.check_perm(b, bad)[0] > 0
    dup = perm.copy()
    dup[5] = dup[6]
    assert oracle.check_perm(b, dup)[0] > 0
    # equal strings out of index order are rejected
    b2 = from_strings([b"same", b"same", b"other"])
    assert oracle.check_perm(b2, np.array([2, 0, 1], np.uint32))[0] == 0
    assert oracle.check_perm(b2, np.array([2, 1, 0], np.uint32))[0] == 1


def test_batched_oracle_is_per_instance():
    b = config4(n_inst=12, lo=1, hi=3000)
    perm, _ = oracle.sort_batched(b)
    for k in range(12):
        lo, hi = int(b.seg_offsets[k]), int(b.seg_offsets[k + 1])
        sub = b.subset(lo, hi)
        np.testing.assert_array_equal(perm[lo:hi], _brute(sub) + lo)


def test_empty_and_single():
    for strs in ([], [b""], [b"x"], [b"", b""]):
        b = from_strings(strs)
        perm, _ = oracle.sort(b)
        np.testing.assert_array_equal(perm, _brute(b))


def test_check_perm_batched_detects_errors():
    b = config4(n_inst=10, lo=1, hi=500)
    perm, _ = oracle.sort_batched(b)
    assert oracle.check_perm_batched(b, perm)[0] == 0
    bad = perm.copy()
    lo = int(b.seg_offsets[3])
    bad[[lo, lo + 1]] = bad[[lo + 1, lo]]
    assert oracle.check_perm_batched(b, bad)[0] > 0
    # a global sort is not a per-instance sort
    glob, _ = oracle.sort(b)
    assert oracle.check_perm_batched(b, glob)[0] > 0


# ------------------------------------------------------------------ full-byte coder
@pytest.mark.parametrize("family", BYTES_FAMILIES)
def test_bytes8_encode_matches_bitstring(family):
    b = adversarial_bytes(family, seed=7, n=400)
    codes, bad = oracle.encode(b, "bytes8")
    assert bad == 0  # every byte value is in the domain
    assert [int(c) for c in codes] == [_bitstring_code(s, "bytes8") for s in b.strings()]


@pytest.mark.parametrize("alphabet,max_len", [((0x00, 0x7F, 0x80, 0xFF), 9),
                                              ((0x00, 0x01, 0xFE, 0xFF), 9)])
def test_bytes8_coder_monotone_exhaustive(alphabet, max_len):
    # every string of up to nine bytes over values either side of 0x80: codes
    # never decrease in byte order, and two strings share a code exactly when
    # their first eight bytes, zero-padded, agree
    strs = sorted(bytes(t) for t in _all_strings(alphabet, max_len))
    codes, bad = oracle.encode(from_strings(strs, "bytes8"))
    assert bad == 0
    c = codes.astype(object)
    assert np.all(np.diff(c) >= 0)
    pad = [s[:8] + bytes(8 - min(len(s), 8)) for s in strs]
    same_code = c[1:] == c[:-1]
    same_pad = np.array([pad[k] == pad[k + 1] for k in range(len(strs) - 1)])
    np.testing.assert_array_equal(same_code, same_pad)


@pytest.mark.parametrize("family", BYTES_FAMILIES)
def test_bytes8_sort_matches_bruteforce(family):
    b = adversarial_bytes(family, seed=3, n=1500)
    perm, bad = oracle.sort(b)
    assert bad == 0
    np.testing.assert_array_equal(perm, _brute(b))


def test_bytes8_sort_utf8_text():
    # bytes order of UTF-8 is code point order: the brute force compares the
    # decoded strings by code points as a second witness
    b = utf8_words(n=20000, seed=5)
    perm, _ = oracle.sort(b)
    np.testing.assert_array_equal(perm, _brute(b))
    text = [s.decode("utf-8") for s in b.strings()]
    by_cp = sorted(range(b.n), key=lambda i: [ord(ch) for ch in text[i]])
    np.testing.assert_array_equal(perm, np.array(by_cp, dtype=np.uint32))


def test_coder_independence_bytes8():
    # on ASCII text the full-byte coder, the 7-bit coder and the null coder
    # give the same permutation
    for b in (adversarial("nul", n=800), adversarial("prefix9", n=800), config2(n=4000)):
        ref, _ = oracle.sort(b, "ascii7")
        np.testing.assert_array_equal(ref, oracle.sort(b, "bytes8")[0])
    for fam in BYTES_FAMILIES:
        b = adversarial_bytes(fam, seed=9, n=600)
        np.testing.assert_array_equal(oracle.sort(b)[0], oracle.sort(b, "null")[0])
