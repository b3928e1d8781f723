"""The perfect bit of the ASCII sort key, checked exhaustively on the CPU.

The plain and batched sorts order ASCII strings by code << 1 | f instead of
the code of Algorithm 4, where f = 0 exactly when the string has at most nine
bytes and none of them is NUL (the per-string form of the paper's "perfect"
coding, Algorithm 3 and Sec. 3.4).  Two claims make that exact:

* the shifted key is still monotone: x < y never gives key(x) > key(y);
* equal keys with f = 0 belong to identical strings, so such runs need no
  fix-up at all.

Both are checked over every string of up to ten bytes from an alphabet with
NUL, two letters and 0x7F (the largest byte the coder accepts), with the code
taken from the oracle's encoder.
"""

import itertools

import numpy as np

import oracle
from workloads import from_strings


def _keys(strings):
    codes = oracle.encode(from_strings(strings, "ascii7"))[0].astype(np.uint64)
    flags = np.array([1 if (len(s) > 9 or 0 in s[:9]) else 0 for s in strings], dtype=np.uint64)
    return (codes << np.uint64(1)) | flags, flags


def test_perfect_bit_monotone_and_identity():
    alpha = (0x00, 0x61, 0x62, 0x7F)
    strings = [b""]
    for L in range(1, 10):
        strings += [bytes(t) for t in itertools.product(alpha, repeat=L)]
    # one ten-byte string per nine-byte prefix, so every equal-code class
    # also holds a string longer than nine bytes
    strings += [bytes(t) + bytes([alpha[i % 4]])
                for i, t in enumerate(itertools.product(alpha, repeat=9))]
    strings.sort()
    keys, flags = _keys(strings)
    # monotone: sorted strings give non-decreasing keys
    assert np.all(keys[1:] >= keys[:-1])
    # equal keys with f = 0 are identical strings (here: every string is
    # distinct, so no two f = 0 strings may share a key)
    perfect = keys[flags == 0]
    assert len(np.unique(perfect)) == len(perfect)


def test_perfect_bit_catches_a_wrong_flag():
    # a planted mistake: a flag that ignores NULs gives "a", "a\0" and
    # "a\0\0" (one code) the same key with f = 0 although they differ
    strings = sorted([b"a", b"a\0", b"a\0\0", b"ab"])
    codes = oracle.encode(from_strings(strings, "ascii7"))[0].astype(np.uint64)
    wrong = np.array([1 if len(s) > 9 else 0 for s in strings], dtype=np.uint64)
    keys = (codes << np.uint64(1)) | wrong
    assert len(np.unique(keys[wrong == 0])) < int((wrong == 0).sum())
