"""Pins for the oracle's global fix-up (Step 3 as a full stable pass, Sec. 3.1)
and Algorithm 1 with a lossy coder (Sec. 3.2: a code may invert two objects
with probability p; the Appendix's deliberate mis-coding).

* any codes -- exact husky codes, a fraction p replaced by random values
  (p from 0 to 1), codes that reverse the order, constant codes -- give the
  brute-force stable sort (Python's ``sorted`` over the strings, index order
  for ties);
* the global pass alone, from any starting order (shuffled, reversed,
  sorted), gives the same permutation;
* a planted mistake (no index tie-break) is caught when equal strings arrive
  out of index order.
"""

import numpy as np
import pytest

import oracle
from workloads import adversarial, config2, config3, utf8_words


def _brute(b):
    strs = b.strings()
    return np.array(sorted(range(b.n), key=lambda i: strs[i]), dtype=np.uint32)


def _miscoded(codes, p, seed):
    rng = np.random.default_rng(seed)
    c = np.array(codes, dtype=np.uint64, copy=True)
    hit = rng.random(c.size) < p
    c[hit] = rng.integers(0, 2**64 - 1, size=int(hit.sum()), dtype=np.uint64, endpoint=True)
    return c


@pytest.mark.parametrize("p", [0.0, 0.01, 0.1, 0.25, 0.5, 1.0])
@pytest.mark.parametrize("maker", [lambda: config2(n=6000, seed=3), lambda: config3(n=5000, seed=4),
                                   lambda: adversarial("identical", n=3000),
                                   lambda: utf8_words(n=4000, seed=5)],
                         ids=["config2", "config3", "identical", "utf8"])
def test_lossy_sort_matches_bruteforce(maker, p):
    b = maker()
    codes, _ = oracle.encode(b, "bytes8" if b.coder == "bytes8" else None)
    np.testing.assert_array_equal(oracle.sort_lossy(b, _miscoded(codes, p, 7)), _brute(b))


def test_adversarial_codes():
    b = config2(n=5000, seed=8)
    codes, _ = oracle.encode(b)
    ref = _brute(b)
    rev = (np.uint64(2**64 - 1) - codes).astype(np.uint64)  # inverts every pair
    np.testing.assert_array_equal(oracle.sort_lossy(b, rev), ref)
    np.testing.assert_array_equal(oracle.sort_lossy(b, np.zeros(b.n, np.uint64)), ref)


@pytest.mark.parametrize("start", ["shuffled", "reversed", "sorted"])
def test_global_pass_from_any_order(start):
    b = adversarial("nul", n=3000, seed=2)
    ref = _brute(b)
    idx = {"shuffled": np.random.default_rng(1).permutation(b.n), "reversed": np.arange(b.n)[::-1],
           "sorted": ref}[start].astype(np.uint32)
    np.testing.assert_array_equal(oracle.fixup_global(b, idx), ref)


def test_planted_missing_tie_break_is_caught():
    # equal strings arriving out of index order: a stable pass without the
    # index tie-break keeps their arrival order, which the pins reject
    b = adversarial("identical", n=2000, seed=4)
    idx = np.arange(b.n, dtype=np.uint32)[::-1].copy()
    strs = b.strings()
    planted = np.array(sorted(idx.tolist(), key=lambda i: strs[i]), dtype=np.uint32)  # stable, no tie-break
    assert not np.array_equal(planted, _brute(b))
    np.testing.assert_array_equal(oracle.fixup_global(b, idx), _brute(b))
