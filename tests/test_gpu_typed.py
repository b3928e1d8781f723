"""GPU: the coders of the other object types (int32, int64, float64, date-times,
big integers, decimals, tuples) against their oracle.

* codes: bit-exact against the oracle's husky code of every record (edge
  records and generated data, date-times inside and outside the window);
* sorts: the permutation equals the oracle's (which the brute-force sort by
  value pins) on the paper's sizes (20,000 to 500,000 records), ragged
  sizes, tiny and empty inputs, every comparator edge (NaNs of any sign and
  payload, -0.0, equal decimals of different scales, redundant sign bytes,
  NULs inside tuple strings);
* out-of-domain records are counted and raise in the binding.
"""

import struct

import numpy as np
import pytest

from oracle import typed as ot
from workloads.typed import TYPED, typed

pytestmark = pytest.mark.gpu


def _u32(t):
    return t.cpu().numpy().view(np.uint32)


class _Batch:
    def __init__(self, t, recs):
        self.type = t
        self.count = len(recs)
        if t in ot.FIXED_SIZE:
            self.data = np.frombuffer(b"".join(recs) or b"\0" * 16, dtype=np.uint8).copy()
            self.offsets = None
        else:
            lens = np.array([len(r) for r in recs], dtype=np.int64)
            self.offsets = np.concatenate([[0], np.cumsum(lens)]).astype(np.uint64)
            self.data = np.frombuffer(b"".join(recs) or b"\0", dtype=np.uint8).copy()

    @property
    def n(self):
        return self.count


def _edges(t):
    from test_oracle_typed import _edge_records

    return _edge_records(t)


@pytest.mark.parametrize("t", TYPED)
def test_codes_match_oracle(gpu_lib, t):
    for b in (typed(t, n=30_000, seed=11), _Batch(t, _edges(t))):
        r, o = gpu_lib.typed_to_device(b)
        got = gpu_lib.encode_typed(r, o, t, b.n).cpu().numpy().view(np.uint64)
        want, _ = ot.encode(b)
        ok = np.array([ot.in_domain(t, rec) for rec in ot.records(b)])  # codes of others: unspecified
        assert ok.mean() > 0.9
        np.testing.assert_array_equal(got[ok], want[ok])


@pytest.mark.parametrize("t", TYPED)
@pytest.mark.parametrize("n", [20_000, 500_000, 65_537])
def test_sort_matches_oracle(gpu_lib, t, n):
    b = typed(t, n=n, seed=n % 97 + 2)
    r, o = gpu_lib.typed_to_device(b)
    perm = _u32(gpu_lib.sort_typed(r, o, t, b.n))
    want, bad = ot.sort(b)
    assert bad == 0
    np.testing.assert_array_equal(perm, want)


@pytest.mark.parametrize("t", TYPED)
def test_sort_edges_tiny_and_empty(gpu_lib, t):
    import torch

    recs = _edges(t)
    rng = np.random.default_rng(3)
    for k in (0, 1, 2, 7, len(recs), 5000):
        pick = recs if k == len(recs) else [recs[i] for i in rng.integers(0, len(recs), size=k)]
        b = _Batch(t, pick)
        r, o = gpu_lib.typed_to_device(b)
        perm = gpu_lib.sort_typed(r, o, t, b.n)
        assert perm.numel() == b.n
        if b.n:
            np.testing.assert_array_equal(_u32(perm), ot.sort(b)[0])
    del torch


def test_datetime_window(gpu_lib):
    # only out-of-window date-times share codes; a window that holds none of
    # them makes every code tie-free, one that holds all of them too
    b = typed("datetime", n=100_000, seed=21)
    r, o = gpu_lib.typed_to_device(b)
    want = ot.sort(b)[0]
    for base in (1970, 1600, 3000):
        np.testing.assert_array_equal(_u32(gpu_lib.sort_typed(r, o, "datetime", b.n, base_year=base)), want)
        got = gpu_lib.encode_typed(r, o, "datetime", b.n, base_year=base).cpu().numpy().view(np.uint64)
        np.testing.assert_array_equal(got, ot.encode(b, base_year=base)[0])


def test_out_of_domain_records_raise(gpu_lib):
    bad = struct.pack("<i5B3xI", 2000, 13, 1, 0, 0, 0, 0)
    good = struct.pack("<i5B3xI", 2000, 1, 1, 0, 0, 0, 0)
    b = _Batch("datetime", [good, bad, good])
    r, o = gpu_lib.typed_to_device(b)
    with pytest.raises(gpu_lib.DomainError):
        gpu_lib.sort_typed(r, o, "datetime", b.n)
    b = _Batch("decimal", [struct.pack("<i", 0) + bytes(17), struct.pack("<i", 1) + b"\x05",
                           struct.pack("<i", 20000) + b"\x01"])
    r, o = gpu_lib.typed_to_device(b)
    with pytest.raises(gpu_lib.DomainError):
        gpu_lib.sort_typed(r, o, "decimal", b.n)
    b = _Batch("tuple", [b"\x01\x02", struct.pack("<q", 3) + b"x"])
    r, o = gpu_lib.typed_to_device(b)
    with pytest.raises(gpu_lib.DomainError):
        gpu_lib.sort_typed(r, o, "tuple", b.n)
