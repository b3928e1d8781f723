"""Pins for the oracle of the non-string coders (numbers, date-times, big
numbers, tuples) against what their definitions fix.

* worked codes derived by hand (tests/golden/typed_codes.tsv);
* the whole sort against a brute-force stable sort by value (Python's own
  int / float / Fraction / tuple order), on generated data and edge sets;
* the coder contract of Sec. 3.2: codes never decrease along the value
  order; the perfect coders (int32, int64, float64, date-times inside the
  128-year window) give equal codes only to equal values;
* the order keys: unsigned byte order of the keys is the value order, and
  keys are equal exactly for equal values (every pair of an edge set);
* coder independence: the null coder gives the same permutation.
"""

import itertools
import math
import os
import struct

import numpy as np
import pytest

from oracle import typed as ot
from workloads.typed import TYPED, typed

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "typed_codes.tsv")


def _golden():
    rows = []
    for line in open(GOLDEN):
        if line.startswith("#") or not line.strip():
            continue
        t, rec, code, _ = line.rstrip("\n").split("\t")
        rows.append((t, bytes.fromhex(rec), int(code, 16)))
    return rows


@pytest.mark.parametrize("row", _golden(), ids=lambda r: f"{r[0]}:{r[1].hex()[:12]}")
def test_golden_codes(row):
    t, rec, code = row
    assert ot.code(t, rec, 1970) == code


class _Batch:
    def __init__(self, t, recs):
        self.type = t
        self.count = len(recs)
        if t in ot.FIXED_SIZE:
            self.data = np.frombuffer(b"".join(recs), dtype=np.uint8)
            self.offsets = None
        else:
            lens = np.array([len(r) for r in recs], dtype=np.int64)
            self.offsets = np.concatenate([[0], np.cumsum(lens)]).astype(np.uint64)
            self.data = np.frombuffer(b"".join(recs) or b"\0", dtype=np.uint8)

    @property
    def n(self):
        return self.count


def _edge_records(t):
    if t == "int32":
        vals = [-(1 << 31), -(1 << 31) + 1, -2, -1, 0, 1, 2, (1 << 31) - 1]
        return [struct.pack("<i", v) for v in vals]
    if t == "int64":
        vals = [-(1 << 63), -(1 << 63) + 1, -(1 << 32), -1, 0, 1, 1 << 32, (1 << 63) - 1]
        return [struct.pack("<q", v) for v in vals]
    if t == "float64":
        vals = [0.0, -0.0, 1.0, -1.0, 5e-324, -5e-324, 1e308, -1e308, math.inf, -math.inf, 0.5, -0.5]
        recs = [struct.pack("<d", v) for v in vals]
        recs += [struct.pack("<Q", b) for b in (0x7FF8000000000000, 0xFFF8000000000000, 0x7FF0000000000001,
                                                0xFFFFFFFFFFFFFFFF)]
        return recs
    if t == "datetime":
        recs = []
        for y in (1600, 1969, 1970, 2000, 2097, 2098, 2500, -(1 << 31), (1 << 31) - 1):
            for f in ((1, 1, 0, 0, 0, 0), (12, 31, 23, 59, 59, 999_999_999), (6, 15, 12, 30, 30, 1)):
                recs.append(struct.pack("<i5B3xI", y, *f))
        return recs
    if t == "bigint":
        vals = [0, 1, -1, 127, 128, -128, -129, 255, 256, -256, -257, 1 << 64, -(1 << 64), (1 << 200) + 3,
                -(1 << 200)]
        recs = [b""]
        for v in vals:
            L = max(1, (v.bit_length() + 8) // 8)
            recs.append(v.to_bytes(L, "big", signed=True))
            recs.append(v.to_bytes(L + 2, "big", signed=True))  # redundant sign bytes
        return recs
    if t == "decimal":
        recs = []
        for u, s in ((0, 0), (0, 7), (15, 1), (150, 2), (-15, 1), (-150, 2), (1, 0), (10, 1), (100, 0),
                     (1, -2), (151, 2), (-151, 2), (2, 0), (19, 1), (-1, 0), (-2, 0), (1, 20), (-1, 20),
                     ((1 << 127) - 1, 0), (-(1 << 127), 0), (123456789, -16000), (-123456789, 16000)):
            L = max(1, ((u if u >= 0 else ~u).bit_length() + 8) // 8)  # shortest form
            recs.append(struct.pack("<i", s) + u.to_bytes(L, "big", signed=True))
        recs.append(struct.pack("<i", 3))  # empty unscaled = 0
        return recs
    if t == "tuple":
        recs = []
        for s in (b"", b"a", b"a\x00", b"a\x00\x00", b"a\x01", b"ab", b"\x00", b"\xff", b"b"):
            for v in (-(1 << 63), -1, 0, 1, (1 << 63) - 1):
                recs.append(struct.pack("<q", v) + s)
        return recs
    raise ValueError(t)


def _brute(b):
    vals = [ot.value(b.type, r) for r in ot.records(b)]
    return np.array(sorted(range(b.n), key=lambda i: vals[i]), dtype=np.uint32)


@pytest.mark.parametrize("t", TYPED)
def test_sort_matches_bruteforce_generated(t):
    b = typed(t, n=20_000, seed=3)
    perm, bad = ot.sort(b)
    assert bad == 0
    np.testing.assert_array_equal(perm, _brute(b))


@pytest.mark.parametrize("t", TYPED)
def test_sort_matches_bruteforce_edges(t):
    recs = _edge_records(t)
    rng = np.random.default_rng(1)
    recs = [recs[i] for i in rng.integers(0, len(recs), size=400)]
    b = _Batch(t, recs)
    np.testing.assert_array_equal(ot.sort(b)[0], _brute(b))


@pytest.mark.parametrize("t", TYPED)
def test_codes_monotone_and_perfect(t):
    recs = _edge_records(t) + ot.records(typed(t, n=3000, seed=5))
    vals = [ot.value(t, r) for r in recs]
    codes = [ot.code(t, r) for r in recs]
    order = sorted(range(len(recs)), key=lambda i: vals[i])
    for a, c in zip(order, order[1:]):
        assert codes[a] <= codes[c], (recs[a].hex(), recs[c].hex())
        if vals[a] == vals[c]:
            assert codes[a] == codes[c]
    perfect = t in ("int32", "int64", "float64") or t == "datetime"
    if perfect:
        for a, c in zip(order, order[1:]):
            if t == "datetime" and not (1970 <= vals[a][0] < 2098 and 1970 <= vals[c][0] < 2098):
                continue
            assert (codes[a] == codes[c]) == (vals[a] == vals[c])


@pytest.mark.parametrize("t", ["bigint", "decimal", "tuple", "datetime"])
def test_order_keys_every_pair(t):
    recs = _edge_records(t)
    keys = [ot.order_key(t, r) for r in recs]
    vals = [ot.value(t, r) for r in recs]
    for i, j in itertools.product(range(len(recs)), repeat=2):
        assert (keys[i] < keys[j]) == (vals[i] < vals[j]), (recs[i].hex(), recs[j].hex())
        assert (keys[i] == keys[j]) == (vals[i] == vals[j])


@pytest.mark.parametrize("t", TYPED)
def test_coder_independence(t):
    b = typed(t, n=5000, seed=9)
    np.testing.assert_array_equal(ot.sort(b)[0], ot.sort(b, coder="null")[0])


def test_domain_counts():
    bad_dt = struct.pack("<i5B3xI", 2000, 13, 1, 0, 0, 0, 0)  # month 13
    b = _Batch("datetime", [bad_dt, struct.pack("<i5B3xI", 2000, 1, 1, 0, 0, 0, 0)])
    assert ot.encode(b)[1] == 1
    big = struct.pack("<i", 0) + bytes(17)  # 17-byte unscaled value
    b = _Batch("decimal", [big, struct.pack("<i", 1) + b"\x05", struct.pack("<i", 16001) + b"\x01"])
    assert ot.encode(b)[1] == 2


def _battery(t):
    """Failed pin names for type t (empty: all pass)."""
    failed = []
    for tt, rec, c in _golden():
        if tt == t and ot.code(t, rec, 1970) != c:
            failed.append("golden")
            break
    recs = _edge_records(t)
    rng = np.random.default_rng(2)
    b = _Batch(t, [recs[i] for i in rng.integers(0, len(recs), size=300)])
    if not np.array_equal(ot.sort(b)[0], _brute(b)):
        failed.append("brute")
    if t in ("bigint", "decimal", "tuple", "datetime"):
        keys = [ot.order_key(t, r) for r in recs]
        vals = [ot.value(t, r) for r in recs]
        if any((keys[i] < keys[j]) != (vals[i] < vals[j]) for i in range(len(recs)) for j in range(len(recs))):
            failed.append("keys")
    return failed


_real_code, _real_key = ot.code, ot.order_key


def _plant_float_no_canonical_nan(t, r, base_year=1970):
    if t == "float64":
        b = struct.unpack("<Q", r)[0]
        return (~b & ot.M64) if b >> 63 else b | (1 << 63)
    return _real_code(t, r, base_year)


def _plant_int32_unsigned(t, r, base_year=1970):
    if t == "int32":
        return struct.unpack("<I", r)[0] << 32
    return _real_code(t, r, base_year)


def _plant_datetime_day_before_month(t, r, base_year=1970):
    if t == "datetime":
        y, mo, d, h, mi, s, ns = ot.datetime_fields(r)
        r = struct.pack("<i5B3xI", y, d % 16, mo, h, mi, s, ns)
    return _real_code(t, r, base_year)


def _plant_bigint_no_length(t, r):
    if t == "bigint":
        return _real_key(t, r)[2:]
    return _real_key(t, r)


def _plant_decimal_keep_trailing_zeros(t, r):
    if t == "decimal":
        scale, u = ot.decimal_parts(r)
        if u:
            d = str(abs(u))
            return (b"\x02" if u > 0 else b"\x00") + (len(d) - scale + 32768).to_bytes(2, "big") + \
                ot._bcd(d)
    return _real_key(t, r)


def _plant_tuple_no_escape(t, r):
    if t == "tuple":
        v = struct.unpack("<q", r[:8])[0]
        return r[8:] + b"\x00" + ((v + (1 << 63)) & ot.M64).to_bytes(8, "big")
    return _real_key(t, r)


PLANTS = {
    "float_no_canonical_nan": ("float64", "code", _plant_float_no_canonical_nan),
    "int32_unsigned": ("int32", "code", _plant_int32_unsigned),
    "datetime_day_before_month": ("datetime", "code", _plant_datetime_day_before_month),
    "bigint_no_length": ("bigint", "order_key", _plant_bigint_no_length),
    "decimal_keep_trailing_zeros": ("decimal", "order_key", _plant_decimal_keep_trailing_zeros),
    "tuple_no_escape": ("tuple", "order_key", _plant_tuple_no_escape),
}


@pytest.mark.parametrize("name", sorted(PLANTS))
def test_planted_mistake_is_caught(name, monkeypatch):
    t, fn, plant = PLANTS[name]
    assert _battery(t) == []
    monkeypatch.setattr(ot, fn, plant)
    assert _battery(t) != [], f"{name} not caught"
