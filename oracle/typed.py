"""Oracle of the non-string coders -- test infrastructure only.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this module; it shares nothing with the HIP path.

The paper names other object types that are costly to compare and that a
husky code speeds up: date-times (a "perfect" coder for nanosecond
resolution over 128 years, Sec. 3.2), the numeric types Integer, Long,
Double, BigInteger and BigDecimal, and tuples (Sec. 6, "Improvements
Summary").  It defines none of these coders beyond that bit budget; the
readings here are:

* records (the objects as bytes): int32 / int64 / float64 little-endian;
  a date-time is 16 bytes {int32 year; u8 month, day, hour, minute, second;
  3 pad bytes; u32 nano}; a big integer is its two's-complement big-endian
  bytes (empty = 0); a decimal is a 4-byte little-endian int32 scale followed
  by the two's-complement big-endian unscaled value (value = unscaled x
  10^-scale); a tuple is an 8-byte little-endian int64 followed by a byte
  string, compared string first, then the integer;
* comparators: numeric value (Java's compareTo: a decimal's scale does not
  matter, 1.5 == 1.50); doubles in Java's Double.compare order (-inf < ... <
  -0.0 < 0.0 < ... < inf < NaN, every NaN equal); date-times field by field;
* the husky codes (never decreasing in the comparator's order): int32 ->
  (x + 2^31) << 32; int64 -> x + 2^63; float64 -> the IEEE bits with the sign
  flipped for positives and all bits flipped for negatives (NaN made
  canonical first); date-time -> 1 + its fields packed into 63 bits
  (year - base: 7 bits for 128 years, month 4, day 5, hour 5, minute 6,
  second 6, nano 30) inside the window [base, base + 128), 0 below it and
  2^63 + 1 above it.  The first four are perfect (equal codes only for equal
  values; the date-time one inside its window), so Step 3 has nothing to do;
* big integers, decimals and tuples code through an order-preserving byte
  key (``order_key``): the code is the key's first eight bytes, big-endian.

``sort`` follows the method: code, stable sort by code, then a stable sort
of every run of equal codes by the full comparator.
"""

from __future__ import annotations

import math
import struct
from fractions import Fraction

import numpy as np

TYPES = ("int32", "int64", "float64", "datetime", "bigint", "decimal", "tuple")
FIXED_SIZE = {"int32": 4, "int64": 8, "float64": 8, "datetime": 16}
M64 = (1 << 64) - 1

# domain limits of the variable-length types
BIGINT_MAX_BYTES = 32767
DECIMAL_MAX_UNSCALED_BYTES = 16
DECIMAL_MAX_SCALE = 16000


def records(batch):
    """The records of a typed batch as a list of ``bytes``."""
    data = batch.data.tobytes()
    if batch.offsets is None:
        w = FIXED_SIZE[batch.type]
        return [data[i * w:(i + 1) * w] for i in range(batch.n)]
    o = batch.offsets
    return [data[int(o[i]):int(o[i + 1])] for i in range(batch.n)]


# ------------------------------------------------------------------ values and comparators
def _signed_be(b: bytes) -> int:
    return int.from_bytes(b, "big", signed=True) if b else 0


def datetime_fields(r: bytes):
    year, month, day, hour, minute, second, _p0, _p1, _p2, nano = struct.unpack("<i5B3BI", r)
    return year, month, day, hour, minute, second, nano


def datetime_valid(f) -> bool:
    _y, month, day, hour, minute, second, nano = f
    return 1 <= month <= 12 and 1 <= day <= 31 and hour <= 23 and minute <= 59 and second <= 59 \
        and nano < 1_000_000_000


def decimal_parts(r: bytes):
    """(scale, unscaled) of a decimal record."""
    scale = struct.unpack("<i", r[:4])[0]
    return scale, _signed_be(r[4:])


def in_domain(type_: str, r: bytes) -> bool:
    if type_ == "datetime":
        return datetime_valid(datetime_fields(r))
    if type_ == "bigint":
        return len(r) <= BIGINT_MAX_BYTES
    if type_ == "decimal":
        return len(r) >= 4 and len(r) - 4 <= DECIMAL_MAX_UNSCALED_BYTES and \
            abs(struct.unpack("<i", r[:4])[0]) <= DECIMAL_MAX_SCALE
    return True


def value(type_: str, r: bytes):
    """A Python object whose natural order is the type's comparator."""
    if type_ == "int32":
        return struct.unpack("<i", r)[0]
    if type_ == "int64":
        return struct.unpack("<q", r)[0]
    if type_ == "float64":
        x = struct.unpack("<d", r)[0]
        if math.isnan(x):
            return (1, 0.0, 0)
        return (0, x, 0 if math.copysign(1.0, x) < 0 else 1)  # -0.0 before 0.0
    if type_ == "datetime":
        return datetime_fields(r)
    if type_ == "bigint":
        return _signed_be(r)
    if type_ == "decimal":
        scale, u = decimal_parts(r)
        return Fraction(u, 10 ** scale) if scale >= 0 else Fraction(u * 10 ** (-scale))
    if type_ == "tuple":
        return (r[8:], struct.unpack("<q", r[:8])[0])
    raise ValueError(type_)


# ------------------------------------------------------------------ order-preserving keys
def _min_twos(b: bytes) -> bytes:
    """Shortest two's-complement big-endian bytes of the same value (0 -> 00)."""
    v = _signed_be(b)
    n = 1
    while not (-(1 << (8 * n - 1)) <= v < (1 << (8 * n - 1))):
        n += 1
    return v.to_bytes(n, "big", signed=True)


def _bcd(digits: str) -> bytes:
    """Two decimal digits per byte, each nibble digit + 1; an odd count ends in a 0 nibble."""
    nib = [int(c) + 1 for c in digits] + ([0] if len(digits) % 2 else [])
    return bytes((nib[k] << 4) | nib[k + 1] for k in range(0, len(nib), 2))


def order_key(type_: str, r: bytes) -> bytes:
    """Bytes whose unsigned lexicographic order (a proper prefix first) is the
    comparator's order, and that are equal exactly for equal values."""
    if type_ == "bigint":
        m = _min_twos(r)
        L = len(m)
        head = (0x8000 + L) if m[0] < 0x80 else (0x7FFF - L)
        return head.to_bytes(2, "big") + m
    if type_ == "decimal":
        scale, u = decimal_parts(r)
        if u == 0:
            return b"\x01"
        d = str(abs(u))
        t = len(d) - len(d.rstrip("0"))
        d = d.rstrip("0")
        E = len(d) + t - scale  # value = 0.d x 10^E
        body = (E + 32768).to_bytes(2, "big") + _bcd(d)
        if u > 0:
            return b"\x02" + body
        return b"\x00" + bytes(0xFF - c for c in body) + b"\xff"
    if type_ == "tuple":
        s = r[8:].replace(b"\x00", b"\x00\xff")
        v = struct.unpack("<q", r[:8])[0]
        return s + b"\x00\x00" + ((v + (1 << 63)) & M64).to_bytes(8, "big")
    if type_ == "datetime":
        year, month, day, hour, minute, second, nano = datetime_fields(r)
        return ((year + (1 << 31)) & 0xFFFFFFFF).to_bytes(4, "big") + \
            bytes([month, day, hour, minute, second]) + nano.to_bytes(4, "big")
    raise ValueError(type_)


# ------------------------------------------------------------------ husky codes
def code(type_: str, r: bytes, base_year: int = 1970) -> int:
    if type_ == "int32":
        return (struct.unpack("<i", r)[0] + (1 << 31)) << 32
    if type_ == "int64":
        return (struct.unpack("<q", r)[0] + (1 << 63)) & M64
    if type_ == "float64":
        b = struct.unpack("<Q", r)[0]
        if (b >> 52) & 0x7FF == 0x7FF and b & ((1 << 52) - 1):
            b = 0x7FF8000000000000  # every NaN as the canonical one
        return (~b & M64) if b >> 63 else b | (1 << 63)
    if type_ == "datetime":
        year, month, day, hour, minute, second, nano = datetime_fields(r)
        if year < base_year:
            return 0
        if year >= base_year + 128:
            return (1 << 63) + 1
        packed = year - base_year
        for v, bits in ((month, 4), (day, 5), (hour, 5), (minute, 6), (second, 6), (nano, 30)):
            packed = (packed << bits) | v
        return 1 + packed
    k = order_key(type_, r)[:8]
    return int.from_bytes(k + bytes(8 - len(k)), "big")


# ------------------------------------------------------------------ the method
def encode(batch, base_year: int = 1970):
    """(codes uint64[n], out-of-domain records)."""
    recs = records(batch)
    codes = np.array([code(batch.type, r, base_year) for r in recs], dtype=np.uint64)
    bad = sum(0 if in_domain(batch.type, r) else 1 for r in recs)
    return codes, bad


def sort(batch, base_year: int = 1970, coder=None):
    """Huskysort of a typed batch: (perm uint32[n], out-of-domain records).
    coder: None for the type's own husky code, "null" for every code 0."""
    recs = records(batch)
    n = len(recs)
    codes, bad = encode(batch, base_year)
    if coder == "null":
        codes = np.zeros(n, dtype=np.uint64)
    order = sorted(range(n), key=lambda i: int(codes[i]))  # Step 2 (stable)
    vals = [value(batch.type, r) for r in recs]
    out = []
    a = 0
    while a < n:  # Step 3: every run of equal codes, stably, by the comparator
        z = a + 1
        while z < n and codes[order[z]] == codes[order[a]]:
            z += 1
        out.extend(sorted(order[a:z], key=lambda i: vals[i]))
        a = z
    return np.array(out, dtype=np.uint32), bad
