"""Seeded typed records for the non-string coders (numbers, date-times, big
numbers, tuples).  Like the string generators this module only draws data:
records are plain bytes, the layouts documented in ``include/husky.h``
(``husky_type``).  The paper measures these types on 20,000-500,000
elements (Sec. 6, "Improvements Summary") without describing its data; the
generators below mix uniform draws, duplicates, extremes and the edge values
of each comparator.
"""

from __future__ import annotations

from dataclasses import dataclass
from typing import List, Optional

import numpy as np

from .gen import _rng

TYPED = ("int32", "int64", "float64", "datetime", "bigint", "decimal", "tuple")
TYPE_IDS = {t: i for i, t in enumerate(TYPED)}
FIXED_SIZE = {"int32": 4, "int64": 8, "float64": 8, "datetime": 16}

DATETIME_DTYPE = np.dtype([("year", "<i4"), ("month", "u1"), ("day", "u1"), ("hour", "u1"),
                           ("minute", "u1"), ("second", "u1"), ("pad", "u1", 3), ("nano", "<u4")])
assert DATETIME_DTYPE.itemsize == 16


@dataclass
class TypedBatch:
    type: str
    data: np.ndarray                 # uint8 records, back to back
    offsets: Optional[np.ndarray]    # uint64[n + 1] byte offsets (variable-length types)
    count: int
    name: str = ""

    @property
    def n(self) -> int:
        return self.count


def _fixed(type_, arr: np.ndarray, name) -> TypedBatch:
    data = np.ascontiguousarray(arr).view(np.uint8).reshape(-1).copy()
    return TypedBatch(type_, data, None, int(arr.shape[0]), name)


def _var(type_, recs: List[bytes], name) -> TypedBatch:
    lens = np.array([len(r) for r in recs], dtype=np.int64)
    off = np.concatenate([[0], np.cumsum(lens)]).astype(np.uint64)
    data = np.frombuffer(b"".join(recs), dtype=np.uint8).copy() if recs else np.zeros(0, np.uint8)
    return TypedBatch(type_, data, off, len(recs), name)


def typed(type_: str, n: int = 100_000, seed: int = 1, base_year: int = 1970) -> TypedBatch:
    rng = _rng(seed, 7, TYPE_IDS[type_])
    name = f"{type_}(n={n},seed={seed})"
    if type_ in ("int32", "int64"):
        dt = np.int32 if type_ == "int32" else np.int64
        info = np.iinfo(dt)
        v = rng.integers(info.min, info.max, size=n, dtype=dt, endpoint=True)
        dup = rng.random(n) < 0.2  # duplicates of a small pool
        v[dup] = rng.integers(-50, 50, size=int(dup.sum())).astype(dt)
        ext = rng.random(n) < 0.01
        v[ext] = rng.choice(np.array([info.min, info.min + 1, -1, 0, 1, info.max - 1, info.max], dtype=dt),
                            size=int(ext.sum()))
        return _fixed(type_, v, name)
    if type_ == "float64":
        v = rng.standard_normal(n) * 10.0 ** rng.uniform(-30, 30, size=n)
        kind = rng.random(n)
        specials = np.array([0.0, -0.0, np.inf, -np.inf, np.nan, 5e-324, -5e-324, 2.2250738585072014e-308,
                             1.0, -1.0, 1.7976931348623157e308], dtype=np.float64)
        sp = kind < 0.03
        v[sp] = rng.choice(specials, size=int(sp.sum()))
        dup = (kind >= 0.03) & (kind < 0.15)
        v[dup] = rng.integers(-20, 20, size=int(dup.sum())) / 4.0
        bits = v.view(np.uint64).copy()
        nan_payload = (kind >= 0.15) & (kind < 0.16)  # NaNs of either sign and any payload
        bits[nan_payload] = (np.uint64(0x7FF0000000000001) + rng.integers(0, 1 << 51, size=int(nan_payload.sum()),
                                                                            dtype=np.uint64)) | \
            (rng.integers(0, 2, size=int(nan_payload.sum()), dtype=np.uint64) << np.uint64(63))
        return _fixed(type_, bits.view(np.float64), name)
    if type_ == "datetime":
        a = np.zeros(n, dtype=DATETIME_DTYPE)
        inside = rng.random(n) < 0.9
        a["year"] = np.where(inside, rng.integers(base_year, base_year + 128, size=n),
                             np.where(rng.random(n) < 0.5, rng.integers(1600, base_year, size=n),
                                      rng.integers(base_year + 128, 2500, size=n)))
        a["month"] = rng.integers(1, 13, size=n)
        a["day"] = rng.integers(1, 29, size=n)
        a["hour"] = rng.integers(0, 24, size=n)
        a["minute"] = rng.integers(0, 60, size=n)
        a["second"] = rng.integers(0, 60, size=n)
        a["nano"] = rng.integers(0, 1_000_000_000, size=n)
        # a fifth share a coarse timestamp (equal up to the second or exactly)
        coarse = rng.random(n) < 0.2
        a["nano"][coarse] = rng.choice([0, 500_000_000], size=int(coarse.sum()))
        a["second"][coarse] = 0
        a["minute"][coarse] = 0
        edges = rng.random(n) < 0.01
        a["year"][edges] = rng.choice([base_year - 1, base_year, base_year + 127, base_year + 128,
                                       -(1 << 31), (1 << 31) - 1], size=int(edges.sum()))
        return _fixed(type_, a, name)
    recs: List[bytes] = []
    if type_ == "bigint":
        pool = [bytes([0]), bytes([0xFF]), bytes([0x7F]), bytes([0x80]), bytes([0, 0x80]),
                bytes([0xFF, 0x7F]), bytes([0, 0, 0, 5]), bytes([0xFF, 0xFF, 0xFE]), b""]
        for _ in range(n):
            r = rng.random()
            if r < 0.05:
                recs.append(pool[int(rng.integers(0, len(pool)))])
            elif r < 0.25:  # small values, sometimes with redundant sign bytes
                v = int(rng.integers(-300, 300))
                L = max(1, (v.bit_length() + 8) // 8) + int(rng.integers(0, 3))
                recs.append(v.to_bytes(L, "big", signed=True))
            else:
                L = int(np.exp(rng.uniform(0, np.log(40))))
                recs.append(bytes(rng.integers(0, 256, size=L, dtype=np.uint8).tolist()))
        return _var(type_, recs, name)
    if type_ == "decimal":
        for _ in range(n):
            r = rng.random()
            if r < 0.3:  # equal values written with different scales
                u, s = int(rng.integers(-60, 60)), int(rng.integers(0, 4))
                k = int(rng.integers(0, 4))
                u, s = u * 10 ** k, s + k
            else:
                L = int(rng.integers(0, 17))
                u = int.from_bytes(bytes(rng.integers(0, 256, size=L, dtype=np.uint8).tolist()), "big",
                                   signed=True) if L else 0
                s = int(rng.integers(-20, 31))
            L = max(1, (u.bit_length() + 8) // 8)
            body = u.to_bytes(L, "big", signed=True) if (u or rng.random() < 0.5) else b""
            if len(body) > 16:
                body = body[-16:]
            recs.append(int(s).to_bytes(4, "little", signed=True) + body)
        return _var(type_, recs, name)
    if type_ == "tuple":
        words = [b"", b"a", b"ab", b"ab\x00", b"abc", b"b", b"alpha", b"alphabet", b"\x00", b"zz\xff"] + \
            [bytes(rng.integers(97, 123, size=int(rng.integers(1, 14)), dtype=np.uint8).tolist())
             for _ in range(200)]
        w = 1.0 / np.arange(1, len(words) + 1) ** 1.1
        w /= w.sum()
        pick = rng.choice(len(words), size=n, p=w)
        vals = np.where(rng.random(n) < 0.5, rng.integers(-5, 5, size=n),
                        rng.integers(-(1 << 62), 1 << 62, size=n)).astype(np.int64)
        for k in range(n):
            recs.append(int(vals[k]).to_bytes(8, "little", signed=True) + words[int(pick[k])])
        return _var(type_, recs, name)
    raise ValueError(type_)
