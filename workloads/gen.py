"""Generators for the five string workloads and the adversarial test families.

The paper measures on words split from the Leipzig corpora (Sec. 4.1, "Data
Source"); those files are not available here, so seeded synthetic inputs of the
same kind stand in for them:

* config 1 -- 100,000 lowercase strings, length uniform 1..16 (small case);
* config 2 -- 2^24 strings: 60 % Zipf(1.1) draws from a 200,000-word vocabulary
  (word length geometric with mean 8, at most 24) and 40 % one of 1,000 random
  12-character prefixes plus a random 4..20 character suffix (stands in for the
  English words, with long equal-code runs);
* config 3 -- 2^23 UTF-16 strings of 2..5 units from U+4E00..U+9FA5 (stands in
  for the Chinese words);
* config 4 -- 4,096 independent instances, sizes log-uniform in [64, 262,144],
  each drawn like config 2 with its own seed (batched form);
* config 5 -- 2e8 URL-like strings ``h<host>/<seg>[/<seg>...]`` with Zipf(1.2)
  hosts (learned-CDF form);
* utf8_words -- UTF-8 text of several scripts (bytes of any value, for the
  full-byte coder), a third of it sharing long prefixes;
* the ``bytes*`` adversarial families -- byte strings over 0x00..0xFF that
  stress the full-byte coder's edges.

Every draw goes through ``numpy.random.Generator`` (PCG64) seeded from a
``SeedSequence``; the same seed gives the same bytes on every machine with the
same numpy.
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Dict, List, Optional, Sequence

import numpy as np

LOWER_A = 97  # 'a'
LOWER_Z1 = 123  # one past 'z'

CONFIG_SIZES = {
    1: 100_000,
    2: 1 << 24,
    3: 1 << 23,
    4: 4096,  # number of instances
    5: 200_000_000,
}


@dataclass
class StringBatch:
    elems: np.ndarray
    offsets: np.ndarray
    coder: str  # "ascii7" or "utf16"
    name: str = ""
    seg_offsets: Optional[np.ndarray] = None
    meta: Dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.offsets.shape[0] - 1)

    @property
    def elem_bytes(self) -> int:
        return int(self.elems.dtype.itemsize)

    def lengths(self) -> np.ndarray:
        return np.diff(self.offsets).astype(np.int64)

    def string(self, i: int):
        """String i as ``bytes`` (ASCII) or a tuple of code units (UTF-16)."""
        a, b = int(self.offsets[i]), int(self.offsets[i + 1])
        s = self.elems[a:b]
        return s.tobytes() if self.elems.dtype == np.uint8 else tuple(int(u) for u in s)

    def strings(self) -> List:
        return [self.string(i) for i in range(self.n)]

    def subset(self, lo: int, hi: int) -> "StringBatch":
        """Strings lo..hi-1 as a batch of their own (offsets rebased to 0)."""
        a, b = int(self.offsets[lo]), int(self.offsets[hi])
        return StringBatch(
            elems=np.ascontiguousarray(self.elems[a:b]),
            offsets=(self.offsets[lo:hi + 1] - self.offsets[lo]).astype(np.uint64),
            coder=self.coder,
            name=f"{self.name}[{lo}:{hi}]",
        )


def _rng(*key: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence(list(key))))


def _offsets_from_lengths(lens: np.ndarray) -> np.ndarray:
    off = np.empty(lens.shape[0] + 1, dtype=np.uint64)
    off[0] = 0
    np.cumsum(lens, dtype=np.uint64, out=off[1:])
    return off


def _scatter_copies(out: np.ndarray, dst_starts: np.ndarray, pool: np.ndarray,
                    src_starts: np.ndarray, lens: np.ndarray, chunk: int = 1 << 22) -> None:
    """out[dst_starts[i] + j] = pool[src_starts[i] + j] for j < lens[i] (chunked, vectorised)."""
    n = lens.shape[0]
    for lo in range(0, n, chunk):
        hi = min(n, lo + chunk)
        ln = lens[lo:hi].astype(np.int64)
        tot = int(ln.sum())
        if tot == 0:
            continue
        first = np.empty(hi - lo, dtype=np.int64)
        first[0] = 0
        np.cumsum(ln[:-1], out=first[1:])
        j = np.arange(tot, dtype=np.int64) - np.repeat(first, ln)
        out[np.repeat(dst_starts[lo:hi].astype(np.int64), ln) + j] = \
            pool[np.repeat(src_starts[lo:hi].astype(np.int64), ln) + j]


def from_strings(strings: Sequence, coder: str = "ascii7", name: str = "list") -> StringBatch:
    """Pack a Python list of ``bytes`` (ascii7, bytes8) or unit sequences (utf16)."""
    if coder in ("ascii7", "bytes8"):
        lens = np.array([len(s) for s in strings], dtype=np.int64)
        elems = np.frombuffer(b"".join(bytes(s) for s in strings), dtype=np.uint8).copy()
    elif coder in ("utf16", "utf16_paper"):
        lens = np.array([len(s) for s in strings], dtype=np.int64)
        flat = [int(u) for s in strings for u in s]
        elems = np.array(flat, dtype=np.uint16)
    else:
        raise ValueError(coder)
    return StringBatch(elems=elems, offsets=_offsets_from_lengths(lens), coder=coder, name=name)


# --------------------------------------------------------------------------- config 1
def config1(seed: int = 1, n: int = CONFIG_SIZES[1]) -> StringBatch:
    rng = _rng(seed, 1)
    lens = rng.integers(1, 17, size=n, dtype=np.int64)
    off = _offsets_from_lengths(lens)
    elems = rng.integers(LOWER_A, LOWER_Z1, size=int(off[-1]), dtype=np.uint8)
    return StringBatch(elems, off, "ascii7", name=f"config1(n={n},seed={seed})",
                       meta={"length": "uniform 1..16", "alphabet": "a-z"})


# --------------------------------------------------------------------------- config 2
class _Config2Tables:
    """Vocabulary and prefix set shared by config 2 and every config-4 instance."""

    VOCAB = 200_000
    PREFIXES = 1_000
    PREFIX_LEN = 12
    ZIPF_S = 1.1
    GEO_P = 1.0 / 8.0
    MAX_WORD = 24

    def __init__(self, seed: int):
        rng = _rng(seed, 2, 0)
        lens = rng.geometric(self.GEO_P, size=self.VOCAB).astype(np.int64)
        bad = lens > self.MAX_WORD
        while bad.any():  # resample words longer than 24
            lens[bad] = rng.geometric(self.GEO_P, size=int(bad.sum()))
            bad = lens > self.MAX_WORD
        self.vocab_len = lens
        self.vocab_off = np.concatenate([[0], np.cumsum(lens)[:-1]]).astype(np.int64)
        self.vocab_bytes = rng.integers(LOWER_A, LOWER_Z1, size=int(lens.sum()), dtype=np.uint8)
        self.prefix_bytes = rng.integers(LOWER_A, LOWER_Z1, size=self.PREFIXES * self.PREFIX_LEN,
                                         dtype=np.uint8)
        w = np.arange(1, self.VOCAB + 1, dtype=np.float64) ** (-self.ZIPF_S)
        cdf = np.cumsum(w)
        self.zipf_cdf = cdf / cdf[-1]


_TABLE_CACHE: Dict[int, _Config2Tables] = {}


def _tables(seed: int) -> _Config2Tables:
    if seed not in _TABLE_CACHE:
        _TABLE_CACHE[seed] = _Config2Tables(seed)
    return _TABLE_CACHE[seed]


def _config2_draw(tab: _Config2Tables, rng: np.random.Generator, n: int):
    """Return (elems, offsets) of n config-2 strings drawn with rng."""
    n_vocab = (6 * n) // 10  # exactly floor(0.6 n) vocabulary draws
    n_pref = n - n_vocab
    u = rng.random(n_vocab)
    word = np.minimum(np.searchsorted(tab.zipf_cdf, u, side="right"), tab.VOCAB - 1)
    pid = rng.integers(0, tab.PREFIXES, size=n_pref, dtype=np.int64)
    suf = rng.integers(4, 21, size=n_pref, dtype=np.int64)
    # kind/source before shuffling: vocabulary draws first, then prefixed strings
    lens = np.concatenate([tab.vocab_len[word], tab.PREFIX_LEN + suf])
    perm = rng.permutation(n)
    lens = lens[perm]
    off = _offsets_from_lengths(lens)
    total = int(off[-1])
    elems = rng.integers(LOWER_A, LOWER_Z1, size=total, dtype=np.uint8)  # suffix bytes
    pool = np.concatenate([tab.vocab_bytes, tab.prefix_bytes])
    src = np.concatenate([tab.vocab_off[word], tab.vocab_bytes.shape[0] + pid * tab.PREFIX_LEN])[perm]
    cpy = np.concatenate([tab.vocab_len[word], np.full(n_pref, tab.PREFIX_LEN, dtype=np.int64)])[perm]
    _scatter_copies(elems, off[:-1], pool, src, cpy)
    return elems, off


def config2(seed: int = 1, n: int = CONFIG_SIZES[2]) -> StringBatch:
    tab = _tables(seed)
    elems, off = _config2_draw(tab, _rng(seed, 2, 1), n)
    return StringBatch(elems, off, "ascii7", name=f"config2(n={n},seed={seed})",
                       meta={"vocab": tab.VOCAB, "zipf_s": tab.ZIPF_S, "prefixes": tab.PREFIXES,
                             "vocab_fraction": 0.6})


# --------------------------------------------------------------------------- config 3
def config3(seed: int = 1, n: int = CONFIG_SIZES[3]) -> StringBatch:
    rng = _rng(seed, 3)
    lens = rng.integers(2, 6, size=n, dtype=np.int64)
    off = _offsets_from_lengths(lens)
    elems = rng.integers(0x4E00, 0x9FA6, size=int(off[-1]), dtype=np.uint16)
    return StringBatch(elems, off, "utf16", name=f"config3(n={n},seed={seed})",
                       meta={"length": "uniform 2..5", "units": "U+4E00..U+9FA5"})


# --------------------------------------------------------------------------- config 4
def config4_sizes(seed: int = 1, n_inst: int = CONFIG_SIZES[4], lo: int = 64,
                  hi: int = 262_144) -> np.ndarray:
    rng = _rng(seed, 4, 0)
    s = np.floor(np.exp(rng.uniform(math.log(lo), math.log(hi), size=n_inst))).astype(np.int64)
    return np.clip(s, lo, hi)


def config4(seed: int = 1, n_inst: int = CONFIG_SIZES[4], lo: int = 64, hi: int = 262_144,
            sizes: Optional[np.ndarray] = None) -> StringBatch:
    """Batched workload: instance k drawn like config 2 with its own seed (seed, 4, 1, k)."""
    tab = _tables(seed)
    if sizes is None:
        sizes = config4_sizes(seed, n_inst, lo, hi)
    sizes = np.asarray(sizes, dtype=np.int64)
    parts_e, parts_o = [], []
    base = 0
    for k, sz in enumerate(sizes):
        e, o = _config2_draw(tab, _rng(seed, 4, 1, k), int(sz))
        parts_e.append(e)
        parts_o.append(o[:-1] + np.uint64(base))
        base += int(o[-1])
    elems = np.concatenate(parts_e) if parts_e else np.zeros(0, np.uint8)
    off = np.concatenate(parts_o + [np.array([base], dtype=np.uint64)]).astype(np.uint64)
    seg = _offsets_from_lengths(sizes)
    return StringBatch(elems, off, "ascii7", name=f"config4(inst={len(sizes)},seed={seed})",
                       seg_offsets=seg, meta={"sizes": "log-uniform", "lo": lo, "hi": hi})


# --------------------------------------------------------------------------- config 5
def config5(seed: int = 1, n: int = CONFIG_SIZES[5], hosts: int = 10_000,
            chunk: int = 1 << 23) -> StringBatch:
    """'h' + host id + '/' + 1..4 segments of 3..10 lowercase letters joined by '/'."""
    rng = _rng(seed, 5, 0)
    host_perm = rng.permutation(hosts)  # Zipf rank r -> host id host_perm[r - 1]
    w = np.arange(1, hosts + 1, dtype=np.float64) ** (-1.2)
    cdf = np.cumsum(w)
    cdf /= cdf[-1]
    host_str = [b"h" + str(int(h)).encode() + b"/" for h in host_perm]
    host_len = np.array([len(s) for s in host_str], dtype=np.int64)
    host_off = np.concatenate([[0], np.cumsum(host_len)[:-1]]).astype(np.int64)
    host_pool = np.frombuffer(b"".join(host_str), dtype=np.uint8)

    rng = _rng(seed, 5, 1)
    ranks = np.empty(n, dtype=np.int64)
    nseg = np.empty(n, dtype=np.int64)
    seglen = np.empty((n, 4), dtype=np.int64)
    for lo in range(0, n, chunk):
        hi = min(n, lo + chunk)
        ranks[lo:hi] = np.minimum(np.searchsorted(cdf, rng.random(hi - lo), side="right"), hosts - 1)
        nseg[lo:hi] = rng.integers(1, 5, size=hi - lo)
        seglen[lo:hi] = rng.integers(3, 11, size=(hi - lo, 4))
    seglen[np.arange(4)[None, :] >= nseg[:, None]] = 0
    hl = host_len[ranks]
    lens = hl + seglen.sum(axis=1) + (nseg - 1)
    off = _offsets_from_lengths(lens)
    total = int(off[-1])
    elems = np.empty(total, dtype=np.uint8)
    for lo in range(0, total, 1 << 28):
        hi = min(total, lo + (1 << 28))
        elems[lo:hi] = rng.integers(LOWER_A, LOWER_Z1, size=hi - lo, dtype=np.uint8)
    _scatter_copies(elems, off[:-1], host_pool, host_off[ranks], hl)
    # separators between path segments
    pos = off[:-1].astype(np.int64) + hl
    for j in range(1, 4):
        pos = pos + seglen[:, j - 1]
        has = nseg > j
        elems[pos[has]] = ord("/")
        pos = pos + 1
    del seglen
    return StringBatch(elems, off, "ascii7", name=f"config5(n={n},seed={seed})",
                       meta={"hosts": hosts, "zipf_s": 1.2, "host_map": "seeded permutation"})


# --------------------------------------------------------------------------- adversarial
ADVERSARIAL_FAMILIES = (
    "empty", "nul", "identical", "prefix9", "prefix12", "high_after9", "len_edges",
    "alphabet3", "mixed", "utf16_edges", "utf16_prefix4", "utf16_full",
)


def adversarial(family: str, seed: int = 1, n: int = 2000) -> StringBatch:
    """Small inputs that stress the coder's edges (Alg. 4 padding, masking, NULs, ties)."""
    rng = _rng(seed, 100, ADVERSARIAL_FAMILIES.index(family))
    if family.startswith("utf16"):
        return _adversarial_utf16(family, rng, n)

    def rand_bytes(lo, hi, k):
        return bytes(rng.integers(lo, hi, size=k, dtype=np.uint8).tolist())

    out: List[bytes] = []
    if family == "empty":
        for _ in range(n):
            r = rng.random()
            out.append(b"" if r < 0.4 else rand_bytes(97, 100, int(rng.integers(1, 4))))
    elif family == "nul":
        base = [b"ab", b"ab\0", b"ab\0\0", b"a", b"a\0", b"\0", b"", b"abcdefghi\0", b"abcdefghi",
                b"abcdefghi\0\0", b"abcdefghij\0", b"\0\0\0\0\0\0\0\0\0\0"]
        for _ in range(n):
            if rng.random() < 0.5:
                out.append(base[int(rng.integers(0, len(base)))])
            else:
                k = int(rng.integers(0, 20))
                s = bytearray(rand_bytes(97, 99, k))
                for p in range(k):
                    if rng.random() < 0.3:
                        s[p] = 0
                out.append(bytes(s))
    elif family == "identical":
        words = [b"supercalifragilistic", b"abcdefghijklmnopqrstuvwxyz", b"short", b"abcdefghi",
                 b"abcdefghij" * 5]
        for _ in range(n):
            out.append(words[int(rng.integers(0, len(words)))] if rng.random() < 0.95
                       else rand_bytes(97, 123, int(rng.integers(1, 30))))
    elif family in ("prefix9", "prefix12"):
        plen = 9 if family == "prefix9" else 12
        prefixes = [rand_bytes(97, 123, plen) for _ in range(5)]
        for _ in range(n):
            p = prefixes[int(rng.integers(0, 5))]
            k = int(rng.integers(0, 25))
            out.append(p[: int(rng.integers(0, plen + 1))] if rng.random() < 0.1
                       else p + rand_bytes(97, 100, k))
    elif family == "high_after9":
        prefixes = [rand_bytes(97, 99, 9) for _ in range(3)]
        for _ in range(n):
            k = int(rng.integers(0, 20))
            out.append(prefixes[int(rng.integers(0, 3))] + rand_bytes(0, 256, k))
    elif family == "len_edges":
        p = b"abcdefghijklmnopqrstuvwxyz"
        for _ in range(n):
            L = int(rng.choice([7, 8, 9, 10, 15, 16, 17, 23, 24, 30]))
            s = bytearray(p[:L] if L <= 26 else p + p[: L - 26])
            if rng.random() < 0.5 and L > 0:
                s[int(rng.integers(0, L))] = int(rng.integers(97, 100))
            out.append(bytes(s))
    elif family == "alphabet3":
        alpha = np.array([0x00, 0x61, 0x7F], dtype=np.uint8)
        for _ in range(n):
            k = int(rng.integers(0, 14))
            out.append(bytes(alpha[rng.integers(0, 3, size=k)].tolist()))
    elif family == "mixed":
        for _ in range(n):
            k = int(rng.integers(0, 40))
            out.append(rand_bytes(0, 128, min(k, 9)) + rand_bytes(0, 256, max(0, k - 9)))
    else:
        raise ValueError(family)
    return from_strings(out, "ascii7", name=f"adv:{family}(n={n},seed={seed})")


def _adversarial_utf16(family: str, rng: np.random.Generator, n: int) -> StringBatch:
    out: List[tuple] = []
    if family == "utf16_edges":
        base = [(), (0,), (0, 0), (0x4E00,), (0x4E00, 0), (0x4E00, 0x4E00, 0x4E00, 0x4E00),
                (0x4E00, 0x4E00, 0x4E00, 0x4E01), (0x4E00, 0x4E00, 0x4E00, 0x4E00, 0x4E00),
                (0xFFFF,) * 4, (0xFFFF,) * 5, (0x8000,), (0x7FFF, 0xFFFF)]
        for _ in range(n):
            if rng.random() < 0.5:
                out.append(base[int(rng.integers(0, len(base)))])
            else:
                k = int(rng.integers(0, 9))
                out.append(tuple(int(x) for x in rng.choice([0, 1, 0x7FFF, 0x8000, 0xFFFF], size=k)))
    elif family == "utf16_prefix4":
        prefixes = [tuple(int(x) for x in rng.integers(0x4E00, 0x9FA6, size=4)) for _ in range(4)]
        for _ in range(n):
            p = prefixes[int(rng.integers(0, 4))]
            k = int(rng.integers(0, 12))
            out.append(p + tuple(int(x) for x in rng.integers(0x4E00, 0x4E03, size=k)))
    elif family == "utf16_full":
        for _ in range(n):
            k = int(rng.integers(0, 12))
            out.append(tuple(int(x) for x in rng.integers(0, 0x10000, size=k)))
    else:
        raise ValueError(family)
    return from_strings(out, "utf16", name=f"adv:{family}(n={n})")


# --------------------------------------------------------------------------- UTF-8 text
# code point ranges of the scripts drawn, and the share of strings written in each
UTF8_SCRIPTS = (
    ("latin_lower", 0x61, 0x7B, 0.40),
    ("latin_accented", 0xC0, 0x180, 0.15),  # Latin-1 Supplement + Latin Extended-A
    ("greek", 0x3B1, 0x3CA, 0.10),
    ("cyrillic", 0x430, 0x450, 0.10),
    ("cjk", 0x4E00, 0x9FA6, 0.20),
    ("emoji", 0x1F600, 0x1F650, 0.05),
)


def _utf8_encode(cps: np.ndarray, lens: np.ndarray):
    """UTF-8 bytes of the code points cps (flat, strings of lens code points each):
    (bytes uint8, byte offsets uint64[n + 1])."""
    cps = cps.astype(np.int64)
    k = 1 + (cps >= 0x80) + (cps >= 0x800) + (cps >= 0x10000)
    start = np.concatenate([[0], np.cumsum(k)]).astype(np.int64)
    out = np.empty(int(start[-1]), dtype=np.uint8)
    lead = np.where(k == 1, cps,
                    np.where(k == 2, 0xC0 | (cps >> 6),
                             np.where(k == 3, 0xE0 | (cps >> 12), 0xF0 | (cps >> 18))))
    out[start[:-1]] = lead.astype(np.uint8)
    for j in range(1, 4):  # continuation byte j of the code points that have one
        has = k > j
        shift = 6 * (k[has] - 1 - j)
        out[start[:-1][has] + j] = (0x80 | ((cps[has] >> shift) & 0x3F)).astype(np.uint8)
    cp_off = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    return out, start[cp_off].astype(np.uint64)


def utf8_words(seed: int = 1, n: int = 1 << 20, prefixes: int = 500) -> StringBatch:
    """UTF-8 strings of 1..12 code points, each in one script of UTF8_SCRIPTS
    (drawn by its share); a third of them are one of `prefixes` seeded 4..7
    code point prefixes (8..28 bytes, so their codes tie) plus 0..6 more code
    points of the prefix's script.  Sorted as bytes this is code point order."""
    rng = _rng(seed, 6, 0)
    shares = np.array([s[3] for s in UTF8_SCRIPTS])
    lo = np.array([s[1] for s in UTF8_SCRIPTS], dtype=np.int64)
    hi = np.array([s[2] for s in UTF8_SCRIPTS], dtype=np.int64)
    # the prefixes: script, length, code points
    p_script = rng.choice(len(UTF8_SCRIPTS), size=prefixes, p=shares)
    p_len = rng.integers(4, 8, size=prefixes)
    p_cps = [rng.integers(lo[s], hi[s], size=int(L)) for s, L in zip(p_script, p_len)]
    rng = _rng(seed, 6, 1)
    use_prefix = rng.random(n) < 1.0 / 3.0
    which = rng.integers(0, prefixes, size=n)
    script = np.where(use_prefix, p_script[which], rng.choice(len(UTF8_SCRIPTS), size=n, p=shares))
    extra = np.where(use_prefix, rng.integers(0, 7, size=n), rng.integers(1, 13, size=n))
    plen = np.where(use_prefix, p_len[which], 0)
    lens = plen + extra
    total = int(lens.sum())
    cps = np.empty(total, dtype=np.int64)
    cp_off = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    # random code points of each string's script, then the prefixes over them
    cps[:] = rng.integers(0, 1 << 40, size=total)
    sc = np.repeat(script, lens)
    cps = lo[sc] + cps % (hi[sc] - lo[sc])
    for i in np.nonzero(use_prefix)[0]:
        p = p_cps[which[i]]
        cps[cp_off[i]:cp_off[i] + len(p)] = p
    elems, off = _utf8_encode(cps, lens)
    return StringBatch(elems, off, "bytes8", name=f"utf8_words(n={n},seed={seed})",
                       meta={"scripts": [s[0] for s in UTF8_SCRIPTS], "prefixes": prefixes})


BYTES_FAMILIES = ("bytes_edges", "bytes_alphabet4", "bytes_prefix8", "bytes_random")


def adversarial_bytes(family: str, seed: int = 1, n: int = 2000) -> StringBatch:
    """Byte strings over the whole range 0x00..0xFF for the full-byte coder: the
    values either side of 0x80, NULs against the code's zero padding, strings
    around the coded length, shared 8-byte prefixes."""
    rng = _rng(seed, 101, BYTES_FAMILIES.index(family))

    def rand_bytes(lo, hi_, k):
        return bytes(rng.integers(lo, hi_, size=k, dtype=np.uint8).tolist())

    out: List[bytes] = []
    if family == "bytes_edges":
        base = [b"", b"\x00", b"\x7f", b"\x80", b"\xff", b"\x80\x00", b"\xff" * 8, b"\xff" * 9,
                b"\x00" * 8, b"\x00" * 9, b"abcdefgh", b"abcdefgh\x00", b"abcdefgh\x80",
                b"abcdefgh\xff", b"abcdefg\x80", b"\x7f" * 8 + b"\x80", b"\xc3\xa9", b"e\xcc\x81"]
        for _ in range(n):
            if rng.random() < 0.5:
                out.append(base[int(rng.integers(0, len(base)))])
            else:
                k = int(rng.integers(0, 18))
                vals = np.array([0x00, 0x01, 0x7F, 0x80, 0x81, 0xFE, 0xFF], dtype=np.uint8)
                out.append(bytes(vals[rng.integers(0, len(vals), size=k)].tolist()))
    elif family == "bytes_alphabet4":
        alpha = np.array([0x00, 0x7F, 0x80, 0xFF], dtype=np.uint8)
        for _ in range(n):
            k = int(rng.integers(0, 13))
            out.append(bytes(alpha[rng.integers(0, 4, size=k)].tolist()))
    elif family == "bytes_prefix8":
        prefixes = [rand_bytes(0, 256, 8) for _ in range(5)] + [b"\xff" * 8, b"\x80" * 8]
        for _ in range(n):
            p = prefixes[int(rng.integers(0, len(prefixes)))]
            k = int(rng.integers(0, 25))
            out.append(p[: int(rng.integers(0, 9))] if rng.random() < 0.1
                       else p + rand_bytes(0x7E, 0x82, k))
    elif family == "bytes_random":
        for _ in range(n):
            out.append(rand_bytes(0, 256, int(rng.integers(0, 40))))
    else:
        raise ValueError(family)
    return from_strings(out, "bytes8", name=f"adv:{family}(n={n},seed={seed})")
