"""Float64 oracle of the learned-CDF model -- test infrastructure only.

The model is a monotone MLP 1 -> 64 -> 64 -> 1 with ReLU activations whose
weights are softplus of free parameters (so every weight is positive and the
output never decreases as the input grows); with monotone=False the raw
parameters are the weights (the deliberately unconstrained variant).
Parameter vector layout (4,353 floats): v1[64], b1[64], v2[64][64] (row =
output unit), b2[64], v3[64], b3.  Loss: mean squared error against target
CDF values.

The fit's deterministic parts are here too, from their definitions: the
SplitMix64 sample indices, the 24-bit cell of a code, the dense cells of a
sorted sample, the cumulative distribution the LUT quantises, and the
equal-depth splitters.

Everything here is written from the definitions with numpy in float64; it
shares nothing with the HIP kernels.
"""

from __future__ import annotations

import numpy as np

H = 64
P = H + H + H * H + H + H + 1  # 4353


def split(p):
    p = np.asarray(p, dtype=np.float64)
    o = 0
    v1 = p[o:o + H]; o += H
    b1 = p[o:o + H]; o += H
    v2 = p[o:o + H * H].reshape(H, H); o += H * H
    b2 = p[o:o + H]; o += H
    v3 = p[o:o + H]; o += H
    b3 = p[o]
    return v1, b1, v2, b2, v3, b3


def softplus(v):
    return np.logaddexp(0.0, v)


def sigmoid(v):
    return 1.0 / (1.0 + np.exp(-v))


def _weight(v, monotone):
    return softplus(v) if monotone else v


def _dweight(v, monotone):
    return sigmoid(v) if monotone else np.ones_like(v)


def forward(p, x, monotone=True):
    """Network output for inputs x (float64 array)."""
    v1, b1, v2, b2, v3, b3 = split(p)
    x = np.asarray(x, dtype=np.float64)
    z1 = np.outer(x, _weight(v1, monotone)) + b1
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ _weight(v2, monotone).T + b2
    h2 = np.maximum(z2, 0.0)
    return h2 @ _weight(v3, monotone) + b3


def loss(p, x, y, monotone=True):
    d = forward(p, x, monotone) - np.asarray(y, dtype=np.float64)
    return float(np.mean(d * d))


def grad(p, x, y, monotone=True):
    """(loss, gradient w.r.t. the parameter vector) by the chain rule."""
    v1, b1, v2, b2, v3, b3 = split(p)
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    B = x.shape[0]
    w1, w2, w3 = _weight(v1, monotone), _weight(v2, monotone), _weight(v3, monotone)
    z1 = np.outer(x, w1) + b1
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ w2.T + b2
    h2 = np.maximum(z2, 0.0)
    out = h2 @ w3 + b3
    d = out - y
    L = float(np.mean(d * d))
    g_out = 2.0 * d / B
    dw3 = h2.T @ g_out
    db3 = g_out.sum()
    dz2 = np.outer(g_out, w3) * (z2 > 0)
    dw2 = dz2.T @ h1
    db2 = dz2.sum(axis=0)
    dz1 = (dz2 @ w2) * (z1 > 0)
    dw1 = dz1.T @ x
    db1 = dz1.sum(axis=0)
    g = np.concatenate([dw1 * _dweight(v1, monotone), db1,
                        (dw2 * _dweight(v2, monotone)).ravel(), db2,
                        dw3 * _dweight(v3, monotone), [db3]])
    return L, g


def numeric_grad(p, x, y, idx, h=1e-6, monotone=True):
    """Central finite differences of the loss at the given parameter indices."""
    p = np.asarray(p, dtype=np.float64).copy()
    out = []
    for i in idx:
        old = p[i]
        p[i] = old + h
        lp = loss(p, x, y, monotone)
        p[i] = old - h
        lm = loss(p, x, y, monotone)
        p[i] = old
        out.append((lp - lm) / (2 * h))
    return np.array(out)


# ----------------------------------------------------------------- the fit's deterministic parts
BUCKETS = 65536
CELLS = 1 << 24
_M64 = (1 << 64) - 1
_GOLDEN = 0x9E3779B97F4A7C15


def splitmix64(x: int) -> int:
    """SplitMix64 output for state x (Steele, Lea and Flood, OOPSLA 2014)."""
    z = (x + _GOLDEN) & _M64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _M64
    return z ^ (z >> 31)


def sample_indices(n: int, S: int, seed: int) -> np.ndarray:
    """String j of the sample: splitmix64(seed + golden * (j + 1)) mod n (with replacement)."""
    return np.array([splitmix64((seed + _GOLDEN * (j + 1)) & _M64) % n for j in range(S)],
                    dtype=np.int64)


def header(sorted_sample):
    """(lo, hi, cp): the sample extremes and the bits of their common prefix."""
    lo, hi = int(sorted_sample[0]), int(sorted_sample[-1])
    cp = 64 if lo == hi else 64 - (lo ^ hi).bit_length()
    return lo, hi, cp


def cell(code: int, lo: int, hi: int, cp: int) -> int:
    """The 24 bits right below the common prefix of the code clamped to [lo, hi]."""
    c = min(max(int(code), lo), hi)
    if cp >= 64:
        return 0
    return ((c << cp) & _M64) >> 40


DENSE_MIN = 16


def dense_cells(sorted_sample, B: int = BUCKETS, min_count: int = DENSE_MIN):
    """Cells holding count * B >= 2 * S sample keys and at least min_count of
    them: (cells ascending, dense keys before each cell (one more entry: all
    dense keys), per-key flag)."""
    lo, hi, cp = header(sorted_sample)
    S = len(sorted_sample)
    w = np.array([cell(c, lo, hi, cp) for c in sorted_sample], dtype=np.int64)
    cells, counts = np.unique(w, return_counts=True)
    c = counts.astype(np.int64)
    dense = cells[(c * B >= 2 * S) & (c >= min_count)]
    flag = np.isin(w, dense)
    cum = [0]
    for d in dense:
        cum.append(cum[-1] + int(np.sum(w == d)))
    return dense, np.array(cum, dtype=np.int64), flag


def cdf_table(f_of_x, dense, cum, S: int):
    """The non-decreasing table of 0.32 fixed-point F(W) for W in [0, 2^24]:
    F(W) = (dense keys in cells < W + (S - dense keys) * f(W / 2^24)) / S,
    then a running maximum, with F(0) = 0 and F(2^24) = 2^32 - 1."""
    W = np.arange(CELLS + 1, dtype=np.int64)
    x = W.astype(np.float64) / CELLS
    before = cum[np.searchsorted(dense, W, side="left")] if len(dense) else np.zeros_like(W)
    F = (before + (S - cum[-1]) * np.clip(f_of_x(x), 0.0, 1.0)) / S
    q = np.minimum(np.floor(F * 4294967295.0), 4294967295.0).astype(np.int64)
    q[0] = 0
    q[-1] = 4294967295
    return np.maximum.accumulate(q)


def splitters(lut, sorted_sample, B: int = BUCKETS):
    """For every cell owning k >= 2 buckets [b0, b1): splitter i (1 <= i < k) =
    the cell's sample key of rank floor(i * m / k) (m = its sample keys),
    stored at b0 + i - 1; all ones when the cell has no sample keys.
    Returns {bucket slot: splitter}."""
    lo, hi, cp = header(sorted_sample)
    w = np.array([cell(c, lo, hi, cp) for c in sorted_sample], dtype=np.int64)
    b = (lut.astype(np.int64) * B) >> 32
    owned = b[1:] - b[:-1]
    out = {}
    for W in np.nonzero(owned >= 2)[0]:
        b0, k = int(b[W]), int(owned[W])
        s_lo = int(np.searchsorted(w, W, side="left"))
        m = int(np.searchsorted(w, W, side="right")) - s_lo
        for i in range(1, k):
            out[b0 + i - 1] = int(sorted_sample[s_lo + (i * m) // k]) if m else _M64
    return out


def sub_bits(k: int, P: int) -> int:
    """Bits of the sub-cell index of a heavy cell owning k >= 2 buckets whose
    splitters share their top P bits."""
    return min(64 - P, 16, (k - 1).bit_length() + 3)


def subtable(lut, split_slots, W: int, B: int = BUCKETS):
    """(first bucket, P, s, prefix, table) of heavy cell W: P = bits shared by its
    first and last splitter, prefix = those bits (the rest zero), table[v] = the
    cell's splitters below prefix | v << (64 - P - s)."""
    b = (lut.astype(np.int64) * B) >> 32
    b0, k = int(b[W]), int(b[W + 1] - b[W])
    spl = np.array([split_slots[b0 + i] for i in range(k - 1)], dtype=np.uint64)
    first, last = int(spl[0]), int(spl[-1])
    P = 64 if first == last else 64 - (first ^ last).bit_length()
    s = sub_bits(k, P)
    prefix = first if P == 64 else (first >> (64 - P)) << (64 - P)
    starts = np.array([prefix | (v << (64 - P - s)) for v in range(1 << s)], dtype=np.uint64)
    # splitters come from the sorted sample, so they are sorted
    table = np.searchsorted(spl, starts, side="left")
    return b0, P, s, prefix, [int(t) for t in table]


def bucket_ids(codes, lut, splitters, lo: int, hi: int, cp: int, B: int = BUCKETS):
    """Bucket of every code: clamp to [lo, hi], cell W; b0 = LUT[W] * B >> 32,
    b1 likewise from LUT[W + 1]; a cell owning k = b1 - b0 >= 2 buckets adds
    the number of its splitters (slots b0 .. b0 + k - 2) not above the code."""
    c = np.clip(np.asarray(codes, dtype=np.uint64), np.uint64(lo), np.uint64(hi))
    if cp >= 64:
        W = np.zeros(c.shape, dtype=np.int64)
    else:
        W = ((c << np.uint64(cp)) >> np.uint64(40)).astype(np.int64)
    b = (np.asarray(lut, dtype=np.int64) * B) >> 32
    b0, b1 = b[W], b[W + 1]
    out = b0.copy()
    heavy = np.nonzero(b1 - b0 >= 2)[0]
    if heavy.size:
        cells = W[heavy]
        for w in np.unique(cells):
            sel = heavy[cells == w]
            lo_b, k = int(b[w]), int(b[w + 1] - b[w])
            spl = np.asarray(splitters[lo_b:lo_b + k - 1], dtype=np.uint64)
            out[sel] = lo_b + np.searchsorted(spl, c[sel], side="right")
    return out
