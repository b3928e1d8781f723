"""GPU: the inference kernel (the network evaluated over all 2^24 + 1 cells, the
running maximum, the 0.32 fixed-point table) against the float64 oracle.

The table the fit builds is compared entry by entry with the oracle's
``cdf_table`` of the same parameters, evaluated in float64, for

* networks the GPU trained itself (monotone and raw weights, a workload with
  no dense cells and one where most of the sample is in dense cells), and
* seeded parameters with sizeable biases fed to the kernel alone
  (``husky_learned_eval_lut``), so every parameter group shapes the output.

Tolerance, from the FP32 arithmetic of one evaluation.  With u = 2^-24 and
M(x) = |b3| + sum_k |w3_k| (|b2_k| + sum_j |W2_kj| (|w1_j| x + |b1_j|)) -- the
network with every weight and bias replaced by its magnitude -- the kernel's
output differs from the exact one by at most (2 + 64 + 64 + 3 * 4) u M(x) to
first order: the first layer's multiply-add, the two 64-term sums of the
later layers, and up to 4 u of relative error in each softplus weight (ReLU
and the clamp to [0, 1] only shrink differences).  The test allows twice
that, 300 u M(x).  The table entry is floor((before + rest f) / S *
(2^32 - 1)), so it may differ by (rest / S) 2^32 * 300 u M(x) + 2 (the two
floors).  A running maximum moves no entry by more than the largest
difference at or before it, so entry W is allowed the running maximum of
those bounds up to W.

The oracle copies with a planted mistake (a bias left out, the 64 x 64 matrix
transposed, a ReLU left out, identity instead of softplus) must each fail that
comparison: the test can see such mistakes.
"""

import math

import numpy as np
import pytest

import oracle
from oracle import learned as ol
from _progress import say
from workloads import config3, config5

pytestmark = pytest.mark.gpu

H = ol.H
U = 2.0 ** -24
C_FP32 = 300.0
CHUNK = 1 << 15


def _layers(p, monotone, plant=None):
    """Weights with the bias as an extra input row: layer(h) = [h, 1] @ A."""
    v1, b1, v2, b2, v3, b3 = ol.split(p)
    w = (lambda v: v) if (not monotone or plant == "identity_weights") else ol.softplus
    w1, w2, w3 = w(v1), w(v2), w(v3)
    if plant == "transpose_w2":
        w2 = w2.T
    if plant == "drop_b2":
        b2 = np.zeros_like(b2)
    if plant == "drop_b3":
        b3 = 0.0
    return (np.vstack([w1, b1]), np.vstack([w2.T, b2]), np.append(w3, b3))


_BUF = {}


def _bufs(n):
    # reused work arrays (fresh multi-megabyte arrays per chunk cost more in
    # page faults than the products themselves); the last column holds the
    # ones that multiply the bias rows
    if n not in _BUF:
        bufs = [np.ones((n, 2)), np.ones((n, ol.H + 1)), np.ones((n, ol.H + 1))]
        _BUF.clear()
        _BUF[n] = bufs
    return _BUF[n]


def _forward(A1, A2, a3, x, relu1=True, relu2=True):
    """float64 forward pass of the network: the oracle's arithmetic (ol.forward),
    with each bias folded into its matrix product."""
    X, H1, H2 = _bufs(x.size)
    X[:, 0] = x
    np.matmul(X, A1, out=H1[:, :ol.H])
    if relu1:
        np.maximum(H1[:, :ol.H], 0.0, out=H1[:, :ol.H])
    np.matmul(H1, A2, out=H2[:, :ol.H])
    if relu2:
        np.maximum(H2[:, :ol.H], 0.0, out=H2[:, :ol.H])
    return H2 @ a3


def _net(p, x, monotone, plant=None):
    """The network at x, optionally with one planted mistake."""
    A1, A2, a3 = _layers(p, monotone, plant)
    return _forward(A1, A2, a3, x, plant != "no_relu1", plant != "no_relu2")


def _chunked(fn, upto=None):
    """fn over x in chunks; with upto, only x[:upto] is evaluated (the rest is 0)."""
    def f(x):
        out = np.zeros_like(x)
        end = x.size if upto is None else min(upto, x.size)
        for a in range(0, end, CHUNK):
            b = min(a + CHUNK, end)
            out[a:b] = fn(x[a:b])
        return out
    return f


def _magnitude(p, x, monotone):
    """M(x): the network with every weight and bias replaced by its magnitude."""
    A1, A2, a3 = (np.abs(a) for a in _layers(p, monotone))
    return _forward(A1, A2, a3, x, False, False)


GRID = 1 << 14


def _tolerance(p, monotone, rest, S):
    """Allowed |GPU - oracle| per table entry.  M never decreases in x >= 0 (all of
    its weights and biases are non-negative), so M at the next multiple of GRID
    cells bounds M over the cells below it."""
    W = np.arange(ol.CELLS + 1, dtype=np.int64)
    knots = np.arange(0, ol.CELLS + GRID, GRID, dtype=np.float64) / ol.CELLS
    M = _magnitude(p, knots, monotone)[(W + GRID - 1) // GRID]
    tol = np.floor((rest / S) * 2.0 ** 32 * C_FP32 * U * M) + 2
    return np.maximum.accumulate(tol)


def _oracle_table(p, monotone, dense, cum, S, plant=None, upto=None):
    """The oracle's table; with upto, only its first `upto` entries are meaningful
    (an entry depends on the cells at or below it only)."""
    return ol.cdf_table(_chunked(lambda xx: _net(p, xx, monotone, plant), upto), dense, cum, S)


def _gpu_u32(t):
    return t.cpu().numpy().view(np.uint32).astype(np.int64)


def _fit(gpu_lib, b, **kw):
    e, o = gpu_lib.to_device(b)
    params = gpu_lib.make_learned_params(**kw)
    model = gpu_lib.fit_learned(e, o, b.coder, params)
    return model


def _oracle_dense(gpu_lib, b, model, frac, seed):
    """The oracle's sample, dense cells and counts for the fit (checked against the model's)."""
    import torch

    h = gpu_lib.learned_header(model)
    S = math.ceil(frac * b.n)
    codes, _ = oracle.encode(b)
    sample = np.sort(codes[ol.sample_indices(b.n, S, seed)]).astype(object)
    dense, cum, _ = ol.dense_cells(sample)
    assert h["sample"] == S and h["dense"] == len(dense) and h["dense_keys"] == cum[-1]
    got = gpu_lib.learned_part(model, "dense", torch.int32, len(dense)).cpu().numpy().view(np.uint32)
    np.testing.assert_array_equal(got, dense)
    return dense, cum, S


def _compare(gpu, ref, tol, what):
    d = np.abs(gpu - ref)
    bad = np.nonzero(d > tol)[0]
    say(what, "max |diff|", int(d.max()), "max tolerance", int(tol.max()),
        "median |diff|", float(np.median(d)), "entries over", bad.size)
    return bad


FITS = [
    # (maker, fit keywords, monotone): UTF-16 CJK strings have no dense cell, so
    # the network alone shapes the table; the URL strings put most of the
    # sample in dense cells and the network models the rest
    (lambda: config3(n=400_000, seed=31), dict(sample_frac=0.05, seed=5), True),
    (lambda: config3(n=400_000, seed=32), dict(sample_frac=0.05, seed=6, mode="unconstrained"), False),
    (lambda: config5(n=300_000, seed=33), dict(sample_frac=0.05, seed=7), True),
]


@pytest.mark.parametrize("maker,kw,monotone", FITS, ids=["utf16_monotone", "utf16_raw", "urls_monotone"])
def test_trained_lut_matches_oracle(gpu_lib, maker, kw, monotone):
    import torch

    b = maker()
    model = _fit(gpu_lib, b, **kw)
    h = gpu_lib.learned_header(model)
    assert h["steps"] > 0 and h["trained"] > 0
    dense, cum, S = _oracle_dense(gpu_lib, b, model, kw["sample_frac"], kw["seed"])
    p = gpu_lib.learned_part(model, "params", torch.float32, ol.P).cpu().numpy().astype(np.float64)
    gpu = _gpu_u32(gpu_lib.learned_part(model, "lut", torch.int32, ol.CELLS + 1))
    ref = _oracle_table(p, monotone, dense, cum, S)
    tol = _tolerance(p, monotone, S - int(cum[-1]), S)
    bad = _compare(gpu, ref, tol, b.name)
    assert bad.size == 0, f"first entries over tolerance: {bad[:8].tolist()}"
    # the kernel alone, called on the model's own parameters, builds the same table
    again = _gpu_u32(gpu_lib.learned_eval_lut(model, mode="monotone" if monotone else "unconstrained"))
    np.testing.assert_array_equal(again, gpu)


def _seeded_params(seed, monotone):
    """Parameters whose every group matters: biases of either sign and of a size that
    moves the output by tenths."""
    rng = np.random.default_rng(seed)
    p = np.empty(ol.P)
    p[0:64] = rng.normal(0.5, 0.5, 64)                  # v1
    p[64:128] = rng.uniform(-1.0, 0.2, 64)              # b1: knots across [0, 1]
    p[128:128 + 4096] = rng.normal(-4.2, 0.8, 4096)     # v2
    p[4224:4288] = rng.normal(-0.05, 0.3, 64)           # b2
    p[4288:4352] = rng.normal(-3.4, 0.6, 64)            # v3
    p[4352] = 0.15                                      # b3
    if not monotone:
        # raw weights: the softplus values with random signs on half of them
        w = np.r_[ol.softplus(p[0:64]), ol.softplus(p[128:4224]), ol.softplus(p[4288:4352])]
        w *= np.where(rng.random(w.size) < 0.5, -1.0, 1.0) * 3.0
        p[0:64], p[128:4224], p[4288:4352] = w[:64], w[64:64 + 4096], w[64 + 4096:]
    return p.astype(np.float32)


# the planted copies are compared on the first PLANT_CELLS entries only
PLANT_CELLS = 1 << 21
PLANTS = ["drop_b2", "drop_b3", "transpose_w2", "no_relu1", "no_relu2"]


@pytest.mark.parametrize("monotone", [True, False], ids=["softplus", "raw"])
def test_eval_lut_seeded_params_and_planted_mistakes(gpu_lib, monotone):
    import torch

    b = config3(n=200_000, seed=34)
    kw = dict(sample_frac=0.05, seed=9, mode="equal_width")
    model = _fit(gpu_lib, b, **kw)
    dense, cum, S = _oracle_dense(gpu_lib, b, model, kw["sample_frac"], kw["seed"])
    p32 = _seeded_params(41, monotone)
    gpu = _gpu_u32(gpu_lib.learned_eval_lut(model, torch.from_numpy(p32).cuda(),
                                            mode="monotone" if monotone else "unconstrained"))
    p = p32.astype(np.float64)
    ref = _oracle_table(p, monotone, dense, cum, S)
    tol = _tolerance(p, monotone, S - int(cum[-1]), S)
    # the table is not flat: the network really is evaluated
    assert np.unique(ref).size > 1000
    bad = _compare(gpu, ref, tol, "seeded " + ("softplus" if monotone else "raw"))
    assert bad.size == 0, f"first entries over tolerance: {bad[:8].tolist()}"
    plants = PLANTS + (["identity_weights"] if monotone else [])
    K = PLANT_CELLS
    for plant in plants:
        wrong = _oracle_table(p, monotone, dense, cum, S, plant=plant, upto=K)
        caught = _compare(gpu[:K], wrong[:K], tol[:K], "planted " + plant).size
        assert caught > 0, f"a planted {plant} in the oracle was not seen"


def test_eval_lut_fixed_forms(gpu_lib):
    # equal-width and constant tables ignore the parameters
    import torch

    b = config5(n=200_000, seed=35)
    kw = dict(sample_frac=0.05, seed=3)
    model = _fit(gpu_lib, b, **kw)
    dense, cum, S = _oracle_dense(gpu_lib, b, model, kw["sample_frac"], kw["seed"])
    for mode, f in (("equal_width", lambda x: x), ("constant", lambda x: np.zeros_like(x))):
        gpu = _gpu_u32(gpu_lib.learned_eval_lut(model, mode=mode))
        ref = ol.cdf_table(f, dense, cum, S)
        assert np.abs(gpu - ref).max() <= 2, mode


def test_eval_lut_rejects_bad_arguments(gpu_lib):
    import torch

    b = config5(n=20_000, seed=36)
    model = _fit(gpu_lib, b, sample_frac=0.1)
    with pytest.raises(gpu_lib.HuskyError):
        gpu_lib.learned_eval_lut(model, mode=9)
    params = torch.zeros(ol.P, dtype=torch.float32, device="cuda")
    with pytest.raises(gpu_lib.HuskyError):  # model not 256-byte aligned
        gpu_lib.learned_eval_lut(model[1:], params, mode="equal_width")
