"""GPU: the learned-CDF form.

* the training kernel's gradient (FP32) against the float64 oracle's chain
  rule, for the monotone and the raw-weight network, on ragged batch sizes
  that span one and many workgroups;
* the fit's deterministic parts against the oracle's definitions: sample
  extremes and common prefix, dense cells and their counts, the CDF table
  (equal-width mode, within two units of 2^-32) and the splitters;
* the LUT is non-decreasing over all 2^24 + 1 entries, whatever the network;
* husky_sort_learned's permutation equals the oracle's on every workload
  shape, with the trained network, with deliberately broken models
  (unconstrained, constant) and with a model fitted on other data.
"""

import math

import numpy as np
import pytest

import oracle
from oracle import learned as ol
from _progress import say
from workloads import ADVERSARIAL_FAMILIES, adversarial, config1, config2, config3, config5

pytestmark = pytest.mark.gpu


def _u32(t):
    return t.cpu().numpy().view(np.uint32)


def _params(seed):
    rng = np.random.default_rng(seed)
    p = np.empty(ol.P)
    p[0:64] = rng.normal(0.54, 0.4, 64)
    p[64:128] = -(np.arange(64) + 0.5) / 64 + rng.normal(0, 0.02, 64)
    p[128:128 + 4096] = rng.normal(-4.15, 0.4, 4096)
    p[4224:4288] = rng.normal(0.0, 0.05, 64)
    p[4288:4352] = rng.normal(-3.45, 0.4, 64)
    p[4352] = 0.05
    return p.astype(np.float32)


@pytest.mark.parametrize("monotone", [True, False], ids=["softplus", "raw"])
@pytest.mark.parametrize("count", [1, 300, 1000, 70_001])
def test_mlp_grad_matches_oracle(gpu_lib, monotone, count):
    import torch

    p = _params(count)
    if not monotone:
        p = (p * 0.2).astype(np.float32)  # keep the raw network's outputs moderate
    rng = np.random.default_rng(count + 7)
    x = rng.random(count).astype(np.float32)
    y = np.sort(rng.random(count)).astype(np.float32)
    g, sse = gpu_lib.mlp_grad(torch.from_numpy(p).cuda(), torch.from_numpy(x).cuda(),
                              torch.from_numpy(y).cuda(), monotone=monotone)
    g = g.cpu().numpy().astype(np.float64)
    L, ref = ol.grad(p.astype(np.float64), x.astype(np.float64), y.astype(np.float64), monotone)
    assert math.isclose(float(sse) / count, L, rel_tol=1e-4, abs_tol=1e-9)
    scale = np.abs(ref).max()
    assert np.linalg.norm(g - ref) <= 1e-4 * np.linalg.norm(ref) + 1e-7
    np.testing.assert_allclose(g, ref, rtol=1e-3, atol=1e-5 * scale)


def _fit(gpu_lib, b, e, o, **kw):
    params = gpu_lib.make_learned_params(**kw)
    ws = gpu_lib.alloc_learned_workspace(b.n)
    model = gpu_lib.fit_learned(e, o, b.coder, params, ws=ws)
    return model, ws


def test_fit_matches_definitions(gpu_lib):
    import torch

    b = config5(n=300_000, seed=3)
    e, o = gpu_lib.to_device(b)
    frac, seed = 0.05, 11
    model, _ = _fit(gpu_lib, b, e, o, sample_frac=frac, seed=seed, mode="equal_width")
    h = gpu_lib.learned_header(model)
    S = math.ceil(frac * b.n)
    codes, _ = oracle.encode(b)
    sample = np.sort(codes[ol.sample_indices(b.n, S, seed)]).astype(object)
    lo, hi, cp = ol.header(sample)
    assert (h["lo"], h["hi"], h["cp"], h["sample"], h["buckets"]) == (lo, hi, cp, S, 65536)
    dense, cum, _ = ol.dense_cells(sample)
    assert h["dense"] == len(dense) and h["dense_keys"] == cum[-1]
    assert h["steps"] == 0 and h["trained"] == 0
    got_dense = gpu_lib.learned_part(model, "dense", torch.int32, len(dense)).cpu().numpy()
    got_cum = gpu_lib.learned_part(model, "dense_cum", torch.int32, len(dense) + 1).cpu().numpy()
    np.testing.assert_array_equal(got_dense.view(np.uint32), dense)
    np.testing.assert_array_equal(got_cum.view(np.uint32), cum)
    say("dense cells", len(dense), "holding", cum[-1], "of", S)
    lut = gpu_lib.learned_part(model, "lut", torch.int32, ol.CELLS + 1).cpu().numpy()
    lut = lut.view(np.uint32).astype(np.int64)
    ref = ol.cdf_table(lambda x: x, dense, cum, S)
    assert np.abs(lut - ref).max() <= 2
    # splitters from the GPU's own table, by the oracle's definition
    spl = gpu_lib.learned_part(model, "splitters", torch.int64, 65536).cpu().numpy().view(np.uint64)
    want = ol.splitters(lut, sample)
    assert h["heavy"] == int(np.sum(((lut[1:] * 65536) >> 32) - ((lut[:-1] * 65536) >> 32) >= 2))
    for slot, v in want.items():
        assert int(spl[slot]) == v, slot
    # sub-cell tables of the heavy cells: the widest ones and a spread of others
    b = (lut * 65536) >> 32
    owned = b[1:] - b[:-1]
    heavy = np.nonzero(owned >= 2)[0]
    pick = list(heavy[np.argsort(-owned[heavy])[:5]]) + list(heavy[:: max(1, len(heavy) // 30)])
    sub = gpu_lib.learned_part(model, "subtab", torch.int16, 16 * 65536).cpu().numpy().view(np.uint16)
    info = gpu_lib.learned_part(model, "cellinfo", torch.int64, ol.CELLS).cpu().numpy().view(np.uint64)
    np.testing.assert_array_equal(info & np.uint64(0xFFFF), b[:-1])
    np.testing.assert_array_equal((info >> np.uint64(16)) & np.uint64(0xFFFF), b[1:])
    for W in sorted(set(int(w) for w in pick)):
        b0, P, sbits, prefix, table = ol.subtable(lut, want, W)
        hd = sub[16 * b0:16 * b0 + 8].astype(np.uint64)
        assert (int(hd[0]), int(hd[1])) == (P, sbits)
        assert int(hd[4] | (hd[5] << 16) | (hd[6] << 32) | (hd[7] << 48)) == prefix
        np.testing.assert_array_equal(sub[16 * b0 + 8:16 * b0 + 8 + (1 << sbits)], table)
        ci = int(info[W])
        e = P - (cp + 24)
        if ci >> 63 == 0:  # the prefix bits below the cell are kept in the cell's entry
            assert e <= 19 and ((ci >> 32) & 127, (ci >> 39) & 31) == (P, sbits)
            below = (((prefix << (cp + 24)) & ((1 << 64) - 1)) >> (64 - e)) if e else 0
            assert (ci >> 44) & 0x7FFFF == below
        else:
            assert e > 19 or P == 64


@pytest.mark.parametrize("mode", ["monotone", "unconstrained"])
def test_lut_non_decreasing_everywhere(gpu_lib, mode):
    import torch

    b = config5(n=200_000, seed=4)
    e, o = gpu_lib.to_device(b)
    model, _ = _fit(gpu_lib, b, e, o, mode=mode, sample_frac=0.05, epochs=3, lr=0.05)
    lut = gpu_lib.learned_part(model, "lut", torch.int32, ol.CELLS + 1).to(torch.int64) & 0xFFFFFFFF
    assert int(lut[0]) == 0 and int(lut[-1]) == 2**32 - 1
    assert bool((lut[1:] >= lut[:-1]).all())
    h = gpu_lib.learned_header(model)
    assert h["steps"] > 0 and h["trained"] == h["sample"] - h["dense_keys"]
    if mode == "monotone":
        assert np.isfinite(h["last_loss"]) and h["last_loss"] < 0.05


def _learned_equals_oracle(gpu_lib, b, **kw):
    e, o = gpu_lib.to_device(b)
    model, ws = _fit(gpu_lib, b, e, o, **kw)
    perm = _u32(gpu_lib.sort_learned(e, o, model, b.coder, ws=ws))
    st = gpu_lib.read_status(ws)
    ref, bad = oracle.sort(b)
    assert bad == 0
    np.testing.assert_array_equal(perm, ref)
    return st


@pytest.mark.parametrize("maker", [lambda: config1(n=100_000), lambda: config2(n=300_000),
                                   lambda: config3(n=200_000), lambda: config5(n=400_000)],
                         ids=["config1", "config2", "config3_utf16", "config5"])
def test_learned_sort_exact(gpu_lib, maker):
    b = maker()
    st = _learned_equals_oracle(gpu_lib, b)
    say(b.name, "overflow buckets", st["overflow_buckets"], "keys", st["overflow_keys"])


@pytest.mark.parametrize("family", ADVERSARIAL_FAMILIES)
def test_learned_sort_adversarial(gpu_lib, family):
    b = adversarial(family, n=3000)
    if b.n == 0:
        pytest.skip("the fit needs at least one string")
    _learned_equals_oracle(gpu_lib, b, sample_frac=0.1)


@pytest.mark.parametrize("mode,dense", [("unconstrained", True), ("constant", True),
                                        ("constant", False), ("untrained", True),
                                        ("equal_width", True)])
def test_broken_or_weak_models_stay_exact(gpu_lib, mode, dense):
    b = config5(n=250_000, seed=6)
    st = _learned_equals_oracle(gpu_lib, b, mode=mode, dense=dense, sample_frac=0.02)
    if mode == "constant" and not dense:
        # every key outside the top cell lands in bucket 0: one giant overflow
        assert st["overflow_keys"] > b.n // 2


def test_single_level_form_exact(gpu_lib):
    # the network alone, no dense cells
    _learned_equals_oracle(gpu_lib, config5(n=250_000, seed=7), dense=False)


def test_model_from_other_data(gpu_lib):
    # codes outside the fitted [lo, hi] clamp to the extreme cells
    fit_on = config5(n=100_000, seed=8)
    e1, o1 = gpu_lib.to_device(fit_on)
    model, _ = _fit(gpu_lib, fit_on, e1, o1)
    b = config2(n=200_000, seed=9)
    e, o = gpu_lib.to_device(b)
    perm = _u32(gpu_lib.sort_learned(e, o, model, "ascii7"))
    np.testing.assert_array_equal(perm, oracle.sort(b)[0])


def test_tiny_and_empty_inputs(gpu_lib):
    import torch

    b = config1(n=1, seed=2)
    e, o = gpu_lib.to_device(b)
    model, _ = _fit(gpu_lib, b, e, o)
    assert _u32(gpu_lib.sort_learned(e, o, model)).tolist() == [0]
    empty_off = torch.zeros(1, dtype=torch.int64, device="cuda")
    assert gpu_lib.sort_learned(e, empty_off, model).numel() == 0
    for n in (2, 3, 17, 4097):
        bb = config2(n=n, seed=n)
        ee, oo = gpu_lib.to_device(bb)
        m2, _ = _fit(gpu_lib, bb, ee, oo, sample_frac=1.0)
        np.testing.assert_array_equal(_u32(gpu_lib.sort_learned(ee, oo, m2)), oracle.sort(bb)[0])


def test_fit_rejects_bad_arguments(gpu_lib):
    b = config1(n=100)
    e, o = gpu_lib.to_device(b)
    for kw in (dict(sample_frac=1.5), dict(sample_frac=-0.1), dict(mode=9)):
        with pytest.raises(gpu_lib.HuskyError):
            _fit(gpu_lib, b, e, o, **kw)


def _model_tables(gpu_lib, model):
    import torch

    h = gpu_lib.learned_header(model)
    lut = gpu_lib.learned_part(model, "lut", torch.int32, ol.CELLS + 1).cpu().numpy()
    spl = gpu_lib.learned_part(model, "splitters", torch.int64, 65536).cpu().numpy().view(np.uint64)
    return h, lut.view(np.uint32).astype(np.int64), spl


@pytest.mark.parametrize("maker,kw", [
    (lambda: config5(n=300_000, seed=12), {}),
    (lambda: config5(n=300_000, seed=13), {"dense": False}),
    (lambda: config3(n=200_000, seed=14), {}),
    (lambda: adversarial("mixed", n=20_000), {"sample_frac": 0.1}),
    (lambda: adversarial("utf16_prefix4", n=20_000), {"sample_frac": 0.1}),
], ids=["config5", "config5_network_alone", "config3_utf16", "mixed", "utf16_prefix4"])
def test_bucket_ids_match_definition(gpu_lib, maker, kw):
    # the sort's per-key bucket function (cell info, sub-cell tables, splitter
    # search) equals the definition evaluated on the model's LUT and splitters
    b = maker()
    e, o = gpu_lib.to_device(b)
    model, _ = _fit(gpu_lib, b, e, o, **kw)
    got = gpu_lib.learned_buckets(e, o, model, b.coder).cpu().numpy().view(np.uint16)
    h, lut, spl = _model_tables(gpu_lib, model)
    codes, _ = oracle.encode(b)
    want = ol.bucket_ids(codes, lut, spl, h["lo"], h["hi"], h["cp"])
    np.testing.assert_array_equal(got.astype(np.int64), want)


def _expected_load(ids):
    # the size of the bucket a random key lands in: sum of load^2 / n
    load = np.bincount(ids.astype(np.int64), minlength=65536).astype(np.float64)
    return float((load * load).sum() / load.sum())


def test_trained_network_balances_buckets(gpu_lib):
    # UTF-16 CJK strings: no cell is dense, so the network alone shapes the
    # buckets; the first code unit only spans U+4E00..U+9FA5, about a third of
    # the cell range, which equal-width cells spread over a third of the
    # buckets (expected load ~3x the ideal n / B).  The trained network must
    # do clearly better than both the equal-width baseline and its own
    # untrained start.  (It cannot reach the ideal: inside each first unit the
    # second unit again fills only a third of the cells, a staircase finer
    # than the network's knots; measured 2.1x ideal against 3.2x and 3.7x.)
    b = config3(n=4_000_000, seed=15)
    e, o = gpu_lib.to_device(b)
    loads = {}
    for mode in ("monotone", "equal_width", "untrained"):
        model, ws = _fit(gpu_lib, b, e, o, mode=mode)
        ids = gpu_lib.learned_buckets(e, o, model, b.coder).cpu().numpy().view(np.uint16)
        loads[mode] = _expected_load(ids)
        perm = _u32(gpu_lib.sort_learned(e, o, model, b.coder, ws=ws))
        assert gpu_lib.check_perm(e, o, torch_from(perm), b.coder) == 0
    ideal = b.n / 65536
    say("expected bucket load (ideal %.1f):" % ideal, {k: round(v, 1) for k, v in loads.items()})
    assert loads["monotone"] < 0.75 * loads["equal_width"]
    assert loads["monotone"] < 0.7 * loads["untrained"]
    assert loads["monotone"] < 2.5 * ideal


def torch_from(a):
    import torch

    return torch.from_numpy(np.ascontiguousarray(a).view(np.int32)).cuda()


@pytest.mark.parametrize("coder", ["ascii7", "utf16"])
def test_learned_long_shared_prefixes(gpu_lib, coder):
    # groups that stay tied after the code and the first refinement key (the
    # first 16 bytes / 7 units agree) inside buckets sorted in LDS, plus
    # identical strings and strings ending inside the shared part: the later
    # refinement rounds must run on exactly those groups
    from workloads import from_strings

    rng = np.random.default_rng(21 if coder == "ascii7" else 22)
    n = 60_000
    if coder == "ascii7":
        prefixes = [bytes(rng.integers(97, 123, size=24, dtype=np.uint8)) for _ in range(40)]
        out = []
        for _ in range(n):
            p = prefixes[int(rng.integers(0, 40))]
            cut = int(rng.integers(5, 25))  # sometimes ends inside the prefix
            out.append(p[:cut] + bytes(rng.integers(97, 100, size=int(rng.integers(0, 4)), dtype=np.uint8)))
    else:
        prefixes = [rng.integers(0x4E00, 0x4E10, size=12).tolist() for _ in range(40)]
        out = []
        for _ in range(n):
            p = prefixes[int(rng.integers(0, 40))]
            cut = int(rng.integers(2, 13))
            out.append(p[:cut] + rng.integers(0x4E00, 0x4E03, size=int(rng.integers(0, 3))).tolist())
    b = from_strings(out, coder)
    st = _learned_equals_oracle(gpu_lib, b, sample_frac=0.05)
    say(coder, "shared prefixes: runs visited", st["runs_fixed"], "rounds", st["large_rounds"])


def test_learned_sort_graph_capture_replay(gpu_lib):
    # with a fixed round count the learned sort never synchronizes, so it can
    # be captured into a HIP graph; every replay must give the eager result
    import torch

    b = config5(n=300_000, seed=23)
    e, o = gpu_lib.to_device(b)
    model, ws = _fit(gpu_lib, b, e, o, sample_frac=0.05)
    max_len = int(np.diff(b.offsets).max())
    t = gpu_lib.make_tuning(max_rounds=gpu_lib.rounds_for(max_len))
    perm = torch.empty(b.n, dtype=torch.int32, device="cuda")
    eager = _u32(gpu_lib.sort_learned(e, o, model, "ascii7", tuning=t, ws=ws, perm=perm)).copy()
    np.testing.assert_array_equal(eager, oracle.sort(b)[0])
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):  # warm-up on the capture stream
        gpu_lib.sort_learned(e, o, model, "ascii7", tuning=t, ws=ws, perm=perm, check_status=False)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        gpu_lib.sort_learned(e, o, model, "ascii7", tuning=t, ws=ws, perm=perm, check_status=False)
    for rep in range(3):
        perm.fill_(-1)  # eager work between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        np.testing.assert_array_equal(_u32(perm), eager, err_msg=f"replay {rep}")
        assert gpu_lib.read_status(ws)["unresolved"] == 0
