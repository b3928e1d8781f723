"""Pins for the float64 learned-CDF oracle: its chain-rule gradient against
central finite differences, and the monotonicity that positive (softplus)
weights and ReLU guarantee."""

import numpy as np

from oracle import learned


def _params(seed):
    rng = np.random.default_rng(seed)
    return rng.normal(0.0, 0.7, size=learned.P)


def test_parameter_count():
    assert learned.P == 64 + 64 + 64 * 64 + 64 + 64 + 1 == 4353


def test_gradient_matches_finite_differences():
    p = _params(1)
    rng = np.random.default_rng(2)
    x = rng.random(300)
    y = np.sort(rng.random(300))
    L, g = learned.grad(p, x, y)
    assert np.isclose(L, learned.loss(p, x, y))
    idx = list(range(0, 64, 7)) + list(range(64, 128, 9)) + list(range(128, 128 + 4096, 97)) + \
        list(range(4224, 4288, 11)) + list(range(4288, 4352, 13)) + [4352]
    # h = 1e-5 balances truncation against float64 roundoff in the loss
    num = learned.numeric_grad(p, x, y, idx, h=1e-5)
    np.testing.assert_allclose(g[idx], num, rtol=5e-5, atol=1e-7)


def test_planted_sign_error_is_caught():
    # a backward pass with a dropped softplus derivative disagrees with the
    # finite differences: the check above would catch that mistake
    p = _params(3)
    rng = np.random.default_rng(4)
    x, y = rng.random(200), rng.random(200)
    _, g = learned.grad(p, x, y)
    v1 = learned.split(p)[0]
    wrong = g[:64] / learned.sigmoid(v1)
    num = learned.numeric_grad(p, x, y, range(64))
    assert not np.allclose(wrong, num, rtol=1e-3)


def test_output_is_monotone_for_any_parameters():
    for seed in range(5):
        p = _params(10 + seed)
        x = np.linspace(0.0, 1.0, 20001)
        f = learned.forward(p, x)
        assert np.all(np.diff(f) >= -1e-12)


def test_unconstrained_gradient_matches_finite_differences():
    p = _params(5) * 0.3
    rng = np.random.default_rng(6)
    x = rng.random(200)
    y = np.sort(rng.random(200))
    _, g = learned.grad(p, x, y, monotone=False)
    idx = list(range(0, 64, 5)) + list(range(128, 128 + 4096, 131)) + list(range(4288, 4353, 8))
    num = learned.numeric_grad(p, x, y, idx, h=1e-5, monotone=False)
    np.testing.assert_allclose(g[idx], num, rtol=5e-5, atol=1e-7)


def test_unconstrained_network_can_decrease():
    # the raw-weight variant is a real fault injection: some parameters make it
    # decrease, which the LUT's running maximum must then absorb
    x = np.linspace(0.0, 1.0, 5001)
    assert any(np.any(np.diff(learned.forward(_params(20 + s), x, monotone=False)) < -1e-9)
               for s in range(5))


def test_splitmix64_reference_sequence():
    # SplitMix64 from state 0: its first three outputs (Steele, Lea, Flood 2014)
    g = learned._GOLDEN
    assert learned.splitmix64(0) == 0xE220A8397B1DCDAF
    assert learned.splitmix64(g) == 0x6E789E6AA1B965F4
    assert learned.splitmix64(2 * g % (1 << 64)) == 0x06C45D188009454F


def test_sample_indices_in_range_and_seeded():
    a = learned.sample_indices(1000, 300, seed=7)
    assert a.min() >= 0 and a.max() < 1000
    np.testing.assert_array_equal(a, learned.sample_indices(1000, 300, seed=7))
    assert not np.array_equal(a, learned.sample_indices(1000, 300, seed=8))
    # roughly uniform: every tenth of the range gets its share
    h = np.bincount(learned.sample_indices(1000, 20000, seed=1) // 100, minlength=10)
    assert h.min() > 1700 and h.max() < 2300


def test_cell_is_the_window_below_the_common_prefix():
    lo, hi = 0x1234_0000_0000_0000, 0x1237_FFFF_FFFF_FFFF
    assert learned.header(np.array([lo, hi], dtype=np.uint64).astype(object)) == (lo, hi, 14)
    # bits 49..26 of the code (24 bits below the 14 shared ones)
    c = 0x1235_6789_ABCD_EF01
    assert learned.cell(c, lo, hi, 14) == (c >> 26) & 0xFFFFFF
    # clamping, and monotone in the code
    assert learned.cell(0, lo, hi, 14) == learned.cell(lo, lo, hi, 14)
    assert learned.cell(1 << 63, lo, hi, 14) == learned.cell(hi, lo, hi, 14) == 0xFFFFFF
    rng = np.random.default_rng(1)
    codes = np.sort(rng.integers(lo, hi, size=2000, dtype=np.uint64))
    cells = [learned.cell(int(v), lo, hi, 14) for v in codes]
    assert all(a <= b for a, b in zip(cells, cells[1:]))
    assert learned.cell(5, 5, 5, 64) == 0


def test_dense_cells_brute_force():
    # B = 8 buckets, S = 16 keys: dense when a cell holds >= 4 sample keys
    lo = 0
    hi = (1 << 63) - 1  # cp = 1: the cell is bits 62..39
    cells = [3, 3, 3, 3, 3, 3, 9, 9, 12, 12, 12, 12, 20, 21, 22, 0xFFFFFF]
    sample = np.array(sorted(c << 39 for c in cells), dtype=object)
    sample[0] = lo
    sample[-1] = hi
    dense, cum, flag = learned.dense_cells(sample, B=8, min_count=1)
    w = [learned.cell(int(c), lo, hi, 1) for c in sample]
    counts = {c: w.count(c) for c in set(w)}
    expect = sorted(c for c, k in counts.items() if k * 8 >= 2 * 16)
    assert list(dense) == expect == [3, 12]
    assert list(cum) == [0, counts[3], counts[3] + counts[12]]
    assert int(flag.sum()) == cum[-1]
    # the floor on the count: cell 3 keeps 5 keys (the first became lo), cell
    # 12 has 4, so only cell 3 is dense with min_count 5
    dense5, cum5, _ = learned.dense_cells(sample, B=8, min_count=5)
    assert list(dense5) == [3] and list(cum5) == [0, counts[3]]


def test_cdf_table_closed_forms():
    W = np.array([0, 1, 1 << 23, (1 << 24) - 1, 1 << 24])
    # no dense cells, f(x) = x: q(W) = floor(W / 2^24 * (2^32 - 1))
    q = learned.cdf_table(lambda x: x, np.zeros(0, dtype=np.int64), np.array([0]), 100)
    assert q[0] == 0 and q[-1] == 2**32 - 1
    for w in W[1:-1]:
        assert q[w] == int(np.floor(w / 2**24 * 4294967295.0))
    assert np.all(np.diff(q) >= 0)
    # every sample key dense (f is irrelevant): a step at each dense cell
    dense = np.array([5, 100])
    cum = np.array([0, 30, 100])
    q2 = learned.cdf_table(lambda x: np.sin(40 * x), dense, cum, 100)
    assert q2[5] == 0 and q2[6] == int(np.floor(0.3 * 4294967295.0)) and q2[100] == q2[6]
    assert q2[101] == 2**32 - 1
    # a decreasing f still gives a non-decreasing table (running maximum)
    q3 = learned.cdf_table(lambda x: 1.0 - x, np.zeros(0, dtype=np.int64), np.array([0]), 10)
    assert np.all(np.diff(q3) >= 0)


def test_splitters_brute_force():
    # B = 8: cells 0 and 1 own no bucket, cell 2 owns [1, 5) and holds 6
    # sample keys, cell 3 onwards owns [5, 7)
    lut = np.zeros(learned.CELLS + 1, dtype=np.int64)
    B = 8
    step = (1 << 32) // B
    lut[3:] = 5 * step
    lut[2] = 1 * step
    lut[-1] = 2**32 - 1
    lo, hi = 0, (1 << 63) - 1
    keys = sorted([(2 << 39) + k for k in (7, 3, 9, 1, 4, 8)] + [(1 << 39), (5 << 39)])
    sample = np.array(keys, dtype=object)
    sample[0], sample[-1] = lo, hi
    out = learned.splitters(lut, sample, B=B)
    in_cell = sorted(k for k in keys if k >> 39 == 2)
    # cell 2 owns [1, 5): k = 4 buckets, m = 6 keys, splitters at ranks 6i // 4
    assert {s: out[s] for s in range(1, 4)} == {1 + i - 1: in_cell[(6 * i) // 4] for i in range(1, 4)}


def test_subtable_brute_force():
    # one heavy cell (cell 2) owning buckets [1, 5) of B = 8: three splitters
    # sharing their top 44 bits, then sub-cells of the next s bits
    B = 8
    step = (1 << 32) // B
    lut = np.zeros(learned.CELLS + 1, dtype=np.int64)
    lut[2] = step
    lut[3:] = 5 * step
    lut[-1] = 2**32 - 1
    base = 2 << 39
    spl_vals = [base | (0b000 << 17) | 5, base | (0b011 << 17) | 9, base | (0b101 << 17) | 1]
    spl = {1 + i: v for i, v in enumerate(spl_vals)}
    b0, P, s, prefix, table = learned.subtable(lut, spl, 2, B=B)
    assert b0 == 1 and P == 44 and s == 5 and prefix == base  # k = 4: ceil(log2 4) + 3
    # splitters strictly below the first code of sub-cell v (bits 19..15)
    brute = [sum(1 for x in spl_vals if x < (base | (v << 15))) for v in range(32)]
    assert table == brute
    assert table[:4] == [0, 1, 1, 1] and table[12] == 1 and table[13] == 2 and table[21] == 3
    # all splitters equal: P = 64, no sub-cells
    same = {1: base | 7, 2: base | 7, 3: base | 7}
    assert learned.subtable(lut, same, 2, B=B)[1:4] == (64, 0, base | 7)


def test_bucket_ids_brute_force():
    # B = 8; cells 0-1 own nothing, cell 2 owns [1, 5) with splitters, cell 3
    # onwards own [5, 7) but cell 3 alone starts there (one bucket each side)
    B = 8
    step = (1 << 32) // B
    lut = np.zeros(learned.CELLS + 1, dtype=np.int64)
    lut[2] = step
    lut[3] = 5 * step
    lut[4:] = 6 * step
    lut[-1] = 2**32 - 1
    lo, hi, cp = 0, (1 << 63) - 1, 1  # cells are bits 62..39
    base = 2 << 39
    spl = np.zeros(B, dtype=np.uint64)
    spl[1:4] = [base | 100, base | 200, base | 200]
    codes = np.array([0, 1 << 39, base, base | 100, base | 150, base | 200, base | 201,
                      3 << 39, 4 << 39, hi], dtype=np.uint64)
    got = learned.bucket_ids(codes, lut, spl, lo, hi, cp, B=B)

    def brute(c):
        W = (int(c) >> 39) & 0xFFFFFF
        b0, b1 = (lut[W] * B) >> 32, (lut[W + 1] * B) >> 32
        if b1 - b0 < 2:
            return b0
        return b0 + sum(1 for j in range(b1 - b0 - 1) if int(spl[b0 + j]) <= int(c))

    assert [int(g) for g in got] == [brute(c) for c in codes] == [0, 0, 1, 2, 2, 4, 4, 5, 6, 6]
    # monotone in the code
    assert np.all(np.diff(got) >= 0)
