"""GPU parity: every HIP result against the CPU oracle, element by element.

Bit-exact comparisons throughout (codes, sorted pairs, permutations).  Sizes
run from a few strings to several radix tiles with ragged tails; the full
workload sizes are covered by tests/test_gpu_sizes_full.py.
"""

import sys

import numpy as np
import pytest

import oracle
from workloads import (ADVERSARIAL_FAMILIES, adversarial, config1, config2, config3, config4,
                       config5, from_strings)

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[case]", *a, file=sys.stderr, flush=True)


def _u64(t):
    return t.cpu().numpy().view(np.uint64)


def _u32(t):
    return t.cpu().numpy().view(np.uint32)


def _sort_gpu(husky, batch, tuning=None):
    e, o = husky.to_device(batch)
    return _u32(husky.sort(e, o, batch.coder, tuning=tuning))


@pytest.mark.parametrize("family", ADVERSARIAL_FAMILIES)
def test_encode_adversarial(gpu_lib, family):
    b = adversarial(family, seed=21, n=3000)
    _say("encode", family)
    e, o = gpu_lib.to_device(b)
    codes, idx = gpu_lib.encode(e, o, b.coder)
    ref, _ = oracle.encode(b)
    np.testing.assert_array_equal(_u64(codes), ref)
    np.testing.assert_array_equal(_u32(idx), np.arange(b.n, dtype=np.uint32))


@pytest.mark.parametrize("maker", [config1, config2, config3, lambda n: config5(n=n)],
                         ids=["c1", "c2", "c3", "c5"])
def test_encode_configs(gpu_lib, maker):
    b = maker(n=200_003)
    _say("encode config", b.name)
    e, o = gpu_lib.to_device(b)
    codes, _ = gpu_lib.encode(e, o, b.coder)
    np.testing.assert_array_equal(_u64(codes), oracle.encode(b)[0])


def test_encode_domain_status(gpu_lib):
    import torch

    b = from_strings([b"abc", b"\x80", b"abcdefgh\xff", b"abcdefghi\xff", b"a\xc3\xa9", b""])
    e, o = gpu_lib.to_device(b)
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    gpu_lib.encode(e, o, "ascii7", status=st)
    assert int(st.item()) == 3


@pytest.mark.parametrize("n", [1, 2, 63, 1000, 4096, 4097, 50_000, 300_001])
@pytest.mark.parametrize("bits", [(0, 64), (0, 63), (5, 37)])
def test_sort_pairs_random(gpu_lib, n, bits):
    import torch

    _say("sort_pairs", n, bits)
    rng = np.random.default_rng(n * 7 + bits[0])
    keys = rng.integers(0, 2**63, size=n, dtype=np.uint64) * np.uint64(2) + rng.integers(0, 2, size=n, dtype=np.uint64)
    # heavy ties: many keys share a few values
    keys[rng.random(n) < 0.3] = np.uint64(12345)
    vals = rng.permutation(n).astype(np.uint32)
    k = torch.from_numpy(keys.view(np.int64)).cuda()
    v = torch.from_numpy(vals.view(np.int32)).cuda()
    gpu_lib.sort_pairs(k, v, bits[0], bits[1])
    lo, hi = bits
    mask = ((1 << (hi - lo)) - 1) << lo
    field = (keys & np.uint64(mask)) >> np.uint64(lo)
    order = np.argsort(field, kind="stable")
    np.testing.assert_array_equal(_u32(v), vals[order])
    np.testing.assert_array_equal(_u64(k), keys[order])


@pytest.mark.parametrize("family", ADVERSARIAL_FAMILIES)
def test_sort_adversarial(gpu_lib, family):
    b = adversarial(family, seed=5, n=5000)
    _say("sort", family)
    ref, bad = oracle.sort(b)
    assert bad == 0
    np.testing.assert_array_equal(_sort_gpu(gpu_lib, b), ref)


def test_sort_config1_full(gpu_lib):
    b = config1()
    _say("sort config1", b.n)
    np.testing.assert_array_equal(_sort_gpu(gpu_lib, b), oracle.sort(b)[0])


@pytest.mark.parametrize("n", [10_007, 300_001])
def test_sort_config2_3_5(gpu_lib, n):
    for b in (config2(n=n), config3(n=n), config5(n=n)):
        _say("sort", b.name)
        np.testing.assert_array_equal(_sort_gpu(gpu_lib, b), oracle.sort(b)[0])


@pytest.mark.parametrize("tuning", [dict(radix_bits=6, tile_items=8, t_small=2, t_medium=64),
                                    dict(radix_bits=7, tile_items=12, t_small=16, t_medium=256),
                                    dict(radix_bits=8, tile_items=16, t_small=64, t_medium=4096),
                                    dict(radix_bits=8, tile_items=8, t_small=4, t_medium=1024)],
                         ids=["b6i8", "b7i12", "b8i16", "b8i8"])
def test_sort_threshold_stress(gpu_lib, tuning):
    t = gpu_lib.make_tuning(**tuning)
    for b in (adversarial("identical", n=20000), adversarial("prefix12", n=20000),
              adversarial("nul", n=20000), config2(n=200_000), adversarial("utf16_prefix4", n=20000)):
        _say("stress", tuning, b.name)
        np.testing.assert_array_equal(_sort_gpu(gpu_lib, b, t), oracle.sort(b)[0])


@pytest.mark.parametrize("kind", ["long_copies", "short_copies", "same_prefix"])
def test_sort_one_code_over_several_tiles(gpu_lib, kind):
    # every code equal and more strings than one radix tile: no digit pass
    # runs, so the indices leave the code sort as the encode kernel wrote them
    # (for one instance it puts each code's low byte in the index's top byte
    # for the first pass's count, which must not reach the permutation)
    rng = np.random.default_rng(31)
    if kind == "long_copies":
        strs = [b"abcdefghijklmnop"] * 9000
    elif kind == "short_copies":
        strs = [b"abcdefg"] * 9000
    else:
        strs = [b"abcdefghi" + bytes(rng.integers(97, 123, size=5, dtype=np.uint8).tolist()) for _ in range(9000)]
    b = from_strings(strs)
    _say("one code", kind, b.n)
    np.testing.assert_array_equal(_sort_gpu(gpu_lib, b), oracle.sort(b)[0])


@pytest.mark.parametrize("items", [8, 12, 16])
def test_sort_tile_edges(gpu_lib, items):
    # the encode kernel reduces each radix tile's OR / AND itself (one
    # workgroup per tile): sizes at, just under and just over one, two and
    # three tiles of every compiled tile size, each checked against the oracle
    tile = 256 * items
    t = gpu_lib.make_tuning(tile_items=items)
    for n in (tile - 1, tile, tile + 1, 2 * tile - 1, 2 * tile + 1, 3 * tile + 7):
        b = config2(n=n, seed=n)
        _say("tile edges", items, n)
        np.testing.assert_array_equal(_sort_gpu(gpu_lib, b, t), oracle.sort(b)[0])


def test_sort_empty_and_tiny(gpu_lib):
    for strs in ([b""], [b"b", b"a"], [b"", b""], [b"x"] * 3, [b"ab\0", b"ab", b"ab"]):
        b = from_strings(strs)
        _say("tiny", strs)
        np.testing.assert_array_equal(_sort_gpu(gpu_lib, b), oracle.sort(b)[0])


def test_fixup_entry_point(gpu_lib):
    import torch

    b = config2(n=100_000)
    _say("fixup", b.name)
    codes, _ = oracle.encode(b)
    c, i = oracle.sort_pairs(codes, np.arange(b.n, dtype=np.uint32))
    e, o = gpu_lib.to_device(b)
    ct = torch.from_numpy(c.view(np.int64)).cuda()
    it = torch.from_numpy(i.view(np.int32)).cuda()
    gpu_lib.fixup(e, o, ct, it, "ascii7")
    np.testing.assert_array_equal(_u32(it), oracle.fixup(b, c, i))


def test_batched_small(gpu_lib):
    import torch

    b = config4(n_inst=40, lo=1, hi=20000)
    _say("batched", b.name, b.n)
    e, o = gpu_lib.to_device(b)
    seg = torch.from_numpy(b.seg_offsets.view(np.int64)).cuda()
    perm = _u32(gpu_lib.sort_batched(e, o, seg, "ascii7"))
    np.testing.assert_array_equal(perm, oracle.sort_batched(b)[0])


def test_domain_violation_raises(gpu_lib):
    b = from_strings([b"abc", b"\x80abc"])
    e, o = gpu_lib.to_device(b)
    with pytest.raises(gpu_lib.DomainError):
        gpu_lib.sort(e, o, "ascii7")


def _perfect_bit_batch(n, seed, short_only_group):
    """Strings c0 + "bbbb" + c5 [+ NUL NUL NUL + 1..5 letters]: codes vary in
    exactly eight bits (c0 in {a, c}: one bit; c5 in 0x01..0x7F: seven), and
    the perfect bit varies too, so with it the code sort needs two 8-bit
    passes and without it one.  With short_only_group the c0 = 'c' strings
    are all six bytes long: their runs hold identical strings only."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        c0 = b"a" if rng.random() < 0.5 else b"c"
        s = c0 + b"bbbb" + bytes([int(rng.integers(1, 128))])
        if not (short_only_group and c0 == b"c") and rng.random() < 0.6:
            s += b"\0\0\0" + bytes(rng.integers(97, 123, size=int(rng.integers(1, 6)), dtype=np.uint8))
        out.append(s)
    return from_strings(out, "ascii7", name=f"perfect_bit(n={n},seed={seed})")


@pytest.mark.parametrize("short_only_group", [False, True])
def test_sort_perfect_bit_left_out(gpu_lib, short_only_group):
    # the perfect bit would cost a digit pass here, so the code sort leaves it
    # out and run detection compares codes without it: every run of equal
    # codes is listed (those of identical short strings too), and the
    # permutation is the oracle's
    b = _perfect_bit_batch(20_000, 77, short_only_group)
    _say("sort perfect bit left out", b.name)
    e, o = gpu_lib.to_device(b)
    ws = gpu_lib.alloc_workspace(b.n, 1, o.device)
    perm = _u32(gpu_lib.sort(e, o, b.coder, ws=ws))
    ref, bad = oracle.sort(b)
    assert bad == 0
    np.testing.assert_array_equal(perm, ref)
    codes = oracle.encode(b)[0]
    _, counts = np.unique(codes, return_counts=True)
    assert gpu_lib.read_status(ws)["runs_fixed"] == int((counts >= 2).sum())


def test_sort_perfect_bit_kept(gpu_lib):
    # config-1 strings: the perfect bit costs no pass (codes vary in 61 bits),
    # so runs of identical strings of at most nine bytes are never listed
    b = config1(seed=9, n=30_000)
    _say("sort perfect bit kept", b.name)
    e, o = gpu_lib.to_device(b)
    ws = gpu_lib.alloc_workspace(b.n, 1, o.device)
    perm = _u32(gpu_lib.sort(e, o, b.coder, ws=ws))
    ref, bad = oracle.sort(b)
    assert bad == 0
    np.testing.assert_array_equal(perm, ref)
    lens = np.diff(b.offsets)
    codes = oracle.encode(b)[0].astype(np.uint64)
    keys = (codes << np.uint64(1)) | (lens > 9).astype(np.uint64)  # no NULs in config 1
    uk, counts = np.unique(keys, return_counts=True)
    flagged = (uk & np.uint64(1)) == 1
    assert gpu_lib.read_status(ws)["runs_fixed"] == int(((counts >= 2) & flagged).sum())
