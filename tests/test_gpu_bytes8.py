"""GPU: the full-byte coder (HUSKY_CODER_BYTES8: the first eight bytes, big-endian,
every byte value in order) and the general refinement step (husky_refine).

* encode: bit-exact against the oracle's coder on every byte family and UTF-8;
* plain, batched and learned sorts: the permutation equals the oracle's on
  the byte families (values either side of 0x80, NULs against the padding,
  shared 8-byte prefixes) and on UTF-8 text of several scripts, at sizes that
  span many tiles and every fix-up tier, with a ragged tail;
* husky_refine: runs of equal keys of any origin -- husky codes (shared 8),
  coarser keys (the first one or two elements), keys that say nothing
  (shared 0: all strings one run, or random keys) -- re-sorted to exactly the
  oracle's Step 3 on the same keys, for bytes and UTF-16 units.
"""

import numpy as np
import pytest

import oracle
from _progress import say
from workloads import (BYTES_FAMILIES, adversarial, adversarial_bytes, config2, config3,
                       from_strings, utf8_words)

pytestmark = pytest.mark.gpu


def _u32(t):
    return t.cpu().numpy().view(np.uint32)


@pytest.mark.parametrize("family", BYTES_FAMILIES)
def test_bytes8_encode_matches_oracle(gpu_lib, family):
    b = adversarial_bytes(family, n=5000)
    e, o = gpu_lib.to_device(b)
    codes, idx = gpu_lib.encode(e, o, "bytes8")
    want, bad = oracle.encode(b, "bytes8")
    assert bad == 0
    np.testing.assert_array_equal(codes.cpu().numpy().view(np.uint64), want)
    np.testing.assert_array_equal(_u32(idx), np.arange(b.n, dtype=np.uint32))


@pytest.mark.parametrize("family", BYTES_FAMILIES)
@pytest.mark.parametrize("n", [3000, 70_001])
def test_bytes8_sort_families(gpu_lib, family, n):
    b = adversarial_bytes(family, n=n, seed=n)
    e, o = gpu_lib.to_device(b)
    perm = _u32(gpu_lib.sort(e, o, "bytes8"))
    ref, bad = oracle.sort(b)
    assert bad == 0
    np.testing.assert_array_equal(perm, ref)


@pytest.mark.parametrize("n", [1, 2, 4097, 300_001, (1 << 21) + 17])
def test_bytes8_sort_utf8(gpu_lib, n):
    b = utf8_words(n=n, seed=n % 1000 + 1)
    e, o = gpu_lib.to_device(b)
    ws = gpu_lib.alloc_workspace(b.n)
    perm = _u32(gpu_lib.sort(e, o, "bytes8", ws=ws))
    st = gpu_lib.read_status(ws)
    ref, _ = oracle.sort(b)
    np.testing.assert_array_equal(perm, ref)
    say(b.name, "runs visited", st["runs_fixed"], "device-wide rounds", st["large_rounds"])


def test_bytes8_ascii_text_same_as_ascii_coder(gpu_lib):
    # on 7-bit text the two byte coders give the same (unique) permutation
    b = config2(n=400_000, seed=12)
    e, o = gpu_lib.to_device(b)
    np.testing.assert_array_equal(_u32(gpu_lib.sort(e, o, "bytes8")), _u32(gpu_lib.sort(e, o, "ascii7")))


def test_bytes8_high_bytes_in_first_nine(gpu_lib):
    # what the 7-bit coder refuses as a domain violation, the byte coder sorts
    b = from_strings([b"\x80", b"a", b"\xff\x00", b"\xc3\xa9t\xc3\xa9", b"abcdefgh\xff", b"abcdefgh\x7f",
                      b""] * 300, "bytes8")
    e, o = gpu_lib.to_device(b)
    with pytest.raises(gpu_lib.DomainError):
        gpu_lib.sort(e, o, "ascii7")
    np.testing.assert_array_equal(_u32(gpu_lib.sort(e, o, "bytes8")), oracle.sort(b)[0])


def test_bytes8_batched(gpu_lib):
    import torch

    b = utf8_words(n=600_000, seed=21)
    rng = np.random.default_rng(21)
    cuts = np.sort(rng.choice(np.arange(1, b.n), size=299, replace=False))
    b.seg_offsets = np.concatenate([[0], cuts, [b.n]]).astype(np.uint64)
    e, o = gpu_lib.to_device(b)
    seg = torch.from_numpy(b.seg_offsets.view(np.int64)).cuda()
    perm = _u32(gpu_lib.sort_batched(e, o, seg, "bytes8"))
    ref, _ = oracle.sort_batched(b)
    np.testing.assert_array_equal(perm, ref)


@pytest.mark.parametrize("maker", [lambda: utf8_words(n=400_000, seed=31),
                                   lambda: adversarial_bytes("bytes_prefix8", n=60_000)],
                         ids=["utf8", "bytes_prefix8"])
def test_bytes8_learned(gpu_lib, maker):
    b = maker()
    e, o = gpu_lib.to_device(b)
    ws = gpu_lib.alloc_learned_workspace(b.n)
    model = gpu_lib.fit_learned(e, o, "bytes8", gpu_lib.make_learned_params(sample_frac=0.05), ws=ws)
    perm = _u32(gpu_lib.sort_learned(e, o, model, "bytes8", ws=ws))
    np.testing.assert_array_equal(perm, oracle.sort(b)[0])


def test_bytes8_fixed_rounds_and_device_check(gpu_lib):
    import torch

    b = adversarial_bytes("bytes_prefix8", n=40_000, seed=5)
    e, o = gpu_lib.to_device(b)
    t = gpu_lib.make_tuning(t_medium=256,
                            max_rounds=gpu_lib.rounds_for(int(np.diff(b.offsets).max()), "bytes8"))
    perm = gpu_lib.sort(e, o, "bytes8", tuning=t)
    ref, _ = oracle.sort(b)
    np.testing.assert_array_equal(_u32(perm), ref)
    assert gpu_lib.check_perm(e, o, perm, "bytes8") == 0
    bad = ref.copy()
    bad[[0, 1]] = bad[[1, 0]]
    assert gpu_lib.check_perm(e, o, torch.from_numpy(bad.view(np.int32)).cuda(), "bytes8") > 0


# ------------------------------------------------------------------ husky_refine
def _refine_case(gpu_lib, b, keys, shared, coder):
    """Sort (keys, index) stably on the host, refine on the GPU, compare with the
    oracle's Step 3 over the same runs."""
    import torch

    keys = np.asarray(keys, dtype=np.uint64)
    sk, idx = oracle.sort_pairs(keys, np.arange(b.n, dtype=np.uint32))
    e, o = gpu_lib.to_device(b)
    dk = torch.from_numpy(sk.view(np.int64)).cuda()
    di = torch.from_numpy(idx.view(np.int32)).cuda()
    got = _u32(gpu_lib.refine(e, o, dk, di, shared, coder))
    want = oracle.fixup(b, sk, idx)
    np.testing.assert_array_equal(got, want)
    return got


def test_refine_husky_codes_bytes8(gpu_lib):
    b = utf8_words(n=250_000, seed=41)
    codes, _ = oracle.encode(b, "bytes8")
    got = _refine_case(gpu_lib, b, codes, 8, "bytes8")
    np.testing.assert_array_equal(got, oracle.sort(b)[0])


@pytest.mark.parametrize("shared", [0, 1, 2])
def test_refine_coarse_keys_bytes(gpu_lib, shared):
    # keys = the first `shared` bytes only (0: every string in one run, which
    # the whole refinement then sorts from its first byte)
    b = adversarial_bytes("bytes_random", n=120_000, seed=43 + shared)
    codes, _ = oracle.encode(b, "bytes8")
    keys = codes >> np.uint64(64 - 8 * shared) if shared else np.zeros(b.n, dtype=np.uint64)
    got = _refine_case(gpu_lib, b, keys, shared, "bytes8")
    if shared == 0:
        np.testing.assert_array_equal(got, oracle.sort(b)[0])


def test_refine_random_keys_say_nothing(gpu_lib):
    # arbitrary keys: runs of equal keys hold unrelated strings; with shared 0
    # each run is sorted by the full comparator and nothing else moves
    b = config2(n=200_000, seed=45)
    rng = np.random.default_rng(45)
    keys = rng.integers(0, 3000, size=b.n).astype(np.uint64)
    _refine_case(gpu_lib, b, keys, 0, "ascii7")


@pytest.mark.parametrize("shared", [0, 1, 4])
def test_refine_utf16(gpu_lib, shared):
    b = adversarial("utf16_prefix4", n=50_000, seed=47) if shared else config3(n=100_000, seed=47)
    codes, _ = oracle.encode(b, "utf16")
    keys = codes >> np.uint64(64 - 16 * shared) if shared else np.zeros(b.n, dtype=np.uint64)
    _refine_case(gpu_lib, b, keys, shared, "utf16")


def test_refine_segments_and_errors(gpu_lib):
    import torch

    b = utf8_words(n=90_000, seed=49)
    b.seg_offsets = np.array([0, 1000, 1001, 50_000, b.n], dtype=np.uint64)
    e, o = gpu_lib.to_device(b)
    keys = np.zeros(b.n, dtype=np.uint64)
    idx = np.arange(b.n, dtype=np.uint32)
    seg = torch.from_numpy(b.seg_offsets.view(np.int64)).cuda()
    dk = torch.from_numpy(keys.view(np.int64)).cuda()
    di = torch.from_numpy(idx.view(np.int32)).cuda()
    got = _u32(gpu_lib.refine(e, o, dk, di, 0, "bytes8", seg_offsets=seg))
    np.testing.assert_array_equal(got, oracle.sort_batched(b)[0])
    with pytest.raises(gpu_lib.HuskyError):
        gpu_lib.refine(e, o, dk, di, 16, "bytes8")
