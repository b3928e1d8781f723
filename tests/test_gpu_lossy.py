"""GPU: Step 3 as a full stable pass (husky_fixup_global) and Algorithm 1 with a
lossy coder (husky_sort_lossy), against the oracle.

* the pass alone turns any order -- shuffled, reversed, already sorted, the
  order of a code sort with collisions -- into the oracle's permutation;
* with exact codes, a fraction p of them replaced by random values (the
  Appendix's deliberate mis-coding, p from 0 to 1), reversed codes and
  constant codes, the lossy sort equals the oracle's on ASCII, UTF-16 and
  UTF-8 text, identical strings and NUL-padded strings, ragged sizes and the
  degenerate n = 0..3.
"""

import numpy as np
import pytest

import oracle
from _progress import say
from workloads import adversarial, adversarial_bytes, config2, config3, utf8_words

pytestmark = pytest.mark.gpu


def _u32(t):
    return t.cpu().numpy().view(np.uint32)


def _dev(a, dtype):
    import torch

    return torch.from_numpy(np.ascontiguousarray(a).view(dtype)).cuda()


def _miscoded(codes, p, seed):
    rng = np.random.default_rng(seed)
    c = np.array(codes, dtype=np.uint64, copy=True)
    hit = rng.random(c.size) < p
    c[hit] = rng.integers(0, 2**64 - 1, size=int(hit.sum()), dtype=np.uint64, endpoint=True)
    return c


MAKERS = {
    "config2": lambda: config2(n=200_003, seed=31),
    "config3": lambda: config3(n=150_001, seed=32),
    "utf8": lambda: utf8_words(n=120_007, seed=33),
    "identical": lambda: adversarial("identical", n=40_000, seed=34),
    "nul": lambda: adversarial("nul", n=30_000, seed=35),
    "bytes_prefix8": lambda: adversarial_bytes("bytes_prefix8", n=30_000, seed=36),
}


def _coder_of(b):
    return b.coder


@pytest.mark.parametrize("name", sorted(MAKERS))
@pytest.mark.parametrize("start", ["shuffled", "reversed", "sorted", "code_sorted"])
def test_global_pass_from_any_order(gpu_lib, name, start):
    import torch

    b = MAKERS[name]()
    e, o = gpu_lib.to_device(b)
    ref, _ = oracle.sort(b)
    if start == "shuffled":
        idx = np.random.default_rng(7).permutation(b.n).astype(np.uint32)
    elif start == "reversed":
        idx = np.arange(b.n, dtype=np.uint32)[::-1].copy()
    elif start == "sorted":
        idx = ref.copy()
    else:  # sorted by the husky code only: runs of equal codes still unsorted
        codes, _ = oracle.encode(b, "bytes8" if b.coder == "bytes8" else None)
        _, idx = oracle.sort_pairs(codes, np.arange(b.n, dtype=np.uint32))
    d = _dev(idx, np.int32)
    gpu_lib.fixup_global(e, o, d, _coder_of(b))
    np.testing.assert_array_equal(_u32(d), ref)
    del torch


@pytest.mark.parametrize("p", [0.0, 0.01, 0.1, 0.25, 0.5, 1.0])
@pytest.mark.parametrize("name", ["config2", "config3", "utf8", "identical"])
def test_lossy_sort_miscoded(gpu_lib, name, p):
    b = MAKERS[name]()
    e, o = gpu_lib.to_device(b)
    codes, _ = oracle.encode(b, "bytes8" if b.coder == "bytes8" else None)
    c = _miscoded(codes, p, 11)
    perm = _u32(gpu_lib.sort_lossy(e, o, _dev(c, np.int64), _coder_of(b)))
    np.testing.assert_array_equal(perm, oracle.sort_lossy(b, c))


def test_lossy_sort_adversarial_codes(gpu_lib):
    b = MAKERS["config2"]()
    e, o = gpu_lib.to_device(b)
    codes, _ = oracle.encode(b)
    ref, _ = oracle.sort(b)
    for c in ((np.uint64(2**64 - 1) - codes).astype(np.uint64), np.zeros(b.n, np.uint64),
              np.arange(b.n, dtype=np.uint64)[::-1].copy()):
        np.testing.assert_array_equal(_u32(gpu_lib.sort_lossy(e, o, _dev(c, np.int64), "ascii7")), ref)


@pytest.mark.parametrize("n", [0, 1, 2, 3, 4097])
def test_lossy_tiny(gpu_lib, n):
    import torch

    b = config2(n=max(n, 1), seed=n + 40)
    if n == 0:
        e, _ = gpu_lib.to_device(b)
        o = torch.zeros(1, dtype=torch.int64, device="cuda")
        assert gpu_lib.sort_lossy(e, o, torch.zeros(1, dtype=torch.int64, device="cuda")).numel() == 0
        return
    e, o = gpu_lib.to_device(b)
    c = _miscoded(oracle.encode(b)[0], 0.5, n)
    np.testing.assert_array_equal(_u32(gpu_lib.sort_lossy(e, o, _dev(c, np.int64))), oracle.sort(b)[0])


def test_lossy_large(gpu_lib):
    # 2^22 + 5 strings, 1 % mis-coded: the oracle checks every adjacent pair
    b = config2(n=(1 << 22) + 5, seed=45)
    e, o = gpu_lib.to_device(b)
    c = _miscoded(oracle.encode(b)[0], 0.01, 45)
    perm = _u32(gpu_lib.sort_lossy(e, o, _dev(c, np.int64)))
    bad, first = oracle.check_perm(b, perm)
    assert bad == 0, first
    say("lossy 2^22: exact")
