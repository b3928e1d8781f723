"""GPU parity of the radix passes over packed varying bits.

A key bit that has the same value in every key of a segment cannot change
that segment's order, so the multi-tile radix passes take their digits over
the varying bits only, packed from the least significant up, whenever that
needs fewer passes than fixed-width digits.  These cases make packing the
cheaper choice:
keys whose varying bits are scattered (five of every eight, or a random
subset), inside a bit range that does not start or end on a digit edge, with
6-, 7- and 8-bit digits, at sizes that go through the single-tile sort and
the multi-tile passes; and batched instances whose varying bits differ (the
multi-tile passes pack the union of the instances' varying bits).
Permutations are compared with numpy's stable sort and with the oracle.
"""

import sys

import numpy as np
import pytest

import oracle
from workloads import from_strings

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[case]", *a, file=sys.stderr, flush=True)


def _u64(t):
    return t.cpu().numpy().view(np.uint64)


def _u32(t):
    return t.cpu().numpy().view(np.uint32)


MASKS = {
    "five_of_eight": np.uint64(0x1F1F1F1F1F1F1F1F),
    "scattered": np.uint64(0x8421_0C30_5005_A0F1),
    "two_runs": np.uint64(0x0000_FFF0_0000_0FFF),
}


@pytest.mark.parametrize("n", [4096, 4097, 50_000, 300_001])
@pytest.mark.parametrize("mask", sorted(MASKS))
@pytest.mark.parametrize("bits", [(0, 64), (3, 61)])
@pytest.mark.parametrize("radix", [(8, 16), (7, 12), (6, 8)], ids=["b8i16", "b7i12", "b6i8"])
def test_sort_pairs_packed(gpu_lib, n, mask, bits, radix):
    import torch

    _say("packed sort_pairs", n, mask, bits, radix)
    rng = np.random.default_rng([n, radix[0], bits[0]])
    base = rng.integers(0, 2**63, size=n, dtype=np.uint64) * np.uint64(2) + rng.integers(0, 2, size=n, dtype=np.uint64)
    fixed = np.uint64(0x5A5A_A5A5_3C3C_C3C3) & ~MASKS[mask]
    keys = (base & MASKS[mask]) | fixed
    keys[rng.random(n) < 0.2] = keys[0]  # ties
    vals = rng.permutation(n).astype(np.uint32)
    k = torch.from_numpy(keys.view(np.int64)).cuda()
    v = torch.from_numpy(vals.view(np.int32)).cuda()
    t = gpu_lib.make_tuning(radix_bits=radix[0], tile_items=radix[1])
    gpu_lib.sort_pairs(k, v, bits[0], bits[1], tuning=t)
    lo, hi = bits
    field = (keys & np.uint64(((1 << (hi - lo)) - 1) << lo)) >> np.uint64(lo)
    order = np.argsort(field, kind="stable")
    np.testing.assert_array_equal(_u32(v), vals[order])
    np.testing.assert_array_equal(_u64(k), keys[order])


def test_batched_instances_with_different_varying_bits(gpu_lib):
    import torch

    # instance alphabets: two letters, ten digits, six capitals, the full
    # lowercase range; sizes on both sides of one radix tile
    rng = np.random.default_rng(17)
    alphabets = [b"ab", b"0123456789", b"ABCDEF", bytes(range(97, 123))]
    sizes = [3000, 9000, 20000, 4096, 4097, 12000, 700, 30000]
    strs, seg = [], [0]
    for j, m in enumerate(sizes):
        alpha = np.frombuffer(alphabets[j % len(alphabets)], dtype=np.uint8)
        for _ in range(m):
            L = int(rng.integers(0, 20))
            strs.append(bytes(alpha[rng.integers(0, len(alpha), size=L)].tolist()))
        seg.append(seg[-1] + m)
    b = from_strings(strs, name="mixed_alphabets")
    b.seg_offsets = np.array(seg, dtype=np.uint64)
    _say("batched packed", b.n)
    e, o = gpu_lib.to_device(b)
    so = torch.from_numpy(b.seg_offsets.view(np.int64)).cuda()
    perm = _u32(gpu_lib.sort_batched(e, o, so, "ascii7"))
    np.testing.assert_array_equal(perm, oracle.sort_batched(b)[0])
