"""GPU parity of the fix-up tier that keeps a run in LDS for all its rounds.

Runs longer than t_medium and at most 8,192 strings are re-sorted by one
workgroup (four size classes: up to 3,072, 4,096, 6,144 and 8,192).  Every
run below is a set of strings sharing a 12-element prefix (so their codes are
equal) with suffixes over a two-letter alphabet, which leaves groups tied for
several refinement rounds, plus exact duplicates (ties that end as identical
strings, kept in index order) and strings that stop inside the shared prefix.
Lengths sit on both sides of every class edge and of the 8,192 limit (a run of
8,193 goes device-wide, and its residual groups come back to this tier).
Permutations are compared with the oracle element by element.
"""

import sys

import numpy as np
import pytest

import oracle
from workloads import from_strings

pytestmark = pytest.mark.gpu

EDGE_LENGTHS = (1025, 2000, 3072, 3073, 4096, 4097, 6144, 6145, 8192, 8193)


def _say(*a):
    print("[case]", *a, file=sys.stderr, flush=True)


def _u32(t):
    return t.cpu().numpy().view(np.uint32)


def _runs_batch(coder, lengths, seed):
    rng = np.random.default_rng([seed, 7, 1])
    lo, hi = (97, 123) if coder == "ascii7" else (0x4E00, 0x9FA6)
    alpha = (97, 98) if coder == "ascii7" else (0x4E00, 0x4E01)
    out = []
    for L in lengths:
        prefix = [int(v) for v in rng.integers(lo, hi, size=12)]
        run = []
        for _ in range(L):
            r = rng.random()
            if run and r < 0.15:
                run.append(run[int(rng.integers(0, len(run)))])  # exact duplicate
            elif r < 0.18:
                run.append(prefix[: int(rng.integers(9, 13))])  # ends inside the prefix
            else:
                k = int(rng.integers(0, 31))
                run.append(prefix + [alpha[int(b)] for b in rng.integers(0, 2, size=k)])
        out.extend(run)
    # a run of identical long strings: tied until the last round
    out.extend([[alpha[0]] * 60] * 5000)
    order = rng.permutation(len(out))
    strs = [out[i] for i in order]
    if coder == "ascii7":
        strs = [bytes(s) for s in strs]
    return from_strings(strs, coder=coder, name=f"lds_runs_{coder}")


def _sort(husky, b, tuning=None, ws=None):
    e, o = husky.to_device(b)
    return _u32(husky.sort(e, o, b.coder, tuning=tuning, ws=ws))


@pytest.mark.parametrize("coder", ["ascii7", "utf16"])
def test_lds_tier_class_edges(gpu_lib, coder):
    b = _runs_batch(coder, EDGE_LENGTHS, seed=3)
    _say("lds edges", coder, b.n)
    np.testing.assert_array_equal(_sort(gpu_lib, b), oracle.sort(b)[0])


@pytest.mark.parametrize("t_medium", [64, 3072, 4096])
def test_lds_tier_thresholds(gpu_lib, t_medium):
    # t_medium 3072 / 4096 leave one or two of the four classes out
    b = _runs_batch("ascii7", (70, 1500, 3100, 4090, 5000, 7000), seed=t_medium)
    _say("lds t_medium", t_medium, b.n)
    t = gpu_lib.make_tuning(t_small=16, t_medium=t_medium)
    np.testing.assert_array_equal(_sort(gpu_lib, b, t), oracle.sort(b)[0])


def test_lds_tier_fixed_rounds(gpu_lib):
    # the LDS tier runs every round a run needs even when the device-wide tier
    # is held to a fixed round count
    b = _runs_batch("ascii7", (2500, 8193, 9000), seed=11)
    _say("lds fixed rounds", b.n)
    max_len = int(np.diff(b.offsets).max())
    t = gpu_lib.make_tuning(max_rounds=gpu_lib.rounds_for(max_len, b.coder))
    ws = gpu_lib.alloc_workspace(b.n)
    perm = _sort(gpu_lib, b, t, ws)
    assert gpu_lib.read_status(ws)["unresolved"] == 0
    np.testing.assert_array_equal(perm, oracle.sort(b)[0])


def test_lds_tier_fixup_entry_point(gpu_lib):
    import torch

    b = _runs_batch("ascii7", (1200, 5000, 8192), seed=5)
    _say("lds fixup entry", b.n)
    codes, _ = oracle.encode(b)
    c, i = oracle.sort_pairs(codes, np.arange(b.n, dtype=np.uint32))
    e, o = gpu_lib.to_device(b)
    ct = torch.from_numpy(c.view(np.int64)).cuda()
    it = torch.from_numpy(i.view(np.int32)).cuda()
    gpu_lib.fixup(e, o, ct, it, "ascii7")
    np.testing.assert_array_equal(_u32(it), oracle.fixup(b, c, i))
