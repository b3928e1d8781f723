"""GPU parity at the full workload sizes, in the launch configuration the
benchmark uses (default tuning, one call per workload).

* 2^24 collision-heavy ASCII strings and 2^23 UTF-16 strings: the whole GPU
  permutation equals the oracle's, element by element.
* 4,096 batched instances (~1.3e8 strings): every instance's slice passes the
  oracle's per-instance check (permutation of its range, adjacent strings in
  order, equal strings in index order -- which together pin the unique stable
  answer), and 48 sampled instances equal the oracle's full sort.
* 2e8 URL-like strings: the oracle's check over every adjacent pair and the
  permutation property; then the learned-CDF form (fitted on the default 1 %
  sample) on the same input must give the same permutation element by
  element, and the device check must find no violation in it.
"""

import numpy as np
import pytest

import oracle
from _progress import say
from workloads import config2, config3, config4, config5

pytestmark = pytest.mark.gpu


def _u32(t):
    return t.cpu().numpy().view(np.uint32)


@pytest.mark.parametrize("maker", [config2, config3], ids=["config2_16M", "config3_8M"])
def test_full_size_exact(gpu_lib, maker):
    b = maker()
    say("full size", b.name, "generated")
    e, o = gpu_lib.to_device(b)
    perm = _u32(gpu_lib.sort(e, o, b.coder))
    say("gpu sort done")
    ref, bad = oracle.sort(b)
    say("oracle done")
    assert bad == 0
    np.testing.assert_array_equal(perm, ref)


def test_full_size_batched(gpu_lib):
    import torch

    b = config4()
    say("batched", b.name, b.n, "strings generated")
    e, o = gpu_lib.to_device(b)
    seg = torch.from_numpy(b.seg_offsets.view(np.int64)).cuda()
    perm = _u32(gpu_lib.sort_batched(e, o, seg, "ascii7"))
    say("gpu batched sort done")
    bad, first = oracle.check_perm_batched(b, perm)
    say("per-instance check done", bad)
    assert bad == 0, f"first bad position {first}"
    rng = np.random.default_rng(4)
    sizes = np.diff(b.seg_offsets)
    pick = set(rng.choice(len(sizes), size=46, replace=False).tolist())
    pick |= {int(np.argmax(sizes)), int(np.argmin(sizes))}
    for k in sorted(pick):
        lo, hi = int(b.seg_offsets[k]), int(b.seg_offsets[k + 1])
        ref, _ = oracle.sort(b.subset(lo, hi))
        np.testing.assert_array_equal(perm[lo:hi], ref + lo)
    say("sampled instances equal the oracle")


def test_full_size_urls(gpu_lib):
    import torch

    b = config5()
    say("urls", b.name, "generated", b.elems.size, "bytes")
    e, o = gpu_lib.to_device(b)
    ws = gpu_lib.alloc_learned_workspace(b.n)
    plain = gpu_lib.sort(e, o, "ascii7", ws=ws)
    perm = _u32(plain)
    say("gpu sort done")
    bad, first = oracle.check_perm(b, perm)
    say("oracle check done", bad)
    assert bad == 0, f"first bad position {first}"
    del perm
    model = gpu_lib.fit_learned(e, o, "ascii7", ws=ws)
    learned = gpu_lib.sort_learned(e, o, model, "ascii7", ws=ws)
    st = gpu_lib.read_status(ws)
    say("learned sort done: overflow buckets", st["overflow_buckets"], "keys", st["overflow_keys"])
    same = bool(torch.equal(learned, plain))
    if not same:
        diff = torch.nonzero(learned != plain)[:8].flatten().tolist()
        raise AssertionError(f"learned permutation differs from the plain one at {diff}")
    assert gpu_lib.check_perm(e, o, learned, "ascii7") == 0
    say("learned permutation equals the plain one and passes the device check")
