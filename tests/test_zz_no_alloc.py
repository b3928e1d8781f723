"""GPU: husky_sort_noalloc (no workspace, no allocation; a fixed per-device
scratch array) gives husky_sort's permutation, on two calls in a row -- the
second with a smaller input, so the scratch holds the first call's contents
-- and rejects inputs above its maximum before enqueueing anything."""

import ctypes

import numpy as np
import pytest

import oracle
from workloads import adversarial, config2, config3

pytestmark = pytest.mark.gpu


def _u32(t):
    return t.cpu().numpy().view(np.uint32)


@pytest.mark.parametrize("first,second", [
    (lambda: config2(n=1 << 20, seed=41), lambda: config2(n=300_001, seed=42)),
    (lambda: config3(n=700_000, seed=43), lambda: adversarial("identical", n=20_000)),
    (lambda: adversarial("prefix12", n=50_000), lambda: config2(n=3, seed=44)),
], ids=["config2_full_then_ragged", "utf16_then_ascii_identical", "prefix12_then_tiny"])
def test_noalloc_equals_sort(gpu_lib, first, second):
    import torch

    for k, make in enumerate((first, second)):
        b = make()
        e, o = gpu_lib.to_device(b)
        want = _u32(gpu_lib.sort(e, o, b.coder))
        perm = torch.full((b.n,), -1, dtype=torch.int32, device="cuda")
        got = _u32(gpu_lib.sort_noalloc(e, o, perm, b.coder))
        np.testing.assert_array_equal(got, want, err_msg=f"call {k}: {b.name}")
        st = gpu_lib.noalloc_status()
        assert st["domain_violations"] == 0 and st["unresolved"] == 0
    # the last one against the oracle as well
    np.testing.assert_array_equal(got, oracle.sort(b)[0])


def test_noalloc_fixed_rounds_and_empty(gpu_lib):
    import torch

    b = adversarial("identical", n=30_000)
    e, o = gpu_lib.to_device(b)
    t = gpu_lib.make_tuning(t_medium=256, max_rounds=gpu_lib.rounds_for(int(np.diff(b.offsets).max())))
    perm = torch.empty(b.n, dtype=torch.int32, device="cuda")
    np.testing.assert_array_equal(_u32(gpu_lib.sort_noalloc(e, o, perm, "ascii7", tuning=t)),
                                  oracle.sort(b)[0])
    empty = torch.zeros(1, dtype=torch.int64, device="cuda")
    assert gpu_lib.sort_noalloc(e, empty, perm, "ascii7").numel() == 0


def test_noalloc_rejects_above_maximum(gpu_lib):
    import torch

    lib = gpu_lib.load()
    n = gpu_lib.NOALLOC_MAX_STRINGS + 1
    offsets = torch.arange(n + 1, dtype=torch.int64, device="cuda")
    elems = torch.full((n,), 97, dtype=torch.uint8, device="cuda")
    perm = torch.full((n,), -1, dtype=torch.int32, device="cuda")
    code = lib.husky_sort_noalloc(0, elems.data_ptr(), offsets.data_ptr(), n, perm.data_ptr(), None,
                                  torch.cuda.current_stream().cuda_stream)
    assert code == 7
    assert "no-allocation" in lib.husky_status_string(code).decode()
    torch.cuda.synchronize()
    assert bool((perm == -1).all())  # nothing was enqueued
