"""GPU: the device exactness check, the fixed-round (graph-capturable) mode,
HIP-graph capture and replay of the batched sort and of a sort whose fix-up
tiers run on side streams, and the autotuner."""

import numpy as np
import pytest

import oracle
from workloads import adversarial, config2, config4, from_strings

pytestmark = pytest.mark.gpu


def _u32(t):
    return t.cpu().numpy().view(np.uint32)


def test_check_perm_device(gpu_lib):
    import torch

    b = config2(n=50_000)
    e, o = gpu_lib.to_device(b)
    ref, _ = oracle.sort(b)
    good = torch.from_numpy(ref.view(np.int32)).cuda()
    assert gpu_lib.check_perm(e, o, good, "ascii7") == 0
    swapped = ref.copy()
    swapped[[100, 101]] = swapped[[101, 100]]
    assert gpu_lib.check_perm(e, o, torch.from_numpy(swapped.view(np.int32)).cuda(), "ascii7") > 0
    dup = ref.copy()
    dup[7] = dup[8]
    assert gpu_lib.check_perm(e, o, torch.from_numpy(dup.view(np.int32)).cuda(), "ascii7") > 0
    # equal strings out of index order
    b2 = from_strings([b"same", b"same", b"other"])
    e2, o2 = gpu_lib.to_device(b2)
    assert gpu_lib.check_perm(e2, o2, torch.tensor([2, 0, 1], dtype=torch.int32).cuda()) == 0
    assert gpu_lib.check_perm(e2, o2, torch.tensor([2, 1, 0], dtype=torch.int32).cuda()) == 1


def test_check_perm_batched_device(gpu_lib):
    import torch

    b = config4(n_inst=30, lo=1, hi=9000)
    e, o = gpu_lib.to_device(b)
    seg = torch.from_numpy(b.seg_offsets.view(np.int64)).cuda()
    ref, _ = oracle.sort_batched(b)
    assert gpu_lib.check_perm(e, o, torch.from_numpy(ref.view(np.int32)).cuda(), "ascii7", seg) == 0
    glob, _ = oracle.sort(b)  # one global sort is not a per-instance sort
    assert gpu_lib.check_perm(e, o, torch.from_numpy(glob.view(np.int32)).cuda(), "ascii7", seg) > 0


@pytest.mark.parametrize("maker", [lambda: config2(n=300_000), lambda: adversarial("identical", n=30000),
                                   lambda: adversarial("prefix12", n=30000)])
def test_fixed_rounds_equal_adaptive(gpu_lib, maker):
    b = maker()
    e, o = gpu_lib.to_device(b)
    max_len = int(np.diff(b.offsets).max())
    t = gpu_lib.make_tuning(t_medium=256, max_rounds=gpu_lib.rounds_for(max_len, b.coder))
    ws = gpu_lib.alloc_workspace(b.n)
    perm = _u32(gpu_lib.sort(e, o, b.coder, tuning=t, ws=ws))
    assert gpu_lib.read_status(ws)["unresolved"] == 0
    np.testing.assert_array_equal(perm, oracle.sort(b)[0])


def _two_level_groups():
    # 20,000 strings sharing 30 bytes, then one of two bytes, 30 more shared
    # bytes and a distinct tail: the first device-wide round splits the run
    # at the differing byte into two groups, each still longer than one
    # workgroup holds in LDS, and only a second round tells them apart
    rng = np.random.default_rng(7)
    tails = [bytes(rng.integers(97, 123, size=6, dtype=np.uint8).tolist()) for _ in range(20_000)]
    return from_strings([b"a"] + [b"x" * 30 + (b"p" if i % 2 else b"q") + b"x" * 30 + t
                                  for i, t in enumerate(tails)])


def test_fixed_rounds_reports_unresolved(gpu_lib):
    b = _two_level_groups()
    e, o = gpu_lib.to_device(b)
    ws = gpu_lib.alloc_workspace(b.n)
    t = gpu_lib.make_tuning(t_medium=256, max_rounds=1)
    gpu_lib.sort(e, o, "ascii7", tuning=t, ws=ws, check_status=False)
    assert gpu_lib.read_status(ws)["unresolved"] > 0
    # the binding's default status check refuses the unfinished permutation,
    # for the plain, batched and learned forms
    with pytest.raises(gpu_lib.UnresolvedError):
        gpu_lib.sort(e, o, "ascii7", tuning=t, ws=ws)
    import torch

    seg = torch.tensor([0, 1, b.n], dtype=torch.int64, device="cuda")  # the two groups in one instance
    with pytest.raises(gpu_lib.UnresolvedError):
        gpu_lib.sort_batched(e, o, seg, "ascii7", tuning=t)
    model = gpu_lib.fit_learned(e, o, "ascii7", gpu_lib.make_learned_params(sample_frac=0.1))
    with pytest.raises(gpu_lib.UnresolvedError):
        gpu_lib.sort_learned(e, o, model, "ascii7", tuning=t)
    # enough rounds: no error, and the oracle's answer
    ok = gpu_lib.make_tuning(t_medium=256, max_rounds=gpu_lib.rounds_for(67))
    np.testing.assert_array_equal(_u32(gpu_lib.sort(e, o, "ascii7", tuning=ok, ws=ws)), oracle.sort(b)[0])


def test_graph_capture_replay_batched(gpu_lib):
    import torch

    b = config4(n_inst=64, lo=16, hi=20000)
    e, o = gpu_lib.to_device(b)
    seg = torch.from_numpy(b.seg_offsets.view(np.int64)).cuda()
    max_len = int(np.diff(b.offsets).max())
    t = gpu_lib.make_tuning(max_rounds=gpu_lib.rounds_for(max_len))
    ws = gpu_lib.alloc_workspace(b.n, 64)
    perm = torch.empty(b.n, dtype=torch.int32, device="cuda")
    eager = _u32(gpu_lib.sort_batched(e, o, seg, "ascii7", tuning=t, ws=ws, perm=perm)).copy()
    np.testing.assert_array_equal(eager, oracle.sort_batched(b)[0])
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):  # warm-up on the capture stream
        gpu_lib.sort_batched(e, o, seg, "ascii7", tuning=t, ws=ws, perm=perm, check_status=False)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        gpu_lib.sort_batched(e, o, seg, "ascii7", tuning=t, ws=ws, perm=perm, check_status=False)
    for rep in range(3):
        perm.fill_(-1)  # eager work between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        np.testing.assert_array_equal(_u32(perm), eager, err_msg=f"replay {rep}")
        assert gpu_lib.read_status(ws)["unresolved"] == 0


def test_graph_capture_replay_side_streams(gpu_lib):
    # a sort large enough that Step 3's tiers run on the library's side
    # streams: the fork and join are captured with the graph, and every
    # replay gives the eager (and the oracle's) permutation
    import torch

    b = config2(seed=4, n=(1 << 21) + 12345)
    e, o = gpu_lib.to_device(b)
    max_len = int(np.diff(b.offsets).max())
    t = gpu_lib.make_tuning(max_rounds=gpu_lib.rounds_for(max_len))
    ws = gpu_lib.alloc_workspace(b.n, 1)
    perm = torch.empty(b.n, dtype=torch.int32, device="cuda")
    eager = _u32(gpu_lib.sort(e, o, "ascii7", tuning=t, ws=ws, perm=perm)).copy()
    np.testing.assert_array_equal(eager, oracle.sort(b)[0])
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):  # warm-up on the capture stream
        gpu_lib.sort(e, o, "ascii7", tuning=t, ws=ws, perm=perm, check_status=False)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        gpu_lib.sort(e, o, "ascii7", tuning=t, ws=ws, perm=perm, check_status=False)
    for rep in range(3):
        perm.fill_(-1)  # eager work between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        np.testing.assert_array_equal(_u32(perm), eager, err_msg=f"replay {rep}")
        assert gpu_lib.read_status(ws)["unresolved"] == 0


def test_tuner_small(gpu_lib, tmp_path, monkeypatch):
    from paper_2012_00866_amd import tuner

    monkeypatch.setenv("HUSKY_TUNING_CACHE", str(tmp_path / "t.json"))
    b = config2(n=200_000)
    e, o = gpu_lib.to_device(b)
    res = tuner.tune(e, o, "ascii7", repeats=2)
    assert all(r["exact"] for r in res["table"])
    assert res["ms"] <= res["default_ms"]
    t = tuner.cached_tuning("ascii7", b.n, False)
    assert t is not None and t.as_dict()["radix_bits"] == res["tuning"]["radix_bits"]
    perm = _u32(gpu_lib.sort(e, o, "ascii7", tuning=t))
    np.testing.assert_array_equal(perm, oracle.sort(b)[0])
    # the binding's "tuned" choice reads the same cache entry
    np.testing.assert_array_equal(_u32(gpu_lib.sort(e, o, "ascii7", tuning="tuned")), perm)
    assert gpu_lib._tuned("tuned", "ascii7", b.n, False).as_dict() == t.as_dict()
    # nothing cached for the batched form of this size: the defaults
    assert gpu_lib._tuned("tuned", "ascii7", b.n, True) is None
