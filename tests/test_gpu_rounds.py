"""GPU: the device-wide refinement rounds without host synchronisation.

By default a sort launches one device-wide round without reading anything
back and finishes every group still tied in one workgroup per group (the
tail).  A round keys each group where its members first differ, so copies of
one string finish in it and a long shared prefix costs no extra round; these
tests use inputs whose long runs split into long groups more than once --
many copies of a few long strings and strings cut from them at random
lengths -- in every form (plain, batched, learned, full-byte, UTF-16,
husky_refine) and check:

* the default permutation equals the oracle's, and the adaptive mode's
  (HUSKY_ROUNDS_ADAPTIVE, the host reading the counts each round);
* the default call can be captured into a HIP graph (a host synchronisation
  inside the capture would fail it) and every replay gives the eager result;
* the counters: default calls report the rounds they launched and nothing
  unresolved.
"""

import numpy as np
import pytest

import oracle
from _progress import say
from workloads import config2, config4, from_strings

pytestmark = pytest.mark.gpu

ADAPTIVE = 0xFFFFFFFF


def _u32(t):
    return t.cpu().numpy().view(np.uint32)


def _long_runs(coder="ascii7", seed=1, n=60_000):
    """Copies of a few long strings (60-120 elements) plus strings that share
    their first 40 elements with them and differ later; groups of > 8,192."""
    rng = np.random.default_rng(seed)
    if coder == "utf16":
        bases = [tuple(int(x) for x in rng.integers(0x4E00, 0x4E08, size=int(rng.integers(30, 60))))
                 for _ in range(4)]
        out = []
        for _ in range(n):
            b = bases[int(rng.integers(0, 4))]
            if rng.random() < 0.5:
                out.append(b)
            else:
                cut = int(rng.integers(20, len(b)))
                out.append(b[:cut] + tuple(int(x) for x in rng.integers(0x4E00, 0x4E02, size=int(rng.integers(0, 5)))))
        return from_strings(out, "utf16")
    bases = [bytes(rng.integers(97, 100, size=int(rng.integers(60, 120)), dtype=np.uint8).tolist())
             for _ in range(4)]
    if coder == "bytes8":
        bases = [bytes((c + 100) % 256 for c in b) for b in bases]
    out = []
    for _ in range(n):
        b = bases[int(rng.integers(0, 4))]
        if rng.random() < 0.5:
            out.append(b)
        else:
            cut = int(rng.integers(40, len(b)))
            out.append(b[:cut] + bytes(rng.integers(97, 99, size=int(rng.integers(0, 6)), dtype=np.uint8).tolist()))
    return from_strings(out, coder)


@pytest.mark.parametrize("coder", ["ascii7", "utf16", "bytes8"])
def test_default_rounds_and_tail_exact(gpu_lib, coder):
    b = _long_runs(coder, seed={"ascii7": 1, "utf16": 2, "bytes8": 3}[coder])
    e, o = gpu_lib.to_device(b)
    ws = gpu_lib.alloc_workspace(b.n)
    perm = _u32(gpu_lib.sort(e, o, coder, ws=ws))
    st = gpu_lib.read_status(ws)
    np.testing.assert_array_equal(perm, oracle.sort(b)[0])
    assert st["unresolved"] == 0 and st["large_rounds"] == 1
    adaptive = _u32(gpu_lib.sort(e, o, coder, tuning=gpu_lib.make_tuning(max_rounds=ADAPTIVE), ws=ws))
    np.testing.assert_array_equal(adaptive, perm)
    say(coder, "adaptive rounds", gpu_lib.read_status(ws)["large_rounds"])


def test_identical_copies_finish_in_one_round(gpu_lib):
    # 9,000 copies of one 60-byte string: the common-prefix pass finds no
    # difference, so the first device-wide round settles them (index order)
    b = from_strings([b"x" * 60] * 9000 + [b"y"])
    e, o = gpu_lib.to_device(b)
    ws = gpu_lib.alloc_workspace(b.n)
    ref = oracle.sort(b)[0]
    perm = _u32(gpu_lib.sort(e, o, "ascii7", tuning=gpu_lib.make_tuning(max_rounds=ADAPTIVE), ws=ws))
    np.testing.assert_array_equal(perm, ref)
    assert gpu_lib.read_status(ws)["large_rounds"] == 1
    np.testing.assert_array_equal(_u32(gpu_lib.sort(e, o, "ascii7", ws=ws)), ref)


def test_tail_groups_after_split(gpu_lib):
    # a run of 20,000 that the round splits at byte 30 into two groups of
    # 10,000 still tied (they share 30 more bytes): the tail finishes them;
    # tails from a small pool leave identical copies, kept in index order
    rng = np.random.default_rng(11)
    pool = [bytes(rng.integers(97, 100, size=int(rng.integers(0, 4)), dtype=np.uint8).tolist())
            for _ in range(40)]
    b = from_strings([b"x" * 30 + (b"p" if i % 2 else b"q") + b"x" * 30 + pool[int(rng.integers(0, 40))]
                      for i in range(20_000)] + [b"a"])
    e, o = gpu_lib.to_device(b)
    ws = gpu_lib.alloc_workspace(b.n)
    np.testing.assert_array_equal(_u32(gpu_lib.sort(e, o, "ascii7", ws=ws)), oracle.sort(b)[0])
    st = gpu_lib.read_status(ws)
    assert st["unresolved"] == 0 and st["large_rounds"] == 1


def test_shared_prefix_beyond_search_span(gpu_lib):
    # 9,000 copies of a 1,500-byte string and 9,000 that differ in its last
    # byte: the common-prefix search gives up after 1,024 bytes and keys the
    # group there; the tail (default) or a second round (adaptive) goes on
    base = b"k" * 1499
    b = from_strings([base + b"z"] * 9000 + [base + b"y"] * 9000 + [b"a"])
    e, o = gpu_lib.to_device(b)
    ref = oracle.sort(b)[0]
    np.testing.assert_array_equal(_u32(gpu_lib.sort(e, o, "ascii7")), ref)
    ws = gpu_lib.alloc_workspace(b.n)
    ad = _u32(gpu_lib.sort(e, o, "ascii7", tuning=gpu_lib.make_tuning(max_rounds=ADAPTIVE), ws=ws))
    np.testing.assert_array_equal(ad, ref)
    assert gpu_lib.read_status(ws)["large_rounds"] == 2


def _wide_groups(seed, n, prefixes=2):
    """A few groups of hundreds of thousands of strings that share 20 bytes
    and differ in the 6 after them: the device-wide round sorts segments of
    more than 64 radix tiles (several scan groups each)."""
    rng = np.random.default_rng(seed)
    heads = [bytes(rng.integers(97, 123, size=20, dtype=np.uint8).tolist()) for _ in range(prefixes)]
    tails = rng.integers(97, 123, size=(n, 6), dtype=np.uint8)
    pick = rng.integers(0, prefixes, size=n)
    return from_strings([heads[int(pick[i])] + tails[i].tobytes() for i in range(n)] + [b"a"])


@pytest.mark.parametrize("adaptive", [False, True])
def test_round_segments_of_several_scan_groups(gpu_lib, adaptive):
    # two groups of ~300,000 (73 tiles each): the round's digit passes scan
    # their counts in more than one group of 64 tiles
    b = _wide_groups(seed=21, n=600_000)
    e, o = gpu_lib.to_device(b)
    ws = gpu_lib.alloc_workspace(b.n)
    tn = gpu_lib.make_tuning(max_rounds=ADAPTIVE) if adaptive else None
    perm = _u32(gpu_lib.sort(e, o, "ascii7", tuning=tn, ws=ws))
    np.testing.assert_array_equal(perm, oracle.sort(b)[0])
    assert gpu_lib.read_status(ws)["unresolved"] == 0


def test_round_segments_of_several_scan_groups_batched(gpu_lib):
    import torch

    b = _wide_groups(seed=22, n=700_000, prefixes=1)
    b.seg_offsets = np.array([0, 250_000, 250_001, b.n], dtype=np.uint64)
    e, o = gpu_lib.to_device(b)
    seg = torch.from_numpy(b.seg_offsets.view(np.int64)).cuda()
    np.testing.assert_array_equal(_u32(gpu_lib.sort_batched(e, o, seg, "ascii7")), oracle.sort_batched(b)[0])


def _edge_group(coder, seed, n=40_000):
    """Runs of more than 8,192 equal codes whose members differ only at the
    common-prefix pass's edges: strings shorter than the coded prefix whose
    codes tie through zero elements (NUL / 0x00 / U+0000 padding), strings that
    are prefixes of others, copies, and differences right at the start of the
    first chunk, at its end and two chunks on."""
    rng = np.random.default_rng(seed)
    if coder == "utf16":
        z, a, b = 0, 0x4E00, 0x4E01
        head = (a,) * 4
        pick = [head[:2], head[:2] + (z,), head[:2] + (z, z), head, head + (a,) * 3,
                head + (a,) * 3 + (b,), head + (a,) * 9, head + (a,) * 9 + (z,), head + (b,)]
        mk = tuple
    else:
        z, a, b = 0, (0xC3 if coder == "bytes8" else ord("q")), (0xFF if coder == "bytes8" else ord("r"))
        m = 8 if coder == "bytes8" else 9
        head = bytes([a]) * m
        pick = [head[:3], head[:3] + b"\0", head[:3] + b"\0\0", head, head + bytes([a]) * 7,
                head + bytes([a]) * 7 + bytes([b]), head + bytes([a]) * 21, head + bytes([a]) * 21 + b"\0",
                head + bytes([b])]
        mk = bytes
    out = [mk(pick[int(rng.integers(0, len(pick)))]) for _ in range(n)]
    return from_strings(out, coder)


@pytest.mark.parametrize("coder", ["ascii7", "utf16", "bytes8"])
def test_common_prefix_pass_edges(gpu_lib, coder):
    b = _edge_group(coder, seed={"ascii7": 5, "utf16": 6, "bytes8": 7}[coder])
    e, o = gpu_lib.to_device(b)
    ref = oracle.sort(b)[0]
    ws = gpu_lib.alloc_workspace(b.n)
    np.testing.assert_array_equal(_u32(gpu_lib.sort(e, o, coder, ws=ws)), ref)
    assert gpu_lib.read_status(ws)["unresolved"] == 0
    ad = _u32(gpu_lib.sort(e, o, coder, tuning=gpu_lib.make_tuning(max_rounds=ADAPTIVE), ws=ws))
    np.testing.assert_array_equal(ad, ref)


def test_default_batched_learned_refine(gpu_lib):
    import torch

    b = _long_runs("ascii7", seed=4, n=50_000)
    e, o = gpu_lib.to_device(b)
    ref = oracle.sort(b)[0]
    # learned form: buckets of > 8,192 copies go to the radix passes, then Step 3
    model = gpu_lib.fit_learned(e, o, "ascii7", gpu_lib.make_learned_params(sample_frac=0.05))
    np.testing.assert_array_equal(_u32(gpu_lib.sort_learned(e, o, model, "ascii7")), ref)
    # husky_refine from all-equal keys
    keys = torch.zeros(b.n, dtype=torch.int64, device="cuda")
    idx = torch.arange(b.n, dtype=torch.int32, device="cuda")
    np.testing.assert_array_equal(_u32(gpu_lib.refine(e, o, keys, idx, 0, "ascii7")), ref)
    # batched: two instances holding long runs
    b.seg_offsets = np.array([0, 20_000, b.n], dtype=np.uint64)
    seg = torch.from_numpy(b.seg_offsets.view(np.int64)).cuda()
    np.testing.assert_array_equal(_u32(gpu_lib.sort_batched(e, o, seg, "ascii7")), oracle.sort_batched(b)[0])


def _capture_replays(gpu_lib, call, check, reps=3):
    import torch

    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):  # warm-up on the capture stream
        call()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        call()
    for rep in range(reps):
        check(rep, before=True)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        check(rep, before=False)


@pytest.mark.parametrize("which", ["long_runs", "config2", "batched"])
def test_default_call_captures_and_replays(gpu_lib, which):
    import torch

    if which == "batched":
        b = config4(n_inst=200, lo=64, hi=60_000, seed=5)
    elif which == "config2":
        b = config2(n=(1 << 21) + 3, seed=6)  # side streams in use
    else:
        b = _long_runs("ascii7", seed=7)
    e, o = gpu_lib.to_device(b)
    seg = torch.from_numpy(b.seg_offsets.view(np.int64)).cuda() if which == "batched" else None
    ns = 1 if seg is None else int(seg.numel()) - 1
    ws = gpu_lib.alloc_workspace(b.n, ns)
    perm = torch.empty(b.n, dtype=torch.int32, device="cuda")

    def call():
        if seg is None:
            gpu_lib.sort(e, o, "ascii7", ws=ws, perm=perm, check_status=False)
        else:
            gpu_lib.sort_batched(e, o, seg, "ascii7", ws=ws, perm=perm, check_status=False)

    call()
    eager = _u32(perm).copy()
    ref = oracle.sort_batched(b)[0] if seg is not None else oracle.sort(b)[0]
    np.testing.assert_array_equal(eager, ref)

    def check(rep, before):
        if before:
            perm.fill_(-1)
        else:
            np.testing.assert_array_equal(_u32(perm), eager, err_msg=f"replay {rep}")
            assert gpu_lib.read_status(ws)["unresolved"] == 0

    _capture_replays(gpu_lib, call, check)
