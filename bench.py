#!/usr/bin/env python3
"""Benchmark of the Huskysort hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

One step is one complete husky_sort (encode, stable radix pair sort, run
detection, tiered fix-up) of the collision-heavy workload: 2^24 ASCII strings,
60 % Zipf(1.1) draws from a 200,000-word vocabulary and 40 % one of 1,000
random 12-character prefixes plus a 4..20 character suffix (seed 1).  Inputs
are resident in HBM before the timed region starts.  Prints one JSON line.

The timed permutation is checked against the CPU oracle's element by element
(and by the device checker); a mismatch ends the run with status 1 and no
line.  The same run then measures the two extensions against the plain path
on their own workloads, each with an identical permutation required:

* "learned": 2e8 URL-like strings, the learned-CDF form (fit on a 1 % sample)
  against the plain GPU sort of the same input, per model variant;
* "batched": 4,096 independent instances (~1.3e8 strings) in one batched call,
  tuned, and replayed from a HIP graph, against a loop of plain calls.

The roofline object is for the radix scatter pass (k_scatter, the kernel with
the most time): its algorithmic traffic is 24 bytes per string per launch
(read and write of the 8-byte code and the 4-byte index), divided by the
pass's average launch duration measured with HIP events on the library's
stream during the timed steps (events that the pass's dispatch records
itself, through hipExtLaunchKernelGGL, so the host's enqueueing is not in
the interval).  `traffic` is the HBM bytes per launch from
the committed FETCH_SIZE / WRITE_SIZE counter summary (null once radix.hip has
changed since).  "pass_roofline" is the same 24 bytes per string over a whole
digit pass (digit counts, the two scans and the scatter).  The CPU baseline is
the plain oracle (single thread) on the same input, median of three runs.
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
COUNTERS_FILE = os.path.join(ROOT, "profiles", "radix_scatter_config2_counters.txt")
RADIX_SRC = os.path.join(ROOT, "paper_2012_00866_amd", "csrc", "radix.hip")


def _function_text(src: str, signature: str) -> str:
    """Text of one function from its signature line to the closing brace at column 0."""
    i = src.index(signature)
    j = src.index("\n}\n", i)
    return src[i:j + 3]


def _src_sha(path: str) -> str:
    """Hash of the scatter kernel's own source: rank_digits, rank_tile and load_striped
    (rank.h), k_scatter."""
    with open(os.path.join(os.path.dirname(path), "rank.h")) as f:
        rank = f.read()
    with open(path) as f:
        src = f.read()
    parts = [_function_text(rank, "__device__ __forceinline__ void rank_digits("),
             _function_text(rank, "__device__ __forceinline__ void rank_tile("),
             _function_text(rank, "__device__ __forceinline__ void load_striped("),
             _function_text(src, "__global__ __launch_bounds__(BLOCK) void k_scatter(")]
    return hashlib.sha256("".join(parts).encode()).hexdigest()[:16]


def _read_summary(path: str) -> dict:
    kv = {}
    if os.path.exists(path):
        with open(path) as f:
            for line in f:
                if "=" in line and not line.lstrip().startswith("#"):
                    k, v = line.split("=", 1)
                    kv[k.strip()] = v.strip()
    return kv


def _traffic_per_launch():
    """HBM bytes per scatter-pass launch from the committed counter summary, or None.

    Only used while the kernel's source is identical to the one the counters
    were taken from."""
    kv = _read_summary(COUNTERS_FILE)
    if kv.get("radix_src_sha") != _src_sha(RADIX_SRC):
        return None
    try:
        return float(kv["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


BUCKET_COUNTERS_FILE = os.path.join(ROOT, "profiles", "learned_bucket_pass_config5_counters.txt")
LEARNED_SRC = os.path.join(ROOT, "paper_2012_00866_amd", "csrc", "learned.hip")


def _bucket_src_sha() -> str:
    """Hash of the bucket pass's own source: rank_digits (rank.h) and k_bscatter."""
    with open(os.path.join(os.path.dirname(LEARNED_SRC), "rank.h")) as f:
        rank = f.read()
    with open(LEARNED_SRC) as f:
        src = f.read()
    parts = [_function_text(rank, "__device__ __forceinline__ void rank_digits("),
             _function_text(src, "__global__ __launch_bounds__(BLOCK) void k_bscatter(")]
    return hashlib.sha256("".join(parts).encode()).hexdigest()[:16]


def _bucket_traffic_per_string():
    """HBM bytes per string for the pair of bucket passes, from the committed
    counter summary, or None once the kernel's source has changed."""
    kv = _read_summary(BUCKET_COUNTERS_FILE)
    if kv.get("bucket_src_sha") != _bucket_src_sha():
        return None
    try:
        return float(kv["hbm_bytes_per_string_both_passes"])
    except (KeyError, ValueError):
        return None


def _host_info():
    """Host CPU model, logical CPUs (all and usable by this process) and RAM."""
    model, mem_kb = "unknown", 0
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
        with open("/proc/meminfo") as f:
            for line in f:
                if line.startswith("MemTotal"):
                    mem_kb = int(line.split()[1])
                    break
    except OSError:
        pass
    usable = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    return {"cpu_model": model, "nproc": os.cpu_count(), "nproc_usable": usable,
            "ram_gib": round(mem_kb / 2**20, 1)}


def _step2_vs_platform(husky, torch, elems, offsets, ws, reps=5):
    """Step 2 alone (husky_sort_pairs on the codes, 12 bytes per key) against the
    platform's radix sort (torch.sort, rocPRIM: the same keys with an int64
    index) on the same codes; HIP events around each sort only."""
    import numpy as np

    codes, idx = husky.encode(elems, offsets, "ascii7")
    c2, i2 = torch.empty_like(codes), torch.empty_like(idx)
    signed = codes ^ torch.tensor(-(1 << 63), dtype=torch.int64, device=codes.device)  # unsigned order

    def timed(prep, run):
        ms = []
        for r in range(reps + 1):
            prep()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            out = run()
            e1.record()
            torch.cuda.synchronize()
            if r:
                ms.append(e0.elapsed_time(e1))
        return float(np.median(ms)), out

    def prep():
        c2.copy_(codes)
        i2.copy_(idx)

    ours_ms, _ = timed(prep, lambda: husky.sort_pairs(c2, i2, ws=ws))
    torch_ms, (_, ti) = timed(lambda: None, lambda: torch.sort(signed, stable=True))
    return {"what": "stable sort of the 2^24 codes with their indices: husky_sort_pairs "
                    "(u64 code, u32 index) vs torch.sort(stable=True) (rocPRIM, i64 index)",
            "husky_sort_pairs_ms": round(ours_ms, 4), "torch_sort_ms": round(torch_ms, 4),
            "identical": bool(torch.equal(ti.to(torch.int32), i2))}


def _cpu_baseline(batch, runs=3):
    """The oracle (single-threaded C++) on the whole workload, median of `runs`
    sorts; returns (baseline object, the oracle's permutation)."""
    import oracle

    times, ref = [], None
    for _ in range(runs):
        t0 = time.perf_counter()
        ref, bad = oracle.sort(batch)
        times.append(time.perf_counter() - t0)
        if bad:
            raise RuntimeError(f"oracle reports {bad} out-of-domain strings")
    dt = sorted(times)[len(times) // 2]
    return {
        "value": round(batch.n / dt / 1e6, 4),
        "unit": "Mstrings/s",
        "cores": 1,
        "kind": "oracle",
        "sample": f"full workload ({batch.n} strings), single-threaded oracle sort, median of "
                  f"{runs} runs ({', '.join(f'{t:.2f}' for t in times)} s)",
        "host": _host_info(),
    }, ref


METRIC = "Mstrings/s sorted (bit-exact) + HBM GB/s % peak; learned & batched vs plain"


def _progress(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--n", type=int, default=1 << 24, help="strings (default 2^24)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-learned", action="store_true", help="leave out the learned comparison")
    ap.add_argument("--no-batched", action="store_true", help="leave out the batched comparison")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run a 256 MiB device copy (calibrates HBM byte counters)")
    ap.add_argument("--mode", choices=["plain", "batched", "learned", "lossy", "typed", "configs"],
                    default="plain",
                    help="plain: the metric's workload (with both comparisons); batched or "
                         "learned: only that comparison, printed as its own line; lossy: the "
                         "mis-coding study; typed: the other object types; configs: the plain "
                         "sort on configs 1 and 3")
    args = ap.parse_args(argv)
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); the sort is not "
              "sharded across GPUs.", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    import paper_2012_00866_amd as husky
    from workloads import config2

    husky.load()
    if args.copy_probe:
        src = torch.ones(256 << 20, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(2):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if args.mode == "learned":
        out = bench_learned(args)
        print(json.dumps(out), flush=True)
        return 0
    if args.mode == "batched":
        out = bench_batched(args)
        print(json.dumps(out), flush=True)
        return 0
    if args.mode == "lossy":
        print(json.dumps(bench_lossy(args)), flush=True)
        return 0
    if args.mode == "typed":
        print(json.dumps(bench_typed(args)), flush=True)
        return 0
    if args.mode == "configs":
        print(json.dumps(bench_configs(args)), flush=True)
        return 0
    batch = config2(seed=1, n=args.n)
    n = batch.n
    elems, offsets = husky.to_device(batch)
    ws = husky.alloc_workspace(n)
    perm = torch.empty(n, dtype=torch.int32, device="cuda")
    stream = torch.cuda.current_stream()
    _progress(f"config 2: {n} strings resident")

    husky.sort(elems, offsets, "ascii7", ws=ws, perm=perm)  # raises on a bad status
    for _ in range(args.warmup):
        husky.sort(elems, offsets, "ascii7", ws=ws, perm=perm, check_status=False)
    torch.cuda.synchronize()

    # timed region: only the scatter pass is bracketed by HIP events (recorded
    # by its dispatch on the library's stream), so the step time is not
    # perturbed by the others
    husky.profile_begin(["radix_scatter"])
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(stream)
    for _ in range(args.steps):
        husky.sort(elems, offsets, "ascii7", ws=ws, perm=perm, check_status=False)
    ev1.record(stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = husky.profile_end()
    status = husky.read_status(ws)
    # the timed output: the device checker here, the oracle's permutation below
    violations = husky.check_perm(elems, offsets, perm, "ascii7")
    got = perm.cpu().numpy().view(np.uint32).copy()
    # per-kernel breakdown: a separate run of the same steps, every class timed
    ksteps = min(args.steps, 10)
    husky.profile_begin()
    for _ in range(ksteps):
        husky.sort(elems, offsets, "ascii7", ws=ws, perm=perm, check_status=False)
    kprof = husky.profile_end()
    _progress(f"plain: {(t1 - t0) * 1e3 / args.steps:.3f} ms per sort")
    step2 = _step2_vs_platform(husky, torch, elems, offsets, ws)
    _progress(f"step 2 alone: {step2['husky_sort_pairs_ms']} ms, torch.sort {step2['torch_sort_ms']} ms")

    ms_per_step = (t1 - t0) * 1e3 / args.steps
    value = n / (ms_per_step / 1e3) / 1e6
    os_ms, os_launches = prof["radix_scatter"]
    avg_ms = os_ms / max(os_launches, 1)
    algo_bytes = 24.0 * n
    achieved = algo_bytes / (avg_ms / 1e3) / 1e9 if avg_ms > 0 else 0.0
    traffic = _traffic_per_launch()
    kernels = {k: {"ms_per_step": round(v[0] / ksteps, 4), "launches_per_step": v[1] / ksteps}
               for k, v in kprof.items() if v[1]}
    # a whole digit pass of the code sort: digit counts + the two scans + the scatter
    passes = kprof["radix_scatter"][1] / ksteps
    # (the device-wide fix-up's own count and scan launches are a class of their own)
    pass_ms = (kprof["radix_count_scan"][0] + kprof["radix_scatter"][0]) / ksteps / max(passes, 1)
    pass_gbs = algo_bytes / (pass_ms / 1e3) / 1e9 if pass_ms > 0 else 0.0

    out = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "Mstrings/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {
            "workload": "collision-heavy ASCII strings (config 2): 60% Zipf(1.1) words from a "
                        "200k vocabulary + 40% 12-char prefix + 4..20 suffix",
            "n": n,
            "seed": 1,
            "coder": "ascii7",
            "elems_bytes": int(batch.elems.size),
            "runs_fixed": status["runs_fixed"],
            "large_rounds": status["large_rounds"],
        },
        "roofline": {
            "kernel": "radix scatter pass (k_scatter)",
            "bound": "hbm",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic,
            "algorithmic_bytes_per_launch": algo_bytes,
            "avg_launch_ms": round(avg_ms, 5),
            "launches_per_step": os_launches / args.steps,
        },
        "pass_roofline": {
            "what": "one whole digit pass of the code sort: k_count + k_group_scan + k_seg_scan "
                    "+ k_scatter, 24 algorithmic bytes per string",
            "bound": "hbm",
            "achieved": round(pass_gbs, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(pass_gbs / HBM_PEAK_GBS, 4),
            "ms_per_pass": round(pass_ms, 5),
            "passes_per_step": passes,
        },
        "kernels": kernels,
        "step2_vs_platform_sort": step2,
        "event_ms_per_step": round(ev0.elapsed_time(ev1) / args.steps, 4),
        "device_check_violations": violations,
    }
    if violations:
        print(f"bench.py: the device check finds {violations} violations in the timed "
              "permutation", file=sys.stderr)
        return 1
    if not args.no_cpu_baseline:
        out["cpu_baseline"], ref = _cpu_baseline(batch)
        if not np.array_equal(got, ref):
            first = int(np.nonzero(got != ref)[0][0])
            print(f"bench.py: the timed permutation differs from the oracle's (first at "
                  f"position {first})", file=sys.stderr)
            return 1
        out["oracle_identical"] = True
        _progress("timed permutation equals the oracle's")
    del elems, offsets, ws, perm, batch
    torch.cuda.empty_cache()
    if not args.no_learned:
        out["learned"] = bench_learned(args)
        torch.cuda.empty_cache()
    if not args.no_batched:
        out["batched"] = bench_batched(args)
    print(json.dumps(out), flush=True)
    return 0


def _time(fn, steps, warmup):
    import torch

    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) * 1e3 / steps


def bench_batched(args):
    """4,096 instances (config 4): one batched call vs a loop of plain calls, tuned and graph forms."""
    import numpy as np
    import torch

    import paper_2012_00866_amd as husky
    from paper_2012_00866_amd import tuner
    from workloads import config4

    t_gen = time.perf_counter()
    batch = config4(seed=1)
    t_gen = time.perf_counter() - t_gen
    n, S = batch.n, batch.seg_offsets.size - 1
    elems, offsets = husky.to_device(batch)
    seg = torch.from_numpy(batch.seg_offsets.view(np.int64)).cuda()
    ws = husky.alloc_workspace(n, S)
    perm = torch.empty(n, dtype=torch.int32, device="cuda")
    steps = max(3, min(args.steps, 10))
    _progress(f"config 4: {n} strings in {S} instances resident ({t_gen:.1f} s to generate)")

    def batched(t=None):
        husky.sort_batched(elems, offsets, seg, "ascii7", tuning=t, ws=ws, perm=perm, check_status=False)

    ms_default = _time(batched, steps, 1)
    ref = perm.clone()
    assert husky.check_perm(elems, offsets, ref, "ascii7", seg) == 0, "batched result not exact"
    res = tuner.tune(elems, offsets, "ascii7", seg, repeats=3)
    tuned = husky.make_tuning(**res["tuning"])
    ms_tuned = _time(lambda: batched(tuned), steps, 1)
    assert torch.equal(perm, ref)
    husky.profile_begin()
    batched(tuned)
    kprof = husky.profile_end()
    # graph: the same call (it never waits for the host), captured once, replayed
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        batched(tuned)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        batched(tuned)
    perm.fill_(-1)
    ms_graph = _time(g.replay, steps, 1)
    assert torch.equal(perm, ref) and husky.read_status(ws)["unresolved"] == 0
    del g
    # loop of plain sorts, one call per instance, same tuning
    ws1 = husky.alloc_workspace(int(np.diff(batch.seg_offsets).max()))
    offs = [(int(batch.seg_offsets[k]), int(batch.seg_offsets[k + 1])) for k in range(S)]

    def loop():
        for lo, hi in offs:
            husky.sort(elems, offsets[lo:hi + 1], "ascii7", tuning=tuned, ws=ws1, perm=perm[lo:hi],
                       check_status=False)

    ms_loop = _time(loop, max(1, steps // 3), 1)
    lp = perm.cpu().numpy().view(np.uint32).astype(np.int64)
    for k, (lo, hi) in enumerate(offs):
        lp[lo:hi] += lo
    assert np.array_equal(lp.astype(np.uint32), ref.cpu().numpy().view(np.uint32)), "loop differs"
    _progress(f"batched: {ms_tuned:.3f} ms tuned, loop of plain sorts {ms_loop:.1f} ms")
    return {
        "metric": "Mstrings/s sorted (bit-exact), batched form",
        "value": round(n / (ms_tuned / 1e3) / 1e6, 3),
        "unit": "Mstrings/s",
        "ms_per_step": round(ms_tuned, 4),
        "steps": steps,
        "config": {"workload": "4,096 independent instances of the collision-heavy distribution, "
                               "sizes log-uniform in [64, 262144]", "n": n, "instances": S,
                   "seed": 1, "generation_s": round(t_gen, 1)},
        "forms_ms": {"batched_default": round(ms_default, 3), "batched_tuned": round(ms_tuned, 3),
                     "batched_graph_replay": round(ms_graph, 3),
                     "loop_of_plain_sorts": round(ms_loop, 3)},
        "speedup_batched_vs_loop": round(ms_loop / ms_tuned, 2),
        "kernels_tuned": _kernels(kprof, 1),
        "identical": True,
        "device_check_violations": 0,
        "tuning": res["tuning"],
        "tuner_table": [{"params": r["params"], "ms": round(r["ms"], 3)} for r in res["table"]],
    }


def bench_lossy(args):
    """The Appendix's mis-coding study on the GPU: config 2 sorted from husky codes of
    which a fraction p is replaced by random values (Step 2 on those codes, then the
    run-local and the full stable Step 3), against the plain sort of the same input."""
    import numpy as np
    import torch

    import oracle
    import paper_2012_00866_amd as husky
    from workloads import config2

    n = args.n if args.n != (1 << 24) else 1 << 22
    batch = config2(seed=1, n=n)
    elems, offsets = husky.to_device(batch)
    codes, _ = oracle.encode(batch)
    steps = max(3, min(args.steps, 10))
    ws = husky.alloc_workspace(n)
    perm = torch.empty(n, dtype=torch.int32, device="cuda")
    ms_plain = _time(lambda: husky.sort(elems, offsets, "ascii7", ws=ws, perm=perm, check_status=False),
                     steps, 1)
    ref = perm.clone()
    lws = torch.empty(int(husky.load().husky_lossy_workspace_bytes(n)), dtype=torch.uint8, device="cuda")
    rows = []
    for p in (0.0, 0.001, 0.01, 0.05, 0.1, 0.25, 0.5, 1.0):
        rng = np.random.default_rng(int(p * 1000) + 1)
        c = codes.copy()
        hit = rng.random(n) < p
        c[hit] = rng.integers(0, 2**64 - 1, size=int(hit.sum()), dtype=np.uint64, endpoint=True)
        dc = torch.from_numpy(c.view(np.int64)).cuda()
        ms = _time(lambda: husky.sort_lossy(elems, offsets, dc, "ascii7", ws=lws, perm=perm), steps, 1)
        assert torch.equal(perm, ref), f"lossy sort differs at p={p}"
        husky.profile_begin(["global_merge"])
        husky.sort_lossy(elems, offsets, dc, "ascii7", ws=lws, perm=perm)
        gm = husky.profile_end()["global_merge"][0]
        rows.append({"p": p, "ms": round(ms, 3), "global_pass_ms": round(gm, 3),
                     "vs_plain": round(ms / ms_plain, 3)})
        _progress(f"lossy p={p}: {ms:.3f} ms (global pass {gm:.3f} ms)")
    return {"metric": "ms per sort, lossy codes (mis-coding rate p) vs the plain sort",
            "config": {"workload": "collision-heavy ASCII strings (config 2)", "n": n, "seed": 1,
                       "miscoding": "each code replaced by a uniform random 64-bit value with "
                                    "probability p (seeded)"},
            "plain_ms": round(ms_plain, 3), "rows": rows, "identical": True}


def bench_typed(args):
    """The other object types: Mrecords/s of husky_sort_typed per type (500,000 records,
    the paper's largest size, and 2^24 records), every permutation checked on the device
    against the oracle's at 500,000."""
    import numpy as np
    import torch

    import paper_2012_00866_amd as husky
    from oracle import typed as ot
    from workloads.typed import TYPED, typed

    steps = max(3, min(args.steps, 10))
    rows = {}
    for t in TYPED:
        for n in (500_000, 1 << 24):
            if n > 500_000 and t in ("bigint", "decimal", "tuple"):
                n = 1 << 22  # the Python generator of these records is slow
            b = typed(t, n=n, seed=1)
            r, o = husky.typed_to_device(b)
            ws = torch.empty(husky.typed_workspace_bytes(t, n, int(r.numel())), dtype=torch.uint8,
                             device="cuda")
            perm = torch.empty(n, dtype=torch.int32, device="cuda")
            ms = _time(lambda: husky.sort_typed(r, o, t, n, ws=ws, perm=perm, check_status=False), steps, 1)
            ok = None
            if n == 500_000:
                ok = bool(np.array_equal(perm.cpu().numpy().view(np.uint32), ot.sort(b)[0]))
                assert ok, f"typed sort of {t} differs from the oracle"
            rows[f"{t}_{n}"] = {"ms": round(ms, 3), "mrecords_s": round(n / ms / 1e3, 1),
                                "record_bytes": int(r.numel()), "oracle_identical": ok}
            _progress(f"typed {t} n={n}: {ms:.3f} ms")
            del r, o, ws, perm, b
    return {"metric": "Mrecords/s sorted (bit-exact), other object types", "rows": rows}


def bench_configs(args):
    """The plain sort on the other string workloads: config 1 (100,000 ASCII strings,
    the small case) and config 3 (2^23 UTF-16 strings), Mstrings/s with a per-class
    kernel breakdown; every permutation equal to the oracle's (config 1) or clean
    under the device check (config 3)."""
    import numpy as np
    import torch

    import oracle
    import paper_2012_00866_amd as husky
    from workloads import config1, config3

    steps = max(5, min(args.steps, 50))
    rows = {}
    for name, make in (("config1", config1), ("config3", config3)):
        b = make(seed=1)
        e, o = husky.to_device(b)
        ws = husky.alloc_workspace(b.n)
        perm = torch.empty(b.n, dtype=torch.int32, device="cuda")
        f = lambda: husky.sort(e, o, b.coder, ws=ws, perm=perm, check_status=False)
        ms = _time(f, steps, 2)
        husky.profile_begin()
        f()
        prof = husky.profile_end()
        viol = husky.check_perm(e, o, perm, b.coder)
        assert viol == 0, f"{name}: the device check found {viol} violations"
        ok = None
        if b.n <= 200_000:
            ok = bool(np.array_equal(perm.cpu().numpy().view(np.uint32), oracle.sort(b)[0]))
            assert ok, f"{name} differs from the oracle"
        rows[name] = {"n": b.n, "coder": b.coder, "ms": round(ms, 4), "mstrings_s": round(b.n / ms / 1e3, 1),
                      "launches": sum(v[1] for v in prof.values()), "kernels": _kernels(prof, 1),
                      "oracle_identical": ok, "device_check_violations": viol}
        _progress(f"{name}: {ms:.4f} ms")
        del e, o, ws, perm, b
    return {"metric": "Mstrings/s sorted (bit-exact), plain sort on configs 1 and 3", "rows": rows}


def _kernels(prof, steps):
    return {k: {"ms_per_step": round(v[0] / steps, 4), "launches_per_step": round(v[1] / steps, 2)}
            for k, v in prof.items() if v[1]}


def bench_learned(args):
    """Config 5 (2e8 URL-like strings): learned-CDF form vs the plain GPU path, same input."""
    import torch

    import paper_2012_00866_amd as husky
    from workloads import config5

    n = 200_000_000 if args.mode != "learned" or args.n == (1 << 24) else args.n
    t_gen = time.perf_counter()
    batch = config5(n=n, seed=1)
    t_gen = time.perf_counter() - t_gen
    mean_len = batch.elems.size / n
    elems, offsets = husky.to_device(batch)
    del batch
    _progress(f"config 5: {n} strings resident ({t_gen:.1f} s to generate)")
    ws = husky.alloc_learned_workspace(n)
    perm = torch.empty(n, dtype=torch.int32, device="cuda")
    steps = max(3, min(args.steps, 10))

    def plain():
        husky.sort(elems, offsets, "ascii7", ws=ws, perm=perm, check_status=False)

    ms_plain = _time(plain, steps, 1)
    ref = perm.clone()
    assert husky.check_perm(elems, offsets, ref, "ascii7") == 0, "plain result not exact"
    husky.profile_begin()
    for _ in range(steps):
        plain()
    k_plain = _kernels(husky.profile_end(), steps)

    def fit(**kw):
        return husky.fit_learned(elems, offsets, "ascii7", husky.make_learned_params(**kw), ws=ws)

    variants = {}
    model = None
    for name, kw in (("monotone", {}), ("equal_width", {"mode": "equal_width"}),
                     ("untrained", {"mode": "untrained"}), ("network_alone", {"dense": False}),
                     ("equal_width_alone", {"mode": "equal_width", "dense": False})):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        m = fit(**kw)
        torch.cuda.synchronize()
        ms_fit = (time.perf_counter() - t0) * 1e3
        ms = _time(lambda: husky.sort_learned(elems, offsets, m, "ascii7", ws=ws, perm=perm,
                                              check_status=False), steps, 1)
        st = husky.read_status(ws)
        same = bool(torch.equal(perm, ref))
        assert same, f"learned form ({name}) differs from the plain path"
        h = husky.learned_header(m)
        ids = husky.learned_buckets(elems, offsets, m, "ascii7")
        _, load = torch.unique(ids, return_counts=True)  # sorts; no atomics on hot buckets
        load = load.to(torch.float64)
        exp_load = float((load * load).sum() / n)
        del ids, load
        variants[name] = {"sort_ms": round(ms, 3), "fit_ms": round(ms_fit, 2),
                          "inclusive_ms": round(ms + ms_fit, 3),
                          "speedup_vs_plain": round(ms_plain / ms, 3), "identical": same,
                          "expected_bucket_load": round(exp_load, 1),
                          "overflow_buckets": st["overflow_buckets"],
                          "overflow_keys_frac": round(st["overflow_keys"] / n, 4),
                          "adam_steps": h["steps"], "dense_cells": h["dense"],
                          "dense_sample_frac": round(h["dense_keys"] / max(h["sample"], 1), 4),
                          "trained_on": h["trained"], "last_loss": round(float(h["last_loss"]), 6)}
        _progress(f"learned {name}: {variants[name]}")
        if name == "monotone":
            model = m
        else:
            del m
    ms_learned = variants["monotone"]["sort_ms"]
    husky.profile_begin()
    for _ in range(steps):
        husky.sort_learned(elems, offsets, model, "ascii7", ws=ws, perm=perm, check_status=False)
    prof = husky.profile_end()
    assert husky.check_perm(elems, offsets, perm, "ascii7") == 0, "learned result not exact"
    k_learned = _kernels(prof, steps)
    ms_bs, nb = prof["learned_bucket_scatter"]
    # roofline of the bucket pass: 42 algorithmic bytes per string per pass
    # (84 for the pair), HIP-event durations on the library's stream
    bs_avg_ms = ms_bs / max(nb, 1)
    bs_achieved = 42.0 * n / (bs_avg_ms / 1e3) / 1e9 if nb else 0.0
    tps = _bucket_traffic_per_string()
    del elems, offsets, ws, perm, ref, model
    return {
        "metric": "Mstrings/s sorted (bit-exact), learned-CDF form vs plain",
        "value": round(n / (ms_learned / 1e3) / 1e6, 3),
        "unit": "Mstrings/s",
        "steps": steps,
        "ms_per_step": ms_learned,
        "config": {"workload": "URL-like strings: 'h' + host id (Zipf 1.2 over 10,000 hosts, "
                               "seeded id permutation) + '/' + 1-4 lowercase segments of 3-10",
                   "n": n, "mean_bytes": round(mean_len, 2), "seed": 1, "sample_frac": 0.01,
                   "buckets": 65536, "ideal_bucket_load": round(n / 65536, 1),
                   "generation_s": round(t_gen, 1)},
        "plain_ms": round(ms_plain, 3),
        "plain_mstrings_s": round(n / (ms_plain / 1e3) / 1e6, 3),
        "speedup_learned_vs_plain": round(ms_plain / ms_learned, 3),
        "fit_ms": variants["monotone"]["fit_ms"],
        "inclusive_ms": round(ms_learned + variants["monotone"]["fit_ms"], 3),
        "identical": True,
        "device_check_violations": 0,
        "variants": variants,
        # the two bucket passes move the 8-byte code, the 2-byte id and the 8-byte
        # first refinement key; the index is written by both and read by the second:
        # 40 + 44 bytes per string for the pair of passes
        "roofline": {
            "kernel": "learned bucket pass (k_bscatter)",
            "bound": "hbm",
            "achieved": round(bs_achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(bs_achieved / HBM_PEAK_GBS, 4),
            "traffic": round(tps * n / 2) if tps else None,
            "algorithmic_bytes_per_launch": 42.0 * n,
            "avg_launch_ms": round(bs_avg_ms, 4),
            "launches_per_step": nb / steps,
        },
        "kernels_learned": k_learned,
        "kernels_plain": k_plain,
    }


if __name__ == "__main__":
    sys.exit(main())
