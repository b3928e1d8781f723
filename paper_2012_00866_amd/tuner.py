"""Autotuner for the launch parameters of husky_sort / husky_sort_batched.

It picks the radix digit width, the radix tile size and the two fix-up
thresholds (t_small: runs sorted by one wavefront; t_medium: runs sorted by
one workgroup) for a workload already resident on the GPU:

* coordinate search: (radix_bits, tile_items) first with default thresholds,
  then t_small, then t_medium, each stage keeping the best so far;
* every candidate is timed with HIP events on the current stream (median of
  `repeats` runs after one warm-up);
* a candidate counts only if its permutation passes the device exactness
  check (husky_check_perm: a permutation of every instance, adjacent strings
  in order, equal strings in index order -- which pins the unique answer)
  and equals the permutation of the default parameters;
* results are cached as JSON per (GPU arch, compute units, coder, log2 n band,
  batched), in $HUSKY_TUNING_CACHE or ~/.cache/husky_mi355x/tuning.json;
  `sort(..., tuning="tuned")` and `sort_batched(..., tuning="tuned")` use the
  cached choice (the library's defaults when there is none).

The exactness gate does not need the oracle: husky_check_perm verifies, on
the device and independently of the sort's kernels, that the output is a
permutation of every instance, that adjacent strings are in the comparator's
order and that equal strings keep index order; those three properties
determine the stable sort uniquely, so a candidate that passes the check
returns exactly the oracle's permutation.
"""

from __future__ import annotations

import json
import math
import os
import time
from typing import Callable, Dict, List, Optional

import numpy as np

from . import (Tuning, check_perm, make_tuning, sort, sort_batched, alloc_workspace)

RADIX = [(b, i) for b in (8, 7, 6) for i in (16, 12, 8)]  # every compiled pair
T_SMALL = [8, 16, 32, 64]
T_MEDIUM = [128, 256, 512, 1024, 2048, 3072, 4096]
DEFAULT = dict(radix_bits=8, tile_items=16, t_small=64, t_medium=1024)


def cache_path() -> str:
    p = os.environ.get("HUSKY_TUNING_CACHE")
    if p:
        return p
    return os.path.join(os.path.expanduser("~"), ".cache", "husky_mi355x", "tuning.json")


def cache_key(coder: str, n: int, batched: bool) -> str:
    import torch

    props = torch.cuda.get_device_properties(torch.cuda.current_device())
    arch = getattr(props, "gcnArchName", "gfx").split(":")[0]
    band = int(round(math.log2(max(n, 2))))
    return f"{arch}|cu{props.multi_processor_count}|{coder}|log2n{band}|{'batched' if batched else 'plain'}"


def load_cache() -> Dict:
    try:
        with open(cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def save_cache(c: Dict) -> None:
    p = cache_path()
    os.makedirs(os.path.dirname(p), exist_ok=True)
    tmp = p + ".tmp"
    with open(tmp, "w") as f:
        json.dump(c, f, indent=1, sort_keys=True)
    os.replace(tmp, p)


def cached_tuning(coder: str, n: int, batched: bool) -> Optional[Tuning]:
    e = load_cache().get(cache_key(coder, n, batched))
    return make_tuning(**e["tuning"]) if e else None


def tune(elems, offsets, coder: str = "ascii7", seg_offsets=None, repeats: int = 5,
         stages=("radix", "t_small", "t_medium"), log: Optional[Callable[[str], None]] = None,
         store: bool = True) -> Dict:
    """Search the launch parameters for this workload; returns the winner and the table."""
    import torch

    n = int(offsets.numel()) - 1
    batched = seg_offsets is not None
    ws = alloc_workspace(n, 1 if seg_offsets is None else int(seg_offsets.numel()) - 1, offsets.device)
    perm = torch.empty(max(n, 1), dtype=torch.int32, device=offsets.device)

    def run(t: Tuning):
        if batched:
            return sort_batched(elems, offsets, seg_offsets, coder, tuning=t, ws=ws, perm=perm,
                                check_status=False)
        return sort(elems, offsets, coder, tuning=t, ws=ws, perm=perm, check_status=False)

    ref = run(make_tuning(**DEFAULT)).clone()
    if check_perm(elems, offsets, ref, coder, seg_offsets) != 0:
        raise RuntimeError("default parameters fail the exactness check")

    table: List[Dict] = []

    def measure(params: Dict) -> float:
        t = make_tuning(**params)
        out = run(t)
        ok = bool(torch.equal(out, ref)) and check_perm(elems, offsets, out, coder, seg_offsets) == 0
        times = []
        if ok:
            for _ in range(repeats):
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record()
                run(t)
                e1.record()
                torch.cuda.synchronize()
                times.append(e0.elapsed_time(e1))
        ms = float(np.median(times)) if ok else float("inf")
        table.append({"params": dict(params), "ms": ms, "exact": ok})
        if log:
            log(f"tune {params} -> {'%.3f ms' % ms if ok else 'REJECTED (not exact)'}")
        return ms

    best = dict(DEFAULT)
    best_ms = measure(best)
    for stage in stages:
        if stage == "radix":
            cands = [dict(best, radix_bits=b, tile_items=i) for b, i in RADIX]
        elif stage == "t_small":
            cands = [dict(best, t_small=v) for v in T_SMALL]
        else:
            cands = [dict(best, t_medium=v) for v in T_MEDIUM if v > best["t_small"]]
        for c in cands:
            if c == best:
                continue
            ms = measure(c)
            if ms < best_ms:
                best, best_ms = c, ms
    result = {"tuning": best, "ms": best_ms, "default_ms": table[0]["ms"], "table": table,
              "key": cache_key(coder, n, batched), "time": time.time()}
    if store:
        c = load_cache()
        c[result["key"]] = {"tuning": best, "ms": best_ms, "default_ms": table[0]["ms"]}
        save_cache(c)
    return result
