"""MI355X Huskysort: Python binding of libhusky.so (C ABI in include/husky.h).

The binding only marshals arguments: every step of the sort runs in the HIP
kernels of ``libhusky.so``.  PyTorch provides device memory and the stream.
If the library has not been built, every call raises ``RuntimeError``; there
is no fallback.

Strings are passed as a packed element tensor plus uint64 element offsets:
``elems`` (uint8 for ASCII and byte strings, int16/uint16 storage of UTF-16
code units) and
``offsets`` (int64 storage of uint64[n + 1]), both on the GPU.
"""

from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhusky.so")

CODERS = {"ascii7": 0, "utf16": 1, "bytes8": 2}
STATUS = {0: "ok", 1: "invalid argument", 2: "domain violation", 3: "workspace",
          4: "HIP runtime error", 5: "unsupported tuning", 6: "groups left tied",
          7: "too many strings for the no-allocation scratch"}


class HuskyError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"{what}: {STATUS.get(code, code)} ({code})")
        self.code = code


class DomainError(HuskyError):
    """An ASCII7 string holds a byte >= 0x80 among its first nine bytes."""


class UnresolvedError(HuskyError):
    """Groups were still tied after tuning.max_rounds fixed rounds: perm is not final."""


def _raise_on_status(ws, what: str):
    """Read the device status block (synchronizes) and raise on a condition that
    leaves the permutation unspecified or not final."""
    st = read_status(ws)
    if st["domain_violations"]:
        raise DomainError(2, f"{what} ({st['domain_violations']} strings)")
    if st["unresolved"]:
        raise UnresolvedError(6, f"{what} ({st['unresolved']} groups; raise tuning.max_rounds)")
    return st


class Tuning(ctypes.Structure):
    _fields_ = [("radix_bits", ctypes.c_int32), ("tile_items", ctypes.c_int32),
                ("t_small", ctypes.c_uint32), ("t_medium", ctypes.c_uint32),
                ("max_rounds", ctypes.c_uint32)]

    def as_dict(self):
        return {f: int(getattr(self, f)) for f, _ in self._fields_}


def make_tuning(radix_bits=0, tile_items=0, t_small=0, t_medium=0, max_rounds=0) -> Tuning:
    return Tuning(int(radix_bits), int(tile_items), int(t_small), int(t_medium), int(max_rounds))


def rounds_for(max_len: int, coder="ascii7") -> int:
    """Fixed device-wide rounds that resolve any run of strings of at most max_len elements."""
    m, c = {0: (9, 7), 1: (4, 3), 2: (8, 7)}[_coder(coder)]
    return max(1, -(-(max(int(max_len), m) - m) // c))


_lib = None

EXPORTS = ("husky_workspace_bytes", "husky_encode", "husky_sort_pairs", "husky_fixup", "husky_refine",
           "husky_sort", "husky_sort_batched", "husky_check_perm", "husky_profile_begin",
           "husky_profile_end", "husky_profile_select", "husky_learned_model_bytes", "husky_learned_offset",
           "husky_learned_workspace_bytes", "husky_learned_fit", "husky_sort_learned",
           "husky_learned_buckets",
           "husky_mlp_grad_workspace_bytes", "husky_mlp_grad", "husky_learned_lut_workspace_bytes",
           "husky_learned_eval_lut", "husky_sort_noalloc", "husky_noalloc_status",
           "husky_typed_workspace_bytes", "husky_encode_typed", "husky_sort_typed",
           "husky_global_workspace_bytes", "husky_fixup_global", "husky_lossy_workspace_bytes",
           "husky_sort_lossy", "husky_status_string")

# kernel classes of husky_profile_end (include/husky.h)
PROFILE_CLASSES = ("encode", "radix_vary", "radix_count_scan", "radix_scatter", "radix_copy_back",
                   "tile_sort", "runs", "fixup_small", "fixup_medium", "large_keys", "segment_setup",
                   "radix_scatter_fixup", "learned_bucket_scatter", "learned_bucket_bounds",
                   "fixup_lds", "global_merge", "radix_count_scan_fixup")

# learned form (include/husky.h)
LEARNED_BUCKETS = 65536
LEARNED_NPARAM = 4353
LEARNED_CELLS = 1 << 24
LEARNED_MODES = {"monotone": 0, "unconstrained": 1, "equal_width": 2, "untrained": 3,
                 "constant": 4}
LEARNED_NO_DENSE = 1
LM_PARTS = {"header": 0, "params": 1, "adam_m": 2, "adam_v": 3, "lut": 4, "splitters": 5,
            "dense": 6, "dense_cum": 7, "subtab": 8, "cellinfo": 9}


class LearnedParams(ctypes.Structure):
    _fields_ = [("sample_frac", ctypes.c_double), ("seed", ctypes.c_uint64),
                ("epochs", ctypes.c_uint32), ("batch", ctypes.c_uint32), ("lr", ctypes.c_float),
                ("mode", ctypes.c_uint32), ("flags", ctypes.c_uint32),
                ("reserved", ctypes.c_uint32)]


class LearnedHeader(ctypes.Structure):
    _fields_ = [("lo", ctypes.c_uint64), ("hi", ctypes.c_uint64), ("cp", ctypes.c_uint32),
                ("buckets", ctypes.c_uint32), ("mode", ctypes.c_uint32),
                ("sample", ctypes.c_uint32), ("steps", ctypes.c_uint32),
                ("last_loss", ctypes.c_float), ("heavy", ctypes.c_uint32),
                ("dense", ctypes.c_uint32), ("dense_keys", ctypes.c_uint32),
                ("trained", ctypes.c_uint32), ("flags", ctypes.c_uint32),
                ("pad", ctypes.c_uint32 * 5)]


def load(path: str = LIB_PATH):
    """Load libhusky.so (raises if it is missing: build it first)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: run `python -m paper_2012_00866_amd.build`")
    lib = ctypes.CDLL(path)
    u64, i32, vp, sz = ctypes.c_uint64, ctypes.c_int, ctypes.c_void_p, ctypes.c_size_t
    tp = ctypes.POINTER(Tuning)
    lib.husky_workspace_bytes.restype = sz
    lib.husky_workspace_bytes.argtypes = [u64, u64]
    lib.husky_encode.restype = i32
    lib.husky_encode.argtypes = [i32, vp, vp, u64, vp, vp, vp, vp]
    lib.husky_sort_pairs.restype = i32
    lib.husky_sort_pairs.argtypes = [vp, vp, u64, i32, i32, vp, sz, tp, vp]
    lib.husky_fixup.restype = i32
    lib.husky_fixup.argtypes = [i32, vp, vp, u64, vp, vp, vp, u64, vp, sz, tp, vp]
    lib.husky_refine.restype = i32
    lib.husky_refine.argtypes = [i32, vp, vp, u64, vp, vp, vp, u64, ctypes.c_uint32, vp, sz, tp, vp]
    lib.husky_sort.restype = i32
    lib.husky_sort.argtypes = [i32, vp, vp, u64, vp, vp, sz, tp, vp]
    lib.husky_sort_batched.restype = i32
    lib.husky_sort_batched.argtypes = [i32, vp, vp, u64, vp, u64, vp, vp, sz, tp, vp]
    lib.husky_check_perm.restype = i32
    lib.husky_check_perm.argtypes = [i32, vp, vp, u64, vp, u64, vp, vp, sz, vp, vp]
    lib.husky_profile_begin.restype = None
    lib.husky_profile_begin.argtypes = []
    lib.husky_profile_end.restype = i32
    lib.husky_profile_end.argtypes = [vp, vp, i32]
    lib.husky_profile_select.restype = None
    lib.husky_profile_select.argtypes = [ctypes.c_uint32]
    lib.husky_learned_model_bytes.restype = sz
    lib.husky_learned_model_bytes.argtypes = []
    lib.husky_learned_offset.restype = sz
    lib.husky_learned_offset.argtypes = [i32]
    lib.husky_learned_workspace_bytes.restype = sz
    lib.husky_learned_workspace_bytes.argtypes = [u64]
    lib.husky_learned_fit.restype = i32
    lib.husky_learned_fit.argtypes = [i32, vp, vp, u64, ctypes.POINTER(LearnedParams), vp, sz, vp,
                                      sz, vp]
    lib.husky_sort_learned.restype = i32
    lib.husky_sort_learned.argtypes = [i32, vp, vp, u64, vp, vp, vp, sz, tp, vp]
    lib.husky_learned_buckets.restype = i32
    lib.husky_learned_buckets.argtypes = [i32, vp, vp, u64, vp, vp, vp, vp]
    lib.husky_mlp_grad_workspace_bytes.restype = sz
    lib.husky_mlp_grad_workspace_bytes.argtypes = [ctypes.c_uint32]
    lib.husky_mlp_grad.restype = i32
    lib.husky_mlp_grad.argtypes = [vp, vp, vp, ctypes.c_uint32, i32, vp, vp, sz, vp]
    lib.husky_learned_lut_workspace_bytes.restype = sz
    lib.husky_learned_lut_workspace_bytes.argtypes = []
    lib.husky_learned_eval_lut.restype = i32
    lib.husky_learned_eval_lut.argtypes = [vp, i32, vp, vp, vp, sz, vp]
    lib.husky_sort_noalloc.restype = i32
    lib.husky_sort_noalloc.argtypes = [i32, vp, vp, u64, vp, tp, vp]
    lib.husky_noalloc_status.restype = i32
    lib.husky_noalloc_status.argtypes = [vp, vp]
    lib.husky_typed_workspace_bytes.restype = sz
    lib.husky_typed_workspace_bytes.argtypes = [i32, u64, u64]
    lib.husky_encode_typed.restype = i32
    lib.husky_encode_typed.argtypes = [i32, vp, vp, u64, ctypes.c_int32, vp, vp, vp]
    lib.husky_sort_typed.restype = i32
    lib.husky_sort_typed.argtypes = [i32, vp, vp, u64, u64, ctypes.c_int32, vp, vp, sz, tp, vp]
    lib.husky_global_workspace_bytes.restype = sz
    lib.husky_global_workspace_bytes.argtypes = [u64]
    lib.husky_fixup_global.restype = i32
    lib.husky_fixup_global.argtypes = [i32, vp, vp, u64, vp, vp, sz, vp]
    lib.husky_lossy_workspace_bytes.restype = sz
    lib.husky_lossy_workspace_bytes.argtypes = [u64]
    lib.husky_sort_lossy.restype = i32
    lib.husky_sort_lossy.argtypes = [i32, vp, vp, u64, vp, vp, vp, sz, tp, vp]
    lib.husky_status_string.restype = ctypes.c_char_p
    lib.husky_status_string.argtypes = [i32]
    _lib = lib
    return lib


# ----------------------------------------------------------------- helpers
def _torch():
    import torch

    return torch


def _ptr(t) -> Optional[int]:
    return None if t is None else int(t.data_ptr())


def _stream(stream=None) -> int:
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


def _coder(c) -> int:
    return CODERS[c] if isinstance(c, str) else int(c)


def _check(code: int, what: str):
    if code != 0:
        raise HuskyError(code, what)


def workspace_bytes(n: int, n_segs: int = 1) -> int:
    return int(load().husky_workspace_bytes(int(n), int(n_segs)))


def alloc_workspace(n: int, n_segs: int = 1, device="cuda"):
    torch = _torch()
    return torch.empty(workspace_bytes(n, n_segs), dtype=torch.uint8, device=device)


STATUS_FIELDS = ("domain_violations", "large_rounds", "runs_fixed", "unresolved",
                 "overflow_buckets", "overflow_keys")


def read_status(ws) -> dict:
    """Device status block (first 24 bytes of the workspace); synchronizes."""
    v = ws[:4 * len(STATUS_FIELDS)].cpu().numpy().view(np.uint32)
    return {f: int(v[i]) for i, f in enumerate(STATUS_FIELDS)}


def to_device(batch, device="cuda"):
    """(elems, offsets) device tensors for a workloads.StringBatch."""
    torch = _torch()
    e = batch.elems
    if e.dtype == np.uint16:
        e = e.view(np.int16)
    if e.size == 0:
        e = np.zeros(8, dtype=e.dtype)
    elems = torch.from_numpy(np.ascontiguousarray(e)).to(device)
    offsets = torch.from_numpy(np.ascontiguousarray(batch.offsets).view(np.int64)).to(device)
    return elems, offsets


def _n_of(offsets) -> int:
    return int(offsets.numel()) - 1


# ----------------------------------------------------------------- entry points
def encode(elems, offsets, coder="ascii7", with_idx=True, status=None, stream=None):
    """Step 1: (codes int64-storage uint64[n], idx int32-storage uint32[n] or None)."""
    torch = _torch()
    lib = load()
    n = _n_of(offsets)
    codes = torch.empty(max(n, 1), dtype=torch.int64, device=offsets.device)
    idx = torch.empty(max(n, 1), dtype=torch.int32, device=offsets.device) if with_idx else None
    _check(lib.husky_encode(_coder(coder), _ptr(elems), _ptr(offsets), n, _ptr(codes), _ptr(idx),
                            _ptr(status), _stream(stream)), "husky_encode")
    return codes[:n], (idx[:n] if idx is not None else None)


def sort_pairs(codes, idx, begin_bit=0, end_bit=64, tuning: Optional[Tuning] = None, ws=None,
               stream=None):
    """Step 2 in place: stable sort of (codes, idx) by bits [begin_bit, end_bit)."""
    lib = load()
    n = int(codes.numel())
    if ws is None:
        ws = alloc_workspace(n, 1, codes.device)
    _check(lib.husky_sort_pairs(_ptr(codes), _ptr(idx), n, int(begin_bit), int(end_bit), _ptr(ws),
                                ws.numel(), ctypes.byref(tuning) if tuning else None,
                                _stream(stream)), "husky_sort_pairs")
    return codes, idx


def fixup(elems, offsets, sorted_codes, idx, coder="ascii7", seg_offsets=None,
          tuning: Optional[Tuning] = None, ws=None, stream=None):
    """Step 3 in place on idx (runs of equal codes re-sorted by the full comparator)."""
    lib = load()
    n = _n_of(offsets)
    ns = 1 if seg_offsets is None else int(seg_offsets.numel()) - 1
    if ws is None:
        ws = alloc_workspace(n, ns, offsets.device)
    _check(lib.husky_fixup(_coder(coder), _ptr(elems), _ptr(offsets), n, _ptr(sorted_codes),
                           _ptr(idx), _ptr(seg_offsets), ns, _ptr(ws), ws.numel(),
                           ctypes.byref(tuning) if tuning else None, _stream(stream)),
           "husky_fixup")
    return idx


def refine(elems, offsets, sorted_keys, idx, shared_elems=0, coder="ascii7", seg_offsets=None,
           tuning: Optional[Tuning] = None, ws=None, stream=None):
    """Re-sort every run of equal sorted_keys by the full comparator, in place on idx;
    every member of a run shares its first min(len, shared_elems) elements (0..15)."""
    lib = load()
    n = _n_of(offsets)
    ns = 1 if seg_offsets is None else int(seg_offsets.numel()) - 1
    if ws is None:
        ws = alloc_workspace(n, ns, offsets.device)
    _check(lib.husky_refine(_coder(coder), _ptr(elems), _ptr(offsets), n, _ptr(sorted_keys),
                            _ptr(idx), _ptr(seg_offsets), ns, int(shared_elems), _ptr(ws), ws.numel(),
                            ctypes.byref(tuning) if tuning else None, _stream(stream)),
           "husky_refine")
    return idx


def _tuned(tuning, coder, n: int, batched: bool) -> Optional[Tuning]:
    """tuning="tuned": the autotuner's cached choice for this GPU, coder, size band
    and form (the library's defaults when nothing is cached); else as given."""
    if isinstance(tuning, str):
        if tuning != "tuned":
            raise ValueError(f"tuning must be a Tuning, None or 'tuned', not {tuning!r}")
        from .tuner import cached_tuning

        return cached_tuning(coder if isinstance(coder, str) else
                             {v: k for k, v in CODERS.items()}[int(coder)], n, batched)
    return tuning


def sort(elems, offsets, coder="ascii7", tuning: Optional[Tuning] = None, ws=None, perm=None,
         stream=None, check_status=True):
    """Algorithm 1 on the GPU: returns perm (int32 storage of uint32[n]).
    tuning: None (defaults), a Tuning, or "tuned" (the autotuner's cached choice)."""
    torch = _torch()
    lib = load()
    n = _n_of(offsets)
    tuning = _tuned(tuning, coder, n, False)
    if ws is None:
        ws = alloc_workspace(n, 1, offsets.device)
    if perm is None:
        perm = torch.empty(max(n, 1), dtype=torch.int32, device=offsets.device)
    _check(lib.husky_sort(_coder(coder), _ptr(elems), _ptr(offsets), n, _ptr(perm), _ptr(ws),
                          ws.numel(), ctypes.byref(tuning) if tuning else None, _stream(stream)),
           "husky_sort")
    if check_status:
        _raise_on_status(ws, "husky_sort")
    return perm[:n]


NOALLOC_MAX_STRINGS = 1 << 20


def sort_noalloc(elems, offsets, perm, coder="ascii7", tuning: Optional[Tuning] = None, stream=None,
                 check_status=True):
    """husky_sort_noalloc: the library allocates nothing and takes no workspace (its
    scratch is a fixed per-device array); perm (int32 storage of uint32[n]) is the
    caller's.  Calls that overlap on one device race."""
    lib = load()
    n = _n_of(offsets)
    _check(lib.husky_sort_noalloc(_coder(coder), _ptr(elems), _ptr(offsets), n, _ptr(perm),
                                  ctypes.byref(tuning) if tuning else None, _stream(stream)),
           "husky_sort_noalloc")
    if check_status:
        st = noalloc_status(stream)
        if st["domain_violations"]:
            raise DomainError(2, f"husky_sort_noalloc ({st['domain_violations']} strings)")
        if st["unresolved"]:
            raise UnresolvedError(6, f"husky_sort_noalloc ({st['unresolved']} groups)")
    return perm[:n]


def noalloc_status(stream=None) -> dict:
    """Status block of the no-allocation scratch on the current device (synchronizes)."""
    v = np.zeros(len(STATUS_FIELDS), dtype=np.uint32)
    _check(load().husky_noalloc_status(v.ctypes.data, _stream(stream)), "husky_noalloc_status")
    return {f: int(v[i]) for i, f in enumerate(STATUS_FIELDS)}


def sort_batched(elems, offsets, seg_offsets, coder="ascii7", tuning: Optional[Tuning] = None,
                 ws=None, perm=None, stream=None, check_status=True):
    """Batched form: every instance sorted on its own; perm holds global indices.
    tuning: None, a Tuning, or "tuned" (the autotuner's cached choice)."""
    torch = _torch()
    lib = load()
    n = _n_of(offsets)
    ns = int(seg_offsets.numel()) - 1
    tuning = _tuned(tuning, coder, n, True)
    if ws is None:
        ws = alloc_workspace(n, ns, offsets.device)
    if perm is None:
        perm = torch.empty(max(n, 1), dtype=torch.int32, device=offsets.device)
    _check(lib.husky_sort_batched(_coder(coder), _ptr(elems), _ptr(offsets), n, _ptr(seg_offsets),
                                  ns, _ptr(perm), _ptr(ws), ws.numel(),
                                  ctypes.byref(tuning) if tuning else None, _stream(stream)),
           "husky_sort_batched")
    if check_status:
        _raise_on_status(ws, "husky_sort_batched")
    return perm[:n]


# ----------------------------------------------------------------- lossy coders
def fixup_global(elems, offsets, idx, coder="ascii7", ws=None, stream=None):
    """The full stable pass: idx (any order of the strings) becomes the stable
    sorting permutation, in place."""
    torch = _torch()
    lib = load()
    n = _n_of(offsets)
    if ws is None:
        ws = torch.empty(int(lib.husky_global_workspace_bytes(n)), dtype=torch.uint8, device=offsets.device)
    _check(lib.husky_fixup_global(_coder(coder), _ptr(elems), _ptr(offsets), n, _ptr(idx), _ptr(ws),
                                  ws.numel(), _stream(stream)), "husky_fixup_global")
    return idx


def sort_lossy(elems, offsets, codes, coder="ascii7", tuning: Optional[Tuning] = None, ws=None, perm=None,
               stream=None):
    """Algorithm 1 with the caller's codes of any quality: the stable sorting permutation."""
    torch = _torch()
    lib = load()
    n = _n_of(offsets)
    if ws is None:
        ws = torch.empty(int(lib.husky_lossy_workspace_bytes(n)), dtype=torch.uint8, device=offsets.device)
    if perm is None:
        perm = torch.empty(max(n, 1), dtype=torch.int32, device=offsets.device)
    _check(lib.husky_sort_lossy(_coder(coder), _ptr(elems), _ptr(offsets), n, _ptr(codes), _ptr(perm),
                                _ptr(ws), ws.numel(), ctypes.byref(tuning) if tuning else None,
                                _stream(stream)), "husky_sort_lossy")
    return perm[:n]


# ----------------------------------------------------------------- typed records
TYPES = {"int32": 0, "int64": 1, "float64": 2, "datetime": 3, "bigint": 4, "decimal": 5, "tuple": 6}
TYPE_WIDTH = {"int32": 4, "int64": 8, "float64": 8, "datetime": 16}


def _type(t) -> int:
    return TYPES[t] if isinstance(t, str) else int(t)


def typed_to_device(batch, device="cuda"):
    """(records uint8 tensor, offsets int64 tensor or None) for a workloads.typed batch."""
    torch = _torch()
    data = batch.data if batch.data.size else np.zeros(8, dtype=np.uint8)
    recs = torch.from_numpy(np.ascontiguousarray(data)).to(device)
    off = None
    if batch.offsets is not None:
        off = torch.from_numpy(np.ascontiguousarray(batch.offsets).view(np.int64)).to(device)
    return recs, off


def typed_workspace_bytes(type_, n: int, record_bytes: int) -> int:
    return int(load().husky_typed_workspace_bytes(_type(type_), int(n), int(record_bytes)))


def encode_typed(records, offsets, type_, n: int, base_year=1970, status=None, stream=None):
    """Step 1 for typed records: the husky codes (int64 storage of uint64[n])."""
    torch = _torch()
    codes = torch.empty(max(n, 1), dtype=torch.int64, device=records.device)
    _check(load().husky_encode_typed(_type(type_), _ptr(records), _ptr(offsets), int(n), int(base_year),
                                     _ptr(codes), _ptr(status), _stream(stream)), "husky_encode_typed")
    return codes[:n]


def sort_typed(records, offsets, type_, n: int, base_year=1970, tuning: Optional[Tuning] = None,
               ws=None, perm=None, stream=None, check_status=True):
    """Huskysort of typed records (numbers, date-times, big numbers, tuples): the
    stable sorting permutation under the type's comparator."""
    torch = _torch()
    lib = load()
    rb = int(records.numel())
    if ws is None:
        ws = torch.empty(typed_workspace_bytes(type_, n, rb), dtype=torch.uint8, device=records.device)
    if perm is None:
        perm = torch.empty(max(n, 1), dtype=torch.int32, device=records.device)
    _check(lib.husky_sort_typed(_type(type_), _ptr(records), _ptr(offsets), int(n), rb, int(base_year),
                                _ptr(perm), _ptr(ws), ws.numel(), ctypes.byref(tuning) if tuning else None,
                                _stream(stream)), "husky_sort_typed")
    if check_status:
        _raise_on_status(ws, "husky_sort_typed")
    return perm[:n]


def check_perm(elems, offsets, perm, coder="ascii7", seg_offsets=None, stream=None) -> int:
    """Violations of the stable-sort property found on the device (0 = exact)."""
    torch = _torch()
    lib = load()
    n = _n_of(offsets)
    ns = 1 if seg_offsets is None else int(seg_offsets.numel()) - 1
    ws = torch.empty(max(4, (n + 31) // 32 * 4), dtype=torch.uint8, device=offsets.device)
    out = torch.zeros(1, dtype=torch.int32, device=offsets.device)
    _check(lib.husky_check_perm(_coder(coder), _ptr(elems), _ptr(offsets), n, _ptr(seg_offsets), ns,
                                _ptr(perm), _ptr(ws), ws.numel(), _ptr(out), _stream(stream)),
           "husky_check_perm")
    return int(out.item())


# ----------------------------------------------------------------- learned form
def learned_model_bytes() -> int:
    return int(load().husky_learned_model_bytes())


def learned_offset(part) -> int:
    return int(load().husky_learned_offset(LM_PARTS[part] if isinstance(part, str) else int(part)))


def learned_workspace_bytes(n: int) -> int:
    return int(load().husky_learned_workspace_bytes(int(n)))


def alloc_learned_workspace(n: int, device="cuda"):
    torch = _torch()
    return torch.empty(learned_workspace_bytes(n), dtype=torch.uint8, device=device)


def make_learned_params(sample_frac=0.0, seed=0, epochs=0, batch=0, lr=0.0, mode="monotone",
                        dense=True) -> LearnedParams:
    m = LEARNED_MODES[mode] if isinstance(mode, str) else int(mode)
    return LearnedParams(float(sample_frac), int(seed), int(epochs), int(batch), float(lr), m,
                         0 if dense else LEARNED_NO_DENSE, 0)


def fit_learned(elems, offsets, coder="ascii7", params: Optional[LearnedParams] = None,
                model=None, ws=None, stream=None):
    """Fit the learned-CDF model on a sample of the strings; returns the model buffer."""
    torch = _torch()
    lib = load()
    n = _n_of(offsets)
    if model is None:
        model = torch.empty(learned_model_bytes(), dtype=torch.uint8, device=offsets.device)
    if ws is None:
        ws = alloc_learned_workspace(n, offsets.device)
    _check(lib.husky_learned_fit(_coder(coder), _ptr(elems), _ptr(offsets), n,
                                 ctypes.byref(params) if params else None, _ptr(model),
                                 model.numel(), _ptr(ws), ws.numel(), _stream(stream)),
           "husky_learned_fit")
    return model


def learned_header(model) -> dict:
    """Header of a fitted model (synchronizes)."""
    raw = model[:ctypes.sizeof(LearnedHeader)].cpu().numpy().tobytes()
    h = LearnedHeader.from_buffer_copy(raw)
    return {f: getattr(h, f) for f, _ in LearnedHeader._fields_ if f != "pad"}


def learned_part(model, part, dtype, count):
    """A view of one part of the model buffer as a typed device tensor."""
    torch = _torch()
    off = learned_offset(part)
    size = torch.empty(0, dtype=dtype).element_size()
    return model[off:off + count * size].view(dtype)


def sort_learned(elems, offsets, model, coder="ascii7", tuning: Optional[Tuning] = None, ws=None,
                 perm=None, stream=None, check_status=True):
    """Learned-CDF form: the same stable permutation as sort(), bucketed by the model."""
    torch = _torch()
    lib = load()
    n = _n_of(offsets)
    if ws is None:
        ws = alloc_learned_workspace(n, offsets.device)
    if perm is None:
        perm = torch.empty(max(n, 1), dtype=torch.int32, device=offsets.device)
    _check(lib.husky_sort_learned(_coder(coder), _ptr(elems), _ptr(offsets), n, _ptr(model),
                                  _ptr(perm), _ptr(ws), ws.numel(),
                                  ctypes.byref(tuning) if tuning else None, _stream(stream)),
           "husky_sort_learned")
    if check_status:
        _raise_on_status(ws, "husky_sort_learned")
    return perm[:n]


def learned_buckets(elems, offsets, model, coder="ascii7", stream=None):
    """Bucket id (int16 storage of uint16[n]) of every string under a fitted model."""
    torch = _torch()
    lib = load()
    n = _n_of(offsets)
    out = torch.empty(max(n, 1), dtype=torch.int16, device=offsets.device)
    _check(lib.husky_learned_buckets(_coder(coder), _ptr(elems), _ptr(offsets), n, _ptr(model),
                                     _ptr(out), None, _stream(stream)), "husky_learned_buckets")
    return out[:n]


def mlp_grad(params, x, y, monotone=True, stream=None):
    """Gradient (float32[NPARAM]) and summed squared error of the network on (x, y)."""
    torch = _torch()
    lib = load()
    count = int(x.numel())
    ws = torch.empty(int(lib.husky_mlp_grad_workspace_bytes(count)), dtype=torch.uint8,
                     device=x.device)
    g = torch.empty(LEARNED_NPARAM + 1, dtype=torch.float32, device=x.device)
    _check(lib.husky_mlp_grad(_ptr(params), _ptr(x), _ptr(y), count, 1 if monotone else 0,
                              _ptr(g), _ptr(ws), ws.numel(), _stream(stream)), "husky_mlp_grad")
    return g[:LEARNED_NPARAM], g[LEARNED_NPARAM]


def learned_eval_lut(model, params=None, mode="monotone", stream=None):
    """The inference kernel alone: the LUT (int32 storage of uint32[2^24 + 1]) of the
    network with raw parameters `params` (float32[NPARAM], default: the model's own)
    over the model's header and dense cells."""
    torch = _torch()
    lib = load()
    if params is None:
        params = learned_part(model, "params", torch.float32, LEARNED_NPARAM)
    m = LEARNED_MODES[mode] if isinstance(mode, str) else int(mode)
    lut = torch.empty(LEARNED_CELLS + 1, dtype=torch.int32, device=model.device)
    ws = torch.empty(int(lib.husky_learned_lut_workspace_bytes()), dtype=torch.uint8,
                     device=model.device)
    _check(lib.husky_learned_eval_lut(_ptr(params), m, _ptr(model), _ptr(lut), _ptr(ws), ws.numel(),
                                      _stream(stream)), "husky_learned_eval_lut")
    return lut


def profile_begin(classes=None):
    """Start per-launch HIP-event timing of the library's kernels (all classes,
    or only the named ones)."""
    mask = 0xFFFFFFFF if classes is None else sum(1 << PROFILE_CLASSES.index(c) for c in classes)
    load().husky_profile_select(mask)
    load().husky_profile_begin()


def profile_end() -> dict:
    """Stop timing; {class: (total_ms, launches)} summed since profile_begin."""
    k = len(PROFILE_CLASSES)
    ms = np.zeros(k, dtype=np.float64)
    cnt = np.zeros(k, dtype=np.uint32)
    _check(load().husky_profile_end(ms.ctypes.data, cnt.ctypes.data, k), "husky_profile_end")
    return {c: (float(ms[i]), int(cnt[i])) for i, c in enumerate(PROFILE_CLASSES)}


def status_string(code: int) -> str:
    return load().husky_status_string(int(code)).decode()
