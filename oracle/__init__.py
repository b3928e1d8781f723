"""Huskysort CPU oracle -- test infrastructure only.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It never touches the HIP library and the
HIP library never touches it; the two share nothing but the seeded input
generators in ``workloads``.

The string oracle lives in ``husky_oracle.cpp`` (plain single-threaded C++,
loaded through ctypes); the learned-CDF oracle (float64 MLP) lives in
``learned.py``.  Coder ids: 0 = ASCII 7-bit x 9, 1 = UTF-16 16-bit x 4
(unsigned), 2 = UTF-16 as printed in the paper (shifted right one bit),
3 = null coder (every code 0), 4 = full bytes (8 x 8 bits, any byte value).
"""

from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "husky_oracle.cpp")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

CODERS = {"ascii7": 0, "utf16": 1, "utf16_paper": 2, "null": 3, "bytes8": 4}


def build(force: bool = True) -> str:
    """Compile the C++ oracle with g++ into oracle/liboracle.so."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["g++", "-O2", "-std=c++17", "-shared", "-fPIC", _SRC, "-o", tmp])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
            build()
        lib = ctypes.CDLL(_LIB_PATH)
        u64, i32, vp = ctypes.c_uint64, ctypes.c_int, ctypes.c_void_p
        lib.oracle_encode.restype = u64
        lib.oracle_encode.argtypes = [i32, vp, vp, u64, vp]
        lib.oracle_sort_pairs.restype = None
        lib.oracle_sort_pairs.argtypes = [vp, vp, u64]
        lib.oracle_fixup.restype = None
        lib.oracle_fixup.argtypes = [i32, vp, vp, u64, vp, vp]
        lib.oracle_sort.restype = u64
        lib.oracle_sort.argtypes = [i32, i32, vp, vp, u64, vp]
        lib.oracle_sort_batched.restype = u64
        lib.oracle_sort_batched.argtypes = [i32, i32, vp, vp, vp, u64, vp]
        lib.oracle_fixup_global.restype = None
        lib.oracle_fixup_global.argtypes = [i32, vp, vp, u64, vp]
        lib.oracle_sort_lossy.restype = None
        lib.oracle_sort_lossy.argtypes = [i32, vp, vp, u64, vp, vp]
        lib.oracle_check_perm.restype = u64
        lib.oracle_check_perm.argtypes = [i32, vp, vp, u64, vp, vp]
        lib.oracle_check_perm_batched.restype = u64
        lib.oracle_check_perm_batched.argtypes = [i32, vp, vp, vp, u64, vp, vp]
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _coder_id(batch, coder):
    c = coder if coder is not None else batch.coder
    return CODERS[c] if isinstance(c, str) else int(c)


def _prep(batch):
    elems = np.ascontiguousarray(batch.elems)
    offsets = np.ascontiguousarray(batch.offsets, dtype=np.uint64)
    if elems.size == 0:  # keep a valid pointer for empty inputs
        elems = np.zeros(1, dtype=batch.elems.dtype)
    return elems, offsets


def encode(batch, coder=None):
    """Step 1: codes uint64[n] and the count of out-of-domain ASCII strings."""
    lib = _load()
    elems, offsets = _prep(batch)
    codes = np.zeros(max(batch.n, 1), dtype=np.uint64)
    bad = lib.oracle_encode(_coder_id(batch, coder), _ptr(elems), _ptr(offsets), batch.n, _ptr(codes))
    return codes[: batch.n], int(bad)


def sort_pairs(codes: np.ndarray, idx: np.ndarray):
    """Step 2: stable sort of (code, idx) by code; returns new arrays."""
    lib = _load()
    c = np.array(codes, dtype=np.uint64, copy=True)
    i = np.array(idx, dtype=np.uint32, copy=True)
    if c.size:
        lib.oracle_sort_pairs(_ptr(c), _ptr(i), c.size)
    return c, i


def fixup(batch, sorted_codes: np.ndarray, idx: np.ndarray) -> np.ndarray:
    """Step 3: re-sort runs of equal codes with the full comparator; returns new idx."""
    lib = _load()
    elems, offsets = _prep(batch)
    c = np.ascontiguousarray(sorted_codes, dtype=np.uint64)
    i = np.array(idx, dtype=np.uint32, copy=True)
    if i.size:
        lib.oracle_fixup(batch.elem_bytes, _ptr(elems), _ptr(offsets), i.size, _ptr(c), _ptr(i))
    return i


def sort(batch, coder=None):
    """Algorithm 1 end to end: (perm uint32[n], domain-violation count)."""
    lib = _load()
    elems, offsets = _prep(batch)
    perm = np.zeros(max(batch.n, 1), dtype=np.uint32)
    bad = lib.oracle_sort(_coder_id(batch, coder), batch.elem_bytes, _ptr(elems), _ptr(offsets),
                          batch.n, _ptr(perm))
    return perm[: batch.n], int(bad)


def fixup_global(batch, idx: np.ndarray) -> np.ndarray:
    """Step 3 as a full stable pass: any order idx -> the stable sorting permutation."""
    lib = _load()
    elems, offsets = _prep(batch)
    i = np.array(idx, dtype=np.uint32, copy=True)
    if i.size:
        lib.oracle_fixup_global(batch.elem_bytes, _ptr(elems), _ptr(offsets), i.size, _ptr(i))
    return i


def sort_lossy(batch, codes: np.ndarray) -> np.ndarray:
    """Algorithm 1 with the given codes (any coder, even one that inverts strings):
    stable sort by code, then the full stable pass."""
    lib = _load()
    elems, offsets = _prep(batch)
    c = np.ascontiguousarray(codes, dtype=np.uint64)
    perm = np.zeros(max(batch.n, 1), dtype=np.uint32)
    if batch.n:
        lib.oracle_sort_lossy(batch.elem_bytes, _ptr(elems), _ptr(offsets), batch.n, _ptr(c), _ptr(perm))
    return perm[: batch.n]


def sort_batched(batch, coder=None):
    """Every instance of a batched workload sorted on its own (global indices)."""
    lib = _load()
    elems, offsets = _prep(batch)
    seg = np.ascontiguousarray(batch.seg_offsets, dtype=np.uint64)
    perm = np.zeros(max(batch.n, 1), dtype=np.uint32)
    bad = lib.oracle_sort_batched(_coder_id(batch, coder), batch.elem_bytes, _ptr(elems),
                                  _ptr(offsets), _ptr(seg), seg.size - 1, _ptr(perm))
    return perm[: batch.n], int(bad)


def check_perm(batch, perm: np.ndarray):
    """(violations, first bad position): zero violations <=> perm is the stable sort."""
    lib = _load()
    elems, offsets = _prep(batch)
    p = np.ascontiguousarray(perm, dtype=np.uint32)
    first = np.zeros(1, dtype=np.uint64)
    bad = lib.oracle_check_perm(batch.elem_bytes, _ptr(elems), _ptr(offsets), batch.n,
                                _ptr(p if p.size else np.zeros(1, np.uint32)), _ptr(first))
    return int(bad), int(first[0])


def check_perm_batched(batch, perm: np.ndarray):
    """(violations, first bad position) of a batched permutation, instance by instance."""
    lib = _load()
    elems, offsets = _prep(batch)
    seg = np.ascontiguousarray(batch.seg_offsets, dtype=np.uint64)
    p = np.ascontiguousarray(perm, dtype=np.uint32)
    first = np.zeros(1, dtype=np.uint64)
    bad = lib.oracle_check_perm_batched(batch.elem_bytes, _ptr(elems), _ptr(offsets), _ptr(seg),
                                        seg.size - 1, _ptr(p if p.size else np.zeros(1, np.uint32)),
                                        _ptr(first))
    return int(bad), int(first[0])
