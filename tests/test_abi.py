"""The C ABI on the host (no GPU needed): libhusky.so loads, exports every
function include/husky.h declares, and rejects bad arguments synchronously,
before any device work."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "husky.h")


@pytest.fixture(scope="module")
def lib():
    import paper_2012_00866_amd as husky

    if not os.path.exists(husky.LIB_PATH):
        from paper_2012_00866_amd import build

        build.build()
    return husky.load()


def _declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"\b(husky_[a-z_]+)\s*\(", text)))


def test_every_declared_symbol_is_exported(lib):
    names = _declared()
    assert "husky_sort" in names and "husky_fixup" in names and "husky_check_perm" in names
    for name in names:
        assert hasattr(lib, name), name


def test_binding_lists_every_export():
    import paper_2012_00866_amd as husky

    assert sorted(husky.EXPORTS) == _declared()


def test_workspace_bytes(lib):
    a = lib.husky_workspace_bytes(1000, 1)
    b = lib.husky_workspace_bytes(1 << 20, 1)
    c = lib.husky_workspace_bytes(1 << 20, 4096)
    assert 0 < a < b <= c
    assert b < 80 * (1 << 20)  # about 50 bytes per string


def test_status_strings(lib):
    for code in range(6):
        assert lib.husky_status_string(code)


def test_argument_errors_are_synchronous(lib):
    import paper_2012_00866_amd as husky

    vp = ctypes.c_void_p
    dummy = vp(256)  # never dereferenced: every call below fails its host checks
    t = husky.make_tuning()
    # bad coder
    assert lib.husky_sort(7, dummy, dummy, 10, dummy, dummy, 1 << 30, ctypes.byref(t), None) == 1
    # n >= 2^32
    assert lib.husky_sort(0, dummy, dummy, 1 << 32, dummy, dummy, 1 << 30, ctypes.byref(t), None) == 1
    # null input pointers with n > 0
    assert lib.husky_sort(0, None, dummy, 10, dummy, dummy, 1 << 30, ctypes.byref(t), None) == 1
    # missing / small / misaligned workspace
    assert lib.husky_sort(0, dummy, dummy, 10, dummy, None, 0, ctypes.byref(t), None) == 3
    assert lib.husky_sort(0, dummy, dummy, 1000, dummy, dummy, 16, ctypes.byref(t), None) == 3
    assert lib.husky_sort(0, dummy, dummy, 10, dummy, vp(257), 1 << 30, ctypes.byref(t), None) == 3
    # bad bit range
    assert lib.husky_sort_pairs(dummy, dummy, 10, 40, 40, dummy, 1 << 30, None, None) == 1
    assert lib.husky_sort_pairs(dummy, dummy, 10, 0, 65, dummy, 1 << 30, None, None) == 1
    # unsupported tuning
    for bad in (husky.make_tuning(radix_bits=5), husky.make_tuning(tile_items=10),
                husky.make_tuning(t_small=65), husky.make_tuning(t_medium=8192),
                husky.make_tuning(t_small=64, t_medium=64), husky.make_tuning(max_rounds=5000)):
        assert lib.husky_sort(0, dummy, dummy, 10, dummy, dummy, 1 << 30, ctypes.byref(bad), None) == 5
    # batched needs instance offsets
    assert lib.husky_sort_batched(0, dummy, dummy, 10, None, 1, dummy, dummy, 1 << 30, None, None) == 1
    # checker needs an output
    assert lib.husky_check_perm(0, dummy, dummy, 10, None, 1, dummy, dummy, 64, None, None) == 1


def test_bench_refuses_several_gpus():
    # one GPU per measurement: any other --gpus value exits with status 2 and
    # says so, before touching a device
    import subprocess
    import sys

    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr
    assert r.stdout.strip() == ""
