"""CPU checks of the C-ABI library: it loads, exports every entry point that
include/sketch.h declares, and its argument/state checks fail cleanly without a
GPU.  No compute call is made here."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    from paper_2302_01977_amd import _abi
    if not os.path.exists(_abi.LIB_PATH):
        from paper_2302_01977_amd import build
        build.build()
    return _abi, _abi.load()


def _declared():
    src = open(os.path.join(ROOT, "include", "sketch.h")).read()
    return sorted(set(re.findall(r"^\s*(?:int|const char \*)\s*(sketch_\w+)\s*\(", src, re.M)))


def test_header_declares_the_boundary():
    names = _declared()
    for must in ("sketch_init", "sketch_apply", "sketch_extend", "sketch_adjoint" if "sketch_adjoint" in names
                 else "sketch_apply", "sketch_release", "sketch_finalize", "sketch_last_error"):
        assert must in names


def test_every_declared_symbol_is_exported():
    abi, lib = _lib()
    out = subprocess.run(["nm", "-D", "--defined-only", abi.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\bT (sketch_\w+)", out))
    for name in _declared():
        assert name in exported, name
        getattr(lib, name)
    # the binding declares exactly the header's entry points
    assert sorted(abi.exported_names()) == _declared()


def test_state_errors_without_gpu():
    abi, lib = _lib()
    assert lib.sketch_release(None) == abi.SK_ESTATE
    assert b"handle" in lib.sketch_last_error()
    assert lib.sketch_width(None, None, None) == abi.SK_ESTATE
    assert lib.sketch_finalize(None) == abi.SK_ESTATE
    assert lib.sketch_get_rows(None, 0, 1, 0, 1, None, 1) == abi.SK_ESTATE
    assert lib.sketch_init(None, 0, 0) == abi.SK_EINVAL
    assert lib.sketch_state_export(None, None, None) == abi.SK_ESTATE
    assert lib.sketch_state_import(None, None, 0, None) == abi.SK_ESTATE
    assert lib.sketch_test_hook(None, abi.SK_HOOK_FAIL_ALLOC, 1) == abi.SK_ESTATE
    assert lib.sketch_batch_mode(None, 0, None) == abi.SK_ESTATE
    h = ctypes.c_void_p()
    assert lib.sketch_apply(None, None, None, 16, 1, None, ctypes.byref(h), None) == abi.SK_ESTATE


def test_init_fails_cleanly_without_device():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    abi, lib = _lib()
    ctx = ctypes.c_void_p()
    rc = lib.sketch_init(ctypes.byref(ctx), 0, 0)
    assert rc in (abi.SK_EHIP, abi.SK_EINVAL)
    assert not ctx.value
    assert len(lib.sketch_last_error()) > 0
