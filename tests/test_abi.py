"""The C ABI library loads and exports every symbol declared in include/*.h
(CPU only: no call here reaches the device)."""
import ctypes
import glob
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        src = open(h).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        names |= set(re.findall(r"\b(chebfilter_\w+)\s*\(", src))
    return sorted(names)


def test_header_declares_the_entry_points():
    names = _declared()
    for n in ("chebfilter_init", "chebfilter_apply_H", "chebfilter_apply_M",
              "chebfilter_apply_Sinv", "chebfilter_filter", "chebfilter_cholqr",
              "chebfilter_rayleigh_ritz", "chebfilter_lanczos_bounds", "chebfilter_destroy"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_1610_02121_amd.binding import LIB_PATH, EXPORTS, load_library
    if not os.path.exists(LIB_PATH):
        pytest.fail("libchebfilter.so is not built (run __graft_entry__.build())")
    lib = load_library()
    for n in _declared():
        assert hasattr(lib, n), n
    assert sorted(EXPORTS) == _declared()
    out = subprocess.run(["nm", "-D", "--defined-only", LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r" T (chebfilter_\w+)", out))
    assert set(_declared()) <= exported


def test_null_arguments_are_rejected_without_device_work():
    from paper_1610_02121_amd.binding import load_library
    lib = load_library()
    h = ctypes.c_void_p()
    assert lib.chebfilter_init(None, None, ctypes.byref(h)) == 1          # CF_EINVAL
    assert h.value is None
    assert b"null" in lib.chebfilter_last_error(None)
    assert lib.chebfilter_destroy(None) == 0
    assert lib.chebfilter_apply_H(None, None, 0, None, 0, 0) == 1
