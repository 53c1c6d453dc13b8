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
        pytest.fail("libchebfilter.so is not built (run python paper_1610_02121_amd/build.py)")
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


def test_bounds_features_transform():
    """The learned-bounds input transform is host code of the library (no GPU):
    energies relative to the last step's theta_N in units of its b - theta_N,
    degree / 100, log10 of the residual-type features over that width."""
    import numpy as np
    from paper_1610_02121_amd.binding import ChebFilterError, bounds_features
    rows = [np.array([-5.0, -2.0, -1.0, 9.0, 40.0, 1e-3, 1e-4, 1e-6]),
            np.array([-5.5, -2.5, -1.5, 10.0 - 1.5 + 1.5, 30.0, 2e-2, 5e-4, 0.0])]
    h = np.concatenate(rows)
    x = bounds_features(h)
    thN, w = -1.5, 10.0 + 1.5
    for s, r in enumerate(rows):
        assert np.allclose(x[8 * s:8 * s + 4], (r[:4] - thN) / w)
        assert np.isclose(x[8 * s + 4], r[4] / 100)
        assert np.allclose(x[8 * s + 5:8 * s + 8], np.log10(r[5:] / w + 1e-30))
    bad = h.copy()
    bad[-5] = bad[-6] - 1.0          # b below theta_N in the last step
    with pytest.raises(ChebFilterError):
        bounds_features(bad)


def test_degree_rule_and_step_summary_host_arithmetic():
    """The learned form's degree rule: the smallest m with T_m(|t(theta_w)|)
    >= 100 (checked with the closed-form T_m), capped where the amplification
    of theta_1 over theta_w reaches 1e12, clamped; the step summary's 8
    numbers on a hand-made case."""
    import numpy as np

    from oracle.filters import chebyshev_T
    from paper_1610_02121_amd.binding import degree_rule, step_summary
    a, b = -0.4, 20.0
    t = lambda x: abs((2.0 * x - a - b) / (b - a))          # noqa: E731
    m = degree_rule(-0.45, -0.5, a, b, 100.0, 1, 10000)
    assert chebyshev_T(m, np.array([t(-0.5)]))[0] >= 100.0
    assert chebyshev_T(m - 1, np.array([t(-0.5)]))[0] < 100.0
    # a deep theta_1: the 1e12 cap applies
    mc = degree_rule(-60.0, -0.5, a, b, 100.0, 1, 10000)
    ratio = chebyshev_T(mc, np.array([t(-60.0)]))[0] / chebyshev_T(mc, np.array([t(-0.5)]))[0]
    ratio1 = chebyshev_T(mc + 1, np.array([t(-60.0)]))[0] / chebyshev_T(mc + 1, np.array([t(-0.5)]))[0]
    assert mc < m and ratio <= 1.2e12 and ratio1 > 0.8e12
    assert degree_rule(-0.45, -0.5, a, b, 100.0, 8, 20) == 20
    out = step_summary(np.array([-1.0, -0.5, -0.4, 0.0]), np.array([-1.1, -0.5, -0.4, 0.0]), 2,
                       20.0, 30, np.array([1e-3, 1e-5, 1.0, 1.0]))
    assert np.allclose(out, [-1.0, -0.5, 0.0, 20.0, 30.0, 1e-3, 5.05e-4, 0.1])
