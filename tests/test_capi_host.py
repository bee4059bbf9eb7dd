"""Host-side checks of the C-ABI library: it loads, exports every entry point
declared in include/lslu.h, and its argument validation answers without a GPU
(no device work is started here)."""

import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lslu.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lslu_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def capi():
    from paper_2409_05239_amd import capi
    return capi


def test_header_declares_expected_entry_points(capi):
    assert _declared() == sorted(capi.EXPORTS)


def test_library_exports_every_declared_symbol(capi):
    raw = ctypes.CDLL(capi.LIB_PATH)
    for name in _declared():
        assert hasattr(raw, name), name


def test_abi_version_and_status_names(capi):
    assert capi.lslu_abi_version() == 11
    assert capi.status_name(0) == "LSLU_OK"
    assert capi.status_name(2) == "LSLU_BREAKDOWN_U"
    assert capi.status_name(-4) == "LSLU_ENONFINITE"
    assert capi.status_name(99) == "LSLU_UNKNOWN"


def test_null_context_is_rejected(capi):
    out = ctypes.c_void_p()
    A = np.ones((2, 2))
    st = capi.lib.lslu_op_dense(None, 2, 2, A.ctypes.data_as(
        ctypes.POINTER(ctypes.c_double)), 0, ctypes.byref(out))
    assert st == capi.LSLU_EINVAL
    assert "no context" in capi.lslu_last_error(None)
    assert capi.lib.lslu_solve(None, None, None, None, None, None, None) == capi.LSLU_EINVAL
    assert capi.lib.lslu_destroy(None) == capi.LSLU_OK
    assert capi.lib.lslu_op_destroy(None) == capi.LSLU_OK


def test_create_without_gpu_reports_device_error(capi):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    out = ctypes.c_void_p()
    assert capi.lib.lslu_create(0, None, ctypes.byref(out)) == capi.LSLU_EDEVICE
    assert not out.value



def test_fp8_values_are_e4m3():
    """The E4M3 rounding the tests hold the FP8 operator mode to, against
    the format's definition: every finite code point (8 + m) 2^(e-10) and
    m 2^-9 rounds to itself, midpoints go to the even neighbour, values past
    448 saturate, and half the smallest subnormal ties to zero."""
    import numpy as np
    from gpu_helpers import e4m3

    assert e4m3(1.0) == 1.0 and e4m3(1.0625) == 1.0 and e4m3(1.1875) == 1.25
    assert e4m3(-1.1875) == -1.25 and e4m3(0.0) == 0.0
    assert e4m3(448.0) == 448.0 and e4m3(470.0) == 448.0 and e4m3(1e6) == 448.0
    assert e4m3(2.0 ** -9) == 2.0 ** -9 and e4m3(2.0 ** -10) == 0.0
    assert e4m3(3 * 2.0 ** -10) == 2 * 2.0 ** -9  # tie to even in the subnormals
    vals = np.array([m * 2.0 ** -9 for m in range(8)]
                    + [(8 + m) * 2.0 ** (e - 10) for e in range(1, 16) for m in range(8)
                       if not (e == 15 and m == 7)])
    assert vals.max() == 448.0 and len(vals) == 127
    assert np.array_equal(e4m3(vals), vals) and np.array_equal(e4m3(-vals), -vals)
    # midpoints between neighbours round to the one with an even last bit
    mids = (vals[1:] + vals[:-1]) / 2
    r = e4m3(mids)
    idx = np.searchsorted(vals, r)
    assert np.all(vals[idx] == r) and np.all((idx % 2 == 0) | (idx == len(vals) - 1))
