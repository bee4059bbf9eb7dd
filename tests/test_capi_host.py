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
    assert capi.lslu_abi_version() == 13
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


class _FakeDeviceTensor:
    """The attributes the binding's argument checks read from a torch CUDA
    tensor, without a GPU (the checks run before any pointer crosses the C
    ABI)."""

    def __init__(self, numel, dtype, device=0, contiguous=True, cuda=True):
        import types
        self._n, self.dtype, self._c = numel, dtype, contiguous
        self.is_cuda = cuda
        self.device = types.SimpleNamespace(index=device)

    def numel(self):
        return self._n

    def is_contiguous(self):
        return self._c

    def data_ptr(self):
        return 0x1000


def test_device_vector_checks(capi):
    import torch
    F = _FakeDeviceTensor
    f32, f64 = torch.float32, torch.float64
    assert capi._vec(F(10, f32), 10, capi.LSLU_FP32, "b", 0).value == 0x1000
    assert capi._vec(F(10, f64), 10, capi.LSLU_FP64, "b", None).value == 0x1000
    assert capi._vec(F(12, f32), 10, capi.LSLU_BF16OP, "X", 0, at_least=True).value
    bad = [
        (F(10, f32, cuda=False), 10, capi.LSLU_FP32, {}, "CUDA tensor"),
        (torch.zeros(10), 10, capi.LSLU_FP32, {}, "CUDA tensor"),
        (F(10, f32), 10, capi.LSLU_FP64, {}, "float64"),
        (F(10, f64), 10, capi.LSLU_FP8OP, {}, "float32"),
        (F(10, f32, contiguous=False), 10, capi.LSLU_FP32, {}, "contiguous"),
        (F(9, f32), 10, capi.LSLU_FP32, {}, "10 entries"),
        (F(11, f32), 10, capi.LSLU_FP32, {}, "10 entries"),
        (F(9, f32), 10, capi.LSLU_FP32, {"at_least": True}, "at least 10"),
        (F(10, f32, device=1), 10, capi.LSLU_FP32, {"device": 0}, "cuda:1"),
    ]
    for t, n, prec, kw, msg in bad:
        with pytest.raises(ValueError, match=msg):
            capi._vec(t, n, prec, "v", kw.get("device"), kw.get("at_least", False))
    with pytest.raises(ValueError, match="required"):
        capi._vec(None, 3, capi.LSLU_FP32, "b")
    assert capi._opt_vec(None, 3, capi.LSLU_FP32, "x0") is None


def test_host_array_checks(capi):
    K = 5
    a = capi._host_ints(np.arange(K + 1), K + 1, "replay_piv_t")
    assert a.dtype == np.int32 and a.shape == (K + 1,)
    with pytest.raises(ValueError, match="at least 6"):
        capi._host_ints(np.arange(K), K + 1, "replay_piv_t")
    rows = capi._sample_rows(np.zeros((2 * K + 3, 7), np.int64), K)
    assert rows.shape == (2 * K + 1, 7) and rows.dtype == np.int32 and rows.flags.c_contiguous
    for shape in [(2 * K, 7), (2 * K + 1, 0), (2 * K + 1, 513), (2 * K + 1,)]:
        with pytest.raises(ValueError, match="pivot_sample"):
            capi._sample_rows(np.zeros(shape, np.int32), K)
