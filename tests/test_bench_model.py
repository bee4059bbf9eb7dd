"""bench.py's algorithmic byte models (host logic, CPU only)."""

import importlib.util
import os

from workloads import config_problem

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_csr_product_bytes():
    b = _bench()
    # 10 nonzeros, float values, 16-bit column indices (5 columns):
    # 10 * (4 + 2) + 4 * (3 + 1) + 4 * 5 + 4 * 3
    assert b.csr_spmv_bytes(10, 3, 5, 4, 4) == 60 + 16 + 20 + 12
    # 70000 columns do not fit 16 bits: 32-bit indices
    assert b.csr_spmv_bytes(10, 3, 70000, 4, 4) == 80 + 16 + 4 * 70000 + 12
    # the boundary: 65536 columns (indices 0..65535) still fit
    assert b.csr_spmv_bytes(10, 3, 65536, 4, 4) == 60 + 16 + 4 * 65536 + 12


def test_recurrence_bytes_of_the_tomography_workload():
    """The per-launch figure the roofline and the profiles quote."""
    b = _bench()
    prob = config_problem("tomo128")
    assert prob.nnz == 7043164
    total = b.recurrence_bytes(prob, 100, 4, 4)
    assert total // 201 == 47449760


def test_vjp_bytes_grows_quadratically():
    b = _bench()
    m = n = 1 << 18
    small, big = b.vjp_bytes(m, n, 20, 4), b.vjp_bytes(m, n, 40, 4)
    # the adjoint updates dominate: about 5 column passes per k, summed over k
    assert 3.0 < big / small < 4.2


def test_equal_error_comparison():
    """The mixed-vs-FP64 comparison: the target is 1.02 x FP64's smallest
    error, each mode's first k at or below it is timed, and "equal" needs
    |e_p - e_64| <= 0.02 e_64 at the compared point."""
    import numpy as np
    b = _bench()
    e64 = np.array([0.9, 0.5, 0.30, 0.20, 0.21, 0.25])
    e32 = np.array([0.9, 0.5, 0.31, 0.203, 0.22, 0.255])   # reaches 0.204 at k = 4
    ebf = np.array([0.9, 0.6, 0.40, 0.35, 0.36, 0.38])     # never within 2 %
    mk = lambda e, ips, ks: dict(errs=e, iters_per_s=ips, ms=1000.0 / ips * len(e),
                                 info={"k_stop": ks}, time_k=lambda k: 2.0 * k)
    res = {"fp64": mk(e64, 100.0, 4), "fp32": mk(e32, 150.0, 4), "bf16op": mk(ebf, 200.0, 5)}
    out = b.equal_error(res)
    assert np.isclose(out["target_rel_err"], 0.204)
    assert out["fp64"]["k_target"] == 4 and out["fp32"]["k_target"] == 4
    assert out["bf16op"]["k_target"] is None and out["bf16op"]["ms_to_target"] is None
    assert out["fp32"]["speedup_iters_per_s"] == 1.5
    assert out["fp32"]["speedup_to_target"] == 1.0
    assert out["fp32"]["equal_at_target"] and out["fp32"]["equal_at_k_stop"]
    assert not out["fp32"]["equal_at_K"]           # 0.255 vs 0.25: 2 % is 0.005
    assert not out["bf16op"]["equal_at_target"] and not out["bf16op"]["equal_at_k_stop"]
    assert out["bf16op"]["rel_err_at_k_stop"] == 0.36 and out["fp64"]["rel_err_at_k_stop"] == 0.20
