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
    # 10 nonzeros, float values: 10 * (4 + 4) + 4 * (3 + 1) + 4 * 5 + 4 * 3
    assert b.csr_spmv_bytes(10, 3, 5, 4, 4) == 80 + 16 + 20 + 12


def test_recurrence_bytes_of_the_tomography_workload():
    """The per-launch figure the roofline and the profiles quote."""
    b = _bench()
    prob = config_problem("tomo128")
    assert prob.nnz == 7043164
    total = b.recurrence_bytes(prob, 100, 4, 4)
    assert total // 201 == 61466007


def test_vjp_bytes_grows_quadratically():
    b = _bench()
    m = n = 1 << 18
    small, big = b.vjp_bytes(m, n, 20, 4), b.vjp_bytes(m, n, 40, 4)
    # the adjoint updates dominate: about 5 column passes per k, summed over k
    assert 3.0 < big / small < 4.2
