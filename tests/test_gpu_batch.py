"""Many problems at once: asynchronous solves on several contexts (one stream
each) against the same solves run one at a time.

Every problem's results must be bit-identical however the solves are
interleaved: the kernels of one solve depend only on that solve's data, and
the waits inside a launch only ever wait for blocks of the same launch that
were dispatched before the waiting block.
"""

import numpy as np
import pytest

from workloads import batch_problems, lambda_grid

pytestmark = pytest.mark.gpu

K = 20


def _prepare(lib, ctxs, probs, prec):
    import torch
    dt = torch.float64 if prec == "fp64" else torch.float32
    items = []
    for i, prob in enumerate(probs):
        c = ctxs[i % len(ctxs)]
        op = lib.make_operator(c, prob, lib.PRECISIONS[prec])
        b = torch.tensor(prob.b, dtype=dt, device="cuda")
        X = torch.zeros((K, prob.n), dtype=dt, device="cuda")
        items.append((c, op, b, X))
    torch.cuda.synchronize()
    return items


def _solve(lib, item, asynchronous=False):
    c, op, b, X = item
    return lib.lslu_solve(c, op, b, K, reg="wgcv", grid=lambda_grid(), grid_relative=True,
                          X=X, asynchronous=asynchronous)


@pytest.mark.parametrize("prec", ["fp32", "bf16op"])
def test_concurrent_solves_match_one_at_a_time(lib, prec):
    import torch
    probs = batch_problems(8, seed=3)
    ctxs = [lib.lslu_create(0) for _ in range(4)]
    try:
        items = _prepare(lib, ctxs, probs, prec)
        print(f"[batch] {prec}: " + ", ".join(p.name for p in probs), flush=True)
        ref = []
        for it in items:  # one at a time, synchronous
            st, x, info = _solve(lib, it)
            ref.append((info, it[3].clone()))
        torch.cuda.synchronize()
        for rep in range(2):  # all contexts busy at once, twice
            out = [None] * len(items)
            for w in range(0, len(items), len(ctxs)):
                wave = list(range(w, min(w + len(ctxs), len(items))))
                pend = {i: _solve(lib, items[i], asynchronous=True) for i in wave}
                for i in wave:
                    st, x, info = lib.lslu_wait(items[i][0], pend[i])
                    out[i] = (info, items[i][3].clone())
            torch.cuda.synchronize()
            for (ri, rX), (oi, oX) in zip(ref, out):
                assert oi["k_done"] == ri["k_done"]
                assert np.array_equal(oi["piv_t"], ri["piv_t"])
                assert np.array_equal(oi["piv_g"], ri["piv_g"])
                assert np.array_equal(oi["H"], ri["H"])
                assert torch.equal(oX, rX)
        for c, op, b, X in items:
            lib.lslu_op_destroy(op)
    finally:
        for c in ctxs:
            lib.lslu_destroy(c)


def test_pending_solve_rules(lib):
    import torch
    probs = batch_problems(2, seed=5)
    c = lib.lslu_create(0)
    try:
        items = _prepare(lib, [c], probs, "fp32")
        # nothing pending: waiting is a no-op
        assert lib.lib.lslu_wait(c) == lib.LSLU_OK
        pend = _solve(lib, items[0], asynchronous=True)
        # a second solve, or a basis copy, while one is pending is refused
        with pytest.raises(lib.LsluError) as ei:
            _solve(lib, items[1])
        assert ei.value.status == lib.LSLU_EINVAL
        dst = torch.zeros((1, probs[0].n), dtype=torch.float32, device="cuda")
        with pytest.raises(lib.LsluError):
            lib.lslu_get_basis(c, 0, 1, dst)
        st, x, info = lib.lslu_wait(c, pend)
        assert info["k_done"] == K
        # timing needs a synchronous solve
        with pytest.raises(lib.LsluError):
            cc, op, b, X = items[1]
            lib.lslu_solve(cc, op, b, K, reg="wgcv", grid=lambda_grid(), grid_relative=True,
                           X=X, asynchronous=True, timing=True)
        for _, op, _, _ in items:
            lib.lslu_op_destroy(op)
    finally:
        lib.lslu_destroy(c)
