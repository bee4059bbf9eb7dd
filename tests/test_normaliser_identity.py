"""The FP32 normalisation identity the GPU kernels rely on (host check).

Basis vectors are normalised by one pivot value v, element by element, and
the products gather the normalised entries on the fly.  In FP32 the kernels
form RN32(RN64(x * RN64(1/v))) instead of the IEEE quotient RN32(x / v): the
FP64 product has relative error at most 2^-52, and a quotient of two 24-bit
numbers is never a float midpoint and lies at least 2^-49 (relative) from
one, so both round to the same float.  This test checks the identity against
NumPy's IEEE float32 division on random bit patterns (all exponents,
subnormals included), basis-like magnitudes and exact quotients."""

import numpy as np


def _check(u, v):
    u = np.asarray(u, np.float32)
    v = np.asarray(v, np.float32)
    ok = np.isfinite(u) & np.isfinite(v) & (v != 0)
    u, v = u[ok], v[ok]
    with np.errstate(all="ignore"):
        ref = u / v
        fast = (u.astype(np.float64) * (1.0 / v.astype(np.float64))).astype(np.float32)
    fin = np.isfinite(ref)
    diff = (ref.view(np.uint32) != fast.view(np.uint32)) & fin
    assert not diff.any(), (u[diff][:3], v[diff][:3])
    return int(fin.sum())


def test_fp32_quotient_from_fp64_reciprocal():
    rng = np.random.default_rng(11)
    n = 0
    for _ in range(3):
        bits = rng.integers(0, 2**32, (2, 1_000_000), dtype=np.uint64).astype(np.uint32)
        n += _check(bits[0].view(np.float32), bits[1].view(np.float32))
        n += _check(rng.standard_normal(1_000_000) * 10.0 ** rng.integers(-8, 8, 1_000_000),
                    rng.standard_normal(1_000_000) * 10.0 ** rng.integers(-8, 8, 1_000_000))
        v = rng.standard_normal(500_000).astype(np.float32)
        q = rng.standard_normal(500_000).astype(np.float32)
        n += _check((v.astype(np.float64) * q).astype(np.float32), v)
        n += _check(rng.integers(1, 2**24, 500_000).astype(np.float32),
                    rng.integers(1, 2**12, 500_000).astype(np.float32))
    assert n > 5_000_000
