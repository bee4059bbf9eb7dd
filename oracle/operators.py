"""Forward models in FP64 (test infrastructure; see the package docstring).

The method only ever touches ``A`` through ``A v`` and ``A^T w`` (Section 1:
"matrix-free"; Algorithm 5 uses one product with each per iteration).  Each
class here exposes ``matvec`` (``A x``) and ``rmatvec`` (``A^T y``) in float64
through a library primitive.

PSF convention (zero boundary, output the same size as the image, PSF of odd
size ``ph x pw`` centred at ``(ph//2, pw//2)``):

    (A x)[i, j]   = sum_{a,b} P[a, b] * x[i - a + ph//2, j - b + pw//2]
    (A^T y)[i, j] = sum_{a,b} P[a, b] * y[i + a - ph//2, j + b - pw//2]

with out-of-range image entries read as zero.  ``A`` is a convolution and
``A^T`` the matching correlation; the CPU tests pin both against a dense matrix
built entry by entry from these formulas.
"""

from __future__ import annotations

import numpy as np
import scipy.ndimage
import scipy.sparse


class DenseOp:
    def __init__(self, A):
        self.A = np.ascontiguousarray(np.asarray(A, dtype=np.float64))
        self.shape = self.A.shape

    def matvec(self, x):
        return self.A @ np.asarray(x, dtype=np.float64)

    def rmatvec(self, y):
        return self.A.T @ np.asarray(y, dtype=np.float64)

    def todense(self):
        return self.A.copy()


class CsrOp:
    def __init__(self, m, n, indptr, indices, data):
        self.S = scipy.sparse.csr_matrix(
            (np.asarray(data, dtype=np.float64), np.asarray(indices),
             np.asarray(indptr)), shape=(m, n))
        self.ST = self.S.T.tocsr()
        self.shape = (m, n)

    def matvec(self, x):
        return self.S @ np.asarray(x, dtype=np.float64)

    def rmatvec(self, y):
        return self.ST @ np.asarray(y, dtype=np.float64)

    def todense(self):
        return self.S.toarray()


class PsfOp:
    def __init__(self, psf, image_shape):
        self.P = np.asarray(psf, dtype=np.float64)
        ph, pw = self.P.shape
        if ph % 2 == 0 or pw % 2 == 0:
            raise ValueError("PSF sizes must be odd")
        self.image_shape = tuple(image_shape)
        n = self.image_shape[0] * self.image_shape[1]
        self.shape = (n, n)

    def matvec(self, x):
        img = np.asarray(x, dtype=np.float64).reshape(self.image_shape)
        out = scipy.ndimage.convolve(img, self.P, mode="constant", cval=0.0)
        return out.reshape(-1)

    def rmatvec(self, y):
        img = np.asarray(y, dtype=np.float64).reshape(self.image_shape)
        out = scipy.ndimage.correlate(img, self.P, mode="constant", cval=0.0)
        return out.reshape(-1)


def make_operator(problem):
    """Build the oracle's operator for a ``workloads.Problem``."""
    if problem.kind == "dense":
        return DenseOp(problem.A)
    if problem.kind == "csr":
        return CsrOp(problem.m, problem.n, problem.indptr, problem.indices,
                     problem.data)
    if problem.kind == "psf":
        return PsfOp(problem.psf, problem.image_shape)
    raise ValueError(problem.kind)
