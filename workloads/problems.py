"""Synthetic problem generators.

Every generator is deterministic in its seed: ``x_true`` is drawn with
``numpy.random.default_rng(seed)`` and the noise with ``default_rng(seed + 1)``.
Noise follows the paper's definition of the noise level (Section 4):
``e = nu * ||A x_true|| * z / ||z||`` with ``z ~ N(0, I_m)``, so that
``||e|| / ||A x_true|| = nu`` exactly (up to rounding).

The three operator families are the ones the paper's problem statement allows
(a matrix-free ``A`` and ``A^T``, Section 1):

* ``dense``  -- a row-major ``m x n`` float64 matrix;
* ``csr``    -- a sparse ray-sum matrix (``indptr`` int64, ``indices`` int32
  sorted within each row, ``data`` float64);
* ``psf``    -- a 2-D point-spread function applied as a zero-boundary,
  same-size convolution of an image stored row-major.

These are stand-ins for the IR Tools test problems of Section 4 (PRtomo and
friends), which are not available here: the tomography generator mirrors
PRtomo's parallel-beam geometry (angles x detector bins), the deblurring
generators use Gaussian PSFs.
"""

from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np
import scipy.ndimage
import scipy.sparse


@dataclasses.dataclass
class Problem:
    """One inverse problem ``b = A x_true + e`` and the data defining ``A``."""

    name: str
    kind: str  # "dense" | "csr" | "psf"
    m: int
    n: int
    x_true: np.ndarray
    b: np.ndarray
    noise_level: float
    A: Optional[np.ndarray] = None  # dense, (m, n) row-major float64
    indptr: Optional[np.ndarray] = None  # csr, (m+1,) int64
    indices: Optional[np.ndarray] = None  # csr, (nnz,) int32
    data: Optional[np.ndarray] = None  # csr, (nnz,) float64
    psf: Optional[np.ndarray] = None  # psf, (ph, pw) float64, odd sizes
    image_shape: Optional[tuple] = None  # psf / tomography image (rows, cols)
    meta: dict = dataclasses.field(default_factory=dict)

    @property
    def nnz(self) -> int:
        return int(self.indptr[-1]) if self.indptr is not None else 0

    def forward(self, x: np.ndarray) -> np.ndarray:
        """``A x`` in float64 -- used only to make the data ``b``."""
        return _forward(self.kind, x, A=self.A, indptr=self.indptr,
                        indices=self.indices, data=self.data, psf=self.psf,
                        image_shape=self.image_shape, m=self.m, n=self.n)


def _forward(kind, x, *, A=None, indptr=None, indices=None, data=None,
             psf=None, image_shape=None, m=None, n=None):
    x = np.asarray(x, dtype=np.float64)
    if kind == "dense":
        return A @ x
    if kind == "csr":
        S = scipy.sparse.csr_matrix((data, indices, indptr), shape=(m, n))
        return S @ x
    if kind == "psf":
        img = x.reshape(image_shape)
        out = scipy.ndimage.convolve(img, psf, mode="constant", cval=0.0)
        return out.reshape(-1)
    raise ValueError(kind)


def _add_noise(Ax: np.ndarray, nu: float, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed + 1)
    z = rng.standard_normal(Ax.shape[0])
    return Ax + nu * np.linalg.norm(Ax) * z / np.linalg.norm(z)


# ---------------------------------------------------------------------------
# 1-D deblurring with a dense Gaussian Toeplitz matrix
# ---------------------------------------------------------------------------

def dense_blur_1d(n: int = 256, width: float = 3.0, nu: float = 0.01,
                  seed: int = 1000) -> Problem:
    """Dense ``n x n`` Gaussian blur, ``a_ij = exp(-(i-j)^2 / (2 width^2))``,
    each row scaled to sum 1 (so ``A`` is not symmetric).  ``x_true`` on the
    grid ``s_i = (i + 1/2)/n`` is three boxes plus two Gaussian bumps."""
    i = np.arange(n, dtype=np.float64)
    A = np.exp(-((i[:, None] - i[None, :]) ** 2) / (2.0 * width * width))
    A /= A.sum(axis=1, keepdims=True)
    rng = np.random.default_rng(seed)
    s = (i + 0.5) / n
    x = np.zeros(n)
    for _ in range(3):
        start = rng.uniform(0.05, 0.75)
        w = rng.uniform(0.05, 0.2)
        h = rng.uniform(0.2, 1.0)
        x += h * ((s >= start) & (s < start + w))
    for _ in range(2):
        c = rng.uniform(0.1, 0.9)
        sd = rng.uniform(0.02, 0.08)
        amp = rng.uniform(0.2, 1.0)
        x += amp * np.exp(-0.5 * ((s - c) / sd) ** 2)
    A = np.ascontiguousarray(A)
    b = _add_noise(A @ x, nu, seed)
    return Problem(name=f"dense_blur_{n}", kind="dense", m=n, n=n, x_true=x,
                   b=b, noise_level=nu, A=A, meta=dict(width=width, seed=seed))


# ---------------------------------------------------------------------------
# Parallel-beam tomography with bilinear ray-length weights
# ---------------------------------------------------------------------------

def ray_matrix(side: int, n_angles: int, n_bins: int, dtau: float = 0.5):
    """Sparse parallel-beam ray-sum matrix for a ``side x side`` image.

    Pixel ``(r, c)`` (row-major column index ``r*side + c``) has its centre at
    ``(c + 1/2 - side/2, r + 1/2 - side/2)``.  Ray ``(a, bin)`` has direction
    angle ``theta_a = a*pi/n_angles`` and signed offset
    ``s = bin - (n_bins - 1)/2`` from the image centre; it is sampled every
    ``dtau`` pixels along its length and each sample adds ``dtau`` times its
    bilinear interpolation weights to the four surrounding pixel centres.
    Duplicate entries are summed; column indices are sorted per row; exact
    zeros are dropped.  Row index is ``a*n_bins + bin``.
    """
    half = side / 2.0
    R = half * math.sqrt(2.0)
    J = int(math.ceil(2.0 * R / dtau))
    tau = -R + (np.arange(J) + 0.5) * dtau
    s = np.arange(n_bins, dtype=np.float64) - (n_bins - 1) / 2.0
    blocks = []
    for a in range(n_angles):
        th = a * math.pi / n_angles
        ct, st = math.cos(th), math.sin(th)
        px = s[:, None] * ct - tau[None, :] * st
        py = s[:, None] * st + tau[None, :] * ct
        u = px + half - 0.5
        v = py + half - 0.5
        c0 = np.floor(u)
        r0 = np.floor(v)
        fu = u - c0
        fv = v - r0
        c0 = c0.astype(np.int64)
        r0 = r0.astype(np.int64)
        rows_l, cols_l, vals_l = [], [], []
        ray = np.broadcast_to(np.arange(n_bins)[:, None], u.shape)
        for dr, dc, w in ((0, 0, (1 - fu) * (1 - fv)), (0, 1, fu * (1 - fv)),
                          (1, 0, (1 - fu) * fv), (1, 1, fu * fv)):
            rr = r0 + dr
            cc = c0 + dc
            ok = (rr >= 0) & (rr < side) & (cc >= 0) & (cc < side) & (w > 0)
            rows_l.append(ray[ok])
            cols_l.append((rr * side + cc)[ok])
            vals_l.append(dtau * w[ok])
        blk = scipy.sparse.coo_matrix(
            (np.concatenate(vals_l),
             (np.concatenate(rows_l), np.concatenate(cols_l))),
            shape=(n_bins, side * side)).tocsr()
        blk.sum_duplicates()
        blocks.append(blk)
    S = scipy.sparse.vstack(blocks, format="csr")
    S.sum_duplicates()
    S.eliminate_zeros()
    S.sort_indices()
    return (S.indptr.astype(np.int64), S.indices.astype(np.int32),
            S.data.astype(np.float64))


def ellipse_phantom(side: int, n_ellipses: int, rng) -> np.ndarray:
    """Sum of ``n_ellipses`` filled ellipses, clipped to [0, 1].  Centres lie
    within radius ``0.7*side/2``; semi-axes ~ U(4, 40) px at side 128 (scaled
    with the side); orientation ~ U(0, pi); intensity ~ U(0, 1)."""
    half = side / 2.0
    scale = side / 128.0
    yy, xx = np.mgrid[0:side, 0:side].astype(np.float64)
    xx = xx + 0.5 - half
    yy = yy + 0.5 - half
    img = np.zeros((side, side))
    for _ in range(n_ellipses):
        rad = 0.7 * half * math.sqrt(rng.uniform())
        phi = rng.uniform(0.0, 2.0 * math.pi)
        cx, cy = rad * math.cos(phi), rad * math.sin(phi)
        ax = rng.uniform(4.0, 40.0) * scale
        ay = rng.uniform(4.0, 40.0) * scale
        ang = rng.uniform(0.0, math.pi)
        inten = rng.uniform(0.0, 1.0)
        ca, sa = math.cos(ang), math.sin(ang)
        xr = (xx - cx) * ca + (yy - cy) * sa
        yr = -(xx - cx) * sa + (yy - cy) * ca
        img += inten * (((xr / ax) ** 2 + (yr / ay) ** 2) <= 1.0)
    return np.clip(img, 0.0, 1.0)


def tomography(side: int = 128, n_angles: int = 180, n_bins: int = 181,
               nu: float = 0.02, seed: int = 1001, n_ellipses: int = 10,
               dtau: float = 0.5) -> Problem:
    """Rectangular tomography problem (``m = n_angles*n_bins``, ``n = side^2``)."""
    indptr, indices, data = ray_matrix(side, n_angles, n_bins, dtau)
    rng = np.random.default_rng(seed)
    x = ellipse_phantom(side, n_ellipses, rng).reshape(-1)
    m, n = n_angles * n_bins, side * side
    S = scipy.sparse.csr_matrix((data, indices, indptr), shape=(m, n))
    b = _add_noise(S @ x, nu, seed)
    return Problem(name=f"tomo_{side}_{n_angles}x{n_bins}", kind="csr", m=m,
                   n=n, x_true=x, b=b, noise_level=nu, indptr=indptr,
                   indices=indices, data=data, image_shape=(side, side),
                   meta=dict(side=side, n_angles=n_angles, n_bins=n_bins,
                             dtau=dtau, seed=seed))


# ---------------------------------------------------------------------------
# 2-D deblurring with a Gaussian PSF
# ---------------------------------------------------------------------------

def gaussian_psf(half_width: int, sigma: float) -> np.ndarray:
    a = np.arange(-half_width, half_width + 1, dtype=np.float64)
    P = np.exp(-(a[:, None] ** 2 + a[None, :] ** 2) / (2.0 * sigma * sigma))
    return P / P.sum()


def blob_phantom(side: int, n_blobs: int, n_rects: int, rng) -> np.ndarray:
    """Piecewise-smooth image: Gaussian blobs (sd ~ U(8, 80) px at side 1024,
    scaled with the side; amplitude ~ U(0.2, 1)) plus axis-aligned rectangles
    carrying linear ramps; clipped to [0, 1]."""
    scale = side / 1024.0
    yy, xx = np.mgrid[0:side, 0:side].astype(np.float64)
    img = np.zeros((side, side))
    for _ in range(n_blobs):
        cx, cy = rng.uniform(0, side), rng.uniform(0, side)
        sd = rng.uniform(8.0, 80.0) * scale
        amp = rng.uniform(0.2, 1.0)
        img += amp * np.exp(-0.5 * (((xx - cx) ** 2 + (yy - cy) ** 2) / (sd * sd)))
    for _ in range(n_rects):
        w = rng.uniform(0.05, 0.3) * side
        h = rng.uniform(0.05, 0.3) * side
        x0 = rng.uniform(0, side - w)
        y0 = rng.uniform(0, side - h)
        v0, v1 = rng.uniform(0.1, 1.0), rng.uniform(0.1, 1.0)
        inside = (xx >= x0) & (xx < x0 + w) & (yy >= y0) & (yy < y0 + h)
        if rng.uniform() < 0.5:
            ramp = v0 + (v1 - v0) * (xx - x0) / w
        else:
            ramp = v0 + (v1 - v0) * (yy - y0) / h
        img += np.where(inside, ramp, 0.0)
    return np.clip(img, 0.0, 1.0)


def psf_deblur(side: int = 1024, half_width: int = 15, sigma: float = 2.5,
               nu: float = 0.01, seed: int = 1002, n_blobs: int = 24,
               n_rects: int = 6, cols: Optional[int] = None) -> Problem:
    """Square (or ``side x cols``) image deblurring, zero boundary, same size."""
    cols = side if cols is None else cols
    P = gaussian_psf(half_width, sigma)
    rng = np.random.default_rng(seed)
    img = blob_phantom(max(side, cols), n_blobs, n_rects, rng)[:side, :cols]
    x = np.ascontiguousarray(img).reshape(-1)
    Ax = scipy.ndimage.convolve(img, P, mode="constant", cval=0.0).reshape(-1)
    b = _add_noise(Ax, nu, seed)
    n = side * cols
    return Problem(name=f"deblur_{side}x{cols}_p{2*half_width+1}", kind="psf",
                   m=n, n=n, x_true=x, b=b, noise_level=nu, psf=P,
                   image_shape=(side, cols),
                   meta=dict(sigma=sigma, half_width=half_width, seed=seed))


# ---------------------------------------------------------------------------
# Small random problems (for the oracle's pins and for edge cases)
# ---------------------------------------------------------------------------

def random_dense(m: int, n: int, seed: int, nu: float = 0.0,
                 integer: bool = False, lo: int = -4, hi: int = 4) -> Problem:
    """Random dense problem.  ``integer=True`` draws integer entries in
    [lo, hi] for ``A`` and ``x_true`` (exact rational arithmetic is then
    possible); the data is then consistent (``nu`` is ignored)."""
    rng = np.random.default_rng(seed)
    if integer:
        A = rng.integers(lo, hi + 1, size=(m, n)).astype(np.float64)
        x = rng.integers(lo, hi + 1, size=n).astype(np.float64)
        b = A @ x
        nu = 0.0
    else:
        A = rng.standard_normal((m, n))
        x = rng.standard_normal(n)
        b = A @ x if nu == 0.0 else _add_noise(A @ x, nu, seed)
    return Problem(name=f"random_{m}x{n}_s{seed}", kind="dense", m=m, n=n,
                   x_true=x, b=b, noise_level=nu, A=np.ascontiguousarray(A),
                   meta=dict(seed=seed, integer=integer))


# ---------------------------------------------------------------------------
# Named workloads
# ---------------------------------------------------------------------------

#: The measured configurations.  ``grid`` is the lambda grid for the projected
#: Tikhonov problem (20 log-spaced points from 1e-4 to 1); ``grid_relative``
#: scales it by the largest singular value of the projected matrix.
CONFIGS = {
    "dense256": dict(make=lambda: dense_blur_1d(256, 3.0, 0.01, 1000),
                     iters=50, precision="fp64", reg="wgcv",
                     grid_relative=False),
    "tomo128": dict(make=lambda: tomography(128, 180, 181, 0.02, 1001),
                    iters=100, precision="fp32", reg="wgcv",
                    grid_relative=True),
    "deblur1024": dict(make=lambda: psf_deblur(1024, 15, 2.5, 0.01, 1002),
                       iters=150, precision="fp64", reg="wgcv",
                       grid_relative=True),
    # A 256 x 256 tomography sibling (180 angles, 362 bins): its CSR pair
    # (about 336 MB in FP32 with 16-bit indices) exceeds the device's 256 MB
    # last-level cache, so its products stream from HBM.
    "tomo256": dict(make=lambda: tomography(256, 180, 362, 0.02, 1201),
                    iters=100, precision="fp32", reg="wgcv",
                    grid_relative=True),
    # The differentiable workload: d ||x_k - x_true||^2 / d (b, lambda) with a
    # fixed lambda (15 x 15 Gaussian PSF, sigma 2).
    "deblur512": dict(make=lambda: psf_deblur(512, 7, 2.0, 0.01, 1005),
                      iters=40, precision="fp32", reg="fixed", lam=0.01,
                      grid_relative=False),
    # Reduced-size siblings used by the parity tests (same recipes).
    "tomo32": dict(make=lambda: tomography(32, 36, 45, 0.02, 1101),
                   iters=30, precision="fp64", reg="wgcv",
                   grid_relative=True),
    "deblur96": dict(make=lambda: psf_deblur(96, 15, 2.5, 0.01, 1102),
                     iters=40, precision="fp64", reg="wgcv",
                     grid_relative=True),
}


def lambda_grid(n_grid: int = 20, lo: float = 1e-4, hi: float = 1.0):
    return np.logspace(math.log10(lo), math.log10(hi), n_grid)


def config_problem(name: str) -> Problem:
    return CONFIGS[name]["make"]()


def pivot_sample_lists(m: int, n: int, K: int, s: int, seed: int = 0) -> np.ndarray:
    """Random candidate rows for the sampled pivot searches of a solve with at
    most K iterations (the variant of Section 2.2 that takes the largest entry
    of a small random sample instead of the infinity norm).

    Search i = 0, 1, ..., 2K resolves, in order: the pivot of r_0 (length m),
    then for k = 1..K the pivot of q (length n) and of u (length m).  Row i of
    the result is a uniformly random sequence of distinct rows of that vector
    (a prefix of a random permutation, drawn from ``default_rng([seed, i])``),
    s + K long, padded with -1 when the vector is shorter.  Taking the first s
    entries that are not earlier pivots gives a sample of s non-pivot rows
    drawn without replacement."""
    L = s + K
    out = np.full((2 * K + 1, L), -1, dtype=np.int32)
    for i in range(2 * K + 1):
        length = m if i % 2 == 0 else n
        rng = np.random.default_rng([seed, i])
        take = min(length, L)
        out[i, :take] = rng.choice(length, size=take, replace=False)
    return out


def batch_problems(count: int, seed: int = 0) -> list:
    """A set of uneven problems for batched solves: alternately a parallel-beam
    tomography problem with side s ~ U{32..96} (s angles, s + 1 bins) and a
    deblurring problem with side ~ U{64..256} and a Gaussian PSF with
    sigma ~ U(1.5, 4) and half-width ceil(3 sigma).  Each problem has its own
    seed."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        if i % 2 == 0:
            side = int(rng.integers(32, 97))
            out.append(tomography(side, side, side + 1, 0.02, seed=seed * 100003 + i))
        else:
            side = int(rng.integers(64, 257))
            sigma = float(rng.uniform(1.5, 4.0))
            out.append(psf_deblur(side, int(math.ceil(3 * sigma)), sigma, 0.01,
                                  seed=seed * 100003 + i))
    return out
