"""ctypes binding of ``include/lslu.h``.

Marshalling only: every function below converts Python arguments (ints,
floats, NumPy host arrays, torch device tensors) into the C ABI's plain
pointers and sizes, calls the entry point of the same name in ``liblslu.so``
and turns a negative status into :class:`LsluError`.  All computation happens
in the library's HIP kernels.  Importing this module fails loudly when the
library has not been built.
"""

from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_double, c_int, c_int32, c_int64, c_void_p

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblslu.so")

LSLU_OK = 0
LSLU_BREAKDOWN_Q = 1
LSLU_BREAKDOWN_U = 2
LSLU_ZERO_RHS = 3
LSLU_EINVAL = -1
LSLU_ENOMEM = -2
LSLU_EDEVICE = -3
LSLU_ENONFINITE = -4
LSLU_EUNSUPPORTED = -5

LSLU_FP64, LSLU_FP32, LSLU_BF16OP, LSLU_FP16OP, LSLU_FP8OP = 0, 1, 2, 3, 4
PRECISIONS = {"fp64": LSLU_FP64, "fp32": LSLU_FP32, "bf16op": LSLU_BF16OP,
              "fp16op": LSLU_FP16OP, "fp8op": LSLU_FP8OP}

LSLU_REG_NONE, LSLU_REG_FIXED, LSLU_REG_WGCV, LSLU_REG_GCV, LSLU_REG_OPTIMAL = range(5)
REGS = {"none": LSLU_REG_NONE, "fixed": LSLU_REG_FIXED, "wgcv": LSLU_REG_WGCV,
        "gcv": LSLU_REG_GCV, "optimal": LSLU_REG_OPTIMAL}

#: Every entry point declared in include/lslu.h.
EXPORTS = (
    "lslu_create", "lslu_destroy", "lslu_last_error", "lslu_status_name",
    "lslu_abi_version", "lslu_op_dense", "lslu_op_csr", "lslu_op_psf",
    "lslu_op_apply", "lslu_op_info", "lslu_op_destroy", "lslu_solve",
    "lslu_wait", "lslu_get_basis", "lslu_vjp", "lslu_op_tile", "lslu_solve_host",
    "lslu_solve_batch", "lslu_solve_static",
)


class lslu_opts(ctypes.Structure):
    _fields_ = [
        ("maxiter", c_int32),
        ("reg", c_int32),
        ("lambda_", c_double),
        ("lambda_grid", POINTER(c_double)),
        ("n_grid", c_int32),
        ("grid_relative", c_int32),
        ("omega", c_double),
        ("x_true_dev", c_void_p),
        ("stop_tol", c_double),
        ("early_stop", c_int32),
        ("X_dev", c_void_p),
        ("replay_piv_t", POINTER(c_int32)),
        ("replay_piv_g", POINTER(c_int32)),
        ("replay_lambda_idx", POINTER(c_int32)),
        ("flags", c_int32),
        ("sample_rows", POINTER(c_int32)),
        ("sample_s", c_int32),
        ("sample_len", c_int32),
    ]


LSLU_FLAG_EAGER = 1
LSLU_FLAG_TIMING = 2
LSLU_FLAG_ASYNC = 4
LSLU_FLAG_GRAD_LAMBDA = 8
LSLU_FLAG_FINAL_ONLY = 16
LSLU_FLAG_PIVOT_SEP = 32


class lslu_result(ctypes.Structure):
    _fields_ = [
        ("status", c_int32),
        ("k_done", c_int32),
        ("k_stop", c_int32),
        ("n_l", c_int32),
        ("n_d", c_int32),
        ("beta", c_double),
        ("piv_t_mismatch", c_int32),
        ("piv_g_mismatch", c_int32),
        ("piv_t", POINTER(c_int32)),
        ("piv_g", POINTER(c_int32)),
        ("own_piv_t", POINTER(c_int32)),
        ("own_piv_g", POINTER(c_int32)),
        ("H", POINTER(c_double)),
        ("W", POINTER(c_double)),
        ("Y", POINTER(c_double)),
        ("lambda_k", POINTER(c_double)),
        ("lambda_idx", POINTER(c_int32)),
        ("ghat", POINTER(c_double)),
        ("sep_lambda", POINTER(c_double)),
        ("sigma_max", POINTER(c_double)),
        ("sigma_min", POINTER(c_double)),
        ("t_recurrence_ms", c_double),
        ("n_recurrence_launches", c_int32),
        ("t_projected_ms", c_double),
        ("t_assemble_ms", c_double),
        ("dloss_dlambda", POINTER(c_double)),
        ("sep_t", POINTER(c_double)),
        ("sep_g", POINTER(c_double)),
    ]


class LsluError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{status_name(status)}: {message}")
        self.status = status


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is missing: build it with "
            "'python -m paper_2409_05239_amd.build' (there is no fallback)")
    # torch's wheel carries its own HIP runtime under a different file name
    # but the same soname.  Loading torch first makes liblslu.so bind to that
    # runtime instance, the one that owns the device tensors passed in;
    # loading liblslu.so first would put a second HIP runtime in the process.
    import torch  # noqa: F401
    lib = ctypes.CDLL(LIB_PATH)
    vp, pp = c_void_p, POINTER(c_void_p)
    sig = {
        "lslu_create": (c_int, [c_int, vp, pp]),
        "lslu_destroy": (c_int, [vp]),
        "lslu_last_error": (ctypes.c_char_p, [vp]),
        "lslu_status_name": (ctypes.c_char_p, [c_int]),
        "lslu_abi_version": (c_int, []),
        "lslu_op_dense": (c_int, [vp, c_int64, c_int64, POINTER(c_double), c_int32, pp]),
        "lslu_op_csr": (c_int, [vp, c_int64, c_int64, c_int64, POINTER(c_int64),
                                POINTER(c_int32), POINTER(c_double), c_int32, pp]),
        "lslu_op_psf": (c_int, [vp, c_int64, c_int64, c_int32, c_int32,
                                POINTER(c_double), c_int32, pp]),
        "lslu_op_apply": (c_int, [vp, vp, c_int32, vp, vp]),
        "lslu_op_info": (c_int, [vp, POINTER(c_int64), POINTER(c_int64), POINTER(c_int32)]),
        "lslu_op_destroy": (c_int, [vp]),
        "lslu_solve": (c_int, [vp, vp, vp, vp, POINTER(lslu_opts), vp,
                               POINTER(lslu_result)]),
        "lslu_solve_static": (c_int, [vp, vp, vp, vp, POINTER(lslu_opts), vp,
                                      POINTER(lslu_result)]),
        "lslu_get_basis": (c_int, [vp, c_int32, c_int32, vp]),
        "lslu_wait": (c_int, [vp]),
        "lslu_vjp": (c_int, [vp, vp, c_int32, vp, vp, POINTER(c_double)]),
        "lslu_op_tile": (c_int, [vp, vp, c_int32, POINTER(c_int32)]),
        "lslu_solve_host": (c_int, [vp, vp, POINTER(c_double), POINTER(c_double),
                                    POINTER(lslu_opts), POINTER(c_double),
                                    POINTER(lslu_result)]),
        "lslu_solve_batch": (c_int, [c_int32, POINTER(c_void_p), POINTER(c_void_p),
                                     POINTER(c_void_p), POINTER(lslu_opts), POINTER(c_void_p),
                                     POINTER(POINTER(lslu_result))]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


lib = _load()


def status_name(status: int) -> str:
    return lib.lslu_status_name(int(status)).decode()


def _check(ctx, status):
    if status < 0:
        msg = lib.lslu_last_error(ctx).decode() if ctx else ""
        raise LsluError(status, msg)
    return status


def _torch_done(dev):
    """Torch's work on its current stream of device ``dev`` (which may still
    be writing the tensors passed in: inputs copied or filled there) must be
    finished before the library's stream runs: the two are not ordered with
    each other."""
    import torch
    torch.cuda.current_stream(0 if dev is None else dev).synchronize()


def _dptr(t):
    return None if t is None else c_void_p(t.data_ptr())


# device of each context made through this binding, and the (m, n, precision)
# of the last solve started on it (what lslu_get_basis copies from)
_CTX_DEVICE = {}
_CTX_SHAPE = {}


def _vec(t, count, precision, name, device=None, at_least=False):
    """Checks a device vector argument before its pointer crosses the C ABI,
    which cannot check it: a contiguous CUDA tensor of the working precision
    (float64 for LSLU_FP64, else float32) holding ``count`` entries (at least
    ``count`` with ``at_least``) on ``device`` (when known).  Returns the
    pointer; raises ValueError otherwise."""
    import torch
    if t is None:
        raise ValueError(f"{name} is required")
    if not getattr(t, "is_cuda", False):
        raise ValueError(f"{name} must be a CUDA tensor")
    want = torch.float64 if precision == LSLU_FP64 else torch.float32
    if t.dtype != want:
        raise ValueError(f"{name} must be {want} for this operator (got {t.dtype})")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    got = t.numel()
    if (got < count) if at_least else (got != count):
        need = f"at least {count}" if at_least else f"{count}"
        raise ValueError(f"{name} must hold {need} entries (got {got})")
    if device is not None and t.device.index != device:
        raise ValueError(f"{name} is on cuda:{t.device.index}, the context on cuda:{device}")
    return c_void_p(t.data_ptr())


def _opt_vec(t, count, precision, name, device=None, at_least=False):
    return None if t is None else _vec(t, count, precision, name, device, at_least)


def _sample_rows(rows, K):
    """Candidate rows of the sampled pivot searches: a 2-D int32 array with
    at least 2 K + 1 rows (the library reads the first 2 K + 1) of 1..512
    entries."""
    rows = np.ascontiguousarray(rows, dtype=np.int32)
    if rows.ndim != 2 or rows.shape[0] < 2 * K + 1 or not 1 <= rows.shape[1] <= 512:
        raise ValueError(f"pivot_sample rows must be (>= {2 * K + 1}) x (1..512), "
                         f"got {rows.shape}")
    return rows[:2 * K + 1]


def _host_ints(arr, min_len, name):
    """A host int32 array argument the library reads ``min_len`` entries of."""
    a = np.ascontiguousarray(arr, dtype=np.int32).reshape(-1)
    if a.shape[0] < min_len:
        raise ValueError(f"{name} must hold at least {min_len} entries (got {a.shape[0]})")
    return a


def _np(a, dtype):
    a = np.ascontiguousarray(a, dtype=dtype)
    return a, a.ctypes.data_as(POINTER(np.ctypeslib.as_ctypes_type(dtype)))


def _torch_dtype(precision):
    import torch
    return torch.float64 if precision == LSLU_FP64 else torch.float32


# ------------------------------------------------------------------ context

def lslu_abi_version() -> int:
    return lib.lslu_abi_version()


def lslu_create(device: int = 0, stream=None):
    """``stream``: a ``torch.cuda.Stream`` (or raw handle); default torch's
    current stream on ``device``."""
    if stream is None:
        import torch
        stream = torch.cuda.current_stream(device)
    handle = getattr(stream, "cuda_stream", stream)
    out = c_void_p()
    st = lib.lslu_create(int(device), c_void_p(handle), ctypes.byref(out))
    if st < 0:
        raise LsluError(st, "lslu_create failed (no gfx950 device?)")
    _CTX_DEVICE[out.value] = int(device)
    return out


def lslu_destroy(ctx):
    _CTX_DEVICE.pop(ctx.value, None)
    _CTX_SHAPE.pop(ctx.value, None)
    return lib.lslu_destroy(ctx)


def lslu_last_error(ctx) -> str:
    return lib.lslu_last_error(ctx).decode()


# ---------------------------------------------------------------- operators

def lslu_op_dense(ctx, A, precision=LSLU_FP64):
    A, pA = _np(A, np.float64)
    m, n = A.shape
    out = c_void_p()
    _check(ctx, lib.lslu_op_dense(ctx, m, n, pA, int(precision), ctypes.byref(out)))
    return out


def lslu_op_csr(ctx, m, n, indptr, indices, data, precision=LSLU_FP64):
    ip, pip = _np(indptr, np.int64)
    ix, pix = _np(indices, np.int32)
    dv, pdv = _np(data, np.float64)
    out = c_void_p()
    _check(ctx, lib.lslu_op_csr(ctx, int(m), int(n), int(ip[-1]), pip, pix, pdv,
                                int(precision), ctypes.byref(out)))
    return out


def lslu_op_psf(ctx, rows, cols, psf, precision=LSLU_FP64):
    P, pP = _np(psf, np.float64)
    ph, pw = P.shape
    out = c_void_p()
    _check(ctx, lib.lslu_op_psf(ctx, int(rows), int(cols), int(ph), int(pw), pP,
                                int(precision), ctypes.byref(out)))
    return out


def lslu_op_apply(ctx, op, transpose, x, y):
    """``x``/``y``: torch device tensors in the operator's working precision
    (n and m entries for A x, m and n for A^T x)."""
    m, n, prec = lslu_op_info(op)
    nin, nout = (m, n) if transpose else (n, m)
    dev = _CTX_DEVICE.get(ctx.value)
    px = _vec(x, nin, prec, "x", dev)
    py = _vec(y, nout, prec, "y", dev)
    _torch_done(dev)
    _check(ctx, lib.lslu_op_apply(ctx, op, int(transpose), px, py))
    # asynchronous on the library's stream: y is complete when this returns
    import torch
    torch.cuda.synchronize(0 if dev is None else dev)


def lslu_op_tile(ctx, op, rows_per_lane=0):
    """Set (2, 4, 8) or measure (0) the tile shape of a PSF operator's
    products; returns the shape in use."""
    r = c_int32(0)
    _check(ctx, lib.lslu_op_tile(ctx, op, int(rows_per_lane), ctypes.byref(r)))
    return r.value


def lslu_op_info(op):
    m, n, p = c_int64(), c_int64(), c_int32()
    _check(None, lib.lslu_op_info(op, ctypes.byref(m), ctypes.byref(n), ctypes.byref(p)))
    return m.value, n.value, p.value


def lslu_op_destroy(op):
    return lib.lslu_op_destroy(op)


def make_operator(ctx, problem, precision=LSLU_FP64):
    """Operator for a ``workloads.Problem``."""
    if problem.kind == "dense":
        return lslu_op_dense(ctx, problem.A, precision)
    if problem.kind == "csr":
        return lslu_op_csr(ctx, problem.m, problem.n, problem.indptr,
                           problem.indices, problem.data, precision)
    if problem.kind == "psf":
        rows, cols = problem.image_shape
        return lslu_op_psf(ctx, rows, cols, problem.psf, precision)
    raise ValueError(problem.kind)


# -------------------------------------------------------------------- solve

def lslu_solve(ctx, op, b, maxiter, reg="none", lam=0.0, grid=None,
               grid_relative=False, omega=0.0, x0=None, x_true=None,
               stop_tol=0.0, early_stop=False, X=None, x_out=None,
               replay_piv_t=None, replay_piv_g=None, replay_lambda_idx=None,
               eager=False, timing=False, pivot_sample=None, asynchronous=False,
               grad_lambda=False, static=False, final_only=False, pivot_sep=False):
    """Run the solver.  ``b``, ``x0``, ``X``, ``x_out`` are torch device
    tensors in the working precision (``x_out`` is allocated when None).
    ``pivot_sample = (rows, s)`` selects sampled pivots: ``rows`` is the
    (2 maxiter + 1) x L int32 array of candidate rows per search.
    ``static=True`` calls ``lslu_solve_static`` (the same solve with its
    device workspace in the library's fixed array: no allocation; device
    vectors only, synchronous).
    ``asynchronous=True`` enqueues the solve and returns a ``Pending``;
    ``lslu_wait(ctx, pending)`` completes it and returns the same triple.
    ``grad_lambda=True`` (needs ``x_true``) adds ``info["dloss_dlambda"]``.
    ``final_only=True`` forms only the returned iterate (no ``X``).
    ``pivot_sep=True`` adds ``info["sep_t"]`` and ``info["sep_g"]``, the
    separation of every pivot search.
    With ``b`` (and ``x0``) given as NumPy arrays the call goes through
    ``lslu_solve_host`` (host arrays in FP64, synchronous) and ``x_out`` is a
    NumPy array.
    Returns ``(status, x_out, info)`` where ``info`` holds the host-side
    results as NumPy arrays."""
    import torch
    m, n, prec = lslu_op_info(op)
    K = int(maxiter)
    host_io = isinstance(b, np.ndarray)
    if host_io and asynchronous:
        raise ValueError("host arrays need a synchronous solve")
    if static and (host_io or asynchronous or timing):
        raise ValueError("lslu_solve_static takes device vectors and is synchronous")
    dev = _CTX_DEVICE.get(ctx.value)
    if not host_io:
        _vec(b, m, prec, "b", dev)
        _opt_vec(x0, n, prec, "x0", dev)
    if x_out is None:
        x_out = (np.empty(n) if host_io
                 else torch.empty(n, dtype=_torch_dtype(prec), device=b.device))
    elif not host_io:
        _vec(x_out, n, prec, "x_out", dev)
    if final_only and X is not None:
        raise ValueError("final_only forms no iterates for X")
    _opt_vec(X, n * K, prec, "X", dev, at_least=True)
    _opt_vec(x_true, n, prec, "x_true", dev)
    o = lslu_opts()
    o.maxiter = K
    o.reg = REGS[reg] if isinstance(reg, str) else int(reg)
    o.lambda_ = float(lam)
    keep = []
    if grid is not None:
        g, pg = _np(np.asarray(grid, dtype=np.float64).reshape(-1), np.float64)
        keep.append(g)
        o.lambda_grid = pg
        o.n_grid = g.shape[0]
    o.grid_relative = 1 if grid_relative else 0
    o.omega = float(omega)
    o.x_true_dev = _dptr(x_true)
    o.stop_tol = float(stop_tol)
    o.early_stop = 1 if early_stop else 0
    o.X_dev = _dptr(X)
    o.flags = ((LSLU_FLAG_EAGER if eager else 0) | (LSLU_FLAG_TIMING if timing else 0)
               | (LSLU_FLAG_ASYNC if asynchronous else 0)
               | (LSLU_FLAG_GRAD_LAMBDA if grad_lambda else 0)
               | (LSLU_FLAG_FINAL_ONLY if final_only else 0)
               | (LSLU_FLAG_PIVOT_SEP if pivot_sep else 0))
    # the library reads K + 1, K and K entries of the replay arrays
    for name, arr, need in (("replay_piv_t", replay_piv_t, K + 1),
                            ("replay_piv_g", replay_piv_g, K),
                            ("replay_lambda_idx", replay_lambda_idx, K)):
        if arr is not None:
            a, pa = _np(_host_ints(arr, need, name), np.int32)
            keep.append(a)
            setattr(o, name, pa)
    if pivot_sample is not None:
        rows, ssz = pivot_sample
        rows = _sample_rows(rows, K)
        a, pa = _np(rows.reshape(-1), np.int32)
        keep.append(a)
        o.sample_rows = pa
        o.sample_s = int(ssz)
        o.sample_len = int(rows.shape[1])
    r = lslu_result()
    host = dict(
        piv_t=np.full(K + 1, -1, np.int32), piv_g=np.full(K, -1, np.int32),
        own_piv_t=np.full(K + 1, -1, np.int32), own_piv_g=np.full(K, -1, np.int32),
        H=np.zeros((K, K + 1)), W=np.zeros((K, K)), Y=np.zeros((K, K)),
        lambda_k=np.zeros(K), lambda_idx=np.zeros(K, np.int32), ghat=np.zeros(K),
        sep_lambda=np.zeros(K), sigma_max=np.zeros(K), sigma_min=np.zeros(K))
    if grad_lambda:
        host["dloss_dlambda"] = np.zeros(K)
    if pivot_sep:
        host["sep_t"] = np.zeros(K + 1)
        host["sep_g"] = np.zeros(K)
    for name, arr in host.items():
        ct = c_int32 if arr.dtype == np.int32 else c_double
        setattr(r, name, arr.ctypes.data_as(POINTER(ct)))
    _SERIAL[ctx.value] = _SERIAL.get(ctx.value, 0) + 1  # any solve replaces the last
    if host_io:
        bh, pb = _np(b, np.float64)
        x0h = None if x0 is None else _np(x0, np.float64)
        if bh.shape != (m,) or (x0h is not None and x0h[0].shape != (n,)):
            raise ValueError("b must hold m and x0 n float64 values")
        if x_out.dtype != np.float64 or not x_out.flags.c_contiguous or x_out.shape != (n,):
            raise ValueError("x_out must be a contiguous float64 array of n entries")
        st = _check(ctx, lib.lslu_solve_host(
            ctx, op, pb, None if x0h is None else x0h[1], ctypes.byref(o),
            x_out.ctypes.data_as(POINTER(c_double)), ctypes.byref(r)))
        _CTX_SHAPE[ctx.value] = (m, n, prec)  # the solve the context now holds
        return st, x_out, _info(st, r, host, timing)
    entry = lib.lslu_solve_static if static else lib.lslu_solve
    _torch_done(dev)
    st = _check(ctx, entry(ctx, op, _dptr(b), _dptr(x0), ctypes.byref(o),
                           _dptr(x_out), ctypes.byref(r)))
    if static:
        _CTX_SHAPE.pop(ctx.value, None)  # the context holds no basis now
        return st, x_out, _info(st, r, host, timing)
    _CTX_SHAPE[ctx.value] = (m, n, prec)
    if asynchronous:
        # everything the library may still write or read stays referenced
        return Pending(r, host, keep, x_out, (b, x0, X, x_true), timing)
    return st, x_out, _info(st, r, host, timing)


def lslu_solve_batch(ctxs, ops, bs, maxiter, reg="none", lam=0.0, grid=None,
                     grid_relative=False, omega=0.0, stop_tol=0.0, early_stop=False):
    """Solve len(ops) problems together (merged recurrence launches); one
    context per problem, all dense or all CSR in one precision.  ``bs`` are
    device tensors.  Returns ``(status, [(x_out, info), ...])``."""
    import torch
    P = len(ops)
    K = int(maxiter)
    o = lslu_opts()
    o.maxiter = K
    o.reg = REGS[reg] if isinstance(reg, str) else int(reg)
    o.lambda_ = float(lam)
    keep = []
    if grid is not None:
        g, pg = _np(grid, np.float64)
        keep.append(g)
        o.lambda_grid = pg
        o.n_grid = g.shape[0]
    o.grid_relative = 1 if grid_relative else 0
    o.omega = float(omega)
    o.stop_tol = float(stop_tol)
    o.early_stop = 1 if early_stop else 0
    xs, rs, hosts = [], [], []
    if not (len(ctxs) == len(ops) == len(bs)):
        raise ValueError("one context, operator and b per problem")
    for i, (c, op, b) in enumerate(zip(ctxs, ops, bs)):
        m, n, prec = lslu_op_info(op)
        _vec(b, m, prec, f"b[{i}]", _CTX_DEVICE.get(c.value))
        xs.append(torch.empty(n, dtype=_torch_dtype(prec), device=b.device))
        r = lslu_result()
        host = dict(
            piv_t=np.full(K + 1, -1, np.int32), piv_g=np.full(K, -1, np.int32),
            own_piv_t=np.full(K + 1, -1, np.int32), own_piv_g=np.full(K, -1, np.int32),
            H=np.zeros((K, K + 1)), W=np.zeros((K, K)), Y=np.zeros((K, K)),
            lambda_k=np.zeros(K), lambda_idx=np.zeros(K, np.int32), ghat=np.zeros(K),
            sep_lambda=np.zeros(K), sigma_max=np.zeros(K), sigma_min=np.zeros(K))
        for name, arr in host.items():
            ct = c_int32 if arr.dtype == np.int32 else c_double
            setattr(r, name, arr.ctypes.data_as(POINTER(ct)))
        rs.append(r)
        hosts.append(host)
    for c in ctxs:
        _SERIAL[c.value] = _SERIAL.get(c.value, 0) + 1
    arr_c = (c_void_p * P)(*[c.value for c in ctxs])
    arr_o = (c_void_p * P)(*[op.value for op in ops])
    arr_b = (c_void_p * P)(*[b.data_ptr() for b in bs])
    arr_x = (c_void_p * P)(*[x.data_ptr() for x in xs])
    arr_r = (POINTER(lslu_result) * P)(*[ctypes.pointer(r) for r in rs])
    _torch_done(_CTX_DEVICE.get(ctxs[0].value))
    st = _check(ctxs[0], lib.lslu_solve_batch(P, arr_c, arr_o, arr_b, ctypes.byref(o),
                                              arr_x, arr_r))
    for c, op in zip(ctxs, ops):
        _CTX_SHAPE[c.value] = lslu_op_info(op)
    out = []
    for x, r, host in zip(xs, rs, hosts):
        out.append((x, _info(r.status, r, host, False)))
    return st, out


class Pending:
    """An enqueued asynchronous solve (see ``lslu_solve``)."""

    def __init__(self, r, host, keep, x_out, refs, timing):
        self.r, self.host, self.keep, self.x_out, self.refs = r, host, keep, x_out, refs
        self.timing = timing


def lslu_wait(ctx, pending):
    """Completes the context's pending solve; returns ``(status, x_out, info)``."""
    st = _check(ctx, lib.lslu_wait(ctx))
    return st, pending.x_out, _info(st, pending.r, pending.host, pending.timing)


def _info(st, r, host, timing):
    info = dict(status=st, k_done=r.k_done, k_stop=r.k_stop, n_l=r.n_l, n_d=r.n_d,
                beta=r.beta, piv_t_mismatch=r.piv_t_mismatch,
                piv_g_mismatch=r.piv_g_mismatch)
    # column-major (K+1) x K etc. were filled into row-major (K, K+1) buffers
    info.update(piv_t=host["piv_t"], piv_g=host["piv_g"],
                own_piv_t=host["own_piv_t"], own_piv_g=host["own_piv_g"],
                H=host["H"].T.copy(), W=host["W"].T.copy(), Y=host["Y"].T.copy(),
                lambda_k=host["lambda_k"], lambda_idx=host["lambda_idx"],
                ghat=host["ghat"], sep_lambda=host["sep_lambda"],
                sigma_max=host["sigma_max"], sigma_min=host["sigma_min"])
    for name in ("dloss_dlambda", "sep_t", "sep_g"):
        if name in host:
            info[name] = host[name]
    if timing:
        info["timing"] = dict(t_recurrence_ms=r.t_recurrence_ms,
                              n_recurrence_launches=r.n_recurrence_launches,
                              t_projected_ms=r.t_projected_ms,
                              t_assemble_ms=r.t_assemble_ms)
    return info


_SERIAL = {}


def solve_serial(ctx):
    """Number of solves started on ``ctx`` through this binding (lslu_vjp
    differentiates the last one)."""
    return _SERIAL.get(ctx.value, 0)


def lslu_vjp(ctx, op, k, xbar, bbar=None):
    """Reverse pass of the context's last completed solve (which used ``op``):
    returns ``(bbar, lambda_bar)`` with ``bbar = (d x_k/d b)^T xbar`` (a device
    tensor of m entries, allocated when None) and ``lambda_bar = xbar^T
    d x_k/d lambda``, pivots, x_0 and lambda_k held fixed."""
    import torch
    m, n, prec = lslu_op_info(op)
    dev = _CTX_DEVICE.get(ctx.value)
    px = _vec(xbar, n, prec, "xbar", dev)
    if bbar is None:
        bbar = torch.empty(m, dtype=_torch_dtype(prec), device=xbar.device)
    pb = _vec(bbar, m, prec, "bbar", dev)
    lb = c_double(0.0)
    _torch_done(dev)
    _check(ctx, lib.lslu_vjp(ctx, op, int(k), px, pb, ctypes.byref(lb)))
    return bbar, lb.value


def lslu_get_basis(ctx, which, count, dst):
    """Copies ``count`` basis vectors of the context's last solve (L for
    ``which`` = 0, D for 1) into the device tensor ``dst`` (at least count
    vectors of n, resp. m, entries)."""
    shape = _CTX_SHAPE.get(ctx.value)
    if shape is None:
        raise ValueError("no solve was started on this context through this binding")
    m, n, prec = shape
    dev = _CTX_DEVICE.get(ctx.value)
    p = _vec(dst, int(count) * (n if which == 0 else m), prec, "dst", dev, at_least=True)
    _torch_done(dev)
    _check(ctx, lib.lslu_get_basis(ctx, int(which), int(count), p))
    import torch
    torch.cuda.synchronize(0 if dev is None else dev)
