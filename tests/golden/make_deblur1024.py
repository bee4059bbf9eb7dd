"""Writes ``deblur1024_fp64.npz``: the FP64 oracle's Hybrid LSLU solve of the
1024 x 1024 deblurring workload (31 x 31 Gaussian PSF, sigma 2.5, zero
boundary, 1 % noise, 150 iterations, weighted GCV on the relative grid of 20
log-spaced values), for the full-size GPU parity test.

It calls only the oracle (Algorithm 5 with Algorithm 4's pivoting, the
projected problem of Section 3.2.1) and the seeded input generator; nothing
here touches the HIP library.  The solve takes about ten minutes on one core
and holds about 4 GB.

What is stored (a 1024^2 iterate is 8 MB, so the vectors are sampled):

* the whole small output of the method: pivots t, g; beta; H, W; the
  projected solutions Y; lambda_k, its grid index and separation; Ghat(k);
  k_stop; the separation of every pivot search;
* per k: ||x_k||, ||x_k - x_true|| / ||x_true||, ||b - A x_k|| / ||b||, and
  the condition number of H_{k+1,k};
* at 1024 seeded pixels: every iterate x_k and every basis vector l_j, d_j.

Run from the repository root: ``python tests/golden/make_deblur1024.py``.
"""

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from oracle import RegParam, make_operator  # noqa: E402
from oracle.hessenberg import hybrid_lslu  # noqa: E402
from workloads import config_problem, lambda_grid  # noqa: E402

K = 150
N_PIX = 1024
PIX_SEED = 20241024


def main(out=os.path.join(HERE, "deblur1024_fp64.npz")):
    t0 = time.time()
    prob = config_problem("deblur1024")
    op = make_operator(prob)
    grid = lambda_grid()
    reg = RegParam("wgcv", grid=grid, grid_relative=True)
    print(f"[golden] {prob.name}: m = n = {prob.n}, K = {K}", flush=True)
    R = hybrid_lslu(op, prob.b, K, reg)
    print(f"[golden] solve done in {time.time() - t0:.0f} s, k_done = {R.k_done}, "
          f"status = {int(R.status)}", flush=True)
    kd = R.k_done
    nb = np.linalg.norm(prob.b)
    nxt = np.linalg.norm(prob.x_true)
    xnorm = np.array([np.linalg.norm(R.X[:, k]) for k in range(kd)])
    err_true = np.array([np.linalg.norm(R.X[:, k] - prob.x_true) / nxt for k in range(kd)])
    res = np.array([np.linalg.norm(prob.b - op.matvec(R.X[:, k])) / nb for k in range(kd)])
    cond = np.array([np.linalg.cond(R.H[:k + 1, :k]) for k in range(1, kd + 1)])
    pix = np.sort(np.random.default_rng(PIX_SEED).choice(prob.n, N_PIX, replace=False))
    np.savez_compressed(
        out,
        K=K, k_done=kd, status=int(R.status), k_stop=R.k_stop, beta=R.beta,
        piv_t=np.asarray(R.piv_t, np.int32), piv_g=np.asarray(R.piv_g, np.int32),
        H=R.H, W=R.W, Y=R.Y, lambdas=R.lambdas, lambda_idx=R.lambda_idx,
        sep_lambda=R.sep_lambda, ghat=R.ghat,
        sep_t=np.asarray(R.sep_t), sep_g=np.asarray(R.sep_g),
        xnorm=xnorm, err_true=err_true, res=res, cond=cond,
        grid=grid, pix=pix.astype(np.int64),
        X_pix=R.X[pix, :], L_pix=R.L[pix, :], D_pix=R.D[pix, :])
    print(f"[golden] wrote {out} ({os.path.getsize(out) / 1e6:.2f} MB) after "
          f"{time.time() - t0:.0f} s; min error {err_true.min():.5f} at k = "
          f"{int(np.argmin(err_true)) + 1}", flush=True)


if __name__ == "__main__":
    main()
