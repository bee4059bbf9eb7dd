"""Plain FP64 CPU oracle for LSLU and Hybrid LSLU.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import or call anything here.  The HIP
library never does, and this package never imports the library: the two share
no code.  Inputs for both come from the ``workloads`` package.

The oracle is written from the paper (Brown, Chung, Nagy, Sabate Landman,
"Inner Product Free Krylov Methods for Large-Scale Inverse Problems"):

* ``hessenberg.hybrid_lslu`` -- Algorithm 5 (Hybrid LSLU), with the pivoting of
  Algorithm 4 (rectangular Hessenberg process with pivoting); LSLU is the
  lambda = 0 case (Section 3);
* ``hessenberg.square_hessenberg_pivoted`` -- Algorithm 2 (square Hessenberg
  process with pivoting), used only as a cross-check through relation (eq. h1);
* ``exact.hybrid_lslu_exact`` -- the same steps in exact rational arithmetic;
* ``projected`` -- the projected Tikhonov problem (eq. TSP) through the SVD of
  the small Hessenberg matrix, GCV (eq. gcv2), weighted GCV (eq. wgcv_projected1
  and its SVD form), the optimal parameter (eq. lambda) and the stopping
  function (eq. stop2);
* ``operators`` -- the three forward models (dense, CSR, PSF).

Every function says which passage it follows.  Readings taken where the paper
is silent or inconsistent are listed in the module that applies them.

Parity pins: every function here is pinned by a CPU test in ``tests/`` against
something other than itself (relations the paper proves, exact arithmetic,
closed forms, brute-force minimisation, Krylov subspaces from an orthogonal
process).  No function is "parity unpinned".
"""

from .operators import DenseOp, CsrOp, PsfOp, make_operator  # noqa: F401
from .projected import (  # noqa: F401
    RegParam,
    projected_svd,
    tikhonov_coeffs,
    gcv_value,
    wgcv_value,
    ghat_value,
)
from .hessenberg import (  # noqa: F401
    Status,
    hybrid_lslu,
    square_hessenberg_pivoted,
)
