"""Seeded synthetic inverse problems (inputs only).

This package builds test problems ``b = A x_true + e`` with the shapes, value
distributions and noise model of the paper's experiments (Section 4: noise level
``||e|| / ||A x_true||``).  It holds none of the solver's arithmetic: it draws
random numbers, samples a forward model (a matrix, a sparse ray-sum matrix or a
point-spread function) and applies that forward model once to make the data.

Both the CPU oracle (``oracle/``) and the HIP library's tests and benchmark read
their inputs from here, and from nowhere else, so the two sides always solve the
same problem.  Nothing here imports either side.
"""

from .problems import (  # noqa: F401
    Problem,
    dense_blur_1d,
    tomography,
    psf_deblur,
    random_dense,
    config_problem,
    CONFIGS,
    lambda_grid,
    pivot_sample_lists,
    batch_problems,
)
