"""FP64 CPU oracle for u-series electrostatics -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The GPU library never calls it and
shares no code with it; the two meet only through the seeded input
generators, which hold none of the method's arithmetic.

``useries_oracle.c`` is the u-series reference (near part by a brute-force
image sum, far part by direct periodic image sums of each separable Gaussian,
plus the k-space form of App. F eq. F1 as an independent cross-check);
``ewald.py`` is a converged classical Ewald sum (Sec. II, eqs. 6-10) used to
pin the oracle on tiny inputs.
"""
from .core import (Params, build, load, eval_full, eval_near, eval_far, far_kspace,
                   forces_subset, far_inf, near_kernel, bsa_bound,
                   eq33_bound, solve_c0, solve_c1, c1_w0, series_len, term,
                   far_inf0, near_integral, num_threads, mellin_gauss, trunc_bound,
                   c1_w0a, solve_c1a)
from .ewald import ewald

__all__ = ["Params", "build", "load", "eval_full", "eval_near", "eval_far", "far_kspace",
           "forces_subset", "far_inf", "near_kernel", "bsa_bound",
           "eq33_bound", "solve_c0", "solve_c1", "c1_w0", "series_len", "term",
           "far_inf0", "near_integral", "num_threads", "mellin_gauss", "trunc_bound",
           "c1_w0a", "solve_c1a", "ewald"]
