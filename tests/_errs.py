"""Error measures of the parity tests.

Each result vector x (mean, variance, w) of the GPU path is compared with
the oracle's x_ref in two ways:
  norm  ||x - x_ref||_2 / ||x_ref||_2      (the tolerances' normwise reading)
  max   max|x - x_ref| / max|x_ref|        (catches a few bad points that a
                                            norm over many points would hide)
Both are asserted against the same bound: 1e-10 for the FP64 path, 1e-5 on
the mean and 1e-4 on the variance for the mixed paths.
"""
import numpy as np

TOL64 = 1e-10
TOL_MEAN_MIXED = 1e-5
TOL_VAR_MIXED = 1e-4


def norm_err(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def max_err(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def errs(a, b):
    """(normwise, max-relative) error of a against b."""
    return norm_err(a, b), max_err(a, b)


def fmt(e):
    return f"{e[0]:.3e}/{e[1]:.3e}"


def assert_within(e, tol, what):
    assert e[0] <= tol and e[1] <= tol, f"{what}: norm {e[0]:.3e}, max {e[1]:.3e} > {tol:.0e}"
