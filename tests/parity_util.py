"""Shared helpers of the parity tests: relative max-norm error per field."""
import numpy as np

TOL = {"fp64": 1e-12, "fp32": 2e-5, "mixed": 2e-5}
FLOOR = {"fp64": 1e-30, "fp32": 1e-12, "mixed": 1e-12}


def rel_err(a, b, prec):
    """max |a - b| / max(max |b|, floor) over the whole field."""
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.abs(a - b).max() / max(float(np.abs(b).max()), FLOOR[prec]))


def compare_moments(got, ref, prec, fields=("phi", "rhoH", "T", "fl", "rho", "u", "p", "mdot"), tol=None):
    tol = TOL[prec] if tol is None else tol
    errs = {k: rel_err(got[k], ref[k], prec) for k in fields}
    bad = {k: v for k, v in errs.items() if not v <= tol}
    return errs, bad
