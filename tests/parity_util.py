"""Shared helpers of the parity tests: relative max-norm error per field.

The liquid fraction in float32 storage is compared as psi f_l, psi = sum of
the volume fractions of the freezing phases.  f_l itself comes from the
inversion of eq. (H), f_l = (rho H - E_s) / (E_l - E_s), whose latent range
E_l - E_s is proportional to psi: where hardly any freezing material is
present (a gas cell at T = T_melt, psi ~ 1e-4) a float32 rounding of rho H
at 1e-7 relative moves f_l by 1e-4, although nothing in the method depends
on f_l there.  Every use of f_l in the method (the penalty f_s psi, the
mixture density and the volume source) weights it by the freezing phase
fractions, and psi f_l = (rho H - E_s) / (rho^l L) is as well conditioned
as rho H.  In float64 f_l is compared directly.
"""
import numpy as np

TOL = {"fp64": 1e-12, "fp32": 2e-5, "mixed": 2e-5}
FLOOR = {"fp64": 1e-30, "fp32": 1e-12, "mixed": 1e-12}
FIELDS = ("phi", "rhoH", "T", "fl", "rho", "u", "p", "mdot")


def rel_err(a, b, prec):
    """max |a - b| / max(max |b|, floor) over the whole field."""
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.abs(a - b).max() / max(float(np.abs(b).max()), FLOOR[prec]))


def freezing_fraction(phi, params):
    """psi = sum of phi_p over the phases that freeze."""
    N = params["nphase"]
    return sum(phi[q] for q in range(N) if params["freezes"][q])


def compare_moments(got, ref, prec, params, fields=FIELDS, tol=None):
    """Per-field errors and the fields above tol.  In float32 storage the
    key "fl" holds the error of psi f_l (psi from the reference phi); the
    raw f_l error is reported under "fl_raw" and not checked."""
    tol = TOL[prec] if tol is None else tol
    errs, checked = {}, []
    for k in fields:
        if k == "fl" and prec != "fp64":
            psi = freezing_fraction(ref["phi"], params)
            errs["fl"] = rel_err(psi * got["fl"], psi * ref["fl"], prec)
            errs["fl_raw"] = rel_err(got["fl"], ref["fl"], prec)
        else:
            errs[k] = rel_err(got[k], ref[k], prec)
        checked.append(k)
    bad = {k: errs[k] for k in checked if not errs[k] <= tol}
    return errs, bad
