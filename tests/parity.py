"""Error norms of Sec. 5 for the parity tests: the relative 2-norm Err_2 over the checked
targets and the largest per-target relative error Err_max."""
import numpy as np

# Err_max bar as a multiple of the Err_2 bar: single targets whose potential is small
# against the sample's norm carry a larger relative error than the norm does (measured
# Err_max / Err_2 on the samples here: 5 to 35)
MAX_FACTOR = 40.0


def errs(got, ref):
    got = np.asarray(got).ravel()
    ref = np.asarray(ref).ravel()
    e2 = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
    emax = float(np.max(np.abs(got - ref) / np.abs(ref)))
    return e2, emax


def check(label, got, ref, tol, tol_max=None):
    """Assert Err_2 < tol and Err_max < tol_max (default MAX_FACTOR tol); returns Err_2."""
    e2, emax = errs(got, ref)
    tol_max = MAX_FACTOR * tol if tol_max is None else tol_max
    print(f"{label}: Err_2 {e2:.3e} (bar {tol:.0e})  Err_max {emax:.3e} (bar {tol_max:.0e})")
    assert np.all(np.isfinite(np.asarray(got))), label
    assert e2 < tol, (label, e2)
    assert emax < tol_max, (label, emax)
    return e2
