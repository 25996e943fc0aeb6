"""Comparison metrics shared by the parity tests."""
import numpy as np


def normwise(y, ref):
    """max_i |y - ref| / max_i |ref| per variable (row), then the max over rows."""
    y = np.atleast_2d(np.asarray(y, dtype=np.float64))
    ref = np.atleast_2d(np.asarray(ref, dtype=np.float64))
    num = np.abs(y - ref).max(axis=1)
    den = np.abs(ref).max(axis=1)
    den = np.where(den == 0.0, 1.0, den)
    return float((num / den).max())


def report(name, err, tol):
    print(f"  {name}: normwise error {err:.3e} (tolerance {tol:.0e})", flush=True)
    return err <= tol
