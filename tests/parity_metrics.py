"""Error metrics of the parity tests. A global relative RMS can hide one bad
sub-filter path (one column of the [nblock][lblock] frame matrix), which is
exactly where the inverse is ill-conditioned (paths near N/2, Section 4.1),
so the tests also bound the worst column."""
import numpy as np


def rel(a, ref) -> float:
    a = np.asarray(a)
    ref = np.asarray(ref)
    return float(np.linalg.norm((a - ref).ravel()) / np.linalg.norm(ref.ravel()))


def worst_column_rel(a, ref, ncol: int):
    """max over columns n of |a[:, n] - ref[:, n]| / |ref[:, n]| for arrays
    laid out [rows][ncol] (a timestream: ncol = lblock, one column per
    sub-filter path). Returns (worst error, its column)."""
    A = np.asarray(a).reshape(-1, ncol)
    R = np.asarray(ref).reshape(-1, ncol)
    num = np.linalg.norm(A - R, axis=0)
    den = np.linalg.norm(R, axis=0)
    e = num / np.where(den > 0, den, 1.0)
    k = int(np.argmax(e))
    return float(e[k]), k
