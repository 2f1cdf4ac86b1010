"""O5: the block operator application of the Krylov solvers, by definition
(test infrastructure only, like the rest of this package).

Y[i][k] = sum_j A[i][j] X[j][k] mod p for a CSR matrix A, and the same for the
transpose, Y[j][k] = sum_i A[i][j] X[i][k] mod p (the block form of "apply A"
and "apply A^T" of the Wiedemann and Lanczos methods).  Every product is taken
modulo p before the per-row sum, so int64 holds the sums exactly.
"""

import numpy as np


def spmm(row_ptr, col_ind, val, ncols, X, p, trans=False):
    row_ptr = np.asarray(row_ptr, dtype=np.int64)
    col_ind = np.asarray(col_ind, dtype=np.int64)
    val = np.asarray(val, dtype=np.int64) % p
    X = np.asarray(X, dtype=np.int64) % p
    if X.ndim == 1:
        X = X[:, None]
    r = len(row_ptr) - 1
    rows = np.repeat(np.arange(r, dtype=np.int64), np.diff(row_ptr))
    if trans:
        src, dst, nout = rows, col_ind, ncols
    else:
        src, dst, nout = col_ind, rows, r
    terms = (val[:, None] * X[src]) % p
    Y = np.zeros((nout, X.shape[1]), dtype=np.int64)
    np.add.at(Y, dst, terms)
    return Y % p
