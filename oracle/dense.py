"""Oracle O3: dense Gaussian elimination over Python integers (test infrastructure only).

Used to pin the elimination stage independently of the pivot / non-pivot
split.  For the Macaulay matrix A of a step (Definition "Sparse Macaulay matrix
for a batch"), the reduced row echelon form is unique for its row space, so:

* rank(A) = (number of pivot columns) + rank of the reduced trailing block, and
* the rows of RREF(A) whose leading column is not the leading column of any
  row of A are exactly the rows of RREF of the reduced trailing block,

because the row space of the reduced trailing block is the part of the row
space of A supported on the non-pivot columns.
"""


def rref(rows, ncols, p):
    """Reduced row echelon form mod p.  rows: list of lists of ints.
    Returns (list of nonzero monic rows in pivot order, list of pivot columns)."""
    M = [[v % p for v in r] for r in rows]
    piv_rows, piv_cols = [], []
    r0 = 0
    for c in range(ncols):
        pr = None
        for i in range(r0, len(M)):
            if M[i][c]:
                pr = i
                break
        if pr is None:
            continue
        M[r0], M[pr] = M[pr], M[r0]
        inv = pow(M[r0][c], p - 2, p)
        M[r0] = [v * inv % p for v in M[r0]]
        for i in range(len(M)):
            if i != r0 and M[i][c]:
                f = M[i][c]
                M[i] = [(a - f * b) % p for a, b in zip(M[i], M[r0])]
        piv_cols.append(c)
        r0 += 1
    return M[:r0], piv_cols


def csr_to_dense(row_ptr, col_ind, val, ncols):
    out = []
    for i in range(len(row_ptr) - 1):
        r = [0] * ncols
        for q in range(row_ptr[i], row_ptr[i + 1]):
            r[col_ind[q]] = val[q]
        out.append(r)
    return out


def left_kernel(rows, ncols, p):
    """A basis of {v : v^T A = 0} for the dense matrix `rows` (r x ncols).

    Gaussian elimination on [A | I] using pivots in the A part only; the rows
    whose A part ends up zero carry, in their identity part, the coefficients
    of a vanishing row combination."""
    r = len(rows)
    M = [[v % p for v in rows[i]] + [1 if j == i else 0 for j in range(r)] for i in range(r)]
    r0 = 0
    for c in range(ncols):
        pr = None
        for i in range(r0, r):
            if M[i][c]:
                pr = i
                break
        if pr is None:
            continue
        M[r0], M[pr] = M[pr], M[r0]
        inv = pow(M[r0][c], p - 2, p)
        M[r0] = [v * inv % p for v in M[r0]]
        for i in range(r):
            if i != r0 and M[i][c]:
                f = M[i][c]
                M[i] = [(a - f * b) % p for a, b in zip(M[i], M[r0])]
        r0 += 1
    return [row[ncols:] for row in M[r0:]]
