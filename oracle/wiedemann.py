"""O6: block Wiedemann over F_p for left-kernel vectors of a sparse matrix
(test infrastructure only, like the rest of this package).

The paper's Krylov branch (section "Block Wiedemann and Block Lanczos": kernel
vectors via black-box linear algebra; Remark "Syzygies, revisited") looks for
v != 0 with v^T A = 0 - by Proposition "Kernel equals syzygies under
dictionary closure" these are the (truncated) syzygies among the shifted
reducers of a Macaulay matrix - using only products of A and A^T with blocks
of b vectors.  The readings taken here (the paper names the method and its
references, not its steps):

* Operator.  A is r x N; the square operator is B = A D A^T (r x r) with D a
  diagonal of nonzero field elements given as input.  ker A^T is inside
  ker B, and the two are equal unless the row space of A meets the kernel of
  A D (which a random D avoids with probability at least 1 - rank/p); every
  vector found is therefore checked against A^T v = 0.
* Sequence (Coppersmith's block form of Wiedemann's scalar sequence):
  Z_0 = B Y and S_t = X^T B^t Z_0 for t = 0 .. L-1, with X, Y given r x b
  blocks, L = 2 ceil(r / b) + 4.
* Generator.  A sigma-basis of F(x) = [S(x)^T ; -I_b] to order L by the
  iterative M-Basis method (Beckermann-Labahn; Giorgi-Jeannerod-Villard),
  shifts (0^b, 1^b): at order k the residual coefficient of every row is
  eliminated row by row in the order of (shift, index), each nonzero row
  pivoting on its first nonzero column and clearing that column from the rows
  after it (fraction-free: row_j <- piv row_j - D_j[c] row_i, no inverses),
  and the pivot rows are then multiplied by x.  A row (g, h) of the
  result has deg g <= s and deg h < s for its shift s, so f_m = g_{s-m}
  satisfies sum_m S_{t+m} f_m = 0 for t = 0 .. L-1-s: a right generator of
  the sequence.  Rows with g != 0 and 2 s + 2 <= L are kept.
* Kernel vectors.  For a generator f of degree s with lowest nonzero
  coefficient m0, u = sum_{m >= m0} B^(m-m0) Y f_m (Horner); the first
  B^e u that B sends to zero (e <= s + 1) is a kernel vector of B, and is
  kept when A^T v = 0.

Everything is exact: products are reduced mod p (numpy int64 for the
operator, Python integers for the small dense steps).
"""

import numpy as np

from . import krylov as o5


def block_len(r, b):
    """Sequence length L = 2 ceil(r / b) + 4."""
    return 2 * (-(-r // b)) + 4


def apply_B(row_ptr, col_ind, val, ncols, d, V, p):
    """B V = A (D (A^T V)) mod p for an r x b block V."""
    U = o5.spmm(row_ptr, col_ind, val, ncols, V, p, trans=True)
    U = (U * (np.asarray(d, dtype=np.int64) % p)[:, None]) % p
    return o5.spmm(row_ptr, col_ind, val, ncols, U, p)


def proj(X, Z, p):
    """X^T Z mod p with exact integers."""
    return np.array((np.asarray(X, dtype=object).T.dot(np.asarray(Z, dtype=object))) % p, dtype=np.int64)


def sequence(row_ptr, col_ind, val, ncols, d, X, Y, p, L):
    """S_t = X^T B^t (B Y), t = 0 .. L-1, as an L x b x b array."""
    Z = apply_B(row_ptr, col_ind, val, ncols, d, Y, p)
    S = []
    for _ in range(L):
        S.append(proj(X, Z, p))
        Z = apply_B(row_ptr, col_ind, val, ncols, d, Z, p)
    return np.array(S, dtype=np.int64)


def residual(P, S, k, b, p):
    """Coefficient of x^k of P F, F = [S(x)^T ; -I]: row i, column c is
    sum_{j<b} sum_l P[i][j][l] S[k-l][c][j] - P[i][b+c][k]."""
    m = 2 * b
    R = [[0] * b for _ in range(m)]
    for i in range(m):
        for c in range(b):
            acc = 0
            for j in range(b):
                row = P[i][j]
                for l in range(0, k + 1):
                    if row[l]:
                        acc += row[l] * int(S[k - l][c][j])
            acc -= P[i][b + c][k]
            R[i][c] = acc % p
    return R


def mbasis(S, b, p, sigma=None):
    """M-Basis to order sigma (default: the sequence length) of
    [S(x)^T ; -I_b], shifts (0^b, 1^b).  Returns (P, shifts): P[i][j] is the
    coefficient list (length sigma + 2: a row's degree is at most its shift,
    at most sigma + 1) of entry (i, j)."""
    L = len(S)
    sigma = L if sigma is None else sigma
    m = 2 * b
    P = [[[0] * (sigma + 2) for _ in range(m)] for _ in range(m)]
    for i in range(m):
        P[i][i][0] = 1
    s = [0] * b + [1] * b
    for k in range(sigma):
        D = residual(P, S, k, b, p)
        order = sorted(range(m), key=lambda i: (s[i], i))
        pivots = []
        for a, i in enumerate(order):
            c = next((c for c in range(b) if D[i][c]), None)
            if c is None:
                continue
            pivots.append(i)
            piv = D[i][c]
            for j in order[a + 1:]:
                if D[j][c]:
                    # fraction-free: row_j <- piv row_j - D_j[c] row_i (a nonzero
                    # multiple of a row stays an approximant of the same degree)
                    f = D[j][c]
                    D[j] = [(piv * x - f * y) % p for x, y in zip(D[j], D[i])]
                    for col in range(m):
                        P[j][col] = [(piv * x - f * y) % p for x, y in zip(P[j][col], P[i][col])]
        for i in pivots:
            for col in range(m):
                P[i][col] = [0] + P[i][col][:-1]
            s[i] += 1
    return P, s


def generators(P, s, b, sigma):
    """Right generators from the rows (g, h) of a sigma-basis: rows with
    g != 0 and 2 s + 2 <= sigma, in the order of (shift, index); each as
    (s, f) with f[m] = g_{s-m} (a list of s + 1 vectors of length b)."""
    out = []
    for i in sorted(range(2 * b), key=lambda i: (s[i], i)):
        g = P[i][:b]
        if not any(any(c) for c in g) or 2 * s[i] + 2 > sigma:
            continue
        out.append((s[i], [[g[j][s[i] - m] for j in range(b)] for m in range(s[i] + 1)]))
    return out


def check_generator(S, f, p):
    """sum_m S_{t+m} f_m = 0 for every t with t + deg < L."""
    deg = len(f) - 1
    for t in range(len(S) - deg):
        acc = np.zeros(S.shape[1], dtype=object)
        for m in range(deg + 1):
            acc = acc + np.asarray(S[t + m], dtype=object).dot(np.asarray(f[m], dtype=object))
        if any(int(x) % p for x in acc):
            return False
    return True


def kernel_vectors(row_ptr, col_ind, val, ncols, d, Y, gens, p):
    """For each generator (s, f): u = sum_{m >= m0} B^(m - m0) Y f_m, then the
    first B^e u (e <= s + 1) with B (B^e u) = 0, kept when it is nonzero and
    A^T v = 0.  Returns (vectors, e-values), vectors as int64 arrays of length r."""
    Y = np.asarray(Y, dtype=np.int64) % p
    vecs, es = [], []
    for deg, f in gens:
        m0 = next(m for m in range(deg + 1) if any(f[m]))
        u = np.zeros(Y.shape[0], dtype=np.int64)
        for m in range(deg, m0 - 1, -1):  # Horner: u <- B u + Y f_m
            u = apply_B(row_ptr, col_ind, val, ncols, d, u[:, None], p)[:, 0]
            u = (u + np.array(np.asarray(Y, dtype=object).dot(np.asarray(f[m], dtype=object)) % p,
                              dtype=np.int64)) % p
        v = u
        found = None
        for e in range(deg + 2):
            if not v.any():
                break
            w = apply_B(row_ptr, col_ind, val, ncols, d, v[:, None], p)[:, 0]
            if not w.any():
                found = (v, e)
                break
            v = w
        if found is None:
            continue
        v = found[0]
        if o5.spmm(row_ptr, col_ind, val, ncols, v[:, None], p, trans=True).any():
            continue  # in ker B but not a syzygy (the row space met ker(A D))
        vecs.append(v)
        es.append(found[1])
    return vecs, es


def left_kernel_block_wiedemann(row_ptr, col_ind, val, ncols, d, X, Y, p):
    """The whole method: sequence, sigma-basis, generators, kernel vectors."""
    r = len(row_ptr) - 1
    b = np.asarray(X).shape[1]
    L = block_len(r, b)
    S = sequence(row_ptr, col_ind, val, ncols, d, X, Y, p, L)
    P, s = mbasis(S, b, p)
    gens = generators(P, s, b, L)
    vecs, es = kernel_vectors(row_ptr, col_ind, val, ncols, d, Y, gens, p)
    return {"S": S, "P": P, "shifts": s, "gens": gens, "vectors": vecs, "e": es, "L": L}
