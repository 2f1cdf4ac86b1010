"""O4: the modular inner loop of the arithmetic microbenchmark, by its
definition (test infrastructure only, like the rest of this package).

Chain i starts at x = x0[i] and applies x <- (b[i] + x * a[i]) mod p
``iters`` times: an update of the form of equation "mod-fma" whose product
takes the running value.  numpy int64 holds every intermediate exactly for
p < 2^31 (x * a < 2^62).  No reduction trick is involved: ``%`` is the
definition of the residue.
"""

import numpy as np


def chains(p, x0, a, b, iters):
    x = np.asarray(x0, dtype=np.int64).copy()
    a = np.asarray(a, dtype=np.int64)
    b = np.asarray(b, dtype=np.int64)
    for _ in range(iters):
        x = (b + x * a) % p
    return x
