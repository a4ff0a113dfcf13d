"""Closed-form Gram matrix of the sensing operator's selected columns.

For A = D_rows F diag(signs) (Eq. (7) with F the orthonormal DCT-II), column
j is  a_j[k] = signs_j c_k cos(pi (2j+1) k / (2N)),  k in rows.  The
product-to-sum identity cos(a) cos(b) = (cos(a-b) + cos(a+b)) / 2 gives

    (A_S^T A_S)[p, q] = 1/2 signs_i signs_j [ g(i' - j') + g(i' + j' + 1) ],
    g(m) = sum_{k in rows} c_k^2 cos(pi m k / N),     i = S[p], j = S[q],

with i', j' the DCT input indices of i and j (i' = i without a permutation
in the randomizer),

a Toeplitz-plus-Hankel matrix whose generator g (even, 2N-periodic) comes
from one length-2N FFT of the weighted row mask.  This is derived here from
the operator's definition; the paper does not state it.  It makes the
explicit pseudo-inverse of Eq. (9) affordable for |S| up to about 10^4.
"""
from __future__ import annotations

import numpy as np
import scipy.fft as sfft

from .operator import SRM, WORKERS


def gram_generator(op: SRM) -> np.ndarray:
    """g(m) for m in [0, 2N)."""
    n = op.n
    w = np.zeros(2 * n)
    ck2 = np.where(op.rows == 0, 1.0 / n, 2.0 / n)
    w[op.rows] = ck2
    # fft gives sum_k w_k exp(-i pi m k / N); its real part is g(m).
    return sfft.fft(w, workers=WORKERS).real


def gram_matrix(op: SRM, supp, g: np.ndarray | None = None) -> np.ndarray:
    """A_S^T A_S (|S| x |S|) in closed form."""
    if op.psi or op.xform:
        raise ValueError("the closed-form Gram holds for the DCT-II with Psi = I only")
    if g is None:
        g = gram_generator(op)
    s = np.asarray(supp, dtype=np.int64)
    sg = op.signs[s]
    q = op.dct_index(s)                       # the DCT input index of each column
    diff = np.abs(q[:, None] - q[None, :])
    summ = q[:, None] + q[None, :] + 1
    return 0.5 * (sg[:, None] * sg[None, :]) * (g[diff] + g[summ])
