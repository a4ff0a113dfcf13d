"""Least-squares step of the greedy algorithms (Sec. II step 3, Eq. (9)).

    s_S = argmin_v || y - A_S v ||_2 = (A_S^T A_S)^-1 A_S^T y

Theorems 1 and 2 of the paper show that the weighted problem (Eq. (10)) and
its normal-equation form (Eq. (11)), which the CG of Algorithm 1 solves, have
this same solution on S.  So the oracle computes the plain definition with
an explicit pseudo-inverse:

* ``ls_dense``: QR/SVD least squares (``numpy.linalg.lstsq``) on the dense
  A_S built from the cosine formula, for small M * |S|;
* ``ls_gram``:  Cholesky of the closed-form Gram (``oracle.gram``) with the
  right-hand side (A^T y)[S] (Psi = I only);
* ``ls_cg``:    only where the Gram would not fit in memory (|S| > 16384):
  plain FP64 conjugate gradients on the normal equations through the
  operator, run to a relative residual of 1e-13 and re-checked with the true
  residual.  This route is cross-checked against the explicit ones on
  smaller supports by the pins.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from .operator import SRM
from .gram import gram_matrix, gram_generator

DENSE_LIMIT = 3.0e7      # M * |S| entries for the dense route (240 MB)
GRAM_LIMIT = 16384       # |S| for the Cholesky route (2 GiB Gram)


def ls_dense(op: SRM, supp, y) -> np.ndarray:
    a = op.columns(supp)
    if np.iscomplexobj(a):
        # real coefficients, complex measurements: the stacked real system
        yc = np.asarray(y, dtype=np.complex128)
        sol, *_ = np.linalg.lstsq(np.vstack([a.real, a.imag]), np.concatenate([yc.real, yc.imag]), rcond=None)
        return sol
    sol, *_ = np.linalg.lstsq(a, np.asarray(y, dtype=np.float64), rcond=None)
    return sol


def ls_gram(op: SRM, supp, y, g: np.ndarray | None = None, aty: np.ndarray | None = None) -> np.ndarray:
    s = np.asarray(supp, dtype=np.int64)
    G = gram_matrix(op, s, g)
    if aty is None:
        aty = op.adjoint(y)
    c = sla.cho_factor(G, lower=True, check_finite=True)
    return sla.cho_solve(c, aty[s], check_finite=False)


def ls_cg(op: SRM, supp, y, tol: float = 1e-13, max_iter: int | None = None,
          x0: np.ndarray | None = None, aty: np.ndarray | None = None):
    """FP64 CG on (A_S^T A_S) v = A_S^T y through the operator.

    Returns (v, iterations).  Stops when ||b - H v|| <= tol ||b|| holds for
    the true residual (recomputed when the recursive one passes)."""
    s = np.asarray(supp, dtype=np.int64)
    n = op.n
    if aty is None:
        aty = op.adjoint(y)
    b = aty[s]

    def happly(v):
        x = np.zeros(n)
        x[s] = v
        return op.adjoint(op.apply(x))[s]

    v = np.zeros(s.size) if x0 is None else np.array(x0, dtype=np.float64)
    r = b - happly(v) if x0 is not None else b.copy()
    d = r.copy()
    rr = r @ r
    bb = b @ b
    if max_iter is None:
        max_iter = 10 * s.size + 50
    it = 0
    while it < max_iter:
        if rr <= (tol * tol) * bb:
            r_true = b - happly(v)
            if r_true @ r_true <= (tol * tol) * bb:
                break
            r = r_true
            d = r.copy()
            rr = r @ r
        q = happly(d)
        alpha = rr / (d @ q)
        v = v + alpha * d
        r = r - alpha * q
        rr_new = r @ r
        d = r + (rr_new / rr) * d
        rr = rr_new
        it += 1
    return v, it


def ls(op: SRM, supp, y, g: np.ndarray | None = None, aty: np.ndarray | None = None,
       route: str = "auto") -> np.ndarray:
    """s_S for a support ``supp`` (any order; the result follows that order)."""
    k = len(supp)
    if k == 0:
        return np.zeros(0)
    if route == "auto":
        if op.m * k <= DENSE_LIMIT:
            route = "dense"
        elif k <= GRAM_LIMIT and not op.psi and not op.xform:   # the closed-form Gram: DCT-II, Psi = I
            route = "gram"
        else:
            route = "cg"
    if route == "dense":
        return ls_dense(op, supp, y)
    if route == "gram":
        return ls_gram(op, supp, y, g, aty)
    if route == "cg":
        return ls_cg(op, supp, y, aty=aty)[0]
    raise ValueError(route)


class LSContext:
    """Caches what every LS call of one recovery shares (A^T y and the Gram generator)."""

    def __init__(self, op: SRM, y, route: str = "auto"):
        self.op = op
        self.y = np.asarray(y, dtype=np.complex128 if getattr(op, "complex_meas", False) else np.float64)
        self.route = route
        self.aty = op.adjoint(self.y)
        self._g = None
        self.calls = 0

    @property
    def g(self):
        if self._g is None:
            self._g = gram_generator(self.op)
        return self._g

    def solve(self, supp) -> np.ndarray:
        self.calls += 1
        k = len(supp)
        route = self.route
        if route == "auto":
            if self.op.m * k <= DENSE_LIMIT:
                route = "dense"
            elif k <= GRAM_LIMIT and not self.op.psi and not self.op.xform:   # closed-form Gram: DCT-II, Psi = I
                route = "gram"
            else:
                route = "cg"
        if route == "dense":
            return ls_dense(self.op, supp, self.y)
        if route == "gram":
            return ls_gram(self.op, supp, self.y, self.g, self.aty)
        return ls_cg(self.op, supp, self.y, aty=self.aty)[0]
