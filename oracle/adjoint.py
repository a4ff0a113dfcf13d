"""Dense FP64 gradient of L = ||s_hat - t||^2 with respect to y.

On a frozen support S the recovered coefficients are the least-squares
solution s_hat_S = G^-1 A_S^T y with G = A_S^T A_S (Sec. II step 3), which is
linear in y: d s_hat_S / d y = G^-1 A_S^T.  Entries of s_hat off S are zero
and do not depend on y.  Hence

    dL/dy = 2 A_S G^-1 (s_hat_S - t_S).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from .operator import SRM


def adjoint_gradient(op: SRM, supp, y, t_dense) -> tuple[np.ndarray, np.ndarray]:
    """Returns (dL/dy as an M-vector, s_hat_S).  With complex measurements the
    gradient is dL/d(Re y) + i dL/d(Im y), from the stacked real system
    [Re A_S; Im A_S] (the coefficients are real)."""
    s = np.asarray(supp, dtype=np.int64)
    a = op.columns(s)
    cplx = np.iscomplexobj(a)
    if cplx:
        yc = np.asarray(y, dtype=np.complex128)
        a = np.vstack([a.real, a.imag])
        yv = np.concatenate([yc.real, yc.imag])
    else:
        yv = np.asarray(y, dtype=np.float64)
    G = a.T @ a
    cf = sla.cho_factor(G, lower=True)
    s_hat = sla.cho_solve(cf, a.T @ yv)
    g = sla.cho_solve(cf, s_hat - np.asarray(t_dense, dtype=np.float64)[s])
    gy = 2.0 * (a @ g)
    if cplx:
        m = gy.size // 2
        gy = gy[:m] + 1j * gy[m:]
    return gy, s_hat
