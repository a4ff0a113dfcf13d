"""Exhaustive l0 search (Eq. (3)) on tiny inputs: the K-column support whose
least-squares fit leaves the smallest residual.  Exponential in N; used only
as a pin for the greedy algorithms."""
from __future__ import annotations

import itertools
import numpy as np

from .operator import SRM


def l0_bruteforce(op: SRM, y, K: int):
    """Returns (support ascending, values, residual norm) minimising ||y - A_S v||."""
    a = op.dense()
    y = np.asarray(y, dtype=np.float64)
    best = (None, None, np.inf)
    for S in itertools.combinations(range(op.n), K):
        cols = a[:, S]
        v, *_ = np.linalg.lstsq(cols, y, rcond=None)
        rn = float(np.linalg.norm(y - cols @ v))
        if rn < best[2]:
            best = (np.asarray(S), v, rn)
    return best
