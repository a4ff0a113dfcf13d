"""Greedy recovery algorithms, step by step, in FP64.

OMP follows Sec. II (steps 1-4) and Algorithm 1 (outer loop): exactly K
iterations of correlation, argmax, support update, least squares, residual.
SP (Dai and Milenkovic) and OMPR (Jain, Tewari and Dhillon) are the other two
greedy algorithms run in Sec. IV; the paper names them but does not restate
them, so they are written here from their original definitions with the
readings below.

Decision rules (the paper leaves ties unstated):
* every selection ranks candidates by (key descending, index ascending); the
  chosen set is the first k of that order;
* OMP's argmax and SP's expansion step only consider indices outside the
  current support (in exact arithmetic the correlation vanishes on the
  support, Theorem 2's orthogonality, so this changes nothing there);
* OMPR drops the element ranked last by the same order over I u {j}.

SP reading: T = top-K of |A^T y|, x = LS(T), r = y - A x; then repeat
  c = A^T r;  D = top-K of |c| outside T;  x~ = LS(T u D);
  T' = top-K of |x~| over T u D;  x' = LS(T'), r' = y - A x';
  stop with (T', x') if T' == T; stop with (T, x) if ||r'|| > ||r||;
  otherwise continue with (T', x', r').  At most ``max_iter`` rounds.

OMPR reading (replacement size l, default 1; step eta = N/M so that
eta * a_j^T r is on the scale of a coefficient, since ||a_j||^2 is M/N on
average):
  I = top-K of |A^T y|, x = LS(I), r = y - A x; then repeat
  stop if ||r|| <= 1e-12 ||y||;  c = A^T r;  J = top-l of |c| outside I
  (for l = 1 the argmax);  z = x + eta c on I u J (x_J = 0);
  keep = top-K of |z| over I u J;  stop if no index of J is kept;
  otherwise I = keep, x = LS(I), r = y - A x.  At most ``max_iter`` steps.

CoSaMP (Needell and Tropp, the other greedy neighbour named with OMPR): see
``cosamp``.

Every decision is logged with its margin (FP64 key gap between the last
chosen and the first rejected candidate).
"""
from __future__ import annotations

import dataclasses
import numpy as np

from .operator import SRM
from .lsq import LSContext


def measurement_vector(op, y) -> np.ndarray:
    """y in FP64: complex for an operator with complex measurements (the
    partial complex Fourier operator), real otherwise."""
    return np.asarray(y, dtype=np.complex128 if getattr(op, "complex_meas", False) else np.float64)


def topk_order(keys: np.ndarray, idx: np.ndarray, k: int) -> np.ndarray:
    """Positions of the first k candidates under (key desc, index asc)."""
    order = np.lexsort((idx, -keys))
    return order[:k]


def _margin(keys: np.ndarray, idx: np.ndarray, k: int) -> float:
    if keys.size <= k:
        return float("inf")
    order = np.lexsort((idx, -keys))
    return float(keys[order[k - 1]] - keys[order[k]])


def argmax_excluding(c: np.ndarray, excluded: np.ndarray):
    """argmax_j |c_j| over j not excluded; ties go to the lowest j.

    Returns (j, margin)."""
    key = np.abs(c).astype(np.float64)
    key[excluded] = -1.0
    j = int(np.argmax(key))          # first occurrence = lowest index on ties
    key2 = key.copy()
    key2[j] = -1.0
    second = key2.max()
    return j, float(key[j] - second) if second >= 0 else float("inf")


def topk_excluding(c: np.ndarray, excluded: np.ndarray | None, k: int):
    """Top-k indices of |c| outside ``excluded`` under (|c| desc, j asc), sorted ascending."""
    idx = np.arange(c.size) if excluded is None else np.flatnonzero(~excluded)
    keys = np.abs(c[idx]).astype(np.float64)
    pos = topk_order(keys, idx, k)
    return np.sort(idx[pos]), _margin(keys, idx, k)


@dataclasses.dataclass
class Result:
    s: np.ndarray                 # dense N-vector, zeros off the support
    support: np.ndarray           # int64, ascending
    iters: int                    # outer iterations (OMP: K; SP: rounds; OMPR: swaps)
    resid_norm: float
    trace: list                   # (step, kind, margin)
    stop: str = ""
    supports: list = dataclasses.field(default_factory=list)  # per-iteration support history
    moves: list = dataclasses.field(default_factory=list)     # OMPR: (entered, dropped) index arrays per swap


def _dense(n, supp, vals):
    s = np.zeros(n)
    s[supp] = vals
    return s


def omp(op: SRM, y, K: int, ls_route: str = "auto") -> Result:
    y = measurement_vector(op, y)
    ctx = LSContext(op, y, ls_route)
    r = y.copy()
    S: list[int] = []
    excluded = np.zeros(op.n, dtype=bool)
    trace = []
    vals = np.zeros(0)
    for i in range(1, K + 1):
        c = op.adjoint(r)
        t, m = argmax_excluding(c, excluded)
        trace.append((i, "argmax", m))
        S.append(t)
        excluded[t] = True
        vals = ctx.solve(S)
        r = y - op.apply_sparse(S, vals)
    order = np.argsort(S)
    supp = np.asarray(S, dtype=np.int64)[order]
    return Result(_dense(op.n, supp, vals[order]), supp, K, float(np.linalg.norm(r)), trace, "K iterations")


def sp(op: SRM, y, K: int, max_iter: int = 100, ls_route: str = "auto") -> Result:
    y = measurement_vector(op, y)
    ctx = LSContext(op, y, ls_route)
    trace = []
    T, m = topk_excluding(ctx.aty, None, K)
    trace.append((0, "init_topk", m))
    x = ctx.solve(T)
    r = y - op.apply_sparse(T, x)
    rn = float(np.linalg.norm(r))
    supports = [T]
    stop = "max_iter"
    it = 0
    for it in range(1, max_iter + 1):
        c = op.adjoint(r)
        excl = np.zeros(op.n, dtype=bool)
        excl[T] = True
        D, m = topk_excluding(c, excl, K)
        trace.append((it, "expand_topk", m))
        Tt = np.union1d(T, D)
        xt = ctx.solve(Tt)
        pos = topk_order(np.abs(xt), Tt, K)
        trace.append((it, "prune_topk", _margin(np.abs(xt), Tt, K)))
        Tn = np.sort(Tt[pos])
        xn = ctx.solve(Tn)
        rn_vec = y - op.apply_sparse(Tn, xn)
        rnn = float(np.linalg.norm(rn_vec))
        if np.array_equal(Tn, T):
            x, r, rn = xn, rn_vec, rnn
            supports.append(Tn)
            stop = "support unchanged"
            break
        if rnn > rn:
            stop = "residual increased"
            break
        T, x, r, rn = Tn, xn, rn_vec, rnn
        supports.append(T)
    return Result(_dense(op.n, T, x), np.asarray(T, dtype=np.int64), it, rn, trace, stop, supports)


def ompr(op: SRM, y, K: int, eta: float | None = None, max_iter: int | None = None,
         ls_route: str = "auto", l: int = 1) -> Result:
    y = measurement_vector(op, y)
    if eta is None:
        eta = op.n / op.m
    if max_iter is None:
        max_iter = 4 * K
    ctx = LSContext(op, y, ls_route)
    trace = []
    I, m = topk_excluding(ctx.aty, None, K)
    trace.append((0, "init_topk", m))
    x = ctx.solve(I)
    r = y - op.apply_sparse(I, x)
    ynorm = float(np.linalg.norm(y))
    stop = "max_iter"
    t = 0
    swaps = 0
    moves = []
    for t in range(1, max_iter + 1):
        if np.linalg.norm(r) <= 1e-12 * ynorm:
            stop = "residual zero"
            break
        c = op.adjoint(r)
        excl = np.zeros(op.n, dtype=bool)
        excl[I] = True
        if l == 1:
            j, m = argmax_excluding(c, excl)
            J = np.array([j], dtype=np.int64)
            trace.append((t, "argmax", m))
        else:
            J, m = topk_excluding(c, excl, l)
            trace.append((t, "enter_topl", m))
        cand = np.append(I, J)
        z = np.append(x + eta * c[I], eta * c[J])
        keys = np.abs(z)
        pos = topk_order(keys, cand, K)
        trace.append((t, "drop", _margin(keys, cand, K)))
        keep = np.sort(cand[pos])
        if not np.isin(J, keep).any():
            stop = "no replacement"
            break
        moves.append((np.setdiff1d(keep, I), np.setdiff1d(I, keep)))
        I = keep
        x = ctx.solve(I)
        r = y - op.apply_sparse(I, x)
        swaps += 1
    return Result(_dense(op.n, I, x), np.asarray(I, dtype=np.int64), swaps,
                  float(np.linalg.norm(r)), trace, stop, moves=moves)


def cosamp(op: SRM, y, K: int, max_iter: int = 100, ls_route: str = "auto") -> Result:
    """CoSaMP (Needell and Tropp) on the same selection and least-squares steps.

    Reading: starting from x = 0, r = y, each round takes the top-2K of |A^T r|
    (over all indices: r is not orthogonal to the columns of a pruned x),
    merges them with the current support, solves least squares on the union
    (2K..3K columns), keeps the top-K magnitudes of that solution as the new
    x (no second solve) and updates r = y - A x.  From the second round on it
    stops with the new (T, x) when the support repeats, and with the previous
    one when ||r|| grows, as SP does; at most ``max_iter`` rounds."""
    y = measurement_vector(op, y)
    ctx = LSContext(op, y, ls_route)
    trace = []
    T = np.zeros(0, dtype=np.int64)
    x = np.zeros(0)
    r = y.copy()
    rn = float(np.linalg.norm(r))
    stop = "max_iter"
    it = 0
    for it in range(1, max_iter + 1):
        c = ctx.aty if it == 1 else op.adjoint(r)
        Om, m = topk_excluding(c, None, 2 * K)
        trace.append((it, "merge_top2k", m))
        U = np.union1d(Om, T)
        b = ctx.solve(U)
        pos = topk_order(np.abs(b), U, K)
        trace.append((it, "prune_topk", _margin(np.abs(b), U, K)))
        order = np.argsort(U[pos])
        Tn = U[pos][order]
        xn = b[pos][order]
        rv = y - op.apply_sparse(Tn, xn)
        rnn = float(np.linalg.norm(rv))
        if it > 1 and np.array_equal(Tn, T):
            T, x, r, rn = Tn, xn, rv, rnn
            stop = "support unchanged"
            break
        if it > 1 and rnn > rn:
            stop = "residual increased"
            break
        T, x, r, rn = Tn, xn, rv, rnn
    return Result(_dense(op.n, T, x), np.asarray(T, dtype=np.int64), it, rn, trace, stop)
