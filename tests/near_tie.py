"""Near-tie certificate for an FP32 OMPR trajectory that leaves the FP64 oracle's.

The paper leaves ties unstated (Eq. (6) and the support update of Algorithm 1
rank by magnitude only).  With noise, an OMPR step compares keys (the
correlations |A^T r| outside the support, then |z| = |x + eta A^T r| on the
support plus the entering index) whose FP64 gaps can be smaller than the error
an FP32 path with a relative CG tolerance `tol` makes in them, so several
trajectories are correct.  This module decides, from the oracle alone, whether
a GPU trajectory is one of them.

Key error bound (norm-wise, so it bounds every element):
    eps = kappa * (tol + c_T * u * log2 N) * ||x||_2
with u = 2^-24 (FP32 unit roundoff), c_T = 4 (a transform's rounding grows
with log2 N), ||x|| the least-squares solution on the current support and
kappa = ((1 + sqrt(|S|/M)) / (1 - sqrt(|S|/M)))^2 the condition estimate of
A_S^T A_S (columns of a random row subset of an orthonormal transform behave
like a random matrix scaled by sqrt(M/N)).  Correlation keys take eps (||A|| =
1); the drop keys z = x + eta c take (1 + eta) eps.

A divergent signal is certified when
  1. at the first step where its swaps differ from the oracle's (both start
     from the same support there), the GPU's choice is within 2 eps of the
     oracle's best in the oracle's own FP64 keys (so the oracle's margin at
     that decision is at most 2 eps as well);
  2. replayed through the oracle on the GPU's own supports, each of the next
     `replay` GPU decisions (swaps, and the final decline if it comes within
     them) is 2 eps-optimal in the oracle's keys;
  3. the GPU's final support is a fixed point of the oracle's OMPR step up to
     2 eps (the oracle, on that support, would decline or swap only across a
     2 eps near-tie), and the GPU's s is within relative L2 `s_tol` of the
     oracle's FP64 least squares on that support.
Anything else is reported as a failure with the step and the gaps found.
"""
from __future__ import annotations

import dataclasses

import numpy as np

import oracle

U32 = 2.0 ** -24
C_T = 4.0


@dataclasses.dataclass
class Verdict:
    ok: bool
    step: int                 # first divergent step (0: the initial top-K)
    kind: str                 # which decision diverged
    gap: float                # oracle key gap between the two choices there
    eps: float                # key error bound used there
    replayed: int = 0         # GPU decisions replayed after the divergence
    s_err: float = float("nan")
    why: str = ""


def kappa(k: int, m: int) -> float:
    rho = np.sqrt(k / m)
    return float(((1.0 + rho) / (1.0 - rho)) ** 2)


def eps_keys(n: int, m: int, k: int, x_norm: float, tol: float) -> float:
    return kappa(k, m) * (tol + C_T * U32 * np.log2(n)) * x_norm


class OracleState:
    """Oracle quantities on a support: x = LS(S) (FP64 operator CG to 1e-13,
    warm-started from the previous support's solution), r, c = A^T r."""

    def __init__(self, op, y, eta):
        self.op, self.y, self.eta = op, y, eta
        self.aty = op.adjoint(y)
        self.prev = None      # (support, x)

    def at(self, supp):
        supp = np.asarray(supp, dtype=np.int64)
        x0 = None
        if self.prev is not None:
            ps, px = self.prev
            pos = {int(j): v for j, v in zip(ps, px)}
            x0 = np.array([pos.get(int(j), 0.0) for j in supp])
        x, _ = oracle.ls_cg(self.op, supp, self.y, tol=1e-13, x0=x0, aty=self.aty)
        self.prev = (supp, x)
        r = self.y - self.op.apply_sparse(supp, x)
        c = self.op.adjoint(r)
        return x, c


def _step_check(st: OracleState, supp, gpu_in, gpu_out, tol):
    """One OMPR decision at `supp` in oracle keys.  gpu_in/gpu_out: the GPU's
    swap (None, None when it declined).  Returns (ok, kind, gap, eps, x)."""
    op, eta = st.op, st.eta
    x, c = st.at(supp)
    eps = eps_keys(op.n, op.m, len(supp), float(np.linalg.norm(x)), tol)
    out = np.ones(op.n, dtype=bool)
    out[supp] = False
    ac = np.abs(c)
    j, _ = oracle.argmax_excluding(c, ~out)
    if gpu_in is not None and gpu_in != j:
        gap = float(ac[j] - ac[gpu_in])
        ok = bool(out[gpu_in]) and gap <= 2 * eps
        if not ok:
            return False, "enter", gap, eps, x
        j = gpu_in                      # the drop is judged on the GPU's candidate set
    cand = np.append(supp, j)
    z = np.abs(np.append(x + eta * c[supp], eta * c[j]))
    ez = (1.0 + eta) * eps
    order = np.lexsort((cand, -z))
    last = int(cand[order[-1]])          # the oracle's drop
    if gpu_in is None:                   # the GPU declined: j must rank last up to 2 eps
        gap = float(z[cand == j][0] - z[order[-1]])
        return gap <= 2 * ez, "decline", gap, ez, x
    if gpu_out not in set(cand.tolist()) or gpu_out == j:
        return False, "drop", float("inf"), ez, x
    gap = float(z[cand == gpu_out][0] - z[order[-1]])
    return gap <= 2 * ez, "drop", gap, ez, x


def certify_ompr(op, y, k, tol, eta, oracle_moves, gpu_moves, gpu_support, gpu_s,
                 replay: int = 16, s_tol: float = 1e-5) -> Verdict:
    """oracle_moves / gpu_moves: lists of (entered, left) per swap, in order;
    gpu_support / gpu_s: the GPU's final support and dense s."""
    y = np.asarray(y, dtype=np.float64)
    st = OracleState(op, y, eta)
    # the GPU's initial support: its final one with the swaps undone
    gsets = [set(int(v) for v in gpu_support)]
    for a, b in reversed(gpu_moves):
        s = set(gsets[-1])
        s.discard(int(a))
        s.add(int(b))
        gsets.append(s)
    gsets.reverse()                      # gsets[t]: after t swaps
    init, m0 = oracle.greedy.topk_excluding(st.aty, None, k)
    osupp = set(int(v) for v in init)
    if gsets[0] != osupp:
        # the initial top-K of |A^T y|: every exchanged pair within 2 eps
        key = np.abs(st.aty)
        eps0 = C_T * U32 * np.log2(op.n) * float(np.linalg.norm(y))
        gin = sorted(gsets[0] - osupp)
        oin = sorted(osupp - gsets[0])
        gap = float(key[oin].max() - key[gin].min())
        if gap > 2 * eps0:
            return Verdict(False, 0, "init", gap, eps0, why="initial top-K differs beyond 2 eps")
        t0, kind, gap0, eps_at = 0, "init", gap, eps0
    else:
        t0 = None
        for t in range(max(len(gpu_moves), len(oracle_moves)) + 1):
            om = oracle_moves[t] if t < len(oracle_moves) else None
            gm = gpu_moves[t] if t < len(gpu_moves) else None
            if om is not None and gm is not None and int(om[0]) == int(gm[0]) and int(om[1]) == int(gm[1]):
                continue
            if om is None and gm is None:
                break
            t0 = t
            break
        if t0 is None:
            return Verdict(False, -1, "none", 0.0, 0.0, why="trajectories agree but the results differ")
        supp = np.array(sorted(gsets[t0]))
        gm = gpu_moves[t0] if t0 < len(gpu_moves) else (None, None)
        ok, kind, gap0, eps_at, _ = _step_check(st, supp, None if gm[0] is None else int(gm[0]),
                                                None if gm[1] is None else int(gm[1]), tol)
        if not ok:
            return Verdict(False, t0 + 1, kind, gap0, eps_at, why="first divergent decision is not a near-tie")
        t0 += 1
    # replay the GPU's next decisions through the oracle on its own supports
    replayed = 0
    t = t0
    while replayed < replay and t <= len(gpu_moves):
        supp = np.array(sorted(gsets[t]))
        gm = gpu_moves[t] if t < len(gpu_moves) else (None, None)
        ok, kind, gap, eps, _ = _step_check(st, supp, gm[0], gm[1], tol)
        replayed += 1
        if not ok:
            return Verdict(False, t + 1, kind, gap, eps, replayed, why="a replayed GPU decision is not eps-optimal")
        t += 1
    # the final support: an OMPR fixed point up to 2 eps, and s against the LS on it
    fin = np.asarray(sorted(gsets[-1]))
    if t <= len(gpu_moves):              # the final decline was not replayed above
        ok, kind, gap, eps, _ = _step_check(st, fin, None, None, tol)
        if not ok:
            return Verdict(False, len(gpu_moves) + 1, "final", gap, eps, replayed,
                           why="final support is not an OMPR fixed point up to 2 eps")
    xf = oracle.ls_cg(op, fin, y, tol=1e-13, aty=st.aty)[0]
    ref = np.zeros(op.n)
    ref[fin] = xf
    s_err = float(np.linalg.norm(np.asarray(gpu_s, dtype=np.float64) - ref) / np.linalg.norm(ref))
    if s_err > s_tol:
        return Verdict(False, t0, kind, gap0, eps_at, replayed, s_err, why="s differs from the LS on its support")
    return Verdict(True, t0, kind, gap0, eps_at, replayed, s_err)


# ------------------------------------------------------------------ Subspace Pursuit
#
# An SP round from a support T (SP as Dai and Milenkovic define it, one of the
# greedy methods of Sec. IV) takes D = the top-K of |A^T r| outside T,
# solves least squares on U = T u D, keeps the top-K of |x~| over U and moves
# there unless the residual grew.  The certificate takes the GPU's supports
# after each round (G_0 the initial top-K of |A^T y|, G_1 .. G_R) and checks
# every round in the oracle's FP64 quantities, with witnesses for what the
# GPU does not report:
#   * the expansion D_g: the oracle's D with the lowest-key members that the
#     GPU did not keep traded for the GPU's entering indices outside it; D_g
#     must be a top-K of |c| up to 2 eps (eps as for OMPR, on |T| = K);
#   * the prune: G_t must be a top-K of |x~| over T u D_g up to 2 eps_U
#     (eps on |U| = 2K, with ||x~||);
#   * the move: ||r(G_t)|| <= ||r(G_{t-1})|| + 2 eps (a residual of an FP32
#     least-squares fit carries the same bound as the correlations).
# The final support G_R must be an SP fixed point up to the same bounds: the
# oracle's next round keeps G_R, or keeping G_R is a top-K of |x~| up to
# 2 eps_U, or the oracle's next support has a residual not below ||r(G_R)||
# by more than 2 eps.  G_0 must be a top-K of |A^T y| up to 2 eps_0
# (eps_0 = c_T u log2 N ||y||).


@dataclasses.dataclass
class SPVerdict:
    ok: bool
    round: int                # the round that failed (or -1)
    kind: str                 # "init", "expand", "prune", "move", "final"
    gaps: list                # (round, kind, gap, bound) for every check made
    s_err: float = float("nan")
    why: str = ""


def _topk_gap(keys, idx, chosen):
    """max key among idx outside `chosen` minus min key among `chosen`
    (<= 0 when `chosen` is an exact top-|chosen| of keys over idx)."""
    inside = np.isin(idx, chosen)
    if inside.all() or not inside.any():
        return float("-inf")
    return float(keys[~inside].max() - keys[inside].min())


def _sp_round(st: OracleState, T, k, tol):
    """Oracle quantities for one SP round from T: x, c, eps, r norm, the
    oracle's D (ascending) and the list of indices outside T."""
    op = st.op
    x, c = st.at(T)
    eps = eps_keys(op.n, op.m, len(T), float(np.linalg.norm(x)), tol)
    rn = float(np.linalg.norm(st.y - op.apply_sparse(T, x)))
    excl = np.zeros(op.n, dtype=bool)
    excl[T] = True
    D, _ = oracle.greedy.topk_excluding(c, excl, k)
    return x, c, eps, rn, D, np.flatnonzero(~excl)


def _ls_on(st: OracleState, U):
    op = st.op
    x, _ = oracle.ls_cg(op, U, st.y, tol=1e-13, aty=st.aty)
    return x


def certify_sp(op, y, k, tol, gpu_supports, gpu_s, s_tol: float = 1e-5) -> SPVerdict:
    """gpu_supports: [G_0, G_1, ..., G_R] (index arrays), G_R the returned
    support; consecutive equal supports are allowed only at the end (a
    round that kept the support).  gpu_s: the GPU's dense s."""
    y = np.asarray(y, dtype=np.float64)
    st = OracleState(op, y, 0.0)
    gs = [np.sort(np.asarray(g, dtype=np.int64)) for g in gpu_supports]
    while len(gs) > 1 and np.array_equal(gs[-1], gs[-2]):
        gs.pop()
    gaps = []
    # G_0: a top-K of |A^T y| up to 2 eps_0
    key0 = np.abs(st.aty)
    eps0 = C_T * U32 * np.log2(op.n) * float(np.linalg.norm(y))
    g = _topk_gap(key0, np.arange(op.n), gs[0])
    gaps.append((0, "init", g, 2 * eps0))
    if g > 2 * eps0:
        return SPVerdict(False, 0, "init", gaps, why="G_0 is not a top-K of |A^T y| up to 2 eps")
    for t in range(1, len(gs) + 1):
        T = gs[t - 1]
        x, c, eps, rn, D, outside = _sp_round(st, T, k, tol)
        ac = np.abs(c)
        final = t == len(gs)
        if final:
            # the next round: the oracle's own, from G_R
            U = np.union1d(T, D)
            xt = _ls_on(st, U)
            epsu = eps_keys(op.n, op.m, len(U), float(np.linalg.norm(xt)), tol)
            g = _topk_gap(np.abs(xt), U, T)
            gaps.append((t, "final-keep", g, 2 * epsu))
            if g <= 2 * epsu:
                break
            Tn = np.sort(U[oracle.greedy.topk_order(np.abs(xt), U, k)])
            xn = _ls_on(st, Tn)
            rnn = float(np.linalg.norm(y - op.apply_sparse(Tn, xn)))
            gaps.append((t, "final-resid", rn - rnn, 2 * eps))
            if rn - rnn <= 2 * eps:
                break
            return SPVerdict(False, t, "final", gaps,
                             why="the final support is not an SP fixed point up to 2 eps")
        G = gs[t]
        E = np.setdiff1d(G, T)
        extra = np.setdiff1d(E, D)
        if extra.size:
            spare = np.setdiff1d(D, G)
            if spare.size < extra.size:
                return SPVerdict(False, t, "expand", gaps, why="more entering indices than D can hold")
            spare = spare[np.argsort(ac[spare], kind="stable")][: extra.size]
            Dg = np.union1d(np.setdiff1d(D, spare), extra)
        else:
            Dg = D
        g = _topk_gap(ac[outside], outside, Dg)
        gaps.append((t, "expand", g, 2 * eps))
        if g > 2 * eps:
            return SPVerdict(False, t, "expand", gaps, why="no expansion within 2 eps explains G_t")
        U = np.union1d(T, Dg)
        if not np.isin(G, U).all():
            return SPVerdict(False, t, "prune", gaps, why="G_t leaves T u D")
        xt = _ls_on(st, U)
        epsu = eps_keys(op.n, op.m, len(U), float(np.linalg.norm(xt)), tol)
        g = _topk_gap(np.abs(xt), U, G)
        gaps.append((t, "prune", g, 2 * epsu))
        if g > 2 * epsu:
            return SPVerdict(False, t, "prune", gaps, why="G_t is not a top-K of |x~| up to 2 eps")
        xg = _ls_on(st, G)
        rng_ = float(np.linalg.norm(y - op.apply_sparse(G, xg)))
        gaps.append((t, "move", rng_ - rn, 2 * eps))
        if rng_ - rn > 2 * eps:
            return SPVerdict(False, t, "move", gaps, why="the residual grew by more than 2 eps")
    fin = gs[-1]
    xf = _ls_on(st, fin)
    ref = np.zeros(op.n)
    ref[fin] = xf
    s_err = float(np.linalg.norm(np.asarray(gpu_s, dtype=np.float64) - ref) / np.linalg.norm(ref))
    if s_err > s_tol:
        return SPVerdict(False, len(gs), "s", gaps, s_err, why="s differs from the LS on its support")
    return SPVerdict(True, -1, "", gaps, s_err)
