"""Pins of the FP64 oracle against facts fixed by the mathematics and the paper.

Each pin checks the oracle against something other than itself: a textbook
identity, a closed form, an invariant stated by the paper's theorems, a
special case that reduces to a known answer, or exhaustive search.  The
planted-mistake tests at the end make sure that plausible slips in the
oracle (wrong DCT type, dropped sign flip, dropped Hankel term, transposed
operand, wrong tie order) are caught by at least one pin.
"""
import itertools

import numpy as np
import pytest

import oracle
import synth
from oracle import operator as oop
import importlib
ogram = importlib.import_module("oracle.gram")
from oracle import greedy as ogreedy
from tests.problems import problem

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


# ------------------------------------------------------------------ P1 DCT
def pin_dct_formula(n=64, seed=0):
    """SciPy route equals the dense cosine formula; F is orthonormal."""
    rng = np.random.default_rng(seed)
    F = oracle.dct2_matrix(n)
    x = rng.standard_normal(n)
    op = oracle.SRM(n, np.arange(n), np.ones(n, dtype=np.int8))
    ok1 = np.allclose(op.apply(x), F @ x, atol=1e-13, rtol=0)
    ok2 = np.allclose(F @ F.T, np.eye(n), atol=1e-13)
    return ok1 and ok2


def pin_dct_basis(n=128):
    """Textbook cosine orthogonality: sum_n cos(pi(2n+1)k/2N) cos(pi(2n+1)k0/2N) = N/2 [k=k0>0],
    so the DCT-II of that cosine is sqrt(N/2) at k0 and 0 elsewhere; the DCT-II of all-ones is sqrt(N) e_0."""
    op = oracle.SRM(n, np.arange(n), np.ones(n, dtype=np.int8))
    ok = True
    nn = np.arange(n)
    for k0 in (1, 5, n // 2, n - 1):
        a = ((2 * nn + 1) * k0) % (4 * n)          # exact angle reduction
        x = np.cos(np.pi * a / (2 * n))
        e = np.zeros(n)
        e[k0] = np.sqrt(n / 2)
        ok &= np.allclose(op.apply(x), e, atol=1e-13 * np.sqrt(n))
    e = np.zeros(n)
    e[0] = np.sqrt(n)
    ok &= np.allclose(op.apply(np.ones(n)), e, atol=1e-13 * np.sqrt(n))
    return bool(ok)


def test_p1_dct_formula():
    for n in (8, 64, 256, 1000):
        assert pin_dct_formula(n)


def test_p1_dct_basis():
    assert pin_dct_basis(128)
    assert pin_dct_basis(4096)


# ------------------------------------------------------------------ P2 A, A^T
def pin_adjoint(n=256, m=77, seed=1):
    """A A^T = I_M (rows of an orthonormal matrix) and <A x, u> = <x, A^T u>;
    the FFT route agrees with the dense formula for A and A^T."""
    rng = np.random.default_rng(seed)
    rows, signs = synth.draw_operator(rng, n, m)
    op = oracle.SRM(n, rows, signs)
    x = rng.standard_normal(n)
    u = rng.standard_normal(m)
    A = op.dense()
    ok = np.allclose(op.apply(op.adjoint(u)), u, atol=1e-13)
    ok &= abs(op.apply(x) @ u - x @ op.adjoint(u)) < 1e-12
    ok &= np.allclose(op.apply(x), A @ x, atol=1e-13)
    ok &= np.allclose(op.adjoint(u), A.T @ u, atol=1e-13)
    ok &= np.allclose(A @ A.T, np.eye(m), atol=1e-13)
    return bool(ok)


def test_p2_adjoint():
    assert pin_adjoint()
    assert pin_adjoint(1024, 300, 2)


# ------------------------------------------------------------------ P3 Gram
def pin_gram(n=256, m=90, k=20, seed=3):
    rng = np.random.default_rng(seed)
    rows, signs = synth.draw_operator(rng, n, m)
    op = oracle.SRM(n, rows, signs)
    S = np.sort(rng.choice(n, k, replace=False))
    S[0] = 0            # include both ends: j = 0 and j = N-1
    S[-1] = n - 1
    As = op.columns(S)
    return bool(np.allclose(oracle.gram_matrix(op, S), As.T @ As, atol=1e-13))


def test_p3_gram():
    assert pin_gram()
    assert pin_gram(4096, 1024, 50, 4)


def test_p3_gram_row0_dc():
    # the DC row (k = 0) has a different scale c_0; make sure it is sampled
    n = 64
    rows = np.array([0, 1, 7, 20, 33, 63])
    signs = np.ones(n, dtype=np.int8)
    signs[::3] = -1
    op = oracle.SRM(n, rows, signs)
    S = np.array([0, 5, 31, 62, 63])
    As = op.columns(S)
    assert np.allclose(oracle.gram_matrix(op, S), As.T @ As, atol=1e-14)


# ------------------------------------------------------------------ P4 LS
def pin_ls_routes(seed=5, n=1024, m=256, k=40, snr=30.0):
    d, op, y = problem(90, seed, n, m, k, "normal", snr)
    S = np.sort(np.concatenate([d.supp[:30], np.setdiff1d(np.arange(n), d.supp)[:10]]))
    a = oracle.ls_dense(op, S, y)
    b = oracle.ls_gram(op, S, y)
    c, _ = oracle.ls_cg(op, S, y, tol=1e-14)
    ok = np.allclose(a, b, atol=1e-12, rtol=0) and np.allclose(a, c, atol=1e-11, rtol=0)
    # Theorems 1-2: the residual is orthogonal to the selected columns
    r = y - op.apply_sparse(S, a)
    ok &= np.linalg.norm(op.columns(S).T @ r) <= 1e-12 * np.linalg.norm(y)
    return bool(ok)


def test_p4_ls_routes_agree_and_orthogonal():
    assert pin_ls_routes()


def test_p4_noiseless_true_support_exact():
    d, op, y = problem(91, 0, 4096, 1024, 50, "normal_min0.1")
    v = oracle.ls(op, d.supp, y)
    assert np.allclose(v, d.vals, atol=1e-12)


def test_p4_single_column_closed_form():
    d, op, y = problem(92, 0, 512, 128, 5, "normal", 20.0)
    t = np.array([37])
    a = op.columns(t)[:, 0]
    assert np.allclose(oracle.ls(op, t, y), [a @ y / (a @ a)], rtol=1e-13)


# ------------------------------------------------------------------ P5 CG (Theorems 4-5)
def test_p5_cg_iteration_bound():
    """Theorem 5: at most |S| iterations (exact arithmetic); allow +2 for rounding."""
    for k in (1, 4, 9, 16):
        d, op, y = problem(93, k, 512, 160, k, "normal", 25.0)
        S = d.supp
        v, it = oracle.ls_cg(op, S, y, tol=1e-12)
        assert it <= k + 2, (k, it)
        assert np.allclose(v, oracle.ls_dense(op, S, y), atol=1e-10)


def test_p5_cg_orthogonal_operator_one_step():
    """M = N makes A orthogonal, A_S^T A_S = I has one eigenvalue: CG stops after 1 iteration (Theorem 4)."""
    rng = np.random.default_rng(7)
    n = 256
    op = oracle.SRM(n, np.arange(n), synth.draw_operator(rng, n, n)[1])
    y = rng.standard_normal(n)
    S = np.sort(rng.choice(n, 30, replace=False))
    v, it = oracle.ls_cg(op, S, y, tol=1e-13)
    assert it == 1
    assert np.allclose(v, op.adjoint(y)[S], atol=1e-13)


# ------------------------------------------------------------------ P6 M = N
def pin_orthogonal_special_case(seed=11, n=512, k=20):
    """With M = N, A is orthogonal, LS on any S is (A^T y)_S and all three
    algorithms return hard thresholding H_K(A^T y)."""
    rng = np.random.default_rng(seed)
    rows, signs = synth.draw_operator(rng, n, n)
    op = oracle.SRM(n, rows, signs)
    y = rng.standard_normal(n)
    c = op.adjoint(y)
    expect = np.sort(np.argsort(-np.abs(c), kind="stable")[:k])
    ok = True
    for f in (oracle.omp, oracle.sp, oracle.ompr):
        kw = {"eta": 1.0} if f is oracle.ompr else {}
        r = f(op, y, k, **kw)
        ok &= np.array_equal(r.support, expect)
        ok &= np.allclose(r.s[expect], c[expect], atol=1e-12)
        if f is oracle.sp:
            ok &= r.iters == 1
        if f is oracle.ompr:
            ok &= r.iters == 0
    return bool(ok)


def test_p6_orthogonal_special_case():
    assert pin_orthogonal_special_case()


def test_p6_orthogonal_special_case_cosamp_omprl():
    """M = N: CoSaMP's first round gives H_K(A^T y), the second repeats it
    (the new correlation vanishes on T and the solve on the union is c there);
    OMPR with l = 3 and eta = 1 finds nothing to replace."""
    rng = np.random.default_rng(13)
    n, k = 512, 20
    rows, signs = synth.draw_operator(rng, n, n)
    op = oracle.SRM(n, rows, signs)
    y = rng.standard_normal(n)
    c = op.adjoint(y)
    expect = np.sort(np.argsort(-np.abs(c), kind="stable")[:k])
    r = oracle.cosamp(op, y, k)
    assert np.array_equal(r.support, expect) and r.iters == 2 and r.stop == "support unchanged"
    assert np.allclose(r.s[expect], c[expect], atol=1e-12)
    q = oracle.ompr(op, y, k, eta=1.0, l=3)
    assert np.array_equal(q.support, expect) and q.iters == 0 and q.stop == "no replacement"


def test_p6_omp_picks_in_decreasing_magnitude():
    rng = np.random.default_rng(12)
    n = 128
    op = oracle.SRM(n, np.arange(n), synth.draw_operator(rng, n, n)[1])
    y = rng.standard_normal(n)
    c = np.abs(op.adjoint(y))
    r = oracle.omp(op, y, 10)
    picks = [t[2] for t in r.trace]
    assert len(picks) == 10
    # the picks follow |c| order: reconstruct from the support
    assert np.array_equal(r.support, np.sort(np.argsort(-c, kind="stable")[:10]))


# ------------------------------------------------------------------ P7 brute force
def _erc(op, S):
    """Tropp's exact recovery condition max_{j not in S} ||A_S^+ a_j||_1 < 1."""
    A = op.dense()
    pinv = np.linalg.pinv(A[:, S])
    others = np.setdiff1d(np.arange(op.n), S)
    return float(np.max(np.abs(pinv @ A[:, others]).sum(axis=0)))


def test_p7_bruteforce_and_omp_under_erc():
    certified = 0
    for seed in range(40):
        d, op, y = problem(94, seed, 16, 10, 2, "normal_min0.1")
        supp, vals, rn = oracle.l0_bruteforce(op, y, 2)
        # noiseless: the true support gives zero residual, so the minimiser does too
        assert rn < 1e-10
        if np.array_equal(supp, d.supp):
            assert np.allclose(vals, d.vals, atol=1e-10)
        if _erc(op, d.supp) < 1.0:
            certified += 1
            r = oracle.omp(op, y, 2)
            assert np.array_equal(r.support, supp)
            assert np.array_equal(r.support, d.supp)
    assert certified >= 5


def test_p7_bruteforce_is_optimal_for_greedy():
    for seed in range(10):
        d, op, y = problem(95, seed, 14, 8, 2, "normal", 15.0)
        _, _, rn = oracle.l0_bruteforce(op, y, 2)
        for f in (oracle.omp, oracle.sp, oracle.ompr, oracle.cosamp):
            assert f(op, y, 2).resid_norm >= rn - 1e-12
        assert oracle.ompr(op, y, 2, l=2).resid_norm >= rn - 1e-12


def test_p7_sp_ompr_single_atom_certificate():
    """K = 1, noiseless y = v a_t: A^T y = v A^T a_t, so whenever ||a_t||^2 exceeds
    every |a_j^T a_t| (j != t) the top-1 of |A^T y| is t, the LS fit is exact and
    SP and OMPR must both return {t} with value v (and equal the l0 minimiser)."""
    certified = 0
    for seed in range(30):
        d, op, y = problem(96, seed, 16, 9, 1, "normal_min0.1")
        A = op.dense()
        t = int(d.supp[0])
        gram_col = np.abs(A.T @ A[:, t])
        if gram_col[t] > np.max(np.delete(gram_col, t)):
            certified += 1
            supp, vals, _ = oracle.l0_bruteforce(op, y, 1)
            for f in (oracle.sp, oracle.ompr):
                r = f(op, y, 1)
                assert np.array_equal(r.support, d.supp) and np.array_equal(r.support, supp)
                assert np.allclose(r.s[t], d.vals[0], atol=1e-12)
    assert certified >= 5


def test_p7_sp_ompr_fixed_points():
    """The returned support satisfies the algorithm's own stopping rule: one more
    SP round from it does not lower the residual, and OMPR finds no replacement."""
    d, op, y = problem(100, 0, 1024, 256, 20, "normal", 15.0)
    r = oracle.sp(op, y, 20)
    T = r.support
    c = op.adjoint(y - op.apply(r.s))
    excl = np.zeros(op.n, dtype=bool)
    excl[T] = True
    D, _ = ogreedy.topk_excluding(c, excl, 20)
    Tt = np.union1d(T, D)
    xt = oracle.ls(op, Tt, y)
    Tn = np.sort(Tt[ogreedy.topk_order(np.abs(xt), Tt, 20)])
    rn = np.linalg.norm(y - op.apply_sparse(Tn, oracle.ls(op, Tn, y)))
    assert np.array_equal(Tn, T) or rn >= r.resid_norm * (1 - 1e-12)
    q = oracle.ompr(op, y, 20)
    if q.stop == "no replacement":
        I = q.support
        c = op.adjoint(y - op.apply(q.s))
        excl = np.zeros(op.n, dtype=bool)
        excl[I] = True
        j, _ = oracle.argmax_excluding(c, excl)
        eta = op.n / op.m
        z = np.append(q.s[I] + eta * c[I], eta * c[j])
        cand = np.append(I, j)
        assert j not in cand[ogreedy.topk_order(np.abs(z), cand, 20)]


def test_p7_ompr_l_fixed_point():
    """OMPR with l = 4 stops only when none of the l entering indices survives
    the top-K of |x + eta A^T r| over I u J."""
    d, op, y = problem(101, 0, 1024, 300, 20, "normal", 15.0)
    q = oracle.ompr(op, y, 20, l=4)
    if q.stop == "no replacement":
        I = q.support
        c = op.adjoint(y - op.apply(q.s))
        excl = np.zeros(op.n, dtype=bool)
        excl[I] = True
        J, _ = ogreedy.topk_excluding(c, excl, 4)
        eta = op.n / op.m
        z = np.append(q.s[I] + eta * c[I], eta * c[J])
        cand = np.append(I, J)
        assert not np.isin(J, cand[ogreedy.topk_order(np.abs(z), cand, 20)]).any()


def test_cosamp_first_round_from_its_definition():
    """One CoSaMP round from x = 0, written out with numpy's own sort: merge the
    2K largest |A^T y|, solve least squares on them by dense lstsq, keep the K
    largest entries of that solution (no second solve)."""
    d, op, y = problem(102, 0, 2048, 600, 25, "normal", 25.0)
    k = 25
    r = oracle.cosamp(op, y, k, max_iter=1)
    c = op.adjoint(y)
    U = np.sort(np.lexsort((np.arange(op.n), -np.abs(c)))[:2 * k])
    b = np.linalg.lstsq(op.columns(U), y, rcond=None)[0]
    keep = np.lexsort((U, -np.abs(b)))[:k]
    T = np.sort(U[keep])
    assert np.array_equal(r.support, T)
    assert np.allclose(r.s[T], b[np.searchsorted(U, T)], atol=1e-11)
    # the pruned least-squares estimate is not the least-squares fit on T
    assert not np.allclose(r.s[T], np.linalg.lstsq(op.columns(T), y, rcond=None)[0], atol=1e-6)


# ------------------------------------------------------------------ exact recovery of well-separated signals
@pytest.mark.parametrize("algo", ["omp", "sp", "ompr", "cosamp", "ompr_l3"])
def test_exact_recovery_well_separated(algo):
    d, op, y = problem(97, 0, 4096, 1024, 50, "normal_min0.1")
    if algo == "ompr_l3":
        r = oracle.ompr(op, y, 50, l=3)
    else:
        r = getattr(oracle, algo)(op, y, 50)
    assert np.array_equal(r.support, d.supp)
    assert np.linalg.norm(r.s - d.s_dense()) <= 1e-12 * np.linalg.norm(d.vals)
    # final residual orthogonal to A_S
    res = y - op.apply(r.s)
    assert np.linalg.norm(op.columns(r.support).T @ res) <= 1e-12 * np.linalg.norm(y)


@pytest.mark.parametrize("algo", ["omp", "sp", "ompr"])
def test_noisy_residual_orthogonal(algo):
    d, op, y = problem(98, 0, 2048, 512, 30, "normal", 20.0)
    r = getattr(oracle, algo)(op, y, 30)
    res = y - op.apply(r.s)
    assert len(r.support) == 30
    assert np.linalg.norm(op.columns(r.support).T @ res) <= 1e-11 * np.linalg.norm(y)


# ------------------------------------------------------------------ P8 selection
def test_p8_selection_ties():
    keys = np.array([3.0, 1.0, 3.0, 0.0, -0.0, 2.0, 3.0, 1.0, 2.0, 0.0])
    idx = np.arange(keys.size)
    ref = sorted(idx.tolist(), key=lambda j: (-abs(keys[j]), j))
    for k in range(1, keys.size + 1):
        pos = ogreedy.topk_order(np.abs(keys), idx, k)
        assert idx[pos].tolist() == ref[:k]
    excl = np.zeros(keys.size, dtype=bool)
    excl[0] = True
    j, m = oracle.argmax_excluding(keys, excl)
    assert j == 2 and m == 0.0
    allzero = np.zeros(7)
    assert oracle.argmax_excluding(allzero, np.zeros(7, dtype=bool))[0] == 0
    sel, _ = ogreedy.topk_excluding(allzero, np.array([True, False, True, False, False, False, False]), 3)
    assert sel.tolist() == [1, 3, 4]


# ------------------------------------------------------------------ decision margins
def test_margins_from_their_definition():
    """The logged margin of a selection is the key of the last chosen
    candidate minus the key of the first rejected one, ranked by (key desc,
    index asc): hand-made keys with known gaps, ties (margin 0) and
    exclusions."""
    keys = np.array([5.0, 3.0, 3.0, 1.0])
    idx = np.arange(4)
    assert ogreedy._margin(keys, idx, 1) == 2.0
    assert ogreedy._margin(keys, idx, 2) == 0.0
    assert ogreedy._margin(keys, idx, 3) == 2.0
    assert ogreedy._margin(keys, idx, 4) == float("inf")       # nothing rejected
    c = np.array([9.0, -4.0, 7.0, -7.0, 1.0])
    excl = np.array([True, False, False, False, False])
    assert oracle.argmax_excluding(c, excl) == (2, 0.0)        # |7| twice: lowest index, margin 0
    assert oracle.argmax_excluding(np.array([9.0, 4.0, -7.0, 6.0]), excl[:4]) == (2, 1.0)
    sel, m = ogreedy.topk_excluding(np.array([0.5, -2.0, 1.5, 0.25, -3.0]), excl, 2)
    assert sel.tolist() == [1, 4] and m == 0.5                  # 2.0 kept, 1.5 rejected


def _sorted_gaps(c):
    a = np.sort(np.abs(c))[::-1]
    return a[:-1] - a[1:]


def test_trace_margins_in_the_orthogonal_case():
    """M = N (A orthogonal): A^T y is computed here from the cosine formula
    written out, independently of the oracle's operator.  Every decision of
    the three algorithms then reduces to a ranking of |A^T y| (the LS on S
    is (A^T y)_S and A^T r is A^T y with S zeroed), so each logged margin
    is a gap of the sorted magnitudes: OMP's i-th argmax the gap after the
    i-th largest, SP's initial top-K and its prune the gap after the K-th,
    its expansion the gap after the 2K-th, and OMPR's (eta = 1) entering
    argmax and drop the gaps after the (K+1)-th and the K-th."""
    rng = np.random.default_rng(41)
    n, k = 256, 12
    rows, signs = synth.draw_operator(rng, n, n)
    op = oracle.SRM(n, rows, signs)
    y = rng.standard_normal(n)
    kk = np.arange(n)[:, None]
    jj = np.arange(n)[None, :]
    F = np.where(kk == 0, np.sqrt(1.0 / n), np.sqrt(2.0 / n)) * np.cos(np.pi * (2 * jj + 1) * kk / (2 * n))
    c = signs * (F.T @ y)
    gap = _sorted_gaps(c)
    r = oracle.omp(op, y, k)
    got = np.array([m for (_, kind, m) in r.trace if kind == "argmax"])
    assert np.allclose(got, gap[:k], rtol=0, atol=1e-12)
    r = oracle.sp(op, y, k)
    tr = {kind: m for (_, kind, m) in r.trace}
    assert abs(tr["init_topk"] - gap[k - 1]) <= 1e-12
    assert abs(tr["expand_topk"] - gap[2 * k - 1]) <= 1e-12      # top-K outside T: ranks K+1..2K
    assert abs(tr["prune_topk"] - gap[k - 1]) <= 1e-12
    r = oracle.ompr(op, y, k, eta=1.0)
    tr = {kind: m for (_, kind, m) in r.trace}
    assert abs(tr["argmax"] - gap[k]) <= 1e-12
    assert abs(tr["drop"] - gap[k - 1]) <= 1e-12
    assert r.stop == "no replacement" and r.moves == []


def _ompr_first_step(A, y, K, eta):
    """One OMPR step written out with dense algebra: the support after it,
    or None if the step declines to swap."""
    n = A.shape[1]
    c0 = A.T @ y
    I = np.sort(sorted(range(n), key=lambda j: (-abs(c0[j]), j))[:K])
    x, *_ = np.linalg.lstsq(A[:, I], y, rcond=None)
    c = A.T @ (y - A[:, I] @ x)
    out = [j for j in range(n) if j not in set(I.tolist())]
    j = sorted(out, key=lambda q: (-abs(c[q]), q))[0]
    cand = list(I) + [j]
    z = dict(zip(I.tolist(), (x + eta * c[I]).tolist()))
    z[j] = eta * c[j]
    keep = sorted(sorted(cand, key=lambda q: (-abs(z[q]), q))[:K])
    return None if j not in keep else np.array(keep)


def test_ompr_default_step_is_n_over_m():
    """OMPR's step eta defaults to N/M (the reading: ||a_j||^2 = M/N on
    average, so eta a_j^T r is on a coefficient's scale).  On tiny problems
    whose first step decides differently for eta = N/M, 1 and M/N (a dense
    sensing matrix from the cosine formula, LS by lstsq), the oracle's first
    step with its default must follow eta = N/M."""
    n, m, K = 32, 8, 2
    kk = np.arange(n)[:, None]
    jj = np.arange(n)[None, :]
    F = np.where(kk == 0, np.sqrt(1.0 / n), np.sqrt(2.0 / n)) * np.cos(np.pi * (2 * jj + 1) * kk / (2 * n))
    found = 0
    for seed in range(400):
        rng = np.random.default_rng([77, seed])
        rows, signs = synth.draw_operator(rng, n, m)
        A = F[rows, :] * signs[None, :]
        y = rng.standard_normal(m)
        outcomes = {e: _ompr_first_step(A, y, K, e) for e in (n / m, 1.0, m / n)}
        key = lambda v: None if v is None else tuple(v.tolist())
        if key(outcomes[n / m]) == key(outcomes[1.0]) or key(outcomes[n / m]) == key(outcomes[m / n]):
            continue
        r = oracle.ompr(oracle.SRM(n, rows, signs), y, K, max_iter=1)
        if outcomes[n / m] is None:
            assert r.stop == "no replacement" and r.moves == [], seed
        else:
            assert r.iters == 1 and np.array_equal(r.support, outcomes[n / m]), seed
        found += 1
        if found == 5:
            break
    assert found == 5


def test_margin_and_step_pins_catch_planted_mistakes(monkeypatch):
    """A margin taken one rank too far, and OMPR's step inverted (M/N) or
    left at 1, each fail the pins above."""
    real_margin = ogreedy._margin

    def margin_off_by_one(keys, idx, k):
        return real_margin(keys, idx, k + 1) if keys.size > k + 1 else real_margin(keys, idx, k)

    with monkeypatch.context() as mp:
        mp.setattr(ogreedy, "_margin", margin_off_by_one)
        with pytest.raises(AssertionError):
            test_margins_from_their_definition()
    real_ompr = ogreedy.ompr
    for wrong in (lambda op: op.m / op.n, lambda op: 1.0):
        def ompr_wrong_eta(op, y, K, eta=None, *a, _w=wrong, **kw):
            return real_ompr(op, y, K, _w(op) if eta is None else eta, *a, **kw)
        with monkeypatch.context() as mp:
            mp.setattr(oracle, "ompr", ompr_wrong_eta)
            with pytest.raises(AssertionError):
                test_ompr_default_step_is_n_over_m()


# ------------------------------------------------------------------ P9 adjoint
def test_p9_adjoint_matches_central_differences():
    d, op, y = problem(99, 0, 1024, 256, 12, "normal", 30.0)
    t = d.s_dense()
    S = d.supp
    g, _ = oracle.adjoint_gradient(op, S, y, t)

    def loss(yy):
        v = oracle.ls_dense(op, S, yy)
        s = np.zeros(op.n)
        s[S] = v
        return float(np.sum((s - t) ** 2))

    rng = np.random.default_rng(0)
    for c in rng.choice(op.m, 16, replace=False):
        h = 1e-3
        e = np.zeros(op.m)
        e[c] = h
        fd = (loss(y + e) - loss(y - e)) / (2 * h)
        assert abs(fd - g[c]) <= 1e-7 * max(1.0, abs(g[c])), (c, fd, g[c])


# ------------------------------------------------------------------ planted mistakes
def _mutants():
    import scipy.fft as sfft

    def apply_dct3(self, x):
        return sfft.dct(self.signs * np.asarray(x, float), type=3, norm="ortho")[self.rows]

    def adjoint_nosign(self, u):
        full = np.zeros(self.n)
        full[self.rows] = u
        return sfft.idct(full, type=2, norm="ortho")

    def gram_no_hankel(op, supp, g=None):
        if g is None:
            g = ogram.gram_generator(op)
        s = np.asarray(supp, dtype=np.int64)
        sg = op.signs[s]
        return 0.5 * (sg[:, None] * sg[None, :]) * (g[np.abs(s[:, None] - s[None, :])] * 2)

    def gram_minus(op, supp, g=None):
        if g is None:
            g = ogram.gram_generator(op)
        s = np.asarray(supp, dtype=np.int64)
        sg = op.signs[s]
        return 0.5 * (sg[:, None] * sg[None, :]) * (g[np.abs(s[:, None] - s[None, :])] - g[s[:, None] + s[None, :] + 1])

    def columns_transposed_angle(self, supp):
        j = np.asarray(supp, dtype=np.int64)[None, :]
        k = self.rows[:, None]
        return oop._dct_scale(k, self.n) * oop._cos_table(j, k, self.n) * self.signs[j]

    def topk_order_wrong_ties(keys, idx, k):
        return np.lexsort((-idx, -keys))[:k]

    return {
        "dct type 3 instead of 2": (oop.SRM, "apply", apply_dct3),
        "adjoint drops sign flip": (oop.SRM, "adjoint", adjoint_nosign),
        "gram drops Hankel term": (ogram, "gram_matrix", gram_no_hankel),
        "gram wrong sign": (ogram, "gram_matrix", gram_minus),
        "columns transposed angle": (oop.SRM, "columns", columns_transposed_angle),
        "ties to highest index": (ogreedy, "topk_order", topk_order_wrong_ties),
    }


ALL_PINS = [pin_dct_formula, pin_dct_basis, pin_adjoint, pin_gram, pin_ls_routes,
            pin_orthogonal_special_case]


def _pin_ties():
    keys = np.array([2.0, 1.0, 2.0, 2.0])
    idx = np.arange(4)
    return ogreedy.topk_order(keys, idx, 2).tolist() == [0, 2]


@pytest.mark.parametrize("name", list(_mutants().keys()))
def test_planted_mistake_is_caught(name, monkeypatch):
    target, attr, repl = _mutants()[name]
    monkeypatch.setattr(target, attr, repl)
    # oracle/__init__ re-exports some names; patch those too
    if target is ogram and attr == "gram_matrix":
        monkeypatch.setattr(importlib.import_module("oracle.lsq"), "gram_matrix", repl)
        monkeypatch.setattr(oracle, "gram_matrix", repl)
    if target is ogreedy and attr == "topk_order":
        monkeypatch.setattr(oracle, "topk_order", repl)
    results = []
    for pin in ALL_PINS + [_pin_ties]:
        try:
            results.append(bool(pin()))
        except Exception:
            results.append(False)
    assert not all(results), f"no pin caught: {name}"


def test_all_pins_pass_unmutated():
    assert all(p() for p in ALL_PINS + [_pin_ties])


# ------------------------------------------------------------------ permutation randomizer
@pytest.mark.parametrize("randomizer", ["perm", "signed_perm"])
def test_p2_permutation_randomizer(randomizer):
    """R as a permutation (the paper's SRM): the FFT route equals the cosine
    formula, A A^T = I, the closed-form Gram equals A_S^T A_S, and A equals the
    unpermuted operator applied to the scattered vector (x'[perm[j]] = x[j])."""
    d = synth.draw_problem(103, 0, 512, 150, 10, "normal", None, randomizer=randomizer)
    op = oracle.SRM(d.n, d.rows, d.signs, d.perm)
    plain = oracle.SRM(d.n, d.rows, d.signs if randomizer == "signed_perm" else np.ones(d.n))
    rng = np.random.default_rng(5)
    x = rng.standard_normal(d.n)
    u = rng.standard_normal(d.m)
    assert np.allclose(op.apply(x), op.dense() @ x, atol=1e-12)
    assert np.allclose(op.apply(op.adjoint(u)), u, atol=1e-13)
    assert abs(op.apply(x) @ u - x @ op.adjoint(u)) < 1e-11
    xs = np.zeros(d.n)
    xs[d.perm] = d.signs * x                      # R x written out
    assert np.allclose(op.apply(x), oracle.SRM(d.n, d.rows, np.ones(d.n)).apply(xs), atol=1e-13)
    S = np.sort(rng.choice(d.n, 25, replace=False))
    a = op.columns(S)
    assert np.allclose(oracle.gram_matrix(op, S), a.T @ a, atol=1e-12)
    assert not np.allclose(op.columns(S), plain.columns(S))        # the permutation matters
    # recovery on the permuted operator: noiseless, well separated
    dd = synth.draw_problem(104, 0, 2048, 512, 25, "normal_min0.1", None, randomizer=randomizer)
    o2 = oracle.SRM(dd.n, dd.rows, dd.signs, dd.perm)
    y = o2.apply_sparse(dd.supp, dd.vals)
    for f in (oracle.omp, oracle.sp, oracle.ompr, oracle.cosamp):
        r = f(o2, y, 25)
        assert np.array_equal(r.support, dd.supp), f.__name__


# ------------------------------------------------------------------ DCT sparsifying basis
@pytest.mark.parametrize("randomizer", ["signs", "perm"])
def test_p2_dct_basis(randomizer):
    """Psi = F (the paper's experiments): A = D F R F equals the product of
    the dense cosine-formula matrices, has orthonormal rows, and its columns
    and adjoint agree with that product; a basis taken as F^T instead of F,
    or left out, gives a different operator."""
    d = synth.draw_problem(105, 0, 256, 90, 8, "normal", None, randomizer=randomizer)
    op = oracle.SRM(d.n, d.rows, d.signs, d.perm, psi=1)
    Fm = oracle.dct2_matrix(d.n)
    Rm = np.zeros((d.n, d.n))
    idx = d.perm if d.perm is not None else np.arange(d.n)
    Rm[idx, np.arange(d.n)] = d.signs
    A = Fm[d.rows] @ Rm @ Fm
    rng = np.random.default_rng(6)
    x = rng.standard_normal(d.n)
    u = rng.standard_normal(d.m)
    assert np.allclose(op.apply(x), A @ x, atol=1e-12)
    assert np.allclose(op.adjoint(u), A.T @ u, atol=1e-12)
    assert np.allclose(A @ A.T, np.eye(d.m), atol=1e-12)
    S = np.sort(rng.choice(d.n, 12, replace=False))
    assert np.allclose(op.columns(S), A[:, S], atol=1e-12)
    assert not np.allclose(A, Fm[d.rows] @ Rm @ Fm.T, atol=1e-3)   # Psi = F^T differs
    assert not np.allclose(A, Fm[d.rows] @ Rm, atol=1e-3)          # Psi = I differs
    with pytest.raises(ValueError):
        oracle.gram_matrix(op, S)                                   # closed form is for Psi = I


def test_p6_orthogonal_special_case_dct_basis():
    """M = N with Psi = F: A = F R F is orthogonal, so every algorithm returns
    hard thresholding of A^T y, and the LS routes agree on the operator."""
    rng = np.random.default_rng(14)
    n, k = 512, 20
    rows, signs = synth.draw_operator(rng, n, n)
    op = oracle.SRM(n, rows, signs, psi=1)
    y = rng.standard_normal(n)
    c = op.adjoint(y)
    expect = np.sort(np.argsort(-np.abs(c), kind="stable")[:k])
    for f in (oracle.omp, oracle.sp, oracle.cosamp):
        r = f(op, y, k)
        assert np.array_equal(r.support, expect), f.__name__
        assert np.allclose(r.s[expect], c[expect], atol=1e-12)
    q = oracle.ompr(op, y, k, eta=1.0)
    assert np.array_equal(q.support, expect) and q.iters == 0


def test_p4_dct_basis_ls_routes_and_recovery():
    """Psi = F: dense QR and operator CG least squares agree and leave a
    residual orthogonal to the columns (Theorems 1-2); a noiseless signal
    sparse in the DCT basis is recovered exactly by all four algorithms."""
    d = synth.draw_problem(106, 0, 2048, 512, 25, "normal_min0.1", None, randomizer="perm")
    op = oracle.SRM(d.n, d.rows, d.signs, d.perm, psi=1)
    y = op.apply_sparse(d.supp, d.vals)
    rng = np.random.default_rng(8)
    yn = y + 0.01 * rng.standard_normal(d.m)
    S = np.sort(rng.choice(d.n, 40, replace=False))
    v1 = oracle.ls_dense(op, S, yn)
    v2, _ = oracle.ls_cg(op, S, yn, tol=1e-13)
    assert np.allclose(v1, v2, atol=1e-10)
    r = yn - op.columns(S) @ v1
    assert np.max(np.abs(op.columns(S).T @ r)) < 1e-10
    for f in (oracle.omp, oracle.sp, oracle.ompr, oracle.cosamp):
        res = f(op, y, 25)
        assert np.array_equal(res.support, d.supp), f.__name__
        assert np.allclose(res.s[d.supp], d.vals, atol=1e-9)


@pytest.mark.parametrize("side,randomizer", [(8, "signs"), (16, "perm")])
def test_p2_dct2d_basis(side, randomizer):
    """Psi = F_n (x) F_n on an n x n image (Sec. III-E with fixed DCT factors):
    A = D F R (F_n (x) F_n) equals the product of dense cosine-formula
    matrices (the Kronecker product written out), has orthonormal rows, and
    its columns and adjoint agree with that product; Psi = F_N (1-D) gives a
    different operator."""
    n = side * side
    d = synth.draw_problem(107, 0, n, n // 3, 5, "normal", None, randomizer=randomizer)
    op = oracle.SRM(n, d.rows, d.signs, d.perm, psi=2)
    Fn = oracle.dct2_matrix(n)
    Fs = oracle.dct2_matrix(side)
    Rm = np.zeros((n, n))
    idx = d.perm if d.perm is not None else np.arange(n)
    Rm[idx, np.arange(n)] = d.signs
    A = Fn[d.rows] @ Rm @ np.kron(Fs, Fs)
    rng = np.random.default_rng(9)
    x = rng.standard_normal(n)
    u = rng.standard_normal(d.m)
    assert np.allclose(op.apply(x), A @ x, atol=1e-12)
    assert np.allclose(op.adjoint(u), A.T @ u, atol=1e-12)
    assert np.allclose(A @ A.T, np.eye(d.m), atol=1e-12)
    S = np.sort(rng.choice(n, 9, replace=False))
    assert np.allclose(op.columns(S), A[:, S], atol=1e-12)
    assert not np.allclose(A, Fn[d.rows] @ Rm @ Fn, atol=1e-3)                   # the 1-D basis differs
    assert not np.allclose(A, Fn[d.rows] @ Rm @ np.kron(Fs, Fs).T, atol=1e-3)    # so does its transpose


def test_p6_dct2d_orthogonal_and_recovery():
    """Psi = F_n (x) F_n: with M = N every algorithm returns hard thresholding
    of A^T y; with M = N/4 the dense and CG least-squares routes agree, and a
    noiseless image sparse in the 2-D DCT basis is recovered exactly."""
    rng = np.random.default_rng(15)
    n, k = 256, 12
    rows, signs = synth.draw_operator(rng, n, n)
    op = oracle.SRM(n, rows, signs, psi=2)
    y = rng.standard_normal(n)
    c = op.adjoint(y)
    expect = np.sort(np.argsort(-np.abs(c), kind="stable")[:k])
    for f in (oracle.omp, oracle.sp, oracle.cosamp):
        r = f(op, y, k)
        assert np.array_equal(r.support, expect), f.__name__
    d = synth.draw_problem(108, 0, 4096, 1024, 25, "normal_min0.1", None, randomizer="perm")
    o2 = oracle.SRM(d.n, d.rows, d.signs, d.perm, psi=2)
    y2 = o2.apply_sparse(d.supp, d.vals)
    S = np.sort(rng.choice(d.n, 40, replace=False))
    v1 = oracle.ls_dense(o2, S, y2)
    v2, _ = oracle.ls_cg(o2, S, y2, tol=1e-13)
    assert np.allclose(v1, v2, atol=1e-10)
    for f in (oracle.omp, oracle.sp, oracle.ompr, oracle.cosamp):
        res = f(o2, y2, 25)
        assert np.array_equal(res.support, d.supp), f.__name__


# ------------------------------------------------------------------ partial Fourier sensing
@pytest.mark.parametrize("psi,randomizer", [(0, "signs"), (0, "perm"), (1, "perm")])
def test_p2_real_fourier_basis(psi, randomizer):
    """F = the orthonormal real Fourier basis: the FFT route equals the dense
    cosine/sine formula (D Rf R, and D Rf R Rf with Psi = F), the rows are
    orthonormal, and sampling rows k and N-k measures the complex Fourier
    coefficient of R x: y_k - i y_{N-k} = sqrt(2/N) FFT(R x)_k (D(FFT(x)) of
    Sec. II), checked against NumPy's complex FFT."""
    n = 256
    d = synth.draw_problem(109, 0, n, 90, 5, "normal", None, randomizer=randomizer)
    op = oracle.SRM(n, d.rows, d.signs, d.perm, psi=psi, xform=1)
    Rf = oracle.rdft_matrix(n)
    Rm = np.zeros((n, n))
    idx = d.perm if d.perm is not None else np.arange(n)
    Rm[idx, np.arange(n)] = d.signs
    A = Rf[d.rows] @ Rm @ (Rf if psi else np.eye(n))
    rng = np.random.default_rng(10)
    x = rng.standard_normal(n)
    u = rng.standard_normal(d.m)
    assert np.allclose(op.apply(x), A @ x, atol=1e-12)
    assert np.allclose(op.adjoint(u), A.T @ u, atol=1e-12)
    assert np.allclose(A @ A.T, np.eye(d.m), atol=1e-12)
    S = np.sort(rng.choice(n, 9, replace=False))
    assert np.allclose(op.columns(S), A[:, S], atol=1e-12)
    with pytest.raises(ValueError):
        oracle.gram_matrix(op, S)
    if psi == 0:
        full = oracle.SRM(n, np.arange(n), d.signs, d.perm, xform=1)
        yf = full.apply(x)
        X = np.fft.fft(Rm @ x)
        k = np.arange(1, n // 2)
        assert np.allclose(yf[k] - 1j * yf[n - k], np.sqrt(2.0 / n) * X[k], atol=1e-12)
        assert np.isclose(yf[0], X[0].real / np.sqrt(n)) and np.isclose(yf[n // 2], X[n // 2].real / np.sqrt(n))


def test_p6_real_fourier_orthogonal_and_recovery():
    """Real Fourier basis: M = N reduces every algorithm to hard thresholding;
    with M = N/4 a noiseless sparse signal is recovered exactly and the dense
    and CG least-squares routes agree."""
    rng = np.random.default_rng(16)
    n, k = 512, 20
    rows, signs = synth.draw_operator(rng, n, n)
    op = oracle.SRM(n, rows, signs, xform=1)
    y = rng.standard_normal(n)
    c = op.adjoint(y)
    expect = np.sort(np.argsort(-np.abs(c), kind="stable")[:k])
    for f in (oracle.omp, oracle.sp, oracle.cosamp):
        assert np.array_equal(f(op, y, k).support, expect), f.__name__
    d = synth.draw_problem(110, 0, 4096, 1024, 25, "normal_min0.1", None, randomizer="perm")
    o2 = oracle.SRM(d.n, d.rows, d.signs, d.perm, xform=1)
    y2 = o2.apply_sparse(d.supp, d.vals)
    S = np.sort(rng.choice(d.n, 40, replace=False))
    assert np.allclose(oracle.ls_dense(o2, S, y2), oracle.ls_cg(o2, S, y2, tol=1e-13)[0], atol=1e-10)
    for f in (oracle.omp, oracle.sp, oracle.ompr, oracle.cosamp):
        assert np.array_equal(f(o2, y2, 25).support, d.supp), f.__name__
