"""The near-tie certificates of tests/near_tie.py, pinned on the CPU: an
oracle trajectory certifies itself (every gap <= 0), and each planted mistake
(a wrong entering index, a wrong kept set, a wrong final support, a wrong s)
fails at the decision it spoils."""
import numpy as np
import pytest

import oracle
from tests.near_tie import certify_ompr, certify_sp
from tests.problems import problem

N, M, K, TOL = 2 ** 12, 2 ** 10, 64, 1e-6


@pytest.fixture(scope="module")
def noisy():
    d, op, y = problem(141, 0, N, M, K, "normal", 25.0, dtype="f32")
    return d, op, y


@pytest.fixture(scope="module")
def sp_run(noisy):
    d, op, y = noisy
    r = oracle.sp(op, y, K)
    assert len(r.supports) >= 2
    return r


def _low_key_outside(op, y, supp, x):
    """An index outside supp whose correlation with the residual is smallest."""
    r = y - op.apply_sparse(supp, x)
    c = np.abs(op.adjoint(r))
    c[supp] = np.inf
    return int(np.argmin(c))


def test_sp_oracle_trajectory_certifies_itself(noisy, sp_run):
    d, op, y = noisy
    v = certify_sp(op, y, K, TOL, sp_run.supports, sp_run.s)
    assert v.ok, v
    assert all(g <= b for (_, _, g, b) in v.gaps)
    assert v.s_err <= 1e-9


def test_sp_planted_wrong_round_fails(noisy, sp_run):
    """G_1 with one index traded for the least correlated one outside T."""
    d, op, y = noisy
    sup = [np.array(s) for s in sp_run.supports]
    x0 = oracle.ls_cg(op, sup[0], y)[0]
    bad = _low_key_outside(op, y, sup[0], x0)
    g1 = np.sort(np.append(np.setdiff1d(sup[1], sup[0])[1:], np.intersect1d(sup[1], sup[0])))
    g1 = np.sort(np.append(g1, bad))
    assert g1.size == K
    v = certify_sp(op, y, K, TOL, [sup[0], g1], sp_run.s)
    assert not v.ok and v.round == 1 and v.kind in ("expand", "prune"), v


def test_sp_planted_wrong_init_and_final_fail(noisy, sp_run):
    d, op, y = noisy
    sup = [np.array(s) for s in sp_run.supports]
    key = np.abs(op.adjoint(y))
    worst = int(np.argmin(np.where(np.isin(np.arange(N), sup[0]), np.inf, key)))
    g0 = np.sort(np.append(sup[0][1:], worst))
    v = certify_sp(op, y, K, TOL, [g0] + sup[1:], sp_run.s)
    assert not v.ok and v.kind == "init", v
    # a final support that is not a fixed point: the initial support alone
    # when SP moved away from it, reported with s of its own LS
    xi = oracle.ls_cg(op, sup[0], y, tol=1e-13)[0]
    si = np.zeros(N)
    si[sup[0]] = xi
    v = certify_sp(op, y, K, TOL, sup[:1], si)
    assert not v.ok and v.kind == "final", v


def test_sp_planted_wrong_s_fails(noisy, sp_run):
    d, op, y = noisy
    s = sp_run.s.copy()
    s[sp_run.support[0]] *= 1.01
    v = certify_sp(op, y, K, TOL, sp_run.supports, s)
    assert not v.ok and v.kind == "s", v


@pytest.fixture(scope="module")
def ompr_run(noisy):
    d, op, y = noisy
    r = oracle.ompr(op, y, K)
    assert len(r.moves) >= 2
    return r


def test_ompr_planted_wrong_enter_fails(noisy, ompr_run):
    """The first swap's entering index traded for the least correlated one."""
    d, op, y = noisy
    moves = [(int(a[0]), int(b[0])) for a, b in ompr_run.moves]
    init = oracle.greedy.topk_excluding(op.adjoint(y), None, K)[0]
    x0 = oracle.ls_cg(op, init, y)[0]
    bad = _low_key_outside(op, y, init, x0)
    gm = [(bad, moves[0][1])] + moves[1:]
    final = set(int(v) for v in ompr_run.support)
    final.discard(moves[0][0])
    final.add(bad)
    v = certify_ompr(op, y, K, TOL, N / M, moves, gm, np.array(sorted(final)), ompr_run.s)
    assert not v.ok and v.step == 1 and v.kind == "enter", v


def test_ompr_equal_trajectories_are_not_certified(noisy, ompr_run):
    """Equal moves with equal results leave nothing to certify (the caller
    compares those directly): the certifier says so rather than passing."""
    d, op, y = noisy
    moves = [(int(a[0]), int(b[0])) for a, b in ompr_run.moves]
    v = certify_ompr(op, y, K, TOL, N / M, moves, moves, ompr_run.support, ompr_run.s)
    assert not v.ok and v.kind == "none"
