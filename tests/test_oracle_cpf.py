"""Pins of the oracle's partial complex Fourier operator (oracle/cpf.py,
A x = D(FFT(x)) of Sec. II for a real signal x) against closed forms and
identities of the DFT, and against the oracle's real partial Fourier operator
on the equivalent real rows:

* a pure tone: x_n = cos(2 pi k0 n / N) has y_k0 = sqrt(N)/2 and zero elsewhere,
  sin gives -i sqrt(N)/2;
* Parseval for a real signal with every frequency of [1, N/2) kept:
  ||A x||^2 = (||x||^2 - |X_0|^2 - |X_{N/2}|^2) / 2, X_0 and X_{N/2} the unitary
  DFT's real coefficients;
* the adjoint identity Re<A x, u> = <x, A* u> and A A* = I/2 (kept frequencies
  below N/2: the conjugate frequency N - k is never kept);
* the real equivalent: frequency k in (0, N/2) is the pair of rows k (cosine)
  and N - k (sine) of the orthonormal real Fourier basis, so with
  y^ = (sqrt 2 Re y_k at row k, -sqrt 2 Im y_k at row N - k) every objective
  satisfies ||y^ - A_r x||^2 = 2 ||y - A x||^2, and OMP, SP, OMPR and CoSaMP
  give the same supports and values on both;
* noiseless exact recovery and the gradient against central differences.
Each planted mistake (a conjugated exponent, a dropped 1/sqrt(N), the
imaginary instead of the real part in the adjoint) must fail one of them."""
import numpy as np
import pytest

import oracle
import synth
from oracle.cpf import CPF


def _op(n=64, m=12, seed=0, signs=None):
    rng = np.random.default_rng(seed)
    fr = np.sort(1 + rng.choice(n // 2 - 1, m, replace=False))
    sg = rng.choice([-1, 1], n) if signs is None else signs
    return CPF(n, fr, sg)


def _real_equivalent(op, y):
    """The real partial Fourier operator on rows k and N - k, and y^."""
    n, fr = op.n, op.rows
    rows = np.concatenate([fr, n - fr[::-1]])
    yhat = np.concatenate([np.sqrt(2.0) * y.real, (-np.sqrt(2.0) * y.imag)[::-1]])
    return oracle.SRM(n, rows, op.signs.astype(np.int8), xform=1), yhat


def _tone_ok(op_cls):
    n, k0 = 64, 5
    op = op_cls(n, np.arange(1, n // 2), np.ones(n))
    t = np.arange(n)
    yc = op.apply(np.cos(2 * np.pi * k0 * t / n))
    ys = op.apply(np.sin(2 * np.pi * k0 * t / n))
    ec = np.zeros(n // 2 - 1, dtype=complex)
    ec[k0 - 1] = np.sqrt(n) / 2
    return np.allclose(yc, ec, atol=1e-12) and np.allclose(ys, -1j * ec, atol=1e-12)


def _adjoint_ok(op):
    rng = np.random.default_rng(3)
    x = rng.standard_normal(op.n)
    u = rng.standard_normal(op.m) + 1j * rng.standard_normal(op.m)
    lhs = np.vdot(u, op.apply(x)).real
    return abs(lhs - x @ op.adjoint(u)) <= 1e-12 * np.linalg.norm(x) * np.linalg.norm(u)


def _half_identity_ok(op):
    a = op.dense()
    astar = np.stack([op.adjoint(e) for e in np.eye(op.m)], axis=1)    # A* as an N x M real matrix
    return np.allclose(a @ astar, 0.5 * np.eye(op.m), atol=1e-12)


def test_tone():
    assert _tone_ok(CPF)


def test_parseval_all_frequencies():
    n = 256
    rng = np.random.default_rng(1)
    sg = rng.choice([-1, 1], n)
    op = CPF(n, np.arange(1, n // 2), sg)
    x = rng.standard_normal(n)
    v = sg * x
    x0 = v.sum() / np.sqrt(n)
    xh = (v * (-1.0) ** np.arange(n)).sum() / np.sqrt(n)
    lhs = np.linalg.norm(op.apply(x)) ** 2
    assert abs(lhs - (v @ v - x0 ** 2 - xh ** 2) / 2) <= 1e-10 * (v @ v)


def test_adjoint_identity_and_half():
    for seed in range(3):
        op = _op(128, 20, seed)
        assert _adjoint_ok(op)
        assert _half_identity_ok(op)


def test_columns_match_apply_at_large_n():
    """The formula route at N = 2^16 (phases reduced mod N) against the FFT route."""
    op = _op(2 ** 16, 300, 4)
    supp = np.array([0, 1, 777, 40000, 65535])
    vals = np.array([1.0, -2.0, 0.5, 3.0, -1.0])
    assert np.allclose(op.columns(supp) @ vals, op.apply_sparse(supp, vals), atol=1e-12)


def test_real_equivalent_objective():
    op = _op(256, 40, 2)
    rng = np.random.default_rng(5)
    y = rng.standard_normal(op.m) + 1j * rng.standard_normal(op.m)
    opr, yhat = _real_equivalent(op, y)
    for _ in range(3):
        x = rng.standard_normal(op.n)
        assert abs(np.linalg.norm(yhat - opr.apply(x)) ** 2 - 2 * np.linalg.norm(y - op.apply(x)) ** 2) \
            <= 1e-9 * np.linalg.norm(yhat) ** 2


@pytest.mark.parametrize("algo", ["omp", "sp", "ompr", "cosamp"])
def test_algorithms_match_the_real_equivalent(algo):
    d = synth.draw_fourier_problem(150, 0, 1024, 120, 20, "normal", 25.0)
    op = CPF(d.n, d.rows, d.signs)
    y0 = op.apply_sparse(d.supp, d.vals)
    y = y0 + d.noise_scale(np.linalg.norm(y0)) * d.noise
    opr, yhat = _real_equivalent(op, y)
    a = getattr(oracle, algo)(op, y, d.k)
    b = getattr(oracle, algo)(opr, yhat, d.k)
    assert np.array_equal(a.support, b.support)
    assert np.allclose(a.s, b.s, atol=1e-9 * np.abs(b.s).max())
    assert abs(a.resid_norm * np.sqrt(2.0) - b.resid_norm) <= 1e-9 * max(1.0, b.resid_norm)


def test_noiseless_exact_recovery():
    d = synth.draw_fourier_problem(151, 0, 4096, 400, 40, "normal_min0.1", None)
    op = CPF(d.n, d.rows, d.signs)
    y = op.apply_sparse(d.supp, d.vals)
    for algo in ("omp", "sp"):
        r = getattr(oracle, algo)(op, y, d.k)
        assert np.array_equal(r.support, d.supp), algo
        assert np.allclose(r.s, d.s_dense(), atol=1e-10)


def test_least_squares_routes_and_gradient():
    d = synth.draw_fourier_problem(152, 0, 2048, 200, 30, "normal", 20.0)
    op = CPF(d.n, d.rows, d.signs)
    y0 = op.apply_sparse(d.supp, d.vals)
    y = y0 + d.noise_scale(np.linalg.norm(y0)) * d.noise
    x_dense = oracle.ls_dense(op, d.supp, y)
    x_cg, _ = oracle.ls_cg(op, d.supp, y)
    assert np.allclose(x_dense, x_cg, atol=1e-10)
    # gradient of ||s_hat - t||^2 against central differences in Re y and Im y
    t = np.zeros(d.n)
    t[d.supp] = d.vals
    from oracle.adjoint import adjoint_gradient
    g, _ = adjoint_gradient(op, d.supp, y, t)
    h = 1e-6
    for i in (0, 17, 199):
        for e in (1.0, 1j):
            yp, ym = y.copy(), y.copy()
            yp[i] += h * e
            ym[i] -= h * e
            lp = np.sum((oracle.ls_dense(op, d.supp, yp) - d.vals) ** 2)
            lm = np.sum((oracle.ls_dense(op, d.supp, ym) - d.vals) ** 2)
            fd = (lp - lm) / (2 * h)
            got = g[i].real if e == 1.0 else g[i].imag
            assert abs(fd - got) <= 1e-5 * max(1.0, abs(got))


# ---------------------------------------------------------------- planted mistakes
class _Conj(CPF):
    def apply(self, x):
        return np.conj(super().apply(x))


class _NoScale(CPF):
    def apply(self, x):
        return super().apply(x) * np.sqrt(self.n)


class _ImagAdjoint(CPF):
    def adjoint(self, u):
        full = np.zeros(self.n, dtype=np.complex128)
        full[self.rows] = u
        return self.signs * (np.fft.ifft(full) * np.sqrt(self.n)).imag


def test_planted_mistakes_fail():
    assert not _tone_ok(_Conj)
    op = _op(128, 20, 0)
    bad = _NoScale(op.n, op.rows, op.signs)
    assert not _adjoint_ok(bad) or not _half_identity_ok(bad)
    bad = _ImagAdjoint(op.n, op.rows, op.signs)
    assert not _adjoint_ok(bad)
