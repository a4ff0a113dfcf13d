"""Sensing operator of Sec. III-A, Eq. (7): Phi = D F R, and A = Phi Psi (Eq. (2)).

* D keeps the sampled rows ``rows`` (M of N, ascending) of an N-vector
  (the "randomly choose M indices" operator of Sec. III-D).
* F is the orthonormal N-point DCT-II,
      (F x)_k = c_k sum_n x_n cos(pi (2n+1) k / (2N)),
      c_0 = sqrt(1/N), c_k = sqrt(2/N) for k >= 1.
  Its transpose (= inverse) is the orthonormal DCT-III.
* R = diag(signs) with signs in {+1, -1}, optionally with a permutation.
* Psi, the sparsifying basis: the identity (``psi = 0``, s sparse directly)
  or, as in the experiments of Sec. IV-A, the orthonormal DCT-II F itself
  (``psi = 1``), or the separable 2-D DCT of Sec. III-E on an n x n image,
  N = n^2 (``psi = 2``): x = vec(F_n S F_n^T), row-major vec.

So with Psi = I, A x = (F (signs * x))[rows] and A^T u = signs * F^T
(zero-fill_rows(u)); with Psi = F, A s = (F R F s)[rows] and
A^T u = F^T R^T F^T zero-fill_rows(u).

Two independent routes are provided: SciPy's FFT-based DCT (``apply``,
``adjoint``) and the dense cosine formula (``columns``, ``dense``) with the
angle reduced exactly in integers, for small problems and for pins.
"""
from __future__ import annotations

import os
import numpy as np
import scipy.fft as sfft

WORKERS = int(os.environ.get("CS_ORACLE_WORKERS", 0)) or os.cpu_count() or 1   # scipy.fft threads


def _dct_scale(k: np.ndarray, n: int) -> np.ndarray:
    return np.where(k == 0, np.sqrt(1.0 / n), np.sqrt(2.0 / n))


def _cos_table(k: np.ndarray, j: np.ndarray, n: int) -> np.ndarray:
    """cos(pi (2j+1) k / (2n)) for broadcast integer arrays k, j.

    The angle is pi * a / (2n) with a = (2j+1) k reduced modulo 4n in exact
    integer arithmetic before the floating-point cosine."""
    a = ((2 * j.astype(np.int64) + 1) * k.astype(np.int64)) % (4 * n)
    return np.cos(np.pi * a.astype(np.float64) / (2.0 * n))


def _rdft_table(q: np.ndarray, t: np.ndarray, n: int) -> np.ndarray:
    """Orthonormal real Fourier basis (partial Fourier sensing of a real
    signal): row q at input t is 1/sqrt(n) (q = 0), (-1)^t / sqrt(n) (q = n/2),
    sqrt(2/n) cos(2 pi q t / n) (0 < q < n/2) and sqrt(2/n) sin(2 pi (n-q) t / n)
    (q > n/2); the angle is reduced exactly in integers."""
    q = q.astype(np.int64)
    t = t.astype(np.int64)
    half = n // 2
    kq = np.where(q > half, n - q, q)
    a = (kq * t) % n
    ang = 2.0 * np.pi * a.astype(np.float64) / n
    val = np.where(q > half, np.sin(ang), np.cos(ang)) * np.sqrt(2.0 / n)
    return np.where((q == 0) | (q == half), np.cos(ang) / np.sqrt(n), val)


def rdft_matrix(n: int) -> np.ndarray:
    """Dense orthonormal real Fourier basis (n x n) from the formula."""
    return _rdft_table(np.arange(n)[:, None], np.arange(n)[None, :], n)


def _rdft(x: np.ndarray, axis: int = 0) -> np.ndarray:
    """The real Fourier basis applied along `axis` through NumPy's real FFT."""
    x = np.moveaxis(np.asarray(x, dtype=np.float64), axis, 0)
    n = x.shape[0]
    half = n // 2
    X = np.fft.rfft(x, axis=0)
    out = np.empty_like(x)
    out[0] = X[0].real / np.sqrt(n)
    out[half] = X[half].real / np.sqrt(n)
    k = np.arange(1, half)
    out[k] = np.sqrt(2.0 / n) * X[k].real
    out[n - k] = -np.sqrt(2.0 / n) * X[k].imag
    return np.moveaxis(out, 0, axis)


def _irdft(u: np.ndarray) -> np.ndarray:
    """Inverse (= transpose) of the real Fourier basis through NumPy's inverse real FFT."""
    u = np.asarray(u, dtype=np.float64)
    n = u.size
    half = n // 2
    X = np.zeros(half + 1, dtype=complex)
    X[0] = u[0] * np.sqrt(n)
    X[half] = u[half] * np.sqrt(n)
    k = np.arange(1, half)
    X[k] = np.sqrt(n / 2.0) * (u[k] - 1j * u[n - k])
    return np.fft.irfft(X, n=n)


def dct2_matrix(n: int) -> np.ndarray:
    """Dense orthonormal DCT-II matrix F (n x n) from the cosine formula."""
    k = np.arange(n)[:, None]
    j = np.arange(n)[None, :]
    return _dct_scale(k, n) * _cos_table(k, j, n)


class SRM:
    """A = D_rows . DCT-II . R . Psi, an M x N operator (FP64).

    R is the randomizer: entry j of x goes to DCT input perm[j] with sign
    signs[j] ((R x)[perm[j]] = signs[j] x[j]); perm = None is the identity, so
    R = diag(signs).  The paper's R is a uniform random permutation (signs all
    +1); the workloads here use the sign flip.  Psi is the identity (psi = 0),
    the DCT-II (psi = 1, A = D F R F) or the 2-D DCT (psi = 2,
    A = D F R (F_n (x) F_n))."""

    def __init__(self, n: int, rows, signs, perm=None, psi: int = 0, xform: int = 0):
        rows = np.asarray(rows, dtype=np.int64)
        signs = np.asarray(signs)
        if rows.ndim != 1 or signs.shape != (n,):
            raise ValueError("rows must be 1-D and signs must have length n")
        if rows.size and (rows[0] < 0 or rows[-1] >= n or np.any(np.diff(rows) <= 0)):
            raise ValueError("rows must be strictly ascending in [0, n)")
        if not np.all(np.abs(signs) == 1):
            raise ValueError("signs must be +-1")
        self.n = int(n)
        self.m = int(rows.size)
        self.rows = rows
        self.signs = signs.astype(np.float64)
        if psi not in (0, 1, 2):
            raise ValueError("psi must be 0, 1 or 2")
        if xform not in (0, 1):
            raise ValueError("xform must be 0 (DCT-II) or 1 (real Fourier)")
        self.xform = int(xform)
        self.psi = int(psi)
        self.side = 0
        if psi == 2:
            side = int(round(np.sqrt(n)))
            if side * side != n:
                raise ValueError("psi = 2 needs N = n^2")
            self.side = side
        self.perm = None
        if perm is not None:
            perm = np.asarray(perm, dtype=np.int64)
            if perm.shape != (n,) or not np.array_equal(np.sort(perm), np.arange(n)):
                raise ValueError("perm must be a permutation of [0, n)")
            self.perm = perm

    def _place(self, x: np.ndarray) -> np.ndarray:
        """R x: the DCT input."""
        v = self.signs * x
        if self.perm is None:
            return v
        out = np.zeros(self.n)
        out[self.perm] = v
        return out

    def _unplace(self, w: np.ndarray) -> np.ndarray:
        """R^T w."""
        return self.signs * (w if self.perm is None else w[self.perm])

    def dct_index(self, j) -> np.ndarray:
        """DCT input index of entry j of x."""
        j = np.asarray(j, dtype=np.int64)
        return j if self.perm is None else self.perm[j]

    def _F(self, v: np.ndarray) -> np.ndarray:
        """The orthonormal transform F: DCT-II, or the real Fourier basis."""
        if self.xform:
            return _rdft(v)
        return sfft.dct(v, type=2, norm="ortho", workers=WORKERS)

    def _Ft(self, w: np.ndarray) -> np.ndarray:
        if self.xform:
            return _irdft(w)
        return sfft.idct(w, type=2, norm="ortho", workers=WORKERS)

    # ---------------------------------------------------------- FFT route
    def apply(self, x: np.ndarray) -> np.ndarray:
        """A x for a dense N-vector x (with psi = 1, F x enters R first)."""
        x = np.asarray(x, dtype=np.float64)
        if self.psi == 1:
            x = self._F(x)
        elif self.psi == 2:
            x = sfft.dctn(x.reshape(self.side, self.side), type=2, norm="ortho", workers=WORKERS).reshape(-1)
        return self._F(self._place(x))[self.rows]

    def apply_sparse(self, supp, vals) -> np.ndarray:
        """A x where x is zero off ``supp`` and equals ``vals`` on it."""
        x = np.zeros(self.n)
        x[np.asarray(supp, dtype=np.int64)] = vals
        return self.apply(x)

    def adjoint(self, u: np.ndarray) -> np.ndarray:
        """A^T u for an M-vector u: zero-fill, orthonormal DCT-III, sign flip."""
        full = np.zeros(self.n)
        full[self.rows] = np.asarray(u, dtype=np.float64)
        w = self._unplace(self._Ft(full))
        if self.psi == 1:
            w = self._Ft(w)
        elif self.psi == 2:
            w = sfft.idctn(w.reshape(self.side, self.side), type=2, norm="ortho", workers=WORKERS).reshape(-1)
        return w

    # ---------------------------------------------------- formula route
    def columns(self, supp) -> np.ndarray:
        """Dense A_S (M x |S|) from the cosine formula.

        With psi = 1 each column is D F R (F e_j), with psi = 2 D F R (Psi e_j)
        for the 2-D basis: Psi's columns from the formula, then R, then F
        through the same formula for N <= 4096 (else SciPy's DCT)."""
        j = np.asarray(supp, dtype=np.int64)[None, :]
        k = self.rows[:, None]
        table = (lambda q, t: _rdft_table(q, t, self.n)) if self.xform else \
            (lambda q, t: _dct_scale(q, self.n) * _cos_table(q, t, self.n))
        if not self.psi:
            return table(k, self.dct_index(j)) * self.signs[j]
        if self.psi == 1:
            i = np.arange(self.n)[:, None]
            fcols = table(i, j)                                         # F e_j, N x |S|
        else:                                                           # vec(F_n E_ab F_n^T) = F_n[:, a] (x) F_n[:, b]
            fs = dct2_matrix(self.side)
            a, b = j[0] // self.side, j[0] % self.side
            fcols = (fs[:, a][:, None, :] * fs[:, b][None, :, :]).reshape(self.n, -1)
        placed = np.zeros_like(fcols)
        idx = self.dct_index(np.arange(self.n))
        placed[idx, :] = self.signs[:, None] * fcols                    # R applied to each column
        if self.n <= 4096:
            return table(k, np.arange(self.n)[None, :]) @ placed
        if self.xform:
            return _rdft(placed, axis=0)[self.rows, :]
        return sfft.dct(placed, type=2, norm="ortho", axis=0, workers=WORKERS)[self.rows, :]

    def dense(self) -> np.ndarray:
        return self.columns(np.arange(self.n))
