"""Partial complex Fourier sensing of a real signal: the operator D(FFT(x)) of
Sec. II (a randomly partial Fourier matrix as Phi, Sec. II and Sec. III-D), in FP64.

    A = D_Omega F R,   (F v)_k = N^(-1/2) sum_n v_n exp(-2 pi i k n / N)

F is the unitary DFT, R = diag(signs) a +-1 sign flip and D_Omega keeps the
frequencies Omega, strictly ascending in [1, N/2).  Each kept frequency gives
one complex measurement.  (For a real signal the coefficients at 0 and N/2 are
real and those at N - k are the conjugates of those at k, so [1, N/2) holds
every complex degree of freedom once.)

The signal is real, so every least-squares problem is over real coefficients
and the adjoint that the greedy steps use is the one of the real inner product
Re<u, v> on C^M:  A* u = R Re(F^H D^T u), with F^H = sqrt(N) IFFT.  The least
squares on a support S is min over real v of ||y - A_S v||_2 (a complex norm),
solved on the stacked real system [Re A_S; Im A_S] v = [Re y; Im y].
"""
from __future__ import annotations

import numpy as np


class CPF:
    """M x N partial complex Fourier operator on real N-vectors (see module)."""

    complex_meas = True    # measurements are complex
    psi = 0                # no sparsifying basis
    xform = 2              # the complex partial Fourier transform
    perm = None

    def __init__(self, n: int, freqs, signs):
        freqs = np.asarray(freqs, dtype=np.int64)
        signs = np.asarray(signs)
        if freqs.ndim != 1 or signs.shape != (n,):
            raise ValueError("freqs must be 1-D and signs must have length n")
        if freqs.size and (freqs[0] < 1 or freqs[-1] >= n // 2 or np.any(np.diff(freqs) <= 0)):
            raise ValueError("freqs must be strictly ascending in [1, n/2)")
        if not np.all(np.abs(signs) == 1):
            raise ValueError("signs must be +-1")
        self.n = int(n)
        self.m = int(freqs.size)
        self.rows = freqs
        self.signs = signs.astype(np.float64)

    def apply(self, x: np.ndarray) -> np.ndarray:
        """A x (complex M-vector) for a real N-vector x."""
        v = self.signs * np.asarray(x, dtype=np.float64)
        return np.fft.fft(v)[self.rows] / np.sqrt(self.n)

    def apply_sparse(self, supp, vals) -> np.ndarray:
        x = np.zeros(self.n)
        x[np.asarray(supp, dtype=np.int64)] = vals
        return self.apply(x)

    def adjoint(self, u: np.ndarray) -> np.ndarray:
        """A* u = R Re(F^H D^T u): zero-fill, unitary inverse DFT, real part, sign flip."""
        full = np.zeros(self.n, dtype=np.complex128)
        full[self.rows] = np.asarray(u, dtype=np.complex128)
        return self.signs * (np.fft.ifft(full) * np.sqrt(self.n)).real

    def columns(self, supp) -> np.ndarray:
        """Dense complex A_S (M x |S|) from the DFT's definition."""
        j = np.asarray(supp, dtype=np.int64)[None, :]
        k = self.rows[:, None]
        # reduce k j mod N before scaling so large N keep the phase exact
        return np.exp(-2j * np.pi * ((k * j) % self.n) / self.n) / np.sqrt(self.n) * self.signs[j]

    def dense(self) -> np.ndarray:
        return self.columns(np.arange(self.n))

