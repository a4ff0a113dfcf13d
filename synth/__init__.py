"""Seeded synthetic inputs for compressive-sensing recovery.

This module only draws random numbers: sampled rows, sign flips, support
positions, nonzero values and unit-variance noise.  It contains none of the
recovery arithmetic (no transform, no least squares), so the FP64 oracle and
the GPU path can both consume what it returns without sharing method code.

Every draw uses ``numpy.random.default_rng([1509, 3979, cfg, sig, stream])``
with fixed streams: 0 operator, 1 signal, 2 noise, 3 per-signal sizes,
4 finite-difference coordinates.  The draw order inside each stream is fixed.

The measurement model is Eq. (2) of the paper, y = A s (+ noise, as in the
experiments section), with A = D * F * R (Eq. (7)): D keeps M of the N rows
(uniformly, without replacement), F is the orthonormal DCT-II and R is a
random +-1 sign flip.
"""
from __future__ import annotations

import dataclasses
import numpy as np

SEED_BASE = (1509, 3979)
STREAM_OPERATOR, STREAM_SIGNAL, STREAM_NOISE, STREAM_SIZES, STREAM_FD = 0, 1, 2, 3, 4


def rng_for(cfg: int, sig: int, stream: int) -> np.random.Generator:
    return np.random.default_rng([SEED_BASE[0], SEED_BASE[1], int(cfg), int(sig), int(stream)])


@dataclasses.dataclass
class Draw:
    """Everything random about one recovery problem.

    rows   : int32[M]  sampled DCT rows, strictly ascending
    signs  : int8[N]   +-1 sign flips
    supp   : int32[K]  true support, strictly ascending
    vals   : float64[K] nonzero values on ``supp``
    noise  : float64[M] unit-variance Gaussian draws, or None (noiseless)
    snr_db : measurement SNR in dB, or None
    """
    n: int
    m: int
    k: int
    rows: np.ndarray
    signs: np.ndarray
    supp: np.ndarray
    vals: np.ndarray
    noise: np.ndarray | None
    snr_db: float | None
    noise_sigma: float | None = None
    perm: np.ndarray | None = None     # randomizer permutation (int32[N]), or None

    def s_dense(self) -> np.ndarray:
        s = np.zeros(self.n)
        s[self.supp] = self.vals
        return s

    def noise_scale(self, y0_norm: float) -> float:
        """Noise standard deviation: ``noise_sigma`` when given, else the one that
        gives ``snr_db``: ||y0|| / sqrt(M) * 10^(-SNR/20)."""
        if self.noise_sigma is not None:
            return float(self.noise_sigma)
        if self.snr_db is None:
            return 0.0
        return float(y0_norm) / np.sqrt(self.m) * 10.0 ** (-self.snr_db / 20.0)


def draw_operator(rng: np.random.Generator, n: int, m: int):
    rows = np.sort(rng.choice(n, m, replace=False)).astype(np.int32)
    signs = (rng.integers(0, 2, n) * 2 - 1).astype(np.int8)
    return rows, signs


def draw_values(rng: np.random.Generator, k: int, kind: str) -> np.ndarray:
    if kind == "normal":
        return rng.standard_normal(k)
    if kind == "normal_min0.1":
        # N(0,1) redrawn until every |v| >= 0.1 (rejection of offending entries)
        v = rng.standard_normal(k)
        bad = np.abs(v) < 0.1
        while bad.any():
            v[bad] = rng.standard_normal(int(bad.sum()))
            bad = np.abs(v) < 0.1
        return v
    if kind == "pm_one_plus_absnormal":
        sgn = rng.integers(0, 2, k) * 2 - 1
        return sgn * (1.0 + np.abs(rng.standard_normal(k)))
    raise ValueError(f"unknown value kind {kind!r}")


def draw_problem(cfg: int, sig: int, n: int, m: int, k: int, values: str = "normal",
                 snr_db: float | None = None, noise_sigma: float | None = None,
                 randomizer: str = "signs") -> Draw:
    """randomizer: "signs" (R = random sign flip), "perm" (R = a uniform random
    permutation, signs all +1: the paper's SRM) or "signed_perm" (both)."""
    if not (1 <= k <= m <= n):
        raise ValueError("need 1 <= K <= M <= N")
    ro = rng_for(cfg, sig, STREAM_OPERATOR)
    rows, signs = draw_operator(ro, n, m)
    perm = None
    if randomizer in ("perm", "signed_perm"):
        perm = ro.permutation(n).astype(np.int32)        # drawn after rows and signs
        if randomizer == "perm":
            signs = np.ones(n, dtype=np.int8)
    rs = rng_for(cfg, sig, STREAM_SIGNAL)
    supp = np.sort(rs.choice(n, k, replace=False)).astype(np.int32)
    vals = draw_values(rs, k, values)
    noise = None
    if snr_db is not None or noise_sigma is not None:
        noise = rng_for(cfg, sig, STREAM_NOISE).standard_normal(m)
    return Draw(n, m, k, rows, signs, supp, vals, noise, snr_db, noise_sigma, perm)


# The paper's experimental set-up (Sec. IV-A): M = N/4, K = M/4, Gaussian
# nonzeros with sigma_on = 1, additive noise with sigma = 0.01, R a random
# permutation (Psi = I here); the precision experiment compares exact CG with
# the absolute thresholds 1e-10 and 1e-5.
PAPER_SHAPED = dict(cfg=6, values="normal", noise_sigma=0.01, xis=(1e-10, 1e-5), randomizer="perm")


def paper_problem(n: int, sig: int = 0, randomizer: str = "perm") -> Draw:
    w = PAPER_SHAPED
    return draw_problem(w["cfg"], sig, n, n // 4, n // 16, w["values"], None, w["noise_sigma"], randomizer)


# ---------------------------------------------------------------- workloads
# Named workloads.  ``cfg`` is the seed id.
WORKLOADS = {
    # OMP, one signal, FP64, noiseless, |s_i| >= 0.1
    "omp_n4096": dict(cfg=1, n=4096, m=1024, k=50, values="normal_min0.1", snr_db=None,
                      dtype="f64", tol=1e-10, algos=("omp",)),
    # SP and OMPR, one signal, FP32, 40 dB
    "sp_ompr_n2p20": dict(cfg=2, n=2 ** 20, m=2 ** 18, k=4096, values="normal", snr_db=40.0,
                          dtype="f32", tol=1e-6, algos=("sp", "ompr")),
    # SP, one large signal, FP32 with FP64 CG reductions, noiseless
    "sp_n2p24": dict(cfg=3, n=2 ** 24, m=2 ** 21, k=2 ** 16, values="pm_one_plus_absnormal",
                     snr_db=None, dtype="f32", tol=1e-6, algos=("sp",)),
    # differentiated SP: 64 signals, 30 dB
    "sp_adjoint_n2p16": dict(cfg=5, n=2 ** 16, m=2 ** 14, k=300, values="normal", snr_db=30.0,
                             dtype="f32", tol=1e-6, algos=("sp",), batch=64),
}


# The batched workload: 256 signals with their own sizes (batched_sizes),
# N(0,1) nonzeros, 30 dB noise, FP32, OMPR, CG tol 1e-6.
BATCHED_WORKLOAD = dict(cfg=4, count=256, log_n=(14, 18), values="normal", snr_db=30.0, dtype="f32", tol=1e-6,
                        algos=("ompr",))


def workload_problem(name: str, sig: int = 0) -> Draw:
    w = WORKLOADS[name]
    return draw_problem(w["cfg"], sig, w["n"], w["m"], w["k"], w["values"], w["snr_db"])


def batched_sizes(n_signals: int = 256, cfg: int = 4, log_n=(14, 18)):
    """Per-signal sizes of the batched OMPR workload: N_i in {2^14..2^18}
    (or 2^log_n[0] .. 2^log_n[1]), M_i/N_i ~ U[0.2, 0.4], K_i/N_i ~ U[0.005,
    0.02] (K_i >= 1)."""
    out = []
    lo, hi = log_n
    for sig in range(n_signals):
        r = rng_for(cfg, sig, STREAM_SIZES)
        n = 2 ** (lo + int(r.integers(0, hi - lo + 1)))
        m = int(round(n * r.uniform(0.2, 0.4)))
        k = max(1, int(round(n * r.uniform(0.005, 0.02))))
        out.append((n, m, k))
    return out


def batched_problem(sig: int, cfg: int = 4, log_n=(14, 18)) -> Draw:
    n, m, k = batched_sizes(sig + 1, cfg, log_n)[sig]
    return draw_problem(cfg, sig, n, m, k, "normal", 30.0)


def fd_coordinates(batch: int, m: int, count: int = 32, cfg: int = 5):
    """(signal, coordinate) pairs for central finite differences."""
    r = rng_for(cfg, 0, STREAM_FD)
    sigs = r.integers(0, batch, count)
    coords = r.integers(0, m, count)
    return list(zip(sigs.tolist(), coords.tolist()))


def draw_fourier_problem(cfg: int, sig: int, n: int, m: int, k: int, values: str = "normal",
                         snr_db: float | None = None) -> Draw:
    """A problem for partial complex Fourier sensing of a real signal: ``rows``
    holds M distinct frequencies drawn uniformly from [1, N/2) (ascending), the
    signs are a random +-1 flip, the noise (when ``snr_db`` is given) is
    complex, each entry (a + i b) / sqrt(2) with a, b unit-variance Gaussians."""
    if not (1 <= k <= 2 * m and 1 <= m <= n // 2 - 1):
        raise ValueError("need 1 <= K <= 2M and 1 <= M <= N/2 - 1")
    ro = rng_for(cfg, sig, STREAM_OPERATOR)
    rows = np.sort(1 + ro.choice(n // 2 - 1, m, replace=False)).astype(np.int32)
    signs = (ro.integers(0, 2, n) * 2 - 1).astype(np.int8)
    rs = rng_for(cfg, sig, STREAM_SIGNAL)
    supp = np.sort(rs.choice(n, k, replace=False)).astype(np.int32)
    vals = draw_values(rs, k, values)
    noise = None
    if snr_db is not None:
        g = rng_for(cfg, sig, STREAM_NOISE).standard_normal((2, m))
        noise = (g[0] + 1j * g[1]) / np.sqrt(2.0)
    return Draw(n, m, k, rows, signs, supp, vals, noise, snr_db)
