"""Test inputs: seeded draws from ``synth`` turned into measurements by the oracle.

y = A s (+ noise at the drawn SNR).  FP32 problems hand the GPU float32(y)
and the oracle float64(float32(y)), so both see the same input."""
from __future__ import annotations

import numpy as np

import oracle
import synth


def build(d: synth.Draw, dtype: str = "f64", psi: int = 0, xform: int = 0):
    op = oracle.SRM(d.n, d.rows, d.signs, d.perm, psi, xform)
    y0 = op.apply_sparse(d.supp, d.vals)
    y = y0 + d.noise_scale(np.linalg.norm(y0)) * d.noise if d.noise is not None else y0
    if dtype == "f32":
        y = y.astype(np.float32).astype(np.float64)
    return op, y


def problem(cfg, sig, n, m, k, values="normal", snr_db=None, dtype="f64", randomizer="signs", psi=0, xform=0):
    """psi = 1: s is sparse in the basis F (A = D F R F), psi = 2: in the 2-D
    DCT basis; xform = 1: F is the real Fourier basis (partial Fourier)."""
    d = synth.draw_problem(cfg, sig, n, m, k, values, snr_db, randomizer=randomizer)
    op, y = build(d, dtype, psi, xform)
    return d, op, y
