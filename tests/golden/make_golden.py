"""Writes stored oracle results for full-size workloads (FP64 CPU oracle only).

    python tests/golden/make_golden.py sp_ompr_n2p20      # SP and OMPR, N = 2^20
    python tests/golden/make_golden.py sp_n2p24           # SP, N = 2^24 (noiseless)

Each file holds the measurements the GPU consumes (float32 y, from the
oracle's FP64 y = A s + noise; only up to N = 2^20, larger workloads recompute
y with measurements()) and the oracle's outputs on float64(float32(y)):
support, values, stop reason, outer iterations, the smallest decision margin.
Nothing here touches the GPU library.
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402

OUT = os.path.dirname(os.path.abspath(__file__))


def measurements(name: str, sig: int = 0):
    w = synth.WORKLOADS[name]
    d = synth.workload_problem(name, sig)
    op = oracle.SRM(d.n, d.rows, d.signs)
    y0 = op.apply_sparse(d.supp, d.vals)
    y = y0 + d.noise_scale(np.linalg.norm(y0)) * d.noise if d.noise is not None else y0
    y32 = y.astype(np.float32)
    return w, d, op, y32


def run(name: str, sig: int = 0, store_y: bool = True):
    w, d, op, y32 = measurements(name, sig)
    y = y32.astype(np.float64)
    out = {"y": y32} if store_y else {}
    meta = {"workload": name, "sig": sig, "n": d.n, "m": d.m, "k": d.k}
    for algo in w["algos"]:
        t = time.perf_counter()
        r = getattr(oracle, algo)(op, y, d.k)
        dt = time.perf_counter() - t
        margins = [m for (_, _, m) in r.trace]
        out[f"{algo}_support"] = r.support.astype(np.int32)
        out[f"{algo}_values"] = r.s[r.support]
        meta[algo] = {"stop": r.stop, "iters": int(r.iters), "resid_norm": r.resid_norm,
                      "min_margin": float(min(margins)) if margins else None, "seconds": dt,
                      "true_support_match": bool(np.array_equal(r.support, d.supp))}
        print(name, algo, meta[algo], flush=True)
    path = os.path.join(OUT, f"{name}_sig{sig}.npz")
    np.savez_compressed(path, meta=json.dumps(meta), **out)
    print("wrote", path)


if __name__ == "__main__":
    # y is stored for workloads small enough to keep in the repository (N <= 2^20);
    # larger ones recompute it with the oracle (measurements()).
    for nm in sys.argv[1:]:
        run(nm, store_y=synth.WORKLOADS[nm]["n"] <= 2 ** 20)
