"""Writes stored oracle results for full-size workloads (FP64 CPU oracle only).

    python tests/golden/make_golden.py sp_ompr_n2p20      # SP and OMPR, N = 2^20
    python tests/golden/make_golden.py sp_n2p24           # SP, N = 2^24 (noiseless)
    python tests/golden/make_golden.py sp_ompr_n2p20:3:sp # signal 3, SP only
    python tests/golden/make_golden.py ompr_batched_256 6 # batched OMPR, 256 signals, 6 processes
    python tests/golden/make_golden.py sp_adjoint_n2p16_all 2  # SP on the 64 signals of N = 2^16

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


def count_transforms(op):
    """Counts the N-point transforms the oracle operator runs (wraps its F, F^T)."""
    box = [0]
    f, ft = op._F, op._Ft

    def cf(v):
        box[0] += 1
        return f(v)

    def cft(w):
        box[0] += 1
        return ft(w)

    op._F, op._Ft = cf, cft
    return box


def run(name: str, sig: int = 0, store_y: bool = True, algos=None):
    w, d, op, y32 = measurements(name, sig)
    y = y32.astype(np.float64)
    out = {"y": y32} if store_y else {}
    meta = {"workload": name, "sig": sig, "n": d.n, "m": d.m, "k": d.k}
    counter = count_transforms(op)
    for algo in (algos or w["algos"]):
        counter[0] = 0
        t = time.perf_counter()
        r = getattr(oracle, algo)(op, y, d.k)
        dt = time.perf_counter() - t
        margins = [m for (_, _, m) in r.trace]
        out[f"{algo}_support"] = r.support.astype(np.int32)
        out[f"{algo}_values"] = r.s[r.support]
        meta[algo] = {"stop": r.stop, "iters": int(r.iters), "resid_norm": r.resid_norm,
                      "min_margin": float(min(margins)) if margins else None, "seconds": dt,
                      "transforms": int(counter[0]), "true_support_match": bool(np.array_equal(r.support, d.supp))}
        print(name, algo, meta[algo], flush=True)
    path = os.path.join(OUT, f"{name}_sig{sig}.npz")
    if os.path.exists(path):
        # keep the other algorithms' results already stored for this signal
        old = np.load(path, allow_pickle=False)
        old_meta = json.loads(str(old["meta"]))
        for key in old.files:
            if key != "meta" and key not in out:
                out[key] = old[key]
        for key, val in old_meta.items():
            meta.setdefault(key, val)
    tmp = path + ".tmp.npz"
    np.savez_compressed(tmp, meta=json.dumps(meta), **out)
    os.replace(tmp, path)
    print("wrote", path)


def _batched_one(args):
    """Oracle OMPR on one signal of the batched workload (least squares by the
    oracle's FP64 CG route, tol 1e-13; cross-checked against the explicit
    routes by the pins)."""
    cfg, sig, part_dir = args
    path = os.path.join(part_dir, f"sig{sig:03d}.npz")
    if os.path.exists(path):
        return sig
    d = synth.batched_problem(sig, cfg)
    op = oracle.SRM(d.n, d.rows, d.signs)
    y0 = op.apply_sparse(d.supp, d.vals)
    y = (y0 + d.noise_scale(np.linalg.norm(y0)) * d.noise).astype(np.float32)
    t = time.perf_counter()
    r = oracle.ompr(op, y.astype(np.float64), d.k, ls_route="cg")
    dt = time.perf_counter() - t
    margins = [m for (_, _, m) in r.trace]
    meta = {"sig": sig, "n": d.n, "m": d.m, "k": d.k, "stop": r.stop, "iters": int(r.iters),
            "resid_norm": r.resid_norm, "min_margin": float(min(margins)) if margins else None, "seconds": dt,
            "y_norm": float(np.linalg.norm(y.astype(np.float64))), "y_sum": float(np.sum(y.astype(np.float64)))}
    # the trajectory: the index entering and the index leaving at each swap,
    # and the FP64 margins of each step's two decisions (entering argmax, drop)
    m_enter = np.array([m for (_, kind, m) in r.trace if kind == "argmax"])
    m_drop = np.array([m for (_, kind, m) in r.trace if kind == "drop"])
    np.savez(path + ".tmp.npz", meta=json.dumps(meta), support=r.support.astype(np.int32), values=r.s[r.support],
             moves_in=np.array([mv[0][0] for mv in r.moves], dtype=np.int32),
             moves_out=np.array([mv[1][0] for mv in r.moves], dtype=np.int32),
             margin_enter=m_enter, margin_drop=m_drop, margin_init=np.array([r.trace[0][2]]))
    os.replace(path + ".tmp.npz", path)
    print("batched sig", sig, meta, flush=True)
    return sig


def run_batched(count: int = 256, cfg: int = 4, procs: int = 6, part_dir: str | None = None):
    """All signals of the batched OMPR workload, largest first, in `procs`
    processes; per-signal parts are kept in part_dir so a run can resume, then
    packed into one file (concatenated supports and values + per-signal meta)."""
    import multiprocessing as mp
    part_dir = part_dir or os.path.join(OUT, ".parts_ompr_batched")
    os.makedirs(part_dir, exist_ok=True)
    sizes = synth.batched_sizes(count, cfg)
    order = sorted(range(count), key=lambda i: -sizes[i][0] * sizes[i][2])
    with mp.get_context("spawn").Pool(procs) as pool:
        for _ in pool.imap_unordered(_batched_one, [(cfg, i, part_dir) for i in order]):
            pass
    metas, supps, vals = [], [], []
    traj = {"moves_in": [], "moves_out": [], "margin_enter": [], "margin_drop": []}
    for sig in range(count):
        z = np.load(os.path.join(part_dir, f"sig{sig:03d}.npz"), allow_pickle=False)
        meta = json.loads(str(z["meta"]))
        meta["margin_init"] = float(z["margin_init"][0])
        metas.append(meta)
        supps.append(z["support"])
        vals.append(z["values"])
        for key in traj:
            traj[key].append(z[key])
    offs = np.cumsum([0] + [s.size for s in supps]).astype(np.int64)
    # swaps of signal i: moves_in[moff[i]:moff[i+1]]; decisions of signal i
    # (one more than its swaps when it stopped by declining a replacement):
    # margin_enter / margin_drop[doff[i]:doff[i+1]]
    moff = np.cumsum([0] + [a.size for a in traj["moves_in"]]).astype(np.int64)
    doff = np.cumsum([0] + [a.size for a in traj["margin_enter"]]).astype(np.int64)
    path = os.path.join(OUT, f"ompr_batched_{count}.npz")
    np.savez_compressed(path, meta=json.dumps({"cfg": cfg, "count": count, "ls_route": "cg", "signals": metas}),
                        offsets=offs, support=np.concatenate(supps), values=np.concatenate(vals),
                        move_offsets=moff, decision_offsets=doff,
                        **{key: np.concatenate(v) for key, v in traj.items()})
    print("wrote", path)


def _adjoint_one(sig):
    """Oracle SP on signal `sig` of the 64-signal differentiated workload."""
    w, d, op, y32 = measurements("sp_adjoint_n2p16", sig)
    y = y32.astype(np.float64)
    t = time.perf_counter()
    r = oracle.sp(op, y, d.k)
    meta = {"sig": sig, "stop": r.stop, "iters": int(r.iters), "seconds": time.perf_counter() - t,
            "y_norm": float(np.linalg.norm(y)), "true_support_match": bool(np.array_equal(r.support, d.supp))}
    print("adjoint sig", sig, meta, flush=True)
    return r.support.astype(np.int32), r.s[r.support], meta


def run_adjoint_all(procs: int = 2):
    """SP on all 64 signals of the differentiated workload (N = 2^16, M = 2^14,
    K = 300, 30 dB): supports and values, concatenated, with per-signal meta."""
    import multiprocessing as mp
    count = synth.WORKLOADS["sp_adjoint_n2p16"]["batch"]
    with mp.get_context("spawn").Pool(procs) as pool:
        res = pool.map(_adjoint_one, range(count))
    offs = np.cumsum([0] + [r[0].size for r in res]).astype(np.int64)
    path = os.path.join(OUT, "sp_adjoint_n2p16_all.npz")
    np.savez_compressed(path, meta=json.dumps({"workload": "sp_adjoint_n2p16", "count": count,
                                               "signals": [r[2] for r in res]}),
                        offsets=offs, support=np.concatenate([r[0] for r in res]),
                        values=np.concatenate([r[1] for r in res]))
    print("wrote", path)


if __name__ == "__main__":
    if sys.argv[1:2] == ["sp_adjoint_n2p16_all"]:
        run_adjoint_all(int(sys.argv[2]) if len(sys.argv) > 2 else 2)
        sys.exit(0)
    if sys.argv[1:2] == ["ompr_batched_256"]:
        run_batched(256, 4, int(sys.argv[2]) if len(sys.argv) > 2 else 6)
        sys.exit(0)
    # y is stored for signal 0 of workloads small enough to keep in the repository
    # (N <= 2^20, the benchmark's input); other signals and larger workloads
    # recompute it with the oracle (measurements()).  NAME[:SIG[:ALGO]]
    # picks a signal other than 0 and one of the workload's algorithms.
    for arg in sys.argv[1:]:
        parts = arg.split(":")
        nm = parts[0]
        sg = int(parts[1]) if len(parts) > 1 else 0
        run(nm, sg, store_y=synth.WORKLOADS[nm]["n"] <= 2 ** 20 and sg == 0, algos=parts[2:3] or None)
