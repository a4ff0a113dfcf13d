#!/usr/bin/env python3
"""Throughput benchmark of CG-based greedy recovery on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME] [--algo sp|ompr|omp]

A step is one full recovery (support detection + CG least squares, every
outer iteration, through the operator A = D F R) of one synthetic signal whose
measurements are already resident in HBM.  `value` is recovered signals per
second: a step counts when its support equals the FP64 oracle's and its
coefficients agree to relative L2 <= 1e-5.

Default workload: SP on the one large signal, N = 2^24, M = 2^21, K = 2^16,
FP32 with FP64 CG reductions, noiseless, CG tol 1e-6 with warm starts.  Under
"extra": SP and OMPR on one signal with N = 2^20 (40 dB noise); the batched
256-signal OMPR; the differentiated 64-signal SP; the precision sweep on the
paper's own operator.

Prints ONE JSON line.  Besides metric, value, unit, timing and config it carries
  roofline      the dominant transform pass: algorithmic bytes per launch over
                its average launch time, from HIP events recorded by the
                library on its stream during a profiled replay of the timed
                steps (the timed steps themselves run without events), beside
                the 8 TB/s peak and a device copy measured in the same run;
  cpu_baseline  the FP64 oracle timed on this host's cores on the same input
                (a bounded sample of it where the whole recovery takes minutes).

Oracle side.  Every measurement vector handed to the GPU is formed by the FP64
oracle (y = A s + noise, rounded to FP32), and every expected result is the
oracle's (stored under tests/golden/ by make_golden.py, or computed here on a
subset); the GPU's own outputs never feed the oracle.  The oracle runs only in
the untimed parts of the run.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "signals recovered/s + % HBM roofline vs plain path at rel-err ≤1e-5"
REL_TOL = 1e-5


def host_threads() -> int:
    """Threads the oracle may use on this host: OMP_NUM_THREADS when set (the
    GPU hosts set it to their CPU share), else the CPUs this process may run on."""
    env = os.environ.get("OMP_NUM_THREADS", "")
    if env.isdigit() and int(env) > 0:
        return int(env)
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:
        return os.cpu_count() or 1


# the oracle's FFT threads follow the same count (read when oracle.operator loads)
os.environ.setdefault("CS_ORACLE_WORKERS", str(host_threads()))


def parse():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="sp_n2p24")
    ap.add_argument("--algo", default=None, help="sp, ompr or omp (default: the workload's first)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra", action="store_true", help="headline only (implies every --no-* leg below)")
    ap.add_argument("--no-profile", action="store_true", help="skip the profiled replay (roofline)")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched OMPR leg (256 signals)")
    ap.add_argument("--no-mid", action="store_true", help="skip the N = 2^20 SP/OMPR leg")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the differentiated SP leg (64 signals)")
    ap.add_argument("--no-single-loop", action="store_true", help="batched leg: skip the single-signal loop")
    ap.add_argument("--no-tune", action="store_true", help="keep the default transform shape (no autotuner)")
    ap.add_argument("--retune", action="store_true", help="tune live instead of using the shipped tuner cache")
    ap.add_argument("--write-tune-cache", action="store_true",
                    help="tune every workload size and the batched CG block, write the shipped cache, exit")
    ap.add_argument("--no-xi-sweep", action="store_true", help="skip the precision sweep on the paper's shape")
    ap.add_argument("--xi-sweep-max-log-n", type=int, default=18, help="largest log2 N of the precision sweep")
    ap.add_argument("--copy-mb", type=int, default=0,
                    help="end with three plain device copies of this many MiB (calibrates HBM byte counters)")
    return ap.parse_args()


# The sources that define the transform passes (their bodies, FFTs, device helpers,
# plan layout, launches and instantiations): counters taken on these stay valid
# while none of them changes; the drivers, selection and CG files do not enter.
PASS_SOURCES = ("cs_device.h", "cs_fft.h", "cs_inst.inc", "cs_internal.h", "cs_kernels.h", "cs_transform.hip")


def source_hash() -> str:
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1509_03979_amd", "csrc")
    for f in PASS_SOURCES:
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(f.encode() + fh.read())
    return h.hexdigest()[:16]


# ---------------------------------------------------------------- oracle side
def oracle_y(d, psi: int = 0):
    """y = A s (+ noise) by the FP64 oracle, rounded to FP32 (the GPU's input;
    the oracle's own runs take float64 of it)."""
    import oracle
    op = oracle.SRM(d.n, d.rows, d.signs, d.perm, psi)
    y0 = op.apply_sparse(d.supp, d.vals)
    y = y0 + d.noise_scale(np.linalg.norm(y0)) * d.noise if d.noise is not None else y0
    return op, y


class TransformCounter:
    """Counts the N-point transforms an oracle operator runs (its cost unit)."""

    def __init__(self, op):
        self.count = 0
        f, ft = op._F, op._Ft

        def cf(v):
            self.count += 1
            return f(v)

        def cft(w):
            self.count += 1
            return ft(w)

        op._F, op._Ft = cf, cft


def cpu_baseline_leg(name: str, algo: str, d, y32, gold_meta: dict) -> dict:
    """The FP64 oracle on the same input.  Where its whole recovery takes a few
    tens of seconds it is timed whole; at N = 2^24 (minutes) the sample is the
    recovery's first phase (A^T y, top-K, least squares on K columns,
    residual), and the time per N-point transform it measures is scaled to
    the transforms the oracle's full run performed (counted when its result
    was stored)."""
    import oracle
    op = oracle.SRM(d.n, d.rows, d.signs)
    y = y32.astype(np.float64)
    cnt = TransformCounter(op)
    full_tf = (gold_meta.get(algo) or {}).get("transforms")
    sampled = d.n > 2 ** 22 and full_tf
    t0 = time.perf_counter()
    if sampled:
        r = getattr(oracle, algo)(op, y, d.k, max_iter=0)
    else:
        r = getattr(oracle, algo)(op, y, d.k)
    tc = time.perf_counter() - t0
    if sampled:
        per_tf = tc / cnt.count
        est = per_tf * full_tf
        return {"value": round(1.0 / est, 6), "unit": "signals/s", "cores": host_threads(), "kind": "oracle",
                "sample": (f"first phase of one FP64 {algo.upper()} recovery of the benchmark signal "
                           f"({tc:.1f} s, {cnt.count} N-point transforms, {1e3 * per_tf:.0f} ms each), scaled to "
                           f"the {full_tf} transforms of the oracle's full recovery: {est:.0f} s per signal")}
    ok = bool(np.array_equal(r.support, np.asarray(gold_meta.get("_support", r.support))))
    return {"value": round(1.0 / tc, 6), "unit": "signals/s", "cores": host_threads(), "kind": "oracle",
            "sample": f"one full FP64 {algo.upper()} recovery of the benchmark signal ({tc:.1f} s)",
            "support_matches_stored": ok}


# ---------------------------------------------------------------- helpers
def load_inputs(name: str, torch, cs, sig: int = 0):
    """Seeded draw from synth; y from the stored oracle file when it holds one,
    else formed by the oracle here; expected results from the stored oracle
    run."""
    import synth
    w = synth.WORKLOADS[name]
    d = synth.workload_problem(name, sig)
    op = cs.Operator.from_numpy(d.n, d.rows, d.signs)
    gold_path = os.path.join(ROOT, "tests", "golden", f"{name}_sig{sig}.npz")
    expect = {}
    meta = {}
    g = np.load(gold_path, allow_pickle=False) if os.path.exists(gold_path) else None
    if g is not None:
        meta = json.loads(str(g["meta"]))
        for algo in w["algos"]:
            if f"{algo}_support" in g:
                expect[algo] = (g[f"{algo}_support"].astype(np.int64), g[f"{algo}_values"])
                meta.setdefault(algo, {})["_support"] = expect[algo][0]
    if g is not None and "y" in g:
        y32 = g["y"]
        y_src = "stored FP64 oracle measurements"
    else:
        _, y = oracle_y(d)
        y32 = y.astype(np.float32)
        y_src = "FP64 oracle y = A s (+ noise), rounded to FP32"
    dt = torch.float32 if w["dtype"] == "f32" else torch.float64
    y_dev = torch.as_tensor(y32 if w["dtype"] == "f32" else y32.astype(np.float64), dtype=dt, device="cuda")
    return w, d, op, y_dev, y32, expect, y_src, meta


def recovered(s, supp, exp) -> tuple[bool, float]:
    if exp is None:
        return False, float("nan")
    es, ev = exp
    supp = np.asarray(supp, dtype=np.int64)
    if not np.array_equal(supp, es):
        return False, float("nan")
    ref = np.zeros_like(s, dtype=np.float64)
    ref[es] = ev
    err = float(np.linalg.norm(s - ref) / np.linalg.norm(ref))
    return err <= REL_TOL, err


def profiled_roofline(torch, cs, step, steps: int, traffic_file: str, shape_in_use, copy_gbs=None):
    """Replay `steps` recoveries with per-launch HIP events on the library's
    stream (timing-only events: no system-scope cache flush around the launch)
    and return the roofline of the transform pass class with the largest share
    of transform time, plus the per-class totals.  Launches that exited at once
    because CG had converged are not counted."""
    cs.cs_prof_reset()
    cs.cs_prof_enable(True)
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    prof = cs.cs_prof_read()
    cs.cs_prof_enable(False)
    live = {k: v for k, v in prof.items() if v["launches"] > 0}
    if not live:
        return None, prof
    dom = max(live, key=lambda k: live[k]["total_ms"])
    st = live[dom]
    per_launch_bytes = st["bytes"] / st["launches"]
    avg_us = 1e3 * st["total_ms"] / st["launches"]
    achieved = st["bytes"] / (st["total_ms"] * 1e-3) / 1e9
    traffic = None
    tpath = os.path.join(ROOT, "profiles", traffic_file)
    if os.path.exists(tpath):
        t = json.load(open(tpath))
        cls = t.get("classes", {}).get(dom)
        if t.get("source_hash") == source_hash() and list(t.get("shape", [])) == list(shape_in_use) and cls:
            traffic = cls.get("hbm_bytes_per_launch")
    tot_bytes = sum(v["bytes"] for v in live.values())
    tot_ms = sum(v["total_ms"] for v in live.values())
    loop = tot_bytes / (tot_ms * 1e-3) / 1e9
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic, "kernel": dom,
            "avg_launch_us": round(avg_us, 3), "algorithmic_bytes_per_launch": per_launch_bytes,
            "launches_per_step": st["launches"] / steps,
            "share_of_transform_time": round(st["total_ms"] / tot_ms, 3),
            "all_transform_passes": {"achieved": round(loop, 1), "frac": round(loop / HBM_PEAK_GBS, 4)}}
    if copy_gbs:
        roof["measured_copy_GBs"] = round(copy_gbs, 1)
        roof["frac_of_measured_copy"] = round(achieved / copy_gbs, 4)
    return roof, prof


def copy_bandwidth(torch, mib: int = 2048, reps: int = 5) -> float:
    """Device-to-device copy of `mib` MiB (read + write counted), timed with
    events on the current stream: the bandwidth a plain streaming kernel
    reaches on this GPU."""
    src = torch.ones(mib << 18, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(2):
        dst.copy_(src)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        dst.copy_(src)
    b.record()
    torch.cuda.synchronize()
    gbs = 2.0 * src.numel() * 4 * reps / (a.elapsed_time(b) * 1e-3) / 1e9
    del src, dst
    torch.cuda.empty_cache()
    return gbs


def tuned_shape(cs, w, n, retune: bool):
    import paper_1509_03979_amd.tune as tune
    ent = tune.load(w["dtype"], tune.SHIPPED).get("shapes", {}).get(str(n))
    if ent and not retune:
        return {"shape": list(ent["shape"]), "default": ent.get("default"), "ms_per_happly": ent["ms"],
                "source": "shipped cache"}
    r = tune.tune_shapes([n], w["dtype"], reps=20)[n]
    return {"shape": list(r["shape"]), "default": list(r["default"]), "ms_per_happly": round(r["ms"], 4),
            "all": r["all"], "source": "live"}


def timed_steps(torch, step, steps: int):
    """Per-step wall times (each recovery returns with its results complete)."""
    times, outs = [], []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        a = time.perf_counter()
        outs.append(step())
        times.append(time.perf_counter() - a)
    torch.cuda.synchronize()
    return time.perf_counter() - t0, times, outs


def pct(times, q):
    return round(1e3 * float(np.percentile(np.asarray(times), q)), 4)


# ---------------------------------------------------------------- legs
def mid_leg(torch, cs, steps: int, with_cpu: bool) -> dict:
    """SP and OMPR on one signal with N = 2^20, M = 2^18, K = 4096, 40 dB
    (the working set sits in the 256 MB Infinity Cache: latency-bound)."""
    name = "sp_ompr_n2p20"
    w, d, op, y, y32, expect, y_src, meta = load_inputs(name, torch, cs)
    out = {"workload": name, "n": d.n, "m": d.m, "k": d.k, "y_source": y_src}
    for algo, reps in (("sp", steps), ("ompr", max(1, min(3, steps)))):
        fn = getattr(cs, f"cs_recover_{algo}")
        code = {"sp": cs.CS_ALGO_SP, "ompr": cs.CS_ALGO_OMPR}[algo]
        ws = cs.workspace(cs.CS_F32, op, d.k, code)
        step = lambda: fn(y, op, d.k, w["tol"], ws=ws)
        step()
        el, times, outs = timed_steps(torch, step, reps)
        ok = 0
        err = 0.0
        for s_t, supp_t, _ in outs:
            good, e = recovered(s_t.cpu().numpy().astype(np.float64), supp_t.cpu().numpy(), expect.get(algo))
            ok += int(good)
            err = max(err, e) if good else float("nan")
        r = {"signals_per_s": round(ok / el, 3), "ms_per_signal": round(1e3 * el / reps, 4),
             "p50_ms": pct(times, 50), "p90_ms": pct(times, 90), "recovered": ok, "of": reps,
             "max_rel_err": err, "info": outs[-1][2]}
        if algo == "sp":
            roof, _ = profiled_roofline(torch, cs, step, reps, f"traffic_{name}_sp.json",
                                        tuned_shape(cs, w, d.n, False)["shape"])
            r["roofline"] = roof
            if with_cpu:
                r["cpu_baseline"] = cpu_baseline_leg(name, algo, d, y32, meta)
        out[algo] = r
    return out


def batched_leg(torch, cs, count: int, loop_single: bool) -> dict:
    """Batched OMPR over the 256-signal workload (N_i in 2^14..2^18): one batched
    call per step, checked against the stored FP64 oracle results, beside the
    single-signal call looped over the same signals."""
    import synth
    tol = synth.BATCHED_WORKLOAD["tol"]
    gold = os.path.join(ROOT, "tests", "golden", f"ompr_batched_{count}.npz")
    g = np.load(gold, allow_pickle=False) if os.path.exists(gold) else None
    meta = json.loads(str(g["meta"]))["signals"] if g is not None else None
    ys, ops, ks, draws = [], [], [], []
    y_match = meta is not None
    for sig in range(count):
        d = synth.batched_problem(sig)
        _, y = oracle_y(d)
        y32 = y.astype(np.float32)
        if meta is not None:
            y_match &= abs(float(np.linalg.norm(y32.astype(np.float64))) - meta[sig]["y_norm"]) <= 1e-12 * meta[sig]["y_norm"]
        ys.append(torch.as_tensor(y32, device="cuda"))
        ops.append(cs.Operator.from_numpy(d.n, d.rows, d.signs))
        ks.append(d.k)
        draws.append(d)
    # autotuner: the shipped cache (transform shape per N, batched CG block size)
    # when it covers these sizes, else a live run
    import paper_1509_03979_amd.tune as tune
    ns = sorted({d.n for d in draws})
    ent = tune.load("f32", tune.SHIPPED)
    cached = ent.get("shapes", {})
    if all(str(n) in cached for n in ns) and "cg_block" in ent:
        shapes = {n: {"shape": cached[str(n)]["shape"], "default": cached[str(n)].get("default"),
                      "ms": cached[str(n)]["ms"]} for n in ns}
        cgt = {"cg_block": ent["cg_block"], "all": {}, "source": "shipped cache"}
    else:
        shapes = tune.tune_shapes(ns, "f32", reps=10)
        small = cs.Batch(ys[:32], ops[:32], ks[:32])
        cgt = tune.tune_cg_block(lambda b: cs.cs_recover_ompr_batched(small, tol, cg_block=b), reps=1)
    cgb = cgt["cg_block"]
    batch = cs.Batch(ys, ops, ks)
    cs.cs_recover_ompr_batched(batch, tol, cg_block=cgb)            # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s_list, supp_list, infos = cs.cs_recover_ompr_batched(batch, tol, cg_block=cgb)
    torch.cuda.synchronize()
    tb = time.perf_counter() - t0
    ok = checked = 0
    if g is not None:
        offs = g["offsets"]
        for i in range(count):
            es = g["support"][offs[i]:offs[i + 1]].astype(np.int64)
            ref = np.zeros(draws[i].n)
            ref[es] = g["values"][offs[i]:offs[i + 1]]
            good, _ = recovered(s_list[i].cpu().numpy().astype(np.float64), supp_list[i].cpu().numpy(), (es, ref[es]))
            ok += int(good)
            checked += 1
    mb = sum(i["model_bytes"] for i in infos)
    out = {"signals": count, "tol": tol, "seconds_per_batch": round(tb, 4), "signals_per_s": round(count / tb, 2),
           "on_oracle_trajectory": ok, "checked_against_oracle": checked,
           "other_trajectory": checked - ok,
           "note_other_trajectory": ("signals whose FP32 swaps leave the FP64 oracle's path are classified "
                                     "decision by decision in tests/test_gpu_batched.py (near-tie certificate)"),
           "on_trajectory_signals_per_s": round(ok / tb, 2) if checked else None,
           "inputs_are_oracle_y": True, "y_norms_match_stored": y_match,
           "swaps": sum(i["outer_iters"] for i in infos), "cg_iters": sum(i["cg_iters"] for i in infos),
           "model_gbytes": round(mb / 1e9, 3), "model_gb_per_s": round(mb / tb / 1e9, 1),
           "model_hbm_frac": round(mb / tb / 1e9 / HBM_PEAK_GBS, 4),
           "tuned": {"shapes": {str(n): {"shape": list(r["shape"]), "default": list(r["default"]),
                                         "ms_per_happly": round(r["ms"], 4)} for n, r in shapes.items()},
                     "cg_block": cgb, "cg_block_seconds": {str(k): round(v, 4) for k, v in cgt["all"].items()}}}
    if loop_single:
        t1 = time.perf_counter()
        for i in range(count):
            cs.cs_recover_ompr(ys[i], ops[i], ks[i], tol)
        torch.cuda.synchronize()
        tl = time.perf_counter() - t1
        out.update({"single_loop_seconds": round(tl, 3), "batched_speedup": round(tl / tb, 2)})
    return out


def adjoint_leg(torch, cs, batch: int, reps: int = 3, check: int = 4) -> dict:
    """Differentiated SP on the 64-signal workload (N = 2^16, M = 2^14, K = 300):
    forward recovery of the batch through cs_recover_sp_batched, and forward +
    backward of L = sum_b ||s_b - t_b||^2 with respect to y through the adjoint
    CG, beside the forward alone and beside the single-signal call looped over
    the batch.  The first
    `check` signals are checked against the oracle: its SP support and
    coefficients, and its dense gradient on that support."""
    import oracle
    import synth
    w = synth.WORKLOADS["sp_adjoint_n2p16"]
    ys, ops, ts, oops, y64s, draws = [], [], [], [], [], []
    for sig in range(batch):
        d = synth.workload_problem("sp_adjoint_n2p16", sig)
        oop, y = oracle_y(d)
        y32 = y.astype(np.float32)
        ys.append(torch.as_tensor(y32, device="cuda"))
        y64s.append(y32.astype(np.float64))
        oops.append(oop)
        ops.append(cs.Operator.from_numpy(d.n, d.rows, d.signs))
        ts.append(torch.as_tensor(d.s_dense(), dtype=torch.float32, device="cuda"))
        draws.append(d)
    k, tol = w["k"], w["tol"]

    bt = cs.Batch(ys, ops, [k] * batch, algo=cs.CS_ALGO_SP)

    def fwd_loop():
        return [cs.SPRecover.apply(ys[b], ops[b], k, tol)[0] for b in range(batch)]

    def fwd():
        return cs.cs_recover_sp_batched(bt, tol)

    def fwd_bwd():
        yl = [y.detach().requires_grad_(True) for y in ys]
        s, supp = cs.SPRecoverBatched.apply(yl, ops, k, tol, batch=bt)
        loss = sum(((s[b] - ts[b]) ** 2).sum() for b in range(batch))
        loss.backward()
        return yl, list(zip(s, supp))

    def timed(f):
        f()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            r = f()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / reps, r

    tl, _ = timed(fwd_loop)
    tf, _ = timed(fwd)
    tb, (yl, outs) = timed(fwd_bwd)
    supp_ok, s_err, g_err = 0, 0.0, 0.0
    for b in range(min(check, batch)):
        ref = oracle.sp(oops[b], y64s[b], k)
        s_b = outs[b][0].detach().cpu().numpy().astype(np.float64)
        supp_b = outs[b][1].cpu().numpy()
        if np.array_equal(supp_b, ref.support):
            supp_ok += 1
            s_err = max(s_err, float(np.linalg.norm(s_b - ref.s) / np.linalg.norm(ref.s)))
        g_ref, _ = oracle.adjoint_gradient(oops[b], supp_b, y64s[b], draws[b].s_dense())
        g_b = yl[b].grad.cpu().numpy().astype(np.float64)
        g_err = max(g_err, float(np.linalg.norm(g_b - g_ref) / np.linalg.norm(g_ref)))
    return {"batch": batch, "forward_s": round(tf, 4), "forward_backward_s": round(tb, 4),
            "forward_signals_per_s": round(batch / tf, 1), "forward_backward_signals_per_s": round(batch / tb, 1),
            "backward_over_forward": round((tb - tf) / tf, 3),
            "forward_single_call_loop_s": round(tl, 4), "batched_forward_speedup": round(tl / tf, 2),
            "checked_signals": min(check, batch), "support_matches_oracle": supp_ok,
            "max_rel_err_s": s_err, "max_rel_err_grad_vs_oracle_dense": g_err}


def xi_sweep_leg(torch, cs, ns, algos=("sp", "ompr", "omp")) -> dict:
    """The precision experiment of the paper's Tables II-IV on its own setup:
    M = N/4, K = M/4, N(0,1) nonzeros, noise sigma 0.01, Phi = D F R with R a
    random permutation and the signal sparse in the DCT basis (Psi = F, so
    A = D F R F), FP64: CG run to 'exact' precision (relative 1e-12) and
    stopped at the absolute thresholds ||r|| <= 1e-10 and <= 1e-5 of the CG
    loop test of Algorithm 1.  Per (algorithm, N): seconds per recovery and
    reconstruction SNR 20 log10(||s|| / ||s_hat - s||), with the SNR change
    against exact.  OMP (K iterations) runs up to N = 2^12, OMPR up to 2^14."""
    import synth
    out = {"operator": "A = D F R F (R a uniform random permutation, Psi = DCT-II)"}
    for n in ns:
        d = synth.paper_problem(n)
        op = cs.Operator.from_numpy(d.n, d.rows, d.signs, d.perm, psi=1)
        _, y64 = oracle_y(d, psi=1)
        y = torch.as_tensor(y64, dtype=torch.float64, device="cuda")
        s_np = d.s_dense()
        for algo in algos:
            if n > {"omp": 2 ** 12, "ompr": 2 ** 14}.get(algo, 2 ** 30):
                continue
            fn = getattr(cs, f"cs_recover_{algo}")
            row = {}
            for label, tol, absolute in [("exact", 1e-12, False)] + [(f"xi_{x:g}", x, True)
                                                                     for x in synth.PAPER_SHAPED["xis"]]:
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                s_hat, supp, info = fn(y, op, d.k, tol, tol_abs=absolute)
                torch.cuda.synchronize()
                dt = time.perf_counter() - t0
                err = np.linalg.norm(s_hat.cpu().numpy() - s_np)
                snr = float(20 * np.log10(np.linalg.norm(s_np) / err)) if err > 0 else float("inf")
                row[label] = {"seconds": round(dt, 5), "snr_db": round(snr, 4), "cg_iters": info["cg_iters"],
                              "outer_iters": info["outer_iters"]}
            for label in row:
                row[label]["snr_delta_vs_exact_db"] = round(row[label]["snr_db"] - row["exact"]["snr_db"], 4)
            out[f"{algo}_n{n}"] = row
    return out


def write_tune_cache(torch, cs):
    import paper_1509_03979_amd.tune as tune
    import synth
    bys, bops, bks = [], [], []
    for sig in range(32):
        dd = synth.batched_problem(sig)
        _, y = oracle_y(dd)
        bys.append(torch.as_tensor(y.astype(np.float32), device="cuda"))
        bops.append(cs.Operator.from_numpy(dd.n, dd.rows, dd.signs))
        bks.append(dd.k)
    small = cs.Batch(bys, bops, bks)
    data = tune.tune_workloads(tune.SHIPPED, 20, lambda b: cs.cs_recover_ompr_batched(small, 1e-6, cg_block=b))
    print(json.dumps(data), flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              f"(signals are independent: more GPUs would each take a share of them).", file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_1509_03979_amd as cs
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    if args.write_tune_cache:
        write_tune_cache(torch, cs)
        return
    if args.no_extra:
        args.no_mid = args.no_batched = args.no_adjoint = args.no_xi_sweep = True

    w, d, op, y, y32, expect, y_src, meta = load_inputs(args.workload, torch, cs)
    algo = args.algo or w["algos"][0]
    fn = getattr(cs, f"cs_recover_{algo}")
    dtc = cs.CS_F32 if w["dtype"] == "f32" else cs.CS_F64
    algo_code = {"omp": cs.CS_ALGO_OMP, "sp": cs.CS_ALGO_SP, "ompr": cs.CS_ALGO_OMPR}[algo]
    ws = cs.workspace(dtc, op, d.k, algo_code)
    tol = w["tol"]
    # the autotuner's choice for this device: the shipped cache when it has an
    # entry for this N, else a live tuning run (timed H-applies)
    tuned = None if args.no_tune else tuned_shape(cs, w, d.n, args.retune)
    step = lambda: fn(y, op, d.k, tol, ws=ws)

    for _ in range(args.warmup):
        step()
    elapsed, times, outs = timed_steps(torch, step, args.steps)

    ok_steps = 0
    errs = []
    first_s = outs[0][0].cpu().numpy()
    deterministic = True
    for s_t, supp_t, _ in outs:
        s_np = s_t.cpu().numpy().astype(np.float64)
        ok, err = recovered(s_np, supp_t.cpu().numpy(), expect.get(algo))
        ok_steps += int(ok)
        errs.append(err)
        deterministic &= bool(np.array_equal(s_np, first_s.astype(np.float64)))
    info = outs[-1][2]
    ms = 1e3 * elapsed / args.steps
    value = ok_steps / elapsed

    copy_gbs = copy_bandwidth(torch)
    roof = None
    prof = {}
    if not args.no_profile:
        in_use = tuned["shape"] if tuned else cs.cs_shape_candidates(dtc, d.n)[0]
        roof, prof = profiled_roofline(torch, cs, step, args.steps, f"traffic_{args.workload}_{algo}.json", in_use,
                                       copy_gbs)
    cpu = None if args.no_cpu_baseline else cpu_baseline_leg(args.workload, algo, d, y32, meta)

    extra = {"y_source": y_src, "deterministic": deterministic, "max_rel_err": max(errs) if errs else None,
             "p50_ms": pct(times, 50), "p90_ms": pct(times, 90), "min_ms": pct(times, 0),
             "model_gbytes_per_signal": round(info["model_bytes"] / 1e9, 4),
             "model_hbm_frac_whole_recovery": round(info["model_bytes"] / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
             "measured_copy_GBs": round(copy_gbs, 1),
             "info": info, "transform_prof": prof, "tuned_shape": tuned}
    if not args.no_mid and args.workload != "sp_ompr_n2p20":
        extra["sp_ompr_n2p20"] = mid_leg(torch, cs, args.steps, not args.no_cpu_baseline)
    if not args.no_batched:
        extra["ompr_batched_256"] = batched_leg(torch, cs, 256, not args.no_single_loop)
    if not args.no_adjoint:
        extra["sp_adjoint_n2p16"] = adjoint_leg(torch, cs, 64)
    if not args.no_xi_sweep:
        extra["xi_sweep_paper_shape"] = xi_sweep_leg(torch, cs, [2 ** l for l in range(12, args.xi_sweep_max_log_n + 1, 2)])

    line = {
        "metric": METRIC, "value": round(value, 4), "unit": "signals/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": w["dtype"], "data": "synthetic",
        "config": {"workload": args.workload, "algo": algo, "n": d.n, "m": d.m, "k": d.k, "tol": tol,
                   "snr_db": d.snr_db, "signals_per_step": 1},
        "roofline": roof, "cpu_baseline": cpu, "extra": extra,
    }
    print(json.dumps(line), flush=True)
    if args.copy_mb > 0:
        src = torch.ones(args.copy_mb << 18, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()


if __name__ == "__main__":
    main()
