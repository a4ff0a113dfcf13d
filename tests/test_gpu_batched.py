"""GPU parity of the batched OMPR call (signals of uneven N, M and K recovered
together through captured, replayed batched steps) against the FP64 oracle,
and its agreement with the single-signal call on the same inputs.

Bar per signal: the oracle's support exactly, s within relative L2 1e-5, the
oracle's number of swaps."""
import numpy as np
import pytest

import oracle
import synth
from tests.gpu_common import announce, rel, to_dev, torch_dev
from tests.problems import build

pytestmark = pytest.mark.gpu


def _batch(cfg, count, log_n, dtype):
    torch = torch_dev()
    import paper_1509_03979_amd as cs
    tdt = torch.float64 if dtype == "f64" else torch.float32
    draws, ops, ys, dops = [], [], [], []
    for sig in range(count):
        d = synth.batched_problem(sig, cfg, log_n)
        op, y = build(d, dtype)
        draws.append(d)
        ops.append(op)
        ys.append(y)
        dops.append(cs.Operator.from_numpy(d.n, d.rows, d.signs))
    batch = cs.Batch([to_dev(y, tdt) for y in ys], dops, [d.k for d in draws])
    return draws, ops, ys, dops, batch


@pytest.mark.parametrize("dtype,tol", [("f32", 1e-6), ("f64", 1e-10)])
def test_batched_ompr_matches_oracle(dtype, tol):
    import paper_1509_03979_amd as cs
    draws, ops, ys, dops, batch = _batch(86, 16, (10, 14), dtype)
    announce("batched ompr", dtype, [(d.n, d.m, d.k) for d in draws])
    s_list, supp_list, infos = cs.cs_recover_ompr_batched(batch, tol)
    for i, d in enumerate(draws):
        ref = oracle.ompr(ops[i], ys[i], d.k)
        supp = supp_list[i].cpu().numpy()
        assert np.array_equal(supp, ref.support), (i, np.setdiff1d(supp, ref.support), np.setdiff1d(ref.support, supp))
        assert rel(s_list[i].cpu().numpy(), ref.s) <= 1e-5, i
        assert infos[i]["outer_iters"] == ref.iters, (i, infos[i], ref.iters)
        assert infos[i]["flags"] & ~cs.CS_F_CG_MAXITER == 0, (i, infos[i])


def test_batched_equals_single_and_replays():
    """The same batch twice (the second call replays a fresh graph over the
    outputs of the first) and each signal through the single-signal call:
    identical supports, values within 1e-5."""
    torch = torch_dev()
    import paper_1509_03979_amd as cs
    draws, ops, ys, dops, batch = _batch(87, 12, (12, 15), "f32")
    announce("batched vs single", [(d.n, d.m, d.k) for d in draws])
    s1, p1, i1 = cs.cs_recover_ompr_batched(batch, 1e-6)
    first = [(s.cpu().numpy().copy(), p.cpu().numpy().copy()) for s, p in zip(s1, p1)]
    s2, p2, i2 = cs.cs_recover_ompr_batched(batch, 1e-6)
    for i, d in enumerate(draws):
        assert np.array_equal(first[i][1], p2[i].cpu().numpy())
        assert np.array_equal(first[i][0], s2[i].cpu().numpy())
        ss, sp, si = cs.cs_recover_ompr(batch.ys[i], dops[i], d.k, 1e-6)
        assert np.array_equal(sp.cpu().numpy(), first[i][1]), i
        assert rel(first[i][0], ss.cpu().numpy()) <= 1e-5, i
        assert i1[i]["outer_iters"] == si["outer_iters"], (i, i1[i], si)


def test_batched_single_signal_and_k1():
    """Degenerate batches: one signal; K = 1 (one-column least squares)."""
    torch = torch_dev()
    import paper_1509_03979_amd as cs
    d = synth.draw_problem(88, 0, 2 ** 12, 1000, 1, "normal", None)
    op, y = build(d, "f64")
    dop = cs.Operator.from_numpy(d.n, d.rows, d.signs)
    batch = cs.Batch([to_dev(y, torch.float64)], [dop], [1])
    announce("batched k1")
    s, supp, info = cs.cs_recover_ompr_batched(batch, 1e-12)
    ref = oracle.ompr(op, y, 1)
    assert np.array_equal(supp[0].cpu().numpy(), ref.support)
    assert rel(s[0].cpu().numpy(), ref.s) <= 1e-10


def _workload_256(dtype, tol, cg_block=0):
    import json
    import os
    torch = torch_dev()
    import paper_1509_03979_amd as cs
    path = os.path.join(os.path.dirname(__file__), "golden", "ompr_batched_256.npz")
    if not os.path.exists(path):
        pytest.skip("stored oracle results not generated")
    g = np.load(path, allow_pickle=False)
    meta = json.loads(str(g["meta"]))["signals"]
    offs = g["offsets"]
    w = synth.BATCHED_WORKLOAD
    tdt = torch.float64 if dtype == "f64" else torch.float32
    draws, ys, dops = [], [], []
    for sig in range(w["count"]):
        d = synth.batched_problem(sig, w["cfg"], w["log_n"])
        op, y = build(d, "f32")           # the stored results are on float64(float32(y))
        draws.append(d)
        ys.append(to_dev(y, tdt))
        dops.append(cs.Operator.from_numpy(d.n, d.rows, d.signs))
        assert abs(float(np.linalg.norm(y)) - meta[sig]["y_norm"]) <= 1e-9 * meta[sig]["y_norm"]
    batch = cs.Batch(ys, dops, [d.k for d in draws])
    announce("batched workload 256", dtype, tol)
    s_list, supp_list, infos = cs.cs_recover_ompr_batched(batch, tol, cg_block=cg_block)
    out = []
    for i, d in enumerate(draws):
        es = g["support"][offs[i]:offs[i + 1]].astype(np.int64)
        ev = g["values"][offs[i]:offs[i + 1]]
        ref = np.zeros(d.n)
        ref[es] = ev
        supp = supp_list[i].cpu().numpy()
        same = np.array_equal(supp, es)
        err = rel(s_list[i].cpu().numpy(), ref)
        scale = float(np.max(np.abs(ev))) if ev.size else 1.0
        out.append((i, same, err, meta[i], scale, infos[i]))
    return out


def test_batched_workload_256_fp64_matches_oracle_exactly():
    """The full batched workload (256 signals, N_i in 2^14..2^18, 30 dB) in
    FP64 with CG tol 1e-12: every signal's support equals the stored FP64
    oracle result (tests/golden/ompr_batched_256.npz, written by make_golden.py
    from oracle/ and synth/ only), with the same number of swaps and s within
    1e-8."""
    res = _workload_256("f64", 1e-12)
    bad = [(i, same, err, info["outer_iters"], m["iters"]) for i, same, err, m, _, info in res
           if not same or err > 1e-8 or info["outer_iters"] != m["iters"]]
    assert not bad, bad


def test_batched_workload_256_fp32_against_oracle():
    """The same workload as benchmarked (FP32, tol 1e-6).  A signal passes when
    its support equals the oracle's and s agrees to 1e-5.  A CG tolerance of
    1e-6 cannot resolve decisions whose FP64 margin is below about 1e-6 of the
    key scale, so a different trajectory is accepted only where the oracle
    logged such a near-tie; those signals are reported, and at least 80% of
    the signals must match exactly."""
    res = _workload_256("f32", 1e-6)
    exact = sum(1 for _, same, err, _, _, _ in res if same and err <= 1e-5)
    near = []
    for i, same, err, m, scale, _ in res:
        if same and err <= 1e-5:
            continue
        near.append((i, m["min_margin"] / scale))
        assert m["min_margin"] is not None and m["min_margin"] <= 1e-6 * scale, (i, m)
    print("exact", exact, "certified near-tie trajectories", near, flush=True)
    assert exact >= 0.8 * len(res)


def test_batched_with_permutation_randomizer():
    """Signals whose randomizer is a permutation (the paper's) in one batch."""
    torch = torch_dev()
    import paper_1509_03979_amd as cs
    sizes = synth.batched_sizes(6, 90, (10, 13))
    draws, ops, ys, dops = [], [], [], []
    for sig, (n, m, k) in enumerate(sizes):
        d = synth.draw_problem(90, sig, n, m, k, "normal", 30.0, randomizer="perm" if sig % 2 else "signed_perm")
        op, y = build(d, "f64")
        draws.append(d)
        ops.append(op)
        ys.append(y)
        dops.append(cs.Operator.from_numpy(d.n, d.rows, d.signs, d.perm))
    batch = cs.Batch([to_dev(y, torch.float64) for y in ys], dops, [d.k for d in draws])
    announce("batched perm", sizes)
    s_list, supp_list, infos = cs.cs_recover_ompr_batched(batch, 1e-10)
    for i, d in enumerate(draws):
        ref = oracle.ompr(ops[i], ys[i], d.k)
        assert np.array_equal(supp_list[i].cpu().numpy(), ref.support), i
        assert rel(s_list[i].cpu().numpy(), ref.s) <= 1e-8, i
