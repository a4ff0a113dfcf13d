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
