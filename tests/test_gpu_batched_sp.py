"""cs_recover_sp_batched: many signals recovered by Subspace Pursuit in one
call (signals run concurrently, each through the single-signal driver).

Bar: every signal's result equals cs_recover_sp's on that signal (supports
equal, s within 1e-5; the same kernels run, so in practice bit for bit), and
matches the FP64 oracle's SP; the batched autograd function gives the oracle's
dense gradients."""
import numpy as np
import pytest

import oracle
import synth
from tests.gpu_common import announce, rel, to_dev, torch_dev
from tests.problems import build

pytestmark = pytest.mark.gpu


def _signals(count, dtype="f32"):
    w = synth.WORKLOADS["sp_adjoint_n2p16"]
    out = []
    for sig in range(count):
        # mixed sizes: the 2^16 workload, and smaller ones with other K
        if sig % 3 == 2:
            d = synth.draw_problem(131, sig, 2 ** 12, 1000 + sig, 20 + sig, "normal", 30.0)
        else:
            d = synth.draw_problem(w["cfg"], sig, w["n"], w["m"], w["k"], w["values"], w["snr_db"])
        op, y = build(d, dtype)
        out.append((d, op, y))
    return out


@pytest.mark.parametrize("dtype,tol", [("f32", 1e-6), ("f64", 1e-10)])
def test_sp_batched_equals_single_and_oracle(dtype, tol):
    torch = torch_dev()
    import paper_1509_03979_amd as cs
    tdt = torch.float64 if dtype == "f64" else torch.float32
    sigs = _signals(9, dtype)
    ys = [to_dev(y, tdt) for _, _, y in sigs]
    dops = [cs.Operator.from_numpy(d.n, d.rows, d.signs) for d, _, _ in sigs]
    batch = cs.Batch(ys, dops, [d.k for d, _, _ in sigs], algo=cs.CS_ALGO_SP)
    announce("sp batched", dtype, [(d.n, d.m, d.k) for d, _, _ in sigs])
    s_list, supp_list, infos = cs.cs_recover_sp_batched(batch, tol)
    for i, (d, op, y) in enumerate(sigs):
        s_b, p_b = s_list[i].cpu().numpy(), supp_list[i].cpu().numpy()
        s1, p1, i1 = cs.cs_recover_sp(ys[i], dops[i], d.k, tol)
        assert np.array_equal(p_b, p1.cpu().numpy()), i
        assert rel(s_b, s1.cpu().numpy()) <= 1e-5, i
        assert infos[i]["outer_iters"] == i1["outer_iters"] and infos[i]["flags"] == i1["flags"], (i, infos[i], i1)
        if i < 4 or d.n < 2 ** 16:
            ref = oracle.sp(op, y, d.k)
            assert np.array_equal(p_b, ref.support), i
            assert rel(s_b, ref.s) <= 1e-5, i


def test_sp_batched_repeat_and_single_signal():
    """The same batch twice gives the same outputs; a batch of one signal works."""
    torch = torch_dev()
    import paper_1509_03979_amd as cs
    sigs = _signals(4)
    ys = [to_dev(y, torch.float32) for _, _, y in sigs]
    dops = [cs.Operator.from_numpy(d.n, d.rows, d.signs) for d, _, _ in sigs]
    batch = cs.Batch(ys, dops, [d.k for d, _, _ in sigs], algo=cs.CS_ALGO_SP)
    announce("sp batched repeat")
    s1, p1, _ = cs.cs_recover_sp_batched(batch, 1e-6)
    first = [(s.cpu().numpy().copy(), p.cpu().numpy().copy()) for s, p in zip(s1, p1)]
    s2, p2, _ = cs.cs_recover_sp_batched(batch, 1e-6)
    for i in range(len(sigs)):
        assert np.array_equal(first[i][1], p2[i].cpu().numpy())
        assert np.array_equal(first[i][0], s2[i].cpu().numpy())
    one = cs.Batch(ys[:1], dops[:1], [sigs[0][0].k], algo=cs.CS_ALGO_SP)
    s3, p3, _ = cs.cs_recover_sp_batched(one, 1e-6)
    assert np.array_equal(p3[0].cpu().numpy(), first[0][1])


def test_sp_batched_autograd_matches_oracle_gradient():
    """SPRecoverBatched: forward through one batched call, backward through
    the adjoint CG per signal; y.grad against the oracle's dense gradient."""
    torch = torch_dev()
    import paper_1509_03979_amd as cs
    sigs = _signals(6)
    ys = [to_dev(y, torch.float32).requires_grad_(True) for _, _, y in sigs]
    dops = [cs.Operator.from_numpy(d.n, d.rows, d.signs) for d, _, _ in sigs]
    ks = {d.k for d, _, _ in sigs}
    assert len(ks) > 1       # mixed K: one call per K below
    announce("sp batched autograd")
    for k in sorted(ks):
        idx = [i for i, (d, _, _) in enumerate(sigs) if d.k == k]
        s, supp = cs.SPRecoverBatched.apply([ys[i] for i in idx], [dops[i] for i in idx], k, 1e-6)
        loss = sum(((s[j] - to_dev(sigs[i][0].s_dense(), torch.float32)) ** 2).sum() for j, i in enumerate(idx))
        loss.backward()
        for j, i in enumerate(idx):
            d, op, y = sigs[i]
            g_ref, _ = oracle.adjoint_gradient(op, supp[j].cpu().numpy(), y, d.s_dense())
            assert rel(ys[i].grad.cpu().numpy(), g_ref) <= 1e-3, i


def test_sp_batched_rejects_bad_items():
    torch = torch_dev()
    import paper_1509_03979_amd as cs
    sigs = _signals(2)
    ys = [to_dev(y, torch.float32) for _, _, y in sigs]
    dops = [cs.Operator.from_numpy(d.n, d.rows, d.signs) for d, _, _ in sigs]
    batch = cs.Batch(ys, dops, [d.k for d, _, _ in sigs], algo=cs.CS_ALGO_SP)
    batch.items[1].k = sigs[1][0].m          # 2K > M
    with pytest.raises(cs.CSError) as e:
        cs.cs_recover_sp_batched(batch, 1e-6)
    assert e.value.status == cs.CS_E_SHAPE
