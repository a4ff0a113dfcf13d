"""GPU parity with partial Fourier sensing (Sec. II: Phi x = D(FFT(x))), for a
real signal written as the orthonormal real Fourier basis F (rows k and N-k
hold sqrt(2/N) Re and -sqrt(2/N) Im of Fourier coefficient k; row 0 and N/2 the
real ones), against the FP64 oracle (``SRM(xform=1)``): the operator entry
points (alone, with the basis itself as Psi, and with the 2-D DCT basis),
least squares, the four greedy recoveries, MRI-style sampling of whole
coefficients (rows in k, N-k pairs), the gradient, and a batched call.  Bars
as for the DCT-II operator: FP64 1e-13 / FP32 3e-6 (6e-6 with two transforms)
relative L2; supports exact, s within 1e-5."""
import numpy as np
import pytest

import oracle
import synth
from tests.gpu_common import announce, rel, to_dev, torch_dev
from tests.problems import build, problem

pytestmark = pytest.mark.gpu

OP_CASES = [
    # n, m, randomizer, psi, dtype
    (16, 9, "signs", 0, "f64"), (1024, 301, "perm", 0, "f32"), (4096, 1001, "perm", 0, "f64"),
    (2 ** 16, 2 ** 14, "signed_perm", 0, "f32"), (2 ** 20, 2 ** 18, "perm", 0, "f32"),
    (2 ** 20, 2 ** 18, "signs", 0, "f64"), (2 ** 24, 2 ** 21, "signs", 0, "f32"),
    (4096, 1001, "perm", 1, "f64"), (2 ** 18, 2 ** 16, "perm", 1, "f32"),
    (4096, 1001, "perm", 2, "f64"), (2 ** 20, 2 ** 18, "signs", 2, "f32"),
]


@pytest.mark.parametrize("n,m,randomizer,psi,dt", OP_CASES)
def test_apply_with_real_fourier(n, m, randomizer, psi, dt):
    torch = torch_dev()
    import paper_1509_03979_amd as cs
    tdt = torch.float64 if dt == "f64" else torch.float32
    d = synth.draw_problem(97, 0, n, m, 5, "normal", None, randomizer=randomizer)
    op = oracle.SRM(n, d.rows, d.signs, d.perm, psi=psi, xform=1)
    dop = cs.Operator.from_numpy(n, d.rows, d.signs, d.perm, psi=psi, xform=1)
    rng = np.random.default_rng(6)
    x = rng.standard_normal(n)
    u = rng.standard_normal(m)
    bar = 1e-13 if dt == "f64" else (3e-6 if psi == 0 else 6e-6)
    announce("apply fourier", n, m, randomizer, psi, dt)
    assert rel(cs.cs_apply_A(to_dev(x, tdt), dop).cpu().numpy(), op.apply(x)) <= bar
    atu = cs.cs_apply_At(to_dev(u, tdt), dop).cpu().numpy()
    assert rel(atu, op.adjoint(u)) <= bar
    assert rel(cs.cs_apply_A(to_dev(atu, tdt), dop).cpu().numpy(), u) <= 2 * bar


def test_bad_transform_is_rejected():
    torch = torch_dev()
    import paper_1509_03979_amd as cs
    d = synth.draw_problem(97, 1, 1024, 300, 5, "normal", None)
    dop = cs.Operator.from_numpy(1024, d.rows, d.signs, xform=1)
    ws = cs.workspace(cs.CS_F32, dop, 1, cs.CS_ALGO_OPERATOR)
    dop.c.xform = 3
    with pytest.raises(cs.CSError) as e:
        cs.cs_apply_A(to_dev(np.ones(1024), torch.float32), dop, ws=ws)
    assert e.value.status == cs.CS_E_OP


@pytest.mark.parametrize("n,m,k,dt,tol,bound", [(4096, 1024, 50, "f64", 1e-12, 1e-10),
                                                (2 ** 16, 2 ** 14, 300, "f32", 1e-6, 1e-5)])
def test_ls_solve_with_real_fourier(n, m, k, dt, tol, bound):
    torch = torch_dev()
    import paper_1509_03979_amd as cs
    tdt = torch.float64 if dt == "f64" else torch.float32
    d, op, y = problem(98, k, n, m, k, "normal", 30.0, dt, "perm", xform=1)
    rng = synth.rng_for(98, k, 9)
    wrong = rng.choice(np.setdiff1d(np.arange(n), d.supp), k // 4, replace=False)
    S = np.sort(np.concatenate([d.supp[k // 4:], wrong])).astype(np.int32)
    ref = oracle.ls(op, S, y)
    dop = cs.Operator.from_numpy(n, d.rows, d.signs, d.perm, xform=1)
    announce("ls_solve fourier", n, m, k, dt)
    th, info = cs.cs_ls_solve(to_dev(y, tdt), dop, to_dev(S, torch.int32), tol)
    assert rel(th.cpu().numpy(), ref) <= bound, info


RECOVER_CASES = [
    # name, cfg, n, m, k, values, snr, dtype, tol, randomizer, psi
    ("omp_n4096_f64", 99, 4096, 1024, 50, "normal_min0.1", None, "f64", 1e-10, "perm", 0),
    ("sp_n2p14_f32", 100, 2 ** 14, 2 ** 12, 100, "normal_min0.1", None, "f32", 1e-6, "signs", 0),
    ("sp_n2p14_40db_f64", 101, 2 ** 14, 2 ** 12, 100, "normal", 40.0, "f64", 1e-10, "perm", 0),
    ("ompr_n2p14_f64", 102, 2 ** 14, 2 ** 12, 100, "normal_min0.1", None, "f64", 1e-10, "perm", 0),
    ("cosamp_n2p14_f32", 103, 2 ** 14, 2 ** 12, 100, "normal_min0.1", None, "f32", 1e-6, "perm", 0),
    ("sp_spectrum_n2p14_f64", 104, 2 ** 14, 2 ** 12, 100, "normal_min0.1", None, "f64", 1e-10, "perm", 1),
    ("sp_2d_n2p14_f32", 105, 2 ** 14, 2 ** 12, 100, "normal_min0.1", None, "f32", 1e-6, "perm", 2),
]


@pytest.mark.parametrize("case", RECOVER_CASES, ids=[c[0] for c in RECOVER_CASES])
def test_recover_with_real_fourier(case):
    name, cfg, n, m, k, values, snr, dt, tol, randomizer, psi = case
    torch = torch_dev()
    import paper_1509_03979_amd as cs
    tdt = torch.float64 if dt == "f64" else torch.float32
    d, op, y = problem(cfg, 0, n, m, k, values, snr, dt, randomizer, psi=psi, xform=1)
    algo = name.split("_")[0]
    ref = getattr(oracle, algo)(op, y, k)
    dop = cs.Operator.from_numpy(n, d.rows, d.signs, d.perm, psi=psi, xform=1)
    announce("recover fourier", name)
    s, supp, info = getattr(cs, f"cs_recover_{algo}")(to_dev(y, tdt), dop, k, tol)
    s = s.cpu().numpy()
    supp = supp.cpu().numpy()
    print(name, info, "oracle iters", ref.iters, ref.stop, flush=True)
    assert np.array_equal(supp, ref.support), (np.setdiff1d(supp, ref.support), np.setdiff1d(ref.support, supp))
    assert rel(s, ref.s) <= 1e-5
    assert info["flags"] & ~cs.CS_F_NEAR_TIE == 0, info


@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_mri_style_whole_coefficients(dt):
    """Rows sampled in (k, N-k) pairs, so every measured Fourier coefficient
    is measured whole (real and imaginary part), plus the DC row: SP against
    the oracle on a noiseless sparse signal (the drawn support)."""
    torch = torch_dev()
    import paper_1509_03979_amd as cs
    tdt = torch.float64 if dt == "f64" else torch.float32
    n, pairs, k = 2 ** 14, 2 ** 11, 100
    rng = synth.rng_for(106, 0, 0)
    ks = np.sort(rng.choice(np.arange(1, n // 2), pairs, replace=False))
    rows = np.sort(np.concatenate([[0], ks, n - ks])).astype(np.int32)
    signs = (rng.integers(0, 2, n) * 2 - 1).astype(np.int8)
    perm = rng.permutation(n).astype(np.int32)
    supp = np.sort(rng.choice(n, k, replace=False))
    vals = rng.standard_normal(k)
    vals = np.where(np.abs(vals) < 0.1, 0.1 * np.sign(vals) + vals, vals)
    op = oracle.SRM(n, rows, signs, perm, xform=1)
    y = op.apply_sparse(supp, vals)
    if dt == "f32":
        y = y.astype(np.float32).astype(np.float64)
    ref = oracle.sp(op, y, k)
    assert np.array_equal(ref.support, supp)
    dop = cs.Operator.from_numpy(n, rows, signs, perm, xform=1)
    announce("mri-style sp", dt)
    s, sp_supp, info = cs.cs_recover_sp(to_dev(y, tdt), dop, k, 1e-10 if dt == "f64" else 1e-6)
    assert np.array_equal(sp_supp.cpu().numpy(), ref.support)
    assert rel(s.cpu().numpy(), ref.s) <= 1e-5


@pytest.mark.parametrize("dt,tol,bar", [("f64", 1e-12, 1e-8), ("f32", 1e-6, 1e-3)])
def test_adjoint_ls_with_real_fourier(dt, tol, bar):
    torch = torch_dev()
    import paper_1509_03979_amd as cs
    tdt = torch.float64 if dt == "f64" else torch.float32
    n, m, k = 4096, 1001, 37
    d, op, y = problem(107, 0, n, m, k, "normal", 30.0, dt, "perm", xform=1)
    t = d.s_dense()
    g_ref, s_hat = oracle.adjoint_gradient(op, d.supp, y, t)
    gs = np.random.default_rng(7).standard_normal(n)
    gs[d.supp] = 2.0 * (s_hat - t[d.supp])
    dop = cs.Operator.from_numpy(n, d.rows, d.signs, d.perm, xform=1)
    announce("adjoint_ls fourier", dt)
    gy, info = cs.cs_adjoint_ls(to_dev(gs, tdt), dop, to_dev(d.supp, torch.int32), tol)
    assert rel(gy.cpu().numpy(), g_ref) <= bar
    assert info["flags"] & ~cs.CS_F_NEAR_TIE == 0


def test_batched_ompr_with_real_fourier():
    """Signals of mixed N sensed by partial Fourier operators in one batched
    OMPR call (the batched passes share the row pass and its transform
    switch), each against the oracle."""
    torch = torch_dev()
    import paper_1509_03979_amd as cs
    sizes = synth.batched_sizes(6, 108, (10, 13))
    draws, ops, ys, dops = [], [], [], []
    for sig, (n, m, k) in enumerate(sizes):
        d = synth.draw_problem(108, sig, n, m, k, "normal", 30.0, randomizer="perm")
        op, y = build(d, "f64", 0, 1)
        draws.append(d)
        ops.append(op)
        ys.append(y)
        dops.append(cs.Operator.from_numpy(d.n, d.rows, d.signs, d.perm, xform=1))
    batch = cs.Batch([to_dev(y, torch.float64) for y in ys], dops, [d.k for d in draws])
    announce("batched fourier", sizes)
    s_list, supp_list, infos = cs.cs_recover_ompr_batched(batch, 1e-10)
    for i, d in enumerate(draws):
        ref = oracle.ompr(ops[i], ys[i], d.k)
        assert np.array_equal(supp_list[i].cpu().numpy(), ref.support), i
        assert rel(s_list[i].cpu().numpy(), ref.s) <= 1e-8, i
