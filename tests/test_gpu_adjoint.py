"""GPU parity of the differentiated recovery (the backward of the least-squares
step on the frozen final support) against the FP64 oracle's dense gradient
and against central finite differences.

On a frozen support S the recovered coefficients are s_S = (A_S^T A_S)^-1
A_S^T y (Eq. (11)), so dL/dy = A_S (A_S^T A_S)^-1 (dL/ds)_S: one more CG solve
and one forward apply.  Bar: relative error <= 1e-3 in FP32, 1e-8 in FP64."""
import numpy as np
import pytest

import oracle
import synth
from tests.gpu_common import announce, rel, to_dev, torch_dev
from tests.problems import build, problem

pytestmark = pytest.mark.gpu

ADJ_CASES = [
    # name, cfg, n, m, k, values, snr, dtype, tol, bar
    ("ragged_f64", 90, 2 ** 12, 1001, 37, "normal", 30.0, "f64", 1e-12, 1e-8),
    ("ragged_f32", 90, 2 ** 12, 1001, 37, "normal", 30.0, "f32", 1e-6, 1e-3),
    ("k1_f64", 91, 256, 64, 1, "normal", None, "f64", 1e-12, 1e-8),
    ("n16_f64", 92, 16, 9, 4, "normal", 20.0, "f64", 1e-12, 1e-8),
    ("c5_shape_f32", 5, 2 ** 16, 2 ** 14, 300, "normal", 30.0, "f32", 1e-6, 1e-3),
    ("c5_shape_f64", 5, 2 ** 16, 2 ** 14, 300, "normal", 30.0, "f64", 1e-12, 1e-8),
]


@pytest.mark.parametrize("case", ADJ_CASES, ids=[c[0] for c in ADJ_CASES])
def test_adjoint_ls_matches_oracle(case):
    name, cfg, n, m, k, values, snr, dt, tol, bar = case
    torch = torch_dev()
    import paper_1509_03979_amd as cs
    tdt = torch.float64 if dt == "f64" else torch.float32
    d, op, y = problem(cfg, 0, n, m, k, values, snr, dt)
    t = d.s_dense()
    g_ref, s_hat = oracle.adjoint_gradient(op, d.supp, y, t)
    # dL/ds = 2 (s_hat - t) on S; entries off S must be ignored, so fill them with junk
    gs = np.random.default_rng(7).standard_normal(n)
    gs[d.supp] = 2.0 * (s_hat - t[d.supp])
    dop = cs.Operator.from_numpy(n, d.rows, d.signs)
    announce("adjoint_ls", name)
    gy, info = cs.cs_adjoint_ls(to_dev(gs, tdt), dop, to_dev(d.supp, torch.int32), tol)
    gy = gy.cpu().numpy()
    print(name, info, flush=True)
    assert rel(gy, g_ref) <= bar, rel(gy, g_ref)
    assert info["flags"] == 0


def _c5_signal(sig, dtype="f32"):
    w = synth.WORKLOADS["sp_adjoint_n2p16"]
    d = synth.draw_problem(w["cfg"], sig, w["n"], w["m"], w["k"], w["values"], w["snr_db"])
    op, y = build(d, dtype)
    return w, d, op, y


def _c5_oracle_sp(sig, op, y, k):
    """The oracle's SP on signal `sig` of the 64-signal workload: the stored
    result (tests/golden/sp_adjoint_n2p16_all.npz, written by make_golden.py
    from oracle/ and synth/ only) when present, else computed here."""
    import json
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "sp_adjoint_n2p16_all.npz")
    if os.path.exists(path):
        g = np.load(path, allow_pickle=False)
        offs = g["offsets"]
        meta = json.loads(str(g["meta"]))["signals"][sig]
        assert abs(float(np.linalg.norm(y)) - meta["y_norm"]) <= 1e-12 * meta["y_norm"]
        supp = g["support"][offs[sig]:offs[sig + 1]].astype(np.int64)
        s = np.zeros(op.n)
        s[supp] = g["values"][offs[sig]:offs[sig + 1]]
        return supp, s
    ref = oracle.sp(op, y, k)
    return ref.support, ref.s


@pytest.mark.parametrize("chunk", range(8))
def test_sp_autograd_matches_oracle_gradient(chunk):
    """SPRecover forward + backward of L = ||s_hat - t||^2 on the 64-signal
    workload (signals 8 chunk .. 8 chunk + 7): each support equals the oracle
    SP's, s is within 1e-5, and y.grad equals the oracle's dense gradient on
    that support within 1e-3.  Without the stored oracle results only the
    chunk's first signal runs."""
    import os
    torch = torch_dev()
    import paper_1509_03979_amd as cs
    stored = os.path.exists(os.path.join(os.path.dirname(__file__), "golden", "sp_adjoint_n2p16_all.npz"))
    sigs = range(8 * chunk, 8 * chunk + 8) if stored else [8 * chunk]
    for sig in sigs:
        w, d, op, y = _c5_signal(sig)
        ref_supp, ref_s = _c5_oracle_sp(sig, op, y, d.k)
        dop = cs.Operator.from_numpy(d.n, d.rows, d.signs)
        yt = to_dev(y, torch.float32).requires_grad_(True)
        tt = to_dev(d.s_dense(), torch.float32)
        announce("SPRecover forward/backward", sig)
        s, supp = cs.SPRecover.apply(yt, dop, d.k, w["tol"])
        loss = ((s - tt) ** 2).sum()
        loss.backward()
        supp = supp.cpu().numpy()
        assert np.array_equal(supp, ref_supp), sig
        assert rel(s.detach().cpu().numpy(), ref_s) <= 1e-5, sig
        g_ref, _ = oracle.adjoint_gradient(op, ref_supp, y, d.s_dense())
        err = rel(yt.grad.cpu().numpy(), g_ref)
        print("signal", sig, "grad rel err", err, flush=True)
        assert err <= 1e-3, sig


def test_c5_gradient_matches_central_differences():
    """32 (signal, coordinate) pairs: the FP32 backward against central
    differences (h = 1e-3) of L(y) on the frozen support, L evaluated by the
    oracle's FP64 least squares on that support (Cholesky of the closed-form
    Gram); L is exactly quadratic in y there, so the differences are exact up
    to rounding."""
    torch = torch_dev()
    import paper_1509_03979_amd as cs
    w = synth.WORKLOADS["sp_adjoint_n2p16"]
    pairs = synth.fd_coordinates(w["batch"], w["m"], 32, w["cfg"])
    h = 1e-3
    by_sig = {}
    for sig, c in pairs:
        by_sig.setdefault(sig, []).append(c)
    fd, an = [], []
    for sig, coords in sorted(by_sig.items()):
        _, d, op, y = _c5_signal(sig)
        dop = cs.Operator.from_numpy(d.n, d.rows, d.signs)
        t = d.s_dense()
        yt = to_dev(y, torch.float32).requires_grad_(True)
        announce("fd signal", sig)
        s, supp = cs.SPRecover.apply(yt, dop, d.k, w["tol"])
        ((s - to_dev(t, torch.float32)) ** 2).sum().backward()
        g = yt.grad.cpu().numpy()
        supp_np = supp.cpu().numpy()
        off = float(np.sum(np.delete(t, supp_np) ** 2))

        gen = oracle.gram_generator(op)

        def loss(yy):
            th = oracle.ls_gram(op, supp_np, yy, gen)
            return float(np.sum((th - t[supp_np]) ** 2)) + off

        for c in coords:
            e = np.zeros(d.m)
            e[c] = h
            fd.append((loss(y + e) - loss(y - e)) / (2 * h))
            an.append(g[c])
    fd, an = np.array(fd), np.array(an)
    print("fd", fd[:4], "an", an[:4], flush=True)
    assert rel(an, fd) <= 1e-3
