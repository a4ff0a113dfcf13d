"""GPU parity with partial complex Fourier sensing of a real signal
(cs_op.xform = 2: y = D(FFT(R x)), the operator of Sec. II, complex
measurements) against the FP64 oracle's ``CPF`` (oracle/cpf.py, NumPy's FFT
with the real-inner-product adjoint): the operator entry points, least squares,
OMP / SP / OMPR / CoSaMP recoveries, the gradient (the binding's autograd with a
complex y) and the validation of the frequencies.  Bars as for the real
operators: FP64 1e-13 / FP32 3e-6 relative L2 for the operator; supports exact,
s within 1e-5; the gradient within 1e-8 (FP64) / 1e-3 (FP32)."""
import numpy as np
import pytest

import oracle
import synth
from oracle.cpf import CPF
from tests.gpu_common import announce, rel, to_dev, torch_dev

pytestmark = pytest.mark.gpu


def crel(a, b):
    a = np.asarray(a, dtype=np.complex128)
    b = np.asarray(b, dtype=np.complex128)
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))


def cdev(a, dt):
    """A complex device vector in the working precision."""
    torch = torch_dev()
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.complex128 if dt == "f64" else torch.complex64,
                           device="cuda")


def problem(cfg, sig, n, m, k, values, snr, dt):
    d = synth.draw_fourier_problem(cfg, sig, n, m, k, values, snr)
    op = CPF(d.n, d.rows, d.signs)
    y0 = op.apply_sparse(d.supp, d.vals)
    y = y0 if d.noise is None else y0 + d.noise_scale(np.linalg.norm(y0)) * d.noise
    if dt == "f32":   # the GPU gets complex64(y), the oracle complex128 of it
        y = y.astype(np.complex64).astype(np.complex128)
    return d, op, y


OP_CASES = [(16, 1, "f64"), (16, 7, "f32"), (1024, 301, "f32"), (4096, 2047, "f64"), (2 ** 16, 2 ** 13, "f32"),
            (2 ** 20, 2 ** 17, "f32"), (2 ** 20, 2 ** 17, "f64"), (2 ** 24, 2 ** 20, "f32")]


@pytest.mark.parametrize("n,m,dt", OP_CASES)
def test_apply(n, m, dt):
    torch = torch_dev()
    import paper_1509_03979_amd as cs
    tdt = torch.float64 if dt == "f64" else torch.float32
    d = synth.draw_fourier_problem(160, 0, n, m, 1, "normal", None)
    op = CPF(n, d.rows, d.signs)
    dop = cs.Operator.from_numpy(n, d.rows, d.signs, xform=2)
    rng = np.random.default_rng(7)
    x = rng.standard_normal(n)
    u = rng.standard_normal(m) + 1j * rng.standard_normal(m)
    bar = 1e-13 if dt == "f64" else 3e-6
    announce("apply complex fourier", n, m, dt)
    ax = cs.cs_apply_A(to_dev(x, tdt), dop).cpu().numpy()
    assert crel(ax, op.apply(x)) <= bar
    atu = cs.cs_apply_At(cdev(u, dt), dop).cpu().numpy()
    assert rel(atu, op.adjoint(u)) <= bar
    # A A* = I/2
    assert crel(cs.cs_apply_A(to_dev(atu, tdt), dop).cpu().numpy(), 0.5 * u) <= 2 * bar


def test_bad_frequencies_are_rejected():
    torch = torch_dev()
    import paper_1509_03979_amd as cs
    n = 1024
    rng = np.random.default_rng(8)
    signs = rng.choice([-1, 1], n).astype(np.int8)
    x = to_dev(rng.standard_normal(n), torch.float32)
    for fr in ([0, 5, 9], [3, 512], [5, 3], [1, 2, 2], [600]):
        dop = cs.Operator.from_numpy(n, np.array(fr), signs, xform=2)
        announce("complex fourier bad frequencies", fr)
        with pytest.raises(cs.CSError) as e:
            cs.cs_apply_A(x, dop)
        assert e.value.status == cs.CS_E_OP, fr
    dop = cs.Operator.from_numpy(n, np.arange(1, 512), signs, xform=2, psi=1)
    with pytest.raises(cs.CSError):
        cs.cs_apply_A(x, dop)


RECOVER_CASES = [
    # algo, cfg, n, m, k, values, snr, dtype, tol
    ("omp", 161, 4096, 400, 40, "normal_min0.1", None, "f64", 1e-10),
    ("omp", 162, 4096, 600, 60, "normal", 30.0, "f32", 1e-6),
    ("sp", 163, 2 ** 14, 2000, 400, "normal", 30.0, "f32", 1e-6),
    ("sp", 164, 2 ** 16, 4000, 1000, "normal", None, "f64", 1e-10),
    ("ompr", 165, 2 ** 12, 500, 80, "normal", 25.0, "f32", 1e-6),
    ("cosamp", 166, 2 ** 14, 2000, 300, "normal", 30.0, "f32", 1e-6),
]


@pytest.mark.parametrize("algo,cfg,n,m,k,values,snr,dt,tol", RECOVER_CASES)
def test_recover(algo, cfg, n, m, k, values, snr, dt, tol):
    torch = torch_dev()
    import paper_1509_03979_amd as cs
    d, op, y = problem(cfg, 0, n, m, k, values, snr, dt)
    ref = getattr(oracle, algo)(op, y, k)
    dop = cs.Operator.from_numpy(n, d.rows, d.signs, xform=2)
    announce("recover complex fourier", algo, n, m, k, dt)
    s, supp, info = getattr(cs, f"cs_recover_{algo}")(cdev(y, dt), dop, k, tol)
    assert info["flags"] & ~cs.CS_F_NEAR_TIE == 0, info
    assert np.array_equal(supp.cpu().numpy(), ref.support)
    assert rel(s.cpu().numpy(), ref.s) <= 1e-5
    if snr is None and values == "normal_min0.1":
        assert np.array_equal(ref.support, d.supp)
    # the complex residual norm
    assert abs(info["resid_norm"] - ref.resid_norm) <= 1e-4 * max(ref.resid_norm, 1e-3 * np.linalg.norm(y))
    if algo == "ompr":
        assert info["outer_iters"] == ref.iters


@pytest.mark.parametrize("dt,tol,bound", [("f64", 1e-12, 1e-10), ("f32", 1e-6, 1e-5)])
def test_ls_solve(dt, tol, bound):
    torch = torch_dev()
    import paper_1509_03979_amd as cs
    d, op, y = problem(167, 0, 2 ** 14, 1500, 200, "normal", 20.0, dt)
    rng = synth.rng_for(167, 0, 9)
    wrong = rng.choice(np.setdiff1d(np.arange(d.n), d.supp), 50, replace=False)
    S = np.sort(np.concatenate([d.supp[50:], wrong])).astype(np.int32)
    ref = oracle.ls(op, S, y)
    dop = cs.Operator.from_numpy(d.n, d.rows, d.signs, xform=2)
    announce("ls_solve complex fourier", dt)
    th, info = cs.cs_ls_solve(cdev(y, dt), dop, to_dev(S, torch.int32), tol)
    assert rel(th.cpu().numpy(), ref) <= bound, info
    x = np.zeros(d.n)
    x[S] = ref
    assert abs(info["resid_norm"] - np.linalg.norm(y - op.apply(x))) <= 1e-4 * np.linalg.norm(y)


@pytest.mark.parametrize("dt,bound", [("f64", 1e-8), ("f32", 1e-3)])
def test_gradient_through_sp(dt, bound):
    """SPRecover with a complex y: y.grad = dL/dRe y + i dL/dIm y against the
    oracle's gradient on the frozen support."""
    torch = torch_dev()
    import paper_1509_03979_amd as cs
    d, op, y = problem(168, 0, 2 ** 12, 500, 60, "normal", 30.0, dt)
    dop = cs.Operator.from_numpy(d.n, d.rows, d.signs, xform=2)
    yt = cdev(y, dt).requires_grad_(True)
    announce("gradient complex fourier", dt)
    s, supp = cs.SPRecover.apply(yt, dop, d.k, 1e-12 if dt == "f64" else 1e-6)
    t = d.s_dense()
    loss = ((s - torch.as_tensor(t, dtype=s.dtype, device="cuda")) ** 2).sum()
    loss.backward()
    g_ref, _ = __import__("oracle.adjoint", fromlist=["adjoint_gradient"]).adjoint_gradient(
        op, supp.cpu().numpy(), y, t)
    assert crel(yt.grad.cpu().numpy(), g_ref) <= bound


def test_batched_calls_reject_complex_sensing():
    torch = torch_dev()
    import paper_1509_03979_amd as cs
    d, op, y = problem(169, 0, 1024, 100, 10, "normal", None, "f32")
    dop = cs.Operator.from_numpy(d.n, d.rows, d.signs, xform=2)
    with pytest.raises(cs.CSError):
        cs.Batch([cdev(y, "f32")], [dop], [d.k])
