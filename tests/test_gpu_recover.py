"""GPU parity of the greedy recoveries (OMP, SP, OMPR) against the FP64 oracle.

Supports must match exactly and s must agree to relative L2 <= 1e-5, with no
flag raised (a CG solve that hits its iteration cap fails the case).  The
cases here follow the oracle's trajectory exactly; divergent FP32
trajectories of noisy inputs are classified decision by decision in
tests/test_gpu_batched.py (tests/near_tie.py)."""
import numpy as np
import pytest

import oracle
import synth
from tests.gpu_common import announce, rel, to_dev, torch_dev
from tests.problems import problem

pytestmark = pytest.mark.gpu

RECOVER_CASES = [
    # name, cfg, n, m, k, values, snr, dtype, tol
    ("omp_n4096_f64", 1, 4096, 1024, 50, "normal_min0.1", None, "f64", 1e-10),
    ("omp_n4096_f32", 1, 4096, 1024, 50, "normal_min0.1", None, "f32", 1e-6),
    ("sp_small_noiseless_f64", 80, 2 ** 14, 2 ** 12, 100, "normal_min0.1", None, "f64", 1e-10),
    ("sp_small_noiseless_f32", 80, 2 ** 14, 2 ** 12, 100, "normal_min0.1", None, "f32", 1e-6),
    ("sp_small_40db_f64", 81, 2 ** 14, 2 ** 12, 100, "normal", 40.0, "f64", 1e-10),
    ("ompr_small_noiseless_f64", 82, 2 ** 14, 2 ** 12, 100, "normal_min0.1", None, "f64", 1e-10),
    ("ompr_small_noiseless_f32", 82, 2 ** 14, 2 ** 12, 100, "normal_min0.1", None, "f32", 1e-6),
    ("ompr_small_40db_f64", 83, 2 ** 14, 2 ** 12, 100, "normal", 40.0, "f64", 1e-10),
    ("sp_ragged_f32", 84, 2 ** 12, 1001, 37, "normal_min0.1", None, "f32", 1e-6),
    ("ompr_ragged_f64", 85, 2 ** 12, 777, 29, "normal", 35.0, "f64", 1e-10),
    ("cosamp_small_noiseless_f64", 80, 2 ** 14, 2 ** 12, 100, "normal_min0.1", None, "f64", 1e-10),
    ("cosamp_small_noiseless_f32", 80, 2 ** 14, 2 ** 12, 100, "normal_min0.1", None, "f32", 1e-6),
    ("cosamp_small_40db_f64", 81, 2 ** 14, 2 ** 12, 100, "normal", 40.0, "f64", 1e-10),
    ("cosamp_ragged_f32", 84, 2 ** 12, 1001, 37, "normal_min0.1", None, "f32", 1e-6),
    ("omprl3_small_40db_f64", 83, 2 ** 14, 2 ** 12, 100, "normal", 40.0, "f64", 1e-10),
    ("omprl4_small_noiseless_f32", 82, 2 ** 14, 2 ** 12, 100, "normal_min0.1", None, "f32", 1e-6),
    ("omprl5_ragged_f64", 85, 2 ** 12, 777, 29, "normal", 35.0, "f64", 1e-10),
    # the paper's randomizer: a permutation (signs +1), and a signed permutation
    ("sp_perm_40db_f64", 89, 2 ** 14, 2 ** 12, 100, "normal", 40.0, "f64", 1e-10, "perm"),
    ("ompr_perm_noiseless_f32", 89, 2 ** 14, 2 ** 12, 100, "normal_min0.1", None, "f32", 1e-6, "perm"),
    ("omp_perm_f64", 89, 4096, 1024, 50, "normal_min0.1", None, "f64", 1e-10, "signed_perm"),
    ("cosamp_perm_40db_f64", 89, 2 ** 14, 2 ** 12, 100, "normal", 40.0, "f64", 1e-10, "signed_perm"),
]


def _algo(name):
    """(algorithm, keyword arguments): 'omprl3' is OMPR with l = 3."""
    a = name.split("_")[0]
    if a.startswith("omprl"):
        return "ompr", {"l": int(a[5:])}
    return a, {}


@pytest.mark.parametrize("case", RECOVER_CASES, ids=[c[0] for c in RECOVER_CASES])
def test_recover_matches_oracle(case):
    name, cfg, n, m, k, values, snr, dt, tol = case[:9]
    randomizer = case[9] if len(case) > 9 else "signs"
    torch = torch_dev()
    import paper_1509_03979_amd as cs
    tdt = torch.float64 if dt == "f64" else torch.float32
    d, op, y = problem(cfg, 0, n, m, k, values, snr, dt, randomizer)
    algo, okw = _algo(name)
    ref = getattr(oracle, algo)(op, y, k, **okw)
    dop = cs.Operator.from_numpy(n, d.rows, d.signs, d.perm)
    announce("recover", name)
    fn = getattr(cs, f"cs_recover_{algo}")
    s, supp, info = fn(to_dev(y, tdt), dop, k, tol, **({"ompr_l": okw["l"]} if okw else {}))
    s = s.cpu().numpy()
    supp = supp.cpu().numpy()
    print(name, info, "oracle iters", ref.iters, ref.stop, flush=True)
    assert np.array_equal(supp, ref.support), (np.setdiff1d(supp, ref.support), np.setdiff1d(ref.support, supp))
    assert rel(s, ref.s) <= 1e-5
    assert np.count_nonzero(s[np.setdiff1d(np.arange(n), supp)]) == 0
    assert info["flags"] & ~cs.CS_F_NEAR_TIE == 0, info
    # the smallest decision margin: the GPU's (in its working precision; a lower
    # bound where a top-K did not see its first rejected key) against the
    # oracle's FP64 margins logged on the same trajectory
    om = min(m for (_, _, m) in ref.trace)
    mm = info["min_margin"]
    slack = (1e-9 if dt == "f64" else 1e-4) * float(np.linalg.norm(y))
    assert 0.0 <= mm <= om + slack, (mm, om)
    if algo == "omp":      # argmax decisions only: the runner-up is always seen
        assert abs(mm - om) <= slack, (mm, om)


ZERO_CASES = [
    # name, n, m, k, dtype: y = 0 makes every correlation magnitude equal, so each
    # selection is decided by the index tie-break alone.  At N = 16 all keys sit
    # in one candidate segment; at N = 2^14 and 4096 they overflow the segments
    # and the selection runs its passes over every key.
    ("sp_n16_f64", "sp", 16, 9, 4, "f64"),
    ("sp_n16_f32", "sp", 16, 9, 4, "f32"),
    ("sp_n2p14_f32", "sp", 2 ** 14, 2 ** 12, 100, "f32"),
    ("cosamp_n2p14_f64", "cosamp", 2 ** 14, 2 ** 12, 100, "f64"),
    ("ompr_n2p14_f32", "ompr", 2 ** 14, 2 ** 12, 100, "f32"),
    ("omp_n4096_f64", "omp", 4096, 1024, 20, "f64"),
]


@pytest.mark.parametrize("case", ZERO_CASES, ids=[c[0] for c in ZERO_CASES])
def test_zero_measurement_matches_oracle(case):
    name, algo, n, m, k, dt = case
    torch = torch_dev()
    import paper_1509_03979_amd as cs
    tdt = torch.float64 if dt == "f64" else torch.float32
    d, op, _ = problem(80, 0, n, m, k, "normal_min0.1", None, dt)
    y = np.zeros(m)
    ref = getattr(oracle, algo)(op, y, k)
    dop = cs.Operator.from_numpy(n, d.rows, d.signs)
    announce("recover zero y", name)
    s, supp, info = getattr(cs, f"cs_recover_{algo}")(to_dev(y, tdt), dop, k, 1e-6)
    supp = supp.cpu().numpy()
    print(name, info, flush=True)
    assert np.array_equal(supp, ref.support)
    assert np.array_equal(supp, np.arange(k))
    assert np.count_nonzero(s.cpu().numpy()) == 0
    # every key ties: the margins are 0 and the call says so
    assert info["min_margin"] == 0.0 and info["flags"] & cs.CS_F_NEAR_TIE, info


@pytest.mark.parametrize("psi", [0, 1])
@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_orthogonal_operator_is_hard_thresholding(psi, dt):
    """M = N makes A orthogonal (A^T A = I), so the least squares on any S is
    (A^T y)_S and OMP, SP, OMPR (eta = 1) and CoSaMP all return hard
    thresholding of A^T y: the K largest |A^T y| with those values."""
    torch = torch_dev()
    import paper_1509_03979_amd as cs
    tdt = torch.float64 if dt == "f64" else torch.float32
    n, k = 4096, 60
    rng = synth.rng_for(87, psi, 0)
    rows, signs = synth.draw_operator(rng, n, n)
    op = oracle.SRM(n, rows, signs, psi=psi)
    y = rng.standard_normal(n)
    if dt == "f32":
        y = y.astype(np.float32).astype(np.float64)
    c = op.adjoint(y)
    expect = np.sort(np.argsort(-np.abs(c), kind="stable")[:k])
    dop = cs.Operator.from_numpy(n, rows, signs, psi=psi)
    bar = 1e-12 if dt == "f64" else 1e-5
    for algo, kw in (("omp", {}), ("sp", {}), ("ompr", {"ompr_eta": 1.0}), ("cosamp", {})):
        announce("orthogonal", algo, dt, psi)
        s, supp, info = getattr(cs, f"cs_recover_{algo}")(to_dev(y, tdt), dop, k, 1e-12 if dt == "f64" else 1e-6, **kw)
        assert np.array_equal(supp.cpu().numpy(), expect), algo
        assert rel(s.cpu().numpy()[expect], c[expect]) <= bar, algo


DENSE_FALLBACK_CASES = [
    ("sp_small_noiseless_f32", 80, 2 ** 14, 2 ** 12, 100, "normal_min0.1", None, "f32", 1e-6),
    ("cosamp_small_40db_f64", 81, 2 ** 14, 2 ** 12, 100, "normal", 40.0, "f64", 1e-10),
    ("ompr_small_noiseless_f32", 82, 2 ** 14, 2 ** 12, 100, "normal_min0.1", None, "f32", 1e-6),
    ("sp_n2p16_40db_f32", 84, 2 ** 16, 2 ** 14, 300, "normal", 40.0, "f32", 1e-6),
]


@pytest.mark.parametrize("case", DENSE_FALLBACK_CASES, ids=[c[0] for c in DENSE_FALLBACK_CASES])
def test_top_k_dense_fallback_matches_oracle(case, monkeypatch):
    """Every dense top-K taken through its fallback (radix passes over every
    key, the output bitmap rewritten word by word) instead of the sampled
    band, which the band's checks select only when the sample misleads."""
    name, cfg, n, m, k, values, snr, dt, tol = case
    torch = torch_dev()
    import paper_1509_03979_amd as cs
    tdt = torch.float64 if dt == "f64" else torch.float32
    d, op, y = problem(cfg, 0, n, m, k, values, snr, dt)
    algo = name.split("_")[0]
    ref = getattr(oracle, algo)(op, y, k)
    dop = cs.Operator.from_numpy(n, d.rows, d.signs)
    monkeypatch.setenv("CS_SELECT_DENSE", "1")
    announce("recover dense fallback", name)
    s, supp, info = getattr(cs, f"cs_recover_{algo}")(to_dev(y, tdt), dop, k, tol)
    assert np.array_equal(supp.cpu().numpy(), ref.support)
    assert rel(s.cpu().numpy(), ref.s) <= 1e-5


EDGE_CASES = [
    # algo, n, m, k: one measurement; K = M = N; the smallest SP / OMPR / CoSaMP shapes; M = N
    ("omp", 16, 1, 1), ("omp", 16, 16, 16), ("sp", 16, 2, 1), ("ompr", 32, 4, 2), ("cosamp", 64, 3, 1),
    ("sp", 16, 16, 8), ("ompr", 16, 16, 5),
]


@pytest.mark.parametrize("algo,n,m,k", EDGE_CASES, ids=[f"{a}_n{n}_m{m}_k{k}" for a, n, m, k in EDGE_CASES])
@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_tiny_edge_shapes(algo, n, m, k, dt):
    torch = torch_dev()
    import paper_1509_03979_amd as cs
    tdt = torch.float64 if dt == "f64" else torch.float32
    d, op, y = problem(120, 0, n, m, k, "normal_min0.1", None, dt)
    ref = getattr(oracle, algo)(op, y, k)
    dop = cs.Operator.from_numpy(n, d.rows, d.signs)
    announce("edge", algo, n, m, k, dt)
    s, supp, info = getattr(cs, f"cs_recover_{algo}")(to_dev(y, tdt), dop, k, 1e-12 if dt == "f64" else 1e-6)
    assert np.array_equal(supp.cpu().numpy(), ref.support)
    assert rel(s.cpu().numpy(), ref.s) <= (1e-9 if dt == "f64" else 1e-5)
