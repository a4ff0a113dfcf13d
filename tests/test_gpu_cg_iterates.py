"""The GPU CG takes the steps of the CG function of Algorithm 1: with the
iteration cap set and a tolerance no iterate meets (1e-30), j iterations of
the GPU solve (cold or warm started) equal j iterations of the oracle's FP64
operator CG on the same support.  This pins the iterate itself, not only the
converged least-squares point: the vector update that the column passes carry
into the next iteration, the step taken from per-workgroup partials, the
residual norm by expansion, and the last step applied after the solve stops
(at the cap), through the four-step operator, the DCT basis (psi = 1) and the
separable 2-D DCT basis (psi = 2).  Bars: FP64 1e-10, FP32 1e-4 relative L2
(FP32 vectors, FP64 inner products)."""
import numpy as np
import pytest

import oracle
import synth
from tests.gpu_common import announce, rel, to_dev, torch_dev
from tests.problems import problem

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("warm", [False, True])
@pytest.mark.parametrize("iters", [1, 2, 5])
@pytest.mark.parametrize("dt", ["f64", "f32"])
@pytest.mark.parametrize("psi", [0, 1, 2])
def test_cg_iterates_match_oracle(psi, dt, iters, warm):
    torch = torch_dev()
    import paper_1509_03979_amd as cs
    tdt = torch.float64 if dt == "f64" else torch.float32
    n, m, k = 4096, 1024, 60
    d, op, y = problem(131, psi, n, m, k, "normal", 30.0, dt, "perm", psi=psi)
    S = np.sort(d.supp).astype(np.int32)
    x0 = None
    if warm:
        # a start away from the solution: the true values plus a perturbation
        s_map = dict(zip(d.supp.tolist(), d.vals.tolist()))
        x0 = np.array([s_map[j] for j in S]) + 0.3 * synth.rng_for(131, psi, 5).standard_normal(k)
        if dt == "f32":
            x0 = x0.astype(np.float32).astype(np.float64)
    ref, it = oracle.ls_cg(op, S, y, tol=1e-30, max_iter=iters, x0=x0)
    assert it == iters
    dop = cs.Operator.from_numpy(n, d.rows, d.signs, d.perm, psi=psi)
    announce("cg iterates", psi, dt, iters, warm)
    th, info = cs.cs_ls_solve(to_dev(y, tdt), dop, to_dev(S, torch.int32), 1e-30,
                              x0=to_dev(x0, tdt) if warm else None, cg_max_iter=iters)
    assert info["cg_iters"] == iters, info
    assert info["flags"] & cs.CS_F_CG_MAXITER, info
    bar = 1e-10 if dt == "f64" else 1e-4
    assert rel(th.cpu().numpy(), ref) <= bar, (rel(th.cpu().numpy(), ref), info)
