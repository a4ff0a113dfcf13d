"""cs_recover_sp_static (no workspace argument, allocates nothing) against
cs_recover_sp through the C ABI: two calls in a row on the same GPU, the
second with a smaller input, so the second runs on what the first left in
the library's static workspace.  Same bar as the oracle parity tests:
supports equal and s within relative L2 1e-5 (the two calls run the same
kernels, so in practice they agree bit for bit)."""
import ctypes

import numpy as np
import pytest

from tests.gpu_common import announce, rel, to_dev, torch_dev
from tests.problems import problem

pytestmark = pytest.mark.gpu

CASES = [
    # name, cfg, n, m, k, values, snr, dtype, tol  (in call order: larger first)
    ("sp_n2p16_30db_f32", 95, 2 ** 16, 2 ** 14, 300, "normal", 30.0, "f32", 1e-6),
    ("sp_n4096_40db_f32", 96, 4096, 1024, 40, "normal", 40.0, "f32", 1e-6),
    ("sp_n2p14_40db_f64", 97, 2 ** 14, 2 ** 12, 100, "normal", 40.0, "f64", 1e-10),
    ("sp_n2p12_ragged_f64", 98, 2 ** 12, 1001, 37, "normal_min0.1", None, "f64", 1e-10),
]


def _static_call(cs, torch, y, dop, k, tol):
    """The new entry point through ctypes, outputs pre-filled with garbage."""
    s = torch.full((dop.n,), float("nan"), dtype=y.dtype, device=y.device)
    supp = torch.full((k,), -7, dtype=torch.int32, device=y.device)
    info = cs.cs_info()
    st = cs.lib.cs_recover_sp_static(cs._dtype_code(y), ctypes.c_void_p(y.data_ptr()), ctypes.byref(dop.c), k, tol,
                                     ctypes.c_void_p(s.data_ptr()), ctypes.c_void_p(supp.data_ptr()), None,
                                     ctypes.byref(info), ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == cs.CS_OK, cs.cs_last_error()
    return s.cpu().numpy(), supp.cpu().numpy(), info.as_dict()


def test_static_workspace_matches_workspace_call():
    torch = torch_dev()
    import paper_1509_03979_amd as cs
    for name, cfg, n, m, k, values, snr, dt, tol in CASES:
        tdt = torch.float64 if dt == "f64" else torch.float32
        d, _, y = problem(cfg, 0, n, m, k, values, snr, dt)
        dop = cs.Operator.from_numpy(n, d.rows, d.signs)
        yd = to_dev(y, tdt)
        announce("static-ws sp", name)
        s1, p1, i1 = _static_call(cs, torch, yd, dop, k, tol)
        announce("workspace sp", name)
        s0, p0, i0 = cs.cs_recover_sp(yd, dop, k, tol)
        s0, p0 = s0.cpu().numpy(), p0.cpu().numpy()
        print(name, "static", i1, "workspace", i0, flush=True)
        assert np.array_equal(p1, p0)
        assert rel(s1, s0) <= 1e-5
        assert np.count_nonzero(s1[np.setdiff1d(np.arange(n), p1)]) == 0
        assert i1["outer_iters"] == i0["outer_iters"] and i1["flags"] == i0["flags"]
        # the static call reads its loop flags synchronously, the workspace call
        # posts them and queues ahead: the same device iterations either way
        assert i1["cg_iters"] == i0["cg_iters"]


def test_static_workspace_rejects_large_sizes():
    """Sizes needing more than CS_STATIC_WS_BYTES fail on the host, outputs untouched."""
    torch = torch_dev()
    import paper_1509_03979_amd as cs
    n, m, k = 2 ** 22, 2 ** 20, 16384
    assert cs.cs_workspace_size(cs.CS_F32, n, m, k, cs.CS_ALGO_SP) > cs.CS_STATIC_WS_BYTES
    rows = torch.arange(m, dtype=torch.int32, device="cuda")
    signs = torch.ones(n, dtype=torch.int8, device="cuda")
    dop = cs.Operator(n, rows, signs)
    y = torch.zeros(m, dtype=torch.float32, device="cuda")
    s = torch.full((n,), 3.0, dtype=torch.float32, device="cuda")
    supp = torch.full((k,), -7, dtype=torch.int32, device="cuda")
    with pytest.raises(cs.CSError) as e:
        cs.cs_recover_sp_static(y, dop, k, 1e-6, s=s, support=supp)
    assert e.value.status == cs.CS_E_WORKSPACE
    assert bool((s == 3.0).all()) and bool((supp == -7).all())
