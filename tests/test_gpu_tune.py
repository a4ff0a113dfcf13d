"""Every compiled transform shape gives the operator of the paper (checked
against the FP64 oracle), and the autotuner's choice is one of them and is
the one later calls use."""
import numpy as np
import pytest

import oracle
import synth
from tests.gpu_common import announce, rel, to_dev, torch_dev

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n", [2 ** 12, 2 ** 14, 2 ** 16, 2 ** 18, 2 ** 20])
def test_every_shape_matches_oracle(n):
    torch = torch_dev()
    import paper_1509_03979_amd as cs
    d = synth.draw_problem(95, 0, n, n // 3, 8, "normal", None)
    op = oracle.SRM(n, d.rows, d.signs)
    x = np.random.default_rng(3).standard_normal(n)
    u = np.random.default_rng(4).standard_normal(op.m)
    ax, atu = op.apply(x), op.adjoint(u)
    dop = cs.Operator.from_numpy(n, d.rows, d.signs)
    for dt, tdt, code, bar in (("f32", torch.float32, cs.CS_F32, 2e-6), ("f64", torch.float64, cs.CS_F64, 1e-13)):
        for sh in cs.cs_shape_candidates(code, n):
            announce("shape", n, dt, sh)
            cs.cs_set_shape(code, n, sh)
            try:
                assert rel(cs.cs_apply_A(to_dev(x, tdt), dop).cpu().numpy(), ax) <= bar, sh
                assert rel(cs.cs_apply_At(to_dev(u, tdt), dop).cpu().numpy(), atu) <= bar, sh
            finally:
                cs.cs_set_shape(code, n, None)


def test_tuner_installs_fastest_candidate(tmp_path, monkeypatch):
    torch_dev()
    import paper_1509_03979_amd as cs
    import paper_1509_03979_amd.tune as tune
    monkeypatch.setenv("CS_TUNE_CACHE", str(tmp_path / "tune.json"))
    ns = [2 ** 14, 2 ** 16]
    announce("tune", ns)
    res = tune.tune(ns, "f32", reps=5)
    for n in ns:
        cand = cs.cs_shape_candidates(cs.CS_F32, n)
        assert res[n]["shape"] in cand
        assert res[n]["ms"] == min(res[n]["all"].values())
    ent = tune.load("f32")
    assert {int(k) for k in ent["shapes"]} == set(ns)
    for n in ns:
        cs.cs_set_shape(cs.CS_F32, n, None)
