"""C-ABI checks that need no GPU: the library loads, exports every symbol the
header declares, validates arguments on the host before any device work, and
sizes its workspace as O(N + K)."""
import ctypes
import os
import re

import pytest

import paper_1509_03979_amd as cs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    text = open(os.path.join(ROOT, "include", "cs.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(cs_\w+)\s*\(", text)))


def test_every_declared_symbol_is_exported():
    names = header_functions()
    assert set(names) == set(cs.EXPORTS)
    for name in names:
        assert hasattr(cs.lib, name), name


def test_status_strings():
    for st in (cs.CS_OK, cs.CS_E_INVALID, cs.CS_E_SHAPE, cs.CS_E_OP, cs.CS_E_WORKSPACE, cs.CS_E_HIP):
        assert cs.cs_status_str(st) and cs.cs_status_str(st) != "unknown status"
    assert cs.cs_status_str(99) == "unknown status"


def test_workspace_is_linear_in_n_and_k():
    sz = lambda n, k, algo=cs.CS_ALGO_SP, dt=cs.CS_F32: cs.cs_workspace_size(dt, n, n // 4, k, algo)
    for dt in (cs.CS_F32, cs.CS_F64):
        a, b = sz(2 ** 20, 4096, dt=dt), sz(2 ** 21, 4096, dt=dt)
        assert 1.9 < b / a < 2.1
        esz = 4 if dt == cs.CS_F32 else 8
        # four dense N-vectors plus bitmaps
        assert 4 * esz * 2 ** 20 <= a <= 6 * esz * 2 ** 20
        k1, k2 = sz(2 ** 20, 1000, dt=dt), sz(2 ** 20, 31000, dt=dt)
        assert 0 < k2 - k1 <= 30000 * 2 * (3 * 4 + 7 * esz) + 8192
    assert cs.cs_workspace_size(cs.CS_F32, 1000, 100, 10, cs.CS_ALGO_SP) == 0     # N not a power of two
    assert cs.cs_workspace_size(cs.CS_F32, 1024, 2000, 10, cs.CS_ALGO_SP) == 0    # M > N
    assert cs.cs_workspace_size(cs.CS_F32, 1024, 100, 0, cs.CS_ALGO_SP) == 0      # K < 1
    assert cs.cs_workspace_size(7, 1024, 100, 10, cs.CS_ALGO_SP) == 0             # bad dtype
    assert cs.cs_workspace_size(cs.CS_F32, 2 ** 27, 100, 10, cs.CS_ALGO_SP) == 0  # N too large
    assert cs.cs_workspace_size(cs.CS_F32, 8, 4, 1, cs.CS_ALGO_SP) == 0           # N too small


def test_workspace_for_a_dct_basis():
    """cs_workspace_size_op reads n, m and psi from a host descriptor: Psi = I
    matches cs_workspace_size, the DCT basis adds two N-vectors, the 2-D DCT
    basis four and a stage table (and needs a square N), other psi values and
    batched descriptors with psi = 1 have no size."""
    for dt, esz in ((cs.CS_F32, 4), (cs.CS_F64, 8)):
        n, m, k = 2 ** 16, 2 ** 14, 300
        base = cs.cs_workspace_size(dt, n, m, k, cs.CS_ALGO_SP)
        op0 = cs.cs_op(n, m, None, None, None, 0, 0)
        op1 = cs.cs_op(n, m, None, None, None, 1, 0)
        assert cs.cs_workspace_size_op(dt, op0, k, cs.CS_ALGO_SP) == base
        extra = cs.cs_workspace_size_op(dt, op1, k, cs.CS_ALGO_SP) - base
        assert 2 * esz * n <= extra <= 2 * esz * n + 1024
        extra2 = cs.cs_workspace_size_op(dt, cs.cs_op(n, m, None, None, None, 2, 0), k, cs.CS_ALGO_SP) - base
        assert 4 * esz * n <= extra2 <= 4 * esz * n + 2 * esz * 8192 + 2048
        assert cs.cs_workspace_size_op(dt, cs.cs_op(2 * n, m, None, None, None, 2, 0), k, cs.CS_ALGO_SP) == 0
        assert cs.cs_workspace_size_op(dt, cs.cs_op(n, m, None, None, None, 3, 0), k, cs.CS_ALGO_SP) == 0
        items = (cs.cs_batch_item * 1)()
        items[0].op = op1
        items[0].k = 10
        assert cs.lib.cs_workspace_size_batched(dt, 1, items, cs.CS_ALGO_OMPR) == 0


def test_workspace_for_complex_fourier_sensing():
    """Partial complex Fourier sensing (xform = 2) with M frequencies sizes like
    the real operator with the 2M rows k, N - k, plus the expanded rows and
    data (2M int32 and 2M reals); M above N/2 - 1, psi != 0 and the batched
    calls have no size."""
    for dt, esz in ((cs.CS_F32, 4), (cs.CS_F64, 8)):
        n, m, k = 2 ** 16, 2 ** 13, 300
        real = cs.cs_workspace_size(dt, n, 2 * m, k, cs.CS_ALGO_SP)
        got = cs.cs_workspace_size_op(dt, cs.cs_op(n, m, None, None, None, 0, 2), k, cs.CS_ALGO_SP)
        assert 2 * m * (4 + esz) <= got - real <= 2 * m * (4 + esz) + 512
        assert cs.cs_workspace_size_op(dt, cs.cs_op(n, n // 2 - 1, None, None, None, 0, 2), k, cs.CS_ALGO_SP) > 0
        assert cs.cs_workspace_size_op(dt, cs.cs_op(n, n // 2, None, None, None, 0, 2), k, cs.CS_ALGO_SP) == 0
        assert cs.cs_workspace_size_op(dt, cs.cs_op(n, m, None, None, None, 1, 2), k, cs.CS_ALGO_SP) == 0
        assert cs.cs_workspace_size_op(dt, cs.cs_op(n, m, None, None, None, 0, 3), k, cs.CS_ALGO_SP) == 0
        # K up to 2M real rows; SP needs 2K <= 2M
        assert cs.cs_workspace_size_op(dt, cs.cs_op(n, 100, None, None, None, 0, 2), 150, cs.CS_ALGO_OMP) > 0
        assert cs.cs_workspace_size_op(dt, cs.cs_op(n, 100, None, None, None, 0, 2), 201, cs.CS_ALGO_OMP) == 0
        items = (cs.cs_batch_item * 1)()
        items[0].op = cs.cs_op(n, m, None, None, None, 0, 2)
        items[0].k = 10
        for algo in (cs.CS_ALGO_OMPR, cs.CS_ALGO_SP):
            assert cs.lib.cs_workspace_size_batched(dt, 1, items, algo) == 0


FAKE = 4096          # a 256-aligned fake device address: never dereferenced on these paths


def _call(fn, dt=cs.CS_F32, n=1024, m=256, k=10, tol=1e-6, y=FAKE, s=FAKE, supp=FAKE, ws=FAKE,
          ws_bytes=1 << 40, rows=FAKE, signs=FAKE, op=True):
    o = cs.cs_op(n, m, rows, signs)
    return fn(dt, ctypes.c_void_p(y) if y else None, ctypes.byref(o) if op else None, k, tol,
              ctypes.c_void_p(s) if s else None, ctypes.c_void_p(supp) if supp else None, None,
              ctypes.c_void_p(ws) if ws else None, ws_bytes, None, None)


@pytest.mark.parametrize("fn", [cs.lib.cs_recover_omp, cs.lib.cs_recover_sp, cs.lib.cs_recover_ompr,
                                cs.lib.cs_recover_cosamp])
def test_host_validation(fn):
    assert _call(fn, dt=5) == cs.CS_E_INVALID
    assert _call(fn, op=False) == cs.CS_E_INVALID
    assert _call(fn, rows=0) == cs.CS_E_INVALID
    assert _call(fn, n=1000) == cs.CS_E_SHAPE
    assert _call(fn, n=2 ** 27, m=100) == cs.CS_E_SHAPE
    assert _call(fn, m=2000) == cs.CS_E_SHAPE
    assert _call(fn, m=0) == cs.CS_E_SHAPE
    assert _call(fn, k=0) == cs.CS_E_INVALID
    assert _call(fn, k=300) == cs.CS_E_SHAPE
    assert _call(fn, y=0) == cs.CS_E_INVALID
    assert _call(fn, s=0) == cs.CS_E_INVALID
    assert _call(fn, supp=0) == cs.CS_E_INVALID
    assert _call(fn, tol=0.0) == cs.CS_E_INVALID
    assert _call(fn, tol=-1.0) == cs.CS_E_INVALID
    assert _call(fn, tol=float("nan")) == cs.CS_E_INVALID
    assert _call(fn, tol=float("inf")) == cs.CS_E_INVALID
    assert _call(fn, ws=0) == cs.CS_E_WORKSPACE
    assert _call(fn, ws=FAKE + 8) == cs.CS_E_WORKSPACE
    assert _call(fn, ws_bytes=100) == cs.CS_E_WORKSPACE
    assert cs.cs_last_error()


def test_sp_needs_2k_le_m():
    assert _call(cs.lib.cs_recover_sp, m=256, k=129) == cs.CS_E_SHAPE
    assert _call(cs.lib.cs_recover_cosamp, m=256, k=86) == cs.CS_E_SHAPE         # CoSaMP: 3K <= M
    assert _call(cs.lib.cs_recover_cosamp, m=256, k=85, ws_bytes=100) == cs.CS_E_WORKSPACE
    assert cs.cs_workspace_size(cs.CS_F32, 1024, 256, 86, cs.CS_ALGO_COSAMP) == 0
    o = cs.cs_op(1024, 256, FAKE, FAKE)
    for l in (-1, 11):                                                            # OMPR l in [1, K]
        prm = cs.cs_params(0, 0, 1, 0, 0.0, 0, l)
        assert cs.lib.cs_recover_ompr(cs.CS_F32, ctypes.c_void_p(FAKE), ctypes.byref(o), 10, 1e-6,
                                      ctypes.c_void_p(FAKE), ctypes.c_void_p(FAKE), ctypes.byref(prm),
                                      ctypes.c_void_p(FAKE), 1 << 40, None, None) == cs.CS_E_INVALID
    assert _call(cs.lib.cs_recover_ompr, m=256, k=129, ws_bytes=100) == cs.CS_E_WORKSPACE  # passes shape checks


def test_apply_and_ls_validation():
    o = cs.cs_op(1000, 10, FAKE, FAKE)
    assert cs.lib.cs_apply_A(cs.CS_F32, ctypes.byref(o), ctypes.c_void_p(FAKE), ctypes.c_void_p(FAKE),
                             ctypes.c_void_p(FAKE), 1 << 30, None) == cs.CS_E_SHAPE
    o = cs.cs_op(1024, 10, FAKE, FAKE)
    assert cs.lib.cs_apply_At(cs.CS_F64, ctypes.byref(o), None, ctypes.c_void_p(FAKE),
                              ctypes.c_void_p(FAKE), 1 << 30, None) == cs.CS_E_INVALID
    assert cs.lib.cs_apply_At(cs.CS_F64, ctypes.byref(o), ctypes.c_void_p(FAKE), ctypes.c_void_p(FAKE),
                              ctypes.c_void_p(FAKE), 10, None) == cs.CS_E_WORKSPACE
    assert cs.lib.cs_ls_solve(cs.CS_F32, ctypes.c_void_p(FAKE), ctypes.byref(o), ctypes.c_void_p(FAKE), 11, 1e-6,
                              None, ctypes.c_void_p(FAKE), None, ctypes.c_void_p(FAKE), 1 << 30, None,
                              None) == cs.CS_E_SHAPE
    assert cs.lib.cs_ls_solve(cs.CS_F32, ctypes.c_void_p(FAKE), ctypes.byref(o), ctypes.c_void_p(FAKE), 5, 0.0,
                              None, ctypes.c_void_p(FAKE), None, ctypes.c_void_p(FAKE), 1 << 30, None,
                              None) == cs.CS_E_INVALID


def test_adjoint_validation():
    o = cs.cs_op(1024, 256, FAKE, FAKE)
    adj = cs.lib.cs_adjoint_ls
    p = ctypes.c_void_p(FAKE)
    ok = dict(dt=cs.CS_F32, op=ctypes.byref(o), sup=p, k=10, g=p, tol=1e-6, gy=p, ws=p, wsb=1 << 30)

    def call(**kw):
        a = dict(ok, **kw)
        return adj(a["dt"], a["op"], a["sup"], a["k"], a["g"], a["tol"], a["gy"], None, a["ws"], a["wsb"], None,
                   None)

    assert call(dt=3) == cs.CS_E_INVALID
    assert call(op=None) == cs.CS_E_INVALID
    assert call(sup=None) == cs.CS_E_INVALID
    assert call(g=None) == cs.CS_E_INVALID
    assert call(gy=None) == cs.CS_E_INVALID
    assert call(k=0) == cs.CS_E_INVALID
    assert call(k=257) == cs.CS_E_SHAPE
    assert call(tol=float("nan")) == cs.CS_E_INVALID
    assert call(ws=None) == cs.CS_E_WORKSPACE
    assert call(wsb=64) == cs.CS_E_WORKSPACE
    o2 = cs.cs_op(1000, 256, FAKE, FAKE)
    assert call(op=ctypes.byref(o2)) == cs.CS_E_SHAPE


def test_shape_tuning_abi():
    for n in (16, 2 ** 14, 2 ** 18, 2 ** 20, 2 ** 24, 2 ** 26):
        for dt in (cs.CS_F32, cs.CS_F64):
            cand = cs.cs_shape_candidates(dt, n)
            assert cand, (n, dt)
            l = n.bit_length() - 2                       # log2(N / 2)
            assert all(a + b == l for a, b, _, _ in cand)
            assert len(set(cand)) == len(cand)
            for sh in cand:                              # every candidate installs, then the default returns
                cs.cs_set_shape(dt, n, sh)
            cs.cs_set_shape(dt, n, None)
    assert cs.lib.cs_shape_candidates(cs.CS_F32, 1000, None, 0) == 0
    assert cs.lib.cs_shape_candidates(7, 1024, None, 0) == 0
    with pytest.raises(cs.CSError):
        cs.cs_set_shape(cs.CS_F32, 2 ** 16, (9, 7, 2, 2))   # 9 + 7 is not log2(N/2) = 15
    with pytest.raises(cs.CSError):
        cs.cs_set_shape(cs.CS_F32, 2 ** 16, (8, 7, 0, 1))   # not compiled
    o = cs.cs_op(1 << 16, 100, FAKE, FAKE)
    ms = ctypes.c_double()
    sh = cs.cs_shape(8, 7, 2, 2)
    assert cs.lib.cs_time_shape(cs.CS_F32, ctypes.byref(o), None, 5, ctypes.c_void_p(FAKE), 1 << 30, None,
                                ctypes.byref(ms)) == cs.CS_E_INVALID
    assert cs.lib.cs_time_shape(cs.CS_F32, ctypes.byref(o), ctypes.byref(sh), 0, ctypes.c_void_p(FAKE), 1 << 30,
                                None, ctypes.byref(ms)) == cs.CS_E_INVALID
    assert cs.lib.cs_time_shape(cs.CS_F32, ctypes.byref(o), ctypes.byref(sh), 5, ctypes.c_void_p(FAKE), 10, None,
                                ctypes.byref(ms)) == cs.CS_E_WORKSPACE


def test_batched_validation():
    items = (cs.cs_batch_item * 2)()
    for i in range(2):
        items[i].op = cs.cs_op(1024, 256, FAKE, FAKE)
        items[i].y = items[i].s = items[i].support = FAKE
        items[i].k = 10
    f = cs.lib.cs_recover_ompr_batched
    ok = cs.lib.cs_workspace_size_batched(cs.CS_F32, 2, items, cs.CS_ALGO_OMPR)
    assert ok > 2 * cs.cs_workspace_size(cs.CS_F32, 1024, 256, 10, cs.CS_ALGO_OMPR)
    sp = cs.lib.cs_workspace_size_batched(cs.CS_F32, 2, items, cs.CS_ALGO_SP)
    assert sp >= 2 * cs.cs_workspace_size(cs.CS_F32, 1024, 256, 10, cs.CS_ALGO_SP)
    assert cs.lib.cs_workspace_size_batched(cs.CS_F32, 2, items, cs.CS_ALGO_OMP) == 0
    assert cs.lib.cs_workspace_size_batched(cs.CS_F32, 0, items, cs.CS_ALGO_OMPR) == 0
    ws = ctypes.c_void_p(FAKE)
    assert f(cs.CS_F32, 0, items, 1e-6, None, ws, ok, None, None) == cs.CS_E_INVALID
    assert f(cs.CS_F32, 2, None, 1e-6, None, ws, ok, None, None) == cs.CS_E_INVALID
    assert f(cs.CS_F32, 2, items, 0.0, None, ws, ok, None, None) == cs.CS_E_INVALID
    assert f(cs.CS_F32, 2, items, 1e-6, None, None, ok, None, None) == cs.CS_E_WORKSPACE
    prm = cs.cs_params(0, 0, 1, 100, 0.0)                  # cg_block not a multiple of 64
    assert f(cs.CS_F32, 2, items, 1e-6, ctypes.byref(prm), ws, ok, None, None) == cs.CS_E_INVALID
    items[1].k = 300                                      # K > M
    assert f(cs.CS_F32, 2, items, 1e-6, None, ws, ok, None, None) == cs.CS_E_SHAPE
    items[1].k = 10
    items[1].op = cs.cs_op(1000, 256, FAKE, FAKE)         # N not a power of two
    assert f(cs.CS_F32, 2, items, 1e-6, None, ws, ok, None, None) == cs.CS_E_SHAPE
    items[1].op = cs.cs_op(1024, 256, FAKE, FAKE)
    items[0].y = None
    assert f(cs.CS_F32, 2, items, 1e-6, None, ws, ok, None, None) == cs.CS_E_INVALID


def test_static_workspace_entry_validates_on_the_host():
    """cs_recover_sp_static checks its arguments and the static workspace's
    capacity before any device work (fake device addresses are never read)."""
    def call(dt=cs.CS_F32, n=1024, m=256, k=10, tol=1e-6, y=FAKE, s=FAKE, supp=FAKE):
        o = cs.cs_op(n, m, FAKE, FAKE)
        return cs.lib.cs_recover_sp_static(dt, ctypes.c_void_p(y) if y else None, ctypes.byref(o), k, tol,
                                           ctypes.c_void_p(s) if s else None,
                                           ctypes.c_void_p(supp) if supp else None, None, None, None)
    assert call(dt=5) == cs.CS_E_INVALID
    assert call(y=0) == cs.CS_E_INVALID
    assert call(tol=0.0) == cs.CS_E_INVALID
    assert call(m=256, k=129) == cs.CS_E_SHAPE                   # SP: 2K <= M
    assert call(n=2 ** 22, m=2 ** 20, k=16384) == cs.CS_E_WORKSPACE
    assert call(dt=cs.CS_F64, n=2 ** 21, m=2 ** 19, k=8192) == cs.CS_E_WORKSPACE
    assert "static workspace" in cs.cs_last_error()
    for dt, n in ((cs.CS_F32, 2 ** 21), (cs.CS_F64, 2 ** 20)):   # the largest sizes the header promises
        assert cs.cs_workspace_size(dt, n, n // 4, n // 256, cs.CS_ALGO_SP) <= cs.CS_STATIC_WS_BYTES


def test_sp_batched_validation():
    """cs_recover_sp_batched checks every item on the host first."""
    items = (cs.cs_batch_item * 2)()
    for i in range(2):
        items[i].op = cs.cs_op(1024, 256, FAKE, FAKE)
        items[i].y = items[i].s = items[i].support = FAKE
        items[i].k = 10
    f = cs.lib.cs_recover_sp_batched
    ok = cs.lib.cs_workspace_size_batched(cs.CS_F32, 2, items, cs.CS_ALGO_SP)
    ws = ctypes.c_void_p(FAKE)
    assert f(cs.CS_F32, 0, items, 1e-6, None, ws, ok, None, None) == cs.CS_E_INVALID
    assert f(cs.CS_F32, 2, items, float("nan"), None, ws, ok, None, None) == cs.CS_E_INVALID
    assert f(cs.CS_F32, 2, items, 1e-6, None, None, ok, None, None) == cs.CS_E_WORKSPACE
    items[1].k = 129                                      # SP: 2K > M
    assert f(cs.CS_F32, 2, items, 1e-6, None, ws, ok, None, None) == cs.CS_E_SHAPE
    assert cs.lib.cs_workspace_size_batched(cs.CS_F32, 2, items, cs.CS_ALGO_SP) == 0
    items[1].k = 10
    items[0].support = None
    assert f(cs.CS_F32, 2, items, 1e-6, None, ws, ok, None, None) == cs.CS_E_INVALID
    items[0].support = FAKE
    assert f(cs.CS_F32, 2, items, 1e-6, None, ws, 100, None, None) == cs.CS_E_WORKSPACE
