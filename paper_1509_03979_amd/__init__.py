"""Python binding of libcsrecover (CG-based greedy compressive-sensing recovery on MI355X).

Argument marshalling only: every step of the recovery runs in the HIP library.
PyTorch provides device memory and the stream; the functions below carry the
same names as the C entry points in include/cs.h.

    import torch, paper_1509_03979_amd as cs
    op = cs.Operator(n, rows_dev_int32, signs_dev_int8)
    s, support, info = cs.cs_recover_sp(y_dev, op, k, tol)

The library must be built (``python paper_1509_03979_amd/build.py``); importing
this package without it raises, there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcsrecover.so")

CS_F32, CS_F64 = 0, 1
CS_ALGO_OMP, CS_ALGO_SP, CS_ALGO_OMPR, CS_ALGO_OPERATOR, CS_ALGO_LS, CS_ALGO_COSAMP = 0, 1, 2, 3, 4, 5
CS_OK, CS_E_INVALID, CS_E_SHAPE, CS_E_OP, CS_E_WORKSPACE, CS_E_HIP = 0, -1, -2, -3, -4, -5
CS_F_CG_MAXITER, CS_F_CG_BREAKDOWN, CS_F_OUTER_MAXITER, CS_F_NONFINITE, CS_F_NEAR_TIE = 1, 2, 4, 8, 16

CS_STATIC_WS_BYTES = 64 << 20

EXPORTS = ("cs_workspace_size", "cs_workspace_size_op", "cs_recover_omp", "cs_recover_sp", "cs_recover_ompr", "cs_recover_cosamp",
           "cs_recover_sp_static",
           "cs_ls_solve",
           "cs_adjoint_ls", "cs_workspace_size_batched", "cs_recover_ompr_batched", "cs_recover_sp_batched",
           "cs_apply_A", "cs_apply_At",
           "cs_shape_candidates", "cs_set_shape", "cs_time_shape", "cs_status_str", "cs_last_error",
           "cs_prof_enable", "cs_prof_reset", "cs_prof_read")


class cs_op(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("m", ctypes.c_int64), ("rows", ctypes.c_void_p),
                ("signs", ctypes.c_void_p), ("perm", ctypes.c_void_p), ("psi", ctypes.c_int32),
                ("xform", ctypes.c_int32)]


class cs_params(ctypes.Structure):
    _fields_ = [("cg_max_iter", ctypes.c_int32), ("max_outer", ctypes.c_int32),
                ("warm_start", ctypes.c_int32), ("cg_block", ctypes.c_int32), ("ompr_eta", ctypes.c_double),
                ("tol_abs", ctypes.c_int32), ("ompr_l", ctypes.c_int32)]


class cs_info(ctypes.Structure):
    _fields_ = [("outer_iters", ctypes.c_int32), ("flags", ctypes.c_int32), ("cg_iters", ctypes.c_int64),
                ("transforms", ctypes.c_int64), ("resid_norm", ctypes.c_double),
                ("model_bytes", ctypes.c_double), ("min_margin", ctypes.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class cs_batch_item(ctypes.Structure):
    _fields_ = [("op", cs_op), ("y", ctypes.c_void_p), ("s", ctypes.c_void_p), ("support", ctypes.c_void_p),
                ("k", ctypes.c_int32), ("moves_cap", ctypes.c_int32), ("moves", ctypes.c_void_p)]


class cs_shape(ctypes.Structure):
    _fields_ = [("log_l1", ctypes.c_int32), ("log_l2", ctypes.c_int32), ("log_b", ctypes.c_int32),
                ("log_e", ctypes.c_int32)]

    def as_tuple(self):
        return (self.log_l1, self.log_l2, self.log_b, self.log_e)


class cs_prof_stat(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 32), ("launches", ctypes.c_int64), ("total_ms", ctypes.c_double),
                ("bytes", ctypes.c_double)]


class CSError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{msg} (status {status})")
        self.status = status


def _load():
    # torch ships its own HIP runtime (SONAME libamdhip64.so.7); load it first so
    # the library binds to that same runtime instead of a second copy.
    import torch  # noqa: F401
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python paper_1509_03979_amd/build.py`")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, dbl, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_size_t
    P = ctypes.POINTER
    lib.cs_workspace_size.argtypes = [ctypes.c_int, i64, i64, i32, ctypes.c_int]
    lib.cs_workspace_size.restype = sz
    lib.cs_workspace_size_op.argtypes = [ctypes.c_int, P(cs_op), i32, ctypes.c_int]
    lib.cs_workspace_size_op.restype = sz
    for name in ("cs_recover_omp", "cs_recover_sp", "cs_recover_ompr", "cs_recover_cosamp"):
        f = getattr(lib, name)
        f.argtypes = [ctypes.c_int, vp, P(cs_op), i32, dbl, vp, vp, P(cs_params), vp, sz, P(cs_info), vp]
        f.restype = ctypes.c_int
    lib.cs_recover_sp_static.argtypes = [ctypes.c_int, vp, P(cs_op), i32, dbl, vp, vp, P(cs_params), P(cs_info), vp]
    lib.cs_recover_sp_static.restype = ctypes.c_int
    lib.cs_ls_solve.argtypes = [ctypes.c_int, vp, P(cs_op), vp, i32, dbl, vp, vp, P(cs_params), vp, sz,
                                P(cs_info), vp]
    lib.cs_ls_solve.restype = ctypes.c_int
    lib.cs_adjoint_ls.argtypes = [ctypes.c_int, P(cs_op), vp, i32, vp, dbl, vp, P(cs_params), vp, sz, P(cs_info), vp]
    lib.cs_adjoint_ls.restype = ctypes.c_int
    lib.cs_workspace_size_batched.argtypes = [ctypes.c_int, i32, P(cs_batch_item), ctypes.c_int]
    lib.cs_workspace_size_batched.restype = sz
    lib.cs_recover_ompr_batched.argtypes = [ctypes.c_int, i32, P(cs_batch_item), dbl, P(cs_params), vp, sz,
                                            P(cs_info), vp]
    lib.cs_recover_ompr_batched.restype = ctypes.c_int
    lib.cs_recover_sp_batched.argtypes = [ctypes.c_int, i32, P(cs_batch_item), dbl, P(cs_params), vp, sz,
                                          P(cs_info), vp]
    lib.cs_recover_sp_batched.restype = ctypes.c_int
    for name in ("cs_apply_A", "cs_apply_At"):
        f = getattr(lib, name)
        f.argtypes = [ctypes.c_int, P(cs_op), vp, vp, vp, sz, vp]
        f.restype = ctypes.c_int
    lib.cs_shape_candidates.argtypes = [ctypes.c_int, i64, P(cs_shape), i32]
    lib.cs_shape_candidates.restype = ctypes.c_int
    lib.cs_set_shape.argtypes = [ctypes.c_int, i64, P(cs_shape)]
    lib.cs_set_shape.restype = ctypes.c_int
    lib.cs_time_shape.argtypes = [ctypes.c_int, P(cs_op), P(cs_shape), i32, vp, sz, vp, P(dbl)]
    lib.cs_time_shape.restype = ctypes.c_int
    lib.cs_status_str.argtypes = [ctypes.c_int]
    lib.cs_status_str.restype = ctypes.c_char_p
    lib.cs_last_error.argtypes = []
    lib.cs_last_error.restype = ctypes.c_char_p
    lib.cs_prof_enable.argtypes = [ctypes.c_int]
    lib.cs_prof_enable.restype = ctypes.c_int
    lib.cs_prof_reset.argtypes = []
    lib.cs_prof_reset.restype = None
    lib.cs_prof_read.argtypes = [ctypes.POINTER(cs_prof_stat), ctypes.c_int]
    lib.cs_prof_read.restype = ctypes.c_int
    return lib


lib = _load()


def cs_status_str(status: int) -> str:
    return lib.cs_status_str(status).decode()


def cs_last_error() -> str:
    return lib.cs_last_error().decode()


def cs_prof_enable(on: bool) -> bool:
    return bool(lib.cs_prof_enable(1 if on else 0))


def cs_prof_reset() -> None:
    lib.cs_prof_reset()


def cs_prof_read() -> dict:
    """Per-class launches, total milliseconds and algorithmic bytes of the transform passes."""
    n = lib.cs_prof_read(None, 0)
    arr = (cs_prof_stat * n)()
    n = lib.cs_prof_read(arr, n)
    return {arr[i].name.decode(): {"launches": arr[i].launches, "total_ms": arr[i].total_ms,
                                   "bytes": arr[i].bytes} for i in range(n)}


def cs_workspace_size(dtype: int, n: int, m: int, k: int, algo: int) -> int:
    return int(lib.cs_workspace_size(dtype, n, m, k, algo))


def cs_workspace_size_op(dtype: int, op, k: int, algo: int) -> int:
    """Workspace bytes for an operator descriptor (`Operator` or `cs_op`); a
    DCT sparsifying basis needs two (psi = 1) or four (psi = 2) more N-vectors."""
    c = op.c if hasattr(op, "c") else op
    return int(lib.cs_workspace_size_op(dtype, ctypes.byref(c), k, algo))


def _check(status: int):
    if status != CS_OK:
        raise CSError(status, f"{cs_status_str(status)}: {cs_last_error()}")


# ---------------------------------------------------------------- torch-facing helpers
def _torch():
    import torch
    return torch


def _dtype_code(t) -> int:
    torch = _torch()
    if t.dtype in (torch.float32, torch.complex64):
        return CS_F32
    if t.dtype in (torch.float64, torch.complex128):
        return CS_F64
    raise TypeError("y must be float32 or float64 (complex64 or complex128 for partial complex Fourier sensing)")


def _meas(y, op, what="y"):
    """(dtype code, contiguous tensor whose memory the library reads, real dtype)
    for a measurement-side vector: M reals, or with partial complex Fourier
    sensing (xform = 2) M complex values, passed as (re, im) pairs."""
    torch = _torch()
    y = y.contiguous()
    cplx = getattr(op, "xform", 0) == 2
    if cplx != y.is_complex():
        raise TypeError(f"{what} must be complex exactly when the operator is partial complex Fourier (xform = 2)")
    if y.numel() != op.m or not y.is_cuda:
        raise ValueError(f"{what} must be a device vector of length M")
    real_dtype = y.real.dtype if cplx else y.dtype
    return _dtype_code(y), y, real_dtype


def _meas_empty(op, dtype, device):
    """An output on the measurement side (M reals or M complex values)."""
    torch = _torch()
    if getattr(op, "xform", 0) == 2:
        return torch.empty(op.m, dtype=torch.complex64 if dtype == torch.float32 else torch.complex128, device=device)
    return torch.empty(op.m, dtype=dtype, device=device)


def _stream_ptr(stream):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


class Operator:
    """Sensing operator A = D F R Psi (device descriptor): rows int32 [M]
    ascending, signs int8 [N], optionally perm int32 [N] (the randomizer's
    permutation; None: R is the sign flip alone), and the sparsifying basis
    psi (0: identity, s sparse directly; 1: the orthonormal DCT-II, as in the
    paper's experiments; 2: the separable 2-D DCT on an n x n image, N = n^2,
    s the row-major image of coefficients), and the transform F (xform 0: the
    orthonormal DCT-II; 1: the orthonormal real Fourier basis, partial
    Fourier sensing, where rows k and N-k hold the real and imaginary parts
    of Fourier coefficient k; 2: partial complex Fourier sensing of a real
    signal, rows = the M sampled frequencies in [1, N/2), y complex)."""

    def __init__(self, n: int, rows, signs, perm=None, psi: int = 0, xform: int = 0):
        torch = _torch()
        if rows.dtype != torch.int32 or signs.dtype != torch.int8:
            raise TypeError("rows must be int32 and signs int8")
        if not (rows.is_cuda and signs.is_cuda):
            raise ValueError("rows and signs must be device tensors")
        if perm is not None and (perm.dtype != torch.int32 or not perm.is_cuda or perm.numel() != n):
            raise ValueError("perm must be an int32 device tensor of length N")
        self.n = int(n)
        self.m = int(rows.numel())
        self.rows = rows.contiguous()
        self.signs = signs.contiguous()
        self.perm = perm.contiguous() if perm is not None else None
        self.psi = int(psi)
        self.xform = int(xform)
        self.c = cs_op(self.n, self.m, self.rows.data_ptr(), self.signs.data_ptr(),
                       self.perm.data_ptr() if self.perm is not None else None, self.psi, self.xform)

    @classmethod
    def from_numpy(cls, n, rows, signs, perm=None, device="cuda", psi: int = 0, xform: int = 0):
        torch = _torch()
        return cls(n, torch.as_tensor(rows, dtype=torch.int32, device=device),
                   torch.as_tensor(signs, dtype=torch.int8, device=device),
                   torch.as_tensor(perm, dtype=torch.int32, device=device) if perm is not None else None,
                   psi=psi, xform=xform)


def _params(cg_max_iter=0, max_outer=0, warm_start=1, ompr_eta=0.0, cg_block=0, tol_abs=False, ompr_l=1):
    return cs_params(int(cg_max_iter), int(max_outer), int(warm_start), int(cg_block), float(ompr_eta),
                     int(bool(tol_abs)), int(ompr_l))


def workspace(dtype_code: int, op: Operator, k: int, algo: int, device=None):
    torch = _torch()
    nbytes = cs_workspace_size_op(dtype_code, op, k, algo)
    if nbytes == 0:
        raise CSError(CS_E_SHAPE, "no workspace size for these arguments")
    dev = device if device is not None else op.rows.device
    # 256-byte alignment: the caching allocator returns 512-byte aligned blocks
    return torch.empty(nbytes, dtype=torch.uint8, device=dev)


def _recover(fn, algo, y, op: Operator, k: int, tol: float, ws=None, stream=None, **kw):
    torch = _torch()
    dt, y, rdt = _meas(y, op)
    s = torch.empty(op.n, dtype=rdt, device=y.device)
    supp = torch.empty(k, dtype=torch.int32, device=y.device)
    if ws is None:
        ws = workspace(dt, op, k, algo, y.device)
    info = cs_info()
    prm = _params(**kw)
    st = fn(dt, _ptr(y), ctypes.byref(op.c), int(k), float(tol), _ptr(s), _ptr(supp), ctypes.byref(prm),
            _ptr(ws), ws.numel(), ctypes.byref(info), _stream_ptr(stream))
    _check(st)
    return s, supp, info.as_dict()


def cs_recover_omp(y, op: Operator, k: int, tol: float, ws=None, stream=None, **kw):
    """OMP (Sec. II, Algorithm 1) -> (s [N], support [K] ascending, info)."""
    return _recover(lib.cs_recover_omp, CS_ALGO_OMP, y, op, k, tol, ws, stream, **kw)


def cs_recover_sp(y, op: Operator, k: int, tol: float, ws=None, stream=None, **kw):
    """Subspace Pursuit with CG least squares -> (s, support, info)."""
    return _recover(lib.cs_recover_sp, CS_ALGO_SP, y, op, k, tol, ws, stream, **kw)


def cs_recover_sp_static(y, op: Operator, k: int, tol: float, s=None, support=None, stream=None, **kw):
    """Subspace Pursuit on the library's static device workspace (no workspace
    argument; the call allocates nothing) -> (s, support, info).  Pass `s` [N]
    and `support` [K] to reuse output tensors; sizes beyond CS_STATIC_WS_BYTES
    of workspace raise with status CS_E_WORKSPACE."""
    torch = _torch()
    dt, y, rdt = _meas(y, op)
    if s is None:
        s = torch.empty(op.n, dtype=rdt, device=y.device)
    if support is None:
        support = torch.empty(k, dtype=torch.int32, device=y.device)
    if s.numel() != op.n or s.dtype != rdt or support.numel() != k or support.dtype != torch.int32:
        raise ValueError("s must be [N] in y's (real) dtype and support [K] int32")
    info = cs_info()
    prm = _params(**kw)
    st = lib.cs_recover_sp_static(dt, _ptr(y), ctypes.byref(op.c), int(k), float(tol), _ptr(s), _ptr(support),
                                  ctypes.byref(prm), ctypes.byref(info), _stream_ptr(stream))
    _check(st)
    return s, support, info.as_dict()


def cs_recover_ompr(y, op: Operator, k: int, tol: float, ws=None, stream=None, **kw):
    """OMPR (l = 1) with CG least squares -> (s, support, info)."""
    return _recover(lib.cs_recover_ompr, CS_ALGO_OMPR, y, op, k, tol, ws, stream, **kw)


def cs_recover_cosamp(y, op: Operator, k: int, tol: float, ws=None, stream=None, **kw):
    """CoSaMP with CG least squares -> (s, support, info)."""
    return _recover(lib.cs_recover_cosamp, CS_ALGO_COSAMP, y, op, k, tol, ws, stream, **kw)


def cs_ls_solve(y, op: Operator, support, tol: float, x0=None, ws=None, stream=None, **kw):
    """CG weighted least squares on `support` (the CG function of Algorithm 1) -> (theta [k], info)."""
    torch = _torch()
    dt, y, rdt = _meas(y, op)
    k = int(support.numel())
    theta = torch.empty(k, dtype=rdt, device=y.device)
    if ws is None:
        ws = workspace(dt, op, k, CS_ALGO_LS, y.device)
    info = cs_info()
    prm = _params(**kw)
    st = lib.cs_ls_solve(dt, _ptr(y), ctypes.byref(op.c), _ptr(support.contiguous()), k, float(tol),
                         _ptr(x0.contiguous()) if x0 is not None else None, _ptr(theta), ctypes.byref(prm),
                         _ptr(ws), ws.numel(), ctypes.byref(info), _stream_ptr(stream))
    _check(st)
    return theta, info.as_dict()


def cs_adjoint_ls(grad_s, op: Operator, support, tol: float, ws=None, stream=None, **kw):
    """dL/dy [M] from dL/ds [N] on the frozen support: A_S (A_S^T A_S)^-1 (dL/ds)_S -> (grad_y, info).
    With partial complex Fourier sensing grad_y is complex: dL/dRe y + i dL/dIm y."""
    torch = _torch()
    dt = _dtype_code(grad_s)
    k = int(support.numel())
    grad_s = grad_s.contiguous()
    if grad_s.numel() != op.n or not grad_s.is_cuda:
        raise ValueError("grad_s must be a device vector of length N")
    grad_y = _meas_empty(op, grad_s.dtype, grad_s.device)
    if ws is None:
        ws = workspace(dt, op, k, CS_ALGO_LS, grad_s.device)
    info = cs_info()
    prm = _params(**kw)
    st = lib.cs_adjoint_ls(dt, ctypes.byref(op.c), _ptr(support.contiguous()), k, _ptr(grad_s), float(tol),
                           _ptr(grad_y), ctypes.byref(prm), _ptr(ws), ws.numel(), ctypes.byref(info),
                           _stream_ptr(stream))
    _check(st)
    return grad_y, info.as_dict()


def _flag_check(info: dict, what: str):
    """Errors for results that cannot be trusted, warnings for capped iterations."""
    f = info["flags"]
    if f & (CS_F_NONFINITE | CS_F_CG_BREAKDOWN):
        raise CSError(CS_E_HIP if f & CS_F_NONFINITE else CS_E_INVALID,
                      f"{what}: " + ("a non-finite value" if f & CS_F_NONFINITE else
                                     "CG breakdown (d^T H d <= 0: the support's columns are dependent)"))
    if f & (CS_F_CG_MAXITER | CS_F_OUTER_MAXITER):
        import warnings
        warnings.warn(f"{what}: an iteration cap was reached (flags {f})", RuntimeWarning, stacklevel=3)


def _recover_fn(name: str):
    import torch

    fwd = {"omp": cs_recover_omp, "sp": cs_recover_sp, "ompr": cs_recover_ompr}[name]

    class _Recover(torch.autograd.Function):
        """s = recover(y); the backward is cs_adjoint_ls on the frozen final support.
        The forward's and the backward's cs_info are kept on the function's
        context (``info_fwd``, ``info_bwd``); a non-finite value or a CG
        breakdown (Theorem 3's condition failing) raises, an iteration cap
        warns."""

        @staticmethod
        def forward(ctx, y, op, k, tol, adj_tol=None):
            s, supp, info = fwd(y, op, k, tol)
            _flag_check(info, name + " forward")
            ctx.info_fwd = info
            ctx.save_for_backward(supp)
            ctx.op = op
            ctx.tol = tol if adj_tol is None else adj_tol
            ctx.mark_non_differentiable(supp)
            return s, supp

        @staticmethod
        def backward(ctx, grad_s, grad_supp):
            (supp,) = ctx.saved_tensors
            grad_y, info = cs_adjoint_ls(grad_s, ctx.op, supp, ctx.tol)
            _flag_check(info, name + " backward")
            ctx.info_bwd = info
            return grad_y, None, None, None, None

    _Recover.__name__ = name.upper() + "Recover"
    return _Recover


class _LazyFn:
    def __init__(self, name):
        self.name = name
        self.fn = None

    def apply(self, y, op, k, tol, adj_tol=None):
        """-> (s [N], support [K]); s is differentiable with respect to y."""
        if self.fn is None:
            self.fn = _recover_fn(self.name)
        return self.fn.apply(y, op, k, tol, adj_tol)


OMPRecover, SPRecover, OMPRRecover = _LazyFn("omp"), _LazyFn("sp"), _LazyFn("ompr")


class Batch:
    """Outputs, descriptors and workspace of one batched call, reusable across
    calls with the same signals (the measurements may change in place)."""

    def __init__(self, ys, ops, ks, device=None, moves_cap: int = 0, algo: int = CS_ALGO_OMPR):
        """algo: CS_ALGO_OMPR (cs_recover_ompr_batched) or CS_ALGO_SP
        (cs_recover_sp_batched); it sizes the workspace.  moves_cap > 0
        records each OMPR signal's first moves_cap swaps in self.moves[i]
        (int32 [moves_cap, 2]: entered, left; rows past the signal's swap
        count are left at -1)."""
        torch = _torch()
        if not (len(ys) == len(ops) == len(ks)) or len(ys) == 0:
            raise ValueError("ys, ops and ks must be non-empty and of equal length")
        self.ys = [y.contiguous() for y in ys]
        self.dtype = self.ys[0].dtype
        self.dt = _dtype_code(self.ys[0])
        for y, op in zip(self.ys, ops):
            if y.dtype != self.dtype or y.numel() != op.m or not y.is_cuda:
                raise ValueError("every y must be a device vector of length M in one dtype")
        dev = self.ys[0].device
        self.ops = list(ops)
        self.ks = [int(k) for k in ks]
        self.s = [torch.empty(op.n, dtype=self.dtype, device=dev) for op in self.ops]
        self.supp = [torch.empty(k, dtype=torch.int32, device=dev) for k in self.ks]
        self.moves = [torch.full((int(moves_cap), 2), -1, dtype=torch.int32, device=dev) for _ in self.ks] \
            if moves_cap > 0 else None
        n = len(self.ys)
        self.items = (cs_batch_item * n)()
        for i in range(n):
            it = self.items[i]
            it.op = self.ops[i].c
            it.y = _ptr(self.ys[i])
            it.s = _ptr(self.s[i])
            it.support = _ptr(self.supp[i])
            it.k = self.ks[i]
            if self.moves is not None:
                it.moves_cap = int(moves_cap)
                it.moves = _ptr(self.moves[i])
        self.algo = algo
        nbytes = lib.cs_workspace_size_batched(self.dt, n, self.items, algo)
        if nbytes == 0:
            raise CSError(CS_E_SHAPE, "no batched workspace size for these signals")
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)


def cs_recover_ompr_batched(batch: "Batch", tol: float, stream=None, **kw):
    """OMPR (l = 1) on every signal of `batch` in one batched call -> (s list, support list, info list)."""
    n = len(batch.ys)
    infos = (cs_info * n)()
    prm = _params(**kw)
    st = lib.cs_recover_ompr_batched(batch.dt, n, batch.items, float(tol), ctypes.byref(prm), _ptr(batch.ws),
                                     batch.ws.numel(), infos, _stream_ptr(stream))
    _check(st)
    return batch.s, batch.supp, [infos[i].as_dict() for i in range(n)]


def cs_recover_sp_batched(batch: "Batch", tol: float, stream=None, **kw):
    """SP on every signal of `batch` (built with algo=CS_ALGO_SP) in one call,
    the signals run concurrently -> (s list, support list, info list)."""
    if batch.algo != CS_ALGO_SP:
        raise ValueError("the batch's workspace was sized for another algorithm (use algo=CS_ALGO_SP)")
    n = len(batch.ys)
    infos = (cs_info * n)()
    prm = _params(**kw)
    st = lib.cs_recover_sp_batched(batch.dt, n, batch.items, float(tol), ctypes.byref(prm), _ptr(batch.ws),
                                   batch.ws.numel(), infos, _stream_ptr(stream))
    _check(st)
    return batch.s, batch.supp, [infos[i].as_dict() for i in range(n)]


class SPRecoverBatched:
    """s_b = SP(y_b) for a list of signals through one cs_recover_sp_batched
    call; differentiable with respect to every y_b (the backward is
    cs_adjoint_ls on each frozen final support).  Reuses the Batch's output
    tensors, so the returned s are views the next call overwrites unless the
    caller clones them."""

    @staticmethod
    def apply(ys, ops, k, tol, batch: "Batch" = None, adj_tol=None):
        import torch

        class _Fn(torch.autograd.Function):
            @staticmethod
            def forward(ctx, *yv):
                b = batch if batch is not None else Batch(list(yv), ops, [k] * len(yv), algo=CS_ALGO_SP)
                for i, y in enumerate(yv):
                    if b.ys[i].data_ptr() != y.data_ptr():
                        b.ys[i].copy_(y)
                s, supp, infos = cs_recover_sp_batched(b, tol)
                for info in infos:
                    _flag_check(info, "SP batched forward")
                ctx.supps = [p.clone() for p in supp]
                ctx.mark_non_differentiable(*ctx.supps)
                return tuple(x.clone() for x in s) + tuple(ctx.supps)

            @staticmethod
            def backward(ctx, *grads):
                n = len(ctx.supps)
                out = []
                for i in range(n):
                    g = grads[i]
                    if g is None:
                        out.append(None)
                        continue
                    gy, info = cs_adjoint_ls(g, ops[i], ctx.supps[i], tol if adj_tol is None else adj_tol)
                    _flag_check(info, "SP batched backward")
                    out.append(gy)
                return tuple(out)

        res = _Fn.apply(*ys)
        n = len(ys)
        return list(res[:n]), list(res[n:])


def cs_shape_candidates(dtype_code: int, n: int) -> list:
    """Compiled four-step shapes (log_l1, log_l2, log_b, log_e) for N, the default first."""
    cnt = lib.cs_shape_candidates(dtype_code, n, None, 0)
    arr = (cs_shape * max(cnt, 1))()
    cnt = lib.cs_shape_candidates(dtype_code, n, arr, cnt)
    return [arr[i].as_tuple() for i in range(cnt)]


def cs_set_shape(dtype_code: int, n: int, shape) -> None:
    """Install a candidate shape for every later call at this N (None: the default)."""
    _check(lib.cs_set_shape(dtype_code, n, ctypes.byref(cs_shape(*shape)) if shape is not None else None))


def cs_time_shape(dtype_code: int, op: Operator, shape, reps: int = 20, ws=None, stream=None) -> float:
    """Average ms of one H-apply (three transform passes) with `shape`."""
    if ws is None:
        ws = workspace(dtype_code, op, 1, CS_ALGO_OPERATOR)
    ms = ctypes.c_double(0.0)
    _check(lib.cs_time_shape(dtype_code, ctypes.byref(op.c), ctypes.byref(cs_shape(*shape)), int(reps), _ptr(ws),
                             ws.numel(), _stream_ptr(stream), ctypes.byref(ms)))
    return ms.value


def cs_apply_A(x, op: Operator, ws=None, stream=None):
    """A x for a dense x [N] -> [M] (complex with partial complex Fourier sensing)."""
    torch = _torch()
    dt = _dtype_code(x)
    out = _meas_empty(op, x.dtype, x.device)
    if ws is None:
        ws = workspace(dt, op, 1, CS_ALGO_OPERATOR, x.device)
    _check(lib.cs_apply_A(dt, ctypes.byref(op.c), _ptr(x.contiguous()), _ptr(out), _ptr(ws), ws.numel(),
                          _stream_ptr(stream)))
    return out


def cs_apply_At(u, op: Operator, ws=None, stream=None):
    """A^T u for u [M] -> [N] (with partial complex Fourier sensing u is
    complex and this is the real-inner-product adjoint R^T Re(F^H D^T u))."""
    torch = _torch()
    dt, u, rdt = _meas(u, op, "u")
    out = torch.empty(op.n, dtype=rdt, device=u.device)
    if ws is None:
        ws = workspace(dt, op, 1, CS_ALGO_OPERATOR, u.device)
    _check(lib.cs_apply_At(dt, ctypes.byref(op.c), _ptr(u), _ptr(out), _ptr(ws), ws.numel(),
                           _stream_ptr(stream)))
    return out
