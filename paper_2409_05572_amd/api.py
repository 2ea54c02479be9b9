"""Python binding of the C ABI: argument marshalling only.

Device memory comes from torch (ROCm build); the solver, every n-length
operation and every small dense step run in the HIP library. Nothing here
computes any part of the method.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass, field

import numpy as np

import atexit

from . import _lib
from ._lib import SeInfo, SeParams, check, lib

# Objects still alive when the interpreter exits are not destroyed through
# the library: at that point the HIP runtime, torch and an attached profiler
# finalize in an order this module does not control, and the process exit
# returns the device memory anyway. Explicit close() calls are unaffected.
_EXITING = False


def _mark_exiting():
    global _EXITING
    _EXITING = True


atexit.register(_mark_exiting)


def _ptr(x) -> int:
    """Raw address of a numpy array or a torch tensor."""
    if isinstance(x, np.ndarray):
        return x.ctypes.data
    return x.data_ptr()


class Context:
    """Library context bound to one device and one stream (torch stream or raw)."""

    def __init__(self, device: int = 0, stream=None):
        import torch

        self.device = device
        if stream is None:
            stream = torch.cuda.current_stream(device)
        self._stream = stream
        raw = stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream or 0)
        h = C.c_void_p()
        check(lib().se_ctx_create(device, C.c_void_p(raw), C.byref(h)), "se_ctx_create")
        self._h = h

    @property
    def handle(self):
        return self._h

    def close(self):
        if self._h:
            lib().se_ctx_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        if _EXITING:
            return
        try:
            self.close()
        except Exception:
            pass


class Matrix:
    """Symmetric (or, with complex values, Hermitian) CSR matrix copied to the
    device (se_matrix_create_csr / se_matrix_create_csr_z)."""

    def __init__(self, ctx: Context, n, rowptr, colind, val, anorm, on_device=False):
        self.ctx = ctx
        self.n = int(n)
        if on_device:
            import torch

            self.is_complex = val.dtype == torch.complex128
        else:
            self.is_complex = np.iscomplexobj(val)
            rowptr = np.ascontiguousarray(rowptr, dtype=np.int64)
            colind = np.ascontiguousarray(colind, dtype=np.int32)
            val = np.ascontiguousarray(val, dtype=np.complex128 if self.is_complex else np.float64)
        self._keep = (rowptr, colind, val)
        h = C.c_void_p()
        flags = _lib.SE_MATRIX_DEVICE if on_device else _lib.SE_MATRIX_HOST
        nnz = int(rowptr[-1]) if not on_device else int(colind.numel())
        create = lib().se_matrix_create_csr_z if self.is_complex else lib().se_matrix_create_csr
        st = create(ctx.handle, self.n, nnz, C.c_void_p(_ptr(rowptr)), C.c_void_p(_ptr(colind)),
                    C.c_void_p(_ptr(val)), flags, float(anorm), C.byref(h))
        if st == _lib.SE_ERR_HIP:
            e = lib().se_ctx_last_hip_error(ctx.handle)
            check(st, f"se_matrix_create_csr ({lib().se_hip_error_name(e).decode()})")
        check(st, "se_matrix_create_csr")
        self._h = h
        self._keep = None
        self.anorm = float(lib().se_matrix_anorm(h))  # the given bound, or the Gershgorin estimate for 0

    @classmethod
    def from_csr(cls, ctx: Context, csr) -> "Matrix":
        """From any object with n, rowptr, colind, val and anorm attributes."""
        return cls(ctx, csr.n, csr.rowptr, csr.colind, csr.val, csr.anorm)

    @property
    def handle(self):
        return self._h

    def close(self):
        if self._h:
            lib().se_matrix_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        if _EXITING:
            return
        try:
            self.close()
        except Exception:
            pass


@dataclass
class SolveInfo:
    status: int
    iterations: int
    converged: bool
    n_shrinks: int
    n_expands: int
    max_stop_ratio: float
    max_paper_ratio: float
    time_ms: float
    workspace_bytes: int
    history: np.ndarray = field(default_factory=lambda: np.zeros((0, 8)))
    kern_ms: tuple = ()
    kern_bytes: tuple = ()
    kern_flops: tuple = ()
    kern_calls: tuple = ()
    lp_iterations: int = 0
    n_reprojections: int = 0


PRECISIONS = {"fp64": _lib.SE_FP64, "fp32": _lib.SE_FP32_MIXED, "bf16": _lib.SE_BF16_MIXED}


def params(n_ev, n_extra, solver="lobpcg", strategy="none", tol=1e-8, n_es=0, max_iter=None,
           soft_lock=True, sigma=0.0, time_limit_s=0.0, precision="fp64", r_switch=0.0,
           implicit_pivot=0.0, expand_vectors="xdrop", filter_degree=0, precond="none",
           **strategy_params) -> SeParams:
    p = SeParams()
    lib().se_params_default(C.byref(p))
    p.solver = _lib.SOLVERS[solver]
    p.expand_vectors = _lib.EXPAND_VECTORS[expand_vectors]
    p.filter_degree = int(filter_degree)
    p.precond = _lib.PRECONDS[precond]
    p.precision = PRECISIONS[precision]
    p.r_switch = float(r_switch)
    p.implicit_pivot = float(implicit_pivot)
    p.strategy = _lib.STRATEGIES[strategy]
    p.n_ev, p.n_extra, p.n_es = int(n_ev), int(n_extra), int(n_es)
    p.tol = float(tol)
    p.soft_lock = 1 if soft_lock else 0
    p.sigma = float(sigma)
    p.time_limit_s = float(time_limit_s)
    p.max_iter = int(max_iter if max_iter is not None else (20000 if solver == "si" else 1000))
    for k, v in strategy_params.items():
        setattr(p, k, v)
    return p


def solve(ctx: Context, A: Matrix, X0, n_ev, n_extra, history_cap=0, **kw):
    """Run se_solve.

    X0 is either a host numpy array (n, nb) in Fortran order, a torch device
    tensor of shape (nb, n) (column-major n x nb), or None (the library
    generates the start block from `seed`, see workloads.seeded_uniform_block).
    Returns (lam, V, info) with V on the same side as X0 (host for None): numpy
    (n, n_ev) or a torch (n_ev, n) tensor whose transpose is the eigenvector
    block.
    """
    p = params(n_ev, n_extra, **kw)
    hist = np.zeros((max(history_cap, 0), _lib.SE_HISTORY_FIELDS), dtype=np.float64)
    if history_cap > 0:
        p.history = hist.ctypes.data_as(C.POINTER(C.c_double))
        p.history_cap = history_cap
    info = SeInfo()
    n = A.n
    if X0 is None:
        V = np.zeros((n, n_ev), dtype=np.float64, order="F")
        lam = np.zeros(n_ev, dtype=np.float64)
        p.ptr_mode = _lib.SE_PTR_HOST
    elif isinstance(X0, np.ndarray):
        X0 = np.asfortranarray(X0, dtype=np.float64)
        assert X0.shape == (n, n_ev + n_extra)
        V = np.zeros((n, n_ev), dtype=np.float64, order="F")
        lam = np.zeros(n_ev, dtype=np.float64)
        p.ptr_mode = _lib.SE_PTR_HOST
    else:
        import torch

        assert X0.dtype == torch.float64 and X0.is_contiguous() and X0.shape == (n_ev + n_extra, n)
        V = torch.empty((n_ev, n), dtype=torch.float64, device=X0.device)
        lam = torch.empty(n_ev, dtype=torch.float64, device=X0.device)
        p.ptr_mode = _lib.SE_PTR_DEVICE
    st = lib().se_solve(ctx.handle, A.handle, C.byref(p), C.c_void_p(None if X0 is None else _ptr(X0)),
                        C.c_void_p(_ptr(V)), C.c_void_p(_ptr(lam)), C.byref(info))
    if st < 0:
        err = _lib.SeError(st, f"se_solve (hip_error {info.hip_error}, {info.iterations} iterations)")
        err.hip_error = info.hip_error
        err.history = hist[: info.history_len].copy()
        raise err
    out = SolveInfo(st, info.iterations, bool(info.converged), info.n_shrinks, info.n_expands,
                    info.max_stop_ratio, info.max_paper_ratio, info.time_ms,
                    int(info.workspace_bytes), hist[: info.history_len].copy(),
                    tuple(info.kern_ms), tuple(info.kern_bytes), tuple(info.kern_flops),
                    tuple(info.kern_calls), info.lp_iterations, info.n_reprojections)
    return lam, V, out


def solve_z(ctx: Context, A: Matrix, X0, n_ev, n_extra, history_cap=0, **kw):
    """Run se_solve_z on a complex Hermitian matrix.

    X0: a host numpy complex array (n, nb) (Fortran order is taken), a torch
    complex128 device tensor of shape (nb, n) (column-major n x nb), or None
    (the real seeded block). Returns (lam, V, info) as solve(), V complex.
    """
    assert A.is_complex, "solve_z needs a matrix with complex values"
    p = params(n_ev, n_extra, **kw)
    hist = np.zeros((max(history_cap, 0), _lib.SE_HISTORY_FIELDS), dtype=np.float64)
    if history_cap > 0:
        p.history = hist.ctypes.data_as(C.POINTER(C.c_double))
        p.history_cap = history_cap
    info = SeInfo()
    n = A.n
    if X0 is None or isinstance(X0, np.ndarray):
        if X0 is not None:
            X0 = np.asfortranarray(X0, dtype=np.complex128)
            assert X0.shape == (n, n_ev + n_extra)
        V = np.zeros((n, n_ev), dtype=np.complex128, order="F")
        lam = np.zeros(n_ev, dtype=np.float64)
        p.ptr_mode = _lib.SE_PTR_HOST
    else:
        import torch

        assert X0.dtype == torch.complex128 and X0.is_contiguous() and X0.shape == (n_ev + n_extra, n)
        V = torch.empty((n_ev, n), dtype=torch.complex128, device=X0.device)
        lam = torch.empty(n_ev, dtype=torch.float64, device=X0.device)
        p.ptr_mode = _lib.SE_PTR_DEVICE
    st = lib().se_solve_z(ctx.handle, A.handle, C.byref(p), C.c_void_p(None if X0 is None else _ptr(X0)),
                          C.c_void_p(_ptr(V)), C.c_void_p(_ptr(lam)), C.byref(info))
    if st < 0:
        err = _lib.SeError(st, f"se_solve_z (hip_error {info.hip_error}, {info.iterations} iterations)")
        err.hip_error = info.hip_error
        err.history = hist[: info.history_len].copy()
        raise err
    return lam, V, _info_of(st, info, hist)


def footprint(n, nnz, n_ev, n_extra, precision="fp64", solver="lobpcg") -> int:
    """Device bytes a solve of this shape allocates (the serving admission size)."""
    return int(lib().se_solve_footprint(int(n), int(nnz), int(n_ev), int(n_extra), PRECISIONS[precision],
                                        _lib.SOLVERS[solver]))


def _info_of(st, info, hist):
    return SolveInfo(st, info.iterations, bool(info.converged), info.n_shrinks, info.n_expands,
                     info.max_stop_ratio, info.max_paper_ratio, info.time_ms,
                     int(info.workspace_bytes), hist[: info.history_len].copy(),
                     tuple(info.kern_ms), tuple(info.kern_bytes), tuple(info.kern_flops),
                     tuple(info.kern_calls), info.lp_iterations, info.n_reprojections)


class Server:
    """Continuous-batching solver service on one GPU (se_server_*).

    submit() queues a solve on device tensors and returns a ticket at once;
    wait() blocks for its result. The caller keeps the matrix, X0 and the
    output tensors alive until wait() returns.
    """

    def __init__(self, ctx: Context, hbm_budget_bytes: int, max_slots: int = 4, batched: bool = False):
        """batched: one engine advances all resident solves in lockstep
        (se_server_create_batched); else one worker and stream per slot."""
        self._h = C.c_void_p()
        fn = "se_server_create_batched" if batched else "se_server_create"
        check(getattr(lib(), fn)(ctx.handle, int(hbm_budget_bytes), int(max_slots), C.byref(self._h)), fn)
        self.batched = batched
        self._keep = {}

    def submit(self, A: Matrix, X0, n_ev, n_extra, **kw):
        """X0: torch (nb, n) float64 device tensor. Returns (ticket, lam, V)."""
        import torch

        n = A.n
        assert X0.dtype == torch.float64 and X0.is_contiguous() and X0.shape == (n_ev + n_extra, n)
        p = params(n_ev, n_extra, **kw)
        p.ptr_mode = _lib.SE_PTR_DEVICE
        V = torch.empty((n_ev, n), dtype=torch.float64, device=X0.device)
        lam = torch.empty(n_ev, dtype=torch.float64, device=X0.device)
        t = C.c_uint64()
        check(lib().se_submit(self._h, A.handle, C.byref(p), C.c_void_p(_ptr(X0)), C.c_void_p(_ptr(V)),
                              C.c_void_p(_ptr(lam)), C.byref(t)), "se_submit")
        self._keep[t.value] = (A, X0, V, lam)
        return t.value, lam, V

    def batch_stats(self):
        """(steps, graph_steps) of a batched server's engine."""
        a, b = C.c_int64(), C.c_int64()
        check(lib().se_server_batch_stats(self._h, C.byref(a), C.byref(b)), "se_server_batch_stats")
        return a.value, b.value

    def poll(self, ticket) -> bool:
        d = C.c_int32()
        check(lib().se_poll(self._h, C.c_uint64(ticket), C.byref(d)), "se_poll")
        return bool(d.value)

    def wait(self, ticket):
        """Returns (SolveInfo, queue_ms, run_ms); raises SeError on a failed solve."""
        info = SeInfo()
        q, r = C.c_double(), C.c_double()
        st = lib().se_wait(self._h, C.c_uint64(ticket), C.byref(info), C.byref(q), C.byref(r))
        self._keep.pop(ticket, None)
        if st < 0:
            raise _lib.SeError(st, "se_wait")
        return _info_of(st, info, np.zeros((0, _lib.SE_HISTORY_FIELDS))), q.value, r.value

    def close(self):
        if self._h:
            lib().se_server_destroy(self._h)
            self._h = C.c_void_p()
            self._keep.clear()

    def __del__(self):
        if _EXITING:
            return
        try:
            self.close()
        except Exception:
            pass


# ---- building blocks (device tensors, row-major blocks) ----

def spmm(ctx: Context, A: Matrix, X, Y, w: int):
    check(lib().se_op_spmm(ctx.handle, A.handle, C.c_void_p(_ptr(X)), X.stride(0),
                           C.c_void_p(_ptr(Y)), Y.stride(0), int(w)), "se_op_spmm")


def gram(ctx: Context, U, mu: int, V, mv: int, out):
    check(lib().se_op_gram(ctx.handle, U.shape[0], C.c_void_p(_ptr(U)), U.stride(0), int(mu),
                           C.c_void_p(_ptr(V)), V.stride(0), int(mv), C.c_void_p(_ptr(out))),
          "se_op_gram")


def gram_noalloc(ctx: Context, U, mu: int, V, mv: int, out):
    """C = U^T V through the entry point that allocates nothing (library-held scratch)."""
    check(lib().se_op_gram_noalloc(ctx.handle, U.shape[0], C.c_void_p(_ptr(U)), U.stride(0), int(mu),
                                   C.c_void_p(_ptr(V)), V.stride(0), int(mv), C.c_void_p(_ptr(out))),
          "se_op_gram_noalloc")


def update(ctx: Context, U, K: int, Cm, N: int, Out, beta: float = 0.0):
    check(lib().se_op_update(ctx.handle, U.shape[0], C.c_void_p(_ptr(U)), U.stride(0), int(K),
                             C.c_void_p(_ptr(Cm)), int(N), C.c_void_p(_ptr(Out)), Out.stride(0),
                             float(beta)), "se_op_update")


def _lp_code(t):
    import torch

    if t.dtype == torch.float32:
        return _lib.SE_FP32_MIXED
    if t.dtype == torch.bfloat16:
        return _lib.SE_BF16_MIXED
    raise TypeError(f"low-precision blocks are float32 or bfloat16, not {t.dtype}")


def spmm_lp(ctx: Context, A: Matrix, X, Y, w: int):
    """Y = A X on float32 or bfloat16 blocks (FP32 arithmetic)."""
    check(lib().se_op_spmm_lp(ctx.handle, _lp_code(X), A.handle, C.c_void_p(_ptr(X)), X.stride(0),
                              C.c_void_p(_ptr(Y)), Y.stride(0), int(w)), "se_op_spmm_lp")


def gram_lp(ctx: Context, U, mu: int, V, mv: int, out):
    """out (float64) = U^T V for float32 or bfloat16 blocks."""
    check(lib().se_op_gram_lp(ctx.handle, _lp_code(U), U.shape[0], C.c_void_p(_ptr(U)), U.stride(0),
                              int(mu), C.c_void_p(_ptr(V)), V.stride(0), int(mv), C.c_void_p(_ptr(out))),
          "se_op_gram_lp")


def update_lp(ctx: Context, U, K: int, Cm, N: int, Out, beta: float = 0.0):
    """Out = beta Out + U Cm on float32 or bfloat16 blocks (Cm float64)."""
    check(lib().se_op_update_lp(ctx.handle, _lp_code(U), U.shape[0], C.c_void_p(_ptr(U)), U.stride(0),
                                int(K), C.c_void_p(_ptr(Cm)), int(N), C.c_void_p(_ptr(Out)),
                                Out.stride(0), float(beta)), "se_op_update_lp")


def spmm_z(ctx: Context, A: Matrix, X, Y, w: int):
    """Y = A X on complex128 row-major device blocks."""
    check(lib().se_op_spmm_z(ctx.handle, A.handle, C.c_void_p(_ptr(X)), X.stride(0),
                             C.c_void_p(_ptr(Y)), Y.stride(0), int(w)), "se_op_spmm_z")


def gram_z(ctx: Context, U, mu: int, V, mv: int, out):
    """out (complex128, mu x mv) = U^H V."""
    check(lib().se_op_gram_z(ctx.handle, U.shape[0], C.c_void_p(_ptr(U)), U.stride(0), int(mu),
                             C.c_void_p(_ptr(V)), V.stride(0), int(mv), C.c_void_p(_ptr(out))),
          "se_op_gram_z")


def update_z(ctx: Context, U, K: int, Cm, N: int, Out, beta: float = 0.0):
    """Out = beta Out + U Cm on complex128 blocks."""
    check(lib().se_op_update_z(ctx.handle, U.shape[0], C.c_void_p(_ptr(U)), U.stride(0), int(K),
                               C.c_void_p(_ptr(Cm)), int(N), C.c_void_p(_ptr(Out)), Out.stride(0),
                               float(beta)), "se_op_update_z")


def heev_lowest_z(ctx: Context, A, k: int, w, Z):
    """The k lowest eigenpairs of the Hermitian complex128 m x m matrix A (overwritten)."""
    check(lib().se_op_heev_lowest_z(ctx.handle, A.shape[0], int(k), C.c_void_p(_ptr(A)),
                                    C.c_void_p(_ptr(w)), C.c_void_p(_ptr(Z))), "se_op_heev_lowest_z")


def syev(ctx: Context, A, w, Z):
    check(lib().se_op_syev(ctx.handle, A.shape[0], C.c_void_p(_ptr(A)), C.c_void_p(_ptr(w)),
                           C.c_void_p(_ptr(Z))), "se_op_syev")


def syev_lowest(ctx: Context, A, k: int, w, Z):
    """The k lowest eigenpairs of the m x m matrix A (overwritten); Z is m x k."""
    check(lib().se_op_syev_lowest(ctx.handle, A.shape[0], int(k), C.c_void_p(_ptr(A)),
                                  C.c_void_p(_ptr(w)), C.c_void_p(_ptr(Z))), "se_op_syev_lowest")


def cholqr(ctx: Context, W, w: int) -> int:
    r = C.c_int32()
    check(lib().se_op_cholqr(ctx.handle, W.shape[0], C.c_void_p(_ptr(W)), W.stride(0), int(w),
                             C.byref(r)), "se_op_cholqr")
    return r.value


def strategy_replay(strategy: str, rs, **kw) -> np.ndarray:
    """Replay the library's shrink/expand controller on scripted r(j) values (host only)."""
    p = params(1, 0, strategy=strategy, **kw)
    r = np.ascontiguousarray(rs, dtype=np.float64)
    flags = np.zeros(r.size, dtype=np.int32)
    check(lib().se_strategy_replay(C.byref(p), r.size, r.ctypes.data_as(C.POINTER(C.c_double)),
                                   flags.ctypes.data_as(C.POINTER(C.c_int32))), "se_strategy_replay")
    return flags
