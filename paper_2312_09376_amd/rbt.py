"""Thin PyTorch binding of the C ABI (include/rbt.h).

Argument marshalling only: every step of the method runs in librbt's HIP
kernels. Tensors are column-major (stride (1, ld)): build one from a
row-major tensor with `colmajor(t)`. Device work is enqueued on torch's
current HIP stream; the library's workspace is a torch allocation.
"""
import ctypes

import numpy as np
import torch

from . import _lib
from ._lib import (RBT_BF16, RBT_FP32, RBT_FP64, RBT_IR_CLASSIC, RBT_IR_GMRES, RBT_OP_N,  # noqa: F401
                   RBT_OP_T, check)


def _colmajor_ld(t):
    """Leading dimension of a column-major 2-D tensor, or None if it is not
    one. Strides of size-1 dimensions are ignored (torch leaves them free)."""
    if t.dim() != 2:
        return None
    rows, cols = t.shape
    if rows == 0 or cols == 0:
        return max(1, rows)  # an empty matrix: any leading dimension will do
    if rows > 1 and t.stride(0) != 1:
        return None
    ld = t.stride(1) if cols > 1 else max(1, rows)
    return ld if ld >= max(1, rows) else None


def colmajor(t):
    """Column-major view of t (itself when it already is one, else a copy)."""
    if t.dim() == 1:
        t = t.reshape(-1, 1)
    if _colmajor_ld(t) is not None:
        return t
    return t.t().contiguous().t()


def _ld(t):
    ld = _colmajor_ld(t)
    if ld is None:
        raise ValueError("expected a column-major 2-D tensor (stride (1, ld), ld >= rows)")
    return ld


def _dev_f64(t, name):
    if not (t.is_cuda and t.dtype == torch.float64):
        raise TypeError(f"{name} must be a float64 tensor on a HIP device")


def _stream(device=None):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _p(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def lib():
    return _lib.load()


# ------------------------------------------------------------------ host

def structure(n, depth):
    """(depth, n) int64 array: partner[l-1, i] or -1 (host call)."""
    out = np.zeros((depth, n), dtype=np.int64)
    check(lib().rbt_structure(n, depth, out.ctypes.data_as(ctypes.c_void_p)), "rbt_structure")
    return out


def generate(n, depth, seed):
    """Packed coefficients (n x depth, column-major) computed on the host."""
    U = np.zeros((depth, n), dtype=np.float64)
    V = np.zeros((depth, n), dtype=np.float64)
    check(lib().rbt_generate(n, depth, seed, U.ctypes.data_as(ctypes.c_void_p),
                             V.ctypes.data_as(ctypes.c_void_p)), "rbt_generate")
    return U.T, V.T


def workspace_size(n, nrhs, depth, precision=RBT_FP64):
    return int(lib().rbt_workspace_size(n, nrhs, depth, precision))


def _workspace(n, nrhs, depth, device, precision=RBT_FP64):
    nbytes = max(workspace_size(n, nrhs, depth, precision), 256)
    return torch.empty(nbytes, dtype=torch.uint8, device=device)


# ---------------------------------------------------------------- device

def generate_device(n, depth, seed, device="cuda"):
    U = torch.empty((depth, n), dtype=torch.float64, device=device)
    V = torch.empty((depth, n), dtype=torch.float64, device=device)
    check(lib().rbt_generate_device(n, depth, seed, _p(U), _p(V), _stream(U.device)),
          "rbt_generate_device")
    return U.t(), V.t()


def transform2(A, U, V, depth, out=None, out_dtype=torch.float64):
    """Out = U^T A V; in place when out is A."""
    _dev_f64(A, "A")
    n = A.shape[0]
    if out is None:
        out = torch.empty_strided((n, n), (1, max(1, n)), dtype=out_dtype, device=A.device)
    prec = RBT_FP64 if out.dtype == torch.float64 else RBT_FP32
    check(lib().rbt_transform2(n, _p(A), _ld(A), _p(out), _ld(out), prec, _p(U), _p(V), depth,
                               _stream(A.device)), "rbt_transform2")
    return out


def transform_vec(B, C, depth, op):
    """In place: B <- C^T B (op=RBT_OP_T) or B <- C B (op=RBT_OP_N)."""
    _dev_f64(B, "B")
    check(lib().rbt_transform_vec(B.shape[0], B.shape[1], _p(B), _ld(B), _p(C), depth, op,
                                  _stream(B.device)), "rbt_transform_vec")
    return B


def genp(A, info=None):
    """In-place elimination without pivoting. Returns (A, info)."""
    _dev_f64(A, "A")
    n = A.shape[0]
    info = info if info is not None else torch.zeros(1, dtype=torch.int32, device=A.device)
    check(lib().rbt_genp(n, _p(A), _ld(A), _p(info), _stream(A.device)), "rbt_genp")
    return A, info


def getrs(LU, B, trans=0, work=None):
    """B <- (LU)^-1 B (trans=0) or (LU)^-T B (trans=1), in place."""
    _dev_f64(B, "B")
    n = LU.shape[0]
    work = work if work is not None else _workspace(n, B.shape[1], 0, B.device)
    check(lib().rbt_getrs(n, B.shape[1], _p(LU), _ld(LU), _p(B), _ld(B), trans, _p(work),
                          work.numel(), _stream(B.device)), "rbt_getrs")
    return B


def solve_(A, B, depth=2, seed=2023, info=None, work=None):
    """In place: A <- L\\U of U^T A V, B <- X. Returns (A, B, info, work)."""
    _dev_f64(A, "A")
    _dev_f64(B, "B")
    n, k = A.shape[0], B.shape[1]
    work = work if work is not None else _workspace(n, k, depth, A.device)
    info = info if info is not None else torch.zeros(1, dtype=torch.int32, device=A.device)
    check(lib().rbt_solve_ex(n, k, _p(A), _ld(A), _p(B), _ld(B), depth, seed, _p(info), _p(work),
                             work.numel(), _stream(A.device)), "rbt_solve_ex")
    return A, B, info, work


def solve(A, B, depth=2, seed=2023):
    """X = A^-1 B by the RBT method; A and B are left unchanged."""
    A2 = colmajor(A)
    A2 = A2.clone() if A2.data_ptr() == A.data_ptr() else A2
    B2 = colmajor(B)
    B2 = B2.clone() if B2.data_ptr() == B.data_ptr() else B2
    _, X, info, _ = solve_(A2, B2, depth, seed)
    return X, A2, info


def solve_refine(A, B, depth=2, seed=2023, tol=None, max_iter=10, LU=None, X=None, work=None):
    """Out-of-place solve with FP64 refinement. Returns (X, LU, iters, berr, info, work)."""
    A = colmajor(A)
    B = colmajor(B)
    _dev_f64(A, "A")
    _dev_f64(B, "B")
    n, k = A.shape[0], B.shape[1]
    if tol is None:
        tol = 10.0 * n * 2.0 ** -52
    dev = A.device
    LU = LU if LU is not None else torch.empty_strided((n, n), (1, max(1, n)), dtype=torch.float64, device=dev)
    X = X if X is not None else torch.empty_strided((n, k), (1, max(1, n)), dtype=torch.float64, device=dev)
    work = work if work is not None else _workspace(n, k, depth, dev)
    iters = torch.zeros(1, dtype=torch.int32, device=dev)
    berr = torch.zeros(1, dtype=torch.float64, device=dev)
    info = torch.zeros(1, dtype=torch.int32, device=dev)
    check(lib().rbt_solve_refine(n, k, _p(A), _ld(A), _p(LU), _ld(LU), _p(B), _ld(B), _p(X), _ld(X),
                                 depth, seed, float(tol), int(max_iter), _p(iters), _p(berr),
                                 _p(info), _p(work), work.numel(), _stream(dev)), "rbt_solve_refine")
    return X, LU, iters, berr, info, work


def solve_mixed(A, B, depth=2, seed=2023, prec=RBT_FP32, solver=RBT_IR_CLASSIC, tol=None,
                max_iter=30, LU=None, X=None, work=None):
    """FP32 or BF16-update elimination of A~ with FP64 refinement.
    A, B: FP64 (read only). Returns (X, LU (FP32 factors of A~), iters, berr, info, work)."""
    A = colmajor(A)
    B = colmajor(B)
    _dev_f64(A, "A")
    _dev_f64(B, "B")
    n, k = A.shape[0], B.shape[1]
    if tol is None:
        tol = 10.0 * n * 2.0 ** -52
    dev = A.device
    LU = LU if LU is not None else torch.empty_strided((n, n), (1, max(1, n)), dtype=torch.float32, device=dev)
    if LU.dtype != torch.float32:
        raise TypeError("LU must be float32")
    X = X if X is not None else torch.empty_strided((n, k), (1, max(1, n)), dtype=torch.float64, device=dev)
    work = work if work is not None else _workspace(n, k, depth, dev, prec)
    iters = torch.zeros(1, dtype=torch.int32, device=dev)
    berr = torch.zeros(1, dtype=torch.float64, device=dev)
    info = torch.zeros(1, dtype=torch.int32, device=dev)
    check(lib().rbt_solve_mixed(n, k, _p(A), _ld(A), _p(LU), _ld(LU), _p(B), _ld(B), _p(X), _ld(X),
                                depth, seed, int(prec), int(solver), float(tol), int(max_iter),
                                _p(iters), _p(berr), _p(info), _p(work), work.numel(),
                                _stream(dev)), "rbt_solve_mixed")
    return X, LU, iters, berr, info, work


def solve_mixed_guarded(A, B, depth=2, seed=2023, prec=RBT_FP32, solver=RBT_IR_GMRES, tol=None,
                        max_iter=30, max_iter64=10, LU=None, LU64=None, X=None, work=None):
    """solve_mixed with a fallback to FP64 factors when the low-precision
    refinement cannot reach tol. Returns (X, LU, LU64, iters[2], berr,
    info[2], path, work); path 1 means the FP64 fallback ran (LU64 then holds
    the FP64 factors of A~), path 2 the pivoted re-solve (LU64 holds its
    factors)."""
    A = colmajor(A)
    B = colmajor(B)
    _dev_f64(A, "A")
    _dev_f64(B, "B")
    n, k = A.shape[0], B.shape[1]
    if tol is None:
        tol = 10.0 * n * 2.0 ** -52
    dev = A.device
    LU = LU if LU is not None else torch.empty_strided((n, n), (1, max(1, n)), dtype=torch.float32, device=dev)
    if LU.dtype != torch.float32:
        raise TypeError("LU must be float32")
    LU64 = LU64 if LU64 is not None else torch.empty_strided((n, n), (1, max(1, n)), dtype=torch.float64,
                                                             device=dev)
    if LU64.dtype != torch.float64:
        raise TypeError("LU64 must be float64")
    X = X if X is not None else torch.empty_strided((n, k), (1, max(1, n)), dtype=torch.float64, device=dev)
    work = work if work is not None else _workspace(n, k, depth, dev, prec)
    iters = torch.zeros(2, dtype=torch.int32, device=dev)
    berr = torch.zeros(1, dtype=torch.float64, device=dev)
    info = torch.zeros(2, dtype=torch.int32, device=dev)
    path = torch.zeros(1, dtype=torch.int32, device=dev)
    check(lib().rbt_solve_mixed_guarded(n, k, _p(A), _ld(A), _p(LU), _ld(LU), _p(LU64), _ld(LU64),
                                        _p(B), _ld(B), _p(X), _ld(X), depth, seed, int(prec),
                                        int(solver), float(tol), int(max_iter), int(max_iter64),
                                        _p(iters), _p(berr), _p(info), _p(path), _p(work),
                                        work.numel(), _stream(dev)), "rbt_solve_mixed_guarded")
    return X, LU, LU64, iters, berr, info, path, work


def gepp(A, work=None):
    """Partial-pivoting elimination in place (a copy of A is factored when A
    must be kept: pass A.clone()). Returns (LU, ipiv (1-based), info)."""
    A = colmajor(A)
    _dev_f64(A, "A")
    n = A.shape[0]
    dev = A.device
    work = work if work is not None else _workspace(n, 0, 0, dev)
    ipiv = torch.zeros(max(1, n), dtype=torch.int64, device=dev)
    info = torch.zeros(1, dtype=torch.int32, device=dev)
    check(lib().rbt_gepp(n, _p(A), _ld(A), _p(ipiv), _p(info), _p(work), work.numel(),
                         _stream(dev)), "rbt_gepp")
    return A, ipiv[:n], info


def gepp_solve(LU, ipiv, B, work=None):
    """B <- A^-1 B in place with the factors of gepp."""
    B = colmajor(B)
    _dev_f64(LU, "LU")
    _dev_f64(B, "B")
    n, k = LU.shape[0], B.shape[1]
    work = work if work is not None else _workspace(n, k, 0, LU.device)
    check(lib().rbt_gepp_solve(n, k, _p(LU), _ld(LU), _p(ipiv), _p(B), _ld(B), _p(work),
                               work.numel(), _stream(LU.device)), "rbt_gepp_solve")
    return B


def solve_guarded(A, B, depth=2, seed=2023, tol=None, max_iter=10, LU=None, X=None, work=None):
    """FP64 RBT solve with refinement and the Sec. 5 fallback to partial
    pivoting. Returns (X, LU, iters[2], berr, info[2], path, work); path 2
    means the pivoted re-solve ran (LU then holds its factors)."""
    A = colmajor(A)
    B = colmajor(B)
    _dev_f64(A, "A")
    _dev_f64(B, "B")
    n, k = A.shape[0], B.shape[1]
    if tol is None:
        tol = 10.0 * n * 2.0 ** -52
    dev = A.device
    LU = LU if LU is not None else torch.empty_strided((n, n), (1, max(1, n)), dtype=torch.float64,
                                                       device=dev)
    X = X if X is not None else torch.empty_strided((n, k), (1, max(1, n)), dtype=torch.float64,
                                                    device=dev)
    work = work if work is not None else _workspace(n, k, depth, dev)
    iters = torch.zeros(2, dtype=torch.int32, device=dev)
    berr = torch.zeros(1, dtype=torch.float64, device=dev)
    info = torch.zeros(2, dtype=torch.int32, device=dev)
    path = torch.zeros(1, dtype=torch.int32, device=dev)
    check(lib().rbt_solve_guarded(n, k, _p(A), _ld(A), _p(LU), _ld(LU), _p(B), _ld(B), _p(X),
                                  _ld(X), depth, seed, float(tol), int(max_iter), _p(iters),
                                  _p(berr), _p(info), _p(path), _p(work), work.numel(),
                                  _stream(dev)), "rbt_solve_guarded")
    return X, LU, iters, berr, info, path, work


class BatchPlan:
    """Sizes, workspace and device descriptor arrays of a planned batch."""

    def __init__(self, ns, ks, depth, prec, device="cuda"):
        ns = np.ascontiguousarray(np.asarray(ns, dtype=np.int64))
        ks = np.ascontiguousarray(np.asarray(ks, dtype=np.int64))
        if ns.shape != ks.shape or ns.ndim != 1:
            raise ValueError("ns and ks must be 1-D arrays of the same length")
        self.ns, self.ks, self.depth, self.prec = ns, ks, int(depth), int(prec)
        self.batch = int(ns.size)
        # launch shape chosen by the autotuner for this precision (or None:
        # the library's current options)
        from . import tune
        self.tuned = tune.load_table().get("bf16" if self.prec == RBT_BF16 else "fp32")
        vp = ctypes.c_void_p
        nbytes = lib().rbt_batched_workspace_size(self.batch, ns.ctypes.data_as(vp),
                                                  ks.ctypes.data_as(vp), self.depth, self.prec)
        if nbytes == 0 and self.batch > 0:
            raise _lib.RBTError("rbt_batched_workspace_size rejected the sizes")
        self.work = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=device)
        check(lib().rbt_batched_plan(self.batch, ns.ctypes.data_as(vp), ks.ctypes.data_as(vp),
                                     self.depth, self.prec, _p(self.work), self.work.numel(),
                                     _stream(self.work.device)), "rbt_batched_plan")


def batched_plan(ns, ks, depth=2, prec=RBT_FP32, device="cuda"):
    return BatchPlan(ns, ks, depth, prec, device)


class BatchArgs:
    """Device descriptor arrays (pointers and leading dimensions of A, B, X)
    and per-system outputs of a batched solve; building them copies to the
    device, launching with them does not."""

    def __init__(self, plan, As, Bs, Xs=None):
        if len(As) != plan.batch or len(Bs) != plan.batch:
            raise ValueError("batch size does not match the plan")
        dev = plan.work.device
        As = [colmajor(a) for a in As]
        Bs = [colmajor(b) for b in Bs]
        for s, (a, b) in enumerate(zip(As, Bs)):
            _dev_f64(a, f"As[{s}]")
            _dev_f64(b, f"Bs[{s}]")
            if a.shape != (plan.ns[s], plan.ns[s]) or b.shape != (plan.ns[s], plan.ks[s]):
                raise ValueError(f"system {s}: shapes {tuple(a.shape)}, {tuple(b.shape)} do not "
                                 f"match the plan ({plan.ns[s]}, {plan.ks[s]})")
        if Xs is None:
            Xs = [torch.empty_strided((int(n), int(k)), (1, max(1, int(n))), dtype=torch.float64,
                                      device=dev) for n, k in zip(plan.ns, plan.ks)]
        for s, x in enumerate(Xs):
            _dev_f64(x, f"Xs[{s}]")
            _ld(x)

        def ptrs(ts):
            return torch.tensor([t.data_ptr() for t in ts], dtype=torch.int64, device=dev)

        def lds(ts):
            return torch.tensor([_ld(t) for t in ts], dtype=torch.int64, device=dev)

        self.As, self.Bs, self.Xs = As, Bs, Xs
        self.pA, self.lA, self.pB, self.lB = ptrs(As), lds(As), ptrs(Bs), lds(Bs)
        self.pX, self.lX = ptrs(Xs), lds(Xs)
        nb = max(1, plan.batch)
        self.iters = torch.zeros(nb, dtype=torch.int32, device=dev)
        self.berr = torch.zeros(nb, dtype=torch.float64, device=dev)
        self.info = torch.zeros(nb, dtype=torch.int32, device=dev)
        self.path = torch.zeros(nb, dtype=torch.int32, device=dev)


def solve_batched_launch(plan, args, seed=2023, tol=-10.0, max_iter=30, tuned=True):
    """Enqueue the batched solve on the current stream (no allocation, no
    copy, no synchronization: capturable in a HIP graph). tol < 0 means
    |tol| n_s eps64 for system s. tuned: apply the autotuned launch shape of
    the plan's precision first (a schedule choice; results are identical)."""
    if tuned and plan.tuned is not None:
        set_option(_lib.RBT_OPT_BATCH_TILE_COLS2_MIN_N, plan.tuned["tile_cols2_min_n"])
        set_option(_lib.RBT_OPT_BATCH_WGS_PER_CU, plan.tuned["wgs_per_cu"])
    check(lib().rbt_solve_batched(plan.batch, _p(args.pA), _p(args.lA), _p(args.pB), _p(args.lB),
                                  _p(args.pX), _p(args.lX), plan.depth, seed, plan.prec,
                                  float(tol), int(max_iter), _p(args.iters), _p(args.berr),
                                  _p(args.info), _p(args.path), _p(plan.work), plan.work.numel(),
                                  _stream(plan.work.device)), "rbt_solve_batched")


def solve_batched(plan, As, Bs, seed=2023, tol=None, max_iter=30, Xs=None):
    """Solve the planned batch: As[s] (n x n), Bs[s] (n x nrhs) column-major
    FP64 device tensors. tol < 0 means |tol| n_s eps64 for system s (default
    10 n_s eps64). Returns (Xs, iters, berr, info); iters/berr/info are
    device tensors with one entry per system."""
    args = BatchArgs(plan, As, Bs, Xs)
    solve_batched_launch(plan, args, seed, -10.0 if tol is None else tol, max_iter)
    return args.Xs, args.iters, args.berr, args.info


def backward_error(A, X, B, work=None):
    """Eq. 7 (infinity norms), maximum over columns, as a device scalar."""
    A, X, B = colmajor(A), colmajor(X), colmajor(B)
    n, k = A.shape[0], X.shape[1]
    work = work if work is not None else _workspace(n, k, 0, A.device)
    berr = torch.zeros(1, dtype=torch.float64, device=A.device)
    check(lib().rbt_backward_error(n, k, _p(A), _ld(A), _p(X), _ld(X), _p(B), _ld(B), _p(berr),
                                   _p(work), work.numel(), _stream(A.device)), "rbt_backward_error")
    return berr


def timing_enable(on=True, stages=None):
    """Record HIP events around each stage of the composite entry points
    (stages: names from _lib.STAGES to time; None: all of them)."""
    mask = ((1 << _lib.RBT_STAGE_COUNT) - 1 if stages is None
            else sum(1 << _lib.STAGES.index(s) for s in stages))
    set_option(_lib.RBT_OPT_TIMING_STAGES, mask)
    check(lib().rbt_timing_enable(1 if on else 0), "rbt_timing_enable")


def timing_read():
    """Per-stage totals since the last read: {stage: (ms, launches, work)}."""
    n = _lib.RBT_STAGE_COUNT
    ms = np.zeros(n)
    cnt = np.zeros(n, dtype=np.int64)
    work = np.zeros(n)
    check(lib().rbt_timing_read(n, ms.ctypes.data_as(ctypes.c_void_p),
                                cnt.ctypes.data_as(ctypes.c_void_p),
                                work.ctypes.data_as(ctypes.c_void_p)), "rbt_timing_read")
    return {name: (float(ms[i]), int(cnt[i]), float(work[i])) for i, name in enumerate(_lib.STAGES)}


def set_option(option, value):
    check(lib().rbt_set_option(option, int(value)), "rbt_set_option")


def get_option(option):
    return int(lib().rbt_get_option(option))


def solve_backward(LU, X, G, depth=2, seed=2023, need_dA=True, work=None):
    """Adjoint of X = A^-1 B: returns (dA, dB) = (-A^-T G X^T, A^-T G).

    LU are the factors of U^T A V from the forward solve with the same
    (depth, seed); X is the forward solution. dA is None when not needed.
    """
    LU, X, G = colmajor(LU), colmajor(X), colmajor(G)
    _dev_f64(LU, "LU")
    _dev_f64(G, "G")
    n, k = LU.shape[0], G.shape[1]
    dev = LU.device
    dB = torch.empty_strided((n, k), (1, max(1, n)), dtype=torch.float64, device=dev)
    dA = torch.empty_strided((n, n), (1, max(1, n)), dtype=torch.float64, device=dev) if need_dA else None
    work = work if work is not None else _workspace(n, k, depth, dev)
    check(lib().rbt_solve_backward(n, k, _p(LU), _ld(LU), _p(X), _ld(X), _p(G), _ld(G), _p(dA),
                                   _ld(dA) if dA is not None else max(1, n), _p(dB), _ld(dB),
                                   depth, seed, _p(work), work.numel(), _stream(dev)),
          "rbt_solve_backward")
    return dA, dB


def solve_backward_mixed(LU, A, X, G, depth=2, seed=2023, tol=None, max_iter=30, need_dA=True,
                         work=None):
    """Adjoint of the mixed-precision solve: LU (FP32 factors of U^T A V from
    solve_mixed), A the original FP64 matrix (for the FP64 refinement of
    A^-T G). Returns (dA, dB, iters, berr)."""
    LU, A, X, G = colmajor(LU), colmajor(A), colmajor(X), colmajor(G)
    if not (LU.is_cuda and LU.dtype == torch.float32):
        raise TypeError("LU must be a float32 tensor on a HIP device")
    _dev_f64(A, "A")
    _dev_f64(G, "G")
    n, k = LU.shape[0], G.shape[1]
    if tol is None:
        tol = 10.0 * n * 2.0 ** -52
    dev = LU.device
    dB = torch.empty_strided((n, k), (1, max(1, n)), dtype=torch.float64, device=dev)
    dA = torch.empty_strided((n, n), (1, max(1, n)), dtype=torch.float64, device=dev) if need_dA else None
    work = work if work is not None else _workspace(n, k, depth, dev, RBT_FP32)
    iters = torch.zeros(1, dtype=torch.int32, device=dev)
    berr = torch.zeros(1, dtype=torch.float64, device=dev)
    check(lib().rbt_solve_backward_mixed(n, k, _p(LU), _ld(LU), _p(A), _ld(A), _p(X), _ld(X),
                                         _p(G), _ld(G), _p(dA),
                                         _ld(dA) if dA is not None else max(1, n), _p(dB),
                                         _ld(dB), depth, seed, float(tol), int(max_iter),
                                         _p(iters), _p(berr), _p(work), work.numel(),
                                         _stream(dev)), "rbt_solve_backward_mixed")
    return dA, dB, iters, berr


class RBTSolve(torch.autograd.Function):
    """X = A^-1 B by the RBT method, differentiable in A and B.

    Forward: the FP64 solve with refinement (A is kept for the residuals);
    backward: the adjoint through the same butterflies and saved factors
    (rbt_solve_backward)."""

    @staticmethod
    def forward(ctx, A, B, depth=2, seed=2023, max_iter=10):
        vec = B.dim() == 1
        B2 = B.reshape(-1, 1) if vec else B
        X, LU, _, _, _, _ = solve_refine(A.detach(), B2.detach(), depth, seed, max_iter=max_iter)
        ctx.save_for_backward(LU, X)
        ctx.depth, ctx.seed, ctx.vec = depth, seed, vec
        out = X.reshape(-1) if vec else X
        return out.clone(memory_format=torch.contiguous_format)

    @staticmethod
    def backward(ctx, G):
        LU, X = ctx.saved_tensors
        G2 = G.reshape(-1, 1) if ctx.vec else G
        dA, dB = solve_backward(LU, X, G2.contiguous(), ctx.depth, ctx.seed,
                                need_dA=ctx.needs_input_grad[0])
        if ctx.vec:
            dB = dB.reshape(-1)
        return dA, dB, None, None, None


class RBTSolveMixed(torch.autograd.Function):
    """X = A^-1 B with the FP32 (or BF16-update) factors and FP64 GMRES or
    classical refinement, differentiable in A and B; the backward solve
    reuses the FP32 factors and refines A^-T G in FP64 against A."""

    @staticmethod
    def forward(ctx, A, B, depth=2, seed=2023, max_iter=30, prec=RBT_FP32, solver=RBT_IR_GMRES):
        vec = B.dim() == 1
        B2 = B.reshape(-1, 1) if vec else B
        Ad = colmajor(A.detach())
        X, LU, _, _, _, _ = solve_mixed(Ad, B2.detach(), depth, seed, prec=prec, solver=solver,
                                        max_iter=max_iter)
        ctx.save_for_backward(LU, Ad, X)
        ctx.depth, ctx.seed, ctx.vec, ctx.max_iter = depth, seed, vec, max_iter
        out = X.reshape(-1) if vec else X
        return out.clone(memory_format=torch.contiguous_format)

    @staticmethod
    def backward(ctx, G):
        LU, Ad, X = ctx.saved_tensors
        G2 = G.reshape(-1, 1) if ctx.vec else G
        dA, dB, _, _ = solve_backward_mixed(LU, Ad, X, G2.contiguous(), ctx.depth, ctx.seed,
                                            max_iter=ctx.max_iter,
                                            need_dA=ctx.needs_input_grad[0])
        if ctx.vec:
            dB = dB.reshape(-1)
        return dA, dB, None, None, None, None, None


def rbt_solve(A, B, depth=2, seed=2023, max_iter=10, prec=RBT_FP64):
    """Differentiable X = A^-1 B (FP64 tensors on the device). prec RBT_FP32
    or RBT_BF16: low-precision factors with FP64 GMRES refinement (forward)
    and FP64 refinement of the adjoint solve (backward)."""
    if prec != RBT_FP64:
        return RBTSolveMixed.apply(A, B, depth, seed, max(max_iter, 30), prec, RBT_IR_GMRES)
    return RBTSolve.apply(A, B, depth, seed, max_iter)
