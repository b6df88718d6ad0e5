"""ctypes binding of libconcord.so (argument marshalling only).

Every step of a solve runs in the library's HIP kernels; this module only
turns torch tensors into device pointers and the status codes into Python
exceptions.  torch is imported first so that the library binds to the HIP
runtime torch has already loaded (one runtime per process).
"""
from __future__ import annotations

import ctypes
import os
import warnings

import torch  # noqa: F401  (must be loaded before libconcord.so)

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libconcord.so")

F32, F64 = 0, 1
INPUT_S, INPUT_Y = 0, 1
OK, NOT_CONVERGED = 0, 1
EINVAL, ENONFINITE, ENOTPD, ENOMEM, EDEVICE, ELAUNCH, ESCRATCH = -1, -2, -3, -4, -5, -6, -7
NOALLOC_SCRATCH_BYTES = 64 << 20  # CONCORD_NOALLOC_SCRATCH_BYTES


class ConcordInfo(ctypes.Structure):
    _fields_ = [
        ("sweeps", ctypes.c_int32),
        ("status", ctypes.c_int32),
        ("delta", ctypes.c_double),
        ("tol_eff", ctypes.c_double),
        ("nnz_upper", ctypes.c_int64),
        ("objective", ctypes.c_double),
        ("elapsed_ms", ctypes.c_double),
        ("gram_ms", ctypes.c_double),
        ("sweep_ms", ctypes.c_double),
        ("moved_pairs", ctypes.c_int64),
        ("moved_diag", ctypes.c_int64),
        ("row_groups", ctypes.c_int32),
        ("col_slices", ctypes.c_int32),
        ("w_in_lds", ctypes.c_int32),
        ("block_threads", ctypes.c_int32),
        ("pending_depth", ctypes.c_int32),
        ("active_sweeps", ctypes.c_int32),
    ]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


class ConcordJointInfo(ctypes.Structure):
    _fields_ = [
        ("sweeps", ctypes.c_int32),
        ("status", ctypes.c_int32),
        ("delta", ctypes.c_double),
        ("tol_eff", ctypes.c_double),
        ("nnz_upper", ctypes.c_int64 * 2),
        ("differ_upper", ctypes.c_int64),
        ("objective", ctypes.c_double),
        ("elapsed_ms", ctypes.c_double),
        ("gram_ms", ctypes.c_double),
        ("sweep_ms", ctypes.c_double),
        ("moved_pairs", ctypes.c_int64),
        ("moved_diag", ctypes.c_int64),
        ("row_groups", ctypes.c_int32),
        ("col_slices", ctypes.c_int32),
        ("w_in_lds", ctypes.c_int32),
        ("block_threads", ctypes.c_int32),
        ("pending_depth", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
    ]

    def as_dict(self) -> dict:
        d = {k: getattr(self, k) for k, _ in self._fields_ if k != "reserved"}
        d["nnz_upper"] = (int(self.nnz_upper[0]), int(self.nnz_upper[1]))
        return d


class ConcordOptions(ctypes.Structure):
    _fields_ = [
        ("row_groups", ctypes.c_int32),
        ("col_slices", ctypes.c_int32),
        ("block_threads", ctypes.c_int32),
        ("w_in_lds", ctypes.c_int32),
        ("pending_depth", ctypes.c_int32),
        ("delta_trace", ctypes.POINTER(ctypes.c_double)),
        ("device_timestamps", ctypes.c_void_p),
        ("timestamp_steps", ctypes.c_int32),
        ("sync_rewrites", ctypes.c_int32),
        ("w_out", ctypes.c_void_p),
        ("active_set", ctypes.c_int32),
        ("active_maxit", ctypes.c_int32),
    ]


class ConcordBatchOptions(ctypes.Structure):
    _fields_ = [
        ("workgroups", ctypes.c_int32),
        ("block_threads", ctypes.c_int32),
        ("pending_depth", ctypes.c_int32),
        ("cols_per_lane", ctypes.c_int32),
        ("problem_workgroups", ctypes.POINTER(ctypes.c_int32)),
        ("problem_col_slices", ctypes.POINTER(ctypes.c_int32)),
        ("sync_rewrites", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
    ]


class ConcordError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"concord error {code}: {msg}")
        self.code = code


class NotConvergedWarning(UserWarning):
    pass


_lib = None


def load(path: str = LIB_PATH):
    """Load the built library; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(
            f"{path} is missing: build it with `python -c 'import __graft_entry__ as g; g.build()'` "
            "(there is no CPU fallback)")
    lib = ctypes.CDLL(path)
    vp, i64, i32, dbl = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_double
    lib.concord_fit.argtypes = [ctypes.c_int, vp, i64, i64, dbl, dbl, i32, ctypes.c_int, vp, vp,
                                ctypes.POINTER(ConcordInfo), vp]
    lib.concord_fit.restype = ctypes.c_int
    lib.concord_fit_noalloc.argtypes = lib.concord_fit.argtypes
    lib.concord_fit_noalloc.restype = ctypes.c_int
    lib.concord_fit_ex.argtypes = lib.concord_fit.argtypes + [ctypes.POINTER(ConcordOptions)]
    lib.concord_fit_ex.restype = ctypes.c_int
    lib.concord_fit_batched_ex.argtypes = [
        i32, ctypes.c_int, ctypes.POINTER(vp), ctypes.POINTER(i64), ctypes.POINTER(i64), i32,
        ctypes.POINTER(dbl), dbl, i32, ctypes.c_int, ctypes.POINTER(vp),
        ctypes.POINTER(ConcordInfo), vp, ctypes.POINTER(ConcordBatchOptions)]
    lib.concord_fit_batched_ex.restype = ctypes.c_int
    lib.concord_fit_batched.argtypes = lib.concord_fit_batched_ex.argtypes[:-1]
    lib.concord_fit_batched.restype = ctypes.c_int
    lib.concord_backward_ex.argtypes = [vp, vp, i64, vp, vp, ctypes.POINTER(dbl), dbl, i32,
                                        ctypes.c_int, ctypes.POINTER(ConcordInfo), vp,
                                        ctypes.POINTER(ConcordOptions)]
    lib.concord_backward_ex.restype = ctypes.c_int
    lib.concord_backward.argtypes = lib.concord_backward_ex.argtypes[:-1]
    lib.concord_backward.restype = ctypes.c_int
    lib.concord_fit_joint_ex.argtypes = [ctypes.c_int, vp, vp, i64, i64, i64, dbl, dbl, dbl, i32,
                                         ctypes.c_int, vp, vp, vp, vp,
                                         ctypes.POINTER(ConcordJointInfo), vp,
                                         ctypes.POINTER(ConcordOptions)]
    lib.concord_fit_joint_ex.restype = ctypes.c_int
    lib.concord_fit_joint.argtypes = lib.concord_fit_joint_ex.argtypes[:-1]
    lib.concord_fit_joint.restype = ctypes.c_int
    lib.concord_gram.argtypes = [vp, i64, i64, ctypes.c_int, vp, vp]
    lib.concord_gram.restype = ctypes.c_int
    lib.concord_schedule.argtypes = [i64, ctypes.POINTER(ctypes.c_int32)]
    lib.concord_schedule.restype = i64
    lib.concord_strerror.argtypes = [ctypes.c_int]
    lib.concord_strerror.restype = ctypes.c_char_p
    lib.concord_version.argtypes = []
    lib.concord_version.restype = ctypes.c_char_p
    _lib = lib
    return lib


def strerror(code: int) -> str:
    return load().concord_strerror(int(code)).decode()


def _dtype_code(t: torch.Tensor) -> int:
    if t.dtype == torch.float64:
        return F64
    if t.dtype == torch.float32:
        return F32
    raise TypeError(f"unsupported dtype {t.dtype}; use float32 or float64")


def _check_dev(t: torch.Tensor, name: str):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


def _stream_handle(stream) -> ctypes.c_void_p:
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _raise(code: int, what: str):
    if code < 0:
        raise ConcordError(code, f"{what}: {strerror(code)}")
    if code == NOT_CONVERGED:
        warnings.warn(f"{what}: {strerror(code)}", NotConvergedWarning, stacklevel=3)


def fit(X: torch.Tensor, lam: float, tol: float = 1e-6, maxit: int = 500, *, kind: str = "S",
        omega0: torch.Tensor | None = None, out: torch.Tensor | None = None, stream=None,
        row_groups: int = 0, col_slices: int = 0, block_threads: int = 0, w_in_lds: int = 0,
        pending_depth: int = 0, sync_rewrites: bool = False, trace: bool = False,
        check: bool = True,
        timestamps: torch.Tensor | None = None, w_out: torch.Tensor | None = None,
        active_set: bool = False, active_maxit: int = 0):
    """One CONCORD-PCD solve.  X is S (p x p) or, with kind='Y', Y (n x p).

    Returns (omega, info dict); info['delta_trace'] holds every sweep's delta
    when ``trace`` is set.  Raises ConcordError on a negative status (unless
    check=False) and warns when the sweep limit was reached.
    """
    lib = load()
    _check_dev(X, "X")
    dt = _dtype_code(X)
    if kind == "S":
        if X.dim() != 2 or X.shape[0] != X.shape[1]:
            raise ValueError("S must be square")
        p, n, kc = X.shape[0], 0, INPUT_S
    elif kind == "Y":
        if X.dim() != 2:
            raise ValueError("Y must be a matrix")
        n, p, kc = X.shape[0], X.shape[1], INPUT_Y
    else:
        raise ValueError("kind must be 'S' or 'Y'")
    if out is None:
        out = torch.empty((p, p), dtype=X.dtype, device=X.device)
    _check_dev(out, "out")
    if out.dtype != X.dtype or tuple(out.shape) != (p, p):
        raise ValueError("out must be p x p with X's dtype")
    o0 = None
    if omega0 is not None:
        _check_dev(omega0, "omega0")
        if omega0.dtype != X.dtype or tuple(omega0.shape) != (p, p):
            raise ValueError("omega0 must be p x p with X's dtype")
        o0 = ctypes.c_void_p(omega0.data_ptr())
    info = ConcordInfo()
    opts = ConcordOptions(row_groups, col_slices, block_threads, w_in_lds, pending_depth, None,
                          None, 0, int(bool(sync_rewrites)), None, int(bool(active_set)),
                          int(active_maxit))
    if w_out is not None:
        _check_dev(w_out, "w_out")
        if w_out.dtype != X.dtype or tuple(w_out.shape) != (p, p):
            raise ValueError("w_out must be p x p with X's dtype")
        opts.w_out = w_out.data_ptr()
    if timestamps is not None:
        # int64 device tensor of shape (workgroups, steps, 3)
        _check_dev(timestamps, "timestamps")
        opts.device_timestamps = timestamps.data_ptr()
        opts.timestamp_steps = int(timestamps.shape[1])
    tr = None
    if trace:
        tr = (ctypes.c_double * int(maxit))()
        opts.delta_trace = ctypes.cast(tr, ctypes.POINTER(ctypes.c_double))
    with torch.cuda.device(X.device):
        code = lib.concord_fit_ex(kc, ctypes.c_void_p(X.data_ptr()), n, p, float(lam), float(tol),
                                  int(maxit), dt, o0, ctypes.c_void_p(out.data_ptr()),
                                  ctypes.byref(info), _stream_handle(stream), ctypes.byref(opts))
    d = info.as_dict()
    d["code"] = code
    if tr is not None:
        d["delta_trace"] = [tr[k] for k in range(max(0, info.sweeps))]
    if check:
        _raise(code, "concord_fit")
    return out, d


def fit_noalloc(X: torch.Tensor, lam: float, tol: float = 1e-6, maxit: int = 500, *,
                kind: str = "S", omega0: torch.Tensor | None = None,
                out: torch.Tensor | None = None, stream=None, check: bool = True):
    """concord_fit_noalloc: one solve in the library's fixed device scratch
    (no device allocation inside the call).  ``out`` must be given by callers
    that cannot allocate; otherwise it is allocated here, before the call.
    Returns (omega, info dict); the device times in info read 0."""
    lib = load()
    _check_dev(X, "X")
    dt = _dtype_code(X)
    if kind == "S":
        if X.dim() != 2 or X.shape[0] != X.shape[1]:
            raise ValueError("S must be square")
        p, n, kc = X.shape[0], 0, INPUT_S
    elif kind == "Y":
        if X.dim() != 2:
            raise ValueError("Y must be a matrix")
        n, p, kc = X.shape[0], X.shape[1], INPUT_Y
    else:
        raise ValueError("kind must be 'S' or 'Y'")
    if out is None:
        out = torch.empty((p, p), dtype=X.dtype, device=X.device)
    _check_dev(out, "out")
    if out.dtype != X.dtype or tuple(out.shape) != (p, p):
        raise ValueError("out must be p x p with X's dtype")
    o0 = None
    if omega0 is not None:
        _check_dev(omega0, "omega0")
        if omega0.dtype != X.dtype or tuple(omega0.shape) != (p, p):
            raise ValueError("omega0 must be p x p with X's dtype")
        o0 = ctypes.c_void_p(omega0.data_ptr())
    info = ConcordInfo()
    with torch.cuda.device(X.device):
        code = lib.concord_fit_noalloc(kc, ctypes.c_void_p(X.data_ptr()), n, p, float(lam),
                                       float(tol), int(maxit), dt, o0,
                                       ctypes.c_void_p(out.data_ptr()), ctypes.byref(info),
                                       _stream_handle(stream))
    d = info.as_dict()
    d["code"] = code
    if check:
        _raise(code, "concord_fit_noalloc")
    return out, d


def fit_joint(X1: torch.Tensor, X2: torch.Tensor, lam1: float, lam2: float, tol: float = 1e-6,
              maxit: int = 500, *, kind: str = "S", omega0=(None, None), outs=None,
              stream=None, row_groups: int = 0, col_slices: int = 0, block_threads: int = 0,
              w_in_lds: int = 0, pending_depth: int = 0, sync_rewrites: bool = False,
              trace: bool = False,
              check: bool = True):
    """Joint estimation of two precision matrices with a fused penalty
    (Section 6).  X1, X2 are S_1, S_2 (p x p) or, with kind='Y', Y_1, Y_2
    (n_m x p).  Returns (omega_1, omega_2, info dict)."""
    lib = load()
    for t, nm in ((X1, "X1"), (X2, "X2")):
        _check_dev(t, nm)
        if t.dim() != 2:
            raise ValueError(f"{nm} must be a matrix")
    if X1.dtype != X2.dtype or X1.device != X2.device:
        raise ValueError("X1 and X2 must share dtype and device")
    dt = _dtype_code(X1)
    if kind == "S":
        if X1.shape[0] != X1.shape[1] or tuple(X2.shape) != tuple(X1.shape):
            raise ValueError("S_1 and S_2 must be square and of one size")
        p, n1, n2, kc = X1.shape[0], 0, 0, INPUT_S
    elif kind == "Y":
        if X1.shape[1] != X2.shape[1]:
            raise ValueError("Y_1 and Y_2 must have the same number of columns")
        p, n1, n2, kc = X1.shape[1], X1.shape[0], X2.shape[0], INPUT_Y
    else:
        raise ValueError("kind must be 'S' or 'Y'")
    if outs is None:
        outs = (torch.empty((p, p), dtype=X1.dtype, device=X1.device),
                torch.empty((p, p), dtype=X1.dtype, device=X1.device))
    for o in outs:
        _check_dev(o, "out")
        if o.dtype != X1.dtype or tuple(o.shape) != (p, p):
            raise ValueError("outputs must be p x p with the inputs' dtype")
    o0 = []
    for o in omega0:
        if o is None:
            o0.append(None)
            continue
        _check_dev(o, "omega0")
        if o.dtype != X1.dtype or tuple(o.shape) != (p, p):
            raise ValueError("omega0 must be p x p with the inputs' dtype")
        o0.append(ctypes.c_void_p(o.data_ptr()))
    info = ConcordJointInfo()
    opts = ConcordOptions(row_groups, col_slices, block_threads, w_in_lds, pending_depth, None,
                          None, 0, int(bool(sync_rewrites)), None, 0, 0)
    tr = None
    if trace:
        tr = (ctypes.c_double * int(maxit))()
        opts.delta_trace = ctypes.cast(tr, ctypes.POINTER(ctypes.c_double))
    with torch.cuda.device(X1.device):
        code = lib.concord_fit_joint_ex(
            kc, ctypes.c_void_p(X1.data_ptr()), ctypes.c_void_p(X2.data_ptr()), n1, n2, p,
            float(lam1), float(lam2), float(tol), int(maxit), dt, o0[0], o0[1],
            ctypes.c_void_p(outs[0].data_ptr()), ctypes.c_void_p(outs[1].data_ptr()),
            ctypes.byref(info), _stream_handle(stream), ctypes.byref(opts))
    d = info.as_dict()
    d["code"] = code
    if tr is not None:
        d["delta_trace"] = [tr[k] for k in range(max(0, info.sweeps))]
    if check:
        _raise(code, "concord_fit_joint")
    return outs[0], outs[1], d


def fit_batched(Xs, lambdas, tol: float = 1e-6, maxit: int = 500, *, kind: str = "S",
                outs=None, stream=None, workgroups: int = 0, block_threads: int = 0,
                pending_depth: int = 0, problem_workgroups=None, problem_col_slices=None,
                cols_per_lane: int = 0, sync_rewrites: bool = False, check: bool = True):
    """B independent solves along lambda paths in one persistent launch.

    Xs: list of B device tensors (S_b, or Y_b with kind='Y'), one dtype.
    lambdas: B x L nested sequence (or one length-L sequence for all).
    Returns (omegas, infos, code): omegas[b][l] is the p_b x p_b Omega at
    lambdas[b][l] (warm-started from omegas[b][l - 1]); infos[b][l] its dict.
    Launch options: ``problem_workgroups`` (workgroups per problem),
    ``problem_col_slices`` (how many column slices they form), ``cols_per_lane``
    (2 or 4) and ``block_threads``; see concord_batch_options.
    """
    import numpy as np
    lib = load()
    B = len(Xs)
    if B < 1:
        raise ValueError("need at least one problem")
    lam = np.asarray(lambdas, dtype=np.float64)
    if lam.ndim == 1:
        lam = np.broadcast_to(lam, (B, lam.shape[0]))
    if lam.ndim != 2 or lam.shape[0] != B:
        raise ValueError("lambdas must be B x L")
    lam = np.ascontiguousarray(lam)
    L = lam.shape[1]
    dt = _dtype_code(Xs[0])
    ps, ns = [], []
    for b, X in enumerate(Xs):
        _check_dev(X, f"Xs[{b}]")
        if X.dtype != Xs[0].dtype or X.device != Xs[0].device:
            raise ValueError("all problems must share dtype and device")
        if kind == "S":
            if X.dim() != 2 or X.shape[0] != X.shape[1]:
                raise ValueError("S must be square")
            ps.append(X.shape[0])
            ns.append(0)
        elif kind == "Y":
            if X.dim() != 2:
                raise ValueError("Y must be a matrix")
            ns.append(X.shape[0])
            ps.append(X.shape[1])
        else:
            raise ValueError("kind must be 'S' or 'Y'")
    if outs is None:
        outs = [[torch.empty((ps[b], ps[b]), dtype=Xs[0].dtype, device=Xs[0].device)
                 for _ in range(L)] for b in range(B)]
    for b in range(B):
        if len(outs[b]) != L:
            raise ValueError("outs must be B x L")
        for l in range(L):
            o = outs[b][l]
            _check_dev(o, "outs")
            if o.dtype != Xs[0].dtype or tuple(o.shape) != (ps[b], ps[b]):
                raise ValueError("each output must be p_b x p_b with the inputs' dtype")
    vp = ctypes.c_void_p
    xa = (vp * B)(*[X.data_ptr() for X in Xs])
    na = (ctypes.c_int64 * B)(*ns)
    pa = (ctypes.c_int64 * B)(*ps)
    la = (ctypes.c_double * (B * L))(*lam.ravel().tolist())
    oa = (vp * (B * L))(*[outs[b][l].data_ptr() for b in range(B) for l in range(L)])
    infos = (ConcordInfo * (B * L))()
    opts = ConcordBatchOptions(workgroups, block_threads, pending_depth, cols_per_lane, None,
                               None, int(bool(sync_rewrites)), 0)
    pw = pc = None
    if problem_workgroups is not None:
        if len(problem_workgroups) != B:
            raise ValueError("problem_workgroups needs one count per problem")
        pw = (ctypes.c_int32 * B)(*[int(x) for x in problem_workgroups])
        opts.problem_workgroups = ctypes.cast(pw, ctypes.POINTER(ctypes.c_int32))
    if problem_col_slices is not None:
        if len(problem_col_slices) != B:
            raise ValueError("problem_col_slices needs one count per problem")
        pc = (ctypes.c_int32 * B)(*[int(x) for x in problem_col_slices])
        opts.problem_col_slices = ctypes.cast(pc, ctypes.POINTER(ctypes.c_int32))
    with torch.cuda.device(Xs[0].device):
        code = lib.concord_fit_batched_ex(B, INPUT_S if kind == "S" else INPUT_Y, xa, na, pa, L,
                                          la, float(tol), int(maxit), dt, oa, infos,
                                          _stream_handle(stream), ctypes.byref(opts))
    di = [[infos[b * L + l].as_dict() for l in range(L)] for b in range(B)]
    if check:
        _raise(code, "concord_fit_batched")
    return outs, di, code


def backward(S: torch.Tensor, omega: torch.Tensor, grad_omega: torch.Tensor, tol: float = 1e-10,
             maxit: int = 2000, *, out: torch.Tensor | None = None, stream=None,
             row_groups: int = 0, col_slices: int = 0, block_threads: int = 0,
             w_in_lds: int = 0, pending_depth: int = 0, sync_rewrites: bool = False,
             check: bool = True):
    """Implicit gradient of Omega-hat = fit(S, lam): returns (dL/dS, dL/dlam, info)
    for dL/dOmega-hat = grad_omega.  dL/dS is the symmetric gradient."""
    lib = load()
    for t, name in ((S, "S"), (omega, "omega"), (grad_omega, "grad_omega")):
        _check_dev(t, name)
        if t.dtype != S.dtype or t.dim() != 2 or t.shape[0] != t.shape[1] \
                or t.shape[0] != S.shape[0]:
            raise ValueError(f"{name} must be p x p with S's dtype")
    p = S.shape[0]
    dt = _dtype_code(S)
    if out is None:
        out = torch.empty((p, p), dtype=S.dtype, device=S.device)
    _check_dev(out, "out")
    info = ConcordInfo()
    gl = ctypes.c_double(0.0)
    opts = ConcordOptions(row_groups, col_slices, block_threads, w_in_lds, pending_depth, None,
                          None, 0, int(bool(sync_rewrites)), None)
    with torch.cuda.device(S.device):
        code = lib.concord_backward_ex(ctypes.c_void_p(S.data_ptr()),
                                       ctypes.c_void_p(omega.data_ptr()), p,
                                       ctypes.c_void_p(grad_omega.data_ptr()),
                                       ctypes.c_void_p(out.data_ptr()), ctypes.byref(gl),
                                       float(tol), int(maxit), dt, ctypes.byref(info),
                                       _stream_handle(stream), ctypes.byref(opts))
    d = info.as_dict()
    d["code"] = code
    if check:
        _raise(code, "concord_backward")
    return out, gl.value, d


def gram(Y: torch.Tensor, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """S = Y^T Y / n on the device (matrix-core kernel)."""
    lib = load()
    _check_dev(Y, "Y")
    dt = _dtype_code(Y)
    n, p = Y.shape
    if out is None:
        out = torch.empty((p, p), dtype=Y.dtype, device=Y.device)
    _check_dev(out, "out")
    with torch.cuda.device(Y.device):
        code = lib.concord_gram(ctypes.c_void_p(Y.data_ptr()), n, p, dt,
                                ctypes.c_void_p(out.data_ptr()), _stream_handle(stream))
    _raise(code, "concord_gram")
    return out


def schedule(p: int):
    """Closed-form round-robin table (host): int32 array (m, p_even // 2, 2)."""
    import numpy as np
    lib = load()
    pe = p + (p & 1)
    m, h = pe - 1, pe // 2
    buf = np.zeros((max(m, 0), h, 2), dtype=np.int32)
    got = lib.concord_schedule(int(p), buf.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
    if got < 0:
        raise ConcordError(int(got), strerror(int(got)))
    return buf
