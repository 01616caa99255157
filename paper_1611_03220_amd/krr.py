"""Python binding of libkrr (ctypes). Argument marshalling only: every step runs in the
HIP library. Tensors are torch device tensors; the library enqueues on torch's current
stream. Loading fails loudly when the library is missing: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libkrr.so")

OK, E_ARG, E_NOT_SPD, E_NO_CONV, E_BREAKDOWN, E_HIP, E_WORKSPACE = range(7)
STATUS_NAMES = {0: "OK", 1: "E_ARG", 2: "E_NOT_SPD", 3: "E_NO_CONV", 4: "E_BREAKDOWN",
                5: "E_HIP", 6: "E_WORKSPACE"}
PREC = {"fp64": 0, "f16x3": 1, "bf16x3": 2}
(OP_FEATURES, OP_PRECOND_FACTOR, OP_KERNEL_MATMAT, OP_PCG_SOLVE, OP_GRAD, OP_PRECOND_APPLY,
 OP_DSIGMA_INNER, OP_GAUSSIAN_PROJECT, OP_PRECOND_TEST, OP_ADAPTIVE_FEATURES,
 OP_AUTOTUNE) = range(11)

_i64 = ctypes.c_int64
_i32 = ctypes.c_int32
_dbl = ctypes.c_double
_vp = ctypes.c_void_p
_sz = ctypes.c_size_t


class KRRError(RuntimeError):
    def __init__(self, status: int, msg: str, report=None, info: int = 0):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status
        self.report = report
        self.info = info


class PCGOpts(ctypes.Structure):
    _fields_ = [("tol", _dbl), ("max_iter", _i32), ("prec", _i32), ("use_precond", _i32),
                ("check_every", _i32), ("lambda_p", _dbl), ("true_residual", _i32),
                ("refine", _i32), ("warm_start", _i32)]


class PCGReport(ctypes.Structure):
    _fields_ = [("iters", _i32), ("converged_cols", _i32), ("breakdown_cols", _i32),
                ("refine_steps", _i32), ("relres_rec", ctypes.POINTER(_dbl)),
                ("relres_true", ctypes.POINTER(_dbl)), ("history", ctypes.POINTER(_dbl)),
                ("history_cap", _i32), ("history_len", _i32), ("matmat_calls", _i32),
                ("matmat_ms", _dbl)]


BATCH_MAX_M = 16


class BatchProblem(ctypes.Structure):
    _fields_ = [("X", _vp), ("n", _i64), ("d", _i64), ("ldx", _i64), ("sigma", _dbl),
                ("lam", _dbl), ("lambda_p", _dbl), ("Ut", _vp), ("s", _i64), ("ldu", _i64),
                ("Y", _vp), ("ldy", _i64), ("alpha", _vp), ("lda", _i64), ("m", _i64)]


class Kernel(ctypes.Structure):
    """krr_kernel: the Gaussian or the polynomial kernel (Sec. 6)."""
    _fields_ = [("kind", _i32), ("degree", _i32), ("sigma", _dbl), ("gamma", _dbl),
                ("coef0", _dbl)]

    @classmethod
    def gaussian(cls, sigma: float) -> "Kernel":
        return cls(0, 1, float(sigma), 0.0, 0.0)

    @classmethod
    def polynomial(cls, gamma: float, coef0: float, degree: int) -> "Kernel":
        return cls(1, int(degree), 1.0, float(gamma), float(coef0))


class PrecondTestReport(ctypes.Structure):
    """krr_precond_test_report (Thm. 4 test of a candidate sketch)."""
    _fields_ = [("cond1", _dbl), ("ratio_lo", _dbl), ("ratio_hi", _dbl), ("rank", _i32),
                ("passed", _i32), ("power_iters", _i32), ("jacobi_sweeps", _i32)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


class TuneReport(ctypes.Structure):
    """krr_tune_report."""
    _fields_ = [("candidates", _i32), ("default_nsplit", _i32), ("default_pass_width", _i32),
                ("nsplit", _i32), ("pass_width", _i32), ("default_ms", _dbl), ("best_ms", _dbl)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


class SetupProblem(ctypes.Structure):
    """krr_setup_problem."""
    _fields_ = [("X", _vp), ("n", _i64), ("d", _i64), ("ldx", _i64), ("W", _vp), ("b", _vp),
                ("s", _i64), ("lambda_p", _dbl), ("Z", _vp), ("ldz", _i64), ("C", _vp),
                ("Ut", _vp), ("ldu", _i64), ("info", _i64)]


class BatchReport(ctypes.Structure):
    _fields_ = [("iters", _i32), ("converged_cols", _i32), ("breakdown_cols", _i32),
                ("refine_steps", _i32),
                ("relres_rec", ctypes.POINTER(_dbl)), ("relres_true", ctypes.POINTER(_dbl)),
                ("col_iters", ctypes.POINTER(_i32)), ("product_ms", _dbl), ("iteration_ms", _dbl), ("tiles_per_item", _i32),
                ("work_items", _i32)]


_lib = None


def lib():
    """Load libkrr.so (built by ``paper_1611_03220_amd.build``)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"libkrr.so not found at {LIB_PATH}: run paper_1611_03220_amd.build.build()")
    import torch.cuda  # noqa: F401  (the HIP runtime torch loaded is the one libkrr binds to)
    L = ctypes.CDLL(LIB_PATH)
    L.krr_workspace_bytes.restype = _sz
    L.krr_workspace_bytes.argtypes = [_i32, _i64, _i64, _i64, _i64, _i64, _i32]
    L.krr_last_error.restype = ctypes.c_char_p
    L.krr_version.restype = ctypes.c_char_p
    L.krr_pcg_defaults.argtypes = [ctypes.POINTER(PCGOpts)]
    L.krr_features.restype = _i32
    L.krr_features.argtypes = [_vp, _i64, _i64, _i64, _vp, _vp, _i64, _vp, _i64, _vp, _sz, _vp]
    L.krr_precond_factor.restype = _i32
    L.krr_precond_factor.argtypes = [_vp, _i64, _i64, _i64, _dbl, _vp, _vp, _i64, _vp, _sz,
                                     ctypes.POINTER(_i64), _vp]
    L.krr_precond_apply.restype = _i32
    L.krr_precond_apply.argtypes = [_vp, _i64, _i64, _i64, _dbl, _vp, _i64, _i64, _vp, _i64, _vp,
                                    _sz, _vp]
    L.krr_kernel_matmat.restype = _i32
    L.krr_kernel_matmat.argtypes = [_vp, _i64, _i64, _vp, _i64, _i64, _i64, _dbl, _dbl, _vp, _i64,
                                    _i64, _vp, _i64, _i32, _i32, _vp, _sz, _vp]
    L.krr_pcg_solve.restype = _i32
    L.krr_pcg_solve.argtypes = [_vp, _i64, _i64, _i64, _dbl, _dbl, _vp, _i64, _i64, _vp, _i64,
                                _vp, _i64, _i64, ctypes.POINTER(PCGOpts),
                                ctypes.POINTER(PCGReport), _vp, _sz, _vp]
    L.krr_grad.restype = _i32
    L.krr_grad.argtypes = [_vp, _i64, _i64, _i64, _dbl, _vp, _vp, _i64, _i64,
                           ctypes.POINTER(_dbl), ctypes.POINTER(_dbl), _i32, _vp, _sz, _vp]
    L.krr_kernel_matmat_k.restype = _i32
    L.krr_kernel_matmat_k.argtypes = [ctypes.POINTER(Kernel), _vp, _i64, _i64, _vp, _i64, _i64,
                                      _i64, _dbl, _vp, _i64, _i64, _vp, _i64, _i32, _i32, _vp,
                                      _sz, _vp]
    L.krr_pcg_solve_k.restype = _i32
    L.krr_pcg_solve_k.argtypes = [ctypes.POINTER(Kernel), _vp, _i64, _i64, _i64, _dbl, _vp, _i64,
                                  _i64, _vp, _i64, _vp, _i64, _i64, ctypes.POINTER(PCGOpts),
                                  ctypes.POINTER(PCGReport), _vp, _sz, _vp]
    L.krr_tensorsketch.restype = _i32
    L.krr_tensorsketch.argtypes = [_vp, _i64, _i64, _i64, _dbl, _dbl, _i32, _vp, _vp, _i64, _vp,
                                   _i64, _vp]
    L.krr_srht.restype = _i32
    L.krr_srht.argtypes = [_vp, _i64, _i64, _i64, _vp, _vp, _i64, _vp, _i64, _vp]
    L.krr_gaussian_project.restype = _i32
    L.krr_gaussian_project.argtypes = [_vp, _i64, _i64, _i64, _vp, _i64, _vp, _i64, _vp, _sz, _vp]
    L.krr_precond_test.restype = _i32
    L.krr_precond_test.argtypes = [ctypes.POINTER(Kernel), _vp, _i64, _i64, _i64, _vp, _i64, _i64,
                                   _dbl, _i32, _i32, ctypes.POINTER(PrecondTestReport), _vp, _sz,
                                   _vp]
    L.krr_adaptive_features.restype = _i32
    L.krr_adaptive_features.argtypes = [ctypes.POINTER(Kernel), _vp, _i64, _i64, _i64, _dbl, _vp,
                                        _vp, _vp, _vp, _i64, _i64, _vp, _i64,
                                        ctypes.POINTER(_i64), ctypes.POINTER(PrecondTestReport),
                                        _i32, ctypes.POINTER(_i32), _i32, _i32, _vp, _sz, _vp]
    L.krr_autotune_matmat.restype = _i32
    L.krr_autotune_matmat.argtypes = [ctypes.POINTER(Kernel), _vp, _i64, _i64, _i64, _i64, _i32,
                                      ctypes.POINTER(TuneReport), _vp, _sz, _vp]
    L.krr_tune_cache_save.restype = _i32
    L.krr_tune_cache_save.argtypes = [ctypes.c_char_p]
    L.krr_tune_cache_load.restype = _i32
    L.krr_tune_cache_load.argtypes = [ctypes.c_char_p]
    L.krr_tune_cache_clear.restype = None
    L.krr_tune_cache_size.restype = _i32
    L.krr_tune_digest.restype = ctypes.c_char_p
    L.krr_setup_many_workspace_bytes.restype = _sz
    L.krr_setup_many_workspace_bytes.argtypes = [ctypes.POINTER(SetupProblem), _i32, _i32]
    L.krr_setup_many.restype = _i32
    L.krr_setup_many.argtypes = [ctypes.POINTER(SetupProblem), _i32, _i32, _vp, _sz, _vp]
    L.krr_kernel_matmat_noalloc.restype = _i32
    L.krr_kernel_matmat_noalloc.argtypes = [_vp, _i64, _i64, _vp, _i64, _i64, _i64, _dbl, _dbl,
                                            _vp, _i64, _i64, _vp, _i64, _i32, _i32, _vp]
    L.krr_kernel_dsigma_inner.restype = _i32
    L.krr_kernel_dsigma_inner.argtypes = [_vp, _i64, _i64, _vp, _i64, _i64, _i64, _dbl, _vp, _i64,
                                          _i64, _vp, _i64, ctypes.POINTER(_dbl), _i32, _vp, _sz,
                                          _vp]
    L.krr_batch_plan_create.restype = _i32
    L.krr_batch_plan_create.argtypes = [ctypes.POINTER(BatchProblem), _i32,
                                        ctypes.POINTER(PCGOpts), ctypes.POINTER(_vp), _vp]
    L.krr_batch_solve.restype = _i32
    L.krr_batch_solve.argtypes = [_vp, ctypes.POINTER(BatchReport), _vp]
    L.krr_batch_plan_destroy.restype = None
    L.krr_batch_plan_destroy.argtypes = [_vp]
    _lib = L
    return L


EXPORTED = ["krr_workspace_bytes", "krr_last_error", "krr_version", "krr_pcg_defaults",
            "krr_features", "krr_precond_factor", "krr_precond_apply", "krr_kernel_matmat",
            "krr_pcg_solve",
            "krr_grad", "krr_kernel_dsigma_inner", "krr_kernel_matmat_noalloc",
            "krr_kernel_matmat_k", "krr_pcg_solve_k", "krr_tensorsketch", "krr_srht",
            "krr_gaussian_project", "krr_precond_test", "krr_adaptive_features",
            "krr_autotune_matmat", "krr_tune_cache_save", "krr_tune_cache_load",
            "krr_tune_cache_clear", "krr_tune_cache_size", "krr_tune_digest",
            "krr_setup_many", "krr_setup_many_workspace_bytes",
            "krr_batch_plan_create", "krr_batch_solve", "krr_batch_plan_destroy"]
NOALLOC_SCRATCH_BYTES = 64 << 20   # KRR_NOALLOC_SCRATCH_BYTES


def last_error() -> str:
    return lib().krr_last_error().decode()


def version() -> str:
    return lib().krr_version().decode()


def workspace_bytes(op: int, n1: int, n2: int, d: int, s: int, m: int, prec: int) -> int:
    return int(lib().krr_workspace_bytes(op, n1, n2, d, s, m, prec))


def _prec(p) -> int:
    return PREC[p] if isinstance(p, str) else int(p)


def _stream() -> int:
    return torch.cuda.current_stream().cuda_stream


def _check(t: torch.Tensor, dtype, name: str, cols: int | None = None):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a device tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if t.dim() == 2 and t.shape[1] > 1 and t.stride(1) != 1:
        raise ValueError(f"{name} must be row-major with unit column stride")
    if cols is not None and t.shape[-1] != cols:
        raise ValueError(f"{name} has {t.shape[-1]} columns, expected {cols}")


def _ld(t: torch.Tensor) -> int:
    if t.dim() != 2:
        return 1
    return max(t.stride(0), t.shape[1])


def _ws(nbytes: int, device) -> torch.Tensor:
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)


def _raise(status: int, report=None, info: int = 0):
    if status != OK:
        raise KRRError(status, last_error(), report, info)


# ---------------------------------------------------------------- entry points
def features(X: torch.Tensor, W: torch.Tensor, b: torch.Tensor) -> torch.Tensor:
    """Z = sqrt(2/s) cos(X W + b) (n x s, FP32)."""
    _check(X, torch.float32, "X")
    _check(W, torch.float32, "W")
    _check(b, torch.float32, "b")
    n, d = X.shape
    s = W.shape[1]
    if W.shape[0] != d or W.stride(0) != s or b.numel() != s:
        raise ValueError("W must be d x s contiguous and b of length s")
    Z = torch.empty((n, s), dtype=torch.float32, device=X.device)
    ws = _ws(workspace_bytes(OP_FEATURES, n, n, d, s, 0, 1), X.device)
    st = lib().krr_features(X.data_ptr(), n, d, _ld(X), W.data_ptr(), b.data_ptr(), s,
                            Z.data_ptr(), s, ws.data_ptr(), ws.numel(), _stream())
    _raise(st)
    return Z


def precond_factor(Z: torch.Tensor, lambda_p: float):
    """(C, Ut) with C C^T = Z^T Z + lambda_p I (FP64 s x s) and Ut = Z C^{-T} (FP32 n x s)."""
    _check(Z, torch.float32, "Z")
    n, s = Z.shape
    C = torch.empty((s, s), dtype=torch.float64, device=Z.device)
    Ut = torch.empty((n, s), dtype=torch.float32, device=Z.device)
    ws = _ws(workspace_bytes(OP_PRECOND_FACTOR, n, n, 0, s, 0, 1), Z.device)
    info = _i64(0)
    st = lib().krr_precond_factor(Z.data_ptr(), n, s, _ld(Z), float(lambda_p), C.data_ptr(),
                                  Ut.data_ptr(), s, ws.data_ptr(), ws.numel(), ctypes.byref(info),
                                  _stream())
    _raise(st, info=info.value)
    return C, Ut


def precond_apply(Ut: torch.Tensor, lambda_p: float, R: torch.Tensor) -> torch.Tensor:
    """(Z Z^T + lambda_p I)^{-1} R = (R - Ut (Ut^T R)) / lambda_p (FP64 R and result)."""
    _check(Ut, torch.float32, "Ut")
    vec = R.dim() == 1
    R2 = R[:, None] if vec else R
    _check(R2, torch.float64, "R")
    n, s = Ut.shape
    m = R2.shape[1]
    if R2.shape[0] != n:
        raise ValueError("R rows must match Ut")
    out = torch.empty((n, m), dtype=torch.float64, device=Ut.device)
    ws = _ws(workspace_bytes(OP_PRECOND_APPLY, n, n, 0, s, m, 0), Ut.device)
    st = lib().krr_precond_apply(Ut.data_ptr(), n, s, _ld(Ut), float(lambda_p), R2.data_ptr(), m,
                                 _ld(R2), out.data_ptr(), m, ws.data_ptr(), ws.numel(), _stream())
    _raise(st)
    return out[:, 0] if vec else out


def kernel_matmat_k(kernel: "Kernel", X1: torch.Tensor, X2: torch.Tensor, V: torch.Tensor,
                    shift: float = 0.0, deriv: bool = False, prec="f16x3",
                    out: torch.Tensor | None = None) -> torch.Tensor:
    """OUT = K(X1, X2) V + shift V for a kernel descriptor (krr_kernel_matmat_k)."""
    _check(X1, torch.float32, "X1")
    _check(X2, torch.float32, "X2")
    vec = V.dim() == 1
    V2 = V[:, None] if vec else V
    _check(V2, torch.float64, "V")
    n1, d = X1.shape
    n2 = X2.shape[0]
    m = V2.shape[1]
    if X2.shape[1] != d or V2.shape[0] != n2:
        raise ValueError("shape mismatch")
    if out is None:
        out = torch.empty((n1, m), dtype=torch.float64, device=X1.device)
    p = _prec(prec)
    ws = _ws(workspace_bytes(OP_KERNEL_MATMAT, n1, n2, d, 0, m, p), X1.device)
    st = lib().krr_kernel_matmat_k(ctypes.byref(kernel), X1.data_ptr(), n1, _ld(X1), X2.data_ptr(),
                                   n2, _ld(X2), d, float(shift), V2.data_ptr(), m, _ld(V2),
                                   out.data_ptr(), _ld(out), int(bool(deriv)), p, ws.data_ptr(),
                                   ws.numel(), _stream())
    _raise(st)
    return out[:, 0] if vec else out


def tensorsketch(X: torch.Tensor, gamma: float, coef0: float, degree: int, hash_: torch.Tensor,
                 sign: torch.Tensor, s: int, out: torch.Tensor | None = None) -> torch.Tensor:
    """TensorSketch features (krr_tensorsketch) of [sqrt(gamma) x, sqrt(c)]: n x s FP32.
    hash_: q x (d + 1) int32, sign: q x (d + 1) FP32 of +-1 (device tensors)."""
    _check(X, torch.float32, "X")
    n, d = X.shape
    h = hash_.to(torch.int32) if hash_.dtype != torch.int32 else hash_
    _check(h, torch.int32, "hash")
    _check(sign, torch.float32, "sign")
    if tuple(h.shape) != (int(degree), d + 1) or tuple(sign.shape) != (int(degree), d + 1):
        raise ValueError("hash and sign must be degree x (d + 1)")
    if not h.is_contiguous() or not sign.is_contiguous():
        raise ValueError("hash and sign must be contiguous")
    if out is None:
        out = torch.empty((n, int(s)), dtype=torch.float32, device=X.device)
    _check(out, torch.float32, "out")
    st = lib().krr_tensorsketch(X.data_ptr(), n, d, _ld(X), float(gamma), float(coef0),
                                int(degree), h.data_ptr(), sign.data_ptr(), int(s),
                                out.data_ptr(), _ld(out), _stream())
    _raise(st)
    return out


def srht(Z1: torch.Tensor, signs: torch.Tensor, sample: torch.Tensor,
         out: torch.Tensor | None = None) -> torch.Tensor:
    """Z2 = Z1 S^T, S = s2^{-1/2} P H D (krr_srht); signs: s1 FP32 +-1, sample: s2 int32."""
    _check(Z1, torch.float32, "Z1")
    n, s1 = Z1.shape
    smp = sample.to(torch.int32) if sample.dtype != torch.int32 else sample
    _check(smp, torch.int32, "sample")
    _check(signs, torch.float32, "signs")
    if signs.numel() != s1 or not signs.is_contiguous() or not smp.is_contiguous():
        raise ValueError("signs must hold s1 values; signs and sample must be contiguous")
    s2 = smp.numel()
    if out is None:
        out = torch.empty((n, s2), dtype=torch.float32, device=Z1.device)
    _check(out, torch.float32, "out")
    st = lib().krr_srht(Z1.data_ptr(), n, s1, _ld(Z1), signs.data_ptr(), smp.data_ptr(), s2,
                        out.data_ptr(), _ld(out), _stream())
    _raise(st)
    return out


def gaussian_project(Z2: torch.Tensor, S3: torch.Tensor,
                     out: torch.Tensor | None = None) -> torch.Tensor:
    """Z3 = s3^{-1/2} Z2 S3^T (krr_gaussian_project); S3: s3 x s2 FP32, N(0, 1) entries."""
    _check(Z2, torch.float32, "Z2")
    _check(S3, torch.float32, "S3")
    n, s2 = Z2.shape
    s3 = S3.shape[0]
    if S3.shape[1] != s2 or not S3.is_contiguous():
        raise ValueError("S3 must be a contiguous s3 x s2 matrix")
    if out is None:
        out = torch.empty((n, s3), dtype=torch.float32, device=Z2.device)
    _check(out, torch.float32, "out")
    ws = _ws(workspace_bytes(OP_GAUSSIAN_PROJECT, n, n, s2, s3, 0, 1), Z2.device)
    st = lib().krr_gaussian_project(Z2.data_ptr(), n, s2, _ld(Z2), S3.data_ptr(), s3,
                                    out.data_ptr(), _ld(out), ws.data_ptr(), ws.numel(), _stream())
    _raise(st)
    return out


def setup_many(problems: list, nstreams: int = 4) -> list:
    """Features and factor for many problems at once (krr_setup_many). Each problem is a dict
    with X, W, b, lam (lambda_p); returns [(Z, C, Ut), ...] in the same order."""
    arr = (SetupProblem * len(problems))()
    keep = []
    for i, pr in enumerate(problems):
        X, W, b = pr["X"], pr["W"], pr["b"]
        _check(X, torch.float32, "X")
        _check(W, torch.float32, "W")
        _check(b, torch.float32, "b")
        n, d = X.shape
        s = W.shape[1]
        if W.shape[0] != d or not W.is_contiguous() or b.numel() != s:
            raise ValueError("W must be a contiguous d x s matrix and b hold s values")
        Z = torch.empty((n, s), dtype=torch.float32, device=X.device)
        C = torch.empty((s, s), dtype=torch.float64, device=X.device)
        Ut = torch.empty((n, s), dtype=torch.float32, device=X.device)
        arr[i] = SetupProblem(X.data_ptr(), n, d, _ld(X), W.data_ptr(), b.data_ptr(), s,
                              float(pr["lam"]), Z.data_ptr(), s, C.data_ptr(), Ut.data_ptr(), s, 0)
        keep.append((Z, C, Ut))
    nb = lib().krr_setup_many_workspace_bytes(arr, len(problems), int(nstreams))
    ws = _ws(nb, problems[0]["X"].device)
    st = lib().krr_setup_many(arr, len(problems), int(nstreams), ws.data_ptr(), ws.numel(),
                              _stream())
    _raise(st, info=max(int(arr[i].info) for i in range(len(problems))))
    return keep


def autotune_matmat(kernel: "Kernel", X: torch.Tensor, m: int, prec="f16x3") -> TuneReport:
    """Time the product's launch candidates for K(X, X) V with m columns and store the best
    in the library's tuning table (krr_autotune_matmat)."""
    _check(X, torch.float32, "X")
    n, d = X.shape
    p = _prec(prec)
    ws = _ws(workspace_bytes(OP_AUTOTUNE, n, n, d, 0, int(m), p), X.device)
    rep = TuneReport()
    st = lib().krr_autotune_matmat(ctypes.byref(kernel), X.data_ptr(), n, d, _ld(X), int(m), p,
                                   ctypes.byref(rep), ws.data_ptr(), ws.numel(), _stream())
    _raise(st)
    return rep


def tune_cache_save(path: str) -> bool:
    return bool(lib().krr_tune_cache_save(path.encode()))


def tune_cache_load(path: str) -> bool:
    return bool(lib().krr_tune_cache_load(path.encode()))


def tune_cache_clear() -> None:
    lib().krr_tune_cache_clear()


def tune_cache_size() -> int:
    return int(lib().krr_tune_cache_size())


def tune_digest() -> str:
    return lib().krr_tune_digest().decode()


def precond_test(kernel: "Kernel", X: torch.Tensor, Z: torch.Tensor, lam: float,
                 power_iters: int = 40, prec="f16x3") -> PrecondTestReport:
    """The Thm. 4 test of a candidate sketch Z (krr_precond_test)."""
    _check(X, torch.float32, "X")
    _check(Z, torch.float32, "Z")
    n, d = X.shape
    s = Z.shape[1]
    if Z.shape[0] != n:
        raise ValueError("Z rows must match X")
    p = _prec(prec)
    ws = _ws(workspace_bytes(OP_PRECOND_TEST, n, n, d, s, 0, p), X.device)
    rep = PrecondTestReport()
    st = lib().krr_precond_test(ctypes.byref(kernel), X.data_ptr(), n, d, _ld(X), Z.data_ptr(), s,
                                _ld(Z), float(lam), int(power_iters), p, ctypes.byref(rep),
                                ws.data_ptr(), ws.numel(), _stream())
    _raise(st)
    return rep


def adaptive_features(kernel: "Kernel", X: torch.Tensor, lam: float, s0: int, s_max: int,
                      W: torch.Tensor | None = None, b: torch.Tensor | None = None,
                      hash_: torch.Tensor | None = None, sign: torch.Tensor | None = None,
                      power_iters: int = 40, prec="f16x3"):
    """Sec. 5 doubling rule (krr_adaptive_features). Returns (Z[:, :s], s, history)."""
    _check(X, torch.float32, "X")
    n, d = X.shape
    ptrs = []
    for t, name, dt in ((W, "W", torch.float32), (b, "b", torch.float32),
                        (hash_, "hash", torch.int32), (sign, "sign", torch.float32)):
        if t is not None:
            _check(t, dt, name)
            if not t.is_contiguous():
                raise ValueError(f"{name} must be contiguous")
        ptrs.append(t.data_ptr() if t is not None else None)
    Z = torch.empty((n, int(s_max)), dtype=torch.float32, device=X.device)
    p = _prec(prec)
    ws = _ws(workspace_bytes(OP_ADAPTIVE_FEATURES, n, n, d, int(s_max), 0, p), X.device)
    cap = 32
    hist = (PrecondTestReport * cap)()
    hlen = _i32(0)
    s_out = _i64(0)
    st = lib().krr_adaptive_features(ctypes.byref(kernel), X.data_ptr(), n, d, _ld(X), float(lam),
                                     ptrs[0], ptrs[1], ptrs[2], ptrs[3], int(s0), int(s_max),
                                     Z.data_ptr(), _ld(Z), ctypes.byref(s_out), hist, cap,
                                     ctypes.byref(hlen), int(power_iters), p, ws.data_ptr(),
                                     ws.numel(), _stream())
    _raise(st)
    s = int(s_out.value)
    return Z[:, :s], s, [hist[i].as_dict() for i in range(min(hlen.value, cap))]


def kernel_matmat(X1: torch.Tensor, X2: torch.Tensor, sigma: float, V: torch.Tensor,
                  shift: float = 0.0, deriv: bool = False, prec="f16x3",
                  out: torch.Tensor | None = None) -> torch.Tensor:
    """OUT = K(X1, X2) V + shift V (deriv: dK/dsigma instead of K). FP64 V and OUT."""
    _check(X1, torch.float32, "X1")
    _check(X2, torch.float32, "X2")
    vec = V.dim() == 1
    V2 = V[:, None] if vec else V
    _check(V2, torch.float64, "V")
    n1, d = X1.shape
    n2 = X2.shape[0]
    m = V2.shape[1]
    if X2.shape[1] != d or V2.shape[0] != n2:
        raise ValueError("shape mismatch")
    if out is None:
        out = torch.empty((n1, m), dtype=torch.float64, device=X1.device)
    p = _prec(prec)
    ws = _ws(workspace_bytes(OP_KERNEL_MATMAT, n1, n2, d, 0, m, p), X1.device)
    st = lib().krr_kernel_matmat(X1.data_ptr(), n1, _ld(X1), X2.data_ptr(), n2, _ld(X2), d,
                                 float(sigma), float(shift), V2.data_ptr(), m, _ld(V2),
                                 out.data_ptr(), _ld(out), int(bool(deriv)), p, ws.data_ptr(),
                                 ws.numel(), _stream())
    _raise(st)
    return out[:, 0] if vec else out


def kernel_matmat_noalloc(X1: torch.Tensor, X2: torch.Tensor, sigma: float, V: torch.Tensor,
                          out: torch.Tensor, shift: float = 0.0, deriv: bool = False,
                          prec="f16x3") -> torch.Tensor:
    """kernel_matmat through the allocation-free entry point: the library's fixed per-GPU
    scratch array instead of a workspace; `out` (n1 x m FP64) is caller-provided, so this
    call allocates no device memory."""
    _check(X1, torch.float32, "X1")
    _check(X2, torch.float32, "X2")
    vec = V.dim() == 1
    V2 = V[:, None] if vec else V
    O2 = out[:, None] if out.dim() == 1 else out
    _check(V2, torch.float64, "V")
    _check(O2, torch.float64, "out")
    n1, d = X1.shape
    n2 = X2.shape[0]
    m = V2.shape[1]
    if X2.shape[1] != d or V2.shape[0] != n2 or tuple(O2.shape) != (n1, m):
        raise ValueError("shape mismatch")
    st = lib().krr_kernel_matmat_noalloc(X1.data_ptr(), n1, _ld(X1), X2.data_ptr(), n2, _ld(X2),
                                         d, float(sigma), float(shift), V2.data_ptr(), m, _ld(V2),
                                         O2.data_ptr(), _ld(O2), int(bool(deriv)), _prec(prec),
                                         _stream())
    _raise(st)
    return out


@dataclasses.dataclass
class SolveReport:
    status: int
    iters: int
    converged_cols: int
    breakdown_cols: int
    refine_steps: int
    relres_rec: list
    relres_true: list
    history: list
    matmat_calls: int = 0
    matmat_ms: float = 0.0


def pcg_solve_k(kernel: "Kernel", X: torch.Tensor, lam: float, Ut: torch.Tensor | None,
                Y: torch.Tensor, **kw):
    """pcg_solve for a kernel descriptor (krr_pcg_solve_k). Returns (alpha, SolveReport)."""
    return pcg_solve(X, None, lam, Ut, Y, kernel=kernel, **kw)


def pcg_solve(X: torch.Tensor, sigma: float | None, lam: float, Ut: torch.Tensor | None,
              Y: torch.Tensor, tol: float = 1e-6, max_iter: int = 1000, prec="f16x3",
              use_precond: bool = True, lambda_p: float | None = None, check_every: int = 1,
              true_residual: bool = True, refine: int = 0, alpha0: torch.Tensor | None = None,
              raise_on_error: bool = True, history_cap: int = 4096,
              kernel: "Kernel | None" = None):
    """Solve (K + lam I) alpha = Y by PCG (Gaussian kernel of bandwidth sigma, or `kernel`).
    Returns (alpha, SolveReport)."""
    _check(X, torch.float32, "X")
    vec = Y.dim() == 1
    Y2 = Y[:, None] if vec else Y
    _check(Y2, torch.float64, "Y")
    n, d = X.shape
    m = Y2.shape[1]
    if Y2.shape[0] != n:
        raise ValueError("Y rows must match X")
    if use_precond:
        if Ut is None:
            raise ValueError("use_precond needs Ut")
        _check(Ut, torch.float32, "Ut")
        s, ldu, uptr = Ut.shape[1], _ld(Ut), Ut.data_ptr()
    else:
        s, ldu, uptr = 0, 0, None
    p = _prec(prec)
    alpha = torch.zeros((n, m), dtype=torch.float64, device=X.device)
    if alpha0 is not None:
        alpha.copy_(alpha0.reshape(n, m))
    opts = PCGOpts()
    lib().krr_pcg_defaults(ctypes.byref(opts))
    opts.tol, opts.max_iter, opts.prec = float(tol), int(max_iter), p
    opts.use_precond, opts.check_every = int(bool(use_precond)), int(check_every)
    opts.lambda_p = float(lambda_p) if lambda_p else 0.0
    opts.true_residual, opts.refine = int(bool(true_residual)), int(refine)
    opts.warm_start = int(alpha0 is not None)
    rec = (_dbl * m)()
    tru = (_dbl * m)()
    hist = (_dbl * history_cap)()
    rep = PCGReport()
    rep.relres_rec = ctypes.cast(rec, ctypes.POINTER(_dbl))
    rep.relres_true = ctypes.cast(tru, ctypes.POINTER(_dbl))
    rep.history = ctypes.cast(hist, ctypes.POINTER(_dbl))
    rep.history_cap = history_cap
    ws = _ws(workspace_bytes(OP_PCG_SOLVE, n, n, d, s, m, p), X.device)
    if kernel is None:
        st = lib().krr_pcg_solve(X.data_ptr(), n, d, _ld(X), float(sigma), float(lam), uptr, s,
                                 ldu, Y2.data_ptr(), _ld(Y2), alpha.data_ptr(), m, m,
                                 ctypes.byref(opts), ctypes.byref(rep), ws.data_ptr(), ws.numel(),
                                 _stream())
    else:
        st = lib().krr_pcg_solve_k(ctypes.byref(kernel), X.data_ptr(), n, d, _ld(X), float(lam),
                                   uptr, s, ldu, Y2.data_ptr(), _ld(Y2), alpha.data_ptr(), m, m,
                                   ctypes.byref(opts), ctypes.byref(rep), ws.data_ptr(),
                                   ws.numel(), _stream())
    report = SolveReport(st, rep.iters, rep.converged_cols, rep.breakdown_cols, rep.refine_steps,
                         [rec[i] for i in range(m)], [tru[i] for i in range(m)],
                         [hist[i] for i in range(rep.history_len)], rep.matmat_calls,
                         rep.matmat_ms)
    if raise_on_error and st not in (OK,):
        if st in (E_NO_CONV, E_BREAKDOWN):
            raise KRRError(st, last_error(), report)
        _raise(st, report)
    return (alpha[:, 0] if vec else alpha), report


def grad(X: torch.Tensor, sigma: float, alpha: torch.Tensor, abar: torch.Tensor, prec="f16x3"):
    """(-<abar, dK/dsigma alpha>, -<abar, alpha>)."""
    _check(X, torch.float32, "X")
    a2 = alpha[:, None] if alpha.dim() == 1 else alpha
    b2 = abar[:, None] if abar.dim() == 1 else abar
    _check(a2, torch.float64, "alpha")
    _check(b2, torch.float64, "abar")
    if a2.shape != b2.shape or a2.stride() != b2.stride():
        raise ValueError("alpha and abar must have the same shape and layout")
    n, d = X.shape
    m = a2.shape[1]
    p = _prec(prec)
    ws = _ws(workspace_bytes(OP_GRAD, n, n, d, 0, m, p), X.device)
    ds, dl = _dbl(0.0), _dbl(0.0)
    st = lib().krr_grad(X.data_ptr(), n, d, _ld(X), float(sigma), a2.data_ptr(), b2.data_ptr(), m,
                        _ld(a2), ctypes.byref(ds), ctypes.byref(dl), p, ws.data_ptr(), ws.numel(),
                        _stream())
    _raise(st)
    return ds.value, dl.value


def kernel_dsigma_inner(X1: torch.Tensor, X2: torch.Tensor, sigma: float, V: torch.Tensor,
                        G: torch.Tensor, prec="fp64") -> float:
    """<G, (dK(X1, X2)/dsigma) V> in FP64 (the direct sigma-term of a loss on K(X1, X2) V)."""
    _check(X1, torch.float32, "X1")
    _check(X2, torch.float32, "X2")
    V2 = V[:, None] if V.dim() == 1 else V
    G2 = G[:, None] if G.dim() == 1 else G
    _check(V2, torch.float64, "V")
    _check(G2, torch.float64, "G")
    n1, d = X1.shape
    n2 = X2.shape[0]
    m = V2.shape[1]
    if X2.shape[1] != d or V2.shape[0] != n2 or tuple(G2.shape) != (n1, m):
        raise ValueError("shape mismatch")
    p = _prec(prec)
    ws = _ws(workspace_bytes(OP_DSIGMA_INNER, n1, n2, d, 0, m, p), X1.device)
    out = _dbl(0.0)
    st = lib().krr_kernel_dsigma_inner(X1.data_ptr(), n1, _ld(X1), X2.data_ptr(), n2, _ld(X2), d,
                                       float(sigma), V2.data_ptr(), m, _ld(V2), G2.data_ptr(),
                                       _ld(G2), ctypes.byref(out), p, ws.data_ptr(), ws.numel(),
                                       _stream())
    _raise(st)
    return out.value


@dataclasses.dataclass
class BatchSolveReport:
    status: int
    iters: int
    converged_cols: int
    breakdown_cols: int
    refine_steps: int
    relres_rec: list       # per problem: list of its m columns
    relres_true: list
    col_iters: list        # per problem: iterations of each column (first solve)
    product_ms: float
    iteration_ms: float
    tiles_per_item: int
    work_items: int


class BatchPlan:
    """Many independent problems (K_p + lam_p I) alpha_p = Y_p solved together: one persistent
    kernel-product launch per PCG iteration, check_every iterations per replayed graph (one
    host read of the active count per replay).

    problems: list of dicts with keys X (n x d FP32), sigma, lam, Y (n x m FP64, m <= 16) and
    optionally Ut (n x s FP32) and lambda_p. The plan keeps references to every tensor and
    owns the solutions (``alphas``). Points are prepared at construction."""

    def __init__(self, problems, tol: float = 1e-6, max_iter: int = 1000,
                 use_precond: bool = True, check_every: int = 4, true_residual: bool = True,
                 refine: int = 0):
        self._keep = []
        n_p = len(problems)
        arr = (BatchProblem * n_p)()
        self.alphas = []
        self.ms = []
        for i, pr in enumerate(problems):
            X, Y = pr["X"], pr["Y"]
            _check(X, torch.float32, f"problems[{i}].X")
            Y2 = Y[:, None] if Y.dim() == 1 else Y
            _check(Y2, torch.float64, f"problems[{i}].Y")
            n, d = X.shape
            m = Y2.shape[1]
            if Y2.shape[0] != n:
                raise ValueError(f"problems[{i}]: Y rows must match X")
            alpha = torch.zeros((n, m), dtype=torch.float64, device=X.device)
            Ut = pr.get("Ut")
            b = arr[i]
            b.X, b.n, b.d, b.ldx = X.data_ptr(), n, d, _ld(X)
            b.sigma, b.lam = float(pr["sigma"]), float(pr["lam"])
            b.lambda_p = float(pr.get("lambda_p") or 0.0)
            if Ut is not None:
                _check(Ut, torch.float32, f"problems[{i}].Ut")
                b.Ut, b.s, b.ldu = Ut.data_ptr(), Ut.shape[1], _ld(Ut)
            else:
                b.Ut, b.s, b.ldu = None, 0, 0
            b.Y, b.ldy = Y2.data_ptr(), _ld(Y2)
            b.alpha, b.lda, b.m = alpha.data_ptr(), m, m
            self._keep += [X, Y2, Ut]
            self.alphas.append(alpha)
            self.ms.append(m)
        opts = PCGOpts()
        lib().krr_pcg_defaults(ctypes.byref(opts))
        opts.tol, opts.max_iter, opts.prec = float(tol), int(max_iter), PREC["f16x3"]
        opts.use_precond, opts.check_every = int(bool(use_precond)), int(check_every)
        opts.true_residual, opts.refine = int(bool(true_residual)), int(refine)
        self._problems = arr
        self._handle = _vp(None)
        st = lib().krr_batch_plan_create(arr, n_p, ctypes.byref(opts), ctypes.byref(self._handle),
                                         _stream())
        _raise(st)
        self.count = n_p

    def solve(self, raise_on_error: bool = True):
        """Run PCG on every problem; returns (alphas, BatchSolveReport)."""
        if not self._handle:
            raise RuntimeError("plan destroyed")
        k = self.count * BATCH_MAX_M
        rec, tru, cit = (_dbl * k)(), (_dbl * k)(), (_i32 * k)()
        rep = BatchReport()
        rep.relres_rec = ctypes.cast(rec, ctypes.POINTER(_dbl))
        rep.relres_true = ctypes.cast(tru, ctypes.POINTER(_dbl))
        rep.col_iters = ctypes.cast(cit, ctypes.POINTER(_i32))
        st = lib().krr_batch_solve(self._handle, ctypes.byref(rep), _stream())
        per = lambda a: [[a[i * BATCH_MAX_M + c] for c in range(m)] for i, m in enumerate(self.ms)]
        report = BatchSolveReport(st, rep.iters, rep.converged_cols, rep.breakdown_cols,
                                  rep.refine_steps, per(rec),
                                  per(tru), per(cit), rep.product_ms, rep.iteration_ms, rep.tiles_per_item,
                                  rep.work_items)
        if raise_on_error and st != OK:
            raise KRRError(st, last_error(), report)
        return self.alphas, report

    def close(self):
        if self._handle:
            lib().krr_batch_plan_destroy(self._handle)
            self._handle = _vp(None)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

