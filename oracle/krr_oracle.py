"""Plain, slow, obviously correct CPU FP64 oracle.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, the smoke check and the CPU-baseline
leg of ``bench.py``; never by the product path, and it imports nothing from it.

Every function follows a passage of Avron, Clarkson, Woodruff, "Faster Kernel Ridge
Regression Using Sketching and Preconditioning" (arXiv 1611.03220), cited in its
docstring. Arithmetic is FP64 throughout. The Gaussian kernel is formed from the
*difference* form sum_k (x_ik - z_k)^2, deliberately not the norm expansion the GPU
path uses, so the two share no arithmetic.

Readings of the paper taken here (each is also listed in the design notes):
  * RFF scale: sqrt(2/s), so that E[z(x)^T z(y)] = k(x, y) holds exactly (the printed
    s^{-1/2} is off by the factor 2 that the identity E[2 cos(a+b) cos(c+b)] = cos(a-c)
    needs). Offsets b are drawn per feature (b in R^s).
  * Cholesky convention: lower C with C C^T = Z^T Z + lambda_p I and U = C^{-1} Z^T, so
    U^T U = Z (Z^T Z + lambda_p I)^{-1} Z^T, which is what the Woodbury form needs and
    does not depend on the convention.
  * Preconditioner regulariser lambda_p is a parameter (default lambda, Alg. 1; Table 2
    varies it).
  * PCG: the standard method (Shewchuk's form, which the paper cites for its bound),
    started from zero (Thm. 1), stopped on the recursive residual
    ||r_j|| <= tol ||y_j|| for every right-hand side (Sec. 6), columns independent and
    frozen once converged.
  * Squared distances are formed as sums of squared coordinate differences, which are
    never negative, so no clamp at zero is needed or applied.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np
import scipy.linalg as sla

__all__ = [
    "sq_dists", "gaussian_kernel", "gaussian_kernel_dsigma", "kernel_matmat",
    "krr_solve_dense", "rff_features", "NotSPDError", "precond_factor", "precond_apply",
    "PCGResult", "pcg", "krr_pcg", "relres_true", "statistical_dimension",
    "preconditioned_spectrum", "cg_iteration_bound", "validation_loss_and_grads",
    "rfm_weights", "STATUS_OK", "STATUS_NO_CONV", "STATUS_BREAKDOWN",
]

STATUS_OK = 0
STATUS_NO_CONV = 3
STATUS_BREAKDOWN = 4


# --------------------------------------------------------------------------- kernel
def sq_dists(X1: np.ndarray, X2: np.ndarray, block: int = 256) -> np.ndarray:
    """Squared Euclidean distances D_ij = sum_k (x1_ik - x2_jk)^2 in FP64.

    Difference form, evaluated block by block (Sec. 6 defines the Gaussian kernel on
    ||x - z||^2). The block of rows is capped so the difference array stays near 2^24
    elements.
    """
    X1 = np.asarray(X1, np.float64)
    X2 = np.asarray(X2, np.float64)
    block = max(1, min(block, (1 << 24) // max(1, X2.shape[0] * X2.shape[1])))
    D = np.empty((X1.shape[0], X2.shape[0]))
    for a in range(0, X1.shape[0], block):
        diff = X1[a:a + block, None, :] - X2[None, :, :]
        D[a:a + block] = np.einsum("ijk,ijk->ij", diff, diff)
    return D


def gaussian_kernel(X1, X2, sigma: float) -> np.ndarray:
    """K_ij = exp(-||x_i - z_j||^2 / (2 sigma^2)): the Gaussian kernel of Sec. 6."""
    return np.exp(-sq_dists(X1, X2) / (2.0 * sigma * sigma))


def gaussian_kernel_dsigma(X1, X2, sigma: float) -> np.ndarray:
    """dK/dsigma = K * ||x - z||^2 / sigma^3 (derivative of the Sec. 6 kernel)."""
    D = sq_dists(X1, X2)
    return np.exp(-D / (2.0 * sigma * sigma)) * D / sigma ** 3


def kernel_matmat(X1, X2, sigma: float, V, shift: float = 0.0, deriv: bool = False,
                  rows=None, block: int = 512) -> np.ndarray:
    """OUT = K(X1, X2) V + shift * V, matrix-free over row blocks of X1.

    The per-iteration product of the PCG in Alg. 1 (the dominant cost, Sec. 3.1), with
    K never stored whole. ``deriv`` swaps K for dK/dsigma. ``rows`` restricts the
    output to the given rows of X1 (for sampled checks at large n). ``shift`` is only
    meaningful for the square case X1 == X2 (it adds lambda * V for K + lambda I).
    """
    X1 = np.asarray(X1, np.float64)
    X2 = np.asarray(X2, np.float64)
    V = np.asarray(V, np.float64)
    vec = V.ndim == 1
    if vec:
        V = V[:, None]
    idx = np.arange(X1.shape[0]) if rows is None else np.asarray(rows)
    out = np.empty((idx.shape[0], V.shape[1]))
    for a in range(0, idx.shape[0], block):
        ii = idx[a:a + block]
        Kb = (gaussian_kernel_dsigma if deriv else gaussian_kernel)(X1[ii], X2, sigma)
        out[a:a + block] = Kb @ V
        if shift:
            out[a:a + block] += shift * V[ii]
    return out[:, 0] if vec else out


def krr_solve_dense(X, sigma: float, lam: float, Y) -> np.ndarray:
    """c = (K + lambda I_n)^{-1} y by dense Cholesky (Eq. 1; lambda > 0 is assumed)."""
    K = gaussian_kernel(X, X, sigma)
    K[np.diag_indices_from(K)] += lam
    return sla.cho_solve(sla.cho_factor(K, lower=True), np.asarray(Y, np.float64))


# ---------------------------------------------------------------- random features
def rff_features(X, W, b) -> np.ndarray:
    """Z = sqrt(2/s) cos(X W + b): random Fourier features (Sec. 2.2), rows z_i.

    W is d x s with columns w_l ~ N(0, sigma^-2 I), b in [0, 2 pi)^s; both are drawn by
    the caller and passed in.
    """
    W = np.asarray(W, np.float64)
    s = W.shape[1]
    return math.sqrt(2.0 / s) * np.cos(np.asarray(X, np.float64) @ W + np.asarray(b, np.float64)[None, :])


def rfm_weights(Z, Y, lam: float) -> np.ndarray:
    """w = (Z^T Z + lambda I_s)^{-1} Z^T y: the Random Features Method model (Sec. 2.2)."""
    Z = np.asarray(Z, np.float64)
    G = Z.T @ Z + lam * np.eye(Z.shape[1])
    return np.linalg.solve(G, Z.T @ np.asarray(Y, np.float64))


class NotSPDError(Exception):
    """Z^T Z + lambda_p I was not numerically positive definite; ``info`` is pivot+1."""

    def __init__(self, info: int):
        super().__init__(f"matrix not positive definite at pivot {info - 1}")
        self.info = info


def precond_factor(Z, lambda_p: float):
    """Preconditioner set-up of Alg. 1 (Sec. 3.1): G = Z^T Z + lambda_p I_s, lower C with C C^T = G, U = C^{-1} Z^T.

    Returns (C, U) with C s x s lower triangular and U s x n. Raises NotSPDError when
    G is not positive definite (only possible with lambda_p <= 0 or non-finite Z).
    """
    Z = np.asarray(Z, np.float64)
    G = Z.T @ Z
    G[np.diag_indices_from(G)] += lambda_p
    try:
        C = np.linalg.cholesky(G)
    except np.linalg.LinAlgError:
        # locate the first failing pivot by the leading-minor test
        for k in range(1, G.shape[0] + 1):
            try:
                np.linalg.cholesky(G[:k, :k])
            except np.linalg.LinAlgError:
                raise NotSPDError(k) from None
        raise NotSPDError(G.shape[0]) from None
    if not np.all(np.isfinite(C)):
        raise NotSPDError(1)
    U = sla.solve_triangular(C, Z.T, lower=True)
    return C, U


def precond_apply(U, lambda_p: float, R) -> np.ndarray:
    """(Z Z^T + lambda_p I_n)^{-1} R = lambda_p^{-1} (R - U^T (U R)) (Woodbury, Sec. 3.1)."""
    U = np.asarray(U, np.float64)
    R = np.asarray(R, np.float64)
    return (R - U.T @ (U @ R)) / lambda_p


# -------------------------------------------------------------------------- PCG
@dataclasses.dataclass
class PCGResult:
    x: np.ndarray           # n x m solution
    iters: int              # iterations taken (max over columns)
    relres: np.ndarray      # per-column recursive relative residual at exit
    converged: np.ndarray   # per-column bool
    status: int             # STATUS_OK / STATUS_NO_CONV / STATUS_BREAKDOWN
    col_iters: np.ndarray   # per-column iteration at which it converged (or stopped)
    history: list           # per-iteration max relative recursive residual over active columns


def pcg(apply_A, Y, apply_M=None, tol: float = 1e-6, max_iter: int = 1000, x0=None) -> PCGResult:
    """Preconditioned conjugate gradients on A x = y, one independent run per column.

    The solve of Alg. 1: (K + lambda I) c = y by PCG with a fixed SPD preconditioner,
    starting from zero (Thm. 1), stopping when ||y_j - A x_j|| <= tol ||y_j|| (tracked on
    the recursive residual) for every column (Sec. 6). Standard PCG: alpha = rho/<p, Ap>,
    beta = rho_new/rho. A column whose curvature <p, Ap> is not positive or not finite is
    frozen and reported as a breakdown.
    """
    Y = np.asarray(Y, np.float64)
    vec = Y.ndim == 1
    if vec:
        Y = Y[:, None]
    n, m = Y.shape
    M = apply_M if apply_M is not None else (lambda v: v.copy())
    x = np.zeros((n, m)) if x0 is None else np.array(x0, np.float64).reshape(n, m)
    r = Y - apply_A(x) if x0 is not None else Y.copy()
    ynorm = np.linalg.norm(Y, axis=0)
    r0n = np.linalg.norm(r, axis=0)
    broken = ~(np.isfinite(ynorm) & np.isfinite(r0n))  # non-finite data: breakdown at once
    active = ~broken & (r0n > tol * ynorm)
    col_iters = np.zeros(m, int)
    z = M(r)
    p = z.copy()
    rho = np.einsum("ij,ij->j", r, z)
    history = []
    it = 0
    while active.any() and it < max_iter:
        it += 1
        q = apply_A(p)
        pq = np.einsum("ij,ij->j", p, q)
        bad = active & ~(np.isfinite(pq) & (pq > 0))
        broken |= bad
        active &= ~bad
        a = np.where(active, rho / np.where(active, pq, 1.0), 0.0)
        x += a * p
        r -= a * q
        rn = np.linalg.norm(r, axis=0)
        col_iters[active] = it
        newly = active & (rn <= tol * ynorm)
        active &= ~newly
        history.append(float(np.max(np.where(np.isfinite(rn), rn, 0.0) / np.where(ynorm > 0, ynorm, 1.0))))
        if not active.any():
            break
        z = M(r)
        rho_new = np.einsum("ij,ij->j", r, z)
        beta = np.where(active, rho_new / np.where(active, rho, 1.0), 0.0)
        p = np.where(active, z + beta * p, p)
        rho = np.where(active, rho_new, rho)
    with np.errstate(invalid="ignore", divide="ignore"):
        relres = np.linalg.norm(r, axis=0) / np.where(ynorm > 0, ynorm, 1.0)
    converged = (relres <= tol) & ~broken
    status = STATUS_BREAKDOWN if broken.any() else (STATUS_OK if converged.all() else STATUS_NO_CONV)
    if vec:
        x = x[:, 0]
    return PCGResult(x, it, relres, converged, status, col_iters, history)


def krr_pcg(X, sigma: float, lam: float, Y, U=None, lambda_p=None, tol=1e-6, max_iter=1000,
            dense: bool = True, x0=None) -> PCGResult:
    """Alg. 1 end to end given U: PCG on (K + lambda I) c = y with M^{-1} from U.

    ``dense`` forms K once (small n); otherwise every product is matrix-free.
    ``U=None`` runs plain (unpreconditioned) CG, the baseline of Table 4.
    """
    X = np.asarray(X, np.float64)
    if dense:
        A = gaussian_kernel(X, X, sigma)
        A[np.diag_indices_from(A)] += lam
        apply_A = lambda v: A @ v  # noqa: E731
    else:
        apply_A = lambda v: kernel_matmat(X, X, sigma, v, shift=lam)  # noqa: E731
    lp = lam if lambda_p is None else lambda_p
    apply_M = None if U is None else (lambda v: precond_apply(U, lp, v))
    return pcg(apply_A, Y, apply_M, tol=tol, max_iter=max_iter, x0=x0)


def relres_true(X, sigma: float, lam: float, alpha, Y, rows=None) -> np.ndarray:
    """Per-column ||y - (K + lambda I) c|| / ||y|| in FP64 (the Sec. 6 stopping quantity).

    With ``rows`` given, both norms are taken over those rows only (a sampled check).
    """
    Y = np.asarray(Y, np.float64)
    alpha = np.asarray(alpha, np.float64)
    if Y.ndim == 1:
        Y, alpha = Y[:, None], alpha[:, None]
    Ax = kernel_matmat(X, X, sigma, alpha, rows=rows)
    idx = np.arange(Y.shape[0]) if rows is None else np.asarray(rows)
    Ax += lam * alpha[idx]
    return np.linalg.norm(Y[idx] - Ax, axis=0) / np.linalg.norm(Y[idx], axis=0)


# ------------------------------------------------------------------- diagnostics
def statistical_dimension(Kmat, lam: float) -> float:
    """s_lambda(K) = Tr((K + lambda I)^{-1} K) (Thm. 1)."""
    ev = np.linalg.eigvalsh(np.asarray(Kmat, np.float64))
    ev = np.clip(ev, 0.0, None)
    return float(np.sum(ev / (ev + lam)))


def preconditioned_spectrum(Kmat, lam: float, Z, lambda_p: float) -> np.ndarray:
    """Eigenvalues of (Z Z^T + lambda_p I)^{-1} (K + lambda I), via the symmetric form
    L^{-1} A L^{-T} with L L^T = Z Z^T + lambda_p I (dense; small n only)."""
    n = Kmat.shape[0]
    A = np.asarray(Kmat, np.float64) + lam * np.eye(n)
    Zf = np.asarray(Z, np.float64)
    Mm = Zf @ Zf.T + lambda_p * np.eye(n)
    L = np.linalg.cholesky(Mm)
    T = sla.solve_triangular(L, A, lower=True)
    T = sla.solve_triangular(L, T.T, lower=True)
    return np.linalg.eigvalsh(0.5 * (T + T.T))


def cg_iteration_bound(kappa: float, eps: float) -> int:
    """ceil(sqrt(kappa) ln(2/eps) / 2): CG iterations that reduce the A-norm error by eps
    when the (preconditioned) condition number is kappa (proof of Thm. 1)."""
    return int(math.ceil(math.sqrt(kappa) * math.log(2.0 / eps) / 2.0))


# ------------------------------------------------------------------ gradients
def validation_loss_and_grads(Xtr, Ytr, Xv, Yv, sigma: float, lam: float):
    """Validation loss L = 1/2 ||K_vt c - Y_v||_F^2 with c = (K + lambda I)^{-1} Y_tr,
    and its exact derivatives by the adjoint method, all with dense FP64 solves.

    dL/dlambda = -<abar, c>, dL/dsigma = <R, dK_vt/dsigma c> - <abar, dK/dsigma c>,
    where R = K_vt c - Y_v and abar = (K + lambda I)^{-1} K_vt^T R. The training solve is
    Eq. 1; the loss and its derivatives are not in the paper (they define the
    differentiation workload). Returns a dict with the loss, both gradients and the
    intermediate quantities.
    """
    Xtr = np.asarray(Xtr, np.float64)
    Xv = np.asarray(Xv, np.float64)
    Ytr = np.asarray(Ytr, np.float64)
    Yv = np.asarray(Yv, np.float64)
    K = gaussian_kernel(Xtr, Xtr, sigma)
    A = K.copy()
    A[np.diag_indices_from(A)] += lam
    cf = sla.cho_factor(A, lower=True)
    c = sla.cho_solve(cf, Ytr)
    Kvt = gaussian_kernel(Xv, Xtr, sigma)
    R = Kvt @ c - Yv
    loss = 0.5 * float(np.sum(R * R))
    abar = sla.cho_solve(cf, Kvt.T @ R)
    dK = gaussian_kernel_dsigma(Xtr, Xtr, sigma)
    dKvt = gaussian_kernel_dsigma(Xv, Xtr, sigma)
    dl_dlam = -float(np.sum(abar * c))
    dl_dsig = float(np.sum(R * (dKvt @ c))) - float(np.sum(abar * (dK @ c)))
    return {"loss": loss, "dL_dsigma": dl_dsig, "dL_dlambda": dl_dlam, "alpha": c,
            "abar": abar, "R": R,
            "dsigma_direct": float(np.sum(R * (dKvt @ c))),
            "dsigma_solve": -float(np.sum(abar * (dK @ c)))}
