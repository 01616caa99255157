"""Plain CPU FP64 oracle of the paper's sketching components.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, the smoke check and the CPU-baseline
leg of ``bench.py``; never by the product path, and it imports nothing from it.

Covers the polynomial kernel with TensorSketch features (Sec. 2.2, Thm. 1, the
polynomial workload of the Experiments section, Sec. 6), multiple-level sketching with a
subsampled randomized Walsh-Hadamard transform and a Gaussian projection (Def. 2,
Thm. 3, Alg. 2; Sec. 4) and the test of a candidate preconditioner that drives the
adaptive choice of the sketch size (Thm. 4; Sec. 5). FP64 throughout. Random choices
(hash functions, signs, sampled coordinates, Gaussian matrices) are inputs drawn by the
caller, so the oracle and the GPU path see the same sketch.

Readings of the paper taken here (each is also listed in the design notes):
  * TensorSketch hash: H(i_1..i_q) = (h_1(i_1) + ... + h_q(i_q)) mod s and sign
    G = g_1(i_1) g_2(i_2) ... g_q(i_q) (the printed "mod m" and "g_2(i_1)" are read as
    typos for s and g_2(i_2)). Fully random tables h_k: [d] -> [s], g_k: [d] -> {+1, -1}
    satisfy every k-wise independence the definition asks for.
  * Non-homogeneous polynomial kernel (gamma x^T z + c)^q: TensorSketch is applied to the
    augmented point [sqrt(gamma) x, sqrt(c)] (the remark after Thm. 1: one constant
    feature), so the sketch estimates the kernel without extra scaling.
  * SRHT: S = s^{-1/2} P H D with H the +-1 Walsh-Hadamard matrix of Def. 2 and P
    sampling s of the s1 coordinates uniformly without replacement. Every sampled
    coordinate is uniform, and ||H D x||^2 = s1 ||x||^2, so E||S x||^2 = ||x||^2 with this
    scale. A first-level sketch whose width is not a power of two is padded with zero
    columns to the next one (zero columns do not change Z Z^T).
  * Alg. 2 forms Z_3 = s_3^{-1/2} Z_2 S_3^T with S_3 standard normal, and the
    preconditioner is Z_3 Z_3^T + lambda I; its factor step reads Z as the last sketch
    (the printed algorithm has no separate Cholesky line for Z_3).
  * Thm. 4 condition 2 ("for all x, ||V_q^T P x||^2 = (1 +- 0.1) ||Z^T P x||^2") is
    evaluated exactly at small n: on the range of P the ratio's extremes are the
    extreme eigenvalues of Lambda^{-1/2} U_k^T K U_k Lambda^{-1/2}, where Z Z^T's
    eigenvectors above the threshold are U_k with eigenvalues Lambda.
"""
from __future__ import annotations

import itertools
import math

import numpy as np

__all__ = [
    "polynomial_kernel", "poly_kernel_matmat", "poly_solve_dense", "poly_augment",
    "count_sketch", "tensor_sketch_matrix", "monomials", "tensor_sketch_dense",
    "tensor_sketch_fft", "hadamard", "srht_matrix", "srht_apply", "gaussian_project",
    "precond_test", "adaptive_sketch_size",
]


# ------------------------------------------------------------------ polynomial kernel
def polynomial_kernel(X1, X2, gamma: float, coef0: float, degree: int) -> np.ndarray:
    """K_ij = (gamma <x_i, z_j> + c)^q: the polynomial kernel of the Experiments section
    (Sec. 6); gamma = 1, c = 0 is the homogeneous kernel of Sec. 2.2 and Thm. 1."""
    G = np.asarray(X1, np.float64) @ np.asarray(X2, np.float64).T
    return (gamma * G + coef0) ** int(degree)


def poly_kernel_matmat(X1, X2, gamma: float, coef0: float, degree: int, V,
                       shift: float = 0.0, rows=None, block: int = 512) -> np.ndarray:
    """OUT = K(X1, X2) V + shift V for the polynomial kernel, matrix-free over row blocks
    (the per-iteration product of the PCG in Alg. 1)."""
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
        out[a:a + block] = polynomial_kernel(X1[ii], X2, gamma, coef0, degree) @ V
        if shift:
            out[a:a + block] += shift * V[ii]
    return out[:, 0] if vec else out


def poly_solve_dense(X, gamma: float, coef0: float, degree: int, lam: float, Y) -> np.ndarray:
    """c = (K + lambda I)^{-1} y for the polynomial kernel (Eq. 1), dense solve."""
    K = polynomial_kernel(X, X, gamma, coef0, degree)
    K[np.diag_indices_from(K)] += lam
    return np.linalg.solve(K, np.asarray(Y, np.float64))


def poly_augment(X, gamma: float, coef0: float) -> np.ndarray:
    """Rows [sqrt(gamma) x, sqrt(c)]: <aug(x), aug(z)> = gamma x^T z + c, so the homogeneous
    degree-q kernel of the augmented points is the non-homogeneous kernel (remark after
    Thm. 1)."""
    X = np.asarray(X, np.float64)
    return np.hstack([math.sqrt(gamma) * X, np.full((X.shape[0], 1), math.sqrt(coef0))])


# ---------------------------------------------------------------------- TensorSketch
def count_sketch(x, h, g, s: int) -> np.ndarray:
    """CountSketch of one vector (Sec. 2.2): z_i = sum over j with h(j) = i of g(j) x_j."""
    z = np.zeros(s)
    for j in range(len(x)):
        z[int(h[j])] += float(g[j]) * float(x[j])
    return z


def monomials(x, q: int) -> np.ndarray:
    """v_q(x): all d^q degree-q monomials x_{i_1} ... x_{i_q}, indexed by (i_1, .., i_q) in
    lexicographic order (Sec. 2.2), so that <v_q(x), v_q(z)> = (x^T z)^q."""
    v = np.ones(1)
    for _ in range(q):
        v = np.kron(v, np.asarray(x, np.float64))
    return v


def tensor_sketch_matrix(h, g, s: int) -> np.ndarray:
    """The s x d^q TensorSketch matrix S of Sec. 2.2: column (i_1, .., i_q) is
    G(i_1..i_q) e_{H(i_1..i_q)} with H = sum_k h_k(i_k) mod s and G = prod_k g_k(i_k).
    h, g: q x d arrays (hash values in [0, s), signs +-1). Small d and q only."""
    h = np.asarray(h)
    g = np.asarray(g, np.float64)
    q, d = h.shape
    S = np.zeros((s, d ** q))
    for col, idx in enumerate(itertools.product(range(d), repeat=q)):
        H = sum(int(h[k, idx[k]]) for k in range(q)) % s
        G = 1.0
        for k in range(q):
            G *= g[k, idx[k]]
        S[H, col] = G
    return S


def tensor_sketch_dense(X, h, g, s: int) -> np.ndarray:
    """phi(x) = S v_q(x) for every row of X, from the explicit matrix (the definition)."""
    h = np.asarray(h)
    S = tensor_sketch_matrix(h, g, s)
    return np.stack([S @ monomials(x, h.shape[0]) for x in np.asarray(X, np.float64)])


def tensor_sketch_fft(X, h, g, s: int) -> np.ndarray:
    """phi(x) for every row of X by the fast evaluation the paper cites (Pagh): the
    circular convolution of the q CountSketches, computed as the inverse FFT of the
    product of their FFTs. Equal to tensor_sketch_dense up to rounding."""
    h = np.asarray(h)
    g = np.asarray(g, np.float64)
    q = h.shape[0]
    X = np.asarray(X, np.float64)
    out = np.empty((X.shape[0], s))
    for i, x in enumerate(X):
        F = np.ones(s, dtype=np.complex128)
        for k in range(q):
            F = F * np.fft.fft(count_sketch(x, h[k], g[k], s))
        out[i] = np.real(np.fft.ifft(F))
    return out


# ----------------------------------------------------------- multiple-level sketching
def hadamard(m: int) -> np.ndarray:
    """The m x m Walsh-Hadamard matrix by its recursive definition (Sec. 4):
    H_m = [[H_{m/2}, H_{m/2}], [H_{m/2}, -H_{m/2}]], H_1 = [1]; m a power of two."""
    if m < 1 or m & (m - 1):
        raise ValueError("m must be a power of two")
    H = np.ones((1, 1))
    while H.shape[0] < m:
        H = np.block([[H, H], [H, -H]])
    return H


def srht_matrix(signs, sample, s1: int) -> np.ndarray:
    """S = s^{-1/2} P H D (Def. 2), s = len(sample): D = diag(signs) (random +-1), H the
    s1 x s1 Walsh-Hadamard matrix, P the rows `sample` of the identity (coordinates drawn
    uniformly at random by the caller)."""
    sample = np.asarray(sample)
    s = sample.shape[0]
    H = hadamard(s1)
    return (H[sample, :] * np.asarray(signs, np.float64)[None, :]) / math.sqrt(s)


def srht_apply(Z1, signs, sample) -> np.ndarray:
    """Z_2 = Z_1 S_2^T: the SRHT applied to the rows of Z_1 (Alg. 2)."""
    Z1 = np.asarray(Z1, np.float64)
    return Z1 @ srht_matrix(signs, sample, Z1.shape[1]).T


def gaussian_project(Z2, S3) -> np.ndarray:
    """Z_3 = s_3^{-1/2} Z_2 S_3^T with S_3 (s_3 x s_2) standard normal (Alg. 2)."""
    S3 = np.asarray(S3, np.float64)
    return np.asarray(Z2, np.float64) @ S3.T / math.sqrt(S3.shape[0])


# ----------------------------------------------------- adaptive sketch size (Thm. 4)
def precond_test(Kmat, Z, lam: float, frac: float = 0.05):
    """The two quantities of Thm. 4 for a candidate Z (dense; small n only).

    P projects on the eigenvectors of Z Z^T with eigenvalues above frac * lambda.
    Returns (c1, (lo, hi), k): c1 = ||(I - P) K (I - P)||_2 (condition 1 asks
    c1 <= 0.1 lambda); lo, hi = the extremes of ||V_q^T P x||^2 / ||Z^T P x||^2 over x in
    the range of P with K = V_q V_q^T (condition 2 asks both within 1 +- 0.1); k = the
    rank of P.
    """
    K = np.asarray(Kmat, np.float64)
    Z = np.asarray(Z, np.float64)
    n = K.shape[0]
    ev, U = np.linalg.eigh(Z @ Z.T)
    keep = ev > frac * lam
    Uk, ek = U[:, keep], ev[keep]
    Pm = Uk @ Uk.T
    Q = np.eye(n) - Pm
    c1 = float(np.max(np.abs(np.linalg.eigvalsh(Q @ K @ Q))))
    if Uk.shape[1] == 0:
        return c1, (1.0, 1.0), 0
    B = (Uk.T @ K @ Uk) / np.sqrt(ek)[:, None] / np.sqrt(ek)[None, :]
    r = np.linalg.eigvalsh(0.5 * (B + B.T))
    return c1, (float(r[0]), float(r[-1])), int(Uk.shape[1])


def adaptive_sketch_size(Kmat, make_Z, lam: float, s0: int, s_max: int):
    """Sec. 5: start from s0 features and double s until the candidate passes both
    conditions of Thm. 4 (or s would exceed s_max). make_Z(s) returns the n x s sketch.
    Returns (s, Z, history) with history = [(s, c1, lo, hi, passed), ...]."""
    s, hist = s0, []
    while True:
        Z = make_Z(s)
        c1, (lo, hi), _ = precond_test(Kmat, Z, lam)
        ok = c1 <= 0.1 * lam and 0.9 <= lo and hi <= 1.1
        hist.append((s, c1, lo, hi, ok))
        if ok or 2 * s > s_max:
            return s, Z, hist
        s *= 2
