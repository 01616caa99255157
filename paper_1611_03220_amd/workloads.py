"""Seeded synthetic workloads (inputs only).

This module generates the inputs that both the HIP path and the CPU oracle consume:
points X, right-hand sides Y, the kernel bandwidth sigma and ridge lambda, and the
random draws of the feature map (W, b). It holds none of the method's arithmetic.

Every array is generated in FP64 with ``numpy.random.default_rng(161103220 + 1000*family
+ stream)`` and rounded once to FP32 where it is a data input (X, W, b); those FP32
values are the canonical inputs for both sides. Streams: 0 points, 1 labels / teacher,
2 feature-map draws (W, b), 3 bandwidth pairs, 4 noise.

Shapes follow the workloads the paper measures on (Sec. 6: one-vs-all classification
label matrices, Gaussian kernel, sigma and lambda as hyper-parameters); no dataset
from the paper is reproduced, synthetic stand-ins of the same shape are generated.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

SEED_BASE = 161103220


def rng_for(family: int, stream: int, salt: int = 0) -> np.random.Generator:
    return np.random.default_rng(SEED_BASE + 1000 * family + stream + 100000 * salt)


@dataclasses.dataclass
class Workload:
    name: str
    X: np.ndarray            # n x d float32 (canonical)
    Y: np.ndarray            # n x m float64
    sigma: float
    lam: float
    s: int
    W: np.ndarray            # d x s float32, columns ~ N(0, sigma^-2 I)
    b: np.ndarray            # s float32, U[0, 2 pi)
    tol: float
    Xv: np.ndarray | None = None   # validation points (differentiation workload)
    Yv: np.ndarray | None = None

    @property
    def n(self):
        return self.X.shape[0]

    @property
    def d(self):
        return self.X.shape[1]

    @property
    def m(self):
        return self.Y.shape[1]


def median_distance(X: np.ndarray, rng: np.random.Generator, npairs: int = 1 << 20) -> float:
    """Median Euclidean distance over ``npairs`` seeded distinct pairs, in FP64."""
    n = X.shape[0]
    npairs = min(npairs, n * (n - 1))
    i = rng.integers(0, n, npairs)
    j = rng.integers(0, n - 1, npairs)
    j = j + (j >= i)  # distinct partner
    Xd = X.astype(np.float64)
    out = np.empty(npairs)
    step = 1 << 16
    for a in range(0, npairs, step):
        diff = Xd[i[a:a + step]] - Xd[j[a:a + step]]
        out[a:a + step] = np.sqrt(np.einsum("ij,ij->i", diff, diff))
    return float(np.median(out))


def rff_draw(d: int, s: int, sigma: float, rng: np.random.Generator):
    """W = G / sigma with G ~ N(0, 1) (d x s) and b ~ U[0, 2 pi) (s), rounded to FP32."""
    W = (rng.standard_normal((d, s)) / sigma).astype(np.float32)
    b = rng.uniform(0.0, 2.0 * math.pi, s).astype(np.float32)
    return W, b


def one_vs_all(labels: np.ndarray, k: int) -> np.ndarray:
    Y = -np.ones((labels.shape[0], k))
    Y[np.arange(labels.shape[0]), labels] = 1.0
    return Y


def plain_fp64(n: int = 2000, d: int = 8, s: int = 200, lam_per_n: float = 1e-3,
               tol: float = 1e-10, salt: int = 0) -> Workload:
    """Single-RHS regression: X ~ N(0,1), sigma = sqrt(d), lambda = 1e-3 n,
    y = sin(X u) + 0.1 eps with u ~ N(0, I/d)."""
    family = 0
    X = rng_for(family, 0, salt).standard_normal((n, d)).astype(np.float32)
    u = rng_for(family, 1, salt).standard_normal(d) / math.sqrt(d)
    eps = rng_for(family, 4, salt).standard_normal(n)
    Y = np.ascontiguousarray((np.sin(X.astype(np.float64) @ u) + 0.1 * eps)[:, None])
    sigma = math.sqrt(d)
    W, b = rff_draw(d, s, sigma, rng_for(family, 2, salt))
    return Workload("plain_fp64", X, Y, sigma, lam_per_n * n, s, W, b, tol)


def mixture_multi_rhs(n: int = 65536, d: int = 54, k: int = 7, s: int = 2048,
                      lam_per_n: float = 1e-4, tol: float = 1e-6, salt: int = 0) -> Workload:
    """k-component Gaussian mixture (means ~ N(0, 4 I), unit covariance, uniform weights),
    standardised per column; k one-vs-all +-1 columns; sigma = median pairwise distance
    (the same kernel as scaling X to unit median distance with sigma = 1)."""
    family = 1
    r0 = rng_for(family, 0, salt)
    means = 2.0 * r0.standard_normal((k, d))
    lab = rng_for(family, 1, salt).integers(0, k, n)
    X = means[lab] + r0.standard_normal((n, d))
    X = (X - X.mean(0)) / X.std(0)
    X = X.astype(np.float32)
    sigma = median_distance(X, rng_for(family, 3, salt))
    W, b = rff_draw(d, s, sigma, rng_for(family, 2, salt))
    return Workload("mixture_multi_rhs", X, one_vs_all(lab, k), sigma, lam_per_n * n, s, W, b, tol)


def pixels(n: int = 262144, d: int = 784, k: int = 10, s: int = 8192,
           lam_per_n: float = 1e-5, tol: float = 1e-6, salt: int = 0) -> Workload:
    """Pixel-like points in [0, 1]: 80% zeros, nonzeros ~ U(0, 1); k one-vs-all columns
    from the argmax of a random linear teacher applied to the centred points."""
    family = 2
    r0 = rng_for(family, 0, salt)
    X = np.zeros((n, d), np.float32)
    for a in range(0, n, 8192):
        blk = r0.uniform(0.0, 1.0, (min(8192, n - a), d))
        blk[r0.random(blk.shape) < 0.8] = 0.0
        X[a:a + blk.shape[0]] = blk
    T = rng_for(family, 1, salt).standard_normal((d, k))
    mu = X.astype(np.float64).mean(0)
    lab = np.empty(n, np.int64)
    for a in range(0, n, 8192):
        lab[a:a + 8192] = np.argmax((X[a:a + 8192].astype(np.float64) - mu) @ T, axis=1)
    sigma = median_distance(X, rng_for(family, 3, salt))
    W, b = rff_draw(d, s, sigma, rng_for(family, 2, salt))
    return Workload("pixels", X, one_vs_all(lab, k), sigma, lam_per_n * n, s, W, b, tol)


def correlated_differentiation(n: int = 131072, n_val: int = 16384, d: int = 440, k: int = 147,
                               s: int = 4096, lam_per_n: float = 1e-4, tol: float = 1e-6,
                               salt: int = 0) -> Workload:
    """X = G A^T / sqrt(d) with G, A ~ N(0,1) (covariance A A^T / d); k one-vs-all columns
    from the argmax of a random linear teacher; n training plus n_val validation points;
    sigma = median training distance, lambda = 1e-4 n."""
    family = 4
    r0 = rng_for(family, 0, salt)
    A = r0.standard_normal((d, d))
    tot = n + n_val
    X = np.empty((tot, d), np.float32)
    for a in range(0, tot, 8192):
        m_ = min(8192, tot - a)
        X[a:a + m_] = (r0.standard_normal((m_, d)) @ A.T / math.sqrt(d)).astype(np.float32)
    T = rng_for(family, 1, salt).standard_normal((d, k))
    lab = np.empty(tot, np.int64)
    for a in range(0, tot, 8192):
        lab[a:a + 8192] = np.argmax(X[a:a + 8192].astype(np.float64) @ T, axis=1)
    Yall = one_vs_all(lab, k)
    Xtr, Xv = X[:n], X[n:]
    sigma = median_distance(Xtr, rng_for(family, 3, salt))
    W, b = rff_draw(d, s, sigma, rng_for(family, 2, salt))
    return Workload("correlated_differentiation", Xtr, Yall[:n], sigma, lam_per_n * n, s, W, b,
                    tol, Xv=Xv, Yv=Yall[n:])


def batched_instances(count: int = 64, n_lo: int = 1024, n_hi: int = 16384,
                      dims=(16, 32, 64, 128), tol: float = 1e-6, salt: int = 0) -> list:
    """``count`` independent problems: n log-uniform in [n_lo, n_hi], d uniform over
    ``dims``, X ~ N(0,1), s = n/8, 1..4 right-hand sides y = sin(X u) + 0.1 eps,
    lambda log-uniform in [1e-6, 1e-2] n, sigma = sqrt(d)."""
    family = 3
    meta = rng_for(family, 1, salt)
    out = []
    for t in range(count):
        n = int(round(math.exp(meta.uniform(math.log(n_lo), math.log(n_hi)))))
        d = int(meta.choice(dims))
        m = int(meta.integers(1, 5))
        lam = math.exp(meta.uniform(math.log(1e-6), math.log(1e-2))) * n
        X = rng_for(family, 0, salt * 1000 + t + 1).standard_normal((n, d)).astype(np.float32)
        u = rng_for(family, 1, salt * 1000 + t + 1).standard_normal((d, m)) / math.sqrt(d)
        eps = rng_for(family, 4, salt * 1000 + t + 1).standard_normal((n, m))
        Y = np.sin(X.astype(np.float64) @ u) + 0.1 * eps
        sigma = math.sqrt(d)
        s = max(1, n // 8)
        W, b = rff_draw(d, s, sigma, rng_for(family, 2, salt * 1000 + t + 1))
        out.append(Workload(f"batched_{t}", X, Y, sigma, lam, s, W, b, tol))
    return out


# ------------------------------------------------------------ polynomial kernel workloads
@dataclasses.dataclass
class PolyWorkload:
    """A polynomial-kernel problem (gamma x^T z + c)^q with its TensorSketch draw."""
    name: str
    X: np.ndarray            # n x d float32
    Y: np.ndarray            # n x m float64
    gamma: float
    coef0: float
    degree: int
    lam: float
    s: int
    hash: np.ndarray         # degree x (d + 1) int32 in [0, s)
    sign: np.ndarray         # degree x (d + 1) float32 of +-1
    tol: float

    @property
    def n(self):
        return self.X.shape[0]

    @property
    def d(self):
        return self.X.shape[1]

    @property
    def m(self):
        return self.Y.shape[1]


def tensorsketch_draw(d: int, q: int, s: int, rng: np.random.Generator):
    """Hashes h_k: [d + 1] -> [s] and signs g_k: [d + 1] -> {+1, -1} for q CountSketches of the
    augmented points (fully random tables)."""
    h = rng.integers(0, s, size=(q, d + 1)).astype(np.int32)
    g = rng.choice(np.array([-1.0, 1.0], np.float32), size=(q, d + 1)).astype(np.float32)
    return h, g


def polynomial_mixture(n: int = 65536, d: int = 54, k: int = 7, s: int = 2048, degree: int = 3,
                       lam_per_n: float = 1e-4, tol: float = 1e-6, salt: int = 0) -> PolyWorkload:
    """The mixture points and labels of mixture_multi_rhs with the polynomial kernel
    (x^T z / d + 1)^3 (gamma = 1/d, c = 1, q = 3) and s TensorSketch features."""
    w = mixture_multi_rhs(n=n, d=d, k=k, s=2, lam_per_n=lam_per_n, tol=tol, salt=salt)
    h, g = tensorsketch_draw(d, degree, s, rng_for(6, 2, salt))
    return PolyWorkload("polynomial_mixture", w.X, w.Y, 1.0 / d, 1.0, degree, lam_per_n * n, s,
                        h, g, tol)


def multilevel_draw(s1: int, s2: int, s3: int, rng: np.random.Generator):
    """Random parts of the multiple-level sketch: SRHT signs (s1), s2 coordinates sampled
    without replacement from the power-of-two padded width, and the s3 x s2 standard normal
    projection, all FP32 / int32."""
    p = 1
    while p < s1:
        p *= 2
    signs = rng.choice(np.array([-1.0, 1.0], np.float32), size=s1).astype(np.float32)
    sample = np.sort(rng.choice(p, size=s2, replace=False)).astype(np.int32)
    S3 = rng.standard_normal((s3, s2)).astype(np.float32)
    return signs, sample, S3
