"""GPU parity of the wide large-d pass: up to 160 right-hand-side columns share one distance
pass (NCT = 10 column tiles of 16, V^T tiles staged through LDS one piece per thread per
chunk step). Same per-entry bounds as the other mixed products (derived in
test_gpu_parity.py and test_gpu_poly.py): m = 65 (the narrowest wide pass), 147 (the
differentiation workload's class count), 160 (a full pass) and 161 (a full pass and a
one-column pass), with K, dK/dsigma and the polynomial kernel, square and rectangular.
"""
import math

import numpy as np
import pytest
import torch

import oracle as O
from oracle import sketch_oracle as SO
from paper_1611_03220_amd import krr

pytestmark = pytest.mark.gpu

LN2 = math.log(2.0)


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    krr.lib()
    return torch.device("cuda:0")


def _t(a, dev):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


def _tau(X1, X2, sigma, d):
    kp = int(math.ceil((d + 2) / 32) * 32)
    c = math.log2(math.e) / (2 * sigma * sigma)
    nu = max(float((X1.astype(np.float64) ** 2).sum(1).max()), float((X2.astype(np.float64) ** 2).sum(1).max()))
    return LN2 * (2 * 2.0 ** -22 + kp * 2.0 ** -24) * 4 * c * nu + 2.0 ** -22 + 16 * 2.0 ** -24


def _bound(X1, X2, sigma, V, deriv, d):
    tau = _tau(X1, X2, sigma, d)
    if not deriv:
        return tau * (O.gaussian_kernel(X1, X2, sigma) @ np.abs(V))
    c = math.log2(math.e) / (2 * sigma ** 2)
    Kd = O.gaussian_kernel(X1, X2, sigma)
    return tau * (np.abs(O.gaussian_kernel_dsigma(X1, X2, sigma)) @ np.abs(V)) \
        + ((tau / LN2) / c * Kd / sigma ** 3) @ np.abs(V)


@pytest.mark.parametrize("n1,n2,d,m", [(300, 300, 440, 65), (517, 517, 440, 147), (200, 333, 300, 160),
                                       (257, 257, 160, 161), (129, 70, 784, 147)])
def test_wide_pass_matches_oracle(dev, n1, n2, d, m):
    rng = np.random.default_rng(1200 + n1 + d + m)
    X1 = rng.standard_normal((n1, d)).astype(np.float32)
    X2 = X1 if n1 == n2 else rng.standard_normal((n2, d)).astype(np.float32)
    V = rng.standard_normal((n2, m))
    sigma = 0.8 * math.sqrt(d)
    A = _t(X1, dev)
    B = A if n1 == n2 else _t(X2, dev)
    for deriv in (False, True):
        got = krr.kernel_matmat(A, B, sigma, _t(V, dev), deriv=deriv).cpu().numpy()
        ref = O.kernel_matmat(X1, X2, sigma, V, deriv=deriv)
        bound = _bound(X1, X2, sigma, V, deriv, d)
        assert np.all(np.abs(got - ref) <= bound), (deriv, np.max(np.abs(got - ref) / bound))


def test_wide_pass_polynomial(dev):
    rng = np.random.default_rng(1210)
    n, d, m, gamma, c, q = 400, 300, 147, 0.004, 1.0, 3
    X = rng.standard_normal((n, d)).astype(np.float32)
    V = rng.standard_normal((n, m))
    Xg = _t(X, dev)
    out = krr.kernel_matmat_k(krr.Kernel.polynomial(gamma, c, q), Xg, Xg, _t(V, dev)).cpu().numpy()
    ref = SO.poly_kernel_matmat(X, X, gamma, c, q, V)
    nu = float((X.astype(np.float64) ** 2).sum(1).max())
    e = math.frexp(gamma * nu + c)[1]
    T = 2.0 ** (e + (e & 1))
    kp = int(math.ceil((d + 2) / 32) * 32)
    KV = np.abs(SO.polynomial_kernel(X, X, gamma, c, q)) @ np.abs(V)
    bound = T ** q * (q * (2.0 ** -21 + kp * 2.0 ** -24) + 2.0 ** -22 + 2.0 ** -25) * np.abs(V).sum(0)[None, :] \
        + 16 * 2.0 ** -24 * KV
    assert np.all(np.abs(out - ref) <= bound), np.max(np.abs(out - ref) / bound)


def test_wide_pass_grouped_launch_sampled_rows(dev):
    """The differentiation workload's product shape class (d = 440, 147 columns) at
    n = 16384 + 77: the grouped 8-split launch, checked on 32 sampled rows."""
    rng = np.random.default_rng(1211)
    n, d, m = 16384 + 77, 440, 147
    X = (rng.standard_normal((n, d)) / math.sqrt(2.0)).astype(np.float32)
    V = rng.standard_normal((n, m))
    sigma = 0.9 * math.sqrt(d)
    Xg = _t(X, dev)
    got = krr.kernel_matmat(Xg, Xg, sigma, _t(V, dev)).cpu().numpy()
    rows = np.sort(rng.choice(n, 32, replace=False))
    rows[0], rows[-1] = 0, n - 1
    ref = O.kernel_matmat(X, X, sigma, V, rows=rows)
    tau = _tau(X, X, sigma, d)
    bound = tau * (O.gaussian_kernel(X[rows], X, sigma) @ np.abs(V))
    assert np.all(np.abs(got[rows] - ref) <= bound), np.max(np.abs(got[rows] - ref) / bound)


@pytest.mark.parametrize("n1,n2,d,m", [(300, 300, 440, 147), (200, 333, 300, 160), (129, 140, 160, 161),
                                       (150, 150, 784, 65)])
def test_wide_pass_fp64(dev, n1, n2, d, m):
    """The FP64 large-d product's 160-column pass (V^T tile loaded in four slices over the
    first chunks): 1e-12 relative to (|K| |V|)_i, value and sigma-derivative, the smallest
    chunk count (d = 160: five 32-wide chunks) included."""
    rng = np.random.default_rng(1300 + n1 + d + m)
    X1 = rng.standard_normal((n1, d)).astype(np.float32)
    X2 = X1 if n1 == n2 else rng.standard_normal((n2, d)).astype(np.float32)
    V = rng.standard_normal((n2, m))
    sigma = 0.8 * math.sqrt(d)
    A = _t(X1, dev)
    B = A if n1 == n2 else _t(X2, dev)
    for deriv in (False, True):
        got = krr.kernel_matmat(A, B, sigma, _t(V, dev), deriv=deriv, prec="fp64").cpu().numpy()
        ref = O.kernel_matmat(X1, X2, sigma, V, deriv=deriv)
        K = (O.gaussian_kernel_dsigma if deriv else O.gaussian_kernel)(X1, X2, sigma)
        bound = 1e-12 * (np.abs(K) @ np.abs(V))
        assert np.all(np.abs(got - ref) <= bound), (deriv, np.max(np.abs(got - ref) / bound))
