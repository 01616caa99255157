"""GPU parity of the symmetric large-d kernel product K(X, X) V (both sides the same points,
d large enough for the LDS-streamed product, passes of up to 16 columns): each off-diagonal
pair of 128-row blocks is formed once and serves both triangles, the transposed side summed
in 64-bit fixed point; small d takes the general kernel (also checked here). The exact
symmetry K_ij = K_ji makes it the same product as the general one, so the same per-entry
bounds apply (derived in test_gpu_parity.py and test_gpu_poly.py); it is checked against the
oracle, against the general path on a copy of the points, for determinism, for non-finite
propagation and at the launch shapes of the large workloads (grouped launch, many block
pairs) on sampled rows.
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


def _tau(X, sigma, d):
    kp = int(math.ceil((d + 2) / 32) * 32)
    c = math.log2(math.e) / (2 * sigma * sigma)
    nu = float((X.astype(np.float64) ** 2).sum(1).max())
    return LN2 * (2 * 2.0 ** -22 + kp * 2.0 ** -24) * 4 * c * nu + 2.0 ** -22 + 16 * 2.0 ** -24


def _bound(X, sigma, V, deriv, d, rows=None):
    Xr = X if rows is None else X[rows]
    tau = _tau(X, sigma, d)
    if not deriv:
        return tau * (O.gaussian_kernel(Xr, X, sigma) @ np.abs(V))
    c = math.log2(math.e) / (2 * sigma ** 2)
    Kd = O.gaussian_kernel(Xr, X, sigma)
    return tau * (np.abs(O.gaussian_kernel_dsigma(Xr, X, sigma)) @ np.abs(V)) \
        + ((tau / LN2) / c * Kd / sigma ** 3) @ np.abs(V)


# n: one block, a ragged pair list with a middle block (odd count), an even count; m: packed
# (<= 8), separate hi/lo (9..16), and 17 (two 16-row tiles: the general kernel)
@pytest.mark.parametrize("n,d,m", [(1, 150, 3), (128, 200, 1), (677, 150, 8), (677, 300, 10),
                                   (1000, 784, 16), (517, 440, 17), (300, 129, 5),
                                   # small d: the general register-resident kernel on the
                                   # same points
                                   (677, 54, 7), (1000, 40, 16), (129, 80, 9), (300, 126, 1),
                                   (257, 20, 4), (200, 54, 17), (64, 62, 2)])
def test_sym_matches_oracle_and_general_path(dev, n, d, m):
    rng = np.random.default_rng(900 + n + d + m)
    X = rng.standard_normal((n, d)).astype(np.float32)
    V = rng.standard_normal((n, m))
    sigma = 0.8 * math.sqrt(d)
    Xg = _t(X, dev)
    for deriv in (False, True):
        got = krr.kernel_matmat(Xg, Xg, sigma, _t(V, dev), deriv=deriv).cpu().numpy()
        ref = O.kernel_matmat(X, X, sigma, V, deriv=deriv)
        bound = _bound(X, sigma, V, deriv, d)
        assert np.all(np.abs(got - ref) <= bound), (deriv, np.max(np.abs(got - ref) / bound))
        # the general kernel on a copy of the points (a different buffer): same bound, so the
        # two differ by at most twice it
        gen = krr.kernel_matmat(Xg, Xg.clone(), sigma, _t(V, dev), deriv=deriv).cpu().numpy()
        assert np.all(np.abs(got - gen) <= 2 * bound)


def test_sym_shift_and_strided_points(dev):
    """shift adds lambda V; points given as a strided view (ld > d) of a wider array."""
    rng = np.random.default_rng(931)
    n, d, m = 900, 260, 6
    Xw = rng.standard_normal((n, d + 7)).astype(np.float32)
    X = Xw[:, :d]
    V = rng.standard_normal((n, m))
    Xg = _t(Xw, dev)[:, :d]
    got = krr.kernel_matmat(Xg, Xg, 14.0, _t(V, dev), shift=0.3).cpu().numpy()
    ref = O.kernel_matmat(X, X, 14.0, V, shift=0.3)
    bound = _bound(X, 14.0, V, False, d) + 1e-15 * 0.3 * np.abs(V)
    assert np.all(np.abs(got - ref) <= bound), np.max(np.abs(got - ref) / bound)


def test_sym_deterministic(dev):
    """The fixed-point column side makes repeated products bit-identical."""
    rng = np.random.default_rng(932)
    X = _t(rng.standard_normal((3000, 200)).astype(np.float32), dev)
    V = _t(rng.standard_normal((3000, 10)), dev)
    a = krr.kernel_matmat(X, X, 12.0, V)
    b = krr.kernel_matmat(X, X, 12.0, V)
    assert torch.equal(a, b)


def test_sym_nonfinite_column_propagates(dev):
    """A NaN in V[5, 1] reaches every row of column 1 through both triangles; the other
    columns stay finite and match the oracle."""
    rng = np.random.default_rng(933)
    n, d, m = 700, 180, 4
    X = rng.standard_normal((n, d)).astype(np.float32)
    V = rng.standard_normal((n, m))
    V[5, 1] = np.nan
    Xg = _t(X, dev)
    got = krr.kernel_matmat(Xg, Xg, 0.9 * math.sqrt(d), _t(V, dev)).cpu().numpy()
    assert np.isnan(got[:, 1]).all()
    keep = [0, 2, 3]
    ref = O.kernel_matmat(X, X, 0.9 * math.sqrt(d), V[:, keep])
    bound = _bound(X, 0.9 * math.sqrt(d), V[:, keep], False, d)
    assert np.all(np.abs(got[:, keep] - ref) <= bound)


@pytest.mark.parametrize("q,gamma,c", [(3, 0.01, 1.0), (2, 0.004, 0.5)])
def test_sym_polynomial(dev, q, gamma, c):
    rng = np.random.default_rng(934 + q)
    n, d, m = 600, 300, 10
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


def test_sym_many_pairs_grouped_launch(dev):
    """65 block pairs with 8 column splits: the XCD-grouped launch of the symmetric kernel,
    with splits that cross from one row block of a pair to the other; 40 sampled rows,
    including the ragged last one."""
    rng = np.random.default_rng(935)
    n, d, m = 64 * 2 * 128 + 2 * 128 + 77, 200, 10
    X = rng.random((n, d)).astype(np.float32)
    X[rng.random((n, d)) < 0.5] = 0.0
    V = rng.standard_normal((n, m))
    sigma = float(np.sqrt(np.median(((X[:200, None, :] - X[None, 200:400, :]) ** 2).sum(-1))))
    Xg = _t(X, dev)
    got = krr.kernel_matmat(Xg, Xg, sigma, _t(V, dev)).cpu().numpy()
    rows = np.sort(rng.choice(n, 40, replace=False))
    rows[0], rows[-1] = 0, n - 1
    ref = O.kernel_matmat(X, X, sigma, V, rows=rows)
    bound = _bound(X, sigma, V, False, d, rows=rows)
    assert np.all(np.abs(got[rows] - ref) <= bound), np.max(np.abs(got[rows] - ref) / bound)


def test_same_points_small_d_sampled(dev):
    """K(X, X) V with small d at a mixture-like size (n = 20000 + 33, d = 54, 7 columns,
    shift; the general kernel): sampled rows against the oracle, and determinism."""
    rng = np.random.default_rng(936)
    n, d, m = 20033, 54, 7
    X = rng.standard_normal((n, d)).astype(np.float32)
    V = rng.standard_normal((n, m))
    sigma = 0.6 * math.sqrt(d)
    Xg, Vg = _t(X, dev), _t(V, dev)
    got = krr.kernel_matmat(Xg, Xg, sigma, Vg, shift=0.25).cpu().numpy()
    again = krr.kernel_matmat(Xg, Xg, sigma, Vg, shift=0.25).cpu().numpy()
    assert np.array_equal(got, again)
    rows = np.sort(rng.choice(n, 40, replace=False))
    rows[0], rows[-1] = 0, n - 1
    ref = O.kernel_matmat(X, X, sigma, V, shift=0.25, rows=rows)
    bound = _bound(X, sigma, V, False, d, rows=rows) + 1e-15 * 0.25 * np.abs(V[rows])
    assert np.all(np.abs(got[rows] - ref) <= bound), np.max(np.abs(got[rows] - ref) / bound)


@pytest.mark.parametrize("n,d,m", [(677, 150, 7), (300, 784, 10), (1000, 440, 16), (129, 160, 1),
                                   (1, 200, 2), (517, 300, 17)])
def test_sym_fp64(dev, n, d, m):
    """The symmetric FP64 large-d product (one pass of at most 16 columns; m = 17 takes the
    general kernel): 1e-12 relative to (|K| |V|)_i like every FP64 product, K and dK/dsigma,
    against the oracle; bit-identical on a repeat (two-word fixed-point column side). For
    dK/dsigma the diagonal adds the rounding of a coincident pair's distance,
    D = nu_i + nu_i - 2 <x_i, x_i> ~ 1e-15 nu_i instead of 0, times dscale |V_i| (the oracle's
    difference form gives exactly 0 there)."""
    rng = np.random.default_rng(1400 + n + d + m)
    X = rng.standard_normal((n, d)).astype(np.float32)
    V = rng.standard_normal((n, m)) * np.exp(rng.standard_normal((n, 1)))
    sigma = 0.8 * math.sqrt(d)
    Xg, Vg = _t(X, dev), _t(V, dev)
    for deriv in (False, True):
        got = krr.kernel_matmat(Xg, Xg, sigma, Vg, deriv=deriv, prec="fp64")
        again = krr.kernel_matmat(Xg, Xg, sigma, Vg, deriv=deriv, prec="fp64")
        assert torch.equal(got, again)
        got = got.cpu().numpy()
        ref = O.kernel_matmat(X, X, sigma, V, deriv=deriv)
        K = (O.gaussian_kernel_dsigma if deriv else O.gaussian_kernel)(X, X, sigma)
        bound = 1e-12 * (np.abs(K) @ np.abs(V))
        if deriv:
            nu = (X.astype(np.float64) ** 2).sum(1)[:, None]
            bound = bound + 1e-14 * nu / sigma ** 3 * np.abs(V)
        assert np.all(np.abs(got - ref) <= bound), (deriv, np.max(np.abs(got - ref) / bound))


def test_sym_fp64_nonfinite_and_sampled_large(dev):
    """FP64 symmetric product: a NaN in V reaches its whole column through both triangles; and
    at n = 16384 + 300 (66 block pairs, 8 splits) 24 sampled rows meet the 1e-12 bound."""
    rng = np.random.default_rng(1450)
    n, d, m = 700, 180, 3
    X = rng.standard_normal((n, d)).astype(np.float32)
    V = rng.standard_normal((n, m))
    V[9, 2] = np.nan
    Xg = _t(X, dev)
    got = krr.kernel_matmat(Xg, Xg, 0.9 * math.sqrt(d), _t(V, dev), prec="fp64").cpu().numpy()
    assert np.isnan(got[:, 2]).all() and np.isfinite(got[:, :2]).all()
    n, d, m = 16384 + 300, 200, 10
    X = rng.random((n, d)).astype(np.float32)
    V = rng.standard_normal((n, m))
    sigma = 0.5 * math.sqrt(d)
    Xg = _t(X, dev)
    got = krr.kernel_matmat(Xg, Xg, sigma, _t(V, dev), prec="fp64").cpu().numpy()
    rows = np.sort(rng.choice(n, 24, replace=False))
    rows[0], rows[-1] = 0, n - 1
    ref = O.kernel_matmat(X, X, sigma, V, rows=rows)
    bound = 1e-12 * (O.gaussian_kernel(X[rows], X, sigma) @ np.abs(V))
    assert np.all(np.abs(got[rows] - ref) <= bound), np.max(np.abs(got[rows] - ref) / bound)
