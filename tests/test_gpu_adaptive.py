"""GPU parity of the adaptive sketch size (Sec. 5, Thm. 4): the preconditioner test of a
candidate sketch against the oracle's exact test, the cases whose outcome is fixed by the
mathematics (an exact factorisation passes, a scaled one fails condition 2), and the doubling
rule.

The GPU test estimates ||(I - P) K (I - P)|| and the extreme ratios by power iteration, so its
values approach the oracle's exact ones from inside: a Rayleigh quotient never exceeds the
largest eigenvalue (up to the product's rounding), and with the iteration counts used here it
comes within the stated fraction when the oracle's own spectrum shows a clear gap.
"""
import math

import numpy as np
import pytest
import torch

import oracle as O
from oracle import sketch_oracle as SO
from paper_1611_03220_amd import krr
from paper_1611_03220_amd import workloads as WL

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    krr.lib()
    return torch.device("cuda:0")


def _t(a, dev):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


def test_exact_factor_passes_and_scaled_factor_fails(dev):
    """Linear kernel (q = 1): Z = [sqrt(gamma) X, sqrt(c)] gives Z Z^T = K exactly, so on range(P)
    the ratio is 1 and (I - P) K (I - P) keeps only eigenvalues below 0.05 lambda: the test
    passes. Z scaled by sqrt(2) makes Z Z^T = 2 K: the ratio is 1/2 and condition 2 fails."""
    rng = np.random.default_rng(110)
    n, d, lam = 800, 6, 0.5
    X = rng.standard_normal((n, d)).astype(np.float32)
    k = krr.Kernel.polynomial(0.3, 1.0, 1)
    Z = SO.poly_augment(X, 0.3, 1.0).astype(np.float32)
    for prec in ("fp64", "f16x3"):
        r = krr.precond_test(k, _t(X, dev), _t(Z, dev), lam, power_iters=40, prec=prec)
        assert r.rank == d + 1
        assert r.passed == 1, r.as_dict()
        assert abs(r.ratio_lo - 1.0) < 1e-4 and abs(r.ratio_hi - 1.0) < 1e-4, r.as_dict()
        r2 = krr.precond_test(k, _t(X, dev), _t(math.sqrt(2) * Z, dev), lam, power_iters=40, prec=prec)
        assert r2.passed == 0
        assert abs(r2.ratio_lo - 0.5) < 1e-4 and abs(r2.ratio_hi - 0.5) < 1e-4, r2.as_dict()


@pytest.mark.parametrize("prec", ["fp64", "f16x3"])
def test_precond_test_matches_oracle(dev, prec):
    """A TensorSketch candidate for a low-rank polynomial kernel: the rank of P equals the
    oracle's, and the power-iteration estimates lie within the exact values and close to them."""
    rng = np.random.default_rng(111)
    n, d, q, s, lam = 700, 4, 2, 64, 0.05
    X = (rng.standard_normal((n, d)) / math.sqrt(d)).astype(np.float32)
    h, g = WL.tensorsketch_draw(d, q, s, rng)
    k = krr.Kernel.polynomial(1.0, 0.5, q)
    Zg = krr.tensorsketch(_t(X, dev), 1.0, 0.5, q, _t(h, dev), _t(g, dev), s)
    Z = Zg.cpu().numpy().astype(np.float64)  # the GPU's own sketch, tested on both sides
    K = SO.polynomial_kernel(X, X, 1.0, 0.5, q)
    ev = np.linalg.eigvalsh(Z.T @ Z)
    thr = 0.05 * lam
    assert np.min(np.abs(ev - thr) / thr) > 1e-3  # no eigenvalue on the threshold
    c1, (lo, hi), rank = SO.precond_test(K, Z, lam)
    r = krr.precond_test(k, _t(X, dev), Zg, lam, power_iters=80, prec=prec)
    assert r.rank == rank
    # U is formed by the split MFMA GEMM (FP16 hi/lo, about 2^-21 relative) in both cases
    tol = 1e-5
    assert r.cond1 <= c1 * (1 + tol) + tol and r.cond1 >= 0.9 * c1, (r.as_dict(), c1)
    assert r.ratio_hi <= hi * (1 + tol) and r.ratio_hi >= hi - 0.02 * hi, (r.as_dict(), hi)
    assert r.ratio_lo >= lo * (1 - tol) - tol and r.ratio_lo <= lo + 0.02 * hi, (r.as_dict(), lo)
    assert r.passed == int(c1 <= 0.1 * lam and lo >= 0.9 and hi <= 1.1) or abs(c1 - 0.1 * lam) < 0.02 * lam


def test_adaptive_doubling_polynomial(dev):
    """Sec. 5: s doubles from s0 until the TensorSketch candidate passes (here d = 2, q = 2: nine
    augmented monomials, so a collision-free sketch reproduces K exactly and must pass); the
    sizes tried are
    s0, 2 s0, ...; every failed size fails the oracle's exact test too (or sits within the
    estimate's margin), and the accepted sketch preconditions PCG to 1e-6 within the CG bound
    of its measured condition number (proof of Thm. 1)."""
    rng = np.random.default_rng(112)
    n, d, q, lam = 1500, 2, 2, 1.0
    X = (rng.standard_normal((n, d)) / math.sqrt(d)).astype(np.float32)
    s_max = 1024
    h, g = WL.tensorsketch_draw(d, q, s_max, rng)
    k = krr.Kernel.polynomial(1.0, 1.0, q)
    Zs, s, hist = krr.adaptive_features(k, _t(X, dev), lam, 4, s_max, hash_=_t(h, dev),
                                        sign=_t(g, dev), power_iters=60, prec="fp64")
    assert s == 4 * 2 ** (len(hist) - 1)
    assert hist[-1]["passed"] == 1 and all(hh["passed"] == 0 for hh in hist[:-1])
    K = SO.polynomial_kernel(X, X, 1.0, 1.0, q)
    for i, hh in enumerate(hist[:-1]):
        si = 4 * 2 ** i
        Zo = SO.tensor_sketch_fft(SO.poly_augment(X, 1.0, 1.0), h % si, g, si)
        c1, (lo, hi), _ = SO.precond_test(K, Zo, lam)
        exact_pass = c1 <= 0.1 * lam and lo >= 0.9 and hi <= 1.1
        assert not exact_pass or abs(c1 - 0.1 * lam) < 0.05 * lam or min(abs(lo - 0.9), abs(hi - 1.1)) < 0.05
    # the accepted preconditioner
    Y = rng.standard_normal((n, 2))
    _, Ut = krr.precond_factor(Zs.contiguous(), lam)
    a, rep = krr.pcg_solve_k(k, _t(X, dev), lam, Ut, _t(Y, dev), tol=1e-6, prec="fp64")
    A = K + lam * np.eye(n)
    R = Y - A @ a.cpu().numpy()
    assert np.max(np.linalg.norm(R, axis=0) / np.linalg.norm(Y, axis=0)) <= 1e-6
    ev = O.preconditioned_spectrum(K, lam, Zs.cpu().numpy(), lam)
    assert ev[-1] / ev[0] <= 4.0, (ev[0], ev[-1])
    # ||r|| / ||y|| <= sqrt(kappa(A)) ||e||_A / ||c||_A, so the CG bound with
    # eps = 1e-6 / sqrt(kappa(A)) covers the residual stopping rule
    eA = np.linalg.eigvalsh(A)
    T = O.cg_iteration_bound(ev[-1] / ev[0], 1e-6 / math.sqrt(eA[-1] / eA[0]))
    assert rep.iters <= T + 2, (rep.iters, T)
