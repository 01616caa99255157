"""GPU parity of the multiple-level sketch (Sec. 4, Def. 2, Thm. 3, Alg. 2): the SRHT and the
Gaussian projection against the sketching oracle, and the three-level preconditioner in the
PCG solve.

Bounds follow the arithmetic:
  * SRHT (FP32 fast transform): every output is a +- sum of all p inputs formed in log2 p
    pairwise stages, so |Z2 - Z2_ref|_it <= (log2 p + 2) 2^-24 sum_j |z_ij| / sqrt(s2).
  * Gaussian projection (FP16 hi/lo split GEMM, three products, FP32 accumulate):
    |Z3 - Z3_ref|_ij <= (2^-21 + s2 2^-24) sum_k |Z2_ik| |S3_jk| / sqrt(s3) + 2^-24 |Z3_ref|_ij
    (the split error of both operands, FP32 accumulation over s2 terms, the FP32 store).
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


@pytest.mark.parametrize("n,s1,s2", [(300, 64, 32), (257, 1000, 300), (130, 8192, 4096),
                                     (64, 16384, 2048), (50, 3, 4), (1, 128, 128)])
def test_srht_parity(dev, n, s1, s2):
    rng = np.random.default_rng(90 + s1)
    Z1 = rng.standard_normal((n, s1)).astype(np.float32)
    signs, sample, _ = WL.multilevel_draw(s1, s2, 1, rng)
    Z2 = krr.srht(_t(Z1, dev), _t(signs, dev), _t(sample, dev)).cpu().numpy()
    p = 1 << int(math.ceil(math.log2(s1))) if s1 > 1 else 1
    Zp = np.zeros((n, p))
    Zp[:, :s1] = Z1
    sp = np.ones(p)
    sp[:s1] = signs
    ref = SO.srht_apply(Zp, sp, sample)
    bound = (math.log2(p) + 2) * 2.0 ** -24 * np.abs(Z1).astype(np.float64).sum(1, keepdims=True) / math.sqrt(s2)
    assert np.all(np.abs(Z2 - ref) <= bound), np.max(np.abs(Z2 - ref) / bound)


def test_srht_full_sample_is_orthogonal(dev):
    """Sampling every coordinate: S is orthogonal, so Z2 Z2^T = Z1 Z1^T up to rounding."""
    rng = np.random.default_rng(95)
    Z1 = rng.standard_normal((40, 256)).astype(np.float32)
    signs, sample, _ = WL.multilevel_draw(256, 256, 1, rng)
    Z2 = krr.srht(_t(Z1, dev), _t(signs, dev), _t(sample, dev)).cpu().numpy().astype(np.float64)
    G1 = Z1.astype(np.float64) @ Z1.T.astype(np.float64)
    np.testing.assert_allclose(Z2 @ Z2.T, G1, rtol=0, atol=1e-5 * np.abs(G1).max())


@pytest.mark.parametrize("n,s2,s3", [(300, 512, 256), (1000, 100, 37), (129, 4096, 2048), (5, 33, 1)])
def test_gaussian_project_parity(dev, n, s2, s3):
    rng = np.random.default_rng(100 + s2)
    Z2 = rng.standard_normal((n, s2)).astype(np.float32)
    _, _, S3 = WL.multilevel_draw(s2, s2, s3, rng)
    Z3 = krr.gaussian_project(_t(Z2, dev), _t(S3, dev)).cpu().numpy()
    ref = SO.gaussian_project(Z2, S3)
    absprod = np.abs(Z2).astype(np.float64) @ np.abs(S3).astype(np.float64).T
    bound = (2.0 ** -21 + s2 * 2.0 ** -24) * absprod / math.sqrt(s3) + 2.0 ** -24 * np.abs(ref)
    assert np.all(np.abs(Z3 - ref) <= bound), np.max(np.abs(Z3 - ref) / bound)


@pytest.mark.parametrize("prec", ["fp64", "f16x3"])
def test_multilevel_preconditioned_solve(dev, prec):
    """Alg. 2 on the GPU: random Fourier features (s1) -> SRHT (s2) -> Gaussian projection (s3)
    -> factor -> PCG. Meets 1e-6 in the oracle's FP64 residual; the iteration count follows the
    oracle's PCG with the oracle's own three-level sketch of the same draws (FP64 product:
    within 2; mixed product: the first solve within 15 % + 5)."""
    w = WL.mixture_multi_rhs(n=3000, s=1024)
    s2, s3 = 512, 256
    signs, sample, S3 = WL.multilevel_draw(w.s, s2, s3, np.random.default_rng(7))
    X, Y = _t(w.X, dev), _t(w.Y, dev)
    Z1 = krr.features(X, _t(w.W, dev), _t(w.b, dev))
    Z2 = krr.srht(Z1, _t(signs, dev), _t(sample, dev))
    Z3 = krr.gaussian_project(Z2, _t(S3, dev))
    _, Ut = krr.precond_factor(Z3, w.lam)
    a, rep = krr.pcg_solve(X, w.sigma, w.lam, Ut, Y, tol=1e-6, prec=prec, refine=3)
    rel = O.relres_true(w.X, w.sigma, w.lam, a.cpu().numpy(), w.Y)
    assert rel.max() <= 1e-6, rel
    Zo1 = O.rff_features(w.X, w.W, w.b)
    Zo3 = SO.gaussian_project(SO.srht_apply(Zo1, signs, sample), S3)
    _, U = O.precond_factor(Zo3, w.lam)
    res = O.krr_pcg(w.X, w.sigma, w.lam, w.Y, U=U, tol=1e-6)
    if prec == "fp64":
        assert abs(rep.iters - res.iters) <= 2, (rep.iters, res.iters)
    else:
        _, rep0 = krr.pcg_solve(X, w.sigma, w.lam, Ut, Y, tol=1e-6, prec=prec, refine=0,
                                raise_on_error=False)
        assert rep0.converged_cols == w.m
        assert rep0.iters <= 1.15 * res.iters + 5, (rep0.iters, res.iters)
