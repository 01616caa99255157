"""GPU parity: every entry point of the C ABI against the CPU FP64 oracle on the same
seeded inputs, element by element where sizes allow and on sampled rows at full size.

Tolerances follow from the arithmetic of each path (derivations in the design notes):
  * mixed kernel product, per output entry i:
        |OUT_gpu - OUT_ref|_i <= tau * (|K| |V|)_i
    with tau = ln2 * (2 e_split + Kp 2^-24) * 4 c nu_max + 2^-22 + 16 2^-24, where
    e_split = 2^-22 (FP16 hi/lo) or 2^-16 (BF16 hi/lo), c = log2(e)/(2 sigma^2) and
    nu_max = max ||x||^2 (worst-case bound of the split products, FP32 accumulation over
    the Kp augmented components, exp2 rounding and FP32 partial sums of 16 terms);
  * FP64 kernel product: 1e-12 relative to (|K| |V|)_i;
  * solves: the FP64 true residual ||y - (K + lambda I) alpha|| / ||y|| computed by the
    oracle must meet the requested tolerance (1e-10 FP64, 1e-6 mixed).
"""
import math

import numpy as np
import pytest
import torch

import oracle as O
from paper_1611_03220_amd import krr
from paper_1611_03220_amd import workloads as WL

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


def _tau(prec, X1, X2, sigma, d):
    if prec == "fp64":
        return 1e-12
    e_split = 2.0 ** -22 if prec == "f16x3" else 2.0 ** -16
    kp = int(math.ceil((d + 2) / 32) * 32)
    c = math.log2(math.e) / (2 * sigma * sigma)
    nu = max(float((X1.astype(np.float64) ** 2).sum(1).max()), float((X2.astype(np.float64) ** 2).sum(1).max()))
    return LN2 * (2 * e_split + kp * 2.0 ** -24) * 4 * c * nu + 2.0 ** -22 + 16 * 2.0 ** -24


def _abs_bound(X1, X2, sigma, V, deriv):
    K = (O.gaussian_kernel_dsigma if deriv else O.gaussian_kernel)(X1, X2, sigma)
    return np.abs(K) @ np.abs(V)


MATMAT_CASES = [
    # n1, n2, d, m, square
    (300, 517, 54, 7, False),
    (64, 64, 8, 1, True),
    (1, 130, 3, 2, False),
    (257, 257, 30, 9, True),     # nine columns: hi and lo parts in separate operands
    (190, 333, 20, 8, False),    # eight columns: hi and lo parts packed in one operand
    (100, 2000, 126, 3, False),  # Kp = 128
    (70, 90, 254, 1, False),     # largest d of the register-resident mixed kernel
    (129, 65, 1, 5, False),
    # d + 2 past a 32-column step: Gaussian F16X3 rows without the norm columns (the norm
    # terms added in the epilogue), one, two and three 32-column steps, packed, split and
    # 32-column right-hand-side passes
    (300, 411, 64, 7, False),
    (257, 257, 32, 9, True),
    (190, 333, 96, 3, False),
    (150, 260, 63, 20, False),
]


@pytest.mark.parametrize("prec", ["f16x3", "bf16x3", "fp64"])
@pytest.mark.parametrize("case", MATMAT_CASES)
def test_matmat_parity(dev, prec, case):
    n1, n2, d, m, square = case
    rng = np.random.default_rng(n1 * 7 + n2 + d)
    X2 = rng.standard_normal((n2, d)).astype(np.float32)
    X1 = X2 if square else (1.3 * rng.standard_normal((n1, d))).astype(np.float32)
    V = rng.standard_normal((n2, m))
    sigma = 0.7 * math.sqrt(d)
    shift = 0.37 if square else 0.0
    out = krr.kernel_matmat(_t(X1, dev), _t(X2, dev), sigma, _t(V, dev), shift=shift, prec=prec)
    got = out.cpu().numpy()
    ref = O.kernel_matmat(X1, X2, sigma, V, shift=shift)
    bound = _tau(prec, X1, X2, sigma, d) * _abs_bound(X1, X2, sigma, V, False) + 1e-300
    if square:
        bound = bound + shift * 1e-15 * np.abs(V)
    assert np.all(np.abs(got - ref) <= bound), np.max(np.abs(got - ref) / bound)


@pytest.mark.parametrize("prec", ["f16x3", "fp64"])
@pytest.mark.parametrize("d", [20, 64])
def test_matmat_deriv_parity(dev, prec, d):
    rng = np.random.default_rng(5)
    X1 = rng.standard_normal((200, d)).astype(np.float32)
    X2 = rng.standard_normal((333, d)).astype(np.float32)
    V = rng.standard_normal((333, 4))
    sigma = 3.1 * math.sqrt(d / 20)
    got = krr.kernel_matmat(_t(X1, dev), _t(X2, dev), sigma, _t(V, dev), deriv=True, prec=prec).cpu().numpy()
    ref = O.kernel_matmat(X1, X2, sigma, V, deriv=True)
    # dk/dsigma = k * D / sigma^3: the relative error of D adds to that of k; D is formed as
    # -log2(k)/c, so its absolute error is that of S (bounded as in _tau) divided by c
    tau = _tau(prec, X1, X2, sigma, d)
    c = math.log2(math.e) / (2 * sigma ** 2)
    D = O.sq_dists(X1, X2)
    Kd = np.exp(-D / (2 * sigma ** 2))
    extra = (tau / LN2) / c * Kd / sigma ** 3 if prec != "fp64" else 1e-12 * Kd * (1 + D) / sigma ** 3
    bound = tau * (np.abs(O.gaussian_kernel_dsigma(X1, X2, sigma)) @ np.abs(V)) + extra @ np.abs(V)
    assert np.all(np.abs(got - ref) <= bound), np.max(np.abs(got - ref) / bound)


def test_matmat_deterministic(dev):
    rng = np.random.default_rng(6)
    X = _t(rng.standard_normal((3000, 16)).astype(np.float32), dev)
    V = _t(rng.standard_normal((3000, 3)), dev)
    a = krr.kernel_matmat(X, X, 4.0, V, shift=1.0)
    b = krr.kernel_matmat(X, X, 4.0, V, shift=1.0)
    assert torch.equal(a, b)


def test_matmat_full_size_sampled_rows(dev):
    """The benchmark's product (n = 65536, d = 54, m = 7, shift lambda) in its launch
    configuration, checked on 48 sampled rows against the oracle."""
    w = WL.mixture_multi_rhs()
    rng = np.random.default_rng(11)
    V = rng.standard_normal((w.n, w.m))
    X = _t(w.X, dev)
    got = krr.kernel_matmat(X, X, w.sigma, _t(V, dev), shift=w.lam).cpu().numpy()
    rows = np.sort(rng.choice(w.n, 48, replace=False))
    rows[-1] = w.n - 1  # ragged tail of the last tile
    ref = O.kernel_matmat(w.X, w.X, w.sigma, V, shift=w.lam, rows=rows)
    Kabs = O.gaussian_kernel(w.X[rows], w.X, w.sigma)
    bound = _tau("f16x3", w.X, w.X, w.sigma, w.d) * (Kabs @ np.abs(V)) + 1e-15 * w.lam * np.abs(V[rows])
    assert np.all(np.abs(got[rows] - ref) <= bound), np.max(np.abs(got[rows] - ref) / bound)


# ------------------------------------------------------------------ features
def test_features_parity(dev):
    w = WL.plain_fp64()
    Z = krr.features(_t(w.X, dev), _t(w.W, dev), _t(w.b, dev)).cpu().numpy()
    ref = O.rff_features(w.X, w.W, w.b)
    # argument error of the split product (3 products, FP32 accumulate over d_pad = 32
    # terms) plus the FP32 rounding of the argument and of cos
    XW = np.abs(w.X.astype(np.float64)) @ np.abs(w.W.astype(np.float64))
    e_arg = (2 * 2.0 ** -22 + 32 * 2.0 ** -24) * XW + 2.0 ** -23 * (XW + 2 * np.pi)
    bound = math.sqrt(2.0 / w.s) * (e_arg + 2.0 ** -22)
    assert np.all(np.abs(Z - ref) <= bound), np.max(np.abs(Z - ref) / bound)


def test_features_ragged_shapes(dev):
    rng = np.random.default_rng(8)
    X = rng.standard_normal((77, 5)).astype(np.float32)
    W = rng.standard_normal((5, 45)).astype(np.float32)
    b = rng.uniform(0, 2 * np.pi, 45).astype(np.float32)
    Z = krr.features(_t(X, dev), _t(W, dev), _t(b, dev)).cpu().numpy()
    np.testing.assert_allclose(Z, O.rff_features(X, W, b), rtol=0, atol=2e-6 * math.sqrt(2 / 45) * 40)


# ------------------------------------------------------------- preconditioner
def _factor_case(n=2000, d=8, s=200, lam=2.0, seed=0):
    w = WL.plain_fp64(n=n, d=d, s=s)
    Z = O.rff_features(w.X, w.W, w.b).astype(np.float32)
    return Z, lam


@pytest.mark.parametrize("shape", [(2000, 200), (1000, 130), (700, 64), (3000, 520), (3000, 400),
                                   (2500, 1100)])
def test_precond_factor_parity(dev, shape):
    n, s = shape
    Z, lam = _factor_case(n=n, s=s)
    C, Ut = krr.precond_factor(_t(Z, dev), lam)
    C, Ut = C.cpu().numpy(), Ut.cpu().numpy().astype(np.float64)
    Z64 = Z.astype(np.float64)
    G = Z64.T @ Z64 + lam * np.eye(s)
    assert np.allclose(np.triu(C, 1), 0) and (np.diag(C) > 0).all()
    # backward error of the factor: Gram on split MFMA with FP32 sums of n/nsplit terms
    back = np.linalg.norm(C @ C.T - G) / np.linalg.norm(G)
    assert back <= 4 * (2 * 2.0 ** -22 + math.sqrt(n) * 2.0 ** -24), back
    # Ut solves C Ut^T = Z^T (one GEMM with the FP64 inverse, FP32 output)
    rel = np.linalg.norm(C @ Ut.T - Z64.T) / np.linalg.norm(Z64)
    assert rel <= 8 * (2 * 2.0 ** -22 + math.sqrt(s) * 2.0 ** -24) * np.linalg.cond(C), rel
    # the Woodbury operator built from the GPU factor equals (Z Z^T + lam I)^{-1}
    v = np.random.default_rng(1).standard_normal((n, 2))
    got = (v - Ut @ (Ut.T @ v)) / lam
    ref = np.linalg.solve(Z64 @ Z64.T + lam * np.eye(n), v)
    kappa = np.linalg.cond(Z64 @ Z64.T + lam * np.eye(n))
    assert np.linalg.norm(got - ref) / np.linalg.norm(ref) <= kappa * 8 * back + 1e-12


def test_precond_factor_not_spd(dev):
    Z, lam = _factor_case(n=500, s=64)
    Z[10, 3] = np.nan
    with pytest.raises(krr.KRRError) as e:
        krr.precond_factor(_t(Z, dev), lam)
    assert e.value.status == krr.E_NOT_SPD and e.value.info >= 1


# ------------------------------------------------------------------ solves
@pytest.mark.parametrize("n,s,m,ldr", [(3000, 256, 7, 7), (1000, 200, 1, 3), (777, 37, 20, 24),
                                       (129, 64, 16, 16), (5000, 1000, 4, 4)])
def test_precond_apply_parity(dev, n, s, m, ldr):
    """Woodbury apply against the oracle on the same Ut: FP64 sums of exact FP32 products,
    bounded by 4 (n + s) u64 (|Ut| (|Ut|^T |R|) + |R|) / lambda_p element-wise."""
    rng = np.random.default_rng(n + s + m)
    Ut = (rng.standard_normal((n, s)) / math.sqrt(n)).astype(np.float32)
    Rfull = rng.standard_normal((n, ldr))
    R = Rfull[:, :m]
    lam_p = 0.37
    got = krr.precond_apply(_t(Ut, dev), lam_p, _t(Rfull, dev)[:, :m])  # row stride ldr
    ref = O.precond_apply(Ut.astype(np.float64).T, lam_p, R)
    U = np.abs(Ut.astype(np.float64))
    bound = 4 * (n + s) * 2.0 ** -53 * (U @ (U.T @ np.abs(R)) + np.abs(R)) / lam_p
    assert np.all(np.abs(got.cpu().numpy() - ref) <= bound + 1e-300)


def test_precond_apply_benchmark_size(dev):
    """The benchmark's preconditioner (n = 65536, s = 2048, m = 7) applied to a random
    residual, against the oracle's apply on the same Ut."""
    w = WL.mixture_multi_rhs()
    X = _t(w.X, dev)
    Z = krr.features(X, _t(w.W, dev), _t(w.b, dev))
    _, Ut = krr.precond_factor(Z, w.lam)
    R = np.random.default_rng(5).standard_normal((w.n, w.m))
    got = krr.precond_apply(Ut, w.lam, _t(R, dev)).cpu().numpy()
    Uh = Ut.cpu().numpy().astype(np.float64)
    ref = O.precond_apply(Uh.T, w.lam, R)
    U = np.abs(Uh)
    bound = 4 * (w.n + w.s) * 2.0 ** -53 * (U @ (U.T @ np.abs(R)) + np.abs(R)) / w.lam
    assert np.all(np.abs(got - ref) <= bound)


def test_pcg_fp64_plain_workload(dev):
    """n = 2000, d = 8, s = 200, lambda = 2, FP64 to 1e-10 (the plain-method workload)."""
    w = WL.plain_fp64()
    X = _t(w.X, dev)
    Z = krr.features(X, _t(w.W, dev), _t(w.b, dev))
    _, Ut = krr.precond_factor(Z, w.lam)
    alpha, rep = krr.pcg_solve(X, w.sigma, w.lam, Ut, _t(w.Y, dev), tol=1e-10, prec="fp64")
    a = alpha.cpu().numpy()
    assert O.relres_true(w.X, w.sigma, w.lam, a, w.Y).max() <= 1e-10
    assert max(rep.relres_true) <= 1e-10
    K = O.gaussian_kernel(w.X, w.X, w.sigma)
    A = K + w.lam * np.eye(w.n)
    ref = np.linalg.solve(A, w.Y)
    kappa = np.linalg.cond(A)
    assert np.linalg.norm(a - ref) / np.linalg.norm(ref) <= kappa * 1e-10
    # the oracle's PCG with its own features and factor (same W, b) takes the same steps
    Zo = O.rff_features(w.X, w.W, w.b)
    _, Uo = O.precond_factor(Zo, w.lam)
    orc = O.krr_pcg(w.X, w.sigma, w.lam, w.Y, U=Uo, tol=1e-10)
    assert abs(rep.iters - orc.iters) <= 2, (rep.iters, orc.iters)


@pytest.mark.parametrize("prec", ["f16x3", "fp64"])
def test_pcg_mixture_reduced(dev, prec):
    """The multi-RHS workload recipe at n = 6000, s = 384: every column reaches 1e-6 in the
    oracle's FP64 true residual. The mixed product's floor sits near 1e-6 on this smaller,
    relatively more ill-conditioned instance (lambda = 0.6), so the mixed solve runs with
    FP64-residual refinement, which is how it certifies the tolerance."""
    w = WL.mixture_multi_rhs(n=6000, s=384)
    X = _t(w.X, dev)
    Z = krr.features(X, _t(w.W, dev), _t(w.b, dev))
    _, Ut = krr.precond_factor(Z, w.lam)
    alpha, rep = krr.pcg_solve(X, w.sigma, w.lam, Ut, _t(w.Y, dev), tol=1e-6, prec=prec,
                               refine=2 if prec != "fp64" else 0)
    a = alpha.cpu().numpy()
    rel = O.relres_true(w.X, w.sigma, w.lam, a, w.Y)
    assert rel.max() <= 1e-6, rel
    np.testing.assert_allclose(rep.relres_true, rel, rtol=1e-3, atol=1e-12)
    # same preconditioner in the oracle's FP64 PCG: iteration counts agree closely
    # (refinement adds the iterations of its correction solves)
    Uo = Ut.cpu().numpy().astype(np.float64).T
    orc = O.krr_pcg(w.X, w.sigma, w.lam, w.Y, U=Uo, tol=1e-6)
    first = rep.iters if rep.refine_steps == 0 else None
    if first is not None:
        assert abs(first - orc.iters) <= max(2, orc.iters // 10), (rep.iters, orc.iters)
    else:
        assert orc.iters - 2 <= rep.iters <= 2 * orc.iters, (rep.iters, orc.iters)


def test_pcg_unpreconditioned_and_lambda_p(dev):
    w = WL.mixture_multi_rhs(n=1500, s=128)
    X, Y = _t(w.X, dev), _t(w.Y, dev)
    a0, r0 = krr.pcg_solve(X, w.sigma, w.lam, None, Y, tol=1e-8, prec="fp64", use_precond=False)
    assert O.relres_true(w.X, w.sigma, w.lam, a0.cpu().numpy(), w.Y).max() <= 1e-8
    Z = krr.features(X, _t(w.W, dev), _t(w.b, dev))
    _, Ut = krr.precond_factor(Z, 10 * w.lam)
    a1, r1 = krr.pcg_solve(X, w.sigma, w.lam, Ut, Y, tol=1e-8, prec="fp64", lambda_p=10 * w.lam)
    assert O.relres_true(w.X, w.sigma, w.lam, a1.cpu().numpy(), w.Y).max() <= 1e-8
    assert r1.iters < r0.iters


def test_pcg_breakdown_and_noconv(dev):
    w = WL.mixture_multi_rhs(n=1200, s=96)
    Y = w.Y[:, :3].copy()
    Y[5, 1] = np.nan
    X = _t(w.X, dev)
    Z = krr.features(X, _t(w.W, dev), _t(w.b, dev))
    _, Ut = krr.precond_factor(Z, w.lam)
    with pytest.raises(krr.KRRError) as e:
        krr.pcg_solve(X, w.sigma, w.lam, Ut, _t(Y, dev), tol=1e-6)
    rep = e.value.report
    assert e.value.status == krr.E_BREAKDOWN and rep.breakdown_cols == 1 and rep.converged_cols == 2
    a, rep = krr.pcg_solve(X, w.sigma, w.lam, Ut, _t(w.Y, dev), tol=1e-12, max_iter=1,
                           raise_on_error=False)
    assert rep.status == krr.E_NO_CONV and rep.iters == 1
    assert torch.isfinite(a).all() and a.abs().sum() > 0


def test_pcg_warm_start_resume(dev):
    w = WL.mixture_multi_rhs(n=2000, s=128)
    X, Y = _t(w.X, dev), _t(w.Y, dev)
    Z = krr.features(X, _t(w.W, dev), _t(w.b, dev))
    _, Ut = krr.precond_factor(Z, w.lam)
    a1, r1 = krr.pcg_solve(X, w.sigma, w.lam, Ut, Y, tol=1e-8, max_iter=4, prec="fp64", raise_on_error=False)
    assert r1.status == krr.E_NO_CONV
    a2, r2 = krr.pcg_solve(X, w.sigma, w.lam, Ut, Y, tol=1e-8, prec="fp64", alpha0=a1)
    assert O.relres_true(w.X, w.sigma, w.lam, a2.cpu().numpy(), w.Y).max() <= 1e-8


def test_refinement_below_mixed_floor(dev):
    """Tolerance below the mixed product's floor: FP64-residual refinement reaches it."""
    w = WL.mixture_multi_rhs(n=3000, s=256)
    X, Y = _t(w.X, dev), _t(w.Y, dev)
    Z = krr.features(X, _t(w.W, dev), _t(w.b, dev))
    _, Ut = krr.precond_factor(Z, w.lam)
    a, rep = krr.pcg_solve(X, w.sigma, w.lam, Ut, Y, tol=1e-10, prec="f16x3", refine=4)
    assert rep.refine_steps >= 1
    assert O.relres_true(w.X, w.sigma, w.lam, a.cpu().numpy(), w.Y).max() <= 1e-10


def test_pcg_full_size_sampled(dev):
    """The benchmark solve (n = 65536, m = 7, s = 2048) to 1e-6: the GPU's FP64 true residual
    meets the tolerance and the oracle's residual on sampled rows agrees with it."""
    w = WL.mixture_multi_rhs()
    X, Y = _t(w.X, dev), _t(w.Y, dev)
    Z = krr.features(X, _t(w.W, dev), _t(w.b, dev))
    _, Ut = krr.precond_factor(Z, w.lam)
    alpha, rep = krr.pcg_solve(X, w.sigma, w.lam, Ut, Y, tol=1e-6, refine=2)
    assert max(rep.relres_true) <= 1e-6
    a = alpha.cpu().numpy()
    rows = np.sort(np.random.default_rng(3).choice(w.n, 256, replace=False))
    rows[-1] = w.n - 1
    _check_fp64_residual(X, w, alpha, a, rows, rep, dev)


def _check_fp64_residual(X, w, alpha, a, rows, rep, dev, Kr=None):
    """The library's FP64 residual, element by element: its FP64 product (K + lambda I) alpha
    on the sampled rows equals the oracle's within 1e-12 (|K| |alpha| + lambda |alpha|), and
    the per-column norm of Y - (K + lambda I) alpha over all rows, formed from that product,
    is the relres_true the solve reported."""
    prod = krr.kernel_matmat(X, X, w.sigma, alpha, shift=w.lam, prec="fp64").cpu().numpy()
    if Kr is None:
        Kr = O.gaussian_kernel(w.X[rows], w.X, w.sigma)
    ref = Kr @ a + w.lam * a[rows]
    bound = 1e-12 * (np.abs(Kr) @ np.abs(a) + w.lam * np.abs(a[rows]))
    assert np.all(np.abs(prod[rows] - ref) <= bound), np.max(np.abs(prod[rows] - ref) / bound)
    rel = np.linalg.norm(w.Y - prod, axis=0) / np.linalg.norm(w.Y, axis=0)
    np.testing.assert_allclose(rel, rep.relres_true, rtol=1e-8)
    # the oracle's own residual on the sampled rows, as a norm estimate
    est = np.linalg.norm(w.Y[rows] - ref, axis=0) / np.linalg.norm(w.Y[rows], axis=0)
    assert est.max() <= 4e-6, est


# -------------------------------------------------------------------- grad
@pytest.mark.parametrize("prec", ["fp64", "f16x3"])
def test_grad_parity(dev, prec):
    rng = np.random.default_rng(9)
    n, d, m = 700, 12, 3
    X = rng.standard_normal((n, d)).astype(np.float32)
    al = rng.standard_normal((n, m))
    ab = rng.standard_normal((n, m))
    sigma = 2.5
    ds, dl = krr.grad(_t(X, dev), sigma, _t(al, dev), _t(ab, dev), prec=prec)
    ref_s = -float(np.sum(ab * O.kernel_matmat(X, X, sigma, al, deriv=True)))
    ref_l = -float(np.sum(ab * al))
    scale = float(np.sum(np.abs(ab) * (np.abs(O.gaussian_kernel_dsigma(X, X, sigma)) @ np.abs(al))))
    tol = 1e-12 if prec == "fp64" else 1e-5
    assert abs(ds - ref_s) <= tol * scale
    assert dl == pytest.approx(ref_l, rel=1e-13)


# ------------------------------------------------------------ large d, many RHS
@pytest.mark.parametrize("case", [(150, 333, 300, 5), (200, 257, 440, 40), (64, 128, 130, 33)])
def test_matmat_large_d_and_many_columns(dev, case):
    """d beyond the register-resident kernel (both operands through LDS) and m > 32
    (several column passes)."""
    n1, n2, d, m = case
    _large_d_case(dev, n1, n2, d, m)


@pytest.mark.parametrize("case", [(150, 333, 300, 5), (200, 257, 440, 40), (64, 300, 784, 10),
                                  (129, 65, 136, 17), (40, 50, 16500, 2)])
def test_matmat_fp64_large_d(dev, case):
    """FP64 product with d > 128 (FP32 coordinates through LDS, FP64 MFMA): 1e-12 relative to
    (|K| |V|)_i, value and sigma-derivative, ragged row and column counts, two column passes
    (m = 40) and a long k loop (d = 16500)."""
    n1, n2, d, m = case
    rng = np.random.default_rng(d + m + 1)
    X1 = rng.standard_normal((n1, d)).astype(np.float32)
    X2 = rng.standard_normal((n2, d)).astype(np.float32)
    V = rng.standard_normal((n2, m))
    sigma = 0.8 * math.sqrt(d)
    for deriv in (False, True):
        got = krr.kernel_matmat(_t(X1, dev), _t(X2, dev), sigma, _t(V, dev), deriv=deriv,
                                prec="fp64").cpu().numpy()
        ref = O.kernel_matmat(X1, X2, sigma, V, deriv=deriv)
        bound = 1e-12 * _abs_bound(X1, X2, sigma, V, deriv)
        assert np.all(np.abs(got - ref) <= bound), (deriv, np.max(np.abs(got - ref) / bound))


def test_matmat_fp64_wide_dynamic_range(dev):
    """FP64 product (integer-slice inner products for d <= 128) on rows whose entries span
    30 binades, so the fixed-point slices round the smallest ones, with d over one 64-wide
    chunk, a zero row and duplicate points: 1e-12 relative to (|K| |V|)_i, value and
    sigma-derivative."""
    rng = np.random.default_rng(11)
    for n1, n2, d, m in [(150, 211, 40, 3), (97, 130, 100, 18)]:
        scales = 2.0 ** rng.integers(-20, 10, size=d)
        X1 = (rng.standard_normal((n1, d)) * scales).astype(np.float32)
        X2 = (rng.standard_normal((n2, d)) * scales).astype(np.float32)
        X1[3] = 0.0
        X2[5] = X2[7]
        X1[9] = X2[7]
        V = rng.standard_normal((n2, m))
        sigma = 0.8 * float(np.sqrt((scales ** 2).sum()))
        for deriv in (False, True):
            got = krr.kernel_matmat(_t(X1, dev), _t(X2, dev), sigma, _t(V, dev), deriv=deriv,
                                    prec="fp64").cpu().numpy()
            ref = O.kernel_matmat(X1, X2, sigma, V, deriv=deriv)
            bound = 1e-12 * _abs_bound(X1, X2, sigma, V, deriv) + 1e-300
            assert np.all(np.abs(got - ref) <= bound), (d, deriv, np.max(np.abs(got - ref) / bound))


def test_matmat_fp64_nan_point_propagates(dev):
    """A NaN coordinate makes every output of the FP64 product NaN, as in the oracle (every
    row meets the NaN point); the other rows of a product without it stay finite."""
    rng = np.random.default_rng(12)
    X = rng.standard_normal((70, 9)).astype(np.float32)
    V = rng.standard_normal((70, 2))
    X[13, 4] = np.nan
    got = krr.kernel_matmat(_t(X, dev), _t(X, dev), 3.0, _t(V, dev), prec="fp64").cpu().numpy()
    ref = O.kernel_matmat(X, X, 3.0, V)
    assert np.isnan(ref).all() and np.isnan(got).all()
    got2 = krr.kernel_matmat(_t(X[:13], dev), _t(X[14:], dev), 3.0, _t(V[14:], dev),
                             prec="fp64").cpu().numpy()
    assert np.isfinite(got2).all()


def _large_d_case(dev, n1, n2, d, m):
    rng = np.random.default_rng(d + m)
    X1 = rng.standard_normal((n1, d)).astype(np.float32)
    X2 = rng.standard_normal((n2, d)).astype(np.float32)
    V = rng.standard_normal((n2, m))
    sigma = 0.8 * math.sqrt(d)
    for deriv in (False, True):
        got = krr.kernel_matmat(_t(X1, dev), _t(X2, dev), sigma, _t(V, dev), deriv=deriv).cpu().numpy()
        ref = O.kernel_matmat(X1, X2, sigma, V, deriv=deriv)
        tau = _tau("f16x3", X1, X2, sigma, d)
        if deriv:
            c = math.log2(math.e) / (2 * sigma ** 2)
            Kd = O.gaussian_kernel(X1, X2, sigma)
            bound = tau * (np.abs(O.gaussian_kernel_dsigma(X1, X2, sigma)) @ np.abs(V)) \
                + ((tau / LN2) / c * Kd / sigma ** 3) @ np.abs(V)
        else:
            bound = tau * _abs_bound(X1, X2, sigma, V, False)
        assert np.all(np.abs(got - ref) <= bound), (deriv, np.max(np.abs(got - ref) / bound))


# -------------------------------------------------------- differentiation
def _diff_workload():
    return WL.correlated_differentiation(n=3072, n_val=384, d=440, k=147, s=256)


@pytest.mark.parametrize("prec,deriv_prec", [("fp64", "fp64"), ("f16x3", "fp64"), ("f16x3", "f16x3")])
def test_validation_gradient_matches_oracle(dev, prec, deriv_prec):
    """The differentiation workload's recipe (d = 440, 147 classes) at n = 3072 + 384:
    validation loss and its sigma / lambda gradients through the adjoint PCG against the
    oracle's dense FP64 adjoint gradients (bound: 1e-4 relative), with the dK/dsigma
    products in FP64 (the default) or mixed (measured within 5e-6 on this recipe)."""
    from paper_1611_03220_amd import autograd as KA
    w = _diff_workload()
    Xtr, Xv = _t(w.X, dev), _t(w.Xv, dev)
    Ytr, Yv = _t(w.Y, dev), _t(w.Yv, dev)
    Z = krr.features(Xtr, _t(w.W, dev), _t(w.b, dev))
    _, Ut = krr.precond_factor(Z, w.lam)
    sig = torch.tensor(w.sigma, dtype=torch.float64, device=dev, requires_grad=True)
    lam = torch.tensor(w.lam, dtype=torch.float64, device=dev, requires_grad=True)
    L = KA.validation_loss(Xtr, Ytr, Xv, Yv, sig, lam, Ut, prec=prec, deriv_prec=deriv_prec,
                           tol=1e-9, refine=3)
    L.backward()
    ref = O.validation_loss_and_grads(w.X, w.Y, w.Xv, w.Yv, w.sigma, w.lam)
    assert float(L) == pytest.approx(ref["loss"], rel=1e-6)
    assert float(sig.grad) == pytest.approx(ref["dL_dsigma"], rel=1e-4)
    assert float(lam.grad) == pytest.approx(ref["dL_dlambda"], rel=1e-4)


def test_validation_gradient_central_differences(dev):
    """Central differences of the GPU FP64 loss in log sigma and log lambda (h = 1e-4) agree
    with the adjoint gradient of the mixed path."""
    from paper_1611_03220_amd import autograd as KA
    w = WL.correlated_differentiation(n=2048, n_val=256, d=440, k=20, s=192)
    Xtr, Xv = _t(w.X, dev), _t(w.Xv, dev)
    Ytr, Yv = _t(w.Y, dev), _t(w.Yv, dev)
    Z = krr.features(Xtr, _t(w.W, dev), _t(w.b, dev))
    _, Ut = krr.precond_factor(Z, w.lam)

    def loss(s_, l_, prec):
        return float(KA.validation_loss(Xtr, Ytr, Xv, Yv, s_, l_, Ut, prec=prec, tol=1e-12,
                                        max_iter=2000))

    sig = torch.tensor(w.sigma, dtype=torch.float64, device=dev, requires_grad=True)
    lam = torch.tensor(w.lam, dtype=torch.float64, device=dev, requires_grad=True)
    KA.validation_loss(Xtr, Ytr, Xv, Yv, sig, lam, Ut, prec="f16x3", tol=1e-9, refine=3).backward()
    h = 1e-4
    fd_s = (loss(w.sigma * math.exp(h), w.lam, "fp64") - loss(w.sigma * math.exp(-h), w.lam, "fp64")) / (2 * h) / w.sigma
    fd_l = (loss(w.sigma, w.lam * math.exp(h), "fp64") - loss(w.sigma, w.lam * math.exp(-h), "fp64")) / (2 * h) / w.lam
    assert float(sig.grad) == pytest.approx(fd_s, rel=1e-4)
    assert float(lam.grad) == pytest.approx(fd_l, rel=1e-4)


# ------------------------------------------------------------ full-size workloads
def test_pixels_full_size_sampled(dev):
    """The large dense-feature workload (n = 262144, d = 784, 10 right-hand sides,
    s = 8192) at full size: the kernel product on sampled rows against the oracle (same
    bound as the small cases) and the solve to 1e-6, whose FP64 true residual the oracle's
    residual on sampled rows confirms."""
    w = WL.pixels()
    X, Y = _t(w.X, dev), _t(w.Y, dev)
    rows = np.sort(np.random.default_rng(11).choice(w.n, 40, replace=False))
    rows[-1] = w.n - 1
    V = np.random.default_rng(12).standard_normal((w.n, w.m))
    got = krr.kernel_matmat(X, X, w.sigma, _t(V, dev)).cpu().numpy()[rows]
    Kr = O.gaussian_kernel(w.X[rows], w.X, w.sigma)
    ref = Kr @ V
    tau = _tau("f16x3", w.X[rows], w.X, w.sigma, w.d)
    assert np.all(np.abs(got - ref) <= tau * (np.abs(Kr) @ np.abs(V)))
    Z = krr.features(X, _t(w.W, dev), _t(w.b, dev))
    _, Ut = krr.precond_factor(Z, w.lam)
    del Z
    alpha, rep = krr.pcg_solve(X, w.sigma, w.lam, Ut, Y, tol=1e-6, refine=3)
    assert max(rep.relres_true) <= 1e-6
    a = alpha.cpu().numpy()
    _check_fp64_residual(X, w, alpha, a, rows, rep, dev, Kr=Kr)


def test_differentiation_full_size_central_differences(dev):
    """The differentiation workload at full size (n = 131072 + 16384, d = 440, 147 columns,
    s = 4096): the adjoint gradients of the mixed path against central differences (log
    sigma, log lambda, h = 1e-4) of the loss evaluated with refined solves to 1e-10 and the
    FP64 validation product; 1e-4 relative."""
    from paper_1611_03220_amd import autograd as KA
    w = WL.correlated_differentiation()
    Xtr, Xv = _t(w.X, dev), _t(w.Xv, dev)
    Ytr, Yv = _t(w.Y, dev), _t(w.Yv, dev)
    Z = krr.features(Xtr, _t(w.W, dev), _t(w.b, dev))
    _, Ut = krr.precond_factor(Z, w.lam)
    del Z
    sig = torch.tensor(w.sigma, dtype=torch.float64, device=dev, requires_grad=True)
    lam = torch.tensor(w.lam, dtype=torch.float64, device=dev, requires_grad=True)
    KA.validation_loss(Xtr, Ytr, Xv, Yv, sig, lam, Ut, tol=1e-9, refine=4).backward()

    def loss(s_, l_):
        with torch.no_grad():
            return float(KA.validation_loss(Xtr, Ytr, Xv, Yv, s_, l_, Ut, tol=1e-10, refine=6))

    h = 1e-4
    fd_s = (loss(w.sigma * math.exp(h), w.lam) - loss(w.sigma * math.exp(-h), w.lam)) / (2 * h) / w.sigma
    fd_l = (loss(w.sigma, w.lam * math.exp(h)) - loss(w.sigma, w.lam * math.exp(-h))) / (2 * h) / w.lam
    assert float(sig.grad) == pytest.approx(fd_s, rel=1e-4)
    assert float(lam.grad) == pytest.approx(fd_l, rel=1e-4)
