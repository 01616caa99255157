"""CPU pins of the sketching oracle (polynomial kernel, CountSketch / TensorSketch, SRHT,
Gaussian projection, the Thm. 4 test) against what the paper and the mathematics fix:
hand-computed values, exact expectations over every sign table, the fast (FFT) evaluation
against the definition, Thm. 1's spectral bound and iteration count, closed forms."""
import itertools
import math
import os

import numpy as np
import pytest

import oracle as O
from oracle import sketch_oracle as SO


def _golden(golden_dir):
    vals = {}
    with open(os.path.join(golden_dir, "sketch_values.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                name, v = line.split()[:2]
                vals[name] = np.array([float(t) for t in v.split(",")])
    return vals


# --------------------------------------------------------------------- polynomial
def test_polynomial_kernel_hand_values(golden_dir):
    g = _golden(golden_dir)
    k = SO.polynomial_kernel(np.array([[1.0, 2.0]]), np.array([[3.0, -1.0]]), 0.5, 1.0, 3)
    assert k[0, 0] == g["poly_a"][0]
    k = SO.polynomial_kernel(np.array([[0.5, 0.5, 1.0]]), np.array([[2.0, -4.0, 0.25]]), 2.0, 0.5, 3)
    assert k[0, 0] == g["poly_b"][0]


def test_polynomial_kernel_is_psd_and_symmetric():
    rng = np.random.default_rng(1)
    X = rng.standard_normal((80, 5))
    for q, c in ((1, 0.0), (2, 1.0), (3, 0.5), (4, 2.0)):
        K = SO.polynomial_kernel(X, X, 0.3, c, q)
        assert np.array_equal(K, K.T)
        ev = np.linalg.eigvalsh(K)
        assert ev[0] >= -1e-10 * ev[-1], (q, ev[0])


def test_augmented_homogeneous_kernel_equals_nonhomogeneous():
    """Remark after Thm. 1: one constant feature turns (x^T z)^q into (gamma x^T z + c)^q."""
    rng = np.random.default_rng(2)
    X, Z = rng.standard_normal((30, 4)), rng.standard_normal((20, 4))
    A, B = SO.poly_augment(X, 0.7, 1.3), SO.poly_augment(Z, 0.7, 1.3)
    np.testing.assert_allclose(SO.polynomial_kernel(A, B, 1.0, 0.0, 3),
                               SO.polynomial_kernel(X, Z, 0.7, 1.3, 3), rtol=1e-12)


def test_poly_matmat_blocked_equals_dense_and_rows():
    rng = np.random.default_rng(3)
    X, V = rng.standard_normal((150, 6)), rng.standard_normal((150, 3))
    K = SO.polynomial_kernel(X, X, 0.2, 1.0, 3)
    out = SO.poly_kernel_matmat(X, X, 0.2, 1.0, 3, V, shift=0.4, block=37)
    np.testing.assert_allclose(out, K @ V + 0.4 * V, rtol=1e-12, atol=1e-12)
    rows = np.array([5, 77, 149])
    np.testing.assert_allclose(SO.poly_kernel_matmat(X, X, 0.2, 1.0, 3, V, shift=0.4, rows=rows),
                               out[rows], rtol=1e-13)


def test_poly_solve_constant_kernel_sherman_morrison():
    """gamma = 0: K = c^q 1 1^T, so (K + lambda I)^{-1} y = (y - 1 c^q (1^T y)/(lambda + n c^q))/lambda."""
    rng = np.random.default_rng(4)
    n, lam, c, q = 60, 0.3, 1.5, 3
    X, y = rng.standard_normal((n, 3)), rng.standard_normal(n)
    got = SO.poly_solve_dense(X, 0.0, c, q, lam, y)
    cq = c ** q
    ref = (y - cq * y.sum() / (lam + n * cq)) / lam
    np.testing.assert_allclose(got, ref, rtol=1e-10)


# ---------------------------------------------------------------------- sketches
def test_count_sketch_hand_value(golden_dir):
    g = _golden(golden_dir)
    z = SO.count_sketch([1, 2, 3, 4], [0, 2, 0, 1], [1, -1, -1, 1], 3)
    np.testing.assert_array_equal(z, g["cs_a"])


def test_tensor_sketch_hand_value_both_evaluations(golden_dir):
    g = _golden(golden_dir)
    h = np.array([[0, 1], [2, 2]])
    sg = np.array([[1, -1], [1, 1]])
    x = np.array([[1.0, 2.0]])
    np.testing.assert_array_equal(SO.tensor_sketch_dense(x, h, sg, 3)[0], g["ts_a"])
    np.testing.assert_allclose(SO.tensor_sketch_fft(x, h, sg, 3)[0], g["ts_a"], atol=1e-12)


def test_monomials_inner_product_is_the_kernel():
    rng = np.random.default_rng(5)
    x, z = rng.standard_normal(4), rng.standard_normal(4)
    for q in (1, 2, 3):
        assert SO.monomials(x, q) @ SO.monomials(z, q) == pytest.approx((x @ z) ** q, rel=1e-12)


@pytest.mark.parametrize("q,d,s", [(1, 4, 3), (2, 3, 4), (3, 2, 5)])
def test_tensor_sketch_exact_expectation_over_all_signs(q, d, s):
    """For any fixed hashes, the average of <phi(x), phi(z)> over every sign table equals
    (x^T z)^q exactly: distinct monomials carry independent signs (Sec. 2.2). Reading
    g_2(i_1) for g_2(i_2), or dropping a sign, fails this."""
    rng = np.random.default_rng(6 + q)
    x, z = rng.standard_normal(d), rng.standard_normal(d)
    h = rng.integers(0, s, size=(q, d))
    acc, cnt = 0.0, 0
    for bits in itertools.product((1.0, -1.0), repeat=q * d):
        sg = np.array(bits).reshape(q, d)
        P = SO.tensor_sketch_dense(np.stack([x, z]), h, sg, s)
        acc += P[0] @ P[1]
        cnt += 1
    assert acc / cnt == pytest.approx((x @ z) ** q, rel=1e-10, abs=1e-12)


@pytest.mark.parametrize("q,d,s", [(2, 5, 16), (3, 3, 8), (2, 4, 7)])
def test_tensor_sketch_fft_equals_definition(q, d, s):
    rng = np.random.default_rng(10 + q + s)
    X = rng.standard_normal((6, d))
    h = rng.integers(0, s, size=(q, d))
    sg = rng.choice([-1.0, 1.0], size=(q, d))
    np.testing.assert_allclose(SO.tensor_sketch_fft(X, h, sg, s), SO.tensor_sketch_dense(X, h, sg, s),
                               atol=1e-12 * (1 + np.abs(X).max() ** q * d ** q))


def test_tensor_sketch_multiplication_lemma_monte_carlo():
    """Lemma (ANW14) behind Thm. 1: E||A S^T S B^T - A B^T||_F^2 <= (2 + 3^q)/s ||A||_F^2 ||B||_F^2;
    the Monte Carlo mean over 300 seeded draws stays below the bound, and the mean of
    Z Z^T is K within the Monte Carlo error."""
    rng = np.random.default_rng(20)
    q, d, s, n = 2, 4, 64, 6
    X = rng.standard_normal((n, d)) / math.sqrt(d)
    Vq = np.stack([SO.monomials(x, q) for x in X])
    K = Vq @ Vq.T
    errs, mean = [], np.zeros((n, n))
    for _ in range(300):
        h = rng.integers(0, s, size=(q, d))
        sg = rng.choice([-1.0, 1.0], size=(q, d))
        Z = SO.tensor_sketch_fft(X, h, sg, s)
        errs.append(np.sum((Z @ Z.T - K) ** 2))
        mean += Z @ Z.T / 300
    bound = (2 + 3 ** q) / s * np.sum(Vq ** 2) ** 2
    assert np.mean(errs) <= bound
    se = math.sqrt(np.mean(errs) / 300)
    assert np.linalg.norm(mean - K) <= 5 * se


def test_theorem1_spectrum_and_iteration_count():
    """Thm. 1: with ||Q S^T S Q^T - Q Q^T||_2 <= 1/2 (what s >= 4 (2 + 3^q) s_lambda^2 / delta buys),
    (2/3)(Z Z^T + lambda I) <= K + lambda I <= 2 (Z Z^T + lambda I), so the preconditioned
    spectrum lies in [1/2, 3/2] (kappa <= 3) and T = ceil(sqrt(3)/2 ln(2/eps)) PCG steps
    reach ||c_T - c||_A <= eps ||c||_A."""
    rng = np.random.default_rng(21)
    q, d, n, lam = 2, 3, 40, 4.0
    X = rng.standard_normal((n, d)) / math.sqrt(d)
    Vq = np.stack([SO.monomials(x, q) for x in X])
    K = Vq @ Vq.T
    sl = O.statistical_dimension(K, lam)
    s = 1 << int(math.ceil(math.log2(4 * (2 + 3 ** q) * sl ** 2 / 0.5)))
    h = rng.integers(0, s, size=(q, d))
    sg = rng.choice([-1.0, 1.0], size=(q, d))
    Z = SO.tensor_sketch_fft(X, h, sg, s)
    # lambda-LQ factorisation of V_q: L L^T = V_q V_q^T + lambda I, Q = L^{-1} V_q
    L = np.linalg.cholesky(K + lam * np.eye(n))
    Q = np.linalg.solve(L, Vq)
    S = SO.tensor_sketch_matrix(h, sg, s)
    dev = np.linalg.norm(Q @ S.T @ S @ Q.T - Q @ Q.T, 2)
    assert dev <= 0.5
    ev = O.preconditioned_spectrum(K, lam, Z, lam)
    assert ev[0] >= 0.5 - 1e-12 and ev[-1] <= 1.5 + 1e-12
    for eps in (1e-3, 1e-6):
        T = int(math.ceil(math.sqrt(3) / 2 * math.log(2 / eps)))
        y = rng.standard_normal(n)
        A = K + lam * np.eye(n)
        C, U = O.precond_factor(Z, lam)
        res = O.pcg(lambda v: A @ v, y, lambda v: O.precond_apply(U, lam, v), tol=1e-300,
                    max_iter=T)
        c = np.linalg.solve(A, y)
        e = res.x - c
        assert math.sqrt(e @ A @ e) <= eps * math.sqrt(c @ A @ c)


# ------------------------------------------------------------ multiple-level sketching
def test_hadamard_recursion_and_orthogonality(golden_dir):
    g = _golden(golden_dir)
    H4 = SO.hadamard(4)
    np.testing.assert_array_equal(H4[1], g["hadamard4_row1"])
    for m in (1, 2, 8, 64):
        H = SO.hadamard(m)
        np.testing.assert_array_equal(H @ H.T, m * np.eye(m))
        np.testing.assert_array_equal(H, H.T)
    with pytest.raises(ValueError):
        SO.hadamard(12)


def test_srht_hand_value(golden_dir):
    g = _golden(golden_dir)
    z = SO.srht_apply(np.array([[1.0, 2.0, 3.0, 4.0]]), [1, -1, 1, 1], [1, 3])[0]
    np.testing.assert_allclose(z, g["srht_a"], rtol=1e-15)


def test_srht_norm_preserved_in_expectation():
    """E||S x||^2 = ||x||^2 (Def. 2 scale): exact average over every sample position."""
    rng = np.random.default_rng(30)
    s1 = 16
    x = rng.standard_normal(s1)
    signs = rng.choice([-1.0, 1.0], size=s1)
    tot = 0.0
    for i in range(s1):  # a one-row SRHT sampling row i, every i equally likely
        tot += np.sum(SO.srht_apply(x[None, :], signs, [i]) ** 2)
    assert tot / s1 == pytest.approx(x @ x, rel=1e-12)


def test_full_srht_is_orthogonal():
    """Sampling every row: S^T S = I exactly (H D / sqrt(s1) is orthogonal)."""
    rng = np.random.default_rng(31)
    s1 = 32
    S = SO.srht_matrix(rng.choice([-1.0, 1.0], size=s1), np.arange(s1), s1)
    np.testing.assert_allclose(S.T @ S, np.eye(s1), atol=1e-14)


def test_gaussian_projection_scale_and_multilevel_preconditioner():
    """Alg. 2: Z_3 = s_3^{-1/2} Z_2 S_3^T keeps Z Z^T in expectation (Monte Carlo), and the
    three-level sketch of a polynomial problem still gives a preconditioner whose PCG
    reaches the dense solution (Thm. 3 setting)."""
    rng = np.random.default_rng(32)
    Z2 = rng.standard_normal((5, 8))
    acc = np.zeros((5, 5))
    for _ in range(2000):
        Z3 = SO.gaussian_project(Z2, rng.standard_normal((4, 8)))
        acc += Z3 @ Z3.T / 2000
    assert np.linalg.norm(acc - Z2 @ Z2.T) <= 0.1 * np.linalg.norm(Z2 @ Z2.T)
    q, d, n, lam = 2, 4, 120, 0.5
    X = rng.standard_normal((n, d)) / math.sqrt(d)
    A = SO.polynomial_kernel(X, X, 1.0, 0.0, q) + lam * np.eye(n)
    s1, s2, s3 = 256, 64, 32
    Z1 = SO.tensor_sketch_fft(X, rng.integers(0, s1, size=(q, d)), rng.choice([-1.0, 1.0], size=(q, d)), s1)
    Z2 = SO.srht_apply(Z1, rng.choice([-1.0, 1.0], size=s1), rng.choice(s1, size=s2, replace=False))
    Z3 = SO.gaussian_project(Z2, rng.standard_normal((s3, s2)))
    y = rng.standard_normal(n)
    _, U = O.precond_factor(Z3, lam)
    res = O.pcg(lambda v: A @ v, y, lambda v: O.precond_apply(U, lam, v), tol=1e-10, max_iter=500)
    np.testing.assert_allclose(res.x, np.linalg.solve(A, y), rtol=1e-6, atol=1e-8)


# ---------------------------------------------------------------- adaptive sketch size
def test_precond_test_exact_features_pass_and_zero_features_fail():
    """Thm. 4's conditions: Z with Z Z^T = K exactly (s = n, Z = V_q) has c1 = ||(I-P)K(I-P)||
    below 0.05 lambda by construction and ratio 1 on range(P); Z = 0 has P = 0 and
    c1 = ||K||."""
    rng = np.random.default_rng(40)
    q, d, n, lam = 2, 3, 30, 0.2
    X = rng.standard_normal((n, d))
    Vq = np.stack([SO.monomials(x, q) for x in X])
    K = Vq @ Vq.T
    c1, (lo, hi), k = SO.precond_test(K, Vq, lam)
    assert c1 <= 0.05 * lam + 1e-9 and lo == pytest.approx(1.0, abs=1e-9) and hi == pytest.approx(1.0, abs=1e-9)
    c1, (lo, hi), k = SO.precond_test(K, np.zeros((n, 4)), lam)
    assert k == 0 and c1 == pytest.approx(np.linalg.eigvalsh(K)[-1], rel=1e-12)


def test_precond_test_scaled_features_fail_condition_two():
    """Z = sqrt(2) V_q: Z Z^T = 2K, so the ratio ||V_q^T P x||^2 / ||Z^T P x||^2 is exactly 1/2
    on range(P) and condition 2 fails while condition 1 still holds."""
    rng = np.random.default_rng(41)
    X = rng.standard_normal((25, 3))
    Vq = np.stack([SO.monomials(x, 2) for x in X])
    K = Vq @ Vq.T
    c1, (lo, hi), _ = SO.precond_test(K, math.sqrt(2) * Vq, 0.3)
    assert lo == pytest.approx(0.5, rel=1e-9) and hi == pytest.approx(0.5, rel=1e-9)
    assert c1 <= 0.03 + 1e-9


def test_adaptive_sketch_size_doubles_until_the_test_passes():
    """Sec. 5: s doubles from s0 until the TensorSketch candidate passes Thm. 4's test; the
    returned preconditioner gives a bounded condition number (Thm. 4 conclusion: the
    guarantees of Thm. 1 hold)."""
    rng = np.random.default_rng(42)
    q, d, n, lam = 2, 3, 60, 2.0
    X = rng.standard_normal((n, d)) / math.sqrt(d)
    K = SO.polynomial_kernel(X, X, 1.0, 0.0, q)
    h_all = rng.integers(0, 1 << 14, size=(q, d))
    sg = rng.choice([-1.0, 1.0], size=(q, d))
    make = lambda s: SO.tensor_sketch_fft(X, h_all % s, sg, s)  # noqa: E731
    s, Z, hist = SO.adaptive_sketch_size(K, make, lam, 2, 1 << 14)
    assert hist[-1][4] and all(not h[4] for h in hist[:-1])
    assert [h[0] for h in hist] == [2 * 2 ** i for i in range(len(hist))]
    ev = O.preconditioned_spectrum(K, lam, Z, lam)
    assert ev[-1] / ev[0] <= 3.0
