"""The allocation-free kernel product (krr_kernel_matmat_noalloc) against the workspace
entry point (krr_kernel_matmat), through the C ABI: same kernels, so the outputs must agree
bit for bit; two calls in a row on the shared per-GPU scratch array, the second smaller (its
leftovers from the first must not leak into the result), then the oracle's product as the
independent reference at the mixed product's per-entry bound, and the size limit."""
import ctypes
import math

import numpy as np
import pytest
import torch

import oracle as O
from paper_1611_03220_amd import krr

pytestmark = pytest.mark.gpu


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
    nu = max(float((X1.astype(np.float64) ** 2).sum(1).max()),
             float((X2.astype(np.float64) ** 2).sum(1).max()))
    return math.log(2) * (2 * 2.0 ** -22 + kp * 2.0 ** -24) * 4 * c * nu + 2.0 ** -22 + 16 * 2.0 ** -24


@pytest.mark.parametrize("prec", ["f16x3", "fp64"])
def test_noalloc_matches_workspace_entry_point(dev, prec):
    rng = np.random.default_rng(77)
    cases = [(3000, 2500, 54, 7, 0.0, False), (700, 700, 20, 3, 0.5, False),
             (1200, 900, 130, 5, 0.0, True)]
    for n1, n2, d, m, shift, deriv in cases:  # large first, then smaller
        print(f"noalloc case n1={n1} n2={n2} d={d} m={m} prec={prec} deriv={deriv}", flush=True)
        X1 = rng.standard_normal((n1, d)).astype(np.float32)
        X2 = X1 if shift else rng.standard_normal((n2, d)).astype(np.float32)
        V = rng.standard_normal((n2, m))
        sigma = 0.9 * math.sqrt(d)
        tX1, tX2, tV = _t(X1, dev), _t(X2, dev), _t(V, dev)
        ref = krr.kernel_matmat(tX1, tX2, sigma, tV, shift=shift, deriv=deriv, prec=prec)
        out = torch.full((n1, m), float("nan"), dtype=torch.float64, device=dev)
        krr.kernel_matmat_noalloc(tX1, tX2, sigma, tV, out, shift=shift, deriv=deriv, prec=prec)
        torch.cuda.synchronize()
        a, b = out.cpu().numpy(), ref.cpu().numpy()
        assert np.array_equal(a, b), np.abs(a - b).max()
        if not deriv:
            # independent reference: the oracle's FP64 product, per-entry bound of the path
            rows = rng.choice(n1, size=64, replace=False)
            o = O.kernel_matmat(X1, X2, sigma, V, shift=shift, rows=rows)
            Kabs = np.exp(-O.sq_dists(X1[rows], X2) / (2 * sigma ** 2))
            tau = 1e-12 if prec == "fp64" else _tau(X1, X2, sigma, d)
            bound = tau * (Kabs @ np.abs(V)) + 1e-15
            assert np.all(np.abs(a[rows] - o) <= bound)


def test_noalloc_rejects_problems_beyond_the_scratch_size(dev):
    n = 40000
    need = krr.workspace_bytes(krr.OP_KERNEL_MATMAT, n, n, 128, 0, 16, 1)
    assert need > krr.NOALLOC_SCRATCH_BYTES
    X = torch.zeros((n, 128), dtype=torch.float32, device=dev)
    V = torch.zeros((n, 16), dtype=torch.float64, device=dev)
    out = torch.zeros((n, 16), dtype=torch.float64, device=dev)
    with pytest.raises(krr.KRRError) as ei:
        krr.kernel_matmat_noalloc(X, X, 1.0, V, out)
    assert ei.value.status == krr.E_WORKSPACE and "scratch" in str(ei.value)
    assert float(out.abs().max()) == 0.0  # nothing was launched
