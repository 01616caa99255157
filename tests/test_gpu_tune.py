"""GPU checks of the product autotuner: the timed candidates, the stored choice, and the
parity of products that run with the tuned launch (same per-entry bounds as the parity
suite: tuning changes only how the column range is split, i.e. the order of the FP64 sums)."""
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
    yield torch.device("cuda:0")
    krr.tune_cache_clear()


def _t(a, dev):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


def _tau(X, sigma, d):
    kp = int(math.ceil((d + 2) / 32) * 32)
    c = math.log2(math.e) / (2 * sigma * sigma)
    nu = float((X.astype(np.float64) ** 2).sum(1).max())
    return math.log(2) * (2 * 2.0 ** -22 + kp * 2.0 ** -24) * 4 * c * nu + 2.0 ** -22 + 16 * 2.0 ** -24


@pytest.mark.parametrize("n,d,m,prec", [(16384, 54, 7, "f16x3"), (8192, 54, 7, "fp64"),
                                        (9000, 300, 40, "f16x3")])
def test_autotune_then_parity(dev, n, d, m, prec, tmp_path):
    rng = np.random.default_rng(120 + d)
    X = rng.standard_normal((n, d)).astype(np.float32)
    sigma = math.sqrt(d)
    krr.tune_cache_clear()
    rep = krr.autotune_matmat(krr.Kernel.gaussian(sigma), _t(X, dev), m, prec=prec)
    assert rep.candidates >= 2
    assert rep.best_ms <= rep.default_ms and rep.best_ms > 0
    assert rep.nsplit >= 1 and rep.pass_width in (32, 64, 160)
    assert krr.tune_cache_size() == 1
    # the tuned launch is now in use for this shape
    V = rng.standard_normal((n, m))
    out = krr.kernel_matmat(_t(X, dev), _t(X, dev), sigma, _t(V, dev), prec=prec).cpu().numpy()
    rows = rng.choice(n, size=48, replace=False)
    ref = O.kernel_matmat(X, X, sigma, V, rows=rows)
    Kabs = np.exp(-O.sq_dists(X[rows], X) / (2 * sigma ** 2))
    tau = 1e-12 if prec == "fp64" else _tau(X, sigma, d)
    assert np.all(np.abs(out[rows] - ref) <= tau * (Kabs @ np.abs(V)))
    # the table survives a save / clear / load cycle
    path = str(tmp_path / "t.json")
    assert krr.tune_cache_save(path)
    krr.tune_cache_clear()
    assert krr.tune_cache_load(path) and krr.tune_cache_size() == 1
    out2 = krr.kernel_matmat(_t(X, dev), _t(X, dev), sigma, _t(V, dev), prec=prec).cpu().numpy()
    assert np.array_equal(out, out2)
