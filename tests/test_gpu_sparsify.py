"""The paper's sparsifier with its L1-NNLS solves on the GPU
(hrir_sparsify_device, hrir_tune_sigma_device; Sec. III-D, Eqs. (14)-(16),
Sec. IV-E) against the FP64 oracle, and against the host path of the same
library.

Bar: as for the host path -- fixed-lambda gains to the float32 rounding of
the tap table (1e-6 relative), the same NNZE, the lambda of the search to
1e-9 relative and the same support, the same tuned bandwidth and its
spectral distortion to 1e-9.  The device runs the host's steps in the host's
order in FP64 without contracted multiply-adds, so device and host results
are also compared bit for bit."""
import math

import numpy as np
import pytest

import oracle
import oracle.l1 as L
import synth

pytestmark = pytest.mark.gpu


def H():
    import paper_1502_03162_amd
    return paper_1502_03162_amd


@pytest.fixture(scope="module")
def hset():
    hs = synth.hrir_set(4, 4, 5)
    X = hs.h
    lf = 32
    lg = X.shape[1] - lf + 1
    f, _, _ = oracle.factorize(X, lf, 300, oracle.rand_g0(11, X.shape[0], lg), lambda0=0.2)
    return X, f, lg


def _dense(r, i, lg):
    g = np.zeros(lg)
    np.add.at(g, r["p"][i], r["g"][i].astype(np.float64))
    return g


def _same_tables(a, b):
    """Device against host: the same bits (same steps, same order, FP64
    without contracted multiply-adds on both sides)."""
    for key in ("p", "g", "nnze", "lambda", "err_db"):
        assert np.array_equal(a[key], b[key]), key


@pytest.mark.parametrize("kind,sigma", [("I", None), ("W", 35.0), ("C", 1.2), ("W", math.inf)])
def test_fixed_lambda_device_matches_oracle(dev, hset, kind, sigma):
    X, f, lg = hset
    n = X.shape[0]
    lam = np.random.default_rng(2).uniform(0.0, 0.05, n)
    r = H().sparsify(X, f, lg, kind, sigma=sigma, lam=lam, device=True)
    for i in range(n):
        go = L.sparsify(f, X[i], lg, kind, math.inf if sigma is None else sigma, lam[i])
        gl = _dense(r, i, lg)
        assert r["nnze"][i] == np.count_nonzero(go)
        assert np.max(np.abs(gl - go)) <= 1e-6 * max(np.max(np.abs(go)), 1e-30)
        assert r["lambda"][i] == lam[i]
    _same_tables(r, H().sparsify(X, f, lg, kind, sigma=sigma, lam=lam))


@pytest.mark.parametrize("target", [6, 12, 16])
def test_lambda_search_device_matches_oracle(dev, hset, target):
    X, f, lg = hset
    r = H().sparsify(X, f, target, "I", target_nnze=target, device=True)
    for i in range(X.shape[0]):
        lam_o, g_o = L.lambda_for_nnze(f, X[i], lg, target)
        assert r["nnze"][i] <= target
        assert abs(r["lambda"][i] - lam_o) <= 1e-9 * max(lam_o, 1e-30)
        assert np.max(np.abs(_dense(r, i, lg) - g_o)) <= 1e-6 * max(np.max(np.abs(g_o)), 1e-30)
    _same_tables(r, H().sparsify(X, f, target, "I", target_nnze=target))


def test_window_per_row_sigma_device(dev, hset):
    """Per-row bandwidths (several designs in one launch), lambda searched."""
    X, f, lg = hset
    n = X.shape[0]
    sig = np.array([15.0, 35.0, math.inf, 60.0])[np.arange(n) % 4]
    r = H().sparsify(X, f, 16, "W", sigma=sig, target_nnze=16, device=True)
    for i in (0, 1, 2, 3, n - 1):
        lam_o, g_o = L.lambda_for_nnze(f, X[i], lg, 16, "W", sig[i])
        assert abs(r["lambda"][i] - lam_o) <= 1e-9 * max(lam_o, 1e-30)
        assert np.max(np.abs(_dense(r, i, lg) - g_o)) <= 1e-6 * max(np.max(np.abs(g_o)), 1e-30)
    _same_tables(r, H().sparsify(X, f, 16, "W", sigma=sig, target_nnze=16))


def test_sigma_tuning_device_matches_oracle(dev, hset):
    X, f, lg = hset
    grid = L.PAPER_SIGMA_GRID + [math.inf]
    sig, sd = H().tune_sigma(X, f, grid, device=True)
    for i in range(0, X.shape[0], 3):
        s_o, sd_o, _ = L.tune_sigma(f, X[i], lg, grid)
        assert sig[i] == s_o
        assert abs(sd[i] - sd_o) <= 1e-9
    sig_h, sd_h = H().tune_sigma(X, f, grid)
    assert np.array_equal(sig, sig_h) and np.array_equal(sd, sd_h)


def test_sigma_tuning_at_target_sparsity_device(dev, hset):
    X, f, lg = hset
    grid = [20.0, 60.0, math.inf]
    sig, sd = H().tune_sigma(X, f, grid, target_nnze=6, device=True)
    for i in (0, 13, 27):
        s_o, sd_o, _ = L.tune_sigma(f, X[i], lg, grid, target=6)
        assert sig[i] == s_o
        assert abs(sd[i] - sd_o) <= 1e-9
    sig_h, sd_h = H().tune_sigma(X, f, grid, target_nnze=6)
    assert np.array_equal(sig, sig_h) and np.array_equal(sd, sd_h)


def test_device_limits_and_errors(dev, hset):
    X, f, lg = hset
    h = H()
    # lg above the device solver's limit of 256 taps
    Xl = np.tile(X[:2], (1, 4))                          # m = 800, lf = 32 -> lg = 769
    with pytest.raises(h.HrirError) as e:
        h.sparsify(Xl, f, 16, "I", lam=0.01, device=True)
    assert e.value.code == h.HRIR_EINVAL
    # argument checks are the host call's
    with pytest.raises(h.HrirError) as e:
        h.sparsify(X, f, 16, "W", lam=0.01, device=True)     # window without sigma
    assert e.value.code == h.HRIR_EINVAL
