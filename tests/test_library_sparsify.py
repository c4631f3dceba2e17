"""The library's sparsifier (hrir_sparsify, hrir_tune_sigma; Sec. III-D,
Eqs. (14)-(16), Sec. IV-E) against the FP64 oracle on the same inputs.  Host
only: no GPU needed.  The library returns float32 gains, so fixed-lambda
solutions agree to float rounding; the lambda search and the sigma choice
are decisions both sides take in FP64 on the same bisection and grid."""
import math

import numpy as np
import pytest

import oracle
import oracle.l1 as L
import paper_1502_03162_amd as H
import synth


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


@pytest.mark.parametrize("kind,sigma", [("I", None), ("W", 35.0), ("C", 1.2), ("W", math.inf)])
def test_fixed_lambda_matches_oracle(hset, kind, sigma):
    X, f, lg = hset
    n = X.shape[0]
    lam = np.random.default_rng(2).uniform(0.0, 0.05, n)
    r = H.sparsify(X, f, lg, kind, sigma=sigma, lam=lam)
    for i in range(n):
        go = L.sparsify(f, X[i], lg, kind, math.inf if sigma is None else sigma, lam[i])
        gl = _dense(r, i, lg)
        assert r["nnze"][i] == np.count_nonzero(go)
        assert np.max(np.abs(gl - go)) <= 1e-6 * max(np.max(np.abs(go)), 1e-30)
        e_or = 10 * np.log10(np.sum((X[i] - np.convolve(f, go)) ** 2) / np.sum(X[i] ** 2))
        assert abs(r["err_db"][i] - e_or) <= 1e-4
        assert r["lambda"][i] == lam[i]


@pytest.mark.parametrize("target", [6, 12])
def test_lambda_search_matches_oracle(hset, target):
    X, f, lg = hset
    r = H.sparsify(X, f, target, "I", target_nnze=target)
    for i in range(X.shape[0]):
        lam_o, g_o = L.lambda_for_nnze(f, X[i], lg, target)
        assert r["nnze"][i] <= target
        assert abs(r["lambda"][i] - lam_o) <= 1e-9 * max(lam_o, 1e-30)
        assert np.max(np.abs(_dense(r, i, lg) - g_o)) <= 1e-6 * max(np.max(np.abs(g_o)), 1e-30)
        # ascending positions, padding (0, 0) after the kept taps
        nz = r["nnze"][i]
        assert np.all(np.diff(r["p"][i][:nz]) > 0)
        assert np.all(r["p"][i][nz:] == 0) and np.all(r["g"][i][nz:] == 0)


def test_sigma_tuning_matches_oracle(hset):
    X, f, lg = hset
    grid = L.PAPER_SIGMA_GRID + [math.inf]
    sig, sd = H.tune_sigma(X, f, grid)
    for i in range(0, X.shape[0], 3):
        s_o, sd_o, _ = L.tune_sigma(f, X[i], lg, grid)
        assert sig[i] == s_o
        assert abs(sd[i] - sd_o) <= 1e-9


def test_sigma_tuning_at_target_sparsity_matches_oracle(hset):
    X, f, lg = hset
    grid = [20.0, 60.0, math.inf]
    sig, sd = H.tune_sigma(X, f, grid, target_nnze=6)
    for i in (0, 13, 27):
        s_o, sd_o, _ = L.tune_sigma(f, X[i], lg, grid, target=6)
        assert sig[i] == s_o
        assert abs(sd[i] - sd_o) <= 1e-9


def test_k_slot_cut_keeps_the_largest(hset):
    X, f, lg = hset
    full = H.sparsify(X, f, lg, "I", lam=0.0)
    cut = H.sparsify(X, f, 5, "I", lam=0.0)
    for i in range(X.shape[0]):
        assert cut["nnze"][i] == full["nnze"][i]
        g = _dense(full, i, lg)
        keep = np.sort(np.argsort(-g, kind="stable")[:min(5, full["nnze"][i])])
        nk = len(keep)
        np.testing.assert_array_equal(cut["p"][i][:nk], keep)
        np.testing.assert_array_equal(cut["g"][i][:nk], g[keep].astype(np.float32))


def test_argument_errors(hset):
    X, f, lg = hset
    for kw in [dict(transform="W", sigma=None, lam=0.0), dict(transform="C", sigma=math.inf, lam=0.0),
               dict(transform="W", sigma=-1.0, lam=0.0), dict(transform="I", lam=-1.0),
               dict(transform="I", lam=None, target_nnze=-1)]:
        with pytest.raises(H.HrirError) as e:
            H.sparsify(X, f, 8, **kw)
        assert e.value.code == H.HRIR_EINVAL
    with pytest.raises(H.HrirError):
        H.sparsify(X, f, 0, "I", lam=0.0)
    with pytest.raises(H.HrirError):
        H.tune_sigma(X, f, [10.0, 0.0])
    with pytest.raises(H.HrirError):
        H.tune_sigma(X, f, [10.0], target_nnze=-1)
    bad = X.copy()
    bad[0, 3] = np.nan
    with pytest.raises(H.HrirError):
        H.sparsify(bad, f, 8, "I", lam=0.0)
