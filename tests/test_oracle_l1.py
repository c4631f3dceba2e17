"""Pins of the oracle's sparsifier (Sec. III-D, Eqs. (14)-(16); sigma tuning
of Sec. IV-E) to facts that do not come from the oracle itself: brute force
over every support, the KKT conditions of Eq. (14), the closed-form lambda at
which g = 0 becomes optimal, and invariants of the transforms."""
import itertools
import math

import numpy as np
import pytest

import oracle
import oracle.l1 as L
import synth


def _brute(A, b, lam):
    """Minimum of ||A g - b||^2 + lam sum(g) over g >= 0 by enumerating every
    support: on a support S the minimiser of the smooth problem solves
    A_S^T A_S z = A_S^T b - lam / 2; keep the feasible one of least cost."""
    n = A.shape[1]
    best = None
    for mask in itertools.product([0, 1], repeat=n):
        idx = [i for i in range(n) if mask[i]]
        z = np.zeros(n)
        if idx:
            z[idx] = np.linalg.solve(A[:, idx].T @ A[:, idx], A[:, idx].T @ b - 0.5 * lam)
        if np.any(z < 0):
            continue
        v = L.objective(A, b, lam, z)
        if best is None or v < best[0]:
            best = (v, z)
    return best[1]


@pytest.mark.parametrize("lam", [0.0, 0.1, 1.0, 5.0])
def test_l1_nnls_equals_brute_force_over_supports(lam):
    rng = np.random.default_rng(int(lam * 10) + 3)
    worst = 0.0
    for _ in range(60):
        m, n = int(rng.integers(3, 11)), int(rng.integers(1, 8))
        A = rng.standard_normal((m, n))
        if np.linalg.matrix_rank(A) < n:
            continue
        b = rng.standard_normal(m)
        worst = max(worst, float(np.max(np.abs(L.l1_nnls(A, b, lam) - _brute(A, b, lam)))))
    assert worst <= 1e-10, worst


def test_l1_nnls_at_zero_lambda_equals_plain_nnls():
    rng = np.random.default_rng(5)
    A = rng.standard_normal((60, 25))
    b = rng.standard_normal(60)
    assert np.max(np.abs(L.l1_nnls(A, b, 0.0) - oracle.nnls(A, b))) <= 1e-12


def _setup(n_az=3, n_el=4):
    hs = synth.hrir_set(3, n_az, n_el)
    X = hs.h
    lf = 32
    lg = X.shape[1] - lf + 1
    f, G, _ = oracle.factorize(X, lf, 300, oracle.rand_g0(9, X.shape[0], lg), lambda0=0.2)
    return X, f, lg


@pytest.mark.parametrize("kind,sigma", [("I", math.inf), ("W", 30.0), ("C", 1.5)])
def test_kkt_conditions_on_hrirs(kind, sigma):
    """Stationarity: the gradient 2 A^T (A g - b) + lam is zero on the
    support and non-negative off it; g >= 0 (before the 1e-4 discard)."""
    X, f, lg = _setup()
    T = L.toeplitz_f(f, lg)
    D = L.transform(kind, T.shape[0], sigma)
    A = D @ T
    for i in range(0, X.shape[0], 5):
        b = D @ X[i]
        lam = 0.02 * L.lambda_max(f, X[i], lg, kind, sigma)
        g = L.l1_nnls(A, b, lam)
        grad = 2.0 * A.T @ (A @ g - b) + lam
        scale = float(np.max(np.abs(2.0 * A.T @ b))) + lam
        assert np.all(g >= 0)
        assert np.max(np.abs(grad[g > 0])) <= 1e-9 * scale
        assert np.min(grad[g == 0], initial=0.0) >= -1e-9 * scale


def test_lambda_max_is_where_the_solution_vanishes():
    X, f, lg = _setup()
    for i in (0, 7, 13):
        lm = L.lambda_max(f, X[i], lg)
        assert np.count_nonzero(L.sparsify(f, X[i], lg, lam=lm * 1.000001, thresh=0.0)) == 0
        g = L.sparsify(f, X[i], lg, lam=0.99 * lm, thresh=0.0)
        j = int(np.argmax(L.toeplitz_f(f, lg).T @ X[i]))
        assert g[j] > 0 and np.count_nonzero(g) >= 1


def test_transform_invariants():
    m = 60
    assert np.array_equal(L.transform("W", m, math.inf), np.eye(m))
    W = L.transform("W", m, 20.0)
    d = np.diag(W)
    assert np.count_nonzero(W - np.diag(d)) == 0 and d[0] == 1.0 and np.all(np.diff(d) < 0)
    assert abs(d[20] - math.exp(-1.0)) <= 1e-15                      # v_sigma(sigma) = e^-1
    C = L.transform("C", m, 2.0)
    assert np.allclose(C, C.T) and np.all(np.linalg.eigvalsh(C) > 0)
    # a Gaussian of unit area: interior rows sum to 1 (to the Poisson-summation error)
    assert np.max(np.abs(C[20:40].sum(axis=1) - 1.0)) <= 1e-9
    for i in range(m - 1):                                            # Toeplitz
        assert np.allclose(np.diag(C, i), C[0, i])


def test_threshold_discards_small_entries():
    X, f, lg = _setup()
    for i in range(0, X.shape[0], 4):
        g = L.sparsify(f, X[i], lg, lam=0.0)
        assert not np.any((np.abs(g) > 0) & (np.abs(g) <= 1e-4))
        g_raw = L.sparsify(f, X[i], lg, lam=0.0, thresh=0.0)
        assert np.array_equal(g, np.where(np.abs(g_raw) <= 1e-4, 0.0, g_raw))


@pytest.mark.parametrize("target", [4, 9, 16])
def test_lambda_search_meets_the_target_at_its_boundary(target):
    X, f, lg = _setup()
    for i in (1, 6, 11, 20):
        lam, g = L.lambda_for_nnze(f, X[i], lg, target)
        assert np.count_nonzero(g) <= target
        np.testing.assert_array_equal(g, L.sparsify(f, X[i], lg, lam=lam))
        if lam > 0:
            # just below the returned lambda the solution keeps more entries
            assert np.count_nonzero(L.sparsify(f, X[i], lg, lam=lam * (1 - 1e-9))) > target


def test_sigma_tuning_never_worse_than_identity():
    X, f, lg = _setup()
    grid = L.PAPER_SIGMA_GRID + [math.inf]
    for i in range(0, X.shape[0], 6):
        s, sd, g = L.tune_sigma(f, X[i], lg, grid)
        g_id = L.sparsify(f, X[i], lg)
        sd_id = oracle.spectral_distortion(X[i], np.convolve(f, g_id))
        assert sd <= sd_id + 1e-12
        assert s in grid
        s1, sd1, g1 = L.tune_sigma(f, X[i], lg, [math.inf])
        assert s1 == math.inf and np.array_equal(g1, g_id) and sd1 == sd_id


def test_sigma_tuning_at_target_sparsity_never_worse_than_identity():
    """Tuned at the target sparsity (lambda searched per bandwidth), the grid
    holds the identity (sigma = inf), so the chosen SD is at most the
    identity's; D_W(inf) reproduces the identity's search exactly."""
    X, f, lg = _setup()
    grid = [20.0, 60.0, math.inf]
    for i in (0, 9, 17):
        s, sd, g = L.tune_sigma(f, X[i], lg, grid, target=6)
        _, g_id = L.lambda_for_nnze(f, X[i], lg, 6)
        sd_id = oracle.spectral_distortion(X[i], np.convolve(f, g_id))
        assert np.count_nonzero(g) <= 6
        assert sd <= sd_id + 1e-12
        s1, sd1, g1 = L.tune_sigma(f, X[i], lg, [math.inf], target=6)
        assert s1 == math.inf and np.array_equal(g1, g_id) and sd1 == sd_id

