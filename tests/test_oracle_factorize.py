"""Pins of the oracle's factorization (Sec. III-C, Alg. 1), top-K selection
and non-negative refit against independent definitions: least squares on the
explicit design matrix, Lawson-Hanson NNLS from scipy, KKT conditions,
monotone cost of the multiplicative update, and brute-force top-K."""
import json
import math
import os

import numpy as np
import pytest
from scipy.optimize import nnls as scipy_nnls

import oracle
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def toeplitz_T(f, m):
    """T(f) in R^{m x lg}: column j is f shifted down by j (Eq. (12))."""
    lf = f.size
    lg = m - lf + 1
    T = np.zeros((m, lg))
    for j in range(lg):
        T[j:j + lf, j] = f
    return T


def test_splitmix64_published_outputs():
    gold = json.load(open(os.path.join(GOLDEN, "splitmix64.json")))
    out = oracle.splitmix64(gold["seed"], len(gold["first_outputs_hex"]))
    assert [f"{int(x):016x}" for x in out] == gold["first_outputs_hex"]


def test_rand_g0_range_and_determinism():
    a = oracle.rand_g0(5, 7, 11)
    b = oracle.rand_g0(5, 7, 11)
    assert np.array_equal(a, b)
    assert np.all(a > 0) and np.all(a <= 1)
    raw = oracle.splitmix64(5, 77)
    assert a.ravel()[3] == ((int(raw[3]) >> 11) + 1) * 2.0 ** -53


def test_fstep_equals_lstsq_on_design_matrix():
    """The resonance step is the least-squares minimiser over f of
    sum_i ||x_i - f * g_i||^2, i.e. lstsq on the stacked convolution matrices."""
    rng = np.random.default_rng(0)
    for (N, M, lf) in [(7, 12, 4), (5, 20, 9), (3, 9, 1), (9, 16, 16)]:
        lg = M - lf + 1
        X = rng.standard_normal((N, M))
        G = rng.uniform(0.1, 1.0, size=(N, lg))
        D = np.zeros((N * M, lf))
        for i in range(N):
            for n in range(lf):
                D[i * M + n:i * M + n + lg, n] = G[i]
        ref = np.linalg.lstsq(D, X.ravel(), rcond=None)[0]
        f = oracle.fstep(X, lf, G)
        assert np.linalg.norm(f - ref) / np.linalg.norm(ref) < 1e-10


def test_gstep_keeps_nonneg_and_decreases_cost():
    rng = np.random.default_rng(1)
    N, M, lf = 9, 30, 6
    lg = M - lf + 1
    X = rng.standard_normal((N, M))
    f = rng.standard_normal(lf)
    G = rng.uniform(0.0, 1.0, size=(N, lg))
    c_prev = oracle.cost(X, f, G)
    for _ in range(50):
        G = oracle.gstep(X, f, G, 1)
        assert np.all(G >= 0)
        c = oracle.cost(X, f, G)
        assert c <= c_prev * (1 + 1e-13)
        c_prev = c


def test_gstep_l1_decreases_penalised_objective():
    rng = np.random.default_rng(2)
    N, M, lf = 6, 25, 5
    lg = M - lf + 1
    X = rng.standard_normal((N, M))
    f = rng.standard_normal(lf)
    G = rng.uniform(0.0, 1.0, size=(N, lg))
    lam = 0.3
    obj = lambda G: oracle.cost(X, f, G) + lam * G.sum()
    prev = obj(G)
    for _ in range(50):
        G = oracle.gstep(X, f, G, 1, lam)
        cur = obj(G)
        assert cur <= prev * (1 + 1e-13)
        prev = cur


def test_gstep_fixed_point_is_nnls_per_row():
    """With f fixed, repeated multiplicative updates converge to the
    non-negative least-squares solution of every row (Lawson-Hanson)."""
    rng = np.random.default_rng(3)
    N, M, lf = 4, 14, 5
    lg = M - lf + 1
    f = rng.standard_normal(lf)
    X = rng.standard_normal((N, M))
    G = oracle.gstep(X, f, np.full((N, lg), 0.5), 200000)
    T = toeplitz_T(f, M)
    for i in range(N):
        ref = scipy_nnls(T, X[i])[0]
        assert np.max(np.abs(G[i] - ref)) < 1e-6


def test_gstep_l1_fixed_point_is_shifted_nnls():
    """min ||x - T g||^2 + lam 1^T g over g >= 0 equals NNLS with target
    x - (lam/2) T (T^T T)^{-1} 1 (completing the square)."""
    rng = np.random.default_rng(4)
    N, M, lf = 3, 14, 5
    lg = M - lf + 1
    lam = 0.2
    f = rng.standard_normal(lf)
    X = rng.standard_normal((N, M))
    G = oracle.gstep(X, f, np.full((N, lg), 0.5), 200000, lam)
    T = toeplitz_T(f, M)
    shift = 0.5 * lam * T @ np.linalg.solve(T.T @ T, np.ones(lg))
    for i in range(N):
        ref = scipy_nnls(T, X[i] - shift)[0]
        assert np.max(np.abs(G[i] - ref)) < 1e-6


def test_lambda_schedule():
    assert oracle.lambda_at(0.2, 0, 100) == 0.2
    assert oracle.lambda_at(0.2, 9, 100) == 0.2
    assert abs(oracle.lambda_at(0.2, 30, 100) - 0.2 * 1000 ** -0.5) < 1e-15
    assert oracle.lambda_at(0.2, 50, 100) == 0.0
    assert oracle.lambda_at(0.2, 99, 100) == 0.0


def test_factorize_plain_alg1_monotone_and_unit_f():
    """lambda0 = 0 is Alg. 1: the cost of Eq. (3) never increases (exact f
    step, monotone G step), f is unit norm and G stays non-negative."""
    hs = synth.hrir_set(3, 2, 3)
    X = hs.h
    G0 = oracle.rand_g0(11, X.shape[0], X.shape[1] - 31)
    f, G, tr = oracle.factorize(X, 32, 60, G0, 0.0)
    assert abs(np.linalg.norm(f) - 1) < 1e-12
    assert np.all(G >= 0)
    assert np.all(np.diff(tr) <= 1e-12 * tr[0])
    assert abs(tr[-1] - oracle.cost(X, f, G)) <= 1e-12 * tr[-1]


def test_factorize_rescaling_leaves_alg1_unchanged():
    """Rescaling f to unit norm each iteration does not change Alg. 1's
    iterates (the update ratio is invariant to f -> a f, G -> G / a)."""
    rng = np.random.default_rng(5)
    N, M, lf = 6, 24, 5
    X = rng.standard_normal((N, M))
    G0 = oracle.rand_g0(3, N, M - lf + 1)
    f, G, _ = oracle.factorize(X, lf, 8, G0, 0.0)
    Gp = G0.copy()
    for _ in range(8):
        fp = oracle.fstep(X, lf, Gp)
        Gp = oracle.gstep(X, fp, Gp, 1)
    s = np.linalg.norm(fp)
    assert np.max(np.abs(f - fp / s)) < 1e-10
    assert np.max(np.abs(G - Gp * s)) < 1e-10 * np.max(G)


def test_factorize_synthetic_reaches_minus_30_db_dense():
    """On a synthetic set built as resonance * sparse reflections, the L1
    continuation reaches a reconstruction error below -30 dB."""
    hs = synth.hrir_set(0, 5, 10)
    X = hs.h
    f, G, tr = oracle.factorize(X, 32, 800, oracle.rand_g0(7, X.shape[0], 169), 0.2)
    rec = oracle.reconstruct(f, G)
    assert oracle.e_db(X, rec) < -30.0
    assert abs(abs(f @ hs.r) - 1.0) < 5e-3


def test_topk_brute_force_with_ties_and_padding():
    rng = np.random.default_rng(6)
    G = rng.integers(0, 4, size=(50, 12)).astype(np.float64)  # many ties and zeros
    for k in (1, 3, 5, 12):
        p, g, nnz = oracle.topk(G, k)
        for i in range(G.shape[0]):
            pos = [j for j in range(G.shape[1]) if G[i, j] > 0]
            order = sorted(pos, key=lambda j: (-G[i, j], j))[:k]
            exp = sorted(order)
            assert nnz[i] == len(exp)
            assert list(p[i, :nnz[i]]) == exp
            assert np.array_equal(g[i, :nnz[i]], G[i, exp])
            assert np.all(p[i, nnz[i]:] == 0) and np.all(g[i, nnz[i]:] == 0)


def test_nnls_matches_scipy_and_kkt():
    rng = np.random.default_rng(7)
    for (m, n) in [(10, 3), (30, 12), (200, 16), (8, 8)]:
        A = rng.standard_normal((m, n))
        b = rng.standard_normal(m)
        x = oracle.nnls(A, b)
        ref = scipy_nnls(A, b)[0]
        assert np.max(np.abs(x - ref)) < 1e-9 * max(1, np.max(np.abs(ref)))
        w = A.T @ (b - A @ x)
        assert np.all(x >= 0)
        assert np.all(w <= 1e-9)
        assert np.all(np.abs(w[x > 0]) <= 1e-9)


def test_refit_equals_nnls_on_support():
    rng = np.random.default_rng(8)
    N, M, lf = 5, 60, 12
    lg = M - lf + 1
    f = rng.standard_normal(lf)
    X = rng.standard_normal((N, M))
    G = rng.uniform(0, 1, size=(N, lg))
    p, g, nnz = oracle.topk(G, 6)
    gr = oracle.refit(X, f, p, nnz)
    T = toeplitz_T(f, M)
    for i in range(N):
        ref = scipy_nnls(T[:, p[i, :nnz[i]]], X[i])[0]
        assert np.max(np.abs(gr[i, :nnz[i]] - ref)) < 1e-9


def test_cost_is_eq3_frobenius_norm():
    """or_cost is the objective of Eq. (3), ||X^T - T(f) G^T||_F^2 with T(f)
    the Toeplitz matrix of Eq. (12): computed here from scipy's Toeplitz
    constructor and a matrix product (no convolution), it agrees to
    rounding; G = 0 gives ||X||_F^2, and exact factors give 0."""
    from scipy.linalg import toeplitz
    rng = np.random.default_rng(21)
    for (N, M, lf) in [(6, 12, 4), (4, 30, 7), (3, 5, 5), (2, 9, 1)]:
        lg = M - lf + 1
        X = rng.standard_normal((N, M))
        f = rng.standard_normal(lf)
        G = rng.uniform(0.0, 1.0, size=(N, lg))
        T = toeplitz(np.concatenate([f, np.zeros(M - lf)]), np.concatenate([[f[0]], np.zeros(lg - 1)]))
        assert T.shape == (M, lg)
        ref = float(np.sum((X.T - T @ G.T) ** 2))
        assert abs(oracle.cost(X, f, G) - ref) <= 1e-12 * ref
        assert abs(oracle.cost(X, f, np.zeros_like(G)) - np.sum(X ** 2)) <= 1e-12 * np.sum(X ** 2)
        Xe = (T @ G.T).T
        assert oracle.cost(Xe, f, G) <= 1e-24 * np.sum(Xe ** 2)
