"""FP64 oracle of the paper's own sparsifier -- TEST INFRASTRUCTURE ONLY.

Only the tests and the benchmark may import this module; it shares no code
with the GPU library.  With the resonance filter f fixed, each reflection
filter is the solution of the penalised L1-NNLS problem of Eq. (14),

    min_g || D (T(f) g - x) ||_2^2 + lambda * sum(g),   g >= 0,

(for g >= 0 the L1 norm is the plain sum), for a residual transform D: the
identity D_I, the Gaussian convolution D_C of Eq. (15) or the Gaussian time
window D_W of Eq. (16).  Entries of magnitude <= 1e-4 are then discarded
(Sec. III-D).  lambda can be searched per filter for a target NNZE, and the
window bandwidth sigma tuned per HRIR over a grid by spectral distortion
(Sec. IV-E, with lambda = 0 as in the paper's table).

The solver is Lawson and Hanson's active-set NNLS with the L1 term's
constant gradient lambda / 2 carried in the optimality test and in the
passive-set subproblem.  Parity status: l1_nnls pinned by brute force over every
support on small problems and by the KKT conditions; transforms by their
definitions' invariants; the lambda search and sigma tuning by the
properties their results must have (tests/test_oracle_l1.py).
"""
from __future__ import annotations

import math

import numpy as np

from . import spectral_distortion

THRESH = 1e-4


def toeplitz_f(f, lg: int) -> np.ndarray:
    """T(f) of Eq. (12): the (lf + lg - 1) x lg matrix with T[i, j] = f[i - j],
    so that T(f) g is the full convolution f * g."""
    f = np.asarray(f, dtype=np.float64)
    m = f.size + lg - 1
    T = np.zeros((m, lg))
    for j in range(lg):
        T[j:j + f.size, j] = f
    return T


def transform(kind: str, m: int, sigma: float = math.inf) -> np.ndarray:
    """Residual transform D (m x m): 'I' identity; 'C' the Toeplitz matrix of
    the Gaussian N_sigma(k) = exp(-k^2 / (2 sigma^2)) / (sigma sqrt(2 pi)),
    k = i - j (Eq. (15)); 'W' diag(exp(-x^2 / sigma^2)), x = 0..m-1 (Eq. (16)).
    sigma = inf makes 'W' the identity."""
    if kind == "I":
        return np.eye(m)
    x = np.arange(m, dtype=np.float64)
    if kind == "W":
        if math.isinf(sigma):
            return np.eye(m)
        return np.diag(np.exp(-(x * x) / (sigma * sigma)))
    if kind == "C":
        k = x[:, None] - x[None, :]
        return np.exp(-(k * k) / (2.0 * sigma * sigma)) / (sigma * math.sqrt(2.0 * math.pi))
    raise ValueError(kind)


def l1_nnls(A, b, lam: float, max_iter: int = 0) -> np.ndarray:
    """argmin ||A g - b||^2 + lam * sum(g) over g >= 0: the Lawson-Hanson
    active-set method with the linear term carried through.  The (halved,
    negated) gradient is w = A^T (b - A g) - lam / 2; a coordinate enters the
    passive set while its w is positive, and the passive subproblem is the
    stationarity condition A_P^T A_P z = A_P^T b - lam / 2.  Columns that the
    transform has scaled to (numerically) nothing never enter, so no full
    factorisation of A^T A is needed."""
    A = np.asarray(A, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    n = A.shape[1]
    x = np.zeros(n)
    passive = np.zeros(n, dtype=bool)
    atb = A.T @ b
    tol = 1e-12 * max(float(np.max(np.abs(atb))) if n else 0.0, 1e-300)
    max_iter = max_iter or 3 * n + 10
    Q = A.T @ A

    def sub(P):
        idx = np.nonzero(P)[0]
        z = np.zeros(n)
        z[idx] = np.linalg.solve(Q[np.ix_(idx, idx)], atb[idx] - 0.5 * lam)
        return z

    for _ in range(max_iter):
        w = atb - Q @ x - 0.5 * lam
        w[passive] = -np.inf
        j = int(np.argmax(w))
        if not n or w[j] <= tol:
            break
        passive[j] = True
        for _ in range(max_iter):
            z = sub(passive)
            if np.all(z[passive] > 0.0):
                x = z
                break
            # step back to the boundary: the first passive coordinate to hit 0
            neg = passive & (z <= 0.0)
            alpha = float(np.min(x[neg] / (x[neg] - z[neg])))
            x = x + alpha * (z - x)
            passive &= x > 1e-300
            x[~passive] = 0.0
    return x


def objective(A, b, lam: float, g) -> float:
    r = np.asarray(A) @ np.asarray(g) - np.asarray(b)
    return float(r @ r + lam * np.sum(g))


def sparsify(f, x, lg: int, kind: str = "I", sigma: float = math.inf, lam: float = 0.0,
             thresh: float = THRESH) -> np.ndarray:
    """Reflection filter of one HRIR x (length lf + lg - 1) by Eq. (14), then
    the 1e-4 discard."""
    T = toeplitz_f(f, lg)
    D = transform(kind, T.shape[0], sigma)
    g = l1_nnls(D @ T, D @ np.asarray(x, dtype=np.float64), lam)
    g[np.abs(g) <= thresh] = 0.0
    return g


def lambda_max(f, x, lg: int, kind: str = "I", sigma: float = math.inf) -> float:
    """Smallest lambda at which g = 0 solves Eq. (14): the gradient at 0,
    -2 A^T b + lambda, is then non-negative (A = D T(f), b = D x)."""
    T = toeplitz_f(f, lg)
    D = transform(kind, T.shape[0], sigma)
    return max(0.0, 2.0 * float(np.max((D @ T).T @ (D @ np.asarray(x, dtype=np.float64)))))


def lambda_for_nnze(f, x, lg: int, target: int, kind: str = "I", sigma: float = math.inf,
                    thresh: float = THRESH, steps: int = 50):
    """Smallest lambda found by geometric bisection on [1e-12, 1] * lambda_max
    whose solution keeps at most `target` entries: lambda = 0 if that already
    does.  Returns (lambda, g)."""
    g0 = sparsify(f, x, lg, kind, sigma, 0.0, thresh)
    if np.count_nonzero(g0) <= target:
        return 0.0, g0
    hi = lambda_max(f, x, lg, kind, sigma)
    lo = hi * 1e-12
    g_hi = np.zeros(lg)
    for _ in range(steps):
        mid = math.sqrt(lo * hi)
        g = sparsify(f, x, lg, kind, sigma, mid, thresh)
        if np.count_nonzero(g) <= target:
            hi, g_hi = mid, g
        else:
            lo = mid
    return hi, g_hi


def tune_sigma(f, x, lg: int, grid, lam: float = 0.0, thresh: float = THRESH, target: int = 0):
    """Window bandwidth of D_W minimising the SD (Eq. (17)) of f * g against x
    over the grid (inf = identity).  Each bandwidth's g solves Eq. (14) at
    lambda = lam, or, with target > 0, at the lambda of lambda_for_nnze
    (at most `target` entries).  Ties keep the earlier grid entry.
    Returns (sigma, sd, g)."""
    best = None
    for s in grid:
        if target > 0:
            _, g = lambda_for_nnze(f, x, lg, target, "W", float(s), thresh)
        else:
            g = sparsify(f, x, lg, "W", float(s), lam, thresh)
        sd = spectral_distortion(x, np.convolve(np.asarray(f, dtype=np.float64), g))
        if best is None or sd < best[1]:
            best = (float(s), sd, g)
    return best


# sigma grid of the paper's table: 15 + 2 (0:24), then 100, 160, 250
PAPER_SIGMA_GRID = [15.0 + 2.0 * i for i in range(25)] + [100.0, 160.0, 250.0]
