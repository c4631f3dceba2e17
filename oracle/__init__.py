"""FP64 CPU oracle for the sparse-HRIR method -- TEST INFRASTRUCTURE ONLY.

Only the tests, ``__graft_entry__.smoke()`` and the benchmark's CPU-baseline
leg may import this package.  It shares no code with the GPU library
(``paper_1502_03162_amd``) and never imports it.

The numerical routines live in ``oracle.c`` (plain C, double precision,
built to ``liboracle.so`` by ``build()``); this module marshals numpy arrays
into them and adds the error metrics of Sec. IV-B and the cost model of
Sec. IV-F, which are one-line formulas.

Parity status per routine (what pins each one is in ``tests/test_oracle_*``):
  conv_direct, conv_fft, conv_fft_ola, dense_render, sparse_render,
  sparse_render_points, block_render, moving_render, fstep, gstep, factorize
  (cost trace and fixed-point properties), topk, nnls, refit, metrics, cost
  model -- pinned.  The paper's sparsifier is in ``oracle.l1`` and the
  surrogate network in ``oracle.mlp``, each with its own pins.
  The exact f / G values of a factorization are not unique (positive scale,
  local minima); only properties and library-vs-oracle agreement from the same
  G0 pin them.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from ctypes import POINTER, c_double, c_int, c_int32, c_int64, c_uint64

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile oracle.c with gcc -O2 (no fast-math) and OpenMP."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-Wall",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build()
    lib = ctypes.CDLL(_LIB)
    P_d, P_i32, P_i64, P_u64 = POINTER(c_double), POINTER(c_int32), POINTER(c_int64), POINTER(c_uint64)
    sig = {
        "or_conv_direct": (None, [P_d, c_int64, P_d, c_int64, P_d]),
        "or_conv_fft": (c_int, [P_d, c_int64, P_d, c_int64, P_d]),
        "or_conv_fft_ola": (c_int, [P_d, c_int64, P_d, c_int64, c_int64, P_d]),
        "or_dense_render": (None, [P_d, c_int64, P_d, c_int64, P_d]),
        "or_sparse_render": (c_int, [P_d, c_int64, P_d, c_int64, P_i32, P_d, c_int64, c_int64, P_d]),
        "or_sparse_render_jobs": (c_int, [P_d, c_int64, P_d, P_i64, P_i64, c_int64, P_i32, P_d,
                                          c_int64, c_int64, P_i32, c_int64, P_d, P_i64]),
        "or_dense_render_jobs": (c_int, [P_d, P_i64, P_i64, P_d, c_int64, P_i32, c_int64, P_d, P_i64]),
        "or_sparse_render_points": (None, [P_d, c_int64, P_d, c_int64, P_i32, P_d, c_int64,
                                           P_i64, c_int64, P_d]),
        "or_moving_render": (c_int, [P_d, c_int64, P_d, c_int64, P_i32, P_d, c_int64, c_int64, P_i32, c_int64,
                                     c_int64, P_d]),
        "or_block_render_step": (c_int, [P_d, c_int64, P_i32, P_d, c_int64, c_int64, P_d, P_d,
                                         P_d, c_int64, c_int, P_d]),
        "or_splitmix64": (None, [c_uint64, c_int64, P_u64]),
        "or_rand_g0": (None, [c_uint64, c_int64, c_int64, P_d]),
        "or_fstep": (c_int, [P_d, c_int64, c_int64, c_int64, P_d, P_d]),
        "or_gstep": (c_int, [P_d, c_int64, c_int64, c_int64, P_d, P_d, c_int64, c_double]),
        "or_lambda_at": (c_double, [c_double, c_int64, c_int64]),
        "or_cost": (c_double, [P_d, c_int64, c_int64, c_int64, P_d, P_d]),
        "or_factorize": (c_int, [P_d, c_int64, c_int64, c_int64, c_int64, c_double, P_d, P_d, P_d]),
        "or_topk": (None, [P_d, c_int64, c_int64, c_int64, P_i32, P_d, P_i32]),
        "or_nnls": (c_int, [P_d, c_int64, c_int64, P_d, P_d, c_double]),
        "or_refit": (c_int, [P_d, c_int64, c_int64, c_int64, P_d, P_i32, P_i32, c_int64, P_d]),
        "or_num_threads": (c_int, []),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def num_threads() -> int:
    """Threads the oracle's parallel loops use."""
    return int(_load().or_num_threads())


def _d(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _i64(a):
    return np.ascontiguousarray(a, dtype=np.int64)


def _p(a, ct):
    return a.ctypes.data_as(POINTER(ct))


def _check(rc, what):
    if rc != 0:
        raise RuntimeError(f"oracle {what} failed with status {rc}")


# ---------------------------------------------------------------------------
# Convolution (Sec. I footnotes) and rendering (Eq. (2), Sec. IV-F)
# ---------------------------------------------------------------------------
def conv_direct(a, b) -> np.ndarray:
    a, b = _d(a), _d(b)
    c = np.empty(a.size + b.size - 1)
    _load().or_conv_direct(_p(a, c_double), a.size, _p(b, c_double), b.size, _p(c, c_double))
    return c


def conv_fft(a, b) -> np.ndarray:
    a, b = _d(a), _d(b)
    c = np.empty(a.size + b.size - 1)
    _check(_load().or_conv_fft(_p(a, c_double), a.size, _p(b, c_double), b.size, _p(c, c_double)), "conv_fft")
    return c


def conv_fft_ola(a, b, block: int) -> np.ndarray:
    a, b = _d(a), _d(b)
    c = np.empty(a.size + b.size - 1)
    _check(_load().or_conv_fft_ola(_p(a, c_double), a.size, _p(b, c_double), b.size, block,
                                   _p(c, c_double)), "conv_fft_ola")
    return c


def dense_render(s, h) -> np.ndarray:
    s, h = _d(s), _d(h)
    out = np.empty(s.size + h.size - 1)
    _load().or_dense_render(_p(s, c_double), s.size, _p(h, c_double), h.size, _p(out, c_double))
    return out


def sparse_render(r, s, p, g, lg: int) -> np.ndarray:
    """One source, one reflection filter given as K taps (p, g)."""
    r, s, p, g = _d(r), _d(s), _i32(p), _d(g)
    out = np.empty(s.size + r.size + lg - 2)
    _check(_load().or_sparse_render(_p(r, c_double), r.size, _p(s, c_double), s.size, _p(p, c_int32),
                                    _p(g, c_double), p.size, lg, _p(out, c_double)), "sparse_render")
    return out


def _layout(src_len, jobs, row_len_fn):
    src_len = _i64(src_len)
    jobs = _i32(jobs).reshape(-1, 2)
    lens = np.array([row_len_fn(src_len[s]) for s in jobs[:, 0]], dtype=np.int64)
    out_off = np.zeros(jobs.shape[0], dtype=np.int64)
    if jobs.shape[0] > 1:
        out_off[1:] = np.cumsum(lens)[:-1]
    return src_len, jobs, lens, out_off


def sparse_render_jobs(r, src, src_off, src_len, p, g, lg: int, jobs):
    """Batched render; returns a list of rows (one per job)."""
    r, src, src_off, p, g = _d(r), _d(src), _i64(src_off), _i32(p), _d(g)
    lf = r.size
    k = p.shape[1]
    src_len, jobs, lens, out_off = _layout(src_len, jobs, lambda n: n + lf + lg - 2)
    out = np.empty(int(lens.sum()))
    _check(_load().or_sparse_render_jobs(_p(r, c_double), lf, _p(src, c_double), _p(src_off, c_int64),
                                         _p(src_len, c_int64), src_len.size, _p(p, c_int32),
                                         _p(g, c_double), k, lg, _p(jobs, c_int32), jobs.shape[0],
                                         _p(out, c_double), _p(out_off, c_int64)), "sparse_render_jobs")
    return [out[o:o + n] for o, n in zip(out_off, lens)]


def dense_render_jobs(src, src_off, src_len, h, jobs):
    src, src_off, h = _d(src), _i64(src_off), _d(h)
    m = h.shape[1]
    src_len, jobs, lens, out_off = _layout(src_len, jobs, lambda n: n + m - 1)
    out = np.empty(int(lens.sum()))
    _check(_load().or_dense_render_jobs(_p(src, c_double), _p(src_off, c_int64), _p(src_len, c_int64),
                                        _p(h, c_double), m, _p(jobs, c_int32), jobs.shape[0],
                                        _p(out, c_double), _p(out_off, c_int64)), "dense_render_jobs")
    return [out[o:o + n] for o, n in zip(out_off, lens)]


def sparse_render_points(r, s, p, g, t) -> np.ndarray:
    """Output samples at positions t, each from its definition."""
    r, s, p, g, t = _d(r), _d(s), _i32(p), _d(g), _i64(t)
    out = np.empty(t.size)
    _load().or_sparse_render_points(_p(r, c_double), r.size, _p(s, c_double), s.size, _p(p, c_int32),
                                    _p(g, c_double), p.size, _p(t, c_int64), t.size, _p(out, c_double))
    return out


def moving_render(r, src, p, g, lg: int, filt, seg: int, fade: int) -> np.ndarray:
    """One ear of a moving source: filt[j] is segment j's row of the tap
    table (p, g: [F][k]); see or_moving_render."""
    r, src, p, g, filt = _d(r), _d(src), _i32(p), _d(g), _i32(filt)
    n = src.size
    assert filt.size == (n + seg - 1) // seg
    out = np.empty(n + r.size + lg - 2)
    _check(_load().or_moving_render(_p(r, c_double), r.size, _p(src, c_double), n, _p(p, c_int32), _p(g, c_double),
                                    p.shape[1], lg, _p(filt, c_int32), seg, fade, _p(out, c_double)),
           "moving_render")
    return out


class BlockRenderer:
    """Partitioned render of one stream: call ``push(block)`` per block, then
    ``flush()`` for the lf + lg - 2 tail samples."""

    def __init__(self, r, p, g, lg: int):
        self.r, self.p, self.g = _d(r), _i32(p), _d(g)
        self.lg = lg
        self.hs = np.zeros(self.r.size - 1)
        self.hz = np.zeros(lg - 1)

    def _step(self, blk, flush):
        blk = _d(blk)
        n = self.r.size + self.lg - 2 if flush else blk.size
        out = np.empty(n)
        hs = self.hs if self.hs.size else np.zeros(1)
        hz = self.hz if self.hz.size else np.zeros(1)
        _check(_load().or_block_render_step(_p(self.r, c_double), self.r.size, _p(self.p, c_int32),
                                            _p(self.g, c_double), self.p.size, self.lg, _p(hs, c_double),
                                            _p(hz, c_double), _p(blk if blk.size else np.zeros(1), c_double),
                                            blk.size, int(flush), _p(out, c_double)), "block_render")
        return out

    def push(self, blk):
        return self._step(blk, False)

    def flush(self):
        return self._step(np.zeros(0), True)


# ---------------------------------------------------------------------------
# Factorization (Sec. III, Alg. 1), top-K and refit
# ---------------------------------------------------------------------------
def splitmix64(seed: int, n: int) -> np.ndarray:
    out = np.empty(n, dtype=np.uint64)
    _load().or_splitmix64(c_uint64(seed), n, _p(out, c_uint64))
    return out


def rand_g0(seed: int, n: int, lg: int) -> np.ndarray:
    G = np.empty((n, lg))
    _load().or_rand_g0(c_uint64(seed), n, lg, _p(G, c_double))
    return G


def fstep(X, lf: int, G) -> np.ndarray:
    X, G = _d(X), _d(G)
    N, M = X.shape
    f = np.empty(lf)
    _check(_load().or_fstep(_p(X, c_double), N, M, lf, _p(G, c_double), _p(f, c_double)), "fstep")
    return f


def gstep(X, f, G, iters: int = 1, lam: float = 0.0) -> np.ndarray:
    X, f = _d(X), _d(f)
    G = np.array(G, dtype=np.float64, order="C", copy=True)
    N, M = X.shape
    _check(_load().or_gstep(_p(X, c_double), N, M, f.size, _p(f, c_double), _p(G, c_double), iters, lam),
           "gstep")
    return G


def lambda_at(lambda0: float, t: int, T: int) -> float:
    return float(_load().or_lambda_at(lambda0, t, T))


def cost(X, f, G) -> float:
    X, f, G = _d(X), _d(f), _d(G)
    N, M = X.shape
    return float(_load().or_cost(_p(X, c_double), N, M, f.size, _p(f, c_double), _p(G, c_double)))


def factorize(X, lf: int, iters: int, G0, lambda0: float = 0.0):
    """Alg. 1 from the given G0 (L1 continuation when lambda0 > 0).
    Returns (f unit-norm, G, cost trace)."""
    X = _d(X)
    N, M = X.shape
    G = np.array(G0, dtype=np.float64, order="C", copy=True)
    f = np.empty(lf)
    tr = np.empty(max(iters, 1))
    _check(_load().or_factorize(_p(X, c_double), N, M, lf, iters, lambda0, _p(G, c_double),
                                _p(f, c_double), _p(tr, c_double)), "factorize")
    return f, G, tr[:iters]


def topk(G, k: int):
    """Top-K support per row: (p int32[N][k], g f64[N][k], nnz int32[N])."""
    G = _d(G)
    N, lg = G.shape
    p = np.empty((N, k), dtype=np.int32)
    g = np.empty((N, k))
    nnz = np.empty(N, dtype=np.int32)
    _load().or_topk(_p(G, c_double), N, lg, k, _p(p, c_int32), _p(g, c_double), _p(nnz, c_int32))
    return p, g, nnz


def nnls(A, b) -> np.ndarray:
    A, b = _d(A), _d(b)
    m, n = A.shape
    x = np.empty(n)
    tol = 1e-12 * float(np.max(np.abs(A.T @ b))) if n else 0.0
    _check(_load().or_nnls(_p(A, c_double), m, n, _p(b, c_double), _p(x, c_double), tol), "nnls")
    return x


def refit(X, f, p, nnz) -> np.ndarray:
    X, f, p, nnz = _d(X), _d(f), _i32(p), _i32(nnz)
    N, M = X.shape
    k = p.shape[1]
    g = np.empty((N, k))
    _check(_load().or_refit(_p(X, c_double), N, M, f.size, _p(f, c_double), _p(p, c_int32),
                            _p(nnz, c_int32), k, _p(g, c_double)), "refit")
    return g


def scatter_taps(p, g, lg: int) -> np.ndarray:
    """Dense reflection filters [N][lg] from K-tap tables (padding adds 0)."""
    p = np.asarray(p)
    g = np.asarray(g, dtype=np.float64)
    out = np.zeros((p.shape[0], lg))
    for i in range(p.shape[0]):
        for j in range(p.shape[1]):
            out[i, p[i, j]] += g[i, j]
    return out


def reconstruct(f, G) -> np.ndarray:
    """HRIRs f * g_i for every row of G (the product T(f) G_i^T of Eq. (12))."""
    return np.stack([conv_direct(f, G[i]) for i in range(G.shape[0])])


# ---------------------------------------------------------------------------
# Metrics (Sec. IV-B) and cost model (Sec. IV-F)
# ---------------------------------------------------------------------------
def rel_l2(y, yref) -> float:
    y, yref = np.asarray(y, dtype=np.float64), np.asarray(yref, dtype=np.float64)
    den = np.linalg.norm(yref)
    return float(np.linalg.norm(y - yref) / den) if den > 0 else float(np.linalg.norm(y))


def e_db(H, Hhat) -> float:
    """Normalised energy error 10 log10(sum ||h - hhat||^2 / sum ||h||^2)."""
    H, Hhat = np.asarray(H, dtype=np.float64), np.asarray(Hhat, dtype=np.float64)
    num = float(np.sum((H - Hhat) ** 2))
    den = float(np.sum(H * H))
    return 10.0 * math.log10(num / den) if num > 0 else -math.inf


def rmse(X, Xhat) -> float:
    """RMSE of Eq. (17): sqrt(||X - F G^T||_F^2 / (M N))."""
    X, Xhat = np.asarray(X, dtype=np.float64), np.asarray(Xhat, dtype=np.float64)
    return float(np.sqrt(np.sum((X - Xhat) ** 2) / X.size))


def spectral_distortion(h, hhat) -> float:
    """SD of Eq. (17) over the M bins of a length-M DFT; |Hhat| floored at
    1e-12 max|Hhat| so the logarithm stays finite."""
    H = np.abs(np.fft.fft(np.asarray(h, dtype=np.float64)))
    Hh = np.abs(np.fft.fft(np.asarray(hhat, dtype=np.float64)))
    floor = 1e-12 * max(float(Hh.max()), 1e-300)
    Hh = np.maximum(Hh, floor)
    H = np.maximum(H, 1e-12 * max(float(H.max()), 1e-300))
    return float(np.sqrt(np.mean((20.0 * np.log10(H / Hh)) ** 2)))


def nnze(g, thresh: float = 1e-4) -> np.ndarray:
    """Number of entries with magnitude above the 1e-4 discard level (Sec. III-D)."""
    return np.sum(np.abs(np.asarray(g)) > thresh, axis=-1)


def direct_cost(nx: int, ny: int) -> int:
    """Real flops per output sample of direct convolution: min(|x|, |y|)."""
    return min(nx, ny)


def fft_cost(nx: int, ny: int) -> float:
    """Complex flops per output sample of split-radix FFT convolution,
    68/9 (|y| log2 |y| + |y|) / (|y| - |x| + 1)."""
    return 68.0 / 9.0 * (ny * math.log2(ny) + ny) / (ny - nx + 1)


def crossover(ny: int) -> int:
    """Largest |x| for which the direct cost is below the FFT cost."""
    nx = 1
    while direct_cost(nx + 1, ny) < fft_cost(nx + 1, ny):
        nx += 1
    return nx
