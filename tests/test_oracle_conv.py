"""Pins of the oracle's convolution and rendering routines against what the
mathematics fixes: numpy's convolution, deltas, linearity, shift invariance,
associativity (Eq. (2)), brute-force equality of direct and FFT convolution,
and block-split invariance of partitioned rendering (Sec. IV-F)."""
import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.filterwarnings("ignore")


def rel(a, b):
    return np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(b), 1e-300)


def test_direct_matches_numpy_convolve():
    rng = np.random.default_rng(0)
    for na in (1, 2, 5, 31, 64, 200):
        for nb in (1, 3, 32, 169):
            a, b = rng.standard_normal(na), rng.standard_normal(nb)
            c = oracle.conv_direct(a, b)
            assert c.size == na + nb - 1
            assert rel(c, np.convolve(a, b)) < 1e-14


def test_direct_delta_and_shift():
    rng = np.random.default_rng(1)
    b = rng.standard_normal(37)
    d = np.zeros(1); d[0] = 1.0
    assert np.array_equal(oracle.conv_direct(d, b), b)
    for p in (1, 5, 40):
        dp = np.zeros(p + 1); dp[p] = 1.0
        c = oracle.conv_direct(dp, b)
        assert np.array_equal(c[:p], np.zeros(p)) and np.array_equal(c[p:], b)


def test_direct_linearity_commutativity_shift_invariance():
    rng = np.random.default_rng(2)
    a, a2, b = rng.standard_normal(50), rng.standard_normal(50), rng.standard_normal(20)
    lhs = oracle.conv_direct(2.5 * a - 0.75 * a2, b)
    rhs = 2.5 * oracle.conv_direct(a, b) - 0.75 * oracle.conv_direct(a2, b)
    assert rel(lhs, rhs) < 1e-14
    assert rel(oracle.conv_direct(a, b), oracle.conv_direct(b, a)) < 1e-14
    shifted = np.concatenate([np.zeros(7), a])
    assert rel(oracle.conv_direct(shifted, b)[7:], oracle.conv_direct(a, b)) < 1e-15


def test_fft_equals_direct_brute_force():
    rng = np.random.default_rng(3)
    for na in range(1, 65):
        a = rng.standard_normal(na)
        for nb in (1, 2, 3, 7, 31, 32, 33, 64):
            b = rng.standard_normal(nb)
            assert rel(oracle.conv_fft(a, b), oracle.conv_direct(a, b)) < 1e-12, (na, nb)


def test_fft_matches_numpy_fft():
    rng = np.random.default_rng(4)
    a, b = rng.standard_normal(1000), rng.standard_normal(200)
    L = 2048
    ref = np.fft.irfft(np.fft.rfft(a, L) * np.fft.rfft(b, L), L)[: a.size + b.size - 1]
    assert rel(oracle.conv_fft(a, b), ref) < 1e-12


@pytest.mark.parametrize("block", [1, 2, 7, 64, 199, 200, 1000, 5000])
def test_fft_overlap_add_equals_direct(block):
    rng = np.random.default_rng(5)
    a, b = rng.standard_normal(3000), rng.standard_normal(200)
    assert rel(oracle.conv_fft_ola(a, b, block), oracle.conv_direct(a, b)) < 1e-12


def _scatter(p, g, lg):
    d = np.zeros(lg)
    for pk, gk in zip(p, g):
        d[pk] += gk
    return d


def test_sparse_render_associativity():
    """(s * r) * g == s * (r * g) with g the taps scattered to length lg (Eq. (2))."""
    rng = np.random.default_rng(6)
    lf, lg, ns = 32, 169, 3000
    r, s = rng.standard_normal(lf), rng.standard_normal(ns)
    for k in (1, 8, 16, 32):
        p = np.sort(rng.choice(lg, size=k, replace=False)).astype(np.int32)
        g = rng.uniform(0, 1, size=k)
        out = oracle.sparse_render(r, s, p, g, lg)
        assert out.size == ns + lf + lg - 2
        ref = np.convolve(s, np.convolve(r, _scatter(p, g, lg)))
        assert rel(out, ref) < 1e-13


def test_sparse_render_single_tap_is_shift_of_z():
    rng = np.random.default_rng(7)
    lf, lg, ns = 20, 50, 300
    r, s = rng.standard_normal(lf), rng.standard_normal(ns)
    z = np.convolve(r, s)
    for p in (0, 1, 13, lg - 1):
        out = oracle.sparse_render(r, s, np.array([p]), np.array([1.0]), lg)
        exp = np.zeros(ns + lf + lg - 2)
        exp[p:p + z.size] = z
        assert rel(out, exp) < 1e-14
        assert np.all(out[:p] == 0) and np.all(out[p + z.size:] == 0)


def test_sparse_render_padding_taps_contribute_nothing():
    rng = np.random.default_rng(8)
    r, s = rng.standard_normal(8), rng.standard_normal(100)
    p = np.array([3, 9, 0, 0], dtype=np.int32)
    g = np.array([0.5, 0.25, 0.0, 0.0])
    a = oracle.sparse_render(r, s, p, g, 16)
    b = oracle.sparse_render(r, s, p[:2], g[:2], 16)
    assert np.array_equal(a, b)


def test_exact_reconstruction_full_taps_equals_dense():
    """K = lg with the true reflection filter renders the full HRIR h = r * g
    (no truncation, since lf + lg - 1 = M, Eq. (12))."""
    rng = np.random.default_rng(9)
    lf, m = 32, 200
    lg = m - lf + 1
    r, s = rng.standard_normal(lf), rng.standard_normal(4000)
    g = rng.uniform(0, 1, size=lg)
    h = np.convolve(r, g)
    assert h.size == m
    sp = oracle.sparse_render(r, s, np.arange(lg, dtype=np.int32), g, lg)
    dn = oracle.dense_render(s, h)
    assert rel(sp, dn) < 1e-13


def test_points_and_jobs_match_single_render():
    rng = np.random.default_rng(10)
    lf, lg = 32, 169
    r = rng.standard_normal(lf)
    lens = [1, 31, 199, 500, 4097]
    srcs = [rng.standard_normal(n) for n in lens]
    off = np.concatenate([[0], np.cumsum(lens)[:-1]])
    F, K = 6, 16
    p = np.stack([np.sort(rng.choice(lg, size=K, replace=False)) for _ in range(F)]).astype(np.int32)
    g = rng.uniform(0, 1, size=(F, K))
    jobs = np.array([(i, (i * 3 + j) % F) for i in range(len(lens)) for j in range(2)], dtype=np.int32)
    rows = oracle.sparse_render_jobs(r, np.concatenate(srcs), off, lens, p, g, lg, jobs)
    for (si, f), row in zip(jobs, rows):
        ref = oracle.sparse_render(r, srcs[si], p[f], g[f], lg)
        assert np.array_equal(row, ref)
        t = np.unique(np.concatenate([[0, row.size - 1], rng.integers(0, row.size, 20)]))
        pts = oracle.sparse_render_points(r, srcs[si], p[f], g[f], t)
        assert rel(pts, ref[t]) < 1e-13


def test_dense_jobs_match_single_render():
    rng = np.random.default_rng(11)
    h = rng.standard_normal((3, 200))
    lens = [5, 300]
    srcs = [rng.standard_normal(n) for n in lens]
    jobs = np.array([(0, 2), (1, 0), (1, 1)], dtype=np.int32)
    rows = oracle.dense_render_jobs(np.concatenate(srcs), [0, 5], lens, h, jobs)
    for (si, f), row in zip(jobs, rows):
        assert np.array_equal(row, oracle.dense_render(srcs[si], h[f]))


@pytest.mark.parametrize("seed", range(6))
def test_block_render_concatenation_equals_one_shot(seed):
    """Partitioned rendering with carried s- and z-history reproduces the
    one-shot render for any block split, including 1-sample blocks and blocks
    shorter than the history."""
    rng = np.random.default_rng(100 + seed)
    lf, lg = (32, 169) if seed % 2 == 0 else (7, 20)
    ns = int(rng.integers(1, 2000))
    r, s = rng.standard_normal(lf), rng.standard_normal(ns)
    K = min(16, lg)
    p = np.sort(rng.choice(lg, size=K, replace=False)).astype(np.int32)
    g = rng.uniform(0, 1, size=K)
    cuts, pos = [], 0
    while pos < ns:
        b = int(rng.choice([1, 2, 5, 30, 64, 500, 1024]))
        cuts.append(s[pos:pos + b])
        pos += b
    br = oracle.BlockRenderer(r, p, g, lg)
    out = np.concatenate([br.push(c) for c in cuts] + [br.flush()])
    ref = oracle.sparse_render(r, s, p, g, lg)
    assert out.size == ref.size
    assert rel(out, ref) < 1e-13


def _fma32_chain(terms_a, terms_b):
    """FP32 fma chain over axis 0: acc = fl32(a_i b_i + acc), the product of
    two FP32 values exact in FP64, one rounding per step as an fma."""
    acc = np.zeros(terms_a.shape[1:], dtype=np.float32)
    for a, b in zip(terms_a, terms_b):
        acc = (a.astype(np.float64) * b.astype(np.float64) + acc.astype(np.float64)).astype(np.float32)
    return acc


def test_fp32_render_bound_holds_and_is_tight():
    """The per-sample bound the GPU parity tests use (tests/fp32bound.py):
    an FP32 emulation of the render's two fma chains (z over the lf
    resonance taps, then the K kept taps on the rounded z) stays inside it
    at every sample, and the worst sample comes within a factor of 200 of
    it (2.8 % of the bound here; rounding errors add up like a random walk,
    the bound like a straight line), so the bound is not vacuous."""
    import fp32bound
    rng = np.random.default_rng(5)
    lf, lg, k = 32, 169, 16
    r = rng.standard_normal(lf).astype(np.float32)
    s = (rng.standard_normal(6000) * 0.3).astype(np.float32)
    p = np.sort(rng.choice(lg, k, replace=False)).astype(np.int32)
    g = rng.uniform(0, 1, k).astype(np.float32)
    t = np.arange(0, s.size + lf + lg - 2, 7)
    # z32[u] for every u the taps reach: chain over n of r[n] s[u - n]
    umax = t.max()
    u = np.arange(umax + 1)
    sa = np.stack([np.where((u - n >= 0) & (u - n < s.size), s[np.clip(u - n, 0, s.size - 1)], 0).astype(np.float32)
                   for n in range(lf)])
    z32 = _fma32_chain(np.repeat(r[:, None], u.size, axis=1), sa)
    zt = np.stack([np.where(t - pk >= 0, z32[np.clip(t - pk, 0, umax)], 0).astype(np.float32) for pk in p])
    y32 = _fma32_chain(np.repeat(g[:, None], t.size, axis=1), zt)
    y = oracle.sparse_render_points(r, s, p, g.astype(np.float64), t)
    err = np.abs(y32.astype(np.float64) - y)
    bound = fp32bound.render_bound(r, s, p, g, t, k)
    assert np.all(err <= bound)
    assert np.max(err / np.maximum(bound, 1e-300)) > 0.005
