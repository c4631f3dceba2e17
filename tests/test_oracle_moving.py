"""Pins of the oracle's moving-source render against static renders of the
same source (Eq. (2) with one reflection filter), which are pinned
themselves: one filter for every segment reproduces the static render; with
no fade each segment's samples equal the static render with that segment's
filter; inside a fade the output is the stated linear blend of the two
static renders."""
import numpy as np
import pytest

import oracle
import synth

LF, LG, K, F = 11, 40, 6, 7


def _setup(seed, n):
    rng = np.random.default_rng(seed)
    r = rng.standard_normal(LF)
    p, g = synth.random_taps(seed + 1, F, K, LG, nnz_min=2)
    s = synth.white(seed + 2, n).astype(np.float64)
    return r, p, g.astype(np.float64), s, rng


@pytest.mark.parametrize("n,seg,fade", [(1000, 256, 64), (1024, 256, 0), (700, 512, 256), (3, 256, 64)])
def test_one_filter_everywhere_is_the_static_render(n, seg, fade):
    r, p, g, s, _ = _setup(n, n)
    filt = np.full((n + seg - 1) // seg, 4, dtype=np.int32)
    y = oracle.moving_render(r, s, p, g, LG, filt, seg, fade)
    ref = oracle.sparse_render(r, s, p[4], g[4], LG)
    assert y.shape == ref.shape
    assert np.max(np.abs(y - ref)) <= 1e-13 * max(np.max(np.abs(ref)), 1e-300)


@pytest.mark.parametrize("n,seg,fade", [(2000, 256, 0), (2000, 256, 64), (1800, 512, 100)])
def test_segments_and_fades_follow_the_static_renders(n, seg, fade):
    r, p, g, s, rng = _setup(7 + n + fade, n)
    n_seg = (n + seg - 1) // seg
    filt = rng.integers(0, F, n_seg).astype(np.int32)
    y = oracle.moving_render(r, s, p, g, LG, filt, seg, fade)
    stat = {f: oracle.sparse_render(r, s, p[f], g[f], LG) for f in set(filt.tolist())}
    for t in range(y.size):
        jr = t // seg
        j = min(jr, n_seg - 1)
        want = stat[filt[j]][t]
        u = t - j * seg
        if fade > 0 and j >= 1 and jr == j and u < fade:
            a = (u + 1) / fade
            want = a * want + (1 - a) * stat[filt[j - 1]][t]
        assert abs(y[t] - want) <= 1e-12 * (1 + abs(want)), t


@pytest.mark.parametrize("fade", [64, 17, 1])
def test_crossfade_weight_is_a_linear_ramp(fade):
    """The crossfade is linear over `fade` samples: with a zero filter after
    the change, out = (1 - a(u)) y_old, so a(u) can be read off the output;
    it must rise by exactly 1/fade per sample and reach 1 (the new filter
    alone) at the fade's last sample.  Swapping the two filters gives
    weights a(u) and 1 - a(u) the other way round, so the two outputs add
    up to the sum of the static renders at every sample."""
    n, seg = 1024, 256
    r, p, g, s, _ = _setup(40 + fade, n)
    g = g.copy()
    g[0] = 0.0                                        # filter 0: no taps
    filt = np.array([3, 0, 3, 0], dtype=np.int32)
    y = oracle.moving_render(r, s, p, g, LG, filt, seg, fade)
    y_old = oracle.sparse_render(r, s, p[3], g[3], LG)
    u = np.arange(fade)
    t = seg + u                                       # the first fade (3 -> 0)
    ok = np.abs(y_old[t]) > 1e-3 * np.max(np.abs(y_old))
    a = 1.0 - y[t][ok] / y_old[t][ok]
    assert np.allclose(a, (u[ok] + 1) / fade, rtol=0, atol=1e-9)
    assert abs(y[seg + fade - 1]) <= 1e-12 * np.max(np.abs(y_old))
    ya = oracle.moving_render(r, s, p, g, LG, np.array([3, 5, 3, 5], np.int32), seg, fade)
    yb = oracle.moving_render(r, s, p, g, LG, np.array([5, 3, 5, 3], np.int32), seg, fade)
    y5 = oracle.sparse_render(r, s, p[5], g[5], LG)
    tt = np.arange(seg, n)
    assert np.max(np.abs(ya[tt] + yb[tt] - y_old[tt] - y5[tt])) <= 1e-12 * np.max(np.abs(y_old))


def _fma32(a, b, c):
    """fl32(a b + c) for FP32 a, b, c (the product is exact in FP64)."""
    return (np.asarray(a, np.float64) * np.asarray(b, np.float64) + np.asarray(c, np.float64)).astype(np.float32)


def test_fp32_moving_bound_holds():
    """The per-sample bound the GPU moving test uses (tests/fp32bound.py):
    an FP32 emulation of the kernel's arithmetic -- z as a chain of lf fmas,
    each filter's output as a chain of K fmas in tap order, and inside a
    crossfade a = (u + 1) / fade, b = (1 - a) y_{j-1}, y = fma(a, y_j, b),
    all rounded to FP32 -- stays inside it at every sample, and its worst
    sample comes within a factor of 200 of it."""
    import fp32bound
    rng = np.random.default_rng(8)
    lf, lg, k, nf, seg, fade = 32, 169, 16, 9, 256, 64
    r = rng.standard_normal(lf).astype(np.float32)
    s = (rng.standard_normal(2000) * 0.3).astype(np.float32)
    p, g = synth.random_taps(3, nf, k, lg, nnz_min=k)
    g = g.astype(np.float32)
    n_seg = (s.size + seg - 1) // seg
    filt = rng.integers(0, nf, n_seg).astype(np.int32)
    L = s.size + lf + lg - 2
    # z32[u], u < L: chain over the resonance taps
    z = np.zeros(L, np.float32)
    for n in range(lf):
        sh = np.zeros(L, np.float32)
        sh[n:n + s.size] = s
        z = _fma32(r[n], sh, z)
    t = np.arange(L)

    def chain(f):
        acc = np.zeros(L, np.float32)
        for q in range(k):
            zz = np.where(t - p[f, q] >= 0, z[np.clip(t - p[f, q], 0, L - 1)], 0).astype(np.float32)
            acc = _fma32(g[f, q], zz, acc)
        return acc

    ys = {f: chain(f) for f in np.unique(filt)}
    j = np.minimum(t // seg, n_seg - 1)
    y = np.array([ys[filt[jj]][i] for i, jj in enumerate(j)], np.float32)
    blend = (t // seg >= 1) & (t // seg < n_seg) & (t % seg < fade)
    for i in np.nonzero(blend)[0]:
        u = i % seg
        a = np.float32(np.float32(u + 1) / np.float32(fade))
        b = np.float32(np.float32(np.float32(1.0) - a) * ys[filt[j[i] - 1]][i])
        y[i] = _fma32(a, y[i], b)
    ref = oracle.moving_render(r, s, p, g.astype(np.float64), lg, filt, seg, fade)
    bound = fp32bound.moving_bound(r, s, p, g, lg, filt, seg, fade, k)
    err = np.abs(y.astype(np.float64) - ref)
    assert np.all(err <= bound)
    assert np.max(err / np.maximum(bound, 1e-300)) > 0.005
