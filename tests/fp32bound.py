"""Per-sample error bound of the FP32 render at output positions t.

z is a chain of lf fmas (resonance taps) and each output a chain of k fmas
(kept taps) on the rounded z; r, s and g are the same FP32 values on both
sides, so

    |y32[t] - y[t]| <= (gamma_lf + gamma_k + gamma_lf gamma_k) * m[t],
    m[t] = sum_k g_k sum_n |r_n| |s[t - p_k - n]|,

with gamma_n = n u / (1 - n u), u = 2^-24 (error analysis of recursive
summation with one rounding per fma).  m is the oracle's render definition
applied to |r| and |s|; the factor lf + k + 4 covers the gamma products."""
import numpy as np

import oracle

U32 = 2.0 ** -24


def render_bound(r, src, p, g, t, k):
    mag = oracle.sparse_render_points(np.abs(np.asarray(r, np.float64)), np.abs(np.asarray(src, np.float64)), p,
                                      np.asarray(g, np.float64), t)
    return (len(r) + k + 4) * U32 * mag


def moving_bound(r, src, p, g, lg, filt, seg, fade, k):
    """Per-sample error bound of the FP32 moving render of one ear (filter
    filt[j] for segment j, a linear crossfade over the first `fade` samples
    of segments j >= 1).  Outside a crossfade it is render_bound's; inside,
    y = a y_j + (1 - a) y_{j-1} is formed in FP32 from the two chains' sums
    (a = (u + 1) / fade rounded, b = (1 - a) y_{j-1} rounded, then one fma),
    which adds a few roundings of |y_j| + |y_{j-1}|: the bound there is
    (lf + k + 8) u (m_j + m_{j-1}), m the magnitudes of both filters' hard
    renders (the oracle's moving render on |r|, |s| with no crossfade)."""
    r64 = np.abs(np.asarray(r, np.float64))
    s64 = np.abs(np.asarray(src, np.float64))
    filt = np.asarray(filt, np.int32)
    m_cur = oracle.moving_render(r64, s64, p, np.asarray(g, np.float64), lg, filt, seg, 0)
    prev = np.concatenate([filt[:1], filt[:-1]])
    m_prev = oracle.moving_render(r64, s64, p, np.asarray(g, np.float64), lg, prev, seg, 0)
    t = np.arange(m_cur.size)
    j = t // seg
    blend = (j >= 1) & (j < filt.size) & (t % seg < fade)
    c = len(r) + k + 8
    return c * U32 * (m_cur + np.where(blend, m_prev, 0.0))
