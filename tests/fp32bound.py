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
