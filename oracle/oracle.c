/*
 * FP64 CPU oracle for the sparse head-related impulse response method
 * (Luo, Zotkin, Duraiswami, "Sparse Head-Related Impulse Response for
 * Efficient Direct Convolution", arXiv 1502.03162).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the rendering library calls this
 * file; only the tests, the smoke check and the benchmark's CPU-baseline leg
 * load it.  It shares no code, headers or tables with the GPU path.
 *
 * Every routine is the plain definition (or the paper's algorithm step by
 * step) in double precision, with no blocking or reordering beyond what the
 * definition states.  Index conventions are 0-based; the paper's footnote on
 * direct convolution is 1-based.
 *
 * Sizes are int64_t, arrays are row-major, and every output buffer is
 * allocated by the caller.  Functions returning int give 0 on success and a
 * negative value on bad arguments or a failed solve.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_OK 0
#define OR_EINVAL (-1)
#define OR_ENOTPD (-3)
#define OR_ENOMEM (-2)

/* ------------------------------------------------------------------------
 * O1. Direct convolution (Sec. I, footnote on direct convolution):
 *     c[n] = sum_j a[j] * b[n - j],  n in [0, na + nb - 1).
 * --------------------------------------------------------------------- */
void or_conv_direct(const double* a, int64_t na, const double* b, int64_t nb, double* c) {
    const int64_t nc = na + nb - 1;
    for (int64_t n = 0; n < nc; ++n) {
        double acc = 0.0;
        for (int64_t j = 0; j < na; ++j) {
            const int64_t i = n - j;
            if (i >= 0 && i < nb) acc += a[j] * b[i];
        }
        c[n] = acc;
    }
}

/* ------------------------------------------------------------------------
 * O2. FFT convolution (Sec. I, footnote on Fourier-transform convolution):
 *     a * b = IFFT(FFT(a) o FFT(b)) with both zero-padded to a power of two
 *     L >= na + nb - 1; keep the real part of the first na + nb - 1 values.
 *     Own iterative radix-2 transform (Cooley-Tukey, decimation in time).
 * --------------------------------------------------------------------- */
static void fft_radix2(double* re, double* im, int64_t L, int inverse) {
    /* bit-reversal permutation */
    for (int64_t i = 1, j = 0; i < L; ++i) {
        int64_t bit = L >> 1;
        for (; j & bit; bit >>= 1) j ^= bit;
        j ^= bit;
        if (i < j) {
            double t = re[i]; re[i] = re[j]; re[j] = t;
            t = im[i]; im[i] = im[j]; im[j] = t;
        }
    }
    const double sgn = inverse ? 1.0 : -1.0;
    for (int64_t len = 2; len <= L; len <<= 1) {
        const int64_t half = len >> 1;
        for (int64_t k = 0; k < half; ++k) {
            const double ang = sgn * 2.0 * M_PI * (double)k / (double)len;
            const double wr = cos(ang), wi = sin(ang);
            for (int64_t s = 0; s < L; s += len) {
                const int64_t u = s + k, v = s + k + half;
                const double xr = re[v] * wr - im[v] * wi;
                const double xi = re[v] * wi + im[v] * wr;
                re[v] = re[u] - xr; im[v] = im[u] - xi;
                re[u] += xr;        im[u] += xi;
            }
        }
    }
    if (inverse) {
        for (int64_t i = 0; i < L; ++i) { re[i] /= (double)L; im[i] /= (double)L; }
    }
}

int or_conv_fft(const double* a, int64_t na, const double* b, int64_t nb, double* c) {
    if (na < 1 || nb < 1) return OR_EINVAL;
    const int64_t nc = na + nb - 1;
    int64_t L = 1;
    while (L < nc) L <<= 1;
    double* buf = (double*)calloc((size_t)(4 * L), sizeof(double));
    if (!buf) return OR_ENOMEM;
    double *ar = buf, *ai = buf + L, *br = buf + 2 * L, *bi = buf + 3 * L;
    memcpy(ar, a, (size_t)na * sizeof(double));
    memcpy(br, b, (size_t)nb * sizeof(double));
    fft_radix2(ar, ai, L, 0);
    fft_radix2(br, bi, L, 0);
    for (int64_t i = 0; i < L; ++i) {
        const double xr = ar[i] * br[i] - ai[i] * bi[i];
        const double xi = ar[i] * bi[i] + ai[i] * br[i];
        ar[i] = xr; ai[i] = xi;
    }
    fft_radix2(ar, ai, L, 1);
    memcpy(c, ar, (size_t)nc * sizeof(double));
    free(buf);
    return OR_OK;
}

/* Block (partitioned) FFT convolution, overlap-add form: a is cut into
 * blocks of `block` samples, each block is FFT-convolved with b, and the
 * block results are added at the block's offset (Sec. IV-F). */
int or_conv_fft_ola(const double* a, int64_t na, const double* b, int64_t nb, int64_t block, double* c) {
    if (na < 1 || nb < 1 || block < 1) return OR_EINVAL;
    const int64_t nc = na + nb - 1;
    memset(c, 0, (size_t)nc * sizeof(double));
    double* part = (double*)malloc((size_t)(block + nb - 1) * sizeof(double));
    if (!part) return OR_ENOMEM;
    for (int64_t s = 0; s < na; s += block) {
        const int64_t len = (na - s < block) ? na - s : block;
        int rc = or_conv_fft(a + s, len, b, nb, part);
        if (rc) { free(part); return rc; }
        for (int64_t i = 0; i < len + nb - 1; ++i) c[s + i] += part[i];
    }
    free(part);
    return OR_OK;
}

/* ------------------------------------------------------------------------
 * O3. Dense render: out = s * h for one HRIR h (O1).
 * O4. Sparse render (Eq. (2), rendered in the (s * f) * g order of Sec. II):
 *     z = r * s (O1), then out[t] = sum_k g_k z[t - p_k] for
 *     t in [0, ns + lf + lg - 2), with z = 0 outside [0, ns + lf - 1).
 *     Taps (p_k, g_k) are the K kept entries of one reflection filter; the
 *     zero-gain padding entries contribute nothing.
 * --------------------------------------------------------------------- */
void or_dense_render(const double* s, int64_t ns, const double* h, int64_t m, double* out) {
    or_conv_direct(s, ns, h, m, out);
}

static void sparse_from_z(const double* z, int64_t nz, const int32_t* p, const double* g, int64_t k,
                          int64_t nout, double* out) {
    for (int64_t t = 0; t < nout; ++t) {
        double acc = 0.0;
        for (int64_t j = 0; j < k; ++j) {
            const int64_t u = t - (int64_t)p[j];
            if (u >= 0 && u < nz) acc += g[j] * z[u];
        }
        out[t] = acc;
    }
}

int or_sparse_render(const double* r, int64_t lf, const double* s, int64_t ns,
                     const int32_t* p, const double* g, int64_t k, int64_t lg, double* out) {
    if (lf < 1 || ns < 1 || k < 1 || lg < 1) return OR_EINVAL;
    const int64_t nz = ns + lf - 1;
    double* z = (double*)malloc((size_t)nz * sizeof(double));
    if (!z) return OR_ENOMEM;
    or_conv_direct(r, lf, s, ns, z);
    sparse_from_z(z, nz, p, g, k, ns + lf + lg - 2, out);
    free(z);
    return OR_OK;
}

/* Batched sparse render over a job list: z is formed once per source
 * (the direction-independent pre-filtering of Sec. II) and shared by every
 * job of that source.  jobs[2*j] = source, jobs[2*j+1] = filter.  Job j's
 * row (length src_len + lf + lg - 2) is written at out + out_off[j].
 * Parallel over jobs with OpenMP when built with it. */
int or_sparse_render_jobs(const double* r, int64_t lf, const double* src, const int64_t* src_off,
                          const int64_t* src_len, int64_t n_src, const int32_t* p, const double* g,
                          int64_t k, int64_t lg, const int32_t* jobs, int64_t n_jobs,
                          double* out, const int64_t* out_off) {
    double** z = (double**)calloc((size_t)n_src, sizeof(double*));
    if (!z) return OR_ENOMEM;
    int rc = OR_OK;
    for (int64_t i = 0; i < n_src && rc == OR_OK; ++i) {
        z[i] = (double*)malloc((size_t)(src_len[i] + lf - 1) * sizeof(double));
        if (!z[i]) rc = OR_ENOMEM;
    }
    if (rc == OR_OK) {
#pragma omp parallel for schedule(dynamic, 1)
        for (int64_t i = 0; i < n_src; ++i) or_conv_direct(r, lf, src + src_off[i], src_len[i], z[i]);
#pragma omp parallel for schedule(dynamic, 1)
        for (int64_t j = 0; j < n_jobs; ++j) {
            const int64_t si = jobs[2 * j], f = jobs[2 * j + 1];
            sparse_from_z(z[si], src_len[si] + lf - 1, p + f * k, g + f * k, k,
                          src_len[si] + lf + lg - 2, out + out_off[j]);
        }
    }
    for (int64_t i = 0; i < n_src; ++i) free(z[i]);
    free(z);
    return rc;
}

/* One output sample of a sparse render: sum_q g[q] z[t - p[q]], z zero
 * outside [0, nz). */
static double tap_sum(const double* z, int64_t nz, const int32_t* p, const double* g, int64_t k, int64_t t) {
    double acc = 0.0;
    for (int64_t q = 0; q < k; ++q) {
        const int64_t u = t - p[q];
        if (u >= 0 && u < nz) acc += g[q] * z[u];
    }
    return acc;
}

/* Moving source, one ear: the reflection filter changes every seg samples
 * (filt[j] is segment j's row of the tap table, n_seg = ceil(n / seg)).
 * Output sample t uses segment j = min(t / seg, n_seg - 1); in the first
 * fade samples of a segment j >= 1 (u = t - j seg < fade, t / seg = j) it is
 * a y_j + (1 - a) y_{j-1} with a = (u + 1) / fade, y_j the render with
 * segment j's filter.  z = r * s (Eq. (2)); out has n + lf + lg - 2 samples. */
int or_moving_render(const double* r, int64_t lf, const double* src, int64_t n, const int32_t* p,
                     const double* g, int64_t k, int64_t lg, const int32_t* filt, int64_t seg, int64_t fade,
                     double* out) {
    const int64_t nz = n + lf - 1, n_out = n + lf + lg - 2, n_seg = (n + seg - 1) / seg;
    double* z = (double*)malloc((size_t)nz * sizeof(double));
    if (!z) return OR_ENOMEM;
    or_conv_direct(r, lf, src, n, z);
#pragma omp parallel for schedule(static)
    for (int64_t t = 0; t < n_out; ++t) {
        const int64_t jr = t / seg;
        const int64_t j = jr < n_seg - 1 ? jr : n_seg - 1;
        double y = tap_sum(z, nz, p + (int64_t)filt[j] * k, g + (int64_t)filt[j] * k, k, t);
        const int64_t u = t - j * seg;
        if (fade > 0 && j >= 1 && jr == j && u < fade) {
            const double a = (double)(u + 1) / (double)fade;
            const double y0 = tap_sum(z, nz, p + (int64_t)filt[j - 1] * k, g + (int64_t)filt[j - 1] * k, k, t);
            y = a * y + (1.0 - a) * y0;
        }
        out[t] = y;
    }
    free(z);
    return OR_OK;
}

/* Dense render over a job list (h: [F][m]), parallel over jobs. */
int or_dense_render_jobs(const double* src, const int64_t* src_off, const int64_t* src_len,
                         const double* h, int64_t m, const int32_t* jobs, int64_t n_jobs,
                         double* out, const int64_t* out_off) {
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t j = 0; j < n_jobs; ++j) {
        const int64_t si = jobs[2 * j], f = jobs[2 * j + 1];
        or_conv_direct(src + src_off[si], src_len[si], h + f * m, m, out + out_off[j]);
    }
    return OR_OK;
}

/* Single output samples of the sparse render, each computed from its
 * definition: out[t] = sum_k g_k sum_n r[n] s[t - p_k - n]. */
void or_sparse_render_points(const double* r, int64_t lf, const double* s, int64_t ns,
                             const int32_t* p, const double* g, int64_t k,
                             const int64_t* t, int64_t nt, double* out) {
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < nt; ++i) {
        double acc = 0.0;
        for (int64_t j = 0; j < k; ++j) {
            double zu = 0.0;
            const int64_t u = t[i] - (int64_t)p[j];
            for (int64_t n = 0; n < lf; ++n) {
                const int64_t q = u - n;
                if (q >= 0 && q < ns) zu += r[n] * s[q];
            }
            acc += g[j] * zu;
        }
        out[i] = acc;
    }
}

/* ------------------------------------------------------------------------
 * O5. Block (partitioned) sparse render (Sec. IV-F: partitioned time-domain
 * convolution has no latency and no memory overhead).  The source arrives in
 * blocks of arbitrary length; output sample t is emitted with input sample t.
 * State carried between blocks: the last lf - 1 source samples and the last
 * lg - 1 values of z.  A final call with blen = 0 and flush = 1 emits the
 * lf + lg - 2 tail samples.  hist_s: [lf-1], hist_z: [lg-1], oldest first,
 * zero at stream start.
 * --------------------------------------------------------------------- */
int or_block_render_step(const double* r, int64_t lf, const int32_t* p, const double* g, int64_t k,
                         int64_t lg, double* hist_s, double* hist_z,
                         const double* blk, int64_t blen, int flush, double* out) {
    const int64_t hs = lf - 1, hz = lg - 1;
    const int64_t n = flush ? lf + lg - 2 : blen;
    /* extended source: history then the new samples (zeros when flushing) */
    double* sx = (double*)calloc((size_t)(hs + n), sizeof(double));
    double* zx = (double*)calloc((size_t)(hz + n), sizeof(double));
    if (!sx || !zx) { free(sx); free(zx); return OR_ENOMEM; }
    memcpy(sx, hist_s, (size_t)hs * sizeof(double));
    if (!flush) memcpy(sx + hs, blk, (size_t)n * sizeof(double));
    memcpy(zx, hist_z, (size_t)hz * sizeof(double));
    for (int64_t u = 0; u < n; ++u) {           /* z for the new time steps */
        double acc = 0.0;
        for (int64_t q = 0; q < lf; ++q) acc += r[q] * sx[hs + u - q];
        zx[hz + u] = acc;
    }
    for (int64_t t = 0; t < n; ++t) {           /* gather over the taps */
        double acc = 0.0;
        for (int64_t j = 0; j < k; ++j) acc += g[j] * zx[hz + t - p[j]];
        out[t] = acc;
    }
    memcpy(hist_s, sx + n, (size_t)hs * sizeof(double));
    memcpy(hist_z, zx + n, (size_t)hz * sizeof(double));
    free(sx); free(zx);
    return OR_OK;
}

/* ------------------------------------------------------------------------
 * O6. Toeplitz-constrained semi-NMF (Sec. III-C and Alg. 1).
 *
 * Layout: X is [N][M], one HRIR per row (the paper's X has them as columns,
 * so X_paper[m][i] = X[i][m]); G is [N][lg]; f has lf = M - lg + 1 taps.
 * The banded Toeplitz matrix of Eq. (12) is T(f)[m][j] = f[m - j] for
 * 0 <= m - j < lf (an M x lg matrix), so T(f) G_i^T = f * g_i.
 * --------------------------------------------------------------------- */

/* SplitMix64 (Steele, Lea and Flood, 2014): state += golden gamma, then the
 * variant-13 finaliser.  Uniform (0, 1] as ((x >> 11) + 1) * 2^-53. */
static uint64_t splitmix64_next(uint64_t* state) {
    uint64_t z = (*state += 0x9E3779B97F4A7C15ULL);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

void or_splitmix64(uint64_t seed, int64_t n, uint64_t* out) {
    uint64_t st = seed;
    for (int64_t i = 0; i < n; ++i) out[i] = splitmix64_next(&st);
}

/* Alg. 1, first step: G <- rand(N, lg), i.i.d. U(0, 1], row-major draw order. */
void or_rand_g0(uint64_t seed, int64_t n, int64_t lg, double* G) {
    uint64_t st = seed;
    for (int64_t i = 0; i < n * lg; ++i)
        G[i] = (double)((splitmix64_next(&st) >> 11) + 1) * (1.0 / 9007199254740992.0);
}

/* Cholesky solve of the symmetric positive definite system A x = b (n x n). */
static int cholesky_solve(double* A, int64_t n, double* b) {
    for (int64_t j = 0; j < n; ++j) {
        double d = A[j * n + j];
        for (int64_t q = 0; q < j; ++q) d -= A[j * n + q] * A[j * n + q];
        if (!(d > 0.0)) return OR_ENOTPD;
        d = sqrt(d);
        A[j * n + j] = d;
        for (int64_t i = j + 1; i < n; ++i) {
            double v = A[i * n + j];
            for (int64_t q = 0; q < j; ++q) v -= A[i * n + q] * A[j * n + q];
            A[i * n + j] = v / d;
        }
    }
    for (int64_t i = 0; i < n; ++i) {           /* L y = b */
        double v = b[i];
        for (int64_t q = 0; q < i; ++q) v -= A[i * n + q] * b[q];
        b[i] = v / A[i * n + i];
    }
    for (int64_t i = n - 1; i >= 0; --i) {      /* L^T x = y */
        double v = b[i];
        for (int64_t q = i + 1; q < n; ++q) v -= A[q * n + i] * b[q];
        b[i] = v / A[i * n + i];
    }
    return OR_OK;
}

/* Resonance step (Eqs. (9)-(11) restricted to the lf unknowns of Eq. (13)):
 * with C = G^T G, A[n][n'] = sum_j C[j][j + n - n'] over valid j (the trace
 * of G^T G against the square shift by n - n'), b[n] = sum_i sum_j
 * G[i][j] X[i][j + n] (the trace of the shifted X G); then f = A^{-1} b. */
int or_fstep(const double* X, int64_t N, int64_t M, int64_t lf, const double* G, double* f) {
    const int64_t lg = M - lf + 1;
    if (lf < 1 || lg < 1 || N < 1) return OR_EINVAL;
    double* C = (double*)calloc((size_t)(lg * lg), sizeof(double));
    double* A = (double*)calloc((size_t)(lf * lf), sizeof(double));
    if (!C || !A) { free(C); free(A); return OR_ENOMEM; }
    for (int64_t j = 0; j < lg; ++j)
        for (int64_t l = 0; l < lg; ++l) {
            double acc = 0.0;
            for (int64_t i = 0; i < N; ++i) acc += G[i * lg + j] * G[i * lg + l];
            C[j * lg + l] = acc;
        }
    for (int64_t n = 0; n < lf; ++n)
        for (int64_t n2 = 0; n2 < lf; ++n2) {
            double acc = 0.0;
            for (int64_t j = 0; j < lg; ++j) {
                const int64_t l = j + n - n2;
                if (l >= 0 && l < lg) acc += C[j * lg + l];
            }
            A[n * lf + n2] = acc;
        }
    for (int64_t n = 0; n < lf; ++n) {
        double acc = 0.0;
        for (int64_t i = 0; i < N; ++i)
            for (int64_t j = 0; j < lg; ++j) acc += G[i * lg + j] * X[i * M + j + n];
        f[n] = acc;
    }
    const int rc = cholesky_solve(A, lf, f);
    free(C); free(A);
    return rc;
}

/* Reflection step (Eq. (4), multiplicative semi-NMF update with F = T(f)):
 * P = X^T F (here X[i] . F[:, j]), Q = F^T F,
 * G_ij <- G_ij sqrt((P+_ij + (G Q-)_ij) / (P-_ij + (G Q+)_ij)),
 * Q+ = (|Q| + Q)/2, Q- = (|Q| - Q)/2.  An entry that is already zero stays
 * zero (the update is multiplicative); for G_ij > 0 the denominator is at
 * least G_ij ||f||^2 > 0. `iters` updates with f fixed.
 * lam >= 0 adds the L1 weight of Eq. (14) to the objective,
 * ||X - F G^T||^2 + lam sum G; its gradient lam enters the update's
 * denominator as lam / 2 (lam = 0 is Eq. (4) unchanged). */
int or_gstep(const double* X, int64_t N, int64_t M, int64_t lf, const double* f, double* G, int64_t iters,
             double lam) {
    const int64_t lg = M - lf + 1;
    if (lf < 1 || lg < 1 || N < 1) return OR_EINVAL;
    double* F = (double*)calloc((size_t)(M * lg), sizeof(double));
    double* Q = (double*)calloc((size_t)(lg * lg), sizeof(double));
    double* P = (double*)calloc((size_t)(N * lg), sizeof(double));
    double* Gn = (double*)calloc((size_t)(N * lg), sizeof(double));
    if (!F || !Q || !P || !Gn) { free(F); free(Q); free(P); free(Gn); return OR_ENOMEM; }
    for (int64_t m = 0; m < M; ++m)
        for (int64_t j = 0; j < lg; ++j) {
            const int64_t d = m - j;
            F[m * lg + j] = (d >= 0 && d < lf) ? f[d] : 0.0;
        }
    for (int64_t j = 0; j < lg; ++j)
        for (int64_t l = 0; l < lg; ++l) {
            double acc = 0.0;
            for (int64_t m = 0; m < M; ++m) acc += F[m * lg + j] * F[m * lg + l];
            Q[j * lg + l] = acc;
        }
    for (int64_t i = 0; i < N; ++i)
        for (int64_t j = 0; j < lg; ++j) {
            double acc = 0.0;
            for (int64_t m = 0; m < M; ++m) acc += X[i * M + m] * F[m * lg + j];
            P[i * lg + j] = acc;
        }
    for (int64_t it = 0; it < iters; ++it) {
        for (int64_t i = 0; i < N; ++i)
            for (int64_t j = 0; j < lg; ++j) {
                const double gij = G[i * lg + j];
                if (gij == 0.0) { Gn[i * lg + j] = 0.0; continue; }
                double gqp = 0.0, gqm = 0.0;
                for (int64_t l = 0; l < lg; ++l) {
                    const double q = Q[l * lg + j];
                    gqp += G[i * lg + l] * (fabs(q) + q) * 0.5;
                    gqm += G[i * lg + l] * (fabs(q) - q) * 0.5;
                }
                const double pij = P[i * lg + j];
                const double num = (fabs(pij) + pij) * 0.5 + gqm;
                const double den = (fabs(pij) - pij) * 0.5 + gqp + 0.5 * lam;
                Gn[i * lg + j] = gij * sqrt(num / den);
            }
        memcpy(G, Gn, (size_t)(N * lg) * sizeof(double));
    }
    free(F); free(Q); free(P); free(Gn);
    return OR_OK;
}

/* Frobenius cost of Eq. (3): sum_i || x_i - f * g_i ||^2. */
double or_cost(const double* X, int64_t N, int64_t M, int64_t lf, const double* f, const double* G) {
    const int64_t lg = M - lf + 1;
    double* rec = (double*)malloc((size_t)M * sizeof(double));
    double cost = 0.0;
    for (int64_t i = 0; i < N; ++i) {
        or_conv_direct(f, lf, G + i * lg, lg, rec);
        for (int64_t m = 0; m < M; ++m) {
            const double e = X[i * M + m] - rec[m];
            cost += e * e;
        }
    }
    free(rec);
    return cost;
}

/* L1 weight at iteration t of T (0-based): lambda0 for the first 10% of the
 * iterations, then a geometric decay by 10^3 up to 50%, then 0 for the last
 * half, so the final iterations are Alg. 1 unchanged. */
double or_lambda_at(double lambda0, int64_t t, int64_t T) {
    const double a = 0.1 * (double)T, b = 0.5 * (double)T;
    if ((double)t < a) return lambda0;
    if ((double)t < b) return lambda0 * pow(1000.0, -((double)t - a) / (b - a));
    return 0.0;
}

/* Alg. 1: given G (initialised by the caller, e.g. with or_rand_g0), repeat
 * T times { f <- resonance step; rescale so ||f||_2 = 1 and G by the inverse
 * factor (the product f * g_i is unchanged); G <- one reflection step with
 * L1 weight or_lambda_at(lambda0, t, T) }, recording the cost of Eq. (3)
 * after each iteration.  With lambda0 = 0 every step is the paper's, and the
 * rescaling leaves the multiplicative update unchanged (its ratio is
 * invariant to f -> a f, G -> G / a). */
int or_factorize(const double* X, int64_t N, int64_t M, int64_t lf, int64_t T, double lambda0,
                 double* G, double* f, double* cost) {
    const int64_t lg = M - lf + 1;
    for (int64_t t = 0; t < T; ++t) {
        int rc = or_fstep(X, N, M, lf, G, f);
        if (rc) return rc;
        double nrm = 0.0;
        for (int64_t n = 0; n < lf; ++n) nrm += f[n] * f[n];
        nrm = sqrt(nrm);
        if (!(nrm > 0.0)) return OR_ENOTPD;
        for (int64_t n = 0; n < lf; ++n) f[n] /= nrm;
        for (int64_t i = 0; i < N * lg; ++i) G[i] *= nrm;
        rc = or_gstep(X, N, M, lf, f, G, 1, or_lambda_at(lambda0, t, T));
        if (rc) return rc;
        if (cost) cost[t] = or_cost(X, N, M, lf, f, G);
    }
    return OR_OK;
}

/* ------------------------------------------------------------------------
 * O7. Top-K selection and non-negative refit.
 *
 * Top-K: per row, the K largest strictly positive entries (ties -> lower
 * index), reported in ascending position; slots beyond the number found are
 * (p = 0, g = 0).  nnz[i] = number of real taps.
 * --------------------------------------------------------------------- */
void or_topk(const double* G, int64_t N, int64_t lg, int64_t K, int32_t* p, double* g, int32_t* nnz) {
    char* taken = (char*)malloc((size_t)lg);
    for (int64_t i = 0; i < N; ++i) {
        memset(taken, 0, (size_t)lg);
        int64_t cnt = 0;
        for (int64_t k = 0; k < K; ++k) {
            int64_t best = -1;
            for (int64_t j = 0; j < lg; ++j) {
                if (taken[j] || !(G[i * lg + j] > 0.0)) continue;
                if (best < 0 || G[i * lg + j] > G[i * lg + best]) best = j;
            }
            if (best < 0) break;
            taken[best] = 1;
            ++cnt;
        }
        int64_t k = 0;
        for (int64_t j = 0; j < lg; ++j)
            if (taken[j]) { p[i * K + k] = (int32_t)j; g[i * K + k] = G[i * lg + j]; ++k; }
        for (; k < K; ++k) { p[i * K + k] = 0; g[i * K + k] = 0.0; }
        nnz[i] = (int32_t)cnt;
    }
    free(taken);
}

/* Least squares min ||A x - b|| for a full-column-rank m x n A (m >= n) by
 * Householder QR.  A and b are overwritten. */
static int lsq_householder(double* A, int64_t m, int64_t n, double* b, double* x) {
    for (int64_t j = 0; j < n; ++j) {
        double nrm = 0.0;
        for (int64_t i = j; i < m; ++i) nrm += A[i * n + j] * A[i * n + j];
        nrm = sqrt(nrm);
        if (!(nrm > 0.0)) return OR_ENOTPD;
        const double alpha = A[j * n + j] > 0.0 ? -nrm : nrm;
        /* v = a_j - alpha e_j, stored in column j below the diagonal */
        A[j * n + j] -= alpha;
        double vnorm2 = 0.0;
        for (int64_t i = j; i < m; ++i) vnorm2 += A[i * n + j] * A[i * n + j];
        for (int64_t c = j + 1; c < n; ++c) {
            double d = 0.0;
            for (int64_t i = j; i < m; ++i) d += A[i * n + j] * A[i * n + c];
            d = 2.0 * d / vnorm2;
            for (int64_t i = j; i < m; ++i) A[i * n + c] -= d * A[i * n + j];
        }
        double d = 0.0;
        for (int64_t i = j; i < m; ++i) d += A[i * n + j] * b[i];
        d = 2.0 * d / vnorm2;
        for (int64_t i = j; i < m; ++i) b[i] -= d * A[i * n + j];
        A[j * n + j] = alpha;   /* R's diagonal */
    }
    for (int64_t j = n - 1; j >= 0; --j) {
        double v = b[j];
        for (int64_t c = j + 1; c < n; ++c) v -= A[j * n + c] * x[c];
        x[j] = v / A[j * n + j];
    }
    return OR_OK;
}

/* Non-negative least squares min ||A x - b||, x >= 0 (Lawson and Hanson's
 * active-set method, the NNLS the paper builds its sparsifier on).
 * A is m x n row-major.  Stops when every dual entry outside the passive
 * set is <= tol. */
int or_nnls(const double* A, int64_t m, int64_t n, const double* b, double* x, double tol) {
    char* inP = (char*)calloc((size_t)n, 1);
    double* w = (double*)malloc((size_t)n * sizeof(double));
    double* z = (double*)malloc((size_t)n * sizeof(double));
    double* As = (double*)malloc((size_t)(m * n) * sizeof(double));
    double* bs = (double*)malloc((size_t)m * sizeof(double));
    double* zs = (double*)malloc((size_t)n * sizeof(double));
    int64_t* idx = (int64_t*)malloc((size_t)n * sizeof(int64_t));
    int rc = OR_OK;
    for (int64_t j = 0; j < n; ++j) x[j] = 0.0;
    for (int64_t outer = 0; outer < 3 * n + 10; ++outer) {
        /* dual w = A^T (b - A x) */
        for (int64_t j = 0; j < n; ++j) {
            double acc = 0.0;
            for (int64_t i = 0; i < m; ++i) {
                double res = b[i];
                for (int64_t c = 0; c < n; ++c) res -= A[i * n + c] * x[c];
                acc += A[i * n + j] * res;
            }
            w[j] = acc;
        }
        int64_t t = -1;
        for (int64_t j = 0; j < n; ++j)
            if (!inP[j] && w[j] > tol && (t < 0 || w[j] > w[t])) t = j;
        if (t < 0) break;
        inP[t] = 1;
        int64_t inner = 0;
        for (;;) {
            /* unconstrained least squares on the passive set */
            int64_t np = 0;
            for (int64_t j = 0; j < n; ++j) if (inP[j]) idx[np++] = j;
            for (int64_t i = 0; i < m; ++i) {
                for (int64_t c = 0; c < np; ++c) As[i * np + c] = A[i * n + idx[c]];
                bs[i] = b[i];
            }
            rc = lsq_householder(As, m, np, bs, zs);
            if (rc) goto done;
            for (int64_t j = 0; j < n; ++j) z[j] = 0.0;
            for (int64_t c = 0; c < np; ++c) z[idx[c]] = zs[c];
            int feasible = 1;
            for (int64_t c = 0; c < np; ++c) if (!(zs[c] > 0.0)) feasible = 0;
            if (feasible) { for (int64_t j = 0; j < n; ++j) x[j] = z[j]; break; }
            /* step back to the boundary */
            double alpha = 2.0;
            for (int64_t c = 0; c < np; ++c) {
                const int64_t j = idx[c];
                if (!(z[j] > 0.0)) {
                    const double a = x[j] / (x[j] - z[j]);
                    if (a < alpha) alpha = a;
                }
            }
            for (int64_t j = 0; j < n; ++j) x[j] += alpha * (z[j] - x[j]);
            double xmax = 0.0;
            for (int64_t j = 0; j < n; ++j) if (x[j] > xmax) xmax = x[j];
            for (int64_t j = 0; j < n; ++j)
                if (inP[j] && !(x[j] > 1e-15 * xmax)) { inP[j] = 0; x[j] = 0.0; }
            if (++inner > n + 1) break;   /* each pass removes at least one index */
        }
    }
done:
    free(inP); free(w); free(z); free(As); free(bs); free(zs); free(idx);
    return rc;
}

/* Refit of the kept gains: with f fixed, each row's gains on its support S
 * solve min_{gamma >= 0} || x_i - T(f)[:, S] gamma ||^2 (Eq. (14) with
 * lambda = 0 on the support and the identity transform). */
int or_refit(const double* X, int64_t N, int64_t M, int64_t lf, const double* f,
             const int32_t* p, const int32_t* nnz, int64_t K, double* g) {
    const int64_t lg = M - lf + 1;
    (void)lg;
    double* A = (double*)malloc((size_t)(M * K) * sizeof(double));
    double* x = (double*)malloc((size_t)K * sizeof(double));
    int rc = OR_OK;
    for (int64_t i = 0; i < N && rc == OR_OK; ++i) {
        const int64_t n = nnz[i];
        for (int64_t m = 0; m < M; ++m)
            for (int64_t c = 0; c < n; ++c) {
                const int64_t d = m - (int64_t)p[i * K + c];
                A[m * n + c] = (d >= 0 && d < lf) ? f[d] : 0.0;
            }
        double scale = 0.0;               /* dual tolerance relative to |A^T x_i| */
        for (int64_t c = 0; c < n; ++c) {
            double d = 0.0;
            for (int64_t m = 0; m < M; ++m) d += A[m * n + c] * X[i * M + m];
            if (fabs(d) > scale) scale = fabs(d);
        }
        if (n > 0) rc = or_nnls(A, M, n, X + i * M, x, 1e-12 * scale);
        for (int64_t c = 0; c < K; ++c) g[i * K + c] = (c < n) ? x[c] : 0.0;
    }
    free(A); free(x);
    return rc;
}

/* Threads an OpenMP parallel region of this library uses (1 without OpenMP). */
int or_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
