// The paper's own sparsifier (Sec. III-D): with the resonance filter f
// fixed, each reflection filter solves the penalised L1-NNLS problem of
// Eq. (14),
//     min_g ||D (T(f) g - x)||^2 + lambda sum(g),  g >= 0,
// for a residual transform D (identity, the Gaussian convolution of Eq. (15)
// or the Gaussian time window of Eq. (16)); entries at or below a threshold
// (1e-4 in the paper) are then discarded.  lambda may be given per filter or
// searched for a target NNZE; the window bandwidth may be tuned per HRIR over
// a grid by spectral distortion (Sec. IV-E).  Host, FP64.
//
// With A = D T(f) and b = D x the problem is min 1/2 g^T H g - c^T g over
// g >= 0 with H = A^T A and c = A^T b - lambda / 2, solved by the same
// active-set NNLS as the top-K refit.  H depends only on (transform, sigma),
// so it is formed once per bandwidth and shared by every filter.
#include <cmath>
#include <cstring>
#include <vector>

#include "hrir_internal.h"

namespace hrir {
namespace {

struct Design {
    int m = 0, lg = 0;
    std::vector<double> A;     // m x lg, row-major: A = D T(f)
    std::vector<double> D;     // m x m (dense), or empty for a diagonal / identity
    std::vector<double> dg;    // diagonal of D (window), empty otherwise
    std::vector<double> H;     // lg x lg: A^T A
};

double gauss_conv(double k, double sigma) {
    return std::exp(-(k * k) / (2.0 * sigma * sigma)) / (sigma * std::sqrt(2.0 * M_PI));
}

// A = D T(f), with T(f)[i][j] = f[i - j] (m = lf + lg - 1 rows).
void build_design(Design& d, const double* f, int lf, int lg, int transform, double sigma) {
    const int m = lf + lg - 1;
    d.m = m;
    d.lg = lg;
    d.D.clear();
    d.dg.clear();
    if (transform == HRIR_D_WINDOW && std::isfinite(sigma)) {
        d.dg.resize(m);
        for (int i = 0; i < m; ++i) d.dg[i] = std::exp(-((double)i * i) / (sigma * sigma));
    } else if (transform == HRIR_D_CONV) {
        d.D.resize((size_t)m * m);
        for (int i = 0; i < m; ++i)
            for (int j = 0; j < m; ++j) d.D[(size_t)i * m + j] = gauss_conv((double)(i - j), sigma);
    }
    d.A.assign((size_t)m * lg, 0.0);
    for (int j = 0; j < lg; ++j)
        for (int q = 0; q < lf; ++q) d.A[(size_t)(j + q) * lg + j] = f[q];
    if (!d.dg.empty()) {
        for (int i = 0; i < m; ++i)
            for (int j = 0; j < lg; ++j) d.A[(size_t)i * lg + j] *= d.dg[i];
    } else if (!d.D.empty()) {
        std::vector<double> T = d.A;
        for (int i = 0; i < m; ++i)
            for (int j = 0; j < lg; ++j) {
                double v = 0.0;
                for (int q = j; q < std::min(m, j + lf); ++q) v += d.D[(size_t)i * m + q] * T[(size_t)q * lg + j];
                d.A[(size_t)i * lg + j] = v;
            }
    }
    d.H.assign((size_t)lg * lg, 0.0);
    for (int a = 0; a < lg; ++a)
        for (int b = a; b < lg; ++b) {
            double v = 0.0;
            for (int i = 0; i < m; ++i) v += d.A[(size_t)i * lg + a] * d.A[(size_t)i * lg + b];
            d.H[(size_t)a * lg + b] = v;
            d.H[(size_t)b * lg + a] = v;
        }
}

// c0 = A^T (D x): the lambda-free part of the linear term.
void design_rhs(const Design& d, const double* x, std::vector<double>& c0) {
    std::vector<double> b(d.m);
    for (int i = 0; i < d.m; ++i) {
        if (!d.dg.empty()) {
            b[i] = d.dg[i] * x[i];
        } else if (!d.D.empty()) {
            double v = 0.0;
            for (int q = 0; q < d.m; ++q) v += d.D[(size_t)i * d.m + q] * x[q];
            b[i] = v;
        } else {
            b[i] = x[i];
        }
    }
    c0.assign(d.lg, 0.0);
    for (int i = 0; i < d.m; ++i)
        for (int j = 0; j < d.lg; ++j) c0[j] += d.A[(size_t)i * d.lg + j] * b[i];
}

// One L1-NNLS solve into y (warm: starting from y's current contents) and
// the discard into g; returns the status and the NNZE.
int solve_one(const Design& d, const std::vector<double>& c0, double lambda, double thresh, std::vector<double>& c,
              std::vector<double>& y, bool warm, double* g, int* nnze) {
    c.resize(d.lg);
    y.resize(d.lg, 0.0);
    for (int j = 0; j < d.lg; ++j) c[j] = c0[j] - 0.5 * lambda;
    const int rc = nnls_normal(d.H, c, d.lg, y.data(), warm);
    if (rc) return rc;
    int nz = 0;
    for (int j = 0; j < d.lg; ++j) {
        g[j] = std::fabs(y[j]) <= thresh ? 0.0 : y[j];
        nz += g[j] != 0.0;
    }
    *nnze = nz;
    return HRIR_OK;
}

// Geometric bisection on [1e-12, 1] * lambda_max for the smallest lambda whose
// solution keeps at most `target` entries (lambda = 0 if it already does).
int search_lambda(const Design& d, const std::vector<double>& c0, int target, double thresh, double* g,
                  double* lambda_out, int* nnze_out) {
    std::vector<double> c, y, gt(d.lg);
    int nz = 0;
    int rc = solve_one(d, c0, 0.0, thresh, c, y, false, g, &nz);
    if (rc) return rc;
    if (nz <= target) {
        *lambda_out = 0.0;
        *nnze_out = nz;
        return HRIR_OK;
    }
    double cmax = 0.0;
    for (double v : c0) cmax = std::max(cmax, v);
    double hi = 2.0 * cmax, lo = hi * 1e-12;
    std::fill(g, g + d.lg, 0.0);
    int nz_hi = 0;
    for (int it = 0; it < 50; ++it) {
        const double mid = std::sqrt(lo * hi);
        // each step starts from the previous step's minimiser (unthresholded)
        rc = solve_one(d, c0, mid, thresh, c, y, true, gt.data(), &nz);
        if (rc) return rc;
        if (nz <= target) {
            hi = mid;
            nz_hi = nz;
            std::memcpy(g, gt.data(), sizeof(double) * d.lg);
        } else {
            lo = mid;
        }
    }
    *lambda_out = hi;
    *nnze_out = nz_hi;
    return HRIR_OK;
}

// Magnitudes of the length-m DFT through a cosine / sine table built once.
struct Dft {
    int m = 0;
    std::vector<double> cs, sn;    // m x m
    explicit Dft(int m_) : m(m_), cs((size_t)m_ * m_), sn((size_t)m_ * m_) {
        for (int k = 0; k < m; ++k)
            for (int t = 0; t < m; ++t) {
                const double ang = -2.0 * M_PI * (double)(((int64_t)k * t) % m) / (double)m;
                cs[(size_t)k * m + t] = std::cos(ang);
                sn[(size_t)k * m + t] = std::sin(ang);
            }
    }
    // |DFT(h)| floored at 1e-12 of its maximum
    void floored_magnitude(const double* h, double* mag) const {
        double mx = 0.0;
        for (int k = 0; k < m; ++k) {
            double re = 0.0, im = 0.0;
            for (int t = 0; t < m; ++t) {
                re += h[t] * cs[(size_t)k * m + t];
                im += h[t] * sn[(size_t)k * m + t];
            }
            mag[k] = std::hypot(re, im);
            mx = std::max(mx, mag[k]);
        }
        const double fl = 1e-12 * std::max(mx, 1e-300);
        for (int k = 0; k < m; ++k) mag[k] = std::max(mag[k], fl);
    }
};

// Spectral distortion (Eq. (17)) between two floored magnitude spectra.
double spectral_distortion(const double* a, const double* b, int m) {
    double acc = 0.0;
    for (int k = 0; k < m; ++k) {
        const double v = 20.0 * std::log10(a[k] / b[k]);
        acc += v * v;
    }
    return std::sqrt(acc / m);
}

void convolve(const double* f, int lf, const double* g, int lg, double* y) {
    const int m = lf + lg - 1;
    for (int t = 0; t < m; ++t) y[t] = 0.0;
    for (int j = 0; j < lg; ++j)
        if (g[j] != 0.0)
            for (int q = 0; q < lf; ++q) y[j + q] += f[q] * g[j];
}

// Writes row i's tap table (the k largest kept entries, ties to the lower
// position, ascending positions, padded with (0, 0)) and its error.
void finish_row(const double* X, int m, const double* f, int lf, int lg, int k, int64_t i, const double* g,
                int nz, double lam, int32_t* p_out, float* g_out, int32_t* nnze_out, double* lambda_out,
                double* err_db_out) {
    std::vector<int> idx;
    for (int j = 0; j < lg; ++j)
        if (g[j] != 0.0) idx.push_back(j);
    if ((int)idx.size() > k) {
        std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) { return g[a] > g[b]; });
        idx.resize(k);
        std::sort(idx.begin(), idx.end());
    }
    std::vector<double> gk(lg, 0.0);
    for (int a = 0; a < k; ++a) {
        const bool real = a < (int)idx.size();
        p_out[(size_t)i * k + a] = real ? idx[a] : 0;
        g_out[(size_t)i * k + a] = real ? (float)g[idx[a]] : 0.0f;
        if (real) gk[idx[a]] = g[idx[a]];
    }
    if (nnze_out) nnze_out[i] = nz;
    if (lambda_out) lambda_out[i] = lam;
    if (err_db_out) {
        const double* x = X + (size_t)i * m;
        std::vector<double> y(m);
        convolve(f, lf, gk.data(), lg, y.data());
        double e = 0.0, ex = 0.0;
        for (int t = 0; t < m; ++t) {
            e += (x[t] - y[t]) * (x[t] - y[t]);
            ex += x[t] * x[t];
        }
        err_db_out[i] = (ex > 0.0 && e > 0.0) ? 10.0 * std::log10(e / ex) : (e > 0.0 ? INFINITY : -INFINITY);
    }
}

// Every distinct design's H, concatenated ([n_designs][lg][lg]), for the
// device solver.
std::vector<double> stack_h(const std::vector<Design>& designs, int lg) {
    std::vector<double> H(designs.size() * (size_t)lg * lg);
    for (size_t u = 0; u < designs.size(); ++u)
        std::copy(designs[u].H.begin(), designs[u].H.end(), H.begin() + u * (size_t)lg * lg);
    return H;
}

int check_common(const double* X, int n, int m, const double* f, int lf, const char* fn) {
    if (!X || !f) return fail(HRIR_EINVAL, "%s: null pointer", fn);
    if (n < 1 || lf < 1 || m < lf) return fail(HRIR_EINVAL, "%s: need n >= 1 and 1 <= lf <= m", fn);
    if ((int64_t)m * m > (int64_t)1 << 26) return fail(HRIR_EINVAL, "%s: m=%d too large", fn, m);
    for (int64_t i = 0; i < (int64_t)n * m; ++i)
        if (!std::isfinite(X[i])) return fail(HRIR_EINVAL, "%s: X has a non-finite entry", fn);
    for (int q = 0; q < lf; ++q)
        if (!std::isfinite(f[q])) return fail(HRIR_EINVAL, "%s: f has a non-finite entry", fn);
    return HRIR_OK;
}

}  // namespace
}  // namespace hrir

using hrir::fail;

namespace {

int sparsify_impl(const double* X, int32_t n, int32_t m, const double* f, int32_t lf, int32_t transform,
                  const double* sigma, const double* lambda, int32_t target_nnze, double threshold, int32_t k,
                  int32_t* p_out, float* g_out, int32_t* nnze_out, double* lambda_out, double* err_db_out,
                  bool device) {
    hrir::clear_error();
    int rc = hrir::check_common(X, n, m, f, lf, "hrir_sparsify");
    if (rc) return rc;
    if (!p_out || !g_out) return fail(HRIR_EINVAL, "hrir_sparsify: null output pointer");
    if (transform != HRIR_D_IDENTITY && transform != HRIR_D_CONV && transform != HRIR_D_WINDOW)
        return fail(HRIR_EINVAL, "hrir_sparsify: unknown transform %d", transform);
    if (transform != HRIR_D_IDENTITY) {
        if (!sigma) return fail(HRIR_EINVAL, "hrir_sparsify: transform %d needs sigma", transform);
        for (int i = 0; i < n; ++i)
            if (!(sigma[i] > 0.0) || (transform == HRIR_D_CONV && !std::isfinite(sigma[i])))
                return fail(HRIR_EINVAL, "hrir_sparsify: sigma[%d]=%g invalid", i, sigma[i]);
    }
    if (lambda) {
        for (int i = 0; i < n; ++i)
            if (!(lambda[i] >= 0.0) || !std::isfinite(lambda[i]))
                return fail(HRIR_EINVAL, "hrir_sparsify: lambda[%d]=%g invalid", i, lambda[i]);
    } else if (target_nnze < 0) {
        return fail(HRIR_EINVAL, "hrir_sparsify: target_nnze=%d < 0", target_nnze);
    }
    if (!(threshold >= 0.0)) return fail(HRIR_EINVAL, "hrir_sparsify: threshold < 0");
    if (k < 1) return fail(HRIR_EINVAL, "hrir_sparsify: k=%d < 1", k);
    const int lg = m - lf + 1;

    // one design per distinct bandwidth, in order of first use
    std::vector<double> keys;
    std::vector<int> which(n, 0);
    for (int i = 0; i < n; ++i) {
        const double s = transform == HRIR_D_IDENTITY ? INFINITY : sigma[i];
        int w = -1;
        for (size_t u = 0; u < keys.size(); ++u)
            if (keys[u] == s || (std::isinf(keys[u]) && std::isinf(s))) w = (int)u;
        if (w < 0) {
            w = (int)keys.size();
            keys.push_back(s);
        }
        which[i] = w;
    }
    std::vector<hrir::Design> designs(keys.size());
    hrir::parallel_for((int64_t)keys.size(), [&](int64_t u) {
        hrir::build_design(designs[u], f, lf, lg, transform, keys[u]);
    });

    if (device) {
        // the solves on the GPU, everything around them on the host
        std::vector<double> C((size_t)n * lg), G((size_t)n * lg), lam(n);
        std::vector<int> nz(n);
        hrir::parallel_for(n, [&](int64_t i) {
            std::vector<double> c0;
            hrir::design_rhs(designs[which[i]], X + (size_t)i * m, c0);
            std::copy(c0.begin(), c0.end(), C.begin() + i * lg);
        });
        const std::vector<double> Hs = hrir::stack_h(designs, lg);
        rc = hrir::l1_solve_device(Hs.data(), (int)designs.size(), lg, C.data(), which.data(), n, lambda,
                                   target_nnze, threshold, G.data(), lam.data(), nz.data());
        if (rc) return rc;
        hrir::parallel_for(n, [&](int64_t i) {
            hrir::finish_row(X, m, f, lf, lg, k, i, G.data() + i * lg, nz[i], lam[i], p_out, g_out, nnze_out,
                             lambda_out, err_db_out);
        });
        return HRIR_OK;
    }
    std::vector<int> status(n, 0);
    hrir::parallel_for(n, [&](int64_t i) {
        const hrir::Design& d = designs[which[i]];
        std::vector<double> c0, c, y, g(lg);
        hrir::design_rhs(d, X + (size_t)i * m, c0);
        double lam = 0.0;
        int nz = 0;
        int st;
        if (lambda) {
            lam = lambda[i];
            st = hrir::solve_one(d, c0, lam, threshold, c, y, false, g.data(), &nz);
        } else {
            st = hrir::search_lambda(d, c0, target_nnze, threshold, g.data(), &lam, &nz);
        }
        status[i] = st;
        if (st) return;
        hrir::finish_row(X, m, f, lf, lg, k, i, g.data(), nz, lam, p_out, g_out, nnze_out, lambda_out, err_db_out);
    });
    for (int i = 0; i < n; ++i)
        if (status[i]) return fail(status[i], "hrir_sparsify: NNLS failed on row %d", i);
    return HRIR_OK;
}

}  // namespace

extern "C" int hrir_sparsify(const double* X, int32_t n, int32_t m, const double* f, int32_t lf, int32_t transform,
                             const double* sigma, const double* lambda, int32_t target_nnze, double threshold,
                             int32_t k, int32_t* p_out, float* g_out, int32_t* nnze_out, double* lambda_out,
                             double* err_db_out) {
    return sparsify_impl(X, n, m, f, lf, transform, sigma, lambda, target_nnze, threshold, k, p_out, g_out, nnze_out,
                         lambda_out, err_db_out, false);
}

extern "C" int hrir_sparsify_device(const double* X, int32_t n, int32_t m, const double* f, int32_t lf,
                                    int32_t transform, const double* sigma, const double* lambda,
                                    int32_t target_nnze, double threshold, int32_t k, int32_t* p_out, float* g_out,
                                    int32_t* nnze_out, double* lambda_out, double* err_db_out) {
    return sparsify_impl(X, n, m, f, lf, transform, sigma, lambda, target_nnze, threshold, k, p_out, g_out, nnze_out,
                         lambda_out, err_db_out, true);
}

namespace {

int tune_sigma_impl(const double* X, int32_t n, int32_t m, const double* f, int32_t lf, const double* grid,
                    int32_t n_grid, double lambda, int32_t target_nnze, double threshold, double* sigma_out,
                    double* sd_out, bool device) {
    hrir::clear_error();
    int rc = hrir::check_common(X, n, m, f, lf, "hrir_tune_sigma");
    if (rc) return rc;
    if (!grid || n_grid < 1 || !sigma_out) return fail(HRIR_EINVAL, "hrir_tune_sigma: empty grid or null output");
    for (int u = 0; u < n_grid; ++u)
        if (!(grid[u] > 0.0)) return fail(HRIR_EINVAL, "hrir_tune_sigma: grid[%d]=%g must be > 0", u, grid[u]);
    if (!(lambda >= 0.0) || !std::isfinite(lambda)) return fail(HRIR_EINVAL, "hrir_tune_sigma: lambda invalid");
    if (target_nnze < 0) return fail(HRIR_EINVAL, "hrir_tune_sigma: target_nnze=%d < 0", target_nnze);
    if (!(threshold >= 0.0)) return fail(HRIR_EINVAL, "hrir_tune_sigma: threshold < 0");
    const int lg = m - lf + 1;
    std::vector<hrir::Design> designs(n_grid);
    hrir::parallel_for(n_grid, [&](int64_t u) {
        hrir::build_design(designs[u], f, lf, lg, HRIR_D_WINDOW, grid[u]);
    });
    const hrir::Dft dft(m);
    // the solution of row i at grid entry u: on the device all n * n_grid
    // problems at once (problem i * n_grid + u), else per row on the host
    std::vector<double> G;
    if (device) {
        const int64_t np = (int64_t)n * n_grid;
        if (np > INT32_MAX / 2) return fail(HRIR_EINVAL, "hrir_tune_sigma: too many problems");
        std::vector<double> C((size_t)np * lg), lam(np, lambda), lam_out(np);
        std::vector<int> which(np), nz(np);
        hrir::parallel_for(n, [&](int64_t i) {
            std::vector<double> c0;
            for (int u = 0; u < n_grid; ++u) {
                hrir::design_rhs(designs[u], X + (size_t)i * m, c0);
                std::copy(c0.begin(), c0.end(), C.begin() + (i * n_grid + u) * lg);
                which[i * n_grid + u] = u;
            }
        });
        G.resize((size_t)np * lg);
        const std::vector<double> Hs = hrir::stack_h(designs, lg);
        rc = hrir::l1_solve_device(Hs.data(), n_grid, lg, C.data(), which.data(), (int)np,
                                   target_nnze > 0 ? nullptr : lam.data(), target_nnze, threshold, G.data(),
                                   lam_out.data(), nz.data());
        if (rc) return rc;
    }
    std::vector<int> status(n, 0);
    hrir::parallel_for(n, [&](int64_t i) {
        const double* x = X + (size_t)i * m;
        std::vector<double> c0, c, yh, gh(lg), y(m), mx(m), my(m);
        dft.floored_magnitude(x, mx.data());
        double best = INFINITY, best_s = grid[0];
        for (int u = 0; u < n_grid; ++u) {
            const double* g = gh.data();
            if (device) {
                g = G.data() + (i * n_grid + u) * lg;
            } else {
                hrir::design_rhs(designs[u], x, c0);
                int nz = 0;
                double lam = lambda;
                const int st = target_nnze > 0
                                   ? hrir::search_lambda(designs[u], c0, target_nnze, threshold, gh.data(), &lam, &nz)
                                   : hrir::solve_one(designs[u], c0, lambda, threshold, c, yh, false, gh.data(), &nz);
                if (st) {
                    status[i] = st;
                    return;
                }
            }
            hrir::convolve(f, lf, g, lg, y.data());
            dft.floored_magnitude(y.data(), my.data());
            const double sd = hrir::spectral_distortion(mx.data(), my.data(), m);
            if (sd < best) {
                best = sd;
                best_s = grid[u];
            }
        }
        sigma_out[i] = best_s;
        if (sd_out) sd_out[i] = best;
    });
    for (int i = 0; i < n; ++i)
        if (status[i]) return fail(status[i], "hrir_tune_sigma: NNLS failed on row %d", i);
    return HRIR_OK;
}

}  // namespace

extern "C" int hrir_tune_sigma(const double* X, int32_t n, int32_t m, const double* f, int32_t lf,
                               const double* grid, int32_t n_grid, double lambda, int32_t target_nnze,
                               double threshold, double* sigma_out, double* sd_out) {
    return tune_sigma_impl(X, n, m, f, lf, grid, n_grid, lambda, target_nnze, threshold, sigma_out, sd_out, false);
}

extern "C" int hrir_tune_sigma_device(const double* X, int32_t n, int32_t m, const double* f, int32_t lf,
                                      const double* grid, int32_t n_grid, double lambda, int32_t target_nnze,
                                      double threshold, double* sigma_out, double* sd_out) {
    return tune_sigma_impl(X, n, m, f, lf, grid, n_grid, lambda, target_nnze, threshold, sigma_out, sd_out, true);
}

// Fallback rule of the surrogate: directions are compared by the angle between
// their unit vectors in the interaural-polar convention of the direction grid
// (lateral angle az, polar angle el): (sin az, cos az cos el, cos az sin el).
extern "C" int surrogate_select(const double* q_az, const double* q_el, int32_t n_q, const double* val_az,
                                const double* val_el, const double* val_err_db, int32_t n_val, const double* meas_az,
                                const double* meas_el, int32_t n_meas, double max_err_db, int32_t* choice) {
    hrir::clear_error();
    if (n_q < 0 || n_val < 1 || n_meas < 1) return fail(HRIR_EINVAL, "surrogate_select: need n_val, n_meas >= 1");
    if ((n_q > 0 && (!q_az || !q_el || !choice)) || !val_az || !val_el || !val_err_db || !meas_az || !meas_el)
        return fail(HRIR_EINVAL, "surrogate_select: null pointer");
    auto unit = [](double az, double el, double* v) {
        v[0] = std::sin(az);
        v[1] = std::cos(az) * std::cos(el);
        v[2] = std::cos(az) * std::sin(el);
    };
    std::vector<double> V((size_t)n_val * 3), Ms((size_t)n_meas * 3);
    for (int i = 0; i < n_val; ++i) unit(val_az[i], val_el[i], &V[(size_t)i * 3]);
    for (int i = 0; i < n_meas; ++i) unit(meas_az[i], meas_el[i], &Ms[(size_t)i * 3]);
    // nearest by largest dot product; ties keep the lower index
    auto nearest = [](const std::vector<double>& T, int n, const double* v) {
        int best = 0;
        double bd = -2.0;
        for (int i = 0; i < n; ++i) {
            const double d = T[(size_t)i * 3] * v[0] + T[(size_t)i * 3 + 1] * v[1] + T[(size_t)i * 3 + 2] * v[2];
            if (d > bd) {
                bd = d;
                best = i;
            }
        }
        return best;
    };
    hrir::parallel_for(n_q, [&](int64_t i) {
        double v[3];
        unit(q_az[i], q_el[i], v);
        const int nv = nearest(V, n_val, v);
        choice[i] = val_err_db[nv] > max_err_db ? nearest(Ms, n_meas, v) : -1;
    });
    return HRIR_OK;
}
