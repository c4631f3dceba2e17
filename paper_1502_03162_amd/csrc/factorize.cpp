// Host-side factorization of an HRIR set into one resonance filter and sparse
// non-negative reflection filters: Toeplitz-constrained semi-NMF (Sec. III-C,
// Alg. 1), top-K support selection, and a non-negative least-squares refit of
// the kept gains (Eq. (14) with lambda = 0 on the support).  FP64.
//
// Every matrix the paper forms is banded Toeplitz here and is never built:
//  * resonance system (Eqs. (10), (11) restricted to the lf unknowns of
//    Eq. (13)): A[q][q'] = a[|q - q'|] with a[d] = sum_i sum_j G_ij G_i,j+d,
//    and b[q] = sum_i sum_j G_ij X_i,j+q;
//  * reflection update (Eq. (4) with F = T(f)): X^T F is a per-row
//    cross-correlation of X with f, and F^T F is the autocorrelation of f,
//    zero beyond lag lf - 1, so G (F^T F)^{+/-} costs O(n lg lf).
// Sums over rows are formed per row and then added in row order, so results
// do not depend on the number of threads.
#include <cmath>
#include <cstring>
#include <numeric>

#include "hrir_internal.h"

namespace hrir {
namespace {

uint64_t splitmix_next(uint64_t& state) {
    state += 0x9E3779B97F4A7C15ull;
    uint64_t z = state;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}


}  // namespace

// L1 weight at iteration t of T: hold for 10%, geometric decay by 1e3 until
// 50%, then zero.
double l1_weight(double lambda0, int t, int T) {
    const double hold = 0.1 * T, stop = 0.5 * T;
    if (t < hold) return lambda0;
    if (t < stop) return lambda0 * std::pow(1000.0, -(t - hold) / (stop - hold));
    return 0.0;
}

// In-place Cholesky factorisation of an s x s SPD matrix (lower triangle)
// followed by the two triangular solves for rhs.  Returns false if not PD.
bool spd_solve(std::vector<double>& H, int s, double* rhs) {
    for (int c = 0; c < s; ++c) {
        double d = H[c * s + c];
        for (int q = 0; q < c; ++q) d -= H[c * s + q] * H[c * s + q];
        if (!(d > 0.0) || !std::isfinite(d)) return false;
        const double l = std::sqrt(d);
        H[c * s + c] = l;
        for (int rr = c + 1; rr < s; ++rr) {
            double v = H[rr * s + c];
            for (int q = 0; q < c; ++q) v -= H[rr * s + q] * H[c * s + q];
            H[rr * s + c] = v / l;
        }
    }
    for (int rr = 0; rr < s; ++rr) {
        double v = rhs[rr];
        for (int q = 0; q < rr; ++q) v -= H[rr * s + q] * rhs[q];
        rhs[rr] = v / H[rr * s + rr];
    }
    // back substitution, each row's terms from the last unknown down (the
    // order a column-at-a-time solve on the device takes too)
    for (int rr = s - 1; rr >= 0; --rr) {
        double v = rhs[rr];
        for (int q = s - 1; q > rr; --q) v -= H[q * s + rr] * rhs[q];
        rhs[rr] = v / H[rr * s + rr];
    }
    return true;
}

namespace {

struct Problem {
    const double* X;
    int n, m, lf, lg;
};

// f <- argmin_f sum_i ||x_i - f * g_i||^2 for fixed G.
int resonance_step(const Problem& pr, const double* G, double* f, std::vector<double>& part) {
    const int lf = pr.lf, lg = pr.lg, m = pr.m;
    part.assign((size_t)pr.n * 2 * lf, 0.0);
    parallel_for(pr.n, [&](int64_t i) {
        const double* g = G + i * lg;
        const double* x = pr.X + i * m;
        double* a = &part[(size_t)i * 2 * lf];
        double* b = a + lf;
        for (int d = 0; d < lf; ++d) {
            double s = 0.0;
            for (int j = 0; j + d < lg; ++j) s += g[j] * g[j + d];
            a[d] = s;
        }
        for (int q = 0; q < lf; ++q) {
            double s = 0.0;
            for (int j = 0; j < lg; ++j) s += g[j] * x[j + q];
            b[q] = s;
        }
    });
    std::vector<double> a(lf, 0.0);
    for (int64_t i = 0; i < pr.n; ++i)
        for (int d = 0; d < lf; ++d) {
            a[d] += part[(size_t)i * 2 * lf + d];
            if (i == 0) f[d] = 0.0;
            f[d] += part[(size_t)i * 2 * lf + lf + d];
        }
    std::vector<double> A((size_t)lf * lf);
    for (int q = 0; q < lf; ++q)
        for (int q2 = 0; q2 < lf; ++q2) A[(size_t)q * lf + q2] = a[std::abs(q - q2)];
    if (!spd_solve(A, lf, f))
        return fail(HRIR_ENOTPD, "resonance system is not positive definite (G has no energy?)");
    return HRIR_OK;
}

// Autocorrelation of f at lags [0, lf): the non-zero band of F^T F.
void autocorr(const double* f, int lf, double* ac) {
    for (int d = 0; d < lf; ++d) {
        double s = 0.0;
        for (int q = 0; q + d < lf; ++q) s += f[q] * f[q + d];
        ac[d] = s;
    }
}

// One multiplicative reflection update (Eq. (4)), L1 weight lam.
void reflection_step(const Problem& pr, const double* f, const double* G, double* Gn, double lam) {
    const int lf = pr.lf, lg = pr.lg, m = pr.m;
    std::vector<double> ac(lf), qp(lf), qm(lf);
    autocorr(f, lf, ac.data());
    for (int d = 0; d < lf; ++d) {
        qp[d] = 0.5 * (std::fabs(ac[d]) + ac[d]);
        qm[d] = 0.5 * (std::fabs(ac[d]) - ac[d]);
    }
    const double half_lam = 0.5 * lam;
    parallel_for(pr.n, [&](int64_t i) {
        const double* g = G + (size_t)i * lg;
        const double* x = pr.X + (size_t)i * m;
        double* gn = Gn + (size_t)i * lg;
        for (int j = 0; j < lg; ++j) {
            if (g[j] == 0.0) { gn[j] = 0.0; continue; }
            double xf = 0.0;                       // (X^T F)_ij
            for (int q = 0; q < lf; ++q) xf += x[j + q] * f[q];
            double up = 0.0, um = 0.0;              // (G Q+)_ij, (G Q-)_ij
            const int l0 = std::max(0, j - lf + 1), l1 = std::min(lg - 1, j + lf - 1);
            for (int l = l0; l <= l1; ++l) {
                const int d = std::abs(l - j);
                up += g[l] * qp[d];
                um += g[l] * qm[d];
            }
            const double num = 0.5 * (std::fabs(xf) + xf) + um;
            const double den = 0.5 * (std::fabs(xf) - xf) + up + half_lam;
            gn[j] = g[j] * std::sqrt(num / den);
        }
    });
}

double residual_energy_row(const double* x, int m, const double* f, int lf, const double* g, int lg) {
    double e = 0.0;
    for (int t = 0; t < m; ++t) {
        double rec = 0.0;
        const int j0 = std::max(0, t - lf + 1), j1 = std::min(lg - 1, t);
        for (int j = j0; j <= j1; ++j) rec += f[t - j] * g[j];
        const double d = x[t] - rec;
        e += d * d;
    }
    return e;
}


}  // namespace

// Lawson-Hanson active set on the normal equations: min 1/2 y^T H y - c^T y,
// y >= 0, with H = A^T A (s x s) and c = A^T x.
int nnls_normal(const std::vector<double>& H, const std::vector<double>& c, int s, double* y, bool warm) {
    std::vector<char> passive(s, 0);
    std::vector<double> w(s), z(s), Hs, rhs;
    std::vector<int> idx;
    double cmax = 0.0;
    for (int j = 0; j < s; ++j) cmax = std::max(cmax, std::fabs(c[j]));
    const double tol = 1e-12 * cmax;
    // a warm start keeps y (>= 0) and takes its support as the passive set;
    // the first step then solves on that set before any entry is added
    bool solve_first = false;
    for (int j = 0; j < s; ++j) {
        if (warm && y[j] > 0.0) {
            passive[j] = 1;
            solve_first = true;
        } else {
            y[j] = 0.0;
        }
    }
    for (int outer = 0; outer < 3 * s + 10; ++outer) {
        if (!solve_first) {
            for (int j = 0; j < s; ++j) {
                double v = c[j];
                for (int q = 0; q < s; ++q) v -= H[(size_t)j * s + q] * y[q];
                w[j] = v;
            }
            int best = -1;
            for (int j = 0; j < s; ++j)
                if (!passive[j] && w[j] > tol && (best < 0 || w[j] > w[best])) best = j;
            if (best < 0) break;
            passive[best] = 1;
        }
        solve_first = false;
        for (int inner = 0; inner <= s + 1; ++inner) {
            idx.clear();
            for (int j = 0; j < s; ++j)
                if (passive[j]) idx.push_back(j);
            const int np = (int)idx.size();
            Hs.assign((size_t)np * np, 0.0);
            rhs.assign(np, 0.0);
            for (int a = 0; a < np; ++a) {
                rhs[a] = c[idx[a]];
                for (int b = 0; b < np; ++b) Hs[(size_t)a * np + b] = H[(size_t)idx[a] * s + idx[b]];
            }
            if (np > 0 && !spd_solve(Hs, np, rhs.data()))
                return fail(HRIR_ENOTPD, "NNLS refit: support columns are linearly dependent");
            bool all_pos = true;
            for (int a = 0; a < np; ++a)
                if (!(rhs[a] > 0.0)) all_pos = false;
            std::fill(z.begin(), z.end(), 0.0);
            for (int a = 0; a < np; ++a) z[idx[a]] = rhs[a];
            if (all_pos) {
                for (int j = 0; j < s; ++j) y[j] = z[j];
                break;
            }
            double alpha = 1.0;
            for (int a = 0; a < np; ++a) {
                const int j = idx[a];
                if (!(z[j] > 0.0)) alpha = std::min(alpha, y[j] / (y[j] - z[j]));
            }
            double ymax = 0.0;
            for (int j = 0; j < s; ++j) {
                y[j] += alpha * (z[j] - y[j]);
                ymax = std::max(ymax, y[j]);
            }
            for (int j = 0; j < s; ++j)
                if (passive[j] && !(y[j] > 1e-15 * ymax)) { passive[j] = 0; y[j] = 0.0; }
        }
    }
    return HRIR_OK;
}

}  // namespace hrir

using hrir::fail;

extern "C" int hrir_factorize(const double* X, int32_t n, int32_t m, int32_t lf, int32_t iters,
                              uint64_t seed, const double* g0, double lambda0, int32_t k,
                              uint32_t flags, double* f_out, double* gdense_out, int32_t* p_out,
                              float* g_out, int32_t* nnz_out, double* err_db_out,
                              double* cost_out) {
    hrir::clear_error();
    if (!X || !f_out || !p_out || !g_out) return fail(HRIR_EINVAL, "hrir_factorize: null required pointer");
    if (n < 1 || m < 1 || lf < 1 || lf > m || iters < 1)
        return fail(HRIR_EINVAL, "hrir_factorize: need n >= 1, 1 <= lf <= m, iters >= 1 (n=%d m=%d lf=%d iters=%d)",
                    n, m, lf, iters);
    const int lg = m - lf + 1;
    if (k < 1 || k > lg) return fail(HRIR_EINVAL, "hrir_factorize: need 1 <= k <= lg = %d (k=%d)", lg, k);
    if (!(lambda0 >= 0.0) || !std::isfinite(lambda0))
        return fail(HRIR_EINVAL, "hrir_factorize: lambda0 must be finite and >= 0");
    if (flags & ~(HRIR_REFIT_NNLS | HRIR_FACTORIZE_DEVICE))
        return fail(HRIR_EINVAL, "hrir_factorize: unknown flags 0x%x", flags);
    for (int64_t i = 0; i < (int64_t)n * m; ++i)
        if (!std::isfinite(X[i])) return fail(HRIR_EINVAL, "hrir_factorize: X[%lld] is not finite", (long long)i);

    const hrir::Problem pr{X, n, m, lf, lg};
    const size_t ng = (size_t)n * lg;
    std::vector<double> G(ng), Gn(ng), part, f(lf);
    try {
        if (g0) {
            for (size_t i = 0; i < ng; ++i) {
                if (!(g0[i] > 0.0) || !std::isfinite(g0[i]))
                    return fail(HRIR_EINVAL, "hrir_factorize: g0 entries must be finite and > 0");
                G[i] = g0[i];
            }
        } else {
            uint64_t st = seed;
            for (size_t i = 0; i < ng; ++i)
                G[i] = (double)((hrir::splitmix_next(st) >> 11) + 1) * 0x1.0p-53;
        }
    } catch (...) {
        return fail(HRIR_ENOMEM, "hrir_factorize: out of host memory");
    }

    std::vector<double> rowe(n);
    if (flags & HRIR_FACTORIZE_DEVICE) {
        const int rc = hrir::factorize_iterate_device(X, n, m, lf, iters, lambda0, G.data(), f.data(), cost_out);
        if (rc) return rc;
    }
    for (int t = 0; t < iters && !(flags & HRIR_FACTORIZE_DEVICE); ++t) {
        int rc = hrir::resonance_step(pr, G.data(), f.data(), part);
        if (rc) return rc;
        double nrm = 0.0;
        for (int q = 0; q < lf; ++q) nrm += f[q] * f[q];
        nrm = std::sqrt(nrm);
        if (!(nrm > 0.0)) return fail(HRIR_ENOTPD, "hrir_factorize: resonance filter vanished");
        for (int q = 0; q < lf; ++q) f[q] /= nrm;
        for (size_t i = 0; i < ng; ++i) G[i] *= nrm;
        hrir::reflection_step(pr, f.data(), G.data(), Gn.data(), hrir::l1_weight(lambda0, t, iters));
        G.swap(Gn);
        if (cost_out) {
            hrir::parallel_for(n, [&](int64_t i) {
                rowe[i] = hrir::residual_energy_row(X + (size_t)i * m, m, f.data(), lf, G.data() + (size_t)i * lg, lg);
            });
            double c = 0.0;
            for (int i = 0; i < n; ++i) c += rowe[i];
            cost_out[t] = c;
        }
    }
    for (int q = 0; q < lf; ++q) f_out[q] = f[q];
    if (gdense_out) std::memcpy(gdense_out, G.data(), ng * sizeof(double));

    // Top-K support per row, then (optionally) the non-negative refit.
    std::vector<double> ac(lf);
    hrir::autocorr(f.data(), lf, ac.data());
    std::vector<int> status(n, HRIR_OK);
    std::vector<double> gk((size_t)n * k, 0.0);
    std::vector<int> pk((size_t)n * k, 0), nz(n, 0);
    hrir::parallel_for(n, [&](int64_t i) {
        const double* g = G.data() + (size_t)i * lg;
        std::vector<int> cand;
        for (int j = 0; j < lg; ++j)
            if (g[j] > 0.0) cand.push_back(j);
        const int keep = std::min<int>(k, (int)cand.size());
        std::partial_sort(cand.begin(), cand.begin() + keep, cand.end(), [g](int a, int b) {
            return g[a] > g[b] || (g[a] == g[b] && a < b);
        });
        std::sort(cand.begin(), cand.begin() + keep);
        nz[i] = keep;
        for (int a = 0; a < keep; ++a) {
            pk[(size_t)i * k + a] = cand[a];
            gk[(size_t)i * k + a] = g[cand[a]];
        }
        if ((flags & HRIR_REFIT_NNLS) && keep > 0) {
            const double* x = X + (size_t)i * m;
            std::vector<double> H((size_t)keep * keep), c(keep), y(keep);
            for (int a = 0; a < keep; ++a) {
                for (int b = 0; b < keep; ++b) {
                    const int d = std::abs(cand[a] - cand[b]);
                    H[(size_t)a * keep + b] = d < lf ? ac[d] : 0.0;
                }
                double s = 0.0;
                for (int q = 0; q < lf; ++q) s += x[cand[a] + q] * f[q];
                c[a] = s;
            }
            status[i] = hrir::nnls_normal(H, c, keep, y.data());
            for (int a = 0; a < keep; ++a) gk[(size_t)i * k + a] = y[a];
        }
    });
    for (int i = 0; i < n; ++i)
        if (status[i]) return fail(status[i], "hrir_factorize: NNLS refit failed on row %d", i);
    for (size_t i = 0; i < (size_t)n * k; ++i) {
        p_out[i] = pk[i];
        g_out[i] = (float)gk[i];
    }
    if (nnz_out)
        for (int i = 0; i < n; ++i) nnz_out[i] = nz[i];
    if (err_db_out) {
        hrir::parallel_for(n, [&](int64_t i) {
            std::vector<double> gd(lg, 0.0);
            for (int a = 0; a < k; ++a) gd[pk[(size_t)i * k + a]] += gk[(size_t)i * k + a];
            const double* x = X + (size_t)i * m;
            const double e = hrir::residual_energy_row(x, m, f.data(), lf, gd.data(), lg);
            double ex = 0.0;
            for (int t = 0; t < m; ++t) ex += x[t] * x[t];
            err_db_out[i] = (ex > 0.0 && e > 0.0) ? 10.0 * std::log10(e / ex) : (e > 0.0 ? INFINITY : -INFINITY);
        });
    }
    return HRIR_OK;
}
