// Internal declarations shared by the host and device translation units of
// libhrir.so (error reporting, plan layout, a small thread pool helper).
#pragma once

#include <cstdint>
#include <cstdio>
#include <string>
#include <thread>
#include <vector>
#include <algorithm>

#include "hrir.h"

namespace hrir {

// Sets the thread-local last-error message and returns `code`.
int fail(int code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
void clear_error();
const char* last_error();

// In-place Cholesky solve of the s x s SPD system H y = rhs (rhs overwritten
// with y).  Returns false if H is not positive definite.
bool spd_solve(std::vector<double>& H, int s, double* rhs);
// L1 weight of the reflection update at iteration t of T (hrir_factorize).
double l1_weight(double lambda0, int t, int T);
// The iterations of Alg. 1 on the current GPU in FP64 (factorize_device.hip):
// G (host, n x (m - lf + 1)) in and out, f (host, lf) out with unit norm,
// cost (host, iters, or null) as in hrir_factorize.  Same arithmetic and order
// as the host iterations.
int factorize_iterate_device(const double* X, int n, int m, int lf, int iters, double lambda0, double* G,
                             double* f, double* cost);

// The L1-NNLS solves of the sparsifier on the current GPU (l1_device.hip):
// problem p minimises 1/2 g^T H_d g - (c0_p - lambda_p / 2)^T g over g >= 0
// with H_d = H + design[p] * s * s (host f64[n_designs][s][s]) and c0_p = c0
// + p * s (host), at lambda[p] (host, or null: the sparsifier's lambda search
// for at most `target` entries), then discards entries <= thresh.  Outputs
// (host): g_out f64[n_prob][s], lambda_out f64[n_prob], nnze_out i32[n_prob].
// Same steps as the host's solve (nnls_normal, the bisection).  Status code
// as in hrir.h; s <= 256.
int l1_solve_device(const double* H, int n_designs, int s, const double* c0, const int* design, int n_prob,
                    const double* lambda, int target, double thresh, double* g_out, double* lambda_out,
                    int* nnze_out);

// Lawson-Hanson active-set solution of min 1/2 y^T H y - c^T y over y >= 0,
// H the s x s normal matrix.  Status code as in hrir.h.
// warm: start from y (entries > 0 form the passive set) instead of zero;
// the result is the same minimiser, reached in fewer steps from a nearby one.
int nnls_normal(const std::vector<double>& H, const std::vector<double>& c, int s, double* y, bool warm = false);

// Runs body(i) for i in [0, n) on up to hardware_concurrency threads with
// static contiguous chunks.  Results must not depend on the thread count:
// callers write disjoint outputs and reduce sequentially afterwards.
template <class F>
void parallel_for(int64_t n, F&& body) {
    unsigned hw = std::thread::hardware_concurrency();
    int64_t nt = std::min<int64_t>(hw ? hw : 1, 32);
    if (n < 64 || nt <= 1) {
        for (int64_t i = 0; i < n; ++i) body(i);
        return;
    }
    nt = std::min<int64_t>(nt, n);
    std::vector<std::thread> th;
    th.reserve(nt);
    for (int64_t t = 0; t < nt; ++t) {
        const int64_t b = n * t / nt, e = n * (t + 1) / nt;
        th.emplace_back([b, e, &body] {
            for (int64_t i = b; i < e; ++i) body(i);
        });
    }
    for (auto& x : th) x.join();
}

}  // namespace hrir
