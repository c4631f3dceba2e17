// The paper's sparsifier (Sec. III-D, Eq. (14)) on the GPU in FP64: many
// independent L1-NNLS problems
//     min 1/2 g^T H g - (c0 - lambda / 2)^T g  over g >= 0,
// each either at a given lambda or with lambda searched for a target NNZE,
// then the discard of entries at or below a threshold.  H = A^T A of the
// design A = D T(f) is shared by every problem of one residual transform and
// bandwidth; c0 = A^T D x is per problem.  The host (sparsify.cpp) forms H
// and c0, this file runs the solves, the host finishes (top-k, errors,
// spectral distortion).
//
// One 64-lane workgroup per problem at a time (a static stride over the
// problems), every step in the order of the host's active-set solver
// (Lawson-Hanson on the normal equations, a Cholesky solve of the passive
// block, the same lambda bisection): every element sees the same
// operations in the same order as on the host (the Cholesky is right-looking
// here, column after column, which applies an element's products in the
// order the host's left-looking sum does), reductions are exact (max, min,
// argmax with ties to the lower index), and this file is compiled without
// contracting multiply-adds, so device and host give the same bits.  Lanes
// share the independent work: gradient entries, the rows of each Cholesky
// column and of each substitution step, the updates of g.
#include <hip/hip_runtime.h>

#include <cmath>
#include <vector>

#include "hrir_internal.h"

namespace hrir {
namespace {

constexpr int kL1Lanes = 64;
constexpr int kL1LgMax = 256;
// Passive blocks up to kHsLds x kHsLds live in LDS, larger ones in the
// workgroup's global scratch.  The LDS of a problem is sized by its lg at
// launch (six FP64 vectors, two index vectors, this block): at lg = 169 a
// workgroup takes 18 KB, so 8 fit per CU (a 48 x 48 block and lg-256
// vectors took 33 KB: 4 per CU, one wave per SIMD).
constexpr int kHsLds = 32;

struct L1Work {
    double* y;        // current solution
    double* w;        // gradient c - H y
    double* z;        // passive-set solution
    double* c;        // c0 - lambda / 2
    double* rhs;      // passive right-hand side / solution
    int* passive;
    int* idx;         // passive indices, ascending
    double* hs_lds;   // kHsLds x kHsLds (LDS)
    double* hs_glb;   // lg x lg global scratch of this workgroup
};

// Exact wave reductions through LDS (one workgroup = one wave).
__device__ double red_max(double v, double* sh) {
    const int l = threadIdx.x;
    sh[l] = v;
    __syncthreads();
    for (int s = kL1Lanes / 2; s > 0; s >>= 1) {
        if (l < s) sh[l] = fmax(sh[l], sh[l + s]);
        __syncthreads();
    }
    const double r = sh[0];
    __syncthreads();
    return r;
}

// In-place Cholesky of the np x np block A (row-major, lower triangle) and
// the two triangular solves for rhs, with each element's operations in the
// order of spd_solve() in factorize.cpp: the right-looking update below
// subtracts an element's products over q = 0, 1, ... before its division,
// the forward solve over q = 0, 1, ..., the back solve over q = np-1, ....
// Returns 0 if A is not positive definite.
__device__ int chol_solve_wave(double* A, int np, double* rhs, int* shi) {
    const int l = threadIdx.x;
    for (int c = 0; c < np; ++c) {
        if (l == 0) {
            const double d = A[c * np + c];
            const int good = (d > 0.0) && isfinite(d);
            shi[2] = good;
            if (good) A[c * np + c] = sqrt(d);
        }
        __syncthreads();
        if (!shi[2]) return 0;
        const double lc = A[c * np + c];
        for (int rr = c + 1 + l; rr < np; rr += kL1Lanes) A[rr * np + c] = A[rr * np + c] / lc;
        __syncthreads();
        // trailing update of the rows below c: A[rr][cc] -= L[rr][c] L[cc][c], c < cc <= rr
        for (int rr = c + 1 + l; rr < np; rr += kL1Lanes) {
            const double lr = A[rr * np + c];
            for (int cc = c + 1; cc <= rr; ++cc) A[rr * np + cc] -= lr * A[cc * np + c];
        }
        __syncthreads();
    }
    for (int k = 0; k < np; ++k) {
        if (l == 0) rhs[k] = rhs[k] / A[k * np + k];
        __syncthreads();
        const double xk = rhs[k];
        for (int r = k + 1 + l; r < np; r += kL1Lanes) rhs[r] -= A[r * np + k] * xk;
        __syncthreads();
    }
    for (int k = np - 1; k >= 0; --k) {
        if (l == 0) rhs[k] = rhs[k] / A[k * np + k];
        __syncthreads();
        const double xk = rhs[k];
        for (int r = l; r < k; r += kL1Lanes) rhs[r] -= A[k * np + r] * xk;
        __syncthreads();
    }
    return 1;
}

// Lawson-Hanson active set on the normal equations; returns 0 or ENOTPD.
// Same steps as nnls_normal() in factorize.cpp, including its warm start
// (W.y kept, its entries > 0 the passive set, which is solved on first).
__device__ int nnls_wave(const double* __restrict__ H, int s, L1Work& W, double* sh, int* shi, bool warm) {
    const int l = threadIdx.x;
    double cm = 0.0;
    for (int j = l; j < s; j += kL1Lanes) cm = fmax(cm, fabs(W.c[j]));
    const double tol = 1e-12 * red_max(cm, sh);
    int on = 0;
    for (int j = l; j < s; j += kL1Lanes) {
        const bool keep = warm && W.y[j] > 0.0;
        W.passive[j] = keep ? 1 : 0;
        if (!keep) W.y[j] = 0.0;
        on |= keep ? 1 : 0;
    }
    bool solve_first = __any(on);
    if (l == 0) shi[1] = 0;
    __syncthreads();
    for (int outer = 0; outer < 3 * s + 10; ++outer) {
        if (!solve_first) {
            // w = c - H y, each entry's terms in increasing q; y is zero outside
            // the passive set (idx, from the last inner step) and a zero term
            // leaves the sum unchanged, so only passive columns are visited
            const int npv = shi[1];
            for (int j = l; j < s; j += kL1Lanes) {
                double v = W.c[j];
                const double* hr = H + (int64_t)j * s;
                for (int a = 0; a < npv; ++a) {
                    const int q = W.idx[a];
                    v -= hr[q] * W.y[q];
                }
                W.w[j] = v;
            }
            // the largest w among the non-passive entries above tol, ties to the
            // lower index: per lane over its entries in increasing j, then over
            // the lanes in index order
            int bj = -1;
            double bw = 0.0;
            for (int j = l; j < s; j += kL1Lanes)
                if (!W.passive[j] && W.w[j] > tol && (bj < 0 || W.w[j] > bw)) {
                    bj = j;
                    bw = W.w[j];
                }
            sh[l] = bw;
            shi[4 + l] = bj;
            __syncthreads();
            if (l == 0) {
                int best = -1;
                double wb = 0.0;
                for (int k = 0; k < kL1Lanes; ++k) {
                    const int j = shi[4 + k];
                    if (j >= 0 && (best < 0 || sh[k] > wb || (sh[k] == wb && j < best))) {
                        best = j;
                        wb = sh[k];
                    }
                }
                shi[0] = best;
                if (best >= 0) W.passive[best] = 1;
            }
            __syncthreads();
            if (shi[0] < 0) break;
        }
        solve_first = false;
        for (int inner = 0; inner <= s + 1; ++inner) {
            // passive indices in ascending order: a ballot per 64 entries
            int np = 0;
            for (int j0 = 0; j0 < s; j0 += kL1Lanes) {
                const int j = j0 + l;
                const bool on = j < s && W.passive[j];
                const unsigned long long mask = __ballot(on);
                if (on) W.idx[np + __popcll(mask & ((1ull << l) - 1ull))] = j;
                np += __popcll(mask);
            }
            if (l == 0) shi[1] = np;
            __syncthreads();
            double* A = np <= kHsLds ? W.hs_lds : W.hs_glb;
            for (int e = l; e < np * np; e += kL1Lanes) {
                const int a = e / np, b = e - a * np;
                A[e] = H[(int64_t)W.idx[a] * s + W.idx[b]];
            }
            for (int a = l; a < np; a += kL1Lanes) W.rhs[a] = W.c[W.idx[a]];
            __syncthreads();
            if (!chol_solve_wave(A, np, W.rhs, shi)) return HRIR_ENOTPD;
            int pos = 1;
            for (int a = l; a < np; a += kL1Lanes)
                if (!(W.rhs[a] > 0.0)) pos = 0;
            const bool all_pos = __all(pos);
            for (int j = l; j < s; j += kL1Lanes) W.z[j] = 0.0;
            __syncthreads();
            for (int a = l; a < np; a += kL1Lanes) W.z[W.idx[a]] = W.rhs[a];
            __syncthreads();
            if (all_pos) {
                for (int j = l; j < s; j += kL1Lanes) W.y[j] = W.z[j];
                __syncthreads();
                break;
            }
            // step length: the smallest y / (y - z) over passive entries with
            // z <= 0, and 1 (the host's running min from 1 skips nothing else)
            double am = 1.0;
            for (int a = l; a < np; a += kL1Lanes) {
                const int j = W.idx[a];
                if (!(W.z[j] > 0.0)) {
                    const double v = W.y[j] / (W.y[j] - W.z[j]);
                    if (v < am) am = v;
                }
            }
            sh[l] = am;
            __syncthreads();
            if (l == 0) {
                double alpha = 1.0;
                for (int k = 0; k < kL1Lanes; ++k)
                    if (sh[k] < alpha) alpha = sh[k];
                sh[kL1Lanes] = alpha;
            }
            __syncthreads();
            const double alpha = sh[kL1Lanes];
            double ym = 0.0;
            for (int j = l; j < s; j += kL1Lanes) {
                W.y[j] += alpha * (W.z[j] - W.y[j]);
                ym = fmax(ym, W.y[j]);
            }
            const double ymax = red_max(ym, sh);
            for (int j = l; j < s; j += kL1Lanes)
                if (W.passive[j] && !(W.y[j] > 1e-15 * ymax)) {
                    W.passive[j] = 0;
                    W.y[j] = 0.0;
                }
            __syncthreads();
        }
    }
    return HRIR_OK;
}

// One solve at lambda and the discard: g (lds or global, s entries), NNZE.
__device__ int solve_at(const double* __restrict__ H, const double* __restrict__ c0, int s, double lambda,
                        double thresh, double* g, L1Work& W, double* sh, int* shi, int* nnze, bool warm) {
    const int l = threadIdx.x;
    for (int j = l; j < s; j += kL1Lanes) W.c[j] = c0[j] - 0.5 * lambda;
    __syncthreads();
    const int rc = nnls_wave(H, s, W, sh, shi, warm);
    if (rc) return rc;
    int nz = 0;
    for (int j = l; j < s; j += kL1Lanes) {
        double v = W.y[j];
        if (fabs(v) <= thresh) v = 0.0;
        g[j] = v;
        nz += v != 0.0;
    }
    shi[4 + l] = nz;
    __syncthreads();
    if (l == 0) {
        int t = 0;
        for (int k = 0; k < kL1Lanes; ++k) t += shi[4 + k];
        shi[3] = t;
    }
    __syncthreads();
    *nnze = shi[3];
    __syncthreads();
    return HRIR_OK;
}

// LDS bytes of a problem of lg = s (the layout at the top of k_l1_solve).
size_t l1_lds_bytes(int s) {
    return sizeof(double) * ((size_t)6 * s + kHsLds * kHsLds + kL1Lanes + 1) +
           sizeof(int) * ((size_t)4 + kL1Lanes + 2 * (size_t)s);
}

// Problems p = blockIdx.x, blockIdx.x + gridDim.x, ...: problem p uses design
// H + design[p] * s * s and c0 + p * s; lambda[p] if lambda is given, else the
// search for at most `target` entries.  Outputs g[p][s], lambda_out[p],
// nnze[p], status[p].
__global__ __launch_bounds__(kL1Lanes) void k_l1_solve(const double* __restrict__ H, const double* __restrict__ c0,
                                                       const int* __restrict__ design, int n_prob, int s,
                                                       const double* __restrict__ lambda, int target, double thresh,
                                                       double* __restrict__ g_out, double* __restrict__ lambda_out,
                                                       int* __restrict__ nnze_out, int* __restrict__ status,
                                                       double* __restrict__ scratch) {
    // LDS (l1_lds_bytes): y, w, z, c, rhs, gt (s doubles each), the passive
    // block, the reduction buffers, then passive and idx (s ints each)
    extern __shared__ double smem[];
    double* sy = smem;
    double* sw = sy + s;
    double* sz = sw + s;
    double* sc = sz + s;
    double* srhs = sc + s;
    double* sgt = srhs + s;
    double* shs = sgt + s;
    double* sh = shs + kHsLds * kHsLds;
    int* shi = reinterpret_cast<int*>(sh + kL1Lanes + 1);
    int* spas = shi + 4 + kL1Lanes;
    int* sidx = spas + s;
    L1Work W{sy, sw, sz, sc, srhs, spas, sidx, shs, scratch + (int64_t)blockIdx.x * s * s};
    const int l = threadIdx.x;
    for (int p = blockIdx.x; p < n_prob; p += gridDim.x) {
        const double* Hp = H + (int64_t)design[p] * s * s;
        const double* cp = c0 + (int64_t)p * s;
        double* g = g_out + (int64_t)p * s;
        int nz = 0, rc = HRIR_OK;
        double lam = 0.0;
        if (lambda) {
            lam = lambda[p];
            rc = solve_at(Hp, cp, s, lam, thresh, g, W, sh, shi, &nz, false);
        } else {
            // lambda = 0 first; else geometric bisection on [1e-12, 1] * 2 max(c0),
            // each step starting from the previous step's minimiser (W.y)
            rc = solve_at(Hp, cp, s, 0.0, thresh, g, W, sh, shi, &nz, false);
            if (rc == HRIR_OK && nz > target) {
                double cm = 0.0;
                for (int j = l; j < s; j += kL1Lanes) cm = fmax(cm, cp[j]);
                double hi = 2.0 * red_max(cm, sh), lo = hi * 1e-12;
                for (int j = l; j < s; j += kL1Lanes) g[j] = 0.0;
                int nz_hi = 0;
                for (int it = 0; it < 50 && rc == HRIR_OK; ++it) {
                    const double mid = sqrt(lo * hi);
                    int nzm = 0;
                    rc = solve_at(Hp, cp, s, mid, thresh, sgt, W, sh, shi, &nzm, true);
                    if (rc) break;
                    if (nzm <= target) {
                        hi = mid;
                        nz_hi = nzm;
                        for (int j = l; j < s; j += kL1Lanes) g[j] = sgt[j];
                    } else {
                        lo = mid;
                    }
                    __syncthreads();
                }
                lam = hi;
                nz = nz_hi;
            }
        }
        if (l == 0) {
            status[p] = rc;
            lambda_out[p] = lam;
            nnze_out[p] = nz;
        }
        __syncthreads();
    }
}

}  // namespace

int l1_solve_device(const double* H, int n_designs, int s, const double* c0, const int* design, int n_prob,
                    const double* lambda, int target, double thresh, double* g_out, double* lambda_out,
                    int* nnze_out) {
    if (n_prob <= 0) return HRIR_OK;
    if (s < 1 || s > kL1LgMax) return fail(HRIR_EINVAL, "device L1-NNLS: lg=%d outside [1, %d]", s, kL1LgMax);
    int dev = 0, cus = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    const size_t lds = l1_lds_bytes(s);
    int per_cu = 0;
    if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_l1_solve, kL1Lanes, lds);
    const int grid = std::max(1, std::min(n_prob, std::max(per_cu, 1) * std::max(cus, 1)));
    double *dH = nullptr, *dc = nullptr, *dlam = nullptr, *dg = nullptr, *dlo = nullptr, *dws = nullptr;
    int *dd = nullptr, *dnz = nullptr, *dst = nullptr;
    const size_t ss = (size_t)s * s;
    if (e == hipSuccess) e = hipMalloc(&dH, sizeof(double) * ss * n_designs);
    if (e == hipSuccess) e = hipMalloc(&dc, sizeof(double) * (size_t)s * n_prob);
    if (e == hipSuccess) e = hipMalloc(&dd, sizeof(int) * n_prob);
    if (e == hipSuccess && lambda) e = hipMalloc(&dlam, sizeof(double) * n_prob);
    if (e == hipSuccess) e = hipMalloc(&dg, sizeof(double) * (size_t)s * n_prob);
    if (e == hipSuccess) e = hipMalloc(&dlo, sizeof(double) * n_prob);
    if (e == hipSuccess) e = hipMalloc(&dnz, sizeof(int) * n_prob);
    if (e == hipSuccess) e = hipMalloc(&dst, sizeof(int) * n_prob);
    if (e == hipSuccess) e = hipMalloc(&dws, sizeof(double) * ss * grid);
    if (e == hipSuccess) e = hipMemcpy(dH, H, sizeof(double) * ss * n_designs, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(dc, c0, sizeof(double) * (size_t)s * n_prob, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(dd, design, sizeof(int) * n_prob, hipMemcpyHostToDevice);
    if (e == hipSuccess && lambda) e = hipMemcpy(dlam, lambda, sizeof(double) * n_prob, hipMemcpyHostToDevice);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_l1_solve, dim3(grid), dim3(kL1Lanes), lds, nullptr, dH, dc, dd, n_prob, s, dlam, target,
                           thresh, dg, dlo, dnz, dst, dws);
        e = hipGetLastError();
    }
    std::vector<int> st(n_prob, 0);
    if (e == hipSuccess) e = hipMemcpy(g_out, dg, sizeof(double) * (size_t)s * n_prob, hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(lambda_out, dlo, sizeof(double) * n_prob, hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(nnze_out, dnz, sizeof(int) * n_prob, hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(st.data(), dst, sizeof(int) * n_prob, hipMemcpyDeviceToHost);
    for (void* ptr : {(void*)dH, (void*)dc, (void*)dd, (void*)dlam, (void*)dg, (void*)dlo, (void*)dnz, (void*)dst,
                      (void*)dws})
        (void)hipFree(ptr);
    if (e != hipSuccess)
        return fail(e == hipErrorOutOfMemory ? HRIR_ENOMEM : HRIR_EDEVICE, "device L1-NNLS: %s", hipGetErrorString(e));
    for (int p = 0; p < n_prob; ++p)
        if (st[p]) return fail(st[p], "device L1-NNLS: support columns are linearly dependent (problem %d)", p);
    return HRIR_OK;
}

}  // namespace hrir
