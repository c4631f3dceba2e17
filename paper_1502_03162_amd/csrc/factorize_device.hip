// Alg. 1 (Sec. III-C) on the GPU in FP64: the iterations of the
// Toeplitz-constrained semi-NMF that hrir_factorize runs on the host, for
// HRIR sets where host time matters.  Same arithmetic as the host code in
// factorize.cpp (per-row partial sums, a left-looking Cholesky, the
// multiplicative update of Eq. (4) with the L1 weight of Eq. (14)); the row
// sums run over a few blocks of consecutive rows, each in row order, then the
// blocks in order, and this file is compiled without contracting
// multiply-adds, so the two paths agree to rounding (the tests hold them to
// 1e-12) and every run gives the same bits.  Every matrix of the paper is banded Toeplitz and never built:
//   resonance system (Eqs. (10)-(11) on the lf unknowns of Eq. (13)):
//     A[q][q'] = a[|q - q'|], a[d] = sum_i sum_j G_ij G_i,j+d,
//     b[q] = sum_i sum_j G_ij X_i,j+q;
//   reflection update: (X^T F)_ij = sum_q X_i,j+q f_q and
//     (G Q+-)_ij = sum_l G_il Q+-[|l - j|] with Q = autocorrelation of f.
// Per iteration: one wave per row forms that row's a and b; one workgroup
// adds the rows, solves for f, normalises it (the scale moves into G) and
// forms Q+ and Q-; one thread per entry of G applies the update.
#include <hip/hip_runtime.h>

#include <cmath>
#include <vector>

#include "hrir_internal.h"

namespace hrir {
namespace {

constexpr int kLfMax = 64;          // resonance lengths the device path serves
constexpr int kSolveThreads = 256;

// part[i][d] = sum_{j + d < lg} g_ij g_i,j+d (d < lf), part[i][lf + q] = sum_j g_ij x_i,j+q.
// The row's g and x are staged in LDS (lg + m doubles, sized by the launch).
__global__ __launch_bounds__(64) void k_res_rows(const double* __restrict__ X, const double* __restrict__ G, int m,
                                                 int lf, int lg, double* __restrict__ part) {
    extern __shared__ double row[];
    const int i = blockIdx.x;
    double* g = row;
    double* x = row + lg;
    for (int j = threadIdx.x; j < lg; j += 64) g[j] = G[(int64_t)i * lg + j];
    for (int j = threadIdx.x; j < m; j += 64) x[j] = X[(int64_t)i * m + j];
    __syncthreads();
    double* out = part + (int64_t)i * 2 * lf;
    for (int u = threadIdx.x; u < 2 * lf; u += 64) {
        double s = 0.0;
        if (u < lf) {
            for (int j = 0; j + u < lg; ++j) s += g[j] * g[j + u];
        } else {
            const int q = u - lf;
            for (int j = 0; j < lg; ++j) s += g[j] * x[j + q];
        }
        out[u] = s;
    }
}

// Adds the rows' partial sums in row order, solves A f = b (Cholesky), sets
// nrm = ||f||, f /= nrm, and Q+-[d] from the autocorrelation of f.
// state[0] = nrm; status[0] != 0 if A was not positive definite or f vanished.
__global__ __launch_bounds__(kSolveThreads) void k_res_solve(const double* __restrict__ part, int n, int lf,
                                                             double* __restrict__ f, double* __restrict__ qp,
                                                             double* __restrict__ qm, double* __restrict__ state,
                                                             int* __restrict__ status) {
    __shared__ double ab[2 * kLfMax];
    __shared__ double blk[kSolveThreads];
    __shared__ double L[kLfMax][kLfMax];
    __shared__ double rhs[kLfMax];
    __shared__ int bad;
    const int tid = threadIdx.x;
    if (tid == 0) bad = 0;
    // column u of the row partials: nb blocks of consecutive rows, each summed
    // in row order by one thread (sixteen loads issued before their adds),
    // then the blocks added in order
    const int cols = 2 * lf, nb = kSolveThreads / cols;
    const int per = (n + nb - 1) / nb;
    if (tid < cols * nb) {
        const int u = tid % cols, b = tid / cols;
        const int i0 = b * per, i1 = min(n, i0 + per);
        double s = 0.0;
        int i = i0;
        for (; i + 16 <= i1; i += 16) {
            double v[16];
#pragma unroll
            for (int w = 0; w < 16; ++w) v[w] = part[(int64_t)(i + w) * cols + u];
#pragma unroll
            for (int w = 0; w < 16; ++w) s += v[w];
        }
        for (; i < i1; ++i) s += part[(int64_t)i * cols + u];
        blk[tid] = s;
    }
    __syncthreads();
    if (tid < cols) {
        double s = blk[tid];
        for (int b = 1; b < nb; ++b) s += blk[b * cols + tid];
        ab[tid] = s;
    }
    __syncthreads();
    for (int e = tid; e < lf * lf; e += kSolveThreads) {
        const int r = e / lf, c = e % lf;
        L[r][c] = ab[r > c ? r - c : c - r];
    }
    if (tid < lf) rhs[tid] = ab[lf + tid];
    __syncthreads();
    // left-looking Cholesky, column by column (the host's order)
    for (int c = 0; c < lf; ++c) {
        if (tid == 0) {
            double d = L[c][c];
            for (int q = 0; q < c; ++q) d -= L[c][q] * L[c][q];
            if (!(d > 0.0) || !isfinite(d)) {
                bad = 1;
                d = 1.0;
            }
            L[c][c] = sqrt(d);
        }
        __syncthreads();
        for (int r = c + 1 + tid; r < lf; r += kSolveThreads) {
            double v = L[r][c];
            for (int q = 0; q < c; ++q) v -= L[r][q] * L[c][q];
            L[r][c] = v / L[c][c];
        }
        __syncthreads();
    }
    if (tid == 0) {
        for (int r = 0; r < lf; ++r) {
            double v = rhs[r];
            for (int q = 0; q < r; ++q) v -= L[r][q] * rhs[q];
            rhs[r] = v / L[r][r];
        }
        for (int r = lf - 1; r >= 0; --r) {
            double v = rhs[r];
            for (int q = r + 1; q < lf; ++q) v -= L[q][r] * rhs[q];
            rhs[r] = v / L[r][r];
        }
        double nrm = 0.0;
        for (int q = 0; q < lf; ++q) nrm += rhs[q] * rhs[q];
        nrm = sqrt(nrm);
        if (!(nrm > 0.0)) {
            bad = 1;
            nrm = 1.0;
        }
        for (int q = 0; q < lf; ++q) rhs[q] /= nrm;
        state[0] = nrm;
        if (bad) status[0] = 1;
    }
    __syncthreads();
    if (tid < lf) f[tid] = rhs[tid];
    if (tid < lf) {
        double s = 0.0;
        for (int q = 0; q + tid < lf; ++q) s += rhs[q] * rhs[q + tid];
        qp[tid] = 0.5 * (fabs(s) + s);
        qm[tid] = 0.5 * (fabs(s) - s);
    }
}

// Gn_ij from the scaled G (G nrm) by Eq. (4) with L1 weight lam.
__global__ __launch_bounds__(256) void k_refl(const double* __restrict__ X, const double* __restrict__ G,
                                              double* __restrict__ Gn, const double* __restrict__ f,
                                              const double* __restrict__ qp, const double* __restrict__ qm,
                                              const double* __restrict__ state, int n, int m, int lf, int lg,
                                              double half_lam) {
    const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e >= (int64_t)n * lg) return;
    const int i = (int)(e / lg), j = (int)(e % lg);
    const double nrm = state[0];
    const double* g = G + (int64_t)i * lg;
    const double* x = X + (int64_t)i * m;
    const double gj = g[j] * nrm;
    if (gj == 0.0) {
        Gn[e] = 0.0;
        return;
    }
    double xf = 0.0;
    for (int q = 0; q < lf; ++q) xf += x[j + q] * f[q];
    double up = 0.0, um = 0.0;
    const int l0 = j - lf + 1 > 0 ? j - lf + 1 : 0, l1 = j + lf - 1 < lg - 1 ? j + lf - 1 : lg - 1;
    for (int l = l0; l <= l1; ++l) {
        const int d = l > j ? l - j : j - l;
        const double gl = g[l] * nrm;
        up += gl * qp[d];
        um += gl * qm[d];
    }
    const double num = 0.5 * (fabs(xf) + xf) + um;
    const double den = 0.5 * (fabs(xf) - xf) + up + half_lam;
    Gn[e] = gj * sqrt(num / den);
}

// rowe[i] = ||x_i - f * g_i||^2 (Eq. (3), one row).
__global__ __launch_bounds__(64) void k_cost_rows(const double* __restrict__ X, const double* __restrict__ G,
                                                  const double* __restrict__ f, int m, int lf, int lg,
                                                  double* __restrict__ rowe) {
    __shared__ double red[64];
    const int i = blockIdx.x;
    const double* g = G + (int64_t)i * lg;
    const double* x = X + (int64_t)i * m;
    double e = 0.0;
    for (int t = threadIdx.x; t < m; t += 64) {
        double rec = 0.0;
        const int j0 = t - lf + 1 > 0 ? t - lf + 1 : 0, j1 = t < lg - 1 ? t : lg - 1;
        for (int jj = j0; jj <= j1; ++jj) rec += f[t - jj] * g[jj];
        const double d = x[t] - rec;
        e += d * d;
    }
    red[threadIdx.x] = e;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int u = 0; u < 64; ++u) s += red[u];
        rowe[i] = s;
    }
}

__global__ void k_cost_sum(const double* __restrict__ rowe, int n, double* __restrict__ cost_t) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        double c = 0.0;
        for (int i = 0; i < n; ++i) c += rowe[i];
        *cost_t = c;
    }
}

struct DevBuf {
    void* p = nullptr;
    ~DevBuf() { (void)hipFree(p); }
};

}  // namespace

int factorize_iterate_device(const double* X, int n, int m, int lf, int iters, double lambda0, double* G,
                             double* f, double* cost) {
    if (lf > kLfMax)
        return fail(HRIR_EINVAL, "hrir_factorize: the device path serves lf <= %d (lf=%d)", kLfMax, lf);
    const int lg = m - lf + 1;
    const size_t row_lds = sizeof(double) * (size_t)(lg + m);
    if (row_lds > 64 * 1024)
        return fail(HRIR_EINVAL, "hrir_factorize: the device path serves rows of at most %d taps", 64 * 1024 / 16);
    const size_t ng = (size_t)n * lg;
    DevBuf dX, dG, dGn, dpart, df, dq, dstate, dstatus, drowe, dcost;
    hipError_t e = hipMalloc(&dX.p, sizeof(double) * (size_t)n * m);
    if (e == hipSuccess) e = hipMalloc(&dG.p, sizeof(double) * ng);
    if (e == hipSuccess) e = hipMalloc(&dGn.p, sizeof(double) * ng);
    if (e == hipSuccess) e = hipMalloc(&dpart.p, sizeof(double) * (size_t)n * 2 * lf);
    if (e == hipSuccess) e = hipMalloc(&df.p, sizeof(double) * lf);
    if (e == hipSuccess) e = hipMalloc(&dq.p, sizeof(double) * 2 * lf);
    if (e == hipSuccess) e = hipMalloc(&dstate.p, sizeof(double));
    if (e == hipSuccess) e = hipMalloc(&dstatus.p, sizeof(int));
    if (e == hipSuccess && cost) e = hipMalloc(&drowe.p, sizeof(double) * n);
    if (e == hipSuccess && cost) e = hipMalloc(&dcost.p, sizeof(double) * iters);
    if (e != hipSuccess)
        return fail(e == hipErrorOutOfMemory ? HRIR_ENOMEM : HRIR_EDEVICE, "hrir_factorize: %s",
                    hipGetErrorString(e));
    hipStream_t st = nullptr;
    e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
    if (e != hipSuccess) return fail(HRIR_EDEVICE, "hrir_factorize: %s", hipGetErrorString(e));
    auto* X_d = static_cast<double*>(dX.p);
    auto* G_d = static_cast<double*>(dG.p);
    auto* Gn_d = static_cast<double*>(dGn.p);
    auto* part = static_cast<double*>(dpart.p);
    auto* f_d = static_cast<double*>(df.p);
    auto* qp = static_cast<double*>(dq.p);
    auto* qm = qp + lf;
    auto* state = static_cast<double*>(dstate.p);
    auto* status = static_cast<int*>(dstatus.p);
    e = hipMemcpyAsync(X_d, X, sizeof(double) * (size_t)n * m, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(G_d, G, sizeof(double) * ng, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemsetAsync(status, 0, sizeof(int), st);
    const unsigned refl_grid = (unsigned)((ng + 255) / 256);
    for (int t = 0; t < iters && e == hipSuccess; ++t) {
        hipLaunchKernelGGL(k_res_rows, dim3(n), dim3(64), row_lds, st, X_d, G_d, m, lf, lg, part);
        hipLaunchKernelGGL(k_res_solve, dim3(1), dim3(kSolveThreads), 0, st, part, n, lf, f_d, qp, qm, state,
                           status);
        hipLaunchKernelGGL(k_refl, dim3(refl_grid), dim3(256), 0, st, X_d, G_d, Gn_d, f_d, qp, qm, state, n, m,
                           lf, lg, 0.5 * l1_weight(lambda0, t, iters));
        std::swap(G_d, Gn_d);
        if (cost) {
            hipLaunchKernelGGL(k_cost_rows, dim3(n), dim3(64), 0, st, X_d, G_d, f_d, m, lf, lg,
                               static_cast<double*>(drowe.p));
            hipLaunchKernelGGL(k_cost_sum, dim3(1), dim3(64), 0, st, static_cast<const double*>(drowe.p), n,
                               static_cast<double*>(dcost.p) + t);
        }
        e = hipGetLastError();
    }
    int bad = 0;
    if (e == hipSuccess) e = hipMemcpyAsync(f, f_d, sizeof(double) * lf, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipMemcpyAsync(G, G_d, sizeof(double) * ng, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess && cost)
        e = hipMemcpyAsync(cost, dcost.p, sizeof(double) * iters, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipMemcpyAsync(&bad, status, sizeof(int), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    (void)hipStreamDestroy(st);
    if (e != hipSuccess) return fail(HRIR_EDEVICE, "hrir_factorize: %s", hipGetErrorString(e));
    if (bad) return fail(HRIR_ENOTPD, "hrir_factorize: resonance system not positive definite or f vanished");
    return HRIR_OK;
}

}  // namespace hrir
