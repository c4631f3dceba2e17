// Sparse-HRIR rendering on gfx950 (CDNA4, wave64).
//
// The method renders a source s through the HRIR of one direction and ear as
// (s * f) * g (Eq. (2)): z = f * s is direction independent and is formed
// once per source; each (direction, ear) is then a K-tap gather
//     out[t] = sum_k g_k z[t - p_k],   t in [0, len(s) + lf + lg - 2),
// whose cost is proportional to the number of kept taps (Sec. IV-F).
//
// Work unit ("tile"): one source, TB consecutive output samples, and a group
// of that source's jobs.  A 256-thread workgroup
//   1. stages s[t0 - (lg-1) - (lf-1), t0 + TB) in LDS (zero outside the
//      signal),
//   2. forms z[t0 - (lg-1), t0 + TB) in LDS with the resonance FIR (each
//      thread keeps an 8-output sliding window of s in registers; the filter
//      taps are wave-uniform and live in scalar registers),
//   3. renders every job of the group from that z tile: each wave takes
//      (job, 1024-sample chunk) pairs; a job's taps are wave-uniform scalar
//      loads; lane l accumulates 16 outputs t = c0 + l + 64 j in registers
//      over the K taps (z read from LDS), then stores them coalesced.
// z never goes to HBM, and each z tile is shared by all directions and ears
// of its source: the HBM traffic is one read of s plus one write per output.
//
// Summation order per output is fixed (FIR taps 0..lf-1, then kept taps
// 0..K-1, each a single fma into one accumulator), so every launch shape and
// batching of the same job gives bitwise identical results.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <mutex>

#include "hrir_internal.h"
#include "render_common.h"
#include "render_quad.h"

namespace hrir {

// ---------------------------------------------------------------------------
// Tile body: stage s, resonance FIR into LDS, sparse gather from LDS.
// ---------------------------------------------------------------------------
template <int LFP, int KP>
__device__ __forceinline__ void render_tile(const TileDesc& td, const float* __restrict__ src,
                                            const JobDesc* __restrict__ jobs,
                                            const float* __restrict__ r, const int* __restrict__ P,
                                            const float* __restrict__ Gv, float* __restrict__ out,
                                            int lg, int TB, float* s_win, float* z_win) {
    const int tid = threadIdx.x;
    const int H = lg - 1;
    stage_z<LFP>(td, src, r, H, TB, s_win, z_win);

    // 3. gather: (job, chunk) pairs round-robin over the waves
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
    const int tile_len = min(TB, td.out_len - td.t0);
    const int nchunk = (tile_len + kChunk - 1) / kChunk;
    const int npairs = td.job_count * nchunk;
    for (int pi = wave; pi < npairs; pi += kWaves) {
        const int q = pi / nchunk;
        const int c = pi - q * nchunk;
        const JobDesc jd = jobs[td.job_begin + q];
        const int* pp = P + (int64_t)jd.filt * KP;
        const float* gg = Gv + (int64_t)jd.filt * KP;
        int pk[KP];
        float gk[KP];
#pragma unroll
        for (int k = 0; k < KP; ++k) { pk[k] = pp[k]; gk[k] = gg[k]; }
        float acc[kR];
#pragma unroll
        for (int j = 0; j < kR; ++j) acc[j] = 0.0f;
        const float* zl = z_win + (c * kChunk + lane + H);
        // Two-stage pipeline: the LDS reads of tap k+1 are in flight while the
        // fmas of tap k run.  pin() materialises the accumulators and is a
        // compiler memory barrier, so no tap's reads are hoisted further and
        // no fmas are deferred (either would exhaust the VGPRs).
        float zv[2][kR];
#pragma unroll
        for (int j = 0; j < kR; ++j) zv[0][j] = zl[64 * j - pk[0]];
#pragma unroll
        for (int k = 0; k < KP; ++k) {
            if (k + 1 < KP) {
#pragma unroll
                for (int j = 0; j < kR; ++j) zv[(k + 1) & 1][j] = zl[64 * j - pk[k + 1]];
            }
#pragma unroll
            for (int j = 0; j < kR; ++j) acc[j] = fmaf(gk[k], zv[k & 1][j], acc[j]);
            pin16(acc);
        }
        float* o = out + jd.out_off + td.t0 + c * kChunk + lane;
        const int lim = tile_len - c * kChunk - lane;
#pragma unroll
        for (int j = 0; j < kR; ++j)
            if (64 * j < lim) o[64 * j] = acc[j];
    }
}

template <int LFP, int KP>
__global__ __launch_bounds__(kThreads, kMinWaves) void k_render_tiles(const float* __restrict__ src,
                                                           const TileDesc* __restrict__ tiles,
                                                           const JobDesc* __restrict__ jobs,
                                                           const float* __restrict__ r,
                                                           const int* __restrict__ P,
                                                           const float* __restrict__ Gv,
                                                           float* __restrict__ out, int lg, int TB) {
    extern __shared__ float4 smem4[];
    float* s_win = reinterpret_cast<float*>(smem4);
    float* z_win = s_win + lds_s_len(TB, lg, LFP);
    const TileDesc td = tiles[blockIdx.x];
    render_tile<LFP, KP>(td, src, jobs, r, P, Gv, out, lg, TB, s_win, z_win);
}

// Persistent variant: a fixed grid drains the tile list through a device
// counter.  ctr[0] hands out tiles, ctr[1] counts finished workgroups; the
// last workgroup to finish resets both, so the next launch (or graph replay)
// starts from zero without a memset.
template <int LFP, int KP>
__global__ __launch_bounds__(kThreads, kMinWaves) void k_render_persistent(const float* __restrict__ src,
                                                                const TileDesc* __restrict__ tiles,
                                                                int n_tiles,
                                                                const JobDesc* __restrict__ jobs,
                                                                const float* __restrict__ r,
                                                                const int* __restrict__ P,
                                                                const float* __restrict__ Gv,
                                                                float* __restrict__ out, int lg, int TB,
                                                                int* __restrict__ ctr) {
    extern __shared__ float4 smem4[];
    float* s_win = reinterpret_cast<float*>(smem4);
    float* z_win = s_win + lds_s_len(TB, lg, LFP);
    __shared__ int s_next;
    for (;;) {
        if (threadIdx.x == 0) s_next = atomicAdd(&ctr[0], 1);
        __syncthreads();
        const int t = s_next;
        __syncthreads();
        if (t >= n_tiles) break;
        const TileDesc td = tiles[t];
        render_tile<LFP, KP>(td, src, jobs, r, P, Gv, out, lg, TB, s_win, z_win);
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        __threadfence();
        const int done = atomicAdd(&ctr[1], 1);
        if (done == (int)gridDim.x - 1) {
            atomicExch(&ctr[0], 0);
            atomicExch(&ctr[1], 0);
        }
    }
}

// ---------------------------------------------------------------------------
// Unfused reference path: z to HBM, then a gather that reads it from HBM.
// ---------------------------------------------------------------------------
constexpr int kZChunk = 4096;

template <int LFP>
__global__ __launch_bounds__(kThreads) void k_resonance(const float* __restrict__ src,
                                                        const ZDesc* __restrict__ zd,
                                                        const float* __restrict__ r, int lf,
                                                        float* __restrict__ zbuf) {
    const ZDesc d = zd[blockIdx.x];
    const int nz = d.src_len + lf - 1;
    const float* sp = src + d.src_off;
    for (int v = d.v0 + threadIdx.x; v < min(d.v0 + kZChunk, nz); v += kThreads) {
        float acc = 0.0f;
#pragma unroll
        for (int n = 0; n < LFP; ++n) {
            const int q = v - n;
            const float sv = (q >= 0 && q < d.src_len) ? sp[q] : 0.0f;
            acc = fmaf(r[n], sv, acc);
        }
        zbuf[d.z_off + v] = acc;
    }
}

template <int KP>
__global__ __launch_bounds__(kThreads) void k_gather(const GDesc* __restrict__ gd,
                                                     const float* __restrict__ zbuf,
                                                     const int* __restrict__ P,
                                                     const float* __restrict__ Gv,
                                                     float* __restrict__ out) {
    const GDesc d = gd[blockIdx.x];
    const int* pp = P + (int64_t)d.filt * KP;
    const float* gg = Gv + (int64_t)d.filt * KP;
    const float* z = zbuf + d.z_off;
    for (int t = d.t0 + threadIdx.x; t < min(d.t0 + kZChunk, d.out_len); t += kThreads) {
        float acc = 0.0f;
#pragma unroll
        for (int k = 0; k < KP; ++k) {
            const int u = t - pp[k];
            const float zv = (u >= 0 && u < d.nz) ? z[u] : 0.0f;
            acc = fmaf(gg[k], zv, acc);
        }
        out[d.out_off + t] = acc;
    }
}

}  // namespace hrir

// ===========================================================================
// Host side: plans, batches, launches.
// ===========================================================================
using namespace hrir;

struct hrir_plan {
    int lf, lfp, k, kp, lg, n_filters, device;
    int n_res = 1;            // resonance filters (regions)
    std::vector<int> res;     // region of each filter (empty when n_res == 1)
    float* d_r = nullptr;   // [n_res][lfp], zero padded
    int* d_p = nullptr;     // [n_filters][kp], padded with (0, 0)
    float* d_g = nullptr;
    uint64_t rows_gen = 1;    // bumped by every rewrite of tap rows (spconv_plan_topk)
};

struct hrir_batch {
    const hrir_plan* plan = nullptr;
    int flags = 0, TB = 0, group = 0, grid = 0;
    int kind = 0;                             // KIND_* below
    int nt = 512;                             // threads per workgroup of the quad kernel
    bool direct = false;                      // quad kernel: every tile takes the direct stage
    int64_t n_tiles = 0, n_jobs = 0;
    int64_t src_extent = 0, out_extent = 0;   // elements the job list touches
    size_t lds_bytes = 0;
    TileDesc* d_tiles = nullptr;
    JobDesc* d_jobs = nullptr;
    int* d_ctr = nullptr;
    // unfused
    ZDesc* d_z = nullptr;
    GDesc* d_gd = nullptr;
    float* d_zbuf = nullptr;
    int64_t n_z = 0, n_gd = 0;
    // graph
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipStream_t cap_stream = nullptr;
    const float* g_src = nullptr;
    float* g_out = nullptr;
};

namespace {

enum { KIND_QUAD = 0, KIND_REGWIN = 1, KIND_LDS_GATHER = 2, KIND_UNFUSED = 3 };

#define HIP_TRY(expr)                                                                         \
    do {                                                                                      \
        hipError_t e_ = (expr);                                                               \
        if (e_ != hipSuccess)                                                                 \
            return fail(e_ == hipErrorOutOfMemory ? HRIR_ENOMEM : HRIR_EDEVICE, "%s: %s", #expr, \
                        hipGetErrorString(e_));                                               \
    } while (0)

int pad_lf(int lf) { return lf <= 16 ? 16 : (lf <= 32 ? 32 : 64); }
int pad_k(int k) { return k <= 4 ? 4 : k <= 8 ? 8 : k <= 16 ? 16 : k <= 32 ? 32 : 64; }

template <int LFP, int KP>
void* tiles_kernel_ptr() { return reinterpret_cast<void*>(&k_render_tiles<LFP, KP>); }

// Launch dispatch over the padded (lf, K) instantiations.
template <class F>
int dispatch(int lfp, int kp, F&& f) {
#define HRIR_CASE(L, K) \
    if (lfp == L && kp == K) return f(std::integral_constant<int, L>{}, std::integral_constant<int, K>{});
    HRIR_CASE(16, 4) HRIR_CASE(16, 8) HRIR_CASE(16, 16) HRIR_CASE(16, 32) HRIR_CASE(16, 64)
    HRIR_CASE(32, 4) HRIR_CASE(32, 8) HRIR_CASE(32, 16) HRIR_CASE(32, 32) HRIR_CASE(32, 64)
    HRIR_CASE(64, 4) HRIR_CASE(64, 8) HRIR_CASE(64, 16) HRIR_CASE(64, 32) HRIR_CASE(64, 64)
#undef HRIR_CASE
    return fail(HRIR_EINVAL, "no kernel for lf pad %d, k pad %d", lfp, kp);
}

void free_batch(hrir_batch* b) {
    if (!b) return;
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
    (void)hipFree(b->d_tiles);
    (void)hipFree(b->d_jobs);
    (void)hipFree(b->d_ctr);
    (void)hipFree(b->d_z);
    (void)hipFree(b->d_gd);
    (void)hipFree(b->d_zbuf);
    delete b;
}

int launch(hrir_batch* b, const float* d_src, float* d_out, hipStream_t st) {
    const hrir_plan* pl = b->plan;
    if (b->n_jobs == 0) return HRIR_OK;
    if (b->flags & SPCONV_UNFUSED) {
        int rc = dispatch(pl->lfp, pl->kp, [&](auto L, auto K) -> int {
            hipLaunchKernelGGL((k_resonance<decltype(L)::value>), dim3((unsigned)b->n_z), dim3(kThreads), 0, st,
                               d_src, b->d_z, pl->d_r, pl->lf, b->d_zbuf);
            hipLaunchKernelGGL((k_gather<decltype(K)::value>), dim3((unsigned)b->n_gd), dim3(kThreads), 0, st,
                               b->d_gd, b->d_zbuf, pl->d_p, pl->d_g, d_out);
            return HRIR_OK;
        });
        if (rc) return rc;
    } else if (b->kind == KIND_QUAD) {
        int rc = quad_launch(pl->lfp, pl->kp, b->nt, (b->flags & SPCONV_PERSISTENT) != 0, b->direct, b->grid,
                             b->lds_bytes, st, d_src, b->d_tiles, (int)b->n_tiles, b->d_jobs, pl->d_r, pl->d_p,
                             pl->d_g, d_out, pl->lg, b->TB, b->d_ctr);
        if (rc) return rc;
    } else if (b->kind == KIND_REGWIN) {
        int rc = rw_launch(pl->lfp, (b->flags & SPCONV_PERSISTENT) != 0, b->grid, b->lds_bytes, st, d_src, b->d_tiles,
                           (int)b->n_tiles, b->d_jobs, pl->d_r, pl->d_p, pl->d_g, d_out, pl->kp, pl->k, b->TB,
                           b->d_ctr);
        if (rc) return rc;
    } else if (b->flags & SPCONV_PERSISTENT) {
        int rc = dispatch(pl->lfp, pl->kp, [&](auto L, auto K) -> int {
            hipLaunchKernelGGL((k_render_persistent<decltype(L)::value, decltype(K)::value>), dim3(b->grid),
                               dim3(kThreads), b->lds_bytes, st, d_src, b->d_tiles, (int)b->n_tiles, b->d_jobs,
                               pl->d_r, pl->d_p, pl->d_g, d_out, pl->lg, b->TB, b->d_ctr);
            return HRIR_OK;
        });
        if (rc) return rc;
    } else {
        int rc = dispatch(pl->lfp, pl->kp, [&](auto L, auto K) -> int {
            hipLaunchKernelGGL((k_render_tiles<decltype(L)::value, decltype(K)::value>), dim3((unsigned)b->n_tiles),
                               dim3(kThreads), b->lds_bytes, st, d_src, b->d_tiles, b->d_jobs, pl->d_r, pl->d_p,
                               pl->d_g, d_out, pl->lg, b->TB);
            return HRIR_OK;
        });
        if (rc) return rc;
    }
    HIP_TRY(hipGetLastError());
    return HRIR_OK;
}

}  // namespace

extern "C" int spconv_plan_multi(const float* r, int32_t n_res, int32_t lf, const int32_t* res, const int32_t* p,
                                 const float* g, int32_t n_filters, int32_t k, int32_t lg, hrir_plan** out) {
    clear_error();
    if (!r || !p || !g || !out || (n_res > 1 && !res)) return fail(HRIR_EINVAL, "spconv_plan: null pointer");
    *out = nullptr;
    if (n_res < 1 || n_res > 64) return fail(HRIR_EINVAL, "spconv_plan: n_res=%d outside [1, 64]", n_res);
    if (lf < 1 || lf > 64) return fail(HRIR_EINVAL, "spconv_plan: lf=%d outside [1, 64]", lf);
    if (k < 1 || k > 64) return fail(HRIR_EINVAL, "spconv_plan: k=%d outside [1, 64]", k);
    if (lg < 1 || lg > 2048) return fail(HRIR_EINVAL, "spconv_plan: lg=%d outside [1, 2048]", lg);
    if (n_filters < 1) return fail(HRIR_EINVAL, "spconv_plan: n_filters=%d < 1", n_filters);
    for (int i = 0; i < n_res * lf; ++i)
        if (!std::isfinite(r[i])) return fail(HRIR_EINVAL, "spconv_plan: r[%d] not finite", i);
    if (n_res > 1)
        for (int f = 0; f < n_filters; ++f)
            if (res[f] < 0 || res[f] >= n_res)
                return fail(HRIR_EINVAL, "spconv_plan: region %d of filter %d outside [0, %d)", res[f], f, n_res);
    for (int64_t i = 0; i < (int64_t)n_filters * k; ++i) {
        if (p[i] < 0 || p[i] >= lg)
            return fail(HRIR_EINVAL, "spconv_plan: p[%lld]=%d outside [0, %d)", (long long)i, p[i], lg);
        if (!(g[i] >= 0.0f) || !std::isfinite(g[i]))
            return fail(HRIR_EINVAL, "spconv_plan: g[%lld] must be finite and >= 0", (long long)i);
    }
    auto* pl = new (std::nothrow) hrir_plan;
    if (!pl) return fail(HRIR_ENOMEM, "spconv_plan: out of host memory");
    pl->lf = lf; pl->lfp = pad_lf(lf); pl->k = k; pl->kp = pad_k(k); pl->lg = lg; pl->n_filters = n_filters;
    pl->n_res = n_res;
    if (n_res > 1) pl->res.assign(res, res + n_filters);
    std::vector<float> hr((size_t)n_res * pl->lfp, 0.0f);
    for (int q = 0; q < n_res; ++q) std::memcpy(hr.data() + (size_t)q * pl->lfp, r + (size_t)q * lf, sizeof(float) * lf);
    std::vector<int> hp((size_t)n_filters * pl->kp, 0);
    std::vector<float> hg((size_t)n_filters * pl->kp, 0.0f);
    for (int f = 0; f < n_filters; ++f)
        for (int j = 0; j < k; ++j) {
            hp[(size_t)f * pl->kp + j] = p[(size_t)f * k + j];
            hg[(size_t)f * pl->kp + j] = g[(size_t)f * k + j];
        }
    auto bail = [&](int code) { (void)hipFree(pl->d_r); (void)hipFree(pl->d_p); (void)hipFree(pl->d_g); delete pl; return code; };
    hipError_t e = hipGetDevice(&pl->device);
    if (e == hipSuccess) e = hipMalloc(&pl->d_r, hr.size() * sizeof(float));
    if (e == hipSuccess) e = hipMalloc(&pl->d_p, hp.size() * sizeof(int));
    if (e == hipSuccess) e = hipMalloc(&pl->d_g, hg.size() * sizeof(float));
    if (e == hipSuccess) e = hipMemcpy(pl->d_r, hr.data(), hr.size() * sizeof(float), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(pl->d_p, hp.data(), hp.size() * sizeof(int), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(pl->d_g, hg.data(), hg.size() * sizeof(float), hipMemcpyHostToDevice);
    if (e != hipSuccess)
        return bail(fail(e == hipErrorOutOfMemory ? HRIR_ENOMEM : HRIR_EDEVICE, "spconv_plan: %s", hipGetErrorString(e)));
    *out = pl;
    return HRIR_OK;
}

extern "C" int spconv_plan(const float* r, int32_t lf, const int32_t* p, const float* g, int32_t n_filters,
                           int32_t k, int32_t lg, hrir_plan** out) {
    return spconv_plan_multi(r, 1, lf, nullptr, p, g, n_filters, k, lg, out);
}

namespace hrir {
PlanView plan_view(const hrir_plan* pl) {
    return PlanView{pl->lf, pl->lfp, pl->k, pl->kp, pl->lg, pl->n_filters, pl->device, pl->n_res,
                    pl->d_r, pl->d_p, pl->d_g, pl->rows_gen};
}
void plan_rows_changed(hrir_plan* pl) { ++pl->rows_gen; }
}  // namespace hrir

extern "C" int spconv_plan_shape(const hrir_plan* plan, int32_t* lf_k_lg3) {
    clear_error();
    if (!plan || !lf_k_lg3) return fail(HRIR_EINVAL, "spconv_plan_shape: null pointer");
    lf_k_lg3[0] = plan->lf;
    lf_k_lg3[1] = plan->k;
    lf_k_lg3[2] = plan->lg;
    return HRIR_OK;
}

extern "C" int spconv_plan_device(const hrir_plan* plan, const float** r, const int** p, const float** g,
                                  int32_t* lfp_kp_nf3) {
    clear_error();
    if (!plan || !r || !p || !g || !lfp_kp_nf3) return fail(HRIR_EINVAL, "spconv_plan_device: null pointer");
    *r = plan->d_r;
    *p = plan->d_p;
    *g = plan->d_g;
    lfp_kp_nf3[0] = plan->lfp;
    lfp_kp_nf3[1] = plan->kp;
    lfp_kp_nf3[2] = plan->n_filters;
    return HRIR_OK;
}

extern "C" int spconv_plan_read(const hrir_plan* plan, int32_t first_row, int32_t n_rows, int32_t* p_out,
                                float* g_out) {
    clear_error();
    if (!plan || (n_rows > 0 && (!p_out || !g_out))) return fail(HRIR_EINVAL, "spconv_plan_read: null pointer");
    if (first_row < 0 || n_rows < 0 || (int64_t)first_row + n_rows > plan->n_filters)
        return fail(HRIR_EINVAL, "spconv_plan_read: rows outside the plan");
    std::vector<int> hp((size_t)n_rows * plan->kp);
    std::vector<float> hg((size_t)n_rows * plan->kp);
    hipError_t e = hipDeviceSynchronize();
    if (e == hipSuccess && n_rows > 0)
        e = hipMemcpy(hp.data(), plan->d_p + (size_t)first_row * plan->kp, hp.size() * sizeof(int),
                      hipMemcpyDeviceToHost);
    if (e == hipSuccess && n_rows > 0)
        e = hipMemcpy(hg.data(), plan->d_g + (size_t)first_row * plan->kp, hg.size() * sizeof(float),
                      hipMemcpyDeviceToHost);
    if (e != hipSuccess) return fail(HRIR_EDEVICE, "spconv_plan_read: %s", hipGetErrorString(e));
    for (int i = 0; i < n_rows; ++i)
        for (int j = 0; j < plan->k; ++j) {
            p_out[(size_t)i * plan->k + j] = hp[(size_t)i * plan->kp + j];
            g_out[(size_t)i * plan->k + j] = hg[(size_t)i * plan->kp + j];
        }
    return HRIR_OK;
}

extern "C" void spconv_plan_destroy(hrir_plan* plan) {
    if (!plan) return;
    (void)hipFree(plan->d_r);
    (void)hipFree(plan->d_p);
    (void)hipFree(plan->d_g);
    delete plan;
}

namespace {

// Source and job-list checks shared by the batch and one-shot entry points.
int check_jobs(const hrir_plan* plan, const int64_t* src_off, const int64_t* src_len, int32_t n_src,
               const spconv_job* jobs, int32_t n_jobs, const char* who) {
    const int lf = plan->lf, lg = plan->lg;
    for (int i = 0; i < n_src; ++i) {
        if (src_len[i] < 1 || src_len[i] > (int64_t)INT32_MAX - lf - lg)
            return fail(HRIR_EINVAL, "%s: src_len[%d]=%lld out of range", who, i, (long long)src_len[i]);
        if (src_off[i] < 0) return fail(HRIR_EINVAL, "%s: src_off[%d] < 0", who, i);
    }
    for (int j = 0; j < n_jobs; ++j) {
        if (jobs[j].src < 0 || jobs[j].src >= n_src)
            return fail(HRIR_EINVAL, "%s: job %d source %d out of range", who, j, jobs[j].src);
        if (jobs[j].filt < 0 || jobs[j].filt >= plan->n_filters)
            return fail(HRIR_EINVAL, "%s: job %d filter %d out of range", who, j, jobs[j].filt);
        if (jobs[j].out_off < 0) return fail(HRIR_EINVAL, "%s: job %d out_off < 0", who, j);
    }
    return HRIR_OK;
}

int job_region(const hrir_plan* plan, int filt) { return plan->n_res > 1 ? plan->res[filt] : 0; }

// Job indices grouped by source, then by region, keeping list order inside a
// group: a tile's jobs share one z = r_region * s.  In place (no allocation).
void order_jobs(const hrir_plan* plan, const spconv_job* jobs, int n_jobs, int* order) {
    for (int j = 0; j < n_jobs; ++j) order[j] = j;
    std::sort(order, order + n_jobs, [&](int a, int c) {
        if (jobs[a].src != jobs[c].src) return jobs[a].src < jobs[c].src;
        const int ra = job_region(plan, jobs[a].filt), rc = job_region(plan, jobs[c].filt);
        if (ra != rc) return ra < rc;
        return a < c;
    });
}

// Calls run(s, region, j0, j1) for each run [j0, j1) of ordered jobs that
// share a source and a region.
template <class F>
void for_each_run(const hrir_plan* plan, const spconv_job* jobs, const int* order, int n_jobs, F&& run) {
    for (int j0 = 0; j0 < n_jobs;) {
        const int s = jobs[order[j0]].src;
        const int rg = job_region(plan, jobs[order[j0]].filt);
        int j1 = j0;
        while (j1 < n_jobs && jobs[order[j1]].src == s && job_region(plan, jobs[order[j1]].filt) == rg) ++j1;
        run(s, rg, j0, j1);
        j0 = j1;
    }
}

// Largest work first: the hardware dispatcher (or the persistent queue) then
// finishes a ragged job mix with small tiles at the end.  Equal work keeps
// the creation order (job range, then time), so the order is unique.
void order_tiles(TileDesc* t, int64_t n, int tile) {
    std::sort(t, t + n, [tile](const TileDesc& a, const TileDesc& c) {
        const int64_t wa = (int64_t)a.job_count * std::min<int64_t>(tile, a.out_len - a.t0);
        const int64_t wc = (int64_t)c.job_count * std::min<int64_t>(tile, c.out_len - c.t0);
        if (wa != wc) return wa > wc;
        if (a.job_begin != c.job_begin) return a.job_begin < c.job_begin;
        return a.t0 < c.t0;
    });
}

}  // namespace

extern "C" int spconv_batch_create(const hrir_plan* plan, const int64_t* src_off, const int64_t* src_len,
                                   int32_t n_src, const spconv_job* jobs, int32_t n_jobs, int32_t tile,
                                   int32_t group, int32_t flags, hrir_batch** out) {
    clear_error();
    if (!plan || !out || (n_src > 0 && (!src_off || !src_len)) || (n_jobs > 0 && !jobs))
        return fail(HRIR_EINVAL, "spconv_batch_create: null pointer");
    *out = nullptr;
    if (n_src < 0 || n_jobs < 0) return fail(HRIR_EINVAL, "spconv_batch_create: negative count");
    if (flags & ~(SPCONV_PERSISTENT | SPCONV_GRAPH | SPCONV_UNFUSED | SPCONV_LDS_GATHER | SPCONV_REGWIN | SPCONV_WG256))
        return fail(HRIR_EINVAL, "spconv_batch_create: unknown flags 0x%x", flags);
    const int kflags = flags & (SPCONV_UNFUSED | SPCONV_LDS_GATHER | SPCONV_REGWIN);
    if (kflags & (kflags - 1))
        return fail(HRIR_EINVAL, "spconv_batch_create: UNFUSED, LDS_GATHER and REGWIN are exclusive");
    if ((flags & SPCONV_UNFUSED) && (flags & SPCONV_PERSISTENT))
        return fail(HRIR_EINVAL, "spconv_batch_create: UNFUSED and PERSISTENT are exclusive");
    if ((flags & SPCONV_REGWIN) && plan->lg > kHW + 1)
        return fail(HRIR_EINVAL, "spconv_batch_create: the register-window kernel needs lg <= %d (lg=%d)", kHW + 1,
                    plan->lg);
    const int kind = (flags & SPCONV_UNFUSED) ? KIND_UNFUSED
                     : (flags & SPCONV_REGWIN) ? KIND_REGWIN
                     : (flags & SPCONV_LDS_GATHER) ? KIND_LDS_GATHER
                                                   : KIND_QUAD;
    const int tile_unit = kind == KIND_REGWIN ? kTileRW : kChunk;
    const int tile_max = kind == KIND_QUAD ? kQuadTileMax : 16384;
    if (tile == 0) tile = kind == KIND_REGWIN ? kTileRW : kind == KIND_QUAD ? 2048 : 4096;
    if (tile < tile_unit || tile % tile_unit || tile > tile_max)
        return fail(HRIR_EINVAL, "spconv_batch_create: tile=%d must be a multiple of %d in [%d, %d]", tile,
                    tile_unit, tile_unit, tile_max);
    if (group < 0) return fail(HRIR_EINVAL, "spconv_batch_create: group < 0");
    if ((flags & SPCONV_WG256) && kind != KIND_QUAD)
        return fail(HRIR_EINVAL, "spconv_batch_create: WG256 needs the default kernel");
    if ((flags & SPCONV_WG256) && tile + plan->lg + 2 > kQSmallCover)
        return fail(HRIR_EINVAL, "spconv_batch_create: WG256 needs tile + lg + 2 <= %d (tile %d, lg %d)", kQSmallCover,
                    tile, plan->lg);
    if (plan->n_res > 1 && kind != KIND_QUAD)
        return fail(HRIR_EINVAL, "spconv_batch_create: a plan with %d resonance filters needs the default kernel",
                    plan->n_res);
    const int lf = plan->lf, lg = plan->lg;
    if (int rc = check_jobs(plan, src_off, src_len, n_src, jobs, n_jobs, "spconv_batch_create")) return rc;
    auto* b = new (std::nothrow) hrir_batch;
    if (!b) return fail(HRIR_ENOMEM, "spconv_batch_create: out of host memory");
    b->plan = plan; b->flags = flags; b->TB = tile; b->n_jobs = n_jobs; b->kind = kind;
    b->nt = (flags & SPCONV_WG256) ? 256 : 512;
    for (int j = 0; j < n_jobs; ++j) {
        const int s = jobs[j].src;
        b->src_extent = std::max(b->src_extent, src_off[s] + src_len[s]);
        b->out_extent = std::max(b->out_extent, jobs[j].out_off + src_len[s] + lf + lg - 2);
    }
    std::vector<int> order(n_jobs);
    order_jobs(plan, jobs, n_jobs, order.data());
    std::vector<JobDesc> hj(n_jobs);
    for (int j = 0; j < n_jobs; ++j) hj[j] = JobDesc{jobs[order[j]].out_off, jobs[order[j]].filt, 0};
    std::vector<TileDesc> ht;
    std::vector<ZDesc> hz;
    std::vector<GDesc> hg;
    int64_t zsize = 0;
    int max_group = 0;
    for_each_run(plan, jobs, order.data(), n_jobs, [&](int s, int rg, int j0, int j1) {
        const int njs = j1 - j0;
        const int gsz = group > 0 ? std::min(group, njs) : njs;
        max_group = std::max(max_group, gsz);
        const int64_t out_len = src_len[s] + lf + lg - 2;
        for (int g0 = j0; g0 < j1; g0 += gsz)
            for (int64_t t0 = 0; t0 < out_len; t0 += tile)
                ht.push_back(TileDesc{src_off[s], (int32_t)src_len[s], (int32_t)out_len, (int32_t)t0, g0,
                                      std::min(gsz, j1 - g0), rg});
        if (flags & SPCONV_UNFUSED) {
            const int64_t nz = src_len[s] + lf - 1;
            for (int64_t v0 = 0; v0 < nz; v0 += kZChunk)
                hz.push_back(ZDesc{src_off[s], zsize, (int32_t)src_len[s], (int32_t)v0});
            for (int j = j0; j < j1; ++j)
                for (int64_t t0 = 0; t0 < out_len; t0 += kZChunk)
                    hg.push_back(GDesc{hj[j].out_off, zsize, (int32_t)out_len, (int32_t)nz, (int32_t)t0, hj[j].filt});
            zsize += round_up((int)std::min<int64_t>(nz, INT32_MAX - 64), 64);
        }
    });
    order_tiles(ht.data(), (int64_t)ht.size(), tile);
    b->n_tiles = (int64_t)ht.size();
    b->group = max_group;
    b->lds_bytes = kind == KIND_REGWIN ? (size_t)rw_lds_bytes(tile, plan->lfp)
                   : kind == KIND_QUAD ? (size_t)quad_lds_bytes(tile, lg, plan->lfp)
                                       : sizeof(float) * (size_t)(lds_s_len(tile, lg, plan->lfp) + lds_z_len(tile, lg));
    b->n_z = (int64_t)hz.size();
    b->n_gd = (int64_t)hg.size();
    auto bail = [&](int code) { free_batch(b); return code; };
    if (b->lds_bytes > 160 * 1024)
        return bail(fail(HRIR_EINVAL, "spconv_batch_create: tile %d with lg %d needs %zu B of LDS (> 160 KiB)", tile, lg,
                         b->lds_bytes));
    if (b->n_tiles > INT32_MAX) return bail(fail(HRIR_EINVAL, "spconv_batch_create: too many tiles"));
    b->direct = quad_direct(ht.data(), (int64_t)ht.size());
    hipError_t e = hipSuccess;
    if (n_jobs > 0) {
        e = hipMalloc(&b->d_tiles, ht.size() * sizeof(TileDesc));
        if (e == hipSuccess) e = hipMalloc(&b->d_jobs, hj.size() * sizeof(JobDesc));
        if (e == hipSuccess) e = hipMemcpy(b->d_tiles, ht.data(), ht.size() * sizeof(TileDesc), hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(b->d_jobs, hj.data(), hj.size() * sizeof(JobDesc), hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMalloc(&b->d_ctr, 2 * sizeof(int));
        if (e == hipSuccess) e = hipMemset(b->d_ctr, 0, 2 * sizeof(int));
        if (e == hipSuccess && (flags & SPCONV_UNFUSED)) {
            e = hipMalloc(&b->d_z, hz.size() * sizeof(ZDesc));
            if (e == hipSuccess) e = hipMalloc(&b->d_gd, hg.size() * sizeof(GDesc));
            if (e == hipSuccess) e = hipMalloc(&b->d_zbuf, (size_t)zsize * sizeof(float));
            if (e == hipSuccess) e = hipMemcpy(b->d_z, hz.data(), hz.size() * sizeof(ZDesc), hipMemcpyHostToDevice);
            if (e == hipSuccess) e = hipMemcpy(b->d_gd, hg.data(), hg.size() * sizeof(GDesc), hipMemcpyHostToDevice);
        }
    }
    if (e != hipSuccess)
        return bail(fail(e == hipErrorOutOfMemory ? HRIR_ENOMEM : HRIR_EDEVICE, "spconv_batch_create: %s",
                         hipGetErrorString(e)));
    // Kernel attributes and the persistent grid size.
    int rc = kind == KIND_REGWIN ? rw_prepare(plan->lfp, b->lds_bytes, (flags & SPCONV_PERSISTENT) != 0, b->n_tiles,
                                              &b->grid)
             : kind == KIND_QUAD ? quad_prepare(plan->lfp, plan->kp, b->nt, b->lds_bytes,
                                                (flags & SPCONV_PERSISTENT) != 0, b->n_tiles, &b->grid)
                                 : dispatch(plan->lfp, plan->kp, [&](auto L, auto K) -> int {
        constexpr int LV = decltype(L)::value, KV = decltype(K)::value;
        const void* kt = reinterpret_cast<const void*>(&k_render_tiles<LV, KV>);
        const void* kpers = reinterpret_cast<const void*>(&k_render_persistent<LV, KV>);
        HIP_TRY(hipFuncSetAttribute(kt, hipFuncAttributeMaxDynamicSharedMemorySize, (int)b->lds_bytes));
        HIP_TRY(hipFuncSetAttribute(kpers, hipFuncAttributeMaxDynamicSharedMemorySize, (int)b->lds_bytes));
        if (flags & SPCONV_PERSISTENT) {
            int per_cu = 0, dev = 0, cus = 0;
            HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kpers, kThreads, b->lds_bytes));
            HIP_TRY(hipGetDevice(&dev));
            HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
            b->grid = (int)std::min<int64_t>(std::max(per_cu, 1) * (int64_t)cus, std::max<int64_t>(b->n_tiles, 1));
        } else {
            b->grid = (int)std::max<int64_t>(b->n_tiles, 0);
        }
        return HRIR_OK;
    });
    if (rc) return bail(rc);
    *out = b;
    return HRIR_OK;
}

extern "C" int spconv_batch_render(hrir_batch* b, const float* d_src, int64_t src_elems, float* d_out,
                                   int64_t out_elems, void* stream) {
    clear_error();
    if (!b) return fail(HRIR_EINVAL, "spconv_batch_render: null batch");
    if (b->n_jobs == 0) return HRIR_OK;
    if (!d_src || !d_out) return fail(HRIR_EINVAL, "spconv_batch_render: null device pointer");
    if (src_elems < b->src_extent || out_elems < b->out_extent)
        return fail(HRIR_EINVAL, "spconv_batch_render: buffers too small (src %lld < %lld or out %lld < %lld)",
                    (long long)src_elems, (long long)b->src_extent, (long long)out_elems, (long long)b->out_extent);
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    if (!(b->flags & SPCONV_GRAPH)) return launch(b, d_src, d_out, st);
    if (!b->exec) {
        HIP_TRY(hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking));
        HIP_TRY(hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal));
        int rc = launch(b, d_src, d_out, b->cap_stream);
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamEndCapture(b->cap_stream, &g);
        if (rc) { if (g) (void)hipGraphDestroy(g); return rc; }
        if (e != hipSuccess) return fail(HRIR_EDEVICE, "graph capture: %s", hipGetErrorString(e));
        b->graph = g;
        HIP_TRY(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
        b->g_src = d_src;
        b->g_out = d_out;
    } else if (d_src != b->g_src || d_out != b->g_out) {
        return fail(HRIR_EINVAL, "spconv_batch_render: graph batch replayed with different buffers");
    }
    HIP_TRY(hipGraphLaunch(b->exec, st));
    return HRIR_OK;
}

extern "C" int spconv_batch_info(const hrir_batch* b, int64_t* info5) {
    clear_error();
    if (!b || !info5) return fail(HRIR_EINVAL, "spconv_batch_info: null pointer");
    info5[0] = b->n_tiles;
    info5[1] = b->TB;
    info5[2] = b->group;
    info5[3] = b->grid;
    info5[4] = b->kind;
    return HRIR_OK;
}

extern "C" void spconv_batch_destroy(hrir_batch* b) { free_batch(b); }

extern "C" int spconv_render(const hrir_plan* plan, const float* d_src, int64_t src_elems, const int64_t* src_off,
                             const int64_t* src_len, int32_t n_src, const spconv_job* jobs, int32_t n_jobs,
                             float* d_out, int64_t out_elems, void* stream) {
    hrir_batch* b = nullptr;
    int rc = spconv_batch_create(plan, src_off, src_len, n_src, jobs, n_jobs, 0, 0, 0, &b);
    if (rc) return rc;
    rc = spconv_batch_render(b, d_src, src_elems, d_out, out_elems, stream);
    hipError_t e = hipStreamSynchronize(reinterpret_cast<hipStream_t>(stream));
    free_batch(b);
    if (rc) return rc;
    if (e != hipSuccess) return fail(HRIR_EDEVICE, "spconv_render: %s", hipGetErrorString(e));
    return HRIR_OK;
}

// ===========================================================================
// Allocation-free one-shot render: the tile and job descriptors of
// spconv_render live in a fixed device array instead of a batch's hipMalloc'd
// table, for callers that cannot allocate device memory.
// ===========================================================================
namespace {

constexpr size_t kNaJobBytes = sizeof(JobDesc) * SPCONV_NOALLOC_MAX_JOBS;
constexpr size_t kNaBytes = kNaJobBytes + sizeof(TileDesc) * SPCONV_NOALLOC_MAX_TILES;
constexpr int kNaMaxDevices = 64;
static_assert(kNaJobBytes % 256 == 0, "tile descriptors start 256-byte aligned");

// Host-side state, all guarded by na_mutex: the device address of `scratch`
// on each device (from hipGetSymbolAddress on the first call there), and the
// host staging of the descriptors (static, so no call allocates).
std::mutex na_mutex;
unsigned char* na_dev[kNaMaxDevices];
int na_order[SPCONV_NOALLOC_MAX_JOBS];
JobDesc na_jobs[SPCONV_NOALLOC_MAX_JOBS];
TileDesc na_tiles[SPCONV_NOALLOC_MAX_TILES];

}  // namespace

// Job descriptors at offset 0, tile descriptors after them.  Host code never
// passes this name to a kernel or a copy: it uses the address returned by
// hipGetSymbolAddress for the current device.
static __device__ __align__(256) unsigned char scratch[kNaBytes];

extern "C" int spconv_render_noalloc(const hrir_plan* plan, const float* d_src, int64_t src_elems,
                                     const int64_t* src_off, const int64_t* src_len, int32_t n_src,
                                     const spconv_job* jobs, int32_t n_jobs, float* d_out, int64_t out_elems,
                                     void* stream) {
    static const char* who = "spconv_render_noalloc";
    clear_error();
    if (!plan || (n_src > 0 && (!src_off || !src_len)) || (n_jobs > 0 && !jobs))
        return fail(HRIR_EINVAL, "%s: null pointer", who);
    if (n_src < 0 || n_jobs < 0) return fail(HRIR_EINVAL, "%s: negative count", who);
    if (n_jobs > SPCONV_NOALLOC_MAX_JOBS)
        return fail(HRIR_EINVAL, "%s: %d jobs exceed the limit of %d", who, n_jobs, SPCONV_NOALLOC_MAX_JOBS);
    if (int rc = check_jobs(plan, src_off, src_len, n_src, jobs, n_jobs, who)) return rc;
    if (n_jobs == 0) return HRIR_OK;
    const int lf = plan->lf, lg = plan->lg, tile = 2048;
    const size_t lds_bytes = (size_t)quad_lds_bytes(tile, lg, plan->lfp);
    if (lds_bytes > 160 * 1024) return fail(HRIR_EINVAL, "%s: lg %d needs %zu B of LDS (> 160 KiB)", who, lg, lds_bytes);

    std::lock_guard<std::mutex> lock(na_mutex);
    // the limits and the buffer extents are checked before any device work
    order_jobs(plan, jobs, n_jobs, na_order);
    int64_t n_tiles = 0;
    for_each_run(plan, jobs, na_order, n_jobs, [&](int s, int, int, int) {
        n_tiles += (src_len[s] + lf + lg - 2 + tile - 1) / tile;
    });
    if (n_tiles > SPCONV_NOALLOC_MAX_TILES)
        return fail(HRIR_EINVAL, "%s: %lld tiles of %d outputs exceed the limit of %d", who, (long long)n_tiles, tile,
                    SPCONV_NOALLOC_MAX_TILES);
    if (!d_src || !d_out) return fail(HRIR_EINVAL, "%s: null device pointer", who);
    int64_t src_extent = 0, out_extent = 0;
    for (int j = 0; j < n_jobs; ++j) {
        const int s = jobs[j].src;
        src_extent = std::max(src_extent, src_off[s] + src_len[s]);
        out_extent = std::max(out_extent, jobs[j].out_off + src_len[s] + lf + lg - 2);
    }
    if (src_elems < src_extent || out_elems < out_extent)
        return fail(HRIR_EINVAL, "%s: buffers too small (src %lld < %lld or out %lld < %lld)", who,
                    (long long)src_elems, (long long)src_extent, (long long)out_elems, (long long)out_extent);
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kNaMaxDevices) return fail(HRIR_EINVAL, "%s: device %d >= %d", who, dev, kNaMaxDevices);
    if (dev != plan->device) return fail(HRIR_EINVAL, "%s: current device %d, plan on %d", who, dev, plan->device);
    if (!na_dev[dev]) {
        void* ptr = nullptr;
        HIP_TRY(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        na_dev[dev] = static_cast<unsigned char*>(ptr);
    }
    JobDesc* d_jobs = reinterpret_cast<JobDesc*>(na_dev[dev]);
    TileDesc* d_tiles = reinterpret_cast<TileDesc*>(na_dev[dev] + kNaJobBytes);

    for (int j = 0; j < n_jobs; ++j) na_jobs[j] = JobDesc{jobs[na_order[j]].out_off, jobs[na_order[j]].filt, 0};
    int64_t nt = 0;
    for_each_run(plan, jobs, na_order, n_jobs, [&](int s, int rg, int j0, int j1) {
        const int64_t out_len = src_len[s] + lf + lg - 2;
        for (int64_t t0 = 0; t0 < out_len; t0 += tile)
            na_tiles[nt++] = TileDesc{src_off[s], (int32_t)src_len[s], (int32_t)out_len, (int32_t)t0, j0, j1 - j0, rg};
    });
    order_tiles(na_tiles, nt, tile);

    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    int grid = 0;
    if (int rc = quad_prepare(plan->lfp, plan->kp, 512, lds_bytes, false, nt, &grid)) return rc;
    // the staging arrays and the device descriptors are reused by the next
    // call: whatever happens, wait for this one before the lock is released
    hipError_t e = hipMemcpyAsync(d_jobs, na_jobs, sizeof(JobDesc) * (size_t)n_jobs, hipMemcpyHostToDevice, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(d_tiles, na_tiles, sizeof(TileDesc) * (size_t)nt, hipMemcpyHostToDevice, st);
    int rc = HRIR_OK;
    if (e == hipSuccess) {
        rc = quad_launch(plan->lfp, plan->kp, 512, false, quad_direct(na_tiles, nt), grid, lds_bytes, st, d_src,
                         d_tiles, (int)nt, d_jobs, plan->d_r, plan->d_p, plan->d_g, d_out, lg, tile, nullptr);
        if (rc == HRIR_OK) e = hipGetLastError();
    }
    const hipError_t es = hipStreamSynchronize(st);
    if (rc) return rc;
    if (e == hipSuccess) e = es;
    if (e != hipSuccess) return fail(HRIR_EDEVICE, "%s: %s", who, hipGetErrorString(e));
    return HRIR_OK;
}
