// Dense direct convolution of sources with full-length HRIRs on gfx950: the
// comparison leg for the sparse renderer (direct convolution costs the
// filter length per output sample, Sec. IV-F).
//
//     out[t] = sum_{m < M} h[m] s[t - m],   t in [0, len(s) + M - 1).
//
// Tile: one source, kDTile outputs, up to kDGroup of that source's jobs.
// The workgroup stages s[t0 - (kDM - 1), t0 + kDTile) and the group's HRIRs
// (zero padded to kDM = 200 taps) in LDS.  Lane l of wave w owns kDR
// consecutive outputs and keeps the kDR + kDM - 1 source samples they read in
// registers, loaded once per tile; every job then costs kDM * kDR fmas with
// static register operands and the taps broadcast from LDS, four per 16-byte
// read.  Results leave through a per-wave LDS slab so that each global store
// instruction writes 1 KiB contiguously.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>

#include "hrir_internal.h"
#include "render_common.h"

namespace hrir {

constexpr int kDM = 200;                  // taps served (HRIRs up to 200 taps)
constexpr int kDR = 8;                    // consecutive outputs per lane
constexpr int kDWin = kDR + kDM - 1;      // window registers per lane
constexpr int kDSeg = 64 * kDR;           // outputs per wave
constexpr int kDTile = kWaves * kDSeg;    // outputs per tile (2048)
constexpr int kDGroup = 16;               // jobs per tile
constexpr int kDRowS = 12;                // slab row stride (floats)
constexpr int kDSlab = 64 * kDRowS;
static_assert(kDM % 4 == 0 && kDSeg % 256 == 0, "dense layout");

struct DTile {                            // 32 bytes
    int64_t src_off;
    int32_t src_len;
    int32_t out_len;                      // src_len + m - 1
    int32_t t0;
    int32_t job_begin;
    int32_t job_count;
    int32_t pad;
};

__host__ __device__ inline int dense_s_len() { return round_up(kDTile + kDM - 1, 4) + 4; }
__host__ __device__ inline int dense_lds_floats() {
    const int a = dense_s_len() > kWaves * kDSlab ? dense_s_len() : kWaves * kDSlab;
    return a + kDGroup * kDM;
}

__global__ __launch_bounds__(kThreads, 2) void k_dense(const float* __restrict__ src, const DTile* __restrict__ tiles,
                                                       const JobDesc* __restrict__ jobs,
                                                       const float* __restrict__ h, float* __restrict__ out) {
    extern __shared__ float4 smem4[];
    float* lds = reinterpret_cast<float*>(smem4);
    const int s_len = dense_s_len();
    float* s_win = lds;                                   // later the transpose slabs
    float* taps = lds + (s_len > kWaves * kDSlab ? s_len : kWaves * kDSlab);
    const DTile td = tiles[blockIdx.x];
    const int tid = threadIdx.x;

    // stage s[t0 - (kDM-1) + i], zero outside [0, src_len), and the taps
    const int64_t sbase = (int64_t)td.t0 - (kDM - 1);
    const float* sp = src + td.src_off;
    for (int i = tid; i < s_len; i += kThreads) {
        const int64_t q = sbase + i;
        s_win[i] = (q >= 0 && q < td.src_len) ? sp[q] : 0.0f;
    }
    for (int i = tid; i < td.job_count * kDM; i += kThreads) {
        const int q = i / kDM, m = i - q * kDM;
        taps[i] = h[(int64_t)jobs[td.job_begin + q].filt * kDM + m];
    }
    __syncthreads();

    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
    const int seg = wave * kDSeg;
    const int tile_len = min(kDTile, td.out_len - td.t0);
    // w[u] = s[t0 + seg + kDR lane - (kDM - 1) + u]
    float w[kDWin];
    {
        const float* sl = s_win + seg + kDR * lane;
#pragma unroll
        for (int u = 0; u < kDWin - 3; u += 4) {
            const float4 v = *reinterpret_cast<const float4*>(sl + u);
            w[u] = v.x; w[u + 1] = v.y; w[u + 2] = v.z; w[u + 3] = v.w;
        }
#pragma unroll
        for (int u = (kDWin / 4) * 4; u < kDWin; ++u) w[u] = sl[u];
    }
    __syncthreads();                                      // s_win is reused as slabs below
    if (seg >= tile_len) return;
    const int seg_len = min(kDSeg, tile_len - seg);
    float* slab = s_win + wave * kDSlab;
    for (int q = 0; q < td.job_count; ++q) {
        const JobDesc jd = jobs[td.job_begin + q];
        const float* tq = taps + q * kDM;
        float acc[kDR];
#pragma unroll
        for (int i = 0; i < kDR; ++i) acc[i] = 0.0f;
#pragma unroll
        for (int m = 0; m < kDM; m += 4) {
            const float4 hv = *reinterpret_cast<const float4*>(tq + m);   // same address in every lane
            const float hm[4] = {hv.x, hv.y, hv.z, hv.w};
#pragma unroll
            for (int e = 0; e < 4; ++e)
#pragma unroll
                for (int i = 0; i < kDR; ++i) acc[i] = fmaf(hm[e], w[i + kDM - 1 - (m + e)], acc[i]);
        }
        int ln;
        asm volatile("" : "=v"(ln) : "0"(static_cast<int>(threadIdx.x & 63)));
#pragma unroll
        for (int i = 0; i < kDR; i += 4)
            *reinterpret_cast<float4*>(slab + ln * kDRowS + i) = make_float4(acc[i], acc[i + 1], acc[i + 2], acc[i + 3]);
        constexpr int kPass = kDSeg / 256;
        float4 v[kPass];
#pragma unroll
        for (int c = 0; c < kPass; ++c) {
            const int qo = 256 * c + 4 * ln;
            v[c] = *reinterpret_cast<const float4*>(slab + (qo / kDR) * kDRowS + (qo % kDR));
        }
        float* orow = out + jd.out_off + td.t0 + seg;
        if (seg_len == kDSeg && ((reinterpret_cast<uintptr_t>(orow) & 15) == 0)) {
#pragma unroll
            for (int c = 0; c < kPass; ++c) *reinterpret_cast<float4*>(orow + 256 * c + 4 * ln) = v[c];
        } else {
#pragma unroll
            for (int c = 0; c < kPass; ++c) {
                const int qo = 256 * c + 4 * ln;
                if (qo + 0 < seg_len) orow[qo + 0] = v[c].x;
                if (qo + 1 < seg_len) orow[qo + 1] = v[c].y;
                if (qo + 2 < seg_len) orow[qo + 2] = v[c].z;
                if (qo + 3 < seg_len) orow[qo + 3] = v[c].w;
            }
        }
    }
}

}  // namespace hrir

using namespace hrir;

struct hrir_dense {
    int m = 0, n_filters = 0;
    float* d_h = nullptr;                 // [n_filters][kDM], zero padded
};

struct hrir_dense_batch {
    const hrir_dense* plan = nullptr;
    int64_t n_tiles = 0, n_jobs = 0, src_extent = 0, out_extent = 0;
    DTile* d_tiles = nullptr;
    JobDesc* d_jobs = nullptr;
};

extern "C" int dense_plan(const float* h, int32_t n_filters, int32_t m, hrir_dense** out) {
    clear_error();
    if (!h || !out) return fail(HRIR_EINVAL, "dense_plan: null pointer");
    *out = nullptr;
    if (m < 1 || m > kDM) return fail(HRIR_EINVAL, "dense_plan: m=%d outside [1, %d]", m, kDM);
    if (n_filters < 1) return fail(HRIR_EINVAL, "dense_plan: n_filters=%d < 1", n_filters);
    for (int64_t i = 0; i < (int64_t)n_filters * m; ++i)
        if (!std::isfinite(h[i])) return fail(HRIR_EINVAL, "dense_plan: h[%lld] not finite", (long long)i);
    std::vector<float> hp((size_t)n_filters * kDM, 0.0f);
    for (int f = 0; f < n_filters; ++f) std::memcpy(&hp[(size_t)f * kDM], h + (size_t)f * m, sizeof(float) * m);
    auto* p = new (std::nothrow) hrir_dense;
    if (!p) return fail(HRIR_ENOMEM, "dense_plan: out of host memory");
    p->m = m;
    p->n_filters = n_filters;
    hipError_t e = hipMalloc(&p->d_h, hp.size() * sizeof(float));
    if (e == hipSuccess) e = hipMemcpy(p->d_h, hp.data(), hp.size() * sizeof(float), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        (void)hipFree(p->d_h);
        delete p;
        return fail(e == hipErrorOutOfMemory ? HRIR_ENOMEM : HRIR_EDEVICE, "dense_plan: %s", hipGetErrorString(e));
    }
    *out = p;
    return HRIR_OK;
}

extern "C" void dense_plan_destroy(hrir_dense* p) {
    if (!p) return;
    (void)hipFree(p->d_h);
    delete p;
}

extern "C" int dense_batch_create(const hrir_dense* plan, const int64_t* src_off, const int64_t* src_len,
                                  int32_t n_src, const spconv_job* jobs, int32_t n_jobs, hrir_dense_batch** out) {
    clear_error();
    if (!plan || !out || (n_src > 0 && (!src_off || !src_len)) || (n_jobs > 0 && !jobs))
        return fail(HRIR_EINVAL, "dense_batch_create: null pointer");
    *out = nullptr;
    if (n_src < 0 || n_jobs < 0) return fail(HRIR_EINVAL, "dense_batch_create: negative count");
    for (int i = 0; i < n_src; ++i) {
        if (src_len[i] < 1 || src_len[i] > (int64_t)INT32_MAX - kDM)
            return fail(HRIR_EINVAL, "dense_batch_create: src_len[%d] out of range", i);
        if (src_off[i] < 0) return fail(HRIR_EINVAL, "dense_batch_create: src_off[%d] < 0", i);
    }
    auto* b = new (std::nothrow) hrir_dense_batch;
    if (!b) return fail(HRIR_ENOMEM, "dense_batch_create: out of host memory");
    b->plan = plan;
    b->n_jobs = n_jobs;
    std::vector<int> order(n_jobs);
    for (int j = 0; j < n_jobs; ++j) {
        if (jobs[j].src < 0 || jobs[j].src >= n_src || jobs[j].filt < 0 || jobs[j].filt >= plan->n_filters ||
            jobs[j].out_off < 0) {
            delete b;
            return fail(HRIR_EINVAL, "dense_batch_create: job %d out of range", j);
        }
        order[j] = j;
        const int s = jobs[j].src;
        b->src_extent = std::max(b->src_extent, src_off[s] + src_len[s]);
        b->out_extent = std::max(b->out_extent, jobs[j].out_off + src_len[s] + plan->m - 1);
    }
    std::stable_sort(order.begin(), order.end(), [jobs](int a, int c) { return jobs[a].src < jobs[c].src; });
    std::vector<JobDesc> hj(n_jobs);
    for (int j = 0; j < n_jobs; ++j) hj[j] = JobDesc{jobs[order[j]].out_off, jobs[order[j]].filt, 0};
    std::vector<DTile> ht;
    for (int j0 = 0; j0 < n_jobs;) {
        const int s = jobs[order[j0]].src;
        int j1 = j0;
        while (j1 < n_jobs && jobs[order[j1]].src == s) ++j1;
        const int64_t out_len = src_len[s] + plan->m - 1;
        for (int g0 = j0; g0 < j1; g0 += kDGroup)
            for (int64_t t0 = 0; t0 < out_len; t0 += kDTile)
                ht.push_back(DTile{src_off[s], (int32_t)src_len[s], (int32_t)out_len, (int32_t)t0, g0,
                                   std::min(kDGroup, j1 - g0), 0});
        j0 = j1;
    }
    b->n_tiles = (int64_t)ht.size();
    hipError_t e = hipSuccess;
    if (n_jobs > 0) {
        e = hipMalloc(&b->d_tiles, ht.size() * sizeof(DTile));
        if (e == hipSuccess) e = hipMalloc(&b->d_jobs, hj.size() * sizeof(JobDesc));
        if (e == hipSuccess) e = hipMemcpy(b->d_tiles, ht.data(), ht.size() * sizeof(DTile), hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(b->d_jobs, hj.data(), hj.size() * sizeof(JobDesc), hipMemcpyHostToDevice);
        if (e == hipSuccess)
            e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_dense), hipFuncAttributeMaxDynamicSharedMemorySize,
                                    (int)(sizeof(float) * dense_lds_floats()));
    }
    if (e != hipSuccess) {
        (void)hipFree(b->d_tiles);
        (void)hipFree(b->d_jobs);
        delete b;
        return fail(e == hipErrorOutOfMemory ? HRIR_ENOMEM : HRIR_EDEVICE, "dense_batch_create: %s",
                    hipGetErrorString(e));
    }
    *out = b;
    return HRIR_OK;
}

extern "C" int dense_batch_render(hrir_dense_batch* b, const float* d_src, int64_t src_elems, float* d_out,
                                  int64_t out_elems, void* stream) {
    clear_error();
    if (!b) return fail(HRIR_EINVAL, "dense_batch_render: null batch");
    if (b->n_jobs == 0) return HRIR_OK;
    if (!d_src || !d_out) return fail(HRIR_EINVAL, "dense_batch_render: null device pointer");
    if (src_elems < b->src_extent || out_elems < b->out_extent)
        return fail(HRIR_EINVAL, "dense_batch_render: buffers too small (src %lld < %lld or out %lld < %lld)",
                    (long long)src_elems, (long long)b->src_extent, (long long)out_elems, (long long)b->out_extent);
    hipLaunchKernelGGL(k_dense, dim3((unsigned)b->n_tiles), dim3(kThreads), sizeof(float) * dense_lds_floats(),
                       reinterpret_cast<hipStream_t>(stream), d_src, b->d_tiles, b->d_jobs, b->plan->d_h, d_out);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(HRIR_EDEVICE, "dense_batch_render: %s", hipGetErrorString(e));
    return HRIR_OK;
}

extern "C" void dense_batch_destroy(hrir_dense_batch* b) {
    if (!b) return;
    (void)hipFree(b->d_tiles);
    (void)hipFree(b->d_jobs);
    delete b;
}
