// Partitioned (block) rendering with per-stream history resident on the
// device: the real-time form of the renderer (Sec. IV-F: time-domain
// partitioned convolution adds no latency and no memory overhead).
//
// Each stream owns a slot with the last LFP-1 source samples and the last
// lg-1 values of z.  One workgroup renders one block of one stream:
//     s_ext = [s history | block],  z_new = r * s_ext (FIR over the block),
//     z_ext = [z history | z_new],  out_e[t] = sum_k g_{e,k} z_ext[H + t - p_{e,k}]
// for both ears, then writes the last samples of s_ext and z_ext back to the
// slot.  Output sample t of the stream is emitted with input sample t; a
// flush block (zero input of lf + lg - 2 samples) emits the tail.  The FIR
// and the gather sum in the same order as the offline kernels, so any block
// split of a stream reproduces the offline render bit for bit.
#include <hip/hip_runtime.h>

#include <cstring>
#include <type_traits>
#include <vector>

#include "block_internal.h"
#include "render_common.h"

namespace hrir {

// One workgroup renders one job at a time; a persistent grid strides over
// the job table (count read from device memory), a plain grid has one
// workgroup per job.
template <int LFP, int KP>
__global__ __launch_bounds__(kThreads) void k_block(const float* __restrict__ in, const BJob* __restrict__ jobs,
                                                    const int32_t* __restrict__ count, int n_jobs,
                                                    float* __restrict__ hist, int hist_stride,
                                                    const float* __restrict__ r, const int* __restrict__ P,
                                                    const float* __restrict__ Gv, int kp, int lf, int lg,
                                                    float* __restrict__ out) {
    extern __shared__ float4 smem4[];
    float* s_ext = reinterpret_cast<float*>(smem4);                 // [LFP-1 + m]
    const int H = lg - 1, HS = LFP - 1;
    const int tid = threadIdx.x;
    const int nj = count ? *count : n_jobs;
    for (int ji = blockIdx.x; ji < nj; ji += gridDim.x) {
        const BJob j = jobs[ji];
        const bool flush = (j.flags & kJobFlush) != 0;
        const int m = flush ? lf + lg - 2 : j.n;                    // samples in and out
        float* z_ext = s_ext + round_up(HS + m, 4);                  // [H + m]
        float* hs = hist + (int64_t)j.slot * hist_stride;           // s history then z history
        float* hz = hs + HS;
        for (int i = tid; i < HS; i += kThreads) s_ext[i] = hs[i];
        for (int i = tid; i < m; i += kThreads) s_ext[HS + i] = flush ? 0.0f : in[j.in_off + i];
        for (int i = tid; i < H; i += kThreads) z_ext[i] = hz[i];
        __syncthreads();
        // z_ext[H + u] = sum_n r[n] s_ext[HS + u - n], n ascending (the offline order)
        for (int u = tid; u < m; u += kThreads) {
            float acc = 0.0f;
#pragma unroll
            for (int n = 0; n < LFP; ++n) acc = fmaf(r[n], s_ext[HS + u - n], acc);
            z_ext[H + u] = acc;
        }
        __syncthreads();
        // both ears; taps in slot order (padding taps beyond k have gain 0)
        int pl[KP], pr[KP];
        float gl[KP], gr[KP];
#pragma unroll
        for (int q = 0; q < KP; ++q) {
            pl[q] = P[(int64_t)j.filt_l * kp + q];
            gl[q] = Gv[(int64_t)j.filt_l * kp + q];
            pr[q] = P[(int64_t)j.filt_r * kp + q];
            gr[q] = Gv[(int64_t)j.filt_r * kp + q];
        }
        for (int t = tid; t < m; t += kThreads) {
            float al = 0.0f, ar = 0.0f;
#pragma unroll
            for (int q = 0; q < KP; ++q) {
                al = fmaf(gl[q], z_ext[H + t - pl[q]], al);
                ar = fmaf(gr[q], z_ext[H + t - pr[q]], ar);
            }
            out[j.out_off + t] = al;
            out[j.out_off + m + t] = ar;
        }
        // new histories: the last HS samples of s_ext and H values of z_ext,
        // or zeros when the stream ends here
        const bool reset = (j.flags & kJobReset) != 0;
        for (int i = tid; i < HS; i += kThreads) hs[i] = reset ? 0.0f : s_ext[m + i];
        for (int i = tid; i < H; i += kThreads) hz[i] = reset ? 0.0f : z_ext[m + i];
        __syncthreads();                                            // LDS is reused by the next job
    }
}

// Zero the histories of the listed slots (a fill kernel, so the call is safe
// to capture in a graph).
__global__ void k_block_reset(float* __restrict__ hist, int hist_stride, const int32_t* __restrict__ slots, int n) {
    const int i = blockIdx.x;
    if (i >= n) return;
    float* h = hist + (int64_t)slots[i] * hist_stride;
    for (int e = threadIdx.x; e < hist_stride; e += blockDim.x) h[e] = 0.0f;
}

}  // namespace hrir

using namespace hrir;

struct hrir_plan;  // defined in render.hip; accessed through spconv_plan_device

extern "C" int spconv_plan_device(const hrir_plan* plan, const float** r, const int** p, const float** g,
                                  int32_t* lfp_kp_nf3);

struct hrir_streams {
    const hrir_plan* plan = nullptr;
    int lf = 0, lfp = 0, k = 0, kp = 0, lg = 0, n_filters = 0;
    int max_streams = 0, hist_stride = 0, n_filt = 0, device = 0;
    int call_id = 0;
    float* d_hist = nullptr;
    // job tables (double buffered) in pinned, coherent host memory that the
    // kernel reads in place: a launch needs no copy command before it
    BJob* h_jobs[2] = {nullptr, nullptr};
    BJob* d_jobs[2] = {nullptr, nullptr};   // device addresses of h_jobs
    int32_t* h_slots = nullptr;
    int32_t* d_slots = nullptr;
    hipEvent_t slots_used = nullptr;     // after the last reset kernel (reads d_slots)
    hipEvent_t used[2] = {nullptr, nullptr};
    int cap = 0, cur = 0;
    std::vector<int> seen;               // per-call uniqueness check
};

namespace hrir {

BlockShape block_shape(const hrir_streams* s) {
    return BlockShape{s->lf, s->lfp, s->k, s->kp, s->lg, s->n_filt, s->max_streams, s->hist_stride, s->device};
}

size_t block_lds_bytes(const BlockShape& sh, int max_m) {
    return sizeof(float) * (size_t)(round_up(sh.lfp - 1 + max_m, 4) + sh.lg - 1 + max_m);
}

hipError_t block_enqueue(const hrir_streams* s, const float* d_in, const BJob* d_jobs, const int32_t* d_count,
                         int n_jobs, int grid, int max_m, float* d_out, hipStream_t st) {
    const float* dr;
    const int* dp;
    const float* dg;
    int32_t lk[3];
    if (spconv_plan_device(s->plan, &dr, &dp, &dg, lk) != HRIR_OK) return hipErrorInvalidValue;
    const size_t lds = block_lds_bytes(block_shape(s), max_m);
    bool launched = false;
    auto go = [&](auto L, auto K) {
        constexpr int LV = decltype(L)::value, KV = decltype(K)::value;
        if (s->lfp == LV && s->kp == KV) {
            hipLaunchKernelGGL((k_block<LV, KV>), dim3(grid), dim3(kThreads), lds, st, d_in, d_jobs, d_count, n_jobs,
                               s->d_hist, s->hist_stride, dr, dp, dg, s->kp, s->lf, s->lg, d_out);
            launched = true;
        }
    };
    using I16 = std::integral_constant<int, 16>;
    using I32 = std::integral_constant<int, 32>;
    using I64 = std::integral_constant<int, 64>;
    using K4 = std::integral_constant<int, 4>;
    using K8 = std::integral_constant<int, 8>;
    go(I16{}, K4{}); go(I16{}, K8{}); go(I16{}, I16{}); go(I16{}, I32{}); go(I16{}, I64{});
    go(I32{}, K4{}); go(I32{}, K8{}); go(I32{}, I16{}); go(I32{}, I32{}); go(I32{}, I64{});
    go(I64{}, K4{}); go(I64{}, K8{}); go(I64{}, I16{}); go(I64{}, I32{}); go(I64{}, I64{});
    if (!launched) return hipErrorInvalidConfiguration;
    return hipGetLastError();
}

}  // namespace hrir

namespace {

void free_streams(hrir_streams* s) {
    if (!s) return;
    (void)hipFree(s->d_hist);
    for (int i = 0; i < 2; ++i) {
        (void)hipHostFree(s->h_jobs[i]);
        if (s->used[i]) (void)hipEventDestroy(s->used[i]);
    }
    (void)hipHostFree(s->h_slots);
    (void)hipFree(s->d_slots);
    if (s->slots_used) (void)hipEventDestroy(s->slots_used);
    delete s;
}

}  // namespace

extern "C" int block_streams_create(const hrir_plan* plan, int32_t max_streams, hrir_streams** out) {
    clear_error();
    if (!plan || !out) return fail(HRIR_EINVAL, "block_streams_create: null pointer");
    *out = nullptr;
    if (max_streams < 1 || max_streams > (1 << 20))
        return fail(HRIR_EINVAL, "block_streams_create: max_streams=%d outside [1, 2^20]", max_streams);
    int32_t shp[3], lk[3];
    const float* dr;
    const int* dp;
    const float* dg;
    int rc = spconv_plan_shape(plan, shp);
    if (rc) return rc;
    if (plan_view(plan).n_res > 1)
        return fail(HRIR_EINVAL, "block_streams_create: the plan has %d resonance filters; block rendering uses one",
                    plan_view(plan).n_res);
    rc = spconv_plan_device(plan, &dr, &dp, &dg, lk);
    if (rc) return rc;
    auto* s = new (std::nothrow) hrir_streams;
    if (!s) return fail(HRIR_ENOMEM, "block_streams_create: out of host memory");
    s->plan = plan;
    s->lf = shp[0]; s->k = shp[1]; s->lg = shp[2]; s->lfp = lk[0]; s->kp = lk[1]; s->n_filt = lk[2];
    s->max_streams = max_streams;
    hipError_t e0 = hipGetDevice(&s->device);
    if (e0 != hipSuccess) {
        delete s;
        return fail(HRIR_EDEVICE, "block_streams_create: %s", hipGetErrorString(e0));
    }
    s->hist_stride = round_up(s->lfp - 1 + s->lg - 1, 4);
    s->cap = max_streams;
    hipError_t e = hipMalloc(&s->d_hist, (size_t)max_streams * s->hist_stride * sizeof(float));
    for (int i = 0; i < 2 && e == hipSuccess; ++i) {
        e = hipHostMalloc(&s->h_jobs[i], (size_t)s->cap * sizeof(BJob), hipHostMallocMapped | hipHostMallocCoherent);
        if (e == hipSuccess) e = hipHostGetDevicePointer(reinterpret_cast<void**>(&s->d_jobs[i]), s->h_jobs[i], 0);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&s->used[i], hipEventDisableTiming);
    }
    if (e == hipSuccess) e = hipHostMalloc(&s->h_slots, (size_t)max_streams * sizeof(int32_t), hipHostMallocDefault);
    if (e == hipSuccess) e = hipMalloc(&s->d_slots, (size_t)max_streams * sizeof(int32_t));
    if (e == hipSuccess) e = hipEventCreateWithFlags(&s->slots_used, hipEventDisableTiming);
    if (e == hipSuccess) {
        // all histories start at zero
        for (int i = 0; i < max_streams; ++i) s->h_slots[i] = i;
        e = hipMemcpy(s->d_slots, s->h_slots, (size_t)max_streams * sizeof(int32_t), hipMemcpyHostToDevice);
        if (e == hipSuccess) {
            hipLaunchKernelGGL(k_block_reset, dim3(max_streams), dim3(64), 0, 0, s->d_hist, s->hist_stride, s->d_slots,
                               max_streams);
            e = hipDeviceSynchronize();
        }
    }
    if (e != hipSuccess) {
        free_streams(s);
        return fail(e == hipErrorOutOfMemory ? HRIR_ENOMEM : HRIR_EDEVICE, "block_streams_create: %s",
                    hipGetErrorString(e));
    }
    s->seen.assign(max_streams, -1);
    *out = s;
    return HRIR_OK;
}

extern "C" void block_streams_destroy(hrir_streams* s) {
    if (s) (void)hipDeviceSynchronize();
    free_streams(s);
}

extern "C" int block_streams_reset(hrir_streams* s, const int32_t* slots, int32_t n, void* stream) {
    clear_error();
    if (!s || (n > 0 && !slots)) return fail(HRIR_EINVAL, "block_streams_reset: null pointer");
    if (n < 0 || n > s->max_streams) return fail(HRIR_EINVAL, "block_streams_reset: n=%d out of range", n);
    if (n == 0) return HRIR_OK;
    for (int i = 0; i < n; ++i)
        if (slots[i] < 0 || slots[i] >= s->max_streams)
            return fail(HRIR_EINVAL, "block_streams_reset: slot %d out of range", slots[i]);
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    // the slot lists (host staging and device copy) are free once the last
    // reset kernel, on whatever stream, has run
    hipError_t e = hipEventSynchronize(s->slots_used);
    if (e == hipSuccess) {
        std::memcpy(s->h_slots, slots, sizeof(int32_t) * n);
        e = hipMemcpyAsync(s->d_slots, s->h_slots, sizeof(int32_t) * n, hipMemcpyHostToDevice, st);
    }
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_block_reset, dim3(n), dim3(64), 0, st, s->d_hist, s->hist_stride, s->d_slots, n);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipEventRecord(s->slots_used, st);
    if (e != hipSuccess) return fail(HRIR_EDEVICE, "block_streams_reset: %s", hipGetErrorString(e));
    return HRIR_OK;
}

extern "C" int block_render(hrir_streams* s, const float* d_in, int64_t in_elems, const block_job* jobs,
                            int32_t n_jobs, float* d_out, int64_t out_elems, void* stream) {
    clear_error();
    if (!s || (n_jobs > 0 && (!jobs || !d_out))) return fail(HRIR_EINVAL, "block_render: null pointer");
    if (n_jobs < 0 || n_jobs > s->max_streams) return fail(HRIR_EINVAL, "block_render: n_jobs=%d out of range", n_jobs);
    if (n_jobs == 0) return HRIR_OK;
    const int call_id = ++s->call_id;
    const int tail = s->lf + s->lg - 2;
    int max_m = 0;
    for (int i = 0; i < n_jobs; ++i) {
        const block_job& j = jobs[i];
        if (j.stream_id < 0 || j.stream_id >= s->max_streams)
            return fail(HRIR_EINVAL, "block_render: job %d stream %d out of range", i, j.stream_id);
        if (s->seen[j.stream_id] == call_id)
            return fail(HRIR_EINVAL, "block_render: stream %d appears twice in one call", j.stream_id);
        s->seen[j.stream_id] = call_id;
        if (j.filt_l < 0 || j.filt_l >= s->n_filt || j.filt_r < 0 || j.filt_r >= s->n_filt)
            return fail(HRIR_EINVAL, "block_render: job %d filter out of range", i);
        const bool flush = (j.flags & BLOCK_FLUSH) != 0;
        if (j.flags & ~BLOCK_FLUSH) return fail(HRIR_EINVAL, "block_render: job %d unknown flags", i);
        const int m = flush ? tail : j.n;
        if (!flush && (j.n < 1 || j.n > kBlockMax))
            return fail(HRIR_EINVAL, "block_render: job %d block length %d outside [1, %d]", i, j.n, kBlockMax);
        if (!flush && (j.in_off < 0 || !d_in || j.in_off + j.n > in_elems))
            return fail(HRIR_EINVAL, "block_render: job %d input outside the buffer", i);
        if (j.out_off < 0 || j.out_off + 2 * (int64_t)m > out_elems)
            return fail(HRIR_EINVAL, "block_render: job %d output outside the buffer", i);
        max_m = std::max(max_m, m);
    }
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const int b = s->cur;
    s->cur ^= 1;
    // this half of the job table is free once the kernel that last read it
    // (two calls ago) has finished
    hipError_t e = hipEventSynchronize(s->used[b]);
    if (e != hipSuccess) return fail(HRIR_EDEVICE, "block_render: %s", hipGetErrorString(e));
    for (int i = 0; i < n_jobs; ++i) {
        const block_job& j = jobs[i];
        s->h_jobs[b][i] = BJob{j.stream_id, j.n, j.filt_l, j.filt_r, (j.flags & BLOCK_FLUSH) ? kJobFlush : 0, 0,
                               j.in_off, j.out_off};
    }
    const float* din = d_in ? d_in : d_out;   // flush-only calls read no input
    e = block_enqueue(s, din, s->d_jobs[b], nullptr, n_jobs, n_jobs, max_m, d_out, st);
    if (e == hipSuccess) e = hipEventRecord(s->used[b], st);
    if (e != hipSuccess) return fail(HRIR_EDEVICE, "block_render: %s", hipGetErrorString(e));
    return HRIR_OK;
}
