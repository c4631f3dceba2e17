// Moving sources and the device-side top-K that feeds them.
//
// A moving source changes direction every seg_len samples: output sample t of
// ear e uses the filter of segment j = min(t / seg_len, n_seg - 1), and over
// the first `fade` samples of a segment (j >= 1) it blends linearly from the
// previous segment's filter,
//     y[t] = a (g_j * z)[t] + (1 - a) (g_{j-1} * z)[t],  a = (u + 1) / fade,
// u = t - j seg_len, with z = r * s once per source (Eq. (2)).  Filters are
// rows of a plan's tap table; spconv_plan_topk writes rows of that table on
// the device from dense predictions (the surrogate network's outputs), so a
// predicted filter never leaves the GPU.
//
// Kernel: the quad tile of render_quad.h (one source, TB outputs, z as four
// shifted LDS copies) and work items of NJ x 256 outputs x one ear (NJ quads
// per lane, 256 outputs apart); seg_len and TB are multiples of NJ x 256, so
// an item lies inside one segment and only an item that starts a segment
// blends, over its first `fade` outputs (fade <= 256), one output per lane.
// Taps come from a table the device forms from the plan's rows (offsets into
// the quad copies, then gains; formed again after the library rewrites
// rows), read with scalar loads: a tap costs one address add and NJ 16-byte
// z reads for 4 NJ fmas, with the gain a scalar operand.  z is formed by the
// direct stage (FIR windows read from global memory, one barrier).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <type_traits>
#include <vector>

#include "hrir_internal.h"
#include "render_common.h"
#include "render_quad.h"

namespace hrir {

constexpr int kMovItem = 256;     // outputs per work item (one quad per lane)

// A filter's taps as the kernel reads them: KP offsets into the quad copies
// (tap position p reads copy c = (H - p) mod 4 at element c CS + H - p - c,
// where z at output t - p sits for the quad starting at output t), then the
// KP gains.  Formed on the device for every row of the plan by the first
// render and again by the first render after the library rewrites rows
// (spconv_plan_topk), so rows predicted on the device are seen.
template <int KP>
__global__ __launch_bounds__(256) void k_moving_taps(const int* __restrict__ P, const float* __restrict__ Gv,
                                                     int n_filters, int H, int CS, int* __restrict__ tbl) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n_filters * KP) return;
    const int f = i / KP, q = i % KP;
    const int p = P[i];
    const int c = (H - p) & 3;
    tbl[f * 2 * KP + q] = c * CS + H - p - c;
    tbl[f * 2 * KP + KP + q] = __float_as_int(Gv[i]);
}

// The tap table as a constant-address-space pointer: loads through it at
// wave-uniform addresses become scalar loads into SGPRs, so offsets and
// gains feed the LDS addresses and the fmas as scalar operands, with no
// LDS staging and no lane-to-scalar moves.  The table and the segment
// filters do not change while the render kernel runs.
template <class T>
using cptr = const __attribute__((address_space(4))) T*;
template <class T>
__device__ __forceinline__ cptr<T> as_const(const T* p) {
    return (cptr<T>)p;
}

// acc[jj][i] += g_k z[t - p_k] over the filter's KP taps, in tap order, for
// this lane's NJ quads (256 outputs apart): one aligned 16-byte LDS read per
// quad and tap at zo + offset (zo: the lane's first quad).  Taps in groups
// of 4; the empty asm (no instruction) over the accumulators and zo makes
// the next group's reads depend on this group's fmas, so they are not all
// hoisted and in flight at once (4 VGPRs per quad and tap).
template <int KP, int NJ>
__device__ __forceinline__ void gather_taps(const float* lds, int zo, cptr<int> T, float (&acc)[NJ][4]) {
    static_assert(KP % 4 == 0, "taps come in groups of 4");
    const cptr<float> G = reinterpret_cast<cptr<float>>(T + KP);
#pragma unroll
    for (int q0 = 0; q0 < KP; q0 += 4) {
        float4 v[4][NJ];
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int jj = 0; jj < NJ; ++jj)
                v[u][jj] = *reinterpret_cast<const float4*>(lds + zo + T[q0 + u] + 256 * jj);
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int jj = 0; jj < NJ; ++jj) {
                const float g = G[q0 + u];
                acc[jj][0] = fmaf(g, v[u][jj].x, acc[jj][0]);
                acc[jj][1] = fmaf(g, v[u][jj].y, acc[jj][1]);
                acc[jj][2] = fmaf(g, v[u][jj].z, acc[jj][2]);
                acc[jj][3] = fmaf(g, v[u][jj].w, acc[jj][3]);
            }
#pragma unroll
        for (int jj = 0; jj < NJ; ++jj)
            asm volatile("" : "+v"(acc[jj][0]), "+v"(acc[jj][1]), "+v"(acc[jj][2]), "+v"(acc[jj][3]), "+v"(zo));
    }
}

template <int LFP, int KP, int NJ>
__global__ __launch_bounds__(kQThreads, 4) void k_render_moving(const float* __restrict__ src,
                                                                const TileDesc* __restrict__ tiles,
                                                                const int32_t* __restrict__ seg_filt, int n_seg,
                                                                int seg_len, int fade, const float* __restrict__ r,
                                                                const int* __restrict__ taps,
                                                                float* __restrict__ out, int64_t out_stride, int lg,
                                                                int TB) {
    constexpr int IL = NJ * kMovItem;                            // outputs per work item
    extern __shared__ float4 smem4[];
    float* lds = reinterpret_cast<float*>(smem4);
    const TileDesc td = tiles[blockIdx.x];
    const int tid = threadIdx.x;
    const int s = td.job_begin;                                  // source index
    const int tile_len = min(TB, td.out_len - td.t0);
    const cptr<int32_t> sf = as_const(seg_filt) + (int64_t)s * n_seg * 2;
    const cptr<int> tc = as_const(taps);
    quad_stage_direct<LFP>(td, src, r, lg, TB, lds, tid);
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
    const int n_items = 2 * ((tile_len + IL - 1) / IL);
    for (int it = wave; it < n_items; it += kQWaves) {
        const int e = it & 1, blk = it >> 1;
        const int t_blk = td.t0 + IL * blk;
        const int j_raw = t_blk / seg_len;
        const int j = min(j_raw, n_seg - 1);
        float acc[NJ][4];
#pragma unroll
        for (int jj = 0; jj < NJ; ++jj) acc[jj][0] = acc[jj][1] = acc[jj][2] = acc[jj][3] = 0.0f;
        gather_taps<KP, NJ>(lds, IL * blk + 4 * lane, tc + (int64_t)sf[2 * j + e] * 2 * KP, acc);
        if (fade > 0 && j_raw == j && j >= 1 && t_blk == j * seg_len) {
            // The previous segment's filter over the first `fade` outputs, one
            // output u per lane: offset o reads element IL blk + u + o, z at
            // output t_blk + u - p, consecutive lanes on consecutive banks.
            // Then each value moves to the lane that holds its output: lane
            // L's outputs 4L + i, i < 4, are output (4L + i) mod 64 of pass
            // L / 16.  Each output is the fma chain in tap order that the quad
            // gather forms.
            const cptr<int> T0 = tc + (int64_t)sf[2 * (j - 1) + e] * 2 * KP;
            const cptr<float> G0 = reinterpret_cast<cptr<float>>(T0 + KP);
            float prev[4] = {0.0f, 0.0f, 0.0f, 0.0f};
            for (int m = 0; 64 * m < fade; ++m) {
                const float* zu = lds + IL * blk + 64 * m + lane;
                float y = 0.0f;
#pragma unroll
                for (int q = 0; q < KP; ++q) y = fmaf(G0[q], zu[T0[q]], y);
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const float v = __shfl(y, (4 * lane + i) & 63);
                    if ((lane >> 4) == m) prev[i] = v;
                }
            }
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int u = 4 * lane + i;
                if (u < fade) {
                    // one rounding order in every instantiation: (1 - a) y0, then fma
                    const float a = (float)(u + 1) / (float)fade;
                    const float b = (1.0f - a) * prev[i];
                    acc[0][i] = fmaf(a, acc[0][i], b);
                }
            }
        }
#pragma unroll
        for (int jj = 0; jj < NJ; ++jj) {
            float* orow = out + ((int64_t)s * 2 + e) * out_stride + t_blk + kMovItem * jj;
            const int lim = tile_len - IL * blk - kMovItem * jj;
            if (lim >= kMovItem && ((reinterpret_cast<uintptr_t>(orow) & 15) == 0)) {
                *reinterpret_cast<float4*>(orow + 4 * lane) =
                    make_float4(acc[jj][0], acc[jj][1], acc[jj][2], acc[jj][3]);
            } else {
#pragma unroll
                for (int i = 0; i < 4; ++i)
                    if (4 * lane + i < lim) orow[4 * lane + i] = acc[jj][i];
            }
        }
    }
}

// One wave per row: the k largest finite positive entries of dense[row][0..width),
// ties to the lower position, written in ascending position order to the tap
// table rows first + row, padded with (0, 0).
constexpr int kTopkPer = 32;      // entries per lane: width <= 2048
__global__ __launch_bounds__(64) void k_topk(const float* __restrict__ dense, int64_t row_stride, int width,
                                             int n_rows, int k, int kp, int first, int* __restrict__ P,
                                             float* __restrict__ Gv) {
    const int row = blockIdx.x;
    if (row >= n_rows) return;
    const int lane = threadIdx.x;
    const float* d = dense + (int64_t)row * row_stride;
    float v[kTopkPer];
#pragma unroll
    for (int q = 0; q < kTopkPer; ++q) {
        const int j = q * 64 + lane;
        const float x = j < width ? d[j] : 0.0f;
        v[q] = (x > 0.0f && x < INFINITY) ? x : 0.0f;           // only finite positive entries are taps
    }
    int mine_pos = -1;                                           // the entry this lane holds after the loop
    float mine_val = 0.0f;
    int cnt = 0;
    for (int round = 0; round < k; ++round) {
        // this lane's best: largest value, lowest position among equals
        float bv = 0.0f;
        int bj = 1 << 30;
#pragma unroll
        for (int q = 0; q < kTopkPer; ++q) {
            const int j = q * 64 + lane;
            if (v[q] > bv) {
                bv = v[q];
                bj = j;
            }
        }
        // wave maximum by (value desc, position asc)
        for (int off = 32; off > 0; off >>= 1) {
            const float ov = __shfl_xor(bv, off);
            const int oj = __shfl_xor(bj, off);
            if (ov > bv || (ov == bv && oj < bj)) {
                bv = ov;
                bj = oj;
            }
        }
        if (!(bv > 0.0f)) break;                                 // no positive entry left
        if ((bj & 63) == lane) {                                 // the owner drops it
#pragma unroll
            for (int q = 0; q < kTopkPer; ++q)
                if (q == (bj >> 6)) v[q] = 0.0f;
        }
        if (lane == round) {
            mine_pos = bj;
            mine_val = bv;
        }
        ++cnt;
    }
    // ascending positions: rank of each selected entry among the selected
    int rank = 0;
    for (int q = 0; q < cnt; ++q) {
        const int oj = __shfl(mine_pos, q);
        rank += (oj < mine_pos) ? 1 : 0;
    }
    int* pr = P + (int64_t)(first + row) * kp;
    float* gr = Gv + (int64_t)(first + row) * kp;
    if (lane < cnt) {
        pr[rank] = mine_pos;
        gr[rank] = mine_val;
    }
    for (int q = cnt + lane; q < kp; q += 64) {
        pr[q] = 0;
        gr[q] = 0.0f;
    }
}

}  // namespace hrir

using namespace hrir;

extern "C" int spconv_plan_topk(hrir_plan* plan, int32_t first_row, const float* d_dense, int32_t n_rows,
                                int64_t row_stride, int32_t width, void* stream) {
    clear_error();
    if (!plan || (n_rows > 0 && !d_dense)) return fail(HRIR_EINVAL, "spconv_plan_topk: null pointer");
    const PlanView pv = plan_view(plan);
    if (n_rows < 0 || first_row < 0 || (int64_t)first_row + n_rows > pv.n_filters)
        return fail(HRIR_EINVAL, "spconv_plan_topk: rows [%d, %lld) outside the plan's %d filters", first_row,
                    (long long)first_row + n_rows, pv.n_filters);
    if (width < 1 || width > pv.lg || width > 64 * kTopkPer)
        return fail(HRIR_EINVAL, "spconv_plan_topk: width=%d outside [1, min(lg=%d, %d)]", width, pv.lg,
                    64 * kTopkPer);
    if (row_stride < width) return fail(HRIR_EINVAL, "spconv_plan_topk: row_stride < width");
    if (n_rows == 0) return HRIR_OK;
    hipLaunchKernelGGL(k_topk, dim3(n_rows), dim3(64), 0, reinterpret_cast<hipStream_t>(stream), d_dense, row_stride,
                       width, n_rows, pv.k, pv.kp, first_row, pv.d_p, pv.d_g);
    plan_rows_changed(plan);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(HRIR_EDEVICE, "spconv_plan_topk: %s", hipGetErrorString(e));
    return HRIR_OK;
}

struct hrir_moving {
    const hrir_plan* plan = nullptr;
    int n_src = 0, n_seg = 0, seg_len = 0, fade = 0, TB = 2048;
    int nj = 1;                                   // quads per lane and work item
    int64_t src_len = 0, out_len = 0;
    int64_t n_tiles = 0;
    size_t lds = 0;
    TileDesc* d_tiles = nullptr;
    int* d_taps = nullptr;                        // n_filters x 2 kp: quad-copy offsets, then gains
    uint64_t taps_gen = 0;                        // the plan's rows_gen the table was formed from
    hipEvent_t taps_ready = nullptr;              // recorded after the kernel that formed it
    int32_t* d_seg[2] = {nullptr, nullptr};     // double-buffered segment tables
    int32_t* h_seg[2] = {nullptr, nullptr};     // pinned staging
    // The segment table of a call is uploaded on its own stream, so the
    // upload overlaps the previous call's kernels: copied[b] (copy stream)
    // orders the kernels after it, read[b] (caller's stream) orders the next
    // upload into half b after the kernel that reads it.
    hipStream_t copy = nullptr;
    hipEvent_t copied[2] = {nullptr, nullptr};
    hipEvent_t read[2] = {nullptr, nullptr};
    int cur = 0;
};

namespace {

void free_moving(hrir_moving* m) {
    if (!m) return;
    (void)hipFree(m->d_tiles);
    (void)hipFree(m->d_taps);
    if (m->copy) (void)hipStreamDestroy(m->copy);
    if (m->taps_ready) (void)hipEventDestroy(m->taps_ready);
    for (int i = 0; i < 2; ++i) {
        (void)hipFree(m->d_seg[i]);
        (void)hipHostFree(m->h_seg[i]);
        if (m->copied[i]) (void)hipEventDestroy(m->copied[i]);
        if (m->read[i]) (void)hipEventDestroy(m->read[i]);
    }
    delete m;
}

template <class F>
int with_lf_k(int lfp, int kp, F&& f) {
#define HRIR_MCASE(L, K) \
    if (lfp == L && kp == K) return f(std::integral_constant<int, L>{}, std::integral_constant<int, K>{});
    HRIR_MCASE(16, 4) HRIR_MCASE(16, 8) HRIR_MCASE(16, 16) HRIR_MCASE(16, 32) HRIR_MCASE(16, 64)
    HRIR_MCASE(32, 4) HRIR_MCASE(32, 8) HRIR_MCASE(32, 16) HRIR_MCASE(32, 32) HRIR_MCASE(32, 64)
    HRIR_MCASE(64, 4) HRIR_MCASE(64, 8) HRIR_MCASE(64, 16) HRIR_MCASE(64, 32) HRIR_MCASE(64, 64)
#undef HRIR_MCASE
    return fail(HRIR_EINVAL, "no moving-source kernel for lf pad %d, k pad %d", lfp, kp);
}

}  // namespace

extern "C" int moving_create(const hrir_plan* plan, int32_t n_src, int64_t src_len, int32_t seg_len, int32_t fade,
                             int32_t tile, hrir_moving** out) {
    clear_error();
    if (!plan || !out) return fail(HRIR_EINVAL, "moving_create: null pointer");
    *out = nullptr;
    const PlanView pv = plan_view(plan);
    if (pv.n_res > 1) return fail(HRIR_EINVAL, "moving_create: the plan has %d resonance filters; moving sources use one", pv.n_res);
    if (n_src < 1) return fail(HRIR_EINVAL, "moving_create: n_src=%d < 1", n_src);
    if (src_len < 1 || src_len > (int64_t)1 << 30) return fail(HRIR_EINVAL, "moving_create: src_len out of range");
    if (seg_len < kMovItem || seg_len % kMovItem)
        return fail(HRIR_EINVAL, "moving_create: seg_len=%d must be a positive multiple of %d", seg_len, kMovItem);
    if (fade < 0 || fade > kMovItem) return fail(HRIR_EINVAL, "moving_create: fade=%d outside [0, %d]", fade, kMovItem);
    if (tile == 0) {
        // 3,072-sample tiles where three fit in a CU's LDS (counted in 1 KiB
        // granules), else 2,048 (four per CU, the wave limit): more outputs
        // resident per CU hide more of each tile's load -> FIR -> gather chain
        const int l3 = (int)sizeof(float) * lds_quad_len(3072, pv.lg, pv.lfp);
        tile = 3 * ((l3 + 1023) / 1024 * 1024) <= 160 * 1024 ? 3072 : 2048;
    }
    if (tile < kMovItem || tile % kMovItem || tile > kQuadTileMax)
        return fail(HRIR_EINVAL, "moving_create: tile=%d must be a multiple of %d in [%d, %d]", tile, kMovItem,
                    kMovItem, kQuadTileMax);
    auto* m = new (std::nothrow) hrir_moving;
    if (!m) return fail(HRIR_ENOMEM, "moving_create: out of host memory");
    m->plan = plan;
    m->n_src = n_src;
    m->src_len = src_len;
    m->seg_len = seg_len;
    m->fade = fade;
    m->TB = tile;
    m->nj = (seg_len % (2 * kMovItem) == 0 && tile % (2 * kMovItem) == 0) ? 2 : 1;
    m->n_seg = (int)((src_len + seg_len - 1) / seg_len);
    m->out_len = src_len + pv.lf + pv.lg - 2;
    m->lds = sizeof(float) * (size_t)lds_quad_len(m->TB, pv.lg, pv.lfp);
    std::vector<TileDesc> ht;
    for (int s = 0; s < n_src; ++s)
        for (int64_t t0 = 0; t0 < m->out_len; t0 += m->TB)
            ht.push_back(TileDesc{(int64_t)s * src_len, (int32_t)src_len, (int32_t)m->out_len, (int32_t)t0, s, 2, 0});
    m->n_tiles = (int64_t)ht.size();
    const size_t seg_bytes = sizeof(int32_t) * (size_t)n_src * m->n_seg * 2;
    hipError_t e = m->lds > 160 * 1024 ? hipErrorInvalidValue : hipSuccess;
    if (e == hipSuccess) e = hipMalloc(&m->d_tiles, ht.size() * sizeof(TileDesc));
    if (e == hipSuccess) e = hipMalloc(&m->d_taps, sizeof(int) * (size_t)pv.n_filters * 2 * pv.kp);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&m->copy, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&m->taps_ready, hipEventDisableTiming);
    if (e == hipSuccess)
        e = hipMemcpy(m->d_tiles, ht.data(), ht.size() * sizeof(TileDesc), hipMemcpyHostToDevice);
    for (int i = 0; i < 2 && e == hipSuccess; ++i) {
        e = hipMalloc(&m->d_seg[i], seg_bytes);
        if (e == hipSuccess) e = hipHostMalloc((void**)&m->h_seg[i], seg_bytes, hipHostMallocDefault);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&m->copied[i], hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&m->read[i], hipEventDisableTiming);
    }
    if (e == hipSuccess) {
        const int rc = with_lf_k(pv.lfp, pv.kp, [&](auto L, auto K) -> int {
            constexpr int LV = decltype(L)::value, KV = decltype(K)::value;
            const void* k = m->nj == 2 ? reinterpret_cast<const void*>(&k_render_moving<LV, KV, 2>)
                                       : reinterpret_cast<const void*>(&k_render_moving<LV, KV, 1>);
            e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)m->lds);
            return HRIR_OK;
        });
        if (rc) {
            free_moving(m);
            return rc;
        }
    }
    if (e != hipSuccess) {
        free_moving(m);
        return fail(e == hipErrorOutOfMemory ? HRIR_ENOMEM : HRIR_EDEVICE, "moving_create: %s",
                    hipGetErrorString(e));
    }
    *out = m;
    return HRIR_OK;
}

extern "C" int moving_render(hrir_moving* m, const float* d_src, int64_t src_elems, const int32_t* seg_filt,
                             float* d_out, int64_t out_stride, int64_t out_elems, void* stream) {
    clear_error();
    if (!m || !d_src || !seg_filt || !d_out) return fail(HRIR_EINVAL, "moving_render: null pointer");
    const PlanView pv = plan_view(m->plan);
    if (src_elems < (int64_t)m->n_src * m->src_len)
        return fail(HRIR_EINVAL, "moving_render: source buffer holds %lld < %lld samples", (long long)src_elems,
                    (long long)m->n_src * m->src_len);
    if (out_stride < m->out_len) return fail(HRIR_EINVAL, "moving_render: out_stride < %lld", (long long)m->out_len);
    if (out_elems < (2 * (int64_t)m->n_src - 1) * out_stride + m->out_len)
        return fail(HRIR_EINVAL, "moving_render: output buffer too small");
    const int64_t n_ent = (int64_t)m->n_src * m->n_seg * 2;
    for (int64_t i = 0; i < n_ent; ++i)
        if (seg_filt[i] < 0 || seg_filt[i] >= pv.n_filters)
            return fail(HRIR_EINVAL, "moving_render: segment filter %lld = %d outside [0, %d)", (long long)i,
                        seg_filt[i], pv.n_filters);
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const int b = m->cur;
    m->cur ^= 1;
    // the upload that last read the pinned half b has finished
    hipError_t e = hipEventSynchronize(m->copied[b]);
    if (e == hipSuccess) {
        std::memcpy(m->h_seg[b], seg_filt, sizeof(int32_t) * (size_t)n_ent);
        e = hipStreamWaitEvent(m->copy, m->read[b], 0);   // the kernel that last read d_seg[b]
    }
    if (e == hipSuccess)
        e = hipMemcpyAsync(m->d_seg[b], m->h_seg[b], sizeof(int32_t) * (size_t)n_ent, hipMemcpyHostToDevice,
                           m->copy);
    if (e == hipSuccess) e = hipEventRecord(m->copied[b], m->copy);
    if (e == hipSuccess) e = hipStreamWaitEvent(st, m->copied[b], 0);
    if (e != hipSuccess) return fail(HRIR_EDEVICE, "moving_render: %s", hipGetErrorString(e));
    int rc = with_lf_k(pv.lfp, pv.kp, [&](auto L, auto K) -> int {
        constexpr int LV = decltype(L)::value, KV = decltype(K)::value;
        const int H = pv.lg - 1;
        // the tap table, formed again only when the library has rewritten
        // the plan's rows since it was last formed
        if (pv.rows_gen != m->taps_gen) {
            hipLaunchKernelGGL((k_moving_taps<KV>), dim3((unsigned)((pv.n_filters * KV + 255) / 256)), dim3(256), 0,
                               st, pv.d_p, pv.d_g, pv.n_filters, H, quad_cs(m->TB, H), m->d_taps);
            e = hipEventRecord(m->taps_ready, st);
            if (e == hipSuccess) m->taps_gen = pv.rows_gen;
        } else {
            e = hipStreamWaitEvent(st, m->taps_ready, 0);
        }
        if (e != hipSuccess) return fail(HRIR_EDEVICE, "moving_render: %s", hipGetErrorString(e));
        if (m->nj == 2)
            hipLaunchKernelGGL((k_render_moving<LV, KV, 2>), dim3((unsigned)m->n_tiles), dim3(kQThreads), m->lds, st,
                               d_src, m->d_tiles, m->d_seg[b], m->n_seg, m->seg_len, m->fade, pv.d_r, m->d_taps,
                               d_out, out_stride, pv.lg, m->TB);
        else
            hipLaunchKernelGGL((k_render_moving<LV, KV, 1>), dim3((unsigned)m->n_tiles), dim3(kQThreads), m->lds, st,
                               d_src, m->d_tiles, m->d_seg[b], m->n_seg, m->seg_len, m->fade, pv.d_r, m->d_taps,
                               d_out, out_stride, pv.lg, m->TB);
        return HRIR_OK;
    });
    if (rc) return rc;
    e = hipGetLastError();
    if (e == hipSuccess) e = hipEventRecord(m->read[b], st);
    if (e != hipSuccess) return fail(HRIR_EDEVICE, "moving_render: %s", hipGetErrorString(e));
    return HRIR_OK;
}

extern "C" int moving_info(const hrir_moving* m, int64_t* info4) {
    clear_error();
    if (!m || !info4) return fail(HRIR_EINVAL, "moving_info: null pointer");
    info4[0] = m->n_seg;
    info4[1] = m->out_len;
    info4[2] = m->n_tiles;
    info4[3] = m->TB;
    return HRIR_OK;
}

extern "C" void moving_destroy(hrir_moving* m) {
    if (m) (void)hipDeviceSynchronize();
    free_moving(m);
}
