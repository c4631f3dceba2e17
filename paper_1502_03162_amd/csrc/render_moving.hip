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
// blends, over its first quad (fade <= 256).  Taps are staged in LDS as
// offsets into the quad copies (c CS + H - p - c for position p, c = (H - p)
// mod 4) with their gains, read 4 at a time, so a tap costs one address add
// and NJ 16-byte z reads for 4 NJ fmas.
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

// Filters a tile can need: both ears of every segment it overlaps and of the
// segment before (its last samples fade into the tile's first segment).
__host__ __device__ inline int moving_tile_filters(int TB) { return 2 * (TB / kMovItem + 2); }
// The filter-row slots, rounded up so the tap arrays after them are 16-byte aligned.
__host__ __device__ inline int moving_row_slots(int TB) { return (moving_tile_filters(TB) + 3) / 4 * 4; }

// LDS floats after the z copies: filter rows, then their tap offsets and gains.
template <int KP>
__host__ __device__ inline int moving_tap_lds(int TB) {
    return moving_row_slots(TB) + 2 * KP * moving_tile_filters(TB);
}

// Empty asm over the accumulators that clobbers memory: LDS reads of the
// next group of taps are not hoisted above it (all of them in flight at once
// would take 4 VGPRs per tap and read and cost occupancy).  Emits no
// instruction.
template <int NJ>
__device__ __forceinline__ void pin_acc(float (&a)[NJ][4]) {
#pragma unroll
    for (int jj = 0; jj < NJ; ++jj)
        asm volatile("" : "+v"(a[jj][0]), "+v"(a[jj][1]), "+v"(a[jj][2]), "+v"(a[jj][3]) : : "memory");
}

// offs, gs: one filter's staged taps (LDS offsets into the quad copies and
// gains; 16-byte aligned, every lane reads the same words).  Taps in groups
// of 4 (KP is a multiple of 4), accumulated in tap order; the first NJ of
// the item's quads, 256 outputs apart.
template <int KP, int NJ, int NA>
__device__ __forceinline__ void quad_taps(const float* zl, const int* offs, const float* gs, float (&acc)[NA][4]) {
    static_assert(KP % 4 == 0, "taps come in groups of 4");
    static_assert(NJ <= NA, "accumulators for every quad");
#pragma unroll
    for (int q0 = 0; q0 < KP; q0 += 4) {
        const int4 o4 = *reinterpret_cast<const int4*>(offs + q0);
        const float4 g4 = *reinterpret_cast<const float4*>(gs + q0);
        // the same words for every lane: keep the taps in scalar registers
        const int o[4] = {__builtin_amdgcn_readfirstlane(o4.x), __builtin_amdgcn_readfirstlane(o4.y),
                          __builtin_amdgcn_readfirstlane(o4.z), __builtin_amdgcn_readfirstlane(o4.w)};
        const float g[4] = {__int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(g4.x))),
                            __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(g4.y))),
                            __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(g4.z))),
                            __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(g4.w)))};
        float4 v[4][NJ];
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int jj = 0; jj < NJ; ++jj) v[u][jj] = *reinterpret_cast<const float4*>(zl + o[u] + 256 * jj);
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int jj = 0; jj < NJ; ++jj) {
                acc[jj][0] = fmaf(g[u], v[u][jj].x, acc[jj][0]);
                acc[jj][1] = fmaf(g[u], v[u][jj].y, acc[jj][1]);
                acc[jj][2] = fmaf(g[u], v[u][jj].z, acc[jj][2]);
                acc[jj][3] = fmaf(g[u], v[u][jj].w, acc[jj][3]);
            }
        pin_acc<NA>(acc);
    }
}

template <int LFP, int KP, int NJ>
__global__ __launch_bounds__(kQThreads, 4) void k_render_moving(const float* __restrict__ src,
                                                                const TileDesc* __restrict__ tiles,
                                                                const int32_t* __restrict__ seg_filt, int n_seg,
                                                                int seg_len, int fade, const float* __restrict__ r,
                                                                const int* __restrict__ P,
                                                                const float* __restrict__ Gv,
                                                                float* __restrict__ out, int64_t out_stride, int lg,
                                                                int TB) {
    constexpr int IL = NJ * kMovItem;                            // outputs per work item
    extern __shared__ float4 smem4[];
    float* lds = reinterpret_cast<float*>(smem4);
    const TileDesc td = tiles[blockIdx.x];
    const int tid = threadIdx.x;
    const int s = td.job_begin;                                  // source index
    const int tile_len = min(TB, td.out_len - td.t0);
    const int H = lg - 1, CS = quad_cs(TB, H);
    // The tile's filters: segments j_lo .. j_hi, both ears.  Their rows are
    // read before the source is staged and their taps copied into LDS while
    // the source window is ready, so no work item waits on a chain of
    // global loads (segment -> filter row -> taps).
    const int j_first = min(td.t0 / seg_len, n_seg - 1);
    const int j_lo = max(j_first - 1, 0);
    const int j_hi = min((td.t0 + tile_len - 1) / seg_len, n_seg - 1);
    const int n_fl = 2 * (j_hi - j_lo + 1);
    const int64_t row = (int64_t)s * n_seg;
    int f_mine = 0;
    if (tid < n_fl) f_mine = seg_filt[(row + j_lo) * 2 + tid];
    int* lds_f = reinterpret_cast<int*>(lds + lds_quad_len(TB, lg, LFP));
    int* lds_o = lds_f + moving_row_slots(TB);
    float* lds_g = reinterpret_cast<float*>(lds_o + moving_tile_filters(TB) * KP);
    quad_stage<LFP>(td, src, r, lg, TB, lds, tid, [&]() {
        if (tid < n_fl) lds_f[tid] = f_mine;
        __syncthreads();
        for (int a = tid; a < n_fl * KP; a += kQThreads) {
            const int64_t o = (int64_t)lds_f[a / KP] * KP + a % KP;
            const int p = P[o];
            const int c = (H - p) & 3;
            lds_o[a] = c * CS + (H - p - c);
            lds_g[a] = Gv[o];
        }
    });
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
    const int n_items = 2 * ((tile_len + IL - 1) / IL);
    for (int it = wave; it < n_items; it += kQWaves) {
        const int e = it & 1, blk = it >> 1;
        const int t_blk = td.t0 + IL * blk;
        const int j_raw = t_blk / seg_len;
        const int j = min(j_raw, n_seg - 1);
        const int fi = 2 * (j - j_lo) + e;
        const float* zl = lds + IL * blk + 4 * lane;
        float acc[NJ][4];
#pragma unroll
        for (int jj = 0; jj < NJ; ++jj) acc[jj][0] = acc[jj][1] = acc[jj][2] = acc[jj][3] = 0.0f;
        quad_taps<KP, NJ>(zl, lds_o + fi * KP, lds_g + fi * KP, acc);
        if (fade > 0 && j_raw == j && j >= 1 && t_blk == j * seg_len && 4 * lane < fade) {
            // the previous segment's filter over the first quad (fade <= 256),
            // in the lanes whose outputs blend (the others skip its LDS reads;
            // the taps are the same words for every lane, so any active lane
            // gives them to readfirstlane)
            float acc0[1][4] = {{0.0f, 0.0f, 0.0f, 0.0f}};
            quad_taps<KP, 1>(zl, lds_o + (fi - 2) * KP, lds_g + (fi - 2) * KP, acc0);
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int u = 4 * lane + i;
                if (u < fade) {
                    // one rounding order in every instantiation: (1 - a) y0, then fma
                    const float a = (float)(u + 1) / (float)fade;
                    const float b = (1.0f - a) * acc0[0][i];
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
    int32_t* d_seg[2] = {nullptr, nullptr};     // double-buffered segment tables
    int32_t* h_seg[2] = {nullptr, nullptr};     // pinned staging
    hipEvent_t used[2] = {nullptr, nullptr};
    int cur = 0;
};

namespace {

void free_moving(hrir_moving* m) {
    if (!m) return;
    (void)hipFree(m->d_tiles);
    for (int i = 0; i < 2; ++i) {
        (void)hipFree(m->d_seg[i]);
        (void)hipHostFree(m->h_seg[i]);
        if (m->used[i]) (void)hipEventDestroy(m->used[i]);
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
    if (tile == 0) tile = 2560;     // 2048..4096 measured within 5 % for 2 rows per source
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
    const int rc_lds = with_lf_k(pv.lfp, pv.kp, [&](auto, auto K) -> int {
        m->lds = sizeof(float) * (size_t)(lds_quad_len(m->TB, pv.lg, pv.lfp) + moving_tap_lds<decltype(K)::value>(m->TB));
        return HRIR_OK;
    });
    if (rc_lds) {
        free_moving(m);
        return rc_lds;
    }
    std::vector<TileDesc> ht;
    for (int s = 0; s < n_src; ++s)
        for (int64_t t0 = 0; t0 < m->out_len; t0 += m->TB)
            ht.push_back(TileDesc{(int64_t)s * src_len, (int32_t)src_len, (int32_t)m->out_len, (int32_t)t0, s, 2, 0});
    m->n_tiles = (int64_t)ht.size();
    const size_t seg_bytes = sizeof(int32_t) * (size_t)n_src * m->n_seg * 2;
    hipError_t e = m->lds > 160 * 1024 ? hipErrorInvalidValue : hipSuccess;
    if (e == hipSuccess) e = hipMalloc(&m->d_tiles, ht.size() * sizeof(TileDesc));
    if (e == hipSuccess)
        e = hipMemcpy(m->d_tiles, ht.data(), ht.size() * sizeof(TileDesc), hipMemcpyHostToDevice);
    for (int i = 0; i < 2 && e == hipSuccess; ++i) {
        e = hipMalloc(&m->d_seg[i], seg_bytes);
        if (e == hipSuccess) e = hipHostMalloc((void**)&m->h_seg[i], seg_bytes, hipHostMallocDefault);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&m->used[i], hipEventDisableTiming);
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
    hipError_t e = hipEventSynchronize(m->used[b]);        // the copy that last read this half has run
    if (e == hipSuccess) {
        std::memcpy(m->h_seg[b], seg_filt, sizeof(int32_t) * (size_t)n_ent);
        e = hipMemcpyAsync(m->d_seg[b], m->h_seg[b], sizeof(int32_t) * (size_t)n_ent, hipMemcpyHostToDevice, st);
    }
    if (e == hipSuccess) e = hipEventRecord(m->used[b], st);
    if (e != hipSuccess) return fail(HRIR_EDEVICE, "moving_render: %s", hipGetErrorString(e));
    int rc = with_lf_k(pv.lfp, pv.kp, [&](auto L, auto K) -> int {
        constexpr int LV = decltype(L)::value, KV = decltype(K)::value;
        if (m->nj == 2)
            hipLaunchKernelGGL((k_render_moving<LV, KV, 2>), dim3((unsigned)m->n_tiles), dim3(kQThreads), m->lds, st,
                               d_src, m->d_tiles, m->d_seg[b], m->n_seg, m->seg_len, m->fade, pv.d_r, pv.d_p, pv.d_g,
                               d_out, out_stride, pv.lg, m->TB);
        else
            hipLaunchKernelGGL((k_render_moving<LV, KV, 1>), dim3((unsigned)m->n_tiles), dim3(kQThreads), m->lds, st,
                               d_src, m->d_tiles, m->d_seg[b], m->n_seg, m->seg_len, m->fade, pv.d_r, pv.d_p, pv.d_g,
                               d_out, out_stride, pv.lg, m->TB);
        return HRIR_OK;
    });
    if (rc) return rc;
    e = hipGetLastError();
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
