// Register-window sparse render kernel for gfx950.
//
// Built with the structurizer told to leave uniform regions alone: the tap
// dispatch below is a tree of scalar branches on a wave-uniform value, and
// structurizing it would add flow blocks whose phis shuffle the accumulators
// after every tap.
#include <hip/hip_runtime.h>

#include "hrir_internal.h"
#include "render_common.h"

namespace hrir {

// ---------------------------------------------------------------------------
// Register-window kernel (reflection length <= kHW + 1).
//
// Lane l of wave w owns kRW consecutive outputs of the tile and keeps the z
// values they can read, z[t - kHW .. t + kRW), in kWin VGPRs (kRW = 24 keeps
// window + accumulators at ~216 VGPRs: no spills, 2 waves per SIMD).  The window is
// loaded from LDS once per tile and then reused by every job of the tile, so
// the gather itself does no LDS traffic: tap (p, g) is kRW fmas reading
// window registers at static offsets, selected by a balanced binary tree of
// scalar branches on the wave-uniform p.  Results go through a per-wave LDS
// slab (lane-contiguous in, 16-byte lane-interleaved out) so that every
// global store instruction writes 1 KiB contiguously.
// ---------------------------------------------------------------------------
constexpr int kWin = kRW + kHW;          // window registers per lane (192)
constexpr int kSeg = 64 * kRW;           // outputs per wave pass (1536)
static_assert(kTileRW == kWaves * kSeg, "tile pass");
constexpr int kRowS = 36;                // slab row stride: 144 B, so 16 lanes cover all 64 banks
constexpr int kSlab = 64 * kRowS;        // per-wave transpose slab
static_assert(kRW % 4 == 0 && kRW <= kRowS && kSeg % 256 == 0, "slab layout");

template <int P>
__device__ __forceinline__ void tap_fma(float (&acc)[kRW], const float (&w)[kWin], float g) {
#pragma unroll
    for (int i = 0; i < kRW; ++i) acc[i] = fmaf(g, w[i + kHW - P], acc[i]);
    // Empty markers, distinct per position, that take the accumulators as
    // operands: the fmas of this case must finish inside it, so the compiler
    // cannot merge the cases into one dynamically indexed body (which would
    // move the window out of registers).
    asm volatile("; tap %12 lo"
                 : "+v"(acc[0]), "+v"(acc[1]), "+v"(acc[2]), "+v"(acc[3]), "+v"(acc[4]), "+v"(acc[5]),
                   "+v"(acc[6]), "+v"(acc[7]), "+v"(acc[8]), "+v"(acc[9]), "+v"(acc[10]), "+v"(acc[11])
                 : "i"(P));
    asm volatile("; tap %12 hi"
                 : "+v"(acc[12]), "+v"(acc[13]), "+v"(acc[14]), "+v"(acc[15]), "+v"(acc[16]), "+v"(acc[17]),
                   "+v"(acc[18]), "+v"(acc[19]), "+v"(acc[20]), "+v"(acc[21]), "+v"(acc[22]), "+v"(acc[23])
                 : "i"(P));
}

// Balanced binary dispatch on the wave-uniform tap position p in [LO, HI].
template <int LO, int HI>
__device__ __forceinline__ void tap_dispatch(int p, float (&acc)[kRW], const float (&w)[kWin], float g) {
    if constexpr (LO == HI) {
        tap_fma<LO>(acc, w, g);
    } else {
        constexpr int MID = (LO + HI) / 2;
        if (p <= MID) tap_dispatch<LO, MID>(p, acc, w, g);
        else tap_dispatch<MID + 1, HI>(p, acc, w, g);
    }
}

__host__ __device__ inline int lds_rw_len(int TB, int lfp) {
    const int s_len = round_up(TB + kHW, kZpt) + lfp + 4;
    const int a = s_len > kWaves * kSlab ? s_len : kWaves * kSlab;
    return a + round_up(TB + kHW, kZpt);
}

template <int LFP>
__device__ __forceinline__ void render_tile_rw(const TileDesc& td, const float* __restrict__ src,
                                               const JobDesc* __restrict__ jobs, const float* __restrict__ r,
                                               const int* __restrict__ P, const float* __restrict__ Gv,
                                               float* __restrict__ out, int kp, int k, int TB, float* lds) {
    const int s_len = round_up(TB + kHW, kZpt) + LFP + 4;
    float* s_win = lds;                                   // reused as transpose slabs after the FIR
    float* z_win = lds + (s_len > kWaves * kSlab ? s_len : kWaves * kSlab);
    stage_z<LFP>(td, src, r, kHW, TB, s_win, z_win);

    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int tile_len = min(TB, td.out_len - td.t0);
    float* slab = s_win + wave * kSlab;
    for (int seg = wave * kSeg; seg < tile_len; seg += kWaves * kSeg) {
        // window: w[u] = z_win[seg + kRW * lane + u] = z[t0 + seg + kRW * lane - kHW + u]
        float w[kWin];
        const float* zl = z_win + seg + kRW * lane;
#pragma unroll
        for (int u = 0; u < kWin; u += 4) {
            const float4 v = *reinterpret_cast<const float4*>(zl + u);
            w[u] = v.x; w[u + 1] = v.y; w[u + 2] = v.z; w[u + 3] = v.w;
        }
        const int seg_len = min(kSeg, tile_len - seg);
        for (int q = 0; q < td.job_count; ++q) {
            const JobDesc jd = jobs[td.job_begin + q];
            const int* pp = P + (int64_t)jd.filt * kp;
            const float* gg = Gv + (int64_t)jd.filt * kp;
            float acc[kRW];
#pragma unroll
            for (int i = 0; i < kRW; ++i) acc[i] = 0.0f;
            int pn = pp[0];
            float gn = gg[0];
#pragma unroll 1
            for (int j = 0; j < k; ++j) {
                const int pc = __builtin_amdgcn_readfirstlane(pn);
                const float gc = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(gn)));
                if (j + 1 < k) { pn = pp[j + 1]; gn = gg[j + 1]; }
                tap_dispatch<0, kHW>(pc, acc, w, gc);
            }
            // Lane index re-derived here through an opaque copy, so no
            // lane-dependent address stays live across the tap loop (the
            // window and accumulators already use ~232 VGPRs).
            int ln;
            asm volatile("" : "=v"(ln) : "0"(static_cast<int>(threadIdx.x & 63)));
            // lane-contiguous -> slab (row stride kRowS floats)
#pragma unroll
            for (int i = 0; i < kRW; i += 4)
                *reinterpret_cast<float4*>(slab + ln * kRowS + i) =
                    make_float4(acc[i], acc[i + 1], acc[i + 2], acc[i + 3]);
            // slab -> global: pass c writes outputs seg + 256 c + 4 lane + [0, 4);
            // every slab read is issued before the first store waits on one.
            constexpr int kPass = kSeg / 256;
            float4 v[kPass];
#pragma unroll
            for (int c = 0; c < kPass; ++c) {
                const int qo = 256 * c + 4 * ln;            // output index within the segment
                v[c] = *reinterpret_cast<const float4*>(slab + (qo / kRW) * kRowS + (qo % kRW));
            }
            float* orow = out + jd.out_off + td.t0 + seg;
            if (seg_len == kSeg && ((reinterpret_cast<uintptr_t>(orow) & 15) == 0)) {
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
}

template <int LFP>
__global__ __launch_bounds__(kThreads, 2) void k_render_rw(const float* __restrict__ src,
                                                           const TileDesc* __restrict__ tiles,
                                                           const JobDesc* __restrict__ jobs,
                                                           const float* __restrict__ r,
                                                           const int* __restrict__ P,
                                                           const float* __restrict__ Gv,
                                                           float* __restrict__ out, int kp, int k, int TB) {
    extern __shared__ float4 smem4[];
    const TileDesc td = tiles[blockIdx.x];
    render_tile_rw<LFP>(td, src, jobs, r, P, Gv, out, kp, k, TB, reinterpret_cast<float*>(smem4));
}

template <int LFP>
__global__ __launch_bounds__(kThreads, 2) void k_render_rw_persistent(const float* __restrict__ src,
                                                                      const TileDesc* __restrict__ tiles,
                                                                      int n_tiles,
                                                                      const JobDesc* __restrict__ jobs,
                                                                      const float* __restrict__ r,
                                                                      const int* __restrict__ P,
                                                                      const float* __restrict__ Gv,
                                                                      float* __restrict__ out, int kp, int k,
                                                                      int TB, int* __restrict__ ctr) {
    extern __shared__ float4 smem4[];
    __shared__ int s_next;
    for (;;) {
        if (threadIdx.x == 0) s_next = atomicAdd(&ctr[0], 1);
        __syncthreads();
        const int t = s_next;
        __syncthreads();
        if (t >= n_tiles) break;
        const TileDesc td = tiles[t];
        render_tile_rw<LFP>(td, src, jobs, r, P, Gv, out, kp, k, TB, reinterpret_cast<float*>(smem4));
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


int rw_lds_bytes(int TB, int lfp) { return (int)sizeof(float) * lds_rw_len(TB, lfp); }

template <class F>
static int with_lf(int lfp, F&& f) {
    if (lfp == 16) return f(std::integral_constant<int, 16>{});
    if (lfp == 32) return f(std::integral_constant<int, 32>{});
    if (lfp == 64) return f(std::integral_constant<int, 64>{});
    return fail(HRIR_EINVAL, "no register-window kernel for lf pad %d", lfp);
}

int rw_prepare(int lfp, size_t lds_bytes, bool persistent, int64_t n_tiles, int* grid) {
    return with_lf(lfp, [&](auto L) -> int {
        constexpr int LV = decltype(L)::value;
        const void* kt = reinterpret_cast<const void*>(&k_render_rw<LV>);
        const void* kpers = reinterpret_cast<const void*>(&k_render_rw_persistent<LV>);
        hipError_t e = hipFuncSetAttribute(kt, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes);
        if (e == hipSuccess)
            e = hipFuncSetAttribute(kpers, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes);
        if (e != hipSuccess) return fail(HRIR_EDEVICE, "rw_prepare: %s", hipGetErrorString(e));
        if (!persistent) {
            *grid = (int)n_tiles;
            return HRIR_OK;
        }
        int per_cu = 0, dev = 0, cus = 0;
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kpers, kThreads, lds_bytes);
        if (e == hipSuccess) e = hipGetDevice(&dev);
        if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        if (e != hipSuccess) return fail(HRIR_EDEVICE, "rw_prepare: %s", hipGetErrorString(e));
        *grid = (int)std::min<int64_t>((int64_t)std::max(per_cu, 1) * cus, std::max<int64_t>(n_tiles, 1));
        return HRIR_OK;
    });
}

int rw_launch(int lfp, bool persistent, int grid, size_t lds_bytes, hipStream_t st, const float* src,
              const TileDesc* tiles, int n_tiles, const JobDesc* jobs, const float* r, const int* P,
              const float* Gv, float* out, int kp, int k, int TB, int* ctr) {
    return with_lf(lfp, [&](auto L) -> int {
        constexpr int LV = decltype(L)::value;
        if (persistent)
            hipLaunchKernelGGL((k_render_rw_persistent<LV>), dim3(grid), dim3(kThreads), lds_bytes, st, src, tiles,
                               n_tiles, jobs, r, P, Gv, out, kp, k, TB, ctr);
        else
            hipLaunchKernelGGL((k_render_rw<LV>), dim3((unsigned)n_tiles), dim3(kThreads), lds_bytes, st, src, tiles,
                               jobs, r, P, Gv, out, kp, k, TB);
        return HRIR_OK;
    });
}

}  // namespace hrir
