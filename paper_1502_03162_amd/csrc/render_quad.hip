// Quad LDS-gather sparse render kernel for gfx950 (the default render path).
//
// Same tiling as the other fused kernels (one source, TB outputs, a group of
// that source's (direction, ear) jobs per workgroup; z formed in LDS by the
// resonance FIR and shared by every job of the tile), but the z tile is kept
// as four copies shifted by 0..3 samples:
//     Zc[m] = z[t0 - H + m + c],   c = 0..3.
// Lane l of a wave owns outputs q = c0 + 4 l + 256 j + i (i < 4, j < 4) of
// a 1024-output chunk.  For a tap at position p the four outputs of a quad
// read z[t0 + q - p + i] = Zc[q + H - p - c + i] with c = (H - p) mod 4,
// and q + H - p - c is a multiple of 4: one aligned 16-byte LDS read feeds 4
// fmas, and the lanes of a wave read 1 KiB of consecutive LDS (no bank
// conflicts).  The quad layout also makes every global store 16 bytes per
// lane, 1 KiB per wave instruction.
//
// The FIR keeps its z values in registers across a barrier, so the copies
// can overwrite the staged source: LDS per tile is 4 (TB + H) floats.
//
// Workgroups have 8 waves: with 4 tiles resident per CU (LDS-bound at
// TB = 2048) that is 32 waves per CU, enough outstanding stores and LDS reads
// to keep both pipes busy while some waves wait on the source reads of a new
// tile, which queue behind the output writes in HBM.
//
// Summation order per output: FIR taps 0..lf-1, then kept taps 0..K-1, one
// fma each into one accumulator -- the order of every other kernel, so the
// results are bitwise identical to theirs.
#include <hip/hip_runtime.h>

#include "hrir_internal.h"
#include "render_common.h"
#include "render_quad.h"

namespace hrir {

// Tiles with at least this many jobs stage their source at raised wave
// priority (measured: 2-3 % faster at 40 jobs per tile, slower at 1..16).
// A batch whose tiles all have fewer jobs runs the direct stage instead
// (FIR windows read from global memory, one barrier per tile instead of
// three): measured 3-5 % faster on the uneven workload and 2 % slower at 40
// jobs per tile, where its extra vector-memory loads compete with the
// tile's 40 row stores.
constexpr int kQPrioJobs = 24;

// DIRECT: the tile reads its FIR windows from global memory
// (quad_stage_direct); otherwise it stages the source window in LDS
// (quad_stage), at raised priority with at least kQPrioJobs jobs.
template <int LFP, int KP, int NT, bool DIRECT>
__device__ __forceinline__ void render_tile_quad(const TileDesc& td, const float* __restrict__ src,
                                                 const JobDesc* __restrict__ jobs, const float* __restrict__ r,
                                                 const int* __restrict__ P, const float* __restrict__ Gv,
                                                 float* __restrict__ out, int lg, int TB, float* lds, int tid) {
    constexpr int kWv = NT / 64;
    // both stages form the same z, bit for bit
    if (DIRECT)
        quad_stage_direct<LFP, NT>(td, src, r + (int64_t)td.res * LFP, lg, TB, lds, tid);
    else
        quad_stage<LFP, NT>(td, src, r + (int64_t)td.res * LFP, lg, TB, lds, tid, NoHook{},
                            td.job_count >= kQPrioJobs);
    const int H = lg - 1;
    const int CS = quad_cs(TB, H);
    const float* zc = lds;

    // gather.  With at least one job per wave, a wave renders whole jobs
    // (job q = wave, wave + 4, ..., every chunk of it) so a job's taps are
    // loaded once per tile; with fewer jobs the (job, chunk) pairs go
    // round-robin so that every wave has work.
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
    const int tile_len = min(TB, td.out_len - td.t0);
    const int nchunk = (tile_len + kQChunk - 1) / kQChunk;
    int pk[KP];
    float gk[KP];
    auto load_taps = [&](const JobDesc& jd) {
        const int* pp = P + (int64_t)jd.filt * KP;
        const float* gg = Gv + (int64_t)jd.filt * KP;
#pragma unroll
        for (int k = 0; k < KP; ++k) { pk[k] = pp[k]; gk[k] = gg[k]; }
    };
    auto render_chunk = [&](const JobDesc& jd, int ch) {
            float acc[kQR];
#pragma unroll
            for (int j = 0; j < kQR; ++j) acc[j] = 0.0f;
            const float* zl = zc + ch * kQChunk + 4 * lane;
            // Two-stage pipeline as in the other LDS kernel: reads of tap k+1 in
            // flight during the fmas of tap k; pin16 keeps the compiler from
            // hoisting every tap's reads.
            float4 zv[2][4];
            {
                const int c = (H - pk[0]) & 3;
                const float* a = zl + c * CS + (H - pk[0] - c);
#pragma unroll
                for (int j = 0; j < 4; ++j) zv[0][j] = *reinterpret_cast<const float4*>(a + 256 * j);
            }
#pragma unroll
            for (int k = 0; k < KP; ++k) {
                if (k + 1 < KP) {
                    const int c = (H - pk[k + 1]) & 3;
                    const float* a = zl + c * CS + (H - pk[k + 1] - c);
#pragma unroll
                    for (int j = 0; j < 4; ++j) zv[(k + 1) & 1][j] = *reinterpret_cast<const float4*>(a + 256 * j);
                }
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const float4 v = zv[k & 1][j];
                    acc[4 * j + 0] = fmaf(gk[k], v.x, acc[4 * j + 0]);
                    acc[4 * j + 1] = fmaf(gk[k], v.y, acc[4 * j + 1]);
                    acc[4 * j + 2] = fmaf(gk[k], v.z, acc[4 * j + 2]);
                    acc[4 * j + 3] = fmaf(gk[k], v.w, acc[4 * j + 3]);
                }
                pin16(acc);
            }
            float* orow = out + jd.out_off + td.t0 + ch * kQChunk;
            const int lim = tile_len - ch * kQChunk;    // valid outputs in this chunk (uniform)
            if (lim >= kQChunk && ((reinterpret_cast<uintptr_t>(orow) & 15) == 0)) {
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    *reinterpret_cast<float4*>(orow + 4 * lane + 256 * j) =
                        make_float4(acc[4 * j], acc[4 * j + 1], acc[4 * j + 2], acc[4 * j + 3]);
            } else {
#pragma unroll
                for (int j = 0; j < 4; ++j)
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const int qo = 4 * lane + 256 * j + i;
                        if (qo < lim) orow[qo] = acc[4 * j + i];
                    }
            }
    };
    if (td.job_count >= kWv) {
        for (int q = wave; q < td.job_count; q += kWv) {
            const JobDesc jd = jobs[td.job_begin + q];
            load_taps(jd);
            // one chunk body in the loop: unrolling it doubles the hot code
#pragma unroll 1
            for (int ch = 0; ch < nchunk; ++ch) render_chunk(jd, ch);
        }
    } else {
#pragma unroll 1
        for (int it = wave; it < td.job_count * nchunk; it += kWv) {
            const int q = it / nchunk;
            const JobDesc jd = jobs[td.job_begin + q];
            load_taps(jd);
            render_chunk(jd, it - q * nchunk);
        }
    }
}

// Held to 64 VGPRs (8 waves per SIMD) for lf <= 32, so that 4 workgroups of
// 512 threads (LDS at the default tile) or 8 of 256 fit per CU; for longer
// resonance filters 512-thread workgroups may take more registers.
template <int LFP, int KP, int NT, bool DIRECT>
__global__ __launch_bounds__(NT, (LFP <= 32 || NT == 256) ? 8 : 4) void k_render_quad(
    const float* __restrict__ src, const TileDesc* __restrict__ tiles, const JobDesc* __restrict__ jobs,
    const float* __restrict__ r, const int* __restrict__ P, const float* __restrict__ Gv, float* __restrict__ out,
    int lg, int TB) {
    extern __shared__ float4 smem4[];
    const TileDesc td = tiles[blockIdx.x];
    render_tile_quad<LFP, KP, NT, DIRECT>(td, src, jobs, r, P, Gv, out, lg, TB, reinterpret_cast<float*>(smem4),
                                          (int)threadIdx.x);
}

// Persistent variant over the device tile counter (see k_render_persistent).
// For lf <= 32 it is held to 64 VGPRs (8 waves per SIMD, 4 tiles per CU like
// the one-tile kernel), which costs a few spilled dwords per lane at some
// tap counts (none at K = 16); with 73 VGPRs it would fit 3 tiles per CU,
// and the loop measured 2-5 % slower.  Its tiles always take the direct
// stage: with both stages in the loop it spilled more and measured 2-6 %
// slower.
template <int LFP, int KP, int NT>
__global__ __launch_bounds__(NT, (LFP <= 32 || NT == 256) ? 8 : 4) void k_render_quad_persistent(
    const float* __restrict__ src, const TileDesc* __restrict__ tiles, int n_tiles,
    const JobDesc* __restrict__ jobs, const float* __restrict__ r, const int* __restrict__ P,
    const float* __restrict__ Gv, float* __restrict__ out, int lg, int TB, int* __restrict__ ctr) {
    extern __shared__ float4 smem4[];
    __shared__ int s_next;
    for (;;) {
        if (threadIdx.x == 0) s_next = atomicAdd(&ctr[0], 1);
        __syncthreads();
        const int t = s_next;
        __syncthreads();
        if (t >= n_tiles) break;
        // s_next is read again after the barrier: the same value (thread 0
        // writes it only after the tile's last barrier), but the compiler
        // cannot prove it, so the thread index below varies per tile and
        // nothing derived from it is hoisted out of this loop -- hoisted
        // values stay live across tiles and cost occupancy
        const int zero = s_next - t;
        const int tid = (int)threadIdx.x + zero;
        const int z = __builtin_amdgcn_readfirstlane(zero);
        const TileDesc td = tiles[t];
        render_tile_quad<LFP, KP, NT, true>(td, src + z, jobs + z, r + z, P + z, Gv + z, out + z, lg + z, TB + z,
                                            reinterpret_cast<float*>(smem4), tid);
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

int quad_lds_bytes(int TB, int lg, int lfp) { return (int)sizeof(float) * lds_quad_len(TB, lg, lfp); }

template <class F>
static int with_lf_k(int lfp, int kp, F&& f) {
#define HRIR_QCASE(L, K) \
    if (lfp == L && kp == K) return f(std::integral_constant<int, L>{}, std::integral_constant<int, K>{});
    HRIR_QCASE(16, 4) HRIR_QCASE(16, 8) HRIR_QCASE(16, 16) HRIR_QCASE(16, 32) HRIR_QCASE(16, 64)
    HRIR_QCASE(32, 4) HRIR_QCASE(32, 8) HRIR_QCASE(32, 16) HRIR_QCASE(32, 32) HRIR_QCASE(32, 64)
    HRIR_QCASE(64, 4) HRIR_QCASE(64, 8) HRIR_QCASE(64, 16) HRIR_QCASE(64, 32) HRIR_QCASE(64, 64)
#undef HRIR_QCASE
    return fail(HRIR_EINVAL, "no quad kernel for lf pad %d, k pad %d", lfp, kp);
}

template <class F>
static int with_nt(int nt, F&& f) {
    if (nt == 512) return f(std::integral_constant<int, 512>{});
    if (nt == 256) return f(std::integral_constant<int, 256>{});
    return fail(HRIR_EINVAL, "no quad kernel with %d threads", nt);
}

int quad_prepare(int lfp, int kp, int nt, size_t lds_bytes, bool persistent, int64_t n_tiles, int* grid) {
    return with_lf_k(lfp, kp, [&](auto L, auto K) -> int {
        return with_nt(nt, [&](auto N) -> int {
            constexpr int LV = decltype(L)::value, KV = decltype(K)::value, NV = decltype(N)::value;
            const void* kt = reinterpret_cast<const void*>(&k_render_quad<LV, KV, NV, false>);
            const void* kd = reinterpret_cast<const void*>(&k_render_quad<LV, KV, NV, true>);
            const void* kpers = reinterpret_cast<const void*>(&k_render_quad_persistent<LV, KV, NV>);
            hipError_t e = hipFuncSetAttribute(kt, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes);
            if (e == hipSuccess) e = hipFuncSetAttribute(kd, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes);
            if (e == hipSuccess)
                e = hipFuncSetAttribute(kpers, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes);
            if (e != hipSuccess) return fail(HRIR_EDEVICE, "quad_prepare: %s", hipGetErrorString(e));
            if (!persistent) {
                *grid = (int)n_tiles;
                return HRIR_OK;
            }
            int per_cu = 0, dev = 0, cus = 0;
            e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kpers, NV, lds_bytes);
            if (e == hipSuccess) e = hipGetDevice(&dev);
            if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
            if (e != hipSuccess) return fail(HRIR_EDEVICE, "quad_prepare: %s", hipGetErrorString(e));
            *grid = (int)std::min<int64_t>((int64_t)std::max(per_cu, 1) * cus, std::max<int64_t>(n_tiles, 1));
            return HRIR_OK;
        });
    });
}

bool quad_direct(const TileDesc* tiles, int64_t n_tiles) {
    for (int64_t i = 0; i < n_tiles; ++i)
        if (tiles[i].job_count >= kQPrioJobs) return false;
    return true;
}

int quad_launch(int lfp, int kp, int nt, bool persistent, bool direct, int grid, size_t lds_bytes, hipStream_t st,
                const float* src, const TileDesc* tiles, int n_tiles, const JobDesc* jobs, const float* r,
                const int* P, const float* Gv, float* out, int lg, int TB, int* ctr) {
    return with_lf_k(lfp, kp, [&](auto L, auto K) -> int {
        return with_nt(nt, [&](auto N) -> int {
            constexpr int LV = decltype(L)::value, KV = decltype(K)::value, NV = decltype(N)::value;
            if (persistent)
                hipLaunchKernelGGL((k_render_quad_persistent<LV, KV, NV>), dim3(grid), dim3(NV), lds_bytes, st, src,
                                   tiles, n_tiles, jobs, r, P, Gv, out, lg, TB, ctr);
            else if (direct)
                hipLaunchKernelGGL((k_render_quad<LV, KV, NV, true>), dim3((unsigned)n_tiles), dim3(NV), lds_bytes,
                                   st, src, tiles, jobs, r, P, Gv, out, lg, TB);
            else
                hipLaunchKernelGGL((k_render_quad<LV, KV, NV, false>), dim3((unsigned)n_tiles), dim3(NV), lds_bytes,
                                   st, src, tiles, jobs, r, P, Gv, out, lg, TB);
            return HRIR_OK;
        });
    });
}

}  // namespace hrir
