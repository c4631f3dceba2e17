// The z tile of the quad LDS-gather kernels (render_quad.hip,
// render_moving.hip): the resonance FIR forms z in registers, from a source
// window staged in LDS (quad_stage) or read by each thread from global
// memory (quad_stage_direct), and z is written as four copies shifted by
// 0..3 samples, Zc[m] = z[t0 - H + m + c], so that every tap of every quad of
// outputs is one aligned 16-byte LDS read.
#pragma once

#include <hip/hip_runtime.h>

#include "render_common.h"

namespace hrir {

constexpr int kQR = 16;               // outputs per lane per chunk (4 quads)
constexpr int kQChunk = 64 * kQR;     // outputs per wave per chunk
constexpr int kQThreads = 512;        // 8 wave64 per workgroup
constexpr int kQWaves = kQThreads / 64;
constexpr int kQPass = 2;             // FIR passes of 8 z values per thread (8192 z: tiles up to 4096)
static_assert(kQChunk == 1024, "quad chunk");
static_assert(kQPass * kQThreads * kZpt >= kQuadTileMax + 2048 + 3, "FIR passes cover the largest tile");
constexpr int kQSmallCover = kQPass * 256 * kZpt;   // z values the FIR of a 256-thread workgroup covers
static_assert(kZpt == 8, "the copy stores rotate 8 values per lane by lane / 8");
typedef float f8v __attribute__((ext_vector_type(8)));

// Floats per shifted copy: holds m < TB + H (+ padding so that the copies
// start on different banks).
__host__ __device__ inline int quad_cs(int TB, int H) { return round_up(TB + H + 4, 8) + 4; }

__host__ __device__ inline int lds_quad_len(int TB, int lg, int lfp) {
    const int H = lg - 1;
    const int s_len = round_up(TB + H + 3, kZpt) + lfp + 4;
    const int c_len = 4 * quad_cs(TB, H);
    return s_len > c_len ? s_len : c_len;
}

// Writes one thread's 8 z values, z_win[u0 .. u0 + 7], into the four
// shifted copies: Zc[m] = z_win[m + c] for m < mlim; interior groups of 8
// without tests.
__device__ __forceinline__ void quad_copies(const float (&zz)[kZpt], int u0, int mlim, int CS, float* zc, int tid) {
    if (u0 >= 4 && u0 + kZpt <= mlim) {
        float* z0 = zc + u0;
        *reinterpret_cast<float4*>(z0) = make_float4(zz[0], zz[1], zz[2], zz[3]);
        *reinterpret_cast<float4*>(z0 + 4) = make_float4(zz[4], zz[5], zz[6], zz[7]);
        // Copies 1..3 are not 16-byte aligned: one dword per lane per
        // store.  Lanes are 8 dwords apart, so if every lane stored the
        // same element a, 8 lanes would share each bank.  Store k writes
        // element (k + lane / 8) mod 8 instead, which puts the 64 lanes
        // on 64 different banks; the lane's values are rotated by
        // lane / 8 to match: a vector of 8 rotated by 1, 2 and 4 under
        // the bits of g, 8 selects per stage on one condition.  (On an
        // array indexed inside a loop the compiler merges the stages into
        // an 8-way select per value, about five times the instructions.)
        const int g = (tid >> 3) & 7;
        f8v zr = {zz[0], zz[1], zz[2], zz[3], zz[4], zz[5], zz[6], zz[7]};
        if (g & 1) zr = __builtin_shufflevector(zr, zr, 1, 2, 3, 4, 5, 6, 7, 0);
        if (g & 2) zr = __builtin_shufflevector(zr, zr, 2, 3, 4, 5, 6, 7, 0, 1);
        if (g & 4) zr = __builtin_shufflevector(zr, zr, 4, 5, 6, 7, 0, 1, 2, 3);
        // zr[k] = zz[(k + g) mod 8], stored at element (k + g) mod 8.
        // The element offsets pass through an empty asm (no instruction):
        // seen through, they let the compiler turn the rotated stores back
        // into fixed-offset stores of values picked by 8-way selects.
        int ok[kZpt];
#pragma unroll
        for (int k = 0; k < kZpt; ++k) ok[k] = (k + g) & (kZpt - 1);
        asm volatile("" : "+v"(ok[0]), "+v"(ok[1]), "+v"(ok[2]), "+v"(ok[3]), "+v"(ok[4]), "+v"(ok[5]),
                          "+v"(ok[6]), "+v"(ok[7]));
#pragma unroll
        for (int c = 1; c < 4; ++c)
#pragma unroll
            for (int k = 0; k < kZpt; ++k) zc[c * CS + u0 + ok[k] - c] = zr[k];
    } else {
#pragma unroll
        for (int c = 0; c < 4; ++c)
#pragma unroll
            for (int a = 0; a < kZpt; ++a) {
                const int m = u0 + a - c;
                if (m >= 0 && m < mlim) zc[c * CS + m] = zz[a];
            }
    }
}

// Stages the tile's source, runs the FIR and writes the four shifted copies
// of z into lds (ends with a barrier).  H = lg - 1; CS = quad_cs(TB, H).
// Only the z values the tile's outputs read are formed (a ragged last tile
// forms fewer); the bounds come from the tile, so in a loop over tiles the
// compiler cannot hoist them and keep them live across tiles.
// after_source() runs once the source window is in LDS (after a barrier)
// and before the FIR: a caller can stage its own tables there, outside the
// first lds_quad_len floats, while the FIR's inputs are ready.
struct NoHook {
    __device__ void operator()() const {}
};

// tid: this thread's index in the workgroup (a persistent caller passes one
// the compiler cannot see as loop-invariant, so that nothing derived from
// it is hoisted out of its loop over tiles).
// prio (wave-uniform): raise the waves' issue priority while the source
// window is loaded, so a new tile's loads go out ahead of other tiles'
// gathers on the CU; it pays when the gather is long (many jobs per tile).
// NT: threads of the workgroup (512, or 256 when TB + lg + 2 <= 4096, so
// that the two FIR passes of 8 z values per thread still cover the tile).
template <int LFP, int NT = kQThreads, class Hook = NoHook>
__device__ __forceinline__ void quad_stage(const TileDesc& td, const float* __restrict__ src,
                                           const float* __restrict__ r, int lg, int TB, float* lds, int tid,
                                           Hook&& after_source = Hook{}, bool prio = false) {
    static_assert(NT == 512 || NT == 256, "quad workgroups have 256 or 512 threads");
    const int H = lg - 1;
    const int tile_len = min(TB, td.out_len - td.t0);
    const int NZ = tile_len + H + 3;           // z_win[u], u < NZ, covers every quad read
    const int nz8 = round_up(NZ, kZpt);
    const int CS = quad_cs(TB, H);
    float* s_win = lds;
    float* zc = lds;                           // the copies overwrite s_win after the FIR

    if (prio) __builtin_amdgcn_s_setprio(2);
    stage_s<LFP, NT>(td, src, H, nz8, s_win, tid);
    after_source();
    if (prio) __builtin_amdgcn_s_setprio(0);

    // FIR into registers: zz[ps][a] = z_win[u0 + a], u0 = 8 (256 ps + tid)
    float rr[LFP];
#pragma unroll
    for (int n = 0; n < LFP; ++n) rr[n] = r[n];
    float zz[kQPass][kZpt];
#pragma unroll
    for (int ps = 0; ps < kQPass; ++ps) {
        const int u0 = (ps * NT + tid) * kZpt;
        if (u0 < nz8) {
            float w[LFP + kZpt];
#pragma unroll
            for (int i = 0; i < LFP + kZpt; i += 4) {
                const float4 v = *reinterpret_cast<const float4*>(s_win + u0 + i);
                w[i] = v.x; w[i + 1] = v.y; w[i + 2] = v.z; w[i + 3] = v.w;
            }
#pragma unroll
            for (int a = 0; a < kZpt; ++a) {
                float acc = 0.0f;
#pragma unroll
                for (int n = 0; n < LFP; ++n) acc = fmaf(rr[n], w[a + LFP - 1 - n], acc);
                zz[ps][a] = acc;
            }
        }
    }
    __syncthreads();                            // every read of s_win is done
    // Zc[m] = z_win[m + c] for m < tile_len + H
    const int mlim = tile_len + H;
#pragma unroll
    for (int ps = 0; ps < kQPass; ++ps) {
        const int u0 = (ps * NT + tid) * kZpt;
        if (u0 < nz8) quad_copies(zz[ps], u0, mlim, CS, zc, tid);
    }
    __syncthreads();
}

// The same z tile with no source window in LDS: each thread reads its FIR
// window (LFP + 7 samples for its 8 z values) straight from global memory,
// where neighbouring threads' windows overlap in the vector cache, and
// writes its z values into the copies at once, so a tile takes one barrier
// instead of three.  The z values are quad_stage's, bit for bit (same
// windows, same fma order).  In a loop over tiles the caller's barrier
// after the previous tile's gather must precede it (the copies are written
// without one).
template <int LFP, int NT = kQThreads>
__device__ __forceinline__ void quad_stage_direct(const TileDesc& td, const float* __restrict__ src,
                                                  const float* __restrict__ r, int lg, int TB, float* zc, int tid,
                                                  bool prio = false) {
    static_assert(NT == 512 || NT == 256, "quad workgroups have 256 or 512 threads");
    const int H = lg - 1;
    const int tile_len = min(TB, td.out_len - td.t0);
    const int nz8 = round_up(tile_len + H + 3, kZpt);
    const int CS = quad_cs(TB, H);
    const int mlim = tile_len + H;
    // window sample i of z_win[u0] is source sample sbase + u0 + i
    const int64_t sbase = (int64_t)td.t0 - H - (LFP - 1);
    const float* sp = src + td.src_off;
    const bool interior = sbase >= 0 && sbase + nz8 + LFP <= td.src_len;
    float rr[LFP];
#pragma unroll
    for (int n = 0; n < LFP; ++n) rr[n] = r[n];
#pragma unroll
    for (int ps = 0; ps < kQPass; ++ps) {
        const int u0 = (ps * NT + tid) * kZpt;
        if (u0 >= nz8) continue;
        float w[LFP + kZpt];
        if (prio) __builtin_amdgcn_s_setprio(2);
        if (interior) {
#pragma unroll
            for (int i = 0; i < LFP + kZpt; i += 4) {
                const f4u x = *reinterpret_cast<const f4u*>(sp + sbase + u0 + i);
                w[i] = x.x; w[i + 1] = x.y; w[i + 2] = x.z; w[i + 3] = x.w;
            }
        } else {
#pragma unroll
            for (int i = 0; i < LFP + kZpt; ++i) {
                const int64_t q = sbase + u0 + i;
                w[i] = (q >= 0 && q < td.src_len) ? sp[q] : 0.0f;
            }
        }
        if (prio) __builtin_amdgcn_s_setprio(0);
        float zz[kZpt];
#pragma unroll
        for (int a = 0; a < kZpt; ++a) {
            float acc = 0.0f;
#pragma unroll
            for (int n = 0; n < LFP; ++n) acc = fmaf(rr[n], w[a + LFP - 1 - n], acc);
            zz[a] = acc;
        }
        quad_copies(zz, u0, mlim, CS, zc, tid);
    }
    __syncthreads();
}

}  // namespace hrir
