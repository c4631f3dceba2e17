// Device-side pieces shared by the render kernels: launch constants, work
// descriptors, and the staging of one source tile with its resonance FIR.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace hrir {

constexpr int kThreads = 256;   // 4 wave64 per workgroup
constexpr int kWaves = kThreads / 64;
constexpr int kR = 16;          // outputs per lane per chunk
constexpr int kChunk = 64 * kR; // outputs per wave per chunk
constexpr int kZpt = 8;         // z values per thread per FIR pass
constexpr int kStageV = 8;      // 16-byte source loads per thread in flight while staging

// float4 with 4-byte alignment: global_load_dwordx4 at any dword address.
typedef float f4u __attribute__((ext_vector_type(4), aligned(4)));
constexpr int kMinWaves = 4;    // waves per SIMD the render kernels must fit (<= 128 VGPRs)

struct TileDesc {               // 32 bytes
    int64_t src_off;            // element offset of the source in d_src
    int32_t src_len;
    int32_t out_len;            // src_len + lf + lg - 2
    int32_t t0;                 // first output sample of the tile
    int32_t job_begin;          // into the job table (jobs sorted by source)
    int32_t job_count;
    int32_t res;                // resonance filter (region) of the tile's jobs
};

struct JobDesc {                // 16 bytes
    int64_t out_off;
    int32_t filt;
    int32_t pad;
};

struct ZDesc {                  // unfused path: one chunk of z of one source
    int64_t src_off;
    int64_t z_off;
    int32_t src_len;
    int32_t v0;
};

struct GDesc {                  // unfused path: one chunk of one job
    int64_t out_off;
    int64_t z_off;
    int32_t out_len;
    int32_t nz;
    int32_t t0;
    int32_t filt;
};

__host__ __device__ constexpr int round_up(int a, int b) { return (a + b - 1) / b * b; }

// Empty asm that takes 16 accumulators as read-write VGPR operands and
// clobbers memory: values are materialised here, and memory operations are
// not moved across it.  It emits no instruction.
__device__ __forceinline__ void pin16(float (&a)[16]) {
    asm volatile("" : "+v"(a[0]), "+v"(a[1]), "+v"(a[2]), "+v"(a[3]), "+v"(a[4]), "+v"(a[5]), "+v"(a[6]),
                      "+v"(a[7]), "+v"(a[8]), "+v"(a[9]), "+v"(a[10]), "+v"(a[11]), "+v"(a[12]),
                      "+v"(a[13]), "+v"(a[14]), "+v"(a[15])
                 :
                 : "memory");
}

// LDS floats needed by one tile: s window then z window.
__host__ __device__ inline int lds_s_len(int TB, int lg, int lfp) { return round_up(TB + lg - 1, kZpt) + lfp + 4; }
__host__ __device__ inline int lds_z_len(int TB, int lg) { return round_up(TB + lg - 1, kZpt); }

// Stage s_win[i] = s[t0 - H - (LFP-1) + i] for i < nz8 + LFP + 4 in LDS (zero
// outside the signal), enough for z_win[u] = z[t0 - H + u], u < nz8 (a
// multiple of 8).  Ends with a barrier.
template <int LFP, int NT = kThreads>
__device__ __forceinline__ void stage_s(const TileDesc& td, const float* __restrict__ src, int H, int nz8,
                                        float* s_win,
                                        int tid) {
    const int ns = nz8 + LFP + 4;
    // 1. stage s[sbase + i], zero outside [0, src_len).  Interior tiles use
    //    16-byte loads (any dword alignment), kStageV per thread in flight
    //    before any LDS write, so staging costs about one HBM latency.
    const int64_t sbase = (int64_t)td.t0 - H - (LFP - 1);
    const float* sp = src + td.src_off;
    const int ns4 = ns / 4;
    if (sbase >= 0 && sbase + ns <= td.src_len) {
        // interior tile (the tile-uniform common case): no per-element tests
        for (int b4 = 0; b4 < ns4; b4 += NT * kStageV) {
            float4 v[kStageV];
#pragma unroll
            for (int u = 0; u < kStageV; ++u) {
                const int i4 = min(b4 + u * NT + tid, ns4 - 1);
                const f4u x = *reinterpret_cast<const f4u*>(sp + sbase + 4 * i4);
                v[u] = make_float4(x.x, x.y, x.z, x.w);
            }
#pragma unroll
            for (int u = 0; u < kStageV; ++u) {
                const int i4 = b4 + u * NT + tid;
                if (i4 < ns4) *reinterpret_cast<float4*>(s_win + 4 * i4) = v[u];
            }
        }
    } else {
        // tile overlapping either end of the source: zero outside [0, src_len)
        for (int i = tid; i < ns; i += NT) {
            const int64_t q = sbase + i;
            s_win[i] = (q >= 0 && q < td.src_len) ? sp[q] : 0.0f;
        }
    }
    __syncthreads();
}

// Form z_win[u] = z[t0 - H + u] = sum_n r[n] s_win[u + LFP - 1 - n] for
// u < round_up(TB + H, 8) after staging the source.  Ends with a barrier.
template <int LFP>
__device__ __forceinline__ void stage_z(const TileDesc& td, const float* __restrict__ src,
                                        const float* __restrict__ r, int H, int TB, float* s_win,
                                        float* z_win) {
    const int tid = threadIdx.x;
    const int nz8 = round_up(TB + H, kZpt);
    stage_s<LFP>(td, src, H, nz8, s_win, (int)threadIdx.x);

    // 2. z_win[u] = z[t0 - H + u] = sum_n r[n] s_win[u + LFP - 1 - n]
    float rr[LFP];
#pragma unroll
    for (int n = 0; n < LFP; ++n) rr[n] = r[n];
    for (int u0 = tid * kZpt; u0 < nz8; u0 += kThreads * kZpt) {
        float w[LFP + kZpt];
#pragma unroll
        for (int i = 0; i < LFP + kZpt; i += 4) {
            const float4 v = *reinterpret_cast<const float4*>(s_win + u0 + i);
            w[i] = v.x; w[i + 1] = v.y; w[i + 2] = v.z; w[i + 3] = v.w;
        }
        float zz[kZpt];
#pragma unroll
        for (int a = 0; a < kZpt; ++a) {
            float acc = 0.0f;
#pragma unroll
            for (int n = 0; n < LFP; ++n) acc = fmaf(rr[n], w[a + LFP - 1 - n], acc);
            zz[a] = acc;
        }
        *reinterpret_cast<float4*>(z_win + u0) = make_float4(zz[0], zz[1], zz[2], zz[3]);
        *reinterpret_cast<float4*>(z_win + u0 + 4) = make_float4(zz[4], zz[5], zz[6], zz[7]);
    }
    __syncthreads();
}


// Register-window kernel (render_rw.hip): largest tap position it serves and
// its tile granularity.
constexpr int kHW = 168;
constexpr int kRW = 24;
constexpr int kTileRW = 4 * 64 * kRW;

// LDS bytes of one register-window tile.
int rw_lds_bytes(int TB, int lfp);
// Sets the kernels' LDS limit; for persistent launches also returns the grid
// (resident workgroups, at most n_tiles).  Status code as in hrir.h.
int rw_prepare(int lfp, size_t lds_bytes, bool persistent, int64_t n_tiles, int* grid);
// Enqueues the register-window kernel.
int rw_launch(int lfp, bool persistent, int grid, size_t lds_bytes, hipStream_t st, const float* src,
              const TileDesc* tiles, int n_tiles, const JobDesc* jobs, const float* r, const int* P,
              const float* Gv, float* out, int kp, int k, int TB, int* ctr);

// Quad LDS-gather kernel (render_quad.hip), the default render path.
int quad_lds_bytes(int TB, int lg, int lfp);
// nt: threads per workgroup, 512 or 256 (256 needs TB + lg + 2 <= 4096).
int quad_prepare(int lfp, int kp, int nt, size_t lds_bytes, bool persistent, int64_t n_tiles, int* grid);
// True when every tile has fewer jobs than the staging-priority threshold:
// the one-tile quad kernel then takes the direct stage (the persistent one
// always does).
bool quad_direct(const TileDesc* tiles, int64_t n_tiles);
int quad_launch(int lfp, int kp, int nt, bool persistent, bool direct, int grid, size_t lds_bytes, hipStream_t st,
                const float* src, const TileDesc* tiles, int n_tiles, const JobDesc* jobs, const float* r,
                const int* P, const float* Gv, float* out, int lg, int TB, int* ctr);
constexpr int kQuadTileMax = 4096;

// Shape and device tables of a plan (render.hip owns the struct).
struct PlanView {
    int lf, lfp, k, kp, lg, n_filters, device, n_res;
    float* d_r;
    int* d_p;
    float* d_g;
    uint64_t rows_gen;      // changes whenever the library rewrites tap rows
};
}  // namespace hrir
struct hrir_plan;
namespace hrir {
PlanView plan_view(const hrir_plan* plan);
// Marks the plan's tap rows as rewritten (called by every library routine
// that writes them after creation).
void plan_rows_changed(hrir_plan* plan);

}  // namespace hrir
