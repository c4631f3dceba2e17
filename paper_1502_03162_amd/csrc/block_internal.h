// Internal interface of the block renderer shared by block.hip (kernels and
// the block_* entry points) and server.cpp (the streaming request loop).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "hrir_internal.h"

namespace hrir {

constexpr int kBlockMax = 4096;           // input samples per block

// Job flags as the kernel sees them.
constexpr int kJobFlush = 1;              // zero input of lf + lg - 2 samples: emit the tail
constexpr int kJobReset = 2;              // zero the slot's history after the block (stream ends)

struct BJob {                             // device job table entry (32 bytes)
    int32_t slot, n, filt_l, filt_r, flags, pad;
    int64_t in_off, out_off;
};

struct BlockShape {
    int lf, lfp, k, kp, lg, n_filt, max_streams, hist_stride, device;
};

BlockShape block_shape(const hrir_streams* s);

// Samples in and out per ear of one job (n, or the tail for a flush).
inline int block_job_len(const BlockShape& sh, const BJob& j) {
    return (j.flags & kJobFlush) ? sh.lf + sh.lg - 2 : j.n;
}

// Dynamic LDS bytes of a block launch whose longest job has max_m samples.
size_t block_lds_bytes(const BlockShape& sh, int max_m);

// Enqueues the block kernel on `st`.  Jobs are read from the device table
// d_jobs; the job count is *d_count when d_count is not null (a persistent
// grid of `grid` workgroups strides over the table), else n_jobs with one
// workgroup per job.  The caller has validated every job against the buffers.
hipError_t block_enqueue(const hrir_streams* s, const float* d_in, const BJob* d_jobs, const int32_t* d_count,
                         int n_jobs, int grid, int max_m, float* d_out, hipStream_t st);

}  // namespace hrir
