// Partitioned FFT convolution (overlap-add) on the GPU: the frequency-domain
// comparison leg (Sec. I footnote on FFT convolution; Sec. IV-F names the
// partitioned block form and its cost).  Transforms are hipFFT calls.
//
// Each source is cut into blocks of B = nfft - m + 1 samples.  Per render:
//   1. k_ola_blocks: every block, zero padded to nfft, into xb[NB][nfft];
//   2. R2C of all source blocks (shared by every filter of that source);
//   3. k_ola_mul: Y[jb] = X[block(jb)] * H[filt(jb)] / nfft for every
//      (job, block) pair jb (filter spectra H are computed at create time);
//   4. C2R of all Y into yt[NJB][nfft];
//   5. k_ola_add: out[t] = sum of the (at most two) block results covering t.
#include <hip/hip_runtime.h>
#include <hipfft/hipfft.h>

#include <cmath>
#include <cstring>

#include "hrir_internal.h"
#include "render_common.h"

namespace hrir {

struct OlaBlock {        // one block of one source
    int64_t src_off;
    int32_t src_len;
    int32_t s0;          // first source sample of the block
};

struct OlaJob {          // one job: output row and where its block results live
    int64_t out_off;
    int64_t jb0;         // first (job, block) index
    int32_t out_len;     // src_len + m - 1
    int32_t nb;          // blocks of the source
    int32_t blk0;        // first source-block index of the source
    int32_t filt;        // row of the filter-spectrum table
};

__global__ void k_ola_blocks(const float* __restrict__ src, const OlaBlock* __restrict__ blocks, int B, int nfft,
                             float* __restrict__ xb) {
    const OlaBlock b = blocks[blockIdx.x];
    float* o = xb + (int64_t)blockIdx.x * nfft;
    for (int i = threadIdx.x; i < nfft; i += blockDim.x) {
        const int64_t q = (int64_t)b.s0 + i;
        o[i] = (i < B && q < b.src_len) ? src[b.src_off + q] : 0.0f;
    }
}

// grid: (ceil(nbins / 256), NJB); jb -> (job, block) via the per-jb tables
__global__ void k_ola_mul(const float2* __restrict__ X, const float2* __restrict__ Hs, const int32_t* __restrict__ jb_blk,
                          const int32_t* __restrict__ jb_filt, int nbins, float scale, float2* __restrict__ Y) {
    const int64_t jb = blockIdx.y;
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nbins) return;
    const float2 x = X[(int64_t)jb_blk[jb] * nbins + k];
    const float2 h = Hs[(int64_t)jb_filt[jb] * nbins + k];
    Y[jb * nbins + k] = make_float2((x.x * h.x - x.y * h.y) * scale, (x.x * h.y + x.y * h.x) * scale);
}

// grid: (ceil(max_out_len / 1024), n_jobs); 256 threads, 4 outputs each
__global__ void k_ola_add(const float* __restrict__ yt, const OlaJob* __restrict__ jobs, int B, int nfft,
                          float* __restrict__ out) {
    const OlaJob j = jobs[blockIdx.y];
    const int t0 = blockIdx.x * 1024 + threadIdx.x;
    for (int u = 0; u < 4; ++u) {
        const int t = t0 + 256 * u;
        if (t >= j.out_len) return;
        const int b = t / B;                       // block whose start is at or before t
        float acc = 0.0f;
        if (b < j.nb) acc += yt[(j.jb0 + b) * nfft + (t - b * B)];
        if (b >= 1 && t - (b - 1) * B < nfft) acc += yt[(j.jb0 + b - 1) * nfft + (t - (b - 1) * B)];
        out[j.out_off + t] = acc;
    }
}

}  // namespace hrir

using namespace hrir;

struct hrir_fft {
    int m = 0, nfft = 0, B = 0, nbins = 0;
    int64_t NB = 0, NJB = 0, n_jobs = 0, src_extent = 0, out_extent = 0, max_out_len = 0;
    OlaBlock* d_blocks = nullptr;
    OlaJob* d_jobs = nullptr;
    int32_t* d_jb_blk = nullptr;
    int32_t* d_jb_filt = nullptr;
    float2* d_H = nullptr;      // [n_used_filters][nbins]
    float* d_xb = nullptr;      // [NB][nfft]
    float2* d_X = nullptr;      // [NB][nbins]
    float2* d_Y = nullptr;      // [NJB][nbins]
    float* d_yt = nullptr;      // [NJB][nfft]
    hipfftHandle fwd = 0, inv = 0;
    bool has_fwd = false, has_inv = false;
};

namespace {

void free_fft(hrir_fft* f) {
    if (!f) return;
    if (f->has_fwd) (void)hipfftDestroy(f->fwd);
    if (f->has_inv) (void)hipfftDestroy(f->inv);
    for (void* p : {(void*)f->d_blocks, (void*)f->d_jobs, (void*)f->d_jb_blk, (void*)f->d_jb_filt, (void*)f->d_H,
                    (void*)f->d_xb, (void*)f->d_X, (void*)f->d_Y, (void*)f->d_yt})
        (void)hipFree(p);
    delete f;
}

int fft_fail(hipfftResult r, const char* what) { return fail(HRIR_EDEVICE, "%s: hipFFT error %d", what, (int)r); }

}  // namespace

extern "C" int fftola_create(const float* h, int32_t n_filters, int32_t m, int32_t nfft, const int64_t* src_off,
                             const int64_t* src_len, int32_t n_src, const spconv_job* jobs, int32_t n_jobs,
                             hrir_fft** out) {
    clear_error();
    if (!h || !out || (n_src > 0 && (!src_off || !src_len)) || (n_jobs > 0 && !jobs))
        return fail(HRIR_EINVAL, "fftola_create: null pointer");
    *out = nullptr;
    if (m < 1 || n_filters < 1 || n_src < 0 || n_jobs < 0) return fail(HRIR_EINVAL, "fftola_create: bad sizes");
    if (nfft < 2 * m || nfft > (1 << 20) || (nfft & (nfft - 1)))
        return fail(HRIR_EINVAL, "fftola_create: nfft=%d must be a power of two >= 2m and <= 2^20", nfft);
    for (int i = 0; i < n_src; ++i)
        if (src_len[i] < 1 || src_len[i] > (int64_t)INT32_MAX - m || src_off[i] < 0)
            return fail(HRIR_EINVAL, "fftola_create: source %d out of range", i);
    auto* f = new (std::nothrow) hrir_fft;
    if (!f) return fail(HRIR_ENOMEM, "fftola_create: out of host memory");
    f->m = m; f->nfft = nfft; f->B = nfft - m + 1; f->nbins = nfft / 2 + 1; f->n_jobs = n_jobs;
    auto bail = [&](int code) { free_fft(f); return code; };

    // blocks of the sources that have jobs; (job, block) tables
    std::vector<int> blk0(n_src, -1);
    std::vector<OlaBlock> hb;
    std::vector<int> used_filt(n_filters, -1);
    int n_used = 0;
    for (int j = 0; j < n_jobs; ++j) {
        const int s = jobs[j].src;
        if (s < 0 || s >= n_src || jobs[j].filt < 0 || jobs[j].filt >= n_filters || jobs[j].out_off < 0)
            return bail(fail(HRIR_EINVAL, "fftola_create: job %d out of range", j));
        if (blk0[s] < 0) {
            blk0[s] = (int)hb.size();
            for (int64_t s0 = 0; s0 < src_len[s]; s0 += f->B)
                hb.push_back(OlaBlock{src_off[s], (int32_t)src_len[s], (int32_t)s0});
        }
        if (used_filt[jobs[j].filt] < 0) used_filt[jobs[j].filt] = n_used++;
        f->src_extent = std::max(f->src_extent, src_off[s] + src_len[s]);
        f->out_extent = std::max(f->out_extent, jobs[j].out_off + src_len[s] + m - 1);
        f->max_out_len = std::max<int64_t>(f->max_out_len, src_len[s] + m - 1);
    }
    std::vector<OlaJob> hj(n_jobs);
    std::vector<int32_t> jbb, jbf;
    for (int j = 0; j < n_jobs; ++j) {
        const int s = jobs[j].src;
        const int nb = (int)((src_len[s] + f->B - 1) / f->B);
        hj[j] = OlaJob{jobs[j].out_off, (int64_t)jbb.size(), (int32_t)(src_len[s] + m - 1), nb, blk0[s],
                       used_filt[jobs[j].filt]};
        for (int b = 0; b < nb; ++b) {
            jbb.push_back(blk0[s] + b);
            jbf.push_back(used_filt[jobs[j].filt]);
        }
    }
    f->NB = (int64_t)hb.size();
    f->NJB = (int64_t)jbb.size();
    if (n_jobs == 0) { *out = f; return HRIR_OK; }
    if (f->NB > INT32_MAX || f->NJB > 65535LL * 65535LL)
        return bail(fail(HRIR_EINVAL, "fftola_create: too many blocks for nfft=%d", nfft));

    // filter spectra of the used filters
    std::vector<float> hp((size_t)n_used * nfft, 0.0f);
    for (int fi = 0; fi < n_filters; ++fi)
        if (used_filt[fi] >= 0) std::memcpy(&hp[(size_t)used_filt[fi] * nfft], h + (size_t)fi * m, sizeof(float) * m);
    hipError_t e = hipSuccess;
    float* d_hp = nullptr;
    const size_t nb = (size_t)f->nbins;
    e = hipMalloc(&f->d_blocks, hb.size() * sizeof(OlaBlock));
    if (e == hipSuccess) e = hipMalloc(&f->d_jobs, hj.size() * sizeof(OlaJob));
    if (e == hipSuccess) e = hipMalloc(&f->d_jb_blk, jbb.size() * sizeof(int32_t));
    if (e == hipSuccess) e = hipMalloc(&f->d_jb_filt, jbf.size() * sizeof(int32_t));
    if (e == hipSuccess) e = hipMalloc(&f->d_H, (size_t)n_used * nb * sizeof(float2));
    if (e == hipSuccess) e = hipMalloc(&f->d_xb, (size_t)f->NB * nfft * sizeof(float));
    if (e == hipSuccess) e = hipMalloc(&f->d_X, (size_t)f->NB * nb * sizeof(float2));
    if (e == hipSuccess) e = hipMalloc(&f->d_Y, (size_t)f->NJB * nb * sizeof(float2));
    if (e == hipSuccess) e = hipMalloc(&f->d_yt, (size_t)f->NJB * nfft * sizeof(float));
    if (e == hipSuccess) e = hipMalloc(&d_hp, hp.size() * sizeof(float));
    if (e == hipSuccess) e = hipMemcpy(f->d_blocks, hb.data(), hb.size() * sizeof(OlaBlock), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(f->d_jobs, hj.data(), hj.size() * sizeof(OlaJob), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(f->d_jb_blk, jbb.data(), jbb.size() * sizeof(int32_t), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(f->d_jb_filt, jbf.data(), jbf.size() * sizeof(int32_t), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(d_hp, hp.data(), hp.size() * sizeof(float), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        (void)hipFree(d_hp);
        return bail(fail(e == hipErrorOutOfMemory ? HRIR_ENOMEM : HRIR_EDEVICE, "fftola_create: %s",
                         hipGetErrorString(e)));
    }
    int n = nfft;
    hipfftResult r = hipfftPlanMany(&f->fwd, 1, &n, nullptr, 1, nfft, nullptr, 1, (int)nb, HIPFFT_R2C, (int)f->NB);
    if (r != HIPFFT_SUCCESS) { (void)hipFree(d_hp); return bail(fft_fail(r, "fftola_create: R2C plan")); }
    f->has_fwd = true;
    // filter spectra with a one-off plan over the used filters
    hipfftHandle hplan;
    r = hipfftPlanMany(&hplan, 1, &n, nullptr, 1, nfft, nullptr, 1, (int)nb, HIPFFT_R2C, n_used);
    if (r == HIPFFT_SUCCESS) {
        r = hipfftExecR2C(hplan, d_hp, reinterpret_cast<hipfftComplex*>(f->d_H));
        (void)hipDeviceSynchronize();
        (void)hipfftDestroy(hplan);
    }
    (void)hipFree(d_hp);
    if (r != HIPFFT_SUCCESS) return bail(fft_fail(r, "fftola_create: filter spectra"));
    r = hipfftPlanMany(&f->inv, 1, &n, nullptr, 1, (int)nb, nullptr, 1, nfft, HIPFFT_C2R, (int)f->NJB);
    if (r != HIPFFT_SUCCESS) return bail(fft_fail(r, "fftola_create: C2R plan"));
    f->has_inv = true;
    *out = f;
    return HRIR_OK;
}

extern "C" int fftola_render(hrir_fft* f, const float* d_src, int64_t src_elems, float* d_out, int64_t out_elems,
                             void* stream) {
    clear_error();
    if (!f) return fail(HRIR_EINVAL, "fftola_render: null handle");
    if (f->n_jobs == 0) return HRIR_OK;
    if (!d_src || !d_out) return fail(HRIR_EINVAL, "fftola_render: null device pointer");
    if (src_elems < f->src_extent || out_elems < f->out_extent)
        return fail(HRIR_EINVAL, "fftola_render: buffers too small");
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    hipLaunchKernelGGL(k_ola_blocks, dim3((unsigned)f->NB), dim3(256), 0, st, d_src, f->d_blocks, f->B, f->nfft,
                       f->d_xb);
    hipfftResult r = hipfftSetStream(f->fwd, st);
    if (r == HIPFFT_SUCCESS) r = hipfftExecR2C(f->fwd, f->d_xb, reinterpret_cast<hipfftComplex*>(f->d_X));
    if (r != HIPFFT_SUCCESS) return fft_fail(r, "fftola_render: R2C");
    // jb across grid.y in slices of 65535
    for (int64_t jb0 = 0; jb0 < f->NJB; jb0 += 65535) {
        const unsigned ny = (unsigned)std::min<int64_t>(65535, f->NJB - jb0);
        hipLaunchKernelGGL(k_ola_mul, dim3((f->nbins + 255) / 256, ny), dim3(256), 0, st, f->d_X, f->d_H,
                           f->d_jb_blk + jb0, f->d_jb_filt + jb0, f->nbins, 1.0f / (float)f->nfft,
                           f->d_Y + jb0 * f->nbins);
    }
    r = hipfftSetStream(f->inv, st);
    if (r == HIPFFT_SUCCESS)
        r = hipfftExecC2R(f->inv, reinterpret_cast<hipfftComplex*>(f->d_Y), f->d_yt);
    if (r != HIPFFT_SUCCESS) return fft_fail(r, "fftola_render: C2R");
    for (int64_t j0 = 0; j0 < f->n_jobs; j0 += 65535) {
        const unsigned ny = (unsigned)std::min<int64_t>(65535, f->n_jobs - j0);
        hipLaunchKernelGGL(k_ola_add, dim3((unsigned)((f->max_out_len + 1023) / 1024), ny), dim3(256), 0, st, f->d_yt,
                           f->d_jobs + j0, f->B, f->nfft, d_out);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(HRIR_EDEVICE, "fftola_render: %s", hipGetErrorString(e));
    return HRIR_OK;
}

extern "C" int fftola_info(const hrir_fft* f, int64_t* info4) {
    clear_error();
    if (!f || !info4) return fail(HRIR_EINVAL, "fftola_info: null pointer");
    info4[0] = f->nfft;
    info4[1] = f->B;
    info4[2] = f->NB;
    info4[3] = f->NJB;
    return HRIR_OK;
}

extern "C" void fftola_destroy(hrir_fft* f) { free_fft(f); }
