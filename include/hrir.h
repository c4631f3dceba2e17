/*
 * hrir.h -- C ABI of libhrir.so, an MI355X (gfx950) renderer for sparse
 * head-related impulse responses (Luo, Zotkin, Duraiswami, arXiv 1502.03162).
 *
 * The method models every HRIR x as x ~= f * g with one direction-independent
 * "resonance" filter f and one sparse, non-negative "reflection" filter g per
 * direction and ear (Sec. II, Eq. (1)).  A source s is then rendered as
 * (s * f) * g (Eq. (2)): z = f * s once per source, and per (direction, ear)
 * a K-tap gather  out[t] = sum_k g_k z[t - p_k].
 *
 * Conventions for every call:
 *   - Status: 0 on success, a negative HRIR_E* code on failure.  The message
 *     of the last failure on the calling thread is hrir_last_error().  No C++
 *     exception crosses this interface.
 *   - Every buffer is allocated and owned by the caller unless stated
 *     otherwise.  "Host" pointers are ordinary CPU memory; "device" pointers
 *     are HIP device memory of the current device (e.g. a torch tensor's
 *     data_ptr()).  Opaque handles are owned by the library and released by
 *     the matching *_destroy call.
 *   - Matrices are row-major.  A "filter" is one (direction, ear) HRIR; the
 *     HRIR set is laid out one HRIR per row.
 *   - Stream arguments are hipStream_t passed as void* (0 = null stream).
 *     Asynchronous calls return after enqueueing; device buffers must stay
 *     valid until the stream has reached the work.
 */
#ifndef HRIR_H
#define HRIR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define HRIR_OK 0
#define HRIR_EINVAL (-1)   /* bad argument: size, range, null pointer */
#define HRIR_ENOMEM (-2)   /* host or device allocation failed */
#define HRIR_ENOTPD (-3)   /* the resonance system of Eq. (11) is not positive definite */
#define HRIR_EAGAIN (-4)   /* no free slot or memory; retry later (never blocks) */
#define HRIR_EDEVICE (-5)  /* a HIP runtime call or kernel launch failed */

/* Thread-local message of the last failing call on this thread ("" if none).
 * The pointer stays valid until the next library call on this thread. */
const char* hrir_last_error(void);

/* ------------------------------------------------------------------------
 * Factorization: Toeplitz-constrained semi-NMF (Sec. III-C, Alg. 1),
 * followed by top-K sparsification.  Host memory, FP64, synchronous; the
 * iterations run on the host's cores, or on the GPU with
 * HRIR_FACTORIZE_DEVICE.
 *
 * X            host f64[n][m]: the HRIR set, one HRIR per row.
 * lf           resonance length (the paper's M - K + 1, Eq. (13)); the
 *              reflection length is lg = m - lf + 1 (so lf + lg - 1 = m).
 * iters        iterations T of Alg. 1 (>= 1).
 * seed, g0     initial G: if g0 (host f64[n][lg], entries > 0) is given it
 *              is used as is, else G0 ~ U(0, 1] from SplitMix64(seed) in
 *              row-major order (Alg. 1, first step).
 * lambda0      L1 weight of Eq. (14) applied inside the reflection update:
 *              lambda0 for the first 10% of the iterations, a geometric decay
 *              by 10^3 until 50%, 0 for the last half.  0 runs Alg. 1
 *              unchanged.  f is rescaled to unit norm every iteration
 *              (the product f * g is unchanged by it).
 * k            taps kept per reflection filter (1 <= k <= lg): the k largest
 *              positive entries of each row of G (ties to the lower index),
 *              stored in ascending position; rows with fewer positive entries
 *              are padded with (p = 0, g = 0) after their real taps.
 * flags        HRIR_REFIT_NNLS: replace the kept gains by the non-negative
 *              least-squares fit of the HRIR on that support with f fixed
 *              (Eq. (14) with lambda = 0 on the support).
 *              HRIR_FACTORIZE_DEVICE: run the iterations of Alg. 1 on the
 *              current GPU (FP64, the host's arithmetic and order; lf <= 64
 *              and m <= 4096, EINVAL otherwise); inputs and outputs stay in
 *              host memory and the call still returns when everything is
 *              done.
 * Outputs (host): f_out f64[lf] with ||f||_2 = 1; gdense_out f64[n][lg]
 * (optional) the dense G scaled to that f; p_out int32[n][k]; g_out
 * f32[n][k]; nnz_out int32[n] (optional) real taps per row; err_db_out
 * f64[n] (optional) 10 log10(||x_i - f * ghat_i||^2 / ||x_i||^2) of the
 * kept taps; cost_out f64[iters] (optional) ||X - F G^T||_F^2 after each
 * iteration (Eq. (3)).
 * Errors: EINVAL on sizes out of range or null required pointers; ENOTPD if
 * the resonance system is singular (e.g. G = 0); ENOMEM.
 * ---------------------------------------------------------------------- */
#define HRIR_REFIT_NNLS 1u
#define HRIR_FACTORIZE_DEVICE 2u

int hrir_factorize(const double* X, int32_t n, int32_t m, int32_t lf, int32_t iters,
                   uint64_t seed, const double* g0, double lambda0, int32_t k, uint32_t flags,
                   double* f_out, double* gdense_out, int32_t* p_out, float* g_out,
                   int32_t* nnz_out, double* err_db_out, double* cost_out);

/* ------------------------------------------------------------------------
 * The paper's sparsifier (Sec. III-D): with the resonance filter f fixed,
 * each reflection filter solves the penalised L1-NNLS problem of Eq. (14),
 *     min_g ||D (f * g - x)||^2 + lambda sum(g),  g >= 0,
 * for a residual transform D, and entries <= threshold (1e-4 in the paper)
 * are discarded.  Host only, FP64, synchronous; rows run in parallel and the
 * results do not depend on the thread count.
 *
 * Transforms: HRIR_D_IDENTITY; HRIR_D_CONV, the Toeplitz matrix of the
 * Gaussian N_sigma(k) = exp(-k^2 / 2 sigma^2) / (sigma sqrt(2 pi)) (Eq. (15));
 * HRIR_D_WINDOW, diag(exp(-t^2 / sigma^2)), t = 0..m-1 (Eq. (16); sigma =
 * +inf is the identity).
 *
 * hrir_sparsify
 *   X, n, m      host f64[n][m], one HRIR per row (m = lf + lg - 1).
 *   f, lf        host f64[lf], the fixed resonance filter.
 *   sigma        host f64[n] per-row bandwidth (null for HRIR_D_IDENTITY).
 *   lambda       host f64[n] per-row L1 weight, or null: then each row's
 *                lambda is the smallest found by 50 steps of geometric
 *                bisection on [1e-12, 1] * lambda_max (lambda_max = 2 max
 *                A^T D x, where g = 0 becomes optimal) whose solution keeps
 *                at most target_nnze entries; 0 if lambda = 0 already does.
 *   threshold    discard level (>= 0).
 *   k            output slots per row: the kept entries in ascending position
 *                order, padded with (p = 0, g = 0); a row with more than k
 *                entries keeps its k largest (ties to the lower position).
 *   p_out, g_out host i32[n][k], f32[n][k] (a tap table for spconv_plan).
 *   nnze_out     host i32[n] or null: entries kept before the k-slot cut.
 *   lambda_out   host f64[n] or null: the lambda used.
 *   err_db_out   host f64[n] or null: 10 log10(||x - f * g||^2 / ||x||^2)
 *                of the k-slot filter.
 * hrir_tune_sigma
 *   For each row, the window bandwidth in grid[0..n_grid) (each > 0, +inf
 *   allowed) whose HRIR_D_WINDOW solution minimises the spectral distortion
 *   of f * g against x (Eq. (17) over the m bins of a length-m DFT,
 *   magnitudes floored at 1e-12 of their maximum); ties keep the earlier
 *   grid entry (Sec. IV-E).  The solution for each bandwidth uses the given
 *   lambda when target_nnze = 0, else the lambda of hrir_sparsify's search
 *   for at most target_nnze entries (bandwidth tuned at the sparsity the
 *   filters will have).  sigma_out host f64[n], sd_out host f64[n] or null.
 * Errors: EINVAL (sizes, null pointers, non-finite inputs, bad sigma or
 * lambda), ENOTPD (a support whose columns are dependent).
 * ---------------------------------------------------------------------- */
#define HRIR_D_IDENTITY 0
#define HRIR_D_CONV 1
#define HRIR_D_WINDOW 2

int hrir_sparsify(const double* X, int32_t n, int32_t m, const double* f, int32_t lf, int32_t transform,
                  const double* sigma, const double* lambda, int32_t target_nnze, double threshold, int32_t k,
                  int32_t* p_out, float* g_out, int32_t* nnze_out, double* lambda_out, double* err_db_out);
int hrir_tune_sigma(const double* X, int32_t n, int32_t m, const double* f, int32_t lf, const double* grid,
                    int32_t n_grid, double lambda, int32_t target_nnze, double threshold, double* sigma_out,
                    double* sd_out);

/* The same two calls with the L1-NNLS solves (Eq. (14), and the lambda
 * search) on the current GPU in FP64: the host forms the normal matrices and
 * right-hand sides, one wavefront per (row, bandwidth) problem runs the
 * host's active-set steps and bisection in the host's order, and the host
 * finishes (tap tables, errors, spectral distortion).  Same arguments,
 * outputs and errors as the host calls (the device path needs
 * m - lf + 1 <= 256; EINVAL otherwise, EDEVICE / ENOMEM on device
 * failures); inputs and outputs are host memory and the calls return when
 * everything is done. */
int hrir_sparsify_device(const double* X, int32_t n, int32_t m, const double* f, int32_t lf, int32_t transform,
                         const double* sigma, const double* lambda, int32_t target_nnze, double threshold,
                         int32_t k, int32_t* p_out, float* g_out, int32_t* nnze_out, double* lambda_out,
                         double* err_db_out);
int hrir_tune_sigma_device(const double* X, int32_t n, int32_t m, const double* f, int32_t lf,
                           const double* grid, int32_t n_grid, double lambda, int32_t target_nnze,
                           double threshold, double* sigma_out, double* sd_out);

/* ------------------------------------------------------------------------
 * Render plan: the resonance filter and the sparse tap table on the device.
 * (Eq. (2) rendered as (s * f) * g; Sec. IV-F: cost proportional to the
 * number of kept taps.)
 *
 * r            host f32[lf], 1 <= lf <= 64.
 * p, g         host int32[n_filters][k] positions in [0, lg) and f32 gains
 *              >= 0 (padding taps may repeat a position with gain 0).
 * k            1 <= k <= 64.  lg: reflection length, 1 <= lg <= 2048.
 * The plan copies everything to plan-owned device memory (current device)
 * and is immutable afterwards (except rows rewritten by spconv_plan_topk):
 * renders on different streams may share it.
 *
 * spconv_plan_multi: one resonance filter per region of space (the paper's
 * proposed remedy for contralateral error, Sec. IV-D: separate
 * decompositions for sub-regions).  r is host f32[n_res][lf], 1 <= n_res <=
 * 64; res host int32[n_filters] gives each filter's region (may be null
 * when n_res = 1).  A source rendered at filters of several regions forms
 * one z = r_region * s per region; batches group a source's jobs by region.
 * Such plans render with the default kernel only (the other kernels, block
 * rendering, streaming and moving sources refuse them with EINVAL).
 * spconv_plan is spconv_plan_multi with n_res = 1.
 * Errors: EINVAL (ranges, p outside [0, lg), negative or non-finite g,
 * regions out of range), ENOMEM, EDEVICE.
 * ---------------------------------------------------------------------- */
typedef struct hrir_plan hrir_plan;

int spconv_plan(const float* r, int32_t lf, const int32_t* p, const float* g, int32_t n_filters,
                int32_t k, int32_t lg, hrir_plan** out);
int spconv_plan_multi(const float* r, int32_t n_res, int32_t lf, const int32_t* res, const int32_t* p,
                      const float* g, int32_t n_filters, int32_t k, int32_t lg, hrir_plan** out);
void spconv_plan_destroy(hrir_plan* plan);
/* host int32[3]: lf, k, lg of the plan. */
int spconv_plan_shape(const hrir_plan* plan, int32_t* lf_k_lg3);
/* The plan's device tables (owned by the plan): r f32[lfp] (zero padded),
 * p int32[n_filters][kp], g f32[n_filters][kp] (padded with (0, 0)), and
 * host int32[3] = lfp, kp, n_filters. */
int spconv_plan_device(const hrir_plan* plan, const float** r, const int** p, const float** g,
                       int32_t* lfp_kp_nf3);

/* One render job: source `src` through filter `filt` into one output row of
 * length src_len[src] + lf + lg - 2 starting at element out_off of the
 * output buffer.  Rows of different jobs must not overlap. */
typedef struct {
    int32_t src;
    int32_t filt;
    int64_t out_off;
} spconv_job;

/* ------------------------------------------------------------------------
 * Batch: a fixed job list over a fixed set of sources, prepared once and
 * rendered many times (the offline path, and the ragged job mix of many
 * sources, directions and ears in one launch).
 *
 * src_off, src_len host int64[n_src]: source i is d_src[src_off[i] ...
 *              src_off[i] + src_len[i]) of the buffer passed at render time;
 *              src_len >= 1.
 * jobs         host spconv_job[n_jobs]; n_jobs may be 0 (render is a no-op).
 * tile         outputs per work tile: a multiple of 1024 up to 4096 for the
 *              default kernel (default 2048), of 1024 up to 16384 for
 *              LDS_GATHER (default 4096), of 6144 up to 16384 for REGWIN
 *              (default 6144).
 * group        max jobs sharing one staged z tile (0 = all jobs of a source).
 * flags        SPCONV_PERSISTENT: one persistent launch over a device tile
 *              queue instead of one workgroup per tile.
 *              SPCONV_GRAPH: capture the launch in a HIP graph on first
 *              render and replay it afterwards (same d_src/d_out required).
 *              SPCONV_UNFUSED: write z to a batch-owned device buffer with a
 *              separate resonance kernel, then gather from it (reference
 *              path for the fused kernel).
 *              SPCONV_LDS_GATHER: fused kernel that reads each tap's z from
 *              one LDS copy of the z tile, 8 bytes per lane per read.
 *              SPCONV_REGWIN: fused kernel that keeps each lane's z window
 *              in registers (needs lg <= 169).
 *              Default: the fused quad kernel, which keeps 4 shifted copies
 *              of the z tile in LDS so every tap read is 16 bytes per lane.
 *              SPCONV_WG256: the quad kernel with 256-thread workgroups
 *              instead of 512 (twice as many tiles resident per CU when LDS
 *              allows; needs tile + lg + 2 <= 4096).
 *              All kernels sum every output in the same order, so results
 *              are bitwise identical across kernels and launch shapes.
 * The batch owns its device descriptor table (and z buffer when unfused).
 * Errors: EINVAL (bad indices, lengths, overlapping rows are not checked),
 * ENOMEM, EDEVICE.
 * ---------------------------------------------------------------------- */
#define SPCONV_PERSISTENT 1
#define SPCONV_GRAPH 2
#define SPCONV_UNFUSED 4
#define SPCONV_LDS_GATHER 8
#define SPCONV_REGWIN 16
#define SPCONV_WG256 32

typedef struct hrir_batch hrir_batch;

int spconv_batch_create(const hrir_plan* plan, const int64_t* src_off, const int64_t* src_len,
                        int32_t n_src, const spconv_job* jobs, int32_t n_jobs, int32_t tile,
                        int32_t group, int32_t flags, hrir_batch** out);

/* Enqueue the batch on `stream`: reads d_src (device f32, src_elems
 * elements), writes every job's output row in d_out (device f32, out_elems
 * elements).  Asynchronous.  Output elements outside the job rows are not
 * touched.
 * Errors: EINVAL (null pointers; a source or job row that does not fit in
 * the given element counts; SPCONV_GRAPH batch with different buffers than
 * its first render), EDEVICE. */
int spconv_batch_render(hrir_batch* batch, const float* d_src, int64_t src_elems, float* d_out,
                        int64_t out_elems, void* stream);

/* Launch-shape facts of a batch (host int64[5], in this order): number of
 * tiles, tile length, jobs per group, grid size of the launch, kernel
 * (0 quad, 1 register window, 2 LDS gather, 3 unfused). */
int spconv_batch_info(const hrir_batch* batch, int64_t* info5);
void spconv_batch_destroy(hrir_batch* batch);

/* Autotuner: for this job list, time every (tile, group, persistent) shape
 * the default kernel accepts (tile 1024..4096, group 0/4/8/16, workgroups of
 * 512 or 256 threads) with HIP
 * events, 1 warm-up + 3 timed renders each on `stream`, and return the
 * fastest (tile, group, flags) and its ms per render.  force_flags
 * (SPCONV_PERSISTENT and/or SPCONV_LDS_GATHER, or 0) is part of every
 * candidate; with SPCONV_PERSISTENT only persistent shapes are timed.  d_out is used as
 * scratch output (every job row is overwritten).  With cache_path (JSON,
 * may not exist yet) a result stored under the same key (K, lf, lg and the
 * job list's shape class: log2 of the output samples, jobs per source, log2
 * of the sources, force_flags) is returned without timing, and new results
 * are stored.
 * Synchronous.  Errors: EINVAL, EDEVICE. */
int spconv_autotune(const hrir_plan* plan, const float* d_src, int64_t src_elems, const int64_t* src_off,
                    const int64_t* src_len, int32_t n_src, const spconv_job* jobs, int32_t n_jobs, float* d_out,
                    int64_t out_elems, void* stream, const char* cache_path, int32_t force_flags,
                    int32_t* tile_out, int32_t* group_out, int32_t* flags_out, double* ms_out);

/* One-shot render: create a batch with default tiling, render it on
 * `stream`, wait for the stream, destroy the batch.  Synchronous.  Same
 * arguments and errors as spconv_batch_create + spconv_batch_render. */
int spconv_render(const hrir_plan* plan, const float* d_src, int64_t src_elems, const int64_t* src_off,
                  const int64_t* src_len, int32_t n_src, const spconv_job* jobs, int32_t n_jobs,
                  float* d_out, int64_t out_elems, void* stream);

/* Allocation-free one-shot render, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Same arguments, kernel, tiling and results (bit for
 * bit) as spconv_render, which allocates a descriptor table per call; here
 * the tile and job descriptors go into one fixed device array of the
 * library (2.25 MiB per device, held until the process ends), staged from
 * fixed host arrays.  The call makes no device or host allocation, is
 * synchronous (it waits for `stream` before returning), and calls from
 * several host threads are serialised by a lock; the array keeps the last
 * call's descriptors.  The current device must be the plan's.
 * Limits: n_jobs <= SPCONV_NOALLOC_MAX_JOBS, and at most
 * SPCONV_NOALLOC_MAX_TILES tiles of 2048 outputs, where a source with
 * output length L (= src_len + lf + lg - 2) and any number of jobs counts
 * ceil(L / 2048) tiles (per resonance region of its jobs).
 * Errors: EINVAL (as spconv_render, and either limit exceeded, checked
 * before any device work), EDEVICE. */
#define SPCONV_NOALLOC_MAX_JOBS 16384
#define SPCONV_NOALLOC_MAX_TILES 65536
int spconv_render_noalloc(const hrir_plan* plan, const float* d_src, int64_t src_elems, const int64_t* src_off,
                          const int64_t* src_len, int32_t n_src, const spconv_job* jobs, int32_t n_jobs,
                          float* d_out, int64_t out_elems, void* stream);

/* ------------------------------------------------------------------------
 * Dense direct render: the comparison leg, out = s * h with a full HRIR
 * (direct convolution costs the filter length per output, Sec. IV-F).
 *
 * dense_plan   h host f32[n_filters][m], 1 <= m <= 200, copied to the device.
 * dense_batch_create / _render / _destroy: as spconv_batch_*, with output
 *              rows of length src_len + m - 1 at each job's out_off.
 * Errors: EINVAL (ranges, non-finite h, buffers too small), ENOMEM, EDEVICE.
 * ---------------------------------------------------------------------- */
typedef struct hrir_dense hrir_dense;
typedef struct hrir_dense_batch hrir_dense_batch;

int dense_plan(const float* h, int32_t n_filters, int32_t m, hrir_dense** out);
void dense_plan_destroy(hrir_dense* plan);
int dense_batch_create(const hrir_dense* plan, const int64_t* src_off, const int64_t* src_len, int32_t n_src,
                       const spconv_job* jobs, int32_t n_jobs, hrir_dense_batch** out);
int dense_batch_render(hrir_dense_batch* batch, const float* d_src, int64_t src_elems, float* d_out,
                       int64_t out_elems, void* stream);
void dense_batch_destroy(hrir_dense_batch* batch);

/* ------------------------------------------------------------------------
 * Partitioned FFT convolution, overlap-add form: the frequency-domain
 * comparison leg (FFT convolution, Sec. I; block form and cost, Sec. IV-F).
 *
 * fftola_create  h host f32[n_filters][m]; nfft a power of two, 2m <= nfft
 *                <= 2^20; blocks of nfft - m + 1 source samples.  Plans the
 *                batched transforms (hipFFT), computes the spectra of the used
 *                filters and allocates the block buffers for this job list
 *                (rows as in dense_batch_*).  Synchronous.
 * fftola_render  enqueues block gather, R2C, spectrum products, C2R and the
 *                overlap-add on `stream`.
 * fftola_info    host int64[4]: nfft, block length, source blocks, (job,
 *                block) pairs.
 * Errors: EINVAL, ENOMEM, EDEVICE (hipFFT failures included).
 * ---------------------------------------------------------------------- */
typedef struct hrir_fft hrir_fft;

int fftola_create(const float* h, int32_t n_filters, int32_t m, int32_t nfft, const int64_t* src_off,
                  const int64_t* src_len, int32_t n_src, const spconv_job* jobs, int32_t n_jobs, hrir_fft** out);
int fftola_render(hrir_fft* plan, const float* d_src, int64_t src_elems, float* d_out, int64_t out_elems,
                  void* stream);
int fftola_info(const hrir_fft* plan, int64_t* info4);
void fftola_destroy(hrir_fft* plan);

/* ------------------------------------------------------------------------
 * Block (partitioned) rendering with device-resident stream history: the
 * real-time form (Sec. IV-F: time-domain partitioned convolution adds no
 * latency).  Each stream slot keeps the last lf - 1 source samples and the
 * last lg - 1 values of z = f * s in device memory; rendering a block emits
 * the block's output samples for both ears (sample t with input sample t)
 * and updates the slot.  Any split of a stream into blocks, followed by a
 * flush, reproduces spconv_render of the whole stream bit for bit.
 *
 * block_streams_create  max_streams slots (1..2^20), histories zeroed; the
 *                       plan must outlive the object.
 * block_streams_reset   zero the listed slots (start of a new stream).
 * block_render          one launch for n_jobs blocks, at most one per slot.
 *     d_in      device f32: block i is d_in[in_off, in_off + n), n in
 *               [1, 4096]; unused for flush blocks (may be null if every
 *               block is a flush).
 *     d_out     device f32: block i writes m samples of the left ear
 *               (filt_l) at out_off and m of the right ear (filt_r) at
 *               out_off + m; m = n, or lf + lg - 2 for a flush block.
 *     The job table is copied into pinned, coherent host memory (double
 *     buffered) that the kernel reads in place -- no copy command precedes
 *     the launch -- so the call returns after enqueueing and jobs may be
 *     reused at once; a call waits only for the kernel of the call before
 *     the previous one (it reads the same half).  Renders of one stream
 *     object are ordered on the streams they are enqueued on: successive
 *     calls that touch the same slot must use one HIP stream (or order
 *     their streams), and calls on one object must not overlap in time
 *     (one host thread at a time).
 * Errors: EINVAL (ranges, a stream twice in one call, buffers too small),
 * EDEVICE.
 * ---------------------------------------------------------------------- */
#define BLOCK_FLUSH 1

typedef struct {
    int32_t stream_id;   /* slot */
    int32_t n;           /* input samples (ignored for a flush) */
    int32_t filt_l;      /* left-ear filter */
    int32_t filt_r;      /* right-ear filter */
    int32_t flags;       /* BLOCK_FLUSH: emit the lf + lg - 2 tail samples */
    int32_t pad;
    int64_t in_off;
    int64_t out_off;
} block_job;

typedef struct hrir_streams hrir_streams;

int block_streams_create(const hrir_plan* plan, int32_t max_streams, hrir_streams** out);
int block_streams_reset(hrir_streams* streams, const int32_t* slots, int32_t n, void* stream);
int block_render(hrir_streams* streams, const float* d_in, int64_t in_elems, const block_job* jobs, int32_t n_jobs,
                 float* d_out, int64_t out_elems, void* stream);
void block_streams_destroy(hrir_streams* streams);

/* ------------------------------------------------------------------------
 * Streaming request loop with continuous batching: the serving form of the
 * block renderer above (Sec. IV-F; Eq. (2) applied block by block, so each
 * output sample leaves with its input sample).
 *
 * Blocks of many streams are submitted from host memory at any time.  A
 * loop thread gathers what has arrived into the next launch (a
 * "generation": at most one block per stream, as a stream's blocks run in
 * order through its device-resident history) and starts it while fewer than
 * two generations are on the GPU, so blocks that arrive during a render join
 * the following one.  Generation buffers (device memory plus pinned host
 * staging) form a ring sized from hbm_budget; a block that no buffer can
 * take is refused with HRIR_EAGAIN, never waited for.  The result of every
 * block is the same bits whatever else shares its launch.
 *
 * stream_open    max_streams stream slots (1..2^20) with zeroed histories;
 *                hbm_budget bounds the device bytes of histories plus the
 *                generation ring (EINVAL if it cannot hold two generations
 *                of one maximal block); 0 sizes it as a quarter of the
 *                device memory free at the call (hipMemGetInfo), and
 *                ENOMEM if what the budget places on the device exceeds
 *                the free memory.  flags: STREAM_DIRECT_LAUNCH sizes
 *                each launch to its batch (one workgroup per block) instead
 *                of replaying a HIP graph of a persistent launch;
 *                STREAM_ZERO_COPY keeps the generation ring (job tables,
 *                input blocks, outputs) in pinned, coherent host memory
 *                that the kernel reads and writes in place -- a launch needs
 *                no copy commands, and hbm_budget then bounds the
 *                histories plus that pinned ring; STREAM_SLEEPING_COMPLETION
 *                makes the completion thread wait for each generation in
 *                the HIP runtime (a blocking-sync event: the thread sleeps
 *                until the GPU signals) instead of polling the event with
 *                pauses, which frees a host core for other servers at the
 *                cost of the wake-up latency.  Starts a loop thread and
 *                a completion thread on the current device.
 * stream_submit  copies n samples (1..4096) of host_block; the caller keeps
 *                its buffer.  filt_l/filt_r are the block's left/right
 *                filters (a direction change takes effect at the block
 *                boundary).  EAGAIN when no generation buffer has room:
 *                poll, then submit again.
 * stream_end     queues the stream's flush: its result carries the last
 *                lf + lg - 2 output samples (flags STREAM_RESULT_TAIL) and
 *                the stream's history is zeroed, so the id may start a new
 *                stream at once.  EAGAIN as for stream_submit.
 * stream_poll    moves up to max finished results to out[] in completion
 *                order (per stream, submission order) and returns their
 *                count.  A result's out points to 2 * n host floats owned by
 *                the server (left ear, then right ear), valid until the next
 *                stream_poll call on this server.  timeout_us: 0 returns at
 *                once, > 0 waits up to that long for a result, < 0 waits
 *                until one is ready; it never waits when nothing is queued
 *                or running.  A failed device call is reported here as
 *                EDEVICE once its earlier results are drained.
 * stream_info    host int64[8]: launches, results, output samples per ear,
 *                submits refused with EAGAIN, largest launch (blocks),
 *                generation buffers, samples per generation, blocks queued
 *                but not launched.
 * stream_close   renders what is queued, waits for the GPU and frees
 *                everything; results not polled are dropped.  No other call
 *                on the server may run during or after it.
 * stream_submit, stream_end, stream_poll and stream_info may be called from
 * several threads at once; submissions take no lock (a compare-and-swap on
 * the open generation reserves a job slot and its samples).  The calls for
 * one stream id must not overlap in time: a stream's blocks run in the
 * order its (one) submitting thread made them.  Times are CLOCK_MONOTONIC nanoseconds: submit,
 * launch of the result's generation, and the moment the completion thread
 * saw its output in host memory.
 * ---------------------------------------------------------------------- */
#define STREAM_DIRECT_LAUNCH 1
#define STREAM_ZERO_COPY 2
#define STREAM_SLEEPING_COMPLETION 4
#define STREAM_RESULT_TAIL 1

typedef struct hrir_server hrir_server;

typedef struct {
    uint64_t tag;           /* as submitted */
    int32_t stream_id;
    int32_t n;              /* output samples per ear */
    const float* out;       /* host f32[2][n], server owned, valid until the next poll */
    int64_t t_submit_ns;
    int64_t t_launch_ns;
    int64_t t_done_ns;
    int32_t flags;          /* STREAM_RESULT_TAIL for the result of stream_end */
    int32_t pad;
} hrir_result;

int stream_open(const hrir_plan* plan, int32_t max_streams, int64_t hbm_budget, int32_t flags, hrir_server** out);
int stream_submit(hrir_server* server, int32_t stream_id, const float* host_block, int32_t n, int32_t filt_l,
                  int32_t filt_r, uint64_t tag);
int stream_end(hrir_server* server, int32_t stream_id, int32_t filt_l, int32_t filt_r, uint64_t tag);
int stream_poll(hrir_server* server, hrir_result* out, int32_t max, int32_t timeout_us);
int stream_info(const hrir_server* server, int64_t* info8);
void stream_close(hrir_server* server);

/* ------------------------------------------------------------------------
 * Moving sources (Eq. (2) with the direction, i.e. the reflection filter,
 * changing over time) and the device-side top-K that turns dense predicted
 * reflection filters into plan rows.
 *
 * spconv_plan_topk  for each of n_rows rows of d_dense (device f32, row i at
 *                   d_dense + i * row_stride), the plan's k largest finite
 *                   positive entries among the first `width` (<= lg), ties to
 *                   the lower position, in ascending position order, padded
 *                   with (0, 0), are written to plan rows first_row + i.  The
 *                   update is ordered on `stream`: renders that use those rows
 *                   must follow it on that stream (or wait for it).
 * spconv_plan_read  copies plan rows [first_row, first_row + n_rows) back to
 *                   host i32 / f32 [n_rows][k] (waits for the device).
 * moving_create     n_src sources of src_len samples each, contiguous in
 *                   the source buffer (source i at i * src_len); the direction
 *                   changes every seg_len samples (a multiple of 256);
 *                   n_seg = ceil(src_len / seg_len).  Output sample t of an
 *                   ear uses the filter of segment j = min(t / seg_len,
 *                   n_seg - 1); in its first `fade` (0..256) samples, u =
 *                   t - j seg_len < fade with j >= 1, the output is
 *                   a y_j + (1 - a) y_{j-1}, a = (u + 1) / fade, y_j the render
 *                   with segment j's filter.  tile: outputs per workgroup, a
 *                   multiple of 256 up to 4096 (0: 3072 where three such
 *                   tiles fit in a CU's LDS, else 2048).  The plan must
 *                   outlive the object.
 * moving_render     seg_filt host i32[n_src][n_seg][2] plan rows (left,
 *                   right) per segment, validated and staged through pinned
 *                   memory (double buffered) and uploaded on a stream of the
 *                   object's own, so the upload overlaps the previous
 *                   call's kernels; the kernels on `stream` wait for it
 *                   (device events, no host wait).  The render kernel's tap
 *                   table is formed from the plan's rows (a small kernel on
 *                   `stream`) by the first call and again by the first call
 *                   after spconv_plan_topk rewrites rows, so rows predicted
 *                   on the device before the call are used.  d_out device
 *                   f32: the row of (source i, ear e) at (2 i + e) *
 *                   out_stride, out_stride >= src_len + lf + lg - 2.
 * moving_info       host int64[4]: n_seg, output row length, tiles, tile length.
 * Errors: EINVAL, ENOMEM, EDEVICE.
 * ---------------------------------------------------------------------- */
typedef struct hrir_moving hrir_moving;

int spconv_plan_topk(hrir_plan* plan, int32_t first_row, const float* d_dense, int32_t n_rows, int64_t row_stride,
                     int32_t width, void* stream);
int spconv_plan_read(const hrir_plan* plan, int32_t first_row, int32_t n_rows, int32_t* p_out, float* g_out);
int moving_create(const hrir_plan* plan, int32_t n_src, int64_t src_len, int32_t seg_len, int32_t fade,
                  int32_t tile, hrir_moving** out);
int moving_render(hrir_moving* moving, const float* d_src, int64_t src_elems, const int32_t* seg_filt, float* d_out,
                  int64_t out_stride, int64_t out_elems, void* stream);
int moving_info(const hrir_moving* moving, int64_t* info4);
void moving_destroy(hrir_moving* moving);

/* ------------------------------------------------------------------------
 * Direction-conditioned surrogate: an MLP that predicts a direction's dense
 * reflection filters (the sparse non-negative factor of Eq. (1)) from
 * (sin az, cos az, sin el, cos el), trained on factorizations of the
 * measured directions (Alg. 1) so that directions between them get filters
 * too.  Layer l maps sizes[l] -> sizes[l + 1], ReLU on every layer but the
 * last, which is linear; the taps are its largest positive outputs
 * (spconv_plan_topk), hence non-negative.  FP32 master weights; activations are
 * stored as bfloat16 between layers (inputs included, round to nearest
 * even); products accumulate in FP32 on MFMA; loss = mean squared error
 * over all outputs; Adam (beta 0.9 / 0.999, eps 1e-8) with bias correction.
 *
 * mlp_create      sizes[0..n_layers], each 1..4096; max_batch rows per pass
 *                 (1..2^20).  Parameters start at zero: set them first.
 * mlp_num_params  total parameter count (-1 for a null handle).
 * mlp_set_params  host f32 flat parameters: W0 (sizes[0] x sizes[1],
 *                 row-major), b0, W1, b1, ...; resets Adam's moments and
 *                 step.  Synchronous.
 * mlp_get_params  the same layout back to host memory.  Synchronous.
 * mlp_forward     d_x device f32 [n][sizes[0]] -> d_y device f32
 *                 [n][sizes[n_layers]], any n >= 0 (chunks of max_batch).
 * mlp_grads       one forward + backward pass on n <= max_batch rows with
 *                 targets d_t device f32 [n][out], no update; gradients to
 *                 host f32 (parameter layout) and the loss, if non-null.
 * mlp_train       `steps` full-batch Adam steps on (d_x, d_t); the step is a
 *                 HIP graph captured on the first call for these buffers,
 *                 batch and learning rate, then replayed.  loss (host, may be
 *                 null) receives the loss of the last step's forward pass
 *                 (the call then waits for the GPU).
 * Device buffers belong to the caller and must stay valid until the stream
 * reaches the work.  Errors: EINVAL, ENOMEM, EDEVICE.
 * ---------------------------------------------------------------------- */
/* surrogate_select: the fallback rule for directions the surrogate predicts.
 * For each query direction (radians, the grid's interaural-polar angles:
 * lateral az, polar el), the nearest validation direction by the angle
 * between unit vectors (sin az, cos az cos el, cos az sin el) decides: if
 * the surrogate's error measured there, val_err_db, exceeds max_err_db, the
 * query takes the nearest measured direction (choice = its index), else the
 * surrogate (choice = -1).  Ties go to the lower index.  Host, synchronous. */
int surrogate_select(const double* q_az, const double* q_el, int32_t n_q, const double* val_az, const double* val_el,
                     const double* val_err_db, int32_t n_val, const double* meas_az, const double* meas_el,
                     int32_t n_meas, double max_err_db, int32_t* choice);

typedef struct hrir_mlp hrir_mlp;

int mlp_create(const int32_t* sizes, int32_t n_layers, int32_t max_batch, hrir_mlp** out);
int64_t mlp_num_params(const hrir_mlp* mlp);
int mlp_set_params(hrir_mlp* mlp, const float* params, int64_t n);
int mlp_get_params(const hrir_mlp* mlp, float* params, int64_t n);
int mlp_forward(hrir_mlp* mlp, const float* d_x, int32_t n, float* d_y, void* stream);
int mlp_grads(hrir_mlp* mlp, const float* d_x, const float* d_t, int32_t n, float* grads, double* loss,
              void* stream);
int mlp_train(hrir_mlp* mlp, const float* d_x, const float* d_t, int32_t n, int32_t steps, float lr, double* loss,
              void* stream);
void mlp_destroy(hrir_mlp* mlp);

/* ------------------------------------------------------------------------
 * Load generator for the streaming loop (a client of the stream_* calls
 * above, for measurement).  Open loop: block arrivals form a Poisson process
 * of rate_hz blocks/s over all streams for duration_s seconds; each arrival
 * picks a stream uniformly in [0, n_streams), a length uniformly in
 * [block_min, block_max] (<= 4096) and a block of that length at a random
 * offset of the host signal; each stream keeps a random direction (filter
 * pair 2d, 2d + 1 with d < n_filters / 2) that changes every ~16 blocks.
 * A refused block (EAGAIN) is retried until admitted; its latency counts
 * from its arrival time.  rate_hz <= 0 submits back to back for duration_s
 * (the saturation rate).  At most max_blocks blocks are submitted.  With
 * submit_threads = T > 1 the arrivals come from T threads, each a Poisson
 * process of rate_hz / T over its own streams.  A
 * polling thread collects the results; the call returns when all are in,
 * or with EDEVICE if none arrives for 30 s after submission ends.
 * A refused block is retried after a growing pause (retrying at once would
 * hold up the threads that free room).  Latencies: arrival -> done (p50/p99/max), submit -> done
 * (p50/p99), and the two parts outside the server: arrival -> admitted and
 * done -> collected (p99/max); arrival -> admitted splits into the
 * generator's own lag (arrival -> first submit attempt) and the wait of
 * refused blocks (back-pressure).
 * The server must not be polled by anyone else meanwhile.
 * ---------------------------------------------------------------------- */
typedef struct {
    int32_t n_streams;
    int32_t block_min;
    int32_t block_max;
    int32_t n_filters;
    double rate_hz;
    double duration_s;
    uint64_t seed;
    int64_t max_blocks;
    const float* signal;     /* host f32[signal_len] */
    int64_t signal_len;
    int32_t submit_threads;  /* submitting threads (0 or 1: one); thread t serves the t-th of T contiguous stream ranges */
    int32_t pad;
} stream_load;

typedef struct {
    int64_t blocks;          /* blocks submitted (and rendered) */
    int64_t out_samples;     /* output samples, both ears */
    int64_t eagain;          /* refusals while admitting */
    int64_t launches;        /* generations launched */
    double offered_hz;       /* rate_hz, 0 for back to back */
    double achieved_hz;      /* blocks / wall_s */
    double out_samples_per_s;
    double submit_s;         /* time spent submitting */
    double wall_s;           /* first arrival to last result */
    double mean_batch;       /* blocks per launch */
    double p50_ms, p99_ms, max_ms;
    double p50_server_ms, p99_server_ms;
    double p99_admit_ms, max_admit_ms;     /* arrival -> admitted by stream_submit */
    double p99_collect_ms, max_collect_ms; /* done -> collected by the polling thread */
    double max_wait_ms;      /* longest submit -> launch of its generation */
    double max_launch_ms;    /* longest launch -> done of a generation */
    double p99_gen_lag_ms, max_gen_lag_ms; /* arrival -> first offered to stream_submit: the generator's
                                              own delay; large only when it cannot keep its schedule */
} stream_load_stats;

int stream_loadgen(hrir_server* server, const stream_load* cfg, stream_load_stats* stats);

#ifdef __cplusplus
}
#endif

#endif /* HRIR_H */
