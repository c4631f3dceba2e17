// Direction-conditioned surrogate of the reflection filters: an MLP with ReLU
// hidden layers and a linear output layer from (sin az, cos az, sin el,
// cos el) to a direction's dense reflection filters, trained on the
// factorizations the method produces (Alg. 1), so that filters for
// directions between the measured ones come from the model.  Taps are the
// largest positive outputs (spconv_plan_topk), so they are non-negative as
// Eq. (1) requires; a ReLU on the output layer would instead leave output
// units that never recover from zero.
//
// Precision: FP32 master weights, bfloat16 activations between layers (round
// to nearest even), FP32 accumulation.  The contractions run on MFMA
// (v_mfma_f32_32x32x2f32): bf16 activations widen exactly to FP32, so the
// weights are used at full FP32 precision.  Gradients and Adam are FP32.
//
// A training step is a fixed sequence of launches (forward GEMMs, loss
// gradient, weight / bias / activation gradients, Adam, step counter), so it
// is captured once per (batch, buffers) as a HIP graph and replayed.  Every
// reduction runs in a fixed order: results do not depend on timing.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <vector>

#include "hrir_internal.h"

namespace hrir {
namespace {

typedef float f32x16 __attribute__((ext_vector_type(16)));

__device__ __forceinline__ float bf16_to_f32(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// Round to nearest even; NaN stays NaN.
__device__ __forceinline__ uint16_t f32_to_bf16(float f) {
    const uint32_t u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x7fffffu)) return (uint16_t)((u >> 16) | 0x40);
    const uint32_t r = u + 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(r >> 16);
}

template <class T> __device__ __forceinline__ float load_elt(const T* p, int64_t i);
template <> __device__ __forceinline__ float load_elt<float>(const float* p, int64_t i) { return p[i]; }
template <> __device__ __forceinline__ float load_elt<uint16_t>(const uint16_t* p, int64_t i) {
    return bf16_to_f32(p[i]);
}

struct Epi {
    const float* bias;          // per output column, or null
    const uint16_t* mask;       // bf16 [M][N] (row stride mask_ld): zero where mask <= 0, or null
    int64_t mask_ld;
    int relu;
    int out_bf16;               // store bf16 (else fp32)
    void* out;
    int64_t out_ld;
};

__device__ __forceinline__ void epilogue(const Epi& e, int i, int j, float x) {
    if (e.bias) x += e.bias[j];
    if (e.relu) x = fmaxf(x, 0.0f);
    if (e.mask && !(bf16_to_f32(e.mask[(int64_t)i * e.mask_ld + j]) > 0.0f)) x = 0.0f;
    if (e.out_bf16)
        static_cast<uint16_t*>(e.out)[(int64_t)i * e.out_ld + j] = f32_to_bf16(x);
    else
        static_cast<float*>(e.out)[(int64_t)i * e.out_ld + j] = x;
}

// C[M][N] = A[M][K] B[K][N]; A(i, k) = A[i sa_r + k sa_c], B(k, j) = B[k sb_r + j sb_c].
// One workgroup per 32 x 32 output tile (MFMA 32x32x2).  With W = 4 its
// waves take consecutive quarters of the block's contraction range, so each
// runs a quarter of the dependent load -> MFMA chain (for launches with few
// tiles), and their partial tiles are added through LDS in wave order (the
// same bits on every run); W = 1 when the tiles alone fill the GPU.  With
// gridDim.z > 1 the contraction is also split over blocks: block z sums k in
// [z k_chunk, (z + 1) k_chunk) and writes its raw partial tile to
// ws[z][M][N]; k_splitk_reduce adds the parts in order and applies the
// epilogue.  k_chunk is a multiple of 16 W.
template <class TA, int W>
__global__ __launch_bounds__(64 * W) void k_gemm(const TA* __restrict__ A, int64_t sa_r, int64_t sa_c,
                                                 const float* __restrict__ B, int64_t sb_r, int64_t sb_c, int M,
                                                 int N, int K, int k_chunk, Epi e, float* __restrict__ ws) {
    __shared__ float part[W > 1 ? W : 1][16][64];
    const int lane = threadIdx.x & 63, w = W > 1 ? (int)(threadIdx.x >> 6) : 0;
    const int row0 = blockIdx.y * 32, col0 = blockIdx.x * 32;
    const int ai = row0 + (lane & 31), bj = col0 + (lane & 31), kk = lane >> 5;
    const int kw = k_chunk / W;
    const int kb = blockIdx.z * k_chunk + w * kw;
    const int ke = min(K, kb + kw);
    f32x16 acc = {};
    // eight k-steps per iteration: their loads are issued together, then the MFMAs
    for (int k0 = kb; k0 < ke; k0 += 16) {
        float a[8], b[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int k = k0 + 2 * u + kk;
            a[u] = (ai < M && k < ke) ? load_elt<TA>(A, (int64_t)ai * sa_r + (int64_t)k * sa_c) : 0.0f;
            b[u] = (bj < N && k < ke) ? B[(int64_t)k * sb_r + (int64_t)bj * sb_c] : 0.0f;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a[u], b[u], acc, 0, 0, 0);
    }
    if (W > 1) {
#pragma unroll
        for (int v = 0; v < 16; ++v) part[w][v][lane] = acc[v];
        __syncthreads();
    }
    // wave w finishes accumulator entries v = (16 / W) w ... of every lane:
    // entry v of lane l is C[row0 + (v & 3) + 4 (l >> 5) + 8 (v >> 2)][col0 + (l & 31)]
#pragma unroll
    for (int q = 0; q < 16 / W; ++q) {
        const int v = w * (16 / W) + q;
        float x;
        if (W > 1) {
            x = part[0][v][lane];
#pragma unroll
            for (int u = 1; u < W; ++u) x += part[u][v][lane];
        } else {
            x = acc[v];
        }
        const int i = row0 + (v & 3) + 4 * (lane >> 5) + 8 * (v >> 2);
        const int j = col0 + (lane & 31);
        if (i >= M || j >= N) continue;
        if (gridDim.z > 1)
            ws[((int64_t)blockIdx.z * M + i) * N + j] = x;
        else
            epilogue(e, i, j, x);
    }
}

__global__ void k_splitk_reduce(const float* __restrict__ ws, int splits, int M, int N, Epi e) {
    const int64_t total = (int64_t)M * N;
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < total; q += (int64_t)gridDim.x * blockDim.x) {
        float s = 0.0f;
        for (int z = 0; z < splits; ++z) s += ws[z * total + q];
        epilogue(e, (int)(q / N), (int)(q % N), s);
    }
}

__global__ void k_to_bf16(const float* __restrict__ x, int64_t n, uint16_t* __restrict__ y) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        y[i] = f32_to_bf16(x[i]);
}

// dz = scale (y - t) (the output layer is linear); per-block partial sums of
// (y - t)^2 in fixed order.
constexpr int kLossThreads = 256;
__global__ __launch_bounds__(kLossThreads) void k_loss_grad(const float* __restrict__ y, const float* __restrict__ t,
                                                            int64_t n, float scale, float* __restrict__ dz,
                                                            double* __restrict__ part) {
    __shared__ double red[kLossThreads];
    double s = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)kLossThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kLossThreads) {
        const float d = y[i] - t[i];
        s += (double)d * d;
        dz[i] = scale * d;
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = kLossThreads / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// out[j] = sum_i dz[i][j].  A workgroup takes 64 columns (one coalesced
// row segment per wave load); its 16 waves take the rows i = w, w + 16, ...
// with four running sums each (rows 64c + w + 16q go to sum q), and the
// 64 partial sums of a column are added in a fixed order through LDS, so
// the result depends only on rows and cols: replays give the same bits.
constexpr int kColsumWaves = 16;

__global__ void __launch_bounds__(64 * kColsumWaves) k_colsum(const float* __restrict__ dz, int rows, int cols,
                                                               float* __restrict__ out) {
    __shared__ float part[kColsumWaves][64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int j = blockIdx.x * 64 + lane;
    float s[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    if (j < cols) {
        int i = w;
        for (; i + 3 * kColsumWaves < rows; i += 4 * kColsumWaves)
            for (int q = 0; q < 4; ++q) s[q] += dz[(int64_t)(i + q * kColsumWaves) * cols + j];
        if (i < rows) s[0] += dz[(int64_t)i * cols + j];
        if (i + kColsumWaves < rows) s[1] += dz[(int64_t)(i + kColsumWaves) * cols + j];
        if (i + 2 * kColsumWaves < rows) s[2] += dz[(int64_t)(i + 2 * kColsumWaves) * cols + j];
    }
    part[w][lane] = (s[0] + s[1]) + (s[2] + s[3]);
    __syncthreads();
    if (w == 0 && j < cols) {
        float t = 0.0f;
        for (int v = 0; v < kColsumWaves; ++v) t += part[v][lane];
        out[j] = t;
    }
}

// Adam with bias correction; the step number is *step + 1 (the counter is
// advanced by k_step_inc after this kernel).
__global__ void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, int64_t n, float lr, float b1, float b2, float eps,
                       const int* __restrict__ step) {
    const int t = *step + 1;
    const float c1 = 1.0f - powf(b1, (float)t), c2 = 1.0f - powf(b2, (float)t);
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const float gi = g[i];
        const float mi = b1 * m[i] + (1.0f - b1) * gi;
        const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    }
}

__global__ void k_step_inc(int* step) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *step += 1;
}

int cdiv(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }

}  // namespace
}  // namespace hrir

using namespace hrir;

struct hrir_mlp {
    std::vector<int> sizes;                 // sizes[0] inputs ... sizes[L] outputs
    int L = 0, max_batch = 0;
    int64_t n_params = 0;
    std::vector<int64_t> w_off, b_off;      // into the flat parameter buffer
    float *d_p = nullptr, *d_g = nullptr, *d_m = nullptr, *d_v = nullptr;
    std::vector<uint16_t*> d_act;           // bf16 [max_batch][sizes[l]], l < L
    float* d_out = nullptr;                 // fp32 [max_batch][sizes[L]]
    float* d_dz[2] = {nullptr, nullptr};    // fp32 gradients of pre-activations (ping-pong)
    float* d_ws = nullptr;                  // split-K partial tiles
    int64_t ws_elems = 0;
    int* d_step = nullptr;
    double* d_part = nullptr;               // loss partial sums
    int n_part = 0;
    // training graph for (n, x, t)
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipStream_t cap = nullptr;
    int g_n = -1;
    const float *g_x = nullptr, *g_t = nullptr;
    float g_lr = 0.0f;
};

namespace {

void free_mlp(hrir_mlp* m) {
    if (!m) return;
    if (m->exec) (void)hipGraphExecDestroy(m->exec);
    if (m->graph) (void)hipGraphDestroy(m->graph);
    if (m->cap) (void)hipStreamDestroy(m->cap);
    for (float* p : {m->d_p, m->d_g, m->d_m, m->d_v, m->d_out, m->d_dz[0], m->d_dz[1], m->d_ws}) (void)hipFree(p);
    for (uint16_t* p : m->d_act) (void)hipFree(p);
    (void)hipFree(m->d_step);
    (void)hipFree(m->d_part);
    delete m;
}

constexpr int kMaxSplits = 16;

// Launches C = A B with the epilogue; contractions much longer than the
// output is wide (the weight gradients, over the batch) are split over up
// to kMaxSplits blocks when the workspace holds the partial tiles.
hipError_t gemm(hrir_mlp* m, hipStream_t st, bool a_bf16, const void* A, int64_t sa_r, int64_t sa_c, const float* B,
                int64_t sb_r, int64_t sb_c, int M, int N, int K, const Epi& e) {
    const int tiles = cdiv(M, 32) * cdiv(N, 32);
    // four waves per tile while the tiles leave most of the GPU idle
    const bool quad = tiles < 2048;
    const int kStep = quad ? 64 : 16;                      // k_chunk granularity: 16 per wave
    int splits = 1;
    if (tiles < 256 && K >= 512) {
        splits = std::min<int>(kMaxSplits, std::max(1, K / 256));
        while (splits > 1 && (int64_t)splits * M * N > m->ws_elems) --splits;
    }
    const int k_chunk = (cdiv(K, splits) + kStep - 1) / kStep * kStep;
    splits = cdiv(K, k_chunk);
    const dim3 grid(cdiv(N, 32), cdiv(M, 32), splits);
    const auto* Ab = static_cast<const uint16_t*>(A);
    const auto* Af = static_cast<const float*>(A);
    if (a_bf16 && quad)
        hipLaunchKernelGGL((k_gemm<uint16_t, 4>), grid, dim3(256), 0, st, Ab, sa_r, sa_c, B, sb_r, sb_c, M, N, K,
                           k_chunk, e, m->d_ws);
    else if (a_bf16)
        hipLaunchKernelGGL((k_gemm<uint16_t, 1>), grid, dim3(64), 0, st, Ab, sa_r, sa_c, B, sb_r, sb_c, M, N, K,
                           k_chunk, e, m->d_ws);
    else if (quad)
        hipLaunchKernelGGL((k_gemm<float, 4>), grid, dim3(256), 0, st, Af, sa_r, sa_c, B, sb_r, sb_c, M, N, K,
                           k_chunk, e, m->d_ws);
    else
        hipLaunchKernelGGL((k_gemm<float, 1>), grid, dim3(64), 0, st, Af, sa_r, sa_c, B, sb_r, sb_c, M, N, K, k_chunk,
                           e, m->d_ws);
    if (splits > 1)
        hipLaunchKernelGGL(k_splitk_reduce, dim3(std::min(cdiv((int64_t)M * N, 256), 1024)), dim3(256), 0, st, m->d_ws,
                           splits, M, N, e);
    return hipGetLastError();
}

// Forward pass of n rows whose bf16 inputs are in d_act[0]; outputs in d_out.
hipError_t forward(hrir_mlp* m, int n, hipStream_t st) {
    for (int l = 0; l < m->L; ++l) {
        const int k = m->sizes[l], o = m->sizes[l + 1];
        const bool last = l + 1 == m->L;
        Epi e{m->d_p + m->b_off[l], nullptr, 0, last ? 0 : 1, last ? 0 : 1,
              last ? static_cast<void*>(m->d_out) : static_cast<void*>(m->d_act[l + 1]), o};
        hipError_t r = gemm(m, st, true, m->d_act[l], k, 1, m->d_p + m->w_off[l], o, 1, n, o, k, e);
        if (r != hipSuccess) return r;
    }
    return hipSuccess;
}

// Loss gradient and backward pass (after forward); gradients into d_g.
hipError_t backward(hrir_mlp* m, int n, const float* d_t, hipStream_t st) {
    const int nout = m->sizes[m->L];
    const int64_t nel = (int64_t)n * nout;
    hipLaunchKernelGGL(k_loss_grad, dim3(m->n_part), dim3(kLossThreads), 0, st, m->d_out, d_t, nel,
                       (float)(2.0 / (double)nel), m->d_dz[0], m->d_part);
    hipError_t r = hipGetLastError();
    int cur = 0;
    for (int l = m->L - 1; l >= 0 && r == hipSuccess; --l) {
        const int k = m->sizes[l], o = m->sizes[l + 1];
        const float* dz = m->d_dz[cur];
        // dW = act_l^T dz (k x o, contraction over the n rows)
        Epi ew{nullptr, nullptr, 0, 0, 0, m->d_g + m->w_off[l], o};
        r = gemm(m, st, true, m->d_act[l], 1, k, dz, o, 1, k, o, n, ew);
        if (r != hipSuccess) break;
        hipLaunchKernelGGL(k_colsum, dim3(cdiv(o, 64)), dim3(64 * kColsumWaves), 0, st, dz, n, o,
                           m->d_g + m->b_off[l]);
        r = hipGetLastError();
        if (r != hipSuccess || l == 0) break;
        // dz_{l-1} = (dz W^T) [act_l > 0]  (n x k, contraction over o)
        Epi eh{nullptr, m->d_act[l], k, 0, 0, m->d_dz[cur ^ 1], k};
        r = gemm(m, st, false, dz, o, 1, m->d_p + m->w_off[l], 1, o, n, k, o, eh);
        cur ^= 1;
    }
    return r;
}

hipError_t upload_inputs(hrir_mlp* m, const float* d_x, int n, hipStream_t st) {
    const int64_t el = (int64_t)n * m->sizes[0];
    hipLaunchKernelGGL(k_to_bf16, dim3(std::max(1, std::min(cdiv(el, 256), 1024))), dim3(256), 0, st, d_x, el,
                       m->d_act[0]);
    return hipGetLastError();
}

int read_loss(hrir_mlp* m, int n, hipStream_t st, double* loss) {
    std::vector<double> part(m->n_part);
    hipError_t e = hipMemcpyAsync(part.data(), m->d_part, sizeof(double) * m->n_part, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return fail(HRIR_EDEVICE, "mlp: %s", hipGetErrorString(e));
    double s = 0.0;
    for (double v : part) s += v;
    *loss = s / ((double)n * m->sizes[m->L]);
    return HRIR_OK;
}

}  // namespace

extern "C" int mlp_create(const int32_t* sizes, int32_t n_layers, int32_t max_batch, hrir_mlp** out) {
    clear_error();
    if (!sizes || !out) return fail(HRIR_EINVAL, "mlp_create: null pointer");
    *out = nullptr;
    if (n_layers < 1 || n_layers > 16) return fail(HRIR_EINVAL, "mlp_create: n_layers=%d outside [1, 16]", n_layers);
    if (max_batch < 1 || max_batch > (1 << 20))
        return fail(HRIR_EINVAL, "mlp_create: max_batch=%d outside [1, 2^20]", max_batch);
    for (int l = 0; l <= n_layers; ++l)
        if (sizes[l] < 1 || sizes[l] > 4096) return fail(HRIR_EINVAL, "mlp_create: sizes[%d]=%d outside [1, 4096]", l, sizes[l]);
    auto* m = new (std::nothrow) hrir_mlp;
    if (!m) return fail(HRIR_ENOMEM, "mlp_create: out of host memory");
    m->sizes.assign(sizes, sizes + n_layers + 1);
    m->L = n_layers;
    m->max_batch = max_batch;
    int64_t off = 0;
    int widest = 0;
    for (int l = 0; l < n_layers; ++l) {
        m->w_off.push_back(off);
        off += (int64_t)sizes[l] * sizes[l + 1];
        m->b_off.push_back(off);
        off += sizes[l + 1];
        widest = std::max(widest, sizes[l + 1]);
    }
    m->n_params = off;
    int64_t widest_layer = 0;
    for (int l = 0; l < n_layers; ++l) widest_layer = std::max<int64_t>(widest_layer, (int64_t)sizes[l] * sizes[l + 1]);
    m->ws_elems = kMaxSplits * widest_layer;
    m->n_part = std::max(1, std::min(cdiv((int64_t)max_batch * sizes[n_layers], kLossThreads), 512));
    hipError_t e = hipSuccess;
    for (float** p : {&m->d_p, &m->d_g, &m->d_m, &m->d_v})
        if (e == hipSuccess) e = hipMalloc(p, sizeof(float) * off);
    m->d_act.assign(n_layers, nullptr);
    for (int l = 0; l < n_layers && e == hipSuccess; ++l)
        e = hipMalloc(&m->d_act[l], sizeof(uint16_t) * (size_t)max_batch * sizes[l]);
    if (e == hipSuccess) e = hipMalloc(&m->d_out, sizeof(float) * (size_t)max_batch * sizes[n_layers]);
    for (int i = 0; i < 2 && e == hipSuccess; ++i) e = hipMalloc(&m->d_dz[i], sizeof(float) * (size_t)max_batch * widest);
    if (e == hipSuccess) e = hipMalloc(&m->d_ws, sizeof(float) * m->ws_elems);
    if (e == hipSuccess) e = hipMalloc(&m->d_step, sizeof(int));
    if (e == hipSuccess) e = hipMalloc(&m->d_part, sizeof(double) * m->n_part);
    if (e == hipSuccess) e = hipMemset(m->d_step, 0, sizeof(int));
    for (float* p : {m->d_p, m->d_m, m->d_v})
        if (e == hipSuccess) e = hipMemset(p, 0, sizeof(float) * off);
    if (e != hipSuccess) {
        free_mlp(m);
        return fail(e == hipErrorOutOfMemory ? HRIR_ENOMEM : HRIR_EDEVICE, "mlp_create: %s", hipGetErrorString(e));
    }
    *out = m;
    return HRIR_OK;
}

extern "C" int64_t mlp_num_params(const hrir_mlp* m) { return m ? m->n_params : -1; }

extern "C" int mlp_set_params(hrir_mlp* m, const float* params, int64_t n) {
    clear_error();
    if (!m || !params) return fail(HRIR_EINVAL, "mlp_set_params: null pointer");
    if (n != m->n_params) return fail(HRIR_EINVAL, "mlp_set_params: %lld values for %lld parameters", (long long)n,
                                      (long long)m->n_params);
    for (int64_t i = 0; i < n; ++i)
        if (!std::isfinite(params[i])) return fail(HRIR_EINVAL, "mlp_set_params: parameter %lld not finite", (long long)i);
    hipError_t e = hipDeviceSynchronize();
    if (e == hipSuccess) e = hipMemcpy(m->d_p, params, sizeof(float) * n, hipMemcpyHostToDevice);
    for (float* p : {m->d_m, m->d_v})
        if (e == hipSuccess) e = hipMemset(p, 0, sizeof(float) * n);
    if (e == hipSuccess) e = hipMemset(m->d_step, 0, sizeof(int));
    if (e != hipSuccess) return fail(HRIR_EDEVICE, "mlp_set_params: %s", hipGetErrorString(e));
    return HRIR_OK;
}

extern "C" int mlp_get_params(const hrir_mlp* m, float* params, int64_t n) {
    clear_error();
    if (!m || !params) return fail(HRIR_EINVAL, "mlp_get_params: null pointer");
    if (n != m->n_params) return fail(HRIR_EINVAL, "mlp_get_params: room for %lld values, %lld parameters",
                                      (long long)n, (long long)m->n_params);
    hipError_t e = hipDeviceSynchronize();
    if (e == hipSuccess) e = hipMemcpy(params, m->d_p, sizeof(float) * n, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return fail(HRIR_EDEVICE, "mlp_get_params: %s", hipGetErrorString(e));
    return HRIR_OK;
}

extern "C" int mlp_forward(hrir_mlp* m, const float* d_x, int32_t n, float* d_y, void* stream) {
    clear_error();
    if (!m || (n > 0 && (!d_x || !d_y))) return fail(HRIR_EINVAL, "mlp_forward: null pointer");
    if (n < 0) return fail(HRIR_EINVAL, "mlp_forward: n=%d < 0", n);
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const int nin = m->sizes[0], nout = m->sizes[m->L];
    for (int r0 = 0; r0 < n; r0 += m->max_batch) {
        const int nb = std::min(m->max_batch, n - r0);
        hipError_t e = upload_inputs(m, d_x + (int64_t)r0 * nin, nb, st);
        if (e == hipSuccess) e = forward(m, nb, st);
        if (e == hipSuccess)
            e = hipMemcpyAsync(d_y + (int64_t)r0 * nout, m->d_out, sizeof(float) * (size_t)nb * nout,
                               hipMemcpyDeviceToDevice, st);
        if (e != hipSuccess) return fail(HRIR_EDEVICE, "mlp_forward: %s", hipGetErrorString(e));
    }
    return HRIR_OK;
}

extern "C" int mlp_grads(hrir_mlp* m, const float* d_x, const float* d_t, int32_t n, float* grads, double* loss,
                         void* stream) {
    clear_error();
    if (!m || !d_x || !d_t) return fail(HRIR_EINVAL, "mlp_grads: null pointer");
    if (n < 1 || n > m->max_batch) return fail(HRIR_EINVAL, "mlp_grads: n=%d outside [1, %d]", n, m->max_batch);
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    hipError_t e = upload_inputs(m, d_x, n, st);
    if (e == hipSuccess) e = forward(m, n, st);
    if (e == hipSuccess) e = backward(m, n, d_t, st);
    if (e == hipSuccess && grads)
        e = hipMemcpyAsync(grads, m->d_g, sizeof(float) * m->n_params, hipMemcpyDeviceToHost, st);
    if (e != hipSuccess) return fail(HRIR_EDEVICE, "mlp_grads: %s", hipGetErrorString(e));
    if (loss) return read_loss(m, n, st, loss);
    e = hipStreamSynchronize(st);
    if (e != hipSuccess) return fail(HRIR_EDEVICE, "mlp_grads: %s", hipGetErrorString(e));
    return HRIR_OK;
}

extern "C" int mlp_train(hrir_mlp* m, const float* d_x, const float* d_t, int32_t n, int32_t steps, float lr,
                         double* loss, void* stream) {
    clear_error();
    if (!m || !d_x || !d_t) return fail(HRIR_EINVAL, "mlp_train: null pointer");
    if (n < 1 || n > m->max_batch) return fail(HRIR_EINVAL, "mlp_train: n=%d outside [1, %d]", n, m->max_batch);
    if (steps < 0) return fail(HRIR_EINVAL, "mlp_train: steps=%d < 0", steps);
    if (!(lr > 0.0f) || !std::isfinite(lr)) return fail(HRIR_EINVAL, "mlp_train: lr must be finite and > 0");
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    hipError_t e = upload_inputs(m, d_x, n, st);
    if (e != hipSuccess) return fail(HRIR_EDEVICE, "mlp_train: %s", hipGetErrorString(e));
    if (!m->exec || m->g_n != n || m->g_x != d_x || m->g_t != d_t || m->g_lr != lr) {
        // capture one step: forward, loss gradient, backward, Adam, counter
        if (m->exec) (void)hipGraphExecDestroy(m->exec);
        if (m->graph) (void)hipGraphDestroy(m->graph);
        m->exec = nullptr;
        m->graph = nullptr;
        if (!m->cap) e = hipStreamCreateWithFlags(&m->cap, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipStreamBeginCapture(m->cap, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess) {
            hipError_t ek = forward(m, n, m->cap);
            if (ek == hipSuccess) ek = backward(m, n, d_t, m->cap);
            if (ek == hipSuccess) {
                hipLaunchKernelGGL(k_adam, dim3(std::min(cdiv(m->n_params, 256), 1024)), dim3(256), 0, m->cap, m->d_p,
                                   m->d_g, m->d_m, m->d_v, m->n_params, lr, 0.9f, 0.999f, 1e-8f, m->d_step);
                ek = hipGetLastError();
            }
            if (ek == hipSuccess) {
                hipLaunchKernelGGL(k_step_inc, dim3(1), dim3(64), 0, m->cap, m->d_step);
                ek = hipGetLastError();
            }
            e = hipStreamEndCapture(m->cap, &m->graph);
            if (e == hipSuccess) e = ek;
        }
        if (e == hipSuccess) e = hipGraphInstantiate(&m->exec, m->graph, nullptr, nullptr, 0);
        if (e != hipSuccess) return fail(HRIR_EDEVICE, "mlp_train: graph capture: %s", hipGetErrorString(e));
        m->g_n = n;
        m->g_x = d_x;
        m->g_t = d_t;
        m->g_lr = lr;
    }
    for (int s = 0; s < steps && e == hipSuccess; ++s) e = hipGraphLaunch(m->exec, st);
    if (e != hipSuccess) return fail(HRIR_EDEVICE, "mlp_train: %s", hipGetErrorString(e));
    if (loss) return read_loss(m, n, st, loss);    // loss of the last step's forward pass
    return HRIR_OK;
}

extern "C" void mlp_destroy(hrir_mlp* m) {
    if (m) (void)hipDeviceSynchronize();
    free_mlp(m);
}
