// Learned surrogate: a three-layer network n_in -> h -> h -> n_out that
// predicts magnification histograms from lens parameters, for the
// parameter-space exploration of the Bayesian Monte Carlo analysis that
// motivates fast map generation (arXiv:1703.09707, Sec. 1).
//
// Weights are stored in BF16 (rounded from FP32 master copies that Adam
// updates); activations and accumulation are FP32.  GELU (erf form) follows
// the first two layers; the output is a softmax, trained with cross-entropy
// against shooter histograms.  Parameter layout (FP32, flat):
// W1[n_in][h], b1[h], W2[h][h], b2[h], W3[h][n_out], b3[n_out].
//
// One LDS-tiled FP32 GEMM on the matrix cores serves every product of the
// forward and backward passes; it computes C[M][N] = sum_k A(m, k) B(k, n)
// with A and B read directly or transposed, B in FP32 or BF16 (widened to
// FP32 exactly), and a fused epilogue.  The products are FP32 MFMAs
// (v_mfma_f32_16x16x4f32: FP32 operands and accumulation, so activations
// stay FP32).  All reductions run in a fixed order, so results are
// deterministic.
#include <cmath>
#include <limits>
#include <vector>

#include "raysh_ctx.h"

namespace {

// The network's products are small (M, N and K of at most a few hundred),
// so a product's time is one workgroup's chain of staging round trips, not
// the matrix cores' rate: 32 x 32 tiles give 4 times the workgroups of
// 64 x 64 (64 for a 256 x 256 product), and K-chunks of 64 keep the chain
// at four steps for K = 256.  A training step of the 4-256-256-64 network
// at batch 256 took 387 us with 64 x 64 x 16 tiles, 145 us with these.
constexpr int BM = 32, BN = 32, BK = 64, kGemmThreads = 256;
constexpr int WT = BM / 32;   // 16 x 16 MFMA tiles per wave and dimension (the 4 waves take quarters)

enum Epilogue {
    EPI_STORE = 0,       // C = acc
    EPI_BIAS_GELU = 1,   // Z = acc + bias (into C), H = gelu(Z) (into C2)
    EPI_GELU_GRAD = 2,   // C = acc * gelu'(aux)
    EPI_BIAS = 3         // C = acc + bias
};

__device__ __forceinline__ float bf16_to_f32(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

// Round to nearest, ties to even (finite inputs).
__device__ __forceinline__ uint16_t f32_to_bf16(float f) {
    const uint32_t u = __float_as_uint(f);
    const uint32_t lsb = (u >> 16) & 1u;
    return (uint16_t)((u + 0x7FFFu + lsb) >> 16);
}

__device__ __forceinline__ float gelu(float z) { return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f)); }

__device__ __forceinline__ float gelu_grad(float z) {
    return 0.5f * (1.0f + erff(z * 0.70710678118654752f)) + z * expf(-0.5f * z * z) * 0.39894228040143268f;
}

template <bool A_T, bool B_T, bool B_BF16, int EPI>
__global__ __launch_bounds__(kGemmThreads) void gemm_kernel(const float *__restrict__ A, int lda,
                                                            const void *__restrict__ Bv, int ldb, int M,
                                                            int N, int K, float *__restrict__ C, int ldc,
                                                            const float *__restrict__ bias,
                                                            const float *__restrict__ aux,
                                                            float *__restrict__ C2) {
    __shared__ float As[BK][BM + 4];
    __shared__ float Bs[BK][BN + 4];
    const int lane = threadIdx.x % 64, wave = threadIdx.x / 64;
    const int wm = (wave / 2) * (BM / 2), wn = (wave % 2) * (BN / 2);   // the wave's quarter of the tile
    const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
    typedef float floatx4 __attribute__((ext_vector_type(4)));
    floatx4 acc[WT][WT];
#pragma unroll
    for (int si = 0; si < WT; ++si)
#pragma unroll
        for (int sj = 0; sj < WT; ++sj) acc[si][sj] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
    for (int k0 = 0; k0 < K; k0 += BK) {
        // stage A tile: BM x BK elements, 4 per thread
        for (int e = threadIdx.x; e < BM * BK; e += kGemmThreads) {
            const int mm = A_T ? e % BM : e / BK;
            const int kk = A_T ? e / BM : e % BK;
            const int m = m0 + mm, k = k0 + kk;
            float v = 0.0f;
            if (m < M && k < K) v = A_T ? A[(int64_t)k * lda + m] : A[(int64_t)m * lda + k];
            As[kk][mm] = v;
        }
        // stage B tile: BK x BN elements
        for (int e = threadIdx.x; e < BK * BN; e += kGemmThreads) {
            const int kk = B_T ? e % BK : e / BN;
            const int nn = B_T ? e / BK : e % BN;
            const int k = k0 + kk, n = n0 + nn;
            float v = 0.0f;
            if (k < K && n < N) {
                const int64_t o = B_T ? (int64_t)n * ldb + k : (int64_t)k * ldb + n;
                v = B_BF16 ? bf16_to_f32(((const uint16_t *)Bv)[o]) : ((const float *)Bv)[o];
            }
            Bs[kk][nn] = v;
        }
        __syncthreads();
        // each wave: a 32 x 32 quarter of the tile as 2 x 2 MFMA tiles of
        // 16 x 16, four steps of k = 4 per staged chunk.  Operands of
        // v_mfma_f32_16x16x4f32: lane l gives A(row l % 16, k l / 16) and
        // B(k l / 16, column l % 16).
#pragma unroll
        for (int kq = 0; kq < BK; kq += 4) {
            const int kk = kq + lane / 16;
            float a[WT], b[WT];
#pragma unroll
            for (int si = 0; si < WT; ++si) a[si] = As[kk][wm + si * 16 + lane % 16];
#pragma unroll
            for (int sj = 0; sj < WT; ++sj) b[sj] = Bs[kk][wn + sj * 16 + lane % 16];
#pragma unroll
            for (int si = 0; si < WT; ++si)
#pragma unroll
                for (int sj = 0; sj < WT; ++sj)
                    acc[si][sj] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[si], b[sj], acc[si][sj], 0, 0, 0);
        }
        __syncthreads();
    }
    // lane l holds rows 4 (l / 16) + r, column l % 16 of each 16 x 16 tile
#pragma unroll
    for (int si = 0; si < WT; ++si)
#pragma unroll
        for (int sj = 0; sj < WT; ++sj)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int m = m0 + wm + si * 16 + 4 * (lane / 16) + r;
                const int n = n0 + wn + sj * 16 + lane % 16;
                if (m >= M || n >= N) continue;
                const int64_t o = (int64_t)m * ldc + n;
                float v = acc[si][sj][r];
                if (EPI == EPI_BIAS || EPI == EPI_BIAS_GELU) v += bias[n];
                if (EPI == EPI_GELU_GRAD) v *= gelu_grad(aux[o]);
                C[o] = v;
                if (EPI == EPI_BIAS_GELU) C2[o] = gelu(v);
            }
}

template <bool A_T, bool B_T, bool B_BF16, int EPI>
void gemm(hipStream_t s, const float *A, int lda, const void *B, int ldb, int M, int N, int K, float *C,
          int ldc, const float *bias = nullptr, const float *aux = nullptr, float *C2 = nullptr) {
    dim3 grid((N + BN - 1) / BN, (M + BM - 1) / BM);
    hipLaunchKernelGGL((gemm_kernel<A_T, B_T, B_BF16, EPI>), grid, dim3(kGemmThreads), 0, s, A, lda, B, ldb,
                       M, N, K, C, ldc, bias, aux, C2);
}

// Softmax over each row of Z (one wave per row), the row's cross-entropy
// against T, and dZ = (P - T) / B.
__global__ __launch_bounds__(64) void softmax_xent_kernel(const float *__restrict__ Z,
                                                          const float *__restrict__ T, int B, int N,
                                                          float *__restrict__ P, float *__restrict__ dZ,
                                                          float *__restrict__ row_loss) {
    const int b = blockIdx.x;
    const float *z = Z + (int64_t)b * N;
    float mx = -INFINITY;
    for (int j = threadIdx.x; j < N; j += 64) mx = fmaxf(mx, z[j]);
    for (int off = 32; off > 0; off >>= 1) mx = fmaxf(mx, __shfl_xor(mx, off, 64));
    float se = 0.0f;
    for (int j = threadIdx.x; j < N; j += 64) se += expf(z[j] - mx);
    for (int off = 32; off > 0; off >>= 1) se += __shfl_xor(se, off, 64);
    const float lse = logf(se);
    float l = 0.0f;
    for (int j = threadIdx.x; j < N; j += 64) {
        const float logp = z[j] - mx - lse;
        const float p = expf(logp);
        if (P) P[(int64_t)b * N + j] = p;
        if (T) {
            const float t = T[(int64_t)b * N + j];
            l -= t * logp;
            if (dZ) dZ[(int64_t)b * N + j] = (p - t) / (float)B;
        }
    }
    for (int off = 32; off > 0; off >>= 1) l += __shfl_xor(l, off, 64);
    if (row_loss && threadIdx.x == 0) row_loss[b] = l;
}

// out[n] = sum_b X[b][n] in a fixed order: a workgroup takes kSumCols
// columns; thread (column c, group r) sums rows r, r + kSumGroups, ... in
// order, and the groups' partial sums are then added in order of r.
constexpr int kSumCols = 16, kSumGroups = 16;

__global__ __launch_bounds__(kSumCols * kSumGroups) void column_sum_kernel(const float *__restrict__ X, int B,
                                                                           int N, float *__restrict__ out) {
    __shared__ float part[kSumGroups][kSumCols + 1];
    const int c = threadIdx.x % kSumCols, r = threadIdx.x / kSumCols;
    const int n = blockIdx.x * kSumCols + c;
    float s = 0.0f;
    if (n < N)
        for (int b = r; b < B; b += kSumGroups) s += X[(int64_t)b * N + n];
    part[r][c] = s;
    __syncthreads();
    if (r == 0 && n < N) {
        float t = 0.0f;
        for (int g = 0; g < kSumGroups; ++g) t += part[g][c];
        out[n] = t;
    }
}

// Mean of row losses (one workgroup, fixed order).
__global__ void mean_loss_kernel(const float *__restrict__ row_loss, int B, float *__restrict__ loss) {
    __shared__ float part[256];
    float s = 0.0f;
    for (int b = threadIdx.x; b < B; b += 256) s += row_loss[b];
    part[threadIdx.x] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        float t = 0.0f;
        for (int i = 0; i < 256; ++i) t += part[i];
        *loss = t / (float)B;
    }
}

// Adam on FP32 masters; BF16 copies of the weight entries are refreshed.
__global__ void adam_kernel(float *__restrict__ master, uint16_t *__restrict__ w16, const int64_t *__restrict__ w_of,
                            const float *__restrict__ g, float *__restrict__ m, float *__restrict__ v,
                            int64_t n, float lr, float b1, float b2, float eps, float bc1, float bc2) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float p = master[i] - lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
    master[i] = p;
    const int64_t w = w_of[i];
    if (w >= 0) w16[w] = f32_to_bf16(p);
}

__global__ void to_bf16_kernel(const float *__restrict__ master, uint16_t *__restrict__ w16,
                               const int64_t *__restrict__ w_of, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t w = w_of[i];
    if (w >= 0) w16[w] = f32_to_bf16(master[i]);
}

}  // namespace

struct raysh_mlp {
    int device = 0;
    hipStream_t stream = nullptr;
    int n_in = 0, h = 0, n_out = 0, max_batch = 0;
    int64_t n_params = 0, n_weights = 0;
    int64_t off[6] = {};        // offsets of W1, b1, W2, b2, W3, b3 in the flat parameters
    int64_t woff[3] = {};       // offsets of W1, W2, W3 in the BF16 weight array
    int64_t step = 0;
    float *master = nullptr, *grad = nullptr, *m = nullptr, *v = nullptr;
    uint16_t *w16 = nullptr;
    int64_t *w_of = nullptr;    // flat parameter index -> BF16 weight index or -1
    float *Z1 = nullptr, *H1 = nullptr, *Z2 = nullptr, *H2 = nullptr, *Z3 = nullptr, *P = nullptr;
    float *dZ3 = nullptr, *dZ2 = nullptr, *dZ1 = nullptr, *row_loss = nullptr;
    bool has_grad = false;
    std::vector<void *> allocs;
};

namespace {

int mlp_alloc(raysh_mlp *p, void **ptr, size_t bytes) {
    hipError_t e = hipMalloc(ptr, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return set_error(RAYSH_ENOMEM, "raysh_mlp: device allocation of %zu bytes failed", bytes);
    }
    p->allocs.push_back(*ptr);
    return RAYSH_OK;
}

void mlp_release(raysh_mlp *p) {
    for (void *a : p->allocs) (void)hipFree(a);
    p->allocs.clear();
}

int check_batch(const raysh_mlp *p, int32_t batch) {
    if (batch < 1 || batch > p->max_batch)
        return set_error(RAYSH_EINVAL, "batch %d outside [1, %d]", batch, p->max_batch);
    return RAYSH_OK;
}

// Forward pass into the context's activation buffers.
void forward(raysh_mlp *p, const float *x, int B) {
    hipStream_t s = p->stream;
    const float *b1 = p->master + p->off[1], *b2 = p->master + p->off[3], *b3 = p->master + p->off[5];
    gemm<false, false, true, EPI_BIAS_GELU>(s, x, p->n_in, p->w16 + p->woff[0], p->h, B, p->h, p->n_in, p->Z1,
                                            p->h, b1, nullptr, p->H1);
    gemm<false, false, true, EPI_BIAS_GELU>(s, p->H1, p->h, p->w16 + p->woff[1], p->h, B, p->h, p->h, p->Z2,
                                            p->h, b2, nullptr, p->H2);
    gemm<false, false, true, EPI_BIAS>(s, p->H2, p->h, p->w16 + p->woff[2], p->n_out, B, p->n_out, p->h,
                                       p->Z3, p->n_out, b3);
}

}  // namespace

extern "C" {

int raysh_mlp_create(raysh_mlp **out, int device, void *hip_stream, int32_t n_in, int32_t n_hidden,
                     int32_t n_out, int32_t max_batch, const float *params) {
    if (!out) return set_error(RAYSH_EINVAL, "out is NULL");
    if (n_in < 1 || n_hidden < 1 || n_out < 1 || max_batch < 1)
        return set_error(RAYSH_EINVAL, "layer sizes and max_batch must be >= 1");
    if (n_in > 4096 || n_hidden > 4096 || n_out > 4096 || max_batch > (1 << 20))
        return set_error(RAYSH_EINVAL, "layer sizes above 4096 or max_batch above 2^20");
    if (!params) return set_error(RAYSH_EINVAL, "params is NULL");
    const int64_t h = n_hidden;
    const int64_t sizes[6] = {(int64_t)n_in * h, h, h * h, h, h * n_out, n_out};
    int64_t total = 0;
    for (int64_t sz : sizes) total += sz;
    for (int64_t i = 0; i < total; ++i)
        if (!std::isfinite(params[i])) return set_error(RAYSH_EINVAL, "parameter %lld is not finite", (long long)i);
    if (device < 0) return set_error(RAYSH_EINVAL, "device < 0");
    DeviceGuard g(device);
    if (!g.ok) return set_error(RAYSH_EDEVICE, "hipSetDevice(%d) failed", device);

    raysh_mlp *p = new raysh_mlp();
    p->device = device;
    p->stream = (hipStream_t)hip_stream;
    p->n_in = n_in;
    p->h = n_hidden;
    p->n_out = n_out;
    p->max_batch = max_batch;
    p->n_params = total;
    int64_t o = 0;
    for (int i = 0; i < 6; ++i) {
        p->off[i] = o;
        o += sizes[i];
    }
    p->woff[0] = 0;
    p->woff[1] = sizes[0];
    p->woff[2] = sizes[0] + sizes[2];
    p->n_weights = sizes[0] + sizes[2] + sizes[4];
    std::vector<int64_t> w_of(total, -1);
    for (int64_t i = 0; i < sizes[0]; ++i) w_of[p->off[0] + i] = p->woff[0] + i;
    for (int64_t i = 0; i < sizes[2]; ++i) w_of[p->off[2] + i] = p->woff[1] + i;
    for (int64_t i = 0; i < sizes[4]; ++i) w_of[p->off[4] + i] = p->woff[2] + i;

    const int64_t Bh = (int64_t)max_batch * h, Bo = (int64_t)max_batch * n_out;
    int r = RAYSH_OK;
    void *tmp = nullptr;
#define ALLOC(field, type, count)                                            \
    if (r == RAYSH_OK) {                                                     \
        r = mlp_alloc(p, &tmp, (size_t)(count) * sizeof(type));              \
        p->field = (type *)tmp;                                              \
    }
    ALLOC(master, float, total)
    ALLOC(grad, float, total)
    ALLOC(m, float, total)
    ALLOC(v, float, total)
    ALLOC(w16, uint16_t, p->n_weights)
    ALLOC(w_of, int64_t, total)
    ALLOC(Z1, float, Bh)
    ALLOC(H1, float, Bh)
    ALLOC(Z2, float, Bh)
    ALLOC(H2, float, Bh)
    ALLOC(Z3, float, Bo)
    ALLOC(P, float, Bo)
    ALLOC(dZ3, float, Bo)
    ALLOC(dZ2, float, Bh)
    ALLOC(dZ1, float, Bh)
    ALLOC(row_loss, float, max_batch)
#undef ALLOC
    hipError_t e = hipSuccess;
    if (r == RAYSH_OK) {
        e = hipMemcpy(p->master, params, total * sizeof(float), hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(p->w_of, w_of.data(), total * sizeof(int64_t), hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemset(p->m, 0, total * sizeof(float));
        if (e == hipSuccess) e = hipMemset(p->v, 0, total * sizeof(float));
        if (e == hipSuccess) {
            hipLaunchKernelGGL(to_bf16_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, p->stream,
                               p->master, p->w16, p->w_of, total);
            e = hipGetLastError();
        }
        if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
        if (e != hipSuccess) r = hip_error(e, "raysh_mlp_create");
    }
    if (r != RAYSH_OK) {
        mlp_release(p);
        delete p;
        return r;
    }
    *out = p;
    return set_ok();
}

int64_t raysh_mlp_n_params(const raysh_mlp *p) { return p ? p->n_params : 0; }

int raysh_mlp_get_params(const raysh_mlp *p, float *params) {
    if (!p || !params) return set_error(RAYSH_EINVAL, "NULL argument");
    DeviceGuard g(p->device);
    hipError_t e = hipMemcpyAsync(params, p->master, p->n_params * sizeof(float), hipMemcpyDeviceToHost, p->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
    if (e != hipSuccess) return hip_error(e, "raysh_mlp_get_params");
    return set_ok();
}

int raysh_mlp_forward(raysh_mlp *p, const float *x, int32_t batch, float *probs) {
    if (!p) return set_error(RAYSH_EINVAL, "mlp is NULL");
    if (int r = check_batch(p, batch)) return r;
    if (!x || !probs) return set_error(RAYSH_EINVAL, "NULL buffer");
    DeviceGuard g(p->device);
    if (!g.ok) return set_error(RAYSH_EDEVICE, "hipSetDevice(%d) failed", p->device);
    if (int r = validate_device_ptr(x, (size_t)batch * p->n_in * 4, p->device, "x")) return r;
    if (int r = validate_device_ptr(probs, (size_t)batch * p->n_out * 4, p->device, "probs")) return r;
    forward(p, x, batch);
    hipLaunchKernelGGL(softmax_xent_kernel, dim3(batch), dim3(64), 0, p->stream, p->Z3, nullptr, batch, p->n_out,
                       probs, nullptr, nullptr);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_error(e, "raysh_mlp_forward");
    return set_ok();
}

int raysh_mlp_gradient(raysh_mlp *p, const float *x, const float *target, int32_t batch, float *grads,
                       float *loss) {
    if (!p) return set_error(RAYSH_EINVAL, "mlp is NULL");
    if (int r = check_batch(p, batch)) return r;
    if (!x || !target) return set_error(RAYSH_EINVAL, "NULL buffer");
    DeviceGuard g(p->device);
    if (!g.ok) return set_error(RAYSH_EDEVICE, "hipSetDevice(%d) failed", p->device);
    if (int r = validate_device_ptr(x, (size_t)batch * p->n_in * 4, p->device, "x")) return r;
    if (int r = validate_device_ptr(target, (size_t)batch * p->n_out * 4, p->device, "target")) return r;
    if (grads)
        if (int r = validate_device_ptr(grads, (size_t)p->n_params * 4, p->device, "grads")) return r;
    if (loss)
        if (int r = validate_device_ptr(loss, 4, p->device, "loss")) return r;
    hipStream_t s = p->stream;
    const int B = batch, h = p->h, ni = p->n_in, no = p->n_out;
    forward(p, x, B);
    hipLaunchKernelGGL(softmax_xent_kernel, dim3(B), dim3(64), 0, s, p->Z3, target, B, no, p->P, p->dZ3,
                       p->row_loss);
    float *G = p->grad;
    // layer 3
    gemm<true, false, false, EPI_STORE>(s, p->H2, h, p->dZ3, no, h, no, B, G + p->off[4], no);
    hipLaunchKernelGGL(column_sum_kernel, dim3((no + kSumCols - 1) / kSumCols), dim3(kSumCols * kSumGroups), 0,
                       s, p->dZ3, B, no, G + p->off[5]);
    gemm<false, true, true, EPI_GELU_GRAD>(s, p->dZ3, no, p->w16 + p->woff[2], no, B, h, no, p->dZ2, h, nullptr,
                                           p->Z2);
    // layer 2
    gemm<true, false, false, EPI_STORE>(s, p->H1, h, p->dZ2, h, h, h, B, G + p->off[2], h);
    hipLaunchKernelGGL(column_sum_kernel, dim3((h + kSumCols - 1) / kSumCols), dim3(kSumCols * kSumGroups), 0,
                       s, p->dZ2, B, h, G + p->off[3]);
    gemm<false, true, true, EPI_GELU_GRAD>(s, p->dZ2, h, p->w16 + p->woff[1], h, B, h, h, p->dZ1, h, nullptr,
                                           p->Z1);
    // layer 1
    gemm<true, false, false, EPI_STORE>(s, x, ni, p->dZ1, h, ni, h, B, G + p->off[0], h);
    hipLaunchKernelGGL(column_sum_kernel, dim3((h + kSumCols - 1) / kSumCols), dim3(kSumCols * kSumGroups), 0,
                       s, p->dZ1, B, h, G + p->off[1]);
    if (loss) hipLaunchKernelGGL(mean_loss_kernel, dim3(1), dim3(256), 0, s, p->row_loss, B, loss);
    if (grads) {
        hipError_t e = hipMemcpyAsync(grads, G, p->n_params * sizeof(float), hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess) return hip_error(e, "raysh_mlp_gradient");
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_error(e, "raysh_mlp_gradient");
    p->has_grad = true;
    return set_ok();
}

int raysh_mlp_adam_step(raysh_mlp *p, float lr, float beta1, float beta2, float eps) {
    if (!p) return set_error(RAYSH_EINVAL, "mlp is NULL");
    if (!p->has_grad) return set_error(RAYSH_EINVAL, "no gradient computed yet");
    if (!(std::isfinite(lr) && lr > 0) || !(beta1 >= 0 && beta1 < 1) || !(beta2 >= 0 && beta2 < 1) ||
        !(std::isfinite(eps) && eps >= 0))
        return set_error(RAYSH_EINVAL, "Adam hyper-parameters out of range");
    DeviceGuard g(p->device);
    if (!g.ok) return set_error(RAYSH_EDEVICE, "hipSetDevice(%d) failed", p->device);
    p->step += 1;
    const float bc1 = (float)(1.0 - std::pow((double)beta1, (double)p->step));
    const float bc2 = (float)(1.0 - std::pow((double)beta2, (double)p->step));
    hipLaunchKernelGGL(adam_kernel, dim3((unsigned)((p->n_params + 255) / 256)), dim3(256), 0, p->stream,
                       p->master, p->w16, p->w_of, p->grad, p->m, p->v, p->n_params, lr, beta1, beta2, eps, bc1,
                       bc2);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_error(e, "raysh_mlp_adam_step");
    return set_ok();
}

int raysh_mlp_train_step(raysh_mlp *p, const float *x, const float *target, int32_t batch, float lr,
                         float beta1, float beta2, float eps, float *loss) {
    if (int r = raysh_mlp_gradient(p, x, target, batch, nullptr, loss)) return r;
    return raysh_mlp_adam_step(p, lr, beta1, beta2, eps);
}

int raysh_mlp_sync(raysh_mlp *p) {
    if (!p) return set_error(RAYSH_EINVAL, "mlp is NULL");
    DeviceGuard g(p->device);
    hipError_t e = hipStreamSynchronize(p->stream);
    if (e != hipSuccess) return hip_error(e, "raysh_mlp_sync");
    return set_ok();
}

int raysh_mlp_free(raysh_mlp *p) {
    if (!p) return set_ok();
    {
        DeviceGuard g(p->device);
        (void)hipStreamSynchronize(p->stream);
        mlp_release(p);
    }
    delete p;
    return set_ok();
}

}  // extern "C"
