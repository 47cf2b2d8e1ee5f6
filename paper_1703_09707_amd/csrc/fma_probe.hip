// A measurement aid, not part of the method: a kernel whose instruction
// count is known in advance, to check what the VALU counters of a profiler
// count (wave instructions per FMA, and the factor of 64 lanes and 2 FLOP
// that turns them into FLOPs) and what FMA rate a box sustains at the clock
// it holds under full FP64 or FP32 load.
//
// Each lane keeps kChains independent FMA chains a <- a * b + c (b and c are
// kernel arguments, so no multiply or add can be folded) for n_iter steps,
// then adds its chains and stores one value: per wave, exactly
// kChains * n_iter v_fma instructions of the chosen precision, kChains - 1
// adds and no other floating-point arithmetic.  With a_0 = lane index +
// chain index, b = 1 and c = 1 every step is exact, so the stored value is
// known: sum over chains of (lane + chain + n_iter).
#include <limits>

#include "raysh_ctx.h"

namespace {

constexpr int kProbeThreads = 256;
constexpr int kChains = 8;   // independent chains hide the FMA latency

__device__ __forceinline__ double fma_of(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float fma_of(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

template <typename T>
__global__ __launch_bounds__(kProbeThreads) void fma_probe_kernel(int n_iter, T b, T c, T *__restrict__ out) {
    const int lane = threadIdx.x % 64;
    T a[kChains];
#pragma unroll
    for (int i = 0; i < kChains; ++i) a[i] = (T)(lane + i);
    for (int it = 0; it < n_iter; ++it) {
#pragma unroll
        for (int i = 0; i < kChains; ++i) a[i] = fma_of(a[i], b, c);
    }
    T s = a[0];
#pragma unroll
    for (int i = 1; i < kChains; ++i) s = s + a[i];
    out[(int64_t)blockIdx.x * kProbeThreads + threadIdx.x] = s;
}

}  // namespace

extern "C" int raysh_fma_probe(int precision, int64_t n_blocks, int32_t n_iter, void *out, void *hip_stream) {
    if (precision != RAYSH_FP64 && precision != RAYSH_FP32_BULK)
        return set_error(RAYSH_EINVAL, "raysh_fma_probe: precision must be RAYSH_FP64 or RAYSH_FP32_BULK");
    if (n_blocks < 1 || n_blocks > std::numeric_limits<int32_t>::max())
        return set_error(RAYSH_EINVAL, "raysh_fma_probe: n_blocks outside [1, 2^31-1]");
    if (n_iter < 1) return set_error(RAYSH_EINVAL, "raysh_fma_probe: n_iter < 1");
    if (!out) return set_error(RAYSH_EINVAL, "raysh_fma_probe: out is NULL");
    hipPointerAttribute_t attr{};
    if (hipPointerGetAttributes(&attr, out) != hipSuccess) {
        (void)hipGetLastError();
        return set_error(RAYSH_EINVAL, "raysh_fma_probe: out is not device memory");
    }
    const int device = attr.device;
    DeviceGuard g(device);
    if (!g.ok) return set_error(RAYSH_EDEVICE, "hipSetDevice(%d) failed", device);
    const size_t elem = precision == RAYSH_FP64 ? sizeof(double) : sizeof(float);
    if (int r = validate_device_ptr(out, (size_t)n_blocks * kProbeThreads * elem, device, "out")) return r;
    hipStream_t s = (hipStream_t)hip_stream;
    if (precision == RAYSH_FP64)
        hipLaunchKernelGGL(fma_probe_kernel<double>, dim3((unsigned)n_blocks), dim3(kProbeThreads), 0, s, n_iter,
                           1.0, 1.0, (double *)out);
    else
        hipLaunchKernelGGL(fma_probe_kernel<float>, dim3((unsigned)n_blocks), dim3(kProbeThreads), 0, s, n_iter,
                           1.0f, 1.0f, (float *)out);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_error(e, "raysh_fma_probe");
    return set_ok();
}
