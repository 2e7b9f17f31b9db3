// probe.hip -- measured peaks of the units the library's kernels are bound
// by, for rooflines against what this device sustains beside the datasheet:
// HBM (a plain copy), the FP32 VALU (FMA chains in three encodings, packed
// FP32 off like every kernel here), the transcendental unit (exp2), and the
// MFMA pipes the library uses (BF16 16x16x32, FP32 16x16x4, FP64 16x16x4).
//
// Each compute probe runs 8 wavefronts per SIMD on every CU with independent
// accumulator chains, so issue and not latency bounds it; the results are
// summed into one store per lane so that nothing is eliminated.  Times are
// HIP events around one launch after a warm-up launch.
#include "gpdf_internal.hpp"

using namespace gpdf;

namespace {

typedef __bf16 pbf16x8 __attribute__((ext_vector_type(8)));
typedef float pf32x4 __attribute__((ext_vector_type(4)));
typedef double pf64x4 __attribute__((ext_vector_type(4)));

constexpr int kProbeT = 256;
constexpr unsigned kProbeBlocks = 256 * 8;   // 8 wavefronts per SIMD on 256 CUs (4 SIMDs, 256-thread blocks)

__global__ __launch_bounds__(kProbeT) void k_probe_copy(const float4 *__restrict__ a, float4 *__restrict__ b,
                                                        int64_t n) {
    const int64_t stride = int64_t(gridDim.x) * blockDim.x;
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride) b[i] = a[i];
}

// 16 independent FMA chains per lane, `iters` rounds, in three encodings:
//   FORM 0  v = fma(a, b, v), a and b per-lane registers: v_fmac_f32 (VOP2)
//   FORM 1  v = fma(v, a, c), a and c per-lane registers: v_fma_f32 (VOP3)
//   FORM 2  v = fma(v, K, c), K a compile-time constant: v_fmamk_f32 (VOP2
//           with a literal)
template <int FORM>
__global__ __launch_bounds__(kProbeT) void k_probe_fma(float *out, int iters, float x) {
    float v[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) v[k] = x + float(k) * 1e-3f + float(threadIdx.x) * 1e-6f;
    const float a = 0.999f + float(threadIdx.x) * 1e-9f, b = 1e-4f + float(threadIdx.x) * 1e-12f;
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            if constexpr (FORM == 0) v[k] = fmaf(a, b, v[k]);
            else if constexpr (FORM == 1) v[k] = fmaf(v[k], a, b);
            else v[k] = fmaf(v[k], 0.999f, b);
        }
    }
    float s = 0.f;
#pragma unroll
    for (int k = 0; k < 16; ++k) s += v[k];
    out[int64_t(blockIdx.x) * blockDim.x + threadIdx.x] = s;
}

// 8 independent exp2 chains per lane: v <- 2^-v (the negation is a source
// modifier of the instruction, so every instruction of the loop is an exp2;
// the chains converge to about 0.64 and stay finite)
__global__ __launch_bounds__(kProbeT) void k_probe_exp(float *out, int iters, float x) {
    float v[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) v[k] = x - float(k) * 1e-3f - float(threadIdx.x) * 1e-7f;
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int k = 0; k < 8; ++k) v[k] = __builtin_amdgcn_exp2f(-v[k]);
    }
    float s = 0.f;
#pragma unroll
    for (int k = 0; k < 8; ++k) s += v[k];
    out[int64_t(blockIdx.x) * blockDim.x + threadIdx.x] = s;
}

// 4 independent accumulators per wavefront for each MFMA shape
__global__ __launch_bounds__(kProbeT) void k_probe_mfma_bf16(float *out, int iters) {
    pbf16x8 a, b;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        a[k] = (__bf16)(1e-3f * float(k + (threadIdx.x & 7)));
        b[k] = (__bf16)(1e-3f * float(k + 1));
    }
    pf32x4 acc[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[j] = pf32x4{0.f, 0.f, 0.f, 0.f};
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[j], 0, 0, 0);
    }
    float s = 0.f;
#pragma unroll
    for (int j = 0; j < 4; ++j) s += acc[j][0] + acc[j][1] + acc[j][2] + acc[j][3];
    out[int64_t(blockIdx.x) * blockDim.x + threadIdx.x] = s;
}

__global__ __launch_bounds__(kProbeT) void k_probe_mfma_f32(float *out, int iters) {
    const float a = 1e-3f * float(threadIdx.x & 15), b = 1e-3f;
    pf32x4 acc[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[j] = pf32x4{0.f, 0.f, 0.f, 0.f};
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc[j], 0, 0, 0);
    }
    float s = 0.f;
#pragma unroll
    for (int j = 0; j < 4; ++j) s += acc[j][0] + acc[j][1] + acc[j][2] + acc[j][3];
    out[int64_t(blockIdx.x) * blockDim.x + threadIdx.x] = s;
}

__global__ __launch_bounds__(kProbeT) void k_probe_mfma_f64(float *out, int iters) {
    const double a = 1e-3 * double(threadIdx.x & 15), b = 1e-3;
    pf64x4 acc[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[j] = pf64x4{0.0, 0.0, 0.0, 0.0};
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[j], 0, 0, 0);
    }
    double s = 0.0;
#pragma unroll
    for (int j = 0; j < 4; ++j) s += acc[j][0] + acc[j][1] + acc[j][2] + acc[j][3];
    out[int64_t(blockIdx.x) * blockDim.x + threadIdx.x] = float(s);
}

template <class F>
hipError_t time_launch(hipStream_t s, F &&launch, float *ms) {
    hipEvent_t a, b;
    hipError_t e;
    if ((e = hipEventCreate(&a)) != hipSuccess) return e;
    if ((e = hipEventCreate(&b)) != hipSuccess) {
        (void)hipEventDestroy(a);
        return e;
    }
    launch();   // warm-up
    (void)hipEventRecord(a, s);
    launch();
    (void)hipEventRecord(b, s);
    if ((e = hipEventSynchronize(b)) == hipSuccess) e = hipEventElapsedTime(ms, a, b);
    if (e == hipSuccess) e = hipGetLastError();
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    return e;
}

}  // namespace

// h_out[9] receives: HBM copy GB/s (bytes read + written), FP32 FMA
// TFLOP/s (an FMA is 2 flop) in the VOP2 register form, exp2 Gop/s, BF16,
// FP32 and FP64 MFMA TFLOP/s, the copy size in GiB, FP32 FMA TFLOP/s in the
// VOP3 form and in the VOP2 literal form.
extern "C" gpdf_status gpdf_measure_peaks(gpdf_ctx *c, double *h_out, int32_t n_out) {
    if (!c || !h_out || n_out < 9) return GPDF_E_INVALID_ARG;
    if (hipError_t je = join_train(c); je != hipSuccess) return hip_fail(c, je, "join");
    hipStream_t s = c->stream;
    hipError_t e;
    const int64_t nvec = int64_t(1) << 26;   // 1 GiB of float4
    float4 *a = nullptr, *b = nullptr;
    float *out = nullptr;
    const int64_t nthreads = int64_t(kProbeBlocks) * kProbeT;
    if ((e = hipMallocAsync((void **)&a, sizeof(float4) * nvec, s)) != hipSuccess ||
        (e = hipMallocAsync((void **)&b, sizeof(float4) * nvec, s)) != hipSuccess ||
        (e = hipMallocAsync((void **)&out, sizeof(float) * nthreads, s)) != hipSuccess)
        return hip_fail(c, e, "measure_peaks: allocate");
    (void)hipMemsetAsync(a, 0, sizeof(float4) * nvec, s);
    float ms[8] = {};
    const int it_fma = 4096, it_exp = 2048, it_mfma = 2048;
    if ((e = time_launch(s, [&] {
             hipLaunchKernelGGL(k_probe_copy, dim3(8192), dim3(kProbeT), 0, s, a, b, nvec);
         }, &ms[0])) != hipSuccess ||
        (e = time_launch(s, [&] {
             hipLaunchKernelGGL(k_probe_fma<0>, dim3(kProbeBlocks), dim3(kProbeT), 0, s, out, it_fma, 0.5f);
         }, &ms[1])) != hipSuccess ||
        (e = time_launch(s, [&] {
             hipLaunchKernelGGL(k_probe_fma<1>, dim3(kProbeBlocks), dim3(kProbeT), 0, s, out, it_fma, 0.5f);
         }, &ms[6])) != hipSuccess ||
        (e = time_launch(s, [&] {
             hipLaunchKernelGGL(k_probe_fma<2>, dim3(kProbeBlocks), dim3(kProbeT), 0, s, out, it_fma, 0.5f);
         }, &ms[7])) != hipSuccess ||
        (e = time_launch(s, [&] {
             hipLaunchKernelGGL(k_probe_exp, dim3(kProbeBlocks), dim3(kProbeT), 0, s, out, it_exp, 0.25f);
         }, &ms[2])) != hipSuccess ||
        (e = time_launch(s, [&] {
             hipLaunchKernelGGL(k_probe_mfma_bf16, dim3(kProbeBlocks), dim3(kProbeT), 0, s, out, it_mfma);
         }, &ms[3])) != hipSuccess ||
        (e = time_launch(s, [&] {
             hipLaunchKernelGGL(k_probe_mfma_f32, dim3(kProbeBlocks), dim3(kProbeT), 0, s, out, it_mfma);
         }, &ms[4])) != hipSuccess ||
        (e = time_launch(s, [&] {
             hipLaunchKernelGGL(k_probe_mfma_f64, dim3(kProbeBlocks), dim3(kProbeT), 0, s, out, it_mfma);
         }, &ms[5])) != hipSuccess) {
        (void)hipFreeAsync(a, s);
        (void)hipFreeAsync(b, s);
        (void)hipFreeAsync(out, s);
        return hip_fail(c, e, "measure_peaks: run");
    }
    (void)hipFreeAsync(a, s);
    (void)hipFreeAsync(b, s);
    (void)hipFreeAsync(out, s);
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_fail(c, e, "measure_peaks: sync");
    const double waves = double(nthreads) / 64.0;
    h_out[0] = 2.0 * 16.0 * double(nvec) / (ms[0] * 1e-3) / 1e9;
    h_out[1] = double(nthreads) * 16.0 * it_fma * 2.0 / (ms[1] * 1e-3) / 1e12;
    h_out[2] = double(nthreads) * 8.0 * it_exp / (ms[2] * 1e-3) / 1e9;
    h_out[3] = waves * 4.0 * it_mfma * (2.0 * 16 * 16 * 32) / (ms[3] * 1e-3) / 1e12;
    h_out[4] = waves * 4.0 * it_mfma * (2.0 * 16 * 16 * 4) / (ms[4] * 1e-3) / 1e12;
    h_out[5] = waves * 4.0 * it_mfma * (2.0 * 16 * 16 * 4) / (ms[5] * 1e-3) / 1e12;
    h_out[6] = double(sizeof(float4) * nvec) / double(1 << 30);
    h_out[7] = double(nthreads) * 16.0 * it_fma * 2.0 / (ms[6] * 1e-3) / 1e12;
    h_out[8] = double(nthreads) * 16.0 * it_fma * 2.0 / (ms[7] * 1e-3) / 1e12;
    return GPDF_OK;
}
