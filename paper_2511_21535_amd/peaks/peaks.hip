// Microbenchmarks for measured roofline denominators: FP32 FMA issue,
// v_rsq_f32 issue and FP32 matrix-core throughput, each a long loop of
// independent operations with one store per thread at the end.
#include <hip/hip_runtime.h>

#include "p2p_peaks.h"

namespace {

constexpr int kBlock = 256;

__global__ __launch_bounds__(kBlock) void k_peak_fma(float *__restrict__ out, int iters, float a, float b) {
    float x[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) x[k] = static_cast<float>(threadIdx.x + k) * 1e-3f;
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int u = 0; u < 16; ++u) {
#pragma unroll
            for (int k = 0; k < 8; ++k) x[k] = fmaf(x[k], a, b);
        }
    }
    float s = 0.f;
#pragma unroll
    for (int k = 0; k < 8; ++k) s += x[k];
    out[static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x] = s;
}

__global__ __launch_bounds__(kBlock) void k_peak_rsq(float *__restrict__ out, int iters, float a) {
    float x[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) x[k] = a + static_cast<float>(threadIdx.x + k);
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int u = 0; u < 8; ++u) {
#pragma unroll
            for (int k = 0; k < 8; ++k) x[k] = __builtin_amdgcn_rsqf(x[k]);
        }
    }
    float s = 0.f;
#pragma unroll
    for (int k = 0; k < 8; ++k) s += x[k];
    out[static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x] = s;
}

typedef float f32x4 __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(kBlock) void k_peak_mfma(float *__restrict__ out, int iters, float a) {
    const float p = a * static_cast<float>(threadIdx.x & 63), q = 1.0f - p;
    f32x4 c[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) c[k] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int u = 0; u < 8; ++u) {
#pragma unroll
            for (int k = 0; k < 4; ++k) c[k] = __builtin_amdgcn_mfma_f32_16x16x4f32(p, q, c[k], 0, 0, 0);
        }
    }
    float s = 0.f;
#pragma unroll
    for (int k = 0; k < 4; ++k) s += c[k][0] + c[k][1] + c[k][2] + c[k][3];
    out[static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x] = s;
}

bool bad(const float *out, int64_t blocks, int32_t iters) {
    return out == nullptr || blocks < 1 || blocks > 0x7fffffff || iters < 1;
}

}  // namespace

extern "C" int p2pk_valu_fma(float *out, int64_t blocks, int32_t iters, void *stream) {
    if (bad(out, blocks, iters)) return -1;
    k_peak_fma<<<static_cast<unsigned>(blocks), kBlock, 0, static_cast<hipStream_t>(stream)>>>(
        out, iters, 0.999999f, 1e-7f);
    return static_cast<int>(hipGetLastError());
}

extern "C" int p2pk_valu_rsq(float *out, int64_t blocks, int32_t iters, void *stream) {
    if (bad(out, blocks, iters)) return -1;
    k_peak_rsq<<<static_cast<unsigned>(blocks), kBlock, 0, static_cast<hipStream_t>(stream)>>>(out, iters, 2.0f);
    return static_cast<int>(hipGetLastError());
}

extern "C" int p2pk_mfma_f32(float *out, int64_t blocks, int32_t iters, void *stream) {
    if (bad(out, blocks, iters)) return -1;
    k_peak_mfma<<<static_cast<unsigned>(blocks), kBlock, 0, static_cast<hipStream_t>(stream)>>>(out, iters,
                                                                                              1e-3f);
    return static_cast<int>(hipGetLastError());
}
