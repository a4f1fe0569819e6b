// Achievable-peak probes of the GPU the library runs on, so that rooflines are measured,
// not only quoted (the paper measures its GPU's attainable bandwidth with a DAXPY for the
// same purpose, Sec. 6):
//   * STREAM triad a = b + s c over FP64 arrays much larger than the caches (24 bytes of
//     HBM traffic per element);
//   * matrix-core throughput: every wave of a full grid issues long chains of independent
//     16x16x4 MFMA products in FP32 or FP64 (2048 flops each), no memory traffic;
//   * co-execution: the same products, independent FP32 vector FMAs, or both in every wave,
//     timed apart, to see whether the two kinds of work overlap on a SIMD.
#include <hip/hip_runtime.h>

#include "hw_kernels.h"

namespace {

__global__ void __launch_bounds__(256) k_triad(double* __restrict__ a, const double* __restrict__ b,
                                               const double* __restrict__ c, double s, int64_t n)
{
    // two doubles per lane per access (16-byte loads and stores)
    const int64_t n2 = n / 2;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    auto* a2 = reinterpret_cast<double2*>(a);
    auto* b2 = reinterpret_cast<const double2*>(b);
    auto* c2 = reinterpret_cast<const double2*>(c);
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n2; i += stride) {
        const double2 x = b2[i], y = c2[i];
        a2[i] = make_double2(x.x + s * y.x, x.y + s * y.y);
    }
}

typedef float f4 __attribute__((ext_vector_type(4)));
typedef double d4 __attribute__((ext_vector_type(4)));

// CH independent accumulation chains per wave, `iters` rounds; the result is written so
// that the products are not removed
template <typename T, int CH>
__global__ void __launch_bounds__(256) k_mfma(T* __restrict__ sink, int iters)
{
    typedef T vec __attribute__((ext_vector_type(4)));
    const T a = T(1) + T(threadIdx.x) * T(1e-7), b = T(1) - T(threadIdx.x) * T(1e-7);
    vec acc[CH];
#pragma unroll
    for (int c = 0; c < CH; ++c) acc[c] = vec{T(c), T(0), T(0), T(0)};
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int c = 0; c < CH; ++c) {
            if constexpr (sizeof(T) == 4) acc[c] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc[c], 0, 0, 0);
            else acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[c], 0, 0, 0);
        }
    }
    T s = T(0);
#pragma unroll
    for (int c = 0; c < CH; ++c) s += acc[c][0] + acc[c][1] + acc[c][2] + acc[c][3];
    sink[(int64_t)blockIdx.x * blockDim.x + threadIdx.x] = s;
}

// MODE 0: 4 independent FP32 products per round; 1: 32 independent FP32 FMAs per round
// (about the issue time of one product); 2: both
template <int MODE>
__global__ void __launch_bounds__(256) k_coexec(float* __restrict__ sink, int iters)
{
    const float a = 1.0f + threadIdx.x * 1e-7f, b = 1.0f - threadIdx.x * 1e-7f;
    f4 acc[4];
    float v[16];
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[c] = f4{float(c), 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int c = 0; c < 16; ++c) v[c] = threadIdx.x * 1e-3f + c;
    for (int it = 0; it < iters; ++it) {
        if (MODE != 1) {
#pragma unroll
            for (int c = 0; c < 4; ++c) acc[c] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc[c], 0, 0, 0);
        }
        if (MODE != 0) {
#pragma unroll
            for (int r = 0; r < 2; ++r)
#pragma unroll
                for (int c = 0; c < 16; ++c) v[c] = __builtin_fmaf(v[c], a, b);
        }
    }
    float s = 0.0f;
#pragma unroll
    for (int c = 0; c < 4; ++c) s += acc[c][0] + acc[c][1] + acc[c][2] + acc[c][3];
#pragma unroll
    for (int c = 0; c < 16; ++c) s += v[c];
    sink[(int64_t)blockIdx.x * blockDim.x + threadIdx.x] = s;
}

} // namespace

hipError_t hw_probe_coexec_launch(int mode, float* sink, int groups, int iters, hipStream_t st)
{
    if (groups < 1 || iters < 1) return hipErrorInvalidValue;
    if (mode == 0) hipLaunchKernelGGL(k_coexec<0>, dim3(groups), dim3(256), 0, st, sink, iters);
    else if (mode == 1) hipLaunchKernelGGL(k_coexec<1>, dim3(groups), dim3(256), 0, st, sink, iters);
    else if (mode == 2) hipLaunchKernelGGL(k_coexec<2>, dim3(groups), dim3(256), 0, st, sink, iters);
    else return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t hw_probe_triad_launch(double* a, const double* b, const double* c, int64_t n, hipStream_t st)
{
    if (n < 2 || (n & 1)) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_triad, dim3(256 * 16), dim3(256), 0, st, a, b, c, 3.0, n);
    return hipGetLastError();
}

hipError_t hw_probe_mfma_launch(bool fp64, void* sink, int groups, int iters, hipStream_t st)
{
    if (groups < 1 || iters < 1) return hipErrorInvalidValue;
    if (fp64) hipLaunchKernelGGL((k_mfma<double, 8>), dim3(groups), dim3(256), 0, st, (double*)sink, iters);
    else hipLaunchKernelGGL((k_mfma<float, 8>), dim3(groups), dim3(256), 0, st, (float*)sink, iters);
    return hipGetLastError();
}
