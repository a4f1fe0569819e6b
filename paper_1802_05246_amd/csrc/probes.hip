// Achievable-peak probes of the GPU the library runs on, so that rooflines are measured,
// not only quoted (the paper measures its GPU's attainable bandwidth with a DAXPY for the
// same purpose, Sec. 6):
//   * STREAM triad a = b + s c over FP64 arrays much larger than the caches (24 bytes of
//     HBM traffic per element);
//   * matrix-core throughput: every wave of a full grid issues long chains of independent
//     16x16x4 MFMA products in FP32 or FP64 (2048 flops each), no memory traffic.
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

} // namespace

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
