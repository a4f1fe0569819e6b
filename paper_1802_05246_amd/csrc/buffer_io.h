// Device helpers of the kernels that address node arrays one row or layer at a time
// (kernel_cmap2d.hip, kernel_cmap3d.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

// Buffer loads and stores of one element at a 32-bit byte offset from a buffer resource
// (a wave-uniform 64-bit base and a size, in scalar registers): the per-lane address is the
// offset alone, with no 64-bit vector arithmetic per access.  Offsets past the size read
// zero and drop stores.
__device__ inline __amdgpu_buffer_rsrc_t make_rsrc(const void* base, uint32_t bytes)
{
    // gfx9 resource word 3: raw (untyped) 32-bit elements
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, 0x00020000);
}
template <typename T>
struct BufIO;
template <>
struct BufIO<float> {
    static __device__ inline float load(__amdgpu_buffer_rsrc_t r, uint32_t o)
    {
        return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, o, 0, 0));
    }
    static __device__ inline void store(float v, __amdgpu_buffer_rsrc_t r, uint32_t o)
    {
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, o, 0, 0);
    }
};
template <>
struct BufIO<double> {
    typedef unsigned int W __attribute__((ext_vector_type(2)));
    static __device__ inline double load(__amdgpu_buffer_rsrc_t r, uint32_t o)
    {
        return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, o, 0, 0));
    }
    static __device__ inline void store(double v, __amdgpu_buffer_rsrc_t r, uint32_t o)
    {
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(W, v), r, o, 0, 0);
    }
};

} // namespace
