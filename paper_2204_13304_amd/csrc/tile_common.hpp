// tile_common.hpp -- device helpers shared by the tiled wavefront sweep
// kernels: raw buffer loads and stores with out-of-range offsets (which read
// 0 and drop stores), and the epoch-tagged boundary records through which
// neighbouring tiles hand over their boundary rows.
#pragma once

#include <hip/hip_runtime.h>

namespace m2s {

// Raw buffer load; a byte offset at or past the end of the buffer reads 0.
template <typename T>
__device__ __forceinline__ T buf_load(__amdgpu_buffer_rsrc_t rs, unsigned off)
{
    if constexpr (sizeof(T) == 8)
        return __builtin_bit_cast(
            T, __builtin_amdgcn_raw_buffer_load_b64(rs, (int)off, 0, 0));
    else
        return __builtin_bit_cast(
            T, __builtin_amdgcn_raw_buffer_load_b32(rs, (int)off, 0, 0));
}

// Boundary-store record: a value tagged with the launch epoch.  For FP64
// the record is {lo, epoch, hi, epoch}: each 8-byte half is written and
// read as one unit, so matching epochs in both halves mean both halves of
// the value are from this launch.  FP32: {value, epoch}.
template <typename T>
struct Rec;
template <>
struct Rec<double> {
    using V = __attribute__((ext_vector_type(4))) unsigned;
    static constexpr unsigned bytes = 16;
    __device__ static V make(double v, unsigned ep)
    {
        const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
        return V{(unsigned)b, ep, (unsigned)(b >> 32), ep};
    }
    __device__ static bool ready(V r, unsigned ep)
    {
        return r.y == ep && r.w == ep;
    }
    __device__ static double value(V r)
    {
        return __builtin_bit_cast(
            double, (unsigned long long)r.x | ((unsigned long long)r.z << 32));
    }
    __device__ static V load(__amdgpu_buffer_rsrc_t rs, unsigned off)
    {
        return __builtin_amdgcn_raw_buffer_load_b128(rs, (int)off, 0, 16);
    }
    __device__ static void store(__amdgpu_buffer_rsrc_t rs, unsigned off, V r)
    {
        __builtin_amdgcn_raw_buffer_store_b128(r, rs, (int)off, 0, 16);
    }
};
template <>
struct Rec<float> {
    using V = __attribute__((ext_vector_type(2))) unsigned;
    static constexpr unsigned bytes = 8;
    __device__ static V make(float v, unsigned ep)
    {
        return V{__builtin_bit_cast(unsigned, v), ep};
    }
    __device__ static bool ready(V r, unsigned ep) { return r.y == ep; }
    __device__ static float value(V r)
    {
        return __builtin_bit_cast(float, r.x);
    }
    __device__ static V load(__amdgpu_buffer_rsrc_t rs, unsigned off)
    {
        return __builtin_amdgcn_raw_buffer_load_b64(rs, (int)off, 0, 16);
    }
    __device__ static void store(__amdgpu_buffer_rsrc_t rs, unsigned off, V r)
    {
        __builtin_amdgcn_raw_buffer_store_b64(r, rs, (int)off, 0, 16);
    }
};

// Raw buffer store; a byte offset at or past the end of the buffer is
// dropped.  aux 16 sets sc1: the store is made coherent at device scope,
// like an agent-scope atomic store.
template <typename T, int AUX>
__device__ __forceinline__ void buf_store(__amdgpu_buffer_rsrc_t rs,
                                          unsigned off, T v)
{
    if constexpr (sizeof(T) == 8)
        __builtin_amdgcn_raw_buffer_store_b64(
            __builtin_bit_cast(__attribute__((ext_vector_type(2))) unsigned,
                               v),
            rs, (int)off, 0, AUX);
    else
        __builtin_amdgcn_raw_buffer_store_b32(
            __builtin_bit_cast(unsigned, v), rs, (int)off, 0, AUX);
}

}  // namespace m2s
