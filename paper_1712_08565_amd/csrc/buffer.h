// Raw buffer loads for gfx950 (internal): the base address and a per-plane
// byte offset live in scalar registers, the lane's byte offset in a vector
// register, so streaming loads need no 64-bit vector address arithmetic.
// Offsets are unsigned 32-bit bytes and every caller keeps base + scalar offset
// + vector offset inside the resource's allocation (no reliance on the range
// check of raw buffers).
#pragma once

#include <hip/hip_runtime.h>

namespace wqfd {

// word 3 of the resource descriptor for gfx9-family raw buffers
constexpr int kBufferWord3 = 0x00020000;

__device__ inline __amdgpu_buffer_rsrc_t buf_rsrc(const void* base) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, -1, kBufferWord3);
}

template <typename T>
__device__ inline T buf_load(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff) {
    if constexpr (sizeof(T) == 8)
        return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(r, (int)voff, (int)soff, 0));
    else
        return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(r, (int)voff, (int)soff, 0));
}

}  // namespace wqfd
