// Raw buffer stores for gfx950 (internal): the counterpart of buf_load in
// buffer.h (vector stores; base and plane offset in scalar registers, the
// lane's byte offset in a vector register).
#pragma once

#include "buffer.h"

namespace wqfd {

template <typename T>
__device__ inline void buf_store(T v, __amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff) {
    if constexpr (sizeof(T) == 8) {
        using V = decltype(__builtin_amdgcn_raw_buffer_load_b64(r, 0, 0, 0));
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(V, v), r, (int)voff, (int)soff, 0);
    } else {
        using V = decltype(__builtin_amdgcn_raw_buffer_load_b32(r, 0, 0, 0));
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(V, v), r, (int)voff, (int)soff, 0);
    }
}

}  // namespace wqfd
