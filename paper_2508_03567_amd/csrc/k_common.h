// Layout helpers used by the interleaved decoders.
#pragma once

#include <algorithm>

#include "ldpcx_internal.h"

namespace ldpcx {

// out[c * ld_out + r] = (r < rows) ? in[r * ld_in + c] : 0 for r < rows_out, c < cols.
template <typename T>
hipError_t transpose(const T *in, long rows, long cols, long ld_in, T *out, long rows_out, long ld_out,
                     hipStream_t s);

// Fill `bytes` (multiple of 4) with a 32-bit pattern.
hipError_t fill_u32(void *p, size_t bytes, uint32_t v, hipStream_t s);

// Wave-wide OR of a 64-bit value (all lanes receive the result).
__device__ __forceinline__ uint64_t wave_or64(uint64_t v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v |= __shfl_xor(v, o, 64);
    return v;
}

}  // namespace ldpcx
