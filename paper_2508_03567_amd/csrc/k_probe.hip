// Device peak probe for the integer rooflines: the packed 16-bit VALU issue rate.
//
// Every lane runs `iters` rounds of 8 independent chains, each round one packed add
// and one packed max per chain (16 VALU instructions), so the issue rate of a full
// device of such waves is the VALU peak the Min-Max and min-sum kernels are quoted
// against (spec: 256 CUs x 4 SIMDs x 2.4 GHz / 4 cycles per wave instruction).
#include <hip/hip_runtime.h>

#include "runtime.h"

namespace {

typedef short v2 __attribute__((ext_vector_type(2)));

__global__ void __launch_bounds__(256) k_valu_probe(int iters, uint32_t seed, uint32_t *out) {
    v2 a[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) a[j] = __builtin_bit_cast(v2, seed ^ (threadIdx.x * 0x9E3779B9u) ^ (uint32_t)j);
    const v2 d = __builtin_bit_cast(v2, seed | 0x00010001u), b = __builtin_bit_cast(v2, seed * 3u);
#pragma unroll 4
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int j = 0; j < 8; ++j) a[j] = __builtin_elementwise_max(a[j] + d, b);
    }
    uint32_t x = 0;
#pragma unroll
    for (int j = 0; j < 8; ++j) x ^= __builtin_bit_cast(uint32_t, a[j]);
    if (x == seed) out[blockIdx.x & 63] = x;  // keeps the chains live; practically never taken
}

}  // namespace

using namespace ldpcx;

extern "C" ldpcx_status ldpcx_valu_probe(int32_t blocks, int32_t iters, void *stream) {
    if (blocks < 1 || iters < 1) return fail(LDPCX_E_INVAL, "blocks and iters must be positive");
    hipStream_t s = (hipStream_t)stream;
    uint32_t *out = nullptr;
    if (hipMallocAsync((void **)&out, 64 * sizeof(uint32_t), s) != hipSuccess)
        return fail(LDPCX_E_NOMEM, "probe output");
    hipLaunchKernelGGL(k_valu_probe, dim3((unsigned)blocks), dim3(256), 0, s, iters, 0x2545F491u, out);
    const hipError_t e = hipGetLastError();
    (void)hipFreeAsync(out, s);
    if (e != hipSuccess) return fail_hip(e, "VALU probe launch");
    return LDPCX_OK;
}
