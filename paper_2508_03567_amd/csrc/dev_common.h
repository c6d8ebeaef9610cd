// Device helpers shared by every decoder: packed 16-bit types and operations, the
// magnitude normalisation of the min-sum variants, and layout transposes and fills
// written as block-level device functions (block index passed explicitly).
#pragma once

#include "ldpcx_internal.h"

namespace ldpcx {
namespace dev {

typedef short v2s __attribute__((ext_vector_type(2)));

__device__ __forceinline__ v2s splat(int x) { return (v2s){(short)x, (short)x}; }
__device__ __forceinline__ v2s pmin(v2s a, v2s b) { return __builtin_elementwise_min(a, b); }
__device__ __forceinline__ v2s pmax(v2s a, v2s b) { return __builtin_elementwise_max(a, b); }
__device__ __forceinline__ v2s as_v2s(uint32_t u) { return __builtin_bit_cast(v2s, u); }
__device__ __forceinline__ uint32_t as_u32(v2s v) { return __builtin_bit_cast(uint32_t, v); }

// Magnitude normalisation of the min-sum variants on packed pairs, one formula for
// the three rules: f(m) = max(((m * num) >> shift) - off, 0) with (num, shift, off)
// = (num, shift, 0) for NMS, (1, 0, off) for OMS and (1, 0, 0) for MS.
struct PkNorm {
    v2s num, shift, off;
};

__device__ __forceinline__ PkNorm pk_norm_params(const BinRule &R) {
    PkNorm P;
    const bool nms = R.rule == LDPCX_RULE_NMS, oms = R.rule == LDPCX_RULE_OMS;
    P.num = splat(nms ? R.nms_num : 1);
    P.shift = splat(nms ? R.nms_shift : 0);
    P.off = splat(oms ? R.oms_offset : 0);
    return P;
}

__device__ __forceinline__ v2s pk_norm(const PkNorm &P, v2s m) {
    return pmax(((m * P.num) >> P.shift) - P.off, splat(0));
}

// Tiled transpose, one 64 x 64 tile per block of 256 threads:
// out[c * ld_out + r] = (r < rows) ? in[r * ld_in + c] : 0 for r < rows_out, c < cols.
struct TransposeArgs {
    const void *in;
    void *out;
    long rows, cols, ld_in, rows_out, ld_out;
    int elem;  // 1 or 2 bytes
};

template <typename T>
__device__ __forceinline__ void transpose_tile(const TransposeArgs &A, long bx, long by, unsigned char *lds) {
    T(*tile)[65] = (T(*)[65])lds;
    const T *in = (const T *)A.in;
    T *out = (T *)A.out;
    const long c0 = bx * 64, r0 = by * 64;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    for (int i = ty; i < 64; i += 4) {
        const long r = r0 + i, c = c0 + tx;
        T v = T(0);
        if (r < A.rows && c < A.cols) v = in[r * A.ld_in + c];
        tile[i][tx] = v;
    }
    __syncthreads();
    for (int i = ty; i < 64; i += 4) {
        const long c = c0 + i, r = r0 + tx;
        if (c < A.cols && r < A.rows_out) out[c * A.ld_out + r] = tile[tx][i];
    }
    __syncthreads();
}

__device__ __forceinline__ void transpose_block(const TransposeArgs &A, long bx, long by, unsigned char *lds) {
    if (A.elem == 2) transpose_tile<int16_t>(A, bx, by, lds);
    else transpose_tile<int8_t>(A, bx, by, lds);
}

__host__ __device__ inline long transpose_gx(const TransposeArgs &A) { return (A.cols + 63) / 64; }
__host__ __device__ inline long transpose_gy(const TransposeArgs &A) { return (A.rows_out + 63) / 64; }

struct FillArgs {
    uint32_t *p;
    size_t n;
    uint32_t v;
};

// Block bx of a fill split in blocks of 256 x 16 words.
__device__ __forceinline__ void fill_block(const FillArgs &A, long bx) {
    const size_t base = (size_t)bx * 4096;
    for (int k = 0; k < 16; ++k) {
        const size_t i = base + (size_t)k * 256 + threadIdx.x;
        if (i < A.n) A.p[i] = A.v;
    }
}

__host__ __device__ inline long fill_gx(const FillArgs &A) { return (long)((A.n + 4095) / 4096); }

// Index of the calling wavefront in its workgroup, as a wave-uniform (scalar) value,
// so that everything derived from it (node and edge indices, offsets) stays scalar.
__device__ __forceinline__ int wave_id() { return __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)); }

// Wave-wide OR of a 64-bit value (all lanes receive the result).
__device__ __forceinline__ uint64_t wave_or64(uint64_t v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v |= __shfl_xor(v, o, 64);
    return v;
}

}  // namespace dev
}  // namespace ldpcx
