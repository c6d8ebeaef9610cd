// Layout kernels shared by the interleaved decoders: tiled transposes between the
// caller's codeword-major layout [batch][...] and the codeword-per-lane layout
// [...][Bp] (Bp = batch rounded up to 64), plus a small fill kernel (used instead
// of memset so that the sequences stay capturable in a HIP graph).
#include "k_common.h"

namespace ldpcx {

namespace {

// out[c * ld_out + r] = (r < rows) ? in[r * ld_in + c] : 0   for r < rows_out, c < cols
template <typename T>
__global__ void __launch_bounds__(256) k_transpose(const T *__restrict__ in, long rows, long cols, long ld_in,
                                                   T *__restrict__ out, long rows_out, long ld_out) {
    __shared__ T tile[64][65];
    const long c0 = (long)blockIdx.x * 64, r0 = (long)blockIdx.y * 64;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;  // 64 x 4
    for (int i = ty; i < 64; i += 4) {
        const long r = r0 + i, c = c0 + tx;
        T v = T(0);
        if (r < rows && c < cols) v = in[r * ld_in + c];
        tile[i][tx] = v;
    }
    __syncthreads();
    for (int i = ty; i < 64; i += 4) {
        const long c = c0 + i, r = r0 + tx;
        if (c < cols && r < rows_out) out[c * ld_out + r] = tile[tx][i];
    }
}

__global__ void __launch_bounds__(256) k_fill_u32(uint32_t *p, size_t n, uint32_t v) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        p[i] = v;
}

}  // namespace

template <typename T>
hipError_t transpose(const T *in, long rows, long cols, long ld_in, T *out, long rows_out, long ld_out,
                     hipStream_t s) {
    if (cols <= 0 || rows_out <= 0) return hipSuccess;
    dim3 grid((unsigned)((cols + 63) / 64), (unsigned)((rows_out + 63) / 64));
    hipLaunchKernelGGL(k_transpose<T>, grid, dim3(256), 0, s, in, rows, cols, ld_in, out, rows_out, ld_out);
    return hipGetLastError();
}

template hipError_t transpose<int8_t>(const int8_t *, long, long, long, int8_t *, long, long, hipStream_t);
template hipError_t transpose<uint8_t>(const uint8_t *, long, long, long, uint8_t *, long, long, hipStream_t);
template hipError_t transpose<int16_t>(const int16_t *, long, long, long, int16_t *, long, long, hipStream_t);

hipError_t fill_u32(void *p, size_t bytes, uint32_t v, hipStream_t s) {
    const size_t n = bytes / 4;
    if (n == 0) return hipSuccess;
    const unsigned grid = (unsigned)std::min<size_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(k_fill_u32, dim3(grid), dim3(256), 0, s, (uint32_t *)p, n, v);
    return hipGetLastError();
}

}  // namespace ldpcx
