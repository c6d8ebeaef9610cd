// Launch sequence of the large-field Min-Max decoder (g = 128, 256): one kernel per
// phase, every wavefront an independent (node, codeword) unit; the phase bodies are
// the device functions of dev_nbw.h.
#include <algorithm>

#include "dev_nbw.h"

namespace ldpcx {

namespace {

using dev::nbw::Args;

__device__ __forceinline__ long unit_of(int wpb) { return (long)blockIdx.x * wpb + dev::wave_id(); }

__global__ void __launch_bounds__(256) k_fill(dev::FillArgs F) { dev::fill_block(F, blockIdx.x); }
template <int G>
__global__ void __launch_bounds__(256) k_init_e(Args A) { dev::nbw::init_edge_unit<G>(A, unit_of(4)); }
template <int G>
__global__ void __launch_bounds__(256) k_init_v(Args A) { dev::nbw::init_var_unit<G>(A, unit_of(4)); }
__global__ void __launch_bounds__(256) k_syn(Args A, int slot) {
    dev::nbw::syn_thread(A, slot, (long)blockIdx.x * 256 + threadIdx.x);
}
template <int G>
__global__ void __launch_bounds__(256) k_cn(Args A, int k, int wpb, int words) {
    extern __shared__ __align__(16) uint32_t lds[];
    const int w = dev::wave_id();
    if (w >= wpb) return;
    dev::nbw::cn_unit<G>(A, k, unit_of(wpb), lds + (size_t)w * words);
}
template <int G>
__global__ void __launch_bounds__(256) k_vn(Args A, int k) { dev::nbw::vn_unit<G>(A, k, unit_of(4)); }
__global__ void __launch_bounds__(256) k_fin(Args A) { dev::nbw::fin_thread(A, (long)blockIdx.x * 256 + threadIdx.x); }
template <int G>
__global__ void __launch_bounds__(256) k_dump(Args A, const int16_t *src, int16_t *dst) {
    dev::nbw::dump_unit<G>(A, src, dst, unit_of(4));
}

unsigned blocks(long units, int per) { return (unsigned)((units + per - 1) / per); }

hipError_t fill(const dev::FillArgs &F, hipStream_t s) {
    if (F.n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill, dim3((unsigned)dev::fill_gx(F)), dim3(256), 0, s, F);
    return hipGetLastError();
}

template <int G>
hipError_t run(const Args &A, hipStream_t s) {
    const DevCode &C = A.C;
    const long B = A.batch;
    const dim3 blk(256);
    hipError_t e;
    const dev::nbw::Carve cv = dev::nbw::carve(C, A.max_iters, A.batch);
    if ((e = fill(dev::FillArgs{(uint32_t *)A.w.unsat, (cv.it - cv.unsat) / 4, 0u}, s)) != hipSuccess) return e;
    if ((e = fill(dev::FillArgs{(uint32_t *)A.w.it, (size_t)(B + 1) / 2, 0u}, s)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_init_e<G>, dim3(blocks(C.E * B, 4)), blk, 0, s, A);
    hipLaunchKernelGGL(k_init_v<G>, dim3(blocks(C.n * B, 4)), blk, 0, s, A);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    const int words = (int)dev::nbw::cn_words_per_wave(G, C.dc_max);
    int wpb = (int)std::min<size_t>(4, (size_t)(64 * 1024) / ((size_t)words * 4));
    if (wpb < 1) return hipErrorInvalidConfiguration;
    const size_t smem = (size_t)wpb * words * 4;
    for (int k = 1; k <= A.max_iters; ++k) {
        if (A.early_stop) hipLaunchKernelGGL(k_syn, dim3(blocks(C.m * B, 256)), blk, 0, s, A, k);
        hipLaunchKernelGGL(k_cn<G>, dim3(blocks(C.m * B, wpb)), dim3(64 * wpb), smem, s, A, k, wpb, words);
        hipLaunchKernelGGL(k_vn<G>, dim3(blocks(C.n * B, 4)), blk, 0, s, A, k);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_syn, dim3(blocks(C.m * B, 256)), blk, 0, s, A, 0);
    hipLaunchKernelGGL(k_fin, dim3(blocks(B, 256)), blk, 0, s, A);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (A.io.dump_a) {
        hipLaunchKernelGGL(k_dump<G>, dim3(blocks(C.E * B, 4)), blk, 0, s, A, (const int16_t *)A.w.alpha,
                           (int16_t *)A.io.dump_a);
        hipLaunchKernelGGL(k_dump<G>, dim3(blocks(C.E * B, 4)), blk, 0, s, A, (const int16_t *)A.w.beta,
                           (int16_t *)A.io.dump_b);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace

size_t nbw_work_bytes(const DevCode &C, int max_iters, int batch) { return dev::nbw::carve(C, max_iters, batch).total; }

hipError_t launch_nbw(const DevCode &C, int max_iters, int early_stop, int batch, int amax, void *ws,
                      const DecodeIO &io, hipStream_t s) {
    const Args A = dev::nbw::make_args(C, max_iters, early_stop, batch, amax, ws, io);
    switch (C.g) {
    case 128: return run<128>(A, s);
    case 256: return run<256>(A, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace ldpcx
