// Launch sequence of the interleaved binary min-sum decoder (flooding): one
// kernel per phase, the phase bodies being the device functions of dev_bin_il.h.
#include "dev_bin_il.h"

namespace ldpcx {

namespace {

using dev::il::Args;

__global__ void __launch_bounds__(256) k_tr(dev::TransposeArgs T) {
    __shared__ __align__(16) unsigned char tile[64 * 65 * 2];
    dev::transpose_block(T, blockIdx.x, blockIdx.y, tile);
}
__global__ void __launch_bounds__(256) k_fill(dev::FillArgs F) { dev::fill_block(F, blockIdx.x); }
__global__ void __launch_bounds__(256) k_init(Args A) { dev::il::init_block(A, blockIdx.x); }
__global__ void __launch_bounds__(256) k_syn(Args A, int slot) { dev::il::syn_block(A, slot, blockIdx.x); }
__global__ void __launch_bounds__(256) k_cn(Args A, int k) { dev::il::cn_block(A, k, blockIdx.x, blockIdx.y); }
__global__ void __launch_bounds__(256) k_vn(Args A, int k) { dev::il::vn_block(A, k, blockIdx.x, blockIdx.y); }
__global__ void __launch_bounds__(256) k_bytes(Args A) { dev::il::bytes_block(A, blockIdx.x); }
__global__ void __launch_bounds__(256) k_fin(Args A) { dev::il::fin_block(A, blockIdx.x); }
__global__ void __launch_bounds__(256) k_dump(Args A, int8_t *q_t, int8_t *r_t) {
    dev::il::dump_block(A, q_t, r_t, blockIdx.x, blockIdx.y);
}

hipError_t tr(const dev::TransposeArgs &T, hipStream_t s) {
    if (T.cols <= 0 || T.rows_out <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_tr, dim3((unsigned)dev::transpose_gx(T), (unsigned)dev::transpose_gy(T)), dim3(256), 0, s,
                       T);
    return hipGetLastError();
}

hipError_t fill(const dev::FillArgs &F, hipStream_t s) {
    if (F.n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill, dim3((unsigned)dev::fill_gx(F)), dim3(256), 0, s, F);
    return hipGetLastError();
}

#define LDPCX_CHECK(x)                   \
    do {                                 \
        hipError_t e_ = (x);             \
        if (e_ != hipSuccess) return e_; \
    } while (0)

}  // namespace

size_t bin_il_work_bytes(const DevCode &C, int max_iters, int batch) {
    return dev::il::carve(C, max_iters, batch).total;
}

hipError_t launch_bin_il(const DevCode &C, const BinRule &R, int max_iters, int early_stop, int batch, void *ws,
                         const DecodeIO &io, int8_t *dump_scratch, hipStream_t s) {
    const Args A = dev::il::make_args(C, R, max_iters, early_stop, batch, ws, io);
    const dim3 blk(256);
    LDPCX_CHECK(tr(dev::il::tr_in(A), s));
    hipLaunchKernelGGL(k_init, dim3((unsigned)dev::il::grid_init(A)), blk, 0, s, A);
    LDPCX_CHECK(hipGetLastError());
    LDPCX_CHECK(fill(dev::il::fill_st(A), s));
    LDPCX_CHECK(fill(dev::il::fill_unsat(A), s));
    LDPCX_CHECK(fill(dev::il::fill_it(A), s));
    const dim3 gcn((unsigned)dev::il::grid_cn_x(A), (unsigned)A.Gn);
    const dim3 gvn((unsigned)dev::il::grid_vn_x(A), (unsigned)A.Gn);
    const dim3 gsyn((unsigned)dev::il::grid_syn(A));
    for (int k = 1; k <= max_iters; ++k) {
        if (early_stop) hipLaunchKernelGGL(k_syn, gsyn, blk, 0, s, A, k);
        hipLaunchKernelGGL(k_cn, gcn, blk, 0, s, A, k);
        hipLaunchKernelGGL(k_vn, gvn, blk, 0, s, A, k);
        LDPCX_CHECK(hipGetLastError());
    }
    hipLaunchKernelGGL(k_syn, gsyn, blk, 0, s, A, 0);
    hipLaunchKernelGGL(k_fin, dim3((unsigned)dev::il::grid_fin(A)), blk, 0, s, A);
    hipLaunchKernelGGL(k_bytes, dim3((unsigned)dev::il::grid_bytes(A)), blk, 0, s, A);
    LDPCX_CHECK(hipGetLastError());
    LDPCX_CHECK(tr(dev::il::tr_out(A), s));
    if (io.dump_a) {
        const size_t Bp = A.Bp;
        int8_t *q_t = dump_scratch;
        int8_t *r_t = dump_scratch + align_up((size_t)C.E * Bp, 256);
        hipLaunchKernelGGL(k_dump, gcn, blk, 0, s, A, q_t, r_t);
        LDPCX_CHECK(hipGetLastError());
        LDPCX_CHECK(tr(dev::TransposeArgs{q_t, io.dump_a, C.E, batch, (long)Bp, C.E, C.E, 1}, s));
        LDPCX_CHECK(tr(dev::TransposeArgs{r_t, io.dump_b, C.E, batch, (long)Bp, C.E, C.E, 1}, s));
        LDPCX_CHECK(tr(dev::TransposeArgs{A.w.lam, io.dump_c, C.n, batch, (long)Bp, C.n, C.n, 2}, s));
    }
    return hipSuccess;
}

}  // namespace ldpcx
