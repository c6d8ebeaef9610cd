// Launch sequence of the interleaved binary min-sum decoder (flooding): one
// kernel per phase, the phase bodies being the device functions of dev_bin_il.h.
// A batch larger than the sub-batch runs as consecutive launch sequences over
// slices of the codewords (each slice's state stays small enough to remain
// resident in the last-level cache, and every offset fits 31 bits).
#include <algorithm>

#include "dev_bin_il.h"

namespace ldpcx {

namespace {

using dev::il::Args;

__global__ void __launch_bounds__(256) k_tr(dev::TransposeArgs T) {
    __shared__ __align__(16) unsigned char tile[64 * 65 * 2];
    dev::transpose_block(T, blockIdx.x, blockIdx.y, tile);
}
__global__ void __launch_bounds__(256) k_fill(dev::FillArgs F) { dev::fill_block(F, blockIdx.x); }
__global__ void __launch_bounds__(256) k_init_edges(Args A) { dev::il::init_edges_block(A, blockIdx.x, blockIdx.y); }
__global__ void __launch_bounds__(256) k_init_vars(Args A) { dev::il::init_vars_block(A, blockIdx.x, blockIdx.y); }
__global__ void __launch_bounds__(256) k_syn(Args A, int slot) { dev::il::syn_block(A, slot, blockIdx.x); }
template <int DC>
__global__ void __launch_bounds__(256) k_cn(Args A, int k) { dev::il::cn_block<DC>(A, k, blockIdx.x, blockIdx.y); }
__global__ void __launch_bounds__(256) k_vn(Args A, int k) { dev::il::vn_block(A, k, blockIdx.x, blockIdx.y); }
__global__ void __launch_bounds__(256) k_bytes(Args A) { dev::il::bytes_block(A, blockIdx.x); }
__global__ void __launch_bounds__(256) k_fin(Args A) { dev::il::fin_block(A, blockIdx.x); }
__global__ void __launch_bounds__(256) k_lambda(Args A, int16_t *lam_t) {
    dev::il::lambda_block(A, lam_t, blockIdx.x, blockIdx.y);
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

// One launch sequence over `batch` codewords (batch <= the sub-batch limit).
hipError_t run_slice(const DevCode &C, const BinRule &R, int max_iters, int early_stop, int batch, void *ws,
                     const DecodeIO &io, int8_t *dump_scratch, hipStream_t s) {
    const Args A = dev::il::make_args(C, R, max_iters, early_stop, batch, ws, io);
    const dim3 blk(256);
    LDPCX_CHECK(tr(dev::il::tr_in(A), s));
    LDPCX_CHECK(fill(dev::il::fill_unsat(A), s));
    LDPCX_CHECK(fill(dev::il::fill_it(A), s));
    const unsigned G = (unsigned)A.G;
    hipLaunchKernelGGL(k_init_edges, dim3((unsigned)dev::il::grid_edges_x(A), G), blk, 0, s, A);
    hipLaunchKernelGGL(k_init_vars, dim3((unsigned)dev::il::grid_vars_x(A), G), blk, 0, s, A);
    LDPCX_CHECK(hipGetLastError());
    const dim3 gcn((unsigned)dev::il::grid_rows_x(A), G);
    const dim3 gvn((unsigned)dev::il::grid_vars_x(A), G);
    const dim3 gsyn((unsigned)dev::il::grid_syn(A));
    const dim3 gvnw((unsigned)dev::il::grid_vn_x(A), G);
    for (int k = 1; k <= max_iters; ++k) {
        if (early_stop) hipLaunchKernelGGL(k_syn, gsyn, blk, 0, s, A, k);
        if (C.dc_max <= 8) hipLaunchKernelGGL(k_cn<8>, gcn, blk, 0, s, A, k);
        else hipLaunchKernelGGL(k_cn<kBinDcMax>, gcn, blk, 0, s, A, k);
        hipLaunchKernelGGL(k_vn, gvnw, blk, 0, s, A, k);
        LDPCX_CHECK(hipGetLastError());
    }
    hipLaunchKernelGGL(k_syn, gsyn, blk, 0, s, A, 0);
    hipLaunchKernelGGL(k_fin, dim3((unsigned)dev::il::grid_fin(A)), blk, 0, s, A);
    hipLaunchKernelGGL(k_bytes, dim3((unsigned)dev::il::grid_bytes(A)), blk, 0, s, A);
    LDPCX_CHECK(hipGetLastError());
    LDPCX_CHECK(tr(dev::il::tr_out(A), s));
    if (io.dump_a) {
        const long Bp = A.Bp;
        int16_t *lam_t = (int16_t *)dump_scratch;
        hipLaunchKernelGGL(k_lambda, gvn, blk, 0, s, A, lam_t);
        LDPCX_CHECK(hipGetLastError());
        LDPCX_CHECK(tr(dev::TransposeArgs{A.w.q, io.dump_a, C.E, batch, Bp, C.E, C.E, 1}, s));
        LDPCX_CHECK(tr(dev::TransposeArgs{A.w.r, io.dump_b, C.E, batch, Bp, C.E, C.E, 1}, s));
        LDPCX_CHECK(tr(dev::TransposeArgs{lam_t, io.dump_c, C.n, batch, Bp, C.n, C.n, 2}, s));
    }
    return hipSuccess;
}

}  // namespace

int bin_il_sub_batch(const DevCode &C, int batch, int want) {
    int sub = want > 0 ? want : 512;
    sub = std::min(sub, dev::il::max_sub_batch(C));
    sub = dev::il::pad_group(std::max(sub, 1));
    return std::min(sub, dev::il::pad_group(std::max(batch, 1)));
}

size_t bin_il_work_bytes(const DevCode &C, int max_iters, int batch, int sub) {
    return dev::il::carve(C, max_iters, std::min(batch, bin_il_sub_batch(C, batch, sub))).total;
}

size_t bin_il_dump_bytes(const DevCode &C, int batch, int sub) {
    return align_up((size_t)C.n * dev::il::pad_group(std::min(batch, bin_il_sub_batch(C, batch, sub))) * 2, 256);
}

hipError_t launch_bin_il(const DevCode &C, const BinRule &R, int max_iters, int early_stop, int batch, int sub,
                         void *ws, const DecodeIO &io, int8_t *dump_scratch, hipStream_t s) {
    const int step = bin_il_sub_batch(C, batch, sub);
    const size_t nbytes = (size_t)(C.n + 7) / 8;
    for (int b0 = 0; b0 < batch; b0 += step) {
        const int nb = std::min(step, batch - b0);
        DecodeIO sl = io;
        sl.llr = (const int8_t *)io.llr + (size_t)b0 * C.n;
        sl.hard = (uint8_t *)io.hard + (size_t)b0 * nbytes;
        sl.ok = io.ok + b0;
        sl.iters = io.iters + b0;
        if (io.dump_a) {
            sl.dump_a = (int8_t *)io.dump_a + (size_t)b0 * C.E;
            sl.dump_b = (int8_t *)io.dump_b + (size_t)b0 * C.E;
            sl.dump_c = (int16_t *)io.dump_c + (size_t)b0 * C.n;
        }
        LDPCX_CHECK(run_slice(C, R, max_iters, early_stop, nb, ws, sl, dump_scratch, s));
    }
    return hipSuccess;
}

}  // namespace ldpcx
