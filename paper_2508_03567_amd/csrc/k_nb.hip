// Launch sequences of the Min-Max decoders over GF(4)..GF(64) (the device functions
// of dev_nb.h): one kernel per phase for the flooding and layered schedules on
// HBM-resident messages, or one kernel per batch slice for the LDS-resident family.
#include <algorithm>

#include "dev_nb.h"

namespace ldpcx {

namespace {

using dev::nb::Args;

__global__ void __launch_bounds__(256) k_tr(dev::TransposeArgs T) {
    __shared__ __align__(16) unsigned char tile[64 * 65 * 2];
    dev::transpose_block(T, blockIdx.x, blockIdx.y, tile);
}
__global__ void __launch_bounds__(256) k_fill(dev::FillArgs F) { dev::fill_block(F, blockIdx.x); }
// Node-by-group kernels run on a 1-D grid numbered group-fastest: consecutive blocks take
// the same nodes for neighbouring groups of 64 codewords, so the rows that run together
// are adjacent in the [node][entry][codeword] arrays.
__device__ __forceinline__ int blk_node(int Gn) { return (int)(blockIdx.x / (unsigned)Gn); }
__device__ __forceinline__ int blk_group(int Gn) { return (int)(blockIdx.x % (unsigned)Gn); }

template <int G>
__global__ void __launch_bounds__(256) k_init(Args A, int alpha) {
    dev::nb::init_block<G>(A, blk_node(A.Gn), blk_group(A.Gn), alpha != 0);
}
__global__ void __launch_bounds__(256) k_syn(Args A, int slot) {
    dev::nb::syn_block(A, slot, blk_node(A.Gn), blk_group(A.Gn));
}
template <int G>
__global__ void __launch_bounds__(256) k_cn(Args A, int k, int wpb) {
    extern __shared__ __align__(16) uint32_t lds[];
    dev::nb::cn_block<G>(A, k, wpb, blk_node(A.Gn), blk_group(A.Gn), lds);
}
template <int G>
__global__ void __launch_bounds__(256) k_vn(Args A, int k) { dev::nb::vn_block<G>(A, k, blk_node(A.Gn), blk_group(A.Gn)); }
template <int G>
__global__ void __launch_bounds__(256) k_cnf(Args A, int k, int wpb, const int16_t *beta_old, int16_t *beta_new) {
    extern __shared__ __align__(16) uint32_t lds[];
    dev::nb::cnf_block<G>(A, k, wpb, blk_node(A.Gn), blk_group(A.Gn), lds, beta_old, beta_new);
}
template <int G>
__global__ void __launch_bounds__(256) k_lal(Args A, int k, int layer) {
    dev::nb::lay_alpha_block<G>(A, k, layer, blk_node(A.Gn), blk_group(A.Gn));
}
template <int G>
__global__ void __launch_bounds__(256) k_lcn(Args A, int k, int layer, int wpb) {
    extern __shared__ __align__(16) uint32_t lds[];
    dev::nb::lay_cn_block<G>(A, k, layer, wpb, blk_node(A.Gn), blk_group(A.Gn), lds);
}
template <int G>
__global__ void __launch_bounds__(256) k_lcnf(Args A, int k, int layer, int wpb) {
    extern __shared__ __align__(16) uint32_t lds[];
    dev::nb::lay_cnf_block<G>(A, k, layer, wpb, blk_node(A.Gn), blk_group(A.Gn), lds);
}
template <int G>
__global__ void __launch_bounds__(256) k_dec(Args A, int k) { dev::nb::dec_block<G>(A, k, blk_node(A.Gn), blk_group(A.Gn)); }
__global__ void __launch_bounds__(256) k_fin(Args A) { dev::nb::fin_block(A, blockIdx.x); }
template <int G>
__global__ void __launch_bounds__(256) k_fdump(Args A) { dev::nb::fdump_block<G>(A, blk_node(A.Gn), blk_group(A.Gn)); }
// One group of 64 codewords per workgroup, messages in LDS.
template <int G, bool GL>
__global__ void __launch_bounds__(1024) k_nbl(Args A, int layered, int waves) {
    extern __shared__ __align__(16) unsigned char lds8[];
    dev::nb::lds_group<G, GL>(A, layered != 0, waves, blockIdx.x, lds8);
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

dim3 lin(long nodes, int Gn) { return dim3((unsigned)(nodes * Gn)); }

template <int G>
hipError_t run(const Args &A, bool layered, hipStream_t s) {
    hipError_t e;
    const long most = std::max<long>({dev::nb::grid_init_x(A), A.C.m, A.C.nb_emax});
    if (most * A.Gn >= (1L << 31)) return hipErrorInvalidConfiguration;
    if ((e = tr(dev::nb::tr_in(A), s)) != hipSuccess) return e;
    const dim3 blk(256);
    // Every variable of degree 2: the alphas formed inside the check node, in flooding
    // (fused, also under the debug dump, which then forms the final alphas once) and
    // layered schedules (dv2; the dump there keeps the stored alphas, which depend on the
    // order of the layers).
    const bool deg2 = A.C.dv_max == 2 && A.C.E == 2 * A.C.n;
    const bool fused = !layered && deg2;
    const bool dv2 = fused || (deg2 && !A.io.dump_a);
    hipLaunchKernelGGL(k_init<G>, lin(dev::nb::grid_init_x(A), A.Gn), blk, 0, s, A, dv2 ? 0 : 1);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = fill(dev::nb::fill_unsat(A), s)) != hipSuccess) return e;
    if ((e = fill(dev::nb::fill_it(A), s)) != hipSuccess) return e;
    const int wpb = dev::nb::cn_waves(A, 64 * 1024);
    if (wpb < 1) return hipErrorInvalidConfiguration;
    const size_t smem = dev::nb::cn_lds_bytes(A, wpb);
    const dim3 gcn = lin((A.C.m + wpb - 1) / wpb, A.Gn);
    const dim3 gsy = lin(dev::nb::grid_rows_x(A), A.Gn);
    const dim3 gvn = lin(dev::nb::grid_vn_x(A), A.Gn);
    const dim3 glay = lin((A.C.nb_lmax + wpb - 1) / wpb, A.Gn);
    const dim3 glal = lin((A.C.nb_emax + 3) / 4, A.Gn);
    for (int k = 1; k <= A.max_iters; ++k) {
        if (A.early_stop) hipLaunchKernelGGL(k_syn, gsy, blk, 0, s, A, k);
        if (layered) {
            // two launches per layer (its alphas, then its check nodes): the checks of a
            // layer share no variable
            for (int l = 0; l < A.C.nb_nl; ++l) {
                if (dv2) {
                    hipLaunchKernelGGL(k_lcnf<G>, glay, dim3(64 * wpb), smem, s, A, k, l, wpb);
                } else {
                    hipLaunchKernelGGL(k_lal<G>, glal, blk, 0, s, A, k, l);
                    hipLaunchKernelGGL(k_lcn<G>, glay, dim3(64 * wpb), smem, s, A, k, l, wpb);
                }
            }
            hipLaunchKernelGGL(k_dec<G>, gvn, blk, 0, s, A, k);
        } else if (fused) {
            // Flooding with the alphas formed inside the check node: the betas alternate
            // between two arrays (the alpha array is free for it), and the decisions are
            // formed only where they are used (every iteration under early stopping,
            // else after the last one).
            int16_t *bo = (k & 1) ? A.w.beta : A.w.alpha, *bn = (k & 1) ? A.w.alpha : A.w.beta;
            hipLaunchKernelGGL(k_cnf<G>, gcn, dim3(64 * wpb), smem, s, A, k, wpb, bo, bn);
            if (A.early_stop || k == A.max_iters) {
                Args D = A;
                D.w.beta = bn;
                hipLaunchKernelGGL(k_dec<G>, gvn, blk, 0, s, D, k);
            }
        } else {
            hipLaunchKernelGGL(k_cn<G>, gcn, dim3(64 * wpb), smem, s, A, k, wpb);
            hipLaunchKernelGGL(k_vn<G>, gvn, blk, 0, s, A, k);
        }
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_syn, gsy, blk, 0, s, A, 0);
    hipLaunchKernelGGL(k_fin, dim3((unsigned)dev::nb::grid_fin(A)), blk, 0, s, A);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = tr(dev::nb::tr_out(A), s)) != hipSuccess) return e;
    if (A.io.dump_a && fused) {
        hipLaunchKernelGGL(k_fdump<G>, lin((A.C.E + 3) / 4, A.Gn), blk, 0, s, A);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    } else if (A.io.dump_a) {
        const long rows = (long)A.C.E * G;
        if ((e = tr(dev::TransposeArgs{A.w.alpha, A.io.dump_a, rows, A.batch, A.Bp, rows, rows, 2}, s)) != hipSuccess)
            return e;
        if ((e = tr(dev::TransposeArgs{A.w.beta, A.io.dump_b, rows, A.batch, A.Bp, rows, rows, 2}, s)) != hipSuccess)
            return e;
    }
    return hipSuccess;
}

template <int G, bool GL>
hipError_t launch_group_kernel(const Args &A, bool layered, int waves, hipStream_t s) {
    const size_t lds = dev::nb::lds_plan(A.C, A.fslots, waves, GL).total;
    allow_full_lds((const void *)k_nbl<G, GL>);
    hipLaunchKernelGGL((k_nbl<G, GL>), dim3((unsigned)A.Gn), dim3(64 * waves), lds, s, A, layered ? 1 : 0, waves);
    return hipGetLastError();
}

template <int G>
hipError_t run_lds(const Args &A, bool layered, int waves, hipStream_t s) {
    hipError_t e;
    if ((e = tr(dev::nb::tr_in(A), s)) != hipSuccess) return e;
    // channel vectors staged in LDS too when they fit
    const bool gl = dev::nb::lds_plan(A.C, A.fslots, waves, true).total <= (size_t)160 * 1024;
    e = gl ? launch_group_kernel<G, true>(A, layered, waves, s) : launch_group_kernel<G, false>(A, layered, waves, s);
    if (e != hipSuccess) return e;
    if ((e = tr(dev::nb::tr_out(A), s)) != hipSuccess) return e;
    if (A.io.dump_a) {
        const long rows = (long)A.C.E * G;
        if ((e = tr(dev::TransposeArgs{A.w.alpha, A.io.dump_a, rows, A.batch, A.Bp, rows, rows, 2}, s)) != hipSuccess)
            return e;
        if ((e = tr(dev::TransposeArgs{A.w.beta, A.io.dump_b, rows, A.batch, A.Bp, rows, rows, 2}, s)) != hipSuccess)
            return e;
    }
    return hipSuccess;
}

}  // namespace

size_t nb_lds_bytes(const DevCode &C, int waves) {
    const int fslots = C.dc_max > 3 ? C.dc_max - 3 : 1;
    return dev::nb::lds_plan(C, fslots, waves, false).total;
}

hipError_t launch_nb_lds(const DevCode &C, int max_iters, int early_stop, int layered, int batch, int amax, int waves,
                         void *ws, const DecodeIO &io, hipStream_t s) {
    if (C.g > 64 || (waves != 4 && waves != 8 && waves != 16) || nb_lds_bytes(C, waves) > (size_t)160 * 1024)
        return hipErrorInvalidValue;
    if (layered && (C.nb_nl < 1 || C.nb_lmax < 1 || C.nb_emax < 1)) return hipErrorInvalidValue;
    const int step = nb_slice(C, batch);
    for (int b0 = 0; b0 < batch; b0 += step) {
        const int nb = std::min(step, batch - b0);
        DecodeIO sl = io;
        sl.llr = (const int16_t *)io.llr + (size_t)b0 * C.n * C.g;
        sl.hard = (uint8_t *)io.hard + (size_t)b0 * C.n;
        sl.ok = io.ok + b0;
        sl.iters = io.iters + b0;
        if (io.dump_a) {
            sl.dump_a = (int16_t *)io.dump_a + (size_t)b0 * C.E * C.g;
            sl.dump_b = (int16_t *)io.dump_b + (size_t)b0 * C.E * C.g;
        }
        const Args A = dev::nb::make_args(C, max_iters, early_stop, nb, amax, ws, sl);
        hipError_t e;
        switch (C.g) {
        case 4: e = run_lds<4>(A, layered != 0, waves, s); break;
        case 8: e = run_lds<8>(A, layered != 0, waves, s); break;
        case 16: e = run_lds<16>(A, layered != 0, waves, s); break;
        case 32: e = run_lds<32>(A, layered != 0, waves, s); break;
        case 64: e = run_lds<64>(A, layered != 0, waves, s); break;
        default: e = hipErrorInvalidValue;
        }
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

bool nb_supported(int g) { return g == 4 || g == 8 || g == 16 || g == 32 || g == 64 || g == 128 || g == 256; }

int nb_slice(const DevCode &C, int batch) {
    // every byte offset into an [E][g][Bp] message array must fit 31 bits
    long step = ((1L << 31) - 1) / (2L * C.E * C.g);
    step = step / 64 * 64;
    if (step < 64) step = 64;
    return (int)std::min<long>(step, std::max(batch, 1));
}

size_t nb_work_bytes(const DevCode &C, int max_iters, int batch) {
    if (C.g >= 128) return nbw_work_bytes(C, max_iters, batch);
    return dev::nb::carve(C, max_iters, nb_slice(C, batch)).total;
}

hipError_t launch_nb(const DevCode &C, int max_iters, int early_stop, int layered, int batch, int amax, void *ws,
                     const DecodeIO &io, hipStream_t s) {
    if (C.g >= 128) {
        if (layered) return hipErrorInvalidValue;
        return launch_nbw(C, max_iters, early_stop, batch, amax, ws, io, s);
    }
    if (layered && (C.nb_nl < 1 || C.nb_lmax < 1 || C.nb_emax < 1)) return hipErrorInvalidValue;
    const int step = nb_slice(C, batch);
    for (int b0 = 0; b0 < batch; b0 += step) {
        const int nb = std::min(step, batch - b0);
        DecodeIO sl = io;
        sl.llr = (const int16_t *)io.llr + (size_t)b0 * C.n * C.g;
        sl.hard = (uint8_t *)io.hard + (size_t)b0 * C.n;
        sl.ok = io.ok + b0;
        sl.iters = io.iters + b0;
        if (io.dump_a) {
            sl.dump_a = (int16_t *)io.dump_a + (size_t)b0 * C.E * C.g;
            sl.dump_b = (int16_t *)io.dump_b + (size_t)b0 * C.E * C.g;
        }
        const Args A = dev::nb::make_args(C, max_iters, early_stop, nb, amax, ws, sl);
        hipError_t e;
        switch (C.g) {
        case 4: e = run<4>(A, layered != 0, s); break;
        case 8: e = run<8>(A, layered != 0, s); break;
        case 16: e = run<16>(A, layered != 0, s); break;
        case 32: e = run<32>(A, layered != 0, s); break;
        case 64: e = run<64>(A, layered != 0, s); break;
        default: e = hipErrorInvalidValue;
        }
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace ldpcx
