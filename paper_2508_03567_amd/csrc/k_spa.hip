// Launch sequences of the fixed-point FFT-SPA decoder (Alg. 1): the wave kernels (one
// kernel per phase, or one per iteration where the variable phase is fused into the
// check phase; every wavefront an independent (node, codeword group) unit) and the
// LDS-resident kernel (one launch per decode).  The bodies are the device functions of
// dev_spa.h.
#include <algorithm>

#include "dev_spa.h"

namespace ldpcx {

namespace {

using dev::spa::Args;

__device__ __forceinline__ long unit_id() { return (long)blockIdx.x * 4 + dev::wave_id(); }

__global__ void __launch_bounds__(256) k_fill(dev::FillArgs F) { dev::fill_block(F, blockIdx.x); }
// lanes per codeword of the channel-vector kernel (at most 16 entries per lane)
template <int G>
constexpr int init_lanes() { return G > 64 ? 16 : 4; }
template <int G>
__global__ void __launch_bounds__(256) k_init(Args A, int write_u) {
    dev::spa::init_unit<G, init_lanes<G>()>(A, unit_id(), write_u != 0);
}
__global__ void __launch_bounds__(256) k_syn(Args A, int slot) {
    dev::spa::syn_thread(A, slot, (long)blockIdx.x * 256 + threadIdx.x);
}
template <int G, int DC>
__global__ void __launch_bounds__(256) k_cn(Args A, int k) { dev::spa::cn_unit<G, DC>(A, k, unit_id()); }
template <int G, int DV>
__global__ void __launch_bounds__(256) k_vn(Args A, int k) { dev::spa::vn_unit<G, DV>(A, k, unit_id()); }
template <int G, int DC>
__global__ void __launch_bounds__(256) k_cnf(Args A, int k, const int *v_old, int *v_new) {
    dev::spa::cnf_unit<G, DC>(A, k, unit_id(), v_old, v_new);
}
template <int G>
__global__ void __launch_bounds__(256) k_dec(Args A, int k, const int *v_cur) { dev::spa::dec_unit<G>(A, k, unit_id(), v_cur); }
template <int G>
__global__ void __launch_bounds__(1024) k_spa_lds(Args A, int cw) {
    extern __shared__ __align__(16) unsigned char lds[];
    dev::spa::lds_decode<G>(A, cw, lds, blockIdx.x);
}
__global__ void __launch_bounds__(256) k_fin(Args A) { dev::spa::fin_thread(A, (long)blockIdx.x * 256 + threadIdx.x); }
template <int G>
__global__ void __launch_bounds__(256) k_fdump(Args A) { dev::spa::fdump_unit<G>(A, unit_id()); }
__global__ void __launch_bounds__(256) k_dump(Args A, const int *src, int *dst) {
    dev::spa::dump_thread(A, src, dst, (long)blockIdx.x * 256 + threadIdx.x);
}

unsigned blocks(long units, int per) { return (unsigned)((units + per - 1) / per); }

hipError_t fill(const dev::FillArgs &F, hipStream_t s) {
    if (F.n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill, dim3((unsigned)dev::fill_gx(F)), dim3(256), 0, s, F);
    return hipGetLastError();
}

// The register arrays of the check and variable phases are sized by degree bounds
// (4 or 16 for checks, 4 or 16 for variables) chosen from the code's largest degrees.
template <int G, int DC, int DV>
hipError_t run(const Args &A, hipStream_t s) {
    const DevCode &C = A.C;
    const long B = A.batch;
    // codeword groups of each kernel (its lanes per codeword set the group size)
    constexpr int CI = dev::spa::Geo<G, init_lanes<G>()>::CPW;
    constexpr int CC = dev::spa::Geo<G, dev::spa::lanes_for<G, DC>()>::CPW;
    constexpr int CV = dev::spa::Geo<G, dev::spa::lanes_for<G, DV>()>::CPW;
    const long gi = (B + CI - 1) / CI, gc = (B + CC - 1) / CC, gv = (B + CV - 1) / CV;
    const dim3 blk(256);
    hipError_t e;
    const dev::spa::Carve cv = dev::spa::carve(C, A.max_iters, A.batch);
    if ((e = fill(dev::FillArgs{(uint32_t *)A.w.unsat, (cv.it - cv.unsat) / 4, 0u}, s)) != hipSuccess) return e;
    if ((e = fill(dev::FillArgs{(uint32_t *)A.w.it, (size_t)(B + 1) / 2, 0u}, s)) != hipSuccess) return e;
    // Every variable of degree 2: flooding fused into the check node, v alternating
    // between the v and u arrays, decisions only where they are used (the debug dump then
    // forms the final u once).
    const bool fused = C.dv_max == 2 && C.E == 2 * C.n;
    hipLaunchKernelGGL(k_init<G>, dim3(blocks(C.n * gi, 4)), blk, 0, s, A, fused ? 0 : 1);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    constexpr int CD = dev::spa::Geo<G, dev::spa::lanes_for<G, 4>()>::CPW;
    const long gd = (B + CD - 1) / CD;
    for (int k = 1; k <= A.max_iters; ++k) {
        if (A.early_stop) hipLaunchKernelGGL(k_syn, dim3(blocks(C.m * B, 256)), blk, 0, s, A, k);
        if (fused) {
            int *vo = (k & 1) ? A.w.v : A.w.u, *vn = (k & 1) ? A.w.u : A.w.v;
            hipLaunchKernelGGL((k_cnf<G, DC>), dim3(blocks(C.m * gc, 4)), blk, 0, s, A, k, vo, vn);
            if (A.early_stop || k == A.max_iters)
                hipLaunchKernelGGL(k_dec<G>, dim3(blocks(C.n * gd, 4)), blk, 0, s, A, k, (const int *)vn);
        } else {
            hipLaunchKernelGGL((k_cn<G, DC>), dim3(blocks(C.m * gc, 4)), blk, 0, s, A, k);
            hipLaunchKernelGGL((k_vn<G, DV>), dim3(blocks(C.n * gv, 4)), blk, 0, s, A, k);
        }
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_syn, dim3(blocks(C.m * B, 256)), blk, 0, s, A, 0);
    hipLaunchKernelGGL(k_fin, dim3(blocks(B, 256)), blk, 0, s, A);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (A.io.dump_a && fused) {
        hipLaunchKernelGGL(k_fdump<G>, dim3(blocks(C.n * gd, 4)), blk, 0, s, A);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    } else if (A.io.dump_a) {
        const long total = (long)C.E * B * G;
        hipLaunchKernelGGL(k_dump, dim3(blocks(total, 256)), blk, 0, s, A, (const int *)A.w.u, (int *)A.io.dump_a);
        hipLaunchKernelGGL(k_dump, dim3(blocks(total, 256)), blk, 0, s, A, (const int *)A.w.v, (int *)A.io.dump_b);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    return hipSuccess;
}

template <int G>
hipError_t run_degrees(const Args &A, bool small_dc, bool small_dv, hipStream_t s) {
    constexpr int D = kNbDcMax, V = dev::spa::kVnRegs;
    if constexpr (G > 64) {  // check and variable degrees up to 4 only (spa_supported)
        (void)small_dc, (void)small_dv;
        return run<G, 4, 4>(A, s);
    } else {
        if (small_dc) return small_dv ? run<G, 4, 4>(A, s) : run<G, 4, V>(A, s);
        return small_dv ? run<G, D, 4>(A, s) : run<G, D, V>(A, s);
    }
}

template <int G>
hipError_t run_lds(const Args &A, int cw, int threads, hipStream_t s) {
    const size_t lds = dev::spa::lds_layout(A.C, cw).total;
    allow_full_lds((const void *)k_spa_lds<G>);
    hipLaunchKernelGGL(k_spa_lds<G>, dim3(blocks(A.batch, cw)), dim3(threads), lds, s, A, cw);
    return hipGetLastError();
}

}  // namespace

bool spa_supported(const DevCode &C) {
    if (C.g > 64) return (C.g == 128 || C.g == 256) && C.dc_max <= 4 && C.dv_max <= 4;
    return C.g >= 4 && C.dc_max <= kNbDcMax && C.dv_max <= dev::spa::kVnRegs;
}

int spa_cw_per_wave(const DevCode &C) {
    return C.dc_max <= 4 ? 64 / std::min(16, std::max(4, C.g / 4)) : 64 / std::min(C.g, 16);
}

size_t spa_work_bytes(const DevCode &C, int max_iters, int batch) { return dev::spa::carve(C, max_iters, batch).total; }

hipError_t launch_spa(const DevCode &C, int max_iters, int early_stop, int batch, void *ws, const DecodeIO &io,
                      hipStream_t s) {
    const Args A = dev::spa::make_args(C, max_iters, early_stop, batch, ws, io);
    const bool small_dc = C.dc_max <= 4, small_dv = C.dv_max <= 4;
    switch (C.g) {
    case 4: return run_degrees<4>(A, small_dc, small_dv, s);
    case 8: return run_degrees<8>(A, small_dc, small_dv, s);
    case 16: return run_degrees<16>(A, small_dc, small_dv, s);
    case 32: return run_degrees<32>(A, small_dc, small_dv, s);
    case 64: return run_degrees<64>(A, small_dc, small_dv, s);
    case 128: return run_degrees<128>(A, small_dc, small_dv, s);
    case 256: return run_degrees<256>(A, small_dc, small_dv, s);
    default: return hipErrorInvalidValue;
    }
}

size_t spa_lds_bytes(const DevCode &C, int cw) { return dev::spa::lds_layout(C, cw).total; }

bool spa_lds_supported(const DevCode &C) {
    return spa_supported(C) && C.g <= 64 && C.dc_max <= 4 && C.dv_max <= 4 && spa_lds_bytes(C, 1) <= kSpaLdsMax;
}

int spa_lds_cpw(const DevCode &C) { return 64 / std::max(4, C.g / 4); }

int spa_lds_fit(const DevCode &C) {
    int cw = 64;
    while (cw > 1 && spa_lds_bytes(C, cw) > kSpaLdsMax) --cw;
    return cw;
}

int spa_lds_cw(const DevCode &C, int batch) {
    const int fit = std::min(spa_lds_fit(C), 32), cpw = spa_lds_cpw(C);
    int cw = fit >= cpw ? fit - fit % cpw : fit;
    // small batches: at least one workgroup per compute unit rather than full groups
    cw = std::min(cw, std::max(1, (batch + 255) / 256));
    return std::max(1, std::min(cw, batch));
}

hipError_t launch_spa_lds(const DevCode &C, int max_iters, int early_stop, int batch, int cw, int threads,
                          const DecodeIO &io, hipStream_t s) {
    if (!spa_lds_supported(C) || cw < 1 || spa_lds_bytes(C, cw) > kSpaLdsMax ||
        (threads != 256 && threads != 512 && threads != 1024))
        return hipErrorInvalidValue;
    if (batch == 0) return hipSuccess;
    Args A{};
    A.C = C;
    A.max_iters = max_iters;
    A.early_stop = early_stop;
    A.batch = batch;
    A.io = io;
    switch (C.g) {
    case 4: return run_lds<4>(A, cw, threads, s);
    case 8: return run_lds<8>(A, cw, threads, s);
    case 16: return run_lds<16>(A, cw, threads, s);
    case 32: return run_lds<32>(A, cw, threads, s);
    case 64: return run_lds<64>(A, cw, threads, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace ldpcx
