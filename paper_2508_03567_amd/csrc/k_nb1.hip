// Min-Max with one codeword per workgroup, every message in LDS (plan family 7); the
// device code is dev_nb1.h.  One workgroup per codeword, all iterations in one launch.
#include <algorithm>

#include "dev_nb1.h"

namespace ldpcx {

namespace {

// Degree bound 4: up to 1024 threads; degree bound 16 keeps its larger register arrays
// without spilling at 256 threads.  AF: alpha-free decoding (degree bound 4 only).
template <int G, int DC, class M, bool AF>
__global__ void __launch_bounds__(DC <= 4 ? 1024 : 256) k_nb1(dev::nb1::Job J) {
    extern __shared__ __align__(16) unsigned char lds[];
    dev::nb1::decode_cw<G, DC, M, AF>(J, blockIdx.x, lds);
}

template <int G, int DC, class M, bool AF>
hipError_t run(const dev::nb1::Job &J, int threads, size_t lds, hipStream_t s) {
    allow_full_lds((const void *)k_nb1<G, DC, M, AF>);
    hipLaunchKernelGGL((k_nb1<G, DC, M, AF>), dim3(J.batch), dim3(threads), lds, s, J);
    return hipGetLastError();
}

template <int G, class M>
hipError_t run_dc(const dev::nb1::Job &J, bool af, int threads, size_t lds, hipStream_t s) {
    if (J.C.dc_max <= 4) return af ? run<G, 4, M, true>(J, threads, lds, s) : run<G, 4, M, false>(J, threads, lds, s);
    return run<G, kNbDcMax, M, false>(J, std::min(threads, 256), lds, s);
}

template <int G>
hipError_t run_m(const dev::nb1::Job &J, bool af, int threads, size_t lds, hipStream_t s) {
    return dev::nb1::msg_bytes(J.amax) == 1 ? run_dc<G, uint8_t>(J, af, threads, lds, s)
                                            : run_dc<G, int16_t>(J, af, threads, lds, s);
}

}  // namespace

size_t nb1_lds_bytes(const DevCode &C, int amax) { return dev::nb1::layout(C, dev::nb1::msg_bytes(amax)).total; }

bool nb1_alpha_free(const DevCode &C, int layered, bool dump, int threads) {
    // every variable of degree 2, check degree bound 4, 16-bit table entries
    if (C.dv_max != 2 || C.E != 2 * C.n || C.dc_max > 4 || C.n > 65535 || C.E > 65535) return false;
    if (layered) return !dump;  // the dump reports stored alphas of the layered schedule
    const int S = C.g >= 8 ? C.g / 8 : 1;
    const int segs = threads / 64 * (64 / S);
    return C.m <= 2 * segs;  // at most two checks per segment
}

bool nb1_supported(const DevCode &C, int amax) {
    return C.g >= 4 && C.g <= 64 && C.dc_max <= kNbDcMax && nb1_lds_bytes(C, amax) <= (size_t)160 * 1024;
}

hipError_t launch_nb1(const DevCode &C, int max_iters, int early_stop, int layered, int batch, int amax, int threads,
                      const DecodeIO &io, hipStream_t s) {
    if (!nb1_supported(C, amax) || threads < 64 || threads > 1024 || threads % 64) return hipErrorInvalidValue;
    if (layered && (C.nb_nl < 1 || C.nb_lmax < 1 || C.nb_emax < 1)) return hipErrorInvalidValue;
    if (batch <= 0) return hipSuccess;
    const dev::nb1::Job J{C, max_iters, early_stop, layered, amax, batch, io};
    const bool af = nb1_alpha_free(C, layered, io.dump_a != nullptr, threads);
    const size_t lds = dev::nb1::layout(C, dev::nb1::msg_bytes(amax), af).total;
    switch (C.g) {
    case 4: return run_m<4>(J, af, threads, lds, s);
    case 8: return run_m<8>(J, af, threads, lds, s);
    case 16: return run_m<16>(J, af, threads, lds, s);
    case 32: return run_m<32>(J, af, threads, lds, s);
    case 64: return run_m<64>(J, af, threads, lds, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace ldpcx
