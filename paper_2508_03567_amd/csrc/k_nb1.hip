// Min-Max with one codeword per workgroup, every message in LDS (plan family 7); the
// device code is dev_nb1.h.  One workgroup per codeword, all iterations in one launch.
#include <algorithm>

#include "dev_nb1.h"

namespace ldpcx {

namespace {

// Degree bound 4: up to 1024 threads; degree bound 16 keeps its larger register arrays
// without spilling at 256 threads.
template <int G, int DC>
__global__ void __launch_bounds__(DC <= 4 ? 1024 : 256) k_nb1(dev::nb1::Job J) {
    extern __shared__ __align__(16) unsigned char lds[];
    dev::nb1::decode_cw<G, DC>(J, blockIdx.x, lds);
}

template <int G, int DC>
hipError_t run(const dev::nb1::Job &J, int threads, size_t lds, hipStream_t s) {
    allow_full_lds((const void *)k_nb1<G, DC>);
    hipLaunchKernelGGL((k_nb1<G, DC>), dim3(J.batch), dim3(threads), lds, s, J);
    return hipGetLastError();
}

template <int G>
hipError_t run_dc(const dev::nb1::Job &J, int threads, size_t lds, hipStream_t s) {
    return J.C.dc_max <= 4 ? run<G, 4>(J, threads, lds, s) : run<G, kNbDcMax>(J, std::min(threads, 256), lds, s);
}

}  // namespace

size_t nb1_lds_bytes(const DevCode &C) { return dev::nb1::layout(C).total; }

bool nb1_supported(const DevCode &C) {
    return C.g >= 4 && C.g <= 64 && C.dc_max <= kNbDcMax && nb1_lds_bytes(C) <= (size_t)160 * 1024;
}

hipError_t launch_nb1(const DevCode &C, int max_iters, int early_stop, int layered, int batch, int amax, int threads,
                      const DecodeIO &io, hipStream_t s) {
    if (!nb1_supported(C) || (threads != 256 && threads != 512 && threads != 1024)) return hipErrorInvalidValue;
    if (layered && (C.nb_nl < 1 || C.nb_lmax < 1 || C.nb_emax < 1)) return hipErrorInvalidValue;
    if (batch <= 0) return hipSuccess;
    const dev::nb1::Job J{C, max_iters, early_stop, layered, amax, batch, io};
    const size_t lds = nb1_lds_bytes(C);
    switch (C.g) {
    case 4: return run_dc<4>(J, threads, lds, s);
    case 8: return run_dc<8>(J, threads, lds, s);
    case 16: return run_dc<16>(J, threads, lds, s);
    case 32: return run_dc<32>(J, threads, lds, s);
    case 64: return run_dc<64>(J, threads, lds, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace ldpcx
