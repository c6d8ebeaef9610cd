// LDS-resident binary min-sum decoder (flooding and layered schedules).
//
// One workgroup decodes `cpw` whole codewords and keeps all of their state on
// chip for every iteration: the a posteriori sums Lambda (int16, one per
// variable node), the compressed check-node state (32 bits per check: two
// smallest magnitudes, position of the smallest and the sign of every incoming
// message) and, for flooding, the channel LLRs.  Only the channel input and the
// decisions cross HBM.  A thread processes one check row at a time with the
// incoming messages in registers; the check rule is the min-sum form of the
// binary (GF(2)) Min-Max check node (sec. 2.2, Alg. 2 with g = 2).
#include "dev_bin_lds.h"

namespace ldpcx {

namespace {

template <bool LAYERED>
__global__ void __launch_bounds__(1024) k_bin_lds(DevCode C, BinRule R, int max_iters, int early_stop, int batch,
                                                  int cpw, DecodeIO io) {
    extern __shared__ __align__(16) unsigned char smem[];
    dev::lds::lds_item<LAYERED>(C, R, max_iters, early_stop, batch, cpw, io, blockIdx.x, smem);
}

}  // namespace

size_t bin_lds_smem_bytes(const DevCode &C, int layered, int cpw) {
    return dev::lds::lds_layout(C.n, C.m, layered, cpw).total;
}

hipError_t launch_bin_lds(const DevCode &C, const BinRule &R, int max_iters, int early_stop, int layered,
                          int batch, int cpw, int threads, const DecodeIO &io, hipStream_t s) {
    const size_t smem = bin_lds_smem_bytes(C, layered, cpw);
    const int grid = (batch + cpw - 1) / cpw;
    if (layered) {
        allow_full_lds((const void *)k_bin_lds<true>);
        hipLaunchKernelGGL(k_bin_lds<true>, dim3(grid), dim3(threads), smem, s, C, R, max_iters, early_stop,
                           batch, cpw, io);
    } else {
        allow_full_lds((const void *)k_bin_lds<false>);
        hipLaunchKernelGGL(k_bin_lds<false>, dim3(grid), dim3(threads), smem, s, C, R, max_iters, early_stop,
                           batch, cpw, io);
    }
    return hipGetLastError();
}

}  // namespace ldpcx
