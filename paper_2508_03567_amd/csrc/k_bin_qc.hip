// Binary min-sum for quasi-cyclic codes, two codewords per lane in packed
// 16-bit arithmetic (flooding and layered schedules).
//
// A QC code is described by its base matrix: layer l (one block row of Z
// checks) has dc_l nonzero Z x Z circulant blocks (column block c, shift s);
// row i of that layer connects to variables c Z + (i + s) mod Z.  A workgroup
// decodes `npairs` pairs of codewords; thread (pair p, row i) owns row i of
// every layer, so the check-to-variable messages of its rows never leave its
// registers (one packed int16 pair per edge).  The a posteriori sums Lambda of
// the pair live in LDS as packed int16 pairs, so every LDS access and every
// VALU operation serves two codewords (v_pk_sub_i16, v_pk_max_i16, ...).
// Column indices come from the (block, shift) descriptors, staged in LDS.
//
// Every layer is processed as MD edges without branches, so all Lambda loads of
// a row are in flight together: edges beyond the layer's degree are virtual and
// read a private dummy slot holding a large positive value, so they enter the
// check with magnitude msg_max and a positive sign, which changes neither the
// two smallest magnitudes nor the sign parity (every real check has degree >= 2).
//
// The argmin position of the check-node state is not needed: an edge whose
// magnitude equals the minimum gets the second minimum, which equals the
// minimum when the minimum is tied.  The magnitude normalisation is one
// formula for the three rules: f(m) = max(((m * num) >> shift) - off, 0)
// with (num, shift, off) = (num, shift, 0) for NMS, (1, 0, off) for OMS and
// (1, 0, 0) for MS.
#include "dev_bin_qc.h"

namespace ldpcx {

namespace {

using namespace dev;

// ES: early termination compiled in (the fixed-iteration variant drops its merges).
template <int ML, int MD, bool LAYERED, bool ES>
__global__ void __launch_bounds__(512) k_bin_qc(QcDesc Q, DevCode C, BinRule R, int max_iters, int early_stop,
                                                int batch, int npairs, DecodeIO io) {
    extern __shared__ __align__(16) uint32_t lds[];
    qc_item<ML, MD, LAYERED, ES>(Q, C, R, max_iters, early_stop, batch, npairs, io, blockIdx.x, lds);
}

// Flooding with the layers in parallel (qc_item_lp): Z * npairs * nl threads.
template <int ML, int MD, bool ES>
__global__ void __launch_bounds__(1024) k_bin_qc_lp(QcDesc Q, DevCode C, BinRule R, int max_iters, int early_stop,
                                                    int batch, int npairs, DecodeIO io) {
    extern __shared__ __align__(16) uint32_t lds[];
    qc_item_lp<ML, MD, ES>(Q, C, R, max_iters, early_stop, batch, npairs, io, blockIdx.x, lds);
}

template <int ML, int MD, bool ES>
hipError_t launch_lp_es(const QcDesc &Q, const DevCode &C, const BinRule &R, int max_iters, int early_stop, int batch,
                        int npairs, const DecodeIO &io, hipStream_t s) {
    const size_t smem = qc_smem_bytes(ML, MD, C, Q.Z, false, npairs);
    const int pairs = (batch + 1) / 2;
    const int grid = (pairs + npairs - 1) / npairs;
    allow_full_lds((const void *)k_bin_qc_lp<ML, MD, ES>);
    hipLaunchKernelGGL((k_bin_qc_lp<ML, MD, ES>), dim3(grid), dim3(Q.Z * npairs * Q.nl), smem, s, Q, C, R, max_iters,
                       early_stop, batch, npairs, io);
    return hipGetLastError();
}

template <int ML, int MD, bool LAYERED, bool ES>
hipError_t launch_es(const QcDesc &Q, const DevCode &C, const BinRule &R, int max_iters, int early_stop, int batch,
                     int npairs, const DecodeIO &io, hipStream_t s) {
    const size_t smem = qc_smem_bytes(ML, MD, C, Q.Z, LAYERED, npairs);
    const int pairs = (batch + 1) / 2;
    const int grid = (pairs + npairs - 1) / npairs;
    allow_full_lds((const void *)k_bin_qc<ML, MD, LAYERED, ES>);
    hipLaunchKernelGGL((k_bin_qc<ML, MD, LAYERED, ES>), dim3(grid), dim3(Q.Z * npairs), smem, s, Q, C, R, max_iters,
                       early_stop, batch, npairs, io);
    return hipGetLastError();
}

template <int ML, int MD, bool LAYERED>
hipError_t launch_shape(const QcDesc &Q, const DevCode &C, const BinRule &R, int max_iters, int early_stop,
                        int batch, int npairs, const DecodeIO &io, hipStream_t s) {
    return early_stop ? launch_es<ML, MD, LAYERED, true>(Q, C, R, max_iters, early_stop, batch, npairs, io, s)
                      : launch_es<ML, MD, LAYERED, false>(Q, C, R, max_iters, early_stop, batch, npairs, io, s);
}

template <bool LAYERED>
hipError_t dispatch(const QcDesc &Q, const DevCode &C, const BinRule &R, int max_iters, int early_stop, int batch,
                    int npairs, const DecodeIO &io, hipStream_t s) {
    int ml, md;
    qc_shape_of(Q, ml, md);
#define LDPCX_LAUNCH(L_, D_) \
    if (ml == L_ && md == D_) return launch_shape<L_, D_, LAYERED>(Q, C, R, max_iters, early_stop, batch, npairs, io, s);
    LDPCX_QC_SHAPES(LDPCX_LAUNCH)
#undef LDPCX_LAUNCH
    return hipErrorInvalidConfiguration;
}

}  // namespace

size_t bin_qc_smem_bytes(const QcDesc &Q, const DevCode &C, int layered, int npairs) {
    int ml, md;
    qc_shape_of(Q, ml, md);
    if (!ml) return (size_t)-1;
    return qc_smem_bytes(ml, md, C, Q.Z, layered, npairs);
}

bool bin_qc_lp_ok(const QcDesc &Q, int npairs) {
    return Q.nl > 1 && Q.nl <= kQcMaxL && (Q.Z * npairs) % 64 == 0 && Q.Z * npairs * Q.nl <= 1024;
}

hipError_t launch_bin_qc_lp(const QcDesc &Q, const DevCode &C, const BinRule &R, int max_iters, int early_stop,
                            int batch, int npairs, const DecodeIO &io, hipStream_t s) {
    if (!bin_qc_lp_ok(Q, npairs)) return hipErrorInvalidConfiguration;
    int ml, md;
    qc_shape_of(Q, ml, md);
#define LDPCX_LAUNCH_LP(L_, D_)                                                                                  \
    if (ml == L_ && md == D_)                                                                                    \
        return early_stop ? launch_lp_es<L_, D_, true>(Q, C, R, max_iters, early_stop, batch, npairs, io, s)    \
                          : launch_lp_es<L_, D_, false>(Q, C, R, max_iters, early_stop, batch, npairs, io, s);
    LDPCX_QC_SHAPES(LDPCX_LAUNCH_LP)
#undef LDPCX_LAUNCH_LP
    return hipErrorInvalidConfiguration;
}

hipError_t launch_bin_qc(const QcDesc &Q, const DevCode &C, const BinRule &R, int max_iters, int early_stop,
                         int layered, int batch, int npairs, const DecodeIO &io, hipStream_t s) {
    if (Q.Z * npairs > 512 || Q.nl > kQcMaxL) return hipErrorInvalidConfiguration;
    return layered ? dispatch<true>(Q, C, R, max_iters, early_stop, batch, npairs, io, s)
                   : dispatch<false>(Q, C, R, max_iters, early_stop, batch, npairs, io, s);
}

}  // namespace ldpcx
