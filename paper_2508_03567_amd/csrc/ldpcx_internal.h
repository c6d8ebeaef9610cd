// Internal declarations shared by the HIP kernels and the host runtime of libldpcx.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "../../include/ldpcx.h"

namespace ldpcx {

constexpr int kBinDcMax = 14;  // binary check state: 7b min1 | 7b min2 | 4b argmin | 14 sign bits
constexpr int kNbDcMax = 16;
constexpr int kWave = 64;
constexpr int kSpaWeights = 72;  // symbol costs c >= 70 have weight 0 in Q24

// Read-only device image of a code handle.
struct DevCode {
    int n, m, E, g, p, z, nlayers, dc_max, dv_max;
    const int *row_ptr;    // [m + 1]
    const int *col_idx;    // [E]
    const int *vn_ptr;     // [n + 1]  edges of each variable node (CSC)
    const int *vn_ref;     // [E] binary: (check << 4) | position in row ; g > 2: edge id
    const int *vn_edge;    // [E] CSR edge id of every CSC entry
    const uint8_t *h;      // [E] GF coefficient (g > 2)
    const uint8_t *hinv;   // [E] its inverse (g > 2)
    const uint8_t *gfmul;  // [g * g] multiplication table (g > 2)
    const int *spa_w;      // [kSpaWeights] channel weights round(2^24 exp(-c / 4)) of the FFT-SPA decoder
    // Layers of the layered Min-Max schedule (g > 2): greedy colouring of the checks in
    // ascending order, each check in the lowest layer that holds no check sharing a variable.
    int nb_nl, nb_lmax, nb_emax;  // number of layers, checks and edges in the largest
    const int *nbl_ptr;    // [nb_nl + 1]
    const int *nbl_chk;    // [m] checks layer by layer, ascending within a layer
    const int *nbl_eptr;   // [nb_nl + 1]
    const int *nbl_edge;   // [E] edges of those checks in the same order
};

struct BinRule {
    int rule, nms_num, nms_shift, oms_offset, msg_max;
};

// Outputs of one decode.  Dump pointers may be null.
struct DecodeIO {
    const void *llr;
    void *hard;
    uint8_t *ok;
    int16_t *iters;
    void *dump_a, *dump_b, *dump_c;
};

// Binary check-node state packed in 32 bits: |min1| (7b), |min2| (7b), argmin (4b),
// sign bit of every incoming message (bit 18 + position).
__host__ __device__ inline uint32_t st_pack(int m1, int m2, int idx, uint32_t signs) {
    return (uint32_t)m1 | ((uint32_t)m2 << 7) | ((uint32_t)idx << 14) | (signs << 18);
}

// Magnitude normalisation f of the min-sum variants.
__device__ __forceinline__ int bin_norm(const BinRule &R, int m) {
    if (R.rule == LDPCX_RULE_NMS) return (R.nms_num * m) >> R.nms_shift;
    if (R.rule == LDPCX_RULE_OMS) return m > R.oms_offset ? m - R.oms_offset : 0;
    return m;
}

// Outgoing check-to-variable message of position j given an unpacked state.
__device__ __forceinline__ int bin_r(int j, int fm1, int fm2, int idx, uint32_t signs, uint32_t parity) {
    int mag = (j == idx) ? fm2 : fm1;
    uint32_t neg = parity ^ ((signs >> j) & 1u);
    return neg ? -mag : mag;
}

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

// Raise a kernel's dynamic-LDS limit to 160 KB on the current device, once per (kernel,
// device); thread-safe, best effort (a kernel whose launch needs more than 64 KB then
// fails at launch if the attribute could not be set).
void allow_full_lds(const void *kernel);

// ---------------------------------------------------------------- launchers
// Each returns a hipError_t from the launch (hipSuccess when enqueued).

// LDS-resident binary decoder: one workgroup decodes `cpw` whole codewords.
hipError_t launch_bin_lds(const DevCode &C, const BinRule &R, int max_iters, int early_stop,
                          int layered, int batch, int cpw, int threads, const DecodeIO &io,
                          hipStream_t s);
size_t bin_lds_smem_bytes(const DevCode &C, int layered, int cpw);

// Quasi-cyclic description: layer l has dc[l] circulant blocks (column block col, shift sh).
constexpr int kQcMaxL = 16, kQcMaxDc = 8;
struct QcDesc {
    int Z, nl;
    int dc[kQcMaxL];
    short col[kQcMaxL][kQcMaxDc];
    short sh[kQcMaxL][kQcMaxDc];
    const int2 *edges;  // device copy: edges[l * kQcMaxDc + j] = {col * Z, sh}
};

// Packed two-codewords-per-lane decoder for QC codes: a workgroup of Z * npairs threads
// decodes 2 * npairs codewords, messages in registers, Lambda in LDS.
hipError_t launch_bin_qc(const QcDesc &Q, const DevCode &C, const BinRule &R, int max_iters, int early_stop,
                         int layered, int batch, int npairs, const DecodeIO &io, hipStream_t s);
size_t bin_qc_smem_bytes(const QcDesc &Q, const DevCode &C, int layered, int npairs);

// Interleaved binary flooding decoder (two codewords per lane), state in device memory.
struct BinIlWork {
    int8_t *L;        // [n][Bp] channel LLRs
    int8_t *q;        // [E][Bp] variable-to-check messages (CSR edge order)
    int8_t *r;        // [E][Bp] check-to-variable messages
    uint64_t *hb;     // [n][Bp/64] hard-decision bits
    uint64_t *unsat;  // [(max_iters + 1)][Bp/64] unsatisfied-codeword masks per syndrome test
    int16_t *it;      // [Bp]
};
// Codewords per launch sequence for a requested sub-batch (0 = default): a multiple of
// 128, at most the batch (rounded up) and the 31-bit offset limit of the code.
int bin_il_sub_batch(const DevCode &C, int batch, int sub);
size_t bin_il_work_bytes(const DevCode &C, int max_iters, int batch, int sub);
size_t bin_il_dump_bytes(const DevCode &C, int batch, int sub);
// ws: workspace of bin_il_work_bytes; dump_scratch: bin_il_dump_bytes when io dumps.
hipError_t launch_bin_il(const DevCode &C, const BinRule &R, int max_iters, int early_stop, int batch, int sub,
                         void *ws, const DecodeIO &io, int8_t *dump_scratch, hipStream_t s);

// Interleaved Min-Max decoder over GF(g).
struct NbWork {
    int16_t *gam;     // [n][g][Bp]
    int16_t *alpha;   // [E][g][Bp]
    int16_t *beta;    // [E][g][Bp]
    uint8_t *hard;    // [n][Bp]
    uint64_t *unsat;  // [(max_iters + 1)][Bp/64]
    int16_t *it;      // [Bp]
};
// Fixed-point FFT-SPA (g <= 64): codeword-major rows per node / edge, Q24 int32.
struct SpaWork {
    int *p;          // [n][batch][g] channel probabilities
    int *u;          // [E][batch][g] variable-to-check messages
    int *v;          // [E][batch][g] check-to-variable messages (depermuted)
    uint8_t *unsat;  // [(max_iters + 1)][batch]
    int16_t *it;     // [batch]
};
bool spa_supported(const DevCode &C);
size_t spa_work_bytes(const DevCode &C, int max_iters, int batch);
int spa_cw_per_wave(const DevCode &C);  // codewords per wave of the check-node kernel
hipError_t launch_spa(const DevCode &C, int max_iters, int early_stop, int batch, void *ws, const DecodeIO &io,
                      hipStream_t s);
// FFT-SPA with cw codewords per workgroup and every vector in LDS (check and variable
// degrees <= 4, spa_lds_bytes(C, cw) <= kSpaLdsMax, 256, 512 or 1024 threads); no workspace.
constexpr size_t kSpaLdsMax = 160 * 1024;
bool spa_lds_supported(const DevCode &C);
size_t spa_lds_bytes(const DevCode &C, int cw);
int spa_lds_cpw(const DevCode &C);  // codewords per wave of its phases
int spa_lds_fit(const DevCode &C);  // largest cw <= 64 whose vectors fit
// Default group: the largest multiple of spa_lds_cpw up to 32 codewords that fits (else
// the largest group that fits), fewer for batches under 256 groups.
int spa_lds_cw(const DevCode &C, int batch);
hipError_t launch_spa_lds(const DevCode &C, int max_iters, int early_stop, int batch, int cw, int threads,
                          const DecodeIO &io, hipStream_t s);

// Min-Max for g = 128, 256: codeword-major rows per edge.
struct NbwWork {
    int16_t *alpha;  // [E][batch][g]
    int16_t *beta;   // [E][batch][g]
    uint8_t *unsat;  // [(max_iters + 1)][batch]
    int16_t *it;     // [batch]
};
// Codewords per launch sequence of the interleaved Min-Max decoder (31-bit offsets).
int nb_slice(const DevCode &C, int batch);
size_t nb_work_bytes(const DevCode &C, int max_iters, int batch);
// Min-Max with one group of 64 codewords per workgroup and its messages in LDS (g <= 64,
// waves = 4, 8 or 16 per workgroup, nb_lds_bytes(C, waves) <= 160 KB); same workspace as
// launch_nb.
size_t nb_lds_bytes(const DevCode &C, int waves);
hipError_t launch_nb_lds(const DevCode &C, int max_iters, int early_stop, int layered, int batch, int amax, int waves,
                         void *ws, const DecodeIO &io, hipStream_t s);
// amax: message bound (32767 for 16-bit messages, 127 for the 8-bit variant).  layered:
// the layered schedule over the layers of DevCode (g <= 64).
hipError_t launch_nb(const DevCode &C, int max_iters, int early_stop, int layered, int batch, int amax, void *ws,
                     const DecodeIO &io, hipStream_t s);
// Min-Max with one codeword per workgroup and all its messages in LDS (g <= 64, check
// degree <= 16, nb1_lds_bytes(C, amax) <= 160 KB; a multiple of 64 threads up to 1024, at
// most 256 used for check degrees above 4); no workspace, both schedules.  Messages are stored in
// 8 bits when the bound amax is at most 255, else in 16 bits.
size_t nb1_lds_bytes(const DevCode &C, int amax);
bool nb1_supported(const DevCode &C, int amax);
// Whether launch_nb1 decodes alpha-free (no stored alphas) for these arguments.
bool nb1_alpha_free(const DevCode &C, int layered, bool dump, int threads);
hipError_t launch_nb1(const DevCode &C, int max_iters, int early_stop, int layered, int batch, int amax, int threads,
                      const DecodeIO &io, hipStream_t s);
// Field sizes with a compiled Min-Max kernel (4..64 interleaved, 128 and 256 wide).
bool nb_supported(int g);
// The wide (g >= 128) decoder: workspace bytes and launch sequence.
size_t nbw_work_bytes(const DevCode &C, int max_iters, int batch);
hipError_t launch_nbw(const DevCode &C, int max_iters, int early_stop, int batch, int amax, void *ws,
                      const DecodeIO &io, hipStream_t s);

__host__ __device__ inline size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }
__host__ __device__ inline int pad64(int b) { return (b + 63) & ~63; }

}  // namespace ldpcx
