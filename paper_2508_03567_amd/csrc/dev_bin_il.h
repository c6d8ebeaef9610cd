// Interleaved binary min-sum decoder (flooding), for codes whose per-codeword
// state does not fit on chip (e.g. n = 64800), as block-level device functions.
//
// Layout: every per-node quantity is stored as [node][Bp] with the codeword
// index fastest, so a wavefront holds 64 codewords (one per lane) of the same
// node: every gather through the Tanner graph is a uniform (scalar) index and
// every memory access is one contiguous 64-128-256 byte segment.  Per
// iteration one phase runs the check nodes (one wave per check and 64
// codewords) and one the variable nodes, with compressed check state (32 bits
// per check and codeword) kept in device memory between them.  Hard decisions
// are kept as 64-bit lane masks per variable node, so the syndrome of 64
// codewords is a XOR of dc words per check.
//
// All functions assume blocks of 256 threads (4 waves); the block index is
// passed explicitly so the same code runs from its own kernel launch or as a
// task of the persistent ragged engine.
#pragma once

#include "dev_common.h"

namespace ldpcx {
namespace dev {
namespace il {

struct Args {
    DevCode C;
    BinRule R;
    int max_iters, early_stop, batch, Bp, Gn;
    BinIlWork w;
    uint8_t *bytes_t;  // [ceil(n/8)][Bp] staging of the packed decisions
    DecodeIO io;
};

struct Unp {
    int fm1, fm2, idx;
    uint32_t signs, parity;
};

__device__ __forceinline__ Unp unp(const BinRule &R, uint32_t s) {
    Unp u;
    u.fm1 = bin_norm(R, (int)(s & 127u));
    u.fm2 = bin_norm(R, (int)((s >> 7) & 127u));
    u.idx = (int)((s >> 14) & 15u);
    u.signs = s >> 18;
    u.parity = __popc(u.signs) & 1u;
    return u;
}

__device__ __forceinline__ bool lane_active(int early, const uint64_t *unsat_slot, int g, int lane, int b, int batch) {
    if (b >= batch) return false;
    return !early || ((unsat_slot[g] >> lane) & 1ull);
}

// Virtual grids (blocks of 256 threads) of the phases.
__host__ __device__ inline long grid_init(const Args &A) { return ((long)A.C.n * A.Bp + 255) / 256; }
__host__ __device__ inline long grid_syn(const Args &A) { return ((long)((A.C.m + 31) / 32) * A.Gn + 255) / 256; }
__host__ __device__ inline long grid_cn_x(const Args &A) { return (A.C.m + 3) / 4; }
__host__ __device__ inline long grid_vn_x(const Args &A) { return (A.C.n + 3) / 4; }
__host__ __device__ inline long grid_bytes(const Args &A) { return ((long)((A.C.n + 7) / 8) * A.Bp + 255) / 256; }
__host__ __device__ inline long grid_fin(const Args &A) { return (A.batch + 255) / 256; }

// Lambda = L, hard-decision masks of iteration 0.
__device__ __forceinline__ void init_block(const Args &A, long bx) {
    const long i = bx * 256 + threadIdx.x;
    if (i >= (long)A.C.n * A.Bp) return;
    const int v = (int)(i / A.Bp);
    const int b = (int)(i - (long)v * A.Bp);
    const int8_t l = A.w.L[i];
    A.w.lam[i] = l;
    const uint64_t bits = __ballot(l < 0 && b < A.batch);
    if ((threadIdx.x & 63) == 0) A.w.hb[(long)v * A.Gn + (b >> 6)] = bits;
}

// Syndrome test for every (group of 64 codewords, block of 32 checks): ORs the
// per-check parity masks into the unsatisfied-codeword mask of each group.
__device__ __forceinline__ void syn_block(const Args &A, int slot_k, long bx) {
    const DevCode &C = A.C;
    uint64_t *slot = A.w.unsat + (size_t)slot_k * A.Gn;
    const long t = bx * 256 + threadIdx.x;
    const int g = (int)(t % A.Gn);
    const int chunk = (int)(t / A.Gn);
    const int r0 = chunk * 32;
    if (r0 >= C.m) return;
    const int r1 = min(C.m, r0 + 32);
    uint64_t acc = 0;
    for (int row = r0; row < r1; ++row) {
        uint64_t p = 0;
        for (int e = C.row_ptr[row]; e < C.row_ptr[row + 1]; ++e) p ^= A.w.hb[(long)C.col_idx[e] * A.Gn + g];
        acc |= p;
    }
    if (acc) atomicOr((unsigned long long *)&slot[g], (unsigned long long)acc);
}

// Check-node phase of iteration k: one wave per (check, group of 64 codewords).
__device__ __forceinline__ void cn_block(const Args &A, int k, int bx, int by) {
    const DevCode &C = A.C;
    const BinRule &R = A.R;
    const int lane = threadIdx.x & 63;
    const int row = bx * 4 + (threadIdx.x >> 6);
    if (row >= C.m) return;
    const int g = by;
    const int b = g * 64 + lane;
    const uint64_t *slot = A.w.unsat + (size_t)k * A.Gn;
    const bool act = lane_active(A.early_stop, slot, g, lane, b, A.batch);
    if (__ballot(act) == 0) return;
    const int e0 = C.row_ptr[row];
    const int dc = C.row_ptr[row + 1] - e0;
    const long off = (long)row * A.Bp + b;
    const Unp o = unp(R, A.w.st[off]);
    const int mm = R.msg_max;
    int m1 = 1 << 20, m2 = 1 << 20, idx = 0;
    uint32_t sg = 0;
#pragma unroll
    for (int j = 0; j < kBinDcMax; ++j) {
        if (j < dc) {
            const int v = C.col_idx[e0 + j];
            const int q =
                clampi((int)A.w.lam[(long)v * A.Bp + b] - bin_r(j, o.fm1, o.fm2, o.idx, o.signs, o.parity), -mm, mm);
            const int a = q < 0 ? -q : q;
            sg |= (uint32_t)(q < 0) << j;
            if (a < m1) {
                m2 = m1;
                m1 = a;
                idx = j;
            } else if (a < m2) {
                m2 = a;
            }
        }
    }
    if (act) A.w.st[off] = st_pack(m1, m2, idx, sg);
}

// Variable-node phase of iteration k: one wave per (variable, group).
__device__ __forceinline__ void vn_block(const Args &A, int k, int bx, int by) {
    const DevCode &C = A.C;
    const BinRule &R = A.R;
    const int lane = threadIdx.x & 63;
    const int v = bx * 4 + (threadIdx.x >> 6);
    if (v >= C.n) return;
    const int g = by;
    const int b = g * 64 + lane;
    const uint64_t *slot = A.w.unsat + (size_t)k * A.Gn;
    const bool act = lane_active(A.early_stop, slot, g, lane, b, A.batch);
    if (__ballot(act) == 0) return;
    const long off = (long)v * A.Bp + b;
    int acc = A.w.L[off];
    const int t1 = C.vn_ptr[v + 1];
    for (int t = C.vn_ptr[v]; t < t1; ++t) {
        const int ref = C.vn_ref[t];
        const Unp u = unp(R, A.w.st[(long)(ref >> 4) * A.Bp + b]);
        acc += bin_r(ref & 15, u.fm1, u.fm2, u.idx, u.signs, u.parity);
    }
    int fin = acc;
    if (act) A.w.lam[off] = (int16_t)acc;
    else fin = A.w.lam[off];
    const uint64_t bits = __ballot(fin < 0 && b < A.batch);
    if (lane == 0) A.w.hb[(long)v * A.Gn + g] = bits;
    if (v == 0 && act) A.w.it[b] = (int16_t)k;
}

// Packed decision bytes in the interleaved layout.
__device__ __forceinline__ void bytes_block(const Args &A, long bx) {
    const int n = A.C.n;
    const long i = bx * 256 + threadIdx.x;
    const int nbytes = (n + 7) >> 3;
    if (i >= (long)nbytes * A.Bp) return;
    const int j = (int)(i / A.Bp);
    const int b = (int)(i - (long)j * A.Bp);
    const int g = b >> 6, lane = b & 63;
    uint32_t byte = 0;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const int v = 8 * j + k;
        if (v < n) byte |= (uint32_t)((A.w.hb[(long)v * A.Gn + g] >> lane) & 1ull) << k;
    }
    A.bytes_t[i] = (uint8_t)byte;
}

// Syndrome flags (final test in slot 0) and iteration counts.
__device__ __forceinline__ void fin_block(const Args &A, long bx) {
    const int b = (int)(bx * 256 + threadIdx.x);
    if (b >= A.batch) return;
    A.io.ok[b] = ((A.w.unsat[b >> 6] >> (b & 63)) & 1ull) ? 0 : 1;
    A.io.iters[b] = A.w.it[b];
}

// Per-edge messages in the interleaved layout, for the debug dump.
__device__ __forceinline__ void dump_block(const Args &A, int8_t *q_t, int8_t *r_t, int bx, int by) {
    const DevCode &C = A.C;
    const BinRule &R = A.R;
    const int lane = threadIdx.x & 63;
    const int row = bx * 4 + (threadIdx.x >> 6);
    if (row >= C.m) return;
    const int b = by * 64 + lane;
    const Unp u = unp(R, A.w.st[(long)row * A.Bp + b]);
    const int e0 = C.row_ptr[row], e1 = C.row_ptr[row + 1];
    for (int e = e0; e < e1; ++e) {
        const int r = bin_r(e - e0, u.fm1, u.fm2, u.idx, u.signs, u.parity);
        r_t[(long)e * A.Bp + b] = (int8_t)r;
        q_t[(long)e * A.Bp + b] =
            (int8_t)clampi((int)A.w.lam[(long)C.col_idx[e] * A.Bp + b] - r, -R.msg_max, R.msg_max);
    }
}

struct Carve {
    size_t L, lam, st, hb, unsat, it, bytes, total;
};

inline Carve carve(const DevCode &C, int max_iters, int batch) {
    const size_t Bp = pad64(batch), Gn = Bp / 64;
    Carve c;
    size_t o = 0;
    c.L = o;
    o = align_up(o + (size_t)C.n * Bp, 256);
    c.lam = o;
    o = align_up(o + (size_t)C.n * Bp * 2, 256);
    c.st = o;
    o = align_up(o + (size_t)C.m * Bp * 4, 256);
    c.hb = o;
    o = align_up(o + (size_t)C.n * Gn * 8, 256);
    c.unsat = o;
    o = align_up(o + (size_t)(max_iters + 1) * Gn * 8, 256);
    c.it = o;
    o = align_up(o + Bp * 2, 256);
    c.bytes = o;
    o = align_up(o + (size_t)((C.n + 7) / 8) * Bp, 256);
    c.total = o;
    return c;
}

// Argument block of one decode over the workspace at `base`.
inline Args make_args(const DevCode &C, const BinRule &R, int max_iters, int early_stop, int batch, void *base,
                      const DecodeIO &io) {
    Args A;
    A.C = C;
    A.R = R;
    A.max_iters = max_iters;
    A.early_stop = early_stop;
    A.batch = batch;
    A.Bp = pad64(batch);
    A.Gn = A.Bp / 64;
    const Carve c = carve(C, max_iters, batch);
    char *p = (char *)base;
    A.w.L = (int8_t *)(p + c.L);
    A.w.lam = (int16_t *)(p + c.lam);
    A.w.st = (uint32_t *)(p + c.st);
    A.w.hb = (uint64_t *)(p + c.hb);
    A.w.unsat = (uint64_t *)(p + c.unsat);
    A.w.it = (int16_t *)(p + c.it);
    A.bytes_t = (uint8_t *)(p + c.bytes);
    A.io = io;
    return A;
}

// Transposes in and out of the interleaved layout.
inline TransposeArgs tr_in(const Args &A) {
    return TransposeArgs{A.io.llr, A.w.L, A.batch, A.C.n, A.C.n, A.Bp, A.Bp, 1};
}
inline TransposeArgs tr_out(const Args &A) {
    const long nb = (A.C.n + 7) / 8;
    return TransposeArgs{A.bytes_t, A.io.hard, nb, A.batch, A.Bp, nb, nb, 1};
}
inline FillArgs fill_st(const Args &A) { return FillArgs{A.w.st, (size_t)A.C.m * A.Bp, 0u}; }
inline FillArgs fill_unsat(const Args &A) {
    return FillArgs{(uint32_t *)A.w.unsat, (size_t)(A.max_iters + 1) * A.Gn * 2, 0u};
}
inline FillArgs fill_it(const Args &A) { return FillArgs{(uint32_t *)A.w.it, (size_t)A.Bp / 2, 0u}; }

}  // namespace il
}  // namespace dev
}  // namespace ldpcx
