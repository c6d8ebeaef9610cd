// Interleaved binary min-sum decoder (flooding) for codes whose per-codeword
// state does not fit on chip (e.g. n = 64800), as block-level device functions.
//
// Layout: every per-node and per-edge quantity is stored as [node or edge][Bp]
// with the codeword index fastest (Bp = batch padded to 128).  Each lane holds two
// adjacent codewords in packed 16-bit arithmetic, so a wavefront covers a group
// of 128 codewords of one node or edge: every access is one contiguous 128-byte
// segment at a wave-uniform index, issued as a buffer load or store whose scalar
// offset carries the index (no per-lane address arithmetic).
//
// Messages live on the edges as int8: the check-node phase reads the
// variable-to-check messages q of its edges (contiguous in CSR order) and writes
// the check-to-variable messages r; the variable-node phase gathers r of its
// edges, forms Lambda = L + sum r (exact in int16), writes q = sat(Lambda - r)
// back to every edge and the hard decisions as 64-bit lane masks (one per
// codeword of the lane pair).  Per codeword and iteration this moves about
// 4E + n bytes.  Codewords that stopped (early termination) keep every message:
// a wave whose lanes are partly stopped merges old and new values per byte.
//
// All functions assume blocks of 256 threads (4 waves); the block index is passed
// explicitly so that the same code runs from its own kernel launch or inside one
// workgroup of the persistent ragged engine.
#pragma once

#include "dev_common.h"

namespace ldpcx {
namespace dev {
namespace il {

constexpr int kGroup = 128;                   // codewords per wavefront (two per lane)
constexpr int kVnRegs = 8;                    // check messages a variable keeps in registers
constexpr uint32_t kRsrcWord3 = 0x00020000u;  // raw (untyped) buffer resource, gfx9 family

struct Args {
    DevCode C;
    BinRule R;
    int max_iters, early_stop, batch, Bp, G;  // G = Bp / 128 groups
    BinIlWork w;
    uint8_t *bytes_t;  // [ceil(n/8)][Bp] staging of the packed decisions
    DecodeIO io;
};

__device__ __forceinline__ __amdgpu_buffer_rsrc_t rsrc(const void *p, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, (int)bytes, (int)kRsrcWord3);
}

// Two int8 codeword values (bytes 0 and 1 of x) -> packed int16 pair, sign extended.
__device__ __forceinline__ v2s unpack8(uint32_t x) {
    return as_v2s(__builtin_amdgcn_perm(x, x, 0x010C000Cu)) >> splat(8);
}

// Packed int16 pair (values in int8 range) -> two bytes.
__device__ __forceinline__ uint32_t pack8(v2s v) { return __builtin_amdgcn_perm(as_u32(v), as_u32(v), 0x0C0C0200u); }

__device__ __forceinline__ uint32_t ld8x2(__amdgpu_buffer_rsrc_t r, uint32_t vo, uint32_t so) {
    return __builtin_amdgcn_raw_buffer_load_b16(r, (int)vo, (int)so, 0);
}
__device__ __forceinline__ void st8x2(uint32_t v, __amdgpu_buffer_rsrc_t r, uint32_t vo, uint32_t so) {
    __builtin_amdgcn_raw_buffer_store_b16((unsigned short)v, r, (int)vo, (int)so, 0);
}

// Activity of the two codewords of each lane at iteration k.  Codewords beyond the
// batch count as active (their inputs are zero and stay zero), so that a wave of a
// partly filled group is not treated as mixed.
struct Act {
    uint32_t m8;   // per byte: 0xFF where the codeword is active
    uint32_t m16;  // per int16 half: 0xFFFF where active
    bool any, all;
};

__device__ __forceinline__ Act activity(const Args &A, int k, int g, int lane) {
    Act a{0xFFFFu, 0xFFFFFFFFu, true, true};
    if (!A.early_stop) return a;
    const uint64_t *slot = A.w.unsat + (size_t)k * 2 * A.G + 2 * g;
    const int b0 = g * kGroup + 2 * lane;
    const bool u0 = (slot[0] >> lane) & 1ull, u1 = (slot[1] >> lane) & 1ull;
    const bool a0 = u0 || b0 >= A.batch, a1 = u1 || b0 + 1 >= A.batch;
    a.m8 = (a0 ? 0x00FFu : 0u) | (a1 ? 0xFF00u : 0u);
    a.m16 = (a0 ? 0x0000FFFFu : 0u) | (a1 ? 0xFFFF0000u : 0u);
    a.any = __ballot(u0 || u1) != 0;  // only real codewords can be unsatisfied
    a.all = __ballot(!(a0 && a1)) == 0;
    return a;
}

// (M & a) | (~M & b)
__device__ __forceinline__ uint32_t merge(uint32_t M, uint32_t a, uint32_t b) { return (M & a) | (~M & b); }

// Virtual grids (blocks of 256 threads, 4 waves) of the phases.
__host__ __device__ inline long grid_rows_x(const Args &A) { return (A.C.m + 3) / 4; }
__host__ __device__ inline long grid_vars_x(const Args &A) { return (A.C.n + 3) / 4; }
__host__ __device__ inline long grid_edges_x(const Args &A) { return (A.C.E + 3) / 4; }
__host__ __device__ inline long grid_syn(const Args &A) { return ((long)((A.C.m + 31) / 32) * 2 * A.G + 255) / 256; }
__host__ __device__ inline long grid_bytes(const Args &A) { return ((long)((A.C.n + 7) / 8) * A.Bp + 255) / 256; }
__host__ __device__ inline long grid_fin(const Args &A) { return (A.batch + 255) / 256; }

// q = sat(L) of the edge's variable, r = 0 (wave per (edge, group)).
__device__ __forceinline__ void init_edges_block(const Args &A, int bx, int g) {
    const int e = bx * 4 + wave_id();
    if (e >= A.C.E) return;
    const uint32_t vo = 2 * (threadIdx.x & 63), gb = (uint32_t)g * kGroup, Bp = (uint32_t)A.Bp;
    const auto rL = rsrc(A.w.L, (uint32_t)A.C.n * Bp);
    const auto rq = rsrc(A.w.q, (uint32_t)A.C.E * Bp);
    const auto rr = rsrc(A.w.r, (uint32_t)A.C.E * Bp);
    const uint32_t v = (uint32_t)A.C.col_idx[e];
    const v2s L = unpack8(ld8x2(rL, vo, v * Bp + gb));
    st8x2(pack8(pmin(pmax(L, splat(-A.R.msg_max)), splat(A.R.msg_max))), rq, vo, (uint32_t)e * Bp + gb);
    st8x2(0u, rr, vo, (uint32_t)e * Bp + gb);
}

// Decisions of iteration 0 (wave per (variable, group)).
__device__ __forceinline__ void init_vars_block(const Args &A, int bx, int g) {
    const int v = bx * 4 + wave_id();
    if (v >= A.C.n) return;
    const int lane = threadIdx.x & 63;
    const uint32_t vo = 2 * lane, gb = (uint32_t)g * kGroup, Bp = (uint32_t)A.Bp;
    const auto rL = rsrc(A.w.L, (uint32_t)A.C.n * Bp);
    const uint32_t s = as_u32(unpack8(ld8x2(rL, vo, (uint32_t)v * Bp + gb)));
    const uint64_t b0 = __ballot((s >> 15) & 1u), b1 = __ballot(s >> 31);
    uint64_t *hb = A.w.hb + (size_t)v * 2 * A.G + 2 * g;
    if (lane == 0) hb[0] = b0;
    if (lane == 1) hb[1] = b1;
}

// Syndrome test: for every (decision word, block of 32 checks) the OR of the parity
// masks, accumulated into the unsatisfied-codeword mask of slot_k.  Word 2g + h
// holds codeword 128 g + 2 l + h in bit l.
__device__ __forceinline__ void syn_block(const Args &A, int slot_k, long bx) {
    const DevCode &C = A.C;
    const int W = 2 * A.G;
    uint64_t *slot = A.w.unsat + (size_t)slot_k * W;
    const long t = bx * 256 + threadIdx.x;
    const int wd = (int)(t % W);
    const int chunk = (int)(t / W);
    const int r0 = chunk * 32;
    if (r0 >= C.m) return;
    const int r1 = min(C.m, r0 + 32);
    uint64_t acc = 0;
    for (int row = r0; row < r1; ++row) {
        uint64_t p = 0;
        for (int e = C.row_ptr[row]; e < C.row_ptr[row + 1]; ++e) p ^= A.w.hb[(size_t)C.col_idx[e] * W + wd];
        acc |= p;
    }
    if (acc) atomicOr((unsigned long long *)&slot[wd], (unsigned long long)acc);
}

// Check-node phase of iteration k: one wave per (check, group of 128 codewords).
// Outgoing magnitude: f(min2) on the edge holding the minimum, f(min1) elsewhere
// (equal when the minimum is tied); sign: product of the other signs.
__device__ __forceinline__ void cn_block(const Args &A, int k, int bx, int g) {
    const DevCode &C = A.C;
    const int lane = threadIdx.x & 63;
    const int row = bx * 4 + wave_id();
    if (row >= C.m) return;
    const Act act = activity(A, k, g, lane);
    if (!act.any) return;
    const uint32_t vo = 2 * lane, gb = (uint32_t)g * kGroup, Bp = (uint32_t)A.Bp;
    const auto rq = rsrc(A.w.q, (uint32_t)C.E * Bp);
    const auto rr = rsrc(A.w.r, (uint32_t)C.E * Bp);
    const int e0 = C.row_ptr[row];
    const int dc = C.row_ptr[row + 1] - e0;
    const PkNorm NP = pk_norm_params(A.R);
    v2s av[kBinDcMax];
    uint32_t sv[kBinDcMax];
    v2s m1 = splat(0x7FFF), m2 = splat(0x7FFF);
    uint32_t stot = 0;
#pragma unroll
    for (int j = 0; j < kBinDcMax; ++j) {
        if (j < dc) {
            const v2s q = unpack8(ld8x2(rq, vo, (uint32_t)(e0 + j) * Bp + gb));
            const uint32_t sg = as_u32(q >> splat(15));
            const v2s a = pmax(q, -q);
            m2 = pmin(m2, pmax(m1, a));
            m1 = pmin(m1, a);
            stot ^= sg;
            av[j] = a;
            sv[j] = sg;
        }
    }
    const v2s f1 = pk_norm(NP, m1), f2 = pk_norm(NP, m2);
    const v2s df = f1 - f2;
#pragma unroll
    for (int j = 0; j < kBinDcMax; ++j) {
        if (j < dc) {
            const v2s t = pmin(av[j] - m1, splat(1));  // 0 where this edge holds the minimum
            const v2s mag = f2 + t * df;
            const uint32_t sr = stot ^ sv[j];
            uint32_t rn = pack8(as_v2s(as_u32(mag) ^ sr) - as_v2s(sr));
            const uint32_t so = (uint32_t)(e0 + j) * Bp + gb;
            if (!act.all) rn = merge(act.m8, rn, ld8x2(rr, vo, so));
            st8x2(rn, rr, vo, so);
        }
    }
}

// Variable-node phase of iteration k: one wave per (variable, group).
__device__ __forceinline__ void vn_block(const Args &A, int k, int bx, int g) {
    const DevCode &C = A.C;
    const int lane = threadIdx.x & 63;
    const int v = bx * 4 + wave_id();
    if (v >= C.n) return;
    const Act act = activity(A, k, g, lane);
    if (!act.any) return;
    const uint32_t vo = 2 * lane, gb = (uint32_t)g * kGroup, Bp = (uint32_t)A.Bp;
    const auto rL = rsrc(A.w.L, (uint32_t)C.n * Bp);
    const auto rq = rsrc(A.w.q, (uint32_t)C.E * Bp);
    const auto rr = rsrc(A.w.r, (uint32_t)C.E * Bp);
    const int t0 = C.vn_ptr[v];
    const int dv = C.vn_ptr[v + 1] - t0;
    v2s S = unpack8(ld8x2(rL, vo, (uint32_t)v * Bp + gb));
    v2s rv[kVnRegs];
    uint32_t ev[kVnRegs];
#pragma unroll
    for (int t = 0; t < kVnRegs; ++t) {
        if (t < dv) {
            ev[t] = (uint32_t)C.vn_edge[t0 + t] * Bp + gb;
            rv[t] = unpack8(ld8x2(rr, vo, ev[t]));
            S = S + rv[t];
        }
    }
    for (int t = kVnRegs; t < dv; ++t) S = S + unpack8(ld8x2(rr, vo, (uint32_t)C.vn_edge[t0 + t] * Bp + gb));
    const v2s mm = splat(A.R.msg_max), nmm = splat(-A.R.msg_max);
#pragma unroll
    for (int t = 0; t < kVnRegs; ++t) {
        if (t < dv) {
            uint32_t qn = pack8(pmin(pmax(S - rv[t], nmm), mm));
            if (!act.all) qn = merge(act.m8, qn, ld8x2(rq, vo, ev[t]));
            st8x2(qn, rq, vo, ev[t]);
        }
    }
    for (int t = kVnRegs; t < dv; ++t) {
        const uint32_t so = (uint32_t)C.vn_edge[t0 + t] * Bp + gb;
        uint32_t qn = pack8(pmin(pmax(S - unpack8(ld8x2(rr, vo, so)), nmm), mm));
        if (!act.all) qn = merge(act.m8, qn, ld8x2(rq, vo, so));
        st8x2(qn, rq, vo, so);
    }
    const uint32_t s = as_u32(S);
    uint64_t b0 = __ballot((s >> 15) & 1u), b1 = __ballot(s >> 31);
    uint64_t *hb = A.w.hb + (size_t)v * 2 * A.G + 2 * g;
    if (!act.all) {
        const uint64_t k0 = __ballot(act.m16 & 1u), k1 = __ballot(act.m16 >> 31);
        b0 = (b0 & k0) | (hb[0] & ~k0);
        b1 = (b1 & k1) | (hb[1] & ~k1);
    }
    if (lane == 0) hb[0] = b0;
    if (lane == 1) hb[1] = b1;
    if (v == 0) {
        uint32_t *itp = (uint32_t *)(A.w.it + g * kGroup) + lane;
        const uint32_t kk = (uint32_t)k | ((uint32_t)k << 16);
        *itp = act.all ? kk : merge(act.m16, kk, *itp);
    }
}

// Decision bit of codeword b for variable v.
__device__ __forceinline__ uint32_t hbit(const Args &A, int v, int b) {
    const int g = b / kGroup, rem = b - g * kGroup;
    return (uint32_t)((A.w.hb[(size_t)v * 2 * A.G + 2 * g + (rem & 1)] >> (rem >> 1)) & 1ull);
}

// Packed decision bytes in the interleaved layout.
__device__ __forceinline__ void bytes_block(const Args &A, long bx) {
    const int n = A.C.n;
    const long i = bx * 256 + threadIdx.x;
    const int nbytes = (n + 7) >> 3;
    if (i >= (long)nbytes * A.Bp) return;
    const int j = (int)(i / A.Bp);
    const int b = (int)(i - (long)j * A.Bp);
    uint32_t byte = 0;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const int v = 8 * j + q;
        if (v < n) byte |= hbit(A, v, b) << q;
    }
    A.bytes_t[i] = (uint8_t)byte;
}

// Syndrome flags (final test in slot 0) and iteration counts.
__device__ __forceinline__ void fin_block(const Args &A, long bx) {
    const int b = (int)(bx * 256 + threadIdx.x);
    if (b >= A.batch) return;
    const int g = b / kGroup, rem = b - g * kGroup;
    A.io.ok[b] = ((A.w.unsat[2 * g + (rem & 1)] >> (rem >> 1)) & 1ull) ? 0 : 1;
    A.io.iters[b] = A.w.it[b];
}

// Lambda = L + sum r per variable in the interleaved layout, for the debug dump.
__device__ __forceinline__ void lambda_block(const Args &A, int16_t *lam_t, int bx, int g) {
    const DevCode &C = A.C;
    const int lane = threadIdx.x & 63;
    const int v = bx * 4 + wave_id();
    if (v >= C.n) return;
    const uint32_t vo = 2 * lane, gb = (uint32_t)g * kGroup, Bp = (uint32_t)A.Bp;
    const auto rL = rsrc(A.w.L, (uint32_t)C.n * Bp);
    const auto rr = rsrc(A.w.r, (uint32_t)C.E * Bp);
    v2s S = unpack8(ld8x2(rL, vo, (uint32_t)v * Bp + gb));
    for (int t = C.vn_ptr[v]; t < C.vn_ptr[v + 1]; ++t)
        S = S + unpack8(ld8x2(rr, vo, (uint32_t)C.vn_edge[t] * Bp + gb));
    *(uint32_t *)(lam_t + (size_t)v * A.Bp + gb + vo) = as_u32(S);
}

__host__ __device__ inline int pad128(int b) { return (b + 127) & ~127; }

struct Carve {
    size_t L, q, r, hb, unsat, it, bytes, total;
};

inline Carve carve(const DevCode &C, int max_iters, int batch) {
    const size_t Bp = pad128(batch), W = Bp / 64;
    Carve c;
    size_t o = 0;
    c.L = o;
    o = align_up(o + (size_t)C.n * Bp, 256);
    c.q = o;
    o = align_up(o + (size_t)C.E * Bp, 256);
    c.r = o;
    o = align_up(o + (size_t)C.E * Bp, 256);
    c.hb = o;
    o = align_up(o + (size_t)C.n * W * 8, 256);
    c.unsat = o;
    o = align_up(o + (size_t)(max_iters + 1) * W * 8, 256);
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
    A.Bp = pad128(batch);
    A.G = A.Bp / kGroup;
    const Carve c = carve(C, max_iters, batch);
    char *p = (char *)base;
    A.w.L = (int8_t *)(p + c.L);
    A.w.q = (int8_t *)(p + c.q);
    A.w.r = (int8_t *)(p + c.r);
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
inline FillArgs fill_unsat(const Args &A) {
    return FillArgs{(uint32_t *)A.w.unsat, (size_t)(A.max_iters + 1) * 2 * A.G * 2, 0u};
}
inline FillArgs fill_it(const Args &A) { return FillArgs{(uint32_t *)A.w.it, (size_t)A.Bp / 2, 0u}; }

// Largest batch one launch sequence may take, so that every byte offset into a
// per-edge or per-variable array (and the int16 Lambda of the dump) fits 31 bits.
inline int max_sub_batch(const DevCode &C) {
    const size_t per = (size_t)(C.E > 2 * C.n ? C.E : 2 * C.n);
    size_t b = (((size_t)1 << 31) - 1) / (per > 0 ? per : 1);
    b = b / kGroup * kGroup;
    if (b < (size_t)kGroup) b = kGroup;
    if (b > ((size_t)1 << 20)) b = (size_t)1 << 20;
    return (int)b;
}

}  // namespace il
}  // namespace dev
}  // namespace ldpcx
