// Interleaved binary min-sum decoder (flooding) for codes whose per-codeword
// state does not fit on chip (e.g. n = 64800), as block-level device functions.
//
// Layout: every per-node and per-edge quantity is stored as [node or edge][Bp]
// with the codeword index fastest (Bp = batch padded to 256).  Each lane holds four
// adjacent codewords as two packed int16 pairs, so a wavefront covers a group of
// 256 codewords of one node or edge: every access is one contiguous 256-byte
// segment at a wave-uniform index, issued as a buffer load or store whose scalar
// offset carries the index (no per-lane address arithmetic), and every wave keeps
// several kilobytes of loads in flight.
//
// Messages live on the edges as int8: the check-node phase reads the
// variable-to-check messages q of its edges (contiguous in CSR order) and writes
// the check-to-variable messages r; the variable-node phase gathers r of its
// edges, forms Lambda = L + sum r (exact in int16), writes q = sat(Lambda - r)
// back to every edge and the hard decisions as 64-bit lane masks (one per
// codeword position in the lane).  Per codeword and iteration this moves about
// 4E + n bytes.  Codewords that stopped (early termination) keep every message:
// a wave whose lanes are partly stopped merges old and new values per byte.
//
// All functions assume blocks of 256 threads (4 waves); the block index is passed
// explicitly, so a launch may map its blocks onto (node, group) in any order.
#pragma once

#include "dev_common.h"

namespace ldpcx {
namespace dev {
namespace il {

constexpr int kPairs = 2;                     // packed int16 pairs per lane
constexpr int kLaneCw = 2 * kPairs;           // codewords per lane
constexpr int kGroup = 64 * kLaneCw;          // codewords per wavefront
constexpr int kVnRegs = 8;                    // check messages a variable keeps in registers
constexpr int kVnPerWave = 2;                 // variables of one variable-node wave
constexpr uint32_t kRsrcWord3 = 0x00020000u;  // raw (untyped) buffer resource, gfx9 family

struct Args {
    DevCode C;
    BinRule R;
    int max_iters, early_stop, batch, Bp, G;  // G = Bp / kGroup groups
    BinIlWork w;
    uint8_t *bytes_t;  // [ceil(n/8)][Bp] staging of the packed decisions
    DecodeIO io;
};

typedef v2s Pk[kPairs];  // the lane's codewords: pair p holds codewords 2p (low half) and 2p + 1

__device__ __forceinline__ __amdgpu_buffer_rsrc_t rsrc(const void *p, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, (int)bytes, (int)kRsrcWord3);
}

// The lane's int8 codeword values (bytes 0..3 of x) -> packed int16 pairs, sign extended.
__device__ __forceinline__ void unpack(uint32_t x, Pk &p) {
    p[0] = as_v2s(__builtin_amdgcn_perm(x, x, 0x010C000Cu)) >> splat(8);
    p[1] = as_v2s(__builtin_amdgcn_perm(x, x, 0x030C020Cu)) >> splat(8);
}

// Packed int16 pairs (values in int8 range) -> the lane's four bytes.
__device__ __forceinline__ uint32_t pack(const Pk &p) {
    return __builtin_amdgcn_perm(as_u32(p[1]), as_u32(p[0]), 0x06040200u);
}

__device__ __forceinline__ uint32_t ld(__amdgpu_buffer_rsrc_t r, uint32_t vo, uint32_t so) {
    return __builtin_amdgcn_raw_buffer_load_b32(r, (int)vo, (int)so, 0);
}
__device__ __forceinline__ void st(uint32_t v, __amdgpu_buffer_rsrc_t r, uint32_t vo, uint32_t so) {
    __builtin_amdgcn_raw_buffer_store_b32(v, r, (int)vo, (int)so, 0);
}

__device__ __forceinline__ uint32_t lane_off() { return kLaneCw * (threadIdx.x & 63); }

// Activity of the lane's codewords at iteration k.  Codewords beyond the batch
// count as active (their inputs are zero and stay zero), so that a wave of a partly
// filled group is not treated as mixed.
struct Act {
    uint32_t m8;            // per byte: 0xFF where the codeword is active
    uint32_t m16[kPairs];   // per int16 half of each pair: 0xFFFF where active
    bool any, all;
};

// Word kLaneCw * g + h of a slot holds codeword kGroup * g + kLaneCw * l + h in bit l.
__device__ __forceinline__ Act activity(const Args &A, int k, int g, int lane) {
    Act a;
    a.m8 = 0xFFFFFFFFu;
    for (int p = 0; p < kPairs; ++p) a.m16[p] = 0xFFFFFFFFu;
    a.any = a.all = true;
    if (!A.early_stop) return a;
    const uint64_t *slot = A.w.unsat + ((size_t)k * A.G + g) * kLaneCw;
    const int b0 = g * kGroup + kLaneCw * lane;
    bool un = false, inact = false;
    a.m8 = 0;
#pragma unroll
    for (int h = 0; h < kLaneCw; ++h) {
        const bool u = (slot[h] >> lane) & 1ull;
        const bool act = u || b0 + h >= A.batch;
        un |= u;
        inact |= !act;
        if (act) a.m8 |= 0xFFu << (8 * h);
    }
#pragma unroll
    for (int p = 0; p < kPairs; ++p)
        a.m16[p] = ((a.m8 >> (16 * p)) & 0xFFu ? 0x0000FFFFu : 0u) | ((a.m8 >> (16 * p + 8)) & 0xFFu ? 0xFFFF0000u : 0u);
    a.any = __ballot(un) != 0;  // only real codewords can be unsatisfied
    a.all = __ballot(inact) == 0;
    return a;
}

// (M & a) | (~M & b)
__device__ __forceinline__ uint32_t merge(uint32_t M, uint32_t a, uint32_t b) { return (M & a) | (~M & b); }

// Sign bit of codeword h of the lane (from the packed sums).
__device__ __forceinline__ bool neg_of(const Pk &S, int h) { return (as_u32(S[h >> 1]) >> (h & 1 ? 31 : 15)) & 1u; }

// Virtual grids (blocks of 256 threads, 4 waves) of the phases.
__host__ __device__ inline long grid_rows_x(const Args &A) { return (A.C.m + 3) / 4; }
__host__ __device__ inline long grid_vars_x(const Args &A) { return (A.C.n + 3) / 4; }
__host__ __device__ inline long grid_vn_x(const Args &A) { return (A.C.n + 4 * kVnPerWave - 1) / (4 * kVnPerWave); }
__host__ __device__ inline long grid_edges_x(const Args &A) { return (A.C.E + 3) / 4; }
__host__ __device__ inline long grid_syn(const Args &A) {
    return ((long)((A.C.m + 31) / 32) * kLaneCw * A.G + 255) / 256;
}
__host__ __device__ inline long grid_bytes(const Args &A) { return ((long)((A.C.n + 7) / 8) * A.Bp + 255) / 256; }
__host__ __device__ inline long grid_fin(const Args &A) { return (A.batch + 255) / 256; }

// q = sat(L) of the edge's variable, r = 0 (wave per (edge, group)).
__device__ __forceinline__ void init_edges_block(const Args &A, int bx, int g) {
    const int e = bx * 4 + wave_id();
    if (e >= A.C.E) return;
    const uint32_t vo = lane_off(), gb = (uint32_t)g * kGroup, Bp = (uint32_t)A.Bp;
    const auto rL = rsrc(A.w.L, (uint32_t)A.C.n * Bp);
    const auto rq = rsrc(A.w.q, (uint32_t)A.C.E * Bp);
    const auto rr = rsrc(A.w.r, (uint32_t)A.C.E * Bp);
    const uint32_t v = (uint32_t)A.C.col_idx[e];
    Pk L;
    unpack(ld(rL, vo, v * Bp + gb), L);
#pragma unroll
    for (int p = 0; p < kPairs; ++p) L[p] = pmin(pmax(L[p], splat(-A.R.msg_max)), splat(A.R.msg_max));
    st(pack(L), rq, vo, (uint32_t)e * Bp + gb);
    st(0u, rr, vo, (uint32_t)e * Bp + gb);
}

// Decision words of one variable: lane h (< kLaneCw) stores word h.
__device__ __forceinline__ void store_hb(const Args &A, int v, int g, const Pk &S, const Act *act) {
    const int lane = threadIdx.x & 63;
    uint64_t *hb = A.w.hb + ((size_t)v * A.G + g) * kLaneCw;
    uint64_t mine = 0;
#pragma unroll
    for (int h = 0; h < kLaneCw; ++h) {
        uint64_t b = __ballot(neg_of(S, h));
        if (act && !act->all) {
            const uint64_t keep = __ballot((act->m8 >> (8 * h)) & 1u);
            b = (b & keep) | (hb[h] & ~keep);
        }
        if (lane == h) mine = b;
    }
    if (lane < kLaneCw) hb[lane] = mine;
}

// Decisions of iteration 0 (wave per (variable, group)).
__device__ __forceinline__ void init_vars_block(const Args &A, int bx, int g) {
    const int v = bx * 4 + wave_id();
    if (v >= A.C.n) return;
    const uint32_t vo = lane_off(), gb = (uint32_t)g * kGroup, Bp = (uint32_t)A.Bp;
    const auto rL = rsrc(A.w.L, (uint32_t)A.C.n * Bp);
    Pk L;
    unpack(ld(rL, vo, (uint32_t)v * Bp + gb), L);
    store_hb(A, v, g, L, nullptr);
}

// Syndrome test: for every (decision word, block of 32 checks) the OR of the parity
// masks, accumulated into the unsatisfied-codeword mask of slot_k.
__device__ __forceinline__ void syn_block(const Args &A, int slot_k, long bx) {
    const DevCode &C = A.C;
    const int W = kLaneCw * A.G;
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

// Check-node phase of iteration k: one wave per (check, group).  DC bounds the check
// degree.  Outgoing magnitude: f(min2) on the edge holding the minimum, f(min1)
// elsewhere (equal when the minimum is tied); sign: product of the other signs.
template <int DC>
__device__ __forceinline__ void cn_block(const Args &A, int k, int bx, int g) {
    const DevCode &C = A.C;
    const int lane = threadIdx.x & 63;
    const int row = bx * 4 + wave_id();
    if (row >= C.m) return;
    const Act act = activity(A, k, g, lane);
    if (!act.any) return;
    const uint32_t vo = lane_off(), gb = (uint32_t)g * kGroup, Bp = (uint32_t)A.Bp;
    const auto rq = rsrc(A.w.q, (uint32_t)C.E * Bp);
    const auto rr = rsrc(A.w.r, (uint32_t)C.E * Bp);
    const int e0 = C.row_ptr[row];
    const int dc = C.row_ptr[row + 1] - e0;
    const PkNorm NP = pk_norm_params(A.R);
    uint32_t raw[DC];
#pragma unroll
    for (int j = 0; j < DC; ++j)
        if (j < dc) raw[j] = ld(rq, vo, (uint32_t)(e0 + j) * Bp + gb);
    Pk m1, m2, f1, cs;
    Pk av[DC];
    uint32_t sv[DC][kPairs], stot[kPairs];
#pragma unroll
    for (int p = 0; p < kPairs; ++p) {
        m1[p] = m2[p] = splat(0x7FFF);
        stot[p] = 0;
    }
#pragma unroll
    for (int j = 0; j < DC; ++j) {
        if (j < dc) {
            Pk q;
            unpack(raw[j], q);
#pragma unroll
            for (int p = 0; p < kPairs; ++p) {
                const v2s a = pmax(q[p], -q[p]);
                m2[p] = pmin(m2[p], pmax(m1[p], a));
                m1[p] = pmin(m1[p], a);
                sv[j][p] = as_u32(q[p] >> splat(15));
                stot[p] ^= sv[j][p];
                av[j][p] = a;
            }
        }
    }
    // Magnitude out of edge j: f(min2) where the edge holds the minimum (a = min1), else
    // f(min1).  With magnitudes in [0, 127] and f(min2) - f(min1) <= min2 - min1 <= 127
    // (normalisation factor at most 1) that is max(f(min1), f(min2) + 128 (min1 - a)),
    // exact in int16: one multiply-add and one maximum per pair.  -128 is opaque to the
    // compiler so that the product stays one v_pk_mad_u16.
    int kn128 = (int)0xFF80FF80u;
    asm volatile("" : "+s"(kn128));
    const v2s neg128 = as_v2s((uint32_t)kn128);
#pragma unroll
    for (int p = 0; p < kPairs; ++p) {
        f1[p] = pk_norm(NP, m1[p]);
        cs[p] = pk_norm(NP, m2[p]) - m1[p] * neg128;
    }
#pragma unroll
    for (int j = 0; j < DC; ++j) {
        if (j < dc) {
            Pk rn;
#pragma unroll
            for (int p = 0; p < kPairs; ++p) {
                const v2s mag = pmax(f1[p], av[j][p] * neg128 + cs[p]);
                const uint32_t sr = stot[p] ^ sv[j][p];
                rn[p] = as_v2s(as_u32(mag) ^ sr) - as_v2s(sr);
            }
            uint32_t w = pack(rn);
            const uint32_t so = (uint32_t)(e0 + j) * Bp + gb;
            if (!act.all) w = merge(act.m8, w, ld(rr, vo, so));
            st(w, rr, vo, so);
        }
    }
}

// Variable-node phase of iteration k: one wave per (kVnPerWave consecutive variables,
// group).  The wave issues the loads of all its variables before it sums any of them:
// a wave's life is mostly index and message latency, so two variables per wave keep
// more bytes in flight (three measured slower).  The unpacked messages of the first
// kVnRegs edges stay in registers for the outgoing messages.
__device__ __forceinline__ void vn_block(const Args &A, int k, int bx, int g) {
    constexpr int NV = kVnPerWave;
    const DevCode &C = A.C;
    const int lane = threadIdx.x & 63;
    const int v0 = (bx * 4 + wave_id()) * NV;
    if (v0 >= C.n) return;
    const Act act = activity(A, k, g, lane);
    if (!act.any) return;
    const uint32_t vo = lane_off(), gb = (uint32_t)g * kGroup, Bp = (uint32_t)A.Bp;
    const auto rL = rsrc(A.w.L, (uint32_t)C.n * Bp);
    const auto rq = rsrc(A.w.q, (uint32_t)C.E * Bp);
    const auto rr = rsrc(A.w.r, (uint32_t)C.E * Bp);
    int t0[NV], dv[NV];
    uint32_t lw[NV], rw[NV][kVnRegs], ev[NV][kVnRegs];
#pragma unroll
    for (int i = 0; i < NV; ++i) {
        const bool ok = v0 + i < C.n;
        t0[i] = ok ? C.vn_ptr[v0 + i] : 0;
        dv[i] = ok ? C.vn_ptr[v0 + i + 1] - t0[i] : 0;
    }
#pragma unroll
    for (int i = 0; i < NV; ++i) {
        if (v0 + i < C.n) lw[i] = ld(rL, vo, (uint32_t)(v0 + i) * Bp + gb);
#pragma unroll
        for (int t = 0; t < kVnRegs; ++t) {
            if (t < dv[i]) {
                ev[i][t] = (uint32_t)C.vn_edge[t0[i] + t] * Bp + gb;
                rw[i][t] = ld(rr, vo, ev[i][t]);
            }
        }
    }
    const v2s mm = splat(A.R.msg_max), nmm = splat(-A.R.msg_max);
#pragma unroll
    for (int i = 0; i < NV; ++i) {
        if (v0 + i >= C.n) break;
        Pk S, ru[kVnRegs];
        unpack(lw[i], S);
#pragma unroll
        for (int t = 0; t < kVnRegs; ++t) {
            if (t < dv[i]) {
                unpack(rw[i][t], ru[t]);
#pragma unroll
                for (int p = 0; p < kPairs; ++p) S[p] = S[p] + ru[t][p];
            }
        }
        for (int t = kVnRegs; t < dv[i]; ++t) {
            Pk r;
            unpack(ld(rr, vo, (uint32_t)C.vn_edge[t0[i] + t] * Bp + gb), r);
#pragma unroll
            for (int p = 0; p < kPairs; ++p) S[p] = S[p] + r[p];
        }
        auto qword = [&](const Pk &r, uint32_t so) {
            Pk q;
#pragma unroll
            for (int p = 0; p < kPairs; ++p) q[p] = pmin(pmax(S[p] - r[p], nmm), mm);
            uint32_t w = pack(q);
            if (!act.all) w = merge(act.m8, w, ld(rq, vo, so));
            st(w, rq, vo, so);
        };
#pragma unroll
        for (int t = 0; t < kVnRegs; ++t)
            if (t < dv[i]) qword(ru[t], ev[i][t]);
        for (int t = kVnRegs; t < dv[i]; ++t) {
            const uint32_t so = (uint32_t)C.vn_edge[t0[i] + t] * Bp + gb;
            Pk r;
            unpack(ld(rr, vo, so), r);
            qword(r, so);
        }
        store_hb(A, v0 + i, g, S, &act);
    }
    if (v0 == 0) {
        uint32_t *itp = (uint32_t *)(A.w.it + (size_t)g * kGroup) + kPairs * lane;
        const uint32_t kk = (uint32_t)k | ((uint32_t)k << 16);
#pragma unroll
        for (int p = 0; p < kPairs; ++p) itp[p] = act.all ? kk : merge(act.m16[p], kk, itp[p]);
    }
}

// Decision bit of codeword b for variable v.
__device__ __forceinline__ uint32_t hbit(const Args &A, int v, int b) {
    const int g = b / kGroup, rem = b - g * kGroup;
    return (uint32_t)((A.w.hb[((size_t)v * A.G + g) * kLaneCw + (rem % kLaneCw)] >> (rem / kLaneCw)) & 1ull);
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

// Unsatisfied bit of codeword b in slot k.
__device__ __forceinline__ bool unsat_bit(const Args &A, int k, int b) {
    const int g = b / kGroup, rem = b - g * kGroup;
    return (A.w.unsat[((size_t)k * A.G + g) * kLaneCw + (rem % kLaneCw)] >> (rem / kLaneCw)) & 1ull;
}

// Syndrome flags (final test in slot 0) and iteration counts.
__device__ __forceinline__ void fin_block(const Args &A, long bx) {
    const int b = (int)(bx * 256 + threadIdx.x);
    if (b >= A.batch) return;
    A.io.ok[b] = unsat_bit(A, 0, b) ? 0 : 1;
    A.io.iters[b] = A.w.it[b];
}

// Lambda = L + sum r per variable in the interleaved layout, for the debug dump.
__device__ __forceinline__ void lambda_block(const Args &A, int16_t *lam_t, int bx, int g) {
    const DevCode &C = A.C;
    const int v = bx * 4 + wave_id();
    if (v >= C.n) return;
    const uint32_t vo = lane_off(), gb = (uint32_t)g * kGroup, Bp = (uint32_t)A.Bp;
    const auto rL = rsrc(A.w.L, (uint32_t)C.n * Bp);
    const auto rr = rsrc(A.w.r, (uint32_t)C.E * Bp);
    Pk S;
    unpack(ld(rL, vo, (uint32_t)v * Bp + gb), S);
    for (int t = C.vn_ptr[v]; t < C.vn_ptr[v + 1]; ++t) {
        Pk r;
        unpack(ld(rr, vo, (uint32_t)C.vn_edge[t] * Bp + gb), r);
#pragma unroll
        for (int p = 0; p < kPairs; ++p) S[p] = S[p] + r[p];
    }
    uint32_t *out = (uint32_t *)(lam_t + (size_t)v * A.Bp + gb + vo);
#pragma unroll
    for (int p = 0; p < kPairs; ++p) out[p] = as_u32(S[p]);
}

__host__ __device__ inline int pad_group(int b) { return (b + kGroup - 1) / kGroup * kGroup; }

struct Carve {
    size_t L, q, r, hb, unsat, it, bytes, total;
};

inline Carve carve(const DevCode &C, int max_iters, int batch) {
    const size_t Bp = pad_group(batch), W = Bp / 64;
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
    A.Bp = pad_group(batch);
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
    return FillArgs{(uint32_t *)A.w.unsat, (size_t)(A.max_iters + 1) * kLaneCw * A.G * 2, 0u};
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
