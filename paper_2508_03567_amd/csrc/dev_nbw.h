// Min-Max decoder (Alg. 2) for large fields, g = 128 or 256, as wave-level device
// functions.
//
// Mapping: one wavefront per (node, codeword); its lanes cover the g entries of the
// messages, two adjacent entries per packed int16 pair (g / 128 pairs per lane).
// Messages are stored codeword-major per edge, [edge][codeword][x], so every vector a
// wave touches is one contiguous 2g-byte row; the channel vectors gamma are read in
// place from the caller's [codeword][node][x] input.
//
// Check node: the permuted input vectors a~_j(t) = alpha_j(h_j^-1 t) are staged in
// LDS (the permutation is folded into the loads).  The forward and backward
// recursions of eqs. (7)-(10) and the middle outputs of eq. (13) are XOR
// (min,max)-convolutions R(s) = min_t max(X(s ^ t), Y(t)) computed with the lanes
// over the outputs s: lane pair q holds s = 2q, 2q + 1, and for the two inputs
// t = 2u, 2u + 1 it reads the single LDS pair X[q ^ u] (halves swapped for the odd
// t) and the broadcast pair Y[u], so each step costs one LDS read and four packed
// max/min instructions for four (max, min) evaluations.  As in the small-field
// kernel, F at the last edge and B at the first edge are not computed:
// 3 (dc - 2) convolutions per check.  The outputs beta_j(x) = beta~_j(h_j x) are
// written back through the same kind of indexed LDS read.
//
// Variable node: lanes over x accumulate the APP sums (int32), the decision is a
// wave-wide minimum of (APP << 9 | x), i.e. the lowest x on ties, and every outgoing
// alpha is normalised by its own wave-wide minimum (eqs. (14)-(15)).
#pragma once

#include "dev_common.h"

namespace ldpcx {
namespace dev {
namespace nbw {

struct Args {
    DevCode C;
    int max_iters, early_stop, batch;
    int amax;  // message bound: alpha and the channel vectors are clipped to it
    NbwWork w;
    DecodeIO io;
};

// Make LDS writes of this wave visible to its other lanes before they read them.
__device__ __forceinline__ void lds_sync_wave() { asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory"); }

__device__ __forceinline__ int wave_min(int v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o, 64));
    return v;
}

// R = X (*) Y over GF(G) with X, Y, R packed-pair vectors of G/2 words in LDS.
template <int G>
__device__ __forceinline__ void conv(const uint32_t *X, const uint32_t *Y, uint32_t *R, int lane) {
    constexpr int P = G / 128;
    v2s r[P];
#pragma unroll
    for (int p = 0; p < P; ++p) r[p] = splat(0x7FFF);
#pragma unroll 4
    for (int u = 0; u < G / 2; ++u) {
        const v2s y = as_v2s(Y[u]);
#pragma unroll
        for (int p = 0; p < P; ++p) {
            const v2s a = as_v2s(X[(lane + 64 * p) ^ u]);
            r[p] = pmin(r[p], pmax(a, y.xx));
            r[p] = pmin(r[p], pmax(a.yx, y.yy));
        }
    }
#pragma unroll
    for (int p = 0; p < P; ++p) R[lane + 64 * p] = as_u32(r[p]);
    lds_sync_wave();
}

// LDS words per wave of the check-node phase for checks of degree <= dc_max:
// permuted inputs (dc), forward vectors (dc - 2), two backward vectors and one output.
inline size_t cn_words_per_wave(int g, int dc_max) { return (size_t)(2 * dc_max + 1) * (g / 2); }

__host__ __device__ inline size_t row_off(int e, int b, int batch, int g) { return ((size_t)e * batch + b) * g; }

__device__ __forceinline__ bool active(const Args &A, int k, int b) {
    return b < A.batch && (!A.early_stop || A.w.unsat[(size_t)k * A.batch + b]);
}

// Check-node phase of iteration k: wave `unit` = (check, codeword).
template <int G>
__device__ __forceinline__ void cn_unit(const Args &A, int k, long unit, uint32_t *lds) {
    constexpr int H = G / 2;
    const DevCode &C = A.C;
    const int row = (int)(unit / A.batch), b = (int)(unit - (long)row * A.batch);
    if (row >= C.m || !active(A, k, b)) return;
    const int lane = threadIdx.x & 63;
    const int e0 = C.row_ptr[row];
    const int dc = C.row_ptr[row + 1] - e0;
    uint32_t *ain = lds;                      // [dc][H] permuted inputs
    uint32_t *fwd = ain + (size_t)dc * H;     // [dc - 2][H] forward vectors F_1..F_{dc-2}
    uint32_t *bk0 = fwd + (size_t)(dc > 2 ? dc - 2 : 0) * H;
    uint32_t *bk1 = bk0 + H;
    uint32_t *out = bk1 + H;
    const uint8_t *mul = C.gfmul;
    // a~_j(t) = alpha_j(hinv_j t) for t = 2q, 2q + 1
    for (int j = 0; j < dc; ++j) {
        const int e = e0 + j;
        const int16_t *src = A.w.alpha + row_off(e, b, A.batch, G);
        const uint8_t *mrow = mul + (size_t)C.hinv[e] * G;
#pragma unroll
        for (int p = 0; p < G / 128; ++p) {
            const int q = lane + 64 * p;
            const v2s v = (v2s){src[mrow[2 * q]], src[mrow[2 * q + 1]]};
            ain[(size_t)j * H + q] = as_u32(v);
        }
    }
    lds_sync_wave();
    // beta_j(x) = beta~_j(h_j x), written to the edge's row
    auto store = [&](int j, const uint32_t *bt) {
        const int e = e0 + j;
        const uint8_t *mrow = mul + (size_t)C.h[e] * G;
        const int16_t *bt16 = (const int16_t *)bt;
        uint32_t *dst = (uint32_t *)(A.w.beta + row_off(e, b, A.batch, G));
#pragma unroll
        for (int p = 0; p < G / 128; ++p) {
            const int q = lane + 64 * p;
            dst[q] = as_u32((v2s){bt16[mrow[2 * q]], bt16[mrow[2 * q + 1]]});
        }
    };
    // forward: F_j = F_{j-1} (*) a~_j, F_0 = a~_0
    for (int j = 1; j <= dc - 2; ++j) {
        const uint32_t *prev = j == 1 ? ain : fwd + (size_t)(j - 2) * H;
        conv<G>(prev, ain + (size_t)j * H, fwd + (size_t)(j - 1) * H, lane);
    }
    store(dc - 1, dc >= 3 ? fwd + (size_t)(dc - 3) * H : ain);  // eq. (12): F_{dc-2}
    // backward with the middle outputs: beta~_j = F_{j-1} (*) B_{j+1}, B_j = B_{j+1} (*) a~_j
    const uint32_t *bcur = ain + (size_t)(dc - 1) * H;
    for (int j = dc - 2; j >= 1; --j) {
        const uint32_t *fprev = j == 1 ? ain : fwd + (size_t)(j - 2) * H;
        conv<G>(fprev, bcur, out, lane);
        store(j, out);
        uint32_t *bnext = (bcur == bk0) ? bk1 : bk0;
        conv<G>(bcur, ain + (size_t)j * H, bnext, lane);
        bcur = bnext;
    }
    store(0, bcur);  // eq. (11): B_1
}

// Variable-node update (eqs. (14)-(15)) and decision: wave `unit` = (variable, codeword).
template <int G>
__device__ __forceinline__ void vn_unit(const Args &A, int k, long unit) {
    constexpr int NE = G / 64;  // entries per lane: x = lane + 64 i
    const DevCode &C = A.C;
    const int v = (int)(unit / A.batch), b = (int)(unit - (long)v * A.batch);
    if (v >= C.n || !active(A, k, b)) return;
    const int lane = threadIdx.x & 63;
    const int16_t *gam = (const int16_t *)A.io.llr + ((size_t)b * C.n + v) * G;
    int S[NE];
#pragma unroll
    for (int i = 0; i < NE; ++i) S[i] = min((int)gam[lane + 64 * i], A.amax);
    const int t0 = C.vn_ptr[v], t1 = C.vn_ptr[v + 1];
    for (int t = t0; t < t1; ++t) {
        const int16_t *bp = A.w.beta + row_off(C.vn_ref[t], b, A.batch, G);
#pragma unroll
        for (int i = 0; i < NE; ++i) S[i] += bp[lane + 64 * i];
    }
    int key = 0x7FFFFFFF;
#pragma unroll
    for (int i = 0; i < NE; ++i) key = min(key, (S[i] << 9) | (lane + 64 * i));
    key = wave_min(key);
    if (lane == 0) {
        ((uint8_t *)A.io.hard)[(size_t)b * C.n + v] = (uint8_t)(key & 0x1FF);
        if (v == 0) A.w.it[b] = (int16_t)k;
    }
    for (int t = t0; t < t1; ++t) {
        const int e = C.vn_ref[t];
        const int16_t *bp = A.w.beta + row_off(e, b, A.batch, G);
        int a[NE];
        int mn = 0x7FFFFFFF;
#pragma unroll
        for (int i = 0; i < NE; ++i) {
            a[i] = S[i] - bp[lane + 64 * i];
            mn = min(mn, a[i]);
        }
        mn = wave_min(mn);
        int16_t *ap = A.w.alpha + row_off(e, b, A.batch, G);
#pragma unroll
        for (int i = 0; i < NE; ++i) ap[lane + 64 * i] = (int16_t)min(a[i] - mn, A.amax);
    }
}

// alpha^(0) = gamma of the edge's variable, beta = 0: wave `unit` = (edge, codeword).
template <int G>
__device__ __forceinline__ void init_edge_unit(const Args &A, long unit) {
    const DevCode &C = A.C;
    const int e = (int)(unit / A.batch), b = (int)(unit - (long)e * A.batch);
    if (e >= C.E) return;
    const int lane = threadIdx.x & 63;
    const uint32_t *gam = (const uint32_t *)((const int16_t *)A.io.llr + ((size_t)b * C.n + C.col_idx[e]) * G);
    uint32_t *ap = (uint32_t *)(A.w.alpha + row_off(e, b, A.batch, G));
    uint32_t *bp = (uint32_t *)(A.w.beta + row_off(e, b, A.batch, G));
#pragma unroll
    for (int p = 0; p < G / 128; ++p) {
        ap[lane + 64 * p] = as_u32(pmin(as_v2s(gam[lane + 64 * p]), splat(A.amax)));
        bp[lane + 64 * p] = 0u;
    }
}

// Decision of iteration 0 (most likely channel symbol, lowest x on ties): wave
// `unit` = (variable, codeword).
template <int G>
__device__ __forceinline__ void init_var_unit(const Args &A, long unit) {
    constexpr int NE = G / 64;
    const DevCode &C = A.C;
    const int v = (int)(unit / A.batch), b = (int)(unit - (long)v * A.batch);
    if (v >= C.n) return;
    const int lane = threadIdx.x & 63;
    const int16_t *gam = (const int16_t *)A.io.llr + ((size_t)b * C.n + v) * G;
    int key = 0x7FFFFFFF;
#pragma unroll
    for (int i = 0; i < NE; ++i) key = min(key, (min((int)gam[lane + 64 * i], A.amax) << 9) | (lane + 64 * i));
    key = wave_min(key);
    if (lane == 0) ((uint8_t *)A.io.hard)[(size_t)b * C.n + v] = (uint8_t)(key & 0x1FF);
}

// Syndrome test: thread per (check, codeword); marks the codeword unsatisfied in slot_k.
__device__ __forceinline__ void syn_thread(const Args &A, int slot_k, long t) {
    const DevCode &C = A.C;
    const int row = (int)(t / A.batch), b = (int)(t - (long)row * A.batch);
    if (row >= C.m) return;
    const uint8_t *hard = (const uint8_t *)A.io.hard + (size_t)b * C.n;
    int s = 0;
    for (int e = C.row_ptr[row]; e < C.row_ptr[row + 1]; ++e) s ^= C.gfmul[C.h[e] * C.g + hard[C.col_idx[e]]];
    if (s) A.w.unsat[(size_t)slot_k * A.batch + b] = 1;
}

__device__ __forceinline__ void fin_thread(const Args &A, long t) {
    if (t >= A.batch) return;
    A.io.ok[t] = A.w.unsat[t] ? 0 : 1;
    A.io.iters[t] = A.w.it[t];
}

// Row copy [E][batch][G] -> [batch][E][G] for the debug dump: wave `unit` = (edge, codeword).
template <int G>
__device__ __forceinline__ void dump_unit(const Args &A, const int16_t *src, int16_t *dst, long unit) {
    const int e = (int)(unit / A.batch), b = (int)(unit - (long)e * A.batch);
    if (e >= A.C.E) return;
    const int lane = threadIdx.x & 63;
    const uint32_t *s = (const uint32_t *)(src + row_off(e, b, A.batch, G));
    uint32_t *d = (uint32_t *)(dst + ((size_t)b * A.C.E + e) * G);
#pragma unroll
    for (int p = 0; p < G / 128; ++p) d[lane + 64 * p] = s[lane + 64 * p];
}

struct Carve {
    size_t alpha, beta, unsat, it, total;
};

inline Carve carve(const DevCode &C, int max_iters, int batch) {
    Carve c;
    size_t o = 0;
    c.alpha = o;
    o = align_up(o + (size_t)C.E * batch * C.g * 2, 256);
    c.beta = o;
    o = align_up(o + (size_t)C.E * batch * C.g * 2, 256);
    c.unsat = o;
    o = align_up(o + (size_t)(max_iters + 1) * batch, 256);
    c.it = o;
    o = align_up(o + (size_t)batch * 2, 256);
    c.total = o;
    return c;
}

inline Args make_args(const DevCode &C, int max_iters, int early_stop, int batch, int amax, void *base,
                      const DecodeIO &io) {
    Args A;
    A.C = C;
    A.amax = amax;
    A.max_iters = max_iters;
    A.early_stop = early_stop;
    A.batch = batch;
    const Carve c = carve(C, max_iters, batch);
    char *p = (char *)base;
    A.w.alpha = (int16_t *)(p + c.alpha);
    A.w.beta = (int16_t *)(p + c.beta);
    A.w.unsat = (uint8_t *)(p + c.unsat);
    A.w.it = (int16_t *)(p + c.it);
    A.io = io;
    return A;
}

}  // namespace nbw
}  // namespace dev
}  // namespace ldpcx
