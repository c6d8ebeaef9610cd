// Min-Max (Alg. 2) with one codeword per workgroup and every message in LDS, lanes
// over the field entries.
//
// The workgroup holds the clipped channel vectors gamma', the alpha and beta messages
// of every edge ([node or edge][x] int16), the multiplication table, the edge
// coefficients and the decisions of its codeword in LDS, and runs every iteration of
// that codeword alone: no device-memory traffic but the input and the outputs, and no
// other workgroup involved, which is what lets one codeword be an item of the
// persistent ragged kernel.  It fits codes whose messages of one codeword fit 160 KB
// (the (2,4)-regular GF(64) code of 192 symbols takes 128 KB).
//
// Message storage: signed 16-bit (exact for every value the arithmetic stores, costs
// below 0 included), or 8-bit when the message bound is at most 255 (the 8-bit variant
// of sec. 5, bound 127): with costs >= 0 every stored alpha, beta and gamma' then lies
// in [0, bound], so bytes hold them exactly, the arithmetic stays 16/32-bit and the
// results are those of the 16-bit storage; the LDS per codeword halves (66 KB for the
// GF(64) code, so two codewords share a compute unit).
//
// Mapping: a message vector of G entries lives on a segment of S = G / R lanes, lane j
// of the segment holding the R consecutive entries R j .. R j + R - 1 as R / 2 packed
// int16 pairs (R = 8, or G below 8); a wave holds 64 / S vectors, one per check or
// variable it works on.  The (min, max) XOR-convolution behind eqs. (9), (10) and (13),
//   (X (*) Y)(s) = min_t max(X(s ^ t), Y(t)),
// splits t = R t_hi + t_lo: for each t_hi the lane fetches the block of lane j ^ t_hi
// (X) and of lane t_hi (Y) of its segment with ds_swizzle, and the t_lo part is a
// butterfly over its registers (entry i ^ t_lo, halves swapped for odd t_lo), so every
// (max, min) pair costs one packed max and one packed min as in the interleaved kernel.
// The permutation by the edge coefficient (eqs. (7)-(8), (11)-(12)) is folded into the
// LDS gathers and scatters of each edge's row: entry t of the permuted vector is entry
// h^-1 t of the stored one.
//
// Codes whose variables all have degree 2 (the (2, dc)-regular codes of the GF(q)
// workloads) can run without stored alphas ("alpha-free"): the alpha of edge e is then
// gamma' plus the beta of its variable's other edge e', shifted to minimum 0 and
// clipped (eqs. (14)-(15)), so the check node forms it from gamma' and beta at the
// permuted positions it would have read.  The LDS per codeword drops by one message
// array (GF(64), n = 192, 16-bit: 78 KB instead of 125 KB, two codewords per compute
// unit).  Flooding keeps every check's inputs of iteration k in registers across a
// barrier before any beta of iteration k is written (each segment holds at most two
// checks); the layers of the layered schedule share no variable, so a check there
// reads only betas that no other check of its layer writes.  The results are those of
// the stored-alpha decoder, message for message.
#pragma once

#include "dev_common.h"

namespace ldpcx {
namespace dev {
namespace nb1 {

struct Job {
    DevCode C;
    int max_iters, early_stop, layered, amax, batch;
    DecodeIO io;
};

// Bytes of one stored message entry for a message bound.
__host__ __device__ inline int msg_bytes(int amax) { return amax <= 255 ? 1 : 2; }

template <int G>
struct Geo {
    static constexpr int R = G >= 8 ? 8 : G;  // entries per lane
    static constexpr int S = G / R;           // lanes per vector
    static constexpr int H = R / 2;           // packed pairs per lane
    static constexpr int VPW = 64 / S;        // vectors per wave
};

struct Layout {
    size_t gam, alpha, beta, mul, hinv, h, hard, flags, vt, total;
};

// af: alpha-free (no alpha array; a [E] table of (variable, other edge) instead).
__host__ __device__ inline Layout layout(const DevCode &C, int mb, bool af = false) {
    const size_t G = (size_t)C.g;
    Layout L;
    size_t o = 0;
    L.gam = o;
    o = align_up(o + mb * (size_t)C.n * G, 16);
    L.alpha = o;
    if (!af) o = align_up(o + mb * (size_t)C.E * G, 16);
    L.beta = o;
    o = align_up(o + mb * (size_t)C.E * G, 16);
    L.mul = o;
    o = align_up(o + G * G, 16);
    L.hinv = o;
    o = align_up(o + (size_t)C.E, 16);
    L.h = o;
    o = align_up(o + (size_t)C.E, 16);
    L.hard = o;
    o = align_up(o + (size_t)C.n, 16);
    L.flags = o;
    o += 16;
    L.vt = o;
    if (af) o = align_up(o + 4 * (size_t)C.E, 16);
    L.total = o;
    return L;
}

// ds_swizzle within groups of lanes (constant patterns; th is a literal after unrolling):
// the value of lane (lane ^ th), and the value of lane th of the lane's group of S.
__device__ __forceinline__ int swz_xor(int v, int th) {
    switch (th) {
    case 1: return __builtin_amdgcn_ds_swizzle(v, 0x041F);
    case 2: return __builtin_amdgcn_ds_swizzle(v, 0x081F);
    case 3: return __builtin_amdgcn_ds_swizzle(v, 0x0C1F);
    case 4: return __builtin_amdgcn_ds_swizzle(v, 0x101F);
    case 5: return __builtin_amdgcn_ds_swizzle(v, 0x141F);
    case 6: return __builtin_amdgcn_ds_swizzle(v, 0x181F);
    case 7: return __builtin_amdgcn_ds_swizzle(v, 0x1C1F);
    default: return v;
    }
}

template <int S>
__device__ __forceinline__ int swz_bcast(int v, int th) {
    constexpr int A = 0x1F & ~(S - 1);
    if (S == 1) return v;
    switch (th) {
    case 0: return __builtin_amdgcn_ds_swizzle(v, A);
    case 1: return __builtin_amdgcn_ds_swizzle(v, A | (1 << 5));
    case 2: return __builtin_amdgcn_ds_swizzle(v, A | (2 << 5));
    case 3: return __builtin_amdgcn_ds_swizzle(v, A | (3 << 5));
    case 4: return __builtin_amdgcn_ds_swizzle(v, A | (4 << 5));
    case 5: return __builtin_amdgcn_ds_swizzle(v, A | (5 << 5));
    case 6: return __builtin_amdgcn_ds_swizzle(v, A | (6 << 5));
    default: return __builtin_amdgcn_ds_swizzle(v, A | (7 << 5));
    }
}

// O = X (*) Y over the lanes of the segment.
template <int G>
__device__ __forceinline__ void conv(const v2s (&X)[Geo<G>::H], const v2s (&Y)[Geo<G>::H], v2s (&O)[Geo<G>::H]) {
    constexpr int R = Geo<G>::R, S = Geo<G>::S, H = Geo<G>::H;
#pragma unroll
    for (int th = 0; th < S; ++th) {
        v2s xb[H], yb[H];
#pragma unroll
        for (int p = 0; p < H; ++p) {
            xb[p] = th == 0 ? X[p] : as_v2s((uint32_t)swz_xor((int)as_u32(X[p]), th));
            yb[p] = as_v2s((uint32_t)swz_bcast<S>((int)as_u32(Y[p]), th));
        }
#pragma unroll
        for (int tl = 0; tl < R; ++tl) {
            const v2s bt = (tl & 1) ? yb[tl >> 1].yy : yb[tl >> 1].xx;
#pragma unroll
            for (int p = 0; p < H; ++p) {
                v2s a = xb[p ^ (tl >> 1)];
                if (tl & 1) a = a.yx;
                const v2s v = pmax(a, bt);
                O[p] = (th == 0 && tl == 0) ? v : pmin(O[p], v);
            }
        }
    }
}

// Minimum over the segment (every lane of it receives it).
template <int S>
__device__ __forceinline__ int seg_min(int v) {
#pragma unroll
    for (int o = 1; o < S; o <<= 1) v = min(v, swz_xor(v, o));
    return v;
}

// Entries t = R j .. R j + R - 1 of edge e's message permuted by its coefficient,
// m~(t) = m(h^-1 t): the multiplication-table row of h^-1 gives the positions.
template <int G>
__device__ __forceinline__ void perm_pos(const uint8_t *mul, int hinv, int j, uint8_t (&pos)[Geo<G>::R]) {
    constexpr int R = Geo<G>::R;
    const uint8_t *row = mul + hinv * G + R * j;
    if (R == 8) {
        const uint2 w = *(const uint2 *)row;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            pos[i] = (uint8_t)(w.x >> (8 * i));
            pos[i + 4] = (uint8_t)(w.y >> (8 * i));
        }
    } else {
        const uint32_t w = *(const uint32_t *)row;
#pragma unroll
        for (int i = 0; i < R; ++i) pos[i] = (uint8_t)(w >> (8 * i));
    }
}

template <int G, class M>
__device__ __forceinline__ void load_perm(const M *msg, const uint8_t *mul, int hinv, int e, int j,
                                          v2s (&out)[Geo<G>::H]) {
    constexpr int R = Geo<G>::R, H = Geo<G>::H;
    uint8_t pos[R];
    perm_pos<G>(mul, hinv, j, pos);
    const M *m = msg + (size_t)e * G;
#pragma unroll
    for (int p = 0; p < H; ++p) out[p] = (v2s){(short)m[pos[2 * p]], (short)m[pos[2 * p + 1]]};
}

// Write back a permuted vector at the same positions (m(h^-1 t) = m~(t)).
template <int G, class M>
__device__ __forceinline__ void store_deperm(M *msg, const uint8_t *mul, int hinv, int e, int j,
                                             const v2s (&v)[Geo<G>::H]) {
    constexpr int R = Geo<G>::R, H = Geo<G>::H;
    uint8_t pos[R];
    perm_pos<G>(mul, hinv, j, pos);
    M *m = msg + (size_t)e * G;
#pragma unroll
    for (int p = 0; p < H; ++p) {
        m[pos[2 * p]] = (M)v[p].x;
        m[pos[2 * p + 1]] = (M)v[p].y;
    }
}

// Check-node update of check r (eqs. (7)-(13)) by one segment: the forward vectors
// F_0 .. F_{dc-2} in registers, the backward vector running down from the last edge,
// the betas of the middle edges from F_{j-1} and B_{j+1}; F at the last edge and B at
// the first are never used by the outputs and are not formed.
template <int G, int DC, class M>
__device__ __forceinline__ void check_out(const v2s (&a)[DC][Geo<G>::H], M *bl, const uint8_t *mul,
                                          const uint8_t *hinvl, int e0, int dc, int j) {
    constexpr int H = Geo<G>::H;
    v2s F[DC][H], Bv[H], t[H];
#pragma unroll
    for (int p = 0; p < H; ++p) F[0][p] = a[0][p];
#pragma unroll
    for (int q = 1; q < DC - 1; ++q)
        if (q <= dc - 2) conv<G>(F[q - 1], a[q], F[q]);
    // last edge: beta~ = F_{dc-2}; backward vector starts at the last edge's alpha~
#pragma unroll
    for (int q = 1; q < DC; ++q)
        if (q == dc - 1) {
            store_deperm<G, M>(bl, mul, hinvl[e0 + q], e0 + q, j, F[q - 1]);
#pragma unroll
            for (int p = 0; p < H; ++p) Bv[p] = a[q][p];
        }
#pragma unroll
    for (int q = DC - 2; q >= 1; --q)
        if (q <= dc - 2) {
            conv<G>(F[q - 1], Bv, t);
            store_deperm<G, M>(bl, mul, hinvl[e0 + q], e0 + q, j, t);
            conv<G>(Bv, a[q], t);
#pragma unroll
            for (int p = 0; p < H; ++p) Bv[p] = t[p];
        }
    store_deperm<G, M>(bl, mul, hinvl[e0], e0, j, Bv);
}

template <int G, int DC, class M>
__device__ __forceinline__ void check(const DevCode &C, const M *al, M *bl, const uint8_t *mul,
                                      const uint8_t *hinvl, int r, int j) {
    const int e0 = C.row_ptr[r], dc = C.row_ptr[r + 1] - e0;
    v2s a[DC][Geo<G>::H];
#pragma unroll
    for (int q = 0; q < DC; ++q)
        if (q < dc) load_perm<G, M>(al, mul, hinvl[e0 + q], e0 + q, j, a[q]);
    check_out<G, DC, M>(a, bl, mul, hinvl, e0, dc, j);
}

// alpha~ of edge e (variable v, whose other edge is eo) at the lane's permuted positions,
// formed from the stored gamma' and beta_eo (alpha-free decoding): the minimum over
// the vector does not depend on the permutation.  first: alpha^(0) = gamma' itself.
template <int G, class M>
__device__ __forceinline__ void alpha_fly(const M *gl, const M *bl, const uint8_t *mul, int hinv, int v, int eo,
                                          int j, int amax, bool first, v2s (&out)[Geo<G>::H]) {
    constexpr int R = Geo<G>::R, S = Geo<G>::S, H = Geo<G>::H;
    uint8_t pos[R];
    perm_pos<G>(mul, hinv, j, pos);
    const M *gv = gl + (size_t)v * G, *be = bl + (size_t)eo * G;
    int s[R];
#pragma unroll
    for (int i = 0; i < R; ++i) s[i] = (int)gv[pos[i]];
    if (!first) {
#pragma unroll
        for (int i = 0; i < R; ++i) s[i] += (int)be[pos[i]];
        int mn = s[0];
#pragma unroll
        for (int i = 1; i < R; ++i) mn = min(mn, s[i]);
        mn = seg_min<S>(mn);
#pragma unroll
        for (int i = 0; i < R; ++i) s[i] = min(s[i] - mn, amax);
    }
#pragma unroll
    for (int p = 0; p < H; ++p) out[p] = (v2s){(short)s[2 * p], (short)s[2 * p + 1]};
}

// Inputs alpha~ of check r's edges, formed on the fly (alpha-free decoding); vt[e] holds
// (variable of e) | (other edge of that variable) << 16.
template <int G, int DC, class M>
__device__ __forceinline__ void load_fly(const DevCode &C, const M *gl, const M *bl, const uint8_t *mul,
                                         const uint8_t *hinvl, const uint32_t *vt, int r, int j, int amax, bool first,
                                         v2s (&a)[DC][Geo<G>::H]) {
    const int e0 = C.row_ptr[r], dc = C.row_ptr[r + 1] - e0;
#pragma unroll
    for (int q = 0; q < DC; ++q)
        if (q < dc) {
            const uint32_t w = vt[e0 + q];
            alpha_fly<G, M>(gl, bl, mul, hinvl[e0 + q], (int)(w & 0xFFFFu), (int)(w >> 16), j, amax, first, a[q]);
        }
}

// Sum of gamma' and the betas of variable v's edges (all, or all but edge `skip`), for
// the lane's R entries, in 32 bits.
template <int G, class M>
__device__ __forceinline__ void var_sum(const DevCode &C, const M *gl, const M *bl, int v, int j, int skip,
                                        int (&s)[Geo<G>::R]) {
    constexpr int R = Geo<G>::R;
    const M *gr = gl + (size_t)v * G + R * j;
#pragma unroll
    for (int i = 0; i < R; ++i) s[i] = (int)gr[i];
    for (int t = C.vn_ptr[v]; t < C.vn_ptr[v + 1]; ++t) {
        const int e = C.vn_ref[t];
        if (e == skip) continue;
        const M *br = bl + (size_t)e * G + R * j;
#pragma unroll
        for (int i = 0; i < R; ++i) s[i] += (int)br[i];
    }
}

// alpha of edge e (eq. (14)-(15) of its variable v): gamma' plus the betas of v's other
// edges, shifted to minimum 0 and clipped to amax.
template <int G, class M>
__device__ __forceinline__ void alpha_edge(const DevCode &C, const M *gl, const M *bl, M *al, int v, int e, int j,
                                           int amax) {
    constexpr int R = Geo<G>::R, S = Geo<G>::S;
    int s[R];
    var_sum<G, M>(C, gl, bl, v, j, e, s);
    int mn = s[0];
#pragma unroll
    for (int i = 1; i < R; ++i) mn = min(mn, s[i]);
    mn = seg_min<S>(mn);
    M *ar = al + (size_t)e * G + R * j;
#pragma unroll
    for (int i = 0; i < R; ++i) ar[i] = (M)min(s[i] - mn, amax);
}

// Decision of variable v: the lowest x minimising gamma'(x) + sum of its betas (x).
template <int G, class M>
__device__ __forceinline__ void decide(const DevCode &C, const M *gl, const M *bl, uint8_t *hl, int v, int j) {
    constexpr int R = Geo<G>::R, S = Geo<G>::S;
    int s[R];
    var_sum<G, M>(C, gl, bl, v, j, -1, s);
    int key = s[0] * G + R * j;
#pragma unroll
    for (int i = 1; i < R; ++i) key = min(key, s[i] * G + R * j + i);
    key = seg_min<S>(key);
    if (j == 0) hl[v] = (uint8_t)(key & (G - 1));
}

// 1 when every check is satisfied by the decisions in LDS (all threads cooperate; ends
// with the result visible to every thread).  slot alternates between calls so that the
// flag cleared for the next call is never the one being read.
__device__ __forceinline__ bool syndrome_ok(const DevCode &C, const uint8_t *mul, const uint8_t *hl_h,
                                            const uint8_t *hard, int *flags, int slot) {
    for (int r = threadIdx.x; r < C.m; r += blockDim.x) {
        int s = 0;
        for (int e = C.row_ptr[r]; e < C.row_ptr[r + 1]; ++e) s ^= mul[hl_h[e] * C.g + hard[C.col_idx[e]]];
        if (s) flags[slot] = 1;
    }
    __syncthreads();
    const bool ok = flags[slot] == 0;
    if (threadIdx.x == 0) flags[slot ^ 1] = 0;
    __syncthreads();
    return ok;
}

// The whole decode of codeword b by the calling workgroup (any multiple of 64 threads),
// messages stored as M (int16_t, or uint8_t when the bound is at most 255).  Ends with
// a barrier, so the caller may reuse the LDS right after.  AF: alpha-free decoding
// (every variable of degree 2; flooding needs at most two checks per segment, and the
// debug dump is only taken with flooding).
template <int G, int DC, class M, bool AF = false>
__device__ __forceinline__ void decode_cw(const Job &J, int b, unsigned char *lds) {
    constexpr int S = Geo<G>::S, VPW = Geo<G>::VPW, H = Geo<G>::H, R = Geo<G>::R;
    const DevCode &C = J.C;
    const Layout Y = layout(C, (int)sizeof(M), AF);
    M *gl = (M *)(lds + Y.gam), *al = (M *)(lds + Y.alpha), *bl = (M *)(lds + Y.beta);
    uint8_t *mul = lds + Y.mul, *hinvl = lds + Y.hinv, *hl_h = lds + Y.h, *hard = lds + Y.hard;
    int *flags = (int *)(lds + Y.flags);
    uint32_t *vt = (uint32_t *)(lds + Y.vt);
    const int tid = threadIdx.x, nthr = blockDim.x;
    const int lane = tid & 63, seg = lane / S, j = lane % S;
    const int segs = (nthr >> 6) * VPW, myseg = wave_id() * VPW + seg;  // segments of the workgroup
    const int amax = J.amax;

    // stage: clipped channel vectors, tables, alpha^(0) = gamma', beta = 0
    const int16_t *src = (const int16_t *)J.io.llr + (size_t)b * C.n * G;
    for (int i = tid; i < C.n * G; i += nthr) gl[i] = (M)min((int)src[i], amax);
    for (int i = tid; i < G * G; i += nthr) mul[i] = C.gfmul[i];
    for (int i = tid; i < C.E; i += nthr) {
        hinvl[i] = C.hinv[i];
        hl_h[i] = C.h[i];
    }
    if (tid < 4) flags[tid] = 0;
    if (AF) {
        for (int v = tid; v < C.n; v += nthr) {
            const int t = C.vn_ptr[v], e0 = C.vn_ref[t], e1 = C.vn_ref[t + 1];
            vt[e0] = (uint32_t)v | ((uint32_t)e1 << 16);
            vt[e1] = (uint32_t)v | ((uint32_t)e0 << 16);
        }
    }
    __syncthreads();
    for (int i = tid; i < C.E * G; i += nthr) {
        if (!AF) {
            const int e = i / G, x = i - e * G;
            al[i] = gl[(size_t)C.col_idx[e] * G + x];
        }
        bl[i] = 0;
    }
    __syncthreads();
    // decision of iteration 0: the lowest x minimising gamma'
    for (int v = myseg; v < C.n; v += segs) decide<G, M>(C, gl, bl, hard, v, j);
    __syncthreads();

    int it = 0, slot = 0;
    for (int k = 1; k <= J.max_iters; ++k) {
        if (J.early_stop) {
            const bool done = syndrome_ok(C, mul, hl_h, hard, flags, slot);
            slot ^= 1;
            if (done) break;
        }
        const bool need_dec = J.early_stop || k == J.max_iters;
        if (AF && !J.layered) {
            // every check's inputs of this iteration (from the betas of the last) are in
            // registers before any beta of this iteration is written
            v2s a[2][DC][H];
            const int r0 = myseg, r1 = myseg + segs;
            if (r0 < C.m) load_fly<G, DC, M>(C, gl, bl, mul, hinvl, vt, r0, j, amax, k == 1, a[0]);
            if (r1 < C.m) load_fly<G, DC, M>(C, gl, bl, mul, hinvl, vt, r1, j, amax, k == 1, a[1]);
            __syncthreads();
            if (r0 < C.m) check_out<G, DC, M>(a[0], bl, mul, hinvl, C.row_ptr[r0], C.row_ptr[r0 + 1] - C.row_ptr[r0], j);
            if (r1 < C.m) check_out<G, DC, M>(a[1], bl, mul, hinvl, C.row_ptr[r1], C.row_ptr[r1 + 1] - C.row_ptr[r1], j);
            __syncthreads();
            if (need_dec) {
                for (int v = myseg; v < C.n; v += segs) decide<G, M>(C, gl, bl, hard, v, j);
                __syncthreads();
            }
        } else if (AF) {
            for (int l = 0; l < C.nb_nl; ++l) {
                for (int i = C.nbl_ptr[l] + myseg; i < C.nbl_ptr[l + 1]; i += segs) {
                    const int r = C.nbl_chk[i];
                    v2s a[DC][H];
                    load_fly<G, DC, M>(C, gl, bl, mul, hinvl, vt, r, j, amax, false, a);
                    check_out<G, DC, M>(a, bl, mul, hinvl, C.row_ptr[r], C.row_ptr[r + 1] - C.row_ptr[r], j);
                }
                __syncthreads();
            }
            if (need_dec) {
                for (int v = myseg; v < C.n; v += segs) decide<G, M>(C, gl, bl, hard, v, j);
                __syncthreads();
            }
        } else if (!J.layered) {
            for (int r = myseg; r < C.m; r += segs) check<G, DC, M>(C, al, bl, mul, hinvl, r, j);
            __syncthreads();
            for (int t = myseg; t < C.E; t += segs) {
                const int e = C.vn_edge[t];
                alpha_edge<G, M>(C, gl, bl, al, C.col_idx[e], e, j, amax);
            }
            if (need_dec)
                for (int v = myseg; v < C.n; v += segs) decide<G, M>(C, gl, bl, hard, v, j);
            __syncthreads();
        } else {
            for (int l = 0; l < C.nb_nl; ++l) {
                for (int i = C.nbl_eptr[l] + myseg; i < C.nbl_eptr[l + 1]; i += segs) {
                    const int e = C.nbl_edge[i];
                    alpha_edge<G, M>(C, gl, bl, al, C.col_idx[e], e, j, amax);
                }
                __syncthreads();
                for (int i = C.nbl_ptr[l] + myseg; i < C.nbl_ptr[l + 1]; i += segs)
                    check<G, DC, M>(C, al, bl, mul, hinvl, C.nbl_chk[i], j);
                __syncthreads();
            }
            if (need_dec) {
                for (int v = myseg; v < C.n; v += segs) decide<G, M>(C, gl, bl, hard, v, j);
                __syncthreads();
            }
        }
        it = k;
    }
    const bool ok = syndrome_ok(C, mul, hl_h, hard, flags, slot);
    if (tid == 0) {
        J.io.ok[b] = ok ? 1 : 0;
        J.io.iters[b] = (int16_t)it;
    }
    uint8_t *hout = (uint8_t *)J.io.hard + (size_t)b * C.n;
    for (int v = tid; v < C.n; v += nthr) hout[v] = hard[v];
    if (J.io.dump_a) {
        int16_t *da = (int16_t *)J.io.dump_a + (size_t)b * C.E * G, *db = (int16_t *)J.io.dump_b + (size_t)b * C.E * G;
        if (AF) {
            // the alphas the flooding decoder would hold now: gamma' plus the other edge's
            // beta, normalised (gamma' itself before any iteration)
            for (int e = myseg; e < C.E; e += segs) {
                const uint32_t w = vt[e];
                const M *gv = gl + (size_t)(w & 0xFFFFu) * G + R * j, *be = bl + (size_t)(w >> 16) * G + R * j;
                int s[R];
#pragma unroll
                for (int i = 0; i < R; ++i) s[i] = (int)gv[i] + (it > 0 ? (int)be[i] : 0);
                if (it > 0) {
                    int mn = s[0];
#pragma unroll
                    for (int i = 1; i < R; ++i) mn = min(mn, s[i]);
                    mn = seg_min<S>(mn);
#pragma unroll
                    for (int i = 0; i < R; ++i) s[i] = min(s[i] - mn, amax);
                }
#pragma unroll
                for (int i = 0; i < R; ++i) da[(size_t)e * G + R * j + i] = (int16_t)s[i];
            }
            for (int i = tid; i < C.E * G; i += nthr) db[i] = (int16_t)bl[i];
        } else {
            for (int i = tid; i < C.E * G; i += nthr) {
                da[i] = (int16_t)al[i];
                db[i] = (int16_t)bl[i];
            }
        }
    }
    __syncthreads();
}

}  // namespace nb1
}  // namespace dev
}  // namespace ldpcx
