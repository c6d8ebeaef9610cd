// Interleaved Min-Max decoder over GF(g), g = 2^p <= 64 (Alg. 2), as
// block-level device functions (blocks of 256 threads, block index explicit).
//
// Mapping: lane = codeword.  A wavefront processes one check node for 64
// codewords; each lane holds whole g-entry messages in registers as packed
// 16-bit pairs.  The forward/backward recursions of eqs. (9)-(10) and the
// middle outputs of eq. (13) become XOR (min,max)-convolutions
//     (A (*) B)(s) = min_t max(A(s ^ t), B(t))
// of messages that were first permuted by the edge coefficient
// (a~(t) = alpha(h^-1 t), the "multiply by h" of sec. 2.2; with that
// substitution x' + h x'' = x becomes x' ^ t = x).  Because every lane of a
// wave works on the same check, the permutation index h^-1 t is uniform across
// the wave and the permutation is done by the loads themselves: each load is a
// contiguous 128-byte segment of [edge][x][codeword] memory.  The convolution
// is fully unrolled over compile-time register indices (no cross-lane traffic,
// no LDS), two entries per v_pk_max_i16 / v_pk_min_i16.  Only the forward
// vectors needed by later middle outputs go through LDS.  Forward at the last
// edge and backward at the first edge are never used by eqs. (11)-(13) and are
// not computed (3(dc-2) convolutions per check instead of 4dc-6).
//
// The check node (cn_core) reads and writes messages through accessors, so the
// same code serves four arrangements: the messages in HBM with one launch per
// phase (flooding: cn_block / vn_block); flooding for codes whose variables all have
// degree 2 with the alphas formed inside the check node from gamma and the other
// edge's beta, the betas alternating between two arrays and the decisions formed only
// where they are used (cnf_block / dec_block); the layered schedule (layers of checks
// sharing no variable, alphas formed per check from the current betas:
// lay_alpha_block / lay_cn_block); and short codes whose messages of one group of 64
// codewords fit in LDS, decoded by one workgroup through every iteration
// (lds_group).
#pragma once

#include "dev_common.h"

namespace ldpcx {
namespace dev {
namespace nb {

struct Args {
    DevCode C;
    int max_iters, early_stop, batch, Bp, Gn, fslots;
    int amax;  // message bound: alpha and the channel vectors are clipped to it
    NbWork w;
    DecodeIO io;
};

template <int G>
__device__ __forceinline__ void conv(const v2s (&A)[G / 2], const v2s (&B)[G / 2], v2s (&R)[G / 2]) {
    constexpr int H = G / 2;
#pragma unroll
    for (int t = 0; t < G; ++t) {
        const v2s bt = (t & 1) ? B[t >> 1].yy : B[t >> 1].xx;
#pragma unroll
        for (int p = 0; p < H; ++p) {
            v2s a = A[p ^ (t >> 1)];
            if (t & 1) a = a.yx;
            const v2s v = __builtin_elementwise_max(a, bt);
            R[p] = (t == 0) ? v : __builtin_elementwise_min(R[p], v);
        }
    }
}

// Entry t of the (uniform) multiplication-table row: the row is read as 32-bit words
// through the scalar cache and the byte extracted on the scalar unit.
__device__ __forceinline__ uint32_t mrow_at(const uint32_t *mw, int t) {
    return (__builtin_amdgcn_readfirstlane(mw[t >> 2]) >> (8 * (t & 3))) & 0xFFu;
}

// Message arrays in the interleaved layout in HBM, [edge][x][Bp] int16.  Every access is
// a buffer load or store whose scalar offset carries (edge, x) and whose lane offset is
// the codeword.
struct HbmMsg {
    __amdgpu_buffer_rsrc_t rs;
    uint32_t Bp2;       // bytes between entries of one edge
    uint32_t lane_off;  // 2 b

    // a~(t) = msg(hinv * t) for one edge (mrow: the multiplication-table row of hinv).
    template <int G>
    __device__ __forceinline__ void load_perm(int e, const uint8_t *mrow, v2s (&A)[G / 2]) const {
        const uint32_t *mw = (const uint32_t *)mrow;
        const uint32_t base = __builtin_amdgcn_readfirstlane((uint32_t)e * G * Bp2);
#pragma unroll
        for (int t = 0; t < G; t += 2) {
            const uint32_t x0 = mrow_at(mw, t), x1 = mrow_at(mw, t + 1);
            const uint32_t lo = __builtin_amdgcn_raw_buffer_load_b16(rs, (int)lane_off, (int)(base + x0 * Bp2), 0);
            const uint32_t hi = __builtin_amdgcn_raw_buffer_load_b16(rs, (int)lane_off, (int)(base + x1 * Bp2), 0);
            A[t >> 1] = as_v2s(lo | (hi << 16));
        }
    }
    // msg(x) = v~(h x) stored for one edge: entry t goes to x = hinv * t.
    template <int G>
    __device__ __forceinline__ void store_deperm(int e, const uint8_t *mrow, const v2s (&V)[G / 2], bool act) const {
        if (!act) return;
        const uint32_t *mw = (const uint32_t *)mrow;
        const uint32_t base = __builtin_amdgcn_readfirstlane((uint32_t)e * G * Bp2);
#pragma unroll
        for (int t = 0; t < G; t += 2) {
            const uint32_t w = as_u32(V[t >> 1]);
            const uint32_t s0 = base + mrow_at(mw, t) * Bp2;
            const uint32_t s1 = base + mrow_at(mw, t + 1) * Bp2;
            __builtin_amdgcn_raw_buffer_store_b16((unsigned short)(w & 0xFFFFu), rs, (int)lane_off, (int)s0, 0);
            __builtin_amdgcn_raw_buffer_store_b16((unsigned short)(w >> 16), rs, (int)lane_off, (int)s1, 0);
        }
    }
};

// Message arrays of one group of 64 codewords resident in LDS, [edge][x][64] int16.
struct LdsMsg {
    uint16_t *p;
    int lane;

    template <int G>
    __device__ __forceinline__ void load_perm(int e, const uint8_t *mrow, v2s (&A)[G / 2]) const {
        const uint32_t *mw = (const uint32_t *)mrow;
        const uint16_t *q = p + (size_t)e * G * 64 + lane;
#pragma unroll
        for (int t = 0; t < G; t += 2) {
            const uint32_t lo = q[mrow_at(mw, t) * 64], hi = q[mrow_at(mw, t + 1) * 64];
            A[t >> 1] = as_v2s(lo | (hi << 16));
        }
    }
    template <int G>
    __device__ __forceinline__ void store_deperm(int e, const uint8_t *mrow, const v2s (&V)[G / 2], bool act) const {
        if (!act) return;
        const uint32_t *mw = (const uint32_t *)mrow;
        uint16_t *q = p + (size_t)e * G * 64 + lane;
#pragma unroll
        for (int t = 0; t < G; t += 2) {
            const uint32_t w = as_u32(V[t >> 1]);
            q[mrow_at(mw, t) * 64] = (uint16_t)(w & 0xFFFFu);
            q[mrow_at(mw, t + 1) * 64] = (uint16_t)(w >> 16);
        }
    }
};

__device__ __forceinline__ __amdgpu_buffer_rsrc_t msg_rsrc(const int16_t *p, const Args &A);

template <int G>
__device__ __forceinline__ void lds_put(uint32_t *slot, int lane, const v2s (&V)[G / 2]) {
#pragma unroll
    for (int p = 0; p < G / 2; ++p) slot[p * 64 + lane] = __builtin_bit_cast(uint32_t, V[p]);
}

template <int G>
__device__ __forceinline__ void lds_get(const uint32_t *slot, int lane, v2s (&V)[G / 2]) {
#pragma unroll
    for (int p = 0; p < G / 2; ++p) V[p] = __builtin_bit_cast(v2s, slot[p * 64 + lane]);
}

// Waves per block of the check-node phase and its LDS need (forward vectors kept
// for the middle outputs: fslots x (G/2) x 64 lanes x 4 bytes per wave).
inline int cn_waves(const Args &A, size_t lds_budget) {
    const size_t per_wave = (size_t)A.fslots * (A.C.g / 2) * 64 * 4;
    const size_t w = lds_budget / per_wave;
    return (int)(w >= 4 ? 4 : w);
}
inline size_t cn_lds_bytes(const Args &A, int waves) { return (size_t)waves * A.fslots * (A.C.g / 2) * 64 * 4; }

// Whether codeword b (lane `lane` of group g) still runs in iteration k.
__device__ __forceinline__ bool active(const Args &A, int k, int g, int lane) {
    const int b = g * 64 + lane;
    return b < A.batch && (!A.early_stop || ((A.w.unsat[(size_t)k * A.Gn + g] >> lane) & 1ull));
}

// Check node of `row` (eqs. (7)-(13)) for the 64 codewords of one group: alpha read and
// beta written through the message accessors; fs: this wave's forward-vector slots in
// LDS; only lanes with `act` store.
// mul, hinv: the multiplication table and the inverse coefficients (HBM or LDS copies).
template <int G, class MA, class MB>
__device__ __forceinline__ void cn_core(const DevCode &C, const uint8_t *mul, const uint8_t *hinv, const MA &alpha,
                                        const MB &beta, int row, bool act, uint32_t *fs) {
    constexpr int H = G / 2;
    const int lane = threadIdx.x & 63;
    const int e0 = C.row_ptr[row];
    const int dc = C.row_ptr[row + 1] - e0;
    v2s X[H], Y[H], R[H];
    alpha.template load_perm<G>(e0, mul + hinv[e0] * G, X);
    const int nf = dc - 2;
    for (int s = 0; s < 3 * nf; ++s) {
        int kind, j;
        if (s < nf) {
            kind = 0;
            j = s + 1;
            alpha.template load_perm<G>(e0 + j, mul + hinv[e0 + j] * G, Y);
        } else {
            const int t = s - nf;
            j = dc - 2 - (t >> 1);
            if (t == 0) {
                // X = F_{dc-2} is the output of the last edge (eq. (12)); start the backward pass.
                beta.template store_deperm<G>(e0 + dc - 1, mul + hinv[e0 + dc - 1] * G, X, act);
                alpha.template load_perm<G>(e0 + dc - 1, mul + hinv[e0 + dc - 1] * G, X);
            }
            if ((t & 1) == 0) {
                kind = 1;  // middle output: F_{j-1} (*) B_{j+1}
                if (j == 1) alpha.template load_perm<G>(e0, mul + hinv[e0] * G, Y);
                else lds_get<G>(fs + (size_t)(j - 2) * H * 64, lane, Y);
            } else {
                kind = 2;  // B_j = B_{j+1} (*) a~_j
                alpha.template load_perm<G>(e0 + j, mul + hinv[e0 + j] * G, Y);
            }
        }
        conv<G>(X, Y, R);
        if (kind == 1) {
            beta.template store_deperm<G>(e0 + j, mul + hinv[e0 + j] * G, R, act);
        } else {
#pragma unroll
            for (int p = 0; p < H; ++p) X[p] = R[p];
            if (kind == 0 && j <= dc - 3) lds_put<G>(fs + (size_t)(j - 1) * H * 64, lane, X);
        }
    }
    if (nf == 0) {
        beta.template store_deperm<G>(e0 + 1, mul + hinv[e0 + 1] * G, X, act);
        alpha.template load_perm<G>(e0 + 1, mul + hinv[e0 + 1] * G, X);
    }
    beta.template store_deperm<G>(e0, mul + hinv[e0] * G, X, act);
}

// The check node on the HBM-resident messages, wave w of the block.
template <int G>
__device__ __forceinline__ void cn_row(const Args &A, int row, int w, int g, bool act, uint32_t *lds) {
    const uint32_t lo = 2u * (uint32_t)(g * 64 + (threadIdx.x & 63));
    const HbmMsg alpha{msg_rsrc(A.w.alpha, A), 2u * (uint32_t)A.Bp, lo};
    const HbmMsg beta{msg_rsrc(A.w.beta, A), 2u * (uint32_t)A.Bp, lo};
    cn_core<G>(A.C, A.C.gfmul, A.C.hinv, alpha, beta, row, act, lds + (size_t)w * A.fslots * (G / 2) * 64);
}

// Check-node phase of iteration k: wave (threadIdx.x / 64) of virtual block (bx, by)
// processes check bx * wpb + wave for codewords [64 by, 64 by + 64).
template <int G>
__device__ __forceinline__ void cn_block(const Args &A, int k, int wpb, int bx, int by, uint32_t *lds) {
    const int w = wave_id();
    if (w >= wpb) return;
    const int row = bx * wpb + w;
    if (row >= A.C.m) return;
    const bool act = active(A, k, by, threadIdx.x & 63);
    if (__ballot(act) == 0) return;
    cn_row<G>(A, row, w, by, act, lds);
}

// Flooding alphas formed inside the check node (eq. (14)) for codes whose variables all
// have degree 2: the clipped channel vector of the edge's variable plus the previous
// iteration's beta of the variable's other edge, shifted to minimum 0 and clipped to the
// message bound, read through the same permutation as an alpha row in HBM.  This
// replaces the variable node's alpha stores and the check node's alpha loads by loads
// of gamma and of the other beta.  The sums S are kept as unsigned 16-bit pairs while
// the minimum is found; betas lie in [0, 32767], so with channel costs in [0, 32767]
// every S fits and the alphas follow with two packed operations per pair.  A wave with
// a sum outside [0, 65535] (negative costs) reloads and forms them in 32 bits.
typedef unsigned short v2u __attribute__((ext_vector_type(2)));

struct FusedAlpha {
    __amdgpu_buffer_rsrc_t gam, beta;  // [n][x][Bp] channel vectors, [E][x][Bp] previous betas
    uint32_t Bp2, lane_off;
    int amax;
    const int *col_idx, *vn_ptr, *vn_ref;

    __device__ __forceinline__ int ld(__amdgpu_buffer_rsrc_t r, uint32_t soff) const {
        return (int)(int16_t)__builtin_amdgcn_raw_buffer_load_b16(r, (int)lane_off, (int)soff, 0);
    }

    template <int G>
    __device__ __forceinline__ void load_perm(int e, const uint8_t *mrow, v2s (&A)[G / 2]) const {
        const uint32_t *mw = (const uint32_t *)mrow;
        const int v = __builtin_amdgcn_readfirstlane(col_idx[e]);
        const int q0 = __builtin_amdgcn_readfirstlane(vn_ptr[v]);
        const int f0 = __builtin_amdgcn_readfirstlane(vn_ref[q0]), f1 = __builtin_amdgcn_readfirstlane(vn_ref[q0 + 1]);
        const uint32_t gb = __builtin_amdgcn_readfirstlane((uint32_t)v * G * Bp2);
        const uint32_t fb = __builtin_amdgcn_readfirstlane((uint32_t)(f0 == e ? f1 : f0) * G * Bp2);
        auto sum_at = [&](int t) {
            const uint32_t xo = mrow_at(mw, t) * Bp2;
            return min(ld(gam, gb + xo), amax) + ld(beta, fb + xo);
        };
        int mn = 0x7fffffff;
        uint32_t wide = 0;  // bits above 16 of any sum (negative sums set them all)
#pragma unroll
        for (int t = 0; t < G; t += 2) {
            const int s0 = sum_at(t), s1 = sum_at(t + 1);
            mn = min(mn, min(s0, s1));
            wide |= ((uint32_t)s0 | (uint32_t)s1) >> 16;
            A[t >> 1] = as_v2s(((uint32_t)s0 & 0xFFFFu) | ((uint32_t)s1 << 16));
        }
        if (__ballot(wide != 0) == 0) {
            const v2u m = (v2u){(unsigned short)mn, (unsigned short)mn}, cap = (v2u){(unsigned short)amax, (unsigned short)amax};
#pragma unroll
            for (int p = 0; p < G / 2; ++p) {
                const v2u d = __builtin_bit_cast(v2u, A[p]) - m;  // S - min, no wrap: S >= min
                A[p] = __builtin_bit_cast(v2s, __builtin_elementwise_min(d, cap));
            }
            return;
        }
        // Reload pair by pair (the barriers keep the compiler from holding the G 32-bit
        // sums or hoisting the reloads, so this rare path costs the common one no registers).
#pragma unroll
        for (int t = 0; t < G; t += 2) {
            asm volatile("" ::: "memory");
            const uint32_t a0 = (uint32_t)min(sum_at(t) - mn, amax), a1 = (uint32_t)min(sum_at(t + 1) - mn, amax);
            A[t >> 1] = as_v2s(a0 | (a1 << 16));
        }
    }
};

// Buffer resource over the [n][x][Bp] channel vectors.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t gam_rsrc(const Args &A) {
    const uint32_t bytes = (uint32_t)A.C.n * (uint32_t)A.C.g * (uint32_t)A.Bp * 2u;
    return __builtin_amdgcn_make_buffer_rsrc(A.w.gam, (short)0, (int)bytes, 0x00020000);
}

// A posteriori sums S(x) = gamma'(x) + sum of the variable's betas (eq. (15)) for the
// lane's codeword, by buffer loads whose scalar offset carries (variable or edge, entry)
// and whose lane offset is the codeword; returns the arg-min (lowest x on ties) as the
// minimum of the keys S(x) * 64 + x.
template <int G>
__device__ __forceinline__ int app_sums(const Args &A, int v, uint32_t lo, int (&S)[G]) {
    const DevCode &C = A.C;
    const uint32_t Bp2 = 2u * (uint32_t)A.Bp;
    const __amdgpu_buffer_rsrc_t rg = gam_rsrc(A), rb = msg_rsrc(A.w.beta, A);
    const uint32_t gb = __builtin_amdgcn_readfirstlane((uint32_t)v * G * Bp2);
#pragma unroll
    for (int x = 0; x < G; ++x)
        S[x] = min((int)(int16_t)__builtin_amdgcn_raw_buffer_load_b16(rg, (int)lo, (int)(gb + x * Bp2), 0), A.amax);
    for (int t = C.vn_ptr[v]; t < C.vn_ptr[v + 1]; ++t) {
        const uint32_t fb = __builtin_amdgcn_readfirstlane((uint32_t)C.vn_ref[t] * G * Bp2);
#pragma unroll
        for (int x = 0; x < G; ++x)
            S[x] += (int)(int16_t)__builtin_amdgcn_raw_buffer_load_b16(rb, (int)lo, (int)(fb + x * Bp2), 0);
    }
    int key = S[0] * 64;
#pragma unroll
    for (int x = 1; x < G; ++x) key = min(key, S[x] * 64 + x);
    return key & 63;
}

// Decision of iteration k without the alphas (layered schedule, fused flooding): one
// wave per (variable, group).
template <int G>
__device__ __forceinline__ void dec_block(const Args &A, int k, int bx, int by) {
    const int lane = threadIdx.x & 63;
    const int v = bx * 4 + wave_id();
    if (v >= A.C.n) return;
    const int b = by * 64 + lane;
    const bool act = active(A, k, by, lane);
    if (__ballot(act) == 0) return;
    int S[G];
    const int best = app_sums<G>(A, v, 2u * (uint32_t)b, S);
    if (act) {
        A.w.hard[(long)v * A.Bp + b] = (uint8_t)best;
        if (v == 0) A.w.it[b] = (int16_t)k;
    }
}

// Fused flooding check node of iteration k (alphas from gamma and beta_old, betas to
// beta_new): wave w of virtual block (bx, by) as in cn_block.
template <int G>
__device__ __forceinline__ void cnf_block(const Args &A, int k, int wpb, int bx, int by, uint32_t *lds,
                                          const int16_t *beta_old, int16_t *beta_new) {
    const int w = wave_id();
    if (w >= wpb) return;
    const int row = bx * wpb + w;
    if (row >= A.C.m) return;
    const bool act = active(A, k, by, threadIdx.x & 63);
    if (__ballot(act) == 0) return;
    const uint32_t lo = 2u * (uint32_t)(by * 64 + (threadIdx.x & 63));
    const FusedAlpha alpha{gam_rsrc(A), msg_rsrc(beta_old, A), 2u * (uint32_t)A.Bp, lo, A.amax,
                           A.C.col_idx, A.C.vn_ptr, A.C.vn_ref};
    const HbmMsg beta{msg_rsrc(beta_new, A), 2u * (uint32_t)A.Bp, lo};
    cn_core<G>(A.C, A.C.gfmul, A.C.hinv, alpha, beta, row, act, lds + (size_t)w * A.fslots * (G / 2) * 64);
}

// Layered schedule: alpha of edge e from eq. (14) with the betas as they stand, i.e. the
// channel vector of its variable plus the betas of the variable's other edges, shifted
// to minimum 0 and clipped to the message bound.
template <int G>
__device__ __forceinline__ void alpha_edge(const Args &A, int e, int b, bool act) {
    const DevCode &C = A.C;
    const long Bp = A.Bp;
    const int v = C.col_idx[e];
    int S[G];
    const int16_t *gp = A.w.gam + (long)v * G * Bp + b;
#pragma unroll
    for (int x = 0; x < G; ++x) S[x] = min((int)gp[(long)x * Bp], A.amax);
    for (int t = C.vn_ptr[v]; t < C.vn_ptr[v + 1]; ++t) {
        const int f = C.vn_ref[t];
        if (f == e) continue;
        const int16_t *bp = A.w.beta + (long)f * G * Bp + b;
#pragma unroll
        for (int x = 0; x < G; ++x) S[x] += bp[(long)x * Bp];
    }
    int mn = S[0];
#pragma unroll
    for (int x = 1; x < G; ++x) mn = min(mn, S[x]);
    if (act) {
        int16_t *ap = A.w.alpha + (long)e * G * Bp + b;
#pragma unroll
        for (int x = 0; x < G; ++x) ap[(long)x * Bp] = (int16_t)min(S[x] - mn, A.amax);
    }
}

// Layered schedule, iteration k, layer `layer` (checks sharing no variable), first
// step: the alphas of the layer's edges.  Wave per (edge of the layer, group).
template <int G>
__device__ __forceinline__ void lay_alpha_block(const Args &A, int k, int layer, int bx, int by) {
    const DevCode &C = A.C;
    const int i = C.nbl_eptr[layer] + bx * 4 + wave_id();
    if (i >= C.nbl_eptr[layer + 1]) return;
    const int e = __builtin_amdgcn_readfirstlane(C.nbl_edge[i]);
    const int lane = threadIdx.x & 63;
    const bool act = active(A, k, by, lane);
    if (__ballot(act) == 0) return;
    alpha_edge<G>(A, e, by * 64 + lane, act);
}

// Second step: the check nodes of the layer.  Wave w of virtual block (bx, by) takes the
// layer's check number bx * wpb + w for codewords [64 by, 64 by + 64).
template <int G>
__device__ __forceinline__ void lay_cn_block(const Args &A, int k, int layer, int wpb, int bx, int by, uint32_t *lds) {
    const DevCode &C = A.C;
    const int w = wave_id();
    if (w >= wpb) return;
    const int i = C.nbl_ptr[layer] + bx * wpb + w;
    if (i >= C.nbl_ptr[layer + 1]) return;
    const int row = __builtin_amdgcn_readfirstlane(C.nbl_chk[i]);
    const bool act = active(A, k, by, threadIdx.x & 63);
    if (__ballot(act) == 0) return;
    cn_row<G>(A, row, w, by, act, lds);
}

// Layered schedule for codes whose variables all have degree 2, one launch per layer: the
// layer's check nodes form their alphas themselves (FusedAlpha on the betas as they
// stand).  The other edge of an edge's variable belongs to a check of another layer, so
// the betas read are never those the launch writes.
template <int G>
__device__ __forceinline__ void lay_cnf_block(const Args &A, int k, int layer, int wpb, int bx, int by,
                                              uint32_t *lds) {
    const DevCode &C = A.C;
    const int w = wave_id();
    if (w >= wpb) return;
    const int i = C.nbl_ptr[layer] + bx * wpb + w;
    if (i >= C.nbl_ptr[layer + 1]) return;
    const int row = __builtin_amdgcn_readfirstlane(C.nbl_chk[i]);
    const bool act = active(A, k, by, threadIdx.x & 63);
    if (__ballot(act) == 0) return;
    const uint32_t lo = 2u * (uint32_t)(by * 64 + (threadIdx.x & 63));
    const __amdgpu_buffer_rsrc_t rb = msg_rsrc(A.w.beta, A);
    const FusedAlpha alpha{gam_rsrc(A), rb, 2u * (uint32_t)A.Bp, lo, A.amax, C.col_idx, C.vn_ptr, C.vn_ref};
    const HbmMsg beta{rb, 2u * (uint32_t)A.Bp, lo};
    cn_core<G>(C, C.gfmul, C.hinv, alpha, beta, row, act, lds + (size_t)w * A.fslots * (G / 2) * 64);
}

// Variable-node update (eqs. (14)-(15)) and decision: one wave per (variable, group).
// (Global loads with 64-bit addresses measured a few per cent faster here than buffer
// loads, unlike the decision-only kernel.)
template <int G>
__device__ __forceinline__ void vn_block(const Args &A, int k, int bx, int by) {
    const DevCode &C = A.C;
    const long Bp = A.Bp;
    const int lane = threadIdx.x & 63;
    const int v = bx * 4 + wave_id();
    if (v >= C.n) return;
    const int g = by;
    const int b = g * 64 + lane;
    const uint64_t *slot = A.w.unsat + (size_t)k * A.Gn;
    const bool act = b < A.batch && (!A.early_stop || ((slot[g] >> lane) & 1ull));
    if (__ballot(act) == 0) return;
    int S[G];
    const int16_t *gp = A.w.gam + (long)v * G * Bp + b;
#pragma unroll
    for (int x = 0; x < G; ++x) S[x] = min((int)gp[(long)x * Bp], A.amax);
    const int t0 = C.vn_ptr[v], t1 = C.vn_ptr[v + 1];
    for (int t = t0; t < t1; ++t) {
        const int16_t *bp = A.w.beta + (long)C.vn_ref[t] * G * Bp + b;
#pragma unroll
        for (int x = 0; x < G; ++x) S[x] += bp[(long)x * Bp];
    }
    int best = 0, bv = S[0];
#pragma unroll
    for (int x = 1; x < G; ++x)
        if (S[x] < bv) {
            bv = S[x];
            best = x;
        }
    if (act) {
        A.w.hard[(long)v * Bp + b] = (uint8_t)best;
        if (v == 0) A.w.it[b] = (int16_t)k;
    }
    for (int t = t0; t < t1; ++t) {
        const int e = C.vn_ref[t];
        const int16_t *bp = A.w.beta + (long)e * G * Bp + b;
        int a[G];
        int mn = 0x7fffffff;
#pragma unroll
        for (int x = 0; x < G; ++x) {
            a[x] = S[x] - bp[(long)x * Bp];
            mn = min(mn, a[x]);
        }
        if (act) {
            int16_t *ap = A.w.alpha + (long)e * G * Bp + b;
#pragma unroll
            for (int x = 0; x < G; ++x) ap[(long)x * Bp] = (int16_t)min(a[x] - mn, A.amax);
        }
    }
}

// Syndrome sum_j h_j c_j over GF(g) for one check and 64 codewords (wave per (check, group)).
__device__ __forceinline__ void syn_block(const Args &A, int slot_k, int bx, int by) {
    const DevCode &C = A.C;
    const int lane = threadIdx.x & 63;
    const int row = bx * 4 + wave_id();
    if (row >= C.m) return;
    const int g = by;
    const int b = g * 64 + lane;
    int s = 0;
    for (int e = C.row_ptr[row]; e < C.row_ptr[row + 1]; ++e)
        s ^= C.gfmul[C.h[e] * C.g + A.w.hard[(long)C.col_idx[e] * A.Bp + b]];
    const uint64_t bits = __ballot(s != 0 && b < A.batch);
    if (lane == 0 && bits)
        atomicOr((unsigned long long *)&A.w.unsat[(size_t)slot_k * A.Gn + g], (unsigned long long)bits);
}

// alpha^(0) = gamma of the edge's variable (unless `alpha` is false: the fused flooding
// forms its alphas itself), beta = 0, decision of iteration 0 (wave per (edge or
// variable, group)).
template <int G>
__device__ __forceinline__ void init_block(const Args &A, int bx, int by, bool alpha = true) {
    const DevCode &C = A.C;
    const long Bp = A.Bp;
    const int lane = threadIdx.x & 63;
    const int e = bx * 4 + wave_id();
    const int b = by * 64 + lane;
    if (e < C.E) {
        const int16_t *gp = A.w.gam + (long)C.col_idx[e] * G * Bp + b;
        int16_t *ap = A.w.alpha + (long)e * G * Bp + b;
        int16_t *bp = A.w.beta + (long)e * G * Bp + b;
#pragma unroll 8
        for (int x = 0; x < G; ++x) {
            if (alpha) ap[(long)x * Bp] = (int16_t)min((int)gp[(long)x * Bp], A.amax);
            bp[(long)x * Bp] = 0;
        }
    }
    if (e < C.n) {
        // most likely channel symbol, lowest x on ties
        const int16_t *gp = A.w.gam + (long)e * G * Bp + b;
        int best = 0, bv = min((int)gp[0], A.amax);
        for (int x = 1; x < G; ++x) {
            const int val = min((int)gp[(long)x * Bp], A.amax);
            if (val < bv) {
                bv = val;
                best = x;
            }
        }
        A.w.hard[(long)e * Bp + b] = (uint8_t)best;
    }
}

// ------------------------------------ one group per workgroup, messages resident in LDS
// For codes whose alpha and beta for one group of 64 codewords fit in LDS: a workgroup
// of `waves` waves decodes one group through every iteration with alpha, beta and the
// decisions in LDS ([edge][x][64] and [variable][64]), reading the channel vectors from
// the transposed input in HBM; waves split the checks and the variables of each phase,
// with a barrier between phases.  The arithmetic is that of the kernels above.

struct LdsPlan {
    size_t gam, alpha, beta, hard, mul, fs, red, total;
};

// gam_lds: the clipped channel vectors are staged in LDS too ([variable][x][64]).
__host__ __device__ inline LdsPlan lds_plan(const DevCode &C, int fslots, int waves, bool gam_lds) {
    LdsPlan L;
    size_t o = 0;
    L.gam = o;
    if (gam_lds) o += (size_t)C.n * C.g * 128;
    L.alpha = o;
    o += (size_t)C.E * C.g * 128;
    L.beta = o;
    o += (size_t)C.E * C.g * 128;
    L.hard = o;
    o += ((size_t)C.n * 64 + 15) / 16 * 16;
    L.mul = o;  // multiplication table, then hinv and h of every edge
    o += ((size_t)C.g * C.g + 2 * (size_t)C.E + 15) / 16 * 16;
    L.fs = o;
    o += (size_t)waves * fslots * (C.g / 2) * 64 * 4;
    L.red = o;
    o += 8 * (size_t)waves;
    L.total = o;
    return L;
}

// Unsatisfied codewords of the group (bit = lane), uniform over the workgroup.
__device__ __forceinline__ uint64_t lds_syndrome(const DevCode &C, const uint8_t *mul, const uint8_t *h,
                                                 const uint8_t *hl, bool valid, int waves, uint64_t *red) {
    const int lane = threadIdx.x & 63, w = wave_id();
    uint64_t acc = 0;
    for (int r = w; r < C.m; r += waves) {
        int s = 0;
        for (int e = C.row_ptr[r]; e < C.row_ptr[r + 1]; ++e) s ^= mul[h[e] * C.g + hl[C.col_idx[e] * 64 + lane]];
        acc |= __ballot(s != 0 && valid);
    }
    if (lane == 0) red[w] = acc;
    __syncthreads();
    uint64_t u = 0;
    for (int q = 0; q < waves; ++q) u |= red[q];
    __syncthreads();
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)u);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(u >> 32));
    return ((uint64_t)hi << 32) | lo;
}

// Variable node v on the LDS messages (eqs. (14)-(15)); kAlpha = false: decision only.
// The clipped channel vector gamma'(x) of variable v for the lane's codeword, from LDS
// ([variable][x][64]) or from the transposed input in HBM.
template <int G, bool GL>
struct Gamma {
    const int16_t *hbm;  // A.w.gam + b
    const uint16_t *lds;  // staged copy + lane
    long Bp;
    int amax;
    __device__ __forceinline__ int at(int v, int x) const {
        if (GL) return (int16_t)lds[((size_t)v * G + x) * 64];
        return min((int)hbm[((long)v * G + x) * Bp], amax);
    }
};

template <int G, bool kAlpha, bool GL>
__device__ __forceinline__ void lds_vn(const Args &A, const Gamma<G, GL> &gam, uint16_t *al, const uint16_t *bl,
                                       uint8_t *hl, int v, bool act) {
    const DevCode &C = A.C;
    const int lane = threadIdx.x & 63;
    int S[G];
#pragma unroll
    for (int x = 0; x < G; ++x) S[x] = gam.at(v, x);
    const int t0 = C.vn_ptr[v], t1 = C.vn_ptr[v + 1];
    for (int t = t0; t < t1; ++t) {
        const uint16_t *bp = bl + (size_t)C.vn_ref[t] * G * 64 + lane;
#pragma unroll
        for (int x = 0; x < G; ++x) S[x] += (int16_t)bp[x * 64];
    }
    int best = 0, bv = S[0];
#pragma unroll
    for (int x = 1; x < G; ++x)
        if (S[x] < bv) {
            bv = S[x];
            best = x;
        }
    if (act) hl[v * 64 + lane] = (uint8_t)best;
    if (!kAlpha) return;
    for (int t = t0; t < t1; ++t) {
        const int e = C.vn_ref[t];
        const uint16_t *bp = bl + (size_t)e * G * 64 + lane;
        int a[G];
        int mn = 0x7fffffff;
#pragma unroll
        for (int x = 0; x < G; ++x) {
            a[x] = S[x] - (int16_t)bp[x * 64];
            mn = min(mn, a[x]);
        }
        if (act) {
            uint16_t *ap = al + (size_t)e * G * 64 + lane;
#pragma unroll
            for (int x = 0; x < G; ++x) ap[x * 64] = (uint16_t)min(a[x] - mn, A.amax);
        }
    }
}

// Layered schedule: alpha of edge e from eq. (14) with the LDS betas as they stand.
template <int G, bool GL>
__device__ __forceinline__ void lds_alpha_edge(const Args &A, const Gamma<G, GL> &gam, uint16_t *al,
                                               const uint16_t *bl, int e, bool act) {
    const DevCode &C = A.C;
    const int lane = threadIdx.x & 63;
    const int v = C.col_idx[e];
    int S[G];
#pragma unroll
    for (int x = 0; x < G; ++x) S[x] = gam.at(v, x);
    for (int t = C.vn_ptr[v]; t < C.vn_ptr[v + 1]; ++t) {
        const int f = C.vn_ref[t];
        if (f == e) continue;
        const uint16_t *bp = bl + (size_t)f * G * 64 + lane;
#pragma unroll
        for (int x = 0; x < G; ++x) S[x] += (int16_t)bp[x * 64];
    }
    int mn = S[0];
#pragma unroll
    for (int x = 1; x < G; ++x) mn = min(mn, S[x]);
    if (act) {
        uint16_t *ap = al + (size_t)e * G * 64 + lane;
#pragma unroll
        for (int x = 0; x < G; ++x) ap[x * 64] = (uint16_t)min(S[x] - mn, A.amax);
    }
}

// The whole decode of group g (every phase, every iteration) by the calling workgroup.
template <int G, bool GL>
__device__ __forceinline__ void lds_group(const Args &A, bool layered, int waves, int g, unsigned char *lds) {
    const DevCode &C = A.C;
    const int lane = threadIdx.x & 63, w = wave_id();
    const int b = g * 64 + lane;
    const bool valid = b < A.batch;
    const LdsPlan P = lds_plan(C, A.fslots, waves, GL);
    uint16_t *gl = (uint16_t *)(lds + P.gam);
    uint16_t *al = (uint16_t *)(lds + P.alpha);
    uint16_t *bl = (uint16_t *)(lds + P.beta);
    uint8_t *hl = lds + P.hard;
    uint8_t *ml = lds + P.mul;
    uint8_t *hinvl = ml + G * G, *hl_h = hinvl + C.E;
    uint32_t *fs = (uint32_t *)(lds + P.fs) + (size_t)w * A.fslots * (G / 2) * 64;
    uint64_t *red = (uint64_t *)(lds + P.red);
    for (int i = threadIdx.x; i < G * G; i += 64 * waves) ml[i] = C.gfmul[i];
    for (int i = threadIdx.x; i < C.E; i += 64 * waves) {
        hinvl[i] = C.hinv[i];
        hl_h[i] = C.h[i];
    }
    const Gamma<G, false> ghbm{A.w.gam + b, nullptr, A.Bp, A.amax};
    const Gamma<G, GL> gam{A.w.gam + b, gl + lane, A.Bp, A.amax};
    if (GL) {
        for (int v = w; v < C.n; v += waves)
#pragma unroll 8
            for (int x = 0; x < G; ++x) gl[((size_t)v * G + x) * 64 + lane] = (uint16_t)ghbm.at(v, x);
    }
    // alpha^(0) = gamma', beta = 0, decision of iteration 0
    for (int e = w; e < C.E; e += waves) {
        const int v = C.col_idx[e];
#pragma unroll 8
        for (int x = 0; x < G; ++x) {
            al[((size_t)e * G + x) * 64 + lane] = (uint16_t)ghbm.at(v, x);
            bl[((size_t)e * G + x) * 64 + lane] = 0;
        }
    }
    for (int v = w; v < C.n; v += waves) {
        int best = 0, bv = ghbm.at(v, 0);
        for (int x = 1; x < G; ++x) {
            const int val = ghbm.at(v, x);
            if (val < bv) {
                bv = val;
                best = x;
            }
        }
        hl[v * 64 + lane] = (uint8_t)best;
    }
    __syncthreads();
    int it = 0;
    for (int k = 1; k <= A.max_iters; ++k) {
        bool act = valid;
        if (A.early_stop) {
            const uint64_t u = lds_syndrome(C, ml, hl_h, hl, valid, waves, red);
            if (u == 0) break;  // every codeword of the group is done
            act = act && ((u >> lane) & 1ull);
        }
        const LdsMsg am{al, lane}, bm{bl, lane};
        if (!layered) {
            for (int r = w; r < C.m; r += waves) cn_core<G>(C, ml, hinvl, am, bm, r, act, fs);
            __syncthreads();
            for (int v = w; v < C.n; v += waves) lds_vn<G, true, GL>(A, gam, al, bl, hl, v, act);
            __syncthreads();
        } else {
            for (int l = 0; l < C.nb_nl; ++l) {
                for (int i = C.nbl_eptr[l] + w; i < C.nbl_eptr[l + 1]; i += waves)
                    lds_alpha_edge<G, GL>(A, gam, al, bl, __builtin_amdgcn_readfirstlane(C.nbl_edge[i]), act);
                __syncthreads();
                for (int i = C.nbl_ptr[l] + w; i < C.nbl_ptr[l + 1]; i += waves)
                    cn_core<G>(C, ml, hinvl, am, bm, __builtin_amdgcn_readfirstlane(C.nbl_chk[i]), act, fs);
                __syncthreads();
            }
            for (int v = w; v < C.n; v += waves) lds_vn<G, false, GL>(A, gam, al, bl, hl, v, act);
            __syncthreads();
        }
        if (act) it = k;
    }
    const uint64_t u0 = lds_syndrome(C, ml, hl_h, hl, valid, waves, red);
    if (w == 0 && valid) {
        A.io.ok[b] = ((u0 >> lane) & 1ull) ? 0 : 1;
        A.io.iters[b] = (int16_t)it;
    }
    // decisions (and, for the debug dump, the messages) back to the HBM layout
    for (int v = w; v < C.n; v += waves) A.w.hard[(long)v * A.Bp + b] = hl[v * 64 + lane];
    if (A.io.dump_a) {
        for (int e = w; e < C.E; e += waves)
            for (int x = 0; x < G; ++x) {
                A.w.alpha[((long)e * G + x) * A.Bp + b] = (int16_t)al[((size_t)e * G + x) * 64 + lane];
                A.w.beta[((long)e * G + x) * A.Bp + b] = (int16_t)bl[((size_t)e * G + x) * 64 + lane];
            }
    }
}

// Debug dump after the fused flooding: the betas of codeword b sit in the array its last
// iteration wrote (odd iteration counts: the alpha array, which the fused flooding uses
// as its second beta array), and its alphas are those the two-phase variable node forms
// from them (eqs. (14)-(15); gamma' itself before any iteration).  Thread per (edge,
// codeword), written straight to the [batch][E][G] dump.
template <int G>
__device__ __forceinline__ void fdump_block(const Args &A, int bx, int by) {
    const DevCode &C = A.C;
    const long Bp = A.Bp;
    const int e = bx * 4 + wave_id();
    const int b = by * 64 + (threadIdx.x & 63);
    if (e >= C.E || b >= A.batch) return;
    const int it = A.w.it[b];
    const int16_t *src = (it & 1) ? A.w.alpha : A.w.beta;
    const int v = C.col_idx[e];
    const int q0 = C.vn_ptr[v];
    const int f = C.vn_ref[q0] == e ? C.vn_ref[q0 + 1] : C.vn_ref[q0];
    const int16_t *gp = A.w.gam + (long)v * G * Bp + b;
    const int16_t *bf = src + (long)f * G * Bp + b, *be = src + (long)e * G * Bp + b;
    int16_t *da = (int16_t *)A.io.dump_a + ((size_t)b * C.E + e) * G;
    int16_t *db = (int16_t *)A.io.dump_b + ((size_t)b * C.E + e) * G;
    int mn = 0x7fffffff;
    if (it > 0)
        for (int x = 0; x < G; ++x) mn = min(mn, min((int)gp[(long)x * Bp], A.amax) + bf[(long)x * Bp]);
    for (int x = 0; x < G; ++x) {
        const int s = min((int)gp[(long)x * Bp], A.amax);
        da[x] = (int16_t)(it > 0 ? min(s + bf[(long)x * Bp] - mn, A.amax) : s);
        db[x] = be[(long)x * Bp];
    }
}

__device__ __forceinline__ void fin_block(const Args &A, long bx) {
    const int b = (int)(bx * 256 + threadIdx.x);
    if (b >= A.batch) return;
    A.io.ok[b] = ((A.w.unsat[b >> 6] >> (b & 63)) & 1ull) ? 0 : 1;
    A.io.iters[b] = A.w.it[b];
}

// Buffer resource over an [E][G][Bp] int16 message array (the host keeps its size
// within 31 bits by slicing the batch).
__device__ __forceinline__ __amdgpu_buffer_rsrc_t msg_rsrc(const int16_t *p, const Args &A) {
    const uint32_t bytes = (uint32_t)A.C.E * (uint32_t)A.C.g * (uint32_t)A.Bp * 2u;
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<int16_t *>(p), (short)0, (int)bytes, 0x00020000);
}

__host__ __device__ inline long grid_init_x(const Args &A) { return ((A.C.E > A.C.n ? A.C.E : A.C.n) + 3) / 4; }
__host__ __device__ inline long grid_rows_x(const Args &A) { return (A.C.m + 3) / 4; }
__host__ __device__ inline long grid_vn_x(const Args &A) { return (A.C.n + 3) / 4; }
__host__ __device__ inline long grid_fin(const Args &A) { return (A.batch + 255) / 256; }

struct Carve {
    size_t gam, alpha, beta, hard, unsat, it, total;
};

inline Carve carve(const DevCode &C, int max_iters, int batch) {
    const size_t Bp = pad64(batch), Gn = Bp / 64;
    Carve c;
    size_t o = 0;
    c.gam = o;
    o = align_up(o + (size_t)C.n * C.g * Bp * 2, 256);
    c.alpha = o;
    o = align_up(o + (size_t)C.E * C.g * Bp * 2, 256);
    c.beta = o;
    o = align_up(o + (size_t)C.E * C.g * Bp * 2, 256);
    c.hard = o;
    o = align_up(o + (size_t)C.n * Bp, 256);
    c.unsat = o;
    o = align_up(o + (size_t)(max_iters + 1) * Gn * 8, 256);
    c.it = o;
    o = align_up(o + Bp * 2, 256);
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
    A.Bp = pad64(batch);
    A.Gn = A.Bp / 64;
    A.fslots = C.dc_max > 3 ? C.dc_max - 3 : 1;
    const Carve c = carve(C, max_iters, batch);
    char *p = (char *)base;
    A.w.gam = (int16_t *)(p + c.gam);
    A.w.alpha = (int16_t *)(p + c.alpha);
    A.w.beta = (int16_t *)(p + c.beta);
    A.w.hard = (uint8_t *)(p + c.hard);
    A.w.unsat = (uint64_t *)(p + c.unsat);
    A.w.it = (int16_t *)(p + c.it);
    A.io = io;
    return A;
}

inline TransposeArgs tr_in(const Args &A) {
    const long cols = (long)A.C.n * A.C.g;
    return TransposeArgs{A.io.llr, A.w.gam, A.batch, cols, cols, A.Bp, A.Bp, 2};
}
inline TransposeArgs tr_out(const Args &A) {
    return TransposeArgs{A.w.hard, A.io.hard, A.C.n, A.batch, A.Bp, A.C.n, A.C.n, 1};
}
inline FillArgs fill_unsat(const Args &A) {
    return FillArgs{(uint32_t *)A.w.unsat, (size_t)(A.max_iters + 1) * A.Gn * 2, 0u};
}
inline FillArgs fill_it(const Args &A) { return FillArgs{(uint32_t *)A.w.it, (size_t)A.Bp / 2, 0u}; }

}  // namespace nb
}  // namespace dev
}  // namespace ldpcx
