// Packed two-codewords-per-lane min-sum decoder for quasi-cyclic codes, as a
// workgroup-level device function (see k_bin_qc.hip for the design).
#pragma once

#include <type_traits>

#include "dev_common.h"

namespace ldpcx {
namespace dev {

// Byte offset of the Lambda word of an edge {4 c Z, 4 s} for row i (given as 4 i):
// 4 (c Z + (i + s) mod Z), with the wrap done as an unsigned minimum (i + s < 2Z
// since s < Z).  Virtual edges carry {4 n, 0} and map row i to its dummy slot n + i.
__device__ __forceinline__ uint32_t qc_off(int2 e, uint32_t i4, uint32_t Z4) {
    const uint32_t x = i4 + (uint32_t)e.y;
    return (uint32_t)e.x + min(x, x - Z4);
}

__device__ __forceinline__ uint32_t &lds_word(uint32_t *base, uint32_t off) {
    return *(uint32_t *)((char *)base + off);
}

// (M & a) | (~M & b) (one v_bfi_b32).
__device__ __forceinline__ uint32_t bfi(uint32_t M, uint32_t a, uint32_t b) { return (M & a) | (~M & b); }

// Dummy slot contents for virtual edges: +16383 in both halves.  Minus any check
// message (|r| <= 127) it stays positive and above msg_max, so a virtual edge
// always enters its check with magnitude msg_max and sign +, which never changes
// the two smallest magnitudes (real ones are <= msg_max) or the sign parity, and
// its decision bit is 0 for the parity test.
constexpr uint32_t kDummy = 0x3FFF3FFFu;

// LDS of a QC workgroup: [ML][MD] layer descriptors; [ML][Z] rows of 8 16-bit byte
// offsets of the rows' Lambda words (one 16-byte LDS read per row and layer instead of
// the index arithmetic of every edge); [npairs][ld] packed Lambda; in flooding
// [npairs][ld] packed channel LLRs; then the pairs' parity flags and done bits and the
// [2 npairs] iteration counts.
struct QcLds {
    int2 *sdesc;
    uint16_t *offs;
    uint32_t *lam, *Lch;
    int *unsat, *done, *itc;
};

template <int ML, int MD>
__device__ __forceinline__ QcLds qc_lds(uint32_t *lds, int Z, int npairs, int ld, bool layered) {
    QcLds S;
    S.sdesc = (int2 *)lds;
    S.offs = (uint16_t *)(lds + 2 * ML * MD);
    S.lam = lds + 2 * ML * MD + 4 * ML * Z;
    S.Lch = S.lam + (size_t)npairs * ld;
    S.unsat = (int *)(S.lam + (size_t)(layered ? 1 : 2) * npairs * ld);
    S.done = S.unsat + npairs;
    S.itc = S.done + npairs;
    return S;
}

// Staging of codewords [cw0, cw0 + 2 npairs): layer descriptors and row offsets, Lambda
// (and in flooding its channel copy) from the input LLRs with +16383 in the dummy slots
// of virtual edges, cleared flags (codewords past the batch count as done).  Ends with
// a barrier.
template <int ML, int MD>
__device__ __forceinline__ void qc_stage(const QcLds &S, const QcDesc &Q, const DevCode &C, const DecodeIO &io,
                                         int batch, int npairs, int cw0, int ld, bool layered) {
    const int n = C.n, Z = Q.Z, nl = Q.nl;
    const uint32_t Z4 = 4 * Z;
    const int tid = threadIdx.x, T = blockDim.x;
    for (int idx = tid; idx < ML * MD; idx += T) {
        const int l = idx / MD, j = idx - l * MD;
        const int2 e = (l < nl && j < Q.dc[l]) ? Q.edges[l * kQcMaxDc + j] : make_int2(n, 0);
        S.sdesc[idx] = make_int2(4 * e.x, 4 * e.y);
    }
    __syncthreads();
    for (int idx = tid; idx < ML * Z; idx += T) {
        const int l = idx / Z, i = idx - l * Z;
        uint16_t *o = S.offs + 8 * idx;
#pragma unroll
        for (int j = 0; j < 8; ++j) o[j] = j < MD ? (uint16_t)qc_off(S.sdesc[l * MD + j], 4 * i, Z4) : (uint16_t)0;
    }
    const int8_t *llr = (const int8_t *)io.llr;
    for (int idx = tid; idx < npairs * ld; idx += T) {
        const int pp = idx / ld, v = idx - pp * ld;
        const int c0 = cw0 + 2 * pp;
        short lo = 0x3FFF, hi = 0x3FFF;
        if (v < n) {
            lo = c0 < batch ? (short)llr[(size_t)c0 * n + v] : (short)0;
            hi = c0 + 1 < batch ? (short)llr[(size_t)(c0 + 1) * n + v] : (short)0;
        }
        const uint32_t w = as_u32((v2s){lo, hi});
        S.lam[idx] = w;
        if (!layered) S.Lch[idx] = w;
    }
    for (int idx = tid; idx < npairs; idx += T) {
        const int c0 = cw0 + 2 * idx;
        S.unsat[idx] = 0;
        S.done[idx] = (c0 < batch ? 0 : 1) | (c0 + 1 < batch ? 0 : 2);
        S.itc[2 * idx] = S.itc[2 * idx + 1] = 0;
    }
    __syncthreads();
}

// Outputs once the final syndrome is in the flags: ok and iteration counts, the packed
// hard decisions and, with the debug dump, Lambda (the per-edge messages are the
// caller's).
__device__ __forceinline__ void qc_outputs(const QcLds &S, const DecodeIO &io, int n, int batch, int npairs, int cw0,
                                           int ld) {
    const int tid = threadIdx.x, T = blockDim.x;
    const int ncw = min(2 * npairs, batch - cw0);
    if (tid < ncw) {
        io.ok[cw0 + tid] = ((S.unsat[tid >> 1] >> (tid & 1)) & 1) ? 0 : 1;
        io.iters[cw0 + tid] = (int16_t)S.itc[tid];
    }
    const int nbytes = (n + 7) >> 3;
    uint8_t *hard = (uint8_t *)io.hard + (size_t)cw0 * nbytes;
    for (int idx = tid; idx < ncw * nbytes; idx += T) {
        const int c = idx / nbytes, jb = idx - c * nbytes;
        const uint32_t *lp = S.lam + (size_t)(c >> 1) * ld;
        const int sh = (c & 1) ? 31 : 15;
        uint32_t byte = 0;
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const int v = 8 * jb + b;
            if (v < n) byte |= ((lp[v] >> sh) & 1u) << b;
        }
        hard[idx] = (uint8_t)byte;
    }
    if (io.dump_a) {
        int16_t *dl = (int16_t *)io.dump_c;
        for (int idx = tid; idx < ncw * n; idx += T) {
            const int c = idx / n, v = idx - c * n;
            dl[(size_t)(cw0 + c) * n + v] = as_v2s(S.lam[(size_t)(c >> 1) * ld + v])[c & 1];
        }
    }
}

// Decode codewords [2 npairs blk, 2 npairs (blk + 1)) with the calling workgroup.
// Threads beyond Z * npairs take part in the barriers only.  Ends with a barrier,
// so the caller may reuse the LDS right after.  ES = false compiles the early-stop
// logic out (only valid with early_stop == 0).
template <int ML, int MD, bool LAYERED, bool ES = true>
__device__ __forceinline__ void qc_item(const QcDesc &Q, const DevCode &C, const BinRule &R, int max_iters, int early_stop, int batch,
                        int npairs, const DecodeIO &io, int blk, uint32_t *lds) {
    const int n = C.n, E = C.E, Z = Q.Z, nl = Q.nl;
    const int ld = n + Z;  // per-pair Lambda row: n variables + Z dummy slots
    const uint32_t Z4 = 4 * Z;
    const int tid = threadIdx.x, T = blockDim.x;
    const bool act = tid < Z * npairs;
    const int p = act ? tid / Z : 0, i0 = act ? tid - p * Z : 0;
    const int cw0 = blk * npairs * 2;
    if (cw0 >= batch) return;
    const QcLds S = qc_lds<ML, MD>(lds, Z, npairs, ld, LAYERED);
    uint16_t *offs = S.offs;
    uint32_t *lam = S.lam, *Lch = S.Lch;
    int *unsat = S.unsat, *done = S.done, *itc = S.itc;
    const v2s mm = splat(R.msg_max), nmm = splat(-R.msg_max);
    const PkNorm NP = pk_norm_params(R);
    int rule = __builtin_amdgcn_readfirstlane(R.rule);  // uniform: scalar branches below
    asm volatile("" : "+s"(rule));
    // -128 in both halves, opaque to the compiler so that a * -128 + c stays one
    // v_pk_mad_u16 instead of a shift and a subtraction
    int kn128 = (int)0xFF80FF80u;
    asm volatile("" : "+s"(kn128));
    const v2s neg128 = as_v2s((uint32_t)kn128);
    // f1 = f(m1), f2 = f(m2) for the rule (each branch exact for its rule)
    auto norm2 = [&](v2s m1, v2s m2, v2s &f1, v2s &f2) {
        if (rule == LDPCX_RULE_NMS) {
            f1 = (m1 * NP.num) >> NP.shift;
            f2 = (m2 * NP.num) >> NP.shift;
        } else if (rule == LDPCX_RULE_OMS) {
            f1 = pmax(m1 - NP.off, splat(0));
            f2 = pmax(m2 - NP.off, splat(0));
        } else {
            f1 = m1;
            f2 = m2;
        }
    };

    qc_stage<ML, MD>(S, Q, C, io, batch, npairs, cw0, ld, LAYERED);
    // Flooding adds every layer's messages to Lambda at once with 32-bit LDS atomic adds
    // on the packed pair; Lambda's low halves (and the channel copy's) are kept offset by
    // 2^15 meanwhile so that the carry between the halves is exact (as in qc_item_lp).
    constexpr uint32_t kB = LAYERED ? 0u : 0x8000u;
    if (!LAYERED) {
        for (int idx = tid; idx < npairs * ld; idx += T) {
            lam[idx] ^= kB;
            Lch[idx] ^= kB;
        }
        __syncthreads();
    }

    v2s r[ML][MD];
#pragma unroll
    for (int l = 0; l < ML; ++l)
#pragma unroll
        for (int j = 0; j < MD; ++j) r[l][j] = splat(0);

    uint32_t *lamp = lam + (size_t)p * ld;
    // byte offsets of this thread's row in layer l
    auto row_offs = [&](int l, uint32_t (&vv)[MD]) {
        const uint4 w = *(const uint4 *)(offs + 8 * (l * Z + i0));
        const uint32_t ws[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
        for (int j = 0; j < MD; ++j) vv[j] = (j & 1) ? ws[j >> 1] >> 16 : ws[j >> 1] & 0xFFFFu;
    };

    // Parity of the current hard decisions of this thread's rows, as a 2-bit mask
    // (one bit per codeword); virtual edges read a dummy slot whose sign bits are 0.
    auto row_parities = [&]() -> int {
        int any = 0;
        if (!act) return 0;
#pragma unroll
        for (int l = 0; l < ML; ++l) {
            if (l < nl) {
                uint32_t vv[MD];
                row_offs(l, vv);
                uint32_t x = (MD & 1) ? kB : 0u;  // each word's low sign bit is flipped by the offset
#pragma unroll
                for (int j = 0; j < MD; ++j) x ^= lds_word(lamp, vv[j]);
                any |= (int)((x >> 15) & 1u) | (int)((x >> 30) & 2u);
            }
        }
        return any;
    };

    uint32_t M = 0xFFFFFFFFu;  // halves (codewords) still being decoded
    for (int k = 1; k <= max_iters; ++k) {
        if (ES && early_stop) {
            const int any = row_parities();
            if (any) atomicOr(&unsat[p], any);
            __syncthreads();
            if (tid < npairs) {
                done[tid] |= (~unsat[tid]) & 3;
                unsat[tid] = 0;
            }
            __syncthreads();
            int all = 1;
            for (int q = 0; q < npairs; ++q) all &= done[q] == 3;
            if (all) break;
            const int d = done[p];
            M = ((d & 1) ? 0u : 0x0000FFFFu) | ((d & 2) ? 0u : 0xFFFF0000u);
        }
#pragma unroll
        for (int l = 0; l < ML; ++l) {
            if (l < nl) {
              if (act) {
                int dc = __builtin_amdgcn_readfirstlane(Q.dc[l]);  // uniform by construction
                asm volatile("" : "+s"(dc));
                // One straight-line body per layer-degree class, with DD edge slots (slots at
                // or beyond the degree run as virtual edges).  Each step runs over all the
                // slots before the next starts, so that the dependent packed operations of
                // one edge are separated by those of the others (no hazard wait states).
                auto layer = [&](auto dd_tag) {
                    constexpr int DD = decltype(dd_tag)::value;
                    uint32_t vv[MD], sv[MD], sr[MD];
                    v2s qv[MD], nq[MD], av[MD], mg[MD];
                    row_offs(l, vv);
#pragma unroll
                    for (int j = 0; j < DD; ++j) qv[j] = as_v2s(lds_word(lamp, vv[j]) ^ kB) - r[l][j];
                    // |clamp(q, +-msg_max)| = min(|q|, msg_max); the sign of q is the sign of clamp(q)
#pragma unroll
                    for (int j = 0; j < DD; ++j) nq[j] = -qv[j];
#pragma unroll
                    for (int j = 0; j < DD; ++j) sv[j] = as_u32(qv[j] >> splat(15));
#pragma unroll
                    for (int j = 0; j < DD; ++j) av[j] = pmax(qv[j], nq[j]);
#pragma unroll
                    for (int j = 0; j < DD; ++j) av[j] = pmin(av[j], mm);
                    v2s m1 = splat(0x7FFF), m2 = splat(0x7FFF);
                    uint32_t stot = 0;
#pragma unroll
                    for (int j = 0; j < DD; ++j) {
                        m2 = pmin(m2, pmax(m1, av[j]));
                        m1 = pmin(m1, av[j]);
                        stot ^= sv[j];
                    }
                    v2s f1, f2;
                    norm2(m1, m2, f1, f2);
                    // Magnitude out of edge j: f2 where the edge holds the minimum (a = m1), else
                    // f1.  With all magnitudes in [0, 127] and 128 >= f2 - f1, that is
                    // max(f1, f2 + 128 (m1 - a)), exact in 16 bits (the sum lies in [-16256, 16383]).
                    const v2s cs = f2 - m1 * neg128;
#pragma unroll
                    for (int j = 0; j < DD; ++j) mg[j] = av[j] * neg128 + cs;
#pragma unroll
                    for (int j = 0; j < DD; ++j) sr[j] = stot ^ sv[j];
#pragma unroll
                    for (int j = 0; j < DD; ++j) mg[j] = pmax(f1, mg[j]);
#pragma unroll
                    for (int j = 0; j < DD; ++j) mg[j] = as_v2s(as_u32(mg[j]) ^ sr[j]);
#pragma unroll
                    for (int j = 0; j < DD; ++j) {
                        const v2s rn = mg[j] - as_v2s(sr[j]);
                        r[l][j] = ES ? as_v2s(bfi(M, as_u32(rn), as_u32(r[l][j]))) : rn;
                    }
                    if (LAYERED) {
#pragma unroll
                        for (int j = 0; j < DD; ++j) lds_word(lamp, vv[j]) = as_u32(qv[j] + r[l][j]);
                        // virtual edges wrote q + r into their dummy slot: restore it
                        if (dc < DD) lamp[n + i0] = kDummy;
                    }
                };
                if (dc >= MD) layer(std::integral_constant<int, MD>{});
                else if (dc == MD - 1) layer(std::integral_constant<int, MD - 1>{});
                else layer(std::integral_constant<int, MD - 2>{});
              }
                if (LAYERED) __syncthreads();
            }
        }
        if (!LAYERED) {
            __syncthreads();
            for (int idx = tid; idx < npairs * ld; idx += T) lam[idx] = Lch[idx];
            __syncthreads();
            if (act) {
#pragma unroll
                for (int l = 0; l < ML; ++l) {
                    if (l < nl) {
                        const int dc = Q.dc[l];
                        uint32_t vv[MD];
                        row_offs(l, vv);
#pragma unroll
                        for (int j = 0; j < MD; ++j) {
                            if (j < dc) {
                                const uint32_t d = as_u32(r[l][j]);
                                atomicAdd(&lds_word(lamp, vv[j]), d - ((d & 0x8000u) << 1));
                            }
                        }
                    }
                }
            }
            __syncthreads();
        }
        if (tid < 2 * npairs && !((done[tid >> 1] >> (tid & 1)) & 1)) itc[tid] = k;
    }

    // Syndrome of the final decision (then Lambda back to plain packed int16).
    __syncthreads();
    {
        const int any = row_parities();
        if (any) atomicOr(&unsat[p], any);
    }
    __syncthreads();
    if (!LAYERED) {
        for (int idx = tid; idx < npairs * ld; idx += T) lam[idx] ^= kB;
        __syncthreads();
    }
    if (io.dump_a) {
        int8_t *dq = (int8_t *)io.dump_a;
        int8_t *dr = (int8_t *)io.dump_b;
        const int i = i0;
#pragma unroll
        for (int l = 0; l < ML; ++l) {
            if (act && l < nl) {
                const int e0 = C.row_ptr[l * Z + i];
#pragma unroll
                for (int j = 0; j < MD; ++j)
                    if (j < Q.dc[l]) {
                        const v2s lv = as_v2s(lds_word(lamp, qc_off(S.sdesc[l * MD + j], 4 * i, Z4)));
                        const v2s qc = pmin(pmax(lv - r[l][j], nmm), mm);
                        for (int h = 0; h < 2; ++h) {
                            const int c = cw0 + 2 * p + h;
                            if (c < batch) {
                                dr[(size_t)c * E + e0 + j] = (int8_t)r[l][j][h];
                                dq[(size_t)c * E + e0 + j] = (int8_t)qc[h];
                            }
                        }
                    }
            }
        }
    }
    qc_outputs(S, io, n, batch, npairs, cw0, ld);
    __syncthreads();
}

// Flooding with the layers in parallel: thread (layer l, pair, row i) owns row i of layer l
// only, so a workgroup of Z * npairs * nl threads runs every check node of an iteration at
// once (nl times the waves of qc_item, each with one layer's messages in registers).
// Z * npairs is a multiple of 64, so a wave holds rows of one layer and the layer degree
// is uniform in it.  The variable-node update adds each edge's change r_new - r_old to
// Lambda in place (Lambda_old + sum (r_new - r_old) = L + sum r_new, exactly), every layer
// at once, with 32-bit LDS atomic adds on the packed pair.  For the carry out of the low
// half to be right, the low halves of Lambda are kept offset by 2^15 (x ^ 0x8000, always
// in [0, 65535] since Lambda is exact in int16) while the iterations run: adding the
// unsigned low half of a delta then carries out exactly when the delta is negative, and
// the high half of the addend is lowered by that carry.  One barrier after the check
// nodes and one after the adds per iteration.  LDS layout of qc_item's layered schedule.
template <int ML, int MD, bool ES>
__device__ __forceinline__ void qc_item_lp(const QcDesc &Q, const DevCode &C, const BinRule &R, int max_iters,
                                           int early_stop, int batch, int npairs, const DecodeIO &io, int blk,
                                           uint32_t *lds) {
    const int n = C.n, E = C.E, Z = Q.Z, nl = Q.nl;
    const int ld = n + Z;
    const int tid = threadIdx.x, T = blockDim.x;
    const int per = Z * npairs;                       // threads of one layer
    const int lt = tid / per, rem = tid - lt * per;   // this thread's layer
    const bool act = lt < nl;
    const int p = act ? rem / Z : 0, i0 = act ? rem - p * Z : 0;
    const int cw0 = blk * npairs * 2;
    if (cw0 >= batch) return;
    const QcLds S = qc_lds<ML, MD>(lds, Z, npairs, ld, true);
    uint16_t *offs = S.offs;
    uint32_t *lam = S.lam;
    int *unsat = S.unsat, *done = S.done, *itc = S.itc;
    const v2s mm = splat(R.msg_max), nmm = splat(-R.msg_max);
    const PkNorm NP = pk_norm_params(R);
    int rule = __builtin_amdgcn_readfirstlane(R.rule);
    asm volatile("" : "+s"(rule));
    int kn128 = (int)0xFF80FF80u;  // -128 in both halves, opaque (one v_pk_mad_u16 below)
    asm volatile("" : "+s"(kn128));
    const v2s neg128 = as_v2s((uint32_t)kn128);
    constexpr uint32_t kBias = 0x8000u;  // offset of Lambda's low halves during the iterations

    qc_stage<ML, MD>(S, Q, C, io, batch, npairs, cw0, ld, true);
    for (int idx = tid; idx < npairs * ld; idx += T) lam[idx] ^= kBias;
    __syncthreads();

    uint32_t *lamp = lam + (size_t)p * ld;
    uint32_t vv[MD];
    int dc = 0;
    if (act) {
        const uint4 w = *(const uint4 *)(offs + 8 * (lt * Z + i0));
        const uint32_t ws[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
        for (int j = 0; j < MD; ++j) vv[j] = (j & 1) ? ws[j >> 1] >> 16 : ws[j >> 1] & 0xFFFFu;
        dc = Q.dc[lt];
    }
    dc = __builtin_amdgcn_readfirstlane(dc);  // uniform: a wave holds rows of one layer
    asm volatile("" : "+s"(dc));
    v2s r[MD], dr[MD];  // the row's messages and their change in this iteration
#pragma unroll
    for (int j = 0; j < MD; ++j) r[j] = dr[j] = splat(0);

    // parity of this thread's row under the current decisions (2 bits, one per codeword);
    // each of the MD words carries the offset's flipped low sign bit
    auto row_parity = [&]() -> int {
        if (!act) return 0;
        uint32_t x = (MD & 1) ? kBias : 0u;
#pragma unroll
        for (int j = 0; j < MD; ++j) x ^= lds_word(lamp, vv[j]);
        return (int)((x >> 15) & 1u) | (int)((x >> 30) & 2u);
    };
    // check node of this thread's row: DD edge slots (those at or beyond dc are virtual)
    uint32_t M = 0xFFFFFFFFu;
    auto check = [&](auto dd_tag) {
        constexpr int DD = decltype(dd_tag)::value;
        uint32_t sv[MD], sr[MD];
        v2s qv[MD], nq[MD], av[MD], mg[MD];
#pragma unroll
        for (int j = 0; j < DD; ++j) qv[j] = as_v2s(lds_word(lamp, vv[j]) ^ kBias) - r[j];
#pragma unroll
        for (int j = 0; j < DD; ++j) nq[j] = -qv[j];
#pragma unroll
        for (int j = 0; j < DD; ++j) sv[j] = as_u32(qv[j] >> splat(15));
#pragma unroll
        for (int j = 0; j < DD; ++j) av[j] = pmax(qv[j], nq[j]);
#pragma unroll
        for (int j = 0; j < DD; ++j) av[j] = pmin(av[j], mm);
        v2s m1 = splat(0x7FFF), m2 = splat(0x7FFF);
        uint32_t stot = 0;
#pragma unroll
        for (int j = 0; j < DD; ++j) {
            m2 = pmin(m2, pmax(m1, av[j]));
            m1 = pmin(m1, av[j]);
            stot ^= sv[j];
        }
        v2s f1, f2;
        if (rule == LDPCX_RULE_NMS) {
            f1 = (m1 * NP.num) >> NP.shift;
            f2 = (m2 * NP.num) >> NP.shift;
        } else if (rule == LDPCX_RULE_OMS) {
            f1 = pmax(m1 - NP.off, splat(0));
            f2 = pmax(m2 - NP.off, splat(0));
        } else {
            f1 = m1;
            f2 = m2;
        }
        // magnitude out of edge j: f2 where a = m1, else f1 (as in qc_item)
        const v2s cs = f2 - m1 * neg128;
#pragma unroll
        for (int j = 0; j < DD; ++j) mg[j] = av[j] * neg128 + cs;
#pragma unroll
        for (int j = 0; j < DD; ++j) sr[j] = stot ^ sv[j];
#pragma unroll
        for (int j = 0; j < DD; ++j) mg[j] = pmax(f1, mg[j]);
#pragma unroll
        for (int j = 0; j < DD; ++j) mg[j] = as_v2s(as_u32(mg[j]) ^ sr[j]);
#pragma unroll
        for (int j = 0; j < DD; ++j) {
            v2s rn = mg[j] - as_v2s(sr[j]);
            if (ES) rn = as_v2s(bfi(M, as_u32(rn), as_u32(r[j])));
            dr[j] = rn - r[j];
            r[j] = rn;
        }
    };

    for (int k = 1; k <= max_iters; ++k) {
        if (ES && early_stop) {
            const int any = row_parity();
            if (any) atomicOr(&unsat[p], any);
            __syncthreads();
            if (tid < npairs) {
                done[tid] |= (~unsat[tid]) & 3;
                unsat[tid] = 0;
            }
            __syncthreads();
            int all = 1;
            for (int q = 0; q < npairs; ++q) all &= done[q] == 3;
            if (all) break;
            const int d = done[p];
            M = ((d & 1) ? 0u : 0x0000FFFFu) | ((d & 2) ? 0u : 0xFFFF0000u);
        }
        if (act) {
            if (dc >= MD) check(std::integral_constant<int, MD>{});
            else if (dc == MD - 1) check(std::integral_constant<int, MD - 1>{});
            else check(std::integral_constant<int, MD - 2>{});
        }
        __syncthreads();  // every check node has read Lambda
        if (act) {
#pragma unroll
            for (int j = 0; j < MD; ++j) {
                if (j < dc) {
                    const uint32_t d = as_u32(dr[j]);
                    atomicAdd(&lds_word(lamp, vv[j]), d - ((d & 0x8000u) << 1));
                }
            }
        }
        __syncthreads();
        if (tid < 2 * npairs && !((done[tid >> 1] >> (tid & 1)) & 1)) itc[tid] = k;
    }

    // Syndrome of the final decision, then Lambda back to plain packed int16.
    __syncthreads();
    {
        const int any = row_parity();
        if (any) atomicOr(&unsat[p], any);
    }
    __syncthreads();
    for (int idx = tid; idx < npairs * ld; idx += T) lam[idx] ^= kBias;
    __syncthreads();
    if (io.dump_a) {
        int8_t *dq = (int8_t *)io.dump_a;
        int8_t *dr = (int8_t *)io.dump_b;
        if (act) {
            const int e0 = C.row_ptr[lt * Z + i0];
#pragma unroll
            for (int j = 0; j < MD; ++j)
                if (j < dc) {
                    const v2s lv = as_v2s(lds_word(lamp, vv[j]));
                    const v2s qc = pmin(pmax(lv - r[j], nmm), mm);
                    for (int h = 0; h < 2; ++h) {
                        const int c = cw0 + 2 * p + h;
                        if (c < batch) {
                            dr[(size_t)c * E + e0 + j] = (int8_t)r[j][h];
                            dq[(size_t)c * E + e0 + j] = (int8_t)qc[h];
                        }
                    }
                }
        }
    }
    qc_outputs(S, io, n, batch, npairs, cw0, ld);
    __syncthreads();
}

// Register arrays are sized by the number of layers (ML) and the largest layer degree (MD).
#define LDPCX_QC_SHAPES(X) X(4, 6) X(4, 8) X(8, 6) X(8, 8) X(12, 7) X(12, 8) X(16, 6) X(16, 8)

inline void qc_shape_of(const QcDesc &Q, int &ml, int &md) {
    int d = 0;
    for (int l = 0; l < Q.nl; ++l) d = Q.dc[l] > d ? Q.dc[l] : d;
    ml = md = 0;
#define LDPCX_PICK(L_, D_)              \
    if (!ml && Q.nl <= L_ && d <= D_) { \
        ml = L_;                        \
        md = D_;                        \
    }
    LDPCX_QC_SHAPES(LDPCX_PICK)
#undef LDPCX_PICK
}

inline size_t qc_smem_bytes(int ML, int MD, const DevCode &C, int Z, int layered, int npairs) {
    return sizeof(int2) * ML * MD + (size_t)ML * Z * 16 + (size_t)(layered ? 1 : 2) * npairs * (C.n + Z) * 4 +
           (size_t)npairs * 16;
}

}  // namespace dev
}  // namespace ldpcx
