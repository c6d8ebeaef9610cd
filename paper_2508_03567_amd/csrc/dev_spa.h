// Fixed-point FFT-SPA decoder (Alg. 1) for fields up to GF(256), as wave-level device
// functions (GF(128) and GF(256) for check and variable degrees up to 4).
//
// Arithmetic: probabilities in Q24 (2^24 = 1); the transform of eq. (3) over GF(2^q)
// is the Walsh-Hadamard transform, exact in 32-bit integers (the inverse in 64 bits
// above GF(64), where its sums reach g 2^24); products of two Q24
// numbers are floor((a b + 2^23) / 2^24), taken in ascending edge order; the inverse
// transform is followed by a floor division by g and a clamp at 0; a vector z is
// normalised (eq. (6)) as floor((z(x) R + 2^21) / 2^22) with R = floor(2^46 / sum z);
// channel vectors come from the symbol costs gamma through the weights
// W(c) = round(2^24 exp(-c / 4)).
//
// Mapping: a wavefront covers 64 / S codewords of one node, a segment of S lanes per
// codeword (S = 4, 8 or 16, at most g, chosen per kernel from the degree bound: the
// more entries a lane holds, the more butterflies stay in registers, but the more
// registers each message takes, which costs occupancy beyond 4 entries); lane j of a segment holds the
// R = g / S consecutive entries x = j R .. j R + R - 1.  The transform runs its
// butterflies over the register bits in registers and over the lane bits with DPP
// moves inside a row of 16 lanes (quad_perm for directions 1 and 2, row_half_mirror
// for direction 7, row_ror:8 for direction 8).  Directions {1, 2, 7, 8} span the lane
// index space, so with each butterfly's sign taken from the dual basis (j0^j2, j1^j2,
// j2, j3; j0, j1 for S = 4) the lane part is the Walsh-Hadamard transform in linearly
// relabelled coordinates: the transformed values are those of the plain transform at
// fixed permuted positions, the elementwise products see the same integer pairs, and
// forward then inverse gives exactly g times the XOR convolution in the original
// index.  Segment sums, maxima and the arg-max reduce over the same directions.  The
// permutation by the edge coefficient is folded into the check node's loads (gather)
// and the depermutation into its stores (scatter to the same positions).  Messages
// are stored codeword-major per edge, [edge][codeword][x] (int32), whatever S is.
// Products that share a leading run of factors (ascending order) are computed once.
#pragma once

#include "dev_common.h"

namespace ldpcx {
namespace dev {
namespace spa {

constexpr int kQ = 24;
constexpr int kVnRegs = 16;  // largest variable degree (its incoming messages stay in registers)

struct Args {
    DevCode C;
    int max_iters, early_stop, batch;
    SpaWork w;
    DecodeIO io;
};

// Lanes per codeword for a kernel whose register arrays hold D messages: up to 4
// entries per lane for degrees up to 4, fewer above.
template <int G, int D>
constexpr int lanes_for() {
    return D <= 4 ? (G / 4 > 16 ? 16 : (G / 4 > 4 ? G / 4 : 4)) : (G < 16 ? G : 16);
}

// Entries per lane, codewords per wave, log2(g).
template <int G, int S>
struct Geo {
    static_assert(S == 4 || S == 8 || S == 16, "segments of 4, 8 or 16 lanes");
    static constexpr int R = G / S;
    static constexpr int CPW = 64 / S;
    static constexpr int P = G == 256 ? 8 : G == 128 ? 7 : G == 64 ? 6 : G == 32 ? 5 : G == 16 ? 4 : G == 8 ? 3 : 2;
};

__device__ __forceinline__ int qmul(int a, int b) {
    return (int)(((long long)a * b + (1ll << (kQ - 1))) >> kQ);
}

// floor(2^46 / s) for 0 < s < 2^33: the double quotient is within one unit of the
// exact one (its error is far below 1 for quotients < 2^47), and two integer checks
// make it exact.
__device__ __forceinline__ long long recip46(long long s) {
    long long q = (long long)(70368744177664.0 / (double)s);
    if (q * s > (1ll << 46)) --q;
    if ((q + 1) * s <= (1ll << 46)) ++q;
    return q;
}

// DPP move of v inside each row of 16 lanes; every control used reads a lane of the
// same row, so no lane is out of bounds and the move needs no old value.
template <int CTRL>
__device__ __forceinline__ int dpp(int v) {
    return __builtin_amdgcn_mov_dpp(v, CTRL, 0xF, 0xF, true);
}
constexpr int kDppXor1 = 0xB1;      // quad_perm [1,0,3,2]
constexpr int kDppXor2 = 0x4E;      // quad_perm [2,3,0,1]
constexpr int kDppMirror8 = 0x141;  // row_half_mirror: j -> j ^ 7 inside 8 lanes
constexpr int kDppRor8 = 0x128;     // row_ror:8: j -> j ^ 8 inside 16 lanes

// Butterfly signs of the lane directions 1, 2, 7, 8 (the dual basis of the lane index)
// as masks (-1 on the lane that takes the difference, 0 on the one that takes the sum),
// and the per-lane constant the xor form of the lane stages leaves behind.
struct Signs {
    int d1, d2, d7, d8, corr;
};

// One lane stage in two VALU operations: o + (v ^ mask) is o + v on a sum lane and
// o - v - 1 on a difference lane.  The stages are affine with a data-independent
// offset, so the transform of x comes out as T(x) + T'(0); wht subtracts corr = T'(0).
template <int CTRL, int R>
__device__ __forceinline__ void lane_stage(int (&v)[R], int mask) {
#pragma unroll
    for (int r = 0; r < R; ++r) v[r] = dpp<CTRL>(v[r]) + (v[r] ^ mask);
}

template <int S, int R>
__device__ __forceinline__ void lane_stages(int (&v)[R], const Signs &sg) {
    lane_stage<kDppXor1>(v, sg.d1);
    lane_stage<kDppXor2>(v, sg.d2);
    if (S >= 8) lane_stage<kDppMirror8>(v, sg.d7);
    if (S >= 16) lane_stage<kDppRor8>(v, sg.d8);
}

template <int S>
__device__ __forceinline__ Signs signs_of(int j) {
    Signs s;
    if (S >= 8) {
        s.d1 = -((j ^ (j >> 2)) & 1);
        s.d2 = -(((j >> 1) ^ (j >> 2)) & 1);
        s.d7 = -((j >> 2) & 1);
        s.d8 = -((j >> 3) & 1);
    } else {
        s.d1 = -(j & 1);
        s.d2 = -((j >> 1) & 1);
        s.d7 = s.d8 = 0;
    }
    int z[1] = {0};
    s.corr = 0;
    lane_stages<S>(z, s);
    s.corr = z[0];
    return s;
}

// DPP move of a 64-bit value (both halves through the same control).
template <int CTRL>
__device__ __forceinline__ long long dpp64(long long v) {
    const int lo = dpp<CTRL>((int)(uint32_t)v), hi = dpp<CTRL>((int)(v >> 32));
    return (long long)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

template <int CTRL, int R>
__device__ __forceinline__ void lane_stage64(long long (&v)[R], int mask) {
#pragma unroll
    for (int r = 0; r < R; ++r) v[r] = dpp64<CTRL>(v[r]) + (v[r] ^ (long long)mask);
}

// The same transform in 64 bits (for the inverse above GF(64)); the per-lane constant of
// the lane stages is the same small integer as in 32 bits.
template <int S, int R>
__device__ __forceinline__ void wht64(long long (&v)[R], const Signs &sg) {
#pragma unroll
    for (int s = 1; s < R; s <<= 1) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
            if (!(r & s)) {
                const long long a = v[r], b = v[r | s];
                v[r] = a + b;
                v[r | s] = a - b;
            }
        }
    }
    lane_stage64<kDppXor1>(v, sg.d1);
    lane_stage64<kDppXor2>(v, sg.d2);
    if (S >= 8) lane_stage64<kDppMirror8>(v, sg.d7);
    if (S >= 16) lane_stage64<kDppRor8>(v, sg.d8);
#pragma unroll
    for (int r = 0; r < R; ++r) v[r] -= (long long)sg.corr;
}

// Walsh-Hadamard transform of the segment (relabelled in the lane bits, see above).
template <int S, int R>
__device__ __forceinline__ void wht(int (&v)[R], const Signs &sg) {
#pragma unroll
    for (int s = 1; s < R; s <<= 1) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
            if (!(r & s)) {
                const int a = v[r], b = v[r | s];
                v[r] = a + b;
                v[r | s] = a - b;
            }
        }
    }
    lane_stages<S>(v, sg);
#pragma unroll
    for (int r = 0; r < R; ++r) v[r] -= sg.corr;
}

template <int S>
__device__ __forceinline__ int seg_sum(int v) {
    v += dpp<kDppXor1>(v);
    v += dpp<kDppXor2>(v);
    if (S >= 8) v += dpp<kDppMirror8>(v);
    if (S >= 16) v += dpp<kDppRor8>(v);
    return v;
}

// Segment sum of per-lane values below 2^31 whose total may exceed 32 bits.
template <int S>
__device__ __forceinline__ long long seg_sum64(int v) {
    long long s = v;
    s += dpp64<kDppXor1>(s);
    s += dpp64<kDppXor2>(s);
    if (S >= 8) s += dpp64<kDppMirror8>(s);
    if (S >= 16) s += dpp64<kDppRor8>(s);
    return s;
}

template <int S>
__device__ __forceinline__ int seg_max(int v) {
    v = max(v, dpp<kDppXor1>(v));
    v = max(v, dpp<kDppXor2>(v));
    if (S >= 8) v = max(v, dpp<kDppMirror8>(v));
    if (S >= 16) v = max(v, dpp<kDppRor8>(v));
    return v;
}

// out = norm(z) for this lane's entries; `fallback` when the segment sum is 0.
template <int S, int R>
__device__ __forceinline__ void normalise(const int (&z)[R], const int (&fallback)[R], int (&out)[R]) {
    int ls = 0;
#pragma unroll
    for (int r = 0; r < R; ++r) ls += z[r];
    // up to GF(64) the segment sum stays below 2^31; above it can reach g 2^24 (channel
    // vectors with many equal costs) and is taken in 64 bits
    long long s;
    if constexpr (S * R > 64) s = seg_sum64<S>(ls);
    else s = seg_sum<S>(ls);
    if (s <= 0) {
#pragma unroll
        for (int r = 0; r < R; ++r) out[r] = fallback[r];
        return;
    }
    const long long q = recip46(s);
#pragma unroll
    for (int r = 0; r < R; ++r) out[r] = (int)(((long long)z[r] * q + (1ll << 21)) >> 22);
}

// Arg-max over the segment with the lowest x on ties (values < 2^25); x0 = this
// lane's first entry.
template <int S, int R>
__device__ __forceinline__ int seg_argmax(const int (&val)[R], int x0) {
    if constexpr (S * R > 64) {
        // above GF(64) the symbol no longer fits beside the value in 32 bits: the maximum
        // first, then the lowest x holding it
        int m = val[0];
#pragma unroll
        for (int r = 1; r < R; ++r) m = max(m, val[r]);
        m = seg_max<S>(m);
        int x = S * R;
#pragma unroll
        for (int r = R - 1; r >= 0; --r)
            if (val[r] == m) x = x0 + r;
        return -seg_max<S>(-x);
    }
    int key = val[0] * 64 + (63 - x0);
#pragma unroll
    for (int r = 1; r < R; ++r) key = max(key, val[r] * 64 + (63 - x0 - r));
    key = seg_max<S>(key);
    return 63 - (key & 63);
}

__host__ __device__ inline size_t row(int node, int b, int batch, int g) { return ((size_t)node * batch + b) * g; }

__device__ __forceinline__ bool active(const Args &A, int k, int b) {
    return b < A.batch && (!A.early_stop || A.w.unsat[(size_t)k * A.batch + b]);
}

// Lane geometry of wave `unit` = (node, group of 64 / S codewords).
struct Lane {
    int node, b, j, x0;
};

template <int G, int S>
__device__ __forceinline__ Lane lane_of(const Args &A, long unit) {
    constexpr int CPW = Geo<G, S>::CPW;
    const int lane = threadIdx.x & 63;
    const long groups = (A.batch + CPW - 1) / CPW;
    Lane L;
    L.node = (int)(unit / groups);
    const int grp = (int)(unit - (long)L.node * groups);
    L.b = grp * CPW + lane / S;
    L.j = lane % S;
    L.x0 = L.j * Geo<G, S>::R;
    return L;
}

// Make this wave's LDS writes visible to its other lanes (and its reads complete)
// before the next LDS access.
__device__ __forceinline__ void lds_sync_wave() { asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory"); }

// The R consecutive entries x0 .. x0 + R - 1 of a row (16-byte aligned for R >= 4).
template <int R>
__device__ __forceinline__ void load_row(const int *p, int (&v)[R]) {
    if constexpr (R >= 4) {
#pragma unroll
        for (int q = 0; q < R / 4; ++q) {
            const int4 t = ((const int4 *)p)[q];
            v[4 * q] = t.x, v[4 * q + 1] = t.y, v[4 * q + 2] = t.z, v[4 * q + 3] = t.w;
        }
    } else if constexpr (R == 2) {
        const int2 t = *(const int2 *)p;
        v[0] = t.x, v[1] = t.y;
    } else {
        v[0] = p[0];
    }
}

template <int R>
__device__ __forceinline__ void store_row(int *p, const int (&v)[R]) {
    if constexpr (R >= 4) {
#pragma unroll
        for (int q = 0; q < R / 4; ++q) ((int4 *)p)[q] = make_int4(v[4 * q], v[4 * q + 1], v[4 * q + 2], v[4 * q + 3]);
    } else if constexpr (R == 2) {
        *(int2 *)p = make_int2(v[0], v[1]);
    } else {
        p[0] = v[0];
    }
}

// Row c of the multiplication table at entries x0 .. x0 + R - 1, one byte each, packed
// four to a word (the table is 256-byte aligned and x0 a multiple of R).
template <int G, int R>
struct MulRow {
    static constexpr int W = (R + 3) / 4;
    uint32_t w[W];
    __device__ __forceinline__ void load(const DevCode &C, int c, int x0) {
        const uint8_t *t = C.gfmul + c * G + x0;
        if constexpr (R >= 4) {
#pragma unroll
            for (int q = 0; q < W; ++q) w[q] = ((const uint32_t *)t)[q];
        } else if constexpr (R == 2) {
            w[0] = *(const uint16_t *)t;
        } else {
            w[0] = *t;
        }
    }
    __device__ __forceinline__ int operator[](int r) const { return (w[r >> 2] >> (8 * (r & 3))) & 0xFF; }
};

// Channel vectors, u = p (unless write_u is false: the fused flooding forms u itself)
// and v = 0 on every edge of the variable, decision of iteration 0: wave `unit` =
// (variable, group).
template <int G, int S>
__device__ __forceinline__ void init_unit(const Args &A, long unit, bool write_u = true) {
    constexpr int R = Geo<G, S>::R;
    const DevCode &C = A.C;
    const Lane L = lane_of<G, S>(A, unit);
    if (L.node >= C.n) return;
    const bool real = L.b < A.batch;
    const int16_t *src = (const int16_t *)A.io.llr + ((size_t)(real ? L.b : 0) * C.n + L.node) * G + L.x0;
    int w[R], fb[R], p[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int c = real ? min(max((int)src[r], 0), kSpaWeights - 1) : 0;
        w[r] = C.spa_w[c];
        fb[r] = (1 << kQ) / G;
    }
    normalise<S>(w, fb, p);
    const int best = seg_argmax<S>(p, L.x0);
    if (!real) return;
    store_row<R>(A.w.p + row(L.node, L.b, A.batch, G) + L.x0, p);
    const int zero[R] = {};
    for (int t = C.vn_ptr[L.node]; t < C.vn_ptr[L.node + 1]; ++t) {
        if (write_u) store_row<R>(A.w.u + row(C.vn_ref[t], L.b, A.batch, G) + L.x0, p);
        store_row<R>(A.w.v + row(C.vn_ref[t], L.b, A.batch, G) + L.x0, zero);  // v = 0 until a check writes it
    }
    if (L.j == 0) ((uint8_t *)A.io.hard)[(size_t)L.b * C.n + L.node] = (uint8_t)best;
}

// Check-node arithmetic of eqs. (2)-(4) for one lane: load_u(j, ix, U) fills the
// permuted inputs u'(t) = u(h^-1 t) of edge j (ix: positions h^-1 x of this lane's
// entries), store_v(n, ix, v) writes output n at the same positions (v'(h^-1 z) = v(z)).
// Output n takes the product of every other transformed input in ascending order; pre
// holds the product of inputs 0 .. n-1, shared by the outputs after it.
template <int G, int S, int DC, class LoadU, class StoreV>
__device__ __forceinline__ void cn_core(const DevCode &C, int e0, int dc, int x0, const Signs &sg, LoadU load_u,
                                        StoreV store_v) {
    constexpr int R = Geo<G, S>::R, P = Geo<G, S>::P;
    int U[DC][R];
    MulRow<G, R> ix[DC];
#pragma unroll
    for (int j = 0; j < DC; ++j) {
        if (j < dc) {
            ix[j].load(C, C.hinv[e0 + j], x0);
            load_u(j, ix[j], U[j]);
            wht<S>(U[j], sg);
        }
    }
    int pre[R];
#pragma unroll
    for (int n = 0; n < DC; ++n) {
        if (n < dc) {
            int acc[R];
#pragma unroll
            for (int r = 0; r < R; ++r) acc[r] = n > 0 ? pre[r] : (dc > 1 ? U[1][r] : 0);
#pragma unroll
            for (int j = 0; j < DC; ++j) {
                if (j < dc && j > (n > 0 ? n : 1)) {
#pragma unroll
                    for (int r = 0; r < R; ++r) acc[r] = qmul(acc[r], U[j][r]);
                }
            }
            if constexpr (G > 64) {
                // the inverse sums reach g 2^24: 64 bits, then floor(. / g) clamped at 0
                long long a64[R];
#pragma unroll
                for (int r = 0; r < R; ++r) a64[r] = acc[r];
                wht64<S>(a64, sg);
#pragma unroll
                for (int r = 0; r < R; ++r) acc[r] = (int)max(a64[r] >> P, 0ll);
            } else {
                wht<S>(acc, sg);
#pragma unroll
                for (int r = 0; r < R; ++r) acc[r] = max(acc[r] >> P, 0);  // floor(. / g), clamped at 0
            }
            store_v(n, ix[n], acc);
            if (n + 1 < dc) {
#pragma unroll
                for (int r = 0; r < R; ++r) pre[r] = n > 0 ? qmul(pre[r], U[n][r]) : U[0][r];
            }
        }
    }
}

// Variable-node arithmetic of eqs. (5)-(6) for one lane: vv holds the dv incoming
// messages, store_u(m, u) writes u_m = norm(p times every incoming message but m,
// ascending); pre holds p times messages 0 .. m-1 and ends as the a posteriori product,
// whose arg-max is returned.
template <int S, int R, int DV, class StoreU>
__device__ __forceinline__ int vn_core(int dv, int x0, const int (&p)[R], const int (&vv)[DV][R], StoreU store_u) {
    int pre[R];
#pragma unroll
    for (int r = 0; r < R; ++r) pre[r] = p[r];
#pragma unroll
    for (int m = 0; m < DV; ++m) {
        if (m < dv) {
            int z[R], u[R];
#pragma unroll
            for (int r = 0; r < R; ++r) z[r] = pre[r];
#pragma unroll
            for (int t = 0; t < DV; ++t)
                if (t < dv && t > m) {
#pragma unroll
                    for (int r = 0; r < R; ++r) z[r] = qmul(z[r], vv[t][r]);
                }
            normalise<S>(z, p, u);
            store_u(m, u);
#pragma unroll
            for (int r = 0; r < R; ++r) pre[r] = qmul(pre[r], vv[m][r]);
        }
    }
    return seg_argmax<S>(pre, x0);
}

// Check-node phase of iteration k: wave `unit` = (check, group), for check degrees up
// to DC.  Rows move between HBM and registers whole (R consecutive entries per lane);
// the permutations go through this wave's LDS row of each codeword.
template <int G, int DC>
__device__ __forceinline__ void cn_unit(const Args &A, int k, long unit) {
    constexpr int S = lanes_for<G, DC>(), R = Geo<G, S>::R;
    const DevCode &C = A.C;
    const Lane L = lane_of<G, S>(A, unit);
    if (L.node >= C.m) return;
    const bool act = active(A, k, L.b);
    if (__ballot(act) == 0) return;
    const int e0 = C.row_ptr[L.node];
    const int dc = C.row_ptr[L.node + 1] - e0;
    const int bb = L.b < A.batch ? L.b : A.batch - 1;  // lanes past the batch read a valid row
    __shared__ __align__(16) int stage[4][64 * R];
    int *srow = stage[threadIdx.x >> 6] + ((threadIdx.x & 63) / S) * G;
    auto load_u = [&](int j, const MulRow<G, R> &ix, int (&U)[R]) {
        int t[R];
        load_row<R>(A.w.u + row(e0 + j, bb, A.batch, G) + L.x0, t);
        store_row<R>(srow + L.x0, t);
        lds_sync_wave();
#pragma unroll
        for (int r = 0; r < R; ++r) U[r] = srow[ix[r]];
        lds_sync_wave();
    };
    auto store_v = [&](int n, const MulRow<G, R> &ix, const int (&v)[R]) {
#pragma unroll
        for (int r = 0; r < R; ++r) srow[ix[r]] = v[r];
        lds_sync_wave();
        int t[R];
        load_row<R>(srow + L.x0, t);
        lds_sync_wave();
        if (act) store_row<R>(A.w.v + row(e0 + n, L.b, A.batch, G) + L.x0, t);
    };
    cn_core<G, S, DC>(C, e0, dc, L.x0, signs_of<S>(L.j), load_u, store_v);
}

// Flooding for codes whose variables all have degree 2, fused into the check node: the
// check forms each incoming u = norm(p times the other edge's v of the previous
// iteration) itself (eqs. (5)-(6) with one factor), so the variable-node phase and
// its u stores disappear; v alternates between the v and u arrays (v_old -> v_new).
// With v = 0 before the first iteration the product is 0 and norm falls back to p,
// which is u before the first iteration.
template <int G, int DC>
__device__ __forceinline__ void cnf_unit(const Args &A, int k, long unit, const int *v_old, int *v_new) {
    constexpr int S = lanes_for<G, DC>(), R = Geo<G, S>::R;
    const DevCode &C = A.C;
    const Lane L = lane_of<G, S>(A, unit);
    if (L.node >= C.m) return;
    const bool act = active(A, k, L.b);
    if (__ballot(act) == 0) return;
    const int e0 = C.row_ptr[L.node];
    const int dc = C.row_ptr[L.node + 1] - e0;
    const int bb = L.b < A.batch ? L.b : A.batch - 1;
    __shared__ __align__(16) int stage[4][64 * R];
    int *srow = stage[threadIdx.x >> 6] + ((threadIdx.x & 63) / S) * G;
    auto load_u = [&](int j, const MulRow<G, R> &ix, int (&U)[R]) {
        const int e = e0 + j;
        const int var = C.col_idx[e];
        const int q0 = C.vn_ptr[var];
        const int f = C.vn_ref[q0] == e ? C.vn_ref[q0 + 1] : C.vn_ref[q0];
        int p[R], vo[R], z[R], u[R];
        load_row<R>(A.w.p + row(var, bb, A.batch, G) + L.x0, p);
        load_row<R>(v_old + row(f, bb, A.batch, G) + L.x0, vo);
#pragma unroll
        for (int r = 0; r < R; ++r) z[r] = qmul(p[r], vo[r]);
        normalise<S>(z, p, u);
        store_row<R>(srow + L.x0, u);
        lds_sync_wave();
#pragma unroll
        for (int r = 0; r < R; ++r) U[r] = srow[ix[r]];
        lds_sync_wave();
    };
    auto store_v = [&](int n, const MulRow<G, R> &ix, const int (&v)[R]) {
#pragma unroll
        for (int r = 0; r < R; ++r) srow[ix[r]] = v[r];
        lds_sync_wave();
        int t[R];
        load_row<R>(srow + L.x0, t);
        lds_sync_wave();
        if (act) store_row<R>(v_new + row(e0 + n, L.b, A.batch, G) + L.x0, t);
    };
    cn_core<G, S, DC>(C, e0, dc, L.x0, signs_of<S>(L.j), load_u, store_v);
}

// Decision of iteration k for codes whose variables all have degree 2 (the a posteriori
// product p v_0 v_1 in ascending edge order): wave `unit` = (variable, group).
template <int G>
__device__ __forceinline__ void dec_unit(const Args &A, int k, long unit, const int *v_cur) {
    constexpr int S = lanes_for<G, 4>(), R = Geo<G, S>::R;
    const DevCode &C = A.C;
    const Lane L = lane_of<G, S>(A, unit);
    if (L.node >= C.n) return;
    const bool act = active(A, k, L.b);
    if (__ballot(act) == 0) return;
    const int bb = L.b < A.batch ? L.b : A.batch - 1;
    const int t0 = C.vn_ptr[L.node];
    int p[R], v0[R], v1[R], app[R];
    load_row<R>(A.w.p + row(L.node, bb, A.batch, G) + L.x0, p);
    load_row<R>(v_cur + row(C.vn_ref[t0], bb, A.batch, G) + L.x0, v0);
    load_row<R>(v_cur + row(C.vn_ref[t0 + 1], bb, A.batch, G) + L.x0, v1);
#pragma unroll
    for (int r = 0; r < R; ++r) app[r] = qmul(qmul(p[r], v0[r]), v1[r]);
    const int best = seg_argmax<S>(app, L.x0);
    if (act && L.j == 0) {
        ((uint8_t *)A.io.hard)[(size_t)L.b * C.n + L.node] = (uint8_t)best;
        if (L.node == 0) A.w.it[L.b] = (int16_t)k;
    }
}

// Debug dump after the fused flooding: the v of codeword b sit in the array its last
// iteration wrote (odd iteration counts: the u array, the fused flooding's second v
// array), and each edge's u is the one the two-phase variable node forms from them
// (eqs. (5)-(6) with the other edge's v; p itself before any iteration, where v = 0).
// Wave `unit` = (variable, group), written straight to the [batch][E][G] dump.
template <int G>
__device__ __forceinline__ void fdump_unit(const Args &A, long unit) {
    constexpr int S = lanes_for<G, 4>(), R = Geo<G, S>::R;
    const DevCode &C = A.C;
    const Lane L = lane_of<G, S>(A, unit);
    if (L.node >= C.n) return;
    const int bb = L.b < A.batch ? L.b : A.batch - 1;
    const int *src = (A.w.it[bb] & 1) ? A.w.u : A.w.v;
    const int t0 = C.vn_ptr[L.node];
    const int e0 = C.vn_ref[t0], e1 = C.vn_ref[t0 + 1];
    int p[R], v0[R], v1[R], z[R], u0[R], u1[R];
    load_row<R>(A.w.p + row(L.node, bb, A.batch, G) + L.x0, p);
    load_row<R>(src + row(e0, bb, A.batch, G) + L.x0, v0);
    load_row<R>(src + row(e1, bb, A.batch, G) + L.x0, v1);
#pragma unroll
    for (int r = 0; r < R; ++r) z[r] = qmul(p[r], v1[r]);
    normalise<S>(z, p, u0);
#pragma unroll
    for (int r = 0; r < R; ++r) z[r] = qmul(p[r], v0[r]);
    normalise<S>(z, p, u1);
    if (L.b >= A.batch) return;
    int *da = (int *)A.io.dump_a, *db = (int *)A.io.dump_b;
    const size_t o0 = ((size_t)L.b * C.E + e0) * G + L.x0, o1 = ((size_t)L.b * C.E + e1) * G + L.x0;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        da[o0 + r] = u0[r];
        da[o1 + r] = u1[r];
        db[o0 + r] = v0[r];
        db[o1 + r] = v1[r];
    }
}

// Variable-node phase of iteration k and decision: wave `unit` = (variable, group), for
// variable degrees up to DV.
template <int G, int DV>
__device__ __forceinline__ void vn_unit(const Args &A, int k, long unit) {
    constexpr int S = lanes_for<G, DV>(), R = Geo<G, S>::R;
    const DevCode &C = A.C;
    const Lane L = lane_of<G, S>(A, unit);
    if (L.node >= C.n) return;
    const bool act = active(A, k, L.b);
    if (__ballot(act) == 0) return;
    const int bb = L.b < A.batch ? L.b : A.batch - 1;
    const int t0 = C.vn_ptr[L.node];
    const int dv = C.vn_ptr[L.node + 1] - t0;
    int p[R];
    load_row<R>(A.w.p + row(L.node, bb, A.batch, G) + L.x0, p);
    int vv[DV][R];
#pragma unroll
    for (int t = 0; t < DV; ++t)
        if (t < dv) load_row<R>(A.w.v + row(C.vn_ref[t0 + t], bb, A.batch, G) + L.x0, vv[t]);
    auto store_u = [&](int m, const int (&u)[R]) {
        if (act) store_row<R>(A.w.u + row(C.vn_ref[t0 + m], L.b, A.batch, G) + L.x0, u);
    };
    const int best = vn_core<S, R, DV>(dv, L.x0, p, vv, store_u);
    if (act && L.j == 0) {
        ((uint8_t *)A.io.hard)[(size_t)L.b * C.n + L.node] = (uint8_t)best;
        if (L.node == 0) A.w.it[L.b] = (int16_t)k;
    }
}

// ---------------------------------------------------------------------------------
// LDS-resident variant for short codes with degrees up to 4: one workgroup decodes cw
// codewords with every vector in LDS, all iterations in one launch.  LDS layout (bytes):
// p [n][cw][g], u [E][cw][g], v [E][cw][g] (int32), four int flags, the last active
// iteration [cw] (int16), unsatisfied flags [3][cw] (two iteration slots and the final
// test), decisions [n][cw].
struct LdsLayout {
    size_t p, u, v, any, its, unsat, hard, total;
};

__host__ __device__ inline LdsLayout lds_layout(const DevCode &C, int cw) {
    LdsLayout Y;
    const size_t vec = (size_t)cw * C.g * 4;
    Y.p = 0;
    Y.u = Y.p + (size_t)C.n * vec;
    Y.v = Y.u + (size_t)C.E * vec;
    Y.any = Y.v + (size_t)C.E * vec;
    Y.its = Y.any + 16;
    Y.unsat = Y.its + (size_t)cw * 2;
    Y.hard = Y.unsat + (size_t)cw * 3;
    Y.total = (Y.hard + (size_t)C.n * cw + 15) & ~(size_t)15;
    return Y;
}

// Syndrome of the decisions in LDS, thread per (check, local codeword): marks unsat[lc]
// and *any.
__device__ __forceinline__ void lds_syndrome(const DevCode &C, const uint8_t *hard, int cw, int cnt, uint8_t *unsat,
                                             int *any) {
    for (int t = threadIdx.x; t < C.m * cnt; t += blockDim.x) {
        const int r = t / cnt, lc = t - r * cnt;
        int sy = 0;
        for (int e = C.row_ptr[r]; e < C.row_ptr[r + 1]; ++e) sy ^= C.gfmul[C.h[e] * C.g + hard[C.col_idx[e] * cw + lc]];
        if (sy) {
            unsat[lc] = 1;
            *any = 1;
        }
    }
}

// Codewords [blk cw, blk cw + cw) by the calling workgroup (blk: the kernel's block
// index, or an item index of the ragged kernel).
template <int G>
__device__ __forceinline__ void lds_decode(const Args &A, int cw, unsigned char *lds, int blk) {
    constexpr int D = 4, S = lanes_for<G, D>(), R = Geo<G, S>::R, CPW = Geo<G, S>::CPW;
    const DevCode &C = A.C;
    const LdsLayout Y = lds_layout(C, cw);
    int *Pl = (int *)(lds + Y.p), *Ul = (int *)(lds + Y.u), *Vl = (int *)(lds + Y.v);
    int *any = (int *)(lds + Y.any);
    int16_t *its = (int16_t *)(lds + Y.its);
    uint8_t *unsat = lds + Y.unsat;
    uint8_t *hard = lds + Y.hard;
    const int base = blk * cw;
    const int cnt = min(cw, A.batch - base);
    const int tid = threadIdx.x, nthr = blockDim.x;
    const int waves = nthr >> 6, wave = wave_id();
    const int lane = tid & 63, j = lane % S, x0 = j * R;
    const int groups = (cnt + CPW - 1) / CPW;
    auto lrow = [&](int *arr, int node, int lc) { return arr + ((size_t)node * cw + lc) * G; };
    for (int t = tid; t < 3 * cw; t += nthr) unsat[t] = 0;
    for (int t = tid; t < cw; t += nthr) its[t] = 0;
    if (tid < 4) any[tid] = 0;
    const Signs sg = signs_of<S>(j);
    // Every variable of degree 2 and no dump: the check phase forms u itself from p and
    // the other edge's v, v alternating between the v and u arrays, decisions only where
    // used (as in the wave kernels' fused flooding).
    const bool fused = !A.io.dump_a && C.dv_max == 2 && C.E == 2 * C.n;
    // channel vectors, u = p (two-phase only) and v = 0 on every edge, decisions of
    // iteration 0
    for (int unit = wave; unit < C.n * groups; unit += waves) {
        const int node = unit / groups, lc = (unit - node * groups) * CPW + lane / S;
        const bool real = lc < cnt;
        const int lr = real ? lc : cnt - 1;
        const int16_t *src = (const int16_t *)A.io.llr + ((size_t)(base + lr) * C.n + node) * G + x0;
        int w[R], fb[R], p[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            w[r] = C.spa_w[min(max((int)src[r], 0), kSpaWeights - 1)];
            fb[r] = (1 << kQ) / G;
        }
        normalise<S>(w, fb, p);
        const int best = seg_argmax<S>(p, x0);
        if (real) {
            store_row<R>(lrow(Pl, node, lc) + x0, p);
            const int zero[R] = {};
            for (int t = C.vn_ptr[node]; t < C.vn_ptr[node + 1]; ++t) {
                if (!fused) store_row<R>(lrow(Ul, C.vn_ref[t], lc) + x0, p);
                store_row<R>(lrow(Vl, C.vn_ref[t], lc) + x0, zero);
            }
            if (j == 0) hard[node * cw + lc] = (uint8_t)best;
        }
    }
    __syncthreads();
    for (int k = 1; k <= A.max_iters; ++k) {
        const int slot = k & 1;
        if (A.early_stop) {
            lds_syndrome(C, hard, cw, cnt, unsat + slot * cw, any + slot);
            __syncthreads();
            if (any[slot] == 0) break;  // every codeword satisfied: nothing changes any more
            // the other slot was last read before the previous iteration's final barrier
            for (int t = tid; t < cw; t += nthr) unsat[(slot ^ 1) * cw + t] = 0;
            if (tid == 0) any[slot ^ 1] = 0;
        }
        const uint8_t *us = unsat + slot * cw;
        if (fused) {
            const int *vo = (k & 1) ? Vl : Ul;
            int *vn = (k & 1) ? Ul : Vl;
            for (int unit = wave; unit < C.m * groups; unit += waves) {
                const int node = unit / groups, lc = (unit - node * groups) * CPW + lane / S;
                const bool act = lc < cnt && (!A.early_stop || us[lc]);
                if (__ballot(act) == 0) continue;
                const int lr = lc < cnt ? lc : cnt - 1;
                const int e0 = C.row_ptr[node];
                auto load_u = [&](int jj, const MulRow<G, R> &ix, int (&U)[R]) {
                    const int e = e0 + jj;
                    const int var = C.col_idx[e];
                    const int q0 = C.vn_ptr[var];
                    const int f = C.vn_ref[q0] == e ? C.vn_ref[q0 + 1] : C.vn_ref[q0];
                    const int *pr = lrow(Pl, var, lr), *vr = vo + ((size_t)f * cw + lr) * G;
                    int p[R], z[R], u[R];
#pragma unroll
                    for (int r = 0; r < R; ++r) {
                        // the permuted entry x' = h^-1 t of u is formed from p(x') and v(x')
                        p[r] = pr[ix[r]];
                        z[r] = qmul(p[r], vr[ix[r]]);
                    }
                    normalise<S>(z, p, u);
#pragma unroll
                    for (int r = 0; r < R; ++r) U[r] = u[r];
                };
                auto store_v = [&](int n, const MulRow<G, R> &ix, const int (&v)[R]) {
                    if (act) {
                        int *r0 = vn + ((size_t)(e0 + n) * cw + lc) * G;
#pragma unroll
                        for (int r = 0; r < R; ++r) r0[ix[r]] = v[r];
                    }
                };
                cn_core<G, S, D>(C, e0, C.row_ptr[node + 1] - e0, x0, sg, load_u, store_v);
            }
            __syncthreads();
            if (A.early_stop || k == A.max_iters) {
                for (int unit = wave; unit < C.n * groups; unit += waves) {
                    const int node = unit / groups, lc = (unit - node * groups) * CPW + lane / S;
                    const bool act = lc < cnt && (!A.early_stop || us[lc]);
                    if (__ballot(act) == 0) continue;
                    const int lr = lc < cnt ? lc : cnt - 1;
                    const int t0 = C.vn_ptr[node];
                    int p[R], v0[R], v1[R], app[R];
                    load_row<R>(lrow(Pl, node, lr) + x0, p);
                    load_row<R>(vn + ((size_t)C.vn_ref[t0] * cw + lr) * G + x0, v0);
                    load_row<R>(vn + ((size_t)C.vn_ref[t0 + 1] * cw + lr) * G + x0, v1);
#pragma unroll
                    for (int r = 0; r < R; ++r) app[r] = qmul(qmul(p[r], v0[r]), v1[r]);
                    const int best = seg_argmax<S>(app, x0);
                    if (act && j == 0) {
                        hard[node * cw + lc] = (uint8_t)best;
                        if (node == 0) its[lc] = (int16_t)k;
                    }
                }
                __syncthreads();
            }
            continue;
        }
        for (int unit = wave; unit < C.m * groups; unit += waves) {
            const int node = unit / groups, lc = (unit - node * groups) * CPW + lane / S;
            const bool act = lc < cnt && (!A.early_stop || us[lc]);
            if (__ballot(act) == 0) continue;
            const int lr = lc < cnt ? lc : cnt - 1;
            const int e0 = C.row_ptr[node];
            auto load_u = [&](int jj, const MulRow<G, R> &ix, int (&U)[R]) {
                const int *r0 = lrow(Ul, e0 + jj, lr);
#pragma unroll
                for (int r = 0; r < R; ++r) U[r] = r0[ix[r]];
            };
            auto store_v = [&](int n, const MulRow<G, R> &ix, const int (&v)[R]) {
                if (act) {
                    int *r0 = lrow(Vl, e0 + n, lc);
#pragma unroll
                    for (int r = 0; r < R; ++r) r0[ix[r]] = v[r];
                }
            };
            cn_core<G, S, D>(C, e0, C.row_ptr[node + 1] - e0, x0, sg, load_u, store_v);
        }
        __syncthreads();
        for (int unit = wave; unit < C.n * groups; unit += waves) {
            const int node = unit / groups, lc = (unit - node * groups) * CPW + lane / S;
            const bool act = lc < cnt && (!A.early_stop || us[lc]);
            if (__ballot(act) == 0) continue;
            const int lr = lc < cnt ? lc : cnt - 1;
            const int t0 = C.vn_ptr[node];
            const int dv = C.vn_ptr[node + 1] - t0;
            int p[R], vv[D][R];
            load_row<R>(lrow(Pl, node, lr) + x0, p);
#pragma unroll
            for (int t = 0; t < D; ++t)
                if (t < dv) load_row<R>(lrow(Vl, C.vn_ref[t0 + t], lr) + x0, vv[t]);
            auto store_u = [&](int m, const int (&u)[R]) {
                if (act) store_row<R>(lrow(Ul, C.vn_ref[t0 + m], lc) + x0, u);
            };
            const int best = vn_core<S, R, D>(dv, x0, p, vv, store_u);
            if (act && j == 0) {
                hard[node * cw + lc] = (uint8_t)best;
                if (node == 0) its[lc] = (int16_t)k;
            }
        }
        __syncthreads();
    }
    lds_syndrome(C, hard, cw, cnt, unsat + 2 * cw, any + 2);
    __syncthreads();
    for (int t = tid; t < cnt; t += nthr) {
        A.io.ok[base + t] = unsat[2 * cw + t] ? 0 : 1;
        A.io.iters[base + t] = its[t];
    }
    uint8_t *hout = (uint8_t *)A.io.hard;
    for (int t = tid; t < C.n * cnt; t += nthr) {
        const int node = t / cnt, lc = t - node * cnt;
        hout[(size_t)(base + lc) * C.n + node] = hard[node * cw + lc];
    }
    if (A.io.dump_a) {
        const int per_e = cnt * G;
        for (int t = tid; t < C.E * per_e; t += nthr) {
            const int e = t / per_e, r = t - e * per_e, lc = r / G, x = r - lc * G;
            const size_t o = ((size_t)(base + lc) * C.E + e) * G + x;
            ((int *)A.io.dump_a)[o] = lrow(Ul, e, lc)[x];
            ((int *)A.io.dump_b)[o] = lrow(Vl, e, lc)[x];
        }
    }
}

// Syndrome test: thread per (check, codeword); marks the codeword unsatisfied in slot_k.
__device__ __forceinline__ void syn_thread(const Args &A, int slot_k, long t) {
    const DevCode &C = A.C;
    const int r = (int)(t / A.batch), b = (int)(t - (long)r * A.batch);
    if (r >= C.m) return;
    const uint8_t *hard = (const uint8_t *)A.io.hard + (size_t)b * C.n;
    int s = 0;
    for (int e = C.row_ptr[r]; e < C.row_ptr[r + 1]; ++e) s ^= C.gfmul[C.h[e] * C.g + hard[C.col_idx[e]]];
    if (s) A.w.unsat[(size_t)slot_k * A.batch + b] = 1;
}

__device__ __forceinline__ void fin_thread(const Args &A, long t) {
    if (t >= A.batch) return;
    A.io.ok[t] = A.w.unsat[t] ? 0 : 1;
    A.io.iters[t] = A.w.it[t];
}

// [E][batch][G] -> [batch][E][G] for the debug dump: thread per entry.
__device__ __forceinline__ void dump_thread(const Args &A, const int *src, int *dst, long t) {
    const int G = A.C.g;
    const long per_edge = (long)A.batch * G;
    const int e = (int)(t / per_edge);
    if (e >= A.C.E) return;
    const long r = t - (long)e * per_edge;
    const int b = (int)(r / G), x = (int)(r - (long)b * G);
    dst[((size_t)b * A.C.E + e) * G + x] = src[t];
}

struct Carve {
    size_t p, u, v, unsat, it, total;
};

inline Carve carve(const DevCode &C, int max_iters, int batch) {
    Carve c;
    size_t o = 0;
    c.p = o;
    o = align_up(o + (size_t)C.n * batch * C.g * 4, 256);
    c.u = o;
    o = align_up(o + (size_t)C.E * batch * C.g * 4, 256);
    c.v = o;
    o = align_up(o + (size_t)C.E * batch * C.g * 4, 256);
    c.unsat = o;
    o = align_up(o + (size_t)(max_iters + 1) * batch, 256);
    c.it = o;
    o = align_up(o + (size_t)batch * 2, 256);
    c.total = o;
    return c;
}

inline Args make_args(const DevCode &C, int max_iters, int early_stop, int batch, void *base, const DecodeIO &io) {
    Args A;
    A.C = C;
    A.max_iters = max_iters;
    A.early_stop = early_stop;
    A.batch = batch;
    const Carve c = carve(C, max_iters, batch);
    char *q = (char *)base;
    A.w.p = (int *)(q + c.p);
    A.w.u = (int *)(q + c.u);
    A.w.v = (int *)(q + c.v);
    A.w.unsat = (uint8_t *)(q + c.unsat);
    A.w.it = (int16_t *)(q + c.it);
    A.io = io;
    return A;
}

}  // namespace spa
}  // namespace dev
}  // namespace ldpcx
