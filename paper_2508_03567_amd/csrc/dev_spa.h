// Fixed-point FFT-SPA decoder (Alg. 1) for fields up to GF(64), as wave-level device
// functions.
//
// Arithmetic: probabilities in Q24 (2^24 = 1); the transform of eq. (8) over GF(2^q)
// is the Walsh-Hadamard transform, exact in 32-bit integers; products of two Q24
// numbers are floor((a b + 2^23) / 2^24), taken in ascending edge order; the inverse
// transform is followed by a floor division by g and a clamp at 0; a vector z is
// normalised (eq. (11)) as floor((z(x) R + 2^21) / 2^22) with R = floor(2^46 / sum z);
// channel vectors come from the symbol costs gamma through the weights
// W(c) = round(2^24 exp(-c / 4)).
//
// Mapping: a wavefront covers 64 / g codewords of one node, a segment of g lanes per
// codeword with lane x holding entry x.  The transform butterflies, the segment sums
// and the arg-max are xor-shuffles inside the segment; the permutation by the edge
// coefficient is folded into the loads, the depermutation is one indexed shuffle.
// Messages are stored codeword-major per edge, [edge][codeword][x] (int32).
#pragma once

#include "dev_common.h"

namespace ldpcx {
namespace dev {
namespace spa {

constexpr int kQ = 24;
constexpr int kVnRegs = 16;  // incoming check messages a variable keeps in registers

struct Args {
    DevCode C;
    int max_iters, early_stop, batch;
    SpaWork w;
    DecodeIO io;
};

__device__ __forceinline__ int qmul(int a, int b) {
    return (int)(((long long)a * b + (1ll << (kQ - 1))) >> kQ);
}

// Walsh-Hadamard transform of the segment (lane x holds entry x).
template <int G>
__device__ __forceinline__ int wht(int val, int x) {
#pragma unroll
    for (int s = 1; s < G; s <<= 1) {
        const int o = __shfl_xor(val, s, 64);
        val = (x & s) ? o - val : val + o;
    }
    return val;
}

template <int G>
__device__ __forceinline__ int seg_sum(int v) {
#pragma unroll
    for (int s = 1; s < G; s <<= 1) v += __shfl_xor(v, s, 64);
    return v;
}

template <int G>
__device__ __forceinline__ int seg_max(int v) {
#pragma unroll
    for (int s = 1; s < G; s <<= 1) v = max(v, __shfl_xor(v, s, 64));
    return v;
}

// norm(z) for this lane's entry; `fallback` when the segment sum is 0.
template <int G>
__device__ __forceinline__ int normalise(int z, int fallback) {
    const int s = seg_sum<G>(z);
    if (s <= 0) return fallback;
    const long long r = (1ll << 46) / s;
    return (int)(((long long)z * r + (1ll << 21)) >> 22);
}

// Arg-max over the segment with the lowest x on ties (values < 2^25).
template <int G>
__device__ __forceinline__ int seg_argmax(int val, int x) {
    const int key = seg_max<G>(val * 64 + (63 - x));
    return 63 - (key & 63);
}

__host__ __device__ inline size_t row(int node, int b, int batch, int g) { return ((size_t)node * batch + b) * g; }

__device__ __forceinline__ bool active(const Args &A, int k, int b) {
    return b < A.batch && (!A.early_stop || A.w.unsat[(size_t)k * A.batch + b]);
}

// Lane geometry of wave `unit` = (node, group of 64 / G codewords).
struct Lane {
    int node, b, x, seg_base;
};

template <int G>
__device__ __forceinline__ Lane lane_of(const Args &A, long unit) {
    constexpr int CPW = 64 / G;
    const int lane = threadIdx.x & 63;
    const long groups = (A.batch + CPW - 1) / CPW;
    Lane L;
    L.node = (int)(unit / groups);
    const int grp = (int)(unit - (long)L.node * groups);
    L.b = grp * CPW + lane / G;
    L.x = lane % G;
    L.seg_base = lane - L.x;
    return L;
}

// Channel vectors, u = p on every edge of the variable, decision of iteration 0:
// wave `unit` = (variable, group).
template <int G>
__device__ __forceinline__ void init_unit(const Args &A, long unit) {
    const DevCode &C = A.C;
    const Lane L = lane_of<G>(A, unit);
    if (L.node >= C.n) return;
    const bool real = L.b < A.batch;
    int c = real ? ((const int16_t *)A.io.llr)[((size_t)L.b * C.n + L.node) * G + L.x] : 0;
    c = min(max(c, 0), kSpaWeights - 1);
    const int w = C.spa_w[c];
    const int p = normalise<G>(w, (1 << kQ) / G);
    const int best = seg_argmax<G>(p, L.x);
    if (!real) return;
    A.w.p[row(L.node, L.b, A.batch, G) + L.x] = p;
    for (int t = C.vn_ptr[L.node]; t < C.vn_ptr[L.node + 1]; ++t) A.w.u[row(C.vn_ref[t], L.b, A.batch, G) + L.x] = p;
    if (L.x == 0) ((uint8_t *)A.io.hard)[(size_t)L.b * C.n + L.node] = (uint8_t)best;
}

// Check-node phase of iteration k (eqs. (7)-(9)): wave `unit` = (check, group).
template <int G>
__device__ __forceinline__ void cn_unit(const Args &A, int k, long unit) {
    constexpr int P = G == 64 ? 6 : G == 32 ? 5 : G == 16 ? 4 : G == 8 ? 3 : G == 4 ? 2 : 1;
    const DevCode &C = A.C;
    const Lane L = lane_of<G>(A, unit);
    if (L.node >= C.m) return;
    const bool act = active(A, k, L.b);
    if (__ballot(act) == 0) return;
    const int e0 = C.row_ptr[L.node];
    const int dc = C.row_ptr[L.node + 1] - e0;
    const int bb = L.b < A.batch ? L.b : A.batch - 1;  // lanes past the batch read a valid row
    int U[kNbDcMax];
#pragma unroll
    for (int j = 0; j < kNbDcMax; ++j) {
        if (j < dc) {
            const int e = e0 + j;
            const int idx = C.gfmul[C.hinv[e] * G + L.x];  // u'(t) = u(h^-1 t)
            U[j] = wht<G>(A.w.u[row(e, bb, A.batch, G) + idx], L.x);
        }
    }
#pragma unroll
    for (int n = 0; n < kNbDcMax; ++n) {
        if (n < dc) {
            int acc = 0;
            bool first = true;
#pragma unroll
            for (int j = 0; j < kNbDcMax; ++j) {
                if (j < dc && j != n) {
                    acc = first ? U[j] : qmul(acc, U[j]);
                    first = false;
                }
            }
            const int t = wht<G>(acc, L.x) >> P;  // floor(. / g)
            const int v = max(t, 0);
            const int e = e0 + n;
            const int vp = __shfl(v, L.seg_base + C.gfmul[C.h[e] * G + L.x], 64);  // v'(x) = v(h x)
            if (act) A.w.v[row(e, L.b, A.batch, G) + L.x] = vp;
        }
    }
}

// Variable-node phase of iteration k (eqs. (10)-(11)) and decision: wave `unit` =
// (variable, group).
template <int G>
__device__ __forceinline__ void vn_unit(const Args &A, int k, long unit) {
    const DevCode &C = A.C;
    const Lane L = lane_of<G>(A, unit);
    if (L.node >= C.n) return;
    const bool act = active(A, k, L.b);
    if (__ballot(act) == 0) return;
    const int bb = L.b < A.batch ? L.b : A.batch - 1;
    const int t0 = C.vn_ptr[L.node];
    const int dv = C.vn_ptr[L.node + 1] - t0;
    const int p = A.w.p[row(L.node, bb, A.batch, G) + L.x];
    int vv[kVnRegs];
#pragma unroll
    for (int t = 0; t < kVnRegs; ++t)
        if (t < dv) vv[t] = A.w.v[row(C.vn_ref[t0 + t], bb, A.batch, G) + L.x];
#pragma unroll
    for (int m = 0; m < kVnRegs; ++m) {
        if (m < dv) {
            int z = p;
#pragma unroll
            for (int t = 0; t < kVnRegs; ++t)
                if (t < dv && t != m) z = qmul(z, vv[t]);
            const int u = normalise<G>(z, p);
            if (act) A.w.u[row(C.vn_ref[t0 + m], L.b, A.batch, G) + L.x] = u;
        }
    }
    int app = p;
#pragma unroll
    for (int t = 0; t < kVnRegs; ++t)
        if (t < dv) app = qmul(app, vv[t]);
    const int best = seg_argmax<G>(app, L.x);
    if (act && L.x == 0) {
        ((uint8_t *)A.io.hard)[(size_t)L.b * C.n + L.node] = (uint8_t)best;
        if (L.node == 0) A.w.it[L.b] = (int16_t)k;
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
