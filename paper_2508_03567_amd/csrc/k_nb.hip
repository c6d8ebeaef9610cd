// Interleaved Min-Max decoder over GF(g), g = 2^p <= 64 (Alg. 2).
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
#include "k_common.h"

namespace ldpcx {

namespace {

typedef short v2s __attribute__((ext_vector_type(2)));

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

// a~(t) = msg(hinv * t) for one edge, loaded straight from [edge][x][Bp] memory.
template <int G>
__device__ __forceinline__ void load_perm(const int16_t *__restrict__ msg, long Bp, int e, const uint8_t *__restrict__ mrow,
                                          int b, v2s (&A)[G / 2]) {
    const int16_t *base = msg + (long)e * G * Bp + b;
#pragma unroll
    for (int t = 0; t < G; t += 2) {
        const int x0 = mrow[t], x1 = mrow[t + 1];
        A[t >> 1] = (v2s){base[(long)x0 * Bp], base[(long)x1 * Bp]};
    }
}

// msg(x) = v~(h x) stored for one edge: entry t goes to x = hinv * t.
template <int G>
__device__ __forceinline__ void store_deperm(int16_t *__restrict__ msg, long Bp, int e, const uint8_t *__restrict__ mrow,
                                             int b, const v2s (&V)[G / 2], bool act) {
    int16_t *base = msg + (long)e * G * Bp + b;
    if (!act) return;
#pragma unroll
    for (int t = 0; t < G; t += 2) {
        base[(long)mrow[t] * Bp] = V[t >> 1].x;
        base[(long)mrow[t + 1] * Bp] = V[t >> 1].y;
    }
}

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

template <int G>
__global__ void __launch_bounds__(256) k_nb_cn(DevCode C, int Bp, int early, int batch, int fslots,
                                               const int16_t *__restrict__ alpha, int16_t *__restrict__ beta,
                                               const uint64_t *__restrict__ unsat_slot) {
    extern __shared__ uint32_t lds[];
    constexpr int H = G / 2;
    const int lane = threadIdx.x & 63;
    const int w = threadIdx.x >> 6;
    const int row = blockIdx.x * (blockDim.x >> 6) + w;
    if (row >= C.m) return;
    const int g = blockIdx.y;
    const int b = g * 64 + lane;
    const bool act = b < batch && (!early || ((unsat_slot[g] >> lane) & 1ull));
    if (__ballot(act) == 0) return;
    uint32_t *fs = lds + (size_t)w * fslots * H * 64;
    const int e0 = C.row_ptr[row];
    const int dc = C.row_ptr[row + 1] - e0;
    const uint8_t *mul = C.gfmul;
    v2s X[H], Y[H], R[H];
    load_perm<G>(alpha, Bp, e0, mul + C.hinv[e0] * G, b, X);
    const int nf = dc - 2;
    for (int s = 0; s < 3 * nf; ++s) {
        int kind, j;
        if (s < nf) {
            kind = 0;
            j = s + 1;
            load_perm<G>(alpha, Bp, e0 + j, mul + C.hinv[e0 + j] * G, b, Y);
        } else {
            const int t = s - nf;
            j = dc - 2 - (t >> 1);
            if (t == 0) {
                // X = F_{dc-2} is the output of the last edge (eq. (12)); start the backward pass.
                store_deperm<G>(beta, Bp, e0 + dc - 1, mul + C.hinv[e0 + dc - 1] * G, b, X, act);
                load_perm<G>(alpha, Bp, e0 + dc - 1, mul + C.hinv[e0 + dc - 1] * G, b, X);
            }
            if ((t & 1) == 0) {
                kind = 1;  // middle output: F_{j-1} (*) B_{j+1}
                if (j == 1) load_perm<G>(alpha, Bp, e0, mul + C.hinv[e0] * G, b, Y);
                else lds_get<G>(fs + (size_t)(j - 2) * H * 64, lane, Y);
            } else {
                kind = 2;  // B_j = B_{j+1} (*) a~_j
                load_perm<G>(alpha, Bp, e0 + j, mul + C.hinv[e0 + j] * G, b, Y);
            }
        }
        conv<G>(X, Y, R);
        if (kind == 1) {
            store_deperm<G>(beta, Bp, e0 + j, mul + C.hinv[e0 + j] * G, b, R, act);
        } else {
#pragma unroll
            for (int p = 0; p < H; ++p) X[p] = R[p];
            if (kind == 0 && j <= dc - 3) lds_put<G>(fs + (size_t)(j - 1) * H * 64, lane, X);
        }
    }
    if (nf == 0) {
        store_deperm<G>(beta, Bp, e0 + 1, mul + C.hinv[e0 + 1] * G, b, X, act);
        load_perm<G>(alpha, Bp, e0 + 1, mul + C.hinv[e0 + 1] * G, b, X);
    }
    store_deperm<G>(beta, Bp, e0, mul + C.hinv[e0] * G, b, X, act);
}

// Variable-node update (eqs. (14)-(15)) and decision for one variable node of 64 codewords.
template <int G>
__global__ void __launch_bounds__(256) k_nb_vn(DevCode C, int Bp, int k, int early, int batch,
                                               const int16_t *__restrict__ gam, int16_t *__restrict__ alpha,
                                               const int16_t *__restrict__ beta, uint8_t *__restrict__ hard,
                                               int16_t *__restrict__ it, const uint64_t *__restrict__ unsat_slot) {
    const int lane = threadIdx.x & 63;
    const int v = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (v >= C.n) return;
    const int g = blockIdx.y;
    const int b = g * 64 + lane;
    const bool act = b < batch && (!early || ((unsat_slot[g] >> lane) & 1ull));
    if (__ballot(act) == 0) return;
    int S[G];
    const int16_t *gp = gam + (long)v * G * Bp + b;
#pragma unroll
    for (int x = 0; x < G; ++x) S[x] = gp[(long)x * Bp];
    const int t0 = C.vn_ptr[v], t1 = C.vn_ptr[v + 1];
    for (int t = t0; t < t1; ++t) {
        const int16_t *bp = beta + (long)C.vn_ref[t] * G * Bp + b;
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
        hard[(long)v * Bp + b] = (uint8_t)best;
        if (v == 0) it[b] = (int16_t)k;
    }
    for (int t = t0; t < t1; ++t) {
        const int e = C.vn_ref[t];
        const int16_t *bp = beta + (long)e * G * Bp + b;
        int a[G];
        int mn = 0x7fffffff;
#pragma unroll
        for (int x = 0; x < G; ++x) {
            a[x] = S[x] - bp[(long)x * Bp];
            mn = min(mn, a[x]);
        }
        if (act) {
            int16_t *ap = alpha + (long)e * G * Bp + b;
#pragma unroll
            for (int x = 0; x < G; ++x) ap[(long)x * Bp] = (int16_t)min(a[x] - mn, 32767);
        }
    }
}

// Syndrome sum_j h_j c_j over GF(g) for one check and 64 codewords.
__global__ void __launch_bounds__(256) k_nb_syn(DevCode C, int Bp, int batch, const uint8_t *__restrict__ hard,
                                                uint64_t *__restrict__ unsat_slot) {
    const int lane = threadIdx.x & 63;
    const int row = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (row >= C.m) return;
    const int g = blockIdx.y;
    const int b = g * 64 + lane;
    int s = 0;
    for (int e = C.row_ptr[row]; e < C.row_ptr[row + 1]; ++e)
        s ^= C.gfmul[C.h[e] * C.g + hard[(long)C.col_idx[e] * Bp + b]];
    const uint64_t bits = __ballot(s != 0 && b < batch);
    if (lane == 0 && bits) atomicOr((unsigned long long *)&unsat_slot[g], (unsigned long long)bits);
}

template <int G>
__global__ void __launch_bounds__(256) k_nb_init(DevCode C, int Bp, const int16_t *__restrict__ gam,
                                                 int16_t *__restrict__ alpha, int16_t *__restrict__ beta,
                                                 uint8_t *__restrict__ hard) {
    // one wave per (edge, group): alpha^(0) = gamma of the edge's variable, beta = 0
    const int lane = threadIdx.x & 63;
    const int e = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const int b = blockIdx.y * 64 + lane;
    if (e < C.E) {
        const int16_t *gp = gam + (long)C.col_idx[e] * G * Bp + b;
        int16_t *ap = alpha + (long)e * G * Bp + b;
        int16_t *bp = beta + (long)e * G * Bp + b;
#pragma unroll 8
        for (int x = 0; x < G; ++x) {
            ap[(long)x * Bp] = gp[(long)x * Bp];
            bp[(long)x * Bp] = 0;
        }
    }
    if (e < C.n) {
        // decision of iteration 0: most likely channel symbol, lowest x on ties
        const int16_t *gp = gam + (long)e * G * Bp + b;
        int best = 0, bv = gp[0];
        for (int x = 1; x < G; ++x) {
            const int val = gp[(long)x * Bp];
            if (val < bv) {
                bv = val;
                best = x;
            }
        }
        hard[(long)e * Bp + b] = (uint8_t)best;
    }
}

__global__ void __launch_bounds__(256) k_nb_fin(int batch, const uint64_t *__restrict__ unsat_final,
                                                const int16_t *__restrict__ it, uint8_t *__restrict__ ok,
                                                int16_t *__restrict__ iters) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= batch) return;
    ok[b] = ((unsat_final[b >> 6] >> (b & 63)) & 1ull) ? 0 : 1;
    iters[b] = it[b];
}

struct Carve {
    size_t gam, alpha, beta, hard, unsat, it, total;
};

Carve carve(const DevCode &C, int max_iters, int batch) {
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

template <int G>
hipError_t run(const DevCode &C, int max_iters, int early_stop, int batch, const NbWork &w, const DecodeIO &io,
               hipStream_t s) {
    const int Bp = pad64(batch), Gn = Bp / 64;
    hipError_t e;
    if ((e = transpose<int16_t>((const int16_t *)io.llr, batch, (long)C.n * G, (long)C.n * G, w.gam, Bp, Bp, s)) !=
        hipSuccess)
        return e;
    const int rows_init = C.E > C.n ? C.E : C.n;
    hipLaunchKernelGGL(k_nb_init<G>, dim3((unsigned)((rows_init + 3) / 4), (unsigned)Gn), dim3(256), 0, s, C, Bp,
                       w.gam, w.alpha, w.beta, w.hard);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = fill_u32(w.unsat, (size_t)(max_iters + 1) * Gn * 8, 0u, s)) != hipSuccess) return e;
    if ((e = fill_u32(w.it, align_up((size_t)Bp * 2, 4), 0u, s)) != hipSuccess) return e;
    const int fslots = C.dc_max > 3 ? C.dc_max - 3 : 1;
    // forward vectors kept for the middle outputs: fslots x (G/2) x 64 lanes x 4 bytes per wave
    const size_t per_wave = (size_t)fslots * (G / 2) * 64 * 4;
    int wpb = (int)std::min<size_t>(4, (size_t)(64 * 1024) / per_wave);
    if (wpb < 1) return hipErrorInvalidConfiguration;
    const size_t smem = (size_t)wpb * per_wave;
    const dim3 blk(256);
    const dim3 bcn(64 * wpb);
    const dim3 gcn((unsigned)((C.m + wpb - 1) / wpb), (unsigned)Gn);
    const dim3 gsy((unsigned)((C.m + 3) / 4), (unsigned)Gn);
    const dim3 gvn((unsigned)((C.n + 3) / 4), (unsigned)Gn);
    for (int k = 1; k <= max_iters; ++k) {
        uint64_t *slot = w.unsat + (size_t)k * Gn;
        if (early_stop) hipLaunchKernelGGL(k_nb_syn, gsy, blk, 0, s, C, Bp, batch, w.hard, slot);
        hipLaunchKernelGGL(k_nb_cn<G>, gcn, bcn, smem, s, C, Bp, early_stop, batch, fslots, w.alpha, w.beta, slot);
        hipLaunchKernelGGL(k_nb_vn<G>, gvn, blk, 0, s, C, Bp, k, early_stop, batch, w.gam, w.alpha, w.beta, w.hard,
                           w.it, slot);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_nb_syn, gsy, blk, 0, s, C, Bp, batch, w.hard, w.unsat);
    hipLaunchKernelGGL(k_nb_fin, dim3((unsigned)((batch + 255) / 256)), blk, 0, s, batch, w.unsat, w.it, io.ok,
                       io.iters);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = transpose<uint8_t>(w.hard, C.n, batch, Bp, (uint8_t *)io.hard, C.n, C.n, s)) != hipSuccess) return e;
    if (io.dump_a) {
        const long rows = (long)C.E * G;
        if ((e = transpose<int16_t>(w.alpha, rows, batch, Bp, (int16_t *)io.dump_a, rows, rows, s)) != hipSuccess)
            return e;
        if ((e = transpose<int16_t>(w.beta, rows, batch, Bp, (int16_t *)io.dump_b, rows, rows, s)) != hipSuccess)
            return e;
    }
    return hipSuccess;
}

}  // namespace

bool nb_supported(int g) { return g == 4 || g == 8 || g == 16 || g == 32 || g == 64; }

size_t nb_work_bytes(const DevCode &C, int max_iters, int batch) { return carve(C, max_iters, batch).total; }

void nb_carve(void *base, const DevCode &C, int max_iters, int batch, NbWork &w) {
    const Carve c = carve(C, max_iters, batch);
    char *p = (char *)base;
    w.gam = (int16_t *)(p + c.gam);
    w.alpha = (int16_t *)(p + c.alpha);
    w.beta = (int16_t *)(p + c.beta);
    w.hard = (uint8_t *)(p + c.hard);
    w.unsat = (uint64_t *)(p + c.unsat);
    w.it = (int16_t *)(p + c.it);
}

hipError_t launch_nb(const DevCode &C, int max_iters, int early_stop, int batch, const NbWork &w, const DecodeIO &io,
                     hipStream_t s) {
    switch (C.g) {
    case 4: return run<4>(C, max_iters, early_stop, batch, w, io, s);
    case 8: return run<8>(C, max_iters, early_stop, batch, w, io, s);
    case 16: return run<16>(C, max_iters, early_stop, batch, w, io, s);
    case 32: return run<32>(C, max_iters, early_stop, batch, w, io, s);
    case 64: return run<64>(C, max_iters, early_stop, batch, w, io, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace ldpcx
