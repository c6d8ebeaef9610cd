// LDS-resident binary min-sum decoder (flooding and layered schedules), as a
// workgroup-level device function.
//
// One workgroup decodes `cpw` whole codewords and keeps all of their state on
// chip for every iteration: the a posteriori sums Lambda (int16, one per
// variable node), the compressed check-node state (32 bits per check: two
// smallest magnitudes, position of the smallest and the sign of every incoming
// message) and, for flooding, the channel LLRs.  Only the channel input and the
// decisions cross HBM.  A thread processes one check row at a time with the
// incoming messages in registers; the check rule is the min-sum form of the
// binary (GF(2)) Min-Max check node (sec. 2.2, Alg. 2 with g = 2).
#pragma once

#include "dev_common.h"

namespace ldpcx {
namespace dev {
namespace lds {


struct LdsLayout {
    size_t lam, st, L, flags, total;
};

__host__ __device__ inline LdsLayout lds_layout(int n, int m, int layered, int cpw) {
    LdsLayout o;
    o.lam = 0;
    o.st = align_up((size_t)2 * n * cpw, 16);
    o.L = o.st + (size_t)4 * m * cpw;
    o.flags = align_up(o.L + (layered ? 0 : (size_t)n * cpw), 16);
    o.total = o.flags + (size_t)3 * 4 * cpw;
    return o;
}

struct Unpacked {
    int fm1, fm2, idx;
    uint32_t signs, parity;
};

__device__ __forceinline__ Unpacked unpack(const BinRule &R, uint32_t s) {
    Unpacked u;
    u.fm1 = bin_norm(R, (int)(s & 127u));
    u.fm2 = bin_norm(R, (int)((s >> 7) & 127u));
    u.idx = (int)((s >> 14) & 15u);
    u.signs = s >> 18;
    u.parity = __popc(u.signs) & 1u;
    return u;
}

// Process one check row: read Lambda of its variables and the row's previous
// state, form q = Lambda - r_old, compute the new state from the saturated
// messages clamp(q, +-msg_max); in layered mode also write Lambda = q + r_new
// back (exact, so Lambda stays L + sum of the current check messages).
// Returns the new packed state.
template <bool WRITE_LAM>
__device__ __forceinline__ uint32_t row_update(const DevCode &C, const BinRule &R, int row,
                                               int16_t *__restrict__ lam, uint32_t st_old) {
    const int b = C.row_ptr[row];
    const int dc = C.row_ptr[row + 1] - b;
    const int *__restrict__ cols = C.col_idx + b;
    const Unpacked o = unpack(R, st_old);
    const int mm = R.msg_max;
    int q[kBinDcMax];
    int v[kBinDcMax];
    int m1 = 1 << 20, m2 = 1 << 20, idx = 0;
    uint32_t sg = 0;
#pragma unroll
    for (int j = 0; j < kBinDcMax; ++j) {
        if (j < dc) {
            const int vv = cols[j];
            v[j] = vv;
            const int qraw = (int)lam[vv] - bin_r(j, o.fm1, o.fm2, o.idx, o.signs, o.parity);
            q[j] = qraw;
            const int qq = clampi(qraw, -mm, mm);
            const int a = qq < 0 ? -qq : qq;
            sg |= (uint32_t)(qq < 0) << j;
            if (a < m1) {
                m2 = m1;
                m1 = a;
                idx = j;
            } else if (a < m2) {
                m2 = a;
            }
        }
    }
    if (WRITE_LAM) {
        const int fm1 = bin_norm(R, m1), fm2 = bin_norm(R, m2);
        const uint32_t par = __popc(sg) & 1u;
#pragma unroll
        for (int j = 0; j < kBinDcMax; ++j)
            if (j < dc) lam[v[j]] = (int16_t)(q[j] + bin_r(j, fm1, fm2, idx, sg, par));
    }
    return st_pack(m1, m2, idx, sg);
}

// Flooding variable-node update: Lambda_v = L_v + sum of the incoming check messages.
__device__ __forceinline__ int vn_sum(const DevCode &C, const BinRule &R, int v, int Lv,
                                      const uint32_t *__restrict__ st) {
    int acc = Lv;
    const int t1 = C.vn_ptr[v + 1];
    for (int t = C.vn_ptr[v]; t < t1; ++t) {
        const int ref = C.vn_ref[t];
        const Unpacked u = unpack(R, st[ref >> 4]);
        acc += bin_r(ref & 15, u.fm1, u.fm2, u.idx, u.signs, u.parity);
    }
    return acc;
}

// Mark every codeword of the workgroup whose current decision violates a check.
__device__ __forceinline__ void syndrome_pass(const DevCode &C, int ncw, const int16_t *lam,
                                              const int *done, int *unsat, bool skip_done) {
    const int n = C.n, m = C.m, T = blockDim.x;
    for (int i = threadIdx.x; i < ncw * m; i += T) {
        const int c = i / m;
        const int row = i - c * m;
        if (skip_done && done[c]) continue;
        const int b = C.row_ptr[row], e1 = C.row_ptr[row + 1];
        uint32_t par = 0;
        for (int e = b; e < e1; ++e) par ^= (uint32_t)(lam[c * n + C.col_idx[e]] < 0);
        if (par) unsat[c] = 1;
    }
}

// Decode codewords [cpw blk, cpw (blk + 1)) with the calling workgroup (any block
// size).  Ends with a barrier, so the caller may reuse the LDS right after.
template <bool LAYERED>
__device__ __forceinline__ void lds_item(const DevCode &C, const BinRule &R, int max_iters, int early_stop, int batch,
                                         int cpw, const DecodeIO &io, int blk, unsigned char *smem) {
    const int n = C.n, m = C.m, E = C.E;
    const int T = blockDim.x, tid = threadIdx.x;
    const int cw0 = blk * cpw;
    const int ncw = min(cpw, batch - cw0);
    if (ncw <= 0) return;
    const LdsLayout lay = lds_layout(n, m, LAYERED, cpw);
    int16_t *lam = (int16_t *)(smem + lay.lam);
    uint32_t *st = (uint32_t *)(smem + lay.st);
    int8_t *Ls = (int8_t *)(smem + lay.L);
    int *unsat = (int *)(smem + lay.flags);
    int *done = unsat + cpw;
    int *itc = done + cpw;

    const int8_t *llr = (const int8_t *)io.llr + (size_t)cw0 * n;
    for (int i = tid; i < ncw * n; i += T) {
        const int8_t l = llr[i];
        lam[i] = l;
        if (!LAYERED) Ls[i] = l;
    }
    for (int i = tid; i < ncw * m; i += T) st[i] = 0u;
    for (int i = tid; i < cpw; i += T) {
        unsat[i] = 0;
        done[i] = i >= ncw;
        itc[i] = 0;
    }
    __syncthreads();

    const int z = C.z > 0 ? C.z : 1;
    for (int k = 1; k <= max_iters; ++k) {
        if (early_stop) {
            syndrome_pass(C, ncw, lam, done, unsat, true);
            __syncthreads();
            if (tid < ncw) {
                if (!done[tid] && !unsat[tid]) done[tid] = 1;
                unsat[tid] = 0;
            }
            __syncthreads();
            int all = 1;
            for (int c = 0; c < ncw; ++c) all &= done[c];
            if (all) break;
        }
        if (LAYERED) {
            for (int l = 0; l < C.nlayers; ++l) {
                for (int i = tid; i < ncw * z; i += T) {
                    const int c = i / z;
                    if (done[c]) continue;
                    const int row = l * z + (i - c * z);
                    st[c * m + row] = row_update<true>(C, R, row, lam + c * n, st[c * m + row]);
                }
                __syncthreads();
            }
        } else {
            for (int i = tid; i < ncw * m; i += T) {
                const int c = i / m;
                if (done[c]) continue;
                const int row = i - c * m;
                st[i] = row_update<false>(C, R, row, lam + c * n, st[i]);
            }
            __syncthreads();
            for (int i = tid; i < ncw * n; i += T) {
                const int c = i / n;
                if (done[c]) continue;
                const int v = i - c * n;
                lam[i] = (int16_t)vn_sum(C, R, v, Ls[i], st + c * m);
            }
            __syncthreads();
        }
        if (tid < ncw && !done[tid]) itc[tid] = k;
    }

    // Syndrome of the final decision.
    __syncthreads();
    if (tid < cpw) unsat[tid] = 0;
    __syncthreads();
    syndrome_pass(C, ncw, lam, done, unsat, false);
    __syncthreads();
    if (tid < ncw) {
        io.ok[cw0 + tid] = unsat[tid] ? 0 : 1;
        io.iters[cw0 + tid] = (int16_t)itc[tid];
    }
    const int nbytes = (n + 7) >> 3;
    uint8_t *hard = (uint8_t *)io.hard + (size_t)cw0 * nbytes;
    for (int i = tid; i < ncw * nbytes; i += T) {
        const int c = i / nbytes;
        const int j = i - c * nbytes;
        uint32_t byte = 0;
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const int v = 8 * j + b;
            if (v < n && lam[c * n + v] < 0) byte |= 1u << b;
        }
        hard[i] = (uint8_t)byte;
    }
    if (io.dump_a) {
        int8_t *dq = (int8_t *)io.dump_a + (size_t)cw0 * E;
        int8_t *dr = (int8_t *)io.dump_b + (size_t)cw0 * E;
        int16_t *dl = (int16_t *)io.dump_c + (size_t)cw0 * n;
        for (int i = tid; i < ncw * m; i += T) {
            const int c = i / m;
            const int row = i - c * m;
            const Unpacked u = unpack(R, st[i]);
            const int b = C.row_ptr[row], e1 = C.row_ptr[row + 1];
            for (int e = b; e < e1; ++e) {
                const int r = bin_r(e - b, u.fm1, u.fm2, u.idx, u.signs, u.parity);
                dr[(size_t)c * E + e] = (int8_t)r;
                dq[(size_t)c * E + e] =
                    (int8_t)clampi((int)lam[c * n + C.col_idx[e]] - r, -R.msg_max, R.msg_max);
            }
        }
        for (int i = tid; i < ncw * n; i += T) dl[i] = lam[i];
    }
    __syncthreads();
}

}  // namespace lds
}  // namespace dev
}  // namespace ldpcx
