// Interleaved binary min-sum decoder (flooding), for codes whose per-codeword
// state does not fit on chip (e.g. n = 64800).
//
// Layout: every per-node quantity is stored as [node][Bp] with the codeword
// index fastest, so a wavefront holds 64 codewords (one per lane) of the same
// node: every gather through the Tanner graph is a uniform (scalar) index and
// every memory access is one contiguous 64-128-256 byte segment.  Per
// iteration one kernel runs the check-node phase (one wave per check and
// 64 codewords) and one the variable-node phase, with compressed check state
// (32 bits per check and codeword) kept in device memory between them.
// Hard decisions are kept as 64-bit lane masks per variable node, so the
// syndrome of 64 codewords is a XOR of dc words per check.
#include "k_common.h"

namespace ldpcx {

namespace {

struct Unp {
    int fm1, fm2, idx;
    uint32_t signs, parity;
};

__device__ __forceinline__ Unp unp(const BinRule &R, uint32_t s) {
    Unp u;
    u.fm1 = bin_norm(R, (int)(s & 127u));
    u.fm2 = bin_norm(R, (int)((s >> 7) & 127u));
    u.idx = (int)((s >> 14) & 15u);
    u.signs = s >> 18;
    u.parity = __popc(u.signs) & 1u;
    return u;
}

__device__ __forceinline__ bool lane_active(int early, const uint64_t *unsat_slot, int g, int lane, int b,
                                            int batch) {
    if (b >= batch) return false;
    return !early || ((unsat_slot[g] >> lane) & 1ull);
}

__global__ void __launch_bounds__(256) k_bil_init(int n, int Bp, int Gn, int batch, const int8_t *__restrict__ L,
                                                  int16_t *__restrict__ lam, uint64_t *__restrict__ hb) {
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (long)n * Bp) return;
    const int v = (int)(i / Bp);
    const int b = (int)(i - (long)v * Bp);
    const int8_t l = L[i];
    lam[i] = l;
    const uint64_t bits = __ballot(l < 0 && b < batch);
    if ((threadIdx.x & 63) == 0) hb[(long)v * Gn + (b >> 6)] = bits;
}

// Syndrome test for every (group of 64 codewords, block of 32 checks): ORs the
// per-check parity masks and records the unsatisfied codewords of each group.
__global__ void __launch_bounds__(256) k_bil_syn(DevCode C, int Gn, const uint64_t *__restrict__ hb,
                                                 uint64_t *__restrict__ unsat_slot) {
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const int g = (int)(t % Gn);
    const int chunk = (int)(t / Gn);
    const int r0 = chunk * 32;
    if (r0 >= C.m) return;
    const int r1 = min(C.m, r0 + 32);
    uint64_t acc = 0;
    for (int row = r0; row < r1; ++row) {
        uint64_t p = 0;
        for (int e = C.row_ptr[row]; e < C.row_ptr[row + 1]; ++e) p ^= hb[(long)C.col_idx[e] * Gn + g];
        acc |= p;
    }
    if (acc) atomicOr((unsigned long long *)&unsat_slot[g], (unsigned long long)acc);
}

__global__ void __launch_bounds__(256) k_bil_cn(DevCode C, BinRule R, int Bp, int early, int batch,
                                                const int16_t *__restrict__ lam, uint32_t *__restrict__ st,
                                                const uint64_t *__restrict__ unsat_slot) {
    const int lane = threadIdx.x & 63;
    const int row = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (row >= C.m) return;
    const int g = blockIdx.y;
    const int b = g * 64 + lane;
    const bool act = lane_active(early, unsat_slot, g, lane, b, batch);
    if (__ballot(act) == 0) return;
    const int e0 = C.row_ptr[row];
    const int dc = C.row_ptr[row + 1] - e0;
    const long off = (long)row * Bp + b;
    const Unp o = unp(R, st[off]);
    const int mm = R.msg_max;
    int m1 = 1 << 20, m2 = 1 << 20, idx = 0;
    uint32_t sg = 0;
#pragma unroll
    for (int j = 0; j < kBinDcMax; ++j) {
        if (j < dc) {
            const int v = C.col_idx[e0 + j];
            const int q = clampi((int)lam[(long)v * Bp + b] - bin_r(j, o.fm1, o.fm2, o.idx, o.signs, o.parity), -mm, mm);
            const int a = q < 0 ? -q : q;
            sg |= (uint32_t)(q < 0) << j;
            if (a < m1) {
                m2 = m1;
                m1 = a;
                idx = j;
            } else if (a < m2) {
                m2 = a;
            }
        }
    }
    if (act) st[off] = st_pack(m1, m2, idx, sg);
}

__global__ void __launch_bounds__(256) k_bil_vn(DevCode C, BinRule R, int Bp, int Gn, int k, int early, int batch,
                                                const int8_t *__restrict__ L, int16_t *__restrict__ lam,
                                                const uint32_t *__restrict__ st, uint64_t *__restrict__ hb,
                                                int16_t *__restrict__ it, const uint64_t *__restrict__ unsat_slot) {
    const int lane = threadIdx.x & 63;
    const int v = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (v >= C.n) return;
    const int g = blockIdx.y;
    const int b = g * 64 + lane;
    const bool act = lane_active(early, unsat_slot, g, lane, b, batch);
    const uint64_t amask = __ballot(act);
    if (amask == 0) return;
    const long off = (long)v * Bp + b;
    int acc = L[off];
    const int t1 = C.vn_ptr[v + 1];
    for (int t = C.vn_ptr[v]; t < t1; ++t) {
        const int ref = C.vn_ref[t];
        const Unp u = unp(R, st[(long)(ref >> 4) * Bp + b]);
        acc += bin_r(ref & 15, u.fm1, u.fm2, u.idx, u.signs, u.parity);
    }
    int fin = acc;
    if (act) lam[off] = (int16_t)acc;
    else fin = lam[off];
    const uint64_t bits = __ballot(fin < 0 && b < batch);
    if (lane == 0) hb[(long)v * Gn + g] = bits;
    if (v == 0 && act) it[b] = (int16_t)k;
}

__global__ void __launch_bounds__(256) k_bil_bytes(int n, int Bp, int Gn, const uint64_t *__restrict__ hb,
                                                   uint8_t *__restrict__ bytes_t) {
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const int nbytes = (n + 7) >> 3;
    if (i >= (long)nbytes * Bp) return;
    const int j = (int)(i / Bp);
    const int b = (int)(i - (long)j * Bp);
    const int g = b >> 6, lane = b & 63;
    uint32_t byte = 0;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const int v = 8 * j + k;
        if (v < n) byte |= (uint32_t)((hb[(long)v * Gn + g] >> lane) & 1ull) << k;
    }
    bytes_t[i] = (uint8_t)byte;
}

__global__ void __launch_bounds__(256) k_bil_fin(int batch, int Gn, const uint64_t *__restrict__ unsat_final,
                                                 const int16_t *__restrict__ it, uint8_t *__restrict__ ok,
                                                 int16_t *__restrict__ iters) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= batch) return;
    ok[b] = ((unsat_final[b >> 6] >> (b & 63)) & 1ull) ? 0 : 1;
    iters[b] = it[b];
}

// Per-edge messages in the interleaved layout, for the debug dump.
__global__ void __launch_bounds__(256) k_bil_dump(DevCode C, BinRule R, int Bp, const int16_t *__restrict__ lam,
                                                  const uint32_t *__restrict__ st, int8_t *__restrict__ q_t,
                                                  int8_t *__restrict__ r_t) {
    const int lane = threadIdx.x & 63;
    const int row = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (row >= C.m) return;
    const int b = blockIdx.y * 64 + lane;
    const Unp u = unp(R, st[(long)row * Bp + b]);
    const int e0 = C.row_ptr[row], e1 = C.row_ptr[row + 1];
    for (int e = e0; e < e1; ++e) {
        const int r = bin_r(e - e0, u.fm1, u.fm2, u.idx, u.signs, u.parity);
        r_t[(long)e * Bp + b] = (int8_t)r;
        q_t[(long)e * Bp + b] = (int8_t)clampi((int)lam[(long)C.col_idx[e] * Bp + b] - r, -R.msg_max, R.msg_max);
    }
}

struct Carve {
    size_t L, lam, st, hb, unsat, it, bytes, total;
};

Carve carve(const DevCode &C, int max_iters, int batch) {
    const size_t Bp = pad64(batch), Gn = Bp / 64;
    Carve c;
    size_t o = 0;
    c.L = o;
    o = align_up(o + (size_t)C.n * Bp, 256);
    c.lam = o;
    o = align_up(o + (size_t)C.n * Bp * 2, 256);
    c.st = o;
    o = align_up(o + (size_t)C.m * Bp * 4, 256);
    c.hb = o;
    o = align_up(o + (size_t)C.n * Gn * 8, 256);
    c.unsat = o;
    o = align_up(o + (size_t)(max_iters + 1) * Gn * 8, 256);
    c.it = o;
    o = align_up(o + Bp * 2, 256);
    c.bytes = o;
    o = align_up(o + (size_t)((C.n + 7) / 8) * Bp, 256);
    c.total = o;
    return c;
}

}  // namespace

size_t bin_il_work_bytes(const DevCode &C, int max_iters, int batch) { return carve(C, max_iters, batch).total; }

void bin_il_carve(void *base, const DevCode &C, int max_iters, int batch, BinIlWork &w) {
    const Carve c = carve(C, max_iters, batch);
    char *p = (char *)base;
    w.L = (int8_t *)(p + c.L);
    w.lam = (int16_t *)(p + c.lam);
    w.st = (uint32_t *)(p + c.st);
    w.hb = (uint64_t *)(p + c.hb);
    w.unsat = (uint64_t *)(p + c.unsat);
    w.it = (int16_t *)(p + c.it);
    // the packed-byte staging buffer follows `it`
}

#define LDPCX_CHECK(x)                           \
    do {                                         \
        hipError_t e_ = (x);                     \
        if (e_ != hipSuccess) return e_;         \
    } while (0)

hipError_t launch_bin_il(const DevCode &C, const BinRule &R, int max_iters, int early_stop, int batch,
                         const BinIlWork &w, const DecodeIO &io, hipStream_t s) {
    const int Bp = pad64(batch), Gn = Bp / 64;
    const int n = C.n, m = C.m;
    const Carve cv = carve(C, max_iters, batch);
    uint8_t *bytes_t = (uint8_t *)((char *)w.L + (cv.bytes - cv.L));
    LDPCX_CHECK(transpose<int8_t>((const int8_t *)io.llr, batch, n, n, w.L, Bp, Bp, s));
    {
        const long tot = (long)n * Bp;
        hipLaunchKernelGGL(k_bil_init, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, n, Bp, Gn, batch, w.L,
                           w.lam, w.hb);
        LDPCX_CHECK(hipGetLastError());
    }
    LDPCX_CHECK(fill_u32(w.st, (size_t)m * Bp * 4, 0u, s));
    LDPCX_CHECK(fill_u32(w.unsat, (size_t)(max_iters + 1) * Gn * 8, 0u, s));
    LDPCX_CHECK(fill_u32(w.it, align_up((size_t)Bp * 2, 4), 0u, s));
    const dim3 blk(256);
    const dim3 gcn((unsigned)((m + 3) / 4), (unsigned)Gn);
    const dim3 gvn((unsigned)((n + 3) / 4), (unsigned)Gn);
    const long syn_threads = (long)((m + 31) / 32) * Gn;
    const dim3 gsyn((unsigned)((syn_threads + 255) / 256));
    for (int k = 1; k <= max_iters; ++k) {
        uint64_t *slot = w.unsat + (size_t)k * Gn;
        if (early_stop) hipLaunchKernelGGL(k_bil_syn, gsyn, blk, 0, s, C, Gn, w.hb, slot);
        hipLaunchKernelGGL(k_bil_cn, gcn, blk, 0, s, C, R, Bp, early_stop, batch, w.lam, w.st, slot);
        hipLaunchKernelGGL(k_bil_vn, gvn, blk, 0, s, C, R, Bp, Gn, k, early_stop, batch, w.L, w.lam, w.st, w.hb,
                           w.it, slot);
        LDPCX_CHECK(hipGetLastError());
    }
    hipLaunchKernelGGL(k_bil_syn, gsyn, blk, 0, s, C, Gn, w.hb, w.unsat);
    hipLaunchKernelGGL(k_bil_fin, dim3((unsigned)((batch + 255) / 256)), blk, 0, s, batch, Gn, w.unsat, w.it, io.ok,
                       io.iters);
    const int nbytes = (n + 7) / 8;
    {
        const long tot = (long)nbytes * Bp;
        hipLaunchKernelGGL(k_bil_bytes, dim3((unsigned)((tot + 255) / 256)), blk, 0, s, n, Bp, Gn, w.hb, bytes_t);
    }
    LDPCX_CHECK(hipGetLastError());
    LDPCX_CHECK(transpose<uint8_t>(bytes_t, nbytes, batch, Bp, (uint8_t *)io.hard, nbytes, nbytes, s));
    return hipSuccess;
}

hipError_t launch_bin_il_dump(const DevCode &C, const BinRule &R, int batch, const BinIlWork &w, int8_t *q_t,
                              int8_t *r_t, void *dq, void *dr, void *dlam, hipStream_t s) {
    const int Bp = pad64(batch), Gn = Bp / 64;
    hipLaunchKernelGGL(k_bil_dump, dim3((unsigned)((C.m + 3) / 4), (unsigned)Gn), dim3(256), 0, s, C, R, Bp, w.lam,
                       w.st, q_t, r_t);
    LDPCX_CHECK(hipGetLastError());
    LDPCX_CHECK(transpose<int8_t>(q_t, C.E, batch, Bp, (int8_t *)dq, C.E, C.E, s));
    LDPCX_CHECK(transpose<int8_t>(r_t, C.E, batch, Bp, (int8_t *)dr, C.E, C.E, s));
    LDPCX_CHECK(transpose<int16_t>(w.lam, C.n, batch, Bp, (int16_t *)dlam, C.n, C.n, s));
    return hipSuccess;
}

}  // namespace ldpcx
