// Ragged persistent engine: one kernel launch decodes a batch of jobs over
// different codes, sizes and decoder families.
//
// Every job is cut into workgroup-local items that share nothing with other
// items, so no workgroup ever waits for another and the launch cannot deadlock
// whatever the residency of its workgroups:
//   - quasi-cyclic jobs: one item per 2 * npairs codewords (packed decoder);
//   - other binary codes whose state fits on chip: one item per cpw codewords
//     (LDS-resident decoder);
//   - long binary codes (interleaved layout) and Min-Max jobs: one item per
//     group of 64 codewords, running every phase of the interleaved decoder
//     (layout transpose, init, per iteration syndrome test, check nodes and
//     variable nodes, then the final test and the outputs) inside one
//     workgroup, with a barrier between phases.  Items of one job touch
//     disjoint lanes of the job's workspace.  An item stops iterating as soon
//     as none of its codewords is unsatisfied, which gives the same results as
//     running the remaining iterations with every lane inactive.
// The host estimates the cost of every item, sorts them longest first and
// assigns them greedily to the least-loaded workgroup of a grid sized to the
// resident capacity of the device (LPT schedule); each workgroup then runs its
// own list.
#include <algorithm>
#include <cstdio>
#include <cstring>
#include <queue>
#include <vector>

#include "dev_bin_il.h"
#include "dev_bin_lds.h"
#include "dev_bin_qc.h"
#include "dev_nb.h"
#include "runtime.h"

namespace ldpcx {

namespace {

enum ItemType { I_QC = 0, I_LDS = 1, I_IL = 2, I_NB = 3 };

struct JobDesc {
    int family, layered, npairs, cpw, ml, md;
    QcDesc qc;
    DevCode C;
    BinRule R;
    int max_iters, early_stop, batch;
    DecodeIO io;
    dev::il::Args il;
    dev::nb::Args nb;
    dev::TransposeArgs tin, tout;
};

struct Item {
    int type, job, blk, pad;
};

constexpr int kThreads = 256;
constexpr size_t kTileBytes = 64 * 65 * 2;
constexpr size_t kStaticLds = 256;  // upper bound of the kernel's static LDS

template <bool LAYERED>
__device__ __forceinline__ void run_qc(const JobDesc &J, int blk, uint32_t *lds) {
#define LDPCX_QC_RUN(L_, D_)                                                                                     \
    if (J.ml == L_ && J.md == D_) {                                                                              \
        dev::qc_item<L_, D_, LAYERED>(J.qc, J.C, J.R, J.max_iters, J.early_stop, J.batch, J.npairs, J.io, blk, \
                                      lds);                                                                      \
        return;                                                                                                  \
    }
    LDPCX_QC_SHAPES(LDPCX_QC_RUN)
#undef LDPCX_QC_RUN
}

// OR of one 64-bit mask per wave over the workgroup, written to unsat[slot][g];
// returns the result (uniform).
__device__ __forceinline__ uint64_t group_or(uint64_t v, uint64_t *unsat, long slot_word, uint64_t *red) {
    v = dev::wave_or64(v);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    const uint64_t u = red[0] | red[1] | red[2] | red[3];
    if (threadIdx.x == 0) unsat[slot_word] = u;
    __syncthreads();
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)u);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(u >> 32));
    return ((uint64_t)hi << 32) | lo;
}

// ------------------------------------------------ interleaved binary, one group
// Syndrome of one group of codewords: the kLaneCw decision words of group g in
// slot_k; returns their OR (uniform).
__device__ uint64_t il_syn(const dev::il::Args &A, int slot_k, int g, uint64_t *red) {
    constexpr int H = dev::il::kLaneCw;
    const DevCode &C = A.C;
    const int W = H * A.G;
    uint64_t acc[H];
    for (int h = 0; h < H; ++h) acc[h] = 0;
    for (int row = threadIdx.x; row < C.m; row += kThreads) {
        uint64_t p[H];
        for (int h = 0; h < H; ++h) p[h] = 0;
        for (int e = C.row_ptr[row]; e < C.row_ptr[row + 1]; ++e) {
            const uint64_t *hw = A.w.hb + (size_t)C.col_idx[e] * W + (size_t)H * g;
            for (int h = 0; h < H; ++h) p[h] ^= hw[h];
        }
        for (int h = 0; h < H; ++h) acc[h] |= p[h];
    }
    const int w = threadIdx.x >> 6;
    for (int h = 0; h < H; ++h) {
        acc[h] = dev::wave_or64(acc[h]);
        if ((threadIdx.x & 63) == 0) red[H * w + h] = acc[h];
    }
    __syncthreads();
    uint64_t u = 0;
    if (threadIdx.x < H) {
        uint64_t x = 0;
        for (int q = 0; q < kThreads / 64; ++q) x |= red[H * q + threadIdx.x];
        A.w.unsat[(size_t)slot_k * W + (size_t)H * g + threadIdx.x] = x;
    }
    for (int i = 0; i < H * (kThreads / 64); ++i) u |= red[i];
    __syncthreads();
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)u);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(u >> 32));
    return ((uint64_t)hi << 32) | lo;
}

// Every phase of the interleaved binary decoder for the codewords of group g.
__device__ void il_group(const JobDesc &J, int g, uint32_t *lds, uint64_t *red) {
    using namespace dev::il;
    const Args &A = J.il;
    const DevCode &C = A.C;
    constexpr int Q = kGroup / 64;  // 64-row transpose tiles per group
    unsigned char *tile = (unsigned char *)lds;
    const long gx_in = dev::transpose_gx(J.tin);
    for (int qt = 0; qt < Q; ++qt)
        for (long bx = 0; bx < gx_in; ++bx) dev::transpose_block(J.tin, bx, Q * g + qt, tile);
    for (int s = threadIdx.x; s < (A.max_iters + 1) * kLaneCw; s += kThreads)
        A.w.unsat[((size_t)(s / kLaneCw) * A.G + g) * kLaneCw + s % kLaneCw] = 0;
    for (int t = threadIdx.x; t < kGroup; t += kThreads) A.w.it[g * kGroup + t] = 0;
    __syncthreads();
    const int ge = (int)grid_edges_x(A), gv = (int)grid_vars_x(A), gr = (int)grid_rows_x(A);
    for (int bx = 0; bx < ge; ++bx) init_edges_block(A, bx, g);
    for (int bx = 0; bx < gv; ++bx) init_vars_block(A, bx, g);
    __syncthreads();
    for (int k = 1; k <= A.max_iters; ++k) {
        if (A.early_stop && il_syn(A, k, g, red) == 0) break;
        if (C.dc_max <= 8)
            for (int bx = 0; bx < gr; ++bx) cn_block<8>(A, k, bx, g);
        else
            for (int bx = 0; bx < gr; ++bx) cn_block<kBinDcMax>(A, k, bx, g);
        __syncthreads();
        for (int bx = 0; bx < gv; ++bx) vn_block(A, k, bx, g);
        __syncthreads();
    }
    il_syn(A, 0, g, red);
    for (int t = threadIdx.x; t < kGroup; t += kThreads) {
        const int b = g * kGroup + t;
        if (b < A.batch) {
            A.io.ok[b] = unsat_bit(A, 0, b) ? 0 : 1;
            A.io.iters[b] = A.w.it[b];
        }
    }
    const int nbytes = (C.n + 7) >> 3;
    for (int idx = threadIdx.x; idx < nbytes * kGroup; idx += kThreads) {
        const int j = idx / kGroup, b = g * kGroup + idx % kGroup;
        uint32_t byte = 0;
        for (int q = 0; q < 8; ++q) {
            const int v = 8 * j + q;
            if (v < C.n) byte |= hbit(A, v, b) << q;
        }
        A.bytes_t[(size_t)j * A.Bp + b] = (uint8_t)byte;
    }
    __syncthreads();
    const long gy_out = dev::transpose_gy(J.tout);
    for (int qt = 0; qt < Q; ++qt)
        for (long by = 0; by < gy_out; ++by) dev::transpose_block(J.tout, Q * g + qt, by, tile);
}

// --------------------------------------------------------- Min-Max, one group
__device__ uint64_t nb_syn(const dev::nb::Args &A, int slot_k, int g, uint64_t *red) {
    const DevCode &C = A.C;
    const int lane = threadIdx.x & 63, w = dev::wave_id();
    const int b = g * 64 + lane;
    uint64_t acc = 0;
    for (int row = w; row < C.m; row += 4) {
        int s = 0;
        for (int e = C.row_ptr[row]; e < C.row_ptr[row + 1]; ++e)
            s ^= C.gfmul[C.h[e] * C.g + A.w.hard[(long)C.col_idx[e] * A.Bp + b]];
        acc |= __ballot(s != 0 && b < A.batch);
    }
    return group_or(acc, A.w.unsat, (long)slot_k * A.Gn + g, red);
}

template <int G>
__device__ void nb_group(const JobDesc &J, int g, uint32_t *lds, uint64_t *red) {
    const dev::nb::Args &A = J.nb;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int b = g * 64 + lane;
    unsigned char *tile = (unsigned char *)lds;
    const long gx_in = dev::transpose_gx(J.tin);
    for (long bx = 0; bx < gx_in; ++bx) dev::transpose_block(J.tin, bx, g, tile);
    for (int s = threadIdx.x; s <= A.max_iters; s += kThreads) A.w.unsat[(long)s * A.Gn + g] = 0;
    if (w == 0) A.w.it[b] = 0;
    const int gi = (int)dev::nb::grid_init_x(A);
    for (int bx = 0; bx < gi; ++bx) dev::nb::init_block<G>(A, bx, g);
    __syncthreads();
    const int gr = (int)dev::nb::grid_rows_x(A), gv = (int)dev::nb::grid_vn_x(A);
    for (int k = 1; k <= A.max_iters; ++k) {
        if (A.early_stop && nb_syn(A, k, g, red) == 0) break;
        for (int bx = 0; bx < gr; ++bx) dev::nb::cn_block<G>(A, k, 4, bx, g, lds);
        __syncthreads();
        for (int bx = 0; bx < gv; ++bx) dev::nb::vn_block<G>(A, k, bx, g);
        __syncthreads();
    }
    const uint64_t u = nb_syn(A, 0, g, red);
    if (w == 0 && b < A.batch) {
        A.io.ok[b] = ((u >> lane) & 1ull) ? 0 : 1;
        A.io.iters[b] = A.w.it[b];
    }
    const long gy_out = dev::transpose_gy(J.tout);
    for (long by = 0; by < gy_out; ++by) dev::transpose_block(J.tout, g, by, tile);
}

// IL: whether the interleaved families are compiled in (they dominate the register
// budget, so mixes of workgroup-resident codes run a variant without them).
template <bool IL>
__device__ __forceinline__ void run_item(const JobDesc &J, const Item &it, uint32_t *lds, uint64_t *red) {
    switch (it.type) {
    case I_QC:
        if (J.layered) run_qc<true>(J, it.blk, lds);
        else run_qc<false>(J, it.blk, lds);
        break;
    case I_LDS:
        if (J.layered)
            dev::lds::lds_item<true>(J.C, J.R, J.max_iters, J.early_stop, J.batch, J.cpw, J.io, it.blk,
                                     (unsigned char *)lds);
        else
            dev::lds::lds_item<false>(J.C, J.R, J.max_iters, J.early_stop, J.batch, J.cpw, J.io, it.blk,
                                      (unsigned char *)lds);
        break;
    case I_IL:
        if (IL) il_group(J, it.blk, lds, red);
        break;
    default:
        if (!IL) break;
        switch (J.C.g) {
        case 4: nb_group<4>(J, it.blk, lds, red); break;
        case 8: nb_group<8>(J, it.blk, lds, red); break;
        case 16: nb_group<16>(J, it.blk, lds, red); break;
        case 32: nb_group<32>(J, it.blk, lds, red); break;
        case 64: nb_group<64>(J, it.blk, lds, red); break;
        default: break;  // other fields never become items (rejected on the host)
        }
    }
}

// Workgroup w runs items [wg_ptr[w], wg_ptr[w + 1]) in order.
template <bool IL>
__global__ void __launch_bounds__(kThreads) k_ragged(const JobDesc *__restrict__ jobs,
                                                     const Item *__restrict__ items,
                                                     const int *__restrict__ wg_ptr) {
    extern __shared__ __align__(16) uint32_t lds[];
    __shared__ uint64_t red[4 * dev::il::kLaneCw];
    const int i0 = wg_ptr[blockIdx.x], i1 = wg_ptr[blockIdx.x + 1];
    for (int i = i0; i < i1; ++i) {
        const Item it = items[i];
        run_item<IL>(jobs[it.job], it, lds, red);
        __syncthreads();
    }
}

// Relative cost of one item (arbitrary units, only compared with each other).
double item_cost(const JobDesc &J, const DevCode &C) {
    const double it = std::max(1, J.max_iters), E = C.E;
    switch (J.family) {
    case FAMILY_BIN_QC: return it * E * 2.0 / std::max(1, J.qc.Z);
    case FAMILY_BIN_LDS: return it * E * J.cpw / kThreads;
    case FAMILY_BIN_IL: return it * E * (double)dev::il::kGroup * 2.0 / kThreads;
    default: return it * E * 3.0 * C.g * C.g / 2.0 * 64.0 / kThreads / 8.0;
    }
}

}  // namespace

}  // namespace ldpcx

using namespace ldpcx;

extern "C" ldpcx_status ldpcx_decode_ragged(const ldpcx_job *jobs, int32_t njobs, void *stream) {
    try {
        if (njobs < 0 || (njobs > 0 && !jobs)) return fail(LDPCX_E_INVAL, "bad job list");
        if (njobs == 0) return LDPCX_OK;
        hipStream_t s = (hipStream_t)stream;
        std::vector<JobDesc> J(njobs);
        std::vector<Item> items;
        std::vector<double> cost;
        std::vector<void *> workspaces;
        auto cleanup = [&]() {
            for (void *w : workspaces) (void)hipFreeAsync(w, s);
        };
        int device = -1;
        size_t lds = kTileBytes;
        for (int j = 0; j < njobs; ++j) {
            const ldpcx_job &jb = jobs[j];
            if (!jb.code) return cleanup(), fail(LDPCX_E_INVAL, "job without code");
            ldpcx_code *c = const_cast<ldpcx_code *>(jb.code);
            ldpcx_status st = check_params(c, &jb.params);
            if (st != LDPCX_OK) return cleanup(), st;
            if (c->nb_unsupported) return cleanup(), fail(LDPCX_E_UNSUPPORTED, "no Min-Max kernel for this field size");
            if (jb.params.rule == LDPCX_RULE_SPA)
                return cleanup(), fail(LDPCX_E_UNSUPPORTED, "the FFT-SPA decoder has no workgroup-local item; decode "
                                                            "it with ldpcx_decode");
            if (c->g > 64)
                return cleanup(), fail(LDPCX_E_UNSUPPORTED, "fields above GF(64) have no workgroup-local item; decode them "
                                                            "with ldpcx_decode");
            if (device < 0) {
                if ((st = check_device(c)) != LDPCX_OK) return cleanup(), st;
                device = c->device;
            } else if (c->device != device) {
                return cleanup(), fail(LDPCX_E_INVAL, "jobs on different devices");
            }
            if (jb.batch < 0) return cleanup(), fail(LDPCX_E_INVAL, "batch < 0");
            if (jb.batch == 0) continue;
            if (!jb.llr || !jb.hard || !jb.syndrome_ok || !jb.iters) return cleanup(), fail(LDPCX_E_INVAL, "null buffer");
            const ldpcx_decode_params &p = jb.params;
            // Dynamic LDS available next to the kernel's own small static array.
            const size_t cap = (size_t)device_info(device).lds_per_block - kStaticLds;
            Plan pl = plan_for(c, &p, jb.batch);
            JobDesc &D = J[j];
            std::memset(&D, 0, sizeof D);
            D.C = c->dev;
            D.R = bin_rule(&p);
            D.max_iters = p.max_iters;
            D.early_stop = p.early_stop;
            D.batch = jb.batch;
            D.io = DecodeIO{jb.llr, jb.hard, jb.syndrome_ok, jb.iters, nullptr, nullptr, nullptr};
            D.layered = pl.schedule == LDPCX_SCHED_LAYERED;
            if (pl.family == FAMILY_NB && D.layered)
                return cleanup(), fail(LDPCX_E_UNSUPPORTED, "layered Min-Max runs through ldpcx_decode only");
            auto add = [&](int type, long count) {
                for (long i = 0; i < count; ++i) items.push_back(Item{type, j, (int)i, 0});
                const double cst = item_cost(D, D.C);
                cost.insert(cost.end(), (size_t)count, cst);
            };
            // Workgroup-local items run in workgroups of kThreads threads.
            if (pl.family == FAMILY_BIN_QC && c->qc.Z > kThreads) pl.family = FAMILY_BIN_LDS;
            if (pl.family == FAMILY_BIN_QC) {
                int ml, md;
                dev::qc_shape_of(c->qc, ml, md);
                if (!ml) {
                    pl.family = FAMILY_BIN_LDS;
                } else {
                    int np = std::max(1, std::min(pl.cpw / 2, kThreads / c->qc.Z));
                    while (np > 1 && dev::qc_smem_bytes(ml, md, D.C, c->qc.Z, D.layered, np) > cap)
                        --np;
                    D.family = FAMILY_BIN_QC;
                    D.qc = c->qc;
                    D.npairs = np;
                    D.ml = ml;
                    D.md = md;
                    lds = std::max(lds, dev::qc_smem_bytes(ml, md, D.C, c->qc.Z, D.layered, np));
                    add(I_QC, ((jb.batch + 1) / 2 + np - 1) / np);
                    continue;
                }
            }
            if (pl.family == FAMILY_BIN_LDS) {
                const size_t per_cw = bin_lds_smem_bytes(D.C, D.layered, 1);
                if (per_cw > cap)
                    return cleanup(), fail(LDPCX_E_UNSUPPORTED, "code state does not fit the LDS of one workgroup");
                int cpw = std::max(1, pl.cpw);
                while (cpw > 1 && bin_lds_smem_bytes(D.C, D.layered, cpw) > cap) --cpw;
                D.family = FAMILY_BIN_LDS;
                D.cpw = cpw;
                lds = std::max(lds, bin_lds_smem_bytes(D.C, D.layered, cpw));
                add(I_LDS, (jb.batch + cpw - 1) / cpw);
                continue;
            }
            // Interleaved families: a workspace per job, one item per group of 64 codewords.
            D.family = pl.family;
            if ((pl.family == FAMILY_BIN_IL && jb.batch > dev::il::max_sub_batch(D.C)) ||
                (pl.family == FAMILY_NB && jb.batch > nb_slice(D.C, jb.batch + 64)))
                return cleanup(), fail(LDPCX_E_UNSUPPORTED, "batch too large for one interleaved workspace");
            const size_t bytes = pl.family == FAMILY_BIN_IL ? dev::il::carve(D.C, p.max_iters, jb.batch).total
                                                            : nb_work_bytes(D.C, p.max_iters, jb.batch);
            void *ws = nullptr;
            if (hipMallocAsync(&ws, bytes, s) != hipSuccess) return cleanup(), fail(LDPCX_E_NOMEM, "workspace");
            workspaces.push_back(ws);
            if (pl.family == FAMILY_BIN_IL) {
                D.il = dev::il::make_args(D.C, D.R, p.max_iters, p.early_stop, jb.batch, ws, D.io);
                D.tin = dev::il::tr_in(D.il);
                D.tout = dev::il::tr_out(D.il);
                add(I_IL, D.il.G);
            } else {
                const long groups = pad64(jb.batch) / 64;
                D.nb = dev::nb::make_args(D.C, p.max_iters, p.early_stop, jb.batch, nb_amax(&p), ws, D.io);
                const size_t need = dev::nb::cn_lds_bytes(D.nb, 4);
                if (need > cap)
                    return cleanup(), fail(LDPCX_E_UNSUPPORTED, "check degree too large for the persistent engine");
                lds = std::max(lds, need);
                D.tin = dev::nb::tr_in(D.nb);
                D.tout = dev::nb::tr_out(D.nb);
                add(I_NB, groups);
            }
        }
        if (items.empty()) return cleanup(), LDPCX_OK;
        if (lds > (size_t)device_info(device).lds_per_block - kStaticLds)
            return cleanup(), fail(LDPCX_E_UNSUPPORTED, "job mix needs more LDS than one workgroup has");

        // Errors of the calls above were checked where they happened; clear the sticky
        // last-error state so that the launch check below reports the launch only.
        (void)hipGetLastError();
        bool any_il = false;
        for (const Item &it : items) any_il |= it.type == I_IL || it.type == I_NB;
        const void *kern = any_il ? (const void *)k_ragged<true> : (const void *)k_ragged<false>;
        if (lds > 64 * 1024) {
            hipError_t ea = hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
            if (ea != hipSuccess) return cleanup(), fail_hip(ea, "persistent kernel LDS attribute");
        }
        int per_cu = 0;
        hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, kThreads, lds);
        if (e != hipSuccess || per_cu < 1) return cleanup(), fail(LDPCX_E_UNSUPPORTED, "persistent kernel does not fit");
        const int grid = (int)std::min<long>((long)per_cu * device_info(device).cus, (long)items.size());

        // LPT: longest item first, each to the least-loaded workgroup.
        std::vector<int> order(items.size());
        for (size_t i = 0; i < order.size(); ++i) order[i] = (int)i;
        std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cost[a] > cost[b]; });
        std::vector<std::vector<int>> lists(grid);
        {
            typedef std::pair<double, int> Load;
            std::priority_queue<Load, std::vector<Load>, std::greater<Load>> heap;
            for (int w = 0; w < grid; ++w) heap.push(Load(0.0, w));
            for (int i : order) {
                Load l = heap.top();
                heap.pop();
                lists[l.second].push_back(i);
                heap.push(Load(l.first + cost[i], l.second));
            }
        }
        std::vector<Item> flat;
        std::vector<int> wg_ptr(grid + 1, 0);
        flat.reserve(items.size());
        for (int w = 0; w < grid; ++w) {
            for (int i : lists[w]) flat.push_back(items[i]);
            wg_ptr[w + 1] = (int)flat.size();
        }

        // One device table: jobs, items, workgroup ranges.
        const size_t o_items = align_up(sizeof(JobDesc) * njobs, 256);
        const size_t o_ptr = align_up(o_items + sizeof(Item) * flat.size(), 256);
        const size_t total = align_up(o_ptr + sizeof(int) * wg_ptr.size(), 256);
        char *dbuf = nullptr;
        if (hipMallocAsync((void **)&dbuf, total, s) != hipSuccess) return cleanup(), fail(LDPCX_E_NOMEM, "item table");
        workspaces.push_back(dbuf);
        std::vector<char> host(total, 0);
        std::memcpy(host.data(), J.data(), sizeof(JobDesc) * njobs);
        std::memcpy(host.data() + o_items, flat.data(), sizeof(Item) * flat.size());
        std::memcpy(host.data() + o_ptr, wg_ptr.data(), sizeof(int) * wg_ptr.size());
        ldpcx_status st = upload_async(dbuf, host.data(), total, device, s);
        if (st != LDPCX_OK) return cleanup(), st;
        const JobDesc *djobs = (const JobDesc *)dbuf;
        const Item *ditems = (const Item *)(dbuf + o_items);
        const int *dptr = (const int *)(dbuf + o_ptr);
        if (any_il) hipLaunchKernelGGL(k_ragged<true>, dim3(grid), dim3(kThreads), lds, s, djobs, ditems, dptr);
        else hipLaunchKernelGGL(k_ragged<false>, dim3(grid), dim3(kThreads), lds, s, djobs, ditems, dptr);
        e = hipGetLastError();
        cleanup();
        if (e != hipSuccess) {
            char msg[160];
            snprintf(msg, sizeof msg, "persistent kernel launch (grid %d, %zu bytes of LDS)", grid, lds);
            return fail_hip(e, msg);
        }
        return LDPCX_OK;
    } catch (const std::exception &ex) {
        return fail(LDPCX_E_NOMEM, ex.what());
    }
}
