// Ragged batches: one call decodes a batch of jobs over different codes, sizes and
// decoder families.
//
// Jobs of the workgroup-local families run as items of one persistent kernel.  Every
// such job is cut into items that share nothing with other items, so no workgroup
// ever waits for another and the launch cannot deadlock whatever the residency of its
// workgroups:
//   - quasi-cyclic jobs: one item per 2 * npairs codewords (packed decoder);
//   - other binary codes whose state fits on chip: one item per cpw codewords
//     (LDS-resident decoder);
//   - Min-Max over GF(4)..GF(64) whose messages of one codeword fit a workgroup's LDS:
//     one item per codeword (lanes over field entries, every message in LDS);
//   - FFT-SPA codes of the LDS-resident family: one item per group of codewords.
// Items run as up to five launches of the persistent kernel, one after the other on
// the stream, each an instance compiled for one kind of item: binary items (256
// threads), Min-Max items of check degree <= 4 (1024 threads: one codeword's checks
// spread over 16 waves), alpha-free Min-Max items over GF(64) (512 threads at 128
// VGPRs: two codewords per compute unit), Min-Max items of larger check degree (256
// threads, for their larger register arrays) and FFT-SPA items (1024 threads).  A
// kernel's register and LDS allocation is the maximum over what it may run, so each
// kind keeps the occupancy its own footprint allows.
// The host estimates the cost of every item and sorts them longest first; a grid
// sized to the resident capacity of the device then takes items from that list
// through one device counter: each workgroup claims the next item with one atomic
// add, runs it, and claims again until the list is exhausted.  A workgroup whose
// item stops early (every codeword's syndrome satisfied) therefore moves on at once,
// so the load stays balanced under early termination without any estimate of it,
// and no workgroup ever waits for another.
//
// Jobs whose state does not fit a workgroup (long binary codes in the interleaved
// layout, Min-Max over GF(128) and GF(256) or with larger codewords, FFT-SPA outside its
// LDS-resident family) would leave one workgroup to sweep every check and variable
// of a group of codewords in device memory, each iteration, alone.  They are gathered
// instead per (code, parameters, resolved schedule) into one batch and run as that
// batch's own launch sequence on the same stream, after the persistent kernel;
// codewords are decoded independently, so every job still gets exactly what a decode
// of it alone gives.
#include <algorithm>
#include <cstdio>
#include <cstring>
#include <vector>

#include "dev_bin_lds.h"
#include "dev_bin_qc.h"
#include "dev_nb1.h"
#include "dev_spa.h"
#include "runtime.h"

namespace ldpcx {

namespace {

enum ItemType { I_QC = 0, I_LDS = 1, I_NB1 = 2, I_SPA = 3 };

struct JobDesc {
    int family, layered, npairs, cpw, ml, md;
    QcDesc qc;
    DevCode C;
    BinRule R;
    int max_iters, early_stop, batch, amax;
    int af;  // Min-Max items: alpha-free decoding
    DecodeIO io;
};

struct Item {
    int type, job, blk, pad;
};

constexpr int kThreads = 256;  // binary items (their decoders use at most 256 threads)
constexpr size_t kStaticLds = 256;  // upper bound of the kernel's static LDS
enum Kind { K_BIN = 0, K_GF4 = 1, K_GF16 = 2, K_SPA = 3, K_AF = 4 };
constexpr int kKinds = 5;
// Min-Max items of check degree up to 4 and FFT-SPA items run in workgroups of 1024
// threads; alpha-free Min-Max items in workgroups of 512 threads capped at 128 VGPRs,
// so that two share a compute unit (78 KB of LDS per GF(64) codeword).
__host__ __device__ constexpr int kind_threads(int k) {
    return k == K_GF4 || k == K_SPA ? 1024 : k == K_AF ? 512 : 256;
}

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

// Alpha-free items over GF(64) only: with the other fields' alpha-free decoders in the
// same kernel instance its registers spill past 128 VGPRs.
constexpr int kAfField = 64;

template <int DC, class M>
__device__ __forceinline__ void run_nb1_m(const JobDesc &J, int b, uint32_t *lds) {
    const dev::nb1::Job N{J.C, J.max_iters, J.early_stop, J.layered, J.amax, J.batch, J.io};
    unsigned char *l = (unsigned char *)lds;
    switch (J.C.g) {
    case 4: dev::nb1::decode_cw<4, DC, M>(N, b, l); break;
    case 8: dev::nb1::decode_cw<8, DC, M>(N, b, l); break;
    case 16: dev::nb1::decode_cw<16, DC, M>(N, b, l); break;
    case 32: dev::nb1::decode_cw<32, DC, M>(N, b, l); break;
    default: dev::nb1::decode_cw<64, DC, M>(N, b, l); break;
    }
}

// Alpha-free item: the host marks only GF(64) jobs of check degree <= 4 alpha-free.
template <class M>
__device__ __forceinline__ void run_nb1_af_m(const JobDesc &J, int b, uint32_t *lds) {
    const dev::nb1::Job N{J.C, J.max_iters, J.early_stop, J.layered, J.amax, J.batch, J.io};
    dev::nb1::decode_cw<kAfField, 4, M, true>(N, b, (unsigned char *)lds);
}

template <int DC>
__device__ __forceinline__ void run_nb1(const JobDesc &J, int b, uint32_t *lds) {
    if (dev::nb1::msg_bytes(J.amax) == 1) run_nb1_m<DC, uint8_t>(J, b, lds);
    else run_nb1_m<DC, int16_t>(J, b, lds);
}

__device__ __forceinline__ void run_nb1_af(const JobDesc &J, int b, uint32_t *lds) {
    if (dev::nb1::msg_bytes(J.amax) == 1) run_nb1_af_m<uint8_t>(J, b, lds);
    else run_nb1_af_m<int16_t>(J, b, lds);
}

__device__ __forceinline__ void run_spa(const JobDesc &J, int blk, uint32_t *lds) {
    dev::spa::Args A;
    A.C = J.C;
    A.max_iters = J.max_iters;
    A.early_stop = J.early_stop;
    A.batch = J.batch;
    A.w = SpaWork{};
    A.io = J.io;
    unsigned char *l = (unsigned char *)lds;
    switch (J.C.g) {
    case 4: dev::spa::lds_decode<4>(A, J.cpw, l, blk); break;
    case 8: dev::spa::lds_decode<8>(A, J.cpw, l, blk); break;
    case 16: dev::spa::lds_decode<16>(A, J.cpw, l, blk); break;
    case 32: dev::spa::lds_decode<32>(A, J.cpw, l, blk); break;
    default: dev::spa::lds_decode<64>(A, J.cpw, l, blk); break;
    }
}

template <int K>
__device__ __forceinline__ void run_item(const JobDesc &J, const Item &it, uint32_t *lds) {
    if (K == K_GF4) {
        run_nb1<4>(J, it.blk, lds);
    } else if (K == K_AF) {
        run_nb1_af(J, it.blk, lds);
    } else if (K == K_SPA) {
        run_spa(J, it.blk, lds);
    } else if (K == K_GF16) {
        run_nb1<kNbDcMax>(J, it.blk, lds);
    } else if (it.type == I_QC) {
        if (J.layered) run_qc<true>(J, it.blk, lds);
        else run_qc<false>(J, it.blk, lds);
    } else if (J.layered) {
        dev::lds::lds_item<true>(J.C, J.R, J.max_iters, J.early_stop, J.batch, J.cpw, J.io, it.blk,
                                 (unsigned char *)lds);
    } else {
        dev::lds::lds_item<false>(J.C, J.R, J.max_iters, J.early_stop, J.batch, J.cpw, J.io, it.blk,
                                  (unsigned char *)lds);
    }
}

// Every workgroup claims items from the shared counter (zero at launch) until the
// list is exhausted.  Claims are the only inter-workgroup interaction: an atomic add
// that never waits, so the launch completes whatever the residency of its workgroups.
template <int K>
__device__ __forceinline__ void claim_loop(const JobDesc *__restrict__ jobs, const Item *__restrict__ items,
                                           int nitems, int *__restrict__ next, uint32_t *lds, int &claim) {
    for (;;) {
        if (threadIdx.x == 0) claim = atomicAdd(next, 1);
        __syncthreads();
        const int i = claim;
        __syncthreads();  // every thread has read the claim before thread 0 overwrites it
        if (i >= nitems) break;
        const Item it = items[i];
        run_item<K>(jobs[it.job], it, lds);
        __syncthreads();
    }
}

template <int K>
__global__ void __launch_bounds__(kind_threads(K)) k_ragged(const JobDesc *__restrict__ jobs,
                                                     const Item *__restrict__ items, int nitems,
                                                     int *__restrict__ next) {
    extern __shared__ __align__(16) uint32_t lds[];
    __shared__ int claim;
    claim_loop<K>(jobs, items, nitems, next, lds, claim);
}

// The alpha-free kind: four waves per SIMD (128 VGPRs), two workgroups per compute unit.
__global__ void __launch_bounds__(kind_threads(K_AF)) __attribute__((amdgpu_waves_per_eu(4)))
k_ragged_af(const JobDesc *__restrict__ jobs, const Item *__restrict__ items, int nitems, int *__restrict__ next) {
    extern __shared__ __align__(16) uint32_t lds[];
    __shared__ int claim;
    claim_loop<K_AF>(jobs, items, nitems, next, lds, claim);
}

// Relative cost of one item (arbitrary units, only compared within a launch).
double item_cost(const JobDesc &J, const DevCode &C) {
    const double it = std::max(1, J.max_iters), E = C.E;
    if (J.family == FAMILY_BIN_QC) return it * E * 2.0 / std::max(1, J.qc.Z);
    if (J.family == FAMILY_NB1) return it * E * (double)C.g * C.g;
    if (J.family == FAMILY_SPA_LDS) return it * E * J.cpw * (double)C.g;
    return it * E * J.cpw / kThreads;
}

// A job run outside the persistent kernel, with the schedule its plan resolved to.
struct WideJob {
    int job;
    ldpcx_code *code;
    ldpcx_decode_params params;
};

// Decode the wide jobs: one launch sequence per (code, parameters), over the jobs'
// codewords gathered into one batch (a single job decodes in place).
ldpcx_status run_wide(const ldpcx_job *jobs, std::vector<WideJob> &wide, hipStream_t s) {
    std::vector<bool> done(wide.size(), false);
    for (size_t a = 0; a < wide.size(); ++a) {
        if (done[a]) continue;
        std::vector<size_t> grp;
        for (size_t b = a; b < wide.size(); ++b)
            if (!done[b] && wide[b].code == wide[a].code &&
                std::memcmp(&wide[b].params, &wide[a].params, sizeof(ldpcx_decode_params)) == 0) {
                grp.push_back(b);
                done[b] = true;
            }
        ldpcx_code *c = wide[a].code;
        const ldpcx_decode_params &p = wide[a].params;
        const size_t n = c->dev.n, g = c->g;
        const size_t in_cw = g == 2 ? n : n * g * 2, out_cw = g == 2 ? (n + 7) / 8 : n;
        if (grp.size() == 1) {
            const ldpcx_job &jb = jobs[wide[a].job];
            const DecodeIO io{jb.llr, jb.hard, jb.syndrome_ok, jb.iters, nullptr, nullptr, nullptr};
            const ldpcx_status st = run_plan(c, &p, plan_for(c, &p, jb.batch), jb.batch, io, s, false);
            if (st != LDPCX_OK) return st;
            continue;
        }
        size_t total = 0;
        for (size_t i : grp) total += (size_t)jobs[wide[i].job].batch;
        if (total > (size_t)INT32_MAX) return fail(LDPCX_E_UNSUPPORTED, "too many codewords in one ragged batch");
        const size_t o_hard = align_up(total * in_cw, 256);
        const size_t o_ok = align_up(o_hard + total * out_cw, 256);
        const size_t o_it = align_up(o_ok + total, 256);
        const size_t bytes = align_up(o_it + 2 * total, 256);
        char *buf = nullptr;
        if (hipMallocAsync((void **)&buf, bytes, s) != hipSuccess) return fail(LDPCX_E_NOMEM, "ragged gather buffers");
        hipError_t e = hipSuccess;
        size_t off = 0;
        for (size_t i : grp) {
            const ldpcx_job &jb = jobs[wide[i].job];
            if (e == hipSuccess)
                e = hipMemcpyAsync(buf + off * in_cw, jb.llr, (size_t)jb.batch * in_cw, hipMemcpyDeviceToDevice, s);
            off += (size_t)jb.batch;
        }
        ldpcx_status st = LDPCX_OK;
        if (e == hipSuccess) {
            const DecodeIO io{buf, buf + o_hard, (uint8_t *)(buf + o_ok), (int16_t *)(buf + o_it), nullptr, nullptr,
                              nullptr};
            st = run_plan(c, &p, plan_for(c, &p, (int)total), (int)total, io, s, false);
        }
        off = 0;
        for (size_t i : grp) {
            const ldpcx_job &jb = jobs[wide[i].job];
            const size_t nb = (size_t)jb.batch;
            if (st == LDPCX_OK && e == hipSuccess)
                e = hipMemcpyAsync(jb.hard, buf + o_hard + off * out_cw, nb * out_cw, hipMemcpyDeviceToDevice, s);
            if (st == LDPCX_OK && e == hipSuccess)
                e = hipMemcpyAsync(jb.syndrome_ok, buf + o_ok + off, nb, hipMemcpyDeviceToDevice, s);
            if (st == LDPCX_OK && e == hipSuccess)
                e = hipMemcpyAsync(jb.iters, buf + o_it + 2 * off, 2 * nb, hipMemcpyDeviceToDevice, s);
            off += nb;
        }
        (void)hipFreeAsync(buf, s);
        if (st != LDPCX_OK) return st;
        if (e != hipSuccess) return fail_hip(e, "ragged gather copies");
    }
    return LDPCX_OK;
}

}  // namespace

bool ragged_nb1_items(const ldpcx_code *c, const ldpcx_decode_params *p) {
    const int amax = nb_amax(p);
    const size_t cap = (size_t)device_info(c->device).lds_per_block - kStaticLds;
    return p->rule == LDPCX_RULE_MINMAX && nb1_supported(c->dev, amax) && c->dev.m >= 32 &&
           nb1_lds_bytes(c->dev, amax) <= cap;
}

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
        std::vector<size_t> need;  // LDS bytes of each item
        std::vector<void *> workspaces;
        std::vector<WideJob> wide;
        auto cleanup = [&]() {
            for (void *w : workspaces) (void)hipFreeAsync(w, s);
        };
        int device = -1;
        for (int j = 0; j < njobs; ++j) {
            const ldpcx_job &jb = jobs[j];
            if (!jb.code) return cleanup(), fail(LDPCX_E_INVAL, "job without code");
            ldpcx_code *c = const_cast<ldpcx_code *>(jb.code);
            ldpcx_status st = check_params(c, &jb.params);
            if (st != LDPCX_OK) return cleanup(), st;
            if (c->nb_unsupported) return cleanup(), fail(LDPCX_E_UNSUPPORTED, "no Min-Max kernel for this field size");
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
            D.amax = nb_amax(&p);
            D.io = DecodeIO{jb.llr, jb.hard, jb.syndrome_ok, jb.iters, nullptr, nullptr, nullptr};
            D.layered = pl.schedule == LDPCX_SCHED_LAYERED;
            auto add = [&](int type, long count, size_t bytes) {
                for (long i = 0; i < count; ++i) items.push_back(Item{type, j, (int)i, 0});
                const double cst = item_cost(D, D.C);
                cost.insert(cost.end(), (size_t)count, cst);
                need.insert(need.end(), (size_t)count, bytes);
            };
            if (c->g > 2) {
                // Min-Max: one codeword per item when its messages fit a workgroup and the
                // code has enough checks to occupy the workgroup's lanes
                if (ragged_nb1_items(c, &p)) {
                    D.family = FAMILY_NB1;
                    D.af = D.C.dc_max <= 4 && D.C.g == kAfField && nb1_alpha_free(D.C, D.layered, false, kind_threads(K_AF));
                    add(I_NB1, jb.batch, dev::nb1::layout(D.C, dev::nb1::msg_bytes(D.amax), D.af != 0).total);
                    continue;
                }
                // FFT-SPA of the LDS-resident family: one item per group of codewords
                if (p.rule == LDPCX_RULE_SPA && pl.family == FAMILY_SPA_LDS && spa_lds_bytes(D.C, pl.cpw) <= cap) {
                    D.family = FAMILY_SPA_LDS;
                    D.cpw = pl.cpw;
                    add(I_SPA, (jb.batch + pl.cpw - 1) / pl.cpw, spa_lds_bytes(D.C, pl.cpw));
                    continue;
                }
            }
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
                    add(I_QC, ((jb.batch + 1) / 2 + np - 1) / np, dev::qc_smem_bytes(ml, md, D.C, c->qc.Z, D.layered, np));
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
                add(I_LDS, (jb.batch + cpw - 1) / cpw, bin_lds_smem_bytes(D.C, D.layered, cpw));
                continue;
            }
            // The whole-device families: decoded after the persistent kernel, with the
            // schedule resolved as for this job alone.
            WideJob wj{j, c, p};
            wj.params.schedule = pl.schedule;
            wide.push_back(wj);
        }
        if (items.empty()) return cleanup(), run_wide(jobs, wide, s);

        // One launch class per item kind; within each, longest item first (the claims
        // then follow that order: greedy list scheduling).
        std::vector<int> order(items.size());
        for (size_t i = 0; i < order.size(); ++i) order[i] = (int)i;
        std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cost[a] > cost[b]; });
        std::vector<Item> cls[kKinds];
        size_t lds[kKinds] = {0, 0, 0, 0, 0};
        for (int i : order) {
            const Item &it = items[i];
            const int k = it.type == I_SPA   ? K_SPA
                          : it.type != I_NB1 ? K_BIN
                          : J[it.job].af     ? K_AF
                          : J[it.job].C.dc_max <= 4 ? K_GF4
                                                    : K_GF16;
            cls[k].push_back(it);
            lds[k] = std::max(lds[k], need[i]);
        }

        // One device table: jobs, the item lists, their claim counters (uploaded as zero).
        size_t o_it[kKinds];
        size_t o = align_up(sizeof(JobDesc) * njobs, 256);
        for (int k = 0; k < kKinds; ++k) {
            o_it[k] = o;
            o = align_up(o + sizeof(Item) * cls[k].size(), 256);
        }
        const size_t o_ctr = o;
        const size_t total = align_up(o_ctr + kKinds * sizeof(int), 256);
        char *dbuf = nullptr;
        if (hipMallocAsync((void **)&dbuf, total, s) != hipSuccess) return cleanup(), fail(LDPCX_E_NOMEM, "item table");
        workspaces.push_back(dbuf);
        std::vector<char> host(total, 0);
        std::memcpy(host.data(), J.data(), sizeof(JobDesc) * njobs);
        for (int k = 0; k < kKinds; ++k)
            if (!cls[k].empty()) std::memcpy(host.data() + o_it[k], cls[k].data(), sizeof(Item) * cls[k].size());
        ldpcx_status st = upload_async(dbuf, host.data(), total, device, s);
        if (st != LDPCX_OK) return cleanup(), st;
        const JobDesc *djobs = (const JobDesc *)dbuf;

        // Errors of the calls above were checked where they happened; clear the sticky
        // last-error state so that the launch checks below report the launches only.
        (void)hipGetLastError();
        const void *kerns[kKinds] = {(const void *)k_ragged<K_BIN>, (const void *)k_ragged<K_GF4>,
                                     (const void *)k_ragged<K_GF16>, (const void *)k_ragged<K_SPA>,
                                     (const void *)k_ragged_af};
        for (int k = 0; k < kKinds; ++k) {
            if (cls[k].empty()) continue;
            const void *kern = kerns[k];
            allow_full_lds(kern);
            int per_cu = 0;
            const int thr = kind_threads(k);
            hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, thr, lds[k]);
            if (e != hipSuccess || per_cu < 1)
                return cleanup(), fail(LDPCX_E_UNSUPPORTED, "persistent kernel does not fit");
            const int grid = (int)std::min<long>((long)per_cu * device_info(device).cus, (long)cls[k].size());
            const Item *ditems = (const Item *)(dbuf + o_it[k]);
            int *dnext = (int *)(dbuf + o_ctr) + k;
            const int ni = (int)cls[k].size();
            if (k == K_GF4) hipLaunchKernelGGL(k_ragged<K_GF4>, dim3(grid), dim3(thr), lds[k], s, djobs, ditems, ni, dnext);
            else if (k == K_AF) hipLaunchKernelGGL(k_ragged_af, dim3(grid), dim3(thr), lds[k], s, djobs, ditems, ni, dnext);
            else if (k == K_GF16) hipLaunchKernelGGL(k_ragged<K_GF16>, dim3(grid), dim3(thr), lds[k], s, djobs, ditems, ni, dnext);
            else if (k == K_SPA) hipLaunchKernelGGL(k_ragged<K_SPA>, dim3(grid), dim3(thr), lds[k], s, djobs, ditems, ni, dnext);
            else hipLaunchKernelGGL(k_ragged<K_BIN>, dim3(grid), dim3(thr), lds[k], s, djobs, ditems, ni, dnext);
            e = hipGetLastError();
            if (e != hipSuccess) {
                cleanup();
                char msg[160];
                snprintf(msg, sizeof msg, "persistent kernel launch (grid %d, %zu bytes of LDS)", grid, lds[k]);
                return fail_hip(e, msg);
            }
        }
        cleanup();
        return run_wide(jobs, wide, s);
    } catch (const std::exception &ex) {
        return fail(LDPCX_E_NOMEM, ex.what());
    }
}
