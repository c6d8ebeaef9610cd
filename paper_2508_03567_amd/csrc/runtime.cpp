// Host runtime of libldpcx: code handles, validation, launch planning and the
// plain per-code decode entry points of the C-ABI.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <set>
#include <string>
#include <utility>
#include <vector>

#include "runtime.h"

namespace ldpcx {

thread_local std::string g_err;

ldpcx_status fail(ldpcx_status st, const std::string &msg) {
    g_err = msg;
    return st;
}

ldpcx_status fail_hip(hipError_t e, const char *what) {
    return fail(LDPCX_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

namespace {

std::mutex g_dev_mu;
std::map<int, DeviceInfo> g_dev;

// GF(2^p) tables from powers of the primitive element (log/exp construction).
bool build_gf(int g, uint32_t poly, std::vector<uint8_t> &mul, std::vector<uint8_t> &inv) {
    int p = 0;
    while ((1 << p) < g) ++p;
    std::vector<int> ex(2 * g), lg(g, -1);
    int v = 1;
    for (int i = 0; i < g - 1; ++i) {
        if (lg[v] >= 0) return false;  // alpha is not primitive
        ex[i] = v;
        lg[v] = i;
        v <<= 1;
        if (v >> p) v ^= (int)poly;
        if (v >= g) return false;
    }
    if (v != 1) return false;
    for (int i = g - 1; i < 2 * g; ++i) ex[i] = ex[i - (g - 1)];
    mul.assign((size_t)g * g, 0);
    inv.assign(g, 0);
    for (int a = 1; a < g; ++a) {
        for (int b = 1; b < g; ++b) mul[(size_t)a * g + b] = (uint8_t)ex[lg[a] + lg[b]];
        inv[a] = (uint8_t)ex[(g - 1 - lg[a]) % (g - 1)];
    }
    return true;
}

}  // namespace

void allow_full_lds(const void *kernel) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) {
        (void)hipGetLastError();
        return;
    }
    static std::mutex mu;
    static std::set<std::pair<const void *, int>> done;
    std::lock_guard<std::mutex> lk(mu);
    if (!done.insert(std::make_pair(kernel, dev)).second) return;
    (void)hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    (void)hipGetLastError();
}

const DeviceInfo &device_info(int dev) {
    std::lock_guard<std::mutex> lk(g_dev_mu);
    auto it = g_dev.find(dev);
    if (it != g_dev.end()) return it->second;
    DeviceInfo d;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) == hipSuccess) {
        d.cus = prop.multiProcessorCount;
        d.lds_per_block = (int)prop.sharedMemPerBlock;
    }
    // Keep freed stream-ordered workspaces cached in the default pool.
    hipMemPool_t pool;
    if (hipDeviceGetDefaultMemPool(&pool, dev) == hipSuccess) {
        uint64_t thr = UINT64_MAX;
        (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &thr);
    }
    (void)hipGetLastError();  // the pool setting is best effort; leave no sticky error behind
    return g_dev.emplace(dev, d).first->second;
}

ldpcx_status check_params(const ldpcx_code *c, const ldpcx_decode_params *p) {
    if (!p) return fail(LDPCX_E_INVAL, "params is NULL");
    if (p->max_iters < 0 || p->max_iters > 100000) return fail(LDPCX_E_INVAL, "max_iters out of range");
    if (p->schedule < 0 || p->schedule > 2) return fail(LDPCX_E_INVAL, "unknown schedule");
    if (c->g == 2) {
        if (p->rule < 0 || p->rule > 2) return fail(LDPCX_E_INVAL, "binary codes take rule MS, NMS or OMS");
        if (p->msg_max < 1 || p->msg_max > 127) return fail(LDPCX_E_INVAL, "msg_max must be in [1, 127]");
        if (p->rule == LDPCX_RULE_NMS && (p->nms_num < 0 || p->nms_shift < 0 || p->nms_shift > 6 ||
                                          p->nms_num > (1 << p->nms_shift)))
            return fail(LDPCX_E_INVAL, "NMS factor must be nms_num / 2^nms_shift in [0, 1], nms_shift <= 6");
        if (p->rule == LDPCX_RULE_OMS && (p->oms_offset < 0 || p->oms_offset > 127))
            return fail(LDPCX_E_INVAL, "OMS offset out of range");
        if (p->schedule == LDPCX_SCHED_LAYERED && !c->layers_ok)
            return fail(LDPCX_E_INVAL, "layered schedule needs a valid layer size");
    } else {
        if (p->rule != LDPCX_RULE_MINMAX && p->rule != LDPCX_RULE_SPA)
            return fail(LDPCX_E_INVAL, "codes over GF(g > 2) take rule MINMAX or SPA");
        if (p->rule == LDPCX_RULE_SPA && !spa_supported(c->dev))
            return fail(LDPCX_E_UNSUPPORTED, "the FFT-SPA decoder covers GF(4)..GF(64) with check and variable degrees "
                                             "<= 16, and GF(128), GF(256) with degrees <= 4");
        if (p->nb_msg_max < 0 || p->nb_msg_max > 32767) return fail(LDPCX_E_INVAL, "nb_msg_max must be in [0, 32767]");
        if (p->schedule == LDPCX_SCHED_LAYERED && p->rule == LDPCX_RULE_SPA)
            return fail(LDPCX_E_UNSUPPORTED, "the FFT-SPA decoder runs the flooding schedule only");
        if (p->schedule == LDPCX_SCHED_LAYERED && c->g > 64)
            return fail(LDPCX_E_UNSUPPORTED, "layered Min-Max covers GF(4)..GF(64)");
    }
    return LDPCX_OK;
}

int nb_amax(const ldpcx_decode_params *p) { return p->nb_msg_max > 0 ? p->nb_msg_max : 32767; }

BinRule bin_rule(const ldpcx_decode_params *p) {
    BinRule R;
    R.rule = p->rule;
    R.nms_num = p->nms_num;
    R.nms_shift = p->nms_shift;
    R.oms_offset = p->oms_offset;
    R.msg_max = p->msg_max;
    return R;
}

// Default launch plan (overridden by the autotuner's cached choice).
Plan default_plan(const ldpcx_code *c, const ldpcx_decode_params *p, int batch) {
    Plan pl;
    const DeviceInfo &di = device_info(c->device);
    if (c->g > 2 && p->rule == LDPCX_RULE_SPA) {
        pl.schedule = LDPCX_SCHED_FLOODING;
        // Short low-degree codes of which at least half a wave's worth of codewords fits
        // in LDS: every vector on chip (measured faster there), else the wave kernels
        if (spa_lds_supported(c->dev) && 2 * spa_lds_fit(c->dev) >= spa_lds_cpw(c->dev)) {
            pl.family = FAMILY_SPA_LDS;
            pl.cpw = spa_lds_cw(c->dev, std::max(1, batch));
            pl.threads = 1024;
            return pl;
        }
        pl.family = FAMILY_SPA;
        pl.cpw = spa_cw_per_wave(c->dev);
        pl.threads = 256;
        return pl;
    }
    if (c->g > 2) {
        pl.schedule = p->schedule == LDPCX_SCHED_LAYERED ? LDPCX_SCHED_LAYERED : LDPCX_SCHED_FLOODING;
        // Codes whose variables all have degree 2 and with at least 32 checks: one codeword
        // per workgroup, alpha-free at 512 threads (measured fastest on the GF(64) workload)
        if (p->rule == LDPCX_RULE_MINMAX && c->dev.m >= 32 && nb1_supported(c->dev, nb_amax(p)) &&
            nb1_alpha_free(c->dev, pl.schedule == LDPCX_SCHED_LAYERED, false, 512)) {
            pl.family = FAMILY_NB1;
            pl.cpw = 1;
            pl.threads = 512;
            return pl;
        }
        pl.family = FAMILY_NB;
        pl.cpw = 64;
        pl.threads = 256;
        // Short codes whose messages of 64 codewords fit in LDS: one workgroup per group,
        // with as many waves as fit (measured faster wherever it fits)
        if (c->g <= 64) {
            for (int thr : {1024, 512, 256})
                if (nb_lds_bytes(c->dev, thr / 64) <= (size_t)160 * 1024) {
                    pl.family = FAMILY_NB_LDS;
                    pl.threads = thr;
                    break;
                }
        }
        return pl;
    }
    int sched = p->schedule;
    if (sched == LDPCX_SCHED_AUTO) sched = (c->desc.z > 0 && c->layers_ok) ? LDPCX_SCHED_LAYERED : LDPCX_SCHED_FLOODING;
    pl.schedule = sched;
    if (c->qc_ok) {
        pl.family = FAMILY_BIN_QC;
        const int Z = c->qc.Z;
        const int pairs = (batch + 1) / 2;
        int np = std::max(1, std::min(512 / Z, 256 / Z));
        while (np > 1 && (pairs + np - 1) / np < 2 * di.cus) --np;
        while (np > 1 && bin_qc_smem_bytes(c->qc, c->dev, sched == LDPCX_SCHED_LAYERED, np) > (size_t)di.lds_per_block) --np;
        pl.cpw = 2 * np;
        pl.threads = Z * np;
        // Flooding: the layers in parallel where a layer fills whole waves, which shortens
        // each codeword's iteration (on the n = 192 code 2.5x faster than one row per
        // thread at 1000 codewords, and at least as fast from 4096 to 65536)
        if (sched != LDPCX_SCHED_LAYERED) {
            int npl = 1;
            while (npl <= 16 && (Z * npl) % 64) ++npl;
            if (npl <= 16 && bin_qc_lp_ok(c->qc, npl) &&
                bin_qc_smem_bytes(c->qc, c->dev, false, npl) <= (size_t)di.lds_per_block) {
                pl.cpw = 2 * npl;
                pl.threads = Z * npl * c->qc.nl;
            }
        }
        return pl;
    }
    const size_t per_cw = bin_lds_smem_bytes(c->dev, sched == LDPCX_SCHED_LAYERED, 1);
    if (per_cw <= (size_t)64 * 1024 || (sched == LDPCX_SCHED_LAYERED && per_cw <= (size_t)di.lds_per_block)) {
        pl.family = FAMILY_BIN_LDS;
        int cpw = (int)std::max<size_t>(1, (size_t)(40 * 1024) / per_cw);
        cpw = std::min(cpw, 16);
        // keep at least ~2 workgroups per compute unit when the batch allows it
        const int per_cu = std::max(1, batch / std::max(1, 2 * di.cus));
        cpw = std::max(1, std::min(cpw, per_cu));
        while (cpw > 1 && bin_lds_smem_bytes(c->dev, sched == LDPCX_SCHED_LAYERED, cpw) > (size_t)di.lds_per_block) --cpw;
        pl.cpw = cpw;
        const int rows = sched == LDPCX_SCHED_LAYERED ? std::max(1, c->desc.z) : c->dev.m;
        int thr = ((rows * cpw + 63) / 64) * 64;
        pl.threads = std::min(thr, sched == LDPCX_SCHED_LAYERED ? 1024 : 256);
    } else {
        pl.family = FAMILY_BIN_IL;
        pl.schedule = LDPCX_SCHED_FLOODING;
        pl.cpw = bin_il_sub_batch(c->dev, batch, 1024);  // codewords per launch sequence
        pl.threads = 256;
    }
    return pl;
}

Plan plan_for(ldpcx_code *c, const ldpcx_decode_params *p, int batch) {
    {
        std::lock_guard<std::mutex> lk(c->mu);
        auto it = c->tuned.find(tune_key(p, batch));
        if (it != c->tuned.end()) return it->second;
    }
    return default_plan(c, p, batch);
}

uint64_t tune_key(const ldpcx_decode_params *p, int batch) {
    int cls = 0;
    while ((1 << cls) < batch && cls < 40) ++cls;
    return ((uint64_t)p->schedule << 48) | ((uint64_t)p->rule << 40) | ((uint64_t)(p->early_stop != 0) << 39) |
           ((uint64_t)std::min(p->max_iters, 65535) << 16) | (uint64_t)cls;
}

size_t work_bytes(const ldpcx_code *c, const ldpcx_decode_params *p, const Plan &pl, int batch) {
    if (pl.family == FAMILY_BIN_IL) return bin_il_work_bytes(c->dev, p->max_iters, batch, pl.cpw);
    if (pl.family == FAMILY_SPA) return spa_work_bytes(c->dev, p->max_iters, batch);
    if (pl.family == FAMILY_NB || pl.family == FAMILY_NB_LDS) return nb_work_bytes(c->dev, p->max_iters, batch);
    return 0;
}

// Enqueue one decode with an explicit plan.
ldpcx_status run_plan(ldpcx_code *c, const ldpcx_decode_params *p, const Plan &pl, int batch, const DecodeIO &io,
                      hipStream_t s, bool allow_graph) {
    hipError_t e = hipSuccess;
    if (pl.family == FAMILY_BIN_QC) {
        if (!c->qc_ok) return fail(LDPCX_E_UNSUPPORTED, "code has no quasi-cyclic description");
        const int np = pl.cpw / 2;
        if (bin_qc_smem_bytes(c->qc, c->dev, pl.schedule == LDPCX_SCHED_LAYERED, np) > (size_t)device_info(c->device).lds_per_block)
            return fail(LDPCX_E_UNSUPPORTED, "pair state does not fit the LDS of one workgroup");
        const bool lp = pl.schedule != LDPCX_SCHED_LAYERED && pl.threads == c->qc.Z * np * c->qc.nl &&
                        bin_qc_lp_ok(c->qc, np);
        e = lp ? launch_bin_qc_lp(c->qc, c->dev, bin_rule(p), p->max_iters, p->early_stop, batch, np, io, s)
               : launch_bin_qc(c->qc, c->dev, bin_rule(p), p->max_iters, p->early_stop,
                               pl.schedule == LDPCX_SCHED_LAYERED, batch, np, io, s);
        if (e != hipSuccess) return fail_hip(e, "QC decoder launch");
        return LDPCX_OK;
    }
    if (pl.family == FAMILY_BIN_LDS) {
        const size_t smem = bin_lds_smem_bytes(c->dev, pl.schedule == LDPCX_SCHED_LAYERED, pl.cpw);
        if (smem > (size_t)device_info(c->device).lds_per_block)
            return fail(LDPCX_E_UNSUPPORTED, "code state does not fit the LDS of one workgroup");
        e = launch_bin_lds(c->dev, bin_rule(p), p->max_iters, p->early_stop, pl.schedule == LDPCX_SCHED_LAYERED, batch,
                           pl.cpw, pl.threads, io, s);
        if (e != hipSuccess) return fail_hip(e, "binary LDS decoder launch");
        return LDPCX_OK;
    }
    if (pl.family == FAMILY_SPA_LDS) {
        if (!spa_lds_supported(c->dev) || spa_lds_bytes(c->dev, pl.cpw) > kSpaLdsMax)
            return fail(LDPCX_E_UNSUPPORTED, "FFT-SPA vectors do not fit the LDS of one workgroup");
        e = launch_spa_lds(c->dev, p->max_iters, p->early_stop, batch, pl.cpw, pl.threads, io, s);
        if (e != hipSuccess) return fail_hip(e, "LDS-resident FFT-SPA launch");
        return LDPCX_OK;
    }
    if (pl.family == FAMILY_NB1) {
        if (!nb1_supported(c->dev, nb_amax(p)) || p->rule != LDPCX_RULE_MINMAX)
            return fail(LDPCX_E_UNSUPPORTED, "the messages of one codeword do not fit the LDS of one workgroup");
        e = launch_nb1(c->dev, p->max_iters, p->early_stop, pl.schedule == LDPCX_SCHED_LAYERED, batch, nb_amax(p),
                       pl.threads, io, s);
        if (e != hipSuccess) return fail_hip(e, "one-codeword-per-workgroup Min-Max launch");
        return LDPCX_OK;
    }
    if (pl.family == FAMILY_BIN_IL && pl.schedule == LDPCX_SCHED_LAYERED)
        return fail(LDPCX_E_UNSUPPORTED, "the interleaved binary decoder implements the flooding schedule only");
    if (allow_graph && !io.dump_a && graphs_enabled()) {
        ldpcx_status st = run_graph(c, p, pl, batch, io, s);
        if (st != LDPCX_E_UNSUPPORTED) return st;  // else: capture not possible, run eagerly
    }
    size_t bytes = work_bytes(c, p, pl, batch);
    size_t dump_bytes = 0;
    if (io.dump_a && pl.family == FAMILY_BIN_IL) dump_bytes = bin_il_dump_bytes(c->dev, batch, pl.cpw);
    void *ws = nullptr;
    e = hipMallocAsync(&ws, bytes + dump_bytes, s);
    if (e != hipSuccess) return fail(LDPCX_E_NOMEM, std::string("workspace allocation: ") + hipGetErrorString(e));
    e = enqueue_interleaved(c, p, pl, batch, ws, io, dump_bytes ? (int8_t *)ws + bytes : nullptr, s);
    hipError_t e2 = hipFreeAsync(ws, s);
    if (e != hipSuccess) return fail_hip(e, "decoder launch");
    if (e2 != hipSuccess) return fail_hip(e2, "workspace release");
    return LDPCX_OK;
}

hipError_t enqueue_interleaved(ldpcx_code *c, const ldpcx_decode_params *p, const Plan &pl, int batch, void *ws,
                               const DecodeIO &io, int8_t *dump_scratch, hipStream_t s) {
    if (pl.family == FAMILY_BIN_IL)
        return launch_bin_il(c->dev, bin_rule(p), p->max_iters, p->early_stop, batch, pl.cpw, ws, io, dump_scratch,
                             s);
    if (pl.family == FAMILY_SPA) return launch_spa(c->dev, p->max_iters, p->early_stop, batch, ws, io, s);
    if (pl.family == FAMILY_NB_LDS)
        return launch_nb_lds(c->dev, p->max_iters, p->early_stop, pl.schedule == LDPCX_SCHED_LAYERED, batch, nb_amax(p),
                             pl.threads / 64, ws, io, s);
    return launch_nb(c->dev, p->max_iters, p->early_stop, pl.schedule == LDPCX_SCHED_LAYERED, batch, nb_amax(p), ws,
                     io, s);
}

bool graphs_enabled() {
    static const bool on = [] {
        const char *v = getenv("LDPCX_GRAPHS");
        return !(v && v[0] == '0');
    }();
    return on;
}

// Replay a captured launch sequence of the interleaved decoders.  One cached entry per
// (plan, params, batch, buffers) holds its own workspace; an event orders replays of
// the same entry issued on different streams.
ldpcx_status run_graph(ldpcx_code *c, const ldpcx_decode_params *p, const Plan &pl, int batch, const DecodeIO &io,
                       hipStream_t s) {
    GraphKey key{};
    key.family = pl.family;
    key.schedule = pl.schedule;
    key.cpw = pl.cpw;
    key.threads = pl.threads;
    key.batch = batch;
    key.params = *p;
    key.llr = io.llr;
    key.hard = io.hard;
    key.ok = io.ok;
    key.iters = io.iters;
    std::lock_guard<std::mutex> lk(c->graph_mu);
    GraphEntry *ge = nullptr;
    for (auto &g : c->graphs)
        if (std::memcmp(&g.key, &key, sizeof key) == 0) ge = &g;
    if (!ge) {
        if (c->graphs.size() >= 8) {  // evict the least recently used entry
            auto lru = c->graphs.begin();
            for (auto it = c->graphs.begin(); it != c->graphs.end(); ++it)
                if (it->last_use < lru->last_use) lru = it;
            (void)hipEventSynchronize(lru->done);
            release_graph(*lru);
            c->graphs.erase(lru);
        }
        GraphEntry g{};
        g.key = key;
        const size_t bytes = work_bytes(c, p, pl, batch);
        if (hipMalloc(&g.ws, bytes) != hipSuccess) return fail(LDPCX_E_NOMEM, "graph workspace allocation");
        hipStream_t cs = nullptr;
        if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) {
            (void)hipFree(g.ws);
            return fail(LDPCX_E_DEVICE, "capture stream");
        }
        hipGraph_t graph = nullptr;
        hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess) {
            hipError_t el = enqueue_interleaved(c, p, pl, batch, g.ws, io, nullptr, cs);
            e = hipStreamEndCapture(cs, &graph);
            if (el != hipSuccess) e = el;
        }
        if (e == hipSuccess) e = hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0);
        if (graph) (void)hipGraphDestroy(graph);
        (void)hipStreamDestroy(cs);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&g.done, hipEventDisableTiming);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            if (g.exec) (void)hipGraphExecDestroy(g.exec);
            (void)hipFree(g.ws);
            return fail(LDPCX_E_UNSUPPORTED, std::string("graph capture: ") + hipGetErrorString(e));
        }
        c->graphs.push_back(g);
        ge = &c->graphs.back();
    }
    ge->last_use = ++c->graph_clock;
    hipError_t e = hipStreamWaitEvent(s, ge->done, 0);
    if (e == hipSuccess) e = hipGraphLaunch(ge->exec, s);
    if (e == hipSuccess) e = hipEventRecord(ge->done, s);
    if (e != hipSuccess) return fail_hip(e, "graph launch");
    return LDPCX_OK;
}

void release_graph(GraphEntry &g) {
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
    if (g.done) (void)hipEventDestroy(g.done);
    if (g.ws) (void)hipFree(g.ws);
    g = GraphEntry{};
}

namespace {

struct Stage {
    char *p = nullptr;
    size_t cap = 0;
    int device = -1;
    hipEvent_t ev = nullptr;
    bool used = false;
};
std::mutex g_stage_mu;
std::vector<Stage> g_stages;  // kept until the process ends
constexpr size_t kMaxStages = 64;

}  // namespace

ldpcx_status upload_async(void *dst, const void *src, size_t bytes, int device, hipStream_t s) {
    if (bytes == 0) return LDPCX_OK;
    std::lock_guard<std::mutex> lk(g_stage_mu);
    Stage *pick = nullptr;
    for (Stage &st : g_stages) {
        if (st.device != device || st.cap < bytes) continue;
        if (st.used) {
            const hipError_t q = hipEventQuery(st.ev);
            if (q != hipSuccess) {
                (void)hipGetLastError();  // "not ready" is an answer, not an error to report later
                continue;
            }
        }
        pick = &st;
        break;
    }
    if (!pick && g_stages.size() >= kMaxStages) {
        // Every buffer is in flight: wait for the first one that is large enough.
        for (Stage &st : g_stages)
            if (st.device == device && st.cap >= bytes) {
                hipError_t e = hipEventSynchronize(st.ev);
                if (e != hipSuccess) return fail_hip(e, "staging buffer wait");
                pick = &st;
                break;
            }
    }
    if (!pick) {
        Stage st;
        st.device = device;
        st.cap = std::max<size_t>(bytes, 64 * 1024);
        hipError_t e = hipHostMalloc((void **)&st.p, st.cap, hipHostMallocDefault);
        if (e != hipSuccess) return fail_hip(e, "pinned staging buffer");
        e = hipEventCreateWithFlags(&st.ev, hipEventDisableTiming);
        if (e != hipSuccess) {
            (void)hipHostFree(st.p);
            return fail_hip(e, "staging event");
        }
        g_stages.push_back(st);
        pick = &g_stages.back();
    }
    std::memcpy(pick->p, src, bytes);
    hipError_t e = hipMemcpyAsync(dst, pick->p, bytes, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return fail_hip(e, "upload");
    e = hipEventRecord(pick->ev, s);
    if (e != hipSuccess) {
        // Without the event the buffer cannot be reused safely: wait for the copy.
        (void)hipStreamSynchronize(s);
        pick->used = false;
        return fail_hip(e, "staging event record");
    }
    pick->used = true;
    return LDPCX_OK;
}

ldpcx_status check_device(const ldpcx_code *c) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail_hip(e, "hipGetDevice");
    if (dev != c->device) return fail(LDPCX_E_INVAL, "the current device is not the code handle's device");
    return LDPCX_OK;
}

ldpcx_status decode_common(const ldpcx_code *code, const ldpcx_decode_params *params, int32_t batch, const void *llr,
                           void *hard, uint8_t *ok, int16_t *iters, int32_t *sched_used, void *a, void *b, void *cc,
                           void *stream) {
    if (!code) return fail(LDPCX_E_INVAL, "code is NULL");
    ldpcx_code *c = const_cast<ldpcx_code *>(code);
    ldpcx_status st = check_params(c, params);
    if (st != LDPCX_OK) return st;
    if (batch < 0) return fail(LDPCX_E_INVAL, "batch < 0");
    if (batch == 0) return LDPCX_OK;
    if (!llr || !hard || !ok || !iters) return fail(LDPCX_E_INVAL, "null buffer");
    if (a && (!b || (c->g == 2 && !cc))) return fail(LDPCX_E_INVAL, "dump needs every message buffer");
    if ((st = check_device(c)) != LDPCX_OK) return st;
    const Plan pl = plan_for(c, params, batch);
    if (sched_used) *sched_used = pl.schedule;
    DecodeIO io{llr, hard, ok, iters, a, b, cc};
    return run_plan(c, params, pl, batch, io, (hipStream_t)stream);
}

}  // namespace ldpcx

using namespace ldpcx;

extern "C" {

const char *ldpcx_last_error(void) { return g_err.c_str(); }

const char *ldpcx_version(void) { return "ldpcx 0.1 (gfx950)"; }

ldpcx_status ldpcx_code_create(const ldpcx_code_desc *d, ldpcx_code **out) {
    try {
        if (!d || !out) return fail(LDPCX_E_INVAL, "null argument");
        *out = nullptr;
        const int g = d->g;
        if (g < 2 || g > 256 || (g & (g - 1))) return fail(LDPCX_E_INVAL, "g must be a power of two in [2, 256]");
        if (d->n < 1 || d->m < 1) return fail(LDPCX_E_INVAL, "n and m must be positive");
        if (!d->row_ptr || !d->col_idx) return fail(LDPCX_E_INVAL, "row_ptr/col_idx is NULL");
        if (g > 2 && !d->h_val) return fail(LDPCX_E_INVAL, "h_val is required for g > 2");
        const int n = d->n, m = d->m;
        if (d->row_ptr[0] != 0) return fail(LDPCX_E_INVAL, "row_ptr[0] must be 0");
        for (int i = 0; i < m; ++i)
            if (d->row_ptr[i + 1] < d->row_ptr[i]) return fail(LDPCX_E_INVAL, "row_ptr must be non-decreasing");
        const int E = d->row_ptr[m];
        if (E < 2) return fail(LDPCX_E_INVAL, "too few nonzeros");
        if ((long long)m >= (1LL << 27)) return fail(LDPCX_E_UNSUPPORTED, "too many checks");
        const int dc_lim = g == 2 ? kBinDcMax : kNbDcMax;
        int dc_max = 0;
        for (int i = 0; i < m; ++i) {
            const int dc = d->row_ptr[i + 1] - d->row_ptr[i];
            if (dc < 2) return fail(LDPCX_E_INVAL, "every check needs degree >= 2");
            if (dc > dc_lim) return fail(LDPCX_E_UNSUPPORTED, "check degree above the supported maximum");
            dc_max = std::max(dc_max, dc);
            for (int e = d->row_ptr[i]; e < d->row_ptr[i + 1]; ++e) {
                const int col = d->col_idx[e];
                if (col < 0 || col >= n) return fail(LDPCX_E_INVAL, "column index out of range");
                if (e > d->row_ptr[i] && col <= d->col_idx[e - 1])
                    return fail(LDPCX_E_INVAL, "columns must be strictly ascending within a row");
                if (g > 2 && (d->h_val[e] == 0 || d->h_val[e] >= g))
                    return fail(LDPCX_E_INVAL, "GF coefficient must be nonzero and < g");
            }
        }
        ldpcx_code *c = new ldpcx_code();
        c->desc = *d;
        c->g = g;
        c->row_ptr.assign(d->row_ptr, d->row_ptr + m + 1);
        c->col_idx.assign(d->col_idx, d->col_idx + E);
        if (g > 2) {
            c->h.assign(d->h_val, d->h_val + E);
            std::vector<uint8_t> inv;
            if (!build_gf(g, d->prim_poly, c->gfmul, inv)) {
                delete c;
                return fail(LDPCX_E_INVAL, "prim_poly is not primitive for this field size");
            }
            c->hinv.resize(E);
            for (int e = 0; e < E; ++e) c->hinv[e] = inv[c->h[e]];
        }
        // CSC: edges of each variable node, in ascending check order.
        c->vn_ptr.assign(n + 1, 0);
        for (int e = 0; e < E; ++e) c->vn_ptr[c->col_idx[e] + 1]++;
        int dv_max = 0;
        for (int v = 0; v < n; ++v) {
            dv_max = std::max(dv_max, c->vn_ptr[v + 1]);
            c->vn_ptr[v + 1] += c->vn_ptr[v];
        }
        if (g == 2 && dv_max > 250) {
            delete c;
            return fail(LDPCX_E_UNSUPPORTED, "variable degree above 250");
        }
        c->vn_ref.assign(E, 0);
        c->vn_edge.assign(E, 0);
        {
            std::vector<int> fill(n, 0);
            for (int i = 0; i < m; ++i)
                for (int e = c->row_ptr[i]; e < c->row_ptr[i + 1]; ++e) {
                    const int v = c->col_idx[e];
                    const int t = c->vn_ptr[v] + fill[v]++;
                    c->vn_ref[t] = g == 2 ? ((i << 4) | (e - c->row_ptr[i])) : e;
                    c->vn_edge[t] = e;
                }
        }
        // Layers: rows [l z, (l + 1) z) must touch disjoint columns.
        c->layers_ok = false;
        if (g == 2) {
            const int z = d->z > 0 ? d->z : 1;
            if (d->z < 0 || m % z != 0) {
                delete c;
                return fail(LDPCX_E_INVAL, "m must be a multiple of the layer size z");
            }
            std::vector<int> mark(n, -1);
            bool ok = true;
            for (int l = 0; l < m / z && ok; ++l)
                for (int e = c->row_ptr[l * z]; e < c->row_ptr[(l + 1) * z] && ok; ++e) {
                    if (mark[c->col_idx[e]] == l) ok = false;
                    mark[c->col_idx[e]] = l;
                }
            if (!ok && d->z > 0) {
                delete c;
                return fail(LDPCX_E_INVAL, "rows of one layer share a column");
            }
            c->layers_ok = ok;
            // Quasi-cyclic structure: every layer of z rows made of z x z circulant blocks.
            // (Lambda offsets of the packed decoder are 16-bit: 4 (n + z) < 65536)
            if (ok && d->z > 0 && n % d->z == 0 && m / d->z <= kQcMaxL && 4L * (n + d->z) < 65536) {
                const int Z = d->z, nl = m / Z;
                bool qc = true;
                c->qc.Z = Z;
                c->qc.nl = nl;
                for (int l = 0; l < nl && qc; ++l) {
                    const int r0 = l * Z;
                    const int dcl = c->row_ptr[r0 + 1] - c->row_ptr[r0];
                    if (dcl > kQcMaxDc) { qc = false; break; }
                    c->qc.dc[l] = dcl;
                    for (int j = 0; j < dcl; ++j) {
                        const int col = c->col_idx[c->row_ptr[r0] + j];
                        c->qc.col[l][j] = (short)(col / Z);
                        c->qc.sh[l][j] = (short)(col % Z);
                    }
                    for (int i = 0; i < Z && qc; ++i) {
                        const int r = r0 + i;
                        if (c->row_ptr[r + 1] - c->row_ptr[r] != dcl) { qc = false; break; }
                        for (int j = 0; j < dcl; ++j) {
                            const int want = c->qc.col[l][j] * Z + (i + c->qc.sh[l][j]) % Z;
                            if (c->col_idx[c->row_ptr[r] + j] != want) { qc = false; break; }
                        }
                    }
                }
                c->qc_ok = qc;
            }
        }
        // Layers of the layered Min-Max schedule: checks in ascending order, each in the
        // lowest layer none of whose checks shares a variable with it.
        std::vector<int> nbl_ptr(1, 0), nbl_chk, nbl_eptr(1, 0), nbl_edge;
        int nb_lmax = 0, nb_emax = 0;
        if (g > 2) {
            std::vector<std::vector<uint8_t>> used;  // [layer][variable]
            std::vector<int> layer_of(m);
            for (int i = 0; i < m; ++i) {
                size_t l = 0;
                for (; l < used.size(); ++l) {
                    bool clash = false;
                    for (int e = c->row_ptr[i]; e < c->row_ptr[i + 1] && !clash; ++e) clash = used[l][c->col_idx[e]] != 0;
                    if (!clash) break;
                }
                if (l == used.size()) used.emplace_back(n, 0);
                for (int e = c->row_ptr[i]; e < c->row_ptr[i + 1]; ++e) used[l][c->col_idx[e]] = 1;
                layer_of[i] = (int)l;
            }
            for (size_t l = 0; l < used.size(); ++l) {
                for (int i = 0; i < m; ++i)
                    if (layer_of[i] == (int)l) {
                        nbl_chk.push_back(i);
                        for (int e = c->row_ptr[i]; e < c->row_ptr[i + 1]; ++e) nbl_edge.push_back(e);
                    }
                nbl_ptr.push_back((int)nbl_chk.size());
                nbl_eptr.push_back((int)nbl_edge.size());
                nb_lmax = std::max(nb_lmax, nbl_ptr.back() - nbl_ptr[nbl_ptr.size() - 2]);
                nb_emax = std::max(nb_emax, nbl_eptr.back() - nbl_eptr[nbl_eptr.size() - 2]);
            }
        }
        const int nb_nl = (int)nbl_ptr.size() - 1;
        hipError_t e = hipGetDevice(&c->device);
        if (e != hipSuccess) {
            delete c;
            return fail_hip(e, "hipGetDevice");
        }
        device_info(c->device);
        // One device block for every array.
        const size_t o_rp = 0;
        const size_t o_ci = align_up(o_rp + 4 * (size_t)(m + 1), 256);
        const size_t o_vp = align_up(o_ci + 4 * (size_t)E, 256);
        const size_t o_vr = align_up(o_vp + 4 * (size_t)(n + 1), 256);
        const size_t o_ve = align_up(o_vr + 4 * (size_t)E, 256);
        const size_t o_h = align_up(o_ve + 4 * (size_t)E, 256);
        const size_t o_hi = align_up(o_h + (size_t)E, 256);
        const size_t o_mul = align_up(o_hi + (size_t)E, 256);
        const size_t o_qc = align_up(o_mul + (size_t)g * g + 4, 256);
        const size_t o_sw = align_up(o_qc + sizeof(int2) * kQcMaxL * kQcMaxDc, 256);
        const size_t o_lp = align_up(o_sw + sizeof(int) * kSpaWeights, 256);
        const size_t o_lc = align_up(o_lp + sizeof(int) * nbl_ptr.size(), 256);
        const size_t o_lep = align_up(o_lc + sizeof(int) * (nbl_chk.size() + 1), 256);
        const size_t o_le = align_up(o_lep + sizeof(int) * nbl_eptr.size(), 256);
        const size_t total = align_up(o_le + sizeof(int) * (nbl_edge.size() + 1), 256);
        e = hipMalloc(&c->dmem, total);
        if (e != hipSuccess) {
            delete c;
            return fail(LDPCX_E_NOMEM, "code upload");
        }
        std::vector<uint8_t> host(total, 0);
        std::memcpy(host.data() + o_rp, c->row_ptr.data(), 4 * (size_t)(m + 1));
        std::memcpy(host.data() + o_ci, c->col_idx.data(), 4 * (size_t)E);
        std::memcpy(host.data() + o_vp, c->vn_ptr.data(), 4 * (size_t)(n + 1));
        std::memcpy(host.data() + o_vr, c->vn_ref.data(), 4 * (size_t)E);
        std::memcpy(host.data() + o_ve, c->vn_edge.data(), 4 * (size_t)E);
        if (g > 2) {
            std::memcpy(host.data() + o_h, c->h.data(), E);
            std::memcpy(host.data() + o_hi, c->hinv.data(), E);
            std::memcpy(host.data() + o_mul, c->gfmul.data(), (size_t)g * g);
        }
        {
            // FFT-SPA channel weights W(c) = round(2^24 exp(-c / 4))
            int *sw = (int *)(host.data() + o_sw);
            for (int cst = 0; cst < kSpaWeights; ++cst) sw[cst] = (int)std::floor(16777216.0 * std::exp(-cst / 4.0) + 0.5);
        }
        std::memcpy(host.data() + o_lp, nbl_ptr.data(), sizeof(int) * nbl_ptr.size());
        if (!nbl_chk.empty()) std::memcpy(host.data() + o_lc, nbl_chk.data(), sizeof(int) * nbl_chk.size());
        std::memcpy(host.data() + o_lep, nbl_eptr.data(), sizeof(int) * nbl_eptr.size());
        if (!nbl_edge.empty()) std::memcpy(host.data() + o_le, nbl_edge.data(), sizeof(int) * nbl_edge.size());
        if (c->qc_ok) {
            int2 *qe = (int2 *)(host.data() + o_qc);
            for (int l = 0; l < c->qc.nl; ++l)
                for (int j = 0; j < c->qc.dc[l]; ++j)
                    qe[l * kQcMaxDc + j] = make_int2(c->qc.col[l][j] * c->qc.Z, c->qc.sh[l][j]);
        }
        e = hipMemcpy(c->dmem, host.data(), total, hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            (void)hipFree(c->dmem);
            delete c;
            return fail_hip(e, "code upload");
        }
        char *b = (char *)c->dmem;
        DevCode &D = c->dev;
        D.n = n;
        D.m = m;
        D.E = E;
        D.g = g;
        D.p = 0;
        while ((1 << D.p) < g) ++D.p;
        D.z = g == 2 ? (d->z > 0 ? d->z : 1) : 0;
        D.nlayers = g == 2 ? m / D.z : 0;
        D.dc_max = dc_max;
        D.dv_max = dv_max;
        D.row_ptr = (const int *)(b + o_rp);
        D.col_idx = (const int *)(b + o_ci);
        D.vn_ptr = (const int *)(b + o_vp);
        D.vn_ref = (const int *)(b + o_vr);
        D.vn_edge = (const int *)(b + o_ve);
        D.h = (const uint8_t *)(b + o_h);
        D.hinv = (const uint8_t *)(b + o_hi);
        D.gfmul = (const uint8_t *)(b + o_mul);
        D.spa_w = (const int *)(b + o_sw);
        D.nb_nl = nb_nl;
        D.nb_lmax = nb_lmax;
        D.nb_emax = nb_emax;
        D.nbl_eptr = (const int *)(b + o_lep);
        D.nbl_edge = (const int *)(b + o_le);
        D.nbl_ptr = (const int *)(b + o_lp);
        D.nbl_chk = (const int *)(b + o_lc);
        c->qc.edges = (const int2 *)(b + o_qc);
        c->hash = code_hash(d);
        tune_cache_load(c);
        if (g > 2 && !nb_supported(g)) {
            // Valid code, but no compiled Min-Max kernel for this field size.
            c->nb_unsupported = true;
        }
        *out = c;
        return LDPCX_OK;
    } catch (const std::exception &ex) {
        return fail(LDPCX_E_NOMEM, ex.what());
    }
}

ldpcx_status ldpcx_code_destroy(ldpcx_code *c) {
    if (!c) return LDPCX_OK;
    (void)hipDeviceSynchronize();
    for (auto &g : c->graphs) release_graph(g);
    if (c->dmem) (void)hipFree(c->dmem);
    delete c;
    return LDPCX_OK;
}

ldpcx_status ldpcx_code_info(const ldpcx_code *c, int32_t *n, int32_t *m, int32_t *nnz, int32_t *g, int32_t *max_dc,
                             int32_t *max_dv) {
    if (!c) return fail(LDPCX_E_INVAL, "code is NULL");
    if (n) *n = c->dev.n;
    if (m) *m = c->dev.m;
    if (nnz) *nnz = c->dev.E;
    if (g) *g = c->g;
    if (max_dc) *max_dc = c->dev.dc_max;
    if (max_dv) *max_dv = c->dev.dv_max;
    return LDPCX_OK;
}

ldpcx_status ldpcx_decode(const ldpcx_code *code, const ldpcx_decode_params *params, int32_t batch, const void *llr,
                          void *hard, uint8_t *syndrome_ok, int16_t *iters, int32_t *schedule_used, void *stream) {
    try {
        if (code && code->nb_unsupported) return fail(LDPCX_E_UNSUPPORTED, "no Min-Max kernel for this field size");
        return decode_common(code, params, batch, llr, hard, syndrome_ok, iters, schedule_used, nullptr, nullptr,
                             nullptr, stream);
    } catch (const std::exception &ex) {
        return fail(LDPCX_E_NOMEM, ex.what());
    }
}

ldpcx_status ldpcx_debug_dump(const ldpcx_code *code, const ldpcx_decode_params *params, int32_t batch,
                              const void *llr, void *hard, uint8_t *syndrome_ok, int16_t *iters, void *msg_a,
                              void *msg_b, void *msg_c, void *stream) {
    try {
        if (!msg_a || !msg_b) return fail(LDPCX_E_INVAL, "dump buffers are NULL");
        if (code && code->nb_unsupported) return fail(LDPCX_E_UNSUPPORTED, "no Min-Max kernel for this field size");
        return decode_common(code, params, batch, llr, hard, syndrome_ok, iters, nullptr, msg_a, msg_b, msg_c, stream);
    } catch (const std::exception &ex) {
        return fail(LDPCX_E_NOMEM, ex.what());
    }
}

ldpcx_status ldpcx_plan_info(const ldpcx_code *code, const ldpcx_decode_params *params, int32_t batch, int32_t *family,
                             int32_t *cw_per_wg, int32_t *threads) {
    if (!code) return fail(LDPCX_E_INVAL, "code is NULL");
    ldpcx_code *c = const_cast<ldpcx_code *>(code);
    ldpcx_status st = check_params(c, params);
    if (st != LDPCX_OK) return st;
    const Plan pl = plan_for(c, params, std::max(1, batch));
    if (family) *family = pl.family;
    if (cw_per_wg) *cw_per_wg = pl.cpw;
    if (threads) *threads = pl.threads;
    return LDPCX_OK;
}

ldpcx_status ldpcx_plan_set(ldpcx_code *c, const ldpcx_decode_params *params, int32_t batch, int32_t family,
                            int32_t cw_per_wg, int32_t threads) {
    if (!c) return fail(LDPCX_E_INVAL, "code is NULL");
    ldpcx_status st = check_params(c, params);
    if (st != LDPCX_OK) return st;
    if (family < 0 || family > 7) return fail(LDPCX_E_INVAL, "unknown kernel family");
    const bool spa_family = family == FAMILY_SPA || family == FAMILY_SPA_LDS;
    if (spa_family != (params->rule == LDPCX_RULE_SPA))
        return fail(LDPCX_E_INVAL, "families 4 and 6 run rule SPA, and rule SPA only those");
    if (family == FAMILY_BIN_QC && !c->qc_ok) return fail(LDPCX_E_UNSUPPORTED, "code has no quasi-cyclic description");
    if ((c->g > 2) != (family == FAMILY_NB || spa_family || family == FAMILY_NB_LDS || family == FAMILY_NB1))
        return fail(LDPCX_E_INVAL, "family does not match the field size");
    Plan pl;
    pl.family = family;
    pl.schedule = params->schedule == LDPCX_SCHED_AUTO ? default_plan(c, params, std::max(1, batch)).schedule
                                                        : params->schedule;
    if (family != FAMILY_BIN_LDS && family != FAMILY_BIN_QC && family != FAMILY_NB && family != FAMILY_NB_LDS &&
        family != FAMILY_NB1 && pl.schedule == LDPCX_SCHED_LAYERED)
        return fail(LDPCX_E_UNSUPPORTED, "this kernel family runs the flooding schedule only");
    if (family == FAMILY_NB && pl.schedule == LDPCX_SCHED_LAYERED && c->g > 64)
        return fail(LDPCX_E_UNSUPPORTED, "layered Min-Max covers GF(4)..GF(64)");
    if (family == FAMILY_BIN_QC) {
        if (cw_per_wg < 2 || cw_per_wg % 2 || c->qc.Z * cw_per_wg / 2 > 512)
            return fail(LDPCX_E_INVAL, "cw_per_wg must be even with Z * cw_per_wg / 2 <= 512");
        if (bin_qc_smem_bytes(c->qc, c->dev, pl.schedule == LDPCX_SCHED_LAYERED, cw_per_wg / 2) >
            (size_t)device_info(c->device).lds_per_block)
            return fail(LDPCX_E_UNSUPPORTED, "state of cw_per_wg codewords does not fit the LDS");
        pl.cpw = cw_per_wg;
        // Z * npairs * nl threads select the layer-parallel flooding kernel
        const int np = cw_per_wg / 2;
        const bool lp = threads == c->qc.Z * np * c->qc.nl && pl.schedule != LDPCX_SCHED_LAYERED && bin_qc_lp_ok(c->qc, np);
        pl.threads = lp ? threads : c->qc.Z * np;
    }
    if (family == FAMILY_BIN_LDS) {
        if (cw_per_wg < 1 || cw_per_wg > 64) return fail(LDPCX_E_INVAL, "cw_per_wg out of range");
        if (threads < 64 || threads > 1024 || threads % 64) return fail(LDPCX_E_INVAL, "threads out of range");
        if (bin_lds_smem_bytes(c->dev, pl.schedule == LDPCX_SCHED_LAYERED, cw_per_wg) >
            (size_t)device_info(c->device).lds_per_block)
            return fail(LDPCX_E_UNSUPPORTED, "state of cw_per_wg codewords does not fit the LDS");
        pl.cpw = cw_per_wg;
        pl.threads = threads;
    }
    if (family == FAMILY_BIN_IL) {
        if (cw_per_wg < 1) return fail(LDPCX_E_INVAL, "cw_per_wg (codewords per launch sequence) must be positive");
        pl.cpw = bin_il_sub_batch(c->dev, std::max(1, batch), cw_per_wg);
        pl.threads = 256;
    }
    if (family == FAMILY_NB) {
        pl.cpw = 64;
        pl.threads = 256;
    }
    if (family == FAMILY_NB_LDS) {
        if (c->g > 64 || params->rule != LDPCX_RULE_MINMAX)
            return fail(LDPCX_E_UNSUPPORTED, "family 5 runs Min-Max over GF(4)..GF(64)");
        if (threads != 256 && threads != 512 && threads != 1024)
            return fail(LDPCX_E_INVAL, "family 5 takes 256, 512 or 1024 threads");
        if (nb_lds_bytes(c->dev, threads / 64) > (size_t)160 * 1024)
            return fail(LDPCX_E_UNSUPPORTED, "the messages of 64 codewords do not fit the LDS of one workgroup");
        pl.cpw = 64;
        pl.threads = threads;
    }
    if (family == FAMILY_NB1) {
        if (c->g > 64 || params->rule != LDPCX_RULE_MINMAX || !nb1_supported(c->dev, nb_amax(params)))
            return fail(LDPCX_E_UNSUPPORTED, "family 7 runs Min-Max over GF(4)..GF(64) for codes whose messages of one "
                                             "codeword fit 160 KB of LDS");
        if (threads < 64 || threads > 1024 || threads % 64)
            return fail(LDPCX_E_INVAL, "family 7 takes a multiple of 64 threads up to 1024");
        pl.cpw = 1;
        pl.threads = threads;
    }
    if (family == FAMILY_SPA) {
        pl.cpw = spa_cw_per_wave(c->dev);
        pl.threads = 256;
    }
    if (family == FAMILY_SPA_LDS) {
        if (!spa_lds_supported(c->dev))
            return fail(LDPCX_E_UNSUPPORTED, "family 6 needs check and variable degrees <= 4 and one codeword's "
                                             "vectors within 160 KB of LDS");
        if (threads != 256 && threads != 512 && threads != 1024)
            return fail(LDPCX_E_INVAL, "family 6 takes 256, 512 or 1024 threads");
        if (cw_per_wg < 1 || cw_per_wg > 64) return fail(LDPCX_E_INVAL, "cw_per_wg out of range");
        if (spa_lds_bytes(c->dev, cw_per_wg) > kSpaLdsMax)
            return fail(LDPCX_E_UNSUPPORTED, "the vectors of cw_per_wg codewords do not fit the LDS of one workgroup");
        pl.cpw = cw_per_wg;
        pl.threads = threads;
    }
    std::lock_guard<std::mutex> lk(c->mu);
    c->tuned[tune_key(params, std::max(1, batch))] = pl;
    return LDPCX_OK;
}

}  // extern "C"
