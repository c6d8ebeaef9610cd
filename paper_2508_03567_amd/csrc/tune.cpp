// Autotuner: times candidate launch plans of one (code, params, batch) on the
// device and caches the fastest in the code handle.  Candidates are the kernel
// family's tunable knobs (codewords per workgroup and threads per workgroup for
// the LDS-resident binary decoder) and, only when the caller asked for the AUTO
// schedule, the schedule itself (flooding versus layered): the two schedules
// are different algorithms, so a fixed schedule is never changed.
#include <algorithm>
#include <vector>

#include "runtime.h"

using namespace ldpcx;

namespace {

std::vector<Plan> candidates(const ldpcx_code *c, const ldpcx_decode_params *p, int batch) {
    std::vector<Plan> out;
    const Plan def = default_plan(c, p, batch);
    out.push_back(def);
    if (c->g > 2 && p->rule == LDPCX_RULE_SPA) {
        // FFT-SPA: the wave kernels and, for short low-degree codes, the LDS-resident
        // kernel
        Plan pl = def;
        pl.family = FAMILY_SPA;
        pl.cpw = spa_cw_per_wave(c->dev);
        pl.threads = 256;
        out.push_back(pl);
        if (spa_lds_supported(c->dev)) {
            // groups: the default one, the largest that fits, and 8, 16 and 32 codewords
            const int fit = std::min(spa_lds_fit(c->dev), std::max(1, batch));
            std::vector<int> cws{spa_lds_cw(c->dev, std::max(1, batch))};
            for (int cw : {fit, 8, 16, 32})
                if (cw <= fit && std::find(cws.begin(), cws.end(), cw) == cws.end()) cws.push_back(cw);
            for (int cw : cws) {
                for (int thr : {256, 512, 1024}) {
                    Plan q;
                    q.family = FAMILY_SPA_LDS;
                    q.schedule = LDPCX_SCHED_FLOODING;
                    q.cpw = cw;
                    q.threads = thr;
                    out.push_back(q);
                }
            }
        }
        return out;
    }
    if (c->g > 2) {
        if (p->rule != LDPCX_RULE_MINMAX || c->g > 64) return out;
        // Min-Max: under AUTO the layered schedule is the other candidate; for codes whose
        // messages of 64 codewords fit in LDS, the one-group-per-workgroup kernel too
        std::vector<int> scheds{def.schedule};
        if (p->schedule == LDPCX_SCHED_AUTO) scheds.push_back(LDPCX_SCHED_LAYERED);
        for (int sched : scheds) {
            Plan pl = def;
            pl.schedule = sched;
            pl.family = FAMILY_NB;
            pl.threads = 256;
            out.push_back(pl);
            for (int thr : {256, 512, 1024}) {
                if (nb_lds_bytes(c->dev, thr / 64) > (size_t)160 * 1024) continue;
                Plan q = pl;
                q.family = FAMILY_NB_LDS;
                q.threads = thr;
                out.push_back(q);
            }
        }
        return out;
    }
    std::vector<int> scheds;
    if (p->schedule == LDPCX_SCHED_AUTO) {
        scheds.push_back(LDPCX_SCHED_FLOODING);
        if (c->layers_ok) scheds.push_back(LDPCX_SCHED_LAYERED);
    } else {
        scheds.push_back(p->schedule);
    }
    const DeviceInfo &di = device_info(c->device);
    for (int sched : scheds) {
        const bool lay = sched == LDPCX_SCHED_LAYERED;
        if (c->qc_ok) {
            for (int np : {1, 2, 3, 4, 6, 8, 12, 16}) {
                if (c->qc.Z * np > 512) break;
                if (bin_qc_smem_bytes(c->qc, c->dev, lay, np) > (size_t)di.lds_per_block) break;
                if (np > 1 && ((batch + 1) / 2 + np - 1) / np < di.cus / 2) break;
                Plan pl;
                pl.family = FAMILY_BIN_QC;
                pl.schedule = sched;
                pl.cpw = 2 * np;
                pl.threads = c->qc.Z * np;
                out.push_back(pl);
            }
        }
        const size_t per_cw = bin_lds_smem_bytes(c->dev, lay, 1);
        if (per_cw <= (size_t)di.lds_per_block) {
            for (int cpw : {1, 2, 3, 4, 6, 8, 12, 16}) {
                if (bin_lds_smem_bytes(c->dev, lay, cpw) > (size_t)di.lds_per_block) break;
                if (cpw > 1 && (batch + cpw - 1) / cpw < di.cus / 2) break;
                const int rows = lay ? std::max(1, c->desc.z) : c->dev.m;
                const int need = ((rows * cpw + 63) / 64) * 64;
                for (int thr : {64, 128, 192, 256, 384, 512, 768, 1024}) {
                    if (thr > need && thr != 64) break;
                    Plan pl;
                    pl.family = FAMILY_BIN_LDS;
                    pl.schedule = sched;
                    pl.cpw = cpw;
                    pl.threads = thr;
                    out.push_back(pl);
                }
            }
        }
        if (!lay) {
            // interleaved: codewords per launch sequence (smaller slices keep their
            // state resident in the last-level cache)
            int last = -1;
            for (int sub : {256, 512, 1024, 2048, 4096}) {
                Plan pl;
                pl.family = FAMILY_BIN_IL;
                pl.schedule = LDPCX_SCHED_FLOODING;
                pl.cpw = bin_il_sub_batch(c->dev, batch, sub);
                pl.threads = 256;
                if (pl.cpw == last) continue;
                last = pl.cpw;
                out.push_back(pl);
            }
        }
    }
    return out;
}

}  // namespace

extern "C" ldpcx_status ldpcx_tune(const ldpcx_code *code, const ldpcx_decode_params *params, int32_t batch,
                                   int32_t *chosen_schedule, float *best_us, void *stream) {
    try {
        if (!code) return fail(LDPCX_E_INVAL, "code is NULL");
        ldpcx_code *c = const_cast<ldpcx_code *>(code);
        ldpcx_status st = check_params(c, params);
        if (st != LDPCX_OK) return st;
        if (batch <= 0) return fail(LDPCX_E_INVAL, "batch must be positive");
        if (c->nb_unsupported) return fail(LDPCX_E_UNSUPPORTED, "no Min-Max kernel for this field size");
        if ((st = check_device(c)) != LDPCX_OK) return st;
        hipStream_t s = (hipStream_t)stream;
        // Synthetic input: all-positive LLRs (timing does not depend on values at a fixed
        // iteration count; early stop is switched off for the measurement).
        ldpcx_decode_params tp = *params;
        tp.early_stop = 0;
        const size_t n = c->dev.n, g = c->g;
        const size_t in_bytes = g == 2 ? (size_t)batch * n : (size_t)batch * n * g * 2;
        const size_t hard_bytes = g == 2 ? (size_t)batch * ((n + 7) / 8) : (size_t)batch * n;
        void *buf = nullptr;
        hipError_t e = hipMalloc(&buf, in_bytes + hard_bytes + 3 * (size_t)batch + 256);
        if (e != hipSuccess) return fail(LDPCX_E_NOMEM, "tuning buffers");
        char *b = (char *)buf;
        (void)hipMemsetAsync(b, g == 2 ? 5 : 1, in_bytes, s);
        DecodeIO io{b, b + in_bytes, (uint8_t *)(b + in_bytes + hard_bytes),
                    (int16_t *)(b + align_up(in_bytes + hard_bytes + batch, 2)), nullptr, nullptr, nullptr};
        hipEvent_t e0, e1;
        (void)hipEventCreate(&e0);
        (void)hipEventCreate(&e1);
        float best = 1e30f;
        Plan bestp = default_plan(c, params, batch);
        for (const Plan &pl : candidates(c, params, batch)) {
            if (run_plan(c, &tp, pl, batch, io, s) != LDPCX_OK) continue;  // warm-up / feasibility
            (void)hipEventRecord(e0, s);
            const int reps = 3;
            bool ok = true;
            for (int r = 0; r < reps && ok; ++r) ok = run_plan(c, &tp, pl, batch, io, s) == LDPCX_OK;
            (void)hipEventRecord(e1, s);
            if (!ok || hipEventSynchronize(e1) != hipSuccess) continue;
            float ms = 0.f;
            (void)hipEventElapsedTime(&ms, e0, e1);
            const float us = ms * 1000.f / reps;
            if (us < best) {
                best = us;
                bestp = pl;
            }
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        (void)hipStreamSynchronize(s);
        (void)hipFree(buf);
        {
            std::lock_guard<std::mutex> lk(c->mu);
            c->tuned[tune_key(params, batch)] = bestp;
        }
        if (chosen_schedule) *chosen_schedule = bestp.schedule;
        if (best_us) *best_us = best;
        g_err.clear();
        return LDPCX_OK;
    } catch (const std::exception &ex) {
        return fail(LDPCX_E_NOMEM, ex.what());
    }
}
