// Autotuner: times candidate launch plans of one (code, params, batch) on the
// device and caches the fastest in the code handle.  Candidates are the kernel
// family's tunable knobs (codewords per workgroup and threads per workgroup for
// the LDS-resident binary decoder) and, only when the caller asked for the AUTO
// schedule, the schedule itself (flooding versus layered): the two schedules
// are different algorithms, so a fixed schedule is never changed.
//
// Tuned plans can persist across processes: when the environment variable
// LDPCX_TUNE_CACHE names a file, every ldpcx_tune result is merged into it and
// ldpcx_code_create loads the entries of its code (by a hash of the description) and
// device (architecture and compute-unit count).  The file is JSON, one entry object
// per line, rewritten through a temporary file and a rename.
#include <algorithm>
#include <cctype>
#include <cinttypes>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "runtime.h"

using namespace ldpcx;

namespace ldpcx {

uint64_t code_hash(const ldpcx_code_desc *d) {
    uint64_t h = 1469598103934665603ULL;  // FNV-1a
    auto mix = [&](const void *p, size_t n) {
        const unsigned char *b = (const unsigned char *)p;
        for (size_t i = 0; i < n; ++i) h = (h ^ b[i]) * 1099511628211ULL;
    };
    const int32_t hdr[5] = {d->g, (int32_t)d->prim_poly, d->n, d->m, d->z};
    mix(hdr, sizeof hdr);
    const int E = d->row_ptr[d->m];
    mix(d->row_ptr, sizeof(int32_t) * (size_t)(d->m + 1));
    mix(d->col_idx, sizeof(int32_t) * (size_t)E);
    if (d->g > 2 && d->h_val) mix(d->h_val, (size_t)E);
    return h;
}

namespace {

std::mutex g_cache_mu;

const char *cache_path() {
    const char *p = getenv("LDPCX_TUNE_CACHE");
    return (p && p[0]) ? p : nullptr;
}

std::string device_tag(int dev) {
    hipDeviceProp_t prop;
    char buf[160];
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) {
        (void)hipGetLastError();
        return "unknown";
    }
    snprintf(buf, sizeof buf, "%s/%d", prop.gcnArchName, prop.multiProcessorCount);
    for (char *q = buf; *q; ++q)
        if (*q == '"' || *q == '\\') *q = '_';
    return buf;
}

struct Entry {
    uint64_t code, key;
    std::string device;
    Plan pl;
    float us;
};

// Value of "name" inside one JSON object's text (strings without their quotes), or "".
std::string json_field(const std::string &obj, const char *name) {
    const std::string key = std::string("\"") + name + "\"";
    size_t p = obj.find(key);
    if (p == std::string::npos) return "";
    p = obj.find(':', p + key.size());
    if (p == std::string::npos) return "";
    ++p;
    while (p < obj.size() && isspace((unsigned char)obj[p])) ++p;
    if (p < obj.size() && obj[p] == '"') {
        const size_t q = obj.find('"', p + 1);
        return q == std::string::npos ? "" : obj.substr(p + 1, q - p - 1);
    }
    size_t q = p;
    while (q < obj.size() && obj[q] != ',' && obj[q] != '}' && !isspace((unsigned char)obj[q])) ++q;
    return obj.substr(p, q - p);
}

// Entries of the cache file: every {...} object with all fields (others are dropped).
std::vector<Entry> read_entries(const char *path) {
    std::vector<Entry> out;
    FILE *f = fopen(path, "r");
    if (!f) return out;
    std::string text;
    char buf[4096];
    size_t got;
    while ((got = fread(buf, 1, sizeof buf, f)) > 0) text.append(buf, got);
    fclose(f);
    for (size_t p = text.find('{'); p != std::string::npos; p = text.find('{', p + 1)) {
        const size_t q = text.find('}', p);
        if (q == std::string::npos) break;
        const std::string obj = text.substr(p, q - p + 1);
        const char *names[8] = {"code", "device", "key", "family", "schedule", "cw_per_wg", "threads", "us"};
        std::string v[8];
        bool all = true;
        for (int i = 0; i < 8 && all; ++i) all = !(v[i] = json_field(obj, names[i])).empty();
        if (!all) continue;
        Entry e;
        e.code = strtoull(v[0].c_str(), nullptr, 16);
        e.device = v[1];
        e.key = strtoull(v[2].c_str(), nullptr, 16);
        e.pl.family = atoi(v[3].c_str());
        e.pl.schedule = atoi(v[4].c_str());
        e.pl.cpw = atoi(v[5].c_str());
        e.pl.threads = atoi(v[6].c_str());
        e.us = (float)atof(v[7].c_str());
        out.push_back(e);
        p = q;
    }
    return out;
}

}  // namespace

void tune_cache_load(ldpcx_code *c) {
    const char *path = cache_path();
    if (!path) return;
    std::lock_guard<std::mutex> lk(g_cache_mu);
    const std::string dev = device_tag(c->device);
    std::lock_guard<std::mutex> lc(c->mu);
    for (const Entry &e : read_entries(path))
        if (e.code == c->hash && e.device == dev && e.pl.family >= 0 && e.pl.family <= FAMILY_SPA_LDS)
            c->tuned[e.key] = e.pl;
}

void tune_cache_store(const ldpcx_code *c, uint64_t key, const Plan &pl, float us) {
    const char *path = cache_path();
    if (!path) return;
    std::lock_guard<std::mutex> lk(g_cache_mu);
    const std::string dev = device_tag(c->device);
    std::vector<Entry> all = read_entries(path);
    all.erase(std::remove_if(all.begin(), all.end(),
                             [&](const Entry &e) { return e.code == c->hash && e.device == dev && e.key == key; }),
              all.end());
    all.push_back(Entry{c->hash, key, dev, pl, us});
    const std::string tmp = std::string(path) + ".tmp";
    FILE *f = fopen(tmp.c_str(), "w");
    if (!f) return;  // best effort: an unwritable cache only costs a re-tune
    fprintf(f, "[\n");
    for (size_t i = 0; i < all.size(); ++i) {
        const Entry &e = all[i];
        fprintf(f,
                " {\"code\": \"%016" PRIx64 "\", \"device\": \"%s\", \"key\": \"%016" PRIx64
                "\", \"family\": %d, \"schedule\": %d, \"cw_per_wg\": %d, \"threads\": %d, \"us\": %.1f}%s\n",
                e.code, e.device.c_str(), e.key, e.pl.family, e.pl.schedule, e.pl.cpw, e.pl.threads, e.us,
                i + 1 < all.size() ? "," : "");
    }
    fprintf(f, "]\n");
    const bool ok = fclose(f) == 0;
    if (ok) (void)std::rename(tmp.c_str(), path);
}

}  // namespace ldpcx

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
            if (nb1_supported(c->dev, nb_amax(p)))
                for (int thr : {256, 512, 768, 1024}) {
                    if (c->dev.dc_max > 4 && thr > 256) break;
                    Plan q = pl;
                    q.family = FAMILY_NB1;
                    q.cpw = 1;
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
                if (!lay && bin_qc_lp_ok(c->qc, np)) {  // flooding with the layers in parallel
                    pl.threads = c->qc.Z * np * c->qc.nl;
                    out.push_back(pl);
                }
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
        tune_cache_store(c, tune_key(params, batch), bestp, best);
        if (chosen_schedule) *chosen_schedule = bestp.schedule;
        if (best_us) *best_us = best;
        g_err.clear();
        return LDPCX_OK;
    } catch (const std::exception &ex) {
        return fail(LDPCX_E_NOMEM, ex.what());
    }
}
