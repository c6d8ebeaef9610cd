// Continuous-batching decode server.
//
// A scheduler thread owns a few launch slots (one stream each).  Whenever a slot
// is free and requests wait, it admits waiting codewords in arrival order while
// the device-memory budget allows, splitting a request that only partly fits at
// a codeword boundary, and launches the admitted chunks together: one pinned
// staging copy of the inputs, one ragged persistent launch for the codes whose
// state fits a workgroup, Min-Max codewords included whatever their number and
// schedule (long interleaved-layout codes, FFT-SPA and Min-Max codes too large for
// one-codeword items get their own launch sequence on the same stream), one copy of the outputs
// back, and an event.  Launches on different slots overlap on the device, so a
// request that arrives while others run starts without waiting for them.
// Completed launches are retired by polling their events: outputs are copied to
// the requests' host buffers and their budget is released.
//
// Every chunk is planned at its own size when it is admitted (the autotuner's choice
// can differ between batch classes); its budget charge counts that plan's workspace
// and its launch runs that exact plan.  Min-Max codewords that run as one-codeword
// items need no workspace and are charged their inputs and outputs only.
//
// Failure handling: a launch whose staging, enqueue or device work fails finishes the
// requests of its chunks with that status (LDPCX_E_DEVICE for a device fault) and
// releases their budget; every other request is unaffected and the scheduler keeps
// serving.  For tests, LDPCX_FAULT_INJECT=launch:N (read at server creation) makes the
// server's N-th launch report LDPCX_E_DEVICE without touching the device.
//
// Locking: `mu` guards the request table, the queue and the counters.  `io_mu`
// is held while a launch reads request inputs from host memory and by cancel, so
// that a cancelled request's host buffers are never touched after cancel
// returns.  Order: io_mu before mu.
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <condition_variable>
#include <deque>
#include <map>
#include <thread>

#include "admit.h"
#include "runtime.h"

namespace ldpcx {
namespace {

using Clock = std::chrono::steady_clock;

// Min-Max chunks of the interleaved family (codes too large for one-codeword items)
// with at least this many groups of 64 codewords run as their own launch sequence
// (parallel over checks and codewords), not as per-group ragged items (one workgroup
// per 64 codewords).
constexpr int kOwnLaunchGroups = 2;
// A ragged launch stops taking chunks once its estimated device time reaches this,
// so that launches stay short and the slots pipeline.
constexpr double kLaunchTargetUs = 1500.0;
// In continuous mode a chunk with its own launch sequence is cut to about this much
// estimated device time, so that one large request spreads over several slots and
// requests behind it are not held for its whole decode.
constexpr double kOwnChunkTargetUs = 4000.0;

struct Request : admit::Req {
    ldpcx_code *code = nullptr;
    ldpcx_decode_params prm{};
    const char *llr = nullptr;
    char *hard = nullptr;
    uint8_t *ok = nullptr;
    int16_t *it = nullptr;
    size_t in_cw = 0, out_cw = 0;  // bytes per codeword of llr / hard
    int family = FAMILY_BIN_LDS;
    bool nb_items = false;  // Min-Max codewords that run as one-codeword items of ragged launches
    int done_cw = 0;   // codewords whose outputs are in host memory
    int inflight = 0;  // chunks on the device
    bool done = false, released = false;
    ldpcx_status status = LDPCX_OK;
    double t_submit = 0, t_admit = -1, t_done = 0;

    bool own() const override;
    int unit() const override;
    size_t bytes(int n) const override;
    double us(int n) const override;
};

struct Chunk {
    uint64_t id = 0;
    int cw0 = 0, ncw = 0;
    Plan plan;                        // the plan this chunk runs (planned at its size)
    size_t charge = 0;                // budget bytes
    size_t o_llr = 0, o_hard = 0;     // offsets in the launch's device buffer
    size_t o_ok = 0, o_it = 0;
    bool own_launch = false;
};

struct Slot {
    hipStream_t s = nullptr;
    hipEvent_t ev = nullptr;
    bool busy = false;
    uint64_t launch_no = 0;  // 1-based launch count of the server
    std::vector<Chunk> chunks;
    size_t charge = 0;
    size_t in_bytes = 0, out_off = 0, out_bytes = 0, dev_bytes = 0;
    char *pin_in = nullptr, *pin_out = nullptr;
    size_t cap_in = 0, cap_out = 0;
    ldpcx_status st = LDPCX_OK;
};

size_t io_bytes(const Request &r, int ncw) {
    return align_up((size_t)ncw * r.in_cw, 256) + align_up((size_t)ncw * r.out_cw, 256) + align_up((size_t)ncw, 256) +
           align_up((size_t)ncw * 2, 256);
}

// Device bytes one chunk of `ncw` codewords holds while in flight, on the plan it runs
// at that size.
size_t chunk_bytes(const Request &r, int ncw) {
    if (r.nb_items) return io_bytes(r, ncw);  // decoded in place, all state in LDS
    const Plan pl = plan_for(r.code, &r.prm, std::max(1, ncw));
    size_t b = io_bytes(r, ncw) + work_bytes(r.code, &r.prm, pl, ncw);
    // a chunk of a whole-device family inside a ragged batch is decoded from a gathered copy
    if (pl.family != FAMILY_BIN_QC && pl.family != FAMILY_BIN_LDS) b += io_bytes(r, ncw);
    return b;
}

// Rough device time of a chunk at the iteration cap (only used to size launches):
// edge updates per microsecond per family, from the kernels' measured throughput.
double est_us(const Request &r, int ncw) {
    const double work = (double)ncw * std::max(1, r.prm.max_iters) * r.code->dev.E;
    switch (r.nb_items ? FAMILY_NB1 : r.family) {
    case FAMILY_BIN_QC: return work / 2.5e6;
    case FAMILY_BIN_LDS: return work / 1.0e6;
    case FAMILY_BIN_IL: return work / 1.1e6;
    case FAMILY_SPA:
    case FAMILY_SPA_LDS: return work * ((double)r.code->g / 64.0) / 2.0e4;
    case FAMILY_NB1: return work * ((double)r.code->g * r.code->g / 4096.0) / 5.0e3;
    default: return work * ((double)r.code->g * r.code->g / 4096.0) / 3.0e3;
    }
}

bool Request::own() const {
    return family == FAMILY_BIN_IL || family == FAMILY_SPA || family == FAMILY_SPA_LDS ||
           ((family == FAMILY_NB || family == FAMILY_NB_LDS) && !nb_items &&
            (code->g > 64 || prm.schedule != LDPCX_SCHED_FLOODING || pad64(batch - next_cw) / 64 >= kOwnLaunchGroups));
}

int Request::unit() const { return family == FAMILY_BIN_IL ? bin_il_sub_batch(code->dev, batch - next_cw, 0) : 64; }

size_t Request::bytes(int n) const { return chunk_bytes(*this, n); }

double Request::us(int n) const { return est_us(*this, n); }

bool grow_pinned(char *&p, size_t &cap, size_t need) {
    if (need <= cap) return true;
    if (p) (void)hipHostFree(p);
    p = nullptr;
    cap = 0;
    size_t c = std::max<size_t>(need, 1 << 20);
    if (hipHostMalloc((void **)&p, c, hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        p = nullptr;
        return false;
    }
    cap = c;
    return true;
}

}  // namespace
}  // namespace ldpcx

using namespace ldpcx;

struct ldpcx_server {
    ldpcx_server_config cfg{};
    int device = 0;
    Clock::time_point t0;
    std::mutex mu, io_mu;
    std::condition_variable cv_work, cv_done;
    bool stop = false;
    uint64_t next_id = 1;
    std::map<uint64_t, Request> reqs;
    std::deque<uint64_t> queue;
    std::vector<Slot> slots;
    size_t in_use = 0, peak = 0;
    uint64_t completed = 0, codewords = 0, launches = 0;
    uint64_t fault_launch = 0;  // LDPCX_FAULT_INJECT=launch:N, 0 = off
    std::thread th;

    double now_us() const { return std::chrono::duration<double, std::micro>(Clock::now() - t0).count(); }

    // Mark request `id` finished and drop what it still has queued (mu held).
    void finish(uint64_t id, Request &r, ldpcx_status st) {
        if (r.done) return;
        r.done = true;
        r.status = st;
        r.t_done = now_us();
        if (st == LDPCX_OK) ++completed;
        for (auto it = queue.begin(); it != queue.end(); ++it)
            if (*it == id) {
                queue.erase(it);
                break;
            }
        cv_done.notify_all();
    }

    void maybe_erase(uint64_t id) {
        auto it = reqs.find(id);
        if (it != reqs.end() && it->second.released && it->second.done && it->second.inflight == 0) reqs.erase(it);
    }

    // Take the chunks of the next launch (mu held).
    std::vector<Chunk> form(bool others_in_flight) {
        admit::Config ac;
        ac.continuous = cfg.mode == LDPCX_SERVE_CONTINUOUS;
        ac.max_launch_cw = cfg.max_launch_cw;
        ac.budget = cfg.hbm_budget;
        ac.launch_target_us = kLaunchTargetUs;
        ac.own_chunk_target_us = kOwnChunkTargetUs;
        const std::vector<admit::Take> takes = admit::form(
            queue, [&](uint64_t id) -> admit::Req & { return reqs.at(id); }, ac, in_use, others_in_flight);
        std::vector<Chunk> out;
        out.reserve(takes.size());
        for (const admit::Take &t : takes) {
            Request &r = reqs.at(t.id);
            Chunk c;
            c.id = t.id;
            c.cw0 = t.cw0;
            c.ncw = t.ncw;
            c.plan = plan_for(r.code, &r.prm, t.ncw);
            c.charge = t.charge;
            c.own_launch = t.own;
            r.inflight += 1;
            if (r.t_admit < 0) r.t_admit = now_us();
            out.push_back(c);
        }
        return out;
    }

    // Stage inputs and enqueue the launch of slot `sl` (mu not held).
    void launch(Slot &sl) {
        sl.st = LDPCX_OK;
        if (fault_launch && sl.launch_no == fault_launch) {
            // injected failure: nothing reaches the device, the event completes at once
            sl.st = fail(LDPCX_E_DEVICE, "injected launch fault");
            if (hipEventRecord(sl.ev, sl.s) != hipSuccess) (void)hipGetLastError();
            return;
        }
        // Device layout: all inputs, then all hard decisions, flags and counts, each
        // chunk 256-byte aligned; the pinned buffers mirror the input and output parts.
        size_t off = 0;
        {
            std::lock_guard<std::mutex> lk(mu);
            for (Chunk &c : sl.chunks) {
                const Request &r = reqs.at(c.id);
                c.o_llr = off;
                off += align_up((size_t)c.ncw * r.in_cw, 256);
            }
            sl.in_bytes = off;
            sl.out_off = off;
            for (Chunk &c : sl.chunks) {
                const Request &r = reqs.at(c.id);
                c.o_hard = off;
                off += align_up((size_t)c.ncw * r.out_cw, 256);
                c.o_ok = off;
                off += align_up((size_t)c.ncw, 256);
                c.o_it = off;
                off += align_up((size_t)c.ncw * 2, 256);
            }
        }
        sl.dev_bytes = off;
        sl.out_bytes = off - sl.out_off;
        char *dbuf = nullptr;
        hipError_t e = hipSuccess;
        {
            std::lock_guard<std::mutex> io(io_mu);
            if (!grow_pinned(sl.pin_in, sl.cap_in, sl.in_bytes) || !grow_pinned(sl.pin_out, sl.cap_out, sl.out_bytes)) {
                sl.st = fail(LDPCX_E_NOMEM, "pinned staging buffers");
            } else {
                for (const Chunk &c : sl.chunks) {
                    const char *src = nullptr;
                    size_t len = 0;
                    {
                        std::lock_guard<std::mutex> lk(mu);
                        const Request &r = reqs.at(c.id);
                        if (!r.done) {
                            src = r.llr + (size_t)c.cw0 * r.in_cw;
                            len = (size_t)c.ncw * r.in_cw;
                        }
                    }
                    if (src) std::memcpy(sl.pin_in + c.o_llr, src, len);
                }
            }
        }
        if (sl.st == LDPCX_OK) {
            e = hipMallocAsync((void **)&dbuf, sl.dev_bytes, sl.s);
            if (e != hipSuccess) sl.st = fail(LDPCX_E_NOMEM, "server device buffer");
        }
        if (sl.st == LDPCX_OK) {
            e = hipMemcpyAsync(dbuf, sl.pin_in, sl.in_bytes, hipMemcpyHostToDevice, sl.s);
            if (e != hipSuccess) sl.st = fail_hip(e, "input upload");
        }
        if (sl.st == LDPCX_OK) {
            std::vector<ldpcx_job> jobs;
            for (const Chunk &c : sl.chunks) {
                Request r;
                {
                    std::lock_guard<std::mutex> lk(mu);
                    r = reqs.at(c.id);
                }
                ldpcx_job j{r.code, r.prm, c.ncw, dbuf + c.o_llr, dbuf + c.o_hard, (uint8_t *)(dbuf + c.o_ok),
                            (int16_t *)(dbuf + c.o_it)};
                if (!c.own_launch) {
                    jobs.push_back(j);
                    continue;
                }
                const DecodeIO io{j.llr, j.hard, j.syndrome_ok, j.iters, nullptr, nullptr, nullptr};
                const ldpcx_status st = run_plan(r.code, &r.prm, c.plan, c.ncw, io, sl.s, false);
                if (st != LDPCX_OK) {
                    sl.st = st;
                    break;
                }
            }
            if (sl.st == LDPCX_OK && !jobs.empty())
                sl.st = ldpcx_decode_ragged(jobs.data(), (int32_t)jobs.size(), sl.s);
        }
        if (sl.st == LDPCX_OK) {
            e = hipMemcpyAsync(sl.pin_out, dbuf + sl.out_off, sl.out_bytes, hipMemcpyDeviceToHost, sl.s);
            if (e != hipSuccess) sl.st = fail_hip(e, "output download");
        }
        if (dbuf) (void)hipFreeAsync(dbuf, sl.s);
        e = hipEventRecord(sl.ev, sl.s);
        if (e != hipSuccess) {
            (void)hipStreamSynchronize(sl.s);
            (void)hipGetLastError();
            (void)hipEventRecord(sl.ev, sl.s);
        }
    }

    // Hand the outputs of a finished launch to its requests (mu held).
    void retire(Slot &sl, bool device_ok) {
        const bool ok = device_ok && sl.st == LDPCX_OK;
        for (const Chunk &c : sl.chunks) {
            auto it = reqs.find(c.id);
            if (it == reqs.end()) continue;
            Request &r = it->second;
            r.inflight -= 1;
            if (!r.done) {
                if (ok) {
                    std::memcpy(r.hard + (size_t)c.cw0 * r.out_cw, sl.pin_out + (c.o_hard - sl.out_off),
                                (size_t)c.ncw * r.out_cw);
                    std::memcpy(r.ok + c.cw0, sl.pin_out + (c.o_ok - sl.out_off), (size_t)c.ncw);
                    std::memcpy(r.it + c.cw0, sl.pin_out + (c.o_it - sl.out_off), (size_t)c.ncw * 2);
                    r.done_cw += c.ncw;
                    codewords += (uint64_t)c.ncw;
                    if (r.done_cw == r.batch) finish(c.id, r, LDPCX_OK);
                } else {
                    finish(c.id, r, sl.st != LDPCX_OK ? sl.st : LDPCX_E_DEVICE);
                }
            }
            maybe_erase(c.id);
        }
        in_use -= sl.charge;
        sl.charge = 0;
        sl.chunks.clear();
        sl.busy = false;
    }

    void run() {
        (void)hipSetDevice(device);
        std::unique_lock<std::mutex> lk(mu);
        for (;;) {
            bool did = false, busy_any = false;
            for (Slot &sl : slots) {
                if (!sl.busy) continue;
                const hipError_t q = hipEventQuery(sl.ev);
                if (q != hipSuccess) (void)hipGetLastError();
                if (q == hipErrorNotReady) {
                    busy_any = true;
                    continue;
                }
                retire(sl, q == hipSuccess);
                did = true;
            }
            if (stop && queue.empty() && !busy_any) break;
            for (Slot &sl : slots) {
                if (sl.busy || queue.empty()) continue;
                std::vector<Chunk> take = form(busy_any);
                if (take.empty()) break;
                sl.busy = true;
                sl.chunks = std::move(take);
                sl.charge = 0;
                for (const Chunk &c : sl.chunks) sl.charge += c.charge;
                in_use += sl.charge;
                peak = std::max(peak, in_use);
                sl.launch_no = ++launches;
                lk.unlock();
                launch(sl);
                lk.lock();
                did = true;
                busy_any = true;
            }
            if (!did) {
                if (busy_any) cv_work.wait_for(lk, std::chrono::microseconds(20));
                else cv_work.wait(lk, [&] { return stop || !queue.empty(); });
            }
        }
    }
};

extern "C" {

ldpcx_status ldpcx_server_create(const ldpcx_server_config *cfg, ldpcx_server **out) {
    try {
        if (!cfg || !out) return fail(LDPCX_E_INVAL, "null argument");
        *out = nullptr;
        if (cfg->hbm_budget == 0) return fail(LDPCX_E_INVAL, "hbm_budget must be positive");
        if (cfg->mode != LDPCX_SERVE_CONTINUOUS && cfg->mode != LDPCX_SERVE_PER_REQUEST)
            return fail(LDPCX_E_INVAL, "unknown serving mode");
        if (cfg->max_inflight < 1 || cfg->max_inflight > 64) return fail(LDPCX_E_INVAL, "max_inflight must be in [1, 64]");
        if (cfg->max_launch_cw < 0) return fail(LDPCX_E_INVAL, "max_launch_cw < 0");
        int dev = 0;
        hipError_t e = hipGetDevice(&dev);
        if (e != hipSuccess) return fail_hip(e, "hipGetDevice");
        device_info(dev);
        ldpcx_server *S = new ldpcx_server();
        S->cfg = *cfg;
        if (S->cfg.mode == LDPCX_SERVE_PER_REQUEST) S->cfg.max_inflight = 1;
        S->device = dev;
        S->t0 = Clock::now();
        {
            const char *fi = getenv("LDPCX_FAULT_INJECT");
            unsigned long long nfi = 0;
            if (fi && sscanf(fi, "launch:%llu", &nfi) == 1) S->fault_launch = nfi;
        }
        S->slots.resize(S->cfg.max_inflight);
        for (Slot &sl : S->slots) {
            e = hipStreamCreateWithFlags(&sl.s, hipStreamNonBlocking);
            if (e == hipSuccess) e = hipEventCreateWithFlags(&sl.ev, hipEventDisableTiming);
            if (e != hipSuccess) {
                for (Slot &t : S->slots) {
                    if (t.ev) (void)hipEventDestroy(t.ev);
                    if (t.s) (void)hipStreamDestroy(t.s);
                }
                delete S;
                return fail_hip(e, "server streams");
            }
        }
        S->th = std::thread([S] { S->run(); });
        *out = S;
        return LDPCX_OK;
    } catch (const std::exception &ex) {
        return fail(LDPCX_E_NOMEM, ex.what());
    }
}

ldpcx_status ldpcx_server_submit(ldpcx_server *srv, const ldpcx_code *code, const ldpcx_decode_params *params,
                                 int32_t batch, const void *llr_host, void *hard_host, uint8_t *syndrome_ok_host,
                                 int16_t *iters_host, uint64_t *ticket) {
    try {
        if (!srv || !code || !ticket) return fail(LDPCX_E_INVAL, "null argument");
        ldpcx_code *c = const_cast<ldpcx_code *>(code);
        ldpcx_status st = check_params(c, params);
        if (st != LDPCX_OK) return st;
        if (batch < 0) return fail(LDPCX_E_INVAL, "batch < 0");
        if (batch > 0 && (!llr_host || !hard_host || !syndrome_ok_host || !iters_host))
            return fail(LDPCX_E_INVAL, "null buffer");
        if (c->device != srv->device) return fail(LDPCX_E_INVAL, "code handle lives on another device");
        if (c->nb_unsupported) return fail(LDPCX_E_UNSUPPORTED, "no Min-Max kernel for this field size");
        Request r;
        r.code = c;
        r.prm = *params;
        r.batch = batch;
        r.llr = (const char *)llr_host;
        r.hard = (char *)hard_host;
        r.ok = syndrome_ok_host;
        r.it = iters_host;
        const int n = c->dev.n;
        r.in_cw = c->g == 2 ? (size_t)n : (size_t)n * c->g * 2;
        r.out_cw = c->g == 2 ? (size_t)(n + 7) / 8 : (size_t)n;
        r.family = plan_for(c, params, std::max(1, batch)).family;
        // Min-Max codes whose codewords are items of the persistent kernel (one codeword
        // per item, any schedule) always join the ragged launches
        r.nb_items = srv->cfg.mode != LDPCX_SERVE_PER_REQUEST && ragged_nb1_items(c, params);
        if (batch > 0 && chunk_bytes(r, 1) > srv->cfg.hbm_budget)
            return fail(LDPCX_E_BUDGET, "one codeword does not fit the server's memory budget");
        std::lock_guard<std::mutex> lk(srv->mu);
        if (srv->stop) return fail(LDPCX_E_CANCELLED, "server is shutting down");
        r.t_submit = srv->now_us();
        const uint64_t id = srv->next_id++;
        Request &in = srv->reqs.emplace(id, r).first->second;
        if (batch == 0) {
            in.t_admit = in.t_submit;
            srv->finish(id, in, LDPCX_OK);
        } else {
            srv->queue.push_back(id);
            srv->cv_work.notify_one();
        }
        *ticket = id;
        return LDPCX_OK;
    } catch (const std::exception &ex) {
        return fail(LDPCX_E_NOMEM, ex.what());
    }
}

ldpcx_status ldpcx_server_poll(ldpcx_server *srv, uint64_t ticket, int32_t *done) {
    if (!srv || !done) return fail(LDPCX_E_INVAL, "null argument");
    std::lock_guard<std::mutex> lk(srv->mu);
    auto it = srv->reqs.find(ticket);
    if (it == srv->reqs.end() || it->second.released) return fail(LDPCX_E_NOTFOUND, "unknown ticket");
    *done = it->second.done ? 1 : 0;
    return LDPCX_OK;
}

ldpcx_status ldpcx_server_wait(ldpcx_server *srv, uint64_t ticket, int32_t timeout_ms, double *t_submit_us,
                               double *t_admit_us, double *t_done_us) {
    if (!srv) return fail(LDPCX_E_INVAL, "null argument");
    std::unique_lock<std::mutex> lk(srv->mu);
    auto it = srv->reqs.find(ticket);
    if (it == srv->reqs.end() || it->second.released) return fail(LDPCX_E_NOTFOUND, "unknown ticket");
    auto is_done = [&] {
        auto j = srv->reqs.find(ticket);
        return j == srv->reqs.end() || j->second.done;
    };
    if (timeout_ms < 0) srv->cv_done.wait(lk, is_done);
    else if (!srv->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), is_done))
        return fail(LDPCX_E_TIMEOUT, "request still pending");
    it = srv->reqs.find(ticket);
    if (it == srv->reqs.end()) return fail(LDPCX_E_NOTFOUND, "unknown ticket");
    Request &r = it->second;
    if (t_submit_us) *t_submit_us = r.t_submit;
    if (t_admit_us) *t_admit_us = r.t_admit;
    if (t_done_us) *t_done_us = r.t_done;
    const ldpcx_status st = r.status;
    r.released = true;
    srv->maybe_erase(ticket);
    if (st == LDPCX_E_CANCELLED) return fail(st, "request was cancelled");
    if (st != LDPCX_OK) return fail(st, "request failed on the device");
    return LDPCX_OK;
}

ldpcx_status ldpcx_server_cancel(ldpcx_server *srv, uint64_t ticket) {
    if (!srv) return fail(LDPCX_E_INVAL, "null argument");
    std::lock_guard<std::mutex> io(srv->io_mu);
    std::lock_guard<std::mutex> lk(srv->mu);
    auto it = srv->reqs.find(ticket);
    if (it == srv->reqs.end() || it->second.released) return fail(LDPCX_E_NOTFOUND, "unknown ticket");
    srv->finish(ticket, it->second, LDPCX_E_CANCELLED);
    return LDPCX_OK;
}

ldpcx_status ldpcx_server_stats(ldpcx_server *srv, uint64_t *completed, uint64_t *codewords, uint64_t *launches,
                                uint64_t *peak_bytes) {
    if (!srv) return fail(LDPCX_E_INVAL, "null argument");
    std::lock_guard<std::mutex> lk(srv->mu);
    if (completed) *completed = srv->completed;
    if (codewords) *codewords = srv->codewords;
    if (launches) *launches = srv->launches;
    if (peak_bytes) *peak_bytes = srv->peak;
    return LDPCX_OK;
}

ldpcx_status ldpcx_server_destroy(ldpcx_server *srv) {
    if (!srv) return fail(LDPCX_E_INVAL, "null argument");
    {
        std::lock_guard<std::mutex> io(srv->io_mu);
        std::lock_guard<std::mutex> lk(srv->mu);
        srv->stop = true;
        while (!srv->queue.empty()) {
            auto it = srv->reqs.find(srv->queue.front());
            if (it != srv->reqs.end()) srv->finish(it->first, it->second, LDPCX_E_CANCELLED);
            else srv->queue.pop_front();
        }
        srv->cv_work.notify_all();
    }
    if (srv->th.joinable()) srv->th.join();
    for (Slot &sl : srv->slots) {
        if (sl.ev) (void)hipEventDestroy(sl.ev);
        if (sl.s) (void)hipStreamDestroy(sl.s);
        if (sl.pin_in) (void)hipHostFree(sl.pin_in);
        if (sl.pin_out) (void)hipHostFree(sl.pin_out);
    }
    delete srv;
    return LDPCX_OK;
}

}  // extern "C"
