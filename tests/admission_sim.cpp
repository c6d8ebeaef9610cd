// CPU simulation of the decode server's admission policy (admit.h) against a fake
// backend: launches complete after their estimated device time (scaled by a random
// factor), requests arrive over time or all at once, and an optional launch fails.  The
// scheduler loop mirrors the server's: retire completed launches, then fill every free
// slot with the chunks the policy takes.  Every invariant of the policy is checked as
// it runs; a violation prints a message and exits with status 1.  On success one JSON
// line of counters is printed.
//
// usage: admission_sim seed continuous(0|1) budget_bytes slots max_launch_cw nreq
//                      arrivals(0: all at once, 1: spread) fail_launch(0: none)
//                      [launch_target_us]
#include <cstdio>
#include <cstdlib>
#include <map>
#include <random>
#include <algorithm>
#include <cmath>
#include <string>

#include "admit.h"

using ldpcx::admit::Config;
using ldpcx::admit::Req;
using ldpcx::admit::Take;

namespace {

[[noreturn]] void die(const std::string &m) {
    std::fprintf(stderr, "admission_sim: %s\n", m.c_str());
    std::exit(1);
}

// Kinds of request: per-codeword bytes, a workspace that grows in steps of 64
// codewords, a granularity and whether the remaining codewords take a launch of their own.
struct FakeReq : Req {
    int kind = 0;
    size_t in_cw = 0, ws_per_group = 0;
    double us_per_cw = 0;
    int admitted = 0, done_cw = 0, nchunks = 0;
    bool failed = false, rejected = false;
    double t_arrive = 0;
    bool own() const override {
        if (kind == 2) return true;                                // long code: always its own launch
        if (kind == 3) return ((batch - next_cw + 63) / 64) >= 2;  // two or more groups of 64
        return false;
    }
    int unit() const override { return kind == 2 ? 48 : 64; }
    size_t bytes(int n) const override { return (size_t)n * in_cw + (size_t)((n + 63) / 64) * ws_per_group; }
    double us(int n) const override { return n * us_per_cw; }
};

struct Launch {
    double t_end = 0;
    std::vector<Take> chunks;
    size_t charge = 0;
    bool fails = false;
};

}  // namespace

int main(int argc, char **argv) {
    if (argc != 9 && argc != 10)
        die("usage: seed continuous budget slots max_launch_cw nreq arrivals fail_launch [launch_target_us]");
    const unsigned seed = (unsigned)std::strtoul(argv[1], nullptr, 10);
    Config cfg;
    cfg.continuous = std::atoi(argv[2]) != 0;
    cfg.budget = (size_t)std::strtoull(argv[3], nullptr, 10);
    int nslots = std::atoi(argv[4]);
    cfg.max_launch_cw = std::atoi(argv[5]);
    const int nreq = std::atoi(argv[6]);
    const bool spread = std::atoi(argv[7]) != 0;
    const long fail_launch = std::atol(argv[8]);
    if (argc == 10) cfg.launch_target_us = std::atof(argv[9]);
    if (!cfg.continuous) nslots = 1;

    std::mt19937_64 rng(seed);
    std::uniform_real_distribution<double> U(0.0, 1.0);
    std::map<uint64_t, FakeReq> reqs;
    double t = 0;
    for (int i = 0; i < nreq; ++i) {
        FakeReq r;
        r.kind = (int)(U(rng) * 4);
        r.batch = (int)std::exp(U(rng) * std::log(4097.0));
        static const size_t in_cw[4] = {192, 2304, 64800, 24576};
        static const size_t ws[4] = {0, 0, 64 * 260000, 64 * 40000};
        static const double us[4] = {0.02, 0.05, 6.0, 1.5};
        r.in_cw = in_cw[r.kind];
        r.ws_per_group = ws[r.kind];
        r.us_per_cw = us[r.kind];
        if (spread) t += -std::log(1.0 - U(rng)) * 300.0;
        r.t_arrive = t;
        reqs.emplace((uint64_t)i + 1, r);
    }

    std::deque<uint64_t> queue;
    std::vector<Launch> slots(nslots);
    std::vector<bool> busy(nslots, false);
    auto lookup = [&](uint64_t id) -> Req & { return reqs.at(id); };
    size_t in_use = 0, peak = 0;
    long launches = 0, chunks = 0, max_busy = 0;
    uint64_t next_arrival = 1;
    double now = 0;

    for (;;) {
        // next event: the earliest completion or arrival
        double t_next = 1e300;
        for (int s = 0; s < nslots; ++s)
            if (busy[s]) t_next = std::min(t_next, slots[s].t_end);
        if (next_arrival <= (uint64_t)nreq) t_next = std::min(t_next, reqs.at(next_arrival).t_arrive);
        if (t_next == 1e300) {
            if (!queue.empty()) die("queue not empty with nothing in flight and no arrival left");
            break;
        }
        now = t_next;
        // retire
        for (int s = 0; s < nslots; ++s) {
            if (!busy[s] || slots[s].t_end > now) continue;
            for (const Take &c : slots[s].chunks) {
                FakeReq &r = reqs.at(c.id);
                if (slots[s].fails) {
                    if (!r.failed) {
                        r.failed = true;
                        for (auto it = queue.begin(); it != queue.end(); ++it)
                            if (*it == c.id) {
                                queue.erase(it);
                                break;
                            }
                    }
                } else if (!r.failed) {
                    r.done_cw += c.ncw;
                }
            }
            if (slots[s].charge > in_use) die("released more budget than held");
            in_use -= slots[s].charge;
            busy[s] = false;
        }
        // arrivals (a request whose single codeword exceeds the budget is rejected at submit)
        while (next_arrival <= (uint64_t)nreq && reqs.at(next_arrival).t_arrive <= now) {
            FakeReq &r = reqs.at(next_arrival);
            if (r.bytes(1) > cfg.budget) r.rejected = true;
            else queue.push_back(next_arrival);
            ++next_arrival;
        }
        // fill free slots
        bool busy_any = false;
        for (int s = 0; s < nslots; ++s) busy_any = busy_any || busy[s];
        for (int s = 0; s < nslots; ++s) {
            if (busy[s] || queue.empty()) continue;
            const std::deque<uint64_t> before = queue;
            std::map<uint64_t, int> next_before;
            for (uint64_t id : before) next_before[id] = reqs.at(id).next_cw;
            std::vector<Take> take = ldpcx::admit::form(queue, lookup, cfg, in_use, busy_any);
            if (take.empty()) {
                if (!busy_any) die("nothing admitted with nothing in flight (no progress)");
                break;
            }
            // chunks come from the front of the queue, in order, each starting where the
            // request's admission stopped, contiguous and non-empty
            size_t charge = 0;
            int ncw = 0;
            double us = 0;
            for (size_t k = 0; k < take.size(); ++k) {
                const Take &c = take[k];
                if (k >= before.size() || before[k] != c.id) die("chunk not taken in queue order");
                FakeReq &r = reqs.at(c.id);
                if (c.ncw <= 0) die("empty chunk");
                if (c.cw0 != next_before[c.id] || c.cw0 != r.admitted) die("chunk does not start where admission stopped");
                if (c.charge != r.bytes(c.ncw)) die("charge differs from the request's bytes");
                if (k > 0 && us >= cfg.launch_target_us) die("ragged launch grew past its time target");
                if (k + 1 < take.size() && c.cw0 + c.ncw != r.batch) die("a partly admitted request was passed");
                if (c.own && take.size() != 1) die("own chunk shares its launch");
                if (cfg.continuous) {
                    // cut to its time target (own launch or ragged batch), in whole units
                    const double per_cw = r.us(1024) / 1024.0;
                    const double target = c.own ? cfg.own_chunk_target_us : cfg.launch_target_us;
                    const double lim_d = target / per_cw;
                    if (c.ncw > lim_d && c.ncw > r.unit())
                        die(c.own ? "own chunk longer than its time target" : "ragged chunk longer than the launch target");
                    // a request that fits its target whole is not split by the cut
                    if (lim_d >= (double)(r.batch - c.cw0) && c.ncw < r.batch - c.cw0 &&
                        r.bytes(r.batch - c.cw0) + in_use + charge <= cfg.budget &&
                        (cfg.max_launch_cw == 0 || ncw + r.batch - c.cw0 <= cfg.max_launch_cw))
                        die("a request that fits its time target was split");
                }
                // arrival order: every earlier request (not rejected or failed) is fully admitted
                for (auto it = reqs.begin(); it != reqs.end() && it->first < c.id; ++it) {
                    const FakeReq &e = it->second;
                    if (!e.rejected && !e.failed && e.admitted < e.batch)
                        die("a later request was admitted before an earlier one");
                }
                r.admitted += c.ncw;
                r.nchunks += 1;
                charge += c.charge;
                ncw += c.ncw;
                us += r.us(c.ncw);
            }
            if (!cfg.continuous && take.size() != 1) die("per-request mode put several chunks in one launch");
            if (cfg.max_launch_cw > 0 && ncw > cfg.max_launch_cw) die("launch exceeds the codeword cap");
            in_use += charge;
            if (in_use > cfg.budget) die("budget exceeded");
            peak = std::max(peak, in_use);
            Launch &L = slots[s];
            L.chunks = take;
            L.charge = charge;
            L.t_end = now + us * (0.5 + U(rng));
            L.fails = ++launches == fail_launch;
            chunks += (long)take.size();
            busy[s] = true;
            busy_any = true;
            long nb = 0;
            for (int q = 0; q < nslots; ++q) nb += busy[q] ? 1 : 0;
            max_busy = std::max(max_busy, nb);
        }
    }

    long split = 0, failed = 0, rejected = 0, cw = 0;
    for (auto &kv : reqs) {
        const FakeReq &r = kv.second;
        if (r.rejected) {
            ++rejected;
            continue;
        }
        if (r.failed) {
            ++failed;
            continue;
        }
        if (r.admitted != r.batch || r.done_cw != r.batch) die("request " + std::to_string(kv.first) + " not completed whole");
        cw += r.batch;
        if (r.nchunks > 1) ++split;
    }
    std::printf("{\"launches\": %ld, \"chunks\": %ld, \"requests\": %d, \"completed_cw\": %ld, \"failed\": %ld, "
                "\"rejected\": %ld, \"split\": %ld, \"peak\": %zu, \"budget\": %zu, \"max_busy\": %ld}\n",
                launches, chunks, nreq, cw, failed, rejected, split, peak, cfg.budget, max_busy);
    return 0;
}
