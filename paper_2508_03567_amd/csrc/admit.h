// Admission policy of the decode server: which waiting codewords the next launch takes.
//
// Host code only (no device calls), so that the server and a CPU simulation of it share
// the same policy.  Requests wait in arrival order.  A launch takes codewords from the
// front of the queue while the device-memory budget allows:
//  * a request that only partly fits is split at a codeword boundary, and nothing behind
//    it is admitted before it is admitted whole (arrival order);
//  * a launch is either one chunk with a launch sequence of its own or a ragged batch of
//    chunks, which stops taking chunks once its estimated device time reaches a target;
//  * in continuous mode every chunk is cut to about a target device time (in whole
//    units of the request's granularity): a chunk with its own launch to the own-chunk
//    target, a chunk of a ragged batch to the launch target, so that one large request
//    spreads over several launches and no launch holds the requests admitted with it for
//    much longer than the target;
//  * while other launches are in flight (memory about to be released), a small piece is
//    not split off a request.
#pragma once

#include <algorithm>
#include <cstddef>
#include <cstdint>
#include <deque>
#include <vector>

namespace ldpcx {
namespace admit {

// A waiting request as the policy sees it.
struct Req {
    int batch = 0;    // codewords of the request
    int next_cw = 0;  // first codeword not yet admitted
    virtual ~Req() = default;
    // Whether the remaining codewords take a launch sequence of their own rather than
    // joining a ragged launch (in continuous mode; per-request mode gives every chunk one).
    virtual bool own() const = 0;
    // Codeword granularity of an own chunk's cut.
    virtual int unit() const = 0;
    // Device bytes a chunk of n codewords holds while in flight (non-decreasing in n).
    virtual size_t bytes(int n) const = 0;
    // Estimated device time of a chunk of n codewords, microseconds.
    virtual double us(int n) const = 0;
};

struct Config {
    bool continuous = true;   // false: one request's chunk per launch, in arrival order
    int max_launch_cw = 0;    // codewords per launch at most (0: no limit)
    size_t budget = 0;        // device bytes of all launches in flight together
    double launch_target_us = 1500.0;
    double own_chunk_target_us = 4000.0;
};

// One admitted chunk: codewords [cw0, cw0 + ncw) of request `id`.
struct Take {
    uint64_t id = 0;
    int cw0 = 0, ncw = 0;
    size_t charge = 0;  // budget bytes
    bool own = false;   // runs as a launch of its own
};

// Largest n in [0, cap] with r.bytes(n) <= avail.
inline int max_fit(const Req &r, int cap, size_t avail) {
    if (cap <= 0 || r.bytes(1) > avail) return 0;
    int lo = 1, hi = cap;
    while (lo < hi) {
        const int mid = lo + (hi - lo + 1) / 2;
        if (r.bytes(mid) <= avail) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Chunks of the next launch, taken from the front of `queue` (fully admitted requests
// leave it; partly admitted ones advance their next_cw).  `lookup(id)` returns the
// request of a queued id; `in_use` is the budget held by launches in flight.
template <class Lookup>
std::vector<Take> form(std::deque<uint64_t> &queue, Lookup &&lookup, const Config &cfg, size_t in_use,
                       bool others_in_flight) {
    std::vector<Take> take;
    size_t charge = 0;
    int cw_total = 0;
    double us = 0;
    while (!queue.empty()) {
        const uint64_t id = queue.front();
        Req &r = lookup(id);
        const bool own = !cfg.continuous || r.own();
        if (own && !take.empty()) break;
        if (!take.empty() && us >= cfg.launch_target_us) break;
        const int rem = r.batch - r.next_cw;
        int cap = rem;
        if (cfg.max_launch_cw > 0) cap = std::min(cap, cfg.max_launch_cw - cw_total);
        if (cfg.continuous) {
            const double per_cw = r.us(1024) / 1024.0;
            const double target = own ? cfg.own_chunk_target_us : cfg.launch_target_us;
            const double lim_d = target / std::max(per_cw, 1e-3);
            if (lim_d < (double)rem) {  // the target cuts the remainder: whole units, at least one
                const int unit = std::max(1, r.unit());
                cap = std::min(cap, std::max(unit, (int)lim_d / unit * unit));
            }
        }
        if (cap <= 0) break;
        if (in_use + charge > cfg.budget) break;
        const int n = max_fit(r, cap, cfg.budget - in_use - charge);
        if (n == 0) break;
        // Do not split off a small piece while memory is about to be released.
        if (n < rem && n < 64 && n < cap && (others_in_flight || !take.empty())) break;
        Take t;
        t.id = id;
        t.cw0 = r.next_cw;
        t.ncw = n;
        t.charge = r.bytes(n);
        t.own = own;
        take.push_back(t);
        us += r.us(n);
        r.next_cw += n;
        charge += t.charge;
        cw_total += n;
        if (r.next_cw < r.batch) break;  // arrival order: nothing passes a partly admitted request
        queue.pop_front();
        if (own) break;
    }
    return take;
}

}  // namespace admit
}  // namespace ldpcx
