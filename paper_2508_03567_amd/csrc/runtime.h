// Host-side structures shared by the runtime, the ragged engine, the autotuner
// and the server.
#pragma once

#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "ldpcx_internal.h"

namespace ldpcx {

enum { FAMILY_BIN_LDS = 0, FAMILY_BIN_IL = 1, FAMILY_NB = 2, FAMILY_BIN_QC = 3, FAMILY_SPA = 4, FAMILY_NB_LDS = 5, FAMILY_SPA_LDS = 6,
       FAMILY_NB1 = 7 };

struct Plan {
    int family = FAMILY_BIN_LDS;
    int schedule = LDPCX_SCHED_FLOODING;
    int cpw = 1;
    int threads = 256;
};

struct DeviceInfo {
    int cus = 256;
    int lds_per_block = 64 * 1024;
};

// A captured launch sequence of the interleaved decoders, keyed by everything that is
// baked into its kernel arguments.
struct GraphKey {
    int family, schedule, cpw, threads, batch;
    ldpcx_decode_params params;
    const void *llr;
    void *hard;
    uint8_t *ok;
    int16_t *iters;
};

struct GraphEntry {
    GraphKey key;
    hipGraphExec_t exec = nullptr;
    hipEvent_t done = nullptr;
    void *ws = nullptr;
    uint64_t last_use = 0;
};

}  // namespace ldpcx

struct ldpcx_code {
    ldpcx_code_desc desc{};
    int g = 2;
    int device = 0;
    bool layers_ok = false;
    bool nb_unsupported = false;
    bool qc_ok = false;
    ldpcx::QcDesc qc{};
    std::vector<int> row_ptr, col_idx, vn_ptr, vn_ref, vn_edge;
    std::vector<uint8_t> h, hinv, gfmul;
    void *dmem = nullptr;
    ldpcx::DevCode dev{};
    std::mutex mu;
    std::map<uint64_t, ldpcx::Plan> tuned;
    uint64_t hash = 0;  // of the code description (persisted tuning results are keyed by it)
    std::mutex graph_mu;
    std::vector<ldpcx::GraphEntry> graphs;
    uint64_t graph_clock = 0;
};

namespace ldpcx {

extern thread_local std::string g_err;
ldpcx_status fail(ldpcx_status st, const std::string &msg);
ldpcx_status fail_hip(hipError_t e, const char *what);
const DeviceInfo &device_info(int dev);
ldpcx_status check_params(const ldpcx_code *c, const ldpcx_decode_params *p);
ldpcx_status check_device(const ldpcx_code *c);
BinRule bin_rule(const ldpcx_decode_params *p);
// QC flooding with the layers in parallel (a workgroup of Z * npairs * nl threads; plans
// mark it by that thread count): whether a shape allows it, and its launch.
bool bin_qc_lp_ok(const QcDesc &Q, int npairs);
hipError_t launch_bin_qc_lp(const QcDesc &Q, const DevCode &C, const BinRule &R, int max_iters, int early_stop,
                            int batch, int npairs, const DecodeIO &io, hipStream_t s);
int nb_amax(const ldpcx_decode_params *p);  // Min-Max message bound of the params
// Whether the ragged decode runs this Min-Max job's codewords as one-codeword items of
// its persistent kernel (any schedule) rather than as a whole-device decode
bool ragged_nb1_items(const ldpcx_code *c, const ldpcx_decode_params *p);
Plan default_plan(const ldpcx_code *c, const ldpcx_decode_params *p, int batch);
Plan plan_for(ldpcx_code *c, const ldpcx_decode_params *p, int batch);
uint64_t tune_key(const ldpcx_decode_params *p, int batch);
// Device workspace of a decode with an interleaved or wave-level family (0 otherwise).
size_t work_bytes(const ldpcx_code *c, const ldpcx_decode_params *p, const Plan &pl, int batch);
// allow_graph = false always enqueues the launch sequence itself (no cached graph keyed
// by the I/O buffers), for callers whose buffers change from call to call.
ldpcx_status run_plan(ldpcx_code *c, const ldpcx_decode_params *p, const Plan &pl, int batch, const DecodeIO &io,
                      hipStream_t s, bool allow_graph = true);
hipError_t enqueue_interleaved(ldpcx_code *c, const ldpcx_decode_params *p, const Plan &pl, int batch, void *ws,
                               const DecodeIO &io, int8_t *dump_scratch, hipStream_t s);
bool graphs_enabled();
ldpcx_status run_graph(ldpcx_code *c, const ldpcx_decode_params *p, const Plan &pl, int batch, const DecodeIO &io,
                       hipStream_t s);
void release_graph(GraphEntry &g);
// Copy `bytes` of host memory to device memory `dst` in the order of stream `s` without
// blocking the host: the data goes through a pinned staging buffer that is reused once
// the copy has completed.
ldpcx_status upload_async(void *dst, const void *src, size_t bytes, int device, hipStream_t s);
// Persisted autotuning (file named by LDPCX_TUNE_CACHE; nothing happens when it is unset):
// load the entries of this code and device into c->tuned, and merge one tuned plan in.
void tune_cache_load(ldpcx_code *c);
void tune_cache_store(const ldpcx_code *c, uint64_t key, const Plan &pl, float us);
uint64_t code_hash(const ldpcx_code_desc *d);

}  // namespace ldpcx
