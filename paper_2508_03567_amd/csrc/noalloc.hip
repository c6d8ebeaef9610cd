// Allocation-free decode: the same decoders as ldpcx_decode, with every workspace
// taken from one static device array per GPU instead of the stream-ordered allocator.
//
// The array lives in this file's device code object, so each GPU that loads the library
// holds its own copy until the process ends.  In host code its name is only a stand-in:
// the device address of a GPU's copy comes from hipGetSymbolAddress, called once per
// device on the first call made with that device current, and only that address is
// ever passed to kernels.  The batch runs as consecutive chunks on the caller's stream,
// each chunk's workspace fitting the array, so chunks reuse it in stream order.  Every
// decoder initialises the workspace it reads, so what an earlier call left there never
// reaches a result.
#include <algorithm>
#include <map>
#include <mutex>

#include "runtime.h"

namespace ldpcx {

namespace {

constexpr size_t kScratchBytes = LDPCX_NOALLOC_SCRATCH_BYTES;

static __device__ __align__(256) char scratch[kScratchBytes];

std::mutex g_scratch_mu;
std::map<int, void *> g_scratch_ptr;  // device -> address of that device's copy

// Device address of the current device's array (looked up once per device).
ldpcx_status scratch_of(int device, void **out) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    auto it = g_scratch_ptr.find(device);
    if (it != g_scratch_ptr.end()) {
        *out = it->second;
        return LDPCX_OK;
    }
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return fail_hip(e != hipSuccess ? e : hipErrorInvalidSymbol, "static scratch address");
    g_scratch_ptr[device] = p;
    *out = p;
    return LDPCX_OK;
}

// I/O of codewords [b0, b0 + nb) of a decode.
DecodeIO io_slice(const ldpcx_code *c, const DecodeIO &io, int b0) {
    const size_t n = c->dev.n, g = c->g;
    const size_t in_cw = g == 2 ? n : n * g * 2, out_cw = g == 2 ? (n + 7) / 8 : n;
    DecodeIO sl = io;
    sl.llr = (const char *)io.llr + (size_t)b0 * in_cw;
    sl.hard = (char *)io.hard + (size_t)b0 * out_cw;
    sl.ok = io.ok + b0;
    sl.iters = io.iters + b0;
    return sl;
}

}  // namespace

}  // namespace ldpcx

using namespace ldpcx;

extern "C" ldpcx_status ldpcx_decode_noalloc(const ldpcx_code *code, const ldpcx_decode_params *params, int32_t batch,
                                             const void *llr, void *hard, uint8_t *syndrome_ok, int16_t *iters,
                                             int32_t *schedule_used, void *stream) {
    try {
        if (!code) return fail(LDPCX_E_INVAL, "code is NULL");
        ldpcx_code *c = const_cast<ldpcx_code *>(code);
        if (c->nb_unsupported) return fail(LDPCX_E_UNSUPPORTED, "no Min-Max kernel for this field size");
        ldpcx_status st = check_params(c, params);
        if (st != LDPCX_OK) return st;
        if (batch < 0) return fail(LDPCX_E_INVAL, "batch < 0");
        if (batch == 0) return LDPCX_OK;
        if (!llr || !hard || !syndrome_ok || !iters) return fail(LDPCX_E_INVAL, "null buffer");
        if ((st = check_device(c)) != LDPCX_OK) return st;
        hipStream_t s = (hipStream_t)stream;
        Plan pl = plan_for(c, params, batch);
        if (schedule_used) *schedule_used = pl.schedule;
        const DecodeIO io{llr, hard, syndrome_ok, iters, nullptr, nullptr, nullptr};
        // Families whose state stays on chip need no workspace: the plain launch allocates nothing.
        if (pl.family == FAMILY_BIN_QC || pl.family == FAMILY_BIN_LDS || pl.family == FAMILY_SPA_LDS ||
            pl.family == FAMILY_NB1)
            return run_plan(c, params, pl, batch, io, s, false);
        void *ws = nullptr;
        if ((st = scratch_of(c->device, &ws)) != LDPCX_OK) return st;
        const char *too_big = "the workspace of the smallest slice exceeds the static scratch of the allocation-free decode";
        int chunk = batch;
        if (pl.family == FAMILY_BIN_IL) {
            // Slices of `sub` codewords reuse one workspace: shrink the slice until it fits.
            int sub = pl.cpw;
            while (bin_il_work_bytes(c->dev, params->max_iters, sub, sub) > kScratchBytes) {
                const int smaller = bin_il_sub_batch(c->dev, sub, sub / 2);
                if (smaller >= sub) return fail(LDPCX_E_UNSUPPORTED, too_big);
                sub = smaller;
            }
            pl.cpw = sub;
        } else {
            while (work_bytes(c, params, pl, chunk) > kScratchBytes) {
                if (chunk <= 1) return fail(LDPCX_E_UNSUPPORTED, too_big);
                chunk = chunk > 128 ? (chunk / 2 + 63) / 64 * 64 : chunk / 2;
            }
        }
        for (int b0 = 0; b0 < batch; b0 += chunk) {
            const int nb = std::min(chunk, batch - b0);
            const hipError_t e = enqueue_interleaved(c, params, pl, nb, ws, io_slice(c, io, b0), nullptr, s);
            if (e != hipSuccess) return fail_hip(e, "decoder launch");
        }
        return LDPCX_OK;
    } catch (const std::exception &ex) {
        return fail(LDPCX_E_NOMEM, ex.what());
    }
}
