// Ragged persistent engine (placeholder until the persistent kernel lands).
#include "runtime.h"
using namespace ldpcx;
extern "C" ldpcx_status ldpcx_decode_ragged(const ldpcx_job *, int32_t, void *) {
    return fail(LDPCX_E_UNSUPPORTED, "ragged engine not built yet");
}
