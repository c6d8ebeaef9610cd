// Continuous-batching server (placeholder).
#include "runtime.h"
using namespace ldpcx;
extern "C" {
ldpcx_status ldpcx_server_create(size_t, int32_t, ldpcx_server **) { return fail(LDPCX_E_UNSUPPORTED, "server not built yet"); }
ldpcx_status ldpcx_server_submit(ldpcx_server *, const ldpcx_code *, const ldpcx_decode_params *, int32_t, const void *, void *, uint8_t *, int16_t *, uint64_t *) { return LDPCX_E_UNSUPPORTED; }
ldpcx_status ldpcx_server_poll(ldpcx_server *, uint64_t, int32_t *) { return LDPCX_E_UNSUPPORTED; }
ldpcx_status ldpcx_server_wait(ldpcx_server *, uint64_t, int32_t, double *, double *, double *) { return LDPCX_E_UNSUPPORTED; }
ldpcx_status ldpcx_server_cancel(ldpcx_server *, uint64_t) { return LDPCX_E_UNSUPPORTED; }
ldpcx_status ldpcx_server_stats(ldpcx_server *, uint64_t *, uint64_t *, uint64_t *, uint64_t *) { return LDPCX_E_UNSUPPORTED; }
ldpcx_status ldpcx_server_destroy(ldpcx_server *) { return LDPCX_E_UNSUPPORTED; }
}
