// cx_server.cpp -- serving: continuous batching of rollout requests.
#include <hip/hip_runtime.h>

#include "cx_ctx.h"

using namespace cx;

extern "C" {
cx_status cx_server_create(size_t, const cx_server_opts *, cx_server **out) {
  if (out) *out = nullptr;
  return fail_status(CX_E_INVALID, "serving not available in this build");
}
cx_status cx_submit(cx_server *, const cx_request *, uint64_t *) { return fail_status(CX_E_INVALID, "no server"); }
cx_status cx_poll(cx_server *, uint64_t, cx_result *) { return fail_status(CX_E_INVALID, "no server"); }
cx_status cx_wait(cx_server *, uint64_t, cx_result *) { return fail_status(CX_E_INVALID, "no server"); }
cx_status cx_cancel(cx_server *, uint64_t) { return fail_status(CX_E_INVALID, "no server"); }
cx_status cx_release(cx_server *, uint64_t) { return fail_status(CX_E_INVALID, "no server"); }
cx_status cx_server_stats(cx_server *, double *, int64_t *, int64_t *) { return fail_status(CX_E_INVALID, "no server"); }
void cx_server_destroy(cx_server *) {}
}
