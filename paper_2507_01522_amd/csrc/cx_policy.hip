// cx_policy.hip -- policy-in-the-loop rollouts (MLP on the matrix cores).
#include <hip/hip_runtime.h>

#include "cx_ctx.h"

namespace cx {

void free_policy(cx_ctx *ctx) { (void)ctx; }

cx_status policy_step(cx_ctx *ctx, int32_t T, cx_out_mode out_mode, const cx_traj *out, bool graph) {
  (void)ctx; (void)T; (void)out_mode; (void)out; (void)graph;
  return fail_status(CX_E_INVALID, "no policy set (cx_set_policy)");
}

}  // namespace cx

using namespace cx;

extern "C" {

cx_status cx_set_policy(cx_ctx *ctx, int32_t hidden, const uint16_t *w1, const uint16_t *b1,
                        const uint16_t *w2, const uint16_t *b2) {
  (void)ctx; (void)hidden; (void)w1; (void)b1; (void)w2; (void)b2;
  return fail_status(CX_E_INVALID, "cx_set_policy: not available in this build");
}

cx_status cx_policy_logits(cx_ctx *ctx, const float *obs_dev, int64_t n, float *logits_dev) {
  (void)ctx; (void)obs_dev; (void)n; (void)logits_dev;
  return fail_status(CX_E_INVALID, "no policy set (cx_set_policy)");
}

}  // extern "C"
