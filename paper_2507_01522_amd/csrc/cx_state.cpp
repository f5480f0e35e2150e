// cx_state.cpp -- packing-independent snapshots of a context's state.
#include <hip/hip_runtime.h>

#include <cstring>
#include <vector>

#include "cx_ctx.h"

namespace cx {

static const uint64_t kMagic = 0x33305843ull;  // "CX03"
static const size_t kHeader = 8 + 8 + 8 + 4 + 4;
static const size_t kPortRec = 4 + 8 + 4 + 4 + 4 + 1 + 4;
static const size_t kBattRec = 8 + 4;

static size_t battery_envs(const cx_ctx *ctx) {
  size_t n = 0;
  for (const ClassRt &c : ctx->classes)
    if (c.comp.battery) n += (size_t)c.n_envs;
  return n;
}

size_t state_blob_bytes(const cx_ctx *ctx) {
  return kHeader + kPortRec * (size_t)ctx->port_count + 8 * (size_t)ctx->n_envs + kBattRec * battery_envs(ctx);
}

}  // namespace cx

using namespace cx;

extern "C" {

cx_status cx_get_state(cx_ctx *ctx, void *host, size_t bytes) {
  if (!ctx || !host) return fail_status(CX_E_INVALID, "NULL argument");
  if (ctx->failed) return fail_status(CX_E_DEVICE, "context has a sticky device error");
  if (bytes < state_blob_bytes(ctx)) return fail_status(CX_E_INVALID, "buffer smaller than cx_info.state_bytes");
  hipError_t e = hipStreamSynchronize(ctx->stream);
  if (e != hipSuccess) return hip_fail(ctx, e, "cx_get_state synchronize");
  const size_t ns = (size_t)ctx->total_slots;
  std::vector<double> qv(ns);
  std::vector<float> uv(ns), cap(ns), pl(ns);
  std::vector<int16_t> dw(ns);
  std::vector<uint8_t> ut(ns);
  std::vector<float> rb(ns);
  std::vector<double> ret((size_t)ctx->n_envs), bsoc((size_t)ctx->n_envs);
  std::vector<float> bp((size_t)ctx->n_envs);
  if ((e = hipMemcpy(qv.data(), ctx->q, 8 * ns, hipMemcpyDeviceToHost)) != hipSuccess ||
      (e = hipMemcpy(bsoc.data(), ctx->bsoc, 8 * bsoc.size(), hipMemcpyDeviceToHost)) != hipSuccess ||
      (e = hipMemcpy(bp.data(), ctx->bp, 4 * bp.size(), hipMemcpyDeviceToHost)) != hipSuccess ||
      (e = hipMemcpy(uv.data(), ctx->u, 4 * ns, hipMemcpyDeviceToHost)) != hipSuccess ||
      (e = hipMemcpy(cap.data(), ctx->cap, 4 * ns, hipMemcpyDeviceToHost)) != hipSuccess ||
      (e = hipMemcpy(pl.data(), ctx->p_last, 4 * ns, hipMemcpyDeviceToHost)) != hipSuccess ||
      (e = hipMemcpy(dw.data(), ctx->dwell, 2 * ns, hipMemcpyDeviceToHost)) != hipSuccess ||
      (e = hipMemcpy(ut.data(), ctx->utype, ns, hipMemcpyDeviceToHost)) != hipSuccess ||
      (e = hipMemcpy(rb.data(), ctx->rbar, 4 * ns, hipMemcpyDeviceToHost)) != hipSuccess ||
      (e = hipMemcpy(ret.data(), ctx->ret, 8 * ret.size(), hipMemcpyDeviceToHost)) != hipSuccess)
    return hip_fail(ctx, e, "cx_get_state copy");
  unsigned char *p = static_cast<unsigned char *>(host);
  const int64_t ne = ctx->n_envs, np = ctx->port_count;
  std::memcpy(p, &kMagic, 8);
  std::memcpy(p + 8, &ne, 8);
  std::memcpy(p + 16, &np, 8);
  std::memcpy(p + 24, &ctx->g, 4);
  std::memcpy(p + 28, &ctx->t_day, 4);
  unsigned char *q = p + kHeader;
  for (const ClassRt &c : ctx->classes) {
    for (int64_t e2 = 0; e2 < c.n_envs; ++e2) {
      for (int i = 0; i < c.comp.N; ++i) {
        const size_t x = (size_t)(c.slot_off + e2 * c.comp.S + c.comp.port_slot[i]);
        const int32_t d = dw[x];
        std::memcpy(q, &d, 4);
        std::memcpy(q + 4, &qv[x], 8);
        std::memcpy(q + 12, &uv[x], 4);
        std::memcpy(q + 16, &cap[x], 4);
        std::memcpy(q + 20, &pl[x], 4);
        q[24] = ut[x];
        std::memcpy(q + 25, &rb[x], 4);
        q += kPortRec;
      }
    }
  }
  std::memcpy(q, ret.data(), 8 * ret.size());
  q += 8 * ret.size();
  for (const ClassRt &c : ctx->classes) {
    if (!c.comp.battery) continue;
    for (int64_t e2 = 0; e2 < c.n_envs; ++e2) {
      std::memcpy(q, &bsoc[(size_t)(c.env_begin + e2)], 8);
      std::memcpy(q + 8, &bp[(size_t)(c.env_begin + e2)], 4);
      q += kBattRec;
    }
  }
  return CX_OK;
}

cx_status cx_set_state(cx_ctx *ctx, const void *host, size_t bytes) {
  if (!ctx || !host) return fail_status(CX_E_INVALID, "NULL argument");
  if (ctx->failed) return fail_status(CX_E_DEVICE, "context has a sticky device error");
  if (bytes < state_blob_bytes(ctx)) return fail_status(CX_E_INVALID, "buffer smaller than cx_info.state_bytes");
  const unsigned char *p = static_cast<const unsigned char *>(host);
  uint64_t magic;
  int64_t ne, np;
  uint32_t g;
  int32_t t_day;
  std::memcpy(&magic, p, 8);
  std::memcpy(&ne, p + 8, 8);
  std::memcpy(&np, p + 16, 8);
  std::memcpy(&g, p + 24, 4);
  std::memcpy(&t_day, p + 28, 4);
  if (magic != kMagic || ne != ctx->n_envs || np != ctx->port_count)
    return fail_status(CX_E_INVALID, "snapshot does not match this context");
  if (t_day < 0 || t_day >= ctx->steps_ep) return fail_status(CX_E_INVALID, "snapshot t_day out of range");
  const size_t ns = (size_t)ctx->total_slots;
  std::vector<double> qv(ns, 0.0);
  std::vector<float> uv(ns, 0.f), cap(ns, 0.f), pl(ns, 0.f);
  std::vector<int16_t> dw(ns, 0);
  std::vector<uint8_t> ut(ns, 0);
  std::vector<float> rb(ns, 0.f);
  std::vector<double> ret((size_t)ctx->n_envs);
  const unsigned char *q = p + kHeader;
  for (const ClassRt &c : ctx->classes) {
    for (int64_t e2 = 0; e2 < c.n_envs; ++e2) {
      for (int i = 0; i < c.comp.N; ++i) {
        const size_t x = (size_t)(c.slot_off + e2 * c.comp.S + c.comp.port_slot[i]);
        int32_t d;
        std::memcpy(&d, q, 4);
        const uint8_t user = q[24];
        if (user > 1 || (user == 1 && !c.comp.users))
          return fail_status(CX_E_INVALID, "snapshot user type invalid for this class");
        if (d > 32767 || d < (user ? -32767 : 0)) return fail_status(CX_E_INVALID, "snapshot dwell out of range");
        dw[x] = (int16_t)d;
        ut[x] = user;
        std::memcpy(&rb[x], q + 25, 4);
        if (!(rb[x] >= 0.f && rb[x] < 1e30f)) return fail_status(CX_E_INVALID, "snapshot car rate invalid");
        std::memcpy(&qv[x], q + 4, 8);
        std::memcpy(&uv[x], q + 12, 4);
        std::memcpy(&cap[x], q + 16, 4);
        std::memcpy(&pl[x], q + 20, 4);
        q += kPortRec;
      }
    }
  }
  std::memcpy(ret.data(), q, 8 * ret.size());
  q += 8 * ret.size();
  std::vector<double> bsoc((size_t)ctx->n_envs, 0.0);
  std::vector<float> bp((size_t)ctx->n_envs, 0.f);
  for (const ClassRt &c : ctx->classes) {
    if (!c.comp.battery) continue;
    for (int64_t e2 = 0; e2 < c.n_envs; ++e2) {
      double v;
      std::memcpy(&v, q, 8);
      if (!(v >= 0.0 && v <= 1.0)) return fail_status(CX_E_INVALID, "snapshot battery SoC out of [0,1]");
      bsoc[(size_t)(c.env_begin + e2)] = v;
      std::memcpy(&bp[(size_t)(c.env_begin + e2)], q + 8, 4);
      q += kBattRec;
    }
  }
  hipError_t e = hipStreamSynchronize(ctx->stream);
  if (e != hipSuccess) return hip_fail(ctx, e, "cx_set_state synchronize");
  if ((e = hipMemcpy(ctx->q, qv.data(), 8 * ns, hipMemcpyHostToDevice)) != hipSuccess ||
      (e = hipMemcpy(ctx->u, uv.data(), 4 * ns, hipMemcpyHostToDevice)) != hipSuccess ||
      (e = hipMemcpy(ctx->cap, cap.data(), 4 * ns, hipMemcpyHostToDevice)) != hipSuccess ||
      (e = hipMemcpy(ctx->p_last, pl.data(), 4 * ns, hipMemcpyHostToDevice)) != hipSuccess ||
      (e = hipMemcpy(ctx->dwell, dw.data(), 2 * ns, hipMemcpyHostToDevice)) != hipSuccess ||
      (e = hipMemcpy(ctx->utype, ut.data(), ns, hipMemcpyHostToDevice)) != hipSuccess ||
      (e = hipMemcpy(ctx->rbar, rb.data(), 4 * ns, hipMemcpyHostToDevice)) != hipSuccess ||
      (e = hipMemcpy(ctx->ret, ret.data(), 8 * ret.size(), hipMemcpyHostToDevice)) != hipSuccess ||
      (e = hipMemcpy(ctx->bsoc, bsoc.data(), 8 * bsoc.size(), hipMemcpyHostToDevice)) != hipSuccess ||
      (e = hipMemcpy(ctx->bp, bp.data(), 4 * bp.size(), hipMemcpyHostToDevice)) != hipSuccess)
    return hip_fail(ctx, e, "cx_set_state copy");
  ctx->g = g;
  ctx->t_day = t_day;
  return CX_OK;
}

}  // extern "C"
