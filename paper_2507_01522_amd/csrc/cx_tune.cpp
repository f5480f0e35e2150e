// cx_tune.cpp -- autotuner of the packing: lanes per station for every class
// and waves per block for the whole launch, timed on the real context.
#include <hip/hip_runtime.h>

#include <cctype>
#include <cstdio>
#include <fstream>
#include <map>
#include <sstream>
#include <string>
#include <vector>

#include "cx_ctx.h"

namespace cx {
namespace {

#ifndef CX_AUTOTUNE_ON
#define CX_AUTOTUNE_ON 0
#endif
constexpr bool kAutotuneEnabled = CX_AUTOTUNE_ON != 0;

std::map<std::string, int> read_cache(const char *path) {
  std::map<std::string, int> m;
  if (!path) return m;
  std::ifstream f(path);
  if (!f) return m;
  std::stringstream ss;
  ss << f.rdbuf();
  const std::string s = ss.str();
  size_t i = 0;
  while ((i = s.find('"', i)) != std::string::npos) {
    const size_t j = s.find('"', i + 1);
    if (j == std::string::npos) break;
    const std::string key = s.substr(i + 1, j - i - 1);
    size_t k = s.find(':', j);
    if (k == std::string::npos) break;
    ++k;
    while (k < s.size() && std::isspace((unsigned char)s[k])) ++k;
    size_t e = k;
    while (e < s.size() && (std::isdigit((unsigned char)s[e]) || s[e] == '-')) ++e;
    if (e > k) m[key] = std::atoi(s.substr(k, e - k).c_str());
    i = e > k ? e : j + 1;
  }
  return m;
}

void write_cache(const char *path, const std::map<std::string, int> &m) {
  if (!path) return;
  std::ofstream f(path);
  f << "{\n";
  size_t n = 0;
  for (const auto &kv : m) f << "  \"" << kv.first << "\": " << kv.second << (++n < m.size() ? ",\n" : "\n");
  f << "}\n";
}

std::string class_key(const ClassRt &c) {
  char b[160];
  long long bucket = 1;
  while (bucket < c.n_envs) bucket <<= 1;
  std::snprintf(b, sizeof b, "lanes:S%d:D%d:N%d:E%lld", c.comp.S, c.comp.D, c.comp.N, bucket);
  return b;
}

std::string ctx_key(const cx_ctx *ctx) {
  std::string k = "wpb";
  for (const auto &c : ctx->classes) {
    char b[64];
    std::snprintf(b, sizeof b, ":%d.%d", c.comp.S, c.lanes);
    k += b;
  }
  long long bucket = 1;
  while (bucket < ctx->n_envs) bucket <<= 1;
  return k + ":E" + std::to_string(bucket);
}

}  // namespace
}  // namespace cx

using namespace cx;

extern "C" cx_status cx_autotune(cx_ctx *ctx, int32_t T_probe, const char *cache_path) {
  if (!ctx) return fail_status(CX_E_INVALID, "context is NULL");
  if (ctx->failed) return fail_status(CX_E_DEVICE, "context has a sticky device error");
  if (T_probe < 1 || T_probe > 4096) return fail_status(CX_E_INVALID, "T_probe must be in 1..4096");
  // Switched off: one call aborted the process inside the tuner without any
  // diagnostic and the cause is not known yet.  The search below stays for
  // when it is found; until then packings, block size and the stage are set
  // with cx_set_packing and cx_set_obs_stage.
  if (!kAutotuneEnabled)
    return fail_status(CX_E_INVALID,
                       "cx_autotune is switched off (an unexplained abort inside it is under investigation); "
                       "set the packing with cx_set_packing and cx_set_obs_stage");
  std::map<std::string, int> cache = read_cache(cache_path);
  hipError_t e;
  void *saved = nullptr, *scratch = nullptr;
  SegDev *seg1 = nullptr;
  std::vector<SegDev> one_segs;
  std::vector<LaunchGroup> one_groups;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  const size_t obs_b = sizeof(float) * (size_t)T_probe * ctx->obs_elems;
  const size_t act_b = (size_t)T_probe * ctx->total_ports;
  const size_t env_b = (size_t)T_probe * ctx->n_envs;
  const uint32_t g_saved = ctx->g;
  const int32_t t_saved = ctx->t_day;
  cx_status st = CX_OK;
  RolloutGraph *probe_ptr = nullptr;
  auto cleanup = [&]() {
    if (probe_ptr) graph_destroy(*probe_ptr);
    if (saved) {
      (void)hipMemcpyAsync(ctx->state_mem, saved, ctx->state_bytes_dev, hipMemcpyDeviceToDevice, ctx->stream);
      (void)hipStreamSynchronize(ctx->stream);
      (void)hipFree(saved);
    }
    if (scratch) (void)hipFree(scratch);
    if (seg1) (void)hipFree(seg1);
    if (ev0) (void)hipEventDestroy(ev0);
    if (ev1) (void)hipEventDestroy(ev1);
    ctx->g = g_saved;
    ctx->t_day = t_saved;
  };
  if (hipMalloc(&saved, ctx->state_bytes_dev) != hipSuccess ||
      hipMalloc(&scratch, obs_b + act_b + sizeof(float) * env_b + env_b + 1024) != hipSuccess ||
      hipMalloc(&seg1, sizeof(SegDev)) != hipSuccess) {
    cleanup();
    return fail_status(CX_E_OOM, "cx_autotune: scratch allocation failed");
  }
  if ((e = hipMemcpyAsync(saved, ctx->state_mem, ctx->state_bytes_dev, hipMemcpyDeviceToDevice, ctx->stream)) !=
          hipSuccess ||
      (e = hipEventCreate(&ev0)) != hipSuccess || (e = hipEventCreate(&ev1)) != hipSuccess) {
    cleanup();
    return hip_fail(ctx, e, "cx_autotune setup");
  }
  unsigned char *sb = static_cast<unsigned char *>(scratch);
  LaunchArgs a = base_args(ctx);
  a.T = T_probe;
  a.mode = CX_ACT_RANDOM;
  a.out_mode = CX_OUT_FULL;
  a.obs = reinterpret_cast<float *>(sb);
  a.act = sb + obs_b;
  a.reward = reinterpret_cast<float *>(sb + ((obs_b + act_b + 255) & ~(size_t)255));
  a.done = sb + ((obs_b + act_b + 255) & ~(size_t)255) + sizeof(float) * env_b;
  // time a launch of the given segment table as rollouts run it (one graph,
  // its kernels concurrent); min over 3 after a warm-up
  RolloutGraph probe;
  probe_ptr = &probe;
  auto time_launch = [&](const SegDev *segs, const std::vector<LaunchGroup> &groups, float *best_ms) -> hipError_t {
    LaunchArgs b = a;
    b.segs = segs;
    float best = 1e30f;
    for (int rep = 0; rep < 4; ++rep) {
      hipError_t r;
      if ((r = hipEventRecord(ev0, ctx->stream)) != hipSuccess) return r;
      if ((r = graph_rollout(probe, b, groups.data(), (int)groups.size(), ctx->stream)) != hipSuccess)
        return r;
      if ((r = hipEventRecord(ev1, ctx->stream)) != hipSuccess) return r;
      if ((r = hipEventSynchronize(ev1)) != hipSuccess) return r;
      float ms = 0.f;
      if ((r = hipEventElapsedTime(&ms, ev0, ev1)) != hipSuccess) return r;
      if (rep > 0 && ms < best) best = ms;
    }
    *best_ms = best;
    return hipSuccess;
  };
  for (size_t ci = 0; ci < ctx->classes.size() && st == CX_OK; ++ci) {
    ClassRt &c = ctx->classes[ci];
    if (c.n_envs == 0) continue;
    const std::string key = class_key(c);
    auto it = cache.find(key);
    if (it != cache.end() && legal_packing(c.comp.S, it->second)) {
      c.lanes = it->second;
      continue;
    }
    int best_l = c.lanes;
    float best_ms = 1e30f;
    for (int L = 4; L <= 64; L <<= 1) {
      if (!legal_packing(c.comp.S, L)) continue;
      c.lanes = L;
      if ((st = rebuild_segments(ctx)) != CX_OK) break;
      SegDev one{};
      for (const SegDev &sg : ctx->segs_host)
        if (sg.cls == c.dev && one.cls == nullptr) one = sg;   // the class's first (largest) segment
      build_groups({one}, {c.tab.dwell_log2}, {c.host_view.kind}, ctx->wpb, &one_segs, &one_groups);
      if ((e = hipMemcpy(seg1, one_segs.data(), sizeof(SegDev), hipMemcpyHostToDevice)) != hipSuccess) {
        st = hip_fail(ctx, e, "cx_autotune segment upload");
        break;
      }
      float ms = 0.f;
      if ((e = time_launch(seg1, one_groups, &ms)) != hipSuccess) {
        st = hip_fail(ctx, e, "cx_autotune timing");
        break;
      }
      if (ms < best_ms) {
        best_ms = ms;
        best_l = L;
      }
    }
    c.lanes = best_l;
    cache[key] = best_l;
  }
  if (st == CX_OK) {
    // waves per block and the observation stage, chosen together (the stage
    // pays where the record stream, not the arithmetic, sets the pace, and
    // what it costs depends on the block size): every pair is timed
    bool any = false;
    for (const ClassRt &c : ctx->classes)
      any = any || (c.n_envs > 0 && c.host_view.kind == kKindSimple);
    const std::string wkey = ctx_key(ctx);
    const std::string skey = "stage" + wkey.substr(3);
    auto wit = cache.find(wkey);
    auto sit = cache.find(skey);
    const bool w_cached = wit != cache.end() && wit->second >= 1 && wit->second <= kMaxWaves;
    const bool s_cached = !any || (sit != cache.end() && (sit->second == 0 || sit->second == 1));
    if (w_cached && s_cached) {
      ctx->wpb = wit->second;
      ctx->stage_obs = any && sit->second != 0;
    } else {
      int best_w = ctx->wpb, best_s = 0;
      float best_ms = 1e30f;
      for (int w : {1, 2, 4, 8}) {
        for (int s = 0; s <= (any ? 1 : 0) && st == CX_OK; ++s) {
          ctx->wpb = w;
          ctx->stage_obs = s != 0;
          if ((st = rebuild_segments(ctx)) != CX_OK) break;
          float ms = 0.f;
          if ((e = time_launch(ctx->segs_dev, ctx->groups, &ms)) != hipSuccess) {
            st = hip_fail(ctx, e, "cx_autotune timing");
            break;
          }
          if (ms < best_ms) {
            best_ms = ms;
            best_w = w;
            best_s = s;
          }
        }
        if (st != CX_OK) break;
      }
      ctx->wpb = best_w;
      ctx->stage_obs = best_s != 0;
      cache[wkey] = best_w;
      if (any) cache[skey] = best_s;
    }
  }
  if (st == CX_OK) st = rebuild_segments(ctx);
  cleanup();
  if (st == CX_OK) write_cache(cache_path, cache);
  return st;
}
