// cx_api.cpp -- contexts and the C ABI of include/cx.h (everything but serving
// and the policy kernels).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <limits>
#include <string>
#include <vector>

#include "cx_ctx.h"
#include "cx_layout.h"

namespace cx {

thread_local std::string g_last_error;

cx_status fail_status(cx_status st, const std::string &msg) {
  g_last_error = msg;
  return st;
}

cx_status hip_fail(cx_ctx *ctx, hipError_t e, const char *what) {
  if (ctx) ctx->failed = true;
  return fail_status(CX_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Host image of one class's device block: ClassDev, per-slot arrays and tables,
// with the struct's pointers resolved against dev_base.  Returns the block size;
// with host == nullptr only the size (and *view, if given) is produced.
size_t class_block(const SpecCopy &sc, const Compiled &k, const Tables &t, unsigned char *dev_base,
                   std::vector<unsigned char> *host, ClassDev *view) {
  const cx_station_spec &s = sc.s;
  size_t off = align256(sizeof(ClassDev));
  auto take = [&](size_t bytes) { size_t o = off; off = align256(off + bytes); return o; };
  const size_t o_port = take(sizeof(int32_t) * k.S);
  const size_t o_pmax = take(sizeof(float) * k.S);
  const size_t o_ipmax = take(sizeof(float) * k.S);
  const size_t o_ieta = take(sizeof(float) * k.S);
  const size_t o_lb = take(sizeof(uint32_t) * k.S);
  const size_t o_cap = take(sizeof(float) * k.S * k.D);
  const size_t o_tp = take(sizeof(uint32_t) * t.tpois_dev.size());
  const size_t o_td = take(sizeof(uint32_t) * t.tdwell_dev.size());
  const size_t o_gl = take(sizeof(float) * t.glob.size());
  const size_t o_pdis = take(sizeof(float) * k.S);
  const size_t o_eta = take(sizeof(float) * k.S);
  const size_t o_days = take(sizeof(float) * t.price_days.size());
  const size_t o_mth = take(sizeof(uint32_t) * 8);
  const size_t o_mdat = take(sizeof(float) * 24);
  const size_t o_sdc = take(sizeof(int32_t) * k.S);
  unsigned char *base = dev_base;
  ClassDev d{};
  d.n_ports = k.N; d.S = k.S; d.D = k.D; d.n_levels = s.n_levels;
  d.steps_ep = s.steps_per_episode; d.obs_dim = k.obs_dim; d.dwell_log2 = t.dwell_log2;
  d.uniform_eta = k.uniform_eta ? 1 : 0;
  d.dt = (float)s.dt_hours; d.inv_dt = (float)(1.0 / s.dt_hours); d.inv_1mtau = (float)(1.0 / (1.0 - s.tau));
  d.p_sell = (float)s.p_sell; d.p_sell_grid = (float)s.p_sell_grid; d.fixed_cost = (float)s.fixed_cost;
  d.alpha_sat = (float)s.alpha_sat; d.alpha_dec = (float)s.alpha_declined; d.price_sigma = (float)s.price_sigma;
  d.cap_lo = (float)s.cap_lo; d.cap_span = (float)(s.cap_hi - s.cap_lo);
  d.soc_lo = (float)s.soc0_lo; d.soc_span = (float)(s.soc0_hi - s.soc0_lo);
  d.tgt_lo = (float)s.tgt_lo; d.tgt_span = (float)(s.tgt_hi - s.tgt_lo);
  d.inv_steps_ep = (float)(1.0 / s.steps_per_episode); d.inv_n_levels = (float)(1.0 / s.n_levels);
  d.inv_eta_uniform = k.inv_eta_uniform;
  d.lvl_lb_uniform = 0;
  for (int lvl = 0; lvl < kMaxLevels; ++lvl) {
    uint32_t v = 0xFF;
    if (lvl < k.D) {
      v = (k.slot_lb[0] >> (8 * lvl)) & 0xFF;
      for (int x = 1; x < k.S; ++x)
        if (((k.slot_lb[x] >> (8 * lvl)) & 0xFF) != v) v = 0xFF;
    }
    d.lvl_lb_uniform |= v << (8 * lvl);
  }
  // SIMPLE: dense, one port maximum and efficiency, one block size and limit per level
  bool simple = k.S == k.N && k.uniform_eta;
  for (int x = 1; x < k.S && simple; ++x) simple = k.slot_pmax[x] == k.slot_pmax[0];
  for (int lvl = 0; lvl < kMaxLevels; ++lvl) {
    float cu = std::numeric_limits<float>::infinity();
    if (lvl < k.D) {
      if (((d.lvl_lb_uniform >> (8 * lvl)) & 0xFF) == 0xFF) simple = false;
      cu = k.slot_cap[(size_t)lvl * k.S];
      for (int x = 1; x < k.S; ++x)
        if (k.slot_cap[(size_t)lvl * k.S + x] != cu) simple = false;
    }
    d.lvl_cap_u[lvl] = cu;
  }
  for (int b = 0; b < kMaxBlockLog2; ++b) d.blk_cap[b] = std::numeric_limits<float>::infinity();
  d.blk_mask = 0;
  for (int lvl = 0; lvl + 1 < k.D; ++lvl) {   // levels below the root
    const uint32_t lb = (d.lvl_lb_uniform >> (8 * lvl)) & 0xFF;
    if (lb < (uint32_t)kMaxBlockLog2) {
      d.blk_cap[lb] = d.lvl_cap_u[lvl];
      d.blk_mask |= 1u << lb;
    }
  }
  d.kind = k.extended() ? kKindExt : simple ? kKindSimple : kKindGeneral;
  d.simple = d.kind == kKindSimple ? 1 : 0;
  d.n_neg = k.v2g ? s.n_levels : 0;
  d.has_batt = k.battery ? 1 : 0;
  d.n_act = k.n_act;
  d.alpha_db = (float)s.alpha_degrad_battery;
  d.alpha_dc = (float)s.alpha_degrad_cars;
  if (k.battery) {
    d.b_cap = s.battery_kwh; d.b_inv_cap = 1.0 / s.battery_kwh;
    d.b_rate = s.battery_kw; d.b_inv_1mtau = 1.0 / (1.0 - s.battery_tau);
    d.b_soc0 = s.battery_soc0; d.b_inv_rate = (float)(1.0 / s.battery_kw);
  }
  d.dt_d = s.dt_hours; d.inv_dt_d = 1.0 / s.dt_hours; d.inv_n_d = 1.0 / s.n_levels;
  d.has_users = k.users ? 1 : 0;
  d.cs_thresh = k.cs_thresh;
  d.user_obs = k.user_obs;
  d.alpha_sat1 = (float)s.alpha_sat1;
  d.beta_sat1 = (float)s.beta_sat1;
  d.n_days = k.n_days;
  d.day_obs = k.day_obs;
  d.inv_n_days = k.n_days > 0 ? (float)(1.0 / k.n_days) : 0.f;
  d.n_models = k.n_models;
  d.dense_nodes = k.dense_nodes;
  d.pmax_u = k.slot_pmax[0];
  d.inv_pmax_u = k.slot_inv_pmax[0];
  // device addresses of the arrays (none in the size-only pass)
  auto at = [base](size_t o) { return base ? base + o : nullptr; };
  d.slot_port = reinterpret_cast<const int32_t *>(at(o_port));
  d.slot_pmax = reinterpret_cast<const float *>(at(o_pmax));
  d.slot_inv_pmax = reinterpret_cast<const float *>(at(o_ipmax));
  d.slot_inv_eta = reinterpret_cast<const float *>(at(o_ieta));
  d.slot_lb = reinterpret_cast<const uint32_t *>(at(o_lb));
  d.slot_cap = reinterpret_cast<const float *>(at(o_cap));
  d.tpois = reinterpret_cast<const uint32_t *>(at(o_tp));
  d.tdwell = reinterpret_cast<const uint32_t *>(at(o_td));
  d.glob = reinterpret_cast<const float *>(at(o_gl));
  d.slot_pdis = reinterpret_cast<const float *>(at(o_pdis));
  d.slot_eta = reinterpret_cast<const float *>(at(o_eta));
  d.price_days = reinterpret_cast<const float *>(at(o_days));
  d.model_thresh = reinterpret_cast<const uint32_t *>(at(o_mth));
  d.model_data = reinterpret_cast<const float *>(at(o_mdat));
  d.slot_dc = reinterpret_cast<const int32_t *>(at(o_sdc));
  if (view) *view = d;
  if (host) {
    host->assign(off, 0);
    std::memcpy(host->data(), &d, sizeof d);
    std::memcpy(host->data() + o_port, k.slot_port.data(), sizeof(int32_t) * k.S);
    std::memcpy(host->data() + o_pmax, k.slot_pmax.data(), sizeof(float) * k.S);
    std::memcpy(host->data() + o_ipmax, k.slot_inv_pmax.data(), sizeof(float) * k.S);
    std::memcpy(host->data() + o_ieta, k.slot_inv_eta.data(), sizeof(float) * k.S);
    std::memcpy(host->data() + o_lb, k.slot_lb.data(), sizeof(uint32_t) * k.S);
    std::memcpy(host->data() + o_cap, k.slot_cap.data(), sizeof(float) * k.S * k.D);
    std::memcpy(host->data() + o_tp, t.tpois_dev.data(), sizeof(uint32_t) * t.tpois_dev.size());
    std::memcpy(host->data() + o_td, t.tdwell_dev.data(), sizeof(uint32_t) * t.tdwell_dev.size());
    std::memcpy(host->data() + o_gl, t.glob.data(), sizeof(float) * t.glob.size());
    std::memcpy(host->data() + o_pdis, k.slot_pdis.data(), sizeof(float) * k.S);
    std::memcpy(host->data() + o_eta, k.slot_eta.data(), sizeof(float) * k.S);
    if (!t.price_days.empty())
      std::memcpy(host->data() + o_days, t.price_days.data(), sizeof(float) * t.price_days.size());
    std::memcpy(host->data() + o_mth, k.model_thresh.data(), sizeof(uint32_t) * 8);
    std::memcpy(host->data() + o_mdat, k.model_data.data(), sizeof(float) * 24);
    std::memcpy(host->data() + o_sdc, k.slot_dc.data(), sizeof(int32_t) * k.S);
  }
  return off;
}

// Upload one class's constants, per-slot arrays and tables into one device block.
static cx_status upload_class(cx_ctx *ctx, ClassRt &c) {
  const size_t bytes = class_block(c.spec, c.comp, c.tab, nullptr, nullptr, nullptr);
  hipError_t e = hipMalloc(&c.dev_mem, bytes);
  if (e != hipSuccess) return fail_status(CX_E_OOM, "hipMalloc of class constants failed");
  ctx->device_bytes += (int64_t)bytes;
  std::vector<unsigned char> host;
  class_block(c.spec, c.comp, c.tab, static_cast<unsigned char *>(c.dev_mem), &host, &c.host_view);
  e = hipMemcpy(c.dev_mem, host.data(), bytes, hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_fail(ctx, e, "upload of class constants");
  c.dev = reinterpret_cast<ClassDev *>(c.dev_mem);
  return CX_OK;
}

bool legal_packing(int S, int lanes) {
  if (lanes < 4 || lanes > 64 || (lanes & (lanes - 1))) return false;
  if (S % lanes) return false;
  const int P = S / lanes;
  return P == 1 || P == 2 || P == 4;
}

int default_lanes(int S) { return S <= 64 ? S : 64; }

// Group segments by packing (one kernel each); groups with more slots per
// station come first so the heaviest waves start first.
void build_groups(const std::vector<SegDev> &in, const std::vector<int> &log2_dwell,
                  const std::vector<int> &kind, int wpb, std::vector<SegDev> *out,
                  std::vector<LaunchGroup> *groups) {
  out->clear();
  groups->clear();
  // launch kind = kNumKinds * packing + kernel kind
  std::vector<int> kinds;
  for (size_t i = 0; i < in.size(); ++i) {
    const int kd = kNumKinds * in[i].pack + kind[i];
    if (std::find(kinds.begin(), kinds.end(), kd) == kinds.end()) kinds.push_back(kd);
  }
  std::stable_sort(kinds.begin(), kinds.end(), [](int a, int b) {
    const int pa = a / kNumKinds, pb = b / kNumKinds;
    return pack_lanes(pa) * pack_per_lane(pa) > pack_lanes(pb) * pack_per_lane(pb);
  });
  for (int kd : kinds) {
    LaunchGroup g;
    g.pack = kd / kNumKinds;
    g.kind = kd % kNumKinds;
    g.seg_begin = (int)out->size();
    for (size_t i = 0; i < in.size(); ++i) {
      if (kNumKinds * in[i].pack + kind[i] != kd) continue;
      g.max_dwell_log2 = std::max(g.max_dwell_log2, log2_dwell[i]);
      g.max_T = std::max(g.max_T, in[i].T);
      g.max_obs_dim = std::max(g.max_obs_dim, in[i].obs_dim);
    }
    // fewer waves per block where the observation stages would not fit
    g.wpb = wpb;
    while (group_stages(g.kind, g.pack) && g.wpb > 1 &&
           group_lds_bytes(g.wpb, g.pack, g.max_obs_dim, g.max_dwell_log2, nullptr, nullptr) > kMaxBlockLds)
      g.wpb >>= 1;
    int blocks = 0;
    for (size_t i = 0; i < in.size(); ++i) {
      if (kNumKinds * in[i].pack + kind[i] != kd) continue;
      SegDev sg = in[i];
      sg.block_begin = blocks;
      blocks += (sg.n_groups + g.wpb - 1) / g.wpb;
      out->push_back(sg);
    }
    g.n_segs = (int)out->size() - g.seg_begin;
    g.n_blocks = blocks;
    groups->push_back(g);
  }
}

void class_segments(const cx_ctx *ctx, const ClassRt &c, int L, int P, std::vector<SegDev> *segs) {
  const int spw = 64 / L;
  // the kernels address a segment's records with 32-bit per-lane byte offsets:
  // a class whose observation block would reach 4 GiB per step is cut into
  // several segments (whole waves each)
  int64_t chunk = (int64_t)(((1ull << 32) - 1) / (4ull * (uint64_t)c.comp.obs_dim));
  chunk -= chunk % 64;
  for (int64_t e0 = 0; e0 < c.n_envs; e0 += chunk) {
    const int64_t n = std::min<int64_t>(chunk, c.n_envs - e0);
    SegDev sg{};
    sg.cls = c.dev;
    sg.env0 = c.env_begin + e0;
    sg.n_envs = n;
    sg.n_groups = (int32_t)((n + spw - 1) / spw);
    sg.pack = pack_id(L, P);
    sg.obs_dim = c.comp.obs_dim;
    sg.seed = ctx->seed;
    const int64_t so = c.slot_off + e0 * c.comp.S;
    sg.q = ctx->q + so;
    sg.u = ctx->u + so;
    sg.cap = ctx->cap + so;
    sg.p_last = ctx->p_last + so;
    sg.dwell = ctx->dwell + so;
    sg.ret = ctx->ret + c.env_begin + e0;
    sg.bsoc = ctx->bsoc + c.env_begin + e0;
    sg.bp = ctx->bp + c.env_begin + e0;
    sg.utype = ctx->utype + so;
    sg.rbar = ctx->rbar + so;
    sg.obs_off = c.obs_off + e0 * c.comp.obs_dim;
    sg.act_off = c.port_off + e0 * c.comp.n_act;
    sg.env_off = c.env_begin + e0;
    segs->push_back(sg);
  }
}

cx_status rebuild_segments(cx_ctx *ctx) {
  std::vector<SegDev> segs;
  std::vector<int> dl;
  std::vector<int> kind;
  for (ClassRt &c : ctx->classes) {
    if (c.n_envs == 0) continue;
    const size_t first = segs.size();
    class_segments(ctx, c, c.lanes, c.comp.S / c.lanes, &segs);
    for (size_t i = first; i < segs.size(); ++i) {
      dl.push_back(c.tab.dwell_log2);
      kind.push_back(c.host_view.kind == kKindSimple && ctx->stage_obs ? kKindSimpleStaged : c.host_view.kind);
    }
  }
  build_groups(segs, dl, kind, ctx->wpb, &ctx->segs_host, &ctx->groups);
  if (!ctx->segs_dev || ctx->segs_host.size() > ctx->segs_cap) {
    if (ctx->segs_dev) {
      hipError_t e = hipStreamSynchronize(ctx->stream);  // launches in flight may still read the old table
      if (e != hipSuccess) return hip_fail(ctx, e, "segment table resize synchronize");
      (void)hipFree(ctx->segs_dev);
      ctx->segs_dev = nullptr;
    }
    const size_t cap = std::max<size_t>(ctx->segs_host.size(), ctx->classes.size());
    hipError_t e = hipMalloc(&ctx->segs_dev, sizeof(SegDev) * std::max<size_t>(1, cap));
    if (e != hipSuccess) return fail_status(CX_E_OOM, "hipMalloc of segment table failed");
    ctx->segs_cap = cap;
  }
  if (!ctx->segs_host.empty()) {
    // work still queued on the context's stream reads the current table
    hipError_t e = ctx->segs_cap ? hipStreamSynchronize(ctx->stream) : hipSuccess;
    if (e != hipSuccess) return hip_fail(ctx, e, "segment table synchronize");
    e = hipMemcpy(ctx->segs_dev, ctx->segs_host.data(), sizeof(SegDev) * ctx->segs_host.size(),
                             hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(ctx, e, "upload of segment table");
  }
  graph_destroy(ctx->graph);
  return CX_OK;
}

LaunchArgs base_args(const cx_ctx *ctx) {
  LaunchArgs a{};
  a.segs = ctx->segs_dev;
  a.n_segs = (int32_t)ctx->segs_host.size();
  a.per_segment = 0;
  a.t_day0 = ctx->t_day;
  a.g0 = ctx->g;
  a.obs_stride = ctx->obs_elems;
  a.act_stride = ctx->total_ports;
  a.env_stride = ctx->n_envs;
  return a;
}

void advance_clock(cx_ctx *ctx, int32_t T) {
  ctx->g += (uint32_t)T;
  ctx->t_day = (int32_t)(((int64_t)ctx->t_day + T) % ctx->steps_ep);
}

static void free_ctx(cx_ctx *ctx) {
  if (!ctx) return;
  graph_destroy(ctx->graph);
  for (auto &c : ctx->classes)
    if (c.dev_mem) (void)hipFree(c.dev_mem);
  if (ctx->state_mem) (void)hipFree(ctx->state_mem);
  if (ctx->segs_dev) (void)hipFree(ctx->segs_dev);
  free_policy(ctx);
  delete ctx;
}

static cx_status create_impl(const cx_station_spec *specs, int32_t n_specs, const int32_t *env_class,
                             int64_t n_envs, uint64_t seed, cx_ctx **out) {
  if (!out) return fail_status(CX_E_INVALID, "out must not be NULL");
  *out = nullptr;
  if (!specs || n_specs < 1 || n_specs > 4096) return fail_status(CX_E_INVALID, "need 1..4096 station specs");
  if (n_envs < 1 || n_envs > (int64_t)1 << 31) return fail_status(CX_E_INVALID, "n_envs must be in 1..2^31");
  std::vector<int64_t> count(n_specs, 0);
  for (int64_t e = 0; e < n_envs; ++e) {
    const int32_t c = env_class ? env_class[e] : 0;
    if (c < 0 || c >= n_specs) return fail_status(CX_E_INVALID, "env_class out of range");
    if (e > 0 && env_class && env_class[e - 1] > c)
      return fail_status(CX_E_INVALID, "env_class must be non-decreasing (classes contiguous)");
    count[c] += 1;
  }
  cx_ctx *ctx = new cx_ctx();
  ctx->seed = seed;
  ctx->n_envs = n_envs;
  ctx->classes.resize(n_specs);
  int64_t env_begin = 0, port_off = 0, obs_off = 0, slot_off = 0, port_count = 0;
  for (int i = 0; i < n_specs; ++i) {
    ClassRt &c = ctx->classes[i];
    std::string err;
    if (!copy_spec(specs[i], &c.spec, &err) || !compile_spec(c.spec, &c.comp, &err)) {
      free_ctx(ctx);
      return fail_status(CX_E_INVALID, "station spec " + std::to_string(i) + ": " + err);
    }
    if (i > 0 && specs[i].steps_per_episode != specs[0].steps_per_episode) {
      free_ctx(ctx);
      return fail_status(CX_E_INVALID, "all specs must share steps_per_episode");
    }
    build_tables(c.spec, &c.tab);
    if (!tables_monotone(c.tab)) {
      free_ctx(ctx);
      return fail_status(CX_E_INVALID, "sampling tables are not monotone");
    }
    c.env_begin = env_begin;
    c.n_envs = count[i];
    c.port_off = port_off;
    c.obs_off = obs_off;
    c.slot_off = slot_off;
    c.lanes = default_lanes(c.comp.S);
    env_begin += c.n_envs;
    port_off += c.n_envs * c.comp.n_act;
    obs_off += c.n_envs * c.comp.obs_dim;
    slot_off += c.n_envs * c.comp.S;
    port_count += c.n_envs * c.comp.N;
  }
  if (hipGetDevice(&ctx->device) != hipSuccess) {
    free_ctx(ctx);
    return fail_status(CX_E_DEVICE, "no HIP device");
  }
  ctx->steps_ep = specs[0].steps_per_episode;
  ctx->total_ports = port_off;
  ctx->obs_elems = obs_off;
  ctx->total_slots = slot_off;
  ctx->port_count = port_count;
  // state: q (double), u / cap / p_last (float), dwell (int16) over all slots; return,
  // battery SoC (double) and battery power (float) per env
  const size_t qbytes = align256(sizeof(double) * (size_t)slot_off);
  const size_t fbytes = align256(sizeof(float) * (size_t)slot_off);
  const size_t dbytes = align256(sizeof(int16_t) * (size_t)slot_off);
  const size_t rbytes = align256(sizeof(double) * (size_t)n_envs);
  const size_t bbytes = align256(sizeof(float) * (size_t)n_envs);
  const size_t ubytes = align256((size_t)slot_off);
  const size_t total = qbytes + 4 * fbytes + dbytes + 2 * rbytes + bbytes + ubytes;
  if (hipMalloc(&ctx->state_mem, total) != hipSuccess) {
    free_ctx(ctx);
    return fail_status(CX_E_OOM, "hipMalloc of station state failed");
  }
  ctx->state_bytes_dev = total;
  ctx->device_bytes += (int64_t)total;
  unsigned char *b = static_cast<unsigned char *>(ctx->state_mem);
  ctx->q = reinterpret_cast<double *>(b);
  ctx->u = reinterpret_cast<float *>(b + qbytes);
  ctx->cap = reinterpret_cast<float *>(b + qbytes + fbytes);
  ctx->p_last = reinterpret_cast<float *>(b + qbytes + 2 * fbytes);
  ctx->dwell = reinterpret_cast<int16_t *>(b + qbytes + 3 * fbytes);
  ctx->ret = reinterpret_cast<double *>(b + qbytes + 3 * fbytes + dbytes);
  ctx->bsoc = reinterpret_cast<double *>(b + qbytes + 3 * fbytes + dbytes + rbytes);
  ctx->bp = reinterpret_cast<float *>(b + qbytes + 3 * fbytes + dbytes + 2 * rbytes);
  ctx->utype = reinterpret_cast<uint8_t *>(b + qbytes + 3 * fbytes + dbytes + 2 * rbytes + bbytes);
  ctx->rbar = reinterpret_cast<float *>(b + qbytes + 3 * fbytes + dbytes + 2 * rbytes + bbytes + ubytes);
  if (hipMemset(ctx->state_mem, 0, total) != hipSuccess) {
    free_ctx(ctx);
    return fail_status(CX_E_DEVICE, "hipMemset of station state failed");
  }
  // station batteries start at their initial SoC
  for (const ClassRt &c : ctx->classes) {
    if (!c.comp.battery || c.n_envs == 0) continue;
    std::vector<double> v((size_t)c.n_envs, c.spec.s.battery_soc0);
    if (hipMemcpy(ctx->bsoc + c.env_begin, v.data(), 8 * v.size(), hipMemcpyHostToDevice) != hipSuccess) {
      free_ctx(ctx);
      return fail_status(CX_E_DEVICE, "upload of battery state failed");
    }
  }
  for (auto &c : ctx->classes) {
    cx_status st = upload_class(ctx, c);
    if (st != CX_OK) {
      free_ctx(ctx);
      return st;
    }
  }
  cx_status st = rebuild_segments(ctx);
  if (st != CX_OK) {
    free_ctx(ctx);
    return st;
  }
  *out = ctx;
  return CX_OK;
}

}  // namespace cx

using namespace cx;

#define CTX_CHECK(ctx)                                                                 \
  do {                                                                                 \
    if (!(ctx)) return fail_status(CX_E_INVALID, "context is NULL");                   \
    if ((ctx)->failed) return fail_status(CX_E_DEVICE, "context has a sticky device error"); \
  } while (0)

extern "C" {

cx_status cx_create(const cx_station_spec *spec, int64_t n_envs, uint64_t seed, cx_ctx **out) {
  return create_impl(spec, 1, nullptr, n_envs, seed, out);
}

cx_status cx_create_multi(const cx_station_spec *specs, int32_t n_specs, const int32_t *env_class,
                          int64_t n_envs, uint64_t seed, cx_ctx **out) {
  if (!env_class) return fail_status(CX_E_INVALID, "env_class must not be NULL");
  return create_impl(specs, n_specs, env_class, n_envs, seed, out);
}

cx_status cx_set_stream(cx_ctx *ctx, void *hip_stream) {
  CTX_CHECK(ctx);
  ctx->stream = static_cast<hipStream_t>(hip_stream);
  return CX_OK;
}

cx_status cx_get_info(const cx_ctx *ctx, cx_info *info) {
  if (!ctx || !info) return fail_status(CX_E_INVALID, "NULL argument");
  info->n_envs = ctx->n_envs;
  info->total_ports = ctx->total_ports;
  info->obs_elems = ctx->obs_elems;
  info->n_classes = (int32_t)ctx->classes.size();
  info->steps_per_episode = ctx->steps_ep;
  info->g = ctx->g;
  info->t_day = ctx->t_day;
  info->seed = ctx->seed;
  info->state_bytes = state_blob_bytes(ctx);
  info->device_bytes = ctx->device_bytes;
  info->obs_stage = ctx->stage_obs ? 1 : 0;
  return CX_OK;
}

cx_status cx_get_class_info(const cx_ctx *ctx, int32_t cls, cx_class_info *info) {
  if (!ctx || !info) return fail_status(CX_E_INVALID, "NULL argument");
  if (cls < 0 || cls >= (int32_t)ctx->classes.size()) return fail_status(CX_E_INVALID, "class out of range");
  const ClassRt &c = ctx->classes[cls];
  info->env_begin = c.env_begin;
  info->n_envs = c.n_envs;
  info->port_offset = c.port_off;
  info->obs_offset = c.obs_off;
  info->n_ports = c.comp.N;
  info->obs_dim = c.comp.obs_dim;
  info->slots = c.comp.S;
  info->levels = c.comp.D;
  info->lanes_per_station = c.lanes;
  info->waves_per_block = ctx->wpb;
  info->n_actions = c.comp.n_act;
  return CX_OK;
}

cx_status cx_reset(cx_ctx *ctx, float *obs_dev) {
  CTX_CHECK(ctx);
  hipError_t e = hipMemsetAsync(ctx->state_mem, 0, ctx->state_bytes_dev, ctx->stream);
  if (e != hipSuccess) return hip_fail(ctx, e, "cx_reset memset");
  for (const ClassRt &c : ctx->classes) {
    if (!c.comp.battery || c.n_envs == 0) continue;
    e = launch_fill_f64(ctx->bsoc + c.env_begin, c.n_envs, c.spec.s.battery_soc0, ctx->stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "cx_reset battery fill");
  }
  ctx->t_day = 0;
  if (obs_dev) {
    for (auto &c : ctx->classes) {
      e = launch_reset_obs_one(c.dev, c.n_envs, obs_dev + c.obs_off, ctx->seed, c.env_begin, ctx->g, ctx->stream);
      if (e != hipSuccess) return hip_fail(ctx, e, "cx_reset observation kernel");
    }
  }
  return CX_OK;
}

cx_status cx_step_ex(cx_ctx *ctx, cx_action_mode mode, const uint8_t *actions_in_dev, const cx_traj *out) {
  CTX_CHECK(ctx);
  if (mode < CX_ACT_EXTERNAL || mode > CX_ACT_POLICY) return fail_status(CX_E_INVALID, "bad action mode");
  if (mode == CX_ACT_EXTERNAL && !actions_in_dev) return fail_status(CX_E_INVALID, "EXTERNAL needs actions");
  if (mode == CX_ACT_POLICY) return policy_step(ctx, 1, CX_OUT_FULL, out, /*graph=*/false);
  LaunchArgs a = base_args(ctx);
  a.T = 1;
  a.mode = mode;
  a.out_mode = CX_OUT_FULL;
  a.act_in = actions_in_dev;
  if (out) {
    a.obs = out->obs; a.act = out->actions; a.reward = out->reward; a.done = out->done;
  }
  hipError_t e = launch_groups(a, ctx->groups.data(), (int)ctx->groups.size(), ctx->stream);
  if (e != hipSuccess) return hip_fail(ctx, e, "cx_step launch");
  advance_clock(ctx, 1);
  return CX_OK;
}

cx_status cx_step(cx_ctx *ctx, const uint8_t *actions_dev, float *obs_dev, float *reward_dev,
                  uint8_t *done_dev) {
  cx_traj t{obs_dev, nullptr, reward_dev, done_dev};
  return cx_step_ex(ctx, CX_ACT_EXTERNAL, actions_dev, &t);
}

cx_status cx_rollout(cx_ctx *ctx, int32_t T, cx_action_mode mode, cx_out_mode out_mode,
                     const uint8_t *actions_in_dev, const cx_traj *out) {
  CTX_CHECK(ctx);
  if (T < 0 || T > (1 << 24)) return fail_status(CX_E_INVALID, "T must be in 0..2^24");
  if (mode < CX_ACT_EXTERNAL || mode > CX_ACT_POLICY) return fail_status(CX_E_INVALID, "bad action mode");
  if (out_mode < CX_OUT_FULL || out_mode > CX_OUT_ACT_REWARD) return fail_status(CX_E_INVALID, "bad out mode");
  if (mode == CX_ACT_EXTERNAL && !actions_in_dev && T > 0) return fail_status(CX_E_INVALID, "EXTERNAL needs actions");
  if (T == 0) return CX_OK;
  if (mode == CX_ACT_POLICY) return policy_step(ctx, T, out_mode, out, /*graph=*/true);
  LaunchArgs a = base_args(ctx);
  a.T = T;
  a.mode = mode;
  a.out_mode = out_mode;
  a.act_in = actions_in_dev;
  if (out) {
    a.obs = out_mode == CX_OUT_FULL ? out->obs : nullptr;
    a.act = out_mode != CX_OUT_REWARD ? out->actions : nullptr;
    a.reward = out->reward;
    a.done = out->done;
  }
  hipError_t e = graph_rollout(ctx->graph, a, ctx->groups.data(), (int)ctx->groups.size(), ctx->stream);
  if (e != hipSuccess) return hip_fail(ctx, e, "cx_rollout graph launch");
  advance_clock(ctx, T);
  return CX_OK;
}

cx_status cx_get_tables(const cx_ctx *ctx, int32_t cls, uint32_t *tpois_host, uint32_t *tdwell_host) {
  if (!ctx) return fail_status(CX_E_INVALID, "context is NULL");
  if (cls < 0 || cls >= (int32_t)ctx->classes.size()) return fail_status(CX_E_INVALID, "class out of range");
  const Tables &t = ctx->classes[cls].tab;
  if (tpois_host) std::memcpy(tpois_host, t.tpois.data(), sizeof(uint32_t) * t.tpois.size());
  if (tdwell_host) std::memcpy(tdwell_host, t.tdwell.data(), sizeof(uint32_t) * t.tdwell.size());
  return CX_OK;
}

cx_status cx_set_packing(cx_ctx *ctx, int32_t cls, int32_t lanes_per_station, int32_t waves_per_block) {
  CTX_CHECK(ctx);
  if (cls < 0 || cls >= (int32_t)ctx->classes.size()) return fail_status(CX_E_INVALID, "class out of range");
  if (!legal_packing(ctx->classes[cls].comp.S, lanes_per_station))
    return fail_status(CX_E_INVALID, "lanes_per_station must be a power of two in 4..64 with 1, 2 or 4 slots per lane");
  if (waves_per_block < 1 || waves_per_block > kMaxWaves) return fail_status(CX_E_INVALID, "waves_per_block must be in 1..8");
  ctx->classes[cls].lanes = lanes_per_station;
  ctx->wpb = waves_per_block;
  return rebuild_segments(ctx);
}

cx_status cx_set_obs_stage(cx_ctx *ctx, int32_t on) {
  CTX_CHECK(ctx);
  if (on != 0 && on != 1) return fail_status(CX_E_INVALID, "on must be 0 or 1");
  ctx->stage_obs = on != 0;
  return rebuild_segments(ctx);
}

cx_status cx_synchronize(cx_ctx *ctx) {
  CTX_CHECK(ctx);
  hipError_t e = hipStreamSynchronize(ctx->stream);
  if (e != hipSuccess) return hip_fail(ctx, e, "stream synchronize");
  return CX_OK;
}

const char *cx_last_error(void) { return g_last_error.c_str(); }

void cx_destroy(cx_ctx *ctx) {
  if (!ctx) return;
  (void)hipStreamSynchronize(ctx->stream);
  free_ctx(ctx);
}

}  // extern "C"

extern "C" {

cx_status cx_compile_layout(const cx_station_spec *spec, int32_t *slots, int32_t *levels, int32_t *slot_port,
                            uint32_t *slot_lb, float *slot_cap) {
  if (!spec) return fail_status(CX_E_INVALID, "spec is NULL");
  SpecCopy sc;
  Compiled k;
  std::string err;
  if (!copy_spec(*spec, &sc, &err) || !compile_spec(sc, &k, &err)) return fail_status(CX_E_INVALID, err);
  if (slots) *slots = k.S;
  if (levels) *levels = k.D;
  for (int s = 0; s < kMaxSlots; ++s) {
    if (slot_port) slot_port[s] = s < k.S ? k.slot_port[s] : -1;
    if (slot_lb) slot_lb[s] = s < k.S ? k.slot_lb[s] : 0u;
    for (int d = 0; d < kMaxLevels && slot_cap; ++d)
      slot_cap[d * kMaxSlots + s] =
          (s < k.S && d < k.D) ? k.slot_cap[(size_t)d * k.S + s] : std::numeric_limits<float>::infinity();
  }
  return CX_OK;
}

cx_status cx_build_tables(const cx_station_spec *spec, uint32_t *tpois, uint32_t *tdwell) {
  if (!spec) return fail_status(CX_E_INVALID, "spec is NULL");
  SpecCopy sc;
  Compiled k;
  std::string err;
  if (!copy_spec(*spec, &sc, &err) || !compile_spec(sc, &k, &err)) return fail_status(CX_E_INVALID, err);
  Tables t;
  build_tables(sc, &t);
  if (tpois) std::memcpy(tpois, t.tpois.data(), sizeof(uint32_t) * t.tpois.size());
  if (tdwell) std::memcpy(tdwell, t.tdwell.data(), sizeof(uint32_t) * t.tdwell.size());
  return CX_OK;
}

}  // extern "C"
