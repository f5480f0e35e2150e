// cx_ctx.h -- the context object behind cx_ctx* and helpers shared by the
// host translation units.
#pragma once

#include <string>
#include <vector>

#include "cx_spec.h"

namespace cx {

struct ClassRt {
  SpecCopy spec;
  Compiled comp;
  Tables tab;
  int64_t env_begin = 0, n_envs = 0, port_off = 0, obs_off = 0, slot_off = 0;
  int lanes = 16;                 // current packing
  void *dev_mem = nullptr;        // ClassDev + per-slot arrays + tables
  ClassDev *dev = nullptr;
  ClassDev host_view{};           // host copy (pointers are device addresses)
};

struct PolicyRt;                  // defined with the policy kernels

}  // namespace cx

struct cx_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  uint64_t seed = 0;
  uint32_t g = 0;
  int32_t t_day = 0;
  int32_t steps_ep = 288;
  int64_t n_envs = 0, total_ports = 0, obs_elems = 0, total_slots = 0;
  int64_t port_count = 0;         // sum of n_ports over the envs (total_ports counts action bytes)
  std::vector<cx::ClassRt> classes;
  // state, env-major slot layout: q = 1 - SoC (double), u = 1 - target SoC,
  // capacity and last power (float), dwell (int16); return per env (double)
  void *state_mem = nullptr;
  size_t state_bytes_dev = 0;
  double *q = nullptr;
  float *u = nullptr, *cap = nullptr, *p_last = nullptr;
  int16_t *dwell = nullptr;
  double *ret = nullptr;
  double *bsoc = nullptr;         // station battery SoC per env (battery classes)
  float *bp = nullptr;            // station battery last power per env
  uint8_t *utype = nullptr;       // user type per slot (1 = charge-sensitive)
  float *rbar = nullptr;          // the car's maximum rate per slot (car models)
  // launch layout: segments grouped by slots per lane, one kernel per group
  cx::SegDev *segs_dev = nullptr;
  size_t segs_cap = 0;            // entries allocated at segs_dev
  std::vector<cx::SegDev> segs_host;
  std::vector<cx::LaunchGroup> groups;
  int wpb = 4;
  // SIMPLE classes of up to 32 lanes per station write their observations
  // through an LDS stage (cx_set_obs_stage / cx_autotune)
  bool stage_obs = false;
  bool failed = false;
  int64_t device_bytes = 0;
  cx::RolloutGraph graph;
  cx::PolicyRt *policy = nullptr;
};

namespace cx {

extern thread_local std::string g_last_error;
cx_status fail_status(cx_status st, const std::string &msg);
cx_status hip_fail(cx_ctx *ctx, hipError_t e, const char *what);
cx_status rebuild_segments(cx_ctx *ctx);
void class_segments(const cx_ctx *ctx, const ClassRt &c, int L, int P, std::vector<SegDev> *segs);
void build_groups(const std::vector<SegDev> &in, const std::vector<int> &log2_dwell,
                  const std::vector<int> &kind, int wpb, std::vector<SegDev> *out,
                  std::vector<LaunchGroup> *groups);
LaunchArgs base_args(const cx_ctx *ctx);
void advance_clock(cx_ctx *ctx, int32_t T);
bool legal_packing(int S, int lanes);
int default_lanes(int S);
size_t state_blob_bytes(const cx_ctx *ctx);
size_t class_block(const SpecCopy &sc, const Compiled &k, const Tables &t, unsigned char *dev_base,
                   std::vector<unsigned char> *host, ClassDev *view);

// policy (cx_policy.hip)
void free_policy(cx_ctx *ctx);
cx_status policy_step(cx_ctx *ctx, int32_t T, cx_out_mode out_mode, const cx_traj *out, bool graph);

}  // namespace cx
