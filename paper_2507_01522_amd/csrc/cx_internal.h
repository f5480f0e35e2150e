// cx_internal.h -- data structures shared by the host runtime and the gfx950
// kernels of the batched EV charging-station step.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "cx.h"

namespace cx {

constexpr int kMaxLevels = 4;    // capacity-tree depth, root included
constexpr int kMaxSlots = 256;   // padded ports per station
constexpr int kPoisK = 24;       // arrival counts are capped at 24 per step
constexpr int kPoisStride = 32;  // threshold row padded with 0xFFFFFFFF for a 5-step bisection
constexpr int kMaxWaves = 8;     // waves per block
constexpr int kMaxBlockLog2 = 9; // aligned slot blocks of 2^0 .. 2^8 slots

// Philox counter domains (word 3 of the counter); see the action / arrival
// / noise derivations in the kernels.
enum : uint32_t { kDomEnv = 0, kDomAct = 1, kDomCar = 2, kDomGum = 3, kDomUser = 4, kDomDay = 5 };

// Packings: lanes per station L in {4,...,64} and slots per lane P in {1,2,4};
// L * P = padded slots of the class.
constexpr int kNumPackings = 15;
// Kernel kinds per packing: general classes, SIMPLE classes (every per-slot
// constant uniform), and extended classes (V2G ports, a station battery or
// charge-sensitive users).
// kKindSimpleStaged: a SIMPLE class whose observations go through the block's
// LDS stage (a context option, cx_set_obs_stage).
enum : int { kKindGeneral = 0, kKindSimple = 1, kKindExt = 2, kKindSimpleStaged = 3, kNumKinds = 4 };
__host__ __device__ constexpr int pack_lanes(int id) { return 4 << (id % 5); }
__host__ __device__ constexpr int pack_per_lane(int id) { return 1 << (id / 5); }
inline int pack_id(int lanes, int per_lane) {
  int li = 0;
  while ((4 << li) != lanes) ++li;
  int pi = per_lane == 1 ? 0 : per_lane == 2 ? 1 : 2;
  return pi * 5 + li;
}

// One compiled station class, in device memory.  Per-slot arrays use the
// padded, aligned slot layout: slot s of a station holds port slot_port[s]
// (-1 for a padding slot that never holds a car).
struct ClassDev {
  int32_t n_ports, S, D, n_levels;
  int32_t steps_ep, obs_dim, dwell_log2, uniform_eta;
  float dt, inv_dt, inv_1mtau, p_sell;
  float p_sell_grid, fixed_cost, alpha_sat, alpha_dec;
  float price_sigma, cap_lo, cap_span, soc_lo;
  float soc_span, tgt_lo, tgt_span, inv_steps_ep;
  float inv_n_levels, inv_eta_uniform;
  uint32_t lvl_lb_uniform;     // per level (8 bits, level 0 = deepest): the block size log2
                               // shared by every slot of the level, 0xFF if they differ
  int32_t simple;              // 1: no padding, one port maximum / efficiency, and per level
                               // one block size and one limit (all per-slot constants uniform)
  float pmax_u, inv_pmax_u;    // the port maximum of a simple class
  float lvl_cap_u[kMaxLevels]; // per level: the limit of a simple class (+inf beyond D)
  // a simple class by block size: blk_cap[k] is the limit of the level below the
  // root whose nodes own aligned blocks of 2^k slots (+inf if none), blk_mask
  // bit k set where there is one
  float blk_cap[kMaxBlockLog2];
  uint32_t blk_mask;
  const int32_t *slot_port;    // [S]
  const float *slot_pmax;      // [S]
  const float *slot_inv_pmax;  // [S]
  const float *slot_inv_eta;   // [S]
  const uint32_t *slot_lb;     // [S]: per level (8 bits, level 0 = deepest) the log2 block size, or
                               // 0x80 | node for a dense level (0: no node of the level covers the slot)
  const float *slot_cap;       // [D][S]: eta_H * I_H of the level's node holding the slot (+inf if none)
  const uint32_t *tpois;       // [steps_ep][32]
  const uint32_t *tdwell;      // [1 << dwell_log2]: thresholds for stays of 2, 3, ... steps
  const float *glob;           // [steps_ep][4]: sin, cos, base price, 0
  // extended classes: V2G ports and the station battery (FP64 constants: the
  // battery is one scalar per station, its arithmetic is kept in FP64), and
  // charge-sensitive users
  int32_t n_neg;               // discharge levels of a port: n_levels (V2G) or 0
  int32_t has_batt;            // 1: a station battery (the (N+1)-th action byte)
  int32_t n_act;               // action bytes per env
  int32_t kind;                // kKind* of the class
  float alpha_db, alpha_dc;    // degradation weights: battery discharge, car discharge
  float b_inv_rate, pad_f;     // 1 / battery maximum rate
  double b_cap, b_inv_cap, b_rate, b_inv_1mtau, b_soc0;
  double dt_d, inv_dt_d, inv_n_d;  // dt, 1/dt, 1/n_levels in FP64
  const float *slot_pdis;      // [S]: discharge maxima
  const float *slot_eta;       // [S]: efficiencies
  int32_t has_users;           // 1: some users are charge-sensitive
  uint32_t cs_thresh;          // a user is charge-sensitive iff its Philox word <= cs_thresh
  int32_t user_obs;            // observation offset of the per-port user flags
  float alpha_sat1, beta_sat1; // c_satisfaction,1 weight and its early-leave weight
  float inv_n_days;            // exploring starts: 1 / n_days
  int32_t n_days, day_obs;     // price days (0: none) and the observation offset of the day features
  int32_t n_models;            // car models (0: none)
  uint32_t dense_nodes;        // dense layout: per level below the root (8 bits) its node count; 0 = aligned
  int32_t pad_dn;
  const float *price_days;     // [n_days][steps_ep]
  const uint32_t *model_thresh;// [8]: model = #{m < n_models : w > model_thresh[m]}
  const float *model_data;     // [8][3]: capacity, AC rate, DC rate
  const int32_t *slot_dc;      // [S]: 1 = DC charger
};

// One class's env range inside a launch.  Static fields are set when the
// context (or serving request) is laid out; dynamic fields are used when the
// launch says so (serving), otherwise the launch arguments apply.
struct SegDev {
  const ClassDev *cls;
  int64_t env0;         // Philox env index of the segment's first env
  int64_t n_envs;
  int32_t n_groups;     // waves needed: ceil(n_envs / stations per wave)
  int32_t block_begin;  // first block of this segment in the launch
  int32_t pack;
  int32_t obs_dim;      // floats per env observation (sizes the LDS record stage of its launch)
  uint64_t seed;
  // state, env-major slot layout, at the segment's first env.  A car is kept
  // as q = 1 - SoC (FP64: the per-step increments are accumulated here),
  // u = 1 - target SoC, its capacity and the last applied power; the energy
  // still wanted is e_rem = (q - u) * cap.  Empty slots hold zeros.
  double *q;
  float *u, *cap, *p_last;
  int16_t *dwell;
  double *ret;
  // offsets of the segment's first env inside the output records
  int64_t obs_off, act_off, env_off;
  // dynamic (per-segment launches only)
  int32_t T, t_day0;
  uint32_t g0;
  int32_t mode, out_mode, pad2;
  float *obs;
  uint8_t *act;
  float *reward;
  uint8_t *done;
  const uint8_t *act_in;
  int64_t obs_stride, act_stride, env_stride;
  // station battery state per env (battery classes): SoC (FP64) and last power
  double *bsoc;
  float *bp;
  // user type per slot (classes with charge-sensitive users): 1 = charge-sensitive
  uint8_t *utype;
  // the car's maximum rate per slot (classes with car models)
  float *rbar;
};

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// Launch-wide arguments (by value).
struct LaunchArgs {
  const SegDev *segs;
  int32_t n_segs;
  int32_t per_segment;  // 1: take T/g0/t_day0/modes/outputs from each segment
  int32_t T, t_day0;
  uint32_t g0;
  int32_t mode, out_mode;
  int32_t lds_tdwell;   // 1: stage the stay thresholds in LDS (set per launch group)
  // observation records staged in LDS (set per launch group): byte offset of
  // the two stage buffers in the dynamic LDS and floats per buffer (0: each
  // lane stores its observation values to HBM itself)
  int32_t stage_off, stage_floats;
  float *obs;
  uint8_t *act;
  float *reward;
  uint8_t *done;
  const uint8_t *act_in;
  int64_t obs_stride, act_stride, env_stride;
  // the fused policy rollout (mode CX_ACT_POLICY): the MLP's weights in
  // fragment order, its sizes, the observation the rollout starts from, and
  // where the block's BF16 observations, hidden units and levels sit in LDS
  struct Pol {
    const float *obs0;    // [envs of the segment table][in_dim], 16-byte aligned rows
    // fragments padded with zeros to the largest sizes (8 K-steps of features,
    // 16 hidden tiles, 8 K-steps of hidden units, 3 level tiles)
    const u32x4 *w1f;     // [16][8][64] fragments of W1^T
    const float *b1;      // [256]
    const u32x4 *w2f;     // [G][3][8][64] fragments of W2^T
    const float *b2f;     // [G][3][16]
    int32_t in_dim, K1, HP, R, G, L1;
    int32_t hb_off, xb_off, act_off;  // LDS byte offsets
  } pol;
};

// One launch group: the segments of one packing, launched by the kernel
// instantiated for that packing.
struct LaunchGroup {
  int pack = 0;         // packing id
  int kind = kKindGeneral;  // kernel kind (kKind*)
  int seg_begin = 0;    // index of the first segment in the device segment table
  int n_segs = 0;
  int n_blocks = 0;
  int max_dwell_log2 = 1;  // largest stay table among its classes (LDS bytes = 4 << this)
  int max_T = 0;           // per-segment launches: the longest horizon among its segments
  int max_obs_dim = 0;     // largest observation among its classes (floats)
  int wpb = 1;             // waves per block: the context's choice, halved until the LDS fits
};

// Does a launch group stage its observations?  Its SIMPLE classes do, in every
// packing, when the context asks for it.
__host__ __device__ constexpr bool group_stages(int kind, int pack) {
  (void)pack;
  return kind == kKindSimpleStaged;
}

// LDS a block may take for its tables and the two observation stages.
constexpr size_t kMaxBlockLds = 64 << 10;
// Per-step tables of a day kept in LDS when a day has at most this many steps:
// the first four arrival thresholds of every step (one 16-byte row each) and
// the base price of every step (so the draws ahead read no device memory).
constexpr int kLdsExoSteps = 512;
constexpr int kLdsExoMinT = 32;   // ... in launches of at least this many steps

// LDS layout of a launch group's blocks: the stay table (4 << dwell_log2
// bytes), the per-step tables (kLdsExoSteps x 20 bytes), then two observation
// stages of waves x stations per wave x the largest observation floats, plus 3
// floats to align them with HBM (rounded to 16 bytes).
inline size_t group_table_bytes(int dwell_log2) {
  return ((((size_t)4 << dwell_log2) + 15) & ~(size_t)15) + (size_t)kLdsExoSteps * 20;
}
// Bytes with the stages; *stage_off / *stage_floats: where the stages begin
// and floats per stage.
inline size_t group_lds_bytes(int wpb, int pack, int max_obs_dim, int dwell_log2, int32_t *stage_off,
                              int32_t *stage_floats) {
  const size_t off = group_table_bytes(dwell_log2);
  const size_t floats =
      ((size_t)wpb * (size_t)(64 / pack_lanes(pack)) * (size_t)max_obs_dim + 3 + 3) & ~(size_t)3;
  if (stage_off) *stage_off = (int32_t)off;
  if (stage_floats) *stage_floats = (int32_t)floats;
  return off + 8 * floats;
}

// The fused policy rollout: blocks of 4 waves of 8-lane stations (32 envs, two
// 16-env tiles of the MLP).  LDS: the stay table, then the stage (one
// buffer of 32 observations), which the hidden units (8 x 2 KiB) overwrite once
// it has been read, then the observations in BF16 (32 x 528 bytes) and a level
// byte per port and env.  Returns the bytes; sets the offsets.
constexpr int kPolRolloutWaves = 4;
constexpr int kPolRolloutEnvs = kPolRolloutWaves * 8;
constexpr int kPolXbRow = 33;  // 16-byte fragments per env row of the BF16 observations (32 used)
inline size_t policy_rollout_lds(int dwell_log2, int obs_dim, int N, int32_t *stage_off,
                                 int32_t *stage_floats, int32_t *hb_off, int32_t *xb_off, int32_t *act_off) {
  auto a16 = [](size_t x) { return (x + 15) & ~(size_t)15; };
  const size_t off = a16((size_t)4 << dwell_log2);  // the stay table only (no per-step tables)
  const size_t floats = ((size_t)kPolRolloutEnvs * obs_dim + 3) & ~(size_t)3;
  const size_t region = a16(std::max(4 * floats, (size_t)8 * (kPolRolloutEnvs / 16) * 64 * 16));
  const size_t xb = off + region;
  const size_t act = xb + (size_t)kPolRolloutEnvs * 16 * kPolXbRow;
  *stage_off = (int32_t)off;
  *stage_floats = (int32_t)floats;
  *hb_off = (int32_t)off;
  *xb_off = (int32_t)xb;
  *act_off = (int32_t)act;
  return act + a16((size_t)kPolRolloutEnvs * N);
}

// The persistent rollout as a HIP graph with one kernel node per launch group
// (no dependencies between them), instantiated once per launch shape and
// re-parameterised on every call.
struct RolloutGraph {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipGraphNode_t node[kNumKinds * kNumPackings] = {};
  int n_nodes = 0;
  int shape[kNumKinds * kNumPackings][4] = {};  // kernel, blocks, waves per block, LDS bytes
};

// Arguments of the policy kernel (cx_policy.hip): the perceptron's weights in
// fragment order and one step's observations in, levels and / or logits out.
struct PolicyArgs {
  const float *obs;  // [n][in_dim]
  int64_t n;
  int32_t in_dim, K1, HP, R, G, N, L1;
  uint32_t g;        // global step of the draws
  const u32x4 *w1f;  // [2 HP][K1][64] fragments of W1^T
  const float *b1;   // [32 HP]
  const u32x4 *w2f;  // [G][R][HP][64] fragments of W2^T
  const float *b2f;  // [G][R][16]
  uint8_t *act;      // [n][N] or NULL
  float *logits;     // [n][N * L1] or NULL
  uint64_t seed;
  int64_t env0;      // Philox index of env 0
};

// Host-side launchers (defined in cx_kernels.hip).  `a.segs` is the base of
// the device segment table; each group launches with its own slice.
hipError_t launch_groups(const LaunchArgs &a, const LaunchGroup *groups, int n_groups, hipStream_t st);
hipError_t launch_policy_rollout(const LaunchArgs &a, int per_lane, int n_blocks, size_t lds, hipStream_t st);
hipError_t graph_rollout(RolloutGraph &g, const LaunchArgs &a, const LaunchGroup *groups, int n_groups,
                         hipStream_t st);
void graph_destroy(RolloutGraph &g);
hipError_t launch_reset_obs_one(const ClassDev *cls_dev, int64_t n_envs, float *obs, uint64_t seed, int64_t env0,
                                uint32_t g, hipStream_t st);
// Sets n doubles at p to v (battery SoC at the start of a day).
hipError_t launch_fill_f64(double *p, int64_t n, double v, hipStream_t st);

}  // namespace cx
