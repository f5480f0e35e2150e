// cx_policy.hip -- policy-in-the-loop rollouts.
//   k_policy  obs -> BF16 -> W1 (tanh) -> W2 -> logits on the matrix cores
//             (v_mfma_f32_16x16x32_bf16, FP32 accumulation), then per port a
//             level drawn from softmax of its logits with one Philox uniform.
// A rollout of a SIMPLE class of 8, 16 or 32 slots is one launch of the fused
// persistent kernel (the rollout kernel with this MLP between its steps,
// cx_kernels.hip): state in registers, observations only in LDS.  Other
// classes, and the rollout that allocates nothing, run two kernels per step:
// k_policy, then the one-step environment kernel with its levels as external
// actions, which writes the next observation.  k_observe gives the
// observation of the state a rollout starts from.
//
// The layout of the two products is described in cx_mlp.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <vector>

#include "cx_ctx.h"
#include "cx_device.h"
#include "cx_mlp.h"

namespace cx {

constexpr int kPolNT = 2;  // 16-env column tiles per wave
constexpr int kPolWaves = 8;  // waves per block sharing each staged weight chunk

struct PolicyRt {
  int hidden = 0, in_dim = 0, N = 0, L1 = 0;
  int K1 = 0, HP = 0, R = 0, G = 0;
  void *mem = nullptr;  // weights in fragment order + FP32 biases
  const u32x4 *w1f = nullptr;
  const float *b1 = nullptr;
  const u32x4 *w2f = nullptr;
  const float *b2f = nullptr;
  // the same weights padded to the largest sizes (zeros), for the fused
  // rollout: W1^T [16 tiles][8 K-steps][64], b1 [256], W2^T [G][3][8][64],
  // b2 [G][3][16]
  const u32x4 *w1p = nullptr;
  const float *b1p = nullptr;
  const u32x4 *w2p = nullptr;
  const float *b2p = nullptr;
  float *obs = nullptr;  // one step of observations (rollouts that do not return them)
  uint8_t *act = nullptr;  // one step of levels (rollouts that do not return them)
  int64_t scratch_envs = 0;
  // the fused rollout's segment table (stations of 8 lanes, 4 waves per block)
  SegDev *segs_dev = nullptr;
  int n_segs = 0, n_blocks = 0;
};

namespace {

// Weight chunks pass through LDS, double-buffered: chunk c < HP holds the two
// W1^T tiles of hidden units 32c..32c+31 (all K-steps), chunk HP + g the R
// tiles of W2^T of port group g.  Every wave of the block reads each chunk, so
// a weight byte leaves L2 once per 16 * kPolNT * kPolWaves envs.
constexpr int kChunkMax = 3 * kPolHP * 64;  // u32x4 per chunk (R * HP or 2 * K1 tiles of 64 lanes)
constexpr int kPerThread = kChunkMax / (64 * kPolWaves);

__device__ __forceinline__ void chunk_src(const PolicyArgs &a, int c, const u32x4 *&src, int &cnt) {
  if (c < a.HP) {
    src = a.w1f + (int64_t)(2 * c) * a.K1 * 64;
    cnt = 2 * a.K1 * 64;
  } else {
    src = a.w2f + (int64_t)(c - a.HP) * a.R * a.HP * 64;
    cnt = a.R * a.HP * 64;
  }
}

__device__ __forceinline__ void fetch_chunk(const PolicyArgs &a, int c, u32x4 (&r)[kPerThread]) {
  const u32x4 *src;
  int cnt;
  chunk_src(a, c, src, cnt);
#pragma unroll
  for (int i = 0; i < kPerThread; ++i) {
    const int idx = (int)threadIdx.x + i * 64 * kPolWaves;
    if (idx < cnt) r[i] = gld(src, idx);
  }
}

__device__ __forceinline__ void put_chunk(const PolicyArgs &a, int c, const u32x4 (&r)[kPerThread], u32x4 *buf) {
  const u32x4 *src;
  int cnt;
  chunk_src(a, c, src, cnt);
#pragma unroll
  for (int i = 0; i < kPerThread; ++i) {
    const int idx = (int)threadIdx.x + i * 64 * kPolWaves;
    if (idx < cnt) buf[idx] = r[i];
  }
}

__global__ __launch_bounds__(64 * kPolWaves) void k_policy(PolicyArgs a) {
  __shared__ u32x4 wbuf[2][kChunkMax];
  const int lane = __lane_id();
  const int col = lane & 15, lg = lane >> 4;
  const int64_t wave = (int64_t)blockIdx.x * kPolWaves + (threadIdx.x >> 6);
  const int64_t e_base = wave * 16 * kPolNT;  // waves past the end still take part in the barriers
  const int n_chunks = a.HP + a.G;
  u32x4 pf[kPerThread];
  fetch_chunk(a, 0, pf);
  put_chunk(a, 0, pf, wbuf[0]);

  // ---- B operand of the first product: 8 consecutive features of one env
  u32x4 ob[kPolK1][kPolNT];
#pragma unroll
  for (int s = 0; s < kPolK1; ++s) {
#pragma unroll
    for (int n = 0; n < kPolNT; ++n) {
      u32x4 v = {0u, 0u, 0u, 0u};
      const int64_t e = e_base + 16 * n + col;
      const int f = 32 * s + 8 * lg;
      if (s < a.K1 && e < a.n && f < a.in_dim) {
        const float *row = a.obs + e * a.in_dim + f;
        typedef float f4 __attribute__((ext_vector_type(4)));
        const f4 x = gld(reinterpret_cast<const f4 *>(row), 0);
        f4 y = {0.f, 0.f, 0.f, 0.f};
        if (f + 4 < a.in_dim) y = gld(reinterpret_cast<const f4 *>(row + 4), 0);
        v = u32x4{pack2(x.x, x.y), pack2(x.z, x.w), pack2(y.x, y.y), pack2(y.z, y.w)};
      }
      ob[s][n] = v;
    }
  }
  __syncthreads();

  // ---- first product, 32 hidden units (two 16-row tiles, one chunk) at a time
  u32x4 h[kPolHP][kPolNT];
#pragma unroll
  for (int mp = 0; mp < kPolHP; ++mp) {
#pragma unroll
    for (int n = 0; n < kPolNT; ++n) h[mp][n] = u32x4{0u, 0u, 0u, 0u};
    if (mp < a.HP) {
      if (mp + 1 < n_chunks) fetch_chunk(a, mp + 1, pf);
      const u32x4 *w = wbuf[mp & 1];
      f32x4 c0[kPolNT], c1[kPolNT];
#pragma unroll
      for (int n = 0; n < kPolNT; ++n) {
        c0[n] = f32x4{0.f, 0.f, 0.f, 0.f};
        c1[n] = f32x4{0.f, 0.f, 0.f, 0.f};
      }
#pragma unroll
      for (int s = 0; s < kPolK1; ++s) {
        if (s < a.K1) {
          const u32x4 a0 = w[s * 64 + lane];
          const u32x4 a1 = w[(a.K1 + s) * 64 + lane];
#pragma unroll
          for (int n = 0; n < kPolNT; ++n) {
            c0[n] = mfma_bf16(a0, ob[s][n], c0[n]);
            c1[n] = mfma_bf16(a1, ob[s][n], c1[n]);
          }
        }
      }
      if (mp + 1 < n_chunks) put_chunk(a, mp + 1, pf, wbuf[(mp + 1) & 1]);
      const f32x4 bA = gld(reinterpret_cast<const f32x4 *>(a.b1 + 32 * mp + 4 * lg), 0);
      const f32x4 bB = gld(reinterpret_cast<const f32x4 *>(a.b1 + 32 * mp + 16 + 4 * lg), 0);
#pragma unroll
      for (int n = 0; n < kPolNT; ++n) h[mp][n] = hidden_frag(c0[n], c1[n], bA, bB);
      __syncthreads();
    }
  }

  // ---- second product per group of 4 ports (one chunk each), then a level
  // per port drawn from softmax of its logits
  const uint32_t k0 = (uint32_t)a.seed, k1 = (uint32_t)(a.seed >> 32);
  const int out_dim = a.N * a.L1;
  for (int grp = 0; grp < a.G; ++grp) {
    const int cidx = a.HP + grp;
    const int port = 4 * grp + lg;
    if (cidx + 1 < n_chunks) fetch_chunk(a, cidx + 1, pf);
    // the uniform of this port's draw: independent of the products, so it is
    // computed in the same straight-line block as the matrix-core work and the
    // two overlap (lanes past the last env or port compute unused draws)
    float ud[kPolNT];
#pragma unroll
    for (int n = 0; n < kPolNT; ++n) {
      const uint32_t env_id = (uint32_t)(a.env0 + e_base + 16 * n + col);
      const U4 w = philox(env_id, a.g, draw_index(port), kDomGum, k0, k1);
      ud[n] = draw_uniform(draw_word(w, port));
    }
    const u32x4 *w = wbuf[cidx & 1];
    f32x4 c[kPolR][kPolNT];
#pragma unroll
    for (int r = 0; r < kPolR; ++r) {
      f32x4 b = {0.f, 0.f, 0.f, 0.f};
      if (r < a.R) b = gld(reinterpret_cast<const f32x4 *>(a.b2f + (int64_t)(grp * a.R + r) * 16 + 4 * lg), 0);
#pragma unroll
      for (int n = 0; n < kPolNT; ++n) c[r][n] = b;
    }
#pragma unroll
    for (int s = 0; s < kPolHP; ++s) {
      if (s < a.HP) {
#pragma unroll
        for (int r = 0; r < kPolR; ++r) {
          if (r < a.R) {
            const u32x4 wf = w[(r * a.HP + s) * 64 + lane];
#pragma unroll
            for (int n = 0; n < kPolNT; ++n) c[r][n] = mfma_bf16(wf, h[s][n], c[r][n]);
          }
        }
      }
    }
    if (cidx + 1 < n_chunks) put_chunk(a, cidx + 1, pf, wbuf[(cidx + 1) & 1]);
    __syncthreads();
#pragma unroll
    for (int n = 0; n < kPolNT; ++n) {
      const int64_t e = e_base + 16 * n + col;
      if (port >= a.N || e >= a.n) continue;
      if (a.logits) {
        float *z = a.logits + e * out_dim + (int64_t)port * a.L1;
#pragma unroll
        for (int r = 0; r < kPolR; ++r) {
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int lev = 4 * r + i;
            if (r < a.R && lev < a.L1) z[lev] = c[r][n][i];
          }
        }
      }
      if (a.act) {
        const f32x4 cn[kPolR] = {c[0][n], c[1][n], c[2][n]};
        const int lev = sample_level(cn, a.R, a.L1, ud[n]);
        a.act[e * a.N + port] = (uint8_t)lev;
      }
    }
  }
}

// Observation of the current state (the features the step kernel records).
__global__ void k_observe(const ClassDev *cls, int64_t n_envs, const double *q, const float *u,
                          const float *p_last, const int16_t *dwell, const uint8_t *utype, const double *bsoc,
                          const float *bp, const float *rbar, int32_t t_day, uint64_t seed, int64_t env0, uint32_t g,
                          float *obs) {
  const ClassDev C = *cls;
  const int S = C.S, N = C.n_ports, dim = C.obs_dim;
  const int64_t total = n_envs * S;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t env = i / S;
    const int s = (int)(i - env * S);
    const int port = C.slot_port[s];
    if (port < 0) continue;
    const int dw = dwell[i];
    const bool cs = C.has_users && utype[i] != 0;
    const bool occ = dw > 0 || cs;
    const float qf = (float)q[i];
    float *o = obs + env * dim + port;
    o[0 * N] = occ ? 1.0f : 0.0f;
    o[1 * N] = occ ? 1.0f - qf : 0.0f;
    o[2 * N] = occ ? qf - u[i] : 0.0f;
    o[3 * N] = (float)dw * C.inv_steps_ep;
    float rh = fminf(1.0f, qf * C.inv_1mtau);
    if (C.n_models > 0) rh *= rbar[i] * C.slot_inv_pmax[s];  // the car's curve, as a share of the port maximum
    o[4 * N] = occ ? rh : 0.0f;
    o[5 * N] = p_last[i] * C.slot_inv_pmax[s];
    if (C.has_users) obs[env * dim + C.user_obs + port] = cs ? 1.0f : 0.0f;
  }
  for (int64_t env = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; env < n_envs;
       env += (int64_t)gridDim.x * blockDim.x) {
    int n_occ = 0;
    for (int s = 0; s < S; ++s)
      n_occ += (dwell[env * S + s] > 0 || (C.has_users && utype[env * S + s] != 0)) ? 1 : 0;
    float *o = obs + env * dim + 6 * N;
    o[0] = C.glob[t_day * 4 + 0];
    o[1] = C.glob[t_day * 4 + 1];
    o[2] = C.glob[t_day * 4 + 2];
    o[3] = (float)n_occ * (1.0f / (float)N);
    if (C.has_batt) {
      o[4] = (float)bsoc[env];
      o[5] = bp[env] * C.b_inv_rate;
    }
    if (C.n_days > 0) {  // the episode's price day, drawn at the step it began
      const int d = episode_day((uint32_t)(env0 + env), g - (uint32_t)t_day, (uint32_t)seed, (uint32_t)(seed >> 32),
                                C.n_days);
      o[2] = C.price_days[(int64_t)d * C.steps_ep + t_day];
      obs[env * dim + C.day_obs] = (float)d * C.inv_n_days;
      obs[env * dim + C.day_obs + 1] = d % 7 >= 5 ? 1.0f : 0.0f;
    }
  }
}

hipError_t launch_policy(const PolicyArgs &a, hipStream_t st) {
  const int64_t waves = (a.n + 16 * kPolNT - 1) / (16 * kPolNT);
  const int64_t blocks = (waves + kPolWaves - 1) / kPolWaves;
  if (blocks == 0) return hipSuccess;
  hipLaunchKernelGGL(k_policy, dim3((unsigned)blocks), dim3(64 * kPolWaves), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_observe(const cx_ctx *ctx, float *obs, hipStream_t st) {
  for (const ClassRt &c : ctx->classes) {
    if (c.n_envs == 0) continue;
    const int64_t work = c.n_envs * c.comp.S;
    const int blocks = (int)std::min<int64_t>(4096, (work + 255) / 256);
    hipLaunchKernelGGL(k_observe, dim3(blocks), dim3(256), 0, st, c.dev, c.n_envs, ctx->q + c.slot_off,
                       ctx->u + c.slot_off, ctx->p_last + c.slot_off, ctx->dwell + c.slot_off,
                       ctx->utype + c.slot_off, ctx->bsoc + c.env_begin, ctx->bp + c.env_begin,
                       ctx->rbar + c.slot_off, ctx->t_day, ctx->seed, c.env_begin, ctx->g, obs + c.obs_off);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

PolicyArgs policy_args(const cx_ctx *ctx, const float *obs, int64_t n) {
  const PolicyRt &p = *ctx->policy;
  PolicyArgs a{};
  a.obs = obs;
  a.n = n;
  a.in_dim = p.in_dim; a.K1 = p.K1; a.HP = p.HP; a.R = p.R; a.G = p.G; a.N = p.N; a.L1 = p.L1;
  a.w1f = p.w1f; a.b1 = p.b1; a.w2f = p.w2f; a.b2f = p.b2f;
  a.seed = ctx->seed;
  a.env0 = ctx->classes[0].env_begin;
  return a;
}

double bf16_to_double(uint16_t b) {
  const uint32_t u = (uint32_t)b << 16;
  float f;
  std::memcpy(&f, &u, 4);
  return f;
}

cx_status ensure_scratch(cx_ctx *ctx) {
  PolicyRt &p = *ctx->policy;
  if (p.scratch_envs >= ctx->n_envs) return CX_OK;
  if (p.obs) (void)hipFree(p.obs);
  if (p.act) (void)hipFree(p.act);
  p.obs = nullptr;
  p.act = nullptr;
  p.scratch_envs = 0;
  if (hipMalloc(&p.obs, sizeof(float) * ctx->obs_elems) != hipSuccess ||
      hipMalloc(&p.act, (size_t)ctx->total_ports) != hipSuccess)
    return fail_status(CX_E_OOM, "policy rollout: scratch allocation failed");
  p.scratch_envs = ctx->n_envs;
  return CX_OK;
}

}  // namespace

void free_policy(cx_ctx *ctx) {
  if (!ctx || !ctx->policy) return;
  PolicyRt *p = ctx->policy;
  if (p->mem) (void)hipFree(p->mem);
  if (p->segs_dev) (void)hipFree(p->segs_dev);
  if (p->obs) (void)hipFree(p->obs);
  if (p->act) (void)hipFree(p->act);
  delete p;
  ctx->policy = nullptr;
}

namespace {

// One policy rollout with the given scratch: obs_scr one step of observations
// (obs_elems floats), act_scr one step of levels (total_ports bytes).  Every
// element of both is written before it is read, so their contents on entry do
// not matter.
cx_status policy_step_with(cx_ctx *ctx, int32_t T, cx_out_mode out_mode, const cx_traj *out, float *obs_scr,
                           uint8_t *act_scr) {
  const bool ret_obs = out && out_mode == CX_OUT_FULL && out->obs;
  const bool ret_act = out && out_mode != CX_OUT_REWARD && out->actions;
  if (ret_obs && (reinterpret_cast<uintptr_t>(out->obs) & 15u) != 0)
    return fail_status(CX_E_INVALID, "policy rollout: obs buffer must be 16-byte aligned");
  hipError_t e = launch_observe(ctx, obs_scr, ctx->stream);
  if (e != hipSuccess) return hip_fail(ctx, e, "policy rollout: observation kernel");
  const float *obs_prev = obs_scr;
  for (int32_t t = 0; t < T; ++t) {
    float *obs_t = ret_obs ? out->obs + (int64_t)t * ctx->obs_elems : obs_scr;
    uint8_t *act_t = ret_act ? out->actions + (int64_t)t * ctx->total_ports : act_scr;
    PolicyArgs pa = policy_args(ctx, obs_prev, ctx->n_envs);
    pa.g = ctx->g + (uint32_t)t;
    pa.act = act_t;
    if ((e = launch_policy(pa, ctx->stream)) != hipSuccess) return hip_fail(ctx, e, "policy kernel");
    LaunchArgs a = base_args(ctx);
    a.T = 1;
    a.g0 = ctx->g + (uint32_t)t;
    a.t_day0 = (int32_t)(((int64_t)ctx->t_day + t) % ctx->steps_ep);
    a.mode = CX_ACT_EXTERNAL;
    a.out_mode = CX_OUT_FULL;
    a.act_in = act_t;
    a.obs = obs_t;
    a.act = nullptr;
    a.reward = out && out->reward ? out->reward + (int64_t)t * ctx->n_envs : nullptr;
    a.done = out && out->done ? out->done + (int64_t)t * ctx->n_envs : nullptr;
    if ((e = launch_groups(a, ctx->groups.data(), (int)ctx->groups.size(), ctx->stream)) !=
        hipSuccess)
      return hip_fail(ctx, e, "policy rollout: step kernel");
    obs_prev = obs_t;
  }
  // the next rollout starts from the observation kernel again (it does not
  // read obs_prev), so the clock is the only state carried here
  advance_clock(ctx, T);
  return CX_OK;
}

}  // namespace

// Scratch of the rollout that allocates nothing (cx_rollout_policy_noalloc):
// a fixed array of the device image, one per GPU the library runs on, held
// until the process ends.  In host code its name is only a stand-in for the
// device array: the address kernels take is looked up per device.
constexpr size_t kNoAllocScratchBytes = (size_t)CX_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// The device address of `scratch` on `device`, looked up on the first call for
// that device with the device current (each GPU has its own copy).
cx_status noalloc_scratch(int device, unsigned char **ptr) {
  if (device < 0 || device >= kMaxDevices) return fail_status(CX_E_INVALID, "device index out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return fail_status(CX_E_DEVICE, std::string("hipGetDevice: ") + hipGetErrorString(e));
    if (cur != device && (e = hipSetDevice(device)) != hipSuccess)
      return fail_status(CX_E_DEVICE, std::string("hipSetDevice: ") + hipGetErrorString(e));
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur != device) (void)hipSetDevice(cur);
    if (e != hipSuccess || !p)
      return fail_status(CX_E_DEVICE, std::string("hipGetSymbolAddress of the no-allocation scratch: ") +
                                          hipGetErrorString(e));
    g_scratch_ptr[device] = p;
  }
  *ptr = static_cast<unsigned char *>(g_scratch_ptr[device]);
  return CX_OK;
}

}  // namespace

namespace {

// The fused rollout runs SIMPLE classes of 8, 16 or 32 slots (stations of 8
// lanes, 1, 2 or 4 slots per lane); others take the two kernels per step.
bool fused_eligible(const cx_ctx *ctx) {
  const ClassRt &c = ctx->classes[0];
  const int S = c.comp.S;
  return c.host_view.kind == kKindSimple && (S == 8 || S == 16 || S == 32);
}

cx_status ensure_fused(cx_ctx *ctx) {
  PolicyRt &p = *ctx->policy;
  if (p.segs_dev) return CX_OK;
  const ClassRt &c = ctx->classes[0];
  std::vector<SegDev> segs;
  class_segments(ctx, c, 8, c.comp.S / 8, &segs);
  int blocks = 0;
  for (SegDev &sg : segs) {
    sg.block_begin = blocks;
    blocks += (sg.n_groups + kPolRolloutWaves - 1) / kPolRolloutWaves;
  }
  void *d = nullptr;
  if (hipMalloc(&d, sizeof(SegDev) * std::max<size_t>(1, segs.size())) != hipSuccess)
    return fail_status(CX_E_OOM, "policy rollout: segment table allocation failed");
  hipError_t e = hipMemcpy(d, segs.data(), sizeof(SegDev) * segs.size(), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    (void)hipFree(d);
    return hip_fail(ctx, e, "policy rollout: segment table upload");
  }
  p.segs_dev = static_cast<SegDev *>(d);
  p.n_segs = (int)segs.size();
  p.n_blocks = blocks;
  return CX_OK;
}

// One launch for the whole rollout: the observation the rollout starts from
// (into the scratch), then the persistent kernel with the MLP between steps.
cx_status fused_rollout(cx_ctx *ctx, int32_t T, cx_out_mode out_mode, const cx_traj *out, size_t lds,
                        const LaunchArgs::Pol &lay) {
  PolicyRt &p = *ctx->policy;
  const ClassRt &c = ctx->classes[0];
  const bool ret_obs = out && out_mode == CX_OUT_FULL && out->obs;
  const bool ret_act = out && out_mode != CX_OUT_REWARD && out->actions;
  hipError_t e = launch_observe(ctx, p.obs, ctx->stream);
  if (e != hipSuccess) return hip_fail(ctx, e, "policy rollout: observation kernel");
  LaunchArgs a = base_args(ctx);
  a.segs = p.segs_dev;
  a.n_segs = p.n_segs;
  a.T = T;
  a.mode = CX_ACT_POLICY;
  a.out_mode = out_mode;
  a.obs = ret_obs ? out->obs : nullptr;
  a.act = ret_act ? out->actions : nullptr;
  a.reward = out ? out->reward : nullptr;
  a.done = out ? out->done : nullptr;
  a.lds_tdwell = 1;
  a.stage_off = lay.hb_off;
  a.stage_floats = (int32_t)(((size_t)kPolRolloutEnvs * c.comp.obs_dim + 3) & ~(size_t)3);
  a.pol = lay;
  a.pol.obs0 = p.obs;
  a.pol.w1f = p.w1p;
  a.pol.b1 = p.b1p;
  a.pol.w2f = p.w2p;
  a.pol.b2f = p.b2p;
  a.pol.in_dim = p.in_dim;
  a.pol.K1 = p.K1;
  a.pol.HP = p.HP;
  a.pol.R = p.R;
  a.pol.G = p.G;
  a.pol.L1 = p.L1;
  if ((e = launch_policy_rollout(a, c.comp.S / 8, p.n_blocks, lds, ctx->stream)) != hipSuccess)
    return hip_fail(ctx, e, "policy rollout kernel");
  advance_clock(ctx, T);
  return CX_OK;
}

}  // namespace

cx_status policy_step(cx_ctx *ctx, int32_t T, cx_out_mode out_mode, const cx_traj *out, bool graph) {
  (void)graph;
  if (!ctx->policy) return fail_status(CX_E_INVALID, "no policy set (cx_set_policy)");
  cx_status st = ensure_scratch(ctx);
  if (st != CX_OK) return st;
  if (fused_eligible(ctx)) {
    const bool ret_obs = out && out_mode == CX_OUT_FULL && out->obs;
    if (ret_obs && (reinterpret_cast<uintptr_t>(out->obs) & 15u) != 0)
      return fail_status(CX_E_INVALID, "policy rollout: obs buffer must be 16-byte aligned");
    const ClassRt &c = ctx->classes[0];
    LaunchArgs::Pol lay{};
    int32_t stage_off = 0, stage_floats = 0;
    const size_t lds = policy_rollout_lds(c.tab.dwell_log2, c.comp.obs_dim, c.comp.N, &stage_off,
                                          &stage_floats, &lay.hb_off, &lay.xb_off, &lay.act_off);
    if (lds <= kMaxBlockLds) {
      if (T == 0) return CX_OK;
      if ((st = ensure_fused(ctx)) != CX_OK) return st;
      return fused_rollout(ctx, T, out_mode, out, lds, lay);
    }
  }
  return policy_step_with(ctx, T, out_mode, out, ctx->policy->obs, ctx->policy->act);
}

}  // namespace cx

using namespace cx;

extern "C" {

cx_status cx_set_policy(cx_ctx *ctx, int32_t hidden, const uint16_t *w1, const uint16_t *b1,
                        const uint16_t *w2, const uint16_t *b2) {
  if (!ctx) return fail_status(CX_E_INVALID, "context is NULL");
  if (ctx->failed) return fail_status(CX_E_DEVICE, "context has a sticky device error");
  if (!w1 || !b1 || !w2 || !b2) return fail_status(CX_E_INVALID, "cx_set_policy: NULL weight array");
  if (ctx->classes.size() != 1) return fail_status(CX_E_INVALID, "cx_set_policy: single-class contexts only");
  const ClassRt &c = ctx->classes[0];
  if (c.comp.extended())
    return fail_status(CX_E_INVALID, "cx_set_policy: charging-only stations only (no V2G, no battery)");
  const int N = c.comp.N, L1 = c.spec.s.n_levels + 1, in_dim = 6 * N + 4;
  if (hidden < 32 || hidden > 32 * kPolHP || hidden % 32 != 0)
    return fail_status(CX_E_INVALID, "cx_set_policy: hidden must be a multiple of 32 in 32..256");
  if (in_dim > 32 * kPolK1)
    return fail_status(CX_E_INVALID, "cx_set_policy: observations longer than 256 (more than 42 ports)");
  if (L1 > 4 * kPolR) return fail_status(CX_E_INVALID, "cx_set_policy: at most 11 levels per port");
  const int K1 = (in_dim + 31) / 32, HP = hidden / 32, R = (L1 + 3) / 4, G = (N + 3) / 4;
  const int out_dim = N * L1;
  // W1^T fragments: tile m (hidden 16m..16m+15), K-step s, lane l -> hidden
  // 16m + l % 16, features 32s + 8 (l / 16) + j
  std::vector<uint16_t> w1f((size_t)2 * HP * K1 * 64 * 8, 0);
  for (int m = 0; m < 2 * HP; ++m)
    for (int s = 0; s < K1; ++s)
      for (int l = 0; l < 64; ++l)
        for (int j = 0; j < 8; ++j) {
          const int f = 32 * s + 8 * (l >> 4) + j, hu = 16 * m + (l & 15);
          if (f < in_dim) w1f[(((size_t)m * K1 + s) * 64 + l) * 8 + j] = w1[(size_t)f * hidden + hu];
        }
  std::vector<float> b1f(hidden);
  for (int j = 0; j < hidden; ++j) b1f[j] = (float)bf16_to_double(b1[j]);
  // W2^T fragments: tile (grp, r), K-step s, lane l -> row l % 16 = port
  // 4 grp + (l % 16) / 4, level 4 r + l % 4; slot j -> hidden unit in the
  // order the first product leaves them in a lane
  std::vector<uint16_t> w2f((size_t)G * R * HP * 64 * 8, 0);
  std::vector<float> b2f((size_t)G * R * 16, 0.f);
  for (int grp = 0; grp < G; ++grp)
    for (int r = 0; r < R; ++r) {
      const int tile = grp * R + r;
      for (int row = 0; row < 16; ++row) {
        const int port = 4 * grp + (row >> 2), lev = 4 * r + (row & 3);
        if (port < N && lev < L1) b2f[(size_t)tile * 16 + row] = (float)bf16_to_double(b2[port * L1 + lev]);
      }
      for (int s = 0; s < HP; ++s)
        for (int l = 0; l < 64; ++l) {
          const int row = l & 15, q = l >> 4;
          const int port = 4 * grp + (row >> 2), lev = 4 * r + (row & 3);
          if (port >= N || lev >= L1) continue;
          const int o = port * L1 + lev;
          for (int j = 0; j < 8; ++j) {
            const int hu = 32 * s + (j < 4 ? 4 * q + j : 16 + 4 * q + (j - 4));
            w2f[((((size_t)tile * HP + s) * 64 + l) * 8) + j] = w2[(size_t)hu * out_dim + o];
          }
        }
    }
  // padded copies: W1^T tile m, K-step s at (m * 8 + s); W2^T tile (grp, r),
  // K-step s at ((grp * 3 + r) * 8 + s)
  std::vector<uint16_t> w1p((size_t)2 * kPolHP * kPolK1 * 64 * 8, 0);
  for (int m = 0; m < 2 * HP; ++m)
    for (int s = 0; s < K1; ++s)
      std::memcpy(&w1p[((size_t)m * kPolK1 + s) * 64 * 8], &w1f[((size_t)m * K1 + s) * 64 * 8], 64 * 8 * 2);
  std::vector<float> b1p((size_t)32 * kPolHP, 0.f);
  std::memcpy(b1p.data(), b1f.data(), (size_t)hidden * 4);
  std::vector<uint16_t> w2p((size_t)G * kPolR * kPolHP * 64 * 8, 0);
  std::vector<float> b2p((size_t)G * kPolR * 16, 0.f);
  for (int grp = 0; grp < G; ++grp)
    for (int r = 0; r < R; ++r) {
      std::memcpy(&b2p[((size_t)grp * kPolR + r) * 16], &b2f[((size_t)grp * R + r) * 16], 16 * 4);
      for (int s = 0; s < HP; ++s)
        std::memcpy(&w2p[(((size_t)grp * kPolR + r) * kPolHP + s) * 64 * 8],
                    &w2f[(((size_t)grp * R + r) * HP + s) * 64 * 8], 64 * 8 * 2);
    }
  const size_t s_w1 = w1f.size() * 2, s_b1 = (size_t)hidden * 4, s_w2 = w2f.size() * 2, s_b2 = b2f.size() * 4;
  const size_t s_w1p = w1p.size() * 2, s_b1p = b1p.size() * 4, s_w2p = w2p.size() * 2, s_b2p = b2p.size() * 4;
  auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
  const size_t o_w1p = al(s_w1) + al(s_b1) + al(s_w2) + al(s_b2);
  const size_t o_b1p = o_w1p + al(s_w1p), o_w2p = o_b1p + al(s_b1p), o_b2p = o_w2p + al(s_w2p);
  const size_t bytes = o_b2p + al(s_b2p);
  void *mem = nullptr;
  if (hipMalloc(&mem, bytes) != hipSuccess) return fail_status(CX_E_OOM, "cx_set_policy: hipMalloc failed");
  unsigned char *b = static_cast<unsigned char *>(mem);
  hipError_t e;
  if ((e = hipMemcpy(b, w1f.data(), s_w1, hipMemcpyHostToDevice)) != hipSuccess ||
      (e = hipMemcpy(b + al(s_w1), b1f.data(), s_b1, hipMemcpyHostToDevice)) != hipSuccess ||
      (e = hipMemcpy(b + al(s_w1) + al(s_b1), w2f.data(), s_w2, hipMemcpyHostToDevice)) != hipSuccess ||
      (e = hipMemcpy(b + al(s_w1) + al(s_b1) + al(s_w2), b2f.data(), s_b2, hipMemcpyHostToDevice)) != hipSuccess ||
      (e = hipMemcpy(b + o_w1p, w1p.data(), s_w1p, hipMemcpyHostToDevice)) != hipSuccess ||
      (e = hipMemcpy(b + o_b1p, b1p.data(), s_b1p, hipMemcpyHostToDevice)) != hipSuccess ||
      (e = hipMemcpy(b + o_w2p, w2p.data(), s_w2p, hipMemcpyHostToDevice)) != hipSuccess ||
      (e = hipMemcpy(b + o_b2p, b2p.data(), s_b2p, hipMemcpyHostToDevice)) != hipSuccess) {
    (void)hipFree(mem);
    return hip_fail(ctx, e, "cx_set_policy upload");
  }
  // replacing a policy waits for work that may still read the old weights
  if ((e = hipStreamSynchronize(ctx->stream)) != hipSuccess) {
    (void)hipFree(mem);
    return hip_fail(ctx, e, "cx_set_policy synchronize");
  }
  PolicyRt *old = ctx->policy;
  PolicyRt *p = new PolicyRt();
  p->hidden = hidden; p->in_dim = in_dim; p->N = N; p->L1 = L1;
  p->K1 = K1; p->HP = HP; p->R = R; p->G = G;
  p->mem = mem;
  p->w1f = reinterpret_cast<const u32x4 *>(b);
  p->b1 = reinterpret_cast<const float *>(b + al(s_w1));
  p->w2f = reinterpret_cast<const u32x4 *>(b + al(s_w1) + al(s_b1));
  p->b2f = reinterpret_cast<const float *>(b + al(s_w1) + al(s_b1) + al(s_w2));
  p->w1p = reinterpret_cast<const u32x4 *>(b + o_w1p);
  p->b1p = reinterpret_cast<const float *>(b + o_b1p);
  p->w2p = reinterpret_cast<const u32x4 *>(b + o_w2p);
  p->b2p = reinterpret_cast<const float *>(b + o_b2p);
  if (old) {  // keep the scratch buffers
    p->obs = old->obs; p->act = old->act; p->scratch_envs = old->scratch_envs;
    old->obs = nullptr; old->act = nullptr;
    ctx->policy = old;
    free_policy(ctx);
  }
  ctx->policy = p;
  return CX_OK;
}

cx_status cx_policy_logits(cx_ctx *ctx, const float *obs_dev, int64_t n, float *logits_dev) {
  if (!ctx) return fail_status(CX_E_INVALID, "context is NULL");
  if (ctx->failed) return fail_status(CX_E_DEVICE, "context has a sticky device error");
  if (!ctx->policy) return fail_status(CX_E_INVALID, "no policy set (cx_set_policy)");
  if (n < 0) return fail_status(CX_E_INVALID, "cx_policy_logits: n < 0");
  if (n > 0 && (!obs_dev || !logits_dev)) return fail_status(CX_E_INVALID, "cx_policy_logits: NULL buffer");
  if (n > 0 && (reinterpret_cast<uintptr_t>(obs_dev) & 15u) != 0)
    return fail_status(CX_E_INVALID, "cx_policy_logits: obs_dev must be 16-byte aligned");
  if (n == 0) return CX_OK;
  PolicyArgs a = policy_args(ctx, obs_dev, n);
  a.logits = logits_dev;
  hipError_t e = launch_policy(a, ctx->stream);
  if (e != hipSuccess) return hip_fail(ctx, e, "cx_policy_logits launch");
  return CX_OK;
}

cx_status cx_policy_sample(cx_ctx *ctx, const float *obs_dev, int64_t n, uint32_t g, uint8_t *act_dev) {
  if (!ctx) return fail_status(CX_E_INVALID, "context is NULL");
  if (ctx->failed) return fail_status(CX_E_DEVICE, "context has a sticky device error");
  if (!ctx->policy) return fail_status(CX_E_INVALID, "no policy set (cx_set_policy)");
  if (n < 0) return fail_status(CX_E_INVALID, "cx_policy_sample: n < 0");
  if (n > 0 && (!obs_dev || !act_dev)) return fail_status(CX_E_INVALID, "cx_policy_sample: NULL buffer");
  if (n > 0 && (reinterpret_cast<uintptr_t>(obs_dev) & 15u) != 0)
    return fail_status(CX_E_INVALID, "cx_policy_sample: obs_dev must be 16-byte aligned");
  if (n == 0) return CX_OK;
  PolicyArgs a = policy_args(ctx, obs_dev, n);
  a.g = g;
  a.act = act_dev;
  hipError_t e = launch_policy(a, ctx->stream);
  if (e != hipSuccess) return hip_fail(ctx, e, "cx_policy_sample launch");
  return CX_OK;
}

cx_status cx_rollout_policy_noalloc(cx_ctx *ctx, int32_t T, cx_out_mode out_mode, const cx_traj *out) {
  if (!ctx) return fail_status(CX_E_INVALID, "context is NULL");
  if (ctx->failed) return fail_status(CX_E_DEVICE, "context has a sticky device error");
  if (T < 0 || T > (1 << 24)) return fail_status(CX_E_INVALID, "T must be in 0..2^24");
  if (out_mode < CX_OUT_FULL || out_mode > CX_OUT_ACT_REWARD) return fail_status(CX_E_INVALID, "bad out mode");
  if (!ctx->policy) return fail_status(CX_E_INVALID, "no policy set (cx_set_policy)");
  // one step of observations (16-byte aligned for the policy kernel), then one of levels
  const size_t obs_bytes = ((size_t)ctx->obs_elems * sizeof(float) + 255) & ~(size_t)255;
  const size_t need = obs_bytes + (size_t)ctx->total_ports;
  if (need > kNoAllocScratchBytes)
    return fail_status(CX_E_INVALID, "cx_rollout_policy_noalloc: the context needs " + std::to_string(need) +
                                         " bytes of scratch per step, more than the fixed " +
                                         std::to_string(kNoAllocScratchBytes) + " bytes");
  if (T == 0) return CX_OK;
  unsigned char *base = nullptr;
  cx_status st = noalloc_scratch(ctx->device, &base);
  if (st != CX_OK) return st;
  return policy_step_with(ctx, T, out_mode, out, reinterpret_cast<float *>(base), base + obs_bytes);
}

cx_status cx_observe(cx_ctx *ctx, float *obs_dev) {
  if (!ctx) return fail_status(CX_E_INVALID, "context is NULL");
  if (ctx->failed) return fail_status(CX_E_DEVICE, "context has a sticky device error");
  if (!obs_dev) return fail_status(CX_E_INVALID, "cx_observe: obs_dev is NULL");
  hipError_t e = launch_observe(ctx, obs_dev, ctx->stream);
  if (e != hipSuccess) return hip_fail(ctx, e, "cx_observe launch");
  return CX_OK;
}

}  // extern "C"
