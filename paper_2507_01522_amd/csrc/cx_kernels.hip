// cx_kernels.hip -- gfx950 kernels of the batched EV charging-station step.
//
// One station occupies L lanes of a 64-wide wavefront and each lane holds P
// slots (L * P = the station's padded slot count); a wave carries 64 / L
// stations.  Slot s of a station lives in lane s % L, register s / L.  A wave
// runs its stations for T steps with the whole state in registers and writes
// the per-step records out; the plain one-step form is the same kernel with
// T = 1.  Per step (App. A.2 order):
//   exogenous draws  (arrivals, price noise; computed L steps ahead, one step
//                     per lane, and broadcast -- they do not depend on the agent)
//   actions          (Philox levels / max / external)
//   apply actions    (clip by port max, charge curve, battery room)
//   projection       (Eq. ArchConst, deepest level first, butterfly sums over
//                     aligned power-of-two slot blocks: DPP inside a row,
//                     permlane swaps across rows, adds across registers; in the
//                     dense layout, one station-wide sum per node of a level)
//   charge, departures, arrivals (ballot + popcount ranks), reward, day end,
//   records (observations lane by lane, or, in the staged SIMPLE kernels,
//   through the block's LDS stage as 16-byte runs).
// Extended classes run their own kernels: V2G ports (signed levels, the
// mirrored discharge curve, two-sided limits, the split of the grid energy),
// a station battery (one FP64 scalar per station that every lane of the station
// updates alike), charge-sensitive users, per-episode price days and car
// models with AC / DC rates.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "cx_device.h"
#include "cx_mlp.h"
#include "cx_internal.h"

namespace cx {
namespace {

// Arrivals of one step: thresholds exceeded by w in a 32-entry row.  The
// first four entries come in one 16-byte load; the full bisection runs only
// when w exceeds all four (rare for the rates used here).
__device__ __forceinline__ int arrivals(const uint32_t *row, uint32_t w) {
  const u32x4 t = gld(reinterpret_cast<const u32x4 *>(row), 0);
  const int m = (int)(w > t.x) + (int)(w > t.y) + (int)(w > t.z) + (int)(w > t.w);
  if (m < 4) return m;
  int pos = 0;
  for (int s = 16; s >= 1; s >>= 1)
    if (gld(row, pos + s - 1) < w) pos += s;
  return pos;
}

// The same with the row's first four thresholds from the block's LDS copy
// (the rest, rarely needed, from device memory).
__device__ __forceinline__ int arrivals_lds(const __attribute__((address_space(3))) u32x4 *first4, const uint32_t *row,
                                            uint32_t w) {
  const u32x4 t = *first4;
  const int m = (int)(w > t.x) + (int)(w > t.y) + (int)(w > t.z) + (int)(w > t.w);
  if (m < 4) return m;
  int pos = 0;
  for (int s = 16; s >= 1; s >>= 1)
    if (gld(row, pos + s - 1) < w) pos += s;
  return pos;
}

// Stay length of an arriving car: 1 + #{thresholds below w}, bisecting the
// table in LDS (staged by the block) or in device memory.
__device__ __forceinline__ int stay_len(const uint32_t *tab, bool in_lds, int log2n, uint32_t w) {
  int pos = 0;
  if (in_lds) {
    const __attribute__((address_space(3))) uint32_t *t = (const __attribute__((address_space(3))) uint32_t *)tab;
    for (int s = 1 << (log2n - 1); s >= 1; s >>= 1)
      if (t[pos + s - 1] < w) pos += s;
  } else {
    for (int s = 1 << (log2n - 1); s >= 1; s >>= 1)
      if (gld(tab, pos + s - 1) < w) pos += s;
  }
  return 1 + pos;
}

// A pointer the compiler may not know to be wave-uniform, held in scalar
// registers (so loads through it can be scalar loads).
template <class T>
__device__ __forceinline__ const T *uniform_ptr(const T *p) {
  const uint64_t v = reinterpret_cast<uint64_t>(p);
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
  return reinterpret_cast<const T *>(((uint64_t)hi << 32) | lo);
}

// Exchange with the lane whose index differs in bit K (K = 0..5), for use in
// butterfly all-reductions.  K = 0, 1: DPP quad permutes.  K = 2, 3: DPP
// mirrors of the half-row / row -- after the steps below K every lane of an
// aligned 2^K group holds the same value, so the mirror lane is as good as the
// XOR partner.  K = 4, 5: the gfx950 row-swap instructions (v_permlane16_swap /
// v_permlane32_swap, plain VALU, no LDS round trip) followed by a select of the
// half that came from the partner.
template <int K>
__device__ __forceinline__ float xlane(float v) {
  const int iv = __float_as_int(v);
  if constexpr (K == 0) return __int_as_float(__builtin_amdgcn_update_dpp(0, iv, 0xB1, 0xF, 0xF, false));
  if constexpr (K == 1) return __int_as_float(__builtin_amdgcn_update_dpp(0, iv, 0x4E, 0xF, 0xF, false));
  if constexpr (K == 2) return __int_as_float(__builtin_amdgcn_update_dpp(0, iv, 0x141, 0xF, 0xF, false));
  if constexpr (K == 3) return __int_as_float(__builtin_amdgcn_update_dpp(0, iv, 0x140, 0xF, 0xF, false));
  if constexpr (K == 4) {
    // rows (0,1,2,3): first result = (r0, r0, r2, r2), second = (r1, r1, r3, r3)
    const auto r = __builtin_amdgcn_permlane16_swap(iv, iv, false, false);
    return __int_as_float((__lane_id() & 16) ? r[0] : r[1]);
  }
  if constexpr (K == 5) {
    // halves (0,1): first result = (h0, h0), second = (h1, h1)
    const auto r = __builtin_amdgcn_permlane32_swap(iv, iv, false, false);
    return __int_as_float((__lane_id() & 32) ? r[0] : r[1]);
  }
  return v;
}

// One butterfly step of a sum: v plus the value of the lane whose index
// differs in bit K.  K = 4, 5: the two halves the row-swap instruction leaves
// are exactly the pair to add (for a lane and its partner alike), so no select.
template <int K>
__device__ __forceinline__ float xsum(float v) {
  if constexpr (K == 4) {
    const int iv = __float_as_int(v);
    const auto r = __builtin_amdgcn_permlane16_swap(iv, iv, false, false);
    return __int_as_float(r[0]) + __int_as_float(r[1]);
  } else if constexpr (K == 5) {
    const int iv = __float_as_int(v);
    const auto r = __builtin_amdgcn_permlane32_swap(iv, iv, false, false);
    return __int_as_float(r[0]) + __int_as_float(r[1]);
  } else {
    return v + xlane<K>(v);
  }
}

// Sum over aligned groups of L lanes (every lane receives its group's sum).
template <int L>
__device__ __forceinline__ float station_sum(float v) {
  if constexpr (L > 1) v = xsum<0>(v);
  if constexpr (L > 2) v = xsum<1>(v);
  if constexpr (L > 4) v = xsum<2>(v);
  if constexpr (L > 8) v = xsum<3>(v);
  if constexpr (L > 16) v = xsum<4>(v);
  if constexpr (L > 32) v = xsum<5>(v);
  return v;
}

// xsum<K> for a K known only as a loop index of an unrolled loop.
template <int L>
__device__ __forceinline__ float xsum_k(float v, int K) {
  if (K == 0) return xsum<0>(v);
  if (K == 1) return xsum<1>(v);
  if (K == 2) return xsum<2>(v);
  if (K == 3) return xsum<3>(v);
  if (K == 4) return xsum<4>(v);
  return xsum<5>(v);
}

// Masked butterfly step: lanes whose block is smaller than 2^(K+1) send 0
// (a select, no branch; lb may vary per lane or be wave-uniform).
template <int K>
__device__ __forceinline__ float masked_step(float v, int lb) {
  const float u = (K < lb) ? v : 0.0f;
  return v + xlane<K>(u);
}

// Sums over aligned blocks of 2^lb lanes (a lane's block: lanes sharing the bits above lb).
template <int L>
__device__ __forceinline__ float block_sum_lanes(float v, int lb) {
  if constexpr (L > 1) v = masked_step<0>(v, lb);
  if constexpr (L > 2) v = masked_step<1>(v, lb);
  if constexpr (L > 4) v = masked_step<2>(v, lb);
  if constexpr (L > 8) v = masked_step<3>(v, lb);
  if constexpr (L > 16) v = masked_step<4>(v, lb);
  if constexpr (L > 32) v = masked_step<5>(v, lb);
  return v;
}

__device__ __forceinline__ float frcp(float x) { return __builtin_amdgcn_rcpf(x); }

// Four random action bytes from two Philox words: each 16-bit half h (low
// half first) gives (h n) >> 16, uniform over 0..n-1 up to 1 / 65536.
__device__ __forceinline__ uint32_t act_bytes(uint32_t wa, uint32_t wb, uint32_t n) {
  const uint32_t b0 = __umul24(wa & 0xFFFFu, n) >> 16, b1 = __umul24(wa >> 16, n) >> 16;
  const uint32_t b2 = __umul24(wb & 0xFFFFu, n) >> 16, b3 = __umul24(wb >> 16, n) >> 16;
  return b0 | (b1 << 8) | (b2 << 16) | (b3 << 24);
}

template <int L>
__device__ __forceinline__ int bcast(int v, int src) {
  if constexpr (L == 64) return __builtin_amdgcn_readlane(v, src);
  const int lane = __lane_id();
  return __builtin_amdgcn_ds_bpermute(((lane & ~(L - 1)) + src) << 2, v);
}
template <int L>
__device__ __forceinline__ float bcastf(float v, int src) {
  return __int_as_float(bcast<L>(__float_as_int(v), src));
}

struct Dyn {
  int32_t T, t_day0;
  uint32_t g0;
  int32_t mode, out_mode;
  float *obs;
  uint8_t *act;
  float *reward;
  uint8_t *done;
  const uint8_t *act_in;
  int64_t obs_stride, act_stride, env_stride;
};

// Store / load at a wave-uniform base plus a per-lane 32-bit byte offset
// (the global "saddr" form: no 64-bit address per lane).
template <class T>
__device__ __forceinline__ void st_at(T *base, uint32_t byte_off, T v) {
  typedef __attribute__((address_space(1))) T gT;
  typedef __attribute__((address_space(1))) char gchar;
  *(gT *)((gchar *)(char *)base + byte_off) = v;
}
template <class T>
__device__ __forceinline__ T ld_at(const T *base, uint32_t byte_off) {
  return *reinterpret_cast<const T *>(reinterpret_cast<const char *>(base) + byte_off);
}

// Observation records staged in LDS (SIMPLE classes).  Per step
// every lane puts its values in the block's stage (the adjacent envs of the
// block's waves, in record order); after the step barrier the block's running
// waves write the stage out as one contiguous run of 16-byte non-temporal
// stores.  HBM takes such whole-line streams much faster than the 4-byte
// stores of every lane, which leave lines partly written (for stations of 8
// lanes, 32 bytes per station and store).
typedef __attribute__((address_space(3))) float lds_float;
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(3))) f32x4 lds_f32x4;

// Write n staged floats to dst (4-byte aligned).  The stage holds them from
// float pad = (dst / 4) mod 4 on, so that LDS and HBM agree on 16-byte chunks:
// the whole chunks go out as one 16-byte buffer store each (a resource over the
// 16-byte-aligned address dst - pad, offset 16 c for chunk c, non-temporal),
// the at most 3 floats before the first and after the last whole chunk one by
// one.  tid / nthreads: this lane among the block's running lanes.
__device__ __forceinline__ void flush_stage(const lds_float *sb, float *dst, int pad, int n, int tid,
                                            int nthreads) {
  const int c_end = (pad + n) >> 2;  // whole chunks: [pad ? 1 : 0, c_end)
  // raw buffer: stride 0, range 2^31 - 1 bytes (offsets stay below 16 n + 64),
  // format word of a plain 32-bit buffer on gfx9-family GPUs
  const __amdgpu_buffer_rsrc_t rs =
      __builtin_amdgcn_make_buffer_rsrc(reinterpret_cast<char *>(dst) - 4 * pad, (short)0, 0x7fffffff, 0x00020000);
  for (int c = (pad ? 1 : 0) + tid; c < c_end; c += nthreads) {
    const f32x4 v = *reinterpret_cast<const lds_f32x4 *>(sb + 4 * c);
    __builtin_amdgcn_raw_buffer_store_b128(v, rs, 16 * c, 0, 2 /* nt */);
  }
  if (pad != 0 || ((pad + n) & 3) != 0) {  // the same in every lane
    const int head = (4 - pad) & 3;         // floats before the first whole chunk
    if (tid < head && tid < n) st_at(dst, 4u * (uint32_t)tid, (float)sb[pad + tid]);
    const int i = 4 * c_end - pad + (tid - 4);  // lanes 4..7: the floats after the last whole chunk
    if (tid >= 4 && tid < 8 && i >= head && i < n) st_at(dst, 4u * (uint32_t)i, (float)sb[pad + i]);
  }
}

// SIMPLE: the class has no padding slots (slot s holds port s, N = L * P), one
// port maximum and efficiency, and per tree level one block size and one limit.
// Port indices and record offsets are then compile-time constants and every
// per-slot constant is wave-uniform (scalar registers).
// EXT: V2G ports, a station battery, charge-sensitive users, price days and / or
// car models (never SIMPLE); each switched on per class by a uniform flag.
// STAGE: observations through the block's LDS stage (SIMPLE classes, when the
// context asks for it): stage / stage_floats are the two
// stage buffers and floats per buffer, g_blk0 the block's first group and
// n_run the number of its waves that run.
typedef __attribute__((address_space(3))) u32x4 lds_u32x4;
typedef __attribute__((address_space(3))) char lds_char;
typedef __attribute__((address_space(3))) uint8_t lds_u8;

// The fused policy rollout: after every step the block's staged observations
// (E = 32 envs, row stride obs_dim floats) go through the MLP on the matrix
// cores and each port gets its level for the next step, in LDS.  The products
// are those of the standalone policy kernel, K-step by K-step in the same
// order, so logits and levels are the same: here the block's 4 waves split the
// hidden units (first product) and the port groups (second) among them, and
// each wave reads its weight fragments from device memory (L2) straight into
// the matrix-core operands.  The K-step loops have compile-time bounds (K1, the
// class's K-steps of 32 features; 8 x 32 hidden units and 3 level tiles, the
// largest, over weights padded with zeros -- such steps add exact zeros), so
// that they are straight-line code whose loads are all issued ahead of the
// matrix-core work.  LDS: hb (8 x 2 hidden-unit fragments, over the stage once
// it has been read), xb (the observations in BF16, 256 features per env, zero
// past in_dim, rows 33 fragments apart so that the 16 envs of a tile fall in
// different banks) and act (a level byte per port and env).  wv: this wave in
// the block; convert: the step left its observations in the FP32 stage.
template <int K1>
__device__ __forceinline__ void policy_phase(const LaunchArgs::Pol &pl, const lds_float *stage, lds_char *lds,
                                             int obs_dim, int N, int blk_envs, int wv, uint32_t env_id0,
                                             uint32_t g, uint32_t k0, uint32_t k1, bool convert) {
  constexpr int W = kPolRolloutWaves, NT = kPolRolloutEnvs / 16, CPR = 4 * K1;  // chunks of 8 per row
  const int lane = __lane_id(), col = lane & 15, lg = lane >> 4, tid = wv * 64 + lane;
  const int in_dim = pl.in_dim, R = pl.R, G = pl.G, L1 = pl.L1;
  lds_u32x4 *xb = reinterpret_cast<lds_u32x4 *>(lds + pl.xb_off);
  lds_u32x4 *hb = reinterpret_cast<lds_u32x4 *>(lds + pl.hb_off);
  lds_u8 *act = reinterpret_cast<lds_u8 *>(lds + pl.act_off);
  const u32x4 zero = {0u, 0u, 0u, 0u};
  // observations -> BF16 (features past in_dim and envs past the block's: 0);
  // a row of the stage starts 16-byte aligned (obs_dim is a multiple of 4).
  // Without observation records the step wrote its values straight into xb
  // (convert = false), whose padding the first conversion zeroed.
  if (convert) {
    for (int c = tid; c < kPolRolloutEnvs * CPR; c += 64 * W) {
      const int e = c / CPR, k = c % CPR, f = 8 * k;
      const lds_float *row = stage + e * obs_dim + f;
      u32x4 v = zero;
      if (e < blk_envs) {
        if (f + 8 <= in_dim) {
          const f32x4 x = *reinterpret_cast<const lds_f32x4 *>(row);
          const f32x4 y = *reinterpret_cast<const lds_f32x4 *>(row + 4);
          v = u32x4{pack2(x.x, x.y), pack2(x.z, x.w), pack2(y.x, y.y), pack2(y.z, y.w)};
        } else if (f < in_dim) {
          float x[8];
#pragma unroll
          for (int j = 0; j < 8; ++j) x[j] = f + j < in_dim ? row[j] : 0.f;
          v = u32x4{pack2(x[0], x[1]), pack2(x[2], x[3]), pack2(x[4], x[5]), pack2(x[6], x[7])};
        }
      }
      xb[e * kPolXbRow + k] = v;
    }
    __syncthreads();
  }
  // first product: this wave's pairs of 16-unit hidden tiles, both pairs per
  // K-step so that each observation fragment is read once.  Weight fragments
  // come in buffer loads: one resource per matrix, the fragment's offset a
  // scalar, the lane's 16 bytes the vector offset (no 64-bit addresses).
  constexpr int NI = kPolHP / W;
  // vector offsets: the lane's 16 bytes, plus 4 KiB for K-steps 4..7; the
  // step's KiB within them goes in the instruction's offset field
  const uint32_t vo[2] = {16u * (uint32_t)lane, 16u * (uint32_t)lane + 4096u};
  const __amdgpu_buffer_rsrc_t w1 =
      __builtin_amdgcn_make_buffer_rsrc(const_cast<u32x4 *>(pl.w1f), (short)0, 2 * kPolHP * kPolK1 * 1024, 0x00020000);
  const __amdgpu_buffer_rsrc_t w2 =
      __builtin_amdgcn_make_buffer_rsrc(const_cast<u32x4 *>(pl.w2f), (short)0, G * kPolR * kPolHP * 1024, 0x00020000);
  f32x4 c0[NI][NT], c1[NI][NT];
#pragma unroll
  for (int i = 0; i < NI; ++i)
#pragma unroll
    for (int n = 0; n < NT; ++n) c0[i][n] = c1[i][n] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int s = 0; s < K1; ++s) {
    u32x4 a0[NI], a1[NI];
#pragma unroll
    for (int i = 0; i < NI; ++i) {
      const int m = 2 * (wv + W * i);  // the pair's first tile
      const uint32_t v = vo[s >> 2] + 1024u * (uint32_t)(s & 3);
      a0[i] = __builtin_bit_cast(u32x4, __builtin_amdgcn_raw_buffer_load_b128(w1, v, m * kPolK1 * 1024, 0));
      a1[i] = __builtin_bit_cast(u32x4, __builtin_amdgcn_raw_buffer_load_b128(w1, v, (m + 1) * kPolK1 * 1024, 0));
    }
#pragma unroll
    for (int n = 0; n < NT; ++n) {
      const u32x4 b = xb[(16 * n + col) * kPolXbRow + 4 * s + lg];
#pragma unroll
      for (int i = 0; i < NI; ++i) {
        c0[i][n] = mfma_bf16(a0[i], b, c0[i][n]);
        c1[i][n] = mfma_bf16(a1[i], b, c1[i][n]);
      }
    }
  }
#pragma unroll
  for (int i = 0; i < NI; ++i) {
    const int mp = wv + W * i;
    const f32x4 bA = gld(reinterpret_cast<const f32x4 *>(pl.b1 + 32 * mp + 4 * lg), 0);
    const f32x4 bB = gld(reinterpret_cast<const f32x4 *>(pl.b1 + 32 * mp + 16 + 4 * lg), 0);
#pragma unroll
    for (int n = 0; n < NT; ++n) hb[(mp * NT + n) * 64 + lane] = hidden_frag(c0[i][n], c1[i][n], bA, bB);
  }
  __syncthreads();
  // second product and the draw, per group of 4 ports.  The lane's ports are
  // 4 wv + lg + 16 i (group wv + 4 i): one Philox call per env serves them all
  U4 dw[NT];
#pragma unroll
  for (int n = 0; n < NT; ++n)
    dw[n] = philox(env_id0 + (uint32_t)(16 * n + col), g, draw_index(4 * wv + lg), kDomGum, k0, k1);
  for (int grp = wv; grp < G; grp += W) {
    const int port = 4 * grp + lg;
    float ud[NT];
#pragma unroll
    for (int n = 0; n < NT; ++n) ud[n] = draw_uniform(draw_word(dw[n], port));
    f32x4 c[kPolR][NT];
#pragma unroll
    for (int r = 0; r < kPolR; ++r) {
      const f32x4 b = gld(reinterpret_cast<const f32x4 *>(pl.b2f + (int64_t)(grp * kPolR + r) * 16 + 4 * lg), 0);
#pragma unroll
      for (int n = 0; n < NT; ++n) c[r][n] = b;
    }
#pragma unroll
    for (int s = 0; s < kPolHP; ++s) {
      u32x4 hv[NT];
#pragma unroll
      for (int n = 0; n < NT; ++n) hv[n] = hb[(s * NT + n) * 64 + lane];
#pragma unroll
      for (int r = 0; r < kPolR; ++r) {
        const u32x4 wf = __builtin_bit_cast(
            u32x4, __builtin_amdgcn_raw_buffer_load_b128(w2, vo[s >> 2] + 1024u * (uint32_t)(s & 3),
                                                         (grp * kPolR + r) * kPolHP * 1024, 0));
#pragma unroll
        for (int n = 0; n < NT; ++n) c[r][n] = mfma_bf16(wf, hv[n], c[r][n]);
      }
    }
#pragma unroll
    for (int n = 0; n < NT; ++n) {
      const int e = 16 * n + col;
      if (port < N && e < blk_envs) {
        const f32x4 cn[kPolR] = {c[0][n], c[1][n], c[2][n]};
        act[e * N + port] = (uint8_t)sample_level(cn, R, L1, ud[n]);
      }
    }
  }
  __syncthreads();
}

// exo_tp / exo_pr: the block's LDS copies of the first four arrival thresholds
// and the base price of every step of the day (NULL: read device memory).
template <int L, int P, bool SIMPLE, bool EXT, bool STAGE, bool POL = false>
__device__ __forceinline__ void run_group(const SegDev &sg, const Dyn &dy, int group, const uint32_t *tdw,
                                          bool tdw_lds, const lds_u32x4 *exo_tp, const lds_float *exo_pr,
                                          lds_float *stage, int stage_floats, int g_blk0, int n_run,
                                          const LaunchArgs::Pol *pol = nullptr, lds_char *lds = nullptr) {
  constexpr int SPW = 64 / L;
  constexpr int LOGL = (L == 4) ? 2 : (L == 8) ? 3 : (L == 16) ? 4 : (L == 32) ? 5 : 6;
  constexpr bool NOPAD = SIMPLE;  // every slot holds a port: slot s = port s
  const ClassDev C = *sg.cls;  // by value: scalar loads once, kept in SGPRs
  const int lane = __lane_id();
  const int l = lane & (L - 1);
  const int sbase = lane & ~(L - 1);
  const int env = group * SPW + (lane >> LOGL);     // env index inside the segment
  const bool active = env < sg.n_envs;
  const int S = NOPAD ? L * P : C.S;
  const int D = C.D;
  const int N = NOPAD ? L * P : C.n_ports;
  const int obs_dim = EXT ? C.obs_dim : 6 * N + 4;
  const int n_act = EXT ? C.n_act : N;      // action bytes per env
  const int n_neg = EXT ? C.n_neg : 0;      // discharge levels of a port
  const bool batt = EXT && C.has_batt != 0;
  const bool users = EXT && C.has_users != 0;  // some users are charge-sensitive
  const int n_days = EXT ? C.n_days : 0;       // exploring starts: price days
  const bool days = n_days > 0;
  const int n_models = EXT ? C.n_models : 0;   // car models (AC / DC rates)
  const bool models = n_models > 0;

  // ---- per-slot constants
  int port[P];
  float pmax[P], inv_pmax[P], inv_eta[P], lcap[kMaxLevels][P];
  float pdis[P], eta[P];  // EXT only
  uint32_t lbp[P];
#pragma unroll
  for (int j = 0; j < P; ++j) {
    const int s = j * L + l;
    port[j] = NOPAD ? s : gld(C.slot_port, s);
    if constexpr (SIMPLE) {
      pmax[j] = C.pmax_u;
      inv_pmax[j] = C.inv_pmax_u;
      inv_eta[j] = C.inv_eta_uniform;
      lbp[j] = C.lvl_lb_uniform;
#pragma unroll
      for (int d = 0; d < kMaxLevels; ++d) lcap[d][j] = C.lvl_cap_u[d];
    } else {
      pmax[j] = gld(C.slot_pmax, s);
      inv_pmax[j] = gld(C.slot_inv_pmax, s);
      inv_eta[j] = gld(C.slot_inv_eta, s);
      lbp[j] = gld(C.slot_lb, s);
#pragma unroll
      for (int d = 0; d < kMaxLevels; ++d) lcap[d][j] = d < D ? gld(C.slot_cap, d * S + s) : __builtin_inff();
    }
    if constexpr (EXT) {
      pdis[j] = gld(C.slot_pdis, s);
      eta[j] = gld(C.slot_eta, s);
    }
  }

  // ---- state
  double q[P];
  float qf[P];  // (float) q, kept in step with q: the FP32 work reads it
  float u[P], cap[P], icap[P], plast[P];
  int dw[P];
  int cs[P];  // EXT: 1 = a charge-sensitive user holds the slot (its dw may be <= 0)
  float rb[P];  // EXT: the car's maximum rate at this port (the port maximum without car models)
  int dc[P];    // EXT with car models: 1 = DC charger
  const int64_t sofs = (int64_t)env * S;
#pragma unroll
  for (int j = 0; j < P; ++j) {
    const int64_t i = sofs + j * L + l;
    q[j] = active ? sg.q[i] : 0.0;
    qf[j] = (float)q[j];
    u[j] = active ? sg.u[i] : 0.f;
    cap[j] = active ? sg.cap[i] : 0.f;
    plast[j] = active ? sg.p_last[i] : 0.f;
    dw[j] = active ? (int)sg.dwell[i] : 0;
    cs[j] = (users && active) ? (int)sg.utype[i] : 0;
    rb[j] = models ? (active ? sg.rbar[i] : 0.f) : pmax[j];
    dc[j] = models ? gld(C.slot_dc, j * L + l) : 0;
    icap[j] = cap[j] > 0.f ? frcp(cap[j]) : 0.f;
  }
  // a slot is occupied while its car's stay runs, or while a charge-sensitive
  // user waits to be charged
#define CX_OCCUPIED(j) (EXT ? (dw[j] > 0 || cs[j] != 0) : dw[j] > 0)
  double ret = active ? sg.ret[env] : 0.0;
  // station battery (EXT): SoC in FP64 and last power, alike in every lane of the station
  double bsoc = 0.0;
  float bpw = 0.f;
  if constexpr (EXT) {
    if (batt && active) {
      bsoc = sg.bsoc[env];
      bpw = sg.bp[env];
    }
  }
  uint32_t bkp[2] = {0u, 0u};  // EXT: the battery's action bytes of the current group of 8 steps
  // limit of the root (the whole station)
  const float c_root = D == 1 ? lcap[0][0] : D == 2 ? lcap[1][0] : D == 3 ? lcap[2][0] : lcap[3][0];

  const uint32_t k0 = (uint32_t)sg.seed, k1 = (uint32_t)(sg.seed >> 32);
  const uint32_t env_id = (uint32_t)(sg.env0 + env);
  // the day clock is the same in every lane: kept in scalar registers, the
  // end-of-day reset is a branch, not selects in every step
  const int steps_ep = __builtin_amdgcn_readfirstlane(C.steps_ep);
  const int n_levels = C.n_levels;
  int t_day = __builtin_amdgcn_readfirstlane(dy.t_day0);
  uint32_t g = dy.g0;
  int dday = 0;  // EXT: price day of the current episode (drawn at its first step)
  if constexpr (EXT) {
    if (days) dday = episode_day(env_id, g - (uint32_t)t_day, k0, k1, n_days);
  }
  int bM = 0, bdw = 1, bus = 0, bmod = 0;
  float bpb = 0.f, bcp = 0.f, bs0 = 0.f, btg = 0.f;
  // 64-lane SIMPLE stations, which often take two cars in a step: the
  // second car (rank 1) drawn ahead as well
  constexpr bool AHEAD2 = SIMPLE && L == 64;
  int bdw1 = 1;
  float bcp1 = 0.f, bs01 = 0.f, btg1 = 0.f;
  // RANDOM: each slot's action bytes of the current group of 8 steps, one per
  // byte (steps 0-3 of the group in kp[0], 4-7 in kp[1])
  uint32_t kp[P][2];
#pragma unroll
  for (int j = 0; j < P; ++j) kp[j][0] = kp[j][1] = 0u;
  const uint64_t smask = (L == 64) ? ~0ull : (((1ull << (L & 63)) - 1ull) << sbase);
  const uint64_t below_mask = (1ull << lane) - 1ull;

  // per-lane byte offsets of this env's records inside a step's segment block
  const uint32_t obs_bo = STAGE ? 0u : (uint32_t)env * (uint32_t)obs_dim * 4u;
  const uint32_t act_bo = (uint32_t)env * (uint32_t)n_act;
  const uint32_t env_bo = (uint32_t)env;
  // wave-uniform record pointers of the current step, advanced every step
  const bool w_obs = dy.out_mode == CX_OUT_FULL && dy.obs != nullptr;
  const bool w_act = (dy.out_mode == CX_OUT_FULL || dy.out_mode == CX_OUT_ACT_REWARD) && dy.act != nullptr;
  float *ob_t = w_obs ? dy.obs + sg.obs_off : nullptr;
  uint8_t *ab_t = w_act ? dy.act + sg.act_off : nullptr;
  const uint8_t *ai_t = dy.act_in ? dy.act_in + sg.act_off : nullptr;
  float *rw_t = dy.reward ? dy.reward + sg.env_off : nullptr;
  uint8_t *dn_t = dy.done ? dy.done + sg.env_off : nullptr;
  const int64_t obs_step = w_obs ? dy.obs_stride : 0;
  const int64_t act_step = (w_act || ai_t) ? dy.act_stride : 0;
  const int64_t env_step = (rw_t || dn_t) ? dy.env_stride : 0;
  // rewards and done flags share their step: each is written under its own
  // flag (with one of them NULL, its advanced pointer is no address)
  const bool w_rew = rw_t != nullptr, w_done = dn_t != nullptr;
  // the block's LDS observation stage (staging packings, whenever observations
  // are written): the block's first env, the floats the block writes per step
  // and this lane's env in the stage
  const int env_blk0 = g_blk0 * SPW;
  const int64_t blk_envs = sg.n_envs - env_blk0 < (int64_t)n_run * SPW ? sg.n_envs - env_blk0 : (int64_t)n_run * SPW;
  const int n_blk = (int)blk_envs * obs_dim;
  const uint32_t stage_bo = (uint32_t)(env - env_blk0) * (uint32_t)obs_dim * 4u;
  // the fused policy: every wave of the block takes part (waves past the last
  // env too, their lanes inactive); the first step's levels come from the
  // observation the rollout starts from, put in the stage
  [[maybe_unused]] const int wv = group - g_blk0;
  [[maybe_unused]] const uint32_t env_id0 = (uint32_t)(sg.env0 + env_blk0);
  // K-steps of 32 features of the first product: the observation of a SIMPLE
  // class has 6 L P + 4 features
  constexpr int kPolSteps1 = (6 * L * P + 4 + 31) / 32;
  if constexpr (POL) {
    const float *src = pol->obs0 + sg.obs_off + (int64_t)env_blk0 * obs_dim;
    for (int i = wv * 64 + lane; i < n_blk; i += kPolRolloutWaves * 64) stage[i] = gld(src, i);
    __syncthreads();
    policy_phase<kPolSteps1>(*pol, stage, lds, obs_dim, N, (int)blk_envs, wv, env_id0, g, k0, k1, true);
  }

  for (int t = 0; t < dy.T; ++t, ++g) {
    // ---- exogenous draws for the next L steps, lane l -> step t + l: the
    // arrival count, the price noise and the first arriving car's profile
    if ((t & (L - 1)) == 0) {
      int td = t_day + l;
      while (td >= steps_ep) td -= steps_ep;
      const uint32_t gl = g + (uint32_t)l;
      const U4 w = philox(env_id, gl, 0u, kDomEnv, k0, k1);
      if (exo_tp)
        bM = active ? arrivals_lds(exo_tp + td, C.tpois + td * kPoisStride, w.x) : 0;
      else
        bM = active ? arrivals(C.tpois + td * kPoisStride, w.x) : 0;
      const float u1 = (float)((w.y >> 8) + 1u) * 0x1p-24f;
      const float u2 = u24(w.z);
      const float z = __builtin_amdgcn_sqrtf(-2.0f * __logf(u1)) * __builtin_amdgcn_cosf(u2);
      float base;
      if (exo_pr) {
        base = exo_pr[td];
      } else {
        // wait for the load here, where it is issued: a load still pending
        // where the two paths join would make every step wait for all the
        // records in flight
        base = gld(C.glob, td * 4 + 2);
        asm volatile("" ::"v"(base));
      }
      if constexpr (EXT) {
        if (days) base = gld(C.price_days, episode_day(env_id, gl - (uint32_t)td, k0, k1, n_days) * steps_ep + td);
      }
      bpb = base + C.price_sigma * z;
      const U4 b = philox(env_id, gl, 0u, kDomCar, k0, k1);
      bcp = C.cap_lo + C.cap_span * u24(b.x);
      if constexpr (EXT) {
        if (models) {  // the car's model fixes its capacity
          bmod = 0;
          for (int m = 0; m < n_models; ++m) bmod += b.x > gld(C.model_thresh, m) ? 1 : 0;
          bcp = gld(C.model_data, 3 * bmod);
        }
      }
      bs0 = C.soc_lo + C.soc_span * u24(b.y);
      btg = C.tgt_lo + C.tgt_span * u24(b.z);
      bdw = stay_len(tdw, tdw_lds, C.dwell_log2, b.w);
      if constexpr (EXT) {
        if (users) bus = philox(env_id, gl, 0u, kDomUser, k0, k1).x <= C.cs_thresh ? 1 : 0;
      }
      if constexpr (AHEAD2) {
        if (__ballot(bM >= 2)) {  // some step ahead brings a second car
          const U4 b1 = philox(env_id, gl, 1u, kDomCar, k0, k1);
          bcp1 = C.cap_lo + C.cap_span * u24(b1.x);
          bs01 = C.soc_lo + C.soc_span * u24(b1.y);
          btg1 = C.tgt_lo + C.tgt_span * u24(b1.z);
          bdw1 = stay_len(tdw, tdw_lds, C.dwell_log2, b1.w);
        }
      }
    }
    const int tb = t & (L - 1);
    const int M = bcast<L>(bM, tb);
    const float pbuy = bcastf<L>(bpb, tb);
    // the observation's time features of the step after this one (scalar loads,
    // issued early; they do not wait for the records in flight)
    const int t_obs = __builtin_amdgcn_readfirstlane(t_day + 1 == steps_ep ? 0 : t_day + 1);
    const float *glob_u = uniform_ptr(C.glob);
    const float gl_sin = sld(glob_u, 4 * t_obs), gl_cos = sld(glob_u, 4 * t_obs + 1),
                gl_price = sld(glob_u, 4 * t_obs + 2);

    // ---- actions: action bytes k (level + n_neg)
    int k[P];
    int kb = 0;  // the battery's action byte (level + n_levels)
    if constexpr (POL) {  // the levels the policy drew after the last step
      const lds_u8 *lv = reinterpret_cast<const lds_u8 *>(lds + pol->act_off) + (env - env_blk0) * N;
#pragma unroll
      for (int j = 0; j < P; ++j) k[j] = active ? (int)lv[port[j]] : 0;
    } else if (dy.mode == CX_ACT_RANDOM) {
      if (t == 0 || (g & 7u) == 0) {
        // one Philox call gives the 8 steps' bytes: its 16-bit halves (low
        // half first) scaled to the n byte values, (h n) >> 16; n <= 255, so
        // the product is exact in a 24-bit multiply.  Action bytes are at most
        // 254 (n_levels <= 254; 127 with discharging).
        const uint32_t nk = (uint32_t)(n_levels + n_neg + 1);
#pragma unroll
        for (int j = 0; j < P; ++j) {
          const U4 w = philox(env_id, g >> 3, (uint32_t)port[j], kDomAct, k0, k1);
          kp[j][0] = act_bytes(w.x, w.y, nk);
          kp[j][1] = act_bytes(w.z, w.w, nk);
        }
        if constexpr (EXT) {
          if (batt) {
            const U4 w = philox(env_id, g >> 3, (uint32_t)N, kDomAct, k0, k1);
            const uint32_t nb = (uint32_t)(2 * n_levels + 1);
            bkp[0] = act_bytes(w.x, w.y, nb);
            bkp[1] = act_bytes(w.z, w.w, nb);
          }
        }
      }
      // the step's byte (wave-uniform selection of register and byte)
      const bool hi4 = (g & 4u) != 0;
      const uint32_t sh = 8u * (g & 3u);
#pragma unroll
      for (int j = 0; j < P; ++j) k[j] = (int)__builtin_amdgcn_ubfe(hi4 ? kp[j][1] : kp[j][0], sh, 8);
      if constexpr (EXT) kb = (int)__builtin_amdgcn_ubfe(hi4 ? bkp[1] : bkp[0], sh, 8);
    } else if (dy.mode == CX_ACT_MAX) {
#pragma unroll
      for (int j = 0; j < P; ++j) k[j] = n_levels + n_neg;
      kb = 2 * n_levels;
    } else {
#pragma unroll
      for (int j = 0; j < P; ++j) {
        int v = 0;
        if (active && port[j] >= 0)
          v = ld_at(ai_t, act_bo + (uint32_t)port[j]);
        k[j] = v > n_levels + n_neg ? n_levels + n_neg : v;
      }
      if constexpr (EXT) {
        int v = 0;
        if (batt && active) v = ld_at(ai_t, act_bo + (uint32_t)N);
        kb = v > 2 * n_levels ? 2 * n_levels : v;
      }
    }

    // ---- apply actions: clip by request, charge curve, battery room; a
    // discharging port (EXT) by its discharge maximum, the charging curve
    // mirrored about SoC 1/2 and the energy stored
    float pw[P];
#pragma unroll
    for (int j = 0; j < P; ++j) {
      const float req = (float)k[j] * C.inv_n_levels * pmax[j];
      const float rhat = pmax[j] * fminf(1.0f, qf[j] * C.inv_1mtau);
      const float room = qf[j] * cap[j] * C.inv_dt;
      if constexpr (EXT) {
        const int lev = k[j] - n_neg;
        const float soc = (float)(1.0 - q[j]);
        const float creq = (float)lev * C.inv_n_levels * pmax[j];
        const float dreq = (float)(-lev) * C.inv_n_levels * pdis[j];
        const float crate = rb[j] * fminf(1.0f, qf[j] * C.inv_1mtau);   // the car's curve
        const float drate = rb[j] * fminf(1.0f, soc * C.inv_1mtau);
        const float stored = soc * cap[j] * C.inv_dt;
        const float p = lev >= 0 ? fminf(fminf(creq, crate), room) : -fminf(fminf(dreq, drate), stored);
        pw[j] = CX_OCCUPIED(j) ? p : 0.0f;
      } else {
        pw[j] = dw[j] > 0 ? fminf(fminf(req, rhat), room) : 0.0f;
      }
    }

    // ---- projection onto the capacity tree (Eq. ArchConst), deepest level
    // first; the root (level D-1) holds the whole station
    float e_net, e_grid, e_out = 0.f;
    if constexpr (SIMPLE) {
      // Every node of a level owns an aligned block of 2^k slots, k the same for
      // the whole level.  One butterfly over the station's slots holds, after k
      // exchange steps, the load of each block of 2^k slots, already scaled by
      // the levels below (a scaled block contributes its limit); so each level
      // is checked when its block size is reached.  A slot's final factor is
      // the product of the factors of the nodes on its path.
      float r[P], F[P];
#pragma unroll
      for (int j = 0; j < P; ++j) {
        r[j] = pw[j];
        F[j] = 1.0f;
      }
      auto check = [&](int k) {
        if ((C.blk_mask >> k) & 1u) {  // a level of blocks of 2^k slots (wave-uniform)
          // a real (scalar) branch: most k have no level, and computing the
          // check for every k and selecting would cost more than it saves
          asm volatile("");
          const float c = C.blk_cap[k];
#pragma unroll
          for (int j = 0; j < P; ++j) {
            const bool over = r[j] > c;
            F[j] = over ? F[j] * (c * frcp(r[j])) : F[j];
            r[j] = over ? c : r[j];
          }
        }
      };
#pragma unroll
      for (int k = 0; k < LOGL; ++k) {
        check(k);
#pragma unroll
        for (int j = 0; j < P; ++j) r[j] = xsum_k<L>(r[j], k);
      }
      if constexpr (P >= 2) {  // blocks of 2 L slots: registers (0, 1) and (2, 3)
        check(LOGL);
        r[0] = r[1] = r[0] + r[1];
        if constexpr (P == 4) r[2] = r[3] = r[2] + r[3];
      }
      if constexpr (P == 4) {  // blocks of 4 L slots: all four registers
        check(LOGL + 1);
        r[0] = r[1] = r[2] = r[3] = r[0] + r[2];
      }
      // the root: the whole station, delivered energy its scaled load (App. A.3)
      const float tot = r[0];
      const bool over = tot > c_root;
      const float f = over ? c_root * frcp(tot) : 1.0f;
#pragma unroll
      for (int j = 0; j < P; ++j) pw[j] *= F[j] * f;
      e_net = C.dt * (over ? c_root : tot);
      e_grid = e_net * C.inv_eta_uniform;
    } else {
#pragma unroll
    for (int d = 0; d < kMaxLevels - 1; ++d) {
      if (d < D - 1) {
        float s[P];
        const int lbu = (int)((C.lvl_lb_uniform >> (8 * d)) & 0xFF);
        const int nd = SIMPLE ? 0 : (int)((C.dense_nodes >> (8 * d)) & 0xFF);
        if (nd != 0) {
          // dense layout: at most 4 nodes on this level, each summed over the
          // whole station from the slots it covers
#pragma unroll
          for (int j = 0; j < P; ++j) s[j] = 0.f;
#pragma unroll
          for (int m = 0; m < 4; ++m) {
            if (m < nd) {
              const uint32_t code = 0x80u | (uint32_t)m;
              float acc = 0.f;
#pragma unroll
              for (int j = 0; j < P; ++j) acc += ((lbp[j] >> (8 * d)) & 0xFFu) == code ? pw[j] : 0.f;
              acc = station_sum<L>(acc);
#pragma unroll
              for (int j = 0; j < P; ++j) s[j] = ((lbp[j] >> (8 * d)) & 0xFFu) == code ? acc : s[j];
            }
          }
        } else if (SIMPLE || lbu != 0xFF) {  // every slot of the level sits in a block of 2^lbu slots
#pragma unroll
          for (int j = 0; j < P; ++j) s[j] = block_sum_lanes<L>(pw[j], lbu);
        } else {
#pragma unroll
          for (int j = 0; j < P; ++j) s[j] = block_sum_lanes<L>(pw[j], (int)((lbp[j] >> (8 * d)) & 0xFF));
        }
        // blocks wider than a row of L slots span whole registers: add across them
        // (aligned layout only: a dense level's sums are already station-wide)
        if constexpr (P >= 2) {
          const int lb0 = nd != 0 ? 0 : (int)((lbp[0] >> (8 * d)) & 0xFF);
          if (lb0 > LOGL) {
            const float a = s[0] + s[1];
            s[0] = a;
            s[1] = a;
          }
          if constexpr (P == 4) {
            const int lb2 = nd != 0 ? 0 : (int)((lbp[2] >> (8 * d)) & 0xFF);
            if (lb2 > LOGL) {
              const float a = s[2] + s[3];
              s[2] = a;
              s[3] = a;
            }
            if (lb0 > LOGL + 1) {
              const float a = s[0] + s[2];
              s[0] = a; s[1] = a; s[2] = a; s[3] = a;
            }
          }
        }
#pragma unroll
        for (int j = 0; j < P; ++j) {
          const float c = lcap[d][j];
          if constexpr (EXT) {
            const float a = fabsf(s[j]);   // the limit bounds the magnitude of the net power
            pw[j] = a > c ? pw[j] * (c * frcp(a)) : pw[j];
          } else {
            pw[j] = s[j] > c ? pw[j] * (c * frcp(s[j])) : pw[j];
          }
        }
      }
    }
    // root: the station total before root scaling; the delivered energy is its
    // scaled value (App. A.3, charging only)
    if constexpr (EXT) {
      float tot = 0.f;
#pragma unroll
      for (int j = 0; j < P; ++j) tot += pw[j];
      tot = station_sum<L>(tot);
      const float a = fabsf(tot);
      const bool over = a > c_root;
      const float f = over ? c_root * frcp(a) : 1.0f;
#pragma unroll
      for (int j = 0; j < P; ++j) pw[j] *= f;
      e_net = C.dt * (over ? copysignf(c_root, tot) : tot);
      // grid energy: charging ports draw e / eta, discharging ports return eta e
      float tg = 0.f, to = 0.f;
#pragma unroll
      for (int j = 0; j < P; ++j) {
        tg += pw[j] > 0.f ? pw[j] * inv_eta[j] : pw[j] * eta[j];
        to += pw[j] < 0.f ? pw[j] * eta[j] : 0.f;
      }
      e_grid = C.dt * station_sum<L>(tg);
      if (C.alpha_dc != 0.0f) e_out = C.dt * station_sum<L>(to);
    } else {
      float tot = 0.f;
#pragma unroll
      for (int j = 0; j < P; ++j) tot += pw[j];
      tot = station_sum<L>(tot);
      const bool over = tot > c_root;
      const float f = over ? c_root * frcp(tot) : 1.0f;
#pragma unroll
      for (int j = 0; j < P; ++j) pw[j] *= f;
      e_net = C.dt * (over ? c_root : tot);
      if (C.uniform_eta) {
        e_grid = e_net * C.inv_eta_uniform;
      } else {
        float tg = 0.f;
#pragma unroll
        for (int j = 0; j < P; ++j) tg += pw[j] * inv_eta[j];
        e_grid = C.dt * station_sum<L>(tg);
      }
    }
    }  // projection of classes that are not SIMPLE

    // ---- the station battery (EXT): the (N+1)-th pole at the grid
    // connection, same curves, FP64 like the cars' q
    float e_b = 0.f;
    if constexpr (EXT) {
      if (batt) {
        const int lev = kb - n_levels;
        const double sb = bsoc;
        double pb;
        if (lev >= 0) {
          const double req = (double)lev * C.inv_n_d * C.b_rate;
          const double rhat = C.b_rate * fmin(1.0, (1.0 - sb) * C.b_inv_1mtau);
          const double room = (1.0 - sb) * C.b_cap * C.inv_dt_d;
          pb = fmin(fmin(req, rhat), room);
        } else {
          const double req = (double)(-lev) * C.inv_n_d * C.b_rate;
          const double rhat = C.b_rate * fmin(1.0, sb * C.b_inv_1mtau);
          const double stored = sb * C.b_cap * C.inv_dt_d;
          pb = -fmin(fmin(req, rhat), stored);
        }
        const double eb = C.dt_d * pb;
        const double ns = sb + eb * C.b_inv_cap;
        bsoc = ns > 1.0 ? 1.0 : (ns < 0.0 ? 0.0 : ns);
        bpw = (float)pb;
        e_b = (float)eb;
      }
    }

    // ---- charge, departures (selects: no branches): a time-sensitive user
    // leaves when its stay ends (c_satisfaction,0: energy still wanted), a
    // charge-sensitive one (EXT) when no energy is wanted any more
    // (c_satisfaction,1: hours overstayed - beta x hours left early)
    float csat = 0.f, csat1 = 0.f;
#pragma unroll
    for (int j = 0; j < P; ++j) {
      const bool occ = CX_OCCUPIED(j);              // pw = 0 and icap = 0 on empty slots
      const float e = C.dt * pw[j];
      const double nq = q[j] - (double)(e * icap[j]);
      q[j] = nq > 0.0 ? nq : 0.0;
      if constexpr (EXT) q[j] = q[j] < 1.0 ? q[j] : 1.0;  // discharging never below SoC 0
      qf[j] = (float)q[j];
      plast[j] = pw[j];
      dw[j] -= occ ? 1 : 0;
      bool dep = occ && dw[j] == 0;
      bool dep0 = dep;  // a time-sensitive user leaves
      if constexpr (EXT) {
        if (users) {
          const bool csu = cs[j] != 0;
          dep = occ && (csu ? q[j] <= (double)u[j] : dw[j] == 0);
          dep0 = dep && !csu;
          const float tl = (float)dw[j] * C.dt;
          csat1 += (dep && csu) ? fmaxf(0.0f, -tl) - C.beta_sat1 * fmaxf(0.0f, tl) : 0.0f;
          cs[j] = dep ? 0 : cs[j];
          dw[j] = dep ? 0 : dw[j];   // a charged user may leave with steps of its stay left
        }
        if (models) rb[j] = dep ? 0.f : rb[j];
      }
      if (C.alpha_sat != 0.0f) {  // energy still wanted by a departing car (c_satisfaction,0)
        const float miss = fmaxf(0.0f, (qf[j] - u[j]) * cap[j]);
        csat += dep0 ? miss : 0.0f;
      }
      q[j] = dep ? 0.0 : q[j];
      qf[j] = dep ? 0.0f : qf[j];
      u[j] = dep ? 0.f : u[j];
      cap[j] = dep ? 0.f : cap[j];
      icap[j] = dep ? 0.f : icap[j];
      plast[j] = dep ? 0.f : plast[j];
    }
    if (C.alpha_sat != 0.0f) csat = station_sum<L>(csat);
    if constexpr (EXT) {
      if (users && C.alpha_sat1 != 0.0f) csat1 = station_sum<L>(csat1);
    }

    // ---- arrivals: first free ports in port order take the accepted cars
    int cnt[P], below[P];
    bool fr[P];
    int n_free = 0;
#pragma unroll
    for (int j = 0; j < P; ++j) {
      fr[j] = (EXT ? !CX_OCCUPIED(j) : dw[j] == 0) && (NOPAD || port[j] >= 0);
      const uint64_t m = __ballot(fr[j]) & smask;
      cnt[j] = __popcll(m);
      below[j] = __popcll(m & below_mask);
      n_free += cnt[j];
    }
    const int acc = M < n_free ? M : n_free;
    const int rej = M - acc;
    if (__ballot(acc > 0)) {
      // the first car's profile was drawn ahead by lane tb of the station
      const float f_cp = bcastf<L>(bcp, tb), f_s0 = bcastf<L>(bs0, tb), f_tg = bcastf<L>(btg, tb);
      const int f_dw = bcast<L>(bdw, tb);
      const int f_us = EXT ? bcast<L>(bus, tb) : 0;
      const int f_mod = EXT ? bcast<L>(bmod, tb) : 0;
      // (AHEAD2) the second car's, when the station takes two
      float f_cp1 = 0.f, f_s01 = 0.f, f_tg1 = 0.f;
      int f_dw1 = 1;
      if constexpr (AHEAD2) {
        if (__ballot(acc > 1)) {
          f_cp1 = bcastf<L>(bcp1, tb);
          f_s01 = bcastf<L>(bs01, tb);
          f_tg1 = bcastf<L>(btg1, tb);
          f_dw1 = bcast<L>(bdw1, tb);
        }
      }
      int run = 0;
#pragma unroll
      for (int j = 0; j < P; ++j) {
        const int rank = run + below[j];
        if (fr[j] && rank < acc) {
          float cp = f_cp, s0 = f_s0, tg = f_tg;
          int dd = f_dw;
          int us = f_us, md = f_mod;
          if (AHEAD2 && rank == 1) {
            cp = f_cp1;
            s0 = f_s01;
            tg = f_tg1;
            dd = f_dw1;
          } else if (rank > 0) {
            const U4 b = philox(env_id, g, (uint32_t)rank, kDomCar, k0, k1);
            cp = C.cap_lo + C.cap_span * u24(b.x);
            if constexpr (EXT) {
              if (models) {
                md = 0;
                for (int m = 0; m < n_models; ++m) md += b.x > gld(C.model_thresh, m) ? 1 : 0;
                cp = gld(C.model_data, 3 * md);
              }
            }
            s0 = C.soc_lo + C.soc_span * u24(b.y);
            tg = C.tgt_lo + C.tgt_span * u24(b.z);
            dd = stay_len(tdw, tdw_lds, C.dwell_log2, b.w);
            if constexpr (EXT) {
              if (users) us = philox(env_id, g, (uint32_t)rank, kDomUser, k0, k1).x <= C.cs_thresh ? 1 : 0;
            }
          }
          dw[j] = dd;
          if constexpr (EXT) {
            cs[j] = us;
            if (models) rb[j] = gld(C.model_data, 3 * md + (dc[j] ? 2 : 1));
          }
          cap[j] = cp;
          icap[j] = frcp(cp);
          q[j] = 1.0 - (double)s0;
          qf[j] = 1.0f - s0;  // the same rounding as (float) q
          u[j] = 1.0f - tg;
          plast[j] = 0.f;
        }
        run += cnt[j];
      }
    }

    // ---- reward (App. A.3)
    float r;
    if constexpr (EXT) {
      const float e_gn = e_grid + e_b;
      const float price = e_gn > 0.0f ? pbuy : C.p_sell_grid;
      r = C.p_sell * e_net - price * e_gn - C.fixed_cost - C.alpha_sat * csat - C.alpha_dec * (float)rej -
          C.alpha_db * fmaxf(0.0f, -e_b) + C.alpha_dc * e_out - C.alpha_sat1 * csat1;
    } else {
      const float price = e_grid > 0.0f ? pbuy : C.p_sell_grid;
      r = C.p_sell * e_net - price * e_grid - C.fixed_cost - C.alpha_sat * csat - C.alpha_dec * (float)rej;
    }
    ret += (double)r;

    // ---- end of day
    t_day += 1;
    const bool done = t_day == steps_ep;
    if (done) {
      t_day = 0;
#pragma unroll
      for (int j = 0; j < P; ++j) {
        dw[j] = 0; q[j] = 0.0; qf[j] = 0.f; u[j] = 0.f; cap[j] = 0.f; icap[j] = 0.f; plast[j] = 0.f;
        if constexpr (EXT) {
          cs[j] = 0;
          if (models) rb[j] = 0.f;
        }
      }
      if constexpr (EXT) {
        if (days) dday = episode_day(env_id, g + 1u, k0, k1, n_days);  // the next episode begins
      }
      if constexpr (EXT) {
        if (batt) {
          bsoc = C.b_soc0;
          bpw = 0.f;
        }
      }
    }

    // ---- records: an env's observation (byte offsets o inside its record)
    // goes to the block's LDS stage, or (wide stations) straight to HBM
    float *const ob_now = ob_t;  // this step's observation block of the segment
    // per-lane offsets, re-read every step: with the 32-bit offset visible at
    // each store the compiler emits the scalar-base form (no 64-bit lane address)
    uint32_t obs_bo_t = obs_bo, act_bo_t = act_bo, env_bo_t = env_bo;
    asm volatile("" : "+v"(obs_bo_t), "+v"(act_bo_t), "+v"(env_bo_t));
    // (the fused policy reads the stage from float 0: its records are 16-byte aligned)
    const int pad = !POL && STAGE && w_obs
                        ? (int)((reinterpret_cast<uintptr_t>(ob_now + (int64_t)env_blk0 * obs_dim) >> 2) & 3u)
                        : 0;
    if (active) {
      if (w_obs || POL) {
        auto obs_record = [&](auto put) {
#pragma unroll
          for (int j = 0; j < P; ++j) {
            if (NOPAD || port[j] >= 0) {
              const bool occ = CX_OCCUPIED(j);
              const uint32_t o = 4u * (uint32_t)port[j];
              put(0u * 4u * N, o, occ ? 1.0f : 0.0f);
              put(1u * 4u * N, o, occ ? 1.0f - qf[j] : 0.0f);
              put(2u * 4u * N, o, occ ? qf[j] - u[j] : 0.0f);
              put(3u * 4u * N, o, (float)dw[j] * C.inv_steps_ep);
              float rh = fminf(1.0f, qf[j] * C.inv_1mtau);
              if constexpr (EXT) {
                if (models) rh *= rb[j] * inv_pmax[j];  // the car's curve, as a share of the port maximum
              }
              put(4u * 4u * N, o, occ ? rh : 0.0f);
              put(5u * 4u * N, o, plast[j] * inv_pmax[j]);
              if constexpr (EXT) {
                if (users) put(4u * (uint32_t)C.user_obs, 4u * (uint32_t)port[j], cs[j] ? 1.0f : 0.0f);
              }
            }
          }
          if (l < 4) {
            const int n_occ = done ? 0 : (N - n_free + acc);
            float gv = l == 3 ? (float)n_occ * (1.0f / (float)N) : l == 0 ? gl_sin : l == 1 ? gl_cos : gl_price;
            if constexpr (EXT) {
              if (days && l == 2) gv = gld(C.price_days, dday * steps_ep + t_day);
            }
            put(4u * (uint32_t)(6 * N), 4u * (uint32_t)l, gv);
          }
          if constexpr (EXT) {
            if (batt && l < 2) put(4u * (uint32_t)(6 * N + 4), 4u * (uint32_t)l, l == 0 ? (float)bsoc : bpw * C.b_inv_rate);
            if (days && l < 2)
              put(4u * (uint32_t)C.day_obs, 4u * (uint32_t)l, l == 0 ? (float)dday * C.inv_n_days : (dday % 7 >= 5 ? 1.0f : 0.0f));
          }
        };
        if (POL && !w_obs) {
          // the fused policy without observation records: the values go to
          // the MLP's BF16 rows directly (their padding was zeroed by the
          // first conversion)
          typedef __attribute__((address_space(3))) uint16_t lds_u16;
          lds_u16 *xr = reinterpret_cast<lds_u16 *>(lds + pol->xb_off) + (env - env_blk0) * (kPolXbRow * 8);
          obs_record([&](uint32_t fo, uint32_t lo, float v) { xr[(fo + lo) >> 2] = (uint16_t)pack2(v, 0.f); });
        } else if constexpr (STAGE) {
          lds_float *sb = stage + (POL ? 0 : (t & 1) * stage_floats) + pad;
          obs_record([&](uint32_t fo, uint32_t lo, float v) {
            *reinterpret_cast<lds_float *>(reinterpret_cast<__attribute__((address_space(3))) char *>(sb) + stage_bo +
                                           fo + lo) = v;
          });
        } else {
          // the feature's offset goes on the wave-uniform base, the lane's on its
          // 32-bit offset
          obs_record([&](uint32_t fo, uint32_t lo, float v) {
            st_at((float *)((char *)ob_now + fo), obs_bo_t + lo, v);
          });
        }
      }
      if (w_act) {
        uint8_t *ab = ab_t;
        bool packed = false;
        if constexpr (NOPAD) {
          // four consecutive ports' bytes gathered into the first lane of each
          // quad and stored as one dword (an env's bytes start at a multiple of
          // 4, N being one; the step's row too when its base is aligned)
          if ((reinterpret_cast<uintptr_t>(ab) & 3u) == 0) {
            packed = true;
#pragma unroll
            for (int j = 0; j < P; ++j) {
              const int b1 = __builtin_amdgcn_update_dpp(0, k[j], 0x55, 0xF, 0xF, false);  // quad lane 1
              const int b2 = __builtin_amdgcn_update_dpp(0, k[j], 0xAA, 0xF, 0xF, false);  // quad lane 2
              const int b3 = __builtin_amdgcn_update_dpp(0, k[j], 0xFF, 0xF, 0xF, false);  // quad lane 3
              const uint32_t w4 =
                  (uint32_t)k[j] | ((uint32_t)b1 << 8) | ((uint32_t)b2 << 16) | ((uint32_t)b3 << 24);
              if ((l & 3) == 0) st_at((uint32_t *)ab, act_bo_t + (uint32_t)port[j], w4);
            }
          }
        }
        if (!packed) {
#pragma unroll
          for (int j = 0; j < P; ++j)
            if (NOPAD || port[j] >= 0) st_at(ab, act_bo_t + (uint32_t)port[j], (uint8_t)k[j]);
        }
        if constexpr (EXT) {
          if (batt && l == 0) st_at(ab, act_bo_t + (uint32_t)N, (uint8_t)kb);
        }
      }
      if (l == 0) {
        if (w_rew) st_at(rw_t, 4u * env_bo_t, r);
        if (w_done) st_at(dn_t, env_bo_t, (uint8_t)(done ? 1 : 0));
      }
    }
    ob_t += obs_step;
    ab_t += act_step;
    ai_t += act_step;
    rw_t += env_step;
    dn_t += env_step;
    // Keep the block's waves on the same step: their records for the step
    // are then adjacent envs' blocks written together, which HBM takes
    // noticeably faster (better row locality) than the same bytes spread over
    // many steps.  Waves that left early (past the last env) do not count.
    __syncthreads();
    // the stage of this step is complete: out to HBM (the next step fills the
    // other buffer; the barrier of that step keeps this one until it is read)
    if (STAGE && w_obs && (!POL || wv < n_run))
      flush_stage(stage + (POL ? 0 : (t & 1) * stage_floats), ob_now + (int64_t)env_blk0 * obs_dim, pad, n_blk,
                  (group - g_blk0) * 64 + lane, n_run * 64);
    if constexpr (POL) {
      // the next step's levels (the phase's barriers keep the stage until the
      // flush above has read it)
      if (t + 1 < dy.T)
        policy_phase<kPolSteps1>(*pol, stage, lds, obs_dim, N, (int)blk_envs, wv, env_id0, g + 1u, k0, k1,
                                 w_obs);
    }
  }

  // ---- state back to HBM
  if (active) {
#pragma unroll
    for (int j = 0; j < P; ++j) {
      const int64_t i = sofs + j * L + l;
      sg.q[i] = q[j];
      sg.u[i] = u[j];
      sg.cap[i] = cap[j];
      sg.p_last[i] = plast[j];
      sg.dwell[i] = (int16_t)dw[j];
      if constexpr (EXT) {
        if (users) sg.utype[i] = (uint8_t)cs[j];
        if (models) sg.rbar[i] = rb[j];
      }
    }
    if (l == 0) sg.ret[env] = ret;
    if constexpr (EXT) {
      if (batt && l == 0) {
        sg.bsoc[env] = bsoc;
        sg.bp[env] = bpw;
      }
    }
  }
}

#undef CX_OCCUPIED

// The launch's blocks are dealt to the chip's 8 XCDs in turn (block i to XCD
// i mod 8).  Numbered so that each XCD's blocks are consecutive, blocks of
// adjacent envs, whose small records (actions, rewards, done flags) share
// 128-byte lines, write those lines through the same L2.
__device__ __forceinline__ int xcd_block() {
  const int i = blockIdx.x, n = gridDim.x;
  const int x = i & 7, q = n >> 3, r = n & 7;
  return x * q + (x < r ? x : r) + (i >> 3);
}

// One kernel per packing (lanes per station L, slots per lane P) and class
// kind (general, SIMPLE, bidirectional), so that each keeps its own register
// budget; the entry points below add the launch bounds of each kind.
template <int L, int P, bool SIMPLE, bool EXT, bool STAGE, bool POL>
__device__ __forceinline__ void rollout_body(LaunchArgs a) {
  extern __shared__ uint32_t lds_tdwell[];
  // (the staged kernels, whose blocks write whole runs of adjacent envs)
  const int b = STAGE ? __builtin_amdgcn_readfirstlane(xcd_block()) : (int)blockIdx.x;
  int lo = 0, hi = a.n_segs - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (a.segs[mid].block_begin <= b) lo = mid;
    else hi = mid - 1;
  }
  // the segment is block-uniform: say so, so its fields come in scalar loads
  lo = __builtin_amdgcn_readfirstlane(lo);
  const SegDev sg = a.segs[lo];
  Dyn dy;
  if (a.per_segment) {
    dy = Dyn{sg.T, sg.t_day0, sg.g0, sg.mode, sg.out_mode, sg.obs, sg.act, sg.reward, sg.done, sg.act_in,
             sg.obs_stride, sg.act_stride, sg.env_stride};
  } else {
    dy = Dyn{a.T, a.t_day0, a.g0, a.mode, a.out_mode, a.obs, a.act, a.reward, a.done, a.act_in,
             a.obs_stride, a.act_stride, a.env_stride};
  }
  // stay-length thresholds in LDS (every wave of the block helps load them
  // before any wave may leave)
  const uint32_t *tdw = sg.cls->tdwell;
  const bool tdw_lds = a.lds_tdwell != 0;
  const lds_u32x4 *exo_tp = nullptr;
  const lds_float *exo_pr = nullptr;
  if (tdw_lds) {
    const int n = 1 << sg.cls->dwell_log2;
    for (int i = threadIdx.x; i < n; i += blockDim.x) lds_tdwell[i] = gld(tdw, i);
    // the day's per-step tables after the (16-byte aligned) stay table, for
    // launches long enough to repay copying them (short ones read them from
    // device memory)
    const int steps = sg.cls->steps_ep;
    if (!POL && steps <= kLdsExoSteps && dy.T >= kLdsExoMinT) {
      __attribute__((address_space(3))) char *base =
          (__attribute__((address_space(3))) char *)lds_tdwell + ((4 * n + 15) & ~15);
      lds_u32x4 *tp = (lds_u32x4 *)base;
      lds_float *pr = (lds_float *)(base + 16 * kLdsExoSteps);
      const uint32_t *tpois = sg.cls->tpois;
      const float *glob = sg.cls->glob;
      for (int i = threadIdx.x; i < steps; i += blockDim.x) {
        tp[i] = gld(reinterpret_cast<const u32x4 *>(tpois + (int64_t)i * kPoisStride), 0);
        pr[i] = gld(glob, 4 * i + 2);
      }
      exo_tp = tp;
      exo_pr = pr;
    }
    __syncthreads();
    tdw = lds_tdwell;
  }
  const int W = blockDim.x >> 6;
  const int g_blk0 = (b - sg.block_begin) * W;  // the block's first group
  const int group = __builtin_amdgcn_readfirstlane(g_blk0 + (int)(threadIdx.x >> 6));
  // (the fused policy keeps every wave: all take part in the MLP)
  if (!POL && group >= sg.n_groups) return;
  const int n_run = min(W, sg.n_groups - g_blk0);  // waves of the block that run
  lds_float *stage =
      a.stage_floats > 0 ? (lds_float *)((__attribute__((address_space(3))) char *)lds_tdwell + a.stage_off) : nullptr;
  run_group<L, P, SIMPLE, EXT, STAGE, POL>(sg, dy, group, tdw, tdw_lds, exo_tp, exo_pr, stage, a.stage_floats,
                                           g_blk0, n_run, &a.pol, (lds_char *)lds_tdwell);
}

template <int L, int P, bool SIMPLE, bool EXT, bool STAGE>
__global__ __launch_bounds__(512) void k_rollout(LaunchArgs a) {
  rollout_body<L, P, SIMPLE, EXT, STAGE, false>(a);
}

// SIMPLE classes of 1 or 2 slots per lane: the kernel held to CX_SIMPLE_WAVES
// waves per SIMD (96 VGPRs at 5, a few of them spilled): their step is issue-
// bound, and the extra waves hide its latencies.
#ifndef CX_SIMPLE_WAVES
#define CX_SIMPLE_WAVES 5
#endif
template <int L, int P, bool STAGE>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(CX_SIMPLE_WAVES))) void k_rollout_simple(
    LaunchArgs a) {
  rollout_body<L, P, true, false, STAGE, false>(a);
}

// The fused policy rollout (4 waves per block): three blocks per CU, so that
// one block's matrix-core work and memory waits overlap the others' steps.
template <int L, int P>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) void k_rollout_policy(LaunchArgs a) {
  rollout_body<L, P, true, false, true, true>(a);
}

// Observation of empty stations at t_day = 0 for every env of one segment
// (env0: Philox index of its first env; g: the step the new episodes begin on).
__global__ void k_reset_obs(const ClassDev *cls, int64_t n_envs, float *obs, uint64_t seed, int64_t env0,
                            uint32_t g) {
  const int64_t dim = cls->obs_dim;
  const int N = cls->n_ports, n_days = cls->n_days, day_obs = cls->day_obs;
  const int64_t total = n_envs * dim;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t f = i % dim;
    float v = 0.f;
    if (f >= 6 * N && f < 6 * N + 3) v = cls->glob[f - 6 * N];
    if (cls->has_batt && f == 6 * N + 4) v = (float)cls->b_soc0;  // a battery starts the day at its initial SoC
    if (n_days > 0 && (f == 6 * N + 2 || f == day_obs || f == day_obs + 1)) {
      const int d = episode_day((uint32_t)(env0 + i / dim), g, (uint32_t)seed, (uint32_t)(seed >> 32), n_days);
      v = f == 6 * N + 2 ? cls->price_days[(int64_t)d * cls->steps_ep]
                         : f == day_obs ? (float)d * cls->inv_n_days : (d % 7 >= 5 ? 1.0f : 0.0f);
    }
    obs[i] = v;
  }
}

__global__ void k_fill_f64(double *p, int64_t n, double v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

using KernelFn = void (*)(LaunchArgs);

// The kernels of one packing: general, SIMPLE, extended, SIMPLE with staged
// observations.
#define CX_KINDS(L, P)                                                                              \
  &k_rollout<L, P, false, false, false>, &k_rollout<L, P, true, false, false>,                        \
      &k_rollout<L, P, false, true, false>, &k_rollout<L, P, true, false, true>
#define CX_KINDS_SIMPLE(L, P)                                                                       \
  &k_rollout<L, P, false, false, false>, &k_rollout_simple<L, P, false>,                              \
      &k_rollout<L, P, false, true, false>, &k_rollout_simple<L, P, true>

// Kernel of each launch kind: packing id (P index * 5 + L index, as pack_id())
// times kNumKinds, plus the kernel kind (kKind*).
const KernelFn kKernels[kNumKinds * kNumPackings] = {
    CX_KINDS_SIMPLE(4, 1), CX_KINDS_SIMPLE(8, 1), CX_KINDS_SIMPLE(16, 1), CX_KINDS_SIMPLE(32, 1),
    CX_KINDS_SIMPLE(64, 1), CX_KINDS_SIMPLE(4, 2), CX_KINDS_SIMPLE(8, 2), CX_KINDS_SIMPLE(16, 2),
    CX_KINDS_SIMPLE(32, 2), CX_KINDS_SIMPLE(64, 2),
    CX_KINDS(4, 4), CX_KINDS(8, 4), CX_KINDS(16, 4), CX_KINDS(32, 4), CX_KINDS(64, 4)};
#undef CX_KINDS
#undef CX_KINDS_SIMPLE

// Arguments of one group's launch: its slice of the segment table and its LDS
// (the stay table; for staging packings the observation stages when
// observations are written).
LaunchArgs group_args(const LaunchArgs &a, const LaunchGroup &g, size_t *lds) {
  LaunchArgs b = a;
  b.segs = a.segs + g.seg_begin;
  b.n_segs = g.n_segs;
  b.lds_tdwell = 1;  // staging the table costs one load per thread and beats device-memory
                     // bisection even for one-step launches
  const bool records =
      group_stages(g.kind, g.pack) && (a.per_segment || (a.out_mode == CX_OUT_FULL && a.obs != nullptr));
  const size_t with_stages = group_lds_bytes(g.wpb, g.pack, g.max_obs_dim, g.max_dwell_log2, &b.stage_off,
                                             &b.stage_floats);
  if (records) {
    *lds = with_stages;
  } else {
    b.stage_floats = 0;
    *lds = group_table_bytes(g.max_dwell_log2);
  }
  return b;
}

}  // namespace

hipError_t launch_groups(const LaunchArgs &a, const LaunchGroup *groups, int n_groups, hipStream_t st) {
  for (int i = 0; i < n_groups; ++i) {
    const LaunchGroup &g = groups[i];
    if (g.n_blocks <= 0) continue;
    size_t lds = 0;
    LaunchArgs b = group_args(a, g, &lds);
    void *params[1] = {&b};
    hipError_t e = hipLaunchKernel(reinterpret_cast<const void *>(kKernels[kNumKinds * g.pack + g.kind]), dim3(g.n_blocks),
                                   dim3(64 * g.wpb), params, lds, st);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// The fused policy rollout of one SIMPLE class: stations of 8 lanes (8, 16 or
// 32 slots), 4 waves per block (32 stations, two 16-env tiles of the MLP).
hipError_t launch_policy_rollout(const LaunchArgs &a, int per_lane, int n_blocks, size_t lds, hipStream_t st) {
  if (n_blocks <= 0) return hipSuccess;
  KernelFn f = per_lane == 1   ? &k_rollout_policy<8, 1>
               : per_lane == 2 ? &k_rollout_policy<8, 2>
               : per_lane == 4 ? &k_rollout_policy<8, 4>
                               : nullptr;
  if (!f) return hipErrorInvalidValue;
  LaunchArgs b = a;
  void *params[1] = {&b};
  return hipLaunchKernel(reinterpret_cast<const void *>(f), dim3(n_blocks), dim3(64 * kPolRolloutWaves), params, lds,
                         st);
}

hipError_t graph_rollout(RolloutGraph &G, const LaunchArgs &a, const LaunchGroup *groups, int n_groups,
                         hipStream_t st) {
  LaunchArgs args[kNumKinds * kNumPackings];
  void *params[kNumKinds * kNumPackings][1];
  hipKernelNodeParams p[kNumKinds * kNumPackings];
  int shape[kNumKinds * kNumPackings][4] = {};
  int n = 0;
  for (int i = 0; i < n_groups && n < kNumKinds * kNumPackings; ++i) {
    const LaunchGroup &g = groups[i];
    if (g.n_blocks <= 0) continue;
    size_t lds = 0;
    args[n] = group_args(a, g, &lds);
    params[n][0] = &args[n];
    p[n] = hipKernelNodeParams{};
    p[n].func = reinterpret_cast<void *>(kKernels[kNumKinds * g.pack + g.kind]);
    p[n].gridDim = dim3(g.n_blocks);
    p[n].blockDim = dim3(64 * g.wpb);
    p[n].sharedMemBytes = (unsigned)lds;
    p[n].kernelParams = params[n];
    p[n].extra = nullptr;
    shape[n][0] = kNumKinds * g.pack + g.kind;
    shape[n][1] = g.n_blocks;
    shape[n][2] = g.wpb;
    shape[n][3] = (int)lds;
    ++n;
  }
  if (n == 0) return hipSuccess;
  bool same = G.exec && G.n_nodes == n;
  for (int i = 0; same && i < n; ++i)
    for (int j = 0; j < 4; ++j) same = same && G.shape[i][j] == shape[i][j];
  hipError_t e;
  if (!same) {
    graph_destroy(G);
    if ((e = hipGraphCreate(&G.graph, 0)) != hipSuccess) return e;
    for (int i = 0; i < n; ++i)
      if ((e = hipGraphAddKernelNode(&G.node[i], G.graph, nullptr, 0, &p[i])) != hipSuccess) return e;
    if ((e = hipGraphInstantiate(&G.exec, G.graph, nullptr, nullptr, 0)) != hipSuccess) return e;
    G.n_nodes = n;
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < 4; ++j) G.shape[i][j] = shape[i][j];
  } else {
    for (int i = 0; i < n; ++i)
      if ((e = hipGraphExecKernelNodeSetParams(G.exec, G.node[i], &p[i])) != hipSuccess) return e;
  }
  return hipGraphLaunch(G.exec, st);
}

void graph_destroy(RolloutGraph &g) {
  if (g.exec) (void)hipGraphExecDestroy(g.exec);
  if (g.graph) (void)hipGraphDestroy(g.graph);
  g = RolloutGraph{};
}

hipError_t launch_reset_obs_one(const ClassDev *cls_dev, int64_t n_envs, float *obs, uint64_t seed, int64_t env0,
                                uint32_t g, hipStream_t st) {
  if (n_envs <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_reset_obs, dim3(256), dim3(256), 0, st, cls_dev, n_envs, obs, seed, env0, g);
  return hipGetLastError();
}

hipError_t launch_fill_f64(double *p, int64_t n, double v, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const int blocks = (int)std::min<int64_t>(1024, (n + 255) / 256);
  hipLaunchKernelGGL(k_fill_f64, dim3(blocks), dim3(256), 0, st, p, n, v);
  return hipGetLastError();
}

}  // namespace cx
