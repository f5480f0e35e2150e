/*
 * cx.h -- C ABI of the MI355X batched EV charging-station simulator.
 *
 * The library advances many independent charging stations by the Chargax
 * transition (Ponse et al., arXiv 2507.01522): per step it applies the agent's
 * per-port power levels (App. A.2 "Apply Actions"), projects them onto the
 * station's capacity tree (Eq. ArchConst), charges the connected cars along the
 * piecewise-linear charging curve (App. A.1 "Car Profiles", App. A.2 "Charge
 * Stationed Cars"), lets time-sensitive users leave (App. A.2 "Departure of
 * Cars"), admits Poisson arrivals first-come-first-served (App. A.2 "Arrival of
 * new Cars", Supp. B.1), computes the profit/penalty reward (App. A.3) and
 * auto-resets stations at the end of the day (Supp. B.1, Table 3).
 *
 * Conventions for every entry point:
 *  - Pointers named *_dev are device memory owned by the caller; they must stay
 *    valid until the context's stream has passed the call.  Pointers named
 *    *_host, specs and descriptor structs are host memory, read during the call.
 *  - All device work is asynchronous on the context's stream (cx_set_stream;
 *    the null stream by default).  cx_synchronize waits for it.
 *  - Errors are returned as cx_status; no exception crosses the ABI.  A failed
 *    kernel launch or device error makes the context sticky-failed
 *    (CX_E_DEVICE from then on).  cx_last_error() gives a thread-local message.
 *  - Determinism: results depend only on the specs, the seed, the env index and
 *    the global step counter g -- not on the launch form, the packing or the
 *    other work sharing the GPU.  Integer outputs are exact; FP32 outputs agree
 *    with an FP64 evaluation of the same equations to ~1e-5 relative.
 *  - A context is used from one thread at a time; the server (cx_server_*) is
 *    thread-safe.
 */
#ifndef CX_H
#define CX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  CX_OK = 0,
  CX_E_INVALID = -1,   /* bad argument or station spec (checked before any device work) */
  CX_E_OOM = -2,       /* device or host allocation failed */
  CX_E_DEVICE = -3,    /* HIP error; sticky for the context */
  CX_E_BUSY = -4,      /* serving: request still running */
  CX_E_BUDGET = -5,    /* serving: request can never fit the memory budget */
  CX_E_CANCELLED = -6, /* serving: request was cancelled */
  CX_E_NOTFOUND = -7   /* serving: unknown ticket */
} cx_status;

/* Where the per-port power levels come from.  A level k in 0..n_levels asks for
 * k / n_levels of the port's maximum power (Supp. B.1: discretisation 10).
 * Ports of a V2G class, and the station battery, also take negative levels
 * -n_levels..-1, asking to discharge |k| / n_levels of the discharge maximum.
 * Levels travel as action bytes: byte = k + lo, where lo = n_levels for a V2G
 * port or the battery and 0 otherwise; a class with a battery has one more
 * action byte per env, after its ports. */
typedef enum {
  CX_ACT_EXTERNAL = 0, /* caller-provided action bytes (above lo + n_levels: clamped)     */
  CX_ACT_RANDOM = 1,   /* uniform bytes from Philox: (h * (lo + n_levels + 1)) >> 16, h a  */
                       /* 16-bit half; one call per action index per 8 steps           */
  CX_ACT_MAX = 2,      /* every port (and the battery) asks for its maximum charge        */
  CX_ACT_POLICY = 3    /* the MLP set by cx_set_policy, a level drawn from its softmax   */
} cx_action_mode;

/* Which per-step records a rollout writes. */
typedef enum {
  CX_OUT_FULL = 0,       /* obs + actions + reward + done */
  CX_OUT_REWARD = 1,     /* reward + done                 */
  CX_OUT_ACT_REWARD = 2  /* actions + reward + done       */
} cx_out_mode;

/* One station architecture and its environment parameters (Sec. 3 "EV Station
 * Layout", App. A.1, Table 3).  The architecture is a tree: internal nodes are
 * splitters / cables / transformers with a power limit and efficiency; node 0
 * is the grid connection and node_parent[i] < i.  Ports (EVSEs) are the leaves
 * and must be listed in depth-first order, i.e. every node's ports are one
 * contiguous range.  All arrays are host memory copied at create.
 * Units: kW, kWh, hours, EUR. */
typedef struct {
  int32_t n_ports;              /* 1..256 */
  int32_t n_nodes;              /* 1..256 */
  const int32_t *node_parent;   /* [n_nodes]; -1 for node 0 */
  const double *node_limit_kw;  /* [n_nodes] > 0 : I_H of Eq. (ArchConst) */
  const double *node_eta;       /* [n_nodes] in (0,1]: eta_H of Eq. (ArchConst) */
  const int32_t *port_parent;   /* [n_ports] node index */
  const double *port_pmax_kw;   /* [n_ports] > 0 : maximum charging rate of the port */
  const double *port_eta;       /* [n_ports] in (0,1]: charging efficiency (App. A.3) */
  double dt_hours;              /* step length (5 min = 1/12) */
  double tau;                   /* charging-curve knee, in (0,1) */
  double p_sell;                /* price charged to car owners, EUR/kWh */
  double p_sell_grid;           /* price when net grid energy <= 0 */
  double fixed_cost;            /* c_dt per step */
  double alpha_sat;             /* weight of c_satisfaction,0 (missing kWh at departure) */
  double alpha_declined;        /* weight of c_declined (rejected cars) */
  int32_t steps_per_episode;    /* 288: one day of 5-minute steps */
  int32_t n_levels;             /* action discretisation (10) */
  double price_base, price_amp, price_sigma; /* p_buy = base + amp sin(2 pi t/S) + sigma z */
  double arrival_peak;          /* Poisson mean at midday: lambda(t) = peak (1 - cos 2 pi t/S)/2 */
  double cap_lo, cap_hi;        /* battery capacity ~ U[cap_lo, cap_hi) kWh */
  double soc0_lo, soc0_hi;      /* arrival SoC ~ U[...)  */
  double tgt_lo, tgt_hi;        /* desired SoC ~ U[...)  */
  double dwell_mu, dwell_sigma; /* stay ~ round(lognormal(mu, sigma)) steps */
  int32_t dwell_max;            /* cap on the stay in steps (<= 4096) */
  /* Optional time-of-day profiles (Sec. 3 "Exogenous State Space", Table 1: the
   * arrival and price data are per step of the day), each steps_per_episode
   * doubles of host memory copied at create, or NULL for the smooth defaults:
   *   arrival_rate[t]  Poisson mean of arrivals at step t of the day, in [0, 8]
   *                    (replaces arrival_peak's curve);
   *   price_table[t]   base buying price per kWh at step t (replaces
   *                    price_base + price_amp sin; the noise sigma z is still added). */
  const double *arrival_rate;
  const double *price_table;
  /* V2G and the station battery (App. A.1 "Endogenous state space", App. A.2
   * "Apply Actions", App. A.3 energy terms and "Battery Degradation").  A V2G
   * port discharges along the charging curve mirrored about SoC = 0.5, never
   * below SoC 0; Eq. (ArchConst) then bounds the magnitude of each node's net
   * power.  The battery is the (N+1)-th pole, at the grid connection outside
   * the capacity tree, with the same (mirrored) curves; it starts every day at
   * battery_soc0.  Grid energy = sum over charging ports of e/eta + sum over
   * discharging ports of eta e + the battery's e. */
  int32_t v2g;                  /* 1: ports also discharge (levels -n_levels..-1)      */
  const double *port_pdis_kw;   /* [n_ports] > 0 discharge maxima, NULL = port_pmax_kw  */
  double battery_kwh;           /* capacity; 0 = no battery                           */
  double battery_kw;            /* its maximum (dis)charging rate r_bar (> 0 if any)   */
  double battery_tau;           /* its charging-curve knee, in (0,1)                   */
  double battery_soc0;          /* its SoC at the start of every day, in [0,1]         */
  double alpha_degrad_battery;  /* weight of c_degrad,battery (energy it discharges)   */
  double alpha_degrad_cars;     /* weight of c_degrad,cars (energy cars feed back)     */
  /* Charge-sensitive users (App. A.1 "User Profiles", App. A.2 "Departure of
   * Cars", App. A.3 c_satisfaction,1): each arriving car's user is charge-
   * sensitive (u = 1) with probability charge_sensitive_share, drawn from
   * Philox (env, g, j, 4) word 0 against an integer threshold.  Such a user
   * leaves at the end of the step in which the energy still wanted reaches zero
   * (e_rem <= 0), not when its planned stay ends: its steps left go negative
   * while it overstays.  On leaving it adds (hours overstayed) - beta_sat1 x
   * (hours left early) to c_satisfaction,1, weighted by alpha_sat1.
   * steps_per_episode must be <= 30000 when the share is > 0. */
  double charge_sensitive_share;  /* in [0,1]; 0 = every user time-sensitive        */
  double alpha_sat1;              /* weight of c_satisfaction,1                      */
  double beta_sat1;               /* its weight of the hours left early              */
  /* Exploring starts (Supp. B.1): n_price_days rows of steps_per_episode base
   * buying prices (host memory, copied at create; NULL / 0 = none).  Each
   * episode uses the row of the day d = (w * n_price_days) >> 32, w = word 0 of
   * Philox (env, g0, 0, 5) where g0 is the global step the episode began on (the
   * noise sigma z is still added); the observation appends [d / n_price_days,
   * 1 if d mod 7 >= 5 (a weekend day) else 0].  Replaces price_table and the
   * default price curve. */
  int32_t n_price_days;
  const double *price_days;
  /* Car models (App. A.1 "Car Profiles": a capacity and a maximum rate per
   * charger type, AC and DC, from a car distribution; both curves share tau):
   * n_car_models (0..8) rows of {probability, capacity kWh, AC rate kW, DC rate
   * kW} (probabilities summing to 1), and port_dc [n_ports] (1 = DC charger;
   * NULL = all AC).  An arriving car's model is the number of cumulative
   * integer thresholds that the capacity word of its CAR draw exceeds; the
   * model fixes its capacity, and its charging curve at port i uses the rate of
   * the port's type (its request is still a share of the port maximum). */
  int32_t n_car_models;
  const double *car_models;
  const int32_t *port_dc;
} cx_station_spec;

typedef struct cx_ctx cx_ctx;

/* Per-step output buffers of a rollout (device memory, caller-owned).  With T
 * steps, record t of every array starts at t * (its per-step size):
 *   obs     float [T][obs_elems]   FULL only; env e at obs_offset(e), 6N+4 floats:
 *           [occupied, SoC, e_rem/C, dwell/S, r_hat/pmax, p_last/pmax] x N ports
 *           (feature-major: feature f of port p at f*N + p), then
 *           [sin 2 pi t/S, cos 2 pi t/S, base price(t), occupied ports / N],
 *           then, with a battery, [battery SoC, battery power / battery_kw],
 *           then, with price days, [episode day / n_price_days, weekend flag],
 *           then, with charge-sensitive users, [u] x N ports (1 = charge-sensitive).
 *           The base price is the episode's day's price with price days.
 *           p_last is negative while a port discharges; dwell/S is negative while a
 *           charge-sensitive user overstays.
 *   actions uint8 [T][total_ports] FULL and ACT_REWARD: the action byte applied per
 *           port (and battery: total_ports counts action bytes).
 *   reward  float [T][n_envs]
 *   done    uint8 [T][n_envs]       1 when the step ended the day (the obs is then the
 *                                   observation of the reset station).
 * A NULL member is not written. */
typedef struct {
  float *obs;
  uint8_t *actions;
  float *reward;
  uint8_t *done;
} cx_traj;

typedef struct {
  int64_t n_envs;
  int64_t total_ports;    /* actions per step */
  int64_t obs_elems;      /* floats of obs per step */
  int32_t n_classes;
  int32_t steps_per_episode;
  uint32_t g;             /* global step counter (advances by every step) */
  int32_t t_day;          /* step within the day, 0..steps_per_episode-1 */
  uint64_t seed;
  size_t state_bytes;     /* size of a cx_get_state snapshot */
  int64_t device_bytes;   /* device memory the context holds */
  int32_t obs_stage;      /* 1: observations go through the LDS stage (cx_set_obs_stage) */
} cx_info;

typedef struct {
  int64_t env_begin, n_envs;     /* the class's env range */
  int64_t port_offset;           /* actions offset of its first env */
  int64_t obs_offset;            /* obs offset of its first env */
  int32_t n_ports, obs_dim;
  int32_t slots;                 /* ports padded to the aligned power-of-two layout */
  int32_t levels;                /* depth of the capacity tree (levels incl. root) */
  int32_t lanes_per_station;     /* current packing: lanes per station */
  int32_t waves_per_block;
  int32_t n_actions;             /* action bytes per env: n_ports (+1 with a battery) */
} cx_class_info;

/* Create a context of n_envs stations of one class (Sec. 3 "EV Station
 * Layout": the capacity tree of Eq. (ArchConst); App. A.1: the endogenous
 * per-port and exogenous state), state = empty stations at t_day = 0, g = 0.
 * seed keys every Philox draw.  spec: host memory, read during the call and
 * copied; *out receives the context, owned by the caller until cx_destroy.
 * The spec is validated here (CX_E_INVALID with a message, nothing allocated);
 * CX_E_OOM if the device state cannot be allocated.  No later call re-checks
 * the spec. */
cx_status cx_create(const cx_station_spec *spec, int64_t n_envs, uint64_t seed, cx_ctx **out);

/* Create a context with several station classes (the uneven-batching form;
 * each class as in cx_create, Sec. 3 and App. A.1): env e has class
 * env_class[e] (host memory, n_envs entries); env_class must be non-decreasing
 * so that every class is one contiguous env range.  All specs must share
 * steps_per_episode.  Errors as for cx_create. */
cx_status cx_create_multi(const cx_station_spec *specs, int32_t n_specs, const int32_t *env_class,
                          int64_t n_envs, uint64_t seed, cx_ctx **out);

/* Use this HIP stream (hipStream_t passed as void*) for all later device work. */
cx_status cx_set_stream(cx_ctx *ctx, void *hip_stream);

/* The layout of a context's records and state (host-side introspection, no
 * device work): cx_get_info fills *info (host) with the totals -- envs, action
 * bytes and observation floats per step, the clock, the snapshot size, the
 * device bytes held; cx_get_class_info fills *info with class cls's env range,
 * its offsets inside a step's action and observation records, its observation
 * length, slot layout, tree depth and current packing.  Together they give, for
 * env e of class c, its actions at port_offset + (e - env_begin) n_actions and
 * its observation at obs_offset + (e - env_begin) obs_dim of every step.
 * CX_E_INVALID for a NULL argument or a class out of range. */
cx_status cx_get_info(const cx_ctx *ctx, cx_info *info);
cx_status cx_get_class_info(const cx_ctx *ctx, int32_t cls, cx_class_info *info);

/* Reset at the start of an episode (Supp. B.1: episodes are one day; Table 3):
 * empty every station, set t_day = 0, the returns to 0 and the station
 * batteries to battery_soc0; g is kept, so a new day draws new noise (and, with
 * price days, a new exploring-start day).  obs_dev (nullable, device, caller-
 * owned, obs_elems floats) receives the reset observation in the obs layout of
 * one step.  Asynchronous on the context's stream. */
cx_status cx_reset(cx_ctx *ctx, float *obs_dev);

/* One environment step (App. A.2 in its order: (i) apply actions -- clip by the
 * port maximum, the charging curve and the battery room, then Eq. (ArchConst)
 * over the capacity tree; (ii) charge stationed cars; (iii) departures; (iv)
 * arrivals first-come-first-served; then the reward of App. A.3 and, at the
 * end of the day, the auto-reset of Supp. B.1), one kernel launch, state read
 * from and written back to HBM (the plain form).  actions_dev: device, caller-
 * owned action bytes [total_ports] (EXTERNAL; bytes above the largest level
 * are clamped).  obs/reward/done receive one record each (layouts of cx_traj
 * with T = 1); obs_dev may be NULL.  CX_E_INVALID for a NULL actions_dev;
 * CX_E_DEVICE (sticky) if the launch fails. */
cx_status cx_step(cx_ctx *ctx, const uint8_t *actions_dev, float *obs_dev, float *reward_dev,
                  uint8_t *done_dev);

/* cx_step (App. A.2 (i)-(iv), App. A.3, Supp. B.1) with any action mode and
 * every output of cx_traj (T = 1).  actions_in_dev is read only for
 * CX_ACT_EXTERNAL; out (host struct of device pointers, nullable members). */
cx_status cx_step_ex(cx_ctx *ctx, cx_action_mode mode, const uint8_t *actions_in_dev,
                     const cx_traj *out);

/* T steps (each one step of App. A.2 (i)-(iv) and App. A.3, with the auto-reset
 * of Supp. B.1 at every day end) in one persistent launch: each wave keeps its
 * stations' state in registers for all T steps and streams the records
 * selected by out_mode to *out (device buffers, caller-owned, layouts of
 * cx_traj; NULL members are not written).  actions_in_dev ([T][total_ports] uint8) is read only for EXTERNAL.
 * The launch is captured once per (T, modes, buffers) into a HIP graph and
 * replayed.  Results equal T calls of cx_step_ex.
 * CX_ACT_POLICY draws every step's levels from the policy (cx_set_policy) on
 * the observation of the state before the step.  For a SIMPLE class of 8, 16
 * or 32 slots (uniform per-level limits, no padding) the whole rollout is one
 * launch of a fused persistent kernel that runs the perceptron between steps,
 * its observations only in on-chip memory; other classes run, per step, the
 * policy kernel (observation -> levels, as cx_policy_sample) and then the
 * one-step kernel with those levels, the observations in between in a scratch
 * buffer of the context unless out_mode is FULL.  Both compute the same
 * products in the same order, so their records are the same.  The rollout
 * starts from the observation of the current state (as cx_observe).  With
 * CX_OUT_FULL, out->obs must be 16-byte aligned.  Requires cx_set_policy. */
cx_status cx_rollout(cx_ctx *ctx, int32_t T, cx_action_mode mode, cx_out_mode out_mode,
                     const uint8_t *actions_in_dev, const cx_traj *out);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): cx_rollout
 * in CX_ACT_POLICY mode whose per-step scratch -- one step of observations
 * (obs_elems floats, rounded up to 256 bytes) and one step of levels
 * (total_ports bytes) -- lives in a fixed array of the library's device image,
 * CX_NOALLOC_SCRATCH_BYTES per GPU, held until the process ends, instead of a
 * buffer the context allocates.  The call allocates nothing (no hipMalloc, no
 * hipFree, no allocating library routine) and always runs the two kernels per
 * step, whose records are bit for bit those of cx_rollout with CX_ACT_POLICY
 * on an equal context (fused or not).  The caller passes the outputs (out, as
 * for cx_rollout) and must have created the context and set its policy
 * beforehand.  CX_E_INVALID (nothing launched) if the context needs more
 * scratch than the fixed size (about 41,000 envs of 32 ports) or has no policy.
 * Every call on one GPU shares that GPU's array, which keeps the last call's
 * contents; nothing in it needs clearing (each element is written before it is
 * read), but calls that overlap on one GPU (several contexts or streams at
 * once) race on it and must be serialised by the caller.  The array's address
 * is looked up on the first call on each device. */
#define CX_NOALLOC_SCRATCH_BYTES 33554432
cx_status cx_rollout_policy_noalloc(cx_ctx *ctx, int32_t T, cx_out_mode out_mode, const cx_traj *out);

/* Policy for CX_ACT_POLICY: a two-layer perceptron obs -> hidden (tanh) ->
 * n_ports*(n_levels+1) logits, BF16 weights (uint16 bit patterns, host memory):
 * w1 [obs_dim][hidden], b1 [hidden], w2 [hidden][n_ports*(n_levels+1)], b2.
 * Products run on the matrix cores in BF16 with FP32 accumulation; the level of
 * each port is drawn from the softmax of its logits: the first level whose
 * cumulative probability exceeds u, u = (top 24 bits of word (port / 16) mod 4
 * of Philox (env, g, port mod 16 + 16 (port / 64), 3) + 1/2) 2^-24 (ports 16
 * apart share a Philox call).
 * Only single-class contexts of charging-only stations (no V2G, no battery). */
cx_status cx_set_policy(cx_ctx *ctx, int32_t hidden, const uint16_t *w1_host, const uint16_t *b1_host,
                        const uint16_t *w2_host, const uint16_t *b2_host);

/* Logits of the policy for n observations (obs_dev [n][obs_dim] float) into
 * logits_dev [n][n_ports*(n_levels+1)] float: the policy's first half alone. */
cx_status cx_policy_logits(cx_ctx *ctx, const float *obs_dev, int64_t n, float *logits_dev);

/* Levels the policy samples for n observations (obs_dev [n][obs_dim] float,
 * 16-byte aligned) at global step g: act_dev [n][n_ports] uint8, the uniforms
 * from Philox counters (env_begin + i, g, ...) of the context's seed -- the
 * policy half of a CX_ACT_POLICY step, exactly as a rollout launches it. */
cx_status cx_policy_sample(cx_ctx *ctx, const float *obs_dev, int64_t n, uint32_t g, uint8_t *act_dev);

/* Observation of the current state of every station (the record layout of
 * cx_traj.obs for one step, Sec. 3 state features): what a policy sees before
 * the next step.  obs_dev: obs_elems floats of device memory, caller-owned. */
cx_status cx_observe(cx_ctx *ctx, float *obs_dev);

/* Snapshot / restore of the whole state (the endogenous state of App. A.1 --
 * per port the car's SoC, target, capacity, stay and last power, the user
 * type; per env the return and the station battery -- plus g and t_day) in a
 * packing-independent host format of cx_info.state_bytes bytes (host memory,
 * caller-owned; CX_E_INVALID if bytes is smaller or, for cx_set_state, the
 * snapshot does not match the context or holds out-of-range values), bit-exact, so a restored context
 * continues exactly as the original.  Both calls synchronise the context's
 * stream.  Format (little endian):
 *   u64 magic 0x33305843 ('CX03'), i64 n_envs, i64 ports (sum of n_ports over
 *   the envs), u32 g, i32 t_day,
 *   then per port in env/port order (29 bytes): i32 dwell (steps left; <= 0 only
 *   for a charge-sensitive user), f64 1 - SoC, f32 1 - target SoC, f32 battery
 *   capacity C, f32 last power, u8 user (1 = charge-sensitive; a port is empty
 *   when dwell <= 0 and user = 0), f32 the car's maximum rate at this port
 *   (classes with car models; 0 otherwise);
 *   then per env: f64 return; then per env of a class with a station battery,
 *   in env order (12 bytes): f64 battery SoC, f32 battery last power.
 *   The energy still wanted is (target - SoC) * C.  An empty port is all zeros. */
cx_status cx_get_state(cx_ctx *ctx, void *host, size_t bytes);
cx_status cx_set_state(cx_ctx *ctx, const void *host, size_t bytes);

/* Copies of class cls's integer sampling tables, as built on the host in FP64:
 * tpois_host [steps_per_episode][24] (arrival thresholds), tdwell_host
 * [dwell_max] (entry 0 unused).  Either pointer may be NULL. */
cx_status cx_get_tables(const cx_ctx *ctx, int32_t cls, uint32_t *tpois_host, uint32_t *tdwell_host);

/* Packing of class cls: lanes per station (a power of two, 4..64, dividing or
 * equal to the padded slot count / 1, 2 or 4 slots per lane) and waves per
 * block (1..8).  Results do not depend on it beyond FP32 rounding order. */
cx_status cx_set_packing(cx_ctx *ctx, int32_t cls, int32_t lanes_per_station, int32_t waves_per_block);

/* on = 1: classes without padding slots, with one port maximum and efficiency
 * and one block size per tree level write their observation records through an
 * LDS stage of each block, as 16-byte stores of whole record runs; on = 0 (the
 * default): every lane stores its own values.  The records are bit for bit the
 * same either way; which is faster depends on the launch (a mixed launch of
 * many classes gains).  CX_E_INVALID unless on is 0 or 1. */
cx_status cx_set_obs_stage(cx_ctx *ctx, int32_t on);

/* Time every legal packing of every class on a T_probe-step rollout (state is
 * saved and restored) and keep the fastest, then every pair of waves per block
 * and observation stage (cx_set_obs_stage) likewise.  cache_path (nullable) is a
 * JSON file of earlier results keyed by class shape, read first and updated.
 * Currently switched off: it returns CX_E_INVALID without touching the context,
 * because one call aborted the process inside it with no diagnostic and the
 * cause has not been found.  Set packings with cx_set_packing and the stage
 * with cx_set_obs_stage instead. */
cx_status cx_autotune(cx_ctx *ctx, int32_t T_probe, const char *cache_path);

cx_status cx_synchronize(cx_ctx *ctx);
const char *cx_last_error(void);
void cx_destroy(cx_ctx *ctx);

/* ---- serving: continuous batching of rollout requests ---------------------
 * A server owns a memory budget on the current device and a scheduler thread.
 * A request is one station class, n_envs stations, a horizon of T steps, a
 * seed, an action mode (RANDOM or MAX) and an output mode; its stations start
 * empty at t_day = 0 with their own step counter g = 0, and its Philox counters
 * use request-local env indices, so its results depend on nothing else that
 * runs.  Requests are admitted first-come-first-served as soon as their state
 * (and their outputs, when the server allocates them) fit the budget; every
 * launch advances all admitted requests together by up to chunk_steps steps,
 * so requests that arrive while others run join at the next chunk boundary.
 * A request's results are bit-identical alone or in any mix. */
typedef struct cx_server cx_server;

typedef struct {
  int32_t chunk_steps;      /* steps per launch (default 144) */
  int32_t max_active;       /* cap on concurrently admitted requests (default 256) */
  int32_t waves_per_block;  /* default 4 */
  int32_t simulate_ns;      /* 0: run on the GPU.  > 0: no device is touched and a chunk
                               takes simulate_ns per env-step on a host clock -- for
                               testing the scheduler without a GPU */
} cx_server_opts;

typedef struct {
  cx_station_spec spec;     /* copied at submit (validated there: CX_E_INVALID) */
  int64_t n_envs;           /* >= 1 */
  int32_t T;                /* >= 1 */
  uint64_t seed;
  cx_out_mode out_mode;
  cx_action_mode act_mode;  /* CX_ACT_RANDOM or CX_ACT_MAX */
  cx_traj out;              /* optional caller-owned device buffers (layouts of cx_traj with
                               this request's n_envs and T); members left NULL that out_mode
                               needs are allocated by the server and count against the budget */
} cx_request;

typedef struct {
  cx_status status;         /* CX_OK when finished, CX_E_CANCELLED, or CX_E_DEVICE */
  int64_t n_envs;
  int32_t T;
  cx_traj traj;             /* where the records are: caller buffers, or server buffers that
                               stay valid until cx_release */
  double submit_s, admit_s, done_s;  /* server clock (seconds since create) */
  int64_t bytes;            /* device bytes held for the request */
} cx_result;

/* Budget: device bytes the server may hold for admitted requests, reserved on
 * the device at create (CX_E_OOM if it cannot be) as one arena; each admitted
 * request takes one contiguous block of it (first fit) until released.  A
 * request that could never fit is refused at submit with CX_E_BUDGET. */
cx_status cx_server_create(size_t hbm_budget_bytes, const cx_server_opts *opts, cx_server **out);
cx_status cx_submit(cx_server *s, const cx_request *req, uint64_t *ticket);
cx_status cx_poll(cx_server *s, uint64_t ticket, cx_result *res);   /* CX_E_BUSY while queued/running */
cx_status cx_wait(cx_server *s, uint64_t ticket, cx_result *res);   /* blocks until done/cancelled */
/* Cancel: a queued request is dropped at once; a running one at its next chunk
 * boundary.  Its result then has status CX_E_CANCELLED. */
cx_status cx_cancel(cx_server *s, uint64_t ticket);
/* Release a finished or cancelled request: its device memory returns to the
 * budget and the ticket becomes unknown (CX_E_NOTFOUND). */
cx_status cx_release(cx_server *s, uint64_t ticket);
/* Totals since create: GPU time of the launched chunks, env-steps completed,
 * number of chunk launches, and the peak of concurrently admitted requests. */
cx_status cx_server_stats(cx_server *s, double *busy_s, int64_t *env_steps, int64_t *launches,
                          int32_t *peak_active);
void cx_server_destroy(cx_server *s);

#ifdef __cplusplus
}
#endif
#endif
