/*
 * cx_oracle.h -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, scalar FP64 simulator of the batched EV charging-station step
 * of Chargax (Ponse, Kleuker, Plaat, Moerland, arXiv 2507.01522).  It is the
 * parity oracle for the HIP library and shares no code with it: its own Philox,
 * its own sampling tables, its own tree handling.  Only the tests, the smoke
 * entry point and the benchmark's CPU-baseline leg may load it.
 *
 * Paper map (section / equation):
 *   exogenous draws   -- App. A.1 "Exogenous state space" (arrival data, car and
 *                        user profiles), Supp. B.1 (Poisson arrivals), Sec. 3
 *                        "Exogenous State Space" (grid prices)
 *   actions           -- Sec. 3 "Action Space", Supp. B.1 (discretised levels)
 *   apply actions     -- App. A.2 "Apply Actions" and Eq. (ArchConst)
 *   charge            -- App. A.2 "Charge Stationed Cars"; charging curve of
 *                        App. A.1 "Car Profiles"
 *   departures        -- App. A.2 "Departure of Cars"
 *   arrivals          -- App. A.2 "Arrival of new Cars"
 *   reward            -- App. A.3 (energy terms, profit Pi, r = Pi - sum alpha c,
 *                        c_satisfaction,0 and c_declined)
 *   episodes          -- Supp. B.1 (24 h episodes), Table 3
 *
 * What pins each function (tests/test_oracle_*.py):
 *   ox_philox4x32_10  -- published Random123 known-answer vectors; rocRAND's
 *                        independent implementation on 2000 random inputs
 *   tables            -- scipy Poisson / lognormal CDFs (within 2^-32)
 *   ox_draw_exo       -- statistics: daily arrivals 43.2, P(M=0)=exp(-lambda),
 *                        uniform car attributes (KS), dwell pmf (chi-square),
 *                        standard-normal noise (KS), daily mean price
 *   ox_draw_actions   -- uniform levels (chi-square); MAX and EXTERNAL exact
 *   ox_project        -- textbook scaling for one node; brute force over all
 *                        11^n actions on six tiny trees (feasible, identity
 *                        when feasible, equal factors per ancestor set, a
 *                        binding constraint above every scaled leaf, monotone)
 *   ox_transition     -- five hand-worked cases; closed-form charge curve;
 *                        dwell timing; day boundary; rollout invariants
 *                        (limits, SoC range, energy balance, occupancy)
 *   ox_policy         -- numpy FP64 products on the decoded BF16 operands;
 *                        sampled level frequencies equal softmax (chi-square);
 *                        BF16 rounding equal to torch's
 *   charge-sensitive  -- (tests/test_oracle_users.py) hand-worked departures on
 *   users (u = 1)        reaching the target, overstay and early-leave terms of
 *                        c_satisfaction,1, share of drawn users (binomial), the
 *                        all-time-sensitive special case equal to the base model
 *   car models        -- (tests/test_oracle_cars.py) model frequencies (chi-square),
 *   (AC / DC)            hand-worked AC and DC clips, the one-model special case
 *                        equal to the base model, P <= the car's rate
 *   exploring starts  -- (tests/test_oracle_days.py) uniform day draws, prices
 *                        following the drawn day's row, a new day at each
 *                        episode, one price day = the per-step price table
 *   V2G / battery     -- (tests/test_oracle_v2g.py) mirror symmetry: a mirrored
 *                        state (SoC -> 1 - SoC) under negated levels draws exactly
 *                        the negated powers through clip and projection;
 *                        hand-worked discharge, projection and energy cases;
 *                        the battery equals a V2G port holding a car of the
 *                        battery's size; uniform signed levels (chi-square)
 *
 * All quantities: power in kW, energy in kWh, time step dt in hours.  The fixed
 * EVSE voltage of Sec. 3 cancels, so currents and powers are interchangeable.
 */
#ifndef CX_ORACLE_H
#define CX_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define OX_K_POIS 24        /* arrival counts are capped at 24 per step          */
#define OX_MAX_PORTS 1024
#define OX_MAX_NODES 1024

/* Philox counter domains (word 3 of the counter). */
#define OX_DOM_ENV 0u       /* ctr = (env, g, 0, 0): arrivals + price noise      */
#define OX_DOM_ACT 1u       /* ctr = (env, g >> 3, port, 1): half g & 7 of 8    */
#define OX_DOM_CAR 2u       /* ctr = (env, g, j, 2): j-th arriving car of step g */
#define OX_DOM_GUM 3u       /* ctr = (env, g, port % 16 + 16 (port / 64), 3): the policy's draw, word (port / 16) % 4 */
#define OX_DOM_USER 4u      /* ctr = (env, g, j, 4): user type of car j, word 0  */
#define OX_DOM_DAY 5u       /* ctr = (env, g0, 0, 5): price day of the episode starting at g0 */

/* action modes */
#define OX_ACT_EXTERNAL 0
#define OX_ACT_RANDOM 1
#define OX_ACT_MAX 2

/* indices into the double parameter vector handed to ox_class_new */
enum {
  OXP_DT = 0, OXP_TAU, OXP_P_SELL, OXP_P_SELL_GRID, OXP_FIXED_COST, OXP_ALPHA_SAT,
  OXP_ALPHA_DEC, OXP_PRICE_BASE, OXP_PRICE_AMP, OXP_PRICE_SIGMA, OXP_ARRIVAL_PEAK,
  OXP_CAP_LO, OXP_CAP_HI, OXP_SOC0_LO, OXP_SOC0_HI, OXP_TGT_LO, OXP_TGT_HI,
  OXP_DWELL_MU, OXP_DWELL_SIGMA, OXP_COUNT
};
/* indices into the int parameter vector */
enum { OXI_STEPS_PER_EPISODE = 0, OXI_N_LEVELS, OXI_DWELL_MAX, OXI_COUNT };

typedef struct ox_class ox_class;

/* Exogenous draws of one env-step (agent independent; App. A.1). */
typedef struct {
  int32_t M;                      /* arriving cars this step, 0..24             */
  double z;                       /* standard normal price noise                */
  double p_buy;                   /* grid buy price                             */
  double car_cap[OX_K_POIS];      /* battery capacity C of car j (kWh)          */
  double car_soc[OX_K_POIS];      /* arrival SoC_0 of car j                     */
  double car_tgt[OX_K_POIS];      /* desired SoC of car j                       */
  int32_t car_dwell[OX_K_POIS];   /* dwell time of car j in steps, >= 1         */
  int32_t car_user[OX_K_POIS];    /* 1: charge-sensitive user (u = 1), else 0   */
  int32_t day, day_next;          /* price day of this step's episode and of the next
                                     step's (-1 without price days)                */
  int32_t car_model[OX_K_POIS];   /* car model of car j (-1 without car models)   */
} ox_exo;

/* Everything one transition reports besides the new state.  e_grid is the net
 * grid energy (grid -> cars + cars -> grid + battery), e_to_grid the (<= 0)
 * energy discharged cars feed back, e_batt the battery's (signed) energy. */
typedef struct {
  double reward, profit, e_net, e_grid, c_sat;
  int32_t M, acc, rej, n_dep, done, n_occ;
  double e_to_grid, e_batt, c_sat1;
} ox_step_info;

/* ---- class (one station architecture + parameters) ---- */
ox_class *ox_class_new(int32_t n_ports, int32_t n_nodes, const int32_t *node_parent,
                       const double *node_limit, const double *node_eta,
                       const int32_t *port_parent, const double *port_pmax,
                       const double *port_eta, const double *params, const int32_t *iparams);
void ox_class_free(ox_class *c);
/* Time-of-day profiles (Sec. 3 "Exogenous State Space", Table 1): per step of the
 * day, the Poisson mean of arrivals and the base buying price; NULL keeps the
 * default curves.  Rebuilds the arrival thresholds. */
void ox_class_set_profiles(ox_class *c, const double *arrival_rate, const double *price_table);
/* V2G and the station battery (App. A.1 "Endogenous state space", App. A.2
 * "Apply Actions", App. A.3).  v2g = 1 lets ports discharge: levels -L..L, a
 * negative level asking for |k|/L of the port's discharge maximum pdis[i]
 * (NULL = the port maximum).  batt = {capacity kWh (0 = no battery), maximum
 * rate kW, tau, SoC at the start of a day, alpha_degrad_battery,
 * alpha_degrad_cars}. */
void ox_class_set_v2g(ox_class *c, int32_t v2g, const double *pdis, const double *batt);
/* Charge-sensitive users (App. A.1 "User Profiles", App. A.2 "Departure of
 * Cars", App. A.3 c_satisfaction,1): each arriving car's user is charge-
 * sensitive with probability share; such a user leaves when the energy still
 * wanted reaches zero, and c_satisfaction,1 (weight alpha) charges the hours
 * stayed past the planned departure minus beta times the hours left early. */
void ox_class_set_users(ox_class *c, double share, double alpha, double beta);
/* Exploring starts (Supp. B.1): n_days rows of steps_per_episode base buying
 * prices; every episode uses the row of a day drawn at its start, and the
 * observation shows that day (day / n_days) and whether it is a weekend day
 * (day mod 7 >= 5). */
void ox_class_set_price_days(ox_class *c, int32_t n_days, const double *price_days);
/* Car models (App. A.1 "Car Profiles": each car has a capacity and a maximum
 * rate per charger type, AC and DC; both curves share tau): n_models rows of
 * {probability, capacity kWh, AC rate kW, DC rate kW}; port_dc[i] = 1 marks a
 * DC port (NULL: all AC).  An arriving car's model replaces the uniform
 * capacity draw (same Philox word), and its curve at port i uses the rate of
 * the port's type instead of the port maximum. */
void ox_class_set_car_models(ox_class *c, int32_t n_models, const double *models, const int32_t *port_dc);
/* The price day of the episode that started at global step g0 (-1 without days). */
int32_t ox_episode_day(const ox_class *c, uint64_t seed, uint32_t env, uint32_t g0);
int32_t ox_class_ports(const ox_class *c);
int32_t ox_class_actions(const ox_class *c);  /* ports + 1 with a battery */
int32_t ox_obs_dim(const ox_class *c);        /* 6 N + 4, + 2 with a battery, + 2 with price
                                                 days, + N with u = 1 users */
/* The action byte of level k at action index i (i = n_ports: the battery). */
int32_t ox_action_code(const ox_class *c, int32_t i, int32_t k);
/* copies of the class's integer sampling tables (steps_per_episode x 24, dwell_max) */
void ox_class_tables(const ox_class *c, uint32_t *tpois, uint32_t *tdwell);

/* ---- primitives ---- */
void ox_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
double ox_u24(uint32_t w);  /* (w >> 8) * 2^-24 */

/* Apply-actions step: clip by port maximum, charging curve and remaining capacity,
 * then project onto the architecture constraints.  P (n_ports) is written.
 * A port is occupied when dwell > 0 or it holds a charge-sensitive user
 * (user[i] = 1; user may be NULL: all time-sensitive).  rbar[i] is the car's
 * maximum rate at port i (NULL: the port maximum, the base model). */
void ox_apply_actions(const ox_class *c, const int32_t *dwell, const int32_t *user, const double *soc,
                      const double *cap, const double *rbar, const int32_t *k, double *P);
/* The projection of Eq. (ArchConst) alone, in place on P. */
void ox_project(const ox_class *c, double *P);

/* The battery's power for level kb at state-of-charge soc_b (0 without one). */
double ox_battery_power(const ox_class *c, double soc_b, int32_t kb);

void ox_draw_exo(const ox_class *c, uint64_t seed, uint32_t env, uint32_t g, int32_t t_day,
                 ox_exo *x);
/* Signed levels of every action index (ox_class_actions entries: the ports,
 * then the battery).  ext holds action bytes (EXTERNAL). */
void ox_draw_actions(const ox_class *c, int32_t mode, uint64_t seed, uint32_t env, uint32_t g,
                     const uint8_t *ext, int32_t *k);

/* One transition of one env, state in place.  user[i] = 1 marks a charge-
 * sensitive user at port i (dwell may then be <= 0: time past the planned
 * departure).  batt = {SoC, last power} of the station battery (NULL without
 * one).  obs (obs_dim) may be NULL; P_out (n_ports) receives the applied powers
 * and may be NULL. */
void ox_transition(const ox_class *c, int32_t *dwell, int32_t *user, double *soc, double *e_rem,
                   double *cap, double *rbar, double *p_last, double *batt, double *ret, int32_t *t_day,
                   const int32_t *k, const ox_exo *x, ox_step_info *info, double *obs, double *P_out);
/* Observation of the current state (used after reset and by the policy). */
void ox_observe(const ox_class *c, const int32_t *dwell, const int32_t *user, const double *soc,
                const double *e_rem, const double *cap, const double *rbar, const double *p_last,
                const double *batt, int32_t t_day, int32_t day, double *obs);

/* ---- batched rollout over many envs (threads over env ranges) ----
 * env_class[n_envs] indexes classes[]; envs may be in any class order.  State
 * arrays are port-major per env, envs concatenated (port offset = prefix sum of
 * the envs' port counts; rbar: the car's rate per port, kept for classes with car
 * models); batt holds {SoC, last power} per env (2 n_envs
 * doubles, used by battery classes only; may be NULL if no class has one).
 * Outputs are time-major:
 *   obs    [T][sum_e obs_dim(e)]   (may be NULL)
 *   act    [T][sum_e actions(e)]   action bytes (may be NULL)
 *   reward [T][n_envs], done [T][n_envs]  (may be NULL)
 *   info   [T][n_envs] (may be NULL)
 * act_in (EXTERNAL mode) has the act layout.  g and t_day are common to all envs
 * and are advanced.  env_ids (may be NULL = 0..n_envs-1) gives each env's index
 * in the Philox counters, so a subset of a large batch can be replayed.
 * Returns the number of threads used. */
int32_t ox_rollout(ox_class *const *classes, const int32_t *env_class, const int64_t *env_ids,
                   int64_t n_envs,
                   uint64_t seed, uint32_t *g, int32_t *t_day, int32_t T, int32_t mode,
                   const uint8_t *act_in, int32_t *dwell, int32_t *user, double *soc, double *e_rem,
                   double *cap, double *rbar, double *p_last, double *batt, double *ret, double *obs, uint8_t *act,
                   double *reward, uint8_t *done, ox_step_info *info, int32_t n_threads);

/* ---- policy (observation -> MLP -> a level per port drawn from softmax) ----
 * Weights are BF16 bit patterns; W1 [in][hidden], W2 [hidden][n_ports*(L+1)].
 * The observation is rounded to BF16 first and the hidden activation after tanh;
 * both products are taken in FP64.  Level of port i: the first l whose
 * cumulative softmax probability F_l exceeds u (level L if none), u = (top 24
 * bits of word 0 of Philox (env, g, i, 3) + 1/2) 2^-24.  logits
 * (n_ports*(L+1)) and margin (n_ports: distance of u from the nearest F_l, l <
 * L) may be NULL. */
void ox_policy(const ox_class *c, int32_t hidden, const uint16_t *w1, const uint16_t *b1,
               const uint16_t *w2, const uint16_t *b2, const double *obs, uint64_t seed,
               uint32_t env, uint32_t g, double *logits, int32_t *k, double *margin);
double ox_bf16_round(double x);

#ifdef __cplusplus
}
#endif
#endif
