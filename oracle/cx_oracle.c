/*
 * cx_oracle.c -- TEST INFRASTRUCTURE ONLY (see cx_oracle.h).
 *
 * Plain scalar FP64 implementation of one Chargax environment step, written from
 * the paper's Appendix A.  Nothing here is blocked, fused or reordered beyond
 * what the equations state; each env is simulated on its own.  Build flags keep
 * IEEE semantics: -O3 -ffp-contract=off, no fast-math.
 */
#include "cx_oracle.h"

#include <math.h>
#include <pthread.h>
#include <stdlib.h>
#include <string.h>

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

struct ox_class {
  int32_t n_ports, n_nodes, max_depth;
  int32_t *node_parent, *node_depth;
  double *node_cap;          /* eta_H * I_H: the right side of Eq. (ArchConst) times eta_H */
  unsigned char *anc;        /* anc[h * n_ports + i] = 1 iff node h lies on port i's path   */
  double *pmax, *peta;
  double *pdis;              /* discharge maximum per port (V2G) */
  int32_t v2g;               /* 1: ports take levels -L..L */
  double b_cap, b_rate, b_tau, b_soc0, a_db, a_dc;  /* battery (b_cap = 0: none), degradation weights */
  double cs_share, a_sat1, beta1;  /* charge-sensitive users: share of arrivals, weight, beta */
  int32_t n_days;            /* exploring starts: price days (0: none) */
  int32_t n_models;          /* car models (0: none) */
  uint32_t model_thresh[8];  /* cumulative thresholds: model = #{m : w > model_thresh[m]} */
  double model_cap[8], model_rac[8], model_rdc[8];
  int32_t *port_dc;          /* [n_ports] 1 = DC charger */
  double *price_days;        /* [n_days][steps_per_episode] */
  uint32_t cs_thresh;        /* a car's user is charge-sensitive iff its word <= cs_thresh (share > 0) */
  double p[OXP_COUNT];
  int32_t ip[OXI_COUNT];
  uint32_t *tpois;           /* [steps_per_episode][24] */
  double *lam;               /* [steps_per_episode] Poisson mean of arrivals per step of the day */
  double *price;             /* [steps_per_episode] base buying price per step of the day */
  uint32_t *tdwell;          /* [dwell_max], entry 0 unused */
};

static int32_t has_days(const ox_class *c) { return c->n_days > 0; }

/* ------------------------------------------------------------------------- */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy
 * as 1, 2, 3", SC'11): ten rounds of two 32x32->64 multiplies with the round
 * keys bumped by the Weyl constants between rounds.                          */
void ox_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  const uint32_t m0 = 0xD2511F53u, m1 = 0xCD9E8D57u;
  const uint32_t w0 = 0x9E3779B9u, w1 = 0xBB67AE85u;
  uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int round = 0; round < 10; ++round) {
    if (round > 0) {
      k0 += w0;
      k1 += w1;
    }
    uint64_t prod0 = (uint64_t)m0 * (uint64_t)x0;
    uint64_t prod1 = (uint64_t)m1 * (uint64_t)x2;
    uint32_t y0 = (uint32_t)(prod1 >> 32) ^ x1 ^ k0;
    uint32_t y1 = (uint32_t)prod1;
    uint32_t y2 = (uint32_t)(prod0 >> 32) ^ x3 ^ k1;
    uint32_t y3 = (uint32_t)prod0;
    x0 = y0; x1 = y1; x2 = y2; x3 = y3;
  }
  out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

static void philox_seeded(uint64_t seed, uint32_t a, uint32_t b, uint32_t c, uint32_t d,
                          uint32_t out[4]) {
  uint32_t ctr[4] = {a, b, c, d};
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  ox_philox4x32_10(ctr, key, out);
}

double ox_u24(uint32_t w) { return (double)(w >> 8) * (1.0 / 16777216.0); }

/* ------------------------------------------------------------------------- */
/* Integer thresholds: T = clamp(ceil(2^32 * F) - 1, 0, 2^32 - 1), so that for a
 * uniform 32-bit word w, P(w <= T) = (T + 1) / 2^32 ~= F.                     */
static uint32_t threshold_u32(double cdf) {
  double x = ceil(cdf * 4294967296.0) - 1.0;
  if (x < 0.0) x = 0.0;
  if (x > 4294967295.0) x = 4294967295.0;
  return (uint32_t)x;
}

/* Arrival counts, Supp. B.1: M(t) ~ Poisson(lambda(t)), lambda(t) the mean of
 * step t of the day (c->lam: the given per-step table, else the synthetic
 * average peak * (1 - cos(2 pi t / S)) / 2 in place of the bundled data).  The
 * CDF is accumulated with the pmf recurrence. */
static void build_tpois(ox_class *c) {
  const int32_t S = c->ip[OXI_STEPS_PER_EPISODE];
  for (int32_t t = 0; t < S; ++t) {
    double lam = c->lam[t];
    double pmf = exp(-lam);
    double cdf = pmf;
    for (int32_t k = 0; k < OX_K_POIS; ++k) {
      if (k > 0) {
        pmf = pmf * lam / (double)k;
        cdf = cdf + pmf;
      }
      c->tpois[t * OX_K_POIS + k] = threshold_u32(cdf);
    }
  }
}

void ox_class_set_users(ox_class *c, double share, double alpha, double beta) {
  c->cs_share = share;
  c->a_sat1 = alpha;
  c->beta1 = beta;
  c->cs_thresh = threshold_u32(share);
}

void ox_class_set_price_days(ox_class *c, int32_t n_days, const double *price_days) {
  const int32_t S = c->ip[OXI_STEPS_PER_EPISODE];
  free(c->price_days);
  c->n_days = n_days;
  c->price_days = (double *)malloc(sizeof(double) * (size_t)n_days * S);
  memcpy(c->price_days, price_days, sizeof(double) * (size_t)n_days * S);
}

void ox_class_set_car_models(ox_class *c, int32_t n_models, const double *models, const int32_t *port_dc) {
  c->n_models = n_models;
  double F = 0.0;
  for (int32_t m = 0; m < n_models; ++m) {
    F += models[4 * m + 0];
    /* the last model takes all the remaining mass */
    c->model_thresh[m] = m + 1 == n_models ? 0xFFFFFFFFu : threshold_u32(F);
    c->model_cap[m] = models[4 * m + 1];
    c->model_rac[m] = models[4 * m + 2];
    c->model_rdc[m] = models[4 * m + 3];
  }
  free(c->port_dc);
  c->port_dc = (int32_t *)calloc((size_t)c->n_ports, sizeof(int32_t));
  if (port_dc) memcpy(c->port_dc, port_dc, sizeof(int32_t) * c->n_ports);
}

int32_t ox_episode_day(const ox_class *c, uint64_t seed, uint32_t env, uint32_t g0) {
  if (!has_days(c)) return -1;
  uint32_t w[4];
  philox_seeded(seed, env, g0, 0u, OX_DOM_DAY, w);
  return (int32_t)(((uint64_t)w[0] * (uint64_t)c->n_days) >> 32);
}

/* Base buying price at step t_day of an episode on price day `day`. */
static double base_price(const ox_class *c, int32_t t_day, int32_t day) {
  if (has_days(c)) return c->price_days[(size_t)day * c->ip[OXI_STEPS_PER_EPISODE] + t_day];
  return c->price[t_day];
}

/* Dwell time, App. A.1 "User Profiles": the lognormal stay length rounded to
 * the nearest step, lumped into 1 below 1.5 and capped at dwell_max.
 * F(x) = erfc(-(ln x - mu) / (sigma sqrt 2)) / 2 is the lognormal CDF. */
static void build_tdwell(ox_class *c) {
  const int32_t D = c->ip[OXI_DWELL_MAX];
  const double mu = c->p[OXP_DWELL_MU], sigma = c->p[OXP_DWELL_SIGMA];
  c->tdwell[0] = 0;
  for (int32_t k = 1; k < D; ++k) {
    double x = (double)k + 0.5;
    double F = 0.5 * erfc(-(log(x) - mu) / (sigma * sqrt(2.0)));
    c->tdwell[k] = threshold_u32(F);
  }
}

ox_class *ox_class_new(int32_t n_ports, int32_t n_nodes, const int32_t *node_parent,
                       const double *node_limit, const double *node_eta,
                       const int32_t *port_parent, const double *port_pmax,
                       const double *port_eta, const double *params, const int32_t *iparams) {
  if (n_ports < 1 || n_ports > OX_MAX_PORTS || n_nodes < 1 || n_nodes > OX_MAX_NODES) return NULL;
  ox_class *c = (ox_class *)calloc(1, sizeof(ox_class));
  c->n_ports = n_ports;
  c->n_nodes = n_nodes;
  memcpy(c->p, params, sizeof(c->p));
  memcpy(c->ip, iparams, sizeof(c->ip));
  c->node_parent = (int32_t *)malloc(sizeof(int32_t) * n_nodes);
  c->node_depth = (int32_t *)malloc(sizeof(int32_t) * n_nodes);
  c->node_cap = (double *)malloc(sizeof(double) * n_nodes);
  c->anc = (unsigned char *)calloc((size_t)n_nodes * n_ports, 1);
  c->pmax = (double *)malloc(sizeof(double) * n_ports);
  c->peta = (double *)malloc(sizeof(double) * n_ports);
  c->pdis = (double *)malloc(sizeof(double) * n_ports);
  c->max_depth = 0;
  for (int32_t h = 0; h < n_nodes; ++h) {
    c->node_parent[h] = node_parent[h];
    c->node_cap[h] = node_eta[h] * node_limit[h];
    int32_t d = 0;
    for (int32_t a = node_parent[h]; a >= 0; a = node_parent[a]) ++d;
    c->node_depth[h] = d;
    if (d > c->max_depth) c->max_depth = d;
  }
  for (int32_t i = 0; i < n_ports; ++i) {
    c->pmax[i] = port_pmax[i];
    c->pdis[i] = port_pmax[i];
    c->peta[i] = port_eta[i];
    for (int32_t a = port_parent[i]; a >= 0; a = node_parent[a]) c->anc[(size_t)a * n_ports + i] = 1;
  }
  c->tpois = (uint32_t *)malloc(sizeof(uint32_t) * c->ip[OXI_STEPS_PER_EPISODE] * OX_K_POIS);
  c->tdwell = (uint32_t *)malloc(sizeof(uint32_t) * c->ip[OXI_DWELL_MAX]);
  /* default time-of-day profiles: smooth arrival curve, sinusoidal base price */
  const int32_t S = c->ip[OXI_STEPS_PER_EPISODE];
  c->lam = (double *)malloc(sizeof(double) * S);
  c->price = (double *)malloc(sizeof(double) * S);
  for (int32_t t = 0; t < S; ++t) {
    c->lam[t] = 0.5 * c->p[OXP_ARRIVAL_PEAK] * (1.0 - cos(2.0 * M_PI * (double)t / (double)S));
    c->price[t] = c->p[OXP_PRICE_BASE] + c->p[OXP_PRICE_AMP] * sin(2.0 * M_PI * (double)t / (double)S);
  }
  build_tpois(c);
  build_tdwell(c);
  return c;
}

void ox_class_free(ox_class *c) {
  if (!c) return;
  free(c->node_parent); free(c->node_depth); free(c->node_cap); free(c->anc);
  free(c->pmax); free(c->peta); free(c->pdis); free(c->price_days); free(c->port_dc); free(c->tpois); free(c->tdwell); free(c->lam); free(c->price);
  free(c);
}

void ox_class_set_profiles(ox_class *c, const double *arrival_rate, const double *price_table) {
  const int32_t S = c->ip[OXI_STEPS_PER_EPISODE];
  if (arrival_rate) memcpy(c->lam, arrival_rate, sizeof(double) * S);
  if (price_table) memcpy(c->price, price_table, sizeof(double) * S);
  build_tpois(c);
}

void ox_class_set_v2g(ox_class *c, int32_t v2g, const double *pdis, const double *batt) {
  c->v2g = v2g ? 1 : 0;
  for (int32_t i = 0; i < c->n_ports; ++i) c->pdis[i] = pdis ? pdis[i] : c->pmax[i];
  c->b_cap = batt[0]; c->b_rate = batt[1]; c->b_tau = batt[2]; c->b_soc0 = batt[3];
  c->a_db = batt[4]; c->a_dc = batt[5];
}

static int32_t has_battery(const ox_class *c) { return c->b_cap > 0.0; }
static int32_t has_users(const ox_class *c) { return c->cs_share > 0.0; }

int32_t ox_class_ports(const ox_class *c) { return c->n_ports; }
int32_t ox_class_actions(const ox_class *c) { return c->n_ports + has_battery(c); }
int32_t ox_obs_dim(const ox_class *c) {
  return 6 * c->n_ports + 4 + 2 * has_battery(c) + 2 * has_days(c) + (has_users(c) ? c->n_ports : 0);
}

/* Levels of action index i run from -lo(i) to L: ports of a V2G class and the
 * battery also discharge (the battery is the (N+1)-th pole, Sec. 3 "Action
 * Space").  The action byte is the level plus lo(i). */
static int32_t neg_levels(const ox_class *c, int32_t i) {
  return (i == c->n_ports || c->v2g) ? c->ip[OXI_N_LEVELS] : 0;
}

int32_t ox_action_code(const ox_class *c, int32_t i, int32_t k) { return k + neg_levels(c, i); }

void ox_class_tables(const ox_class *c, uint32_t *tpois, uint32_t *tdwell) {
  if (tpois) memcpy(tpois, c->tpois, sizeof(uint32_t) * c->ip[OXI_STEPS_PER_EPISODE] * OX_K_POIS);
  if (tdwell) memcpy(tdwell, c->tdwell, sizeof(uint32_t) * c->ip[OXI_DWELL_MAX]);
}

/* ------------------------------------------------------------------------- */
/* Charging curve r_hat(SoC) of App. A.1 "Car Profiles", with r_bar = port max. */
static double charge_rate(double pmax, double tau, double soc) {
  if (soc <= tau) return pmax;
  return (1.0 - soc) * pmax / (1.0 - tau);
}

/* Discharging curve: the charging curve mirrored about SoC = 0.5 (App. A.1). */
static double discharge_rate(double pmax, double tau, double soc) {
  return charge_rate(pmax, tau, 1.0 - soc);
}

/* Power of one pole for signed level k (App. A.2 "Apply Actions"): charging
 * asks for k/L of the charge maximum, clipped by the car's charging curve (its
 * maximum rate rbar) and by the room left in the battery; discharging asks for
 * |k|/L of the discharge maximum, clipped by the mirrored curve and by the
 * energy stored. */
static double pole_power(int32_t k, int32_t L, double pmax, double pdis, double rbar, double tau, double soc,
                         double cap, double dt) {
  if (k >= 0) {
    double v = (double)k / (double)L * pmax;
    double rhat = charge_rate(rbar, tau, soc);
    double room = (1.0 - soc) * cap / dt;
    if (rhat < v) v = rhat;
    if (room < v) v = room;
    return v;
  }
  double v = (double)(-k) / (double)L * pdis;
  double rhat = discharge_rate(rbar, tau, soc);
  double stored = soc * cap / dt;
  if (rhat < v) v = rhat;
  if (stored < v) v = stored;
  return -v;
}

double ox_battery_power(const ox_class *c, double soc_b, int32_t kb) {
  if (!has_battery(c)) return 0.0;
  return pole_power(kb, c->ip[OXI_N_LEVELS], c->b_rate, c->b_rate, c->b_rate, c->b_tau, soc_b, c->b_cap,
                    c->p[OXP_DT]);
}

/* Eq. (ArchConst): for every subtree H, the magnitude of the sum of its leaves'
 * powers <= eta_H I_H (a discharging subtree drives the same hardware in
 * reverse).  Violations are removed by rescaling the leaves of the violated
 * subtree proportionally, deepest subtrees first, so that a parent sees the
 * already rescaled loads of its children. */
void ox_project(const ox_class *c, double *P) {
  const int32_t N = c->n_ports;
  for (int32_t d = c->max_depth; d >= 0; --d) {
    for (int32_t h = 0; h < c->n_nodes; ++h) {
      if (c->node_depth[h] != d) continue;
      const unsigned char *in = c->anc + (size_t)h * N;
      double S = 0.0;
      for (int32_t i = 0; i < N; ++i)
        if (in[i]) S += P[i];
      if (fabs(S) > c->node_cap[h]) {
        double f = c->node_cap[h] / fabs(S);
        for (int32_t i = 0; i < N; ++i)
          if (in[i]) P[i] = P[i] * f;
      }
    }
  }
}

/* App. A.2 "Apply Actions" with absolute discrete levels (Supp. B.1): every
 * occupied port's signed request is clipped (pole_power), then the tree's
 * limits are enforced. */
static int32_t occupied(const int32_t *dwell, const int32_t *user, int32_t i) {
  return dwell[i] > 0 || (user && user[i] == 1);
}

void ox_apply_actions(const ox_class *c, const int32_t *dwell, const int32_t *user, const double *soc,
                      const double *cap, const double *rbar, const int32_t *k, double *P) {
  const double tau = c->p[OXP_TAU], dt = c->p[OXP_DT];
  const int32_t L = c->ip[OXI_N_LEVELS];
  for (int32_t i = 0; i < c->n_ports; ++i)
    P[i] = occupied(dwell, user, i)
               ? pole_power(k[i], L, c->pmax[i], c->pdis[i], rbar ? rbar[i] : c->pmax[i], tau, soc[i], cap[i], dt)
               : 0.0;
  ox_project(c, P);
}

/* ------------------------------------------------------------------------- */
void ox_draw_exo(const ox_class *c, uint64_t seed, uint32_t env, uint32_t g, int32_t t_day,
                 ox_exo *x) {
  uint32_t w[4];
  philox_seeded(seed, env, g, 0u, OX_DOM_ENV, w);
  /* arrivals: M = number of thresholds the word exceeds */
  const uint32_t *row = c->tpois + (size_t)t_day * OX_K_POIS;
  int32_t M = 0;
  for (int32_t k = 0; k < OX_K_POIS; ++k)
    if (w[0] > row[k]) ++M;
  x->M = M;
  /* price noise: Box-Muller on two 24-bit uniforms */
  double u1 = ((double)(w[1] >> 8) + 1.0) * (1.0 / 16777216.0);
  double u2 = ox_u24(w[2]);
  x->z = sqrt(-2.0 * log(u1)) * cos(2.0 * M_PI * u2);
  /* the episode's price day (exploring starts): drawn at the step it began */
  x->day = ox_episode_day(c, seed, env, g - (uint32_t)t_day);
  x->day_next = t_day + 1 == c->ip[OXI_STEPS_PER_EPISODE] ? ox_episode_day(c, seed, env, g + 1u) : x->day;
  x->p_buy = base_price(c, t_day, x->day) + c->p[OXP_PRICE_SIGMA] * x->z;
  /* car and user profiles of every arriving car j (App. A.2 "Arrival of new Cars") */
  const int32_t D = c->ip[OXI_DWELL_MAX];
  for (int32_t j = 0; j < M; ++j) {
    uint32_t b[4];
    philox_seeded(seed, env, g, (uint32_t)j, OX_DOM_CAR, b);
    x->car_cap[j] = c->p[OXP_CAP_LO] + (c->p[OXP_CAP_HI] - c->p[OXP_CAP_LO]) * ox_u24(b[0]);
    x->car_model[j] = -1;
    if (c->n_models > 0) {  /* the car's model (App. A.1 car distribution) fixes its capacity */
      int32_t m = 0;
      for (int32_t q = 0; q < c->n_models; ++q) m += b[0] > c->model_thresh[q];
      x->car_model[j] = m;
      x->car_cap[j] = c->model_cap[m];
    }
    x->car_soc[j] = c->p[OXP_SOC0_LO] + (c->p[OXP_SOC0_HI] - c->p[OXP_SOC0_LO]) * ox_u24(b[1]);
    x->car_tgt[j] = c->p[OXP_TGT_LO] + (c->p[OXP_TGT_HI] - c->p[OXP_TGT_LO]) * ox_u24(b[2]);
    int32_t d = 1;
    for (int32_t k = 1; k < D; ++k)
      if (b[3] > c->tdwell[k]) ++d;
    x->car_dwell[j] = d;
    /* the user's preference u (App. A.1 "User Profiles"): charge-sensitive with
     * probability cs_share */
    x->car_user[j] = 0;
    if (has_users(c)) {
      uint32_t w[4];
      philox_seeded(seed, env, g, (uint32_t)j, OX_DOM_USER, w);
      x->car_user[j] = w[0] <= c->cs_thresh;
    }
  }
}

/* Levels of every action index.  RANDOM: uniform over the index's n = lo + L + 1
 * levels from one 16-bit half h of counter (env, g >> 3, i, ACT) -- word
 * (g & 7) / 2, its low half on even g -- as the code (h n) / 2^16; MAX: level L;
 * EXTERNAL: the given byte minus lo, bytes above lo + L taken as lo + L. */
void ox_draw_actions(const ox_class *c, int32_t mode, uint64_t seed, uint32_t env, uint32_t g,
                     const uint8_t *ext, int32_t *k) {
  const int32_t L = c->ip[OXI_N_LEVELS];
  const int32_t n_act = ox_class_actions(c);
  for (int32_t i = 0; i < n_act; ++i) {
    const int32_t lo = neg_levels(c, i);
    int32_t code;
    if (mode == OX_ACT_RANDOM) {
      uint32_t w[4];
      philox_seeded(seed, env, g >> 3, (uint32_t)i, OX_DOM_ACT, w);
      const uint32_t h = (g & 1u) ? (w[(g & 7u) >> 1] >> 16) : (w[(g & 7u) >> 1] & 0xFFFFu);
      code = (int32_t)(((uint64_t)h * (uint64_t)(lo + L + 1)) >> 16);
    } else if (mode == OX_ACT_MAX) {
      code = lo + L;
    } else {
      code = ext[i] > lo + L ? lo + L : (int32_t)ext[i];
    }
    k[i] = code - lo;
  }
}

/* ------------------------------------------------------------------------- */
void ox_observe(const ox_class *c, const int32_t *dwell, const int32_t *user, const double *soc,
                const double *e_rem, const double *cap, const double *rbar, const double *p_last,
                const double *batt, int32_t t_day, int32_t day, double *obs) {
  const int32_t N = c->n_ports, S = c->ip[OXI_STEPS_PER_EPISODE];
  const double tau = c->p[OXP_TAU];
  int32_t n_occ = 0;
  for (int32_t i = 0; i < N; ++i) {
    int32_t occ = occupied(dwell, user, i);
    n_occ += occ;
    obs[0 * N + i] = occ ? 1.0 : 0.0;
    obs[1 * N + i] = occ ? soc[i] : 0.0;
    obs[2 * N + i] = occ ? e_rem[i] / cap[i] : 0.0;
    obs[3 * N + i] = (double)dwell[i] / (double)S;
    obs[4 * N + i] = occ ? charge_rate(rbar ? rbar[i] : c->pmax[i], tau, soc[i]) / c->pmax[i] : 0.0;
    obs[5 * N + i] = occ ? p_last[i] / c->pmax[i] : 0.0;
  }
  double ang = 2.0 * M_PI * (double)t_day / (double)S;
  obs[6 * N + 0] = sin(ang);
  obs[6 * N + 1] = cos(ang);
  obs[6 * N + 2] = base_price(c, t_day, day);
  obs[6 * N + 3] = (double)n_occ / (double)N;
  if (has_battery(c)) {
    obs[6 * N + 4] = batt[0];
    obs[6 * N + 5] = batt[1] / c->b_rate;
  }
  if (has_days(c)) {   /* the episode's day and whether it falls on a weekend */
    double *o = obs + 6 * N + 4 + 2 * has_battery(c);
    o[0] = (double)day / (double)c->n_days;
    o[1] = day % 7 >= 5 ? 1.0 : 0.0;
  }
  if (has_users(c)) {  /* the user preference u of every port (0 when empty) */
    double *o = obs + 6 * N + 4 + 2 * has_battery(c) + 2 * has_days(c);
    for (int32_t i = 0; i < N; ++i) o[i] = user[i] == 1 ? 1.0 : 0.0;
  }
}

static void clear_port(int32_t i, int32_t *dwell, int32_t *user, double *soc, double *e_rem, double *cap,
                       double *rbar, double *p_last) {
  dwell[i] = 0; user[i] = 0; soc[i] = 0.0; e_rem[i] = 0.0; cap[i] = 0.0; p_last[i] = 0.0;
  if (rbar) rbar[i] = 0.0;
}

/* App. A.2: (i) apply actions, (ii) charge, (iii) departures, (iv) arrivals;
 * then the reward of App. A.3 and the day boundary of Supp. B.1. */
void ox_transition(const ox_class *c, int32_t *dwell, int32_t *user, double *soc, double *e_rem,
                   double *cap, double *rbar, double *p_last, double *batt, double *ret, int32_t *t_day,
                   const int32_t *k, const ox_exo *x, ox_step_info *info, double *obs, double *P_out) {
  if (c->n_models == 0) rbar = NULL;  /* the base model: every car's rate is the port maximum */
  const int32_t N = c->n_ports;
  const double dt = c->p[OXP_DT];
  double P[OX_MAX_PORTS];
  unsigned char was_occ[OX_MAX_PORTS];

  /* (i) apply actions */
  ox_apply_actions(c, dwell, user, soc, cap, rbar, k, P);
  if (P_out)
    for (int32_t i = 0; i < N; ++i) P_out[i] = P[i];

  /* (ii) charge (or discharge) stationed cars; energies of App. A.3: into the
   * cars (net), drawn from the grid for charging (losses 1/eta), fed back by
   * discharging cars (losses eta, <= 0) */
  double e_net = 0.0, e_from_grid = 0.0, e_to_grid = 0.0;
  for (int32_t i = 0; i < N; ++i) {
    was_occ[i] = occupied(dwell, user, i);
    if (!was_occ[i]) continue;
    double e = dt * P[i];
    double s = soc[i] + e / cap[i];
    soc[i] = s > 1.0 ? 1.0 : (s < 0.0 ? 0.0 : s);
    e_rem[i] = e_rem[i] - e;
    e_net += e;
    if (e > 0.0) e_from_grid += e / c->peta[i];
    if (e < 0.0) e_to_grid += c->peta[i] * e;
    p_last[i] = P[i];
    dwell[i] -= 1;
  }
  /* the station battery: the (N+1)-th pole, at the grid connection */
  double e_batt = 0.0;
  if (has_battery(c)) {
    double pb = ox_battery_power(c, batt[0], k[N]);
    e_batt = dt * pb;
    double s = batt[0] + e_batt / c->b_cap;
    batt[0] = s > 1.0 ? 1.0 : (s < 0.0 ? 0.0 : s);
    batt[1] = pb;
  }
  double e_grid = e_from_grid + e_to_grid + e_batt;

  /* (iii) departures: time-sensitive users when no time remains
   * (c_satisfaction,0: the energy still wanted), charge-sensitive users when no
   * energy remains (c_satisfaction,1: hours past the planned departure, minus
   * beta times the hours left early) */
  double c_sat = 0.0, c_sat1 = 0.0;
  int32_t n_dep = 0;
  for (int32_t i = 0; i < N; ++i) {
    if (!was_occ[i]) continue;
    if (user[i] == 1) {
      if (e_rem[i] <= 0.0) {
        double t_left = (double)dwell[i] * dt;
        c_sat1 += (t_left < 0.0 ? -t_left : 0.0) - c->beta1 * (t_left > 0.0 ? t_left : 0.0);
        ++n_dep;
        clear_port(i, dwell, user, soc, e_rem, cap, rbar, p_last);
      }
    } else if (dwell[i] == 0) {
      c_sat += e_rem[i] > 0.0 ? e_rem[i] : 0.0;
      ++n_dep;
      clear_port(i, dwell, user, soc, e_rem, cap, rbar, p_last);
    }
  }

  /* (iv) arrivals: clip by free spots, first free ports in port order */
  int32_t n_free = 0;
  for (int32_t i = 0; i < N; ++i) n_free += !occupied(dwell, user, i);
  int32_t acc = x->M < n_free ? x->M : n_free;
  int32_t rej = x->M - acc;
  int32_t j = 0;
  for (int32_t i = 0; i < N && j < acc; ++i) {
    if (occupied(dwell, user, i)) continue;
    dwell[i] = x->car_dwell[j];
    user[i] = x->car_user[j];
    if (rbar) rbar[i] = c->port_dc[i] ? c->model_rdc[x->car_model[j]] : c->model_rac[x->car_model[j]];
    soc[i] = x->car_soc[j];
    cap[i] = x->car_cap[j];
    e_rem[i] = (x->car_tgt[j] - x->car_soc[j]) * x->car_cap[j];
    p_last[i] = 0.0;
    ++j;
  }

  /* reward: profit minus penalties (satisfaction, declined cars, degradation
   * of the station battery when it discharges and of discharged cars) */
  double price = e_grid > 0.0 ? x->p_buy : c->p[OXP_P_SELL_GRID];
  double profit = c->p[OXP_P_SELL] * e_net - price * e_grid - c->p[OXP_FIXED_COST];
  double c_db = e_batt < 0.0 ? -e_batt : 0.0;
  double c_dc = -e_to_grid;
  double reward = profit - c->p[OXP_ALPHA_SAT] * c_sat - c->p[OXP_ALPHA_DEC] * (double)rej -
                  c->a_db * c_db - c->a_dc * c_dc - c->a_sat1 * c_sat1;
  *ret += reward;

  /* time and the end of the day: every port empties, the battery starts the
   * next day at its initial SoC */
  *t_day += 1;
  int32_t done = *t_day == c->ip[OXI_STEPS_PER_EPISODE];
  if (done) {
    for (int32_t i = 0; i < N; ++i) clear_port(i, dwell, user, soc, e_rem, cap, rbar, p_last);
    if (has_battery(c)) {
      batt[0] = c->b_soc0;
      batt[1] = 0.0;
    }
    *t_day = 0;
  }
  int32_t n_occ = 0;
  for (int32_t i = 0; i < N; ++i) n_occ += occupied(dwell, user, i);

  if (info) {
    info->reward = reward; info->profit = profit; info->e_net = e_net; info->e_grid = e_grid;
    info->c_sat = c_sat; info->M = x->M; info->acc = acc; info->rej = rej; info->n_dep = n_dep;
    info->done = done; info->n_occ = n_occ; info->e_to_grid = e_to_grid; info->e_batt = e_batt;
    info->c_sat1 = c_sat1;
  }
  if (obs) ox_observe(c, dwell, user, soc, e_rem, cap, rbar, p_last, batt, *t_day, x->day_next, obs);
}

/* ------------------------------------------------------------------------- */
typedef struct {
  ox_class *const *classes;
  const int32_t *env_class;
  const int64_t *env_ids;
  const int64_t *port_off, *act_off, *obs_off;
  int64_t total_act, total_obs, n_envs;
  int64_t e_begin, e_end;
  uint64_t seed;
  uint32_t g0;
  int32_t t0, T, mode;
  const uint8_t *act_in;
  int32_t *dwell, *user;
  double *soc, *e_rem, *cap, *rbar, *p_last, *batt, *ret, *obs, *reward;
  uint8_t *act, *done;
  ox_step_info *info;
} rollout_job;

static void *rollout_worker(void *arg) {
  rollout_job *J = (rollout_job *)arg;
  int32_t k[OX_MAX_PORTS + 1];
  ox_exo x;
  for (int64_t e = J->e_begin; e < J->e_end; ++e) {
    const ox_class *c = J->classes[J->env_class[e]];
    const int64_t po = J->port_off[e], ao = J->act_off[e], oo = J->obs_off[e];
    const int32_t n_act = ox_class_actions(c);
    double *bt = J->batt ? J->batt + 2 * e : NULL;
    int32_t t_day = J->t0;
    const uint32_t eid = (uint32_t)(J->env_ids ? J->env_ids[e] : e);
    for (int32_t t = 0; t < J->T; ++t) {
      uint32_t g = J->g0 + (uint32_t)t;
      const uint8_t *ext = J->act_in ? J->act_in + (size_t)t * J->total_act + ao : NULL;
      ox_draw_actions(c, J->mode, J->seed, eid, g, ext, k);
      ox_draw_exo(c, J->seed, eid, g, t_day, &x);
      ox_step_info inf;
      double *o = J->obs ? J->obs + (size_t)t * J->total_obs + oo : NULL;
      ox_transition(c, J->dwell + po, J->user + po, J->soc + po, J->e_rem + po, J->cap + po,
                    J->rbar ? J->rbar + po : NULL, J->p_last + po, bt, J->ret + e, &t_day, k, &x, &inf, o, NULL);
      if (J->act)
        for (int32_t i = 0; i < n_act; ++i)
          J->act[(size_t)t * J->total_act + ao + i] = (uint8_t)ox_action_code(c, i, k[i]);
      if (J->reward) J->reward[(size_t)t * J->n_envs + e] = inf.reward;
      if (J->done) J->done[(size_t)t * J->n_envs + e] = (uint8_t)inf.done;
      if (J->info) J->info[(size_t)t * J->n_envs + e] = inf;
    }
  }
  return NULL;
}

/* First env of worker w of n: contiguous env ranges holding about equal numbers
 * of ports (a step's work grows with the ports), so that classes of different
 * sizes do not leave some workers idle. */
static int64_t balanced_split(const int64_t *port_off, int64_t n_envs, int32_t w, int32_t n) {
  if (w >= n) return n_envs;
  const int64_t target = port_off[n_envs] * w / n;
  int64_t lo = 0, hi = n_envs;  /* the first e with port_off[e] >= target */
  while (lo < hi) {
    const int64_t mid = (lo + hi) / 2;
    if (port_off[mid] < target) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

int32_t ox_rollout(ox_class *const *classes, const int32_t *env_class, const int64_t *env_ids,
                   int64_t n_envs, uint64_t seed, uint32_t *g, int32_t *t_day, int32_t T, int32_t mode,
                   const uint8_t *act_in, int32_t *dwell, int32_t *user, double *soc, double *e_rem,
                   double *cap, double *rbar, double *p_last, double *batt, double *ret, double *obs, uint8_t *act,
                   double *reward, uint8_t *done, ox_step_info *info, int32_t n_threads) {
  int64_t *port_off = (int64_t *)malloc(sizeof(int64_t) * (n_envs + 1));
  int64_t *act_off = (int64_t *)malloc(sizeof(int64_t) * (n_envs + 1));
  int64_t *obs_off = (int64_t *)malloc(sizeof(int64_t) * (n_envs + 1));
  port_off[0] = act_off[0] = obs_off[0] = 0;
  for (int64_t e = 0; e < n_envs; ++e) {
    const ox_class *c = classes[env_class[e]];
    port_off[e + 1] = port_off[e] + c->n_ports;
    act_off[e + 1] = act_off[e] + ox_class_actions(c);
    obs_off[e + 1] = obs_off[e] + ox_obs_dim(c);
  }
  if (n_threads < 1) n_threads = 1;
  if (n_threads > n_envs) n_threads = n_envs > 0 ? (int32_t)n_envs : 1;
  rollout_job *jobs = (rollout_job *)calloc((size_t)n_threads, sizeof(rollout_job));
  pthread_t *th = (pthread_t *)calloc((size_t)n_threads, sizeof(pthread_t));
  for (int32_t w = 0; w < n_threads; ++w) {
    rollout_job *J = &jobs[w];
    J->classes = classes; J->env_class = env_class; J->env_ids = env_ids; J->port_off = port_off;
    J->act_off = act_off; J->obs_off = obs_off;
    J->total_act = act_off[n_envs]; J->total_obs = obs_off[n_envs]; J->n_envs = n_envs;
    J->e_begin = balanced_split(port_off, n_envs, w, n_threads);
    J->e_end = balanced_split(port_off, n_envs, w + 1, n_threads);
    J->seed = seed; J->g0 = *g; J->t0 = *t_day; J->T = T; J->mode = mode; J->act_in = act_in;
    J->dwell = dwell; J->user = user; J->soc = soc; J->e_rem = e_rem; J->cap = cap; J->rbar = rbar;
    J->p_last = p_last;
    J->batt = batt;
    J->ret = ret; J->obs = obs; J->act = act; J->reward = reward; J->done = done; J->info = info;
  }
  if (n_threads == 1) {
    rollout_worker(&jobs[0]);
  } else {
    for (int32_t w = 0; w < n_threads; ++w) pthread_create(&th[w], NULL, rollout_worker, &jobs[w]);
    for (int32_t w = 0; w < n_threads; ++w) pthread_join(th[w], NULL);
  }
  *g += (uint32_t)T;
  *t_day = (int32_t)(((int64_t)*t_day + T) % classes[env_class[0]]->ip[OXI_STEPS_PER_EPISODE]);
  free(jobs); free(th); free(port_off); free(act_off); free(obs_off);
  return n_threads;
}

/* ------------------------------------------------------------------------- */
/* BF16 = the upper 16 bits of an IEEE single; round-to-nearest-even from FP64. */
double ox_bf16_round(double x) {
  if (x == 0.0 || !isfinite(x)) return (double)(float)x;
  int e;
  frexp(x, &e);                       /* x = m 2^e, 0.5 <= |m| < 1 */
  double ulp = ldexp(1.0, e - 8);     /* 8 significant bits */
  double q = x / ulp;
  double r = nearbyint(q);            /* default rounding mode: nearest-even */
  return r * ulp;
}

static double bf16_bits_to_double(uint16_t b) {
  uint32_t u = (uint32_t)b << 16;
  float f;
  memcpy(&f, &u, sizeof f);
  return (double)f;
}

/* Policy of the policy-in-the-loop workload: a two-layer perceptron over the
 * observation, tanh hidden units, one logit per (port, level), and a level per
 * port drawn from the categorical distribution softmax(logits) by inverting its
 * distribution function with one Philox uniform. */
void ox_policy(const ox_class *c, int32_t hidden, const uint16_t *w1, const uint16_t *b1,
               const uint16_t *w2, const uint16_t *b2, const double *obs, uint64_t seed,
               uint32_t env, uint32_t g, double *logits, int32_t *k, double *margin) {
  const int32_t N = c->n_ports, L = c->ip[OXI_N_LEVELS];
  const int32_t in = 6 * N + 4, out = N * (L + 1);
  double *x = (double *)malloc(sizeof(double) * in);
  double *h = (double *)malloc(sizeof(double) * hidden);
  double *z = (double *)malloc(sizeof(double) * out);
  for (int32_t i = 0; i < in; ++i) x[i] = ox_bf16_round(obs[i]);
  for (int32_t j = 0; j < hidden; ++j) {
    double a = bf16_bits_to_double(b1[j]);
    for (int32_t i = 0; i < in; ++i) a += x[i] * bf16_bits_to_double(w1[(size_t)i * hidden + j]);
    h[j] = ox_bf16_round(tanh(a));
  }
  for (int32_t o = 0; o < out; ++o) {
    double a = bf16_bits_to_double(b2[o]);
    for (int32_t j = 0; j < hidden; ++j) a += h[j] * bf16_bits_to_double(w2[(size_t)j * out + o]);
    z[o] = a;
  }
  for (int32_t i = 0; i < N; ++i) {
    const double *zi = z + (size_t)i * (L + 1);
    /* softmax probabilities p_l = exp(z_l - max z) / W */
    double zmax = zi[0];
    for (int32_t l = 1; l <= L; ++l) zmax = zi[l] > zmax ? zi[l] : zmax;
    double e[256], W = 0.0;
    for (int32_t l = 0; l <= L; ++l) {
      e[l] = exp(zi[l] - zmax);
      W += e[l];
    }
    /* u in (0, 1) from the top 24 bits of word (i / 16) mod 4 of Philox
     * (env, g, i mod 16 + 16 (i / 64), 3) -- ports 16 apart share a call; the
     * level is the first l whose distribution function F_l = (p_0 + .. + p_l)
     * exceeds u */
    uint32_t w[4];
    philox_seeded(seed, env, g, (uint32_t)(i % 16 + 16 * (i / 64)), OX_DOM_GUM, w);
    const double u = ((double)(w[(i / 16) % 4] >> 8) + 0.5) * (1.0 / 16777216.0);
    double F = 0.0, near = 1.0;
    int32_t lev = L;
    for (int32_t l = 0; l < L; ++l) {
      F += e[l] / W;
      const double d = fabs(F - u);
      near = d < near ? d : near;
      if (lev == L && F > u) lev = l;
    }
    k[i] = lev;
    if (margin) margin[i] = near;  /* distance of u from the nearest F_l */
  }
  if (logits)
    for (int32_t o = 0; o < out; ++o) logits[o] = z[o];
  free(x); free(h); free(z);
}
