// cx_spec.cpp -- host side: validation of a station spec, compilation of its
// capacity tree into the aligned power-of-two slot layout used by the kernels,
// and the FP64 sampling tables.  Built with -ffp-contract=off: the integer
// tables must be reproducible bit for bit from their FP64 definitions.
#include "cx_spec.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <functional>
#include <limits>

namespace cx {

static bool fail(std::string *err, const std::string &m) {
  if (err) *err = m;
  return false;
}

static int next_pow2(int x) {
  int p = 1;
  while (p < x) p <<= 1;
  return p;
}

static int ilog2(int x) {
  int r = 0;
  while ((1 << r) < x) ++r;
  return r;
}

bool copy_spec(const cx_station_spec &in, SpecCopy *out, std::string *err) {
  if (in.n_ports < 1 || in.n_ports > kMaxSlots) return fail(err, "n_ports must be in 1..256");
  if (in.n_nodes < 1 || in.n_nodes > 256) return fail(err, "n_nodes must be in 1..256");
  if (!in.node_parent || !in.node_limit_kw || !in.node_eta || !in.port_parent || !in.port_pmax_kw ||
      !in.port_eta)
    return fail(err, "station spec arrays must not be NULL");
  out->s = in;
  out->node_parent.assign(in.node_parent, in.node_parent + in.n_nodes);
  out->node_limit.assign(in.node_limit_kw, in.node_limit_kw + in.n_nodes);
  out->node_eta.assign(in.node_eta, in.node_eta + in.n_nodes);
  out->port_parent.assign(in.port_parent, in.port_parent + in.n_ports);
  out->port_pmax.assign(in.port_pmax_kw, in.port_pmax_kw + in.n_ports);
  out->port_eta.assign(in.port_eta, in.port_eta + in.n_ports);
  out->s.node_parent = out->node_parent.data();
  out->s.node_limit_kw = out->node_limit.data();
  out->s.node_eta = out->node_eta.data();
  out->s.port_parent = out->port_parent.data();
  out->s.port_pmax_kw = out->port_pmax.data();
  out->s.port_eta = out->port_eta.data();
  const int S = in.steps_per_episode;
  if ((in.arrival_rate || in.price_table) && (S < 1 || S > 100000))
    return fail(err, "steps_per_episode must be in 1..100000");
  out->arrival_rate.clear();
  out->price_table.clear();
  if (in.arrival_rate) out->arrival_rate.assign(in.arrival_rate, in.arrival_rate + S);
  if (in.price_table) out->price_table.assign(in.price_table, in.price_table + S);
  out->s.arrival_rate = in.arrival_rate ? out->arrival_rate.data() : nullptr;
  out->s.price_table = in.price_table ? out->price_table.data() : nullptr;
  if (in.port_pdis_kw) out->port_pdis.assign(in.port_pdis_kw, in.port_pdis_kw + in.n_ports);
  else out->port_pdis = out->port_pmax;
  out->s.port_pdis_kw = out->port_pdis.data();
  out->price_days.clear();
  if (in.n_price_days < 0 || in.n_price_days > 100000) return fail(err, "n_price_days must be in 0..100000");
  if (in.n_price_days > 0) {
    if (!in.price_days) return fail(err, "price_days must not be NULL when n_price_days > 0");
    if (S < 1 || S > 100000) return fail(err, "steps_per_episode must be in 1..100000");
    if ((int64_t)in.n_price_days * S > (int64_t)1 << 24) return fail(err, "price_days holds more than 2^24 prices");
    out->price_days.assign(in.price_days, in.price_days + (size_t)in.n_price_days * S);
  }
  out->s.price_days = out->price_days.empty() ? nullptr : out->price_days.data();
  if (out->price_days.empty()) out->s.n_price_days = 0;
  if (in.n_car_models < 0 || in.n_car_models > 8) return fail(err, "n_car_models must be in 0..8");
  if (in.n_car_models > 0 && !in.car_models) return fail(err, "car_models must not be NULL when n_car_models > 0");
  out->car_models.assign(in.car_models, in.car_models + 4 * (size_t)in.n_car_models);
  out->s.car_models = out->car_models.empty() ? nullptr : out->car_models.data();
  out->port_dc.assign(in.n_ports, 0);
  if (in.port_dc) out->port_dc.assign(in.port_dc, in.port_dc + in.n_ports);
  out->s.port_dc = out->port_dc.data();
  return true;
}

static bool finite_pos(double x) { return std::isfinite(x) && x > 0.0; }

static uint32_t cdf_threshold(double F);

bool compile_spec(const SpecCopy &sc, Compiled *c, std::string *err) {
  const cx_station_spec &s = sc.s;
  const int N = s.n_ports, H = s.n_nodes;
  // ---- scalar parameters
  if (!finite_pos(s.dt_hours)) return fail(err, "dt_hours must be > 0");
  if (!(s.tau > 0.0 && s.tau < 1.0)) return fail(err, "tau must be in (0,1)");
  if (s.steps_per_episode < 1 || s.steps_per_episode > 100000)
    return fail(err, "steps_per_episode must be in 1..100000");
  if (s.n_levels < 1 || s.n_levels > 254) return fail(err, "n_levels must be in 1..254");
  if (!(s.arrival_peak >= 0.0 && s.arrival_peak <= 8.0)) return fail(err, "arrival_peak must be in [0, 8]");
  if (!(s.cap_lo > 0.0 && s.cap_hi >= s.cap_lo)) return fail(err, "need 0 < cap_lo <= cap_hi");
  if (!(s.soc0_lo >= 0.0 && s.soc0_hi >= s.soc0_lo && s.soc0_hi <= 1.0))
    return fail(err, "need 0 <= soc0_lo <= soc0_hi <= 1");
  if (!(s.tgt_lo >= 0.0 && s.tgt_hi >= s.tgt_lo && s.tgt_hi <= 1.0))
    return fail(err, "need 0 <= tgt_lo <= tgt_hi <= 1");
  if (!(s.dwell_sigma > 0.0) || !std::isfinite(s.dwell_mu)) return fail(err, "bad dwell distribution");
  if (s.dwell_max < 1 || s.dwell_max > 4096) return fail(err, "dwell_max must be in 1..4096");
  for (double v : {s.p_sell, s.p_sell_grid, s.fixed_cost, s.alpha_sat, s.alpha_declined, s.price_base,
                   s.price_amp, s.price_sigma})
    if (!std::isfinite(v)) return fail(err, "prices and penalty weights must be finite");
  for (double v : sc.arrival_rate)
    if (!(v >= 0.0 && v <= 8.0)) return fail(err, "arrival_rate entries must be in [0, 8]");
  for (double v : sc.price_table)
    if (!std::isfinite(v)) return fail(err, "price_table entries must be finite");
  for (double v : sc.price_days)
    if (!std::isfinite(v)) return fail(err, "price_days entries must be finite");
  {
    double psum = 0.0;
    for (int m = 0; m < s.n_car_models; ++m) {
      const double *r = &sc.car_models[4 * (size_t)m];
      if (!(r[0] >= 0.0 && r[0] <= 1.0)) return fail(err, "car model probabilities must be in [0,1]");
      if (!finite_pos(r[1]) || !finite_pos(r[2]) || !finite_pos(r[3]))
        return fail(err, "car model capacity and rates must be > 0");
      psum += r[0];
    }
    if (s.n_car_models > 0 && std::fabs(psum - 1.0) > 1e-6) return fail(err, "car model probabilities must sum to 1");
    for (int32_t v : sc.port_dc)
      if (v != 0 && v != 1) return fail(err, "port_dc entries must be 0 or 1");
  }
  if (s.v2g != 0 && s.v2g != 1) return fail(err, "v2g must be 0 or 1");
  if ((s.v2g || s.battery_kwh > 0.0) && s.n_levels > 127)
    return fail(err, "n_levels must be at most 127 with discharging (signed levels fit an action byte)");
  for (double v : sc.port_pdis)
    if (!finite_pos(v)) return fail(err, "port_pdis_kw must be > 0");
  if (!(s.battery_kwh >= 0.0) || !std::isfinite(s.battery_kwh)) return fail(err, "battery_kwh must be >= 0");
  if (s.battery_kwh > 0.0) {
    if (!finite_pos(s.battery_kw)) return fail(err, "battery_kw must be > 0");
    if (!(s.battery_tau > 0.0 && s.battery_tau < 1.0)) return fail(err, "battery_tau must be in (0,1)");
    if (!(s.battery_soc0 >= 0.0 && s.battery_soc0 <= 1.0)) return fail(err, "battery_soc0 must be in [0,1]");
  }
  if (!std::isfinite(s.alpha_degrad_battery) || !std::isfinite(s.alpha_degrad_cars))
    return fail(err, "degradation weights must be finite");
  if (!(s.charge_sensitive_share >= 0.0 && s.charge_sensitive_share <= 1.0))
    return fail(err, "charge_sensitive_share must be in [0,1]");
  if (!std::isfinite(s.alpha_sat1) || !std::isfinite(s.beta_sat1)) return fail(err, "alpha_sat1, beta_sat1 must be finite");
  if (s.charge_sensitive_share > 0.0 && s.steps_per_episode > 30000)
    return fail(err, "steps_per_episode must be <= 30000 with charge-sensitive users");
  // ---- tree
  if (sc.node_parent[0] != -1) return fail(err, "node 0 must be the root (parent -1)");
  for (int h = 1; h < H; ++h)
    if (sc.node_parent[h] < 0 || sc.node_parent[h] >= h)
      return fail(err, "node_parent[i] must be in [0, i) for i > 0");
  for (int h = 0; h < H; ++h) {
    if (!finite_pos(sc.node_limit[h])) return fail(err, "node limits must be > 0");
    if (!(sc.node_eta[h] > 0.0 && sc.node_eta[h] <= 1.0)) return fail(err, "node_eta must be in (0,1]");
  }
  for (int i = 0; i < N; ++i) {
    if (sc.port_parent[i] < 0 || sc.port_parent[i] >= H) return fail(err, "port_parent out of range");
    if (!finite_pos(sc.port_pmax[i])) return fail(err, "port_pmax_kw must be > 0");
    if (!(sc.port_eta[i] > 0.0 && sc.port_eta[i] <= 1.0)) return fail(err, "port_eta must be in (0,1]");
  }
  std::vector<int> depth(H, 0);
  for (int h = 1; h < H; ++h) depth[h] = depth[sc.node_parent[h]] + 1;
  int max_depth = 0;
  for (int h = 0; h < H; ++h) max_depth = std::max(max_depth, depth[h]);
  const int D = max_depth + 1;
  if (D > kMaxLevels) return fail(err, "capacity tree deeper than 4 levels");
  // port range of every node; must be contiguous (depth-first port order)
  std::vector<int> lo(H, N), hi(H, -1), cnt(H, 0);
  for (int i = 0; i < N; ++i)
    for (int a = sc.port_parent[i]; a >= 0; a = sc.node_parent[a]) {
      lo[a] = std::min(lo[a], i);
      hi[a] = std::max(hi[a], i);
      cnt[a] += 1;
    }
  for (int h = 0; h < H; ++h) {
    if (cnt[h] == 0) return fail(err, "every node must have at least one port below it");
    if (hi[h] - lo[h] + 1 != cnt[h]) return fail(err, "ports must be in depth-first order (node ranges contiguous)");
  }
  // children of each node ordered by their first port
  struct Child { int first; bool is_port; int id; };
  std::vector<std::vector<Child>> kids(H);
  for (int h = 1; h < H; ++h) kids[sc.node_parent[h]].push_back({lo[h], false, h});
  for (int i = 0; i < N; ++i) kids[sc.port_parent[i]].push_back({i, true, i});
  for (auto &k : kids) std::sort(k.begin(), k.end(), [](const Child &a, const Child &b) { return a.first < b.first; });
  // aligned block sizes, bottom-up (children have larger ids than parents)
  std::vector<int> size(H, 1);
  for (int h = H - 1; h >= 0; --h) {
    int cur = 0;
    for (const Child &k : kids[h]) {
      const int cs = k.is_port ? 1 : size[k.id];
      cur = (cur + cs - 1) / cs * cs + cs;
    }
    size[h] = next_pow2(std::max(cur, 1));
  }
  // dense layout when the aligned one pads and every level below the root has
  // at most 4 nodes
  const int S_aligned = std::max(4, size[0]);
  const int S_dense = std::max(4, next_pow2(N));
  std::vector<int> level_nodes(kMaxLevels, 0);
  for (int h = 1; h < H; ++h) level_nodes[(D - 1) - depth[h]] += 1;
  bool few = true;
  for (int d = 0; d + 1 < D; ++d) few = few && level_nodes[d] <= 4;
  const bool dense = few && S_dense < S_aligned;
  const int S = dense ? S_dense : S_aligned;
  if (S > kMaxSlots) return fail(err, "aligned slot layout exceeds 256 slots");
  c->N = N; c->S = S; c->D = D;
  c->slot_port.assign(S, -1);
  c->slot_lb.assign(S, 0u);
  c->slot_cap.assign((size_t)D * S, std::numeric_limits<float>::infinity());
  c->port_slot.assign(N, -1);
  c->dense_nodes = 0;
  if (dense) {
    for (int i = 0; i < N; ++i) {
      c->slot_port[i] = i;
      c->port_slot[i] = i;
    }
    std::vector<int> rank(kMaxLevels, 0);
    for (int h = 0; h < H; ++h) {
      const int d = (D - 1) - depth[h];
      const float capv = (float)(sc.node_eta[h] * sc.node_limit[h]);
      if (h == 0) {  // the root covers the whole station
        for (int x = 0; x < S; ++x) {
          c->slot_lb[x] |= (uint32_t)ilog2(S) << (8 * d);
          c->slot_cap[(size_t)d * S + x] = capv;
        }
        continue;
      }
      const uint32_t code = 0x80u | (uint32_t)rank[d]++;
      for (int x = lo[h]; x <= hi[h]; ++x) {
        c->slot_lb[x] |= code << (8 * d);
        c->slot_cap[(size_t)d * S + x] = capv;
      }
    }
    for (int d = 0; d + 1 < D; ++d) c->dense_nodes |= (uint32_t)level_nodes[d] << (8 * d);
  } else {
    std::function<void(int, int)> place = [&](int h, int base) {
      const int d = (D - 1) - depth[h];            // level 0 = deepest
      const int blk = h == 0 ? S : size[h];
      const float capv = (float)(sc.node_eta[h] * sc.node_limit[h]);
      for (int x = base; x < base + blk; ++x) {
        c->slot_lb[x] = (c->slot_lb[x] & ~(0xFFu << (8 * d))) | ((uint32_t)ilog2(blk) << (8 * d));
        c->slot_cap[(size_t)d * S + x] = capv;
      }
      int cur = 0;
      for (const Child &k : kids[h]) {
        const int cs = k.is_port ? 1 : size[k.id];
        cur = (cur + cs - 1) / cs * cs;
        if (k.is_port) {
          c->slot_port[base + cur] = k.id;
          c->port_slot[k.id] = base + cur;
        } else {
          place(k.id, base + cur);
        }
        cur += cs;
      }
    };
    place(0, 0);
  }
  c->slot_pmax.assign(S, 0.f);
  c->slot_inv_pmax.assign(S, 0.f);
  c->slot_inv_eta.assign(S, 1.f);
  c->slot_pdis.assign(S, 0.f);
  c->slot_eta.assign(S, 1.f);
  bool uni = true;
  for (int i = 0; i < N; ++i) {
    const int x = c->port_slot[i];
    c->slot_pmax[x] = (float)sc.port_pmax[i];
    c->slot_inv_pmax[x] = (float)(1.0 / sc.port_pmax[i]);
    c->slot_inv_eta[x] = (float)(1.0 / sc.port_eta[i]);
    c->slot_pdis[x] = (float)sc.port_pdis[i];
    c->slot_eta[x] = (float)sc.port_eta[i];
    if (sc.port_eta[i] != sc.port_eta[0]) uni = false;
  }
  c->uniform_eta = uni;
  c->inv_eta_uniform = (float)(1.0 / sc.port_eta[0]);
  c->v2g = s.v2g == 1;
  c->battery = s.battery_kwh > 0.0;
  c->users = s.charge_sensitive_share > 0.0;
  c->cs_thresh = c->users ? cdf_threshold(s.charge_sensitive_share) : 0u;
  c->n_act = N + (c->battery ? 1 : 0);
  c->n_days = s.n_price_days;
  c->n_models = s.n_car_models;
  c->model_thresh.assign(8, 0xFFFFFFFFu);
  c->model_data.assign(24, 0.f);
  {
    double F = 0.0;
    for (int m = 0; m < c->n_models; ++m) {
      const double *r = &sc.car_models[4 * (size_t)m];
      F += r[0];
      // model = #{m : w > thresh[m]}; the last model takes the remaining mass
      c->model_thresh[m] = m + 1 == c->n_models ? 0xFFFFFFFFu : cdf_threshold(F);
      c->model_data[3 * m + 0] = (float)r[1];
      c->model_data[3 * m + 1] = (float)r[2];
      c->model_data[3 * m + 2] = (float)r[3];
    }
  }
  c->slot_dc.assign(S, 0);
  for (int i = 0; i < N; ++i) c->slot_dc[c->port_slot[i]] = sc.port_dc[i];
  c->day_obs = 6 * N + 4 + (c->battery ? 2 : 0);
  c->user_obs = c->day_obs + (c->n_days > 0 ? 2 : 0);
  c->obs_dim = c->user_obs + (c->users ? N : 0);
  return true;
}

// T = clamp(ceil(2^32 F) - 1, 0, 2^32 - 1): a uniform 32-bit word w satisfies
// w <= T with probability (T + 1) / 2^32 ~= F.
static uint32_t cdf_threshold(double F) {
  double x = std::ceil(F * 4294967296.0) - 1.0;
  x = std::min(std::max(x, 0.0), 4294967295.0);
  return (uint32_t)x;
}

void build_tables(const SpecCopy &sc, Tables *t) {
  const cx_station_spec &s = sc.s;
  const int Sep = s.steps_per_episode;
  const double two_pi = 2.0 * 3.14159265358979323846;
  // arrivals ~ Poisson(lambda(t)): the given per-step means, else
  // lambda(t) = peak (1 - cos(2 pi t / S)) / 2; CDF by the pmf recurrence
  t->tpois.assign((size_t)Sep * kPoisK, 0u);
  t->tpois_dev.assign((size_t)Sep * kPoisStride, 0xFFFFFFFFu);
  for (int step = 0; step < Sep; ++step) {
    const double lam = sc.arrival_rate.empty()
                           ? 0.5 * s.arrival_peak * (1.0 - std::cos(two_pi * (double)step / (double)Sep))
                           : sc.arrival_rate[step];
    double p = std::exp(-lam), F = p;
    for (int k = 0; k < kPoisK; ++k) {
      if (k > 0) {
        p = p * lam / (double)k;
        F = F + p;
      }
      const uint32_t th = cdf_threshold(F);
      t->tpois[(size_t)step * kPoisK + k] = th;
      t->tpois_dev[(size_t)step * kPoisStride + k] = th;
    }
  }
  // dwell: stay d = nearest integer of a lognormal draw, >= 1, <= dwell_max
  const int Dm = s.dwell_max;
  t->tdwell.assign(Dm, 0u);
  for (int k = 1; k < Dm; ++k) {
    const double x = (double)k + 0.5;
    const double F = 0.5 * std::erfc(-(std::log(x) - s.dwell_mu) / (s.dwell_sigma * std::sqrt(2.0)));
    t->tdwell[k] = cdf_threshold(F);
  }
  int log2n = 1;
  while ((1 << log2n) < Dm) ++log2n;          // Dm - 1 real entries plus one sentinel
  t->dwell_log2 = log2n;
  t->tdwell_dev.assign((size_t)1 << log2n, 0xFFFFFFFFu);
  for (int k = 1; k < Dm; ++k) t->tdwell_dev[k - 1] = t->tdwell[k];
  // per-step constants of the observation and the price
  t->glob.assign((size_t)Sep * 4, 0.f);
  for (int step = 0; step < Sep; ++step) {
    const double a = two_pi * (double)step / (double)Sep;
    t->glob[(size_t)step * 4 + 0] = (float)std::sin(a);
    t->glob[(size_t)step * 4 + 1] = (float)std::cos(a);
    t->glob[(size_t)step * 4 + 2] =
        (float)(sc.price_table.empty() ? s.price_base + s.price_amp * std::sin(a) : sc.price_table[step]);
  }
  t->price_days.assign(sc.price_days.begin(), sc.price_days.end());  // to FP32
}

bool tables_monotone(const Tables &t) {
  for (size_t i = 0; i + 1 < t.tdwell_dev.size(); ++i)
    if (t.tdwell_dev[i] > t.tdwell_dev[i + 1]) return false;
  for (size_t r = 0; r * kPoisStride < t.tpois_dev.size(); ++r)
    for (int k = 0; k + 1 < kPoisStride; ++k)
      if (t.tpois_dev[r * kPoisStride + k] > t.tpois_dev[r * kPoisStride + k + 1]) return false;
  return true;
}

}  // namespace cx
