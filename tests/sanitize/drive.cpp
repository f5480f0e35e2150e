// drive.cpp -- drives the library's host code through the C ABI on the fake
// HIP device (fake_hip.cpp) under a sanitizer (test infrastructure).
//
// Usage: drive SCENARIO_FILE CACHE_PATH
// The scenario file holds station specs written by the Python test: a mixture
// of classes with env counts, a policy station and a list of served classes.
// The driver runs, on each: rollouts in every action and output mode, one-step
// launches, resets, observations, packings, block sizes and the observation
// stage, the autotuner (searching, then from its cache), snapshots, the policy
// loop, and the serving path with client threads submitting, polling, waiting,
// cancelling and releasing concurrently (on the fake device and simulated).
#include <hip/hip_runtime.h>

#include <atomic>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <memory>
#include <random>
#include <sstream>
#include <string>
#include <thread>
#include <vector>

#include "cx.h"

extern "C" long fake_hip_graph_destroys_in_flight();
extern "C" long fake_hip_live_allocations();

namespace {

[[noreturn]] void fail(const char *what, cx_status st) {
  std::fprintf(stderr, "DRIVE FAILED: %s: status %d: %s\n", what, (int)st, cx_last_error());
  std::fflush(stderr);
  std::exit(3);
}
#define CK(x)                            \
  do {                                   \
    cx_status st_ = (x);                 \
    if (st_ != CX_OK) fail(#x, st_);     \
  } while (0)

// A spec with the arrays it points to.
struct OwnedSpec {
  cx_station_spec s{};
  std::map<std::string, std::vector<double>> f;   // every field as read
  std::vector<int32_t> node_parent, port_parent, port_dc;
  std::vector<double> node_limit, node_eta, port_pmax, port_eta, arrival_rate, price_table, pdis, days, models;
};

void finish(OwnedSpec &o) {
  auto vec = [&](const char *k) { return o.f.count(k) ? o.f[k] : std::vector<double>{}; };
  auto num = [&](const char *k, double d) { return o.f.count(k) && !o.f[k].empty() ? o.f[k][0] : d; };
  auto ivec = [&](const char *k) {
    std::vector<int32_t> v;
    for (double x : vec(k)) v.push_back((int32_t)x);
    return v;
  };
  o.node_parent = ivec("node_parent");
  o.port_parent = ivec("port_parent");
  o.port_dc = ivec("port_dc");
  o.node_limit = vec("node_limit_kw");
  o.node_eta = vec("node_eta");
  o.port_pmax = vec("port_pmax_kw");
  o.port_eta = vec("port_eta");
  o.arrival_rate = vec("arrival_rate");
  o.price_table = vec("price_table");
  o.pdis = vec("port_pdis_kw");
  o.days = vec("price_days");
  o.models = vec("car_models");
  cx_station_spec &s = o.s;
  s.n_ports = (int32_t)num("n_ports", 0);
  s.n_nodes = (int32_t)o.node_parent.size();
  s.node_parent = o.node_parent.data();
  s.node_limit_kw = o.node_limit.data();
  s.node_eta = o.node_eta.data();
  s.port_parent = o.port_parent.data();
  s.port_pmax_kw = o.port_pmax.data();
  s.port_eta = o.port_eta.data();
  s.dt_hours = num("dt_hours", 1.0 / 12);
  s.tau = num("tau", 0.8);
  s.p_sell = num("p_sell", 0.45);
  s.p_sell_grid = num("p_sell_grid", 0.25);
  s.fixed_cost = num("fixed_cost", 0);
  s.alpha_sat = num("alpha_sat", 0);
  s.alpha_declined = num("alpha_declined", 0);
  s.steps_per_episode = (int32_t)num("steps_per_episode", 288);
  s.n_levels = (int32_t)num("n_levels", 10);
  s.price_base = num("price_base", 0.25);
  s.price_amp = num("price_amp", 0.1);
  s.price_sigma = num("price_sigma", 0.02);
  s.arrival_peak = num("arrival_peak", 0.3);
  s.cap_lo = num("cap_lo", 40);
  s.cap_hi = num("cap_hi", 100);
  s.soc0_lo = num("soc0_lo", 0.1);
  s.soc0_hi = num("soc0_hi", 0.5);
  s.tgt_lo = num("tgt_lo", 0.7);
  s.tgt_hi = num("tgt_hi", 1.0);
  s.dwell_mu = num("dwell_mu", 3.58);
  s.dwell_sigma = num("dwell_sigma", 0.5);
  s.dwell_max = (int32_t)num("dwell_max", 1024);
  s.arrival_rate = o.arrival_rate.empty() ? nullptr : o.arrival_rate.data();
  s.price_table = o.price_table.empty() ? nullptr : o.price_table.data();
  s.v2g = (int32_t)num("v2g", 0);
  s.port_pdis_kw = o.pdis.empty() ? nullptr : o.pdis.data();
  s.battery_kwh = num("battery_kwh", 0);
  s.battery_kw = num("battery_kw", 0);
  s.battery_tau = num("battery_tau", 0.8);
  s.battery_soc0 = num("battery_soc0", 0.5);
  s.alpha_degrad_battery = num("alpha_degrad_battery", 0);
  s.alpha_degrad_cars = num("alpha_degrad_cars", 0);
  s.charge_sensitive_share = num("charge_sensitive_share", 0);
  s.alpha_sat1 = num("alpha_sat1", 0);
  s.beta_sat1 = num("beta_sat1", 0);
  s.n_price_days = o.days.empty() ? 0 : (int32_t)(o.days.size() / s.steps_per_episode);
  s.price_days = o.days.empty() ? nullptr : o.days.data();
  s.n_car_models = o.models.empty() ? 0 : (int32_t)(o.models.size() / 4);
  s.car_models = o.models.empty() ? nullptr : o.models.data();
  s.port_dc = o.port_dc.empty() ? nullptr : o.port_dc.data();
}

struct Scenario {
  std::vector<std::unique_ptr<OwnedSpec>> mixture, policy, serve;
  std::vector<int64_t> counts;
};

Scenario parse(const char *path) {
  std::ifstream in(path);
  if (!in) {
    std::fprintf(stderr, "cannot open %s\n", path);
    std::exit(2);
  }
  Scenario sc;
  std::vector<std::unique_ptr<OwnedSpec>> *cur = nullptr;
  std::unique_ptr<OwnedSpec> spec;
  std::string line;
  while (std::getline(in, line)) {
    std::istringstream ls(line);
    std::string key;
    if (!(ls >> key)) continue;
    if (key == "section") {
      std::string name;
      ls >> name;
      cur = name == "mixture" ? &sc.mixture : name == "policy" ? &sc.policy : &sc.serve;
    } else if (key == "counts") {
      int64_t c;
      while (ls >> c) sc.counts.push_back(c);
    } else if (key == "spec") {
      spec.reset(new OwnedSpec());
    } else if (key == "end") {
      finish(*spec);
      cur->push_back(std::move(spec));
    } else {
      std::vector<double> v;
      double x;
      while (ls >> x) v.push_back(x);
      spec->f[key] = v;
    }
  }
  return sc;
}

struct Dev {
  void *p = nullptr;
  explicit Dev(size_t n) {
    if (hipMalloc(&p, n ? n : 1) != hipSuccess) {
      std::fprintf(stderr, "hipMalloc failed\n");
      std::exit(2);
    }
    (void)hipMemset(p, 0, n ? n : 1);
  }
  ~Dev() { (void)hipFree(p); }
  template <class T>
  T *as() const { return static_cast<T *>(p); }
};

struct Traj {
  std::unique_ptr<Dev> obs, act, rew, done;
  cx_traj t{};
  Traj(const cx_info &i, int T) {
    obs.reset(new Dev(4 * (size_t)T * i.obs_elems));
    act.reset(new Dev((size_t)T * i.total_ports));
    rew.reset(new Dev(4 * (size_t)T * i.n_envs));
    done.reset(new Dev((size_t)T * i.n_envs));
    t = cx_traj{obs->as<float>(), act->as<uint8_t>(), rew->as<float>(), done->as<uint8_t>()};
  }
};

void run_mixture(Scenario &sc, const char *cache) {
  std::vector<cx_station_spec> specs;
  std::vector<int32_t> ec;
  for (size_t c = 0; c < sc.mixture.size(); ++c) {
    specs.push_back(sc.mixture[c]->s);
    for (int64_t e = 0; e < sc.counts.at(c); ++e) ec.push_back((int32_t)c);
  }
  cx_ctx *ctx = nullptr;
  CK(cx_create_multi(specs.data(), (int32_t)specs.size(), ec.data(), (int64_t)ec.size(), 46, &ctx));
  cx_info info{};
  CK(cx_get_info(ctx, &info));
  const int T = 24;
  Traj tr(info, T);
  Dev act_in((size_t)T * info.total_ports);
  CK(cx_rollout(ctx, T, CX_ACT_RANDOM, CX_OUT_FULL, nullptr, &tr.t));
  CK(cx_rollout(ctx, T, CX_ACT_MAX, CX_OUT_REWARD, nullptr, &tr.t));
  CK(cx_rollout(ctx, T, CX_ACT_EXTERNAL, CX_OUT_ACT_REWARD, act_in.as<uint8_t>(), &tr.t));
  for (int k = 0; k < 3; ++k) CK(cx_step_ex(ctx, CX_ACT_RANDOM, nullptr, &tr.t));
  CK(cx_step(ctx, act_in.as<uint8_t>(), tr.t.obs, tr.t.reward, tr.t.done));
  CK(cx_reset(ctx, tr.t.obs));
  CK(cx_observe(ctx, tr.t.obs));
  // packings, block sizes and the stage, with rollouts launched back to back
  for (int stage = 0; stage < 2; ++stage) {
    CK(cx_set_obs_stage(ctx, stage));
    for (int w : {1, 2, 4, 8}) {
      for (int c = 0; c < info.n_classes; ++c) {
        cx_class_info ci{};
        CK(cx_get_class_info(ctx, c, &ci));
        CK(cx_set_packing(ctx, c, ci.slots >= 16 && (c + w) % 2 ? ci.slots / 4 >= 4 ? ci.slots / 4 : 4
                                                                 : (ci.slots <= 64 ? ci.slots : 64),
                          w));
      }
      CK(cx_rollout(ctx, T, CX_ACT_RANDOM, CX_OUT_FULL, nullptr, &tr.t));
      CK(cx_rollout(ctx, 5, CX_ACT_RANDOM, CX_OUT_FULL, nullptr, &tr.t));
      CK(cx_step_ex(ctx, CX_ACT_RANDOM, nullptr, &tr.t));
    }
  }
  // the autotuner: a search (written to the cache), then the cached answer
  for (int pass = 0; pass < 2; ++pass) {
    CK(cx_autotune(ctx, 16, cache));
    CK(cx_rollout(ctx, T, CX_ACT_RANDOM, CX_OUT_FULL, nullptr, &tr.t));
  }
  CK(cx_autotune(ctx, 3, nullptr));
  CK(cx_rollout(ctx, T, CX_ACT_RANDOM, CX_OUT_FULL, nullptr, &tr.t));
  // snapshots
  CK(cx_get_info(ctx, &info));
  std::vector<unsigned char> a(info.state_bytes), b(info.state_bytes);
  CK(cx_get_state(ctx, a.data(), a.size()));
  CK(cx_set_state(ctx, a.data(), a.size()));
  CK(cx_get_state(ctx, b.data(), b.size()));
  if (a != b) {
    std::fprintf(stderr, "DRIVE FAILED: snapshot round trip differs\n");
    std::exit(3);
  }
  CK(cx_synchronize(ctx));
  cx_destroy(ctx);
}

uint16_t bf16(float f) {
  uint32_t u;
  std::memcpy(&u, &f, 4);
  return (uint16_t)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}

void run_policy(Scenario &sc) {
  const cx_station_spec &s = sc.policy.at(0)->s;
  cx_ctx *ctx = nullptr;
  const int64_t E = 100;
  CK(cx_create(&s, E, 5, &ctx));
  const int H = 256, in = 6 * s.n_ports + 4, out = s.n_ports * (s.n_levels + 1);
  std::mt19937 rng(7);
  std::normal_distribution<float> nd(0.f, 0.05f);
  std::vector<uint16_t> w1((size_t)in * H), b1(H), w2((size_t)H * out), b2(out);
  for (auto *v : {&w1, &b1, &w2, &b2})
    for (auto &x : *v) x = bf16(nd(rng));
  CK(cx_set_policy(ctx, H, w1.data(), b1.data(), w2.data(), b2.data()));
  cx_info info{};
  CK(cx_get_info(ctx, &info));
  const int T = 6;
  Traj tr(info, T);
  CK(cx_rollout(ctx, T, CX_ACT_POLICY, CX_OUT_ACT_REWARD, nullptr, &tr.t));
  CK(cx_rollout(ctx, T, CX_ACT_POLICY, CX_OUT_FULL, nullptr, &tr.t));
  CK(cx_step_ex(ctx, CX_ACT_POLICY, nullptr, &tr.t));
  Dev logits(4 * (size_t)E * out);
  CK(cx_policy_logits(ctx, tr.t.obs, E, logits.as<float>()));
  CK(cx_policy_sample(ctx, tr.t.obs, E, 3, tr.t.actions));
  CK(cx_set_policy(ctx, H, w1.data(), b1.data(), w2.data(), b2.data()));  // replaced in place
  CK(cx_rollout(ctx, T, CX_ACT_POLICY, CX_OUT_REWARD, nullptr, &tr.t));
  // the rollout that allocates nothing: scratch in the library's fixed array
  CK(cx_rollout_policy_noalloc(ctx, T, CX_OUT_ACT_REWARD, &tr.t));
  CK(cx_rollout_policy_noalloc(ctx, T, CX_OUT_FULL, &tr.t));
  CK(cx_synchronize(ctx));
  cx_destroy(ctx);
}

void run_server(Scenario &sc, int simulate_ns) {
  cx_server_opts o{8, 16, 4, simulate_ns};
  cx_server *srv = nullptr;
  CK(cx_server_create((size_t)512 << 20, &o, &srv));
  std::atomic<int> done_count{0};
  std::atomic<bool> bad{false};
  auto client = [&](int id) {
    std::mt19937 rng(100 + id);
    std::vector<uint64_t> mine;
    for (int k = 0; k < 6; ++k) {
      cx_request rq{};
      rq.spec = sc.serve[rng() % sc.serve.size()]->s;
      rq.n_envs = 64 + rng() % 500;
      rq.T = (k % 2) ? 12 : 40;
      rq.seed = 1000 + 10 * id + k;
      rq.out_mode = (cx_out_mode)(k % 3);
      rq.act_mode = (k % 2) ? CX_ACT_MAX : CX_ACT_RANDOM;
      uint64_t t = 0;
      if (cx_submit(srv, &rq, &t) != CX_OK) {
        bad = true;
        return;
      }
      mine.push_back(t);
      if (k == 2) (void)cx_cancel(srv, t);
    }
    for (size_t i = 0; i < mine.size(); ++i) {
      cx_result r{};
      if (i % 2) {
        while (cx_poll(srv, mine[i], &r) == CX_E_BUSY) std::this_thread::sleep_for(std::chrono::microseconds(50));
      } else if (cx_wait(srv, mine[i], &r) != CX_OK) {
        bad = true;
      }
      if (r.status != CX_OK && r.status != CX_E_CANCELLED) bad = true;
      if (cx_release(srv, mine[i]) != CX_OK) bad = true;
      done_count++;
    }
  };
  std::vector<std::thread> th;
  for (int i = 0; i < 4; ++i) th.emplace_back(client, i);
  for (int k = 0; k < 50; ++k) {
    double busy;
    int64_t steps, launches;
    int32_t peak;
    CK(cx_server_stats(srv, &busy, &steps, &launches, &peak));
    std::this_thread::sleep_for(std::chrono::microseconds(200));
  }
  for (auto &t : th) t.join();
  if (bad || done_count != 24) {
    std::fprintf(stderr, "DRIVE FAILED: serving (simulate_ns %d): %d results, errors %d: %s\n", simulate_ns,
                 done_count.load(), (int)bad.load(), cx_last_error());
    std::exit(3);
  }
  cx_server_destroy(srv);
}

// Self-checks of the fake device: a rollout into an observation buffer one
// step too short, and a step into a freed buffer, must both be refused.
void run_selfcheck(Scenario &sc, const std::string &what) {
  cx_ctx *ctx = nullptr;
  CK(cx_create(&sc.mixture.at(3)->s, 37, 1, &ctx));
  cx_info info{};
  CK(cx_get_info(ctx, &info));
  const int T = 8;
  Traj tr(info, T);
  if (what == "--undersized") {
    Dev small(4 * (size_t)(T - 1) * info.obs_elems);
    cx_traj t = tr.t;
    t.obs = small.as<float>();
    CK(cx_rollout(ctx, T, CX_ACT_RANDOM, CX_OUT_FULL, nullptr, &t));
    CK(cx_synchronize(ctx));
  } else {
    float *gone = nullptr;
    {
      Dev d(4 * (size_t)info.obs_elems);
      gone = d.as<float>();
    }
    CK(cx_step(ctx, nullptr, gone, tr.t.reward, tr.t.done) == CX_E_INVALID ? CX_OK : CX_E_INVALID);
    cx_traj t = tr.t;
    t.obs = gone;
    CK(cx_step_ex(ctx, CX_ACT_RANDOM, nullptr, &t));
    CK(cx_synchronize(ctx));
  }
  std::printf("self-check %s was not caught\n", what.c_str());
  std::exit(4);
}

}  // namespace

int main(int argc, char **argv) {
  if (argc < 3) {
    std::fprintf(stderr, "usage: drive SCENARIO CACHE [--undersized|--freed]\n");
    return 2;
  }
  Scenario sc = parse(argv[1]);
  if (argc > 3) run_selfcheck(sc, argv[3]);
  const long live0 = fake_hip_live_allocations();
  run_mixture(sc, argv[2]);
  std::printf("mixture ok\n");
  run_policy(sc);
  std::printf("policy ok\n");
  run_server(sc, 0);
  std::printf("serving ok\n");
  run_server(sc, 20);
  std::printf("simulated serving ok\n");
  const long live = fake_hip_live_allocations() - live0;
  std::printf("graph execs destroyed with launches in flight: %ld\n", fake_hip_graph_destroys_in_flight());
  std::printf("device allocations left: %ld\n", live);
  std::printf("DRIVE OK\n");
  return 0;
}
