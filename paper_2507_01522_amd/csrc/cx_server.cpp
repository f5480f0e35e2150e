// cx_server.cpp -- serving: continuous batching of rollout requests.
//
// One scheduler thread per server.  The server reserves its whole memory
// budget as one device arena at create; a request's block (class constants,
// state, server-owned records) is carved from it first-fit and returned on
// release, so admission makes no allocation call.  Each loop the scheduler
// retires finished chunks, admits queued requests first-come-first-served while
// a block fits, and launches the next chunk: one per-segment launch of the
// rollout kernels in which every admitted request is one segment with its own
// horizon, step counter, seed and output pointers.  Two chunks may be in flight,
// so the GPU never idles while the host prepares the next one; a request that
// arrives joins at the next chunk boundary.  Chunking does not change results:
// the state round-trips HBM exactly and every draw is keyed by the request's
// own (seed, env, step).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "cx_ctx.h"

namespace cx {
namespace {

constexpr int kRing = 8;         // segment-table staging buffers
constexpr int kMaxInflight = 2;  // chunks queued on the stream at once

size_t a256(size_t x) { return (x + 255) & ~(size_t)255; }

enum class RState { Pending, Active, Done, Cancelled, Failed };

struct Req {
  uint64_t ticket = 0;
  SpecCopy spec;
  Compiled comp;
  Tables tab;
  int64_t n_envs = 0;
  int32_t T = 0;
  uint64_t seed = 0;
  cx_out_mode out_mode = CX_OUT_FULL;
  cx_action_mode act_mode = CX_ACT_RANDOM;
  cx_traj user{};                // caller buffers
  cx_traj traj{};                // effective output buffers
  // device layout: [class block | state | server-owned outputs]
  size_t class_bytes = 0, state_bytes = 0, out_bytes = 0, total = 0;
  size_t off_q = 0, off_u = 0, off_cap = 0, off_pl = 0, off_dw = 0, off_ret = 0, off_bsoc = 0, off_bp = 0;
  size_t off_ut = 0, off_rb = 0;
  size_t off_obs = 0, off_act = 0, off_rew = 0, off_done = 0;
  std::vector<unsigned char> class_host;  // kept until the request ends (async upload source)
  ClassDev view{};
  void *mem = nullptr;
  int lanes = 16;
  // progress
  RState state = RState::Pending;
  bool cancel = false;
  int32_t launched = 0;          // steps handed to the GPU
  int32_t retired = 0;           // steps whose chunk finished
  bool admitted = false;         // holds its block of the arena until released
  size_t arena_off = 0;
  int inflight = 0;
  uint32_t g = 0;
  int32_t t_day = 0;
  cx_status status = CX_OK;
  double submit_s = 0, admit_s = 0, done_s = 0;
};

struct Chunk {
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  std::vector<std::pair<uint64_t, int32_t>> members;  // ticket, steps in this chunk
  int64_t env_steps = 0;
  double sim_done = 0;           // simulated completion time (host clock)
};

// First-fit allocator over [0, size): free ranges keyed by offset, coalesced
// on release.
struct Arena {
  size_t size = 0;
  std::map<size_t, size_t> free_ranges;  // offset -> length
  void init(size_t n) {
    size = n;
    free_ranges.clear();
    free_ranges[0] = n;
  }
  bool take(size_t n, size_t *off) {
    for (auto it = free_ranges.begin(); it != free_ranges.end(); ++it) {
      if (it->second < n) continue;
      *off = it->first;
      const size_t rest = it->second - n, at = it->first + n;
      free_ranges.erase(it);
      if (rest) free_ranges[at] = rest;
      return true;
    }
    return false;
  }
  void give(size_t off, size_t n) {
    auto next = free_ranges.lower_bound(off);
    if (next != free_ranges.end() && off + n == next->first) {
      n += next->second;
      next = free_ranges.erase(next);
    }
    if (next != free_ranges.begin()) {
      auto prev = std::prev(next);
      if (prev->first + prev->second == off) {
        prev->second += n;
        return;
      }
    }
    free_ranges[off] = n;
  }
};

}  // namespace
}  // namespace cx

struct cx_server {
  size_t budget = 0, used = 0;
  cx_server_opts opts{};
  bool sim = false;
  int device = 0;
  hipStream_t stream = nullptr;
  // a chunk's kernels (one per packing) run concurrently on these, forked from
  // and joined back into `stream` with events
  static constexpr int kAux = 4;
  hipStream_t aux[kAux] = {};
  hipEvent_t ev_fork = nullptr, ev_join[kAux] = {};
  void *arena_mem = nullptr;   // the budget, reserved at create (none when simulating)
  cx::Arena arena;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::thread th;
  bool stop = false;
  bool failed = false;
  std::map<uint64_t, std::unique_ptr<cx::Req>> reqs;
  std::deque<uint64_t> pending;
  std::vector<uint64_t> active;
  std::deque<cx::Chunk> inflight;
  uint64_t next_ticket = 1;
  cx::SegDev *ring_host[cx::kRing] = {};
  cx::SegDev *ring_dev[cx::kRing] = {};
  hipEvent_t ring_ev[cx::kRing] = {};
  bool ring_used[cx::kRing] = {};
  int ring_next = 0;
  double busy_s = 0;
  int64_t env_steps = 0, launches = 0;
  int32_t peak_active = 0;
  std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();

  double now() const {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
};

namespace cx {
namespace {

// Byte sizes and offsets of a request's device block.
void plan(Req &r) {
  const int64_t E = r.n_envs, S = r.comp.S, A = r.comp.n_act, T = r.T;
  const int64_t od = r.comp.obs_dim;
  r.class_bytes = a256(class_block(r.spec, r.comp, r.tab, nullptr, nullptr, nullptr));
  size_t o = r.class_bytes;
  r.off_q = o; o = a256(o + 8 * (size_t)(E * S));
  r.off_u = o; o = a256(o + 4 * (size_t)(E * S));
  r.off_cap = o; o = a256(o + 4 * (size_t)(E * S));
  r.off_pl = o; o = a256(o + 4 * (size_t)(E * S));
  r.off_dw = o; o = a256(o + 2 * (size_t)(E * S));
  r.off_ret = o; o = a256(o + 8 * (size_t)E);
  r.off_bsoc = o; o = a256(o + (r.comp.battery ? 8 * (size_t)E : 0));
  r.off_bp = o; o = a256(o + (r.comp.battery ? 4 * (size_t)E : 0));
  r.off_ut = o; o = a256(o + (r.comp.users ? (size_t)(E * S) : 0));
  r.off_rb = o; o = a256(o + (r.comp.n_models > 0 ? 4 * (size_t)(E * S) : 0));
  r.state_bytes = o - r.class_bytes;
  const size_t out0 = o;
  const bool want_obs = r.out_mode == CX_OUT_FULL;
  const bool want_act = r.out_mode != CX_OUT_REWARD;
  r.off_obs = r.off_act = r.off_rew = r.off_done = 0;
  if (want_obs && !r.user.obs) { r.off_obs = o; o = a256(o + 4 * (size_t)(T * E * od)); }
  if (want_act && !r.user.actions) { r.off_act = o; o = a256(o + (size_t)(T * E * A)); }
  if (!r.user.reward) { r.off_rew = o; o = a256(o + 4 * (size_t)(T * E)); }
  if (!r.user.done) { r.off_done = o; o = a256(o + (size_t)(T * E)); }
  r.out_bytes = o - out0;
  r.total = o;
}

void bind(Req &r) {
  unsigned char *b = static_cast<unsigned char *>(r.mem);
  const bool want_obs = r.out_mode == CX_OUT_FULL;
  const bool want_act = r.out_mode != CX_OUT_REWARD;
  r.traj.obs = want_obs ? (r.user.obs ? r.user.obs : reinterpret_cast<float *>(b + r.off_obs)) : nullptr;
  r.traj.actions = want_act ? (r.user.actions ? r.user.actions : b + r.off_act) : nullptr;
  r.traj.reward = r.user.reward ? r.user.reward : reinterpret_cast<float *>(b + r.off_rew);
  r.traj.done = r.user.done ? r.user.done : b + r.off_done;
}

cx_status fail(cx_status st, const char *m) { return fail_status(st, m); }

void finish(cx_server *s, Req &r, RState st, cx_status status) {
  r.state = st;
  r.status = status;
  r.done_s = s->now();
  s->active.erase(std::remove(s->active.begin(), s->active.end(), r.ticket), s->active.end());
  s->cv_done.notify_all();
}

// Retire chunks whose completion event has passed (or whose simulated end time has).
bool retire(cx_server *s) {
  bool any = false;
  while (!s->inflight.empty()) {
    Chunk &c = s->inflight.front();
    if (s->sim) {
      if (s->now() < c.sim_done) break;
    } else {
      const hipError_t q = hipEventQuery(c.ev1);
      if (q == hipErrorNotReady) break;
      if (q != hipSuccess) {
        s->failed = true;
        for (auto &m : c.members) {
          auto it = s->reqs.find(m.first);
          if (it != s->reqs.end() && it->second->state == RState::Active)
            finish(s, *it->second, RState::Failed, CX_E_DEVICE);
        }
      } else {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, c.ev0, c.ev1) == hipSuccess) s->busy_s += ms * 1e-3;
      }
      (void)hipEventDestroy(c.ev0);
      (void)hipEventDestroy(c.ev1);
    }
    s->env_steps += c.env_steps;
    for (auto &m : c.members) {
      auto it = s->reqs.find(m.first);
      if (it == s->reqs.end()) continue;
      Req &r = *it->second;
      r.inflight -= 1;
      r.retired += m.second;
      if (r.state != RState::Active) continue;
      if (r.retired == r.T) finish(s, r, RState::Done, CX_OK);
      else if (r.cancel && r.inflight == 0) finish(s, r, RState::Cancelled, CX_E_CANCELLED);
    }
    s->inflight.pop_front();
    any = true;
  }
  return any;
}

// Admit queued requests in arrival order while they fit.
bool admit(cx_server *s) {
  bool any = false;
  while (!s->pending.empty() && (int)s->active.size() < s->opts.max_active) {
    auto it = s->reqs.find(s->pending.front());
    if (it == s->reqs.end() || it->second->state != RState::Pending) {
      s->pending.pop_front();
      continue;
    }
    Req &r = *it->second;
    if (!s->arena.take(r.total, &r.arena_off)) break;   // first come, first served: no skipping ahead
    if (!s->sim) {
      r.mem = static_cast<unsigned char *>(s->arena_mem) + r.arena_off;
      unsigned char *b = static_cast<unsigned char *>(r.mem);
      class_block(r.spec, r.comp, r.tab, b, &r.class_host, &r.view);
      if (hipMemcpyAsync(b, r.class_host.data(), r.class_host.size(), hipMemcpyHostToDevice, s->stream) !=
              hipSuccess ||
          hipMemsetAsync(b + r.class_bytes, 0, r.state_bytes, s->stream) != hipSuccess ||
          (r.comp.battery && launch_fill_f64(reinterpret_cast<double *>(b + r.off_bsoc), r.n_envs,
                                             r.spec.s.battery_soc0, s->stream) != hipSuccess)) {
        s->arena.give(r.arena_off, r.total);
        r.mem = nullptr;
        s->failed = true;
        finish(s, r, RState::Failed, CX_E_DEVICE);
        s->pending.pop_front();
        continue;
      }
      bind(r);
    } else {
      class_block(r.spec, r.comp, r.tab, nullptr, nullptr, &r.view);
    }
    s->used += r.total;
    r.admitted = true;
    r.state = RState::Active;
    r.admit_s = s->now();
    s->active.push_back(r.ticket);
    s->peak_active = std::max<int32_t>(s->peak_active, (int32_t)s->active.size());
    s->pending.pop_front();
    any = true;
  }
  return any;
}

// Launch the next chunk over every admitted request with steps left.
bool launch(cx_server *s) {
  if ((int)s->inflight.size() >= kMaxInflight) return false;
  std::vector<SegDev> segs;
  std::vector<int> dl;
  std::vector<int> kind;
  Chunk c;
  for (uint64_t tk : s->active) {
    Req &r = *s->reqs[tk];
    if (r.cancel || r.launched >= r.T) continue;
    const int32_t n = std::min<int32_t>(s->opts.chunk_steps, r.T - r.launched);
    SegDev sg{};
    const int L = r.lanes, P = r.comp.S / r.lanes, spw = 64 / L;
    unsigned char *b = static_cast<unsigned char *>(r.mem);
    const int64_t E = r.n_envs, A = r.comp.n_act, od = r.comp.obs_dim, t = r.launched;
    sg.cls = reinterpret_cast<const ClassDev *>(b);
    sg.env0 = 0;
    sg.n_envs = E;
    sg.n_groups = (int32_t)((E + spw - 1) / spw);
    sg.pack = pack_id(L, P);
    sg.obs_dim = (int32_t)od;
    sg.seed = r.seed;
    if (b) {
      sg.q = reinterpret_cast<double *>(b + r.off_q);
      sg.u = reinterpret_cast<float *>(b + r.off_u);
      sg.cap = reinterpret_cast<float *>(b + r.off_cap);
      sg.p_last = reinterpret_cast<float *>(b + r.off_pl);
      sg.dwell = reinterpret_cast<int16_t *>(b + r.off_dw);
      sg.ret = reinterpret_cast<double *>(b + r.off_ret);
      sg.bsoc = reinterpret_cast<double *>(b + r.off_bsoc);
      sg.bp = reinterpret_cast<float *>(b + r.off_bp);
      sg.utype = b + r.off_ut;
      sg.rbar = reinterpret_cast<float *>(b + r.off_rb);
      sg.obs = r.traj.obs ? r.traj.obs + t * E * od : nullptr;
      sg.act = r.traj.actions ? r.traj.actions + t * E * A : nullptr;
      sg.reward = r.traj.reward + t * E;
      sg.done = r.traj.done + t * E;
    }
    sg.T = n;
    sg.t_day0 = r.t_day;
    sg.g0 = r.g;
    sg.mode = r.act_mode;
    sg.out_mode = r.out_mode;
    sg.obs_stride = E * od;
    sg.act_stride = E * A;
    sg.env_stride = E;
    segs.push_back(sg);
    dl.push_back(r.tab.dwell_log2);
    kind.push_back(r.view.kind);
    c.members.push_back({tk, n});
    c.env_steps += E * n;
    r.launched += n;
    r.g += (uint32_t)n;
    r.t_day = (int32_t)(((int64_t)r.t_day + n) % r.spec.s.steps_per_episode);
    r.inflight += 1;
  }
  if (c.members.empty()) return false;
  s->launches += 1;
  if (s->sim) {
    const double start = s->inflight.empty() ? s->now() : std::max(s->now(), s->inflight.back().sim_done);
    c.sim_done = start + 1e-9 * (double)s->opts.simulate_ns * (double)c.env_steps;
    s->busy_s += c.sim_done - start;
    s->inflight.push_back(std::move(c));
    return true;
  }
  std::vector<SegDev> ordered;
  std::vector<LaunchGroup> groups;
  build_groups(segs, dl, kind, s->opts.waves_per_block, &ordered, &groups);
  const int slot = s->ring_next;
  s->ring_next = (s->ring_next + 1) % kRing;
  if (s->ring_used[slot]) (void)hipEventSynchronize(s->ring_ev[slot]);  // earlier copy out of this buffer done
  std::memcpy(s->ring_host[slot], ordered.data(), sizeof(SegDev) * ordered.size());
  hipError_t e = hipMemcpyAsync(s->ring_dev[slot], s->ring_host[slot], sizeof(SegDev) * ordered.size(),
                                hipMemcpyHostToDevice, s->stream);
  if (e == hipSuccess) e = hipEventRecord(s->ring_ev[slot], s->stream);
  s->ring_used[slot] = true;
  if (e == hipSuccess) e = hipEventCreate(&c.ev0);
  if (e == hipSuccess) e = hipEventCreate(&c.ev1);
  if (e == hipSuccess) e = hipEventRecord(c.ev0, s->stream);
  LaunchArgs a{};
  a.segs = s->ring_dev[slot];
  a.per_segment = 1;
  if (e == hipSuccess) {
    if (groups.size() <= 1) {
      e = launch_groups(a, groups.data(), (int)groups.size(), s->stream);
    } else {
      // fork: each packing's kernel on its own stream, then join
      const int n_aux = std::min<int>((int)groups.size(), cx_server::kAux);
      e = hipEventRecord(s->ev_fork, s->stream);
      for (int k = 0; k < n_aux && e == hipSuccess; ++k) e = hipStreamWaitEvent(s->aux[k], s->ev_fork, 0);
      for (size_t gi = 0; gi < groups.size() && e == hipSuccess; ++gi)
        e = launch_groups(a, groups.data() + gi, 1, s->aux[gi % n_aux]);
      for (int k = 0; k < n_aux && e == hipSuccess; ++k) {
        e = hipEventRecord(s->ev_join[k], s->aux[k]);
        if (e == hipSuccess) e = hipStreamWaitEvent(s->stream, s->ev_join[k], 0);
      }
    }
  }
  if (e == hipSuccess) e = hipEventRecord(c.ev1, s->stream);
  if (e != hipSuccess) {
    s->failed = true;
    for (auto &m : c.members) finish(s, *s->reqs[m.first], RState::Failed, CX_E_DEVICE);
    if (c.ev0) (void)hipEventDestroy(c.ev0);
    if (c.ev1) (void)hipEventDestroy(c.ev1);
    return true;
  }
  s->inflight.push_back(std::move(c));
  return true;
}

// Requests cancelled while running end once their chunks have retired.
void settle_cancels(cx_server *s) {
  std::vector<uint64_t> done;
  for (uint64_t tk : s->active) {
    Req &r = *s->reqs[tk];
    if (r.cancel && r.inflight == 0) done.push_back(tk);
  }
  for (uint64_t tk : done) finish(s, *s->reqs[tk], RState::Cancelled, CX_E_CANCELLED);
}

void loop(cx_server *s) {
  if (!s->sim) (void)hipSetDevice(s->device);
  std::unique_lock<std::mutex> lk(s->mu);
  while (!s->stop) {
    bool progress = retire(s);
    settle_cancels(s);
    if (!s->failed) {
      progress |= admit(s);
      progress |= launch(s);
    }
    if (progress) continue;
    if (s->inflight.empty())
      s->cv_work.wait(lk);
    else
      s->cv_work.wait_for(lk, std::chrono::microseconds(20));
  }
}

void fill_result(const Req &r, cx_result *res) {
  std::memset(res, 0, sizeof *res);
  res->status = r.status;
  res->n_envs = r.n_envs;
  res->T = r.T;
  res->traj = r.traj;
  res->submit_s = r.submit_s;
  res->admit_s = r.admit_s;
  res->done_s = r.done_s;
  res->bytes = (int64_t)r.total;
}

bool finished(const Req &r) {
  return r.state == RState::Done || r.state == RState::Cancelled || r.state == RState::Failed;
}

}  // namespace
}  // namespace cx

using namespace cx;

extern "C" {

cx_status cx_server_create(size_t hbm_budget_bytes, const cx_server_opts *opts, cx_server **out) {
  if (!out) return fail(CX_E_INVALID, "out must not be NULL");
  *out = nullptr;
  if (hbm_budget_bytes == 0) return fail(CX_E_INVALID, "budget must be > 0");
  cx_server_opts o{32, 256, 4, 0};
  if (opts) o = *opts;
  if (o.chunk_steps <= 0) o.chunk_steps = 144;
  if (o.max_active <= 0) o.max_active = 256;
  if (o.waves_per_block <= 0) o.waves_per_block = 4;
  if (o.chunk_steps > 4096 || o.max_active > 65536 || o.waves_per_block > kMaxWaves || o.simulate_ns < 0)
    return fail(CX_E_INVALID, "server options out of range");
  std::unique_ptr<cx_server> s(new cx_server());
  s->budget = hbm_budget_bytes;
  s->arena.init(hbm_budget_bytes);
  s->opts = o;
  s->sim = o.simulate_ns > 0;
  if (!s->sim) {
    if (hipGetDevice(&s->device) != hipSuccess) return fail(CX_E_DEVICE, "no HIP device");
    if (hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking) != hipSuccess)
      return fail(CX_E_DEVICE, "stream creation failed");
    bool ok = hipEventCreateWithFlags(&s->ev_fork, hipEventDisableTiming) == hipSuccess;
    for (int k = 0; k < cx_server::kAux && ok; ++k)
      ok = hipStreamCreateWithFlags(&s->aux[k], hipStreamNonBlocking) == hipSuccess &&
           hipEventCreateWithFlags(&s->ev_join[k], hipEventDisableTiming) == hipSuccess;
    if (!ok) {
      cx_server_destroy(s.release());
      return fail(CX_E_DEVICE, "server stream creation failed");
    }
    if (hipMalloc(&s->arena_mem, hbm_budget_bytes) != hipSuccess) {
      s->arena_mem = nullptr;
      cx_server_destroy(s.release());
      return fail(CX_E_OOM, "the memory budget could not be reserved on the device");
    }
    const size_t tb = sizeof(SegDev) * (size_t)o.max_active;
    for (int i = 0; i < kRing; ++i) {
      if (hipHostMalloc(reinterpret_cast<void **>(&s->ring_host[i]), tb, hipHostMallocDefault) != hipSuccess ||
          hipMalloc(reinterpret_cast<void **>(&s->ring_dev[i]), tb) != hipSuccess ||
          hipEventCreateWithFlags(&s->ring_ev[i], hipEventDisableTiming) != hipSuccess) {
        cx_server_destroy(s.release());
        return fail(CX_E_OOM, "server staging allocation failed");
      }
    }
  }
  cx_server *raw = s.release();
  raw->th = std::thread(loop, raw);
  *out = raw;
  return CX_OK;
}

cx_status cx_submit(cx_server *s, const cx_request *req, uint64_t *ticket) {
  if (!s || !req || !ticket) return fail(CX_E_INVALID, "NULL argument");
  if (req->n_envs < 1 || req->n_envs > (int64_t)1 << 28) return fail(CX_E_INVALID, "n_envs must be in 1..2^28");
  if (req->T < 1 || req->T > (1 << 20)) return fail(CX_E_INVALID, "T must be in 1..2^20");
  if (req->act_mode != CX_ACT_RANDOM && req->act_mode != CX_ACT_MAX)
    return fail(CX_E_INVALID, "serving runs RANDOM or MAX actions");
  if (req->out_mode < CX_OUT_FULL || req->out_mode > CX_OUT_ACT_REWARD) return fail(CX_E_INVALID, "bad out mode");
  std::unique_ptr<Req> r(new Req());
  std::string err;
  if (!copy_spec(req->spec, &r->spec, &err) || !compile_spec(r->spec, &r->comp, &err))
    return fail_status(CX_E_INVALID, "station spec: " + err);
  build_tables(r->spec, &r->tab);
  if (!tables_monotone(r->tab)) return fail(CX_E_INVALID, "sampling tables are not monotone");
  if ((uint64_t)req->n_envs * (uint64_t)r->comp.obs_dim * 4 >= (1ull << 32))
    return fail(CX_E_INVALID, "request too large for one segment (n_envs * obs_dim * 4 >= 2^32)");
  r->n_envs = req->n_envs;
  r->T = req->T;
  r->seed = req->seed;
  r->out_mode = req->out_mode;
  r->act_mode = req->act_mode;
  r->user = req->out;
  r->lanes = default_lanes(r->comp.S);
  plan(*r);
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->failed) return fail(CX_E_DEVICE, "server has a device error");
  if (r->total > s->budget) return fail(CX_E_BUDGET, "request can never fit the memory budget");
  r->ticket = s->next_ticket++;
  r->submit_s = s->now();
  *ticket = r->ticket;
  s->pending.push_back(r->ticket);
  s->reqs[r->ticket] = std::move(r);
  s->cv_work.notify_all();
  return CX_OK;
}

cx_status cx_poll(cx_server *s, uint64_t ticket, cx_result *res) {
  if (!s || !res) return fail(CX_E_INVALID, "NULL argument");
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return fail(CX_E_NOTFOUND, "unknown ticket");
  fill_result(*it->second, res);
  if (!finished(*it->second)) return CX_E_BUSY;
  return CX_OK;
}

cx_status cx_wait(cx_server *s, uint64_t ticket, cx_result *res) {
  if (!s || !res) return fail(CX_E_INVALID, "NULL argument");
  std::unique_lock<std::mutex> lk(s->mu);
  for (;;) {
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return fail(CX_E_NOTFOUND, "unknown ticket");
    if (finished(*it->second)) {
      fill_result(*it->second, res);
      return CX_OK;
    }
    s->cv_done.wait(lk);
  }
}

cx_status cx_cancel(cx_server *s, uint64_t ticket) {
  if (!s) return fail(CX_E_INVALID, "NULL argument");
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return fail(CX_E_NOTFOUND, "unknown ticket");
  Req &r = *it->second;
  if (r.state == RState::Pending) {
    s->pending.erase(std::remove(s->pending.begin(), s->pending.end(), ticket), s->pending.end());
    r.state = RState::Cancelled;
    r.status = CX_E_CANCELLED;
    r.done_s = s->now();
    s->cv_done.notify_all();
  } else if (r.state == RState::Active) {
    r.cancel = true;
  }
  s->cv_work.notify_all();
  return CX_OK;
}

cx_status cx_release(cx_server *s, uint64_t ticket) {
  if (!s) return fail(CX_E_INVALID, "NULL argument");
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return fail(CX_E_NOTFOUND, "unknown ticket");
  Req &r = *it->second;
  if (!finished(r)) return fail(CX_E_BUSY, "request still queued or running");
  // every chunk that used the block has retired, so it may be handed out again
  if (r.admitted) {
    s->arena.give(r.arena_off, r.total);
    s->used -= r.total;
  }
  s->reqs.erase(it);
  s->cv_work.notify_all();
  return CX_OK;
}

cx_status cx_server_stats(cx_server *s, double *busy_s, int64_t *env_steps, int64_t *launches,
                          int32_t *peak_active) {
  if (!s) return fail(CX_E_INVALID, "NULL argument");
  std::lock_guard<std::mutex> lk(s->mu);
  if (busy_s) *busy_s = s->busy_s;
  if (env_steps) *env_steps = s->env_steps;
  if (launches) *launches = s->launches;
  if (peak_active) *peak_active = s->peak_active;
  return CX_OK;
}

void cx_server_destroy(cx_server *s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
    s->cv_work.notify_all();
  }
  if (s->th.joinable()) s->th.join();
  if (!s->sim) {
    if (s->stream) (void)hipStreamSynchronize(s->stream);
    for (auto &c : s->inflight) {
      if (c.ev0) (void)hipEventDestroy(c.ev0);
      if (c.ev1) (void)hipEventDestroy(c.ev1);
    }
    if (s->arena_mem) (void)hipFree(s->arena_mem);
    for (int i = 0; i < kRing; ++i) {
      if (s->ring_host[i]) (void)hipHostFree(s->ring_host[i]);
      if (s->ring_dev[i]) (void)hipFree(s->ring_dev[i]);
      if (s->ring_ev[i]) (void)hipEventDestroy(s->ring_ev[i]);
    }
    for (int k = 0; k < cx_server::kAux; ++k) {
      if (s->aux[k]) (void)hipStreamSynchronize(s->aux[k]);
      if (s->aux[k]) (void)hipStreamDestroy(s->aux[k]);
      if (s->ev_join[k]) (void)hipEventDestroy(s->ev_join[k]);
    }
    if (s->ev_fork) (void)hipEventDestroy(s->ev_fork);
    if (s->stream) (void)hipStreamDestroy(s->stream);
  }
  delete s;
}

}  // extern "C"
