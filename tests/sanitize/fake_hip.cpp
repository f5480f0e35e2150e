// fake_hip.cpp -- a host-only stand-in for the HIP runtime, for sanitizer
// builds of the library's host code (test infrastructure).
//
// "Device" memory is host heap memory, so AddressSanitizer sees every access the
// fake device makes.  A device thread executes the queued work in order, each
// item after a short random delay, so host code that forgets to wait for the
// device races with it exactly as on a GPU (ThreadSanitizer sees those races).
// Kernels are not computed: a kernel "runs" by checking every range of memory
// that the kernel would read or write, from its launch arguments and the
// segment tables in device memory as they are at execution time -- each range
// must lie inside one live allocation (and is touched, for the sanitizer).
// Graph nodes keep their own copy of the kernel arguments, as the runtime does.
#include <hip/hip_runtime.h>

#include <cxxabi.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <functional>
#include <map>
#include <memory>
#include <mutex>
#include <random>
#include <string>
#include <thread>
#include <vector>

#include "cx_internal.h"

namespace fake {

[[noreturn]] void die(const char *fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  std::fprintf(stderr, "FAKE-HIP ERROR: ");
  std::vfprintf(stderr, fmt, ap);
  std::fprintf(stderr, "\n");
  va_end(ap);
  std::fflush(stderr);
  std::abort();
}

struct Alloc {
  size_t size;
  bool pinned;  // host memory from hipHostMalloc
  bool symbol = false;  // a __device__ variable of the image (lives until the process ends)
};

std::mutex amu;                            // guards allocs and symbols
std::map<uintptr_t, Alloc> allocs;         // live allocations by base address (used after main starts)
// device copies of __device__ variables by host shadow address (filled by the
// module constructors, before main: a function-local static)
struct Symbol {
  size_t size;
  void *dev;
};
std::map<const void *, Symbol> &symbols() {
  static std::map<const void *, Symbol> m;
  return m;
}
std::atomic<long> n_graph_destroy_in_flight{0};

// Does [p, p + n) lie inside one live allocation?  (n = 0: p inside or at its end.)
bool in_alloc(const void *p, size_t n, bool *pinned = nullptr) {
  std::lock_guard<std::mutex> lk(amu);
  const uintptr_t a = reinterpret_cast<uintptr_t>(p);
  auto it = allocs.upper_bound(a);
  if (it == allocs.begin()) return false;
  --it;
  if (a < it->first || a + n > it->first + it->second.size) return false;
  if (pinned) *pinned = it->second.pinned;
  return true;
}

void touch(const void *p, size_t n) {
  if (n == 0) return;
  const volatile unsigned char *b = static_cast<const volatile unsigned char *>(p);
  (void)b[0];
  (void)b[n - 1];
}

// A device range that a kernel or copy accesses: must be in one live allocation.
void need(const void *p, size_t n, const char *what, const std::string &where) {
  if (n == 0) return;
  if (!p) die("%s: %s is NULL (%zu bytes)", where.c_str(), what, n);
  if (!in_alloc(p, n)) die("%s: %s [%p, +%zu) is not inside a live device allocation", where.c_str(), what, p, n);
  touch(p, n);
}

// ---- the device: one FIFO of work, executed by one thread -----------------
struct Op {
  uint64_t seq;
  std::function<void()> run;
};

struct Device {
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Op> q;
  uint64_t next_seq = 1, done_seq = 0;
  double clock_ms = 0;  // device time: advanced by every kernel
  std::thread th;
  bool stop = false;
  std::mt19937 rng{12345};

  Device() { th = std::thread([this] { loop(); }); }
  ~Device() {
    {
      std::lock_guard<std::mutex> lk(mu);
      stop = true;
    }
    cv_work.notify_all();
    th.join();
  }
  void loop() {
    std::unique_lock<std::mutex> lk(mu);
    for (;;) {
      cv_work.wait(lk, [&] { return stop || !q.empty(); });
      if (q.empty()) return;
      Op op = std::move(q.front());
      q.pop_front();
      const int delay_us = (int)(rng() % 40);
      lk.unlock();
      std::this_thread::sleep_for(std::chrono::microseconds(delay_us));
      op.run();
      lk.lock();
      done_seq = op.seq;
      cv_done.notify_all();
    }
  }
  uint64_t push(std::function<void()> f) {
    std::lock_guard<std::mutex> lk(mu);
    const uint64_t s = next_seq++;
    q.push_back(Op{s, std::move(f)});
    cv_work.notify_all();
    return s;
  }
  void wait_for(uint64_t s) {
    std::unique_lock<std::mutex> lk(mu);
    cv_done.wait(lk, [&] { return done_seq >= s; });
  }
  void sync() {
    uint64_t s;
    {
      std::lock_guard<std::mutex> lk(mu);
      s = next_seq - 1;
    }
    wait_for(s);
  }
};

Device &dev() {
  static Device d;
  return d;
}

thread_local hipError_t last_error = hipSuccess;
hipError_t ret(hipError_t e) {
  if (e != hipSuccess) last_error = e;
  return e;
}

// ---- kernels registered by the modules ------------------------------------
struct KernelInfo {
  std::string name;       // demangled
  std::vector<size_t> arg_sizes;
};
// (function-local: the modules register their kernels from static constructors)
std::mutex &kmu() {
  static std::mutex m;
  return m;
}
std::map<const void *, KernelInfo> &kernels() {
  static std::map<const void *, KernelInfo> k;
  return k;
}

size_t type_size(std::string t) {
  while (!t.empty() && t.front() == ' ') t.erase(t.begin());
  while (!t.empty() && t.back() == ' ') t.pop_back();
  if (t.find('*') != std::string::npos) return sizeof(void *);
  if (t.find("LaunchArgs") != std::string::npos) return sizeof(cx::LaunchArgs);
  if (t.find("PolicyArgs") != std::string::npos) return sizeof(cx::PolicyArgs);
  if (t == "long" || t == "unsigned long" || t == "double" || t == "long long" || t == "unsigned long long") return 8;
  if (t == "int" || t == "unsigned int" || t == "float") return 4;
  die("kernel argument of unknown type '%s'", t.c_str());
}

KernelInfo describe(const char *mangled) {
  int st = 0;
  char *d = abi::__cxa_demangle(mangled, nullptr, nullptr, &st);
  if (st != 0 || !d) die("cannot demangle kernel %s", mangled);
  KernelInfo k;
  k.name = d;
  std::free(d);
  // the parameter list is the last top-level parenthesised group
  const size_t close = k.name.rfind(')');
  int depth = 0;
  size_t open = std::string::npos;
  for (size_t i = close; i-- > 0;) {
    if (k.name[i] == ')') ++depth;
    if (k.name[i] == '(') {
      if (depth == 0) {
        open = i;
        break;
      }
      --depth;
    }
  }
  if (open == std::string::npos) die("cannot parse kernel signature %s", k.name.c_str());
  std::string params = k.name.substr(open + 1, close - open - 1);
  depth = 0;
  std::string cur;
  for (char ch : params) {
    if (ch == '<' || ch == '(') ++depth;
    if (ch == '>' || ch == ')') --depth;
    if (ch == ',' && depth == 0) {
      k.arg_sizes.push_back(type_size(cur));
      cur.clear();
    } else {
      cur += ch;
    }
  }
  if (!cur.empty()) k.arg_sizes.push_back(type_size(cur));
  return k;
}

const KernelInfo &kernel(const void *f) {
  std::lock_guard<std::mutex> lk(kmu());
  auto it = kernels().find(f);
  if (it == kernels().end()) die("launch of an unregistered kernel %p", f);
  return it->second;
}

std::vector<std::vector<char>> copy_args(const KernelInfo &k, void **args) {
  std::vector<std::vector<char>> out;
  for (size_t i = 0; i < k.arg_sizes.size(); ++i) {
    const char *p = static_cast<const char *>(args[i]);
    out.emplace_back(p, p + k.arg_sizes[i]);
  }
  return out;
}

// ---- what each kernel accesses ---------------------------------------------
struct Launch {
  const void *func;
  dim3 grid, block;
  size_t lds;
  std::vector<std::vector<char>> args;
};

template <class T>
T arg(const Launch &l, size_t i) {
  T v;
  std::memcpy(&v, l.args.at(i).data(), sizeof v);
  return v;
}

// template arguments <L, P, SIMPLE, EXT, STAGE[, POL]> of a k_rollout instance
void rollout_params(const std::string &n, int *L, int *P, bool *simple, bool *ext, bool *stage, bool *pol) {
  const size_t a = n.find('<');
  int l = 0, p = 0;
  char s1[8] = {0}, s2[8] = {0}, s3[8] = {0}, s4[8] = {0};
  if (n.find("k_rollout_simple<") != std::string::npos) {  // SIMPLE classes: <L, P, STAGE>
    if (a == std::string::npos || std::sscanf(n.c_str() + a, "<%d, %d, %5[a-z]>", &l, &p, s3) != 3)
      die("cannot parse %s", n.c_str());
    *L = l;
    *P = p;
    *simple = true;
    *ext = *pol = false;
    *stage = std::strcmp(s3, "true") == 0;
    return;
  }
  if (n.find("k_rollout_policy<") != std::string::npos) {  // the fused policy rollout: <L, P>
    if (a == std::string::npos || std::sscanf(n.c_str() + a, "<%d, %d>", &l, &p) != 2) die("cannot parse %s", n.c_str());
    *L = l;
    *P = p;
    *simple = *stage = *pol = true;
    *ext = false;
    return;
  }
  const int got = a == std::string::npos ? 0
                                         : std::sscanf(n.c_str() + a, "<%d, %d, %5[a-z], %5[a-z], %5[a-z], %5[a-z]>",
                                                       &l, &p, s1, s2, s3, s4);
  if (got < 5) die("cannot parse %s", n.c_str());
  *L = l;
  *P = p;
  *simple = std::strcmp(s1, "true") == 0;
  *ext = std::strcmp(s2, "true") == 0;
  *stage = std::strcmp(s3, "true") == 0;
  *pol = got == 6 && std::strcmp(s4, "true") == 0;
}

void check_class(const cx::ClassDev *cls, const std::string &w) {
  need(cls, sizeof(cx::ClassDev), "class block", w);
  const cx::ClassDev &C = *cls;
  need(C.slot_port, 4 * (size_t)C.S, "slot_port", w);
  need(C.slot_cap, 4 * (size_t)C.S * C.D, "slot_cap", w);
  need(C.tpois, 4 * (size_t)C.steps_ep * cx::kPoisStride, "arrival thresholds", w);
  need(C.tdwell, (size_t)4 << C.dwell_log2, "stay thresholds", w);
  need(C.glob, 16 * (size_t)C.steps_ep, "per-step globals", w);
  if (C.n_days > 0) need(C.price_days, 4 * (size_t)C.n_days * C.steps_ep, "price days", w);
}

void run_rollout(const Launch &l, const KernelInfo &k) {
  int L, P;
  bool simple, ext, stage, pol;
  rollout_params(k.name, &L, &P, &simple, &ext, &stage, &pol);
  const cx::LaunchArgs a = arg<cx::LaunchArgs>(l, 0);
  const std::string w0 = k.name;
  if (l.block.x % 64 != 0 || l.block.x == 0 || l.block.x > 512 || l.block.y != 1 || l.grid.y != 1)
    die("%s: launch shape %u x %u", w0.c_str(), l.grid.x, l.block.x);
  if (pol) {
    // the fused policy rollout: 4 waves of 8-lane stations, the stage, the
    // hidden units, the BF16 observations and the levels inside the LDS
    const cx::LaunchArgs::Pol &q = a.pol;
    if (L != 8 || !simple || ext || !stage || (int)l.block.x != 64 * cx::kPolRolloutWaves)
      die("%s: fused policy launch of %u threads", w0.c_str(), l.block.x);
    if (a.mode != CX_ACT_POLICY || a.per_segment) die("%s: mode %d", w0.c_str(), a.mode);
    if (q.K1 < 1 || q.K1 > 8 || q.HP < 1 || q.HP > 8 || q.R < 1 || q.R > 3 || q.G < 1 || q.L1 < 2 || q.L1 > 4 * q.R)
      die("%s: MLP sizes K1 %d HP %d R %d G %d L1 %d", w0.c_str(), q.K1, q.HP, q.R, q.G, q.L1);
    if (q.in_dim > 32 * q.K1) die("%s: in_dim %d > 32 K1", w0.c_str(), q.in_dim);
    const size_t stage_end = (size_t)a.stage_off + 4 * (size_t)a.stage_floats;
    const size_t hb_end = (size_t)q.hb_off + (size_t)8 * (cx::kPolRolloutEnvs / 16) * 64 * 16;
    const size_t xb_end = (size_t)q.xb_off + (size_t)cx::kPolRolloutEnvs * 16 * cx::kPolXbRow;
    if (a.stage_floats < cx::kPolRolloutEnvs * q.in_dim) die("%s: stage of %d floats", w0.c_str(), a.stage_floats);
    if (q.hb_off < a.stage_off || std::max(stage_end, hb_end) > (size_t)q.xb_off || xb_end > (size_t)q.act_off)
      die("%s: LDS regions overlap (stage %d+%zu, hb %d, xb %d, act %d)", w0.c_str(), a.stage_off,
          stage_end - a.stage_off, q.hb_off, q.xb_off, q.act_off);
    if ((q.xb_off | q.hb_off | a.stage_off) & 15) die("%s: LDS regions not 16-byte aligned", w0.c_str());
    // padded fragments: 16 hidden tiles x 8 K-steps; G x 3 level tiles x 8 K-steps
    need(q.w1f, 16 * (size_t)16 * 8 * 64, "W1 fragments", w0);
    need(q.b1, 4 * (size_t)256, "b1", w0);
    need(q.w2f, 16 * (size_t)q.G * 3 * 8 * 64, "W2 fragments", w0);
    need(q.b2f, 4 * 16 * (size_t)q.G * 3, "b2", w0);
  }
  if (a.n_segs < 1) die("%s: no segments", w0.c_str());
  need(a.segs, sizeof(cx::SegDev) * (size_t)a.n_segs, "segment table", w0);
  std::vector<cx::SegDev> segs(a.n_segs);
  std::memcpy(segs.data(), a.segs, sizeof(cx::SegDev) * segs.size());  // as the kernel reads it, now
  const int W = (int)l.block.x / 64, SPW = 64 / L;
  const size_t table_lds = a.lds_tdwell ? 0 : 0;
  (void)table_lds;
  for (unsigned b = 0; b < l.grid.x; ++b) {
    int lo = 0, hi = a.n_segs - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (segs[mid].block_begin <= (int)b) lo = mid;
      else hi = mid - 1;
    }
    const cx::SegDev &sg = segs[lo];
    char wb[512];
    std::snprintf(wb, sizeof wb, "%s block %u (segment %d)", w0.c_str(), b, lo);
    const std::string w = wb;
    if (sg.block_begin > (int)b) die("%s: no segment starts at or before the block", w.c_str());
    check_class(sg.cls, w);
    const cx::ClassDev &C = *sg.cls;
    if (a.lds_tdwell && l.lds < ((size_t)4 << C.dwell_log2)) die("%s: LDS %zu < stay table", w.c_str(), l.lds);
    if (C.S != L * P) die("%s: class has %d slots, kernel packs %d x %d", w.c_str(), C.S, L, P);
    if (sg.pack != cx::pack_id(L, P)) die("%s: segment packing %d, kernel %d", w.c_str(), sg.pack, cx::pack_id(L, P));
    const bool kind_ext = C.kind == cx::kKindExt;
    if (kind_ext != ext) die("%s: class kind %d in a kernel with EXT = %d", w.c_str(), C.kind, (int)ext);
    if (simple && C.simple != 1) die("%s: non-SIMPLE class in a SIMPLE kernel", w.c_str());
    const int g_blk0 = ((int)b - sg.block_begin) * W;
    if (g_blk0 >= sg.n_groups) {
      if (pol) die("%s: idle block in a fused policy launch", w.c_str());
      continue;  // idle block
    }
    const int n_run = std::min(W, sg.n_groups - g_blk0);
    const int64_t e0 = (int64_t)g_blk0 * SPW;
    const int64_t e1 = std::min<int64_t>(sg.n_envs, (int64_t)(g_blk0 + n_run) * SPW);
    if (e0 >= e1) die("%s: block runs no env", w.c_str());
    const int64_t n = e1 - e0, S = C.S;
    need(sg.q + e0 * S, 8 * n * S, "q", w);
    need(sg.u + e0 * S, 4 * n * S, "u", w);
    need(sg.cap + e0 * S, 4 * n * S, "capacity", w);
    need(sg.p_last + e0 * S, 4 * n * S, "last power", w);
    need(sg.dwell + e0 * S, 2 * n * S, "dwell", w);
    need(sg.ret + e0, 8 * n, "return", w);
    if (ext && C.has_batt) {
      need(sg.bsoc + e0, 8 * n, "battery SoC", w);
      need(sg.bp + e0, 4 * n, "battery power", w);
    }
    if (ext && C.has_users) need(sg.utype + e0 * S, (size_t)(n * S), "user types", w);
    if (ext && C.n_models > 0) need(sg.rbar + e0 * S, 4 * n * S, "car rates", w);
    if (pol) {
      if (C.n_ports != S || C.S != 8 * P) die("%s: fused policy class of %d ports in %d slots", w.c_str(), C.n_ports, C.S);
      if ((size_t)cx::kPolRolloutEnvs * S > (size_t)l.lds - (size_t)a.pol.act_off)
        die("%s: LDS %zu too small for the levels", w.c_str(), l.lds);
      if (a.pol.in_dim != C.obs_dim) die("%s: MLP input %d, observation %d", w.c_str(), a.pol.in_dim, C.obs_dim);
      if (4 * a.pol.G < C.n_ports) die("%s: %d port groups for %d ports", w.c_str(), a.pol.G, C.n_ports);
      need(a.pol.obs0 + sg.obs_off + e0 * C.obs_dim, 4 * (size_t)(n * C.obs_dim), "start observations", w);
    }
    // records
    int32_t T = a.T, mode = a.mode, out_mode = a.out_mode;
    float *obs = a.obs;
    uint8_t *act = a.act;
    float *rew = a.reward;
    uint8_t *done = a.done;
    const uint8_t *act_in = a.act_in;
    int64_t os = a.obs_stride, as = a.act_stride, es = a.env_stride;
    if (a.per_segment) {
      T = sg.T; mode = sg.mode; out_mode = sg.out_mode; obs = sg.obs; act = sg.act; rew = sg.reward;
      done = sg.done; act_in = sg.act_in; os = sg.obs_stride; as = sg.act_stride; es = sg.env_stride;
    }
    if (T < 1) die("%s: T = %d", w.c_str(), T);
    const bool w_obs = out_mode == CX_OUT_FULL && obs;
    const bool w_act = (out_mode == CX_OUT_FULL || out_mode == CX_OUT_ACT_REWARD) && act;
    const int od = C.obs_dim, na = C.n_act;
    if ((uint64_t)sg.n_envs * (uint64_t)od * 4 >= (1ull << 32)) die("%s: 32-bit observation offsets overflow", w.c_str());
    for (int t : {0, T - 1}) {
      if (w_obs) {
        float *base = obs + sg.obs_off + (int64_t)t * os;
        if (stage) {
          const int pad = (int)((reinterpret_cast<uintptr_t>(base + e0 * od) >> 2) & 3u);
          if (pol && pad != 0) die("%s: fused policy observations not 16-byte aligned", w.c_str());
          const int nf = (int)(n * od);
          const size_t need_lds = (size_t)a.stage_off + (pol ? 4 : 8) * (size_t)a.stage_floats;
          if (a.stage_floats < pad + nf) die("%s: stage of %d floats for %d", w.c_str(), a.stage_floats, pad + nf);
          if (l.lds < need_lds) die("%s: LDS %zu < %zu with the stages", w.c_str(), l.lds, need_lds);
          if (a.stage_off < ((int32_t)4 << C.dwell_log2)) die("%s: stage overlaps the stay table", w.c_str());
          // 16-byte chunks from the aligned address below the run's first float
          const int c_end = (pad + nf) >> 2;
          char *chunk0 = reinterpret_cast<char *>(base + e0 * od) - 4 * pad;
          const int c_begin = pad ? 1 : 0;
          if (c_end > c_begin) need(chunk0 + 16 * c_begin, 16 * (size_t)(c_end - c_begin), "staged observation chunks", w);
        }
        need(base + e0 * od, 4 * (size_t)(n * od), "observations", w);
      }
      if (w_act) need(act + sg.act_off + (int64_t)t * as + e0 * na, (size_t)(n * na), "action records", w);
      if (mode == CX_ACT_EXTERNAL) need(act_in + sg.act_off + (int64_t)t * as + e0 * na, (size_t)(n * na), "action input", w);
      if (rew) need(rew + sg.env_off + (int64_t)t * es + e0, 4 * (size_t)n, "rewards", w);
      if (done) need(done + sg.env_off + (int64_t)t * es + e0, (size_t)n, "done flags", w);
    }
  }
}

void run_policy(const Launch &l) {
  const cx::PolicyArgs a = arg<cx::PolicyArgs>(l, 0);
  const std::string w = "k_policy";
  if (a.n <= 0) die("k_policy: n = %lld", (long long)a.n);
  need(a.obs, 4 * (size_t)(a.n * a.in_dim), "observations", w);
  need(a.w1f, 16 * (size_t)(2 * a.HP) * a.K1 * 64, "W1 fragments", w);
  need(a.b1, 4 * 32 * (size_t)a.HP, "b1", w);
  need(a.w2f, 16 * (size_t)a.G * a.R * a.HP * 64, "W2 fragments", w);
  need(a.b2f, 4 * 16 * (size_t)a.G * a.R, "b2", w);
  if (a.act) need(a.act, (size_t)(a.n * a.N), "levels", w);
  if (a.logits) need(a.logits, 4 * (size_t)(a.n * a.N * a.L1), "logits", w);
  const int64_t waves = (a.n + 31) / 32;
  if ((int64_t)l.grid.x * 8 < waves) die("k_policy: %u blocks for %lld waves", l.grid.x, (long long)waves);
}

void run_kernel(const Launch &l) {
  const KernelInfo &k = kernel(l.func);
  if (k.name.find("k_rollout<") != std::string::npos || k.name.find("k_rollout_policy<") != std::string::npos ||
      k.name.find("k_rollout_simple<") != std::string::npos) {
    run_rollout(l, k);
  } else if (k.name.find("k_policy(") != std::string::npos) {
    run_policy(l);
  } else if (k.name.find("k_reset_obs(") != std::string::npos) {
    const auto *cls = arg<const cx::ClassDev *>(l, 0);
    check_class(cls, k.name);
    need(arg<float *>(l, 2), 4 * (size_t)(arg<int64_t>(l, 1) * cls->obs_dim), "reset observations", k.name);
  } else if (k.name.find("k_fill_f64(") != std::string::npos) {
    need(arg<double *>(l, 0), 8 * (size_t)arg<int64_t>(l, 1), "filled doubles", k.name);
  } else if (k.name.find("k_observe(") != std::string::npos) {
    const auto *cls = arg<const cx::ClassDev *>(l, 0);
    check_class(cls, k.name);
    const int64_t n = arg<int64_t>(l, 1), S = cls->S;
    need(arg<double *>(l, 2), 8 * (size_t)(n * S), "q", k.name);
    need(arg<float *>(l, 3), 4 * (size_t)(n * S), "u", k.name);
    need(arg<float *>(l, 4), 4 * (size_t)(n * S), "last power", k.name);
    need(arg<int16_t *>(l, 5), 2 * (size_t)(n * S), "dwell", k.name);
    need(arg<float *>(l, 14), 4 * (size_t)(n * cls->obs_dim), "observations", k.name);
  } else {
    die("no access model for kernel %s", k.name.c_str());
  }
  std::lock_guard<std::mutex> lk(dev().mu);
  dev().clock_ms += 1e-3 * (double)l.grid.x * l.block.x / 64.0;  // device time of the launch
}

// ---- graphs ----------------------------------------------------------------
struct Node {
  Launch l;
};
struct Graph {
  std::vector<std::unique_ptr<Node>> nodes;
};
struct Exec {
  std::vector<Node *> orig;       // the graph's nodes, for hipGraphExecKernelNodeSetParams
  std::vector<Launch> launches;   // this exec's own copies
  std::shared_ptr<std::atomic<int>> in_flight = std::make_shared<std::atomic<int>>(0);
};

struct Event {
  std::shared_ptr<std::atomic<uint64_t>> seq = std::make_shared<std::atomic<uint64_t>>(0);
  std::shared_ptr<std::atomic<double>> t_ms = std::make_shared<std::atomic<double>>(0);
  std::shared_ptr<std::atomic<bool>> done = std::make_shared<std::atomic<bool>>(false);
};

struct Stream {
  int id;
};

Launch make_launch(const void *func, dim3 g, dim3 b, void **args, size_t lds) {
  const KernelInfo &k = kernel(func);
  return Launch{func, g, b, lds, copy_args(k, args)};
}

}  // namespace fake

using namespace fake;

extern "C" {
void **__hipRegisterFatBinary(const void *) {
  static void *handle = nullptr;
  return &handle;
}
void __hipUnregisterFatBinary(void **) {}
// A __device__ variable: its device copy is host memory of the variable's size,
// made (and entered as a live allocation for the range checks) when its
// address is first asked for; module constructors only record the size.
void __hipRegisterVar(void **, void *var, char *, char *, int, size_t size, int, int) {
  symbols()[var] = Symbol{size, nullptr};
}
void __hipRegisterFunction(void **, const void *hostFunction, char *deviceFunction, const char *, unsigned int,
                           uint3 *, uint3 *, dim3 *, dim3 *, int *) {
  KernelInfo k = describe(deviceFunction);
  std::lock_guard<std::mutex> lk(kmu());
  kernels()[hostFunction] = k;
}
}

namespace {
thread_local dim3 cfg_grid, cfg_block;
thread_local size_t cfg_lds;
thread_local hipStream_t cfg_stream;
}  // namespace

hipError_t __hipPushCallConfiguration(dim3 g, dim3 b, size_t lds, hipStream_t s) {
  cfg_grid = g; cfg_block = b; cfg_lds = lds; cfg_stream = s;
  return hipSuccess;
}
hipError_t __hipPopCallConfiguration(dim3 *g, dim3 *b, size_t *lds, hipStream_t *s) {
  *g = cfg_grid; *b = cfg_block; *lds = cfg_lds; *s = cfg_stream;
  return hipSuccess;
}

hipError_t hipLaunchKernel(const void *f, dim3 g, dim3 b, void **args, size_t lds, hipStream_t) {
  if (g.x == 0 || b.x == 0) return ret(hipErrorInvalidConfiguration);
  if (lds > (160u << 10)) return ret(hipErrorInvalidValue);
  Launch l = make_launch(f, g, b, args, lds);
  dev().push([l] { run_kernel(l); });
  return hipSuccess;
}

hipError_t hipGetSymbolAddress(void **p, const void *symbol) {
  std::lock_guard<std::mutex> lk(amu);
  auto it = symbols().find(symbol);
  if (!p || it == symbols().end()) return ret(hipErrorInvalidSymbol);
  Symbol &v = it->second;
  if (!v.dev) {
    v.dev = std::aligned_alloc(256, std::max<size_t>(256, (v.size + 255) & ~(size_t)255));
    allocs[reinterpret_cast<uintptr_t>(v.dev)] = Alloc{v.size, false, true};
  }
  *p = v.dev;
  return hipSuccess;
}

hipError_t hipGetLastError() {
  hipError_t e = last_error;
  last_error = hipSuccess;
  return e;
}
hipError_t hipPeekAtLastError() { return last_error; }
const char *hipGetErrorString(hipError_t e) { return e == hipSuccess ? "no error" : "fake HIP error"; }
hipError_t hipGetDevice(int *d) {
  *d = 0;
  return hipSuccess;
}
hipError_t hipSetDevice(int d) { return d == 0 ? hipSuccess : ret(hipErrorInvalidDevice); }
hipError_t hipDeviceSynchronize() {
  dev().sync();
  return hipSuccess;
}

hipError_t hipMalloc(void **p, size_t n) {
  if (!p) return ret(hipErrorInvalidValue);
  void *m = std::aligned_alloc(256, std::max<size_t>(256, (n + 255) & ~(size_t)255));
  if (!m) return ret(hipErrorOutOfMemory);
  {
    std::lock_guard<std::mutex> lk(amu);
    allocs[reinterpret_cast<uintptr_t>(m)] = Alloc{n, false};
  }
  *p = m;
  return hipSuccess;
}
hipError_t hipFree(void *p) {
  if (!p) return hipSuccess;
  dev().sync();  // hipFree waits for the device
  {
    std::lock_guard<std::mutex> lk(amu);
    auto it = allocs.find(reinterpret_cast<uintptr_t>(p));
    if (it == allocs.end() || it->second.pinned) die("hipFree of %p: not a live device allocation", p);
    allocs.erase(it);
  }
  std::free(p);
  return hipSuccess;
}
hipError_t hipHostMalloc(void **p, size_t n, unsigned int) {
  void *m = std::aligned_alloc(256, std::max<size_t>(256, (n + 255) & ~(size_t)255));
  if (!m) return ret(hipErrorOutOfMemory);
  {
    std::lock_guard<std::mutex> lk(amu);
    allocs[reinterpret_cast<uintptr_t>(m)] = Alloc{n, true};
  }
  *p = m;
  return hipSuccess;
}
hipError_t hipHostFree(void *p) {
  if (!p) return hipSuccess;
  dev().sync();
  {
    std::lock_guard<std::mutex> lk(amu);
    auto it = allocs.find(reinterpret_cast<uintptr_t>(p));
    if (it == allocs.end() || !it->second.pinned) die("hipHostFree of %p: not pinned host memory", p);
    allocs.erase(it);
  }
  std::free(p);
  return hipSuccess;
}

namespace {
// A copy as the device performs it: device ranges must be live; pageable host
// sources of asynchronous copies are staged at the call, as the runtime does.
hipError_t enqueue_copy(void *dst, const void *src, size_t n, hipMemcpyKind k, bool sync) {
  if (n == 0) return hipSuccess;
  const bool d_dst = k == hipMemcpyHostToDevice || k == hipMemcpyDeviceToDevice;
  const bool d_src = k == hipMemcpyDeviceToHost || k == hipMemcpyDeviceToDevice;
  if (d_dst) need(dst, n, "copy destination", "hipMemcpy");
  if (d_src) need(src, n, "copy source", "hipMemcpy");
  bool pinned = false;
  const bool staged = !d_src && !sync && !(in_alloc(src, n, &pinned) && pinned);
  std::shared_ptr<std::vector<char>> stage;
  if (staged) stage = std::make_shared<std::vector<char>>(static_cast<const char *>(src), static_cast<const char *>(src) + n);
  const uint64_t s = dev().push([=] {
    if (d_dst) need(dst, n, "copy destination", "hipMemcpy (executed)");
    if (d_src) need(src, n, "copy source", "hipMemcpy (executed)");
    std::memcpy(dst, stage ? stage->data() : src, n);
  });
  if (sync) dev().wait_for(s);
  return hipSuccess;
}
}  // namespace

hipError_t hipMemcpy(void *dst, const void *src, size_t n, hipMemcpyKind k) { return enqueue_copy(dst, src, n, k, true); }
hipError_t hipMemcpyAsync(void *dst, const void *src, size_t n, hipMemcpyKind k, hipStream_t) {
  return enqueue_copy(dst, src, n, k, false);
}
hipError_t hipMemset(void *p, int v, size_t n) {
  need(p, n, "memset destination", "hipMemset");
  const uint64_t s = dev().push([=] { std::memset(p, v, n); });
  dev().wait_for(s);
  return hipSuccess;
}
hipError_t hipMemsetAsync(void *p, int v, size_t n, hipStream_t) {
  need(p, n, "memset destination", "hipMemsetAsync");
  dev().push([=] {
    need(p, n, "memset destination", "hipMemsetAsync (executed)");
    std::memset(p, v, n);
  });
  return hipSuccess;
}

hipError_t hipStreamCreateWithFlags(hipStream_t *s, unsigned int) {
  static std::atomic<int> ids{1};
  *s = reinterpret_cast<hipStream_t>(new Stream{ids++});
  return hipSuccess;
}
hipError_t hipStreamDestroy(hipStream_t s) {
  if (!s) return ret(hipErrorInvalidHandle);
  dev().sync();
  delete reinterpret_cast<Stream *>(s);
  return hipSuccess;
}
hipError_t hipStreamSynchronize(hipStream_t) {
  dev().sync();  // one in-order queue: waiting for everything covers the stream
  return hipSuccess;
}
hipError_t hipStreamWaitEvent(hipStream_t, hipEvent_t, unsigned int) { return hipSuccess; }  // in-order queue

hipError_t hipEventCreateWithFlags(hipEvent_t *e, unsigned int) {
  *e = reinterpret_cast<hipEvent_t>(new Event());
  return hipSuccess;
}
hipError_t hipEventCreate(hipEvent_t *e) { return hipEventCreateWithFlags(e, 0); }
hipError_t hipEventDestroy(hipEvent_t e) {
  if (!e) return ret(hipErrorInvalidHandle);
  delete reinterpret_cast<Event *>(e);  // a pending record keeps its shared state alive
  return hipSuccess;
}
hipError_t hipEventRecord(hipEvent_t e, hipStream_t) {
  if (!e) return ret(hipErrorInvalidHandle);
  Event *ev = reinterpret_cast<Event *>(e);
  ev->done->store(false);
  auto done = ev->done;
  auto t = ev->t_ms;
  const uint64_t s = dev().push([done, t] {
    {
      std::lock_guard<std::mutex> lk(dev().mu);
      t->store(dev().clock_ms);
    }
    done->store(true);
  });
  ev->seq->store(s);
  return hipSuccess;
}
hipError_t hipEventSynchronize(hipEvent_t e) {
  if (!e) return ret(hipErrorInvalidHandle);
  Event *ev = reinterpret_cast<Event *>(e);
  const uint64_t s = ev->seq->load();
  if (s) dev().wait_for(s);
  return hipSuccess;
}
hipError_t hipEventQuery(hipEvent_t e) {
  if (!e) return ret(hipErrorInvalidHandle);
  Event *ev = reinterpret_cast<Event *>(e);
  if (ev->seq->load() == 0) return hipSuccess;
  return ev->done->load() ? hipSuccess : hipErrorNotReady;
}
hipError_t hipEventElapsedTime(float *ms, hipEvent_t a, hipEvent_t b) {
  Event *ea = reinterpret_cast<Event *>(a), *eb = reinterpret_cast<Event *>(b);
  if (!ea || !eb || !ea->done->load() || !eb->done->load()) return ret(hipErrorNotReady);
  *ms = (float)(eb->t_ms->load() - ea->t_ms->load());
  return hipSuccess;
}

hipError_t hipGraphCreate(hipGraph_t *g, unsigned int) {
  *g = reinterpret_cast<hipGraph_t>(new Graph());
  return hipSuccess;
}
hipError_t hipGraphDestroy(hipGraph_t g) {
  delete reinterpret_cast<Graph *>(g);
  return hipSuccess;
}
hipError_t hipGraphAddKernelNode(hipGraphNode_t *node, hipGraph_t g, const hipGraphNode_t *, size_t,
                                 const hipKernelNodeParams *p) {
  Graph *G = reinterpret_cast<Graph *>(g);
  if (!G || !p || !p->kernelParams) return ret(hipErrorInvalidValue);
  if (p->extra) die("hipGraphAddKernelNode: 'extra' arguments are not modelled");
  auto n = std::make_unique<Node>();
  n->l = make_launch(p->func, p->gridDim, p->blockDim, p->kernelParams, p->sharedMemBytes);
  *node = reinterpret_cast<hipGraphNode_t>(n.get());
  G->nodes.push_back(std::move(n));
  return hipSuccess;
}
hipError_t hipGraphInstantiate(hipGraphExec_t *ex, hipGraph_t g, hipGraphNode_t *, char *, size_t) {
  Graph *G = reinterpret_cast<Graph *>(g);
  Exec *E = new Exec();
  for (auto &n : G->nodes) {
    E->orig.push_back(n.get());
    E->launches.push_back(n->l);
  }
  *ex = reinterpret_cast<hipGraphExec_t>(E);
  return hipSuccess;
}
hipError_t hipGraphExecKernelNodeSetParams(hipGraphExec_t ex, hipGraphNode_t node, const hipKernelNodeParams *p) {
  Exec *E = reinterpret_cast<Exec *>(ex);
  const auto it = std::find(E->orig.begin(), E->orig.end(), reinterpret_cast<Node *>(node));
  if (it == E->orig.end()) die("hipGraphExecKernelNodeSetParams: the node is not in the graph of this exec");
  Launch &l = E->launches[it - E->orig.begin()];
  if (p->func != l.func) die("hipGraphExecKernelNodeSetParams: the kernel of a node changed");
  l = make_launch(p->func, p->gridDim, p->blockDim, p->kernelParams, p->sharedMemBytes);
  return hipSuccess;
}
hipError_t hipGraphLaunch(hipGraphExec_t ex, hipStream_t) {
  Exec *E = reinterpret_cast<Exec *>(ex);
  if (!E) return ret(hipErrorInvalidHandle);
  for (const Launch &l : E->launches) {
    auto inflight = E->in_flight;
    inflight->fetch_add(1);
    dev().push([l, inflight] {
      run_kernel(l);
      inflight->fetch_sub(1);
    });
  }
  return hipSuccess;
}
hipError_t hipGraphExecDestroy(hipGraphExec_t ex) {
  Exec *E = reinterpret_cast<Exec *>(ex);
  if (E->in_flight->load() != 0) n_graph_destroy_in_flight.fetch_add(1);
  delete E;
  return hipSuccess;
}

extern "C" long fake_hip_graph_destroys_in_flight() { return n_graph_destroy_in_flight.load(); }
extern "C" long fake_hip_live_allocations() {
  std::lock_guard<std::mutex> lk(amu);
  long n = 0;
  for (const auto &a : allocs) n += a.second.symbol ? 0 : 1;
  return n;
}
