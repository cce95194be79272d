// Batched solve of problems with uneven horizons and several sizes (the lqt_ragged entry points
// of lqt.h): validation, workspace planning, the eager solve, and plans (a fixed configuration
// chosen by a small autotuner, replayed with one branch per class on its own stream).
//
// Each class runs the solve over its concatenated horizon in ragged mode (KProb::seg): the element
// build inserts a separator element after every problem, the control and value kernels look up
// the owning problem of a boundary.  After the element build, both scans of a class run in one
// launch whose waves take their tiles (per-lane path) or tree nodes (wave path) from a work queue
// in dependency order, so a plan is four launches per class (constants, elements, clearing of the
// queue's status words, the queue launch), whatever the number of problems.
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/lqt.h"
#include "lqt_internal.hpp"

namespace lqt {
namespace {

constexpr int kMinWaveChunk = 4;  // workspace is laid out for the smallest candidate chunk
const int kWaveChunks[] = {4, 8, 16};

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }
size_t dsize(int dtype) { return dtype == LQT_F64 ? 8 : 4; }

lqt_dims class_dims(const lqt_ragged& c) {
  lqt_dims d;
  memset(&d, 0, sizeof(d));  // lti = 0: the batched solve uses the general build
  d.nx = c.nx;
  d.nu = c.nu;
  d.T = (int32_t)c.rows;
  d.n_steps = c.n_steps;
  d.batch = 1;
  d.dtype = c.dtype;
  d.F_sampled = c.F_sampled;
  d.L_sampled = c.L_sampled;
  d.has_c = c.has_c;
  return d;
}

bool is_wave(const lqt_dims& d) { return lane_ops(d.nx, d.nu, d.dtype) == nullptr; }

lqt_status bad(const char* fmt, int i, const char* what) {
  char buf[256];
  snprintf(buf, sizeof(buf), fmt, i, what);
  return set_error(LQT_EINVAL, buf);
}

lqt_status check_class(const lqt_ragged& c, int i) {
  if (c.dtype != LQT_F64 && c.dtype != LQT_F32) return bad("class %d: %s", i, "invalid dtype");
  if (c.nx < 1 || c.nx > 16) return bad("class %d: %s", i, "nx outside [1, 16]");
  if (c.nu < 1 || c.nu > c.nx) return bad("class %d: %s", i, "nu outside [1, nx]");
  if (c.n_steps < 1 || c.n_steps > 4096) return bad("class %d: %s", i, "n_steps outside [1, 4096]");
  if (c.count < 1) return bad("class %d: %s", i, "count < 1");
  if (c.rows < 2L * c.count) return bad("class %d: %s", i, "rows < 2 count (every T_i >= 1)");
  if (c.rows > 0x7fffffffL) return bad("class %d: %s", i, "rows above 2^31 - 1");
  const size_t es = dsize(c.dtype);
  struct {
    const void* p;
    const char* n;
    size_t a;
  } ptrs[] = {{c.start, "start", 8},  {c.prob.t, "t", es},   {c.prob.F, "F", es},
              {c.prob.L, "L", es},    {c.prob.Q, "Q", es},   {c.prob.R, "R", es},
              {c.prob.r, "r", es},    {c.prob.Qf, "Qf", es}, {c.prob.rf, "rf", es},
              {c.prob.x0, "x0", es},  {c.S, "S", es},        {c.v, "v", es},
              {c.x, "x", es}};
  for (const auto& q : ptrs) {
    if (!q.p) return bad("class %d: %s is NULL", i, q.n);
    if ((uintptr_t)q.p % q.a) return bad("class %d: %s is misaligned", i, q.n);
  }
  if (c.has_c && !c.prob.c) return bad("class %d: %s is NULL", i, "c");
  if (c.u && (uintptr_t)c.u % es) return bad("class %d: %s is misaligned", i, "u");
  return LQT_OK;
}

size_t class_bytes(const lqt_ragged& c) {
  const lqt_dims d = class_dims(c);
  return align256(layout(&d, LQT_CALL_SOLVE, nullptr, nullptr, kMinWaveChunk, c.count));
}

struct ClassRun {
  lqt_ragged c;
  lqt_dims d;
  KProb kp;
  Work w;
};

lqt_status prepare(const lqt_ragged* cls, int ncls, void* ws, size_t ws_bytes,
                   std::vector<ClassRun>& out) {
  if (!cls || ncls < 1) return set_error(LQT_EINVAL, "no classes");
  size_t need = 0;
  for (int i = 0; i < ncls; ++i) {
    lqt_status st = check_class(cls[i], i);
    if (st != LQT_OK) return st;
    need += class_bytes(cls[i]);
  }
  if (!ws) return set_error(LQT_EWORKSPACE, "workspace is NULL");
  if ((uintptr_t)ws % 256) return set_error(LQT_EWORKSPACE, "workspace is not 256-byte aligned");
  if (ws_bytes < need) return set_error(LQT_EWORKSPACE, "workspace too small");
  out.clear();
  char* base = (char*)ws;
  for (int i = 0; i < ncls; ++i) {
    ClassRun r;
    r.c = cls[i];
    r.d = class_dims(cls[i]);
    layout(&r.d, LQT_CALL_SOLVE, base, &r.w, kMinWaveChunk, cls[i].count);
    base += class_bytes(cls[i]);
    KProb& k = r.kp;
    k.nx = r.d.nx;
    k.nu = r.d.nu;
    k.T = r.d.T;
    k.n = r.d.n_steps;
    k.batch = 1;
    k.F_sampled = r.d.F_sampled;
    k.L_sampled = r.d.L_sampled;
    k.has_c = r.d.has_c;
    const lqt_problem& p = cls[i].prob;
    k.t = p.t;
    k.F = p.F;
    k.L = p.L;
    k.c = p.c;
    k.Q = p.Q;
    k.R = p.R;
    k.r = p.r;
    k.Qf = p.Qf;
    k.rf = p.rf;
    k.x0 = p.x0;
    k.consts = r.w.consts;
    k.seg = cls[i].start;
    k.nseg = cls[i].count;
    out.push_back(r);
  }
  return LQT_OK;
}

// Value chunks of the per-lane work-queue scans worth trying for a class of `rows` blocks (more
// blocks per lane only pay once there are enough tiles to fill the device).
std::vector<int> lane_chunks(long rows) {
  if (rows <= (1L << 11)) return {1, 4};
  if (rows < (1L << 19)) return {4, 8};
  return {8, 4};
}

// Every class runs its scans in one launch over a work queue (queue_chunk != 0).
SolveOpts default_opts(const ClassRun& r) {
  SolveOpts o;
  o.wave_chunk = 8;
  o.queue_chunk = is_wave(r.d) ? 1 : lane_chunks(r.c.rows)[0];
  return o;
}

lqt_status run_class(const ClassRun& r, const SolveOpts& o, hipStream_t s) {
  return run_solve(&r.d, r.kp, r.w, r.w.elts, r.c.S, r.c.v, r.c.x, r.c.u, o, s);
}

std::string signature(const std::vector<ClassRun>& cr) {
  std::string k;
  char buf[160];
  for (const auto& r : cr) {
    snprintf(buf, sizeof(buf), "%d,%d,%d,%d,%d,%d,%d,%d,%lld;", r.c.nx, r.c.nu, r.c.n_steps,
             r.c.dtype, r.c.F_sampled, r.c.L_sampled, r.c.has_c, r.c.count, (long long)r.c.rows);
    k += buf;
  }
  return k;
}

struct Choice {
  std::vector<SolveOpts> opts;
  bool parallel = true;
  std::string text;
};

std::mutex g_tune_mu;
std::map<std::string, Choice> g_tune_cache;

// LQT_AUTOTUNE: "off" never tunes (the default configuration, whatever the flags), "on" (the
// default) tunes plans created with LQT_PLAN_AUTOTUNE unless the cache holds their classes,
// "force" tunes every plan afresh.
enum class TuneMode { kOff, kOn, kForce };
TuneMode tune_mode() {
  const char* e = getenv("LQT_AUTOTUNE");
  if (!e) return TuneMode::kOn;
  if (!strcmp(e, "off") || !strcmp(e, "0")) return TuneMode::kOff;
  if (!strcmp(e, "force")) return TuneMode::kForce;
  return TuneMode::kOn;
}

// LQT_TUNE_CACHE=<file>: the cache persists there, one line per entry:
//   <gfx arch> <class signature> <parallel 0|1> <n> (<wave_chunk> <queue_chunk>) x n |<text>
// read when the first plan is created and rewritten after every tuning (under g_tune_mu).
bool g_cache_loaded = false;

std::string device_arch() {
  int dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess)
    return "unknown";
  std::string a = prop.gcnArchName;
  return a.substr(0, a.find(':'));  // without the target features
}

void cache_load_locked() {
  if (g_cache_loaded) return;
  g_cache_loaded = true;
  const char* path = getenv("LQT_TUNE_CACHE");
  if (!path) return;
  FILE* f = fopen(path, "r");
  if (!f) return;
  char line[4096];
  while (fgets(line, sizeof(line), f)) {
    char arch[64], sig[2048];
    int par = 0, n = 0, used = 0;
    if (sscanf(line, "%63s %2047s %d %d%n", arch, sig, &par, &n, &used) != 4 || n < 1 || n > 64)
      continue;
    Choice c;
    c.parallel = par != 0;
    const char* q = line + used;
    bool good = true;
    for (int i = 0; i < n && good; ++i) {
      SolveOpts o;
      int k = 0;
      good = sscanf(q, "%d %d%n", &o.wave_chunk, &o.queue_chunk, &k) == 2;
      q += k;
      c.opts.push_back(o);
    }
    const char* bar = strchr(q, '|');
    if (!good || !bar) continue;
    c.text = std::string(bar + 1);
    while (!c.text.empty() && (c.text.back() == '\n' || c.text.back() == '\r')) c.text.pop_back();
    g_tune_cache[std::string(arch) + " " + sig] = c;
  }
  fclose(f);
}

void cache_save_locked() {
  const char* path = getenv("LQT_TUNE_CACHE");
  if (!path) return;
  const std::string tmp = std::string(path) + ".tmp";
  FILE* f = fopen(tmp.c_str(), "w");
  if (!f) return;
  for (const auto& kv : g_tune_cache) {
    fprintf(f, "%s %d %zu", kv.first.c_str(), kv.second.parallel ? 1 : 0, kv.second.opts.size());
    for (const auto& o : kv.second.opts) fprintf(f, " %d %d", o.wave_chunk, o.queue_chunk);
    fprintf(f, " |%s\n", kv.second.text.c_str());
  }
  const bool ok = fclose(f) == 0;
  if (ok) rename(tmp.c_str(), path);
}

}  // namespace
}  // namespace lqt

struct lqt_plan_s {
  std::vector<lqt::ClassRun> cls;
  lqt::Choice choice;
  std::vector<hipStream_t> branch;
  hipEvent_t fork = nullptr;
  std::vector<hipEvent_t> join;
  // LQT_PLAN_GRAPH: the launch sequence captured once, on a stream of the plan's own, after
  // tuning; replayed with hipGraphLaunch.  `done` is recorded behind every replay so that the
  // executable graph is destroyed only once no replay of it is pending.
  hipStream_t cap = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipEvent_t done = nullptr;
  bool replayed = false;
};

namespace lqt {
namespace {

void release(lqt_plan_s* p) {
  if (p->exec) {
    if (p->replayed) hipEventSynchronize(p->done);
    hipGraphExecDestroy(p->exec);
    p->exec = nullptr;
  }
  if (p->graph) hipGraphDestroy(p->graph);
  p->graph = nullptr;
  if (p->done) hipEventDestroy(p->done);
  p->done = nullptr;
  if (p->cap) hipStreamDestroy(p->cap);
  p->cap = nullptr;
  for (auto e : p->join) hipEventDestroy(e);
  if (p->fork) hipEventDestroy(p->fork);
  for (auto s : p->branch) hipStreamDestroy(s);
  p->join.clear();
  p->fork = nullptr;
  p->branch.clear();
}

#define PLAN_HIP(x)                                                        \
  do {                                                                     \
    hipError_t _e = debug_gate(x);                                         \
    if (_e != hipSuccess) {                                                \
      char _b[256];                                                        \
      snprintf(_b, sizeof(_b), "%s failed: %s%s", #x, hipGetErrorString(_e), \
               debug_gate_note());                                         \
      return set_error(LQT_EHIP, _b);                                      \
    }                                                                      \
  } while (0)

#define PLAN_TRY(x)                      \
  do {                                   \
    lqt_status _s = (x);                 \
    if (_s != LQT_OK) return _s;         \
  } while (0)

// Enqueue the solve of every class on `s`: with `parallel`, each class on its own branch stream
// (forked from and joined back into `s` with events), else one after another on `s`.
lqt_status enqueue(lqt_plan_s* p, const std::vector<SolveOpts>& opts, bool parallel,
                   hipStream_t s) {
  if (!parallel || p->cls.size() < 2) {
    for (size_t i = 0; i < p->cls.size(); ++i) PLAN_TRY(run_class(p->cls[i], opts[i], s));
    return LQT_OK;
  }
  PLAN_HIP(hipEventRecord(p->fork, s));
  for (size_t i = 0; i < p->cls.size(); ++i) {
    PLAN_HIP(hipStreamWaitEvent(p->branch[i], p->fork, 0));
    PLAN_TRY(run_class(p->cls[i], opts[i], p->branch[i]));
    PLAN_HIP(hipEventRecord(p->join[i], p->branch[i]));
    PLAN_HIP(hipStreamWaitEvent(s, p->join[i], 0));
  }
  return LQT_OK;
}

// Milliseconds of fn() on stream s (one untimed run first).
template <class F>
lqt_status time_ms(hipStream_t s, F fn, float* ms) {
  hipEvent_t a, b;
  PLAN_HIP(hipEventCreate(&a));
  if (hipEventCreate(&b) != hipSuccess) {
    hipEventDestroy(a);
    return set_error(LQT_EHIP, "event creation failed");
  }
  lqt_status st = fn();
  hipError_t e = hipSuccess;
  if (st == LQT_OK) e = hipEventRecord(a, s);
  if (st == LQT_OK && e == hipSuccess) st = fn();
  if (st == LQT_OK && e == hipSuccess) e = hipEventRecord(b, s);
  if (st == LQT_OK && e == hipSuccess) e = hipEventSynchronize(b);
  if (st == LQT_OK && e == hipSuccess) e = hipEventElapsedTime(ms, a, b);
  if (st != LQT_OK) hipStreamSynchronize(s);
  hipEventDestroy(a);
  hipEventDestroy(b);
  if (st != LQT_OK) return st;
  if (e != hipSuccess) return set_error(LQT_EHIP, hipGetErrorString(e));
  return LQT_OK;
}

// The autotuner: per class, every candidate option timed alone; then concurrent vs serial
// branches with the chosen options.
lqt_status tune(lqt_plan_s* p, hipStream_t s, Choice* ch) {
  ch->opts.clear();
  std::string text;
  char buf[200];
  for (size_t i = 0; i < p->cls.size(); ++i) {
    const ClassRun& r = p->cls[i];
    std::vector<SolveOpts> cands;
    if (is_wave(r.d)) {
      for (int wc : kWaveChunks) {
        SolveOpts o;
        o.wave_chunk = wc;
        o.queue_chunk = 1;
        cands.push_back(o);
      }
    } else {
      for (int cv : lane_chunks(r.c.rows)) {
        SolveOpts o;
        o.queue_chunk = cv;
        cands.push_back(o);
      }
    }
    float best = 1e30f;
    SolveOpts bo = cands[0];
    for (const auto& o : cands) {
      float ms = 0.f;
      PLAN_TRY(time_ms(s, [&] { return run_class(r, o, s); }, &ms));
      if (ms < best) {
        best = ms;
        bo = o;
      }
    }
    ch->opts.push_back(bo);
    const std::string choice =
        is_wave(r.d) ? "wave path, both trees in one queue launch, " +
                           std::to_string(bo.wave_chunk) + " nodes per wave"
                     : "lane path, both scans in one queue launch, " +
                           std::to_string(bo.queue_chunk) + " blocks per lane (value scan)";
    snprintf(buf, sizeof(buf), "class %zu (nx=%d nu=%d count=%d rows=%lld): %s, %.3f ms; ", i,
             r.c.nx, r.c.nu, r.c.count, (long long)r.c.rows, choice.c_str(), best);
    text += buf;
  }
  ch->parallel = true;
  if (p->cls.size() > 1) {
    float t[2] = {0.f, 0.f};
    for (int par = 0; par < 2; ++par)
      PLAN_TRY(time_ms(s, [&] { return enqueue(p, ch->opts, par == 1, s); }, &t[par]));
    ch->parallel = t[1] <= t[0];
    snprintf(buf, sizeof(buf), "branches %s (%.3f ms concurrent, %.3f ms serial)",
             ch->parallel ? "concurrent" : "serial", t[1], t[0]);
    text += buf;
  } else {
    text += "one class";
  }
  ch->text = text;
  return LQT_OK;
}

// Captures the plan's launch sequence (enqueue with its chosen options) into a graph on the
// plan's own capture stream: the fork and join events and the branch streams are the plan's,
// created before and destroyed after the executable graph; nothing is captured while tuning.
lqt_status capture(lqt_plan_s* p) {
  PLAN_HIP(hipStreamCreateWithFlags(&p->cap, hipStreamNonBlocking));
  PLAN_HIP(hipEventCreateWithFlags(&p->done, hipEventDisableTiming));
  PLAN_HIP(hipStreamBeginCapture(p->cap, hipStreamCaptureModeThreadLocal));
  const lqt_status st = enqueue(p, p->choice.opts, p->choice.parallel, p->cap);
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(p->cap, &g);  // ends the capture on every path
  if (st != LQT_OK) {
    if (g) hipGraphDestroy(g);
    return st;
  }
  if (e != hipSuccess || !g) {
    if (g) hipGraphDestroy(g);
    return set_error(LQT_EHIP, "hipStreamEndCapture failed");
  }
  p->graph = g;
  PLAN_HIP(hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0));
  return LQT_OK;
}

}  // namespace
}  // namespace lqt

using namespace lqt;

extern "C" {

size_t lqt_batched_workspace_size(const lqt_ragged* classes, int32_t nclasses) {
  if (!classes || nclasses < 1) return 0;
  size_t need = 0;
  for (int i = 0; i < nclasses; ++i) {
    const lqt_ragged& c = classes[i];
    if (c.nx < 1 || c.nx > 16 || c.nu < 1 || c.nu > c.nx || c.count < 1 ||
        c.rows < 2L * c.count || c.rows > 0x7fffffffL || c.n_steps < 1 ||
        (c.dtype != LQT_F64 && c.dtype != LQT_F32))
      return 0;
    need += class_bytes(c);
  }
  return need;
}

lqt_status lqt_solve_batched(const lqt_ragged* classes, int32_t nclasses, void* ws,
                             size_t ws_bytes, hipStream_t stream) {
  std::vector<ClassRun> cr;
  PLAN_TRY(prepare(classes, nclasses, ws, ws_bytes, cr));
  for (const auto& r : cr) PLAN_TRY(run_class(r, default_opts(r), stream));
  return clear_error();
}

lqt_status lqt_plan_create(const lqt_ragged* classes, int32_t nclasses, void* ws,
                           size_t ws_bytes, int32_t flags, hipStream_t stream, lqt_plan* plan) {
  if (!plan) return set_error(LQT_EINVAL, "plan is NULL");
  *plan = nullptr;
  if (flags & ~(LQT_PLAN_AUTOTUNE | LQT_PLAN_GRAPH)) return set_error(LQT_EINVAL, "unknown flags");
  lqt_plan_s* p = new lqt_plan_s();
  lqt_status st = prepare(classes, nclasses, ws, ws_bytes, p->cls);
  auto fail_with = [&](lqt_status s) {
    release(p);
    delete p;
    return s;
  };
  if (st != LQT_OK) return fail_with(st);
  if (hipEventCreateWithFlags(&p->fork, hipEventDisableTiming) != hipSuccess)
    return fail_with(set_error(LQT_EHIP, "event creation failed"));
  for (size_t i = 0; i < p->cls.size(); ++i) {
    hipStream_t b;
    hipEvent_t e;
    if (hipStreamCreateWithFlags(&b, hipStreamNonBlocking) != hipSuccess)
      return fail_with(set_error(LQT_EHIP, "stream creation failed"));
    p->branch.push_back(b);
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess)
      return fail_with(set_error(LQT_EHIP, "event creation failed"));
    p->join.push_back(e);
  }
  // class signatures contain no blanks (comma- and semicolon-separated numbers)
  const std::string key = device_arch() + " " + signature(p->cls);
  const TuneMode mode = tune_mode();
  const bool want_tune =
      mode == TuneMode::kForce || (mode == TuneMode::kOn && (flags & LQT_PLAN_AUTOTUNE));
  bool have = false;
  if (want_tune && mode != TuneMode::kForce) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    cache_load_locked();
    auto it = g_tune_cache.find(key);
    if (it != g_tune_cache.end() && it->second.opts.size() == p->cls.size()) {
      p->choice = it->second;
      have = true;
    }
  }
  if (!have) {
    if (want_tune) {
      // Tuning runs are ordered after the caller's pending work on `stream`.
      st = tune(p, stream, &p->choice);
      if (st != LQT_OK) return fail_with(st);
      std::lock_guard<std::mutex> lk(g_tune_mu);
      cache_load_locked();
      g_tune_cache[key] = p->choice;
      cache_save_locked();
    } else {
      for (const auto& r : p->cls) p->choice.opts.push_back(default_opts(r));
      p->choice.parallel = true;
      p->choice.text = "default configuration";
    }
  }
  if (hipStreamSynchronize(stream) != hipSuccess)
    return fail_with(set_error(LQT_EHIP, "stream synchronisation failed"));
  if (flags & LQT_PLAN_GRAPH) {
    st = capture(p);
    if (st != LQT_OK) return fail_with(st);
  }
  *plan = p;
  return clear_error();
}

lqt_status lqt_plan_launch(lqt_plan plan, hipStream_t stream) {
  if (!plan) return set_error(LQT_EINVAL, "plan is NULL");
  if (plan->exec) {
    PLAN_HIP(hipGraphLaunch(plan->exec, stream));
    PLAN_HIP(hipEventRecord(plan->done, stream));
    plan->replayed = true;
  } else {
    PLAN_TRY(enqueue(plan, plan->choice.opts, plan->choice.parallel, stream));
  }
  return clear_error();
}

const char* lqt_plan_config(lqt_plan plan) { return plan ? plan->choice.text.c_str() : ""; }

void lqt_plan_destroy(lqt_plan plan) {
  if (!plan) return;
  release(plan);
  delete plan;
}

}  // extern "C"
