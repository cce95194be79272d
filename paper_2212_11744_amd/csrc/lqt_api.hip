// Host side of the C ABI declared in include/lqt.h: argument validation, workspace planning,
// dispatch to the kernel instantiation of (nx, nu, dtype) and the launch sequence of every stage.
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <initializer_list>
#include <mutex>
#include <string>

#include <atomic>
#include <cstdlib>

#include "../../include/lqt.h"
#include "lqt_internal.hpp"

namespace lqt {

namespace {

thread_local std::string g_last_error;

lqt_status fail(lqt_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return st;
}

lqt_status ok() {
  g_last_error.clear();
  return LQT_OK;
}

// Simulated failures of checked HIP calls (lqt_debug_fail_launch, or LQT_FAIL_LAUNCH=n in the
// environment when the library loads): the n-th checked call from then on reports
// hipErrorLaunchFailure; the call itself is made as usual.
std::atomic<int> g_fail_countdown{[] {
  const char* e = getenv("LQT_FAIL_LAUNCH");
  return e ? atoi(e) : 0;
}()};
thread_local bool g_fail_fired = false;

// Canary mode (lqt_debug_canary, or LQT_CANARY=1|2 in the environment when the library loads):
// 0 off, 1 on, 2 on and every call overwrites its first canary itself after filling it (which
// the check must then report).
std::atomic<int> g_canary{[] {
  const char* e = getenv("LQT_CANARY");
  return e ? atoi(e) : 0;
}()};
constexpr unsigned kCanaryWord = 0xC0DEFACEu;

size_t dsize(int dtype) { return dtype == LQT_F64 ? 8 : 4; }
size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }
long ne_of(int nx) { return 2L * nx * nx + 3L * nx; }
long nv_of(int nx) { return (long)nx * (nx + 1) / 2 + nx; }
long nm_of(int nx) { return (long)nx * nx + nx; }
long padt(long n) { return (n + kEltTile - 1) / kEltTile * kEltTile; }

}  // namespace

hipError_t debug_gate(hipError_t e) {
  if (e != hipSuccess || g_fail_countdown.load(std::memory_order_relaxed) <= 0) return e;
  if (g_fail_countdown.fetch_sub(1) == 1) {
    g_fail_fired = true;
    return hipErrorLaunchFailure;
  }
  return e;
}

const char* debug_gate_note() {
  const bool f = g_fail_fired;
  g_fail_fired = false;
  return f ? " (simulated by lqt_debug_fail_launch)" : "";
}

Tree plan_tree(long T) {
  Tree t;
  t.n[0] = T;
  t.n[1] = (T + kLaneChunk - 1) / kLaneChunk;
  t.levels = 1;
  while (t.n[t.levels] > kWaveSpan && t.levels < kMaxLevels) {
    t.n[t.levels + 1] = (t.n[t.levels] + kWaveSpan - 1) / kWaveSpan;
    ++t.levels;
  }
  return t;
}

// Wave-path trees: n[0] = T, n[l + 1] = ceil(n[l] / wcs[l]) while n[l] > wcs[l], with
// wcs[0] = wc and kWaveUpperChunk above.
WTree wave_tree(long T, int wc) {
  WTree t;
  t.wc = wc;
  for (int l = 0; l <= kMaxLevels; ++l) t.wcs[l] = l == 0 ? wc : kWaveUpperChunk;
  t.n[0] = T;
  t.n[1] = (T + wc - 1) / wc;
  t.levels = 1;
  while (t.n[t.levels] > t.wcs[t.levels] && t.levels < kMaxLevels) {
    const int b = t.wcs[t.levels];
    t.n[t.levels + 1] = (t.n[t.levels] + b - 1) / b;
    ++t.levels;
  }
  return t;
}

// Dispatch over the build shards (see lqt_internal.hpp).
const Ops* lane_ops(int nx, int nu, int dtype) {
  static const Ops* (*const shard[kLaneShards])(int, int, int) = {
      lane_ops_shard<0>, lane_ops_shard<1>, lane_ops_shard<2>, lane_ops_shard<3>};
  static_assert(kLaneShards == 4, "one entry per per-lane shard");
  for (auto f : shard)
    if (const Ops* o = f(nx, nu, dtype)) return o;
  return nullptr;
}

namespace {

const WaveFns* wave_fns(int nx, int dtype) {
  static const WaveFns* (*const shard[kWaveShards])(int, int) = {
      wave_fns_shard<0>, wave_fns_shard<1>, wave_fns_shard<2>, wave_fns_shard<3>,
      wave_fns_shard<4>, wave_fns_shard<5>, wave_fns_shard<6>, wave_fns_shard<7>};
  static_assert(kWaveShards == 8, "one entry per wave shard");
  for (auto f : shard)
    if (const WaveFns* w = f(nx, dtype)) return w;
  return nullptr;
}

}  // namespace

// Stage order of kw_solve_queue: value reduce 1 .. L, value top, value down L - 1 .. 1, value
// bottom, trajectory reduce 2 .. L, trajectory top, trajectory down L - 1 .. 1, bottom.
bool wave_queue(const WTree& t, long batch, const Work& w, WQueue* q) {
  if (t.levels > kWqMaxLevels || !w.wq_done) return false;
  const int L = t.levels;
  q->levels = L;
  for (int l = 0; l <= L; ++l) q->wcs[l] = t.wcs[l];
  for (int l = 0; l <= L; ++l) q->n[l] = t.n[l];
  for (int l = 1; l <= L; ++l) {
    q->vtup[l] = w.vtup[l];
    q->vval[l] = w.vval[l];
    q->tmap[l] = w.tmap[l];
    q->tx[l] = w.tx[l];
  }
  int ns = 0;
  long at = 0;
  auto add = [&](int kind, int level, long nodes) {
    q->kind[ns] = kind;
    q->level[ns] = level;
    q->start[ns] = at;
    at += batch * nodes;
    ++ns;
  };
  enum { VRed = 0, VTop, VDown, VBot, TRed, TTop, TDown, TBot };  // WqKind of lqt_wave.hip
  for (int l = 1; l <= L; ++l) add(VRed, l, t.n[l]);
  add(VTop, L, 1);
  for (int l = L - 1; l >= 1; --l) add(VDown, l, t.n[l + 1]);
  add(VBot, 1, t.n[1]);
  for (int l = 2; l <= L; ++l) add(TRed, l, t.n[l]);
  add(TTop, L, 1);
  for (int l = L - 1; l >= 1; --l) add(TDown, l, t.n[l + 1]);
  add(TBot, 1, t.n[1]);
  q->nst = ns;
  q->total = at;
  q->done = w.wq_done;
  q->bmap = w.bmap;
  return at + 1 <= w.wq_words;
}

hipError_t wave_solve_queue(const KProb& kp, int dtype, const WQueue& q, const void* elts, void* S,
                            void* v, void* x, void* u, hipStream_t s) {
  const WaveFns* f = wave_fns(kp.nx, dtype);
  return f ? f->solve_queue(kp, q, elts, S, v, x, u, s) : hipErrorInvalidValue;
}

hipError_t wave_build(const KProb& kp, int dtype, void* elts, hipStream_t s) {
  const WaveFns* f = wave_fns(kp.nx, dtype);
  return f ? f->build(kp, elts, s) : hipErrorInvalidValue;
}

hipError_t wave_build_fwd(const KProb& kp, int dtype, void* elts, hipStream_t s) {
  const WaveFns* f = wave_fns(kp.nx, dtype);
  return f ? f->build_fwd(kp, elts, s) : hipErrorInvalidValue;
}

hipError_t wave_build_split(const KProb& kp, int dtype, void* elts, hipStream_t s) {
  const WaveFns* f = wave_fns(kp.nx, dtype);
  return f ? f->build_split(kp, elts, s) : hipErrorInvalidValue;
}

hipError_t wave_method2(const KProb& kp, int dtype, const WTree& t, const Work& w,
                        const void* elts, const void* S, const void* v, void* x, void* u,
                        hipStream_t s) {
  const WaveFns* f = wave_fns(kp.nx, dtype);
  return f ? f->method2(kp, t, w, elts, S, v, x, u, s) : hipErrorInvalidValue;
}

hipError_t wave_lti(const KProb& kp, int dtype, void* tab, void* elts, hipStream_t s) {
  const WaveFns* f = wave_fns(kp.nx, dtype);
  if (!f) return hipErrorInvalidValue;
  const hipError_t e = f->lti_prep(kp, tab, s);
  return e != hipSuccess ? e : f->lti_build(kp, tab, elts, s);
}

hipError_t wave_dense(const KProb& kp, int dtype, const void* S, const void* v, const void* x,
                      void* Sd, void* vd, void* xd, void* ud, hipStream_t s) {
  const WaveFns* f = wave_fns(kp.nx, dtype);
  return f ? f->dense(kp, S, v, x, Sd, vd, xd, ud, s) : hipErrorInvalidValue;
}

hipError_t wave_value(const KProb& kp, int dtype, const WTree& t, const Work& w, const void* elts,
                      void* S, void* v, void* maps1, hipStream_t s) {
  const WaveFns* f = wave_fns(kp.nx, dtype);
  return f ? f->value(kp, t, w, elts, S, v, maps1, s) : hipErrorInvalidValue;
}

hipError_t wave_traj(const KProb& kp, int dtype, const WTree& t, const Work& w, const void* elts,
                     const void* S, const void* v, void* x, void* u, bool maps_ready,
                     hipStream_t s) {
  const WaveFns* f = wave_fns(kp.nx, dtype);
  return f ? f->traj(kp, t, w, elts, S, v, x, u, maps_ready, s) : hipErrorInvalidValue;
}

namespace {

Tree tree_for(const lqt_dims* d) { return plan_tree(d->T); }

// Kernel family of a call: the per-lane path (one tuple per lane, registers) where it is
// instantiated (nu <= nx <= 4), otherwise the wavefront-per-tuple path (LDS, any nx <= 16).
bool use_wave(const lqt_dims* d) { return lane_ops(d->nx, d->nu, d->dtype) == nullptr; }

// Blocks per wave at the bottom level of the wave path's trees for single solves and stage calls
// (upper levels: kWaveUpperChunk), also the chunk the workspace is laid out for.  Measured on
// single solves: 4 vs 8 gives nx = 16 at T = 2^14 1.55 vs 1.61 ms and at 2^12 0.68 vs 0.74 ms,
// nx = 8 and 12 within 1 %; 16 is slower for all three, and so are binary trees (2 per wave at
// every level: nx = 16 1.61 ms, nx = 8 at 2^16 1.30 vs 1.23 ms, nx = 12 2.02 vs 1.92 ms).  A solve must not use fewer blocks per
// wave than its workspace was laid out for: the level-1 tree arrays hold ceil(T / chunk) records.
constexpr int kWaveChunk = 4;

WTree wtree_for(const lqt_dims* d) { return wave_tree(d->T, kWaveChunk); }

}  // namespace

// Byte layout of the workspace of one call.  Returns the total; fills w when base != nullptr.
// wc: nodes per wave of the wave path's trees (the layout for wc also serves any larger wc);
// nconsts: number of problems whose constants are prepared (the batch, or the problems of a
// ragged class).
size_t layout(const lqt_dims* d, lqt_call call, char* base, Work* w, int wc, long nconsts,
              bool ws_elts, bool keep_maps) {
  const size_t es = dsize(d->dtype);
  const long B = d->batch;
  size_t off = 0;
  const bool canaries = g_canary.load() != 0;
  if (w) {
    w->ncanary = 0;
    w->canary_armed = false;
  }
  auto take = [&](size_t bytes) -> void* {
    void* p = base ? base + off : nullptr;
    off += align256(bytes);
    if (canaries) {
      if (w && base && w->ncanary < Work::kMaxCanaries) w->canary[w->ncanary++] = (unsigned*)(base + off);
      off += 256;
    }
    return p;
  };
  if (canaries) {
    void* r = take(sizeof(int));
    if (w) w->canary_res = (int*)r;
  }
  void* consts = take(es * nconsts * consts_count(d->nx, d->nu));
  if (w) w->consts = consts;
  void* fl = take(256);  // finite-check flag (taken here: the wave branch below returns early)
  if (w) w->flag = (int*)fl;
  if (d->lti && (call == LQT_CALL_BUILD || call == LQT_CALL_SOLVE)) {
    void* t = take(es * nconsts * lti_count(d->nx, d->n_steps));
    if (w) w->lti = t;
  }
  // The Method 2 trajectory uses the value-scan arrays for its node products and prefix states.
  const bool want_v = call == LQT_CALL_SCAN_VALUE || call == LQT_CALL_SOLVE ||
                      call == LQT_CALL_TRAJ_METHOD2;
  const bool want_t = call == LQT_CALL_FORWARD_TRAJ || call == LQT_CALL_SOLVE;
  if (use_wave(d)) {
    const WTree t = wave_tree(d->T, wc);
    for (int l = 1; l <= t.levels; ++l) {
      if (want_v) {
        void* a = take(es * B * ne_of(d->nx) * t.n[l]);
        void* b = take(es * B * nm_of(d->nx) * t.n[l]);
        if (w) {
          w->vtup[l] = a;
          w->vval[l] = b;
        }
      }
      if (want_t) {
        void* a = take(es * B * nm_of(d->nx) * t.n[l]);
        void* b = take(es * B * d->nx * t.n[l]);
        if (w) {
          w->tmap[l] = a;
          w->tx[l] = b;
        }
      }
      if (call == LQT_CALL_TRAJ_METHOD2) {  // prefix records of the nodes
        void* a = take(es * B * ne_of(d->nx) * t.n[l]);
        if (w) w->vpart[l] = a;
      }
    }
    if (call == LQT_CALL_SOLVE && ws_elts) {
      void* e = take(es * B * ne_of(d->nx) * (size_t)padt(d->T));
      if (w) w->elts = e;
    }
    if (call == LQT_CALL_SOLVE) {
      // every block's closed-loop map, kept by the value sweep for the trajectory sweep
      if (keep_maps) {
        void* bm = take(es * B * nm_of(d->nx) * (size_t)d->T);
        if (w) w->bmap = bm;
      }
      // status words of the queue solve (an item per tree node and stage) and its counter
      long items = 3 * t.n[1] + 2;
      for (int l = 2; l <= t.levels; ++l) items += 4 * t.n[l];
      const long words = B * items + 1;
      void* q = take(sizeof(unsigned) * words);
      if (w) {
        w->wq_done = (unsigned*)q;
        w->wq_words = words;
      }
    }
    return off;
  }
  const Tree t = tree_for(d);
  // Single-pass scans: the counter and status words of a scan first (one clear), then payloads.
  auto take_lb = [&](LbRecs* r, long tile, long nmap, long nst) {
    const long G = (d->T + tile - 1) / tile, NG = (G + kLbGroupTiles - 1) / kLbGroupTiles;
    const long nwords = B + B * G + B * NG;
    unsigned* words = (unsigned*)take(sizeof(unsigned) * nwords);
    void* tagg = take(es * B * nmap * G);
    void* tst = take(es * B * nst * G);
    void* gagg = take(es * B * nmap * NG);
    void* gst = take(es * B * nst * NG);
    if (w) {
      r->ctr = words;
      r->tflag = words ? words + B : nullptr;
      r->gflag = words ? words + B + B * G : nullptr;
      r->tagg = tagg;
      r->tst = tst;
      r->gagg = gagg;
      r->gst = gst;
      r->G = G;
      r->NG = NG;
      r->nwords = nwords;
    }
  };
  // laid out for one block per lane (the most tiles any chunk gives)
  if (call == LQT_CALL_SCAN_VALUE || call == LQT_CALL_SOLVE)
    take_lb(w ? &w->lbv : nullptr, 64, ne_of(d->nx), nv_of(d->nx));
  if (want_t) take_lb(w ? &w->lbt : nullptr, 64, nm_of(d->nx), d->nx);
  // Method 2: the tree of node products and prefix states
  if (call == LQT_CALL_TRAJ_METHOD2) {
    for (int l = 1; l <= t.levels; ++l) {
      const long lanes_above = l < t.levels ? t.n[l + 1] * 64 : 0;
      void* a = take(es * B * ne_of(d->nx) * padt(t.n[l]));
      void* b = take(es * B * nv_of(d->nx) * padt(t.n[l]));
      void* c = lanes_above ? take(es * B * ne_of(d->nx) * padt(lanes_above)) : nullptr;
      if (w) {
        w->vtup[l] = a;
        w->vval[l] = b;
        w->vpart[l] = c;
      }
    }
  }
  if ((call == LQT_CALL_SOLVE && ws_elts) || call == LQT_CALL_BACKWARD) {
    void* e = take(es * B * ne_of(d->nx) * (size_t)padt(d->T));
    if (w) w->elts = e;
  }
  if (call == LQT_CALL_BACKWARD) {
    const long nx = d->nx, ns = nx * (nx + 1) / 2;
    const long ncm = nx * nx + 2 * nx + ns, ncs = ns + nx;
    for (int l = 1; l <= t.levels; ++l) {
      const long lanes_above = l < t.levels ? t.n[l + 1] * 64 : 0;
      void* a = take(es * B * nm_of(d->nx) * padt(t.n[l]));
      void* b = take(es * B * nx * padt(t.n[l]));
      void* c = lanes_above ? take(es * B * nm_of(d->nx) * padt(lanes_above)) : nullptr;
      void* e = take(es * B * ncm * padt(t.n[l]));
      void* f = take(es * B * ncs * padt(t.n[l]));
      void* g = lanes_above ? take(es * B * ncm * padt(lanes_above)) : nullptr;
      if (w) {
        w->lmap[l] = a;
        w->lst[l] = b;
        w->lpart[l] = c;
        w->cmap[l] = e;
        w->cst[l] = f;
        w->cpart[l] = g;
      }
    }
    void* lam = take(es * B * (size_t)(d->T + 1) * nx);
    void* bnd = take(es * B * (size_t)d->T * 2 * nx);
    void* ws = take(es * B * (size_t)((d->T + 63) / 64) * 2 * nx * nx);
    // step start values (A, eta, J parts) of steps 1 .. n - 1 of every block
    void* ck = d->n_steps <= kCkptMaxSteps && d->n_steps > 1
                   ? take(es * B * (size_t)(d->n_steps - 1) * (nx * nx + nx + nx * (nx + 1) / 2) *
                          padt(d->T))
                   : nullptr;
    if (w) w->ckpt = ck;
    // G(t) = L(t) R^{-1} L(t)^T at every sample, when L is sampled
    void* gs = d->L_sampled ? take(es * B * (size_t)(2L * d->n_steps * d->T + 1) * nx * nx)
                            : nullptr;
    if (w) w->gsamp = gs;
    if (w) {
      w->lam = lam;
      w->bnd = bnd;
      w->wsum = ws;
    }
  }
  return off;
}

namespace {

size_t layout(const lqt_dims* d, lqt_call call, char* base, Work* w) {
  return layout(d, call, base, w, kWaveChunk, d->batch, true);
}

lqt_status check_dims_valid(const lqt_dims* d) {
  if (!d) return fail(LQT_EINVAL, "dims is NULL");
  if (d->dtype != LQT_F64 && d->dtype != LQT_F32)
    return fail(LQT_EINVAL, "dtype %d is neither LQT_F64 nor LQT_F32", d->dtype);
  if (d->nx < 1 || d->nx > 16) return fail(LQT_EINVAL, "nx = %d outside [1, 16]", d->nx);
  if (d->nu < 1 || d->nu > d->nx) return fail(LQT_EINVAL, "nu = %d outside [1, nx]", d->nu);
  if (d->T < 1) return fail(LQT_EINVAL, "T = %d: the horizon needs at least one block", d->T);
  if (d->n_steps < 1 || d->n_steps > 4096)
    return fail(LQT_EINVAL, "n_steps = %d outside [1, 4096]", d->n_steps);
  if (d->batch < 1 || d->batch > 65535)
    return fail(LQT_EINVAL, "batch = %d outside [1, 65535]", d->batch);
  if (d->lti && (d->F_sampled || d->L_sampled || d->has_c))
    return fail(LQT_EINVAL, "lti needs constant F and L and c = 0");
  const long double ns = 2.0L * d->n_steps * d->T + 1;
  if (ns * d->nx * d->nx > 9.0e18L) return fail(LQT_EINVAL, "sample arrays too large");
  return LQT_OK;
}

lqt_status check_supported(const lqt_dims* d) { return check_dims_valid(d); }

hipError_t prep(const lqt_dims* d, const KProb& kp, void* consts, hipStream_t s) {
  if (use_wave(d)) return launch_prep(kp, d->dtype, consts, s);
  return lane_ops(d->nx, d->nu, d->dtype)->prep(kp, consts, s);
}

lqt_status check_ptr(const void* p, const char* name, size_t es) {
  if (!p) return fail(LQT_EINVAL, "%s is NULL", name);
  if (((uintptr_t)p) % es) return fail(LQT_EINVAL, "%s is not aligned to its element size", name);
  return LQT_OK;
}

struct CanaryList {
  unsigned* p[Work::kMaxCanaries];
  int n;
};

// One workgroup per slot, one thread per word.
__global__ void k_canary_fill(const CanaryList c, int* res, int spoil) {
  if (blockIdx.x == 0 && threadIdx.x == 0) *res = 0x7fffffff;
  if ((int)blockIdx.x < c.n)
    c.p[blockIdx.x][threadIdx.x] = spoil && blockIdx.x == 0 ? ~kCanaryWord : kCanaryWord;
}

__global__ void k_canary_check(const CanaryList c, int* res) {
  if ((int)blockIdx.x < c.n && c.p[blockIdx.x][threadIdx.x] != kCanaryWord)
    atomicMin(res, (int)blockIdx.x);
}

CanaryList canary_list(const Work& w) {
  CanaryList c;
  c.n = w.ncanary;
  for (int i = 0; i < w.ncanary; ++i) c.p[i] = w.canary[i];
  return c;
}

lqt_status check_ws(const lqt_dims* d, lqt_call call, void* ws, size_t ws_bytes, Work* w,
                    hipStream_t s) {
  const size_t need = layout(d, call, nullptr, nullptr);
  if (need > 0 && !ws) return fail(LQT_EWORKSPACE, "workspace is NULL (%zu bytes needed)", need);
  if (((uintptr_t)ws) % 256) return fail(LQT_EWORKSPACE, "workspace is not 256-byte aligned");
  if (ws_bytes < need)
    return fail(LQT_EWORKSPACE, "workspace has %zu bytes, %zu needed", ws_bytes, need);
  layout(d, call, (char*)ws, w);
  if (w->ncanary > 0 && w->canary_res) {
    hipLaunchKernelGGL(k_canary_fill, dim3((unsigned)w->ncanary), dim3(64), 0, s, canary_list(*w),
                       w->canary_res, g_canary.load() == 2 ? 1 : 0);
    const hipError_t e = debug_gate(hipGetLastError());
    if (e != hipSuccess)
      return fail(LQT_EHIP, "canary fill failed: %s%s", hipGetErrorString(e), debug_gate_note());
    w->canary_armed = true;
  }
  return LQT_OK;
}

#define LQT_TRY(x)                       \
  do {                                   \
    lqt_status _s = (x);                 \
    if (_s != LQT_OK) return _s;         \
  } while (0)

#define LQT_HIP(x)                                                                  \
  do {                                                                              \
    hipError_t _e = debug_gate(x);                                                  \
    if (_e != hipSuccess)                                                           \
      return fail(LQT_EHIP, "%s failed: %s%s", #x, hipGetErrorString(_e),           \
                  debug_gate_note());                                               \
  } while (0)

// ------------------------------------------------------------------------------------------
// Status words of the single-pass scans: zeroed by a fill kernel before every scan (a kernel
// rather than a memset, so that a captured launch sequence replays it as an ordinary node).
// ------------------------------------------------------------------------------------------
__global__ void k_lb_clear(unsigned* __restrict__ w, long n) {
  for (long k = (long)blockIdx.x * blockDim.x + threadIdx.x; k < n;
       k += (long)gridDim.x * blockDim.x)
    w[k] = 0u;
}

}  // namespace

hipError_t lb_clear(const LbRecs& r, hipStream_t s) {
  const long blocks = min((r.nwords + 255) / 256, 1024L);
  hipLaunchKernelGGL(k_lb_clear, dim3((unsigned)blocks), dim3(256), 0, s, r.ctr, r.nwords);
  return hipGetLastError();
}

namespace {

// ------------------------------------------------------------------------------------------
// Finite check of the outputs (LQT_CHECK_FINITE).
// ------------------------------------------------------------------------------------------
__global__ void k_flag_clear(int* flag) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *flag = 0;
}

// Plain arrays of n values.
template <class R>
__global__ void k_nonfinite(const R* __restrict__ a, long n, int* __restrict__ flag) {
  bool bad = false;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    bad |= !isfinite(a[i]);
  if (bad) *flag = 1;
}

// Elements in the tiled layout: only the columns of blocks k < T (tile padding is never written).
template <class R>
__global__ void k_nonfinite_elts(const R* __restrict__ e, int NE, long T, long pt, int batch,
                                 int* __restrict__ flag) {
  const long n = (long)batch * NE * T;
  bool bad = false;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    const long k = i % T, q = (i / T) % NE, p = i / ((long)NE * T);
    const long idx = p * NE * pt + (k >> 9) * (NE * 512L) + q * 512L + ((k & 7) << 6) + ((k & 511) >> 3);
    bad |= !isfinite(e[idx]);
  }
  if (bad) *flag = 1;
}

bool finite_check_on() {
  const char* v = getenv("LQT_CHECK_FINITE");
  return v && *v && strcmp(v, "0") != 0;
}

struct Arr {
  const void* p;  // nullptr: skipped
  long n;         // values
  bool elts;      // tiled element layout (n unused)
};

// Scans the arrays when LQT_CHECK_FINITE is set; LQT_ENONFINITE if any value is NaN or Inf.
// Canary mode: every slot still holds its pattern after the call's work (synchronises s).
lqt_status canary_check(const Work& w, hipStream_t s) {
  if (!w.canary_armed) return LQT_OK;
  hipLaunchKernelGGL(k_canary_check, dim3((unsigned)w.ncanary), dim3(64), 0, s, canary_list(w),
                     w.canary_res);
  int h = 0;
  LQT_HIP(hipGetLastError());
  LQT_HIP(hipMemcpyAsync(&h, w.canary_res, sizeof(int), hipMemcpyDeviceToHost, s));
  LQT_HIP(hipStreamSynchronize(s));
  if (h != 0x7fffffff)
    return fail(LQT_EWORKSPACE,
                "workspace canary %d of %d overwritten (a region was written past its end)", h,
                w.ncanary);
  return LQT_OK;
}

lqt_status finite_check(const lqt_dims* d, const Work& w, hipStream_t s,
                        std::initializer_list<Arr> arrays) {
  LQT_TRY(canary_check(w, s));
  if (!finite_check_on()) return LQT_OK;
  if (!w.flag) return fail(LQT_EWORKSPACE, "no finite-check flag in the workspace layout");
  hipLaunchKernelGGL(k_flag_clear, dim3(1), dim3(64), 0, s, w.flag);
  const dim3 g(1024), b(256);
  for (const Arr& a : arrays) {
    if (!a.p) continue;
    if (a.elts) {
      if (d->dtype == LQT_F64)
        hipLaunchKernelGGL(k_nonfinite_elts<double>, g, b, 0, s, (const double*)a.p, (int)ne_of(d->nx),
                           (long)d->T, padt(d->T), d->batch, w.flag);
      else
        hipLaunchKernelGGL(k_nonfinite_elts<float>, g, b, 0, s, (const float*)a.p, (int)ne_of(d->nx),
                           (long)d->T, padt(d->T), d->batch, w.flag);
    } else if (d->dtype == LQT_F64) {
      hipLaunchKernelGGL(k_nonfinite<double>, g, b, 0, s, (const double*)a.p, a.n, w.flag);
    } else {
      hipLaunchKernelGGL(k_nonfinite<float>, g, b, 0, s, (const float*)a.p, a.n, w.flag);
    }
  }
  int h = 0;
  LQT_HIP(hipGetLastError());
  LQT_HIP(hipMemcpyAsync(&h, w.flag, sizeof(int), hipMemcpyDeviceToHost, s));
  LQT_HIP(hipStreamSynchronize(s));
  if (h) return fail(LQT_ENONFINITE, "an output holds NaN or Inf (LQT_CHECK_FINITE)");
  return LQT_OK;
}

lqt_status check_problem(const lqt_dims* d, const lqt_problem* p, bool need_r, bool need_x0) {
  const size_t es = dsize(d->dtype);
  if (!p) return fail(LQT_EINVAL, "problem is NULL");
  LQT_TRY(check_ptr(p->t, "t", es));
  LQT_TRY(check_ptr(p->F, "F", es));
  LQT_TRY(check_ptr(p->L, "L", es));
  LQT_TRY(check_ptr(p->Q, "Q", es));
  LQT_TRY(check_ptr(p->R, "R", es));
  LQT_TRY(check_ptr(p->Qf, "Qf", es));
  LQT_TRY(check_ptr(p->rf, "rf", es));
  if (need_r) LQT_TRY(check_ptr(p->r, "r", es));
  if (need_x0) LQT_TRY(check_ptr(p->x0, "x0", es));
  if (d->has_c) LQT_TRY(check_ptr(p->c, "c", es));
  return LQT_OK;
}

KProb make_kprob(const lqt_dims* d, const lqt_problem* p, const void* consts) {
  KProb k;
  k.nx = d->nx;
  k.nu = d->nu;
  k.T = d->T;
  k.n = d->n_steps;
  k.batch = d->batch;
  k.F_sampled = d->F_sampled;
  k.L_sampled = d->L_sampled;
  k.has_c = d->has_c;
  k.lti = d->lti;
  k.t = p ? p->t : nullptr;
  k.F = p ? p->F : nullptr;
  k.L = p ? p->L : nullptr;
  k.c = p ? p->c : nullptr;
  k.Q = p ? p->Q : nullptr;
  k.R = p ? p->R : nullptr;
  k.r = p ? p->r : nullptr;
  k.Qf = p ? p->Qf : nullptr;
  k.rf = p ? p->rf : nullptr;
  k.x0 = p ? p->x0 : nullptr;
  k.consts = consts;
  return k;
}

// The records of a single-pass scan with `chunk` blocks per lane: tile and group counts of the
// launch (the arrays are laid out for one block per lane, so they hold any chunk's records).
LbRecs lb_for(const LbRecs& r, long T, int chunk) {
  LbRecs l = r;
  l.G = (T + 64L * chunk - 1) / (64L * chunk);
  l.NG = (l.G + kLbGroupTiles - 1) / kLbGroupTiles;
  return l;
}

// Value scan over elements (single pass; per-lane path).
// cleared: the records' status words were already cleared (the solve clears both scans' at once).
lqt_status run_value(const Ops* o, const KProb& kp, const Work& w, const void* elts, void* S,
                     void* v, hipStream_t s, bool cleared = false) {
  const int c = scan_chunk(kp.T, kScanMaxVChunk);
  if (!cleared) LQT_HIP(lb_clear(w.lbv, s));
  LQT_HIP(o->vscan(kp, elts, S, v, lb_for(w.lbv, kp.T, c), c, s));
  return LQT_OK;
}

// Trajectory scan (single pass; per-lane path): x_k, u_k of every boundary.
lqt_status run_traj(const Ops* o, const KProb& kp, const Work& w, const void* elts,
                    const void* S, const void* v, void* x, void* u, hipStream_t s,
                    bool cleared = false) {
  const int c = traj_chunk(kp.T);
  if (!cleared) LQT_HIP(lb_clear(w.lbt, s));
  LQT_HIP(o->tscan(kp, elts, S, v, x, u, lb_for(w.lbt, kp.T, c), c, s));
  return LQT_OK;
}

}  // namespace
}  // namespace lqt

using namespace lqt;

extern "C" {

size_t lqt_element_count(int32_t nx) { return nx < 1 ? 0 : (size_t)ne_of(nx); }

void lqt_debug_fail_launch(int32_t n) { g_fail_countdown.store(n > 0 ? n : 0); }

void lqt_debug_canary(int32_t mode) { g_canary.store(mode >= 0 && mode <= 2 ? mode : 0); }

size_t lqt_workspace_size(const lqt_dims* dims, lqt_call call) {
  if (check_dims_valid(dims) != LQT_OK) return 0;
  if (call < LQT_CALL_BUILD || call > LQT_CALL_TRAJ_METHOD2) return 0;
  return layout(dims, call, nullptr, nullptr);
}

lqt_status lqt_build_elements(const lqt_dims* dims, const lqt_problem* prob, void* elts, void* ws,
                              size_t ws_bytes, hipStream_t stream) {
  LQT_TRY(check_supported(dims));
  LQT_TRY(check_problem(dims, prob, true, false));
  LQT_TRY(check_ptr(elts, "elts", dsize(dims->dtype)));
  Work w;
  LQT_TRY(check_ws(dims, LQT_CALL_BUILD, ws, ws_bytes, &w, stream));
  KProb kp = make_kprob(dims, prob, w.consts);
  LQT_HIP(prep(dims, kp, w.consts, stream));
  if (use_wave(dims)) {
    if (dims->lti)
      LQT_HIP(wave_lti(kp, dims->dtype, w.lti, elts, stream));
    else
      LQT_HIP(wave_build(kp, dims->dtype, elts, stream));
  } else if (dims->lti) {
    const Ops* o = lane_ops(dims->nx, dims->nu, dims->dtype);
    LQT_HIP(o->lti_prep(kp, w.lti, stream));
    LQT_HIP(o->lti_build(kp, w.lti, elts, stream));
  } else {
    LQT_HIP(lane_ops(dims->nx, dims->nu, dims->dtype)->build(kp, elts, stream));
  }
  LQT_TRY(finite_check(dims, w, stream, {{elts, 0, true}}));
  return ok();
}

lqt_status lqt_build_elements_forward(const lqt_dims* dims, const lqt_problem* prob, void* elts,
                                      void* ws, size_t ws_bytes, hipStream_t stream) {
  LQT_TRY(check_supported(dims));
  LQT_TRY(check_problem(dims, prob, true, false));
  LQT_TRY(check_ptr(elts, "elts", dsize(dims->dtype)));
  Work w;
  LQT_TRY(check_ws(dims, LQT_CALL_BUILD, ws, ws_bytes, &w, stream));
  KProb kp = make_kprob(dims, prob, w.consts);
  LQT_HIP(prep(dims, kp, w.consts, stream));
  if (use_wave(dims))
    LQT_HIP(wave_build_fwd(kp, dims->dtype, elts, stream));
  else
    LQT_HIP(lane_ops(dims->nx, dims->nu, dims->dtype)->build_fwd(kp, elts, stream));
  LQT_TRY(finite_check(dims, w, stream, {{elts, 0, true}}));
  return ok();
}

lqt_status lqt_build_elements_split(const lqt_dims* dims, const lqt_problem* prob, void* elts,
                                    void* ws, size_t ws_bytes, hipStream_t stream) {
  LQT_TRY(check_supported(dims));
  LQT_TRY(check_problem(dims, prob, true, false));
  LQT_TRY(check_ptr(elts, "elts", dsize(dims->dtype)));
  Work w;
  LQT_TRY(check_ws(dims, LQT_CALL_BUILD, ws, ws_bytes, &w, stream));
  KProb kp = make_kprob(dims, prob, w.consts);
  LQT_HIP(prep(dims, kp, w.consts, stream));
  if (use_wave(dims))
    LQT_HIP(wave_build_split(kp, dims->dtype, elts, stream));
  else
    LQT_HIP(lane_ops(dims->nx, dims->nu, dims->dtype)->build_split(kp, elts, stream));
  LQT_TRY(finite_check(dims, w, stream, {{elts, 0, true}}));
  return ok();
}

lqt_status lqt_forward_traj_method2(const lqt_dims* dims, const lqt_problem* prob,
                                    const void* elts, const void* S, const void* v, void* x,
                                    void* u, void* ws, size_t ws_bytes, hipStream_t stream) {
  LQT_TRY(check_supported(dims));
  const size_t es = dsize(dims->dtype);
  if (!prob) return fail(LQT_EINVAL, "problem is NULL");
  LQT_TRY(check_ptr(prob->L, "L", es));
  LQT_TRY(check_ptr(prob->R, "R", es));
  LQT_TRY(check_ptr(prob->x0, "x0", es));
  LQT_TRY(check_ptr(elts, "elts", es));
  LQT_TRY(check_ptr(S, "S", es));
  LQT_TRY(check_ptr(v, "v", es));
  LQT_TRY(check_ptr(x, "x", es));
  if (u) LQT_TRY(check_ptr(u, "u", es));
  Work w;
  LQT_TRY(check_ws(dims, LQT_CALL_TRAJ_METHOD2, ws, ws_bytes, &w, stream));
  KProb kp = make_kprob(dims, prob, w.consts);
  const long nb = dims->batch, T1 = (long)dims->T + 1;
  if (use_wave(dims)) {
    LQT_HIP(prep(dims, kp, w.consts, stream));
    LQT_HIP(wave_method2(kp, dims->dtype, wtree_for(dims), w, elts, S, v, x, u, stream));
    LQT_TRY(finite_check(dims, w, stream,
                         {{x, nb * T1 * dims->nx, false}, {u, nb * T1 * dims->nu, false}}));
    return ok();
  }
  const Ops* o = lane_ops(dims->nx, dims->nu, dims->dtype);
  const Tree t = tree_for(dims);
  LQT_HIP(o->prep(kp, w.consts, stream));
  LQT_HIP(o->vreduce0(kp, elts, w.vtup[1], t.n[1], stream));  // products of 4 blocks
  for (int l = 1; l < t.levels; ++l)
    LQT_HIP(o->m2_up(kp, w.vtup[l], t.n[l], w.vpart[l], w.vtup[l + 1], t.n[l + 1], stream));
  LQT_HIP(o->m2_top(kp, w.vtup[t.levels], t.n[t.levels], w.vval[t.levels], stream));
  for (int l = t.levels - 1; l >= 1; --l)
    LQT_HIP(o->m2_down(kp, w.vtup[l], t.n[l], w.vpart[l], w.vval[l + 1], t.n[l + 1], w.vval[l],
                       stream));
  LQT_HIP(o->m2_bottom(kp, elts, S, v, w.vval[1], t.n[1], x, u, stream));
  LQT_TRY(finite_check(dims, w, stream, {{x, nb * T1 * dims->nx, false}, {u, nb * T1 * dims->nu, false}}));
  return ok();
}

lqt_status lqt_dense_output(const lqt_dims* dims, const lqt_problem* prob, const void* S,
                            const void* v, const void* x, void* Sd, void* vd, void* xd, void* ud,
                            void* ws, size_t ws_bytes, hipStream_t stream) {
  LQT_TRY(check_supported(dims));
  LQT_TRY(check_problem(dims, prob, true, false));
  const size_t es = dsize(dims->dtype);
  LQT_TRY(check_ptr(S, "S", es));
  LQT_TRY(check_ptr(v, "v", es));
  LQT_TRY(check_ptr(x, "x", es));
  LQT_TRY(check_ptr(Sd, "Sd", es));
  LQT_TRY(check_ptr(vd, "vd", es));
  LQT_TRY(check_ptr(xd, "xd", es));
  if (ud) LQT_TRY(check_ptr(ud, "ud", es));
  Work w;
  LQT_TRY(check_ws(dims, LQT_CALL_BUILD, ws, ws_bytes, &w, stream));
  KProb kp = make_kprob(dims, prob, w.consts);
  LQT_HIP(prep(dims, kp, w.consts, stream));
  if (use_wave(dims))
    LQT_HIP(wave_dense(kp, dims->dtype, S, v, x, Sd, vd, xd, ud, stream));
  else
    LQT_HIP(lane_ops(dims->nx, dims->nu, dims->dtype)->dense(kp, S, v, x, Sd, vd, xd, ud, stream));
  const long nb = dims->batch, nodes = (long)dims->n_steps * dims->T + 1, nx = dims->nx;
  LQT_TRY(finite_check(dims, w, stream, {{Sd, nb * nodes * nx * nx, false}, {vd, nb * nodes * nx, false},
                                         {xd, nb * nodes * nx, false}, {ud, nb * nodes * dims->nu, false}}));
  return ok();
}

lqt_status lqt_scan_value(const lqt_dims* dims, const void* elts, const void* Qf, const void* rf,
                          void* S, void* v, void* ws, size_t ws_bytes, hipStream_t stream) {
  LQT_TRY(check_supported(dims));
  const size_t es = dsize(dims->dtype);
  LQT_TRY(check_ptr(elts, "elts", es));
  LQT_TRY(check_ptr(Qf, "Qf", es));
  LQT_TRY(check_ptr(rf, "rf", es));
  LQT_TRY(check_ptr(S, "S", es));
  LQT_TRY(check_ptr(v, "v", es));
  Work w;
  LQT_TRY(check_ws(dims, LQT_CALL_SCAN_VALUE, ws, ws_bytes, &w, stream));
  lqt_problem p;
  memset(&p, 0, sizeof(p));
  p.Qf = Qf;
  p.rf = rf;
  KProb kp = make_kprob(dims, &p, w.consts);
  if (use_wave(dims)) {
    LQT_HIP(wave_value(kp, dims->dtype, wtree_for(dims), w, elts, S, v, nullptr, stream));
  } else {
    const Ops* o = lane_ops(dims->nx, dims->nu, dims->dtype);
    LQT_TRY(run_value(o, kp, w, elts, S, v, stream));
  }
  const long nb = dims->batch, T1 = (long)dims->T + 1, nx = dims->nx;
  LQT_TRY(finite_check(dims, w, stream, {{S, nb * T1 * nx * nx, false}, {v, nb * T1 * nx, false}}));
  return ok();
}

lqt_status lqt_forward_traj(const lqt_dims* dims, const lqt_problem* prob, const void* elts,
                            const void* S, const void* v, void* x, void* u, void* ws,
                            size_t ws_bytes, hipStream_t stream) {
  LQT_TRY(check_supported(dims));
  const size_t es = dsize(dims->dtype);
  if (!prob) return fail(LQT_EINVAL, "problem is NULL");
  LQT_TRY(check_ptr(prob->L, "L", es));
  LQT_TRY(check_ptr(prob->R, "R", es));
  LQT_TRY(check_ptr(prob->x0, "x0", es));
  LQT_TRY(check_ptr(elts, "elts", es));
  LQT_TRY(check_ptr(S, "S", es));
  LQT_TRY(check_ptr(v, "v", es));
  LQT_TRY(check_ptr(x, "x", es));
  if (u) LQT_TRY(check_ptr(u, "u", es));
  Work w;
  LQT_TRY(check_ws(dims, LQT_CALL_FORWARD_TRAJ, ws, ws_bytes, &w, stream));
  KProb kp = make_kprob(dims, prob, w.consts);
  LQT_HIP(prep(dims, kp, w.consts, stream));
  if (use_wave(dims)) {
    LQT_HIP(wave_traj(kp, dims->dtype, wtree_for(dims), w, elts, S, v, x, u, false, stream));
  } else {
    const Ops* o = lane_ops(dims->nx, dims->nu, dims->dtype);
    LQT_TRY(run_traj(o, kp, w, elts, S, v, x, u, stream));
  }
  const long nb = dims->batch, T1 = (long)dims->T + 1;
  LQT_TRY(finite_check(dims, w, stream, {{x, nb * T1 * dims->nx, false}, {u, nb * T1 * dims->nu, false}}));
  return ok();
}

}  // extern "C"

namespace lqt {

// The launch sequence of a full solve (prep, elements, value scan, trajectory scan) for
// validated arguments; shared by lqt_solve and the batched solve.
lqt_status run_solve(const lqt_dims* dims, const KProb& kp, const Work& w, void* e, void* S,
                     void* v, void* x, void* u, const SolveOpts& o, hipStream_t stream) {
  KProb kprep = kp;
  if (kp.seg) kprep.batch = kp.nseg;
  if (use_wave(dims)) {
    LQT_HIP(prep(dims, kprep, w.consts, stream));
    const WTree wt = wave_tree(dims->T, o.wave_chunk);
    if (kp.lti && !kp.seg && w.lti)
      LQT_HIP(wave_lti(kp, dims->dtype, w.lti, e, stream));
    else
      LQT_HIP(wave_build(kp, dims->dtype, e, stream));
    WQueue q;
    if (o.queue_chunk && wave_queue(wt, kp.batch, w, &q)) {
      hipLaunchKernelGGL(k_lb_clear, dim3((unsigned)min((w.wq_words + 255) / 256, 1024L)),
                         dim3(256), 0, stream, w.wq_done, w.wq_words);
      LQT_HIP(hipGetLastError());
      LQT_HIP(wave_solve_queue(kp, dims->dtype, q, e, S, v, x, u, stream));
      return LQT_OK;
    }
    LQT_HIP(wave_value(kp, dims->dtype, wt, w, e, S, v, w.tmap[1], stream));
    LQT_HIP(wave_traj(kp, dims->dtype, wt, w, e, S, v, x, u, true, stream));
    return LQT_OK;
  }
  const Ops* op = lane_ops(dims->nx, dims->nu, dims->dtype);
  // the constants, and both scans' status words cleared in the same launch
  LQT_HIP(op->prep_clear(kprep, w.consts, w.lbv, w.lbt, stream));
  const bool lti = kp.lti && !kp.seg && w.lti;
  if (lti) {
    LQT_HIP(op->lti_prep(kp, w.lti, stream));
    LQT_HIP(op->lti_build(kp, w.lti, e, stream));
  } else {
    LQT_HIP(op->build(kp, e, stream));
  }
  if (o.queue_chunk) {
    const int cv = o.queue_chunk;
    LQT_HIP(op->scan_queue(kp, e, S, v, x, u, lb_for(w.lbv, kp.T, cv),
                             lb_for(w.lbt, kp.T, queue_tchunk(cv)), cv, stream));
    return LQT_OK;
  }
  LQT_TRY(run_value(op, kp, w, e, S, v, stream, true));
  LQT_TRY(run_traj(op, kp, w, e, S, v, x, u, stream, true));
  return LQT_OK;
}

lqt_status set_error(lqt_status st, const char* msg) { return fail(st, "%s", msg); }
lqt_status clear_error() { return ok(); }

}  // namespace lqt

extern "C" {

lqt_status lqt_solve(const lqt_dims* dims, const lqt_problem* prob, void* elts, void* S, void* v,
                     void* x, void* u, void* ws, size_t ws_bytes, hipStream_t stream) {
  LQT_TRY(check_supported(dims));
  LQT_TRY(check_problem(dims, prob, true, true));
  const size_t es = dsize(dims->dtype);
  if (elts) LQT_TRY(check_ptr(elts, "elts", es));
  LQT_TRY(check_ptr(S, "S", es));
  LQT_TRY(check_ptr(v, "v", es));
  LQT_TRY(check_ptr(x, "x", es));
  if (u) LQT_TRY(check_ptr(u, "u", es));
  Work w;
  LQT_TRY(check_ws(dims, LQT_CALL_SOLVE, ws, ws_bytes, &w, stream));
  KProb kp = make_kprob(dims, prob, w.consts);
  void* e = elts ? elts : w.elts;
  SolveOpts o;
  o.wave_chunk = kWaveChunk;
  LQT_TRY(run_solve(dims, kp, w, e, S, v, x, u, o, stream));
  const long nb = dims->batch, T1 = (long)dims->T + 1, nx = dims->nx;
  LQT_TRY(finite_check(dims, w, stream, {{S, nb * T1 * nx * nx, false}, {v, nb * T1 * nx, false},
                                         {x, nb * T1 * nx, false}, {u, nb * T1 * dims->nu, false},
                                         {elts, 0, true}}));
  return ok();
}

}  // extern "C"

// ------------------------------------------------------------------------------------------
// The solve without allocation (lqt_solve_noalloc): its scratch memory is a fixed device array of
// the library, one per GPU the library runs on (each device's copy lives until the process ends).
// Host code only ever uses the device address hipGetSymbolAddress returns for the current
// device, never the array's name.
// ------------------------------------------------------------------------------------------
namespace lqt {
namespace {

constexpr size_t kNoAllocScratchBytes = (size_t)LQT_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of the current device's scratch array (looked up once per device).
lqt_status noalloc_scratch(void** out) {
  int dev = -1;
  LQT_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices)
    return fail(LQT_EUNSUPPORTED, "device %d: the no-allocation entry point serves devices 0..%d",
                dev, kMaxDevices - 1);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(LQT_EHIP, "hipGetSymbolAddress(scratch) failed on device %d: %s", dev,
                  hipGetErrorString(e));
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return LQT_OK;
}

}  // namespace
}  // namespace lqt

extern "C" {

size_t lqt_noalloc_scratch_size(const lqt_dims* dims) {
  if (check_dims_valid(dims) != LQT_OK) return 0;
  return layout(dims, LQT_CALL_SOLVE, nullptr, nullptr, kWaveChunk, dims->batch, false, false);
}

lqt_status lqt_solve_noalloc(const lqt_dims* dims, const lqt_problem* prob, void* elts, void* S,
                             void* v, void* x, void* u, hipStream_t stream) {
  LQT_TRY(check_supported(dims));
  LQT_TRY(check_problem(dims, prob, true, true));
  const size_t es = dsize(dims->dtype);
  LQT_TRY(check_ptr(elts, "elts", es));
  LQT_TRY(check_ptr(S, "S", es));
  LQT_TRY(check_ptr(v, "v", es));
  LQT_TRY(check_ptr(x, "x", es));
  if (u) LQT_TRY(check_ptr(u, "u", es));
  const size_t need =
      layout(dims, LQT_CALL_SOLVE, nullptr, nullptr, kWaveChunk, dims->batch, false, false);
  if (need > kNoAllocScratchBytes)
    return fail(LQT_EWORKSPACE,
                "this problem needs %zu bytes of scratch; the no-allocation entry point has %zu "
                "(use lqt_solve with a workspace)",
                need, kNoAllocScratchBytes);
  void* base = nullptr;
  LQT_TRY(noalloc_scratch(&base));
  Work w;
  layout(dims, LQT_CALL_SOLVE, (char*)base, &w, kWaveChunk, dims->batch, false, false);
  KProb kp = make_kprob(dims, prob, w.consts);
  SolveOpts o;
  o.wave_chunk = kWaveChunk;
  LQT_TRY(run_solve(dims, kp, w, elts, S, v, x, u, o, stream));
  const long nb = dims->batch, T1 = (long)dims->T + 1, nx = dims->nx;
  LQT_TRY(finite_check(dims, w, stream, {{S, nb * T1 * nx * nx, false}, {v, nb * T1 * nx, false},
                                         {x, nb * T1 * nx, false}, {u, nb * T1 * dims->nu, false},
                                         {elts, 0, true}}));
  return ok();
}

lqt_status lqt_backward(const lqt_dims* dims, const lqt_problem* prob, const void* S,
                        const void* v, const void* x, const void* dLdx, void* dQ, void* dR,
                        void* dr, void* dx0, void* dQf, void* drf, void* ws, size_t ws_bytes,
                        hipStream_t stream) {
  LQT_TRY(check_supported(dims));
  const AdjOps* ao = adj_ops(dims->nx, dims->nu, dims->dtype);
  if (!ao || use_wave(dims))
    return fail(LQT_EUNSUPPORTED, "lqt_backward is available for nx <= 4");
  LQT_TRY(check_problem(dims, prob, true, true));
  const size_t es = dsize(dims->dtype);
  LQT_TRY(check_ptr(S, "S", es));
  LQT_TRY(check_ptr(v, "v", es));
  LQT_TRY(check_ptr(x, "x", es));
  LQT_TRY(check_ptr(dLdx, "dLdx", es));
  LQT_TRY(check_ptr(dQ, "dQ", es));
  LQT_TRY(check_ptr(dR, "dR", es));
  LQT_TRY(check_ptr(dr, "dr", es));
  LQT_TRY(check_ptr(dx0, "dx0", es));
  if (dQf) LQT_TRY(check_ptr(dQf, "dQf", es));
  if (drf) LQT_TRY(check_ptr(drf, "drf", es));
  Work w;
  LQT_TRY(check_ws(dims, LQT_CALL_BACKWARD, ws, ws_bytes, &w, stream));
  const Ops* o = lane_ops(dims->nx, dims->nu, dims->dtype);
  KProb kp = make_kprob(dims, prob, w.consts);
  const Tree t = tree_for(dims);
  hipStream_t s = stream;
  LQT_HIP(o->prep(kp, w.consts, s));
  // rebuild the elements; with a checkpoint buffer also keep the RK4 step start values
  if (w.ckpt)
    LQT_HIP(o->build_ckpt(kp, w.elts, w.ckpt, s));
  else
    LQT_HIP(o->build(kp, w.elts, s));
  // lambda_k = xbar_k + Psi_k^T lambda_{k+1} (backward)
  LQT_HIP(ao->lam_bottom(kp, w.elts, S, v, dLdx, w.lmap[1], t.n[1], s));
  for (int l = 1; l < t.levels; ++l)
    LQT_HIP(ao->lam_up(kp, w.lmap[l], t.n[l], w.lpart[l], w.lmap[l + 1], t.n[l + 1], s));
  LQT_HIP(ao->lam_top(kp, dLdx, w.lmap[t.levels], t.n[t.levels], w.lst[t.levels], s));
  for (int l = t.levels - 1; l >= 1; --l)
    LQT_HIP(ao->lam_down(kp, w.lmap[l], t.n[l], w.lpart[l], w.lst[l + 1], t.n[l + 1], w.lst[l], s));
  // (Sbar_k, vbar_k) (forward)
  LQT_HIP(ao->cong_bottom(kp, w.elts, S, v, x, dLdx, w.lst[1], t.n[1], w.lam, w.cmap[1], dx0, s));
  for (int l = 1; l < t.levels; ++l)
    LQT_HIP(ao->cong_up(kp, w.cmap[l], t.n[l], w.cpart[l], w.cmap[l + 1], t.n[l + 1], s));
  LQT_HIP(ao->cong_top(kp, w.cmap[t.levels], t.n[t.levels], w.cst[t.levels], s));
  for (int l = t.levels - 1; l >= 1; --l)
    LQT_HIP(ao->cong_down(kp, w.cmap[l], t.n[l], w.cpart[l], w.cst[l + 1], t.n[l + 1], w.cst[l], s));
  // element gradients, then the RK4 adjoint of every block and the reductions
  LQT_HIP(ao->elem(kp, w.elts, S, v, x, w.lam, w.cst[1], t.n[1], dQf, drf, s));
  LQT_HIP(ao->rk4(kp, w.elts, dr, w.bnd, w.wsum, w.ckpt, w.ckpt != nullptr, w.gsamp, s));
  LQT_HIP(ao->finish(kp, w.bnd, dr, w.wsum, dQ, dR, s));
  const long nb = dims->batch, nx = dims->nx, nu = dims->nu;
  const long ns = 2L * dims->n_steps * dims->T + 1;
  LQT_TRY(finite_check(dims, w, s, {{dQ, nb * nx * nx, false}, {dR, nb * nu * nu, false},
                                    {dr, nb * ns * nx, false}, {dx0, nb * nx, false},
                                    {dQf, nb * nx * nx, false}, {drf, nb * nx, false}}));
  return ok();
}

const char* lqt_status_string(lqt_status s) {
  switch (s) {
    case LQT_OK: return "ok";
    case LQT_EINVAL: return "invalid argument";
    case LQT_EUNSUPPORTED: return "unsupported";
    case LQT_EWORKSPACE: return "workspace missing or too small";
    case LQT_EHIP: return "HIP runtime error";
    case LQT_ENONFINITE: return "non-finite output";
  }
  return "unknown status";
}

const char* lqt_last_error(void) { return g_last_error.c_str(); }

int32_t lqt_version(void) { return 100; }

}  // extern "C"
