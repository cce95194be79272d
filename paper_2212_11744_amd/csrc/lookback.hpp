// Single-pass scans with a decoupled look-back, parameterised by the same "algebra" as the tree
// scans (tree_scan.hpp): Alg::Map (per-interval object), Alg::State, chain (first = earlier in
// time), apply (carries a state across a map in the algebra's direction), identity, shfl_map /
// shfl_state and init (the state at the free end of the horizon).
//
// One wavefront owns one tile of consecutive intervals.  Tiles take their place in the scan from
// an atomic counter, in the order in which the state flows (increasing time for a forward scan,
// decreasing time for a backward one), so a tile only ever waits for tiles that took an earlier
// place and are therefore already running: every wait ends.
//
// Protocol, per tile i (place in the flow order), after its wave has reduced its own intervals to
// the tile aggregate:
//   1. publish the aggregate (status kLbAgg);
//   2. find the state at the tile's free end: look at the records of the preceding places, nearest
//      first, 64 at a time (one per lane); take the nearest one whose inclusive state is published
//      (status kLbIncl) and carry that state across the aggregates in between;
//   3. publish the tile's inclusive state (the state carried across the whole tile).
// A look-back that finds no inclusive state among the tiles of its own group (64 consecutive
// places) continues over group records instead: the last tile of every full group also publishes
// the group aggregate (the composite of its 64 tiles) and, once known, the group's inclusive
// state.  A tile thus resolves its state from at most 63 tile records plus the group records
// before it, however many tiles are still busy; with flat tile records alone the inclusive states
// would advance by at most 64 tiles per look-back round trip.
//
// Memory ordering without cache maintenance (coherent.hpp): every record value and status word is
// accessed with relaxed atomics at agent scope, which are coherent per location across the XCDs
// and go past the per-XCD L2 caches instead of requiring them to be written back or invalidated
// (an agent-scope release or acquire does both, for the whole L2, on every use: with thousands of
// tiles per kernel that flushes the caches the element loads rely on).  A record's payload is
// written by one lane, which waits until those stores are complete at device scope before it
// stores the status word; a reader loads status words, and only once the statuses it needs are
// set does it issue the payload loads.  Status words and the tile counter must be zero when the
// kernel starts (lb_clear).
#pragma once

#include "lane_math.hpp"
#include "lqt_internal.hpp"
#include "wave_tree.hpp"

namespace lqt {

constexpr unsigned kLbAgg = 1;   // aggregate published
constexpr unsigned kLbIncl = 2;  // aggregate and inclusive state published
constexpr unsigned kLbDone = 3;  // inclusive state published and the tile's outputs written
                                 // (set by launches that read the outputs back themselves)
constexpr int kLbGroup = kLbGroupTiles;

// Besides the tree-scan members, an algebra used here provides record access with value q of
// record r at base[q * stride + r]: store_rec / load_rec (maps), sstore_rec / sload_rec (states).
// The records live in an LbRecs (lqt_internal.hpp).

LQT_DEV unsigned lb_flag_load(const unsigned* f) { return lq_flag_load(f); }
LQT_DEV void lb_flag_store(unsigned* f, unsigned v) { lq_flag_store(f, v); }
LQT_DEV void lb_acquire() { lq_acquire(); }

// Place of this wave's tile in the flow order of problem p (one atomic per wave).
LQT_DEV long lb_place(const LbRecs& lb, int p) {
  unsigned i = 0;
  if (threadIdx.x == 0) i = atomicAdd(lb.ctr + p, 1u);
  return (long)__shfl(i, 0, 64);
}

// The composite of two maps of adjacent ranges in which the state passes `far` first and `near`
// second (far is the range farther from the receiving tile).
template <class Alg>
LQT_DEV void lb_cat(const typename Alg::Map& near, const typename Alg::Map& far,
                    typename Alg::Map& out) {
  if (Alg::kForward)
    Alg::chain(far, near, out);  // forward flow: the farther range is the earlier one
  else
    Alg::chain(near, far, out);  // backward flow: the nearer range is the earlier one
}

// Tree reduction over lanes [0, n) (n wave-uniform, lanes >= n ignored): on return lane 0 holds
// the composite of the maps of lanes 0 .. n-1 in which the state passes lane n-1 first and
// lane 0 last.  Other lanes hold partial products.
template <class Alg>
LQT_DEV void lb_reduce(typename Alg::Map& m, int lane, int n) {
  for (int s = 0; (1 << s) < n; ++s) {
    const int d = 1 << s;
    typename Alg::Map y;
    Alg::shfl_map(m, y, min(lane + d, 63));
    if ((lane & (2 * d - 1)) == 0 && lane + d < n) lb_cat<Alg>(m, y, m);
  }
}

// Spins until, among the n records idx - 1 - l (lane l < n), every record nearer than the
// nearest one with its inclusive state has published its aggregate (all n of them if none has an
// inclusive state).  Returns the lane of that nearest inclusive record, or n if there is none.
LQT_DEV int lb_wait(const unsigned* flag, long idx, int n, int lane) {
  for (;;) {
    const unsigned f = lane < n ? lb_flag_load(flag + idx - 1 - lane) : 0u;
    const unsigned long long incl = __ballot(lane < n && f >= kLbIncl);
    const unsigned long long ready = __ballot(lane < n && f >= kLbAgg);
    const int lp = incl ? __ffsll((long long)incl) - 1 : n;
    const unsigned long long need = lp >= 64 ? ~0ull : ((1ull << lp) - 1ull);
    if ((ready & need) == need) return lp;
    __builtin_amdgcn_s_sleep(1);
  }
}

// The state entering group g (carried across every group before it), resolved from the group
// records, 64 groups per round.
template <class Alg, class R>
LQT_DEV void lb_group_state(const KProb& kp, const R* aux, int p, const LbRecs& lb, long g,
                            int lane, typename Alg::State& st) {
  using Map = typename Alg::Map;
  const unsigned* gflag = lb.gflag + (long)p * lb.NG;
  const R* gagg = (const R*)lb.gagg + (long)p * Alg::NMAP * lb.NG;
  const R* gst = (const R*)lb.gst + (long)p * Alg::NST * lb.NG;
  Map acc;  // composite of the groups passed so far (lane 0)
  Alg::identity(acc);
  long top = g - 1;  // nearest group not yet passed
  for (;;) {
    const int n = (int)min(top + 1, 64L);
    const int lp = lb_wait(gflag, top + 1, n, lane);
    lb_acquire();
    Map m;
    if (lane < lp)
      Alg::load_rec(m, gagg, lb.NG, top - lane);
    else
      Alg::identity(m);
    lb_reduce<Alg>(m, lane, lp);
    if (lane == 0 && lp > 0) lb_cat<Alg>(acc, m, acc);
    if (lp < n) {
      Alg::sload_rec(st, gst, lb.NG, top - lp);
      break;
    }
    top -= 64;
    if (top < 0) {
      Alg::init(kp, aux, p, st);
      break;
    }
  }
  if (lane == 0) Alg::apply(acc, st);
  typename Alg::State b;
  Alg::shfl_state(st, b, 0);
  st = b;
}

// Steps 1-3 of the protocol for tile i (place in the flow order) of problem p.  agg: the tile
// aggregate, valid in lane 0 and not needed after the call begins (lane 0 reads it back from
// the record it publishes, which keeps it out of the registers during the look-back).  Returns
// in every lane the state at the tile's free end (the end the state enters from).
template <class Alg, class R>
LQT_DEV void lb_resolve(const KProb& kp, const R* aux, int p, const LbRecs& lb, long i,
                        const typename Alg::Map& agg, int lane, typename Alg::State& st) {
  using Map = typename Alg::Map;
  unsigned* tflag = lb.tflag + (long)p * lb.G;
  unsigned* gflag = lb.gflag + (long)p * lb.NG;
  R* tagg = (R*)lb.tagg + (long)p * Alg::NMAP * lb.G;
  R* tst = (R*)lb.tst + (long)p * Alg::NST * lb.G;
  R* gagg = (R*)lb.gagg + (long)p * Alg::NMAP * lb.NG;
  R* gst = (R*)lb.gst + (long)p * Alg::NST * lb.NG;
  const long g = i / kLbGroup;
  const int q = (int)(i % kLbGroup);
  // 1. the aggregate
  if (lane == 0) {
    Alg::store_rec(agg, tagg, lb.G, i);
    lb_flag_store(tflag + i, kLbAgg);
  }
  // 2. in-group look-back
  int lp;
  Map m;
  if (q == kLbGroup - 1) {
    // The last tile of a group first publishes the group aggregate, for which every tile of the
    // group must have published its own (they only reduce their intervals first: a short wait).
    for (;;) {
      const unsigned f = lane < q ? lb_flag_load(tflag + i - 1 - lane) : kLbAgg;
      if (__ballot(f < kLbAgg) == 0ull) break;
      __builtin_amdgcn_s_sleep(1);
    }
    lb_acquire();
    if (lane < q)
      Alg::load_rec(m, tagg, lb.G, i - 1 - lane);
    else
      Alg::identity(m);
    lb_reduce<Alg>(m, lane, q);
    if (lane == 0) {
      Map ga;
      lb_cat<Alg>(agg, m, ga);
      Alg::store_rec(ga, gagg, lb.NG, g);
      lb_flag_store(gflag + g, kLbAgg);
    }
    lp = lb_wait(tflag, i, q, lane);
    if (lp < q) {
      // an inclusive state inside the group: only the records nearer than it are needed
      lb_acquire();
      if (lane < lp)
        Alg::load_rec(m, tagg, lb.G, i - 1 - lane);
      else
        Alg::identity(m);
      lb_reduce<Alg>(m, lane, lp);
    }
  } else {
    lp = lb_wait(tflag, i, q, lane);
    lb_acquire();
    if (lane < lp)
      Alg::load_rec(m, tagg, lb.G, i - 1 - lane);
    else
      Alg::identity(m);
    lb_reduce<Alg>(m, lane, lp);
  }
  if (lp < q) {
    Alg::sload_rec(st, tst, lb.G, i - 1 - lp);
  } else if (g == 0) {
    Alg::init(kp, aux, p, st);
  } else {
    lb_group_state<Alg, R>(kp, aux, p, lb, g, lane, st);
  }
  if (lane == 0 && lp > 0) Alg::apply(m, st);
  {
    typename Alg::State b;
    Alg::shfl_state(st, b, 0);
    st = b;
  }
  // 3. the inclusive state
  if (lane == 0) {
    typename Alg::State inc = st;
    Map a;
    Alg::load_rec(a, tagg, lb.G, i);  // this lane's own store above
    Alg::apply(a, inc);
    Alg::sstore_rec(inc, tst, lb.G, i);
    lb_flag_store(tflag + i, kLbIncl);
    if (q == kLbGroup - 1) {
      Alg::sstore_rec(inc, gst, lb.NG, g);
      lb_flag_store(gflag + g, kLbIncl);
    }
  }
}

}  // namespace lqt
