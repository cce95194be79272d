// Generic upper levels of the scan trees, parameterised by an "algebra":
//
//   Alg::kForward   true: the state flows forward in time (left end -> right end of a range);
//                   false: backward (right end -> left end), as for value functions.
//   Alg::Map        the per-interval object (a tuple, an affine map, ...), Alg::State the state.
//   Alg::chain(first, second, out)   the object of the concatenated interval, `first` earlier.
//   Alg::apply(map, state)           carries the state across the map's interval in the
//                                    algebra's direction.
//   Alg::identity / load / store / shfl_map, Alg::sload / sstore / shfl_state, Alg::NMAP / NST
//   Alg::init(kp, aux, p, state)     the state at the free end of the horizon (terminal value,
//                                    initial state, ...).
//
// A level reduces 4 consecutive nodes per lane serially, then scans the 64 lane products of a wave
// in registers by recursive doubling (every lane combines with the lane 2^s away at step s), so
// that each lane ends with the product of every lane between itself and the wave's free end.  The
// upward pass stores that exclusive product per lane; the downward pass then needs one
// application per lane to carry the wave's boundary state to the lane's range, where a tree
// replay would need one per level.  The orientation decides which end is "free":
//   backward: lane m absorbs lane m + 2^s (its later neighbour); lane 0 ends with the wave
//             product and the boundary state enters at the right end (after lane 63);
//   forward:  lane r absorbs lane r - 2^s (its earlier neighbour); lane 63 ends with the product
//             and the boundary state enters at the left end (before lane 0).
#pragma once

#include "lane_math.hpp"
#include "wave_tree.hpp"

namespace lqt {

__host__ __device__ inline long padt(long n) { return (n + kTile - 1) / kTile * kTile; }

template <class Alg, class R>
LQT_DEV void serial_chain(const R* __restrict__ s, long j0, long j1, typename Alg::Map& acc) {
  if (j0 >= j1) {
    Alg::identity(acc);
    return;
  }
  if (!Alg::kForward) {
    Alg::load(acc, s, j1 - 1);
    if (j1 - 2 < j0) return;
    typename Alg::Map nxt;
    Alg::load(nxt, s, j1 - 2);
    for (long j = j1 - 2; j >= j0; --j) {
      typename Alg::Map x = nxt;
      if (j - 1 >= j0) Alg::load(nxt, s, j - 1);
      Alg::chain(x, acc, acc);
    }
  } else {
    Alg::load(acc, s, j0);
    if (j0 + 1 >= j1) return;
    typename Alg::Map nxt;
    Alg::load(nxt, s, j0 + 1);
    for (long j = j0 + 1; j < j1; ++j) {
      typename Alg::Map x = nxt;
      if (j + 1 < j1) Alg::load(nxt, s, j + 1);
      Alg::chain(acc, x, acc);
    }
  }
}

// Inclusive scan of the lane products over `levels` doubling steps: on return P holds the product
// of lanes [lane, lane + 2^levels) (backward) or (lane - 2^levels, lane] (forward), clipped to
// the wave.  With 2^levels >= the number of lanes holding data, that is every later (earlier)
// data lane.
template <class Alg>
LQT_DEV void wave_scan(typename Alg::Map& P, int lane, int levels = 6) {
  for (int s = 0; s < levels; ++s) {
    const int d = 1 << s;
    typename Alg::Map y;
    if (!Alg::kForward) {
      Alg::shfl_map(P, y, min(lane + d, 63));
      if (lane + d < 64) Alg::chain(P, y, P);
    } else {
      Alg::shfl_map(P, y, max(lane - d, 0));
      if (lane >= d) Alg::chain(y, P, P);
    }
  }
}

// The lane nearest the wave's free end: its range borders the boundary directly.
template <class Alg>
LQT_DEV constexpr int edge_lane() {
  return Alg::kForward ? 0 : 63;
}

// Exclusive form of wave_scan's result: the product of the lanes strictly between this lane and
// the free end (undefined on the edge lane, which must not use it).
template <class Alg>
LQT_DEV void wave_exclusive(const typename Alg::Map& I, typename Alg::Map& E, int lane) {
  Alg::shfl_map(I, E, Alg::kForward ? max(lane - 1, 0) : min(lane + 1, 63));
}

// Serial downward sweep over the <= 4 nodes [j0, j1): node j receives the state at its free end,
// then the state is carried across node j.
template <class Alg, class R>
LQT_DEV void serial_states(const R* __restrict__ mp, long j0, long j1, typename Alg::State& st,
                           R* __restrict__ so) {
  if (!Alg::kForward) {
    for (long j = j1 - 1; j >= j0; --j) {
      Alg::sstore(st, so, j);
      if (j == j0) break;
      typename Alg::Map m;
      Alg::load(m, mp, j);
      Alg::apply(m, st);
    }
  } else {
    for (long j = j0; j < j1; ++j) {
      Alg::sstore(st, so, j);
      if (j == j1 - 1) break;
      typename Alg::Map m;
      Alg::load(m, mp, j);
      Alg::apply(m, st);
    }
  }
}

// Level l -> l + 1: 256 nodes per wave; each lane's exclusive product kept for the downward pass.
template <class Alg, class R>
__global__ __launch_bounds__(64) void k_up(const R* __restrict__ src, long n_src,
                                           R* __restrict__ part, R* __restrict__ dst,
                                           long n_dst) {
  const int p = blockIdx.y;
  const long gl = (long)blockIdx.x * 64 + threadIdx.x;
  const int lane = threadIdx.x;
  const long w = blockIdx.x;
  if (w >= n_dst) return;
  const long j0 = gl * kChunk, j1 = min(j0 + kChunk, n_src);
  typename Alg::Map P;
  serial_chain<Alg, R>(src + (long)p * Alg::NMAP * padt(n_src), j0, j1, P);
  wave_scan<Alg>(P, lane);
  if (lane == (Alg::kForward ? 63 : 0)) Alg::store(P, dst + (long)p * Alg::NMAP * padt(n_dst), w);
  typename Alg::Map E;
  wave_exclusive<Alg>(P, E, lane);
  Alg::store(E, part + (long)p * Alg::NMAP * padt(n_dst * 64), gl);
}

// Top level (<= 256 nodes, one wave, ceil(n / 64) per lane): scan, boundary state from Alg::init,
// carried to every lane.
template <class Alg, class R>
__global__ __launch_bounds__(64) void k_top(const KProb kp, const R* __restrict__ aux,
                                            const R* __restrict__ src, long n,
                                            R* __restrict__ out) {
  const int p = blockIdx.y;
  const int lane = threadIdx.x;
  const R* mp = src + (long)p * Alg::NMAP * padt(n);
  // As few nodes per lane as fit the wave: the serial chains are the slow part of a short level.
  const long c = n > 64 ? (n + 63) / 64 : 1;
  const long j0 = (long)lane * c, j1 = min(j0 + c, n);
  const long active = (n + c - 1) / c;
  const int levels = tree_levels(active);
  typename Alg::Map P;
  serial_chain<Alg, R>(mp, j0, j1, P);
  wave_scan<Alg>(P, lane, levels);
  typename Alg::Map E;
  wave_exclusive<Alg>(P, E, lane);
  typename Alg::State st;
  Alg::init(kp, aux, p, st);
  // Only lanes with data and with data lanes between them and the free end carry the state (with
  // one data lane, as at the top of a long horizon, the branch is skipped by the whole wave).
  if (lane < active && (Alg::kForward ? lane > 0 : lane + 1 < active)) Alg::apply(E, st);
  serial_states<Alg, R>(mp, j0, j1, st, out + (long)p * Alg::NST * padt(n));
}

// Level l + 1 -> l: states at the free ends of every child node.
template <class Alg, class R>
__global__ __launch_bounds__(64) void k_down(const R* __restrict__ src, long n_child,
                                             const R* __restrict__ part,
                                             const R* __restrict__ st_par, long n_par,
                                             R* __restrict__ st_child) {
  const int p = blockIdx.y;
  const long gl = (long)blockIdx.x * 64 + threadIdx.x;
  const int lane = threadIdx.x;
  const long w = blockIdx.x;
  if (w >= n_par) return;
  typename Alg::State st;
  Alg::sload(st, st_par + (long)p * Alg::NST * padt(n_par), w);
  if (lane != edge_lane<Alg>()) {
    typename Alg::Map E;
    Alg::load(E, part + (long)p * Alg::NMAP * padt(n_par * 64), gl);
    Alg::apply(E, st);
  }
  const long j0 = gl * kChunk, j1 = min(j0 + kChunk, n_child);
  serial_states<Alg, R>(src + (long)p * Alg::NMAP * padt(n_child), j0, j1, st,
                        st_child + (long)p * Alg::NST * padt(n_child));
}

}  // namespace lqt
