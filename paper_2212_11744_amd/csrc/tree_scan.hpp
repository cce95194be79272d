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
// A level reduces 4 consecutive nodes per lane serially, then the 64 lanes of a wave by a
// Blelloch tree in registers; the downward pass replays the tree from the wave's boundary state
// and then each lane's 4 nodes.  The orientation decides which end of a block is "free":
//   backward: lane m absorbs lane m + 2^s (its later neighbour); lane 0 holds the wave product,
//             the boundary state enters at lane 0 (right end) and flows to earlier lanes;
//   forward:  lane r absorbs lane r - 2^s (its earlier neighbour); lane 63 holds the product and
//             the boundary state (left end) enters at the block's last lane.
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

template <class Alg>
LQT_DEV void wave_up(typename Alg::Map& P, int lane, int levels = 6) {
  for (int s = 0; s < levels; ++s) {
    const int d = 1 << s;
    typename Alg::Map y;
    if (!Alg::kForward) {
      Alg::shfl_map(P, y, min(lane + d, 63));
      if ((lane & (2 * d - 1)) == 0) Alg::chain(P, y, P);
    } else {
      Alg::shfl_map(P, y, max(lane - d, 0));
      if ((lane & (2 * d - 1)) == 2 * d - 1) Alg::chain(y, P, P);
    }
  }
}

template <class Alg>
LQT_DEV void wave_down(const typename Alg::Map& P, typename Alg::State& st, int lane,
                       int levels = 6) {
  using State = typename Alg::State;
  for (int s = levels - 1; s >= 0; --s) {
    const int d = 1 << s;
    int holder, worker, other;  // holder: lane with the block's boundary state
    if (!Alg::kForward) {
      holder = lane & ~(2 * d - 1);  // left lane holds the right-end state of the block
      worker = holder + d;           // right half: carries it across its product
      other = holder;
    } else {
      holder = lane | (2 * d - 1);   // right lane holds the left-end state of the block
      worker = holder - d;           // left half: carries it across its product
      other = holder;
    }
    State sb;
    Alg::shfl_state(st, sb, holder);
    State sw = sb;
    if (lane == worker) Alg::apply(P, sw);
    State sx;
    Alg::shfl_state(sw, sx, worker);
    if (lane == worker)
      st = sb;
    else if (lane == other)
      st = sx;
  }
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

// Level l -> l + 1: 256 nodes per wave; lane partials kept for the downward pass.
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
  wave_up<Alg>(P, lane);
  Alg::store(P, part + (long)p * Alg::NMAP * padt(n_dst * 64), gl);
  if (lane == (Alg::kForward ? 63 : 0)) Alg::store(P, dst + (long)p * Alg::NMAP * padt(n_dst), w);
}

// Top level (<= 256 nodes, one wave): up-sweep, boundary state from Alg::init, downward pass.
template <class Alg, class R>
__global__ __launch_bounds__(64) void k_top(const KProb kp, const R* __restrict__ aux,
                                            const R* __restrict__ src, long n,
                                            R* __restrict__ out) {
  const int p = blockIdx.y;
  const int lane = threadIdx.x;
  const R* mp = src + (long)p * Alg::NMAP * padt(n);
  const long j0 = (long)lane * kChunk, j1 = min(j0 + kChunk, n);
  const long active = (n + kChunk - 1) / kChunk;
  const int levels = tree_levels(active);
  typename Alg::Map P;
  serial_chain<Alg, R>(mp, j0, j1, P);
  wave_up<Alg>(P, lane, levels);
  typename Alg::State st;
  Alg::init(kp, aux, p, st);
  wave_down<Alg>(P, st, lane, levels);
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
  typename Alg::Map P;
  Alg::load(P, part + (long)p * Alg::NMAP * padt(n_par * 64), gl);
  wave_down<Alg>(P, st, lane);
  const long j0 = gl * kChunk, j1 = min(j0 + kChunk, n_child);
  serial_states<Alg, R>(src + (long)p * Alg::NMAP * padt(n_child), j0, j1, st,
                        st_child + (long)p * Alg::NST * padt(n_child));
}

}  // namespace lqt
