// Wavefront-level trees over the 64 lanes of a wave (one tuple or affine map per lane), used by
// the upper levels of the scans.  Lanes exchange data with cross-lane shuffles (ds_bpermute);
// every lane executes every shuffle, only the lanes a level needs do arithmetic.
//
// Value tree (reverse orientation, time runs with the lane index):
//   up-sweep   lane m with m % 2^(s+1) == 0 absorbs the block of lane m + 2^s: P_m <- P_m (x) P_q.
//              Afterwards lane q keeps the product of lanes [q, q + 2^low(q)) (low = lowest set
//              bit) and lane 0 the product of the whole wave.
//   down-sweep lane 0 starts with the value at the right end of the wave's range; at level s the
//              right half [q, ..) of block [m, ..) inherits the block's right-end value and the
//              left half gets fold(P_q, value), so every lane ends with the value at the right end
//              of its own range (Theorem 6 applied to the tree).
// Trajectory tree (forward orientation): the mirror image, with lane 63 holding the whole-wave
//   composition and the down-sweep carrying the state at the left end of each block.
#pragma once

#include "lane_math.hpp"

namespace lqt {

template <class R>
LQT_DEV R shfl(R v, int src) {
  return __shfl(v, src, 64);
}

template <int N, class R>
LQT_DEV void shfl_tup(const Tup<N, R>& x, Tup<N, R>& y, int src) {
#pragma unroll
  for (int i = 0; i < N; ++i) {
#pragma unroll
    for (int j = 0; j < N; ++j) y.A[i][j] = shfl(x.A[i][j], src);
    y.b[i] = shfl(x.b[i], src);
    y.e[i] = shfl(x.e[i], src);
  }
#pragma unroll
  for (int i = 0; i < Sym<N>::size; ++i) {
    y.C[i] = shfl(x.C[i], src);
    y.J[i] = shfl(x.J[i], src);
  }
}

template <int N, class R>
LQT_DEV void shfl_aff(const Aff<N, R>& x, Aff<N, R>& y, int src) {
#pragma unroll
  for (int i = 0; i < N; ++i) {
#pragma unroll
    for (int j = 0; j < N; ++j) y.P[i][j] = shfl(x.P[i][j], src);
    y.q[i] = shfl(x.q[i], src);
  }
}

template <int N, class R>
LQT_DEV void shfl_val(const R (&S)[Sym<N>::size], const R (&v)[N], R (&So)[Sym<N>::size],
                      R (&vo)[N], int src) {
#pragma unroll
  for (int i = 0; i < Sym<N>::size; ++i) So[i] = shfl(S[i], src);
#pragma unroll
  for (int i = 0; i < N; ++i) vo[i] = shfl(v[i], src);
}

template <int N, class R>
LQT_DEV void shfl_vec(const R (&x)[N], R (&y)[N], int src) {
#pragma unroll
  for (int i = 0; i < N; ++i) y[i] = shfl(x[i], src);
}

// Number of tree levels needed when only lanes [0, active) hold data: ceil(log2(active)).
LQT_DEV int tree_levels(long active) {
  int l = 0;
  while (l < 6 && (1L << l) < active) ++l;
  return l;
}

// Up-sweep of the value tree over `levels` levels (6 for a full wave): on return P holds this
// lane's partial product (see above).
template <int N, class R>
LQT_DEV void wave_up_value(Tup<N, R>& P, int lane, int levels = 6) {
  for (int s = 0; s < levels; ++s) {
    const int d = 1 << s;
    Tup<N, R> y;
    shfl_tup(P, y, min(lane + d, 63));
    if ((lane & (2 * d - 1)) == 0) {
      Tup<N, R> o;
      combine(P, y, o);
      P = o;
    }
  }
}

// Down-sweep of the value tree: (S, v) enters as the wave's right-end value (read from lane 0)
// and leaves as the value at the right end of this lane's range.  P is the lane's partial.
template <int N, class R>
LQT_DEV void wave_down_value(const Tup<N, R>& P, R (&S)[Sym<N>::size], R (&v)[N], int lane,
                             int levels = 6) {
  constexpr int NS = Sym<N>::size;
  for (int s = levels - 1; s >= 0; --s) {
    const int d = 1 << s;
    const int m = lane & ~(2 * d - 1);  // left lane of this lane's block at level s
    const int q = m + d;                // first lane of the right half
    R Sm[NS], vm[N];
    shfl_val<N, R>(S, v, Sm, vm, m);    // the block's right-end value
    // Right-half leader folds its partial into the block value: left half's right-end value.
    R Sf[NS], vf[N];
#pragma unroll
    for (int i = 0; i < NS; ++i) Sf[i] = Sm[i];
#pragma unroll
    for (int i = 0; i < N; ++i) vf[i] = vm[i];
    if (lane == q) {
      Aff<N, R> unused;
      fold(P, Sf, vf, unused);
    }
    R Sl[NS], vl[N];
    shfl_val<N, R>(Sf, vf, Sl, vl, q);
    if (lane == q) {
#pragma unroll
      for (int i = 0; i < NS; ++i) S[i] = Sm[i];
#pragma unroll
      for (int i = 0; i < N; ++i) v[i] = vm[i];
    } else if (lane == m) {
#pragma unroll
      for (int i = 0; i < NS; ++i) S[i] = Sl[i];
#pragma unroll
      for (int i = 0; i < N; ++i) v[i] = vl[i];
    }
  }
}

// Up-sweep of the trajectory tree: lane r with r % 2^(s+1) == 2^(s+1) - 1 composes the block of
// lane r - 2^s before its own: P_r <- P_r o P_l.  Lane 63 ends with the whole-wave composition;
// lane l keeps the composition of lanes (l - 2^low'(l), l] where low' is the number of trailing
// one bits of l.
template <int N, class R>
LQT_DEV void wave_up_traj(Aff<N, R>& P, int lane, int levels = 6) {
  for (int s = 0; s < levels; ++s) {
    const int d = 1 << s;
    Aff<N, R> y;
    shfl_aff(P, y, max(lane - d, 0));
    if ((lane & (2 * d - 1)) == 2 * d - 1) aff_after(P, y);
  }
}

// Down-sweep of the trajectory tree: x enters as the state at the wave's left end (read from lane
// 63) and leaves as the state at the left end of this lane's range.
template <int N, class R>
LQT_DEV void wave_down_traj(const Aff<N, R>& P, R (&x)[N], int lane, int levels = 6) {
  for (int s = levels - 1; s >= 0; --s) {
    const int d = 1 << s;
    const int r = lane | (2 * d - 1);  // right lane of this lane's block at level s
    const int l = r - d;               // last lane of the left half
    R xr[N];
    shfl_vec<N, R>(x, xr, r);          // the block's left-end state
    R xa[N];
#pragma unroll
    for (int i = 0; i < N; ++i) xa[i] = xr[i];
    if (lane == l) aff_apply(P, xa);   // state after the left half
    R xl[N];
    shfl_vec<N, R>(xa, xl, l);
    if (lane == l) {
#pragma unroll
      for (int i = 0; i < N; ++i) x[i] = xr[i];
    } else if (lane == r) {
#pragma unroll
      for (int i = 0; i < N; ++i) x[i] = xl[i];
    }
  }
}

}  // namespace lqt
