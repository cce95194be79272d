// Cross-lane shuffles of the per-lane objects of the scans (tuples, affine maps, values), used by
// the wave-level scans of the upper tree levels.  They compile to ds_bpermute; every lane of the
// wave executes every shuffle.
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

}  // namespace lqt
