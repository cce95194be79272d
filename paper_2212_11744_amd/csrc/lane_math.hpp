// Register-resident small-matrix algebra of the LQT solver, one problem block (or one tuple) per
// lane, for state sizes N <= 4.  Everything is fully unrolled at compile time so that matrices
// live in VGPRs and every product exposes N*N independent FMA chains.
//
// Representation (shared with the global structure-of-arrays layout of the C ABI):
//   A is held as its deviation from the identity, Ad = A - I.  Blocks are short (A = I + O(h)),
//   so storing A itself would round the O(h) part to the precision of 1 and, in FP32, lose most
//   of it; every formula below is rearranged around Ad so that no small quantity is ever formed
//   as the difference of two numbers close to one.
//   C, J (and the value matrix S) are symmetric and kept as packed upper triangles.
#pragma once

#include <hip/hip_runtime.h>

#define LQT_DEV __device__ __forceinline__

#include "coherent.hpp"
#include "lqt_internal.hpp"

namespace lqt {

template <int N>
struct Sym {
  static constexpr int size = N * (N + 1) / 2;
  // Packed index of (i, j), upper triangle stored row by row.
  static constexpr int at(int i, int j) {
    return i <= j ? i * N - (i * (i - 1)) / 2 + (j - i) : j * N - (j * (j - 1)) / 2 + (i - j);
  }
};

// Offsets of the element components inside one structure-of-arrays record of NE values.
template <int N>
struct Lay {
  static constexpr int NS = Sym<N>::size;
  static constexpr int A = 0;
  static constexpr int B = N * N;
  static constexpr int C = N * N + N;
  static constexpr int E = N * N + N + NS;
  static constexpr int J = N * N + 2 * N + NS;
  static constexpr int NE = 2 * N * N + 3 * N;
  static constexpr int NV = NS + N;     // value record: packed S, then v
  static constexpr int NM = N * N + N;  // affine map record: Psi - I, then alpha
};

// Tiled structure-of-arrays: records of NQ values for items k = 0..n-1 are stored in tiles of
// kTile = 512 items; inside a tile value q of item k sits at row q, column 64 (k % 8) + (k % 512) / 8:
//   index = (k / 512) * NQ * 512 + q * 512 + 64 (k % 8) + (k % 512) / 8.
// A wave access to "item j of every lane" is one contiguous 512-byte row (FP64) when each lane
// owns 8 consecutive items (the value scan), two contiguous 256-byte half-rows when it owns 4 (the
// serial sweeps), and eight 64-byte segments when it owns one (the builds).
constexpr int kTile = kEltTile;
constexpr int kChunk = 4;  // items per lane in every serial sweep

template <int NQ>
LQT_DEV long tix(int q, long k) {
  return (k >> 9) * (NQ * (long)kTile) + (long)q * kTile + ((k & 7) << 6) + ((k & 511) >> 3);
}


// Conditional value function parameters (A - I, b, C, eta, J) of one interval.
template <int N, class R>
struct Tup {
  R A[N][N];
  R b[N];
  R C[Sym<N>::size];
  R e[N];
  R J[Sym<N>::size];
};

// Affine map x -> (I + P) x + q (closed-loop state transition over an interval).
template <int N, class R>
struct Aff {
  R P[N][N];
  R q[N];
};

template <int N, class R>
LQT_DEV void tup_identity(Tup<N, R>& x) {
#pragma unroll
  for (int i = 0; i < N; ++i) {
#pragma unroll
    for (int j = 0; j < N; ++j) x.A[i][j] = R(0);
    x.b[i] = R(0);
    x.e[i] = R(0);
  }
#pragma unroll
  for (int i = 0; i < Sym<N>::size; ++i) {
    x.C[i] = R(0);
    x.J[i] = R(0);
  }
}

template <int N, class R>
LQT_DEV void tup_load(Tup<N, R>& x, const R* __restrict__ base, long k) {
  using L = Lay<N>;
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int j = 0; j < N; ++j) x.A[i][j] = base[tix<L::NE>(L::A + i * N + j, k)];
#pragma unroll
  for (int i = 0; i < N; ++i) x.b[i] = base[tix<L::NE>(L::B + i, k)];
#pragma unroll
  for (int i = 0; i < Sym<N>::size; ++i) x.C[i] = base[tix<L::NE>(L::C + i, k)];
#pragma unroll
  for (int i = 0; i < N; ++i) x.e[i] = base[tix<L::NE>(L::E + i, k)];
#pragma unroll
  for (int i = 0; i < Sym<N>::size; ++i) x.J[i] = base[tix<L::NE>(L::J + i, k)];
}

template <int N, class R>
LQT_DEV void tup_store(const Tup<N, R>& x, R* __restrict__ base, long k) {
  using L = Lay<N>;
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int j = 0; j < N; ++j) base[tix<L::NE>(L::A + i * N + j, k)] = x.A[i][j];
#pragma unroll
  for (int i = 0; i < N; ++i) base[tix<L::NE>(L::B + i, k)] = x.b[i];
#pragma unroll
  for (int i = 0; i < Sym<N>::size; ++i) base[tix<L::NE>(L::C + i, k)] = x.C[i];
#pragma unroll
  for (int i = 0; i < N; ++i) base[tix<L::NE>(L::E + i, k)] = x.e[i];
#pragma unroll
  for (int i = 0; i < Sym<N>::size; ++i) base[tix<L::NE>(L::J + i, k)] = x.J[i];
}

// Records: value q of record r at base[q * stride + r] (element order).
template <class Acc, int N, class R>
LQT_DEV void tup_store_rec(const Tup<N, R>& x, R* base, long stride, long r) {
  using L = Lay<N>;
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int j = 0; j < N; ++j) Acc::st(base + (L::A + i * N + j) * stride + r, x.A[i][j]);
#pragma unroll
  for (int i = 0; i < N; ++i) Acc::st(base + (L::B + i) * stride + r, x.b[i]);
#pragma unroll
  for (int i = 0; i < Sym<N>::size; ++i) Acc::st(base + (L::C + i) * stride + r, x.C[i]);
#pragma unroll
  for (int i = 0; i < N; ++i) Acc::st(base + (L::E + i) * stride + r, x.e[i]);
#pragma unroll
  for (int i = 0; i < Sym<N>::size; ++i) Acc::st(base + (L::J + i) * stride + r, x.J[i]);
}

template <class Acc, int N, class R>
LQT_DEV void tup_load_rec(Tup<N, R>& x, const R* base, long stride, long r) {
  using L = Lay<N>;
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int j = 0; j < N; ++j) x.A[i][j] = Acc::ld(base + (L::A + i * N + j) * stride + r);
#pragma unroll
  for (int i = 0; i < N; ++i) x.b[i] = Acc::ld(base + (L::B + i) * stride + r);
#pragma unroll
  for (int i = 0; i < Sym<N>::size; ++i) x.C[i] = Acc::ld(base + (L::C + i) * stride + r);
#pragma unroll
  for (int i = 0; i < N; ++i) x.e[i] = Acc::ld(base + (L::E + i) * stride + r);
#pragma unroll
  for (int i = 0; i < Sym<N>::size; ++i) x.J[i] = Acc::ld(base + (L::J + i) * stride + r);
}

// 1 / x from the hardware reciprocal estimate refined by two Newton-Raphson steps
// (r <- r + r (1 - x r)): within about an ulp of the quotient for the pivots met here (entries of
// I + C J, Lemma 10), with half the dependent operations of the IEEE division sequence.
LQT_DEV double recip(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = fma(r, fma(-x, r, 1.0), r);
  return fma(r, fma(-x, r, 1.0), r);
}
LQT_DEV float recip(float x) {
  const float r = __builtin_amdgcn_rcpf(x);
  return fmaf(r, fmaf(-x, r, 1.0f), r);
}

// Solve M X = B in place (B <- M^{-1} B) by Gauss-Jordan elimination with partial pivoting.
// The pivot search keeps the first row of largest magnitude.  Row exchanges sit behind a
// data-dependent branch: for the near-identity matrices of short blocks no lane takes it and the
// whole wave skips the exchange.
template <int N, int NB, class R>
LQT_DEV void gj_solve(R (&M)[N][N], R (&B)[N][NB]) {
#pragma unroll
  for (int c = 0; c < N; ++c) {
#pragma unroll
    for (int i = c + 1; i < N; ++i) {
      if (fabs(M[i][c]) > fabs(M[c][c])) {
#pragma unroll
        for (int j = c; j < N; ++j) {
          R t = M[i][j];
          M[i][j] = M[c][j];
          M[c][j] = t;
        }
#pragma unroll
        for (int j = 0; j < NB; ++j) {
          R t = B[i][j];
          B[i][j] = B[c][j];
          B[c][j] = t;
        }
      }
    }
    const R inv = recip(M[c][c]);
#pragma unroll
    for (int j = c + 1; j < N; ++j) M[c][j] *= inv;
#pragma unroll
    for (int j = 0; j < NB; ++j) B[c][j] *= inv;
#pragma unroll
    for (int i = 0; i < N; ++i) {
      if (i == c) continue;
      const R f = M[i][c];
#pragma unroll
      for (int j = c + 1; j < N; ++j) M[i][j] = fma(-f, M[c][j], M[i][j]);
#pragma unroll
      for (int j = 0; j < NB; ++j) B[i][j] = fma(-f, B[c][j], B[i][j]);
    }
  }
}

// Lemma 7 (Sec. IV-A): o = x1 (x) x2 with x1 on [s, tau] (earlier) and x2 on [tau, t] (later).
// With M = I + C1 J2 (invertible by Lemma 10, Appendix B):
//   A = A2 M^{-1} A1,  b = A2 M^{-1} (b1 + C1 eta2) + b2,  C = A2 M^{-1} C1 A2^T + C2,
//   eta = A1^T M^{-T} (eta2 - J2 b1) + eta1,  J = A1^T M^{-T} J2 A1 + J1,
// using (I + J2 C1)^{-1} = M^{-T}.  One factorisation serves all: Y = M^{-1} A1 = I + Yd with
// Yd = M^{-1} (Ad1 - C1 J2), D = M^{-1} C1 and g = M^{-1} (b1 + C1 eta2); then
//   Ad = Ad2 + Yd + Ad2 Yd,  b = g + Ad2 g + b2,  C = (I + Ad2) D (I + Ad2)^T + C2,
//   eta = w + Yd^T w + eta1 (w = eta2 - J2 b1),  J = (I + Yd)^T J2 (I + Ad1) + J1.
// The factorisation shared by both output orders below: M = I + C1 J2 solved against
// B = [Ad1 - C1 J2 | C1 | b1 + C1 eta2], giving [Yd | D | g] = M^{-1} B.
template <int N, class R>
LQT_DEV void combine_solve(const Tup<N, R>& x1, const Tup<N, R>& x2, R (&B)[N][2 * N + 1]) {
  using Y = Sym<N>;
  R M[N][N];
#pragma unroll
  for (int i = 0; i < N; ++i) {
    R g = x1.b[i];
#pragma unroll
    for (int j = 0; j < N; ++j) {
      R s = R(0);
#pragma unroll
      for (int k = 0; k < N; ++k) s = fma(x1.C[Y::at(i, k)], x2.J[Y::at(k, j)], s);
      M[i][j] = (i == j) ? R(1) + s : s;
      B[i][j] = x1.A[i][j] - s;
      B[i][N + j] = x1.C[Y::at(i, j)];
      g = fma(x1.C[Y::at(i, j)], x2.e[j], g);
    }
    B[i][2 * N] = g;
  }
  gj_solve<N, 2 * N + 1>(M, B);
}

// Output parts of the combination from the solved B (see combine).  Each reads only the inputs
// named and writes one component of o; the two orders below rely on that.
template <int N, class R>
LQT_DEV void combine_C(const Tup<N, R>& x2, const R (&B)[N][2 * N + 1], R (&oC)[Sym<N>::size]) {
  using Y = Sym<N>;
  // W = (I + Ad2) D, C = W (I + Ad2)^T + C2 (upper triangle)
  R Wm[N][N];
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int j = 0; j < N; ++j) {
      R s = B[i][N + j];
#pragma unroll
      for (int k = 0; k < N; ++k) s = fma(x2.A[i][k], B[k][N + j], s);
      Wm[i][j] = s;
    }
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int j = i; j < N; ++j) {
      R s = Wm[i][j];
#pragma unroll
      for (int l = 0; l < N; ++l) s = fma(Wm[i][l], x2.A[j][l], s);
      oC[Y::at(i, j)] = x2.C[Y::at(i, j)] + s;
    }
}

template <int N, class R>
LQT_DEV void combine_b(const Tup<N, R>& x2, const R (&B)[N][2 * N + 1], R (&ob)[N]) {
  // b = g + Ad2 g + b2
  R bn[N];
#pragma unroll
  for (int i = 0; i < N; ++i) {
    R s = R(0);
#pragma unroll
    for (int k = 0; k < N; ++k) s = fma(x2.A[i][k], B[k][2 * N], s);
    bn[i] = x2.b[i] + B[i][2 * N] + s;
  }
#pragma unroll
  for (int i = 0; i < N; ++i) ob[i] = bn[i];
}

// w = eta2 - J2 b1
template <int N, class R>
LQT_DEV void combine_w(const Tup<N, R>& x1, const Tup<N, R>& x2, R (&w)[N]) {
  using Y = Sym<N>;
#pragma unroll
  for (int i = 0; i < N; ++i) {
    R s = x2.e[i];
#pragma unroll
    for (int k = 0; k < N; ++k) s = fma(-x2.J[Y::at(i, k)], x1.b[k], s);
    w[i] = s;
  }
}

// eta = w + Yd^T w + eta1 (o.e may be x1.e)
template <int N, class R>
LQT_DEV void combine_e(const R (&e1)[N], const R (&w)[N], const R (&B)[N][2 * N + 1], R (&oe)[N]) {
#pragma unroll
  for (int i = 0; i < N; ++i) {
    R s = R(0);
#pragma unroll
    for (int k = 0; k < N; ++k) s = fma(B[k][i], w[k], s);
    oe[i] = e1[i] + (w[i] + s);
  }
}

// J: P = J2 (I + Ad1), J = (I + Yd)^T P + J1 (upper triangle; o.J may be x1.J or x2.J)
template <int N, class R>
LQT_DEV void combine_J(const Tup<N, R>& x1, const Tup<N, R>& x2, const R (&B)[N][2 * N + 1],
                       R (&oJ)[Sym<N>::size]) {
  using Y = Sym<N>;
  R P[N][N];
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int j = 0; j < N; ++j) {
      R s = x2.J[Y::at(i, j)];
#pragma unroll
      for (int k = 0; k < N; ++k) s = fma(x2.J[Y::at(i, k)], x1.A[k][j], s);
      P[i][j] = s;
    }
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int j = i; j < N; ++j) {
      R s = P[i][j];
#pragma unroll
      for (int k = 0; k < N; ++k) s = fma(B[k][i], P[k][j], s);
      oJ[Y::at(i, j)] = x1.J[Y::at(i, j)] + s;
    }
}

// Ad = Ad2 + Yd + Ad2 Yd (row by row: row i of the result needs only row i of Ad2; o.A may be
// x1.A or x2.A)
template <int N, class R>
LQT_DEV void combine_A(const R (&A2)[N][N], const R (&B)[N][2 * N + 1], R (&oA)[N][N]) {
#pragma unroll
  for (int i = 0; i < N; ++i) {
    R row[N];
#pragma unroll
    for (int j = 0; j < N; ++j) {
      R s = R(0);
#pragma unroll
      for (int k = 0; k < N; ++k) s = fma(A2[i][k], B[k][j], s);
      row[j] = A2[i][j] + B[i][j] + s;
    }
#pragma unroll
    for (int j = 0; j < N; ++j) oA[i][j] = row[j];
  }
}

// Lemma 7 (Sec. IV-A): o = x1 (x) x2 with x1 on [s, tau] (earlier) and x2 on [tau, t] (later).
// With M = I + C1 J2 (invertible by Lemma 10, Appendix B):
//   A = A2 M^{-1} A1,  b = A2 M^{-1} (b1 + C1 eta2) + b2,  C = A2 M^{-1} C1 A2^T + C2,
//   eta = A1^T M^{-T} (eta2 - J2 b1) + eta1,  J = A1^T M^{-T} J2 A1 + J1,
// using (I + J2 C1)^{-1} = M^{-T}.  One factorisation serves all: Y = M^{-1} A1 = I + Yd with
// Yd = M^{-1} (Ad1 - C1 J2), D = M^{-1} C1 and g = M^{-1} (b1 + C1 eta2); then
//   Ad = Ad2 + Yd + Ad2 Yd,  b = g + Ad2 g + b2,  C = (I + Ad2) D (I + Ad2)^T + C2,
//   eta = w + Yd^T w + eta1 (w = eta2 - J2 b1),  J = (I + Yd)^T J2 (I + Ad1) + J1.
// The outputs are produced in an order that consumes each input component before the matching
// output is written, so `o` may alias x2 (the running product of a right-to-left reduction).
template <int N, class R>
LQT_DEV void combine(const Tup<N, R>& x1, const Tup<N, R>& x2, Tup<N, R>& o) {
  R B[N][2 * N + 1];
  combine_solve(x1, x2, B);
  combine_C(x2, B, o.C);
  combine_b(x2, B, o.b);
  R w[N];
  combine_w(x1, x2, w);
  combine_e(x1.e, w, B, o.e);
  combine_J(x1, x2, B, o.J);
  combine_A(x2.A, B, o.A);
}

// x1 <- x1 (x) x2 in place: the same arithmetic as combine, its outputs ordered so that every
// component of x1 is read before it is overwritten (w and J, which read b1 and Ad1, come first),
// which saves the registers of a separate result tuple.
template <int N, class R>
LQT_DEV void combine_into_first(Tup<N, R>& x1, const Tup<N, R>& x2) {
  R B[N][2 * N + 1];
  combine_solve(x1, x2, B);
  R w[N];
  combine_w(x1, x2, w);
  combine_J(x1, x2, B, x1.J);
  combine_e(x1.e, w, B, x1.e);
  combine_C(x2, B, x1.C);
  combine_b(x2, B, x1.b);
  combine_A(x2.A, B, x1.A);
}

// One step of the value recursion: the Lemma with a right operand of the terminal form
// (A = b = C = 0, eta = v, J = S), i.e. V(., t_k) from a_k and V(., t_{k+1}) (Sec. IV-D):
//   Psi = (I + C S)^{-1} A = I + Pd,  Pd = (I + C S)^{-1} (Ad - C S),
//   alpha = (I + C S)^{-1} (b + C v),
//   S' = Psi^T S A + J,  v' = Psi^T (v - S b) + eta.
// (Psi, alpha) is also the closed-loop map x_{k+1} = Psi x_k + alpha of the block (Sec. IV-E), so
// it is returned for the trajectory.  S, v are updated in place.
template <int N, class R>
LQT_DEV void fold(const Tup<N, R>& a, R (&S)[Sym<N>::size], R (&v)[N], Aff<N, R>& m) {
  using Y = Sym<N>;
  R CS[N][N], M[N][N], B[N][N + 1];
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int j = 0; j < N; ++j) {
      R s = R(0);
#pragma unroll
      for (int k = 0; k < N; ++k) s = fma(a.C[Y::at(i, k)], S[Y::at(k, j)], s);
      CS[i][j] = s;
      M[i][j] = (i == j) ? R(1) + s : s;
    }
#pragma unroll
  for (int i = 0; i < N; ++i) {
    R g = a.b[i];
#pragma unroll
    for (int j = 0; j < N; ++j) {
      B[i][j] = a.A[i][j] - CS[i][j];
      g = fma(a.C[Y::at(i, j)], v[j], g);
    }
    B[i][N] = g;
  }
  gj_solve<N, N + 1>(M, B);
#pragma unroll
  for (int i = 0; i < N; ++i) {
#pragma unroll
    for (int j = 0; j < N; ++j) m.P[i][j] = B[i][j];
    m.q[i] = B[i][N];
  }
  // w = v - S b
  R w[N];
#pragma unroll
  for (int i = 0; i < N; ++i) {
    R s = v[i];
#pragma unroll
    for (int k = 0; k < N; ++k) s = fma(-S[Y::at(i, k)], a.b[k], s);
    w[i] = s;
  }
  // X = S (I + Ad);  S' = J + X + Pd^T X (upper);  v' = eta + w + Pd^T w
  R X[N][N];
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int j = 0; j < N; ++j) {
      R s = R(0);
#pragma unroll
      for (int k = 0; k < N; ++k) s = fma(S[Y::at(i, k)], a.A[k][j], s);
      X[i][j] = S[Y::at(i, j)] + s;
    }
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int j = i; j < N; ++j) {
      R s = R(0);
#pragma unroll
      for (int k = 0; k < N; ++k) s = fma(B[k][i], X[k][j], s);
      S[Y::at(i, j)] = a.J[Y::at(i, j)] + (X[i][j] + s);
    }
#pragma unroll
  for (int i = 0; i < N; ++i) {
    R s = R(0);
#pragma unroll
    for (int k = 0; k < N; ++k) s = fma(B[k][i], w[k], s);
    v[i] = a.e[i] + (w[i] + s);
  }
}

// Closed-loop block map only (no value update): Psi, alpha from a_k and S_{k+1}, v_{k+1}.
template <int N, class R>
LQT_DEV void block_map(const R (&Ad)[N][N], const R (&b)[N], const R (&C)[Sym<N>::size],
                       const R (&S)[Sym<N>::size], const R (&v)[N], Aff<N, R>& m) {
  using Y = Sym<N>;
  R M[N][N], B[N][N + 1];
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int j = 0; j < N; ++j) {
      R s = R(0);
#pragma unroll
      for (int k = 0; k < N; ++k) s = fma(C[Y::at(i, k)], S[Y::at(k, j)], s);
      M[i][j] = (i == j) ? R(1) + s : s;
      B[i][j] = Ad[i][j] - s;
    }
#pragma unroll
  for (int i = 0; i < N; ++i) {
    R g = b[i];
#pragma unroll
    for (int j = 0; j < N; ++j) g = fma(C[Y::at(i, j)], v[j], g);
    B[i][N] = g;
  }
  gj_solve<N, N + 1>(M, B);
#pragma unroll
  for (int i = 0; i < N; ++i) {
#pragma unroll
    for (int j = 0; j < N; ++j) m.P[i][j] = B[i][j];
    m.q[i] = B[i][N];
  }
}

template <int N, class R>
LQT_DEV void aff_identity(Aff<N, R>& m) {
#pragma unroll
  for (int i = 0; i < N; ++i) {
#pragma unroll
    for (int j = 0; j < N; ++j) m.P[i][j] = R(0);
    m.q[i] = R(0);
  }
}

// acc <- later o acc  (apply acc first, then `later`):  P = Pa + Pl + Pl Pa,  q = ql + qa + Pl qa.
template <int N, class R>
LQT_DEV void aff_then(Aff<N, R>& acc, const Aff<N, R>& later) {
  R P[N][N], q[N];
#pragma unroll
  for (int i = 0; i < N; ++i) {
#pragma unroll
    for (int j = 0; j < N; ++j) {
      R s = R(0);
#pragma unroll
      for (int k = 0; k < N; ++k) s = fma(later.P[i][k], acc.P[k][j], s);
      P[i][j] = acc.P[i][j] + later.P[i][j] + s;
    }
    R s = R(0);
#pragma unroll
    for (int k = 0; k < N; ++k) s = fma(later.P[i][k], acc.q[k], s);
    q[i] = later.q[i] + acc.q[i] + s;
  }
#pragma unroll
  for (int i = 0; i < N; ++i) {
#pragma unroll
    for (int j = 0; j < N; ++j) acc.P[i][j] = P[i][j];
    acc.q[i] = q[i];
  }
}

// acc <- acc o earlier  (apply `earlier` first, then acc).
template <int N, class R>
LQT_DEV void aff_after(Aff<N, R>& acc, const Aff<N, R>& earlier) {
  R P[N][N], q[N];
#pragma unroll
  for (int i = 0; i < N; ++i) {
#pragma unroll
    for (int j = 0; j < N; ++j) {
      R s = R(0);
#pragma unroll
      for (int k = 0; k < N; ++k) s = fma(acc.P[i][k], earlier.P[k][j], s);
      P[i][j] = earlier.P[i][j] + acc.P[i][j] + s;
    }
    R s = R(0);
#pragma unroll
    for (int k = 0; k < N; ++k) s = fma(acc.P[i][k], earlier.q[k], s);
    q[i] = acc.q[i] + earlier.q[i] + s;
  }
#pragma unroll
  for (int i = 0; i < N; ++i) {
#pragma unroll
    for (int j = 0; j < N; ++j) acc.P[i][j] = P[i][j];
    acc.q[i] = q[i];
  }
}

// x <- (I + P) x + q
template <int N, class R>
LQT_DEV void aff_apply(const Aff<N, R>& m, R (&x)[N]) {
  R y[N];
#pragma unroll
  for (int i = 0; i < N; ++i) {
    R s = R(0);
#pragma unroll
    for (int k = 0; k < N; ++k) s = fma(m.P[i][k], x[k], s);
    y[i] = x[i] + (s + m.q[i]);
  }
#pragma unroll
  for (int i = 0; i < N; ++i) x[i] = y[i];
}

template <int N, class R>
LQT_DEV void aff_load(Aff<N, R>& m, const R* __restrict__ base, long k) {
#pragma unroll
  for (int i = 0; i < N; ++i) {
#pragma unroll
    for (int j = 0; j < N; ++j) m.P[i][j] = base[tix<Lay<N>::NM>(i * N + j, k)];
    m.q[i] = base[tix<Lay<N>::NM>(N * N + i, k)];
  }
}

template <class Acc, int N, class R>
LQT_DEV void aff_store_rec(const Aff<N, R>& m, R* base, long stride, long r) {
#pragma unroll
  for (int i = 0; i < N; ++i) {
#pragma unroll
    for (int j = 0; j < N; ++j) Acc::st(base + (i * N + j) * stride + r, m.P[i][j]);
    Acc::st(base + (N * N + i) * stride + r, m.q[i]);
  }
}

template <class Acc, int N, class R>
LQT_DEV void aff_load_rec(Aff<N, R>& m, const R* base, long stride, long r) {
#pragma unroll
  for (int i = 0; i < N; ++i) {
#pragma unroll
    for (int j = 0; j < N; ++j) m.P[i][j] = Acc::ld(base + (i * N + j) * stride + r);
    m.q[i] = Acc::ld(base + (N * N + i) * stride + r);
  }
}

template <int N, class R>
LQT_DEV void aff_store(const Aff<N, R>& m, R* __restrict__ base, long k) {
#pragma unroll
  for (int i = 0; i < N; ++i) {
#pragma unroll
    for (int j = 0; j < N; ++j) base[tix<Lay<N>::NM>(i * N + j, k)] = m.P[i][j];
    base[tix<Lay<N>::NM>(N * N + i, k)] = m.q[i];
  }
}

}  // namespace lqt
