// Wavefront-per-tuple path for 5 <= nx <= 16 (runtime sizes): one wavefront owns one block (or
// one tree node) and keeps its matrices in LDS; the 64 lanes split the entries of every matrix
// product and elimination step.  The arithmetic is that of the per-lane path (A stored as A - I,
// pivoted Gauss-Jordan solves, the combination rule of Lemma 7, the fold of Theorem 6, the
// closed-loop block maps of Sec. IV-E); only the distribution over lanes differs.
//
// Elements use the tiled layout of the C ABI; tree nodes are records ([batch][n][NQ]) with the
// element's value order: A - I (nx*nx, row-major), b, C (upper triangle, row by row), eta, J.
// Scans: every wave reduces wcs[l] consecutive nodes of level l serially (the bottom chunk chosen at
// run time, upper levels kWaveUpperChunk); level l + 1 has ceil(n_l / wcs[l]) nodes while
// n_l > wcs[l]; the top (<= wcs[L] nodes) is swept by one wave.
#include <cstring>

#include "../../include/lqt.h"
#include "coherent.hpp"
#include "lqt_internal.hpp"

namespace lqt {
namespace {

constexpr int NM = 16;      // largest state size
constexpr int kTile = kEltTile;  // element tile (blocks per tile of the element layout)
#define WDEV __device__ __forceinline__

WDEV int lane_id() { return threadIdx.x & 63; }
// A workgroup barrier.  Most kernels run one wavefront per workgroup; the two-wave tree kernels
// (kw_vreduce2, kw_vdown2) have both of their waves pass the same number of these.
WDEV void wsync() { __syncthreads(); }

WDEV int pk(int i, int j, int n) {  // packed upper index
  if (i > j) {
    int t = i;
    i = j;
    j = t;
  }
  return i * n - (i * (i - 1)) / 2 + (j - i);
}

// 16 x 16 FP64 products on the matrix cores: v_mfma_f64_16x16x4f64 takes A(i, k0 + q) and
// B(k0 + q, j) from lane 16 q + i (resp. 16 q + j) and returns C(q + 4 r, j) in register r of lane
// 16 q + j.  One instruction per 4 steps of the inner dimension; the operands come straight from
// LDS, so a 16^3 product costs 8 LDS reads per lane instead of 128.
typedef double wd4 __attribute__((ext_vector_type(4)));

WDEV void w_gemm16(double* C, const double* A, const double* B, int kk, bool tA, bool tB,
                   double alpha, double beta) {
  const int l = lane_id(), li = l & 15, lq = l >> 4;
  wd4 acc = {0.0, 0.0, 0.0, 0.0};
  for (int k0 = 0; k0 < kk; k0 += 4) {
    const int k = k0 + lq;
    const double a = tA ? A[k * 16 + li] : A[li * kk + k];
    const double b = tB ? B[li * kk + k] : B[k * 16 + li];
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
  }
  wsync();  // C may be an operand
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int e = (lq + 4 * r) * 16 + li;
    C[e] = beta == 0.0 ? alpha * acc[r] : fma(beta, C[e], alpha * acc[r]);
  }
  wsync();
}

// Whether the kernels of state size N use the matrix cores for their 16 x 16 products.
template <int N, class R>
constexpr bool kMfma = N == 16 && sizeof(R) == 8;

// C = alpha * op(A) (op(B) + addI I) + beta * D for a 16 x 16 result with row strides ldc, lda,
// ldb, ldd (op(A)(i, k) = tA ? A[k lda + i] : A[i lda + k], likewise B; D nullable, may be C).
// LDS banks: the 16 lanes of an operand read hold 16 rows i (A) or columns j (B) of one k, so A
// with tA and B without tB are read from consecutive addresses; A without tA (a column of a
// row-major matrix, stride 16 values) puts the 16 lanes on one bank pair.  Symmetric left
// factors are therefore passed with tA, general ones transposed beforehand.
WDEV void w_mm16(double* C, int ldc, const double* A, int lda, bool tA, const double* B, int ldb,
                 bool tB, int kk, double alpha, const double* D, int ldd, double beta,
                 bool addI = false) {
  const int l = lane_id(), li = l & 15, lq = l >> 4;
  wd4 acc = {0.0, 0.0, 0.0, 0.0};
  for (int k0 = 0; k0 < kk; k0 += 4) {
    const int k = k0 + lq;
    const double a = tA ? A[k * lda + li] : A[li * lda + k];
    const double b = (tB ? B[li * ldb + k] : B[k * ldb + li]) + (addI && k == li ? 1.0 : 0.0);
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
  }
  wsync();  // C may be an operand
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int i = lq + 4 * r;
    double v = alpha * acc[r];
    if (D) v = fma(beta, D[i * ldd + li], v);
    C[i * ldc + li] = v;
  }
  wsync();
}

// M (16 x 16, row-major) <- its upper triangle mirrored, plus the upper triangle of `add`.
WDEV void w_symadd16(double* M, const double* add) {
  double t[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const int e = lane_id() + 64 * c, i = e >> 4, j = e & 15;
    const int u = i < j ? i * 16 + j : j * 16 + i;
    t[c] = M[u] + add[u];
  }
  wsync();
#pragma unroll
  for (int c = 0; c < 4; ++c) M[lane_id() + 64 * c] = t[c];
  wsync();
}

// C = alpha * op(A) op(B) + beta * C for n x n (or m x p) matrices in LDS, row-major, ld = cols.
// MF: 16 x 16 FP64 products (inner dimension a multiple of 4) go to the matrix cores.
template <bool MF = false, class R>
WDEV void w_gemm(R* C, const R* A, const R* B, int m, int kk, int p, bool tA, bool tB, R alpha,
                 R beta) {
  if constexpr (MF && sizeof(R) == 8) {
    if (m == 16 && p == 16 && (kk & 3) == 0) {
      w_gemm16((double*)C, (const double*)A, (const double*)B, kk, tA, tB, alpha, beta);
      return;
    }
  }
  for (int e = lane_id(); e < m * p; e += 64) {
    const int i = e / p, j = e % p;
    R s = R(0);
    for (int k = 0; k < kk; ++k) {
      const R a = tA ? A[k * m + i] : A[i * kk + k];
      const R b = tB ? B[j * kk + k] : B[k * p + j];
      s = fma(a, b, s);
    }
    C[e] = beta == R(0) ? alpha * s : fma(beta, C[e], alpha * s);
  }
  wsync();
}

template <class R>
WDEV void w_copy(R* dst, const R* src, int n) {
  for (int e = lane_id(); e < n; e += 64) dst[e] = src[e];
  wsync();
}

template <class R>
WDEV void w_fill(R* dst, R v, int n) {
  for (int e = lane_id(); e < n; e += 64) dst[e] = v;
  wsync();
}

// Lane exchange through DPP (a VALU operand modifier: no LDS round trip): CTRL is the DPP control
// (0xB1 / 0x4E: xor 1 / xor 2 inside each quad; 0x141: mirror inside each half-row of 8 lanes;
// 0x140: mirror inside each row of 16 lanes).
template <int CTRL>
WDEV int w_dpp(int x) {
  return __builtin_amdgcn_update_dpp(x, x, CTRL, 0xF, 0xF, false);
}
template <int CTRL>
WDEV float w_dpp(float x) {
  return __builtin_bit_cast(float, w_dpp<CTRL>(__builtin_bit_cast(int, x)));
}
template <int CTRL>
WDEV double w_dpp(double x) {
  const long long b = __builtin_bit_cast(long long, x);
  const int lo = w_dpp<CTRL>((int)b), hi = w_dpp<CTRL>((int)(b >> 32));
  return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned)lo);
}

// (v, ix) <- the largest v of the RP consecutive lanes of this lane's group (RP = 8 or 16, groups
// aligned), the smallest ix among equal v; every lane of the group ends with the same pair.
template <int CTRL, class R>
WDEV void w_argmax_step(R& v, int& ix) {
  const R vo = w_dpp<CTRL>(v);
  const int io = w_dpp<CTRL>(ix);
  const bool take = (vo > v) | ((vo == v) & (io < ix));  // selects, no branch
  v = take ? vo : v;
  ix = take ? io : ix;
}
template <int RP, class R>
WDEV void w_argmax(R& v, int& ix) {
  w_argmax_step<0xB1>(v, ix);
  w_argmax_step<0x4E>(v, ix);
  w_argmax_step<0x141>(v, ix);
  if constexpr (RP == 16) w_argmax_step<0x140>(v, ix);
}

WDEV double w_readlane(double x, int lane) {
  const long long b = __builtin_bit_cast(long long, x);
  const int lo = __builtin_amdgcn_readlane((int)b, lane);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
  return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned)lo);
}
WDEV float w_readlane(float x, int lane) {
  return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, x), lane));
}

// Solve M X = B in place (B <- M^{-1} B), M N x N, B N x NB with NB <= 2 N + 1, by
// Gauss-Jordan elimination with partial pivoting (the row of largest magnitude among those not yet
// used as pivots, the first one on ties).  The system lives in registers: row i of [M | B]
// belongs to the lanes i + RP c0 (RP = 8 or 16 rows, padded; phase c0 = 0 .. LP - 1 holds columns
// c0, c0 + LP, ..., LP = 64 / RP), so the candidates of a column sit in RP consecutive lanes and
// the pivot search is a DPP reduction; the pivot's index and value reach every lane by readlane.
// Pivoting is implicit: rows stay in place and each remembers the column it was the pivot of,
// which places its solution row at the end.  Per pivot one LDS broadcast of the pivot row and of
// column c, alternating between two buffers of kSolveBuf values so that one barrier per pivot
// suffices, then a branch-free update of every lane's columns (scale the pivot row by 1 / pivot,
// subtract f_i times it from every other row, as in the textbook elimination).  Buffers: M's
// storage, and B's when it holds kSolveBuf values, else M + kSolveBuf (then M must have room for
// two buffers; both are no larger than n^2).  M is destroyed.
template <int N, int NB>
struct WSolveDims {
  static constexpr int RP = N <= 8 ? 8 : 16;
  static constexpr int LP = 64 / RP;
  static constexpr int NT = (N + NB + LP - 1) / LP;  // column slots per lane
  static constexpr int buf = LP * NT + N;  // pivot row (LP NT slots), then column c (N)
  static_assert(buf <= N * N, "a broadcast buffer fits in M");
};

// NB: the number of right-hand columns (2 N + 1 for a combination, N + 1 for a fold, 1 for a
// state), a compile-time constant so that each lane carries only the column slots in use.
template <int N, int NB, class R>
WDEV void w_solve(R* M, R* B) {
  using D = WSolveDims<N, NB>;
  constexpr int RP = D::RP, LP = D::LP, NT = D::NT;
  constexpr int nb = NB, W = N + NB;
  const int l = lane_id(), i = l % RP, c0 = l / RP;
  R x[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const int j = c0 + LP * t;
    const bool in = i < N && j < W;
    const R* src = !in ? M : (j < N ? M + i * N + j : B + i * nb + (j - N));
    const R a = *src;
    x[t] = in ? a : R(0);
  }
  wsync();  // M's and B's storage become the broadcast buffers
  R* const buf0 = M;
  R* const buf1 = N * nb >= D::buf ? B : M + D::buf;
  int mycol = -1;  // the column this lane's row was the pivot of
#pragma unroll
  for (int c = 0; c < N; ++c) {
    const int tc = c / LP, cc = c % LP;
    R* const rowc = (c & 1) ? buf1 : buf0;
    R* const fcol = rowc + LP * NT;
    R v = c0 == cc && i < N && mycol < 0 ? fabs(x[tc]) : R(-1);
    int ix = i;
    w_argmax<RP>(v, ix);
    const int p = __builtin_amdgcn_readlane(ix, cc * RP);  // the group of phase cc holds column c
    const R inv = R(1) / w_readlane(x[tc], p + cc * RP);
    if (i == p) {
      mycol = c;
#pragma unroll
      for (int t = 0; t < NT; ++t) rowc[c0 + LP * t] = x[t];  // slots j >= W hold zeros
    }
    if (c0 == cc && i < N) fcol[i] = x[tc];
    wsync();
    const R f = fcol[i < N ? i : 0];
    R r[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) r[t] = rowc[c0 + LP * t];
    // Every slot is updated: columns <= c of M are not read again, slots j >= W stay zero (the
    // pivot row's are zero) and padding rows are never pivots or written out.
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      const R rj = r[t] * inv;
      x[t] = i == p ? rj : fma(-f, rj, x[t]);
    }
  }
  wsync();  // the last broadcast may have used B's storage
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const int j = c0 + LP * t;
    if (i < N && mycol >= 0 && j >= N && j < W) B[mycol * nb + (j - N)] = x[t];
  }
  wsync();
}

// Tuple in LDS: A (= A - I, full), b, C (full symmetric), e, J (full symmetric).
template <class R>
struct WT {
  R *A, *b, *C, *e, *J;
};

template <class R>
WDEV WT<R> wt_at(R* base, int n) {  // 3 n^2 + 2 n values
  WT<R> t;
  t.A = base;
  t.b = base + n * n;
  t.C = t.b + n;
  t.e = t.C + n * n;
  t.J = t.e + n;
  return t;
}
__host__ __device__ inline int wt_size(int n) { return 3 * n * n + 2 * n; }
__host__ __device__ inline int ne_w(int n) { return 2 * n * n + 3 * n; }

// A tuple in global memory: value q at g[q * st] (st = 1 for tree nodes, kTile for elements).
template <class R>
struct GRef {
  R* g;
  long st;
};

// Element k of problem p in the tiled element layout (tiles of kTile blocks, value-major inside a
// tile, block k at column 64 (k % 8) + (k % 512) / 8).
template <class R>
WDEV GRef<R> elt_ref(R* elts, int p, long k, long T, int NE) {
  const long nt = (T + kTile - 1) / kTile;
  return {elts + ((p * nt + k / kTile) * NE) * kTile + ((k & 7) << 6) + ((k & 511) >> 3), kTile};
}
template <class R>
WDEV GRef<R> rec_ref(R* rec, int p, long k, long n, int NE) {
  return {rec + ((long)p * n + k) * NE, 1};
}

// Acc (coherent.hpp): the access policy of the global side.
template <class Acc = PlainAcc, class R>
WDEV void wt_load(WT<R> t, GRef<const R> g, int n) {
  const int ns = n * (n + 1) / 2;
  const int oB = n * n, oC = oB + n, oE = oC + ns, oJ = oE + n;
  for (int e = lane_id(); e < n * n; e += 64) {
    const int i = e / n, j = e % n;
    t.A[e] = Acc::ld(g.g + e * g.st);
    t.C[e] = Acc::ld(g.g + (oC + pk(i, j, n)) * g.st);
    t.J[e] = Acc::ld(g.g + (oJ + pk(i, j, n)) * g.st);
  }
  for (int i = lane_id(); i < n; i += 64) {
    t.b[i] = Acc::ld(g.g + (oB + i) * g.st);
    t.e[i] = Acc::ld(g.g + (oE + i) * g.st);
  }
  wsync();
}

template <class Acc = PlainAcc, class R>
WDEV void wt_store(WT<R> t, GRef<R> g, int n) {
  const int ns = n * (n + 1) / 2;
  const int oB = n * n, oC = oB + n, oE = oC + ns, oJ = oE + n;
  for (int e = lane_id(); e < n * n; e += 64) {
    const int i = e / n, j = e % n;
    Acc::st(g.g + e * g.st, t.A[e]);
    if (i <= j) {
      Acc::st(g.g + (oC + pk(i, j, n)) * g.st, t.C[e]);
      Acc::st(g.g + (oJ + pk(i, j, n)) * g.st, t.J[e]);
    }
  }
  for (int i = lane_id(); i < n; i += 64) {
    Acc::st(g.g + (oB + i) * g.st, t.b[i]);
    Acc::st(g.g + (oE + i) * g.st, t.e[i]);
  }
  wsync();
}

template <class R>
WDEV void wt_identity(WT<R> t, int n) {
  for (int e = lane_id(); e < n * n; e += 64) t.A[e] = t.C[e] = t.J[e] = R(0);
  for (int i = lane_id(); i < n; i += 64) t.b[i] = t.e[i] = R(0);
  wsync();
}

// Scratch of a combination / fold: 4 n^2 + n (2 n + 1) + 2 n values.
template <class R>
struct WS {
  R *M, *B, *X, *Y, *f;
  int* piv;
};

// Lemma 7 in the deviation form of the per-lane path: o = x1 (x) x2 (o may alias x2).
template <int N, class R>
WDEV void w_combine(WT<R> x1, WT<R> x2, WT<R> o, WS<R> s, int n) {
  const int nb = 2 * n + 1;
  // Ad2^T for the matrix-core products (after the n values of f, inside the scratch)
  R* At = s.f + 2 * n;
  // M = I + C1 J2; B = [Ad1 - C1 J2 | C1 | b1 + C1 eta2]  (C1 symmetric: read by columns)
  w_gemm<kMfma<N, R>>(s.X, x1.C, x2.J, n, n, n, kMfma<N, R>, false, R(1), R(0));
  for (int e = lane_id(); e < n * n; e += 64) {
    const int i = e / n, j = e % n;
    s.M[e] = (i == j ? R(1) : R(0)) + s.X[e];
    s.B[i * nb + j] = x1.A[e] - s.X[e];
    s.B[i * nb + n + j] = x1.C[e];
    if constexpr (kMfma<N, R>) At[j * n + i] = x2.A[e];
  }
  for (int i = lane_id(); i < n; i += 64) {
    R g = x1.b[i];
    for (int k = 0; k < n; ++k) g = fma(x1.C[k * n + i], x2.e[k], g);
    s.B[i * nb + 2 * n] = g;
  }
  wsync();
  w_solve<N, 2 * N + 1>(s.M, s.B);
  if constexpr (kMfma<N, R>) {
    // The same products on the matrix cores; every result goes to scratch first (o may be x2).
    // W = (I + Ad2) D is formed transposed (W^T = D^T (I + Ad2^T)) so that both of its products
    // read their left factor by columns.
    const int l = lane_id();
    w_mm16(s.X, 16, s.B + n, nb, true, At, 16, false, 16, 1.0, nullptr, 16, 0.0, true);  // W^T
    w_mm16(s.Y, 16, s.X, 16, true, At, 16, false, 16, 1.0, nullptr, 16, 0.0, true);  // W (I + Ad2)^T
    w_symadd16(s.Y, x2.C);                                                           // C
    R bn = R(0), en = R(0);
    if (l < n) {
      R t = R(0);
      for (int k = 0; k < n; ++k) t = fma(At[k * n + l], s.B[k * nb + 2 * n], t);
      bn = x2.b[l] + s.B[l * nb + 2 * n] + t;
      R u = x2.e[l];
      for (int k = 0; k < n; ++k) u = fma(-x2.J[k * n + l], x1.b[k], u);
      s.f[l] = u;
    }
    w_mm16(s.X, 16, x2.J, 16, true, x1.A, 16, false, 16, 1.0, x2.J, 16, 1.0);  // P
    w_mm16(s.M, 16, s.B, nb, true, s.X, 16, false, 16, 1.0, s.X, 16, 1.0);    // (I + Yd)^T P
    w_symadd16(s.M, x1.J);                                                     // J
    w_mm16(s.X, 16, At, 16, true, s.B, nb, false, 16, 1.0, s.B, nb, 1.0);     // Yd + Ad2 Yd
    if (l < n) {
      R t = R(0);
      for (int k = 0; k < n; ++k) t = fma(s.B[k * nb + l], s.f[k], t);
      en = x1.e[l] + (s.f[l] + t);
    }
    wsync();
    for (int e = l; e < n * n; e += 64) {
      o.J[e] = s.M[e];
      o.A[e] = x2.A[e] + s.X[e];
      o.C[e] = s.Y[e];
    }
    if (l < n) {
      o.b[l] = bn;
      o.e[l] = en;
    }
    wsync();
    return;
  }
  // W = (I + Ad2) D -> X;  C = W (I + Ad2)^T + C2 -> Y
  for (int e = lane_id(); e < n * n; e += 64) {
    const int i = e / n, j = e % n;
    R t = s.B[i * nb + n + j];
    for (int k = 0; k < n; ++k) t = fma(x2.A[i * n + k], s.B[k * nb + n + j], t);
    s.X[e] = t;
  }
  wsync();
  for (int e = lane_id(); e < n * n; e += 64) {
    const int i = e / n, j = e % n;
    const int a = i < j ? i : j, bb = i < j ? j : i;  // symmetric: compute the upper entry
    R t = s.X[a * n + bb];
    for (int l = 0; l < n; ++l) t = fma(s.X[a * n + l], x2.A[bb * n + l], t);
    s.Y[e] = x2.C[a * n + bb] + t;
  }
  // b = g + Ad2 g + b2 -> f (n values beyond piv scratch use)
  wsync();
  R bn = R(0), en = R(0);
  const int i = lane_id();
  if (i < n) {
    R t = R(0);
    for (int k = 0; k < n; ++k) t = fma(x2.A[i * n + k], s.B[k * nb + 2 * n], t);
    bn = x2.b[i] + s.B[i * nb + 2 * n] + t;
  }
  // w = eta2 - J2 b1 -> f
  if (i < n) {
    R t = x2.e[i];
    for (int k = 0; k < n; ++k) t = fma(-x2.J[i * n + k], x1.b[k], t);
    s.f[i] = t;
  }
  wsync();
  if (i < n) {
    R t = R(0);
    for (int k = 0; k < n; ++k) t = fma(s.B[k * nb + i], s.f[k], t);
    en = x1.e[i] + (s.f[i] + t);
  }
  // P = J2 (I + Ad1) -> X
  wsync();
  for (int e = lane_id(); e < n * n; e += 64) {
    const int r = e / n, j = e % n;
    R t = x2.J[e];
    for (int k = 0; k < n; ++k) t = fma(x2.J[r * n + k], x1.A[k * n + j], t);
    s.X[e] = t;
  }
  wsync();
  // J = (I + Yd)^T P + J1 (upper entry mirrored);  Ad = Ad2 + Yd + Ad2 Yd -> M
  R jn[4], an[4];
  int cnt = 0;
  for (int e = lane_id(); e < n * n; e += 64, ++cnt) {
    const int r = e / n, j = e % n;
    const int a = r < j ? r : j, bb = r < j ? j : r;
    R t = s.X[a * n + bb];
    for (int k = 0; k < n; ++k) t = fma(s.B[k * nb + a], s.X[k * n + bb], t);
    jn[cnt] = x1.J[a * n + bb] + t;
    R u = R(0);
    for (int k = 0; k < n; ++k) u = fma(x2.A[r * n + k], s.B[k * nb + j], u);
    an[cnt] = x2.A[e] + s.B[r * nb + j] + u;
  }
  wsync();
  cnt = 0;
  for (int e = lane_id(); e < n * n; e += 64, ++cnt) {
    o.J[e] = jn[cnt];
    o.A[e] = an[cnt];
    o.C[e] = s.Y[e];
  }
  if (i < n) {
    o.b[i] = bn;
    o.e[i] = en;
  }
  wsync();
}

// Fold with a terminal-form right operand: (S, v) <- a (x) (S, v); also the block map
// (P = Psi - I, q = alpha) into P, q (nullable).  S full symmetric.
template <int N, class R>
WDEV void w_fold(WT<R> a, R* S, R* v, WS<R> s, int n, R* P, R* q) {
  const int nb = n + 1;
  // C and S are symmetric: the left factors and the vector products read them by columns
  w_gemm<kMfma<N, R>>(s.X, a.C, S, n, n, n, kMfma<N, R>, false, R(1), R(0));  // C S
  for (int e = lane_id(); e < n * n; e += 64) {
    const int i = e / n, j = e % n;
    s.M[e] = (i == j ? R(1) : R(0)) + s.X[e];
    s.B[i * nb + j] = a.A[e] - s.X[e];
  }
  for (int i = lane_id(); i < n; i += 64) {
    R g = a.b[i];
    for (int k = 0; k < n; ++k) g = fma(a.C[k * n + i], v[k], g);
    s.B[i * nb + n] = g;
  }
  wsync();
  w_solve<N, N + 1>(s.M, s.B);
  if (P) {
    for (int e = lane_id(); e < n * n; e += 64) P[e] = s.B[(e / n) * nb + e % n];
    for (int i = lane_id(); i < n; i += 64) q[i] = s.B[i * nb + n];
  }
  // w = v - S b -> f;  X = S (I + Ad) -> X
  for (int i = lane_id(); i < n; i += 64) {
    R t = v[i];
    for (int k = 0; k < n; ++k) t = fma(-S[k * n + i], a.b[k], t);
    s.f[i] = t;
  }
  if constexpr (kMfma<N, R>) {
    w_mm16(s.X, 16, S, 16, true, a.A, 16, false, 16, 1.0, S, 16, 1.0);      // S (I + Ad)
    w_mm16(s.M, 16, s.B, nb, true, s.X, 16, false, 16, 1.0, s.X, 16, 1.0);  // (I + Yd)^T X
    w_symadd16(s.M, a.J);
    const int i = lane_id();
    R vn = R(0);
    if (i < n) {
      R t = R(0);
      for (int k = 0; k < n; ++k) t = fma(s.B[k * nb + i], s.f[k], t);
      vn = a.e[i] + (s.f[i] + t);
    }
    wsync();
    for (int e = i; e < n * n; e += 64) S[e] = s.M[e];
    if (i < n) v[i] = vn;
    wsync();
    return;
  }
  for (int e = lane_id(); e < n * n; e += 64) {
    const int i = e / n, j = e % n;
    R t = S[e];
    for (int k = 0; k < n; ++k) t = fma(S[i * n + k], a.A[k * n + j], t);
    s.X[e] = t;
  }
  wsync();
  R sn[4], vn = R(0);
  int cnt = 0;
  for (int e = lane_id(); e < n * n; e += 64, ++cnt) {
    const int r = e / n, j = e % n;
    const int aa = r < j ? r : j, bb = r < j ? j : r;
    R t = R(0);
    for (int k = 0; k < n; ++k) t = fma(s.B[k * nb + aa], s.X[k * n + bb], t);
    sn[cnt] = a.J[aa * n + bb] + (s.X[aa * n + bb] + t);
  }
  const int i = lane_id();
  if (i < n) {
    R t = R(0);
    for (int k = 0; k < n; ++k) t = fma(s.B[k * nb + i], s.f[k], t);
    vn = a.e[i] + (s.f[i] + t);
  }
  wsync();
  cnt = 0;
  for (int e = lane_id(); e < n * n; e += 64, ++cnt) S[e] = sn[cnt];
  if (i < n) v[i] = vn;
  wsync();
}

// Block map only: (P, q) from (Ad, b, C) of a block and (S, v) at its right end.
template <int N, class R>
WDEV void w_block_map(WT<R> a, const R* S, const R* v, WS<R> s, int n, R* P, R* q) {
  const int nb = n + 1;
  w_gemm<kMfma<N, R>>(s.X, a.C, S, n, n, n, kMfma<N, R>, false, R(1), R(0));
  for (int e = lane_id(); e < n * n; e += 64) {
    const int i = e / n, j = e % n;
    s.M[e] = (i == j ? R(1) : R(0)) + s.X[e];
    s.B[i * nb + j] = a.A[e] - s.X[e];
  }
  for (int i = lane_id(); i < n; i += 64) {
    R g = a.b[i];
    for (int k = 0; k < n; ++k) g = fma(a.C[k * n + i], v[k], g);
    s.B[i * nb + n] = g;
  }
  wsync();
  w_solve<N, N + 1>(s.M, s.B);
  for (int e = lane_id(); e < n * n; e += 64) P[e] = s.B[(e / n) * nb + e % n];
  for (int i = lane_id(); i < n; i += 64) q[i] = s.B[i * nb + n];
  wsync();
}

// Affine maps (P = Psi - I, q): acc <- later o acc.  tmp: n^2 + n.
template <class R>
WDEV void w_aff_then(R* aP, R* aq, const R* lP, const R* lq, R* tmp, int n) {
  for (int e = lane_id(); e < n * n; e += 64) {
    const int i = e / n, j = e % n;
    R t = R(0);
    for (int k = 0; k < n; ++k) t = fma(lP[i * n + k], aP[k * n + j], t);
    tmp[e] = aP[e] + lP[e] + t;
  }
  for (int i = lane_id(); i < n; i += 64) {
    R t = R(0);
    for (int k = 0; k < n; ++k) t = fma(lP[i * n + k], aq[k], t);
    tmp[n * n + i] = lq[i] + aq[i] + t;
  }
  wsync();
  for (int e = lane_id(); e < n * n; e += 64) aP[e] = tmp[e];
  for (int i = lane_id(); i < n; i += 64) aq[i] = tmp[n * n + i];
  wsync();
}

// acc <- acc o earlier
template <class R>
WDEV void w_aff_after(R* aP, R* aq, const R* eP, const R* eq, R* tmp, int n) {
  for (int e = lane_id(); e < n * n; e += 64) {
    const int i = e / n, j = e % n;
    R t = R(0);
    for (int k = 0; k < n; ++k) t = fma(aP[i * n + k], eP[k * n + j], t);
    tmp[e] = eP[e] + aP[e] + t;
  }
  for (int i = lane_id(); i < n; i += 64) {
    R t = R(0);
    for (int k = 0; k < n; ++k) t = fma(aP[i * n + k], eq[k], t);
    tmp[n * n + i] = aq[i] + eq[i] + t;
  }
  wsync();
  for (int e = lane_id(); e < n * n; e += 64) aP[e] = tmp[e];
  for (int i = lane_id(); i < n; i += 64) aq[i] = tmp[n * n + i];
  wsync();
}

// x <- x + P x + q (x, tmp in LDS)
template <class R>
WDEV void w_aff_apply(const R* P, const R* q, R* x, R* tmp, int n) {
  for (int i = lane_id(); i < n; i += 64) {
    R t = R(0);
    for (int k = 0; k < n; ++k) t = fma(P[i * n + k], x[k], t);
    tmp[i] = x[i] + (t + q[i]);
  }
  wsync();
  for (int i = lane_id(); i < n; i += 64) x[i] = tmp[i];
  wsync();
}

template <class R>
WDEV void w_aff_identity(R* P, R* q, int n) {
  for (int e = lane_id(); e < n * n; e += 64) P[e] = R(0);
  for (int i = lane_id(); i < n; i += 64) q[i] = R(0);
  wsync();
}

template <class R>
WDEV WS<R> ws_at(R* base, int* piv, int n) {
  WS<R> s;
  s.M = base;
  s.X = s.M + n * n;
  s.Y = s.X + n * n;
  s.B = s.Y + n * n;
  s.f = s.B + n * (2 * n + 1);
  s.piv = piv;
  return s;
}

// ------------------------------------------------------------------------------------------
// Element build (Theorem 8), one wave per block: RK4 on the full matrices.
// ------------------------------------------------------------------------------------------
// Separator element of ragged mode after problem i (see KProb): A - I = -I, b = x0 of problem
// i + 1 (0 after the last), C = 0, eta = Qf_i rf_i, J = Qf_i.
template <class R>
WDEV void w_separator(const KProb& kp, int i, WT<R> y, int n) {
  const R* Qf = (const R*)kp.Qf + (long)i * n * n;
  const R* rf = (const R*)kp.rf + (long)i * n;
  const bool last = i + 1 >= kp.nseg;
  for (int e = lane_id(); e < n * n; e += 64) {
    const int a = e / n, b = e % n;
    y.A[e] = a == b ? R(-1) : R(0);
    y.C[e] = R(0);
    y.J[e] = Qf[(a < b ? a : b) * n + (a < b ? b : a)];
  }
  for (int a = lane_id(); a < n; a += 64) {
    y.b[a] = last ? R(0) : ((const R*)kp.x0)[(long)(i + 1) * n + a];
    R s = R(0);
    for (int b = 0; b < n; ++b) s = fma(Qf[a * n + b], rf[b], s);
    y.e[a] = s;
  }
  wsync();
}

// Where block k's data sits: problem p, sample offset s0 (sample j of the block at
// s0 + 2 n k + j), left end t[tk], constant F of problem pf.
struct WBlk {
  int p;
  long s0, tk, pf;
};

WDEV WBlk wblk_plain(const KProb& kp, int p, long k) {
  return {p, (long)p * (2L * kp.n * kp.T + 1), (long)p * (kp.T + 1) + k, 0};
}

// Scratch of a one-wave element build beside its three tuples: 8 n^2 + 5 n values.
template <int N>
constexpr int kBuildScr = 8 * N * N + 5 * N;

// The last `nsteps` RK4 steps of Theorem 8 on block k, backward from t_{k+1}: y holds the
// element of [t_{k+1} - m h, t_{k+1}] after step m (start from the identity for a full build).
// ac and st are tuple scratch, scr kBuildScr<N> values.  IMP: the reference is the unit impulse
// at sample imp_j of the problem, component imp_i, instead of the problem's r (the
// time-invariant path tabulates the response of b and eta to each sample this way).
template <int N, class R, bool IMP = false>
WDEV void wb_bwd_steps(const KProb& kp, const WBlk& bk, long k, int nsteps, WT<R> y, WT<R> ac,
                       WT<R> st, R* scr, long imp_j = -1, int imp_i = 0) {
  constexpr int NM = N;
  constexpr int n = N;
  const int nu = kp.nu;
  const int nn = kp.n;
  const int p = bk.p;
  const long s0 = bk.s0, tk = bk.tk, pf = bk.pf;
  const R* t = (const R*)kp.t + tk;
  const R* r = (const R*)kp.r;
  const R* Fc = (const R*)kp.F + pf * n * n;  // constant F (per problem when ragged)
  const R* cb = kp.has_c ? (const R*)kp.c : nullptr;
  const R* Qp = (const R*)kp.Q + (long)p * n * n;
  const R* cs = (const R*)kp.consts + (long)p * consts_count(n, nu);
  R* F = scr;
  R* G = F + NM * NM;
  R* K = G + NM * NM;
  R* Lc = K + NM * NM;  // n x nu
  R* T1 = Lc + NM * NM;
  R* kA = T1 + NM * NM;
  R* kC = kA + NM * NM;
  R* kJ = kC + NM * NM;
  R* kb = kJ + NM * NM;
  R* ke = kb + NM;
  R* rv = ke + NM;
  R* cv = rv + NM;
  const R h = (t[1] - t[0]) / R(nn);
  for (int m = 0; m < nsteps; ++m) {
    const long j1 = 2L * nn * k + 2L * (nn - m);
    w_copy(st.A, y.A, n * n);
    w_copy(st.e, y.e, n);
    w_copy(st.J, y.J, n * n);
    for (int s = 0; s < 4; ++s) {
      const long j = s == 0 ? j1 : (s == 3 ? j1 - 2 : j1 - 1);
      const R wk = (s == 0 || s == 3) ? -h / R(6) : -h / R(3);
      const R cn = s == 2 ? -h : -h / R(2);
      const R* Fj = kp.F_sampled ? (const R*)kp.F + (s0 + j) * n * n : Fc;
      for (int e = lane_id(); e < n * n; e += 64) F[e] = Fj[e];
      for (int i = lane_id(); i < n; i += 64) {
        rv[i] = IMP ? (j == imp_j && i == imp_i ? R(1) : R(0)) : r[(s0 + j) * n + i];
        cv[i] = cb ? cb[(s0 + j) * n + i] : R(0);
      }
      if (kp.L_sampled) {
        const R* Lj = (const R*)kp.L + (s0 + j) * n * nu;
        const R* W = cs + consts_off_W(n, nu);
        for (int e = lane_id(); e < n * nu; e += 64) {
          const int i = e / nu, l = e % nu;
          R a = R(0);
          for (int q2 = 0; q2 < nu; ++q2) a = fma(Lj[i * nu + q2], W[q2 * nu + l], a);
          Lc[e] = a;
        }
        wsync();
        w_gemm<kMfma<N, R>>(G, Lc, Lc, n, nu, n, false, true, R(1), R(0));
      } else {
        for (int e = lane_id(); e < n * n; e += 64) G[e] = cs[consts_off_G(n, nu) + e];
        for (int e = lane_id(); e < n * nu; e += 64) Lc[e] = cs[consts_off_Lc(n, nu) + e];
        wsync();
      }
      // K = G J - F
      for (int e = lane_id(); e < n * n; e += 64) K[e] = -F[e];
      wsync();
      w_gemm<kMfma<N, R>>(K, G, st.J, n, n, n, false, false, R(1), R(1));
      // kA = K + Ad K
      w_copy(kA, K, n * n);
      w_gemm<kMfma<N, R>>(kA, st.A, K, n, n, n, false, false, R(1), R(1));
      // kb = -(I + Ad)(G eta + c)
      for (int i = lane_id(); i < n; i += 64) {
        R a = cv[i];
        for (int l = 0; l < n; ++l) a = fma(G[i * n + l], st.e[l], a);
        T1[i] = a;
      }
      wsync();
      for (int i = lane_id(); i < n; i += 64) {
        R a = T1[i];
        for (int l = 0; l < n; ++l) a = fma(st.A[i * n + l], T1[l], a);
        kb[i] = -a;
      }
      // kC = -(A Lc)(A Lc)^T with A Lc = Lc + Ad Lc -> T1 (n x nu)
      wsync();
      w_copy(T1, Lc, n * nu);
      w_gemm<kMfma<N, R>>(T1, st.A, Lc, n, n, nu, false, false, R(1), R(1));
      w_gemm<kMfma<N, R>>(kC, T1, T1, n, nu, n, false, true, R(-1), R(0));
      // ke = K^T eta + J c - Q r
      for (int i = lane_id(); i < n; i += 64) {
        R a = R(0);
        for (int l = 0; l < n; ++l) {
          a = fma(K[l * n + i], st.e[l], a);
          a = fma(st.J[i * n + l], cv[l], a);
          a = fma(-Qp[i * n + l], rv[l], a);
        }
        ke[i] = a;
      }
      // kJ = -Q + J K - F^T J (symmetrised from the upper entry)
      if constexpr (N == 16 && sizeof(R) == 8) {
        wsync();  // ke has read K before the products below run
        w_gemm<kMfma<N, R>>(kJ, st.J, K, n, n, n, false, false, R(1), R(0));
        w_gemm<kMfma<N, R>>(kJ, F, st.J, n, n, n, true, false, R(-1), R(1));
        R v[4];
        int cnt = 0;
        for (int e = lane_id(); e < n * n; e += 64, ++cnt) {
          const int i = e / n, q2 = e % n;
          const int a = i < q2 ? i : q2, bb = i < q2 ? q2 : i;
          v[cnt] = kJ[a * n + bb] - Qp[a * n + bb];
        }
        wsync();
        cnt = 0;
        for (int e = lane_id(); e < n * n; e += 64, ++cnt) kJ[e] = v[cnt];
      } else {
        for (int e = lane_id(); e < n * n; e += 64) {
          const int i = e / n, q2 = e % n;
          const int a = i < q2 ? i : q2, bb = i < q2 ? q2 : i;
          R v = -Qp[a * n + bb];
          for (int l = 0; l < n; ++l) {
            v = fma(st.J[a * n + l], K[l * n + bb], v);
            v = fma(-F[l * n + a], st.J[l * n + bb], v);
          }
          kJ[e] = v;
        }
      }
      wsync();
      // accumulate and form the next stage input
      for (int e = lane_id(); e < n * n; e += 64) {
        ac.A[e] = s == 0 ? fma(wk, kA[e], y.A[e]) : fma(wk, kA[e], ac.A[e]);
        ac.J[e] = s == 0 ? fma(wk, kJ[e], y.J[e]) : fma(wk, kJ[e], ac.J[e]);
        y.C[e] = fma(wk, kC[e], y.C[e]);
        if (s < 3) {
          st.A[e] = fma(cn, kA[e], y.A[e]);
          st.J[e] = fma(cn, kJ[e], y.J[e]);
        }
      }
      for (int i = lane_id(); i < n; i += 64) {
        ac.e[i] = s == 0 ? fma(wk, ke[i], y.e[i]) : fma(wk, ke[i], ac.e[i]);
        y.b[i] = fma(wk, kb[i], y.b[i]);
        if (s < 3) st.e[i] = fma(cn, ke[i], y.e[i]);
      }
      wsync();
    }
    w_copy(y.A, ac.A, n * n);
    w_copy(y.e, ac.e, n);
    w_copy(y.J, ac.J, n * n);
  }
}

template <int N, class R>
__global__ __launch_bounds__(64) void kw_build(const KProb kp, R* __restrict__ elts) {
  constexpr int kTupW = 3 * N * N + 2 * N;
  __shared__ R sh[3 * kTupW + kBuildScr<N>];
  constexpr int n = N;
  const long T = kp.T;
  const long k = blockIdx.x;
  WBlk bk = wblk_plain(kp, blockIdx.y, k);
  WT<R> y = wt_at(sh, n), ac = wt_at(sh + kTupW, n), st = wt_at(sh + 2 * kTupW, n);
  if (kp.seg) {
    const int p = seg_find(kp.seg, kp.nseg, k);
    if (k == kp.seg[p + 1] - 1 || k == T - 1) {
      w_separator(kp, p, y, n);
      wt_store(y, elt_ref(elts, 0, k, T, ne_w(n)), n);
      return;
    }
    bk = {p, (long)p * (1 - 2L * kp.n), k, p};
  }
  wt_identity(y, n);
  wb_bwd_steps<N, R>(kp, bk, k, kp.n, y, ac, st, sh + 3 * kTupW);
  wt_store(y, elt_ref(elts, kp.seg ? 0 : bk.p, k, T, ne_w(n)), n);
}

// ------------------------------------------------------------------------------------------
// Time-invariant path (F, L constant, c = 0, uniform grid).  The RK4 recursion of Theorem 8 for
// A, C, J does not involve r, so every block has the same A, C, J, and b, eta are linear in the
// block's samples r_0 .. r_2n: b = sum_j V_j r_j, eta = sum_j W_j r_j.  kw_lti_prep integrates
// block 0 once per unit impulse (sample j0, component i0; one wave each) to tabulate column i0 of
// V_j0 and W_j0, and A, C, J; kw_build_lti forms every block's element from the table.
// Table of a problem: A - I (n^2, full), C and J (packed upper, the element's order), then
// V_0 .. V_2n and W_0 .. W_2n (n^2 each, row-major).
// ------------------------------------------------------------------------------------------
template <int N, class R>
__global__ __launch_bounds__(64) void kw_lti_prep(const KProb kp, R* __restrict__ tab) {
  constexpr int n = N, kTupW = 3 * N * N + 2 * N, ns = N * (N + 1) / 2;
  __shared__ R sh[3 * kTupW + kBuildScr<N>];
  const int p = blockIdx.y;
  const long m = blockIdx.x;
  const long j0 = m / n;
  const int i0 = (int)(m % n);
  WT<R> y = wt_at(sh, n), ac = wt_at(sh + kTupW, n), st = wt_at(sh + 2 * kTupW, n);
  wt_identity(y, n);
  wb_bwd_steps<N, R, true>(kp, wblk_plain(kp, p, 0), 0, kp.n, y, ac, st, sh + 3 * kTupW, j0, i0);
  R* tp = tab + (long)p * lti_count(n, kp.n);
  R* V = tp + lti_off_V(n) + j0 * n * n;
  R* W = tp + lti_off_W(n, kp.n) + j0 * n * n;
  for (int a = lane_id(); a < n; a += 64) {
    V[a * n + i0] = y.b[a];
    W[a * n + i0] = y.e[a];
  }
  if (m == 0) {
    for (int e = lane_id(); e < n * n; e += 64) {
      const int i = e / n, j = e % n;
      tp[e] = y.A[e];
      if (i <= j) {
        tp[n * n + pk(i, j, n)] = y.C[e];
        tp[n * n + ns + pk(i, j, n)] = y.J[e];
      }
    }
  }
}

// One wave per block: A, C, J copied from the table, b and eta summed over the block's samples
// (lane 2 a + w: row a of V (w = 0) or W (w = 1)).
template <int N, class R>
__global__ __launch_bounds__(64) void kw_build_lti(const KProb kp, const R* __restrict__ tab,
                                                   R* __restrict__ elts) {
  constexpr int n = N, ns = N * (N + 1) / 2;
  const int p = blockIdx.y;
  const long k = blockIdx.x;
  const int nn = kp.n;
  const long T = kp.T;
  const R* tp = tab + (long)p * lti_count(n, nn);
  const GRef<R> g = elt_ref(elts, p, k, T, ne_w(n));
  const int oB = n * n, oC = oB + n, oE = oC + ns, oJ = oE + n;
  for (int q = lane_id(); q < n * n + 2 * ns; q += 64) {
    const int dst = q < n * n ? q : (q < n * n + ns ? oC + (q - n * n) : oJ + (q - n * n - ns));
    g.g[dst * g.st] = tp[q];
  }
  const int l = lane_id();
  if (l < 2 * n) {
    const int a = l >> 1, w = l & 1;
    const R* Mt = tp + (w ? lti_off_W(n, nn) : lti_off_V(n)) + a * n;
    const R* rp = (const R*)kp.r + ((long)p * (2L * nn * T + 1) + 2L * nn * k) * n;
    R acc = R(0);
    for (int j = 0; j <= 2 * nn; ++j)
      for (int i = 0; i < n; ++i) acc = fma(Mt[(long)j * n * n + i], rp[j * n + i], acc);
    g.g[((w ? oE : oB) + a) * g.st] = acc;
  }
}

// ------------------------------------------------------------------------------------------
// Element build from the forward conditional ODEs (Theorem 9, Sec. IV-C), one wave per block:
// with M = F - C Q and A = I + Ad, dAd/dtau = M + M Ad, db/dtau = M b + (F - M) r + c and
// dC/dtau = G + M C + C F^T, integrated by RK4 forward in tau from t_k; eta and J enter no
// right-hand side, so their increments w + Ad^T w (w = Q (r - b)) and P + Ad^T P
// (P = Q (I + Ad)) are added to them directly.  Samples: stage 1 at 2 n k + 2 m, stages 2 and 3
// at + 1, stage 4 at + 2.  Full matrices in LDS as in the Theorem 8 build; C and J take their
// upper entries after every stage (the exact derivatives are symmetric).
// ------------------------------------------------------------------------------------------
// The first `nsteps` steps of block k: y holds the element of [t_k, t_k + m h] after step m
// (start from the identity).  ac and st are tuple scratch (their e and J unused), scr
// kBuildScr<N> values.
// EJ = false leaves eta and J alone (the state formula of Method 2 needs A, b, C only); step(m)
// runs after step m, with y holding the parts on [t_k, t_k + (m + 1) h].
struct WNoStep {
  WDEV void operator()(int) const {}
};

template <int N, class R, bool EJ = true, class STEP = WNoStep>
WDEV void wb_fwd_steps(const KProb& kp, const WBlk& bk, long k, int nsteps, WT<R> y, WT<R> ac,
                       WT<R> st, R* scr, const STEP& step = STEP{}) {
  constexpr int n = N;
  const int nu = kp.nu;
  const int nn = kp.n;
  const int p = bk.p;
  const long s0 = bk.s0;
  const R* t = (const R*)kp.t + bk.tk;
  const R* r = (const R*)kp.r;
  const R* Fc = (const R*)kp.F + bk.pf * n * n;
  const R* cb = kp.has_c ? (const R*)kp.c : nullptr;
  const R* Qp = (const R*)kp.Q + (long)p * n * n;
  const R* cs = (const R*)kp.consts + (long)p * consts_count(n, nu);
  R* F = scr;
  R* G = F + N * N;
  R* Lc = G + N * N;  // n x nu
  R* Qs = Lc + N * N;
  R* M = Qs + N * N;
  R* P = M + N * N;
  R* kC = P + N * N;
  R* X = kC + N * N;  // kJ, then kA
  R* rv = X + N * N;
  R* cv = rv + N;
  R* wv = cv + N;
  R* kb = wv + N;
  R* ke = kb + N;
  for (int e = lane_id(); e < n * n; e += 64) Qs[e] = Qp[e];
  if (!kp.L_sampled) {
    for (int e = lane_id(); e < n * n; e += 64) G[e] = cs[consts_off_G(n, nu) + e];
  }
  wsync();
  const R h = (t[1] - t[0]) / R(nn);
  for (int m = 0; m < nsteps; ++m) {
    const long j0 = 2L * nn * k + 2L * m;
    w_copy(st.A, y.A, n * n);
    w_copy(st.b, y.b, n);
    w_copy(st.C, y.C, n * n);
    for (int s = 0; s < 4; ++s) {
      const long j = s == 0 ? j0 : (s == 3 ? j0 + 2 : j0 + 1);
      const R wk = (s == 0 || s == 3) ? h / R(6) : h / R(3);
      const R cn = s == 2 ? h : h / R(2);
      const R* Fj = kp.F_sampled ? (const R*)kp.F + (s0 + j) * n * n : Fc;
      for (int e = lane_id(); e < n * n; e += 64) F[e] = Fj[e];
      for (int i = lane_id(); i < n; i += 64) {
        rv[i] = r[(s0 + j) * n + i];
        cv[i] = cb ? cb[(s0 + j) * n + i] : R(0);
      }
      if (kp.L_sampled) {
        const R* Lj = (const R*)kp.L + (s0 + j) * n * nu;
        const R* W = cs + consts_off_W(n, nu);
        for (int e = lane_id(); e < n * nu; e += 64) {
          const int i = e / nu, l = e % nu;
          R a = R(0);
          for (int q2 = 0; q2 < nu; ++q2) a = fma(Lj[i * nu + q2], W[q2 * nu + l], a);
          Lc[e] = a;
        }
        wsync();
        w_gemm<kMfma<N, R>>(G, Lc, Lc, n, nu, n, false, true, R(1), R(0));
      } else {
        wsync();
      }
      // M = F - C Q
      w_copy(M, F, n * n);
      w_gemm<kMfma<N, R>>(M, st.C, Qs, n, n, n, false, false, R(-1), R(1));
      if constexpr (EJ) {
        // eta increment: w = Q (r - b), w + Ad^T w
        for (int i = lane_id(); i < n; i += 64) {
          R a = R(0);
          for (int l = 0; l < n; ++l) a = fma(Qs[i * n + l], rv[l] - st.b[l], a);
          wv[i] = a;
        }
        wsync();
        for (int i = lane_id(); i < n; i += 64) {
          R a = wv[i];
          for (int l = 0; l < n; ++l) a = fma(st.A[l * n + i], wv[l], a);
          ke[i] = a;
        }
        // J increment: P = Q + Q Ad, P + Ad^T P
        w_copy(P, Qs, n * n);
        w_gemm<kMfma<N, R>>(P, Qs, st.A, n, n, n, false, false, R(1), R(1));
        w_copy(X, P, n * n);
        w_gemm<kMfma<N, R>>(X, st.A, P, n, n, n, true, false, R(1), R(1));
        for (int e = lane_id(); e < n * n; e += 64) {
          const int i = e / n, q2 = e % n;
          y.J[e] = fma(wk, X[(i < q2 ? i : q2) * n + (i < q2 ? q2 : i)], y.J[e]);
        }
        for (int i = lane_id(); i < n; i += 64) y.e[i] = fma(wk, ke[i], y.e[i]);
      }
      // kb = M b + (F - M) r + c
      for (int i = lane_id(); i < n; i += 64) {
        R a = cv[i];
        for (int l = 0; l < n; ++l) {
          a = fma(M[i * n + l], st.b[l], a);
          a = fma(F[i * n + l] - M[i * n + l], rv[l], a);
        }
        kb[i] = a;
      }
      // kC = G + M C + C F^T
      w_copy(kC, G, n * n);
      w_gemm<kMfma<N, R>>(kC, M, st.C, n, n, n, false, false, R(1), R(1));
      w_gemm<kMfma<N, R>>(kC, st.C, F, n, n, n, false, true, R(1), R(1));
      // kA = M + M Ad
      w_copy(X, M, n * n);
      w_gemm<kMfma<N, R>>(X, M, st.A, n, n, n, false, false, R(1), R(1));
      // accumulate and form the next stage input
      for (int e = lane_id(); e < n * n; e += 64) {
        const int i = e / n, q2 = e % n;
        const R c = kC[(i < q2 ? i : q2) * n + (i < q2 ? q2 : i)];
        ac.A[e] = s == 0 ? fma(wk, X[e], y.A[e]) : fma(wk, X[e], ac.A[e]);
        ac.C[e] = s == 0 ? fma(wk, c, y.C[e]) : fma(wk, c, ac.C[e]);
        if (s < 3) {
          st.A[e] = fma(cn, X[e], y.A[e]);
          st.C[e] = fma(cn, c, y.C[e]);
        }
      }
      for (int i = lane_id(); i < n; i += 64) {
        ac.b[i] = s == 0 ? fma(wk, kb[i], y.b[i]) : fma(wk, kb[i], ac.b[i]);
        if (s < 3) st.b[i] = fma(cn, kb[i], y.b[i]);
      }
      wsync();
    }
    w_copy(y.A, ac.A, n * n);
    w_copy(y.b, ac.b, n);
    w_copy(y.C, ac.C, n * n);
    step(m);
  }
}

template <int N, class R>
__global__ __launch_bounds__(64) void kw_build_fwd(const KProb kp, R* __restrict__ elts) {
  constexpr int kTupW = 3 * N * N + 2 * N;
  __shared__ R sh[3 * kTupW + kBuildScr<N>];
  const long k = blockIdx.x;
  const WBlk bk = wblk_plain(kp, blockIdx.y, k);
  WT<R> y = wt_at(sh, N), ac = wt_at(sh + kTupW, N), st = wt_at(sh + 2 * kTupW, N);
  wt_identity(y, N);
  wb_fwd_steps<N, R>(kp, bk, k, kp.n, y, ac, st, sh + 3 * kTupW);
  wt_store(y, elt_ref(elts, bk.p, k, kp.T, ne_w(N)), N);
}

// ------------------------------------------------------------------------------------------
// Element build with every block split at tau = t_k + floor(n/2) h (Sec. IV-D): Theorem 9 gives
// the element of [t_k, tau], Theorem 8 that of [tau, t_{k+1}], and Lemma 7 joins them.  One wave
// per block does the two parts one after the other: with a wave per block the launch already
// holds T waves, so the halved span of a block buys no occupancy here; the total work is that
// of a full build plus one combination.
// ------------------------------------------------------------------------------------------
template <int N, class R>
__global__ __launch_bounds__(64) void kw_build_split(const KProb kp, R* __restrict__ elts) {
  constexpr int kTupW = 3 * N * N + 2 * N;
  static_assert(4 * N * N + N * (2 * N + 1) + 2 * N <= kBuildScr<N>, "combination scratch");
  __shared__ R sh[4 * kTupW + kBuildScr<N>];
  __shared__ int piv[N];
  const long k = blockIdx.x;
  const int m = kp.n / 2;
  const WBlk bk = wblk_plain(kp, blockIdx.y, k);
  WT<R> f = wt_at(sh, N), y = wt_at(sh + kTupW, N), ac = wt_at(sh + 2 * kTupW, N),
        st = wt_at(sh + 3 * kTupW, N);
  R* scr = sh + 4 * kTupW;
  wt_identity(f, N);
  wt_identity(y, N);
  wb_fwd_steps<N, R>(kp, bk, k, m, f, ac, st, scr);
  wb_bwd_steps<N, R>(kp, bk, k, kp.n - m, y, ac, st, scr);
  w_combine<N>(f, y, y, ws_at(scr, piv, N), N);
  wt_store(y, elt_ref(elts, bk.p, k, kp.T, ne_w(N)), N);
}

// ------------------------------------------------------------------------------------------
// Element build for nx <= 8 with 8 blocks per wave: lane 8 g + i owns row i of every matrix of
// block 8 w + g (A - I, C, J rows, b_i, eta_i) in registers, with its rows of G, Q, F and F^T.
// The products of a stage need other rows of J, K, Lc and A Lc, and the vectors eta and G eta + c;
// each group publishes them in its own LDS area (rows padded to nx + 1 values, so the 8 rows of a
// group sit in different banks) and reads them back after a barrier: three barriers per stage
// for 8 blocks, and each LDS read serves the 8 lanes of a group at once.  Same RK4 recursion of
// Theorem 8 as the per-lane path; J and C are symmetrised from their upper entries after every
// step.
// ------------------------------------------------------------------------------------------
template <int N, class R>
__global__ __launch_bounds__(64) void kw_build_rows(const KProb kp, R* __restrict__ elts) {
  static_assert(N <= 8, "8 lanes per block");
  constexpr int P = N + 1;  // padded row length in LDS
  __shared__ R sJ[8][8 * P], sK[8][8 * P], sL[8][8 * P], sAL[8][8 * P], se[8][8], sw[8][8];
  const int lane = lane_id(), g = lane >> 3, i = lane & 7;
  const int nu = kp.nu;
  const long T = kp.T;
  const int nn = kp.n;
  const long k = (long)blockIdx.x * 8 + g;
  const bool row = i < N;
  bool live = k < T;
  bool sep = false;
  int p = blockIdx.y;
  long s0 = (long)p * (2L * nn * T + 1), tk = (long)p * (T + 1) + k, pf = 0;
  if (kp.seg && live) {
    p = seg_find(kp.seg, kp.nseg, k);
    sep = k == kp.seg[p + 1] - 1 || k == T - 1;
    s0 = (long)p * (1 - 2L * nn);
    tk = k;
    pf = p;
  }
  const bool work = live && !sep;  // this group integrates a block
  const bool act = work && row;    // this lane owns a row of it
  const R* cs = (const R*)kp.consts + (long)p * consts_count(N, nu);
  const R* Qp = (const R*)kp.Q + (long)p * N * N;
  const R* Fc = (const R*)kp.F + pf * N * N;
  // constant rows: G_i, Q_i, F_i, (F^T)_i, Lc_i
  R Gr[N], Qr[N], Fr[N], Fk[N], Lr[N];
#pragma unroll
  for (int q = 0; q < N; ++q) {
    Gr[q] = act ? cs[consts_off_G(N, nu) + i * N + q] : R(0);
    Qr[q] = act ? Qp[i * N + q] : R(0);
    Fr[q] = act ? Fc[i * N + q] : R(0);
    Fk[q] = act ? Fc[q * N + i] : R(0);
    Lr[q] = act && q < nu ? cs[consts_off_Lc(N, nu) + i * nu + q] : R(0);
  }
  const R* W = cs + consts_off_W(N, nu);
  R yA[N], yJ[N], yC[N], aA[N], aJ[N], tA[N], tJ[N];
  R ye = R(0), yb = R(0), ae = R(0), te = R(0);
#pragma unroll
  for (int q = 0; q < N; ++q) yA[q] = yJ[q] = yC[q] = R(0);
  const R h = work ? (((const R*)kp.t)[tk + 1] - ((const R*)kp.t)[tk]) / R(nn) : R(0);
  if (!kp.L_sampled) {
#pragma unroll
    for (int q = 0; q < N; ++q) sL[g][i * P + q] = Lr[q];
  }
  for (int m = 0; m < nn; ++m) {
    const long j1 = 2L * nn * k + 2L * (nn - m);
#pragma unroll
    for (int q = 0; q < N; ++q) {
      tA[q] = yA[q];
      tJ[q] = yJ[q];
    }
    te = ye;
    for (int st = 0; st < 4; ++st) {
      const long j = st == 0 ? j1 : (st == 3 ? j1 - 2 : j1 - 1);
      const R wk = (st == 0 || st == 3) ? -h / R(6) : -h / R(3);
      const R cn = st == 2 ? -h : -h / R(2);
      R rv[N], cv[N];
#pragma unroll
      for (int q = 0; q < N; ++q) {
        rv[q] = act ? ((const R*)kp.r)[(s0 + j) * N + q] : R(0);
        cv[q] = act && kp.has_c ? ((const R*)kp.c)[(s0 + j) * N + q] : R(0);
      }
      if (kp.F_sampled) {
        const R* Fj = (const R*)kp.F + (s0 + j) * N * N;
#pragma unroll
        for (int q = 0; q < N; ++q) {
          Fr[q] = act ? Fj[i * N + q] : R(0);
          Fk[q] = act ? Fj[q * N + i] : R(0);
        }
      }
      if (kp.L_sampled) {  // Lc = L(t_j) W, G = Lc Lc^T
        const R* Lj = (const R*)kp.L + (s0 + j) * N * nu;
#pragma unroll
        for (int l = 0; l < N; ++l) {
          R a = R(0);
          if (act && l < nu)
            for (int q = 0; q < nu; ++q) a = fma(Lj[i * nu + q], W[q * nu + l], a);
          Lr[l] = a;
          sL[g][i * P + l] = a;
        }
        wsync();
#pragma unroll
        for (int q = 0; q < N; ++q) {
          R a = R(0);
#pragma unroll
          for (int l = 0; l < N; ++l) a = fma(Lr[l], sL[g][q * P + l], a);
          Gr[q] = a;
        }
      }
      // publish the stage's J row and eta_i
#pragma unroll
      for (int q = 0; q < N; ++q) sJ[g][i * P + q] = tJ[q];
      se[g][i] = te;
      wsync();
      // K_i = G_i J - F_i;  w_i = G_i eta + c_i
      R K[N];
#pragma unroll
      for (int q = 0; q < N; ++q) {
        R a = -Fr[q];
#pragma unroll
        for (int l = 0; l < N; ++l) a = fma(Gr[l], sJ[g][l * P + q], a);
        K[q] = a;
      }
      R w = row ? cv[i] : R(0);
#pragma unroll
      for (int l = 0; l < N; ++l) w = fma(Gr[l], se[g][l], w);
#pragma unroll
      for (int q = 0; q < N; ++q) sK[g][i * P + q] = K[q];
      sw[g][i] = w;
      wsync();
      // kA_i = K_i + (Ad)_i K;  kb_i = -(w_i + (Ad)_i w);  (A Lc)_i = Lc_i + (Ad)_i Lc
      R kA[N], AL[N], kJ[N];
#pragma unroll
      for (int q = 0; q < N; ++q) {
        R a = K[q];
#pragma unroll
        for (int l = 0; l < N; ++l) a = fma(tA[l], sK[g][l * P + q], a);
        kA[q] = a;
      }
      R kb = w;
#pragma unroll
      for (int l = 0; l < N; ++l) kb = fma(tA[l], sw[g][l], kb);
      kb = -kb;
#pragma unroll
      for (int q = 0; q < N; ++q) {
        R a = Lr[q];
#pragma unroll
        for (int l = 0; l < N; ++l) a = fma(tA[l], sL[g][l * P + q], a);
        AL[q] = q < nu ? a : R(0);
        sAL[g][i * P + q] = AL[q];
      }
      // ke_i = (K^T eta)_i + J_i c - Q_i r;  kJ_i = -Q_i + J_i K - (F^T)_i J
      R ke = R(0);
#pragma unroll
      for (int l = 0; l < N; ++l) {
        ke = fma(sK[g][l * P + i], se[g][l], ke);
        if (kp.has_c) ke = fma(tJ[l], cv[l], ke);
        ke = fma(-Qr[l], rv[l], ke);
      }
#pragma unroll
      for (int q = 0; q < N; ++q) {
        R a = -Qr[q];
#pragma unroll
        for (int l = 0; l < N; ++l) {
          a = fma(tJ[l], sK[g][l * P + q], a);
          a = fma(-Fk[l], sJ[g][l * P + q], a);
        }
        kJ[q] = a;
      }
      wsync();
      // kC_i = -(A Lc)_i (A Lc)^T
#pragma unroll
      for (int q = 0; q < N; ++q) {
        R a = R(0);
#pragma unroll
        for (int l = 0; l < N; ++l) a = fma(AL[l], sAL[g][q * P + l], a);
        yC[q] = fma(-wk, a, yC[q]);
      }
      yb = fma(wk, kb, yb);
#pragma unroll
      for (int q = 0; q < N; ++q) {
        aA[q] = st == 0 ? fma(wk, kA[q], yA[q]) : fma(wk, kA[q], aA[q]);
        aJ[q] = st == 0 ? fma(wk, kJ[q], yJ[q]) : fma(wk, kJ[q], aJ[q]);
        if (st < 3) {
          tA[q] = fma(cn, kA[q], yA[q]);
          tJ[q] = fma(cn, kJ[q], yJ[q]);
        }
      }
      ae = st == 0 ? fma(wk, ke, ye) : fma(wk, ke, ae);
      if (st < 3) te = fma(cn, ke, ye);
    }
    // end of step: new start value; J and C take their upper entries
#pragma unroll
    for (int q = 0; q < N; ++q) {
      yA[q] = aA[q];
      sJ[g][i * P + q] = aJ[q];
      sK[g][i * P + q] = yC[q];
    }
    ye = ae;
    wsync();
#pragma unroll
    for (int q = 0; q < N; ++q) {
      yJ[q] = q < i ? sJ[g][q * P + i] : aJ[q];
      yC[q] = q < i ? sK[g][q * P + i] : yC[q];
    }
    wsync();
  }
  if (!live || !row) return;
  const GRef<R> o = elt_ref(elts, kp.seg ? 0 : p, k, T, ne_w(N));
  const int ns = N * (N + 1) / 2;
  const int oB = N * N, oC = oB + N, oE = oC + ns, oJ = oE + N;
  if (sep) {  // separator after problem p (see KProb): A - I = -I, b = next x0, C = 0
    const R* Qf = (const R*)kp.Qf + (long)p * N * N;
    const R* rf = (const R*)kp.rf + (long)p * N;
    const bool last = p + 1 >= kp.nseg;
    R e = R(0);
#pragma unroll
    for (int q = 0; q < N; ++q) {
      o.g[(i * N + q) * o.st] = q == i ? R(-1) : R(0);
      e = fma(Qf[i * N + q], rf[q], e);
      if (q >= i) {
        o.g[(oC + pk(i, q, N)) * o.st] = R(0);
        o.g[(oJ + pk(i, q, N)) * o.st] = Qf[i * N + q];
      }
    }
    o.g[(oB + i) * o.st] = last ? R(0) : ((const R*)kp.x0)[(long)(p + 1) * N + i];
    o.g[(oE + i) * o.st] = e;
    return;
  }
#pragma unroll
  for (int q = 0; q < N; ++q) {
    o.g[(i * N + q) * o.st] = yA[q];
    if (q >= i) {
      o.g[(oC + pk(i, q, N)) * o.st] = yC[q];
      o.g[(oJ + pk(i, q, N)) * o.st] = yJ[q];
    }
  }
  o.g[(oB + i) * o.st] = yb;
  o.g[(oE + i) * o.st] = ye;
}

// ------------------------------------------------------------------------------------------
// Element build for nx <= 8 in FP64 on the matrix cores, two blocks per wave.  A 16 x 16 product
// tile of v_mfma_f64_16x16x4f64 takes the two blocks' left factors stacked (rows 8 b + i) and
// their right factors side by side (columns 8 b + j), so its diagonal 8 x 8 blocks are the two
// blocks' products (the off-diagonal blocks mix the two and are not used).  In the result layout
// (lane 16 q + j holds entries (q + 4 r, j)) the lanes of columns 8 b .. 8 b + 7 hold rows q and
// q + 4 of block b in registers r = 2 b and 2 b + 1, so every state matrix of the RK4 recursion
// (A - I, J: start, stage, accumulator; C: accumulator) is two registers per lane with nothing
// wasted; only operands pass through LDS (rows padded).  Entries beyond nx are zero throughout.
// Same arithmetic as kw_build_mfma16 (K = G J - F, kA = K + A K, kJ = -Q + J K - F^T J,
// kC = -(A Lc)(A Lc)^T, Theorem 8 with K factored out), two barriers per stage.
// ------------------------------------------------------------------------------------------
template <int N>
__global__ __launch_bounds__(64, 3) void kw_build_mfma8(const KProb kp, double* __restrict__ elts) {
  static_assert(N <= 8, "two blocks of at most 8 states per 16 x 16 tile");
  constexpr int XP = 9, YP = 17;  // padded row lengths: stacked (16 x 8), side by side (8 x 16)
  typedef double R;
  // left factors stacked [16][XP], right factors side by side [8][YP]
  __shared__ R xA[16 * XP], xJ[16 * XP], xG[16 * XP], xFT[16 * XP], xAL[16 * XP];
  __shared__ R yJ[8 * YP], yK[8 * YP], yL[8 * YP], yALT[8 * YP];
  __shared__ R sF[16 * XP], sQ[16 * XP];  // F and Q of each block's problem (row 8 b + i)
  __shared__ R se[2][8], sw[2][8], sr[2][3][8], sc[2][3][8];  // samples: 3 per RK4 step
  const int lane = lane_id(), li = lane & 15, lq = lane >> 4;
  const int b = li >> 3, lj = li & 7;  // block of this lane's columns, column inside the block
  const int nu = kp.nu;
  const long T = kp.T;
  const int nn = kp.n;
  // the two blocks of this wave and their problems
  long kb2[2], s0b[2], tkb[2];
  int pb[2];
  bool liveb[2], sepb[2];
  for (int c = 0; c < 2; ++c) {
    const long k = 2L * blockIdx.x + c;
    int p = blockIdx.y;
    long s0 = (long)p * (2L * nn * T + 1), tk = (long)p * (T + 1) + k;
    bool live = k < T, sep = false;
    if (kp.seg && live) {
      p = seg_find(kp.seg, kp.nseg, k);
      sep = k == kp.seg[p + 1] - 1 || k == T - 1;
      s0 = (long)p * (1 - 2L * nn);
      tk = k;
    }
    kb2[c] = k;
    s0b[c] = s0;
    tkb[c] = tk;
    pb[c] = p;
    liveb[c] = live;
    sepb[c] = sep;
  }
  const bool work0 = liveb[0] && !sepb[0], work1 = liveb[1] && !sepb[1];
  // per-block constants: G (stacked), F (rows 8 b + i), -F^T (stacked), Q, Lc (side by side)
  for (int e = lane; e < 2 * 64; e += 64) {
    const int c = e >> 6, i = (e >> 3) & 7, j = e & 7;
    const bool wk = c == 0 ? work0 : work1;
    const bool in = wk && i < N && j < N;
    const long pc = kp.seg ? pb[c] : 0;
    const R* cs = (const R*)kp.consts + (long)pb[c] * consts_count(N, nu);
    xG[(8 * c + i) * XP + j] = in ? cs[consts_off_G(N, nu) + i * N + j] : R(0);
    sQ[(8 * c + i) * XP + j] = in ? ((const R*)kp.Q)[(long)pb[c] * N * N + i * N + j] : R(0);
    if (!kp.F_sampled) {
      const R* Fc = (const R*)kp.F + pc * N * N;
      sF[(8 * c + i) * XP + j] = in ? Fc[i * N + j] : R(0);
      xFT[(8 * c + i) * XP + j] = in ? -Fc[j * N + i] : R(0);
    }
    yL[i * YP + 8 * c + j] = in && j < nu ? cs[consts_off_Lc(N, nu) + i * nu + j] : R(0);
  }
  const R h0 = work0 ? (((const R*)kp.t)[tkb[0] + 1] - ((const R*)kp.t)[tkb[0]]) / R(nn) : R(0);
  const R h1 = work1 ? (((const R*)kp.t)[tkb[1] + 1] - ((const R*)kp.t)[tkb[1]]) / R(nn) : R(0);
  const R h = b == 0 ? h0 : h1;  // (selects, not indexing: per-lane indices would go to scratch)
  // state: entries (lq + 4 s, lj) of block b in slot s
  R yAs[2], yJs[2], yCs[2], aAs[2], aJs[2], tAs[2], tJs[2];
#pragma unroll
  for (int t = 0; t < 2; ++t) yAs[t] = yJs[t] = yCs[t] = R(0);
  R ye = R(0), yb = R(0), ae = R(0), te = R(0);  // component lj of block b (all four lq alike)
  // Reference (and drift) samples of an RK4 step: lane L < 48 holds sample 2 n (k + 1) - 2 m - o
  // (o = (L % 24) / 8) component L % 8 of block L / 24; the next step's are loaded while the
  // current step runs, so only the first step waits for memory.
  const int pc_ = lane < 48 ? lane / 24 : 0, po = (lane % 24) / 8, pi = lane & 7;
  const bool pl = lane < 48 && (pc_ == 0 ? work0 : work1) && pi < N;
  const long sbase = (pc_ == 0 ? s0b[0] + 2L * nn * kb2[0] : s0b[1] + 2L * nn * kb2[1]) - po;
  auto sample_at = [&](int m, const void* arr) -> R {
    if (!pl || !arr) return R(0);
    return ((const R*)arr)[(sbase + 2L * (nn - m)) * N + pi];
  };
  R nr = sample_at(0, kp.r), ncv = sample_at(0, kp.has_c ? kp.c : nullptr);
  wsync();
  for (int m = 0; m < nn; ++m) {
    if (lane < 48) {
      sr[pc_][po][pi] = nr;
      sc[pc_][po][pi] = ncv;
    }
    if (m + 1 < nn) {
      nr = sample_at(m + 1, kp.r);
      ncv = sample_at(m + 1, kp.has_c ? kp.c : nullptr);
    }
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      tAs[t] = yAs[t];
      tJs[t] = yJs[t];
    }
    te = ye;
#pragma unroll
    for (int st = 0; st < 4; ++st) {
      const int jo = st == 0 ? 0 : (st == 3 ? 2 : 1);  // sample offset below 2 n (k + 1) - 2 m
      const R wk = (st == 0 || st == 3) ? -h / R(6) : -h / R(3);
      const R cn = st == 2 ? -h : -h / R(2);
      if (kp.F_sampled) {
        for (int e = lane; e < 2 * 64; e += 64) {
          const int c = e >> 6, i = (e >> 3) & 7, q = e & 7;
          const bool in = (c == 0 ? work0 : work1) && i < N && q < N;
          const long j = s0b[c] + 2L * nn * kb2[c] + 2L * (nn - m) - jo;
          const R* Fj = (const R*)kp.F + j * N * N;
          sF[(8 * c + i) * XP + q] = in ? Fj[i * N + q] : R(0);
          xFT[(8 * c + i) * XP + q] = in ? -Fj[q * N + i] : R(0);
        }
      }
      if (kp.L_sampled) {  // Lc = L(t_j) W (side by side), G = Lc Lc^T after the barrier
        for (int e = lane; e < 2 * 64; e += 64) {
          const int c = e >> 6, i = (e >> 3) & 7, l = e & 7;
          const bool in = (c == 0 ? work0 : work1) && i < N && l < nu;
          const long j = s0b[c] + 2L * nn * kb2[c] + 2L * (nn - m) - jo;
          const R* Lj = (const R*)kp.L + j * N * nu;
          const R* Wc = (const R*)kp.consts + (long)pb[c] * consts_count(N, nu) + consts_off_W(N, nu);
          R a = R(0);
          if (in)
            for (int q = 0; q < nu; ++q) a = fma(Lj[i * nu + q], Wc[q * nu + l], a);
          yL[i * YP + 8 * c + l] = a;
        }
      }
      // publish the stage values: A (left), J (left and right), eta
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        const int i = lq + 4 * t;
        xA[(8 * b + i) * XP + lj] = tAs[t];
        xJ[(8 * b + i) * XP + lj] = tJs[t];
        yJ[i * YP + li] = tJs[t];
      }
      if (lq == 0) se[b][lj] = te;
      wsync();
      if (kp.L_sampled) {
        for (int e = lane; e < 2 * 64; e += 64) {
          const int c = e >> 6, i = (e >> 3) & 7, q = e & 7;
          R a = R(0);
          for (int l = 0; l < nu; ++l) a = fma(yL[i * YP + 8 * c + l], yL[q * YP + 8 * c + l], a);
          xG[(8 * c + i) * XP + q] = a;
        }
        wsync();
      }
      // K = G J - F
      wd4 K;
#pragma unroll
      for (int r = 0; r < 4; ++r) K[r] = (r >> 1) == b ? -sF[(8 * b + lq + 4 * (r & 1)) * XP + lj] : R(0);
#pragma unroll
      for (int k0 = 0; k0 < 8; k0 += 4)
        K = __builtin_amdgcn_mfma_f64_16x16x4f64(xG[li * XP + k0 + lq], yJ[(k0 + lq) * YP + li], K, 0, 0, 0);
      // A Lc = Lc + (A - I) Lc
      wd4 ALc;
#pragma unroll
      for (int r = 0; r < 4; ++r)
        ALc[r] = (r >> 1) == b ? yL[(lq + 4 * (r & 1)) * YP + li] : R(0);
#pragma unroll
      for (int k0 = 0; k0 < 8; k0 += 4)
        ALc = __builtin_amdgcn_mfma_f64_16x16x4f64(xA[li * XP + k0 + lq], yL[(k0 + lq) * YP + li], ALc, 0, 0, 0);
      // w = G eta + c: lane 16 q + li sums terms 2 q, 2 q + 1 of component lj of block b
      R w = R(0);
#pragma unroll
      for (int t = 0; t < 2; ++t) w = fma(xG[(8 * b + lj) * XP + 2 * lq + t], se[b][2 * lq + t], w);
      w += __shfl_xor(w, 16);
      w += __shfl_xor(w, 32);
      w += sc[b][jo][lj];
      // publish K (right factor) and A Lc (left factor and its transpose as a right factor)
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        const int i = lq + 4 * t;
        const R kv = K[2 * b + t], av = ALc[2 * b + t];
        yK[i * YP + li] = kv;
        xAL[(8 * b + i) * XP + lj] = av;
        yALT[lj * YP + 8 * b + i] = av;
      }
      if (lq == 0) sw[b][lj] = w;
      wsync();
      // kA = K + (A - I) K
      wd4 kA = K;
#pragma unroll
      for (int k0 = 0; k0 < 8; k0 += 4)
        kA = __builtin_amdgcn_mfma_f64_16x16x4f64(xA[li * XP + k0 + lq], yK[(k0 + lq) * YP + li], kA, 0, 0, 0);
      // kJ = -Q + J K - F^T J
      wd4 kJ;
#pragma unroll
      for (int r = 0; r < 4; ++r) kJ[r] = (r >> 1) == b ? -sQ[(8 * b + lq + 4 * (r & 1)) * XP + lj] : R(0);
#pragma unroll
      for (int k0 = 0; k0 < 8; k0 += 4)
        kJ = __builtin_amdgcn_mfma_f64_16x16x4f64(xJ[li * XP + k0 + lq], yK[(k0 + lq) * YP + li], kJ, 0, 0, 0);
#pragma unroll
      for (int k0 = 0; k0 < 8; k0 += 4)
        kJ = __builtin_amdgcn_mfma_f64_16x16x4f64(xFT[li * XP + k0 + lq], yJ[(k0 + lq) * YP + li], kJ, 0, 0, 0);
      // kC = -(A Lc)(A Lc)^T (nu <= 4 columns: one k-slice)
      wd4 kC = {0.0, 0.0, 0.0, 0.0};
      kC = __builtin_amdgcn_mfma_f64_16x16x4f64(lq < nu ? xAL[li * XP + lq] : R(0),
                                                lq < nu ? yALT[lq * YP + li] : R(0), kC, 0, 0, 0);
      if (nu > 4)
        kC = __builtin_amdgcn_mfma_f64_16x16x4f64(4 + lq < nu ? xAL[li * XP + 4 + lq] : R(0),
                                                  4 + lq < nu ? yALT[(4 + lq) * YP + li] : R(0), kC, 0, 0, 0);
      // keta = K^T eta + J c - Q r;  kb = -(w + (A - I) w): component lj of block b, terms 2 q,
      // 2 q + 1 on lane 16 q + li, then a butterfly over q
      R ke = R(0), kbv = R(0);
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        const int q = 2 * lq + t;
        ke = fma(yK[q * YP + li], se[b][q], ke);
        if (kp.has_c) ke = fma(xJ[(8 * b + lj) * XP + q], sc[b][jo][q], ke);
        ke = fma(-sQ[(8 * b + lj) * XP + q], sr[b][jo][q], ke);
        kbv = fma(xA[(8 * b + lj) * XP + q], sw[b][q], kbv);
      }
      ke += __shfl_xor(ke, 16);
      ke += __shfl_xor(ke, 32);
      kbv += __shfl_xor(kbv, 16);
      kbv += __shfl_xor(kbv, 32);
      kbv = -(kbv + sw[b][lj]);
      // RK4 accumulation and the next stage value (this lane's block only)
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        const R ka = kA[2 * b + t], kj = kJ[2 * b + t], kc = kC[2 * b + t];
        aAs[t] = st == 0 ? fma(wk, ka, yAs[t]) : fma(wk, ka, aAs[t]);
        aJs[t] = st == 0 ? fma(wk, kj, yJs[t]) : fma(wk, kj, aJs[t]);
        yCs[t] = fma(-wk, kc, yCs[t]);
        if (st < 3) {
          tAs[t] = fma(cn, ka, yAs[t]);
          tJs[t] = fma(cn, kj, yJs[t]);
        }
      }
      ae = st == 0 ? fma(wk, ke, ye) : fma(wk, ke, ae);
      yb = fma(wk, kbv, yb);
      if (st < 3) te = fma(cn, ke, ye);
      wsync();  // the next stage overwrites the operand buffers
    }
    // end of step: J and C take their upper entries
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      const int i = lq + 4 * t;
      yAs[t] = aAs[t];
      yJ[i * YP + li] = aJs[t];
      yK[i * YP + li] = yCs[t];
    }
    ye = ae;
    wsync();
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      const int i = lq + 4 * t;
      yJs[t] = i > lj ? yJ[lj * YP + 8 * b + i] : aJs[t];
      yCs[t] = i > lj ? yK[lj * YP + 8 * b + i] : yCs[t];
    }
    wsync();
  }
  // outputs of this lane's block (separators write their fixed element)
  if (!liveb[b]) return;
  const int pbl = pb[b];
  const GRef<R> o = elt_ref(elts, kp.seg ? 0 : pbl, kb2[b], T, ne_w(N));
  constexpr int ns = N * (N + 1) / 2;
  constexpr int oB = N * N, oC = oB + N, oE = oC + ns, oJ = oE + N;
  if (sepb[b]) {  // separator after problem p (see KProb): A - I = -I, b = next x0, C = 0, J = Qf
    const R* Qf = (const R*)kp.Qf + (long)pbl * N * N;
    const R* rf = (const R*)kp.rf + (long)pbl * N;
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      const int i = lq + 4 * t;
      if (i < N && lj < N) {
        o.g[(i * N + lj) * o.st] = i == lj ? R(-1) : R(0);
        if (lj >= i) {
          o.g[(oC + pk(i, lj, N)) * o.st] = R(0);
          o.g[(oJ + pk(i, lj, N)) * o.st] = Qf[i * N + lj];
        }
      }
    }
    if (lq == 0 && lj < N) {
      R e = R(0);
      for (int q = 0; q < N; ++q) e = fma(Qf[lj * N + q], rf[q], e);
      o.g[(oB + lj) * o.st] = pbl + 1 >= kp.nseg ? R(0) : ((const R*)kp.x0)[(long)(pbl + 1) * N + lj];
      o.g[(oE + lj) * o.st] = e;
    }
    return;
  }
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    const int i = lq + 4 * t;
    if (i < N && lj < N) {
      o.g[(i * N + lj) * o.st] = yAs[t];
      if (lj >= i) {
        o.g[(oC + pk(i, lj, N)) * o.st] = yCs[t];
        o.g[(oJ + pk(i, lj, N)) * o.st] = yJs[t];
      }
    }
  }
  if (lq == 0 && lj < N) {
    o.g[(oB + lj) * o.st] = yb;
    o.g[(oE + lj) * o.st] = ye;
  }
}

// ------------------------------------------------------------------------------------------
// Element build at nx = 16 in FP64 on the matrix cores, one wave per block.  Every 16 x 16
// matrix of the RK4 state (A - I, J: start value, stage value, accumulator; C: accumulator) stays
// in registers in the result layout of v_mfma_f64_16x16x4f64 (lane 16 q + j holds entries
// (q + 4 r, j), r = 0..3); only the stage values of A, J and the stage's K go through LDS (rows
// padded to 17 values) to become matrix-core operands.  Per stage:
//   publish A, J, eta  | K = G J - F (MFMA from -F),  w = G eta + c,  (A Lc) = Lc + A Lc
//   publish K, w       | kA = K + A K,  kJ = -Q + J K - F^T J,  kC = -(A Lc)(A Lc)^T (MFMA),
//                      | keta = K^T eta + J c - Q r,  kb = -(w + A w); RK4 updates in registers.
// Two barriers per stage.  J and C take their upper entries after every step (as the oracle).
// ------------------------------------------------------------------------------------------
template <int DUMMY = 0>
__global__ __launch_bounds__(64) void kw_build_mfma16(const KProb kp, double* __restrict__ elts) {
  constexpr int N = 16, P = 17;
  typedef double R;
  __shared__ R sA[N * P], sJ[N * P], sK[N * P], sG[N * P], sF[N * P], sQ[N * P], sL[N * P],
      sAL[N * P];
  __shared__ R se[N], sw[N], sr[N], sc[N];
  const int lane = lane_id(), li = lane & 15, lq = lane >> 4;
  const int nu = kp.nu;
  const long T = kp.T;
  const int nn = kp.n;
  const long k = blockIdx.x;
  int p = blockIdx.y;
  long s0 = (long)p * (2L * nn * T + 1), tk = (long)p * (T + 1) + k, pf = 0;
  bool sep = false;
  if (kp.seg) {
    p = seg_find(kp.seg, kp.nseg, k);
    sep = k == kp.seg[p + 1] - 1 || k == T - 1;
    s0 = (long)p * (1 - 2L * nn);
    tk = k;
    pf = p;
  }
  const GRef<R> o = elt_ref(elts, kp.seg ? 0 : p, k, T, ne_w(N));
  const int ns = N * (N + 1) / 2;
  const int oB = N * N, oC = oB + N, oE = oC + ns, oJ = oE + N;
  if (sep) {  // separator after problem p (see KProb): A - I = -I, b = next x0, C = 0, J = Qf
    const R* Qf = (const R*)kp.Qf + (long)p * N * N;
    const R* rf = (const R*)kp.rf + (long)p * N;
    for (int e = lane; e < N * N; e += 64) {
      const int i = e / N, j = e % N;
      o.g[e * o.st] = i == j ? R(-1) : R(0);
      if (j >= i) {
        o.g[(oC + pk(i, j, N)) * o.st] = R(0);
        o.g[(oJ + pk(i, j, N)) * o.st] = Qf[i * N + j];
      }
    }
    if (lane < N) {
      R e = R(0);
      for (int q = 0; q < N; ++q) e = fma(Qf[lane * N + q], rf[q], e);
      o.g[(oB + lane) * o.st] = p + 1 >= kp.nseg ? R(0) : ((const R*)kp.x0)[(long)(p + 1) * N + lane];
      o.g[(oE + lane) * o.st] = e;
    }
    return;
  }
  const R* cs = (const R*)kp.consts + (long)p * consts_count(N, nu);
  const R* Qp = (const R*)kp.Q + (long)p * N * N;
  const R* Fc = (const R*)kp.F + pf * N * N;
  // per-block constants in LDS: G, Q, F (constant case), Lc
  for (int e = lane; e < N * N; e += 64) {
    const int i = e / N, j = e % N;
    sG[i * P + j] = cs[consts_off_G(N, nu) + e];
    sQ[i * P + j] = Qp[e];
    if (!kp.F_sampled) sF[i * P + j] = Fc[e];
  }
  for (int e = lane; e < N * nu; e += 64) sL[(e / nu) * P + e % nu] = cs[consts_off_Lc(N, nu) + e];
  const R* W = cs + consts_off_W(N, nu);
  const R h = (((const R*)kp.t)[tk + 1] - ((const R*)kp.t)[tk]) / R(nn);
  // state in the MFMA result layout: entry (lq + 4 r, li)
  R yA[4], yJ[4], yC[4], aA[4], aJ[4], tA[4], tJ[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) yA[r] = yJ[r] = yC[r] = R(0);
  R ye = R(0), yb = R(0), ae = R(0), te = R(0);  // lanes < 16: component li
  wsync();
  for (int m = 0; m < nn; ++m) {
    const long j1 = 2L * nn * k + 2L * (nn - m);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      tA[r] = yA[r];
      tJ[r] = yJ[r];
    }
    te = ye;
    for (int st = 0; st < 4; ++st) {
      const long j = st == 0 ? j1 : (st == 3 ? j1 - 2 : j1 - 1);
      const R wk = (st == 0 || st == 3) ? -h / R(6) : -h / R(3);
      const R cn = st == 2 ? -h : -h / R(2);
      // samples of this stage; stage values of A, J, eta as operands
      if (lane < N) {
        sr[lane] = ((const R*)kp.r)[(s0 + j) * N + lane];
        sc[lane] = kp.has_c ? ((const R*)kp.c)[(s0 + j) * N + lane] : R(0);
        se[lane] = te;
      }
      if (kp.F_sampled) {
        const R* Fj = (const R*)kp.F + (s0 + j) * N * N;
        for (int e = lane; e < N * N; e += 64) sF[(e / N) * P + e % N] = Fj[e];
      }
      if (kp.L_sampled) {  // Lc = L(t_j) W, G = Lc Lc^T
        const R* Lj = (const R*)kp.L + (s0 + j) * N * nu;
        for (int e = lane; e < N * nu; e += 64) {
          const int i = e / nu, l = e % nu;
          R a = R(0);
          for (int q = 0; q < nu; ++q) a = fma(Lj[i * nu + q], W[q * nu + l], a);
          sL[i * P + l] = a;
        }
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        sA[(lq + 4 * r) * P + li] = tA[r];
        sJ[(lq + 4 * r) * P + li] = tJ[r];
      }
      wsync();
      if (kp.L_sampled) {
        for (int e = lane; e < N * N; e += 64) {
          const int i = e / N, q = e % N;
          R a = R(0);
          for (int l = 0; l < nu; ++l) a = fma(sL[i * P + l], sL[q * P + l], a);
          sG[i * P + q] = a;
        }
        wsync();
      }
      // K = G J - F
      wd4 K;
#pragma unroll
      for (int r = 0; r < 4; ++r) K[r] = -sF[(lq + 4 * r) * P + li];
#pragma unroll
      for (int k0 = 0; k0 < N; k0 += 4) {
        const int kk = k0 + lq;
        K = __builtin_amdgcn_mfma_f64_16x16x4f64(sG[li * P + kk], sJ[kk * P + li], K, 0, 0, 0);
      }
      // w = G eta + c: lanes 16 q + i sum terms 4 q .. 4 q + 3 of component i, then a butterfly
      R w = R(0);
#pragma unroll
      for (int t = 0; t < 4; ++t) w = fma(sG[li * P + 4 * lq + t], se[4 * lq + t], w);
      w += __shfl_xor(w, 16);
      w += __shfl_xor(w, 32);
      w += sc[li];
      // A Lc = Lc + (A - I) Lc on the matrix cores (Lc padded to 16 columns with zeros)
      wd4 ALc;
#pragma unroll
      for (int r = 0; r < 4; ++r) ALc[r] = li < nu ? sL[(lq + 4 * r) * P + li] : R(0);
#pragma unroll
      for (int k0 = 0; k0 < N; k0 += 4) {
        const int kk = k0 + lq;
        ALc = __builtin_amdgcn_mfma_f64_16x16x4f64(sA[li * P + kk], li < nu ? sL[kk * P + li] : R(0),
                                                   ALc, 0, 0, 0);
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        sK[(lq + 4 * r) * P + li] = K[r];
        sAL[(lq + 4 * r) * P + li] = ALc[r];
      }
      if (lane < N) sw[lane] = w;
      wsync();
      // (A Lc)(li, 4 kb + lq): this lane's operand of both factors of -(A Lc)(A Lc)^T
      R AL[4];
#pragma unroll
      for (int kb = 0; kb < 4; ++kb) AL[kb] = 4 * kb + lq < nu ? sAL[li * P + 4 * kb + lq] : R(0);
      // kA = K + (A - I) K
      wd4 kA = K;
#pragma unroll
      for (int k0 = 0; k0 < N; k0 += 4) {
        const int kk = k0 + lq;
        kA = __builtin_amdgcn_mfma_f64_16x16x4f64(sA[li * P + kk], sK[kk * P + li], kA, 0, 0, 0);
      }
      // kJ = -Q + J K - F^T J
      wd4 kJ;
#pragma unroll
      for (int r = 0; r < 4; ++r) kJ[r] = -sQ[(lq + 4 * r) * P + li];
#pragma unroll
      for (int k0 = 0; k0 < N; k0 += 4) {
        const int kk = k0 + lq;
        kJ = __builtin_amdgcn_mfma_f64_16x16x4f64(sJ[li * P + kk], sK[kk * P + li], kJ, 0, 0, 0);
      }
#pragma unroll
      for (int k0 = 0; k0 < N; k0 += 4) {
        const int kk = k0 + lq;
        kJ = __builtin_amdgcn_mfma_f64_16x16x4f64(-sF[kk * P + li], sJ[kk * P + li], kJ, 0, 0, 0);
      }
      // kC = -(A Lc)(A Lc)^T: operand (li, 4 kb + lq) of both factors is this lane's AL[kb]
      wd4 kC = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int kb = 0; kb < 4; ++kb)
        if (4 * kb < nu) kC = __builtin_amdgcn_mfma_f64_16x16x4f64(AL[kb], AL[kb], kC, 0, 0, 0);
      // keta = K^T eta + J c - Q r;  kb = -(w + (A - I) w): component li, terms 4 lq .. 4 lq + 3
      // on lane 16 lq + li, then a butterfly over lq
      R ke = R(0), kbv = R(0);
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int q = 4 * lq + t;
        ke = fma(sK[q * P + li], se[q], ke);
        if (kp.has_c) ke = fma(sJ[li * P + q], sc[q], ke);
        ke = fma(-sQ[li * P + q], sr[q], ke);
        kbv = fma(sA[li * P + q], sw[q], kbv);
      }
      ke += __shfl_xor(ke, 16);
      ke += __shfl_xor(ke, 32);
      kbv += __shfl_xor(kbv, 16);
      kbv += __shfl_xor(kbv, 32);
      kbv = -(kbv + sw[li]);
      // RK4 accumulation and the next stage value
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        aA[r] = st == 0 ? fma(wk, kA[r], yA[r]) : fma(wk, kA[r], aA[r]);
        aJ[r] = st == 0 ? fma(wk, kJ[r], yJ[r]) : fma(wk, kJ[r], aJ[r]);
        yC[r] = fma(-wk, kC[r], yC[r]);
        if (st < 3) {
          tA[r] = fma(cn, kA[r], yA[r]);
          tJ[r] = fma(cn, kJ[r], yJ[r]);
        }
      }
      ae = st == 0 ? fma(wk, ke, ye) : fma(wk, ke, ae);
      yb = fma(wk, kbv, yb);
      if (st < 3) te = fma(cn, ke, ye);
      wsync();  // the next stage overwrites the operand buffers
    }
    // end of step: J and C take their upper entries
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      yA[r] = aA[r];
      sJ[(lq + 4 * r) * P + li] = aJ[r];
      sK[(lq + 4 * r) * P + li] = yC[r];
    }
    ye = ae;
    wsync();
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = lq + 4 * r;
      yJ[r] = i > li ? sJ[li * P + i] : aJ[r];
      yC[r] = i > li ? sK[li * P + i] : yC[r];
    }
    wsync();
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int i = lq + 4 * r;
    o.g[(i * N + li) * o.st] = yA[r];
    if (li >= i) {
      o.g[(oC + pk(i, li, N)) * o.st] = yC[r];
      o.g[(oJ + pk(i, li, N)) * o.st] = yJ[r];
    }
  }
  if (lane < N) {
    o.g[(oB + lane) * o.st] = yb;
    o.g[(oE + lane) * o.st] = ye;
  }
}

// ------------------------------------------------------------------------------------------
// Value tree.  The kernels below are thin launches of device bodies that take their node and
// problem, LDS and access policy A (coherent.hpp) from the caller: A applies to the tree records,
// S, v and x0 passed between the bodies (elements, written by an earlier launch, are plain loads),
// so the same bodies run as one launch per tree level (A = PlainAcc) and as the items of the
// single-launch solve below (A = DevAcc).
// ------------------------------------------------------------------------------------------
template <int N>
struct WSh {  // LDS of the bodies (values of the solve's type)
  static constexpr int kTupW = 3 * N * N + 2 * N, kScr = 4 * N * N + N * (2 * N + 1) + 2 * N;
  static constexpr int vreduce = 2 * kTupW + kScr;
  static constexpr int vfold = kTupW + kScr + N * N + N;
  static constexpr int vbottom = vfold + 3 * (N * N + N);
  static constexpr int treduce = 3 * (N * N + N);
  static constexpr int tsweep = N * N + 3 * N;
  static constexpr int tbottom = kTupW + kScr + N * N + N + N * N + 4 * N + N * N;
  static constexpr int max2(int a, int b) { return a > b ? a : b; }
  static constexpr int all =
      max2(max2(max2(vreduce, vfold), max2(vbottom, treduce)), max2(tsweep, tbottom));
};

// Value records (S full symmetric, v): n^2 + n values.
template <class A = PlainAcc, class R>
WDEV void val_st(const R* S, const R* v, R* g, int n) {
  for (int e = lane_id(); e < n * n; e += 64) A::st(g + e, S[e]);
  for (int i = lane_id(); i < n; i += 64) A::st(g + n * n + i, v[i]);
  wsync();
}
template <class A = PlainAcc, class R>
WDEV void val_ld(R* S, R* v, const R* g, int n) {
  for (int e = lane_id(); e < n * n; e += 64) S[e] = A::ld(g + e);
  for (int i = lane_id(); i < n; i += 64) v[i] = A::ld(g + n * n + i);
  wsync();
}

// Map records (P = Psi - I, q = alpha): n^2 + n values.
template <class A = PlainAcc, class R>
WDEV void map_ld(R* P, R* q, const R* g, int n) {
  for (int e = lane_id(); e < n * n; e += 64) P[e] = A::ld(g + e);
  for (int i = lane_id(); i < n; i += 64) q[i] = A::ld(g + n * n + i);
  wsync();
}
template <class A = PlainAcc, class R>
WDEV void map_st(const R* P, const R* q, R* g, int n) {
  for (int e = lane_id(); e < n * n; e += 64) A::st(g + e, P[e]);
  for (int i = lane_id(); i < n; i += 64) A::st(g + n * n + i, q[i]);
  wsync();
}

// Node i of level l + 1: the product of the wc nodes i wc .. of level l (elements when
// src_elts), right to left.
template <int N, class A, class R>
WDEV void wb_vreduce(R* sh, int* piv, int p, long i, int wc, int src_elts, const R* src,
                     long n_src, R* dst, long n_dst) {
  constexpr int n = N, kTupW = WSh<N>::kTupW;
  const int NE = ne_w(n);
  WT<R> acc = wt_at(sh, n), x = wt_at(sh + kTupW, n);
  WS<R> scr = ws_at(sh + 2 * kTupW, piv, n);
  const long j0 = i * wc, j1 = min(j0 + wc, n_src);
  auto load = [&](WT<R> t, long j) {
    if (src_elts)
      wt_load<PlainAcc>(t, elt_ref(src, p, j, n_src, NE), n);
    else
      wt_load<A>(t, rec_ref(src, p, j, n_src, NE), n);
  };
  load(acc, j1 - 1);
  for (long j = j1 - 2; j >= j0; --j) {
    load(x, j);
    w_combine<N>(x, acc, acc, scr, n);
  }
  wt_store<A>(acc, rec_ref(dst, p, i, n_dst, NE), n);
}

template <int N, class R>
__global__ __launch_bounds__(64) void kw_vreduce(int, int wc, int src_elts,
                                                 const R* __restrict__ src, long n_src,
                                                 R* __restrict__ dst, long n_dst) {
  __shared__ R sh[WSh<N>::vreduce];
  __shared__ int piv;
  if ((long)blockIdx.x >= n_dst) return;
  wb_vreduce<N, PlainAcc>(sh, &piv, blockIdx.y, blockIdx.x, wc, src_elts, src, n_src, dst, n_dst);
}

// The values at the right ends of the n_top top nodes: the terminal value carried leftwards.
template <int N, class A, class R>
WDEV void wb_vtop(R* sh, int* piv, const KProb& kp, int p, const R* tup, long n_top, R* val) {
  constexpr int n = N, kTupW = WSh<N>::kTupW, kScr = WSh<N>::kScr;
  const int NE = ne_w(n);
  WT<R> a = wt_at(sh, n);
  WS<R> scr = ws_at(sh + kTupW, piv, n);
  R* S = sh + kTupW + kScr;
  R* v = S + n * n;
  const R* Qf = (const R*)kp.Qf + (long)p * n * n;
  const R* rf = (const R*)kp.rf + (long)p * n;
  for (int e = lane_id(); e < n * n; e += 64) {
    const int i = e / n, j = e % n;
    S[e] = Qf[(i < j ? i : j) * n + (i < j ? j : i)];
  }
  for (int i = lane_id(); i < n; i += 64) {
    R t = R(0);
    for (int j = 0; j < n; ++j) t = fma(Qf[i * n + j], rf[j], t);
    v[i] = t;
  }
  wsync();
  const int VR = n * n + n;
  for (long j = n_top - 1; j >= 0; --j) {
    val_st<A>(S, v, val + ((long)p * n_top + j) * VR, n);
    if (j == 0) break;
    wt_load<A>(a, rec_ref(tup, p, j, n_top, NE), n);
    w_fold<N>(a, S, v, scr, n, (R*)nullptr, (R*)nullptr);
  }
}

template <int N, class R>
__global__ __launch_bounds__(64) void kw_vtop(const KProb kp, const R* __restrict__ tup, long n_top,
                                              R* __restrict__ val) {
  __shared__ R sh[WSh<N>::vfold];
  __shared__ int piv;
  wb_vtop<N, PlainAcc>(sh, &piv, kp, blockIdx.y, tup, n_top, val);
}

// Values at the right ends of the children of node i of level l + 1, from the node's own.
template <int N, class A, class R>
WDEV void wb_vdown(R* sh, int* piv, int p, long i, int wc, const R* tup, long n_child,
                   const R* val_in, long n_par, R* val_out) {
  constexpr int n = N, kTupW = WSh<N>::kTupW, kScr = WSh<N>::kScr;
  const int NE = ne_w(n), VR = n * n + n;
  WT<R> a = wt_at(sh, n);
  WS<R> scr = ws_at(sh + kTupW, piv, n);
  R* S = sh + kTupW + kScr;
  R* v = S + n * n;
  val_ld<A>(S, v, val_in + ((long)p * n_par + i) * VR, n);
  const long j0 = i * wc, j1 = min(j0 + wc, n_child);
  for (long j = j1 - 1; j >= j0; --j) {
    val_st<A>(S, v, val_out + ((long)p * n_child + j) * VR, n);
    if (j == j0) break;
    wt_load<A>(a, rec_ref(tup, p, j, n_child, NE), n);
    w_fold<N>(a, S, v, scr, n, (R*)nullptr, (R*)nullptr);
  }
}

template <int N, class R>
__global__ __launch_bounds__(64) void kw_vdown(int, int wc, const R* __restrict__ tup, long n_child,
                                               const R* __restrict__ val_in, long n_par,
                                               R* __restrict__ val_out) {
  __shared__ R sh[WSh<N>::vfold];
  __shared__ int piv;
  if ((long)blockIdx.x >= n_par) return;
  wb_vdown<N, PlainAcc>(sh, &piv, blockIdx.y, blockIdx.x, wc, tup, n_child, val_in, n_par,
                        val_out);
}

// Two-wave form of a value-tree level above the leaves, for levels of few nodes (each node's
// chain of combinations, not the device's throughput, sets their time).  Node i of level l + 1
// from its four children t0 .. t3 of level l: wave 0 forms t0 (x) t1 while wave 1 forms
// t2 (x) t3, then wave 0 combines the two (the Lemma 7 combination is associative), two
// combinations deep instead of three.  Wave 1 also writes t2 (x) t3 over t2's record, where the
// down-sweep of the same level (kw_vdown2) reads it: that sweep needs the pair product and not
// t2.  A node with fewer children (the last of a level) takes the sequential product on both
// waves and wave 0 stores it.  Where one wave has a step the other lacks, the other repeats a
// step of the same kind on its own LDS copy or takes the barrier alone, so both pass the same
// barriers; the wave index is made wave-uniform (readfirstlane), so such branches are scalar.
// LEFT: keep t0 (x) t1 over t1's record instead, for Method 2's down-sweep (kw_m2_down2), which
// builds prefixes from the left and needs t0, the left pair and t2.
template <int N, class R, bool LEFT = false>
__global__ __launch_bounds__(128) void kw_vreduce2(int wc, R* __restrict__ src, long n_src,
                                                   R* __restrict__ dst, long n_dst) {
  constexpr int n = N, kTupW = WSh<N>::kTupW;
  __shared__ R sh[2][WSh<N>::vreduce];
  __shared__ int piv[2];
  if ((long)blockIdx.x >= n_dst) return;
  const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int p = blockIdx.y, NE = ne_w(n);
  const long i = blockIdx.x;
  WT<R> acc = wt_at(sh[w], n), x = wt_at(sh[w] + kTupW, n);
  WS<R> scr = ws_at(sh[w] + 2 * kTupW, &piv[w], n);
  const R* in = src;
  const long j0 = i * wc, j1 = min(j0 + wc, n_src);
  if (j1 - j0 == 4) {
    const long ja = j0 + 2 * w;
    wt_load<PlainAcc>(x, rec_ref(in, p, ja, n_src, NE), n);
    wt_load<PlainAcc>(acc, rec_ref(in, p, ja + 1, n_src, NE), n);
    w_combine<N>(x, acc, acc, scr, n);  // wave w: t_2w (x) t_2w+1
    if (w == (LEFT ? 0 : 1))
      wt_store<PlainAcc>(acc, rec_ref(src, p, LEFT ? j0 + 1 : j0 + 2, n_src, NE), n);
    else
      wsync();
    // wave 0: (t0 t1) (x) (t2 t3) from wave 1's LDS; wave 1: a combination of its own copy of t2
    // with itself, discarded (it leaves wave 1's product, which wave 0 reads, untouched)
    const WT<R> right = wt_at(sh[1], n);
    w_combine<N>(w == 0 ? acc : x, w == 0 ? right : x, w == 0 ? acc : x, scr, n);
  } else {
    wt_load<PlainAcc>(acc, rec_ref(in, p, j1 - 1, n_src, NE), n);
    for (long j = j1 - 2; j >= j0; --j) {
      wt_load<PlainAcc>(x, rec_ref(in, p, j, n_src, NE), n);
      w_combine<N>(x, acc, acc, scr, n);
    }
  }
  if (w == 0)
    wt_store<PlainAcc>(acc, rec_ref(dst, p, i, n_dst, NE), n);
  else
    wsync();
}

// Down-sweep of a level reduced by kw_vreduce2: the values at the right ends of node i's children
// from the node's own.  With four children, wave 0 stores the node's value as child 3's and folds
// t3 into it (child 2) while wave 1 folds the pair product t2 (x) t3 (child 1) and then t1 (child
// 0): two folds deep instead of three.  Fewer children: the sequential sweep on both waves, wave 0
// storing.  Barriers as in kw_vreduce2.
template <int N, class R>
__global__ __launch_bounds__(128) void kw_vdown2(int wc, const R* __restrict__ tup, long n_child,
                                                 const R* __restrict__ val_in, long n_par,
                                                 R* __restrict__ val_out) {
  constexpr int n = N, kTupW = WSh<N>::kTupW, kScr = WSh<N>::kScr;
  __shared__ R sh[2][WSh<N>::vfold];
  __shared__ int piv[2];
  if ((long)blockIdx.x >= n_par) return;
  const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int p = blockIdx.y, NE = ne_w(n), VR = n * n + n;
  const long i = blockIdx.x;
  WT<R> a = wt_at(sh[w], n);
  WS<R> scr = ws_at(sh[w] + kTupW, &piv[w], n);
  R* S = sh[w] + kTupW + kScr;
  R* v = S + n * n;
  R* out = val_out + (long)p * n_child * VR;
  val_ld<PlainAcc>(S, v, val_in + ((long)p * n_par + i) * VR, n);
  const long j0 = i * wc, j1 = min(j0 + wc, n_child);
  if (j1 - j0 == 4) {
    if (w == 0)
      val_st<PlainAcc>(S, v, out + (j0 + 3) * VR, n);
    else
      wsync();
    // wave 0: t3 (child 2); wave 1: the pair product t2 (x) t3 in t2's slot (child 1)
    wt_load<PlainAcc>(a, rec_ref(tup, p, w == 0 ? j0 + 3 : j0 + 2, n_child, NE), n);
    w_fold<N>(a, S, v, scr, n, (R*)nullptr, (R*)nullptr);
    val_st<PlainAcc>(S, v, out + (w == 0 ? j0 + 2 : j0 + 1) * VR, n);
    // wave 1: t1 (child 0); wave 0 folds the same record into its own copy, discarded
    wt_load<PlainAcc>(a, rec_ref(tup, p, j0 + 1, n_child, NE), n);
    w_fold<N>(a, S, v, scr, n, (R*)nullptr, (R*)nullptr);
    if (w == 1)
      val_st<PlainAcc>(S, v, out + j0 * VR, n);
    else
      wsync();
  } else {
    for (long j = j1 - 1; j >= j0; --j) {
      if (w == 0)
        val_st<PlainAcc>(S, v, out + j * VR, n);
      else
        wsync();
      if (j == j0) break;
      wt_load<PlainAcc>(a, rec_ref(tup, p, j, n_child, NE), n);
      w_fold<N>(a, S, v, scr, n, (R*)nullptr, (R*)nullptr);
    }
  }
}

// Values of every block from the value at the right end of each chunk; level 1 of the
// trajectory tree (composition of the chunk's block maps) when maps1 != nullptr, and every
// block's closed-loop map ([batch][T] records P = Psi - I, q = alpha; the fold computes it on the
// way) when bmaps != nullptr.
template <int N, class A, class R>
WDEV void wb_vbottom(R* sh, int* piv, const KProb& kp, int p, long i, int wc, const R* elts,
                     const R* val1, long n1, R* Sout, R* vout, R* maps1, R* bmaps) {
  constexpr int n = N, kTupW = WSh<N>::kTupW, kScr = WSh<N>::kScr;
  const long T = kp.T;
  const int NE = ne_w(n), VR = n * n + n, MR = n * n + n;
  WT<R> a = wt_at(sh, n);
  WS<R> scr = ws_at(sh + kTupW, piv, n);
  R* S = sh + kTupW + kScr;
  R* v = S + n * n;
  R* aP = v + n;
  R* aq = aP + n * n;
  R* mP = aq + n;
  R* mq = mP + n * n;
  R* tmp = mq + n;
  val_ld<A>(S, v, val1 + ((long)p * n1 + i) * VR, n);
  R* Sp = Sout + (long)p * (T + 1) * n * n;
  R* vp = vout + (long)p * (T + 1) * n;
  const long j0 = i * wc, j1 = min(j0 + wc, T);
  if (j1 == T && !kp.seg) {
    for (int e = lane_id(); e < n * n; e += 64) A::st(Sp + T * n * n + e, S[e]);
    for (int q = lane_id(); q < n; q += 64) A::st(vp + T * n + q, v[q]);
  }
  w_aff_identity(aP, aq, n);
  for (long k = j1 - 1; k >= j0; --k) {
    wt_load<PlainAcc>(a, elt_ref(elts, p, k, T, NE), n);
    w_fold<N>(a, S, v, scr, n, mP, mq);
    for (int e = lane_id(); e < n * n; e += 64) A::st(Sp + k * n * n + e, S[e]);
    for (int q = lane_id(); q < n; q += 64) A::st(vp + k * n + q, v[q]);
    if (bmaps) map_st<A>(mP, mq, bmaps + ((long)p * T + k) * MR, n);
    if (maps1) w_aff_after(aP, aq, mP, mq, tmp, n);
  }
  if (maps1) {
    R* g = maps1 + ((long)p * n1 + i) * MR;
    for (int e = lane_id(); e < n * n; e += 64) A::st(g + e, aP[e]);
    for (int q = lane_id(); q < n; q += 64) A::st(g + n * n + q, aq[q]);
  }
}

template <int N, class R>
__global__ __launch_bounds__(64) void kw_vbottom(const KProb kp, int wc, const R* __restrict__ elts,
                                                 const R* __restrict__ val1, long n1,
                                                 R* __restrict__ Sout, R* __restrict__ vout,
                                                 R* __restrict__ maps1, R* __restrict__ bmaps) {
  __shared__ R sh[WSh<N>::vbottom];
  __shared__ int piv;
  if ((long)blockIdx.x >= n1) return;
  wb_vbottom<N, PlainAcc>(sh, &piv, kp, blockIdx.y, blockIdx.x, wc, elts, val1, n1, Sout, vout,
                          maps1, bmaps);
}

// ------------------------------------------------------------------------------------------
// Trajectory tree.
// ------------------------------------------------------------------------------------------

// Gain R^{-1} L^T (nu x n, row-major) of problem pk into Kc, L at global sample s when sampled.
template <class R>
WDEV void w_gain(const KProb& kp, int pk, long s, R* Kc, int n, int nu) {
  const R* cs = (const R*)kp.consts + (long)pk * consts_count(n, nu);
  if (kp.L_sampled) {
    const R* Lk = (const R*)kp.L + s * n * nu;
    const R* Ri = cs + consts_off_Rinv(n, nu);
    for (int e = lane_id(); e < nu * n; e += 64) {
      const int l = e / n, j = e % n;
      R a = R(0);
      for (int q = 0; q < nu; ++q) a = fma(Ri[l * nu + q], Lk[j * nu + q], a);
      Kc[e] = a;
    }
  } else {
    for (int e = lane_id(); e < nu * n; e += 64) Kc[e] = cs[consts_off_Kc(n, nu) + e];
  }
  wsync();
}

// u = -Kc (S x - v) with S (full), v, x, Kc in LDS; g: n values of scratch.
template <class R>
WDEV void w_control(const R* Kc, const R* S, const R* v, const R* x, R* g, R* u, int n, int nu) {
  for (int r = lane_id(); r < n; r += 64) {
    R a = -v[r];
    for (int j = 0; j < n; ++j) a = fma(S[r * n + j], x[j], a);
    g[r] = a;
  }
  wsync();
  for (int l = lane_id(); l < nu; l += 64) {
    R a = R(0);
    for (int j = 0; j < n; ++j) a = fma(-Kc[l * n + j], g[j], a);
    u[l] = a;
  }
  wsync();
}

// The Method 2 state x = (I + C S)^{-1} (xk + Ad xk + b + C v) (Sec. IV-E) for the parts Ad, b, C
// of an interval that starts at xk, and S, v at its right end; M, B: 2 n^2 and n values of scratch
// (the solve with one right-hand side keeps both of its broadcast buffers in M's).
template <int N, class R>
WDEV void w_m2_state(const R* Ad, const R* b, const R* C, const R* xk, const R* S, const R* v,
                     R* M, R* B, R* x, int n) {
  for (int e = lane_id(); e < n * n; e += 64) {
    const int i = e / n, j = e % n;
    R a = i == j ? R(1) : R(0);
    for (int l = 0; l < n; ++l) a = fma(C[i * n + l], S[l * n + j], a);
    M[e] = a;
  }
  for (int i = lane_id(); i < n; i += 64) {
    R a = xk[i] + b[i];
    for (int l = 0; l < n; ++l) {
      a = fma(Ad[i * n + l], xk[l], a);
      a = fma(C[i * n + l], v[l], a);
    }
    B[i] = a;
  }
  wsync();
  w_solve<N, 1>(M, B);
  for (int i = lane_id(); i < n; i += 64) x[i] = B[i];
  wsync();
}

// (S_{k+1}, v_{k+1}) into LDS; zeros for the last block in ragged mode (a separator, whose map
// does not depend on them; row T does not exist there).
template <class A = PlainAcc, class R>
WDEV void w_right_value(const KProb& kp, const R* Sp, const R* vp, long k, R* S, R* v, int n) {
  const bool none = kp.seg && k + 1 >= kp.T;
  for (int e = lane_id(); e < n * n; e += 64) S[e] = none ? R(0) : A::ld(Sp + (k + 1) * n * n + e);
  for (int q = lane_id(); q < n; q += 64) v[q] = none ? R(0) : A::ld(vp + (k + 1) * n + q);
  wsync();
}

template <int N, class R>
__global__ __launch_bounds__(64) void kw_tbottom_reduce(const KProb kp, int wc, const R* __restrict__ elts,
                                                        const R* __restrict__ Sg,
                                                        const R* __restrict__ vg,
                                                        R* __restrict__ maps1, long n1) {
  constexpr int kTupW = WSh<N>::kTupW, kScr = WSh<N>::kScr;
  __shared__ R sh[WSh<N>::vbottom];
  __shared__ int piv;
  const int p = blockIdx.y;
  const long i = blockIdx.x;
  if (i >= n1) return;
  constexpr int n = N;
  const long T = kp.T;
  const int NE = ne_w(n), MR = n * n + n;
  WT<R> a = wt_at(sh, n);
  WS<R> scr = ws_at(sh + kTupW, &piv, n);
  R* S = sh + kTupW + kScr;
  R* v = S + n * n;
  R* aP = v + n;
  R* aq = aP + n * n;
  R* mP = aq + n;
  R* mq = mP + n * n;
  R* tmp = mq + n;
  const R* Sp = Sg + (long)p * (T + 1) * n * n;
  const R* vp = vg + (long)p * (T + 1) * n;
  const long j0 = i * wc, j1 = min(j0 + wc, T);
  w_aff_identity(aP, aq, n);
  for (long k = j0; k < j1; ++k) {
    wt_load(a, elt_ref(elts, p, k, T, NE), n);
    w_right_value(kp, Sp, vp, k, S, v, n);
    w_block_map<N>(a, S, v, scr, n, mP, mq);
    w_aff_then(aP, aq, mP, mq, tmp, n);
  }
  map_st(aP, aq, maps1 + ((long)p * n1 + i) * MR, n);
}

// Map of node i of level l + 1: the composition of the wc maps i wc .. of level l (time order).
template <int N, class A, class R>
WDEV void wb_treduce(R* sh, int p, long i, int wc, const R* src, long n_src, R* dst, long n_dst) {
  constexpr int n = N;
  const int MR = n * n + n;
  R* aP = sh;
  R* aq = aP + n * n;
  R* mP = aq + n;
  R* mq = mP + n * n;
  R* tmp = mq + n;
  const long j0 = i * wc, j1 = min(j0 + wc, n_src);
  map_ld<A>(aP, aq, src + ((long)p * n_src + j0) * MR, n);
  for (long j = j0 + 1; j < j1; ++j) {
    map_ld<A>(mP, mq, src + ((long)p * n_src + j) * MR, n);
    w_aff_then(aP, aq, mP, mq, tmp, n);
  }
  map_st<A>(aP, aq, dst + ((long)p * n_dst + i) * MR, n);
}

template <int N, class R>
__global__ __launch_bounds__(64) void kw_treduce(int, int wc, const R* __restrict__ src, long n_src,
                                                 R* __restrict__ dst, long n_dst) {
  __shared__ R sh[WSh<N>::treduce];
  if ((long)blockIdx.x >= n_dst) return;
  wb_treduce<N, PlainAcc>(sh, blockIdx.y, blockIdx.x, wc, src, n_src, dst, n_dst);
}

// x at the left ends of the n_top top nodes: x0 carried rightwards.
template <int N, class A, class R>
WDEV void wb_ttop(R* sh, const KProb& kp, int p, const R* maps, long n_top, R* xs) {
  constexpr int n = N;
  const int MR = n * n + n;
  R* mP = sh;
  R* mq = mP + n * n;
  R* x = mq + n;
  R* tmp = x + n;
  for (int q = lane_id(); q < n; q += 64) x[q] = ((const R*)kp.x0)[(long)p * n + q];
  wsync();
  for (long j = 0; j < n_top; ++j) {
    for (int q = lane_id(); q < n; q += 64) A::st(xs + ((long)p * n_top + j) * n + q, x[q]);
    if (j == n_top - 1) break;
    map_ld<A>(mP, mq, maps + ((long)p * n_top + j) * MR, n);
    w_aff_apply(mP, mq, x, tmp, n);
  }
  wsync();
}

template <int N, class R>
__global__ __launch_bounds__(64) void kw_ttop(const KProb kp, const R* __restrict__ maps, long n_top,
                                              R* __restrict__ xs) {
  __shared__ R sh[WSh<N>::tsweep];
  wb_ttop<N, PlainAcc>(sh, kp, blockIdx.y, maps, n_top, xs);
}

// x at the left ends of the children of node i of level l + 1, from the node's own.
template <int N, class A, class R>
WDEV void wb_tdown(R* sh, int p, long i, int wc, const R* maps, long n_child, const R* x_in,
                   long n_par, R* x_out) {
  constexpr int n = N;
  const int MR = n * n + n;
  R* mP = sh;
  R* mq = mP + n * n;
  R* x = mq + n;
  R* tmp = x + n;
  for (int q = lane_id(); q < n; q += 64) x[q] = A::ld(x_in + ((long)p * n_par + i) * n + q);
  wsync();
  const long j0 = i * wc, j1 = min(j0 + wc, n_child);
  for (long j = j0; j < j1; ++j) {
    for (int q = lane_id(); q < n; q += 64) A::st(x_out + ((long)p * n_child + j) * n + q, x[q]);
    if (j == j1 - 1) break;
    map_ld<A>(mP, mq, maps + ((long)p * n_child + j) * MR, n);
    w_aff_apply(mP, mq, x, tmp, n);
  }
  wsync();
}

template <int N, class R>
__global__ __launch_bounds__(64) void kw_tdown(int, int wc, const R* __restrict__ maps, long n_child,
                                               const R* __restrict__ x_in, long n_par,
                                               R* __restrict__ x_out) {
  __shared__ R sh[WSh<N>::tsweep];
  if ((long)blockIdx.x >= n_par) return;
  wb_tdown<N, PlainAcc>(sh, blockIdx.y, blockIdx.x, wc, maps, n_child, x_in, n_par, x_out);
}

// x_k and u_k = -R^{-1} L(t_k)^T (S_k x_k - v_k) of every block of a chunk; the block maps are
// loaded from bmaps (see wb_vbottom) when given, else computed from the elements and S, v.
template <int N, class A, class R>
WDEV void wb_tbottom(R* sh, int* piv, const KProb& kp, int p, long i, int wc, const R* elts,
                     const R* Sg, const R* vg, const R* x1, long n1, R* xout, R* uout,
                     const R* bmaps) {
  constexpr int n = N, kTupW = WSh<N>::kTupW, kScr = WSh<N>::kScr;
  const int nu = kp.nu;
  const long T = kp.T;
  const int NE = ne_w(n);
  WT<R> a = wt_at(sh, n);
  WS<R> scr = ws_at(sh + kTupW, piv, n);
  R* S = sh + kTupW + kScr;
  R* v = S + n * n;
  R* mP = v + n;
  R* mq = mP + n * n;
  R* x = mq + n;
  R* tmp = x + n;
  R* g = tmp + n;
  R* Kc = g + n;  // nu x n
  const R* Sp = Sg + (long)p * (T + 1) * n * n;
  const R* vp = vg + (long)p * (T + 1) * n;
  R* xp = xout + (long)p * (T + 1) * n;
  R* up = uout ? uout + (long)p * (T + 1) * nu : nullptr;
  for (int q = lane_id(); q < n; q += 64) x[q] = A::ld(x1 + ((long)p * n1 + i) * n + q);
  wsync();
  const long j0 = i * wc, j1 = min(j0 + wc, T);
  auto control = [&](long k) {
    if (!up) return;
    // Gain of the problem owning boundary k (looked up in ragged mode).
    const int pk = kp.seg ? seg_find(kp.seg, kp.nseg, k) : p;
    const long s0 = kp.seg ? (long)pk * (1 - 2L * kp.n) : (long)p * (2L * kp.n * T + 1);
    w_gain(kp, pk, s0 + 2L * kp.n * k, Kc, n, nu);
    for (int r = lane_id(); r < n; r += 64) {
      R s = -A::ld(vp + k * n + r);
      for (int j = 0; j < n; ++j) s = fma(A::ld(Sp + k * n * n + r * n + j), x[j], s);
      g[r] = s;
    }
    wsync();
    for (int l = lane_id(); l < nu; l += 64) {
      R s = R(0);
      for (int j = 0; j < n; ++j) s = fma(-Kc[l * n + j], g[j], s);
      up[k * nu + l] = s;
    }
    wsync();
  };
  for (long k = j0; k < j1; ++k) {
    for (int q = lane_id(); q < n; q += 64) xp[k * n + q] = x[q];
    control(k);
    if (bmaps) {
      map_ld<A>(mP, mq, bmaps + ((long)p * T + k) * (n * n + n), n);
    } else {
      wt_load<PlainAcc>(a, elt_ref(elts, p, k, T, NE), n);
      w_right_value<A>(kp, Sp, vp, k, S, v, n);
      w_block_map<N>(a, S, v, scr, n, mP, mq);
    }
    w_aff_apply(mP, mq, x, tmp, n);
  }
  if (j1 == T && !kp.seg) {
    for (int q = lane_id(); q < n; q += 64) xp[T * n + q] = x[q];
    control(T);
  }
}

template <int N, class R>
__global__ __launch_bounds__(64) void kw_tbottom(const KProb kp, int wc, const R* __restrict__ elts,
                                                 const R* __restrict__ Sg, const R* __restrict__ vg,
                                                 const R* __restrict__ x1, long n1,
                                                 R* __restrict__ xout, R* __restrict__ uout,
                                                 const R* __restrict__ bmaps) {
  __shared__ R sh[WSh<N>::tbottom];
  __shared__ int piv;
  if ((long)blockIdx.x >= n1) return;
  wb_tbottom<N, PlainAcc>(sh, &piv, kp, blockIdx.y, blockIdx.x, wc, elts, Sg, vg, x1, n1, xout,
                          uout, bmaps);
}

// ------------------------------------------------------------------------------------------
// Method 2 (Sec. IV-E): x_k from the prefix a_0 (x) ... (x) a_{k-1} (Lemma 7) and S_k, v_k by the
// state formula of w_m2_state with xk = x0.  The node products of the tree are those of the value
// scan's reduce (kw_vreduce; a product does not depend on the direction it is read in); the
// prefix of each node (the product of every block before it) goes down the tree as a tuple
// record, and the bottom extends each leaf's prefix block by block.
// ------------------------------------------------------------------------------------------
template <int N>
struct WM2Sh {
  static constexpr int kTupW = 3 * N * N + 2 * N, kScr = 4 * N * N + N * (2 * N + 1) + 2 * N;
  static constexpr int sweep = 2 * kTupW + kScr;
  static constexpr int bottom = sweep + 3 * N * N + 6 * N;
};

// Prefix records of the children j0 .. j1 - 1 of a node whose own prefix is in run: each child's
// prefix, then run (x) child (tup: the children's products, or nullptr for the identity start).
template <int N, class R>
WDEV void wb_m2_sweep(R* sh, int* piv, int p, long j0, long j1, const R* tup, long n_child,
                      R* pre, WT<R> run) {
  constexpr int n = N;
  const int NE = ne_w(n);
  WT<R> a = wt_at(sh + WM2Sh<N>::kTupW, n);
  WS<R> scr = ws_at(sh + 2 * WM2Sh<N>::kTupW, piv, n);
  for (long j = j0; j < j1; ++j) {
    wt_store(run, rec_ref(pre, p, j, n_child, NE), n);
    if (j + 1 == j1) break;
    wt_load<PlainAcc>(a, rec_ref(tup, p, j, n_child, NE), n);
    w_combine<N>(run, a, a, scr, n);
    const WT<R> t = run;
    run = a;
    a = t;
  }
}

template <int N, class R>
__global__ __launch_bounds__(64) void kw_m2_top(const R* __restrict__ tup, long n_top,
                                                R* __restrict__ pre) {
  __shared__ R sh[WM2Sh<N>::sweep];
  __shared__ int piv;
  WT<R> run = wt_at(sh, N);
  wt_identity(run, N);
  wb_m2_sweep<N, R>(sh, &piv, blockIdx.y, 0, n_top, tup, n_top, pre, run);
}

template <int N, class R>
__global__ __launch_bounds__(64) void kw_m2_down(int wc, const R* __restrict__ tup, long n_child,
                                                 const R* __restrict__ pre_in, long n_par,
                                                 R* __restrict__ pre_out) {
  __shared__ R sh[WM2Sh<N>::sweep];
  __shared__ int piv;
  const long i = blockIdx.x;
  if (i >= n_par) return;
  WT<R> run = wt_at(sh, N);
  wt_load<PlainAcc>(run, rec_ref(pre_in, blockIdx.y, i, n_par, ne_w(N)), N);
  wb_m2_sweep<N, R>(sh, &piv, blockIdx.y, i * wc, min(i * wc + wc, n_child), tup, n_child,
                    pre_out, run);
}

// Down-sweep of a level reduced by kw_vreduce2<N, R, true> (left pair products t0 (x) t1 in t1's
// records): with four children, wave 0 stores the node's prefix as child 0's and forms
// prefix (x) t0 (child 1) while wave 1 forms prefix (x) (t0 t1) (child 2) and then (x) t2
// (child 3): two combinations deep instead of three.  Fewer children: the sequential sweep on
// both waves, wave 0 storing.  Barriers as in kw_vreduce2.
template <int N, class R>
__global__ __launch_bounds__(128) void kw_m2_down2(int wc, const R* __restrict__ tup, long n_child,
                                                   const R* __restrict__ pre_in, long n_par,
                                                   R* __restrict__ pre_out) {
  constexpr int n = N, kTupW = WM2Sh<N>::kTupW;
  __shared__ R sh[2][WM2Sh<N>::sweep];
  __shared__ int piv[2];
  if ((long)blockIdx.x >= n_par) return;
  const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int p = blockIdx.y, NE = ne_w(n);
  const long i = blockIdx.x;
  WT<R> run = wt_at(sh[w], n), a = wt_at(sh[w] + kTupW, n);
  WS<R> scr = ws_at(sh[w] + 2 * kTupW, &piv[w], n);
  wt_load<PlainAcc>(run, rec_ref(pre_in, p, i, n_par, NE), n);
  const long j0 = i * wc, j1 = min(j0 + wc, n_child);
  if (j1 - j0 == 4) {
    if (w == 0)
      wt_store<PlainAcc>(run, rec_ref(pre_out, p, j0, n_child, NE), n);
    else
      wsync();
    // wave 0: t0 (child 1); wave 1: the left pair product in t1's slot (child 2)
    wt_load<PlainAcc>(a, rec_ref(tup, p, j0 + w, n_child, NE), n);
    w_combine<N>(run, a, a, scr, n);
    wt_store<PlainAcc>(a, rec_ref(pre_out, p, j0 + 1 + w, n_child, NE), n);
    // wave 1: (x) t2 (child 3); wave 0 forms the same kind of product on its copy, discarded
    wt_load<PlainAcc>(run, rec_ref(tup, p, j0 + 2, n_child, NE), n);
    w_combine<N>(a, run, run, scr, n);
    if (w == 1)
      wt_store<PlainAcc>(run, rec_ref(pre_out, p, j0 + 3, n_child, NE), n);
    else
      wsync();
  } else {
    for (long j = j0; j < j1; ++j) {
      if (w == 0)
        wt_store<PlainAcc>(run, rec_ref(pre_out, p, j, n_child, NE), n);
      else
        wsync();
      if (j + 1 == j1) break;
      wt_load<PlainAcc>(a, rec_ref(tup, p, j, n_child, NE), n);
      w_combine<N>(run, a, a, scr, n);
      const WT<R> t = run;
      run = a;
      a = t;
    }
  }
}

template <int N, class R>
__global__ __launch_bounds__(64) void kw_m2_bottom(const KProb kp, int wc, const R* __restrict__ elts,
                                                   const R* __restrict__ Sg,
                                                   const R* __restrict__ vg,
                                                   const R* __restrict__ pre1, long n1,
                                                   R* __restrict__ xout, R* __restrict__ uout) {
  constexpr int n = N, kTupW = WM2Sh<N>::kTupW;
  __shared__ R sh[WM2Sh<N>::bottom];
  __shared__ int piv;
  const int p = blockIdx.y;
  const long i = blockIdx.x;
  if (i >= n1) return;
  const int nu = kp.nu;
  const long T = kp.T;
  const int NE = ne_w(n);
  WT<R> run = wt_at(sh, n), a = wt_at(sh + kTupW, n);
  WS<R> scr = ws_at(sh + 2 * kTupW, &piv, n);
  R* S = sh + WM2Sh<N>::sweep;
  R* M = S + n * n;
  R* Kc = M + n * n;  // right after M: the state solve takes M and Kc as its 2 n^2 values
  R* v = Kc + n * n;
  R* x0 = v + n;
  R* x = x0 + n;
  R* B = x + n;
  R* g = B + n;
  R* u = g + n;
  const R* Sp = Sg + (long)p * (T + 1) * n * n;
  const R* vp = vg + (long)p * (T + 1) * n;
  R* xp = xout + (long)p * (T + 1) * n;
  R* up = uout ? uout + (long)p * (T + 1) * nu : nullptr;
  const long s0 = (long)p * (2L * kp.n * T + 1);
  for (int q = lane_id(); q < n; q += 64) x0[q] = ((const R*)kp.x0)[(long)p * n + q];
  wt_load<PlainAcc>(run, rec_ref(pre1, p, i, n1, NE), n);
  auto emit = [&](long k) {
    for (int e = lane_id(); e < n * n; e += 64) S[e] = Sp[k * n * n + e];
    for (int q = lane_id(); q < n; q += 64) v[q] = vp[k * n + q];
    wsync();
    w_m2_state<N>(run.A, run.b, run.C, x0, S, v, M, B, x, n);
    for (int q = lane_id(); q < n; q += 64) xp[k * n + q] = x[q];
    if (up) {
      w_gain(kp, p, s0 + 2L * kp.n * k, Kc, n, nu);
      w_control(Kc, S, v, x, g, u, n, nu);
      for (int l = lane_id(); l < nu; l += 64) up[k * nu + l] = u[l];
    }
  };
  const long j0 = i * wc, j1 = min(j0 + wc, T);
  for (long k = j0; k < j1; ++k) {
    emit(k);
    if (k + 1 == j1 && j1 < T) break;
    wt_load<PlainAcc>(a, elt_ref(elts, p, k, T, NE), n);
    w_combine<N>(run, a, a, scr, n);
    const WT<R> t = run;
    run = a;
    a = t;
  }
  if (j1 == T) emit(T);
}

// ------------------------------------------------------------------------------------------
// Values inside the blocks (Sec. VI-A), one wave per block k.  At the nodes t_k + m h
// (m = 1 .. n - 1):
//   S, v by classical RK4 on their backward ODEs (Sec. II-B) from S_{k+1}, v_{k+1}:
//     dS/dt = -F^T S - S F - Q + S G S,  dv/dt = -Q r - F^T v + S G v + S c;
//   x by the Method 2 formula with the forward parts of Theorem 9 on [t_k, t_k + m h] (the steps
//     of the forward build without eta, J), x_k at the left end;
//   u by the control law at the node's sample.
// Node n k carries the block-boundary values and node n T those at t_T.  The forward sweep reads
// the interior S, v back from the outputs the same wave wrote (L2-resident by then).
// ------------------------------------------------------------------------------------------
template <int N>
struct WDenseSh {
  static constexpr int kTupW = 3 * N * N + 2 * N;
  static constexpr int riccati = 9 * N * N + 6 * N;
  static constexpr int fwd = 3 * kTupW + kBuildScr<N>;
  static constexpr int extra = 3 * N * N + 5 * N;
  static constexpr int all = (riccati > fwd ? riccati : fwd) + extra;
};

template <int N, class R>
__global__ __launch_bounds__(64) void kw_dense(const KProb kp, const R* __restrict__ Sg,
                                               const R* __restrict__ vg,
                                               const R* __restrict__ xg, R* __restrict__ Sd,
                                               R* __restrict__ vd, R* __restrict__ xd,
                                               R* __restrict__ ud) {
  constexpr int n = N, kTupW = WDenseSh<N>::kTupW;
  __shared__ R sh[WDenseSh<N>::all];
  const int p = blockIdx.y;
  const long k = blockIdx.x;
  const int nn = kp.n, nu = kp.nu;
  const long T = kp.T;
  const long nodes = (long)nn * T + 1;
  const WBlk bk = wblk_plain(kp, p, k);
  const R* Sp = Sg + (long)p * (T + 1) * n * n;
  const R* vp = vg + (long)p * (T + 1) * n;
  const R* xp = xg + (long)p * (T + 1) * n;
  R* Sdp = Sd + (long)p * nodes * n * n;
  R* vdp = vd + (long)p * nodes * n;
  R* xdp = xd + (long)p * nodes * n;
  R* udp = ud ? ud + (long)p * nodes * nu : nullptr;
  const R* t = (const R*)kp.t + bk.tk;
  const R h = (t[1] - t[0]) / R(nn);
  // node-level scratch, beside both sweeps' areas
  R* Sn = sh + (WDenseSh<N>::all - WDenseSh<N>::extra);
  R* Mn = Sn + n * n;
  R* Kc = Mn + n * n;  // right after Mn: the state solve takes Mn and Kc as its 2 n^2 values
  R* vn = Kc + n * n;
  R* xk = vn + n;
  R* xn = xk + n;
  R* Bn = xn + n;
  R* gn = Bn + n;
  auto emit_u = [&](long node) {  // from Sn, vn, xn
    if (!udp) return;
    w_gain(kp, p, bk.s0 + 2 * node, Kc, n, nu);
    w_control(Kc, Sn, vn, xn, gn, Bn, n, nu);
    for (int l = lane_id(); l < nu; l += 64) udp[node * nu + l] = Bn[l];
    wsync();
  };

  // ---- backward sweep: S, v at nodes n k + n - 1 down to n k + 1 ----
  {
    R* F = sh;
    R* G = F + n * n;
    R* Lc = G + n * n;
    R* Qs = Lc + n * n;
    R* P = Qs + n * n;
    R* kS = P + n * n;
    R* S = kS + n * n;
    R* sS = S + n * n;
    R* aS = sS + n * n;
    R* rv = aS + n * n;
    R* cv = rv + n;
    R* v = cv + n;
    R* sv = v + n;
    R* av = sv + n;
    R* kv = av + n;
    const R* Fc = (const R*)kp.F;
    const R* Qp = (const R*)kp.Q + (long)p * n * n;
    const R* cs = (const R*)kp.consts + (long)p * consts_count(n, nu);
    const R* cb = kp.has_c ? (const R*)kp.c : nullptr;
    for (int e = lane_id(); e < n * n; e += 64) {
      Qs[e] = Qp[e];
      S[e] = Sp[(k + 1) * n * n + e];
      if (!kp.L_sampled) G[e] = cs[consts_off_G(n, nu) + e];
    }
    for (int i = lane_id(); i < n; i += 64) v[i] = vp[(k + 1) * n + i];
    wsync();
    for (int mp = 0; mp < nn - 1; ++mp) {
      const long j1 = 2L * nn * k + 2L * (nn - mp);  // sample at t = t_{k+1} - mp h
      w_copy(sS, S, n * n);
      w_copy(sv, v, n);
      for (int st = 0; st < 4; ++st) {
        const long j = st == 0 ? j1 : (st == 3 ? j1 - 2 : j1 - 1);
        const R wk = (st == 0 || st == 3) ? h / R(6) : h / R(3);
        const R cn = st == 2 ? h : h / R(2);
        const R* Fj = kp.F_sampled ? (const R*)kp.F + (bk.s0 + j) * n * n : Fc;
        for (int e = lane_id(); e < n * n; e += 64) F[e] = Fj[e];
        for (int i = lane_id(); i < n; i += 64) {
          rv[i] = ((const R*)kp.r)[(bk.s0 + j) * n + i];
          cv[i] = cb ? cb[(bk.s0 + j) * n + i] : R(0);
        }
        if (kp.L_sampled) {
          const R* Lj = (const R*)kp.L + (bk.s0 + j) * n * nu;
          const R* W = cs + consts_off_W(n, nu);
          for (int e = lane_id(); e < n * nu; e += 64) {
            const int i = e / nu, l = e % nu;
            R a = R(0);
            for (int q2 = 0; q2 < nu; ++q2) a = fma(Lj[i * nu + q2], W[q2 * nu + l], a);
            Lc[e] = a;
          }
          wsync();
          w_gemm<kMfma<N, R>>(G, Lc, Lc, n, nu, n, false, true, R(1), R(0));
        } else {
          wsync();
        }
        // P = S G;  kS = -F^T S - S F - Q + P S (upper entries);  kv = -Q r - F^T v + P v + S c
        w_gemm<kMfma<N, R>>(P, sS, G, n, n, n, false, false, R(1), R(0));
        for (int e = lane_id(); e < n * n; e += 64) kS[e] = -Qs[e];
        wsync();
        w_gemm<kMfma<N, R>>(kS, F, sS, n, n, n, true, false, R(-1), R(1));
        w_gemm<kMfma<N, R>>(kS, sS, F, n, n, n, false, false, R(-1), R(1));
        w_gemm<kMfma<N, R>>(kS, P, sS, n, n, n, false, false, R(1), R(1));
        for (int i = lane_id(); i < n; i += 64) {
          R a = R(0);
          for (int l = 0; l < n; ++l) {
            a = fma(-Qs[i * n + l], rv[l], a);
            a = fma(-F[l * n + i], sv[l], a);
            a = fma(P[i * n + l], sv[l], a);
            a = fma(sS[i * n + l], cv[l], a);
          }
          kv[i] = a;
        }
        wsync();
        for (int e = lane_id(); e < n * n; e += 64) {
          const int i = e / n, q2 = e % n;
          const R ks = kS[(i < q2 ? i : q2) * n + (i < q2 ? q2 : i)];
          aS[e] = st == 0 ? fma(-wk, ks, S[e]) : fma(-wk, ks, aS[e]);
          if (st < 3) sS[e] = fma(-cn, ks, S[e]);
        }
        for (int i = lane_id(); i < n; i += 64) {
          av[i] = st == 0 ? fma(-wk, kv[i], v[i]) : fma(-wk, kv[i], av[i]);
          if (st < 3) sv[i] = fma(-cn, kv[i], v[i]);
        }
        wsync();
      }
      const long node = (long)nn * k + (nn - mp - 1);
      for (int e = lane_id(); e < n * n; e += 64) {
        S[e] = aS[e];
        Sdp[node * n * n + e] = aS[e];
      }
      for (int i = lane_id(); i < n; i += 64) {
        v[i] = av[i];
        vdp[node * n + i] = av[i];
      }
      wsync();
    }
  }

  // ---- block-boundary nodes ----
  auto boundary = [&](long kb) {
    const long node = (long)nn * kb;
    for (int e = lane_id(); e < n * n; e += 64) {
      Sn[e] = Sp[kb * n * n + e];
      Sdp[node * n * n + e] = Sn[e];
    }
    for (int i = lane_id(); i < n; i += 64) {
      vn[i] = vp[kb * n + i];
      xn[i] = xp[kb * n + i];
      vdp[node * n + i] = vn[i];
      xdp[node * n + i] = xn[i];
    }
    wsync();
    emit_u(node);
  };
  boundary(k);
  for (int i = lane_id(); i < n; i += 64) xk[i] = xn[i];
  if (k == T - 1) boundary(T);
  wsync();

  // ---- forward sweep: Theorem 9 parts, x and u at nodes n k + 1 .. n k + n - 1 ----
  WT<R> y = wt_at(sh, n), ac = wt_at(sh + kTupW, n), st = wt_at(sh + 2 * kTupW, n);
  wt_identity(y, n);
  auto step = [&](int m) {
    const long node = (long)nn * k + m + 1;
    for (int e = lane_id(); e < n * n; e += 64) Sn[e] = Sdp[node * n * n + e];
    for (int i = lane_id(); i < n; i += 64) vn[i] = vdp[node * n + i];
    wsync();
    w_m2_state<N>(y.A, y.b, y.C, xk, Sn, vn, Mn, Bn, xn, n);
    for (int i = lane_id(); i < n; i += 64) xdp[node * n + i] = xn[i];
    emit_u(node);
  };
  wb_fwd_steps<N, R, false>(kp, bk, k, nn - 1, y, ac, st, sh + 3 * kTupW, step);
}

// ------------------------------------------------------------------------------------------
// The whole solve after the element build (both trees, every level) in one launch over a work
// queue.  The items are the nodes of every stage, in the order of the per-level launches above:
//   value reduce (levels 1 .. L), value top, value down (levels L - 1 .. 1), value bottom,
//   trajectory reduce (levels 2 .. L), trajectory top, trajectory down (L - 1 .. 1), bottom,
// problem-minor within a stage.  Every wave takes the next item from a counter, waits until the
// items it reads from are done (their status words, set after their stores are complete), runs
// the body and marks its own item done.  An item only reads from items of earlier stages, which
// were taken from the counter earlier and whose waves are therefore running, so every wait ends;
// an item reads only what the items it waits for wrote or what those items waited for in turn.
// ------------------------------------------------------------------------------------------
enum WqKind : int { kWqVRed = 0, kWqVTop, kWqVDown, kWqVBot, kWqTRed, kWqTTop, kWqTDown, kWqTBot };

template <int N, class R>
__global__ __launch_bounds__(64) void kw_solve_queue(const KProb kp, const WQueue q,
                                                     const R* __restrict__ elts, R* __restrict__ S,
                                                     R* __restrict__ v, R* __restrict__ x,
                                                     R* __restrict__ u) {
  __shared__ R sh[WSh<N>::all];
  __shared__ int piv;
  const int lane = lane_id();
  unsigned it0 = 0;
  if (lane == 0) it0 = atomicAdd(q.done + q.total, 1u);  // the counter follows the status words
  const long it = (long)__shfl(it0, 0, 64);
  if (it >= q.total) return;
  int s = 0;
  while (s + 1 < q.nst && q.start[s + 1] <= it) ++s;
  const long B = kp.batch, L = q.levels;
  auto wcs = [&](long lv) { return (long)q.wcs[lv]; };  // nodes of level lv per node of lv + 1
  const int p = (int)((it - q.start[s]) % B);
  const long i = (it - q.start[s]) / B;
  // stage index of each kind (see the order above)
  auto st_vred = [&](long l) { return (int)(l - 1); };
  auto st_vdown = [&](long l) { return (int)(2 * L - l); };  // l = L - 1 .. 1
  const int st_vtop = (int)L, st_vbot = (int)(2 * L);
  auto st_tred = [&](long l) { return (int)(2 * L + l - 1); };  // l = 2 .. L
  auto st_tdown = [&](long l) { return (int)(4 * L - l); };     // l = L - 1 .. 1
  const int st_ttop = (int)(3 * L);
  // waits until nodes a .. b - 1 of stage t (problem p) are done
  auto wait = [&](int t, long a, long b) {
    const unsigned* f = q.done + q.start[t] + p;
    for (;;) {
      const unsigned d = a + lane < b ? lq_flag_load(f + (a + lane) * B) : 1u;
      if (__ballot(d == 0u) == 0ull) break;
      __builtin_amdgcn_s_sleep(1);
    }
    lq_acquire();
  };
  const int kind = q.kind[s];
  const long l = q.level[s];
  const R* e = elts;
  switch (kind) {
    case kWqVRed: {  // node i of level l from nodes i wcs(l - 1) .. of level l - 1
      const long b = wcs(l - 1);
      if (l > 1) wait(st_vred(l - 1), i * b, min(i * b + b, q.n[l - 1]));
      wb_vreduce<N, DevAcc>(sh, &piv, p, i, (int)b, l == 1, l == 1 ? e : (const R*)q.vtup[l - 1],
                            q.n[l - 1], (R*)q.vtup[l], q.n[l]);
      break;
    }
    case kWqVTop:
      wait(st_vred(L), 0, q.n[L]);
      wb_vtop<N, DevAcc>(sh, &piv, kp, p, (const R*)q.vtup[L], q.n[L], (R*)q.vval[L]);
      break;
    case kWqVDown:  // node i of level l + 1 -> its children at level l
      if (l + 1 == L)
        wait(st_vtop, 0, 1);
      else
        wait(st_vdown(l + 1), i / wcs(l + 1), i / wcs(l + 1) + 1);
      wb_vdown<N, DevAcc>(sh, &piv, p, i, (int)wcs(l), (const R*)q.vtup[l], q.n[l],
                          (const R*)q.vval[l + 1], q.n[l + 1], (R*)q.vval[l]);
      break;
    case kWqVBot:
      if (L == 1)
        wait(st_vtop, 0, 1);
      else
        wait(st_vdown(1), i / wcs(1), i / wcs(1) + 1);
      wb_vbottom<N, DevAcc>(sh, &piv, kp, p, i, (int)wcs(0), e, (const R*)q.vval[1], q.n[1], S, v,
                            (R*)q.tmap[1], (R*)q.bmap);
      break;
    case kWqTRed: {
      const long b = wcs(l - 1);
      wait(l == 2 ? st_vbot : st_tred(l - 1), i * b, min(i * b + b, q.n[l - 1]));
      wb_treduce<N, DevAcc>(sh, p, i, (int)b, (const R*)q.tmap[l - 1], q.n[l - 1], (R*)q.tmap[l],
                            q.n[l]);
      break;
    }
    case kWqTTop:
      wait(L == 1 ? st_vbot : st_tred(L), 0, q.n[L]);
      wb_ttop<N, DevAcc>(sh, kp, p, (const R*)q.tmap[L], q.n[L], (R*)q.tx[L]);
      break;
    case kWqTDown:
      if (l + 1 == L)
        wait(st_ttop, 0, 1);
      else
        wait(st_tdown(l + 1), i / wcs(l + 1), i / wcs(l + 1) + 1);
      wb_tdown<N, DevAcc>(sh, p, i, (int)wcs(l), (const R*)q.tmap[l], q.n[l],
                          (const R*)q.tx[l + 1], q.n[l + 1], (R*)q.tx[l]);
      break;
    case kWqTBot:
      if (L == 1)
        wait(st_ttop, 0, 1);
      else
        wait(st_tdown(1), i / wcs(1), i / wcs(1) + 1);
      wb_tbottom<N, DevAcc>(sh, &piv, kp, p, i, (int)wcs(0), e, S, v, (const R*)q.tx[1], q.n[1], x, u,
                            (const R*)q.bmap);
      break;
  }
  if (lane == 0) lq_flag_store(q.done + it, 1u);
}

}  // namespace

// ------------------------------------------------------------------------------------------
// Host orchestration of this path.
// ------------------------------------------------------------------------------------------

namespace {

template <int N, class R>
hipError_t wave_build_t(const KProb& kp, void* elts, hipStream_t s) {
  if constexpr (N <= 8 && sizeof(R) == 8)
    hipLaunchKernelGGL((kw_build_mfma8<N>), dim3((unsigned)((kp.T + 1) / 2), kp.batch), dim3(64), 0,
                       s, kp, (double*)elts);
  else if constexpr (N <= 8)
    hipLaunchKernelGGL((kw_build_rows<N, R>), dim3((unsigned)((kp.T + 7) / 8), kp.batch), dim3(64),
                       0, s, kp, (R*)elts);
  else if constexpr (kMfma<N, R>)
    hipLaunchKernelGGL(kw_build_mfma16<0>, dim3((unsigned)kp.T, kp.batch), dim3(64), 0, s, kp,
                       (double*)elts);
  else
    hipLaunchKernelGGL((kw_build<N, R>), dim3((unsigned)kp.T, kp.batch), dim3(64), 0, s, kp,
                       (R*)elts);
  return hipGetLastError();
}

template <int N, class R>
hipError_t wave_build_fwd_t(const KProb& kp, void* elts, hipStream_t s) {
  hipLaunchKernelGGL((kw_build_fwd<N, R>), dim3((unsigned)kp.T, kp.batch), dim3(64), 0, s, kp,
                     (R*)elts);
  return hipGetLastError();
}

template <int N, class R>
hipError_t wave_build_split_t(const KProb& kp, void* elts, hipStream_t s) {
  hipLaunchKernelGGL((kw_build_split<N, R>), dim3((unsigned)kp.T, kp.batch), dim3(64), 0, s, kp,
                     (R*)elts);
  return hipGetLastError();
}

template <int N, class R>
hipError_t wave_lti_prep_t(const KProb& kp, void* tab, hipStream_t s) {
  hipLaunchKernelGGL((kw_lti_prep<N, R>), dim3((unsigned)((2 * kp.n + 1) * N), kp.batch), dim3(64),
                     0, s, kp, (R*)tab);
  return hipGetLastError();
}

template <int N, class R>
hipError_t wave_lti_build_t(const KProb& kp, const void* tab, void* elts, hipStream_t s) {
  hipLaunchKernelGGL((kw_build_lti<N, R>), dim3((unsigned)kp.T, kp.batch), dim3(64), 0, s, kp,
                     (const R*)tab, (R*)elts);
  return hipGetLastError();
}

// Largest level (nodes x problems) that the value and Method 2 trees run on two waves per node:
// its workgroups hold two bodies' LDS each (51 KB at nx = 16 in FP64, three per CU), so wider
// levels, whose time is throughput rather than chain latency, keep one wave per node.
constexpr long kTwoWaveNodes = 512;

template <int N, class R>
hipError_t wave_method2_t(const KProb& kp, const WTree& t, const Work& w, const void* elts,
                          const void* S, const void* v, void* x, void* u, hipStream_t s) {
  const int n = N;
  const dim3 b(64);
  hipLaunchKernelGGL((kw_vreduce<N, R>), dim3((unsigned)t.n[1], kp.batch), b, 0, s, n, t.wc, 1,
                     (const R*)elts, t.n[0], (R*)w.vtup[1], t.n[1]);
  // Levels of few nodes on two waves per node, reduce and down-sweep alike (the reduce leaves
  // left pair products in the records the down-sweep reads).
  auto two_wave = [&](int l) { return t.wcs[l] == 4 && t.n[l + 1] * kp.batch <= kTwoWaveNodes; };
  for (int l = 1; l < t.levels; ++l) {
    if (two_wave(l))
      hipLaunchKernelGGL((kw_vreduce2<N, R, true>), dim3((unsigned)t.n[l + 1], kp.batch),
                         dim3(128), 0, s, t.wcs[l], (R*)w.vtup[l], t.n[l], (R*)w.vtup[l + 1],
                         t.n[l + 1]);
    else
      hipLaunchKernelGGL((kw_vreduce<N, R>), dim3((unsigned)t.n[l + 1], kp.batch), b, 0, s, n,
                         t.wcs[l], 0, (const R*)w.vtup[l], t.n[l], (R*)w.vtup[l + 1], t.n[l + 1]);
  }
  hipLaunchKernelGGL((kw_m2_top<N, R>), dim3(1, kp.batch), b, 0, s, (const R*)w.vtup[t.levels],
                     t.n[t.levels], (R*)w.vpart[t.levels]);
  for (int l = t.levels - 1; l >= 1; --l) {
    if (two_wave(l))
      hipLaunchKernelGGL((kw_m2_down2<N, R>), dim3((unsigned)t.n[l + 1], kp.batch), dim3(128), 0,
                         s, t.wcs[l], (const R*)w.vtup[l], t.n[l], (const R*)w.vpart[l + 1],
                         t.n[l + 1], (R*)w.vpart[l]);
    else
      hipLaunchKernelGGL((kw_m2_down<N, R>), dim3((unsigned)t.n[l + 1], kp.batch), b, 0, s,
                         t.wcs[l], (const R*)w.vtup[l], t.n[l], (const R*)w.vpart[l + 1],
                         t.n[l + 1], (R*)w.vpart[l]);
  }
  hipLaunchKernelGGL((kw_m2_bottom<N, R>), dim3((unsigned)t.n[1], kp.batch), b, 0, s, kp, t.wc,
                     (const R*)elts, (const R*)S, (const R*)v, (const R*)w.vpart[1], t.n[1],
                     (R*)x, (R*)u);
  return hipGetLastError();
}

template <int N, class R>
hipError_t wave_dense_t(const KProb& kp, const void* S, const void* v, const void* x, void* Sd,
                        void* vd, void* xd, void* ud, hipStream_t s) {
  hipLaunchKernelGGL((kw_dense<N, R>), dim3((unsigned)kp.T, kp.batch), dim3(64), 0, s, kp,
                     (const R*)S, (const R*)v, (const R*)x, (R*)Sd, (R*)vd, (R*)xd, (R*)ud);
  return hipGetLastError();
}

template <int N, class R>
hipError_t wave_value_t(const KProb& kp, const WTree& t, const Work& w, const void* elts, void* S,
                        void* v, void* maps1, hipStream_t s) {
  const int n = N, wc = t.wc;
  const dim3 b(64);
  hipLaunchKernelGGL((kw_vreduce<N, R>), dim3((unsigned)t.n[1], kp.batch), b, 0, s, n, wc, 1,
                     (const R*)elts, t.n[0], (R*)w.vtup[1], t.n[1]);
  // Levels of few nodes run on two waves per node (kw_vreduce2 / kw_vdown2); a level's
  // reduce and down-sweep take the same form (the two-wave reduce leaves pair products in the
  // records its down-sweep reads).
  auto two_wave = [&](int l) { return t.wcs[l] == 4 && t.n[l + 1] * kp.batch <= kTwoWaveNodes; };
  for (int l = 1; l < t.levels; ++l) {
    if (two_wave(l))
      hipLaunchKernelGGL((kw_vreduce2<N, R>), dim3((unsigned)t.n[l + 1], kp.batch), dim3(128), 0,
                         s, t.wcs[l], (R*)w.vtup[l], t.n[l], (R*)w.vtup[l + 1], t.n[l + 1]);
    else
      hipLaunchKernelGGL((kw_vreduce<N, R>), dim3((unsigned)t.n[l + 1], kp.batch), b, 0, s, n,
                         t.wcs[l], 0, (const R*)w.vtup[l], t.n[l], (R*)w.vtup[l + 1], t.n[l + 1]);
  }
  hipLaunchKernelGGL((kw_vtop<N, R>), dim3(1, kp.batch), b, 0, s, kp, (const R*)w.vtup[t.levels],
                     t.n[t.levels], (R*)w.vval[t.levels]);
  for (int l = t.levels - 1; l >= 1; --l) {
    if (two_wave(l))
      hipLaunchKernelGGL((kw_vdown2<N, R>), dim3((unsigned)t.n[l + 1], kp.batch), dim3(128), 0,
                         s, t.wcs[l], (const R*)w.vtup[l], t.n[l], (const R*)w.vval[l + 1],
                         t.n[l + 1], (R*)w.vval[l]);
    else
      hipLaunchKernelGGL((kw_vdown<N, R>), dim3((unsigned)t.n[l + 1], kp.batch), b, 0, s, n,
                         t.wcs[l], (const R*)w.vtup[l], t.n[l], (const R*)w.vval[l + 1],
                         t.n[l + 1], (R*)w.vval[l]);
  }
  hipLaunchKernelGGL((kw_vbottom<N, R>), dim3((unsigned)t.n[1], kp.batch), b, 0, s, kp, wc,
                     (const R*)elts, (const R*)w.vval[1], t.n[1], (R*)S, (R*)v, (R*)maps1,
                     (R*)(maps1 ? w.bmap : nullptr));
  return hipGetLastError();
}

template <int N, class R>
hipError_t wave_traj_t(const KProb& kp, const WTree& t, const Work& w, const void* elts,
                       const void* S, const void* v, void* x, void* u, bool maps_ready,
                       hipStream_t s) {
  const int n = N, wc = t.wc;
  const dim3 b(64);
  if (!maps_ready)
    hipLaunchKernelGGL((kw_tbottom_reduce<N, R>), dim3((unsigned)t.n[1], kp.batch), b, 0, s, kp,
                       wc, (const R*)elts, (const R*)S, (const R*)v, (R*)w.tmap[1], t.n[1]);
  for (int l = 1; l < t.levels; ++l)
    hipLaunchKernelGGL((kw_treduce<N, R>), dim3((unsigned)t.n[l + 1], kp.batch), b, 0, s, n,
                       t.wcs[l], (const R*)w.tmap[l], t.n[l], (R*)w.tmap[l + 1], t.n[l + 1]);
  hipLaunchKernelGGL((kw_ttop<N, R>), dim3(1, kp.batch), b, 0, s, kp, (const R*)w.tmap[t.levels],
                     t.n[t.levels], (R*)w.tx[t.levels]);
  for (int l = t.levels - 1; l >= 1; --l)
    hipLaunchKernelGGL((kw_tdown<N, R>), dim3((unsigned)t.n[l + 1], kp.batch), b, 0, s, n,
                       t.wcs[l], (const R*)w.tmap[l], t.n[l], (const R*)w.tx[l + 1], t.n[l + 1],
                       (R*)w.tx[l]);
  hipLaunchKernelGGL((kw_tbottom<N, R>), dim3((unsigned)t.n[1], kp.batch), b, 0, s, kp, wc,
                     (const R*)elts, (const R*)S, (const R*)v, (const R*)w.tx[1], t.n[1], (R*)x,
                     (R*)u, (const R*)(maps_ready ? w.bmap : nullptr));
  return hipGetLastError();
}

template <int N, class R>
hipError_t wave_solve_queue_t(const KProb& kp, const WQueue& q, const void* elts, void* S, void* v,
                              void* x, void* u, hipStream_t s) {
  hipLaunchKernelGGL((kw_solve_queue<N, R>), dim3((unsigned)q.total), dim3(64), 0, s, kp, q,
                     (const R*)elts, (R*)S, (R*)v, (R*)x, (R*)u);
  return hipGetLastError();
}

#ifndef LQT_SHARD
#define LQT_SHARD 0
#endif
static_assert(LQT_SHARD >= 0 && LQT_SHARD < kWaveShards, "LQT_SHARD out of range");

template <int N, class R>
struct Fns {
  static const WaveFns* get() {
    if constexpr (wave_shard(N, sizeof(R) == 4) == LQT_SHARD) {
      static const WaveFns f = {wave_build_t<N, R>,       wave_value_t<N, R>,
                                wave_traj_t<N, R>,        wave_solve_queue_t<N, R>,
                                wave_build_fwd_t<N, R>,   wave_build_split_t<N, R>,
                                wave_method2_t<N, R>,     wave_dense_t<N, R>,
                                wave_lti_prep_t<N, R>,    wave_lti_build_t<N, R>};
      return &f;
    } else {
      return nullptr;
    }
  }
};

template <class R>
const WaveFns* fns_for(int nx) {
  switch (nx) {
    case 5: return Fns<5, R>::get();
    case 6: return Fns<6, R>::get();
    case 7: return Fns<7, R>::get();
    case 8: return Fns<8, R>::get();
    case 9: return Fns<9, R>::get();
    case 10: return Fns<10, R>::get();
    case 11: return Fns<11, R>::get();
    case 12: return Fns<12, R>::get();
    case 13: return Fns<13, R>::get();
    case 14: return Fns<14, R>::get();
    case 15: return Fns<15, R>::get();
    case 16: return Fns<16, R>::get();
  }
  return nullptr;
}

}  // namespace

template <>
const WaveFns* wave_fns_shard<LQT_SHARD>(int nx, int dtype) {
  return dtype == 0 ? fns_for<double>(nx) : fns_for<float>(nx);
}

}  // namespace lqt
