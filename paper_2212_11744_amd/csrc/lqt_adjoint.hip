// Adjoint of lqt_solve (1 <= nu <= nx <= 4): gradients of a loss L(x_0, ..., x_T) with
// respect to Q, R, the reference samples r, x0, Qf and rf; F and L constant or sampled, with or
// without a drift c (none of them differentiated).
//
// The forward scheme is: elements a_k from RK4 on Theorem 8 (Sec. IV-B); values
// (S_k, v_k) = a_k (x) (S_{k+1}, v_{k+1}) from the terminal value (Qf, Qf rf) (Theorem 6,
// Sec. IV-D); states x_{k+1} = Psi_k x_k + alpha_k with Psi_k = M_k^{-1} A_k,
// alpha_k = M_k^{-1} (b_k + C_k v_{k+1}), M_k = I + C_k S_{k+1} (Sec. IV-E).  Its exact discrete
// adjoint, with xbar_k = dL/dx_k given:
//   lambda_T = xbar_T,  lambda_k = xbar_k + Psi_k^T lambda_{k+1}            (reverse affine scan)
//   mu_k = M_k^{-T} lambda_{k+1}
//   (Sbar_0, vbar_0) = 0,
//   Sbar_{k+1} = Psi Sbar_k Psi^T - sym(Psi vbar_k alpha^T) - sym(C mu x_{k+1}^T),
//   vbar_{k+1} = Psi vbar_k + C mu                                         (forward scan)
// where Sbar_k, vbar_k are the total gradients with respect to S_k, v_k (the linear parts compose
// like the trajectory maps, so this recursion is itself an associative scan).  Per block, the
// gradient with respect to the element, with S = S_{k+1}, v = v_{k+1}, y = M^{-T} (v - S b),
// p = S x_{k+1} - v:
//   Jbar = Sbar_k, etabar = vbar_k,
//   Abar = 2 S Psi Sbar_k + y vbar_k^T + mu x_k^T,   bbar = -S Psi vbar_k + mu,
//   Cbar = -(S Psi) Sbar_k (S Psi)^T - sym(S Psi vbar_k y^T) - sym(mu p^T),
// and the element gradient is carried back through the RK4 steps of the block (discrete adjoint,
// the forward steps recomputed from the block's boundary values) to Q, G = L R^{-1} L^T and the
// reference samples; R gets -R^{-1} L^T Gbar L R^{-1}.  Matrix gradients are symmetric: the
// derivative for symmetric perturbations of Q, R, Qf.
#include "lane_math.hpp"
#include "lqt_internal.hpp"
#include "tree_scan.hpp"
#include "wave_tree.hpp"

namespace lqt {
namespace {

template <int N, int NU>
struct CS {
  static constexpr int G = 0, Lc = N * N, Kc = N * N + N * NU, W = N * N + 2 * N * NU,
                       Rinv = N * N + 2 * N * NU + NU * NU, size = N * N + 2 * N * NU + 2 * NU * NU;
};

constexpr int kT = 64;

__device__ inline long gidx() { return (long)blockIdx.x * blockDim.x + threadIdx.x; }

template <int N, class R>
LQT_DEV void Sfull(const R (&Sp)[Sym<N>::size], R (&S)[N][N]) {
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int j = 0; j < N; ++j) S[i][j] = Sp[Sym<N>::at(i, j)];
}

// Packed adjoint of a symmetric matrix from its symmetric gradient X: the stored entry (i, j),
// i < j, stands for both (i, j) and (j, i).
template <int N, class R>
LQT_DEV void pack_grad(const R (&X)[N][N], R (&P)[Sym<N>::size]) {
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int j = i; j < N; ++j) P[Sym<N>::at(i, j)] = i == j ? X[i][i] : X[i][j] + X[j][i];
}

// ------------------------------------------------------------------------------------------
// Algebras of the two adjoint scans.
// ------------------------------------------------------------------------------------------
// lambda scan: map lambda -> (I + P) lambda + q with P = Psi_k^T - I, q = xbar_k; backward.
template <int N, class R>
struct LamAlg {
  static constexpr bool kForward = false;
  static constexpr int NMAP = Lay<N>::NM, NST = N;
  using Map = Aff<N, R>;
  struct State {
    R x[N];
  };
  static LQT_DEV void identity(Map& m) { aff_identity(m); }
  static LQT_DEV void load(Map& m, const R* b, long k) { aff_load(m, b, k); }
  static LQT_DEV void store(const Map& m, R* b, long k) { aff_store(m, b, k); }
  // first covers the earlier interval: lambda at its left end = first(second(lambda right)).
  static LQT_DEV void chain(const Map& first, const Map& second, Map& out) {
    Map o = first;
    aff_after(o, second);
    out = o;
  }
  static LQT_DEV void apply(const Map& m, State& st) { aff_apply(m, st.x); }
  static LQT_DEV void sload(State& st, const R* b, long k) {
#pragma unroll
    for (int q = 0; q < N; ++q) st.x[q] = b[tix<N>(q, k)];
  }
  static LQT_DEV void sstore(const State& st, R* b, long k) {
#pragma unroll
    for (int q = 0; q < N; ++q) b[tix<N>(q, k)] = st.x[q];
  }
  static LQT_DEV void shfl_map(const Map& x, Map& y, int src) { shfl_aff(x, y, src); }
  static LQT_DEV void shfl_state(const State& x, State& y, int src) { shfl_vec<N, R>(x.x, y.x, src); }
  // aux: dL/dx [batch][T+1][N]; lambda_T = xbar_T.
  static LQT_DEV void init(const KProb& kp, const R* aux, int p, State& st) {
#pragma unroll
    for (int q = 0; q < N; ++q) st.x[q] = aux[((long)p * (kp.T + 1) + kp.T) * N + q];
  }
};

// (Sbar, vbar) scan: map (Sbar, vbar) -> (Psi Sbar Psi^T - sym(Psi vbar alpha^T) + FS,
// Psi vbar + Fv), Psi = I + P; forward.
template <int N, class R>
struct CongMap {
  R P[N][N];
  R a[N];
  R FS[Sym<N>::size];
  R Fv[N];
};

template <int N, class R>
LQT_DEV void cong_apply(const CongMap<N, R>& m, R (&Sb)[Sym<N>::size], R (&vb)[N]) {
  using Y = Sym<N>;
  R Ps[N][N];  // Psi Sbar
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int j = 0; j < N; ++j) {
      R s = Sb[Y::at(i, j)];
#pragma unroll
      for (int k = 0; k < N; ++k) s = fma(m.P[i][k], Sb[Y::at(k, j)], s);
      Ps[i][j] = s;
    }
  R pv[N];  // Psi vbar
#pragma unroll
  for (int i = 0; i < N; ++i) {
    R s = vb[i];
#pragma unroll
    for (int k = 0; k < N; ++k) s = fma(m.P[i][k], vb[k], s);
    pv[i] = s;
  }
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int j = i; j < N; ++j) {
      R s = Ps[i][j];  // (Psi Sbar) Psi^T = Ps (I + P^T)
#pragma unroll
      for (int k = 0; k < N; ++k) s = fma(Ps[i][k], m.P[j][k], s);
      s -= R(0.5) * (pv[i] * m.a[j] + pv[j] * m.a[i]);
      Sb[Y::at(i, j)] = s + m.FS[Y::at(i, j)];
    }
#pragma unroll
  for (int i = 0; i < N; ++i) vb[i] = pv[i] + m.Fv[i];
}

template <int N, class R>
struct CongAlg {
  static constexpr bool kForward = true;
  static constexpr int NS = Sym<N>::size;
  static constexpr int NMAP = N * N + 2 * N + NS, NST = NS + N;
  using Map = CongMap<N, R>;
  struct State {
    R S[Sym<N>::size];
    R v[N];
  };
  static LQT_DEV void identity(Map& m) {
#pragma unroll
    for (int i = 0; i < N; ++i) {
#pragma unroll
      for (int j = 0; j < N; ++j) m.P[i][j] = R(0);
      m.a[i] = R(0);
      m.Fv[i] = R(0);
    }
#pragma unroll
    for (int i = 0; i < NS; ++i) m.FS[i] = R(0);
  }
  static LQT_DEV void load(Map& m, const R* b, long k) {
#pragma unroll
    for (int i = 0; i < N; ++i) {
#pragma unroll
      for (int j = 0; j < N; ++j) m.P[i][j] = b[tix<NMAP>(i * N + j, k)];
      m.a[i] = b[tix<NMAP>(N * N + i, k)];
      m.Fv[i] = b[tix<NMAP>(N * N + N + NS + i, k)];
    }
#pragma unroll
    for (int i = 0; i < NS; ++i) m.FS[i] = b[tix<NMAP>(N * N + N + i, k)];
  }
  static LQT_DEV void store(const Map& m, R* b, long k) {
#pragma unroll
    for (int i = 0; i < N; ++i) {
#pragma unroll
      for (int j = 0; j < N; ++j) b[tix<NMAP>(i * N + j, k)] = m.P[i][j];
      b[tix<NMAP>(N * N + i, k)] = m.a[i];
      b[tix<NMAP>(N * N + N + NS + i, k)] = m.Fv[i];
    }
#pragma unroll
    for (int i = 0; i < NS; ++i) b[tix<NMAP>(N * N + N + i, k)] = m.FS[i];
  }
  // out = second after first: Psi = Psi2 Psi1, alpha = Psi2 alpha1 + alpha2,
  // F = L2(F1) + F2 with L2 the linear part of `second`.
  static LQT_DEV void chain(const Map& first, const Map& second, Map& out) {
    Map o;
    R FS[NS], Fv[N];
#pragma unroll
    for (int i = 0; i < NS; ++i) FS[i] = first.FS[i];
#pragma unroll
    for (int i = 0; i < N; ++i) Fv[i] = first.Fv[i];
    cong_apply(second, FS, Fv);  // L2(F1) + F2
#pragma unroll
    for (int i = 0; i < NS; ++i) o.FS[i] = FS[i];
#pragma unroll
    for (int i = 0; i < N; ++i) o.Fv[i] = Fv[i];
#pragma unroll
    for (int i = 0; i < N; ++i) {
#pragma unroll
      for (int j = 0; j < N; ++j) {
        R s = R(0);
#pragma unroll
        for (int k = 0; k < N; ++k) s = fma(second.P[i][k], first.P[k][j], s);
        o.P[i][j] = first.P[i][j] + second.P[i][j] + s;
      }
      R s = R(0);
#pragma unroll
      for (int k = 0; k < N; ++k) s = fma(second.P[i][k], first.a[k], s);
      o.a[i] = second.a[i] + first.a[i] + s;
    }
    out = o;
  }
  static LQT_DEV void apply(const Map& m, State& st) { cong_apply(m, st.S, st.v); }
  static LQT_DEV void sload(State& st, const R* b, long k) {
#pragma unroll
    for (int q = 0; q < NS; ++q) st.S[q] = b[tix<NST>(q, k)];
#pragma unroll
    for (int q = 0; q < N; ++q) st.v[q] = b[tix<NST>(NS + q, k)];
  }
  static LQT_DEV void sstore(const State& st, R* b, long k) {
#pragma unroll
    for (int q = 0; q < NS; ++q) b[tix<NST>(q, k)] = st.S[q];
#pragma unroll
    for (int q = 0; q < N; ++q) b[tix<NST>(NS + q, k)] = st.v[q];
  }
  static LQT_DEV void shfl_map(const Map& x, Map& y, int src) {
#pragma unroll
    for (int i = 0; i < N; ++i) {
#pragma unroll
      for (int j = 0; j < N; ++j) y.P[i][j] = shfl(x.P[i][j], src);
      y.a[i] = shfl(x.a[i], src);
      y.Fv[i] = shfl(x.Fv[i], src);
    }
#pragma unroll
    for (int i = 0; i < NS; ++i) y.FS[i] = shfl(x.FS[i], src);
  }
  static LQT_DEV void shfl_state(const State& x, State& y, int src) {
    shfl_val<N, R>(x.S, x.v, y.S, y.v, src);
  }
  static LQT_DEV void init(const KProb&, const R*, int, State& st) {
#pragma unroll
    for (int q = 0; q < NS; ++q) st.S[q] = R(0);
#pragma unroll
    for (int q = 0; q < N; ++q) st.v[q] = R(0);
  }
};

// ------------------------------------------------------------------------------------------
// Per-block pieces shared by the bottom kernels.
// ------------------------------------------------------------------------------------------
template <int N, class R>
struct BlockCtx {
  R S[Sym<N>::size];  // S_{k+1}
  R v[N];             // v_{k+1}
  R Pd[N][N];         // Psi_k - I
  R al[N];            // alpha_k
};

template <int N, class R>
LQT_DEV void block_ctx(const Tup<N, R>& a, const R* Sg, const R* vg, long k, BlockCtx<N, R>& c) {
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int j = i; j < N; ++j) c.S[Sym<N>::at(i, j)] = Sg[(k + 1) * N * N + i * N + j];
#pragma unroll
  for (int i = 0; i < N; ++i) c.v[i] = vg[(k + 1) * N + i];
  Aff<N, R> m;
  block_map<N, R>(a.A, a.b, a.C, c.S, c.v, m);
#pragma unroll
  for (int i = 0; i < N; ++i) {
#pragma unroll
    for (int j = 0; j < N; ++j) c.Pd[i][j] = m.P[i][j];
    c.al[i] = m.q[i];
  }
}

// Solve (I + S C) X = B for NB right-hand sides (I + S C = M^T).
template <int N, int NB, class R>
LQT_DEV void solve_MT(const Tup<N, R>& a, const R (&S)[Sym<N>::size], R (&B)[N][NB]) {
  R Mt[N][N];
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int j = 0; j < N; ++j) {
      R s = R(0);
#pragma unroll
      for (int k = 0; k < N; ++k) s = fma(S[Sym<N>::at(i, k)], a.C[Sym<N>::at(k, j)], s);
      Mt[i][j] = (i == j) ? R(1) + s : s;
    }
  gj_solve<N, NB, R>(Mt, B);
}

// (A) level 1 of the lambda scan: per lane, the composition of its blocks' maps
// lambda_k = Psi_k^T lambda_{k+1} + xbar_k.
template <int N, class R>
__global__ __launch_bounds__(kT) void k_adj_lam_bottom(const KProb kp, const R* __restrict__ elts,
                                                       const R* __restrict__ Sg,
                                                       const R* __restrict__ vg,
                                                       const R* __restrict__ xbar,
                                                       R* __restrict__ maps1, long n1) {
  const int p = blockIdx.y;
  const long i = gidx();
  if (i >= n1) return;
  const long T = kp.T;
  const R* ep = elts + (long)p * Lay<N>::NE * padt(T);
  const R* Sp = Sg + (long)p * (T + 1) * N * N;
  const R* vp = vg + (long)p * (T + 1) * N;
  const R* xb = xbar + (long)p * (T + 1) * N;
  const long j0 = i * kChunk, j1 = min(j0 + kChunk, T);
  Aff<N, R> acc;
  aff_identity(acc);
  for (long k = j1 - 1; k >= j0; --k) {
    Tup<N, R> a;
    tup_load(a, ep, k);
    BlockCtx<N, R> c;
    block_ctx<N, R>(a, Sp, vp, k, c);
    Aff<N, R> m;
#pragma unroll
    for (int r = 0; r < N; ++r) {
#pragma unroll
      for (int q = 0; q < N; ++q) m.P[r][q] = c.Pd[q][r];
      m.q[r] = xb[k * N + r];
    }
    LamAlg<N, R>::chain(m, acc, acc);
  }
  aff_store(acc, maps1 + (long)p * Lay<N>::NM * padt(n1), i);
}

// (C) lambda of every block and level 1 of the (Sbar, vbar) scan.
template <int N, class R>
__global__ __launch_bounds__(kT) void k_adj_cong_bottom(const KProb kp, const R* __restrict__ elts,
                                                        const R* __restrict__ Sg,
                                                        const R* __restrict__ vg,
                                                        const R* __restrict__ xg,
                                                        const R* __restrict__ xbar,
                                                        const R* __restrict__ lam1, long n1,
                                                        R* __restrict__ lam, R* __restrict__ maps1,
                                                        R* __restrict__ dx0) {
  using Y = Sym<N>;
  const int p = blockIdx.y;
  const long i = gidx();
  if (i >= n1) return;
  const long T = kp.T;
  const R* ep = elts + (long)p * Lay<N>::NE * padt(T);
  const R* Sp = Sg + (long)p * (T + 1) * N * N;
  const R* vp = vg + (long)p * (T + 1) * N;
  const R* xp = xg + (long)p * (T + 1) * N;
  const R* xb = xbar + (long)p * (T + 1) * N;
  R* lp = lam + (long)p * (T + 1) * N;
  R l[N];  // lambda at the right end of the lane's range
#pragma unroll
  for (int q = 0; q < N; ++q) l[q] = lam1[(long)p * N * padt(n1) + tix<N>(q, i)];
  const long j0 = i * kChunk, j1 = min(j0 + kChunk, T);
  if (j1 == T) {
#pragma unroll
    for (int q = 0; q < N; ++q) lp[T * N + q] = l[q];
  }
  CongMap<N, R> acc;
  CongAlg<N, R>::identity(acc);
  for (long k = j1 - 1; k >= j0; --k) {
    Tup<N, R> a;
    tup_load(a, ep, k);
    BlockCtx<N, R> c;
    block_ctx<N, R>(a, Sp, vp, k, c);
    R B[N][1];
#pragma unroll
    for (int q = 0; q < N; ++q) B[q][0] = l[q];
    solve_MT<N, 1, R>(a, c.S, B);  // mu = M^{-T} lambda_{k+1}
    R Cmu[N];
#pragma unroll
    for (int r = 0; r < N; ++r) {
      R s = R(0);
#pragma unroll
      for (int q = 0; q < N; ++q) s = fma(a.C[Y::at(r, q)], B[q][0], s);
      Cmu[r] = s;
    }
    CongMap<N, R> m;
#pragma unroll
    for (int r = 0; r < N; ++r) {
#pragma unroll
      for (int q = 0; q < N; ++q) m.P[r][q] = c.Pd[r][q];
      m.a[r] = c.al[r];
      m.Fv[r] = Cmu[r];
    }
    R x1[N];
#pragma unroll
    for (int q = 0; q < N; ++q) x1[q] = xp[(k + 1) * N + q];
#pragma unroll
    for (int r = 0; r < N; ++r)
#pragma unroll
      for (int q = r; q < N; ++q) m.FS[Y::at(r, q)] = R(-0.5) * (Cmu[r] * x1[q] + Cmu[q] * x1[r]);
    CongAlg<N, R>::chain(m, acc, acc);
    // lambda_k = Psi_k^T lambda_{k+1} + xbar_k
    R ln[N];
#pragma unroll
    for (int r = 0; r < N; ++r) {
      R s = l[r] + xb[k * N + r];
#pragma unroll
      for (int q = 0; q < N; ++q) s = fma(c.Pd[q][r], l[q], s);
      ln[r] = s;
    }
#pragma unroll
    for (int q = 0; q < N; ++q) {
      l[q] = ln[q];
      lp[k * N + q] = ln[q];
    }
  }
  if (j0 == 0 && dx0) {
#pragma unroll
    for (int q = 0; q < N; ++q) dx0[(long)p * N + q] = l[q];
  }
  CongAlg<N, R>::store(acc, maps1 + (long)p * CongAlg<N, R>::NMAP * padt(n1), i);
}

// (E1) element gradients of every block; the element array is overwritten with them.  The lane
// that owns block T - 1 also writes the terminal gradients.
template <int N, class R>
__global__ __launch_bounds__(kT) void k_adj_elem(const KProb kp, R* __restrict__ elts,
                                                 const R* __restrict__ Sg, const R* __restrict__ vg,
                                                 const R* __restrict__ xg, const R* __restrict__ lam,
                                                 const R* __restrict__ sv1, long n1,
                                                 R* __restrict__ dQf, R* __restrict__ drf) {
  using Y = Sym<N>;
  constexpr int NS = Y::size;
  const int p = blockIdx.y;
  const long i = gidx();
  if (i >= n1) return;
  const long T = kp.T;
  R* ep = elts + (long)p * Lay<N>::NE * padt(T);
  const R* Sp = Sg + (long)p * (T + 1) * N * N;
  const R* vp = vg + (long)p * (T + 1) * N;
  const R* xp = xg + (long)p * (T + 1) * N;
  const R* lp = lam + (long)p * (T + 1) * N;
  R Sb[NS], vb[N];
  {
    typename CongAlg<N, R>::State st;
    CongAlg<N, R>::sload(st, sv1 + (long)p * CongAlg<N, R>::NST * padt(n1), i);
#pragma unroll
    for (int q = 0; q < NS; ++q) Sb[q] = st.S[q];
#pragma unroll
    for (int q = 0; q < N; ++q) vb[q] = st.v[q];
  }
  const long j0 = i * kChunk, j1 = min(j0 + kChunk, T);
  for (long k = j0; k < j1; ++k) {
    Tup<N, R> a;
    tup_load(a, ep, k);
    BlockCtx<N, R> c;
    block_ctx<N, R>(a, Sp, vp, k, c);
    R S[N][N];
    Sfull<N, R>(c.S, S);
    R xk[N], xk1[N], lk1[N];
#pragma unroll
    for (int q = 0; q < N; ++q) {
      xk[q] = xp[k * N + q];
      xk1[q] = xp[(k + 1) * N + q];
      lk1[q] = lp[(k + 1) * N + q];
    }
    // mu = M^{-T} lambda_{k+1}, y = M^{-T} (v - S b)
    R B[N][2];
#pragma unroll
    for (int r = 0; r < N; ++r) {
      R s = c.v[r];
#pragma unroll
      for (int q = 0; q < N; ++q) s = fma(-S[r][q], a.b[q], s);
      B[r][0] = lk1[r];
      B[r][1] = s;
    }
    solve_MT<N, 2, R>(a, c.S, B);
    R SP[N][N];  // S Psi
#pragma unroll
    for (int r = 0; r < N; ++r)
#pragma unroll
      for (int q = 0; q < N; ++q) {
        R s = S[r][q];
#pragma unroll
        for (int m = 0; m < N; ++m) s = fma(S[r][m], c.Pd[m][q], s);
        SP[r][q] = s;
      }
    R SB[N][N];
    Sfull<N, R>(Sb, SB);
    R SPS[N][N];  // S Psi Sbar
#pragma unroll
    for (int r = 0; r < N; ++r)
#pragma unroll
      for (int q = 0; q < N; ++q) {
        R s = R(0);
#pragma unroll
        for (int m = 0; m < N; ++m) s = fma(SP[r][m], SB[m][q], s);
        SPS[r][q] = s;
      }
    R spv[N];  // S Psi vbar
#pragma unroll
    for (int r = 0; r < N; ++r) {
      R s = R(0);
#pragma unroll
      for (int q = 0; q < N; ++q) s = fma(SP[r][q], vb[q], s);
      spv[r] = s;
    }
    R pk1[N];  // S x_{k+1} - v
#pragma unroll
    for (int r = 0; r < N; ++r) {
      R s = -c.v[r];
#pragma unroll
      for (int q = 0; q < N; ++q) s = fma(S[r][q], xk1[q], s);
      pk1[r] = s;
    }
    Tup<N, R> g;
#pragma unroll
    for (int r = 0; r < N; ++r) {
#pragma unroll
      for (int q = 0; q < N; ++q)
        g.A[r][q] = R(2) * SPS[r][q] + B[r][1] * vb[q] + B[r][0] * xk[q];
      g.b[r] = B[r][0] - spv[r];
      g.e[r] = vb[r];
    }
    {
      R Cs[N][N];
#pragma unroll
      for (int r = 0; r < N; ++r)
#pragma unroll
        for (int q = 0; q < N; ++q) {
          R s = R(0);
#pragma unroll
          for (int m = 0; m < N; ++m) s = fma(SPS[r][m], SP[q][m], s);
          Cs[r][q] = -s - R(0.5) * (spv[r] * B[q][1] + spv[q] * B[r][1]) -
                     R(0.5) * (B[r][0] * pk1[q] + B[q][0] * pk1[r]);
        }
      pack_grad<N, R>(Cs, g.C);
      pack_grad<N, R>(SB, g.J);
    }
    tup_store(g, ep, k);
    // advance (Sbar, vbar) across block k
    CongMap<N, R> m;
    R Cmu[N];
#pragma unroll
    for (int r = 0; r < N; ++r) {
      R s = R(0);
#pragma unroll
      for (int q = 0; q < N; ++q) s = fma(a.C[Y::at(r, q)], B[q][0], s);
      Cmu[r] = s;
    }
#pragma unroll
    for (int r = 0; r < N; ++r) {
#pragma unroll
      for (int q = 0; q < N; ++q) m.P[r][q] = c.Pd[r][q];
      m.a[r] = c.al[r];
      m.Fv[r] = Cmu[r];
    }
#pragma unroll
    for (int r = 0; r < N; ++r)
#pragma unroll
      for (int q = r; q < N; ++q) m.FS[Y::at(r, q)] = R(-0.5) * (Cmu[r] * xk1[q] + Cmu[q] * xk1[r]);
    cong_apply(m, Sb, vb);
  }
  if (j1 == T) {
    // Qf enters through S_T = Qf and v_T = Qf rf.
    const R* Qf = (const R*)kp.Qf + (long)p * N * N;
    const R* rf = (const R*)kp.rf + (long)p * N;
    if (dQf) {
#pragma unroll
      for (int r = 0; r < N; ++r)
#pragma unroll
        for (int q = 0; q < N; ++q)
          dQf[(long)p * N * N + r * N + q] =
              Sb[Y::at(r, q)] + R(0.5) * (vb[r] * rf[q] + vb[q] * rf[r]);
    }
    if (drf) {
#pragma unroll
      for (int r = 0; r < N; ++r) {
        R s = R(0);
#pragma unroll
        for (int q = 0; q < N; ++q) s = fma(Qf[q * N + r], vb[q], s);
        drf[(long)p * N + r] = s;
      }
    }
  }
}

// ------------------------------------------------------------------------------------------
// (E2) RK4 discrete adjoint of the element build, one block per lane.
//
// Right-hand side of Theorem 8 on the (Ad, eta, J) part of a stage value (b and C never enter a
// right-hand side, so their adjoints pass through the steps unchanged):
//   K = G J - F, w = G eta, fAd = K + Ad K, fb = -(w + Ad w), fC = -(A G A^T) (upper),
//   feta = K^T eta - Q r, fJ = -Q + J K - F^T J (upper), A = I + Ad.
// F, G, Q are the same for every lane of a workgroup and are read from LDS.  Register use is
// kept low: the step's start value and the running sum of stage adjoints live in per-lane LDS
// slots, stage values are recomputed from the step's start value when their adjoint is formed,
// and the Q and G adjoints are accumulated as their symmetric parts (packed), which is all the
// symmetric gradients need.
// ------------------------------------------------------------------------------------------
template <int N, class R>
struct Stage {
  R A[N][N];
  R e[N];
  R J[Sym<N>::size];
};

template <int N>
struct StageLay {
  static constexpr int A = 0, E = N * N, J = N * N + N, size = N * N + N + Sym<N>::size;
};

// Per-lane LDS slot: value v of lane l at base[v * kT + l].
template <int N, class R>
LQT_DEV void stage_to_lds(const Stage<N, R>& y, R* base, int lane) {
  using L = StageLay<N>;
#pragma unroll
  for (int i = 0; i < N; ++i) {
#pragma unroll
    for (int q = 0; q < N; ++q) base[(L::A + i * N + q) * kT + lane] = y.A[i][q];
    base[(L::E + i) * kT + lane] = y.e[i];
  }
#pragma unroll
  for (int i = 0; i < Sym<N>::size; ++i) base[(L::J + i) * kT + lane] = y.J[i];
}

template <int N, class R>
LQT_DEV void stage_from_lds(Stage<N, R>& y, const R* base, int lane) {
  using L = StageLay<N>;
#pragma unroll
  for (int i = 0; i < N; ++i) {
#pragma unroll
    for (int q = 0; q < N; ++q) y.A[i][q] = base[(L::A + i * N + q) * kT + lane];
    y.e[i] = base[(L::E + i) * kT + lane];
  }
#pragma unroll
  for (int i = 0; i < Sym<N>::size; ++i) y.J[i] = base[(L::J + i) * kT + lane];
}

template <int N, class R>
LQT_DEV void stage_add_lds(const Stage<N, R>& y, R* base, int lane) {
  using L = StageLay<N>;
#pragma unroll
  for (int i = 0; i < N; ++i) {
#pragma unroll
    for (int q = 0; q < N; ++q) base[(L::A + i * N + q) * kT + lane] += y.A[i][q];
    base[(L::E + i) * kT + lane] += y.e[i];
  }
#pragma unroll
  for (int i = 0; i < Sym<N>::size; ++i) base[(L::J + i) * kT + lane] += y.J[i];
}

// Stage value of block k in a global buffer laid out [value][stride] (coalesced over blocks).
template <int N, class R>
LQT_DEV void stage_to_global(const Stage<N, R>& y, R* base, long stride, long k) {
  using L = StageLay<N>;
#pragma unroll
  for (int i = 0; i < N; ++i) {
#pragma unroll
    for (int q = 0; q < N; ++q) base[(L::A + i * N + q) * stride + k] = y.A[i][q];
    base[(L::E + i) * stride + k] = y.e[i];
  }
#pragma unroll
  for (int i = 0; i < Sym<N>::size; ++i) base[(L::J + i) * stride + k] = y.J[i];
}

template <int N, class R>
LQT_DEV void stage_from_global(Stage<N, R>& y, const R* base, long stride, long k) {
  using L = StageLay<N>;
#pragma unroll
  for (int i = 0; i < N; ++i) {
#pragma unroll
    for (int q = 0; q < N; ++q) y.A[i][q] = base[(L::A + i * N + q) * stride + k];
    y.e[i] = base[(L::E + i) * stride + k];
  }
#pragma unroll
  for (int i = 0; i < Sym<N>::size; ++i) y.J[i] = base[(L::J + i) * stride + k];
}

// Compiler-only memory barrier (no instruction): values written to LDS are read back from LDS.
LQT_DEV void lds_fence() { asm volatile("" ::: "memory"); }

template <int N, class R>
LQT_DEV void stage_zero(Stage<N, R>& y) {
#pragma unroll
  for (int i = 0; i < N; ++i) {
#pragma unroll
    for (int q = 0; q < N; ++q) y.A[i][q] = R(0);
    y.e[i] = R(0);
  }
#pragma unroll
  for (int i = 0; i < Sym<N>::size; ++i) y.J[i] = R(0);
}

// o = y + c k (A, eta, J parts)
template <int N, class R>
LQT_DEV void stage_axpy(const Stage<N, R>& y, R c, const Stage<N, R>& k, Stage<N, R>& o) {
#pragma unroll
  for (int i = 0; i < N; ++i) {
#pragma unroll
    for (int q = 0; q < N; ++q) o.A[i][q] = fma(c, k.A[i][q], y.A[i][q]);
    o.e[i] = fma(c, k.e[i], y.e[i]);
  }
#pragma unroll
  for (int i = 0; i < Sym<N>::size; ++i) o.J[i] = fma(c, k.J[i], y.J[i]);
}

// Coefficients of the right-hand side at one sample: F, G row-major N x N, the drift c
// (nullptr: none).
template <class R>
struct Cf {
  const R* F;
  const R* G;
  const R* c;
};

// Where the coefficients of sample j are.  SMP = false: constant F and G (one pointer each, the
// same for the whole wave) and no drift.  SMP = true: F + j fs, G + j gs (fs, gs zero for a
// constant one) and c + j N when c != nullptr.
template <int N, class R, bool SMP>
struct CoefSrc {
  const R* F;
  long fs;
  const R* G;
  long gs;
  const R* c;
  LQT_DEV Cf<R> at(long j) const {
    if constexpr (SMP)
      return {F + j * fs, G + j * gs, c ? c + j * N : nullptr};
    else
      return {F, G, nullptr};
  }
};

// The (Ad, eta, J) part of the right-hand side (D: a drift may be present).  Q: row-major.
template <int N, class R, bool D>
LQT_DEV void rhs_aej(const Stage<N, R>& y, const Cf<R>& cf, const R* Q, const R (&r)[N],
                     Stage<N, R>& f) {
  using Y = Sym<N>;
  const R* F = cf.F;
  const R* G = cf.G;
  R K[N][N];
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int q = 0; q < N; ++q) {
      R s = -F[i * N + q];
#pragma unroll
      for (int l = 0; l < N; ++l) s = fma(G[i * N + l], y.J[Y::at(l, q)], s);
      K[i][q] = s;
    }
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int q = 0; q < N; ++q) {
      R s = K[i][q];
#pragma unroll
      for (int l = 0; l < N; ++l) s = fma(y.A[i][l], K[l][q], s);
      f.A[i][q] = s;
    }
#pragma unroll
  for (int i = 0; i < N; ++i) {
    R s = R(0);
#pragma unroll
    for (int l = 0; l < N; ++l) {
      s = fma(K[l][i], y.e[l], s);
      s = fma(-Q[i * N + l], r[l], s);
    }
    if constexpr (D) {
      if (cf.c) {  // + J c
#pragma unroll
        for (int l = 0; l < N; ++l) s = fma(y.J[Y::at(i, l)], cf.c[l], s);
      }
    }
    f.e[i] = s;
  }
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int q = i; q < N; ++q) {
      R s = -Q[i * N + q];
#pragma unroll
      for (int l = 0; l < N; ++l) {
        s = fma(y.J[Y::at(i, l)], K[l][q], s);
        s = fma(-F[l * N + i], y.J[Y::at(l, q)], s);
      }
      f.J[Y::at(i, q)] = s;
    }
}

// Vector-Jacobian product of the right-hand side at stage value y.  The output adjoint has
// (Ad, eta, J) parts g and b, C parts c1 * yb_b, c1 * yb_C (packed upper C, J adjoints).
// Returns the adjoint of y's (Ad, eta, J) in `out`, accumulates the symmetric parts of the Q and
// G adjoints (packed, per-lane LDS slots Qs, Gs) and the adjoint of this stage's reference
// sample into rb.  The phases are ordered so that each temporary dies early (register pressure).
// With a drift (D and cf.c): w = G eta + c in the b right-hand side, and the J c term of the
// eta right-hand side adds g.eta c^T to the J adjoint.
template <int N, class R, bool D>
LQT_DEV void rhs_vjp(const Stage<N, R>& y, const Stage<N, R>& g, R c1, const R (&yb_b)[N],
                     const R (&yb_C)[Sym<N>::size], const Cf<R>& cf, const R* Q,
                     const R (&r)[N], Stage<N, R>& out, R* Qs, R* Gs, int lane, R (&rb)[N]) {
  using Y = Sym<N>;
  const R* F = cf.F;
  const R* G = cf.G;
  // Bs = Bc + Bc^T from the C adjoint (upper triangular Bc); Bj upper triangular from g.J.
  auto Bs = [&](int i, int l) -> R {
    return i == l ? R(2) * c1 * yb_C[Y::at(i, i)] : c1 * yb_C[Y::at(i, l)];
  };
  auto Bj = [&](int i, int l) -> R { return l >= i ? g.J[Y::at(i, l)] : R(0); };
  // K = G J - F
  R K[N][N];
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int q = 0; q < N; ++q) {
      R s = -F[i * N + q];
#pragma unroll
      for (int l = 0; l < N; ++l) s = fma(G[i * N + l], y.J[Y::at(l, q)], s);
      K[i][q] = s;
    }
  lds_fence();
  // Kb = (I + Ad)^T gA + eta ge^T + J Bj
  R Kb[N][N];
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int q = 0; q < N; ++q) {
      R s = fma(y.e[i], g.e[q], g.A[i][q]);
#pragma unroll
      for (int l = 0; l < N; ++l) {
        s = fma(y.A[l][i], g.A[l][q], s);
        s = fma(y.J[Y::at(i, l)], Bj(l, q), s);
      }
      Kb[i][q] = s;
    }
  // out.J: Jb = Bj K^T - F Bj + G Kb folded onto the packed entries as it is formed.
#pragma unroll
  for (int i = 0; i < Y::size; ++i) out.J[i] = R(0);
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int q = 0; q < N; ++q) {
      R s = R(0);
#pragma unroll
      for (int l = 0; l < N; ++l) {
        s = fma(Bj(i, l), K[q][l], s);
        s = fma(-F[i * N + l], Bj(l, q), s);
        s = fma(G[i * N + l], Kb[l][q], s);
      }
      if constexpr (D) {
        if (cf.c) s = fma(g.e[i], cf.c[q], s);
      }
      out.J[Y::at(i, q)] += s;
    }
  // Qs: symmetric parts of -ge r^T and of -Bj (upper entries).
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int q = i; q < N; ++q) {
      const R outer = R(0.5) * (g.e[i] * r[q] + g.e[q] * r[i]);
      Qs[Y::at(i, q) * kT + lane] -= outer + (i == q ? Bj(i, i) : R(0.5) * Bj(i, q));
    }
  lds_fence();
  // wb = -(I + Ad)^T gb,  w = G eta
  R wb[N], w[N];
#pragma unroll
  for (int i = 0; i < N; ++i) {
    R s = yb_b[i], t = R(0);
#pragma unroll
    for (int l = 0; l < N; ++l) {
      s = fma(y.A[l][i], yb_b[l], s);
      t = fma(G[i * N + l], y.e[l], t);
    }
    wb[i] = -c1 * s;
    if constexpr (D) {
      if (cf.c) t += cf.c[i];
    }
    w[i] = t;
  }
  // Gs: symmetric parts of Kb J and wb eta^T.
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int q = i; q < N; ++q) {
      R s = R(0), t = R(0);
#pragma unroll
      for (int l = 0; l < N; ++l) {
        s = fma(Kb[i][l], y.J[Y::at(l, q)], s);
        t = fma(Kb[q][l], y.J[Y::at(l, i)], t);
      }
      Gs[Y::at(i, q) * kT + lane] += R(0.5) * (s + t + wb[i] * y.e[q] + wb[q] * y.e[i]);
    }
  lds_fence();
  // out.eta = K ge + G wb;  rb -= Q ge
#pragma unroll
  for (int i = 0; i < N; ++i) {
    R s = R(0), t = R(0);
#pragma unroll
    for (int l = 0; l < N; ++l) {
      s = fma(K[i][l], g.e[l], s);
      s = fma(G[i * N + l], wb[l], s);
      t = fma(Q[i * N + l], g.e[l], t);
    }
    out.e[i] = s;
    rb[i] -= t;
  }
  lds_fence();
  // out.A = gA K^T - gb w^T - Bs A G, with A G = G + Ad G.
#pragma unroll
  for (int q = 0; q < N; ++q) {
    R AGq[N];  // column q of A G
#pragma unroll
    for (int l = 0; l < N; ++l) {
      R s = G[l * N + q];
#pragma unroll
      for (int m = 0; m < N; ++m) s = fma(y.A[l][m], G[m * N + q], s);
      AGq[l] = s;
    }
#pragma unroll
    for (int i = 0; i < N; ++i) {
      R s = -c1 * yb_b[i] * w[q];
#pragma unroll
      for (int l = 0; l < N; ++l) {
        s = fma(g.A[i][l], K[q][l], s);
        s = fma(-Bs(i, l), AGq[l], s);
      }
      out.A[i][q] = s;
    }
  }
  // Gs -= 1/2 A^T Bs A (already symmetric), column by column of Bs A.
#pragma unroll
  for (int q = 0; q < N; ++q) {
    R BsAq[N];
#pragma unroll
    for (int l = 0; l < N; ++l) {
      R s = Bs(l, q);
#pragma unroll
      for (int m = 0; m < N; ++m) s = fma(Bs(l, m), y.A[m][q], s);
      BsAq[l] = s;
    }
#pragma unroll
    for (int i = 0; i <= q; ++i) {
      R s = BsAq[i];
#pragma unroll
      for (int l = 0; l < N; ++l) s = fma(y.A[l][i], BsAq[l], s);
      Gs[Y::at(i, q) * kT + lane] = fma(R(-0.5), s, Gs[Y::at(i, q) * kT + lane]);
    }
  }
}

template <int N, class R>
LQT_DEV void sample_r(const R* rp, long j, R (&r)[N]) {
#pragma unroll
  for (int q = 0; q < N; ++q) r[q] = rp[j * N + q];
}

// One classical RK4 step of -h (hp = -h) from the sample j1 (stage 1) to j1 - 2 (stage 4).
template <int N, class R, bool SMP>
LQT_DEV void rk4_forward(Stage<N, R>& y, long j1, R hp, const R* rp,
                         const CoefSrc<N, R, SMP>& cs, const R* Q) {
  R r[N];
  Stage<N, R> acc, s, k;
  const R w6 = hp / R(6), w3 = hp / R(3);
  sample_r<N, R>(rp, j1, r);
  rhs_aej<N, R, SMP>(y, cs.at(j1), Q, r, k);
  stage_axpy(y, w6, k, acc);
  stage_axpy(y, R(0.5) * hp, k, s);
  sample_r<N, R>(rp, j1 - 1, r);
  lds_fence();
  rhs_aej<N, R, SMP>(s, cs.at(j1 - 1), Q, r, k);
  stage_axpy(acc, w3, k, acc);
  stage_axpy(y, R(0.5) * hp, k, s);
  lds_fence();
  rhs_aej<N, R, SMP>(s, cs.at(j1 - 1), Q, r, k);
  stage_axpy(acc, w3, k, acc);
  stage_axpy(y, hp, k, s);
  sample_r<N, R>(rp, j1 - 2, r);
  lds_fence();
  rhs_aej<N, R, SMP>(s, cs.at(j1 - 2), Q, r, k);
  stage_axpy(acc, w6, k, y);
}

// Stage value `stage` (2, 3 or 4) of the RK4 step starting at y (samples j1, j1 - 1).
template <int N, class R, bool SMP>
LQT_DEV void stage_value(const Stage<N, R>& y, int stage, long j1, R hp, const R* rp,
                         const CoefSrc<N, R, SMP>& cs, const R* Q, Stage<N, R>& s) {
  R r[N];
  Stage<N, R> k;
  sample_r<N, R>(rp, j1, r);
  rhs_aej<N, R, SMP>(y, cs.at(j1), Q, r, k);
  stage_axpy(y, R(0.5) * hp, k, s);
  if (stage == 2) return;
  sample_r<N, R>(rp, j1 - 1, r);
  lds_fence();
  rhs_aej<N, R, SMP>(s, cs.at(j1 - 1), Q, r, k);
  stage_axpy(y, R(0.5) * hp, k, s);
  if (stage == 3) return;
  lds_fence();
  rhs_aej<N, R, SMP>(s, cs.at(j1 - 1), Q, r, k);
  stage_axpy(y, hp, k, s);
}

// Sampled L: the G adjoint of one stage (packed symmetric, per-lane slots gL) becomes the adjoint
// of W = R^{-1} through G = L W L^T at the stage's sample: Wbar += L^T Gbar L (packed symmetric,
// slots wL); gL is cleared for the next stage.
template <int N, int NU, class R>
LQT_DEV void wbar_stage(R* gL, const R* L, R* wL, int lane) {
  using Y = Sym<N>;
  using U = Sym<NU>;
  R GL[N][NU];
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int m = 0; m < NU; ++m) {
      R s = R(0);
#pragma unroll
      for (int l = 0; l < N; ++l) s = fma(gL[Y::at(i, l) * kT + lane], L[l * NU + m], s);
      GL[i][m] = s;
    }
#pragma unroll
  for (int a = 0; a < NU; ++a)
#pragma unroll
    for (int b = a; b < NU; ++b) {
      R s = R(0);
#pragma unroll
      for (int i = 0; i < N; ++i) s = fma(L[i * NU + a], GL[i][b], s);
      wL[U::at(a, b) * kT + lane] += s;
    }
#pragma unroll
  for (int i = 0; i < Y::size; ++i) gL[i * kT + lane] = R(0);
}

// g = c1 * yb + c2 * sn on the (Ad, eta, J) parts.
template <int N, class R>
LQT_DEV void stage_seed(R c1, const Tup<N, R>& yb, R c2, const Stage<N, R>& sn, Stage<N, R>& g) {
#pragma unroll
  for (int i = 0; i < N; ++i) {
#pragma unroll
    for (int q = 0; q < N; ++q) g.A[i][q] = fma(c2, sn.A[i][q], c1 * yb.A[i][q]);
    g.e[i] = fma(c2, sn.e[i], c1 * yb.e[i]);
  }
#pragma unroll
  for (int i = 0; i < Sym<N>::size; ++i) g.J[i] = fma(c2, sn.J[i], c1 * yb.J[i]);
}

// SMP: sampled F or L, or a drift c (per-lane coefficients at every stage; gsamp holds G at every
// sample when L is sampled).  Otherwise F, G are the problem's constants.
template <int N, int NU, class R, bool SMP>
__global__ __launch_bounds__(kT) void k_adj_rk4(const KProb kp, const R* __restrict__ abar,
                                               R* __restrict__ dr, R* __restrict__ bnd,
                                               R* __restrict__ wsum, R* __restrict__ ckpt,
                                               int ckpt_ready, const R* __restrict__ cF,
                                               const R* __restrict__ cG,
                                               const R* __restrict__ cQ,
                                               const R* __restrict__ gsamp) {
  using Y = Sym<N>;
  using U = Sym<NU>;
  constexpr int NS = Y::size, SL = StageLay<N>::size, NW = SMP ? U::size : 1;
  // per-lane slots: step start value, running sum of stage adjoints, symmetric Q and G adjoints
  // (40 KB in FP64 at nx = 4, so four workgroups fit the 160 KB of LDS of a CU; F, G and Q are
  // read through the scalar cache instead of being staged here); with sampled L also the
  // adjoint of R^{-1} (wL), the G adjoint then holding one stage's part at a time
  __shared__ R yL[SL * kT], aL[SL * kT], qL[NS * kT], gL[NS * kT], wL[NW * kT];
  const int p = blockIdx.y;
  const long k = gidx();
  const long T = kp.T;
  const int lane = threadIdx.x;
  const int n = kp.n;
  const long nsamp = 2L * n * T + 1;
  const R* rp = (const R*)kp.r + (long)p * nsamp * N;
#pragma unroll
  for (int i = 0; i < NS; ++i) {
    qL[i * kT + lane] = R(0);
    gL[i * kT + lane] = R(0);
  }
#pragma unroll
  for (int i = 0; i < NW; ++i) wL[i * kT + lane] = R(0);
  CoefSrc<N, R, SMP> cs;
  cs.F = cF;
  cs.fs = 0;
  cs.G = cG + (long)p * CS<N, NU>::size;
  cs.gs = 0;
  cs.c = nullptr;
  const bool Lsmp = SMP && kp.L_sampled;
  const R* Lp = Lsmp ? (const R*)kp.L + (long)p * nsamp * N * NU : nullptr;  // sampled L
  if constexpr (SMP) {
    if (kp.F_sampled) {
      cs.F = (const R*)kp.F + (long)p * nsamp * N * N;
      cs.fs = N * N;
    }
    if (kp.L_sampled) {
      cs.G = gsamp + (long)p * nsamp * N * N;
      cs.gs = N * N;
    }
    if (kp.has_c) cs.c = (const R*)kp.c + (long)p * nsamp * N;
  }
  const R* vQ = cQ + (long)p * N * N;
  R* vq = qL;
  R* vg = gL;
  // Compiler memory barriers below keep the per-lane LDS slots in LDS: without them the values
  // stored there would be forwarded in registers and raise register pressure.
  if (k < T) {
    const R* tg = (const R*)kp.t + (long)p * (T + 1);
    const R hp = -(tg[k + 1] - tg[k]) / R(n);
    const R w6 = hp / R(6), w3 = hp / R(3);
    Tup<N, R> yb;
    tup_load(yb, abar + (long)p * Lay<N>::NE * padt(T), k);
    R* drp = dr + (long)p * nsamp * N;
    // Sample j1 of step m (its first stage) is sample j1 - 2 of step m + 1 (its last stage):
    // the stage-1 adjoint is carried to the next (earlier) step and written once.
    R carry[N];
#pragma unroll
    for (int q = 0; q < N; ++q) carry[q] = R(0);
    // Step start values: with a checkpoint buffer, y_1 .. y_{n-1} are read from it (layout
    // [problem][step - 1][value][block], coalesced over the blocks of a wave), written by the
    // element build of the backward pass (ckpt_ready) or else by one forward pass here; without
    // a buffer, y_m is recomputed from y_0 = 0 for every step.
    const long ck_stride = padt(T);
    R* ckp = ckpt ? ckpt + (long)p * (n - 1) * SL * ck_stride : nullptr;
    if (ckp && !ckpt_ready) {
      Stage<N, R> y;
      stage_zero(y);
#pragma unroll 1
      for (int mm = 0; mm < n - 1; ++mm) {
        rk4_forward(y, 2L * n * k + 2L * (n - mm), hp, rp, cs, vQ);
        stage_to_global(y, ckp + (long)mm * SL * ck_stride, ck_stride, k);
      }
    }
#pragma unroll 1
    for (int m = n - 1; m >= 0; --m) {
      const long j1 = 2L * n * k + 2L * (n - m);
      {
        Stage<N, R> y;
        stage_zero(y);
        if (ckp && m > 0) {
          stage_from_global(y, ckp + (long)(m - 1) * SL * ck_stride, ck_stride, k);
        } else if (!ckp) {
#pragma unroll 1
          for (int mm = 0; mm < m; ++mm)
            rk4_forward(y, 2L * n * k + 2L * (n - mm), hp, rp, cs, vQ);
        }
        stage_to_lds(y, yL, lane);
        Stage<N, R> z;
        stage_zero(z);
        stage_to_lds(z, aL, lane);
      }
      lds_fence();
      // Reference-sample adjoints: j1 (stage 1), j1 - 1 (stages 2, 3), j1 - 2 (stage 4).  The
      // block's first sample (step n - 1, stage 4) and last sample (step 0, stage 1) are shared
      // with the neighbouring blocks and summed by k_adj_bnd; sample j1 of step m is sample
      // j1 - 2 of step m + 1, so the stage-1 adjoint is carried to the next (earlier) step.
      Stage<N, R> sn;  // adjoint of the later stage's input
      // stage 4: kbar4 = w6 ybar
      {
        Stage<N, R> y, s, g;
        R r[N], rbs[N];
        stage_from_lds(y, yL, lane);
        stage_value(y, 4, j1, hp, rp, cs, vQ, s);
        stage_zero(sn);
        stage_seed(w6, yb, R(0), sn, g);
        sample_r<N, R>(rp, j1 - 2, r);
#pragma unroll
        for (int q = 0; q < N; ++q) rbs[q] = R(0);
        rhs_vjp<N, R, SMP>(s, g, w6, yb.b, yb.C, cs.at(j1 - 2), vQ, r, sn, vq, vg, lane, rbs);
        if (Lsmp) wbar_stage<N, NU, R>(gL, Lp + (j1 - 2) * N * NU, wL, lane);
        stage_add_lds(sn, aL, lane);
        if (m == n - 1) {
#pragma unroll
          for (int q = 0; q < N; ++q) bnd[((long)p * T + k) * 2 * N + q] = rbs[q];
        } else {
#pragma unroll
          for (int q = 0; q < N; ++q) drp[(j1 - 2) * N + q] = rbs[q] + carry[q];
        }
      }
      lds_fence();
      // stage 3: kbar3 = w3 ybar + h s4bar
      {
        Stage<N, R> y, s, g;
        R r[N], rbs[N];
        stage_from_lds(y, yL, lane);
        stage_value(y, 3, j1, hp, rp, cs, vQ, s);
        stage_seed(w3, yb, hp, sn, g);
        sample_r<N, R>(rp, j1 - 1, r);
#pragma unroll
        for (int q = 0; q < N; ++q) rbs[q] = R(0);
        rhs_vjp<N, R, SMP>(s, g, w3, yb.b, yb.C, cs.at(j1 - 1), vQ, r, sn, vq, vg, lane, rbs);
        if (Lsmp) wbar_stage<N, NU, R>(gL, Lp + (j1 - 1) * N * NU, wL, lane);
        stage_add_lds(sn, aL, lane);
#pragma unroll
        for (int q = 0; q < N; ++q) drp[(j1 - 1) * N + q] = rbs[q];
      }
      lds_fence();
      // stage 2: kbar2 = w3 ybar + h/2 s3bar
      {
        Stage<N, R> y, s, g;
        R r[N], rbs[N];
        stage_from_lds(y, yL, lane);
        stage_value(y, 2, j1, hp, rp, cs, vQ, s);
        stage_seed(w3, yb, R(0.5) * hp, sn, g);
        sample_r<N, R>(rp, j1 - 1, r);
#pragma unroll
        for (int q = 0; q < N; ++q) rbs[q] = drp[(j1 - 1) * N + q];
        rhs_vjp<N, R, SMP>(s, g, w3, yb.b, yb.C, cs.at(j1 - 1), vQ, r, sn, vq, vg, lane, rbs);
        if (Lsmp) wbar_stage<N, NU, R>(gL, Lp + (j1 - 1) * N * NU, wL, lane);
        stage_add_lds(sn, aL, lane);
#pragma unroll
        for (int q = 0; q < N; ++q) drp[(j1 - 1) * N + q] = rbs[q];
      }
      lds_fence();
      // stage 1: kbar1 = w6 ybar + h/2 s2bar, at the step's start value
      {
        Stage<N, R> y, g;
        R r[N];
        stage_from_lds(y, yL, lane);
        stage_seed(w6, yb, R(0.5) * hp, sn, g);
        sample_r<N, R>(rp, j1, r);
#pragma unroll
        for (int q = 0; q < N; ++q) carry[q] = R(0);
        rhs_vjp<N, R, SMP>(y, g, w6, yb.b, yb.C, cs.at(j1), vQ, r, sn, vq, vg, lane, carry);
        if (Lsmp) wbar_stage<N, NU, R>(gL, Lp + j1 * N * NU, wL, lane);
        stage_add_lds(sn, aL, lane);
      }
      lds_fence();
      // ybar of the step's start value: ybar + sum of the stage-input adjoints
      {
        Stage<N, R> a;
        stage_from_lds(a, aL, lane);
#pragma unroll
        for (int i = 0; i < N; ++i) {
#pragma unroll
          for (int q = 0; q < N; ++q) yb.A[i][q] += a.A[i][q];
          yb.e[i] += a.e[i];
        }
#pragma unroll
        for (int i = 0; i < NS; ++i) yb.J[i] += a.J[i];
      }
    }
#pragma unroll
    for (int q = 0; q < N; ++q) bnd[((long)p * T + k) * 2 * N + N + q] = carry[q];
  }
  // Wave sums of the symmetric Q and G adjoints (deterministic, one record per wave); with sampled
  // L the G part of the record holds the adjoint of R^{-1} instead (packed, nu (nu + 1) / 2).
  R Qs[NS], Gs[NS];
#pragma unroll
  for (int i = 0; i < NS; ++i) {
    R a = qL[i * kT + lane];
    R b = Lsmp ? (i < U::size ? wL[(i < NW ? i : 0) * kT + lane] : R(0)) : gL[i * kT + lane];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      a += __shfl_xor(a, off, 64);
      b += __shfl_xor(b, off, 64);
    }
    Qs[i] = a;
    Gs[i] = b;
  }
  if (lane == 0) {
    const long nw = (T + kT - 1) / kT;
    R* ws = wsum + ((long)p * nw + blockIdx.x) * 2 * NS;
#pragma unroll
    for (int i = 0; i < NS; ++i) {
      ws[i] = Qs[i];
      ws[NS + i] = Gs[i];
    }
  }
}

// Reference samples on block boundaries: sample 2 n k is the last of block k - 1 and the first
// of block k.
template <int N, class R>
__global__ __launch_bounds__(kT) void k_adj_bnd(const KProb kp, const R* __restrict__ bnd,
                                               R* __restrict__ dr) {
  const int p = blockIdx.y;
  const long k = gidx();
  const long T = kp.T;
  if (k > T) return;
  const long nsamp = 2L * kp.n * T + 1;
  R* drp = dr + (long)p * nsamp * N;
#pragma unroll
  for (int q = 0; q < N; ++q) {
    R s = R(0);
    if (k < T) s += bnd[((long)p * T + k) * 2 * N + q];
    if (k > 0) s += bnd[((long)p * T + k - 1) * 2 * N + N + q];
    drp[2L * kp.n * k * N + q] = s;
  }
}

// Per problem: Q and G adjoints summed over the waves, symmetrised; R from G = L R^{-1} L^T:
// Rbar = -Kc Gbar Kc^T with Kc = R^{-1} L^T.
template <int N, int NU, class R>
__global__ __launch_bounds__(kT) void k_adj_sum(const KProb kp, const R* __restrict__ wsum,
                                               R* __restrict__ dQ, R* __restrict__ dR) {
  using Y = Sym<N>;
  constexpr int NS = Y::size;
  const int p = blockIdx.y;
  const int lane = threadIdx.x;
  const long nw = (kp.T + kT - 1) / kT;
  R acc[2 * NS];
#pragma unroll
  for (int i = 0; i < 2 * NS; ++i) acc[i] = R(0);
  for (long w = lane; w < nw; w += kT) {
    const R* ws = wsum + ((long)p * nw + w) * 2 * NS;
#pragma unroll
    for (int i = 0; i < 2 * NS; ++i) acc[i] += ws[i];
  }
#pragma unroll
  for (int i = 0; i < 2 * NS; ++i) {
    R a = acc[i];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) a += __shfl_xor(a, off, 64);
    acc[i] = a;
  }
  if (lane != 0) return;
  R Gs[N][N];
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int q = 0; q < N; ++q) {
      dQ[(long)p * N * N + i * N + q] = acc[Y::at(i, q)];
      Gs[i][q] = acc[NS + Y::at(i, q)];
    }
  const R* cs = (const R*)kp.consts + (long)p * CS<N, NU>::size;
  if (kp.L_sampled) {
    // G = L(t) W L(t)^T sample by sample: the record holds Wbar (W = R^{-1}, packed);
    // Rbar = -W Wbar W
    using U = Sym<NU>;
    const R* Wi = cs + CS<N, NU>::Rinv;
    R WB[NU][NU];
#pragma unroll
    for (int a = 0; a < NU; ++a)
#pragma unroll
      for (int m = 0; m < NU; ++m) {
        R t = R(0);
#pragma unroll
        for (int q = 0; q < NU; ++q) t = fma(Wi[a * NU + q], acc[NS + U::at(q, m)], t);
        WB[a][m] = t;
      }
#pragma unroll
    for (int a = 0; a < NU; ++a)
#pragma unroll
      for (int m = 0; m < NU; ++m) {
        R t = R(0);
#pragma unroll
        for (int q = 0; q < NU; ++q) t = fma(WB[a][q], Wi[q * NU + m], t);
        dR[(long)p * NU * NU + a * NU + m] = -t;
      }
    return;
  }
  R KG[NU][N];
#pragma unroll
  for (int l = 0; l < NU; ++l)
#pragma unroll
    for (int q = 0; q < N; ++q) {
      R s = R(0);
#pragma unroll
      for (int i = 0; i < N; ++i) s = fma(cs[CS<N, NU>::Kc + l * N + i], Gs[i][q], s);
      KG[l][q] = s;
    }
#pragma unroll
  for (int l = 0; l < NU; ++l)
#pragma unroll
    for (int m = 0; m < NU; ++m) {
      R s = R(0);
#pragma unroll
      for (int q = 0; q < N; ++q) s = fma(KG[l][q], cs[CS<N, NU>::Kc + m * N + q], s);
      dR[(long)p * NU * NU + l * NU + m] = -s;
    }
}

// G(t) = L(t) R^{-1} L(t)^T at every sample of a problem with sampled L (full N x N).
template <int N, int NU, class R>
__global__ __launch_bounds__(kT) void k_adj_gsamp(const KProb kp, R* __restrict__ gsamp) {
  const int p = blockIdx.y;
  const long j = gidx();
  const long nsamp = 2L * kp.n * kp.T + 1;
  if (j >= nsamp) return;
  const R* L = (const R*)kp.L + ((long)p * nsamp + j) * N * NU;
  const R* Wi = (const R*)kp.consts + (long)p * CS<N, NU>::size + CS<N, NU>::Rinv;
  R LW[N][NU];
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int m = 0; m < NU; ++m) {
      R t = R(0);
#pragma unroll
      for (int q = 0; q < NU; ++q) t = fma(L[i * NU + q], Wi[q * NU + m], t);
      LW[i][m] = t;
    }
  R* g = gsamp + ((long)p * nsamp + j) * N * N;
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int q = 0; q < N; ++q) {
      R t = R(0);
#pragma unroll
      for (int m = 0; m < NU; ++m) t = fma(LW[i][m], L[q * NU + m], t);
      g[i * N + q] = t;
    }
}

// ------------------------------------------------------------------------------------------
// Launchers.
// ------------------------------------------------------------------------------------------
inline dim3 lanes(long n, int batch) { return dim3((unsigned)((n + kT - 1) / kT), (unsigned)batch, 1); }
inline dim3 waves(long w, int batch) { return dim3((unsigned)w, (unsigned)batch, 1); }

template <int N, int NU, class R>
struct A {
  static hipError_t lam_bottom(const KProb& kp, const void* elts, const void* S, const void* v,
                               const void* xbar, void* maps1, long n1, hipStream_t s) {
    hipLaunchKernelGGL((k_adj_lam_bottom<N, R>), lanes(n1, kp.batch), dim3(kT), 0, s, kp,
                       (const R*)elts, (const R*)S, (const R*)v, (const R*)xbar, (R*)maps1, n1);
    return hipGetLastError();
  }
  static hipError_t lam_up(const KProb& kp, const void* src, long n_src, void* part, void* dst,
                           long n_dst, hipStream_t s) {
    hipLaunchKernelGGL((k_up<LamAlg<N, R>, R>), waves(n_dst, kp.batch), dim3(kT), 0, s,
                       (const R*)src, n_src, (R*)part, (R*)dst, n_dst);
    return hipGetLastError();
  }
  static hipError_t lam_top(const KProb& kp, const void* xbar, const void* src, long n,
                            void* out, hipStream_t s) {
    hipLaunchKernelGGL((k_top<LamAlg<N, R>, R>), dim3(1, kp.batch, 1), dim3(kT), 0, s, kp,
                       (const R*)xbar, (const R*)src, n, (R*)out);
    return hipGetLastError();
  }
  static hipError_t lam_down(const KProb& kp, const void* src, long n_child, const void* part,
                             const void* st_par, long n_par, void* st_child, hipStream_t s) {
    hipLaunchKernelGGL((k_down<LamAlg<N, R>, R>), waves(n_par, kp.batch), dim3(kT), 0, s,
                       (const R*)src, n_child, (const R*)part, (const R*)st_par, n_par,
                       (R*)st_child);
    return hipGetLastError();
  }
  static hipError_t cong_bottom(const KProb& kp, const void* elts, const void* S, const void* v,
                                const void* x, const void* xbar, const void* lam1, long n1,
                                void* lam, void* maps1, void* dx0, hipStream_t s) {
    hipLaunchKernelGGL((k_adj_cong_bottom<N, R>), lanes(n1, kp.batch), dim3(kT), 0, s, kp,
                       (const R*)elts, (const R*)S, (const R*)v, (const R*)x, (const R*)xbar,
                       (const R*)lam1, n1, (R*)lam, (R*)maps1, (R*)dx0);
    return hipGetLastError();
  }
  static hipError_t cong_up(const KProb& kp, const void* src, long n_src, void* part, void* dst,
                            long n_dst, hipStream_t s) {
    hipLaunchKernelGGL((k_up<CongAlg<N, R>, R>), waves(n_dst, kp.batch), dim3(kT), 0, s,
                       (const R*)src, n_src, (R*)part, (R*)dst, n_dst);
    return hipGetLastError();
  }
  static hipError_t cong_top(const KProb& kp, const void* src, long n, void* out, hipStream_t s) {
    hipLaunchKernelGGL((k_top<CongAlg<N, R>, R>), dim3(1, kp.batch, 1), dim3(kT), 0, s, kp,
                       (const R*)nullptr, (const R*)src, n, (R*)out);
    return hipGetLastError();
  }
  static hipError_t cong_down(const KProb& kp, const void* src, long n_child, const void* part,
                              const void* st_par, long n_par, void* st_child, hipStream_t s) {
    hipLaunchKernelGGL((k_down<CongAlg<N, R>, R>), waves(n_par, kp.batch), dim3(kT), 0, s,
                       (const R*)src, n_child, (const R*)part, (const R*)st_par, n_par,
                       (R*)st_child);
    return hipGetLastError();
  }
  static hipError_t elem(const KProb& kp, void* elts, const void* S, const void* v,
                         const void* x, const void* lam, const void* sv1, long n1, void* dQf,
                         void* drf, hipStream_t s) {
    hipLaunchKernelGGL((k_adj_elem<N, R>), lanes(n1, kp.batch), dim3(kT), 0, s, kp, (R*)elts,
                       (const R*)S, (const R*)v, (const R*)x, (const R*)lam, (const R*)sv1, n1,
                       (R*)dQf, (R*)drf);
    return hipGetLastError();
  }
  static hipError_t rk4(const KProb& kp, const void* abar, void* dr, void* bnd, void* wsum,
                        void* ckpt, bool ckpt_ready, void* gsamp, hipStream_t s) {
    if (kp.L_sampled) {
      hipLaunchKernelGGL((k_adj_gsamp<N, NU, R>), lanes(2L * kp.n * kp.T + 1, kp.batch), dim3(kT),
                         0, s, kp, (R*)gsamp);
      const hipError_t e = hipGetLastError();
      if (e != hipSuccess) return e;
    }
    if (kp.F_sampled || kp.L_sampled || kp.has_c)
      hipLaunchKernelGGL((k_adj_rk4<N, NU, R, true>), lanes(kp.T, kp.batch), dim3(kT), 0, s, kp,
                         (const R*)abar, (R*)dr, (R*)bnd, (R*)wsum, (R*)ckpt, (int)ckpt_ready,
                         (const R*)kp.F, (const R*)kp.consts + CS<N, NU>::G, (const R*)kp.Q,
                         (const R*)gsamp);
    else
      hipLaunchKernelGGL((k_adj_rk4<N, NU, R, false>), lanes(kp.T, kp.batch), dim3(kT), 0, s, kp,
                         (const R*)abar, (R*)dr, (R*)bnd, (R*)wsum, (R*)ckpt, (int)ckpt_ready,
                         (const R*)kp.F, (const R*)kp.consts + CS<N, NU>::G, (const R*)kp.Q,
                         (const R*)nullptr);
    return hipGetLastError();
  }
  static hipError_t finish(const KProb& kp, const void* bnd, void* dr, const void* wsum, void* dQ,
                           void* dR, hipStream_t s) {
    hipLaunchKernelGGL((k_adj_bnd<N, R>), lanes(kp.T + 1, kp.batch), dim3(kT), 0, s, kp,
                       (const R*)bnd, (R*)dr);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_adj_sum<N, NU, R>), dim3(1, kp.batch, 1), dim3(kT), 0, s, kp,
                       (const R*)wsum, (R*)dQ, (R*)dR);
    return hipGetLastError();
  }
  static const AdjOps* ops() {
    static const AdjOps o = {lam_bottom, lam_up,   lam_top,  lam_down, cong_bottom,
                             cong_up,    cong_top, cong_down, elem,    rk4,
                             finish};
    return &o;
  }
};

template <class R>
const AdjOps* adj_for(int nx, int nu) {
  switch (nx * 8 + nu) {
    case 1 * 8 + 1: return A<1, 1, R>::ops();
    case 2 * 8 + 1: return A<2, 1, R>::ops();
    case 2 * 8 + 2: return A<2, 2, R>::ops();
    case 3 * 8 + 1: return A<3, 1, R>::ops();
    case 3 * 8 + 2: return A<3, 2, R>::ops();
    case 3 * 8 + 3: return A<3, 3, R>::ops();
    case 4 * 8 + 1: return A<4, 1, R>::ops();
    case 4 * 8 + 2: return A<4, 2, R>::ops();
    case 4 * 8 + 3: return A<4, 3, R>::ops();
    case 4 * 8 + 4: return A<4, 4, R>::ops();
    default: return nullptr;
  }
}

}  // namespace

const AdjOps* adj_ops(int nx, int nu, int dtype) {
  return dtype == 0 ? adj_for<double>(nx, nu) : adj_for<float>(nx, nu);
}

}  // namespace lqt
