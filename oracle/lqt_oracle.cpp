// TEST INFRASTRUCTURE ONLY.
//
// Plain, sequential, double-precision reference ("oracle") for the parallel-in-time solver of the
// continuous-time linear quadratic tracker of Sarkka & Garcia-Fernandez, "Temporal parallelisation
// of the HJB equation and continuous-time linear quadratic control".  Only the test-suite, the
// smoke check and the CPU-baseline leg of the benchmark load this library; the GPU library never
// links, includes or calls it, and it shares no code with it.
//
// Everything here is written for a reader checking it against the paper by eye: dense matrices of
// runtime size, straight loops, Gaussian elimination with partial pivoting, no
// blocking, no fusion and no reordering beyond what the paper's formulas state.
//
// Problem (Sec. II-B, the LQT problem, with H = I so that Q = H^T X H and the reference r lives in
// state space; the terminal weight is Qf = H_f^T X_f H_f with reference rf):
//     dx/dt = F(t) x + L(t) u + c(t),
//     cost  = 1/2 (x(tf) - rf)^T Qf (x(tf) - rf)
//             + int 1/2 (x - r)^T Q (x - r) + 1/2 u^T R u dt.
// Discretisation (the reading shared by the GPU path): T blocks [t_k, t_{k+1}], each integrated
// with n classical RK4 steps of h_k = (t_{k+1} - t_k)/n; r, and F, L, c when time-varying, are
// given at the half-step times t_k + j h_k / 2 (j = 0..2n, global index 2 n k + j).
//
// Functions (each cites the passage it follows):
//   element_backward  - Theorem 8 (Sec. IV-B, backward conditional LQT ODEs) with the boundary
//                       values of a zero-length interval, RK4 in s from t_{k+1} down to t_k.
//   element_forward   - Theorem 9 (Sec. IV-C, forward conditional LQT ODEs), RK4 in tau from t_k
//                       up to t_{k+1}.
//   element_split     - the block split in two (Sec. IV-D): Theorem 9 over the first floor(n/2)
//                       steps, Theorem 8 over the remaining ones, joined by Lemma 7.
//   combine           - Lemma 7 (Sec. IV-A, combination rule of LQT conditional value functions).
//   value_functions   - Theorem 6 (Sec. III-D; suffix products a_k x ... x a_T) with the terminal
//                       element of Sec. IV-D, folded sequentially from the right.
//   trajectory        - optimal trajectory recovery (Sec. IV-E): x_{k+1} is the minimiser over z
//                       of V(x_k, t_k; z, t_{k+1}) + V(z, t_{k+1}), i.e. the Method 2 formula
//                       applied to one block, which is the closed-loop block map of Method 1;
//                       control from the LQT optimal control law (Sec. II-B).
//   trajectory_method2- Method 2 of Sec. IV-E with prefix products a_0 x ... x a_{k-1}.
//   dense_output      - values inside the blocks (Sec. VI-A, parallel method): S, v by RK4 on the
//                       S, v ODEs of Sec. II-B backwards over each block from its right-end value;
//                       x from the intermediate A, b, C of Theorem 9 combined with V(., tau) by
//                       the Method 2 formula (Sec. IV-E); u by the control law (Sec. II-B).
//   oracle_riccati    - the sequential baseline of Sec. VI-A: RK4 on the S, v ODEs of Sec. II-B
//                       on a fine grid, then RK4 on the closed-loop state ODE.
//   objective_*       - derivatives of sum_k <W_k, x_k> with respect to Q, R, r, x0, Qf, rf, by
//                       forward-mode dual numbers (exact JVP of the discrete scheme) and by a
//                       reverse sweep over a recorded tape (the sequential adjoint).
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

namespace oracle {

// ------------------------------------------------------------------------------------------
// Scalar types: double, forward-mode dual numbers, reverse-mode tape variables.
// ------------------------------------------------------------------------------------------
struct Dual {
  double v = 0.0, d = 0.0;
  Dual() {}
  Dual(double x) : v(x), d(0.0) {}
  Dual(double x, double dx) : v(x), d(dx) {}
};
inline Dual operator+(Dual a, Dual b) { return Dual(a.v + b.v, a.d + b.d); }
inline Dual operator-(Dual a, Dual b) { return Dual(a.v - b.v, a.d - b.d); }
inline Dual operator-(Dual a) { return Dual(-a.v, -a.d); }
inline Dual operator*(Dual a, Dual b) { return Dual(a.v * b.v, a.d * b.v + a.v * b.d); }
inline Dual operator/(Dual a, Dual b) {
  double q = a.v / b.v;
  return Dual(q, (a.d - q * b.d) / b.v);
}

struct Tape {
  std::vector<int> p1, p2;
  std::vector<double> w1, w2;
  int push(int a, double wa, int b, double wb) {
    p1.push_back(a);
    w1.push_back(wa);
    p2.push_back(b);
    w2.push_back(wb);
    return (int)p1.size() - 1;
  }
};
static Tape* g_tape = nullptr;

struct Var {
  int id = -1;  // -1: a constant, not on the tape
  double v = 0.0;
  Var() {}
  Var(double x) : id(-1), v(x) {}
};
inline Var mkvar(double v, int a, double wa, int b, double wb) {
  Var r(v);
  if (a >= 0 || b >= 0) r.id = g_tape->push(a, wa, b, wb);
  return r;
}
inline Var leaf(double v) {
  Var r(v);
  r.id = g_tape->push(-1, 0.0, -1, 0.0);
  return r;
}
inline Var operator+(Var a, Var b) { return mkvar(a.v + b.v, a.id, 1.0, b.id, 1.0); }
inline Var operator-(Var a, Var b) { return mkvar(a.v - b.v, a.id, 1.0, b.id, -1.0); }
inline Var operator-(Var a) { return mkvar(-a.v, a.id, -1.0, -1, 0.0); }
inline Var operator*(Var a, Var b) { return mkvar(a.v * b.v, a.id, b.v, b.id, a.v); }
inline Var operator/(Var a, Var b) {
  double q = a.v / b.v;
  return mkvar(q, a.id, 1.0 / b.v, b.id, -q / b.v);
}

inline double value(double x) { return x; }
inline double value(const Dual& x) { return x.v; }
inline double value(const Var& x) { return x.v; }

// ------------------------------------------------------------------------------------------
// Dense matrices of runtime size (vectors are n x 1 matrices).
// ------------------------------------------------------------------------------------------
template <class S>
struct Mat {
  int r = 0, c = 0;
  std::vector<S> a;  // row-major, r * c entries
  Mat() {}
  Mat(int rows, int cols) : r(rows), c(cols), a((size_t)rows * cols, S(0.0)) {}
  S& operator()(int i, int j) { return a[(size_t)i * c + j]; }
  const S& operator()(int i, int j) const { return a[(size_t)i * c + j]; }
};

template <class S>
Mat<S> eye(int n) {
  Mat<S> m(n, n);
  for (int i = 0; i < n; ++i) m(i, i) = S(1.0);
  return m;
}
template <class S>
Mat<S> mul(const Mat<S>& x, const Mat<S>& y) {
  Mat<S> m(x.r, y.c);
  for (int i = 0; i < x.r; ++i)
    for (int j = 0; j < y.c; ++j) {
      S s(0.0);
      for (int k = 0; k < x.c; ++k) s = s + x(i, k) * y(k, j);
      m(i, j) = s;
    }
  return m;
}
template <class S>
Mat<S> tr(const Mat<S>& x) {
  Mat<S> m(x.c, x.r);
  for (int i = 0; i < x.r; ++i)
    for (int j = 0; j < x.c; ++j) m(j, i) = x(i, j);
  return m;
}
template <class S>
Mat<S> add(const Mat<S>& x, const Mat<S>& y) {
  Mat<S> m(x.r, x.c);
  for (int i = 0; i < x.r; ++i)
    for (int j = 0; j < x.c; ++j) m(i, j) = x(i, j) + y(i, j);
  return m;
}
template <class S>
Mat<S> sub(const Mat<S>& x, const Mat<S>& y) {
  Mat<S> m(x.r, x.c);
  for (int i = 0; i < x.r; ++i)
    for (int j = 0; j < x.c; ++j) m(i, j) = x(i, j) - y(i, j);
  return m;
}
template <class S>
Mat<S> neg(const Mat<S>& x) {
  Mat<S> m(x.r, x.c);
  for (int i = 0; i < x.r; ++i)
    for (int j = 0; j < x.c; ++j) m(i, j) = -x(i, j);
  return m;
}
template <class S>
Mat<S> scale(double s, const Mat<S>& x) {
  Mat<S> m(x.r, x.c);
  for (int i = 0; i < x.r; ++i)
    for (int j = 0; j < x.c; ++j) m(i, j) = S(s) * x(i, j);
  return m;
}

// y + a k
template <class S>
Mat<S> axpy_m(const Mat<S>& y, double a, const Mat<S>& k) {
  return add(y, scale(a, k));
}
// Copy the upper triangle onto the lower one (the stored form of a symmetric matrix).
template <class S>
Mat<S> sym_upper(const Mat<S>& x) {
  Mat<S> m = x;
  for (int i = 0; i < x.r; ++i)
    for (int j = 0; j < i; ++j) m(i, j) = x(j, i);
  return m;
}
// Solve M X = B by Gaussian elimination with partial pivoting (largest |pivot|, first row on
// ties) and back substitution.
template <class S>
Mat<S> solve(Mat<S> M, Mat<S> B) {
  const int n = M.r;
  for (int col = 0; col < n; ++col) {
    int p = col;
    for (int i = col + 1; i < n; ++i)
      if (std::fabs(value(M(i, col))) > std::fabs(value(M(p, col)))) p = i;
    if (p != col) {
      for (int j = 0; j < n; ++j) {
        S t = M(col, j);
        M(col, j) = M(p, j);
        M(p, j) = t;
      }
      for (int j = 0; j < B.c; ++j) {
        S t = B(col, j);
        B(col, j) = B(p, j);
        B(p, j) = t;
      }
    }
    for (int i = col + 1; i < n; ++i) {
      S f = M(i, col) / M(col, col);
      for (int j = col; j < n; ++j) M(i, j) = M(i, j) - f * M(col, j);
      for (int j = 0; j < B.c; ++j) B(i, j) = B(i, j) - f * B(col, j);
    }
  }
  Mat<S> X(n, B.c);
  for (int j = 0; j < B.c; ++j)
    for (int i = n - 1; i >= 0; --i) {
      S s = B(i, j);
      for (int k = i + 1; k < n; ++k) s = s - M(i, k) * X(k, j);
      X(i, j) = s / M(i, i);
    }
  return X;
}

// ------------------------------------------------------------------------------------------
// Problem data converted to the scalar type.
// ------------------------------------------------------------------------------------------
}  // namespace oracle


extern "C" {
// Mirrors the Python-side ctypes structure.  Arrays are row-major doubles.
typedef struct {
  int32_t nx, nu, T, n;
  int32_t F_sampled, L_sampled, has_c;
  const double* t;   // [T+1]
  const double* F;   // [nx*nx] or [2nT+1][nx*nx]
  const double* L;   // [nx*nu] or [2nT+1][nx*nu]
  const double* c;   // null or [2nT+1][nx]
  const double* Q;   // [nx*nx]
  const double* R;   // [nu*nu]
  const double* r;   // [2nT+1][nx]
  const double* Qf;  // [nx*nx]
  const double* rf;  // [nx]
  const double* x0;  // [nx]
} oracle_problem;

// Tangent (dual) or seed directions for the differentiable inputs; null members are zero.
typedef struct {
  const double *Q, *R, *r, *Qf, *rf, *x0;
} oracle_inputs_tangent;
}

namespace oracle {

template <class S>
struct Prob {
  int nx = 0, nu = 0, T = 0, n = 0;
  bool F_sampled = false, L_sampled = false, has_c = false;
  const double* t = nullptr;
  const double *F = nullptr, *L = nullptr, *c = nullptr;  // not differentiated
  Mat<S> Q, R, Qf, rf, x0;
  std::vector<S> r;  // [2nT+1][nx]
  long nsamp() const { return 2L * n * T + 1; }
};

template <class S>
S make_input(double v, const double* tangent, long i);
template <>
double make_input<double>(double v, const double*, long) { return v; }
template <>
Dual make_input<Dual>(double v, const double* tangent, long i) {
  return Dual(v, tangent ? tangent[i] : 0.0);
}
template <>
Var make_input<Var>(double v, const double*, long) { return leaf(v); }

template <class S>
Mat<S> load_mat(const double* src, int rows, int cols, const double* tangent) {
  Mat<S> m(rows, cols);
  for (int i = 0; i < rows; ++i)
    for (int j = 0; j < cols; ++j) m(i, j) = make_input<S>(src[i * cols + j], tangent, i * cols + j);
  return m;
}

template <class S>
Prob<S> load_problem(const oracle_problem* p, const oracle_inputs_tangent* tg) {
  Prob<S> q;
  q.nx = p->nx;
  q.nu = p->nu;
  q.T = p->T;
  q.n = p->n;
  q.F_sampled = p->F_sampled != 0;
  q.L_sampled = p->L_sampled != 0;
  q.has_c = p->has_c != 0;
  q.t = p->t;
  q.F = p->F;
  q.L = p->L;
  q.c = p->c;
  q.Q = load_mat<S>(p->Q, q.nx, q.nx, tg ? tg->Q : nullptr);
  q.R = load_mat<S>(p->R, q.nu, q.nu, tg ? tg->R : nullptr);
  q.Qf = load_mat<S>(p->Qf, q.nx, q.nx, tg ? tg->Qf : nullptr);
  q.rf = load_mat<S>(p->rf, q.nx, 1, tg ? tg->rf : nullptr);
  q.x0 = load_mat<S>(p->x0, q.nx, 1, tg ? tg->x0 : nullptr);
  long ns = q.nsamp() * q.nx;
  q.r.resize(ns);
  for (long i = 0; i < ns; ++i) q.r[i] = make_input<S>(p->r[i], tg ? tg->r : nullptr, i);
  return q;
}

template <class S>
Mat<S> F_at(const Prob<S>& p, long j) {
  const double* src = p.F_sampled ? p.F + j * p.nx * p.nx : p.F;
  Mat<S> m(p.nx, p.nx);
  for (int i = 0; i < p.nx; ++i)
    for (int k = 0; k < p.nx; ++k) m(i, k) = S(src[i * p.nx + k]);
  return m;
}
template <class S>
Mat<S> L_at(const Prob<S>& p, long j) {
  const double* src = p.L_sampled ? p.L + j * p.nx * p.nu : p.L;
  Mat<S> m(p.nx, p.nu);
  for (int i = 0; i < p.nx; ++i)
    for (int k = 0; k < p.nu; ++k) m(i, k) = S(src[i * p.nu + k]);
  return m;
}
template <class S>
Mat<S> c_at(const Prob<S>& p, long j) {
  Mat<S> m(p.nx, 1);
  if (p.has_c)
    for (int i = 0; i < p.nx; ++i) m(i, 0) = S(p.c[j * p.nx + i]);
  return m;
}
template <class S>
Mat<S> r_at(const Prob<S>& p, long j) {
  Mat<S> m(p.nx, 1);
  for (int i = 0; i < p.nx; ++i) m(i, 0) = p.r[j * p.nx + i];
  return m;
}

// ------------------------------------------------------------------------------------------
// Conditional value function parameters (A, b, C, eta, J) of the dual form in Section 4.1.
// ------------------------------------------------------------------------------------------
template <class S>
struct Elem {
  Mat<S> A, b, C, eta, J;
};

// Zero-length interval: A = I, b = 0, C = 0, eta = 0, J = 0 (boundary values, Sec. IV-B).
template <class S>
Elem<S> identity_element(int nx) {
  Elem<S> e;
  e.A = eye<S>(nx);
  e.b = Mat<S>(nx, 1);
  e.C = Mat<S>(nx, nx);
  e.eta = Mat<S>(nx, 1);
  e.J = Mat<S>(nx, nx);
  return e;
}

template <class S>
Elem<S> axpy(const Elem<S>& y, double a, const Elem<S>& k) {
  Elem<S> o;
  o.A = add(y.A, scale(a, k.A));
  o.b = add(y.b, scale(a, k.b));
  o.C = add(y.C, scale(a, k.C));
  o.eta = add(y.eta, scale(a, k.eta));
  o.J = add(y.J, scale(a, k.J));
  return o;
}

template <class S>
Mat<S> G_at(const Prob<S>& p, long j) {  // L U^{-1} L^T
  Mat<S> L = L_at(p, j);
  return mul(L, solve(p.R, tr(L)));
}

// Theorem 8 (Sec. IV-B): derivatives with respect to the lower time limit s.
template <class S>
Elem<S> thm2_rhs(const Prob<S>& p, long j, const Elem<S>& y) {
  Mat<S> F = F_at(p, j), c = c_at(p, j), r = r_at(p, j), G = G_at(p, j);
  const Mat<S>& Q = p.Q;
  Elem<S> d;
  d.A = sub(mul(mul(y.A, G), y.J), mul(y.A, F));
  d.b = sub(neg(mul(mul(y.A, G), y.eta)), mul(y.A, c));
  d.C = neg(mul(mul(y.A, G), tr(y.A)));
  d.eta = add(add(sub(neg(mul(Q, r)), mul(tr(F), y.eta)), mul(y.J, c)), mul(mul(y.J, G), y.eta));
  d.J = add(sub(sub(neg(Q), mul(y.J, F)), mul(tr(F), y.J)), mul(mul(y.J, G), y.J));
  return d;
}

// Element a_k = V(., t_k; ., t_{k+1}): integrate Theorem 8 in s from s = t_{k+1} (zero-length
// boundary values) down to s = t_k with n classical RK4 steps of -h.  C and J are symmetrised
// (upper triangle kept) after every step.  With steps < n it stops at s = t_{k+1} - steps h and
// returns V(., t_{k+1} - steps h; ., t_{k+1}).
template <class S>
Elem<S> element_backward(const Prob<S>& p, long k, int steps) {
  const int n = p.n;
  const double h = (p.t[k + 1] - p.t[k]) / n;
  Elem<S> y = identity_element<S>(p.nx);
  for (int m = 0; m < steps; ++m) {
    const long j0 = 2L * n * k + 2L * (n - m);  // sample at s = t_{k+1} - m h
    Elem<S> k1 = thm2_rhs(p, j0, y);
    Elem<S> k2 = thm2_rhs(p, j0 - 1, axpy(y, -0.5 * h, k1));
    Elem<S> k3 = thm2_rhs(p, j0 - 1, axpy(y, -0.5 * h, k2));
    Elem<S> k4 = thm2_rhs(p, j0 - 2, axpy(y, -h, k3));
    Elem<S> sum = axpy(axpy(axpy(k1, 2.0, k2), 2.0, k3), 1.0, k4);
    y = axpy(y, -h / 6.0, sum);
    y.C = sym_upper(y.C);
    y.J = sym_upper(y.J);
  }
  return y;
}

// Theorem 9 (Sec. IV-C): derivatives with respect to the upper time limit tau.
template <class S>
Elem<S> thm3_rhs(const Prob<S>& p, long j, const Elem<S>& y) {
  Mat<S> F = F_at(p, j), c = c_at(p, j), r = r_at(p, j), G = G_at(p, j);
  const Mat<S>& Q = p.Q;
  Elem<S> d;
  d.A = add(neg(mul(mul(y.C, Q), y.A)), mul(F, y.A));
  d.b = add(sub(add(mul(mul(y.C, Q), r), mul(F, y.b)), mul(mul(y.C, Q), y.b)), c);
  d.C = add(add(add(neg(mul(mul(y.C, Q), y.C)), G), mul(F, y.C)), mul(y.C, tr(F)));
  d.eta = sub(mul(mul(tr(y.A), Q), r), mul(mul(tr(y.A), Q), y.b));
  d.J = mul(mul(tr(y.A), Q), y.A);
  return d;
}

// Element a_k from Theorem 9: integrate in tau from tau = t_k (zero-length boundary values) up to
// t_{k+1} with n classical RK4 steps of +h.  With steps < n it stops at tau = t_k + steps h and
// returns V(., t_k; ., t_k + steps h).
template <class S>
Elem<S> element_forward(const Prob<S>& p, long k, int steps) {
  const int n = p.n;
  const double h = (p.t[k + 1] - p.t[k]) / n;
  Elem<S> y = identity_element<S>(p.nx);
  for (int m = 0; m < steps; ++m) {
    const long j0 = 2L * n * k + 2L * m;  // sample at tau = t_k + m h
    Elem<S> k1 = thm3_rhs(p, j0, y);
    Elem<S> k2 = thm3_rhs(p, j0 + 1, axpy(y, 0.5 * h, k1));
    Elem<S> k3 = thm3_rhs(p, j0 + 1, axpy(y, 0.5 * h, k2));
    Elem<S> k4 = thm3_rhs(p, j0 + 2, axpy(y, h, k3));
    Elem<S> sum = axpy(axpy(axpy(k1, 2.0, k2), 2.0, k3), 1.0, k4);
    y = axpy(y, h / 6.0, sum);
    y.C = sym_upper(y.C);
    y.J = sym_upper(y.J);
  }
  return y;
}

// Lemma 7 (Sec. IV-A, LQT combination rule): e1 on [s, tau], e2 on [tau, t] -> e1 (x) e2 on [s, t].
template <class S>
Elem<S> combine(const Elem<S>& e1, const Elem<S>& e2) {
  const int nx = e1.A.r;
  Mat<S> I = eye<S>(nx);
  Mat<S> M = add(I, mul(e1.C, e2.J));  // I + C(s,tau) J(tau,t)
  Mat<S> N = add(I, mul(e2.J, e1.C));  // I + J(tau,t) C(s,tau)
  Elem<S> o;
  o.A = mul(e2.A, solve(M, e1.A));
  o.b = add(mul(e2.A, solve(M, add(e1.b, mul(e1.C, e2.eta)))), e2.b);
  o.C = sym_upper(add(mul(mul(e2.A, solve(M, e1.C)), tr(e2.A)), e2.C));
  o.eta = add(mul(tr(e1.A), solve(N, sub(e2.eta, mul(e2.J, e1.b)))), e1.eta);
  o.J = sym_upper(add(mul(mul(tr(e1.A), solve(N, e2.J)), e1.A), e1.J));
  return o;
}

// Terminal element a_T = V(., t_f; ., t_f^+): A = b = C = 0, eta = Qf rf, J = Qf (Sec. IV-D).
template <class S>
Elem<S> terminal_element(const Prob<S>& p) {
  Elem<S> e;
  e.A = Mat<S>(p.nx, p.nx);
  e.b = Mat<S>(p.nx, 1);
  e.C = Mat<S>(p.nx, p.nx);
  e.eta = mul(p.Qf, p.rf);
  e.J = p.Qf;
  return e;
}

// Element a_k with the block split at tau = t_k + floor(n/2) h (Sec. IV-D): the forward ODEs of
// Theorem 9 give V(., t_k; ., tau), the backward ODEs of Theorem 8 give V(., tau; ., t_{k+1}),
// and Lemma 7 joins them.
template <class S>
Elem<S> element_split(const Prob<S>& p, long k) {
  const int m = p.n / 2;
  return combine(element_forward(p, k, m), element_backward(p, k, p.n - m));
}

// mode 0: Theorem 8, 1: Theorem 9, 2: split block.
template <class S>
Elem<S> element(const Prob<S>& p, long k, int mode) {
  if (mode == 1) return element_forward(p, k, p.n);
  if (mode == 2) return element_split(p, k);
  return element_backward(p, k, p.n);
}

template <class S>
std::vector<Elem<S>> elements(const Prob<S>& p, int mode = 0) {
  std::vector<Elem<S>> a(p.T);
  for (long k = 0; k < p.T; ++k) a[k] = element(p, k, mode);
  return a;
}

// V(., t_k) = a_k (x) a_{k+1} (x) ... (x) a_T, folded from the right: V_k = a_k (x) V_{k+1}.
// Returns the tuples; S_k = J, v_k = eta (Sec. IV-D).
template <class S>
std::vector<Elem<S>> value_functions(const std::vector<Elem<S>>& a, const Elem<S>& aT) {
  const long T = (long)a.size();
  std::vector<Elem<S>> V(T + 1);
  V[T] = aT;
  for (long k = T - 1; k >= 0; --k) V[k] = combine(a[k], V[k + 1]);
  return V;
}

template <class S>
Mat<S> control(const Prob<S>& p, long k, const Mat<S>& Sk, const Mat<S>& vk, const Mat<S>& xk) {
  Mat<S> L = L_at(p, 2L * p.n * k);
  // u = -U^{-1} L^T (S x - v)
  return neg(solve(p.R, mul(tr(L), sub(mul(Sk, xk), vk))));
}

// x_{k+1} = argmin_z V(x_k, t_k; z, t_{k+1}) + V(z, t_{k+1})
//         = (I + C_k S_{k+1})^{-1} (A_k x_k + b_k + C_k v_{k+1}).
template <class S>
void trajectory(const Prob<S>& p, const std::vector<Elem<S>>& a, const std::vector<Elem<S>>& V,
                std::vector<Mat<S>>& x, std::vector<Mat<S>>& u) {
  const long T = p.T;
  x.assign(T + 1, Mat<S>());
  u.assign(T + 1, Mat<S>());
  x[0] = p.x0;
  Mat<S> I = eye<S>(p.nx);
  for (long k = 0; k < T; ++k) {
    const Elem<S>& e = a[k];
    Mat<S> rhs = add(add(mul(e.A, x[k]), e.b), mul(e.C, V[k + 1].eta));
    x[k + 1] = solve(add(I, mul(e.C, V[k + 1].J)), rhs);
  }
  for (long k = 0; k <= T; ++k) u[k] = control(p, k, V[k].J, V[k].eta, x[k]);
}

// Method 2 (Sec. IV-E): x_k = (I + C(t0,t_k) S_k)^{-1} (A(t0,t_k) x0 + b(t0,t_k) + C(t0,t_k) v_k) with the
// prefix products V(., t0; ., t_k) = a_0 (x) ... (x) a_{k-1}.
template <class S>
void trajectory_method2(const Prob<S>& p, const std::vector<Elem<S>>& a,
                        const std::vector<Elem<S>>& V, std::vector<Mat<S>>& x) {
  const long T = p.T;
  x.assign(T + 1, Mat<S>());
  Mat<S> I = eye<S>(p.nx);
  Elem<S> P = identity_element<S>(p.nx);
  for (long k = 0; k <= T; ++k) {
    if (k > 0) P = combine(P, a[k - 1]);
    Mat<S> rhs = add(add(mul(P.A, p.x0), P.b), mul(P.C, V[k].eta));
    x[k] = solve(add(I, mul(P.C, V[k].J)), rhs);
  }
}

// Objective sum_k <W_k, x_k> of the discrete scheme (elements, value fold, trajectory).
template <class S>
S objective(const Prob<S>& p, const double* W) {
  std::vector<Elem<S>> a = elements(p);
  std::vector<Elem<S>> V = value_functions(a, terminal_element(p));
  std::vector<Mat<S>> x, u;
  trajectory(p, a, V, x, u);
  S f(0.0);
  for (long k = 0; k <= p.T; ++k)
    for (int i = 0; i < p.nx; ++i) f = f + S(W[k * p.nx + i]) * x[k](i, 0);
  return f;
}

template <class S>
void store(const Mat<S>& m, double* dst) {
  for (int i = 0; i < m.r; ++i)
    for (int j = 0; j < m.c; ++j) dst[i * m.c + j] = value(m(i, j));
}

}  // namespace oracle

using namespace oracle;

// Values inside the blocks.  Node i = n k + m (m = 0..n-1) is t_k + m h_k, node nT is t_T.  Block
// boundaries take the given values (S_k, v_k, x_k).  Inside block k:
//  - S, v: classical RK4 of -h_k on dS/dt = -F^T S - S F - Q + S G S,
//    dv/dt = -Q r - F^T v + S G v + S c (Sec. II-B) from (S_{k+1}, v_{k+1}), with F, G, c, r at
//    the half-step samples (stage 1 at 2nk + 2(n - m'), stages 2 and 3 at - 1, stage 4 at - 2);
//  - x at t_k + m h: the conditional value function on [t_k, t_k + m h] is the Theorem 9 state
//    after m RK4 steps (A, b, C of element_forward's recursion); with V(., tau) = (S, v) at the node
//    the minimiser is x = (I + C S)^{-1} (A x_k + b + C v) (Method 2 formula, Sec. IV-E);
//  - u = -R^{-1} L(tau)^T (S x - v) with L at sample 2i.
template <class S>
void dense_output(const Prob<S>& p, const std::vector<Mat<S>>& Sb, const std::vector<Mat<S>>& vb,
                  const std::vector<Mat<S>>& xb, std::vector<Mat<S>>& Sd,
                  std::vector<Mat<S>>& vd, std::vector<Mat<S>>& xd, std::vector<Mat<S>>& ud) {
  const int n = p.n;
  const long T = p.T, nodes = (long)n * T + 1;
  Sd.assign(nodes, Mat<S>());
  vd.assign(nodes, Mat<S>());
  xd.assign(nodes, Mat<S>());
  ud.assign(nodes, Mat<S>());
  Mat<S> I = eye<S>(p.nx);
  auto dS = [&](long j, const Mat<S>& Sm) {
    Mat<S> F = F_at(p, j), G = G_at(p, j);
    return add(sub(sub(neg(mul(tr(F), Sm)), mul(Sm, F)), p.Q), mul(mul(Sm, G), Sm));
  };
  auto dv = [&](long j, const Mat<S>& Sm, const Mat<S>& vm) {
    Mat<S> F = F_at(p, j), G = G_at(p, j), c = c_at(p, j), r = r_at(p, j);
    return add(add(sub(neg(mul(p.Q, r)), mul(tr(F), vm)), mul(mul(Sm, G), vm)), mul(Sm, c));
  };
  for (long k = 0; k < T; ++k) {
    const double h = (p.t[k + 1] - p.t[k]) / n;
    Sd[(long)n * k] = Sb[k];
    vd[(long)n * k] = vb[k];
    // backward RK4 on S, v from the block's right end
    Mat<S> Sm = Sb[k + 1], vm = vb[k + 1];
    for (int mp = 0; mp < n - 1; ++mp) {
      const long j1 = 2L * n * k + 2L * (n - mp);
      Mat<S> kS1 = dS(j1, Sm), kv1 = dv(j1, Sm, vm);
      Mat<S> S1 = axpy_m(Sm, -0.5 * h, kS1), v1 = axpy_m(vm, -0.5 * h, kv1);
      Mat<S> kS2 = dS(j1 - 1, S1), kv2 = dv(j1 - 1, S1, v1);
      Mat<S> S2 = axpy_m(Sm, -0.5 * h, kS2), v2 = axpy_m(vm, -0.5 * h, kv2);
      Mat<S> kS3 = dS(j1 - 1, S2), kv3 = dv(j1 - 1, S2, v2);
      Mat<S> S3 = axpy_m(Sm, -h, kS3), v3 = axpy_m(vm, -h, kv3);
      Mat<S> kS4 = dS(j1 - 2, S3), kv4 = dv(j1 - 2, S3, v3);
      Sm = sym_upper(axpy_m(Sm, -h / 6.0, add(add(kS1, scale(2.0, kS2)), add(scale(2.0, kS3), kS4))));
      vm = axpy_m(vm, -h / 6.0, add(add(kv1, scale(2.0, kv2)), add(scale(2.0, kv3), kv4)));
      Sd[(long)n * k + (n - mp - 1)] = Sm;
      vd[(long)n * k + (n - mp - 1)] = vm;
    }
    // forward: Theorem 9 recursion from t_k, x by the Method 2 formula after each step
    xd[(long)n * k] = xb[k];
    Elem<S> y = identity_element<S>(p.nx);
    for (int m = 0; m < n - 1; ++m) {
      const long j0 = 2L * n * k + 2L * m;
      Elem<S> k1 = thm3_rhs(p, j0, y);
      Elem<S> k2 = thm3_rhs(p, j0 + 1, axpy(y, 0.5 * h, k1));
      Elem<S> k3 = thm3_rhs(p, j0 + 1, axpy(y, 0.5 * h, k2));
      Elem<S> k4 = thm3_rhs(p, j0 + 2, axpy(y, h, k3));
      y = axpy(y, h / 6.0, axpy(axpy(axpy(k1, 2.0, k2), 2.0, k3), 1.0, k4));
      y.C = sym_upper(y.C);
      y.J = sym_upper(y.J);
      const long i = (long)n * k + m + 1;
      Mat<S> rhs = add(add(mul(y.A, xb[k]), y.b), mul(y.C, vd[i]));
      xd[i] = solve(add(I, mul(y.C, Sd[i])), rhs);
    }
  }
  Sd[nodes - 1] = Sb[T];
  vd[nodes - 1] = vb[T];
  xd[nodes - 1] = xb[T];
  for (long i = 0; i < nodes; ++i) {
    Mat<S> L = L_at(p, 2 * i);
    Mat<S> g = sub(mul(Sd[i], xd[i]), vd[i]);
    ud[i] = neg(solve(p.R, mul(tr(L), g)));
  }
}

extern "C" {

int oracle_abi_version(void) { return 1; }

// Elements a_0..a_{T-1} (mode 0: Theorem 8, 1: Theorem 9, 2: split block).  Outputs, plain
// matrices: A, C, J [T][nx][nx]; b, eta [T][nx].
int oracle_elements(const oracle_problem* prob, int mode, double* A, double* b, double* C,
                    double* eta, double* J) {
  Prob<double> p = load_problem<double>(prob, nullptr);
  const int nx = p.nx;
  for (long k = 0; k < p.T; ++k) {
    Elem<double> e = element(p, k, mode);
    store(e.A, A + k * nx * nx);
    store(e.b, b + k * nx);
    store(e.C, C + k * nx * nx);
    store(e.eta, eta + k * nx);
    store(e.J, J + k * nx * nx);
  }
  return 0;
}

// One application of Lemma 7.  Tuples are packed as [A (nx*nx), b (nx), C (nx*nx), eta (nx),
// J (nx*nx)].
int oracle_combine(int nx, const double* e1, const double* e2, double* out) {
  auto unpack = [nx](const double* s) {
    Elem<double> e;
    e.A = load_mat<double>(s, nx, nx, nullptr);
    s += nx * nx;
    e.b = load_mat<double>(s, nx, 1, nullptr);
    s += nx;
    e.C = load_mat<double>(s, nx, nx, nullptr);
    s += nx * nx;
    e.eta = load_mat<double>(s, nx, 1, nullptr);
    s += nx;
    e.J = load_mat<double>(s, nx, nx, nullptr);
    return e;
  };
  Elem<double> o = combine(unpack(e1), unpack(e2));
  store(o.A, out);
  out += nx * nx;
  store(o.b, out);
  out += nx;
  store(o.C, out);
  out += nx * nx;
  store(o.eta, out);
  out += nx;
  store(o.J, out);
  return 0;
}

// Value functions from given elements: S [T+1][nx][nx], v [T+1][nx].
int oracle_value(int nx, int T, const double* A, const double* b, const double* C,
                 const double* eta, const double* J, const double* Qf, const double* rf, double* S,
                 double* v) {
  std::vector<Elem<double>> a(T);
  for (long k = 0; k < T; ++k) {
    a[k].A = load_mat<double>(A + k * nx * nx, nx, nx, nullptr);
    a[k].b = load_mat<double>(b + k * nx, nx, 1, nullptr);
    a[k].C = load_mat<double>(C + k * nx * nx, nx, nx, nullptr);
    a[k].eta = load_mat<double>(eta + k * nx, nx, 1, nullptr);
    a[k].J = load_mat<double>(J + k * nx * nx, nx, nx, nullptr);
  }
  Elem<double> aT;
  aT.A = Mat<double>(nx, nx);
  aT.b = Mat<double>(nx, 1);
  aT.C = Mat<double>(nx, nx);
  Mat<double> Qfm = load_mat<double>(Qf, nx, nx, nullptr);
  aT.eta = mul(Qfm, load_mat<double>(rf, nx, 1, nullptr));
  aT.J = Qfm;
  std::vector<Elem<double>> V = value_functions(a, aT);
  for (long k = 0; k <= T; ++k) {
    store(V[k].J, S + k * nx * nx);
    store(V[k].eta, v + k * nx);
  }
  return 0;
}

// The whole discrete scheme: elements (Theorem 8), value fold, trajectory and control.
// S [T+1][nx][nx], v [T+1][nx], x [T+1][nx], u [T+1][nu]; any output may be null.
// method2 != 0 recovers x by Method 2 instead.
int oracle_solve(const oracle_problem* prob, int method2, double* S, double* v, double* x,
                 double* u) {
  Prob<double> p = load_problem<double>(prob, nullptr);
  std::vector<Elem<double>> a = elements(p);
  std::vector<Elem<double>> V = value_functions(a, terminal_element(p));
  std::vector<Mat<double>> xs, us;
  if (method2) {
    trajectory_method2(p, a, V, xs);
    us.assign(p.T + 1, Mat<double>());
    for (long k = 0; k <= p.T; ++k) us[k] = control(p, k, V[k].J, V[k].eta, xs[k]);
  } else {
    trajectory(p, a, V, xs, us);
  }
  const int nx = p.nx, nu = p.nu;
  for (long k = 0; k <= p.T; ++k) {
    if (S) store(V[k].J, S + k * nx * nx);
    if (v) store(V[k].eta, v + k * nx);
    if (x) store(xs[k], x + k * nx);
    if (u) store(us[k], u + k * nu);
  }
  return 0;
}

// Values inside the blocks (dense_output) from the block-boundary S [T+1][nx][nx], v, x [T+1][nx];
// outputs at the nT+1 nodes: Sd [nT+1][nx][nx], vd, xd [nT+1][nx], ud [nT+1][nu].
int oracle_dense(const oracle_problem* prob, const double* S, const double* v, const double* x,
                 double* Sd, double* vd, double* xd, double* ud) {
  Prob<double> p = load_problem<double>(prob, nullptr);
  const int nx = p.nx, nu = p.nu;
  std::vector<Mat<double>> Sb(p.T + 1), vb(p.T + 1), xb(p.T + 1), Sdv, vdv, xdv, udv;
  for (long k = 0; k <= p.T; ++k) {
    Sb[k] = load_mat<double>(S + k * nx * nx, nx, nx, nullptr);
    vb[k] = load_mat<double>(v + k * nx, nx, 1, nullptr);
    xb[k] = load_mat<double>(x + k * nx, nx, 1, nullptr);
  }
  dense_output(p, Sb, vb, xb, Sdv, vdv, xdv, udv);
  for (size_t i = 0; i < Sdv.size(); ++i) {
    store(Sdv[i], Sd + i * nx * nx);
    store(vdv[i], vd + i * nx);
    store(xdv[i], xd + i * nx);
    store(udv[i], ud + i * nu);
  }
  return 0;
}

// Trajectory and control from given elements and value functions (same layouts as above).
int oracle_trajectory(const oracle_problem* prob, const double* A, const double* b,
                      const double* C, const double* S, const double* v, double* x, double* u) {
  Prob<double> p = load_problem<double>(prob, nullptr);
  const int nx = p.nx, nu = p.nu;
  std::vector<Elem<double>> a(p.T), V(p.T + 1);
  for (long k = 0; k < p.T; ++k) {
    a[k].A = load_mat<double>(A + k * nx * nx, nx, nx, nullptr);
    a[k].b = load_mat<double>(b + k * nx, nx, 1, nullptr);
    a[k].C = load_mat<double>(C + k * nx * nx, nx, nx, nullptr);
  }
  for (long k = 0; k <= p.T; ++k) {
    V[k].J = load_mat<double>(S + k * nx * nx, nx, nx, nullptr);
    V[k].eta = load_mat<double>(v + k * nx, nx, 1, nullptr);
  }
  std::vector<Mat<double>> xs, us;
  trajectory(p, a, V, xs, us);
  for (long k = 0; k <= p.T; ++k) {
    store(xs[k], x + k * nx);
    if (u) store(us[k], u + k * nu);
  }
  return 0;
}

// Sequential baseline (seq_bw_fw of Sec. VI-A): classical RK4 on the S, v ODEs of Sec. II-B
// backwards from S(tf) = Qf, v(tf) = Qf rf over N uniform steps of ho = (tf - t0)/N, then RK4 on
// the closed-loop state ODE dx/dt = (F - G S) x + G v + c forwards with steps of 2 ho, so every
// stage time falls on a backward-grid node.  F and L are constant, c = 0.  rfine holds r at the
// 2N+1 half-step times t0 + j ho / 2.  Outputs: S [N+1][nx][nx], v [N+1][nx] at the nodes
// t0 + i ho; x [N/2+1][nx] at t0 + 2 i ho (N must be even); any output may be null.
int oracle_riccati(int nx, int nu, const double* F_, const double* L_, const double* Q_,
                   const double* R_, const double* Qf_, const double* rf_, const double* x0_,
                   double t0, double tf, int N, const double* rfine, double* S_out, double* v_out,
                   double* x_out) {
  Mat<double> F = load_mat<double>(F_, nx, nx, nullptr), L = load_mat<double>(L_, nx, nu, nullptr);
  Mat<double> Q = load_mat<double>(Q_, nx, nx, nullptr), R = load_mat<double>(R_, nu, nu, nullptr);
  Mat<double> Qf = load_mat<double>(Qf_, nx, nx, nullptr);
  Mat<double> G = mul(L, solve(R, tr(L)));
  const double ho = (tf - t0) / N;
  std::vector<Mat<double>> Sg(N + 1), vg(N + 1);
  Sg[N] = Qf;
  vg[N] = mul(Qf, load_mat<double>(rf_, nx, 1, nullptr));
  auto rat = [&](long j) { return load_mat<double>(rfine + j * nx, nx, 1, nullptr); };
  auto dS = [&](const Mat<double>& Sm) {  // dS/dt = -F^T S - S F - Q + S G S
    return add(sub(sub(neg(mul(tr(F), Sm)), mul(Sm, F)), Q), mul(mul(Sm, G), Sm));
  };
  auto dv = [&](const Mat<double>& Sm, const Mat<double>& vm, const Mat<double>& r) {
    // dv/dt = -Q r - F^T v + S G v   (c = 0)
    return add(sub(neg(mul(Q, r)), mul(tr(F), vm)), mul(mul(Sm, G), vm));
  };
  for (int i = N; i >= 1; --i) {
    const long j0 = 2L * i;
    Mat<double> S0 = Sg[i], v0 = vg[i];
    Mat<double> kS1 = dS(S0), kv1 = dv(S0, v0, rat(j0));
    Mat<double> S1 = add(S0, scale(-0.5 * ho, kS1)), v1 = add(v0, scale(-0.5 * ho, kv1));
    Mat<double> kS2 = dS(S1), kv2 = dv(S1, v1, rat(j0 - 1));
    Mat<double> S2 = add(S0, scale(-0.5 * ho, kS2)), v2 = add(v0, scale(-0.5 * ho, kv2));
    Mat<double> kS3 = dS(S2), kv3 = dv(S2, v2, rat(j0 - 1));
    Mat<double> S3 = add(S0, scale(-ho, kS3)), v3 = add(v0, scale(-ho, kv3));
    Mat<double> kS4 = dS(S3), kv4 = dv(S3, v3, rat(j0 - 2));
    Sg[i - 1] = sym_upper(add(S0, scale(-ho / 6.0, add(add(kS1, scale(2.0, kS2)), add(scale(2.0, kS3), kS4)))));
    vg[i - 1] = add(v0, scale(-ho / 6.0, add(add(kv1, scale(2.0, kv2)), add(scale(2.0, kv3), kv4))));
  }
  if (S_out)
    for (int i = 0; i <= N; ++i) store(Sg[i], S_out + (long)i * nx * nx);
  if (v_out)
    for (int i = 0; i <= N; ++i) store(vg[i], v_out + (long)i * nx);
  if (x_out) {
    const double hf = 2.0 * ho;
    auto fx = [&](int node, const Mat<double>& xm) {  // (F - G S) x + G v
      return add(mul(sub(F, mul(G, Sg[node])), xm), mul(G, vg[node]));
    };
    Mat<double> xm = load_mat<double>(x0_, nx, 1, nullptr);
    store(xm, x_out);
    for (int i = 0; 2 * i + 2 <= N; ++i) {
      const int nd = 2 * i;
      Mat<double> k1 = fx(nd, xm);
      Mat<double> k2 = fx(nd + 1, add(xm, scale(0.5 * hf, k1)));
      Mat<double> k3 = fx(nd + 1, add(xm, scale(0.5 * hf, k2)));
      Mat<double> k4 = fx(nd + 2, add(xm, scale(hf, k3)));
      xm = add(xm, scale(hf / 6.0, add(add(k1, scale(2.0, k2)), add(scale(2.0, k3), k4))));
      store(xm, x_out + (long)(i + 1) * nx);
    }
  }
  return 0;
}

// Objective f = sum_k <W_k, x_k> (W [T+1][nx]) and its directional derivative along the tangent
// directions (forward-mode dual numbers through the whole discrete scheme).
int oracle_objective_jvp(const oracle_problem* prob, const double* W,
                         const oracle_inputs_tangent* tangent, double* f, double* df) {
  Prob<Dual> p = load_problem<Dual>(prob, tangent);
  Dual out = objective(p, W);
  *f = out.v;
  *df = out.d;
  return 0;
}

// Gradient of f = sum_k <W_k, x_k> with respect to Q, R, r, Qf, rf, x0 (the sequential adjoint:
// the forward scheme is recorded on a tape and swept backwards).  Gradients are with respect to
// every entry of the matrices as given (no symmetrisation).  Outputs may be null.
int oracle_objective_grad(const oracle_problem* prob, const double* W, double* f, double* gQ,
                          double* gR, double* gr, double* gQf, double* grf, double* gx0) {
  Tape tape;
  g_tape = &tape;
  Prob<Var> p = load_problem<Var>(prob, nullptr);
  Var out = objective(p, W);
  std::vector<double> adj(tape.p1.size(), 0.0);
  if (out.id >= 0) adj[out.id] = 1.0;
  for (long i = (long)tape.p1.size() - 1; i >= 0; --i) {
    const double g = adj[i];
    if (g == 0.0) continue;
    if (tape.p1[i] >= 0) adj[tape.p1[i]] += tape.w1[i] * g;
    if (tape.p2[i] >= 0) adj[tape.p2[i]] += tape.w2[i] * g;
  }
  auto grab = [&](const Mat<Var>& m, double* dst) {
    if (!dst) return;
    for (int i = 0; i < m.r; ++i)
      for (int j = 0; j < m.c; ++j) dst[i * m.c + j] = m(i, j).id >= 0 ? adj[m(i, j).id] : 0.0;
  };
  *f = out.v;
  grab(p.Q, gQ);
  grab(p.R, gR);
  grab(p.Qf, gQf);
  grab(p.rf, grf);
  grab(p.x0, gx0);
  if (gr)
    for (size_t i = 0; i < p.r.size(); ++i) gr[i] = p.r[i].id >= 0 ? adj[p.r[i].id] : 0.0;
  g_tape = nullptr;
  return 0;
}

}  // extern "C"
