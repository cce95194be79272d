// Per-problem constants derived from L and R, computed once per call on the device (one workgroup
// of 64 threads per problem, matrices in LDS; sizes up to 16).  With R = Lr Lr^T (Cholesky) and
// W = Lr^{-T}:
//   Rinv = W W^T = R^{-1},  Lc = L W,  G = Lc Lc^T = L R^{-1} L^T,  Kc = R^{-1} L^T,
// where G is the matrix L U^{-1} L^T of the LQT equations (Sec. II-B, Theorem 8) and Kc the gain of
// the optimal control law u = -U^{-1} L^T (S x - v).  G, Lc, Kc are formed only when L is constant.
#include "lqt_internal.hpp"

namespace lqt {
namespace {

template <class R>
__global__ __launch_bounds__(64) void k_prep(const KProb kp, R* __restrict__ consts) {
  __shared__ R Lr[16 * 16], W[16 * 16], Ri[16 * 16], Lc[16 * 16];
  const int p = blockIdx.x;
  const int t = threadIdx.x;
  const int nx = kp.nx, nu = kp.nu;
  const R* Rm = (const R*)kp.R + (long)p * nu * nu;
  R* cs = consts + (long)p * consts_count(nx, nu);
  // Cholesky R = Lr Lr^T from the lower triangle, column by column (rows below the diagonal in
  // parallel).
  for (int j = 0; j < nu; ++j) {
    if (t == 0) {
      R d = Rm[j * nu + j];
      for (int k = 0; k < j; ++k) d -= Lr[j * 16 + k] * Lr[j * 16 + k];
      Lr[j * 16 + j] = sqrt(d);
    }
    __syncthreads();
    const int i = j + 1 + t;
    if (i < nu) {
      R s = Rm[i * nu + j];
      for (int k = 0; k < j; ++k) s -= Lr[i * 16 + k] * Lr[j * 16 + k];
      Lr[i * 16 + j] = s / Lr[j * 16 + j];
    }
    __syncthreads();
  }
  // Linv = Lr^{-1} (lower) by forward substitution, one column per thread; W = Linv^T.
  if (t < nu) {
    const int c = t;
    for (int i = 0; i < nu; ++i) {
      R s = (i == c) ? R(1) : R(0);
      for (int k = c; k < i; ++k) s -= Lr[i * 16 + k] * W[c * 16 + k];
      W[c * 16 + i] = i < c ? R(0) : s / Lr[i * 16 + i];  // W[c][i] = Linv[i][c]
    }
  }
  __syncthreads();
  const int oW = consts_off_W(nx, nu), oRi = consts_off_Rinv(nx, nu);
  for (int e = t; e < nu * nu; e += 64) {
    const int i = e / nu, j = e % nu;
    cs[oW + e] = W[i * 16 + j];
    R s = R(0);
    for (int k = 0; k < nu; ++k) s += W[i * 16 + k] * W[j * 16 + k];
    cs[oRi + e] = s;
    Ri[i * 16 + j] = s;
  }
  if (kp.L_sampled) return;
  const R* L = (const R*)kp.L + (kp.seg ? (long)p * nx * nu : 0);
  const int oG = consts_off_G(nx, nu), oLc = consts_off_Lc(nx, nu), oK = consts_off_Kc(nx, nu);
  for (int e = t; e < nx * nu; e += 64) {
    const int i = e / nu, l = e % nu;
    R s = R(0);
    for (int q = 0; q < nu; ++q) s += L[i * nu + q] * W[q * 16 + l];
    cs[oLc + e] = s;
    Lc[i * 16 + l] = s;
  }
  __syncthreads();
  for (int e = t; e < nx * nx; e += 64) {
    const int i = e / nx, j = e % nx;
    R s = R(0);
    for (int l = 0; l < nu; ++l) s += Lc[i * 16 + l] * Lc[j * 16 + l];
    cs[oG + e] = s;
  }
  for (int e = t; e < nu * nx; e += 64) {
    const int l = e / nx, j = e % nx;
    R s = R(0);
    for (int q = 0; q < nu; ++q) s += Ri[l * 16 + q] * L[j * nu + q];
    cs[oK + e] = s;
  }
}

}  // namespace

hipError_t launch_prep(const KProb& kp, int dtype, void* consts, hipStream_t stream) {
  const dim3 grid((unsigned)kp.batch), block(64);
  if (dtype == 0)
    hipLaunchKernelGGL(k_prep<double>, grid, block, 0, stream, kp, (double*)consts);
  else
    hipLaunchKernelGGL(k_prep<float>, grid, block, 0, stream, kp, (float*)consts);
  return hipGetLastError();
}

}  // namespace lqt
