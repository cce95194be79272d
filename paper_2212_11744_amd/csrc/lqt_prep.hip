// Per-problem constants derived from L and R, computed once per call on the device (one thread per
// problem; sizes up to 16).  With R = Lr Lr^T (Cholesky) and W = Lr^{-T}:
//   Rinv = W W^T = R^{-1},  Lc = L W,  G = Lc Lc^T = L R^{-1} L^T,  Kc = R^{-1} L^T,
// where G is the matrix L U^{-1} L^T of the LQT equations (Sec. II-B, Theorem 8) and Kc the gain of
// the optimal control law u = -U^{-1} L^T (S x - v).  G, Lc, Kc are formed only when L is constant.
#include "lqt_internal.hpp"

namespace lqt {
namespace {

template <class R>
__global__ void k_prep(const KProb kp, R* __restrict__ consts) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= kp.batch) return;
  const int nx = kp.nx, nu = kp.nu;
  const R* Rm = (const R*)kp.R + (long)p * nu * nu;
  R* cs = consts + (long)p * consts_count(nx, nu);
  R Lr[16][16], W[16][16];
  for (int i = 0; i < nu; ++i)
    for (int j = 0; j < nu; ++j) {
      Lr[i][j] = R(0);
      W[i][j] = R(0);
    }
  // Cholesky R = Lr Lr^T from the lower triangle.
  for (int j = 0; j < nu; ++j) {
    R d = Rm[j * nu + j];
    for (int k = 0; k < j; ++k) d -= Lr[j][k] * Lr[j][k];
    const R ljj = sqrt(d);
    Lr[j][j] = ljj;
    for (int i = j + 1; i < nu; ++i) {
      R s = Rm[i * nu + j];
      for (int k = 0; k < j; ++k) s -= Lr[i][k] * Lr[j][k];
      Lr[i][j] = s / ljj;
    }
  }
  // Linv = Lr^{-1} (lower) by forward substitution on the identity; W = Linv^T.
  for (int c = 0; c < nu; ++c)
    for (int i = c; i < nu; ++i) {
      R s = (i == c) ? R(1) : R(0);
      for (int k = c; k < i; ++k) s -= Lr[i][k] * W[c][k];
      W[c][i] = s / Lr[i][i];  // W[c][i] = Linv[i][c]
    }
  const int oW = consts_off_W(nx, nu), oRi = consts_off_Rinv(nx, nu);
  for (int i = 0; i < nu; ++i)
    for (int j = 0; j < nu; ++j) {
      cs[oW + i * nu + j] = W[i][j];
      R s = R(0);
      for (int k = 0; k < nu; ++k) s += W[i][k] * W[j][k];
      cs[oRi + i * nu + j] = s;
    }
  if (!kp.L_sampled) {
    const R* L = (const R*)kp.L + (kp.seg ? (long)p * nx * nu : 0);
    const int oG = consts_off_G(nx, nu), oLc = consts_off_Lc(nx, nu), oK = consts_off_Kc(nx, nu);
    for (int i = 0; i < nx; ++i)
      for (int l = 0; l < nu; ++l) {
        R s = R(0);
        for (int q = 0; q < nu; ++q) s += L[i * nu + q] * W[q][l];
        cs[oLc + i * nu + l] = s;
      }
    for (int i = 0; i < nx; ++i)
      for (int j = 0; j < nx; ++j) {
        R s = R(0);
        for (int l = 0; l < nu; ++l) s += cs[oLc + i * nu + l] * cs[oLc + j * nu + l];
        cs[oG + i * nx + j] = s;
      }
    for (int l = 0; l < nu; ++l)
      for (int j = 0; j < nx; ++j) {
        R s = R(0);
        for (int q = 0; q < nu; ++q) s += cs[oRi + l * nu + q] * L[j * nu + q];
        cs[oK + l * nx + j] = s;
      }
  }
}

}  // namespace

hipError_t launch_prep(const KProb& kp, int dtype, void* consts, hipStream_t stream) {
  const dim3 grid((kp.batch + 63) / 64), block(64);
  if (dtype == 0)
    hipLaunchKernelGGL(k_prep<double>, grid, block, 0, stream, kp, (double*)consts);
  else
    hipLaunchKernelGGL(k_prep<float>, grid, block, 0, stream, kp, (float*)consts);
  return hipGetLastError();
}

}  // namespace lqt
