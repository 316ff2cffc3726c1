// Eigenvalue sensitivities per element parameter (the differentiation form).
//
// For a B-normalised eigenpair (lambda_i, x_i) of A(theta) x = lambda B(theta) x,
// d lambda_i / d theta_e = x_i^T (dA_e - lambda_i dB_e) x_i, where dA_e, dB_e are
// the element derivative matrices acting on the element's dofs.  For a loss
// L(lambda) with gradient g_i the kernel returns
//   grad_e = sum_i g_i x_{i,e}^T (dA_e - lambda_i dB_e) x_{i,e}.
// One wave per element: lane t handles eigenvectors t, t + 64, ...; the element
// matrices sit in LDS; the 64 lane partial sums are combined by a fixed
// shuffle tree (deterministic).
#include "internal.h"

namespace slrf {
namespace {

constexpr int kElemPerWG = 4; // elements per workgroup (one wave each)

// ND = element dofs (compile time so the element vector stays in registers)
template <int ND>
__global__ __launch_bounds__(256) void k_eig_grad(int n, int k, const double* __restrict__ X,
                                                  const double* __restrict__ lam,
                                                  const double* __restrict__ glam, int nelem,
                                                  const int* __restrict__ dofs,
                                                  const double* __restrict__ dA, int sa,
                                                  const double* __restrict__ dB, int sb,
                                                  double* __restrict__ grad) {
  constexpr int nd = ND;
  __shared__ double sA[kElemPerWG][ND * ND];
  __shared__ double sB[kElemPerWG][ND * ND];
  __shared__ int sd[kElemPerWG][ND];
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int e = blockIdx.x * kElemPerWG + w;
  const bool ok = e < nelem;
  if (ok) {
    const double* a = dA + (size_t)(sa ? e : 0) * sa;
    for (int t = l; t < nd * nd; t += 64) sA[w][t] = a[t];
    if (dB) {
      const double* b = dB + (size_t)(sb ? e : 0) * sb;
      for (int t = l; t < nd * nd; t += 64) sB[w][t] = b[t];
    }
    for (int t = l; t < nd; t += 64) sd[w][t] = dofs[(size_t)e * nd + t];
  }
  __syncthreads();
  if (!ok) return;
  double acc = 0.0;
  for (int i = l; i < k; i += 64) {
    double xe[ND];
#pragma unroll
    for (int a = 0; a < nd; ++a) {
      const int d = sd[w][a];
      xe[a] = d >= 0 ? X[(size_t)i * n + d] : 0.0;
    }
    double qa = 0.0, qb = 0.0;
#pragma unroll
    for (int a = 0; a < nd; ++a) {
      double ya = 0.0, yb = 0.0;
#pragma unroll
      for (int b = 0; b < nd; ++b) {
        ya = fma(sA[w][a * nd + b], xe[b], ya);
        if (dB) yb = fma(sB[w][a * nd + b], xe[b], yb);
      }
      qa = fma(xe[a], ya, qa);
      qb = fma(xe[a], yb, qb);
    }
    acc += glam[i] * (qa - lam[i] * qb);
  }
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
  if (l == 0) grad[e] = acc;
}

}  // namespace

hipError_t launch_eig_grad(int n, int k, const double* X, const double* lam, const double* glam,
                           int nelem, int nd, const int* dofs, const double* dA, int sa,
                           const double* dB, int sb, double* grad, hipStream_t s) {
  if (nelem == 0) return hipSuccess;
  const unsigned blocks = (unsigned)((nelem + kElemPerWG - 1) / kElemPerWG);
  switch (nd) {
    case 4:
      k_eig_grad<4><<<blocks, 256, 0, s>>>(n, k, X, lam, glam, nelem, dofs, dA, sa, dB, sb, grad);
      break;
    case 8:
      k_eig_grad<8><<<blocks, 256, 0, s>>>(n, k, X, lam, glam, nelem, dofs, dA, sa, dB, sb, grad);
      break;
    case 24:
      k_eig_grad<24><<<blocks, 256, 0, s>>>(n, k, X, lam, glam, nelem, dofs, dA, sa, dB, sb,
                                            grad);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace slrf
