// Real FP64 kernels of the outer iteration (Rayleigh-Ritz, B-orthogonalisation,
// residual check) on row-major n x ld blocks, plus setup helpers.
//
// The tall-skinny Gram G = X^T Y and the product Z = X S run on the FP64
// matrix cores (v_mfma_f64_16x16x4f64): operand A is a 16x4 tile (lane l holds
// row l%16, k l/16), operand B a 4x16 tile (lane l holds k l/16, column l%16),
// and the 16x16 accumulator holds in lane l, element v the entry
// (row 4*v + l/16, column l%16) (established by an on-device layout check).
#include "internal.h"

namespace slrf {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

inline unsigned cdiv(size_t a, size_t b) { return (unsigned)((a + b - 1) / b); }

// Y_A = A X, Y_B = B X (one CSR pass), optionally E = A X - theta_c B X.
// One wave per row; lanes cover 64 columns at a time.
__global__ __launch_bounds__(256) void k_spmm_real(int n, const int* __restrict__ rowptr,
                                                   const int* __restrict__ col,
                                                   const double* __restrict__ av,
                                                   const double* __restrict__ bv,
                                                   const double* __restrict__ X, int ld, int nc,
                                                   double* __restrict__ AX,
                                                   double* __restrict__ BX,
                                                   const double* __restrict__ theta,
                                                   double* __restrict__ E) {
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (row >= n) return;
  const int e0 = rowptr[row], e1 = rowptr[row + 1];
  for (int c0 = 0; c0 < nc; c0 += 64) {
    const int c = c0 + lane;
    if (c >= nc) break;
    double sa = 0.0, sb = 0.0;
    for (int e = e0; e < e1; ++e) {
      const double x = X[(size_t)col[e] * ld + c];
      sa = fma(av[e], x, sa);
      sb = fma(bv[e], x, sb);
    }
    const size_t o = (size_t)row * ld + c;
    if (AX) AX[o] = sa;
    if (BX) BX[o] = sb;
    if (E) E[o] = sa - theta[c] * sb;
  }
}

// out[c * ldout + omap(r)] = in[r * ldin + imap(c)] for r < rows, c < cols
// (32x32 LDS tiles); imap / omap are optional index maps (NULL = identity), used
// to apply the library's row order at the column-major <-> row-major boundary.
__global__ __launch_bounds__(256) void k_transpose(const double* __restrict__ in, int rows,
                                                   int cols, int ldin, double* __restrict__ out,
                                                   int ldout, const int* __restrict__ imap,
                                                   const int* __restrict__ omap) {
  __shared__ double tile[32][33];
  const int bx = blockIdx.x * 32, by = blockIdx.y * 32;  // bx over cols, by over rows
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
  for (int j = ty; j < 32; j += 8) {
    const int r = by + j, c = bx + tx;
    if (r < rows && c < cols) tile[j][tx] = in[(size_t)r * ldin + (imap ? imap[c] : c)];
  }
  __syncthreads();
  for (int j = ty; j < 32; j += 8) {
    const int c = bx + j, r = by + tx;
    if (r < rows && c < cols) out[(size_t)c * ldout + (omap ? omap[r] : r)] = tile[tx][j];
  }
}

// Partial Gram over one row chunk: part[chunk][i][j] = sum_{r in chunk} X[r,i] Y[r,j].
// Workgroup tile 64x64 (2x2 waves, each 32x32 = 2x2 MFMA tiles).
__global__ __launch_bounds__(256) void k_gram(int n, int p, int q, const double* __restrict__ X,
                                              int ldx, const double* __restrict__ Y, int ldy,
                                              double* __restrict__ part, int rows_per_chunk) {
  const int nbq = (q + 63) / 64;
  const int ib = (blockIdx.x / nbq) * 64, jb = (blockIdx.x % nbq) * 64;
  const int chunk = blockIdx.y;
  const int wave = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int wi = ib + (wave >> 1) * 32, wj = jb + (wave & 1) * 32;
  const int kk = l >> 4, ii = l & 15;
  const int r0 = chunk * rows_per_chunk, r1 = min(r0 + rows_per_chunk, n);
  d4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = d4{0.0, 0.0, 0.0, 0.0};
  const int ca0 = wi + ii, ca1 = wi + 16 + ii, cb0 = wj + ii, cb1 = wj + 16 + ii;
  for (int r = r0; r < r1; r += 4) {
    const int row = r + kk;
    const bool okr = row < r1;
    const double* xr = X + (size_t)row * ldx;
    const double* yr = Y + (size_t)row * ldy;
    const double a0 = (okr && ca0 < p) ? xr[ca0] : 0.0;
    const double a1 = (okr && ca1 < p) ? xr[ca1] : 0.0;
    const double b0 = (okr && cb0 < q) ? yr[cb0] : 0.0;
    const double b1 = (okr && cb1 < q) ? yr[cb1] : 0.0;
    acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
    acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
    acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
    acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
  }
  double* pc = part + (size_t)chunk * p * q;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = wi + a * 16 + 4 * v + (l >> 4);
        const int j = wj + b * 16 + (l & 15);
        if (i < p && j < q) pc[(size_t)i * q + j] = acc[a][b][v];
      }
}

__global__ void k_chunk_sum(const double* __restrict__ part, int nchunk, int p, int q,
                            double* __restrict__ G, int ldg) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= p * q) return;
  const int i = t / q, j = t % q;
  double s = 0.0;
  for (int c = 0; c < nchunk; ++c) s += part[(size_t)c * p * q + t];
  G[(size_t)i * ldg + j] = s;
}

// Z = alpha X S + beta Z.  Workgroup: 64 rows (4 waves x 16 rows) x 64 columns
// (4 MFMA tiles per wave).
__global__ __launch_bounds__(256) void k_gemm_tall(int n, int p, int q, double alpha,
                                                   const double* __restrict__ X, int ldx,
                                                   const double* __restrict__ S, int lds,
                                                   double beta, double* __restrict__ Z, int ldz) {
  const int wave = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int r0 = blockIdx.x * 64 + wave * 16;
  const int jb = blockIdx.y * 64;
  const int kk = l >> 4, ii = l & 15;
  d4 acc[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) acc[t] = d4{0.0, 0.0, 0.0, 0.0};
  const int arow = r0 + ii;
  const bool okrow = arow < n;
  for (int k0 = 0; k0 < p; k0 += 4) {
    const int kc = k0 + kk;
    const double a = (okrow && kc < p) ? X[(size_t)arow * ldx + kc] : 0.0;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int j = jb + t * 16 + ii;
      const double b = (kc < p && j < q) ? S[(size_t)kc * lds + j] : 0.0;
      acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[t], 0, 0, 0);
    }
  }
#pragma unroll
  for (int t = 0; t < 4; ++t)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int i = r0 + 4 * v + (l >> 4);
      const int j = jb + t * 16 + (l & 15);
      if (i < n && j < q) {
        const size_t o = (size_t)i * ldz + j;
        Z[o] = alpha * acc[t][v] + (beta == 0.0 ? 0.0 : beta * Z[o]);
      }
    }
}

__global__ __launch_bounds__(256) void k_colstats(int n, int nc, const double* __restrict__ X,
                                                  const double* __restrict__ Y, int ld,
                                                  const double* __restrict__ theta,
                                                  const double* __restrict__ W,
                                                  double* __restrict__ part, int rows_per_chunk) {
  const int chunk = blockIdx.x;
  const int r0 = chunk * rows_per_chunk, r1 = min(r0 + rows_per_chunk, n);
  for (int c = threadIdx.x; c < nc; c += 256) {
    double s1 = 0.0, s2 = 0.0;
    const double th = theta ? theta[c] : 0.0;
    for (int r = r0; r < r1; ++r) {
      const size_t o = (size_t)r * ld + c;
      double x = X[o];
      if (theta) x -= th * Y[o];
      s1 = fma(x, x, s1);
      if (W) s2 = fma(W[o], Y[o], s2);
    }
    part[((size_t)chunk * 2 + 0) * nc + c] = s1;
    part[((size_t)chunk * 2 + 1) * nc + c] = s2;
  }
}

__global__ void k_colreduce(const double* __restrict__ part, int nchunk, int nc,
                            double* __restrict__ out, double* __restrict__ out2) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= nc) return;
  double s1 = 0.0, s2 = 0.0;
  for (int k = 0; k < nchunk; ++k) {
    s1 += part[((size_t)k * 2 + 0) * nc + c];
    s2 += part[((size_t)k * 2 + 1) * nc + c];
  }
  if (out) out[c] = s1;
  if (out2) out2[c] = s2;
}

__global__ void k_cast_f32(const double* __restrict__ in, float* __restrict__ out, size_t cnt) {
  const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < cnt) out[t] = (float)in[t];
}

__global__ void k_diag(int n, const int* __restrict__ rowptr, const int* __restrict__ col,
                       const double* __restrict__ av, const double* __restrict__ bv,
                       double* __restrict__ da, double* __restrict__ db, int* __restrict__ missing) {
  const int row = blockIdx.x * blockDim.x + threadIdx.x;
  if (row >= n) return;
  double a = 0.0, b = 0.0;
  int found = 0;
  for (int e = rowptr[row]; e < rowptr[row + 1]; ++e) {
    if (col[e] == row) {
      a = av[e];
      b = bv[e];
      found = 1;
    }
  }
  da[row] = a;
  db[row] = b;
  if (!found) missing[0] = 1;
}

}  // namespace

constexpr int kGramRows = 2048;
constexpr int kColRows = 1024;

int gram_chunks(int n) { return n <= 0 ? 1 : (n + kGramRows - 1) / kGramRows; }
int colstat_chunks(int n) { return n <= 0 ? 1 : (n + kColRows - 1) / kColRows; }

hipError_t launch_spmm_real(const DevPencil& P, const double* X, int ld, int nc, double* AX,
                            double* BX, const double* theta, double* E, hipStream_t s) {
  if (P.n == 0 || nc == 0) return hipSuccess;
  k_spmm_real<<<cdiv(P.n, 4), 256, 0, s>>>(P.n, P.rowptr, P.col, P.a, P.b, X, ld, nc, AX, BX,
                                           theta, E);
  return hipGetLastError();
}

hipError_t launch_transpose(const double* in, int rows, int cols, int ldin, double* out,
                            int ldout, hipStream_t s, const int* imap, const int* omap) {
  if (rows == 0 || cols == 0) return hipSuccess;
  dim3 grid(cdiv(cols, 32), cdiv(rows, 32));
  k_transpose<<<grid, 256, 0, s>>>(in, rows, cols, ldin, out, ldout, imap, omap);
  return hipGetLastError();
}

hipError_t launch_gram(int n, int p, int q, const double* X, int ldx, const double* Y, int ldy,
                       double* part, int nchunk, double* G, int ldg, hipStream_t s) {
  if (p == 0 || q == 0) return hipSuccess;
  const int rows = (n + nchunk - 1) / nchunk;
  const int rpc = ((rows + 3) / 4) * 4;
  dim3 grid(cdiv(p, 64) * cdiv(q, 64), nchunk);
  k_gram<<<grid, 256, 0, s>>>(n, p, q, X, ldx, Y, ldy, part, rpc);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  k_chunk_sum<<<cdiv((size_t)p * q, 256), 256, 0, s>>>(part, nchunk, p, q, G, ldg);
  return hipGetLastError();
}

hipError_t launch_gemm_tall(int n, int p, int q, double alpha, const double* X, int ldx,
                            const double* S, int lds, double beta, double* Z, int ldz,
                            hipStream_t s) {
  if (n == 0 || q == 0) return hipSuccess;
  dim3 grid(cdiv(n, 64), cdiv(q, 64));
  k_gemm_tall<<<grid, 256, 0, s>>>(n, p, q, alpha, X, ldx, S, lds, beta, Z, ldz);
  return hipGetLastError();
}

hipError_t launch_colstats(int n, int nc, const double* X, const double* Y, int ld,
                           const double* theta, const double* W, double* part, int nchunk,
                           double* out, double* out2, hipStream_t s) {
  if (nc == 0) return hipSuccess;
  const int rpc = (n + nchunk - 1) / nchunk;
  k_colstats<<<nchunk, 256, 0, s>>>(n, nc, X, Y, ld, theta, W, part, rpc);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  k_colreduce<<<cdiv(nc, 256), 256, 0, s>>>(part, nchunk, nc, out, out2);
  return hipGetLastError();
}

hipError_t launch_cast_f32(const double* in, float* out, size_t cnt, hipStream_t s) {
  if (cnt == 0) return hipSuccess;
  k_cast_f32<<<cdiv(cnt, 256), 256, 0, s>>>(in, out, cnt);
  return hipGetLastError();
}

hipError_t launch_diag(const DevPencil& P, double* da, double* db, int* missing, hipStream_t s) {
  if (P.n == 0) return hipSuccess;
  k_diag<<<cdiv(P.n, 256), 256, 0, s>>>(P.n, P.rowptr, P.col, P.a, P.b, da, db, missing);
  return hipGetLastError();
}

}  // namespace slrf
