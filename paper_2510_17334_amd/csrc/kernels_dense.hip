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
// One wave per row: the row's entries (column, a, b) are wave-uniform and come
// through scalar loads, four at a time; each lane covers three columns of a
// 192-column slice (lane, lane + 64, lane + 128), with the four entries' X rows
// loaded together.
__global__ __launch_bounds__(256) void k_spmm_real(int n, const int* __restrict__ rowptr,
                                                   const int* __restrict__ col,
                                                   const double* __restrict__ av,
                                                   const double* __restrict__ bv,
                                                   const double* __restrict__ X, int ld, int nc,
                                                   double* __restrict__ AX,
                                                   double* __restrict__ BX,
                                                   const double* __restrict__ theta,
                                                   double* __restrict__ E) {
  // XCD-aware order: each XCD takes a contiguous range of rows, so the X rows
  // a neighbourhood gathers stay in one L2
  const int nblk = (n + 3) / 4;
  const int per = (nblk + 7) / 8;
  const int blk = (int)(blockIdx.x & 7) * per + (int)(blockIdx.x >> 3);
  const int row = __builtin_amdgcn_readfirstlane(blk * 4 + (int)(threadIdx.x >> 6));
  const int lane = threadIdx.x & 63;
  if (blk >= nblk || row >= n) return;
  const int e0 = rowptr[row], e1 = rowptr[row + 1];
  for (int c0 = 0; c0 < nc; c0 += 192) {
    bool ok[3];
    int cc[3];
#pragma unroll
    for (int t = 0; t < 3; ++t) {
      cc[t] = c0 + lane + 64 * t;
      ok[t] = cc[t] < nc;
      if (!ok[t]) cc[t] = 0;  // (an existing column: loaded, not stored)
    }
    double sa[3] = {0.0, 0.0, 0.0}, sb[3] = {0.0, 0.0, 0.0};
    int e = e0;
    for (; e + 4 <= e1; e += 4) {
      int cl[4];
      double a[4], b[4], x[4][3];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        cl[u] = col[e + u];
        a[u] = av[e + u];
        b[u] = bv[e + u];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int t = 0; t < 3; ++t) x[u][t] = X[(size_t)cl[u] * ld + cc[t]];
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int t = 0; t < 3; ++t) {
          sa[t] = fma(a[u], x[u][t], sa[t]);
          sb[t] = fma(b[u], x[u][t], sb[t]);
        }
    }
    for (; e < e1; ++e) {
      const int cl = col[e];
      const double a = av[e], b = bv[e];
#pragma unroll
      for (int t = 0; t < 3; ++t) {
        const double x = X[(size_t)cl * ld + cc[t]];
        sa[t] = fma(a, x, sa[t]);
        sb[t] = fma(b, x, sb[t]);
      }
    }
#pragma unroll
    for (int t = 0; t < 3; ++t) {
      if (!ok[t]) continue;
      const size_t o = (size_t)row * ld + cc[t];
      if (AX) AX[o] = sa[t];
      if (BX) BX[o] = sb[t];
      if (E) E[o] = sa[t] - theta[cc[t]] * sb[t];
    }
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
// Workgroup: one 32x32 tile of G (2x2 MFMA tiles) and one chunk of rows; its
// four waves take interleaved 4-row steps of the chunk (the four together read
// 16 consecutive rows), each loading the next step's operands while its MFMAs
// run, and their partial tiles are summed through LDS in wave order.
__global__ __launch_bounds__(256) void k_gram(int n, int p, int q, const double* __restrict__ X,
                                              int ldx, const double* __restrict__ Y, int ldy,
                                              double* __restrict__ part, int rows_per_chunk,
                                              int nchunk) {
  __shared__ double red[4][32 * 32];
  const int ntj = (q + 31) / 32;
  const long ntile = (long)((p + 31) / 32) * ntj;
  // XCD-aware order: each XCD takes a contiguous range of (chunk, tile) pairs,
  // so the rows of a chunk are fetched into one XCD's L2 for all its tiles
  const long total = ntile * nchunk;
  const long per = (total + 7) / 8;
  const long w8 = (long)(blockIdx.x & 7) * per + (blockIdx.x >> 3);
  if (w8 >= total) return;
  const int chunk = (int)(w8 / ntile);
  const int tile = (int)(w8 % ntile);
  const int ib = (tile / ntj) * 32, jb = (tile % ntj) * 32;
  const int wave = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int kk = l >> 4, ii = l & 15;
  const int r0 = chunk * rows_per_chunk, r1 = min(r0 + rows_per_chunk, n);
  d4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = d4{0.0, 0.0, 0.0, 0.0};
  const int ca0 = ib + ii, ca1 = ib + 16 + ii, cb0 = jb + ii, cb1 = jb + 16 + ii;
  const bool oa0 = ca0 < p, oa1 = ca1 < p, ob0 = cb0 < q, ob1 = cb1 < q;
  auto load = [&](int r, double& a0, double& a1, double& b0, double& b1) {
    const int row = r + kk;
    const bool okr = row < r1;
    const double* xr = X + (size_t)row * ldx;
    const double* yr = Y + (size_t)row * ldy;
    a0 = (okr && oa0) ? xr[ca0] : 0.0;
    a1 = (okr && oa1) ? xr[ca1] : 0.0;
    b0 = (okr && ob0) ? yr[cb0] : 0.0;
    b1 = (okr && ob1) ? yr[cb1] : 0.0;
  };
  // groups of D steps: the next group's operands are loaded while the current
  // group's MFMAs run (rows past the chunk load zeros)
  constexpr int D = 4;
  double a[D][2], b[D][2], na[D][2], nb[D][2];
  int r = r0 + wave * 4;
#pragma unroll
  for (int u = 0; u < D; ++u) load(r + 16 * u, a[u][0], a[u][1], b[u][0], b[u][1]);
  for (; r < r1; r += 16 * D) {
#pragma unroll
    for (int u = 0; u < D; ++u) load(r + 16 * (D + u), na[u][0], na[u][1], nb[u][0], nb[u][1]);
#pragma unroll
    for (int u = 0; u < D; ++u) {
      acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u][0], b[u][0], acc[0][0], 0, 0, 0);
      acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u][0], b[u][1], acc[0][1], 0, 0, 0);
      acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u][1], b[u][0], acc[1][0], 0, 0, 0);
      acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u][1], b[u][1], acc[1][1], 0, 0, 0);
    }
#pragma unroll
    for (int u = 0; u < D; ++u) {
      a[u][0] = na[u][0];
      a[u][1] = na[u][1];
      b[u][0] = nb[u][0];
      b[u][1] = nb[u][1];
    }
  }
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = a * 16 + 4 * v + (l >> 4);
        const int j = b * 16 + (l & 15);
        red[wave][i * 32 + j] = acc[a][b][v];
      }
  __syncthreads();
  double* pc = part + (size_t)chunk * p * q;
  for (int t = threadIdx.x; t < 32 * 32; t += 256) {
    const int i = ib + t / 32, j = jb + t % 32;
    if (i < p && j < q) pc[(size_t)i * q + j] = ((red[0][t] + red[1][t]) + red[2][t]) + red[3][t];
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

// Z = alpha X S + beta Z.  Workgroup: 128 rows (4 waves x 32 rows) x 32
// columns (2x2 MFMA tiles per wave); the 32 columns of S are staged in LDS 64
// rows of k at a time and shared by the waves, each of which loads its next
// X operands while its MFMAs run.
constexpr int kGemmK = 64;
__global__ __launch_bounds__(256) void k_gemm_tall(int n, int p, int q, double alpha,
                                                   const double* __restrict__ X, int ldx,
                                                   const double* __restrict__ S, int lds,
                                                   double beta, double* __restrict__ Z, int ldz) {
  __shared__ double sS[kGemmK][32];
  const int ncb = (q + 31) / 32;
  // XCD-aware order: each XCD takes a contiguous range of (row block, column
  // block) pairs, column blocks fastest, so an X row block is fetched into one
  // L2 for all its column blocks
  const long total = (long)((n + 127) / 128) * ncb;
  const long per = (total + 7) / 8;
  const long w8 = (long)(blockIdx.x & 7) * per + (blockIdx.x >> 3);
  if (w8 >= total) return;
  const int rb = (int)(w8 / ncb), cb = (int)(w8 % ncb);
  const int wave = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int r0 = rb * 128 + wave * 32;
  const int jb = cb * 32;
  const int kk = l >> 4, ii = l & 15;
  d4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = d4{0.0, 0.0, 0.0, 0.0};
  const int ar0 = r0 + ii, ar1 = r0 + 16 + ii;
  const bool ok0 = ar0 < n, ok1 = ar1 < n;
  const double* x0 = X + (size_t)(ok0 ? ar0 : 0) * ldx;
  const double* x1 = X + (size_t)(ok1 ? ar1 : 0) * ldx;
  for (int k0 = 0; k0 < p; k0 += kGemmK) {
    const int kn = min(kGemmK, p - k0);
    __syncthreads();  // (the previous slab is consumed)
    for (int t = threadIdx.x; t < kGemmK * 32; t += 256) {
      const int kr = t / 32, j = jb + t % 32;
      sS[kr][t % 32] = (kr < kn && j < q) ? S[(size_t)(k0 + kr) * lds + j] : 0.0;
    }
    __syncthreads();
    auto ld = [&](int kc, double& a0, double& a1) {
      const bool okk = kc < p;
      a0 = (ok0 && okk) ? x0[kc] : 0.0;
      a1 = (ok1 && okk) ? x1[kc] : 0.0;
    };
    // the slab's X operands in groups of four k-steps, the next group
    // loaded while the current one's MFMAs run (past p: zeros)
    double a[4][2], na[4][2];
#pragma unroll
    for (int u = 0; u < 4; ++u) ld(k0 + 4 * u + kk, a[u][0], a[u][1]);
    for (int kr = 0; kr < kn; kr += 16) {
#pragma unroll
      for (int u = 0; u < 4; ++u) ld(k0 + kr + 16 + 4 * u + kk, na[u][0], na[u][1]);
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int k = kr + 4 * u + kk;  // (< kGemmK + 12: rows past kn hold zeros)
        const double b0 = k < kGemmK ? sS[k][ii] : 0.0, b1 = k < kGemmK ? sS[k][16 + ii] : 0.0;
        acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u][0], b0, acc[0][0], 0, 0, 0);
        acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u][0], b1, acc[0][1], 0, 0, 0);
        acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u][1], b0, acc[1][0], 0, 0, 0);
        acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u][1], b1, acc[1][1], 0, 0, 0);
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        a[u][0] = na[u][0];
        a[u][1] = na[u][1];
      }
    }
  }
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = r0 + a * 16 + 4 * v + (l >> 4);
        const int j = jb + b * 16 + (l & 15);
        if (i < n && j < q) {
          const size_t o = (size_t)i * ldz + j;
          Z[o] = alpha * acc[a][b][v] + (beta == 0.0 ? 0.0 : beta * Z[o]);
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
  k_spmm_real<<<cdiv(cdiv(P.n, 4), 8) * 8, 256, 0, s>>>(P.n, P.rowptr, P.col, P.a, P.b, X, ld,
                                                         nc, AX, BX, theta, E);
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
  const size_t total = (size_t)cdiv(p, 32) * cdiv(q, 32) * nchunk;
  k_gram<<<cdiv(total, 8) * 8, 256, 0, s>>>(n, p, q, X, ldx, Y, ldy, part, rpc, nchunk);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  k_chunk_sum<<<cdiv((size_t)p * q, 256), 256, 0, s>>>(part, nchunk, p, q, G, ldg);
  return hipGetLastError();
}

hipError_t launch_gemm_tall(int n, int p, int q, double alpha, const double* X, int ldx,
                            const double* S, int lds, double beta, double* Z, int ldz,
                            hipStream_t s) {
  if (n == 0 || q == 0) return hipSuccess;
  const size_t total = (size_t)cdiv(n, 128) * cdiv(q, 32);
  k_gemm_tall<<<cdiv(total, 8) * 8, 256, 0, s>>>(n, p, q, alpha, X, ldx, S, lds, beta, Z, ldz);
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
