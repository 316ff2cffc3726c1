// Real FP64 kernels of the outer iteration (Rayleigh-Ritz, B-orthogonalisation,
// residual check) on row-major n x ld blocks, plus setup helpers.
//
// The tall-skinny Gram G = X^T Y and the product Z = X S run on the FP64
// matrix cores (v_mfma_f64_16x16x4f64): operand A is a 16x4 tile (lane l holds
// row l%16, k l/16), operand B a 4x16 tile (lane l holds k l/16, column l%16),
// and the 16x16 accumulator holds in lane l, element v the entry
// (row 4*v + l/16, column l%16) (established by an on-device layout check).
#include <algorithm>
#include <cstdint>

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
// Workgroup: one 160x160 super-tile of G and one chunk of rows; wave w forms the
// 80x80 quarter (w / 2, w % 2) as 5x5 MFMA blocks (200 accumulator registers:
// one wave per SIMD).  Slabs of kGS rows of the super-tile's 160 columns of X
// and of Y are staged in LDS by coalesced loads, double-buffered: the next slab
// is loaded into registers while the waves run the current slab's MFMAs with
// operands read from LDS (row stride 176 doubles: the four rows a 64-lane read
// touches fall in alternate bank halves).  Each quarter is written whole to the
// chunk's partial block; k_chunk_sum adds the chunks in order.
constexpr int kGS = 16;             // rows per LDS slab
constexpr int kGT = 160;            // super-tile side
constexpr int kGStride = 176;       // LDS row stride (doubles)
constexpr int kGPer = kGS * kGT / 2 / 256;  // element pairs per thread, array and slab
static_assert(kGS * kGT / 2 % 256 == 0, "a slab is a whole number of pairs per thread");
template <bool PAIRS>
__global__ __launch_bounds__(256, 1) void k_gram(int n, int p, int q, const double* __restrict__ X,
                                                 int ldx, const double* __restrict__ Y, int ldy,
                                                 double* __restrict__ part, int rows_per_chunk,
                                                 int nchunk) {
  extern __shared__ double sm[];
  double* sX = sm;                          // [2][kGS][kGStride]
  double* sY = sm + 2 * kGS * kGStride;     // [2][kGS][kGStride]
  const int ntj = (q + kGT - 1) / kGT;
  const long ntile = (long)((p + kGT - 1) / kGT) * ntj;
  // XCD-aware order: each XCD takes a contiguous range of (chunk, tile) pairs
  const long total = ntile * nchunk;
  const long per = (total + 7) / 8;
  const long w8 = (long)(blockIdx.x & 7) * per + (blockIdx.x >> 3);
  if (w8 >= total) return;
  const int chunk = (int)(w8 / ntile);
  const int tile = (int)(w8 % ntile);
  const int ib = (tile / ntj) * kGT, jb = (tile % ntj) * kGT;
  const int wave = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int kk = l >> 4, ii = l & 15;
  const int qi = (wave >> 1) * 80, qj = (wave & 1) * 80;
  // (a quarter wholly past p or q has nothing to form)
  const bool live = ib + qi < p && jb + qj < q;
  const int r0 = chunk * rows_per_chunk, r1 = min(r0 + rows_per_chunk, n);
  d4 acc[5][5];
#pragma unroll
  for (int a = 0; a < 5; ++a)
#pragma unroll
    for (int b = 0; b < 5; ++b) acc[a][b] = d4{0.0, 0.0, 0.0, 0.0};
  // staging: pair e = t * 256 + tid of a slab holds row e / 80, columns 2 (e % 80) + {0, 1}
  double2 gx[kGPer], gy[kGPer];
  auto pair = [&](const double* __restrict__ M, int ld, int row, int c0, int lim) {
    const double* m = M + (size_t)row * ld + c0;
    if (PAIRS && c0 + 1 < lim) return *reinterpret_cast<const double2*>(m);
    return make_double2(c0 < lim ? m[0] : 0.0, c0 + 1 < lim ? m[1] : 0.0);
  };
  auto gload = [&](int rs) {
#pragma unroll
    for (int t = 0; t < kGPer; ++t) {
      const int e = t * 256 + threadIdx.x, rr = e / 80, c = 2 * (e % 80);
      const int row = rs + rr;
      const bool ok = row < r1;
      gx[t] = ok ? pair(X, ldx, row, ib + c, p) : make_double2(0.0, 0.0);
      gy[t] = ok ? pair(Y, ldy, row, jb + c, q) : make_double2(0.0, 0.0);
    }
  };
  auto lstore = [&](int buf) {
#pragma unroll
    for (int t = 0; t < kGPer; ++t) {
      const int e = t * 256 + threadIdx.x, rr = e / 80, c = 2 * (e % 80);
      *reinterpret_cast<double2*>(sX + (buf * kGS + rr) * kGStride + c) = gx[t];
      *reinterpret_cast<double2*>(sY + (buf * kGS + rr) * kGStride + c) = gy[t];
    }
  };
  int buf = 0;
  gload(r0);
  lstore(0);
  __syncthreads();
  for (int rs = r0; rs < r1; rs += kGS) {
    const bool more = rs + kGS < r1;
    if (more) gload(rs + kGS);
    if (live) {
      const double* bx = sX + buf * kGS * kGStride + qi + ii;
      const double* by = sY + buf * kGS * kGStride + qj + ii;
#pragma unroll
      for (int st = 0; st < kGS / 4; ++st) {
        double a[5], b[5];
        const int rr = st * 4 + kk;
#pragma unroll
        for (int t = 0; t < 5; ++t) {
          a[t] = bx[rr * kGStride + 16 * t];
          b[t] = by[rr * kGStride + 16 * t];
        }
#pragma unroll
        for (int x = 0; x < 5; ++x)
#pragma unroll
          for (int y = 0; y < 5; ++y)
            acc[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[x], b[y], acc[x][y], 0, 0, 0);
      }
    }
    if (more) lstore(buf ^ 1);
    __syncthreads();  // (the slab is consumed and the next one stored)
    buf ^= 1;
  }
  double* pc = part + (size_t)chunk * p * q;
#pragma unroll
  for (int x = 0; x < 5; ++x)
#pragma unroll
    for (int y = 0; y < 5; ++y)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = ib + qi + x * 16 + 4 * v + (l >> 4);
        const int j = jb + qj + y * 16 + (l & 15);
        if (i < p && j < q) pc[(size_t)i * q + j] = acc[x][y][v];
      }
}

// G = sum of the chunks' partial blocks.  A workgroup takes 64 entries; its four
// waves sum interleaved quarters of the chunks (chunk c to wave c % 4, each in
// chunk order) and the four sums are added in wave order: a fixed order.
__global__ __launch_bounds__(256) void k_chunk_sum(const double* __restrict__ part, int nchunk,
                                                   int p, int q, double* __restrict__ G, int ldg) {
  __shared__ double red[4][64];
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int t = blockIdx.x * 64 + l;
  const size_t pq = (size_t)p * q;
  double s = 0.0;
  if (t < (int)pq)
    for (int c = w; c < nchunk; c += 4) s += part[(size_t)c * pq + t];
  red[w][l] = s;
  __syncthreads();
  if (w == 0 && t < (int)pq) {
    const int i = t / q, j = t % q;
    G[(size_t)i * ldg + j] = ((red[0][l] + red[1][l]) + red[2][l]) + red[3][l];
  }
}

// Z = alpha X S + beta Z.  Workgroup: a 128-row x 160-column block of Z; wave
// w forms rows 64 (w / 2) .. + 64 and columns 80 (w % 2) .. + 80 as 4x5 MFMA
// blocks (20 MFMAs per 9 LDS operand reads).  Slabs of kTK values of k are
// staged in LDS, double-buffered (loaded into registers while the waves run the
// current slab): X's 128 rows x kTK (row stride kTXS) and S's kTK rows x 160
// columns (row stride kGStride), both by coalesced pair loads.  The accumulators
// and the staged pairs take about 270 registers: one wave per SIMD.
constexpr int kTK = 16;             // k per slab
constexpr int kTRows = 128;         // rows of Z per workgroup
constexpr int kTXS = 18;            // LDS row stride of the X slab (doubles)
constexpr int kTXPer = kTRows * kTK / 2 / 256;  // X pairs per thread and slab
constexpr int kTSPer = kTK * kGT / 2 / 256;     // S pairs per thread and slab
static_assert(kTRows * kTK / 2 % 256 == 0 && kTK * kGT / 2 % 256 == 0, "whole pairs per thread");
template <bool PAIRS>
__global__ __launch_bounds__(256, 1) void k_gemm_tall(int n, int p, int q, double alpha,
                                                      const double* __restrict__ X, int ldx,
                                                      const double* __restrict__ S, int lds,
                                                      double beta, double* __restrict__ Z,
                                                      int ldz) {
  extern __shared__ double sm[];
  double* sX = sm;                                  // [2][kTRows][kTXS]
  double* sS = sm + 2 * kTRows * kTXS;              // [2][kTK][kGStride]
  const int ncb = (q + kGT - 1) / kGT;
  // XCD-aware order: each XCD takes a contiguous range of (row block, column
  // block) pairs, column blocks fastest
  const long total = (long)((n + kTRows - 1) / kTRows) * ncb;
  const long per = (total + 7) / 8;
  const long w8 = (long)(blockIdx.x & 7) * per + (blockIdx.x >> 3);
  if (w8 >= total) return;
  const int rb = (int)(w8 / ncb), cbk = (int)(w8 % ncb);
  const int row0 = rb * kTRows, jb = cbk * kGT;
  const int wave = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int kk = l >> 4, ii = l & 15;
  const int wr = (wave >> 1) * 64, wc = (wave & 1) * 80;
  const bool live = row0 + wr < n && jb + wc < q;
  d4 acc[4][5];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 5; ++b) acc[a][b] = d4{0.0, 0.0, 0.0, 0.0};
  auto pair = [&](const double* __restrict__ M, size_t off, int c0, int lim) {
    const double* m = M + off;
    if (PAIRS && c0 + 1 < lim) return *reinterpret_cast<const double2*>(m);
    return make_double2(c0 < lim ? m[0] : 0.0, c0 + 1 < lim ? m[1] : 0.0);
  };
  double2 gx[kTXPer], gs[kTSPer];
  auto gload = [&](int k0) {
#pragma unroll
    for (int t = 0; t < kTXPer; ++t) {  // X pair e: row e / 8, k 2 (e % 8) + {0, 1}
      const int e = t * 256 + threadIdx.x, r = row0 + e / 8, k = k0 + 2 * (e % 8);
      gx[t] = r < n ? pair(X, (size_t)r * ldx + k, k, p) : make_double2(0.0, 0.0);
    }
#pragma unroll
    for (int t = 0; t < kTSPer; ++t) {  // S pair e: k row e / 80, columns 2 (e % 80) + {0, 1}
      const int e = t * 256 + threadIdx.x, k = k0 + e / 80, c = jb + 2 * (e % 80);
      gs[t] = k < p ? pair(S, (size_t)k * lds + c, c, q) : make_double2(0.0, 0.0);
    }
  };
  auto lstore = [&](int buf) {
#pragma unroll
    for (int t = 0; t < kTXPer; ++t) {
      const int e = t * 256 + threadIdx.x;
      *reinterpret_cast<double2*>(sX + (buf * kTRows + e / 8) * kTXS + 2 * (e % 8)) = gx[t];
    }
#pragma unroll
    for (int t = 0; t < kTSPer; ++t) {
      const int e = t * 256 + threadIdx.x;
      *reinterpret_cast<double2*>(sS + (buf * kTK + e / 80) * kGStride + 2 * (e % 80)) = gs[t];
    }
  };
  int buf = 0;
  gload(0);
  lstore(0);
  __syncthreads();
  for (int k0 = 0; k0 < p; k0 += kTK) {
    const bool more = k0 + kTK < p;
    if (more) gload(k0 + kTK);
    if (live) {
      const double* bx = sX + (buf * kTRows + wr + ii) * kTXS + kk;
      const double* bs = sS + (buf * kTK + kk) * kGStride + wc + ii;
#pragma unroll
      for (int st = 0; st < kTK / 4; ++st) {
        double a[4], b[5];
#pragma unroll
        for (int t = 0; t < 4; ++t) a[t] = bx[16 * t * kTXS + 4 * st];
#pragma unroll
        for (int t = 0; t < 5; ++t) b[t] = bs[4 * st * kGStride + 16 * t];
#pragma unroll
        for (int x = 0; x < 4; ++x)
#pragma unroll
          for (int y = 0; y < 5; ++y)
            acc[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[x], b[y], acc[x][y], 0, 0, 0);
      }
    }
    if (more) lstore(buf ^ 1);
    __syncthreads();
    buf ^= 1;
  }
  if (!live) return;
#pragma unroll
  for (int x = 0; x < 4; ++x)
#pragma unroll
    for (int y = 0; y < 5; ++y)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = row0 + wr + x * 16 + 4 * v + (l >> 4);
        const int j = jb + wc + y * 16 + (l & 15);
        if (i < n && j < q) {
          const size_t o = (size_t)i * ldz + j;
          Z[o] = alpha * acc[x][y][v] + (beta == 0.0 ? 0.0 : beta * Z[o]);
        }
      }
}

// Per column c: sum over a chunk of rows of (X - theta_c Y)^2 and of W Y.  A
// workgroup takes one chunk and 64 columns; its four waves take a quarter of
// the chunk's rows each and their partial sums are added in wave order.
__global__ __launch_bounds__(256) void k_colstats(int n, int nc, const double* __restrict__ X,
                                                  const double* __restrict__ Y, int ld,
                                                  const double* __restrict__ theta,
                                                  const double* __restrict__ W,
                                                  double* __restrict__ part, int rows_per_chunk) {
  __shared__ double red[2][4][64];
  const int chunk = blockIdx.x;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int c = blockIdx.y * 64 + lane;
  const int r0 = chunk * rows_per_chunk, r1 = min(r0 + rows_per_chunk, n);
  const int q = (rows_per_chunk + 3) / 4;
  const int a0 = min(r0 + w * q, r1), a1 = min(a0 + q, r1);
  double s1 = 0.0, s2 = 0.0;
  if (c < nc) {
    const double th = theta ? theta[c] : 0.0;
#pragma unroll 4
    for (int r = a0; r < a1; ++r) {
      const size_t o = (size_t)r * ld + c;
      double x = X[o];
      if (theta) x -= th * Y[o];
      s1 = fma(x, x, s1);
      if (W) s2 = fma(W[o], Y[o], s2);
    }
  }
  red[0][w][lane] = s1;
  red[1][w][lane] = s2;
  __syncthreads();
  if (w == 0 && c < nc) {
    part[((size_t)chunk * 2 + 0) * nc + c] =
        ((red[0][0][lane] + red[0][1][lane]) + red[0][2][lane]) + red[0][3][lane];
    part[((size_t)chunk * 2 + 1) * nc + c] =
        ((red[1][0][lane] + red[1][1][lane]) + red[1][2][lane]) + red[1][3][lane];
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

constexpr int kGramWG = 256;          // Gram workgroups per launch: one per CU
constexpr int kGramMinRows = 4 * kGS;  // fewest rows per chunk
constexpr int kColRows = 1024;

namespace {
// Row chunks of a p x q Gram: kGramWG workgroups over its super-tiles (fewer when
// the chunks would hold under kGramMinRows rows).  nchunk * p * q never exceeds
// gram_part_doubles(n, pq) for p, q <= pq: nchunk <= kGramWG / ntile with
// p * q <= ntile * kGT^2, and nchunk <= cdiv(n, kGramMinRows) with p * q <= pq^2.
int gram_nchunk(int n, int p, int q) {
  const int ntile = cdiv(p, kGT) * cdiv(q, kGT);
  const int by_rows = n <= 0 ? 1 : cdiv(n, kGramMinRows);
  return std::max(1, std::min(by_rows, kGramWG / std::max(ntile, 1)));
}
}  // namespace

size_t gram_part_doubles(int n, int pq) {
  const size_t by_rows = (size_t)(n <= 0 ? 1 : cdiv(n, kGramMinRows)) * pq * pq;
  return std::min((size_t)kGramWG * kGT * kGT, by_rows);
}
int colstat_chunks(int n) { return n <= 0 ? 1 : (n + kColRows - 1) / kColRows; }

hipError_t launch_spmm_real(const DevPencil& P, const double* X, int ld, int nc, double* AX,
                            double* BX, const double* theta, double* E, hipStream_t s) {
  if (P.n == 0 || nc == 0) return hipSuccess;
  hipError_t err = hipSuccess;
  if (launch_spmm_real_halo(P, X, ld, nc, AX, BX, theta, E, s, err)) return err;
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
                       double* part, double* G, int ldg, hipStream_t s) {
  if (p == 0 || q == 0) return hipSuccess;
  const int nchunk = gram_nchunk(n, p, q);
  // (rows per chunk: whole slabs; the last chunk may be short or, rounded up, empty)
  const int rows = (n + nchunk - 1) / nchunk;
  const int rpc = ((rows + kGS - 1) / kGS) * kGS;
  const size_t total = (size_t)cdiv(p, kGT) * cdiv(q, kGT) * nchunk;
  const size_t lds = sizeof(double) * 4 * kGS * kGStride;  // 90 KB of the 160 KB per CU
  static const bool lds_ok = [] {
    const int b = (int)(sizeof(double) * 4 * kGS * kGStride);
    return hipFuncSetAttribute(reinterpret_cast<const void*>(&k_gram<true>),
                               hipFuncAttributeMaxDynamicSharedMemorySize, b) == hipSuccess &&
           hipFuncSetAttribute(reinterpret_cast<const void*>(&k_gram<false>),
                               hipFuncAttributeMaxDynamicSharedMemorySize, b) == hipSuccess;
  }();
  if (!lds_ok) return hipErrorInvalidConfiguration;
  const bool pairs = ((ldx | ldy) & 1) == 0 && ((reinterpret_cast<uintptr_t>(X) |
                                                 reinterpret_cast<uintptr_t>(Y)) & 15) == 0;
  if (pairs)
    k_gram<true><<<cdiv(total, 8) * 8, 256, lds, s>>>(n, p, q, X, ldx, Y, ldy, part, rpc, nchunk);
  else
    k_gram<false><<<cdiv(total, 8) * 8, 256, lds, s>>>(n, p, q, X, ldx, Y, ldy, part, rpc, nchunk);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  k_chunk_sum<<<cdiv((size_t)p * q, 64), 256, 0, s>>>(part, nchunk, p, q, G, ldg);
  return hipGetLastError();
}

hipError_t launch_gemm_tall(int n, int p, int q, double alpha, const double* X, int ldx,
                            const double* S, int lds, double beta, double* Z, int ldz,
                            hipStream_t s) {
  if (n == 0 || q == 0) return hipSuccess;
  if (p == 0) {
    // (no k: Z = beta Z; not used by the library, kept well defined)
    return beta == 1.0 ? hipSuccess : hipErrorInvalidValue;
  }
  const size_t total = (size_t)cdiv(n, kTRows) * cdiv(q, kGT);
  const size_t bytes = sizeof(double) * 2 * (kTRows * kTXS + kTK * kGStride);  // 58 KB
  static const bool lds_ok = [] {
    const int b = (int)(sizeof(double) * 2 * (kTRows * kTXS + kTK * kGStride));
    return hipFuncSetAttribute(reinterpret_cast<const void*>(&k_gemm_tall<true>),
                               hipFuncAttributeMaxDynamicSharedMemorySize, b) == hipSuccess &&
           hipFuncSetAttribute(reinterpret_cast<const void*>(&k_gemm_tall<false>),
                               hipFuncAttributeMaxDynamicSharedMemorySize, b) == hipSuccess;
  }();
  if (!lds_ok) return hipErrorInvalidConfiguration;
  const bool pairs = ((ldx | lds) & 1) == 0 && ((reinterpret_cast<uintptr_t>(X) |
                                                 reinterpret_cast<uintptr_t>(S)) & 15) == 0;
  if (pairs)
    k_gemm_tall<true><<<cdiv(total, 8) * 8, 256, bytes, s>>>(n, p, q, alpha, X, ldx, S, lds, beta,
                                                             Z, ldz);
  else
    k_gemm_tall<false><<<cdiv(total, 8) * 8, 256, bytes, s>>>(n, p, q, alpha, X, ldx, S, lds, beta,
                                                              Z, ldz);
  return hipGetLastError();
}

hipError_t launch_colstats(int n, int nc, const double* X, const double* Y, int ld,
                           const double* theta, const double* W, double* part, int nchunk,
                           double* out, double* out2, hipStream_t s) {
  if (nc == 0) return hipSuccess;
  const int rpc = (n + nchunk - 1) / nchunk;
  k_colstats<<<dim3(nchunk, cdiv(nc, 64)), 256, 0, s>>>(n, nc, X, Y, ld, theta, W, part, rpc);
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
