// Batched complex block kernels of the filter's inner solves (gfx950, wave64).
//
// Every (pole, column) system of Eq. (2) is a slot of the resident pool; the
// complex vectors of all slots live in the panel layout (see internal.h).  One
// GCR step (Section 3.2 solver, restarted, right-preconditioned, classical
// Gram-Schmidt) is:
//
//   apply : q_k = (A - sigma B) z          (CSR gather, one pass serves all
//           h_i = <q_i, q_k>, i < k          slots of a panel) fused with the
//                                            CGS projections
//   orth  : q_k -= sum beta_i q_i, p_k = z - sum beta_i p_i,
//           partial <q_k, q_k>, <q_k, r>
//   step  : r -= alpha q_k, z = P^-1 r, partial ||r||^2
//
// followed, at cycle ends, by the FP64 solution update y += sum alpha_i p_i and
// the FP64 true residual r = f - (A - sigma B) y (the refinement step of the
// mixed-precision form).  Dot products are accumulated in FP64 in every
// precision; partial sums are written per (row block, slot) and reduced in a
// fixed order by a second kernel, so results are bitwise reproducible.
//
// Workgroups of 256 threads: thread t serves slot lane t % 16 of its panel and
// row subgroup t / 16; a wave covers 4 rows x 16 slots.
#include "internal.h"

namespace slrf {
namespace {

template <typename T>
struct CT;
template <>
struct CT<float> {
  using t = float2;
};
template <>
struct CT<double> {
  using t = double2;
};

__device__ __forceinline__ float mad(float a, float b, float c) { return fmaf(a, b, c); }
__device__ __forceinline__ double mad(double a, double b, double c) { return fma(a, b, c); }

template <typename C>
__device__ __forceinline__ C mk(double x, double y);
template <>
__device__ __forceinline__ float2 mk<float2>(double x, double y) {
  return make_float2((float)x, (float)y);
}
template <>
__device__ __forceinline__ double2 mk<double2>(double x, double y) {
  return make_double2(x, y);
}

// Workgroup -> (row block, panel) tile.  Consecutive workgroups are dealt to
// the 8 XCDs round-robin; each XCD receives a contiguous range of tiles, and
// within a range `group` panels advance together over the row blocks so that
// the CSR rows of a row block are fetched once into that XCD's L2 and reused
// by the panels of the group.
__device__ __forceinline__ bool map_block(const PanelGrid& g, int& rb, int& pan) {
  const long total = (long)g.nrb * g.npan;
  const long per = (total + 7) / 8;
  const long b = blockIdx.x;
  const long t = (b & 7) * per + (b >> 3);
  if (t >= total) return false;
  const long G = g.group;
  const long pg = t / ((long)g.nrb * G);
  const long rem = t - pg * (long)g.nrb * G;
  const long gw = min(G, (long)g.npan - pg * G);
  rb = (int)(rem / gw);
  pan = (int)(pg * G + rem % gw);
  return true;
}

// Sum nv per-thread values over the 16 row subgroups that share a slot lane.
// vals[v] in every thread; result for (v, lane) is delivered through `emit`.
template <int NVMAX, typename Emit>
__device__ __forceinline__ void reduce16(const double* vals, int nv, double* red, Emit emit) {
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
#pragma unroll
  for (int v = 0; v < NVMAX; ++v) {
    if (v < nv) {
      double x = vals[v];
      x += __shfl_xor(x, 16);
      x += __shfl_xor(x, 32);
      if (l < 16) red[(w * NVMAX + v) * 16 + l] = x;
    }
  }
  __syncthreads();
  for (int t = threadIdx.x; t < nv * 16; t += kThreads) {
    const int v = t >> 4, ln = t & 15;
    const double s = ((red[(0 * NVMAX + v) * 16 + ln] + red[(1 * NVMAX + v) * 16 + ln]) +
                      red[(2 * NVMAX + v) * 16 + ln]) +
                     red[(3 * NVMAX + v) * 16 + ln];
    emit(v, ln, s);
  }
}

__device__ __forceinline__ double2 jacobi_inv(double da, double db, double2 sg) {
  // 1 / (da - sigma db)
  const double dx = da - sg.x * db, dy = -sg.y * db;
  const double inv = 1.0 / (dx * dx + dy * dy);
  return make_double2(dx * inv, -dy * inv);
}

// ---------------------------------------------------------------------------
// apply: q_k = (A - sigma B) z, fused CGS projections h_i = <q_i, q_k>, i < k
//
// The workgroup walks its row block 16 rows at a time.  Phase 1 (one thread
// per (row, slot)): CSR gather of z, q written to HBM and to an LDS tile.
// Phase 2 (one thread per (slot, i), i and i + 16): the projections read the
// stored directions q_i for the 16 rows (one coalesced segment per row) and
// the fresh q from LDS.  Each thread owns a complete (slot, i) partial sum of
// the row block, so no cross-thread reduction is needed and the register
// footprint stays small at any k.
// ---------------------------------------------------------------------------
template <typename T, bool DOTS>
__global__ __launch_bounds__(kThreads) void k_apply_dots(
    int n, const int* __restrict__ rowptr, const int* __restrict__ col, const T* __restrict__ av,
    const T* __restrict__ bv, PanelGrid g, const int* __restrict__ active,
    const double2* __restrict__ sigma, const typename CT<T>::t* __restrict__ Z,
    typename CT<T>::t* __restrict__ Qk, const typename CT<T>::t* __restrict__ Qb, size_t vstride,
    int k, double2* __restrict__ part) {
  using C = typename CT<T>::t;
  __shared__ C sq[16][kPanel];
  int rb, pan;
  if (!map_block(g, rb, pan)) return;
  const int lane = threadIdx.x & 15, rs = threadIdx.x >> 4;
  const int slot = pan * kPanel + lane;
  const bool act = active == nullptr || active[slot] != 0;
  if (!__syncthreads_or(act)) return;
  const double2 sg = sigma[slot];
  const T sr = (T)sg.x, si = (T)sg.y;
  const size_t pbase = (size_t)pan * n * kPanel;
  const C* __restrict__ Zp = Z + pbase;
  C* __restrict__ Qp = Qk + pbase;
  const int r0 = rb * g.rpb, r1 = min(r0 + g.rpb, n);
  // phase-2 role of this thread: slot `lane`, projections i0 = rs and i1 = rs + 16
  const int i0 = rs, i1 = rs + 16;
  const C* __restrict__ Q0 = Qb + (size_t)i0 * vstride + pbase;
  const C* __restrict__ Q1 = Qb + (size_t)i1 * vstride + pbase;
  double h0x = 0.0, h0y = 0.0, h1x = 0.0, h1y = 0.0;
  for (int row0 = r0; row0 < r1; row0 += 16) {
    const int row = row0 + rs;
    if (act && row < r1) {
      const int e0 = rowptr[row], e1 = rowptr[row + 1];
      T ar = 0, ai = 0, br = 0, bi = 0;
      int e = e0;
      for (; e + 3 < e1; e += 4) {
        int c[4];
        T a[4], b[4];
        C z[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          c[u] = col[e + u];
          a[u] = av[e + u];
          b[u] = bv[e + u];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) z[u] = Zp[c[u] * kPanel + lane];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          ar = mad(a[u], z[u].x, ar);
          ai = mad(a[u], z[u].y, ai);
          br = mad(b[u], z[u].x, br);
          bi = mad(b[u], z[u].y, bi);
        }
      }
      for (; e < e1; ++e) {
        const int c = col[e];
        const T a = av[e], b = bv[e];
        const C z = Zp[c * kPanel + lane];
        ar = mad(a, z.x, ar);
        ai = mad(a, z.y, ai);
        br = mad(b, z.x, br);
        bi = mad(b, z.y, bi);
      }
      C q;
      q.x = ar - (sr * br - si * bi);
      q.y = ai - (sr * bi + si * br);
      Qp[row * kPanel + lane] = q;
      if constexpr (DOTS) sq[rs][lane] = q;
    }
    if constexpr (DOTS) {
      __syncthreads();
      if (act) {
        const int nr = min(16, r1 - row0);
        if (i0 < k) {
#pragma unroll 4
          for (int rr = 0; rr < nr; ++rr) {
            const C v = Q0[(row0 + rr) * kPanel + lane];
            const C q = sq[rr][lane];
            h0x += (double)v.x * q.x + (double)v.y * q.y;
            h0y += (double)v.x * q.y - (double)v.y * q.x;
          }
        }
        if (i1 < k) {
#pragma unroll 4
          for (int rr = 0; rr < nr; ++rr) {
            const C v = Q1[(row0 + rr) * kPanel + lane];
            const C q = sq[rr][lane];
            h1x += (double)v.x * q.x + (double)v.y * q.y;
            h1y += (double)v.x * q.y - (double)v.y * q.x;
          }
        }
      }
      __syncthreads();
    }
  }
  if constexpr (DOTS) {
    if (i0 < k) part[((size_t)rb * g.ND + i0) * g.C + slot] = make_double2(h0x, h0y);
    if (i1 < k) part[((size_t)rb * g.ND + i1) * g.C + slot] = make_double2(h1x, h1y);
  }
}

// ---------------------------------------------------------------------------
// orth: q_k -= sum beta_i q_i ; p_k = z - sum beta_i p_i ; partial <q,q>, <q,r>
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(kThreads) void k_orth(
    int n, PanelGrid g, const int* __restrict__ active, typename CT<T>::t* __restrict__ Qk,
    typename CT<T>::t* __restrict__ Pk, const typename CT<T>::t* __restrict__ Z,
    const typename CT<T>::t* __restrict__ R, const typename CT<T>::t* __restrict__ Qb,
    const typename CT<T>::t* __restrict__ Pb, size_t vstride, int k,
    const double2* __restrict__ beta, double2* __restrict__ part) {
  using C = typename CT<T>::t;
  __shared__ double2 sb[kMaxRestart * kPanel];
  __shared__ double red[4 * 3 * 16];
  int rb, pan;
  if (!map_block(g, rb, pan)) return;
  const int lane = threadIdx.x & 15, rs = threadIdx.x >> 4;
  const int slot = pan * kPanel + lane;
  const bool act = active[slot] != 0;
  if (!__syncthreads_or(act)) return;
  for (int t = threadIdx.x; t < k * kPanel; t += kThreads)
    sb[t] = beta[(size_t)(t >> 4) * g.C + pan * kPanel + (t & 15)];
  __syncthreads();
  double acc[3] = {0.0, 0.0, 0.0};
  const size_t base = (size_t)pan * n;
  const int r0 = rb * g.rpb, r1 = min(r0 + g.rpb, n);
  if (act) {
    for (int row = r0 + rs; row < r1; row += 16) {
      const size_t off = (base + row) * kPanel + lane;
      const C q = Qk[off];
      const C z = Z[off];
      double qx = q.x, qy = q.y, px = z.x, py = z.y;
#pragma unroll 4
      for (int i = 0; i < k; ++i) {
        const double2 b = sb[i * kPanel + lane];
        const C vq = Qb[(size_t)i * vstride + off];
        const C vp = Pb[(size_t)i * vstride + off];
        qx -= b.x * vq.x - b.y * vq.y;
        qy -= b.x * vq.y + b.y * vq.x;
        px -= b.x * vp.x - b.y * vp.y;
        py -= b.x * vp.y + b.y * vp.x;
      }
      const C qn = mk<C>(qx, qy);
      Qk[off] = qn;
      Pk[off] = mk<C>(px, py);
      const C r = R[off];
      const double nx = qn.x, ny = qn.y;
      acc[0] += nx * nx + ny * ny;
      acc[1] += nx * r.x + ny * r.y;
      acc[2] += nx * r.y - ny * r.x;
    }
  }
  reduce16<3>(acc, 3, red, [&](int v, int ln, double s) {
    const size_t dst = ((size_t)rb * g.ND + (v == 0 ? 0 : 1)) * g.C + pan * kPanel + ln;
    double* d = reinterpret_cast<double*>(part + dst);
    if (v == 0) {
      d[0] = s;
      d[1] = 0.0;
    } else {
      d[v - 1] = s;
    }
  });
}

// ---------------------------------------------------------------------------
// step: r -= alpha q_k ; z = P^-1 r ; partial ||r||^2
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(kThreads) void k_step(
    int n, PanelGrid g, const int* __restrict__ active, const double2* __restrict__ sigma,
    const double* __restrict__ da, const double* __restrict__ db, int pc,
    typename CT<T>::t* __restrict__ R, typename CT<T>::t* __restrict__ Z,
    const typename CT<T>::t* __restrict__ Qk, const double2* __restrict__ alpha_k,
    double2* __restrict__ part) {
  using C = typename CT<T>::t;
  __shared__ double red[4 * 1 * 16];
  int rb, pan;
  if (!map_block(g, rb, pan)) return;
  const int lane = threadIdx.x & 15, rs = threadIdx.x >> 4;
  const int slot = pan * kPanel + lane;
  const bool act = active[slot] != 0;
  if (!__syncthreads_or(act)) return;
  const double2 al = alpha_k[slot];
  const double2 sg = sigma[slot];
  double acc[1] = {0.0};
  const size_t base = (size_t)pan * n;
  const int r0 = rb * g.rpb, r1 = min(r0 + g.rpb, n);
  if (act) {
    for (int row = r0 + rs; row < r1; row += 16) {
      const size_t off = (base + row) * kPanel + lane;
      const C r = R[off];
      const C q = Qk[off];
      const C rn = mk<C>(r.x - (al.x * q.x - al.y * q.y), r.y - (al.x * q.y + al.y * q.x));
      R[off] = rn;
      const double x = rn.x, y = rn.y;
      if (pc) {
        const double2 d = jacobi_inv(da[row], db[row], sg);
        Z[off] = mk<C>(x * d.x - y * d.y, x * d.y + y * d.x);
      } else {
        Z[off] = rn;
      }
      acc[0] += x * x + y * y;
    }
  }
  reduce16<1>(acc, 1, red, [&](int, int ln, double s) {
    part[((size_t)rb * g.ND) * g.C + pan * kPanel + ln] = make_double2(s, 0.0);
  });
}

// ---------------------------------------------------------------------------
// yupdate: y += sum_{i<kk} alpha_i p_i   (FP64 solution)
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(kThreads) void k_yupdate(int n, PanelGrid g,
                                                      const int* __restrict__ sys,
                                                      double2* __restrict__ Y,
                                                      const typename CT<T>::t* __restrict__ Pb,
                                                      size_t vstride, int kk,
                                                      const double2* __restrict__ alpha) {
  using C = typename CT<T>::t;
  __shared__ double2 sa[kMaxRestart * kPanel];
  int rb, pan;
  if (!map_block(g, rb, pan)) return;
  const int lane = threadIdx.x & 15, rs = threadIdx.x >> 4;
  const int slot = pan * kPanel + lane;
  const bool occ = sys[slot] >= 0;
  if (!__syncthreads_or(occ)) return;
  for (int t = threadIdx.x; t < kk * kPanel; t += kThreads)
    sa[t] = alpha[(size_t)(t >> 4) * g.C + pan * kPanel + (t & 15)];
  __syncthreads();
  if (!occ) return;
  const size_t base = (size_t)pan * n;
  const int r0 = rb * g.rpb, r1 = min(r0 + g.rpb, n);
  for (int row = r0 + rs; row < r1; row += 16) {
    const size_t off = (base + row) * kPanel + lane;
    double2 y = Y[off];
#pragma unroll 4
    for (int i = 0; i < kk; ++i) {
      const double2 a = sa[i * kPanel + lane];
      const C p = Pb[(size_t)i * vstride + off];
      y.x += a.x * p.x - a.y * p.y;
      y.y += a.x * p.y + a.y * p.x;
    }
    Y[off] = y;
  }
}

// ---------------------------------------------------------------------------
// true_resid: r = f - (A - sigma B) y in FP64 ; R, Z (inner precision) ; ||r||^2
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(kThreads) void k_true_resid(
    int n, const int* __restrict__ rowptr, const int* __restrict__ col,
    const double* __restrict__ av, const double* __restrict__ bv, const double* __restrict__ da,
    const double* __restrict__ db, int pc, PanelGrid g, const int* __restrict__ sys,
    const int* __restrict__ scol, const double2* __restrict__ sigma,
    const double2* __restrict__ Y, const double* __restrict__ F, int ldf,
    typename CT<T>::t* __restrict__ R, typename CT<T>::t* __restrict__ Z,
    double2* __restrict__ part) {
  using C = typename CT<T>::t;
  __shared__ double red[4 * 1 * 16];
  int rb, pan;
  if (!map_block(g, rb, pan)) return;
  const int lane = threadIdx.x & 15, rs = threadIdx.x >> 4;
  const int slot = pan * kPanel + lane;
  const bool occ = sys[slot] >= 0;
  if (!__syncthreads_or(occ)) return;
  double acc[1] = {0.0};
  const size_t base = (size_t)pan * n;
  const int r0 = rb * g.rpb, r1 = min(r0 + g.rpb, n);
  if (occ) {
    const double2 sg = sigma[slot];
    const int c = scol[slot];
    for (int row = r0 + rs; row < r1; row += 16) {
      const int e0 = rowptr[row], e1 = rowptr[row + 1];
      double ar = 0, ai = 0, br = 0, bi = 0;
      for (int e = e0; e < e1; ++e) {
        const int cc = col[e];
        const double a = av[e], b = bv[e];
        const double2 y = Y[(base + cc) * kPanel + lane];
        ar = fma(a, y.x, ar);
        ai = fma(a, y.y, ai);
        br = fma(b, y.x, br);
        bi = fma(b, y.y, bi);
      }
      const double mx = ar - (sg.x * br - sg.y * bi);
      const double my = ai - (sg.x * bi + sg.y * br);
      const double x = F[(size_t)row * ldf + c] - mx, y = -my;
      const size_t off = (base + row) * kPanel + lane;
      R[off] = mk<C>(x, y);
      if (pc) {
        const double2 d = jacobi_inv(da[row], db[row], sg);
        Z[off] = mk<C>(x * d.x - y * d.y, x * d.y + y * d.x);
      } else {
        Z[off] = mk<C>(x, y);
      }
      acc[0] += x * x + y * y;
    }
  }
  reduce16<1>(acc, 1, red, [&](int, int ln, double s) {
    part[((size_t)rb * g.ND) * g.C + pan * kPanel + ln] = make_double2(s, 0.0);
  });
}

// ---------------------------------------------------------------------------
// admit: compact continuing slots and initialise newly admitted systems
//   y0 = 0, r0 = f                              (cold start)
//   y0 = x / (theta - sigma), r0 = (A - theta B) x / (sigma - theta)
//                                               (warm start, Proposition 4.1)
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(kThreads) void k_admit(
    int n, const double* __restrict__ da, const double* __restrict__ db, int pc, PanelGrid g,
    const int* __restrict__ sys, const int* __restrict__ src, const int* __restrict__ scol,
    const double2* __restrict__ sigma, const double* __restrict__ theta,
    const double2* __restrict__ Yold, const typename CT<T>::t* __restrict__ Rold,
    const typename CT<T>::t* __restrict__ Zold, double2* __restrict__ Ynew,
    typename CT<T>::t* __restrict__ Rnew, typename CT<T>::t* __restrict__ Znew,
    const double* __restrict__ F, const double* __restrict__ E, const double* __restrict__ X,
    int ld, int warm, double2* __restrict__ part) {
  using C = typename CT<T>::t;
  __shared__ double red[4 * 1 * 16];
  int rb, pan;
  if (!map_block(g, rb, pan)) return;
  const int lane = threadIdx.x & 15, rs = threadIdx.x >> 4;
  const int slot = pan * kPanel + lane;
  const bool occ = sys[slot] >= 0;
  if (!__syncthreads_or(occ)) return;
  double acc[1] = {0.0};
  const size_t base = (size_t)pan * n;
  const int r0 = rb * g.rpb, r1 = min(r0 + g.rpb, n);
  if (occ) {
    const int s0 = src[slot];
    if (s0 >= 0) {
      const size_t obase = (size_t)(s0 / kPanel) * n;
      const int ol = s0 % kPanel;
      for (int row = r0 + rs; row < r1; row += 16) {
        const size_t off = (base + row) * kPanel + lane;
        const size_t oo = (obase + row) * kPanel + ol;
        Ynew[off] = Yold[oo];
        Rnew[off] = Rold[oo];
        Znew[off] = Zold[oo];
      }
    } else {
      const double2 sg = sigma[slot];
      const int c = scol[slot];
      double2 inv_ts = make_double2(0.0, 0.0);  // 1 / (theta - sigma)
      double2 inv_st = make_double2(0.0, 0.0);  // 1 / (sigma - theta)
      if (warm) {
        const double dx = theta[slot] - sg.x, dy = -sg.y;
        const double q = 1.0 / (dx * dx + dy * dy);
        inv_ts = make_double2(dx * q, -dy * q);
        inv_st = make_double2(-inv_ts.x, -inv_ts.y);
      }
      for (int row = r0 + rs; row < r1; row += 16) {
        const size_t off = (base + row) * kPanel + lane;
        double x, y;
        if (warm) {
          const double xv = X[(size_t)row * ld + c];
          Ynew[off] = make_double2(xv * inv_ts.x, xv * inv_ts.y);
          const double ev = E[(size_t)row * ld + c];
          x = ev * inv_st.x;
          y = ev * inv_st.y;
        } else {
          Ynew[off] = make_double2(0.0, 0.0);
          x = F[(size_t)row * ld + c];
          y = 0.0;
        }
        Rnew[off] = mk<C>(x, y);
        if (pc) {
          const double2 d = jacobi_inv(da[row], db[row], sg);
          Znew[off] = mk<C>(x * d.x - y * d.y, x * d.y + y * d.x);
        } else {
          Znew[off] = mk<C>(x, y);
        }
        acc[0] += x * x + y * y;
      }
    }
  }
  reduce16<1>(acc, 1, red, [&](int, int ln, double s) {
    part[((size_t)rb * g.ND) * g.C + pan * kPanel + ln] = make_double2(s, 0.0);
  });
}

// retire: copy the FP64 solution of finished slots to the per-system store.
__global__ __launch_bounds__(kThreads) void k_retire(int n, PanelGrid g,
                                                     const int* __restrict__ rsys,
                                                     const double2* __restrict__ Y,
                                                     double2* __restrict__ Ystore) {
  int rb, pan;
  if (!map_block(g, rb, pan)) return;
  const int lane = threadIdx.x & 15, rs = threadIdx.x >> 4;
  const int slot = pan * kPanel + lane;
  const int s = rsys[slot];
  if (s < 0) return;
  const size_t base = (size_t)pan * n, sbase = (size_t)(s / kPanel) * n;
  const int sl = s % kPanel;
  const int r0 = rb * g.rpb, r1 = min(r0 + g.rpb, n);
  for (int row = r0 + rs; row < r1; row += 16)
    Ystore[(sbase + row) * kPanel + sl] = Y[(base + row) * kPanel + lane];
}

// filter sum: U[row, c] = sum_j 2 Re(w_j y_{c N + j}[row]), poles in increasing j
__global__ __launch_bounds__(kThreads) void k_filter_sum(int n, int ncols, int npoles,
                                                         const double2* __restrict__ Ys,
                                                         const double2* __restrict__ w,
                                                         double* __restrict__ Ur) {
  const size_t t = (size_t)blockIdx.x * kThreads + threadIdx.x;
  if (t >= (size_t)n * ncols) return;
  const int row = (int)(t / ncols), c = (int)(t % ncols);
  double u = 0.0;
  for (int j = 0; j < npoles; ++j) {
    const int s = c * npoles + j;
    const double2 y = Ys[((size_t)(s / kPanel) * n + row) * kPanel + s % kPanel];
    const double2 wj = w[j];
    u += 2.0 * (wj.x * y.x - wj.y * y.y);
  }
  Ur[t] = u;
}

// second-stage reduction of per-row-block partial sums (fixed order)
__global__ __launch_bounds__(kThreads) void k_reduce(const double2* __restrict__ part, int nrb,
                                                     int ND, int C, int nd, int nslots,
                                                     double2* __restrict__ out) {
  const int t = blockIdx.x * kThreads + threadIdx.x;
  if (t >= nd * nslots) return;
  const int d = t / nslots, slot = t % nslots;
  double2 s[4] = {};
  int rb = 0;
  for (; rb + 3 < nrb; rb += 4) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const double2 v = part[((size_t)(rb + u) * ND + d) * C + slot];
      s[u].x += v.x;
      s[u].y += v.y;
    }
  }
  for (; rb < nrb; ++rb) {
    const double2 v = part[((size_t)rb * ND + d) * C + slot];
    s[0].x += v.x;
    s[0].y += v.y;
  }
  out[(size_t)d * C + slot] =
      make_double2((s[0].x + s[1].x) + (s[2].x + s[3].x), (s[0].y + s[1].y) + (s[2].y + s[3].y));
}

__global__ void k_fin_beta(const double2* __restrict__ red, int k, int C, int nslots,
                           const int* __restrict__ active, const double* __restrict__ qq,
                           double2* __restrict__ beta) {
  const int slot = blockIdx.x * blockDim.x + threadIdx.x;
  if (slot >= nslots) return;
  const bool act = active[slot] != 0;
  for (int i = 0; i < k; ++i) {
    const double q = qq[(size_t)i * C + slot];
    const double2 h = red[(size_t)i * C + slot];
    beta[(size_t)i * C + slot] =
        (act && q > 0.0) ? make_double2(h.x / q, h.y / q) : make_double2(0.0, 0.0);
  }
}

__global__ void k_fin_alpha(const double2* __restrict__ red, int k, int C, int nslots,
                            int* __restrict__ active, double* __restrict__ qq,
                            double2* __restrict__ alpha) {
  const int slot = blockIdx.x * blockDim.x + threadIdx.x;
  if (slot >= nslots) return;
  const double q = red[slot].x;
  const double2 qr = red[(size_t)C + slot];
  const bool act = active[slot] != 0;
  double2 a = make_double2(0.0, 0.0);
  if (act && q > 0.0) a = make_double2(qr.x / q, qr.y / q);
  if (act && !(q > 0.0)) active[slot] = 0;  // breakdown: direction vanished
  qq[(size_t)k * C + slot] = q;
  alpha[(size_t)k * C + slot] = a;
}

__global__ void k_fin_rnorm(const double2* __restrict__ red, int nslots,
                            const int* __restrict__ sys, int* __restrict__ active,
                            const double* __restrict__ target2, int* __restrict__ its,
                            int* __restrict__ status, int itcap) {
  const int slot = blockIdx.x * blockDim.x + threadIdx.x;
  if (slot >= nslots) return;
  const int s = sys[slot];
  if (s < 0 || active[slot] == 0) return;
  const int it = its[s] + 1;
  its[s] = it;
  const double rn2 = red[slot].x;
  if (!(rn2 == rn2) || rn2 > 1e300) {
    status[slot] = 3;
    active[slot] = 0;
    return;
  }
  if (rn2 <= target2[slot] || it >= itcap) active[slot] = 0;
}

__global__ void k_fin_true(const double2* __restrict__ red, int nslots, int from_admit,
                           const int* __restrict__ sys, const int* __restrict__ src,
                           const int* __restrict__ scol, int* __restrict__ active,
                           double* __restrict__ target2, const double* __restrict__ fnorm2,
                           const int* __restrict__ its, double* __restrict__ sys_rn2,
                           int* __restrict__ status, double tol, double inner_rtol,
                           double safety, int itcap) {
  const int slot = blockIdx.x * blockDim.x + threadIdx.x;
  if (slot >= nslots) return;
  const int s = sys[slot];
  if (s < 0) {
    status[slot] = -1;
    active[slot] = 0;
    return;
  }
  double rn2;
  if (from_admit && src[slot] >= 0)
    rn2 = sys_rn2[s];
  else
    rn2 = red[slot].x;
  sys_rn2[s] = rn2;
  const double f2 = fnorm2[scol[slot]];
  const double tol2 = tol * tol * f2;
  int st;
  if (!(rn2 == rn2) || rn2 > 1e300)
    st = 3;
  else if (rn2 <= tol2)
    st = 1;
  else if (its[s] >= itcap)
    st = 2;
  else
    st = 0;
  status[slot] = st;
  active[slot] = st == 0 ? 1 : 0;
  target2[slot] = fmax(inner_rtol * inner_rtol * rn2, safety * safety * tol2);
}

inline unsigned cdiv(size_t a, size_t b) { return (unsigned)((a + b - 1) / b); }

}  // namespace

// ------------------------------- launchers ---------------------------------

template <typename T>
static const T* vals_a(const DevPencil& P);
template <>
const float* vals_a<float>(const DevPencil& P) {
  return P.a32;
}
template <>
const double* vals_a<double>(const DevPencil& P) {
  return P.a;
}
template <typename T>
static const T* vals_b(const DevPencil& P);
template <>
const float* vals_b<float>(const DevPencil& P) {
  return P.b32;
}
template <>
const double* vals_b<double>(const DevPencil& P) {
  return P.b;
}

template <typename T>
hipError_t launch_apply_dots(const DevPencil& P, const PanelGrid& g, const SlotTables& st,
                             const void* Z, void* Qk, const void* Qbase, size_t vstride, int k,
                             double2* part, bool, hipStream_t s) {
  using C = typename CT<T>::t;
  const dim3 grid(g.blocks()), block(kThreads);
  auto Zc = static_cast<const C*>(Z);
  auto Qc = static_cast<C*>(Qk);
  auto Qb = static_cast<const C*>(Qbase);
  if (k == 0)
    k_apply_dots<T, false><<<grid, block, 0, s>>>(P.n, P.rowptr, P.col, vals_a<T>(P),
                                                  vals_b<T>(P), g, st.active, st.sigma, Zc, Qc,
                                                  Qb, vstride, k, part);
  else
    k_apply_dots<T, true><<<grid, block, 0, s>>>(P.n, P.rowptr, P.col, vals_a<T>(P),
                                                 vals_b<T>(P), g, st.active, st.sigma, Zc, Qc,
                                                 Qb, vstride, k, part);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_spmm_panel(const DevPencil& P, const PanelGrid& g, const double2* sigma_slot,
                             const void* Z, void* Q, hipStream_t s) {
  using C = typename CT<T>::t;
  k_apply_dots<T, false><<<g.blocks(), kThreads, 0, s>>>(
      P.n, P.rowptr, P.col, vals_a<T>(P), vals_b<T>(P), g, nullptr, sigma_slot,
      static_cast<const C*>(Z), static_cast<C*>(Q), nullptr, 0, 0, nullptr);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_orth(const DevPencil& P, const PanelGrid& g, const SlotTables& st, void* Qk,
                       void* Pk, const void* Z, const void* R, const void* Qbase,
                       const void* Pbase, size_t vstride, int k, const double2* beta,
                       double2* part, hipStream_t s) {
  using C = typename CT<T>::t;
  k_orth<T><<<g.blocks(), kThreads, 0, s>>>(P.n, g, st.active, static_cast<C*>(Qk),
                                            static_cast<C*>(Pk), static_cast<const C*>(Z),
                                            static_cast<const C*>(R),
                                            static_cast<const C*>(Qbase),
                                            static_cast<const C*>(Pbase), vstride, k, beta, part);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_step(const DevPencil& P, const PanelGrid& g, const SlotTables& st, void* R,
                       void* Z, const void* Qk, const double2* alpha_k, double2* part,
                       bool precond, hipStream_t s) {
  using C = typename CT<T>::t;
  k_step<T><<<g.blocks(), kThreads, 0, s>>>(P.n, g, st.active, st.sigma, P.da, P.db,
                                            precond ? 1 : 0, static_cast<C*>(R),
                                            static_cast<C*>(Z), static_cast<const C*>(Qk),
                                            alpha_k, part);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_yupdate(int n, const PanelGrid& g, const SlotTables& st, double2* Y,
                          const void* Pbase, size_t vstride, int kk, const double2* alpha,
                          hipStream_t s) {
  using C = typename CT<T>::t;
  k_yupdate<T><<<g.blocks(), kThreads, 0, s>>>(n, g, st.sys, Y, static_cast<const C*>(Pbase),
                                               vstride, kk, alpha);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_true_resid(const DevPencil& P, const PanelGrid& g, const SlotTables& st,
                             const double2* Y, const double* F, int ldf, void* R, void* Z,
                             double2* part, bool precond, hipStream_t s) {
  using C = typename CT<T>::t;
  k_true_resid<T><<<g.blocks(), kThreads, 0, s>>>(
      P.n, P.rowptr, P.col, P.a, P.b, P.da, P.db, precond ? 1 : 0, g, st.sys, st.col, st.sigma,
      Y, F, ldf, static_cast<C*>(R), static_cast<C*>(Z), part);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_admit(const DevPencil& P, const PanelGrid& g, const SlotTables& st,
                        const double2* Yold, const void* Rold, const void* Zold, double2* Ynew,
                        void* Rnew, void* Znew, const double* F, const double* E,
                        const double* X, int ld, bool warm, double2* part, bool precond,
                        hipStream_t s) {
  using C = typename CT<T>::t;
  k_admit<T><<<g.blocks(), kThreads, 0, s>>>(
      P.n, P.da, P.db, precond ? 1 : 0, g, st.sys, st.src, st.col, st.sigma, st.theta, Yold,
      static_cast<const C*>(Rold), static_cast<const C*>(Zold), Ynew, static_cast<C*>(Rnew),
      static_cast<C*>(Znew), F, E, X, ld, warm ? 1 : 0, part);
  return hipGetLastError();
}

hipError_t launch_retire(int n, const PanelGrid& g, const int* retire_sys, const double2* Y,
                           double2* Ystore, hipStream_t s) {
  k_retire<<<g.blocks(), kThreads, 0, s>>>(n, g, retire_sys, Y, Ystore);
  return hipGetLastError();
}

hipError_t launch_filter_sum(int n, int ncols, int npoles, const double2* Ystore,
                             const double2* w, double* Ur, hipStream_t s) {
  const size_t tot = (size_t)n * ncols;
  if (tot == 0) return hipSuccess;
  k_filter_sum<<<cdiv(tot, kThreads), kThreads, 0, s>>>(n, ncols, npoles, Ystore, w, Ur);
  return hipGetLastError();
}

hipError_t launch_reduce(const double2* part, int nrb, int ND, int C, int nd, int nslots,
                         double2* out, hipStream_t s) {
  const size_t tot = (size_t)nd * nslots;
  if (tot == 0) return hipSuccess;
  k_reduce<<<cdiv(tot, kThreads), kThreads, 0, s>>>(part, nrb, ND, C, nd, nslots, out);
  return hipGetLastError();
}

hipError_t launch_fin_beta(const double2* red, int k, int C, int nslots, const SlotTables& st,
                           const SlotScalars& sc, hipStream_t s) {
  k_fin_beta<<<cdiv(nslots, 256), 256, 0, s>>>(red, k, C, nslots, st.active, sc.qq, sc.beta);
  return hipGetLastError();
}
hipError_t launch_fin_alpha(const double2* red, int k, int C, int nslots, const SlotTables& st,
                            const SlotScalars& sc, hipStream_t s) {
  k_fin_alpha<<<cdiv(nslots, 256), 256, 0, s>>>(red, k, C, nslots, st.active, sc.qq, sc.alpha);
  return hipGetLastError();
}
hipError_t launch_fin_rnorm(const double2* red, int nslots, const SlotTables& st,
                            const SlotScalars& sc, int itcap, hipStream_t s) {
  k_fin_rnorm<<<cdiv(nslots, 256), 256, 0, s>>>(red, nslots, st.sys, st.active, sc.target2,
                                                sc.sys_its, sc.status, itcap);
  return hipGetLastError();
}
hipError_t launch_fin_true(const double2* red, int nslots, const SlotTables& st,
                           const SlotScalars& sc, double tol, double inner_rtol, double safety,
                           int itcap, hipStream_t s) {
  // from_admit is encoded by a non-null src table in st
  k_fin_true<<<cdiv(nslots, 256), 256, 0, s>>>(red, nslots, st.src != nullptr ? 1 : 0, st.sys,
                                               st.src, st.col, st.active, sc.target2, sc.fnorm2,
                                               sc.sys_its, sc.sys_rn2, sc.status, tol,
                                               inner_rtol, safety, itcap);
  return hipGetLastError();
}

#define SLRF_INST(T)                                                                         \
  template hipError_t launch_apply_dots<T>(const DevPencil&, const PanelGrid&,               \
                                           const SlotTables&, const void*, void*,            \
                                           const void*, size_t, int, double2*, bool,         \
                                           hipStream_t);                                     \
  template hipError_t launch_spmm_panel<T>(const DevPencil&, const PanelGrid&,               \
                                           const double2*, const void*, void*, hipStream_t); \
  template hipError_t launch_orth<T>(const DevPencil&, const PanelGrid&, const SlotTables&,  \
                                     void*, void*, const void*, const void*, const void*,    \
                                     const void*, size_t, int, const double2*, double2*,     \
                                     hipStream_t);                                           \
  template hipError_t launch_step<T>(const DevPencil&, const PanelGrid&, const SlotTables&,  \
                                     void*, void*, const void*, const double2*, double2*,    \
                                     bool, hipStream_t);                                     \
  template hipError_t launch_yupdate<T>(int, const PanelGrid&, const SlotTables&, double2*,  \
                                        const void*, size_t, int, const double2*,            \
                                        hipStream_t);                                        \
  template hipError_t launch_true_resid<T>(const DevPencil&, const PanelGrid&,               \
                                           const SlotTables&, const double2*, const double*, \
                                           int, void*, void*, double2*, bool, hipStream_t);  \
  template hipError_t launch_admit<T>(const DevPencil&, const PanelGrid&, const SlotTables&, \
                                      const double2*, const void*, const void*, double2*,    \
                                      void*, void*, const double*, const double*,            \
                                      const double*, int, bool, double2*, bool, hipStream_t);

SLRF_INST(float)
SLRF_INST(double)

}  // namespace slrf
