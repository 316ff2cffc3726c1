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
#include <type_traits>

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
// apply (LDS-staged CSR): the same operation as k_apply_dots for pencils whose
// row blocks fit in LDS.  A workgroup owns a block of rows and a group of G
// panels; for each sub-block of `sub` rows the CSR entries (col, a, b) are
// staged once in LDS and reused by all G panels, so the only global loads of
// the gather are the 16-byte lane vectors of z (two complex floats or one
// complex double per lane; one 128/256-byte segment per panel row).  The CGS
// projections of each pass are formed from an LDS tile of the fresh q, one
// thread per (slot pair, i) for complex float and per (slot, i, i + 16) for
// complex double.
// ---------------------------------------------------------------------------
template <typename T>
struct LaneVec;
template <>
struct LaneVec<float> {
  using V = float4;
  static constexpr int SPL = 2;  // slots per lane
};
template <>
struct LaneVec<double> {
  using V = double2;
  static constexpr int SPL = 1;
};

__device__ __forceinline__ bool map_tile(int nrb, int ncg, int group, int& rb, int& cg) {
  const long total = (long)nrb * ncg;
  const long per = (total + 7) / 8;
  const long b = blockIdx.x;
  const long t = (b & 7) * per + (b >> 3);
  if (t >= total) return false;
  const long G = group;
  const long pg = t / ((long)nrb * G);
  const long rem = t - pg * (long)nrb * G;
  const long gw = min(G, (long)ncg - pg * G);
  rb = (int)(rem / gw);
  cg = (int)(pg * G + rem % gw);
  return true;
}

__device__ __forceinline__ double lv_z(const float4& v) { return v.z; }
__device__ __forceinline__ double lv_w(const float4& v) { return v.w; }
__device__ __forceinline__ double lv_z(const double2&) { return 0.0; }
__device__ __forceinline__ double lv_w(const double2&) { return 0.0; }
__device__ __forceinline__ void lv_set_zw(float4& v, float z, float w) {
  v.z = z;
  v.w = w;
}
__device__ __forceinline__ void lv_set_zw(double2&, double, double) {}

template <typename T, int SPL>
__device__ __forceinline__ void lane_fma(T* acc, T a, T b, const typename LaneVec<T>::V& z) {
  if constexpr (SPL == 2) {
    acc[0] = mad(a, z.x, acc[0]);
    acc[1] = mad(a, z.y, acc[1]);
    acc[2] = mad(b, z.x, acc[2]);
    acc[3] = mad(b, z.y, acc[3]);
    acc[4] = mad(a, z.z, acc[4]);
    acc[5] = mad(a, z.w, acc[5]);
    acc[6] = mad(b, z.z, acc[6]);
    acc[7] = mad(b, z.w, acc[7]);
  } else {
    acc[0] = mad(a, z.x, acc[0]);
    acc[1] = mad(a, z.y, acc[1]);
    acc[2] = mad(b, z.x, acc[2]);
    acc[3] = mad(b, z.y, acc[3]);
  }
}

// Epilogues of the LDS-staged operator sweep (M = A - sigma B, x gathered):
//   kEpiApply : out = M x                      (GCR direction q, optional CGS dots)
//   kEpiResid : out = b - M x                  (AMG level residual)
//   kEpiJacobi: out = x + omega D^-1 (b - M x) (AMG damped-Jacobi sweep, D = diag M)
constexpr int kEpiApply = 0, kEpiResid = 1, kEpiJacobi = 2;
// kEpiResidH: the residual b - M x stored as complex bfloat16 (the level-0
// residual of the V-cycle, which only the restriction and the up-step read)
constexpr int kEpiResidH = 3;

// complex bfloat16 in one 32-bit word (re in the low half); rounding to the
// nearest even
__device__ __forceinline__ unsigned bf16_rne(float x) {
  const unsigned u = __float_as_uint(x);
  // a NaN stays a (quiet) NaN: the rounding carry could otherwise wrap its
  // payload into the sign bit
  if ((u & 0x7FFFFFFFu) > 0x7F800000u) return (u >> 16) | 0x0040u;
  return (u + 0x7FFFu + ((u >> 16) & 1u)) >> 16;
}
__device__ __forceinline__ unsigned pack_cbf16(float re, float im) {
  return bf16_rne(re) | (bf16_rne(im) << 16);
}
__device__ __forceinline__ float4 unpack_cbf16x2(uint2 h) {
  return make_float4(__uint_as_float(h.x << 16), __uint_as_float(h.x & 0xFFFF0000u),
                     __uint_as_float(h.y << 16), __uint_as_float(h.y & 0xFFFF0000u));
}

template <typename T, bool DOTS, int G, int EPI = kEpiApply, int UNR = 8>
__global__ __launch_bounds__(kThreads) void k_apply_lds(
    int n, const int* __restrict__ rowptr, const int* __restrict__ col, const T* __restrict__ av,
    const T* __restrict__ bv, PanelGrid g, int sub, int lds_nnz, const int* __restrict__ active,
    const double2* __restrict__ sigma, const typename CT<T>::t* __restrict__ Z,
    typename CT<T>::t* __restrict__ Qk, const typename CT<T>::t* __restrict__ Qb, size_t vstride,
    int k, double2* __restrict__ part, const typename CT<T>::t* __restrict__ Bin = nullptr,
    const double* __restrict__ da = nullptr, const double* __restrict__ db = nullptr,
    double omega = 0.0) {
  using V = typename LaneVec<T>::V;
  constexpr int SPL = LaneVec<T>::SPL;
  constexpr int LPR = kPanel / SPL;    // lanes per row
  constexpr int RPP = kThreads / LPR;  // rows per pass
  extern __shared__ __attribute__((aligned(16))) double smem_d[];  // 16-byte vectors live here
  T* s_a = reinterpret_cast<T*>(smem_d);
  T* s_b = s_a + lds_nnz;
  int* s_col = reinterpret_cast<int*>(s_b + lds_nnz);
  int* s_rp = s_col + lds_nnz;
  __shared__ V sq[RPP][LPR];
  __shared__ int s_act[G][kPanel];
  __shared__ int s_pany[G];
  const int ncg = (g.npan + G - 1) / G;
  int rb, cg;
  if (!map_tile(g.nrb, ncg, g.group, rb, cg)) return;
  const int tid = threadIdx.x;
  const int lr = tid % LPR, rr = tid / LPR;
  const int pan0 = cg * G;
  for (int t = tid; t < G * kPanel; t += kThreads) {
    const int gg = t / kPanel, p = pan0 + gg;
    s_act[gg][t % kPanel] =
        (p < g.npan) ? (active == nullptr ? 1 : (active[p * kPanel + t % kPanel] != 0)) : 0;
  }
  __syncthreads();
  if (tid < G) {
    int any = 0;
    for (int l = 0; l < kPanel; ++l) any |= s_act[tid][l];
    s_pany[tid] = any;
  }
  __syncthreads();
  double h[G][4];
#pragma unroll
  for (int gg = 0; gg < G; ++gg)
#pragma unroll
    for (int v = 0; v < 4; ++v) h[gg][v] = 0.0;
  // projection role of this thread: lane vector d_lane of a row, direction(s)
  const int d_lane = (SPL == 2) ? (tid & 7) : (tid & 15);
  const int d_i0 = (SPL == 2) ? (tid >> 3) : (tid >> 4);
  const int d_i1 = d_i0 + 16;
  const int R0 = rb * g.rpb, R1 = min(R0 + g.rpb, n);
  for (int s0 = R0; s0 < R1; s0 += sub) {
    const int s1 = min(s0 + sub, R1);
    const int eb = rowptr[s0];
    const int nsub = rowptr[s1] - eb;
    for (int t = tid; t <= s1 - s0; t += kThreads) s_rp[t] = rowptr[s0 + t] - eb;
    for (int t = tid; t < nsub; t += kThreads) {
      s_col[t] = col[eb + t];
      s_a[t] = av[eb + t];
      s_b[t] = bv[eb + t];
    }
    __syncthreads();
#pragma unroll
    for (int gg = 0; gg < G; ++gg) {
      if (!s_pany[gg]) continue;
      const int pan = pan0 + gg;
      const size_t pbase = (size_t)pan * n * kPanel;
      const V* __restrict__ Zp = reinterpret_cast<const V*>(Z + pbase);
      V* __restrict__ Qp = reinterpret_cast<V*>(Qk + pbase);
      T sr[SPL], si[SPL];
#pragma unroll
      for (int u = 0; u < SPL; ++u) {
        const double2 sgm = sigma[pan * kPanel + lr * SPL + u];
        sr[u] = (T)sgm.x;
        si[u] = (T)sgm.y;
      }
      for (int p0 = s0; p0 < s1; p0 += RPP) {
        const int row = p0 + rr;
        if (row < s1) {
          const int e0 = s_rp[row - s0], e1 = s_rp[row - s0 + 1];
          T acc[4 * SPL];
#pragma unroll
          for (int v = 0; v < 4 * SPL; ++v) acc[v] = 0;
          // batches of UNR gathers in flight; the last batch is predicated, so a
          // row costs ceil(nnz / UNR) memory round trips
          for (int e = e0; e < e1; e += UNR) {
            V z[UNR];
#pragma unroll
            for (int u = 0; u < UNR; ++u) {
              if (e + u < e1)
                z[u] = Zp[s_col[e + u] * LPR + lr];
              else
                z[u] = V{};
            }
#pragma unroll
            for (int u = 0; u < UNR; ++u) {
              const bool ok = e + u < e1;
              lane_fma<T, SPL>(acc, ok ? s_a[e + u] : T(0), ok ? s_b[e + u] : T(0), z[u]);
            }
          }
          V q;
          q.x = acc[0] - (sr[0] * acc[2] - si[0] * acc[3]);
          q.y = acc[1] - (sr[0] * acc[3] + si[0] * acc[2]);
          if constexpr (SPL == 2) {
            q.z = acc[4] - (sr[1] * acc[6] - si[1] * acc[7]);
            q.w = acc[5] - (sr[1] * acc[7] + si[1] * acc[6]);
          }
          if constexpr (EPI != kEpiApply) {
            const V bb = reinterpret_cast<const V*>(Bin + pbase)[row * LPR + lr];
            V rres;  // b - M x
            rres.x = bb.x - q.x;
            rres.y = bb.y - q.y;
            if constexpr (SPL == 2) {
              rres.z = bb.z - q.z;
              rres.w = bb.w - q.w;
            }
            if constexpr (EPI == kEpiResid) {
              q = rres;
            } else {
              const V xo = Zp[row * LPR + lr];
              const double dav = da[row], dbv = db[row];
#pragma unroll
              for (int u = 0; u < SPL; ++u) {
                const double dx = dav - (double)sr[u] * dbv, dy = -(double)si[u] * dbv;
                const double iv = omega / (dx * dx + dy * dy);
                const double ix = dx * iv, iy = -dy * iv;  // omega / (d)
                const double rx = u == 0 ? rres.x : lv_z(rres), ry = u == 0 ? rres.y : lv_w(rres);
                const double ox = u == 0 ? xo.x : lv_z(xo), oy = u == 0 ? xo.y : lv_w(xo);
                const T nx = (T)(ox + rx * ix - ry * iy), ny = (T)(oy + rx * iy + ry * ix);
                if (u == 0) {
                  q.x = nx;
                  q.y = ny;
                } else {
                  lv_set_zw(q, nx, ny);
                }
              }
            }
          }
          Qp[row * LPR + lr] = q;
          if constexpr (DOTS) sq[rr][lr] = q;
        }
        if constexpr (DOTS) {
          __syncthreads();
          const int nr = min(RPP, s1 - p0);
          if (d_i0 < k) {
            const V* __restrict__ Qi =
                reinterpret_cast<const V*>(Qb + (size_t)d_i0 * vstride + pbase);
#pragma unroll 4
            for (int r2 = 0; r2 < nr; ++r2) {
              const V v = Qi[(p0 + r2) * LPR + d_lane];
              const V qq = sq[r2][d_lane];
              h[gg][0] += (double)v.x * qq.x + (double)v.y * qq.y;
              h[gg][1] += (double)v.x * qq.y - (double)v.y * qq.x;
              if constexpr (SPL == 2) {
                h[gg][2] += (double)v.z * qq.z + (double)v.w * qq.w;
                h[gg][3] += (double)v.z * qq.w - (double)v.w * qq.z;
              }
            }
          }
          if constexpr (SPL == 1) {
            if (d_i1 < k) {
              const V* __restrict__ Qi =
                  reinterpret_cast<const V*>(Qb + (size_t)d_i1 * vstride + pbase);
#pragma unroll 4
              for (int r2 = 0; r2 < nr; ++r2) {
                const V v = Qi[(p0 + r2) * LPR + d_lane];
                const V qq = sq[r2][d_lane];
                h[gg][2] += (double)v.x * qq.x + (double)v.y * qq.y;
                h[gg][3] += (double)v.x * qq.y - (double)v.y * qq.x;
              }
            }
          }
          __syncthreads();
        }
      }
    }
    __syncthreads();
  }
  if constexpr (DOTS) {
#pragma unroll
    for (int gg = 0; gg < G; ++gg) {
      if (!s_pany[gg]) continue;
      const int slot0 = (pan0 + gg) * kPanel;
      if constexpr (SPL == 2) {
        if (d_i0 < k) {
          double2* dst = part + ((size_t)rb * g.ND + d_i0) * g.C + slot0 + 2 * d_lane;
          dst[0] = make_double2(h[gg][0], h[gg][1]);
          dst[1] = make_double2(h[gg][2], h[gg][3]);
        }
      } else {
        if (d_i0 < k)
          part[((size_t)rb * g.ND + d_i0) * g.C + slot0 + d_lane] =
              make_double2(h[gg][0], h[gg][1]);
        if (d_i1 < k)
          part[((size_t)rb * g.ND + d_i1) * g.C + slot0 + d_lane] =
              make_double2(h[gg][2], h[gg][3]);
      }
    }
  }
}

// ---------------------------------------------------------------------------
// apply (halo tiles): the operator sweep with the gathered operand read from
// LDS.  A workgroup owns one row tile and a run of G units (a unit is a
// 128-byte column slice of a panel: a whole complex-float panel or half a
// complex-double panel).  For each unit it copies the tile's halo rows of z
// (every row the tile's entries reference: one 128-byte line each) into LDS,
// the loads for the next unit in flight while the current one is formed;
// the tile is formed 32 rows per pass, each wave taking one 8-row slice,
// with the slice-ordered coefficients of the pass (local halo indices and
// (a, b) pairs) also staged in LDS by wide coalesced copies, the copy of the
// next pass in flight while the current one is formed (a tile of one pass
// stages its coefficients once for all its units).  Vector-memory
// traffic per row and unit is thus the tile's share of its halo plus the
// coefficients; the per-nonzero reads all come from LDS.  Entries of a row
// are summed in CSR order, as in the CSR kernels, so the result is bitwise
// that of the CSR sweeps.  Plain sweeps only (the GCR apply without
// projections and the AMG level operators).
// ---------------------------------------------------------------------------
struct HaloView {
  int ntile;
  int emax;
  const int* trow;
  const int* hptr;
  const int* halo;
  const int* sptr;
  const int* slen;
  const unsigned short* lcol;
  const void* ab;
};

// A subset of a halo layout's entries (the prolongator's within an image's
// pattern) in grouped slices of its own, on the same tiles and halo rows.
struct PSubView {
  int emax;
  const int* sptr;
  const unsigned short* lcol;
  const void* v;
};

// Local columns staged in LDS as byte offsets of the halo row: every staged
// halo row is 128 bytes (eight 16-byte lane vectors) and local indices stay
// below 512 (the tile halo caps), so shifting a packed pair of 16-bit indices
// left by 7 scales both halves at once.
// Local columns are staged in LDS as 32-bit byte offsets of the halo row
// (every staged halo row is 128 bytes: eight 16-byte lane vectors), so one
// 16-byte read yields a group's four operand addresses.  `v` holds eight
// 16-bit local columns; `out` receives their eight offsets.
__device__ __forceinline__ void halo_stage_cols(uint4 v, uint4* out) {
  out[0] = make_uint4((v.x & 0xffffu) << 7, (v.x >> 16) << 7, (v.y & 0xffffu) << 7,
                      (v.y >> 16) << 7);
  out[1] = make_uint4((v.z & 0xffffu) << 7, (v.z >> 16) << 7, (v.w & 0xffffu) << 7,
                      (v.w >> 16) << 7);
}
template <typename V>
__device__ __forceinline__ V halo_at(const V* base, unsigned byte_off) {
  return *reinterpret_cast<const V*>(reinterpret_cast<const char*>(base) + byte_off);
}

// The 4-entry groups of a wave's slice in order (wdt: the slice width, a
// multiple of 4, uniform across the wave): body(j, offsets) gets the group's
// four operand byte offsets.  Each group's offsets are read one group ahead,
// before the current group's operand reads, in two alternating registers.
template <typename F>
__device__ __forceinline__ void halo_slice_groups(const unsigned* plc, int wdt, F&& body) {
  if (wdt <= 0) return;
  uint4 ca = *reinterpret_cast<const uint4*>(plc);
  for (int j = 0;; j += 8) {
    // (the last group re-reads its own offsets; the empty asm keeps each read
    // where it is: otherwise it is sunk next to its use)
    const uint4 cb = *reinterpret_cast<const uint4*>(plc + min(j + 4, wdt - 4) * 8);
    asm volatile("" ::: "memory");
    body(j, ca);
    if (j + 4 >= wdt) break;
    ca = *reinterpret_cast<const uint4*>(plc + min(j + 8, wdt - 4) * 8);
    asm volatile("" ::: "memory");
    body(j + 4, cb);
    if (j + 8 >= wdt) break;
  }
}
__device__ __forceinline__ void halo_ab4(const float2* p, float2 (&ab)[4]) {
  const float4 u = reinterpret_cast<const float4*>(p)[0];
  const float4 v = reinterpret_cast<const float4*>(p)[1];
  ab[0] = make_float2(u.x, u.y);
  ab[1] = make_float2(u.z, u.w);
  ab[2] = make_float2(v.x, v.y);
  ab[3] = make_float2(v.z, v.w);
}
__device__ __forceinline__ void halo_ab4(const double2* p, double2 (&ab)[4]) {
#pragma unroll
  for (int i = 0; i < 4; ++i) ab[i] = p[i];
}
__device__ __forceinline__ void halo_val4(const float* p, float (&v)[4]) {
  const float4 u = *reinterpret_cast<const float4*>(p);
  v[0] = u.x;
  v[1] = u.y;
  v[2] = u.z;
  v[3] = u.w;
}
__device__ __forceinline__ void halo_val4(const double* p, double (&v)[4]) {
  const double2 u = reinterpret_cast<const double2*>(p)[0];
  const double2 w = reinterpret_cast<const double2*>(p)[1];
  v[0] = u.x;
  v[1] = u.y;
  v[2] = w.x;
  v[3] = w.y;
}

// (ZH: the gathered operand z is complex bfloat16, widened to complex float
// when staged; complex-float sweeps only)
template <typename T, int EPI, bool ZH = false>
__global__ __launch_bounds__(kThreads) void k_apply_halo(
    int n, HaloView hv, PanelGrid g, int G, const int* __restrict__ active,
    const double2* __restrict__ sigma, const typename CT<T>::t* __restrict__ Z,
    typename CT<T>::t* __restrict__ Qk, const typename CT<T>::t* __restrict__ Bin,
    const double* __restrict__ da, const double* __restrict__ db, double omega) {
  using V = typename LaneVec<T>::V;
  using AB = typename CT<T>::t;              // (a, b) coefficient pair
  constexpr int SPL = LaneVec<T>::SPL;       // systems per lane vector
  constexpr int UPP = SPL == 2 ? 1 : 2;      // units per panel
  constexpr int LPRF = kPanel / SPL;         // lane vectors per panel row
  constexpr int SPU = kPanel / UPP;          // systems per unit
  constexpr int UNR = 4;                     // = kHaloPad
  static_assert(kHaloTileRows == 8 * (kThreads / 64), "one 8-row slice per wave");
  extern __shared__ __attribute__((aligned(16))) double smem_d[];  // 16-byte vectors live here
  V* sZ = reinterpret_cast<V*>(smem_d);                            // [hmax][8]
  AB* s_ab = reinterpret_cast<AB*>(sZ + (size_t)g.rpb * 8);        // [emax]
  unsigned* s_lc = reinterpret_cast<unsigned*>(s_ab + hv.emax);  // [emax]
  int* sH = reinterpret_cast<int*>(s_lc + hv.emax);                          // [hmax]
  __shared__ int s_sp[kHaloTileRows / 8 + 1];  // slice offsets of the tile
  __shared__ int s_uact[kHaloMaxG];
  const int nunit = g.npan * UPP;
  const int nug = (nunit + G - 1) / G;
  int tile, ug;
  if (!map_tile(hv.ntile, nug, g.group, tile, ug)) return;
  const int tid = threadIdx.x, w = tid >> 6, rr = (tid >> 3) & 7, lr = tid & 7;
  const int r0 = hv.trow[tile], r1 = hv.trow[tile + 1];
  const int h0 = hv.hptr[tile], H = hv.hptr[tile + 1] - h0;
  // (the format's tiles hold at most kHaloTileRows rows: nsl <= 4)
  const int nsl = (r1 - r0 + 7) >> 3, sl0 = r0 >> 3;
  for (int t = tid; t < H; t += kThreads) sH[t] = hv.halo[h0 + t];
  if (tid <= nsl) s_sp[tid] = hv.sptr[sl0 + tid];
  // active units of the block (a unit with no iterating system is skipped)
  if (tid < G) {
    const int u = ug * G + tid;
    int any = 0;
    if (u < nunit) {
      const int b = (u / UPP) * kPanel + (u % UPP) * SPU;
      for (int l = 0; l < SPU; ++l) any |= (active == nullptr || active[b + l] != 0) ? 1 : 0;
    }
    s_uact[tid] = any;
  }
  __syncthreads();  // (also orders the tile tables in LDS before their first use)
  int gu = 0;
  while (gu < G && !s_uact[gu]) ++gu;
  if (gu >= G) return;
  // the halo of a unit is loaded into registers while the previous unit is
  // formed (the whole halo fits: H <= kHaloMaxH)
  // staged elements per halo row: eight 16-byte complex-float lane vectors, or
  // (complex bfloat16) four 16-byte vectors of four systems each
  constexpr int EPR = ZH ? 4 : 8;
  constexpr int HP = (kHaloMaxH * EPR + kThreads - 1) / kThreads;
  using HV = typename std::conditional<ZH, uint4, V>::type;  // staged element as loaded
  HV hreg[HP];
  // element offsets of this thread's share of the halo within a unit (the
  // same for every unit of the tile); past the halo a thread loads row 0 and
  // stores nothing (the loads stay unconditional, so they are issued here and
  // not where the values are consumed)
  unsigned hoff[HP];
#pragma unroll
  for (int i = 0; i < HP; ++i) {
    const int t = i * kThreads + tid;
    hoff[i] = (unsigned)((t < H * EPR ? sH[t / EPR] * (ZH ? 4 : LPRF) : 0) + (t % EPR));
  }
#define SLRF_HALO_ISSUE(GX)                                                              \
  do {                                                                                   \
    const int ux_ = ug * G + (GX);                                                       \
    const HV* __restrict__ zx_ =                                                         \
        ZH ? reinterpret_cast<const HV*>(Z) + (size_t)(ux_ / UPP) * n * 4                \
           : reinterpret_cast<const HV*>(Z + (size_t)(ux_ / UPP) * n * kPanel) + (ux_ % UPP) * 8; \
    _Pragma("unroll") for (int i_ = 0; i_ < HP; ++i_) {                                  \
      /* (through a local: a direct element copy leaves hreg in scratch) */              \
      const HV v_ = zx_[hoff[i_]];                                                       \
      hreg[i_] = v_;                                                                     \
    }                                                                                    \
  } while (0)
  SLRF_HALO_ISSUE(gu);
  // the tile's slice-ordered coefficients, staged once for all its units:
  // 16-byte chunks of the lcol segment and of the (a, b) segment (both start
  // on 16-byte boundaries: slices hold multiples of 8 entries)
  {
    const int e0 = s_sp[0] * 8, ne = (s_sp[nsl] - s_sp[0]) * 8;
    const int nlc = ne / 8, nab = ne * (int)sizeof(AB) / 16;
    const uint4* __restrict__ glc = reinterpret_cast<const uint4*>(hv.lcol) + e0 / 8;
    const uint4* __restrict__ gab =
        static_cast<const uint4*>(hv.ab) + (size_t)e0 * sizeof(AB) / 16;
    for (int t = tid; t < nlc; t += kThreads)
      halo_stage_cols(glc[t], reinterpret_cast<uint4*>(s_lc) + 2 * t);
    for (int t = tid; t < nab; t += kThreads) reinterpret_cast<uint4*>(s_ab)[t] = gab[t];
  }
  // this wave's slice
  const int row = r0 + w * 8 + rr;
  // (a wave's slice width is uniform across the wave: scalar loop control)
  const int wdt = __builtin_amdgcn_readfirstlane(w < nsl ? s_sp[w + 1] - s_sp[w] : 0);
  const int soff = w < nsl ? (s_sp[w] - s_sp[0]) * 8 + rr * 4 : 0;  // (groups of 4)
  while (gu < G) {
    const int u = ug * G + gu;
    const int pan = u / UPP, half = u % UPP;
    const int sys0 = pan * kPanel + half * SPU;
    const size_t pbase = (size_t)pan * n * kPanel;
    const V* __restrict__ Zu = reinterpret_cast<const V*>(Z + pbase) + half * 8;
    V* __restrict__ Qu = reinterpret_cast<V*>(Qk + pbase) + half * 8;
#pragma unroll
    for (int i = 0; i < HP; ++i) {
      const int t = i * kThreads + tid;
      if constexpr (ZH) {
        if constexpr (SPL == 2)
          if (t < H * 4) {
            const int hr = t >> 2, q = t & 3;
            sZ[hr * 8 + 2 * q] = unpack_cbf16x2(make_uint2(hreg[i].x, hreg[i].y));
            sZ[hr * 8 + 2 * q + 1] = unpack_cbf16x2(make_uint2(hreg[i].z, hreg[i].w));
          }
      } else {
        if (t < H * 8) sZ[t] = hreg[i];
      }
    }
    int gn = gu + 1;
    while (gn < G && !s_uact[gn]) ++gn;
    T sr[SPL], si[SPL];
#pragma unroll
    for (int q = 0; q < SPL; ++q) {
      const double2 sgm = sigma[sys0 + lr * SPL + q];
      sr[q] = (T)sgm.x;
      si[q] = (T)sgm.y;
    }
    __syncthreads();
    if (gn < G) SLRF_HALO_ISSUE(gn);
    if (w < nsl) {
      // slice widths are multiples of UNR; padding entries carry zero
      // coefficients and a valid local column, so no entry is predicated
      const AB* __restrict__ pab = s_ab + soff;
      const unsigned* __restrict__ plc = s_lc + soff;
      const V* __restrict__ pz = sZ + lr;
      T acc[4 * SPL];
#pragma unroll
      for (int v = 0; v < 4 * SPL; ++v) acc[v] = 0;
      // (a group's local columns are read one group ahead, so the operand
      // reads of a group wait on one LDS round trip, not two)
      halo_slice_groups(plc, wdt, [&](int j, const uint4& co) {
        V z[UNR];
        AB ab[UNR];
        halo_ab4(pab + j * 8, ab);
        z[0] = halo_at(pz, co.x);
        z[1] = halo_at(pz, co.y);
        z[2] = halo_at(pz, co.z);
        z[3] = halo_at(pz, co.w);
#pragma unroll
        for (int uu = 0; uu < UNR; ++uu) lane_fma<T, SPL>(acc, ab[uu].x, ab[uu].y, z[uu]);
      });
      if (row < r1) {
        V q;
        q.x = acc[0] - (sr[0] * acc[2] - si[0] * acc[3]);
        q.y = acc[1] - (sr[0] * acc[3] + si[0] * acc[2]);
        if constexpr (SPL == 2) {
          q.z = acc[4] - (sr[1] * acc[6] - si[1] * acc[7]);
          q.w = acc[5] - (sr[1] * acc[7] + si[1] * acc[6]);
        }
        if constexpr (EPI != kEpiApply) {
          const V bb = (reinterpret_cast<const V*>(Bin + pbase) + half * 8)[row * LPRF + lr];
          V rres;  // b - M x
          rres.x = bb.x - q.x;
          rres.y = bb.y - q.y;
          if constexpr (SPL == 2) {
            rres.z = bb.z - q.z;
            rres.w = bb.w - q.w;
          }
          if constexpr (EPI == kEpiResid || EPI == kEpiResidH) {
            q = rres;
          } else {
            const V xo = Zu[row * LPRF + lr];
            const double dav = da[row], dbv = db[row];
#pragma unroll
            for (int c = 0; c < SPL; ++c) {
              const double dx = dav - (double)sr[c] * dbv, dy = -(double)si[c] * dbv;
              const double iv = omega / (dx * dx + dy * dy);
              const double ix = dx * iv, iy = -dy * iv;  // omega / (d)
              const double rx = c == 0 ? rres.x : lv_z(rres), ry = c == 0 ? rres.y : lv_w(rres);
              const double ox = c == 0 ? xo.x : lv_z(xo), oy = c == 0 ? xo.y : lv_w(xo);
              const T nx = (T)(ox + rx * ix - ry * iy), ny = (T)(oy + rx * iy + ry * ix);
              if (c == 0) {
                q.x = nx;
                q.y = ny;
              } else {
                lv_set_zw(q, nx, ny);
              }
            }
          }
        }
        if constexpr (EPI == kEpiResidH) {
          if constexpr (SPL == 2)
            reinterpret_cast<uint2*>(Qk)[((size_t)pan * n + row) * 8 + lr] =
                make_uint2(pack_cbf16(q.x, q.y), pack_cbf16(lv_z(q), lv_w(q)));
        } else {
          Qu[row * LPRF + lr] = q;
        }
      }
    }
    __syncthreads();  // the unit's halo consumed: LDS is free for the next one
    gu = gn;
  }
}
#undef SLRF_HALO_ISSUE

// ---------------------------------------------------------------------------
// Fused level-0 up-step of the V-cycle on the image tiles of P: per fine row
// and system, acc_a = sum (A P)_rc e_c, acc_b = sum (B P)_rc e_c and
// acc_p = sum P_rc e_c over the row's image entries, then
//   out = x0 + acc_p + omega D^-1 (r1 - (acc_a - sigma acc_b)).
// The workgroup layout follows k_apply_halo: one 32-row tile, a run of G
// units, the tile's coefficients staged once, each unit's coarse halo rows of
// e copied into LDS (loaded into registers while the previous unit is formed).
// ---------------------------------------------------------------------------
// (HR1: r1 and x0 are complex bfloat16, complex-float sweeps only; HM: the
// largest coarse halo of a tile the staging registers cover)
template <typename T, bool HR1, int HM>
__global__ __launch_bounds__(kThreads) void k_post_image(
    int n, int nc, HaloView hv, PSubView pw, PanelGrid g, int G,
    const int* __restrict__ active, const double2* __restrict__ sigma,
    const typename CT<T>::t* __restrict__ E, const typename CT<T>::t* __restrict__ X0,
    const typename CT<T>::t* __restrict__ R1, typename CT<T>::t* __restrict__ Out,
    const double* __restrict__ da, const double* __restrict__ db, double omega) {
  using V = typename LaneVec<T>::V;
  using AB = typename CT<T>::t;
  constexpr int SPL = LaneVec<T>::SPL;
  constexpr int UPP = SPL == 2 ? 1 : 2;
  constexpr int LPRF = kPanel / SPL;
  constexpr int SPU = kPanel / UPP;
  constexpr int UNR = 4;  // = kHaloPad
  extern __shared__ __attribute__((aligned(16))) double smem_d[];  // 16-byte vectors live here
  V* sZ = reinterpret_cast<V*>(smem_d);                            // [hmax][8]
  AB* s_ab = reinterpret_cast<AB*>(sZ + (size_t)g.rpb * 8);        // [emax]
  T* s_p = reinterpret_cast<T*>(s_ab + hv.emax);                   // [pemax] P's values
  unsigned* s_lc = reinterpret_cast<unsigned*>(s_p + pw.emax);     // [emax]
  unsigned* s_plc = s_lc + hv.emax;                                // [pemax] P's offsets
  int* sH = reinterpret_cast<int*>(s_plc + pw.emax);              // [hmax]
  __shared__ int s_sp[kHaloTileRows / 8 + 1];
  __shared__ int s_psp[kHaloTileRows / 8 + 1];
  __shared__ int s_uact[kHaloMaxG];
  const int nunit = g.npan * UPP;
  const int nug = (nunit + G - 1) / G;
  int tile, ug;
  if (!map_tile(hv.ntile, nug, g.group, tile, ug)) return;
  const int tid = threadIdx.x, w = tid >> 6, rr = (tid >> 3) & 7, lr = tid & 7;
  const int r0 = hv.trow[tile], r1 = hv.trow[tile + 1];
  const int h0 = hv.hptr[tile], H = hv.hptr[tile + 1] - h0;
  const int nsl = (r1 - r0 + 7) >> 3, sl0 = r0 >> 3;  // (nsl <= 4: format invariant)
  for (int t = tid; t < H; t += kThreads) sH[t] = hv.halo[h0 + t];
  if (tid <= nsl) {
    s_sp[tid] = hv.sptr[sl0 + tid];
    s_psp[tid] = pw.sptr[sl0 + tid];
  }
  if (tid < G) {
    const int u = ug * G + tid;
    int any = 0;
    if (u < nunit) {
      const int b = (u / UPP) * kPanel + (u % UPP) * SPU;
      for (int l = 0; l < SPU; ++l) any |= (active == nullptr || active[b + l] != 0) ? 1 : 0;
    }
    s_uact[tid] = any;
  }
  __syncthreads();
  int gu = 0;
  while (gu < G && !s_uact[gu]) ++gu;
  if (gu >= G) return;
  constexpr int HP = (HM * 8 + kThreads - 1) / kThreads;
  V hreg[HP];
  // this thread's coarse-halo element offsets, the same for every unit (row 0
  // past the halo: the loads stay unconditional and are not stored)
  unsigned hoff[HP];
#pragma unroll
  for (int i = 0; i < HP; ++i) {
    const int t = i * kThreads + tid;
    hoff[i] = (unsigned)((t < H * 8 ? sH[t >> 3] * LPRF : 0) + (t & 7));
  }
#define SLRF_IMG_ISSUE(GX)                                                                  \
  do {                                                                                      \
    const int ux_ = ug * G + (GX);                                                          \
    const V* __restrict__ ex_ =                                                             \
        reinterpret_cast<const V*>(E + (size_t)(ux_ / UPP) * nc * kPanel) + (ux_ % UPP) * 8; \
    _Pragma("unroll") for (int i_ = 0; i_ < HP; ++i_) {                                     \
      const V v_ = ex_[hoff[i_]];                                                           \
      hreg[i_] = v_;                                                                        \
    }                                                                                       \
  } while (0)
  SLRF_IMG_ISSUE(gu);
  {
    // the images' coefficients (A P, B P) and, apart, P's own entries
    const int e0 = s_sp[0] * 8, ne = (s_sp[nsl] - s_sp[0]) * 8;
    const int nlc = ne / 8, nab = ne * (int)sizeof(AB) / 16;
    const uint4* __restrict__ glc = reinterpret_cast<const uint4*>(hv.lcol) + e0 / 8;
    const uint4* __restrict__ gab =
        static_cast<const uint4*>(hv.ab) + (size_t)e0 * sizeof(AB) / 16;
    for (int t = tid; t < nlc; t += kThreads)
      halo_stage_cols(glc[t], reinterpret_cast<uint4*>(s_lc) + 2 * t);
    for (int t = tid; t < nab; t += kThreads) reinterpret_cast<uint4*>(s_ab)[t] = gab[t];
    const int pe0 = s_psp[0] * 8, pne = (s_psp[nsl] - s_psp[0]) * 8;
    const int npl = pne / 8, npv = pne * (int)sizeof(T) / 16;
    const uint4* __restrict__ gplc = reinterpret_cast<const uint4*>(pw.lcol) + pe0 / 8;
    const uint4* __restrict__ gpv =
        static_cast<const uint4*>(pw.v) + (size_t)pe0 * sizeof(T) / 16;
    for (int t = tid; t < npl; t += kThreads)
      halo_stage_cols(gplc[t], reinterpret_cast<uint4*>(s_plc) + 2 * t);
    for (int t = tid; t < npv; t += kThreads) reinterpret_cast<uint4*>(s_p)[t] = gpv[t];
  }
  const int row = r0 + w * 8 + rr;
  // (a wave's slice width is uniform across the wave: scalar loop control)
  const int wdt = __builtin_amdgcn_readfirstlane(w < nsl ? s_sp[w + 1] - s_sp[w] : 0);
  const int soff = w < nsl ? (s_sp[w] - s_sp[0]) * 8 + rr * 4 : 0;  // (groups of 4)
  const int pwdt = __builtin_amdgcn_readfirstlane(w < nsl ? s_psp[w + 1] - s_psp[w] : 0);
  const int psoff = w < nsl ? (s_psp[w] - s_psp[0]) * 8 + rr * 4 : 0;
  while (gu < G) {
    const int u = ug * G + gu;
    const int pan = u / UPP, half = u % UPP;
    const int sys0 = pan * kPanel + half * SPU;
    const size_t pbase = (size_t)pan * n * kPanel;
#pragma unroll
    for (int i = 0; i < HP; ++i) {
      const int t = i * kThreads + tid;
      if (t < H * 8) sZ[t] = hreg[i];
    }
    int gn = gu + 1;
    while (gn < G && !s_uact[gn]) ++gn;
    T sr[SPL], si[SPL];
#pragma unroll
    for (int q = 0; q < SPL; ++q) {
      const double2 sgm = sigma[sys0 + lr * SPL + q];
      sr[q] = (T)sgm.x;
      si[q] = (T)sgm.y;
    }
    __syncthreads();
    if (gn < G) SLRF_IMG_ISSUE(gn);
    if (w < nsl) {
      const AB* __restrict__ pab = s_ab + soff;
      const unsigned* __restrict__ plc = s_lc + soff;
      const V* __restrict__ pz = sZ + lr;
      T acc[4 * SPL], accp[2 * SPL];
#pragma unroll
      for (int v = 0; v < 4 * SPL; ++v) acc[v] = 0;
#pragma unroll
      for (int v = 0; v < 2 * SPL; ++v) accp[v] = 0;
      halo_slice_groups(plc, wdt, [&](int j, const uint4& co) {
        V z[UNR];
        AB ab[UNR];
        halo_ab4(pab + j * 8, ab);
        z[0] = halo_at(pz, co.x);
        z[1] = halo_at(pz, co.y);
        z[2] = halo_at(pz, co.z);
        z[3] = halo_at(pz, co.w);
#pragma unroll
        for (int uu = 0; uu < UNR; ++uu) lane_fma<T, SPL>(acc, ab[uu].x, ab[uu].y, z[uu]);
      });
      // P's entries are a subset of the image's pattern, kept in slices of
      // their own so that the rows' zeros of P cost nothing
      const T* __restrict__ pp = s_p + psoff;
      halo_slice_groups(s_plc + psoff, pwdt, [&](int j, const uint4& co) {
        V z[UNR];
        T pw[UNR];
        halo_val4(pp + j * 8, pw);
        z[0] = halo_at(pz, co.x);
        z[1] = halo_at(pz, co.y);
        z[2] = halo_at(pz, co.z);
        z[3] = halo_at(pz, co.w);
#pragma unroll
        for (int uu = 0; uu < UNR; ++uu) {
          accp[0] = mad(pw[uu], (T)z[uu].x, accp[0]);
          accp[1] = mad(pw[uu], (T)z[uu].y, accp[1]);
          if constexpr (SPL == 2) {
            accp[2] = mad(pw[uu], (T)lv_z(z[uu]), accp[2]);
            accp[3] = mad(pw[uu], (T)lv_w(z[uu]), accp[3]);
          }
        }
      });
      if (row < r1) {
        const size_t off = (size_t)row * LPRF + lr;
        V xo, ro;
        if constexpr (HR1) {
          if constexpr (SPL == 2) {
            const size_t ho = ((size_t)pan * n + row) * 8 + lr;
            xo = unpack_cbf16x2(reinterpret_cast<const uint2*>(X0)[ho]);
            ro = unpack_cbf16x2(reinterpret_cast<const uint2*>(R1)[ho]);
          }
        } else {
          xo = (reinterpret_cast<const V*>(X0 + pbase) + half * 8)[off];
          ro = (reinterpret_cast<const V*>(R1 + pbase) + half * 8)[off];
        }
        // (the smoother scaling in the vector precision: the V-cycle is a
        // preconditioner, its arithmetic precision is the sweep's)
        const T dav = (T)da[row], dbv = (T)db[row], om = (T)omega;
        V q;
#pragma unroll
        for (int c = 0; c < SPL; ++c) {
          // M P e for system c, then s = r1 - M P e and x = x0 + P e
          const T mr = acc[4 * c + 0] - (sr[c] * acc[4 * c + 2] - si[c] * acc[4 * c + 3]);
          const T mi = acc[4 * c + 1] - (sr[c] * acc[4 * c + 3] + si[c] * acc[4 * c + 2]);
          const T rx = (c == 0 ? ro.x : (T)lv_z(ro)) - mr;
          const T ry = (c == 0 ? ro.y : (T)lv_w(ro)) - mi;
          const T ox = (c == 0 ? xo.x : (T)lv_z(xo)) + accp[2 * c];
          const T oy = (c == 0 ? xo.y : (T)lv_w(xo)) + accp[2 * c + 1];
          const T dx = dav - sr[c] * dbv, dy = -si[c] * dbv;
          const T iv = om / (dx * dx + dy * dy);
          const T ix = dx * iv, iy = -dy * iv;  // omega / (d)
          const T nx = ox + rx * ix - ry * iy, ny = oy + rx * iy + ry * ix;
          if (c == 0) {
            q.x = nx;
            q.y = ny;
          } else {
            lv_set_zw(q, nx, ny);
          }
        }
        (reinterpret_cast<V*>(Out + pbase) + half * 8)[off] = q;
      }
    }
    __syncthreads();  // the unit's halo consumed
    gu = gn;
  }
}
#undef SLRF_IMG_ISSUE

// ---------------------------------------------------------------------------
// FP64 true residual on the halo tiles: r = f - (A - sigma B) y for the
// complex-double solution y (staged per unit and tile in LDS as in
// k_apply_halo<double>), written as R in the inner precision and as Z
// (point Jacobi, copy, or nothing).  A row's entries are summed in CSR order
// with the same fused multiply-adds as k_true_resid (padding entries add
// exact zeros), so R and Z are bitwise those of the CSR kernel.  The norms
// are taken by k_rnorm over R.
// ---------------------------------------------------------------------------
template <typename TI>
__global__ __launch_bounds__(kThreads) void k_true_halo(
    int n, HaloView hv, PanelGrid g, int G, const int* __restrict__ sys,
    const int* __restrict__ scol, const double2* __restrict__ sigma,
    const double2* __restrict__ Y, const double* __restrict__ F, int ldf,
    typename CT<TI>::t* __restrict__ R, typename CT<TI>::t* __restrict__ Z,
    const double* __restrict__ da, const double* __restrict__ db, int pc) {
  using V = double2;
  using C = typename CT<TI>::t;
  constexpr int UPP = 2, LPRF = kPanel, SPU = kPanel / UPP, UNR = 4;
  extern __shared__ __attribute__((aligned(16))) double smem_d[];  // 16-byte vectors live here
  V* sZ = reinterpret_cast<V*>(smem_d);                            // [hmax][8]
  double2* s_ab = reinterpret_cast<double2*>(sZ + (size_t)g.rpb * 8);          // [emax]
  unsigned* s_lc = reinterpret_cast<unsigned*>(s_ab + hv.emax);  // [emax]
  int* sH = reinterpret_cast<int*>(s_lc + hv.emax);                          // [hmax]
  __shared__ int s_sp[kHaloTileRows / 8 + 1];
  __shared__ int s_uact[kHaloMaxG];
  const int nunit = g.npan * UPP;
  const int nug = (nunit + G - 1) / G;
  int tile, ug;
  if (!map_tile(hv.ntile, nug, g.group, tile, ug)) return;
  const int tid = threadIdx.x, w = tid >> 6, rr = (tid >> 3) & 7, lr = tid & 7;
  const int r0 = hv.trow[tile], r1 = hv.trow[tile + 1];
  const int h0 = hv.hptr[tile], H = hv.hptr[tile + 1] - h0;
  const int nsl = (r1 - r0 + 7) >> 3, sl0 = r0 >> 3;  // (nsl <= 4: format invariant)
  for (int t = tid; t < H; t += kThreads) sH[t] = hv.halo[h0 + t];
  if (tid <= nsl) s_sp[tid] = hv.sptr[sl0 + tid];
  if (tid < G) {
    const int u = ug * G + tid;
    int any = 0;
    if (u < nunit) {
      const int b = (u / UPP) * kPanel + (u % UPP) * SPU;
      for (int l = 0; l < SPU; ++l) any |= sys[b + l] >= 0 ? 1 : 0;
    }
    s_uact[tid] = any;
  }
  __syncthreads();
  int gu = 0;
  while (gu < G && !s_uact[gu]) ++gu;
  if (gu >= G) return;
  constexpr int HP = (kHaloMaxH * 8 + kThreads - 1) / kThreads;
  V hreg[HP];
  // this thread's halo element offsets, the same for every unit (row 0 past
  // the halo: the loads stay unconditional and are not stored)
  unsigned hoff[HP];
#pragma unroll
  for (int i = 0; i < HP; ++i) {
    const int t = i * kThreads + tid;
    hoff[i] = (unsigned)((t < H * 8 ? sH[t >> 3] * LPRF : 0) + (t & 7));
  }
#define SLRF_TRUE_ISSUE(GX)                                                              \
  do {                                                                                   \
    const int ux_ = ug * G + (GX);                                                       \
    const V* __restrict__ yx_ = Y + (size_t)(ux_ / UPP) * n * kPanel + (ux_ % UPP) * 8;  \
    _Pragma("unroll") for (int i_ = 0; i_ < HP; ++i_) {                                  \
      const V v_ = yx_[hoff[i_]];                                                        \
      hreg[i_] = v_;                                                                     \
    }                                                                                    \
  } while (0)
  SLRF_TRUE_ISSUE(gu);
  {
    const int e0 = s_sp[0] * 8, ne = (s_sp[nsl] - s_sp[0]) * 8;
    const uint4* __restrict__ glc = reinterpret_cast<const uint4*>(hv.lcol) + e0 / 8;
    const uint4* __restrict__ gab = static_cast<const uint4*>(hv.ab) + e0;
    for (int t = tid; t < ne / 8; t += kThreads)
      halo_stage_cols(glc[t], reinterpret_cast<uint4*>(s_lc) + 2 * t);
    for (int t = tid; t < ne; t += kThreads) reinterpret_cast<uint4*>(s_ab)[t] = gab[t];
  }
  const int row = r0 + w * 8 + rr;
  // (a wave's slice width is uniform across the wave: scalar loop control)
  const int wdt = __builtin_amdgcn_readfirstlane(w < nsl ? s_sp[w + 1] - s_sp[w] : 0);
  const int soff = w < nsl ? (s_sp[w] - s_sp[0]) * 8 + rr * 4 : 0;  // (groups of 4)
  while (gu < G) {
    const int u = ug * G + gu;
    const int pan = u / UPP, half = u % UPP;
    const int slot = pan * kPanel + half * SPU + lr;
#pragma unroll
    for (int i = 0; i < HP; ++i) {
      const int t = i * kThreads + tid;
      if (t < H * 8) sZ[t] = hreg[i];
    }
    int gn = gu + 1;
    while (gn < G && !s_uact[gn]) ++gn;
    const bool occ = sys[slot] >= 0;
    const double2 sg = occ ? sigma[slot] : make_double2(0.0, 0.0);
    const int cl = occ ? scol[slot] : 0;
    __syncthreads();
    if (gn < G) SLRF_TRUE_ISSUE(gn);
    if (w < nsl && occ) {
      const double2* __restrict__ pab = s_ab + soff;
      const unsigned* __restrict__ plc = s_lc + soff;
      const V* __restrict__ pz = sZ + lr;
      double ar = 0, ai = 0, br = 0, bi = 0;
      halo_slice_groups(plc, wdt, [&](int j, const uint4& co) {
        V z[UNR];
        double2 ab[UNR];
        halo_ab4(pab + j * 8, ab);
        z[0] = halo_at(pz, co.x);
        z[1] = halo_at(pz, co.y);
        z[2] = halo_at(pz, co.z);
        z[3] = halo_at(pz, co.w);
#pragma unroll
        for (int uu = 0; uu < UNR; ++uu) {
          ar = fma(ab[uu].x, z[uu].x, ar);
          ai = fma(ab[uu].x, z[uu].y, ai);
          br = fma(ab[uu].y, z[uu].x, br);
          bi = fma(ab[uu].y, z[uu].y, bi);
        }
      });
      if (row < r1) {
        const double mx = ar - (sg.x * br - sg.y * bi);
        const double my = ai - (sg.x * bi + sg.y * br);
        const double x = F[(size_t)row * ldf + cl] - mx, y = -my;
        const size_t off = ((size_t)pan * n + row) * kPanel + half * SPU + lr;
        R[off] = mk<C>(x, y);
        if (pc == 1) {
          const double2 d = jacobi_inv(da[row], db[row], sg);
          Z[off] = mk<C>(x * d.x - y * d.y, x * d.y + y * d.x);
        } else if (pc == 0) {
          Z[off] = mk<C>(x, y);
        }
      }
    }
    __syncthreads();  // the unit's halo consumed
    gu = gn;
  }
}
#undef SLRF_TRUE_ISSUE

// Y_A = A X and Y_B = B X (optionally E = Y_A - theta_c Y_B) for a row-major
// real FP64 block X (row stride ld, even; nc even) on the halo tiles of the
// complex-double sweep.  A pair of columns fills one 16-byte lane element the
// way one complex system does there, so a unit is 16 columns (8 lanes x 2):
// each workgroup takes one tile, stages its coefficients once and its halo
// rows of X per unit (loaded into registers while the previous unit is
// formed).  A row's entries are summed in CSR order, the padding adding
// zeros, so the results equal the CSR kernel's.
__global__ __launch_bounds__(kThreads) void k_spmm_real_halo(
    int n, HaloView hv, int hmax, int nunit, int G, const double* __restrict__ X, int ld,
    int nc, double* __restrict__ AX, double* __restrict__ BX,
    const double* __restrict__ theta, double* __restrict__ E) {
  using V = double2;
  constexpr int UNR = 4;  // = kHaloPad
  extern __shared__ __attribute__((aligned(16))) double smem_d[];
  V* sZ = reinterpret_cast<V*>(smem_d);                                  // [hmax][8]
  double2* s_ab = reinterpret_cast<double2*>(sZ + (size_t)hmax * 8);    // [emax]
  unsigned* s_lc = reinterpret_cast<unsigned*>(s_ab + hv.emax);         // [emax]
  int* sH = reinterpret_cast<int*>(s_lc + hv.emax);                     // [hmax]
  __shared__ int s_sp[kHaloTileRows / 8 + 1];
  const int nug = (nunit + G - 1) / G;
  int tile, ug;
  if (!map_tile(hv.ntile, nug, 1, tile, ug)) return;
  const int tid = threadIdx.x, w = tid >> 6, rr = (tid >> 3) & 7, lr = tid & 7;
  const int r0 = hv.trow[tile], r1 = hv.trow[tile + 1];
  const int h0 = hv.hptr[tile], H = hv.hptr[tile + 1] - h0;
  const int nsl = (r1 - r0 + 7) >> 3, sl0 = r0 >> 3;
  for (int t = tid; t < H; t += kThreads) sH[t] = hv.halo[h0 + t];
  if (tid <= nsl) s_sp[tid] = hv.sptr[sl0 + tid];
  __syncthreads();
  const int gend = min(G, nunit - ug * G);  // units of this group
  constexpr int HP = (kHaloMaxH * 8 + kThreads - 1) / kThreads;
  V hreg[HP];
  // this thread's halo elements: halo row t / 8, column pair t % 8 = lr of
  // the unit (past the halo: row 0, loaded and not stored)
  unsigned hoff[HP];
#pragma unroll
  for (int i = 0; i < HP; ++i) {
    const int t = i * kThreads + tid;
    hoff[i] = (unsigned)((t < H * 8 ? sH[t >> 3] * (ld >> 1) : 0) + (t & 7));
  }
  const V* __restrict__ Xv = reinterpret_cast<const V*>(X);
#define SLRF_RX_ISSUE(GX)                                                           \
  do {                                                                              \
    const int c0_ = (ug * G + (GX)) * 16;                                           \
    const V* __restrict__ xu_ = Xv + (c0_ >> 1);                                     \
    _Pragma("unroll") for (int i_ = 0; i_ < HP; ++i_) {                             \
      /* (every element of this thread is column pair lr; past nc: zero) */         \
      const V v_ = c0_ + 2 * lr < nc ? xu_[hoff[i_]] : make_double2(0.0, 0.0);       \
      hreg[i_] = v_;                                                                \
    }                                                                               \
  } while (0)
  SLRF_RX_ISSUE(0);
  {
    const int e0 = s_sp[0] * 8, ne = (s_sp[nsl] - s_sp[0]) * 8;
    const int nlc = ne / 8, nab = ne * (int)sizeof(double2) / 16;
    const uint4* __restrict__ glc = reinterpret_cast<const uint4*>(hv.lcol) + e0 / 8;
    const uint4* __restrict__ gab =
        static_cast<const uint4*>(hv.ab) + (size_t)e0 * sizeof(double2) / 16;
    for (int t = tid; t < nlc; t += kThreads)
      halo_stage_cols(glc[t], reinterpret_cast<uint4*>(s_lc) + 2 * t);
    for (int t = tid; t < nab; t += kThreads) reinterpret_cast<uint4*>(s_ab)[t] = gab[t];
  }
  const int row = r0 + w * 8 + rr;
  const int wdt = __builtin_amdgcn_readfirstlane(w < nsl ? s_sp[w + 1] - s_sp[w] : 0);
  const int soff = w < nsl ? (s_sp[w] - s_sp[0]) * 8 + rr * 4 : 0;
  for (int gu = 0; gu < gend; ++gu) {
#pragma unroll
    for (int i = 0; i < HP; ++i) {
      const int t = i * kThreads + tid;
      if (t < H * 8) sZ[t] = hreg[i];
    }
    __syncthreads();
    if (gu + 1 < gend) SLRF_RX_ISSUE(gu + 1);
    if (w < nsl) {
      const double2* __restrict__ pab = s_ab + soff;
      const unsigned* __restrict__ plc = s_lc + soff;
      const V* __restrict__ pz = sZ + lr;
      double acc[4] = {0.0, 0.0, 0.0, 0.0};
      halo_slice_groups(plc, wdt, [&](int j, const uint4& co) {
        V z[UNR];
        double2 ab[UNR];
        halo_ab4(pab + j * 8, ab);
        z[0] = halo_at(pz, co.x);
        z[1] = halo_at(pz, co.y);
        z[2] = halo_at(pz, co.z);
        z[3] = halo_at(pz, co.w);
#pragma unroll
        for (int uu = 0; uu < UNR; ++uu) lane_fma<double, 1>(acc, ab[uu].x, ab[uu].y, z[uu]);
      });
      const int c = (ug * G + gu) * 16 + 2 * lr;
      if (row < r1 && c < nc) {
        const size_t o = (size_t)row * ld + c;
        if (AX) {
          AX[o] = acc[0];
          AX[o + 1] = acc[1];
        }
        if (BX) {
          BX[o] = acc[2];
          BX[o + 1] = acc[3];
        }
        if (E) {
          E[o] = acc[0] - theta[c] * acc[2];
          E[o + 1] = acc[1] - theta[c + 1] * acc[3];
        }
      }
    }
    __syncthreads();  // the unit's halo consumed
  }
}
#undef SLRF_RX_ISSUE

// ||r||^2 per slot from the stored residual R, as partial sums per row block
// (rows r0 + 16 i of the block summed per thread, then the 16 row groups).
template <typename TI>
__global__ __launch_bounds__(kThreads) void k_rnorm(int n, PanelGrid g,
                                                    const int* __restrict__ sys,
                                                    const typename CT<TI>::t* __restrict__ R,
                                                    double2* __restrict__ part) {
  __shared__ double red[4 * 1 * 16];
  int rb, pan;
  if (!map_block(g, rb, pan)) return;
  const int lane = threadIdx.x & 15, rs = threadIdx.x >> 4;
  const bool occ = sys[pan * kPanel + lane] >= 0;
  if (!__syncthreads_or(occ)) return;
  double acc[1] = {0.0};
  const size_t base = (size_t)pan * n;
  const int r0 = rb * g.rpb, r1 = min(r0 + g.rpb, n);
  if (occ)
    for (int row = r0 + rs; row < r1; row += 16) {
      const auto v = R[(base + row) * kPanel + lane];
      const double x = v.x, y = v.y;
      acc[0] += x * x + y * y;
    }
  reduce16<1>(acc, 1, red, [&](int, int ln, double s) {
    part[((size_t)rb * g.ND) * g.C + pan * kPanel + ln] = make_double2(s, 0.0);
  });
}

// ---------------------------------------------------------------------------
// Row-group ("union") shifted SpMM.  Rows are taken in groups of R = 4
// consecutive rows; a group stores the union of its rows' columns once and,
// per union entry, the R coefficients of A and of B (zero where a row has no
// entry).  One 16-byte lane-vector gather of z then feeds all R rows of the
// group, so the number of gathers per row drops from nnz/row to the union
// size / R (about 2x fewer for 27-point stencils).  A workgroup stages the
// group data of 8 groups (32 rows) in LDS and its waves serve four panels at
// once (two per pass for complex double).
// ---------------------------------------------------------------------------
constexpr int kGrpR = 4;     // rows per group
constexpr int kGrpSub = 8;   // groups per staged sub-block (32 rows)

template <typename T, int EPI>
__global__ __launch_bounds__(kThreads) void k_spmm_grp(
    int n, const int* __restrict__ gptr, const int* __restrict__ gcol, const T* __restrict__ gca,
    const T* __restrict__ gcb, const double* __restrict__ da, const double* __restrict__ db,
    double omega, PanelGrid g, int lds_ent, const int* __restrict__ active,
    const double2* __restrict__ sigma, const typename CT<T>::t* __restrict__ Z,
    const typename CT<T>::t* __restrict__ Bin, typename CT<T>::t* __restrict__ Out) {
  using V = typename LaneVec<T>::V;
  constexpr int SPL = LaneVec<T>::SPL;
  constexpr int LPR = kPanel / SPL;                    // lanes per panel row
  constexpr int PPP = kThreads / (LPR * kGrpSub);      // panels per pass (4 or 2)
  constexpr int NPASS = 4 / PPP;                       // passes for 4 panels
  constexpr int R = kGrpR;
  extern __shared__ __attribute__((aligned(16))) double smem_d[];  // 16-byte vectors live here
  T* s_a = reinterpret_cast<T*>(smem_d);               // [lds_ent][R]
  T* s_b = s_a + (size_t)lds_ent * R;
  int* s_col = reinterpret_cast<int*>(s_b + (size_t)lds_ent * R);
  int* s_gp = s_col + lds_ent;                          // [kGrpSub + 1]
  __shared__ int s_any[4];
  const int ncg = (g.npan + 3) / 4;
  int rb, cg;
  if (!map_tile(g.nrb, ncg, g.group, rb, cg)) return;
  const int tid = threadIdx.x;
  const int lr = tid % LPR, gi = (tid / LPR) % kGrpSub, pw = tid / (LPR * kGrpSub);
  const int pan0 = cg * 4;
  if (tid < 4) {
    const int p = pan0 + tid;
    int any = 0;
    if (p < g.npan)
      for (int l = 0; l < kPanel; ++l) any |= active == nullptr ? 1 : (active[p * kPanel + l] != 0);
    s_any[tid] = any;
  }
  const int R0 = rb * g.rpb, R1 = min(R0 + g.rpb, n);
  const int ngrp_total = (n + R - 1) / R;
  for (int s0 = R0; s0 < R1; s0 += R * kGrpSub) {
    const int g0 = s0 / R;
    const int g1 = min(g0 + kGrpSub, ngrp_total);
    const int eb = gptr[g0];
    const int ne = gptr[g1] - eb;
    __syncthreads();  // previous sub-block done with LDS (and s_any visible)
    for (int t = tid; t <= g1 - g0; t += kThreads) s_gp[t] = gptr[g0 + t] - eb;
    for (int t = tid; t < ne; t += kThreads) s_col[t] = gcol[eb + t];
    for (int t = tid; t < ne * R; t += kThreads) {
      s_a[t] = gca[(size_t)eb * R + t];
      s_b[t] = gcb[(size_t)eb * R + t];
    }
    __syncthreads();
#pragma unroll
    for (int pass = 0; pass < NPASS; ++pass) {
      const int pl = pass * PPP + pw;  // panel of the group handled by this wave set
      const int pan = pan0 + pl;
      if (!s_any[pl] || g0 + gi >= g1) continue;
      const size_t pbase = (size_t)pan * n * kPanel;
      const V* __restrict__ Zp = reinterpret_cast<const V*>(Z + pbase);
      T acc[R][4 * SPL];
#pragma unroll
      for (int r = 0; r < R; ++r)
#pragma unroll
        for (int v = 0; v < 4 * SPL; ++v) acc[r][v] = 0;
      const int e0 = s_gp[gi], e1 = s_gp[gi + 1];
      int e = e0;
      for (; e + 3 < e1; e += 4) {
        V z[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) z[u] = Zp[s_col[e + u] * LPR + lr];
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
          for (int r = 0; r < R; ++r)
            lane_fma<T, SPL>(acc[r], s_a[(e + u) * R + r], s_b[(e + u) * R + r], z[u]);
      }
      for (; e < e1; ++e) {
        const V zz = Zp[s_col[e] * LPR + lr];
#pragma unroll
        for (int r = 0; r < R; ++r) lane_fma<T, SPL>(acc[r], s_a[e * R + r], s_b[e * R + r], zz);
      }
      T sr[SPL], si[SPL];
#pragma unroll
      for (int u = 0; u < SPL; ++u) {
        const double2 sgm = sigma[pan * kPanel + lr * SPL + u];
        sr[u] = (T)sgm.x;
        si[u] = (T)sgm.y;
      }
      V* __restrict__ Op = reinterpret_cast<V*>(Out + pbase);
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int row = (g0 + gi) * R + r;
        if (row >= n) break;
        V q;
        q.x = acc[r][0] - (sr[0] * acc[r][2] - si[0] * acc[r][3]);
        q.y = acc[r][1] - (sr[0] * acc[r][3] + si[0] * acc[r][2]);
        if constexpr (SPL == 2) {
          q.z = acc[r][4] - (sr[1] * acc[r][6] - si[1] * acc[r][7]);
          q.w = acc[r][5] - (sr[1] * acc[r][7] + si[1] * acc[r][6]);
        }
        if constexpr (EPI != kEpiApply) {
          const V bb = reinterpret_cast<const V*>(Bin + pbase)[row * LPR + lr];
          V rres;
          rres.x = bb.x - q.x;
          rres.y = bb.y - q.y;
          if constexpr (SPL == 2) {
            rres.z = bb.z - q.z;
            rres.w = bb.w - q.w;
          }
          if constexpr (EPI == kEpiResid) {
            q = rres;
          } else {
            const V xo = Zp[row * LPR + lr];
            const double dav = da[row], dbv = db[row];
#pragma unroll
            for (int u = 0; u < SPL; ++u) {
              const double dx = dav - (double)sr[u] * dbv, dy = -(double)si[u] * dbv;
              const double iv = omega / (dx * dx + dy * dy);
              const double ix = dx * iv, iy = -dy * iv;
              const double rx = u == 0 ? rres.x : lv_z(rres), ry = u == 0 ? rres.y : lv_w(rres);
              const double ox = u == 0 ? xo.x : lv_z(xo), oy = u == 0 ? xo.y : lv_w(xo);
              const T nx = (T)(ox + rx * ix - ry * iy), ny = (T)(oy + rx * iy + ry * ix);
              if (u == 0) {
                q.x = nx;
                q.y = ny;
              } else {
                lv_set_zw(q, nx, ny);
              }
            }
          }
        }
        Op[row * LPR + lr] = q;
      }
    }
  }
}

// CGS projections h_i = <q_i, q_k>, i < k, from the stored directions and the
// fresh q_k (a streaming pass over k + 1 vectors): thread (row subgroup, slot)
// keeps the k partial sums in registers, then the 16 row subgroups are combined
// in a fixed order (shuffles + LDS), one partial per (row block, i, slot).
template <typename T, int MAXK>
__global__ __launch_bounds__(kThreads) void k_dots(int n, PanelGrid g,
                                                   const int* __restrict__ active,
                                                   const typename CT<T>::t* __restrict__ Qk,
                                                   const typename CT<T>::t* __restrict__ Qb,
                                                   size_t vstride, int k,
                                                   double2* __restrict__ part) {
  using C = typename CT<T>::t;
  constexpr int NV = 2 * MAXK;
  __shared__ double red[4 * NV * 16];
  int rb, pan;
  if (!map_block(g, rb, pan)) return;
  const int lane = threadIdx.x & 15, rs = threadIdx.x >> 4;
  const int slot = pan * kPanel + lane;
  const bool act = active == nullptr || active[slot] != 0;
  if (!__syncthreads_or(act)) return;
  const size_t pbase = (size_t)pan * n * kPanel;
  double h[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) h[v] = 0.0;
  const int r0 = rb * g.rpb, r1 = min(r0 + g.rpb, n);
  if (act) {
    for (int row = r0 + rs; row < r1; row += 16) {
      const size_t off = pbase + (size_t)row * kPanel + lane;
      const C q = Qk[off];
      const double qx = q.x, qy = q.y;
#pragma unroll
      for (int i = 0; i < MAXK; ++i) {
        if (i < k) {
          const C v = Qb[(size_t)i * vstride + off];
          h[2 * i] += (double)v.x * qx + (double)v.y * qy;
          h[2 * i + 1] += (double)v.x * qy - (double)v.y * qx;
        }
      }
    }
  }
  reduce16<NV>(h, 2 * k, red, [&](int v, int ln, double sv) {
    double* dst = reinterpret_cast<double*>(part + ((size_t)rb * g.ND + (v >> 1)) * g.C +
                                            pan * kPanel + ln);
    dst[v & 1] = sv;
  });
}

// ---------------------------------------------------------------------------
// orth: q_k -= sum beta_i q_i ; p_k = z - sum beta_i p_i ; partial <q,q>, <q,r>
// ---------------------------------------------------------------------------

// ---------------------------------------------------------------------------
// step: r -= alpha q_k ; z = P^-1 r ; partial ||r||^2
// ---------------------------------------------------------------------------

// ---------------------------------------------------------------------------
// yupdate: y += sum_{i<kk} alpha_i p_i   (FP64 solution)
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(kThreads) void k_yupdate(
    int n, PanelGrid g, const int* __restrict__ sys, double2* __restrict__ Y,
    const typename CT<T>::t* __restrict__ Z0, const typename CT<T>::t* __restrict__ Zb,
    size_t vstride, int kk, const double2* __restrict__ alpha,
    const double2* __restrict__ bhist) {
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
  // coefficients of the z_j: sum_k alpha_k p_k with p_K = z_K - sum_{i<K}
  // beta_iK p_i; peeling p_K off from the top: g_K = a_K, a_i -= a_K beta_iK
  if (threadIdx.x < kPanel) {
    const int sl = pan * kPanel + threadIdx.x;
    for (int K = kk - 1; K > 0; --K) {
      const double2 aK = sa[K * kPanel + threadIdx.x];
      if (aK.x == 0.0 && aK.y == 0.0) continue;
      for (int i = 0; i < K; ++i) {
        const double2 b = bhist[((size_t)K * kMaxRestart + i) * g.C + sl];
        double2 ai = sa[i * kPanel + threadIdx.x];
        ai.x -= aK.x * b.x - aK.y * b.y;
        ai.y -= aK.x * b.y + aK.y * b.x;
        sa[i * kPanel + threadIdx.x] = ai;
      }
    }
  }
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
      // a slot that stopped within the cycle has zero coefficients for the
      // later steps and no z_i formed there (the buffer holds whatever it held
      // before): skip the term instead of multiplying it by zero
      if (a.x == 0.0 && a.y == 0.0) continue;
      const C p = i == 0 ? Z0[off] : Zb[(size_t)i * vstride + off];
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
      if (pc == 1) {
        const double2 d = jacobi_inv(da[row], db[row], sg);
        Z[off] = mk<C>(x * d.x - y * d.y, x * d.y + y * d.x);
      } else if (pc == 0) {
        Z[off] = mk<C>(x, y);
      }
      acc[0] += x * x + y * y;
    }
  }
  reduce16<1>(acc, 1, red, [&](int, int ln, double s) {
    part[((size_t)rb * g.ND) * g.C + pan * kPanel + ln] = make_double2(s, 0.0);
  });
}

// The same residual with the rows' CSR data staged in LDS once per workgroup
// and shared by G panels, UNR gathers of y in flight per lane.  Each thread
// visits the same rows in the same order and sums the entries of a row in CSR
// order, so the residual and the partial norms are bitwise those of
// k_true_resid.
template <typename T, int G, int UNR>
__global__ __launch_bounds__(kThreads) void k_true_resid_lds(
    int n, const int* __restrict__ rowptr, const int* __restrict__ col,
    const double* __restrict__ av, const double* __restrict__ bv, const double* __restrict__ da,
    const double* __restrict__ db, int pc, PanelGrid g, int sub, int lds_nnz,
    const int* __restrict__ sys, const int* __restrict__ scol, const double2* __restrict__ sigma,
    const double2* __restrict__ Y, const double* __restrict__ F, int ldf,
    typename CT<T>::t* __restrict__ R, typename CT<T>::t* __restrict__ Z,
    double2* __restrict__ part) {
  using C = typename CT<T>::t;
  extern __shared__ __attribute__((aligned(16))) double smem_d[];  // 16-byte vectors live here
  double* s_a = smem_d;
  double* s_b = s_a + lds_nnz;
  int* s_col = reinterpret_cast<int*>(s_b + lds_nnz);
  int* s_rp = s_col + lds_nnz;
  __shared__ double red[4 * G * 16];
  const int ncg = (g.npan + G - 1) / G;
  int rb, cg;
  if (!map_tile(g.nrb, ncg, g.group, rb, cg)) return;
  const int tid = threadIdx.x, lane = tid & 15, rs = tid >> 4;
  const int pan0 = cg * G;
  bool occ[G];
  double2 sg[G];
  int cl[G];
#pragma unroll
  for (int gg = 0; gg < G; ++gg) {
    const int p = pan0 + gg, slot = p * kPanel + lane;
    occ[gg] = p < g.npan && sys[slot] >= 0;
    sg[gg] = occ[gg] ? sigma[slot] : make_double2(0.0, 0.0);
    cl[gg] = occ[gg] ? scol[slot] : 0;
  }
  double acc[G];
#pragma unroll
  for (int gg = 0; gg < G; ++gg) acc[gg] = 0.0;
  const int R0 = rb * g.rpb, R1 = min(R0 + g.rpb, n);
  for (int s0 = R0; s0 < R1; s0 += sub) {
    const int s1 = min(s0 + sub, R1);
    const int eb = rowptr[s0];
    const int nsub = rowptr[s1] - eb;
    for (int t = tid; t <= s1 - s0; t += kThreads) s_rp[t] = rowptr[s0 + t] - eb;
    for (int t = tid; t < nsub; t += kThreads) {
      s_col[t] = col[eb + t];
      s_a[t] = av[eb + t];
      s_b[t] = bv[eb + t];
    }
    __syncthreads();
#pragma unroll
    for (int gg = 0; gg < G; ++gg) {
      if (!occ[gg]) continue;
      const size_t base = (size_t)(pan0 + gg) * n;
      for (int row = s0 + rs; row < s1; row += 16) {
        const int e0 = s_rp[row - s0], e1 = s_rp[row - s0 + 1];
        double ar = 0, ai = 0, br = 0, bi = 0;
        for (int e = e0; e < e1; e += UNR) {
          double2 y[UNR];
#pragma unroll
          for (int u = 0; u < UNR; ++u)
            y[u] = e + u < e1 ? Y[(base + s_col[e + u]) * kPanel + lane] : make_double2(0.0, 0.0);
#pragma unroll
          for (int u = 0; u < UNR; ++u) {
            if (e + u < e1) {
              const double a = s_a[e + u], b = s_b[e + u];
              ar = fma(a, y[u].x, ar);
              ai = fma(a, y[u].y, ai);
              br = fma(b, y[u].x, br);
              bi = fma(b, y[u].y, bi);
            }
          }
        }
        const double mx = ar - (sg[gg].x * br - sg[gg].y * bi);
        const double my = ai - (sg[gg].x * bi + sg[gg].y * br);
        const double x = F[(size_t)row * ldf + cl[gg]] - mx, y = -my;
        const size_t off = (base + row) * kPanel + lane;
        R[off] = mk<C>(x, y);
        if (pc == 1) {
          const double2 d = jacobi_inv(da[row], db[row], sg[gg]);
          Z[off] = mk<C>(x * d.x - y * d.y, x * d.y + y * d.x);
        } else if (pc == 0) {
          Z[off] = mk<C>(x, y);
        }
        acc[gg] += x * x + y * y;
      }
    }
    __syncthreads();
  }
  reduce16<G>(acc, G, red, [&](int v, int ln, double s) {
    if (pan0 + v < g.npan)
      part[((size_t)rb * g.ND) * g.C + (pan0 + v) * kPanel + ln] = make_double2(s, 0.0);
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
        if (pc == 1) {
          const double2 d = jacobi_inv(da[row], db[row], sg);
          Znew[off] = mk<C>(x * d.x - y * d.y, x * d.y + y * d.x);
        } else if (pc == 0) {
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

// The same sum when npoles divides 16 (a column's poles share a store panel):
// threads follow the store order (one 16-lane group per panel row), so the
// loads are contiguous, and the first lane of each column's npoles lanes adds
// their terms in increasing j (the order of k_filter_sum: identical results).
__global__ __launch_bounds__(kThreads) void k_filter_sum_p(int n, int ncols, int npoles,
                                                           long total,
                                                           const double2* __restrict__ Ys,
                                                           const double2* __restrict__ w,
                                                           double* __restrict__ Ur) {
  const long t = (long)blockIdx.x * kThreads + threadIdx.x;
  const int l = (int)(t & 15);
  const long pr = t >> 4;  // panel * n + row
  const int pan = (int)(pr / n), row = (int)(pr % n);
  const int s = pan * kPanel + l, c = s / npoles, j = s % npoles;
  double term = 0.0;
  if (t < total && c < ncols) {
    const double2 y = Ys[t];
    const double2 wj = w[j];
    term = 2.0 * (wj.x * y.x - wj.y * y.y);
  }
  const int lane = threadIdx.x & 63;
  double u = 0.0 + term;
  for (int jj = 1; jj < npoles; ++jj) {
    const double v = __shfl(term, (lane + jj) & 63);
    u += v;
  }
  if (t < total && c < ncols && j == 0) Ur[(size_t)row * ncols + c] = u;
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
                           double2* __restrict__ beta, double2* __restrict__ bhist) {
  const int slot = blockIdx.x * blockDim.x + threadIdx.x;
  if (slot >= nslots) return;
  const bool act = active[slot] != 0;
  for (int i = 0; i < k; ++i) {
    const double q = qq[(size_t)i * C + slot];
    const double2 h = red[(size_t)i * C + slot];
    const double2 b = (act && q > 0.0) ? make_double2(h.x / q, h.y / q) : make_double2(0.0, 0.0);
    beta[(size_t)i * C + slot] = b;
    bhist[((size_t)k * kMaxRestart + i) * C + slot] = b;
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
  if (red == nullptr) return;  // (last step of a cycle: counted only)
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

// ---------------------------------------------------------------------------
// AMG V-cycle kernels on level vectors in panel layout (rows = level size).
// ---------------------------------------------------------------------------
// Level operator sweep with a plain CSR gather (any row length):
//   EPI kEpiResid : out = b - (A_l - sigma B_l) x
//   EPI kEpiJacobi: out = x + omega D^-1 (b - (A_l - sigma B_l) x)
template <typename T, int EPI>
__global__ __launch_bounds__(kThreads) void k_lvl_simple(
    int n, const int* __restrict__ rowptr, const int* __restrict__ col, const T* __restrict__ av,
    const T* __restrict__ bv, const double* __restrict__ da, const double* __restrict__ db,
    double omega, PanelGrid g, const int* __restrict__ active, const double2* __restrict__ sigma,
    const typename CT<T>::t* __restrict__ X, const typename CT<T>::t* __restrict__ Bin,
    typename CT<T>::t* __restrict__ Out) {
  using C = typename CT<T>::t;
  int rb, pan;
  if (!map_block(g, rb, pan)) return;
  const int lane = threadIdx.x & 15, rs = threadIdx.x >> 4;
  const int slot = pan * kPanel + lane;
  if (active != nullptr && active[slot] == 0) return;
  const double2 sg = sigma[slot];
  const size_t pbase = (size_t)pan * n * kPanel;
  const C* __restrict__ Xp = X + pbase;
  const int r0 = rb * g.rpb, r1 = min(r0 + g.rpb, n);
  for (int row = r0 + rs; row < r1; row += 16) {
    T ar = 0, ai = 0, br = 0, bi = 0;
    for (int e = rowptr[row]; e < rowptr[row + 1]; ++e) {
      const C z = Xp[col[e] * kPanel + lane];
      const T a = av[e], b = bv[e];
      ar = mad(a, z.x, ar);
      ai = mad(a, z.y, ai);
      br = mad(b, z.x, br);
      bi = mad(b, z.y, bi);
    }
    const size_t off = pbase + (size_t)row * kPanel + lane;
    const C bb = Bin[off];
    const double rx = (double)bb.x - ((double)ar - (sg.x * br - sg.y * bi));
    const double ry = (double)bb.y - ((double)ai - (sg.x * bi + sg.y * br));
    if constexpr (EPI == kEpiResid) {
      Out[off] = mk<C>(rx, ry);
    } else {
      const double2 d = jacobi_inv(da[row], db[row], sg);
      const C xo = Xp[row * kPanel + lane];
      Out[off] = mk<C>(xo.x + omega * (rx * d.x - ry * d.y), xo.y + omega * (rx * d.y + ry * d.x));
    }
  }
}

// first smoothing step from a zero guess: out = omega D^-1 b (OH: out as
// complex bfloat16, complex-float sweeps only)
template <typename T, bool OH = false>
__global__ __launch_bounds__(kThreads) void k_lvl_jacobi0(
    int n, const double* __restrict__ da, const double* __restrict__ db, double omega, PanelGrid g,
    const int* __restrict__ active, const double2* __restrict__ sigma,
    const typename CT<T>::t* __restrict__ Bin, typename CT<T>::t* __restrict__ Out) {
  using C = typename CT<T>::t;
  int rb, pan;
  if (!map_block(g, rb, pan)) return;
  const int lane = threadIdx.x & 15, rs = threadIdx.x >> 4;
  const int slot = pan * kPanel + lane;
  if (active != nullptr && active[slot] == 0) return;
  const double2 sg = sigma[slot];
  const size_t pbase = (size_t)pan * n * kPanel;
  const int r0 = rb * g.rpb, r1 = min(r0 + g.rpb, n);
  for (int row = r0 + rs; row < r1; row += 16) {
    const size_t off = pbase + (size_t)row * kPanel + lane;
    const C bb = Bin[off];
    const double2 d = jacobi_inv(da[row], db[row], sg);
    if constexpr (OH)
      reinterpret_cast<unsigned*>(Out)[off] = pack_cbf16(
          (float)(omega * (bb.x * d.x - bb.y * d.y)), (float)(omega * (bb.x * d.y + bb.y * d.x)));
    else
      Out[off] = mk<C>(omega * (bb.x * d.x - bb.y * d.y), omega * (bb.x * d.y + bb.y * d.x));
  }
}

// The active slots grouped by pole (a group's order is arbitrary: every slot's
// coarse solution is formed on its own): poff[j] .. poff[j + 1] in plist.
__global__ __launch_bounds__(kThreads) void k_pole_lists(int nslot, int npoles,
                                                         const int* __restrict__ active,
                                                         const int* __restrict__ sys,
                                                         int* __restrict__ plist,
                                                         int* __restrict__ poff) {
  __shared__ int cnt[kMaxPoles], cur[kMaxPoles];
  const int tid = threadIdx.x;
  for (int j = tid; j < npoles; j += kThreads) cnt[j] = 0;
  __syncthreads();
  for (int s = tid; s < nslot; s += kThreads) {
    const int sy = sys[s];
    if (sy >= 0 && (active == nullptr || active[s] != 0)) atomicAdd(&cnt[sy % npoles], 1);
  }
  __syncthreads();
  if (tid == 0) {
    int acc = 0;
    for (int j = 0; j < npoles; ++j) {
      cur[j] = acc;
      poff[j] = acc;
      acc += cnt[j];
    }
    poff[npoles] = acc;
  }
  __syncthreads();
  for (int s = tid; s < nslot; s += kThreads) {
    const int sy = sys[s];
    if (sy >= 0 && (active == nullptr || active[s] != 0))
      plist[atomicAdd(&cur[sy % npoles], 1)] = s;
  }
}

// Coarsest level as one product per pole: X_j = (A_c - sigma_j B_c)^{-1} B_j
// over the slots of pole j.  A workgroup forms 32 rows by 32 slots of one
// pole (2 rows x 2 slots per thread), the inverse's rows and the gathered
// right-hand sides staged through LDS in chunks of 32 columns, FP64
// accumulation in column order.  Workgroup b takes pole b mod npoles: with 8
// poles each XCD reads one pole's inverse.
constexpr int kCgRows = 32, kCgSlots = 32, kCgK = 32, kCgRT = kCgRows / 16;
template <typename T>
__global__ __launch_bounds__(kThreads) void k_coarse_gemm(
    int nc, int npoles, int nrt, const int* __restrict__ plist, const int* __restrict__ poff,
    const typename CT<T>::t* __restrict__ Minv, const typename CT<T>::t* __restrict__ Bin,
    typename CT<T>::t* __restrict__ Out) {
  using C = typename CT<T>::t;
  const int p = (int)(blockIdx.x % (unsigned)npoles);
  const int rest = (int)(blockIdx.x / (unsigned)npoles);
  const int rt = rest % nrt, stile = rest / nrt;
  const int s0 = poff[p] + stile * kCgSlots, s1 = poff[p + 1];
  if (s0 >= s1) return;
  __shared__ double2 Ms[kCgRows][kCgK + 1];
  __shared__ double2 Bs[kCgK][kCgSlots];
  __shared__ int sl[kCgSlots];
  const int tid = threadIdx.x;
  if (tid < kCgSlots) sl[tid] = s0 + tid < s1 ? plist[s0 + tid] : -1;
  const int tx = tid & 15, ty = tid >> 4;
  const int r0 = rt * kCgRows;
  const C* __restrict__ Mp = Minv + (size_t)p * nc * nc;
  double2 acc[kCgRT][2];
#pragma unroll
  for (int i = 0; i < kCgRT; ++i) acc[i][0] = acc[i][1] = make_double2(0.0, 0.0);
  __syncthreads();
  for (int k0 = 0; k0 < nc; k0 += kCgK) {
    for (int e = tid; e < kCgRows * kCgK; e += kThreads) {
      const int r = e / kCgK, k = e % kCgK, gr = r0 + r, gk = k0 + k;
      double2 v = make_double2(0.0, 0.0);
      if (gr < nc && gk < nc) {
        const C m = Mp[(size_t)gr * nc + gk];
        v = make_double2(m.x, m.y);
      }
      Ms[r][k] = v;
    }
    for (int e = tid; e < kCgK * kCgSlots; e += kThreads) {
      const int k = e / kCgSlots, j = e % kCgSlots, sj = sl[j], gk = k0 + k;
      double2 v = make_double2(0.0, 0.0);
      if (sj >= 0 && gk < nc) {
        const C b = Bin[((size_t)(sj / kPanel) * nc + gk) * kPanel + sj % kPanel];
        v = make_double2(b.x, b.y);
      }
      Bs[k][j] = v;
    }
    __syncthreads();
#pragma unroll 4
    for (int k = 0; k < kCgK; ++k) {
      const double2 b0 = Bs[k][2 * tx], b1 = Bs[k][2 * tx + 1];
#pragma unroll
      for (int i = 0; i < kCgRT; ++i) {
        const double2 m = Ms[kCgRT * ty + i][k];
        acc[i][0].x += m.x * b0.x - m.y * b0.y;
        acc[i][0].y += m.x * b0.y + m.y * b0.x;
        acc[i][1].x += m.x * b1.x - m.y * b1.y;
        acc[i][1].y += m.x * b1.y + m.y * b1.x;
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < kCgRT; ++i) {
    const int row = r0 + kCgRT * ty + i;
    if (row >= nc) continue;
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int sj = sl[2 * tx + j];
      if (sj >= 0)
        Out[((size_t)(sj / kPanel) * nc + row) * kPanel + sj % kPanel] =
            mk<C>(acc[i][j].x, acc[i][j].y);
    }
  }
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

constexpr int kGroupPanels = 4;  // panels per workgroup in the LDS-staged SpMM

template <typename T>
static size_t lds_bytes(int sub, int nnz) {
  return (size_t)nnz * (2 * sizeof(T) + sizeof(int)) + (size_t)(sub + 1) * sizeof(int);
}

// gathers in flight per lane in the CSR-LDS kernels, from the variant code
template <typename T>
static int lds_unroll(const DevPencil& P) {
  const int var = std::is_same<T, float>::value ? P.var32 : P.var64;
  return (var == kSpmmCsrLds16 || var == kSpmmHalo) ? 16 : (var == kSpmmCsrLds32 ? 32 : 8);
}

// Staging plan: rows per sub-block (64 or 32) whose largest CSR slice fits in
// 48 KB of LDS; false when neither does (then the gather reads the CSR from
// global memory).
template <typename T>
static bool lds_fit(const DevPencil& P, int rpb, int& sub, int& cap, size_t& bytes) {
  const int cands[2] = {64, 32};
  const int caps[2] = {P.max_nnz_sub64, P.max_nnz_sub32};
  for (int i = 0; i < 2; ++i) {
    if (caps[i] <= 0 || rpb % cands[i] != 0) continue;
    const size_t b = lds_bytes<T>(cands[i], caps[i]);
    if (b <= 48 * 1024) {
      sub = cands[i];
      cap = caps[i];
      bytes = b;
      return true;
    }
  }
  return false;
}

// rows staged in LDS for the CSR-LDS sweeps, unless the variant is another one
template <typename T>
static bool lds_plan(const DevPencil& P, int rpb, int& sub, int& cap, size_t& bytes) {
  const int var = std::is_same<T, float>::value ? P.var32 : P.var64;
  if (var == kSpmmCsrDirect || var == kSpmmGroup) return false;
  return lds_fit<T>(P, rpb, sub, cap, bytes);
}

template <typename T>
static size_t grp_lds_bytes(int ent) {
  return (size_t)ent * (2 * kGrpR * sizeof(T) + sizeof(int)) + (kGrpSub + 1) * sizeof(int);
}

template <typename T>
static const T* grp_a(const DevPencil& P);
template <>
const float* grp_a<float>(const DevPencil& P) {
  return P.gca32;
}
template <>
const double* grp_a<double>(const DevPencil& P) {
  return P.gca;
}
template <typename T>
static const T* grp_b(const DevPencil& P);
template <>
const float* grp_b<float>(const DevPencil& P) {
  return P.gcb32;
}
template <>
const double* grp_b<double>(const DevPencil& P) {
  return P.gcb;
}

// Row-group SpMM with epilogue; false when the pencil has no row-group format
// (or it does not fit in LDS) so the caller falls back to the CSR kernels.
template <typename T>
static bool launch_grp(const DevPencil& P, const PanelGrid& g, const SlotTables& st, int epi,
                       double omega, const void* Z, const void* Bin, void* Out, hipStream_t s,
                       hipError_t& err) {
  using C = typename CT<T>::t;
  const int var = std::is_same<T, float>::value ? P.var32 : P.var64;
  if (var != kSpmmAuto && var != kSpmmGroup) return false;
  if (P.gptr == nullptr || g.rpb % (kGrpR * kGrpSub) != 0) return false;
  const size_t bytes = grp_lds_bytes<T>(P.grp_lds_ent);
  if (bytes > 48 * 1024) return false;
  PanelGrid gg = g;
  const int ncg = (g.npan + 3) / 4;
  gg.group = ncg < 4 ? ncg : 4;
  const long total = (long)g.nrb * ncg;
  const unsigned blocks = (unsigned)(((total + 7) / 8) * 8);
  auto Zc = static_cast<const C*>(Z);
  auto Bc = static_cast<const C*>(Bin);
  auto Oc = static_cast<C*>(Out);
  if (epi == kEpiApply)
    k_spmm_grp<T, kEpiApply><<<blocks, kThreads, bytes, s>>>(
        P.n, P.gptr, P.gcol, grp_a<T>(P), grp_b<T>(P), P.da, P.db, omega, gg, P.grp_lds_ent,
        st.active, st.sigma, Zc, Bc, Oc);
  else if (epi == kEpiResid)
    k_spmm_grp<T, kEpiResid><<<blocks, kThreads, bytes, s>>>(
        P.n, P.gptr, P.gcol, grp_a<T>(P), grp_b<T>(P), P.da, P.db, omega, gg, P.grp_lds_ent,
        st.active, st.sigma, Zc, Bc, Oc);
  else
    k_spmm_grp<T, kEpiJacobi><<<blocks, kThreads, bytes, s>>>(
        P.n, P.gptr, P.gcol, grp_a<T>(P), grp_b<T>(P), P.da, P.db, omega, gg, P.grp_lds_ent,
        st.active, st.sigma, Zc, Bc, Oc);
  err = hipGetLastError();
  return true;
}


// ---------------------------------------------------------------------------
// Streaming GCR kernels with 16-byte lane vectors (LaneVec: two complex floats
// or one complex double per lane; LPR lanes per panel row, 256 / LPR rows per
// pass).  Per-slot partial sums are combined over the row subgroups by a fixed
// xor-shuffle tree inside each wave and a fixed-order sum over the 4 waves.
// ---------------------------------------------------------------------------
template <int NVS, int LPR, typename Emit>
__device__ __forceinline__ void reduce_lv(double* vals, int nvs, double* red, Emit emit) {
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
#pragma unroll
  for (int v = 0; v < NVS; ++v) {
    if (v < nvs) {
      double x = vals[v];
#pragma unroll
      for (int off = LPR; off < 64; off <<= 1) x += __shfl_xor(x, off);
      if (l < LPR) red[(w * NVS + v) * LPR + l] = x;
    }
  }
  __syncthreads();
  for (int t = threadIdx.x; t < nvs * LPR; t += kThreads) {
    const int v = t / LPR, lr = t % LPR;
    const double sum = ((red[(0 * NVS + v) * LPR + lr] + red[(1 * NVS + v) * LPR + lr]) +
                        red[(2 * NVS + v) * LPR + lr]) +
                       red[(3 * NVS + v) * LPR + lr];
    emit(v, lr, sum);
  }
}

// complex components of a lane vector: slot c (< SPL) -> (re, im)
template <typename T>
__device__ __forceinline__ void lv_get(const typename LaneVec<T>::V& v, int c, double& re,
                                       double& im) {
  if (c == 0) {
    re = v.x;
    im = v.y;
  } else {
    re = lv_z(v);
    im = lv_w(v);
  }
}

// h_i = <q_i, q_k>, i < k <= MAXK, partial sums per (row block, slot).
// HQ: the stored q_i are complex bfloat16 (one 8-byte pair of systems per
// lane at ((panel * n + row) * 8 + lane) of slot i; complex-float only).
template <typename T, int MAXK, bool HQ = false>
__global__ __launch_bounds__(kThreads) void k_dots_lv(int n, PanelGrid g,
                                                      const int* __restrict__ active,
                                                      const typename CT<T>::t* __restrict__ Qk,
                                                      const typename CT<T>::t* __restrict__ Qb,
                                                      size_t vstride, int k,
                                                      double2* __restrict__ part) {
  using V = typename LaneVec<T>::V;
  constexpr int SPL = LaneVec<T>::SPL;
  constexpr int LPR = kPanel / SPL;
  constexpr int RPP = kThreads / LPR;
  constexpr int NVS = 2 * MAXK * SPL;
  __shared__ double red[4 * NVS * LPR];
  int rb, pan;
  if (!map_block(g, rb, pan)) return;
  const int tid = threadIdx.x, lr = tid % LPR, rs = tid / LPR;
  const bool a = tid < kPanel && (active == nullptr || active[pan * kPanel + tid] != 0);
  if (!__syncthreads_or(a)) return;
  const size_t pbase = (size_t)pan * n * kPanel;
  const V* __restrict__ Qp = reinterpret_cast<const V*>(Qk + pbase);
  double h[NVS];
#pragma unroll
  for (int v = 0; v < NVS; ++v) h[v] = 0.0;
  const int r0 = rb * g.rpb, r1 = min(r0 + g.rpb, n);
  for (int row = r0 + rs; row < r1; row += RPP) {
    const size_t off = (size_t)row * LPR + lr;
    const V q = Qp[off];
#pragma unroll
    for (int i = 0; i < MAXK; ++i) {
      if (i < k) {
        V vq;
        if constexpr (HQ && SPL == 2)
          vq = unpack_cbf16x2(reinterpret_cast<const uint2*>(Qb + (size_t)i * vstride)
                                  [((size_t)pan * n + row) * 8 + lr]);
        else
          vq = reinterpret_cast<const V*>(Qb + (size_t)i * vstride + pbase)[off];
#pragma unroll
        for (int c = 0; c < SPL; ++c) {
          double qx, qy, vx, vy;
          lv_get<T>(q, c, qx, qy);
          lv_get<T>(vq, c, vx, vy);
          h[(2 * i) * SPL + c] += vx * qx + vy * qy;
          h[(2 * i + 1) * SPL + c] += vx * qy - vy * qx;
        }
      }
    }
  }
  reduce_lv<NVS, LPR>(h, 2 * k * SPL, red, [&](int v, int ln, double sum) {
    // v = (2 i + re/im) * SPL + c; slot = ln * SPL + c
    const int c = v % SPL, vi = v / SPL;
    double* dst = reinterpret_cast<double*>(part + ((size_t)rb * g.ND + (vi >> 1)) * g.C +
                                            pan * kPanel + ln * SPL + c);
    dst[vi & 1] = sum;
  });
}

// q_k = w - sum_i beta_i q_i from the image w in Qk; partial <q_k, q_k>,
// <q_k, r>.  q_k is written to Qout when store is set (Qout may alias Qk).
// HQ: the stored q_i and q_k are complex bfloat16 (layout as in k_dots_lv),
// and the partial sums are taken from the rounded q_k, so that every later
// use of q_k sees the same vector.
template <typename T, bool HQ = false>
__global__ __launch_bounds__(kThreads) void k_orth_lv(
    int n, PanelGrid g, const int* __restrict__ active, const typename CT<T>::t* Qk,
    const typename CT<T>::t* __restrict__ R, const typename CT<T>::t* __restrict__ Qb,
    size_t vstride, int k, const double2* __restrict__ beta, double2* __restrict__ part,
    typename CT<T>::t* Qout, int store) {
  using V = typename LaneVec<T>::V;
  constexpr int SPL = LaneVec<T>::SPL;
  constexpr int LPR = kPanel / SPL;
  constexpr int RPP = kThreads / LPR;
  constexpr int NVS = 3 * SPL;
  __shared__ double2 sb[kMaxRestart * kPanel];
  __shared__ double red[4 * NVS * LPR];
  int rb, pan;
  if (!map_block(g, rb, pan)) return;
  const int tid = threadIdx.x, lr = tid % LPR, rs = tid / LPR;
  const bool a = tid < kPanel && active[pan * kPanel + tid] != 0;
  if (!__syncthreads_or(a)) return;
  for (int t = tid; t < k * kPanel; t += kThreads)
    sb[t] = beta[(size_t)(t >> 4) * g.C + pan * kPanel + (t & 15)];
  __syncthreads();
  const size_t pbase = (size_t)pan * n * kPanel;
  const V* Qp = reinterpret_cast<const V*>(Qk + pbase);
  V* Op = reinterpret_cast<V*>(Qout + pbase);
  const V* __restrict__ Rp = reinterpret_cast<const V*>(R + pbase);
  double acc[NVS];
#pragma unroll
  for (int v = 0; v < NVS; ++v) acc[v] = 0.0;
  const int r0 = rb * g.rpb, r1 = min(r0 + g.rpb, n);
  for (int row = r0 + rs; row < r1; row += RPP) {
    const size_t off = (size_t)row * LPR + lr;
    const V q = Qp[off];
    double qx[SPL], qy[SPL];
#pragma unroll
    for (int c = 0; c < SPL; ++c) lv_get<T>(q, c, qx[c], qy[c]);
#pragma unroll 4
    for (int i = 0; i < k; ++i) {
      V vq;
      if constexpr (HQ && SPL == 2)
        vq = unpack_cbf16x2(reinterpret_cast<const uint2*>(Qb + (size_t)i * vstride)
                                [((size_t)pan * n + row) * 8 + lr]);
      else
        vq = reinterpret_cast<const V*>(Qb + (size_t)i * vstride + pbase)[off];
#pragma unroll
      for (int c = 0; c < SPL; ++c) {
        const double2 b = sb[i * kPanel + lr * SPL + c];
        double vx, vy;
        lv_get<T>(vq, c, vx, vy);
        qx[c] -= b.x * vx - b.y * vy;
        qy[c] -= b.x * vy + b.y * vx;
      }
    }
    V qn;
    qn.x = (T)qx[0];
    qn.y = (T)qy[0];
    if constexpr (SPL == 2) lv_set_zw(qn, (T)qx[1], (T)qy[1]);
    if constexpr (HQ && SPL == 2) {
      const uint2 hq = make_uint2(pack_cbf16(qn.x, qn.y), pack_cbf16(lv_z(qn), lv_w(qn)));
      qn = unpack_cbf16x2(hq);
      if (store) reinterpret_cast<uint2*>(Qout)[((size_t)pan * n + row) * 8 + lr] = hq;
    } else {
      if (store) Op[off] = qn;
    }
    const V r = Rp[off];
#pragma unroll
    for (int c = 0; c < SPL; ++c) {
      double nx, ny, rx, ry;
      lv_get<T>(qn, c, nx, ny);
      lv_get<T>(r, c, rx, ry);
      acc[0 * SPL + c] += nx * nx + ny * ny;
      acc[1 * SPL + c] += nx * rx + ny * ry;
      acc[2 * SPL + c] += nx * ry - ny * rx;
    }
  }
  reduce_lv<NVS, LPR>(acc, NVS, red, [&](int v, int ln, double sum) {
    const int c = v % SPL, vi = v / SPL;  // 0: <q,q>, 1: Re <q,r>, 2: Im <q,r>
    const size_t dst = ((size_t)rb * g.ND + (vi == 0 ? 0 : 1)) * g.C + pan * kPanel + ln * SPL + c;
    double* d = reinterpret_cast<double*>(part + dst);
    if (vi == 0) {
      d[0] = sum;
      d[1] = 0.0;
    } else {
      d[vi - 1] = sum;
    }
  });
}

// r -= alpha q, partial ||r||^2, and z from the new r: pc 0 copy, 1 Jacobi,
// 2 none, 3 omega D^-1 r (the first smoothing step of the next V-cycle, from
// the stored r exactly as the level-0 jacobi0 kernel forms it), 4 the same
// stored as complex bfloat16 (complex-float sweeps).  HQ: q_k is stored as
// complex bfloat16 (layout as in k_dots_lv).
template <typename T, bool HQ = false>
__global__ __launch_bounds__(kThreads) void k_step_lv(
    int n, PanelGrid g, const int* __restrict__ active, const double2* __restrict__ sigma,
    const double* __restrict__ da, const double* __restrict__ db, int pc, double omega,
    typename CT<T>::t* __restrict__ R, typename CT<T>::t* __restrict__ Z,
    const typename CT<T>::t* __restrict__ Qk, const double2* __restrict__ alpha_k,
    double2* __restrict__ part) {
  using V = typename LaneVec<T>::V;
  constexpr int SPL = LaneVec<T>::SPL;
  constexpr int LPR = kPanel / SPL;
  constexpr int RPP = kThreads / LPR;
  __shared__ double red[4 * SPL * LPR];
  int rb, pan;
  if (!map_block(g, rb, pan)) return;
  const int tid = threadIdx.x, lr = tid % LPR, rs = tid / LPR;
  const bool a = tid < kPanel && active[pan * kPanel + tid] != 0;
  if (!__syncthreads_or(a)) return;
  double2 al[SPL], sg[SPL];
#pragma unroll
  for (int c = 0; c < SPL; ++c) {
    al[c] = alpha_k[pan * kPanel + lr * SPL + c];
    sg[c] = sigma[pan * kPanel + lr * SPL + c];
  }
  const size_t pbase = (size_t)pan * n * kPanel;
  V* __restrict__ Rp = reinterpret_cast<V*>(R + pbase);
  V* __restrict__ Zp = Z != nullptr ? reinterpret_cast<V*>(Z + pbase) : nullptr;
  const V* __restrict__ Qp = reinterpret_cast<const V*>(Qk + pbase);
  double acc[SPL];
#pragma unroll
  for (int c = 0; c < SPL; ++c) acc[c] = 0.0;
  const int r0 = rb * g.rpb, r1 = min(r0 + g.rpb, n);
  for (int row = r0 + rs; row < r1; row += RPP) {
    const size_t off = (size_t)row * LPR + lr;
    const V r = Rp[off];
    V q;
    if constexpr (HQ && SPL == 2)
      q = unpack_cbf16x2(reinterpret_cast<const uint2*>(Qk)[((size_t)pan * n + row) * 8 + lr]);
    else
      q = Qp[off];
    V rn, zn;
#pragma unroll
    for (int c = 0; c < SPL; ++c) {
      double rx, ry, qx, qy;
      lv_get<T>(r, c, rx, ry);
      lv_get<T>(q, c, qx, qy);
      const T nx = (T)(rx - (al[c].x * qx - al[c].y * qy));
      const T ny = (T)(ry - (al[c].x * qy + al[c].y * qx));
      const double x = nx, y = ny;
      acc[c] += x * x + y * y;
      T zx = nx, zy = ny;
      if (pc == 1) {
        const double2 d = jacobi_inv(da[row], db[row], sg[c]);
        zx = (T)(x * d.x - y * d.y);
        zy = (T)(x * d.y + y * d.x);
      } else if (pc == 3 || pc == 4) {
        const double2 d = jacobi_inv(da[row], db[row], sg[c]);
        zx = (T)(omega * (x * d.x - y * d.y));
        zy = (T)(omega * (x * d.y + y * d.x));
      }
      if (c == 0) {
        rn.x = nx;
        rn.y = ny;
        zn.x = zx;
        zn.y = zy;
      } else {
        lv_set_zw(rn, nx, ny);
        lv_set_zw(zn, zx, zy);
      }
    }
    Rp[off] = rn;
    if (Zp != nullptr && pc == 4) {
      if constexpr (SPL == 2)
        reinterpret_cast<uint2*>(Z)[((size_t)pan * n + row) * 8 + lr] =
            make_uint2(pack_cbf16(zn.x, zn.y), pack_cbf16(lv_z(zn), lv_w(zn)));
    } else if (Zp != nullptr && pc != 2) {
      Zp[off] = zn;
    }
  }
  reduce_lv<SPL, LPR>(acc, SPL, red, [&](int c, int ln, double sum) {
    part[((size_t)rb * g.ND) * g.C + pan * kPanel + ln * SPL + c] = make_double2(sum, 0.0);
  });
}

template <typename T>
HaloView halo_view(const DevPencil& P) {
  HaloView v;
  v.ntile = P.hx_ntile;
  v.emax = P.hx_emax;
  v.trow = P.hx_trow;
  v.hptr = P.hx_hptr;
  v.halo = P.hx_halo;
  v.sptr = P.hx_sptr;
  v.slen = P.hx_slen;
  v.lcol = P.hx_lcol;
  v.ab = std::is_same<T, float>::value ? static_cast<const void*>(P.hx_ab32)
                                       : static_cast<const void*>(P.hx_ab64);
  return v;
}

template <typename T>
size_t halo_lds_bytes(const DevPencil& P) {
  return (size_t)P.hx_hmax * (8 * sizeof(typename LaneVec<T>::V) + sizeof(int)) +
         (size_t)P.hx_emax * (2 * sizeof(T) + sizeof(unsigned));  // (a, b), column offset
}

template <typename T>
bool halo_selected(const DevPencil& P) {
  const int var = std::is_same<T, float>::value ? P.var32 : P.var64;
  // (the halo kernels address a unit's rows with 32-bit element offsets)
  return var == kSpmmHalo && P.n <= (1 << 28) && P.hx_ntile > 0 && P.hx_hmax <= kHaloMaxH &&
         halo_lds_bytes<T>(P) <= 96 * 1024;
}

// Halo-tile sweep: returns false when the pencil's kernel choice for T is not
// the halo format (nothing launched).
template <typename T>
bool launch_halo(const DevPencil& P, const PanelGrid& g, const SlotTables& st, int epi,
                 double omega, const void* Z, const void* Bin, void* Out, hipStream_t s,
                 hipError_t& err) {
  using C = typename CT<T>::t;
  if (!halo_selected<T>(P)) return false;
  constexpr int UPP = std::is_same<T, float>::value ? 1 : 2;
  const int G = kHaloMaxG;
  const int nug = (g.npan * UPP + G - 1) / G;
  PanelGrid gg = g;
  // every tile of one run of G units before the next run: the same panels
  // of neighbouring tiles are swept close together in time (halo rows
  // shared through L2)
  gg.group = 1;
  gg.rpb = P.hx_hmax;  // LDS halo rows (the kernel's carve-up of dynamic LDS)
  const long total = (long)P.hx_ntile * nug;
  const unsigned blocks = (unsigned)(((total + 7) / 8) * 8);
  const size_t bytes = halo_lds_bytes<T>(P);
  const HaloView hv = halo_view<T>(P);
  auto Zc = static_cast<const C*>(Z);
  auto Bc = static_cast<const C*>(Bin);
  auto Oc = static_cast<C*>(Out);
#define SLRF_HALO(E)                                                                      \
  k_apply_halo<T, E><<<blocks, kThreads, bytes, s>>>(P.n, hv, gg, G, st.active, st.sigma, \
                                                     Zc, Oc, Bc, P.da, P.db, omega)
  if (epi == kEpiApply)
    SLRF_HALO(kEpiApply);
  else if (epi == kEpiResid)
    SLRF_HALO(kEpiResid);
  else
    SLRF_HALO(kEpiJacobi);
#undef SLRF_HALO
  err = hipGetLastError();
  return true;
}

template <typename T>
bool sweep_is_halo(const DevPencil& P) {
  return halo_selected<T>(P);
}

template <typename T>
bool launch_resid_bf16(const DevPencil& P, const PanelGrid& g, const SlotTables& st,
                       const void* X, const void* Bin, void* Out, hipStream_t s,
                       hipError_t& err, bool x_bf16) {
  using C = typename CT<T>::t;
  if (!std::is_same<T, float>::value || !halo_selected<T>(P)) return false;
  const int G = kHaloMaxG;
  const int nug = (g.npan + G - 1) / G;
  PanelGrid gg = g;
  // every tile of one run of G units before the next run: the same panels
  // of neighbouring tiles are swept close together in time (halo rows
  // shared through L2)
  gg.group = 1;
  gg.rpb = P.hx_hmax;
  const long total = (long)P.hx_ntile * nug;
  const unsigned blocks = (unsigned)(((total + 7) / 8) * 8);
#define SLRF_RH(ZH)                                                                          \
  k_apply_halo<T, kEpiResidH, ZH><<<blocks, kThreads, halo_lds_bytes<T>(P), s>>>(            \
      P.n, halo_view<T>(P), gg, G, st.active, st.sigma, static_cast<const C*>(X),            \
      static_cast<C*>(Out), static_cast<const C*>(Bin), P.da, P.db, 0.0)
  if (x_bf16)
    SLRF_RH(true);
  else
    SLRF_RH(false);
#undef SLRF_RH
  err = hipGetLastError();
  return true;
}

template <typename T>
bool launch_post_image(const DevImage& I, const DevPencil& P, const PanelGrid& g,
                       const SlotTables& st, double omega, const void* E, const void* X0,
                       const void* R1, void* Out, hipStream_t s, hipError_t& err,
                       bool r1_bf16) {
  using C = typename CT<T>::t;
  if (I.ntile == 0 || I.hmax > kImgMaxH2) return false;
  err = hipSuccess;
  constexpr int UPP = std::is_same<T, float>::value ? 1 : 2;
  const int G = kHaloMaxG;
  const int nug = (g.npan * UPP + G - 1) / G;
  PanelGrid gg = g;
  // every tile of one run of G units before the next run: the same panels
  // of neighbouring tiles are swept close together in time (halo rows
  // shared through L2)
  gg.group = 1;
  gg.rpb = I.hmax;  // LDS halo rows (the kernel's carve-up of dynamic LDS)
  const long total = (long)I.ntile * nug;
  const unsigned blocks = (unsigned)(((total + 7) / 8) * 8);
  const size_t bytes = (size_t)I.hmax * (8 * sizeof(typename LaneVec<T>::V) + sizeof(int)) +
                       (size_t)I.emax * (2 * sizeof(T) + sizeof(unsigned)) +
                       (size_t)I.pemax * (sizeof(T) + sizeof(unsigned));
  HaloView hv;
  hv.ntile = I.ntile;
  hv.emax = I.emax;
  hv.trow = I.trow;
  hv.hptr = I.hptr;
  hv.halo = I.halo;
  hv.sptr = I.sptr;
  hv.slen = nullptr;
  hv.lcol = I.lcol;
  hv.ab = std::is_same<T, float>::value ? static_cast<const void*>(I.ab32)
                                        : static_cast<const void*>(I.ab64);
  PSubView pw;
  pw.emax = I.pemax;
  pw.sptr = I.psptr;
  pw.lcol = I.plcol;
  pw.v = std::is_same<T, float>::value ? static_cast<const void*>(I.p32)
                                       : static_cast<const void*>(I.p64);
  // (beyond 64 KiB of dynamic LDS the kernel must be allowed the size first)
#define SLRF_POST(H, HM)                                                                         \
  if (bytes > 65536 &&                                                                           \
      hipFuncSetAttribute(reinterpret_cast<const void*>(&k_post_image<T, H, HM>),                \
                          hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) != hipSuccess) \
    err = hipErrorInvalidValue;                                                                  \
  else                                                                                           \
    k_post_image<T, H, HM><<<blocks, kThreads, bytes, s>>>(                                      \
      P.n, I.nc, hv, pw, gg, G, st.active, st.sigma, static_cast<const C*>(E),                   \
      static_cast<const C*>(X0), static_cast<const C*>(R1), static_cast<C*>(Out), P.da, P.db, \
      omega)
  const bool wide = I.hmax > kImgMaxH;
  if (r1_bf16 && std::is_same<T, float>::value) {
    if (wide) SLRF_POST(true, kImgMaxH2); else SLRF_POST(true, kImgMaxH);
  } else {
    if (wide) SLRF_POST(false, kImgMaxH2); else SLRF_POST(false, kImgMaxH);
  }
#undef SLRF_POST
  if (err == hipSuccess) err = hipGetLastError();
  return true;
}

template <typename T>
hipError_t launch_dots(const DevPencil& P, const PanelGrid& g, const SlotTables& st,
                       const void* Qk, const void* Qbase, size_t vstride, int k, double2* part,
                       hipStream_t s, bool hq) {
  using C = typename CT<T>::t;
  auto Qc = static_cast<const C*>(Qk);
  auto Qb = static_cast<const C*>(Qbase);
  if (k <= 0) return hipSuccess;
  // (the accumulators of MAXK directions stay live whatever k is: the
  // smallest instantiation that holds k keeps the register count down)
  if (hq) {
    if (!std::is_same<T, float>::value || k > 8) return hipErrorInvalidValue;
    if (k <= 2)
      k_dots_lv<T, 2, true><<<g.blocks(), kThreads, 0, s>>>(P.n, g, st.active, Qc, Qb, vstride,
                                                             k, part);
    else if (k <= 4)
      k_dots_lv<T, 4, true><<<g.blocks(), kThreads, 0, s>>>(P.n, g, st.active, Qc, Qb, vstride,
                                                             k, part);
    else
      k_dots_lv<T, 8, true><<<g.blocks(), kThreads, 0, s>>>(P.n, g, st.active, Qc, Qb, vstride,
                                                             k, part);
    return hipGetLastError();
  }
  if (k <= 2)
    k_dots_lv<T, 2><<<g.blocks(), kThreads, 0, s>>>(P.n, g, st.active, Qc, Qb, vstride, k,
                                                     part);
  else if (k <= 4)
    k_dots_lv<T, 4><<<g.blocks(), kThreads, 0, s>>>(P.n, g, st.active, Qc, Qb, vstride, k,
                                                     part);
  else if (k <= 8)
    k_dots_lv<T, 8><<<g.blocks(), kThreads, 0, s>>>(P.n, g, st.active, Qc, Qb, vstride, k,
                                                     part);
  else if (k <= 16)
    k_dots<T, 16><<<g.blocks(), kThreads, 0, s>>>(P.n, g, st.active, Qc, Qb, vstride, k, part);
  else
    k_dots<T, 32><<<g.blocks(), kThreads, 0, s>>>(P.n, g, st.active, Qc, Qb, vstride, k, part);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_sweep(const DevPencil& P, const PanelGrid& g, const SlotTables& st,
                        const void* Z, void* Out, hipStream_t s) {
  return launch_apply_dots<T>(P, g, st, Z, Out, nullptr, 0, 0, nullptr, false, s);
}

template <typename T>
hipError_t launch_apply_dots(const DevPencil& P, const PanelGrid& g, const SlotTables& st,
                             const void* Z, void* Qk, const void* Qbase, size_t vstride, int k,
                             double2* part, bool, hipStream_t s) {
  using C = typename CT<T>::t;
  auto Zc = static_cast<const C*>(Z);
  auto Qc = static_cast<C*>(Qk);
  auto Qb = static_cast<const C*>(Qbase);
  {
    hipError_t err = hipSuccess;
    // wave-uniform row-group sweep, then the CGS projections as a separate pass
    if (launch_ugroup<T>(P, g, st, kEpiApply, 0.0, Z, nullptr, Qk, s, err)) {
      if (err != hipSuccess || k == 0) return err;
      return launch_dots<T>(P, g, st, Qk, Qbase, vstride, k, part, s, false);
    }
    // halo sweep, then the CGS projections as a separate streaming pass
    if (launch_halo<T>(P, g, st, kEpiApply, 0.0, Z, nullptr, Qk, s, err)) {
      if (err != hipSuccess || k == 0) return err;
      return launch_dots<T>(P, g, st, Qk, Qbase, vstride, k, part, s, false);
    }
    if (launch_grp<T>(P, g, st, kEpiApply, 0.0, Z, nullptr, Qk, s, err)) {
      if (err != hipSuccess || k == 0) return err;
      if (k <= 8)
        k_dots<T, 8><<<g.blocks(), kThreads, 0, s>>>(P.n, g, st.active, Qc, Qb, vstride, k, part);
      else if (k <= 16)
        k_dots<T, 16><<<g.blocks(), kThreads, 0, s>>>(P.n, g, st.active, Qc, Qb, vstride, k, part);
      else
        k_dots<T, 32><<<g.blocks(), kThreads, 0, s>>>(P.n, g, st.active, Qc, Qb, vstride, k, part);
      return hipGetLastError();
    }
  }
  int sub = 0, cap = 0;
  size_t bytes = 0;
  if (lds_plan<T>(P, g.rpb, sub, cap, bytes)) {
    PanelGrid gg = g;
    const int ncg = (g.npan + kGroupPanels - 1) / kGroupPanels;
    gg.group = ncg < 4 ? ncg : 4;
    const long total = (long)g.nrb * ncg;
    const unsigned blocks = (unsigned)(((total + 7) / 8) * 8);
    const int unr = lds_unroll<T>(P);
#define SLRF_LDS_APPLY(DOTS, U)                                                             \
  k_apply_lds<T, DOTS, kGroupPanels, kEpiApply, U><<<blocks, kThreads, bytes, s>>>(          \
      P.n, P.rowptr, P.col, vals_a<T>(P), vals_b<T>(P), gg, sub, cap, st.active, st.sigma, Zc, \
      Qc, Qb, vstride, k, part)
    if (k == 0) {
      if (unr == 16) SLRF_LDS_APPLY(false, 16);
      else if (unr == 32) SLRF_LDS_APPLY(false, 32);
      else SLRF_LDS_APPLY(false, 8);
    } else {
      if (unr == 16) SLRF_LDS_APPLY(true, 16);
      else if (unr == 32) SLRF_LDS_APPLY(true, 32);
      else SLRF_LDS_APPLY(true, 8);
    }
#undef SLRF_LDS_APPLY
    return hipGetLastError();
  }
  const dim3 grid(g.blocks()), block(kThreads);
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
  SlotTables st;
  st.sigma = sigma_slot;
  st.active = nullptr;
  return launch_apply_dots<T>(P, g, st, Z, Q, nullptr, 0, 0, nullptr, false, s);
}

template <typename T>
hipError_t launch_orth(const DevPencil& P, const PanelGrid& g, const SlotTables& st,
                       const void* Qk, const void* R, const void* Qbase, size_t vstride, int k,
                       const double2* beta, double2* part, hipStream_t s, void* Qout,
                       bool store, bool hq) {
  using C = typename CT<T>::t;
  if (hq) {
    if (!std::is_same<T, float>::value) return hipErrorInvalidValue;
    k_orth_lv<T, true><<<g.blocks(), kThreads, 0, s>>>(
        P.n, g, st.active, static_cast<const C*>(Qk), static_cast<const C*>(R),
        static_cast<const C*>(Qbase), vstride, k, beta, part, static_cast<C*>(Qout),
        store ? 1 : 0);
    return hipGetLastError();
  }
  k_orth_lv<T><<<g.blocks(), kThreads, 0, s>>>(
      P.n, g, st.active, static_cast<const C*>(Qk), static_cast<const C*>(R),
      static_cast<const C*>(Qbase), vstride, k, beta, part, static_cast<C*>(Qout),
      store ? 1 : 0);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_step(const DevPencil& P, const PanelGrid& g, const SlotTables& st, void* R,
                       void* Z, const void* Qk, const double2* alpha_k, double2* part,
                       int precond, double omega, hipStream_t s, bool hq) {
  using C = typename CT<T>::t;
  if (hq) {
    if (!std::is_same<T, float>::value) return hipErrorInvalidValue;
    k_step_lv<T, true><<<g.blocks(), kThreads, 0, s>>>(
        P.n, g, st.active, st.sigma, P.da, P.db, precond, omega, static_cast<C*>(R),
        static_cast<C*>(Z), static_cast<const C*>(Qk), alpha_k, part);
    return hipGetLastError();
  }
  k_step_lv<T><<<g.blocks(), kThreads, 0, s>>>(P.n, g, st.active, st.sigma, P.da, P.db,
                                               precond, omega, static_cast<C*>(R),
                                               static_cast<C*>(Z), static_cast<const C*>(Qk),
                                               alpha_k, part);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_yupdate(int n, const PanelGrid& g, const SlotTables& st, double2* Y,
                          const void* Z0, const void* Zbase, size_t vstride, int kk,
                          const double2* alpha, const double2* bhist, hipStream_t s) {
  using C = typename CT<T>::t;
  k_yupdate<T><<<g.blocks(), kThreads, 0, s>>>(n, g, st.sys, Y, static_cast<const C*>(Z0),
                                               static_cast<const C*>(Zbase), vstride, kk,
                                               alpha, bhist);
  return hipGetLastError();
}

bool launch_spmm_real_halo(const DevPencil& P, const double* X, int ld, int nc, double* AX,
                           double* BX, const double* theta, double* E, hipStream_t s,
                           hipError_t& err) {
  // (on rows of many entries the tiles' halos are wide and the CSR kernel is
  // faster: 48^3 elasticity, 78 entries per row, 300 columns: 6.1 against
  // 3.9 ms; the 27-point Q1 pencil at 160 columns: 0.37 against 0.74 ms)
  if (P.hx_ntile == 0 || P.hx_ab64 == nullptr || nc <= 0 || (nc & 1) || (ld & 1) ||
      (reinterpret_cast<uintptr_t>(X) & 15) || P.nnz > 40L * P.n)
    return false;
  const int G = kHaloMaxG;
  const int nunit = (nc + 15) / 16;
  const int nug = (nunit + G - 1) / G;
  const long total = (long)P.hx_ntile * nug;
  const unsigned blocks = (unsigned)(((total + 7) / 8) * 8);
  k_spmm_real_halo<<<blocks, kThreads, halo_lds_bytes<double>(P), s>>>(
      P.n, halo_view<double>(P), P.hx_hmax, nunit, G, X, ld, nc, AX, BX, theta, E);
  err = hipGetLastError();
  return true;
}

template <typename T>
hipError_t launch_true_resid(const DevPencil& P, const PanelGrid& g, const SlotTables& st,
                             const double2* Y, const double* F, int ldf, void* R, void* Z,
                             double2* part, int precond, hipStream_t s) {
  using C = typename CT<T>::t;
  if (halo_selected<double>(P)) {
    // halo tiles (the complex-double sweep's format) and a norm pass over R
    const int G = kHaloMaxG;
    const int nug = (g.npan * 2 + G - 1) / G;
    PanelGrid gg = g;
    // every tile of one run of G units before the next run: the same panels
    // of neighbouring tiles are swept close together in time (halo rows
    // shared through L2)
    gg.group = 1;
    gg.rpb = P.hx_hmax;
    const long total = (long)P.hx_ntile * nug;
    const unsigned blocks = (unsigned)(((total + 7) / 8) * 8);
    k_true_halo<T><<<blocks, kThreads, halo_lds_bytes<double>(P), s>>>(
        P.n, halo_view<double>(P), gg, G, st.sys, st.col, st.sigma, Y, F, ldf,
        static_cast<C*>(R), static_cast<C*>(Z), P.da, P.db, precond);
    k_rnorm<T><<<g.blocks(), kThreads, 0, s>>>(P.n, g, st.sys, static_cast<const C*>(R), part);
    return hipGetLastError();
  }
  int sub = 0, cap = 0;
  size_t bytes = 0;
  if (lds_fit<double>(P, g.rpb, sub, cap, bytes)) {
    PanelGrid gg = g;
    const int ncg = (g.npan + kGroupPanels - 1) / kGroupPanels;
    gg.group = ncg < 4 ? ncg : 4;
    const long total = (long)g.nrb * ncg;
    const unsigned blocks = (unsigned)(((total + 7) / 8) * 8);
    k_true_resid_lds<T, kGroupPanels, 8><<<blocks, kThreads, bytes, s>>>(
        P.n, P.rowptr, P.col, P.a, P.b, P.da, P.db, precond, gg, sub, cap, st.sys, st.col,
        st.sigma, Y, F, ldf, static_cast<C*>(R), static_cast<C*>(Z), part);
    return hipGetLastError();
  }
  k_true_resid<T><<<g.blocks(), kThreads, 0, s>>>(
      P.n, P.rowptr, P.col, P.a, P.b, P.da, P.db, precond, g, st.sys, st.col, st.sigma,
      Y, F, ldf, static_cast<C*>(R), static_cast<C*>(Z), part);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_admit(const DevPencil& P, const PanelGrid& g, const SlotTables& st,
                        const double2* Yold, const void* Rold, const void* Zold, double2* Ynew,
                        void* Rnew, void* Znew, const double* F, const double* E,
                        const double* X, int ld, bool warm, double2* part, int precond,
                        hipStream_t s) {
  using C = typename CT<T>::t;
  k_admit<T><<<g.blocks(), kThreads, 0, s>>>(
      P.n, P.da, P.db, precond, g, st.sys, st.src, st.col, st.sigma, st.theta, Yold,
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
  if (npoles >= 1 && kPanel % npoles == 0) {
    const long total = (long)((ncols * npoles + kPanel - 1) / kPanel) * n * kPanel;
    k_filter_sum_p<<<cdiv((size_t)total, kThreads), kThreads, 0, s>>>(n, ncols, npoles, total,
                                                                      Ystore, w, Ur);
    return hipGetLastError();
  }
  k_filter_sum<<<cdiv(tot, kThreads), kThreads, 0, s>>>(n, ncols, npoles, Ystore, w, Ur);
  return hipGetLastError();
}

// Second stage with the row blocks split over the 16 waves of a workgroup
// (wave w takes rb = w, w + 16, ...; lanes take 64 consecutive slots, so the
// loads coalesce), then the 16 wave sums in wave order: a fixed order.
__global__ __launch_bounds__(1024) void k_reduce16w(const double2* __restrict__ part, int nrb,
                                                    int ND, int C, int nd, int nslots,
                                                    double2* __restrict__ out) {
  __shared__ double2 red[16][64];
  const int nsc = (nslots + 63) / 64;
  const int d = blockIdx.x / nsc, slot = (blockIdx.x % nsc) * 64 + (threadIdx.x & 63);
  const int w = threadIdx.x >> 6;
  double2 s[2] = {};
  if (slot < nslots) {
    int i = 0;
    for (int rb = w; rb < nrb; rb += 16, ++i) {
      const double2 v = part[((size_t)rb * ND + d) * C + slot];
      s[i & 1].x += v.x;
      s[i & 1].y += v.y;
    }
  }
  red[w][threadIdx.x & 63] = make_double2(s[0].x + s[1].x, s[0].y + s[1].y);
  __syncthreads();
  if (w == 0 && slot < nslots) {
    double2 t = red[0][threadIdx.x];
    for (int k = 1; k < 16; ++k) {
      t.x += red[k][threadIdx.x].x;
      t.y += red[k][threadIdx.x].y;
    }
    out[(size_t)d * C + slot] = t;
  }
}

hipError_t launch_reduce(const double2* part, int nrb, int ND, int C, int nd, int nslots,
                         double2* out, hipStream_t s) {
  const size_t tot = (size_t)nd * nslots;
  if (tot == 0) return hipSuccess;
  if (nrb >= 64) {
    k_reduce16w<<<(unsigned)(nd * ((nslots + 63) / 64)), 1024, 0, s>>>(part, nrb, ND, C, nd,
                                                                         nslots, out);
    return hipGetLastError();
  }
  k_reduce<<<cdiv(tot, kThreads), kThreads, 0, s>>>(part, nrb, ND, C, nd, nslots, out);
  return hipGetLastError();
}

hipError_t launch_fin_beta(const double2* red, int k, int C, int nslots, const SlotTables& st,
                           const SlotScalars& sc, hipStream_t s) {
  k_fin_beta<<<cdiv(nslots, 256), 256, 0, s>>>(red, k, C, nslots, st.active, sc.qq, sc.beta,
                                                sc.bhist);
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
  template bool sweep_is_halo<T>(const DevPencil&);                                          \
  template hipError_t launch_sweep<T>(const DevPencil&, const PanelGrid&, const SlotTables&, \
                                      const void*, void*, hipStream_t);                      \
  template hipError_t launch_dots<T>(const DevPencil&, const PanelGrid&, const SlotTables&,  \
                                     const void*, const void*, size_t, int, double2*,        \
                                     hipStream_t, bool);                                     \
  template hipError_t launch_apply_dots<T>(const DevPencil&, const PanelGrid&,               \
                                           const SlotTables&, const void*, void*,            \
                                           const void*, size_t, int, double2*, bool,         \
                                           hipStream_t);                                     \
  template hipError_t launch_spmm_panel<T>(const DevPencil&, const PanelGrid&,               \
                                           const double2*, const void*, void*, hipStream_t); \
  template hipError_t launch_orth<T>(const DevPencil&, const PanelGrid&, const SlotTables&,  \
                                     const void*, const void*, const void*, size_t, int,     \
                                     const double2*, double2*, hipStream_t, void*, bool,     \
                                     bool);                                                  \
  template hipError_t launch_step<T>(const DevPencil&, const PanelGrid&, const SlotTables&,  \
                                     void*, void*, const void*, const double2*, double2*,    \
                                     int, double, hipStream_t, bool);                       \
  template hipError_t launch_yupdate<T>(int, const PanelGrid&, const SlotTables&, double2*,  \
                                        const void*, const void*, size_t, int,               \
                                        const double2*, const double2*, hipStream_t);        \
  template hipError_t launch_true_resid<T>(const DevPencil&, const PanelGrid&,               \
                                           const SlotTables&, const double2*, const double*, \
                                           int, void*, void*, double2*, int, hipStream_t);   \
  template hipError_t launch_admit<T>(const DevPencil&, const PanelGrid&, const SlotTables&, \
                                      const double2*, const void*, const void*, double2*,    \
                                      void*, void*, const double*, const double*,            \
                                      const double*, int, bool, double2*, int, hipStream_t);

SLRF_INST(float)
SLRF_INST(double)

// ----------------------------- AMG launchers --------------------------------
template <typename T>
hipError_t launch_lvl_op(const DevPencil& L, const PanelGrid& g, const SlotTables& st, int epi,
                         double omega, const void* X, const void* Bin, void* Out, hipStream_t s) {
  using C = typename CT<T>::t;
  auto Xc = static_cast<const C*>(X);
  auto Bc = static_cast<const C*>(Bin);
  auto Oc = static_cast<C*>(Out);
  {
    hipError_t err = hipSuccess;
    if (launch_ugroup<T>(L, g, st, epi, omega, X, Bin, Out, s, err)) return err;
    if (launch_halo<T>(L, g, st, epi, omega, X, Bin, Out, s, err)) return err;
    if (launch_grp<T>(L, g, st, epi, omega, X, Bin, Out, s, err)) return err;
  }
  // (no partial sums here: a coarse level takes shorter row blocks, down to
  // 64 rows, until the launch has enough workgroups to fill the chip)
  const int ncg = (g.npan + kGroupPanels - 1) / kGroupPanels;
  int rpb = g.rpb;
  while (rpb > 64 && (long)((L.n + rpb - 1) / rpb) * ncg < 8192) rpb /= 2;
  int sub = 0, cap = 0;
  size_t bytes = 0;
  if (lds_plan<T>(L, rpb, sub, cap, bytes)) {
    PanelGrid gg = g;
    gg.rpb = rpb;
    gg.nrb = (L.n + rpb - 1) / rpb;
    gg.group = ncg < 4 ? ncg : 4;
    const long total = (long)gg.nrb * ncg;
    const unsigned blocks = (unsigned)(((total + 7) / 8) * 8);
    const int unr = lds_unroll<T>(L);
#define SLRF_LDS_LVL(E, U)                                                                   \
  k_apply_lds<T, false, kGroupPanels, E, U><<<blocks, kThreads, bytes, s>>>(                  \
      L.n, L.rowptr, L.col, vals_a<T>(L), vals_b<T>(L), gg, sub, cap, st.active, st.sigma, Xc, \
      Oc, nullptr, 0, 0, nullptr, Bc, L.da, L.db, omega)
    if (epi == kEpiResid) {
      if (unr == 16) SLRF_LDS_LVL(kEpiResid, 16);
      else if (unr == 32) SLRF_LDS_LVL(kEpiResid, 32);
      else SLRF_LDS_LVL(kEpiResid, 8);
    } else {
      if (unr == 16) SLRF_LDS_LVL(kEpiJacobi, 16);
      else if (unr == 32) SLRF_LDS_LVL(kEpiJacobi, 32);
      else SLRF_LDS_LVL(kEpiJacobi, 8);
    }
#undef SLRF_LDS_LVL
    return hipGetLastError();
  }
  if (epi == kEpiResid)
    k_lvl_simple<T, kEpiResid><<<g.blocks(), kThreads, 0, s>>>(
        L.n, L.rowptr, L.col, vals_a<T>(L), vals_b<T>(L), L.da, L.db, omega, g, st.active,
        st.sigma, Xc, Bc, Oc);
  else
    k_lvl_simple<T, kEpiJacobi><<<g.blocks(), kThreads, 0, s>>>(
        L.n, L.rowptr, L.col, vals_a<T>(L), vals_b<T>(L), L.da, L.db, omega, g, st.active,
        st.sigma, Xc, Bc, Oc);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_lvl_jacobi0(const DevPencil& L, const PanelGrid& g, const SlotTables& st,
                              double omega, const void* Bin, void* Out, hipStream_t s,
                              bool out_bf16) {
  using C = typename CT<T>::t;
  if (out_bf16 && std::is_same<T, float>::value)
    k_lvl_jacobi0<T, true><<<g.blocks(), kThreads, 0, s>>>(L.n, L.da, L.db, omega, g, st.active,
                                                           st.sigma, static_cast<const C*>(Bin),
                                                           static_cast<C*>(Out));
  else
    k_lvl_jacobi0<T><<<g.blocks(), kThreads, 0, s>>>(L.n, L.da, L.db, omega, g, st.active,
                                                     st.sigma, static_cast<const C*>(Bin),
                                                     static_cast<C*>(Out));
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// AMG transfers with 16-byte lane vectors (two complex floats or one complex
// double per lane).  Prolongation (short rows of P): 8 or 4 fine rows per wave,
// one coarse-row gather per entry, optional accumulation into the output.
// Restriction (long rows of R = P^T): one wave per (coarse row, panel), its
// lane groups take every EG-th entry, then a fixed xor-shuffle tree sums the
// groups (deterministic order).
// ---------------------------------------------------------------------------
template <typename T, bool ADD>
__global__ __launch_bounds__(kThreads) void k_prolong(
    int nout, int nin, const int* __restrict__ rowptr, const int* __restrict__ col,
    const T* __restrict__ v, PanelGrid g, const int* __restrict__ active,
    const typename CT<T>::t* __restrict__ In, typename CT<T>::t* __restrict__ Out) {
  using V = typename LaneVec<T>::V;
  constexpr int SPL = LaneVec<T>::SPL;
  constexpr int LPR = kPanel / SPL;
  constexpr int RPP = kThreads / LPR;
  int rb, pan;
  if (!map_block(g, rb, pan)) return;
  const int tid = threadIdx.x, lr = tid % LPR, rr = tid / LPR;
  const bool a = tid < kPanel && (active == nullptr || active[pan * kPanel + tid] != 0);
  if (!__syncthreads_or(a)) return;
  const V* __restrict__ Ip = reinterpret_cast<const V*>(In + (size_t)pan * nin * kPanel);
  V* __restrict__ Op = reinterpret_cast<V*>(Out + (size_t)pan * nout * kPanel);
  const int r0 = rb * g.rpb, r1 = min(r0 + g.rpb, nout);
  for (int row = r0 + rr; row < r1; row += RPP) {
    const int e0 = rowptr[row], e1 = rowptr[row + 1];
    T acc[2 * SPL];
#pragma unroll
    for (int c = 0; c < 2 * SPL; ++c) acc[c] = 0;
    for (int e = e0; e < e1; e += 4) {
      V z[4];
      T w[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        z[u] = V{};
        w[u] = 0;
        if (e + u < e1) {
          w[u] = v[e + u];
          z[u] = Ip[(size_t)col[e + u] * LPR + lr];
        }
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        acc[0] = mad(w[u], z[u].x, acc[0]);
        acc[1] = mad(w[u], z[u].y, acc[1]);
        if constexpr (SPL == 2) {
          acc[2] = mad(w[u], (T)lv_z(z[u]), acc[2]);
          acc[3] = mad(w[u], (T)lv_w(z[u]), acc[3]);
        }
      }
    }
    V o;
    o.x = acc[0];
    o.y = acc[1];
    if constexpr (SPL == 2) lv_set_zw(o, acc[2], acc[3]);
    if constexpr (ADD) {
      const V p = Op[(size_t)row * LPR + lr];
      o.x += p.x;
      o.y += p.y;
      if constexpr (SPL == 2) lv_set_zw(o, (T)(lv_z(o) + lv_z(p)), (T)(lv_w(o) + lv_w(p)));
    }
    Op[(size_t)row * LPR + lr] = o;
  }
}

// Prolongation with the rows of P staged in LDS (64 rows at a time) once per
// workgroup and shared by G panels; UNR coarse-row gathers in flight per lane.
// Entries are summed in CSR order as in k_prolong (same result bitwise).
template <typename T, bool ADD, int G>
__global__ __launch_bounds__(kThreads) void k_prolong_lds(
    int nout, int nin, const int* __restrict__ rowptr, const int* __restrict__ col,
    const T* __restrict__ v, PanelGrid g, int lds_nnz, const int* __restrict__ active,
    const typename CT<T>::t* __restrict__ In, typename CT<T>::t* __restrict__ Out) {
  using V = typename LaneVec<T>::V;
  constexpr int SPL = LaneVec<T>::SPL;
  constexpr int LPR = kPanel / SPL;
  constexpr int RPP = kThreads / LPR;
  constexpr int SUB = 64;
  constexpr int UNR = 4;
  extern __shared__ __attribute__((aligned(16))) double smem_d[];
  T* s_v = reinterpret_cast<T*>(smem_d);
  int* s_col = reinterpret_cast<int*>(s_v + lds_nnz);
  __shared__ int s_rp[SUB + 1];
  __shared__ int s_pany[G];
  const int ncg = (g.npan + G - 1) / G;
  int rb, cg;
  if (!map_tile(g.nrb, ncg, g.group, rb, cg)) return;
  const int tid = threadIdx.x, lr = tid % LPR, rr = tid / LPR;
  const int pan0 = cg * G;
  if (tid < G) {
    const int p = pan0 + tid;
    int any = 0;
    if (p < g.npan)
      for (int l = 0; l < kPanel; ++l) any |= (active == nullptr || active[p * kPanel + l] != 0);
    s_pany[tid] = any;
  }
  const int R0 = rb * g.rpb, R1 = min(R0 + g.rpb, nout);
  for (int s0 = R0; s0 < R1; s0 += SUB) {
    const int s1 = min(s0 + SUB, R1);
    const int eb = rowptr[s0];
    const int nsub = rowptr[s1] - eb;
    for (int t = tid; t <= s1 - s0; t += kThreads) s_rp[t] = rowptr[s0 + t] - eb;
    for (int t = tid; t < nsub; t += kThreads) {
      s_col[t] = col[eb + t];
      s_v[t] = v[eb + t];
    }
    __syncthreads();
#pragma unroll
    for (int gg = 0; gg < G; ++gg) {
      if (!s_pany[gg]) continue;
      const int pan = pan0 + gg;
      const V* __restrict__ Ip = reinterpret_cast<const V*>(In + (size_t)pan * nin * kPanel);
      V* __restrict__ Op = reinterpret_cast<V*>(Out + (size_t)pan * nout * kPanel);
      for (int row = s0 + rr; row < s1; row += RPP) {
        const int e0 = s_rp[row - s0], e1 = s_rp[row - s0 + 1];
        T acc[2 * SPL];
#pragma unroll
        for (int c = 0; c < 2 * SPL; ++c) acc[c] = 0;
        for (int e = e0; e < e1; e += UNR) {
          V z[UNR];
          T w[UNR];
#pragma unroll
          for (int u = 0; u < UNR; ++u) {
            z[u] = V{};
            w[u] = 0;
            if (e + u < e1) {
              w[u] = s_v[e + u];
              z[u] = Ip[(size_t)s_col[e + u] * LPR + lr];
            }
          }
#pragma unroll
          for (int u = 0; u < UNR; ++u) {
            acc[0] = mad(w[u], z[u].x, acc[0]);
            acc[1] = mad(w[u], z[u].y, acc[1]);
            if constexpr (SPL == 2) {
              acc[2] = mad(w[u], (T)lv_z(z[u]), acc[2]);
              acc[3] = mad(w[u], (T)lv_w(z[u]), acc[3]);
            }
          }
        }
        V o;
        o.x = acc[0];
        o.y = acc[1];
        if constexpr (SPL == 2) lv_set_zw(o, acc[2], acc[3]);
        if constexpr (ADD) {
          const V p = Op[(size_t)row * LPR + lr];
          o.x += p.x;
          o.y += p.y;
          if constexpr (SPL == 2) lv_set_zw(o, (T)(lv_z(o) + lv_z(p)), (T)(lv_w(o) + lv_w(p)));
        }
        Op[(size_t)row * LPR + lr] = o;
      }
    }
    __syncthreads();
  }
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_restrict(
    int nout, int nin, const int* __restrict__ rowptr, const int* __restrict__ col,
    const T* __restrict__ v, int npan, const int* __restrict__ active,
    const typename CT<T>::t* __restrict__ In, typename CT<T>::t* __restrict__ Out) {
  using V = typename LaneVec<T>::V;
  constexpr int SPL = LaneVec<T>::SPL;
  constexpr int LPR = kPanel / SPL;  // lanes per panel row
  constexpr int EG = 64 / LPR;       // entry groups per wave
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63, lr = l % LPR, eg = l / LPR;
  // Work item t = (group of 4 panels, coarse row), row-minor.  Workgroups are
  // dealt to the 8 XCDs round-robin; each XCD takes one contiguous range of t,
  // so neighbouring coarse rows of a panel group, whose fine supports
  // overlap, gather through the same L2.
  const int ngrp = (npan + 3) / 4;
  const long total = (long)nout * ngrp;
  const long per = (total + 7) / 8;
  const long b = blockIdx.x;
  const long t = (b & 7) * per + (b >> 3);
  if (t >= total) return;
  const int row = (int)(t % nout);
  const int pan = (int)(t / nout) * 4 + w;
  if (pan >= npan) return;  // whole waves (no workgroup barrier below)
  const bool a = l < kPanel && (active == nullptr || active[pan * kPanel + l] != 0);
  if (!__any(a)) return;
  const V* __restrict__ Ip = reinterpret_cast<const V*>(In + (size_t)pan * nin * kPanel);
  V* __restrict__ Op = reinterpret_cast<V*>(Out + (size_t)pan * nout * kPanel);
  const int e0 = rowptr[row], e1 = rowptr[row + 1];
  T acc[2 * SPL];
#pragma unroll
  for (int c = 0; c < 2 * SPL; ++c) acc[c] = 0;
  // U entries per entry group and round, all column indices of a round loaded
  // before its gathers are issued
  constexpr int U = 8;
  for (int e = e0 + eg; e < e1; e += U * EG) {
    int ci[U];
    T wv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int ee = e + u * EG;
      ci[u] = ee < e1 ? col[ee] : -1;
      wv[u] = ee < e1 ? v[ee] : (T)0;
    }
    V z[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      z[u] = V{};
      if (ci[u] >= 0) z[u] = Ip[(size_t)ci[u] * LPR + lr];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      acc[0] = mad(wv[u], z[u].x, acc[0]);
      acc[1] = mad(wv[u], z[u].y, acc[1]);
      if constexpr (SPL == 2) {
        acc[2] = mad(wv[u], (T)lv_z(z[u]), acc[2]);
        acc[3] = mad(wv[u], (T)lv_w(z[u]), acc[3]);
      }
    }
  }
#pragma unroll
  for (int off = LPR; off < 64; off <<= 1)
#pragma unroll
    for (int c = 0; c < 2 * SPL; ++c) acc[c] += __shfl_xor(acc[c], off);
  if (eg == 0) {
    V o;
    o.x = acc[0];
    o.y = acc[1];
    if constexpr (SPL == 2) lv_set_zw(o, acc[2], acc[3]);
    Op[(size_t)row * LPR + lr] = o;
  }
}

// Restriction of the complex-bfloat16 level-0 residual: as k_restrict, but a
// lane gathers 16 bytes (four systems) of a fine row, four lanes cover the
// row's 16 systems and one wave-wide gather reads 16 fine rows.  (With 8-byte
// gathers, eight lanes per row, the kernel took 20 % longer: its time follows
// the number of gather instructions, not the bytes.)
__global__ __launch_bounds__(kThreads) void k_restrict_h(
    int nout, int nin, const int* __restrict__ rowptr, const int* __restrict__ col,
    const float* __restrict__ v, int npan, const int* __restrict__ active,
    const float2* __restrict__ In, float2* __restrict__ Out) {
  constexpr int LPR = 4;        // lanes per fine row (4 systems each)
  constexpr int EG = 64 / LPR;  // entry groups per wave
  constexpr int U = 4;          // entries per entry group and round
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63, lr = l % LPR, eg = l / LPR;
  // work order as in k_restrict (a contiguous range of (panel group, coarse
  // row) items per XCD)
  const int ngrp = (npan + 3) / 4;
  const long total = (long)nout * ngrp;
  const long per = (total + 7) / 8;
  const long b = blockIdx.x;
  const long t = (b & 7) * per + (b >> 3);
  if (t >= total) return;
  const int row = (int)(t % nout);
  const int pan = (int)(t / nout) * 4 + w;
  if (pan >= npan) return;  // whole waves (no workgroup barrier below)
  const bool a = l < kPanel && (active == nullptr || active[pan * kPanel + l] != 0);
  if (!__any(a)) return;
  // the panel's fine rows: 64 bytes each, as four 16-byte lane vectors
  const uint4* __restrict__ Ih = reinterpret_cast<const uint4*>(In) + (size_t)pan * nin * LPR;
  const int e0 = rowptr[row], e1 = rowptr[row + 1];
  float acc[8];
#pragma unroll
  for (int c = 0; c < 8; ++c) acc[c] = 0.0f;
  for (int e = e0 + eg; e < e1; e += U * EG) {
    int ci[U];
    float wv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int ee = e + u * EG;
      ci[u] = ee < e1 ? col[ee] : -1;
      wv[u] = ee < e1 ? v[ee] : 0.0f;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (ci[u] >= 0) {
        const uint4 h = Ih[(size_t)ci[u] * LPR + lr];
        const float4 z0 = unpack_cbf16x2(make_uint2(h.x, h.y));
        const float4 z1 = unpack_cbf16x2(make_uint2(h.z, h.w));
        acc[0] = fmaf(wv[u], z0.x, acc[0]);
        acc[1] = fmaf(wv[u], z0.y, acc[1]);
        acc[2] = fmaf(wv[u], z0.z, acc[2]);
        acc[3] = fmaf(wv[u], z0.w, acc[3]);
        acc[4] = fmaf(wv[u], z1.x, acc[4]);
        acc[5] = fmaf(wv[u], z1.y, acc[5]);
        acc[6] = fmaf(wv[u], z1.z, acc[6]);
        acc[7] = fmaf(wv[u], z1.w, acc[7]);
      }
    }
  }
#pragma unroll
  for (int off = LPR; off < 64; off <<= 1)
#pragma unroll
    for (int c = 0; c < 8; ++c) acc[c] += __shfl_xor(acc[c], off);
  if (eg == 0) {
    // systems 4 lr .. 4 lr + 3 of the coarse row, as two complex-float pairs
    float4* Op = reinterpret_cast<float4*>(Out + ((size_t)pan * nout + row) * kPanel);
    Op[2 * lr] = make_float4(acc[0], acc[1], acc[2], acc[3]);
    Op[2 * lr + 1] = make_float4(acc[4], acc[5], acc[6], acc[7]);
  }
}

template <typename T>
hipError_t launch_restrict_bf16(const DevTransfer& M, const PanelGrid& g, const SlotTables& st,
                                const void* In, void* Out, hipStream_t s) {
  if (!std::is_same<T, float>::value) return hipErrorInvalidValue;
  const T* v = reinterpret_cast<const T*>(M.v32);
  const long nblk = ((long)M.nrows * ((g.npan + 3) / 4) + 7) / 8 * 8;
  if constexpr (std::is_same<T, float>::value)
    k_restrict_h<<<(unsigned)nblk, kThreads, 0, s>>>(M.nrows, M.ncols, M.rowptr, M.col, v,
                                                     g.npan, st.active,
                                                     static_cast<const float2*>(In),
                                                     static_cast<float2*>(Out));
  return hipGetLastError();
}

template <typename T>
hipError_t launch_transfer(const DevTransfer& M, const PanelGrid& g, const SlotTables& st,
                           const void* In, void* Out, bool add, hipStream_t s) {
  using C = typename CT<T>::t;
  const T* v = std::is_same<T, float>::value ? reinterpret_cast<const T*>(M.v32)
                                             : reinterpret_cast<const T*>(M.v);
  auto Ic = static_cast<const C*>(In);
  auto Oc = static_cast<C*>(Out);
  if (!add && M.nnz > 16 * M.nrows) {
    const long nblk = ((long)M.nrows * ((g.npan + 3) / 4) + 7) / 8 * 8;
    k_restrict<T><<<(unsigned)nblk, kThreads, 0, s>>>(M.nrows, M.ncols, M.rowptr, M.col, v,
                                                      g.npan, st.active, Ic, Oc);
    return hipGetLastError();
  }
  const size_t lbytes = (size_t)M.max_sub64 * (sizeof(T) + sizeof(int));
  if (M.max_sub64 > 0 && lbytes <= 32 * 1024) {
    constexpr int G = 4;
    PanelGrid gg = g;
    const int ncg = (g.npan + G - 1) / G;
    gg.group = ncg < 4 ? ncg : 4;
    const long total = (long)g.nrb * ncg;
    const unsigned blocks = (unsigned)(((total + 7) / 8) * 8);
    if (add)
      k_prolong_lds<T, true, G><<<blocks, kThreads, lbytes, s>>>(
          M.nrows, M.ncols, M.rowptr, M.col, v, gg, M.max_sub64, st.active, Ic, Oc);
    else
      k_prolong_lds<T, false, G><<<blocks, kThreads, lbytes, s>>>(
          M.nrows, M.ncols, M.rowptr, M.col, v, gg, M.max_sub64, st.active, Ic, Oc);
    return hipGetLastError();
  }
  if (add)
    k_prolong<T, true><<<g.blocks(), kThreads, 0, s>>>(M.nrows, M.ncols, M.rowptr, M.col, v, g,
                                                       st.active, Ic, Oc);
  else
    k_prolong<T, false><<<g.blocks(), kThreads, 0, s>>>(M.nrows, M.ncols, M.rowptr, M.col, v,
                                                        g, st.active, Ic, Oc);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_coarse_solve(int nc, const PanelGrid& g, const SlotTables& st, int npoles,
                               const void* Minv, const void* In, void* Out, hipStream_t s) {
  using C = typename CT<T>::t;
  // the slot tables carry the pole-list scratch (npoles <= kMaxPoles at setup)
  if (st.plist == nullptr || st.poff == nullptr || npoles > kMaxPoles) return hipErrorInvalidValue;
  const int nslot = g.npan * kPanel;
  if (nslot == 0) return hipSuccess;
  k_pole_lists<<<1, kThreads, 0, s>>>(nslot, npoles, st.active, st.sys, st.plist, st.poff);
  const int nrt = (nc + kCgRows - 1) / kCgRows;
  const long nblk = (long)npoles * nrt * ((nslot + kCgSlots - 1) / kCgSlots);
  k_coarse_gemm<T><<<(unsigned)nblk, kThreads, 0, s>>>(
      nc, npoles, nrt, st.plist, st.poff, static_cast<const C*>(Minv),
      static_cast<const C*>(In), static_cast<C*>(Out));
  return hipGetLastError();
}

#define SLRF_INST_AMG(T)                                                                       \
  template hipError_t launch_lvl_op<T>(const DevPencil&, const PanelGrid&, const SlotTables&,  \
                                       int, double, const void*, const void*, void*,           \
                                       hipStream_t);                                           \
  template hipError_t launch_lvl_jacobi0<T>(const DevPencil&, const PanelGrid&,                \
                                            const SlotTables&, double, const void*, void*,     \
                                            hipStream_t, bool);                                \
  template hipError_t launch_transfer<T>(const DevTransfer&, const PanelGrid&,                 \
                                         const SlotTables&, const void*, void*, bool,          \
                                         hipStream_t);                                         \
  template hipError_t launch_coarse_solve<T>(int, const PanelGrid&, const SlotTables&, int,    \
                                             const void*, const void*, void*, hipStream_t);   \
  template bool launch_post_image<T>(const DevImage&, const DevPencil&, const PanelGrid&,       \
                                     const SlotTables&, double, const void*, const void*,       \
                                     const void*, void*, hipStream_t, hipError_t&, bool);       \
  template bool launch_resid_bf16<T>(const DevPencil&, const PanelGrid&, const SlotTables&,     \
                                     const void*, const void*, void*, hipStream_t, hipError_t&, \
                                     bool);                                                     \
  template hipError_t launch_restrict_bf16<T>(const DevTransfer&, const PanelGrid&,             \
                                              const SlotTables&, const void*, void*, hipStream_t);
SLRF_INST_AMG(float)
SLRF_INST_AMG(double)


}  // namespace slrf
