// Wave-uniform shifted sweep over row groups (the row-group format of
// ugroup_host.h): q = (A - sigma B) z for a batch of systems in panel layout.
//
// A wave forms R consecutive rows at once for 8 units (a unit is a 128-byte
// column slice of a panel row: a complex-float panel or half a complex-double
// panel), lane l serving unit l / 8 and the 16-byte lane vector l % 8 of it.
// Every lane of the wave walks the same list of the group's distinct columns,
// so the list entries and their coefficients are wave-uniform and come in
// through scalar loads, and each gathered z row (one buffer load per lane
// whose row offset is a scalar) feeds every group row that references it:
// the FMAs of one entry use one z read for up to R rows.  Rows meet their
// entries in increasing column order, the order of the CSR kernels.
#include <type_traits>

#include "internal.h"
#include "ugroup_host.h"

namespace slrf {
namespace {

template <typename T>
struct UG;
template <>
struct UG<float> {
  using V = float4;   // lane vector: two complex-float systems
  using AB = float2;  // (a, b)
  using C = float2;
  static constexpr int SPL = 2, UPP = 1;
};
template <>
struct UG<double> {
  using V = double2;  // one complex-double system
  using AB = double2;
  using C = double2;
  static constexpr int SPL = 1, UPP = 2;
};

constexpr int kUgUnits = 8;         // units per wave
constexpr int kUgWaves = 4;         // waves per workgroup
constexpr int kUgGroupsPerWave = 8; // consecutive groups a wave forms in turn

template <typename T, int SPL, typename V>
__device__ __forceinline__ void ug_fma(T* acc, T a, T b, const V& z) {
  if constexpr (SPL == 2) {
    acc[0] = fmaf(a, z.x, acc[0]);
    acc[1] = fmaf(a, z.y, acc[1]);
    acc[2] = fmaf(b, z.x, acc[2]);
    acc[3] = fmaf(b, z.y, acc[3]);
    acc[4] = fmaf(a, z.z, acc[4]);
    acc[5] = fmaf(a, z.w, acc[5]);
    acc[6] = fmaf(b, z.z, acc[6]);
    acc[7] = fmaf(b, z.w, acc[7]);
  } else {
    acc[0] = fma(a, z.x, acc[0]);
    acc[1] = fma(a, z.y, acc[1]);
    acc[2] = fma(b, z.x, acc[2]);
    acc[3] = fma(b, z.y, acc[3]);
  }
}

// EPI 0: Q = M Z; 1: Q = B - M Z (level residual); 2: Q = Z + omega D^-1 (B - M Z)
// (damped-Jacobi sweep, D = diag M), with M = A - sigma B.
template <typename T, int R, int U, int EPI>
__global__ __launch_bounds__(kUgWaves * 64) void k_sweep_ug(
    int n, int ngroups, const int* __restrict__ gptr, const int* __restrict__ ent,
    const typename UG<T>::AB* __restrict__ uab, int nunit, int npg, long nwork,
    const int* __restrict__ active, const double2* __restrict__ sigma,
    const typename UG<T>::C* __restrict__ Z, typename UG<T>::C* __restrict__ Q,
    const typename UG<T>::C* __restrict__ Bin, const double* __restrict__ da,
    const double* __restrict__ db, double omega) {
  using V = typename UG<T>::V;
  using AB = typename UG<T>::AB;
  using Cx = typename UG<T>::C;
  constexpr int SPL = UG<T>::SPL, UPP = UG<T>::UPP;
  constexpr int LPR = kPanel / SPL;                     // lane vectors per panel row
  constexpr unsigned ROWB = kPanel * sizeof(Cx);        // bytes per panel row
  constexpr int CMASK = (1 << kUGroupMaskShift) - 1;
  // work item (chunk of groups, run of kUgWaves panel groups): the waves of a
  // workgroup form the same groups for different panel groups, so a chunk's
  // entries and coefficients are fetched once per compute unit
  const long per = (nwork + 7) / 8;
  const long t = (long)(blockIdx.x & 7) * per + (blockIdx.x >> 3);
  if (t >= nwork) return;
  const int npgw = (npg + kUgWaves - 1) / kUgWaves;
  const int chunk = (int)(t / npgw);
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int pg = (int)(t % npgw) * kUgWaves + w;
  if (pg >= npg) return;
  const int lane = threadIdx.x & 63;
  const int u = lane >> 3, lv = lane & 7;
  const int unit = pg * kUgUnits + u;
  const bool uok = unit < nunit;
  const int ucl = uok ? unit : pg * kUgUnits;  // an existing unit for the loads
  const int panel = ucl / UPP, half = ucl % UPP;
  const int sys0 = panel * kPanel + half * (kPanel / UPP) + lv * SPL;
  bool act = uok;
  if (active != nullptr && uok) {
    act = false;
#pragma unroll
    for (int q = 0; q < SPL; ++q) act |= active[sys0 + q] != 0;
  }
  if (__ballot(act) == 0) return;  // (wave-uniform: no active system in the wave)
  const int g0 = chunk * kUgGroupsPerWave;
  const int g1 = min(g0 + kUgGroupsPerWave, ngroups);
  if (g0 >= g1) return;
  const int npan = (nunit + UPP - 1) / UPP;
  const int pan0 = (pg * kUgUnits) / UPP;
  const char* zbase = reinterpret_cast<const char*>(Z) + (size_t)pan0 * n * ROWB;
  const size_t zbytes = (size_t)(npan - pan0) * n * ROWB;
  const __amdgpu_buffer_rsrc_t rsrc = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<char*>(zbase), (short)0, (int)(zbytes < 0xFFFFFFFFull ? zbytes : 0xFFFFFFFFull),
      0x00020000);
  const unsigned voff = (unsigned)((size_t)(panel - pan0) * n * ROWB) + half * 128u + lv * 16u;
  T sr[SPL], si[SPL];
#pragma unroll
  for (int q = 0; q < SPL; ++q) {
    const double2 sg = sigma[sys0 + q];
    sr[q] = (T)sg.x;
    si[q] = (T)sg.y;
  }
  V* __restrict__ Ql = reinterpret_cast<V*>(Q) + (size_t)panel * n * LPR + half * 8 + lv;
  T acc[R][4 * SPL];
#pragma unroll
  for (int r = 0; r < R; ++r)
#pragma unroll
    for (int v = 0; v < 4 * SPL; ++v) acc[r][v] = 0;
  // software pipeline over the chunks of U entries of groups g0 .. g1 - 1:
  // entries two chunks ahead and coefficients one chunk ahead (scalar loads),
  // z one chunk ahead (buffer loads); the entry arrays carry two chunks of
  // padding past the last group, so the look-ahead loads stay in bounds
  int e = gptr[g0];
  const int eend = gptr[g1];
  int gcur = g0, gbnd = gptr[g0 + 1];
  int en0[U], en1[U], en2[U];
  AB ab0[U][R], ab1[U][R];
  V z0[U], z1[U];
#pragma unroll
  for (int uu = 0; uu < U; ++uu) {
    en0[uu] = ent[e + uu];
    en1[uu] = ent[e + U + uu];
  }
#pragma unroll
  for (int uu = 0; uu < U; ++uu)
#pragma unroll
    for (int r = 0; r < R; ++r) ab0[uu][r] = uab[(size_t)(e + uu) * R + r];
#pragma unroll
  for (int uu = 0; uu < U; ++uu)
    z0[uu] = __builtin_bit_cast(
        V, __builtin_amdgcn_raw_buffer_load_b128(rsrc, voff, (unsigned)(en0[uu] & CMASK) * ROWB,
                                                 0));
  for (; e < eend; e += U) {
    // next chunk's z, the chunk after it's entries, next chunk's coefficients
#pragma unroll
    for (int uu = 0; uu < U; ++uu)
      z1[uu] = __builtin_bit_cast(
          V, __builtin_amdgcn_raw_buffer_load_b128(rsrc, voff,
                                                   (unsigned)(en1[uu] & CMASK) * ROWB, 0));
#pragma unroll
    for (int uu = 0; uu < U; ++uu) en2[uu] = ent[e + 2 * U + uu];
#pragma unroll
    for (int uu = 0; uu < U; ++uu)
#pragma unroll
      for (int r = 0; r < R; ++r) ab1[uu][r] = uab[(size_t)(e + U + uu) * R + r];
#pragma unroll
    for (int uu = 0; uu < U; ++uu)
#pragma unroll
      for (int r = 0; r < R; ++r)
        if ((en0[uu] >> (kUGroupMaskShift + r)) & 1)
          ug_fma<T, SPL>(acc[r], ab0[uu][r].x, ab0[uu][r].y, z0[uu]);
    if (e + U == gbnd) {
      // group gcur complete: write its rows, start the next group
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int row = gcur * R + r;
        if (row < n && uok) {
          V q;
          q.x = acc[r][0] - (sr[0] * acc[r][2] - si[0] * acc[r][3]);
          q.y = acc[r][1] - (sr[0] * acc[r][3] + si[0] * acc[r][2]);
          if constexpr (SPL == 2) {
            q.z = acc[r][4] - (sr[1] * acc[r][6] - si[1] * acc[r][7]);
            q.w = acc[r][5] - (sr[1] * acc[r][7] + si[1] * acc[r][6]);
          }
          if constexpr (EPI != 0) {
            const size_t li = ((size_t)panel * n + row) * LPR + half * 8 + lv;
            const V bb = reinterpret_cast<const V*>(Bin)[li];
            q.x = bb.x - q.x;  // b - M x
            q.y = bb.y - q.y;
            if constexpr (SPL == 2) {
              q.z = bb.z - q.z;
              q.w = bb.w - q.w;
            }
            if constexpr (EPI == 2) {
              const V xo = reinterpret_cast<const V*>(Z)[li];
              const double dav = da[row], dbv = db[row];
              T ov[2 * SPL] = {xo.x, xo.y};
              T rv[2 * SPL] = {q.x, q.y};
              if constexpr (SPL == 2) {
                ov[2] = xo.z; ov[3] = xo.w; rv[2] = q.z; rv[3] = q.w;
              }
              T nv[2 * SPL];
#pragma unroll
              for (int c = 0; c < SPL; ++c) {
                const double dx = dav - (double)sr[c] * dbv, dy = -(double)si[c] * dbv;
                const double iv = omega / (dx * dx + dy * dy);
                const double ix = dx * iv, iy = -dy * iv;  // omega / d
                const double rx = rv[2 * c], ry = rv[2 * c + 1];
                nv[2 * c] = (T)((double)ov[2 * c] + rx * ix - ry * iy);
                nv[2 * c + 1] = (T)((double)ov[2 * c + 1] + rx * iy + ry * ix);
              }
              q.x = nv[0];
              q.y = nv[1];
              if constexpr (SPL == 2) {
                q.z = nv[2];
                q.w = nv[3];
              }
            }
          }
          Ql[(size_t)row * LPR] = q;
        }
#pragma unroll
        for (int v = 0; v < 4 * SPL; ++v) acc[r][v] = 0;
      }
      ++gcur;
      gbnd = gcur < g1 ? gptr[gcur + 1] : eend;
    }
#pragma unroll
    for (int uu = 0; uu < U; ++uu) {
      en0[uu] = en1[uu];
      en1[uu] = en2[uu];
      z0[uu] = z1[uu];
#pragma unroll
      for (int r = 0; r < R; ++r) ab0[uu][r] = ab1[uu][r];
    }
  }
}

}  // namespace

template <typename T>
bool ugroup_selected(const DevPencil& P) {
  const int var = std::is_same<T, float>::value ? P.var32 : P.var64;
  // (buffer offsets are 32-bit: a wave's panels span at most 8 n 128 bytes)
  return var == kSpmmUGroup && P.ug_ngroups > 0 && P.ug_R == 4 && P.n < (1 << 22);
}

template <typename T>
bool launch_ugroup(const DevPencil& P, const PanelGrid& g, const SlotTables& st, int epi,
                   double omega, const void* Z, const void* Bin, void* Out, hipStream_t s,
                   hipError_t& err) {
  if (!ugroup_selected<T>(P) || epi < 0 || epi > 2) return false;
  constexpr int UPP = UG<T>::UPP;
  const int nunit = g.npan * UPP;
  const int npg = (nunit + kUgUnits - 1) / kUgUnits;
  const long nchunk = (P.ug_ngroups + kUgGroupsPerWave - 1) / kUgGroupsPerWave;
  const long nwork = nchunk * ((npg + kUgWaves - 1) / kUgWaves);
  const unsigned blocks = (unsigned)(((nwork + 7) / 8) * 8);
  using AB = typename UG<T>::AB;
  const AB* ab;
  if constexpr (std::is_same<T, float>::value) ab = P.ug_ab32; else ab = P.ug_ab64;
  using Cx = typename UG<T>::C;
#define SLRF_UG(E)                                                                          \
  k_sweep_ug<T, 4, 4, E><<<blocks, kUgWaves * 64, 0, s>>>(                                   \
      P.n, P.ug_ngroups, P.ug_gptr, P.ug_ent, ab, nunit, npg, nwork, st.active, st.sigma,    \
      static_cast<const Cx*>(Z), static_cast<Cx*>(Out), static_cast<const Cx*>(Bin), P.da,  \
      P.db, omega)
  if (epi == 0)
    SLRF_UG(0);
  else if (epi == 1)
    SLRF_UG(1);
  else
    SLRF_UG(2);
#undef SLRF_UG
  err = hipGetLastError();
  return true;
}

template bool ugroup_selected<float>(const DevPencil&);
template bool ugroup_selected<double>(const DevPencil&);
template bool launch_ugroup<float>(const DevPencil&, const PanelGrid&, const SlotTables&, int,
                                   double, const void*, const void*, void*, hipStream_t,
                                   hipError_t&);
template bool launch_ugroup<double>(const DevPencil&, const PanelGrid&, const SlotTables&, int,
                                    double, const void*, const void*, void*, hipStream_t,
                                    hipError_t&);

}  // namespace slrf
