// Device products of one smoothed-aggregation level: rho(D^-1 A), A T, the
// smoothed prolongator P, R = P^T, A P and B P, and the Galerkin products
// R (A P), R (B P).  Built without floating-point contraction (a product is
// rounded before it is added, as in the host code), with every sum in the host
// code's order, so the values equal the host's bit for bit.
#include "amg_device.h"

#include <hipcub/hipcub.hpp>

#include <chrono>
#include <climits>
#include <cmath>
#include <vector>

namespace slrf {
namespace {

constexpr int kHS = 2 * kAmgRowCap;  // hash slots of one output row
constexpr int kHSBits = 11;
static_assert((1 << kHSBits) == kHS, "hash table size");

__device__ __forceinline__ int hslot(int col) {
  return (int)(((unsigned)col * 2654435761u) >> (32 - kHSBits));
}

// Inserts col into a row's table (linear probing); true when it was new.
// A full table sets *ovf (probing is bounded by the table size).
__device__ bool hinsert(int* keys, int col, int* ovf) {
  int h = hslot(col);
  for (int probe = 0; probe < kHS; ++probe) {
    const int old = atomicCAS(&keys[h], -1, col);
    if (old == -1) return true;
    if (old == col) return false;
    h = (h + 1) & (kHS - 1);
  }
  atomicExch(ovf, 1);
  return false;
}

__device__ int hfind(const int* keys, int col) {
  int h = hslot(col);
  for (int probe = 0; probe < kHS; ++probe) {
    const int k = keys[h];
    if (k == col || k == -1) return k == col ? h : -1;
    h = (h + 1) & (kHS - 1);
  }
  return -1;
}

__global__ void k_fill_int(int* v, int m, int val) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < m) v[t] = val;
}

// d_i = a_ii (1 where the row stores no diagonal)
__global__ void k_diag_a(int n, const int* __restrict__ rp, const int* __restrict__ ci,
                         const double* __restrict__ a, double* __restrict__ d) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double v = 1.0;
  for (int e = rp[i]; e < rp[i + 1]; ++e)
    if (ci[e] == i) v = a[e];
  d[i] = v;
}

// y = D^-1 A x (each row summed in CSR order)
__global__ void k_dinv_a(int n, const int* __restrict__ rp, const int* __restrict__ ci,
                         const double* __restrict__ a, const double* __restrict__ d,
                         const double* __restrict__ x, double* __restrict__ y) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double s = 0.0;
  for (int e = rp[i]; e < rp[i + 1]; ++e) s += a[e] * x[ci[e]];
  y[i] = s / d[i];
}

// ||y||^2 summed in row order (one thread: the host code's order)
__global__ void k_norm2_ordered(int n, const double* __restrict__ y, double* __restrict__ out) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  double s = 0.0;
  for (int i = 0; i < n; ++i) s += y[i] * y[i];
  *out = s;
}

__global__ void k_scale_div(int n, const double* __restrict__ y, double r, double* __restrict__ x) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] = y[i] / r;
}

// Distinct columns of each row of X Y, one wavefront per row.  A row with more
// than kAmgRowCap of them gets count 0 and raises *flag.
__global__ __launch_bounds__(64) void k_spgemm_count(int nrows, const int* __restrict__ xrp,
                                                     const int* __restrict__ xci,
                                                     const int* __restrict__ yrp,
                                                     const int* __restrict__ yci,
                                                     int* __restrict__ cnt, int* __restrict__ flag) {
  __shared__ int keys[kHS];
  __shared__ int nk, ovf;
  const int i = blockIdx.x, lane = threadIdx.x;
  if (i >= nrows) return;
  for (int t = lane; t < kHS; t += 64) keys[t] = -1;
  if (lane == 0) {
    nk = 0;
    ovf = 0;
  }
  __syncthreads();
  for (int e = xrp[i]; e < xrp[i + 1]; ++e) {
    const int k = xci[e];
    for (int f = yrp[k] + lane; f < yrp[k + 1]; f += 64)
      if (hinsert(keys, yci[f], &ovf)) atomicAdd(&nk, 1);
  }
  __syncthreads();
  if (lane == 0) {
    const bool bad = ovf != 0 || nk > kAmgRowCap;
    cnt[i] = bad ? 0 : nk;
    if (bad) atomicExch(flag, 1);
  }
}

// X Y row by row, one wavefront per row: the row's distinct columns sorted
// (bitonic, in LDS), then its values summed in Gustavson order: X's entries
// in order, each one's Y row in order, every product rounded before it is
// added.  The lanes form 64 products and their output positions at a time;
// one lane adds them in order.  MODE 0: c1 = x1 y1; 1: c1 = x1 y1, c2 = x2 y1;
// 2: c1 = x1 y1, c2 = x1 y2.
template <int MODE>
__global__ __launch_bounds__(64) void k_spgemm_fill(
    int nrows, const int* __restrict__ xrp, const int* __restrict__ xci,
    const double* __restrict__ x1, const double* __restrict__ x2, const int* __restrict__ yrp,
    const int* __restrict__ yci, const double* __restrict__ y1, const double* __restrict__ y2,
    const int* __restrict__ crp, int* __restrict__ cci, double* __restrict__ c1,
    double* __restrict__ c2) {
  __shared__ int keys[kHS];
  __shared__ int pos[kHS];
  __shared__ int list[kAmgRowCap];
  __shared__ double a1[kAmgRowCap], a2[kAmgRowCap];
  __shared__ int cp[64];
  __shared__ double p1[64], p2[64];
  __shared__ int nk, ovf;
  const int i = blockIdx.x, lane = threadIdx.x;
  if (i >= nrows) return;
  for (int t = lane; t < kHS; t += 64) keys[t] = -1;
  if (lane == 0) {
    nk = 0;
    ovf = 0;
  }
  __syncthreads();
  for (int e = xrp[i]; e < xrp[i + 1]; ++e) {
    const int k = xci[e];
    for (int f = yrp[k] + lane; f < yrp[k + 1]; f += 64) {
      const int col = yci[f];
      if (hinsert(keys, col, &ovf)) {
        const int q = atomicAdd(&nk, 1);
        if (q < kAmgRowCap) list[q] = col;
      }
    }
  }
  __syncthreads();
  const int U = nk;
  if (ovf != 0 || U > kAmgRowCap) return;  // (flagged by the count pass)
  int P2 = 1;
  while (P2 < U) P2 <<= 1;
  for (int t = U + lane; t < P2; t += 64) list[t] = INT_MAX;
  __syncthreads();
  for (int size = 2; size <= P2; size <<= 1)
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int t = lane; t < P2 / 2; t += 64) {
        const int lo = 2 * t - (t & (stride - 1)), hi = lo + stride;
        const bool up = (lo & size) == 0;
        const int va = list[lo], vb = list[hi];
        if ((va > vb) == up) {
          list[lo] = vb;
          list[hi] = va;
        }
      }
      __syncthreads();
    }
  const int base = crp[i];
  for (int t = lane; t < U; t += 64) {
    const int col = list[t];
    cci[base + t] = col;
    pos[hfind(keys, col)] = t;
    a1[t] = 0.0;
    a2[t] = 0.0;
  }
  __syncthreads();
  for (int e = xrp[i]; e < xrp[i + 1]; ++e) {
    const int k = xci[e];
    const double xv1 = x1[e];
    const double xv2 = MODE == 1 ? x2[e] : 0.0;
    const int fe = yrp[k + 1];
    for (int f0 = yrp[k]; f0 < fe; f0 += 64) {
      const int f = f0 + lane;
      if (f < fe) {
        cp[lane] = pos[hfind(keys, yci[f])];
        const double yv1 = y1[f];
        p1[lane] = xv1 * yv1;
        if (MODE == 1) p2[lane] = xv2 * yv1;
        if (MODE == 2) p2[lane] = xv1 * y2[f];
      }
      __syncthreads();
      if (lane == 0) {
        const int m = min(64, fe - f0);
        for (int t = 0; t < m; ++t) {
          a1[cp[t]] += p1[t];
          if (MODE != 0) a2[cp[t]] += p2[t];
        }
      }
      __syncthreads();
    }
  }
  for (int t = lane; t < U; t += 64) {
    c1[base + t] = a1[t];
    if (MODE != 0) c2[base + t] = a2[t];
  }
}

// P = T - w D^-1 A T on the pattern of A T (T's entry added where its column
// occurs): the host code's expression for every entry
__global__ void k_form_p(int n, const int* __restrict__ arp, const int* __restrict__ aci,
                         const double* __restrict__ at, const int* __restrict__ trp,
                         const int* __restrict__ tci, const double* __restrict__ tv,
                         const double* __restrict__ d, double w, double* __restrict__ pv) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int f = trp[i];
  for (int e = arp[i]; e < arp[i + 1]; ++e) {
    double v = -w * at[e] / d[i];
    while (f < trp[i + 1] && tci[f] < aci[e]) ++f;
    if (f < trp[i + 1] && tci[f] == aci[e]) v += tv[f];
    pv[e] = v;
  }
}

__global__ void k_entry_rows(int n, const int* __restrict__ rp, int* __restrict__ row) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (int e = rp[i]; e < rp[i + 1]; ++e) row[e] = i;
}

__global__ void k_iota(int m, int* __restrict__ v) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < m) v[t] = t;
}

__global__ void k_count_cols(int nnz, const int* __restrict__ ci, int* __restrict__ cnt) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < nnz) atomicAdd(&cnt[ci[t]], 1);
}

__global__ void k_gather_transpose(int nnz, const int* __restrict__ perm,
                                   const int* __restrict__ row, const double* __restrict__ v,
                                   int* __restrict__ tci, double* __restrict__ tv) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nnz) return;
  const int e = perm[t];
  tci[t] = row[e];
  tv[t] = v[e];
}

inline unsigned blocks_of(long m, int b) { return (unsigned)((m + b - 1) / b); }

// A device CSR matrix with one or two value arrays.
struct DCsr {
  int n = 0, m = 0, nnz = 0;
  int* rp = nullptr;
  int* ci = nullptr;
  double* v1 = nullptr;
  double* v2 = nullptr;
};

struct Builder {
  DeviceAmgNumeric& num;
  std::string& err;
  hipStream_t s;
  size_t taken = 0;

  template <typename T>
  T* take(size_t count) {
    const size_t bytes = std::max<size_t>(count, 1) * sizeof(T);
    void* p = num.take(bytes);
    if (!p) {
      err = "workspace too small for the device AMG setup";
      return nullptr;
    }
    taken += (bytes + 255) / 256 * 256;
    return static_cast<T*>(p);
  }
  template <typename T>
  T* up(const std::vector<T>& v) {
    T* p = take<T>(v.size());
    if (p && !v.empty() &&
        hipMemcpyAsync(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s) != hipSuccess) {
      err = "upload failed";
      return nullptr;
    }
    return p;
  }
  template <typename T>
  bool down(std::vector<T>& v, const T* p, size_t count) {
    v.resize(count);
    if (count == 0) return true;
    if (hipMemcpyAsync(v.data(), p, count * sizeof(T), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) {
      err = "download failed";
      return false;
    }
    return true;
  }
  bool ok(hipError_t e, const char* what) {
    if (e == hipSuccess) e = hipGetLastError();
    if (e != hipSuccess) {
      err = std::string(what) + ": " + hipGetErrorString(e);
      return false;
    }
    return true;
  }

  // exclusive prefix sums of cnt[0 .. m] into out[0 .. m] (cnt[m] = 0)
  bool scan(const int* cnt, int* out, int m) {
    size_t tb = 0;
    if (!ok(hipcub::DeviceScan::ExclusiveSum(nullptr, tb, cnt, out, m + 1, s), "scan size"))
      return false;
    void* tmp = take<char>(tb);
    if (!tmp) return false;
    return ok(hipcub::DeviceScan::ExclusiveSum(tmp, tb, cnt, out, m + 1, s), "scan");
  }

  // C = X Y; mode as k_spgemm_fill
  bool spgemm(const DCsr& X, const DCsr& Y, int mode, DCsr& C) {
    C = DCsr();
    C.n = X.n;
    C.m = Y.m;
    int* cnt = take<int>((size_t)X.n + 1);
    int* flag = take<int>(1);
    C.rp = take<int>((size_t)X.n + 1);
    if (!cnt || !flag || !C.rp) return false;
    k_fill_int<<<blocks_of(X.n + 1, 256), 256, 0, s>>>(cnt, X.n + 1, 0);
    k_fill_int<<<1, 64, 0, s>>>(flag, 1, 0);
    if (X.n > 0)
      k_spgemm_count<<<X.n, 64, 0, s>>>(X.n, X.rp, X.ci, Y.rp, Y.ci, cnt, flag);
    if (!ok(hipSuccess, "product count") || !scan(cnt, C.rp, X.n)) return false;
    int hv[2] = {0, 0};
    if (!ok(hipMemcpyAsync(&hv[0], flag, sizeof(int), hipMemcpyDeviceToHost, s), "flag") ||
        !ok(hipMemcpyAsync(&hv[1], C.rp + X.n, sizeof(int), hipMemcpyDeviceToHost, s), "nnz") ||
        !ok(hipStreamSynchronize(s), "sync"))
      return false;
    if (hv[0] != 0) {
      err = "a product row has more than " + std::to_string(kAmgRowCap) + " distinct columns";
      return false;
    }
    C.nnz = hv[1];
    C.ci = take<int>(C.nnz);
    C.v1 = take<double>(C.nnz);
    if (mode != 0) C.v2 = take<double>(C.nnz);
    if (!C.ci || !C.v1 || (mode != 0 && !C.v2)) return false;
    if (X.n > 0) {
      if (mode == 0)
        k_spgemm_fill<0><<<X.n, 64, 0, s>>>(X.n, X.rp, X.ci, X.v1, nullptr, Y.rp, Y.ci, Y.v1,
                                            nullptr, C.rp, C.ci, C.v1, nullptr);
      else if (mode == 1)
        k_spgemm_fill<1><<<X.n, 64, 0, s>>>(X.n, X.rp, X.ci, X.v1, X.v2, Y.rp, Y.ci, Y.v1,
                                            nullptr, C.rp, C.ci, C.v1, C.v2);
      else
        k_spgemm_fill<2><<<X.n, 64, 0, s>>>(X.n, X.rp, X.ci, X.v1, nullptr, Y.rp, Y.ci, Y.v1,
                                            Y.v2, C.rp, C.ci, C.v1, C.v2);
    }
    return ok(hipSuccess, "product fill");
  }

  // T = M^T for an n x m matrix M (one value array): rows of T list M's rows
  // in increasing order (a stable sort of the entries by column)
  bool transpose(const DCsr& M, DCsr& T) {
    T = DCsr();
    T.n = M.m;
    T.m = M.n;
    T.nnz = M.nnz;
    int* row = take<int>(M.nnz);
    int* idx = take<int>(M.nnz);
    int* perm = take<int>(M.nnz);
    int* keys = take<int>(M.nnz);
    int* cnt = take<int>((size_t)M.m + 1);
    T.rp = take<int>((size_t)M.m + 1);
    T.ci = take<int>(M.nnz);
    T.v1 = take<double>(M.nnz);
    if (!row || !idx || !perm || !keys || !cnt || !T.rp || !T.ci || !T.v1) return false;
    k_fill_int<<<blocks_of(M.m + 1, 256), 256, 0, s>>>(cnt, M.m + 1, 0);
    if (M.n > 0) k_entry_rows<<<blocks_of(M.n, 256), 256, 0, s>>>(M.n, M.rp, row);
    if (M.nnz > 0) {
      k_iota<<<blocks_of(M.nnz, 256), 256, 0, s>>>(M.nnz, idx);
      k_count_cols<<<blocks_of(M.nnz, 256), 256, 0, s>>>(M.nnz, M.ci, cnt);
    }
    if (!ok(hipSuccess, "transpose count") || !scan(cnt, T.rp, M.m)) return false;
    if (M.nnz == 0) return true;
    int bits = 1;
    while ((1L << bits) <= M.m) ++bits;
    size_t tb = 0;
    if (!ok(hipcub::DeviceRadixSort::SortPairs(nullptr, tb, M.ci, keys, idx, perm, M.nnz, 0, bits,
                                               s),
            "sort size"))
      return false;
    void* tmp = take<char>(tb);
    if (!tmp ||
        !ok(hipcub::DeviceRadixSort::SortPairs(tmp, tb, M.ci, keys, idx, perm, M.nnz, 0, bits, s),
            "sort"))
      return false;
    k_gather_transpose<<<blocks_of(M.nnz, 256), 256, 0, s>>>(M.nnz, perm, row, M.v1, T.ci, T.v1);
    return ok(hipSuccess, "transpose gather");
  }

  bool download(const DCsr& M, std::vector<int>& rp, std::vector<int>& ci, std::vector<double>& v1,
                std::vector<double>* v2) {
    return down(rp, M.rp, (size_t)M.n + 1) && down(ci, M.ci, M.nnz) && down(v1, M.v1, M.nnz) &&
           (v2 == nullptr || down(*v2, M.v2, M.nnz));
  }
};

}  // namespace

bool DeviceAmgNumeric::level(const HostLevel& L, int nc, const std::vector<int>& trp,
                             const std::vector<int>& tci, const std::vector<double>& tv,
                             double omega_p, double& rho, HostCsrP& P, HostCsrP& R,
                             HostLevel& APBP, HostLevel& C, std::string& err) {
  const auto t0 = std::chrono::steady_clock::now();
  Builder b{*this, err, stream};
  bool good = [&]() -> bool {
    const int n = L.n;
    DCsr A;
    A.n = n;
    A.m = n;
    A.nnz = (int)L.ci.size();
    A.rp = b.up(L.rp);
    A.ci = b.up(L.ci);
    A.v1 = b.up(L.a);
    A.v2 = b.up(L.b);
    DCsr T;
    T.n = n;
    T.m = nc;
    T.nnz = (int)tci.size();
    T.rp = b.up(trp);
    T.ci = b.up(tci);
    T.v1 = b.up(tv);
    double* d = b.take<double>(n);
    double* x = b.up(rho_start_vector(n));
    double* y = b.take<double>(n);
    double* nrm = b.take<double>(1);
    if (!A.rp || !A.ci || !A.v1 || !A.v2 || !T.rp || !T.ci || !T.v1 || !d || !x || !y || !nrm)
      return false;
    k_diag_a<<<blocks_of(n, 256), 256, 0, stream>>>(n, A.rp, A.ci, A.v1, d);
    // rho(D^-1 A): 20 power steps, the norm's square root and the scaling
    // factor taken on the host as in the host code
    rho = 1.0;
    bool degenerate = false;
    for (int it = 0; it < 20 && !degenerate; ++it) {
      k_dinv_a<<<blocks_of(n, 256), 256, 0, stream>>>(n, A.rp, A.ci, A.v1, d, x, y);
      k_norm2_ordered<<<1, 64, 0, stream>>>(n, y, nrm);
      double h2 = 0.0;
      if (!b.ok(hipMemcpyAsync(&h2, nrm, sizeof(double), hipMemcpyDeviceToHost, stream), "norm") ||
          !b.ok(hipStreamSynchronize(stream), "norm sync"))
        return false;
      rho = std::sqrt(h2);
      if (!(rho > 0.0)) {
        rho = 1.0;
        degenerate = true;
        break;
      }
      k_scale_div<<<blocks_of(n, 256), 256, 0, stream>>>(n, y, rho, x);
    }
    DCsr AT, Pd, Rd, AB, Cd;
    if (!b.spgemm(DCsr{n, n, A.nnz, A.rp, A.ci, A.v1, nullptr}, T, 0, AT)) return false;
    const double w = omega_p / rho;
    Pd = AT;
    Pd.v1 = b.take<double>(AT.nnz);
    if (!Pd.v1) return false;
    k_form_p<<<blocks_of(n, 256), 256, 0, stream>>>(n, AT.rp, AT.ci, AT.v1, T.rp, T.ci, T.v1, d, w,
                                                    Pd.v1);
    if (!b.ok(hipSuccess, "prolongator")) return false;
    if (!b.transpose(Pd, Rd)) return false;
    if (!b.spgemm(A, Pd, 1, AB)) return false;
    if (!b.spgemm(Rd, AB, 2, Cd)) return false;
    P = HostCsrP();
    P.n = n;
    P.m = nc;
    R = HostCsrP();
    R.n = nc;
    R.m = n;
    APBP = HostLevel();
    APBP.n = n;
    C = HostLevel();
    C.n = nc;
    return b.download(Pd, P.rp, P.ci, P.v, nullptr) && b.download(Rd, R.rp, R.ci, R.v, nullptr) &&
           b.download(AB, APBP.rp, APBP.ci, APBP.a, &APBP.b) &&
           b.download(Cd, C.rp, C.ci, C.a, &C.b);
  }();
  peak_bytes = std::max(peak_bytes, b.taken);
  if (release) release();
  seconds += std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  return good;
}

}  // namespace slrf
