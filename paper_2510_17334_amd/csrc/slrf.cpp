// C ABI and host orchestration of the MI355X rational-filter eigensolver.
//
// slrf_filter runs every (pole, column) shifted system of Eq. (2) through a
// resident pool of "slots" on the GPU.  Systems enter the pool in order
// s = c * N + j, iterate in Krylov cycles (restarted GCR, Section 3.2), and at
// each cycle boundary the host (a) folds the cycle's directions into the FP64
// solution, (b) recomputes the FP64 true residual, (c) retires converged or
// capped systems to the per-system solution store, (d) compacts the survivors
// to the front of the pool and admits waiting systems into the freed slots.
// The mixed-precision form runs the cycles in complex FP32 and is otherwise the
// same loop: the boundary steps are the FP64 iterative-refinement steps.
// Host <-> device traffic inside a filter call is limited to per-slot flags.
#include "slrf.h"

#include <algorithm>
#include <atomic>
#include <chrono>
#include <numeric>
#include <thread>
#include <map>
#include <memory>
#include <mutex>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "amg_device.h"
#include "amg_host.h"
#include "halo_host.h"
#include "ugroup_host.h"
#include "dense_host.h"
#include "internal.h"

using namespace slrf;

namespace {

struct Timer {
  std::vector<hipEvent_t> pool;
  struct Rec {
    int cls;
    hipEvent_t a, b;
  };
  std::vector<Rec> pending;
  size_t used = 0;
  hipEvent_t get() {
    if (used == pool.size()) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) return nullptr;
      pool.push_back(e);
    }
    return pool[used++];
  }
  void reset() {
    pending.clear();
    used = 0;
  }
  ~Timer() {
    for (auto e : pool) (void)hipEventDestroy(e);
  }
};

}  // namespace

// Device copy of the AMG hierarchy (levels >= 1; level 0 is the pencil).
struct DevAmg {
  bool ready = false;
  std::vector<DevPencil> lv;            // levels 1 .. L-1
  std::vector<DevTransfer> P, R;        // P[l]: n_l x n_{l+1}, R[l] = P[l]^T
  std::vector<int> n;                   // level sizes, n[0] = fine
  int nc = 0;                           // coarsest size
  void* inv64 = nullptr;                // [pole][nc][nc] complex double
  void* inv32 = nullptr;                // [pole][nc][nc] complex float
  std::vector<double> omega;            // Jacobi smoothing weight per level (all but the coarsest)
  std::vector<DevImage> img;            // img[l]: image (A_l P_l, B_l P_l) for the fused
                                        // up-step of level l (ntile 0 if absent)
  size_t nnz_all = 0;                   // level + transfer nonzeros (byte accounting)
};

// The caller's workspace: persistent pencil data at the bottom (placed by
// setup), then a stack of per-call buffers (each entry point releases what it
// carved).  The library never allocates device memory itself.
struct Arena {
  char* base = nullptr;
  size_t cap = 0;       // bytes
  size_t top = 0;       // first free byte
  size_t persist = 0;   // end of the persistent data
  size_t short_by = 0;  // after a failed carve: bytes missing
};

struct slrf_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  DevPencil P;
  double gamma = 0.0;
  int N = 0;
  std::vector<double2> poles, weights;
  slrf_options opt{};
  std::string err;
  // persistent arrays inside the workspace
  float* a32 = nullptr;
  float* b32 = nullptr;
  double* da = nullptr;
  double* db = nullptr;
  double2* d_w = nullptr;
  // locality row order (the permuted pencil is kept in the workspace); order[new] = old
  int* order = nullptr;
  std::vector<int> h_order;
  int block = 0;  // dofs per node
  Arena ar;
  std::vector<int> h_flags;  // host mirror of per-slot flags
  // byte accounting of a Krylov cycle: its kernels are counted with the
  // systems active at the cycle start; the per-system terms are settled at the
  // next boundary from the steps each system actually took (active steps
  // form a prefix of the cycle)
  struct Deferred {
    int cls, k;
    double per_sys;
    bool sweep;
  };
  std::vector<Deferred> defer;
  int defer_k = -1;  // step of the cycle being issued (-1: outside a cycle)
  Timer timer;
  slrf_filter_stats* cur_stats = nullptr;
  DevAmg amg;
};

namespace {

#define HIPCHK(x)                                                     \
  do {                                                                \
    hipError_t e_ = (x);                                              \
    if (e_ != hipSuccess) return fail_hip(h, e_, #x, __LINE__);       \
  } while (0)

slrf_status fail(slrf_ctx* h, slrf_status s, const std::string& msg) {
  if (h) h->err = msg;
  return s;
}

slrf_status fail_hip(slrf_ctx* h, hipError_t e, const char* what, int line) {
  char buf[512];
  if (e == hipErrorOutOfMemory && h && h->ar.short_by > 0) {
    std::snprintf(buf, sizeof(buf),
                  "workspace of %zu bytes too small: %s needs %zu more bytes (slrf.cpp:%d)",
                  h->ar.cap, what, h->ar.short_by, line);
    h->ar.short_by = 0;
  } else {
    std::snprintf(buf, sizeof(buf), "HIP error %d (%s) in %s at slrf.cpp:%d", (int)e,
                  hipGetErrorString(e), what, line);
  }
  if (h) h->err = buf;
  return e == hipErrorOutOfMemory ? SLRF_E_NOMEM : SLRF_E_HIP;
}

// automatic It_max-linear: this fraction of the median iterations of the
// first outer iteration's solves, at least kAutoItMaxMin
constexpr double kAutoItMaxFrac = 0.5;
constexpr int kAutoItMaxMin = 3;

constexpr size_t kAlign = 256;
inline size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// Carve `bytes` from the top of the workspace (256-byte aligned).
hipError_t carve(slrf_ctx* h, size_t bytes, void** out) {
  Arena& A = h->ar;
  const size_t off = align_up(A.top);
  const size_t need = align_up(std::max<size_t>(bytes, 1));
  if (off + need > A.cap) {
    A.short_by = off + need - A.cap;
    *out = nullptr;
    return hipErrorOutOfMemory;
  }
  *out = A.base + off;
  A.top = off + need;
  return hipSuccess;
}

template <typename P>
hipError_t carve_t(slrf_ctx* h, size_t count, P** out) {
  void* p = nullptr;
  hipError_t e = carve(h, count * sizeof(P), &p);
  *out = static_cast<P*>(p);
  return e;
}

// Releases on scope exit everything carved after its construction.
struct Frame {
  slrf_ctx* h;
  size_t top;
  explicit Frame(slrf_ctx* hh) : h(hh), top(hh->ar.top) {}
  ~Frame() { h->ar.top = top; }
};

// Kernel-class timing and byte accounting.
struct Scope {
  slrf_ctx* h;
  int cls;
  hipEvent_t b = nullptr;
  Scope(slrf_ctx* hh, int c, double bytes) : h(hh), cls(c) {
    if (cls < 0) return;  // not recorded
    if (h->cur_stats) {
      h->cur_stats->launches[cls] += 1;
      h->cur_stats->bytes[cls] += bytes;
    }
    if (h->opt.timing && h->cur_stats) {
      hipEvent_t a = h->timer.get();
      b = h->timer.get();
      if (a && b) {
        (void)hipEventRecord(a, h->stream);
        h->timer.pending.push_back({cls, a, b});
      } else {
        b = nullptr;
      }
    }
  }
  ~Scope() {
    if (b) (void)hipEventRecord(b, h->stream);
  }
};

void defer_bytes(slrf_ctx* h, int cls, double per_sys, bool sweep = false) {
  if (h->cur_stats && h->defer_k >= 0) h->defer.push_back({cls, h->defer_k, per_sys, sweep});
}

// nact_k[k]: systems active at step k of the finished cycle; nact0 those the
// cycle's launches were counted with.
void settle_bytes(slrf_ctx* h, const std::vector<int>& nact_k, int nact0) {
  if (h->cur_stats)
    for (const auto& d : h->defer) {
      const int a = d.k < (int)nact_k.size() ? nact_k[d.k] : 0;
      h->cur_stats->bytes[d.cls] += (double)(a - nact0) * d.per_sys;
      if (d.sweep) h->cur_stats->sweep_systems += a - nact0;
    }
  h->defer.clear();
}

void harvest_timers(slrf_ctx* h) {
  if (!h->cur_stats) {
    h->timer.reset();
    return;
  }
  for (auto& r : h->timer.pending) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) h->cur_stats->ms[r.cls] += ms;
  }
  h->timer.reset();
}

hipError_t sync(slrf_ctx* h) {
  hipError_t e = hipStreamSynchronize(h->stream);
  if (e == hipSuccess) harvest_timers(h);
  return e;
}

slrf_status validate_options(slrf_ctx* h, const slrf_options& o) {
  if (o.precision != SLRF_PREC_FP64 && o.precision != SLRF_PREC_MIXED)
    return fail(h, SLRF_E_ARG, "precision must be SLRF_PREC_FP64 or SLRF_PREC_MIXED");
  if (o.precond != SLRF_PC_NONE && o.precond != SLRF_PC_JACOBI && o.precond != SLRF_PC_AMG)
    return fail(h, SLRF_E_ARG, "unknown preconditioner");
  if (o.restart < 1 || o.restart > kMaxRestart)
    return fail(h, SLRF_E_ARG, "restart must be in [1, 32]");
  if (o.maxit_lin < 1) return fail(h, SLRF_E_ARG, "maxit_lin must be >= 1");
  if (o.it_max_lin < -1) return fail(h, SLRF_E_ARG, "it_max_lin must be >= -1");
  if (!(o.tol_lin >= 0.0) || !(o.tol_eig > 0.0))
    return fail(h, SLRF_E_ARG, "tolerances must be positive");
  if (!(o.inner_rtol >= 0.0 && o.inner_rtol < 1.0))
    return fail(h, SLRF_E_ARG, "inner_rtol must be in [0, 1)");
  if (o.max_outer < 1) return fail(h, SLRF_E_ARG, "max_outer must be >= 1");
  if (o.max_slots < 0 || o.max_slots % kPanel != 0)
    return fail(h, SLRF_E_ARG, "max_slots must be a non-negative multiple of 16");
  if (o.amg_block < 0 || o.amg_block > 8) return fail(h, SLRF_E_ARG, "amg_block must be 0..8");
  if (o.amg_block > 1 && h && h->P.n > 0 && h->P.n % o.amg_block != 0)
    return fail(h, SLRF_E_ARG, "n must be a multiple of amg_block");
  if (o.spmm_variant < 0 || o.spmm_variant >= kSpmmVariants)
    return fail(h, SLRF_E_ARG, "spmm_variant must be 0..7");
  if (o.amg_setup != SLRF_AMG_HOST && o.amg_setup != SLRF_AMG_DEVICE)
    return fail(h, SLRF_E_ARG, "amg_setup must be SLRF_AMG_HOST or SLRF_AMG_DEVICE");
  if (o.amg_coarse_min < 0 || o.amg_coarse_min > AmgParams().dense_max)
    return fail(h, SLRF_E_ARG, "amg_coarse_min must be 0..2048");
  return SLRF_OK;
}

PanelGrid make_grid(int n, int C, int occ, int ND) {
  PanelGrid g;
  g.rpb = n >= 65536 ? 512 : (n >= 8192 ? 256 : 64);
  g.nrb = (n + g.rpb - 1) / g.rpb;
  g.npan = (occ + kPanel - 1) / kPanel;
  g.group = 8;
  g.C = C;
  g.ND = ND;
  return g;
}

int nrb_for(int n) {
  const int rpb = n >= 65536 ? 512 : (n >= 8192 ? 256 : 64);
  return (n + rpb - 1) / rpb;
}


// ---------------------------------------------------------------------------
// AMG: host build (once per handle, first use) and the device V-cycle
// ---------------------------------------------------------------------------
int max_slice_of(const std::vector<int>& rp, int n, int sub) {
  int mx = 0;
  for (int r = 0; r < n; r += sub) mx = std::max(mx, rp[std::min(r + sub, n)] - rp[r]);
  return mx;
}

// ---------------------------------------------------------------------------
// Host analysis of a pencil (everything setup derives from A and B on the
// host): validation, row order, the sweep formats and the AMG hierarchy.  The
// same analysis sizes the workspace (slrf_workspace_size) and fills it
// (slrf_setup); the last one is kept, keyed by a hash of the CSR contents and
// the options it depends on, so that the pair costs one analysis.
// ---------------------------------------------------------------------------
struct HostImage {
  bool ok = false;
  int nc = 0;
  HostHalo hx;
  HostHaloSub p;   // P's nonzeros on the image tiles
};

struct HostSetup {
  int n = 0, nnz = 0, block = 1;
  bool reorder = false;
  std::vector<int> order;            // order[new] = old (reorder only)
  std::vector<int> rp, ci;           // the pencil in its final row order
  std::vector<double> a, b;
  std::vector<int> gp, gc;           // row-group union format
  std::vector<double> ga, gb;
  int grp_ent = 0;
  bool has_halo = false;
  HostHalo hx;
  bool has_ug = false;
  HostUGroup ug;
  int max64 = 0, max32 = 0;
  bool has_amg = false;
  AmgHierarchy H;                    // without the per-pole coarse inverses
  std::vector<HostImage> img;        // img[l], l < levels - 1
  // SLRF_AMG_DEVICE: the hierarchy is built by slrf_setup (parameters kept here)
  bool amg_device = false;
  AmgParams amg_prm;
  std::vector<double> amg_xyz;       // node coordinates in the final order (or empty)
};

uint64_t fnv1a(uint64_t h, const void* p, size_t bytes) {
  const unsigned char* c = static_cast<const unsigned char*>(p);
  for (size_t i = 0; i < bytes; ++i) h = (h ^ c[i]) * 1099511628211ull;
  return h;
}

std::mutex g_an_mu;
uint64_t g_an_key = 0;
std::shared_ptr<const HostSetup> g_an;

// The level images (A_l P_l, B_l P_l with P_l's values) in halo tiles over the
// next level's rows, from the Galerkin products the hierarchy kept (which are
// then dropped).
void amg_images(AmgHierarchy& H, std::vector<HostImage>& img) {
  const int L = (int)H.levels.size();
  img.assign(std::max(L - 1, 0), HostImage());
  for (int l = 0; l + 1 < L; ++l) {
    std::vector<double> ipv;
    const HostLevel& lvl = H.levels[l];
    HostImage& I = img[l];
    const HostLevel& ab = H.img[l];
    // tiles under a 64-row coarse halo where the image allows, else under 128
    // (the up-step's halo staging is compiled for either)
    I.ok = image_p_values(ab, H.P[l], ipv) &&
           (build_halo(lvl.n, ab.rp, ab.ci, ab.a, ab.b, kImgMaxH, kHaloTileRows, I.hx, &ipv) ||
            build_halo(lvl.n, ab.rp, ab.ci, ab.a, ab.b, kImgMaxH2, kHaloTileRows, I.hx, &ipv));
    if (I.ok) build_halo_sub(lvl.n, I.hx, I.p);
    I.nc = H.P[l].m;
  }
  H.img.clear();
  H.img.shrink_to_fit();
}

// Reads and validates A and B (device CSR, shared pattern, sorted, diagonal
// present) and computes the host analysis; nullptr with `err` set on failure.
std::shared_ptr<const HostSetup> analyse(const slrf_csr* A, const slrf_csr* B,
                                         const slrf_options& opt, std::string& err,
                                         slrf_status& st) {
  st = SLRF_E_ARG;
  if (!A || !B) { err = "null argument"; return nullptr; }
  if (A->n <= 0 || A->nnz <= 0 || A->n != B->n || A->nnz != B->nnz) {
    err = "A and B must be non-empty with equal n and nnz";
    return nullptr;
  }
  if (!A->rowptr || !A->col || !A->val || !B->rowptr || !B->col || !B->val) {
    err = "null CSR array";
    return nullptr;
  }
  const int n = A->n, nnz = A->nnz;
  std::vector<int> rp(n + 1), cl(nnz), rp2(n + 1), cl2(nnz);
  std::vector<double> av(nnz), bv(nnz);
  if (hipMemcpy(rp.data(), A->rowptr, sizeof(int) * (n + 1), hipMemcpyDeviceToHost) ||
      hipMemcpy(cl.data(), A->col, sizeof(int) * nnz, hipMemcpyDeviceToHost) ||
      hipMemcpy(rp2.data(), B->rowptr, sizeof(int) * (n + 1), hipMemcpyDeviceToHost) ||
      hipMemcpy(cl2.data(), B->col, sizeof(int) * nnz, hipMemcpyDeviceToHost) ||
      hipMemcpy(av.data(), A->val, sizeof(double) * nnz, hipMemcpyDeviceToHost) ||
      hipMemcpy(bv.data(), B->val, sizeof(double) * nnz, hipMemcpyDeviceToHost)) {
    err = "CSR arrays are not readable device memory";
    return nullptr;
  }
  if (rp[0] != 0 || rp[n] != nnz) { err = "rowptr[0] must be 0 and rowptr[n] nnz"; return nullptr; }
  for (int i = 0; i < n; ++i) {
    if (rp[i + 1] < rp[i]) { err = "rowptr must be nondecreasing"; return nullptr; }
    bool diag = false;
    for (int e = rp[i]; e < rp[i + 1]; ++e) {
      if (cl[e] < 0 || cl[e] >= n) { err = "column index out of range"; return nullptr; }
      if (e > rp[i] && cl[e] <= cl[e - 1]) {
        err = "column indices must be strictly increasing within a row";
        return nullptr;
      }
      diag |= cl[e] == i;
    }
    if (!diag) { err = "every row must store its diagonal entry"; return nullptr; }
  }
  if (rp != rp2 || cl != cl2) { err = "A and B must share one CSR pattern"; return nullptr; }
  const bool amg = opt.precond == SLRF_PC_AMG;
  uint64_t key = 1469598103934665603ull;
  key = fnv1a(key, rp.data(), rp.size() * sizeof(int));
  key = fnv1a(key, cl.data(), cl.size() * sizeof(int));
  key = fnv1a(key, av.data(), av.size() * sizeof(double));
  key = fnv1a(key, bv.data(), bv.size() * sizeof(double));
  const int32_t kopt[7] = {opt.reorder, opt.amg_block, amg ? 1 : 0, n,
                           opt.node_xyz != nullptr ? 1 : 0, opt.amg_setup,
                           opt.amg_coarse_min};
  key = fnv1a(key, kopt, sizeof(kopt));
  if (opt.node_xyz) key = fnv1a(key, opt.node_xyz, sizeof(double) * n);
  {
    std::lock_guard<std::mutex> lk(g_an_mu);
    if (g_an && g_an_key == key) {
      st = SLRF_OK;
      return g_an;
    }
  }
  auto hs = std::make_shared<HostSetup>();
  hs->n = n;
  hs->nnz = nnz;
  {
    HostLevel L0;
    L0.n = n;
    L0.rp = rp;
    L0.ci = cl;
    hs->block = opt.amg_block > 0 ? opt.amg_block : detect_block(L0);
  }
  if (n % hs->block != 0) { err = "n must be a multiple of amg_block"; return nullptr; }
  hs->reorder = opt.reorder != 0;
  if (hs->reorder) {
    // Locality order (nested aggregation of the graph of A): the pencil is
    // kept permuted and the order applied at the boundary.
    HostLevel L0;
    L0.n = n;
    L0.rp = rp;
    L0.ci = cl;
    L0.a = av;
    locality_order(L0, hs->order, hs->block);
    std::vector<int> inv(n);
    for (int i = 0; i < n; ++i) inv[hs->order[i]] = i;
    hs->rp.assign(n + 1, 0);
    hs->ci.resize(nnz);
    hs->a.resize(nnz);
    hs->b.resize(nnz);
    std::vector<std::pair<int, int>> row;
    for (int i = 0; i < n; ++i) {
      const int o = hs->order[i];
      row.clear();
      for (int e = rp[o]; e < rp[o + 1]; ++e) row.push_back({inv[cl[e]], e});
      std::sort(row.begin(), row.end());
      int k = hs->rp[i];
      for (auto& pr : row) {
        hs->ci[k] = pr.first;
        hs->a[k] = av[pr.second];
        hs->b[k] = bv[pr.second];
        ++k;
      }
      hs->rp[i + 1] = k;
    }
  } else {
    hs->rp = rp;
    hs->ci = cl;
    hs->a = av;
    hs->b = bv;
  }
  {
    // Row-group (union) format: groups of 4 consecutive rows, the union of
    // their columns once per group and 4 coefficients of A and of B per entry.
    const int R = 4, ng = (n + R - 1) / R;
    hs->gp.assign(ng + 1, 0);
    std::vector<int> u;
    for (int gi = 0; gi < ng; ++gi) {
      const int r0 = gi * R, r1 = std::min(r0 + R, n);
      u.assign(hs->ci.begin() + hs->rp[r0], hs->ci.begin() + hs->rp[r1]);
      std::sort(u.begin(), u.end());
      u.erase(std::unique(u.begin(), u.end()), u.end());
      const size_t base = hs->gc.size();
      hs->gc.insert(hs->gc.end(), u.begin(), u.end());
      hs->ga.resize(hs->gc.size() * R, 0.0);
      hs->gb.resize(hs->gc.size() * R, 0.0);
      for (int r = r0; r < r1; ++r)
        for (int e = hs->rp[r]; e < hs->rp[r + 1]; ++e) {
          const size_t pos =
              base + (std::lower_bound(u.begin(), u.end(), hs->ci[e]) - u.begin());
          hs->ga[pos * R + (r - r0)] = hs->a[e];
          hs->gb[pos * R + (r - r0)] = hs->b[e];
        }
      hs->gp[gi + 1] = (int)hs->gc.size();
    }
    for (int g0 = 0; g0 < ng; g0 += 8)
      hs->grp_ent = std::max(hs->grp_ent, hs->gp[std::min(g0 + 8, ng)] - hs->gp[g0]);
  }
  // halo tiles (absent when one 8-row slice references more columns than a
  // tile holds) and the wave-uniform row groups
  hs->has_halo = build_halo(n, hs->rp, hs->ci, hs->a, hs->b, kHaloMaxH, kHaloTileRows, hs->hx);
  hs->has_ug = build_ugroup(n, hs->rp, hs->ci, hs->a, hs->b, 4, 4, hs->ug);
  hs->max64 = max_slice_of(hs->rp, n, 64);
  hs->max32 = max_slice_of(hs->rp, n, 32);
  if (amg) {
    HostLevel fine;
    fine.n = n;
    fine.rp = hs->rp;
    fine.ci = hs->ci;
    fine.a = hs->a;
    fine.b = hs->b;
    AmgParams prm;
    prm.block = hs->block;
    prm.coarse_min = opt.amg_coarse_min;
    std::vector<double> xyz;
    if (opt.node_xyz && (hs->block == 2 || hs->block == 3)) {
      // coordinates in the final node order (a node's dofs stay together)
      const int bs = hs->block;
      xyz.resize(n);
      for (int k = 0; k < n / bs; ++k) {
        const int old = hs->reorder ? hs->order[bs * k] / bs : k;
        for (int c = 0; c < bs; ++c) xyz[(size_t)k * bs + c] = opt.node_xyz[(size_t)old * bs + c];
      }
      prm.xyz = &xyz;
    }
    if (opt.amg_setup == SLRF_AMG_DEVICE) {
      // built by slrf_setup, on the GPU, in the caller's workspace
      hs->amg_device = true;
      hs->amg_prm = prm;
      hs->amg_prm.xyz = nullptr;
      hs->amg_xyz = std::move(xyz);
    } else {
      std::string aerr;
      if (!amg_build(fine, {}, prm, hs->H, aerr)) {
        err = "AMG setup: " + aerr;
        return nullptr;
      }
      amg_images(hs->H, hs->img);
      hs->has_amg = true;
    }
  }
  std::lock_guard<std::mutex> lk(g_an_mu);
  g_an_key = key;
  g_an = hs;
  st = SLRF_OK;
  return g_an;
}

// Places the persistent device data of a pencil in the workspace, in a fixed
// order: with `dry` it only counts the bytes (the same sequence, so the count
// is exact); otherwise it carves and uploads and points the handle at it.
struct Placer {
  slrf_ctx* h;
  bool dry;
  size_t bytes = 0;
  hipError_t room(size_t b, void** out) {
    if (dry) {
      bytes = align_up(bytes) + align_up(std::max<size_t>(b, 1));
      *out = nullptr;
      return hipSuccess;
    }
    return carve(h, b, out);
  }
  template <typename V>
  hipError_t put(const std::vector<V>& v, const V** out) {
    void* p = nullptr;
    hipError_t e = room(v.size() * sizeof(V), &p);
    if (e != hipSuccess || dry) {
      *out = static_cast<const V*>(p);
      return e;
    }
    if (!v.empty()) e = hipMemcpy(p, v.data(), v.size() * sizeof(V), hipMemcpyHostToDevice);
    *out = static_cast<const V*>(p);
    return e;
  }
};

template <typename V>
std::vector<float> to_f32(const std::vector<V>& v) { return std::vector<float>(v.begin(), v.end()); }

// The fine pencil: permuted copy, row-group / halo / row-group-sweep formats,
// FP32 values, diagonals (filled by kernels afterwards), weights.
hipError_t place_pencil(slrf_ctx* h, const HostSetup& hs, Placer& pl, const slrf_csr* A,
                        const slrf_csr* B) {
  hipError_t e;
  DevPencil& P = h->P;
  P.n = hs.n;
  P.nnz = hs.nnz;
  if (hs.reorder) {
    const int* ord;
    if ((e = pl.put(hs.order, &ord)) != hipSuccess) return e;
    h->order = const_cast<int*>(ord);
    if ((e = pl.put(hs.rp, &P.rowptr)) != hipSuccess) return e;
    if ((e = pl.put(hs.ci, &P.col)) != hipSuccess) return e;
    if ((e = pl.put(hs.a, &P.a)) != hipSuccess) return e;
    if ((e = pl.put(hs.b, &P.b)) != hipSuccess) return e;
  } else {
    h->order = nullptr;
    P.rowptr = A ? A->rowptr : nullptr;
    P.col = A ? A->col : nullptr;
    P.a = A ? A->val : nullptr;
    P.b = B ? B->val : nullptr;
  }
  if ((e = pl.put(hs.gp, &P.gptr)) != hipSuccess) return e;
  if ((e = pl.put(hs.gc, &P.gcol)) != hipSuccess) return e;
  if ((e = pl.put(hs.ga, &P.gca)) != hipSuccess) return e;
  if ((e = pl.put(hs.gb, &P.gcb)) != hipSuccess) return e;
  if ((e = pl.put(pl.dry ? std::vector<float>(hs.ga.size()) : to_f32(hs.ga), &P.gca32)) != hipSuccess)
    return e;
  if ((e = pl.put(pl.dry ? std::vector<float>(hs.gb.size()) : to_f32(hs.gb), &P.gcb32)) != hipSuccess)
    return e;
  P.grp_lds_ent = hs.grp_ent;
  if (hs.has_halo) {
    const HostHalo& hx = hs.hx;
    std::vector<float2> ab32;
    std::vector<double2> ab64;
    ab32.resize(hx.ab.size() / 2);
    ab64.resize(hx.ab.size() / 2);
    if (!pl.dry)
      for (size_t i = 0; i < ab64.size(); ++i) {
        ab64[i] = make_double2(hx.ab[2 * i], hx.ab[2 * i + 1]);
        ab32[i] = make_float2((float)hx.ab[2 * i], (float)hx.ab[2 * i + 1]);
      }
    if ((e = pl.put(hx.trow, &P.hx_trow)) != hipSuccess) return e;
    if ((e = pl.put(hx.hptr, &P.hx_hptr)) != hipSuccess) return e;
    if ((e = pl.put(hx.halo, &P.hx_halo)) != hipSuccess) return e;
    if ((e = pl.put(hx.sptr, &P.hx_sptr)) != hipSuccess) return e;
    if ((e = pl.put(hx.slen, &P.hx_slen)) != hipSuccess) return e;
    if ((e = pl.put(hx.lcol, &P.hx_lcol)) != hipSuccess) return e;
    if ((e = pl.put(ab32, &P.hx_ab32)) != hipSuccess) return e;
    if ((e = pl.put(ab64, &P.hx_ab64)) != hipSuccess) return e;
    P.hx_ntile = hx.ntile;
    P.hx_hmax = hx.hmax;
    P.hx_emax = hx.emax;
  }
  if (hs.has_ug) {
    const HostUGroup& ug = hs.ug;
    std::vector<float2> ab32(ug.ab.size() / 2);
    std::vector<double2> ab64(ug.ab.size() / 2);
    if (!pl.dry)
      for (size_t i = 0; i < ab64.size(); ++i) {
        ab64[i] = make_double2(ug.ab[2 * i], ug.ab[2 * i + 1]);
        ab32[i] = make_float2((float)ug.ab[2 * i], (float)ug.ab[2 * i + 1]);
      }
    if ((e = pl.put(ug.gptr, &P.ug_gptr)) != hipSuccess) return e;
    if ((e = pl.put(ug.ent, &P.ug_ent)) != hipSuccess) return e;
    if ((e = pl.put(ab32, &P.ug_ab32)) != hipSuccess) return e;
    if ((e = pl.put(ab64, &P.ug_ab64)) != hipSuccess) return e;
    P.ug_R = ug.R;
    P.ug_ngroups = ug.ngroups;
  }
  P.max_nnz_sub64 = hs.max64;
  P.max_nnz_sub32 = hs.max32;
  void* v;
  if ((e = pl.room(sizeof(float) * hs.nnz, &v)) != hipSuccess) return e;
  h->a32 = static_cast<float*>(v);
  if ((e = pl.room(sizeof(float) * hs.nnz, &v)) != hipSuccess) return e;
  h->b32 = static_cast<float*>(v);
  if ((e = pl.room(sizeof(double) * hs.n, &v)) != hipSuccess) return e;
  h->da = static_cast<double*>(v);
  if ((e = pl.room(sizeof(double) * hs.n, &v)) != hipSuccess) return e;
  h->db = static_cast<double*>(v);
  if ((e = pl.room(sizeof(double2) * 64, &v)) != hipSuccess) return e;  // pole weights
  h->d_w = static_cast<double2*>(v);
  P.a32 = h->a32;
  P.b32 = h->b32;
  P.da = h->da;
  P.db = h->db;
  return hipSuccess;
}

// The AMG hierarchy (levels >= 1, transfers, images) and, for `npoles` poles,
// room for the coarsest-level inverses (filled by setup).
hipError_t place_amg(slrf_ctx* h, const AmgHierarchy& H, const std::vector<HostImage>& img,
                     Placer& pl, int npoles) {
  hipError_t e;
  DevAmg& A = h->amg;
  const int L = (int)H.levels.size();
  A = DevAmg();
  for (auto& lv : H.levels) A.n.push_back(lv.n);
  // smoothing weight 1.5 / rho(D^-1 A_l): omega * rho stays below 2 on every
  // pencil; on the 3D Q1 benchmark pencil it needs the fewest GCR iterations
  // of the weights 1.0 .. 1.95 over rho (4/3: 4 % more, 1.65: 5 % more, 1.8:
  // 35 % more, 1.95 does not converge)
  for (double r : H.rho) A.omega.push_back(r > 0.0 ? 1.5 / r : 0.7);
  for (int l = 1; l < L; ++l) {
    const HostLevel& hl = H.levels[l];
    DevPencil d;
    d.n = hl.n;
    d.nnz = (int)hl.ci.size();
    std::vector<double> da(hl.n, 0.0), db(hl.n, 0.0);
    for (int i = 0; i < hl.n; ++i)
      for (int k = hl.rp[i]; k < hl.rp[i + 1]; ++k)
        if (hl.ci[k] == i) {
          da[i] = hl.a[k];
          db[i] = hl.b[k];
        }
    if ((e = pl.put(hl.rp, &d.rowptr)) != hipSuccess) return e;
    if ((e = pl.put(hl.ci, &d.col)) != hipSuccess) return e;
    if ((e = pl.put(hl.a, &d.a)) != hipSuccess) return e;
    if ((e = pl.put(hl.b, &d.b)) != hipSuccess) return e;
    if ((e = pl.put(to_f32(hl.a), &d.a32)) != hipSuccess) return e;
    if ((e = pl.put(to_f32(hl.b), &d.b32)) != hipSuccess) return e;
    if ((e = pl.put(da, &d.da)) != hipSuccess) return e;
    if ((e = pl.put(db, &d.db)) != hipSuccess) return e;
    d.max_nnz_sub64 = max_slice_of(hl.rp, hl.n, 64);
    d.max_nnz_sub32 = max_slice_of(hl.rp, hl.n, 32);
    A.lv.push_back(d);
    A.nnz_all += d.nnz;
  }
  auto up_tr = [&](const HostCsrP& M, DevTransfer& d) -> hipError_t {
    d.nrows = M.n;
    d.ncols = M.m;
    d.nnz = (int)M.ci.size();
    d.max_sub64 = max_slice_of(M.rp, M.n, 64);
    hipError_t e2;
    if ((e2 = pl.put(M.rp, &d.rowptr)) != hipSuccess) return e2;
    if ((e2 = pl.put(M.ci, &d.col)) != hipSuccess) return e2;
    if ((e2 = pl.put(M.v, &d.v)) != hipSuccess) return e2;
    return pl.put(to_f32(M.v), &d.v32);
  };
  for (int l = 0; l + 1 < L; ++l) {
    DevTransfer P, R;
    if ((e = up_tr(H.P[l], P)) != hipSuccess) return e;
    if ((e = up_tr(H.R[l], R)) != hipSuccess) return e;
    A.P.push_back(P);
    A.R.push_back(R);
    A.nnz_all += P.nnz + R.nnz;
  }
  // images (A_l P_l, B_l P_l) with P_l's values, in 32-row halo tiles over
  // the next level's rows: the fused up-step of level l (absent when a
  // tile's coarse halo would exceed kImgMaxH2 rows)
  A.img.assign(L, DevImage());
  for (int l = 0; l + 1 < L; ++l) {
    const HostImage& hi = img[l];
    if (!hi.ok) continue;
    const HostHalo& hx = hi.hx;
    DevImage& I = A.img[l];
    std::vector<double2> ab64(hx.ab.size() / 2);
    std::vector<float2> ab32(ab64.size());
    for (size_t i = 0; i < ab64.size(); ++i) {
      ab64[i] = make_double2(hx.ab[2 * i], hx.ab[2 * i + 1]);
      ab32[i] = make_float2((float)hx.ab[2 * i], (float)hx.ab[2 * i + 1]);
    }
    if ((e = pl.put(hx.trow, &I.trow)) != hipSuccess) return e;
    if ((e = pl.put(hx.hptr, &I.hptr)) != hipSuccess) return e;
    if ((e = pl.put(hx.halo, &I.halo)) != hipSuccess) return e;
    if ((e = pl.put(hx.sptr, &I.sptr)) != hipSuccess) return e;
    if ((e = pl.put(hx.lcol, &I.lcol)) != hipSuccess) return e;
    if ((e = pl.put(ab32, &I.ab32)) != hipSuccess) return e;
    if ((e = pl.put(ab64, &I.ab64)) != hipSuccess) return e;
    if ((e = pl.put(hi.p.sptr, &I.psptr)) != hipSuccess) return e;
    if ((e = pl.put(hi.p.lcol, &I.plcol)) != hipSuccess) return e;
    if ((e = pl.put(to_f32(hi.p.v), &I.p32)) != hipSuccess) return e;
    if ((e = pl.put(hi.p.v, &I.p64)) != hipSuccess) return e;
    I.pemax = hi.p.emax;
    I.nc = hi.nc;
    I.hmax = hx.hmax;
    I.emax = hx.emax;
    I.ntile = hx.ntile;
    A.nnz_all += hx.lcol.size();
  }
  A.nc = H.levels.back().n;
  const size_t ninv = (size_t)npoles * A.nc * A.nc;
  if ((e = pl.room(ninv * sizeof(double2), &A.inv64)) != hipSuccess) return e;
  if ((e = pl.room(ninv * sizeof(float2), &A.inv32)) != hipSuccess) return e;
  A.ready = !pl.dry;
  return hipSuccess;
}

size_t persistent_bytes(const HostSetup& hs, int npoles) {
  slrf_ctx tmp;
  Placer pl{&tmp, true};
  (void)place_pencil(&tmp, hs, pl, nullptr, nullptr);
  if (hs.has_amg) (void)place_amg(&tmp, hs.H, hs.img, pl, npoles);
  return align_up(pl.bytes);
}

// SLRF_AMG_DEVICE: what slrf_workspace_size reserves for a hierarchy it has not
// built (levels, P and R, the images and the coarse inverses): 200 bytes per
// fine nonzero, 64 per fine row and the largest dense coarsest level for
// every pole.  The 48^3 elasticity hierarchy (26.9 M nonzeros) takes about a
// fifth of it.
size_t amg_device_bound(const HostSetup& hs, int npoles) {
  const size_t nc = (size_t)hs.amg_prm.dense_max;
  return align_up((size_t)hs.nnz * 200 + (size_t)hs.n * 64 + (size_t)npoles * nc * nc * 24);
}

// Level vectors of the V-cycle for a pool of C slots.
struct AmgVecs {
  void* W0 = nullptr;   // level-0 smoothed iterate
  void* T0 = nullptr;   // level-0 residual
  std::vector<void*> X, W, B, T;  // per level (index 0 unused)
};

// level sizes nlev (nlev[0] = fine)
size_t amg_vec_bytes(const std::vector<int>& nlev, int C, size_t sT) {
  if (nlev.empty()) return 0;
  size_t b = 2 * (size_t)C * nlev[0] * sT;
  for (size_t l = 1; l < nlev.size(); ++l) b += 4 * (size_t)C * nlev[l] * sT;
  return b;
}
size_t amg_vec_bytes(const DevAmg& A, int C, size_t sT) { return amg_vec_bytes(A.n, C, sT); }

template <typename T>
slrf_status amg_vectors(slrf_ctx* h, int C, AmgVecs& v) {
  const DevAmg& A = h->amg;
  const size_t sT = 2 * sizeof(T);
  char* base;
  HIPCHK(carve_t(h, amg_vec_bytes(A, C, sT), &base));
  size_t off = 0;
  auto take = [&](size_t rows) {
    void* p = base + off;
    off += (size_t)C * rows * sT;
    return p;
  };
  v.W0 = take(A.n[0]);
  v.T0 = take(A.n[0]);
  const size_t L = A.n.size();
  v.X.assign(L, nullptr);
  v.W.assign(L, nullptr);
  v.B.assign(L, nullptr);
  v.T.assign(L, nullptr);
  for (size_t l = 1; l < L; ++l) {
    v.X[l] = take(A.n[l]);
    v.W[l] = take(A.n[l]);
    v.B[l] = take(A.n[l]);
    v.T[l] = take(A.n[l]);
  }
  return SLRF_OK;
}

// Complex-float sweeps on a pencil with halo tiles and a level-0 image keep
// the level-0 V-cycle vectors the GCR step and the sweeps exchange (the
// pre-smoothed iterate x0 and its residual r1) in complex bfloat16.
template <typename T>
bool amg_level0_bf16(const slrf_ctx* h) {
  const DevAmg& A = h->amg;
  return std::is_same<T, float>::value && sweep_is_halo<T>(h->P) && !A.img.empty() &&
         A.img[0].ntile > 0 && A.img[0].hmax <= kImgMaxH2;
}

// z = V(r): one V-cycle (damped-Jacobi pre/post smoothing from a zero guess,
// Galerkin coarse correction, dense coarsest solve) for every active slot.
// pre0_done: the level-0 pre-smoothing omega D^-1 r is already in v.W0.
template <typename T>
slrf_status vcycle(slrf_ctx* h, const AmgVecs& v, int C, int occ, int ND, const SlotTables& st,
                   const void* Rin, void* Zout, int nact, bool pre0_done) {
  const DevAmg& A = h->amg;
  hipStream_t s = h->stream;
  const int L = (int)A.n.size();
  const size_t sT = 2 * sizeof(T);
  const void* inv = std::is_same<T, float>::value ? A.inv32 : A.inv64;
  {
    double per_sys = 0.0;
    for (int l = 0; l < L; ++l) per_sys += 10.0 * (double)A.n[l] * sT;
    const double bytes = nact * per_sys + (double)(h->P.nnz + A.nnz_all) * (4.0 + 2.0 * sizeof(T));
    Scope sp(h, SLRF_K_PRECOND, bytes);
    defer_bytes(h, SLRF_K_PRECOND, per_sys);
    if (L == 1) {
      HIPCHK(launch_coarse_solve<T>(A.nc, make_grid(A.nc, C, occ, ND), st, h->N, inv, Rin, Zout,
                                    s));
      return SLRF_OK;
    }
    auto lvl = [&](int l) -> const DevPencil& { return l == 0 ? h->P : A.lv[l - 1]; };
    const double fine_csr = (double)h->P.nnz * (4.0 + 2.0 * sizeof(T)) + 4.0 * (A.n[0] + 1);
    std::vector<const void*> b(L, nullptr);
    std::vector<void*> x(L, nullptr);
    b[0] = Rin;
    const bool r16 = amg_level0_bf16<T>(h);
    for (int l = 0; l + 1 < L; ++l) {
      const PanelGrid g = make_grid(A.n[l], C, occ, ND);
      void* xb = l == 0 ? v.W0 : v.X[l];
      void* r = l == 0 ? v.T0 : v.T[l];
      // (level 0: the GCR step that formed r may already have written xb)
      if (l > 0 || !pre0_done)
        HIPCHK(launch_lvl_jacobi0<T>(lvl(l), g, st, A.omega[l], b[l], xb, s, l == 0 && r16));
      const bool h16 = l == 0 && r16;
      {
        const bool fine = l == 0 && sweep_is_halo<T>(h->P);
        Scope sw(h, fine ? SLRF_K_SWEEP : -1,
                 (double)nact * A.n[0] * sT * (h16 ? 2.0 : 3.0) + fine_csr);
        if (fine && h->cur_stats) h->cur_stats->sweep_systems += nact;
        if (fine) defer_bytes(h, SLRF_K_SWEEP, (double)A.n[0] * sT * (h16 ? 2.0 : 3.0), true);
        hipError_t err = hipSuccess;
        if (h16 && launch_resid_bf16<T>(h->P, g, st, xb, b[l], r, s, err, true))
          HIPCHK(err);
        else
          HIPCHK(launch_lvl_op<T>(lvl(l), g, st, kEpiResidOp, A.omega[l], xb, b[l], r, s));
      }
      const PanelGrid gc = make_grid(A.n[l + 1], C, occ, ND);
      if (h16)
        HIPCHK(launch_restrict_bf16<T>(A.R[l], gc, st, r, v.B[l + 1], s));
      else
        HIPCHK(launch_transfer<T>(A.R[l], gc, st, r, v.B[l + 1], false, s));
      b[l + 1] = v.B[l + 1];
      x[l] = xb;
    }
    HIPCHK(launch_coarse_solve<T>(A.nc, make_grid(A.nc, C, occ, ND), st, h->N, inv, b[L - 1],
                                  v.X[L - 1], s));
    x[L - 1] = v.X[L - 1];
    for (int l = L - 2; l >= 0; --l) {
      const PanelGrid g = make_grid(A.n[l], C, occ, ND);
      void* out = l == 0 ? Zout : v.W[l];
      {
        // prolongation and post-smoothing of level l in one pass
        hipError_t err = hipSuccess;
        if (launch_post_image<T>(A.img[l], lvl(l), g, st, A.omega[l], x[l + 1], x[l],
                                 l == 0 ? v.T0 : v.T[l], out, s, err, l == 0 && r16)) {
          HIPCHK(err);
          x[l] = out;
          continue;
        }
      }
      HIPCHK(launch_transfer<T>(A.P[l], g, st, x[l + 1], x[l], true, s));
      const bool fine = l == 0 && sweep_is_halo<T>(h->P);
      Scope sw(h, fine ? SLRF_K_SWEEP : -1, (double)nact * A.n[0] * sT * 3.0 + fine_csr);
      if (fine && h->cur_stats) h->cur_stats->sweep_systems += nact;
      if (fine) defer_bytes(h, SLRF_K_SWEEP, (double)A.n[0] * sT * 3.0, true);
      HIPCHK(launch_lvl_op<T>(lvl(l), g, st, kEpiJacobiOp, A.omega[l], x[l], b[l], out, s));
      x[l] = out;
    }
  }
  (void)sT;
  return SLRF_OK;
}


// ---------------------------------------------------------------------------
// SpMM autotuner: time every applicable kernel variant on the actual pencil
// (a 256-system panel batch in each precision) and keep the fastest.  The
// choice is cached per process by shape class (n bucket, nonzeros per row).
// ---------------------------------------------------------------------------
std::mutex g_tune_mu;
std::map<std::pair<int, int>, std::pair<int, int>> g_tune_cache;

template <typename T>
float time_spmm_variant(slrf_ctx* h, int var, void* Z, void* Q, const double2* sig, int nsys) {
  DevPencil P = h->P;
  if (std::is_same<T, float>::value) P.var32 = var; else P.var64 = var;
  const PanelGrid g = make_grid(P.n, nsys, nsys, 2);
  hipEvent_t a, b;
  if (hipEventCreate(&a) || hipEventCreate(&b)) return 1e30f;
  float best = 1e30f;
  for (int rep = 0; rep < 4; ++rep) {
    (void)hipEventRecord(a, h->stream);
    if (launch_spmm_panel<T>(P, g, sig, Z, Q, h->stream) != hipSuccess) break;
    (void)hipEventRecord(b, h->stream);
    (void)hipEventSynchronize(b);
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, a, b);
    if (rep > 0) best = std::min(best, ms);
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  return best;
}

slrf_status autotune_spmm(slrf_ctx* h) {
  const int n = h->P.n;
  const int nnz_row = (int)std::lround((double)h->P.nnz / n);
  int nb = 0;
  while ((1 << (nb + 1)) <= n) ++nb;
  const auto key = std::make_pair(nb, nnz_row);
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune_cache.find(key);
    if (it != g_tune_cache.end()) {
      h->P.var32 = it->second.first;
      h->P.var64 = it->second.second;
      return SLRF_OK;
    }
  }
  // a batch of up to 256 systems in each precision, carved from the free part
  // of the workspace (fewer when it is small; the defaults are kept when not
  // even one panel fits)
  Frame fr(h);
  const size_t avail = h->ar.cap > align_up(h->ar.top) ? h->ar.cap - align_up(h->ar.top) : 0;
  const size_t per_sys = 2 * (size_t)n * 16 + 16 + 4 * kAlign / kPanel;
  const int nsys = (int)std::min<size_t>(256, avail / per_sys / kPanel * kPanel);
  if (nsys < kPanel) return SLRF_OK;
  void *Z = nullptr, *Q = nullptr, *sg = nullptr;
  const size_t bytes = (size_t)nsys * n * 16;
  HIPCHK(carve(h, bytes, &Z));
  HIPCHK(carve(h, bytes, &Q));
  HIPCHK(carve(h, sizeof(double2) * nsys, &sg));
  std::vector<double2> sig(nsys);
  for (int i = 0; i < nsys; ++i) sig[i] = h->poles[i % h->N];
  HIPCHK(hipMemcpy(sg, sig.data(), sizeof(double2) * nsys, hipMemcpyHostToDevice));
  HIPCHK(hipMemsetAsync(Z, 0, bytes, h->stream));
  const int vars[7] = {kSpmmGroup,     kSpmmCsrLds, kSpmmCsrLds16, kSpmmCsrLds32,
                       kSpmmCsrDirect, kSpmmHalo,   kSpmmUGroup};
  int best32 = kSpmmAuto, best64 = kSpmmAuto;
  float t32 = 1e30f, t64 = 1e30f;
  for (int v : vars) {
    if (v == kSpmmHalo && h->P.hx_ntile == 0) continue;
    if (v == kSpmmUGroup && h->P.ug_ngroups == 0) continue;
    const float a = time_spmm_variant<float>(h, v, Z, Q, static_cast<double2*>(sg), nsys);
    if (a < t32) { t32 = a; best32 = v; }
    const float b = time_spmm_variant<double>(h, v, Z, Q, static_cast<double2*>(sg), nsys);
    if (b < t64) { t64 = b; best64 = v; }
  }
  (void)hipStreamSynchronize(h->stream);
  h->P.var32 = best32;
  h->P.var64 = best64;
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune_cache[key] = std::make_pair(best32, best64);
  return SLRF_OK;
}

// Workspace of one filter call: a fixed part (blocks of the columns, the
// per-system solution store, statistics) and a part per resident slot.  Both
// include the alignment of every carve.
size_t filter_fixed_bytes(int n, int nc, int N) {
  const size_t S = (size_t)N * nc;
  const size_t Spad = (S + kPanel - 1) / kPanel * kPanel;
  return 4 * (size_t)n * nc * sizeof(double) + (nc + 1) * sizeof(double) +
         Spad * n * 16 + (3 * S + 8 + kMaxPoles + 1) * sizeof(int) +
         (2 * (size_t)colstat_chunks(n) * nc + 2) * sizeof(double) + 16 * kAlign;
}

size_t filter_slot_bytes(int n, int m, size_t sT, const std::vector<int>& amg_levels) {
  const int ND = std::max(m, 2);
  size_t b = (size_t)n * (2 * 16 + 4 * sT + 2 * (size_t)m * sT) +
             (size_t)nrb_for(n) * ND * 16 + (size_t)ND * 16 + 7 * sizeof(int) +
             3 * sizeof(double) +
             ((size_t)5 * kMaxRestart + 1 + 2 * (size_t)kMaxRestart * kMaxRestart) * sizeof(double);
  return b + amg_vec_bytes(amg_levels, 1, sT);
}

// Rayleigh-Ritz on nc columns against nl locked ones (rr_rowmajor's buffers
// plus the entry points' row-major copies of U and of the locked block).
size_t rr_bytes(int n, int nc, int nl) {
  const size_t pq = std::max(nc, nl);
  return (size_t)n * (6 * (size_t)nc + 2 * (size_t)nl) * sizeof(double) +
         (gram_part_doubles(n, (int)pq) + 16) * sizeof(double) +
         (3 * pq * pq + 4 * pq + 16) * sizeof(double) +
         (2 * (size_t)colstat_chunks(n) * nc + 2) * sizeof(double) + 16 * kAlign;
}

// Per-call workspace of slrf_solve with an L-column subspace (the largest
// call: the subspace blocks, then the filter with C resident slots or the
// Rayleigh-Ritz step), which also covers slrf_filter and slrf_rayleigh_ritz
// on up to L columns.
size_t call_bytes(int n, int L, int N, const slrf_options& o, const std::vector<int>& amg_levels,
                  int C) {
  const size_t sT = o.precision == SLRF_PREC_MIXED ? 8 : 16;
  const size_t sub = ((size_t)n * 3 * L + 2 * (size_t)L + 16) * sizeof(double) + kAlign;
  const size_t flt = filter_fixed_bytes(n, L, N) +
                     (size_t)C * (filter_slot_bytes(n, o.restart, sT, amg_levels) +
                                  16 * kAlign / kPanel);
  return sub + std::max(flt, rr_bytes(n, L, L)) + 4 * kAlign;
}

// ---------------------------------------------------------------------------
// slrf_filter
// ---------------------------------------------------------------------------
template <typename T>
slrf_status run_filter(slrf_ctx* h, int nc, const double* X, const double* theta, double* U,
                       slrf_filter_stats* st) {
  const auto t0 = std::chrono::steady_clock::now();
  const int n = h->P.n, N = h->N, S = N * nc, m = h->opt.restart;
  const size_t sT = 2 * sizeof(T);
  const bool amg = h->opt.precond == SLRF_PC_AMG;
  const int pc = amg ? 2 : (h->opt.precond == SLRF_PC_JACOBI ? 1 : 0);
  if (amg && !h->amg.ready)
    return fail(h, SLRF_E_ARG, "the AMG preconditioner needs a handle set up with it");
  const bool warm = theta != nullptr;
  const bool mixed = std::is_same<T, float>::value;
  const double inner_rtol = mixed ? h->opt.inner_rtol : 0.0;
  const double safety = mixed ? 0.5 : 0.9;
  int itcap = h->opt.maxit_lin;
  if (h->opt.it_max_lin > 0) itcap = std::min(itcap, h->opt.it_max_lin);
  hipStream_t s = h->stream;
  const int ND = std::max(m, 2);

  const int Spad = (S + kPanel - 1) / kPanel * kPanel;
  // resident slots: every system at once when the workspace holds them, else
  // as many whole panels as fit (the pool then streams the systems through)
  const size_t fixed = filter_fixed_bytes(n, nc, N);
  const size_t slot = filter_slot_bytes(n, m, sT, amg ? h->amg.n : std::vector<int>()) +
                      16 * kAlign / kPanel;
  const size_t avail = h->ar.cap > align_up(h->ar.top) ? h->ar.cap - align_up(h->ar.top) : 0;
  int C = Spad;
  if (h->opt.max_slots > 0) C = std::min(C, h->opt.max_slots);
  if (fixed + (size_t)C * slot > avail) {
    const size_t fit = avail > fixed ? (avail - fixed) / slot : 0;
    C = (int)std::min<size_t>((size_t)C, fit) / kPanel * kPanel;
  }
  if (C < kPanel) {
    char buf[256];
    std::snprintf(buf, sizeof(buf),
                  "workspace too small: a filter of %d columns needs %zu bytes for one panel "
                  "of 16 systems, %zu are free",
                  nc, fixed + kPanel * slot, avail);
    return fail(h, SLRF_E_NOMEM, buf);
  }
  const int nrb = nrb_for(n);

  AmgVecs av;
  if (amg) {
    const slrf_status vs = amg_vectors<T>(h, C, av);
    if (vs != SLRF_OK) return vs;
  }
  // the GCR step writes the next V-cycle's level-0 pre-smoothing (hierarchies
  // of two or more levels; a single level is the dense solve alone)
  const bool fuse0 = amg && h->amg.n.size() > 1;
  double *Xr, *F, *E = nullptr, *Ur, *fn2;
  double2 *Ys, *Ya, *Yb, *part, *red;
  void *Ra, *Rb, *Za, *Zb, *Q, *Pb;
  HIPCHK(carve_t(h, (size_t)n * nc, &Xr));
  HIPCHK(carve_t(h, (size_t)n * nc, &F));
  if (warm) HIPCHK(carve_t(h, (size_t)n * nc, &E));
  HIPCHK(carve_t(h, (size_t)n * nc, &Ur));
  HIPCHK(carve_t(h, (size_t)nc + 1, &fn2));
  HIPCHK(carve_t(h, (size_t)Spad * n, &Ys));
  HIPCHK(carve_t(h, (size_t)C * n, &Ya));
  HIPCHK(carve_t(h, (size_t)C * n, &Yb));
  HIPCHK(carve(h, (size_t)C * n * sT, &Ra));
  HIPCHK(carve(h, (size_t)C * n * sT, &Rb));
  HIPCHK(carve(h, (size_t)C * n * sT, &Za));
  HIPCHK(carve(h, (size_t)C * n * sT, &Zb));
  HIPCHK(carve(h, (size_t)m * C * n * sT, &Q));
  HIPCHK(carve(h, (size_t)m * C * n * sT, &Pb));
  HIPCHK(carve_t(h, (size_t)nrb * ND * C, &part));
  HIPCHK(carve_t(h, (size_t)ND * C, &red));
  // slot tables: int: sys, col, src, active, status, retire (6C), the slots
  // grouped by pole (C) and the groups' offsets (kMaxPoles + 1); double2
  // sigma (C); double theta (C)
  int* itab;
  double* dtab;
  HIPCHK(carve_t(h, (size_t)7 * C + kMaxPoles + 1, &itab));
  HIPCHK(carve_t(h, (size_t)3 * C, &dtab));
  int *d_sys = itab, *d_col = itab + C, *d_src = itab + 2 * C, *d_act = itab + 3 * C,
      *d_status = itab + 4 * C, *d_retire = itab + 5 * C;
  double2* d_sigma = reinterpret_cast<double2*>(dtab);
  double* d_theta_slot = dtab + 2 * C;
  // scalars: beta, alpha (kMaxRestart*C double2 each), qq (kMaxRestart*C), target2 (C)
  double* scal;
  HIPCHK(carve_t(h,
                 (size_t)kMaxRestart * C * 5 + C + (size_t)kMaxRestart * kMaxRestart * C * 2,
                 &scal));
  SlotScalars sc;
  sc.beta = reinterpret_cast<double2*>(scal);
  sc.alpha = reinterpret_cast<double2*>(scal + (size_t)2 * kMaxRestart * C);
  sc.qq = scal + (size_t)4 * kMaxRestart * C;
  sc.target2 = scal + (size_t)5 * kMaxRestart * C;
  sc.bhist = reinterpret_cast<double2*>(scal + (size_t)5 * kMaxRestart * C + C);
  sc.fnorm2 = fn2;
  int* sysi;
  HIPCHK(carve_t(h, (size_t)3 * S + 8, &sysi));
  sc.sys_its = sysi;
  sc.sys_rn2 = reinterpret_cast<double*>(sysi + S + (S & 1));
  sc.status = d_status;
  h->h_flags.assign((size_t)std::max(C, S) * 2 + 16, 0);
  int* hflags = h->h_flags.data();

  // ----- right-hand sides: F = B X (and E = (A - theta B) X for the warm start)
  {
    Scope sp(h, SLRF_K_OTHER, 16.0 * n * nc);
    HIPCHK(launch_transpose(X, nc, n, n, Xr, nc, s, h->order));  // col-major -> row-major
  }
  {
    Scope sp(h, SLRF_K_OTHER, (warm ? 24.0 : 16.0) * n * nc + 20.0 * h->P.nnz);
    HIPCHK(launch_spmm_real(h->P, Xr, nc, nc, nullptr, F, warm ? theta : nullptr, E, s));
  }
  {
    double* cpart;
    const int nch = colstat_chunks(n);
    HIPCHK(carve_t(h, (size_t)2 * nch * nc + 2, &cpart));
    Scope sp(h, SLRF_K_OTHER, 8.0 * n * nc);
    HIPCHK(launch_colstats(n, nc, F, nullptr, nc, nullptr, nullptr, cpart, nch, fn2, nullptr, s));
  }
  HIPCHK(hipMemsetAsync(sc.sys_its, 0, sizeof(int) * S, s));

  // host-side pool state
  std::vector<int> h_sys(C, -1), h_col(C, 0), h_src(C, -1);
  std::vector<double2> h_sig(C, make_double2(0, 0));
  std::vector<double> h_th(C, 0.0);
  std::vector<double> h_theta_col;
  if (warm) {
    h_theta_col.resize(nc);
    HIPCHK(hipMemcpyAsync(h_theta_col.data(), theta, sizeof(double) * nc, hipMemcpyDeviceToHost,
                          s));
  }
  HIPCHK(sync(h));
  int next = 0;  // next system to admit
  int occ = 0;   // occupied slots (a prefix of the pool after compaction)
  int cur = 0;   // which of the double buffers holds the live state
  double2* Ybuf[2] = {Ya, Yb};
  void* Rbuf[2] = {Ra, Rb};
  void* Zbuf[2] = {Za, Zb};
  std::vector<int> status(C, -1);
  int kk_last = 0;
  int cycles = 0;
  bool numeric = false;
  const size_t vstride = (size_t)C * n;  // elements between consecutive P_i / Q_i
  // Complex-float cycles on the halo sweep keep the CGS basis q_0 .. q_{m-2}
  // in complex bfloat16 (the first half of each Q slot): GCR keeps using the
  // rounded vectors consistently (projections, residual update), the solution
  // update never reads them, and each cycle ends on an FP64 true residual.
  // Warm-started calls (Algorithm 2) keep the basis in complex float: with the
  // rounded basis, Algorithm 2 with locking and warm start took 28-39 outer
  // iterations instead of 7 on two of the 64 uneven diffusion pencils (cold
  // starts: 7 either way).
  const bool hq = std::is_same<T, float>::value && sweep_is_halo<T>(h->P) && m <= 9 && !warm;
  const double csr_bytes = (double)h->P.nnz * (4.0 + 2.0 * sizeof(T)) + 4.0 * (n + 1);

  int cyc_nact0 = 0, cyc_occ = 0;        // the last cycle's starting actives / slots
  std::vector<int> its_h(S, 0), its_start(C, 0);
  SlotTables tabs;
  tabs.sys = d_sys;
  tabs.sigma = d_sigma;
  tabs.col = d_col;
  tabs.theta = d_theta_slot;
  tabs.active = d_act;
  tabs.plist = itab + 6 * (size_t)C;
  tabs.poff = itab + 7 * (size_t)C;

  while (true) {
    // ----- cycle boundary: fold directions into y, FP64 true residual, status
    if (occ > 0) {
      const PanelGrid g = make_grid(n, C, occ, ND);
      SlotTables t0 = tabs;
      t0.src = nullptr;
      if (kk_last > 0) {
        Scope sp(h, SLRF_K_RESID, (double)occ * n * (32.0 + kk_last * sT));
        HIPCHK(launch_yupdate<T>(n, g, t0, Ybuf[cur], Zbuf[cur], Pb, vstride, kk_last,
                                 sc.alpha, sc.bhist, s));
      }
      {
        Scope sp(h, SLRF_K_RESID, (double)occ * n * (16.0 + 8.0 + 2 * sT) + 20.0 * h->P.nnz);
        HIPCHK(launch_true_resid<T>(h->P, g, t0, Ybuf[cur], F, nc, Rbuf[cur], Zbuf[cur], part,
                                    pc, s));
      }
      {
        Scope sp(h, SLRF_K_REDUCE, 16.0 * nrb * occ);
        HIPCHK(launch_reduce(part, nrb, ND, C, 1, occ, red, s));
        HIPCHK(launch_fin_true(red, occ, t0, sc, h->opt.tol_lin, inner_rtol, safety, itcap, s));
      }
      HIPCHK(hipMemcpyAsync(hflags, d_status, sizeof(int) * occ, hipMemcpyDeviceToHost, s));
      HIPCHK(hipMemcpyAsync(its_h.data(), sc.sys_its, sizeof(int) * S, hipMemcpyDeviceToHost, s));
      HIPCHK(sync(h));
      for (int i = 0; i < occ; ++i) status[i] = hflags[i];
      if (!h->defer.empty()) {
        std::vector<int> nact_k(m, 0);
        for (int i = 0; i < cyc_occ; ++i) {
          const int steps = h_sys[i] >= 0 ? its_h[h_sys[i]] - its_start[i] : 0;
          for (int k = 0; k < std::min(steps, m); ++k) ++nact_k[k];
        }
        settle_bytes(h, nact_k, cyc_nact0);
      }
    }
    // ----- retire finished systems, compact the survivors, admit new ones
    int nret = 0;
    std::vector<int> keep;
    keep.reserve(occ);
    std::vector<int> h_ret(C, -1);
    for (int i = 0; i < occ; ++i) {
      if (status[i] == 0) {
        keep.push_back(i);
      } else {
        h_ret[i] = h_sys[i];
        ++nret;
        if (status[i] == 3) numeric = true;
      }
    }
    const int nadmit = std::min(C - (int)keep.size(), S - next);
    if (nret > 0) {
      HIPCHK(hipMemcpyAsync(d_retire, h_ret.data(), sizeof(int) * C, hipMemcpyHostToDevice, s));
      const PanelGrid g = make_grid(n, C, occ, ND);
      Scope sp(h, SLRF_K_OTHER, 32.0 * nret * n);
      HIPCHK(launch_retire(n, g, d_retire, Ybuf[cur], Ys, s));
    }
    if (numeric) break;
    if (nret > 0 || nadmit > 0) {
      std::vector<int> ns(C, -1), ncl(C, 0), nsrc(C, -1);
      std::vector<double2> nsg(C, make_double2(0, 0));
      std::vector<double> nth(C, 0.0);
      int t = 0;
      for (int i : keep) {
        ns[t] = h_sys[i];
        ncl[t] = h_col[i];
        nsg[t] = h_sig[i];
        nth[t] = h_th[i];
        nsrc[t] = i;
        ++t;
      }
      for (int a = 0; a < nadmit; ++a, ++t, ++next) {
        const int sys = next, c = sys / N, j = sys % N;
        ns[t] = sys;
        ncl[t] = c;
        nsg[t] = h->poles[j];
        nth[t] = warm ? h_theta_col[c] : 0.0;
        nsrc[t] = -1;
      }
      const int nocc = t;
      h_sys = ns;
      h_col = ncl;
      h_src = nsrc;
      h_sig = nsg;
      h_th = nth;
      HIPCHK(hipMemcpyAsync(d_sys, h_sys.data(), sizeof(int) * C, hipMemcpyHostToDevice, s));
      HIPCHK(hipMemcpyAsync(d_col, h_col.data(), sizeof(int) * C, hipMemcpyHostToDevice, s));
      HIPCHK(hipMemcpyAsync(d_src, h_src.data(), sizeof(int) * C, hipMemcpyHostToDevice, s));
      HIPCHK(hipMemcpyAsync(d_sigma, h_sig.data(), sizeof(double2) * C, hipMemcpyHostToDevice,
                            s));
      HIPCHK(hipMemcpyAsync(d_theta_slot, h_th.data(), sizeof(double) * C,
                            hipMemcpyHostToDevice, s));
      occ = nocc;
      if (occ > 0) {
        const PanelGrid g = make_grid(n, C, occ, ND);
        SlotTables ta = tabs;
        ta.src = d_src;
        {
          Scope sp(h, SLRF_K_OTHER,
                   (double)keep.size() * n * 2 * (16.0 + 2 * sT) +
                       (double)nadmit * n * (16.0 + 2 * sT + (warm ? 16.0 : 8.0)));
          HIPCHK(launch_admit<T>(h->P, g, ta, Ybuf[cur], Rbuf[cur], Zbuf[cur], Ybuf[1 - cur],
                                 Rbuf[1 - cur], Zbuf[1 - cur], F, E, Xr, nc, warm, part, pc, s));
        }
        cur = 1 - cur;
        {
          Scope sp(h, SLRF_K_REDUCE, 16.0 * nrb * occ);
          HIPCHK(launch_reduce(part, nrb, ND, C, 1, occ, red, s));
          HIPCHK(launch_fin_true(red, occ, ta, sc, h->opt.tol_lin, inner_rtol, safety, itcap,
                                 s));
        }
        HIPCHK(hipMemcpyAsync(hflags, d_status, sizeof(int) * occ, hipMemcpyDeviceToHost, s));
        HIPCHK(sync(h));
        for (int i = 0; i < occ; ++i) status[i] = hflags[i];
      }
    }
    if (occ == 0) break;
    for (int i = 0; i < occ; ++i) its_start[i] = h_sys[i] >= 0 ? its_h[h_sys[i]] : 0;
    // active count after the boundary
    int nact = 0;
    for (int i = 0; i < occ; ++i) nact += status[i] == 0 ? 1 : 0;
    kk_last = 0;
    if (nact == 0) continue;  // everything resident is finished: next boundary retires it
    ++cycles;
    // ----- one Krylov cycle (at most m GCR steps)
    const PanelGrid g = make_grid(n, C, occ, ND);
    SlotTables tc = tabs;
    tc.src = nullptr;
    void* R = Rbuf[cur];
    // the preconditioned vectors of the cycle: z_0 in the (compacted) Z buffer,
    // z_k (k >= 1) in the direction store, all kept for the solution update
    auto zk = [&](int k) -> void* {
      return k == 0 ? Zbuf[cur] : static_cast<void*>(static_cast<char*>(Pb) +
                                                     (size_t)k * vstride * sT);
    };
    // The m steps are issued without reading anything back: a system whose
    // cycle ended (inner reduction reached, cap, breakdown) stays inactive and
    // the kernels skip it; the boundary reads the flags once.
    const int nact0 = nact;
    for (int k = 0; k < m; ++k) {
      h->defer_k = k;
      char* Qk = static_cast<char*>(Q) + (size_t)k * vstride * sT;
      // the image w = M z_k: in place in slot k, or (complex bfloat16 basis)
      // in the last slot, whose q is never stored
      void* Wk = hq ? static_cast<char*>(Q) + (size_t)(m - 1) * vstride * sT : Qk;
      const double qb = hq ? 0.5 : 1.0;  // bytes of a stored q relative to w
      void* Z = zk(k);
      if (amg) {
        const slrf_status vs = vcycle<T>(h, av, C, occ, ND, tc, R, Z, nact, fuse0 && k > 0);
        if (vs != SLRF_OK) return vs;
      }
      if (sweep_is_halo<T>(h->P)) {
        Scope sp(h, SLRF_K_APPLY,
                 (double)nact * n * sT * (k > 0 ? 3.0 + qb * k : 2.0) + csr_bytes);
        defer_bytes(h, SLRF_K_APPLY, (double)n * sT * (k > 0 ? 3.0 + qb * k : 2.0));
        {
          Scope sw(h, SLRF_K_SWEEP, (double)nact * n * sT * 2.0 + csr_bytes);
          if (h->cur_stats) h->cur_stats->sweep_systems += nact;
          defer_bytes(h, SLRF_K_SWEEP, (double)n * sT * 2.0, true);
          HIPCHK(launch_sweep<T>(h->P, g, tc, Z, Wk, s));
        }
        HIPCHK(launch_dots<T>(h->P, g, tc, Wk, Q, vstride, k, part, s, hq));
      } else {
        Scope sp(h, SLRF_K_APPLY, (double)nact * n * sT * (k + 2) + csr_bytes);
        defer_bytes(h, SLRF_K_APPLY, (double)n * sT * (k + 2));
        HIPCHK(launch_apply_dots<T>(h->P, g, tc, Z, Qk, Q, vstride, k, part, pc, s));
      }
      if (k > 0) {
        Scope sp(h, SLRF_K_REDUCE, 16.0 * nrb * occ * k);
        HIPCHK(launch_reduce(part, nrb, ND, C, k, occ, red, s));
        HIPCHK(launch_fin_beta(red, k, C, occ, tc, sc, s));
      }
      {
        // q_k is stored unless no later step reads it: the cycle's last q, and
        // (full-precision basis) q_0, which is w itself
        const bool store = k + 1 < m && (hq || k > 0);
        Scope sp(h, SLRF_K_ORTH, (double)nact * n * sT * (2.0 + qb * k + (store ? qb : 0.0)));
        defer_bytes(h, SLRF_K_ORTH, (double)n * sT * (2.0 + qb * k + (store ? qb : 0.0)));
        HIPCHK(launch_orth<T>(h->P, g, tc, Wk, R, Q, vstride, k, sc.beta, part, s, Qk, store,
                              hq));
      }
      {
        Scope sp(h, SLRF_K_REDUCE, 32.0 * nrb * occ);
        HIPCHK(launch_reduce(part, nrb, ND, C, 2, occ, red, s));
        HIPCHK(launch_fin_alpha(red, k, C, occ, tc, sc, s));
      }
      if (k + 1 < m) {
        {
          Scope sp(h, SLRF_K_STEP, (double)nact * n * sT * (3.0 + qb));
          defer_bytes(h, SLRF_K_STEP, (double)n * sT * (3.0 + qb));
          // with the AMG, the step also forms the next V-cycle's level-0
          // pre-smoothing (saves that kernel's read of r)
          void* znext = fuse0 ? av.W0 : zk(k + 1);
          HIPCHK(launch_step<T>(h->P, g, tc, R, znext, Qk, sc.alpha + (size_t)k * C, part,
                                fuse0 ? (amg_level0_bf16<T>(h) ? 4 : 3) : pc,
                                fuse0 ? h->amg.omega[0] : 0.0, s, hq));
        }
        Scope sp(h, SLRF_K_REDUCE, 16.0 * nrb * occ);
        HIPCHK(launch_reduce(part, nrb, ND, C, 1, occ, red, s));
        HIPCHK(launch_fin_rnorm(red, occ, tc, sc, itcap, s));
      } else {
        // last step of the cycle: the boundary recomputes r from y in FP64
        // (and tests it), so the recursive update of r is skipped; the step
        // is only counted
        HIPCHK(launch_fin_rnorm(nullptr, occ, tc, sc, itcap, s));
      }
      kk_last = k + 1;
    }
    h->defer_k = -1;
    cyc_nact0 = nact0;
    cyc_occ = occ;
  }

  // ----- filter sum U = sum_j 2 Re(w_j Y_j) and back to column-major
  {
    Scope sp(h, SLRF_K_OTHER, (double)S * n * 16.0 + 8.0 * n * nc);
    HIPCHK(launch_filter_sum(n, nc, N, Ys, h->d_w, Ur, s));
  }
  {
    Scope sp(h, SLRF_K_OTHER, 16.0 * n * nc);
    HIPCHK(launch_transpose(Ur, n, nc, nc, U, n, s, nullptr, h->order));
  }
  // ----- statistics
  std::vector<int> its(S);
  std::vector<double> rn2(S), f2(nc);
  HIPCHK(hipMemcpyAsync(its.data(), sc.sys_its, sizeof(int) * S, hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(rn2.data(), sc.sys_rn2, sizeof(double) * S, hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(f2.data(), fn2, sizeof(double) * nc, hipMemcpyDeviceToHost, s));
  HIPCHK(sync(h));
  int conv = 0, capped = 0;
  double maxrel = 0.0;
  int64_t tot = 0;
  int mn = S > 0 ? its[0] : 0, mx = 0;
  std::vector<int64_t> pole_sum(N, 0);
  for (int sys = 0; sys < S; ++sys) {
    const int c = sys / N;
    const double rel = f2[c] > 0 ? std::sqrt(rn2[sys] / f2[c]) : std::sqrt(rn2[sys]);
    const bool ok = rn2[sys] <= h->opt.tol_lin * h->opt.tol_lin * f2[c];
    conv += ok ? 1 : 0;
    capped += ok ? 0 : 1;
    maxrel = std::max(maxrel, rel);
    tot += its[sys];
    mn = std::min(mn, its[sys]);
    mx = std::max(mx, its[sys]);
    pole_sum[sys % N] += its[sys];
  }
  if (st) {
    st->nsystems = S;
    st->total_iters = tot;
    st->min_iters = mn;
    st->max_iters = mx;
    st->cycles = cycles;
    st->converged = conv;
    st->capped = capped;
    int64_t pmin = INT64_MAX, pmax = 0;
    for (int j = 0; j < N; ++j) {
      pmin = std::min(pmin, pole_sum[j]);
      pmax = std::max(pmax, pole_sum[j]);
    }
    st->max_pole_iters_ratio_x1000 = pmin > 0 ? (int32_t)(1000.0 * pmax / pmin) : 0;
    st->max_rel_resid = maxrel;
    st->spmm_variant = std::is_same<T, float>::value ? h->P.var32 : h->P.var64;
    st->basis_bf16 = hq ? 1 : 0;
    if (st->sys_iters) std::memcpy(st->sys_iters, its.data(), sizeof(int) * S);
    st->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
  if (numeric) return fail(h, SLRF_E_NUMERIC, "NaN or Inf in a residual norm");
  if (capped > 0 && h->opt.it_max_lin == 0)
    return fail(h, SLRF_E_NOCONV, "some shifted systems reached maxit_lin before tol_lin");
  return SLRF_OK;
}

// ---------------------------------------------------------------------------
// Rayleigh-Ritz on a row-major block (internal)
// ---------------------------------------------------------------------------
// Ur: n x nc row-major (in: filtered block; out: Ritz vectors V).  Xl/BXl:
// row-major n x nl locked vectors and B times them.  Outputs: theta_h, res_h
// (host), and AV/BV (row-major) when the buffers are given.
slrf_status rr_rowmajor(slrf_ctx* h, int nc, double* Ur, int nl, const double* Xl,
                        const double* BXl, std::vector<double>& theta_h,
                        std::vector<double>& res_h, double** BV_out) {
  const int n = h->P.n;
  hipStream_t s = h->stream;
  double *AU, *BU, *V, *AV, *BV, *gpart, *small, *cpart;
  HIPCHK(carve_t(h, (size_t)n * nc, &AU));
  HIPCHK(carve_t(h, (size_t)n * nc, &BU));
  HIPCHK(carve_t(h, (size_t)n * nc, &V));
  HIPCHK(carve_t(h, (size_t)n * nc, &AV));
  HIPCHK(carve_t(h, (size_t)n * nc, &BV));
  const int pq = std::max(nc, nl);
  HIPCHK(carve_t(h, gram_part_doubles(n, pq) + 16, &gpart));
  HIPCHK(carve_t(h, (size_t)3 * pq * pq + 4 * pq + 16, &small));
  const int cch = colstat_chunks(n);
  HIPCHK(carve_t(h, (size_t)2 * cch * nc + 2, &cpart));
  double* Gd = small;                          // nc x nc or nl x nc
  double* Gd2 = small + (size_t)pq * pq;       // second Gram
  double* Sd = small + (size_t)2 * pq * pq;    // S
  double* thd = small + (size_t)3 * pq * pq;   // theta (device)
  double* r2 = thd + pq;
  double* vb = r2 + pq;

  if (nl > 0) {
    // U <- U - X (X^T B U), twice (Algorithm 2, B-orthogonalisation vs locked X)
    HIPCHK(launch_spmm_real(h->P, Ur, nc, nc, nullptr, BU, nullptr, nullptr, s));
    for (int pass = 0; pass < 2; ++pass) {
      HIPCHK(launch_gram(n, nl, nc, Xl, nl, BU, nc, gpart, Gd, nc, s));
      HIPCHK(launch_gemm_tall(n, nl, nc, -1.0, Xl, nl, Gd, nc, 1.0, Ur, nc, s));
      if (pass == 0) HIPCHK(launch_gemm_tall(n, nl, nc, -1.0, BXl, nl, Gd, nc, 1.0, BU, nc, s));
    }
  }
  HIPCHK(launch_spmm_real(h->P, Ur, nc, nc, AU, BU, nullptr, nullptr, s));
  HIPCHK(launch_gram(n, nc, nc, Ur, nc, AU, nc, gpart, Gd, nc, s));
  HIPCHK(launch_gram(n, nc, nc, Ur, nc, BU, nc, gpart, Gd2, nc, s));
  std::vector<double> Ah((size_t)nc * nc), Bh((size_t)nc * nc), Sh((size_t)nc * nc);
  HIPCHK(hipMemcpyAsync(Ah.data(), Gd, sizeof(double) * nc * nc, hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(Bh.data(), Gd2, sizeof(double) * nc * nc, hipMemcpyDeviceToHost, s));
  HIPCHK(sync(h));
  theta_h.assign(nc, 0.0);
  int fb = 0;
  const int kgood = sym_gen_eig(nc, Ah.data(), Bh.data(), theta_h.data(), Sh.data(), &fb);
  if (kgood < 0) return fail(h, SLRF_E_BREAKDOWN, "projected eigenproblem failed");
  HIPCHK(hipMemcpyAsync(Sd, Sh.data(), sizeof(double) * nc * nc, hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(thd, theta_h.data(), sizeof(double) * nc, hipMemcpyHostToDevice, s));
  HIPCHK(launch_gemm_tall(n, nc, nc, 1.0, Ur, nc, Sd, nc, 0.0, V, nc, s));
  HIPCHK(launch_gemm_tall(n, nc, nc, 1.0, AU, nc, Sd, nc, 0.0, AV, nc, s));
  HIPCHK(launch_gemm_tall(n, nc, nc, 1.0, BU, nc, Sd, nc, 0.0, BV, nc, s));
  // residual norms ||AV - theta BV|| and ||v||_B^2 = v^T B v
  std::vector<double> thr(theta_h);
  for (auto& t : thr)
    if (!std::isfinite(t)) t = 0.0;
  HIPCHK(hipMemcpyAsync(thd, thr.data(), sizeof(double) * nc, hipMemcpyHostToDevice, s));
  HIPCHK(launch_colstats(n, nc, AV, BV, nc, thd, V, cpart, cch, r2, vb, s));
  HIPCHK(hipMemcpyAsync(Ur, V, sizeof(double) * n * nc, hipMemcpyDeviceToDevice, s));
  std::vector<double> r2h(nc), vbh(nc);
  HIPCHK(hipMemcpyAsync(r2h.data(), r2, sizeof(double) * nc, hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(vbh.data(), vb, sizeof(double) * nc, hipMemcpyDeviceToHost, s));
  HIPCHK(sync(h));
  res_h.assign(nc, HUGE_VAL);
  for (int c = 0; c < nc; ++c) {
    if (c >= kgood || !std::isfinite(theta_h[c])) continue;
    const double den = std::fabs(theta_h[c]) * std::sqrt(std::max(vbh[c], 0.0));
    res_h[c] = den > 0 ? std::sqrt(std::max(r2h[c], 0.0)) / den : HUGE_VAL;
  }
  if (BV_out) *BV_out = BV;
  return SLRF_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// Allocation-free sweep: a per-device scratch array for the pole table of
// slrf_shifted_spmm_noalloc.  Host code never passes the array's name to a
// kernel or a copy: its device address is looked up once per device (with that
// device current, at the first slrf_setup on it) and that address is used.
// ---------------------------------------------------------------------------
namespace {

constexpr int kNoallocMaxSys = 65536;  // systems per call (a 1 MiB pole table)
constexpr int kNoallocMaxDev = 64;

__device__ __align__(256) double2 scratch[kNoallocMaxSys];

std::mutex g_scratch_mu;
void* g_scratch_ptr[kNoallocMaxDev] = {};

// Resolve (once) the address of this device's copy of `scratch`; the device
// must be current.  Returns nullptr on failure.
void* scratch_address(int device) {
  if (device < 0 || device >= kNoallocMaxDev) return nullptr;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess) return nullptr;
    g_scratch_ptr[device] = ptr;
  }
  return g_scratch_ptr[device];
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
// ---------------------------------------------------------------------------
// Batched entry points: a pool of host threads drains a queue of handles in
// descending order of work; each thread drives its handle's pool loop on the
// handle's stream, so kernels of different pencils overlap on the device.
// ---------------------------------------------------------------------------
namespace {

template <typename F>
slrf_status run_batch(int32_t nh, const slrf_handle* hs, const std::vector<double>& work,
                      int32_t nthreads, F&& one) {
  std::vector<int> order(nh);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return work[a] > work[b]; });
  std::vector<slrf_status> res(nh, SLRF_OK);
  std::atomic<int> next{0};
  const int nt = std::max(1, std::min<int>(nthreads > 0 ? nthreads : 8, nh));
  auto worker = [&]() {
    // each handle works in its own workspace
    for (;;) {
      const int k = next.fetch_add(1);
      if (k >= nh) break;
      const int i = order[k];
      if (hipSetDevice(hs[i]->device) != hipSuccess) {
        res[i] = SLRF_E_HIP;
        continue;
      }
      res[i] = one(i);
      (void)hipStreamSynchronize(hs[i]->stream);
    }
  };
  std::vector<std::thread> pool;
  for (int t = 1; t < nt; ++t) pool.emplace_back(worker);
  worker();
  for (auto& th : pool) th.join();
  for (int i = 0; i < nh; ++i)
    if (res[i] != SLRF_OK) return res[i];
  return SLRF_OK;
}

bool distinct_handles(int32_t nh, const slrf_handle* hs) {
  std::vector<slrf_handle> v(hs, hs + nh);
  std::sort(v.begin(), v.end());
  return std::adjacent_find(v.begin(), v.end()) == v.end() &&
         std::find(v.begin(), v.end(), nullptr) == v.end();
}

}  // namespace

extern "C" {

const char* slrf_status_string(slrf_status s) {
  switch (s) {
    case SLRF_OK: return "ok";
    case SLRF_E_ARG: return "invalid argument";
    case SLRF_E_NOMEM: return "out of memory";
    case SLRF_E_HIP: return "HIP runtime error";
    case SLRF_E_BREAKDOWN: return "breakdown in the projected problem";
    case SLRF_E_NOCONV: return "iteration cap reached";
    case SLRF_E_NUMERIC: return "NaN or Inf detected";
    case SLRF_E_NOGPU: return "no usable GPU";
  }
  return "unknown status";
}

const char* slrf_last_error(slrf_handle h) { return h ? h->err.c_str() : "null handle"; }

void slrf_default_options(slrf_options* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->precision = SLRF_PREC_FP64;
  o->precond = SLRF_PC_JACOBI;
  o->restart = 30;
  o->maxit_lin = 10000;
  o->it_max_lin = 0;
  o->max_outer = 100;
  o->warm_start = 0;
  o->lock = 0;
  o->timing = 0;
  o->max_slots = 0;
  o->reorder = 1;
  o->spmm_variant = 0;
  o->tol_lin = 1e-10;
  o->inner_rtol = 1e-5;
  o->tol_eig = 1e-8;
  o->amg_block = 0;
  o->node_xyz = nullptr;
  o->amg_setup = SLRF_AMG_HOST;
  o->amg_coarse_min = 0;
}

int32_t slrf_get_n(slrf_handle h) { return h ? h->P.n : -1; }

slrf_status slrf_get_row_order(slrf_handle h, int32_t* order) {
  if (!h || !order) return SLRF_E_ARG;
  for (int i = 0; i < h->P.n; ++i) order[i] = h->h_order.empty() ? i : h->h_order[i];
  return SLRF_OK;
}

slrf_status slrf_workspace_size(const slrf_csr* A, const slrf_csr* B, int32_t L, int32_t npoles,
                                const slrf_options* opt, size_t* full_bytes, size_t* min_bytes) {
  if (!full_bytes || L < 1 || npoles < 1 || npoles > 64) return SLRF_E_ARG;
  slrf_options o;
  if (opt) o = *opt; else slrf_default_options(&o);
  if (validate_options(nullptr, o) != SLRF_OK) return SLRF_E_ARG;
  std::string err;
  slrf_status st;
  auto hs = analyse(A, B, o, err, st);
  if (!hs) return st;
  size_t pers = persistent_bytes(*hs, npoles);
  std::vector<int> lev;
  for (auto& lv : hs->H.levels) lev.push_back(lv.n);
  if (hs->amg_device) {
    // (the hierarchy is built by slrf_setup: a bound, and coarse levels taken
    // to hold at most half the fine rows)
    pers += amg_device_bound(*hs, npoles);
    lev = {hs->n, std::max(1, hs->n / 2)};
  }
  const int S = npoles * L;
  int full = (S + kPanel - 1) / kPanel * kPanel;
  if (o.max_slots > 0) full = std::min(full, o.max_slots);
  *full_bytes = pers + call_bytes(hs->n, L, npoles, o, lev, full);
  if (min_bytes) *min_bytes = pers + call_bytes(hs->n, L, npoles, o, lev, kPanel);
  return SLRF_OK;
}

slrf_status slrf_setup(slrf_handle* out, const slrf_csr* A, const slrf_csr* B, double gamma,
                       int32_t npoles, const slrf_zd* poles, const slrf_zd* weights,
                       const slrf_options* opt, void* workspace, size_t ws_bytes, void* stream) {
  if (!out) return SLRF_E_ARG;
  *out = nullptr;
  auto* h = new (std::nothrow) slrf_ctx();
  if (!h) return SLRF_E_NOMEM;
  auto bad = [&](slrf_status st, const std::string& m) {
    h->err = m;
    *out = h;  // hand the handle back so slrf_last_error works; caller destroys
    return st;
  };
  if (!A || !B || !poles || !weights) return bad(SLRF_E_ARG, "null argument");
  if (!workspace || ws_bytes < 2 * kAlign)
    return bad(SLRF_E_ARG, "a device workspace is required (size it with slrf_workspace_size)");
  if (!(gamma > 0.0) || !std::isfinite(gamma)) return bad(SLRF_E_ARG, "gamma must be > 0");
  if (npoles < 1 || npoles > 64) return bad(SLRF_E_ARG, "npoles must be in [1, 64]");
  if (opt) h->opt = *opt; else slrf_default_options(&h->opt);
  {
    slrf_status vs = validate_options(h, h->opt);
    if (vs != SLRF_OK) {
      *out = h;
      return vs;
    }
  }
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev == 0)
    return bad(SLRF_E_NOGPU, "no HIP device visible");
  if (hipGetDevice(&h->device) != hipSuccess) return bad(SLRF_E_NOGPU, "hipGetDevice failed");
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, h->device) != hipSuccess)
    return bad(SLRF_E_NOGPU, "hipGetDeviceProperties failed");
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    return bad(SLRF_E_NOGPU, std::string("library built for gfx950, device is ") + prop.gcnArchName);
  if (!scratch_address(h->device))
    return bad(SLRF_E_HIP, "address of the sweep scratch array could not be resolved");
  h->stream = static_cast<hipStream_t>(stream);
  for (int j = 0; j < npoles; ++j) {
    if (!(poles[j].im > 0.0)) return bad(SLRF_E_ARG, "poles must lie in the upper half plane");
    if (!std::isfinite(poles[j].re) || !std::isfinite(weights[j].re) ||
        !std::isfinite(weights[j].im))
      return bad(SLRF_E_ARG, "non-finite pole or weight");
    h->poles.push_back(make_double2(poles[j].re, poles[j].im));
    h->weights.push_back(make_double2(weights[j].re, weights[j].im));
  }
  h->N = npoles;
  h->gamma = gamma;
  {
    // the workspace, from its first 256-byte boundary
    const uintptr_t p0 = reinterpret_cast<uintptr_t>(workspace);
    const uintptr_t p1 = (p0 + kAlign - 1) / kAlign * kAlign;
    h->ar.base = reinterpret_cast<char*>(p1);
    h->ar.cap = ws_bytes - (size_t)(p1 - p0);
    h->ar.top = 0;
  }
  std::string err;
  slrf_status ast;
  auto hs = analyse(A, B, h->opt, err, ast);
  if (!hs) return bad(ast, err);
  h->block = hs->block;
  h->h_order = hs->order;
  hipStream_t s = h->stream;
  // SLRF_AMG_DEVICE: the hierarchy built here (products on the GPU)
  AmgHierarchy Hdev;
  std::vector<HostImage> imgdev;
  const AmgHierarchy* Hp = hs->has_amg ? &hs->H : nullptr;
  const std::vector<HostImage>* imgp = hs->has_amg ? &hs->img : nullptr;
  {
    Placer pl{h, false};
    hipError_t e = place_pencil(h, *hs, pl, A, B);
    if (e == hipSuccess && hs->amg_device) {
      // the products run in the workspace above the pencil data and are
      // released level by level, before the hierarchy itself is placed there
      HostLevel fine;
      fine.n = hs->n;
      fine.rp = hs->rp;
      fine.ci = hs->ci;
      fine.a = hs->a;
      fine.b = hs->b;
      AmgParams prm = hs->amg_prm;
      if (!hs->amg_xyz.empty()) prm.xyz = &hs->amg_xyz;
      DeviceAmgNumeric num;
      num.stream = s;
      const size_t top0 = h->ar.top;
      size_t short_by = 0;
      num.take = [h, &short_by](size_t bytes) -> void* {
        void* p = nullptr;
        if (carve(h, bytes, &p) != hipSuccess) {
          short_by = std::max(short_by, h->ar.short_by);
          return nullptr;
        }
        return p;
      };
      num.release = [h, top0]() { h->ar.top = top0; };
      std::string aerr;
      const bool built = amg_build(fine, {}, prm, Hdev, aerr, &num);
      h->ar.top = top0;
      if (!built) {
        if (short_by > 0) {
          char buf[256];
          std::snprintf(buf, sizeof(buf),
                        "workspace too small for the device AMG setup (%zu more bytes needed)",
                        short_by);
          return bad(SLRF_E_NOMEM, buf);
        }
        return bad(SLRF_E_ARG, "AMG setup: " + aerr);
      }
      amg_images(Hdev, imgdev);
      Hp = &Hdev;
      imgp = &imgdev;
    }
    if (e == hipSuccess && Hp) e = place_amg(h, *Hp, *imgp, pl, npoles);
    if (e == hipErrorOutOfMemory) {
      char buf[256];
      std::snprintf(buf, sizeof(buf),
                    "workspace of %zu bytes too small for the pencil data (%zu bytes; see "
                    "slrf_workspace_size)",
                    h->ar.cap,
                    persistent_bytes(*hs, npoles) +
                        (hs->amg_device ? amg_device_bound(*hs, npoles) : 0));
      return bad(SLRF_E_NOMEM, buf);
    }
    if (e != hipSuccess) return bad(SLRF_E_HIP, "upload of the pencil data failed");
  }
  if (Hp) {
    // per-pole dense inverses of the coarsest level operators
    AmgHierarchy top;
    top.levels.push_back(Hp->levels.back());
    std::vector<std::complex<double>> pz;
    for (auto& p : h->poles) pz.emplace_back(p.x, p.y);
    std::string aerr;
    if (!amg_coarse_inverses(top, pz, aerr)) return bad(SLRF_E_ARG, "AMG setup: " + aerr);
    std::vector<double2> i64(top.coarse_inv.size());
    std::vector<float2> i32(top.coarse_inv.size());
    for (size_t i = 0; i < top.coarse_inv.size(); ++i) {
      i64[i] = make_double2(top.coarse_inv[i].real(), top.coarse_inv[i].imag());
      i32[i] = make_float2((float)top.coarse_inv[i].real(), (float)top.coarse_inv[i].imag());
    }
    if (hipMemcpy(h->amg.inv64, i64.data(), sizeof(double2) * i64.size(), hipMemcpyHostToDevice) ||
        hipMemcpy(h->amg.inv32, i32.data(), sizeof(float2) * i32.size(), hipMemcpyHostToDevice))
      return bad(SLRF_E_HIP, "upload of the AMG coarse inverses failed");
  }
  h->ar.persist = h->ar.top;
  {
    // FP32 values, diagonals (a missing one is flagged), pole weights
    Frame fr(h);
    int* d_missing = nullptr;
    int missing = 0;
    if (carve_t(h, 1, &d_missing) != hipSuccess)
      return bad(SLRF_E_NOMEM, "workspace too small for setup");
    if (hipMemsetAsync(d_missing, 0, sizeof(int), s) ||
        launch_cast_f32(h->P.a, h->a32, hs->nnz, s) ||
        launch_cast_f32(h->P.b, h->b32, hs->nnz, s) ||
        launch_diag(h->P, h->da, h->db, d_missing, s) ||
        hipMemcpyAsync(h->d_w, h->weights.data(), sizeof(double2) * npoles,
                       hipMemcpyHostToDevice, s) ||
        hipMemcpyAsync(&missing, d_missing, sizeof(int), hipMemcpyDeviceToHost, s) ||
        hipStreamSynchronize(s))
      return bad(SLRF_E_HIP, "setup kernels failed");
    if (missing) return bad(SLRF_E_ARG, "missing diagonal entry");
  }
  h->P.var32 = h->P.var64 = h->opt.spmm_variant;
  if (h->opt.spmm_variant == kSpmmAuto && hs->n >= 4096) {
    const slrf_status ts = autotune_spmm(h);
    if (ts != SLRF_OK) {
      *out = h;
      return ts;
    }
  }
  *out = h;
  return SLRF_OK;
}

void slrf_destroy(slrf_handle h) {
  if (!h) return;
  if (h->stream) (void)hipStreamSynchronize(h->stream);
  else (void)hipDeviceSynchronize();
  delete h;  // (the workspace belongs to the caller)
}

slrf_status slrf_set_options(slrf_handle h, const slrf_options* opt) {
  if (!h || !opt) return SLRF_E_ARG;
  slrf_status s = validate_options(h, *opt);
  if (s != SLRF_OK) return s;
  if (opt->precond == SLRF_PC_AMG && !h->amg.ready)
    return fail(h, SLRF_E_ARG, "the AMG hierarchy is built at setup: set precond there");
  if (opt->reorder != h->opt.reorder || opt->amg_block != h->opt.amg_block ||
      opt->amg_setup != h->opt.amg_setup || opt->amg_coarse_min != h->opt.amg_coarse_min)
    return fail(h, SLRF_E_ARG,
                "reorder, amg_block, amg_setup and amg_coarse_min are fixed at setup");
  h->opt = *opt;
  if (opt->spmm_variant != kSpmmAuto) h->P.var32 = h->P.var64 = opt->spmm_variant;
  return SLRF_OK;
}

slrf_status slrf_filter(slrf_handle h, int32_t ncols, const double* X, const double* theta_warm,
                        double* U, slrf_filter_stats* st) {
  if (!h) return SLRF_E_ARG;
  if (ncols < 1 || !X || !U) return fail(h, SLRF_E_ARG, "ncols >= 1 and non-null X, U required");
  if (X == U) return fail(h, SLRF_E_ARG, "U may not alias X");
  if (st) {
    int32_t* keep = st->sys_iters;
    std::memset(st, 0, sizeof(*st));
    st->sys_iters = keep;
  }
  h->cur_stats = st;
  Frame fr(h);
  slrf_status r = h->opt.precision == SLRF_PREC_MIXED
                      ? run_filter<float>(h, ncols, X, theta_warm, U, st)
                      : run_filter<double>(h, ncols, X, theta_warm, U, st);
  h->cur_stats = nullptr;
  h->timer.reset();
  return r;
}

slrf_status slrf_rayleigh_ritz(slrf_handle h, int32_t ncols, double* U, int32_t nlocked,
                               const double* Xlocked, double* theta, double* resid) {
  if (!h) return SLRF_E_ARG;
  if (ncols < 1 || !U || !theta || !resid || nlocked < 0 || (nlocked > 0 && !Xlocked))
    return fail(h, SLRF_E_ARG, "bad Rayleigh-Ritz arguments");
  const int n = h->P.n;
  hipStream_t s = h->stream;
  Frame fr(h);
  double *Ur, *Xl = nullptr, *BXl = nullptr;
  HIPCHK(carve_t(h, (size_t)n * ncols, &Ur));
  HIPCHK(launch_transpose(U, ncols, n, n, Ur, ncols, s, h->order));
  if (nlocked > 0) {
    HIPCHK(carve_t(h, (size_t)n * nlocked, &Xl));
    HIPCHK(carve_t(h, (size_t)n * nlocked, &BXl));
    HIPCHK(launch_transpose(Xlocked, nlocked, n, n, Xl, nlocked, s, h->order));
    HIPCHK(launch_spmm_real(h->P, Xl, nlocked, nlocked, nullptr, BXl, nullptr, nullptr, s));
  }
  std::vector<double> th, res;
  slrf_status r = rr_rowmajor(h, ncols, Ur, nlocked, Xl, BXl, th, res, nullptr);
  if (r != SLRF_OK) return r;
  HIPCHK(launch_transpose(Ur, n, ncols, ncols, U, n, s, nullptr, h->order));
  HIPCHK(hipMemcpyAsync(theta, th.data(), sizeof(double) * ncols, hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(resid, res.data(), sizeof(double) * ncols, hipMemcpyHostToDevice, s));
  HIPCHK(hipStreamSynchronize(s));
  return SLRF_OK;
}

slrf_status slrf_solve(slrf_handle h, int32_t nev, int32_t L, const double* V1, double* theta_out,
                       double* X_out, int32_t* nconv_out, slrf_solve_stats* stats) {
  if (!h) return SLRF_E_ARG;
  if (nev < 1 || L < nev || !V1 || !theta_out || !X_out)
    return fail(h, SLRF_E_ARG, "need 1 <= nev <= L and non-null buffers");
  const auto t0 = std::chrono::steady_clock::now();
  const int n = h->P.n;
  hipStream_t s = h->stream;
  const bool alg2 = h->opt.lock != 0;
  const bool warm = h->opt.warm_start != 0;
  if (nconv_out) *nconv_out = 0;
  if (stats) std::memset(stats, 0, sizeof(*stats));
  Frame fr(h);
  double *V, *U, *Xlk, *th_d;
  HIPCHK(carve_t(h, (size_t)n * (2 * L + nev) + 2 * L + 16, &V));
  U = V + (size_t)n * L;
  Xlk = U + (size_t)n * L;  // locked vectors, column-major n x nev
  th_d = Xlk + (size_t)n * nev;
  HIPCHK(hipMemcpyAsync(V, V1, sizeof(double) * n * L, hipMemcpyDeviceToDevice, s));
  std::vector<double> Theta;  // locked values
  std::vector<double> th_warm;
  int nconv = 0;
  slrf_status result = SLRF_E_NOCONV;
  std::vector<double> lastTheta;
  std::vector<int> lastIdx;
  double fsec = 0, rsec = 0;
  int auto_cap = 0;  // automatic It_max-linear (it_max_lin = -1)
  int k = 1;
  for (; k <= h->opt.max_outer; ++k) {
    const int nact = alg2 ? L - nconv : L;
    if (nact <= 0) break;
    slrf_filter_stats fst;
    std::memset(&fst, 0, sizeof(fst));
    // automatic It_max-linear: the first outer iteration solves to tol_lin and
    // its per-system iteration counts set the cap of the later (warm-started)
    // ones
    const int itmax_user = h->opt.it_max_lin;
    std::vector<int32_t> its_first;
    if (itmax_user < 0) {
      if (k == 1) {
        its_first.assign((size_t)nact * h->N, 0);
        fst.sys_iters = its_first.data();
        h->opt.it_max_lin = 0;
      } else {
        h->opt.it_max_lin = auto_cap;
      }
    }
    if (warm && !th_warm.empty())
      HIPCHK(hipMemcpyAsync(th_d, th_warm.data(), sizeof(double) * nact, hipMemcpyHostToDevice,
                            s));
    const auto tf = std::chrono::steady_clock::now();
    slrf_status fs = slrf_filter(h, nact, V, (warm && !th_warm.empty()) ? th_d : nullptr, U, &fst);
    h->opt.it_max_lin = itmax_user;
    if (fs != SLRF_OK && fs != SLRF_E_NOCONV) return fs;
    if (itmax_user < 0 && k == 1 && !its_first.empty()) {
      std::vector<int32_t> v(its_first);
      std::nth_element(v.begin(), v.begin() + v.size() / 2, v.end());
      auto_cap = std::max(kAutoItMaxMin, (int)std::ceil(kAutoItMaxFrac * v[v.size() / 2]));
    }
    fsec += std::chrono::duration<double>(std::chrono::steady_clock::now() - tf).count();
    if (stats) stats->inner_iters += fst.total_iters;
    // Rayleigh-Ritz (with B-orthogonalisation against the locked set)
    const auto tr = std::chrono::steady_clock::now();
    Frame fit(h);
    double *Ur, *Xl = nullptr, *BXl = nullptr;
    HIPCHK(carve_t(h, (size_t)n * nact, &Ur));
    HIPCHK(launch_transpose(U, nact, n, n, Ur, nact, s, h->order));
    const int nl = alg2 ? nconv : 0;
    if (nl > 0) {
      HIPCHK(carve_t(h, (size_t)n * nl, &Xl));
      HIPCHK(carve_t(h, (size_t)n * nl, &BXl));
      HIPCHK(launch_transpose(Xlk, nl, n, n, Xl, nl, s, h->order));
      HIPCHK(launch_spmm_real(h->P, Xl, nl, nl, nullptr, BXl, nullptr, nullptr, s));
    }
    std::vector<double> th, res;
    slrf_status r = rr_rowmajor(h, nact, Ur, nl, Xl, BXl, th, res, nullptr);
    if (r != SLRF_OK) return r;
    HIPCHK(launch_transpose(Ur, n, nact, nact, U, n, s, nullptr, h->order));  // Ritz vectors
    rsec += std::chrono::duration<double>(std::chrono::steady_clock::now() - tr).count();
    std::vector<int> conv, rest;
    for (int c = 0; c < nact; ++c) {
      const bool ok = th[c] > 0.0 && th[c] <= h->gamma && res[c] < h->opt.tol_eig;
      (ok ? conv : rest).push_back(c);
    }
    if (!alg2) {
      lastTheta = th;
      lastIdx = conv;
      if ((int)conv.size() >= nev) {
        for (int i = 0; i < nev; ++i)
          HIPCHK(hipMemcpyAsync(X_out + (size_t)i * n, U + (size_t)conv[i] * n,
                                sizeof(double) * n, hipMemcpyDeviceToDevice, s));
        std::vector<double> tout(nev);
        for (int i = 0; i < nev; ++i) tout[i] = th[conv[i]];
        HIPCHK(hipMemcpyAsync(theta_out, tout.data(), sizeof(double) * nev,
                              hipMemcpyHostToDevice, s));
        nconv = nev;
        result = SLRF_OK;
        break;
      }
      std::swap(V, U);  // V_{k+1} = all Ritz vectors
      th_warm = th;
    } else {
      for (int c : conv) {
        if (nconv >= nev) break;
        HIPCHK(hipMemcpyAsync(Xlk + (size_t)nconv * n, U + (size_t)c * n, sizeof(double) * n,
                              hipMemcpyDeviceToDevice, s));
        Theta.push_back(th[c]);
        ++nconv;
      }
      if (nconv >= nev) {
        result = SLRF_OK;
        break;
      }
      const int nnext = L - nconv;
      th_warm.clear();
      for (int i = 0; i < nnext && i < (int)rest.size(); ++i) {
        HIPCHK(hipMemcpyAsync(V + (size_t)i * n, U + (size_t)rest[i] * n, sizeof(double) * n,
                              hipMemcpyDeviceToDevice, s));
        th_warm.push_back(th[rest[i]]);
      }
      // fewer unconverged Ritz vectors than needed cannot happen (nact - |conv| = L - nconv)
    }
  }
  if (alg2) {
    // sort the locked pairs ascending into the outputs
    std::vector<int> ord(Theta.size());
    for (size_t i = 0; i < ord.size(); ++i) ord[i] = (int)i;
    std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) { return Theta[a] < Theta[b]; });
    const int nout = std::min<int>(nev, (int)ord.size());
    std::vector<double> tout(nout);
    for (int i = 0; i < nout; ++i) {
      tout[i] = Theta[ord[i]];
      HIPCHK(hipMemcpyAsync(X_out + (size_t)i * n, Xlk + (size_t)ord[i] * n, sizeof(double) * n,
                            hipMemcpyDeviceToDevice, s));
    }
    if (nout > 0)
      HIPCHK(hipMemcpyAsync(theta_out, tout.data(), sizeof(double) * nout, hipMemcpyHostToDevice,
                            s));
  } else if (result != SLRF_OK) {
    const int nout = std::min<int>(nev, (int)lastIdx.size());
    std::vector<double> tout(nout);
    for (int i = 0; i < nout; ++i) {
      tout[i] = lastTheta[lastIdx[i]];
      HIPCHK(hipMemcpyAsync(X_out + (size_t)i * n, V + (size_t)lastIdx[i] * n,
                            sizeof(double) * n, hipMemcpyDeviceToDevice, s));
    }
    if (nout > 0)
      HIPCHK(hipMemcpyAsync(theta_out, tout.data(), sizeof(double) * nout, hipMemcpyHostToDevice,
                            s));
    nconv = nout;
  }
  HIPCHK(hipStreamSynchronize(s));
  if (nconv_out) *nconv_out = nconv;
  if (stats) {
    stats->outer_iters = std::min(k, h->opt.max_outer);
    stats->auto_it_max = h->opt.it_max_lin < 0 ? auto_cap : 0;
    stats->nconv = nconv;
    stats->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    stats->filter_seconds = fsec;
    stats->rr_seconds = rsec;
  }
  if (result != SLRF_OK) return fail(h, SLRF_E_NOCONV, "max_outer reached before nev pairs");
  return SLRF_OK;
}

slrf_status slrf_shifted_spmm(slrf_handle h, int32_t nsys, const int32_t* pole, int32_t precision,
                              const void* Z, void* Q, double* ms_out) {
  if (!h) return SLRF_E_ARG;
  if (nsys < 1 || !pole || !Z || !Q) return fail(h, SLRF_E_ARG, "bad shifted_spmm arguments");
  if (precision != SLRF_PREC_FP64 && precision != SLRF_PREC_MIXED)
    return fail(h, SLRF_E_ARG, "bad precision");
  const int C = (nsys + kPanel - 1) / kPanel * kPanel;
  std::vector<double2> sg(C, make_double2(0.0, 0.0));
  for (int i = 0; i < nsys; ++i) {
    if (pole[i] < 0 || pole[i] >= h->N) return fail(h, SLRF_E_ARG, "pole index out of range");
    sg[i] = h->poles[pole[i]];
  }
  Frame fr(h);
  double* dtab;
  HIPCHK(carve_t(h, (size_t)3 * C, &dtab));
  hipStream_t s = h->stream;
  HIPCHK(hipMemcpyAsync(dtab, sg.data(), sizeof(double2) * C, hipMemcpyHostToDevice, s));
  const PanelGrid g = make_grid(h->P.n, C, C, 2);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (ms_out) {
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    HIPCHK(hipEventRecord(e0, s));
  }
  const double2* sgd = reinterpret_cast<const double2*>(dtab);
  if (precision == SLRF_PREC_FP64)
    HIPCHK(launch_spmm_panel<double>(h->P, g, sgd, Z, Q, s));
  else
    HIPCHK(launch_spmm_panel<float>(h->P, g, sgd, Z, Q, s));
  if (ms_out) {
    HIPCHK(hipEventRecord(e1, s));
    HIPCHK(hipEventSynchronize(e1));
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, e0, e1));
    *ms_out = ms;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
  } else {
    HIPCHK(hipStreamSynchronize(s));
  }
  return SLRF_OK;
}

slrf_status slrf_shifted_spmm_noalloc(slrf_handle h, int32_t nsys, const int32_t* pole,
                                      int32_t precision, const void* Z, void* Q) {
  if (!h) return SLRF_E_ARG;
  if (nsys < 1 || !pole || !Z || !Q) return fail(h, SLRF_E_ARG, "bad shifted_spmm arguments");
  if (precision != SLRF_PREC_FP64 && precision != SLRF_PREC_MIXED)
    return fail(h, SLRF_E_ARG, "bad precision");
  const int C = (nsys + kPanel - 1) / kPanel * kPanel;
  if (C > kNoallocMaxSys)
    return fail(h, SLRF_E_ARG, "slrf_shifted_spmm_noalloc: nsys rounded up to 16 exceeds the "
                               "65536 systems of the scratch pole table");
  for (int i = 0; i < nsys; ++i)
    if (pole[i] < 0 || pole[i] >= h->N) return fail(h, SLRF_E_ARG, "pole index out of range");
  double2* sig = static_cast<double2*>(scratch_address(h->device));
  if (!sig) return fail(h, SLRF_E_HIP, "sweep scratch array not resolved on this device");
  hipStream_t s = h->stream;
  // Fill the pole table (padding systems get sigma = 0, as in slrf_shifted_spmm)
  // through a fixed host staging array: each chunk's copy is ordered on the
  // stream after earlier work that may still read the table, and completes
  // before the array is refilled.
  constexpr int kChunk = 1024;
  double2 stage[kChunk];
  for (int b = 0; b < C; b += kChunk) {
    const int cnt = std::min(kChunk, C - b);
    for (int i = 0; i < cnt; ++i)
      stage[i] = b + i < nsys ? h->poles[pole[b + i]] : make_double2(0.0, 0.0);
    HIPCHK(hipMemcpyAsync(sig + b, stage, sizeof(double2) * cnt, hipMemcpyHostToDevice, s));
    HIPCHK(hipStreamSynchronize(s));
  }
  const PanelGrid g = make_grid(h->P.n, C, C, 2);
  if (precision == SLRF_PREC_FP64)
    HIPCHK(launch_spmm_panel<double>(h->P, g, sig, Z, Q, s));
  else
    HIPCHK(launch_spmm_panel<float>(h->P, g, sig, Z, Q, s));
  HIPCHK(hipStreamSynchronize(s));
  return SLRF_OK;
}

// Host checks of slrf_eig_grad's element data (nullptr when valid).
static const char* grad_args_error(int32_t n, int32_t nelem, int32_t ndof_e,
                                   const int32_t* dofs, int32_t dA_stride, int64_t dA_len,
                                   bool has_dB, int32_t dB_stride, int64_t dB_len) {
  if (ndof_e != 4 && ndof_e != 8 && ndof_e != 24) return "ndof_e must be 4, 8 or 24";
  if (nelem < 0 || n < 1) return "bad element count or problem size";
  const int64_t mat = (int64_t)ndof_e * ndof_e;
  auto span_ok = [&](int32_t stride, int64_t len) {
    if (stride < 0 || (stride > 0 && stride < mat)) return false;
    const int64_t need = nelem == 0 ? 0 : (stride == 0 ? mat : (int64_t)(nelem - 1) * stride + mat);
    return len >= need;
  };
  if (!span_ok(dA_stride, dA_len))
    return "dA: stride must be 0 or >= ndof_e^2 and dA_len must cover every element matrix";
  if (has_dB && !span_ok(dB_stride, dB_len))
    return "dB: stride must be 0 or >= ndof_e^2 and dB_len must cover every element matrix";
  for (int64_t i = 0; i < (int64_t)nelem * ndof_e; ++i)
    if (dofs[i] < -1 || dofs[i] >= n) return "elem_dofs holds a dof outside [-1, n)";
  return nullptr;
}

int32_t slrf_host_check_grad_args(int32_t n, int32_t nelem, int32_t ndof_e,
                                  const int32_t* elem_dofs, int32_t dA_stride, int64_t dA_len,
                                  int32_t has_dB, int32_t dB_stride, int64_t dB_len) {
  if (nelem > 0 && !elem_dofs) return SLRF_E_ARG;
  return grad_args_error(n, nelem, ndof_e, elem_dofs, dA_stride, dA_len, has_dB != 0, dB_stride,
                         dB_len)
             ? SLRF_E_ARG
             : SLRF_OK;
}

slrf_status slrf_eig_grad(slrf_handle h, int32_t k, const double* X, const double* lam,
                          const double* glam, int32_t nelem, int32_t ndof_e,
                          const int32_t* elem_dofs, const double* dA, int32_t dA_stride,
                          int64_t dA_len, const double* dB, int32_t dB_stride, int64_t dB_len,
                          double* grad) {
  if (!h) return SLRF_E_ARG;
  if (k < 0 || nelem < 0 || (k > 0 && (!X || !lam || !glam)) ||
      (nelem > 0 && (!elem_dofs || !dA || !grad)))
    return fail(h, SLRF_E_ARG, "bad eig_grad arguments");
  if (nelem == 0) {
    if (ndof_e != 4 && ndof_e != 8 && ndof_e != 24)
      return fail(h, SLRF_E_ARG, "ndof_e must be 4, 8 or 24");
    return SLRF_OK;
  }
  {
    // every dof in [-1, n) (the kernel gathers X rows by these indices) and
    // every element matrix inside its array
    std::vector<int32_t> dofs((size_t)nelem * ndof_e);
    if (ndof_e == 4 || ndof_e == 8 || ndof_e == 24) {
      HIPCHK(hipMemcpyAsync(dofs.data(), elem_dofs, sizeof(int32_t) * dofs.size(),
                            hipMemcpyDeviceToHost, h->stream));
      HIPCHK(hipStreamSynchronize(h->stream));
    }
    const char* why = grad_args_error(h->P.n, nelem, ndof_e, dofs.data(), dA_stride, dA_len,
                                      dB != nullptr, dB_stride, dB_len);
    if (why) return fail(h, SLRF_E_ARG, why);
  }
  HIPCHK(launch_eig_grad(h->P.n, k, X, lam, glam, nelem, ndof_e, elem_dofs, dA, dA_stride, dB,
                         dB_stride, grad, h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  return SLRF_OK;
}

int32_t slrf_host_projected_eig(int32_t n, const double* Ah, const double* Bh, double* theta,
                                double* S) {
  if (n < 0 || (n > 0 && (!Ah || !Bh || !theta || !S))) return -1;
  int fb = 0;
  return sym_gen_eig(n, Ah, Bh, theta, S, &fb);
}

slrf_status slrf_filter_batch(int32_t nh, const slrf_handle* hs, const int32_t* ncols,
                              const double* const* X, const double* const* theta_warm,
                              double* const* U, slrf_filter_stats* stats, int32_t nthreads) {
  if (nh < 0) return SLRF_E_ARG;
  if (nh == 0) return SLRF_OK;
  if (!hs || !ncols || !X || !U || !distinct_handles(nh, hs)) return SLRF_E_ARG;
  std::vector<double> work(nh);
  for (int i = 0; i < nh; ++i) work[i] = (double)hs[i]->P.nnz * ncols[i] * hs[i]->N;
  return run_batch(nh, hs, work, nthreads, [&](int i) {
    return slrf_filter(hs[i], ncols[i], X[i], theta_warm ? theta_warm[i] : nullptr, U[i],
                       stats ? &stats[i] : nullptr);
  });
}

slrf_status slrf_solve_batch(int32_t nh, const slrf_handle* hs, const int32_t* nev,
                             const int32_t* L, const double* const* V1,
                             double* const* theta_out, double* const* X_out,
                             int32_t* nconv_out, slrf_solve_stats* stats, int32_t nthreads) {
  if (nh < 0) return SLRF_E_ARG;
  if (nh == 0) return SLRF_OK;
  if (!hs || !nev || !L || !V1 || !theta_out || !X_out || !distinct_handles(nh, hs))
    return SLRF_E_ARG;
  std::vector<double> work(nh);
  for (int i = 0; i < nh; ++i) work[i] = (double)hs[i]->P.nnz * L[i] * hs[i]->N;
  return run_batch(nh, hs, work, nthreads, [&](int i) {
    return slrf_solve(hs[i], nev[i], L[i], V1[i], theta_out[i], X_out[i],
                      nconv_out ? &nconv_out[i] : nullptr, stats ? &stats[i] : nullptr);
  });
}

}  // extern "C"
