// Host setup of the shared-hierarchy smoothed-aggregation AMG preconditioner.
//
// The paper preconditions GCR with PETSc's GAMG and builds it once, reusing it
// for every pole (Section 3.2).  Here one real hierarchy is built from the
// stiffness matrix: P_l (smoothed aggregation), A_{l+1} = P_l^T A_l P_l and
// B_{l+1} = P_l^T B_l P_l on one shared pattern, so that for any pole
// P^T (A - sigma B) P = A_c - sigma B_c and the level operators of every pole
// come from the same arrays.  The coarsest level is inverted densely per pole.
#include "amg_host.h"

#include <algorithm>
#include <atomic>
#include <cmath>
#include <complex>
#include <numeric>
#include <random>
#include <thread>

namespace slrf {

std::vector<double> rho_start_vector(int n) {
  std::vector<double> x(n);
  std::mt19937_64 rng(12345);
  std::normal_distribution<double> nd(0.0, 1.0);
  for (auto& v : x) v = nd(rng);
  return x;
}

namespace {

// Gustavson product C = X * Y (pattern only + values for one or two value
// arrays of X sharing its pattern).  Rows of C are sorted.
struct SpRow {
  std::vector<int> marker, cols;
  std::vector<double> acc1, acc2;
  explicit SpRow(int ncols) : marker(ncols, -1), acc1(ncols, 0.0), acc2(ncols, 0.0) {}
};

// Y is given by (rp, ci, v).  X has two value arrays xa, xb (xb may be null).
void spgemm2(int nrows, int ncols, const std::vector<int>& xrp, const std::vector<int>& xci,
             const std::vector<double>& xa, const std::vector<double>* xb,
             const std::vector<int>& yrp, const std::vector<int>& yci,
             const std::vector<double>& yv, std::vector<int>& crp, std::vector<int>& cci,
             std::vector<double>& ca, std::vector<double>* cb) {
  SpRow w(ncols);
  crp.assign(nrows + 1, 0);
  cci.clear();
  ca.clear();
  if (cb) cb->clear();
  for (int i = 0; i < nrows; ++i) {
    w.cols.clear();
    for (int e = xrp[i]; e < xrp[i + 1]; ++e) {
      const int k = xci[e];
      const double va = xa[e], vb = xb ? (*xb)[e] : 0.0;
      for (int f = yrp[k]; f < yrp[k + 1]; ++f) {
        const int j = yci[f];
        if (w.marker[j] != i) {
          w.marker[j] = i;
          w.cols.push_back(j);
          w.acc1[j] = 0.0;
          w.acc2[j] = 0.0;
        }
        w.acc1[j] += va * yv[f];
        w.acc2[j] += vb * yv[f];
      }
    }
    std::sort(w.cols.begin(), w.cols.end());
    for (int j : w.cols) {
      cci.push_back(j);
      ca.push_back(w.acc1[j]);
      if (cb) cb->push_back(w.acc2[j]);
    }
    crp[i + 1] = (int)cci.size();
  }
}

void transpose(int nrows, int ncols, const std::vector<int>& rp, const std::vector<int>& ci,
               const std::vector<double>& v, std::vector<int>& trp, std::vector<int>& tci,
               std::vector<double>& tv) {
  trp.assign(ncols + 1, 0);
  for (int e = 0; e < rp[nrows]; ++e) trp[ci[e] + 1]++;
  for (int j = 0; j < ncols; ++j) trp[j + 1] += trp[j];
  tci.assign(rp[nrows], 0);
  tv.assign(rp[nrows], 0.0);
  std::vector<int> pos(trp.begin(), trp.end() - 1);
  for (int i = 0; i < nrows; ++i)
    for (int e = rp[i]; e < rp[i + 1]; ++e) {
      const int p = pos[ci[e]]++;
      tci[p] = i;
      tv[p] = v[e];
    }
}

// Greedy aggregation on the strength graph (three passes: seed aggregates of
// fully unaggregated neighbourhoods, attach leftovers to a neighbouring
// aggregate, group what remains).
int aggregate(const HostLevel& L, double theta, std::vector<int>& agg) {
  const int n = L.n;
  std::vector<double> d(n, 0.0);
  for (int i = 0; i < n; ++i)
    for (int e = L.rp[i]; e < L.rp[i + 1]; ++e)
      if (L.ci[e] == i) d[i] = L.a[e];
  auto strong = [&](int i, int e) {
    const int j = L.ci[e];
    if (j == i) return false;
    const double v = std::fabs(L.a[e]);
    return v > theta * std::sqrt(std::fabs(d[i] * d[j])) && v > 1e-14 * std::fabs(d[i]);
  };
  agg.assign(n, -1);
  int na = 0;
  for (int i = 0; i < n; ++i) {
    if (agg[i] >= 0) continue;
    bool free = true;
    for (int e = L.rp[i]; e < L.rp[i + 1] && free; ++e)
      if (strong(i, e) && agg[L.ci[e]] >= 0) free = false;
    if (!free) continue;
    agg[i] = na;
    for (int e = L.rp[i]; e < L.rp[i + 1]; ++e)
      if (strong(i, e)) agg[L.ci[e]] = na;
    ++na;
  }
  std::vector<int> pass2(n, -1);
  for (int i = 0; i < n; ++i) {
    if (agg[i] >= 0) continue;
    for (int e = L.rp[i]; e < L.rp[i + 1]; ++e)
      if (strong(i, e) && agg[L.ci[e]] >= 0) {
        pass2[i] = agg[L.ci[e]];
        break;
      }
  }
  for (int i = 0; i < n; ++i)
    if (agg[i] < 0 && pass2[i] >= 0) agg[i] = pass2[i];
  for (int i = 0; i < n; ++i) {
    if (agg[i] >= 0) continue;
    agg[i] = na;
    for (int e = L.rp[i]; e < L.rp[i + 1]; ++e)
      if (strong(i, e) && agg[L.ci[e]] < 0) agg[L.ci[e]] = na;
    ++na;
  }
  return na;
}

// spectral radius of D^{-1} A by power iteration
double rho_dinv_a(const HostLevel& L) {
  const int n = L.n;
  std::vector<double> d(n, 1.0), x(n), y(n);
  for (int i = 0; i < n; ++i)
    for (int e = L.rp[i]; e < L.rp[i + 1]; ++e)
      if (L.ci[e] == i) d[i] = L.a[e];
  x = rho_start_vector(n);
  double rho = 1.0;
  for (int it = 0; it < 20; ++it) {
    double nrm = 0.0;
    for (int i = 0; i < n; ++i) {
      double s = 0.0;
      for (int e = L.rp[i]; e < L.rp[i + 1]; ++e) s += L.a[e] * x[L.ci[e]];
      y[i] = s / d[i];
      nrm += y[i] * y[i];
    }
    rho = std::sqrt(nrm);
    if (!(rho > 0.0)) return 1.0;
    for (int i = 0; i < n; ++i) x[i] = y[i] / rho;
  }
  return rho;
}

// Dense inverse of a complex matrix by Gauss-Jordan with partial pivoting.
// In-place Gauss-Jordan inversion with partial pivoting (row exchanges
// recorded, undone on the columns at the end): n^3 complex multiply-adds, the
// real and imaginary parts kept apart so the row updates vectorise.
bool invert_dense(int n, std::vector<std::complex<double>>& M) {
  std::vector<double> re((size_t)n * n), im((size_t)n * n);
  for (size_t i = 0; i < re.size(); ++i) {
    re[i] = M[i].real();
    im[i] = M[i].imag();
  }
  std::vector<int> perm(n);
  for (int c = 0; c < n; ++c) {
    int piv = c;
    double best = std::hypot(re[(size_t)c * n + c], im[(size_t)c * n + c]);
    for (int r = c + 1; r < n; ++r) {
      const double v = std::hypot(re[(size_t)r * n + c], im[(size_t)r * n + c]);
      if (v > best) {
        best = v;
        piv = r;
      }
    }
    if (!(best > 0.0)) return false;
    perm[c] = piv;
    if (piv != c) {
      std::swap_ranges(re.begin() + (size_t)c * n, re.begin() + (size_t)(c + 1) * n,
                       re.begin() + (size_t)piv * n);
      std::swap_ranges(im.begin() + (size_t)c * n, im.begin() + (size_t)(c + 1) * n,
                       im.begin() + (size_t)piv * n);
    }
    double* cr = re.data() + (size_t)c * n;
    double* ci = im.data() + (size_t)c * n;
    // 1 / pivot
    const double d = cr[c] * cr[c] + ci[c] * ci[c];
    const double pr = cr[c] / d, pi = -ci[c] / d;
    cr[c] = 1.0;
    ci[c] = 0.0;
    for (int k = 0; k < n; ++k) {
      const double xr = cr[k], xi = ci[k];
      cr[k] = xr * pr - xi * pi;
      ci[k] = xr * pi + xi * pr;
    }
    for (int r = 0; r < n; ++r) {
      if (r == c) continue;
      double* rr = re.data() + (size_t)r * n;
      double* ri = im.data() + (size_t)r * n;
      const double fr = rr[c], fi = ri[c];
      if (fr == 0.0 && fi == 0.0) continue;
      rr[c] = 0.0;
      ri[c] = 0.0;
      for (int k = 0; k < n; ++k) {
        rr[k] -= fr * cr[k] - fi * ci[k];
        ri[k] -= fr * ci[k] + fi * cr[k];
      }
    }
  }
  // the row exchanges of A become column exchanges of A^-1, in reverse order
  for (int c = n - 1; c >= 0; --c) {
    const int q = perm[c];
    if (q == c) continue;
    for (int r = 0; r < n; ++r) {
      std::swap(re[(size_t)r * n + c], re[(size_t)r * n + q]);
      std::swap(im[(size_t)r * n + c], im[(size_t)r * n + q]);
    }
  }
  for (size_t i = 0; i < re.size(); ++i) M[i] = std::complex<double>(re[i], im[i]);
  return true;
}

// Node graph of a node-major pencil with `bs` dofs per node: entry (I, J) holds
// the Frobenius norm of the bs x bs block of A (rows of a node share one
// column list made of whole blocks).
HostLevel node_graph(const HostLevel& L, int bs) {
  HostLevel G;
  const int nn = L.n / bs;
  G.n = nn;
  G.rp.assign(nn + 1, 0);
  for (int I = 0; I < nn; ++I) {
    const int len = L.rp[bs * I + 1] - L.rp[bs * I];
    for (int k = 0; k < len; k += bs) {
      double f = 0.0;
      for (int r = 0; r < bs; ++r) {
        const int e0 = L.rp[bs * I + r] + k;
        for (int c = 0; c < bs; ++c) f += L.a[e0 + c] * L.a[e0 + c];
      }
      G.ci.push_back(L.ci[L.rp[bs * I] + k] / bs);
      G.a.push_back(std::sqrt(f));
    }
    G.rp[I + 1] = (int)G.ci.size();
  }
  return G;
}

}  // namespace

int detect_block(const HostLevel& L) {
  for (int bs : {3, 2}) {
    if (L.n % bs != 0) continue;
    bool ok = true;
    for (int I = 0; I < L.n / bs && ok; ++I) {
      const int r0 = bs * I;
      const int len = L.rp[r0 + 1] - L.rp[r0];
      if (len % bs != 0) ok = false;
      for (int r = 1; r < bs && ok; ++r) {
        if (L.rp[r0 + r + 1] - L.rp[r0 + r] != len) {
          ok = false;
          break;
        }
        for (int k = 0; k < len; ++k)
          if (L.ci[L.rp[r0 + r] + k] != L.ci[L.rp[r0] + k]) {
            ok = false;
            break;
          }
      }
      for (int k = 0; k < len && ok; k += bs)
        for (int c = 0; c < bs; ++c) {
          const int j = L.ci[L.rp[r0] + k + c];
          if (j % bs != c || j / bs != L.ci[L.rp[r0] + k] / bs) {
            ok = false;
            break;
          }
        }
    }
    if (ok) return bs;
  }
  return 1;
}

void locality_order(const HostLevel& fine, std::vector<int>& order, int block) {
  if (block > 1) {
    std::vector<int> norder;
    locality_order(node_graph(fine, block), norder, 1);
    order.resize(fine.n);
    for (size_t k = 0; k < norder.size(); ++k)
      for (int c = 0; c < block; ++c) order[block * k + c] = block * norder[k] + c;
    return;
  }
  // Nested aggregation of the matrix graph: rows are sorted by their
  // ancestor at every aggregation level (coarsest first), so rows of one
  // aggregate are contiguous and aggregates of one parent are contiguous.
  const int n = fine.n;
  std::vector<std::vector<int>> anc;  // anc[l][i]: level-(l+1) ancestor of fine row i
  HostLevel cur;
  cur.n = n;
  cur.rp = fine.rp;
  cur.ci = fine.ci;
  cur.a = fine.a;
  std::vector<int> up(n);
  for (int i = 0; i < n; ++i) up[i] = i;
  while (cur.n > 64 && anc.size() < 12) {
    std::vector<int> agg;
    const int na = aggregate(cur, 0.0, agg);
    if (na >= cur.n || na == 0) break;
    for (int i = 0; i < n; ++i) up[i] = agg[up[i]];
    anc.push_back(up);
    // graph of the aggregates (values: magnitudes summed, diagonal kept)
    std::vector<std::vector<std::pair<int, double>>> rows(na);
    for (int i = 0; i < cur.n; ++i)
      for (int e = cur.rp[i]; e < cur.rp[i + 1]; ++e)
        rows[agg[i]].push_back({agg[cur.ci[e]], std::fabs(cur.a[e])});
    HostLevel nxt;
    nxt.n = na;
    nxt.rp.assign(na + 1, 0);
    for (int c = 0; c < na; ++c) {
      auto& r = rows[c];
      std::sort(r.begin(), r.end());
      int last = -1;
      for (auto& pr : r) {
        if (pr.first == last) {
          nxt.a.back() += pr.second;
        } else {
          nxt.ci.push_back(pr.first);
          nxt.a.push_back(pr.second);
          last = pr.first;
        }
      }
      nxt.rp[c + 1] = (int)nxt.ci.size();
    }
    cur = std::move(nxt);
  }
  order.resize(n);
  for (int i = 0; i < n; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
    for (int l = (int)anc.size() - 1; l >= 0; --l)
      if (anc[l][x] != anc[l][y]) return anc[l][x] < anc[l][y];
    return x < y;
  });
}

// One level's products on the host: rho(D^-1 A) by power iteration,
// A T, P = T - (omega_p / rho) D^-1 A T (T's entries added where A T has the
// column), R = P^T, A P and B P on one pattern, and C = R (A P), R (B P)
// (Gustavson order throughout, C not yet symmetrised).
bool host_level_products(const HostLevel& L, int nc, const std::vector<int>& trp,
                         const std::vector<int>& tci, const std::vector<double>& tv,
                         double omega_p, double& rho, HostCsrP& P, HostCsrP& R,
                         HostLevel& APBP, HostLevel& C) {
  const int n = L.n;
  rho = rho_dinv_a(L);
  std::vector<int> arp, aci;
  std::vector<double> at;
  spgemm2(n, nc, L.rp, L.ci, L.a, nullptr, trp, tci, tv, arp, aci, at, nullptr);
  std::vector<double> d(n, 1.0);
  for (int i = 0; i < n; ++i)
    for (int e = L.rp[i]; e < L.rp[i + 1]; ++e)
      if (L.ci[e] == i) d[i] = L.a[e];
  P = HostCsrP();
  P.n = n;
  P.m = nc;
  P.rp = arp;
  P.ci = aci;
  P.v.resize(at.size());
  const double w = omega_p / rho;
  for (int i = 0; i < n; ++i) {
    // (A T has every column of T's row i: A holds the diagonal)
    int f = trp[i];
    for (int e = arp[i]; e < arp[i + 1]; ++e) {
      double v = -w * at[e] / d[i];
      while (f < trp[i + 1] && tci[f] < aci[e]) ++f;
      if (f < trp[i + 1] && tci[f] == aci[e]) v += tv[f];
      P.v[e] = v;
    }
  }
  R = HostCsrP();
  R.n = nc;
  R.m = n;
  transpose(n, nc, P.rp, P.ci, P.v, R.rp, R.ci, R.v);
  // Galerkin: AP, BP (shared pattern), then R (AP), R (BP)
  std::vector<int> aprp, apci;
  std::vector<double> apa, apb;
  spgemm2(n, nc, L.rp, L.ci, L.a, &L.b, P.rp, P.ci, P.v, aprp, apci, apa, &apb);
  C = HostLevel();
  C.n = nc;
  // R * (AP) and R * (BP) on one pattern: multiply R (single value array)
  // into the two value arrays of AP/BP by swapping roles: C = R * AP and
  // C' = R * BP share the pattern because AP and BP do.
  {
    SpRow wr(nc);
    C.rp.assign(nc + 1, 0);
    for (int i = 0; i < nc; ++i) {
      wr.cols.clear();
      for (int e = R.rp[i]; e < R.rp[i + 1]; ++e) {
        const int k = R.ci[e];
        const double rv = R.v[e];
        for (int f = aprp[k]; f < aprp[k + 1]; ++f) {
          const int j = apci[f];
          if (wr.marker[j] != i) {
            wr.marker[j] = i;
            wr.cols.push_back(j);
            wr.acc1[j] = 0.0;
            wr.acc2[j] = 0.0;
          }
          wr.acc1[j] += rv * apa[f];
          wr.acc2[j] += rv * apb[f];
        }
      }
      std::sort(wr.cols.begin(), wr.cols.end());
      for (int j : wr.cols) {
        C.ci.push_back(j);
        // symmetrise the tiny rounding asymmetry later by averaging with the transpose
        C.a.push_back(wr.acc1[j]);
        C.b.push_back(wr.acc2[j]);
      }
      C.rp[i + 1] = (int)C.ci.size();
    }
  }
  APBP = HostLevel();
  APBP.n = n;
  APBP.rp = std::move(aprp);
  APBP.ci = std::move(apci);
  APBP.a = std::move(apa);
  APBP.b = std::move(apb);
  return true;
}

bool amg_build(const HostLevel& fine, const std::vector<std::complex<double>>& poles,
               const AmgParams& prm, AmgHierarchy& H, std::string& err, AmgNumeric* num) {
  H.levels.clear();
  H.P.clear();
  H.R.clear();
  H.rho.clear();
  H.img.clear();
  H.levels.push_back(fine);
  // near-nullspace candidates of the current level (n x kns, row-major): the
  // constant (scalar), one translation per component, or the rigid-body modes
  int lev_block = prm.block;
  int kns = 1;
  std::vector<double> ns;
  {
    const int n0 = fine.n;
    const int bs0 = prm.block > 1 && n0 % prm.block == 0 ? prm.block : 1;
    const bool rigid = prm.xyz != nullptr && (bs0 == 2 || bs0 == 3) &&
                       prm.xyz->size() == (size_t)n0;
    if (rigid) {
      kns = bs0 == 3 ? 6 : 3;
      ns.assign((size_t)n0 * kns, 0.0);
      for (int node = 0; node < n0 / bs0; ++node) {
        const double* x = prm.xyz->data() + (size_t)node * bs0;
        for (int c = 0; c < bs0; ++c) ns[((size_t)node * bs0 + c) * kns + c] = 1.0;
        if (bs0 == 3) {
          // rotations about x, y, z: (0, -z, y), (z, 0, -x), (-y, x, 0)
          double* r0 = &ns[((size_t)node * 3) * kns];
          double* r1 = &ns[((size_t)node * 3 + 1) * kns];
          double* r2 = &ns[((size_t)node * 3 + 2) * kns];
          r1[3] = -x[2];
          r2[3] = x[1];
          r0[4] = x[2];
          r2[4] = -x[0];
          r0[5] = -x[1];
          r1[5] = x[0];
        } else {
          ns[((size_t)node * 2) * kns + 2] = -x[1];
          ns[((size_t)node * 2 + 1) * kns + 2] = x[0];
        }
      }
    } else {
      kns = bs0;
      ns.assign((size_t)n0 * kns, 0.0);
      for (int i = 0; i < n0; ++i) ns[(size_t)i * kns + i % bs0] = 1.0;
    }
    lev_block = bs0;
  }
  const bool rigid_modes = kns > lev_block;
  while (H.levels.back().n > prm.coarse_max && (int)H.levels.size() < prm.max_levels) {
    const HostLevel& L = H.levels.back();
    const int n = L.n;
    const int bs = lev_block > 1 && n % lev_block == 0 ? lev_block : 1;
    // aggregates of dofs (whole nodes when bs > 1)
    std::vector<int> dagg(n);
    auto aggregate_at = [&](double theta, std::vector<int>& out) {
      if (bs > 1) {
        std::vector<int> nagg;
        const int k = aggregate(node_graph(L, bs), theta, nagg);
        for (int i = 0; i < n; ++i) out[i] = nagg[i / bs];
        return k;
      }
      return aggregate(L, theta, out);
    };
    // coarse dofs: kns columns per aggregate (fewer where dependent ones drop)
    const int ncols = rigid_modes ? kns : bs;
    int na = aggregate_at(prm.theta, dagg);
    if (prm.coarse_min > 0 && (long)na * ncols < prm.coarse_min) {
      // too small a coarse space: smaller aggregates (a higher strength
      // threshold) whose coarse dofs still at most halve the level; failing
      // that, this level is the coarsest if the dense solve takes it
      bool found = false;
      int best = na;
      std::vector<int> trial(n), best_agg;
      for (double th = 0.01; th <= 0.64 && !found; th *= 2.0) {
        if (th <= prm.theta) continue;
        const int k = aggregate_at(th, trial);
        if (2L * k * ncols > n) continue;
        if ((long)k * ncols >= prm.coarse_min) {
          na = k;
          dagg.swap(trial);
          found = true;
        } else if (k > best) {
          best = k;
          best_agg = trial;
        }
      }
      if (!found) {
        if (n <= prm.dense_max) break;
        // too large for the dense solve: the largest coarse space that halves
        if (best > na) {
          na = best;
          dagg.swap(best_agg);
        }
      }
    }
    if (na == 0) break;
    // tentative prolongator T: per aggregate, an orthonormal basis of the
    // near-nullspace rows restricted to it (modified Gram-Schmidt, twice, with
    // dependent columns dropped), the R factor becoming the next level's rows
    std::vector<std::vector<int>> rows(na);
    for (int i = 0; i < n; ++i) rows[dagg[i]].push_back(i);
    std::vector<int> cbase(na + 1, 0);
    std::vector<std::vector<double>> Qa(na), Ra(na);
    std::vector<int> ka(na, 0);
    for (int a = 0; a < na; ++a) {
      const auto& r = rows[a];
      const int nr = (int)r.size();
      std::vector<double>& Q = Qa[a];  // nr x k (column j at j * nr)
      std::vector<double> R;           // k x kns
      for (int j = 0; j < kns; ++j) {
        std::vector<double> v(nr);
        double n0 = 0.0;
        for (int t = 0; t < nr; ++t) {
          v[t] = ns[(size_t)r[t] * kns + j];
          n0 += v[t] * v[t];
        }
        n0 = std::sqrt(n0);
        std::vector<double> coef(ka[a], 0.0);
        for (int pass = 0; pass < 2; ++pass)
          for (int i = 0; i < ka[a]; ++i) {
            double d = 0.0;
            for (int t = 0; t < nr; ++t) d += Q[(size_t)i * nr + t] * v[t];
            coef[i] += d;
            for (int t = 0; t < nr; ++t) v[t] -= d * Q[(size_t)i * nr + t];
          }
        double nv = 0.0;
        for (double x : v) nv += x * x;
        nv = std::sqrt(nv);
        const bool keep = n0 > 0.0 && nv > 1e-10 * n0;
        // R columns: coefficients of column j on the kept q_i (and on q_j)
        R.resize((size_t)(ka[a] + (keep ? 1 : 0)) * kns, 0.0);
        if (keep) {
          // (row ka[a] of R is new: shift nothing, rows are appended)
          for (int t = 0; t < nr; ++t) Q.push_back(v[t] / nv);
          for (int i = 0; i < ka[a]; ++i) R[(size_t)i * kns + j] = coef[i];
          R[(size_t)ka[a] * kns + j] = nv;
          ++ka[a];
        } else {
          for (int i = 0; i < ka[a]; ++i) R[(size_t)i * kns + j] = coef[i];
        }
      }
      Ra[a] = R;
      cbase[a + 1] = cbase[a] + ka[a];
    }
    const int nc = cbase[na];
    if (nc >= n || nc == 0) break;  // no coarsening possible
    std::vector<int> trp(n + 1, 0), tci;
    std::vector<double> tv;
    {
      std::vector<int> pos(n, -1);  // position of dof i in its aggregate's row list
      for (int a = 0; a < na; ++a)
        for (size_t t = 0; t < rows[a].size(); ++t) pos[rows[a][t]] = (int)t;
      for (int i = 0; i < n; ++i) {
        const int a = dagg[i], nr = (int)rows[a].size();
        for (int j = 0; j < ka[a]; ++j) {
          const double q = Qa[a][(size_t)j * nr + pos[i]];
          if (q == 0.0) continue;
          tci.push_back(cbase[a] + j);
          tv.push_back(q);
        }
        trp[i + 1] = (int)tci.size();
      }
    }
    // (a row of T holds at most one entry per column: the diagonal-block
    // term of P adds T's value in that column)
    std::vector<double> ns_next((size_t)nc * kns, 0.0);
    for (int a = 0; a < na; ++a)
      for (int j = 0; j < ka[a]; ++j)
        for (int c = 0; c < kns; ++c)
          ns_next[(size_t)(cbase[a] + j) * kns + c] = Ra[a][(size_t)j * kns + c];
    // P = T - (omega / rho) D^{-1} A T, R = P^T, A P and B P, C = R (A P), R (B P)
    double rho = 1.0;
    HostCsrP P, R;
    HostLevel APBP, C;
    {
      std::string nerr;
      const bool ok = num ? num->level(L, nc, trp, tci, tv, prm.omega_p, rho, P, R, APBP, C, nerr)
                          : host_level_products(L, nc, trp, tci, tv, prm.omega_p, rho, P, R, APBP, C);
      if (!ok) {
        err = "AMG products: " + nerr;
        return false;
      }
    }
    H.rho.push_back(rho);
    // enforce exact symmetry of the coarse operators: (C + C^T)/2 on the shared pattern
    {
      std::vector<int> trp2, tci2;
      std::vector<double> ta, tb;
      transpose(nc, nc, C.rp, C.ci, C.a, trp2, tci2, ta);
      transpose(nc, nc, C.rp, C.ci, C.b, trp2, tci2, tb);
      if (trp2 == C.rp && tci2 == C.ci) {
        for (size_t e = 0; e < C.a.size(); ++e) {
          C.a[e] = 0.5 * (C.a[e] + ta[e]);
          C.b[e] = 0.5 * (C.b[e] + tb[e]);
        }
      }
    }
    H.img.push_back(std::move(APBP));
    H.P.push_back(std::move(P));
    H.R.push_back(std::move(R));
    H.levels.push_back(std::move(C));
    ns.swap(ns_next);
    // translations alone keep whole nodes of bs dofs; with rigid-body modes
    // the aggregates' dof counts vary and coarser levels aggregate scalar dofs
    if (rigid_modes) lev_block = 1;
  }
  const int nc = H.levels.back().n;
  if (nc > prm.dense_max) {
    err = "AMG coarsest level too large for a dense solve (" + std::to_string(nc) + ")";
    return false;
  }
  H.nc = nc;
  return amg_coarse_inverses(H, poles, err);
}

bool amg_coarse_inverses(AmgHierarchy& H, const std::vector<std::complex<double>>& poles,
                         std::string& err) {
  // dense per-pole inverses of the coarsest operator
  const HostLevel& Lc = H.levels.back();
  const int nc = Lc.n;
  H.nc = nc;
  H.coarse_inv.assign(poles.size() * (size_t)nc * nc, 0.0);
  // one host thread per pole (each inversion is independent and n^3)
  const int np = (int)poles.size();
  std::vector<char> ok(np, 1);
  auto one = [&](int j) {
    std::vector<std::complex<double>> M((size_t)nc * nc, 0.0);
    for (int i = 0; i < nc; ++i)
      for (int e = Lc.rp[i]; e < Lc.rp[i + 1]; ++e)
        M[(size_t)i * nc + Lc.ci[e]] = Lc.a[e] - poles[j] * Lc.b[e];
    ok[j] = invert_dense(nc, M) ? 1 : 0;
    if (ok[j]) std::copy(M.begin(), M.end(), H.coarse_inv.begin() + j * (size_t)nc * nc);
  };
  const int nt = std::max(1, std::min(np, (int)std::thread::hardware_concurrency()));
  if (nt <= 1 || (double)nc * nc * nc < 1e7) {
    for (int j = 0; j < np; ++j) one(j);
  } else {
    // (a thread that cannot be started leaves its share to the others, and
    // to this thread when none started)
    std::atomic<int> next(0);
    std::vector<std::thread> pool;
    auto work = [&] {
      for (int j = next++; j < np; j = next++) one(j);
    };
    for (int t = 0; t < nt; ++t) {
      try {
        pool.emplace_back(work);
      } catch (...) {
        break;
      }
    }
    for (auto& t : pool) t.join();
    work();
  }
  for (int j = 0; j < np; ++j)
    if (!ok[j]) {
      err = "singular coarsest AMG operator";
      return false;
    }
  return true;
}

namespace {
bool p_on_pattern(int n, const std::vector<int>& rp, const std::vector<int>& ci, const HostCsrP& P,
                  std::vector<double>& pv) {
  pv.assign(ci.size(), 0.0);
  std::vector<int> at(P.m, -1);  // entry of column c in the current row
  for (int i = 0; i < n; ++i) {
    for (int e = rp[i]; e < rp[i + 1]; ++e) at[ci[e]] = e;
    for (int f = P.rp[i]; f < P.rp[i + 1]; ++f) {
      const int e = at[P.ci[f]];
      if (e < rp[i] || e >= rp[i + 1]) return false;
      pv[e] += P.v[f];
    }
    for (int e = rp[i]; e < rp[i + 1]; ++e) at[ci[e]] = -1;
  }
  return true;
}
}  // namespace

bool fine_image(const HostLevel& L, const HostCsrP& P, std::vector<int>& rp,
                std::vector<int>& ci, std::vector<double>& ap, std::vector<double>& bp,
                std::vector<double>& pv) {
  spgemm2(L.n, P.m, L.rp, L.ci, L.a, &L.b, P.rp, P.ci, P.v, rp, ci, ap, &bp);
  return p_on_pattern(L.n, rp, ci, P, pv);
}

bool image_p_values(const HostLevel& APBP, const HostCsrP& P, std::vector<double>& pv) {
  return p_on_pattern(APBP.n, APBP.rp, APBP.ci, P, pv);
}

}  // namespace slrf
