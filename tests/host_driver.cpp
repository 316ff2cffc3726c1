// Test driver for the library's host-side setup code (no GPU): reads a CSR
// pencil, runs one routine and writes its result as raw arrays for the Python
// checks in test_host_cpp.py.
//   host_driver <pencil.bin> <out.bin> order <block>
//   host_driver <pencil.bin> <out.bin> block
//   host_driver <pencil.bin> <out.bin> halo <hmax> <rows_cap>
//   host_driver <pencil.bin> <out.bin> amg <block> <sigma_re> <sigma_im> [<xyz.bin>]
//   host_driver <pencil.bin> <out.bin> ugroup <R> <U>
// pencil.bin: int32 n, int32 nnz, int32 rp[n+1], int32 ci[nnz], f64 a[nnz], f64 b[nnz]
#include <complex>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "amg_host.h"
#include "halo_host.h"
#include "ugroup_host.h"

using namespace slrf;

static FILE* g_out = nullptr;
template <typename V>
static void put(const std::vector<V>& v) {
  const int64_t k = (int64_t)v.size();
  std::fwrite(&k, sizeof(k), 1, g_out);
  if (k) std::fwrite(v.data(), sizeof(V), v.size(), g_out);
}
static void put_i(int64_t x) { std::fwrite(&x, sizeof(x), 1, g_out); }

int main(int argc, char** argv) {
  if (argc < 4) return 2;
  FILE* f = std::fopen(argv[1], "rb");
  if (!f) return 3;
  int n = 0, nnz = 0;
  if (std::fread(&n, 4, 1, f) != 1 || std::fread(&nnz, 4, 1, f) != 1) return 3;
  HostLevel L;
  L.n = n;
  L.rp.resize(n + 1);
  L.ci.resize(nnz);
  L.a.resize(nnz);
  L.b.resize(nnz);
  if (std::fread(L.rp.data(), 4, n + 1, f) != (size_t)n + 1 ||
      std::fread(L.ci.data(), 4, nnz, f) != (size_t)nnz ||
      std::fread(L.a.data(), 8, nnz, f) != (size_t)nnz ||
      std::fread(L.b.data(), 8, nnz, f) != (size_t)nnz)
    return 3;
  std::fclose(f);
  g_out = std::fopen(argv[2], "wb");
  if (!g_out) return 4;
  const std::string mode = argv[3];
  if (mode == "order") {
    std::vector<int> order;
    locality_order(L, order, std::atoi(argv[4]));
    put(order);
  } else if (mode == "block") {
    put_i(detect_block(L));
  } else if (mode == "halo") {
    HostHalo H;
    const bool ok = build_halo(n, L.rp, L.ci, L.a, L.b, std::atoi(argv[4]), std::atoi(argv[5]), H);
    put_i(ok ? 1 : 0);
    put_i(H.hmax);
    put_i(H.emax);
    put(H.trow);
    put(H.hptr);
    put(H.halo);
    put(H.sptr);
    put(H.slen);
    put(H.lcol);
    put(H.ab);
  } else if (mode == "amg") {
    AmgParams prm;
    prm.block = std::atoi(argv[4]);
    std::vector<double> xyz;
    // optional trailing argument cmin=<k>: AmgParams::coarse_min
    if (argc > 7 && std::strncmp(argv[argc - 1], "cmin=", 5) == 0) {
      prm.coarse_min = std::atoi(argv[argc - 1] + 5);
      --argc;
    }
    if (argc > 7) {  // node coordinates: float64 [n] (nodes x block)
      FILE* fx = std::fopen(argv[7], "rb");
      if (!fx) return 3;
      xyz.resize(n);
      if (std::fread(xyz.data(), 8, n, fx) != (size_t)n) return 3;
      std::fclose(fx);
      prm.xyz = &xyz;
    }
    AmgHierarchy H;
    std::string err;
    std::vector<std::complex<double>> poles{{std::atof(argv[5]), std::atof(argv[6])}};
    const bool ok = amg_build(L, poles, prm, H, err);
    put_i(ok ? 1 : 0);
    put_i((int64_t)H.levels.size());
    for (size_t l = 0; l < H.levels.size(); ++l) {
      put_i(H.levels[l].n);
      put(H.levels[l].rp);
      put(H.levels[l].ci);
      put(H.levels[l].a);
      put(H.levels[l].b);
    }
    for (size_t l = 0; l < H.P.size(); ++l) {
      put_i(H.P[l].n);
      put_i(H.P[l].m);
      put(H.P[l].rp);
      put(H.P[l].ci);
      put(H.P[l].v);
      put_i(H.R[l].n);
      put(H.R[l].rp);
      put(H.R[l].ci);
      put(H.R[l].v);
    }
    put(H.rho);
    put_i(H.nc);
    put(H.coarse_inv);
  } else if (mode == "image") {
    // fine image of P_0 and its halo-tile layout with P's values as the third array
    AmgParams prm;
    prm.block = std::atoi(argv[4]);
    AmgHierarchy H;
    std::string err;
    std::vector<std::complex<double>> poles{{1.0, 1.0}};
    bool ok = amg_build(L, poles, prm, H, err) && H.P.size() >= 1;
    std::vector<int> rp, ci;
    std::vector<double> ap, bp, pv;
    ok = ok && fine_image(L, H.P[0], rp, ci, ap, bp, pv);
    HostHalo X;
    const bool hok = ok && build_halo(n, rp, ci, ap, bp, std::atoi(argv[5]), std::atoi(argv[6]), X, &pv);
    put_i(ok ? 1 : 0);
    put_i(hok ? 1 : 0);
    put_i(ok ? H.P[0].m : 0);
    put(H.P.empty() ? std::vector<int>() : H.P[0].rp);
    put(H.P.empty() ? std::vector<int>() : H.P[0].ci);
    put(H.P.empty() ? std::vector<double>() : H.P[0].v);
    put(rp);
    put(ci);
    put(ap);
    put(bp);
    put(pv);
    put_i(X.hmax);
    put(X.trow);
    put(X.hptr);
    put(X.halo);
    put(X.sptr);
    put(X.slen);
    put(X.lcol);
    put(X.ab);
    put(X.c);
    HostHaloSub S;
    if (hok) build_halo_sub(n, X, S);
    put_i(S.emax);
    put(S.sptr);
    put(S.lcol);
    put(S.v);
  } else if (mode == "ugroup") {
    HostUGroup G;
    const bool ok = build_ugroup(n, L.rp, L.ci, L.a, L.b, std::atoi(argv[4]), std::atoi(argv[5]), G);
    put_i(ok ? 1 : 0);
    put(G.gptr);
    put(G.ent);
    put(G.ab);
  } else {
    return 2;
  }
  std::fclose(g_out);
  return 0;
}
