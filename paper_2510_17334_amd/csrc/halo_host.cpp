#include "halo_host.h"

#include <algorithm>

namespace slrf {

bool build_halo(int n, const std::vector<int>& rp, const std::vector<int>& ci,
                const std::vector<double>& a, const std::vector<double>& b, int hmax,
                int rows_cap, HostHalo& out, const std::vector<double>* c) {
  out = HostHalo();
  if (n <= 0 || hmax < 1 || hmax > 65535) return false;
  const int S = kHaloSlice;
  const int nslice = (n + S - 1) / S;
  int ncol = n;
  for (int e = 0; e < rp[n]; ++e) ncol = std::max(ncol, ci[e] + 1);
  // ---- tiles: greedy growth by whole slices under the halo and row caps
  std::vector<int> stamp(ncol, -1);
  out.trow.push_back(0);
  out.hptr.push_back(0);
  int tile = 0, hcount = 0, trows = 0;
  std::vector<int> fresh;
  for (int s = 0; s < nslice; ++s) {
    const int r0 = s * S, r1 = std::min(r0 + S, n);
    fresh.clear();
    for (int e = rp[r0]; e < rp[r1]; ++e) {
      const int c = ci[e];
      if (stamp[c] != tile) {
        stamp[c] = tile;
        fresh.push_back(c);
      }
    }
    if (trows > 0 && (hcount + (int)fresh.size() > hmax || trows + (r1 - r0) > rows_cap)) {
      // close the current tile; this slice opens the next one
      for (int c : fresh) stamp[c] = -1;
      out.trow.push_back(r0);
      ++tile;
      hcount = 0;
      trows = 0;
      fresh.clear();
      for (int e = rp[r0]; e < rp[r1]; ++e) {
        const int c = ci[e];
        if (stamp[c] != tile) {
          stamp[c] = tile;
          fresh.push_back(c);
        }
      }
    }
    if ((int)fresh.size() > hmax) return false;
    hcount += (int)fresh.size();
    trows += r1 - r0;
  }
  out.trow.push_back(n);
  out.ntile = (int)out.trow.size() - 1;
  // ---- halos (sorted) and local indices
  std::vector<int> pos(ncol, -1);
  std::vector<int> h;
  out.sptr.assign(nslice + 1, 0);
  out.slen.assign((size_t)nslice * S, 0);
  for (int s = 0; s < nslice; ++s) {
    int wdt = 0;
    for (int t = 0; t < S; ++t) {
      const int r = s * S + t;
      if (r < n) {
        out.slen[(size_t)s * S + t] = rp[r + 1] - rp[r];
        wdt = std::max(wdt, rp[r + 1] - rp[r]);
      }
    }
    out.sptr[s + 1] = out.sptr[s] + (wdt + kHaloPad - 1) / kHaloPad * kHaloPad;
  }
  const size_t nent = (size_t)out.sptr[nslice] * S;
  out.lcol.assign(nent, 0);
  out.ab.assign(2 * nent, 0.0);
  if (c) out.c.assign(nent, 0.0);
  for (int t = 0; t < out.ntile; ++t) {
    const int r0 = out.trow[t], r1 = out.trow[t + 1];
    h.assign(ci.begin() + rp[r0], ci.begin() + rp[r1]);
    std::sort(h.begin(), h.end());
    h.erase(std::unique(h.begin(), h.end()), h.end());
    for (size_t i = 0; i < h.size(); ++i) pos[h[i]] = (int)i;
    out.hmax = std::max(out.hmax, (int)h.size());
    out.halo.insert(out.halo.end(), h.begin(), h.end());
    out.hptr.push_back((int)out.halo.size());
    for (int r = r0; r < r1; ++r) {
      const int s = r / S, ln = r % S;
      for (int e = rp[r]; e < rp[r + 1]; ++e) {
        const size_t k = halo_entry(out.sptr[s], e - rp[r], ln);
        out.lcol[k] = (uint16_t)pos[ci[e]];
        out.ab[2 * k] = a[e];
        out.ab[2 * k + 1] = b[e];
        if (c) out.c[k] = (*c)[e];
      }
    }
    for (int c : h) pos[c] = -1;
  }
  for (int t = 0; t < out.ntile; ++t) {
    const int s0 = out.trow[t] / S, s1 = (out.trow[t + 1] + S - 1) / S;
    for (int a = s0; a < s1; a += kHaloPassSlices) {
      const int b = std::min(a + kHaloPassSlices, s1);
      out.emax = std::max(out.emax, (out.sptr[b] - out.sptr[a]) * S);
    }
  }
  return out.hmax <= hmax;
}

void build_halo_sub(int n, const HostHalo& hx, HostHaloSub& out) {
  out = HostHaloSub();
  const int S = kHaloSlice;
  const int nslice = (n + S - 1) / S;
  out.sptr.assign(nslice + 1, 0);
  for (int s = 0; s < nslice; ++s) {
    int wdt = 0;
    for (int t = 0; t < S; ++t) {
      const int r = s * S + t;
      if (r >= n) break;
      int cnt = 0;
      for (int j = 0; j < hx.slen[r]; ++j) cnt += hx.c[halo_entry(hx.sptr[s], j, t)] != 0.0;
      wdt = std::max(wdt, cnt);
    }
    out.sptr[s + 1] = out.sptr[s] + (wdt + kHaloPad - 1) / kHaloPad * kHaloPad;
  }
  const size_t nent = (size_t)out.sptr[nslice] * S;
  out.lcol.assign(nent, 0);
  out.v.assign(nent, 0.0);
  for (int s = 0; s < nslice; ++s)
    for (int t = 0; t < S; ++t) {
      const int r = s * S + t;
      if (r >= n) break;
      int q = 0;
      for (int j = 0; j < hx.slen[r]; ++j) {
        const size_t k = halo_entry(hx.sptr[s], j, t);
        if (hx.c[k] == 0.0) continue;
        const size_t kk = halo_entry(out.sptr[s], q++, t);
        out.lcol[kk] = hx.lcol[k];
        out.v[kk] = hx.c[k];
      }
    }
  for (int t = 0; t < hx.ntile; ++t) {
    const int s0 = hx.trow[t] / S, s1 = (hx.trow[t + 1] + S - 1) / S;
    for (int a = s0; a < s1; a += kHaloPassSlices) {
      const int b = std::min(a + kHaloPassSlices, s1);
      out.emax = std::max(out.emax, (out.sptr[b] - out.sptr[a]) * S);
    }
  }
}

}  // namespace slrf
