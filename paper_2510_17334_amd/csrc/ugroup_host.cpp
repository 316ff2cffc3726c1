#include "ugroup_host.h"

#include <algorithm>
#include <tuple>

namespace slrf {

bool build_ugroup(int n, const std::vector<int>& rp, const std::vector<int>& ci,
                  const std::vector<double>& a, const std::vector<double>& b, int R, int U,
                  HostUGroup& out) {
  out = HostUGroup();
  if (n <= 0 || R < 1 || R > 4 || U < 1 || n >= (1 << kUGroupMaskShift)) return false;
  out.R = R;
  out.U = U;
  out.ngroups = (n + R - 1) / R;
  out.gptr.assign(out.ngroups + 1, 0);
  std::vector<std::tuple<int, int, int>> items;  // (column, group row, CSR entry)
  for (int g = 0; g < out.ngroups; ++g) {
    const int r0 = g * R, r1 = std::min(r0 + R, n);
    items.clear();
    for (int r = r0; r < r1; ++r) {
      if (rp[r + 1] <= rp[r]) return false;
      for (int e = rp[r]; e < rp[r + 1]; ++e) items.emplace_back(ci[e], r - r0, e);
    }
    std::sort(items.begin(), items.end());
    const size_t first = out.ent.size();
    for (size_t i = 0; i < items.size();) {
      const int c = std::get<0>(items[i]);
      int mask = 0;
      const size_t base = out.ab.size();
      out.ab.resize(base + 2 * (size_t)R, 0.0);
      for (; i < items.size() && std::get<0>(items[i]) == c; ++i) {
        const int r = std::get<1>(items[i]), e = std::get<2>(items[i]);
        mask |= 1 << r;
        out.ab[base + 2 * r] = a[e];
        out.ab[base + 2 * r + 1] = b[e];
      }
      out.ent.push_back(c | (mask << kUGroupMaskShift));
    }
    const int col0 = out.ent[first] & ((1 << kUGroupMaskShift) - 1);
    while ((out.ent.size() - first) % U != 0) {
      out.ent.push_back(col0);
      out.ab.resize(out.ab.size() + 2 * (size_t)R, 0.0);
    }
    out.gptr[g + 1] = (int)out.ent.size();
  }
  // two chunks of padding past the last group (look-ahead loads of the sweep)
  const int colz = out.ent.empty() ? 0 : (out.ent.back() & ((1 << kUGroupMaskShift) - 1));
  for (int k = 0; k < 2 * U; ++k) {
    out.ent.push_back(colz);
    out.ab.resize(out.ab.size() + 2 * (size_t)R, 0.0);
  }
  return true;
}

}  // namespace slrf
