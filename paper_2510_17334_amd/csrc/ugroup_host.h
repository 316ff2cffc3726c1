// Host construction of the row-group format of a CSR pencil for the
// wave-uniform shifted sweep: consecutive rows in groups of R, one list of the
// group's distinct columns per group (sorted), each list entry carrying the
// mask of the group rows that reference the column and R coefficient pairs
// (a, b) (zero where the row has no entry).
#pragma once

#include <cstdint>
#include <vector>

namespace slrf {

struct HostUGroup {
  int R = 0, U = 0;        // rows per group, entries per unrolled chunk
  int ngroups = 0;
  std::vector<int> gptr;   // [ngroups + 1] entry offsets (multiples of U)
  std::vector<int> ent;    // [nent] column | (mask << kUGroupMaskShift)
  std::vector<double> ab;  // [nent][R][2] (a, b) per entry and group row
};

constexpr int kUGroupMaskShift = 28;  // columns below 2^28, masks of up to 4 rows

// Groups rows r0 = g R ... g R + R - 1 (the last group may be short).  Each
// group's entry count is padded to a multiple of U with entries of mask 0
// (column of the group's first entry, coefficients 0).  Within a group the
// entries are sorted by column, so every row meets its own entries in CSR
// order.  2 U entries of mask 0 follow the last group (look-ahead padding:
// gptr[ngroups] is the end of the real entries).  Returns false when R is not
// in 1..4, n >= 2^28 or a row is empty.
bool build_ugroup(int n, const std::vector<int>& rp, const std::vector<int>& ci,
                  const std::vector<double>& a, const std::vector<double>& b, int R, int U,
                  HostUGroup& out);

}  // namespace slrf
