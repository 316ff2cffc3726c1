// Host construction of the halo-tile format of a CSR pencil (shifted SpMM with
// the gathered operand staged in LDS).
#pragma once

#include <cstddef>
#include <cstdint>
#include <vector>

namespace slrf {

// Rows are cut into tiles made of whole slices of kHaloSlice consecutive rows.
// A tile's halo is the sorted set of columns its rows reference; a tile grows
// slice by slice while its halo stays within hmax entries and its rows within
// rows_cap.  Entries are stored slice-major in groups of kHaloPad per row:
// entry j of row r (slice s = r / 8, lane t = r % 8) sits at
// sptr[s] * 8 + (j / 4) * 32 + t * 4 + j % 4, so one row's four entries of a
// group are contiguous (one 8-byte read of their local columns, 16-byte reads
// of their coefficients) and the 8 rows' groups follow each other; the column
// is given as the position in the tile's halo; slen holds the row lengths (0
// past n), a slice is as wide as its longest row rounded up to a multiple of kHaloPad, and
// shorter rows are padded with entries of local column 0 and coefficients 0
// (they add 0 * z for a halo row of the same system: the kernels need no
// per-entry predicate).
struct HostHalo {
  int ntile = 0, hmax = 0;
  int emax = 0;            // most entries of a pass (4 consecutive slices of a tile)
  std::vector<int> trow;   // [ntile + 1] first row of each tile
  std::vector<int> hptr;   // [ntile + 1] offsets into halo
  std::vector<int> halo;   // halo rows of all tiles
  std::vector<int> sptr;   // [nslice + 1] slice offsets in steps of 8 entries
  std::vector<int> slen;   // [nslice * 8] row lengths
  std::vector<uint16_t> lcol;   // local column (halo position) per entry
  std::vector<double> ab;  // (a, b) per entry, interleaved
  std::vector<double> c;   // optional third value per entry (same layout as lcol)
};

constexpr int kHaloSlice = 8;
constexpr int kHaloPassSlices = 4;  // slices formed together by one workgroup pass
constexpr int kHaloPad = 4;         // slice widths are multiples of this (= the group size)

// Position of entry j of lane t in slice s (sptr_s = sptr[s]).
inline size_t halo_entry(int sptr_s, int j, int t) {
  return (size_t)sptr_s * kHaloSlice + (size_t)(j / kHaloPad) * (kHaloSlice * kHaloPad) +
         (size_t)t * kHaloPad + (size_t)(j % kHaloPad);
}

// The entries of a halo layout whose third value (c) is nonzero, on the same
// tiles and halo positions, in a grouped slice layout of their own (same
// entry placement rule; each row's entries keep their order): the prolongator
// P inside the layout of its images A P, B P.
struct HostHaloSub {
  int emax = 0;                 // most entries of a pass (4 consecutive slices of a tile)
  std::vector<int> sptr;        // [nslice + 1] slice offsets in steps of 8 entries
  std::vector<uint16_t> lcol;   // local column (halo position) per entry
  std::vector<double> v;        // value per entry
};
void build_halo_sub(int n, const HostHalo& hx, HostHaloSub& out);

// Returns false (format not built) when a single slice references more than
// hmax columns or hmax exceeds the 16-bit local index range.  The matrix may
// be rectangular (columns are any non-negative indices); `c`, when given, is a
// third value array on the same pattern, laid out like the entries into out.c.
bool build_halo(int n, const std::vector<int>& rp, const std::vector<int>& ci,
                const std::vector<double>& a, const std::vector<double>& b, int hmax,
                int rows_cap, HostHalo& out, const std::vector<double>* c = nullptr);

}  // namespace slrf
