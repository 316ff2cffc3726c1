// Host data of the smoothed-aggregation AMG hierarchy shared by all poles.
#pragma once

#include <complex>
#include <string>
#include <vector>

namespace slrf {

// One level operator pair (A_l, B_l) on a shared, row-sorted CSR pattern.
struct HostLevel {
  int n = 0;
  std::vector<int> rp, ci;
  std::vector<double> a, b;
};

// A rectangular real CSR matrix (n x m): prolongator P_l or restriction P_l^T.
struct HostCsrP {
  int n = 0, m = 0;
  std::vector<int> rp, ci;
  std::vector<double> v;
};

struct AmgParams {
  double theta = 0.0;     // strength threshold |a_ij| > theta sqrt(a_ii a_jj)
  double omega_p = 4.0 / 3.0;  // prolongator smoothing weight (times 1/rho(D^-1 A))
  int coarse_max = 400;   // stop coarsening at or below this size
  int dense_max = 2048;   // largest coarsest level inverted densely
  int max_levels = 10;
  int block = 1;          // dofs per node (node-major numbering): nodes are aggregated,
                          // and each aggregate gets one tentative column per dof
  // node coordinates (nodes x block, node-major, same node order as the
  // fine level) for block 2 or 3: the tentative prolongator then carries the
  // rigid-body modes (translations and rotations: 3 in 2D, 6 in 3D) instead
  // of the translations alone, and the coarser levels aggregate scalar dofs
  // with the modes carried as the R factors of the aggregates
  const std::vector<double>* xyz = nullptr;
};

struct AmgHierarchy {
  std::vector<HostLevel> levels;  // levels[0] = fine pencil
  std::vector<HostCsrP> P, R;     // P[l]: n_l x n_{l+1}, R[l] = P[l]^T
  std::vector<double> rho;        // rho[l] = spectral radius estimate of D_l^{-1} A_l
  int nc = 0;                     // coarsest size
  std::vector<std::complex<double>> coarse_inv;  // [pole][nc][nc] row-major
};

// Locality ordering of the rows (order[new] = old) from nested aggregation
// (of the node graph when block > 1, keeping each node's dofs together).
void locality_order(const HostLevel& fine, std::vector<int>& order, int block = 1);

// Dofs per node of a node-major pencil: 3 or 2 when every node's rows share
// one column list made of whole node blocks, else 1.
int detect_block(const HostLevel& L);

// Builds the hierarchy and, for the given poles (none: skipped), the dense
// inverses of the coarsest level operators A_c - sigma_j B_c.
bool amg_build(const HostLevel& fine, const std::vector<std::complex<double>>& poles,
               const AmgParams& prm, AmgHierarchy& H, std::string& err);
// (Re)computes H.coarse_inv for the given poles.
bool amg_coarse_inverses(AmgHierarchy& H, const std::vector<std::complex<double>>& poles,
                         std::string& err);

// The fine-level images of the prolongator, A P and B P (n x P.m, one shared
// row-sorted pattern), and P's values on that pattern (zero where P has no
// entry; P's pattern lies inside it because every row of A has its diagonal).
// Returns false if some entry of P falls outside the pattern.
bool fine_image(const HostLevel& L, const HostCsrP& P, std::vector<int>& rp,
                std::vector<int>& ci, std::vector<double>& ap, std::vector<double>& bp,
                std::vector<double>& pv);

}  // namespace slrf
