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
  // smallest coarse level worth forming: where the aggregation would leave
  // fewer coarse dofs, the strength threshold is raised (0.01, 0.02, ... 0.64)
  // to the first value that leaves at least this many while still halving the
  // level; if none does, a level that fits the dense solve becomes the
  // coarsest, and a larger one takes the largest halving coarse space the
  // thresholds gave (0: off)
  int coarse_min = 0;
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
  // img[l]: A_l P_l and B_l P_l (a and b on one row-sorted pattern), formed for
  // the Galerkin product and kept for the fine-level images (may be cleared)
  std::vector<HostLevel> img;
};

// Locality ordering of the rows (order[new] = old) from nested aggregation
// (of the node graph when block > 1, keeping each node's dofs together).
void locality_order(const HostLevel& fine, std::vector<int>& order, int block = 1);

// Dofs per node of a node-major pencil: 3 or 2 when every node's rows share
// one column list made of whole node blocks, else 1.
int detect_block(const HostLevel& L);

// The numeric work of one level, given the level operator L and the tentative
// prolongator T (n x nc): rho = rho(D^-1 A) by 20 power steps from a fixed
// seeded start, P = T - (omega_p / rho) D^-1 A T, R = P^T, APBP = (A P, B P) on
// one pattern and C = (R (A P), R (B P)), every product in Gustavson order with
// row-sorted output (C not yet symmetrised).
struct AmgNumeric {
  virtual ~AmgNumeric() = default;
  virtual bool level(const HostLevel& L, int nc, const std::vector<int>& trp,
                     const std::vector<int>& tci, const std::vector<double>& tv, double omega_p,
                     double& rho, HostCsrP& P, HostCsrP& R, HostLevel& APBP, HostLevel& C,
                     std::string& err) = 0;
};
// The host implementation of AmgNumeric::level.
bool host_level_products(const HostLevel& L, int nc, const std::vector<int>& trp,
                         const std::vector<int>& tci, const std::vector<double>& tv,
                         double omega_p, double& rho, HostCsrP& P, HostCsrP& R,
                         HostLevel& APBP, HostLevel& C);
// The power iteration's start vector for a level of n rows.
std::vector<double> rho_start_vector(int n);

// Builds the hierarchy and, for the given poles (none: skipped), the dense
// inverses of the coarsest level operators A_c - sigma_j B_c.  The aggregation
// and the tentative prolongators run on the host; each level's products run
// through `num` (the host's own when null).
bool amg_build(const HostLevel& fine, const std::vector<std::complex<double>>& poles,
               const AmgParams& prm, AmgHierarchy& H, std::string& err,
               AmgNumeric* num = nullptr);
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
// P's values on the pattern of its images (APBP: the A P / B P pattern of
// AmgHierarchy::img); false if some entry of P falls outside it.
bool image_p_values(const HostLevel& APBP, const HostCsrP& P, std::vector<double>& pv);

}  // namespace slrf
