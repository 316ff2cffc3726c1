// Device construction of the numeric part of one smoothed-aggregation level
// (the products of the Galerkin coarsening and the prolongator smoothing).
#pragma once

#include <hip/hip_runtime.h>

#include <functional>
#include <string>

#include "amg_host.h"

namespace slrf {

// AmgNumeric on the GPU.  The products are formed in the host code's order
// (Gustavson row order, products rounded before they are added, the power
// iteration's norm summed in row order), so every value equals the host's.
// Scratch memory comes from `take` (256-byte aligned device memory, nullptr
// when the caller's workspace is exhausted); `release` frees everything taken
// so far and is called at the end of each level, after the results have been
// copied back to the host.
struct DeviceAmgNumeric : AmgNumeric {
  std::function<void*(size_t)> take;
  std::function<void()> release;
  hipStream_t stream = nullptr;
  double seconds = 0.0;      // wall time of the levels built so far
  size_t peak_bytes = 0;     // most scratch one level took
  bool level(const HostLevel& L, int nc, const std::vector<int>& trp,
             const std::vector<int>& tci, const std::vector<double>& tv, double omega_p,
             double& rho, HostCsrP& P, HostCsrP& R, HostLevel& APBP, HostLevel& C,
             std::string& err) override;
};

// Most distinct columns of one output row of the device products; a level
// whose products exceed it is reported as an error (the host build has no
// such limit).
constexpr int kAmgRowCap = 1024;

}  // namespace slrf
