// Host FP64 dense helpers for the small projected problems (row-major, ld = n).
#pragma once

namespace slrf {

// G = R^T R in place (R upper); false if G is not numerically positive definite.
bool chol_upper(int n, double* G);
// In-place inverse of an upper-triangular matrix.
void tri_upper_inverse(int n, double* R);
// Symmetric eigen-decomposition: w ascending, V orthonormal eigenvectors (columns).
bool sym_eig(int n, const double* A, double* w, double* V);
// Symmetric-definite generalised problem Ah s = theta Bh s with S^T Bh S = I and
// theta ascending; returns the number of pairs (< n when Bh was numerically
// singular and had to be truncated; trailing theta set to +inf), -1 on failure.
int sym_gen_eig(int n, const double* Ah, const double* Bh, double* theta, double* S,
                int* used_fallback);

}  // namespace slrf
