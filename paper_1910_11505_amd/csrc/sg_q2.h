// Q2 (biquadratic) form of the SG operator apply and load (Sec. 2.2: the
// paper's spatial space).  n2 elements per side; the unknowns of a mode are
// the (2 n2 - 1)^2 interior nodes of the twice-refined grid, node
// (ix, iy) at (iy-1)(2 n2 - 1) + (ix-1); vectors are mode-major.  Gauss
// points: 3 x 3 per element; per-point device arrays are local-point major,
// q = (3 qy + qx) n2^2 + e with e = ey n2 + ex, so that consecutive threads
// (consecutive elements) touch consecutive addresses.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace sg {

// KL variables a Gauss point carries at most (the problem limit on M)
constexpr int kQ2MaxM = 12;

// the Hermite translation matrix T(g) of the factored apply
// (sum_k a_k G_k = a_min I + exp(mu + |g|^2/2) T T^T) as two CSR lists of its
// nonzeros T_{alpha beta} = c * g^(alpha - beta), beta <= alpha:
//  by column beta: ptr1 (P+1), row index alpha, c, packed exponents;
//  by row alpha:   ptr2 (P+1), column index beta, c, packed exponents.
// Exponents are packed 4 bits per KL variable (variable m at bits 4m..4m+3).
struct Q2TDev {
  const int *ptr1 = nullptr, *idx1 = nullptr, *ptr2 = nullptr, *idx2 = nullptr;
  const double *c1 = nullptr, *c2 = nullptr;
  const uint64_t *e1 = nullptr, *e2 = nullptr;
};

// W = K U on Q2.  g: KL values at the Gauss points, M x 9 n2^2 (point
// fastest).  grad and y: device scratch of 2 P 9 n2^2 doubles each (the
// per-point gradients, overwritten by the fluxes, and T^T grad).
void launch_q2_apply(hipStream_t s, int n2, int M, int P, double mu, double a_min,
                     const double* g, const Q2TDev& T, const double* U, double* W, double* grad,
                     double* y);

// F = e_0 (x) M f: f at the (2 n2 + 1)^2 refined-grid nodes; modes > 0 zero.
void launch_q2_rhs(hipStream_t s, int n2, int P, const double* f, double* F);

}  // namespace sg
