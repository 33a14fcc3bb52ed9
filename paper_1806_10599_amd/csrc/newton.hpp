// Control of the Newton iteration shared by single and batched solves.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

namespace rve {

// Share of the residual used by the superlinear term of forcing mode 2.
constexpr double kForcingTheta = 0.05;

// Relative tolerance of the linear solve of a Newton iteration that starts
// at the FP64 relative residual rel (inexact Newton; the equilibrium test
// itself never changes):
//   0: cg_tol;
//   1: min(0.1, max(cg_tol, newton_tol / (4 rel))): only as tight as
//      reaching the equilibrium tolerance needs (the linear part of the
//      next residual at most a quarter of the tolerance);
//   2: min(0.1, max(cg_tol, newton_tol / (2 rel), kForcingTheta * rel)):
//      half of the tolerance for the linear part (the quadratic remainder
//      of the last correction is orders of magnitude below it), and never
//      tighter than kForcingTheta * rel: far from equilibrium the next
//      residual is dominated by the quadratic term of Newton's method,
//      which a tighter solve cannot reduce.
// (host and device: the batch takes the decision on the device)
__host__ __device__ inline double forcing_eta(int32_t mode, double cg_tol,
                                              double newton_tol, double rel) {
  if (mode == 0 || !(rel > 0.0)) return cg_tol;
  double eta = fmax(cg_tol, (mode == 2 ? 0.5 : 0.25) * newton_tol / rel);
  if (mode == 2) eta = fmax(eta, kForcingTheta * rel);
  return fmin(0.1, eta);
}

}  // namespace rve
