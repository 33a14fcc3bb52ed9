// Shared device/host helpers of the HIP library (no method arithmetic).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <stdexcept>
#include <string>

namespace rve {

template <typename T>
struct cplx {
  T x, y;
};

template <typename T>
__device__ __forceinline__ cplx<T> cadd(cplx<T> a, cplx<T> b) {
  return {a.x + b.x, a.y + b.y};
}
template <typename T>
__device__ __forceinline__ cplx<T> csub(cplx<T> a, cplx<T> b) {
  return {a.x - b.x, a.y - b.y};
}
template <typename T>
__device__ __forceinline__ cplx<T> cmul(cplx<T> a, cplx<T> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename T>
__device__ __forceinline__ cplx<T> cconj(cplx<T> a) {
  return {a.x, -a.y};
}
template <typename T>
__device__ __forceinline__ cplx<T> cscale(cplx<T> a, T s) {
  return {a.x * s, a.y * s};
}

// Error carried out of the engine to the C ABI.
struct Error : std::runtime_error {
  int code;
  Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

#define RVE_HIP(expr)                                                       \
  do {                                                                      \
    hipError_t e_ = (expr);                                                 \
    if (e_ != hipSuccess)                                                   \
      throw ::rve::Error(-3, std::string(#expr) + ": " +                    \
                                 hipGetErrorString(e_));                    \
  } while (0)

// Device-side scalars of one CG solve (and the residual norms).
struct Scalars {
  double rr;        // r.r of the current CG residual
  double rr_new;
  double pAp;
  double alpha;
  double beta;
  double bb;        // ||b||^2
  double eta2bb;    // cg_tol^2 ||b||^2
  double res2;      // ||G(P)||^2 (FP64)
  double P2;        // ||P||^2
  int32_t done;     // CG finished (converged, breakdown or cap)
  int32_t converged;
  int32_t breakdown;
  int32_t iters;
  int32_t max_iters;
  int32_t first;    // next pass-A call starts a new direction p = r
  int32_t fails;    // return-mapping failures of the last evaluation
  int32_t inactive;  // batch: this RVE takes no part in the current work
  int32_t commit;    // batch: commit this RVE's trial state
  int32_t pad;
  double pbar[9];   // <P> of the last residual evaluation
};

constexpr int kBlock = 256;

}  // namespace rve
