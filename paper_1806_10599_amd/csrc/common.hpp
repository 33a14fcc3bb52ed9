// Shared device/host helpers of the HIP library (no method arithmetic).
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>

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

// Events for the next kernel launch made through rve::launch.  The live
// kernel timer sets them just before a timed launch; the launch then records
// them at the start and at the end of that kernel's own execution (AMD's
// extended launch), so the timing holds the kernel alone.
struct NextLaunchEvents {
  hipEvent_t start = nullptr;
  hipEvent_t stop = nullptr;
};
inline thread_local NextLaunchEvents g_next_launch_events;

template <typename F, typename... Args>
inline void launch(F kernel, dim3 grid, dim3 block, uint32_t lds,
                   hipStream_t s, Args... args) {
  NextLaunchEvents& ev = g_next_launch_events;
  if (ev.start) {
    hipEvent_t a = ev.start, b = ev.stop;
    ev = NextLaunchEvents{};
    hipExtLaunchKernelGGL(kernel, grid, block, lds, s, a, b, 0, args...);
  } else {
    hipLaunchKernelGGL(kernel, grid, block, lds, s, args...);
  }
}

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
  // CG iteration k has parity k & 1; slot q holds r.r and the number of
  // completed updates published by the direction kernel of parity q
  double rrs[2];
  int32_t its[2];
  // alpha of the iteration of parity q (published by its forward pass), and
  // whether the CG run has stopped as of that iteration (no update may
  // follow: the direction kernel of the next iteration returns at once)
  double alphas[2];
  int32_t halt[2];
};

constexpr int kBlock = 256;

// Deterministic block sum (blockDim.x a multiple of 64; every thread of the
// block must call it): a butterfly inside each wavefront (both lanes of a
// pair add the same two numbers, so every lane ends with the same value),
// then the wave sums in wave order.  red holds at least blockDim.x / 64
// doubles.  The same inputs give the same bits in every block and launch.
__device__ __forceinline__ double block_sum_fixed(double v, double* red) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  const int nw = (int)(blockDim.x >> 6);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double r = red[0];
  for (int i = 1; i < nw; ++i) r += red[i];
  __syncthreads();
  return r;
}

}  // namespace rve
