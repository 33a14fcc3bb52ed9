// Device-side CG scalar logic (text after Eq. 16: alpha = r.r / p.Ap,
// beta = r_new.r_new / r.r, stop at ||r|| <= eta ||b|| or p.Ap <= 0) and the
// fixed-order reductions of the per-block partial sums.
#pragma once

#include "common.hpp"
#include "kernels.hpp"

namespace rve {

// fixed-order tree over the block (deterministic for a given block size)
__device__ __forceinline__ double cg_block_reduce(double v, double* red) {
  const int t = threadIdx.x;
  red[t] = v;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (t < s) red[t] += red[t + s];
    __syncthreads();
  }
  const double r = red[0];
  __syncthreads();
  return r;
}

// sum of partial[0 .. count) by one block: each thread sums a strided
// subset in index order, then the block tree
__device__ __forceinline__ double cg_sum_partials(const double* partial,
                                                  int count, double* red) {
  double acc = 0.0;
  for (int i = threadIdx.x; i < count; i += blockDim.x) acc += partial[i];
  return cg_block_reduce(acc, red);
}

// the scalar update of RED_INIT / RED_ALPHA / RED_BETA given the total
__device__ __forceinline__ void cg_scalar_update(int op, double tot,
                                                 Scalars* sc) {
  if (op == RED_INIT) {
    sc->bb = tot;
    sc->rr = tot;
    sc->eta2bb = sc->eta2bb * tot;  // eta^2 was stored by the init kernel
    sc->iters = 0;
    sc->first = 1;
    sc->breakdown = 0;
    sc->converged = (tot == 0.0) ? 1 : 0;
    sc->done = sc->converged;
    sc->alpha = 0.0;
    sc->beta = 0.0;
  } else if (op == RED_ALPHA) {
    sc->pAp = tot;
    if (!(tot > 0.0) || !isfinite(tot)) {
      sc->breakdown = 1;
      sc->done = 1;
      sc->iters += 1;
    } else {
      sc->alpha = sc->rr / tot;
    }
  } else if (op == RED_BETA) {
    sc->iters += 1;
    sc->rr_new = tot;
    sc->first = 0;
    if (tot <= sc->eta2bb) {
      sc->converged = 1;
      sc->done = 1;
    } else if (sc->iters >= sc->max_iters || !isfinite(tot)) {
      sc->done = 1;
    } else {
      sc->beta = tot / sc->rr;
      sc->rr = tot;
    }
  }
}

}  // namespace rve
