// Block bodies of the batched CG helper kernels (elementwise update,
// initial residual, per-RVE scalar reductions), shared by their one-launch
// kernels and the persistent CG kernel.  A body takes the index of the
// block it plays (the launch's blockIdx.x, or a virtual block of a
// persistent kernel) and returns early when its RVE takes no part.
#pragma once

#include "cg_scalars.hpp"
#include "kernels.hpp"

namespace rve {

__device__ __forceinline__ int seg_item_of(const SegItem* items, int nitems,
                                           int blk) {
  int r = 0;
  while (r + 1 < nitems && items[r + 1].blk0 <= blk) ++r;
  return r;
}

// per RVE: r = -r64 (active) or 0 (inactive), x = 0, partial sums of r.r
template <typename T>
__device__ __forceinline__ void cg_init_batch_block(
    const SegItem* __restrict__ items, int nitems, int64_t cs,
    const double* __restrict__ r64, T* __restrict__ r, T* __restrict__ x,
    int blk, double* red) {
  const SegItem& it = items[seg_item_of(items, nitems, blk)];
  const bool act = !it.sc->inactive;
  const int lb = blk - it.blk0;
  const int64_t nv = it.n9 / 9;
  double acc = 0.0;
  for (int64_t e = (int64_t)lb * blockDim.x + threadIdx.x; e < it.n9;
       e += (int64_t)it.nblk * blockDim.x) {
    const int64_t i = (e / nv) * cs + it.off + (e % nv);
    const T b = act ? T(-r64[i]) : T(0);
    r[i] = b;
    x[i] = T(0);
    acc += double(b) * double(b);
  }
  const double t = block_sum_fixed(acc, red);
  if (threadIdx.x == 0) it.partial[lb] = t;
}

// x += alpha p, r -= alpha Ap, partial sums of the new r.r
template <typename T>
__device__ __forceinline__ void cg_update_batch_block(
    const SegItem* __restrict__ items, int nitems, int64_t cs,
    T* __restrict__ x, T* __restrict__ r, const T* __restrict__ p,
    const T* __restrict__ Ap, int blk, double* red) {
  const SegItem& it = items[seg_item_of(items, nitems, blk)];
  if (it.sc->done) return;
  const T alpha = T(it.sc->alpha);
  const int lb = blk - it.blk0;
  const int64_t nv = it.n9 / 9;
  double acc = 0.0;
  for (int64_t e = (int64_t)lb * blockDim.x + threadIdx.x; e < it.n9;
       e += (int64_t)it.nblk * blockDim.x) {
    const int64_t i = (e / nv) * cs + it.off + (e % nv);
    x[i] += alpha * p[i];
    const T rn = r[i] - alpha * Ap[i];
    r[i] = rn;
    acc += double(rn) * double(rn);
  }
  const double t = block_sum_fixed(acc, red);
  if (threadIdx.x == 0) it.partial[lb] = t;
}

// the scalars of RVE b from its partial sums (one block), same logic as the
// single-RVE reduction
__device__ __forceinline__ void reduce_batch_block(
    int op, const RedItem* __restrict__ items, Scalars* __restrict__ scs,
    int b, double* red) {
  const RedItem& it = items[b];
  Scalars* sc = scs + b;
  if (op == RED_RESID && sc->inactive) return;
  if ((op == RED_ALPHA || op == RED_BETA) && sc->done) return;
  double acc = 0.0;
  for (int i = threadIdx.x; i < it.count; i += blockDim.x) acc += it.partial[i];
  const double tot = block_sum_fixed(acc, red);
  if (op == RED_RESID) {
    double a2 = 0.0;
    for (int i = threadIdx.x; i < 9 * it.nss; i += blockDim.x) a2 += it.psq[i];
    const double P2 = block_sum_fixed(a2, red);
    for (int c = 0; c < 9; ++c) {
      double a1 = 0.0;
      for (int i = threadIdx.x; i < it.nss; i += blockDim.x)
        a1 += it.psum[c * it.nss + i];
      const double m = block_sum_fixed(a1, red);
      if (threadIdx.x == 0) sc->pbar[c] = m * it.invN3;
    }
    if (threadIdx.x == 0) {
      sc->res2 = tot;
      sc->P2 = P2;
    }
    return;
  }
  if (threadIdx.x != 0) return;
  if (op == RED_INIT) {
    sc->bb = tot;
    sc->rr = tot;
    sc->eta2bb = sc->eta2bb * tot;
    sc->iters = 0;
    sc->first = 1;
    sc->breakdown = 0;
    sc->converged = (tot == 0.0) ? 1 : 0;
    sc->done = (sc->converged || sc->inactive) ? 1 : 0;
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
