// Device-side CG scalar logic (text after Eq. 16: alpha = r.r / p.Ap,
// beta = r_new.r_new / r.r, stop at ||r|| <= eta ||b|| or p.Ap <= 0; the
// single-RVE path forms p.Ap as p.(K:p), see cg_alpha_publish) and the
// fixed-order reductions of the per-block partial sums.
#pragma once

#include "common.hpp"
#include "kernels.hpp"

namespace rve {

// fixed-order reduction over the block (deterministic for a given block
// size)
__device__ __forceinline__ double cg_block_reduce(double v, double* red) {
  return block_sum_fixed(v, red);
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
    sc->rrs[0] = tot;
    sc->rrs[1] = 0.0;
    sc->its[0] = 0;
    sc->its[1] = -1;  // iteration 0 has no previous update
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
    sc->alphas[0] = sc->alphas[1] = 0.0;
    sc->halt[0] = sc->halt[1] = 0;
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

// Copies the scalars into the host's coherent pinned buffer pub (plain
// vector stores, which reach host memory uncached and are complete when
// the kernel is; the host reads them after waiting for an event recorded
// behind the kernel).  Called by every thread of the block: the barrier
// orders the block's own writes to sc before the copy, which reads them
// back from L2 rather than from the scalar cache.
__device__ __forceinline__ void publish_scalars(const Scalars* sc,
                                                Scalars* pub) {
  static_assert(sizeof(Scalars) % 8 == 0, "Scalars copied in 8-byte words");
  constexpr int W = (int)(sizeof(Scalars) / 8);
  __syncthreads();
  const unsigned long long* src = reinterpret_cast<const unsigned long long*>(sc);
  unsigned long long* dst = reinterpret_cast<unsigned long long*>(pub);
  for (int i = threadIdx.x; i < W; i += blockDim.x)
    dst[i] = __hip_atomic_load(src + i, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
}

// ---- reductions consumed by the next kernel ----------------------------------
// Instead of a one-block reduction launch between two kernels, every block
// of the consuming kernel sums the producer's partials itself in a fixed
// order (every consumer of the same partials in the same order, so all get
// the same number) and takes the scalar decision locally; block 0 alone
// publishes the result.  Iteration k (parity p = k & 1) reads slot p ^ 1
// and publishes slot p, so no block reads what another block of the same
// launch writes.

struct BetaStep {
  bool first;   // iteration 0: the direction is r itself
  bool stop;    // converged, capped or non-finite: no further work
  double beta;
};

// The r.r partials of the last inverse pass are summed by every wavefront
// of the consumer on its own: lane l adds partial[l], partial[l + 64], ...
// in index order, then a butterfly over the wavefront (both lanes of a pair
// add the same two numbers), so every wavefront of every consuming kernel
// gets the same bits, with no barrier or LDS.  The first PU loads of each
// lane can be issued early (load), away from the sum (sum).
template <int PU>
struct RrPartials {
  double v[PU];
  __device__ __forceinline__ void load(const double* __restrict__ partial,
                                       int count) {
    const int l = threadIdx.x & 63;
#pragma unroll
    for (int u = 0; u < PU; ++u) {
      const int i = l + 64 * u;
      v[u] = partial[i < count ? i : count - 1];  // clamped: no branch
    }
  }
  __device__ __forceinline__ double sum(const double* __restrict__ partial,
                                        int count) const {
    const int l = threadIdx.x & 63;
    double acc = 0.0;
#pragma unroll
    for (int u = 0; u < PU; ++u) acc += (l + 64 * u < count) ? v[u] : 0.0;
    for (int i = l + 64 * PU; i < count; i += 64) acc += partial[i];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
    return acc;
  }
};

// The CG decision of the direction kernel of parity p (RED_BETA's
// decision) from rr, the sum of the last inverse pass's r.r partials;
// prev = its[p ^ 1] >= 0 (not iteration 0).
__device__ __forceinline__ BetaStep cg_beta_step(Scalars* sc, int p, int prev,
                                                 double rr) {
  BetaStep d{false, false, 0.0};
  const int q = p ^ 1;
  const int k = prev + 1;
  const double rr_prev = sc->rrs[q];
  const bool conv = rr <= sc->eta2bb;
  d.stop = conv || k >= sc->max_iters || !isfinite(rr);
  d.beta = d.stop ? 0.0 : rr / rr_prev;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    sc->rrs[p] = rr;
    sc->its[p] = k;
    sc->iters = k;
    sc->rr_new = rr;
    sc->first = 0;
    if (conv) sc->converged = 1;
    if (d.stop) {
      sc->done = 1;
      sc->halt[p] = 1;
    } else {
      sc->beta = d.beta;
      sc->rr = rr;
    }
  }
  return d;
}

// In the direction kernel of parity p (and in the chunk-closing kernel and
// the fused forward pass): reduce the r.r partials of the last inverse pass
// and take the decision, unless this is iteration 0.
__device__ __forceinline__ BetaStep cg_beta_consume(const double* partial,
                                                    int count, Scalars* sc,
                                                    int p) {
  const int prev = sc->its[p ^ 1];
  if (prev < 0) return BetaStep{true, false, 0.0};
  RrPartials<8> rp;
  rp.load(partial, count);
  return cg_beta_step(sc, p, prev, rp.sum(partial, count));
}

// In block 0 of the forward pass of parity p: reduce the p.(K:p) partials of
// the direction kernel and publish alpha_k = r.r / p.(K:p).  Since p lies in
// the range of the projection G (r and every direction are outputs of G, up
// to rounding) and G is an orthogonal projection, p.G(K:p) = p.(K:p): alpha
// is known before the FFT passes, and the inverse pass can apply
// r -= alpha G(K:p) itself.
__device__ __forceinline__ void cg_alpha_publish(const double* partial,
                                                 int count, Scalars* sc,
                                                 int p, double* red) {
  const double pAp = cg_sum_partials(partial, count, red);
  if (threadIdx.x == 0) {
    sc->pAp = pAp;
    if (!(pAp > 0.0) || !isfinite(pAp)) {
      sc->breakdown = 1;
      sc->done = 1;
      sc->halt[p] = 1;
      sc->iters = sc->its[p] + 1;
    } else {
      const double al = sc->rrs[p] / pAp;
      sc->alpha = al;
      sc->alphas[p] = al;
    }
  }
}

}  // namespace rve
