// Elementwise and reduction kernels of the Newton-CG increment:
//   predictor F = F_prev + dFbar (Sec. 2.1, Eq. 12 with the homogeneous
//   first guess), CG vector updates with FP64-accumulated dot products and
//   fixed-order (deterministic) reductions (text after Eq. 16), the Newton
//   update F += dF, the commit of the increment with the fatigue indicators
//   of Sec. 3.3, Eqs. 23-24.
#include "batch_cg.hpp"
#include "cg_scalars.hpp"
#include "kernels.hpp"
#include "newton.hpp"

namespace rve {

namespace {

__device__ __forceinline__ double block_reduce(double v, double* red) {
  return block_sum_fixed(v, red);
}

}  // namespace

__global__ void predict_kernel(double* __restrict__ F,
                               const double* __restrict__ Fp, int64_t N,
                               double d0, double d1, double d2, double d3,
                               double d4, double d5, double d6, double d7,
                               double d8) {
  const double d[9] = {d0, d1, d2, d3, d4, d5, d6, d7, d8};
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < 9 * N;
       i += (int64_t)gridDim.x * blockDim.x)
    F[i] = Fp[i] + d[i / N];
}

void launch_predict(double* F, const double* Fprev, const double dFbar[9],
                    int64_t N, hipStream_t s) {
  hipLaunchKernelGGL(predict_kernel, dim3(2048), dim3(kBlock), 0, s, F, Fprev,
                     N, dFbar[0], dFbar[1], dFbar[2], dFbar[3], dFbar[4],
                     dFbar[5], dFbar[6], dFbar[7], dFbar[8]);
}

// r = -r64 (rounded to T), x = 0, partial sums of r.r
template <typename T>
__global__ __launch_bounds__(kBlock) void cg_init_kernel(
    const double* __restrict__ r64, T* __restrict__ r, T* __restrict__ x,
    double* __restrict__ partial, int64_t n9) {
  __shared__ double red[kBlock];
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n9;
       i += (int64_t)gridDim.x * blockDim.x) {
    const T b = T(-r64[i]);
    r[i] = b;
    x[i] = T(0);
    acc += double(b) * double(b);
  }
  const double t = block_reduce(acc, red);
  if (threadIdx.x == 0) partial[blockIdx.x] = t;
}

template <typename T>
void launch_cg_init(const double* r64, T* r, T* x, double* partial, int nblk,
                    int64_t n9, hipStream_t s) {
  hipLaunchKernelGGL((cg_init_kernel<T>), dim3(nblk), dim3(kBlock), 0, s, r64,
                     r, x, partial, n9);
}

// CG direction and material product (Sec. 2.1, Eqs. 15-16): per voxel
// p = r (first iteration) or r + beta p_old, then y = K : p
// (y_c = sum_d K[9c + d] p_d); one voxel per thread, K streamed once,
// coalesced per component.  With partial != null (a CG run) the kernel
// takes the CG decision itself from the r.r partials of the last inverse
// pass and, from the second iteration on, applies the previous iteration's
// x += alpha p_old (its alpha was published by that iteration's forward
// pass); it returns at once when the previous iteration halted the run, and
// applies only the pending x update when this one stops it.  The decision
// waits for the partials while the voxel's r, p_old and first KP entries of
// K are already in flight: their loads are issued first, unconditionally
// (clamped indices), so that the partial sum's latency hides behind them.
// Without partial it takes first, beta and alpha from the scalars (kernel
// timing).  With pkp != null each block writes its partial of p . (K : p).
template <typename T, int PU>
__global__ __launch_bounds__(kBlock) void kp_kernel(
    const T* __restrict__ K, const T* __restrict__ r,
    const T* __restrict__ p_old, T* __restrict__ p_new, T* __restrict__ y,
    T* __restrict__ x, Scalars* __restrict__ sc, int64_t N,
    const double* __restrict__ partial, int count,
    double* __restrict__ pkp, int parity) {
  // FP32: the voxel's r, p_old and first KP entries of K loaded before the
  // decision, the rest of K right after it (about 120 VGPRs, four waves per
  // SIMD); FP64: everything after it, K read inside the product (holding
  // the data across the decision would halve the occupancy)
  constexpr bool kEarly = sizeof(T) == 4;
  constexpr int KP = kEarly ? 36 : 0;
  __shared__ double red[kBlock];
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t vl = v < N ? v : N - 1;
  RrPartials<kEarly ? PU : 1> rp;
  if (partial && kEarly) rp.load(partial, count);
  T kv[81], rv[9], pv[9];
  auto load_vectors = [&] {
#pragma unroll
    for (int d = 0; d < 9; ++d) {
      rv[d] = r[d * N + vl];
      pv[d] = p_old[d * N + vl];
    }
  };
  if constexpr (kEarly) load_vectors();
#pragma unroll
  for (int i = 0; i < KP; ++i) kv[i] = K[i * N + vl];
  bool first, upd, stop = false;
  T beta, alpha_prev;
  if (partial) {
    // every flag read here was written by an earlier launch: block 0 of this
    // launch publishes slot `parity` (and done), which no block reads
    const int q = parity ^ 1;
    if (sc->halt[q]) {
      if (blockIdx.x == 0 && threadIdx.x == 0) sc->halt[parity] = 1;
      return;
    }
    const int prev = sc->its[q];
    first = prev < 0;
    BetaStep d{first, false, 0.0};
    if (!first) {
      if constexpr (!kEarly) rp.load(partial, count);
      d = cg_beta_step(sc, parity, prev, rp.sum(partial, count));
    }
    if (first && sc->done) return;  // b = 0: nothing to solve
    upd = !first && x != nullptr;
    alpha_prev = T(sc->alphas[q]);
    stop = d.stop;
    beta = T(d.beta);
  } else {
    if (sc->done) return;
    first = sc->first != 0;
    beta = T(sc->beta);
    upd = x != nullptr;
    alpha_prev = T(sc->alpha);
  }
  if constexpr (!kEarly) load_vectors();
  double acc = 0.0;
  if (v < N) {
    if (stop) {
#pragma unroll
      for (int d = 0; d < 9; ++d)
        if (upd) x[d * N + v] += alpha_prev * pv[d];
      return;
    }
    if constexpr (kEarly) {
#pragma unroll
      for (int i = KP; i < 81; ++i) kv[i] = K[i * N + v];
    }
    T pd[9];
#pragma unroll
    for (int d = 0; d < 9; ++d) {
      T val = rv[d];
      if (!first) val += beta * pv[d];
      if (upd) x[d * N + v] += alpha_prev * pv[d];
      pd[d] = val;
      p_new[d * N + v] = val;
    }
#pragma unroll
    for (int c = 0; c < 9; ++c) {
      T acc_c = T(0);
#pragma unroll
      for (int d = 0; d < 9; ++d)
        acc_c += (kEarly ? kv[9 * c + d] : K[(9 * c + d) * N + v]) * pd[d];
      y[c * N + v] = acc_c;
      acc += double(pd[c]) * double(acc_c);
    }
  }
  if (stop) return;
  if (pkp) {
    const double t = block_reduce(acc, red);
    if (threadIdx.x == 0) pkp[blockIdx.x] = t;
  }
}

int kp_blocks(int64_t N) { return (int)((N + kBlock - 1) / kBlock); }

template <typename T>
void launch_kp(const T* K, const T* r, const T* p_old, T* p_new, T* y,
               Scalars* sc, int64_t N, hipStream_t s, const double* partial,
               int count, int parity, T* x, double* pkp) {
  // early partial loads per lane: all of them up to 576 (64^3 with one
  // component per slab block) or 1152 partials
  const dim3 grid((unsigned)kp_blocks(N));
  if (count <= 9 * 64)
    launch((kp_kernel<T, 9>), grid, dim3(kBlock), 0, s, K, r, p_old, p_new, y,
           x, sc, N, partial, count, pkp, parity);
  else
    launch((kp_kernel<T, 18>), grid, dim3(kBlock), 0, s, K, r, p_old, p_new,
           y, x, sc, N, partial, count, pkp, parity);
}

template void launch_kp<float>(const float*, const float*, const float*,
                               float*, float*, Scalars*, int64_t, hipStream_t,
                               const double*, int, int, float*, double*);
template void launch_kp<double>(const double*, const double*, const double*,
                                double*, double*, Scalars*, int64_t,
                                hipStream_t, const double*, int, int, double*,
                                double*);

template <typename T>
__global__ void add_to_F_kernel(double* __restrict__ F,
                                const T* __restrict__ x, int64_t n9) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n9;
       i += (int64_t)gridDim.x * blockDim.x)
    F[i] += double(x[i]);
}

template <typename T>
void launch_add_to_F(double* F, const T* x, int64_t n9, hipStream_t s) {
  hipLaunchKernelGGL((add_to_F_kernel<T>), dim3(2048), dim3(kBlock), 0, s, F,
                     x, n9);
}

template <typename T>
__global__ void convert_kernel(const double* __restrict__ in,
                               T* __restrict__ out, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    out[i] = T(in[i]);
}

template <typename T>
void launch_convert(const double* in, T* out, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL((convert_kernel<T>), dim3(2048), dim3(kBlock), 0, s, in,
                     out, n);
}

// Single-block fixed-order reductions that also advance the CG scalars.
__global__ __launch_bounds__(kBlock) void reduce_kernel(
    int op, const double* __restrict__ partial, int count,
    const double* __restrict__ psum, const double* __restrict__ psq, int nss,
    double invN3, Scalars* __restrict__ sc, double* __restrict__ pbar,
    Scalars* pub) {
  __shared__ double red[kBlock];
  if ((op == RED_ALPHA || op == RED_BETA) && sc->done) return;
  const double tot = cg_sum_partials(partial, count, red);
  if (op == RED_RESID) {
    double a2 = 0.0;
    for (int i = threadIdx.x; i < 9 * nss; i += blockDim.x) a2 += psq[i];
    const double P2 = block_reduce(a2, red);
    for (int c = 0; c < 9; ++c) {
      double a1 = 0.0;
      for (int i = threadIdx.x; i < nss; i += blockDim.x) a1 += psum[c * nss + i];
      const double m = block_reduce(a1, red);
      if (threadIdx.x == 0) pbar[c] = m * invN3;
    }
    if (threadIdx.x == 0) {
      sc->res2 = tot;
      sc->P2 = P2;
    }
    if (pub) publish_scalars(sc, pub);
    return;
  }
  if (threadIdx.x != 0) return;
  cg_scalar_update(op, tot, sc);
}

// End of a CG chunk: the decision the direction kernel of the next
// iteration (parity p) would take, published for the host; it writes only
// slot p, which that kernel rewrites with the same values.  When it stops
// the run, that direction kernel (always queued after it) still applies the
// pending x += alpha p.
__global__ __launch_bounds__(kBlock) void cg_close_kernel(
    const double* __restrict__ partial, int count, Scalars* __restrict__ sc,
    int p, Scalars* pub) {
  if (!sc->done) (void)cg_beta_consume(partial, count, sc, p);
  if (pub) publish_scalars(sc, pub);
}

void launch_cg_close(const double* partial, int count, Scalars* sc,
                     int parity, hipStream_t s, Scalars* pub) {
  hipLaunchKernelGGL(cg_close_kernel, dim3(1), dim3(kBlock), 0, s, partial,
                     count, sc, parity, pub);
}

void launch_reduce(int op, const double* partial, int count,
                   const double* psum, const double* psq, int nss,
                   double invN3, Scalars* sc, double* pbar, hipStream_t s,
                   Scalars* pub) {
  hipLaunchKernelGGL(reduce_kernel, dim3(1), dim3(kBlock), 0, s, op, partial,
                     count, psum, psq, nss, invN3, sc, pbar, pub);
}

__global__ void init_scalars_kernel(Scalars* sc, int max_iters, double eta) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    sc->max_iters = max_iters;
    sc->eta2bb = eta * eta;
    sc->done = 0;
    sc->fails = 0;
  }
}

__global__ void bench_scalars_kernel(Scalars* sc) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    // a matvec on p = r + 0 p_old that leaves the vectors unchanged
    // (alpha = beta = 0) and reads p_old as every iteration after the first
    sc->done = 0;
    sc->first = 0;
    sc->alpha = 0.0;
    sc->beta = 0.0;
    sc->alphas[0] = sc->alphas[1] = 0.0;
  }
}

void launch_bench_scalars(Scalars* sc, hipStream_t s) {
  hipLaunchKernelGGL(bench_scalars_kernel, dim3(1), dim3(64), 0, s, sc);
}

void launch_init_scalars(Scalars* sc, int max_iters, double eta,
                         hipStream_t s) {
  hipLaunchKernelGGL(init_scalars_kernel, dim3(1), dim3(64), 0, s, sc,
                     max_iters, eta);
}

// Commit: accumulate the indicator fields from the converged trial state.
//   dLp = sum_a dg_a s_a (x) m_a;  Pcyc += sqrt(2/3 dLp:dLp);
//   Pcyc_lit += dLp:dLp / dt;  W_a += tau_a dg_a.
__global__ __launch_bounds__(kBlock) void commit_kernel(CommitArgs A) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= A.N) return;
  const int64_t N = A.N;
  const double* __restrict__ tb = A.table + (int64_t)A.phase[v] * kTableStride;
  if (tb[0] != 0.0) return;  // elastic particles accumulate nothing
  double dLp[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  double dg[12];
#pragma unroll
  for (int al = 0; al < 12; ++al) {
    dg[al] = A.dg_t[al * N + v];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j)
        dLp[3 * i + j] += dg[al] * tb[kTabS + 3 * al + i] * tb[kTabM + 3 * al + j];
  }
  double dd = 0.0;
#pragma unroll
  for (int i = 0; i < 9; ++i) dd += dLp[i] * dLp[i];
  A.pcyc[v] += sqrt(2.0 / 3.0 * dd);
  A.pcyc_lit[v] += dd / A.dt;
  // resolved shear stresses at the converged state
  double F[9], Fpi[9], Fe[9];
#pragma unroll
  for (int c = 0; c < 9; ++c) {
    F[c] = A.F[c * N + v];
    Fpi[c] = A.Fpi_t[c * N + v];
  }
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j)
      Fe[3 * i + j] = F[3 * i] * Fpi[j] + F[3 * i + 1] * Fpi[3 + j] +
                      F[3 * i + 2] * Fpi[6 + j];
  double C[9];
#pragma unroll
  for (int p = 0; p < 3; ++p)
#pragma unroll
    for (int q = 0; q < 3; ++q)
      C[3 * p + q] = Fe[p] * Fe[q] + Fe[3 + p] * Fe[3 + q] + Fe[6 + p] * Fe[6 + q];
  const double E[6] = {0.5 * (C[0] - 1.0), 0.5 * (C[4] - 1.0),
                       0.5 * (C[8] - 1.0), 0.5 * C[5],
                       0.5 * C[2],         0.5 * C[1]};
  const double w[6] = {1, 1, 1, 2, 2, 2};
  double S[6];
#pragma unroll
  for (int I = 0; I < 6; ++I) {
    double acc = 0.0;
#pragma unroll
    for (int J = 0; J < 6; ++J) acc += tb[kTabC + 6 * I + J] * w[J] * E[J];
    S[I] = acc;
  }
#pragma unroll
  for (int al = 0; al < 12; ++al) {
    const double* s = tb + kTabS + 3 * al;
    const double* m = tb + kTabM + 3 * al;
    const double Sm0 = S[0] * m[0] + S[5] * m[1] + S[4] * m[2];
    const double Sm1 = S[5] * m[0] + S[1] * m[1] + S[3] * m[2];
    const double Sm2 = S[4] * m[0] + S[3] * m[1] + S[2] * m[2];
    const double tau = s[0] * Sm0 + s[1] * Sm1 + s[2] * Sm2;
    A.wcyc[al * N + v] += tau * dg[al];
  }
}

void launch_commit(const CommitArgs& a, hipStream_t s) {
  const int64_t grid = (a.N + kBlock - 1) / kBlock;
  hipLaunchKernelGGL(commit_kernel, dim3((unsigned)grid), dim3(kBlock), 0, s, a);
}

__global__ void fill_i32_kernel(int32_t* p, int32_t v, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}
__global__ void fill_f64_kernel(double* p, double v, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

void launch_fill_i32(int32_t* p, int32_t v, int64_t n, hipStream_t s) {
  const int64_t g = (n + kBlock - 1) / kBlock;
  hipLaunchKernelGGL(fill_i32_kernel, dim3((unsigned)(g < 2048 ? (g > 0 ? g : 1) : 2048)),
                     dim3(kBlock), 0, s, p, v, n);
}
void launch_fill_f64(double* p, double v, int64_t n, hipStream_t s) {
  const int64_t g = (n + kBlock - 1) / kBlock;
  hipLaunchKernelGGL(fill_f64_kernel, dim3((unsigned)(g < 2048 ? (g > 0 ? g : 1) : 2048)),
                     dim3(kBlock), 0, s, p, v, n);
}

// sigma = P F^T / det F
__global__ void cauchy_kernel(const double* __restrict__ F,
                              const double* __restrict__ P,
                              double* __restrict__ sig, int64_t N) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= N) return;
  double f[9], p[9];
#pragma unroll
  for (int c = 0; c < 9; ++c) {
    f[c] = F[c * N + v];
    p[c] = P[c * N + v];
  }
  const double J = f[0] * (f[4] * f[8] - f[5] * f[7]) -
                   f[1] * (f[3] * f[8] - f[5] * f[6]) +
                   f[2] * (f[3] * f[7] - f[4] * f[6]);
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j)
      sig[(3 * i + j) * N + v] =
          (p[3 * i] * f[3 * j] + p[3 * i + 1] * f[3 * j + 1] +
           p[3 * i + 2] * f[3 * j + 2]) / J;
}

void launch_cauchy(const double* F, const double* P, double* sig, int64_t N,
                   hipStream_t s) {
  const int64_t g = (N + kBlock - 1) / kBlock;
  hipLaunchKernelGGL(cauchy_kernel, dim3((unsigned)g), dim3(kBlock), 0, s, F, P,
                     sig, N);
}

template void launch_cg_init<float>(const double*, float*, float*, double*,
                                    int, int64_t, hipStream_t);
template void launch_cg_init<double>(const double*, double*, double*, double*,
                                     int, int64_t, hipStream_t);
template void launch_add_to_F<float>(double*, const float*, int64_t,
                                     hipStream_t);
template void launch_add_to_F<double>(double*, const double*, int64_t,
                                      hipStream_t);
template void launch_convert<float>(const double*, float*, int64_t,
                                    hipStream_t);
template void launch_convert<double>(const double*, double*, int64_t,
                                     hipStream_t);


// ------------------------------------------------------------------ batch
// (block bodies in batch_cg.hpp)
template <typename T>
__global__ __launch_bounds__(kBlock) void cg_init_batch_kernel(
    const SegItem* __restrict__ items, int nitems, int64_t cs,
    const double* __restrict__ r64, T* __restrict__ r, T* __restrict__ x) {
  __shared__ double red[kBlock / 64];
  cg_init_batch_block<T>(items, nitems, cs, r64, r, x, blockIdx.x, red);
}

template <typename T>
void launch_cg_init_batch(const SegItem* items, int nitems, int blocks,
                          int64_t cs, const double* r64, T* r, T* x,
                          hipStream_t s) {
  hipLaunchKernelGGL((cg_init_batch_kernel<T>), dim3(blocks), dim3(kBlock), 0,
                     s, items, nitems, cs, r64, r, x);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void cg_update_batch_kernel(
    const SegItem* __restrict__ items, int nitems, int64_t cs,
    T* __restrict__ x, T* __restrict__ r, const T* __restrict__ p,
    const T* __restrict__ Ap) {
  __shared__ double red[kBlock / 64];
  cg_update_batch_block<T>(items, nitems, cs, x, r, p, Ap, blockIdx.x, red);
}

template <typename T>
void launch_cg_update_batch(const SegItem* items, int nitems, int blocks,
                            int64_t cs, T* x, T* r, const T* p, const T* Ap,
                            hipStream_t s) {
  hipLaunchKernelGGL((cg_update_batch_kernel<T>), dim3(blocks), dim3(kBlock),
                     0, s, items, nitems, cs, x, r, p, Ap);
}

// one block per RVE
__global__ __launch_bounds__(kBlock) void reduce_batch_kernel(
    int op, const RedItem* __restrict__ items, Scalars* __restrict__ scs) {
  __shared__ double red[kBlock / 64];
  reduce_batch_block(op, items, scs, blockIdx.x, red);
}

void launch_reduce_batch(int op, const RedItem* items, int nitems,
                         Scalars* scs, hipStream_t s) {
  hipLaunchKernelGGL(reduce_batch_kernel, dim3(nitems), dim3(kBlock), 0, s, op,
                     items, scs);
}

__global__ void newton_control_batch_kernel(Scalars* __restrict__ scs,
                                            BatchLog* __restrict__ log,
                                            int nitems, int it, NewtonCtl ctl) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nitems) return;
  Scalars& sc = scs[b];
  BatchLog& L = log[b];
  if (L.status != 1) return;
  if (it > 0) {  // the linear solve of the previous iteration
    if (it - 1 < kBatchLog) L.cg_hist[it - 1] = sc.iters;
    L.cg_total += sc.iters;
    L.breakdowns += sc.breakdown ? 1 : 0;
  }
  const double res = sqrt(sc.res2), pn = sqrt(sc.P2);
  const double rel = pn > 0.0 ? res / pn : 0.0;
  if (it < kBatchLog) L.res_hist[it] = rel;
  if (it == 0) L.predictor_rel = rel;
  L.rel = rel;
  for (int c = 0; c < 9; ++c) L.pbar[c] = sc.pbar[c];
  L.newton_iters = it;
  int st = 1;
  if (sc.fails > 0) {
    L.fails = sc.fails;
    st = -5;   // RVE_ELOCAL
  } else if (res <= ctl.newton_tol * pn) {
    st = 0;    // RVE_OK
    sc.commit = 1;
  } else if (it >= ctl.newton_max) {
    st = -4;   // RVE_ENOTCONV
  }
  L.status = st;
  if (st != 1) {
    sc.inactive = 1;
    sc.done = 1;
    return;
  }
  const double eta = forcing_eta(ctl.forcing, ctl.cg_tol, ctl.newton_tol, rel);
  sc.max_iters = ctl.cg_max;
  sc.eta2bb = eta * eta;
  sc.done = 0;
  sc.fails = 0;
}

void launch_newton_control_batch(Scalars* scs, BatchLog* log, int nitems,
                                 int it, const NewtonCtl& ctl, hipStream_t s) {
  hipLaunchKernelGGL(newton_control_batch_kernel,
                     dim3((unsigned)((nitems + 63) / 64)), dim3(64), 0, s, scs,
                     log, nitems, it, ctl);
}

__global__ void predict_batch_kernel(double* __restrict__ F,
                                     const double* __restrict__ Fp,
                                     const uint8_t* __restrict__ vrve,
                                     const double* __restrict__ dF, int64_t N) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < 9 * N;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t c = i / N;
    F[i] = Fp[i] + dF[9 * vrve[i - c * N] + c];
  }
}

void launch_predict_batch(double* F, const double* Fprev, const uint8_t* vrve,
                          const double* dF, int64_t N, hipStream_t s) {
  hipLaunchKernelGGL(predict_batch_kernel, dim3(2048), dim3(kBlock), 0, s, F,
                     Fprev, vrve, dF, N);
}

// commit of the RVEs flagged in their scalars: committed state <- trial,
// F_prev <- F, the fluctuation increment, and the indicator fields
__global__ __launch_bounds__(kBlock) void commit_batch_kernel(CommitBatchArgs A) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= A.N) return;
  const int b = A.vrve[v];
  if (!A.scs[b].commit) return;
  const int64_t N = A.N;
  double F[9], Fpi[9];
#pragma unroll
  for (int c = 0; c < 9; ++c) {
    F[c] = A.F[c * N + v];
    Fpi[c] = A.Fpi_t[c * N + v];
    A.dFt[c * N + v] = F[c] - A.Fprev[c * N + v] - A.dF[9 * b + c];
    A.Fprev[c * N + v] = F[c];
    A.Pc[c * N + v] = A.P[c * N + v];
    A.Fpi_c[c * N + v] = Fpi[c];
  }
  double dg[12];
#pragma unroll
  for (int al = 0; al < 12; ++al) {
    dg[al] = A.dg_t[al * N + v];
    A.dg_c[al * N + v] = dg[al];
    A.chi_c[al * N + v] = A.chi_t[al * N + v];
  }
  const double* __restrict__ tb = A.table + (int64_t)A.phase[v] * kTableStride;
  if (tb[0] != 0.0) return;
  double dLp[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll
  for (int al = 0; al < 12; ++al)
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j)
        dLp[3 * i + j] += dg[al] * tb[kTabS + 3 * al + i] * tb[kTabM + 3 * al + j];
  double dd = 0.0;
#pragma unroll
  for (int i = 0; i < 9; ++i) dd += dLp[i] * dLp[i];
  A.pcyc[v] += sqrt(2.0 / 3.0 * dd);
  A.pcyc_lit[v] += dd / A.dt;
  double Fe[9];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j)
      Fe[3 * i + j] = F[3 * i] * Fpi[j] + F[3 * i + 1] * Fpi[3 + j] +
                      F[3 * i + 2] * Fpi[6 + j];
  double C[9];
#pragma unroll
  for (int p = 0; p < 3; ++p)
#pragma unroll
    for (int q = 0; q < 3; ++q)
      C[3 * p + q] = Fe[p] * Fe[q] + Fe[3 + p] * Fe[3 + q] + Fe[6 + p] * Fe[6 + q];
  const double E[6] = {0.5 * (C[0] - 1.0), 0.5 * (C[4] - 1.0),
                       0.5 * (C[8] - 1.0), 0.5 * C[5],
                       0.5 * C[2],         0.5 * C[1]};
  const double w[6] = {1, 1, 1, 2, 2, 2};
  double S[6];
#pragma unroll
  for (int I = 0; I < 6; ++I) {
    double acc = 0.0;
#pragma unroll
    for (int J = 0; J < 6; ++J) acc += tb[kTabC + 6 * I + J] * w[J] * E[J];
    S[I] = acc;
  }
#pragma unroll
  for (int al = 0; al < 12; ++al) {
    const double* s = tb + kTabS + 3 * al;
    const double* m = tb + kTabM + 3 * al;
    const double Sm0 = S[0] * m[0] + S[5] * m[1] + S[4] * m[2];
    const double Sm1 = S[5] * m[0] + S[1] * m[1] + S[3] * m[2];
    const double Sm2 = S[4] * m[0] + S[3] * m[1] + S[2] * m[2];
    A.wcyc[al * N + v] += (s[0] * Sm0 + s[1] * Sm1 + s[2] * Sm2) * dg[al];
  }
}

void launch_commit_batch(const CommitBatchArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(commit_batch_kernel, dim3((unsigned)((a.N + kBlock - 1) / kBlock)),
                     dim3(kBlock), 0, s, a);
}

template void launch_cg_init_batch<float>(const SegItem*, int, int, int64_t,
                                          const double*, float*, float*,
                                          hipStream_t);
template void launch_cg_init_batch<double>(const SegItem*, int, int, int64_t,
                                           const double*, double*, double*,
                                           hipStream_t);
template void launch_cg_update_batch<float>(const SegItem*, int, int, int64_t,
                                            float*, float*, const float*,
                                            const float*, hipStream_t);
template void launch_cg_update_batch<double>(const SegItem*, int, int, int64_t,
                                             double*, double*, const double*,
                                             const double*, hipStream_t);

}  // namespace rve
