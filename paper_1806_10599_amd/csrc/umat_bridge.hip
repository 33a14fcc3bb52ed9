// User materials in the form of a commercial FE code's finite-strain user
// subroutine (Appendix A): the material returns the Cauchy stress sigma and
// the tangent C of the Jaumann rate of the Kirchhoff stress (6x6 in the
// order 11, 22, 33, 12, 13, 23 with engineering shears, Eq. A.2); the FFT
// solver needs P = J sigma F^-T (Eq. A.1) and K = dP/dF (Eq. A.16).  One
// FP64 thread per voxel, structure-of-arrays; output planes are written
// with non-temporal stores (they are not read again by these kernels; about
// 4 % faster than plain stores on the fused bridge).
//
// Also here: the example user material (a compressible neo-Hookean solid in
// that form) that the user-material interface ships with.
#include "kernels.hpp"

namespace rve {

namespace {

// position of the pair (i, j) in the 6-component order 11, 22, 33, 12, 13, 23
__device__ __forceinline__ int vpair(int i, int j) {
  if (i == j) return i;
  return 2 + i + j;  // (0,1) -> 3, (0,2) -> 4, (1,2) -> 5
}

template <typename T>
__device__ __forceinline__ void st_nt(T* p, double x) {
  __builtin_nontemporal_store((T)x, p);
}

// one voxel: P (Eq. A.1) if WP, K (Eq. A.16) if WK
template <typename T, bool WP, bool WK>
__device__ __forceinline__ void bridge_voxel(int64_t v, int64_t N,
                                             const double* __restrict__ Fg,
                                             const double* __restrict__ sg,
                                             const double* __restrict__ Dg,
                                             double* __restrict__ Pg,
                                             T* __restrict__ Kg) {
  double F[9], s6[6];
#pragma unroll
  for (int c = 0; c < 9; ++c) F[c] = Fg[c * N + v];
#pragma unroll
  for (int c = 0; c < 6; ++c) s6[c] = sg[c * N + v];
  // J and F^-1 (adjugate / J)
  const double a00 = F[4] * F[8] - F[5] * F[7], a01 = F[2] * F[7] - F[1] * F[8],
               a02 = F[1] * F[5] - F[2] * F[4];
  const double a10 = F[5] * F[6] - F[3] * F[8], a11 = F[0] * F[8] - F[2] * F[6],
               a12 = F[2] * F[3] - F[0] * F[5];
  const double a20 = F[3] * F[7] - F[4] * F[6], a21 = F[1] * F[6] - F[0] * F[7],
               a22 = F[0] * F[4] - F[1] * F[3];
  const double J = F[0] * a00 + F[1] * a10 + F[2] * a20;
  const double iJ = 1.0 / J;
  const double Fi[9] = {a00 * iJ, a01 * iJ, a02 * iJ, a10 * iJ, a11 * iJ,
                        a12 * iJ, a20 * iJ, a21 * iJ, a22 * iJ};
  // tau = J sigma (symmetric)
  double tau[9];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) tau[3 * i + j] = J * s6[vpair(i, j)];
  // B_il = tau_ip F^-1_lp, which is also P_il
  double B[9];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      double acc = 0.0;
#pragma unroll
      for (int p = 0; p < 3; ++p) acc += tau[3 * i + p] * Fi[3 * j + p];
      B[3 * i + j] = acc;
      if (WP) st_nt(&Pg[(3 * i + j) * N + v], acc);
    }
  if (!WK) return;
  double D[36];
#pragma unroll
  for (int c = 0; c < 36; ++c) D[c] = Dg[c * N + v];
  // K_ijkl = sum_p dtau_ipkl F^-1_jp - B_il F^-1_jk with
  // dtau_ipkl = J C_ipkm F^-1_lm + 1/2 d_ik B_pl - 1/2 F^-1_li tau_kp
  //             + 1/2 d_pk B_il - 1/2 F^-1_lp tau_ik
#pragma unroll
  for (int kl = 0; kl < 9; ++kl) {
    const int k = kl / 3, l = kl - 3 * (kl / 3);
    double dt[9];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int p = 0; p < 3; ++p) {
        const int I = vpair(i, p);
        double acc = 0.0;
#pragma unroll
        for (int m = 0; m < 3; ++m) acc += D[6 * I + vpair(k, m)] * Fi[3 * l + m];
        double t = J * acc - 0.5 * Fi[3 * l + i] * tau[3 * k + p] -
                   0.5 * Fi[3 * l + p] * tau[3 * i + k];
        if (i == k) t += 0.5 * B[3 * p + l];
        if (p == k) t += 0.5 * B[3 * i + l];
        dt[3 * i + p] = t;
      }
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        double acc = -B[3 * i + l] * Fi[3 * j + k];
#pragma unroll
        for (int p = 0; p < 3; ++p) acc += dt[3 * i + p] * Fi[3 * j + p];
        st_nt(&Kg[(int64_t)(9 * (3 * i + j) + kl) * N + v], acc);
      }
  }
}

template <typename T, bool WP, bool WK>
__global__ __launch_bounds__(256) void umat_bridge_kernel(
    const double* __restrict__ F, const double* __restrict__ sigma,
    const double* __restrict__ D, int64_t N, double* __restrict__ P,
    T* __restrict__ K) {
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < N;
       v += (int64_t)gridDim.x * blockDim.x)
    bridge_voxel<T, WP, WK>(v, N, F, sigma, D, P, K);
}

// grid-stride launches: at most 8192 blocks (32 per CU); each thread then
// walks the voxels v, v + 8192*256, ...
dim3 stride_grid(int64_t N) {
  const int64_t g = (N + 255) / 256;
  return dim3((unsigned)(g < 8192 ? g : 8192));
}

// Example user material: compressible neo-Hookean solid.  State variables
// (component-major, nsv >= 3): mu, lambda, and the sum of |J - J_prev| over
// converged increments.  Kirchhoff stress tau = mu (B - I) + lambda ln J I;
// Jaumann tangent J C_ijkl = lambda d_ij d_kl + (mu - lambda ln J)
// (d_ik d_jl + d_il d_jk) + 1/2 (d_ik tau_jl + d_il tau_jk + tau_ik d_jl
// + tau_il d_jk).  A voxel with J <= 0 counts as a local failure.
__global__ __launch_bounds__(256) void neo_hooke_umat_kernel(
    const double* __restrict__ F1, const double* __restrict__ F0,
    const double* __restrict__ sv0, double* __restrict__ sv1, int nsv,
    double* __restrict__ sig, double* __restrict__ dds,
    int32_t* __restrict__ fails, int64_t N) {
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < N;
       v += (int64_t)gridDim.x * blockDim.x) {
    double F[9], G[9];
#pragma unroll
    for (int c = 0; c < 9; ++c) {
      F[c] = F1[c * N + v];
      G[c] = F0[c * N + v];
    }
    const double mu = sv0[v], lam = sv0[N + v];
    const double J = F[0] * (F[4] * F[8] - F[5] * F[7]) -
                     F[1] * (F[3] * F[8] - F[5] * F[6]) +
                     F[2] * (F[3] * F[7] - F[4] * F[6]);
    const double J0 = G[0] * (G[4] * G[8] - G[5] * G[7]) -
                      G[1] * (G[3] * G[8] - G[5] * G[6]) +
                      G[2] * (G[3] * G[7] - G[4] * G[6]);
    const bool ok = J > 0.0 && J < INFINITY;
    if (!ok) atomicAdd(fails, 1);
    const double Jc = ok ? J : 1.0;
    const double lnJ = log(Jc), iJ = 1.0 / Jc;
    double tau[9];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        double b = 0.0;
#pragma unroll
        for (int k = 0; k < 3; ++k) b += F[3 * i + k] * F[3 * j + k];
        tau[3 * i + j] = mu * (b - (i == j ? 1.0 : 0.0)) + (i == j ? lam * lnJ : 0.0);
      }
    const int pi[6] = {0, 1, 2, 0, 0, 1}, pj[6] = {0, 1, 2, 1, 2, 2};
#pragma unroll
    for (int a = 0; a < 6; ++a)
      sig[a * N + v] = ok ? tau[3 * pi[a] + pj[a]] * iJ : 0.0;
    const double m2 = mu - lam * lnJ;
#pragma unroll
    for (int a = 0; a < 6; ++a)
#pragma unroll
      for (int b = 0; b < 6; ++b) {
        const int i = pi[a], j = pj[a], k = pi[b], l = pj[b];
        const double dik = i == k, djl = j == l, dil = i == l, djk = j == k;
        double c = lam * (double)(i == j) * (double)(k == l) +
                   m2 * (dik * djl + dil * djk) +
                   0.5 * (dik * tau[3 * j + l] + dil * tau[3 * j + k] +
                          tau[3 * i + k] * djl + tau[3 * i + l] * djk);
        dds[(6 * a + b) * N + v] = c * iJ;
      }
    for (int c = 0; c < nsv; ++c) {
      double s = sv0[c * N + v];
      if (c == 2) s += fabs(J - J0);
      sv1[c * N + v] = s;
    }
  }
}

}  // namespace

void launch_umat_bridge(const double* F, const double* sigma,
                        const double* ddsdde, int64_t N, double* P, double* K,
                        hipStream_t s) {
  if (N <= 0) return;
  hipLaunchKernelGGL((umat_bridge_kernel<double, true, true>), stride_grid(N),
                     dim3(256), 0, s, F, sigma, ddsdde, N, P, K);
}

void launch_umat_piola(const double* F, const double* sigma, int64_t N,
                       double* P, hipStream_t s) {
  if (N <= 0) return;
  hipLaunchKernelGGL((umat_bridge_kernel<double, true, false>), stride_grid(N),
                     dim3(256), 0, s, F, sigma, (const double*)nullptr, N, P,
                     (double*)nullptr);
}

template <typename T>
void launch_umat_tangent(const double* F, const double* sigma,
                         const double* ddsdde, int64_t N, T* K, hipStream_t s) {
  if (N <= 0) return;
  hipLaunchKernelGGL((umat_bridge_kernel<T, false, true>), stride_grid(N),
                     dim3(256), 0, s, F, sigma, ddsdde, N, (double*)nullptr, K);
}
template void launch_umat_tangent<float>(const double*, const double*,
                                         const double*, int64_t, float*,
                                         hipStream_t);
template void launch_umat_tangent<double>(const double*, const double*,
                                          const double*, int64_t, double*,
                                          hipStream_t);

void launch_neo_hooke_umat(const double* F1, const double* F0,
                           const double* sv0, double* sv1, int nsv,
                           double* sigma, double* ddsdde, int32_t* fails,
                           int64_t N, hipStream_t s) {
  if (N <= 0) return;
  hipLaunchKernelGGL(neo_hooke_umat_kernel, stride_grid(N), dim3(256), 0, s,
                     F1, F0, sv0, sv1, nsv, sigma, ddsdde, fails, N);
}

}  // namespace rve
