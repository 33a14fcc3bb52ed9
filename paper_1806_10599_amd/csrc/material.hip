// Point constitutive update (Sec. 2.1, Eq. 2) and material tangent
// K = dP/dF (Eq. 13) in FP64: the return mapping runs four lanes per voxel
// (three slip systems per lane), the tangent one lane per voxel.
//
// Grains: FCC crystal plasticity with the power-law flow rule of Sec. 3.2,
// Eq. 22 (constant critical stress g, rate exponent n) and an
// Armstrong-Frederick back stress, integrated by backward Euler over dt at
// the committed state (Fp^-1_0, chi_0):
//   Fp^-1 = Fp^-1_0 (I - sum_a dg_a s_a (x) m_a),  Fe = F Fp^-1,
//   S = C : (Fe^T Fe - I)/2,  tau_a = s_a . S m_a,
//   chi_a = (chi_0a + c dg_a)/(1 + d |dg_a|),  x_a = (tau_a - chi_a)/g,
//   P = Fe S Fp^-T.
// The 12 slips solve R_a = asinh(dg_a/a) - asinh(|x_a|^n sign x_a) = 0
// (a = dt gdot0), which has the roots of dg_a = a |x_a|^n sign x_a but stays
// well scaled under large overstress.  Damped Newton with backtracking on
// |R|^2/2; a failed warm-started solve is retried from zero slips.  R is
// formed in FP64 with one logarithm per slip (flow_residual); the Jacobian,
// which only steers the iteration towards the root of R, in FP32.
//
// The 12x12 Jacobian is diag(D) + U W^T with rank-6 factors (the resolved
// stresses depend on the slips only through the symmetric elastic strain),
// so each Newton step and each tangent column costs one 6x6 solve
// (Sherman-Morrison-Woodbury) instead of a 12x12 one.
//
// Work order: crystal voxels first, then the particle voxels (an index list
// built with the microstructure), so that wavefronts iterating the local
// solve carry no particle lanes.
//
// Particles: isotropic St-Venant-Kirchhoff, P = F S, S = lam tr(E) I + 2 mu E.
#include "kernels.hpp"

#ifndef RVE_TAN_MINB32
#define RVE_TAN_MINB32 2
#endif

namespace rve {

namespace {

constexpr int LOCAL_MAXIT = 60;
constexpr double LOCAL_RTOL = 1e-10;
constexpr double LOCAL_ATOL = 1e-18;
constexpr double LOCAL_RFLOOR = 1e-10;

// Voigt order 11, 22, 33, 23, 13, 12
__device__ constexpr double VW[6] = {1, 1, 1, 2, 2, 2};

// Hides an offset of zero from the optimizer so that table entries are
// re-read (from cache) at each use instead of being hoisted out of the local
// Newton loop into registers, which would exhaust the register file.  The
// pointer itself stays visible, so the loads remain global-memory loads
// (not flat ones).  The asm is empty: no instruction is emitted and no
// memory is accessed.
__device__ __forceinline__ const double* opaque(const double* p) {
  int64_t z = 0;
  asm volatile("" : "+v"(z));
  return p + z;
}

__device__ __forceinline__ double sgn(double x) {
  return (x > 0.0) ? 1.0 : ((x < 0.0) ? -1.0 : 0.0);
}

// asinh(|x|^n sign x) and its derivative d/dx = n y / (|x| sqrt(1 + y^2)),
// y = |x|^n.  For the integer exponents of the flow rule y is formed by
// repeated squaring and asinh(y) = log1p(y + y (y / (1 + sqrt(1 + y^2))))
// (an exact identity that needs no logarithm of |x| and no exponential);
// past |x| = 1e7 (y^2 would leave the FP64 range) and for other exponents
// the form through s = min(y, 1/y) = exp(-|n ln|x||) is used:
//   y >= 1: asinh(y) = n ln|x| + log1p(q),                q = sqrt(1 + s^2)
//   y <  1: asinh(y) = log1p(s + s^2 / (1 + q)).
__device__ __forceinline__ double ipow_n(double b, int ni) {
  if (ni == 20) {   // the workloads' exponent: five products
    const double b2 = b * b, b4 = b2 * b2, b8 = b4 * b4, b16 = b8 * b8;
    return b16 * b4;
  }
  double y = 1.0;
  for (int e = ni; e; e >>= 1) {   // uniform over the wavefront
    if (e & 1) y *= b;
    b *= b;
  }
  return y;
}

__device__ __forceinline__ void asinh_pow(double x, double n, int ni,
                                          double& val, double& der) {
  const double ax = fabs(x);
  if (ni > 0 && ax < 1e7) {
    const double y = ipow_n(ax, ni);
    const double q = sqrt(fma(y, y, 1.0));
    val = copysign(log1p(y + y * (y / (1.0 + q))), x);
    der = (ax > 0.0) ? n * (y / (ax * q)) : 0.0;
    return;
  }
  const double e = n * log(ax);          // ln y (-inf at x = 0)
  const bool big = e > 0.0;
  const double s = exp(-fabs(e));        // 0 at x = 0
  const double q = sqrt(1.0 + s * s);
  const double L = log1p(big ? q : s + s * s / (1.0 + q));
  val = sgn(x) * ((big ? e : 0.0) + L);
  der = (ax > 0.0) ? n * (big ? 1.0 : s) / (ax * q) : 0.0;
}

// The local residual R = asinh(u) - asinh(|x|^n sign x), u = dg / a, with
// one logarithm: asinh(u) = su ln A, A = |u| + sqrt(1 + u^2), and
// asinh(|x|^n sign x) = sx ln B, B = y + sqrt(1 + y^2), y = |x|^n, so
// R = s ln(A / B) when the signs agree (or one is zero; s the nonzero one)
// and R = su ln(A B) when they differ -- exact identities.  Near the root
// A / B is close to one and ln(A / B) carries an absolute error of a few
// units of 1e-16 (the two-logarithm difference carries that much relative
// to ln A).  The derivative of asinh(|x|^n sign x) (Jacobian only) is
// returned in single precision.  Past |x| = 1e7 and for non-integer n the
// two functions are evaluated apart (asinh_pow, asinh_bf).
__device__ __forceinline__ double asinh_bf(double u);
__device__ __forceinline__ void flow_residual(double t, double inv_a, double x,
                                              double n, int ni, double& R,
                                              float& der) {
  const double ax = fabs(x);
  if (ni > 0 && ax < 1e7) {
    const double y = ipow_n(ax, ni);
    const double B = y + sqrt(fma(y, y, 1.0));
    const double au = fabs(t * inv_a);
    const double A = au + sqrt(fma(au, au, 1.0));
    const double su = (t > 0.0) ? 1.0 : ((t < 0.0) ? -1.0 : 0.0);
    const double sx = (x > 0.0) ? 1.0 : ((x < 0.0) ? -1.0 : 0.0);
    const bool differ = su * sx < 0.0;
    const double s = (su != 0.0) ? su : sx;
    R = s * log(differ ? A * B : A / B);
    const float yf = (float)y;
    const float r = (y >= 1e18) ? 1.0f : yf * rsqrtf(fmaf(yf, yf, 1.0f));
    der = (ax > 1e-30) ? (float)n * r * __builtin_amdgcn_rcpf((float)ax) : 0.0f;
    return;
  }
  double val, d;
  asinh_pow(x, n, ni, val, d);
  R = asinh_bf(t * inv_a) - val;
  der = (float)d;
}

// asinh(u) in one branch-free form, exact for every u:
// asinh(|u|) = log1p(|u| + u^2 / (1 + sqrt(1 + u^2))), with the quotient
// written as |u| (|u| / (1 + q)) so that it cannot overflow.
__device__ __forceinline__ double asinh_bf(double u) {
  const double au = fabs(u);
  const double q = sqrt(1.0 + au * au);
  return copysign(log1p(au + au * (au / (1.0 + q))), u);
}

__device__ __forceinline__ void mm3(const double* A, const double* B,
                                    double* C) {
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j)
      C[3 * i + j] = A[3 * i] * B[j] + A[3 * i + 1] * B[3 + j] +
                     A[3 * i + 2] * B[6 + j];
}

// S (Voigt) = C : E (Voigt), C_IJ from the table
__device__ __forceinline__ void cmul6(const double* __restrict__ Cv,
                                      const double* E, double* S) {
  double We[6];
#pragma unroll
  for (int J = 0; J < 6; ++J) We[J] = VW[J] * E[J];
#pragma unroll
  for (int I = 0; I < 6; ++I) {
    double acc = 0.0;
#pragma unroll
    for (int J = 0; J < 6; ++J) acc += Cv[6 * I + J] * We[J];
    S[I] = acc;
  }
}

struct CpEval {
  double Fe[9];
  double S[6];
  double chi[12];
  double h[12];   // d asinh(|x|^n sign x) / dx, x = (tau - chi)/g
};

// d/dx asinh(|x|^n sign x) = n y / (|x| sqrt(1 + y^2)), y = |x|^n (FP64;
// the same branches as asinh_pow, without the function value)
__device__ __forceinline__ double flow_slope(double x, double n, int ni) {
  const double ax = fabs(x);
  if (ni > 0 && ax < 1e7) {
    const double y = ipow_n(ax, ni);
    return (ax > 0.0) ? n * (y / (ax * sqrt(fma(y, y, 1.0)))) : 0.0;
  }
  double val, der;
  asinh_pow(x, n, ni, val, der);
  return der;
}

// State at the converged slips dg for the tangent (elastic deformation,
// stress, back stresses, flow slopes).  Fes = F Fp^-1_0.
__device__ __forceinline__ void cp_eval(const double* Fes,
                                        const double* chi0, const double* dg,
                                        const double* __restrict__ tb,
                                        const LawParams& lp, double a,
                                        CpEval& e) {
  tb = opaque(tb);
#pragma unroll
  for (int i = 0; i < 9; ++i) e.Fe[i] = Fes[i];
#pragma unroll
  for (int al = 0; al < 12; ++al) {
    const double s0 = tb[kTabS + 3 * al], s1 = tb[kTabS + 3 * al + 1],
                 s2 = tb[kTabS + 3 * al + 2];
    const double m0 = tb[kTabM + 3 * al], m1 = tb[kTabM + 3 * al + 1],
                 m2 = tb[kTabM + 3 * al + 2];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const double u = dg[al] * (Fes[3 * i] * s0 + Fes[3 * i + 1] * s1 +
                                 Fes[3 * i + 2] * s2);
      e.Fe[3 * i] -= u * m0;
      e.Fe[3 * i + 1] -= u * m1;
      e.Fe[3 * i + 2] -= u * m2;
    }
  }
  double C[9];
#pragma unroll
  for (int p = 0; p < 3; ++p)
#pragma unroll
    for (int q = 0; q < 3; ++q)
      C[3 * p + q] = e.Fe[p] * e.Fe[q] + e.Fe[3 + p] * e.Fe[3 + q] +
                     e.Fe[6 + p] * e.Fe[6 + q];
  const double E[6] = {0.5 * (C[0] - 1.0), 0.5 * (C[4] - 1.0),
                       0.5 * (C[8] - 1.0), 0.5 * C[5],
                       0.5 * C[2],         0.5 * C[1]};
  cmul6(tb + kTabC, E, e.S);
  const double* S = e.S;
#pragma unroll
  for (int al = 0; al < 12; ++al) {
    const double s0 = tb[kTabS + 3 * al], s1 = tb[kTabS + 3 * al + 1],
                 s2 = tb[kTabS + 3 * al + 2];
    const double m0 = tb[kTabM + 3 * al], m1 = tb[kTabM + 3 * al + 1],
                 m2 = tb[kTabM + 3 * al + 2];
    const double Sm0 = S[0] * m0 + S[5] * m1 + S[4] * m2;
    const double Sm1 = S[5] * m0 + S[1] * m1 + S[3] * m2;
    const double Sm2 = S[4] * m0 + S[3] * m1 + S[2] * m2;
    const double tau = s0 * Sm0 + s1 * Sm1 + s2 * Sm2;
    const double chi = (chi0[al] + lp.c_af * dg[al]) / (1.0 + lp.d_af * fabs(dg[al]));
    const double x = (tau - chi) * lp.inv_g;
    e.chi[al] = chi;
    e.h[al] = flow_slope(x, lp.nexp, lp.nint);
  }
}

// Q = Fe^T Fes
__device__ __forceinline__ void make_Q(const double* Fe, const double* Fes,
                                       double* Q) {
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j)
      Q[3 * i + j] = Fe[i] * Fes[j] + Fe[3 + i] * Fes[3 + j] +
                     Fe[6 + i] * Fes[6 + j];
}

// V_a = sym((Q s_a) (x) m_a) in Voigt order, in the precision T of Q
template <typename T>
__device__ __forceinline__ void make_V(const T* Q, const double* __restrict__ tb,
                                       int al, T* V) {
  const T s0 = (T)tb[kTabS + 3 * al], s1 = (T)tb[kTabS + 3 * al + 1],
          s2 = (T)tb[kTabS + 3 * al + 2];
  const T m[3] = {(T)tb[kTabM + 3 * al], (T)tb[kTabM + 3 * al + 1],
                  (T)tb[kTabM + 3 * al + 2]};
  T qs[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) qs[i] = Q[3 * i] * s0 + Q[3 * i + 1] * s1 + Q[3 * i + 2] * s2;
  V[0] = qs[0] * m[0];
  V[1] = qs[1] * m[1];
  V[2] = qs[2] * m[2];
  V[3] = T(0.5) * (qs[1] * m[2] + qs[2] * m[1]);
  V[4] = T(0.5) * (qs[0] * m[2] + qs[2] * m[0]);
  V[5] = T(0.5) * (qs[0] * m[1] + qs[1] * m[0]);
}

// Gaussian elimination of the 6x6 capacitance matrix with partial pivoting
// by compare-and-swap; the swap decisions are kept for later right-hand sides.
template <typename T>
struct LU6T {
  T M[36];
  T ip[6];   // reciprocals of the pivots
  uint32_t swaps;
};
using LU6 = LU6T<double>;

template <typename T>
__device__ __forceinline__ void lu6_factor(LU6T<T>& L) {
  uint32_t sw = 0;
  int bit = 0;
#pragma unroll
  for (int k = 0; k < 6; ++k) {
#pragma unroll
    for (int r = k + 1; r < 6; ++r) {
      const bool s = fabs(L.M[6 * r + k]) > fabs(L.M[6 * k + k]);
      if (s) {
        // columns < k hold the multipliers of earlier steps; they stay with
        // the step that made them (the solve applies swap k, then step k)
#pragma unroll
        for (int j = k; j < 6; ++j) {
          const T t = L.M[6 * k + j];
          L.M[6 * k + j] = L.M[6 * r + j];
          L.M[6 * r + j] = t;
        }
      }
      sw |= (s ? 1u : 0u) << bit;
      ++bit;
    }
    const T inv = T(1) / L.M[6 * k + k];
    L.ip[k] = inv;
#pragma unroll
    for (int r = k + 1; r < 6; ++r) {
      const T f = L.M[6 * r + k] * inv;
      L.M[6 * r + k] = f;
#pragma unroll
      for (int j = k + 1; j < 6; ++j) L.M[6 * r + j] -= f * L.M[6 * k + j];
    }
  }
  L.swaps = sw;
}

template <typename T>
__device__ __forceinline__ void lu6_solve(const LU6T<T>& L, T* z) {
  int bit = 0;
#pragma unroll
  for (int k = 0; k < 6; ++k) {
#pragma unroll
    for (int r = k + 1; r < 6; ++r) {
      if ((L.swaps >> bit) & 1u) {
        const T t = z[k];
        z[k] = z[r];
        z[r] = t;
      }
      ++bit;
    }
#pragma unroll
    for (int r = k + 1; r < 6; ++r) z[r] -= L.M[6 * r + k] * z[k];
  }
#pragma unroll
  for (int k = 5; k >= 0; --k) {
    T acc = z[k];
#pragma unroll
    for (int j = k + 1; j < 6; ++j) acc -= L.M[6 * k + j] * z[j];
    z[k] = acc * L.ip[k];
  }
}

// Diagonal D, factor h and the factored capacitance matrix at the slips dg,
// in the precision T (the state e comes from an FP64 evaluation).
template <typename T>
__device__ __forceinline__ void cp_jacobian(const CpEval& e, const double* Fes,
                                            const double* dg,
                                            const double* __restrict__ tb,
                                            const LawParams& lp, double a,
                                            T* D, T* hg, T* Q, LU6T<T>& L) {
  tb = opaque(tb);
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j)
      Q[3 * i + j] = (T)(e.Fe[i] * Fes[j] + e.Fe[3 + i] * Fes[3 + j] +
                         e.Fe[6 + i] * Fes[6 + j]);
#pragma unroll
  for (int i = 0; i < 36; ++i) L.M[i] = (i % 7 == 0) ? T(1) : T(0);
#pragma unroll
  for (int al = 0; al < 12; ++al) {
    const double ad = fabs(dg[al]);
    const double dchi = (lp.c_af - lp.d_af * sgn(dg[al]) * e.chi[al]) / (1.0 + lp.d_af * ad);
    const double hgd = e.h[al] * lp.inv_g;
    hg[al] = (T)hgd;
    // D holds the reciprocal of the diagonal of the local Jacobian
    D[al] = (T)(1.0 / (1.0 / sqrt(a * a + dg[al] * dg[al]) + hgd * dchi));
    T V[6];
    make_V(Q, tb, al, V);
    const T f = hg[al] * D[al];
    // row factor of the rank-one term, formed once per slip
    T w[6];
#pragma unroll
    for (int J = 0; J < 6; ++J) w[J] = f * (T)(VW[J] * tb[kTabN + 6 * al + J]);
#pragma unroll
    for (int I = 0; I < 6; ++I)
#pragma unroll
      for (int J = 0; J < 6; ++J) L.M[6 * I + J] += V[I] * w[J];
  }
  lu6_factor(L);
}

// out = J^-1 rhs with J = diag(D) + U W^T, U_a = hg_a w N_a, W_a = V_a
// (iD = 1/D from cp_jacobian)
template <typename T>
__device__ __forceinline__ void cp_jsolve(const T* rhs, const T* iD,
                                          const T* hg, const T* Q,
                                          const double* __restrict__ tb,
                                          const LU6T<T>& L, T* out) {
  tb = opaque(tb);
  T z[6] = {0, 0, 0, 0, 0, 0};
#pragma unroll
  for (int al = 0; al < 12; ++al) {
    out[al] = rhs[al] * iD[al];
    T V[6];
    make_V(Q, tb, al, V);
#pragma unroll
    for (int I = 0; I < 6; ++I) z[I] += V[I] * out[al];
  }
  lu6_solve(L, z);
#pragma unroll
  for (int al = 0; al < 12; ++al) {
    T u = 0;
#pragma unroll
    for (int J = 0; J < 6; ++J) u += (T)(VW[J] * tb[kTabN + 6 * al + J]) * z[J];
    out[al] -= hg[al] * u * iD[al];
  }
}

// C = A B (3x3, row-major) and S = C : E (Voigt, C_IJ from the table) in T
template <typename T>
__device__ __forceinline__ void mm3t(const T* A, const T* B, T* C) {
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j)
      C[3 * i + j] = A[3 * i] * B[j] + A[3 * i + 1] * B[3 + j] +
                     A[3 * i + 2] * B[6 + j];
}
template <typename T>
__device__ __forceinline__ void cmul6t(const double* __restrict__ Cv,
                                       const T* E, T* S) {
#pragma unroll
  for (int I = 0; I < 6; ++I) {
    T acc = 0;
#pragma unroll
    for (int J = 0; J < 6; ++J) acc += (T)(Cv[6 * I + J] * VW[J]) * E[J];
    S[I] = acc;
  }
}

__device__ __forceinline__ void load9(const double* __restrict__ p, int64_t v,
                                      int64_t N, double* o) {
#pragma unroll
  for (int c = 0; c < 9; ++c) o[c] = p[c * N + v];
}

// ---- return mapping with several lanes per voxel ----------------------------
// LPV consecutive lanes (2 or 4, inside one quad) share a voxel; lane h of
// the group owns the slips kOwn*h .. kOwn*h + kOwn - 1 (kOwn = 12 / LPV).
// Sums over slips are formed per lane and completed across the group in a
// butterfly (x + other at each level: the same value on every lane, since
// floating-point addition commutes), so all lanes of a voxel take every
// decision on identical numbers and run the same iterations.  Splitting the
// per-slip state removes the register spills of the one-lane kernel.

// the value of lane (this ^ X) within the quad, X in {1, 2}
template <int X>
__device__ __forceinline__ double quad_xor(double x) {
  constexpr int ctrl = (X == 1) ? 0xB1 : 0x4E;  // quad_perm 1,0,3,2 / 2,3,0,1
  const unsigned long long u = (unsigned long long)__double_as_longlong(x);
  const int lo = __builtin_amdgcn_mov_dpp((int)(unsigned)(u & 0xffffffffull),
                                          ctrl, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_mov_dpp((int)(unsigned)(u >> 32), ctrl, 0xF,
                                          0xF, false);
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) |
                                          (unsigned long long)(unsigned)lo));
}
template <int LPV>
__device__ __forceinline__ double grp_sum(double x) {
  x = x + quad_xor<1>(x);
  if constexpr (LPV == 4) x = x + quad_xor<2>(x);
  return x;
}
template <int LPV>
__device__ __forceinline__ double grp_max(double x) {
  x = fmax(x, quad_xor<1>(x));
  if constexpr (LPV == 4) x = fmax(x, quad_xor<2>(x));
  return x;
}

// R, h of the own slips at t = dg + lam*step and Q = Fe^T Fes
template <int LPV, int kOwn = 12 / LPV>
__device__ __forceinline__ void pr_eval(const double* Fes,
                                        const double* __restrict__ chi0p,
                                        int64_t N, int h, const double* dg,
                                        const double* step, double lam,
                                        const double* __restrict__ tb0,
                                        const LawParams& lp, double a,
                                        double* R, float* hd, float* Q) {
  double dFe[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) dFe[i] = 0.0;
#pragma unroll
  for (int j = 0; j < kOwn; ++j) {
    const double* __restrict__ tb = opaque(tb0) + 3 * (kOwn * h + j);
    const double t = dg[j] + lam * step[j];
    const double s0 = tb[kTabS], s1 = tb[kTabS + 1], s2 = tb[kTabS + 2];
    const double m0 = tb[kTabM], m1 = tb[kTabM + 1], m2 = tb[kTabM + 2];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const double u = t * (Fes[3 * i] * s0 + Fes[3 * i + 1] * s1 +
                            Fes[3 * i + 2] * s2);
      dFe[3 * i] += u * m0;
      dFe[3 * i + 1] += u * m1;
      dFe[3 * i + 2] += u * m2;
    }
  }
  double Fe[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) Fe[i] = Fes[i] - grp_sum<LPV>(dFe[i]);
  double S[6];
  {
    double C[9];
#pragma unroll
    for (int p = 0; p < 3; ++p)
#pragma unroll
      for (int q = 0; q < 3; ++q)
        C[3 * p + q] = Fe[p] * Fe[q] + Fe[3 + p] * Fe[3 + q] + Fe[6 + p] * Fe[6 + q];
    const double E[6] = {0.5 * (C[0] - 1.0), 0.5 * (C[4] - 1.0),
                         0.5 * (C[8] - 1.0), 0.5 * C[5],
                         0.5 * C[2],         0.5 * C[1]};
    cmul6(opaque(tb0) + kTabC, E, S);
  }
#pragma unroll
  for (int j = 0; j < kOwn; ++j) {
    const double* __restrict__ tb = opaque(tb0) + 3 * (kOwn * h + j);
    const double t = dg[j] + lam * step[j];
    const double s0 = tb[kTabS], s1 = tb[kTabS + 1], s2 = tb[kTabS + 2];
    const double m0 = tb[kTabM], m1 = tb[kTabM + 1], m2 = tb[kTabM + 2];
    const double Sm0 = S[0] * m0 + S[5] * m1 + S[4] * m2;
    const double Sm1 = S[5] * m0 + S[1] * m1 + S[3] * m2;
    const double Sm2 = S[4] * m0 + S[3] * m1 + S[2] * m2;
    const double tau = s0 * Sm0 + s1 * Sm1 + s2 * Sm2;
    const double chi0 = opaque(chi0p)[(kOwn * h + j) * N];
    const double chi = (chi0 + lp.c_af * t) / (1.0 + lp.d_af * fabs(t));
    const double x = (tau - chi) * lp.inv_g;
    float der;
    flow_residual(t, lp.inv_a, x, lp.nexp, lp.nint, R[j], der);
    hd[j] = der;
  }
  // Q = Fe^T Fes for the Jacobian, which only steers the Newton iteration
  // (its root is that of R, formed in FP64): single precision
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j)
      Q[3 * i + j] = (float)(Fe[i] * Fes[j] + Fe[3 + i] * Fes[3 + j] +
                             Fe[6 + i] * Fes[6 + j]);
}

// V_a = sym((Q s_a) (x) m_a) in Voigt order, single precision
__device__ __forceinline__ void make_Vf(const float* Q,
                                        const double* __restrict__ tb, int al,
                                        float* V) {
  const float s0 = (float)tb[kTabS + 3 * al], s1 = (float)tb[kTabS + 3 * al + 1],
              s2 = (float)tb[kTabS + 3 * al + 2];
  const float m0 = (float)tb[kTabM + 3 * al], m1 = (float)tb[kTabM + 3 * al + 1],
              m2 = (float)tb[kTabM + 3 * al + 2];
  float qs[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) qs[i] = Q[3 * i] * s0 + Q[3 * i + 1] * s1 + Q[3 * i + 2] * s2;
  V[0] = qs[0] * m0;
  V[1] = qs[1] * m1;
  V[2] = qs[2] * m2;
  V[3] = 0.5f * (qs[1] * m2 + qs[2] * m1);
  V[4] = 0.5f * (qs[0] * m2 + qs[2] * m0);
  V[5] = 0.5f * (qs[0] * m1 + qs[1] * m0);
}

template <int LPV>
__device__ __forceinline__ float grp_sumf(float x) {
  x = x + __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(
              __builtin_bit_cast(int, x), 0xB1, 0xF, 0xF, false));
  if constexpr (LPV == 4)
    x = x + __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(
                __builtin_bit_cast(int, x), 0x4E, 0xF, 0xF, false));
  return x;
}

// Newton step of the own slips: step = -J^-1 R, J = diag(D) + U W^T.  The
// Jacobian only steers the iteration (the root is that of the FP64
// residual R), so it is formed and solved in single precision: the step
// is then exact to single-precision rounding, which leaves the local
// Newton iteration converging as before to the FP64 root.
template <int LPV, int kOwn = 12 / LPV>
__device__ __forceinline__ void pr_step(const double* dg, const double* R,
                                        const float* hd, const float* Q,
                                        const double* __restrict__ chi0p,
                                        int64_t N, int h,
                                        const double* __restrict__ tb0,
                                        const LawParams& lp, double a,
                                        double* step) {
  LU6T<float> L;
#pragma unroll
  for (int i = 0; i < 36; ++i) L.M[i] = 0.0f;
  float D[kOwn];
  const float inv_g = (float)lp.inv_g, c_af = (float)lp.c_af,
              d_af = (float)lp.d_af, a2 = (float)(a * a);
#pragma unroll
  for (int j = 0; j < kOwn; ++j) {
    const int al = kOwn * h + j;
    const double* __restrict__ tb = opaque(tb0);
    const float chi0 = (float)opaque(chi0p)[al * N];
    const float dgf = (float)dg[j];
    const float den = 1.0f / (1.0f + d_af * fabsf(dgf));
    const float chi = (chi0 + c_af * dgf) * den;
    const float sg = (dgf > 0.0f) ? 1.0f : ((dgf < 0.0f) ? -1.0f : 0.0f);
    const float dchi = (c_af - d_af * sg * chi) * den;
    // D holds the reciprocal of the diagonal of the local Jacobian
    D[j] = 1.0f / (rsqrtf(a2 + dgf * dgf) + hd[j] * inv_g * dchi);
    float V[6];
    make_Vf(Q, tb, al, V);
    const float f = hd[j] * inv_g * D[j];
    // row factor of the rank-one term, formed once per slip
    float w[6];
#pragma unroll
    for (int J = 0; J < 6; ++J) w[J] = f * (float)(VW[J] * tb[kTabN + 6 * al + J]);
#pragma unroll
    for (int I = 0; I < 6; ++I)
#pragma unroll
      for (int J = 0; J < 6; ++J) L.M[6 * I + J] += V[I] * w[J];
    step[j] = -R[j] * (double)D[j];
  }
#pragma unroll
  for (int i = 0; i < 36; ++i) L.M[i] = ((i % 7 == 0) ? 1.0f : 0.0f) + grp_sumf<LPV>(L.M[i]);
  lu6_factor(L);
  float z[6] = {0, 0, 0, 0, 0, 0};
#pragma unroll
  for (int j = 0; j < kOwn; ++j) {
    float V[6];
    make_Vf(Q, opaque(tb0), kOwn * h + j, V);
    const float sj = (float)step[j];
#pragma unroll
    for (int I = 0; I < 6; ++I) z[I] += V[I] * sj;
  }
#pragma unroll
  for (int I = 0; I < 6; ++I) z[I] = grp_sumf<LPV>(z[I]);
  lu6_solve(L, z);
#pragma unroll
  for (int j = 0; j < kOwn; ++j) {
    const double* __restrict__ tb = opaque(tb0) + kTabN + 6 * (kOwn * h + j);
    float u = 0.0f;
#pragma unroll
    for (int J = 0; J < 6; ++J) u += (float)(VW[J] * tb[J]) * z[J];
    step[j] -= (double)(hd[j] * inv_g * u * D[j]);
  }
}

template <int kOwn>
__device__ __forceinline__ double own_half_sq(const double* R) {
  double m = 0.0;
#pragma unroll
  for (int j = 0; j < kOwn; ++j) m += R[j] * R[j];
  return 0.5 * m;
}

// damped Newton with Armijo backtracking on |R|^2/2 over the group (the
// iteration of the one-lane formulation); dg holds the own slips
template <int LPV, int kOwn = 12 / LPV>
__device__ __forceinline__ bool pr_local_solve(const double* Fes,
                                               const double* __restrict__ chi0p,
                                               int64_t N, int h, double* dg,
                                               const double* __restrict__ tb,
                                               const LawParams& lp, double a,
                                               int& iters, int& evals) {
  double R[kOwn], step[kOwn];
  float hd[kOwn], Q[9];
#pragma unroll
  for (int j = 0; j < kOwn; ++j) step[j] = 0.0;
  pr_eval<LPV>(Fes, chi0p, N, h, dg, step, 0.0, tb, lp, a, R, hd, Q);
  ++evals;
  for (int it = 0; it < LOCAL_MAXIT; ++it) {
    ++iters;
    pr_step<LPV>(dg, R, hd, Q, chi0p, N, h, tb, lp, a, step);
    double smax = 0.0, dmax = 0.0, rmax = 0.0, bad = 0.0;
#pragma unroll
    for (int j = 0; j < kOwn; ++j) {
      smax = fmax(smax, fabs(step[j]));
      dmax = fmax(dmax, fabs(dg[j] + step[j]));
      rmax = fmax(rmax, fabs(R[j]));
      bad = isfinite(step[j]) ? bad : 1.0;
    }
    smax = grp_max<LPV>(smax);
    dmax = grp_max<LPV>(dmax);
    rmax = grp_max<LPV>(rmax);
    bad = grp_max<LPV>(bad);
    if (bad == 0.0 && smax <= LOCAL_ATOL + LOCAL_RTOL * dmax) {
#pragma unroll
      for (int j = 0; j < kOwn; ++j) dg[j] += step[j];
      return true;
    }
    const double merit0 = grp_sum<LPV>(own_half_sq<kOwn>(R));
    double lam = 1.0, lam_used = 1.0;
    bool accepted = false;
    for (int ls = 0; ls < 40; ++ls) {
      pr_eval<LPV>(Fes, chi0p, N, h, dg, step, lam, tb, lp, a, R, hd, Q);
      ++evals;
      lam_used = lam;
      const double mt = grp_sum<LPV>(own_half_sq<kOwn>(R));
      if (isfinite(mt) && mt <= (1.0 - 1e-4 * lam) * merit0) {
        accepted = true;
        break;
      }
      lam *= 0.5;
    }
    double nf = 0.0;
#pragma unroll
    for (int j = 0; j < kOwn; ++j) {
      dg[j] = dg[j] + lam_used * step[j];
      nf = isfinite(dg[j]) ? nf : 1.0;
    }
    if (grp_max<LPV>(nf) != 0.0) return false;
    if (!accepted && rmax <= LOCAL_RFLOOR) return true;
  }
  return false;
}

}  // namespace

// LPV lanes per voxel (see pr_eval); 256 threads per block
template <int LPV, int MINB>
__global__ __launch_bounds__(256, MINB) void return_map_group_kernel(ConstArgs A) {
  constexpr int kOwn = 12 / LPV;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t g = t / LPV;
  const int h = (int)(t % LPV);
  if (g >= A.N) return;  // all lanes of a voxel leave together
  const int64_t v = A.order ? (int64_t)A.order[g] : g;
  if (A.vrve && A.scs[A.vrve[v]].inactive) return;
  const int64_t N = A.N;
  const double* __restrict__ tb = A.table + (int64_t)A.phase[v] * kTableStride;
  double F[9];
  load9(A.F, v, N, F);
  if (tb[0] != 0.0) {  // isotropic SVK particle
    const double lam = tb[kTabLam], mu = tb[kTabMu];
    double C[9];
#pragma unroll
    for (int p = 0; p < 3; ++p)
#pragma unroll
      for (int q = 0; q < 3; ++q)
        C[3 * p + q] = F[p] * F[q] + F[3 + p] * F[3 + q] + F[6 + p] * F[6 + q];
    const double tr = 0.5 * (C[0] + C[4] + C[8] - 3.0);
    double S[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) S[i] = mu * (C[i] - ((i % 4 == 0) ? 1.0 : 0.0));
    S[0] += lam * tr;
    S[4] += lam * tr;
    S[8] += lam * tr;
    double P[9];
    mm3(F, S, P);
#pragma unroll
    for (int c = 0; c < 9; ++c)
      if (c % LPV == h) {
        A.P[c * N + v] = P[c];
        A.Fpi[c * N + v] = A.Fpi0[c * N + v];
      }
#pragma unroll
    for (int j = 0; j < kOwn; ++j) {
      const int al = kOwn * h + j;
      A.chi[al * N + v] = A.chi0[al * N + v];
      A.dg[al * N + v] = 0.0;
    }
    if (A.iters && h == 0) {
      A.iters[v] = -1;  // particle voxel
      A.evals[v] = 0;
    }
    return;
  }
  double dg[kOwn];
  double warm = 0.0;
#pragma unroll
  for (int j = 0; j < kOwn; ++j) {
    dg[j] = A.dg0 ? A.dg0[(kOwn * h + j) * N + v] : 0.0;
    warm = (dg[j] != 0.0) ? 1.0 : warm;
  }
  warm = grp_max<LPV>(warm);
  double Fes[9];
  {
    double Fpi0[9];
    load9(A.Fpi0, v, N, Fpi0);
    mm3(F, Fpi0, Fes);
  }
  const double a = A.lp.dt * A.lp.gdot0;
  const double* chi0p = A.chi0 + v;
  int iters = 0, evals = 0;
  bool ok = false;
  for (int attempt = 0; attempt < 2 && !ok; ++attempt) {
    if (attempt == 1) {
      if (warm == 0.0) break;
#pragma unroll
      for (int j = 0; j < kOwn; ++j) dg[j] = 0.0;  // retry from zero slips
    }
    ok = pr_local_solve<LPV>(Fes, chi0p, N, h, dg, tb, A.lp, a, iters, evals);
  }
  if (!ok && h == 0) atomicAdd(A.vrve ? &A.scs[A.vrve[v]].fails : A.fails, 1);
  // final state: Fp^-1 = Fp^-1_0 (I - sum dg s (x) m), Fe = F Fp^-1,
  // S = C : Ee, P = Fe S Fp^-T
  double Fpi0[9];
  load9(opaque(A.Fpi0), v, N, Fpi0);
  double dFpi[9], dFe[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) dFpi[i] = dFe[i] = 0.0;
#pragma unroll
  for (int j = 0; j < kOwn; ++j) {
    const double* __restrict__ tj = opaque(tb) + 3 * (kOwn * h + j);
    const double s0 = tj[kTabS], s1 = tj[kTabS + 1], s2 = tj[kTabS + 2];
    const double m0 = tj[kTabM], m1 = tj[kTabM + 1], m2 = tj[kTabM + 2];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const double u = dg[j] * (Fpi0[3 * i] * s0 + Fpi0[3 * i + 1] * s1 +
                                Fpi0[3 * i + 2] * s2);
      dFpi[3 * i] += u * m0;
      dFpi[3 * i + 1] += u * m1;
      dFpi[3 * i + 2] += u * m2;
      const double w = dg[j] * (Fes[3 * i] * s0 + Fes[3 * i + 1] * s1 +
                                Fes[3 * i + 2] * s2);
      dFe[3 * i] += w * m0;
      dFe[3 * i + 1] += w * m1;
      dFe[3 * i + 2] += w * m2;
    }
  }
  double Fpi[9], Fe[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    Fpi[i] = Fpi0[i] - grp_sum<LPV>(dFpi[i]);
    Fe[i] = Fes[i] - grp_sum<LPV>(dFe[i]);
  }
  double S[6];
  {
    double C[9];
#pragma unroll
    for (int p = 0; p < 3; ++p)
#pragma unroll
      for (int q = 0; q < 3; ++q)
        C[3 * p + q] = Fe[p] * Fe[q] + Fe[3 + p] * Fe[3 + q] + Fe[6 + p] * Fe[6 + q];
    const double E[6] = {0.5 * (C[0] - 1.0), 0.5 * (C[4] - 1.0),
                         0.5 * (C[8] - 1.0), 0.5 * C[5],
                         0.5 * C[2],         0.5 * C[1]};
    cmul6(opaque(tb) + kTabC, E, S);
  }
  const double Sf[9] = {S[0], S[5], S[4], S[5], S[1], S[3], S[4], S[3], S[2]};
  double FeS[9];
  mm3(Fe, Sf, FeS);
#pragma unroll
  for (int c = 0; c < 9; ++c) {
    if (c % LPV != h) continue;
    const int i = c / 3, j = c - 3 * (c / 3);
    const double P = FeS[3 * i] * Fpi[3 * j] + FeS[3 * i + 1] * Fpi[3 * j + 1] +
                     FeS[3 * i + 2] * Fpi[3 * j + 2];
    A.P[c * N + v] = P;
    A.Fpi[c * N + v] = Fpi[c];
  }
#pragma unroll
  for (int j = 0; j < kOwn; ++j) {
    const int al = kOwn * h + j;
    const double chi0 = A.chi0[al * N + v];
    A.chi[al * N + v] = (chi0 + A.lp.c_af * dg[j]) / (1.0 + A.lp.d_af * fabs(dg[j]));
    A.dg[al * N + v] = dg[j];
  }
  if (A.iters && h == 0) {
    A.iters[v] = iters;
    A.evals[v] = evals;
  }
}

// Work counts of the last return mapping: stats[0] += local Newton steps,
// [1] += residual evaluations, [2] += crystal voxels, [3] += particle voxels
__global__ __launch_bounds__(256) void rm_count_kernel(
    const int32_t* __restrict__ iters, const int32_t* __restrict__ evals,
    int64_t N, unsigned long long* __restrict__ stats) {
  __shared__ unsigned long long red[4][256];
  unsigned long long c[4] = {0, 0, 0, 0};
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < N;
       v += (int64_t)gridDim.x * blockDim.x) {
    const int it = iters[v];
    if (it < 0) {
      c[3] += 1;
    } else {
      c[0] += (unsigned long long)it;
      c[1] += (unsigned long long)evals[v];
      c[2] += 1;
    }
  }
  for (int k = 0; k < 4; ++k) red[k][threadIdx.x] = c[k];
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w)
      for (int k = 0; k < 4; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x < 4) atomicAdd(&stats[threadIdx.x], red[threadIdx.x][0]);
}

// FP32 linear algebra (mixed mode): two waves per SIMD with 448 B of scratch
// per lane beat one wave without (0.336 against 0.382 ms at 64^3)
template <typename TK>
__global__ __launch_bounds__(128, sizeof(TK) == 4 ? RVE_TAN_MINB32 : 1) void
tangent_kernel(TangentArgs<TK> A) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= A.N) return;
  const int64_t v = A.order ? (int64_t)A.order[i] : i;
  if (A.vrve && A.scs[A.vrve[v]].inactive) return;
  const int64_t N = A.N;
  const double* __restrict__ tb = A.table + (int64_t)A.phase[v] * kTableStride;
  double F[9];
  load9(A.F, v, N, F);
  if (tb[0] != 0.0) {
    // K_ijkl = d_ik S_lj + lam F_ij F_kl + mu F_il F_kj + mu (F F^T)_ik d_jl
    const double lam = tb[kTabLam], mu = tb[kTabMu];
    double C[9], B[9];
#pragma unroll
    for (int p = 0; p < 3; ++p)
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        C[3 * p + q] = F[p] * F[q] + F[3 + p] * F[3 + q] + F[6 + p] * F[6 + q];
        B[3 * p + q] = F[3 * p] * F[3 * q] + F[3 * p + 1] * F[3 * q + 1] +
                       F[3 * p + 2] * F[3 * q + 2];
      }
    const double tr = 0.5 * (C[0] + C[4] + C[8] - 3.0);
    double S[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) S[i] = mu * (C[i] - ((i % 4 == 0) ? 1.0 : 0.0));
    S[0] += lam * tr;
    S[4] += lam * tr;
    S[8] += lam * tr;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j)
#pragma unroll
        for (int k = 0; k < 3; ++k)
#pragma unroll
          for (int l = 0; l < 3; ++l) {
            double K = lam * F[3 * i + j] * F[3 * k + l] + mu * F[3 * i + l] * F[3 * k + j];
            if (i == k) K += S[3 * l + j];
            if (j == l) K += mu * B[3 * i + k];
            A.K[(int64_t)(9 * (3 * i + j) + 3 * k + l) * N + v] = TK(K);
          }
    return;
  }
  // the state at the converged slips in FP64; the linear algebra of the
  // tangent (6x6 factorisation, nine Woodbury solves) and its assembly in
  // the precision of K (FP32 for the single-precision CG of mixed mode)
  using TC = TK;
  double Fpi0[9], chi0[12], dg[12];
  load9(A.Fpi0, v, N, Fpi0);
#pragma unroll
  for (int al = 0; al < 12; ++al) {
    chi0[al] = A.chi0[al * N + v];
    dg[al] = A.dg[al * N + v];
  }
  double Fes[9];
  mm3(F, Fpi0, Fes);
  const double a = A.lp.dt * A.lp.gdot0;
  CpEval e;
  cp_eval(Fes, chi0, dg, tb, A.lp, a, e);
  TC D[12], hg[12], Q[9];
  LU6T<TC> L;
  cp_jacobian(e, Fes, dg, tb, A.lp, a, D, hg, Q, L);
  TC Fpi[9], Fe[9], Fpi0c[9], Fesc[9];
  {
    double Fpid[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) Fpid[i] = Fpi0[i];
#pragma unroll
    for (int al = 0; al < 12; ++al) {
      const double s0 = tb[kTabS + 3 * al], s1 = tb[kTabS + 3 * al + 1],
                   s2 = tb[kTabS + 3 * al + 2];
      const double m0 = tb[kTabM + 3 * al], m1 = tb[kTabM + 3 * al + 1],
                   m2 = tb[kTabM + 3 * al + 2];
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        const double u = dg[al] * (Fpi0[3 * i] * s0 + Fpi0[3 * i + 1] * s1 +
                                   Fpi0[3 * i + 2] * s2);
        Fpid[3 * i] -= u * m0;
        Fpid[3 * i + 1] -= u * m1;
        Fpid[3 * i + 2] -= u * m2;
      }
    }
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      Fpi[i] = (TC)Fpid[i];
      Fe[i] = (TC)e.Fe[i];
      Fpi0c[i] = (TC)Fpi0[i];
      Fesc[i] = (TC)Fes[i];
    }
  }
  const TC Sf[9] = {(TC)e.S[0], (TC)e.S[5], (TC)e.S[4], (TC)e.S[5], (TC)e.S[1],
                    (TC)e.S[3], (TC)e.S[4], (TC)e.S[3], (TC)e.S[2]};
  TC PS[9], FeS[9], B[9];
  mm3t(Fpi, Sf, PS);   // Fp^-1 S
  mm3t(Fe, Sf, FeS);   // Fe S
#pragma unroll
  for (int l = 0; l < 3; ++l)
#pragma unroll
    for (int j = 0; j < 3; ++j)
      B[3 * l + j] = PS[3 * l] * Fpi[3 * j] + PS[3 * l + 1] * Fpi[3 * j + 1] +
                     PS[3 * l + 2] * Fpi[3 * j + 2];  // Fp^-1 S Fp^-T
  const double* Cv = tb + kTabC;
#pragma unroll 1
  for (int kl = 0; kl < 9; ++kl) {
    const int k = kl / 3, l = kl - 3 * (kl / 3);
    // rows k of Fe and l of Fp^-1, B row l: selects keep them in registers
    TC fk[3], pl[3], Bl[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      fk[c] = (k == 0) ? Fe[c] : ((k == 1) ? Fe[3 + c] : Fe[6 + c]);
      pl[c] = (l == 0) ? Fpi[c] : ((l == 1) ? Fpi[3 + c] : Fpi[6 + c]);
      Bl[c] = (l == 0) ? B[c] : ((l == 1) ? B[3 + c] : B[6 + c]);
    }
    // dR/dF_kl: b_a = (h_a/g) fk . N_a pl  (dtau_a/dF = Fe N_a Fp^-T)
    TC b[12], gcol[12];
#pragma unroll
    for (int al = 0; al < 12; ++al) {
      const double* Na = tb + kTabN + 6 * al;
      const TC N0 = (TC)Na[0], N1 = (TC)Na[1], N2 = (TC)Na[2], N3 = (TC)Na[3],
               N4 = (TC)Na[4], N5 = (TC)Na[5];
      const TC Np0 = N0 * pl[0] + N5 * pl[1] + N4 * pl[2];
      const TC Np1 = N5 * pl[0] + N1 * pl[1] + N3 * pl[2];
      const TC Np2 = N4 * pl[0] + N3 * pl[1] + N2 * pl[2];
      b[al] = hg[al] * (fk[0] * Np0 + fk[1] * Np1 + fk[2] * Np2);
    }
    cp_jsolve(b, D, hg, Q, tb, L, gcol);  // d dg / d F_kl
    // sigma = C : sym(fk (x) pl) - C : sum_a g_a V_a
    TC E[6], acc6[6] = {0, 0, 0, 0, 0, 0}, acc9[9];
    E[0] = fk[0] * pl[0];
    E[1] = fk[1] * pl[1];
    E[2] = fk[2] * pl[2];
    E[3] = TC(0.5) * (fk[1] * pl[2] + fk[2] * pl[1]);
    E[4] = TC(0.5) * (fk[0] * pl[2] + fk[2] * pl[0]);
    E[5] = TC(0.5) * (fk[0] * pl[1] + fk[1] * pl[0]);
#pragma unroll
    for (int i = 0; i < 9; ++i) acc9[i] = 0;
#pragma unroll
    for (int al = 0; al < 12; ++al) {
      TC V[6];
      make_V(Q, tb, al, V);
#pragma unroll
      for (int I = 0; I < 6; ++I) acc6[I] += gcol[al] * V[I];
      const TC s[3] = {(TC)tb[kTabS + 3 * al], (TC)tb[kTabS + 3 * al + 1],
                       (TC)tb[kTabS + 3 * al + 2]};
      const TC m[3] = {(TC)tb[kTabM + 3 * al], (TC)tb[kTabM + 3 * al + 1],
                       (TC)tb[kTabM + 3 * al + 2]};
      TC u[3], vv[3], w[3], y[3];
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        u[i] = Fesc[3 * i] * s[0] + Fesc[3 * i + 1] * s[1] + Fesc[3 * i + 2] * s[2];
        vv[i] = PS[3 * i] * m[0] + PS[3 * i + 1] * m[1] + PS[3 * i + 2] * m[2];
        w[i] = FeS[3 * i] * m[0] + FeS[3 * i + 1] * m[1] + FeS[3 * i + 2] * m[2];
        y[i] = Fpi0c[3 * i] * s[0] + Fpi0c[3 * i + 1] * s[1] + Fpi0c[3 * i + 2] * s[2];
      }
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j)
          acc9[3 * i + j] += gcol[al] * (u[i] * vv[j] + w[i] * y[j]);
    }
#pragma unroll
    for (int I = 0; I < 6; ++I) E[I] -= acc6[I];
    TC sg[6];
    cmul6t(Cv, E, sg);
    const TC sf[9] = {sg[0], sg[5], sg[4], sg[5], sg[1],
                      sg[3], sg[4], sg[3], sg[2]};
    TC Fs[9];
    mm3t(Fe, sf, Fs);
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        TC K = Fs[3 * i] * Fpi[3 * j] + Fs[3 * i + 1] * Fpi[3 * j + 1] +
               Fs[3 * i + 2] * Fpi[3 * j + 2] - acc9[3 * i + j];
        if (i == k) K += Bl[j];
        A.K[(int64_t)(9 * (3 * i + j) + kl) * N + v] = TK(K);
      }
  }
}

// four lanes per voxel at two waves per SIMD: the fastest of the measured
// shapes (2 or 4 lanes, 1 or 2 waves per SIMD) at 64^3
void launch_return_map(const ConstArgs& a, hipStream_t s) {
  constexpr int kLanes = 4, kBlk = 256;
  const int64_t grid = (kLanes * a.N + kBlk - 1) / kBlk;
  launch(return_map_group_kernel<kLanes, 2>, dim3((unsigned)grid), dim3(kBlk),
         0, s, a);
}

void launch_rm_count(const int32_t* iters, const int32_t* evals, int64_t N,
                     unsigned long long* stats, hipStream_t s) {
  hipLaunchKernelGGL(rm_count_kernel, dim3(512), dim3(256), 0, s, iters, evals,
                     N, stats);
}

template <typename TK>
void launch_tangent(const TangentArgs<TK>& a, hipStream_t s) {
  const int blk = 128;
  const int64_t grid = (a.N + blk - 1) / blk;
  launch((tangent_kernel<TK>), dim3((unsigned)grid), dim3(blk), 0,
                     s, a);
}

template void launch_tangent<float>(const TangentArgs<float>&, hipStream_t);
template void launch_tangent<double>(const TangentArgs<double>&, hipStream_t);

}  // namespace rve
