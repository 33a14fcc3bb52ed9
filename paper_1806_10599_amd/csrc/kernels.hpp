// Launch interfaces of the HIP kernels (host side sees only these).
#pragma once

#include "common.hpp"

namespace rve {

enum { SRC_FIELD = 0, SRC_KP = 1 };
enum { DST_NORM = 0, DST_DOT = 1 };

template <typename T>
struct SlabFwdArgs {
  const T* field;      // SRC_FIELD: [9][N^3]
  const T* K;          // SRC_KP: [81][N^3]
  const T* r;          // SRC_KP: CG residual
  const T* p_old;      // SRC_KP: previous direction
  T* p_new;            // SRC_KP: new direction (written)
  cplx<T>* spec;       // [9][N][N][N/2]
  const cplx<T>* tw;   // exp(-2 pi i m / N)
  double* psum;        // optional [9][N] per-slab sums
  double* psq;         // optional [9][N] per-slab sums of squares
  const Scalars* sc;
};

template <typename T>
struct PencilArgs {
  cplx<T>* spec;
  const cplx<T>* tw;
  const T* vt;         // [3][N] wave-vector components per axis
  T invN3;
  const Scalars* sc;   // optional early exit
};

template <typename T, typename TO>
struct SlabInvArgs {
  const cplx<T>* spec;
  const cplx<T>* tw;
  TO* out;             // [9][N^3]
  const T* pdot;       // DST_DOT: direction for p . Ap
  double* partial;     // per block
  const Scalars* sc;   // optional early exit
};

template <typename T>
struct SpectralLaunch {
  int src = SRC_FIELD, dst = DST_NORM;
  const T* in_field = nullptr;
  const T* K = nullptr;
  const T* r = nullptr;
  const T* p_old = nullptr;
  T* p_new = nullptr;
  cplx<T>* spec = nullptr;
  const cplx<T>* tw = nullptr;
  const T* vt = nullptr;
  double* psum = nullptr;
  double* psq = nullptr;
  T* out_T = nullptr;
  double* out_d = nullptr;
  double* partial_inv = nullptr;
  Scalars* sc = nullptr;
  int passes = 7;   // bit 0: pass A, bit 1: pass B, bit 2: pass C
};

template <typename T>
void launch_G(int n, const SpectralLaunch<T>& L, hipStream_t s);
int slab_blocks(int n, bool fp64);

// ---------------------------------------------------------- constitutive
// Per-label table, kTableStride doubles per label:
//   [0] law (0 crystal, 1 isotropic SVK)
//   crystal: s[12][3] at kTabS, m[12][3] at kTabM, Nsym[12][6] at kTabN
//            (C : sym(S0) in Voigt order 11,22,33,23,13,12), Cv[6][6] at
//            kTabC (C_IJ in the same order), orientation R[3][3] at kTabR
//   SVK: lambda at kTabLam, mu at kTabMu
constexpr int kTableStride = 200;
constexpr int kTabS = 8, kTabM = 44, kTabN = 80, kTabC = 152, kTabR = 188;
constexpr int kTabLam = 8, kTabMu = 9;

struct LawParams {
  double gdot0, g, nexp, c_af, d_af, dt;
};

struct ConstArgs {
  const double* F;       // [9][N]
  const double* Fpi0;    // committed [9][N]
  const double* chi0;    // committed [12][N]
  const double* dg0;     // starting slips [12][N] or null (zeros)
  const int32_t* phase;  // [N]
  const double* table;   // [labels][kTableStride]
  double* P;             // [9][N]
  double* Fpi;           // trial [9][N]
  double* chi;           // trial [12][N]
  double* dg;            // trial [12][N]
  int32_t* fails;        // counter
  int32_t* iters;        // optional per-voxel local iterations
  LawParams lp;
  int64_t N;
};

template <typename TK>
struct TangentArgs {
  const double* F;
  const double* Fpi0;
  const double* chi0;
  const double* dg;      // converged trial slips
  const int32_t* phase;
  const double* table;
  TK* K;                 // [81][N]
  LawParams lp;
  int64_t N;
};

void launch_return_map(const ConstArgs& a, hipStream_t s);
template <typename TK>
void launch_tangent(const TangentArgs<TK>& a, hipStream_t s);

// ------------------------------------------------------------- solver ops
struct CommitArgs {
  const double* F;
  const double* Fpi_t;
  const double* dg_t;
  const int32_t* phase;
  const double* table;
  double* pcyc;
  double* pcyc_lit;
  double* wcyc;
  double dt;
  int64_t N;
};

void launch_predict(double* F, const double* Fprev, const double dFbar[9],
                    int64_t N, hipStream_t s);
template <typename T>
void launch_cg_init(const double* r64, T* r, T* x, double* partial, int nblk,
                    int64_t n9, hipStream_t s);
template <typename T>
void launch_cg_update(T* x, T* r, const T* p, const T* Ap, const Scalars* sc,
                      double* partial, int nblk, int64_t n9, hipStream_t s);
template <typename T>
void launch_add_to_F(double* F, const T* x, int64_t n9, hipStream_t s);
template <typename T>
void launch_convert(const double* in, T* out, int64_t n, hipStream_t s);

enum { RED_INIT = 0, RED_ALPHA = 1, RED_BETA = 2, RED_RESID = 3 };
void launch_reduce(int op, const double* partial, int count,
                   const double* psum, const double* psq, int nslab_sums,
                   double invN3, Scalars* sc, double* pbar, hipStream_t s);
void launch_commit(const CommitArgs& a, hipStream_t s);
void launch_fill_i32(int32_t* p, int32_t v, int64_t n, hipStream_t s);
void launch_fill_f64(double* p, double v, int64_t n, hipStream_t s);
void launch_cauchy(const double* F, const double* P, double* sig, int64_t N,
                   hipStream_t s);
void launch_init_scalars(Scalars* sc, int max_iters, double eta, hipStream_t s);
void launch_bench_scalars(Scalars* sc, hipStream_t s);

constexpr int kRedBlocks = 1024;  // grid of the elementwise reductions

}  // namespace rve
