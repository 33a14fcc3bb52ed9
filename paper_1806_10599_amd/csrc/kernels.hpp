// Launch interfaces of the HIP kernels (host side sees only these).
#pragma once

#include "common.hpp"

namespace rve {

enum { SRC_FIELD = 0, SRC_KP = 1 };
// pass C outputs: the field (||out||^2 partials), the field and p . out
// partials (batched CG), r -= alpha out in place (single-RVE CG)
enum { DST_NORM = 0, DST_DOT = 1, DST_CG = 2 };

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
  int64_t cs;          // component stride of the real fields (N^3, or the
                       // voxel count of a batch arena)
  // optional (CG run): block 0 reduces these p.(K:p) partials and publishes
  // alpha in slot `parity` of scw (cg_alpha_publish)
  const double* pkp = nullptr;
  int pkp_count = 0;
  int parity = 0;
  Scalars* scw = nullptr;
  // SRC_KP in a single-RVE CG run (the direction kernel folded into pass A):
  // the r.r partials of the last inverse pass (beta), the iterate x (the
  // previous iteration's x += alpha p_old on this block's components) and
  // the per-block partials of p . (K:p) written for pass B's alpha
  const double* pinv = nullptr;
  int pinv_count = 0;
  T* x = nullptr;
  double* pkp_out = nullptr;
};

// The direction step a pass-A block applies with SRC_KP: p = r (first) or
// r + beta p_old, and with upd the pending x += alpha p_old
template <typename T>
struct KpStep {
  bool first;
  T beta;
  bool upd;
  T alpha;
};

template <typename T>
struct PencilArgs {
  cplx<T>* spec;
  const cplx<T>* tw;
  const T* vt;         // [3][N] wave-vector components per axis
  T invN3;
  const Scalars* sc;   // optional early exit
  // optional (fused single-RVE CG run): block 0 reduces pass A's p.(K:p)
  // partials and publishes alpha in slot `parity` of scw
  const double* pkp = nullptr;
  int pkp_count = 0;
  int parity = 0;
  Scalars* scw = nullptr;
};

template <typename T, typename TO>
struct SlabInvArgs {
  const cplx<T>* spec;
  const cplx<T>* tw;
  TO* out;             // [9][N^3]
  const T* pdot;       // DST_DOT: direction for p . Ap
  double* partial;     // per block
  const Scalars* sc;   // optional early exit
  int64_t cs;          // component stride of out / pdot
  // DST_CG: r -= alpha G(y) in place with alpha = sc->alphas[parity]; the
  // partials are those of the new r . r (out is not written)
  T* rio = nullptr;
  int parity = 0;
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
  // CG run (dst = DST_CG): the p.(K:p) partials for alpha (published by
  // pass A with src = SRC_FIELD, by pass B with src = SRC_KP, whose pass A
  // writes them), the residual updated in place by pass C, and the
  // iteration's parity
  const double* pkp = nullptr;
  int pkp_count = 0;
  T* r_io = nullptr;
  int parity = 0;
  // fused CG run (src = SRC_KP): the r.r partials of the last pass C and the
  // iterate x, as the direction kernel takes them
  const double* pinv = nullptr;
  int pinv_count = 0;
  T* x = nullptr;
  int passes = 7;   // bit 0: pass A, bit 1: pass B, bit 2: pass C
  int cpb = 0;      // components per slab block in passes A and C (1 or 3;
                    // 0: the default of the grid edge and precision)
  int tt = 0;       // kz columns per pass-B block (4, 8 or 16; 0: default)
};

template <typename T>
void launch_G(int n, const SpectralLaunch<T>& L, hipStream_t s);
// G in FP64 with the static scratch array of noalloc.hip (no allocation)
void noalloc_apply_G(int n, const double L[3], int projection, const double* in,
                     double* out, hipStream_t s);
// block counts of the slab (A, C) and pencil (B) grids; 0 = default schedule
int slab_blocks(int n, bool fp64, int cpb = 0);
int pencil_blocks(int n, bool fp64, int tt = 0);
// whether a (cpb, tt) schedule exists for the grid edge and precision
bool schedule_valid(int n, bool fp64, int cpb, int tt);

// One RVE of a batch: where its voxels, spectrum and scalars live and where
// its blocks start in the pass-A/C (blk[0]) and pass-B (blk[1]) grids.
template <typename T>
struct SpecItem {
  int n;
  int blk[2];
  int cpb;              // components per slab block (1 or 3)
  int tt;               // kz columns per pencil block (4, 8 or 16)
  int pad;
  int64_t off;          // voxel offset in the arena
  int64_t soff;         // complex offset of the spectrum
  const cplx<T>* tw;
  const T* vt;
  Scalars* sc;          // this RVE's scalars
  double* partial;      // pass-C partials (slab_blocks entries)
  double* psum;         // residual pass sums [9][n]
  double* psq;
};

template <typename T>
struct BatchSpec {
  const SpecItem<T>* items;
  int nitems;
  int cpbs = 3;         // slab schedules among the items (bit 0: cpb 1,
                        // bit 1: cpb 3)
  int64_t cs;           // voxels in the arena (component stride)
  const T* field;       // SRC_FIELD input
  const T* K;
  const T* r;
  const T* p_old;
  T* p_new;
  cplx<T>* spec;
};

// passes of a batch: src SRC_FIELD (residual: out_d, norms) or SRC_KP (CG:
// out_T = Ap, p.Ap partials); block counts of the three grids
template <typename T>
void launch_G_batch(const BatchSpec<T>& b, int src, T* out_T, double* out_d,
                    int blocksA, int blocksB, size_t ldsA, size_t ldsB,
                    hipStream_t s);
// dynamic LDS of the batched slab and pencil passes of one grid edge
// under a schedule (throws for an invalid one)
template <typename T>
void batch_lds(int n, int cpb, int tt, size_t& slab, size_t& pencil);
void default_schedule(int n, bool fp64, int& cpb, int& tt);


bool batch_supported(int n);
template <typename T>
void batch_allow_lds(size_t slab, size_t pencil);

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
  double inv_g, inv_a;   // 1/g and 1/(dt gdot0), formed once on the host
  int32_t nint;          // nexp when it is an integer in [1, 64], else 0
};

// the flow-rule exponent as an integer when it is one (powers by products)
inline int32_t flow_exponent_int(double n) {
  const int32_t ni = (int32_t)n;
  return ((double)ni == n && ni >= 1 && ni <= 64) ? ni : 0;
}

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
  int32_t* iters;        // optional per-voxel local Newton steps (-1: particle)
  int32_t* evals;        // with iters: per-voxel residual evaluations
  LawParams lp;
  int64_t N;
  const uint8_t* vrve;   // batch: RVE of each voxel (null for one RVE)
  Scalars* scs;          // batch: per-RVE flags (skip when inactive) and
                         // per-RVE failure counts (fails unused)
  const int32_t* order;  // optional voxel of each work item: crystal voxels
                         // first, then the particle voxels (null: identity)
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
  const uint8_t* vrve;
  const Scalars* scs;
  const int32_t* order;  // optional work order (as ConstArgs::order)
};

void launch_return_map(const ConstArgs& a, hipStream_t s);
// Appendix A bridge: F [9][N], sigma [6][N], ddsdde [36][N] -> P [9][N]
// (Eq. A.1), K [81][N] (Eq. A.16); fused, P only, K only (in T)
void launch_umat_bridge(const double* F, const double* sigma,
                        const double* ddsdde, int64_t N, double* P, double* K,
                        hipStream_t s);
void launch_umat_piola(const double* F, const double* sigma, int64_t N,
                       double* P, hipStream_t s);
template <typename T>
void launch_umat_tangent(const double* F, const double* sigma,
                         const double* ddsdde, int64_t N, T* K, hipStream_t s);
// example user material (compressible neo-Hookean) in the same form
void launch_neo_hooke_umat(const double* F1, const double* F0,
                           const double* sv0, double* sv1, int nsv,
                           double* sigma, double* ddsdde, int32_t* fails,
                           int64_t N, hipStream_t s);
void launch_rm_count(const int32_t* iters, const int32_t* evals, int64_t N,
                     unsigned long long* stats, hipStream_t s);
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
// partial: r.r partials of the last inverse pass (a CG run; the kernel also
// applies the previous iteration's x += alpha p_old when x != null); null:
// first, beta and alpha from the scalars.  pkp: per-block p . (K : p), one
// entry per block of the grid (kp_blocks).
template <typename T>
void launch_kp(const T* K, const T* r, const T* p_old, T* p_new, T* y,
               Scalars* sc, int64_t N, hipStream_t s,
               const double* partial = nullptr, int count = 0, int parity = 0,
               T* x = nullptr, double* pkp = nullptr);
int kp_blocks(int64_t N);  // one voxel per thread
// the CG decision after the last update of a chunk; parity: that of the
// iteration that would follow; pub (coherent pinned host memory, or null):
// where the kernel also copies the scalars for the host
void launch_cg_close(const double* partial, int count, Scalars* sc,
                     int parity, hipStream_t s, Scalars* pub = nullptr);
template <typename T>
void launch_add_to_F(double* F, const T* x, int64_t n9, hipStream_t s);
template <typename T>
void launch_convert(const double* in, T* out, int64_t n, hipStream_t s);

enum { RED_INIT = 0, RED_ALPHA = 1, RED_BETA = 2, RED_RESID = 3 };
// pub: as for launch_cg_close (RED_RESID only)
void launch_reduce(int op, const double* partial, int count,
                   const double* psum, const double* psq, int nslab_sums,
                   double invN3, Scalars* sc, double* pbar, hipStream_t s,
                   Scalars* pub = nullptr);
void launch_commit(const CommitArgs& a, hipStream_t s);
void launch_fill_i32(int32_t* p, int32_t v, int64_t n, hipStream_t s);
void launch_fill_f64(double* p, double v, int64_t n, hipStream_t s);
void launch_cauchy(const double* F, const double* P, double* sig, int64_t N,
                   hipStream_t s);
void launch_init_scalars(Scalars* sc, int max_iters, double eta, hipStream_t s);
void launch_bench_scalars(Scalars* sc, hipStream_t s);

constexpr int kRedBlocks = 1024;  // grid of the elementwise reductions

// ---------------------------------------------------------- batch helpers
// Elementwise batch kernels give each RVE its own run of blocks so that
// every block's partial sum belongs to one RVE.
struct SegItem {
  int64_t off;      // voxel offset in the arena
  int64_t n9;       // 9 * voxels of this RVE
  int blk0;         // first block of this RVE
  int nblk;
  double* partial;  // per-block partials of this RVE (nblk entries)
  Scalars* sc;
};
struct RedItem {
  const double* partial;
  int count;
  const double* psum;
  const double* psq;
  int nss;
  double invN3;
};
// CG of a whole batch in one launch of resident blocks (grid barriers between
// passes); even / odd: the pass arguments of even and odd iterations (p_old
// and p_new swapped)
template <typename T>
struct BatchCG {
  BatchSpec<T> even, odd;
  const SegItem* seg;
  int seg_blocks;
  const RedItem* red_inv;   // p.Ap partials of the inverse pass
  const RedItem* red_seg;   // r.r partials of the update
  Scalars* scs;
  int nitems;
  int blocksA, blocksB;
  int64_t cs;
  T* x;
  T* r;
  T* Ap;
  int max_iters;            // iterations of this launch at most
  unsigned* bar;            // barrier state (kBatchBarWords words, zero at
                            // start but for the generation)
  int* err;                 // set when a barrier waited past its bound
};
constexpr int kBatchBarWords = 32 * 10;
template <typename T>
void launch_cg_batch_persistent(const BatchCG<T>& c, int grid, size_t lds,
                                hipStream_t s);
// blocks of the persistent CG kernel that are resident at once
template <typename T>
int cg_batch_persistent_grid(size_t lds);
template <typename T>
void launch_cg_init_batch(const SegItem* items, int nitems, int blocks,
                          int64_t cs, const double* r64, T* r, T* x,
                          hipStream_t s);
template <typename T>
void launch_cg_update_batch(const SegItem* items, int nitems, int blocks,
                            int64_t cs, T* x, T* r, const T* p, const T* Ap,
                            hipStream_t s);
void launch_reduce_batch(int op, const RedItem* items, int nitems,
                         Scalars* scs, hipStream_t s);
void launch_predict_batch(double* F, const double* Fprev, const uint8_t* vrve,
                          const double* dF /*[B][9]*/, int64_t N,
                          hipStream_t s);
struct CommitBatchArgs {
  const uint8_t* vrve;
  const Scalars* scs;
  const double* dF;   // [B][9] macro increments
  const double* F;    // Newton iterate (converged)
  const double* P;
  const double* Fpi_t;
  const double* chi_t;
  const double* dg_t;
  double* Fprev;
  double* Pc;
  double* Fpi_c;
  double* chi_c;
  double* dg_c;
  double* dFt;
  const int32_t* phase;
  const double* table;
  double* pcyc;
  double* pcyc_lit;
  double* wcyc;
  double dt;
  int64_t N;
};
void launch_commit_batch(const CommitBatchArgs& a, hipStream_t s);

// Device-side Newton control of a batch (Sec. 2.1): per RVE the record of
// its increment, written by the control kernel after each FP64 residual
constexpr int kBatchLog = 64;
struct BatchLog {
  int32_t status;        // 1 running, else RVE_OK / RVE_ENOTCONV / RVE_ELOCAL
  int32_t newton_iters;
  int32_t cg_total;
  int32_t breakdowns;
  int32_t fails;
  int32_t pad;
  double rel;            // last relative residual ||G(P)|| / ||P||
  double predictor_rel;
  double pbar[9];
  double res_hist[kBatchLog];
  int32_t cg_hist[kBatchLog];
};
struct NewtonCtl {
  double newton_tol, cg_tol;
  int32_t newton_max, cg_max, forcing;
};
// after the residual of Newton iteration it: book the previous solve's CG
// count, take the decision (commit, local failure, out of budget) and give
// running RVEs their linear-solve tolerance
void launch_newton_control_batch(Scalars* scs, BatchLog* log, int nitems,
                                 int it, const NewtonCtl& ctl, hipStream_t s);

}  // namespace rve
