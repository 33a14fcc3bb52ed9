// The RVE engine: device state of one periodic cell and the increment
// algorithm (Sec. 2.1 of Lucarini & Segurado): homogeneous predictor, Newton
// iterations with an FP64 equilibrium check, CG linear solves of
// G(K : dF) = -G(P), commit of the internal variables on convergence.
#pragma once

#include <memory>
#include <string>
#include <vector>

#include "../../include/rve.h"
#include "fips.hpp"
#include "kernels.hpp"
#include "ktimer.hpp"
#include "nn.hpp"

namespace rve {

class Engine {
 public:
  explicit Engine(const rve_config& cfg);
  ~Engine();

  void set_microstructure(const int32_t* phase, int32_t G, const double* quat,
                          const int32_t* law, const double* params,
                          int32_t nparams);
  // a user material in the Cauchy-stress / Jaumann-tangent form (Appendix A)
  // in place of the crystal-plasticity microstructure
  void set_user_material(rve_umat_fn fn, void* user, int32_t nstatev,
                         const double* statev0);
  int increment(const double Fbar_new[9], double dt, rve_increment_info* info);
  int increment_adaptive(const double Fbar_new[9], double dt, int max_cutbacks,
                         int grow_after, rve_adaptive_info* info);
  void reset_fips();
  void get_field(int field, void* dst, size_t bytes, bool on_device);
  size_t field_bytes(int field) const;
  void get_macro(double out[29]);
  void nonlocal_fips(double width, rve_nonlocal_fips* out, double* grain_pcyc,
                     double* grain_pcyc_lit, int32_t labels, double* band_wcyc,
                     int32_t* band_desc, int64_t band_cap);
  size_t state_size() const;
  void get_state(void* dst, size_t bytes);
  void set_state(const void* src, size_t bytes);
  void debug_apply_G(const double* in, double* out, int precision);
  void debug_constitutive(const double* F, double dt, double* P, double* K,
                          double* dg, int32_t* fails);
  void debug_set_field(int field, const double* src, size_t bytes);
  void bench_kernels(int reps, double* ms, int count);
  void set_timing(uint32_t mask);
  void set_timing_stride(int stride);
  void get_timing(double* ms, int64_t* launches, int count, bool reset,
                  int64_t* seen = nullptr);
  void get_rm_counts(int64_t out[4], bool reset);
  // FFT schedule of the CG matvec: (0, 0) = autotune at the next solve;
  // fused: the direction kernel folded into pass A
  void set_schedule(int cpb, int tt, int fused);
  void tune();
  void get_schedule(int out[3], double* ms) const {
    out[0] = sched_cpb_;
    out[1] = sched_tt_;
    out[2] = sched_fused_;
    if (ms) *ms = sched_ms_;
  }

  // pieces used by the learned warm start
  hipStream_t stream() const { return st_; }
  int n() const { return n_; }
  int64_t voxels() const { return N_; }
  double* dev_F() { return F_; }
  double* dev_Fprev() { return Fprev_; }
  const double* dF_last() const { return dFlast_; }
  void apply_G_fp64(const double* in, double* out);
  const rve_config& config() const { return cfg_; }
  // learned warm start
  void attach_net(Net* net);
  void features(const double Fbar_new[9], uint16_t* dst_dev);
  void target(float* dst_dev);

  std::string err;
  bool poisoned = false;

 private:
  void* alloc(size_t bytes);
  void release(void* p);
  void free_all();
  template <typename T>
  void cg_solve(int& iters, bool& breakdown, double eta);
  template <typename T>
  void cg_iteration(int parity);
  template <typename T, typename Run>
  void cg_iteration_steps(int parity, Run&& run);
  template <typename T>
  void capture_graph();
  template <typename T>
  void autotune();
  void read_scalars(Scalars& h);
  LawParams law_params(double dt) const;
  void residual_passes(const double* P, Scalars* pub = nullptr);
  int evaluate(const double* dg_start, double dt, double& rel,
               double& res, double& pn);
  void commit(double dt);
  template <typename T>
  void tangent(double dt);
  void feature_args(const double Fbar_new[9], FeatArgs& a, double& s_k);
  bool learned_candidate(const double Fbar_new[9]);
  bool extrapolated_candidate(const double Fbar_new[9]);
  void second_trial_set();
  void swap_trial_sets();
  void reset_macro_state();
  // copy of the committed state (device arrays and host macro state) for
  // the rollback of a failed adaptive step
  void take_snapshot();
  void restore_snapshot();
  void require_crystal(const char* what) const;

  rve_config cfg_;
  int n_;
  int64_t N_;
  bool fp64_;
  hipStream_t st_;
  std::vector<std::pair<void*, size_t>> allocs_;

  // committed state
  double *Fprev_, *Pc_, *Fpi_c_, *chi_c_, *dg_c_;
  double *pcyc_, *pcyc_lit_, *wcyc_;
  // Newton scratch
  double *F_, *P_, *Fpi_t_, *chi_t_, *dg_t_, *r64_;
  void* K_;      // [81][N] float (mixed) or double (fp64)
  // CG vectors (T) and spectra
  void *x_, *r_, *p0_, *p1_;
  void* Kp_;     // K : p of the current CG direction
  void* spec_;        // complex T
  void* spec64_;      // complex double (aliases spec_ in fp64 mode)
  double *partial_inv_, *partial_red_, *partial_kp_, *psum_, *psq_;
  Scalars* sc_;
  // coherent pinned: [0] sync reads, [1..2] chunks; sc_pub_: its device
  // address, where the closing and residual kernels write
  Scalars* sc_host_ = nullptr;
  Scalars* sc_pub_ = nullptr;
  hipEvent_t chunk_ev_[2] = {nullptr, nullptr};
  int32_t* phase_;
  int32_t* order_;                 // return-mapping work order (crystal first)
  std::vector<int32_t> order_host_;
  double* table_;
  void *tw32_, *tw64_, *vt32_, *vt64_;
  int nslab32_, nslab64_;
  int sched_cpb_ = 0, sched_tt_ = 0;   // 0: not tuned yet
  int sched_fused_ = 0;
  double sched_ms_ = 0.0;
  int labels_ = 0;
  bool have_micro_ = false;
  // host copies for the non-local indicators' band lists
  std::vector<int32_t> phase_host_;
  std::vector<double> table_host_;
  int G_ = 0;
  FipIndex fips_;
  double params_[RVE_NPARAMS];

  // macro state
  double Fbar_[9];
  double Pbar_[9];
  double Pbar_new_[9];
  double dFlast_[9];
  double t_ = 0.0;
  int64_t increments_ = 0;

  hipStream_t own_stream_ = nullptr;
  void* dbg32_ = nullptr;
  void* dbgspec32_ = nullptr;
  hipGraphExec_t graph_ = nullptr;
  hipGraph_t graph_def_ = nullptr;
  KernelTimer timer_;
  std::vector<KernelTimer::Pair> graph_pairs_;   // timing events inside graph_
  int32_t* rm_iters_ = nullptr;                  // per-voxel work of the
  int32_t* rm_evals_ = nullptr;                  // return mapping (timed runs)
  unsigned long long* rm_stats_ = nullptr;
  Net* net_ = nullptr;
  double* dFt_prev_ = nullptr;        // fluctuation increment of the last increment
  double* dFt_pp_ = nullptr;          // ... and of the increment before it
  double dFbar_prev_[9];
  double dFbar_pp_[9];
  double s_prev_ = 0.0;               // |dF_bar| of the last increment
  double s_pp_ = 0.0;                 // ... and of the one before it
  // FP64 residual of the plain predictor when it was last evaluated, and
  // the fraction of it below which warm_start = 2 keeps a learned candidate
  // without evaluating the plain predictor
  double last_plain_rel_ = 0.0;
  static constexpr double kLearnedDirect = 0.5;
  uint16_t* X0_ = nullptr;            // network input
  float* Ynet_ = nullptr;             // network output
  // user material (Appendix A): callback, state variables [nsv][N]
  // (committed and trial), Cauchy stress [6][N] and 6x6 tangent [36][N] of
  // the last evaluation
  rve_umat_fn umat_fn_ = nullptr;
  void* umat_user_ = nullptr;
  int32_t nsv_ = 0, nsv_cap_ = 0;
  double *sv_c_ = nullptr, *sv_t_ = nullptr, *usig_ = nullptr, *udds_ = nullptr;
  double* snap_ = nullptr;
  size_t snap_cap_ = 0;
  struct HostSnap {
    double Fbar[9], Pbar[9], dFlast[9], dFbar_prev[9], dFbar_pp[9];
    double s_prev, s_pp, t;
    int64_t increments;
  } snap_host_{};
  // second trial set for the learned-vs-plain predictor comparison
  double *F2_ = nullptr, *P2_ = nullptr, *Fpi_t2_ = nullptr, *chi_t2_ = nullptr,
         *dg_t2_ = nullptr, *r64b_ = nullptr;
};

}  // namespace rve
