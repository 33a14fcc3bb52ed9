// A batch of independent RVEs of mixed grid edges solved together: one
// voxel arena for all of them, one launch per pass for the whole batch,
// per-RVE Newton/CG control (converged RVEs drop out of the work).
#pragma once

#include <array>
#include <map>
#include <set>
#include <string>
#include <vector>

#include "../../include/rve.h"
#include "fips.hpp"
#include "kernels.hpp"

namespace rve {

class BatchEngine {
 public:
  BatchEngine(const rve_config& cfg, int count, const int32_t* n);
  ~BatchEngine();
  void set_microstructure(int b, const int32_t* phase, int32_t G,
                          const double* quat, const int32_t* law,
                          const double* params, int32_t nparams);
  int increment(const double* Fbar_all, double dt, rve_increment_info* info);
  void reset_fips();
  void get_field(int b, int field, void* dst, size_t bytes, bool on_device);
  size_t field_bytes(int b, int field) const;
  void get_macro(int b, double out[29]);
  void nonlocal_fips(int b, double width, rve_nonlocal_fips* out,
                     double* grain_pcyc, double* grain_pcyc_lit, int32_t labels,
                     double* band_wcyc, int32_t* band_desc, int64_t band_cap);
  int count() const { return B_; }
  // test hook: out = G(in) with the batched passes in the batch's precision
  void debug_apply_G(const double* in, double* out);
  // per-edge schedule of the batched CG matvec: tuned at the first
  // increment (or now, by tune) unless forced; (0, 0) tunes the edge again
  void tune();
  void set_schedule(int edge, int cpb, int tt);
  void get_schedule(int edge, int out[2], double* ms) const;

 private:
  void* alloc(size_t bytes);
  void release(void* p);
  void upload_scalars();
  void read_scalars();
  template <typename T>
  void cg_iteration(int parity);
  template <typename T>
  void cg_solve(std::vector<int>& iters);
  template <typename T>
  BatchSpec<T> spec(bool cg, int parity) const;
  // device-controlled increment (use_graph): Newton decisions on the
  // device, CG in one persistent launch per linear solve, the predictor and
  // the first Newton iterations replayed from a captured graph
  int increment_device(const double* Fbar_all, double dt,
                       rve_increment_info* info);
  template <typename T>
  void newton_solve_device(int it, const LawParams& lp);
  void newton_eval_device(int it, const LawParams& lp, const double* dg_start);
  void read_logs();
  void build_tables();
  template <typename T>
  void autotune();
  void ensure_tuned();

  rve_config cfg_;
  int B_;
  bool fp64_;
  hipStream_t st_;
  hipStream_t own_stream_ = nullptr;
  std::vector<std::pair<void*, size_t>> allocs_;
  std::vector<int> n_;
  std::vector<int64_t> off_, soff_;
  int64_t Nt_ = 0, St_ = 0;
  // arena fields
  double *Fprev_, *Pc_, *Fpi_c_, *chi_c_, *dg_c_, *pcyc_, *pcyc_lit_, *wcyc_;
  double *F_, *P_, *Fpi_t_, *chi_t_, *dg_t_, *r64_, *dFt_;
  void *K_, *x_, *r_, *p0_, *p1_, *Ap_, *spec_, *spec64_;
  int32_t* phase_;
  uint8_t* vrve_;
  double* table_ = nullptr;
  int table_labels_ = 0;
  std::vector<std::vector<double>> host_tables_;
  std::vector<int> label_count_;
  std::vector<int> label_off_;
  std::vector<std::vector<int32_t>> host_phase_;
  std::vector<bool> have_micro_;
  std::vector<FipIndex> fips_;
  std::vector<double> rel_;   // FP64 relative residual of the current iterate
  double params_[RVE_NPARAMS];
  bool have_params_ = false;
  // per-RVE control
  Scalars* sc_;
  Scalars* sc_host_ = nullptr;
  double* dF_dev_;
  // spectral descriptors (device) and grid sizes
  void *items32_, *items64_;
  int blocksA32_, blocksB32_, blocksA64_, blocksB64_;
  size_t ldsA32_, ldsB32_, ldsA64_, ldsB64_;
  int cpbs32_ = 3, cpbs64_ = 3;  // slab schedules present (BatchSpec::cpbs)
  double* partials_;
  SegItem* seg_;
  int seg_blocks_;
  RedItem *red_inv32_, *red_inv64_, *red_seg_;
  void *tw32_, *tw64_, *vt32_, *vt64_;  // per RVE, concatenated
  std::vector<int64_t> twoff_, vtoff_;  // each RVE's offsets in them
  std::vector<SpecItem<float>> host_it32_;
  std::vector<SpecItem<double>> host_it64_;
  void* tune_items_;                    // the tuner's sub-batch table
  std::map<int, std::array<int, 2>> sched_;  // edge -> (cpb, tt), CG precision
  std::map<int, double> sched_ms_;           // tuned matvec ms per edge
  std::set<int> forced_;
  bool tuned_ = false;
  double *psum_, *psq_;
  // host macro state per RVE
  std::vector<std::array<double, 9>> Fbar_, Pbar_;
  std::vector<double> t_;
  std::vector<int64_t> increments_;
  // device-controlled increments
  BatchLog* log_ = nullptr;
  std::vector<BatchLog> log_host_;
  unsigned* bar_ = nullptr;             // {count, generation, error}
  int persist_grid_ = 0;
  size_t persist_lds_ = 0;
  hipGraphExec_t inc_graph_ = nullptr;  // predictor + first iterations
  hipGraph_t inc_graph_def_ = nullptr;
  double inc_graph_dt_ = -1.0;
  static constexpr int kGraphNewton = 4;  // Newton iterations in the graph
};

}  // namespace rve
