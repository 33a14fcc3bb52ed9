// RVE engine: buffers and the increment algorithm (see engine.hpp).
#include "engine.hpp"
#include "newton.hpp"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>

#include "tables.hpp"

namespace rve {

namespace {

bool supported_n(int n) {
  switch (n) {
    case 16: case 24: case 32: case 40: case 48: case 64: case 96: case 128:
      return true;
  }
  return false;
}

double det3(const double* a) {
  return a[0] * (a[4] * a[8] - a[5] * a[7]) - a[1] * (a[3] * a[8] - a[5] * a[6]) +
         a[2] * (a[3] * a[7] - a[4] * a[6]);
}

constexpr uint64_t kStateMagic = 0x3153455645525652ull;  // "RVERVES1"

struct StateHeader {
  uint64_t magic;
  int64_t n;
  int64_t increments;
  double t;
  double Fbar[9];
  double Pbar[9];
};

}  // namespace

Engine::Engine(const rve_config& cfg) : cfg_(cfg) {
  if (cfg.n[0] != cfg.n[1] || cfg.n[1] != cfg.n[2] || !supported_n(cfg.n[0]))
    throw Error(RVE_EINVAL,
                "grid must be cubic with n in {16,24,32,40,48,64,96,128}");
  if (cfg.projection != RVE_PROJ_CONTINUOUS && cfg.projection != RVE_PROJ_DISCRETE)
    throw Error(RVE_EINVAL, "unknown projection operator");
  if (cfg.precision != RVE_PREC_FP64 && cfg.precision != RVE_PREC_MIXED)
    throw Error(RVE_EINVAL, "unknown precision mode");
  if (cfg.warm_start < 0 || cfg.warm_start > 3)
    throw Error(RVE_EINVAL, "warm_start must be 0, 1, 2 or 3");
  if (cfg.cg_forcing < 0 || cfg.cg_forcing > 2)
    throw Error(RVE_EINVAL, "cg_forcing must be 0, 1 or 2");
  for (int d = 0; d < 3; ++d)
    if (!(cfg.L[d] > 0.0)) throw Error(RVE_EINVAL, "cell lengths must be > 0");
  if (!(cfg.newton_tol > 0.0) || cfg.newton_max_iter < 0 ||
      cfg.newton_max_iter > RVE_MAX_NEWTON_LOG - 1 || !(cfg.cg_tol > 0.0) ||
      cfg.cg_max_iter < 1 || cfg.cg_chunk < 1)
    throw Error(RVE_EINVAL, "bad tolerance or iteration limits");
  if ((cfg.dev_alloc == nullptr) != (cfg.dev_free == nullptr))
    throw Error(RVE_EINVAL, "dev_alloc and dev_free must be given together");
  n_ = cfg.n[0];
  N_ = (int64_t)n_ * n_ * n_;
  fp64_ = cfg.precision == RVE_PREC_FP64;
  st_ = (hipStream_t)cfg.stream;
  if (cfg_.use_graph && st_ == nullptr) {
    // graph capture needs a non-legacy stream; this one is blocking with
    // respect to the default stream, so ordering with it is preserved
    RVE_HIP(hipStreamCreate(&own_stream_));
    st_ = own_stream_;
  }
  if (cfg_.cg_chunk % 2) cfg_.cg_chunk += 1;  // p0/p1 parity per chunk

  const size_t f9 = 9 * N_ * sizeof(double), f12 = 12 * N_ * sizeof(double),
               f1 = N_ * sizeof(double);
  const size_t tsz = fp64_ ? sizeof(double) : sizeof(float);
  Fprev_ = (double*)alloc(f9);
  Pc_ = (double*)alloc(f9);
  Fpi_c_ = (double*)alloc(f9);
  chi_c_ = (double*)alloc(f12);
  dg_c_ = (double*)alloc(f12);
  pcyc_ = (double*)alloc(f1);
  pcyc_lit_ = (double*)alloc(f1);
  wcyc_ = (double*)alloc(f12);
  F_ = (double*)alloc(f9);
  P_ = (double*)alloc(f9);
  Fpi_t_ = (double*)alloc(f9);
  chi_t_ = (double*)alloc(f12);
  dg_t_ = (double*)alloc(f12);
  r64_ = (double*)alloc(f9);
  dFt_prev_ = (double*)alloc(f9);
  dFt_pp_ = (double*)alloc(f9);
  K_ = alloc(81 * N_ * tsz);
  x_ = alloc(9 * N_ * tsz);
  r_ = alloc(9 * N_ * tsz);
  p0_ = alloc(9 * N_ * tsz);
  p1_ = alloc(9 * N_ * tsz);
  Kp_ = alloc(9 * N_ * tsz);
  spec_ = alloc(9 * N_ / 2 * 2 * tsz);
  spec64_ = fp64_ ? spec_ : alloc(9 * N_ / 2 * 2 * sizeof(double));
  nslab32_ = slab_blocks(n_, false);
  nslab64_ = slab_blocks(n_, true);
  // room for the partials of any schedule (one component per slab block)
  partial_inv_ = (double*)alloc(9 * n_ * sizeof(double));
  partial_red_ = (double*)alloc(kRedBlocks * sizeof(double));
  // the direction kernel's partials, or pass A's when it is folded in
  partial_kp_ = (double*)alloc(std::max(kp_blocks(N_), 9 * n_) * sizeof(double));
  psum_ = (double*)alloc(9 * n_ * sizeof(double));
  psq_ = (double*)alloc(9 * n_ * sizeof(double));
  sc_ = (Scalars*)alloc(sizeof(Scalars));
  RVE_HIP(hipMemsetAsync(sc_, 0, sizeof(Scalars), st_));
  // the timed matvecs of the schedule tuner may read these before the
  // solver writes them: start from zeros
  for (void* f : {K_, r_, x_, p0_, p1_})
    RVE_HIP(hipMemsetAsync(f, 0, (f == K_ ? 81 : 9) * N_ * tsz, st_));
  phase_ = (int32_t*)alloc(N_ * sizeof(int32_t));
  order_ = (int32_t*)alloc(N_ * sizeof(int32_t));
  table_ = nullptr;
  // slot 0: synchronous reads; slots 1, 2: the CG chunks' look-ahead reads
  // coherent: the chunk-closing and residual kernels write their slots
  // directly (uncached), no copy kernel behind them
  RVE_HIP(hipHostMalloc((void**)&sc_host_, 3 * sizeof(Scalars),
                        hipHostMallocCoherent | hipHostMallocMapped));
  RVE_HIP(hipHostGetDevicePointer((void**)&sc_pub_, sc_host_, 0));
  RVE_HIP(hipEventCreateWithFlags(&chunk_ev_[0], hipEventDisableTiming));
  RVE_HIP(hipEventCreateWithFlags(&chunk_ev_[1], hipEventDisableTiming));

  std::vector<double> tw = twiddles(n_);
  std::vector<float> tw32(tw.begin(), tw.end());
  std::vector<double> vt = wave_vectors(n_, cfg_.L, cfg_.projection);
  std::vector<float> vt32(vt.begin(), vt.end());
  tw64_ = alloc(tw.size() * sizeof(double));
  tw32_ = alloc(tw32.size() * sizeof(float));
  vt64_ = alloc(vt.size() * sizeof(double));
  vt32_ = alloc(vt32.size() * sizeof(float));
  RVE_HIP(hipMemcpyAsync(tw64_, tw.data(), tw.size() * sizeof(double),
                         hipMemcpyHostToDevice, st_));
  RVE_HIP(hipMemcpyAsync(tw32_, tw32.data(), tw32.size() * sizeof(float),
                         hipMemcpyHostToDevice, st_));
  RVE_HIP(hipMemcpyAsync(vt64_, vt.data(), vt.size() * sizeof(double),
                         hipMemcpyHostToDevice, st_));
  RVE_HIP(hipMemcpyAsync(vt32_, vt32.data(), vt32.size() * sizeof(float),
                         hipMemcpyHostToDevice, st_));
  RVE_HIP(hipStreamSynchronize(st_));
  for (int i = 0; i < 9; ++i) {
    Fbar_[i] = (i % 4 == 0) ? 1.0 : 0.0;
    Pbar_[i] = 0.0;
    dFlast_[i] = 0.0;
    dFbar_prev_[i] = 0.0;
  }
}

Engine::~Engine() {
  if (graph_) hipGraphExecDestroy(graph_);
  if (graph_def_) hipGraphDestroy(graph_def_);
  if (st_) hipStreamSynchronize(st_);
  free_all();
  if (sc_host_) hipHostFree(sc_host_);
  for (hipEvent_t e : chunk_ev_)
    if (e) hipEventDestroy(e);
  if (own_stream_) hipStreamDestroy(own_stream_);
}

void* Engine::alloc(size_t bytes) {
  if (bytes == 0) bytes = 256;
  void* p = nullptr;
  if (cfg_.dev_alloc) {
    p = cfg_.dev_alloc(bytes, (void*)st_, cfg_.alloc_ctx);
    if (!p) throw Error(RVE_ENOMEM, "device allocator returned NULL");
  } else {
    hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      throw Error(RVE_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
    }
  }
  allocs_.push_back({p, bytes});
  return p;
}

void Engine::release(void* p) {
  for (size_t i = 0; i < allocs_.size(); ++i) {
    if (allocs_[i].first != p) continue;
    if (cfg_.dev_free)
      cfg_.dev_free(p, cfg_.alloc_ctx);
    else
      hipFree(p);
    allocs_.erase(allocs_.begin() + i);
    return;
  }
}

void Engine::free_all() {
  for (auto& a : allocs_) {
    if (cfg_.dev_free)
      cfg_.dev_free(a.first, cfg_.alloc_ctx);
    else
      hipFree(a.first);
  }
  allocs_.clear();
}

void Engine::set_microstructure(const int32_t* phase, int32_t G,
                                const double* quat, const int32_t* law,
                                const double* params, int32_t nparams) {
  if (!phase || !quat || !law || !params || G < 1)
    throw Error(RVE_EINVAL, "null microstructure input or G < 1");
  if (nparams < RVE_NPARAMS) throw Error(RVE_EINVAL, "nparams < RVE_NPARAMS");
  for (int64_t v = 0; v < N_; ++v)
    if (phase[v] < 0 || phase[v] >= G)
      throw Error(RVE_EINVAL, "phase label out of [0, G)");
  for (int g = 0; g < G; ++g) {
    if (law[g] != 0 && law[g] != 1) throw Error(RVE_EINVAL, "unknown law id");
    const double q2 = quat[4 * g] * quat[4 * g] + quat[4 * g + 1] * quat[4 * g + 1] +
                      quat[4 * g + 2] * quat[4 * g + 2] +
                      quat[4 * g + 3] * quat[4 * g + 3];
    if (!(std::fabs(q2 - 1.0) < 1e-6)) throw Error(RVE_EINVAL, "quaternion not unit");
  }
  for (int i = 0; i < RVE_NPARAMS; ++i) {
    if (!std::isfinite(params[i])) throw Error(RVE_EINVAL, "non-finite parameter");
    params_[i] = params[i];
  }
  if (!(params_[3] > 0 && params_[4] > 0 && params_[5] >= 1 && params_[7] >= 0))
    throw Error(RVE_EINVAL, "bad flow-rule parameters");
  std::vector<double> tab = label_table(G, quat, law, params_);
  if (G > labels_) {
    table_ = (double*)alloc(tab.size() * sizeof(double));
    labels_ = G;
  }
  RVE_HIP(hipMemcpyAsync(table_, tab.data(), tab.size() * sizeof(double),
                         hipMemcpyHostToDevice, st_));
  RVE_HIP(hipMemcpyAsync(phase_, phase, N_ * sizeof(int32_t),
                         hipMemcpyHostToDevice, st_));
  // work order of the return mapping: crystal voxels first (in index
  // order), then the particle voxels, so that the wavefronts that iterate
  // the local Newton solve carry no particle lanes
  order_host_.clear();
  order_host_.reserve(N_);
  for (int pass = 0; pass < 2; ++pass)
    for (int64_t v = 0; v < N_; ++v)
      if ((law[phase[v]] == 0) == (pass == 0)) order_host_.push_back((int32_t)v);
  RVE_HIP(hipMemcpyAsync(order_, order_host_.data(), N_ * sizeof(int32_t),
                         hipMemcpyHostToDevice, st_));
  phase_host_.assign(phase, phase + N_);
  table_host_ = tab;
  G_ = G;
  fips_.invalidate();
  // reset to F = I, Fp^-1 = I, chi = 0, indicators = 0
  std::vector<double> eye(9 * N_, 0.0);
  for (int c = 0; c < 9; c += 4)
    for (int64_t v = 0; v < N_; ++v) eye[c * N_ + v] = 1.0;
  RVE_HIP(hipMemcpyAsync(Fprev_, eye.data(), 9 * N_ * sizeof(double),
                         hipMemcpyHostToDevice, st_));
  RVE_HIP(hipMemcpyAsync(Fpi_c_, eye.data(), 9 * N_ * sizeof(double),
                         hipMemcpyHostToDevice, st_));
  launch_fill_f64(Pc_, 0.0, 9 * N_, st_);
  launch_fill_f64(chi_c_, 0.0, 12 * N_, st_);
  launch_fill_f64(dg_c_, 0.0, 12 * N_, st_);
  launch_fill_f64(pcyc_, 0.0, N_, st_);
  launch_fill_f64(pcyc_lit_, 0.0, N_, st_);
  launch_fill_f64(wcyc_, 0.0, 12 * N_, st_);
  launch_fill_f64(dFt_prev_, 0.0, 9 * N_, st_);
  launch_fill_f64(dFt_pp_, 0.0, 9 * N_, st_);
  RVE_HIP(hipGetLastError());
  RVE_HIP(hipStreamSynchronize(st_));
  reset_macro_state();
  umat_fn_ = nullptr;
  umat_user_ = nullptr;
  nsv_ = 0;
  have_micro_ = true;
}

void Engine::reset_macro_state() {
  for (int i = 0; i < 9; ++i) {
    Fbar_[i] = (i % 4 == 0) ? 1.0 : 0.0;
    Pbar_[i] = 0.0;
    dFlast_[i] = 0.0;
    dFbar_prev_[i] = 0.0;
    dFbar_pp_[i] = 0.0;
  }
  s_prev_ = 0.0;
  s_pp_ = 0.0;
  t_ = 0.0;
  increments_ = 0;
  last_plain_rel_ = 0.0;
}

void Engine::require_crystal(const char* what) const {
  if (umat_fn_)
    throw Error(RVE_ESTATE, std::string(what) +
                                " needs the crystal-plasticity microstructure, "
                                "not a user material");
}

void Engine::set_user_material(rve_umat_fn fn, void* user, int32_t nstatev,
                               const double* statev0) {
  if (!fn) throw Error(RVE_EINVAL, "null user material");
  if (nstatev < 0 || nstatev > 1024) throw Error(RVE_EINVAL, "nstatev out of [0, 1024]");
  if (nstatev > 0 && !statev0) throw Error(RVE_EINVAL, "null initial state variables");
  if (!usig_) {
    usig_ = (double*)alloc(6 * N_ * sizeof(double));
    udds_ = (double*)alloc(36 * N_ * sizeof(double));
  }
  if (nstatev > nsv_cap_) {
    sv_c_ = (double*)alloc(nstatev * N_ * sizeof(double));
    sv_t_ = (double*)alloc(nstatev * N_ * sizeof(double));
    nsv_cap_ = nstatev;
  }
  if (nstatev > 0)
    RVE_HIP(hipMemcpyAsync(sv_c_, statev0, nstatev * N_ * sizeof(double),
                           hipMemcpyHostToDevice, st_));
  // F = I, P = 0, indicators 0 (not defined for a user material)
  launch_fill_f64(Fprev_, 0.0, 9 * N_, st_);
  for (int c = 0; c < 9; c += 4) launch_fill_f64(Fprev_ + c * N_, 1.0, N_, st_);
  launch_fill_f64(Pc_, 0.0, 9 * N_, st_);
  launch_fill_f64(pcyc_, 0.0, N_, st_);
  launch_fill_f64(pcyc_lit_, 0.0, N_, st_);
  launch_fill_f64(wcyc_, 0.0, 12 * N_, st_);
  launch_fill_f64(dFt_prev_, 0.0, 9 * N_, st_);
  launch_fill_f64(dFt_pp_, 0.0, 9 * N_, st_);
  RVE_HIP(hipGetLastError());
  RVE_HIP(hipStreamSynchronize(st_));
  reset_macro_state();
  umat_fn_ = fn;
  umat_user_ = user;
  nsv_ = nstatev;
  have_micro_ = true;
}

void Engine::read_scalars(Scalars& h) {
  RVE_HIP(hipMemcpyAsync(sc_host_, sc_, sizeof(Scalars), hipMemcpyDeviceToHost,
                         st_));
  RVE_HIP(hipStreamSynchronize(st_));
  h = *sc_host_;
}

LawParams Engine::law_params(double dt) const {
  LawParams lp;
  lp.gdot0 = params_[3];
  lp.g = params_[4];
  lp.nexp = params_[5];
  lp.c_af = params_[6];
  lp.d_af = params_[7];
  lp.dt = dt;
  lp.inv_g = 1.0 / lp.g;
  lp.inv_a = 1.0 / (dt * lp.gdot0);
  lp.nint = flow_exponent_int(lp.nexp);
  return lp;
}

void Engine::residual_passes(const double* P, Scalars* pub) {
  SpectralLaunch<double> L;
  L.src = SRC_FIELD;
  L.in_field = P;
  L.spec = (cplx<double>*)spec64_;
  L.tw = (const cplx<double>*)tw64_;
  L.vt = (const double*)vt64_;
  L.psum = psum_;
  L.psq = psq_;
  L.dst = DST_NORM;
  L.out_d = r64_;
  L.partial_inv = partial_inv_;
  launch_G<double>(n_, L, st_);
  launch_reduce(RED_RESID, partial_inv_, nslab64_, psum_, psq_, n_,
                1.0 / (double)N_, sc_, sc_->pbar, st_, pub);
}

// constitutive update at F_ with the committed state, then r64 = G(P)
int Engine::evaluate(const double* dg_start, double dt, double& rel,
                     double& res, double& pn) {
  launch_fill_i32(&sc_->fails, 0, 1, st_);
  ConstArgs a{};
  a.F = F_;
  a.Fpi0 = Fpi_c_;
  a.chi0 = chi_c_;
  a.dg0 = dg_start;
  a.phase = phase_;
  a.table = table_;
  a.P = P_;
  a.Fpi = Fpi_t_;
  a.chi = chi_t_;
  a.dg = dg_t_;
  a.fails = &sc_->fails;
  a.iters = timer_.on(4) ? rm_iters_ : nullptr;
  a.evals = timer_.on(4) ? rm_evals_ : nullptr;
  a.lp = law_params(dt);
  a.order = order_;
  a.N = N_;
  if (umat_fn_) {
    // user material: sigma and its Jaumann tangent, then P (Eq. A.1)
    const int32_t rc = umat_fn_(umat_user_, F_, Fprev_, sv_c_, sv_t_, nsv_,
                                usig_, udds_, &sc_->fails, N_, dt, (void*)st_);
    if (rc != 0)
      throw Error(RVE_EDEVICE, "user material returned " + std::to_string(rc));
    launch_umat_piola(F_, usig_, N_, P_, st_);
  } else {
    timer_.begin(4, st_);
    launch_return_map(a, st_);
    timer_.end(4, st_);
    if (a.iters) launch_rm_count(rm_iters_, rm_evals_, N_, rm_stats_, st_);
  }
  timer_.begin_span(6, st_);
  residual_passes(P_, sc_pub_);  // the reduction publishes into slot 0
  timer_.end_span(6, st_);
  RVE_HIP(hipGetLastError());
  RVE_HIP(hipStreamSynchronize(st_));
  const Scalars h = *sc_host_;
  timer_.flush();
  res = std::sqrt(h.res2);
  pn = std::sqrt(h.P2);
  rel = pn > 0 ? res / pn : 0.0;
  for (int i = 0; i < 9; ++i) Pbar_new_[i] = h.pbar[i];
  return h.fails;
}

template <typename T>
void Engine::tangent(double dt) {
  TangentArgs<T> a{};
  a.F = F_;
  a.Fpi0 = Fpi_c_;
  a.chi0 = chi_c_;
  a.dg = dg_t_;
  a.phase = phase_;
  a.table = table_;
  a.K = (T*)K_;
  a.lp = law_params(dt);
  a.order = order_;
  a.N = N_;
  if (umat_fn_) {
    // user material: K from the last evaluation's sigma and tangent (Eq. A.16)
    launch_umat_tangent<T>(F_, usig_, udds_, N_, (T*)K_, st_);
    return;
  }
  timer_.begin(5, st_);
  launch_tangent<T>(a, st_);
  timer_.end(5, st_);
}

// One CG iteration as a sequence of launch steps; run(cls, launch) issues a
// step (cls: kernel class for live timing, -1 untimed).
template <typename T, typename Run>
void Engine::cg_iteration_steps(int parity, Run&& run) {
  const bool dbl = sizeof(T) == sizeof(double);
  T* p_new = (T*)(parity ? p0_ : p1_);
  const int nslab = slab_blocks(n_, dbl, sched_cpb_);
  const T* p_old = (const T*)(parity ? p1_ : p0_);
  // beta from the last inverse pass's r.r partials, the previous
  // iteration's x += alpha p_old, p = r + beta p_old and y = K : p with the
  // p . y partials, in one streaming pass (or folded into pass A)
  if (!sched_fused_)
    run(7, [&] {
      launch_kp<T>((const T*)K_, (const T*)r_, p_old, p_new, (T*)Kp_, sc_, N_,
                   st_, partial_inv_, nslab, parity, (T*)x_, partial_kp_);
    });
  // G(y); pass A (pass B when fused) publishes alpha = r.r / p.y, pass C
  // applies r -= alpha G(y) and writes the new r.r partials
  SpectralLaunch<T> L;
  if (sched_fused_) {
    L.src = SRC_KP;
    L.K = (const T*)K_;
    L.r = (const T*)r_;
    L.p_old = p_old;
    L.x = (T*)x_;
    L.pinv = partial_inv_;
    L.pinv_count = nslab;
  } else {
    L.src = SRC_FIELD;
    L.in_field = (const T*)Kp_;
  }
  L.p_new = p_new;
  L.spec = (cplx<T>*)spec_;
  L.tw = (const cplx<T>*)(dbl ? tw64_ : tw32_);
  L.vt = (const T*)(dbl ? vt64_ : vt32_);
  L.dst = DST_CG;
  L.r_io = (T*)r_;
  L.pkp = partial_kp_;
  L.pkp_count = sched_fused_ ? nslab : kp_blocks(N_);
  L.parity = parity;
  L.partial_inv = partial_inv_;
  L.sc = sc_;
  L.cpb = sched_cpb_;
  L.tt = sched_tt_;
  if (timer_.mask() & 7u) {
    for (int pass = 0; pass < 3; ++pass)  // passes A, B, C one by one
      run(pass, [&, pass] {
        SpectralLaunch<T> Lp = L;
        Lp.passes = 1 << pass;
        launch_G<T>(n_, Lp, st_);
      });
  } else {
    run(-1, [&] { launch_G<T>(n_, L, st_); });
  }
}

template <typename T>
void Engine::cg_iteration(int parity) {
  cg_iteration_steps<T>(parity, [&](int cls, auto&& launch) {
    if (cls >= 0) timer_.begin(cls, st_);
    launch();
    if (cls >= 0) timer_.end(cls, st_);
  });
}

// kernel classes launched inside a CG iteration: passes A-C, update, K:p
constexpr uint32_t kCgClasses = 0x8Fu;

// The CG chunk as one graph.  Without live timing the chunk is captured in
// one piece; with it, each step is captured as a child graph and the timed
// steps are bracketed by event-record nodes, linked in launch order.
template <typename T>
void Engine::capture_graph() {
  if (!(timer_.mask() & kCgClasses)) {
    RVE_HIP(hipStreamBeginCapture(st_, hipStreamCaptureModeThreadLocal));
    for (int j = 0; j < cfg_.cg_chunk; ++j) cg_iteration<T>(j & 1);
    launch_cg_close(partial_inv_, slab_blocks(n_, sizeof(T) == 8, sched_cpb_),
                    sc_, 0, st_);
    RVE_HIP(hipStreamEndCapture(st_, &graph_def_));
  } else {
    RVE_HIP(hipGraphCreate(&graph_def_, 0));
    hipGraphNode_t last = nullptr;
    auto add = [&](auto&& make) {
      hipGraphNode_t node;
      make(&node, last ? &last : nullptr, last ? 1 : 0);
      last = node;
    };
    auto step = [&](int cls, auto&& launch) {
      hipGraph_t child;
      RVE_HIP(hipStreamBeginCapture(st_, hipStreamCaptureModeThreadLocal));
      launch();
      RVE_HIP(hipStreamEndCapture(st_, &child));
      const bool timed = cls >= 0 && timer_.on(cls);
      KernelTimer::Pair pr{};
      if (timed) {
        pr = timer_.graph_pair(cls);
        add([&](hipGraphNode_t* n, const hipGraphNode_t* d, size_t nd) {
          RVE_HIP(hipGraphAddEventRecordNode(n, graph_def_, d, nd, pr.second.first));
        });
      }
      add([&](hipGraphNode_t* n, const hipGraphNode_t* d, size_t nd) {
        RVE_HIP(hipGraphAddChildGraphNode(n, graph_def_, d, nd, child));
      });
      RVE_HIP(hipGraphDestroy(child));
      if (timed) {
        add([&](hipGraphNode_t* n, const hipGraphNode_t* d, size_t nd) {
          RVE_HIP(hipGraphAddEventRecordNode(n, graph_def_, d, nd, pr.second.second));
        });
        graph_pairs_.push_back(pr);
      }
    };
    for (int j = 0; j < cfg_.cg_chunk; ++j) cg_iteration_steps<T>(j & 1, step);
    step(-1, [&] {
      launch_cg_close(partial_inv_,
                      slab_blocks(n_, sizeof(T) == 8, sched_cpb_), sc_, 0, st_);
    });
  }
  RVE_HIP(hipGraphInstantiate(&graph_, graph_def_, nullptr, nullptr, 0));
}

// Picks the fastest schedule of the CG matvec G(K : p) for this grid and
// precision (components per slab block in passes A and C, kz columns per
// pass-B block, and whether the direction kernel is folded into pass A) by
// timing one matvec with each valid candidate on the live buffers, with
// alpha = beta = 0 (p = r + 0 p_old, x += 0 p_old: the memory traffic of
// an iteration after the first; the CG vectors are re-initialised
// afterwards): the direction kernel and the three passes, or the three
// passes with the folded pass A.
template <typename T>
void Engine::autotune() {
  const bool dbl = sizeof(T) == sizeof(double);
  hipEvent_t ev[2];
  RVE_HIP(hipEventCreate(&ev[0]));
  RVE_HIP(hipEventCreate(&ev[1]));
  struct Cand {
    int cpb, tt, fused;
  };
  std::vector<Cand> cand;
  for (int fused : {0, 1})
    for (int cpb : {1, 3})
      for (int tt : {4, 8, 16})
        if (schedule_valid(n_, dbl, cpb, tt)) cand.push_back({cpb, tt, fused});
  // alpha = 0 in every slot: the timed passes leave r and x unchanged
  launch_bench_scalars(sc_, st_);
  // three interleaved rounds, the best of each candidate's timings: robust
  // against clock and cache drift between candidates
  std::vector<float> tbest(cand.size(), 0.f);
  constexpr int reps = 4;
  for (int round = 0; round < 3; ++round)
    for (size_t c = 0; c < cand.size(); ++c) {
      SpectralLaunch<T> L;
      if (cand[c].fused) {
        L.src = SRC_KP;
        L.K = (const T*)K_;
        L.r = (const T*)r_;
        L.p_old = (const T*)p0_;
        L.x = (T*)x_;
      } else {
        L.src = SRC_FIELD;
        L.in_field = (const T*)Kp_;
      }
      L.p_new = (T*)p1_;
      L.spec = (cplx<T>*)spec_;
      L.tw = (const cplx<T>*)(dbl ? tw64_ : tw32_);
      L.vt = (const T*)(dbl ? vt64_ : vt32_);
      L.dst = DST_CG;
      L.r_io = (T*)r_;
      L.partial_inv = partial_inv_;
      L.sc = sc_;
      L.cpb = cand[c].cpb;
      L.tt = cand[c].tt;
      auto matvec = [&] {
        if (!cand[c].fused)
          launch_kp<T>((const T*)K_, (const T*)r_, (const T*)p0_, (T*)p1_,
                       (T*)Kp_, sc_, N_, st_, nullptr, 0, 0, (T*)x_,
                       partial_kp_);
        launch_G<T>(n_, L, st_);
      };
      matvec();  // untimed first launch
      RVE_HIP(hipEventRecord(ev[0], st_));
      for (int i = 0; i < reps; ++i) matvec();
      RVE_HIP(hipEventRecord(ev[1], st_));
      RVE_HIP(hipEventSynchronize(ev[1]));
      float t = 0.f;
      RVE_HIP(hipEventElapsedTime(&t, ev[0], ev[1]));
      if (round == 0 || t < tbest[c]) tbest[c] = t;
    }
  float best = 0.f;
  int bi = -1;
  for (size_t c = 0; c < cand.size(); ++c)
    if (bi < 0 || tbest[c] < best) {
      best = tbest[c];
      bi = (int)c;
    }
  hipEventDestroy(ev[0]);
  hipEventDestroy(ev[1]);
  if (bi < 0) throw Error(RVE_EINVAL, "no FFT schedule for this grid");
  sched_cpb_ = cand[bi].cpb;
  sched_tt_ = cand[bi].tt;
  sched_fused_ = cand[bi].fused;
  sched_ms_ = best / reps;
}

void Engine::tune() {
  set_schedule(0, 0, 0);  // drops a captured graph
  if (fp64_) autotune<double>(); else autotune<float>();
}

void Engine::set_schedule(int cpb, int tt, int fused) {
  if (fused != 0 && fused != 1)
    throw Error(RVE_EINVAL, "fused must be 0 or 1");
  if (cpb || tt) {
    if (!schedule_valid(n_, fp64_, cpb, tt))
      throw Error(RVE_EINVAL, "no such FFT schedule for this grid and precision");
  }
  RVE_HIP(hipStreamSynchronize(st_));
  if (graph_) {
    RVE_HIP(hipGraphExecDestroy(graph_));
    graph_ = nullptr;
  }
  if (graph_def_) {
    RVE_HIP(hipGraphDestroy(graph_def_));
    graph_def_ = nullptr;
  }
  timer_.recycle(graph_pairs_);
  sched_cpb_ = cpb;
  sched_tt_ = tt;
  sched_fused_ = (cpb || tt) ? fused : 0;
  sched_ms_ = 0.0;
}

// CG on G(K : x) = b with b = -r64 (text after Eq. 16), from x = 0
template <typename T>
void Engine::cg_solve(int& iters, bool& breakdown, double eta) {
  if (!sched_cpb_) autotune<T>();
  launch_init_scalars(sc_, cfg_.cg_max_iter, eta, st_);
  launch_cg_init<T>(r64_, (T*)r_, (T*)x_, partial_red_, kRedBlocks, 9 * N_, st_);
  launch_reduce(RED_INIT, partial_red_, kRedBlocks, nullptr, nullptr, 0, 0.0,
                sc_, nullptr, st_);
  RVE_HIP(hipGetLastError());
  // Chunks are queued one ahead of the host's convergence check: chunk k+1
  // is enqueued before the scalars of chunk k are waited for, so the device
  // never idles during that round trip.  A chunk queued after convergence
  // does nothing (every CG kernel returns at once when `done` is set), but
  // each of its launches still costs a dispatch.  With direct launches the
  // length of the chunk queued ahead (at most cg_chunk) follows the r.r
  // decay seen so far: the iterations expected to remain after the chunk in
  // flight, at least one, since the direction kernel that follows a chunk
  // whose closing kernel stops the run applies the last x += alpha p.
  int parity = 0;
  auto enqueue = [&](int slot, int len) {
    if (cfg_.use_graph) {
      if (!graph_) capture_graph<T>();
      RVE_HIP(hipGraphLaunch(graph_, st_));
      timer_.replayed(graph_pairs_);
    } else {
      for (int j = 0; j < len; ++j) {
        cg_iteration<T>(parity);
        parity ^= 1;
      }
      // the closing kernel copies the scalars into the slot itself
      launch_cg_close(partial_inv_,
                      slab_blocks(n_, sizeof(T) == 8, sched_cpb_), sc_, parity,
                      st_, sc_pub_ + 1 + slot);
    }
    if (cfg_.use_graph)
      RVE_HIP(hipMemcpyAsync(sc_host_ + 1 + slot, sc_, sizeof(Scalars),
                             hipMemcpyDeviceToHost, st_));
    RVE_HIP(hipEventRecord(chunk_ev_[slot], st_));
    RVE_HIP(hipGetLastError());
  };
  const int full = cfg_.cg_chunk;
  int len[2] = {full, full};   // lengths of the chunks in the two slots
  // the two latest known points (iterations, r.r) of the residual history
  double it0 = -1.0, rr0 = 0.0, it1 = -1.0, rr1 = 0.0, eta2bb = 0.0;
  auto next_len = [&](int inflight) {
    if (cfg_.use_graph || !(it0 >= 0.0) || !(it1 > it0) || !(rr1 > 0.0) ||
        !(rr0 > rr1) || !(eta2bb > 0.0))
      return full;
    // geometric decay per iteration between the two points
    const double lrho = std::log(rr1 / rr0) / (it1 - it0);
    const double need = std::log(eta2bb / rr1) / lrho;  // iterations left
    const double after = need - inflight;
    if (!std::isfinite(after)) return full;
    return std::min(full, std::max(1, (int)std::ceil(after)));
  };
  Scalars h;
  int k = 0;
  enqueue(0, len[0]);
  for (;;) {
    len[(k + 1) & 1] = next_len(len[k & 1]);
    enqueue((k + 1) & 1, len[(k + 1) & 1]);
    RVE_HIP(hipEventSynchronize(chunk_ev_[k & 1]));
    h = sc_host_[1 + (k & 1)];
    if (h.done) break;
    if (it1 < 0.0) {  // the start of the solve: r.r = ||b||^2 at iteration 0
      it1 = 0.0;
      rr1 = h.bb;
    }
    it0 = it1;
    rr0 = rr1;
    it1 = (double)h.iters;
    rr1 = h.rr_new;
    eta2bb = h.eta2bb;
    ++k;
  }
  // the live timings of this solve are read at the next synchronous scalar
  // read, once the queued chunk has drained
  iters = h.iters;
  breakdown = h.breakdown != 0;
}

void Engine::commit(double dt) {
  // fluctuation increments of this increment and of the one before it
  std::swap(dFt_prev_, dFt_pp_);
  nn_fluct_increment(F_, Fprev_, dFlast_, dFt_prev_, N_, st_);
  CommitArgs c{};
  c.F = F_;
  c.Fpi_t = Fpi_t_;
  c.dg_t = dg_t_;
  c.phase = phase_;
  c.table = table_;
  c.pcyc = pcyc_;
  c.pcyc_lit = pcyc_lit_;
  c.wcyc = wcyc_;
  c.dt = dt;
  c.N = N_;
  if (umat_fn_)
    std::swap(sv_c_, sv_t_);
  else
    launch_commit(c, st_);
  RVE_HIP(hipMemcpyAsync(Pc_, P_, 9 * N_ * sizeof(double),
                         hipMemcpyDeviceToDevice, st_));
  RVE_HIP(hipGetLastError());
  std::swap(Fpi_c_, Fpi_t_);
  std::swap(chi_c_, chi_t_);
  std::swap(dg_c_, dg_t_);
  std::swap(Fprev_, F_);
  for (int i = 0; i < 9; ++i) Pbar_[i] = Pbar_new_[i];
}

int Engine::increment(const double Fbar_new[9], double dt,
                      rve_increment_info* info) {
  if (!have_micro_) throw Error(RVE_ESTATE, "no microstructure set");
  if (!(dt > 0.0) || !std::isfinite(dt)) throw Error(RVE_EINVAL, "dt must be > 0");
  for (int i = 0; i < 9; ++i)
    if (!std::isfinite(Fbar_new[i])) throw Error(RVE_EINVAL, "non-finite F_bar");
  if (!(det3(Fbar_new) > 0.0)) throw Error(RVE_EINVAL, "det(F_bar) must be > 0");
  const auto t0 = std::chrono::steady_clock::now();
  rve_increment_info loc;
  std::memset(&loc, 0, sizeof(loc));
  double dF[9];
  for (int i = 0; i < 9; ++i) dF[i] = Fbar_new[i] - Fbar_[i];
  launch_predict(F_, Fprev_, dF, N_, st_);
  const double* dg_start = dg_c_;
  double rel = 0, res = 0, pn = 0;
  int status = RVE_ENOTCONV;
  int pre_fails = -1;
  const bool candidate =
      cfg_.warm_start && !umat_fn_ &&
      (cfg_.warm_start == 3 ? extrapolated_candidate(Fbar_new)
                            : (net_ && learned_candidate(Fbar_new)));
  if (candidate) {
    // learned (or extrapolated) candidate in F2_: evaluate it; with
    // warm_start = 2 or 3 keep it at once when its FP64 residual is well
    // below what the plain predictor reached when last evaluated, otherwise
    // stash it, evaluate the plain predictor and keep the one with the
    // smaller FP64 residual
    std::swap(F_, F2_);
    double relL, resL, pnL;
    const int failsL = evaluate(dg_start, dt, relL, resL, pnL);
    if (cfg_.warm_start >= 2 && failsL == 0 && last_plain_rel_ > 0.0 &&
        relL < kLearnedDirect * last_plain_rel_) {
      rel = relL;
      res = resL;
      pn = pnL;
      pre_fails = 0;
      loc.used_learned = 1;
      loc.plain_predictor_residual = -1.0;   // not evaluated
    } else {
      swap_trial_sets();
      std::swap(F_, F2_);
      double pbarL[9];
      for (int i = 0; i < 9; ++i) pbarL[i] = Pbar_new_[i];
      pre_fails = evaluate(dg_start, dt, rel, res, pn);
      loc.plain_predictor_residual = rel;
      last_plain_rel_ = rel;
      if (failsL == 0 && relL < rel) {
        swap_trial_sets();
        std::swap(F_, F2_);
        rel = relL;
        res = resL;
        pn = pnL;
        pre_fails = 0;
        for (int i = 0; i < 9; ++i) Pbar_new_[i] = pbarL[i];
        loc.used_learned = 1;
      }
    }
  }
  for (int i = 0; i < 9; ++i) dFlast_[i] = dF[i];
  for (int it = 0; it <= cfg_.newton_max_iter; ++it) {
    const int fails = (it == 0 && pre_fails >= 0)
                          ? pre_fails
                          : evaluate(dg_start, dt, rel, res, pn);
    if (it < RVE_MAX_NEWTON_LOG) loc.residual_history[it] = rel;
    if (it == 0) {
      loc.predictor_residual = rel;
      if (!loc.used_learned) {
        loc.plain_predictor_residual = rel;
        last_plain_rel_ = rel;
      }
    }
    loc.residual_rel = rel;
    if (fails > 0) {
      loc.local_failures = fails;
      status = RVE_ELOCAL;
      break;
    }
    if (res <= cfg_.newton_tol * pn) {
      commit(dt);
      double s2 = 0.0, dot = 0.0;
      for (int i = 0; i < 9; ++i) s2 += dF[i] * dF[i];
      for (int i = 0; i < 9; ++i) {
        Fbar_[i] = Fbar_new[i];
        dFbar_pp_[i] = dFbar_prev_[i];
        dFbar_prev_[i] = dF[i];
        (void)dot;
      }
      s_pp_ = s_prev_;
      s_prev_ = std::sqrt(s2);
      t_ += dt;
      ++increments_;
      status = RVE_OK;
      loc.newton_iters = it;
      break;
    }
    if (it == cfg_.newton_max_iter) {
      loc.newton_iters = it;
      status = RVE_ENOTCONV;
      break;
    }
    int iters = 0;
    bool bd = false;
    // linear-solve tolerance: fixed, or (cg_forcing) only as tight as the
    // equilibrium tolerance needs from this residual, never tighter than
    // cg_tol
    const double eta = forcing_eta(cfg_.cg_forcing, cfg_.cg_tol,
                                   cfg_.newton_tol, rel);
    if (fp64_) {
      tangent<double>(dt);
      cg_solve<double>(iters, bd, eta);
      launch_add_to_F<double>(F_, (const double*)x_, 9 * N_, st_);
    } else {
      tangent<float>(dt);
      cg_solve<float>(iters, bd, eta);
      launch_add_to_F<float>(F_, (const float*)x_, 9 * N_, st_);
    }
    RVE_HIP(hipGetLastError());
    if (it < RVE_MAX_NEWTON_LOG) loc.cg_iters[it] = iters;
    loc.cg_iters_total += iters;
    loc.cg_breakdowns += bd ? 1 : 0;
    dg_start = dg_t_;
  }
  for (int i = 0; i < 9; ++i) loc.P_bar[i] = (status == RVE_OK) ? Pbar_[i] : Pbar_new_[i];
  const double J = det3(Fbar_new);
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double s = 0.0;
      for (int k = 0; k < 3; ++k) s += loc.P_bar[3 * i + k] * Fbar_new[3 * j + k];
      loc.sigma_bar[3 * i + j] = s / J;
    }
  loc.status = status;
  loc.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  if (info) *info = loc;
  return status;
}

// committed device arrays and their component counts (user-material state
// variables last)
#define RVE_SNAP_ARRAYS                                                   \
  double* arrs[12] = {Fprev_, Pc_, Fpi_c_, chi_c_, dg_c_, pcyc_, pcyc_lit_, \
                      wcyc_, dFt_prev_, dFt_pp_, sv_c_, nullptr};         \
  const int comps[12] = {9, 9, 9, 12, 12, 1, 1, 12, 9, 9, nsv_, 0};

void Engine::take_snapshot() {
  RVE_SNAP_ARRAYS
  size_t total = 0;
  for (int k = 0; k < 11; ++k) total += (size_t)comps[k];
  const size_t bytes = total * N_ * sizeof(double);
  if (bytes > snap_cap_) {
    if (snap_) release(snap_);
    snap_ = nullptr;
    snap_cap_ = 0;
    snap_ = (double*)alloc(bytes);
    snap_cap_ = bytes;
  }
  double* p = snap_;
  for (int k = 0; k < 11; ++k) {
    if (!comps[k]) continue;
    const size_t b = (size_t)comps[k] * N_ * sizeof(double);
    RVE_HIP(hipMemcpyAsync(p, arrs[k], b, hipMemcpyDeviceToDevice, st_));
    p += (size_t)comps[k] * N_;
  }
  for (int i = 0; i < 9; ++i) {
    snap_host_.Fbar[i] = Fbar_[i];
    snap_host_.Pbar[i] = Pbar_[i];
    snap_host_.dFlast[i] = dFlast_[i];
    snap_host_.dFbar_prev[i] = dFbar_prev_[i];
    snap_host_.dFbar_pp[i] = dFbar_pp_[i];
  }
  snap_host_.s_prev = s_prev_;
  snap_host_.s_pp = s_pp_;
  snap_host_.t = t_;
  snap_host_.increments = increments_;
}

void Engine::restore_snapshot() {
  RVE_SNAP_ARRAYS
  const double* p = snap_;
  for (int k = 0; k < 11; ++k) {
    if (!comps[k]) continue;
    const size_t b = (size_t)comps[k] * N_ * sizeof(double);
    RVE_HIP(hipMemcpyAsync(arrs[k], p, b, hipMemcpyDeviceToDevice, st_));
    p += (size_t)comps[k] * N_;
  }
  RVE_HIP(hipStreamSynchronize(st_));
  for (int i = 0; i < 9; ++i) {
    Fbar_[i] = snap_host_.Fbar[i];
    Pbar_[i] = snap_host_.Pbar[i];
    dFlast_[i] = snap_host_.dFlast[i];
    dFbar_prev_[i] = snap_host_.dFbar_prev[i];
    dFbar_pp_[i] = snap_host_.dFbar_pp[i];
  }
  s_prev_ = snap_host_.s_prev;
  s_pp_ = snap_host_.s_pp;
  t_ = snap_host_.t;
  increments_ = snap_host_.increments;
}
#undef RVE_SNAP_ARRAYS

int Engine::increment_adaptive(const double Fbar_new[9], double dt,
                               int max_cutbacks, int grow_after,
                               rve_adaptive_info* info) {
  if (max_cutbacks < 0 || max_cutbacks > 30 || grow_after < 1)
    throw Error(RVE_EINVAL, "max_cutbacks in [0, 30] and grow_after >= 1");
  const auto t0 = std::chrono::steady_clock::now();
  rve_adaptive_info loc;
  std::memset(&loc, 0, sizeof(loc));
  double F0[9], Fn[9];
  for (int i = 0; i < 9; ++i) {
    F0[i] = Fbar_[i];
    Fn[i] = Fbar_new[i];
  }
  const double hmin = std::ldexp(1.0, -max_cutbacks);
  double done = 0.0, h = 1.0;
  int streak = 0;
  bool snapped = false;
  int status = RVE_OK;
  try {
    while (done < 1.0) {
      h = std::min(h, 1.0 - done);
      const double f = done + h;
      double target[9];
      for (int i = 0; i < 9; ++i)
        target[i] = (f == 1.0) ? Fn[i] : F0[i] + f * (Fn[i] - F0[i]);
      rve_increment_info inc;
      const int st = increment(target, h * dt, &inc);
      loc.last = inc;
      if (st == RVE_OK) {
        ++loc.substeps;
        loc.newton_iters_total += inc.newton_iters;
        loc.cg_iters_total += inc.cg_iters_total;
        if (loc.min_fraction == 0.0 || h < loc.min_fraction) loc.min_fraction = h;
        done = f;
        if (++streak >= grow_after) {
          h *= 2.0;
          streak = 0;
        }
        continue;
      }
      ++loc.cutbacks;
      streak = 0;
      if (!snapped) {
        take_snapshot();   // nothing committed yet: the state of the call
        snapped = true;
      }
      h *= 0.5;
      if (h < hmin) {
        restore_snapshot();
        status = st;
        break;
      }
    }
  } catch (...) {
    if (snapped) restore_snapshot();
    throw;
  }
  loc.status = status;
  loc.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  if (info) *info = loc;
  return status;
}

void Engine::reset_fips() {
  launch_fill_f64(pcyc_, 0.0, N_, st_);
  launch_fill_f64(pcyc_lit_, 0.0, N_, st_);
  launch_fill_f64(wcyc_, 0.0, 12 * N_, st_);
  RVE_HIP(hipGetLastError());
  RVE_HIP(hipStreamSynchronize(st_));
}

size_t Engine::field_bytes(int field) const {
  size_t comps = 0;
  switch (field) {
    case RVE_FIELD_F: case RVE_FIELD_P: case RVE_FIELD_SIGMA:
    case RVE_FIELD_FPINV: comps = 9; break;
    case RVE_FIELD_CHI: case RVE_FIELD_DGAMMA: case RVE_FIELD_WCYC: comps = 12; break;
    case RVE_FIELD_PCYC: case RVE_FIELD_PCYC_LIT: comps = 1; break;
    case RVE_FIELD_STATEV: comps = (size_t)nsv_; break;
    default: throw Error(RVE_EINVAL, "unknown field id");
  }
  return comps * (size_t)N_ * sizeof(double);
}

void Engine::get_field(int field, void* dst, size_t bytes, bool on_device) {
  if (!dst) throw Error(RVE_EINVAL, "null destination");
  const double* src = nullptr;
  size_t need = 0;
  switch (field) {
    case RVE_FIELD_F: src = Fprev_; need = 9; break;
    case RVE_FIELD_P: src = Pc_; need = 9; break;
    case RVE_FIELD_SIGMA:
      launch_cauchy(Fprev_, Pc_, r64_, N_, st_);
      src = r64_;
      need = 9;
      break;
    case RVE_FIELD_FPINV: src = Fpi_c_; need = 9; break;
    case RVE_FIELD_CHI: src = chi_c_; need = 12; break;
    case RVE_FIELD_DGAMMA: src = dg_c_; need = 12; break;
    case RVE_FIELD_STATEV:
      if (!umat_fn_) throw Error(RVE_ESTATE, "no user material set");
      src = sv_c_;
      need = (size_t)nsv_;
      break;
    case RVE_FIELD_PCYC: src = pcyc_; need = 1; break;
    case RVE_FIELD_PCYC_LIT: src = pcyc_lit_; need = 1; break;
    case RVE_FIELD_WCYC: src = wcyc_; need = 12; break;
    default: throw Error(RVE_EINVAL, "unknown field id");
  }
  if (umat_fn_ && (field == RVE_FIELD_FPINV || field == RVE_FIELD_CHI ||
                   field == RVE_FIELD_DGAMMA))
    throw Error(RVE_ESTATE, "crystal-plasticity field requested with a user material");
  need *= N_ * sizeof(double);
  if (bytes < need) throw Error(RVE_EINVAL, "destination too small");
  if (need == 0) return;
  RVE_HIP(hipMemcpyAsync(dst, src, need,
                         on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                         st_));
  RVE_HIP(hipStreamSynchronize(st_));
}

void Engine::get_macro(double out[29]) {
  for (int i = 0; i < 9; ++i) {
    out[i] = Fbar_[i];
    out[9 + i] = Pbar_[i];
  }
  const double J = det3(Fbar_);
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double s = 0.0;
      for (int k = 0; k < 3; ++k) s += Pbar_[3 * i + k] * Fbar_[3 * j + k];
      out[18 + 3 * i + j] = s / J;
    }
  out[27] = t_;
  out[28] = (double)increments_;
}

void Engine::nonlocal_fips(double width, rve_nonlocal_fips* out,
                           double* grain_pcyc, double* grain_pcyc_lit,
                           int32_t labels, double* band_wcyc,
                           int32_t* band_desc, int64_t band_cap) {
  if (!have_micro_) throw Error(RVE_ESTATE, "no microstructure set");
  require_crystal("the non-local indicators");
  if (!fips_.built_for(width)) {
    RVE_HIP(hipStreamSynchronize(st_));
    fips_.build(n_, cfg_.L, phase_host_.data(), table_host_.data(), G_, width,
                [this](size_t b) { return alloc(b); },
                [this](void* p) { release(p); });
  }
  fips_.evaluate(pcyc_, pcyc_lit_, wcyc_, N_, 0, st_, out, grain_pcyc,
                 grain_pcyc_lit, labels, band_wcyc, band_desc, band_cap);
}

size_t Engine::state_size() const {
  return sizeof(StateHeader) + (size_t)(65 + nsv_) * N_ * sizeof(double);
}

void Engine::get_state(void* dst, size_t bytes) {
  if (!dst || bytes < state_size()) throw Error(RVE_EINVAL, "state buffer too small");
  StateHeader h{};
  h.magic = kStateMagic;
  h.n = n_;
  h.increments = increments_;
  h.t = t_;
  for (int i = 0; i < 9; ++i) {
    h.Fbar[i] = Fbar_[i];
    h.Pbar[i] = Pbar_[i];
  }
  char* p = (char*)dst;
  std::memcpy(p, &h, sizeof(h));
  p += sizeof(h);
  const double* arrs[8] = {Fprev_, Pc_, Fpi_c_, chi_c_, dg_c_, pcyc_, pcyc_lit_, wcyc_};
  const int comps[8] = {9, 9, 9, 12, 12, 1, 1, 12};
  for (int k = 0; k < 8; ++k) {
    const size_t b = comps[k] * N_ * sizeof(double);
    RVE_HIP(hipMemcpyAsync(p, arrs[k], b, hipMemcpyDeviceToHost, st_));
    p += b;
  }
  if (nsv_ > 0)
    RVE_HIP(hipMemcpyAsync(p, sv_c_, nsv_ * N_ * sizeof(double),
                           hipMemcpyDeviceToHost, st_));
  RVE_HIP(hipStreamSynchronize(st_));
}

void Engine::set_state(const void* src, size_t bytes) {
  if (!have_micro_) throw Error(RVE_ESTATE, "set the microstructure first");
  if (!src || bytes < state_size()) throw Error(RVE_EINVAL, "state blob too small");
  StateHeader h;
  std::memcpy(&h, src, sizeof(h));
  if (h.magic != kStateMagic || h.n != n_)
    throw Error(RVE_EINVAL, "state blob from another grid or format");
  const char* p = (const char*)src + sizeof(h);
  double* arrs[8] = {Fprev_, Pc_, Fpi_c_, chi_c_, dg_c_, pcyc_, pcyc_lit_, wcyc_};
  const int comps[8] = {9, 9, 9, 12, 12, 1, 1, 12};
  for (int k = 0; k < 8; ++k) {
    const size_t b = comps[k] * N_ * sizeof(double);
    RVE_HIP(hipMemcpyAsync(arrs[k], p, b, hipMemcpyHostToDevice, st_));
    p += b;
  }
  if (nsv_ > 0)
    RVE_HIP(hipMemcpyAsync(sv_c_, p, nsv_ * N_ * sizeof(double),
                           hipMemcpyHostToDevice, st_));
  RVE_HIP(hipStreamSynchronize(st_));
  increments_ = h.increments;
  t_ = h.t;
  for (int i = 0; i < 9; ++i) {
    Fbar_[i] = h.Fbar[i];
    Pbar_[i] = h.Pbar[i];
  }
}

void Engine::apply_G_fp64(const double* in, double* out) {
  SpectralLaunch<double> L;
  L.src = SRC_FIELD;
  L.in_field = in;
  L.spec = (cplx<double>*)spec64_;
  L.tw = (const cplx<double>*)tw64_;
  L.vt = (const double*)vt64_;
  L.dst = DST_NORM;
  L.out_d = out;
  L.partial_inv = partial_inv_;
  launch_G<double>(n_, L, st_);
}

void Engine::debug_apply_G(const double* in, double* out, int precision) {
  if (!in || !out) throw Error(RVE_EINVAL, "null field");
  RVE_HIP(hipMemcpyAsync(r64_, in, 9 * N_ * sizeof(double),
                         hipMemcpyHostToDevice, st_));
  if (precision == RVE_PREC_FP64) {
    apply_G_fp64(r64_, P_);
  } else if (precision == RVE_PREC_MIXED) {
    if (!dbg32_) {
      dbg32_ = alloc(9 * N_ * sizeof(float));
      dbgspec32_ = alloc(9 * N_ / 2 * 2 * sizeof(float));
    }
    launch_convert<float>(r64_, (float*)dbg32_, 9 * N_, st_);
    SpectralLaunch<float> L;
    L.src = SRC_FIELD;
    L.in_field = (const float*)dbg32_;
    L.spec = (cplx<float>*)dbgspec32_;
    L.tw = (const cplx<float>*)tw32_;
    L.vt = (const float*)vt32_;
    L.dst = DST_NORM;
    L.out_d = P_;
    L.partial_inv = partial_inv_;
    launch_G<float>(n_, L, st_);
  } else {
    throw Error(RVE_EINVAL, "unknown precision");
  }
  RVE_HIP(hipGetLastError());
  RVE_HIP(hipMemcpyAsync(out, P_, 9 * N_ * sizeof(double), hipMemcpyDeviceToHost,
                         st_));
  RVE_HIP(hipStreamSynchronize(st_));
}

void Engine::debug_constitutive(const double* F, double dt, double* P, double* K,
                                double* dg, int32_t* fails) {
  if (!have_micro_) throw Error(RVE_ESTATE, "no microstructure set");
  require_crystal("the constitutive test hook");
  if (!F || !(dt > 0)) throw Error(RVE_EINVAL, "null F or dt <= 0");
  RVE_HIP(hipMemcpyAsync(F_, F, 9 * N_ * sizeof(double), hipMemcpyHostToDevice,
                         st_));
  launch_fill_i32(&sc_->fails, 0, 1, st_);
  ConstArgs a{};
  a.F = F_;
  a.Fpi0 = Fpi_c_;
  a.chi0 = chi_c_;
  a.dg0 = nullptr;
  a.phase = phase_;
  a.table = table_;
  a.P = P_;
  a.Fpi = Fpi_t_;
  a.chi = chi_t_;
  a.dg = dg_t_;
  a.fails = &sc_->fails;
  a.lp = law_params(dt);
  a.order = order_;
  a.N = N_;
  launch_return_map(a, st_);
  // the tangent the solver itself forms (FP32 in mixed mode)
  if (K) {
    if (fp64_) tangent<double>(dt); else tangent<float>(dt);
  }
  RVE_HIP(hipGetLastError());
  Scalars h;
  read_scalars(h);
  if (fails) *fails = h.fails;
  if (P)
    RVE_HIP(hipMemcpyAsync(P, P_, 9 * N_ * sizeof(double), hipMemcpyDeviceToHost, st_));
  std::vector<float> K32;
  if (K && fp64_)
    RVE_HIP(hipMemcpyAsync(K, K_, 81 * N_ * sizeof(double),
                           hipMemcpyDeviceToHost, st_));
  if (K && !fp64_) {
    K32.resize(81 * N_);
    RVE_HIP(hipMemcpyAsync(K32.data(), K_, 81 * N_ * sizeof(float),
                           hipMemcpyDeviceToHost, st_));
  }
  if (dg)
    RVE_HIP(hipMemcpyAsync(dg, dg_t_, 12 * N_ * sizeof(double),
                           hipMemcpyDeviceToHost, st_));
  RVE_HIP(hipStreamSynchronize(st_));
  for (size_t i = 0; i < K32.size(); ++i) K[i] = (double)K32[i];
}

void Engine::debug_set_field(int field, const double* src, size_t bytes) {
  double* dst = nullptr;
  size_t need = 0;
  switch (field) {
    case RVE_FIELD_F: dst = Fprev_; need = 9; break;
    case RVE_FIELD_FPINV: dst = Fpi_c_; need = 9; break;
    case RVE_FIELD_CHI: dst = chi_c_; need = 12; break;
    case RVE_FIELD_PCYC: dst = pcyc_; need = 1; break;
    case RVE_FIELD_PCYC_LIT: dst = pcyc_lit_; need = 1; break;
    case RVE_FIELD_WCYC: dst = wcyc_; need = 12; break;
    default: throw Error(RVE_EINVAL, "field cannot be set");
  }
  need *= N_ * sizeof(double);
  if (!src || bytes < need) throw Error(RVE_EINVAL, "source too small");
  RVE_HIP(hipMemcpyAsync(dst, src, need, hipMemcpyHostToDevice, st_));
  RVE_HIP(hipStreamSynchronize(st_));
}

// Kernel classes of the live timing and of bench_kernels:
//   0 pass A (z/y FFT of K:p; under a fused schedule also the direction,
//     the previous x update and K:p)            1 pass B (x FFT, projection)
//   2 pass C (inverse y/z FFT, r -= alpha G(K:p), r.r)
//   3 unused (the vector update rides on classes 2 and 7, or 0)
//   4 return mapping (FP64)                     5 tangent
//   6 FP64 residual G(P) (three passes + reduction)
//   7 direction, previous x update and K:p (unfused schedules)
void Engine::set_timing(uint32_t mask) {
  if (mask == timer_.mask()) return;
  // captured CG graphs hold (or lack) the timing events: capture again
  RVE_HIP(hipStreamSynchronize(st_));
  if (graph_) {
    RVE_HIP(hipGraphExecDestroy(graph_));
    graph_ = nullptr;
  }
  if (graph_def_) {
    RVE_HIP(hipGraphDestroy(graph_def_));
    graph_def_ = nullptr;
  }
  timer_.recycle(graph_pairs_);
  if ((mask >> 4) & 1u) {
    if (!rm_iters_) {
      rm_iters_ = (int32_t*)alloc(N_ * sizeof(int32_t));
      rm_evals_ = (int32_t*)alloc(N_ * sizeof(int32_t));
      rm_stats_ = (unsigned long long*)alloc(4 * sizeof(unsigned long long));
    }
    RVE_HIP(hipMemsetAsync(rm_stats_, 0, 4 * sizeof(unsigned long long), st_));
    RVE_HIP(hipStreamSynchronize(st_));
  }
  timer_.set_mask(mask);
}

// one launch in every `stride` of the CG-iteration classes is timed (direct
// launches; graph-replayed chunks time every launch)
void Engine::set_timing_stride(int stride) {
  if (stride < 1 || stride > 1024) throw Error(RVE_EINVAL, "stride must be in [1, 1024]");
  timer_.set_stride(stride, kCgClasses);
}

void Engine::get_rm_counts(int64_t out[4], bool reset) {
  unsigned long long h[4] = {0, 0, 0, 0};
  if (rm_stats_) {
    RVE_HIP(hipMemcpyAsync(h, rm_stats_, sizeof(h), hipMemcpyDeviceToHost, st_));
    RVE_HIP(hipStreamSynchronize(st_));
    if (reset) {
      RVE_HIP(hipMemsetAsync(rm_stats_, 0, sizeof(h), st_));
      RVE_HIP(hipStreamSynchronize(st_));
    }
  }
  for (int k = 0; k < 4; ++k) out[k] = (int64_t)h[k];
}

void Engine::get_timing(double* ms, int64_t* launches, int count, bool reset,
                        int64_t* seen) {
  if (count < 0) throw Error(RVE_EINVAL, "negative count");
  timer_.read(ms, launches, count, reset, seen);
}

void Engine::bench_kernels(int reps, double* ms, int count) {
  if (!have_micro_ || increments_ < 1)
    throw Error(RVE_ESTATE, "run at least one increment first");
  require_crystal("kernel benchmarking");
  if (reps < 1 || !ms) throw Error(RVE_EINVAL, "bad arguments");
  // these launches are not part of the solver's iteration: keep them out of
  // the live timing
  struct MaskGuard {
    KernelTimer& t;
    uint32_t saved;
    ~MaskGuard() { t.set_mask(saved); }
  } guard{timer_, timer_.mask()};
  timer_.set_mask(0);
  hipEvent_t ev[2];
  RVE_HIP(hipEventCreate(&ev[0]));
  RVE_HIP(hipEventCreate(&ev[1]));
  double out[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  auto timed = [&](int slot, auto&& launch) {
    launch();  // untimed first launch
    RVE_HIP(hipEventRecord(ev[0], st_));
    for (int i = 0; i < reps; ++i) launch();
    RVE_HIP(hipEventRecord(ev[1], st_));
    RVE_HIP(hipEventSynchronize(ev[1]));
    float t = 0.f;
    RVE_HIP(hipEventElapsedTime(&t, ev[0], ev[1]));
    out[slot] = (double)t / reps;
  };
  const double dt = 0.1;
  timed(4, [&] {
    ConstArgs a{};
    a.F = F_;
    a.Fpi0 = Fpi_c_;
    a.chi0 = chi_c_;
    a.dg0 = dg_c_;
    a.phase = phase_;
    a.table = table_;
    a.P = P_;
    a.Fpi = Fpi_t_;
    a.chi = chi_t_;
    a.dg = dg_t_;
    a.fails = &sc_->fails;
    a.lp = law_params(dt);
    a.order = order_;
    a.N = N_;
    launch_return_map(a, st_);
  });
  timed(5, [&] {
    if (fp64_) tangent<double>(dt); else tangent<float>(dt);
  });
  timed(6, [&] { residual_passes(P_); });
  auto passes = [&](auto tag, int mask) {
    using T = decltype(tag);
    const bool dbl = sizeof(T) == sizeof(double);
    SpectralLaunch<T> L;
    if (sched_fused_) {
      L.src = SRC_KP;
      L.K = (const T*)K_;
      L.r = (const T*)r_;
      L.p_old = (const T*)p0_;
      L.x = (T*)x_;
    } else {
      L.src = SRC_FIELD;
      L.in_field = (const T*)Kp_;
    }
    L.p_new = (T*)p1_;
    L.spec = (cplx<T>*)spec_;
    L.tw = (const cplx<T>*)(dbl ? tw64_ : tw32_);
    L.vt = (const T*)(dbl ? vt64_ : vt32_);
    L.dst = DST_CG;
    L.r_io = (T*)r_;
    L.partial_inv = partial_inv_;
    L.sc = sc_;
    L.passes = mask;
    L.cpb = sched_cpb_;
    L.tt = sched_tt_;
    launch_G<T>(n_, L, st_);
  };
  // the CG kernels as a CG run launches them after its first iteration,
  // with alpha = beta = 0 (p = r + 0 p_old, x += 0 p_old, r -= 0 G(y)): the
  // vectors keep their values
  launch_bench_scalars(sc_, st_);
  if (!sched_fused_) timed(7, [&] {
    if (fp64_)
      launch_kp<double>((const double*)K_, (const double*)r_,
                        (const double*)p0_, (double*)p1_, (double*)Kp_, sc_,
                        N_, st_, nullptr, 0, 0, (double*)x_, partial_kp_);
    else
      launch_kp<float>((const float*)K_, (const float*)r_, (const float*)p0_,
                       (float*)p1_, (float*)Kp_, sc_, N_, st_, nullptr, 0, 0,
                       (float*)x_, partial_kp_);
  });
  for (int b = 0; b < 3; ++b) {
    timed(b, [&] {
      if (fp64_) passes(double{}, 1 << b); else passes(float{}, 1 << b);
    });
  }
  RVE_HIP(hipGetLastError());
  RVE_HIP(hipEventDestroy(ev[0]));
  RVE_HIP(hipEventDestroy(ev[1]));
  for (int i = 0; i < count && i < 8; ++i) ms[i] = out[i];
}

void Engine::swap_trial_sets() {
  std::swap(P_, P2_);
  std::swap(Fpi_t_, Fpi_t2_);
  std::swap(chi_t_, chi_t2_);
  std::swap(dg_t_, dg_t2_);
  std::swap(r64_, r64b_);
}

void Engine::attach_net(Net* net) {
  if (net && n_ % 16) throw Error(RVE_EINVAL, "the network needs n divisible by 16");
  if (net && !X0_) {
    X0_ = (uint16_t*)alloc(N_ * kFeat * sizeof(uint16_t));
    Ynet_ = (float*)alloc(N_ * kOut * sizeof(float));
  }
  if (net) second_trial_set();
  net_ = net;
}

// buffers of a candidate predictor evaluated beside the homogeneous one
void Engine::second_trial_set() {
  if (F2_) return;
  const size_t f9 = 9 * N_ * sizeof(double), f12 = 12 * N_ * sizeof(double);
  F2_ = (double*)alloc(f9);
  P2_ = (double*)alloc(f9);
  Fpi_t2_ = (double*)alloc(f9);
  chi_t2_ = (double*)alloc(f12);
  dg_t2_ = (double*)alloc(f12);
  r64b_ = (double*)alloc(f9);
}

void Engine::feature_args(const double Fbar_new[9], FeatArgs& a, double& s_k) {
  double dF[9], s2 = 0.0, dot = 0.0;
  for (int i = 0; i < 9; ++i) {
    dF[i] = Fbar_new[i] - Fbar_[i];
    s2 += dF[i] * dF[i];
    dot += dF[i] * dFbar_prev_[i];
  }
  s_k = std::sqrt(s2);
  a.Fprev = Fprev_;
  a.dFt_prev = dFt_prev_;
  a.dg_prev = dg_c_;
  a.phase = phase_;
  a.table = table_;
  for (int i = 0; i < 9; ++i) {
    a.fbar_prev[i] = Fbar_[i];
    a.dfbar_n[i] = s_k > 0 ? dF[i] / s_k : 0.0;
  }
  a.inv_s_prev = s_prev_ > 0 ? 1.0 / s_prev_ : 0.0;
  a.reversal = (s_k > 0 && s_prev_ > 0) ? dot / (s_k * s_prev_) : 0.0;
  a.N = N_;
}

void Engine::features(const double Fbar_new[9], uint16_t* dst) {
  if (!have_micro_) throw Error(RVE_ESTATE, "no microstructure set");
  require_crystal("the warm-start features");
  if (!dst) throw Error(RVE_EINVAL, "null destination");
  FeatArgs a{};
  double s_k;
  feature_args(Fbar_new, a, s_k);
  a.X = dst;
  nn_features(a, st_);
  RVE_HIP(hipGetLastError());
  RVE_HIP(hipStreamSynchronize(st_));
}

void Engine::target(float* dst) {
  if (increments_ < 1) throw Error(RVE_ESTATE, "no committed increment yet");
  if (!dst) throw Error(RVE_EINVAL, "null destination");
  // the part of the last fluctuation increment that the extrapolation of
  // the one before it (scaled by the load ratio) misses, per |dF_bar|
  double dot = 0.0;
  for (int i = 0; i < 9; ++i) dot += dFbar_prev_[i] * dFbar_pp_[i];
  const double coef = (s_prev_ > 0 && s_pp_ > 0) ? dot / (s_prev_ * s_pp_ * s_pp_) : 0.0;
  nn_target(dFt_prev_, s_prev_ > 0 ? 1.0 / s_prev_ : 0.0, dFt_pp_, coef, dst,
            N_, st_);
  RVE_HIP(hipGetLastError());
  RVE_HIP(hipStreamSynchronize(st_));
}

// F2_ = plain predictor + G(extrapolation + network correction) (projected
// so that it is compatible, periodic and of zero mean)
bool Engine::learned_candidate(const double Fbar_new[9]) {
  if (increments_ < 1) return false;  // no history for the features yet
  FeatArgs a{};
  double s_k;
  feature_args(Fbar_new, a, s_k);
  if (!(s_k > 0)) return false;
  a.X = X0_;
  nn_features(a, st_);
  net_->forward(X0_, n_, Ynet_, st_);
  // the network predicts the correction to the extrapolation c dFt_prev
  // (c = dF_bar : dF_bar_prev / |dF_bar_prev|^2), per |dF_bar|
  nn_output_to_field(Ynet_, s_k, P2_, N_, st_);
  if (s_prev_ > 0) {
    double dot = 0.0;
    for (int i = 0; i < 9; ++i) dot += (Fbar_new[i] - Fbar_[i]) * dFbar_prev_[i];
    nn_axpy_field(P2_, dFt_prev_, dot / (s_prev_ * s_prev_), 9 * N_, st_);
  }
  apply_G_fp64(P2_, r64b_);
  RVE_HIP(hipMemcpyAsync(F2_, F_, 9 * N_ * sizeof(double),
                         hipMemcpyDeviceToDevice, st_));
  nn_axpy_field(F2_, r64b_, 1.0, 9 * N_, st_);
  RVE_HIP(hipGetLastError());
  return true;
}

// F2_ = plain predictor + c G(dFt_prev): the last converged fluctuation
// increment scaled by the load ratio c = (dF_bar : dF_bar_prev) /
// |dF_bar_prev|^2 (the exact predictor of a linear material), the
// zero-cost extrapolation the learned start is measured against
bool Engine::extrapolated_candidate(const double Fbar_new[9]) {
  if (increments_ < 1 || !(s_prev_ > 0)) return false;
  double dot = 0.0;
  for (int i = 0; i < 9; ++i) dot += (Fbar_new[i] - Fbar_[i]) * dFbar_prev_[i];
  const double c = dot / (s_prev_ * s_prev_);
  second_trial_set();
  apply_G_fp64(dFt_prev_, r64b_);
  RVE_HIP(hipMemcpyAsync(F2_, F_, 9 * N_ * sizeof(double),
                         hipMemcpyDeviceToDevice, st_));
  nn_axpy_field(F2_, r64b_, c, 9 * N_, st_);
  RVE_HIP(hipGetLastError());
  return true;
}

}  // namespace rve
