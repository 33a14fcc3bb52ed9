// Batch of RVEs: see batch.hpp.  The increment algorithm is the one of the
// single-RVE engine (Sec. 2.1: predictor, FP64 residual, Newton with CG
// solves of G(K:dF) = -G(P), commit on convergence), run for all RVEs at
// once with per-RVE convergence: an RVE that has converged (or failed)
// leaves the work of the following iterations.
#include "batch.hpp"
#include "newton.hpp"

#include <algorithm>
#include <type_traits>

#include <array>
#include <chrono>
#include <cmath>
#include <cstring>

#include "tables.hpp"

namespace rve {

namespace {
double det3(const double* a) {
  return a[0] * (a[4] * a[8] - a[5] * a[7]) - a[1] * (a[3] * a[8] - a[5] * a[6]) +
         a[2] * (a[3] * a[7] - a[4] * a[6]);
}
}  // namespace

BatchEngine::BatchEngine(const rve_config& cfg, int count, const int32_t* n)
    : cfg_(cfg), B_(count) {
  if (count < 1 || count > 255 || !n)
    throw Error(RVE_EINVAL, "a batch holds 1 to 255 RVEs");
  if (cfg.warm_start) throw Error(RVE_EINVAL, "batches take the homogeneous predictor");
  if (cfg.cg_forcing < 0 || cfg.cg_forcing > 2)
    throw Error(RVE_EINVAL, "cg_forcing must be 0, 1 or 2");
  if (cfg.projection != RVE_PROJ_CONTINUOUS && cfg.projection != RVE_PROJ_DISCRETE)
    throw Error(RVE_EINVAL, "unknown projection operator");
  if (cfg.precision != RVE_PREC_FP64 && cfg.precision != RVE_PREC_MIXED)
    throw Error(RVE_EINVAL, "unknown precision mode");
  if (!(cfg.newton_tol > 0.0) || cfg.newton_max_iter < 0 ||
      cfg.newton_max_iter > RVE_MAX_NEWTON_LOG - 1 || !(cfg.cg_tol > 0.0) ||
      cfg.cg_max_iter < 1 || cfg.cg_chunk < 1)
    throw Error(RVE_EINVAL, "bad tolerance or iteration limits");
  for (int d = 0; d < 3; ++d)
    if (!(cfg.L[d] > 0.0)) throw Error(RVE_EINVAL, "cell lengths must be > 0");
  if ((cfg.dev_alloc == nullptr) != (cfg.dev_free == nullptr))
    throw Error(RVE_EINVAL, "dev_alloc and dev_free must be given together");
  fp64_ = cfg.precision == RVE_PREC_FP64;
  if (cfg_.cg_chunk % 2) cfg_.cg_chunk += 1;
  st_ = (hipStream_t)cfg.stream;
  if (cfg_.use_graph && st_ == nullptr) {
    RVE_HIP(hipStreamCreate(&own_stream_));
    st_ = own_stream_;
  }
  n_.assign(n, n + count);
  off_.resize(B_);
  soff_.resize(B_);
  for (int b = 0; b < B_; ++b) {
    if (!batch_supported(n_[b]))
      throw Error(RVE_EINVAL, "batch grid edges must be in {16,24,32,40,48,64}");
    off_[b] = Nt_;
    soff_[b] = St_;
    const int64_t Nb = (int64_t)n_[b] * n_[b] * n_[b];
    Nt_ += Nb;
    St_ += 9 * Nb / 2;
  }
  const size_t f9 = 9 * Nt_ * sizeof(double), f12 = 12 * Nt_ * sizeof(double),
               f1 = Nt_ * sizeof(double);
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
  dFt_ = (double*)alloc(f9);
  K_ = alloc(81 * Nt_ * tsz);
  x_ = alloc(9 * Nt_ * tsz);
  r_ = alloc(9 * Nt_ * tsz);
  p0_ = alloc(9 * Nt_ * tsz);
  p1_ = alloc(9 * Nt_ * tsz);
  Ap_ = alloc(9 * Nt_ * tsz);
  spec_ = alloc(St_ * 2 * tsz);
  spec64_ = fp64_ ? spec_ : alloc(St_ * 2 * sizeof(double));
  phase_ = (int32_t*)alloc(Nt_ * sizeof(int32_t));
  vrve_ = (uint8_t*)alloc(Nt_);
  sc_ = (Scalars*)alloc(B_ * sizeof(Scalars));
  dF_dev_ = (double*)alloc(B_ * 9 * sizeof(double));
  RVE_HIP(hipHostMalloc((void**)&sc_host_, B_ * sizeof(Scalars), hipHostMallocDefault));
  std::memset(sc_host_, 0, B_ * sizeof(Scalars));

  // per-RVE FFT tables and descriptors
  std::vector<double> tw64, vt64;
  twoff_.resize(B_);
  vtoff_.resize(B_);
  for (int b = 0; b < B_; ++b) {
    twoff_[b] = tw64.size() / 2;
    vtoff_[b] = vt64.size();
    std::vector<double> t = twiddles(n_[b]);
    std::vector<double> v = wave_vectors(n_[b], cfg_.L, cfg_.projection);
    tw64.insert(tw64.end(), t.begin(), t.end());
    vt64.insert(vt64.end(), v.begin(), v.end());
  }
  std::vector<float> tw32(tw64.begin(), tw64.end()), vt32(vt64.begin(), vt64.end());
  tw64_ = alloc(tw64.size() * sizeof(double));
  tw32_ = alloc(tw32.size() * sizeof(float));
  vt64_ = alloc(vt64.size() * sizeof(double));
  vt32_ = alloc(vt32.size() * sizeof(float));
  RVE_HIP(hipMemcpyAsync(tw64_, tw64.data(), tw64.size() * 8, hipMemcpyHostToDevice, st_));
  RVE_HIP(hipMemcpyAsync(tw32_, tw32.data(), tw32.size() * 4, hipMemcpyHostToDevice, st_));
  RVE_HIP(hipMemcpyAsync(vt64_, vt64.data(), vt64.size() * 8, hipMemcpyHostToDevice, st_));
  RVE_HIP(hipMemcpyAsync(vt32_, vt32.data(), vt32.size() * 4, hipMemcpyHostToDevice, st_));

  int64_t psn = 0;
  for (int b = 0; b < B_; ++b) psn += 9 * n_[b];
  psum_ = (double*)alloc(psn * sizeof(double));
  psq_ = (double*)alloc(psn * sizeof(double));
  // partial arenas: pass-C partials per RVE (room for one component per
  // slab block, any schedule), then elementwise partials
  int64_t ppass = 0;
  for (int b = 0; b < B_; ++b) ppass += 9 * n_[b];
  std::vector<SegItem> seg(B_);
  int segb = 0;
  for (int b = 0; b < B_; ++b) {
    const int64_t n9 = 9 * (int64_t)n_[b] * n_[b] * n_[b];
    int nb = (int)((n9 + kBlock * 8 - 1) / (kBlock * 8));
    nb = nb < 1 ? 1 : (nb > 512 ? 512 : nb);
    seg[b].off = off_[b];
    seg[b].n9 = n9;
    seg[b].blk0 = segb;
    seg[b].nblk = nb;
    segb += nb;
  }
  seg_blocks_ = segb;
  partials_ = (double*)alloc((ppass + segb) * sizeof(double));
  std::vector<RedItem> rseg(B_);
  for (int b = 0; b < B_; ++b) {
    seg[b].partial = partials_ + ppass + seg[b].blk0;
    seg[b].sc = sc_ + b;
    rseg[b] = RedItem{seg[b].partial, seg[b].nblk, nullptr, nullptr, 0, 0.0};
  }
  items32_ = alloc(B_ * sizeof(SpecItem<float>));
  items64_ = alloc(B_ * sizeof(SpecItem<double>));
  tune_items_ = alloc(B_ * std::max(sizeof(SpecItem<float>), sizeof(SpecItem<double>)));
  seg_ = (SegItem*)alloc(B_ * sizeof(SegItem));
  red_inv32_ = (RedItem*)alloc(B_ * sizeof(RedItem));
  red_inv64_ = (RedItem*)alloc(B_ * sizeof(RedItem));
  red_seg_ = (RedItem*)alloc(B_ * sizeof(RedItem));
  RVE_HIP(hipMemcpyAsync(seg_, seg.data(), B_ * sizeof(SegItem), hipMemcpyHostToDevice, st_));
  RVE_HIP(hipMemcpyAsync(red_seg_, rseg.data(), B_ * sizeof(RedItem), hipMemcpyHostToDevice, st_));
  std::vector<uint8_t> vr(Nt_);
  for (int b = 0; b < B_; ++b)
    std::memset(vr.data() + off_[b], b, (size_t)n_[b] * n_[b] * n_[b]);
  RVE_HIP(hipMemcpyAsync(vrve_, vr.data(), Nt_, hipMemcpyHostToDevice, st_));
  // the timed matvecs of the schedule tuner read these before the solver
  // writes them: start from zeros
  for (void* f : {K_, r_, p0_, p1_})
    RVE_HIP(hipMemsetAsync(f, 0, (f == K_ ? 81 : 9) * Nt_ * tsz, st_));
  RVE_HIP(hipStreamSynchronize(st_));

  if (cfg_.use_graph) {
    log_ = (BatchLog*)alloc(B_ * sizeof(BatchLog));
    log_host_.resize(B_);
    // grid-barrier words of the persistent CG kernel, then its error flag
    bar_ = (unsigned*)alloc((kBatchBarWords + 1) * sizeof(unsigned));
    launch_fill_i32((int32_t*)bar_, 0, kBatchBarWords + 1, st_);
    RVE_HIP(hipStreamSynchronize(st_));
  }
  build_tables();
  host_phase_.resize(B_);
  host_tables_.resize(B_);
  label_count_.assign(B_, 0);
  have_micro_.assign(B_, false);
  rel_.assign(B_, 0.0);
  label_off_.assign(B_, 0);
  Fbar_.resize(B_);
  Pbar_.resize(B_);
  t_.assign(B_, 0.0);
  increments_.assign(B_, 0);
  for (int b = 0; b < B_; ++b)
    for (int i = 0; i < 9; ++i) {
      Fbar_[b][i] = (i % 4 == 0) ? 1.0 : 0.0;
      Pbar_[b][i] = 0.0;
    }
}

// The descriptor tables of the batched passes for the current schedules:
// per RVE its edge, schedule, first blocks in the slab (A, C) and pencil (B)
// grids, arena offsets, FFT tables, scalars and partials; the per-RVE
// reductions of the pass-C partials; the dynamic LDS and grid sizes.  The
// CG precision's table takes the per-edge schedules (sched_), the other
// (the FP64 residual of a mixed batch) the defaults.
void BatchEngine::build_tables() {
  std::vector<SpecItem<float>> it32(B_);
  std::vector<SpecItem<double>> it64(B_);
  std::vector<RedItem> ri32(B_), ri64(B_);
  int a32 = 0, b32 = 0, a64 = 0, b64 = 0;
  int64_t pp = 0, pso = 0;
  ldsA32_ = ldsB32_ = ldsA64_ = ldsB64_ = 0;
  cpbs32_ = cpbs64_ = 0;
  for (int b = 0; b < B_; ++b) {
    const int nb = n_[b];
    const int64_t Nb = (int64_t)nb * nb * nb;
    auto fill = [&](auto& it, int& accA, int& accB, bool dbl, size_t& la,
                    size_t& lb, RedItem& ri, int& cpbs) {
      using T = std::remove_reference_t<decltype(it.tw[0].x)>;
      int cpb = 0, tt = 0;
      default_schedule(nb, dbl, cpb, tt);
      if (dbl == fp64_) {
        auto f = sched_.find(nb);
        if (f != sched_.end() && f->second[0]) {
          cpb = f->second[0];
          tt = f->second[1];
        }
      }
      const int sA = slab_blocks(nb, dbl, cpb);
      cpbs |= cpb == 3 ? 2 : 1;
      it.n = nb;
      it.cpb = cpb;
      it.tt = tt;
      it.blk[0] = accA;
      it.blk[1] = accB;
      it.off = off_[b];
      it.soff = soff_[b];
      it.sc = sc_ + b;
      it.partial = partials_ + pp;
      it.psum = psum_ + pso;
      it.psq = psq_ + pso;
      it.tw = (const cplx<T>*)(dbl ? tw64_ : tw32_) + twoff_[b];
      it.vt = (const T*)(dbl ? vt64_ : vt32_) + vtoff_[b];
      accA += sA;
      accB += pencil_blocks(nb, dbl, tt);
      size_t s1, s2;
      batch_lds<T>(nb, cpb, tt, s1, s2);
      la = std::max(la, s1);
      lb = std::max(lb, s2);
      ri = RedItem{partials_ + pp, sA, psum_ + pso, psq_ + pso, nb,
                   1.0 / (double)Nb};
    };
    fill(it32[b], a32, b32, false, ldsA32_, ldsB32_, ri32[b], cpbs32_);
    fill(it64[b], a64, b64, true, ldsA64_, ldsB64_, ri64[b], cpbs64_);
    pp += 9 * nb;
    pso += 9 * nb;
  }
  if (ldsA32_ > 65536 || ldsB32_ > 65536) batch_allow_lds<float>(ldsA32_, ldsB32_);
  if (ldsA64_ > 65536 || ldsB64_ > 65536) batch_allow_lds<double>(ldsA64_, ldsB64_);
  blocksA32_ = a32;
  blocksB32_ = b32;
  blocksA64_ = a64;
  blocksB64_ = b64;
  host_it32_ = it32;
  host_it64_ = it64;
  RVE_HIP(hipMemcpyAsync(items32_, it32.data(), B_ * sizeof(SpecItem<float>), hipMemcpyHostToDevice, st_));
  RVE_HIP(hipMemcpyAsync(items64_, it64.data(), B_ * sizeof(SpecItem<double>), hipMemcpyHostToDevice, st_));
  RVE_HIP(hipMemcpyAsync(red_inv32_, ri32.data(), B_ * sizeof(RedItem), hipMemcpyHostToDevice, st_));
  RVE_HIP(hipMemcpyAsync(red_inv64_, ri64.data(), B_ * sizeof(RedItem), hipMemcpyHostToDevice, st_));
  if (cfg_.use_graph) {
    persist_lds_ = fp64_ ? std::max(ldsA64_, ldsB64_) : std::max(ldsA32_, ldsB32_);
    persist_grid_ = fp64_ ? cg_batch_persistent_grid<double>(persist_lds_)
                          : cg_batch_persistent_grid<float>(persist_lds_);
  }
  // a captured increment holds the old tables' grid sizes
  if (inc_graph_) {
    RVE_HIP(hipGraphExecDestroy(inc_graph_));
    inc_graph_ = nullptr;
  }
  if (inc_graph_def_) {
    RVE_HIP(hipGraphDestroy(inc_graph_def_));
    inc_graph_def_ = nullptr;
  }
  inc_graph_dt_ = -1.0;
  RVE_HIP(hipStreamSynchronize(st_));
}

// Per grid edge of the batch (edges with a forced schedule excepted), the
// fastest schedule of the CG matvec G(K : p) (components per slab block,
// kz columns per pencil block): every valid candidate times one matvec of
// this edge's RVEs alone, through the batched passes, with every RVE
// active and beta = 0 (p = r + 0 p_old: the traffic of an iteration after
// the first); three interleaved rounds, the best of each.  The scalars are
// restored afterwards; the passes overwrite only the direction, the
// spectrum, G(K:p) and the partials, all rewritten by the next solve.
template <typename T>
void BatchEngine::autotune() {
  const bool dbl = sizeof(T) == sizeof(double);
  read_scalars();
  std::vector<Scalars> saved(sc_host_, sc_host_ + B_);
  for (int b = 0; b < B_; ++b) {
    sc_host_[b].done = 0;
    sc_host_[b].inactive = 0;
    sc_host_[b].first = 0;
    sc_host_[b].beta = 0.0;
  }
  upload_scalars();
  const std::vector<SpecItem<T>>& full =
      *reinterpret_cast<const std::vector<SpecItem<T>>*>(dbl ? (const void*)&host_it64_
                                                             : (const void*)&host_it32_);
  hipEvent_t ev[2];
  RVE_HIP(hipEventCreate(&ev[0]));
  RVE_HIP(hipEventCreate(&ev[1]));
  std::vector<int> edges(n_);
  std::sort(edges.begin(), edges.end());
  edges.erase(std::unique(edges.begin(), edges.end()), edges.end());
  for (int e : edges) {
    if (forced_.count(e)) continue;
    struct Cand {
      int cpb, tt;
      std::vector<SpecItem<T>> items;
      int bA, bB;
      size_t lA, lB;
    };
    std::vector<Cand> cand;
    for (int cpb : {1, 3})
      for (int tt : {4, 8, 16}) {
        if (!schedule_valid(e, dbl, cpb, tt)) continue;
        Cand c{cpb, tt, {}, 0, 0, 0, 0};
        for (int b = 0; b < B_; ++b) {
          if (n_[b] != e) continue;
          SpecItem<T> it = full[b];
          it.cpb = cpb;
          it.tt = tt;
          it.blk[0] = c.bA;
          it.blk[1] = c.bB;
          c.bA += slab_blocks(e, dbl, cpb);
          c.bB += pencil_blocks(e, dbl, tt);
          c.items.push_back(it);
        }
        batch_lds<T>(e, cpb, tt, c.lA, c.lB);
        if (c.lA > 65536 || c.lB > 65536) batch_allow_lds<T>(c.lA, c.lB);
        cand.push_back(std::move(c));
      }
    std::vector<float> best(cand.size(), 0.f);
    constexpr int reps = 4;
    for (int round = 0; round < 3; ++round)
      for (size_t c = 0; c < cand.size(); ++c) {
        RVE_HIP(hipMemcpyAsync(tune_items_, cand[c].items.data(),
                               cand[c].items.size() * sizeof(SpecItem<T>),
                               hipMemcpyHostToDevice, st_));
        BatchSpec<T> bs = spec<T>(true, 0);
        bs.items = (const SpecItem<T>*)tune_items_;
        bs.nitems = (int)cand[c].items.size();
        bs.cpbs = cand[c].cpb == 3 ? 2 : 1;
        auto matvec = [&] {
          launch_G_batch<T>(bs, SRC_KP, (T*)Ap_, nullptr, cand[c].bA,
                            cand[c].bB, cand[c].lA, cand[c].lB, st_);
        };
        matvec();  // untimed first launch
        RVE_HIP(hipEventRecord(ev[0], st_));
        for (int i = 0; i < reps; ++i) matvec();
        RVE_HIP(hipEventRecord(ev[1], st_));
        RVE_HIP(hipEventSynchronize(ev[1]));
        float t = 0.f;
        RVE_HIP(hipEventElapsedTime(&t, ev[0], ev[1]));
        if (round == 0 || t < best[c]) best[c] = t;
      }
    size_t bi = 0;
    for (size_t c = 1; c < cand.size(); ++c)
      if (best[c] < best[bi]) bi = c;
    if (cand.empty()) throw Error(RVE_EINVAL, "no FFT schedule for a batch edge");
    sched_[e] = {cand[bi].cpb, cand[bi].tt};
    sched_ms_[e] = best[bi] / reps;
  }
  RVE_HIP(hipGetLastError());
  hipEventDestroy(ev[0]);
  hipEventDestroy(ev[1]);
  std::copy(saved.begin(), saved.end(), sc_host_);
  upload_scalars();
  build_tables();
}

void BatchEngine::tune() {
  RVE_HIP(hipStreamSynchronize(st_));
  if (fp64_) autotune<double>(); else autotune<float>();
  tuned_ = true;
}

void BatchEngine::ensure_tuned() {
  if (!tuned_) tune();
}

void BatchEngine::set_schedule(int edge, int cpb, int tt) {
  if (std::find(n_.begin(), n_.end(), edge) == n_.end())
    throw Error(RVE_EINVAL, "no RVE of this grid edge in the batch");
  if (cpb || tt) {
    if (!schedule_valid(edge, fp64_, cpb, tt))
      throw Error(RVE_EINVAL, "no such FFT schedule for this grid edge and precision");
    RVE_HIP(hipStreamSynchronize(st_));
    sched_[edge] = {cpb, tt};
    sched_ms_[edge] = 0.0;
    forced_.insert(edge);
  } else {
    // tune this edge again (with the others) at the next solve
    RVE_HIP(hipStreamSynchronize(st_));
    sched_.erase(edge);
    sched_ms_.erase(edge);
    forced_.erase(edge);
    tuned_ = false;
  }
  build_tables();
}

void BatchEngine::get_schedule(int edge, int out[2], double* ms) const {
  if (std::find(n_.begin(), n_.end(), edge) == n_.end())
    throw Error(RVE_EINVAL, "no RVE of this grid edge in the batch");
  for (int b = 0; b < B_; ++b)
    if (n_[b] == edge) {
      out[0] = fp64_ ? host_it64_[b].cpb : host_it32_[b].cpb;
      out[1] = fp64_ ? host_it64_[b].tt : host_it32_[b].tt;
      break;
    }
  if (ms) {
    auto f = sched_ms_.find(edge);
    *ms = f == sched_ms_.end() ? 0.0 : f->second;
  }
}

BatchEngine::~BatchEngine() {
  if (inc_graph_) hipGraphExecDestroy(inc_graph_);
  if (inc_graph_def_) hipGraphDestroy(inc_graph_def_);
  if (st_) hipStreamSynchronize(st_);
  for (auto& a : allocs_) {
    if (cfg_.dev_free)
      cfg_.dev_free(a.first, cfg_.alloc_ctx);
    else
      hipFree(a.first);
  }
  if (sc_host_) hipHostFree(sc_host_);
  if (own_stream_) hipStreamDestroy(own_stream_);
}

void* BatchEngine::alloc(size_t bytes) {
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

void BatchEngine::release(void* p) {
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

void BatchEngine::nonlocal_fips(int b, double width, rve_nonlocal_fips* out,
                                double* grain_pcyc, double* grain_pcyc_lit,
                                int32_t labels, double* band_wcyc,
                                int32_t* band_desc, int64_t band_cap) {
  if (b < 0 || b >= B_) throw Error(RVE_EINVAL, "RVE index out of range");
  if (!have_micro_[b]) throw Error(RVE_ESTATE, "no microstructure set");
  if ((int)fips_.size() != B_) fips_.resize(B_);
  if (!fips_[b].built_for(width)) {
    RVE_HIP(hipStreamSynchronize(st_));
    fips_[b].build(n_[b], cfg_.L, host_phase_[b].data(),
                   host_tables_[b].data(), label_count_[b], width,
                   [this](size_t s) { return alloc(s); },
                   [this](void* p) { release(p); });
  }
  fips_[b].evaluate(pcyc_, pcyc_lit_, wcyc_, Nt_, off_[b], st_, out, grain_pcyc,
                    grain_pcyc_lit, labels, band_wcyc, band_desc, band_cap);
}

void BatchEngine::set_microstructure(int b, const int32_t* phase, int32_t G,
                                     const double* quat, const int32_t* law,
                                     const double* params, int32_t nparams) {
  if (b < 0 || b >= B_) throw Error(RVE_EINVAL, "RVE index out of range");
  if (!phase || !quat || !law || !params || G < 1)
    throw Error(RVE_EINVAL, "null microstructure input or G < 1");
  if (nparams < RVE_NPARAMS) throw Error(RVE_EINVAL, "nparams < RVE_NPARAMS");
  const int64_t Nb = (int64_t)n_[b] * n_[b] * n_[b];
  for (int64_t v = 0; v < Nb; ++v)
    if (phase[v] < 0 || phase[v] >= G) throw Error(RVE_EINVAL, "phase label out of [0, G)");
  for (int g = 0; g < G; ++g) {
    if (law[g] != 0 && law[g] != 1) throw Error(RVE_EINVAL, "unknown law id");
    const double q2 = quat[4 * g] * quat[4 * g] + quat[4 * g + 1] * quat[4 * g + 1] +
                      quat[4 * g + 2] * quat[4 * g + 2] + quat[4 * g + 3] * quat[4 * g + 3];
    if (!(std::fabs(q2 - 1.0) < 1e-6)) throw Error(RVE_EINVAL, "quaternion not unit");
  }
  if (have_params_) {
    for (int i = 0; i < RVE_NPARAMS; ++i)
      if (params[i] != params_[i])
        throw Error(RVE_EINVAL, "all RVEs of a batch share the material constants");
  } else {
    for (int i = 0; i < RVE_NPARAMS; ++i) params_[i] = params[i];
    have_params_ = true;
  }
  // the label table concatenates the RVEs' tables: labels of RVE k start
  // at label_off_[k]
  host_tables_[b] = label_table(G, quat, law, params_);
  label_count_[b] = G;
  std::vector<double> all;
  int off = 0;
  for (int k = 0; k < B_; ++k) {
    label_off_[k] = off;
    all.insert(all.end(), host_tables_[k].begin(), host_tables_[k].end());
    off += label_count_[k];
  }
  if (off > table_labels_) {
    table_ = (double*)alloc((size_t)off * kTableStride * sizeof(double));
    table_labels_ = off;
  }
  RVE_HIP(hipMemcpyAsync(table_, all.data(), all.size() * sizeof(double),
                         hipMemcpyHostToDevice, st_));
  host_phase_[b].assign(phase, phase + Nb);
  have_micro_[b] = true;
  if ((int)fips_.size() != B_) fips_.resize(B_);
  fips_[b].invalidate();
  // phases of every RVE with its label offset
  std::vector<int32_t> ph(Nt_, 0);
  for (int k = 0; k < B_; ++k) {
    if (!have_micro_[k]) continue;
    for (int64_t v = 0; v < (int64_t)host_phase_[k].size(); ++v)
      ph[off_[k] + v] = host_phase_[k][v] + label_off_[k];
  }
  RVE_HIP(hipMemcpyAsync(phase_, ph.data(), Nt_ * sizeof(int32_t),
                         hipMemcpyHostToDevice, st_));
  // reset this RVE's state
  std::vector<double> eye(Nb), zero(Nb, 0.0);
  for (int c = 0; c < 9; ++c) {
    const double val = (c % 4 == 0) ? 1.0 : 0.0;
    std::fill(eye.begin(), eye.end(), val);
    RVE_HIP(hipMemcpyAsync(Fprev_ + c * Nt_ + off_[b], eye.data(), Nb * 8, hipMemcpyHostToDevice, st_));
    RVE_HIP(hipMemcpyAsync(Fpi_c_ + c * Nt_ + off_[b], eye.data(), Nb * 8, hipMemcpyHostToDevice, st_));
    RVE_HIP(hipMemcpyAsync(Pc_ + c * Nt_ + off_[b], zero.data(), Nb * 8, hipMemcpyHostToDevice, st_));
    RVE_HIP(hipMemcpyAsync(dFt_ + c * Nt_ + off_[b], zero.data(), Nb * 8, hipMemcpyHostToDevice, st_));
  }
  for (int c = 0; c < 12; ++c) {
    RVE_HIP(hipMemcpyAsync(chi_c_ + c * Nt_ + off_[b], zero.data(), Nb * 8, hipMemcpyHostToDevice, st_));
    RVE_HIP(hipMemcpyAsync(dg_c_ + c * Nt_ + off_[b], zero.data(), Nb * 8, hipMemcpyHostToDevice, st_));
    RVE_HIP(hipMemcpyAsync(wcyc_ + c * Nt_ + off_[b], zero.data(), Nb * 8, hipMemcpyHostToDevice, st_));
  }
  RVE_HIP(hipMemcpyAsync(pcyc_ + off_[b], zero.data(), Nb * 8, hipMemcpyHostToDevice, st_));
  RVE_HIP(hipMemcpyAsync(pcyc_lit_ + off_[b], zero.data(), Nb * 8, hipMemcpyHostToDevice, st_));
  RVE_HIP(hipStreamSynchronize(st_));
  for (int i = 0; i < 9; ++i) {
    Fbar_[b][i] = (i % 4 == 0) ? 1.0 : 0.0;
    Pbar_[b][i] = 0.0;
  }
  t_[b] = 0.0;
  increments_[b] = 0;
}

void BatchEngine::upload_scalars() {
  RVE_HIP(hipMemcpyAsync(sc_, sc_host_, B_ * sizeof(Scalars), hipMemcpyHostToDevice, st_));
}

void BatchEngine::read_scalars() {
  RVE_HIP(hipMemcpyAsync(sc_host_, sc_, B_ * sizeof(Scalars), hipMemcpyDeviceToHost, st_));
  RVE_HIP(hipStreamSynchronize(st_));
}

template <typename T>
BatchSpec<T> BatchEngine::spec(bool cg, int parity) const {
  BatchSpec<T> b{};
  const bool dbl = sizeof(T) == sizeof(double);
  b.items = (const SpecItem<T>*)(dbl ? items64_ : items32_);
  b.nitems = B_;
  b.cpbs = dbl ? cpbs64_ : cpbs32_;
  b.cs = Nt_;
  if (cg) {
    b.K = (const T*)K_;
    b.r = (const T*)r_;
    b.p_old = (const T*)(parity ? p1_ : p0_);
    b.p_new = (T*)(parity ? p0_ : p1_);
    b.spec = (cplx<T>*)spec_;
  } else {
    b.field = (const T*)P_;
    b.spec = (cplx<T>*)spec64_;
  }
  return b;
}

template <typename T>
void BatchEngine::cg_iteration(int parity) {
  const bool dbl = sizeof(T) == sizeof(double);
  BatchSpec<T> b = spec<T>(true, parity);
  launch_G_batch<T>(b, SRC_KP, (T*)Ap_, nullptr, dbl ? blocksA64_ : blocksA32_,
                    dbl ? blocksB64_ : blocksB32_, dbl ? ldsA64_ : ldsA32_,
                    dbl ? ldsB64_ : ldsB32_, st_);
  launch_reduce_batch(RED_ALPHA, dbl ? red_inv64_ : red_inv32_, B_, sc_, st_);
  launch_cg_update_batch<T>(seg_, B_, seg_blocks_, Nt_, (T*)x_, (T*)r_,
                            (const T*)b.p_new, (const T*)Ap_, st_);
  launch_reduce_batch(RED_BETA, red_seg_, B_, sc_, st_);
}

template <typename T>
void BatchEngine::cg_solve(std::vector<int>& iters) {
  for (int b = 0; b < B_; ++b) {
    // per-RVE linear-solve tolerance (cg_forcing: as tight as the
    // equilibrium tolerance needs from this RVE's residual)
    const double eta = forcing_eta(cfg_.cg_forcing, cfg_.cg_tol,
                                   cfg_.newton_tol, rel_[b]);
    sc_host_[b].max_iters = cfg_.cg_max_iter;
    sc_host_[b].eta2bb = eta * eta;
    sc_host_[b].done = sc_host_[b].inactive;
  }
  upload_scalars();
  launch_cg_init_batch<T>(seg_, B_, seg_blocks_, Nt_, r64_, (T*)r_, (T*)x_, st_);
  launch_reduce_batch(RED_INIT, red_seg_, B_, sc_, st_);
  RVE_HIP(hipGetLastError());
  int parity = 0;
  for (;;) {
    for (int j = 0; j < cfg_.cg_chunk; ++j) {
      cg_iteration<T>(parity);
      parity ^= 1;
    }
    RVE_HIP(hipGetLastError());
    read_scalars();
    bool all = true;
    for (int b = 0; b < B_; ++b) all = all && sc_host_[b].done;
    if (all) break;
  }
  for (int b = 0; b < B_; ++b) iters[b] = sc_host_[b].inactive ? 0 : sc_host_[b].iters;
}

int BatchEngine::increment(const double* Fbar_all, double dt,
                           rve_increment_info* info) {
  for (int b = 0; b < B_; ++b)
    if (!have_micro_[b]) throw Error(RVE_ESTATE, "every RVE needs a microstructure");
  ensure_tuned();
  if (cfg_.use_graph) return increment_device(Fbar_all, dt, info);
  if (!(dt > 0.0) || !std::isfinite(dt)) throw Error(RVE_EINVAL, "dt must be > 0");
  for (int b = 0; b < B_; ++b) {
    const double* Fb = Fbar_all + 9 * b;
    for (int i = 0; i < 9; ++i)
      if (!std::isfinite(Fb[i])) throw Error(RVE_EINVAL, "non-finite F_bar");
    if (!(det3(Fb) > 0.0)) throw Error(RVE_EINVAL, "det(F_bar) must be > 0");
  }
  const auto t0 = std::chrono::steady_clock::now();
  std::vector<rve_increment_info> loc(B_);
  std::memset(loc.data(), 0, B_ * sizeof(rve_increment_info));
  std::vector<double> dF(9 * B_);
  for (int b = 0; b < B_; ++b)
    for (int i = 0; i < 9; ++i) dF[9 * b + i] = Fbar_all[9 * b + i] - Fbar_[b][i];
  RVE_HIP(hipMemcpyAsync(dF_dev_, dF.data(), 9 * B_ * sizeof(double),
                         hipMemcpyHostToDevice, st_));
  launch_predict_batch(F_, Fprev_, vrve_, dF_dev_, Nt_, st_);
  std::vector<int> status(B_, 1);  // 1 = running
  for (int b = 0; b < B_; ++b) {
    sc_host_[b].inactive = 0;
    sc_host_[b].commit = 0;
  }
  LawParams lp{params_[3], params_[4], params_[5], params_[6], params_[7], dt,
               1.0 / params_[4], 1.0 / (dt * params_[3])};
  lp.nint = flow_exponent_int(lp.nexp);
  const double* dg_start = dg_c_;
  std::vector<int> iters(B_, 0);
  for (int it = 0; it <= cfg_.newton_max_iter; ++it) {
    for (int b = 0; b < B_; ++b) sc_host_[b].fails = 0;
    upload_scalars();
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
    a.fails = nullptr;
    a.lp = lp;
    a.N = Nt_;
    a.vrve = vrve_;
    a.scs = sc_;
    launch_return_map(a, st_);
    BatchSpec<double> rs = spec<double>(false, 0);
    launch_G_batch<double>(rs, SRC_FIELD, nullptr, r64_, blocksA64_, blocksB64_,
                           ldsA64_, ldsB64_, st_);
    launch_reduce_batch(RED_RESID, red_inv64_, B_, sc_, st_);
    RVE_HIP(hipGetLastError());
    read_scalars();
    bool any = false;
    for (int b = 0; b < B_; ++b) {
      if (status[b] != 1) continue;
      Scalars& h = sc_host_[b];
      const double res = std::sqrt(h.res2), pn = std::sqrt(h.P2);
      const double rel = pn > 0 ? res / pn : 0.0;
      rel_[b] = rel;
      if (it < RVE_MAX_NEWTON_LOG) loc[b].residual_history[it] = rel;
      if (it == 0) loc[b].predictor_residual = loc[b].plain_predictor_residual = rel;
      loc[b].residual_rel = rel;
      for (int i = 0; i < 9; ++i) loc[b].P_bar[i] = h.pbar[i];
      loc[b].newton_iters = it;
      if (h.fails > 0) {
        loc[b].local_failures = h.fails;
        status[b] = RVE_ELOCAL;
      } else if (res <= cfg_.newton_tol * pn) {
        status[b] = RVE_OK;
        h.commit = 1;
      } else if (it == cfg_.newton_max_iter) {
        status[b] = RVE_ENOTCONV;
      }
      if (status[b] != 1) h.inactive = 1;
      any = any || status[b] == 1;
    }
    if (!any) break;
    upload_scalars();
    if (fp64_) {
      TangentArgs<double> t{F_, Fpi_c_, chi_c_, dg_t_, phase_, table_, (double*)K_, lp, Nt_, vrve_, sc_};
      launch_tangent<double>(t, st_);
      cg_solve<double>(iters);
      launch_add_to_F<double>(F_, (const double*)x_, 9 * Nt_, st_);
    } else {
      TangentArgs<float> t{F_, Fpi_c_, chi_c_, dg_t_, phase_, table_, (float*)K_, lp, Nt_, vrve_, sc_};
      launch_tangent<float>(t, st_);
      cg_solve<float>(iters);
      launch_add_to_F<float>(F_, (const float*)x_, 9 * Nt_, st_);
    }
    RVE_HIP(hipGetLastError());
    for (int b = 0; b < B_; ++b) {
      if (status[b] != 1) continue;
      if (it < RVE_MAX_NEWTON_LOG) loc[b].cg_iters[it] = iters[b];
      loc[b].cg_iters_total += iters[b];
      loc[b].cg_breakdowns += sc_host_[b].breakdown ? 1 : 0;
    }
    dg_start = dg_t_;
  }
  // commit the converged RVEs
  upload_scalars();
  CommitBatchArgs c{};
  c.vrve = vrve_;
  c.scs = sc_;
  c.dF = dF_dev_;
  c.F = F_;
  c.P = P_;
  c.Fpi_t = Fpi_t_;
  c.chi_t = chi_t_;
  c.dg_t = dg_t_;
  c.Fprev = Fprev_;
  c.Pc = Pc_;
  c.Fpi_c = Fpi_c_;
  c.chi_c = chi_c_;
  c.dg_c = dg_c_;
  c.dFt = dFt_;
  c.phase = phase_;
  c.table = table_;
  c.pcyc = pcyc_;
  c.pcyc_lit = pcyc_lit_;
  c.wcyc = wcyc_;
  c.dt = dt;
  c.N = Nt_;
  launch_commit_batch(c, st_);
  RVE_HIP(hipGetLastError());
  RVE_HIP(hipStreamSynchronize(st_));
  const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  int first_bad = RVE_OK;
  for (int b = 0; b < B_; ++b) {
    if (status[b] == 1) status[b] = RVE_ENOTCONV;
    const double* Fbar_new = Fbar_all + 9 * b;
    const double J = det3(Fbar_new);
    loc[b].status = status[b];
    loc[b].seconds = secs;
    if (status[b] == RVE_OK) {
      for (int i = 0; i < 9; ++i) {
        Fbar_[b][i] = Fbar_new[i];
        Pbar_[b][i] = loc[b].P_bar[i];
      }
      t_[b] += dt;
      ++increments_[b];
    } else if (first_bad == RVE_OK) {
      first_bad = status[b];
    }
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        double s = 0.0;
        for (int k = 0; k < 3; ++k) s += loc[b].P_bar[3 * i + k] * Fbar_new[3 * j + k];
        loc[b].sigma_bar[3 * i + j] = s / J;
      }
    if (info) info[b] = loc[b];
  }
  return first_bad;
}

// ---------------------------------------------- device-controlled increment
// One Newton iteration's evaluation: return mapping at the committed state
// (slips from dg_start), FP64 residual G(P) and norms, the device decision.
void BatchEngine::newton_eval_device(int it, const LawParams& lp,
                                     const double* dg_start) {
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
  a.fails = nullptr;
  a.lp = lp;
  a.N = Nt_;
  a.vrve = vrve_;
  a.scs = sc_;
  launch_return_map(a, st_);
  BatchSpec<double> rs = spec<double>(false, 0);
  launch_G_batch<double>(rs, SRC_FIELD, nullptr, r64_, blocksA64_, blocksB64_,
                         ldsA64_, ldsB64_, st_);
  launch_reduce_batch(RED_RESID, red_inv64_, B_, sc_, st_);
  NewtonCtl ctl{cfg_.newton_tol, cfg_.cg_tol, cfg_.newton_max_iter,
                cfg_.cg_max_iter, cfg_.cg_forcing};
  launch_newton_control_batch(sc_, log_, B_, it, ctl, st_);
}

// One Newton iteration's linear solve: tangent, CG of every running RVE in
// one persistent launch, F += dF.
template <typename T>
void BatchEngine::newton_solve_device(int it, const LawParams& lp) {
  (void)it;
  const bool dbl = sizeof(T) == sizeof(double);
  TangentArgs<T> t{F_, Fpi_c_, chi_c_, dg_t_, phase_, table_, (T*)K_, lp, Nt_,
                   vrve_, sc_};
  launch_tangent<T>(t, st_);
  launch_cg_init_batch<T>(seg_, B_, seg_blocks_, Nt_, r64_, (T*)r_, (T*)x_, st_);
  launch_reduce_batch(RED_INIT, red_seg_, B_, sc_, st_);
  BatchCG<T> c{};
  c.even = spec<T>(true, 0);
  c.odd = spec<T>(true, 1);
  c.seg = seg_;
  c.seg_blocks = seg_blocks_;
  c.red_inv = dbl ? red_inv64_ : red_inv32_;
  c.red_seg = red_seg_;
  c.scs = sc_;
  c.nitems = B_;
  c.blocksA = dbl ? blocksA64_ : blocksA32_;
  c.blocksB = dbl ? blocksB64_ : blocksB32_;
  c.cs = Nt_;
  c.x = (T*)x_;
  c.r = (T*)r_;
  c.Ap = (T*)Ap_;
  c.max_iters = cfg_.cg_max_iter + 1;
  c.bar = bar_;
  c.err = (int*)(bar_ + kBatchBarWords);
  // arrival counts to zero (the generation may keep its value; the flag too)
  launch_fill_i32((int32_t*)bar_ + 1, 0, kBatchBarWords - 1, st_);
  launch_cg_batch_persistent<T>(c, persist_grid_, persist_lds_, st_);
  launch_add_to_F<T>(F_, (const T*)x_, 9 * Nt_, st_);
}

void BatchEngine::read_logs() {
  RVE_HIP(hipMemcpyAsync(log_host_.data(), log_, B_ * sizeof(BatchLog),
                         hipMemcpyDeviceToHost, st_));
  RVE_HIP(hipStreamSynchronize(st_));
}

int BatchEngine::increment_device(const double* Fbar_all, double dt,
                                  rve_increment_info* info) {
  if (!(dt > 0.0) || !std::isfinite(dt)) throw Error(RVE_EINVAL, "dt must be > 0");
  for (int b = 0; b < B_; ++b) {
    const double* Fb = Fbar_all + 9 * b;
    for (int i = 0; i < 9; ++i)
      if (!std::isfinite(Fb[i])) throw Error(RVE_EINVAL, "non-finite F_bar");
    if (!(det3(Fb) > 0.0)) throw Error(RVE_EINVAL, "det(F_bar) must be > 0");
  }
  const auto t0 = std::chrono::steady_clock::now();
  std::vector<double> dF(9 * B_);
  for (int b = 0; b < B_; ++b)
    for (int i = 0; i < 9; ++i) dF[i + 9 * b] = Fbar_all[9 * b + i] - Fbar_[b][i];
  RVE_HIP(hipMemcpyAsync(dF_dev_, dF.data(), 9 * B_ * sizeof(double),
                         hipMemcpyHostToDevice, st_));
  for (int b = 0; b < B_; ++b) {
    sc_host_[b].inactive = 0;
    sc_host_[b].commit = 0;
    sc_host_[b].fails = 0;
    sc_host_[b].done = 0;
    std::memset(&log_host_[b], 0, sizeof(BatchLog));
    log_host_[b].status = 1;
  }
  upload_scalars();
  RVE_HIP(hipMemcpyAsync(log_, log_host_.data(), B_ * sizeof(BatchLog),
                         hipMemcpyHostToDevice, st_));
  LawParams lp{params_[3], params_[4], params_[5], params_[6], params_[7], dt,
               1.0 / params_[4], 1.0 / (dt * params_[3])};
  lp.nint = flow_exponent_int(lp.nexp);
  const int ncap = std::min(kGraphNewton, cfg_.newton_max_iter);
  auto solve = [&](int it) {
    if (fp64_) newton_solve_device<double>(it, lp);
    else newton_solve_device<float>(it, lp);
  };
  // the predictor and Newton iterations 0..ncap, captured once per dt
  if (!inc_graph_ || inc_graph_dt_ != dt) {
    if (inc_graph_) RVE_HIP(hipGraphExecDestroy(inc_graph_));
    if (inc_graph_def_) RVE_HIP(hipGraphDestroy(inc_graph_def_));
    inc_graph_ = nullptr;
    inc_graph_def_ = nullptr;
    RVE_HIP(hipStreamBeginCapture(st_, hipStreamCaptureModeThreadLocal));
    launch_predict_batch(F_, Fprev_, vrve_, dF_dev_, Nt_, st_);
    for (int it = 0; it <= ncap; ++it) {
      newton_eval_device(it, lp, it == 0 ? dg_c_ : dg_t_);
      if (it < ncap) solve(it);
    }
    RVE_HIP(hipStreamEndCapture(st_, &inc_graph_def_));
    RVE_HIP(hipGraphInstantiate(&inc_graph_, inc_graph_def_, nullptr, nullptr, 0));
    inc_graph_dt_ = dt;
  }
  RVE_HIP(hipGraphLaunch(inc_graph_, st_));
  read_logs();
  // RVEs still iterating after the captured iterations go on one Newton
  // iteration at a time
  for (int it = ncap; it < cfg_.newton_max_iter; ++it) {
    bool any = false;
    for (int b = 0; b < B_; ++b) any = any || log_host_[b].status == 1;
    if (!any) break;
    solve(it);
    newton_eval_device(it + 1, lp, dg_t_);
    RVE_HIP(hipGetLastError());
    read_logs();
  }
  unsigned flag = 0;
  RVE_HIP(hipMemcpyAsync(&flag, bar_ + kBatchBarWords, sizeof(flag),
                         hipMemcpyDeviceToHost, st_));
  RVE_HIP(hipStreamSynchronize(st_));
  if (flag != 0)
    throw Error(RVE_EDEVICE, "persistent CG: a grid barrier waited past its bound");
  CommitBatchArgs c{};
  c.vrve = vrve_;
  c.scs = sc_;
  c.dF = dF_dev_;
  c.F = F_;
  c.P = P_;
  c.Fpi_t = Fpi_t_;
  c.chi_t = chi_t_;
  c.dg_t = dg_t_;
  c.Fprev = Fprev_;
  c.Pc = Pc_;
  c.Fpi_c = Fpi_c_;
  c.chi_c = chi_c_;
  c.dg_c = dg_c_;
  c.dFt = dFt_;
  c.phase = phase_;
  c.table = table_;
  c.pcyc = pcyc_;
  c.pcyc_lit = pcyc_lit_;
  c.wcyc = wcyc_;
  c.dt = dt;
  c.N = Nt_;
  launch_commit_batch(c, st_);
  RVE_HIP(hipGetLastError());
  RVE_HIP(hipStreamSynchronize(st_));
  const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  int first_bad = RVE_OK;
  for (int b = 0; b < B_; ++b) {
    const BatchLog& L = log_host_[b];
    rve_increment_info loc;
    std::memset(&loc, 0, sizeof(loc));
    loc.status = (L.status == 1) ? RVE_ENOTCONV : L.status;
    loc.newton_iters = L.newton_iters;
    loc.cg_iters_total = L.cg_total;
    loc.cg_breakdowns = L.breakdowns;
    loc.local_failures = L.fails;
    loc.residual_rel = L.rel;
    loc.predictor_residual = loc.plain_predictor_residual = L.predictor_rel;
    for (int k = 0; k < RVE_MAX_NEWTON_LOG && k < kBatchLog; ++k) {
      loc.residual_history[k] = L.res_hist[k];
      loc.cg_iters[k] = L.cg_hist[k];
    }
    for (int i = 0; i < 9; ++i) loc.P_bar[i] = L.pbar[i];
    loc.seconds = secs;
    const double* Fbar_new = Fbar_all + 9 * b;
    const double J = det3(Fbar_new);
    if (loc.status == RVE_OK) {
      for (int i = 0; i < 9; ++i) {
        Fbar_[b][i] = Fbar_new[i];
        Pbar_[b][i] = loc.P_bar[i];
      }
      t_[b] += dt;
      ++increments_[b];
    } else if (first_bad == RVE_OK) {
      first_bad = loc.status;
    }
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        double s = 0.0;
        for (int k = 0; k < 3; ++k) s += loc.P_bar[3 * i + k] * Fbar_new[3 * j + k];
        loc.sigma_bar[3 * i + j] = s / J;
      }
    if (info) info[b] = loc;
  }
  return first_bad;
}

// G(in) (Sec. 2.1, Eq. 11) of every RVE at once, through the batched pass
// kernels of the residual (FP64 mode) or of the CG precision (mixed mode:
// the input is rounded to FP32 first).  in / out: RVE after RVE, each a
// [9][n_b^3] block of doubles.
void BatchEngine::debug_apply_G(const double* in, double* out) {
  if (!in || !out) throw Error(RVE_EINVAL, "null field");
  int64_t pos = 0;
  for (int b = 0; b < B_; ++b) {
    const int64_t Nb = (int64_t)n_[b] * n_[b] * n_[b];
    for (int c = 0; c < 9; ++c)
      RVE_HIP(hipMemcpyAsync(r64_ + (int64_t)c * Nt_ + off_[b], in + pos + c * Nb,
                             Nb * sizeof(double), hipMemcpyHostToDevice, st_));
    pos += 9 * Nb;
    sc_host_[b].inactive = 0;
    sc_host_[b].done = 0;
  }
  upload_scalars();
  if (fp64_) {
    BatchSpec<double> rs{};
    rs.items = (const SpecItem<double>*)items64_;
    rs.nitems = B_;
    rs.cpbs = cpbs64_;
    rs.cs = Nt_;
    rs.field = r64_;
    rs.spec = (cplx<double>*)spec64_;
    launch_G_batch<double>(rs, SRC_FIELD, nullptr, P_, blocksA64_, blocksB64_,
                           ldsA64_, ldsB64_, st_);
  } else {
    launch_convert<float>(r64_, (float*)x_, 9 * Nt_, st_);
    BatchSpec<float> rs{};
    rs.items = (const SpecItem<float>*)items32_;
    rs.nitems = B_;
    rs.cpbs = cpbs32_;
    rs.cs = Nt_;
    rs.field = (const float*)x_;
    rs.spec = (cplx<float>*)spec_;
    launch_G_batch<float>(rs, SRC_FIELD, nullptr, P_, blocksA32_, blocksB32_,
                          ldsA32_, ldsB32_, st_);
  }
  RVE_HIP(hipGetLastError());
  pos = 0;
  for (int b = 0; b < B_; ++b) {
    const int64_t Nb = (int64_t)n_[b] * n_[b] * n_[b];
    for (int c = 0; c < 9; ++c)
      RVE_HIP(hipMemcpyAsync(out + pos + c * Nb, P_ + (int64_t)c * Nt_ + off_[b],
                             Nb * sizeof(double), hipMemcpyDeviceToHost, st_));
    pos += 9 * Nb;
  }
  RVE_HIP(hipStreamSynchronize(st_));
}

void BatchEngine::reset_fips() {
  launch_fill_f64(pcyc_, 0.0, Nt_, st_);
  launch_fill_f64(pcyc_lit_, 0.0, Nt_, st_);
  launch_fill_f64(wcyc_, 0.0, 12 * Nt_, st_);
  RVE_HIP(hipGetLastError());
  RVE_HIP(hipStreamSynchronize(st_));
}

size_t BatchEngine::field_bytes(int b, int field) const {
  if (b < 0 || b >= B_) throw Error(RVE_EINVAL, "RVE index out of range");
  size_t comps = 0;
  switch (field) {
    case RVE_FIELD_F: case RVE_FIELD_P: case RVE_FIELD_SIGMA:
    case RVE_FIELD_FPINV: comps = 9; break;
    case RVE_FIELD_CHI: case RVE_FIELD_DGAMMA: case RVE_FIELD_WCYC: comps = 12; break;
    case RVE_FIELD_PCYC: case RVE_FIELD_PCYC_LIT: comps = 1; break;
    default: throw Error(RVE_EINVAL, "unknown field id for a batch");
  }
  return comps * (size_t)n_[b] * n_[b] * n_[b] * sizeof(double);
}

void BatchEngine::get_field(int b, int field, void* dst, size_t bytes,
                            bool on_device) {
  if (b < 0 || b >= B_) throw Error(RVE_EINVAL, "RVE index out of range");
  if (!dst) throw Error(RVE_EINVAL, "null destination");
  const double* src = nullptr;
  int comps = 0;
  switch (field) {
    case RVE_FIELD_F: src = Fprev_; comps = 9; break;
    case RVE_FIELD_P: src = Pc_; comps = 9; break;
    case RVE_FIELD_SIGMA:
      launch_cauchy(Fprev_, Pc_, r64_, Nt_, st_);
      src = r64_;
      comps = 9;
      break;
    case RVE_FIELD_FPINV: src = Fpi_c_; comps = 9; break;
    case RVE_FIELD_CHI: src = chi_c_; comps = 12; break;
    case RVE_FIELD_DGAMMA: src = dg_c_; comps = 12; break;
    case RVE_FIELD_PCYC: src = pcyc_; comps = 1; break;
    case RVE_FIELD_PCYC_LIT: src = pcyc_lit_; comps = 1; break;
    case RVE_FIELD_WCYC: src = wcyc_; comps = 12; break;
    default: throw Error(RVE_EINVAL, "unknown field id");
  }
  const int64_t Nb = (int64_t)n_[b] * n_[b] * n_[b];
  if (bytes < (size_t)comps * Nb * sizeof(double)) throw Error(RVE_EINVAL, "destination too small");
  for (int c = 0; c < comps; ++c)
    RVE_HIP(hipMemcpyAsync((char*)dst + (size_t)c * Nb * sizeof(double),
                           src + (int64_t)c * Nt_ + off_[b], Nb * sizeof(double),
                           on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                           st_));
  RVE_HIP(hipStreamSynchronize(st_));
}

void BatchEngine::get_macro(int b, double out[29]) {
  if (b < 0 || b >= B_) throw Error(RVE_EINVAL, "RVE index out of range");
  for (int i = 0; i < 9; ++i) {
    out[i] = Fbar_[b][i];
    out[9 + i] = Pbar_[b][i];
  }
  const double J = det3(Fbar_[b].data());
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double s = 0.0;
      for (int k = 0; k < 3; ++k) s += Pbar_[b][3 * i + k] * Fbar_[b][3 * j + k];
      out[18 + 3 * i + j] = s / J;
    }
  out[27] = t_[b];
  out[28] = (double)increments_[b];
}

}  // namespace rve
