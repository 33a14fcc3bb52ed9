// extern "C" entry points declared in include/rve.h.  Every call converts
// C++ errors to rve_status; a HIP runtime error poisons the handle.
#include <cmath>
#include <cstring>
#include <new>
#include <string>

#include "../../include/rve.h"
#include "batch.hpp"
#include "engine.hpp"
#include "fips.hpp"
#include "tables.hpp"

struct rve_s {
  rve::Engine* eng = nullptr;
  std::string err;
  bool poisoned = false;
};

struct rve_batch_s {
  rve::BatchEngine* eng = nullptr;
  std::string err;
  bool poisoned = false;
};

struct rve_ws_s {
  rve::Net* net = nullptr;
  std::string err;
  bool poisoned = false;
};

namespace {

thread_local std::string g_create_error;

template <class H, class F>
rve_status guarded(H* h, F&& f) {
  if (!h) return RVE_EINVAL;
  if (h->poisoned) {
    h->err = "handle poisoned by an earlier device error: " + h->err;
    return RVE_EDEVICE;
  }
  try {
    h->err.clear();
    return (rve_status)f();
  } catch (const rve::Error& e) {
    h->err = e.what();
    if (e.code == RVE_EDEVICE) h->poisoned = true;
    return (rve_status)e.code;
  } catch (const std::bad_alloc&) {
    h->err = "host allocation failed";
    return RVE_ENOMEM;
  } catch (const std::exception& e) {
    h->err = e.what();
    return RVE_EINVAL;
  }
}

// The fields selected by mask (bit f = field id f), in increasing id order,
// one after another in dst; sizes are checked before anything is copied.
template <class Size, class Copy>
void copy_masked(uint32_t mask, void* dst, size_t dst_bytes, Size&& size,
                 Copy&& copy) {
  if (mask == 0 || (mask >> RVE_FIELD_COUNT) != 0)
    throw rve::Error(RVE_EINVAL, "field mask selects no field or unknown bits");
  if (!dst) throw rve::Error(RVE_EINVAL, "null destination");
  size_t need = 0;
  for (int f = 0; f < RVE_FIELD_COUNT; ++f)
    if (mask & (1u << f)) need += size(f);
  if (dst_bytes < need) throw rve::Error(RVE_EINVAL, "destination too small");
  char* p = (char*)dst;
  for (int f = 0; f < RVE_FIELD_COUNT; ++f) {
    if (!(mask & (1u << f))) continue;
    const size_t b = size(f);
    copy(f, p, b);   // also for an empty field: it raises the state errors
    p += b;
  }
}

}  // namespace

extern "C" {

rve_status rve_config_default(rve_config* cfg) {
  if (!cfg) return RVE_EINVAL;
  std::memset(cfg, 0, sizeof(*cfg));
  cfg->n[0] = cfg->n[1] = cfg->n[2] = 16;
  cfg->L[0] = cfg->L[1] = cfg->L[2] = 1.0;
  cfg->projection = RVE_PROJ_DISCRETE;
  cfg->precision = RVE_PREC_FP64;
  cfg->warm_start = 0;
  cfg->use_graph = 0;
  cfg->newton_tol = 1e-6;
  cfg->newton_max_iter = 25;
  cfg->cg_tol = 1e-4;
  cfg->cg_max_iter = 2000;
  cfg->cg_chunk = 8;
  return RVE_OK;
}

rve_status rve_create(const rve_config* cfg, rve_t* out) {
  if (!cfg || !out) return RVE_EINVAL;
  *out = nullptr;
  rve_s* h = new (std::nothrow) rve_s();
  if (!h) return RVE_ENOMEM;
  try {
    h->eng = new rve::Engine(*cfg);
  } catch (const rve::Error& e) {
    g_create_error = e.what();
    delete h;
    return (rve_status)e.code;
  } catch (const std::exception& e) {
    g_create_error = e.what();
    delete h;
    return RVE_ENOMEM;
  }
  *out = h;
  return RVE_OK;
}

rve_status rve_destroy(rve_t h) {
  if (!h) return RVE_OK;
  delete h->eng;
  delete h;
  return RVE_OK;
}

rve_status rve_set_microstructure(rve_t h, const int32_t* phase, int32_t G,
                                  const double* quat, const int32_t* law,
                                  const double* params, int32_t nparams) {
  return guarded(h, [&] {
    h->eng->set_microstructure(phase, G, quat, law, params, nparams);
    return RVE_OK;
  });
}

rve_status rve_set_user_material(rve_t h, rve_umat_fn fn, void* user,
                                 int32_t nstatev, const double* statev0) {
  return guarded(h, [&] {
    h->eng->set_user_material(fn, user, nstatev, statev0);
    return RVE_OK;
  });
}

int32_t rve_umat_neo_hooke(void* user, const double* F1, const double* F0,
                           const double* statev_old, double* statev_new,
                           int32_t nstatev, double* sigma, double* ddsdde,
                           int32_t* fails, int64_t n, double dt, void* stream) {
  (void)user;
  (void)dt;
  if (nstatev < 3 || n < 0) return -1;
  rve::launch_neo_hooke_umat(F1, F0, statev_old, statev_new, nstatev, sigma,
                             ddsdde, fails, n, (hipStream_t)stream);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

rve_status rve_apply_macro_strain_increment(rve_t h, const double F_bar_new[9],
                                            double dt,
                                            rve_increment_info* info) {
  return guarded(h, [&] {
    if (!F_bar_new) throw rve::Error(RVE_EINVAL, "null F_bar_new");
    return h->eng->increment(F_bar_new, dt, info);
  });
}

rve_status rve_apply_macro_strain_increment_adaptive(
    rve_t h, const double F_bar_new[9], double dt, int32_t max_cutbacks,
    int32_t grow_after, rve_adaptive_info* info) {
  return guarded(h, [&] {
    if (!F_bar_new) throw rve::Error(RVE_EINVAL, "null F_bar_new");
    return (rve_status)h->eng->increment_adaptive(F_bar_new, dt, max_cutbacks,
                                                  grow_after, info);
  });
}

rve_status rve_reset_fips(rve_t h) {
  return guarded(h, [&] {
    h->eng->reset_fips();
    return RVE_OK;
  });
}

rve_status rve_get_fields(rve_t h, uint32_t mask, void* dst, size_t dst_bytes,
                          int32_t dst_on_device) {
  return guarded(h, [&] {
    copy_masked(mask, dst, dst_bytes,
                [&](int f) { return h->eng->field_bytes(f); },
                [&](int f, void* p, size_t b) {
                  h->eng->get_field(f, p, b, dst_on_device != 0);
                });
    return RVE_OK;
  });
}

rve_status rve_get_nonlocal_fips(rve_t h, double band_width,
                                 rve_nonlocal_fips* out, double* grain_pcyc,
                                 double* grain_pcyc_lit, int32_t labels,
                                 double* band_wcyc, int32_t* band_desc,
                                 int64_t band_cap) {
  return guarded(h, [&] {
    h->eng->nonlocal_fips(band_width, out, grain_pcyc, grain_pcyc_lit, labels,
                          band_wcyc, band_desc, band_cap);
    return RVE_OK;
  });
}

rve_status rve_get_macro(rve_t h, double out[29]) {
  return guarded(h, [&] {
    if (!out) throw rve::Error(RVE_EINVAL, "null output");
    h->eng->get_macro(out);
    return RVE_OK;
  });
}

rve_status rve_state_size(rve_t h, size_t* bytes) {
  return guarded(h, [&] {
    if (!bytes) throw rve::Error(RVE_EINVAL, "null output");
    *bytes = h->eng->state_size();
    return RVE_OK;
  });
}

rve_status rve_get_state(rve_t h, void* dst, size_t bytes) {
  return guarded(h, [&] {
    h->eng->get_state(dst, bytes);
    return RVE_OK;
  });
}

rve_status rve_set_state(rve_t h, const void* src, size_t bytes) {
  return guarded(h, [&] {
    h->eng->set_state(src, bytes);
    return RVE_OK;
  });
}

const char* rve_last_error(rve_t h) {
  if (!h) return g_create_error.c_str();
  return h->err.c_str();
}

rve_status rve_apply_G_noalloc(int32_t n, const double L[3],
                               int32_t projection, const double* in,
                               double* out, void* stream) {
  try {
    rve::noalloc_apply_G(n, L, projection, in, out, (hipStream_t)stream);
  } catch (const rve::Error& e) {
    g_create_error = e.what();
    return (rve_status)e.code;
  } catch (const std::exception& e) {
    g_create_error = e.what();
    return RVE_EINVAL;
  }
  return RVE_OK;
}

rve_status rve_debug_apply_G(rve_t h, const double* in, double* out,
                             int32_t precision) {
  return guarded(h, [&] {
    h->eng->debug_apply_G(in, out, precision);
    return RVE_OK;
  });
}

rve_status rve_debug_constitutive(rve_t h, const double* F, double dt,
                                  double* P, double* K, double* dg,
                                  int32_t* fails) {
  return guarded(h, [&] {
    h->eng->debug_constitutive(F, dt, P, K, dg, fails);
    return RVE_OK;
  });
}

rve_status rve_debug_set_field(rve_t h, int32_t field, const double* src,
                               size_t bytes) {
  return guarded(h, [&] {
    h->eng->debug_set_field(field, src, bytes);
    return RVE_OK;
  });
}

rve_status rve_bench_kernels(rve_t h, int32_t reps, double* ms_out,
                             int32_t count) {
  return guarded(h, [&] {
    h->eng->bench_kernels(reps, ms_out, count);
    return RVE_OK;
  });
}

rve_status rve_ws_create(const rve_ws_config* cfg, rve_ws_t* out) {
  if (!cfg || !out) return RVE_EINVAL;
  *out = nullptr;
  if ((cfg->dev_alloc == nullptr) != (cfg->dev_free == nullptr)) return RVE_EINVAL;
  rve_ws_s* h = new (std::nothrow) rve_ws_s();
  if (!h) return RVE_ENOMEM;
  try {
    h->net = new rve::Net((hipStream_t)cfg->stream, cfg->dev_alloc, cfg->dev_free,
                          cfg->alloc_ctx);
  } catch (const rve::Error& e) {
    g_create_error = e.what();
    delete h;
    return (rve_status)e.code;
  } catch (const std::exception& e) {
    g_create_error = e.what();
    delete h;
    return RVE_ENOMEM;
  }
  *out = h;
  return RVE_OK;
}

rve_status rve_ws_destroy(rve_ws_t w) {
  if (!w) return RVE_OK;
  delete w->net;
  delete w;
  return RVE_OK;
}

rve_status rve_ws_param_count(rve_ws_t w, int64_t* count) {
  return guarded(w, [&] {
    if (!count) throw rve::Error(RVE_EINVAL, "null output");
    *count = rve::Net::param_count();
    return RVE_OK;
  });
}

rve_status rve_ws_set_params(rve_ws_t w, const float* params, int64_t count) {
  return guarded(w, [&] {
    w->net->set_params(params, count);
    return RVE_OK;
  });
}

rve_status rve_ws_get_params(rve_ws_t w, float* params, int64_t count) {
  return guarded(w, [&] {
    w->net->get_params(params, count);
    return RVE_OK;
  });
}

rve_status rve_ws_forward(rve_ws_t w, const uint16_t* X, int32_t n, float* Y) {
  return guarded(w, [&] {
    if (!X || !Y) throw rve::Error(RVE_EINVAL, "null buffer");
    w->net->forward(X, n, Y);
    RVE_HIP(hipStreamSynchronize(w->net->stream()));
    return RVE_OK;
  });
}

rve_status rve_ws_train_step(rve_ws_t w, const uint16_t* X, const float* T,
                             int32_t n, float lr, double* loss,
                             float* grad_host) {
  return guarded(w, [&] {
    if (!X || !T) throw rve::Error(RVE_EINVAL, "null buffer");
    const double L = w->net->train_step(X, T, n, lr, grad_host);
    if (loss) *loss = L;
    return RVE_OK;
  });
}

rve_status rve_ws_loss(rve_ws_t w, const uint16_t* X, const float* T,
                       int32_t n, double* loss) {
  return guarded(w, [&] {
    if (!X || !T || !loss) throw rve::Error(RVE_EINVAL, "null buffer");
    *loss = w->net->loss(X, T, n);
    return RVE_OK;
  });
}

const char* rve_ws_last_error(rve_ws_t w) {
  if (!w) return g_create_error.c_str();
  return w->err.c_str();
}

rve_status rve_attach_warm_start(rve_t h, rve_ws_t w) {
  return guarded(h, [&] {
    h->eng->attach_net(w ? w->net : nullptr);
    return RVE_OK;
  });
}

rve_status rve_ws_features(rve_t h, const double F_bar_new[9], uint16_t* X) {
  return guarded(h, [&] {
    if (!F_bar_new) throw rve::Error(RVE_EINVAL, "null F_bar_new");
    h->eng->features(F_bar_new, X);
    return RVE_OK;
  });
}

rve_status rve_ws_target(rve_t h, float* T) {
  return guarded(h, [&] {
    h->eng->target(T);
    return RVE_OK;
  });
}

rve_status rve_set_kernel_timing(rve_t h, uint32_t mask) {
  return guarded(h, [&] {
    h->eng->set_timing(mask);
    return RVE_OK;
  });
}

rve_status rve_set_kernel_timing_stride(rve_t h, int32_t stride) {
  return guarded(h, [&] {
    h->eng->set_timing_stride(stride);
    return RVE_OK;
  });
}

rve_status rve_get_kernel_timing(rve_t h, double* ms_total, int64_t* launches,
                                 int32_t count, int32_t reset) {
  return guarded(h, [&] {
    if (count > 8) throw rve::Error(RVE_EINVAL, "count > 8");
    h->eng->get_timing(ms_total, launches, count, reset != 0);
    return RVE_OK;
  });
}

rve_status rve_get_kernel_launches(rve_t h, int64_t* launches, int32_t count,
                                   int32_t reset) {
  return guarded(h, [&] {
    if (count > 8 || count < 0) throw rve::Error(RVE_EINVAL, "count out of range");
    h->eng->get_timing(nullptr, nullptr, count, reset != 0, launches);
    return RVE_OK;
  });
}

rve_status rve_get_return_map_counts(rve_t h, int64_t out[4], int32_t reset) {
  return guarded(h, [&] {
    if (!out) throw rve::Error(RVE_EINVAL, "null output");
    h->eng->get_rm_counts(out, reset != 0);
    return RVE_OK;
  });
}

rve_status rve_set_fft_schedule(rve_t h, int32_t cpb, int32_t tt,
                                int32_t fused) {
  return guarded(h, [&] {
    h->eng->set_schedule(cpb, tt, fused);
    return RVE_OK;
  });
}

rve_status rve_tune_fft_schedule(rve_t h) {
  return guarded(h, [&] {
    h->eng->tune();
    return RVE_OK;
  });
}

rve_status rve_get_fft_schedule(rve_t h, int32_t out[3], double* ms) {
  return guarded(h, [&] {
    if (!out) throw rve::Error(RVE_EINVAL, "null output");
    int o[3];
    h->eng->get_schedule(o, ms);
    out[0] = o[0];
    out[1] = o[1];
    out[2] = o[2];
    return RVE_OK;
  });
}

rve_status rve_umat_bridge(const double* F, const double* sigma,
                           const double* ddsdde, int64_t n, double* P,
                           double* K, void* stream) {
  if (n < 0 || (n > 0 && (!F || !sigma || !ddsdde || !P || !K))) {
    g_create_error = "rve_umat_bridge: null pointer or n < 0";
    return RVE_EINVAL;
  }
  rve::launch_umat_bridge(F, sigma, ddsdde, n, P, K, (hipStream_t)stream);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    g_create_error = std::string("rve_umat_bridge: ") + hipGetErrorString(e);
    return RVE_EDEVICE;
  }
  return RVE_OK;
}

rve_status rve_batch_create(const rve_config* cfg, int32_t count,
                            const int32_t* n, rve_batch_t* out) {
  if (!cfg || !out || !n) return RVE_EINVAL;
  *out = nullptr;
  rve_batch_s* h = new (std::nothrow) rve_batch_s();
  if (!h) return RVE_ENOMEM;
  try {
    h->eng = new rve::BatchEngine(*cfg, count, n);
  } catch (const rve::Error& e) {
    g_create_error = e.what();
    delete h;
    return (rve_status)e.code;
  } catch (const std::bad_alloc&) {
    g_create_error = "host allocation failed";
    delete h;
    return RVE_ENOMEM;
  }
  *out = h;
  return RVE_OK;
}

rve_status rve_batch_destroy(rve_batch_t h) {
  if (!h) return RVE_OK;
  delete h->eng;
  delete h;
  return RVE_OK;
}

rve_status rve_batch_set_microstructure(rve_batch_t h, int32_t b,
                                        const int32_t* phase, int32_t G,
                                        const double* quat, const int32_t* law,
                                        const double* params, int32_t nparams) {
  return guarded(h, [&] {
    h->eng->set_microstructure(b, phase, G, quat, law, params, nparams);
    return RVE_OK;
  });
}

rve_status rve_batch_apply_macro_strain_increment(rve_batch_t h,
                                                  const double* F_bar_new,
                                                  double dt,
                                                  rve_increment_info* info) {
  return guarded(h, [&] {
    if (!F_bar_new) throw rve::Error(RVE_EINVAL, "null F_bar_new");
    return h->eng->increment(F_bar_new, dt, info);
  });
}

rve_status rve_batch_reset_fips(rve_batch_t h) {
  return guarded(h, [&] {
    h->eng->reset_fips();
    return RVE_OK;
  });
}

rve_status rve_batch_get_fields(rve_batch_t h, int32_t b, uint32_t mask,
                                void* dst, size_t dst_bytes,
                                int32_t dst_on_device) {
  return guarded(h, [&] {
    copy_masked(mask, dst, dst_bytes,
                [&](int f) { return h->eng->field_bytes(b, f); },
                [&](int f, void* p, size_t n) {
                  h->eng->get_field(b, f, p, n, dst_on_device != 0);
                });
    return RVE_OK;
  });
}

rve_status rve_batch_debug_apply_G(rve_batch_t h, const double* in,
                                   double* out) {
  return guarded(h, [&] {
    h->eng->debug_apply_G(in, out);
    return RVE_OK;
  });
}

rve_status rve_batch_tune_fft_schedule(rve_batch_t h) {
  return guarded(h, [&] {
    h->eng->tune();
    return RVE_OK;
  });
}

rve_status rve_batch_set_fft_schedule(rve_batch_t h, int32_t edge,
                                      int32_t cpb, int32_t tt) {
  return guarded(h, [&] {
    h->eng->set_schedule(edge, cpb, tt);
    return RVE_OK;
  });
}

rve_status rve_batch_get_fft_schedule(rve_batch_t h, int32_t edge,
                                      int32_t out[2], double* ms) {
  return guarded(h, [&] {
    if (!out) throw rve::Error(RVE_EINVAL, "null output");
    int o[2];
    h->eng->get_schedule(edge, o, ms);
    out[0] = o[0];
    out[1] = o[1];
    return RVE_OK;
  });
}

rve_status rve_fip_band_lists(int32_t n, const double L[3],
                              const int32_t* phase, int32_t G,
                              const double* quat, const int32_t* law,
                              double band_width, int64_t* bands,
                              int64_t* entries, int32_t* band_desc,
                              int32_t* band_vox, int64_t cap_bands,
                              int64_t cap_entries) {
  try {
    if (n < 1 || n > 1024 || !L || !phase || G < 1 || !quat || !law || !bands ||
        !entries)
      throw rve::Error(RVE_EINVAL, "bad arguments");
    const int64_t N = (int64_t)n * n * n;
    for (int64_t v = 0; v < N; ++v)
      if (phase[v] < 0 || phase[v] >= G)
        throw rve::Error(RVE_EINVAL, "phase label out of [0, G)");
    for (int g = 0; g < G; ++g) {
      if (law[g] != 0 && law[g] != 1) throw rve::Error(RVE_EINVAL, "unknown law id");
      const double q2 = quat[4 * g] * quat[4 * g] + quat[4 * g + 1] * quat[4 * g + 1] +
                        quat[4 * g + 2] * quat[4 * g + 2] + quat[4 * g + 3] * quat[4 * g + 3];
      if (!(std::fabs(q2 - 1.0) < 1e-6)) throw rve::Error(RVE_EINVAL, "quaternion not unit");
    }
    // the slip-plane normals of the label tables do not depend on the
    // material constants
    const double dummy[RVE_NPARAMS] = {1, 0, 1, 1, 1, 1, 0, 0, 1, 0.25};
    const std::vector<double> tab = rve::label_table(G, quat, law, dummy);
    const rve::FipLists fl = rve::fip_lists(n, L, phase, tab.data(), G, band_width);
    const int64_t ng = (int64_t)fl.grain_label.size();
    const int64_t nb = (int64_t)fl.band_meta.size();
    int64_t ne = 0;
    for (int64_t b = 0; b < nb; ++b) ne += fl.segs[ng + b].len;
    *bands = nb;
    *entries = ne;
    if (band_desc || band_vox) {
      if (cap_bands < nb || cap_entries < ne)
        throw rve::Error(RVE_EINVAL, "capacities below the counts");
      int64_t e = 0;
      for (int64_t b = 0; b < nb; ++b) {
        const auto& m = fl.band_meta[b];
        if (band_desc)
          for (int i = 0; i < 4; ++i) band_desc[4 * b + i] = m[i];
        const rve::FipSeg& sg = fl.segs[ng + b];
        if (band_vox)
          for (int32_t i = 0; i < sg.len; ++i) band_vox[e + i] = fl.vox[sg.off + i];
        e += sg.len;
      }
    }
    return RVE_OK;
  } catch (const rve::Error& e) {
    g_create_error = e.what();
    return (rve_status)e.code;
  } catch (const std::exception& e) {
    g_create_error = e.what();
    return RVE_EINVAL;
  }
}

rve_status rve_batch_get_nonlocal_fips(rve_batch_t h, int32_t b,
                                       double band_width,
                                       rve_nonlocal_fips* out,
                                       double* grain_pcyc,
                                       double* grain_pcyc_lit, int32_t labels,
                                       double* band_wcyc, int32_t* band_desc,
                                       int64_t band_cap) {
  return guarded(h, [&] {
    h->eng->nonlocal_fips(b, band_width, out, grain_pcyc, grain_pcyc_lit,
                          labels, band_wcyc, band_desc, band_cap);
    return RVE_OK;
  });
}

rve_status rve_batch_get_macro(rve_batch_t h, int32_t b, double out[29]) {
  return guarded(h, [&] {
    if (!out) throw rve::Error(RVE_EINVAL, "null output");
    h->eng->get_macro(b, out);
    return RVE_OK;
  });
}

const char* rve_batch_last_error(rve_batch_t h) {
  if (!h) return g_create_error.c_str();
  return h->err.c_str();
}

}  // extern "C"
