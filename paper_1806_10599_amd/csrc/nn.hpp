// Warm-start network: launchers of the bf16 MFMA convolution kernels and
// the network object (weights, Adam state, forward and training step).
#pragma once

#include <vector>

#include "common.hpp"

namespace rve {

// feature channels of the network input (real, padded to a multiple of 16)
constexpr int kFeatReal = 40, kFeat = 48;
constexpr int kWidth = 32;
constexpr int kOutReal = 9, kOut = 16;

void nn_conv(int cin, int cout, int epi, const uint16_t* X, const uint16_t* Wf,
             const float* b, uint16_t* Yb, float* Yf, const uint16_t* mask,
             int n, int64_t N, int cout_real, hipStream_t s);
void nn_wgrad(int cin, int cout, const uint16_t* X, const uint16_t* dZ,
              float* part, int nchunks, int64_t chunk, int n, int64_t N,
              hipStream_t s);
void nn_sum_parts(const float* part, int nparts, int64_t size, float* out,
                  hipStream_t s);
void nn_bias_grad(int cout, const uint16_t* dZ, const float* dYf, int64_t N,
                  float* part, int nblk, hipStream_t s);
void nn_mse(const float* Y, const float* T, int cpad, int creal, int64_t N,
            uint16_t* dYb, float* dYf, double* part, int nblk, hipStream_t s);
void nn_adam(float* w, const float* g, float* m, float* v, int64_t size,
             float lr, float b1, float b2, float eps, int step, hipStream_t s);
void nn_pack(const float* W, int cin, int cout, int CIN, int COUT, uint16_t* Wf,
             uint16_t* Wb, hipStream_t s);
void nn_unpad(const float* src, int CIN, int COUT, int cin, int cout,
              float* dst, hipStream_t s);

// per-increment data movement (features, target, prediction)
struct FeatArgs {
  const double* Fprev;     // [9][N] committed F_{k-1}
  const double* dFt_prev;  // [9][N] fluctuation increment of increment k-1
  const double* dg_prev;   // [12][N] slips of increment k-1
  const int32_t* phase;
  const double* table;     // label table (orientation at kTabR, law at 0)
  double fbar_prev[9];     // macro F_{k-1}
  double dfbar_n[9];       // (Fbar_k - Fbar_{k-1}) / s_k
  double inv_s_prev;       // 1 / s_{k-1} (0 when there is no previous)
  double reversal;         // dFbar_k : dFbar_{k-1} / (s_k s_{k-1})
  uint16_t* X;             // [N][kFeat] bf16
  int64_t N;
};
void nn_features(const FeatArgs& a, hipStream_t s);
// T = dFt inv_s - coef dFt2 (first 9 channels; float [N][16])
void nn_target(const double* dFt, double inv_s, const double* dFt2,
               double coef, float* T, int64_t N, hipStream_t s);
void nn_output_to_field(const float* Y, double scale, double* out, int64_t N,
                        hipStream_t s);
void nn_fluct_increment(const double* Fnew, const double* Fold,
                        const double dFbar[9], double* out, int64_t N,
                        hipStream_t s);
// F += a d
void nn_axpy_field(double* F, const double* d, double a, int64_t n9,
                   hipStream_t s);

class Net {
 public:
  using AllocFn = void* (*)(size_t, void*, void*);
  using FreeFn = void (*)(void*, void*);
  Net(hipStream_t s, AllocFn a, FreeFn f, void* ctx);
  ~Net();
  static int64_t param_count();
  void set_params(const float* host, int64_t count);
  void get_params(float* host, int64_t count);
  // X [N][kFeat] bf16 -> Y [N][kOut] f32
  void forward(const uint16_t* X, int n, float* Y, hipStream_t s = nullptr);
  // one Adam step on one sample; returns the loss, optionally the gradient
  double loss(const uint16_t* X, const float* T, int n);  // forward + MSE only
  double train_step(const uint16_t* X, const float* T, int n, float lr,
                    float* grad_host);
  hipStream_t stream() const { return st_; }

 private:
  void* alloc(size_t b);
  void ensure(int64_t N);
  void repack();
  hipStream_t st_;
  AllocFn af_;
  FreeFn ff_;
  void* ctx_;
  std::vector<std::pair<void*, size_t>> allocs_;
  float *w_ = nullptr, *g_ = nullptr, *m_ = nullptr, *v_ = nullptr;
  uint16_t* wf_[4] = {};
  uint16_t* wb_[4] = {};
  int64_t cap_ = 0;
  uint16_t *a1_ = nullptr, *a2_ = nullptr, *a3_ = nullptr;
  uint16_t *d1_ = nullptr, *d2_ = nullptr, *dy_ = nullptr;
  float *yf_ = nullptr, *dyf_ = nullptr, *part_ = nullptr, *wpad_ = nullptr;
  double* lpart_ = nullptr;
  double* lhost_ = nullptr;
  int step_ = 0;
};

}  // namespace rve
