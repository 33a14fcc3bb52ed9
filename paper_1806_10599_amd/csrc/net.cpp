// Warm-start network object: FP32 master parameters with Adam state, bf16
// MFMA fragments, activation scratch sized for the largest grid seen.
#include <cstring>

#include "nn.hpp"

namespace rve {

namespace {
// layer shapes: real (cin, cout) and padded (CIN, COUT)
const int kCin[4] = {kFeatReal, kWidth, kWidth, kWidth};
const int kCout[4] = {kWidth, kWidth, kWidth, kOutReal};
const int kCIN[4] = {kFeat, kWidth, kWidth, kWidth};
const int kCOUT[4] = {kWidth, kWidth, kWidth, kOut};

int64_t layer_off(int k) {
  int64_t o = 0;
  for (int i = 0; i < k; ++i) o += (int64_t)27 * kCin[i] * kCout[i] + kCout[i];
  return o;
}
constexpr int kChunk = 4096;   // voxels per weight-gradient block
constexpr int kBiasBlocks = 64;
constexpr int kLossBlocks = 256;
}  // namespace

int64_t Net::param_count() { return layer_off(4); }

Net::Net(hipStream_t s, AllocFn a, FreeFn f, void* ctx)
    : st_(s), af_(a), ff_(f), ctx_(ctx) {
  const int64_t P = param_count();
  w_ = (float*)alloc(P * sizeof(float));
  g_ = (float*)alloc(P * sizeof(float));
  m_ = (float*)alloc(P * sizeof(float));
  v_ = (float*)alloc(P * sizeof(float));
  for (int k = 0; k < 4; ++k) {
    const size_t fr = (size_t)27 * kCIN[k] * kCOUT[k] * sizeof(uint16_t);
    wf_[k] = (uint16_t*)alloc(fr);
    wb_[k] = (uint16_t*)alloc(fr);
  }
  wpad_ = (float*)alloc((size_t)27 * kFeat * kWidth * sizeof(float));
  lpart_ = (double*)alloc(kLossBlocks * sizeof(double));
  RVE_HIP(hipHostMalloc((void**)&lhost_, kLossBlocks * sizeof(double),
                        hipHostMallocDefault));
  RVE_HIP(hipMemsetAsync(w_, 0, P * sizeof(float), st_));
  RVE_HIP(hipMemsetAsync(m_, 0, P * sizeof(float), st_));
  RVE_HIP(hipMemsetAsync(v_, 0, P * sizeof(float), st_));
  repack();
  RVE_HIP(hipStreamSynchronize(st_));
}

Net::~Net() {
  if (st_) hipStreamSynchronize(st_);
  for (auto& p : allocs_) {
    if (ff_)
      ff_(p.first, ctx_);
    else
      hipFree(p.first);
  }
  if (lhost_) hipHostFree(lhost_);
}

void* Net::alloc(size_t b) {
  void* p = nullptr;
  if (af_) {
    p = af_(b, (void*)st_, ctx_);
    if (!p) throw Error(-2, "device allocator returned NULL");
  } else {
    hipError_t e = hipMalloc(&p, b);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      throw Error(-2, "hipMalloc failed for the network");
    }
  }
  allocs_.push_back({p, b});
  return p;
}

void Net::ensure(int64_t N) {
  if (N <= cap_) return;
  a1_ = (uint16_t*)alloc(N * kWidth * sizeof(uint16_t));
  a2_ = (uint16_t*)alloc(N * kWidth * sizeof(uint16_t));
  a3_ = (uint16_t*)alloc(N * kWidth * sizeof(uint16_t));
  d1_ = (uint16_t*)alloc(N * kWidth * sizeof(uint16_t));
  d2_ = (uint16_t*)alloc(N * kWidth * sizeof(uint16_t));
  dy_ = (uint16_t*)alloc(N * kOut * sizeof(uint16_t));
  yf_ = (float*)alloc(N * kOut * sizeof(float));
  dyf_ = (float*)alloc(N * kOut * sizeof(float));
  const int64_t nch = (N + kChunk - 1) / kChunk;
  part_ = (float*)alloc((size_t)nch * 27 * kFeat * kWidth * sizeof(float));
  cap_ = N;
}

void Net::repack() {
  for (int k = 0; k < 4; ++k)
    nn_pack(w_ + layer_off(k), kCin[k], kCout[k], kCIN[k], kCOUT[k], wf_[k],
            wb_[k], st_);
  RVE_HIP(hipGetLastError());
}

void Net::set_params(const float* host, int64_t count) {
  if (!host || count != param_count())
    throw Error(-1, "parameter vector has the wrong length");
  RVE_HIP(hipMemcpyAsync(w_, host, count * sizeof(float), hipMemcpyHostToDevice,
                         st_));
  RVE_HIP(hipMemsetAsync(m_, 0, count * sizeof(float), st_));
  RVE_HIP(hipMemsetAsync(v_, 0, count * sizeof(float), st_));
  step_ = 0;
  repack();
  RVE_HIP(hipStreamSynchronize(st_));
}

void Net::get_params(float* host, int64_t count) {
  if (!host || count != param_count())
    throw Error(-1, "parameter vector has the wrong length");
  RVE_HIP(hipMemcpyAsync(host, w_, count * sizeof(float), hipMemcpyDeviceToHost,
                         st_));
  RVE_HIP(hipStreamSynchronize(st_));
}

void Net::forward(const uint16_t* X, int n, float* Y, hipStream_t s) {
  if (n % 16) throw Error(-1, "the network needs a grid edge divisible by 16");
  const int64_t N = (int64_t)n * n * n;
  ensure(N);
  // inference inside an increment runs on the RVE's stream; the scratch
  // activations are only touched by work ordered on one stream at a time
  hipStream_t st = s ? s : st_;
  const float* b[4];
  for (int k = 0; k < 4; ++k) b[k] = w_ + layer_off(k) + (int64_t)27 * kCin[k] * kCout[k];
  nn_conv(kFeat, kWidth, 0, X, wf_[0], b[0], a1_, nullptr, nullptr, n, N, kWidth, st);
  nn_conv(kWidth, kWidth, 0, a1_, wf_[1], b[1], a2_, nullptr, nullptr, n, N, kWidth, st);
  nn_conv(kWidth, kWidth, 0, a2_, wf_[2], b[2], a3_, nullptr, nullptr, n, N, kWidth, st);
  nn_conv(kWidth, kOut, 1, a3_, wf_[3], b[3], nullptr, Y, nullptr, n, N, kOutReal, st);
  RVE_HIP(hipGetLastError());
}

double Net::loss(const uint16_t* X, const float* T, int n) {
  if (n % 16) throw Error(-1, "the network needs a grid edge divisible by 16");
  const int64_t N = (int64_t)n * n * n;
  ensure(N);
  forward(X, n, yf_);
  nn_mse(yf_, T, kOut, kOutReal, N, dy_, dyf_, lpart_, kLossBlocks, st_);
  RVE_HIP(hipGetLastError());
  RVE_HIP(hipMemcpyAsync(lhost_, lpart_, kLossBlocks * sizeof(double),
                         hipMemcpyDeviceToHost, st_));
  RVE_HIP(hipStreamSynchronize(st_));
  double L = 0.0;
  for (int i = 0; i < kLossBlocks; ++i) L += lhost_[i];
  return L;
}

double Net::train_step(const uint16_t* X, const float* T, int n, float lr,
                       float* grad_host) {
  if (n % 16) throw Error(-1, "the network needs a grid edge divisible by 16");
  const int64_t N = (int64_t)n * n * n;
  ensure(N);
  forward(X, n, yf_);
  nn_mse(yf_, T, kOut, kOutReal, N, dy_, dyf_, lpart_, kLossBlocks, st_);
  const int nch = (int)((N + kChunk - 1) / kChunk);
  const uint16_t* acts[4] = {X, a1_, a2_, a3_};
  const uint16_t* dz = dy_;          // gradient at the output of layer k
  uint16_t* dbuf[2] = {d1_, d2_};
  float* bpart = part_;              // reused after each layer's dW sum
  for (int k = 3; k >= 0; --k) {
    const int CIN = kCIN[k], COUT = kCOUT[k];
    nn_wgrad(CIN, COUT, acts[k], dz, part_, nch, kChunk, n, N, st_);
    nn_sum_parts(part_, nch, (int64_t)27 * CIN * COUT, wpad_, st_);
    nn_unpad(wpad_, CIN, COUT, kCin[k], kCout[k], g_ + layer_off(k), st_);
    nn_bias_grad(COUT, k == 3 ? nullptr : dz, k == 3 ? dyf_ : nullptr, N, bpart,
                 kBiasBlocks, st_);
    nn_sum_parts(bpart, kBiasBlocks, COUT, wpad_, st_);
    RVE_HIP(hipMemcpyAsync(g_ + layer_off(k) + (int64_t)27 * kCin[k] * kCout[k],
                           wpad_, kCout[k] * sizeof(float),
                           hipMemcpyDeviceToDevice, st_));
    if (k > 0) {
      // gradient at the output of layer k-1, through its ReLU
      uint16_t* out = dbuf[k % 2];
      nn_conv(COUT, CIN, 2, dz, wb_[k], nullptr, out, nullptr, acts[k], n, N,
              CIN, st_);
      dz = out;
    }
  }
  ++step_;
  nn_adam(w_, g_, m_, v_, param_count(), lr, 0.9f, 0.999f, 1e-8f, step_, st_);
  repack();
  RVE_HIP(hipGetLastError());
  if (grad_host)
    RVE_HIP(hipMemcpyAsync(grad_host, g_, param_count() * sizeof(float),
                           hipMemcpyDeviceToHost, st_));
  RVE_HIP(hipMemcpyAsync(lhost_, lpart_, kLossBlocks * sizeof(double),
                         hipMemcpyDeviceToHost, st_));
  RVE_HIP(hipStreamSynchronize(st_));
  double L = 0.0;
  for (int i = 0; i < kLossBlocks; ++i) L += lhost_[i];
  return L;
}

}  // namespace rve
