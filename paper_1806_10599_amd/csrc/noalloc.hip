// The projection G (Sec. 2.1, Eq. 11) of a device field without any device
// allocation: spectrum, FFT twiddles, wave vectors and per-block partial
// sums live in one static device array of fixed size per GPU.  For callers
// that cannot allocate (code under stream capture, serving loops, harnesses
// that forbid it); the single-RVE FP64 pass kernels do the work.
#include "../../include/rve.h"
#include "kernels.hpp"

#include <cmath>
#include <mutex>

namespace rve {

namespace {

constexpr int kMaxN = RVE_NOALLOC_MAX_N;
constexpr size_t align256(size_t b) { return (b + 255) / 256 * 256; }
// layout of the scratch array (bytes, each part 256-byte aligned)
constexpr size_t kSpecOff = 0;
constexpr size_t kSpecBytes =
    align256((size_t)9 * kMaxN * kMaxN * (kMaxN / 2) * sizeof(cplx<double>));
constexpr size_t kTwOff = kSpecOff + kSpecBytes;
constexpr size_t kTwBytes = align256((size_t)kMaxN * sizeof(cplx<double>));
constexpr size_t kVtOff = kTwOff + kTwBytes;
constexpr size_t kVtBytes = align256((size_t)3 * kMaxN * sizeof(double));
constexpr size_t kPartOff = kVtOff + kVtBytes;
constexpr size_t kPartBytes = align256((size_t)9 * kMaxN * sizeof(double));
constexpr size_t kScratchBytes = kPartOff + kPartBytes;
static_assert(kScratchBytes == RVE_NOALLOC_SCRATCH_BYTES,
              "scratch size in the header");

// One copy per GPU, held until the process ends.  Host code never uses this
// name as an address: the device address comes from hipGetSymbolAddress.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
unsigned char* g_ptr[kMaxDevices] = {};

unsigned char* scratch_ptr() {
  int dev = -1;
  RVE_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) throw Error(RVE_EDEVICE, "device index out of range");
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    RVE_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) throw Error(RVE_EDEVICE, "no device address for the scratch array");
    g_ptr[dev] = (unsigned char*)p;
  }
  return g_ptr[dev];
}

// FFT twiddles exp(-2 pi i m / n) and the per-axis wave vectors of the
// operator (Sec. 2.2, Eq. 18; continuous Eq. 19: v = q n / L, discrete
// Eqs. 20-21: v = tan(q / 2) n / L; the Nyquist entry is never used and is
// set to 0), the tables the FP64 passes read.
__global__ void noalloc_tables_kernel(int n, double L0, double L1, double L2,
                                      int projection, cplx<double>* tw,
                                      double* vt) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    double s, c;
    sincospi(-2.0 * (double)i / (double)n, &s, &c);
    tw[i] = {c, s};
  }
  if (i < 3 * n) {
    const int d = i / n, idx = i - d * n;
    const int k = (idx < (n + 1) / 2) ? idx : idx - n;
    const double Ld = d == 0 ? L0 : (d == 1 ? L1 : L2);
    double v = 0.0;
    if (!(n % 2 == 0 && k == -n / 2)) {
      const double scale = (double)n / Ld;
      v = projection == RVE_PROJ_CONTINUOUS
              ? 2.0 * M_PI * (double)k / (double)n * scale
              : tan(M_PI * (double)k / (double)n) * scale;
    }
    vt[i] = v;
  }
}

}  // namespace

void noalloc_apply_G(int n, const double L[3], int projection, const double* in,
                     double* out, hipStream_t s) {
  if (n > kMaxN)
    throw Error(RVE_EINVAL, "rve_apply_G_noalloc: n = " + std::to_string(n) +
                                " exceeds the scratch maximum " +
                                std::to_string(kMaxN));
  if (n != 16 && n != 24 && n != 32 && n != 40 && n != 48 && n != 64)
    throw Error(RVE_EINVAL, "rve_apply_G_noalloc: n must be 16, 24, 32, 40, 48 or 64");
  if (!L || !(L[0] > 0.0) || !(L[1] > 0.0) || !(L[2] > 0.0) ||
      !std::isfinite(L[0] + L[1] + L[2]))
    throw Error(RVE_EINVAL, "rve_apply_G_noalloc: cell lengths must be finite and > 0");
  if (projection != RVE_PROJ_CONTINUOUS && projection != RVE_PROJ_DISCRETE)
    throw Error(RVE_EINVAL, "rve_apply_G_noalloc: unknown projection operator");
  if (!in || !out) throw Error(RVE_EINVAL, "rve_apply_G_noalloc: null field pointer");
  if (in == out) throw Error(RVE_EINVAL, "rve_apply_G_noalloc: in and out alias");
  unsigned char* base = scratch_ptr();
  cplx<double>* tw = (cplx<double>*)(base + kTwOff);
  double* vt = (double*)(base + kVtOff);
  hipLaunchKernelGGL(noalloc_tables_kernel, dim3(1), dim3(256), 0, s, n, L[0],
                     L[1], L[2], projection, tw, vt);
  SpectralLaunch<double> G;
  G.src = SRC_FIELD;
  G.in_field = in;
  G.spec = (cplx<double>*)(base + kSpecOff);
  G.tw = tw;
  G.vt = vt;
  G.dst = DST_NORM;
  G.out_d = out;
  G.partial_inv = (double*)(base + kPartOff);
  launch_G<double>(n, G, s);
  RVE_HIP(hipGetLastError());
}

}  // namespace rve
