// Warm-start network kernels: 3x3x3 circular convolutions as implicit GEMMs
// on the bf16 matrix cores (v_mfma_f32_16x16x16_bf16), FP32 accumulation.
//
// Layouts (all device memory):
//   activations  bf16 [N][C] channels-last (C a multiple of 16), voxel
//                v = (x*n + y)*n + z, periodic neighbours v + d_t;
//   tap t = (dx+1)*9 + (dy+1)*3 + (dz+1);
//   master weights FP32 per layer: W[27][cin][cout] then b[cout];
//   MFMA B fragments bf16 [27][CIN/16][COUT/16][64 lanes][4]: lane l of
//   fragment (t, kc, nt) holds W[t][16 kc + 4 (l/16) + i][16 nt + l%16].
// One wave computes 16 consecutive voxels along z times all output
// channels; lane l feeds voxel row l%16 (A operand: 4 consecutive input
// channels) and receives outputs for voxels 4 (l/16) + i, channel l%16.
#include "nn.hpp"
#include "kernels.hpp"

namespace rve {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint16_t f2bf(float f) {
  // round to nearest even
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) {
  return __uint_as_float(((uint32_t)h) << 16);
}

__device__ __forceinline__ int wrap(int i, int n) {
  return i < 0 ? i + n : (i >= n ? i - n : i);
}

// ------------------------------------------------------------- convolution
// EPI: 0 bias + ReLU -> bf16; 1 bias, linear -> f32; 2 no bias, multiply by
// the mask (mask_act > 0) -> bf16 (backward through the previous ReLU)
//
// A block of four waves computes 256 consecutive voxels (kConvTPW = 4
// 16-voxel tiles per wave; with n % 16 == 0 a block never leaves its x
// plane: for an edge-64 grid one wave is one z line and the block four
// neighbouring y lines).  For each dx slice of the stencil the block stages
// in LDS the B fragments of its nine taps and the input lines it reads
// (its own y lines and one on either side, all z, of plane x + dx, at a
// padded voxel stride), and the waves read both operands of every MFMA
// from LDS: each input datum is fetched from global memory about 4.5 times
// per layer instead of 27.
constexpr int kConvTPW = 4;
constexpr int kConvVox = 4 * kConvTPW * 16;   // voxels per block

// lines of one plane a block stages: its own (at most 256/n + 1 partial
// lines) and one on either side
__host__ __device__ constexpr int conv_lines(int n) {
  return (kConvVox + n - 1) / n + 3;
}
// LDS voxel stride in bf16: CIN + 8 keeps the 16 voxel rows of a fragment
// read on distinct banks and 16-byte staging stores aligned
template <int CIN>
constexpr int conv_cs() { return CIN + 8; }
template <int CIN, int COUT>
constexpr int conv_slice() { return 9 * (CIN / 16) * (COUT / 16) * 64 * 4; }
template <int CIN, int COUT>
size_t conv_lds_bytes(int n) {
  return ((size_t)conv_slice<CIN, COUT>() +
          (size_t)conv_lines(n) * n * conv_cs<CIN>()) * sizeof(uint16_t);
}

template <int CIN, int COUT, int EPI>
__global__ __launch_bounds__(256) void conv_mfma_kernel(
    const uint16_t* __restrict__ X, const uint16_t* __restrict__ Wf,
    const float* __restrict__ bias, uint16_t* __restrict__ Yb,
    float* __restrict__ Yf, const uint16_t* __restrict__ mask_act, int n,
    int64_t N, int cout_real) {
  constexpr int KC = CIN / 16, NT = COUT / 16;
  constexpr int SLICE = conv_slice<CIN, COUT>();  // bf16 of one dx slice
  constexpr int CS = conv_cs<CIN>();
  extern __shared__ __align__(16) uint16_t smem_conv[];
  uint16_t* wl = smem_conv;
  uint16_t* al = smem_conv + SLICE;
  const int lane = threadIdx.x & 63;
  const int row = lane & 15, grp = lane >> 4;
  const int64_t n2 = (int64_t)n * n;
  const int64_t vb = (int64_t)blockIdx.x * kConvVox;   // first voxel
  const int xb = (int)(vb / n2);
  const int yb = (int)((vb / n) % n);                  // first line
  const int nl = conv_lines(n);                        // staged lines
  const int64_t tile0 =
      ((int64_t)blockIdx.x * 4 + (threadIdx.x >> 6)) * kConvTPW;
  int ly0[kConvTPW], zs0[kConvTPW];
  bool ok[kConvTPW];
#pragma unroll
  for (int u = 0; u < kConvTPW; ++u) {
    const int64_t v0 = (tile0 + u) * 16;
    ok[u] = v0 < N;
    const int64_t vv = ok[u] ? v0 : vb;
    zs0[u] = (int)(vv % n);
    ly0[u] = (int)((vv / n) % n) - yb + 1;   // staged line of the tile
  }
  f32x4 acc[kConvTPW][NT];
#pragma unroll
  for (int u = 0; u < kConvTPW; ++u)
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[u][t] = (f32x4){0.f, 0.f, 0.f, 0.f};
  for (int sl = 0; sl < 3; ++sl) {
    const int dx = sl - 1;
    __syncthreads();
    {
      // the fragments of taps 9 sl .. 9 sl + 8 (8-byte copies: the fragment
      // arrays are 8-byte aligned, as every B-fragment load assumes)
      const uint2* src = reinterpret_cast<const uint2*>(Wf + (size_t)sl * SLICE);
      uint2* dst = reinterpret_cast<uint2*>(wl);
      for (int i = threadIdx.x; i < SLICE / 4; i += 256) dst[i] = src[i];
      // lines yb - 1 .. yb + nl - 2 (periodic) of plane x + dx, 16 bytes
      // (8 channels) at a time
      constexpr int CH = CIN / 8;
      const int xp = wrap(xb + dx, n);
      const int items = nl * n * CH;
      for (int i = threadIdx.x; i < items; i += 256) {
        const int c8 = i % CH;
        const int vz = i / CH;            // staged line * n + z
        const int j = vz / n, z = vz - (vz / n) * n;
        const int yg = (yb - 1 + j + 2 * n) % n;
        const uint4 val = *reinterpret_cast<const uint4*>(
            X + (((int64_t)xp * n + yg) * n + z) * CIN + 8 * c8);
        *reinterpret_cast<uint4*>(al + (int64_t)vz * CS + 8 * c8) = val;
      }
    }
    __syncthreads();
    for (int tl = 0; tl < 9; ++tl) {
      const int dy = tl / 3 - 1, dz = tl % 3 - 1;
      const uint16_t* ar[kConvTPW];
#pragma unroll
      for (int u = 0; u < kConvTPW; ++u) {
        const int zz = wrap(zs0[u] + row + dz, n);
        ar[u] = al + ((ly0[u] + dy) * n + zz) * CS + 4 * grp;
      }
#pragma unroll
      for (int kc = 0; kc < KC; ++kc) {
        bf16x4 b[NT];
#pragma unroll
        for (int nt = 0; nt < NT; ++nt)
          b[nt] = *reinterpret_cast<const bf16x4*>(
              wl + (((tl * KC + kc) * NT + nt) * 64 + lane) * 4);
        bf16x4 a[kConvTPW];
#pragma unroll
        for (int u = 0; u < kConvTPW; ++u)
          a[u] = *reinterpret_cast<const bf16x4*>(ar[u] + 16 * kc);
#pragma unroll
        for (int u = 0; u < kConvTPW; ++u)
#pragma unroll
          for (int nt = 0; nt < NT; ++nt)
            acc[u][nt] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(
                a[u], b[nt], acc[u][nt], 0, 0, 0);
      }
    }
  }
#pragma unroll
  for (int u = 0; u < kConvTPW; ++u) {
    if (!ok[u]) continue;
    const int64_t v0 = (tile0 + u) * 16;
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
      const int co = nt * 16 + row;
      // the bias has only the real output channels
      const float bv = (EPI == 2 || co >= cout_real) ? 0.f : bias[co];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int64_t v = v0 + 4 * grp + i;
        float val = acc[u][nt][i] + bv;
        if constexpr (EPI == 0) {
          Yb[v * COUT + co] = f2bf(val > 0.f ? val : 0.f);
        } else if constexpr (EPI == 1) {
          Yf[v * COUT + co] = val;
        } else {
          const float m = bf2f(mask_act[v * COUT + co]);
          Yb[v * COUT + co] = f2bf(m > 0.f ? val : 0.f);
        }
      }
    }
  }
}

// weight gradient partials: part[blk][27][CIN][COUT] for a chunk of voxels
// dW[t][i][o] = sum_v X[v + d_t][i] dZ[v][o]; MFMA with M = i, N = o,
// K = 16 voxels; each block handles one tap and one voxel chunk.
template <int CIN, int COUT>
__global__ __launch_bounds__(256) void conv_wgrad_kernel(
    const uint16_t* __restrict__ X, const uint16_t* __restrict__ dZ,
    float* __restrict__ part, int n, int64_t N, int64_t chunk) {
  constexpr int KC = CIN / 16, NT = COUT / 16;
  __shared__ float red[4][KC * NT * 16 * 16];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int tap = blockIdx.y;
  const int dx = tap / 9 - 1, dy = (tap / 3) % 3 - 1, dz = tap % 3 - 1;
  const int row = lane & 15, grp = lane >> 4;
  f32x4 acc[KC][NT];
#pragma unroll
  for (int a = 0; a < KC; ++a)
#pragma unroll
    for (int b = 0; b < NT; ++b) acc[a][b] = (f32x4){0.f, 0.f, 0.f, 0.f};
  const int64_t vbeg = (int64_t)blockIdx.x * chunk;
  const int64_t vend = (vbeg + chunk < N) ? vbeg + chunk : N;
  for (int64_t vk = vbeg + 16 * wv; vk < vend; vk += 64) {
    // K = 16 voxels vk .. vk+15 (same x, y row since n % 16 == 0)
    int64_t vsrc[4];
    int64_t vdst[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int64_t v = vk + 4 * grp + i;
      const int z = (int)(v % n), yy = (int)((v / n) % n),
                xx = (int)(v / ((int64_t)n * n));
      vsrc[i] = ((int64_t)wrap(xx + dx, n) * n + wrap(yy + dy, n)) * n +
                wrap(z + dz, n);
      vdst[i] = v;
    }
#pragma unroll
    for (int kc = 0; kc < KC; ++kc) {
      bf16x4 a;
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = (short)X[vsrc[i] * CIN + 16 * kc + row];
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) {
        bf16x4 b;
#pragma unroll
        for (int i = 0; i < 4; ++i) b[i] = (short)dZ[vdst[i] * COUT + 16 * nt + row];
        acc[kc][nt] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc[kc][nt], 0, 0, 0);
      }
    }
  }
  // D[4 grp + i][row] = dW[16 kc + 4 grp + i][16 nt + row]
#pragma unroll
  for (int kc = 0; kc < KC; ++kc)
#pragma unroll
    for (int nt = 0; nt < NT; ++nt)
#pragma unroll
      for (int i = 0; i < 4; ++i)
        red[wv][((kc * NT + nt) * 16 + 4 * grp + i) * 16 + row] = acc[kc][nt][i];
  __syncthreads();
  float* out = part + ((size_t)blockIdx.x * 27 + tap) * CIN * COUT;
  for (int e = threadIdx.x; e < KC * NT * 256; e += 256) {
    const float s = red[0][e] + red[1][e] + red[2][e] + red[3][e];
    const int kn = e / 256, r = (e / 16) % 16, c = e % 16;
    const int kc = kn / NT, nt = kn % NT;
    out[(16 * kc + r) * COUT + 16 * nt + c] = s;
  }
}

// sum the per-chunk partials in fixed order: dW[27*CIN*COUT]
__global__ void sum_parts_kernel(const float* __restrict__ part, int nparts,
                                 int64_t size, float* __restrict__ out) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < size;
       e += (int64_t)gridDim.x * blockDim.x) {
    double s = 0.0;
    for (int p = 0; p < nparts; ++p) s += part[(size_t)p * size + e];
    out[e] = (float)s;
  }
}

// bias gradient db[o] = sum_v dZ[v][o] (fixed order per block, then blocks)
template <int COUT>
__global__ __launch_bounds__(256) void bias_grad_kernel(
    const uint16_t* __restrict__ dZ, const float* __restrict__ dYf,
    int64_t N, float* __restrict__ part) {
  __shared__ float red[256];
  for (int o = 0; o < COUT; ++o) {
    float s = 0.f;
    for (int64_t v = (int64_t)blockIdx.x * 256 + threadIdx.x; v < N;
         v += (int64_t)gridDim.x * 256)
      s += dZ ? bf2f(dZ[v * COUT + o]) : dYf[v * COUT + o];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
      if (threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
      __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x * COUT + o] = red[0];
    __syncthreads();
  }
}

// loss L = mean over N*COUT_REAL of (Y - T)^2 and dY = 2 (Y - T)/count,
// written as bf16 (input of the backward convolutions) and f32
__global__ __launch_bounds__(256) void mse_kernel(
    const float* __restrict__ Y, const float* __restrict__ T, int cpad,
    int creal, int64_t N, uint16_t* __restrict__ dYb, float* __restrict__ dYf,
    double* __restrict__ part) {
  __shared__ double red[256];
  const double inv = 1.0 / ((double)N * creal);
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < N * cpad;
       i += (int64_t)gridDim.x * 256) {
    const int c = (int)(i % cpad);
    float g = 0.f;
    if (c < creal) {
      const float d = Y[i] - T[i];
      s += (double)d * d;
      g = (float)(2.0 * d * inv);
    }
    dYb[i] = f2bf(g);
    dYf[i] = g;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if (threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0] * inv;
}

// Adam on the FP32 master parameters (Kingma & Ba), in place
__global__ void adam_kernel(float* __restrict__ w, const float* __restrict__ g,
                            float* __restrict__ m, float* __restrict__ v,
                            int64_t size, float lr, float b1, float b2,
                            float eps, float c1, float c2) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < size;
       i += (int64_t)gridDim.x * blockDim.x) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    w[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  }
}

// master W[27][cin][cout] -> MFMA B fragments for the forward pass, and the
// flipped, transposed fragments of the backward-data pass
// (W'[26 - t][o][i] = W[t][i][o]); padded channels are zero
__global__ void pack_kernel(const float* __restrict__ W, int cin, int cout,
                            int CIN, int COUT, uint16_t* __restrict__ Wf,
                            uint16_t* __restrict__ Wb) {
  const int KC = CIN / 16, NT = COUT / 16;
  const int64_t total = (int64_t)27 * KC * NT * 64 * 4;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(e % 4);
    const int lane = (int)((e / 4) % 64);
    const int64_t f = e / 256;
    const int nt = (int)(f % NT), kc = (int)((f / NT) % KC), t = (int)(f / (NT * KC));
    const int ci = 16 * kc + 4 * (lane / 16) + i, co = 16 * nt + lane % 16;
    const float val = (ci < cin && co < cout) ? W[((size_t)t * cin + ci) * cout + co] : 0.f;
    Wf[e] = f2bf(val);
  }
  // backward data: input channels = COUT, output channels = CIN
  const int KCb = COUT / 16, NTb = CIN / 16;
  const int64_t totb = (int64_t)27 * KCb * NTb * 64 * 4;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < totb;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(e % 4);
    const int lane = (int)((e / 4) % 64);
    const int64_t f = e / 256;
    const int nt = (int)(f % NTb), kc = (int)((f / NTb) % KCb), t = (int)(f / (NTb * KCb));
    const int o = 16 * kc + 4 * (lane / 16) + i, ci = 16 * nt + lane % 16;
    const int ts = 26 - t;
    const float val = (ci < cin && o < cout) ? W[((size_t)ts * cin + ci) * cout + o] : 0.f;
    Wb[e] = f2bf(val);
  }
}

// ----------------------------------------------------------------- launchers
namespace {
template <int CIN, int COUT, int EPI>
void conv_t(const uint16_t* X, const uint16_t* Wf, const float* b, uint16_t* Yb,
            float* Yf, const uint16_t* mask, int n, int64_t N, int creal,
            hipStream_t s) {
  const size_t lds = conv_lds_bytes<CIN, COUT>(n);
  if (lds > 160 * 1024) throw Error(-1, "convolution grid edge too large");
  if (lds > 64 * 1024) {
    // dynamic LDS above 64 KiB is allowed per kernel (once is enough: the
    // attribute only raises the cap)
    static size_t allowed = 0;
    if (lds > allowed) {
      RVE_HIP(hipFuncSetAttribute(
          reinterpret_cast<const void*>(&conv_mfma_kernel<CIN, COUT, EPI>),
          hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
      allowed = lds;
    }
  }
  hipLaunchKernelGGL((conv_mfma_kernel<CIN, COUT, EPI>),
                     dim3((unsigned)((N + kConvVox - 1) / kConvVox)),
                     dim3(256), lds, s, X, Wf, b, Yb, Yf, mask, n, N, creal);
}
}  // namespace

void nn_conv(int cin, int cout, int epi, const uint16_t* X, const uint16_t* Wf,
             const float* b, uint16_t* Yb, float* Yf, const uint16_t* mask,
             int n, int64_t N, int cout_real, hipStream_t s) {
  if (n % 16 || N != (int64_t)n * n * n)
    throw Error(-1, "convolution grid must be n^3 with n % 16 == 0");
#define RVE_CONV(CI, CO)                                                      \
  if (cin == CI && cout == CO) {                                              \
    if (epi == 0) conv_t<CI, CO, 0>(X, Wf, b, Yb, Yf, mask, n, N, cout_real, s);      \
    else if (epi == 1) conv_t<CI, CO, 1>(X, Wf, b, Yb, Yf, mask, n, N, cout_real, s); \
    else conv_t<CI, CO, 2>(X, Wf, b, Yb, Yf, mask, n, N, cout_real, s);               \
    return;                                                                   \
  }
  RVE_CONV(48, 32)
  RVE_CONV(32, 32)
  RVE_CONV(32, 16)
  RVE_CONV(16, 32)
  RVE_CONV(32, 48)
#undef RVE_CONV
  throw Error(-1, "unsupported convolution shape");
}

void nn_wgrad(int cin, int cout, const uint16_t* X, const uint16_t* dZ,
              float* part, int nchunks, int64_t chunk, int n, int64_t N,
              hipStream_t s) {
  dim3 grid((unsigned)nchunks, 27);
  if (cin == 48 && cout == 32)
    hipLaunchKernelGGL((conv_wgrad_kernel<48, 32>), grid, dim3(256), 0, s, X, dZ, part, n, N, chunk);
  else if (cin == 32 && cout == 32)
    hipLaunchKernelGGL((conv_wgrad_kernel<32, 32>), grid, dim3(256), 0, s, X, dZ, part, n, N, chunk);
  else if (cin == 32 && cout == 16)
    hipLaunchKernelGGL((conv_wgrad_kernel<32, 16>), grid, dim3(256), 0, s, X, dZ, part, n, N, chunk);
  else
    throw Error(-1, "unsupported weight-gradient shape");
}

void nn_sum_parts(const float* part, int nparts, int64_t size, float* out,
                  hipStream_t s) {
  hipLaunchKernelGGL(sum_parts_kernel, dim3(256), dim3(256), 0, s, part, nparts,
                     size, out);
}

void nn_bias_grad(int cout, const uint16_t* dZ, const float* dYf, int64_t N,
                  float* part, int nblk, hipStream_t s) {
  if (cout == 32)
    hipLaunchKernelGGL((bias_grad_kernel<32>), dim3(nblk), dim3(256), 0, s, dZ, dYf, N, part);
  else if (cout == 16)
    hipLaunchKernelGGL((bias_grad_kernel<16>), dim3(nblk), dim3(256), 0, s, dZ, dYf, N, part);
  else
    throw Error(-1, "unsupported bias-gradient width");
}

void nn_mse(const float* Y, const float* T, int cpad, int creal, int64_t N,
            uint16_t* dYb, float* dYf, double* part, int nblk, hipStream_t s) {
  hipLaunchKernelGGL(mse_kernel, dim3(nblk), dim3(256), 0, s, Y, T, cpad, creal,
                     N, dYb, dYf, part);
}

void nn_adam(float* w, const float* g, float* m, float* v, int64_t size,
             float lr, float b1, float b2, float eps, int step, hipStream_t s) {
  const float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
  hipLaunchKernelGGL(adam_kernel, dim3(256), dim3(256), 0, s, w, g, m, v, size,
                     lr, b1, b2, eps, c1, c2);
}

void nn_pack(const float* W, int cin, int cout, int CIN, int COUT, uint16_t* Wf,
             uint16_t* Wb, hipStream_t s) {
  hipLaunchKernelGGL(pack_kernel, dim3(128), dim3(256), 0, s, W, cin, cout, CIN,
                     COUT, Wf, Wb);
}


// padded [27][CIN][COUT] -> real [27][cin][cout]
__global__ void unpad_kernel(const float* __restrict__ src, int CIN, int COUT,
                             int cin, int cout, float* __restrict__ dst) {
  const int64_t total = (int64_t)27 * cin * cout;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int o = (int)(e % cout), i = (int)((e / cout) % cin),
              t = (int)(e / ((int64_t)cin * cout));
    dst[e] = src[((size_t)t * CIN + i) * COUT + o];
  }
}

void nn_unpad(const float* src, int CIN, int COUT, int cin, int cout,
              float* dst, hipStream_t s) {
  hipLaunchKernelGGL(unpad_kernel, dim3(128), dim3(256), 0, s, src, CIN, COUT,
                     cin, cout, dst);
}

// network input of one increment (channels, kFeat padded):
//   0-8   (Fbar_k - Fbar_{k-1}) / s_k                 (broadcast)
//   9-17  fluctuation increment of increment k-1 / s_{k-1}
//   18-26 100 (F_{k-1} - Fbar_{k-1})                   (current fluctuation)
//   27-35 orientation matrix of the voxel's grain (zero in particles)
//   36    particle flag
//   37    reversal indicator dFbar_k : dFbar_{k-1} / (s_k s_{k-1})
//   38    sum_a |dgamma_a| of increment k-1 / s_{k-1}
//   39    1
__global__ void features_kernel(FeatArgs a) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= a.N) return;
  const int64_t N = a.N;
  const double* tb = a.table + (int64_t)a.phase[v] * kTableStride;
  const bool part = tb[0] != 0.0;
  float f[kFeat];
#pragma unroll
  for (int c = 0; c < kFeat; ++c) f[c] = 0.f;
#pragma unroll
  for (int c = 0; c < 9; ++c) {
    f[c] = (float)a.dfbar_n[c];
    f[9 + c] = (float)(a.dFt_prev[c * N + v] * a.inv_s_prev);
    f[18 + c] = (float)(100.0 * (a.Fprev[c * N + v] - a.fbar_prev[c]));
    f[27 + c] = part ? 0.f : (float)tb[kTabR + c];
  }
  f[36] = part ? 1.f : 0.f;
  f[37] = (float)a.reversal;
  double sg = 0.0;
#pragma unroll
  for (int al = 0; al < 12; ++al) sg += fabs(a.dg_prev[al * N + v]);
  f[38] = (float)(sg * a.inv_s_prev);
  f[39] = 1.f;
  uint16_t* out = a.X + v * kFeat;
#pragma unroll
  for (int c = 0; c < kFeat; ++c) out[c] = f2bf(f[c]);
}

void nn_features(const FeatArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(features_kernel, dim3((unsigned)((a.N + 255) / 256)),
                     dim3(256), 0, s, a);
}

// T[v][c] = dFt[c][v] / s for c < 9, zero padding up to kOut
__global__ void target_kernel(const double* __restrict__ dFt, double inv_s,
                              const double* __restrict__ dFt2, double coef,
                              float* __restrict__ T, int64_t N) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= N) return;
#pragma unroll
  for (int c = 0; c < kOut; ++c)
    T[v * kOut + c] = (c < kOutReal) ? (float)(dFt[c * N + v] * inv_s -
                                               coef * dFt2[c * N + v])
                                     : 0.f;
}

void nn_target(const double* dFt, double inv_s, const double* dFt2,
               double coef, float* T, int64_t N, hipStream_t s) {
  hipLaunchKernelGGL(target_kernel, dim3((unsigned)((N + 255) / 256)), dim3(256),
                     0, s, dFt, inv_s, dFt2, coef, T, N);
}

// out[c][v] = scale * Y[v][c], c < 9
__global__ void out_field_kernel(const float* __restrict__ Y, double scale,
                                 double* __restrict__ out, int64_t N) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= N) return;
#pragma unroll
  for (int c = 0; c < kOutReal; ++c) out[c * N + v] = scale * (double)Y[v * kOut + c];
}

void nn_output_to_field(const float* Y, double scale, double* out, int64_t N,
                        hipStream_t s) {
  hipLaunchKernelGGL(out_field_kernel, dim3((unsigned)((N + 255) / 256)),
                     dim3(256), 0, s, Y, scale, out, N);
}

// fluctuation increment of a converged increment: F_k - F_{k-1} - dFbar
__global__ void fluct_kernel(const double* __restrict__ Fn,
                             const double* __restrict__ Fo, double d0,
                             double d1, double d2, double d3, double d4,
                             double d5, double d6, double d7, double d8,
                             double* __restrict__ out, int64_t N) {
  const double d[9] = {d0, d1, d2, d3, d4, d5, d6, d7, d8};
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < 9 * N;
       i += (int64_t)gridDim.x * blockDim.x)
    out[i] = Fn[i] - Fo[i] - d[i / N];
}

void nn_fluct_increment(const double* Fnew, const double* Fold,
                        const double dFbar[9], double* out, int64_t N,
                        hipStream_t s) {
  hipLaunchKernelGGL(fluct_kernel, dim3(2048), dim3(256), 0, s, Fnew, Fold,
                     dFbar[0], dFbar[1], dFbar[2], dFbar[3], dFbar[4], dFbar[5],
                     dFbar[6], dFbar[7], dFbar[8], out, N);
}

__global__ void axpy_kernel(double* __restrict__ F, const double* __restrict__ d,
                            double a, int64_t n9) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n9;
       i += (int64_t)gridDim.x * blockDim.x)
    F[i] += a * d[i];
}

void nn_axpy_field(double* F, const double* d, double a, int64_t n9,
                   hipStream_t s) {
  hipLaunchKernelGGL(axpy_kernel, dim3(2048), dim3(256), 0, s, F, d, a, n9);
}

}  // namespace rve
