// Non-local fatigue indicators (Sec. 3.3, Eqs. 25-26): segment means over
// voxel lists and the maxima over segments.  One 64-lane wavefront per
// grain or band: each lane sums a fixed stride of the segment's voxels, a
// butterfly over the wavefront completes the sum, so every launch adds in
// the same order.
#include <cmath>

#include "fips.hpp"

namespace rve {

namespace {

__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) x += __shfl_xor(x, m, 64);
  return x;
}

__global__ __launch_bounds__(256) void fip_grain_kernel(
    const int32_t* __restrict__ vox, const FipSeg* __restrict__ seg, int nseg,
    const double* __restrict__ pcyc, const double* __restrict__ pcyc_lit,
    int64_t base, double* __restrict__ out) {
  const int w = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (w >= nseg) return;  // the whole wavefront leaves together
  const FipSeg sg = seg[w];
  double a = 0.0, b = 0.0;
  for (int i = lane; i < sg.len; i += 64) {
    const int64_t v = base + vox[sg.off + i];
    a += pcyc[v];
    b += pcyc_lit[v];
  }
  a = wave_sum(a);
  b = wave_sum(b);
  if (lane == 0) {
    out[w] = a / (double)sg.len;
    out[nseg + w] = b / (double)sg.len;
  }
}

__global__ __launch_bounds__(256) void fip_band_kernel(
    const int32_t* __restrict__ vox, const FipSeg* __restrict__ seg, int nseg,
    const double* __restrict__ W, int64_t cstride, int64_t base,
    double* __restrict__ val, int32_t* __restrict__ sys) {
  const int w = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (w >= nseg) return;
  const FipSeg sg = seg[w];
  const double* W0 = W + (int64_t)sg.comp * cstride + base;
  double s0 = 0.0, s1 = 0.0, s2 = 0.0;
  for (int i = lane; i < sg.len; i += 64) {
    const int64_t v = vox[sg.off + i];
    s0 += W0[v];
    s1 += W0[cstride + v];
    s2 += W0[2 * cstride + v];
  }
  s0 = wave_sum(s0);
  s1 = wave_sum(s1);
  s2 = wave_sum(s2);
  if (lane == 0) {
    const double cnt = (double)sg.len;
    const double m0 = s0 / cnt, m1 = s1 / cnt, m2 = s2 / cnt;
    int k = 0;
    double m = m0;
    if (m1 > m) { m = m1; k = 1; }
    if (m2 > m) { m = m2; k = 2; }
    val[w] = m;
    sys[w] = sg.comp + k;
  }
}

// largest value and its first index (one block)
__global__ __launch_bounds__(256) void fip_argmax_kernel(
    const double* __restrict__ v, int64_t n, FipMax* __restrict__ out) {
  __shared__ double sv[256];
  __shared__ int64_t si[256];
  const int t = threadIdx.x;
  double best = -INFINITY;
  int64_t bi = -1;
  for (int64_t i = t; i < n; i += 256)
    if (bi < 0 || v[i] > best) {
      best = v[i];
      bi = i;
    }
  sv[t] = best;
  si[t] = bi;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (t < s) {
      const double ov = sv[t + s];
      const int64_t oi = si[t + s];
      if (oi >= 0 && (si[t] < 0 || ov > sv[t] || (ov == sv[t] && oi < si[t]))) {
        sv[t] = ov;
        si[t] = oi;
      }
    }
    __syncthreads();
  }
  if (t == 0) {
    out->val = sv[0];
    out->idx = (int32_t)si[0];
    out->pad = 0;
  }
}

}  // namespace

void launch_fip_grain_means(const int32_t* vox, const FipSeg* seg, int nseg,
                            const double* pcyc, const double* pcyc_lit,
                            int64_t base, double* out, hipStream_t s) {
  if (nseg <= 0) return;
  hipLaunchKernelGGL(fip_grain_kernel, dim3((nseg + 3) / 4), dim3(256), 0, s,
                     vox, seg, nseg, pcyc, pcyc_lit, base, out);
}

void launch_fip_band_means(const int32_t* vox, const FipSeg* seg, int nseg,
                           const double* w, int64_t cstride, int64_t base,
                           double* val, int32_t* sys, hipStream_t s) {
  if (nseg <= 0) return;
  hipLaunchKernelGGL(fip_band_kernel, dim3((nseg + 3) / 4), dim3(256), 0, s,
                     vox, seg, nseg, w, cstride, base, val, sys);
}

void launch_fip_argmax(const double* v, int64_t n, FipMax* out, hipStream_t s) {
  hipLaunchKernelGGL(fip_argmax_kernel, dim3(1), dim3(256), 0, s, v, n, out);
}

}  // namespace rve
