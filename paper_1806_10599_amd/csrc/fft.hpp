// Mixed-radix FFT building blocks for lines held in LDS (gfx950).
//
// A line of length N lives at LDS addresses map(line, e), e = 0..N-1; the map
// lets the slab kernels transform rows, packed columns and pencils without
// copying.  Each Stockham pass (self-sorting, decimation in time) reads the
// R inputs j + r N/R of butterfly j, applies the twiddles
// exp(DIR 2 pi i r (j mod Ns) / (Ns R)), does an R-point DFT in registers and
// writes the outputs to (j div Ns) Ns R + (j mod Ns) + r Ns.  All reads of a
// line finish (barrier) before any write, so a pass works in place.  Lines
// are processed in chunks of whole lines so that every thread owns at most
// one butterfly per pass.  Twiddles come from a per-size table
// tw[m] = exp(-2 pi i m / N) computed on the host in FP64.
#pragma once

#include "common.hpp"

namespace rve {

// ---------------------------------------------------------------- small DFTs
// DIR = -1: X_k = sum_r v_r exp(-2 pi i r k / R); DIR = +1: conjugate kernel.

template <int DIR, typename T>
__device__ __forceinline__ cplx<T> mul_dir_i(cplx<T> a) {  // a * (DIR i)
  return {-T(DIR) * a.y, T(DIR) * a.x};
}

template <int DIR, typename T>
__device__ __forceinline__ void dft2(cplx<T>& a, cplx<T>& b) {
  cplx<T> t = a;
  a = cadd(t, b);
  b = csub(t, b);
}

template <int DIR, typename T>
__device__ __forceinline__ void dft4(cplx<T>& v0, cplx<T>& v1, cplx<T>& v2,
                                     cplx<T>& v3) {
  cplx<T> t0 = cadd(v0, v2), t1 = csub(v0, v2);
  cplx<T> t2 = cadd(v1, v3), t3 = mul_dir_i<DIR>(csub(v1, v3));
  v0 = cadd(t0, t2);
  v2 = csub(t0, t2);
  v1 = cadd(t1, t3);
  v3 = csub(t1, t3);
}

template <int DIR, typename T>
__device__ __forceinline__ void dft3(cplx<T>* v) {
  const T c = T(-0.5);
  const T s = T(DIR) * T(0.86602540378443864676);  // sin(2 pi / 3)
  cplx<T> t = cadd(v[1], v[2]), u = csub(v[1], v[2]);
  cplx<T> m = {v[0].x + c * t.x, v[0].y + c * t.y};
  cplx<T> iu = {-s * u.y, s * u.x};  // i s u
  v[0] = cadd(v[0], t);
  v[1] = cadd(m, iu);
  v[2] = csub(m, iu);
}

template <int DIR, typename T>
__device__ __forceinline__ void dft5(cplx<T>* v) {
  const T c1 = T(0.30901699437494742410);   // cos(2 pi / 5)
  const T c2 = T(-0.80901699437494742410);  // cos(4 pi / 5)
  const T s1 = T(DIR) * T(0.95105651629515357212);  // sin(2 pi / 5)
  const T s2 = T(DIR) * T(0.58778525229247312917);  // sin(4 pi / 5)
  cplx<T> t1 = cadd(v[1], v[4]), t2 = cadd(v[2], v[3]);
  cplx<T> u1 = csub(v[1], v[4]), u2 = csub(v[2], v[3]);
  cplx<T> a1 = {v[0].x + c1 * t1.x + c2 * t2.x, v[0].y + c1 * t1.y + c2 * t2.y};
  cplx<T> a2 = {v[0].x + c2 * t1.x + c1 * t2.x, v[0].y + c2 * t1.y + c1 * t2.y};
  cplx<T> b1 = {s1 * u1.x + s2 * u2.x, s1 * u1.y + s2 * u2.y};
  cplx<T> b2 = {s2 * u1.x - s1 * u2.x, s2 * u1.y - s1 * u2.y};
  cplx<T> ib1 = {-b1.y, b1.x}, ib2 = {-b2.y, b2.x};
  v[0] = cadd(v[0], cadd(t1, t2));
  v[1] = cadd(a1, ib1);
  v[4] = csub(a1, ib1);
  v[2] = cadd(a2, ib2);
  v[3] = csub(a2, ib2);
}

template <int DIR, typename T>
__device__ __forceinline__ void dft8(cplx<T>* v) {
  // even/odd split into two 4-point DFTs, then W8^k twiddles
  cplx<T> e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6];
  cplx<T> o0 = v[1], o1 = v[3], o2 = v[5], o3 = v[7];
  dft4<DIR>(e0, e1, e2, e3);
  dft4<DIR>(o0, o1, o2, o3);
  const T h = T(0.70710678118654752440);
  // W8^1 = h (1 + DIR i), W8^2 = DIR i, W8^3 = h (-1 + DIR i)
  cplx<T> w1 = {h * (o1.x - T(DIR) * o1.y), h * (o1.y + T(DIR) * o1.x)};
  cplx<T> w2 = mul_dir_i<DIR>(o2);
  cplx<T> w3 = {h * (-o3.x - T(DIR) * o3.y), h * (-o3.y + T(DIR) * o3.x)};
  v[0] = cadd(e0, o0);
  v[4] = csub(e0, o0);
  v[1] = cadd(e1, w1);
  v[5] = csub(e1, w1);
  v[2] = cadd(e2, w2);
  v[6] = csub(e2, w2);
  v[3] = cadd(e3, w3);
  v[7] = csub(e3, w3);
}

template <int DIR, typename T>
__device__ __forceinline__ void dft16(cplx<T>* v) {
  // 4 x 4: columns r2 over r1, twiddle W16^{r2 k1}, rows over r2
  cplx<T> y[16];
#pragma unroll
  for (int r2 = 0; r2 < 4; ++r2) {
    cplx<T> a = v[r2], b = v[4 + r2], c = v[8 + r2], d = v[12 + r2];
    dft4<DIR>(a, b, c, d);
    y[0 * 4 + r2] = a;
    y[1 * 4 + r2] = b;
    y[2 * 4 + r2] = c;
    y[3 * 4 + r2] = d;
  }
  const T c1 = T(0.92387953251128675613), s1 = T(0.38268343236508977173);
  const T h = T(0.70710678118654752440);
  // W16^m = (cos(2 pi m/16), DIR sin(2 pi m/16)) for m = r2 k1
  const cplx<T> W[10] = {{T(1), T(0)},
                         {c1, T(DIR) * s1},
                         {h, T(DIR) * h},
                         {s1, T(DIR) * c1},
                         {T(0), T(DIR)},
                         {-s1, T(DIR) * c1},
                         {-h, T(DIR) * h},
                         {-c1, T(DIR) * s1},
                         {T(-1), T(0)},
                         {-c1, -T(DIR) * s1}};
#pragma unroll
  for (int k1 = 1; k1 < 4; ++k1)
#pragma unroll
    for (int r2 = 1; r2 < 4; ++r2) y[k1 * 4 + r2] = cmul(y[k1 * 4 + r2], W[k1 * r2]);
#pragma unroll
  for (int k1 = 0; k1 < 4; ++k1) {
    cplx<T> a = y[k1 * 4 + 0], b = y[k1 * 4 + 1], c = y[k1 * 4 + 2],
            d = y[k1 * 4 + 3];
    dft4<DIR>(a, b, c, d);
    v[k1] = a;
    v[k1 + 4] = b;
    v[k1 + 8] = c;
    v[k1 + 12] = d;
  }
}

template <int R, int DIR, typename T>
__device__ __forceinline__ void dft_small(cplx<T>* v) {
  if constexpr (R == 2) {
    dft2<DIR>(v[0], v[1]);
  } else if constexpr (R == 3) {
    dft3<DIR>(v);
  } else if constexpr (R == 4) {
    dft4<DIR>(v[0], v[1], v[2], v[3]);
  } else if constexpr (R == 5) {
    dft5<DIR>(v);
  } else if constexpr (R == 8) {
    dft8<DIR>(v);
  } else if constexpr (R == 16) {
    dft16<DIR>(v);
  } else {
    static_assert(R == 2, "unsupported radix");
  }
}

// --------------------------------------------------------- Stockham passes
template <int N, int R, int NS, int DIR, typename T, class Map>
__device__ __forceinline__ void stockham_pass(cplx<T>* lds, const cplx<T>* tw,
                                              int nlines, const Map& map) {
  constexpr int BPL = N / R;  // butterflies per line
  const int lpc = (int)blockDim.x / BPL;
  const int t = threadIdx.x;
  // lines vary fastest across threads: the 32 lanes of a half-wave touch 32
  // different lines at the same element, which the odd LDS pitches (and the
  // column and pencil maps) place in distinct banks
  const int lo = t % lpc;
  const int j = t / lpc;
  const bool lane_ok = j < BPL;
  const int k = j % NS;
  for (int l0 = 0; l0 < nlines; l0 += lpc) {
    const int l = l0 + lo;
    const bool active = lane_ok && l < nlines;
    cplx<T> v[R];
    if (active) {
#pragma unroll
      for (int r = 0; r < R; ++r) v[r] = lds[map(l, j + r * BPL)];
      if constexpr (NS > 1) {
#pragma unroll
        for (int r = 1; r < R; ++r) {
          cplx<T> w = tw[(r * k * (N / (NS * R))) % N];
          if constexpr (DIR > 0) w.y = -w.y;
          v[r] = cmul(v[r], w);
        }
      }
    }
    __syncthreads();
    if (active) {
      dft_small<R, DIR>(v);
      const int base = (j / NS) * NS * R + k;
#pragma unroll
      for (int r = 0; r < R; ++r) lds[map(l, base + r * NS)] = v[r];
    }
    __syncthreads();
  }
}

// Full N-point transform of nlines lines; the radix plan per supported size.
template <int N, int DIR, typename T, class Map>
__device__ __forceinline__ void fft_lines(cplx<T>* lds, const cplx<T>* tw,
                                          int nlines, const Map& map) {
  if constexpr (N == 16) {
    stockham_pass<N, 4, 1, DIR>(lds, tw, nlines, map);
    stockham_pass<N, 4, 4, DIR>(lds, tw, nlines, map);
  } else if constexpr (N == 24) {
    stockham_pass<N, 8, 1, DIR>(lds, tw, nlines, map);
    stockham_pass<N, 3, 8, DIR>(lds, tw, nlines, map);
  } else if constexpr (N == 32) {
    stockham_pass<N, 8, 1, DIR>(lds, tw, nlines, map);
    stockham_pass<N, 4, 8, DIR>(lds, tw, nlines, map);
  } else if constexpr (N == 40) {
    stockham_pass<N, 8, 1, DIR>(lds, tw, nlines, map);
    stockham_pass<N, 5, 8, DIR>(lds, tw, nlines, map);
  } else if constexpr (N == 48) {
    stockham_pass<N, 16, 1, DIR>(lds, tw, nlines, map);
    stockham_pass<N, 3, 16, DIR>(lds, tw, nlines, map);
  } else if constexpr (N == 64) {
    stockham_pass<N, 8, 1, DIR>(lds, tw, nlines, map);
    stockham_pass<N, 8, 8, DIR>(lds, tw, nlines, map);
  } else if constexpr (N == 96) {
    stockham_pass<N, 8, 1, DIR>(lds, tw, nlines, map);
    stockham_pass<N, 4, 8, DIR>(lds, tw, nlines, map);
    stockham_pass<N, 3, 32, DIR>(lds, tw, nlines, map);
  } else if constexpr (N == 128) {
    stockham_pass<N, 8, 1, DIR>(lds, tw, nlines, map);
    stockham_pass<N, 16, 8, DIR>(lds, tw, nlines, map);
  } else {
    static_assert(N == 16, "unsupported FFT length");
  }
}

}  // namespace rve
