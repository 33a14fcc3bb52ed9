// The linear map G(A) = F^-1{ Ghat : F(A) } of Sec. 2.1, Eqs. 10-11, and the
// CG matvec G(K : p) of Eqs. 15-16, as three passes over a cubic grid of N^3
// voxels:
//
//   pass A (one block per x-slab and component group): build the real plane
//     (the field itself, or K:p with the CG direction update fused in), pack
//     rows y and y + N/2 as one complex line, FFT along z, unpack the two
//     half spectra in place (kz < N/2; the kz = N/2 Nyquist plane is zeroed
//     by the operator, so its slots hold the kz = 0 column's second half),
//     FFT along y, store the spectrum [c][x][ky][kz] (kz < N/2).
//   pass B (one block per ky and a tile of kz, for one tensor row i): FFT
//     along x of the three components of row i, apply the projection
//     Bhat_ij = v_j (sum_l Ahat_il v_l) / |v|^2 (zero at the null frequency
//     and wherever a component is Nyquist; Sec. 2.2, Eqs. 18-21), fold in
//     the 1/N^3 of the inverse transform, inverse FFT along x.
//   pass C (one block per x-slab and component group): inverse of pass A,
//     writing the real field and a per-block FP64 partial (||out||^2, or the
//     batched CG's dot p . Ap), or, in a single-RVE CG iteration, applying
//     r -= alpha G(K:p) in place with the partials of the new r . r.
//
// Only the delta_ik structure of the operator is used: row i of the output
// depends on row i of the input, so pass B never needs all nine components.
#include "batch_cg.hpp"
#include "cg_scalars.hpp"
#include "common.hpp"
#include "fft.hpp"
#include "kernels.hpp"

namespace rve {

template <int N>
struct SlabGeom {
  static constexpr int H = N / 2;
  static constexpr int PITCH = N + 1;                 // LDS row pitch (complex)
  static constexpr int PLANE = H * PITCH;             // one packed plane
};

// rows of the packed plane: line = q*H + y', element = z
template <int N>
struct RowMap {
  __device__ __forceinline__ int operator()(int line, int e) const {
    const int q = line / SlabGeom<N>::H;
    const int yp = line - q * SlabGeom<N>::H;
    return q * SlabGeom<N>::PLANE + yp * SlabGeom<N>::PITCH + e;
  }
};

// spectral columns: line = q*H + kz, element = ky
template <int N>
struct ColMap {
  __device__ __forceinline__ int operator()(int line, int y) const {
    constexpr int H = SlabGeom<N>::H;
    const int q = line / H;
    const int kz = line - q * H;
    int row, col;
    if (y < H) {
      row = y;
      col = kz;
    } else {
      row = y - H;
      col = (kz == 0) ? H : N - kz;
    }
    return q * SlabGeom<N>::PLANE + row * SlabGeom<N>::PITCH + col;
  }
};

__device__ __forceinline__ int xcd_remap(int b, int nb) {
  // consecutive workgroups land on different XCDs (round robin over 8);
  // give neighbouring logical tiles the same XCD so they share its L2
  if (nb % 8) return b;
  return (b % 8) * (nb / 8) + b / 8;
}

__device__ __forceinline__ double block_sum(double v, double* red) {
  // fixed-order reduction over the block (deterministic)
  return block_sum_fixed(v, red);
}

// items whose global loads are issued together before their LDS stores:
// FP32 eight, or 32 on grids of 128 (whose slab planes leave two blocks per
// CU, so that the registers are there), which makes each pass's loads one
// chunk in flight at once; FP64 one
template <typename T, int N>
constexpr int kStage = sizeof(T) == 4 ? (N >= 128 ? 32 : 8) : 1;

// The twiddles of a body.  DEFER (an FP32 body whose data loads are one
// chunk per thread): loaded into a register at its start (one per thread,
// N <= kBlock) and written to LDS once the data loads are in flight, so
// that their latency overlaps that of the data; otherwise written to LDS
// at once (kept in a register across a loop of chunks, the value would be
// parked in scratch memory).
template <typename T, int N>
constexpr bool kDeferTw(int per) {
  return sizeof(T) == 4 && per <= kStage<T, N>;
}
template <typename T, int N, bool DEFER>
struct TwiddleStage {
  static_assert(N <= kBlock, "one twiddle per thread");
  cplx<T> v;
  __device__ __forceinline__ void load(const cplx<T>* __restrict__ g,
                                       cplx<T>* tw) {
    if constexpr (DEFER)
      v = g[(int)threadIdx.x < N ? (int)threadIdx.x : N - 1];  // no branch
    else if ((int)threadIdx.x < N)
      tw[threadIdx.x] = g[threadIdx.x];
  }
  __device__ __forceinline__ void store(cplx<T>* tw) const {
    if constexpr (DEFER)
      if ((int)threadIdx.x < N) tw[threadIdx.x] = v;
  }
};

// A run's stop flag, read when a body starts and consulted once its first
// data loads are issued (a stopped CG run's passes return without work).
// The relaxed atomic read makes it a vector load issued ahead of the data
// loads, whose in-order completion lets the check wait for it alone; a
// scalar load would be waited for together with the kernel arguments,
// before any data load is issued.
__device__ __forceinline__ int32_t stop_flag(const Scalars* gate) {
  return gate ? __hip_atomic_load(&gate->done, __ATOMIC_RELAXED,
                                  __HIP_MEMORY_SCOPE_AGENT)
              : 0;
}
// The flag's first use: an empty statement that takes the register, so
// that the compiler neither tests the flag (and waits for its load) before
// this point nor moves the data loads above it.
__device__ __forceinline__ bool stopped_now(int32_t f) {
  asm volatile("" : "+v"(f));
  return f != 0;
}

// ------------------------------------------------------------------ pass A
// lb: logical block within this RVE's pass-A grid
// gate: the run's scalars when the pass must return at once on a stopped
// run (returns false then); with SRC_KP the check precedes all work
template <typename T, int N, int CPB, int SRC>
__device__ __forceinline__ bool slab_fwd_body(const SlabFwdArgs<T>& a, int lb,
                                              cplx<T>* lds, cplx<T>* tw,
                                              double* red,
                                              const KpStep<T>& st,
                                              const Scalars* gate = nullptr) {
  constexpr int H = N / 2;
  constexpr int NG = 9 / CPB;
  const int64_t cs = a.cs;
  const int x = lb / NG;
  const int grp = lb - x * NG;
  const int32_t stopped = stop_flag(gate);
  if (SRC == SRC_KP && stopped_now(stopped)) return false;
  constexpr int PER0 = (H * N + kBlock - 1) / kBlock;
  TwiddleStage<T, N, SRC == SRC_FIELD && kDeferTw<T, N>(PER0)> tws;
  tws.load(a.tw, tw);
  double ss[CPB], s1[CPB];
#pragma unroll
  for (int q = 0; q < CPB; ++q) ss[q] = s1[q] = 0.0;

  // build the real plane(s), packed: row y' holds y' (re) and y'+H (im);
  // each thread builds both rows of a (y', z) slot and stores one complex
  if constexpr (SRC == SRC_FIELD) {
    // the loads of a chunk of items are issued together, then the chunk is
    // written to LDS (same per-thread order of the sums as item by item)
    constexpr int PER = (H * N + kBlock - 1) / kBlock;
    constexpr int CH = PER < kStage<T, N> ? PER : kStage<T, N>;
    for (int c0 = 0; c0 < PER; c0 += CH) {
      T val[CH][2][CPB];
#pragma unroll
      for (int u = 0; u < CH; ++u) {
        const int t = threadIdx.x + (c0 + u) * kBlock;
        if (c0 + u < PER && t < H * N) {
          const int yp = t / N, z = t - (t / N) * N;
#pragma unroll
          for (int hh = 0; hh < 2; ++hh) {
            const int64_t v = ((int64_t)x * N + yp + hh * H) * N + z;
#pragma unroll
            for (int q = 0; q < CPB; ++q)
              val[u][hh][q] = a.field[(grp * CPB + q) * cs + v];
          }
        }
      }
#pragma unroll
      for (int u = 0; u < CH; ++u) {
        const int t = threadIdx.x + (c0 + u) * kBlock;
        if (c0 + u < PER && t < H * N) {
          const int yp = t / N, z = t - (t / N) * N;
#pragma unroll
          for (int q = 0; q < CPB; ++q) {
#pragma unroll
            for (int hh = 0; hh < 2; ++hh) {
              ss[q] += double(val[u][hh][q]) * double(val[u][hh][q]);
              s1[q] += double(val[u][hh][q]);
            }
            lds[q * SlabGeom<N>::PLANE + yp * SlabGeom<N>::PITCH + z] =
                cplx<T>{val[u][0][q], val[u][1][q]};
          }
        }
      }
    }
  }
  tws.store(tw);
  if (stopped_now(stopped)) return false;
  double kacc = 0.0;  // p . (K:p) over this block's components
  for (int t = threadIdx.x; SRC == SRC_KP && t < H * N; t += blockDim.x) {
    const int yp = t / N, z = t - (t / N) * N;
    T out[2][CPB];
#pragma unroll
    for (int hh = 0; hh < 2; ++hh) {
      const int64_t v = ((int64_t)x * N + yp + hh * H) * N + z;
      if constexpr (SRC == SRC_FIELD) {
#pragma unroll
        for (int q = 0; q < CPB; ++q)
          out[hh][q] = a.field[(grp * CPB + q) * cs + v];
      } else {
        T pd[9];
#pragma unroll
        for (int d = 0; d < 9; ++d) {
          T val = a.r[d * cs + v];
          if (!st.first) val += st.beta * a.p_old[d * cs + v];
          pd[d] = val;
        }
#pragma unroll
        for (int q = 0; q < CPB; ++q) {
          const int c = grp * CPB + q;
          if (st.upd) a.x[c * cs + v] += st.alpha * a.p_old[c * cs + v];
          a.p_new[c * cs + v] = pd[c];
          T acc = T(0);
#pragma unroll
          for (int d = 0; d < 9; ++d) acc += a.K[(9 * c + d) * cs + v] * pd[d];
          out[hh][q] = acc;
          kacc += double(pd[c]) * double(acc);
        }
      }
    }
#pragma unroll
    for (int q = 0; q < CPB; ++q) {
#pragma unroll
      for (int hh = 0; hh < 2; ++hh) {
        ss[q] += double(out[hh][q]) * double(out[hh][q]);
        s1[q] += double(out[hh][q]);
      }
      lds[q * SlabGeom<N>::PLANE + yp * SlabGeom<N>::PITCH + z] =
          cplx<T>{out[0][q], out[1][q]};
    }
  }
  __syncthreads();

  // FFT along z of the packed rows
  fft_lines<N, -1>(lds, tw, CPB * H, RowMap<N>());

  // unpack the two real-row spectra in place
  for (int t = threadIdx.x; t < CPB * H * H; t += blockDim.x) {
    const int q = t / (H * H);
    const int rem = t - q * H * H;
    const int yp = rem / H, k = rem - (rem / H) * H;
    cplx<T>* row = &lds[q * SlabGeom<N>::PLANE + yp * SlabGeom<N>::PITCH];
    if (k == 0) {
      const cplx<T> z0 = row[0];
      row[0] = {z0.x, T(0)};  // A_0 (real)
      row[H] = {z0.y, T(0)};  // B_0 (real), kept in the Nyquist slot
    } else {
      const cplx<T> zk = row[k], zm = row[N - k];
      const cplx<T> A = {T(0.5) * (zk.x + zm.x), T(0.5) * (zk.y - zm.y)};
      const cplx<T> B = {T(0.5) * (zk.y + zm.y), T(0.5) * (zm.x - zk.x)};
      row[k] = A;
      row[N - k] = B;
    }
  }
  __syncthreads();

  // FFT along y of every kz column
  fft_lines<N, -1>(lds, tw, CPB * H, ColMap<N>());

  // store the spectrum [c][x][ky][kz]
  const ColMap<N> cm;
  for (int t = threadIdx.x; t < CPB * N * H; t += blockDim.x) {
    const int q = t / (N * H);
    const int rem = t - q * N * H;
    const int ky = rem / H, kz = rem - (rem / H) * H;
    const int c = grp * CPB + q;
    a.spec[((size_t)(c * N + x) * N + ky) * H + kz] = lds[cm(q * H + kz, ky)];
  }
  if (SRC == SRC_KP && a.pkp_out) {
    const double t1 = block_sum(kacc, red);
    if (threadIdx.x == 0) a.pkp_out[lb] = t1;
  }
  if (a.psum) {
    // per-slab, per-component sum and sum of squares: [9][N]
#pragma unroll
    for (int q = 0; q < CPB; ++q) {
      const double t1 = block_sum(s1[q], red);
      const double t2 = block_sum(ss[q], red);
      if (threadIdx.x == 0) {
        const int c = grp * CPB + q;
        a.psum[c * N + x] = t1;
        a.psq[c * N + x] = t2;
      }
    }
  }
  return true;
}

// ------------------------------------------------------------------ pass B
template <typename T, int N, int TT>
__device__ __forceinline__ bool pencil_body(const PencilArgs<T>& a, int lb,
                                            cplx<T>* lds, cplx<T>* tw,
                                            const Scalars* gate = nullptr) {
  constexpr int H = N / 2;
  constexpr int TP = TT + 1;  // LDS pitch of a kx row (complex)
  // component planes of the pencil start TT slots apart in the LDS banks, so
  // that the lines of the three components do not share banks
  constexpr int CPS = N * TP + TT;
  constexpr int NTILE = (H + TT - 1) / TT;
  const int i = lb % 3;
  const int rest = lb / 3;
  const int tile = rest % NTILE;
  const int ky = rest / NTILE;
  const int kz0 = tile * TT;
  const int ncol = (H - kz0) < TT ? (H - kz0) : TT;
  const int32_t stopped = stop_flag(gate);

  if (ky == H) {  // Nyquist ky: the projection is zero there
    if (stopped_now(stopped)) return false;
    for (int t = threadIdx.x; t < 3 * N * TT; t += blockDim.x) {
      const int j = t / (N * TT);
      const int rem = t - j * N * TT;
      const int kx = rem / TT, tt = rem - (rem / TT) * TT;
      if (tt < ncol)
        a.spec[((size_t)((3 * i + j) * N + kx) * N + ky) * H + kz0 + tt] = {T(0), T(0)};
    }
    return true;
  }
  constexpr int PER0 = (3 * N * TT + kBlock - 1) / kBlock;
  TwiddleStage<T, N, kDeferTw<T, N>(PER0)> tws;
  tws.load(a.tw, tw);
  {
    constexpr int PER = PER0;
    constexpr int CH = PER < kStage<T, N> ? PER : kStage<T, N>;
    for (int c0 = 0; c0 < PER; c0 += CH) {
      cplx<T> val[CH];
#pragma unroll
      for (int u = 0; u < CH; ++u) {
        const int t = threadIdx.x + (c0 + u) * kBlock;
        val[u] = {T(0), T(0)};
        if (c0 + u < PER && t < 3 * N * TT) {
          const int j = t / (N * TT);
          const int rem = t - j * N * TT;
          const int kx = rem / TT, tt = rem - (rem / TT) * TT;
          if (tt < ncol)
            val[u] = a.spec[((size_t)((3 * i + j) * N + kx) * N + ky) * H + kz0 + tt];
        }
      }
#pragma unroll
      for (int u = 0; u < CH; ++u) {
        const int t = threadIdx.x + (c0 + u) * kBlock;
        if (c0 + u < PER && t < 3 * N * TT) {
          const int j = t / (N * TT);
          const int rem = t - j * N * TT;
          const int kx = rem / TT, tt = rem - (rem / TT) * TT;
          lds[j * CPS + kx * TP + tt] = val[u];
        }
      }
    }
  }
  tws.store(tw);
  if (stopped_now(stopped)) return false;
  __syncthreads();
  auto pm = [](int line, int kx) {
    const int j = line / TT;
    const int tt = line - j * TT;
    return j * CPS + kx * TP + tt;
  };
  fft_lines<N, -1>(lds, tw, 3 * TT, pm);

  // projection, one (kx, kz) point per thread
  const T v2 = a.vt[N + ky];
  for (int t = threadIdx.x; t < N * TT; t += blockDim.x) {
    const int kx = t / TT, tt = t - (t / TT) * TT;
    const int kz = kz0 + tt;
    const T v1 = a.vt[kx];
    const T v3 = a.vt[2 * N + (kz < H ? kz : 0)];
    const bool zero = (kx == H) || (tt >= ncol) || (kx == 0 && ky == 0 && kz == 0);
    const T nrm = v1 * v1 + v2 * v2 + v3 * v3;
    const T inv = zero ? T(0) : a.invN3 / nrm;
    cplx<T> A0 = lds[0 * CPS + kx * TP + tt];
    cplx<T> A1 = lds[1 * CPS + kx * TP + tt];
    cplx<T> A2 = lds[2 * CPS + kx * TP + tt];
    cplx<T> s = {(A0.x * v1 + A1.x * v2 + A2.x * v3) * inv,
                 (A0.y * v1 + A1.y * v2 + A2.y * v3) * inv};
    lds[0 * CPS + kx * TP + tt] = {v1 * s.x, v1 * s.y};
    lds[1 * CPS + kx * TP + tt] = {v2 * s.x, v2 * s.y};
    lds[2 * CPS + kx * TP + tt] = {v3 * s.x, v3 * s.y};
  }
  __syncthreads();
  fft_lines<N, +1>(lds, tw, 3 * TT, pm);
  for (int t = threadIdx.x; t < 3 * N * TT; t += blockDim.x) {
    const int j = t / (N * TT);
    const int rem = t - j * N * TT;
    const int kx = rem / TT, tt = rem - (rem / TT) * TT;
    if (tt < ncol)
      a.spec[((size_t)((3 * i + j) * N + kx) * N + ky) * H + kz0 + tt] =
          lds[j * CPS + kx * TP + tt];
  }
  return true;
}

// ------------------------------------------------------------------ pass C
template <typename T, typename TO, int N, int CPB, int DST>
__device__ __forceinline__ bool slab_inv_body(const SlabInvArgs<T, TO>& a,
                                              int lb, cplx<T>* lds,
                                              cplx<T>* tw, double* red,
                                              const Scalars* gate = nullptr) {
  constexpr int H = N / 2;
  constexpr int NG = 9 / CPB;
  const int64_t cs = a.cs;
  const int x = lb / NG;
  const int grp = lb - x * NG;
  const int32_t stopped = stop_flag(gate);
  constexpr int PER0 = (CPB * N * H + kBlock - 1) / kBlock;
  TwiddleStage<T, N, kDeferTw<T, N>(PER0)> tws;
  tws.load(a.tw, tw);
  // the real-space operand of the output step (r of a CG run, or the dot
  // product's field): when it is one chunk per thread of one component,
  // its loads are issued now and their latency hides behind the transforms
  // (three components would hold 48 more registers across them)
  constexpr int PER2 = (H * N + kBlock - 1) / kBlock;
  constexpr int CH2 = PER2 < kStage<T, N> ? PER2 : kStage<T, N>;
  constexpr bool kSrc = DST == DST_DOT || DST == DST_CG;
  constexpr bool kEarly = kSrc && PER2 <= CH2 && CPB == 1;
  T pve[kEarly ? CH2 : 1][CPB][2];
  auto load_src = [&](int c0, auto& pv) {
    const T* src = (DST == DST_CG) ? a.rio : a.pdot;
#pragma unroll
    for (int u = 0; u < CH2; ++u) {
      const int t = threadIdx.x + (c0 + u) * kBlock;
      if (c0 + u < PER2 && t < H * N) {
        const int yp = t / N, z = t - (t / N) * N;
#pragma unroll
        for (int q = 0; q < CPB; ++q)
#pragma unroll
          for (int hh = 0; hh < 2; ++hh) {
            const int64_t v = ((int64_t)x * N + yp + hh * H) * N + z;
            pv[u][q][hh] = src[(grp * CPB + q) * cs + v];
          }
      }
    }
  };
  if constexpr (kEarly) load_src(0, pve);
  const ColMap<N> cm;
  {
    constexpr int PER = PER0;
    constexpr int CH = PER < kStage<T, N> ? PER : kStage<T, N>;
    for (int c0 = 0; c0 < PER; c0 += CH) {
      cplx<T> val[CH];
#pragma unroll
      for (int u = 0; u < CH; ++u) {
        const int t = threadIdx.x + (c0 + u) * kBlock;
        if (c0 + u < PER && t < CPB * N * H) {
          const int q = t / (N * H);
          const int rem = t - q * N * H;
          const int ky = rem / H, kz = rem - (rem / H) * H;
          const int c = grp * CPB + q;
          val[u] = a.spec[((size_t)(c * N + x) * N + ky) * H + kz];
        }
      }
#pragma unroll
      for (int u = 0; u < CH; ++u) {
        const int t = threadIdx.x + (c0 + u) * kBlock;
        if (c0 + u < PER && t < CPB * N * H) {
          const int q = t / (N * H);
          const int rem = t - q * N * H;
          const int ky = rem / H, kz = rem - (rem / H) * H;
          lds[cm(q * H + kz, ky)] = val[u];
        }
      }
    }
  }
  tws.store(tw);
  if (stopped_now(stopped)) return false;
  T alpha = T(0);
  if constexpr (DST == DST_CG) alpha = T(a.sc->alphas[a.parity]);
  __syncthreads();
  fft_lines<N, +1>(lds, tw, CPB * H, ColMap<N>());

  // pack the two half spectra of rows y' and y'+H into one complex line
  for (int t = threadIdx.x; t < CPB * H * H; t += blockDim.x) {
    const int q = t / (H * H);
    const int rem = t - q * H * H;
    const int yp = rem / H, k = rem - (rem / H) * H;
    cplx<T>* row = &lds[q * SlabGeom<N>::PLANE + yp * SlabGeom<N>::PITCH];
    if (k == 0) {
      const T a0 = row[0].x, b0 = row[H].x;
      row[0] = {a0, b0};
      row[H] = {T(0), T(0)};
    } else {
      const cplx<T> A = row[k], B = row[N - k];
      row[k] = {A.x - B.y, A.y + B.x};        // A + i B
      row[N - k] = {A.x + B.y, B.x - A.y};    // conj(A) + i conj(B)
    }
  }
  __syncthreads();
  fft_lines<N, +1>(lds, tw, CPB * H, RowMap<N>());

  double acc = 0.0;
  {
    // the p (or r) loads of a chunk are issued together (same order of the
    // sum)
    constexpr int PER = PER2;
    constexpr int CH = CH2;
    for (int c0 = 0; c0 < PER; c0 += CH) {
      T pvl[CH2][CPB][2];
      if constexpr (kSrc && !kEarly) load_src(c0, pvl);
#pragma unroll
      for (int u = 0; u < CH; ++u) {
        const int t = threadIdx.x + (c0 + u) * kBlock;
        if (!(c0 + u < PER && t < H * N)) continue;
        const int yp = t / N, z = t - (t / N) * N;
#pragma unroll
        for (int q = 0; q < CPB; ++q) {
          const int c = grp * CPB + q;
          const cplx<T> zz = lds[q * SlabGeom<N>::PLANE + yp * SlabGeom<N>::PITCH + z];
#pragma unroll
          for (int hh = 0; hh < 2; ++hh) {
            const int64_t v = ((int64_t)x * N + yp + hh * H) * N + z;
            const T val = hh ? zz.y : zz.x;
            T src_v = T(0);
            if constexpr (kEarly)
              src_v = pve[u][q][hh];
            else if constexpr (kSrc)
              src_v = pvl[u][q][hh];
            if constexpr (DST == DST_CG) {
              const T rn = src_v - alpha * val;
              a.rio[c * cs + v] = rn;
              acc += double(rn) * double(rn);
            } else if constexpr (DST == DST_DOT) {
              a.out[c * cs + v] = TO(val);
              acc += double(src_v) * double(val);
            } else {
              a.out[c * cs + v] = TO(val);
              acc += double(val) * double(val);
            }
          }
        }
      }
    }
  }
  if (a.partial) {
    double tot = block_sum(acc, red);
    if (threadIdx.x == 0) a.partial[lb] = tot;
  }
  return true;
}

template <typename T, int N>
struct SpectralTraits {
  // components per slab block: three (one tensor row) when the planes fit
  static constexpr int CPB =
      (3 * SlabGeom<N>::PLANE * (int)sizeof(cplx<T>) <= 64 * 1024) ? 3 : 1;
  static constexpr int TT = (sizeof(T) == 4) ? 16 : 8;
  static constexpr size_t SLAB_LDS =
      (CPB * SlabGeom<N>::PLANE + N) * sizeof(cplx<T>) + kBlock * sizeof(double);
  static constexpr size_t PENCIL_LDS =
      (3 * (N * (TT + 1) + TT) + N) * sizeof(cplx<T>);
};

// ---------------------------------------------------- single-RVE kernels
// the direction step of an SRC_KP pass A that takes it from the scalars
// (p = r or r + beta p_old, no x update)
template <typename T>
__device__ __forceinline__ KpStep<T> kp_step_of(const Scalars* sc) {
  if (!sc) return KpStep<T>{true, T(0), false, T(0)};
  return KpStep<T>{sc->first != 0, T(sc->beta), false, T(0)};
}

template <typename T, int N, int CPB, int SRC>
__global__ __launch_bounds__(kBlock) void slab_fwd_kernel(SlabFwdArgs<T> a) {
  __shared__ cplx<T> lds[CPB * SlabGeom<N>::PLANE];
  __shared__ cplx<T> tw[N];
  __shared__ double red[kBlock];
  // done comes from an earlier launch, except after a breakdown that block
  // 0 of this launch publishes at its end (cg_alpha_publish): blocks that
  // read done before that write and go on only fill the spectrum, which
  // the inverse pass of a stopped run never reads (it returns on done).
  // The body reads it and returns once its loads are issued.
  KpStep<T> st = kp_step_of<T>(SRC == SRC_KP ? a.sc : nullptr);
  if (SRC == SRC_KP && a.x) {  // timing of the folded pass: x += alpha p_old
    st.upd = true;
    st.alpha = T(a.sc->alpha);
  }
  if (!slab_fwd_body<T, N, CPB, SRC>(a, xcd_remap(blockIdx.x, gridDim.x), lds,
                                     tw, red, st, a.sc))
    return;
  if (a.pkp && blockIdx.x == 0)
    cg_alpha_publish(a.pkp, a.pkp_count, a.scw, a.parity, red);
}

// Pass A of a single-RVE CG iteration with the direction kernel folded in
// (Sec. 2.1, Eqs. 15-16): every block takes the CG decision of the
// direction kernel itself from the r.r partials of the last pass C (the
// same fixed-order sum in every block, cg_beta_consume), applies the
// previous iteration's x += alpha p_old on its own components, forms
// p = r + beta p_old at each voxel of its slab (all nine components: the
// nine blocks of a slab run on one XCD and share r and p_old through its
// L2), writes its components of p and transforms its rows of K : p, and
// writes its partial of p . (K:p) for the alpha that pass B publishes.  It
// returns at once after a halted iteration, and applies only the pending x
// update when this iteration stops the run.
template <typename T, int N, int CPB>
__global__ __launch_bounds__(kBlock) void slab_fwd_cg_kernel(SlabFwdArgs<T> a) {
  __shared__ cplx<T> lds[CPB * SlabGeom<N>::PLANE];
  __shared__ cplx<T> tw[N];
  __shared__ double red[kBlock];
  Scalars* sc = a.scw;
  // every flag read here was written by an earlier launch: block 0 of this
  // launch publishes slot `parity` (and done), which no block reads
  const int q = a.parity ^ 1;
  if (sc->halt[q]) {
    if (blockIdx.x == 0 && threadIdx.x == 0) sc->halt[a.parity] = 1;
    return;
  }
  const BetaStep d = cg_beta_consume(a.pinv, a.pinv_count, sc, a.parity);
  if (d.first && sc->done) return;  // b = 0: nothing to solve
  const KpStep<T> st{d.first, T(d.beta), !d.first && a.x != nullptr,
                     T(sc->alphas[q])};
  const int lb = xcd_remap(blockIdx.x, gridDim.x);
  if (d.stop) {
    if (st.upd) {
      constexpr int NG = 9 / CPB;
      const int x0 = lb / NG, grp = lb - (lb / NG) * NG;
      for (int t = threadIdx.x; t < N * N; t += blockDim.x) {
        const int64_t v = (int64_t)x0 * N * N + t;
#pragma unroll
        for (int qq = 0; qq < CPB; ++qq) {
          const int c = grp * CPB + qq;
          a.x[c * a.cs + v] += st.alpha * a.p_old[c * a.cs + v];
        }
      }
    }
    return;
  }
  slab_fwd_body<T, N, CPB, SRC_KP>(a, lb, lds, tw, red, st);
}

template <typename T, int N, int TT>
__global__ __launch_bounds__(kBlock) void pencil_proj_kernel(PencilArgs<T> a) {
  __shared__ cplx<T> lds[3 * (N * (TT + 1) + TT)];
  __shared__ cplx<T> tw[N];
  __shared__ double red[kBlock];
  if (!pencil_body<T, N, TT>(a, xcd_remap(blockIdx.x, gridDim.x), lds, tw,
                             a.sc))
    return;
  // fused CG run: alpha = r.r / p.(K:p) from pass A's partials (a breakdown
  // sets done, which the pass-B blocks that already started ignore: their
  // spectrum is not used, pass C returns)
  if (a.pkp && blockIdx.x == 0)
    cg_alpha_publish(a.pkp, a.pkp_count, a.scw, a.parity, red);
}

template <typename T, typename TO, int N, int CPB, int DST>
__global__ __launch_bounds__(kBlock) void slab_inv_kernel(SlabInvArgs<T, TO> a) {
  __shared__ cplx<T> lds[CPB * SlabGeom<N>::PLANE];
  __shared__ cplx<T> tw[N];
  __shared__ double red[kBlock];
  slab_inv_body<T, TO, N, CPB, DST>(a, xcd_remap(blockIdx.x, gridDim.x), lds,
                                    tw, red, a.sc);
}

// three component planes per slab block fit the LDS budget of one block
template <typename T, int N>
constexpr bool cpb3_fits() {
  return 3 * SlabGeom<N>::PLANE * (int)sizeof(cplx<T>) <= 64 * 1024;
}
template <typename T, int N, int TT>
constexpr bool pencil_fits() {
  return (3 * (N * (TT + 1) + TT) + N) * (int)sizeof(cplx<T>) +
             kBlock * (int)sizeof(double) <= 64 * 1024;
}

// ------------------------------------------------------- batched kernels
// Every RVE of a batch in one launch: block -> (RVE, local block) through
// the descriptor table; the RVE's edge and schedule (components per slab
// block, kz columns per pencil block) select the compiled FFT plan.
// Converged or retired RVEs (Scalars::done for CG work, ::inactive for the
// residual) return at once.
#define RVE_BATCH_SIZES(X) X(16) X(24) X(32) X(40) X(48) X(64)

template <typename T>
__device__ __forceinline__ int batch_item(const BatchSpec<T>& b, int pass,
                                          int blk) {
  int r = 0;
  while (r + 1 < b.nitems && b.items[r + 1].blk[pass] <= blk) ++r;
  return r;
}

// one RVE's pass bodies in the dynamic LDS of a batched launch
template <typename T, int NN, int CPB, int SRC>
__device__ __forceinline__ void slab_fwd_item(const SlabFwdArgs<T>& a, int lb,
                                              unsigned char* smem,
                                              const KpStep<T>& st) {
  cplx<T>* lds = reinterpret_cast<cplx<T>*>(smem);
  cplx<T>* tw = lds + CPB * SlabGeom<NN>::PLANE;
  double* red = reinterpret_cast<double*>(tw + NN);
  slab_fwd_body<T, NN, CPB, SRC>(a, lb, lds, tw, red, st);
}
template <typename T, typename TO, int NN, int CPB, int DST>
__device__ __forceinline__ void slab_inv_item(const SlabInvArgs<T, TO>& a,
                                              int lb, unsigned char* smem) {
  cplx<T>* lds = reinterpret_cast<cplx<T>*>(smem);
  cplx<T>* tw = lds + CPB * SlabGeom<NN>::PLANE;
  double* red = reinterpret_cast<double*>(tw + NN);
  slab_inv_body<T, TO, NN, CPB, DST>(a, lb, lds, tw, red);
}
template <typename T, int NN, int TT>
__device__ __forceinline__ void pencil_item(const PencilArgs<T>& a, int lb,
                                            unsigned char* smem) {
  cplx<T>* lds = reinterpret_cast<cplx<T>*>(smem);
  pencil_body<T, NN, TT>(a, lb, lds, lds + 3 * (NN * (TT + 1) + TT));
}

// Each pass as a block body (blk: the block it plays, a launch's blockIdx.x
// or a virtual block of the persistent CG kernel) and a one-launch kernel.
// CPBS: the slab schedules compiled in (bit 0: one component per block,
// bit 1: three), so that a launch whose RVEs all use one of them does not
// carry the registers of the other
template <typename T, int SRC, int CPBS = 3>
__device__ __forceinline__ void slab_fwd_batch_block(const BatchSpec<T>& b,
                                                     int blk,
                                                     unsigned char* smem) {
  const int r = batch_item(b, 0, blk);
  const SpecItem<T>& it = b.items[r];
  if (SRC == SRC_KP ? it.sc->done : it.sc->inactive) return;
  const int lb = blk - it.blk[0];
  SlabFwdArgs<T> a{};
  a.cs = b.cs;
  a.field = b.field ? b.field + it.off : nullptr;
  a.K = b.K ? b.K + it.off : nullptr;
  a.r = b.r ? b.r + it.off : nullptr;
  a.p_old = b.p_old ? b.p_old + it.off : nullptr;
  a.p_new = b.p_new ? b.p_new + it.off : nullptr;
  a.spec = b.spec + it.soff;
  a.tw = it.tw;
  a.psum = it.psum;
  a.psq = it.psq;
  a.sc = it.sc;
  const KpStep<T> st = kp_step_of<T>(SRC == SRC_KP ? it.sc : nullptr);
  switch (it.n) {
#define RVE_CASE(NN)                                                         \
  case NN:                                                                   \
    if constexpr ((CPBS & 2) && cpb3_fits<T, NN>())                          \
      if (it.cpb == 3) {                                                     \
        slab_fwd_item<T, NN, 3, SRC>(a, lb, smem, st);                       \
        break;                                                               \
      }                                                                      \
    if constexpr ((CPBS & 1) || !cpb3_fits<T, NN>())                         \
      slab_fwd_item<T, NN, 1, SRC>(a, lb, smem, st);                         \
    break;
    RVE_BATCH_SIZES(RVE_CASE)
#undef RVE_CASE
  }
}

template <typename T, int SRC, int CPBS>
__global__ __launch_bounds__(kBlock) void slab_fwd_batch_kernel(BatchSpec<T> b) {
  extern __shared__ __align__(16) unsigned char smem[];
  slab_fwd_batch_block<T, SRC, CPBS>(b, blockIdx.x, smem);
}

template <typename T>
__device__ __forceinline__ void pencil_batch_block(const BatchSpec<T>& b,
                                                   int cg, int blk,
                                                   unsigned char* smem) {
  const int r = batch_item(b, 1, blk);
  const SpecItem<T>& it = b.items[r];
  if (cg ? it.sc->done : it.sc->inactive) return;
  const int lb = blk - it.blk[1];
  PencilArgs<T> a{};
  a.spec = b.spec + it.soff;
  a.tw = it.tw;
  a.vt = it.vt;
  a.sc = nullptr;
  switch (it.n) {
#define RVE_CASE(NN)                                                         \
  case NN:                                                                   \
    a.invN3 = T(1.0 / (double(NN) * NN * NN));                               \
    if constexpr (pencil_fits<T, NN, 16>())                                  \
      if (it.tt == 16) {                                                     \
        pencil_item<T, NN, 16>(a, lb, smem);                                 \
        break;                                                               \
      }                                                                      \
    if (it.tt == 4)                                                          \
      pencil_item<T, NN, 4>(a, lb, smem);                                    \
    else                                                                     \
      pencil_item<T, NN, 8>(a, lb, smem);                                    \
    break;
    RVE_BATCH_SIZES(RVE_CASE)
#undef RVE_CASE
  }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void pencil_batch_kernel(BatchSpec<T> b,
                                                              int cg) {
  extern __shared__ __align__(16) unsigned char smem[];
  pencil_batch_block<T>(b, cg, blockIdx.x, smem);
}

template <typename T, typename TO, int DST, int CPBS = 3>
__device__ __forceinline__ void slab_inv_batch_block(const BatchSpec<T>& b,
                                                     TO* out, int blk,
                                                     unsigned char* smem) {
  const int r = batch_item(b, 0, blk);
  const SpecItem<T>& it = b.items[r];
  if (DST == DST_DOT ? it.sc->done : it.sc->inactive) return;
  const int lb = blk - it.blk[0];
  SlabInvArgs<T, TO> a{};
  a.cs = b.cs;
  a.spec = b.spec + it.soff;
  a.tw = it.tw;
  a.out = out + it.off;
  a.pdot = b.p_new ? b.p_new + it.off : nullptr;
  a.partial = it.partial;
  a.sc = nullptr;
  switch (it.n) {
#define RVE_CASE(NN)                                                         \
  case NN:                                                                   \
    if constexpr ((CPBS & 2) && cpb3_fits<T, NN>())                          \
      if (it.cpb == 3) {                                                     \
        slab_inv_item<T, TO, NN, 3, DST>(a, lb, smem);                       \
        break;                                                               \
      }                                                                      \
    if constexpr ((CPBS & 1) || !cpb3_fits<T, NN>())                         \
      slab_inv_item<T, TO, NN, 1, DST>(a, lb, smem);                         \
    break;
    RVE_BATCH_SIZES(RVE_CASE)
#undef RVE_CASE
  }
}

template <typename T, typename TO, int DST, int CPBS>
__global__ __launch_bounds__(kBlock) void slab_inv_batch_kernel(BatchSpec<T> b,
                                                                TO* out) {
  extern __shared__ __align__(16) unsigned char smem[];
  slab_inv_batch_block<T, TO, DST, CPBS>(b, out, blockIdx.x, smem);
}

// ------------------------------------------------- persistent batched CG
// The CG iterations of every RVE of a batch in one launch of resident
// blocks: each iteration runs the three FFT/projection passes of G(K:p)
// (p = r + beta p_old fused into the first), the per-RVE p.Ap reduction,
// the vector update and the r.r reduction, each over all RVEs' blocks,
// with a grid-wide barrier between them; it stops when every RVE's CG is
// done (converged, broken down or at its cap).  A barrier that waits
// beyond a bound (blocks not all resident) sets an error flag and lets the
// kernel run out instead of hanging; the host turns the flag into an error.
// Barrier state (unsigned words, one 128-byte line each part): [0] the
// generation, [32 (1 + g)] the arrival count of group g = blockIdx.x % 8
// (the hardware deals consecutive blocks round-robin over the eight XCDs),
// [32 * 9] the count of groups arrived.  The last block of a group arrives
// at the group count, the last group releases everyone by advancing the
// generation: eight-way instead of all-block contention on one atomic.
constexpr int kBarGroups = 8;
static_assert(32 * (kBarGroups + 2) == kBatchBarWords, "barrier layout");

__device__ __forceinline__ bool grid_barrier(unsigned* bar, unsigned nblocks,
                                             int* err) {
  __syncthreads();
  if (threadIdx.x == 0) {
    __threadfence();
    if (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0) {
      const unsigned g = blockIdx.x % kBarGroups;
      const unsigned members =
          nblocks / kBarGroups + (g < nblocks % kBarGroups ? 1u : 0u);
      const unsigned groups = nblocks < kBarGroups ? nblocks : kBarGroups;
      const unsigned gen =
          __hip_atomic_load(&bar[0], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
      unsigned* gcount = bar + 32 * (1 + g);
      unsigned* top = bar + 32 * (1 + kBarGroups);
      const unsigned a = __hip_atomic_fetch_add(gcount, 1u, __ATOMIC_ACQ_REL,
                                                __HIP_MEMORY_SCOPE_AGENT) + 1u;
      bool release = false;
      if (a == members) {
        __hip_atomic_store(gcount, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const unsigned t = __hip_atomic_fetch_add(top, 1u, __ATOMIC_ACQ_REL,
                                                  __HIP_MEMORY_SCOPE_AGENT) + 1u;
        if (t == groups) {
          __hip_atomic_store(top, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          __hip_atomic_fetch_add(&bar[0], 1u, __ATOMIC_RELEASE,
                                 __HIP_MEMORY_SCOPE_AGENT);
          release = true;
        }
      }
      if (!release) {
        // bounded wait (about a second); another block's timeout ends it too
        long spins = 0;
        while (__hip_atomic_load(&bar[0], __ATOMIC_ACQUIRE,
                                 __HIP_MEMORY_SCOPE_AGENT) == gen) {
          if (++spins > 2000000L) {
            __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            break;
          }
          if ((spins & 255) == 0 &&
              __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
            break;
          __builtin_amdgcn_s_sleep(8);
        }
      }
    }
    __threadfence();
  }
  __syncthreads();
  return __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0;
}

// the passes as calls (not inlined into one body, which would hold the
// registers of all of them at once)
template <typename T>
__device__ __noinline__ void pc_slab_fwd(const BatchSpec<T>& b, int blk,
                                         unsigned char* smem) {
  slab_fwd_batch_block<T, SRC_KP>(b, blk, smem);
}
template <typename T>
__device__ __noinline__ void pc_pencil(const BatchSpec<T>& b, int blk,
                                       unsigned char* smem) {
  pencil_batch_block<T>(b, 1, blk, smem);
}
template <typename T>
__device__ __noinline__ void pc_slab_inv(const BatchSpec<T>& b, T* Ap, int blk,
                                         unsigned char* smem) {
  slab_inv_batch_block<T, T, DST_DOT>(b, Ap, blk, smem);
}
template <typename T>
__device__ __noinline__ void pc_update(const BatchCG<T>& c, const T* p, int blk,
                                       double* red) {
  cg_update_batch_block<T>(c.seg, c.nitems, c.cs, c.x, c.r, p, c.Ap, blk, red);
}
__device__ __noinline__ void pc_reduce(int op, const RedItem* items,
                                       Scalars* scs, int b, double* red) {
  reduce_batch_block(op, items, scs, b, red);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void cg_batch_persistent_kernel(
    BatchCG<T> c) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ double red[kBlock / 64];
  __shared__ int active;
  for (int j = 0; j < c.max_iters; ++j) {
    // every block takes the same decision from the same scalars
    if (threadIdx.x == 0) active = 0;
    __syncthreads();
    for (int b = threadIdx.x; b < c.nitems; b += blockDim.x)
      if (!c.scs[b].done) active = 1;
    __syncthreads();
    if (!active) break;
    const BatchSpec<T>& b = (j & 1) ? c.odd : c.even;
    for (int vb = blockIdx.x; vb < c.blocksA; vb += gridDim.x)
      pc_slab_fwd<T>(b, vb, smem);
    if (!grid_barrier(c.bar, gridDim.x, c.err)) return;
    for (int vb = blockIdx.x; vb < c.blocksB; vb += gridDim.x)
      pc_pencil<T>(b, vb, smem);
    if (!grid_barrier(c.bar, gridDim.x, c.err)) return;
    for (int vb = blockIdx.x; vb < c.blocksA; vb += gridDim.x)
      pc_slab_inv<T>(b, c.Ap, vb, smem);
    if (!grid_barrier(c.bar, gridDim.x, c.err)) return;
    for (int r = blockIdx.x; r < c.nitems; r += gridDim.x)
      pc_reduce(RED_ALPHA, c.red_inv, c.scs, r, red);
    if (!grid_barrier(c.bar, gridDim.x, c.err)) return;
    for (int vb = blockIdx.x; vb < c.seg_blocks; vb += gridDim.x)
      pc_update<T>(c, b.p_new, vb, red);
    if (!grid_barrier(c.bar, gridDim.x, c.err)) return;
    for (int r = blockIdx.x; r < c.nitems; r += gridDim.x)
      pc_reduce(RED_BETA, c.red_seg, c.scs, r, red);
    if (!grid_barrier(c.bar, gridDim.x, c.err)) return;
  }
}

template <typename T>
void launch_cg_batch_persistent(const BatchCG<T>& c, int grid, size_t lds,
                                hipStream_t s) {
  hipLaunchKernelGGL((cg_batch_persistent_kernel<T>), dim3(grid), dim3(kBlock),
                     lds, s, c);
}

template <typename T>
int cg_batch_persistent_grid(size_t lds) {
  int dev = 0, per_cu = 0;
  RVE_HIP(hipGetDevice(&dev));
  hipDeviceProp_t prop;
  RVE_HIP(hipGetDeviceProperties(&prop, dev));
  RVE_HIP(hipFuncSetAttribute(
      reinterpret_cast<const void*>(&cg_batch_persistent_kernel<T>),
      hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  RVE_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(
      &per_cu, reinterpret_cast<const void*>(&cg_batch_persistent_kernel<T>),
      kBlock, lds));
  if (per_cu < 1) throw Error(-3, "persistent CG kernel does not fit a CU");
  return per_cu * prop.multiProcessorCount;
}

template void launch_cg_batch_persistent<float>(const BatchCG<float>&, int,
                                                size_t, hipStream_t);
template void launch_cg_batch_persistent<double>(const BatchCG<double>&, int,
                                                 size_t, hipStream_t);
template int cg_batch_persistent_grid<float>(size_t);
template int cg_batch_persistent_grid<double>(size_t);

// ---------------------------------------------------------------- launchers

template <typename T, int N, int CPB, int TT>
void launch_G_passes(const SpectralLaunch<T>& L, hipStream_t s) {
  constexpr int H = N / 2;
  constexpr int NTILE = (H + TT - 1) / TT;
  const int nslab = N * (9 / CPB);
  if (!(L.passes & 1)) {
  } else if (L.src == SRC_FIELD) {
    SlabFwdArgs<T> fa{};
    fa.cs = (int64_t)N * N * N;
    fa.field = L.in_field;
    fa.spec = L.spec;
    fa.tw = L.tw;
    fa.psum = L.psum;
    fa.psq = L.psq;
    fa.sc = L.sc;
    if (L.pkp) {
      fa.pkp = L.pkp;
      fa.pkp_count = L.pkp_count;
      fa.parity = L.parity;
      fa.scw = L.sc;
    }
    launch((slab_fwd_kernel<T, N, CPB, SRC_FIELD>), dim3(nslab),
                       dim3(kBlock), 0, s, fa);
  } else {
    SlabFwdArgs<T> fa{};
    fa.cs = (int64_t)N * N * N;
    fa.K = L.K;
    fa.r = L.r;
    fa.p_old = L.p_old;
    fa.p_new = L.p_new;
    fa.spec = L.spec;
    fa.tw = L.tw;
    fa.psum = nullptr;
    fa.psq = nullptr;
    fa.sc = L.sc;
    if (L.pinv) {
      // fused CG run: pass A writes the p.(K:p) partials that pass B reduces
      fa.pinv = L.pinv;
      fa.pinv_count = L.pinv_count;
      fa.x = L.x;
      fa.pkp_out = const_cast<double*>(L.pkp);
      fa.parity = L.parity;
      fa.scw = L.sc;
      launch((slab_fwd_cg_kernel<T, N, CPB>), dim3(nslab), dim3(kBlock), 0, s,
             fa);
    } else {
      // direction and K:p from the scalars (with x: x += alpha p_old too)
      fa.x = L.x;
      launch((slab_fwd_kernel<T, N, CPB, SRC_KP>), dim3(nslab),
                         dim3(kBlock), 0, s, fa);
    }
  }
  if (L.passes & 2) {
  PencilArgs<T> pa{};
  pa.spec = L.spec;
  pa.tw = L.tw;
  pa.vt = L.vt;
  pa.invN3 = T(1.0 / (double(N) * N * N));
  pa.sc = L.sc;
  if (L.src == SRC_KP && L.pinv && L.pkp) {
    pa.pkp = L.pkp;
    pa.pkp_count = L.pkp_count;
    pa.parity = L.parity;
    pa.scw = L.sc;
  }
  launch((pencil_proj_kernel<T, N, TT>), dim3(N * NTILE * 3),
                     dim3(kBlock), 0, s, pa);
  }
  if (!(L.passes & 4)) {
  } else if (L.dst == DST_CG) {
    SlabInvArgs<T, T> ia{};
    ia.cs = (int64_t)N * N * N;
    ia.spec = L.spec;
    ia.tw = L.tw;
    ia.out = nullptr;
    ia.pdot = nullptr;
    ia.partial = L.partial_inv;
    ia.sc = L.sc;
    ia.rio = L.r_io;
    ia.parity = L.parity;
    launch((slab_inv_kernel<T, T, N, CPB, DST_CG>), dim3(nslab),
                       dim3(kBlock), 0, s, ia);
  } else if (L.dst == DST_DOT) {
    SlabInvArgs<T, T> ia{};
    ia.cs = (int64_t)N * N * N;
    ia.spec = L.spec;
    ia.tw = L.tw;
    ia.out = L.out_T;
    ia.pdot = L.p_new;
    ia.partial = L.partial_inv;
    ia.sc = L.sc;
    launch((slab_inv_kernel<T, T, N, CPB, DST_DOT>), dim3(nslab),
                       dim3(kBlock), 0, s, ia);
  } else {
    SlabInvArgs<T, double> ia{};
    ia.cs = (int64_t)N * N * N;
    ia.spec = L.spec;
    ia.tw = L.tw;
    ia.out = L.out_d;
    ia.pdot = nullptr;
    ia.partial = L.partial_inv;
    ia.sc = nullptr;
    launch((slab_inv_kernel<T, double, N, CPB, DST_NORM>),
                       dim3(nslab), dim3(kBlock), 0, s, ia);
  }
}

// the schedule (cpb, tt) of one launch; 0 picks the default of the traits
template <typename T, int N>
void launch_G_sched(const SpectralLaunch<T>& L, hipStream_t s) {
  const int cpb = L.cpb ? L.cpb : SpectralTraits<T, N>::CPB;
  const int tt = L.tt ? L.tt : SpectralTraits<T, N>::TT;
  if (cpb == 3) {
    if constexpr (cpb3_fits<T, N>()) {
      if constexpr (pencil_fits<T, N, 16>())
        if (tt == 16) return launch_G_passes<T, N, 3, 16>(L, s);
      if (tt == 8) return launch_G_passes<T, N, 3, 8>(L, s);
      if (tt == 4) return launch_G_passes<T, N, 3, 4>(L, s);
    }
  } else if (cpb == 1) {
    if constexpr (pencil_fits<T, N, 16>())
      if (tt == 16) return launch_G_passes<T, N, 1, 16>(L, s);
    if (tt == 8) return launch_G_passes<T, N, 1, 8>(L, s);
    if (tt == 4) return launch_G_passes<T, N, 1, 4>(L, s);
  }
  throw Error(-1, "unsupported FFT schedule");
}

template <typename T>
void launch_G(int n, const SpectralLaunch<T>& L, hipStream_t s) {
  switch (n) {
    case 16: launch_G_sched<T, 16>(L, s); break;
    case 24: launch_G_sched<T, 24>(L, s); break;
    case 32: launch_G_sched<T, 32>(L, s); break;
    case 40: launch_G_sched<T, 40>(L, s); break;
    case 48: launch_G_sched<T, 48>(L, s); break;
    case 64: launch_G_sched<T, 64>(L, s); break;
    case 96: launch_G_sched<T, 96>(L, s); break;
    case 128: launch_G_sched<T, 128>(L, s); break;
    default: throw Error(-1, "unsupported grid size for the FFT passes");
  }
}

int slab_blocks(int n, bool fp64, int cpb_sel) {
  if (cpb_sel) return n * (9 / cpb_sel);
  auto cpb = [&](auto tag, int nn) -> int {
    using T = decltype(tag);
    switch (nn) {
      case 16: return SpectralTraits<T, 16>::CPB;
      case 24: return SpectralTraits<T, 24>::CPB;
      case 32: return SpectralTraits<T, 32>::CPB;
      case 40: return SpectralTraits<T, 40>::CPB;
      case 48: return SpectralTraits<T, 48>::CPB;
      case 64: return SpectralTraits<T, 64>::CPB;
      case 96: return SpectralTraits<T, 96>::CPB;
      case 128: return SpectralTraits<T, 128>::CPB;
    }
    return 1;
  };
  const int c = fp64 ? cpb(double{}, n) : cpb(float{}, n);
  return n * (9 / c);
}

int pencil_blocks(int n, bool fp64, int tt_sel) {
  const int tt = tt_sel ? tt_sel : (fp64 ? 8 : 16);
  return n * ((n / 2 + tt - 1) / tt) * 3;
}

bool schedule_valid(int n, bool fp64, int cpb, int tt) {
  if (tt != 4 && tt != 8 && tt != 16) return false;
  if (cpb != 1 && cpb != 3) return false;
  auto fits = [&](auto tag) -> bool {
    using T = decltype(tag);
    switch (n) {
#define RVE_FITS(NN)                                                        \
  case NN:                                                                  \
    return (cpb == 1 || cpb3_fits<T, NN>()) &&                              \
           (tt != 16 || pencil_fits<T, NN, 16>());
      RVE_FITS(16) RVE_FITS(24) RVE_FITS(32) RVE_FITS(40) RVE_FITS(48)
      RVE_FITS(64) RVE_FITS(96) RVE_FITS(128)
#undef RVE_FITS
    }
    return false;
  };
  return fp64 ? fits(double{}) : fits(float{});
}

bool batch_supported(int n) {
  switch (n) {
#define RVE_CASE(NN) case NN:
    RVE_BATCH_SIZES(RVE_CASE)
#undef RVE_CASE
    return true;
  }
  return false;
}

template <typename T>
void batch_lds(int n, int cpb, int tt, size_t& slab, size_t& pencil) {
  if (!batch_supported(n)) throw Error(-1, "grid edge not supported in a batch");
  if (!schedule_valid(n, sizeof(T) == 8, cpb, tt))
    throw Error(-1, "no such FFT schedule for this grid edge and precision");
  // the layouts of slab_fwd_item / slab_inv_item and pencil_item
  const size_t plane = (size_t)(n / 2) * (n + 1);
  slab = (cpb * plane + n) * sizeof(cplx<T>) + kBlock * sizeof(double);
  pencil = (3 * ((size_t)n * (tt + 1) + tt) + n) * sizeof(cplx<T>);
}

// the default schedule of a grid edge and precision
void default_schedule(int n, bool fp64, int& cpb, int& tt) {
  auto pick = [&](auto tag) {
    using T = decltype(tag);
    switch (n) {
#define RVE_DEF(NN)                          \
  case NN:                                   \
    cpb = SpectralTraits<T, NN>::CPB;        \
    tt = SpectralTraits<T, NN>::TT;          \
    return;
      RVE_DEF(16) RVE_DEF(24) RVE_DEF(32) RVE_DEF(40) RVE_DEF(48)
      RVE_DEF(64) RVE_DEF(96) RVE_DEF(128)
#undef RVE_DEF
    }
    throw Error(-1, "grid edge not supported");
  };
  if (fp64) pick(double{}); else pick(float{});
}

template <typename T, int CPBS>
void launch_G_batch_cpbs(const BatchSpec<T>& b, int src, T* out_T,
                         double* out_d, int blocksA, int blocksB, size_t ldsA,
                         size_t ldsB, hipStream_t s) {
  if (src == SRC_FIELD) {
    hipLaunchKernelGGL((slab_fwd_batch_kernel<T, SRC_FIELD, CPBS>),
                       dim3(blocksA), dim3(kBlock), ldsA, s, b);
    hipLaunchKernelGGL((pencil_batch_kernel<T>), dim3(blocksB), dim3(kBlock),
                       ldsB, s, b, 0);
    hipLaunchKernelGGL((slab_inv_batch_kernel<T, double, DST_NORM, CPBS>),
                       dim3(blocksA), dim3(kBlock), ldsA, s, b, out_d);
  } else {
    hipLaunchKernelGGL((slab_fwd_batch_kernel<T, SRC_KP, CPBS>), dim3(blocksA),
                       dim3(kBlock), ldsA, s, b);
    hipLaunchKernelGGL((pencil_batch_kernel<T>), dim3(blocksB), dim3(kBlock),
                       ldsB, s, b, 1);
    hipLaunchKernelGGL((slab_inv_batch_kernel<T, T, DST_DOT, CPBS>),
                       dim3(blocksA), dim3(kBlock), ldsA, s, b, out_T);
  }
}

template <typename T>
void launch_G_batch(const BatchSpec<T>& b, int src, T* out_T, double* out_d,
                    int blocksA, int blocksB, size_t ldsA, size_t ldsB,
                    hipStream_t s) {
  if (b.cpbs == 1)
    launch_G_batch_cpbs<T, 1>(b, src, out_T, out_d, blocksA, blocksB, ldsA, ldsB, s);
  else if (b.cpbs == 2)
    launch_G_batch_cpbs<T, 2>(b, src, out_T, out_d, blocksA, blocksB, ldsA, ldsB, s);
  else
    launch_G_batch_cpbs<T, 3>(b, src, out_T, out_d, blocksA, blocksB, ldsA, ldsB, s);
}

// Dynamic LDS above the default 64 KiB must be allowed per kernel before
// the first launch.
template <typename T, int CPBS>
void batch_allow_lds_cpbs(size_t slab) {
  const void* slabs[] = {
      reinterpret_cast<const void*>(&slab_fwd_batch_kernel<T, SRC_FIELD, CPBS>),
      reinterpret_cast<const void*>(&slab_fwd_batch_kernel<T, SRC_KP, CPBS>),
      reinterpret_cast<const void*>(&slab_inv_batch_kernel<T, double, DST_NORM, CPBS>),
      reinterpret_cast<const void*>(&slab_inv_batch_kernel<T, T, DST_DOT, CPBS>)};
  for (const void* f : slabs)
    RVE_HIP(hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)slab));
}

template <typename T>
void batch_allow_lds(size_t slab, size_t pencil) {
  batch_allow_lds_cpbs<T, 1>(slab);
  batch_allow_lds_cpbs<T, 2>(slab);
  batch_allow_lds_cpbs<T, 3>(slab);
  RVE_HIP(hipFuncSetAttribute(
      reinterpret_cast<const void*>(&pencil_batch_kernel<T>),
      hipFuncAttributeMaxDynamicSharedMemorySize, (int)pencil));
}

template void batch_allow_lds<float>(size_t, size_t);
template void batch_allow_lds<double>(size_t, size_t);
template void launch_G_batch<float>(const BatchSpec<float>&, int, float*,
                                    double*, int, int, size_t, size_t,
                                    hipStream_t);
template void launch_G_batch<double>(const BatchSpec<double>&, int, double*,
                                     double*, int, int, size_t, size_t,
                                     hipStream_t);
template void batch_lds<float>(int, int, int, size_t&, size_t&);
template void batch_lds<double>(int, int, int, size_t&, size_t&);
template void launch_G<float>(int, const SpectralLaunch<float>&, hipStream_t);
template void launch_G<double>(int, const SpectralLaunch<double>&, hipStream_t);

}  // namespace rve
