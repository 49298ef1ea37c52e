// Batched self-sorting (Stockham) FFT passes over data held in LDS.
//
// A batch of `ntr` transforms of length N is stored in LDS with element e of
// transform m at buf[(m0 + m) * tstride + e * estride]; rows of a 2-D tile use
// (tstride, estride) = (pitch, 1), columns use (1, pitch).  One radix-R pass with
// NS = product of the radices already applied computes, for every butterfly j in
// [0, N/R):
//     v[r] = in[j + r N/R] * W_{NS R}^{r (j mod NS)},   v = DFT_R(v),
//     out[(j / NS) NS R + (j mod NS) + r NS] = v[r].
// Starting from NS = 1 and multiplying NS by each radix leaves the transform in
// natural order after the last pass.  Passes run in place: all butterflies are
// first read into registers (load), then, after a block barrier, written back
// (store).  Consecutive lanes take consecutive transforms (m fastest), so with
// an odd row pitch both row and column passes spread a wavefront across banks.
//
// Twiddles come from a table tw[k] = exp(-2 pi i k / N), k < N (forward sign);
// inverse passes use the conjugate.
#pragma once

#include "cx.hpp"

namespace elfpie {

// TS / ES are the compile-time transform and element strides, so every LDS address
// of a butterfly is one base register plus immediate offsets.  NTR is the number of
// transforms when known at compile time (0: the runtime value ntr).
template <class T, int N, int R, int NS, bool INV, int NT, int MAXB, int TS, int ES, int NTR = 0>
struct StockhamPass {
  static constexpr int BPT = N / R;            // butterflies per transform
  static_assert(N % (NS * R) == 0, "radix product must divide N");

  // Element index (along the transform) of output r of butterfly j.
  __device__ static __forceinline__ int out_index(int j, int r) {
    const int jm = j % NS;
    return (j / NS) * NS * R + jm + r * NS;
  }

  // Butterfly b = tid + i*NT of a batch of ntr transforms: m = b mod ntr, j = b / ntr.
  __device__ static __forceinline__ void coords(int ntr, int tid, int (&m)[MAXB], int (&j)[MAXB],
                                                bool (&live)[MAXB]) {
    const int n = NTR > 0 ? NTR : ntr;
#pragma unroll
    for (int i = 0; i < MAXB; ++i) {
      const int b = tid + i * NT;
      live[i] = b < n * BPT;
      j[i] = b / n;
      m[i] = b - j[i] * n;
    }
  }

  // Read and transform this thread's butterflies.
  __device__ static __forceinline__ void load(const cx<T>* buf, int m0, const int (&m)[MAXB], const int (&j)[MAXB],
                                              const bool (&live)[MAXB], const cx<T>* tw, cx<T> (&v)[MAXB][R]) {
#pragma unroll
    for (int i = 0; i < MAXB; ++i) {
      if (live[i]) {
        const cx<T>* base = buf + (m0 + m[i]) * TS + j[i] * ES;
        const int jm = j[i] % NS;
#pragma unroll
        for (int r = 0; r < R; ++r) v[i][r] = base[r * BPT * ES];
        if (NS > 1) {
#pragma unroll
          for (int r = 1; r < R; ++r) {
            cx<T> w = tw[r * jm * (N / (NS * R))];
            if (INV) w.y = -w.y;
            v[i][r] = v[i][r] * w;
          }
        }
        dft<T, R, INV>(v[i]);
      }
    }
  }

  __device__ static __forceinline__ void store(cx<T>* buf, int m0, const int (&m)[MAXB], const int (&j)[MAXB],
                                               const bool (&live)[MAXB], const cx<T> (&v)[MAXB][R]) {
#pragma unroll
    for (int i = 0; i < MAXB; ++i) {
      if (live[i]) {
        cx<T>* base = buf + (m0 + m[i]) * TS + out_index(j[i], 0) * ES;
#pragma unroll
        for (int r = 0; r < R; ++r) base[r * NS * ES] = v[i][r];
      }
    }
  }

  // Full in-place pass over transforms m0 .. m0 + ntr - 1: load, barrier, store, barrier.
  __device__ static __forceinline__ void run(cx<T>* buf, int m0, int ntr, const cx<T>* tw, int tid) {
    int m[MAXB], j[MAXB];
    bool live[MAXB];
    coords(ntr, tid, m, j, live);
    cx<T> v[MAXB][R];
    load(buf, m0, m, j, live, tw, v);
    __syncthreads();
    store(buf, m0, m, j, live, v);
    __syncthreads();
  }
};

constexpr int ceil_div(int a, int b) { return (a + b - 1) / b; }

}  // namespace elfpie

namespace elfpie {

// Ordering of LDS accesses within one wavefront (no block barrier): every lane's
// earlier LDS stores are visible to the wavefront's later LDS loads.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Two-pass transform of one line (row or column of an LDS tile) of N = R1 * R2
// points by L = N / R1 lanes of one wavefront, so a wavefront transforms LPW lines
// with no block barrier.  Lane j of a line:
//   pass 1: reads elements j + r L (r < R1), DFT_R1, writes j R1 + r;
//   pass 2: butterflies jj = j + b L (b < B2 = R1 / L) read jj + r R1 (r < R2),
//           twiddle W_N^(r jj), DFT_R2; output r of butterfly jj is element jj + r R1.
// Element e of line t lives at t * PITCH + e (rows) or e * PITCH + t (columns); with
// PITCH = N + L the LPW lines of a wavefront fall on distinct LDS banks.
template <class T, int N, int R1, int R2, int PITCH>
struct LineFft {
  static constexpr int L = N / R1;
  static constexpr int LPW = 64 / L;
  static constexpr int B2 = R1 / L;
  static_assert(R1 * R2 == N && L * LPW == 64 && B2 * L == R1, "line decomposition");

  template <bool ROW>
  __device__ static __forceinline__ int at(int t, int e) { return ROW ? t * PITCH + e : e * PITCH + t; }

  // Transform line t (lanes with valid == false only take part in the wave sync);
  // leaves the outputs in v.
  template <bool INV, bool ROW>
  __device__ static __forceinline__ void run(cx<T>* buf, const cx<T>* tw, int t, int j, bool valid,
                                             cx<T> (&v)[B2][R2]) {
    if (valid) {
      cx<T> a[R1];
#pragma unroll
      for (int r = 0; r < R1; ++r) a[r] = buf[at<ROW>(t, j + r * L)];
      dft<T, R1, INV>(a);
#pragma unroll
      for (int r = 0; r < R1; ++r) buf[at<ROW>(t, j * R1 + r)] = a[r];
    }
    wave_sync();
    if (valid) {
#pragma unroll
      for (int b = 0; b < B2; ++b) {
        const int jj = j + b * L;
#pragma unroll
        for (int r = 0; r < R2; ++r) {
          cx<T> x = buf[at<ROW>(t, jj + r * R1)];
          if (r > 0) {
            cx<T> w = tw[r * jj];
            if (INV) w.y = -w.y;
            x = x * w;
          }
          v[b][r] = x;
        }
        dft<T, R2, INV>(v[b]);
      }
    }
  }

  template <bool ROW>
  __device__ static __forceinline__ void store(cx<T>* buf, int t, int j, bool valid, const cx<T> (&v)[B2][R2]) {
    if (valid) {
#pragma unroll
      for (int b = 0; b < B2; ++b)
#pragma unroll
        for (int r = 0; r < R2; ++r) buf[at<ROW>(t, j + b * L + r * R1)] = v[b][r];
    }
  }
};

}  // namespace elfpie
