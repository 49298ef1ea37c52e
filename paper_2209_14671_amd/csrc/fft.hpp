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

template <class T, int N, int R, int NS, bool INV, int NT, int MAXB>
struct StockhamPass {
  static constexpr int BPT = N / R;            // butterflies per transform
  static_assert(N % (NS * R) == 0, "radix product must divide N");

  // Read and transform this thread's butterflies.  Butterfly b = tid + i*NT of a
  // batch of ntr transforms: m = b mod ntr, j = b / ntr.
  __device__ static __forceinline__ void load(const cx<T>* buf, int m0, int ntr, int tstride, int estride,
                                              const cx<T>* tw, int tid, cx<T> (&v)[MAXB][R]) {
    const int total = ntr * BPT;
#pragma unroll
    for (int i = 0; i < MAXB; ++i) {
      const int b = tid + i * NT;
      if (b < total) {
        const int j = b / ntr;
        const int m = b - j * ntr;
        const cx<T>* base = buf + (m0 + m) * tstride;
        const int jm = j % NS;
#pragma unroll
        for (int r = 0; r < R; ++r) {
          cx<T> a = base[(j + r * BPT) * estride];
          if (NS > 1 && r > 0) {
            cx<T> w = tw[r * jm * (N / (NS * R))];
            if (INV) w.y = -w.y;
            a = a * w;
          }
          v[i][r] = a;
        }
        dft<T, R, INV>(v[i]);
      }
    }
  }

  // Element index (along the transform) of output r of butterfly j.
  __device__ static __forceinline__ int out_index(int j, int r) {
    const int jm = j % NS;
    return (j / NS) * NS * R + jm + r * NS;
  }

  __device__ static __forceinline__ void store(cx<T>* buf, int m0, int ntr, int tstride, int estride, int tid,
                                               const cx<T> (&v)[MAXB][R]) {
    const int total = ntr * BPT;
#pragma unroll
    for (int i = 0; i < MAXB; ++i) {
      const int b = tid + i * NT;
      if (b < total) {
        const int j = b / ntr;
        const int m = b - j * ntr;
        cx<T>* base = buf + (m0 + m) * tstride;
#pragma unroll
        for (int r = 0; r < R; ++r) base[out_index(j, r) * estride] = v[i][r];
      }
    }
  }

  // Full in-place pass: load, barrier, store, barrier.
  __device__ static __forceinline__ void run(cx<T>* buf, int m0, int ntr, int tstride, int estride,
                                             const cx<T>* tw, int tid) {
    cx<T> v[MAXB][R];
    load(buf, m0, ntr, tstride, estride, tw, tid, v);
    __syncthreads();
    store(buf, m0, ntr, tstride, estride, tid, v);
    __syncthreads();
  }
};

constexpr int ceil_div(int a, int b) { return (a + b - 1) / b; }

}  // namespace elfpie
