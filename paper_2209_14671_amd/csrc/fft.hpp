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
// TWB selects the twiddle table: false, the natural table above; true, a table laid out
// per butterfly class, tw[(j mod NS) R + r] = exp(-2 pi i r (j mod NS) / (NS R)), so that the
// R - 1 twiddles of a butterfly are one address plus immediate offsets.
// A runtime divisor with its reciprocal: the quotient b / n for 0 <= b < 2^16 and
// 1 <= n < 2^16 is the high word of b * ceil(2^32 / n) (exact: the rounding-up error of
// the reciprocal times b stays below 1 / n), one multiply instead of a division sequence.
// Made once per kernel for a count that all threads share.
struct Div {
  int n;
  unsigned magic;
};
__device__ __forceinline__ Div make_div(int n) { return {n, n > 1 ? 0xFFFFFFFFu / unsigned(n) + 1u : 0u}; }
__device__ __forceinline__ int div_q(int b, Div d) { return d.n > 1 ? (int)__umulhi((unsigned)b, d.magic) : b; }

template <class T, int N, int R, int NS, bool INV, int NT, int MAXB, int TS, int ES, int NTR = 0,
          bool TWB = false>
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

  // The same for a runtime count held with its reciprocal.
  __device__ static __forceinline__ void coords(Div d, int tid, int (&m)[MAXB], int (&j)[MAXB], bool (&live)[MAXB]) {
#pragma unroll
    for (int i = 0; i < MAXB; ++i) {
      const int b = tid + i * NT;
      live[i] = b < d.n * BPT;
      j[i] = div_q(b, d);
      m[i] = b - j[i] * d.n;
    }
  }

  // Butterfly i of this thread: read, twiddle, transform.
  __device__ static __forceinline__ void load_one(const cx<T>* buf, int m0, int m, int j, const cx<T>* tw,
                                                  cx<T> (&v)[R]) {
    const cx<T>* base = buf + (m0 + m) * TS + j * ES;
    const int jm = j % NS;
#pragma unroll
    for (int r = 0; r < R; ++r) v[r] = base[r * BPT * ES];
    if (NS > 1) {
#pragma unroll
      for (int r = 1; r < R; ++r) {
        cx<T> w = TWB ? tw[jm * R + r] : tw[r * jm * (N / (NS * R))];
        if (INV) w.y = -w.y;
        v[r] = v[r] * w;
      }
    }
    dft<T, R, INV>(v);
  }

  // Read and transform this thread's butterflies.  With two per thread, a wave whose
  // lanes hold any second butterfly runs both as one straight sequence (the reads of both
  // first; a lane without one reads butterfly 0 of transform 0 and drops it at the store),
  // so that the second does not wait behind the first.
  __device__ static __forceinline__ void load(const cx<T>* buf, int m0, const int (&m)[MAXB], const int (&j)[MAXB],
                                              const bool (&live)[MAXB], const cx<T>* tw, cx<T> (&v)[MAXB][R]) {
    if constexpr (MAXB == 2) {
      if (__builtin_amdgcn_ballot_w64(live[1]) != 0) {
        load_one(buf, m0, live[0] ? m[0] : 0, live[0] ? j[0] : 0, tw, v[0]);
        load_one(buf, m0, live[1] ? m[1] : 0, live[1] ? j[1] : 0, tw, v[1]);
        return;
      }
    }
#pragma unroll
    for (int i = 0; i < MAXB; ++i)
      if (live[i]) load_one(buf, m0, m[i], j[i], tw, v[i]);
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
  template <class Count>
  __device__ static __forceinline__ void run(cx<T>* buf, int m0, Count ntr, const cx<T>* tw, int tid) {
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
