// Complex arithmetic and small in-register DFTs for the gfx950 kernels.
//
// Complex numbers are stored interleaved (re, im) and aligned to their full
// size, so a complex<float> is one 8-byte load and a complex<double> one 16-byte
// load.  The DFT butterflies compute X[k] = sum_n a[n] exp(-+2 pi i n k / R)
// (minus for the forward, plus for the inverse transform), unnormalised, with
// inputs and outputs in natural order.
#pragma once

#include <hip/hip_runtime.h>

namespace elfpie {

template <class T>
struct alignas(2 * sizeof(T)) cx {
  T x, y;
};

template <class T> __host__ __device__ __forceinline__ cx<T> operator+(cx<T> a, cx<T> b) { return {a.x + b.x, a.y + b.y}; }
template <class T> __host__ __device__ __forceinline__ cx<T> operator-(cx<T> a, cx<T> b) { return {a.x - b.x, a.y - b.y}; }
template <class T> __host__ __device__ __forceinline__ cx<T> operator*(cx<T> a, cx<T> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <class T> __host__ __device__ __forceinline__ cx<T> scale(cx<T> a, T s) { return {a.x * s, a.y * s}; }
template <class T> __host__ __device__ __forceinline__ cx<T> conj(cx<T> a) { return {a.x, -a.y}; }
// conj(a) * b
template <class T> __host__ __device__ __forceinline__ cx<T> cmulc(cx<T> a, cx<T> b) {
  return {a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x};
}
template <class T> __host__ __device__ __forceinline__ cx<T> mul_i(cx<T> a) { return {-a.y, a.x}; }

#ifndef ELFPIE_FAST_SIGN
#define ELFPIE_FAST_SIGN 1
#endif
// sign(d) in {-1, 0, 1}.  FP32: two operations instead of two compares, two selects and
// a conversion: d * 2^254 (an exponent shift) keeps the sign, is exact or overflows to
// +-inf, and is at least 2^105 in magnitude for every nonzero d (denormals included), so
// the median with -1 and 1 is exactly the sign (zero stays zero).
__device__ __forceinline__ float sign_unit(float d) {
  if (ELFPIE_FAST_SIGN) return __builtin_amdgcn_fmed3f(__builtin_ldexpf(d, 254), -1.0f, 1.0f);
  return float((d > 0.0f) - (d < 0.0f));
}
__device__ __forceinline__ double sign_unit(double d) { return double((d > 0.0) - (d < 0.0)); }
template <class T> __host__ __device__ __forceinline__ cx<T> mul_mi(cx<T> a) { return {a.y, -a.x}; }
template <class T> __host__ __device__ __forceinline__ T norm2(cx<T> a) { return a.x * a.x + a.y * a.y; }
template <class T> __host__ __device__ __forceinline__ cx<T> czero() { return {T(0), T(0)}; }

// Multiply by W_16^j = exp(-2 pi i j / 16) (forward) or its conjugate (inverse), with
// j in [0, 16) a compile-time constant after unrolling.
template <class T, bool INV>
__host__ __device__ __forceinline__ cx<T> twiddle16(cx<T> a, int j) {
  // cos(pi j / 8), sin(pi j / 8) for j = 0..15
  constexpr double c[16] = {1.0, 0.92387953251128675613, 0.70710678118654752440, 0.38268343236508977173,
                            0.0, -0.38268343236508977173, -0.70710678118654752440, -0.92387953251128675613,
                            -1.0, -0.92387953251128675613, -0.70710678118654752440, -0.38268343236508977173,
                            0.0, 0.38268343236508977173, 0.70710678118654752440, 0.92387953251128675613};
  constexpr double s[16] = {0.0, 0.38268343236508977173, 0.70710678118654752440, 0.92387953251128675613,
                            1.0, 0.92387953251128675613, 0.70710678118654752440, 0.38268343236508977173,
                            0.0, -0.38268343236508977173, -0.70710678118654752440, -0.92387953251128675613,
                            -1.0, -0.92387953251128675613, -0.70710678118654752440, -0.38268343236508977173};
  if (j == 0) return a;
  if (j == 4) return INV ? mul_i(a) : mul_mi(a);
  if (j == 8) return {-a.x, -a.y};
  if (j == 12) return INV ? mul_mi(a) : mul_i(a);
  const T cr = T(c[j]);
  const T si = INV ? T(s[j]) : T(-s[j]);  // exp(-+ i pi j / 8) = c -+ i s
  return {a.x * cr - a.y * si, a.x * si + a.y * cr};
}

template <class T, bool INV>
__host__ __device__ __forceinline__ void dft2(cx<T>* v) {
  const cx<T> t = v[0];
  v[0] = t + v[1];
  v[1] = t - v[1];
}

template <class T, bool INV>
__host__ __device__ __forceinline__ void dft4(cx<T>* v) {
  const cx<T> t0 = v[0] + v[2], t1 = v[0] - v[2], t2 = v[1] + v[3];
  cx<T> t3 = v[1] - v[3];
  t3 = INV ? mul_i(t3) : mul_mi(t3);
  v[0] = t0 + t2;
  v[2] = t0 - t2;
  v[1] = t1 + t3;
  v[3] = t1 - t3;
}

// Radix-2 split into two DFT4 halves plus the W8 twiddles.
template <class T, bool INV>
__host__ __device__ __forceinline__ void dft8(cx<T>* v) {
  cx<T> e[4] = {v[0], v[2], v[4], v[6]};
  cx<T> o[4] = {v[1], v[3], v[5], v[7]};
  dft4<T, INV>(e);
  dft4<T, INV>(o);
#pragma unroll
  for (int k = 1; k < 4; ++k) o[k] = twiddle16<T, INV>(o[k], 2 * k);
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    v[k] = e[k] + o[k];
    v[k + 4] = e[k] - o[k];
  }
}

// 4 x 4 decomposition: n = 4 n1 + n2, k = k1 + 4 k2.
template <class T, bool INV>
__host__ __device__ __forceinline__ void dft16(cx<T>* v) {
  cx<T> b[4][4];
#pragma unroll
  for (int n2 = 0; n2 < 4; ++n2) {
    cx<T> t[4] = {v[n2], v[4 + n2], v[8 + n2], v[12 + n2]};
    dft4<T, INV>(t);
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) b[n2][k1] = twiddle16<T, INV>(t[k1], n2 * k1);
  }
#pragma unroll
  for (int k1 = 0; k1 < 4; ++k1) {
    cx<T> t[4] = {b[0][k1], b[1][k1], b[2][k1], b[3][k1]};
    dft4<T, INV>(t);
#pragma unroll
    for (int k2 = 0; k2 < 4; ++k2) v[k1 + 4 * k2] = t[k2];
  }
}

// DFT3: X0 = a + b + c; X1, X2 = a - (b + c)/2 -/+ i s (b - c) with s = sin(2 pi / 3)
// (signs of the i term swapped for the inverse).
template <class T, bool INV>
__host__ __device__ __forceinline__ void dft3(cx<T>* v) {
  const T s3 = T(0.86602540378443864676);
  const cx<T> t1 = v[1] + v[2];
  const cx<T> t2 = v[0] - scale(t1, T(0.5));
  cx<T> t3 = scale(v[1] - v[2], s3);
  t3 = INV ? mul_i(t3) : mul_mi(t3);
  v[0] = v[0] + t1;
  v[1] = t2 + t3;
  v[2] = t2 - t3;
}

// Prime-factor (Good-Thomas) DFT of length P Q with coprime P (a power of two) and
// Q = 3: input n = (Q n1 + P n2) mod PQ, output k with k = k1 (mod P), k = k2 (mod Q);
// W_PQ^(nk) = W_P^(n1 k1) W_Q^(n2 k2), so no twiddles between the two stages.
template <class T, int P, bool INV>
__host__ __device__ __forceinline__ void dft_pfa3(cx<T>* v) {
  constexpr int N = 3 * P;
  cx<T> a[P][3];
#pragma unroll
  for (int n1 = 0; n1 < P; ++n1) {
#pragma unroll
    for (int n2 = 0; n2 < 3; ++n2) a[n1][n2] = v[(3 * n1 + P * n2) % N];
    dft3<T, INV>(a[n1]);
  }
#pragma unroll
  for (int k2 = 0; k2 < 3; ++k2) {
    cx<T> t[P];
#pragma unroll
    for (int n1 = 0; n1 < P; ++n1) t[n1] = a[n1][k2];
    if constexpr (P == 2) dft2<T, INV>(t);
    else if constexpr (P == 4) dft4<T, INV>(t);
    else dft8<T, INV>(t);
#pragma unroll
    for (int k1 = 0; k1 < P; ++k1) {
      // the k in [0, N) with k = k1 (mod P) and k = k2 (mod 3)
      int k = k1;
      while (k % 3 != k2) k += P;
      v[k] = t[k1];
    }
  }
}

template <class T, int R, bool INV>
__host__ __device__ __forceinline__ void dft(cx<T>* v) {
  if constexpr (R == 2) dft2<T, INV>(v);
  else if constexpr (R == 3) dft3<T, INV>(v);
  else if constexpr (R == 4) dft4<T, INV>(v);
  else if constexpr (R == 6) dft_pfa3<T, 2, INV>(v);
  else if constexpr (R == 8) dft8<T, INV>(v);
  else if constexpr (R == 12) dft_pfa3<T, 4, INV>(v);
  else if constexpr (R == 16) dft16<T, INV>(v);
  else if constexpr (R == 24) dft_pfa3<T, 8, INV>(v);
  else static_assert(R == 2, "unsupported radix");
}

}  // namespace elfpie
