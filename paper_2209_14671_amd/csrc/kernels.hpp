// gfx950 kernels of one Elfpie iteration (Zhang et al., arXiv 2209.14671, Sec. 3,
// Algorithm 1).  All transforms are unnormalised DFTs; the unitary scalings and
// the centring of the spectra are folded into the neighbouring elementwise work:
// for even n, ifftshift before / fftshift after a DFT equals a (-1)^(x+y) factor on
// the spatial side, and for the per-LED path that factor cancels between the
// inverse transform (o) and the forward transform of W, because W is o times a
// real field.  So the per-LED path needs no sign at all.
#pragma once

#include <cfloat>
#include <cmath>
#include <type_traits>

#include "cx.hpp"
#include "fft.hpp"
#include "params.hpp"

namespace elfpie {

constexpr int kMaxLo = 256;  // largest low-resolution side any kernel stages in LDS

// ---------------------------------------------------------------------------
// Deterministic block reduction of a double (fixed shuffle and slot order).
// ---------------------------------------------------------------------------
template <int NT>
__device__ __forceinline__ double block_sum(double v, double* scratch /* NT/64 */) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) scratch[wid] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0) {
    for (int i = 0; i < NT / 64; ++i) s += scratch[i];
  }
  __syncthreads();
  return s;  // valid in thread 0
}

// sqrt(x), 1 / sqrt(x) and 1 / x: the hardware instructions (about 1 ulp) in FP32,
// correctly rounded in FP64.
__device__ __forceinline__ float sqrt_t(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ double sqrt_t(double x) { return sqrt(x); }
__device__ __forceinline__ float rsqrt_t(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ double rsqrt_t(double x) { return 1.0 / sqrt(x); }
__device__ __forceinline__ float rcp_t(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double rcp_t(double x) { return 1.0 / x; }

// base[off] with a 32-bit element offset from a block-uniform base, so that the address is
// the base register plus one 32-bit offset register (no 64-bit arithmetic per element).
template <class X>
__device__ __forceinline__ X& at_off(X* base, unsigned off) {
  return *reinterpret_cast<X*>(reinterpret_cast<char*>(base) + off * unsigned(sizeof(X)));
}
template <class X>
__device__ __forceinline__ const X& at_off(const X* base, unsigned off) {
  return *reinterpret_cast<const X*>(reinterpret_cast<const char*>(base) + off * unsigned(sizeof(X)));
}

// L1 term rho(d) = sqrt(d^2 + eps^2) - eps (eps > 0) or |d| and its derivative.
// Per pixel these are a multiply-add and one reciprocal square root in FP32 (no IEEE
// division or square-root expansion); the exact sign of eps = 0 is kept.
template <class T>
__device__ __forceinline__ T rho(T d, T eps) {
  if (eps > T(0)) return sqrt_t(d * d + eps * eps) - eps;
  return fabs(d);
}
template <class T>
__device__ __forceinline__ T omega(T d, T eps) {
  if (eps > T(0)) return d * rsqrt_t(d * d + eps * eps);
  return T((d > T(0)) - (d < T(0)));
}
// 1 / ||c|| for the isotropic normaliser (0 at the origin when eps = 0).
// The scaling g of the fidelity (Eq. 3) on an intensity: sqrt, identity, x^gamma, ln(x + 1).
__device__ __forceinline__ float pow_t(float x, float y) { return powf(x, y); }
__device__ __forceinline__ double pow_t(double x, double y) { return pow(x, y); }
__device__ __forceinline__ float log1p_t(float x) { return log1pf(x); }
__device__ __forceinline__ double log1p_t(double x) { return log1p(x); }

// Residual g(|o|^2) - g(I) from i2 = |o|^2 and the reading m.  SCALED adds the
// Sec. 6.3 scalings (x^gamma, ln(x + 1)); without it only Eq. 4 and Eq. 5 are
// compiled, which keeps the per-pixel code of the common kernel small.
template <bool SCALED, class T>
__device__ __forceinline__ T fid_residual(int fid, T i2, T m, T gam) {
  const T mp = m > T(0) ? m : T(0);
  if (fid == 0) return sqrt_t(i2) - sqrt_t(mp);
  if constexpr (SCALED) {
    if (fid == 2) return pow_t(i2, gam) - pow_t(mp, gam);
    if (fid == 3) return log1p_t(i2) - log1p_t(mp);
  }
  return i2 - m;
}

// dL/d(conj o) = q g'(|o|^2) o; g'(0) is taken as 0 for the powers.
template <bool SCALED, class T>
__device__ __forceinline__ cx<T> fid_wirtinger(int fid, cx<T> ov, T q, T gam) {
  const T i2 = norm2(ov);
  if (fid == 0) return i2 > T(0) ? scale(ov, T(0.5) * q * rsqrt_t(i2)) : czero<T>();
  if constexpr (SCALED) {
    if (fid == 2) return i2 > T(0) ? scale(ov, q * gam * pow_t(i2, gam - T(1))) : czero<T>();
    if (fid == 3) return scale(ov, q / (T(1) + i2));
  }
  return scale(ov, q);
}

template <class T>
__device__ __forceinline__ T inv_norm(T s2, T eps) {
  if (eps > T(0)) return rsqrt_t(s2 + eps * eps);
  return s2 > T(0) ? rsqrt_t(s2) : T(0);
}

// ---------------------------------------------------------------------------
// Per-LED fused kernel: one workgroup per LED, the n_lo x n_lo tile in LDS.
// ---------------------------------------------------------------------------

// Loads kept in flight per batch of a gather of ppt pixels per thread: the largest of
// 8, 6, 4, 3, 2, 1 that divides ppt, so the batches cover exactly ppt pixels.
constexpr int gather_batch(int ppt) {
  return ppt % 8 == 0 ? 8 : ppt % 6 == 0 ? 6 : ppt % 4 == 0 ? 4 : ppt % 3 == 0 ? 3 : ppt % 2 == 0 ? 2 : 1;
}

template <int N> struct LedShape;
#ifndef ELFPIE_LED32_NT
#define ELFPIE_LED32_NT 256
#endif
#ifndef ELFPIE_LED96_NT
#define ELFPIE_LED96_NT 512
#endif
template <> struct LedShape<32> { static constexpr int NT = ELFPIE_LED32_NT, R1 = 8, R2 = 4; };
template <> struct LedShape<96> { static constexpr int NT = ELFPIE_LED96_NT, R1 = 16, R2 = 6; };
#ifndef ELFPIE_LED64_NT
#define ELFPIE_LED64_NT 512
#endif
template <> struct LedShape<64> { static constexpr int NT = ELFPIE_LED64_NT, R1 = 8, R2 = 8; };
#ifndef ELFPIE_LED128_NT
#define ELFPIE_LED128_NT 1024
#endif
template <> struct LedShape<128> { static constexpr int NT = ELFPIE_LED128_NT, R1 = 16, R2 = 8; };

// Steps of the per-LED branch (one LED per workgroup):
//   gather   X = P * M_k Psi on the pupil support                  (Eq. 1)
//   inverse  o = F_B X / (r n_lo): rows holding support, then columns
//   residual e = |o|^2 - I  or  |o| - sqrt(I)                        (Eq. 5 / Eq. 4)
//   features forward differences of e, L1 loss, omega               (Eq. 12)
//   adjoint  q = grad^T omega, dL/d(conj o) = q o  or  q o / (2|o|)  (Eq. 11 / Eq. 10)
//   forward  Y = F_B^H dL/d(conj o): all rows, then support columns
//   outputs  C = conj(P) Y and D = conj(M_k Psi) Y on the support    (Eq. 9, Eq. 18)
// Step mode advances the shared step counter t once per iteration, here: nothing in
// this launch reads it, and the spectrum and pupil updates that follow read the new value.
__device__ __forceinline__ void led_bump_step(const LedArgs& a, int k, int tid) {
  if (a.t_bump && k == 0 && tid == 0) *a.t_bump = *a.t_bump + 1;
}

#ifndef ELFPIE_LED_XCD
#define ELFPIE_LED_XCD 1
#endif
#ifndef ELFPIE_LED_TSUM
#define ELFPIE_LED_TSUM 1
#endif
#ifndef ELFPIE_LED_NBR
#define ELFPIE_LED_NBR 1
#endif
#ifndef ELFPIE_LED_TWB
#define ELFPIE_LED_TWB 1
#endif
#ifndef ELFPIE_LED_AMPC
#define ELFPIE_LED_AMPC 1
#endif
#ifndef ELFPIE_STRIP_TSUM
#define ELFPIE_STRIP_TSUM 1
#endif
#ifndef ELFPIE_OBJ_XCD
#define ELFPIE_OBJ_XCD 1  // object blocks of the per-LED launch: neighbouring strips per XCD
#endif
#ifndef ELFPIE_STRIP_XCD
#define ELFPIE_STRIP_XCD 1
#endif
#ifndef ELFPIE_UPD_PAIR
#define ELFPIE_UPD_PAIR 16  // neighbouring update rows per XCD run (at most)
#endif
// Workgroup b of a launch of n runs on XCD b mod 8.  Renumbering b so that each XCD takes
// a run of consecutive LEDs (neighbours in the LED grid, whose spectrum windows overlap)
// lets their window reads share that XCD's L2.  A bijection of 0 .. n - 1 for any n.
__device__ __forceinline__ int xcd_order(int b, int n) {
  const int q = n / 8, r = n % 8, x = b % 8;
  return x * q + min(x, r) + b / 8;
}

// The object-branch role of the per-LED launch (defined with the other object kernels):
// block b of the launch's nblk object blocks, its shared memory carved from `lds`.
template <class T, int N, int NT>
__device__ void obj_strip_wide(const LedObjArgs& o, int b, char* lds);
template <class T, int N, int NT>
constexpr size_t obj_wide_lds_bytes();
template <class T>
__device__ __forceinline__ cx<T> pupil_gauss3(const cx<T>* P, int n, int p, double w_c, double w_e, double w_k);

// Every pass of each 2-D transform is spread over the whole block (StockhamPass).
// SCALED: compiled with the Sec. 6.3 fidelity scalings (used only for them).
// STORED: the LED_STORED mode (fields read, not recomputed), in its own instantiation.
// NOBJ > 0: the last a.obj.nblk blocks of the launch run the object branch of an
// NOBJ x NOBJ spectrum (obj_strip_wide) in the LDS of the per-LED tile instead.
template <class T, int N, bool SCALED = false, bool STORED = false, int NOBJ = 0>
__global__ __launch_bounds__(LedShape<N>::NT) void k_led(LedArgs a) {
  using Sh = LedShape<N>;
  constexpr int NT = Sh::NT, R1 = Sh::R1, R2 = Sh::R2, PITCH = N + 1;
  static_assert(R1 * R2 == N, "two-pass decomposition");
  constexpr bool TWB = ELFPIE_LED_TWB != 0;
  constexpr int MB1 = ceil_div(N * (N / R1), NT);
  constexpr int MB2 = ceil_div(N * (N / R2), NT);
  static_assert(MB2 * NT == N * R1, "the last pass gives every thread whole butterflies");
  constexpr int PPT = N * N / NT;        // pixels per thread in the gather
  constexpr int GB = PPT <= 16 ? PPT : gather_batch(PPT);  // loads kept in flight per batch
  static_assert(PPT * NT == N * N && PPT % GB == 0, "the gather covers the tile exactly");
  // row passes (transform stride PITCH) and column passes (element stride PITCH)
  using P1iR = StockhamPass<T, N, R1, 1, true, NT, MB1, PITCH, 1>;
  using P2iR = StockhamPass<T, N, R2, R1, true, NT, MB2, PITCH, 1, 0, TWB>;
  using P1iC = StockhamPass<T, N, R1, 1, true, NT, MB1, 1, PITCH, N>;
  using P2iC = StockhamPass<T, N, R2, R1, true, NT, MB2, 1, PITCH, N, TWB>;
  using P1fR = StockhamPass<T, N, R1, 1, false, NT, MB1, PITCH, 1, N>;
  using P2fR = StockhamPass<T, N, R2, R1, false, NT, MB2, PITCH, 1, N, TWB>;
  using P1fC = StockhamPass<T, N, R1, 1, false, NT, MB1, 1, PITCH>;
  using P2fC = StockhamPass<T, N, R2, R1, false, NT, MB2, 1, PITCH, 0, TWB>;

  // the tile; in a launch with object blocks, large enough for their arrays too
  constexpr size_t TILE = size_t(N) * PITCH;
  constexpr size_t OBJ = NOBJ > 0 ? (obj_wide_lds_bytes<T, (NOBJ > 0 ? NOBJ : 512), NT>() + sizeof(cx<T>) - 1) / sizeof(cx<T>) : 0;
  __shared__ cx<T> img[TILE > OBJ ? TILE : OBJ];
  __shared__ cx<T> twl[N];
  __shared__ int4 srow[N];  // per row: first and last support column, offset of s - first
  __shared__ double red[NT / 64];
  // the second passes' twiddles per butterfly class (R1 classes of R2 entries)
  __shared__ cx<T> twb_s[TWB ? N : 1];
  const cx<T>* twb = TWB ? twb_s : twl;

  const int tid = threadIdx.x;
  int nled = gridDim.x;
  if constexpr (NOBJ > 0) {
    static_assert(obj_wide_lds_bytes<T, NOBJ, NT>() <= sizeof(img), "object blocks fit the tile's LDS");
    nled -= a.obj.nblk;
    if ((int)blockIdx.x >= nled) {  // block-uniform: an object block
      // runs of neighbouring strips per XCD: they share the halo columns of T1 and the
      // cache lines of T2 at their edges, which each XCD then fetches and writes back once
      const int bo = blockIdx.x - nled;
      const int sb = ELFPIE_OBJ_XCD ? xcd_order(bo, a.obj.nblk) : bo;
      obj_strip_wide<T, NOBJ, NT>(a.obj, sb, reinterpret_cast<char*>(img));
      return;
    }
  }
  const int k = ELFPIE_LED_XCD ? xcd_order(blockIdx.x, nled) : (int)blockIdx.x;
  led_bump_step(a, k, tid);
  const cx<T>* psi = static_cast<const cx<T>*>(a.psi);
  const cx<T>* P = static_cast<const cx<T>*>(a.P);
  if constexpr (NOBJ > 0) {
    // a slice of the pupil's pre-filtered copy (P is read-only in this launch)
    if (a.obj.Pf) {
      constexpr int NP = N * N;
      const int per = (NP + nled - 1) / nled, p1 = min(NP, (k + 1) * per);
      for (int p = k * per + tid; p < p1; p += NT)
        static_cast<cx<T>*>(a.obj.Pf)[p] = pupil_gauss3<T>(P, N, p, a.obj.w_c, a.obj.w_e, a.obj.w_k);
    }
  }
  for (int i = tid; i < N; i += NT) {
    twl[i] = static_cast<const cx<T>*>(a.tw)[i];
    srow[i] = make_int4(a.xlo[i], a.xhi[i], a.rowoff[i] - a.xlo[i], 0);
    if (TWB) twb_s[i] = static_cast<const cx<T>*>(a.tw)[(i % R2) * (i / R2)];  // W_N^(r jm), N = R1 R2
  }
  const int y0 = a.win[2 * k], x0 = a.win[2 * k + 1];
  const cx<T>* win = psi + (size_t)y0 * a.n_hi + x0;
  const int mode = a.mode;
  constexpr bool stored = STORED;
  __syncthreads();

  // register (i, r) of the last column pass holds pixel y = jj[i] + r R1, x = mm[i]
  int mm[MB2], jj[MB2];
  bool lv[MB2];
  cx<T> o[MB2][R2];
  const bool need_e = (mode & (LED_GRAD | LED_LOSS)) != 0;
  const T* meas = static_cast<const T*>(a.meas) + (size_t)k * N * N;
  T mv[MB2][R2];
  auto load_meas = [&]() {
    if (need_e) {
#pragma unroll
      for (int i = 0; i < MB2; ++i) {
        const int j = jj[i], x = mm[i];
#pragma unroll
        for (int r = 0; r < R2; ++r) mv[i][r] = meas[(size_t)(j + r * R1) * N + x];
      }
    }
  };
  if constexpr (stored) {
    P2iC::coords(N, tid, mm, jj, lv);
    // o from the fields of a forward call, in the kernel's (-1)^(x+y) frame
    const cx<T>* fk = static_cast<const cx<T>*>(a.fields) + (size_t)k * N * N;
#pragma unroll
    for (int i = 0; i < MB2; ++i) {
#pragma unroll
      for (int r = 0; r < R2; ++r) {
        const int y = jj[i] + r * R1, x = mm[i];
        const cx<T> f = fk[y * N + x];
        o[i][r] = ((x + y) & 1) ? cx<T>{-f.x, -f.y} : f;
      }
    }
    load_meas();
  } else {
    // gather X = P * window, zeros off the support: only lanes on the support load, a
    // batch of GB loads in flight at once.
#pragma unroll
    for (int i0 = 0; i0 < PPT; i0 += GB) {
      cx<T> pv[GB], wv[GB];
      bool in[GB];
#pragma unroll
      for (int i = 0; i < GB; ++i) {
        const int p = tid + (i0 + i) * NT;
        const int y = p / N, x = p % N;
        const int4 rw = srow[y];
        in[i] = x >= rw.x && x <= rw.y;
        pv[i] = czero<T>();
        wv[i] = czero<T>();
        if (in[i]) {  // 32-bit offsets from the block's base addresses
          pv[i] = at_off(P, unsigned(p));
          wv[i] = at_off(win, unsigned(y * a.n_hi + x));
        }
      }
#pragma unroll
      for (int i = 0; i < GB; ++i) {
        const int p = tid + (i0 + i) * NT;
        const int y = p / N, x = p % N;
        img[y * PITCH + x] = in[i] ? pv[i] * wv[i] : czero<T>();
      }
    }
    __syncthreads();

    // inverse DFT: rows that hold support pixels, then every column
    const Div nband = make_div(a.y_max - a.y_min + 1);
    P1iR::run(img, a.y_min, nband, twl, tid);
    P2iR::run(img, a.y_min, nband, twb, tid);
    P1iC::run(img, 0, N, twl, tid);
    P2iC::coords(N, tid, mm, jj, lv);
    load_meas();  // in flight during the last pass's loads
    P2iC::load(img, 0, mm, jj, lv, twb, o);
  }
  __syncthreads();

  const T sc = T(a.inv_scale);
  const T osc = stored ? T(1) : sc;  // stored fields are scaled already
  const T eps = T(a.eps);
  const T gam = T(a.fid_gamma);
  // real residual, row pitch PITCH, one row and one element into the (now dead) tile, so
  // that the neighbour reads of the loop below may step one row or column off the grid
  // without leaving the array (such values are discarded by the boundary selects)
  static_assert(2 * N * PITCH > (N + 1) * PITCH + N, "room for the shifted residual");
  T* eb = reinterpret_cast<T*>(img) + (ELFPIE_LED_NBR ? PITCH + 1 : 0);
  // the gradient and loss modes under the amplitude or intensity fidelity (no field or
  // image output): the residual with the fidelity fixed outside the pixel loop
  const bool plain = ELFPIE_LED_AMPC && !SCALED && need_e && !(mode & (LED_FIELDS | LED_INTENS)) &&
                     (a.fidelity == 0 || a.fidelity == 1);
  auto residual_only = [&](auto amp_c) {
    constexpr bool AMP = decltype(amp_c)::value;
#pragma unroll
    for (int i = 0; i < MB2; ++i) {
#pragma unroll
      for (int r = 0; r < R2; ++r) {
        const int y = jj[i] + r * R1;
        const cx<T> ov = scale(o[i][r], osc);
        o[i][r] = ov;
        const T i2 = norm2(ov), m = mv[i][r];
        eb[y * PITCH + mm[i]] = AMP ? sqrt_t(i2) - sqrt_t(m > T(0) ? m : T(0)) : i2 - m;
      }
    }
  };
  if (plain && a.fidelity == 0) residual_only(std::true_type{});
  else if (plain) residual_only(std::false_type{});
  else
#pragma unroll
  for (int i = 0; i < MB2; ++i) {
    const int j = jj[i], x = mm[i];
#pragma unroll
    for (int r = 0; r < R2; ++r) {
      const int y = j + r * R1;
      const cx<T> ov = scale(o[i][r], osc);
      o[i][r] = ov;
      const size_t pix = (size_t)k * N * N + (size_t)y * N + x;
      if (mode & LED_FIELDS) {
        const cx<T> f = ((x + y) & 1) ? cx<T>{-ov.x, -ov.y} : ov;
        static_cast<cx<T>*>(a.fields)[pix] = f;
      }
      const T i2 = norm2(ov);
      if (mode & LED_INTENS) static_cast<T*>(a.intens)[pix] = i2;
      if (need_e) {
        const T m = mv[i][r];
        eb[y * PITCH + x] = fid_residual<SCALED>(a.fidelity, i2, m, gam);
      }
    }
  }
  if (!need_e) return;
  __syncthreads();

  // features, loss and dL/d(conj o), written over the field registers
  auto E = [&](int yy, int xx) -> T { return eb[yy * PITCH + xx]; };
  double lsum = 0.0;
  if (!SCALED && a.norm == 0 && !(eps > T(0))) {
    // the exact anisotropic L1 (omega = sign, rho = |.|) under the intensity or amplitude
    // fidelity, without a branch per pixel: clamped reads and selects; the same
    // arithmetic as the general loop below
    auto sgn = [](T d) { return sign_unit(d); };
    T lpart = T(0);  // this lane's pixels, summed in T and added to the FP64 partial once
    auto fast_pass = [&](auto amp_c) {
    constexpr bool AMP = decltype(amp_c)::value;
#pragma unroll
    for (int i = 0; i < MB2; ++i) {
      const int j = jj[i], x = mm[i];
      const int xr = ELFPIE_LED_NBR ? x + 1 : min(x + 1, N - 1), xl = ELFPIE_LED_NBR ? x - 1 : max(x - 1, 0);
#pragma unroll
      for (int r = 0; r < R2; ++r) {
        const int y = j + r * R1;
        const int yd = ELFPIE_LED_NBR ? y + 1 : min(y + 1, N - 1), yu = ELFPIE_LED_NBR ? y - 1 : max(y - 1, 0);
        const T e = E(y, x), er = E(y, xr), ed = E(yd, x), el = E(y, xl), eu = E(yu, x);
        const T dx0 = (x < N - 1) ? er - e : T(0);
        const T dy0 = (y < N - 1) ? ed - e : T(0);
        const T dxm = (x > 0) ? e - el : T(0);
        const T dym = (y > 0) ? e - eu : T(0);
        const T q = sgn(dxm) - sgn(dx0) + sgn(dym) - sgn(dy0);
        if (ELFPIE_LED_TSUM) lpart += fabs(dx0) + fabs(dy0);
        else lsum += double(fabs(dx0) + fabs(dy0));
        const cx<T> ov = o[i][r];
        if constexpr (AMP) {
          const T i2 = norm2(ov);
          o[i][r] = scale(ov, i2 > T(0) ? T(0.5) * q * rsqrt_t(i2) : T(0));
        } else {
          o[i][r] = scale(ov, q);
        }
      }
    }
    };
    if (a.fidelity == 0) fast_pass(std::true_type{});
    else fast_pass(std::false_type{});
    lsum += double(lpart);
  } else {
#pragma unroll
  for (int i = 0; i < MB2; ++i) {
    const int j = jj[i], x = mm[i];
#pragma unroll
    for (int r = 0; r < R2; ++r) {
      const int y = j + r * R1;
      const T e = E(y, x);
      const T dx0 = (x < N - 1) ? E(y, x + 1) - e : T(0);
      const T dy0 = (y < N - 1) ? E(y + 1, x) - e : T(0);
      T q;
      if (a.norm == 0) {
        const T dxm = (x > 0) ? e - E(y, x - 1) : T(0);
        const T dym = (y > 0) ? e - E(y - 1, x) : T(0);
        q = omega(dxm, eps) - omega(dx0, eps) + omega(dym, eps) - omega(dy0, eps);
        lsum += double(rho(dx0, eps) + rho(dy0, eps));
      } else {
        const T s0 = dx0 * dx0 + dy0 * dy0;
        const T inv0 = inv_norm(s0, eps);
        q = -(dx0 + dy0) * inv0;
        if (x > 0) {  // normaliser at (y, x-1)
          const T el = E(y, x - 1);
          const T gx = e - el;
          const T gy = (y < N - 1) ? E(y + 1, x - 1) - el : T(0);
          q += gx * inv_norm(gx * gx + gy * gy, eps);
        }
        if (y > 0) {  // normaliser at (y-1, x)
          const T eu = E(y - 1, x);
          const T gy = e - eu;
          const T gx = (x < N - 1) ? E(y - 1, x + 1) - eu : T(0);
          q += gy * inv_norm(gx * gx + gy * gy, eps);
        }
        lsum += eps > T(0) ? double(sqrt_t(s0 + eps * eps) - eps) : double(sqrt_t(s0));
      }
      o[i][r] = fid_wirtinger<SCALED>(a.fidelity, o[i][r], q, gam);
    }
  }
  }
  __syncthreads();  // every residual read is done; the tile can be overwritten

  const bool grad = (mode & LED_GRAD) != 0;
  if (grad) {
#pragma unroll
    for (int i = 0; i < MB2; ++i) {
      const int j = jj[i], x = mm[i];
#pragma unroll
      for (int r = 0; r < R2; ++r) img[(j + r * R1) * PITCH + x] = o[i][r];
    }
  }
  // the per-wave sums now; their sum over the block (thread 0, in wave order) at the end,
  // so that no wave waits for it
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) lsum += __shfl_down(lsum, off, 64);
  if ((tid & 63) == 0) red[tid >> 6] = lsum;
  auto store_loss = [&]() {
    if (tid == 0) {
      double tot = 0.0;
      for (int w = 0; w < NT / 64; ++w) tot += red[w];
      a.fid_partial[k] = tot;
    }
  };
  __syncthreads();  // the gradient in the tile (and the slots) before the forward DFT reads it
  if (!grad) {
    store_loss();
    return;
  }

  // forward DFT of dL/d(conj o): all rows, then only columns that hold support
  P1fR::run(img, 0, N, twl, tid);
  P2fR::run(img, 0, N, twb, tid);
  const Div ncol = make_div(a.x_max - a.x_min + 1);
  P1fC::run(img, a.x_min, ncol, twl, tid);
  P2fC::coords(ncol, tid, mm, jj, lv);
  cx<T> Y[MB2][R2];
  P2fC::load(img, a.x_min, mm, jj, lv, twb, Y);

  // contributions on the support; the window and pupil loads are issued together
  cx<T>* C = static_cast<cx<T>*>(a.C) + (size_t)k * a.S;
  cx<T>* D = static_cast<cx<T>*>(a.D) + (size_t)k * a.S;
#pragma unroll
  for (int i = 0; i < MB2; ++i) {
    const bool live = lv[i];
    const int j = jj[i];
    const int x = live ? a.x_min + mm[i] : 0;
    cx<T> pw[R2], ww[R2];
#pragma unroll
    for (int r = 0; r < R2; ++r) {
      const int y = live ? j + r * R1 : 0;
      pw[r] = at_off(P, unsigned(y * N + x));
      ww[r] = at_off(win, unsigned(y * a.n_hi + x));
    }
    if (live) {
      // the support tests and offsets of the column's R2 pixels first, each row entry read
      // whole and used unconditionally (one LDS read, no chain of dependent reads), then
      // the stores
      int so[R2];
      bool ok[R2];
#pragma unroll
      for (int r = 0; r < R2; ++r) {
        const int4 rw = srow[j + r * R1];
        ok[r] = (x >= rw.x) & (x <= rw.y);
        so[r] = ok[r] ? rw.z + x : 0;
      }
#pragma unroll
      for (int r = 0; r < R2; ++r) {
        if (ok[r]) {
          const cx<T> yv = scale(Y[i][r], sc);
          at_off(C, unsigned(so[r])) = cmulc(pw[r], yv);
          at_off(D, unsigned(so[r])) = cmulc(ww[r], yv);
        }
      }
    }
  }
  store_loss();
}

// dL/d(conj o_m) = f o_m for every LED m of an image: the real factor
// f = q g'(S) with S the image's summed intensity (g'(0) taken as 0 for the powers).
template <bool SCALED, class T>
__device__ __forceinline__ T fid_slope(int fid, T S, T q, T gam) {
  if (fid == 0) return S > T(0) ? T(0.5) * q * rsqrt_t(S) : T(0);
  if constexpr (SCALED) {
    if (fid == 2) return S > T(0) ? q * gam * pow_t(S, gam - T(1)) : T(0);
    if (fid == 3) return q / (T(1) + S);
  }
  return q;
}

// ---------------------------------------------------------------------------
// Multiplexed illumination (Eq. 1 with M > 1): one workgroup per image, whose M
// LEDs are handled in turn through the same LDS tile.
//   for each LED m: gather, inverse transform, o_m to `fields` (the caller's
//     output, its stored fields, or plan scratch), S += |o_m|^2;
//   residual g(S) - g(I), features, loss and the factor f = q g'(S);
//   for each LED m: W_m = f o_m read back, forward transform, contributions.
// The fields are kept in the true (centred) frame, as elfpie_forward writes them.
// ---------------------------------------------------------------------------
template <class T, int N, bool SCALED>
__global__ __launch_bounds__(LedShape<N>::NT) void k_led_mux(LedArgs a) {
  using Sh = LedShape<N>;
  constexpr int NT = Sh::NT, R1 = Sh::R1, R2 = Sh::R2, PITCH = N + 1;
  constexpr int MB1 = ceil_div(N * (N / R1), NT);
  constexpr int MB2 = ceil_div(N * (N / R2), NT);
  static_assert(MB2 * NT == N * R1, "the last pass gives every thread whole butterflies");
  constexpr int PPT = N * N / NT;
  constexpr int GB = gather_batch(PPT);
  using P1iR = StockhamPass<T, N, R1, 1, true, NT, MB1, PITCH, 1>;
  using P2iR = StockhamPass<T, N, R2, R1, true, NT, MB2, PITCH, 1>;
  using P1iC = StockhamPass<T, N, R1, 1, true, NT, MB1, 1, PITCH, N>;
  using P2iC = StockhamPass<T, N, R2, R1, true, NT, MB2, 1, PITCH, N>;
  using P1fR = StockhamPass<T, N, R1, 1, false, NT, MB1, PITCH, 1, N>;
  using P2fR = StockhamPass<T, N, R2, R1, false, NT, MB2, PITCH, 1, N>;
  using P1fC = StockhamPass<T, N, R1, 1, false, NT, MB1, 1, PITCH>;
  using P2fC = StockhamPass<T, N, R2, R1, false, NT, MB2, 1, PITCH>;

  __shared__ cx<T> img[N * PITCH];
  __shared__ cx<T> twl[N];
  __shared__ int4 srow[N];  // per row: first and last support column, offset of s - first
  __shared__ double red[NT / 64];

  const int tid = threadIdx.x;
  const int im = blockIdx.x;  // image
  const int M = a.mux;
  led_bump_step(a, im, tid);
  const cx<T>* psi = static_cast<const cx<T>*>(a.psi);
  const cx<T>* P = static_cast<const cx<T>*>(a.P);
  cx<T>* F = static_cast<cx<T>*>(a.fields);
  for (int i = tid; i < N; i += NT) {
    twl[i] = static_cast<const cx<T>*>(a.tw)[i];
    srow[i] = make_int4(a.xlo[i], a.xhi[i], a.rowoff[i] - a.xlo[i], 0);
  }
  const int mode = a.mode;
  const bool stored = (mode & LED_STORED) != 0;
  const T sc = T(a.inv_scale);
  __syncthreads();

  int mm[MB2], jj[MB2];
  bool lv[MB2];
  P2iC::coords(N, tid, mm, jj, lv);
  T S[MB2][R2];
#pragma unroll
  for (int i = 0; i < MB2; ++i)
#pragma unroll
    for (int r = 0; r < R2; ++r) S[i][r] = T(0);

  for (int m = 0; m < M; ++m) {
    const int k = im * M + m;
    cx<T>* Fk = F + (size_t)k * N * N;
    cx<T> o[MB2][R2];
    if (stored) {
#pragma unroll
      for (int i = 0; i < MB2; ++i)
#pragma unroll
        for (int r = 0; r < R2; ++r) o[i][r] = Fk[(jj[i] + r * R1) * N + mm[i]];
    } else {
      const cx<T>* win = psi + (size_t)a.win[2 * k] * a.n_hi + a.win[2 * k + 1];
#pragma unroll
      for (int i0 = 0; i0 < PPT; i0 += GB) {
        cx<T> pv[GB], wv[GB];
#pragma unroll
        for (int i = 0; i < GB; ++i) {
          const int p = tid + (i0 + i) * NT;
          pv[i] = P[p];
          wv[i] = win[(size_t)(p / N) * a.n_hi + p % N];
        }
#pragma unroll
        for (int i = 0; i < GB; ++i) {
          const int p = tid + (i0 + i) * NT;
          const int y = p / N, x = p % N;
          const int4 rw = srow[y];
          img[y * PITCH + x] = (x >= rw.x && x <= rw.y) ? pv[i] * wv[i] : czero<T>();
        }
      }
      __syncthreads();
      const int nband = a.y_max - a.y_min + 1;
      P1iR::run(img, a.y_min, nband, twl, tid);
      P2iR::run(img, a.y_min, nband, twl, tid);
      P1iC::run(img, 0, N, twl, tid);
      P2iC::load(img, 0, mm, jj, lv, twl, o);
      __syncthreads();  // the next LED's gather overwrites the tile
#pragma unroll
      for (int i = 0; i < MB2; ++i)
#pragma unroll
        for (int r = 0; r < R2; ++r) {
          const int y = jj[i] + r * R1, x = mm[i];
          const cx<T> ov = scale(o[i][r], sc);
          o[i][r] = ((x + y) & 1) ? cx<T>{-ov.x, -ov.y} : ov;  // true frame
          Fk[y * N + x] = o[i][r];
        }
    }
#pragma unroll
    for (int i = 0; i < MB2; ++i)
#pragma unroll
      for (int r = 0; r < R2; ++r) S[i][r] += norm2(o[i][r]);
  }

  if (mode & LED_INTENS) {
#pragma unroll
    for (int i = 0; i < MB2; ++i)
#pragma unroll
      for (int r = 0; r < R2; ++r)
        static_cast<T*>(a.intens)[(size_t)im * N * N + (jj[i] + r * R1) * N + mm[i]] = S[i][r];
  }
  if (!(mode & (LED_GRAD | LED_LOSS))) return;

  const T eps = T(a.eps), gam = T(a.fid_gamma);
  const T* meas = static_cast<const T*>(a.meas) + (size_t)im * N * N;
  T* eb = reinterpret_cast<T*>(img);
#pragma unroll
  for (int i = 0; i < MB2; ++i)
#pragma unroll
    for (int r = 0; r < R2; ++r) {
      const int y = jj[i] + r * R1, x = mm[i];
      eb[y * PITCH + x] = fid_residual<SCALED>(a.fidelity, S[i][r], meas[y * N + x], gam);
    }
  __syncthreads();

  auto E = [&](int yy, int xx) -> T { return eb[yy * PITCH + xx]; };
  double lsum = 0.0;
#pragma unroll
  for (int i = 0; i < MB2; ++i) {
    const int j = jj[i], x = mm[i];
#pragma unroll
    for (int r = 0; r < R2; ++r) {
      const int y = j + r * R1;
      const T e = E(y, x);
      const T dx0 = (x < N - 1) ? E(y, x + 1) - e : T(0);
      const T dy0 = (y < N - 1) ? E(y + 1, x) - e : T(0);
      T q;
      if (a.norm == 0) {
        const T dxm = (x > 0) ? e - E(y, x - 1) : T(0);
        const T dym = (y > 0) ? e - E(y - 1, x) : T(0);
        q = omega(dxm, eps) - omega(dx0, eps) + omega(dym, eps) - omega(dy0, eps);
        lsum += double(rho(dx0, eps) + rho(dy0, eps));
      } else {
        const T s0 = dx0 * dx0 + dy0 * dy0;
        q = -(dx0 + dy0) * inv_norm(s0, eps);
        if (x > 0) {
          const T el = E(y, x - 1);
          const T gx = e - el;
          const T gy = (y < N - 1) ? E(y + 1, x - 1) - el : T(0);
          q += gx * inv_norm(gx * gx + gy * gy, eps);
        }
        if (y > 0) {
          const T eu = E(y - 1, x);
          const T gy = e - eu;
          const T gx = (x < N - 1) ? E(y - 1, x + 1) - eu : T(0);
          q += gy * inv_norm(gx * gx + gy * gy, eps);
        }
        lsum += eps > T(0) ? double(sqrt_t(s0 + eps * eps) - eps) : double(sqrt_t(s0));
      }
      S[i][r] = fid_slope<SCALED>(a.fidelity, S[i][r], q, gam);  // S now holds f
    }
  }
  const double tot = block_sum<NT>(lsum, red);  // contains barriers: the residual reads are done
  if (tid == 0) a.fid_partial[im] = tot;
  if (!(mode & LED_GRAD)) return;

  const int ncol = a.x_max - a.x_min + 1;
  for (int m = 0; m < M; ++m) {
    const int k = im * M + m;
    const cx<T>* Fk = F + (size_t)k * N * N;
#pragma unroll
    for (int i = 0; i < MB2; ++i)
#pragma unroll
      for (int r = 0; r < R2; ++r) {
        const int y = jj[i] + r * R1, x = mm[i];
        const cx<T> f = Fk[y * N + x];
        const cx<T> ov = ((x + y) & 1) ? cx<T>{-f.x, -f.y} : f;  // kernel frame
        img[y * PITCH + x] = scale(ov, S[i][r]);
      }
    __syncthreads();
    P1fR::run(img, 0, N, twl, tid);
    P2fR::run(img, 0, N, twl, tid);
    P1fC::run(img, a.x_min, ncol, twl, tid);
    int fm[MB2], fj[MB2];
    bool fl[MB2];
    P2fC::coords(ncol, tid, fm, fj, fl);
    cx<T> Y[MB2][R2];
    P2fC::load(img, a.x_min, fm, fj, fl, twl, Y);
    const cx<T>* win = psi + (size_t)a.win[2 * k] * a.n_hi + a.win[2 * k + 1];
    cx<T>* C = static_cast<cx<T>*>(a.C) + (size_t)k * a.S;
    cx<T>* D = static_cast<cx<T>*>(a.D) + (size_t)k * a.S;
#pragma unroll
    for (int i = 0; i < MB2; ++i) {
      if (!fl[i]) continue;
      const int x = a.x_min + fm[i];
#pragma unroll
      for (int r = 0; r < R2; ++r) {
        const int y = fj[i] + r * R1;
        const int4 rw = srow[y];
        if (x >= rw.x && x <= rw.y) {
          const int s = rw.z + x;
          const cx<T> yv = scale(Y[i][r], sc);
          C[s] = cmulc(P[y * N + x], yv);
          D[s] = cmulc(win[(size_t)y * a.n_hi + x], yv);
        }
      }
    }
    __syncthreads();  // the next LED's W overwrites the tile
  }
}

// ---------------------------------------------------------------------------
// Object-branch FFTs on the n_hi x n_hi spectrum: RPB rows (or columns) per block.
// ---------------------------------------------------------------------------
#ifndef ELFPIE_COLS512
#define ELFPIE_COLS512 8  // columns per block of the 512-point column transform
#endif
// Lines (rows, or columns when COLS) per block and radices of the object-branch transforms.
template <int N, bool COLS = false> struct BigShape;
template <bool C> struct BigShape<128, C> { static constexpr int NT = 128, RPB = 16, R1 = 16, R2 = 8, R3 = 1; };
template <bool C> struct BigShape<256, C> { static constexpr int NT = 128, RPB = 8, R1 = 16, R2 = 16, R3 = 1; };
template <> struct BigShape<512, false> { static constexpr int NT = 128, RPB = 2, R1 = 8, R2 = 8, R3 = 8; };
template <> struct BigShape<512, true> {
  static constexpr int RPB = ELFPIE_COLS512, NT = RPB * 64, R1 = 8, R2 = 8, R3 = 8;
};
template <bool C> struct BigShape<1024, C> { static constexpr int NT = 128, RPB = 2, R1 = 16, R2 = 8, R3 = 8; };
template <bool C> struct BigShape<192, C> { static constexpr int NT = 128, RPB = 8, R1 = 16, R2 = 12, R3 = 1; };
template <bool C> struct BigShape<384, C> { static constexpr int NT = 128, RPB = 2, R1 = 8, R2 = 8, R3 = 6; };
template <bool C> struct BigShape<768, C> { static constexpr int NT = 128, RPB = 2, R1 = 16, R2 = 8, R3 = 6; };

// All passes of an unnormalised DFT of the RPB lines held in buf (line m at
// m * (N + 1)); the outputs of the last pass go to emit(m, e, value).
template <class T, int N, bool INV, bool COLS, class Emit>
__device__ __forceinline__ void fft_lines_lds(cx<T>* buf, const cx<T>* twl, int tid, Emit&& emit) {
  using Sh = BigShape<N, COLS>;
  constexpr int NT = Sh::NT, RPB = Sh::RPB, R1 = Sh::R1, R2 = Sh::R2, R3 = Sh::R3, PITCH = N + 1;
  constexpr int MB1 = ceil_div(RPB * (N / R1), NT);
  constexpr int MB2 = ceil_div(RPB * (N / R2), NT);
  using PA = StockhamPass<T, N, R1, 1, INV, NT, MB1, PITCH, 1, RPB>;
  using PB = StockhamPass<T, N, R2, R1, INV, NT, MB2, PITCH, 1, RPB>;
  PA::run(buf, 0, RPB, twl, tid);
  if constexpr (R3 == 1) {
    int m[MB2], j[MB2];
    bool lv[MB2];
    PB::coords(RPB, tid, m, j, lv);
    cx<T> v[MB2][R2];
    PB::load(buf, 0, m, j, lv, twl, v);
#pragma unroll
    for (int i = 0; i < MB2; ++i)
      if (lv[i]) {
#pragma unroll
        for (int r = 0; r < R2; ++r) emit(m[i], PB::out_index(j[i], r), v[i][r]);
      }
  } else {
    constexpr int MB3 = ceil_div(RPB * (N / R3), NT);
    using PC = StockhamPass<T, N, R3, R1 * R2, INV, NT, MB3, PITCH, 1, RPB>;
    PB::run(buf, 0, RPB, twl, tid);
    int m[MB3], j[MB3];
    bool lv[MB3];
    PC::coords(RPB, tid, m, j, lv);
    cx<T> v[MB3][R3];
    PC::load(buf, 0, m, j, lv, twl, v);
#pragma unroll
    for (int i = 0; i < MB3; ++i)
      if (lv[i]) {
#pragma unroll
        for (int r = 0; r < R3; ++r) emit(m[i], PC::out_index(j[i], r), v[i][r]);
      }
  }
}

template <class T, int NT>
__device__ __forceinline__ void tail_block(const TailArgs& ta, int vb, int tid, double* sbc, double (*red)[4]);
__device__ __forceinline__ void bias_corrections(double lg1, double lg2, double t, double* bc);
template <class T>
__device__ __forceinline__ void pupil_update_body(const PupilArgs& a, const double* sbc, int p);
template <int NT>
__device__ __forceinline__ void finalize_block(const FinArgs& a, int tid, double (*red)[4]);

// Eq. 19 on one pupil pixel p, in two halves so that a caller can issue every load
// early and finish late: the gradient is the sum of the chunk partial sums in chunk
// order (zero off the support).
template <class T>
struct PupilPre {
  static constexpr int MC = 16;  // chunks held in registers; more are read at the finish
  cx<T> part[MC];
  cx<T> xv, mu;
  double v;
  T d;
  int lo, hi;
};
template <class T>
__device__ __forceinline__ void pupil_prefetch(const PupilArgs& a, int p, PupilPre<T>& f);
template <class T>
__device__ __forceinline__ void pupil_finish(const PupilArgs& a, const double* sbc, int p, PupilPre<T>& f);

// Unnormalised DFT (inverse when INV) of every row (COLS = false) or every column
// (COLS = true) of an N x N complex array; in may equal out.  Blocks past the
// N / RPB line blocks run the previous iteration's tail (pupil update, loss), which
// touches none of the arrays transformed here.  As the opening launch of a run (no
// tail then), block 0 clears the run's loss counters.
template <class T, int N, bool INV, bool COLS>
__global__ __launch_bounds__((BigShape<N, COLS>::NT)) void k_fft_lines(const cx<T>* in, cx<T>* out,
                                                                      const cx<T>* tw, TailArgs ta) {
  using Sh = BigShape<N, COLS>;
  constexpr int NT = Sh::NT, RPB = Sh::RPB, R1 = Sh::R1, R2 = Sh::R2, R3 = Sh::R3, PITCH = N + 1;
  constexpr int MB1 = ceil_div(RPB * (N / R1), NT);
  constexpr int MB2 = ceil_div(RPB * (N / R2), NT);
  constexpr int MB3 = ceil_div(RPB * (N / R3), NT);
  constexpr int EPT = RPB * N / NT;
  static_assert(EPT * NT == RPB * N, "whole elements per thread");
  __shared__ cx<T> buf[RPB * PITCH];
  __shared__ cx<T> twl[N];
  __shared__ double tail_sbc[6];
  __shared__ double tail_red[3][4];
  const int tid = threadIdx.x;
  if (blockIdx.x >= N / RPB) {
    tail_block<T, NT>(ta, blockIdx.x - N / RPB, tid, tail_sbc, tail_red);
    return;
  }
  const int l0 = blockIdx.x * RPB;
  if (blockIdx.x == 0 && tid == 0) {
    if (ta.zero_ctr) *ta.zero_ctr = 0;
    if (ta.zero_flag) *ta.zero_flag = 0;
  }
  for (int i = tid; i < N; i += NT) twl[i] = tw[i];
  cx<T> ld[EPT];
#pragma unroll
  for (int i = 0; i < EPT; ++i) {
    const int p = tid + i * NT;
    if (COLS) ld[i] = in[(size_t)(p / RPB) * N + l0 + p % RPB];
    else ld[i] = in[(size_t)(l0 + p / N) * N + p % N];
  }
#pragma unroll
  for (int i = 0; i < EPT; ++i) {
    const int p = tid + i * NT;
    if (COLS) buf[(p % RPB) * PITCH + p / RPB] = ld[i];
    else buf[(p / N) * PITCH + p % N] = ld[i];
  }
  __syncthreads();
  fft_lines_lds<T, N, INV, COLS>(buf, twl, tid, [&](int m, int e, cx<T> v) {
    if (COLS) out[(size_t)e * N + l0 + m] = v;
    else out[(size_t)(l0 + m) * N + e] = v;
  });
}

// All passes of an unnormalised DFT of NL lines of length N held in LDS (line m at
// buf[m * (N + 1) + e]), NT threads, results left in place.
template <int N> struct LineRadix;
template <> struct LineRadix<128> { static constexpr int R1 = 16, R2 = 8, R3 = 1; };
template <> struct LineRadix<256> { static constexpr int R1 = 16, R2 = 16, R3 = 1; };
template <> struct LineRadix<512> { static constexpr int R1 = 8, R2 = 8, R3 = 8; };
template <> struct LineRadix<1024> { static constexpr int R1 = 16, R2 = 8, R3 = 8; };
template <> struct LineRadix<192> { static constexpr int R1 = 16, R2 = 12, R3 = 1; };
template <> struct LineRadix<384> { static constexpr int R1 = 8, R2 = 8, R3 = 6; };
template <> struct LineRadix<768> { static constexpr int R1 = 16, R2 = 8, R3 = 6; };

template <class T, int N, bool INV, int NT, int NL, int PITCH = N + 1>
__device__ __forceinline__ void fft_lines_inplace(cx<T>* buf, const cx<T>* twl, int tid) {
  using Rd = LineRadix<N>;
  constexpr int R1 = Rd::R1, R2 = Rd::R2, R3 = Rd::R3;
  StockhamPass<T, N, R1, 1, INV, NT, ceil_div(NL * (N / R1), NT), PITCH, 1, NL>::run(buf, 0, NL, twl, tid);
  StockhamPass<T, N, R2, R1, INV, NT, ceil_div(NL * (N / R2), NT), PITCH, 1, NL>::run(buf, 0, NL, twl, tid);
  if constexpr (R3 > 1)
    StockhamPass<T, N, R3, R1 * R2, INV, NT, ceil_div(NL * (N / R3), NT), PITCH, 1, NL>::run(buf, 0, NL, twl, tid);
}

// ---------------------------------------------------------------------------
// Object branch on column strips: column inverse DFT, Hessian penalties and their
// gradient (Eq. 6, 7, 13, 14), column forward DFT, for W output columns per block.
// ---------------------------------------------------------------------------
// Input T1 = row-transformed Psi (unnormalised inverse DFT along rows).  The block
// loads the W + 4 columns c0 - 2 .. c0 + W + 1 (the stencils reach two pixels),
// finishes the inverse transform along them, so O = (-1)^(x+y) Ot / n, keeps |O| and
// angle(O), and then, in chunks of CH rows:
//   omega of the three H components of |O| and of angle(O) on columns c0 - 1 .. c0 + W
//   (H zero where its stencil leaves the grid), then on the W own columns
//   q = H^T omega, the loss terms and G = alpha q_a O / (2|O|) + beta q_phi i O / (2(|O|^2 + eta)),
//   stored as (-1)^(x+y) G / n over O.
// Finally the forward DFT along the W own columns, written to T2 (rows still to go).
// The previous iteration's pupil update can ride along, a slice of pixels per block
// (every block has room for it; extra blocks would wait for a free compute unit).
#ifndef ELFPIE_STRIP_W
#define ELFPIE_STRIP_W 2      // output columns per block
#define ELFPIE_STRIP_NT 1024  // threads per block
#define ELFPIE_STRIP_CH 512   // rows per Hessian chunk
#endif
#ifndef ELFPIE_STRIP_NT_SMALL
#define ELFPIE_STRIP_NT_SMALL 512  // threads per block for n_hi <= 256: 6 lines of at most 256 points
#endif
template <int N> struct StripShape {
  // rows per chunk: the configured size when it divides N, else half of N (768 -> 384)
  static constexpr int W = ELFPIE_STRIP_W, NT = N <= 256 ? ELFPIE_STRIP_NT_SMALL : ELFPIE_STRIP_NT,
                       CH = ELFPIE_STRIP_CH >= N ? N : (N % ELFPIE_STRIP_CH == 0 ? ELFPIE_STRIP_CH : N / 2);
  static_assert(N % CH == 0, "whole chunks");
};
#ifndef ELFPIE_STRIP_PAD
#define ELFPIE_STRIP_PAD 1
#endif
// Line pitch (elements) of the strip's LDS lines.  Lanes of a pass walk the lines fastest
// (line m, butterfly j = b / NL), so with a pitch of N + 1 lines m and m + 1 start one
// element apart and the few lines of a strip share banks with the butterflies next to
// them; these pitches (an exhaustive search of the bank load of every pass, 64 banks of
// 4 bytes) spread them over the banks.
constexpr int strip_pitch(int n, int elem_bytes) {
  if (!ELFPIE_STRIP_PAD) return n + 1;
  if (elem_bytes == 8)
    return n == 128 ? 137 : n == 256 ? 261 : n == 384 ? 395 : n == 512 ? 523 : n == 768 ? 795 : n == 1024 ? 1051 : n + 1;
  return n == 128 ? 131 : n == 256 ? 259 : n + 1;
}

template <class T, int N>
__global__ __launch_bounds__(StripShape<N>::NT) void k_obj_strip(HessArgs a, const cx<T>* T1, cx<T>* T2,
                                                                  const cx<T>* tw, TailArgs ta) {
  using Sh = StripShape<N>;
  constexpr int W = Sh::W, NT = Sh::NT, CH = Sh::CH, NL = W + 4, OW = W + 2, OH = CH + 2;
  constexpr int PITCH = strip_pitch(N, sizeof(cx<T>));
  __shared__ cx<T> buf[NL * PITCH];     // line l = column c0 - 2 + l
  __shared__ T sa[NL * N], sp[NL * N];  // |O| and angle(O), line-major
  __shared__ T om[6][OW * OH];          // omega: 3 components of |O|, then of angle(O)
  __shared__ cx<T> twl[N];
  __shared__ double red[NT / 64][2];
  const int tid = threadIdx.x;
  // the previous iteration's pupil update, a slice of pixels per block: loads issued
  // here, the update at the end, so that their latency hides behind the strip's work
  const int pp = blockIdx.x * ta.pupil_ppb + tid;
  const bool pslice = tid < ta.pupil_ppb && pp < ta.pa.n_lo * ta.pa.n_lo;
  constexpr bool early = sizeof(T) == 4;  // FP64 has no registers to spare across the strip
  PupilPre<T> pf;
  if (early && pslice) pupil_prefetch<T>(ta.pa, pp, pf);
  __shared__ double pbc[6];
  if (tid == 0 && ta.pupil_ppb && ta.pa.step) bias_corrections(ta.pa.lg1, ta.pa.lg2, double(*ta.pa.t), pbc);
  // runs of neighbouring strips per XCD: their column segments share cache lines
  const int sidx = ELFPIE_STRIP_XCD ? xcd_order(blockIdx.x, N / W) : (int)blockIdx.x;
  const int c0 = sidx * W;
  const T inv_n = T(a.inv_n), eps = T(a.eps);
  for (int i = tid; i < N; i += NT) twl[i] = tw[i];
  {
    constexpr int EPT = ceil_div(NL * N, NT);
    cx<T> ld[EPT];
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
      const int p = tid + i * NT, l = p % NL, y = p / NL, c = c0 - 2 + l;
      ld[i] = (p < NL * N && c >= 0 && c < N) ? T1[(size_t)y * N + c] : czero<T>();
    }
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
      const int p = tid + i * NT;
      if (p < NL * N) buf[(p % NL) * PITCH + p / NL] = ld[i];
    }
  }
  __syncthreads();
  fft_lines_inplace<T, N, true, NT, NL, PITCH>(buf, twl, tid);
  for (int p = tid; p < NL * N; p += NT) {
    const int l = p / N, y = p % N, c = c0 - 2 + l;
    const cx<T> O = scale(buf[l * PITCH + y], ((c + y) & 1) ? -inv_n : inv_n);
    sa[p] = sqrt_t(norm2(O));
    sp[p] = atan2(O.y, O.x);
  }
  __syncthreads();
  double la = 0.0, lp = 0.0;
  for (int r0 = 0; r0 < N; r0 += CH) {
    // omega on lines 1 .. W + 2 (columns c0 - 1 .. c0 + W), rows r0 - 1 .. r0 + CH.  The
    // exact anisotropic L1 (the default) takes a copy of the loop with omega = sign and
    // rho = |.| and no branch per position: the same arithmetic, selects for the rest.
    auto omega_pass = [&](auto fast_c) {
    constexpr bool FAST = decltype(fast_c)::value;
    T ta_ = T(0), tp_ = T(0);
    for (int p = tid; p < OW * OH; p += NT) {
      const int li = p / OH, yi = p % OH;
      const int l = li + 1, y = r0 - 1 + yi, c = c0 - 2 + l;
      const bool in = y >= 0 && y < N && c >= 0 && c < N;
      const bool vxx = in && c >= 1 && c <= N - 2, vyy = in && y >= 1 && y <= N - 2;
      const bool vxy = in && c <= N - 2 && y <= N - 2;
      // rows clamped into the grid: exact for valid positions, harmless for the others
      const int y0c = min(max(y, 0), N - 1), ymc = min(max(y - 1, 0), N - 1), ypc = min(max(y + 1, 0), N - 1);
      const bool own = l >= 2 && l <= W + 1 && yi >= 1 && yi <= CH && in;
#pragma unroll
      for (int f = 0; f < 2; ++f) {
        const T* src = f == 0 ? sa : sp;
        const T ctr = src[l * N + y0c];
        if constexpr (FAST) {
          const T sl = src[(l - 1) * N + y0c], sr = src[(l + 1) * N + y0c];
          const T su = src[l * N + ymc], sd = src[l * N + ypc], srd = src[(l + 1) * N + ypc];
          const T hxx = vxx ? sl - T(2) * ctr + sr : T(0);
          const T hyy = vyy ? su - T(2) * ctr + sd : T(0);
          const T hxy = vxy ? ctr - sr - sd + srd : T(0);
          auto sgn = [](T d) { return sign_unit(d); };
          om[3 * f + 0][p] = sgn(hxx);
          om[3 * f + 1][p] = sgn(hyy);
          om[3 * f + 2][p] = sgn(hxy);
          if (ELFPIE_STRIP_TSUM) {  // this lane's positions summed in T, added to FP64 per pass
            const T lv = fabs(hxx) + fabs(hyy) + fabs(hxy);
            if (f == 0) ta_ += own ? lv : T(0);
            else tp_ += own ? lv : T(0);
          } else {
            const double lv = double(fabs(hxx)) + double(fabs(hyy)) + double(fabs(hxy));
            if (f == 0) la += own ? lv : 0.0;
            else lp += own ? lv : 0.0;
          }
          continue;
        }
        const T hxx = vxx ? src[(l - 1) * N + y0c] - T(2) * ctr + src[(l + 1) * N + y0c] : T(0);
        const T hyy = vyy ? src[l * N + ymc] - T(2) * ctr + src[l * N + ypc] : T(0);
        const T hxy = vxy ? ctr - src[(l + 1) * N + y0c] - src[l * N + ypc] + src[(l + 1) * N + ypc] : T(0);
        T wxx, wyy, wxy;
        if (a.norm == 0) {
          wxx = omega(hxx, eps);
          wyy = omega(hyy, eps);
          wxy = omega(hxy, eps);
        } else {
          const T inv = inv_norm(hxx * hxx + hyy * hyy + hxy * hxy, eps);
          wxx = hxx * inv;
          wyy = hyy * inv;
          wxy = hxy * inv;
        }
        om[3 * f + 0][p] = wxx;
        om[3 * f + 1][p] = wyy;
        om[3 * f + 2][p] = wxy;
        // loss: own pixels (lines 2 .. W + 1, rows r0 .. r0 + CH - 1), each counted once
        if (own) {
          double lv;
          if (a.norm == 0) {
            lv = double(rho(hxx, eps)) + double(rho(hyy, eps)) + double(rho(hxy, eps));
          } else {
            const T s2 = hxx * hxx + hyy * hyy + hxy * hxy;
            lv = eps > T(0) ? double(sqrt_t(s2 + eps * eps) - eps) : double(sqrt_t(s2));
          }
          if (f == 0) la += lv;
          else lp += lv;
        }
      }
    }
    la += double(ta_);
    lp += double(tp_);
    };
    if (a.norm == 0 && !(eps > T(0))) omega_pass(std::true_type{});
    else omega_pass(std::false_type{});
    __syncthreads();
    if (a.want_grad) {
      for (int p = tid; p < W * CH; p += NT) {
        const int li = p / CH, yi = p % CH;
        const int l = li + 2, y = r0 + yi, c = c0 - 2 + l;
        const int oi = (li + 1) * OH + (yi + 1);  // omega index of the own pixel
        T q[2];
#pragma unroll
        for (int f = 0; f < 2; ++f) {
          const T* wx = om[3 * f + 0];
          const T* wy = om[3 * f + 1];
          const T* wz = om[3 * f + 2];
          q[f] = wx[oi - OH] - T(2) * wx[oi] + wx[oi + OH] + wy[oi - 1] - T(2) * wy[oi] + wy[oi + 1] + wz[oi] -
                 wz[oi - OH] - wz[oi - 1] + wz[oi - OH - 1];
        }
        const T sgn = ((c + y) & 1) ? -inv_n : inv_n;
        const cx<T> O = scale(buf[l * PITCH + y], sgn);
        const T a2 = norm2(O);
        cx<T> G = czero<T>();
        if (a2 > T(0)) G = scale(O, T(0.5) * T(a.alpha) * q[0] * rsqrt_t(a2));
        const T den = a2 + T(a.eta_h);
        if (den > T(0)) G = G + scale(mul_i(O), T(0.5) * T(a.beta) * q[1] * rcp_t(den));
        buf[l * PITCH + y] = scale(G, sgn);
      }
    }
    __syncthreads();
  }
  // deterministic block sums of the two penalty partials
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    la += __shfl_down(la, off, 64);
    lp += __shfl_down(lp, off, 64);
  }
  if ((tid & 63) == 0) {
    red[tid >> 6][0] = la;
    red[tid >> 6][1] = lp;
  }
  __syncthreads();
  if (tid == 0) {
    double s0 = 0.0, s1 = 0.0;
    for (int w = 0; w < NT / 64; ++w) {
      s0 += red[w][0];
      s1 += red[w][1];
    }
    a.partial[2 * sidx + 0] = s0;
    a.partial[2 * sidx + 1] = s1;
  }
  if (a.want_grad) {
    // forward DFT along the own columns (lines 2 .. W + 1), then store
    fft_lines_inplace<T, N, false, NT, W, PITCH>(buf + 2 * PITCH, twl, tid);
    constexpr int EPT = ceil_div(W * N, NT);
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
      const int p = tid + i * NT, l = p % W, y = p / W;
      if (p < W * N) T2[(size_t)y * N + c0 + l] = buf[(l + 2) * PITCH + y];
    }
  }
  if (pslice) {
    if (!early) pupil_prefetch<T>(ta.pa, pp, pf);
    pupil_finish<T>(ta.pa, pbc, pp, pf);  // pbc: written before the first barrier
  }
}

// ---------------------------------------------------------------------------
// The object branch as blocks of the per-LED launch: k_obj_strip's work on a wide strip
// of W <= WMAX output columns per block, so that a few blocks on the compute units the
// LED blocks leave free cover the whole spectrum while those run.
// ---------------------------------------------------------------------------
// Object block b of nblk takes columns c0 = b N / nblk .. c1 - 1 (W = c1 - c0) and the two
// halo columns on each side (NL = W + 4 lines), all in LDS: the column inverse DFT gives
// O = (-1)^(x+y) Ot / n on the lines; then, in chunks of CH rows, |O| and angle(O) of the
// chunk's rows and two halo rows each side (the two rows above carried over from the
// previous chunk, whose own rows have been overwritten by G), omega of the three H
// components on columns c0 - 1 .. c1 and rows r0 - 1 .. r0 + CH (zero where the stencil
// leaves the grid), the loss terms of the own pixels, and on the own pixels
// q = H^T omega and G = alpha q_a O / (2|O|) + beta q_phi i O / (2(|O|^2 + eta)), stored as
// (-1)^(x+y) G / n over O.  Finally the forward DFT along the W own columns into T2.
// The exact anisotropic L1 (omega = sign, the default) keeps omega as bytes, which leaves
// room for chunks of 128 rows; the other forms keep it in the working precision, in
// chunks of 64.  The arithmetic per element is that of k_obj_strip.
template <int N, bool SIGN> struct ObjWide {
  static constexpr int WMAX = 17, CH = 64, NLM = WMAX + 4, OWM = WMAX + 2, OH = CH + 2, RS = CH + 4;
  static constexpr int PITCH = N + 1;  // odd: the lines of a pass spread over the banks
  static_assert(N % CH == 0, "whole chunks");
};

// Shared-memory bytes of one form of obj_strip_wide: lines, twiddles, then the chunk
// arrays -- the sign form: (|O|, angle(O)) pairs and three planes of packed sign pairs,
// reused for the per-thread loss partials; the other forms: |O| and angle(O) planes, six
// omega planes in the working precision, block sums.
template <class T, int N, int NT, bool SIGN>
constexpr size_t obj_wide_form_bytes() {
  using Sh = ObjWide<N, SIGN>;
  constexpr size_t lines = sizeof(cx<T>) * (Sh::NLM * Sh::PITCH + N);
  if constexpr (SIGN) {
    constexpr size_t chunk = 2 * (2 * sizeof(T) * Sh::NLM * Sh::RS + 3 * sizeof(unsigned) * Sh::OWM * Sh::OH);
    constexpr size_t sums = sizeof(double) * (4 * NT);
    return lines + sizeof(cx<T>) + (chunk > sums ? chunk : sums);  // + the 16-byte alignment
  }
  return lines + sizeof(T) * 2 * Sh::NLM * Sh::RS + sizeof(T) * 6 * Sh::OWM * Sh::OH + 8 +
         sizeof(double) * 2 * (NT / 64);
}
template <class T, int N, int NT>
constexpr size_t obj_wide_lds_bytes() {
  return obj_wide_form_bytes<T, N, NT, true>() > obj_wide_form_bytes<T, N, NT, false>()
             ? obj_wide_form_bytes<T, N, NT, true>()
             : obj_wide_form_bytes<T, N, NT, false>();
}

template <class T, int N, int NT, bool SIGN>
__device__ void obj_strip_wide_form(const LedObjArgs& o, int b, char* lds) {
  using Sh = ObjWide<N, SIGN>;
  using OmT = typename std::conditional<SIGN, signed char, T>::type;  // omega storage
  constexpr int CH = Sh::CH, NLM = Sh::NLM, OWM = Sh::OWM, OH = Sh::OH, RS = Sh::RS, PITCH = Sh::PITCH;
  constexpr int PL = OWM * OH;  // one omega plane
  cx<T>* buf = reinterpret_cast<cx<T>*>(lds);  // line l = column c0 - 2 + l
  cx<T>* twl = buf + NLM * PITCH;
  T* sa = reinterpret_cast<T*>(twl + N);  // chunk rows i = y - r0 + 2, line-major
  T* sp = sa + NLM * RS;
  OmT* om = reinterpret_cast<OmT*>(sp + NLM * RS);  // 3 components of |O|, then of angle(O)
  double* red = reinterpret_cast<double*>(lds + ((reinterpret_cast<char*>(om + 6 * PL) - lds + 7) & ~size_t(7)));
  const int tid = threadIdx.x;
  const int c0 = b * N / o.nblk, c1 = (b + 1) * N / o.nblk, W = c1 - c0, NL = W + 4, OW = W + 2;
  const Div dNL = make_div(NL), dW = make_div(W);
  const T inv_n = T(o.inv_n), eps = T(o.eps);
  const cx<T>* T1 = static_cast<const cx<T>*>(o.T1);
  cx<T>* T2 = static_cast<cx<T>*>(o.T2);
  const cx<T>* tw = static_cast<const cx<T>*>(o.tw);
  for (int i = tid; i < N; i += NT) twl[i] = tw[i];
  using Rd = LineRadix<N>;
  constexpr int R1 = Rd::R1, R2 = Rd::R2, R3 = Rd::R3;
  static_assert(R3 > 1, "three passes");
  {
    // inverse DFT along the NL lines; the first pass (no twiddles) reads its butterflies
    // straight from T1: line m = column c0 - 2 + m, element j + r N / R1
    using PA = StockhamPass<T, N, R1, 1, true, NT, ceil_div(NLM * (N / R1), NT), PITCH, 1>;
    constexpr int MB = ceil_div(NLM * (N / R1), NT);
    int m[MB], j[MB];
    bool lv[MB];
    PA::coords(dNL, tid, m, j, lv);
    cx<T> v[MB][R1];
#pragma unroll
    for (int i = 0; i < MB; ++i) {
      const int c = c0 - 2 + m[i];
      const bool ok = lv[i] && c >= 0 && c < N;
#pragma unroll
      for (int r = 0; r < R1; ++r) v[i][r] = ok ? T1[(size_t)(j[i] + r * (N / R1)) * N + c] : czero<T>();
    }
#pragma unroll
    for (int i = 0; i < MB; ++i)
      if (lv[i]) dft<T, R1, true>(v[i]);
    PA::store(buf, 0, m, j, lv, v);
    __syncthreads();
    StockhamPass<T, N, R2, R1, true, NT, ceil_div(NLM * (N / R2), NT), PITCH, 1>::run(buf, 0, dNL, twl, tid);
    StockhamPass<T, N, R3, R1 * R2, true, NT, ceil_div(NLM * (N / R3), NT), PITCH, 1>::run(buf, 0, dNL, twl, tid);
  }
  double la = 0.0, lp = 0.0;
  for (int r0 = 0; r0 < N; r0 += CH) {
    // |O| and angle(O) on chunk rows i0 .. RS - 1 (rows 0, 1 carried over after the first)
    const int i0 = r0 == 0 ? 0 : 2, nr = RS - i0;
    const Div dnr = make_div(nr);
    for (int p = tid; p < NL * nr; p += NT) {
      const int l = div_q(p, dnr), i = i0 + p - l * nr, y = r0 - 2 + i, c = c0 - 2 + l;
      T am = T(0), ph = T(0);
      if (y >= 0 && y < N) {
        const cx<T> O = scale(buf[l * PITCH + y], ((c + y) & 1) ? -inv_n : inv_n);
        am = sqrt_t(norm2(O));
        ph = atan2(O.y, O.x);
      }
      sa[l * RS + i] = am;
      sp[l * RS + i] = ph;
    }
    __syncthreads();
    // omega on lines 1 .. W + 2 (columns c0 - 1 .. c1), rows r0 - 1 .. r0 + CH
    T ta_ = T(0), tp_ = T(0);
    for (int p = tid; p < OW * OH; p += NT) {
      const int li = p / OH, yi = p % OH;
      const int l = li + 1, y = r0 - 1 + yi, c = c0 - 2 + l, i = yi + 1;
      const bool in = y >= 0 && y < N && c >= 0 && c < N;
      const bool vxx = in && c >= 1 && c <= N - 2, vyy = in && y >= 1 && y <= N - 2;
      const bool vxy = in && c <= N - 2 && y <= N - 2;
      const bool own = l >= 2 && l <= W + 1 && yi >= 1 && yi <= CH && in;
#pragma unroll
      for (int f = 0; f < 2; ++f) {
        const T* src = f == 0 ? sa : sp;
        const T ctr = src[l * RS + i];
        const T sl = src[(l - 1) * RS + i], sr = src[(l + 1) * RS + i];
        const T su = src[l * RS + i - 1], sd = src[l * RS + i + 1], srd = src[(l + 1) * RS + i + 1];
        const T hxx = vxx ? sl - T(2) * ctr + sr : T(0);
        const T hyy = vyy ? su - T(2) * ctr + sd : T(0);
        const T hxy = vxy ? ctr - sr - sd + srd : T(0);
        OmT* omf = om + 3 * f * PL + li * OH + yi;
        if constexpr (SIGN) {  // omega = sign, rho = |.|, summed per lane in T
          omf[0] = (signed char)sign_unit(hxx);
          omf[PL] = (signed char)sign_unit(hyy);
          omf[2 * PL] = (signed char)sign_unit(hxy);
          const T lv = fabs(hxx) + fabs(hyy) + fabs(hxy);
          if (f == 0) ta_ += own ? lv : T(0);
          else tp_ += own ? lv : T(0);
        } else {
          T wxx, wyy, wxy;
          if (o.norm == 0) {
            wxx = omega(hxx, eps);
            wyy = omega(hyy, eps);
            wxy = omega(hxy, eps);
          } else {
            const T inv = inv_norm(hxx * hxx + hyy * hyy + hxy * hxy, eps);
            wxx = hxx * inv;
            wyy = hyy * inv;
            wxy = hxy * inv;
          }
          omf[0] = wxx;
          omf[PL] = wyy;
          omf[2 * PL] = wxy;
          if (own) {
            double lv;
            if (o.norm == 0) {
              lv = double(rho(hxx, eps)) + double(rho(hyy, eps)) + double(rho(hxy, eps));
            } else {
              const T s2 = hxx * hxx + hyy * hyy + hxy * hxy;
              lv = eps > T(0) ? double(sqrt_t(s2 + eps * eps) - eps) : double(sqrt_t(s2));
            }
            if (f == 0) la += lv;
            else lp += lv;
          }
        }
      }
    }
    la += double(ta_);
    lp += double(tp_);
    __syncthreads();
    for (int p = tid; p < W * CH; p += NT) {
      const int li = p / CH, yi = p % CH;
      const int l = li + 2, y = r0 + yi, c = c0 + li;
      const int oi = (li + 1) * OH + (yi + 1);  // omega index of the own pixel
      T q[2];
#pragma unroll
      for (int f = 0; f < 2; ++f) {
        const OmT* wx = om + 3 * f * PL;
        const OmT* wy = wx + PL;
        const OmT* wz = wy + PL;
        if constexpr (SIGN) {  // sums of signs: exact in integers, as in T
          q[f] = T(int(wx[oi - OH]) - 2 * int(wx[oi]) + int(wx[oi + OH]) + int(wy[oi - 1]) - 2 * int(wy[oi]) +
                   int(wy[oi + 1]) + int(wz[oi]) - int(wz[oi - OH]) - int(wz[oi - 1]) + int(wz[oi - OH - 1]));
        } else {
          q[f] = wx[oi - OH] - T(2) * wx[oi] + wx[oi + OH] + wy[oi - 1] - T(2) * wy[oi] + wy[oi + 1] + wz[oi] -
                 wz[oi - OH] - wz[oi - 1] + wz[oi - OH - 1];
        }
      }
      const T sgn = ((c + y) & 1) ? -inv_n : inv_n;
      const cx<T> O = scale(buf[l * PITCH + y], sgn);
      const T a2 = norm2(O);
      cx<T> G = czero<T>();
      if (a2 > T(0)) G = scale(O, T(0.5) * T(o.alpha) * q[0] * rsqrt_t(a2));
      const T den = a2 + T(o.eta_h);
      if (den > T(0)) G = G + scale(mul_i(O), T(0.5) * T(o.beta) * q[1] * rcp_t(den));
      buf[l * PITCH + y] = scale(G, sgn);
    }
    // the next chunk's two rows above (this chunk's last two) are kept: their own pixels
    // now hold G in buf
    for (int p = tid; p < 2 * NL; p += NT) {
      const int l = p >> 1, i = p & 1;
      sa[l * RS + i] = sa[l * RS + CH + i];
      sp[l * RS + i] = sp[l * RS + CH + i];
    }
    __syncthreads();
  }
  // deterministic block sums of the two penalty partials
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    la += __shfl_down(la, off, 64);
    lp += __shfl_down(lp, off, 64);
  }
  if ((tid & 63) == 0) {
    red[2 * (tid >> 6) + 0] = la;
    red[2 * (tid >> 6) + 1] = lp;
  }
  __syncthreads();
  if (tid == 0) {
    double s0 = 0.0, s1 = 0.0;
    for (int w = 0; w < NT / 64; ++w) {
      s0 += red[2 * w];
      s1 += red[2 * w + 1];
    }
    o.partial[2 * b + 0] = s0;
    o.partial[2 * b + 1] = s1;
  }
  // forward DFT along the own columns (lines 2 .. W + 1); the last pass stores its outputs
  // straight to T2 (line m = column c0 + m)
  {
    cx<T>* own = buf + 2 * PITCH;
    constexpr int WM = Sh::WMAX;
    StockhamPass<T, N, R1, 1, false, NT, ceil_div(WM * (N / R1), NT), PITCH, 1>::run(own, 0, dW, twl, tid);
    StockhamPass<T, N, R2, R1, false, NT, ceil_div(WM * (N / R2), NT), PITCH, 1>::run(own, 0, dW, twl, tid);
    using PC = StockhamPass<T, N, R3, R1 * R2, false, NT, ceil_div(WM * (N / R3), NT), PITCH, 1>;
    constexpr int MB = ceil_div(WM * (N / R3), NT);
    int m[MB], j[MB];
    bool lv[MB];
    PC::coords(dW, tid, m, j, lv);
    cx<T> v[MB][R3];
    PC::load(own, 0, m, j, lv, twl, v);
#pragma unroll
    for (int i = 0; i < MB; ++i)
      if (lv[i]) {
#pragma unroll
        for (int r = 0; r < R3; ++r) T2[(size_t)PC::out_index(j[i], r) * N + c0 + m[i]] = v[i][r];
      }
  }
}

// atan2(y, x) in FP32 without a library call: the octant symmetries reduce the
// argument to a = min(|x|, |y|) / max(|x|, |y|) in [0, 1], where atan(a) = a P(a^2) with a
// degree-8 polynomial P fitted here to the relative error of atan on [0, 1] (1.7e-8); then
// pi/2 - r where |y| > |x|, pi - r where x < 0, and the sign of y (atan2(+-0, x < 0) =
// +-pi).  Within 5 units of roundoff of the correctly rounded value (|error| <= 3.6e-7)
// for finite arguments; 0 at the origin.
__device__ __forceinline__ float atan2_fast(float y, float x) {
  const float ax = fabsf(x), ay = fabsf(y);
  const float mx = fmaxf(ax, ay), mn = fminf(ax, ay);
  const float a = mx > 0.0f ? mn * __builtin_amdgcn_rcpf(mx) : 0.0f;
  const float s = a * a;
  float p = 0.0029075394850224257f;
  p = __builtin_fmaf(p, s, -0.016316886991262436f);
  p = __builtin_fmaf(p, s, 0.04313173145055771f);
  p = __builtin_fmaf(p, s, -0.07545701414346695f);
  p = __builtin_fmaf(p, s, 0.10663097351789474f);
  p = __builtin_fmaf(p, s, -0.14210361242294312f);
  p = __builtin_fmaf(p, s, 0.19993694126605988f);
  p = __builtin_fmaf(p, s, -0.33333149552345276f);
  float r = __builtin_fmaf(a, p * s, a);
  r = ay > ax ? 1.57079632679489662f - r : r;
  r = x < 0.0f ? 3.14159265358979324f - r : r;
  return __builtin_copysignf(r, y);
}

// The sign form (the exact anisotropic L1, omega = sign, rho = |.|) of an object block in
// FP32: the same method as obj_strip_wide_form, laid out for fewer instructions.  After the
// column inverse DFT, each chunk of CH rows goes through three steps, each thread on a short
// run of rows of one line, so that neighbours along a line are shared in registers:
//   A  (|O|, angle(O)) of every line on the chunk's rows and two halo rows each side (rows
//      off the grid are zero), as pairs;
//   B  the three H components of both fields on lines 1 .. W + 2 and rows r0 - 1 .. r0 + CH
//      (zero where the stencil leaves the grid), their signs packed as half pairs
//      (|O| in the low half, angle(O) in the high half) in one plane per component, and
//      the loss terms of the own pixels;
//   C  on the own pixels q = H^T omega for both fields at once in half arithmetic (sums
//      of at most ten signs, exact), and G as in obj_strip_wide_form, written over O.
// The steps of consecutive chunks overlap (A of one chunk, B of the one before, C of the
// one before that, between two barriers), on two alternating sets of chunk arrays.  The
// per-thread loss partials are reduced in a fixed order after the forward DFT.
template <class T, int N, int NT>
__device__ void obj_strip_wide_sign(const LedObjArgs& o, int b, char* lds) {
  static_assert(sizeof(T) == 4, "packed half signs of FP32 features");
  using Sh = ObjWide<N, true>;
  typedef _Float16 h2 __attribute__((ext_vector_type(2)));
  constexpr int CH = Sh::CH, NLM = Sh::NLM, OWM = Sh::OWM, OH = Sh::OH, RS = Sh::RS, PITCH = Sh::PITCH;
  static_assert(OH % 2 == 0 && CH % 2 == 0, "runs of two rows");
  cx<T>* buf = reinterpret_cast<cx<T>*>(lds);  // line l = column c0 - 2 + l
  cx<T>* twl = buf + NLM * PITCH;
  // two sets of chunk arrays (chunks alternate between them): (|O|, angle(O)) at
  // [l * RS + i] for y = r0 - 2 + i, and the three packed sign planes at [lb * OH + ib]
  // for line lb + 1, y = r0 - 1 + ib
  // the chunk arrays start 16-byte aligned (the B step reads pairs of rows as 16 bytes)
  static_assert(sizeof(cx<T>) == 8 && RS % 2 == 0, "16-byte pairs of rows");
  cx<T>* sf0 = twl + N + ((NLM * PITCH + N) & 1);
  unsigned* om0 = reinterpret_cast<unsigned*>(sf0 + 2 * NLM * RS);
  auto sfb = [&](int c) { return sf0 + (c & 1) * (NLM * RS); };
  auto omb = [&](int c) { return om0 + (c & 1) * (3 * OWM * OH); };
  double* lsum = reinterpret_cast<double*>(sf0);  // after the chunks: 2 NT loss partials
  const int tid = threadIdx.x;
  const int c0 = b * N / o.nblk, c1 = (b + 1) * N / o.nblk, W = c1 - c0, NL = W + 4, LB = W + 2;
  const Div dNL = make_div(NL), dW = make_div(W);
  const T inv_n = T(o.inv_n);
  const cx<T>* T1 = static_cast<const cx<T>*>(o.T1);
  cx<T>* T2 = static_cast<cx<T>*>(o.T2);
  const cx<T>* tw = static_cast<const cx<T>*>(o.tw);
  for (int i = tid; i < N; i += NT) twl[i] = tw[i];
  using Rd = LineRadix<N>;
  constexpr int R1 = Rd::R1, R2 = Rd::R2, R3 = Rd::R3;
  static_assert(R3 > 1, "three passes");
  {
    // inverse DFT along the NL lines; the first pass (no twiddles) reads its butterflies
    // straight from T1: line m = column c0 - 2 + m, element j + r N / R1
    using PA = StockhamPass<T, N, R1, 1, true, NT, ceil_div(NLM * (N / R1), NT), PITCH, 1>;
    constexpr int MB = ceil_div(NLM * (N / R1), NT);
    int m[MB], j[MB];
    bool lv[MB];
    PA::coords(dNL, tid, m, j, lv);
    cx<T> v[MB][R1];
#pragma unroll
    for (int i = 0; i < MB; ++i) {
      const int c = c0 - 2 + m[i];
      const bool ok = lv[i] && c >= 0 && c < N;
#pragma unroll
      for (int r = 0; r < R1; ++r) v[i][r] = ok ? T1[(size_t)(j[i] + r * (N / R1)) * N + c] : czero<T>();
    }
#pragma unroll
    for (int i = 0; i < MB; ++i)
      if (lv[i]) dft<T, R1, true>(v[i]);
    PA::store(buf, 0, m, j, lv, v);
    __syncthreads();
    StockhamPass<T, N, R2, R1, true, NT, ceil_div(NLM * (N / R2), NT), PITCH, 1>::run(buf, 0, dNL, twl, tid);
    StockhamPass<T, N, R3, R1 * R2, true, NT, ceil_div(NLM * (N / R3), NT), PITCH, 1>::run(buf, 0, dNL, twl, tid);
  }
  // (|O|, angle(O)) of Ot at column c, row y; O = (-1)^(x+y) Ot / n, so |O| = |Ot| / n and
  // angle(O) = atan2 of Ot negated where x + y is odd (a positive scale leaves atan2's ratio
  // alone; 1 / n is a power of two, so the scaled parts are exact anyway)
  static_assert((N & (N - 1)) == 0, "1 / n a power of two");
  auto amp_phase = [&](cx<T> Ot, int c, int y) -> cx<T> {
    const bool neg = (c + y) & 1;
    return cx<T>{inv_n * sqrt_t(norm2(Ot)), atan2_fast(neg ? -Ot.y : Ot.y, neg ? -Ot.x : Ot.x)};
  };
  T ta = T(0), tp = T(0);  // this thread's loss terms of the current chunk
  double la = 0.0, lp = 0.0;
  const int cx0 = c0 - 1;   // column of omega line lb = 0
  constexpr int NCH = N / CH;
  // A(c), item q: (|O|, angle(O)) of line l = q / (RS / 2), chunk rows i = q mod RS / 2 and
  // i + RS / 2 (y = r0 - 2 + i), zero off the grid (lines off it hold zeros already; rows off
  // it read a clamped row and are cleared by a select): two independent chains per thread,
  // neighbouring lanes on neighbouring rows
  static_assert(RS % 2 == 0, "two halves of the chunk rows");
  constexpr int RH = RS / 2;
  auto stage_a = [&](int c, int q) {
    const int l = q / RH, i = q % RH;
    const int y = c * CH - 2 + i, cl = c0 - 2 + l;
    const cx<T> o0 = buf[l * PITCH + max(y, 0)], o1 = buf[l * PITCH + min(y + RH, N - 1)];
    const cx<T> v0 = amp_phase(o0, cl, y), v1 = amp_phase(o1, cl, y + RH);
    cx<T>* dst = sfb(c) + l * RS + i;
    dst[0] = y >= 0 ? v0 : czero<T>();
    dst[RH] = y + RH < N ? v1 : czero<T>();
  };
  // B(c) on line lb + 1, rows ib = ib0 and ib0 + 1 (y = r0 - 1 + ib).  IN: every stencil
  // of the two pixels stays on the grid, so that no bound is checked.
  auto stage_b = [&](int c, int lb, int ib0, auto in_c) {
    constexpr bool IN = decltype(in_c)::value;
    const int r0 = c * CH;
    const cx<T>* sf = sfb(c);
    unsigned* omx = omb(c);
    unsigned* omy = omx + OWM * OH;
    unsigned* omz = omy + OWM * OH;
    const int l = lb + 1, c_ = cx0 + lb;
    const bool cin = c_ >= 0 && c_ < N, cxx = c_ >= 1 && c_ <= N - 2, cxy = c_ <= N - 2;
    const bool own_c = l >= 2 && l <= W + 1;
    // f rows i = ib + 1 (y) and neighbours: line l rows i - 1 .. i + 2, lines l - 1 and
    // l + 1 as the stencils need, read as aligned 16-byte pairs of rows ib0 .. ib0 + 3 (ib0
    // even), so that neighbouring lanes read neighbouring 16 bytes
    typedef float f4 __attribute__((ext_vector_type(4)));
    auto pair = [](const cx<T>* p, cx<T>& a, cx<T>& b) {
      const f4 v = *reinterpret_cast<const f4*>(p);
      a = cx<T>{v.x, v.y};
      b = cx<T>{v.z, v.w};
    };
    const cx<T>* sc = sf + l * RS + ib0;
    cx<T> ctr[4], lq[4], rq[4];
    pair(sc, ctr[0], ctr[1]);
    pair(sc + 2, ctr[2], ctr[3]);
    pair(sc - RS, lq[0], lq[1]);
    pair(sc - RS + 2, lq[2], lq[3]);
    pair(sc + RS, rq[0], rq[1]);
    pair(sc + RS + 2, rq[2], rq[3]);
    const cx<T> lft[2] = {lq[1], lq[2]}, rgt[3] = {rq[1], rq[2], rq[3]};
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      const int ib = ib0 + t, y = r0 - 1 + ib;
      const bool in = IN || (cin && y >= 0 && y < N);
      const bool vxx = IN || (in && cxx), vyy = IN || (in && y >= 1 && y <= N - 2);
      const bool vxy = IN || (in && cxy && y <= N - 2);
      const cx<T> f = ctr[t + 1], fl = lft[t], fr = rgt[t], fu = ctr[t], fd = ctr[t + 2], frd = rgt[t + 1];
      // components of |O| (.x) and angle(O) (.y), computed everywhere, then cleared where the
      // stencil leaves the grid by a bit mask (an arithmetic select: no branch, no load
      // moved under a condition)
      auto keep = [](T h, bool v) {
        return __builtin_bit_cast(T, __builtin_bit_cast(unsigned, h) & (v ? 0xffffffffu : 0u));
      };
      const T hxa = keep(fl.x - T(2) * f.x + fr.x, vxx), hxp = keep(fl.y - T(2) * f.y + fr.y, vxx);
      const T hya = keep(fu.x - T(2) * f.x + fd.x, vyy), hyp = keep(fu.y - T(2) * f.y + fd.y, vyy);
      const T hza = keep(f.x - fr.x - fd.x + frd.x, vxy), hzp = keep(f.y - fr.y - fd.y + frd.y, vxy);
      const int oi = lb * OH + ib;
      omx[oi] = __builtin_bit_cast(unsigned, __builtin_amdgcn_cvt_pkrtz(sign_unit(hxa), sign_unit(hxp)));
      omy[oi] = __builtin_bit_cast(unsigned, __builtin_amdgcn_cvt_pkrtz(sign_unit(hya), sign_unit(hyp)));
      omz[oi] = __builtin_bit_cast(unsigned, __builtin_amdgcn_cvt_pkrtz(sign_unit(hza), sign_unit(hzp)));
      const bool own = own_c && ib >= 1 && ib <= CH && in;
      ta += own ? fabs(hxa) + fabs(hya) + fabs(hza) : T(0);
      tp += own ? fabs(hxp) + fabs(hyp) + fabs(hzp) : T(0);
    }
  };
  // C(c), item q: own line l = q / (CH / 2) + 2, rows y = r0 + 2 (q mod CH / 2) and the next.
  // With O = s Ot, s = (-1)^(x+y) / n, the value written, s G, is Ot (ka qa / |Ot| + i kp qp /
  // (|Ot|^2 + eta n^2)) with ka = alpha / (2 n) and kp = beta / 2: the sign s drops out.
  const T ka = T(0.5) * T(o.alpha) * inv_n, kp = T(0.5) * T(o.beta);
  const T eta_n2 = T(o.eta_h) / (inv_n * inv_n);
  auto stage_c = [&](int c, int q) {
    const int r0 = c * CH;
    const unsigned* omx = omb(c);
    const unsigned* omy = omx + OWM * OH;
    const unsigned* omz = omy + OWM * OH;
    const int lc = q / (CH / 2), y0 = r0 + 2 * (q % (CH / 2));
    const int l = lc + 2, lb = lc + 1;
    const int oi0 = lb * OH + (y0 - r0 + 1);  // omega index of the run's first pixel
    cx<T> Ot[2];  // the run's two values of Ot, read first (one wait for every read)
#pragma unroll
    for (int t = 0; t < 2; ++t) Ot[t] = buf[l * PITCH + y0 + t];
    h2 zl[3], zc[3], xr[2], xl[2], yc[4], xc[2];
#pragma unroll
    for (int t = 0; t < 4; ++t) yc[t] = __builtin_bit_cast(h2, omy[oi0 + t - 1]);
#pragma unroll
    for (int t = 0; t < 3; ++t) {
      zc[t] = __builtin_bit_cast(h2, omz[oi0 + t - 1]);
      zl[t] = __builtin_bit_cast(h2, omz[oi0 + t - 1 - OH]);
    }
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      xc[t] = __builtin_bit_cast(h2, omx[oi0 + t]);
      xl[t] = __builtin_bit_cast(h2, omx[oi0 + t - OH]);
      xr[t] = __builtin_bit_cast(h2, omx[oi0 + t + OH]);
    }
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      const int y = y0 + t;
      const h2 two = {_Float16(2), _Float16(2)};
      // q = Dxx^T s_xx + Dyy^T s_yy + Dxy^T s_xy at (y, c), both fields, as a shallow tree
      // (sums of at most ten small integers: exact in any order)
      const h2 qq = ((xl[t] + xr[t]) + (yc[t] + yc[t + 2])) + ((zc[t + 1] + zl[t]) - two * (xc[t] + yc[t + 1])) -
                    (zl[t + 1] + zc[t]);
      const T qa = T(qq.x), qp = T(qq.y);
      const T a2 = norm2(Ot[t]);
      const T den = a2 + eta_n2;
      // the amplitude term where |O| > 0 and the phase term where |O|^2 + eta > 0, as selects
      const T fa = a2 > T(0) ? ka * qa * rsqrt_t(a2) : T(0);
      const T fp = den > T(0) ? kp * qp * rcp_t(den) : T(0);
      buf[l * PITCH + y] = scale(Ot[t], fa) + scale(mul_i(Ot[t]), fp);
    }
  };
  // Software pipeline over the chunks, one barrier per stage: stage s runs A(s) (the
  // next chunk's amplitude and phase, into the other array set), B(s - 1) and C(s - 2).
  // A(s) reads O rows r0(s) - 2 .. r0(s) + 65, which C(s - 2) (own rows r0(s) - 128 ..
  // r0(s) - 65) does not touch; A(s) and B(s - 1) use different (|O|, angle(O)) sets,
  // B(s - 1) and C(s - 2) different sign sets.  The items of the three are shared out
  // over the whole block (below), so that no wave idles while another finishes a stage.
  // The OH / 2 two-row items of B on a line: the KB = OH / 2 - 1 whose rows keep their
  // stencils on the grid in every chunk (the first chunk's rows from 1, the last one's up
  // to N - 2) come first, line after line (at the grid's right edge its last two lines
  // first, as at the left edge); the one item per line that holds the grid's first or last
  // row (or the chunk's last two rows elsewhere) comes after all of those.  So the items
  // that check bounds (these and the two lines at the grid's left or right edge) fill
  // whole runs of 64, and the others run without a check.
  constexpr int KB = OH / 2 - 1;
  static_assert(KB == 32 && CH + 2 == OH, "items 0 .. 31 of a line by a shift");
  const int lrot = c0 + W >= N - 1 ? LB - 2 : 0;
  auto b_item = [&](int c, int q) {
    const int core = LB * KB;
    int lb, k;
    if (q < core) {
      lb = q / KB + lrot;
      lb = lb >= LB ? lb - LB : lb;
      k = q % KB + (c == 0 ? 1 : 0);
    } else {
      lb = q - core;
      k = c == 0 ? 0 : KB;
    }
    const int c_ = cx0 + lb, y0 = c * CH - 1 + 2 * k;
    // one form for the whole wave (the checked one is right for every item): no wave runs both
    const bool fast = c_ >= 1 && c_ <= N - 2 && y0 >= 1 && y0 <= N - 3;
    if (__builtin_amdgcn_ballot_w64(!fast) == 0) stage_b(c, lb, 2 * k, std::true_type{});
    else stage_b(c, lb, 2 * k, std::false_type{});
  };
  // A stage's items go out in runs of 64 (one wave each): the runs of B, then of C, then
  // of A (dearest first), dealt to the 16 waves in a snake order (0 .. 15, 15 .. 0, ...),
  // so that every wave runs one kind of item at a time (the kind is uniform across the
  // wave) and the four waves of each SIMD get about the same work.
  static_assert(NT == 1024, "16 waves");
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
  const int nA = NL * (RS / 2), nB = LB * (OH / 2), nC = W * (CH / 2);
  for (int st = 0; st < NCH + 2; ++st) {
    const int ca = st, cb = st - 1, cc = st - 2;
    const int na = ca < NCH ? nA : 0, nb = cb >= 0 && cb < NCH ? nB : 0, nc = cc >= 0 ? nC : 0;
    const int rb = (nb + 63) >> 6, rc = (nc + 63) >> 6, nrun = rb + rc + ((na + 63) >> 6);
    for (int r = 0;; ++r) {
      const int k = r * 16 + ((r & 1) ? 15 - wv : wv);
      if (k >= nrun) break;
      if (k < rb) {
        const int q = k * 64 + lane;
        if (q < nb) b_item(cb, q);
      } else if (k < rb + rc) {
        const int q = (k - rb) * 64 + lane;
        if (q < nc) stage_c(cc, q);
      } else {
        const int q = (k - rb - rc) * 64 + lane;
        if (q < na) stage_a(ca, q);
      }
    }
    if (nb) {
      la += double(ta);
      lp += double(tp);
      ta = T(0);
      tp = T(0);
    }
    __syncthreads();
  }
  // forward DFT along the own columns (lines 2 .. W + 1); the last pass stores its outputs
  // straight to T2 (line m = column c0 + m).  The loss partials wait in shared memory.
  lsum[tid] = la;
  lsum[NT + tid] = lp;
  // deterministic block sums of the two penalty partials, a level between two passes (the
  // passes' barriers publish each level): 64 threads each add 16 slots in order, 8 threads
  // each 8 of those, thread 0 the 8
  static_assert(NT == 1024, "16 x 8 x 8 slots");
  auto sum_level = [&](int nthr, int nin, int src, int dst) {
    if (tid < nthr) {
      double s0 = 0.0, s1 = 0.0;
      for (int w = 0; w < nin; ++w) {
        s0 += lsum[src + (nthr == 64 ? w * 64 + tid : nin * tid + w)];
        s1 += lsum[src + NT + (nthr == 64 ? w * 64 + tid : nin * tid + w)];
      }
      lsum[dst + tid] = s0;
      lsum[dst + NT + tid] = s1;
    }
  };
  {
    cx<T>* own = buf + 2 * PITCH;
    constexpr int WM = Sh::WMAX;
    StockhamPass<T, N, R1, 1, false, NT, ceil_div(WM * (N / R1), NT), PITCH, 1>::run(own, 0, dW, twl, tid);
    sum_level(64, 16, 0, 2 * NT);  // slots 2 NT .. (the first pass's barriers published lsum)
    StockhamPass<T, N, R2, R1, false, NT, ceil_div(WM * (N / R2), NT), PITCH, 1>::run(own, 0, dW, twl, tid);
    // the last two levels in wave 0, in registers (no barrier): threads 0 .. 7 each add 8
    // level-1 slots in order, and thread 0 adds their eight sums in order, read across lanes
    if (tid < 64) {
      double s0 = 0.0, s1 = 0.0;
      if (tid < 8)
        for (int w = 0; w < 8; ++w) {
          s0 += lsum[2 * NT + 8 * tid + w];
          s1 += lsum[3 * NT + 8 * tid + w];
        }
      double f0 = s0, f1 = s1;
#pragma unroll
      for (int i = 1; i < 8; ++i) {
        f0 += __shfl(s0, i, 64);
        f1 += __shfl(s1, i, 64);
      }
      if (tid == 0) {
        o.partial[2 * b + 0] = f0;
        o.partial[2 * b + 1] = f1;
      }
    }
    using PC = StockhamPass<T, N, R3, R1 * R2, false, NT, ceil_div(WM * (N / R3), NT), PITCH, 1>;
    constexpr int MB = ceil_div(WM * (N / R3), NT);
    int m[MB], j[MB];
    bool lv[MB];
    PC::coords(dW, tid, m, j, lv);
    cx<T> v[MB][R3];
    PC::load(own, 0, m, j, lv, twl, v);
#pragma unroll
    for (int i = 0; i < MB; ++i)
      if (lv[i]) {
#pragma unroll
        for (int r = 0; r < R3; ++r) T2[(size_t)PC::out_index(j[i], r) * N + c0 + m[i]] = v[i][r];
      }
  }
}

template <class T, int N, int NT>
__device__ void obj_strip_wide(const LedObjArgs& o, int b, char* lds) {
  if constexpr (sizeof(T) == 4) {
    if (o.norm == 0 && !(o.eps > 0.0)) {
      obj_strip_wide_sign<T, N, NT>(o, b, lds);
      return;
    }
  }
  obj_strip_wide_form<T, N, NT, false>(o, b, lds);
}

// ---------------------------------------------------------------------------
// Hessian penalties (Eq. 6, 7) and their gradient (Eq. 13, 14) on 16 x 16 tiles.
// ---------------------------------------------------------------------------
// Input: Ot = unnormalised inverse DFT of Psi, so O = (-1)^(x+y) Ot / n.
// H components at p: xx = f(x-1) - 2 f(x) + f(x+1) (1 <= x <= n-2), yy likewise,
// xy = f(p) - f(p+ex) - f(p+ey) + f(p+ex+ey) (x, y <= n-2); each zero elsewhere.
// The gradient at p needs omega within 1 pixel, which needs |O| and angle(O)
// within 2 pixels: the block loads a 20 x 20 patch.
template <class T>
__global__ __launch_bounds__(256) void k_hessian(HessArgs a) {
  constexpr int TS = 16, HP = TS + 4, HO = TS + 2;
  __shared__ T sa[HP][HP + 1], sp[HP][HP + 1];
  __shared__ T om[6][HO][HO + 1];
  __shared__ double red[4];
  const int tid = threadIdx.x;
  const int tx0 = blockIdx.x * TS, ty0 = blockIdx.y * TS;
  const int n = a.n;
  const T inv_n = T(a.inv_n);
  const T eps = T(a.eps);
  const cx<T>* Ot = static_cast<const cx<T>*>(a.Ot);
  for (int p = tid; p < HP * HP; p += 256) {
    const int ly = p / HP, lx = p % HP;
    const int gy = ty0 + ly - 2, gx = tx0 + lx - 2;
    T am = T(0), ph = T(0);
    if (gy >= 0 && gy < n && gx >= 0 && gx < n) {
      cx<T> O = scale(Ot[(size_t)gy * n + gx], ((gx + gy) & 1) ? -inv_n : inv_n);
      am = sqrt_t(norm2(O));
      ph = atan2(O.y, O.x);
    }
    sa[ly][lx] = am;
    sp[ly][lx] = ph;
  }
  __syncthreads();
  double la = 0.0, lp = 0.0;
  for (int p = tid; p < HO * HO; p += 256) {
    const int ly = p / HO, lx = p % HO;          // patch index (ly + 1, lx + 1)
    const int gy = ty0 + ly - 1, gx = tx0 + lx - 1;
    const bool in = gy >= 0 && gy < n && gx >= 0 && gx < n;
    const bool vxx = in && gx >= 1 && gx <= n - 2;
    const bool vyy = in && gy >= 1 && gy <= n - 2;
    const bool vxy = in && gx <= n - 2 && gy <= n - 2;
    const bool own = ly >= 1 && ly <= TS && lx >= 1 && lx <= TS && in;
#pragma unroll
    for (int f = 0; f < 2; ++f) {
      T (*src)[HP + 1] = f == 0 ? sa : sp;
      const int cy = ly + 1, cx_ = lx + 1;
      const T c = src[cy][cx_];
      const T hxx = vxx ? src[cy][cx_ - 1] - T(2) * c + src[cy][cx_ + 1] : T(0);
      const T hyy = vyy ? src[cy - 1][cx_] - T(2) * c + src[cy + 1][cx_] : T(0);
      const T hxy = vxy ? c - src[cy][cx_ + 1] - src[cy + 1][cx_] + src[cy + 1][cx_ + 1] : T(0);
      T wxx, wyy, wxy;
      double l;
      if (a.norm == 0) {
        wxx = omega(hxx, eps);
        wyy = omega(hyy, eps);
        wxy = omega(hxy, eps);
        l = double(rho(hxx, eps)) + double(rho(hyy, eps)) + double(rho(hxy, eps));
      } else {
        const T s2 = hxx * hxx + hyy * hyy + hxy * hxy;
        const T inv = inv_norm(s2, eps);
        wxx = hxx * inv;
        wyy = hyy * inv;
        wxy = hxy * inv;
        l = eps > T(0) ? double(sqrt_t(s2 + eps * eps) - eps) : double(sqrt_t(s2));
      }
      om[3 * f + 0][ly][lx] = wxx;
      om[3 * f + 1][ly][lx] = wyy;
      om[3 * f + 2][ly][lx] = wxy;
      if (own) {
        if (f == 0) la += l;
        else lp += l;
      }
    }
  }
  __syncthreads();
  const int ty = tid / TS, tx = tid % TS;
  const int gy = ty0 + ty, gx = tx0 + tx;
  if (a.want_grad && gy < n && gx < n) {
    const int ly = ty + 1, lx = tx + 1;  // omega index of the own pixel
    T q[2];
#pragma unroll
    for (int f = 0; f < 2; ++f) {
      const T (*wx)[HO + 1] = om[3 * f + 0];
      const T (*wy)[HO + 1] = om[3 * f + 1];
      const T (*wz)[HO + 1] = om[3 * f + 2];
      q[f] = wx[ly][lx - 1] - T(2) * wx[ly][lx] + wx[ly][lx + 1] + wy[ly - 1][lx] - T(2) * wy[ly][lx] +
             wy[ly + 1][lx] + wz[ly][lx] - wz[ly][lx - 1] - wz[ly - 1][lx] + wz[ly - 1][lx - 1];
    }
    const T sgn = ((gx + gy) & 1) ? -inv_n : inv_n;
    const cx<T> O = scale(Ot[(size_t)gy * n + gx], sgn);
    const T a2 = norm2(O);
    const T am = sqrt_t(a2);
    cx<T> G = czero<T>();
    if (am > T(0)) G = scale(O, T(a.alpha) * q[0] / (T(2) * am));
    const T den = a2 + T(a.eta_h);
    if (den > T(0)) G = G + scale(mul_i(O), T(a.beta) * q[1] / (T(2) * den));
    static_cast<cx<T>*>(a.Gt)[(size_t)gy * n + gx] = scale(G, sgn);
  }
  // deterministic block sums of the two penalty partials
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    la += __shfl_down(la, off, 64);
    lp += __shfl_down(lp, off, 64);
  }
  __shared__ double red2[4][2];
  if ((tid & 63) == 0) {
    red2[tid >> 6][0] = la;
    red2[tid >> 6][1] = lp;
  }
  __syncthreads();
  if (tid == 0) {
    const int tile = blockIdx.y * gridDim.x + blockIdx.x;
    a.partial[2 * tile + 0] = red2[0][0] + red2[1][0] + red2[2][0] + red2[3][0];
    a.partial[2 * tile + 1] = red2[0][1] + red2[1][1] + red2[2][1] + red2[3][1];
  }
  (void)red;
}

// ---------------------------------------------------------------------------
// Eq. (19) for one element, FP64 second moment and normaliser.
// ---------------------------------------------------------------------------
template <class T>
__device__ __forceinline__ void adabelief_elem(cx<T>& x, cx<T> g, cx<T>& mu, double& v, T& delta, double g1,
                                               double g2, double eta, double ibc1, double ibc2) {
  const T tg1 = T(g1);
  const cx<T> m = {tg1 * mu.x + (T(1) - tg1) * g.x, tg1 * mu.y + (T(1) - tg1) * g.y};
  const double dxr = double(m.x) - double(g.x), dxi = double(m.y) - double(g.y);
  const double vn = g2 * v + (1.0 - g2) * (dxr * dxr + dxi * dxi);
  const double ratio = (sqrt(double(delta)) + eta) / (sqrt(vn * ibc2) + eta);
  // gamma1 * mu_hat + (1 - gamma1) g, with mu_hat = m / (1 - g1^t); the fused multiply-add
  // is written out so that every kernel that inlines this rounds it the same way
  const double sx = __builtin_fma(g1 * double(m.x), ibc1, (1.0 - g1) * double(g.x));
  const double sy = __builtin_fma(g1 * double(m.y), ibc1, (1.0 - g1) * double(g.y));
  const cx<T> step = {T(ratio * sx), T(ratio * sy)};
  x = x - step;
  delta = tg1 * delta + (T(1) - tg1) * norm2(step);
  mu = m;
  v = vn;
}

// 1 - g1^t, 1 - g2^t and 1 - g1^(t+1) for step t >= 1, from lg = log2(g) (computed
// once on the host; -inf for g = 0): g^t = 2^(t lg), a fraction of the cost of pow.
// bc[3 .. 5] are their reciprocals, so that each element multiplies instead of dividing.
__device__ __forceinline__ void bias_corrections(double lg1, double lg2, double t, double* bc) {
  bc[0] = 1.0 - exp2(t * lg1);
  bc[1] = 1.0 - exp2(t * lg2);
  bc[2] = 1.0 - exp2((t + 1.0) * lg1);
  bc[3] = 1.0 / bc[0];
  bc[4] = 1.0 / bc[1];
  bc[5] = 1.0 / bc[2];
}

// The update rule of the plan (ELFPIE_OPT_*) for one element: Eq. 19, or for the
// comparison of Sec. 6.2 plain gradient descent, NAdam (constant momentum) or
// AdaBelief.  v and the normaliser are FP64; delta is used by Eq. 19 only.
template <class T>
__device__ __forceinline__ void optimizer_elem(int opt, cx<T>& x, cx<T> g, cx<T>& mu, double& v, T& delta,
                                               double g1, double g2, double eta, double lr, const double* bc) {
  if (opt == 0) {
    adabelief_elem(x, g, mu, v, delta, g1, g2, eta, bc[3], bc[4]);
    return;
  }
  if (opt == 1) {
    x = x - cx<T>{T(lr * double(g.x)), T(lr * double(g.y))};
    return;
  }
  const T tg1 = T(g1);
  const cx<T> m = {tg1 * mu.x + (T(1) - tg1) * g.x, tg1 * mu.y + (T(1) - tg1) * g.y};
  double sx, sy, vn;
  if (opt == 2) {  // NAdam: moments of g; look-ahead mean
    vn = g2 * v + (1.0 - g2) * (double(g.x) * double(g.x) + double(g.y) * double(g.y));
    sx = __builtin_fma(g1 * double(m.x), bc[5], (1.0 - g1) * double(g.x) * bc[3]);
    sy = __builtin_fma(g1 * double(m.y), bc[5], (1.0 - g1) * double(g.y) * bc[3]);
  } else {  // AdaBelief: belief (g - m)^2 plus eps
    const double dxr = double(g.x) - double(m.x), dxi = double(g.y) - double(m.y);
    vn = g2 * v + (1.0 - g2) * (dxr * dxr + dxi * dxi) + eta;
    sx = double(m.x) * bc[3];
    sy = double(m.y) * bc[3];
  }
  const double f = lr / (sqrt(vn * bc[4]) + eta);
  x = x - cx<T>{T(f * sx), T(f * sy)};
  mu = m;
  v = vn;
}

// ---------------------------------------------------------------------------
// Pupil: partial sums over LED chunks (Eq. 18) and the Gaussian pre-filter in one
// launch (blocks with blockIdx.y == nch filter), then the update.
// ---------------------------------------------------------------------------
constexpr int kPupilChunk = 16;

// Virtual block vb of the pupil work carried by the spectrum-update launch:
// vb < nsb * nch: partial sum of LED chunk vb / nsb for NT support pixels;
// after that: the 3 x 3 Gaussian of the current pupil (zero padding) for NT pixels.
// The 3 x 3 Gaussian of the n x n pupil P at pixel p (zero padding; Algorithm 1's
// pre-filter): weights w_c at the centre, w_e on the edges, w_k on the corners.
template <class T>
__device__ __forceinline__ cx<T> pupil_gauss3(const cx<T>* P, int n, int p, double w_c, double w_e, double w_k) {
  const int y = p / n, x = p % n;
  cx<T> nb[9];
#pragma unroll
  for (int t = 0; t < 9; ++t) {
    const int yy = min(max(y + t / 3 - 1, 0), n - 1), xx = min(max(x + t % 3 - 1, 0), n - 1);
    nb[t] = P[yy * n + xx];
  }
  cx<T> acc = czero<T>();
#pragma unroll
  for (int t = 0; t < 9; ++t) {
    const int dy = t / 3 - 1, dx = t % 3 - 1;
    const bool in = y + dy >= 0 && y + dy < n && x + dx >= 0 && x + dx < n;
    const int ring = (dy != 0) + (dx != 0);
    const T w = in ? T(ring == 0 ? w_c : (ring == 1 ? w_e : w_k)) : T(0);
    acc = acc + scale(nb[t], w);
  }
  return acc;
}

template <class T, int NT>
__device__ __forceinline__ void pupil_block(const PupilArgs& a, int vb, int tid) {
  const int nsb = (a.S + NT - 1) / NT;
  if (vb >= nsb * a.nch) {
    const int p = (vb - nsb * a.nch) * NT + tid;
    const int n = a.n_lo;
    if (p >= n * n) return;
    static_cast<cx<T>*>(a.Pf_out)[p] = pupil_gauss3<T>(static_cast<const cx<T>*>(a.P), n, p, a.w_c, a.w_e, a.w_k);
    return;
  }
  const int ch = vb / nsb;
  const int s = (vb - ch * nsb) * NT + tid;
  if (s >= a.S) return;
  const cx<T>* D = static_cast<const cx<T>*>(a.D);
  const int k0 = ch * kPupilChunk;
  cx<T> v[kPupilChunk];
#pragma unroll
  for (int j = 0; j < kPupilChunk; ++j) {
    const int k = k0 + j < a.K ? k0 + j : k0;
    v[j] = D[(size_t)k * a.S + s];
  }
  cx<T> acc = czero<T>();
#pragma unroll
  for (int j = 0; j < kPupilChunk; ++j)
    if (k0 + j < a.K) acc = acc + v[j];
  static_cast<cx<T>*>(a.part)[(size_t)ch * a.n_lo * a.n_lo + a.s2p[s]] = acc;
}

// The pupil work of an update launch in which the pupil update completes
// (PupilArgs::final_in_launch), with no dependence between blocks: virtual block vb < nsb
// takes PX support pixels whole.  Its NT / PX groups of PX threads each sum a contiguous
// run of LEDs of every pixel (ascending LED order; lanes on consecutive pixels, so each
// LED's row of D is read in one run), the group sums are added in group order, and the
// first group applies Eq. 19 (or writes the gradient).  Blocks past those update the
// pixels off the support (zero gradient).  red: PX * NT / PX complex of shared memory;
// sbc: the shared bias corrections.
template <class T>
__device__ __forceinline__ void pupil_update_g(const PupilArgs& a, const double* sbc, int p, cx<T> g);

template <class T, int NT>
__device__ __forceinline__ void pupil_block_final(const PupilArgs& a, int vb, int tid, double* sbc, cx<T>* red) {
  constexpr int PX = 32, G = NT / PX;
  static_assert(NT % PX == 0, "whole groups");
  const int nsb = (a.S + PX - 1) / PX;
  if (a.step && tid == 0) bias_corrections(a.lg1, a.lg2, double(*a.t), sbc);
  if (vb >= nsb) {
    __syncthreads();  // sbc
    const int n = a.n_lo, p = (vb - nsb) * NT + tid;
    if (p >= n * n) return;
    const int y = p / n, x = p % n;
    if (x >= a.xlo[y] && x <= a.xhi[y]) return;  // on the support: a pixel block's
    pupil_update_g<T>(a, sbc, p, czero<T>());
    return;
  }
  const int sl = tid % PX, grp = tid / PX;
  const int s = vb * PX + sl;
  const int kc = (a.K + G - 1) / G, k0 = grp * kc, k1 = min(a.K, k0 + kc);
  const cx<T>* D = static_cast<const cx<T>*>(a.D);
  cx<T> acc = czero<T>();
  if (s < a.S) {
    constexpr int B = 8;  // loads in flight per batch
    for (int kb = k0; kb < k1; kb += B) {
      cx<T> v[B];
#pragma unroll
      for (int j = 0; j < B; ++j) v[j] = kb + j < k1 ? D[(size_t)(kb + j) * a.S + s] : czero<T>();
#pragma unroll
      for (int j = 0; j < B; ++j)
        if (kb + j < k1) acc = acc + v[j];
    }
  }
  red[grp * PX + sl] = acc;
  __syncthreads();
  if (grp == 0 && s < a.S) {
    cx<T> g = red[sl];
    for (int q = 1; q < G; ++q) g = g + red[q * PX + sl];
    pupil_update_g<T>(a, sbc, a.s2p[s], g);
  }
}

// Spectrum gradient gather (the segmented sum of the LED contributions that cover
// each pixel, ascending LED order: Eq. 9's sum of M^T C_k, no atomics) plus the
// Hessian gradient, then either the gradient is written or Eq. 19 updates Psi.
// One 16 x 16 tile per block: the tile's LED list and the support row table are
// staged in LDS and up to GB contribution loads per pixel are issued together (an
// off-support entry reads C[0] and is discarded), so the sum keeps its fixed order.
// Blocks past the tiles run the pupil partial sums and pre-filter, which depend
// only on the per-LED kernel, as this launch does.
#ifndef ELFPIE_UPD_GB
#define ELFPIE_UPD_GB 8  // contribution loads in flight per pixel
#endif
template <class T>
__global__ __launch_bounds__(256) void k_update(UpdArgs a, PupilArgs pa) {
  constexpr int GB = ELFPIE_UPD_GB;
  using cint = const __attribute__((address_space(4))) int;  // read-only: wave-uniform reads go scalar
  __shared__ int4 stab[kMaxLo];  // per support row: first column, last column, row base (rowoff - xlo)
  __shared__ double sbc[6];
  const int tid = threadIdx.x;
  const int tile = blockIdx.x;
  if (tile >= a.ntiles) {
    pupil_block<T, 256>(pa, tile - a.ntiles, tid);
    return;
  }
  const int ty0 = (tile / a.ntiles_x) * 16, tx0 = (tile % a.ntiles_x) * 16;
  const int uy = ty0 + tid / 16, ux = tx0 + tid % 16;
  const size_t u = (size_t)uy * a.n_hi + ux;
  for (int i = tid; i < a.n_lo; i += 256) stab[i] = make_int4(a.xlo[i], a.xhi[i], a.rowoff[i] - a.xlo[i], 0);
  if (a.step && tid == 0) {
    const double t = double(*a.t);
    bias_corrections(a.lg1, a.lg2, t, sbc);
  }
  // state loads go out first; they do not depend on the gather
  cx<T> g = static_cast<const cx<T>*>(a.gH)[u];
  cx<T> x = czero<T>(), mu = czero<T>();
  double v = 0.0;
  T d = T(0);
  if (a.step) {
    x = static_cast<cx<T>*>(a.x)[u];
    mu = static_cast<cx<T>*>(a.mu)[u];
    v = a.v[u];
    d = static_cast<T*>(a.delta)[u];
  }
  __syncthreads();
  const cx<T>* C = static_cast<const cx<T>*>(a.C);
  cint* tp = (cint*)a.tile_ptr;
  cint* tl = (cint*)a.tile_led;
  const int b0 = tp[tile], b1 = tp[tile + 1];
  for (int l0 = b0; l0 < b1; l0 += GB) {
    size_t idx[GB];
    bool ok[GB];
#pragma unroll
    for (int j = 0; j < GB; ++j) {
      const int l = min(l0 + j, b1 - 1);  // wave-uniform list entry
      const int k = tl[3 * l], dy = uy - tl[3 * l + 1], dx = ux - tl[3 * l + 2];
      const int4 row = stab[min(max(dy, 0), a.n_lo - 1)];
      ok[j] = l0 + j < b1 && dy >= 0 && dy < a.n_lo && dx >= row.x && dx <= row.y;
      idx[j] = (size_t)k * a.S + row.z + dx;
    }
    // exec-masked loads: lanes off the support issue nothing
    cx<T> cv[GB];
#pragma unroll
    for (int j = 0; j < GB; ++j) cv[j] = ok[j] ? C[idx[j]] : czero<T>();
#pragma unroll
    for (int j = 0; j < GB; ++j) g = g + cv[j];  // adding zero leaves g unchanged
  }
  if (!a.step) {
    static_cast<cx<T>*>(a.g_out)[u] = g;
    return;
  }
  __syncthreads();
  optimizer_elem(a.opt, x, g, mu, v, d, a.g1, a.g2, a.eta, a.lr, sbc);
  static_cast<cx<T>*>(a.x)[u] = x;
  static_cast<cx<T>*>(a.mu)[u] = mu;
  a.v[u] = v;
  static_cast<T*>(a.delta)[u] = d;
}

// The same update on whole rows of the spectrum, with the row transforms on either
// side folded in, so that neither needs a launch of its own:
//   the rows of T2 (the Hessian-term gradient after its column transforms) get their
//   forward row DFT in LDS, which completes gH;
//   g = gH + the LED contributions covering each pixel, summed in ascending LED order
//   (the same terms in the same order as k_update) from per-(row, 16-column segment)
//   lists; a wave's 64 pixels span four segments, one per 16-lane quarter;
//   step mode applies the plan's rule (Eq. 19) and writes the state, gradient mode
//   writes g;
//   with inv, the rows of psi as they leave this launch get their inverse row DFT
//   into T1, the first step of the next iteration's object branch.
// Blocks past the rows run the pupil partial sums and pre-filter, as in k_update, and
// a last block may reduce this iteration's loss (its partials are all written).
#ifndef ELFPIE_UPDR_GB
#define ELFPIE_UPDR_GB 16  // contribution loads in flight per pixel (row form)
#endif
#ifndef ELFPIE_UPDR_PF
#define ELFPIE_UPDR_PF 10  // contribution loads issued before the row transform (one pixel per thread)
#endif
#ifndef ELFPIE_UPDROWS_NT
#define ELFPIE_UPDROWS_NT 512  // threads per block (at most one per pixel of the block's rows)
#endif
#ifndef ELFPIE_UPDROWS_RB
#define ELFPIE_UPDROWS_RB 1  // rows per block where 256 threads cover whole rows
#endif
#ifndef ELFPIE_UPDR_MINW
#define ELFPIE_UPDR_MINW 6
#endif
#ifndef ELFPIE_PUP_RUN
#define ELFPIE_PUP_RUN 8  // neighbouring pupil support groups per XCD run
#endif

// the longest run of neighbouring row blocks per XCD, up to g (a power of two), that deals
// the nr row blocks to the 8 XCDs in whole runs (1: plain round-robin)
constexpr int upd_row_run(int nr, int g) {
  while (g > 1 && nr % (8 * g) != 0) g /= 2;
  return g;
}

template <int N> struct UpdRows {
  static constexpr int RB = (N == 128 || N == 384) ? 2 : ELFPIE_UPDROWS_RB;
  static constexpr int NT0 = ELFPIE_UPDROWS_NT < RB * N ? ELFPIE_UPDROWS_NT : RB * N;
  static constexpr int NT = (RB * N) % NT0 == 0 ? NT0 : 256;
  static constexpr int MINW = N == 512 ? ELFPIE_UPDR_MINW : 1;  // waves per SIMD the registers must allow (512^2)
};

// For the 512^2 spectrum in FP32, three 512-thread row blocks per compute unit (six waves
// per SIMD: at most 80 registers), so that a launch's row and pupil blocks are resident
// together.
template <class T, int N>
__global__ __launch_bounds__(UpdRows<N>::NT, sizeof(T) == 4 ? UpdRows<N>::MINW : 1) void k_update_rows(
    UpdArgs a, PupilArgs pa, FinArgs fa) {
  constexpr int RB = UpdRows<N>::RB, NT = UpdRows<N>::NT, PITCH = N + 1;
  constexpr int PPT = RB * N / NT;  // pixels per thread
  static_assert(PPT * NT == RB * N && N % 64 == 0, "whole pixels per thread, whole segments per wave");
  constexpr int GB = ELFPIE_UPDR_GB;
  __shared__ cx<T> buf[RB * PITCH];
  __shared__ cx<T> twl[N];
  __shared__ double sbc[6];
  __shared__ double fred[3][4];
  const int tid = threadIdx.x;
  if ((int)blockIdx.x >= N / RB + a.pupil_blocks) {  // this iteration's loss
    finalize_block<NT>(fa, tid, fred);
    return;
  }
  // the pupil blocks: first in the launch when the pupil update completes here (their
  // count a multiple of 8, so the rows keep their XCDs), else after the rows
  const int pfirst = pa.final_in_launch ? a.pupil_blocks : 0;
  if (pa.final_in_launch && (int)blockIdx.x < pfirst) {
    static_assert(RB * PITCH >= NT, "the group sums fit the row buffer");
    // runs of R neighbouring support groups per XCD: a group's D reads (32 pixels of every
    // LED) share their first and last cache lines with its neighbours', and within an XCD
    // those lines are fetched once; the runs are dealt to the XCDs in turn
    constexpr int R = ELFPIE_PUP_RUN;
    int vb = blockIdx.x;
    if (R > 1 && pfirst % (8 * R) == 0) vb = (vb / (8 * R)) * 8 * R + (vb % 8) * R + (vb / 8) % R;
    pupil_block_final<T, NT>(pa, vb, tid, sbc, buf);
    return;
  }
  if (!pa.final_in_launch && (int)blockIdx.x >= N / RB) {
    pupil_block<T, NT>(pa, blockIdx.x - N / RB, tid);
    return;
  }
  // runs of G neighbouring rows per XCD (their contribution segments meet in cache lines
  // of C), the runs still spread over the XCDs in turn; G is the longest run up to
  // ELFPIE_UPD_PAIR that divides the rows evenly
  constexpr int G = upd_row_run(N / RB, ELFPIE_UPD_PAIR);
  int rb = blockIdx.x - pfirst;
  if (G > 1) rb = (rb / (8 * G)) * 8 * G + (rb % 8) * G + (rb / 8) % G;
  const int r0 = rb * RB;
  const bool step = a.step != 0, keep_x = step || a.inv;
  for (int i = tid; i < N; i += NT) twl[i] = static_cast<const cx<T>*>(a.tw)[i];
  if (step && tid == 0) bias_corrections(a.lg1, a.lg2, double(*a.t), sbc);
  const cx<T>* Hc = static_cast<const cx<T>*>(a.gH) + (size_t)r0 * N;
#pragma unroll
  for (int i = 0; i < PPT; ++i) {
    const int p = tid + i * NT;
    buf[(p / N) * PITCH + p % N] = Hc[p];
  }
  cx<T> x[PPT], mu[PPT];
  double v[PPT];
  T d[PPT];
  // the parameter and optimiser state of this thread's pixels, needed only at Eq. 19
  auto load_state = [&]() {
#pragma unroll
    for (int i = 0; i < PPT; ++i) {
      const size_t u = (size_t)r0 * N + tid + i * NT;
      x[i] = keep_x ? static_cast<const cx<T>*>(a.x)[u] : czero<T>();
      mu[i] = czero<T>();
      v[i] = 0.0;
      d[i] = T(0);
      if (step) {
        mu[i] = static_cast<const cx<T>*>(a.mu)[u];
        v[i] = a.v[u];
        d[i] = static_cast<const T*>(a.delta)[u];
      }
    }
  };
  const cx<T>* C = static_cast<const cx<T>*>(a.C);
  const int2* se = static_cast<const int2*>(static_cast<const void*>(a.seg_ent));
  // Each pixel's list is that of its 16-column segment, which is also its 16-lane quarter
  // of the wave.  Lane j holds entries j & 15 and 16 + (j & 15) of its quarter's list
  // (one 8-byte load each: contribution base, and the first and last column packed), and
  // the walk hands entry l of each quarter to the quarter's lanes with ds_bpermute, so the
  // wave walks the longest of its four lists rather than the union of them.  Entries past
  // 32 (long lists only) are read by each lane itself.
  static_assert(kUpdSegW == 16, "one list per 16-lane quarter");
  const int lane = tid & 63;
  const int qaddr = (lane & 48) << 2;  // ds_bpermute byte address of the quarter's lane 0
  constexpr int kNone = 0xffff;        // packed columns of a missing entry: first 65535, last 0
  int nw[PPT], lbA[PPT], pkA[PPT], lbB[PPT], pkB[PPT];
#pragma unroll
  for (int i = 0; i < PPT; ++i) {
    const int p = tid + i * NT;
    const int seg = (r0 + p / N) * a.nseg + (p % N) / kUpdSegW;
    const int b0 = a.seg_ptr[seg], nl = a.seg_ptr[seg + 1] - b0;
    const int q = lane & 15;
    const int2 ea = se[q < nl ? b0 + q : 0];  // entry 0 exists, also for an empty list
    const int2 eb = se[q + 16 < nl ? b0 + q + 16 : 0];
    lbA[i] = ea.x;
    pkA[i] = q < nl ? ea.y : kNone;  // a missing entry covers no column
    lbB[i] = eb.x;
    pkB[i] = q + 16 < nl ? eb.y : kNone;
    const int m01 = max(__builtin_amdgcn_readlane(nl, 0), __builtin_amdgcn_readlane(nl, 16));
    const int m23 = max(__builtin_amdgcn_readlane(nl, 32), __builtin_amdgcn_readlane(nl, 48));
    nw[i] = __builtin_amdgcn_readfirstlane(max(m01, m23));  // the wave's longest list
  }
  // entry l (wave-uniform, below 32) of this lane's quarter list: C index base and columns
  auto held = [&](int i, int l, int& base, int& xs, int& xe) {
    const int addr = qaddr | ((l & 15) << 2);
    base = __builtin_amdgcn_ds_bpermute(addr, l < 16 ? lbA[i] : lbB[i]);
    const int pk = __builtin_amdgcn_ds_bpermute(addr, l < 16 ? pkA[i] : pkB[i]);
    xs = pk & 0xffff;
    xe = pk >> 16;
  };
  // with one pixel per thread, the first PG contribution loads go out before the row
  // transform (the barriers there wait for LDS only), and are added after gH, in the
  // same order as the walk below
  constexpr bool PF = PPT == 1;
  constexpr int PG = PF ? ELFPIE_UPDR_PF : 1;  // loads issued early
  static_assert(PG <= 16, "early loads come from the first entries held in lanes");
  cx<T> pre[PG];
  if constexpr (PF) {
    const int ux = tid % N;
    // all hand-overs first, then all loads (one wait on the LDS counter between them)
    int pidx[PG];
    bool pok[PG];
#pragma unroll
    for (int j = 0; j < PG; ++j) {
      int base, xs, xe;
      held(0, j, base, xs, xe);
      pok[j] = ux >= xs && ux <= xe;
      pidx[j] = base + ux;
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int j = 0; j < PG; ++j) pre[j] = pok[j] ? C[pidx[j]] : czero<T>();
  }
  // Loads return in issue order: state loads issued before the list entries would hold up
  // the early contribution loads, and issued before the row DFT they would hold up the walk
  // after it.  In step mode they go out with the walk's first round (or after the row DFT
  // where there is none); in gradient mode (psi alone, for T1) before the row DFT.
  __builtin_amdgcn_sched_barrier(0);
  if (!step) load_state();
  __syncthreads();
  fft_lines_inplace<T, N, false, NT, RB>(buf, twl, tid);  // gH; ends with a barrier

#pragma unroll
  for (int i = 0; i < PPT; ++i) {
    const int p = tid + i * NT;
    const int ux = p % N;
    cx<T>& slot = buf[(p / N) * PITCH + ux];
    cx<T> g = slot;
    // the held entries in rounds of GB loads whose entry numbers are compile-time
    // constants (so the hand-over needs no address arithmetic); a missing entry covers
    // no column, and the rounds past the wave's longest list are skipped
    constexpr int LS = PF ? PG : 0;
    if constexpr (PF) {
#pragma unroll
      for (int j = 0; j < PG; ++j) g = g + pre[j];
    }
#pragma unroll
    for (int l0 = LS; l0 < 32; l0 += GB) {
      if (nw[i] <= l0) break;  // wave-uniform
      int idx[GB];
      bool ok[GB];
#pragma unroll
      for (int j = 0; j < GB; ++j) {
        if (l0 + j >= 32) break;
        int base, xs, xe;
        held(i, l0 + j, base, xs, xe);
        ok[j] = ux >= xs && ux <= xe;
        idx[j] = base + ux;
      }
      cx<T> cv[GB];
#pragma unroll
      for (int j = 0; j < GB; ++j) cv[j] = l0 + j < 32 && ok[j] ? C[idx[j]] : czero<T>();
      if (step && i == 0 && l0 == LS) {
        __builtin_amdgcn_sched_barrier(0);
        load_state();
      }
#pragma unroll
      for (int j = 0; j < GB; ++j) g = g + cv[j];  // adding zero leaves g unchanged
    }
    if (step && i == 0 && nw[0] <= LS) load_state();
    // entries past the 32 held in lanes (long lists only), read by each lane
    if (nw[i] > 32) {
      const int seg = (r0 + p / N) * a.nseg + ux / kUpdSegW;
      const int b0 = a.seg_ptr[seg], nl = a.seg_ptr[seg + 1] - b0;
      for (int l0 = 32; l0 < nw[i]; l0 += GB) {
        int idx[GB];
        bool ok[GB];
#pragma unroll
        for (int j = 0; j < GB; ++j) {
          const int l = l0 + j;
          const int2 e = se[l < nl ? b0 + l : 0];
          ok[j] = l < nl && ux >= (e.y & 0xffff) && ux <= (e.y >> 16);
          idx[j] = e.x + ux;
        }
        cx<T> cv[GB];
#pragma unroll
        for (int j = 0; j < GB; ++j) cv[j] = ok[j] ? C[idx[j]] : czero<T>();
#pragma unroll
        for (int j = 0; j < GB; ++j) g = g + cv[j];
      }
    }
    const size_t u = (size_t)r0 * N + p;
    if (step) {
      optimizer_elem(a.opt, x[i], g, mu[i], v[i], d[i], a.g1, a.g2, a.eta, a.lr, sbc);
      static_cast<cx<T>*>(a.x)[u] = x[i];
      static_cast<cx<T>*>(a.mu)[u] = mu[i];
      a.v[u] = v[i];
      static_cast<T*>(a.delta)[u] = d[i];
    } else {
      static_cast<cx<T>*>(a.g_out)[u] = g;
    }
    slot = x[i];
  }
  if (!a.inv) return;
  __syncthreads();
  fft_lines_inplace<T, N, true, NT, RB>(buf, twl, tid);
  cx<T>* T1 = static_cast<cx<T>*>(a.T1) + (size_t)r0 * N;
#pragma unroll
  for (int i = 0; i < PPT; ++i) {
    const int p = tid + i * NT;
    T1[p] = buf[(p / N) * PITCH + p % N];
  }
}

// ---------------------------------------------------------------------------
// Loss terms of Eq. (8): deterministic FP64 reduction by one block of NT threads.
// The summation order is that of 256 lanes whatever NT is (a thread of a smaller
// block plays 256 / NT lanes), so every launch that carries it gives the same bits.
// ---------------------------------------------------------------------------
template <int NT>
__device__ __forceinline__ void finalize_block(const FinArgs& a, int tid, double (*red)[4]) {
  constexpr int V = NT >= 256 ? 1 : 256 / NT;
  static_assert(NT % 64 == 0 && (NT >= 256 || 256 % NT == 0), "whole wavefronts");
#pragma unroll
  for (int r = 0; r < V; ++r) {
    const int vt = tid + r * NT;
    if (vt < 256) {  // wave-uniform
      double f = 0.0, la = 0.0, lp = 0.0;
      for (int i = vt; i < a.K; i += 256) f += a.fid_partial[i];
#pragma unroll 4
      for (int i = vt; i < a.ntiles; i += 256) {
        la += a.hess_partial[2 * i];
        lp += a.hess_partial[2 * i + 1];
      }
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) {
        f += __shfl_down(f, off, 64);
        la += __shfl_down(la, off, 64);
        lp += __shfl_down(lp, off, 64);
      }
      if ((vt & 63) == 0) {
        red[0][vt >> 6] = f;
        red[1][vt >> 6] = la;
        red[2][vt >> 6] = lp;
      }
    }
  }
  __syncthreads();
  if (tid == 0) {
    const double F = red[0][0] + red[0][1] + red[0][2] + red[0][3];
    const double A = red[1][0] + red[1][1] + red[1][2] + red[1][3];
    const double Ph = red[2][0] + red[2][1] + red[2][2] + red[2][3];
    const double L = F + a.alpha * A + a.beta * Ph;
    if (a.loss4) {
      a.loss4[0] = F;
      a.loss4[1] = A;
      a.loss4[2] = Ph;
      a.loss4[3] = L;
    }
    if (a.hist) {
      const int c = *a.ctr;
      a.hist[4 * c + 0] = F;
      a.hist[4 * c + 1] = A;
      a.hist[4 * c + 2] = Ph;
      a.hist[4 * c + 3] = L;
      *a.ctr = c + 1;
    }
    if (!isfinite(L)) *a.flag = 1;
  }
}

// The pupil partial sums and pre-filter as a launch of their own.
template <class T>
__global__ __launch_bounds__(256) void k_pupil_partial(PupilArgs a) {
  pupil_block<T, 256>(a, blockIdx.x, threadIdx.x);
}

template <class T>
__device__ __forceinline__ void pupil_update_body(const PupilArgs& a, const double* sbc, int p);

// Virtual block vb of an iteration's tail (block-uniform branches): Eq. 19 on NT
// pupil pixels, or the loss reduction.  t already counts this iteration.
template <class T, int NT>
__device__ __forceinline__ void tail_block(const TailArgs& ta, int vb, int tid, double* sbc, double (*red)[4]) {
  if (vb < ta.pupil_blocks) {
    const PupilArgs& a = ta.pa;
    if (a.step && tid == 0) {
      const double t = double(*a.t);
      bias_corrections(a.lg1, a.lg2, t, sbc);
    }
    __syncthreads();
    const int p = vb * NT + tid;
    if (p < a.n_lo * a.n_lo) pupil_update_body<T>(a, sbc, p);
  } else if (ta.fin_block && vb == ta.pupil_blocks) {
    finalize_block<NT>(ta.fin, tid, red);
  }
}

// An iteration's tail as a launch of its own.
template <class T>
__global__ __launch_bounds__(256) void k_tail(TailArgs ta) {
  __shared__ double sbc[6];
  __shared__ double red[3][4];
  tail_block<T, 256>(ta, blockIdx.x, threadIdx.x, sbc, red);
}

// Eq. 19 on one pupil pixel p, in two halves (declared above).

template <class T>
__device__ __forceinline__ void pupil_prefetch(const PupilArgs& a, int p, PupilPre<T>& f) {
  const int n = a.n_lo, y = p / n;
  const size_t A = (size_t)n * n;
  const cx<T>* part = static_cast<const cx<T>*>(a.part);
  f.lo = a.xlo[y];
  f.hi = a.xhi[y];
#pragma unroll
  for (int c = 0; c < PupilPre<T>::MC; ++c) f.part[c] = c < a.nch ? part[c * A + p] : czero<T>();
  f.xv = czero<T>();
  f.mu = czero<T>();
  f.v = 0.0;
  f.d = T(0);
  if (a.step) {
    f.xv = a.filter ? static_cast<const cx<T>*>(a.Pf)[p] : static_cast<const cx<T>*>(a.P)[p];
    f.mu = static_cast<const cx<T>*>(a.mu)[p];
    f.v = a.v[p];
    f.d = static_cast<const T*>(a.delta)[p];
  }
}

template <class T>
__device__ __forceinline__ void pupil_finish(const PupilArgs& a, const double* sbc, int p, PupilPre<T>& f) {
  const int n = a.n_lo, x = p % n;
  const size_t A = (size_t)n * n;
  cx<T> g = czero<T>();
#pragma unroll
  for (int c = 0; c < PupilPre<T>::MC; ++c)
    if (c < a.nch) g = g + f.part[c];
  for (int c = PupilPre<T>::MC; c < a.nch; ++c) g = g + static_cast<const cx<T>*>(a.part)[c * A + p];
  const bool in = x >= f.lo && x <= f.hi;
  if (!in) g = czero<T>();
  if (!a.step) {
    static_cast<cx<T>*>(a.g_out)[p] = g;
    return;
  }
  optimizer_elem(a.opt, f.xv, g, f.mu, f.v, f.d, a.g1, a.g2, a.eta, a.lr, sbc);
  if (a.support && !in) f.xv = czero<T>();
  static_cast<cx<T>*>(a.P_out)[p] = f.xv;
  static_cast<cx<T>*>(a.mu)[p] = f.mu;
  a.v[p] = f.v;
  static_cast<T*>(a.delta)[p] = f.d;
}

template <class T>
__device__ __forceinline__ void pupil_update_body(const PupilArgs& a, const double* sbc, int p) {
  PupilPre<T> f;
  pupil_prefetch<T>(a, p, f);
  pupil_finish<T>(a, sbc, p, f);
}

// Eq. 19 on pupil pixel p with its summed gradient g (zero off the support), or the
// gradient itself; the same arithmetic as pupil_finish.
template <class T>
__device__ __forceinline__ void pupil_update_g(const PupilArgs& a, const double* sbc, int p, cx<T> g) {
  const int n = a.n_lo, y = p / n, x = p % n;
  const bool in = x >= a.xlo[y] && x <= a.xhi[y];
  if (!in) g = czero<T>();
  if (!a.step) {
    static_cast<cx<T>*>(a.g_out)[p] = g;
    return;
  }
  cx<T> xv = a.filter ? static_cast<const cx<T>*>(a.Pf)[p] : static_cast<const cx<T>*>(a.P)[p];
  cx<T> mu = static_cast<const cx<T>*>(a.mu)[p];
  double v = a.v[p];
  T d = static_cast<const T*>(a.delta)[p];
  optimizer_elem(a.opt, xv, g, mu, v, d, a.g1, a.g2, a.eta, a.lr, sbc);
  if (a.support && !in) xv = czero<T>();
  static_cast<cx<T>*>(a.P_out)[p] = xv;
  static_cast<cx<T>*>(a.mu)[p] = mu;
  a.v[p] = v;
  static_cast<T*>(a.delta)[p] = d;
}

// ---------------------------------------------------------------------------
// Automatic penalty weight, Eq. (16) / (17): per LED, the FP64 sum over the
// (n-2)^2 positions where the 3x3 mask fits of |mask (x) g(I_k)|, with the mask
// rows [-1 2 -1], [-2 4 -2], [-1 2 -1] and g the plan's scaling (the identity for
// Eq. 16, sqrt for Eq. 17).
// ---------------------------------------------------------------------------
__device__ __forceinline__ double scaled_reading(double x, int fid, double gam) {
  if (fid == 1) return x;
  const double xp = x > 0.0 ? x : 0.0;
  if (fid == 0) return sqrt(xp);
  if (fid == 2) return pow(xp, gam);
  return log1p(xp);
}

template <class T>
__global__ __launch_bounds__(256) void k_auto_penalty(const T* meas, int n, int fid, double gam, double* part) {
  __shared__ double red[4];
  const int k = blockIdx.x;
  const T* I = meas + (size_t)k * n * n;
  const int m = n - 2;
  double acc = 0.0;
  for (int p = threadIdx.x; p < m * m; p += 256) {
    const int y = p / m, x = p % m;
    double c = 0.0;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        const double w = (j == 1 ? 2.0 : -1.0) * (i == 1 ? 2.0 : 1.0);
        c += w * scaled_reading(double(I[(y + i) * n + x + j]), fid, gam);
      }
    acc += fabs(c);
  }
  const double tot = block_sum<256>(acc, red);
  if (threadIdx.x == 0) part[k] = tot;
}

// ---------------------------------------------------------------------------
// Small utilities.
// ---------------------------------------------------------------------------
template <class E>
__global__ void k_fill(E* p, E val, size_t n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = val;
}

// out[y][x] = (-1)^(x+y) * s * in[y][x]
template <class T>
__global__ void k_sign_scale(const cx<T>* in, cx<T>* out, int n, T s) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (size_t)n * n) return;
  const int y = int(i / n), x = int(i % n);
  out[i] = scale(in[i], ((x + y) & 1) ? -s : s);
}

// Pupil of the initial state: 1 on the support, 0 elsewhere.
template <class T>
__global__ void k_init_pupil(cx<T>* P, const int* xlo, const int* xhi, int n) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n * n) return;
  const int y = p / n, x = p % n;
  P[p] = (x >= xlo[y] && x <= xhi[y]) ? cx<T>{T(1), T(0)} : czero<T>();
}

// Initial spectrum window: (r / n) * fftshift(fft2(sqrt(I_c))) on the support of
// the on-axis LED's window; fftshift after a DFT = (-1)^(x+y) before it.
template <class T, int N>
__global__ __launch_bounds__(LedShape<N>::NT) void k_init_window(const T* meas_c, cx<T>* psi, int y0, int x0,
                                                                 int n_hi, T sc, const int* xlo, const int* xhi,
                                                                 const cx<T>* tw) {
  using Sh = LedShape<N>;
  constexpr int NT = Sh::NT, R1 = Sh::R1, R2 = Sh::R2, PITCH = N + 1;
  constexpr int MB1 = ceil_div(N * (N / R1), NT);
  constexpr int MB2 = ceil_div(N * (N / R2), NT);
  using P1fR = StockhamPass<T, N, R1, 1, false, NT, MB1, PITCH, 1, N>;
  using P2fR = StockhamPass<T, N, R2, R1, false, NT, MB2, PITCH, 1, N>;
  using P1fC = StockhamPass<T, N, R1, 1, false, NT, MB1, 1, PITCH, N>;
  using P2fC = StockhamPass<T, N, R2, R1, false, NT, MB2, 1, PITCH, N>;
  __shared__ cx<T> img[N * PITCH];
  __shared__ cx<T> twl[N];
  const int tid = threadIdx.x;
  for (int i = tid; i < N; i += NT) twl[i] = tw[i];
  for (int p = tid; p < N * N; p += NT) {
    const int y = p / N, x = p % N;
    const T m = meas_c[p];
    const T s = sqrt(m > T(0) ? m : T(0));
    img[y * PITCH + x] = cx<T>{((x + y) & 1) ? -s : s, T(0)};
  }
  __syncthreads();
  P1fR::run(img, 0, N, twl, tid);
  P2fR::run(img, 0, N, twl, tid);
  P1fC::run(img, 0, N, twl, tid);
  int mm[MB2], jj[MB2];
  bool lv[MB2];
  P2fC::coords(N, tid, mm, jj, lv);
  cx<T> Y[MB2][R2];
  P2fC::load(img, 0, mm, jj, lv, twl, Y);
#pragma unroll
  for (int i = 0; i < MB2; ++i) {
    if (lv[i]) {
      const int j = jj[i], x = mm[i];
#pragma unroll
      for (int r = 0; r < R2; ++r) {
        const int y = j + r * R1;
        if (x >= xlo[y] && x <= xhi[y]) psi[(size_t)(y0 + y) * n_hi + x0 + x] = scale(Y[i][r], sc);
      }
    }
  }
}

}  // namespace elfpie
