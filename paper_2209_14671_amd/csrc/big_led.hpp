// Per-LED branch for low-resolution tiles too large for one workgroup's LDS
// (n_lo = 256: a 256^2 complex FP32 tile is 512 KB).  The same computation as
// k_led (Eq. 1, 4/5 and the Sec. 6.3 scalings, 9-12, 18), split into three launches
// that pass the tile through plan scratch in HBM:
//   k_big_rows_inv   gather X = P * M_k Psi on the support, inverse DFT of the rows
//                    that hold support pixels                -> A (band rows only)
//   k_big_cols       per strip of W columns (+1 halo column each side): inverse DFT of
//                    the columns, o, residual, features, omega, loss, dL/d(conj o) on
//                    the own columns, forward DFT of those columns -> B (band rows only)
//   k_big_rows_fwd   forward DFT of the band rows of B, contributions C = conj(P) Y and
//                    D = conj(M_k Psi) Y on the support
// Each LED is independent; blocks are (line group, LED).  As in k_led, the centring
// shifts cancel between the inverse and the forward transform (W is o times a real
// field), so no (-1)^(x+y) factor appears except where fields are written or read.
#pragma once

#include "kernels.hpp"

namespace elfpie {

template <int N> struct BigLed;
#ifndef ELFPIE_BIG_RB
#define ELFPIE_BIG_RB 8
#define ELFPIE_BIG_RNT 256
#define ELFPIE_BIG_W 16
#define ELFPIE_BIG_CNT 512
#endif
template <> struct BigLed<256> {
  static constexpr int RB = ELFPIE_BIG_RB;    // rows per block of the row transforms
  static constexpr int RNT = ELFPIE_BIG_RNT;  // threads of the row transforms
  static constexpr int W = ELFPIE_BIG_W;      // own columns per block of the column kernel
  static constexpr int CNT = ELFPIE_BIG_CNT;  // threads of the column kernel
};
template <> struct BigLed<192> {
  static constexpr int RB = 8, RNT = 256, W = 16, CNT = 512;
};
#ifndef ELFPIE_BIG_XCD
#define ELFPIE_BIG_XCD 1  // XCD-aware workgroup order in the column kernel
#endif
#ifndef ELFPIE_BIGROW_XCD
#define ELFPIE_BIGROW_XCD 1  // and in the row kernels
#endif
#ifndef ELFPIE_BIG_TSUM
#define ELFPIE_BIG_TSUM 1
#endif

// A: K x nband x N (band row yb = y - y_min), unnormalised inverse DFT of the rows.
template <class T, int N>
__global__ __launch_bounds__(BigLed<N>::RNT) void k_big_rows_inv(LedArgs a, cx<T>* A) {
  using Sh = BigLed<N>;
  constexpr int RB = Sh::RB, NT = Sh::RNT, PITCH = N + 1;
  __shared__ cx<T> buf[RB * PITCH];
  __shared__ cx<T> twl[N];
  const int tid = threadIdx.x;
  // runs of neighbouring LEDs per XCD (overlapping spectrum windows share its L2)
  const int L = ELFPIE_BIGROW_XCD ? xcd_order(blockIdx.y * gridDim.x + blockIdx.x, gridDim.x * gridDim.y)
                               : (int)(blockIdx.y * gridDim.x + blockIdx.x);
  const int k = L / gridDim.x;
  const int nband = a.y_max - a.y_min + 1;
  const int yb0 = (L % gridDim.x) * RB;
  for (int i = tid; i < N; i += NT) twl[i] = static_cast<const cx<T>*>(a.tw)[i];
  const cx<T>* P = static_cast<const cx<T>*>(a.P);
  const cx<T>* win = static_cast<const cx<T>*>(a.psi) + (size_t)a.win[2 * k] * a.n_hi + a.win[2 * k + 1];
  for (int p = tid; p < RB * N; p += NT) {
    const int l = p / N, x = p % N, yb = yb0 + l, y = a.y_min + yb;
    cx<T> v = czero<T>();
    if (yb < nband && x >= a.xlo[y] && x <= a.xhi[y]) v = P[y * N + x] * win[(size_t)y * a.n_hi + x];
    buf[l * PITCH + x] = v;
  }
  __syncthreads();
  fft_lines_inplace<T, N, true, NT, RB>(buf, twl, tid);
  cx<T>* Ak = A + (size_t)k * nband * N;
  for (int p = tid; p < RB * N; p += NT) {
    const int l = p / N, x = p % N, yb = yb0 + l;
    if (yb < nband) Ak[(size_t)yb * N + x] = buf[l * PITCH + x];
  }
}

// Strip s of LED k: own columns c0 .. c0 + W - 1, lines l = 0 .. W + 1 hold columns
// c0 - 1 + l.  Writes B (K x nband x N) and the loss partial of its own pixels to
// fid_partial[k * nstrip + s].
template <class T, int N, bool SCALED>
__global__ __launch_bounds__(BigLed<N>::CNT) void k_big_cols(LedArgs a, const cx<T>* A, cx<T>* B) {
  using Sh = BigLed<N>;
  constexpr int W = Sh::W, NT = Sh::CNT, NL = W + 2, PITCH = N + 1, EP = NL + 1;
  constexpr int NSTRIP = N / W;
  __shared__ cx<T> buf[NL * PITCH];  // line l at l * PITCH, element = row y
  __shared__ T eb[N * EP];           // residual, row-major (row y at y * EP): the loops below
                                     // give consecutive lanes consecutive lines
  __shared__ cx<T> twl[N];
  __shared__ double red[NT / 64];
  const int tid = threadIdx.x;
  // Workgroups go to the 8 XCDs in turn (linear id modulo 8), so workgroup b is
  // renumbered so that each XCD runs whole LEDs: the neighbouring strips of an LED read
  // overlapping column segments of A and the measured image, which then share that
  // XCD's L2 instead of being fetched once per XCD.
  int b = blockIdx.y * NSTRIP + blockIdx.x;
  const int nblk = gridDim.y * NSTRIP;
  if (ELFPIE_BIG_XCD && nblk % 8 == 0) b = (b % 8) * (nblk / 8) + b / 8;
  const int s = b % NSTRIP, k = b / NSTRIP;
  const int c0 = s * W;
  const int nband = a.y_max - a.y_min + 1;
  const int mode = a.mode;
  const bool stored = (mode & LED_STORED) != 0;
  led_bump_step(a, s == 0 ? k : 1, tid);  // once per launch: block (0, 0)
  for (int i = tid; i < N; i += NT) twl[i] = static_cast<const cx<T>*>(a.tw)[i];
  const T sc = T(a.inv_scale);
  if (stored) {
    // o from the caller's fields (true frame) into the kernel frame, already scaled
    const cx<T>* Fk = static_cast<const cx<T>*>(a.fields) + (size_t)k * N * N;
    for (int p = tid; p < NL * N; p += NT) {
      const int y = p / NL, l = p % NL, c = c0 - 1 + l;
      cx<T> v = czero<T>();
      if (c >= 0 && c < N) {
        v = Fk[(size_t)y * N + c];
        if ((c + y) & 1) v = cx<T>{-v.x, -v.y};
      }
      buf[l * PITCH + y] = v;
    }
    __syncthreads();
  } else {
    const cx<T>* Ak = A + (size_t)k * nband * N;
    for (int p = tid; p < NL * N; p += NT) {
      const int y = p / NL, l = p % NL, c = c0 - 1 + l, yb = y - a.y_min;
      cx<T> v = czero<T>();
      if (c >= 0 && c < N && yb >= 0 && yb < nband) v = Ak[(size_t)yb * N + c];
      buf[l * PITCH + y] = v;
    }
    __syncthreads();
    fft_lines_inplace<T, N, true, NT, NL>(buf, twl, tid);  // scaled by sc below
  }
  const T gam = T(a.fid_gamma), eps = T(a.eps);
  // the measured stack is read only when the loss or its gradient is wanted: the
  // forward model alone (fields, images) is called without one
  const bool need_e = (mode & (LED_GRAD | LED_LOSS)) != 0;
  const T* meas = need_e ? static_cast<const T*>(a.meas) + (size_t)k * N * N : nullptr;
  // the gradient and loss modes under the amplitude or intensity fidelity: the same
  // residual with the fidelity fixed outside the loop and no output stores to test
  auto residual_only = [&](auto amp_c) {
    constexpr bool AMP = decltype(amp_c)::value;
    for (int p = tid; p < NL * N; p += NT) {
      const int y = p / NL, l = p % NL, c = c0 - 1 + l;
      cx<T> ov = buf[l * PITCH + y];
      if (!stored) {
        ov = scale(ov, sc);
        buf[l * PITCH + y] = ov;
      }
      const T i2 = norm2(ov);
      const bool in = c >= 0 && c < N;
      eb[y * EP + l] = in ? fid_residual<false>(AMP ? 0 : 1, i2, meas[(size_t)y * N + c], gam) : T(0);
    }
  };
  if (!SCALED && need_e && !(mode & (LED_FIELDS | LED_INTENS))) {
    if (a.fidelity == 0) residual_only(std::true_type{});
    else residual_only(std::false_type{});
  } else {
    for (int p = tid; p < NL * N; p += NT) {
      const int y = p / NL, l = p % NL, c = c0 - 1 + l;
      cx<T> ov = buf[l * PITCH + y];
      if (!stored) {
        ov = scale(ov, sc);
        buf[l * PITCH + y] = ov;  // o itself, for the Wirtinger factor below
      }
      const T i2 = norm2(ov);
      const bool in = c >= 0 && c < N;
      if (in && l >= 1 && l <= W) {
        const size_t pix = (size_t)k * N * N + (size_t)y * N + c;
        if (mode & LED_FIELDS) static_cast<cx<T>*>(a.fields)[pix] = ((c + y) & 1) ? cx<T>{-ov.x, -ov.y} : ov;
        if (mode & LED_INTENS) static_cast<T*>(a.intens)[pix] = i2;
      }
      if (need_e) eb[y * EP + l] = in ? fid_residual<SCALED>(a.fidelity, i2, meas[(size_t)y * N + c], gam) : T(0);
    }
  }
  if (!need_e) return;
  __syncthreads();

  // features on the own columns: q = grad^T omega needs e one column to each side
  auto E = [&](int l, int y) -> T { return eb[y * EP + l]; };
  double lsum = 0.0;
  if (!SCALED && a.norm == 0 && !(eps > T(0))) {
    // the exact anisotropic L1 (omega = sign, rho = |.|) under the intensity or amplitude
    // fidelity, without a branch per pixel (the same arithmetic as the general loop)
    const bool amp = a.fidelity == 0;
    auto sgn = [](T d) { return sign_unit(d); };
    T lpart = T(0);  // this lane's pixels, summed in T and added to the FP64 partial once
    for (int p = tid; p < W * N; p += NT) {
      const int y = p / W, l = 1 + p % W, x = c0 - 1 + l;
      const int yd = min(y + 1, N - 1), yu = max(y - 1, 0);
      const T e = E(l, y), er = E(l + 1, y), ed = E(l, yd), el = E(l - 1, y), eu = E(l, yu);
      const T dx0 = (x < N - 1) ? er - e : T(0);
      const T dy0 = (y < N - 1) ? ed - e : T(0);
      const T dxm = (x > 0) ? e - el : T(0);
      const T dym = (y > 0) ? e - eu : T(0);
      const T q = sgn(dxm) - sgn(dx0) + sgn(dym) - sgn(dy0);
      if (ELFPIE_BIG_TSUM) lpart += fabs(dx0) + fabs(dy0);
      else lsum += double(fabs(dx0) + fabs(dy0));
      const cx<T> ov = buf[l * PITCH + y];
      const T i2 = norm2(ov);
      const T fa = i2 > T(0) ? T(0.5) * q * rsqrt_t(i2) : T(0);
      buf[l * PITCH + y] = scale(ov, amp ? fa : q);
    }
    lsum += double(lpart);
  } else
  for (int p = tid; p < W * N; p += NT) {
    const int y = p / W, l = 1 + p % W, x = c0 - 1 + l;
    const T e = E(l, y);
    const T dx0 = (x < N - 1) ? E(l + 1, y) - e : T(0);
    const T dy0 = (y < N - 1) ? E(l, y + 1) - e : T(0);
    T q;
    if (a.norm == 0) {
      const T dxm = (x > 0) ? e - E(l - 1, y) : T(0);
      const T dym = (y > 0) ? e - E(l, y - 1) : T(0);
      q = omega(dxm, eps) - omega(dx0, eps) + omega(dym, eps) - omega(dy0, eps);
      lsum += double(rho(dx0, eps) + rho(dy0, eps));
    } else {
      const T s0 = dx0 * dx0 + dy0 * dy0;
      q = -(dx0 + dy0) * inv_norm(s0, eps);
      if (x > 0) {
        const T el = E(l - 1, y);
        const T gx = e - el;
        const T gy = (y < N - 1) ? E(l - 1, y + 1) - el : T(0);
        q += gx * inv_norm(gx * gx + gy * gy, eps);
      }
      if (y > 0) {
        const T eu = E(l, y - 1);
        const T gy = e - eu;
        const T gx = (x < N - 1) ? E(l + 1, y - 1) - eu : T(0);
        q += gy * inv_norm(gx * gx + gy * gy, eps);
      }
      lsum += eps > T(0) ? double(sqrt_t(s0 + eps * eps) - eps) : double(sqrt_t(s0));
    }
    buf[l * PITCH + y] = fid_wirtinger<SCALED>(a.fidelity, buf[l * PITCH + y], q, gam);
  }
  const double tot = block_sum<NT>(lsum, red);  // contains barriers
  if (tid == 0) a.fid_partial[(size_t)k * NSTRIP + s] = tot;
  if (!(mode & LED_GRAD)) return;

  fft_lines_inplace<T, N, false, NT, W>(buf + PITCH, twl, tid);
  cx<T>* Bk = B + (size_t)k * nband * N;
  for (int p = tid; p < W * nband; p += NT) {
    const int yb = p / W, l = 1 + p % W;
    Bk[(size_t)yb * N + c0 - 1 + l] = buf[l * PITCH + a.y_min + yb];
  }
}

// Forward DFT of the band rows of B and the contributions on the support.
template <class T, int N>
__global__ __launch_bounds__(BigLed<N>::RNT) void k_big_rows_fwd(LedArgs a, const cx<T>* B) {
  using Sh = BigLed<N>;
  constexpr int RB = Sh::RB, NT = Sh::RNT, PITCH = N + 1;
  __shared__ cx<T> buf[RB * PITCH];
  __shared__ cx<T> twl[N];
  const int tid = threadIdx.x;
  // runs of neighbouring LEDs per XCD (overlapping spectrum windows share its L2)
  const int L = ELFPIE_BIGROW_XCD ? xcd_order(blockIdx.y * gridDim.x + blockIdx.x, gridDim.x * gridDim.y)
                               : (int)(blockIdx.y * gridDim.x + blockIdx.x);
  const int k = L / gridDim.x;
  const int nband = a.y_max - a.y_min + 1;
  const int yb0 = (L % gridDim.x) * RB;
  for (int i = tid; i < N; i += NT) twl[i] = static_cast<const cx<T>*>(a.tw)[i];
  const cx<T>* Bk = B + (size_t)k * nband * N;
  for (int p = tid; p < RB * N; p += NT) {
    const int l = p / N, x = p % N, yb = yb0 + l;
    buf[l * PITCH + x] = yb < nband ? Bk[(size_t)yb * N + x] : czero<T>();
  }
  __syncthreads();
  fft_lines_inplace<T, N, false, NT, RB>(buf, twl, tid);
  const T sc = T(a.inv_scale);
  const cx<T>* P = static_cast<const cx<T>*>(a.P);
  const cx<T>* win = static_cast<const cx<T>*>(a.psi) + (size_t)a.win[2 * k] * a.n_hi + a.win[2 * k + 1];
  cx<T>* C = static_cast<cx<T>*>(a.C) + (size_t)k * a.S;
  cx<T>* D = static_cast<cx<T>*>(a.D) + (size_t)k * a.S;
  for (int p = tid; p < RB * N; p += NT) {
    const int l = p / N, x = p % N, yb = yb0 + l, y = a.y_min + yb;
    if (yb >= nband) continue;
    const int lo = a.xlo[y];
    if (x < lo || x > a.xhi[y]) continue;
    const int s = a.rowoff[y] + x - lo;
    const cx<T> yv = scale(buf[l * PITCH + x], sc);
    C[s] = cmulc(P[y * N + x], yv);
    D[s] = cmulc(win[(size_t)y * a.n_hi + x], yv);
  }
}

}  // namespace elfpie

namespace elfpie {

// Initial state for the large tile: (r / n) fftshift(fft2(sqrt(I_c))) on the support of
// the on-axis window, through k_fft_lines.  fftshift after a DFT of even length is the
// (-1)^(x+y) modulation before it.
template <class T>
__global__ void k_init_big_prep(const T* meas_c, cx<T>* out, int n) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n * n) return;
  const int y = p / n, x = p % n;
  const T v = meas_c[p] > T(0) ? sqrt(meas_c[p]) : T(0);
  out[p] = cx<T>{((x + y) & 1) ? -v : v, T(0)};
}

template <class T>
__global__ void k_init_big_place(const cx<T>* spec, cx<T>* psi, int y0, int x0, int n_hi, int n, T sc,
                                 const int* xlo, const int* xhi) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n * n) return;
  const int y = p / n, x = p % n;
  if (x >= xlo[y] && x <= xhi[y]) psi[(size_t)(y0 + y) * n_hi + x0 + x] = scale(spec[p], sc);
}

}  // namespace elfpie
