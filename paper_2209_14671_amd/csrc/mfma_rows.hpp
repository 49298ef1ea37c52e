// Row transforms of the 256^2 per-LED tile as complex GEMMs on the gfx950 matrix cores,
// in split precision: every FP32 operand x is carried as a BF16 pair hi = bf16(x),
// lo = bf16(x - hi), and a product a b as hi_a hi_b + hi_a lo_b + lo_a hi_b, accumulated
// in FP32 (the lo_a lo_b term and the residuals below 2^-16 |x| are dropped, so each
// product carries a relative error of about 2^-16).
//
// The two transforms of Sec. 3.1 that act along the rows of the tile, as matrix products
// with the DFT matrix restricted to the pupil's support box (columns x_min .. x_max):
//   inverse  A[yb][x] = sum_u X[y][u] exp(+2 pi i u x / N),  u in the box      (F_B, Eq. 1)
//   forward  Y[yb][u] = sum_x B[yb][x] exp(-2 pi i u x / N), u in the box      (F_B^H, Eq. 9)
// for the band rows y = y_min + yb.  A and B have the layout of k_big_rows_inv's output
// and k_big_cols' output, so the column kernel between them is shared with the FFT form.
//
// Matrix-core operation: v_mfma_f32_16x16x32_bf16, D (16 x 16) += A (16 x 32) B (32 x 16)
// with, for lane l of the wave: A row l % 16, k = 8 (l / 16) .. + 7; B column l % 16, the
// same k; D column l % 16, rows 4 (l / 16) .. + 3.
// The data operand (left) is split and staged in LDS in that fragment order; the DFT
// operand (right) is a table in the workspace, split on the host from FP64 values, in
// the same order: fragment (k-step ks, n-tile nt, component c) at
// ((ks * ntiles + nt) * 4 + c) * 64 + lane (16-byte units), components re_hi, re_lo,
// im_hi, im_lo.  Complex products: re = Xr Er + (-Xi) Ei, im = Xr Ei + Xi Er.
#pragma once

#include "kernels.hpp"

namespace elfpie {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4;

struct MfmaTabs {
  const bf16x8* inv;  // inverse-row table: k = u - x_min (ksi k-steps), n = x (nti n-tiles)
  const bf16x8* fwd;  // forward-row table: k = x (ksf k-steps), n = u - x_min (ntf n-tiles)
  int ksi, nti, ksf, ntf;
};

// Components of a staged data fragment: Xr hi/lo, Xi hi/lo, -Xi hi/lo.
enum { XR_HI = 0, XR_LO, XI_HI, XI_LO, NXI_HI, NXI_LO, NXC };
enum { ER_HI = 0, ER_LO, EI_HI, EI_LO, NEC };

__device__ __forceinline__ void bf16_split(float x, __bf16& hi, __bf16& lo) {
  hi = (__bf16)x;
  lo = (__bf16)(x - (float)hi);
}

// Stage 8 consecutive k values (one lane's slice) of data row m into the fragment
// buffer: frags[((mt * ks_n + ks) * NXC + c) * 64 + lane], lane = m % 16 + 16 ((k % 32) / 8).
__device__ __forceinline__ void stage_slice(bf16x8* frags, int ks_n, int m, int k0, const cx<float> (&v)[8]) {
  bf16x8 f[NXC];
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    __bf16 h, l;
    bf16_split(v[i].x, h, l);
    f[XR_HI][i] = h;
    f[XR_LO][i] = l;
    bf16_split(v[i].y, h, l);
    f[XI_HI][i] = h;
    f[XI_LO][i] = l;
    f[NXI_HI][i] = -h;  // negation is exact in BF16
    f[NXI_LO][i] = -l;
  }
  const int mt = m / 16, ks = k0 / 32, lane = m % 16 + 16 * ((k0 % 32) / 8);
  bf16x8* dst = frags + ((size_t)(mt * ks_n + ks) * NXC) * 64 + lane;
#pragma unroll
  for (int c = 0; c < NXC; ++c) dst[c * 64] = f[c];
}

// One wave: the 32 x 32 complex output block (m-tiles 0, 1 of the staged data; n-tiles
// nt0, nt0 + 1 of the table, the second skipped when nt0 + 1 >= ntiles) over ks_n k-steps.
__device__ __forceinline__ void mfma_block(const bf16x8* frags, const bf16x8* tab, int ks_n, int ntiles, int nt0,
                                           f32x4 (&acc_r)[2][2], f32x4 (&acc_i)[2][2]) {
  const int lane = threadIdx.x & 63;
  const bool two = nt0 + 1 < ntiles;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      acc_r[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
      acc_i[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
    }
  for (int ks = 0; ks < ks_n; ++ks) {
    bf16x8 A[2][NXC], B[2][NEC];
#pragma unroll
    for (int mt = 0; mt < 2; ++mt)
#pragma unroll
      for (int c = 0; c < NXC; ++c) A[mt][c] = frags[((size_t)(mt * ks_n + ks) * NXC + c) * 64 + lane];
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      const int nt = two ? nt0 + t : nt0;  // a lone last tile is computed twice, stored once
#pragma unroll
      for (int c = 0; c < NEC; ++c) B[t][c] = tab[((size_t)(ks * ntiles + nt) * NEC + c) * 64 + lane];
    }
#pragma unroll
    for (int mt = 0; mt < 2; ++mt)
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        f32x4 r = acc_r[mt][t], im = acc_i[mt][t];
        r = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[mt][XR_HI], B[t][ER_HI], r, 0, 0, 0);
        im = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[mt][XR_HI], B[t][EI_HI], im, 0, 0, 0);
        r = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[mt][NXI_HI], B[t][EI_HI], r, 0, 0, 0);
        im = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[mt][XI_HI], B[t][ER_HI], im, 0, 0, 0);
        r = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[mt][XR_HI], B[t][ER_LO], r, 0, 0, 0);
        im = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[mt][XR_HI], B[t][EI_LO], im, 0, 0, 0);
        r = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[mt][NXI_HI], B[t][EI_LO], r, 0, 0, 0);
        im = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[mt][XI_HI], B[t][ER_LO], im, 0, 0, 0);
        r = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[mt][XR_LO], B[t][ER_HI], r, 0, 0, 0);
        im = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[mt][XR_LO], B[t][EI_HI], im, 0, 0, 0);
        r = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[mt][NXI_LO], B[t][EI_HI], r, 0, 0, 0);
        im = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[mt][XI_LO], B[t][ER_HI], im, 0, 0, 0);
        acc_r[mt][t] = r;
        acc_i[mt][t] = im;
      }
  }
}

template <int N> struct MfmaRows {
  static constexpr int MB = 32;               // band rows per block (two m-tiles)
  static constexpr int NTI = 256;             // threads of the inverse rows: N / 32 waves
  static constexpr int KSF = N / 32;          // k-steps of the forward rows
  static constexpr int KSI_MAX = N / 32;      // k-steps of the inverse rows, at most
  static constexpr int NTF_MAX = N / 16;      // n-tiles of the forward rows, at most
};

// Inverse rows: block (m-group g, LED k) stages X rows yb = 32 g .. 32 g + 31 of LED k
// (zero off the support and past the band) and writes A[k][yb][x] for every x.
// 8 waves, wave w: n-tiles 2 w, 2 w + 1 (N = 256).
template <int N>
__global__ __launch_bounds__(512) void k_mfma_rows_inv(LedArgs a, MfmaTabs t, cx<float>* A) {
  constexpr int MB = MfmaRows<N>::MB;
  __shared__ bf16x8 frags[2 * MfmaRows<N>::KSI_MAX * NXC * 64];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int L = xcd_order(blockIdx.y * gridDim.x + blockIdx.x, gridDim.x * gridDim.y);
  const int k = L / gridDim.x, g = L % gridDim.x;
  const int nband = a.y_max - a.y_min + 1, box = a.x_max - a.x_min + 1, ks_n = t.ksi;
  const cx<float>* P = static_cast<const cx<float>*>(a.P);
  const cx<float>* win = static_cast<const cx<float>*>(a.psi) + (size_t)a.win[2 * k] * a.n_hi + a.win[2 * k + 1];
  // stage: (row m, slice of 8 k) items
  const int nslice = ks_n * 4;
  for (int p = tid; p < MB * nslice; p += blockDim.x) {
    const int m = p / nslice, k0 = (p % nslice) * 8, yb = g * MB + m, y = a.y_min + yb;
    cx<float> v[8];
    const bool row = yb < nband;
    const int lo = row ? a.xlo[y] : 1, hi = row ? a.xhi[y] : 0;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int u = a.x_min + k0 + i;
      v[i] = czero<float>();
      if (k0 + i < box && u >= lo && u <= hi) v[i] = P[y * N + u] * win[(size_t)y * a.n_hi + u];
    }
    stage_slice(frags, ks_n, m, k0, v);
  }
  __syncthreads();
  f32x4 acc_r[2][2], acc_i[2][2];
  const int nt0 = 2 * wave;
  if (nt0 >= t.nti) return;
  mfma_block(frags, t.inv, ks_n, t.nti, nt0, acc_r, acc_i);
  cx<float>* Ak = A + (size_t)k * nband * N;
#pragma unroll
  for (int mt = 0; mt < 2; ++mt)
#pragma unroll
    for (int tt = 0; tt < 2; ++tt) {
      const int x = (nt0 + tt) * 16 + lane % 16;
      if (nt0 + tt >= t.nti) continue;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int yb = g * MB + mt * 16 + 4 * (lane / 16) + i;
        if (yb < nband) Ak[(size_t)yb * N + x] = cx<float>{acc_r[mt][tt][i], acc_i[mt][tt][i]};
      }
    }
}

// Forward rows: block (m-group g, LED k) stages B rows yb = 32 g .. 32 g + 31 of LED k and
// forms Y[yb][u] for u in the box, then the contributions C = conj(P) Y and
// D = conj(M_k Psi) Y on the support (Eq. 9, Eq. 18), Y scaled by 1 / (r n_lo).
// ceil(ntf / 2) waves, wave w: n-tiles 2 w, 2 w + 1.
template <int N>
__global__ __launch_bounds__(512) void k_mfma_rows_fwd(LedArgs a, MfmaTabs t, const cx<float>* B) {
  constexpr int MB = MfmaRows<N>::MB, KS = MfmaRows<N>::KSF;
  __shared__ bf16x8 frags[2 * KS * NXC * 64];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int L = xcd_order(blockIdx.y * gridDim.x + blockIdx.x, gridDim.x * gridDim.y);
  const int k = L / gridDim.x, g = L % gridDim.x;
  const int nband = a.y_max - a.y_min + 1;
  const cx<float>* Bk = B + (size_t)k * nband * N;
  constexpr int nslice = KS * 4;
  for (int p = tid; p < MB * nslice; p += blockDim.x) {
    const int m = p / nslice, k0 = (p % nslice) * 8, yb = g * MB + m;
    cx<float> v[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) v[i] = yb < nband ? Bk[(size_t)yb * N + k0 + i] : czero<float>();
    stage_slice(frags, KS, m, k0, v);
  }
  __syncthreads();
  f32x4 acc_r[2][2], acc_i[2][2];
  const int nt0 = 2 * wave;
  if (nt0 >= t.ntf) return;
  mfma_block(frags, t.fwd, KS, t.ntf, nt0, acc_r, acc_i);
  const float sc = float(a.inv_scale);
  const cx<float>* P = static_cast<const cx<float>*>(a.P);
  const cx<float>* win = static_cast<const cx<float>*>(a.psi) + (size_t)a.win[2 * k] * a.n_hi + a.win[2 * k + 1];
  cx<float>* C = static_cast<cx<float>*>(a.C) + (size_t)k * a.S;
  cx<float>* D = static_cast<cx<float>*>(a.D) + (size_t)k * a.S;
#pragma unroll
  for (int mt = 0; mt < 2; ++mt)
#pragma unroll
    for (int tt = 0; tt < 2; ++tt) {
      if (nt0 + tt >= t.ntf) continue;
      const int u = a.x_min + (nt0 + tt) * 16 + lane % 16;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int yb = g * MB + mt * 16 + 4 * (lane / 16) + i, y = a.y_min + yb;
        if (yb >= nband) continue;
        const int lo = a.xlo[y];
        if (u < lo || u > a.xhi[y]) continue;
        const int s = a.rowoff[y] + u - lo;
        const cx<float> yv = cx<float>{acc_r[mt][tt][i] * sc, acc_i[mt][tt][i] * sc};
        C[s] = cmulc(P[y * N + u], yv);
        D[s] = cmulc(win[(size_t)y * a.n_hi + u], yv);
      }
    }
}

}  // namespace elfpie
