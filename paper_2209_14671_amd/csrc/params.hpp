// Kernel argument blocks shared by the host launcher and the device kernels.
#pragma once

#include <cstdint>

namespace elfpie {

// Width of the column segments of the row-form update's contribution lists: a wave's 64
// pixels of one row span four of them, one per 16-lane quarter.
constexpr int kUpdSegW = 16;

enum LedMode : int {
  LED_GRAD = 1,     // residual, W and the back-projected contributions C, D
  LED_FIELDS = 2,   // write the complex low-resolution fields
  LED_INTENS = 4,   // write |o|^2
  LED_LOSS = 8,     // fidelity loss partial per LED
  LED_STORED = 16   // read the fields (as written by LED_FIELDS) instead of recomputing them
};

// The object branch riding in the per-LED launch: the last nblk blocks of the launch
// each take a wide column strip of the n_hi x n_hi object (the work of k_obj_strip:
// column inverse DFT, Hessian penalties and their gradient, column forward DFT) on the
// compute units that the LED blocks leave free.
struct LedObjArgs {
  const void* T1;       // inverse row transforms of Psi (n_hi x n_hi complex)
  void* T2;             // out: the Hessian-term gradient after its column transforms
  const void* tw;       // n_hi forward twiddles exp(-2 pi i k / n_hi)
  double* partial;      // 2 doubles per object block: sum rho(H|O|), sum rho(H angle O)
  double inv_n;
  double alpha, beta, eta_h, eps;
  int norm;
  int nblk;             // object blocks (0: none)
  // the 3 x 3 Gaussian pre-filter of the pupil (Algorithm 1), taken by the LED blocks in
  // slices while P (LedArgs::P) is read-only, for the pupil update that completes in the
  // update launch
  void* Pf;             // out: the pre-filtered pupil (NULL: not needed)
  double w_c, w_e, w_k; // Gaussian weights: centre, edge, corner
};

struct LedArgs {
  const void* psi;      // n_hi x n_hi complex
  const void* P;        // n_lo x n_lo complex
  const void* meas;     // K x n_lo x n_lo real
  void* C;              // K x S complex: conj(P) Y_k on the support (spectrum gradient part)
  void* D;              // K x S complex: conj(M_k Psi) Y_k on the support (pupil gradient part)
  void* fields;         // K x n_lo x n_lo complex (optional; input in LED_STORED mode)
  void* intens;         // K x n_lo x n_lo real (optional)
  double* fid_partial;  // K doubles
  const int* win;       // K x 2: (row y0, column x0) of each window
  const int* xlo;       // n_lo: first support column of each row
  const int* xhi;       // n_lo: last support column (xlo - 1 for an empty row)
  const int* rowoff;    // n_lo: support index of (y, xlo[y])
  const void* tw;       // n_lo complex forward twiddles exp(-2 pi i k / n_lo)
  int n_hi;
  int S;
  int y_min, y_max;     // rows holding support pixels
  int x_min, x_max;     // columns holding support pixels
  double inv_scale;     // 1 / (r n_lo)
  double eps;           // L1 smoothing
  int mode;
  int fidelity;         // ELFPIE_FID_*: the scaling g of the residual
  int norm;
  double fid_gamma;     // exponent of g(x) = x^gamma
  long long* t_bump;    // step counter, advanced once by block 0 in step mode (else NULL)
  int mux;              // LEDs per image (Eq. 1's M); block b serves LEDs b M .. b M + M - 1
  LedObjArgs obj;       // object blocks of the launch (instantiations with the object role)
};

struct HessArgs {
  const void* Ot;       // unnormalised inverse DFT of Psi (n x n complex), no centring sign
  void* Gt;             // out: (-1)^(x+y) G / n, ready for an unnormalised forward DFT
  double* partial;      // 2 doubles per 16 x 16 tile: sum rho(H|O|), sum rho(H angle O)
  int n;
  double inv_n;
  double alpha, beta, eta_h, eps;
  int norm;
  int want_grad;
};

struct UpdArgs {
  void* x;              // parameter (psi), updated in place in step mode
  void* mu;
  double* v;
  void* delta;
  void* g_out;          // gradient output in gradient mode
  const void* gH;       // n_hi^2 complex gradient of the Hessian terms
  const void* C;        // K x S
  const int* win;
  const int* xlo;
  const int* xhi;
  const int* rowoff;
  const int* tile_ptr;  // CSR over 16 x 16 tiles of the spectrum -> LEDs covering them
  const int* tile_led;  // entries as (LED, window row, window column) triples
  const long long* t;   // step counter, already advanced for this iteration
  int n_hi, n_lo, S, ntiles_x, ntiles;
  double g1, g2, eta;
  double lg1, lg2;      // log2(g1), log2(g2) (-inf for 0): the bias corrections
  double lr;            // step size of the moment methods and SGD
  int opt;              // ELFPIE_OPT_*
  int step;             // 0: write g_out; 1: update with the plan's rule
  int pupil_blocks;     // trailing blocks that run the pupil partial sums / pre-filter
  // the row form (k_update_rows): whole rows per block, row transforms folded in
  const void* tw;       // n_hi forward twiddles
  void* T1;             // out (inv): unnormalised inverse row DFT of psi after this call
  const int* seg_ptr;   // CSR over (row, kUpdSegW-column segment) of the spectrum
  const int* seg_ent;   // entries of 2 ints (8-byte aligned): C index base (index = base +
                        // column), first column | last column << 16; ascending LED order per
                        // segment
  int nseg;             // segments per row (n_hi / kUpdSegW)
  int inv;              // 1: write T1
};

struct FinArgs {
  const double* fid_partial;
  int K;
  const double* hess_partial;
  int ntiles;
  double alpha, beta;
  double* loss4;        // optional
  double* hist;         // optional, indexed by *ctr
  int* ctr;
  int* flag;            // set to 1 when the total loss is not finite
};

struct PupilArgs {
  const void* P;        // current pupil (n_lo^2 complex)
  void* P_out;          // updated pupil (state) in step mode
  const void* Pf;       // pre-filtered pupil (workspace)
  void* Pf_out;
  const void* D;        // K x S
  void* part;           // nch x n_lo^2 complex partial sums on the pupil grid (zero off the support)
  const int* s2p;       // support index -> pupil pixel index
  void* g_out;          // gradient output (gradient mode)
  void* mu;
  double* v;
  void* delta;
  const int* xlo;
  const int* xhi;
  const int* rowoff;
  const long long* t;
  int n_lo, S, K, chunk, nch;
  double w_c, w_e, w_k;  // Gaussian weights: centre, edge, corner
  double g1, g2, eta;
  double lg1, lg2;      // log2(g1), log2(g2) (-inf for 0)
  double lr;
  int opt;
  int step;
  int filter;
  int support;
  // 1: the pupil update completes in the launch that sums the LED contributions, each
  // block taking some support pixels over every LED; further blocks take the pixels off
  // the support.  Pf then comes from the per-LED launch.
  int final_in_launch;
};

// End of an iteration: Eq. 19 on the pupil (or its gradient) and the loss reduction.
// Both read only what earlier launches wrote, so their blocks are independent and
// can ride in any later launch that leaves P, the loss partials and the counters alone.
struct TailArgs {
  PupilArgs pa;
  FinArgs fin;
  int pupil_blocks;     // blocks of the pupil update (0: none)
  int fin_block;        // 1: one more block reduces the loss
  int pupil_ppb;        // riding in the strip launch: pupil pixels per strip block (0: none)
  // the opening launch of a run (the row transforms, no tail riding along): its first
  // block clears the loss history slot counter and the non-finite flag (NULL: neither)
  int* zero_ctr;
  int* zero_flag;
};


}  // namespace elfpie
