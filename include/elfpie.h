/*
 * elfpie.h - C ABI of the MI355X (gfx950) Elfpie reconstruction library.
 *
 * Elfpie (Zhang, Berendschot, Zhou, arXiv 2209.14671) reconstructs the
 * high-resolution spectrum Psi of a sample, and the pupil P of the objective,
 * from a Fourier-ptychographic stack of K low-resolution intensity images
 * (Sec. 3, Algorithm 1).  One iteration, for all K LEDs at once:
 *   - crops each LED's window of Psi and applies the pupil, inverse-transforms
 *     it to a low-resolution field (Sec. 3.1, Eq. 1; M LEDs lit together per
 *     image, M = mux, the images summing their intensities);
 *   - evaluates the L1 data fidelity on image gradients (Eq. 4 or Eq. 5 with
 *     the normaliser of Eq. 12) and the Hessian penalties on the amplitude and
 *     phase of O = F_A Psi (Eq. 6, 7, combined by Eq. 8);
 *   - forms the closed-form Wirtinger gradients wrt conj(Psi) (Eq. 9-15) and
 *     conj(P) (Eq. 18);
 *   - applies the modified AdaBelief update (Eq. 19) to Psi and, optionally,
 *     to P after a 3x3 Gaussian pre-filter (note under Algorithm 1).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Arrays are dense, row-major (row = y, column = x), complex values stored
 * interleaved (re, im), in the precision of the plan: ELFPIE_F32 -> float /
 * complex64, ELFPIE_F64 -> double / complex128.  The AdaBelief second moments
 * v are always double.  Every array pointer is a DEVICE pointer allocated by
 * the caller, aligned to 16 bytes, unless stated "host".  The library never
 * allocates device memory: its workspace is handed in at plan creation and is
 * owned by the caller, who must keep it alive until elfpie_plan_destroy.
 *
 * Transforms are centred and unitary: Psi = fftshift(fft2(O)) / n_hi, so the
 * DC term sits at [n_hi/2, n_hi/2]; the low-resolution field of LED k is
 * o_k = (n_lo / r) * ifft2(ifftshift(P * crop_k(Psi))), r = n_hi / n_lo.
 * LED k's window is centred at n_hi/2 + round(k * FOV) (round half away from
 * zero; k = (kx, ky) in cycles per micrometre, FOV = n_lo * dx_lo).  The pupil
 * support is the disc |u - n_lo/2|^2 <= R^2 (1 + 1e-12), R = NA * FOV / lambda.
 *
 * Streams and errors: every call enqueues its work on `stream` (a hipStream_t;
 * NULL = the default stream) and returns without waiting, except where noted.
 * Argument errors are detected before anything is enqueued and are returned
 * synchronously; the reason is available from elfpie_last_error.  HIP runtime
 * failures return ELFPIE_E_DEVICE.  A plan is not thread-safe; distinct plans
 * are independent.  Results are bitwise reproducible for a given plan and
 * device: no floating-point atomics are used.
 */
#ifndef ELFPIE_H
#define ELFPIE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  ELFPIE_OK = 0,
  ELFPIE_E_INVALID = 1,      /* NULL or misaligned pointer, bad value              */
  ELFPIE_E_RANGE = 2,        /* an LED window falls outside the spectrum           */
  ELFPIE_E_UNSUPPORTED = 3,  /* size / precision combination not implemented      */
  ELFPIE_E_WORKSPACE = 4,    /* workspace smaller than elfpie_workspace_bytes      */
  ELFPIE_E_DEVICE = 5,       /* HIP runtime error                                  */
  ELFPIE_E_NONFINITE = 6     /* a checked run produced a NaN / Inf loss            */
} elfpie_status;

/* The scaling g of the data fidelity (Eq. 3): g(x) = sqrt(x) (Eq. 4), x (Eq. 5), and
 * the two Sec. 6.3 tries, x^gamma (gamma = fid_gamma) and ln(x + 1).  The residual
 * inside the gradient operator is g(|o|^2) - g(I) with negative readings of I taken
 * as 0 (except for g(x) = x); the gradient carries g'(|o|^2), taken as 0 at |o| = 0
 * for the powers. */
enum { ELFPIE_FID_AMPLITUDE = 0, ELFPIE_FID_INTENSITY = 1, ELFPIE_FID_GAMMA = 2, ELFPIE_FID_LOG = 3 };
enum { ELFPIE_NORM_ANISO = 0, ELFPIE_NORM_ISO = 1 };          /* Eq. 12        */
/* The update rule for Psi and P: Eq. 19 (delta^0 = lr^2), or the three rules the
 * paper compares it with (Sec. 6.2, Fig. 13), each with step size lr, decay rates
 * gamma1 / gamma2 and eps = eta_opt: plain gradient descent x -= lr g; NAdam
 * (Dozat 2016, constant momentum: x -= lr m^ / (sqrt(v^) + eps) with
 * m^ = gamma1 m_t / (1 - gamma1^(t+1)) + (1 - gamma1) g / (1 - gamma1^t)); AdaBelief
 * (Zhuang et al. 2020: second moment of (g - m) plus eps).  g = dL/d(conj x);
 * squared magnitudes are squared moduli. */
enum { ELFPIE_OPT_ELFPIE = 0, ELFPIE_OPT_SGD = 1, ELFPIE_OPT_NADAM = 2, ELFPIE_OPT_ADABELIEF = 3 };
/* Arithmetic of the plan.  ELFPIE_F32_MFMA_BF16X3 (n_lo = 256 only): FP32 everywhere
 * except the two row transforms of each LED's low-resolution tile (F_B of Eq. 1 and
 * F_B^H of Eq. 9 along the tile's rows, restricted to the pupil's support box), which are
 * DFT-matrix products on the matrix cores with every FP32 operand split into a BF16 high
 * and low part and three products (hi hi, hi lo, lo hi) accumulated in FP32: each product
 * carries a relative error of about 2^-16 (FP32: 2^-24).  Arrays are as for ELFPIE_F32. */
enum { ELFPIE_F64 = 0, ELFPIE_F32 = 1, ELFPIE_F32_MFMA_BF16X3 = 2 };
enum {
  ELFPIE_LEARN_PUPIL = 1u,    /* update P with Eq. 19 after each Psi update          */
  ELFPIE_PUPIL_SUPPORT = 2u,  /* P is confined to the NA disc (forward uses P * 1_S) */
  ELFPIE_PUPIL_FILTER = 4u    /* 3x3 Gaussian (sigma 1 px) pre-filter before P update */
};

/* Problem statement: Algorithm 1's inputs and the optics of Sec. 4.1. */
typedef struct {
  int32_t n_lo;            /* low-res image side: 32, 64, 96, 128, 192 or 256 (F32);
                              32 or 64 (F64); 192 and 256 need mux = 1                    */
  int32_t upsample;        /* r = n_hi / n_lo; n_hi must be 128, 256, 384, 512, 768 or 1024  */
  int32_t K;               /* number of LEDs (rows of led_k), >= 1; images = K / mux         */
  double wavelength_um;    /* illumination wavelength, > 0                                  */
  double na;               /* objective numerical aperture, > 0                             */
  double dx_lo_um;         /* sample-plane pixel = camera pixel / magnification, > 0         */
  const double *led_k;     /* HOST, K x 2, (kx, ky) = sin(theta) / lambda in 1/um; copied   */
  double alpha, beta;      /* Eq. 8 penalty weights, >= 0                                   */
  double lr;               /* Eq. 19 initial step: delta^0 = lr^2, > 0                      */
  double gamma1, gamma2;   /* Eq. 19 decay rates, in [0, 1)                                 */
  double eta_opt;          /* Eq. 19 stabiliser, >= 0                                       */
  double eta_h;            /* Eq. 14 stabiliser, >= 0                                       */
  double l1_eps;           /* L1 smoothing: rho(x) = sqrt(x^2 + eps^2) - eps; 0 = exact |x| */
  int32_t fidelity;        /* ELFPIE_FID_*                                                  */
  int32_t norm;            /* ELFPIE_NORM_* (fidelity and Hessian terms)                    */
  int32_t precision;       /* ELFPIE_F32, ELFPIE_F64 or ELFPIE_F32_MFMA_BF16X3              */
  uint32_t flags;          /* ELFPIE_LEARN_PUPIL | ELFPIE_PUPIL_SUPPORT | ELFPIE_PUPIL_FILTER */
  double fid_gamma;        /* exponent of ELFPIE_FID_GAMMA, in (0, 4]; ignored otherwise    */
  int32_t optimizer;       /* ELFPIE_OPT_* (default Eq. 19)                                 */
  int32_t mux;             /* M of Eq. 1: LEDs lit together per image, divides K (default 1);
                              image n is lit by LEDs n M .. n M + M - 1 and measures the sum
                              of their intensities.  Every "meas" below has K / mux images.  */
} elfpie_problem;

/* Optimiser state (Eq. 19), all DEVICE pointers owned by the caller.
 * psi, mu_psi: n_hi x n_hi complex; v_psi: n_hi x n_hi double; delta_psi:
 * n_hi x n_hi real.  P, mu_P: n_lo x n_lo complex; v_P: double; delta_P: real.
 * t: one int64, the number of updates done (t = 0 before the first update;
 * the bias corrections of Eq. 19 use t + 1).  A fresh state has mu = v = 0,
 * delta = lr^2, t = 0.  The state is the whole checkpoint: saving these
 * arrays and restoring them continues a run bit-for-bit. */
typedef struct {
  void *psi, *P;
  void *mu_psi;
  double *v_psi;
  void *delta_psi;
  void *mu_P;
  double *v_P;
  void *delta_P;
  int64_t *t;
} elfpie_state;

typedef struct elfpie_plan elfpie_plan;

/* Fill `p` with the defaults of Eq. 19 and Sec. 4.1: alpha = beta = 1e-3,
 * lr = 1e-2, gamma1 = 0.9, gamma2 = 0.999, eta_opt = 1e-8, eta_h = 1e-6,
 * l1_eps = 0, intensity fidelity (fid_gamma = 0.5), anisotropic norm, F32,
 * PUPIL_SUPPORT.
 * Geometry fields are zeroed. */
elfpie_status elfpie_problem_defaults(elfpie_problem *p);

/* Bytes of device workspace a plan for `p` needs (host query, no device work).
 * Fails with the same status elfpie_plan_create would return for `p`. */
elfpie_status elfpie_workspace_bytes(const elfpie_problem *p, size_t *bytes);

/* Validate `p`, compute the LED windows and pupil support (Sec. 3.1, M_k and P),
 * and copy the plan tables into the caller's workspace `d_ws` (device, at least
 * elfpie_workspace_bytes bytes, 256-byte aligned).  Synchronous.  The plan keeps
 * `d_ws` until destroyed.  Errors: E_INVALID (bad pointer or value), E_RANGE
 * (window outside the spectrum), E_UNSUPPORTED (size or precision), E_WORKSPACE. */
elfpie_status elfpie_plan_create(const elfpie_problem *p, void *d_ws, size_t ws_bytes,
                                 elfpie_plan **out);
elfpie_status elfpie_plan_destroy(elfpie_plan *plan);

/* Plan facts for callers sizing their buffers: out[0] = n_hi, out[1] = support
 * pixel count S, out[2] = K, out[3] = n_lo, out[4] = index of the LED nearest
 * the optical axis. `out` is HOST, 5 int32. */
elfpie_status elfpie_plan_info(const elfpie_plan *plan, int32_t *out);

/* Automatic penalty weight, Eq. 16 (intensity) / Eq. 17 (amplitude):
 * alpha = beta = (1/5) sqrt(pi/2) (1/K) sum_k sum |L (x) g(I_k)| / (n_lo^2), with the
 * mask L = [-1 2 -1; -2 4 -2; -1 2 -1] applied where it fits in the image and g the
 * plan's scaling (the Sec. 6.3 ones included).  meas: DEVICE, (K / mux) x n_lo x n_lo
 * real.
 * Per-LED sums run on the device in FP64; *alpha_out (HOST) receives the weight.
 * Synchronises `stream`.  The plan's own alpha and beta are not changed. */
elfpie_status elfpie_auto_penalty(elfpie_plan *plan, const void *meas, double *alpha_out, void *stream);

/* Sets the plan's penalty weights (Eq. 8), e.g. to elfpie_auto_penalty's value.
 * Host-only; later calls use the new weights, also the replays of a batch holding
 * the plan (its graph is captured again).  alpha, beta finite and >= 0. */
elfpie_status elfpie_plan_set_penalty(elfpie_plan *plan, double alpha, double beta);

/* Forward model, Eq. (1): for every LED, o_k = F_B P M_k Psi; image n is the sum
 * of |o_k|^2 over its mux LEDs.
 * psi: n_hi^2 complex; P: n_lo^2 complex.  Optional outputs (NULL to skip):
 * fields: K x n_lo x n_lo complex o_k, one per LED; intens: (K / mux) x n_lo x n_lo
 * real, sum_m |o_(n, m)|^2 per image.
 * If meas ((K / mux) x n_lo x n_lo real) and d_loss4 (4 doubles) are both given, writes
 * [L_fid, L_A, L_Phi, L_fid + alpha L_A + beta L_Phi] (Eq. 4/5, 6, 7, 8). */
elfpie_status elfpie_forward(elfpie_plan *plan, const void *psi, const void *P, const void *meas,
                             void *fields, void *intens, double *d_loss4, void *stream);

/* Loss (Eq. 8) and its gradients at (psi, P): g_psi = dL/d(conj Psi) (Eq. 15,
 * n_hi^2 complex), g_P = dL_fid/d(conj P) (Eq. 18, n_lo^2 complex, zero off the
 * support with ELFPIE_PUPIL_SUPPORT).  g_P or d_loss4 may be NULL.  The per-LED
 * low-resolution fields are recomputed, not stored. */
elfpie_status elfpie_grad(elfpie_plan *plan, const void *psi, const void *P, const void *meas,
                          void *g_psi, void *g_P, double *d_loss4, void *stream);

/* The same loss and gradients as elfpie_grad, from stored fields: `fields`
 * (K x n_lo x n_lo complex, DEVICE) holds the o_k that elfpie_forward wrote for
 * this psi and P, and the per-LED kernel reads them instead of recomputing the
 * crop and inverse transform (the trade-off of reverse-mode differentiation:
 * K n_lo^2 complex kept between the calls against one transform per LED).
 * Results equal elfpie_grad's bit for bit when the fields match. */
elfpie_status elfpie_grad_fields(elfpie_plan *plan, const void *psi, const void *P, const void *meas,
                                 const void *fields, void *g_psi, void *g_P, double *d_loss4, void *stream);

/* elfpie_grad without a plan or a workspace, for callers that cannot allocate device
 * memory (code under graph capture that may not call hipMalloc, tight serving loops,
 * harnesses that forbid allocation).  Same arguments and results as elfpie_grad (the
 * problem `p` in place of a plan: validated, its tables built and copied for each call),
 * bit for bit.  Allocates nothing on the device: the workspace is a static device array
 * of 32 MiB (33554432 bytes) that the library holds on each GPU it runs on until the
 * process ends; a problem whose elfpie_workspace_bytes exceeds it returns
 * ELFPIE_E_WORKSPACE before any device work (512^2 / K = 225 / 128^2 in FP32 needs about
 * 26 MiB).  Each call copies the tables on `stream` and waits for that stream before
 * enqueuing the gradient evaluation, which returns without waiting.  Every call on one
 * GPU uses the same array: calls on one stream are ordered, but calls that overlap on
 * different streams of one GPU race and give wrong results. */
elfpie_status elfpie_grad_noalloc(const elfpie_problem *p, const void *psi, const void *P, const void *meas,
                                  void *g_psi, void *g_P, double *d_loss4, void *stream);

/* One iteration of Algorithm 1 on `state`: gradients at (psi, P), Eq. 19 update
 * of psi, then (ELFPIE_LEARN_PUPIL) pre-filter and Eq. 19 update of P, then t += 1.
 * d_loss4 (optional, device) receives the loss terms at the pre-update state. */
elfpie_status elfpie_step(elfpie_plan *plan, const elfpie_state *state, const void *meas,
                          double *d_loss4, void *stream);

/* n_iter iterations (elfpie_step repeated).  A plan whose object branch rides in the
 * per-LED launch (elfpie_stage_timing's [4]: two long launches per iteration) launches
 * them directly on `stream` and captures nothing.  Other plans replay HIP graphs of 32
 * iterations and then at most one each of 16, 8, 4, 2 and 1, all captured by the first
 * call with these state, stack and history pointers; later calls with the same pointers
 * only replay, so the first call carries the capture cost.  Graphs are captured again
 * after elfpie_plan_set_penalty and when a pointer changes; the old ones are destroyed
 * only after their last replays have finished.  d_loss_hist (optional, device, n_iter x 4
 * doubles) receives each iteration's loss terms.  checked = 1 waits for the
 * stream at the end and returns ELFPIE_E_NONFINITE if any loss was NaN / Inf;
 * checked = 0 returns at once. */
elfpie_status elfpie_run(elfpie_plan *plan, const elfpie_state *state, const void *meas,
                         int32_t n_iter, double *d_loss_hist, int32_t checked, void *stream);

/* O = F_A Psi (Algorithm 1's output; centred unitary inverse transform), and its
 * inverse Psi = F_A^{-1} O.  n_hi^2 complex each; in-place is not allowed. */
elfpie_status elfpie_object_from_spectrum(elfpie_plan *plan, const void *psi, void *obj, void *stream);
elfpie_status elfpie_spectrum_from_object(elfpie_plan *plan, const void *obj, void *psi, void *stream);

/* Initial state: psi = the on-axis LED's window filled, on the pupil support,
 * with (r / n_lo) fftshift(fft2(sqrt(I_c))); zero elsewhere; P = 1 on the
 * support (everywhere without ELFPIE_PUPIL_SUPPORT); mu = v = 0; delta = lr^2;
 * t = 0.  meas: (K / mux) x n_lo x n_lo real; the image of the on-axis LED is used. */
elfpie_status elfpie_init_state(elfpie_plan *plan, const void *meas, const elfpie_state *state,
                                void *stream);

/* Timing of the iteration's stages in isolation: each stage is launched n_rep
 * times back to back on `stream` between two HIP events, on the state's current
 * arrays (the state is left unchanged), and ms_out (HOST, 8 floats) receives the
 * mean milliseconds per launch: [0] per-LED kernel (with the object-branch blocks
 * when the branch rides in it, see [4]), [1] object-branch launches outside it
 * (transforms and Hessian penalties, gradient mode; only the inverse row transforms
 * of psi when the branch rides in the per-LED launch), [2] spectrum gather + update
 * (gradient mode, with the pupil partial sums), [3] iteration tail launched alone
 * (pupil gradient and loss reduction), [4] 1 when the object branch rides in the
 * per-LED launch (512^2 spectrum, 128^2 tiles, FP32, with enough compute units left
 * free by the LED blocks), else 0, [5..7] unused (0).  Inside elfpie_run the tail of
 * every iteration but the last rides in a later launch.  Synchronous. */
elfpie_status elfpie_stage_timing(elfpie_plan *plan, const elfpie_state *state, const void *meas,
                                  int32_t n_rep, float *ms_out, void *stream);

/* Graph bookkeeping of `plan` (host query): out[0] = graphs captured so far (elfpie_run's
 * run graphs and the batch graphs that hold this plan), out[1] = run-graph replays so far.
 * A caller can check that timed calls only replayed (out[0] unchanged across them).
 * `out` is HOST, 2 int64. */
elfpie_status elfpie_plan_stats(const elfpie_plan *plan, int64_t *out);

/* ------------------------------------------------------------------------------------
 * Batches of independent fields of view (tiles), each with its own plan, state and
 * measured stack (sizes and K may differ).  One HIP graph replays one iteration of
 * every tile; the tiles are spread over n_branches parallel graph branches (longest
 * first on the algorithmic byte model, each to the least-loaded branch) so that small
 * tiles share the GPU.  The batch holds the pointers it is given: plans, states and
 * stacks must outlive it and keep their addresses.  A plan may appear in one batch
 * entry only, and must not be used by other calls while the batch runs.
 * ------------------------------------------------------------------------------------ */
typedef struct elfpie_batch elfpie_batch;

/* plans, states, meas: HOST arrays of n_tiles entries (copied); n_branches in 1..8
 * (reduced to n_tiles).  Errors: E_INVALID (NULL or misaligned pointers, a repeated
 * plan, counts out of range), E_DEVICE. */
elfpie_status elfpie_batch_create(elfpie_plan *const *plans, const elfpie_state *states, const void *const *meas,
                                  int32_t n_tiles, int32_t n_branches, elfpie_batch **out);
elfpie_status elfpie_batch_destroy(elfpie_batch *batch);

/* n_iter iterations of Algorithm 1 on every tile, replays of the batch graphs on
 * `stream`: one graph of one iteration of every tile opens a chain of iterations (as
 * elfpie_run does for a single plan), a second continues it n_iter - 1 times, a third
 * closes it.  d_loss_hist: NULL, or a HOST array of n_tiles DEVICE pointers, each
 * n_iter x 4 doubles as in elfpie_run (NULL entries allowed).  The graphs are captured
 * on the first call and again whenever the history pointers, the branch count or a
 * plan's penalty weights change; old graphs are destroyed after their last replays.
 * Results per tile equal those of elfpie_run on that tile alone. */
elfpie_status elfpie_batch_run(elfpie_batch *batch, int32_t n_iter, double *const *d_loss_hist, void *stream);

/* Branch-count tuning: for 1, 2, 4 and 8 branches (at most n_tiles) the batch graph
 * of one gradient evaluation per tile (which leaves the states unchanged) is timed over
 * n_rep replays; ms_out (HOST, 4 floats) receives the mean ms per replay (0 for a
 * skipped count) and the fastest count is kept and returned in *n_branches_out.
 * Synchronous.  Currently switched off: returns ELFPIE_E_UNSUPPORTED after the argument
 * checks (a run of it ended in a host abort whose cause is not found); the branch count
 * given to elfpie_batch_create stays in use. */
elfpie_status elfpie_batch_tune(elfpie_batch *batch, int32_t n_rep, float *ms_out, int32_t *n_branches_out,
                                void *stream);

const char *elfpie_batch_last_error(const elfpie_batch *batch);

/* Text of the last error on `plan` (or of the last plan-less call when plan is NULL). */
const char *elfpie_last_error(const elfpie_plan *plan);

#ifdef __cplusplus
}
#endif

#endif /* ELFPIE_H */
