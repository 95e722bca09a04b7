/*
 * wf.h -- multi-messenger Wiener filter on one AMD MI355X (gfx950).
 *
 * Computes the Wiener filter s = S (S + N)^-1 d (eqn wiener-alt of
 * Huffenberger 2017) of a periodic flat-sky map d whose noise covariance is
 * dense but splits into parts that are each diagonal in some basis
 * (Section 2):
 *     N = N_1/f   (diagonal in the 2-D Fourier basis)
 *       + N_stripe (noise constant along each row, diagonal in the basis of
 *                   row-constant Fourier modes; Section 3.3's m = 0 stripes)
 *       + N_white (diagonal in pixel space; infinite on masked pixels)
 * by iterating the messenger-field equations (eqns ew_t/ew_s, 2mess_t1 to
 * 2mess_s, extended by one messenger per extra term) with the cooling of
 * Section 2 and the adaptive schedule of Section 3.3.
 *
 * Conventions shared by every call:
 *   - a map is ny x nx, row-major (x fastest), periodic;
 *   - a Fourier-diagonal covariance is given on the rfft2 half spectrum,
 *     [ny][nx/2+1] row-major, as the variance of each *unitary* 2-D DFT mode
 *     in pixel-variance units (a spectrum C(l) maps to C(l)/Omega_pix, the
 *     correspondence N = (sigma^2/Omega_pix) I <-> N_l = sigma^2 of Section
 *     3.1); it must satisfy v(-ky, 0) = v(ky, 0) (likewise at kx = nx/2) as
 *     the covariance of a real field does;
 *   - the stripe covariance is the variance of each unitary 1-D DFT mode of
 *     the row value f(y), [ny] in FFT order (stripe map n(x, y) = f(y));
 *   - sizes: nx, ny powers of two in [64, 4096] (FP64 path: up to 2048), or
 *     384, 768, 1536 (a radix-3 pass); other sizes give WF_EUNSUPPORTED;
 *   - every pointer in wf_inputs, s_init and s_out is a DEVICE pointer owned
 *     by the caller; arrays are float (WF_F32) or double (WF_F64) as the
 *     context's precision says; the mask is uint8 (1 observed, 0 masked);
 *   - calls are ordered on the given HIP stream and return after their last
 *     device-to-host readback; one context per host thread at a time.
 * Errors: a negative status leaves outputs untouched; WF_NOT_CONVERGED means
 * the sweep budget ran out and every output is valid.
 */
#ifndef WF_H
#define WF_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  WF_OK = 0,
  WF_NOT_CONVERGED = 1,   /* budget exhausted; s_out and the report are valid */
  WF_EINVAL = -1,         /* bad shape, pointer or option                        */
  WF_ENOTPD = -2,         /* some tau_i <= 0: an empty noise term (Section 3.1)  */
  WF_ENONFINITE = -3,     /* NaN/Inf in the inputs or in the iteration           */
  WF_EDEVICE = -4,        /* a HIP call failed                                   */
  WF_ENOMEM = -5,         /* device allocation failed                            */
  WF_EUNSUPPORTED = -6,   /* size/precision not built                            */
  WF_ESCRATCH = -7        /* wf_solve_noalloc: workspace beyond its static scratch */
} wf_status;

typedef enum { WF_F32 = 0, WF_F64 = 1 } wf_precision;

/* Which chain of messenger fields runs (all have the Wiener filter as fixed
 * point at lambda = 1):
 *  THREE     one level per noise term, signal side first: 1/f (2-D Fourier),
 *            stripe (row basis), white (pixel) -- Section 2 extended to three
 *            terms; a white floor phi = floor_frac * min(N_white) is moved to
 *            the stripe level, whose own smallest eigenvalue is zero;
 *  MERGED    1/f and stripes form one 2-D Fourier-diagonal term (stripes on
 *            the k_x = 0 column), the arrangement of Section 3.3;
 *  AUGMENTED every Fourier-diagonal noise term joins the signal,
 *            S' = S + N_1/f + N_stripe, one messenger carries the white noise
 *            and s = S S'^-1 u -- Appendix A's shortcut for terms that share
 *            the signal's basis.  Fastest to converge. */
typedef enum { WF_CHAIN_THREE = 0, WF_CHAIN_MERGED = 1, WF_CHAIN_AUGMENTED = 2 } wf_chain;

typedef enum { WF_SCHED_FIXED = 0, WF_SCHED_ADAPTIVE = 1 } wf_sched_kind;

typedef struct {
  int32_t ny, nx;        /* map size                                   */
  int32_t precision;     /* wf_precision of inputs, fields and output  */
} wf_shape;

typedef struct {         /* DEVICE pointers, caller-owned, read-only during the call */
  const void* d;         /* [ny*nx] data                                          */
  const void* s_k;       /* [ny*(nx/2+1)] signal mode variance, >= 0              */
  const void* n_pix;     /* [ny*nx] white variance, > 0 on observed pixels        */
  const void* p_oof;     /* [ny*(nx/2+1)] 1/f mode variance >= 0, or NULL (absent);*/
                         /*   +inf projects that mode out of the data (Section 4)  */
  const void* p_stripe;  /* [ny] stripe 1-D mode variance >= 0, or NULL (absent)  */
  const uint8_t* mask;   /* [ny*nx] 1 observed / 0 masked, or NULL (all observed) */
} wf_inputs;
/* The spectra are covariances of real fields, so they are even in k: on the
 * real columns k_x = 0 and k_x = nx/2, s_k and p_oof must hold the same value
 * at k_y and ny - k_y, and p_stripe[k_y] must equal p_stripe[ny - k_y]
 * (exactly; WF_EINVAL otherwise).  The sweep updates those two columns on
 * k_y <= ny/2 and takes the other half by conjugation. */

typedef struct {         /* HOST struct */
  int32_t kind;          /* wf_sched_kind                                               */
  const double* lambda;  /* FIXED: lambda for sweep k is lambda[min(k, n_lambda-1)]     */
  int32_t n_lambda;
  double lambda0;        /* ADAPTIVE (Section 3.3): start value, e.g. 1e4               */
  double shrink_exp;     /*   lambda <- lambda^shrink_exp on a plateau, e.g. 0.7        */
  double plateau_rtol;   /*   plateau: |change of dd2| < plateau_rtol * sweeps * dd2    */
  double snap_eps;       /*   lambda is set to 1 once lambda - 1 < snap_eps             */
  double rtol;           /* stop when lambda == 1 and rho <= rtol (0: never)            */
  int32_t max_sweeps;    /* sweep budget (>= 1)                                         */
  int32_t monitor_every; /* residual evaluated every K sweeps and after the last one    */
  double beta[3];        /* tau_i = beta_i * smallest eigenvalue of N_i (1/f, stripe,   */
                         /*   white); beta < 1 where both chain neighbours are free     */
  double floor_frac;     /* alpha: white floor lent to the stripe level                 */
  int32_t chain;         /* wf_chain                                                    */
  int32_t stop_full;     /* 1: stop test uses hypot(rho, rho_mask) instead of rho       */
  int32_t field_mode;    /* 0: s_init and s_out are the signal s.  1: both are the      */
                         /*   chain's signal-end field u = S_chain x, x = S^-1 s: u = s */
                         /*   for the three-level and merged chains, u = s + N_F x for  */
                         /*   the augmented one (its messenger's signal side, App. A).  */
                         /*   A warm start then hands s_init unsmoothed to the white    */
                         /*   level when the chain has no Fourier-diagonal messenger    */
                         /*   (augmented, or white noise only); with one, the signal    */
                         /*   end is recomputed from t_0 each sweep and modes agree     */
} wf_schedule;

typedef struct {         /* HOST struct filled by wf_solve */
  int32_t status;        /* same as the return value                                    */
  int32_t sweeps;        /* sweeps executed                                             */
  int32_t n_records;     /* monitor records written to the trace                        */
  int32_t n_levels;      /* messenger levels in the chain                               */
  double lambda;         /* lambda of the last sweep                                    */
  double rho;            /* |m (d_rec - d)| / |m d|, d_rec = (I + N S^-1) s (Section 2) */
  double rho_mask;       /* nu |(1-m) S^-1 s| / |m d|, nu = max observed white variance */
  double dd2;            /* sum over observed pixels of (d_rec - d)^2                   */
  double d2;             /* sum over observed pixels of d^2                             */
  double chi2_joint;     /* J_lambda: -2 log of the joint probability of the state      */
                         /*   (eqn 2mess_prob): s^T S^-1 s plus, for every link of the  */
                         /*   chain, difference^T C^-1 difference (C = T_i or Nbar_i),  */
                         /*   at the last check's lambda, summed in float64; each sweep */
                         /*   lowers it at fixed lambda (Appendix A), and at lambda = 1 */
                         /*   its minimum over the messengers is chi^2(s) (Section 2).  */
                         /*   Pixels with Nbar_white = 0 add nothing (t is d there)     */
  double masked_x_norm;  /* |(1-m) S^-1 s|: zero at the Wiener solution                 */
  double tau[3];         /* messenger variances (1/f or merged, stripe, white); 0 absent*/
  double phi;            /* white floor moved to the stripe level                       */
  double kernel_ms[4];   /* profiling (wf_ctx_set_profiling): summed durations of the   */
  int32_t kernel_launches[4]; /* row, column, monitor and controller kernels timed     */
  int32_t refine_rounds; /* wf_solve_refined: float32 solves run (0 for other calls)     */
} wf_report;

/* Create a context (device workspace, FFT tables) for one map shape on the
 * current HIP device.  *out receives the handle; free with wf_ctx_destroy. */
wf_status wf_ctx_create(const wf_shape* shape, void** out);
void wf_ctx_destroy(void* ctx);

/* Fill sch with the defaults: adaptive, lambda0 1e4, shrink 0.7, plateau 1e-2,
 * snap 1e-3, rtol 1e-6, max_sweeps 20000, monitor_every 16,
 * beta {0.9, 0.9, 1.0}, floor_frac 0.5, chain THREE. */
void wf_schedule_default(wf_schedule* sch);

/* Solve.  s_init: DEVICE [ny*nx] warm start (every messenger and data-like
 * field starts at s_init; by Section 2 the start does not change the
 * solution), or NULL for the zero start of Section 2.  s_out: DEVICE
 * [ny*nx].  rep: HOST, may be
 * NULL.  trace: HOST [6 * ceil(max_sweeps / monitor_every)] rows of
 * (sweep index, lambda, rho, dd2, rho_mask, chi2_joint), one per residual
 * check, or NULL. */
wf_status wf_solve(void* ctx, const wf_inputs* in, const wf_schedule* sch,
                   const void* s_init, void* s_out, wf_report* rep,
                   double* trace, hipStream_t stream);

/* wf_solve without a context, for callers that cannot allocate (code that
 * may not call hipMalloc: serving loops, harnesses that forbid it).  The
 * workspace (transit buffer, messenger state, coefficients, monitor buffers,
 * schedule and trace arrays, argument blocks) is carved from a static device
 * array of wf_noalloc_scratch_bytes() bytes (32 MiB) that each GPU the
 * library runs on holds until the process ends; the call allocates no device
 * or pinned host memory and creates no events.  It fits, for instance,
 * maps up to 512 x 512 in float64 and 768 x 768 in float32 with the default
 * schedule budget; shape and schedule are checked before any work and a
 * workspace that does not fit returns WF_ESCRATCH, as does max_sweeps above
 * 65536.  Runs on the current device with the default tiling; inputs,
 * outputs, report, trace and errors as for wf_solve (same kernels, so the
 * results are identical to a wf_solve with a context of that tiling).  Calls
 * that overlap on one GPU share the scratch and race; each call initialises
 * every part of it that it reads.  The host checks the device schedule every
 * 4 chunks with a blocking copy, so up to 4 * monitor_every sweeps may be
 * enqueued past convergence (they return at once). */
wf_status wf_solve_noalloc(const wf_shape* shape, const wf_inputs* in, const wf_schedule* sch,
                           const void* s_init, void* s_out, wf_report* rep, double* trace,
                           hipStream_t stream);
size_t wf_noalloc_scratch_bytes(void);

/* Mixed-precision iterative refinement of the Wiener filter (the refinement
 * is not from the paper; each round is the paper's iteration): float32
 * sweeps, float64 residual.  Round 0 solves the data on the float32
 * context with schedule `first`; x = S^-1 s of that solve is accumulated in
 * float64 on the float64 context and its residual Delta d = d_rec - d of
 * Section 2 is evaluated in float64; while rho > rtol and fewer than
 * max_rounds corrections have run, -Delta d (observed pixels) is solved on
 * the float32 context with schedule `corr` and its x is added.  The filter
 * is linear with inverse (I + N S^-1) on the observed pixels, so each round
 * divides rho by roughly the float32 solve's relative accuracy.  The
 * masked part of x is not seen by the residual: rho_mask stays at the
 * level of round 0 (the same holds for any solve stopped on rho alone).
 *   ctx32, ctx64  contexts of the same shape on the current device, WF_F32
 *                 and WF_F64;
 *   in            float64 DEVICE inputs (as for ctx64); float32 copies are
 *                 made on ctx32 (allocated on its first refined solve);
 *   first, corr   schedules of round 0 and of the corrections (their rtol
 *                 applies to each float32 solve, relative to its own
 *                 right-hand side); corr->field_mode must be 0, and
 *                 first->field_mode selects what s_init and s_out are;
 *   s_init        float64 DEVICE [ny*nx] warm start of round 0 (the signal s,
 *                 or with first->field_mode 1 the chain field u, as for
 *                 wf_solve; rounded to float32 for that solve), or NULL;
 *   s_out         float64 DEVICE [ny*nx], s = S x, or with first->field_mode
 *                 1 the chain field u = S_chain x (as wf_solve's output in
 *                 that mode);
 *   rep           rho and rho_mask of the final float64 residual, total
 *                 sweeps, refine_rounds (= n_records), the float32 solves'
 *                 kernel timing when ctx32 profiles; status WF_OK when
 *                 rho <= rtol, WF_NOT_CONVERGED otherwise (s_out valid);
 *   trace         HOST [4 * (max_rounds + 1)] rows of (round, sweeps so far,
 *                 rho, rho_mask) after each round, or NULL.
 * Synchronises stream. */
wf_status wf_solve_refined(void* ctx32, void* ctx64, const wf_inputs* in,
                           const wf_schedule* first, const wf_schedule* corr, int32_t max_rounds,
                           double rtol, const void* s_init, void* s_out, wf_report* rep,
                           double* trace, hipStream_t stream);

/* Largest batch wf_solve_batch accepts. */
#define WF_BATCH_MAX 1024

/* Solve n independent maps with one schedule (the Section 2 iteration for
 * each; batching is not from the paper: a sky survey yields many maps of a
 * few shapes).  Maps of
 * equal shape and chain kind share every kernel launch (one grid row per
 * map); one chunk of monitor_every sweeps of every map plus their monitors
 * is recorded once as a HIP graph and replayed, and each map keeps its own
 * device-side cooling schedule and stops on its own.
 *   ctxs[n]    distinct contexts of one precision on the current device, one
 *              per map (the context fixes the map's shape and tiling);
 *   inputs[n]  HOST array of per-map inputs (DEVICE pointers inside);
 *   sch        one schedule for every map (adaptive or fixed);
 *   s_init[n]  HOST array of DEVICE warm starts [ny_i*nx_i] (as for
 *              wf_solve; an entry may be NULL), or NULL for zero starts;
 *   s_out[n]   HOST array of DEVICE output pointers [ny_i*nx_i];
 *   reps[n]    HOST reports, or NULL.
 * Returns the most severe error of any map, else
 * WF_NOT_CONVERGED if any map ran out of sweeps, else WF_OK; per-map status
 * is in reps[i].status.  Input errors are found before any sweep runs.
 * The per-map schedules, argument blocks and the pinned read-back ring live
 * in a workspace of ctxs[0], allocated on its first batch and grown only
 * when a larger batch comes (freed with that context); the recorded graph,
 * its streams and events are created per call.  Synchronises stream. */
wf_status wf_solve_batch(void* const* ctxs, int32_t n, const wf_inputs* inputs,
                         const wf_schedule* sch, const void* const* s_init, void* const* s_out,
                         wf_report* reps, hipStream_t stream);

/* Approximate inverse-noise weighting N^-1 d (Section 4): the Wiener filter
 * with a small flat signal covariance S = alpha I gives
 * N^-1 d ~= alpha^-1 [alpha I (alpha I + N)^-1 d], with relative error of
 * order alpha / (smallest eigenvalue of N).  in->s_k is ignored; masked
 * pixels come out as 0 (their inverse variance).  s_init, if given, is a
 * warm start of the signal-side field alpha (alpha + N)^-1 d.  Other
 * arguments, outputs and errors as for wf_solve (sch->field_mode must be 0);
 * out receives the weighted map. */
wf_status wf_inverse_noise_weight(void* ctx, const wf_inputs* in, double alpha,
                                  const wf_schedule* sch, const void* s_init, void* out,
                                  wf_report* rep, double* trace, hipStream_t stream);

/* Unnormalised 2-D real-to-complex FFT with the solver's own kernels:
 * x [ny*nx] real -> X [ny*(nx/2+1)] complex (interleaved re, im), numpy rfft2
 * layout and sign (X_k = sum_p x_p exp(-2 pi i k.p/n)).  DEVICE pointers. */
wf_status wf_rfft2(void* ctx, const void* x, void* X, hipStream_t stream);

/* Inverse of wf_rfft2 including the 1/(nx ny) factor, with numpy irfft2's
 * semantics: inverse FFT over ky, then a real inverse FFT over kx that
 * ignores the imaginary parts of the k_x = 0 and k_x = nx/2 bins. */
wf_status wf_irfft2(void* ctx, const void* X, void* x, hipStream_t stream);

/* Turn per-kernel timing with HIP events on the solve stream on (1) or off. */
wf_status wf_ctx_set_profiling(void* ctx, int32_t enable);

/* Transit-buffer tilings (rows x columns per tile, rows per row block) the
 * library holds, and the one a context uses.  Only tiling 0..count-1 exist;
 * wf_ctx_set_tile returns WF_EUNSUPPORTED for a tiling not built for the
 * context's size and precision.  wf_autotune times the candidates. */
int32_t wf_tile_count(void);
wf_status wf_ctx_set_tile(void* ctx, int32_t tile);
int32_t wf_ctx_get_tile(void* ctx);

/* Autotuner (not from the paper): times a short solve of the caller's map
 * (a fixed cooling ramp of `sweeps` sweeps, 1 <= sweeps <= 4096, monitor
 * every 16) in every tiling built for the context's size and precision, and
 * leaves the context on the fastest.  Tilings other than the default are
 * built for float32 maps whose sides are 256, 768, 1536 or 2048.
 *   in       as for wf_solve (DEVICE inputs of the map to tune on);
 *   scratch  DEVICE [ny*nx] buffer of the context's precision, overwritten
 *            with the probe solves' output;
 *   ms       HOST [wf_tile_count()] milliseconds per probe solve, -1 for a
 *            tiling not built, or NULL;
 *   best     HOST, receives the chosen tiling, or NULL.
 * Synchronises stream; a solve error is returned (the context keeps its
 * previous tiling then). */
wf_status wf_autotune(void* ctx, const wf_inputs* in, int32_t sweeps, void* scratch, double* ms,
                      int32_t* best, hipStream_t stream);

/* Autotuner for batches (not from the paper): the best tiling of a map
 * solved alone can differ from that of many maps of its shape sharing each
 * launch.  For each group of maps of one shape, times short batched solves
 * of that group alone (wf_solve_batch over its maps, the probe schedule of
 * wf_autotune) in every tiling built for the shape, and leaves the group's
 * contexts on the fastest.
 *   ctxs, n, inputs  as for wf_solve_batch;
 *   sweeps           probe length, 1 <= sweeps <= 4096;
 *   s_out[n]         HOST array of DEVICE buffers [ny_i*nx_i] of the contexts'
 *                    precision, overwritten with the probe solves' output;
 *   ms               HOST [n * wf_tile_count()]: ms[i*count + t] is the time in
 *                    milliseconds of one probe solve of map i's group in tiling
 *                    t (-1: not built), or NULL;
 *   best             HOST [n], receives the tiling each context is left on,
 *                    or NULL.
 * Synchronises stream.  A solve error is returned at once: the group being
 * tuned keeps its previous tilings, the groups before it their new ones. */
wf_status wf_autotune_batch(void* const* ctxs, int32_t n, const wf_inputs* inputs,
                            int32_t sweeps, void* const* s_out, double* ms, int32_t* best,
                            hipStream_t stream);

/* Sizes the library was built for, and its precision support. */
int32_t wf_supported(int32_t ny, int32_t nx, int32_t precision);

const char* wf_strerror(int32_t status);

#ifdef __cplusplus
}
#endif
#endif /* WF_H */
