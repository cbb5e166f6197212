/*
 * libargus: batched FP64 Kalman-filter log-likelihood of pulsar-timing
 * residuals on MI355X (gfx950), its gradient, and a learned surrogate.
 *
 * The operation (paper: Functionality, "Kalman filter likelihood
 * evaluation" and "State-space model construction"; Summary): every noise
 * process of a pulsar (spin wandering, OU red noise, a common OU process for
 * the gravitational-wave background, coupled across pulsars by the
 * Hellings-Downs curve) is a linear SDE; stacked, they form one linear
 * Gaussian state-space model whose likelihood the Kalman filter evaluates in
 * O(N) by the prediction-error decomposition
 *     log L = sum_k -1/2 (ln 2 pi + ln S_k + e_k^2 / S_k),
 * e_k the innovation and S_k its variance. The gradient is what the paper's
 * sampler integration consumes (Functionality, "Sampler Integration").
 *
 * Models (per-pulsar state in brackets; r residual phase offset in s, f
 * fractional frequency, a red OU in s, g common OU in s):
 *   ARGUS_M1_SPIN      one pulsar, [r, f]; canonical params
 *                      [log10 sigma_s, EFAC]
 *   ARGUS_M2_PSR4      P independent pulsars, [r, f, a, g] each; canonical
 *                      params: per pulsar [log10 sigma_red, log10 gamma_red,
 *                      EFAC, log10 EQUAD], then [log10 A, gamma] of the common
 *                      power law (mapped to the OU variance over 1/T_span..inf)
 *   ARGUS_M3_JOINT_HD  the same P pulsars in one joint 4P-dim state whose
 *                      common-process noise is Hellings-Downs correlated
 *   ARGUS_M4_PSR5_DM   model 2 with DM variations (Statement of Need: DM
 *                      variations are another latent stochastic process):
 *                      [r, f, a, g, m] per pulsar, m the DM delay at 1400 MHz
 *                      (an OU process, stationary at t0), seen at a TOA of
 *                      radio frequency nu through (1400 MHz / nu)^2;
 *                      canonical params per pulsar [log10 sigma_red,
 *                      log10 gamma_red, EFAC, log10 EQUAD, log10 sigma_dm,
 *                      log10 gamma_dm], then [log10 A, gamma]
 * Measurement: y_k = r + a + g + white, white variance EFAC^2 sigma_k^2 +
 * EQUAD^2 (model 1: EFAC^2 sigma_k^2). Every filter starts from the prior at
 * the epoch t0 = 0 and predicts to its first TOA.
 *
 * Conventions for every call:
 *  - Return value: ARGUS_OK (0) or an ARGUS_E_* code; argus_last_error()
 *    then holds a message (thread-local). Nothing throws across the ABI.
 *  - "dev" pointers are HIP device memory owned by the caller; the library
 *    never frees them. "host" pointers are read during the call only.
 *  - Work is enqueued asynchronously on `stream` (a hipStream_t, may be 0).
 *    Only dataset create/destroy and the first loglike call for a new sample
 *    count (which autotunes) synchronise.
 *  - A numeric failure of one sample does not fail the call: its logL is
 *    -inf, its gradient row 0, and its status word gets ARGUS_S_NONPD
 *    (innovation variance <= 0) or ARGUS_S_NONFINITE (NaN/Inf parameter or
 *    state). The first failure in pulsar order decides the flag; a non-finite
 *    parameter anywhere in the row gives ARGUS_S_NONFINITE.
 *  - A dataset handle keeps per-sample-count workspaces and captured graphs;
 *    calls on one handle from concurrently running streams race.
 */
#ifndef ARGUS_H
#define ARGUS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ARGUS_OK = 0, ARGUS_E_INVAL = 1, ARGUS_E_HIP = 2, ARGUS_E_NOMEM = 3,
       ARGUS_E_UNSUPPORTED = 4 };
enum { ARGUS_S_NONPD = 1, ARGUS_S_NONFINITE = 2 };
enum { ARGUS_M1_SPIN = 1, ARGUS_M2_PSR4 = 2, ARGUS_M3_JOINT_HD = 3, ARGUS_M4_PSR5_DM = 4 };

typedef struct argus_dataset* argus_dataset_t;

typedef struct {
  int32_t model;            /* ARGUS_M1_SPIN / ARGUS_M2_PSR4 / ARGUS_M3_JOINT_HD */
  int32_t n_psr;            /* P >= 1 (model 1: P == 1; model 3: P <= 63) */
  const int64_t* toa_off;   /* host [P+1] CSR offsets into t/y/sigma, off[0]=0 */
  const double* t;          /* host [N] s since the epoch t0 = 0; strictly
                               ascending within a pulsar, >= 0 */
  const double* y;          /* host [N] timing residuals, s */
  const double* sigma;      /* host [N] per-TOA 1-sigma errors, s, > 0 */
  const double* pos;        /* host [P*3] unit vectors; model 3 only, else NULL */
  const double* fixed;      /* host [C] values used for non-free canonical params */
  const uint8_t* free_mask; /* host [C]; nonzero = free. Free params become the
                               columns of theta in canonical order. NULL = all free */
  double t_span;            /* s; sets the common OU rate 2 pi / t_span and the
                               power-law low-frequency cutoff 1 / t_span */
  double s_r, s_f;          /* prior std of r (s) and f at t0 */
  double sigma_s;           /* spin random-walk amplitude (models 2, 3, 4) */
  const double* freq;       /* host [N] radio frequency of each TOA, MHz, > 0;
                               model 4 only, else NULL */
} argus_dataset_desc;

/* Builds the state-space model of a dataset (paper: Functionality,
 * "State-space model construction": the noise processes of every pulsar,
 * and for model 3 their Hellings-Downs coupling, compiled into one model;
 * the TOA data enter as in Functionality, "Standardized Data Input", here
 * as plain arrays): copies the data to the device, orders the joint stream
 * by (t, pulsar), and precomputes per-TOA intervals, the common-process
 * decay and (model 4) the chromatic factors. Validation failures (non-ascending or negative times, non-finite
 * or non-positive errors, bad offsets, a missing position or frequency
 * array) return ARGUS_E_INVAL before any device work; *out is NULL then.
 * C = 2 (model 1), 4P + 2 (models 2, 3) or 6P + 2 (model 4) canonical
 * parameters. Synchronises. Model 4 has the likelihood, its per-pulsar
 * terms, the gradient (tangent sweep) and the samplers; the plain baseline
 * and the smoother return ARGUS_E_UNSUPPORTED for it. */
int argus_dataset_create(const argus_dataset_desc* desc, argus_dataset_t* out);
int argus_dataset_destroy(argus_dataset_t ds);
/* D = number of free parameters (columns of theta). */
int argus_dataset_n_params(argus_dataset_t ds, int32_t* D);

/* logL for S parameter rows (paper: Functionality, "Kalman filter
 * likelihood evaluation": the Kalman filter's prediction-error
 * decomposition over the time-ordered TOAs, O(N)). theta: dev [S*D]
 * row-major FP64; logl: dev [S]; status: dev [S] or NULL. Batched
 * persistent kernel replayed from a captured hipGraph; the first call for a
 * new S autotunes (synchronises). S < 0, a NULL theta (D > 0) or a NULL
 * logl return ARGUS_E_INVAL; S = 0 does nothing. */
int argus_loglike(argus_dataset_t ds, const double* theta, int64_t S,
                  double* logl, int32_t* status, void* stream);

/* argus_loglike for callers that cannot allocate device memory: code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.
 * Models 1, 2 and 4 (model 3 -> ARGUS_E_UNSUPPORTED); same arguments and
 * outputs as argus_loglike, computed by the same filter and reduction
 * kernels in one fixed launch layout (no autotuning, no graph, nothing
 * synchronised). It allocates nothing: the per-(pulsar, sample) terms,
 * status words and per-(64-sample tile, pulsar) flags live in a static 8 MiB
 * device array of the library, one copy per device, held until the process
 * ends, which limits S to round_up(8 P S, 256) + round_up(4 P S, 256) +
 * 4 P ceil(S / 64) <= 8 MiB (47 pulsars: S <= 14,795; one pulsar:
 * S <= 695,424); a larger S returns ARGUS_E_INVAL with the limit
 * in argus_last_error(). Every call on a device shares that device's array:
 * calls that overlap in time on one device (concurrent streams, threads)
 * race and give wrong results. The first call on a device looks up the
 * array's address (no allocation). */
int argus_loglike_noalloc(argus_dataset_t ds, const double* theta, int64_t S,
                          double* logl, int32_t* status, void* stream);

/* Per-pulsar terms of logL (models 1, 2): terms dev [P*S], pulsar-major
 * (terms[p*S + s]); same kernel as argus_loglike, no graph. */
int argus_loglike_terms(argus_dataset_t ds, const double* theta, int64_t S,
                        double* terms, int32_t* status, void* stream);

/* The plain per-sample GPU filter (the same likelihood as argus_loglike,
 * paper: Functionality, "Kalman filter likelihood evaluation", written the
 * textbook way as a baseline): one kernel launch per sample, one thread per
 * pulsar, dense 4 x 4 products, per-TOA transcendentals and divisions, no
 * precompute, no persistence, no graph. Models 1, 2 (others:
 * ARGUS_E_UNSUPPORTED). Same arguments and outputs as argus_loglike. */
int argus_loglike_plain(argus_dataset_t ds, const double* theta, int64_t S,
                        double* logl, int32_t* status, void* stream);

/* logL and its gradient w.r.t. the D free parameters (models 1, 2, 4) (paper:
 * Functionality, "Sampler Integration": samplers consume the likelihood and
 * its gradient). grad: dev [S*D] row-major FP64, caller-owned; rows of
 * failed samples (status != 0) are 0. By default a tangent (forward-mode)
 * sweep carries the derivatives of the filter state along each parameter
 * direction in one pass; the first call for a new S chooses, by timing, how
 * many directions each wave carries (synchronises). With the environment
 * variable ARGUS_GRAD=adjoint the reverse-mode sweep with checkpointed
 * filter states is used instead (models 1, 2; model 4 always uses the
 * tangent sweep); both give the derivative of the same recursion. Model 3
 * returns ARGUS_E_UNSUPPORTED. */
int argus_loglike_grad(argus_dataset_t ds, const double* theta, int64_t S,
                       double* logl, double* grad, int32_t* status,
                       void* stream);

/* One Hamiltonian Monte Carlo transition for each of S independent chains
 * (models 1, 2, 4), the gradient-based sampling the likelihood and its
 * gradient serve (paper: Functionality, "Sampler Integration"). Chain s
 * draws its momentum p = z_s / sqrt(inv_mass) (M = diag(1 / inv_mass)),
 * takes n_leapfrog >= 1 kick-drift-kick steps of size eps[s] on
 * log pi = logL + log prior, the prior uniform on the box [lo, hi], and
 * accepts the end point when logu[s] < H0 - H1, H = -log pi + p^T M^-1 p / 2.
 * A trajectory that leaves the box or meets a failed likelihood (status !=
 * 0) at any leapfrog position is rejected. Each leapfrog position costs one
 * batched gradient evaluation (argus_loglike_grad's sweep).
 *   eps: dev [S]; inv_mass, lo, hi: dev [D]; z: dev [S*D] standard normal
 *   draws; logu: dev [S] log of uniform draws (caller's random numbers)
 *   theta, logl, grad: dev [S*D], [S], [S*D], the chains' current positions,
 *   logL and gradient there (from argus_loglike_grad), updated in place for
 *   accepted chains
 *   accepted: dev [S] int32, incremented for accepted chains
 *   energy_err: dev [S] H1 - H0 (+inf when the trajectory left the box or
 *   met a failed likelihood), or NULL
 * Allocates per-sample-count work buffers on the first call for S. */
int argus_hmc_step(argus_dataset_t ds, int64_t S, int32_t n_leapfrog, const double* eps,
                   const double* inv_mass, const double* lo, const double* hi,
                   const double* z, const double* logu, double* theta, double* logl,
                   double* grad, int32_t* accepted, double* energy_err, void* stream);

/* One No-U-Turn Sampler transition for each of S independent chains (models
 * 1, 2, 4): the sampler of the paper's posteriors (Functionality, "Sampler
 * Integration", and its figure: NUTS, Hoffman & Gelman 2014), with
 * multinomial trajectory sampling and the generalised no-U-turn criterion.
 * Per chain: momentum p = z_s / sqrt(inv_mass); doubling j (< max_depth)
 * grows 2^j leapfrog leaves of size eps[s] in direction dirs[s*max_depth+j]
 * (+1 or -1) from the trajectory end on that side. A leaf diverges when
 * H - H0 > 1000, H is not a number, it leaves the box [lo, hi] or its
 * likelihood fails (H = -logL + p^T M^-1 p / 2). Inside a subtree, halves
 * A, B merge with the proposal taken from B when the merge's uniform
 * u_sub[(s*max_depth + j)*2^(max_depth-1) + m] < exp(W_B - W) (W the
 * log-sum-exp of -H over leaves, m the merge's post-order index within the
 * subtree) and the merged subtree makes a U-turn unless both end momenta,
 * scaled by inv_mass, have a positive dot product with the summed momentum;
 * a U-turn or divergence inside a subtree discards it and ends the
 * transition. A valid subtree's proposal replaces the trajectory's when
 * u_top[s*max_depth + j] < exp(W_sub - W_traj); the trajectory stops at a
 * U-turn between its ends or after max_depth doublings.
 *   eps: dev [S]; inv_mass, lo, hi: dev [D]; z: dev [S*D] standard normal
 *   draws; dirs: dev int32 [S*max_depth]; u_top: dev [S*max_depth];
 *   u_sub: dev [S*max_depth*2^(max_depth-1)] uniforms in (0, 1)
 *   theta, logl, grad: dev [S*D], [S], [S*D], current state in, the
 *   transition's result out (from argus_loglike_grad at the start)
 *   depth, n_leapfrog, divergent: dev int32 [S] out (doublings accepted,
 *   leapfrog steps taken, 1 if the transition ended on a divergence)
 *   accept_stat: dev [S] mean of min(1, exp(H0 - H)) over the leaves, or NULL
 * max_depth in [1, 10]. All chains step together: each leaf is one batched
 * gradient evaluation; the call synchronises the stream after every 8th
 * leaf of a subtree and at its end, to stop when no chain is still
 * building. Allocates per-sample-count work
 * buffers on the first call for S (and for a larger max_depth). */
int argus_nuts_step(argus_dataset_t ds, int64_t S, int32_t max_depth, const double* eps,
                    const double* inv_mass, const double* lo, const double* hi,
                    const double* z, const int32_t* dirs, const double* u_top,
                    const double* u_sub, double* theta, double* logl, double* grad,
                    int32_t* depth, int32_t* n_leapfrog, int32_t* divergent,
                    double* accept_stat, void* stream);

/* Smoothed latent states (models 1, 2, 4): for every TOA k of every pulsar and
 * every sample s, the posterior mean and variance of that pulsar's state
 * components at t_k given all of its TOAs (paper: Summary and Statement of
 * Need: the filter tracks the realised, time-ordered noise; the fixed-interval
 * smoother completes it with the later data). Components c: r, f, a, g
 * (nc = 4) for model 2; r, f (nc = 2) for model 1; r, f, a, g, m (nc = 5)
 * for model 4.
 *   mean: dev [N*nc*S] FP64, element ((k*nc + c)*S + s), k the dataset's
 *         global TOA index (pulsar-major CSR order)
 *   var:  dev, same layout, or NULL for means only
 *   logl, status: dev [S] or NULL, as argus_loglike
 * The entries of a pulsar whose filter fails for a sample (innovation
 * variance not positive, or a non-finite parameter among its own and the
 * common ones) are NaN. Computed without a matrix inverse by the modified
 * Bryson-Frazier recursion over the checkpointed filter: E[x|y] = x - P lam
 * and Cov[x|y] = P - P Lam P with (x, P) filtered and (lam, Lam) the
 * information of the later TOAs about that state. The first call per sample
 * count times one wave per (64-sample tile, pulsar) against a time-parallel
 * form (each pulsar's stream in chunks reversed at once from chained chunk
 * summaries; skipped when its checkpoint store does not fit in device
 * memory) and keeps the faster; the environment variable ARGUS_SMOOTH =
 * seq | tp2 | tp4 | tp8 | tp16 forces a form (any other value:
 * ARGUS_E_INVAL). The time-parallel form keeps a checkpoint before every
 * fourth TOA (112 B per four TOAs and sample; model 4: 160 B). Model 3
 * returns ARGUS_E_UNSUPPORTED; N*nc*S above 2^40 elements, or a pulsar with
 * more than 33,554,431 TOAs, returns ARGUS_E_UNSUPPORTED. */
int argus_smooth(argus_dataset_t ds, const double* theta, int64_t S, double* mean,
                 double* var, double* logl, int32_t* status, void* stream);

/* ---------------------------------------------------------------------
 * Learned surrogate of logL (an MLP d -> w -> w -> w -> 1, SiLU hidden
 * layers) and delayed-acceptance screening with the exact filter as judge
 * (Christen & Fox 2005), for the paper's sampler integration (Functionality,
 * "Sampler Integration"). Hidden layers run on BF16 matrix cores with FP32
 * accumulation; biases, output layer, gradients and Adam state are FP32.
 *
 * Packed FP32 parameter block ("master"), weights row-major output-by-input:
 *   W1 [w x d] | b1 [w] | W2 [w x w] | b2 [w] | W3 [w x w] | b3 [w] |
 *   W4 [w] | b4 [1]          (n = w d + 2 w^2 + 4 w + 1)
 * The caller owns the master block and the Adam moments (device FP32); the
 * handle owns the BF16 copies and activation workspaces. Inputs pass
 * through an affine input map x = T (theta - c), evaluated in FP64 inside
 * the kernels, then are rounded to BF16 (8 significant bits): the map should
 * bring the region the network must resolve to about [-1, 1] in every
 * direction (the box of the training inputs, or for correlated parameters a
 * whitening of their covariance); the network predicts the standardised
 * target (logL - out_mu) / out_sd.
 * ------------------------------------------------------------------- */
typedef struct argus_mlp* argus_mlp_t;

/* d_in in [1, 32]; width a multiple of 64 in [64, 1024]; max_batch (largest
 * training batch) a multiple of 64. Allocates; synchronises. */
int argus_mlp_create(int32_t d_in, int32_t width, int64_t max_batch, argus_mlp_t* out);
int argus_mlp_destroy(argus_mlp_t h);
int argus_mlp_n_params(argus_mlp_t h, int64_t* n);

/* Takes the weights from master (dev [n]) into the handle's BF16/FP32
 * copies and sets the input map to the box map x = 2 (theta - in_lo) /
 * (in_hi - in_lo) - 1 (in_lo, in_hi host [d_in], finite, in_hi > in_lo) and
 * the target standardisation (out_sd > 0). Synchronises the stream. */
int argus_mlp_load(argus_mlp_t h, const float* master, const double* in_lo,
                   const double* in_hi, double out_mu, double out_sd, void* stream);

/* The same with a general affine input map x = T (theta - center): center
 * host [d_in], T host [d_in * d_in] row-major (x_k = sum_j T[k d_in + j]
 * (theta_j - center_j)), all finite; argus_mlp_load is the diagonal case
 * T = diag(2 / (in_hi - in_lo)), center = (in_lo + in_hi) / 2. Synchronises
 * the stream. */
int argus_mlp_load_affine(argus_mlp_t h, const float* master, const double* center,
                          const double* T, double out_mu, double out_sd, void* stream);

/* logl_hat (dev [Q]) for parameter rows theta (dev [Q*d_in] FP64), any Q. */
int argus_surrogate_eval(argus_mlp_t h, const double* theta, int64_t Q,
                         double* logl_hat, void* stream);

/* Loss (dev [1]) = mean over the batch of (net(theta) - (target - mu)/sd)^2
 * and its gradient w.r.t. the packed parameters (grad_out dev [n], or NULL
 * to keep it internal). B a multiple of 64, <= max_batch. */
int argus_mlp_grad(argus_mlp_t h, const double* theta, const double* target,
                   int64_t B, float* grad_out, float* loss_out, void* stream);

/* One training step: argus_mlp_grad, then Adam (beta 0.9, 0.999, eps 1e-8,
 * bias-corrected with step >= 1) on master/adam_m/adam_v in place, then the
 * handle's copies refreshed from the new master. */
int argus_surrogate_train_step(argus_mlp_t h, float* master, float* adam_m,
                               float* adam_v, const double* theta,
                               const double* target, int64_t B, float lr,
                               int64_t step, float* loss_out, void* stream);

/* n_batches training steps in one call (width <= 256, else
 * ARGUS_E_UNSUPPORTED): batch b takes rows order[b*B .. (b+1)*B) (dev int32,
 * each in [0, N)) of theta (dev [N*d_in]) and target (dev [N]) and makes
 * the step of argus_surrogate_train_step numbered step0 + b + 1 (Adam's bias
 * correction); loss_out dev [n_batches] (each batch's loss before its
 * update) or NULL. An epoch is one call with a permutation of the training
 * rows as order; nothing is gathered or copied on the host. */
int argus_surrogate_train_epoch(argus_mlp_t h, float* master, float* adam_m, float* adam_v,
                                const double* theta, const double* target,
                                const int32_t* order, int64_t n_batches, int64_t B, float lr,
                                int64_t step0, float* loss_out, void* stream);

/* Delayed acceptance, stage 1 for Q chains with symmetric proposals: chain i
 * survives when theta_prop[i] lies in [lo, hi] (dev [d]) and
 * logu1[i] < lh_prop[i] - lh_cur[i] (surrogate values). Survivor indices go
 * to idx (dev [Q]) in increasing order, their number to count (dev [1]).
 * work: dev int32 [argus_da_work_size(Q)]; work[0..Q) then holds the
 * stage-1 decisions. */
int argus_da_stage1(const double* theta_prop, const double* lo, const double* hi,
                    const double* lh_cur, const double* lh_prop, const double* logu1,
                    int64_t Q, int32_t d, int32_t* idx, int32_t* count, int32_t* work,
                    void* stream);
int64_t argus_da_work_size(int64_t Q);

/* dst[j] = src[idx[j]] (rows of d doubles) for j < cap; rows past *count
 * repeat the last survivor, so a fixed-size exact evaluation can follow. */
int argus_gather_rows(const double* src, const int32_t* idx, const int32_t* count,
                      int64_t cap, int32_t d, double* dst, void* stream);

/* Stage 2 for the survivors j < *count (chain i = idx[j]): accept when
 * logu2[i] < (ll_prop[j] - ll_cur[i]) - (lh_prop[i] - lh_cur[i]); an accepted
 * chain copies theta_prop[i] into theta_cur[i], updates ll_cur/lh_cur and
 * increments acc[i]. ll_prop: exact logL of the gathered survivors. */
int argus_da_stage2(const int32_t* idx, const int32_t* count, int64_t cap,
                    const double* ll_prop, const double* lh_prop, const double* logu2,
                    const double* theta_prop, double* theta_cur, double* ll_cur,
                    double* lh_cur, int32_t* acc, int32_t d, void* stream);

/* Device diagnostic for roofline reports (not part of the method): the
 * sustained FP64 FMA rate of the current device with every CU busy
 * (one block per CU, waves_per_simd in 1..4 waves on each SIMD, four
 * independent FMA chains per lane, about 1 ms), in TFLOP/s over the span
 * from the first wave's start to the last wave's end on the device's wall
 * clock, and the mean shader clock over the waves in MHz. The published
 * FP64 peak assumes the maximum engine clock; under full FP64 load the clock
 * settles lower, and this is the rate the FP64-VALU kernels can reach.
 * Allocates and synchronises the stream; -> ARGUS_E_INVAL for bad
 * arguments, ARGUS_E_HIP if the launch or a clock query fails. */
int argus_fp64_rate(int32_t waves_per_simd, double* tflops, double* clock_mhz, void* stream);

/* The same diagnostic for the matrix cores: kind 1 = v_mfma_f64_16x16x4f64
 * (FP64, the joint model's downdate), kind 2 = v_mfma_f32_32x32x16_bf16
 * (BF16 with FP32 accumulation, the surrogate), eight independent
 * accumulators per wave. Allocates and synchronises the stream;
 * -> ARGUS_E_INVAL for a bad kind or waves_per_simd, ARGUS_E_HIP if the
 * launch or a clock query fails. */
int argus_mfma_rate(int32_t kind, int32_t waves_per_simd, double* tflops, double* clock_mhz,
                    void* stream);

/* Device diagnostic for roofline reports (not part of the method): the
 * average duration in ms of the per-pulsar filter kernel alone (models 1, 2,
 * 4; for model 2 its fast form without the general pass over flagged items,
 * and without the reduction over pulsars), launched reps times back to back
 * on `stream` in the layout argus_loglike tuned for this S, between two HIP
 * events. Needs a previous argus_loglike call with this S (else
 * ARGUS_E_INVAL); writes only the handle's workspace; synchronises the
 * stream. Model 3 -> ARGUS_E_UNSUPPORTED. */
int argus_filter_kernel_ms(argus_dataset_t ds, const double* theta, int64_t S, int32_t reps,
                           double* ms, void* stream);

/* Human-readable launch configuration chosen for (ds, S), for reports. */
int argus_tune_info(argus_dataset_t ds, int64_t S, char* buf, int32_t len);

/* Message for the last nonzero return on this thread (part of the error
 * convention above, not of the method); valid until the thread's next call
 * into the library. */
const char* argus_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* ARGUS_H */
