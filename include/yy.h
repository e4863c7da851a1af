/*
 * yy.h -- C ABI of libyy, the MI355X (gfx950) implementation of one time step
 * of the improved Yau-Yau filter (arXiv 2509.16896, "An Improved Yau-Yau
 * Algorithm for High Dimensional Nonlinear Filtering Problems").
 *
 * Problem (Sec. 2.1, eq. NonlinearFilter, with the constant isotropic noise
 * coefficients a = q I, b = rho2 I of Table tab:generalformulas):
 *     dx = f(x) dt + sqrt(q) dV,     dy = h(x) dt + sqrt(rho2) dW.
 * The filter keeps log-densities logw[i] at n quasi-random nodes x_i in a box
 * and advances them per step k (Sec. 2.2.2 procedure, Sec. 9 log domain):
 *     propagate  (yy_propagate)          multi-scale Gaussian kernel sum
 *     correct    (yy_loglik_update)      h(x).dy - dt/2 |h(x)|^2, scaled by 1/rho2
 *     normalise  (yy_normalise_moments)  logZ, weights, posterior mean/covariance, ESS
 *     (correct and normalise in one pass over x: yy_loglik_normalise)
 *     restart    (yy_restart)            every few steps, Sec. 6 local restart
 * with nodes from yy_nodes_sobol (Appendix A, Sobol sequence).
 *
 * Conventions for every call:
 *  - Arrays are DEVICE memory owned by the caller unless a comment says host.
 *    Node arrays are row-major [n x r]: coordinate k of node i is x[i*r + k].
 *  - Calls are asynchronous and ordered on the context's stream; outputs are
 *    valid after that stream is synchronised.  Nothing is read back to the
 *    host inside a call, so a sequence of calls can be captured in a graph
 *    once every buffer has been allocated (first call at a given size).
 *  - Every call returns a yy_status and never throws or exits.  Argument
 *    errors are detected on the host before anything is launched; the text
 *    of the last error of the calling thread is returned by yy_last_error().
 *  - Numerical events found on the device (all weights vanished, a negative
 *    multi-scale sum clamped to zero, all resampling weights zero) set bits of
 *    the context's status word, read with yy_get_status().
 *  - Output arrays may not alias input arrays unless the call says in place.
 */
#ifndef YY_H
#define YY_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  YY_OK = 0,
  YY_ERR_ARG = 1,          /* invalid argument (size, pointer, enum value) */
  YY_ERR_ALLOC = 2,        /* device allocation failed */
  YY_ERR_HIP = 3,          /* a HIP runtime call failed; text in yy_last_error() */
  YY_ERR_NUMERIC = 4,      /* reserved for numerical failures reported synchronously */
  YY_ERR_UNSUPPORTED = 5   /* valid but unsupported combination (e.g. r too large) */
} yy_status;

/* Status-word bits (yy_get_status). */
#define YY_FLAG_ALL_ZERO     1u   /* normalisation found every weight zero (-inf) */
#define YY_FLAG_CLAMPED      2u   /* a signed multi-scale sum was <= 0 and was set to -inf */
#define YY_FLAG_RESAMPLE_ZERO 4u  /* resampling weights summed to zero */
#define YY_FLAG_LOW_ESS      8u   /* ESS below the restart's ess_min */
#define YY_FLAG_PROPOSAL_FALLBACK 16u /* a learned restart box failed its checks; the plain box was used */

#define YY_MAX_SCALES 6
#define YY_MAX_R 3600             /* largest state dimension with generated direction numbers */

/* Thread-local text describing the last non-OK status returned on this thread. */
const char* yy_last_error(void);

typedef struct yy_ctx_s* yy_ctx;

/* Creates a context on HIP device `device` that issues all work on `stream`
 * (a hipStream_t; NULL = the device's default stream).  The context owns its
 * scratch buffers and caches; it is not thread safe. */
yy_status yy_create(yy_ctx* out, int device, void* stream);
yy_status yy_destroy(yy_ctx ctx);
/* Changes the stream used by later calls. */
yy_status yy_set_stream(yy_ctx ctx, void* stream);
/* Synchronises the stream, returns the status word and the number of clamped
 * rows accumulated since the last call, and clears both.  Any pointer may be NULL. */
yy_status yy_get_status(yy_ctx ctx, uint32_t* flags, int64_t* nclamped);

/* ------------------------------------------------------------------------ */
/* Model (Sec. 2.1).  Drift f and observation h are chosen from a closed set. */
typedef enum {
  YY_F_ZERO = 0,    /* f(x) = 0 */
  YY_F_COS = 1,     /* f_k(x) = cos(x_k) */
  YY_F_LINEAR = 2,  /* f(x) = A x, A device row-major [r x r] */
  YY_F_PAPER_SINMIX = 3 /* the drift of the large-scale cubic sensor test (Sec. 11,
                         * eq. A&A1): f(x) = sin(x) (A x) + sin(2x) (A1 x) elementwise,
                         * A and A1 upper bidiagonal with diagonal -0.5 / -0.3 and
                         * superdiagonal 0.1 / 0.3: f_k = sin(x_k)(-0.5 x_k + 0.1 x_{k+1})
                         * + sin(2 x_k)(-0.3 x_k + 0.3 x_{k+1}), x_r = 0 */
} yy_drift;

typedef enum {
  YY_H_IDENTITY = 0, /* h(x) = x (m = r) */
  YY_H_CUBE = 1,     /* h_k(x) = (x_k - h_shift)^3 (m = r) */
  YY_H_LINEAR = 2    /* h(x) = H x, H device row-major [m x r] */
} yy_obs;

/* General noise coefficients (Sec. 7, eq. NonlinearFilter_noise, Table tab:generalformulas), created by
 * yy_noise_create; NULL in the model keeps a = q I and b = rho2 I. */
typedef struct yy_noise_s* yy_noise;

typedef struct {
  int32_t r;          /* state dimension, 1 <= r <= YY_MAX_R */
  int32_t m;          /* observation dimension */
  int32_t drift;      /* yy_drift */
  const double* A;    /* device, used when drift == YY_F_LINEAR */
  int32_t obs;        /* yy_obs */
  const double* H;    /* device, used when obs == YY_H_LINEAR */
  double h_shift;
  double q;           /* process-noise variance (> 0; unused where noise gives a) */
  double rho2;        /* observation-noise variance (> 0; unused where noise gives b) */
  yy_noise noise;     /* NULL, or general coefficients a = U U^T and/or b = V V^T */
} yy_model;

/* General noise coefficients for dx = f dt + U dV, dy = h dt + V dW with constant U (r x r) and V
 * (m x m): a = U U^T, b = V V^T, invertible or singular.  Following Sec. 7, the kernel's
 * |.|^2_{a^-1} becomes |.|^2_{a^+} with the Moore-Penrose pseudo-inverse and det a becomes det_+ a
 * (the product of the positive eigenvalues, those above 1e-10 times the largest); the Gaussian
 * constant stays (2 pi tau)^{-r/2} det_+(a)^{-1/2} as the table writes it; the correction becomes
 * h^T b^+ dy - dt/2 h^T b^+ h.  The eigen-decompositions run on the host here, once.  U, V: host
 * row-major [r*r], [m*m], either may be NULL (that coefficient stays isotropic).  The object
 * belongs to ctx's device and must outlive every model that points to it; destroy it before the
 * context.  yy_propagate and yy_loglik_update accept such a model (the batched step does not:
 * YY_ERR_UNSUPPORTED); yy_loglik_normalise then makes the two calls. */
yy_status yy_noise_create(yy_ctx ctx, int32_t r, const double* U, int32_t m, const double* V, yy_noise* out);
yy_status yy_noise_destroy(yy_noise noise);
/* Ranks of a and b (0 where the coefficient stays isotropic) and log det_+ of each; any pointer may be NULL. */
yy_status yy_noise_info(yy_noise noise, int32_t* rank_a, double* logdet_a, int32_t* rank_b, double* logdet_b);

/* Multi-time-scale kernel (Sec. 4.3.3, eq. general_kernel):
 *   K = sum_{j<S} c_j K_{dt/s_j} + c_S delta.
 * s: host array of S distinct positive scale divisors (paper: 1, 2, 4, ...).
 * c: host array of S+1 coefficients, or NULL to solve V c = d with the error
 *    exponents mu_k = (k+2)/2 (the paper's mu_1 = 3/2, mu_2 = 2).
 * form: the first-order kernel K_tau.  YY_FORM_PUSH (0): the Gaussian
 *    N(x_i; x_j + tau f(x_j), tau a) of each source (the transition density of
 *    an Euler step).  YY_FORM_PULL (1): the kernel of Theorem
 *    thm:1storderkernel (eq. kernel, Table tab:generalformulas),
 *    (2 pi tau)^{-r/2} det(a)^{-1/2} exp(-|x_j - x_i + tau f(x_i)|^2_{a^-1} / (2 tau)
 *    - tau div f(x_i)): centred, as a function of the source, at
 *    x_i - tau f(x_i), with the divergence of f at the target.  Both are first
 *    order consistent; the screened forms (BF16X3S, BF16X3P) and the batched
 *    step are push-form only (YY_ERR_UNSUPPORTED).
 * div: pull form: YY_DIV_CLOSED (0) the closed form of the drift's divergence,
 *    YY_DIV_COMPLEX_STEP (1) the complex-step sum of Sec. 8,
 *    sum_k Im f_k(x + i h e_k) / h with h = 1e-20. */
#define YY_FORM_PUSH 0
#define YY_FORM_PULL 1
#define YY_DIV_CLOSED 0
#define YY_DIV_COMPLEX_STEP 1
typedef struct {
  int32_t S;          /* 1 <= S <= YY_MAX_SCALES */
  const double* s;    /* host [S] */
  const double* c;    /* host [S+1] or NULL */
  int32_t form;       /* YY_FORM_PUSH or YY_FORM_PULL */
  int32_t div;        /* YY_DIV_CLOSED or YY_DIV_COMPLEX_STEP (pull form) */
} yy_scales;

/* Solves V c = d of Sec. 4.3.3 on the host (Cramer's rule, as the paper
 * states it).  s: host [S]; c_out: host [S+1]. */
yy_status yy_kernel_coefficients(int32_t S, const double* s, double* c_out);

/* Arithmetic of the pairwise kernel sum in yy_propagate. */
typedef enum {
  YY_PREC_AUTO = 0,      /* VALU for r < 32, BF16X3 otherwise */
  YY_PREC_FP32 = 1,      /* plain FP32: direct differences on the vector ALUs */
  YY_PREC_FP32_MFMA = 2, /* FP32 matrix cores for the distance expansion + exact near pairs */
  YY_PREC_BF16X3 = 3,    /* BF16 hi/lo split (3 products) on matrix cores + exact near pairs */
  YY_PREC_BF16X1 = 4,    /* one BF16 product on matrix cores as a screen + exact near pairs */
  YY_PREC_BF16X3G = 5,   /* BF16X3 for x_i.x_j, one BF16 product for the tau-scaled x_i.f_j */
  YY_PREC_BF16X3S = 6,   /* BF16X3G on the tiles that a screen cannot rule out (below) */
  YY_PREC_BF16X3P = 7    /* BF16X3G on the tiles that a screen on the first 64 coordinates cannot rule out */
} yy_prec;
/* Every matrix-core form keeps each pair whose exponent may lie within 2^-80
 * of its row maximum exact (FP32 direct differences) and drops the others, so
 * all forms agree with YY_PREC_FP32 to FP32 rounding.  In the push form, a row
 * whose self term lies more than 160 bits below the heaviest source weight
 * takes its pair with the heaviest source j* (the first source of maximal
 * weight) in FP64 direct differences, counted once at the start of the row's
 * sum and left out of the tiles and screens.  BF16X3S first runs a
 * screen that forms x_i.x_j with one BF16 product and bounds the tau-scaled
 * x_i.f_j term by |x_i| max_j |f_j|; the split form then visits only the
 * 256-target x 128-source tiles the screen could not rule out.  BF16X3P
 * screens on the first 64 coordinates alone: a sum of squares over some of
 * the coordinates is a lower bound of the squared distance over all of them,
 * so a pair whose partial distance already puts it 2^-80 below the exact
 * self-pair exponent of its row is negligible.  Its screen moves and
 * multiplies 64 of the r coordinates; where the partial distance does not
 * separate the nodes it flags more tiles than the BF16X3S screen, and the
 * result is the same.  Where r > 32 and n > 8192 (more than 32 blocks of 256
 * targets), single runs and runs of a batch alike, the BF16X3P screen forms
 * the products of each pair of target blocks once and judges both
 * orientations from them (the transposed one by a bound per 64 rows, with the
 * doubtful groups rechecked row by row); the flags it raises are those a
 * one-sided screen would raise or more, never fewer, so the result is the
 * same. */

/* ------------------------------------------------------------------------ */
/* Sobol nodes (Appendix A; Sec. 2.2.1 state sampling; Sec. 6 reference set).
 * Points first_index .. first_index+n-1 of the r-dimensional Sobol sequence in
 * Gray-code order, 32-bit codes, optionally scrambled by a random linear
 * (Matousek) scramble plus digital shift keyed by `seed`, mapped to the box:
 *   x[i*r+k] = c_k + hw_k * (code * 2^-31 - 1),  c = (lo+hi)/2, hw = (hi-lo)/2,
 * in double precision without fused multiply-add.
 *   box_lo, box_hi: device [r]; codes: device [n*r] uint32 or NULL;
 *   x: device [n*r] double or NULL.  first_index + n <= 2^32. */
yy_status yy_nodes_sobol(yy_ctx ctx, int32_t r, int64_t n, int64_t first_index, int32_t scramble,
                         uint64_t seed, const double* box_lo, const double* box_hi, uint32_t* codes,
                         double* x);

/* Prediction (Sec. 4 kernel operator, push form; Sec. 9 log-domain prediction).
 *   logw_out[i] = log( sum_s c_s dV sum_j N(x_i; x_j + tau_s f(x_j), q tau_s I) exp(logw_in[j])
 *                      + c_S exp(logw_in[i]) ),   tau_s = dt / s_s,  dV = vol(box) / n.
 * Nodes within 1e-12 of a face of the box (Sec. 4.2, boundary conditions) are
 * excluded as sources and get -inf as targets; a sum <= 0 (possible because
 * some c_s < 0) gives -inf and sets YY_FLAG_CLAMPED.
 *   x: device [n*r] double, the node set; node_version: any value that
 *   changes whenever x or the box change (the context caches the prepared
 *   node set under (x, n, r, drift, node_version)); box_lo/hi: device [r];
 *   logw_in, logw_out: device [n] double, must not alias. */
yy_status yy_propagate(yy_ctx ctx, const yy_model* model, const yy_scales* scales, int32_t prec,
                       int64_t n, const double* x, uint64_t node_version, const double* box_lo,
                       const double* box_hi, double dt, const double* logw_in, double* logw_out);

/* The prediction as a stored operator: the offline / online split of Sec. 10 (the operator
 * matrix of Sec. 4.2, steps 2-3, assembled once; step 5, its product with the weights, every
 * step), in the log domain of Sec. 9.
 * yy_operator_build stores, for the node set x (and model, scales, dt, box as yy_propagate takes
 * them, push or pull form, isotropic or general noise), every kernel value per scale as an FP32
 * base-2 exponent without the weights, E[s][i][j] (FP32 direct differences, the arithmetic of
 * YY_PREC_FP32): S n ceil(n/64)*64 x 4 bytes of device memory (yy_operator_info).  *op: NULL to
 * create a new operator, or one built before on this context to rebuild in place (its memory is
 * reused when large enough).  yy_operator_apply then gives exactly the prediction yy_propagate
 * computes (same combination, constants, boundary rows and clamp; FP32 rounding of the stored
 * exponents), reading the stored operator once: logw_in, logw_out device [n], must not alias.
 * The operator must be destroyed before its context. */
typedef struct yy_operator_s* yy_operator;
yy_status yy_operator_build(yy_ctx ctx, const yy_model* model, const yy_scales* scales, int64_t n, const double* x,
                            uint64_t node_version, const double* box_lo, const double* box_hi, double dt,
                            yy_operator* op);
yy_status yy_operator_apply(yy_operator op, const double* logw_in, double* logw_out);
/* Nodes, scales and device bytes of the stored exponents; any pointer may be NULL. */
yy_status yy_operator_info(yy_operator op, int64_t* n, int32_t* S, int64_t* bytes);
yy_status yy_operator_destroy(yy_operator op);

/* Correction with the Ito term (Sec. 2.2 online stage; Sec. 9 observation
 * update; 1/rho2 from Table tab:generalformulas), in place:
 *   logw[i] += ( h(x_i) . dy - dt/2 |h(x_i)|^2 ) / rho2      (-inf stays -inf)
 *   x: device [n*r]; dy: device [m]; logw: device [n]. */
yy_status yy_loglik_update(yy_ctx ctx, const yy_model* model, int64_t n, const double* x,
                           const double* dy, double dt, double* logw);

/* Normalisation and estimation (Sec. 2.2.2 step 4; Sec. 9 normalisation), in
 * double precision with fixed-order reductions:
 *   logZ = LSE_i logw[i];  logw[i] -= logZ (in place);  w[i] = exp(logw[i]);
 *   mean = sum_i w_i x_i;  cov = sum_i w_i (x_i - mean)(x_i - mean)^T;
 *   ess = 1 / sum_i w_i^2;  *logZ_acc += logZ.
 *   w: device [n] or NULL; logZ_step, logZ_acc (read-modify-write), ess:
 *   device scalars; mean: device [r] or NULL (then x is not read, and cov
 *   must be NULL); cov: device [r*r] or NULL.
 * If every weight is -inf, YY_FLAG_ALL_ZERO is set and the outputs are left
 * unchanged except logZ_step = -inf. */
yy_status yy_normalise_moments(yy_ctx ctx, int64_t n, int32_t r, const double* x, double* logw,
                               double* w, double* logZ_step, double* logZ_acc, double* mean,
                               double* cov, double* ess);

/* yy_normalise_moments without any device allocation, for callers that cannot
 * allocate (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Same arguments, kernels and results (bit for bit) as
 * yy_normalise_moments; its per-block partial sums live in a static device
 * array of (1024 (3 + YY_NOALLOC_MAX_R) + 4) doubles (about 8 MiB), one per
 * GPU, held until the process ends.  Limits: r <= YY_NOALLOC_MAX_R
 * (YY_ERR_UNSUPPORTED otherwise, nothing launched); cov requires the caller's
 * w.  Every call on a GPU shares that GPU's array, so calls on one GPU whose
 * work overlaps (different streams or threads) race; calls ordered on one
 * stream do not.  The array is located at yy_create. */
#define YY_NOALLOC_MAX_R 1024
yy_status yy_normalise_moments_noalloc(yy_ctx ctx, int64_t n, int32_t r, const double* x, double* logw,
                                       double* w, double* logZ_step, double* logZ_acc, double* mean,
                                       double* cov, double* ess);

/* The correction and the normalisation of one step in one call (Sec. 2.2.2
 * steps 3 and 4): the results of yy_loglik_update followed by
 * yy_normalise_moments with cov = NULL.  Where h is componentwise (m = r), r
 * is even and at most 1024 and x and dy are 16-byte aligned, x is read once:
 * each node's updated log-weight enters the weight and mean sums at once,
 * relative to a running maximum (the log-weights are those of
 * yy_loglik_update; logZ, w, mean and ess agree with the two calls to FP64
 * rounding).  Otherwise the call makes the two calls.  Arguments as there;
 * mean and ess are required, w may be NULL. */
yy_status yy_loglik_normalise(yy_ctx ctx, const yy_model* model, int64_t n, const double* x,
                              const double* dy, double dt, double* logw, double* w, double* logZ_step,
                              double* logZ_acc, double* mean, double* ess);

/* Learned restart proposal (not in the paper; the plain restart of Sec. 6 is
 * its fallback).  A multilayer perceptron maps the estimate x_hat (r) through
 * Linear(r, H) -> GELU -> Linear(H, H) -> GELU -> Linear(H, 2r) to (delta, u);
 * GELU is the exact form x Phi(x).  The proposed restart box is centred at
 * x_hat + delta with half-width R exp(u) per coordinate, read as +-3 standard
 * deviations of a diagonal Gaussian s = (R/3) exp(u).  Weights and arithmetic
 * are FP32.  Parameter vector layout (device, FP32): W1 [H x r] row-major,
 * b1 [H], W2 [H x H], b2 [H], W3 [2r x H], b3 [2r]. */
typedef struct yy_proposal_s* yy_proposal;

/* Creates a proposal network on ctx's device; it runs on ctx's stream.
 * params: device [P] initial parameters, or NULL for the default
 * initialisation (W1, W2 uniform in +-1/sqrt(fan_in) from SplitMix64 keyed by
 * seed, b1 = b2 = 0, W3 = b3 = 0 so that the first proposal is the plain box).
 * 1 <= r <= YY_MAX_R, 1 <= hidden <= 1024.  The network must be destroyed
 * before its context. */
yy_status yy_proposal_create(yy_ctx ctx, int32_t r, int32_t hidden, uint64_t seed, const float* params,
                             yy_proposal* out);
yy_status yy_proposal_destroy(yy_proposal p);
/* Number of parameters P = H r + H + H^2 + H + 2 r H + 2 r (host scalar). */
yy_status yy_proposal_num_params(yy_proposal p, int64_t* P);
/* Copies the parameters to / from device [P]; set_params also resets the
 * Adam moments and step count. */
yy_status yy_proposal_get_params(yy_proposal p, float* params);
yy_status yy_proposal_set_params(yy_proposal p, const float* params);
/* Network outputs for B estimates: xhat device [B*r] (FP64, converted to
 * FP32), out device [B*2r] (delta then u per row). */
yy_status yy_proposal_forward(yy_proposal p, int32_t B, const double* xhat, float* out);
/* One training step on B pairs (x_hat of a restart, per-coordinate mean mu
 * and variance var of the posterior samples at the next restart; device
 * [B*r] FP64 each).  Loss = mean over pairs and coordinates of
 *   (var + 0.01 (R/3)^2 + (mu - x_hat - delta)^2) / (2 s^2) + log s,
 * the Gaussian negative log-likelihood of the samples without the constant
 * (1/2) log(2 pi), with a variance floor.  Writes the loss (device FP64
 * scalar, nullable) and the gradient (device [P] FP32, nullable); when
 * update != 0 applies one Adam step (beta1 0.9, beta2 0.999, eps 1e-8,
 * bias-corrected) with learning rate lr. */
yy_status yy_proposal_train_step(yy_proposal p, int32_t B, const double* xhat, const double* mu,
                                 const double* var, double R, double lr, int32_t update, double* loss,
                                 float* grad);

/* Per-coordinate mean and (1/n) variance of the resampled nodes x[idx[t]],
 * t < n (FP64, two passes): the posterior samples a restart produces, used as
 * training targets of the proposal.  x: device [n*r]; idx: device [n];
 * mean, var: device [r]. */
yy_status yy_sample_moments(yy_ctx ctx, int64_t n, int32_t r, const double* x, const int64_t* idx,
                            double* mean, double* var);

/* Local resample-restart (Sec. 6). */
typedef struct {
  double R;           /* half-width of the plain box [mean - R, mean + R]^r */
  double ess_min;     /* YY_FLAG_LOW_ESS is set when ess < ess_min (ess: device scalar or NULL);
                         also the learned box's minimum prior ESS */
  uint64_t seed;      /* key of the resampling random numbers */
  yy_proposal proposal; /* NULL: plain restart; else the learned box with fallback */
  double cover_min;   /* learned box: minimum fraction of sample coordinates inside it */
} yy_restart_params;

/* (1) Integer systematic resampling of the normalised weights w into ancestor
 *     indices idx (W_i = floor(w_i 2^53), C = prefix sums, U = 32 bits of
 *     SplitMix64 keyed by (seed, step), P_t = floor((t 2^32 + U) W / (n 2^32)),
 *     idx[t] = min{i : C_i > P_t}).  idx may be NULL to skip it.
 * (2) The new box: with params->proposal NULL, [mean - R, mean + R]^r (the
 *     plain restart of Sec. 6).  With a proposal, the learned box is used
 *     when (a) at least cover_min of the coordinates of the samples
 *     x_cur[idx[t]] lie inside it, (b) the samples' mean log-density under its
 *     Gaussian is at least that under the plain box's (s = R/3), and (c) the
 *     prior ESS of the new nodes is at least ess_min; otherwise the plain box
 *     is used and YY_FLAG_PROPOSAL_FALLBACK is set.  The box goes to
 *     box_lo/box_hi, and the new nodes x_new = the reference codes mapped to
 *     it (the pre-generated reference set translated to the estimate, Sec. 6).
 * (3) Prior logw_new[i] = -|x_new_i - mean|^2 / 2 (the initial density
 *     N(mean, I) up to a constant), -inf for boundary nodes; not normalised.
 *   codes: device [n*r]; x_cur: device [n*r] (needed with a proposal, may be
 *   NULL otherwise; must not alias x_new); w: device [n]; mean: device [r];
 *   ess: device scalar or NULL; idx: device [n] int64 (required with a
 *   proposal) or NULL; box_lo/hi: device [r]; x_new: device [n*r];
 *   logw_new: device [n]; used: device int32 scalar or NULL, set to 1 when the
 *   learned box was used, else 0. */
yy_status yy_restart(yy_ctx ctx, int64_t n, int32_t r, const uint32_t* codes, const double* x_cur,
                     const double* w, const double* mean, const double* ess, int64_t step,
                     const yy_restart_params* params, int64_t* idx, double* box_lo, double* box_hi,
                     double* x_new, double* logw_new, int32_t* used);

/* ------------------------------------------------------------------------ */
/* Autotuner of the matrix-core pairwise kernel (not in the paper).  For each
 * shape (r[t], n[t]) it builds a synthetic node set (scrambled Sobol nodes in
 * [-1, 1]^r, f = cos, h = x^3, q = rho2 = 0.09, dt = 0.01, uniform weights),
 * times the pairwise kernel of yy_propagate with the given scales and form
 * for 1, 2, 4, ... source splits (up to the number of 128-source tiles, at
 * most 256), `reps` launches each after one warm-up, and records the fastest
 * count in ctx's table; later yy_propagate calls whose padded shape, scale
 * count and form match use it.  nsplit_out: host [count] or NULL.  Not while
 * the stream is being captured. */
yy_status yy_tune(yy_ctx ctx, int32_t count, const int32_t* r, const int64_t* n, const yy_scales* scales,
                  int32_t prec, int32_t reps, int32_t* nsplit_out);

/* ------------------------------------------------------------------------ */
/* Batched filter (not in the paper): many independent filter runs stepped
 * together.  Every kernel of a step is one launch over all runs (each run's
 * block range runs the single-run kernel on the run's arguments, so every run
 * computes exactly what the single-run calls compute); the pairwise kernel
 * takes the work items (run, target block, source split) of all runs in
 * decreasing-cost order.  A step is the prediction (Sec. 4, push form), the
 * log-likelihood update (Sec. 2.2.2), the normalisation and, every
 * restart_every steps (not after the last), the plain restart (Sec. 6); step
 * counters and restart flags live on the device.  The batch owns one context
 * per run on ctx's stream. */
typedef struct {
  yy_model model;          /* f, h, noise of the run (A/H device pointers stay owned by the caller) */
  int64_t n;               /* nodes, 1 .. 2^31 */
  double dt;
  double box_half;         /* initial box [-box_half, box_half]^r, density N(0, I) */
  double R;                /* restart half-width */
  int32_t restart_every;   /* 0: never */
  int32_t K;               /* steps, the same for all runs of a batch */
  uint64_t seed;           /* Sobol scramble and resampling key */
  const double* dys;       /* observation increments: device [K*m] FP64 */
} yy_batch_run;
typedef struct yy_batch_s* yy_batch;

/* Creates the batch and its initial state (step 0: nodes, N(0, I) prior,
 * normalised).  prec: a matrix-core form (YY_PREC_FP32_MFMA, BF16X3, BF16X3G,
 * BF16X3S, BF16X3P or BF16X1).  Each run takes its pairwise sum in that form
 * (the default) or in the plain FP32 form on the vector ALUs (YY_PREC_FP32), as
 * yy_batch_tune (with forms) or yy_batch_set_run_form choose; either way a run
 * computes exactly what the single-run calls compute in its form.  In a
 * BF16X3P batch a run may also take YY_PREC_BF16X3G: BF16X3P's plan with no
 * screen and every tile flagged, i.e. the split form on every tile summed in
 * BF16X3P's order (row floor and the pair with the heaviest source first).  It
 * differs from the single-run BF16X3P call only by the tiles that call's screen
 * drops, whose pairs lie more than 2^-80 below their row's floor, so the
 * results agree to rounding (where the screen spans only 32 coordinates it
 * flags most tiles, and skipping it is faster).
 * max_split: upper bound of the source splits per matrix-core run (0: 16);
 * yy_batch_tune can choose it. */
yy_status yy_batch_create(yy_ctx ctx, int32_t nruns, const yy_batch_run* runs, const yy_scales* scales,
                          int32_t prec, int32_t max_split, yy_batch* out);
yy_status yy_batch_destroy(yy_batch b);
/* Back to step 0 (same nodes and priors as after creation). */
yy_status yy_batch_reset(yy_batch b);
/* One step of every run (error once K steps are taken). */
yy_status yy_batch_step(yy_batch b);
/* Steps every run up to step k_end (<= K) through a HIP graph of two
 * consecutive steps, captured on first use (per parity of the next step) and
 * launched (k_end - k)/2 times; an odd remainder runs eagerly.  ctx's stream
 * must be a created stream (not the null stream) and timing must be off. */
yy_status yy_batch_run_graph(yy_batch b, int32_t k_end);
/* Tunes the pairwise launches on the current state (reps launches per
 * candidate after a warm-up; results discarded): with forms != 0 first each
 * run's form, by timing its single-run pairwise call in the batch's
 * matrix-core form and in the candidates that the bits of forms name: bit 0
 * YY_PREC_FP32, bit 1 (BF16X3P batches) YY_PREC_BF16X3G, timed as the
 * single-run BF16X3G call (runs of equal r and n share one decision; the
 * screened forms' cost depends on the weights, so tune on a state a few steps
 * in); then max_split = 1, 2, 4, ..., 64 on the batched launch.  Keeps the
 * fastest; best_out (host scalar or NULL) receives max_split.  Drops a
 * captured graph. */
yy_status yy_batch_tune(yy_batch b, int32_t reps, int32_t forms, int32_t* best_out);
/* The pairwise form of run `run`: the batch's matrix-core form, YY_PREC_FP32
 * or (BF16X3P batches) YY_PREC_BF16X3G (host scalar). */
yy_status yy_batch_run_form(yy_batch b, int32_t run, int32_t* prec);
/* Sets run `run`'s pairwise form (the batch's form, YY_PREC_FP32, or in a
 * BF16X3P batch YY_PREC_BF16X3G) and
 * rebuilds the launches; the run continues from its current state.  Drops a
 * captured graph; YY_ERR_UNSUPPORTED while the stream is capturing. */
yy_status yy_batch_set_run_form(yy_batch b, int32_t run, int32_t prec);
/* Results of run `run` so far: per-step posterior mean (device [K*r]), log
 * normaliser logZ_k (device [K]) and ESS (device [K]); each nullable.  Copies
 * on ctx's stream. */
yy_status yy_batch_results(yy_batch b, int32_t run, double* mean_hist, double* logZ_hist, double* ess_hist);
/* Steps taken so far (host scalar). */
yy_status yy_batch_step_count(yy_batch b, int32_t* k);
/* yy_screen_count for run `run` of a batch in a screened form (its last
 * propagation).  Synchronises the stream; YY_ERR_ARG for a bad run or a form
 * without a screen. */
yy_status yy_batch_screen_count(yy_batch b, int32_t run, int64_t* flagged, int64_t* tiles);

/* ------------------------------------------------------------------------ */
/* Timing of the pairwise kernel (the dominant kernel of yy_propagate).  While
 * enabled, each yy_propagate records a pair of HIP events on the context's
 * stream around its pairwise kernel.  yy_timing_read synchronises the stream,
 * returns the summed kernel time in milliseconds and the number of timed
 * launches since the last read, and resets both.  Do not enable it while a
 * graph is being captured. */
yy_status yy_timing_enable(yy_ctx ctx, int32_t on);
yy_status yy_timing_read(yy_ctx ctx, double* ms, int64_t* launches);

/* The screen of the last BF16X3S or BF16X3P propagation on this context (a
 * diagnostic of the screened split forms): *tiles = (256-target block,
 * 128-source tile) pairs, *flagged = those recomputed in the split form
 * because some pair in them may lie within 2^-80 of its row maximum.
 * Synchronises the context's stream; YY_ERR_ARG if no screened propagation
 * ran on it. */
yy_status yy_screen_count(yy_ctx ctx, int64_t* flagged, int64_t* tiles);

#ifdef __cplusplus
}
#endif
#endif /* YY_H */
