/*
 * yyo.h -- FP64 CPU oracle of the improved Yau-Yau filter step.
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists so that tests, the smoke
 * check and the benchmark's CPU baseline can check the GPU library against a
 * plain, slow, obviously correct implementation written from the paper.  The
 * product path never links, loads or calls it.  It shares no source, header,
 * table or helper with the GPU library.
 *
 * Everything is double precision, host memory, row-major [n x r] node arrays
 * (coordinate k of node i at x[i*r + k]).  Reductions run sequentially in index
 * order; OpenMP is used only across independent target rows of the
 * propagation.  Build with -ffp-contract=off so no multiply-add is fused.
 *
 * Paper: "An Improved Yau-Yau Algorithm for High Dimensional Nonlinear
 * Filtering Problems" (arXiv 2509.16896).  Each function cites the passage it
 * follows.
 */
#ifndef YYO_H
#define YYO_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Problem statement dx = f(x)dt + sqrt(q) dV, dy = h(x)dt + sqrt(rho2) dW
 * (Sec. 2.1, eq. NonlinearFilter; constant isotropic noise a = qI, b = rho2 I
 * of Table tab:generalformulas). */
enum { YYO_F_ZERO = 0, YYO_F_COS = 1, YYO_F_LINEAR = 2, YYO_F_PAPER_SINMIX = 3 };
enum { YYO_H_IDENTITY = 0, YYO_H_CUBE = 1, YYO_H_LINEAR = 2 };

typedef struct {
  int32_t r, m;
  int32_t drift;      /* YYO_F_*; LINEAR: f(x) = A x, A row-major r x r */
  const double* A;
  int32_t obs;        /* YYO_H_*; CUBE: h_k = (x_k - h_shift)^3 (m = r); LINEAR: h = H x, H m x r */
  const double* H;
  double h_shift;
  double q;           /* process-noise variance */
  double rho2;        /* observation-noise variance */
} yyo_model;

/* ---- counter-based random numbers (SplitMix64, Steele, Lea & Flood 2014) ---- */
/* Output number `counter` (0-based) of a SplitMix64 generator started at state `seed`. */
uint64_t yyo_splitmix64_at(uint64_t seed, uint64_t counter);

/* ---- Sobol points (Appendix A, Sobol sequence) ---- */
/* Primitive polynomial number `idx` (0-based) in the enumeration by degree, then
 * by the integer formed by its middle coefficients.  Returns the degree and
 * writes the polynomial as an integer (bit l = coefficient of x^l). */
int yyo_primitive_poly(int idx, uint32_t* poly);
/* Direction numbers v[d*32 + (k-1)], k = 1..32, of dimensions d < r. */
void yyo_sobol_directions(int32_t r, uint32_t* v);
/* 32-bit Sobol codes of points first..first+n-1 in Gray-code order, optionally
 * scrambled (random linear scramble + digital shift keyed by seed). */
void yyo_sobol_codes(int32_t r, int64_t n, int64_t first, int32_t scramble, uint64_t seed,
                     uint32_t* codes);
/* Map codes to the box: x = c + hw*(code*2^-31 - 1), c = (lo+hi)/2, hw = (hi-lo)/2. */
void yyo_codes_to_points(int32_t r, int64_t n, const uint32_t* codes, const double* lo,
                         const double* hi, double* x);
/* 1 if any coordinate is within 1e-12 of a face of the box (Sec. 4.2, boundary conditions). */
int yyo_is_boundary(int32_t r, const double* xi, const double* lo, const double* hi);

/* ---- multi-scale kernel coefficients (Sec. 4.3.3, V c = d) ---- */
/* Solves V c = d for scale divisors s[0..S-1] with error exponents mu_k = (k+2)/2;
 * writes S+1 coefficients (the last multiplies the identity).  Returns 0 on success. */
int yyo_kernel_coefficients(int32_t S, const double* s, double* c);

/* ---- model functions ---- */
void yyo_drift(const yyo_model* mdl, const double* xi, double* fi);
void yyo_obs(const yyo_model* mdl, const double* xi, double* hi);

/* ---- one filter step ---- */
/* Prediction: logw_out_i = log( sum_s c_s dV sum_j N(x_i; x_j + tau_s f(x_j), q tau_s I) e^{logw_in_j}
 *                              + c_{S+1} e^{logw_in_i} ),  tau_s = dt/s_s, dV = vol(box)/n.
 * Non-positive sums and boundary targets give -inf.  Returns the number of clamped rows. */
int64_t yyo_propagate(const yyo_model* mdl, int32_t S, const double* s, const double* c, int64_t n,
                      const double* x, const double* lo, const double* hi, double dt,
                      const double* logw_in, double* logw_out);
/* Same as yyo_propagate but only for the target rows listed in rows[0..nrows-1]. */
int64_t yyo_propagate_rows(const yyo_model* mdl, int32_t S, const double* s, const double* c,
                           int64_t n, const double* x, const double* lo, const double* hi,
                           double dt, const double* logw_in, int64_t nrows, const int64_t* rows,
                           double* out_rows);
/* ---- kernel options: pull form (Sec. 4.1) and general noise coefficients (Sec. 7) ---- */
enum { YYO_FORM_PUSH = 0, YYO_FORM_PULL = 1 };
enum { YYO_DIV_CLOSED = 0, YYO_DIV_COMPLEX_STEP = 1 };
typedef struct {
  int32_t form;          /* PUSH: N(x_i; x_j + tau f(x_j), tau a).  PULL: the kernel of Theorem
                            thm:1storderkernel (eq. kernel) with the noise of Table tab:generalformulas:
                            K_tau(x_i, x_j) = (2 pi tau)^{-r/2} det(a)^{-1/2}
                              exp(-|x_j - x_i + tau f(x_i)|^2_{a^+} / (2 tau) - tau div f(x_i)) */
  int32_t div_mode;      /* PULL: CLOSED (closed-form divergence) or COMPLEX_STEP (Sec. 8) */
  double cs_step;        /* complex step h of Sec. 8 */
  const double* apinv;   /* NULL: a = q I.  Else a^+ (row-major r x r), the Moore-Penrose pseudo-inverse of
                            a = U U^T (its inverse when a is invertible), Sec. 7 */
  double logdet_a;       /* with apinv: log det_+ a, the log of the product of a's positive eigenvalues */
} yyo_kernel;

/* Divergence of the drift at xi: the closed form (mode CLOSED) or the complex-step sum
 * sum_k Im f_k(x + i h e_k) / h of Sec. 8 (mode COMPLEX_STEP). */
double yyo_divergence(const yyo_model* mdl, const double* xi, int32_t mode, double h);

/* Prediction with the kernel options k (NULL: push form, a = q I, which is yyo_propagate):
 *   logw_out_i = log( sum_s c_s dV sum_j K_{tau_s}(x_i, x_j) e^{logw_in_j} + c_{S+1} e^{logw_in_i} ),
 * K the push or pull kernel with variance tau a (a = q I or the given a^+, det_+ a).  The normalising
 * constant is (2 pi tau)^{-r/2} det_+(a)^{-1/2} in both the invertible and the singular case, as the
 * table writes it.  Boundary targets and non-positive sums give -inf; returns the clamped rows. */
int64_t yyo_propagate_ex(const yyo_model* mdl, const yyo_kernel* k, int32_t S, const double* s,
                         const double* c, int64_t n, const double* x, const double* lo, const double* hi,
                         double dt, const double* logw_in, double* logw_out);
int64_t yyo_propagate_rows_ex(const yyo_model* mdl, const yyo_kernel* k, int32_t S, const double* s,
                              const double* c, int64_t n, const double* x, const double* lo,
                              const double* hi, double dt, const double* logw_in, int64_t nrows,
                              const int64_t* rows, double* out_rows);
/* Correction with observation noise b = V V^T (Table tab:generalformulas, online update):
 *   logw_i += h(x_i)^T b^+ dy - dt/2 h(x_i)^T b^+ h(x_i),   bpinv = b^+ row-major m x m. */
void yyo_loglik_update_ex(const yyo_model* mdl, int64_t n, const double* x, const double* dy, double dt,
                          const double* bpinv, double* logw);

/* Correction: logw_i += (h(x_i).dy - dt/2 |h(x_i)|^2) / rho2. */
void yyo_loglik_update(const yyo_model* mdl, int64_t n, const double* x, const double* dy,
                       double dt, double* logw);
/* Normalisation and moments.  logw is replaced by logw - logZ.  w, cov may be NULL.
 * Returns 0, or 1 if every weight is zero. */
int yyo_normalise_moments(int64_t n, int32_t r, const double* x, double* logw, double* w,
                          double* logZ_step, double* logZ_acc, double* mean, double* cov,
                          double* ess);
/* Integer systematic resampling of normalised weights w; writes n ancestor indices. */
int yyo_resample(int64_t n, const double* w, uint64_t seed, int64_t step, int64_t* idx);
/* Local restart (Sec. 6): box [mean - R, mean + R]^r, nodes = the same reference
 * codes mapped to it, prior log-density -|x - mean|^2/2 (boundary nodes -inf). */
void yyo_restart_nodes(int64_t n, int32_t r, const uint32_t* codes, const double* mean, double R,
                       double* lo, double* hi, double* x_new, double* logw_new);

#ifdef __cplusplus
}
#endif
#endif
