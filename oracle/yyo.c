/*
 * yyo.c -- FP64 CPU oracle of the improved Yau-Yau filter step.
 *
 * TEST INFRASTRUCTURE ONLY (tests, smoke check, CPU baseline of the benchmark).
 * Plain loops, double precision, sequential reductions in index order; OpenMP
 * only across independent target rows of the propagation.  Compiled with
 * -ffp-contract=off.  Shares nothing with the GPU library.
 */
#include "yyo.h"

#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

#define YYO_BOUNDARY_TOL 1e-12      /* Sec. 4.2, step 3: omega = 1e-12 */
#define YYO_DIR_SEED 0x59A0D1CE5EED0001ULL  /* project constant for the initial direction numbers */
#define YYO_DOMAIN_SCRAMBLE 1ULL
#define YYO_DOMAIN_RESAMPLE 2ULL

/* ------------------------------------------------------------------------- */
/* SplitMix64: state advances by the golden gamma, output is the 64-bit mix.  */
uint64_t yyo_splitmix64_at(uint64_t seed, uint64_t counter) {
  uint64_t z = seed + (counter + 1ULL) * 0x9E3779B97F4A7C15ULL;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

/* ------------------------------------------------------------------------- */
/* Primitive polynomials over GF(2).  A polynomial P of degree s with nonzero
 * constant term is primitive iff x has multiplicative order 2^s - 1 modulo P,
 * i.e. x^(2^s-1) = 1 and x^((2^s-1)/q) != 1 for every prime q | 2^s-1.        */
static uint64_t gf2_mulmod(uint64_t a, uint64_t b, uint64_t p, int deg) {
  uint64_t res = 0;
  while (b) {
    if (b & 1ULL) res ^= a;
    b >>= 1;
    a <<= 1;
    if ((a >> deg) & 1ULL) a ^= p;
  }
  return res;
}

static uint64_t gf2_xpow(uint64_t e, uint64_t p, int deg) {
  uint64_t base = 2ULL;  /* the polynomial x */
  if ((base >> deg) & 1ULL) base ^= p;
  uint64_t res = 1ULL;
  while (e) {
    if (e & 1ULL) res = gf2_mulmod(res, base, p, deg);
    base = gf2_mulmod(base, base, p, deg);
    e >>= 1;
  }
  return res;
}

static int gf2_is_primitive(uint64_t p, int deg) {
  uint64_t N = (1ULL << deg) - 1ULL;
  if (gf2_xpow(N, p, deg) != 1ULL) return 0;
  uint64_t m = N;
  for (uint64_t q = 2; q * q <= m; ++q) {
    if (m % q == 0) {
      if (gf2_xpow(N / q, p, deg) == 1ULL) return 0;
      while (m % q == 0) m /= q;
    }
  }
  if (m > 1) {
    if (gf2_xpow(N / m, p, deg) == 1ULL) return 0;
  }
  return 1;
}

/* Enumerate primitive polynomials by degree, then by middle coefficients. */
static int enumerate_primitive(int count, uint32_t* polys, int* degs) {
  int found = 0;
  for (int deg = 1; deg <= 31 && found < count; ++deg) {
    for (uint64_t a = 0; a < (1ULL << (deg - 1)) && found < count; ++a) {
      uint64_t p = (1ULL << deg) | (a << 1) | 1ULL;
      if (gf2_is_primitive(p, deg)) {
        polys[found] = (uint32_t)p;
        degs[found] = deg;
        ++found;
      }
    }
  }
  return found;
}

int yyo_primitive_poly(int idx, uint32_t* poly) {
  uint32_t* polys = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)(idx + 1));
  int* degs = (int*)malloc(sizeof(int) * (size_t)(idx + 1));
  int got = enumerate_primitive(idx + 1, polys, degs);
  int deg = -1;
  if (got == idx + 1) {
    *poly = polys[idx];
    deg = degs[idx];
  }
  free(polys);
  free(degs);
  return deg;
}

/* Direction numbers (Appendix A, Sobol sequence; Bratley-Fox recurrence).
 * Dimension 0 is the van der Corput sequence (all m_k = 1).  Dimension d >= 1
 * uses primitive polynomial d-1 of degree s, x^s + a_1 x^{s-1} + ... + a_{s-1} x + 1,
 * with odd initial values m_k < 2^k (k <= s) drawn from SplitMix64 and
 * m_k = m_{k-s} ^ (m_{k-s} << s) ^ XOR_{l<s} a_l (m_{k-l} << l) for k > s.
 * v_k = m_k * 2^(32-k).                                                     */
void yyo_sobol_directions(int32_t r, uint32_t* v) {
  uint32_t* polys = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)(r > 1 ? r : 1));
  int* degs = (int*)malloc(sizeof(int) * (size_t)(r > 1 ? r : 1));
  if (r > 1) enumerate_primitive(r - 1, polys, degs);
  for (int32_t d = 0; d < r; ++d) {
    uint64_t m[33];
    if (d == 0) {
      for (int k = 1; k <= 32; ++k) m[k] = 1ULL;
    } else {
      uint32_t p = polys[d - 1];
      int s = degs[d - 1];
      uint64_t state = yyo_splitmix64_at(YYO_DIR_SEED, (uint64_t)d);
      for (int k = 1; k <= s && k <= 32; ++k)
        m[k] = (yyo_splitmix64_at(state, (uint64_t)(k - 1)) >> (64 - k)) | 1ULL;
      for (int k = s + 1; k <= 32; ++k) {
        uint64_t val = m[k - s] ^ (m[k - s] << s);
        for (int l = 1; l < s; ++l) {
          uint64_t a_l = (p >> (s - l)) & 1U;
          if (a_l) val ^= (m[k - l] << l);
        }
        m[k] = val;
      }
    }
    for (int k = 1; k <= 32; ++k) v[(size_t)d * 32 + (k - 1)] = (uint32_t)(m[k] << (32 - k));
  }
  free(polys);
  free(degs);
}

/* Random linear scramble (unit lower-triangular in digit order) + digital shift. */
static void scramble_params(uint64_t seed, int32_t d, uint32_t* rows, uint32_t* shift) {
  uint64_t state = yyo_splitmix64_at(yyo_splitmix64_at(seed, YYO_DOMAIN_SCRAMBLE), (uint64_t)d);
  for (int p = 31; p >= 0; --p) {
    uint64_t rnd = yyo_splitmix64_at(state, (uint64_t)(31 - p)) >> 32;
    rows[p] = (uint32_t)(((rnd >> p) << p) | (1ULL << p));
  }
  *shift = (uint32_t)(yyo_splitmix64_at(state, 32) >> 32);
}

static uint32_t parity32(uint32_t x) {
  uint32_t par = 0;
  while (x) {
    par ^= (x & 1U);
    x >>= 1;
  }
  return par;
}

void yyo_sobol_codes(int32_t r, int64_t n, int64_t first, int32_t scramble, uint64_t seed,
                     uint32_t* codes) {
  uint32_t* v = (uint32_t*)malloc(sizeof(uint32_t) * 32 * (size_t)r);
  yyo_sobol_directions(r, v);
  uint32_t* rows = (uint32_t*)malloc(sizeof(uint32_t) * 32 * (size_t)r);
  uint32_t* shifts = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)r);
  for (int32_t d = 0; d < r; ++d) scramble_params(seed, d, rows + 32 * (size_t)d, shifts + d);
  for (int64_t t = 0; t < n; ++t) {
    uint64_t i = (uint64_t)(first + t);
    uint64_t g = i ^ (i >> 1);  /* Gray code of the index */
    for (int32_t d = 0; d < r; ++d) {
      uint32_t code = 0;
      for (int k = 1; k <= 32; ++k)
        if ((g >> (k - 1)) & 1ULL) code ^= v[(size_t)d * 32 + (k - 1)];
      if (scramble) {
        uint32_t out = 0;
        for (int p = 0; p < 32; ++p) out |= parity32(rows[32 * (size_t)d + p] & code) << p;
        code = out ^ shifts[d];
      }
      codes[(size_t)t * r + d] = code;
    }
  }
  free(v);
  free(rows);
  free(shifts);
}

void yyo_codes_to_points(int32_t r, int64_t n, const uint32_t* codes, const double* lo,
                         const double* hi, double* x) {
  for (int64_t i = 0; i < n; ++i)
    for (int32_t k = 0; k < r; ++k) {
      double c = 0.5 * (lo[k] + hi[k]);
      double hw = 0.5 * (hi[k] - lo[k]);
      double u = (double)codes[(size_t)i * r + k] * 0x1p-31 - 1.0;
      x[(size_t)i * r + k] = c + hw * u;
    }
}

int yyo_is_boundary(int32_t r, const double* xi, const double* lo, const double* hi) {
  for (int32_t k = 0; k < r; ++k)
    if (fabs(xi[k] - lo[k]) <= YYO_BOUNDARY_TOL || fabs(hi[k] - xi[k]) <= YYO_BOUNDARY_TOL)
      return 1;
  return 0;
}

/* ------------------------------------------------------------------------- */
/* V c = d (Sec. 4.3.3): row 0 all ones (constant term), row 1 s_j^-1 and 0 for
 * the identity column (dt term), rows 1+k, k = 1..S-1, s_j^-mu_k and 0
 * (eliminated error orders), mu_k = (k+2)/2 as in the paper's example
 * (mu_1 = 3/2, mu_2 = 2).  d = (1, 1, 0, ..., 0).  Gaussian elimination with
 * partial pivoting.                                                          */
int yyo_kernel_coefficients(int32_t S, const double* s, double* c) {
  int N = S + 1;
  double V[16][17];
  if (S < 1 || S > 15) return 1;
  for (int row = 0; row < N; ++row)
    for (int col = 0; col <= N; ++col) V[row][col] = 0.0;
  for (int j = 0; j < N; ++j) V[0][j] = 1.0;
  V[0][N] = 1.0;
  for (int j = 0; j < S; ++j) V[1][j] = 1.0 / s[j];
  V[1][N] = 1.0;
  for (int k = 1; k <= S - 1; ++k) {
    double mu = (k + 2) / 2.0;
    for (int j = 0; j < S; ++j) V[1 + k][j] = pow(s[j], -mu);
    V[1 + k][N] = 0.0;
  }
  for (int col = 0; col < N; ++col) {
    int piv = col;
    for (int row = col + 1; row < N; ++row)
      if (fabs(V[row][col]) > fabs(V[piv][col])) piv = row;
    if (V[piv][col] == 0.0) return 2;
    if (piv != col)
      for (int k = 0; k <= N; ++k) {
        double t = V[col][k];
        V[col][k] = V[piv][k];
        V[piv][k] = t;
      }
    for (int row = col + 1; row < N; ++row) {
      double f = V[row][col] / V[col][col];
      for (int k = col; k <= N; ++k) V[row][k] -= f * V[col][k];
    }
  }
  for (int row = N - 1; row >= 0; --row) {
    double acc = V[row][N];
    for (int k = row + 1; k < N; ++k) acc -= V[row][k] * c[k];
    c[row] = acc / V[row][row];
  }
  return 0;
}

/* ------------------------------------------------------------------------- */
void yyo_drift(const yyo_model* mdl, const double* xi, double* fi) {
  int32_t r = mdl->r;
  for (int32_t k = 0; k < r; ++k) {
    if (mdl->drift == YYO_F_ZERO) {
      fi[k] = 0.0;
    } else if (mdl->drift == YYO_F_COS) {
      fi[k] = cos(xi[k]);
    } else if (mdl->drift == YYO_F_PAPER_SINMIX) {
      /* Sec. 11, large-scale test: sin(x) (A x) + sin(2x) (A1 x) with the
       * bidiagonal A (-0.5 on the diagonal, 0.1 above) and A1 (-0.3, 0.3) */
      const double next = k + 1 < r ? xi[k + 1] : 0.0;
      const double ax = -0.5 * xi[k] + 0.1 * next;
      const double a1x = -0.3 * xi[k] + 0.3 * next;
      fi[k] = sin(xi[k]) * ax + sin(2.0 * xi[k]) * a1x;
    } else {
      double acc = 0.0;
      for (int32_t l = 0; l < r; ++l) acc += mdl->A[(size_t)k * r + l] * xi[l];
      fi[k] = acc;
    }
  }
}

void yyo_obs(const yyo_model* mdl, const double* xi, double* hi) {
  for (int32_t k = 0; k < mdl->m; ++k) {
    if (mdl->obs == YYO_H_IDENTITY) {
      hi[k] = xi[k];
    } else if (mdl->obs == YYO_H_CUBE) {
      double t = xi[k] - mdl->h_shift;
      hi[k] = t * t * t;
    } else {
      double acc = 0.0;
      for (int32_t l = 0; l < mdl->r; ++l) acc += mdl->H[(size_t)k * mdl->r + l] * xi[l];
      hi[k] = acc;
    }
  }
}

/* ------------------------------------------------------------------------- */
/* Divergence of the drift (needed by the pull-form kernel, eq. kernel).      */
static double complex drift_component_cplx(const yyo_model* mdl, const double* xi, int32_t k, double h) {
  /* f_k at x + i h e_k: only coordinate k carries the imaginary step */
  int32_t r = mdl->r;
  double complex z = xi[k] + I * h;
  if (mdl->drift == YYO_F_ZERO) return 0.0;
  if (mdl->drift == YYO_F_COS) return ccos(z);
  if (mdl->drift == YYO_F_PAPER_SINMIX) {
    const double next = k + 1 < r ? xi[k + 1] : 0.0;
    return csin(z) * (-0.5 * z + 0.1 * next) + csin(2.0 * z) * (-0.3 * z + 0.3 * next);
  }
  double complex acc = 0.0;
  for (int32_t l = 0; l < r; ++l) acc += mdl->A[(size_t)k * r + l] * (l == k ? z : (double complex)xi[l]);
  return acc;
}

double yyo_divergence(const yyo_model* mdl, const double* xi, int32_t mode, double h) {
  int32_t r = mdl->r;
  double div = 0.0;
  for (int32_t k = 0; k < r; ++k) {
    if (mode == YYO_DIV_COMPLEX_STEP) {
      div += cimag(drift_component_cplx(mdl, xi, k, h)) / h;
    } else if (mdl->drift == YYO_F_COS) {
      div += -sin(xi[k]);
    } else if (mdl->drift == YYO_F_PAPER_SINMIX) {
      /* d/dx_k of sin(x_k)(-0.5 x_k + 0.1 x_{k+1}) + sin(2 x_k)(-0.3 x_k + 0.3 x_{k+1}) */
      const double next = k + 1 < r ? xi[k + 1] : 0.0;
      div += cos(xi[k]) * (-0.5 * xi[k] + 0.1 * next) - 0.5 * sin(xi[k]) +
             2.0 * cos(2.0 * xi[k]) * (-0.3 * xi[k] + 0.3 * next) - 0.3 * sin(2.0 * xi[k]);
    } else if (mdl->drift == YYO_F_LINEAR) {
      div += mdl->A[(size_t)k * r + k];
    }
  }
  return div;
}

/* ------------------------------------------------------------------------- */
/* Prediction of one target row (Sec. 4.1-4.3 kernel operator, Sec. 9 log-domain
 * prediction).  For scale s the kernel has variance tau_s a (tau_s = dt/s) and
 * is centred at x_j + tau_s f(x_j) (push form) or, as a function of the
 * source x_j, at x_i - tau_s f(x_i) with the factor exp(-tau_s div f(x_i))
 * (pull form, eq. kernel).  The quadrature weight of every source is
 * dV = vol(box)/n.                                                          */
static const yyo_kernel kDefaultKernel = {YYO_FORM_PUSH, YYO_DIV_CLOSED, 1e-20, NULL, 0.0};

static double propagate_row(const yyo_model* mdl, const yyo_kernel* kn, int32_t S, const double* s,
                            const double* c, int64_t n, const double* x, const double* F,
                            const double* div, const char* bnd, double logdV, double dt,
                            const double* logw_in, int64_t i, double* a, double* d, int* clamped) {
  int32_t r = mdl->r;
  const int pull = kn->form == YYO_FORM_PULL;
  *clamped = 0;
  if (bnd[i]) return -INFINITY;
  double T[17];
  double sign[17];
  int nt = 0;
  for (int32_t sc = 0; sc < S; ++sc) {
    double tau = dt / s[sc];
    /* LSE over sources (definition of LSE in Sec. 9): max, then sum. */
    double mx = -INFINITY;
    for (int64_t j = 0; j < n; ++j) {
      if (bnd[j] || logw_in[j] == -INFINITY) {
        a[j] = -INFINITY;
        continue;
      }
      /* displacement of the pair: push x_i - x_j - tau f(x_j); pull x_j - x_i + tau f(x_i) */
      for (int32_t k = 0; k < r; ++k) {
        if (pull)
          d[k] = (x[(size_t)j * r + k] - x[(size_t)i * r + k]) + tau * F[(size_t)i * r + k];
        else
          d[k] = (x[(size_t)i * r + k] - x[(size_t)j * r + k]) - tau * F[(size_t)j * r + k];
      }
      if (kn->apinv) {
        double Q = 0.0;   /* d^T a^+ d */
        for (int32_t k = 0; k < r; ++k) {
          double row = 0.0;
          for (int32_t l = 0; l < r; ++l) row += kn->apinv[(size_t)k * r + l] * d[l];
          Q += d[k] * row;
        }
        a[j] = -Q / (2.0 * tau) + logw_in[j];
      } else {
        double D = 0.0;   /* |d|^2, variance q tau */
        for (int32_t k = 0; k < r; ++k) D += d[k] * d[k];
        a[j] = -D / (2.0 * (mdl->q * tau)) + logw_in[j];
      }
      if (a[j] > mx) mx = a[j];
    }
    if (mx == -INFINITY || c[sc] == 0.0) continue;
    double sum = 0.0;
    for (int64_t j = 0; j < n; ++j)
      if (a[j] != -INFINITY) sum += exp(a[j] - mx);
    double L = mx + log(sum);
    double logconst = kn->apinv ? -0.5 * r * log(2.0 * M_PI * tau) - 0.5 * kn->logdet_a
                                : -0.5 * r * log(2.0 * M_PI * (mdl->q * tau));
    if (pull) logconst -= tau * div[i];
    T[nt] = log(fabs(c[sc])) + logdV + logconst + L;
    sign[nt] = c[sc] > 0 ? 1.0 : -1.0;
    ++nt;
  }
  /* identity term c_{S+1} u(x_i) */
  if (c[S] != 0.0 && logw_in[i] != -INFINITY) {
    T[nt] = log(fabs(c[S])) + logw_in[i];
    sign[nt] = c[S] > 0 ? 1.0 : -1.0;
    ++nt;
  }
  if (nt == 0) return -INFINITY;
  double Mx = T[0];
  for (int t = 1; t < nt; ++t)
    if (T[t] > Mx) Mx = T[t];
  double acc = 0.0;
  for (int t = 0; t < nt; ++t) acc += sign[t] * exp(T[t] - Mx);
  if (!(acc > 0.0)) {
    *clamped = 1;
    return -INFINITY;
  }
  return Mx + log(acc);
}

static void propagate_setup(const yyo_model* mdl, const yyo_kernel* kn, int64_t n, const double* x,
                            const double* lo, const double* hi, double** F, double** div, char** bnd,
                            double* logdV) {
  int32_t r = mdl->r;
  *F = (double*)malloc(sizeof(double) * (size_t)n * (size_t)r);
  *div = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
  *bnd = (char*)malloc((size_t)(n > 0 ? n : 1));
  for (int64_t j = 0; j < n; ++j) {
    yyo_drift(mdl, x + (size_t)j * r, *F + (size_t)j * r);
    (*div)[j] = kn->form == YYO_FORM_PULL ? yyo_divergence(mdl, x + (size_t)j * r, kn->div_mode, kn->cs_step) : 0.0;
    (*bnd)[j] = (char)yyo_is_boundary(r, x + (size_t)j * r, lo, hi);
  }
  double lv = 0.0;
  for (int32_t k = 0; k < r; ++k) lv += log(hi[k] - lo[k]);
  *logdV = lv - log((double)n);
}

int64_t yyo_propagate_rows_ex(const yyo_model* mdl, const yyo_kernel* kn, int32_t S, const double* s,
                              const double* c, int64_t n, const double* x, const double* lo,
                              const double* hi, double dt, const double* logw_in, int64_t nrows,
                              const int64_t* rows, double* out_rows) {
  if (!kn) kn = &kDefaultKernel;
  double *F, *div;
  char* bnd;
  double logdV;
  propagate_setup(mdl, kn, n, x, lo, hi, &F, &div, &bnd, &logdV);
  int64_t nclamped = 0;
#pragma omp parallel reduction(+ : nclamped)
  {
    double* a = (double*)malloc(sizeof(double) * (size_t)n);
    double* d = (double*)malloc(sizeof(double) * (size_t)mdl->r);
#pragma omp for schedule(dynamic, 1)
    for (int64_t t = 0; t < nrows; ++t) {
      int cl;
      out_rows[t] = propagate_row(mdl, kn, S, s, c, n, x, F, div, bnd, logdV, dt, logw_in, rows[t], a, d, &cl);
      nclamped += cl;
    }
    free(a);
    free(d);
  }
  free(F);
  free(div);
  free(bnd);
  return nclamped;
}

int64_t yyo_propagate_ex(const yyo_model* mdl, const yyo_kernel* kn, int32_t S, const double* s,
                         const double* c, int64_t n, const double* x, const double* lo, const double* hi,
                         double dt, const double* logw_in, double* logw_out) {
  if (!kn) kn = &kDefaultKernel;
  double *F, *div;
  char* bnd;
  double logdV;
  propagate_setup(mdl, kn, n, x, lo, hi, &F, &div, &bnd, &logdV);
  int64_t nclamped = 0;
#pragma omp parallel reduction(+ : nclamped)
  {
    double* a = (double*)malloc(sizeof(double) * (size_t)n);
    double* d = (double*)malloc(sizeof(double) * (size_t)mdl->r);
#pragma omp for schedule(dynamic, 16)
    for (int64_t i = 0; i < n; ++i) {
      int cl;
      logw_out[i] = propagate_row(mdl, kn, S, s, c, n, x, F, div, bnd, logdV, dt, logw_in, i, a, d, &cl);
      nclamped += cl;
    }
    free(a);
    free(d);
  }
  free(F);
  free(div);
  free(bnd);
  return nclamped;
}

int64_t yyo_propagate(const yyo_model* mdl, int32_t S, const double* s, const double* c, int64_t n,
                      const double* x, const double* lo, const double* hi, double dt,
                      const double* logw_in, double* logw_out) {
  return yyo_propagate_ex(mdl, NULL, S, s, c, n, x, lo, hi, dt, logw_in, logw_out);
}

int64_t yyo_propagate_rows(const yyo_model* mdl, int32_t S, const double* s, const double* c,
                           int64_t n, const double* x, const double* lo, const double* hi,
                           double dt, const double* logw_in, int64_t nrows, const int64_t* rows,
                           double* out_rows) {
  return yyo_propagate_rows_ex(mdl, NULL, S, s, c, n, x, lo, hi, dt, logw_in, nrows, rows, out_rows);
}

/* ------------------------------------------------------------------------- */
/* Online update with the Ito correction (Sec. 2.2, Sec. 9 observation update;
 * the 1/rho2 scaling is the b^{-1} of Table tab:generalformulas).           */
void yyo_loglik_update(const yyo_model* mdl, int64_t n, const double* x, const double* dy,
                       double dt, double* logw) {
  double* h = (double*)malloc(sizeof(double) * (size_t)mdl->m);
  for (int64_t i = 0; i < n; ++i) {
    if (logw[i] == -INFINITY) continue;
    yyo_obs(mdl, x + (size_t)i * mdl->r, h);
    double dot = 0.0, hh = 0.0;
    for (int32_t k = 0; k < mdl->m; ++k) dot += h[k] * dy[k];
    for (int32_t k = 0; k < mdl->m; ++k) hh += h[k] * h[k];
    logw[i] += (dot - 0.5 * dt * hh) / mdl->rho2;
  }
  free(h);
}

/* Online update with observation noise b = V V^T (Table tab:generalformulas):
 * h^T b^+ dy - dt/2 h^T b^+ h, with the pseudo-inverse b^+ given.            */
void yyo_loglik_update_ex(const yyo_model* mdl, int64_t n, const double* x, const double* dy, double dt,
                          const double* bpinv, double* logw) {
  int32_t m = mdl->m;
  double* h = (double*)malloc(sizeof(double) * (size_t)m);
  for (int64_t i = 0; i < n; ++i) {
    if (logw[i] == -INFINITY) continue;
    yyo_obs(mdl, x + (size_t)i * mdl->r, h);
    double lin = 0.0, quad = 0.0;
    for (int32_t k = 0; k < m; ++k) {
      double bdy = 0.0, bh = 0.0;
      for (int32_t l = 0; l < m; ++l) {
        bdy += bpinv[(size_t)k * m + l] * dy[l];
        bh += bpinv[(size_t)k * m + l] * h[l];
      }
      lin += h[k] * bdy;
      quad += h[k] * bh;
    }
    logw[i] += lin - 0.5 * dt * quad;
  }
  free(h);
}

/* Normalisation in the log domain (Sec. 9) and the weighted estimate
 * (Sec. 2.2.2, step 4), with the weighted covariance and the effective
 * sample size 1/sum w^2.                                                    */
int yyo_normalise_moments(int64_t n, int32_t r, const double* x, double* logw, double* w,
                          double* logZ_step, double* logZ_acc, double* mean, double* cov,
                          double* ess) {
  double mx = -INFINITY;
  for (int64_t i = 0; i < n; ++i)
    if (logw[i] > mx) mx = logw[i];
  if (mx == -INFINITY) {
    *logZ_step = -INFINITY;
    return 1;
  }
  double sum = 0.0;
  for (int64_t i = 0; i < n; ++i) sum += exp(logw[i] - mx);
  double logZ = mx + log(sum);
  *logZ_step = logZ;
  *logZ_acc += logZ;
  double* ww = w ? w : (double*)malloc(sizeof(double) * (size_t)n);
  double s2 = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    logw[i] -= logZ;
    ww[i] = exp(logw[i]);
    s2 += ww[i] * ww[i];
  }
  *ess = 1.0 / s2;
  for (int32_t k = 0; k < r; ++k) {
    double acc = 0.0;
    for (int64_t i = 0; i < n; ++i) acc += ww[i] * x[(size_t)i * r + k];
    mean[k] = acc;
  }
  if (cov) {
    for (int32_t a = 0; a < r; ++a)
      for (int32_t b = 0; b < r; ++b) {
        double acc = 0.0;
        for (int64_t i = 0; i < n; ++i)
          acc += ww[i] * (x[(size_t)i * r + a] - mean[a]) * (x[(size_t)i * r + b] - mean[b]);
        cov[(size_t)a * r + b] = acc;
      }
  }
  if (!w) free(ww);
  return 0;
}

/* Integer systematic resampling.  W_i = floor(w_i 2^53), C = inclusive prefix
 * sums, W = C_{n-1}; U = 32 random bits; position P_t = floor((t 2^32 + U) W /
 * (n 2^32)); ancestor a_t = min{i : C_i > P_t}.                             */
int yyo_resample(int64_t n, const double* w, uint64_t seed, int64_t step, int64_t* idx) {
  uint64_t* C = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)n);
  uint64_t run = 0;
  for (int64_t i = 0; i < n; ++i) {
    double wi = w[i] > 0.0 ? w[i] : 0.0;
    run += (uint64_t)floor(wi * 0x1p53);
    C[i] = run;
  }
  uint64_t W = run;
  if (W == 0) {
    free(C);
    return 1;
  }
  uint64_t U = yyo_splitmix64_at(yyo_splitmix64_at(seed, YYO_DOMAIN_RESAMPLE), (uint64_t)step) >> 32;
  unsigned __int128 denom = ((unsigned __int128)(uint64_t)n) << 32;
  int64_t i = 0;  /* P_t is non-decreasing in t, so the answer never moves left */
  for (int64_t t = 0; t < n; ++t) {
    uint64_t A = ((uint64_t)t << 32) + U;
    uint64_t P = (uint64_t)(((unsigned __int128)A * W) / denom);
    while (C[i] <= P) ++i;
    idx[t] = i;
  }
  free(C);
  return 0;
}

void yyo_restart_nodes(int64_t n, int32_t r, const uint32_t* codes, const double* mean, double R,
                       double* lo, double* hi, double* x_new, double* logw_new) {
  for (int32_t k = 0; k < r; ++k) {
    lo[k] = mean[k] - R;
    hi[k] = mean[k] + R;
  }
  yyo_codes_to_points(r, n, codes, lo, hi, x_new);
  for (int64_t i = 0; i < n; ++i) {
    const double* xi = x_new + (size_t)i * r;
    if (yyo_is_boundary(r, xi, lo, hi)) {
      logw_new[i] = -INFINITY;
      continue;
    }
    double acc = 0.0;
    for (int32_t k = 0; k < r; ++k) acc += (xi[k] - mean[k]) * (xi[k] - mean[k]);
    logw_new[i] = -0.5 * acc;
  }
}
