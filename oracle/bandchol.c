/*
 * Test infrastructure (CPU oracle), not part of the product path.
 *
 * Reference solve of the shifted systems K(s) X = F (the state X(s) of the
 * transfer function in Section 2, eq. (2.2) first line) for a symmetric
 * positive definite band matrix: Cholesky K = L L^T on the band, then the two
 * triangular solves.  It is run in two precisions:
 *   - plain IEEE binary64, and
 *   - double-double ("dd": an unevaluated sum hi + lo of two binary64 numbers,
 *     about 106 significand bits), built from the error-free transformations
 *     TwoSum (Knuth) and TwoProduct via a fused multiply-add (Dekker's
 *     splitting replaced by fma), the standard published construction.
 * The dd solve is the trusted reference when kappa(K) * 2^-53 is not small.
 *
 * Band storage (lower): ab[i*(w+1) + k] = K[i][i-k] for 0 <= k <= w, entries
 * with i-k < 0 are ignored.  Right-hand sides are nrhs contiguous vectors of
 * length n (column-major n x nrhs).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct { double hi, lo; } dd;

static inline dd two_sum(double a, double b) {
  double s = a + b;
  double bb = s - a;
  dd r = {s, (a - (s - bb)) + (b - bb)};
  return r;
}
static inline dd fast_two_sum(double a, double b) { /* requires |a| >= |b| or a == 0 */
  double s = a + b;
  dd r = {s, b - (s - a)};
  return r;
}
static inline dd two_prod(double a, double b) {
  double p = a * b;
  dd r = {p, fma(a, b, -p)};
  return r;
}
static inline dd dd_from(double a) { dd r = {a, 0.0}; return r; }
static inline dd dd_add(dd x, dd y) {
  dd s = two_sum(x.hi, y.hi);
  dd t = two_sum(x.lo, y.lo);
  s.lo += t.hi;
  s = fast_two_sum(s.hi, s.lo);
  s.lo += t.lo;
  return fast_two_sum(s.hi, s.lo);
}
static inline dd dd_neg(dd x) { dd r = {-x.hi, -x.lo}; return r; }
static inline dd dd_sub(dd x, dd y) { return dd_add(x, dd_neg(y)); }
static inline dd dd_mul(dd x, dd y) {
  dd p = two_prod(x.hi, y.hi);
  p.lo += x.hi * y.lo + x.lo * y.hi;
  return fast_two_sum(p.hi, p.lo);
}
static inline dd dd_div(dd x, dd y) {
  /* long division: three binary64 quotient digits */
  double q1 = x.hi / y.hi;
  dd r = dd_sub(x, dd_mul(dd_from(q1), y));
  double q2 = r.hi / y.hi;
  r = dd_sub(r, dd_mul(dd_from(q2), y));
  double q3 = r.hi / y.hi;
  dd q = fast_two_sum(q1, q2);
  return dd_add(q, dd_from(q3));
}
static inline dd dd_sqrt(dd x) {
  /* one Newton step on the binary64 root doubles the accurate bits */
  if (x.hi <= 0.0) return dd_from(sqrt(x.hi));
  double q = sqrt(x.hi);
  dd qq = two_prod(q, q);
  dd rem = dd_sub(x, qq);
  return fast_two_sum(q, rem.hi / (2.0 * q));
}

/* -(i+1) for a non-positive pivot in row i (saturated to stay above the
 * allocation-failure code). */
static int pivot_error(int64_t i) { return i + 1 >= 2147483646 ? -2147483646 : (int)(-(i + 1)); }

/* ---------------- binary64 ---------------- */

static int chol_f64(int64_t n, int w, double* L) {
  const int ld = w + 1;
  for (int64_t i = 0; i < n; ++i) {
    int64_t j0 = i - w < 0 ? 0 : i - w;
    for (int64_t j = j0; j <= i; ++j) {
      double s = L[i * ld + (i - j)];
      for (int64_t k = j0; k < j; ++k) {
        if (j - k > w) continue;
        s -= L[i * ld + (i - k)] * L[j * ld + (j - k)];
      }
      if (j < i) {
        L[i * ld + (i - j)] = s / L[j * ld];
      } else {
        if (!(s > 0.0)) return pivot_error(i);
        L[i * ld] = sqrt(s);
      }
    }
  }
  return 0;
}

static void solve_f64(int64_t n, int w, const double* L, double* x) {
  const int ld = w + 1;
  for (int64_t i = 0; i < n; ++i) {           /* L y = b */
    double s = x[i];
    int64_t j0 = i - w < 0 ? 0 : i - w;
    for (int64_t j = j0; j < i; ++j) s -= L[i * ld + (i - j)] * x[j];
    x[i] = s / L[i * ld];
  }
  for (int64_t i = n - 1; i >= 0; --i) {      /* L^T x = y */
    double s = x[i];
    int64_t j1 = i + w >= n ? n - 1 : i + w;
    for (int64_t j = i + 1; j <= j1; ++j) s -= L[j * ld + (j - i)] * x[j];
    x[i] = s / L[i * ld];
  }
}

/* ---------------- double-double ---------------- */

static int chol_dd(int64_t n, int w, const double* ab, const double* ab_lo, dd* L) {
  const int ld = w + 1;
  for (int64_t i = 0; i < n; ++i) {
    int64_t j0 = i - w < 0 ? 0 : i - w;
    for (int64_t j = j0; j <= i; ++j) {
      dd s = {ab[i * ld + (i - j)], ab_lo ? ab_lo[i * ld + (i - j)] : 0.0};
      for (int64_t k = j0; k < j; ++k) {
        if (j - k > w) continue;
        s = dd_sub(s, dd_mul(L[i * ld + (i - k)], L[j * ld + (j - k)]));
      }
      if (j < i) {
        L[i * ld + (i - j)] = dd_div(s, L[j * ld]);
      } else {
        if (!(s.hi > 0.0)) return pivot_error(i);
        L[i * ld] = dd_sqrt(s);
      }
    }
  }
  return 0;
}

static void solve_dd(int64_t n, int w, const dd* L, const double* b, dd* x) {
  const int ld = w + 1;
  for (int64_t i = 0; i < n; ++i) {
    dd s = dd_from(b[i]);
    int64_t j0 = i - w < 0 ? 0 : i - w;
    for (int64_t j = j0; j < i; ++j) s = dd_sub(s, dd_mul(L[i * ld + (i - j)], x[j]));
    x[i] = dd_div(s, L[i * ld]);
  }
  for (int64_t i = n - 1; i >= 0; --i) {
    dd s = x[i];
    int64_t j1 = i + w >= n ? n - 1 : i + w;
    for (int64_t j = i + 1; j <= j1; ++j) s = dd_sub(s, dd_mul(L[j * ld + (j - i)], x[j]));
    x[i] = dd_div(s, L[i * ld]);
  }
}

/*
 * Solve K X = B for an SPD band matrix.
 *   precision 0: binary64 (ab_lo ignored);  1: double-double, where the band
 *   is ab + ab_lo (ab_lo may be NULL) and x_lo receives the low parts of the
 *   solution (may be NULL).
 * Returns 0 on success, a negative value -(i+1) if the i-th pivot is not
 * positive (matrix not SPD to working precision), -2147483647 on allocation
 * failure.
 */
int oracle_band_solve(int64_t n, int w, const double* ab, const double* ab_lo, int nrhs,
                      const double* b, double* x_hi, double* x_lo, int precision) {
  const int ld = w + 1;
  if (precision == 0) {
    double* L = (double*)malloc(sizeof(double) * (size_t)n * ld);
    if (!L) return -2147483647;
    memcpy(L, ab, sizeof(double) * (size_t)n * ld);
    int st = chol_f64(n, w, L);
    if (st == 0) {
      for (int c = 0; c < nrhs; ++c) {
        memcpy(x_hi + (size_t)c * n, b + (size_t)c * n, sizeof(double) * (size_t)n);
        solve_f64(n, w, L, x_hi + (size_t)c * n);
        if (x_lo) memset(x_lo + (size_t)c * n, 0, sizeof(double) * (size_t)n);
      }
    }
    free(L);
    return st;
  }
  dd* L = (dd*)malloc(sizeof(dd) * (size_t)n * ld);
  dd* x = (dd*)malloc(sizeof(dd) * (size_t)n);
  if (!L || !x) { free(L); free(x); return -2147483647; }
  int st = chol_dd(n, w, ab, ab_lo, L);
  if (st == 0) {
    for (int c = 0; c < nrhs; ++c) {
      solve_dd(n, w, L, b + (size_t)c * n, x);
      for (int64_t i = 0; i < n; ++i) {
        x_hi[(size_t)c * n + i] = x[i].hi;
        if (x_lo) x_lo[(size_t)c * n + i] = x[i].lo;
      }
    }
  }
  free(L);
  free(x);
  return st;
}

/*
 * Residual r = B - K X evaluated in double-double, with X = x_hi + x_lo given
 * exactly; the result is rounded to binary64.  K is symmetric, so the upper
 * part is read from the lower band.
 */
void oracle_band_residual_dd(int64_t n, int w, const double* ab, const double* ab_lo, int nrhs,
                             const double* b, const double* x_hi, const double* x_lo,
                             double* r) {
  const int ld = w + 1;
  for (int c = 0; c < nrhs; ++c) {
    const double* xh = x_hi + (size_t)c * n;
    const double* xl = x_lo ? x_lo + (size_t)c * n : NULL;
    for (int64_t i = 0; i < n; ++i) {
      dd s = dd_from(b[(size_t)c * n + i]);
      int64_t j0 = i - w < 0 ? 0 : i - w;
      int64_t j1 = i + w >= n ? n - 1 : i + w;
      for (int64_t j = j0; j <= j1; ++j) {
        int64_t e = j <= i ? i * ld + (i - j) : j * ld + (j - i);
        dd a = {ab[e], ab_lo ? ab_lo[e] : 0.0};
        dd xj = {xh[j], xl ? xl[j] : 0.0};
        s = dd_sub(s, dd_mul(a, xj));
      }
      r[(size_t)c * n + i] = s.hi + s.lo;
    }
  }
}

/*
 * The shifted operator K(s) = s^2 M + s D + K with D = alpha M + beta K
 * (proportional damping of eq. (1.1); the matrix of X(s) in Section 2),
 * evaluated entrywise in double-double from exact binary64 inputs, on any
 * common storage of M and K (cnt entries).  Following the formula as written:
 * s^2 * M, plus s times the damping entry, plus K.
 */
void oracle_shift_dd(int64_t cnt, const double* m, const double* k, double s, double alpha,
                     double beta, double* out_hi, double* out_lo) {
  dd s2 = two_prod(s, s);
  dd sd = dd_from(s);
  dd al = dd_from(alpha), be = dd_from(beta);
  for (int64_t e = 0; e < cnt; ++e) {
    dd me = dd_from(m[e]), ke = dd_from(k[e]);
    dd damp = dd_add(dd_mul(al, me), dd_mul(be, ke));
    dd v = dd_add(dd_add(dd_mul(s2, me), dd_mul(sd, damp)), ke);
    out_hi[e] = v.hi;
    out_lo[e] = v.lo;
  }
}
