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

/* ================= complex shifts (complex symmetric K(s)) =================
 *
 * For a complex expansion point s, K(s) = s^2 M + s D + K is complex
 * symmetric (K(s)^T = K(s)) but not Hermitian.  Its reference solve is the
 * band factorisation K = L Dg L^T (unit lower L, diagonal Dg, transposes
 * without conjugation), which exists without pivoting when every leading
 * principal minor is nonzero (true for s off the real negative axis region
 * where K(s) is singular), then the triangular and diagonal solves.  Band
 * storage as above, real and imaginary parts in separate arrays; in double-
 * double each part has a high and a low array (low may be NULL = 0).
 */

typedef struct { double re, im; } cf;
typedef struct { dd re, im; } cdd;

static inline cf cf_mul(cf a, cf b) { cf r = {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; return r; }
static inline cf cf_sub(cf a, cf b) { cf r = {a.re - b.re, a.im - b.im}; return r; }
static inline cf cf_div(cf a, cf b) {
  /* Smith's algorithm: scale by the larger component of the divisor */
  if (fabs(b.re) >= fabs(b.im)) {
    double t = b.im / b.re, d = b.re + b.im * t;
    cf r = {(a.re + a.im * t) / d, (a.im - a.re * t) / d};
    return r;
  }
  double t = b.re / b.im, d = b.re * t + b.im;
  cf r = {(a.re * t + a.im) / d, (a.im * t - a.re) / d};
  return r;
}

static inline cdd cdd_from(double re, double im) { cdd r = {dd_from(re), dd_from(im)}; return r; }
static inline cdd cdd_add(cdd a, cdd b) { cdd r = {dd_add(a.re, b.re), dd_add(a.im, b.im)}; return r; }
static inline cdd cdd_sub(cdd a, cdd b) { cdd r = {dd_sub(a.re, b.re), dd_sub(a.im, b.im)}; return r; }
static inline cdd cdd_mul(cdd a, cdd b) {
  cdd r = {dd_sub(dd_mul(a.re, b.re), dd_mul(a.im, b.im)),
           dd_add(dd_mul(a.re, b.im), dd_mul(a.im, b.re))};
  return r;
}
static inline cdd cdd_div(cdd a, cdd b) {
  /* (a / b) = a conj(b) / |b|^2, every product in double-double */
  dd den = dd_add(dd_mul(b.re, b.re), dd_mul(b.im, b.im));
  cdd num = {dd_add(dd_mul(a.re, b.re), dd_mul(a.im, b.im)),
             dd_sub(dd_mul(a.im, b.re), dd_mul(a.re, b.im))};
  cdd r = {dd_div(num.re, den), dd_div(num.im, den)};
  return r;
}
static inline int cdd_zero(cdd a) { return a.re.hi == 0.0 && a.im.hi == 0.0; }

/* L Dg L^T in place on the lower band: diagonal entries become Dg, the
 * others L.  Returns pivot_error(i) for a zero pivot in row i. */
static int ldlt_cf(int64_t n, int w, cf* L) {
  const int ld = w + 1;
  for (int64_t j = 0; j < n; ++j) {
    int64_t k0 = j - w < 0 ? 0 : j - w;
    cf d = L[j * ld];
    for (int64_t k = k0; k < j; ++k) {
      cf ljk = L[j * ld + (j - k)];
      d = cf_sub(d, cf_mul(cf_mul(ljk, ljk), L[k * ld]));
    }
    if (d.re == 0.0 && d.im == 0.0) return pivot_error(j);
    L[j * ld] = d;
    int64_t i1 = j + w >= n ? n - 1 : j + w;
    for (int64_t i = j + 1; i <= i1; ++i) {
      int64_t kk = i - w > k0 ? i - w : k0;
      cf s = L[i * ld + (i - j)];
      for (int64_t k = kk; k < j; ++k)
        s = cf_sub(s, cf_mul(cf_mul(L[i * ld + (i - k)], L[j * ld + (j - k)]), L[k * ld]));
      L[i * ld + (i - j)] = cf_div(s, d);
    }
  }
  return 0;
}

static void solve_cf(int64_t n, int w, const cf* L, cf* x) {
  const int ld = w + 1;
  for (int64_t i = 0; i < n; ++i) {            /* L y = b */
    int64_t j0 = i - w < 0 ? 0 : i - w;
    cf s = x[i];
    for (int64_t j = j0; j < i; ++j) s = cf_sub(s, cf_mul(L[i * ld + (i - j)], x[j]));
    x[i] = s;
  }
  for (int64_t i = 0; i < n; ++i) x[i] = cf_div(x[i], L[i * ld]);   /* Dg z = y */
  for (int64_t i = n - 1; i >= 0; --i) {       /* L^T x = z */
    int64_t j1 = i + w >= n ? n - 1 : i + w;
    cf s = x[i];
    for (int64_t j = i + 1; j <= j1; ++j) s = cf_sub(s, cf_mul(L[j * ld + (j - i)], x[j]));
    x[i] = s;
  }
}

static int ldlt_cdd(int64_t n, int w, cdd* L) {
  const int ld = w + 1;
  for (int64_t j = 0; j < n; ++j) {
    int64_t k0 = j - w < 0 ? 0 : j - w;
    cdd d = L[j * ld];
    for (int64_t k = k0; k < j; ++k) {
      cdd ljk = L[j * ld + (j - k)];
      d = cdd_sub(d, cdd_mul(cdd_mul(ljk, ljk), L[k * ld]));
    }
    if (cdd_zero(d)) return pivot_error(j);
    L[j * ld] = d;
    int64_t i1 = j + w >= n ? n - 1 : j + w;
    for (int64_t i = j + 1; i <= i1; ++i) {
      int64_t kk = i - w > k0 ? i - w : k0;
      cdd s = L[i * ld + (i - j)];
      for (int64_t k = kk; k < j; ++k)
        s = cdd_sub(s, cdd_mul(cdd_mul(L[i * ld + (i - k)], L[j * ld + (j - k)]), L[k * ld]));
      L[i * ld + (i - j)] = cdd_div(s, d);
    }
  }
  return 0;
}

static void solve_cdd(int64_t n, int w, const cdd* L, cdd* x) {
  const int ld = w + 1;
  for (int64_t i = 0; i < n; ++i) {
    int64_t j0 = i - w < 0 ? 0 : i - w;
    cdd s = x[i];
    for (int64_t j = j0; j < i; ++j) s = cdd_sub(s, cdd_mul(L[i * ld + (i - j)], x[j]));
    x[i] = s;
  }
  for (int64_t i = 0; i < n; ++i) x[i] = cdd_div(x[i], L[i * ld]);
  for (int64_t i = n - 1; i >= 0; --i) {
    int64_t j1 = i + w >= n ? n - 1 : i + w;
    cdd s = x[i];
    for (int64_t j = i + 1; j <= j1; ++j) s = cdd_sub(s, cdd_mul(L[j * ld + (j - i)], x[j]));
    x[i] = s;
  }
}

/*
 * Solve K X = B for a complex symmetric band matrix K (lower band: re_hi,
 * im_hi, and in double-double also re_lo, im_lo, each may be NULL = 0) and
 * nrhs complex right-hand sides (b_re, b_im; b_im may be NULL = 0), each n
 * long.  precision 0: binary64 complex; 1: double-double complex, the
 * solution rounded to binary64 in x_re, x_im with the low parts in
 * xl_re, xl_im (may be NULL).  Returns 0, pivot_error(i) for a zero pivot,
 * or -2147483647 on allocation failure.
 */
int oracle_cband_solve(int64_t n, int w, const double* re_hi, const double* re_lo,
                       const double* im_hi, const double* im_lo, int nrhs, const double* b_re,
                       const double* b_im, double* x_re, double* x_im, double* xl_re,
                       double* xl_im, int precision) {
  const int ld = w + 1;
  const size_t nb = (size_t)n * ld;
  if (precision == 0) {
    cf* L = (cf*)malloc(sizeof(cf) * nb);
    cf* x = (cf*)malloc(sizeof(cf) * (size_t)n);
    if (!L || !x) { free(L); free(x); return -2147483647; }
    for (size_t e = 0; e < nb; ++e) { L[e].re = re_hi[e]; L[e].im = im_hi[e]; }
    int st = ldlt_cf(n, w, L);
    for (int c = 0; st == 0 && c < nrhs; ++c) {
      for (int64_t i = 0; i < n; ++i) {
        x[i].re = b_re[(size_t)c * n + i];
        x[i].im = b_im ? b_im[(size_t)c * n + i] : 0.0;
      }
      solve_cf(n, w, L, x);
      for (int64_t i = 0; i < n; ++i) {
        x_re[(size_t)c * n + i] = x[i].re;
        x_im[(size_t)c * n + i] = x[i].im;
        if (xl_re) xl_re[(size_t)c * n + i] = 0.0;
        if (xl_im) xl_im[(size_t)c * n + i] = 0.0;
      }
    }
    free(L);
    free(x);
    return st;
  }
  cdd* L = (cdd*)malloc(sizeof(cdd) * nb);
  cdd* x = (cdd*)malloc(sizeof(cdd) * (size_t)n);
  if (!L || !x) { free(L); free(x); return -2147483647; }
  for (size_t e = 0; e < nb; ++e) {
    L[e].re.hi = re_hi[e];
    L[e].re.lo = re_lo ? re_lo[e] : 0.0;
    L[e].im.hi = im_hi[e];
    L[e].im.lo = im_lo ? im_lo[e] : 0.0;
  }
  int st = ldlt_cdd(n, w, L);
  for (int c = 0; st == 0 && c < nrhs; ++c) {
    for (int64_t i = 0; i < n; ++i)
      x[i] = cdd_from(b_re[(size_t)c * n + i], b_im ? b_im[(size_t)c * n + i] : 0.0);
    solve_cdd(n, w, L, x);
    for (int64_t i = 0; i < n; ++i) {
      x_re[(size_t)c * n + i] = x[i].re.hi + x[i].re.lo;
      x_im[(size_t)c * n + i] = x[i].im.hi + x[i].im.lo;
      if (xl_re) xl_re[(size_t)c * n + i] = x[i].re.lo - ((x[i].re.hi + x[i].re.lo) - x[i].re.hi);
      if (xl_im) xl_im[(size_t)c * n + i] = x[i].im.lo - ((x[i].im.hi + x[i].im.lo) - x[i].im.hi);
    }
  }
  free(L);
  free(x);
  return st;
}

/*
 * K(s) = s^2 M + s D + K for complex s = s_re + i s_im, entrywise in complex
 * double-double from exact binary64 M, K, alpha, beta, s: the formula as
 * written (s^2 times M, plus s times the damping entry, plus K).
 */
void oracle_shift_cdd(int64_t cnt, const double* m, const double* k, double s_re, double s_im,
                      double alpha, double beta, double* re_hi, double* re_lo, double* im_hi,
                      double* im_lo) {
  cdd s = cdd_from(s_re, s_im);
  cdd s2 = cdd_mul(s, s);
  dd al = dd_from(alpha), be = dd_from(beta);
  for (int64_t e = 0; e < cnt; ++e) {
    dd me = dd_from(m[e]), ke = dd_from(k[e]);
    cdd mm = {me, dd_from(0.0)};
    cdd damp = {dd_add(dd_mul(al, me), dd_mul(be, ke)), dd_from(0.0)};
    cdd kk = {ke, dd_from(0.0)};
    cdd v = cdd_add(cdd_add(cdd_mul(s2, mm), cdd_mul(s, damp)), kk);
    re_hi[e] = v.re.hi;
    re_lo[e] = v.re.lo;
    im_hi[e] = v.im.hi;
    im_lo[e] = v.im.lo;
  }
}
