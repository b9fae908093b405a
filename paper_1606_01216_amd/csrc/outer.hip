// Decisions of AIRGA's outer iteration (Algorithm 1): the poles of the
// reduced quadratic pencil lambda^2 Mh + lambda Dh + Kh, whose real parts
// give the next expansion points (Section 5), and the H2 distance between
// two reduced models, which stops both of the algorithm's loops (Section 5
// sets both tolerances to 1e-6).  Small dense host computations: r is the
// reduced order, at most a few hundred.
//
// Both work in the modal form of a reduced model with proportional damping
// Dh = alpha Mh + beta Kh, which the Galerkin projection keeps (eq. (1.4)).
// With Mh = L L^T and the symmetric eigendecomposition
// L^-1 Kh L^-T = Q diag(w2) Q^T, the columns of Phi = L^-T Q are
// Mh-orthonormal, Phi^T Kh Phi = diag(w2) and Phi^T Dh Phi =
// diag(alpha + beta w2), so mode k is the scalar system
// 1 / (s^2 + d_k s + w2_k) with d_k = alpha + beta w2_k.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <vector>

#include "internal.hpp"

namespace airga {
namespace {

inline size_t at(int r, int i, int j) { return (size_t)j * r + i; }

// Lower Cholesky factor of the symmetric r x r matrix a (column-major), in
// place with the upper part cleared; false unless positive definite.
bool cholesky(int r, std::vector<double>& a) {
  for (int j = 0; j < r; ++j) {
    double d = a[at(r, j, j)];
    for (int k = 0; k < j; ++k) d -= a[at(r, j, k)] * a[at(r, j, k)];
    if (!(d > 0.0)) return false;
    const double l = std::sqrt(d);
    a[at(r, j, j)] = l;
    for (int i = j + 1; i < r; ++i) {
      double s = a[at(r, i, j)];
      for (int k = 0; k < j; ++k) s -= a[at(r, i, k)] * a[at(r, j, k)];
      a[at(r, i, j)] = s / l;
    }
    for (int i = 0; i < j; ++i) a[at(r, i, j)] = 0.0;
  }
  return true;
}

// b (r x c) <- L^-1 b, L lower triangular.
void forward(int r, const std::vector<double>& l, int c, std::vector<double>& b) {
  for (int col = 0; col < c; ++col)
    for (int i = 0; i < r; ++i) {
      double s = b[at(r, i, col)];
      for (int k = 0; k < i; ++k) s -= l[at(r, i, k)] * b[at(r, k, col)];
      b[at(r, i, col)] = s / l[at(r, i, i)];
    }
}

// b (r x c) <- L^-T b.
void backward_t(int r, const std::vector<double>& l, int c, std::vector<double>& b) {
  for (int col = 0; col < c; ++col)
    for (int i = r - 1; i >= 0; --i) {
      double s = b[at(r, i, col)];
      for (int k = i + 1; k < r; ++k) s -= l[at(r, k, i)] * b[at(r, k, col)];
      b[at(r, i, col)] = s / l[at(r, i, i)];
    }
}

// Cyclic Jacobi iteration on the symmetric r x r matrix s: on return its
// diagonal holds the eigenvalues and q the eigenvectors as columns (the
// symmetric Schur rotations of Golub and Van Loan, Section 8.5).  An
// off-diagonal entry below 1e-17 sqrt(|a_pp a_qq|) is set to zero instead
// of rotated (the relative criterion that keeps small eigenvalues
// accurate); the sweeps end when none is left.
void jacobi(int r, std::vector<double>& s, std::vector<double>& q) {
  q.assign((size_t)r * r, 0.0);
  for (int i = 0; i < r; ++i) q[at(r, i, i)] = 1.0;
  for (int sweep = 0; sweep < 60; ++sweep) {
    bool rotated = false;
    for (int p = 0; p < r - 1; ++p)
      for (int c = p + 1; c < r; ++c) {
        const double apc = s[at(r, p, c)];
        if (apc == 0.0) continue;
        if (std::fabs(apc) <= 1e-17 * std::sqrt(std::fabs(s[at(r, p, p)] * s[at(r, c, c)]))) {
          s[at(r, p, c)] = 0.0;
          s[at(r, c, p)] = 0.0;
          continue;
        }
        rotated = true;
        const double tau = (s[at(r, c, c)] - s[at(r, p, p)]) / (2.0 * apc);
        const double t = (tau >= 0.0 ? 1.0 : -1.0) / (std::fabs(tau) + std::sqrt(1.0 + tau * tau));
        const double cs = 1.0 / std::sqrt(1.0 + t * t), sn = t * cs;
        for (int k = 0; k < r; ++k) {
          const double a = s[at(r, k, p)], b = s[at(r, k, c)];
          s[at(r, k, p)] = cs * a - sn * b;
          s[at(r, k, c)] = sn * a + cs * b;
        }
        for (int k = 0; k < r; ++k) {
          const double a = s[at(r, p, k)], b = s[at(r, c, k)];
          s[at(r, p, k)] = cs * a - sn * b;
          s[at(r, c, k)] = sn * a + cs * b;
        }
        for (int k = 0; k < r; ++k) {
          const double a = q[at(r, k, p)], b = q[at(r, k, c)];
          q[at(r, k, p)] = cs * a - sn * b;
          q[at(r, k, c)] = sn * a + cs * b;
        }
      }
    if (!rotated) return;
  }
}

// Modal form: w2 ascending, phi the matching Mh-orthonormal columns.
struct Modal {
  std::vector<double> w2, phi;
};

bool all_finite(const double* v, size_t count) {
  for (size_t i = 0; i < count; ++i)
    if (!std::isfinite(v[i])) return false;
  return true;
}

airga_status modal(int r, const double* mh, const double* kh, Modal* out) {
  if (!all_finite(mh, (size_t)r * r) || !all_finite(kh, (size_t)r * r))
    return fail(AIRGA_EINVAL, "reduced M and K must be finite");
  std::vector<double> l(mh, mh + (size_t)r * r);
  // symmetric part of the input (projections are symmetric to rounding)
  for (int j = 0; j < r; ++j)
    for (int i = j + 1; i < r; ++i) l[at(r, i, j)] = 0.5 * (l[at(r, i, j)] + l[at(r, j, i)]);
  if (!cholesky(r, l)) return fail(AIRGA_ENOTSPD, "reduced M is not positive definite");
  // S = L^-1 K L^-T = L^-1 (L^-1 K)^T for symmetric K
  std::vector<double> y(kh, kh + (size_t)r * r);
  forward(r, l, r, y);
  std::vector<double> s((size_t)r * r);
  for (int j = 0; j < r; ++j)
    for (int i = 0; i < r; ++i) s[at(r, i, j)] = y[at(r, j, i)];
  forward(r, l, r, s);
  for (int j = 0; j < r; ++j)
    for (int i = j + 1; i < r; ++i) {
      const double v = 0.5 * (s[at(r, i, j)] + s[at(r, j, i)]);
      s[at(r, i, j)] = v;
      s[at(r, j, i)] = v;
    }
  std::vector<double> q;
  jacobi(r, s, q);
  backward_t(r, l, r, q);  // phi = L^-T Q
  std::vector<int> ord(r);
  std::iota(ord.begin(), ord.end(), 0);
  std::stable_sort(ord.begin(), ord.end(),
                   [&](int a, int b) { return s[at(r, a, a)] < s[at(r, b, b)]; });
  out->w2.resize(r);
  out->phi.resize((size_t)r * r);
  for (int k = 0; k < r; ++k) {
    out->w2[k] = s[at(r, ord[k], ord[k])];
    std::memcpy(&out->phi[at(r, 0, k)], &q[at(r, 0, ord[k])], sizeof(double) * r);
  }
  return AIRGA_OK;
}

// Reduced model in modal coordinates: per mode its w2, damping d and the
// projected input (m values) and outputs (p values each).
struct ModalModel {
  int r = 0, m = 0, p = 0;
  std::vector<double> w2, d, f, cp, cv;  // f: [k][m], cp, cv: [k][p]
};

airga_status modal_model(const airga_reduced_model& a, double alpha, double beta,
                         ModalModel* out) {
  Modal md;
  AIRGA_TRY(modal(a.r, a.mhat, a.khat, &md));
  const int r = a.r, m = a.m, p = a.p;
  out->r = r;
  out->m = m;
  out->p = p;
  out->w2 = md.w2;
  out->d.resize(r);
  out->f.assign((size_t)r * m, 0.0);
  out->cp.assign((size_t)r * p, 0.0);
  out->cv.assign((size_t)r * p, 0.0);
  for (int k = 0; k < r; ++k) {
    out->d[k] = alpha + beta * md.w2[k];
    if (!(out->d[k] > 0.0))
      return fail(AIRGA_EINVAL, "mode %d has no damping: its H2 norm is infinite", k);
    const double* ph = &md.phi[at(r, 0, k)];
    for (int c = 0; c < m; ++c) {
      double s = 0.0;
      for (int i = 0; i < r; ++i) s += ph[i] * a.fhat[at(r, i, c)];
      out->f[(size_t)k * m + c] = s;
    }
    for (int o = 0; o < p; ++o) {
      double sp = 0.0, sv = 0.0;
      for (int i = 0; i < r; ++i) {
        sp += a.cphat[at(p, o, i)] * ph[i];
        if (a.cvhat) sv += a.cvhat[at(p, o, i)] * ph[i];
      }
      out->cp[(size_t)k * p + o] = sp;
      out->cv[(size_t)k * p + o] = sv;
    }
  }
  return AIRGA_OK;
}

// H2 inner product <H_a, H_b>.  For modes k of a and l of b, the cross
// Gramian X of their realisations [[0, 1], [-w2, -d]], input e2, solves
// A_k X + X A_l^T + e2 e2^T = 0; in closed form, with D = d_k + d_l and
// E = w2_k - w2_l:
//   x00 = D / (E^2 + D^2 w2_l + D d_l E),  x01 = E x00 / D = -x10,
//   x11 = w2_l x00 + d_l x01.
// Entry (u, v) is the inner product of mode k's output u with mode l's
// output v (u, v: position, velocity), so the pair contributes
// (f_k . f_l) * sum_uv (c^u_k . c^v_l) x_uv.
double inner(const ModalModel& a, const ModalModel& b) {
  double total = 0.0;
  const int m = a.m, p = a.p;
  for (int k = 0; k < a.r; ++k)
    for (int l = 0; l < b.r; ++l) {
      double ff = 0.0;
      for (int c = 0; c < m; ++c) ff += a.f[(size_t)k * m + c] * b.f[(size_t)l * m + c];
      double pp = 0.0, pv = 0.0, vp = 0.0, vv = 0.0;
      for (int o = 0; o < p; ++o) {
        const double apk = a.cp[(size_t)k * p + o], avk = a.cv[(size_t)k * p + o];
        const double bpl = b.cp[(size_t)l * p + o], bvl = b.cv[(size_t)l * p + o];
        pp += apk * bpl;
        pv += apk * bvl;
        vp += avk * bpl;
        vv += avk * bvl;
      }
      const double dd = a.d[k] + b.d[l], e = a.w2[k] - b.w2[l];
      const double x00 = dd / (e * e + dd * dd * b.w2[l] + dd * b.d[l] * e);
      const double x01 = e * x00 / dd;
      const double x11 = b.w2[l] * x00 + b.d[l] * x01;
      total += ff * (pp * x00 + pv * x01 - vp * x01 + vv * x11);
    }
  return total;
}

airga_status check_model(const airga_reduced_model* a) {
  if (!a || a->r <= 0 || a->m <= 0 || a->p <= 0 || !a->mhat || !a->khat || !a->fhat ||
      !a->cphat)
    return fail(AIRGA_EINVAL, "reduced model: r, m, p must be positive and M, K, F, C_p given");
  const size_t rm = (size_t)a->r * a->m, pr = (size_t)a->p * a->r;
  if (!all_finite(a->fhat, rm) || !all_finite(a->cphat, pr) ||
      (a->cvhat && !all_finite(a->cvhat, pr)))
    return fail(AIRGA_EINVAL, "reduced model: F and C must be finite");
  return AIRGA_OK;
}

}  // namespace
}  // namespace airga

using namespace airga;

extern "C" {

airga_status airga_qep_poles(int32_t r, const double* mhat, const double* khat, double alpha,
                             double beta, double* re, double* im) {
  if (r <= 0 || !mhat || !khat || !re || !im)
    return fail(AIRGA_EINVAL, "qep_poles: r must be positive and every array given");
  if (!std::isfinite(alpha) || !std::isfinite(beta))
    return fail(AIRGA_EINVAL, "qep_poles: alpha and beta must be finite");
  Modal md;
  AIRGA_TRY(modal(r, mhat, khat, &md));
  for (int k = 0; k < r; ++k) {
    const double w2 = md.w2[k], d = alpha + beta * w2;
    const double disc = d * d - 4.0 * w2;
    if (disc < 0.0) {
      const double h = 0.5 * std::sqrt(-disc);
      re[2 * k] = re[2 * k + 1] = -0.5 * d;
      im[2 * k] = h;
      im[2 * k + 1] = -h;
    } else {
      // the root of larger magnitude without cancellation, the other from
      // the product of the roots (w2)
      const double big = -0.5 * (d + std::copysign(std::sqrt(disc), d));
      const double small = big != 0.0 ? w2 / big : 0.0;
      re[2 * k] = small;
      re[2 * k + 1] = big;
      im[2 * k] = im[2 * k + 1] = 0.0;
    }
  }
  return AIRGA_OK;
}

airga_status airga_next_shifts(int32_t count, const double* re, const double* im, int32_t l,
                               double* shifts) {
  if (count < 0 || l <= 0 || !re || !im || !shifts)
    return fail(AIRGA_EINVAL, "next_shifts: count >= 0, l > 0 and every array given");
  if (!all_finite(re, (size_t)count) || !all_finite(im, (size_t)count))
    return fail(AIRGA_EINVAL, "next_shifts: poles must be finite");
  struct Cand {
    double mag, shift;
  };
  std::vector<Cand> c;
  for (int i = 0; i < count; ++i) {
    const double mag = std::hypot(re[i], im[i]);
    const bool real = std::fabs(im[i]) <= 1e-12 * mag;
    if (real || im[i] > 0.0) c.push_back({mag, -re[i]});
  }
  if ((int)c.size() < l)
    return fail(AIRGA_EINVAL, "next_shifts: %d candidates for %d expansion points",
                (int)c.size(), l);
  std::stable_sort(c.begin(), c.end(), [](const Cand& a, const Cand& b) { return a.mag < b.mag; });
  for (int i = 0; i < l; ++i) shifts[i] = c[i].shift;
  std::sort(shifts, shifts + l);
  return AIRGA_OK;
}

airga_status airga_h2_distance(const airga_reduced_model* a, const airga_reduced_model* b,
                               double alpha, double beta, double* out) {
  if (!out) return fail(AIRGA_EINVAL, "h2_distance: null output");
  if (!std::isfinite(alpha) || !std::isfinite(beta))
    return fail(AIRGA_EINVAL, "h2_distance: alpha and beta must be finite");
  AIRGA_TRY(check_model(a));
  if (b) {
    AIRGA_TRY(check_model(b));
    if (b->m != a->m || b->p != a->p)
      return fail(AIRGA_EINVAL, "h2_distance: the models differ in inputs or outputs");
    if ((a->cvhat == nullptr) != (b->cvhat == nullptr))
      return fail(AIRGA_EINVAL, "h2_distance: velocity output given for one model only");
  }
  ModalModel ma, mb;
  AIRGA_TRY(modal_model(*a, alpha, beta, &ma));
  double sq = inner(ma, ma);
  if (b) {
    AIRGA_TRY(modal_model(*b, alpha, beta, &mb));
    sq += inner(mb, mb) - 2.0 * inner(ma, mb);
  }
  *out = std::sqrt(std::max(sq, 0.0));
  return AIRGA_OK;
}

}  // extern "C"
