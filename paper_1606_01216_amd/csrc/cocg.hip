// Complex expansion points.  For complex s the shifted matrix
//     K(s) = (s^2 + alpha s) M + (1 + beta s) K
// is complex symmetric (K(s)^T = K(s)), not Hermitian: the paper keeps its
// points real by taking the real parts of the reduced poles (Section 5);
// this file takes the complex points as they are.  It provides the SPAI of
// K(s) (eq. (3.1) with complex column least squares, equilibrated by the
// principal square root of the diagonal and symmetrised with the plain
// transpose, so the factor stays complex symmetric) and batched conjugate
// orthogonal CG (CG with the bilinear form x^T y; van der Vorst and
// Melissen 1990) for all (shift, column) systems at once, in float64.
//
// Data layout: complex values are interleaved (re, im) doubles.  Solve
// vectors are kind-major like the real solves, vec(kind, b) = ws + (kind B +
// b) n_pad complex entries; padding rows hold zeros.  One wavefront owns one
// 64-row slice (one row per lane), keeps the slice's columns and M, K values
// in registers and sweeps the active systems; partial sums are written per
// (slot, system, wavefront) and summed in a fixed order by one block per
// system.
#include <cmath>
#include <cstring>
#include <vector>

#include "internal.hpp"

namespace airga {
namespace {

struct cplx {
  double re, im;
};
__host__ __device__ __forceinline__ cplx cx(double re, double im = 0.0) { return cplx{re, im}; }
__host__ __device__ __forceinline__ cplx operator+(cplx a, cplx b) { return cplx{a.re + b.re, a.im + b.im}; }
__host__ __device__ __forceinline__ cplx operator-(cplx a, cplx b) { return cplx{a.re - b.re, a.im - b.im}; }
__host__ __device__ __forceinline__ cplx operator*(cplx a, cplx b) {
  return cplx{fma(a.re, b.re, -a.im * b.im), fma(a.re, b.im, a.im * b.re)};
}
__host__ __device__ __forceinline__ cplx operator*(double s, cplx a) { return cplx{s * a.re, s * a.im}; }
__host__ __device__ __forceinline__ cplx conj(cplx a) { return cplx{a.re, -a.im}; }
__host__ __device__ __forceinline__ double abs2(cplx a) { return fma(a.re, a.re, a.im * a.im); }
// a += x * y
__host__ __device__ __forceinline__ void cfma(cplx& a, cplx x, cplx y) {
  a.re = fma(x.re, y.re, fma(-x.im, y.im, a.re));
  a.im = fma(x.re, y.im, fma(x.im, y.re, a.im));
}
// a += s * y for real s
__host__ __device__ __forceinline__ void rfma(cplx& a, double s, cplx y) {
  a.re = fma(s, y.re, a.re);
  a.im = fma(s, y.im, a.im);
}
// a / b by Smith's scaling (the larger component of b divides first)
__host__ __device__ __forceinline__ cplx cdiv(cplx a, cplx b) {
  if (fabs(b.re) >= fabs(b.im)) {
    const double t = b.im / b.re, d = fma(b.im, t, b.re);
    return cplx{fma(a.im, t, a.re) / d, fma(-a.re, t, a.im) / d};
  }
  const double t = b.re / b.im, d = fma(b.re, t, b.im);
  return cplx{fma(a.re, t, a.im) / d, fma(a.im, t, -a.re) / d};
}
// principal square root (branch cut on the negative real axis)
__host__ __device__ __forceinline__ cplx csqrt(cplx z) {
  const double r = hypot(z.re, z.im);
  if (r == 0.0) return cplx{0.0, 0.0};
  if (z.re >= 0.0) {
    const double t = sqrt(0.5 * (r + z.re));
    return cplx{t, z.im / (2.0 * t)};
  }
  const double t = sqrt(0.5 * (r - z.re));
  return cplx{fabs(z.im) / (2.0 * t), copysign(t, z.im)};
}

// Scalar load of a wave-uniform complex value (two float64 scalar loads).
__device__ __forceinline__ cplx sload_c(const cplx* p) {
  const double* d = reinterpret_cast<const double*>(p);
  return cplx{sload(d), sload(d + 1)};
}

// Float complex values for the float32 inner solves of MIXED mode (the
// same operations as cplx, in float).
struct cf {
  float re, im;
};
__device__ __forceinline__ cf operator+(cf a, cf b) { return cf{a.re + b.re, a.im + b.im}; }
__device__ __forceinline__ cf operator*(cf a, cf b) {
  return cf{fmaf(a.re, b.re, -a.im * b.im), fmaf(a.re, b.im, a.im * b.re)};
}
__device__ __forceinline__ float abs2(cf a) { return fmaf(a.re, a.re, a.im * a.im); }
__device__ __forceinline__ void cfma(cf& a, cf x, cf y) {
  a.re = fmaf(x.re, y.re, fmaf(-x.im, y.im, a.re));
  a.im = fmaf(x.re, y.im, fmaf(x.im, y.re, a.im));
}
__device__ __forceinline__ void rfma(cf& a, float s, cf y) {
  a.re = fmaf(s, y.re, a.re);
  a.im = fmaf(s, y.im, a.im);
}
// real type, zero, and conversion from float64 complex, per value type
template <typename V> struct cvt;
template <> struct cvt<cplx> {
  using R = double;
  __device__ static cplx from(cplx z) { return z; }
  __device__ static cplx real(double v) { return cplx{v, 0.0}; }
};
template <> struct cvt<cf> {
  using R = float;
  __device__ static cf from(cplx z) { return cf{(float)z.re, (float)z.im}; }
  __device__ static cf real(double v) { return cf{(float)v, 0.0f}; }
};

// Shift coefficients a = s^2 + alpha s, b = 1 + beta s.
inline void ccoeffs(const Pencil& pen, cplx s, cplx* a, cplx* b) {
  *a = s * s + pen.alpha * s;
  *b = cx(1.0) + pen.beta * s;
}

// ------------------------------------------------------------- assembly

// out (CSR order, interleaved) = a M + b K
__global__ void k_cassemble(PencilDev pd, int64_t stored, cplx a, cplx b, double* __restrict__ out) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= stored) return;
  const int32_t e = pd.csr_pos[i];
  if (e < 0) return;
  const double mv = pd.m64[i], kv = pd.k64[i];
  out[2 * (int64_t)e] = fma(a.re, mv, b.re * kv);
  out[2 * (int64_t)e + 1] = fma(a.im, mv, b.im * kv);
}

// ------------------------------------------------------------------ SPAI

// dinv[r] = 1 / sqrt(K(s)_rr) (1 for padding rows), or 1 without
// equilibration.
__global__ void k_cdinv(PencilDev pd, cplx a, cplx b, int eq, cplx* __restrict__ dinv) {
  const int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (r >= (int64_t)pd.n_slices * kSlice) return;
  cplx v = cx(1.0);
  if (eq && r < pd.n) {
    const int32_t i = pd.diag_pos[r];
    const double mv = pd.m64[i], kv = pd.k64[i];
    const cplx d = cplx{fma(a.re, mv, b.re * kv), fma(a.im, mv, b.im * kv)};
    v = cdiv(cx(1.0), csqrt(d));
  }
  dinv[r] = v;
}

// Row r of the pencil: stored index of entry q is base + 64 q.
__device__ __forceinline__ int32_t row_base(const PencilDev& pd, int64_t r) {
  return pd.slice_ptr[r / kSlice] + (int32_t)(r % kSlice);
}

// Folds one row (row[0..nj), right-hand side rhs) of a column problem into
// the complex Givens QR (R packed upper triangular, qtb = Q^H t): one
// rotation [c s; -conj(s) c] with c real per column turns (R_kk, row_k)
// into (rho, 0).  Returns what is left of the right-hand side, whose
// squared modulus adds to the residual.
template <int MJ>
__device__ __forceinline__ cplx cgivens_row(cplx (&R)[MJ * (MJ + 1) / 2], cplx (&qtb)[MJ],
                                            cplx (&row)[MJ], cplx rhs, int nj) {
#pragma unroll
  for (int kk = 0; kk < MJ; ++kk) {
    if (kk >= nj) break;
    const int dk = kk * MJ - kk * (kk - 1) / 2;  // R(kk, kk) in packed rows
    const cplx x = R[dk], y = row[kk];
    const double ay = abs2(y);
    if (ay == 0.0) continue;
    const double ax2 = abs2(x);
    const double nrm = sqrt(ax2 + ay);
    double c;
    cplx sn;
    if (ax2 == 0.0) {
      c = 0.0;
      sn = (1.0 / sqrt(ay)) * conj(y);
      R[dk] = cx(sqrt(ay));
    } else {
      const double ax = sqrt(ax2);
      const cplx ph = (1.0 / ax) * x;  // x / |x|
      c = ax / nrm;
      sn = (1.0 / nrm) * (ph * conj(y));
      R[dk] = nrm * ph;
    }
    row[kk] = cx(0.0);
#pragma unroll
    for (int q = 0; q < MJ; ++q) {
      if (q <= kk || q >= nj) continue;
      const cplx t1 = R[dk + (q - kk)], t2 = row[q];
      R[dk + (q - kk)] = c * t1 + sn * t2;
      row[q] = c * t2 - conj(sn) * t1;
    }
    const cplx t1 = qtb[kk];
    qtb[kk] = c * t1 + sn * rhs;
    rhs = c * rhs - conj(sn) * t1;
  }
  return rhs;
}

// Scaled entry Khat(r, c) = (K(s)_rc S_r) S_c of a shifted matrix with
// coefficients (a, b) from the pencil's stored entry idx.
__device__ __forceinline__ cplx cscaled(const PencilDev& pd, int32_t idx, cplx a, cplx b, cplx sr,
                                        cplx sc) {
  const double mv = pd.m64[idx], kv = pd.k64[idx];
  const cplx v = cplx{fma(a.re, mv, b.re * kv), fma(a.im, mv, b.im * kv)};
  return (v * sr) * sc;
}

// Column j's least-squares problem min || t(I) - Khat(I, J) p || over
// complex p, Khat = S K(s) S, J = the pattern of column j (= row j), I =
// the rows of Khat(:, J); t = e_j (build) or, for the update (Section 3.2
// at a complex point), t = khat_old_j, the column of S K(s_old) S.  One
// lane per column: the rows of the problem are folded one at a time into a
// complex Givens QR held in registers.  Each row r of I is met through
// every column J_t whose pattern holds it; it is folded at the first such t
// only (row r holds no J_u with u < t), and its entries Khat(r, J_u) are
// picked from row r's own storage (the pattern is symmetric).  The solution
// is written at row j's own positions (column j's coefficient for row J_t at
// entry t of row j).  redo (NULL: every column): only the columns flagged
// there.  The update first tests the column: it keeps q_j = alpha e_j
// (flag skipf[j], counted in *skip_count) when
// ||khat_old_j - alpha khat_new_j|| <= tol ||khat_old_j||.
template <int MJ, bool UPDATE>
__global__ void __launch_bounds__(64) k_cspai_cols(PencilDev pd, cplx a, cplx b,
                                                   const cplx* __restrict__ dinv,
                                                   cplx* __restrict__ hat,
                                                   double* __restrict__ obj,
                                                   const int8_t* __restrict__ redo, cplx ao,
                                                   cplx bo, const double* __restrict__ alpha_d,
                                                   double tol, int8_t* __restrict__ skipf,
                                                   int32_t* __restrict__ skip_count) {
  const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (j >= pd.n) return;
  if (redo && !redo[j]) return;
  const int32_t bj = row_base(pd, j);
  const int nj = pd.row_len[j];
  int32_t J[MJ];
#pragma unroll
  for (int t = 0; t < MJ; ++t) J[t] = t < nj ? pd.col[bj + t * kSlice] : -1;
  const cplx sj = dinv[j];
  if constexpr (UPDATE) {
    const cplx al = cplx{alpha_d[0], alpha_d[1]};
    double n_old = 0.0, n_res = 0.0;
#pragma unroll
    for (int t = 0; t < MJ; ++t) {
      if (t < nj) {
        const int32_t idx = bj + t * kSlice;
        const cplx sc = dinv[J[t]];
        const cplx vo = cscaled(pd, idx, ao, bo, sj, sc);
        const cplx d = vo - al * cscaled(pd, idx, a, b, sj, sc);
        n_old += abs2(vo);
        n_res += abs2(d);
      }
    }
    const bool skipped = sqrt(n_res) <= tol * sqrt(n_old);
    skipf[j] = skipped ? 1 : 0;
    const unsigned long long bal = __ballot(skipped);
    if ((threadIdx.x & 63) == __ffsll((long long)__ballot(1)) - 1)
      atomicAdd(skip_count, (int32_t)__popcll(bal));
    if (skipped) {
      obj[j] = sqrt(n_res);
      return;
    }
  }
  cplx R[MJ * (MJ + 1) / 2];
  cplx qtb[MJ];
#pragma unroll
  for (int q = 0; q < MJ * (MJ + 1) / 2; ++q) R[q] = cx(0.0);
#pragma unroll
  for (int q = 0; q < MJ; ++q) qtb[q] = cx(0.0);
  double res2 = 0.0;
  for (int t = 0; t < nj; ++t) {
    const int64_t k = J[t];
    const int32_t bk = row_base(pd, k);
    const int nk = pd.row_len[k];
    for (int e = 0; e < nk; ++e) {
      const int64_t r = pd.col[bk + e * kSlice];
      const int32_t br = row_base(pd, r);
      const int nr = pd.row_len[r];
      const cplx sr = dinv[r];
      int32_t cr[MJ];
      cplx vr[MJ];
      cplx rhs = cx(0.0);
      bool dup = false;
#pragma unroll
      for (int q = 0; q < MJ; ++q) {
        cr[q] = -2;
        vr[q] = cx(0.0);
        if (q < nr) {
          const int32_t idx = br + q * kSlice;
          cr[q] = pd.col[idx];
          const cplx sc = dinv[cr[q]];
          vr[q] = cscaled(pd, idx, a, b, sr, sc);
          if constexpr (UPDATE) {
            if (cr[q] == (int32_t)j) rhs = cscaled(pd, idx, ao, bo, sr, sc);
          }
        }
      }
      if constexpr (!UPDATE) rhs = cx(r == j ? 1.0 : 0.0);
#pragma unroll
      for (int u = 0; u < MJ; ++u)
#pragma unroll
        for (int q = 0; q < MJ; ++q) dup |= (u < t) && (cr[q] == J[u]);
      if (dup) continue;
      // this row of the problem: Khat(r, J_u) and t(r)
      cplx row[MJ];
#pragma unroll
      for (int u = 0; u < MJ; ++u) {
        row[u] = cx(0.0);
#pragma unroll
        for (int q = 0; q < MJ; ++q)
          if (cr[q] == J[u]) row[u] = vr[q];
      }
      res2 += abs2(cgivens_row<MJ>(R, qtb, row, rhs, nj));
    }
  }
  // back substitution R p = qtb
  cplx p[MJ];
#pragma unroll
  for (int q = MJ - 1; q >= 0; --q) {
    p[q] = cx(0.0);
    if (q >= nj) continue;
    const int dq = q * MJ - q * (q - 1) / 2;
    cplx acc = qtb[q];
#pragma unroll
    for (int u = 0; u < MJ; ++u)
      if (u > q && u < nj) acc = acc - R[dq + (u - q)] * p[u];
    p[q] = cdiv(acc, R[dq]);
  }
#pragma unroll
  for (int t = 0; t < MJ; ++t)
    if (t < nj) hat[bj + t * kSlice] = p[t];
  obj[j] = sqrt(res2);
}

// Update alpha at a complex point: the minimiser of ||Khat_old - alpha
// Khat_new||_F over complex alpha, <Khat_new, Khat_old> / <Khat_new,
// Khat_new> (Hermitian inner product), both scaled by S_new.  Per block of
// 256 rows: part[3 block + (0, 1, 2)] = (Re, Im) of sum conj(khat_new)
// khat_old, and sum |khat_new|^2, summed in a fixed order.
__global__ void __launch_bounds__(256) k_calpha_partial(PencilDev pd, cplx a, cplx b, cplx ao,
                                                        cplx bo, const cplx* __restrict__ dinv,
                                                        double* __restrict__ part) {
  __shared__ double red[3][4];
  const int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  cplx num = cx(0.0);
  double den = 0.0;
  if (r < pd.n) {
    const int32_t br = row_base(pd, r);
    const int nr = pd.row_len[r];
    const cplx sr = dinv[r];
    for (int q = 0; q < nr; ++q) {
      const int32_t idx = br + q * kSlice;
      const cplx sc = dinv[pd.col[idx]];
      const cplx kn = cscaled(pd, idx, a, b, sr, sc);
      cfma(num, conj(kn), cscaled(pd, idx, ao, bo, sr, sc));
      den += abs2(kn);
    }
  }
  const double v[3] = {wave_sum(num.re), wave_sum(num.im), wave_sum(den)};
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0)
    for (int q = 0; q < 3; ++q) red[q][w] = v[q];
  __syncthreads();
  if (threadIdx.x < 3) {
    double t = 0.0;
    for (int i = 0; i < 4; ++i) t += red[threadIdx.x][i];
    part[3 * (int64_t)blockIdx.x + threadIdx.x] = t;
  }
}

// alpha_d[0..1] = the quotient of the block sums (one block, fixed order);
// *skip_count = 0 for the column kernel that follows.
__global__ void __launch_bounds__(256) k_calpha_final(const double* __restrict__ part, int64_t nb,
                                                      double* __restrict__ alpha_d,
                                                      int32_t* __restrict__ skip_count) {
  __shared__ double red[3][256];
  double t[3] = {0.0, 0.0, 0.0};
  for (int64_t i = threadIdx.x; i < nb; i += 256)
    for (int q = 0; q < 3; ++q) t[q] += part[3 * i + q];
  for (int q = 0; q < 3; ++q) red[q][threadIdx.x] = t[q];
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h)
      for (int q = 0; q < 3; ++q) red[q][threadIdx.x] += red[q][threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double den = red[2][0];
    alpha_d[0] = den > 0.0 ? red[0][0] / den : 0.0;
    alpha_d[1] = den > 0.0 ? red[1][0] / den : 0.0;
    *skip_count = 0;
  }
}

// The same column problems from their normal equations, for pencils whose
// rows are consecutive columns in a narrow band (the beam's).  With Khat
// complex symmetric, B = Khat(I, J) has
//     B^H B = (conj(Khat) Khat)(J, J),   B^H e_j = conj(Khat(J, j)),
// because the columns J vanish outside the rows I: every column's Gram
// matrix is a block of the one banded Hermitian matrix H = conj(Khat) Khat,
//     H(i, i + d) = sum over k of conj(Khat(i, k)) Khat(i + d, k).
// One wavefront solves 64 consecutive columns: it stages the scaled rows
// of its window in LDS, forms the upper band of H for the rows the columns'
// patterns cover, and each lane takes the complex Cholesky G = U^H U of its
// column's block (real positive diagonal) and the two triangular solves.
// The residual follows from ||e_j - B p||^2 = 1 - 2 Re(g^H p) + p^H G p.
// After equilibration the blocks are well conditioned on the beam (cond(B)
// below 15 at the points sigma e^(i pi/6)); a column whose Cholesky loses
// more than 8 digits (a pivot below 1e-8 of its diagonal) is flagged in
// redo and solved by k_cspai_cols instead.  The solution is written as
// k_cspai_cols writes it (column j's coefficients at row j's positions).
// The update (UPDATE) solves min ||khat_old_j - B q|| the same way: the Gram
// matrix is the same block, the right-hand side B^H khat_old_j is
//     g_a = sum over k of conj(Khat_new(J_a, k)) Khat_old(j, k)
// (both matrices complex symmetric), ||t||^2 = ||khat_old_j||^2, and the
// skip test comes first, in the same arithmetic as k_cspai_cols<UPDATE>.
//   LDS per wavefront: scaled values vn[MJ][WR] (complex; the update also
//   vo[MJ][WR] of Khat_old), first column and length of each window row,
//   the band hb[R2][2 bw + 1] (complex); WR = R2 = 64 + 2 bw.
constexpr int kCGramMaxBw = 8;
// packed upper-triangular index of (k, l), k <= l, in an MJ x MJ factor
template <int MJ>
__device__ constexpr int ctri(int k, int l) {
  return k * MJ - (k * (k - 1)) / 2 + (l - k);
}
__host__ __device__ inline size_t cspai_gram_lds(int bw, int mj, bool update) {
  const size_t wr = 64 + 2 * (size_t)bw;
  return wr * ((update ? 2 : 1) * mj * sizeof(cplx) + 2 * sizeof(int32_t)) +
         wr * (2 * (size_t)bw + 1) * sizeof(cplx);
}

// Column j's normal equations from the band of H (the solve of k_cspai_gram):
// Cholesky of G = H(J, J) (real positive diagonal), the two triangular
// solves and the residual from the quadratic form.  FULL: every lane's
// column has MJ entries (no per-entry tests).  Returns false (p and res2
// then not final) when a pivot falls below 1e-8 of its diagonal.
template <int MJ, bool UPDATE, bool FULL>
__device__ __forceinline__ bool cgram_column(const cplx* hb, int BW2, int64_t w0, int J0, int nj,
                                             const cplx* vn, const cplx* vo, int WR, int jr,
                                             const int32_t* f0, const int32_t* ln, double t2,
                                             cplx (&p)[MJ], double& res2) {
  cplx Uf[MJ * (MJ + 1) / 2], y[MJ], g[MJ];
  double iu[MJ];
  bool good = FULL || nj > 0;
#pragma unroll
  for (int k = 0; k < MJ; ++k) {
    y[k] = g[k] = p[k] = cx(0.0);
    iu[k] = 0.0;
    if (FULL || k < nj) {
      const cplx* hk = hb + (J0 + k - (int)w0) * BW2;  // H(J_k, J_k + d)
      if constexpr (UPDATE) {
        // sum over k' of conj(Khat_new(J_k, k')) Khat_old(j, k')
        const int ra = J0 + k - (int)w0;
        const int fa = f0[ra], la = ln[ra];
        const int lo = fa > J0 ? fa : J0;
        const int hi = (fa + la < J0 + nj) ? fa + la : J0 + nj;
        cplx acc = cx(0.0);
        for (int c = lo; c < hi; ++c) cfma(acc, conj(vn[(c - fa) * WR + ra]), vo[(c - J0) * WR + jr]);
        g[k] = acc;
      } else {
        g[k] = conj(vn[k * WR + jr]);                   // conj(Khat(j, J_k))
      }
      double dkk = hk[0].re;
#pragma unroll
      for (int m = 0; m < MJ; ++m)
        if (m < k) dkk -= abs2(Uf[ctri<MJ>(m, k)]);
      good = good && dkk > 1e-8 * hk[0].re;
      const double inv = dkk > 0.0 ? 1.0 / sqrt(dkk) : 0.0;
      iu[k] = inv;
      Uf[ctri<MJ>(k, k)] = cx(dkk * inv);
#pragma unroll
      for (int i = 0; i < MJ; ++i) {
        if (i > k && (FULL || i < nj)) {
          cplx gik = hk[i - k];  // G(k, i) = H(J_k, J_i), i > k
#pragma unroll
          for (int m = 0; m < MJ; ++m)
            if (m < k) gik = gik - conj(Uf[ctri<MJ>(m, k)]) * Uf[ctri<MJ>(m, i)];
          Uf[ctri<MJ>(k, i)] = inv * gik;
        }
      }
      cplx yk = g[k];
#pragma unroll
      for (int m = 0; m < MJ; ++m)
        if (m < k) yk = yk - conj(Uf[ctri<MJ>(m, k)]) * y[m];
      y[k] = inv * yk;
    }
  }
  if (!good) return false;
#pragma unroll
  for (int k = MJ - 1; k >= 0; --k) {
    if (FULL || k < nj) {
      cplx acc = y[k];
#pragma unroll
      for (int i = 0; i < MJ; ++i)
        if (i > k && (FULL || i < nj)) acc = acc - Uf[ctri<MJ>(k, i)] * p[i];
      p[k] = iu[k] * acc;
    }
  }
  // ||e_j - B p||^2 = 1 - 2 Re(g^H p) + p^H G p, G Hermitian from the band
  double ghp = 0.0, pgp = 0.0;
#pragma unroll
  for (int k = 0; k < MJ; ++k) {
    if (FULL || k < nj) {
      const cplx* hk = hb + (J0 + k - (int)w0) * BW2;
      ghp += (conj(g[k]) * p[k]).re;
      double row = hk[0].re * abs2(p[k]);
#pragma unroll
      for (int i = 0; i < MJ; ++i)
        if (i > k && (FULL || i < nj)) row += 2.0 * (conj(p[k]) * (hk[i - k] * p[i])).re;
      pgp += row;
    }
  }
  res2 = fma(-2.0, ghp, t2) + pgp;
  res2 = res2 > 0.0 ? res2 : 0.0;
  return true;
}

template <int MJ, bool UPDATE>
__global__ void __launch_bounds__(64) k_cspai_gram(PencilDev pd, cplx a, cplx b,
                                                   const cplx* __restrict__ dinv, int bw,
                                                   cplx* __restrict__ hat,
                                                   double* __restrict__ obj,
                                                   int8_t* __restrict__ redo, cplx ao, cplx bo,
                                                   const double* __restrict__ alpha_d, double tol,
                                                   int8_t* __restrict__ skipf,
                                                   int32_t* __restrict__ skip_count) {
  extern __shared__ double lds_c[];
  const int lane = threadIdx.x;
  const int WR = 64 + 2 * bw;   // window rows [o0 - bw, o0 + 64 + bw)
  const int BW2 = 2 * bw + 1;
  cplx* vn = reinterpret_cast<cplx*>(lds_c);
  cplx* vo = vn + MJ * WR;  // update only
  int32_t* f0 = reinterpret_cast<int32_t*>(vn + (UPDATE ? 2 : 1) * MJ * WR);
  int32_t* ln = f0 + WR;
  cplx* hb = reinterpret_cast<cplx*>(ln + WR);
  const int64_t n = pd.n;
  const int64_t o0 = (int64_t)blockIdx.x * 64;  // first column
  const int64_t w0 = o0 - bw;                   // first window row
  for (int r = lane; r < WR; r += 64) {
    const int64_t row = w0 + r;
    const bool in = row >= 0 && row < n;
    const int len = in ? pd.row_len[row] : 0;
    const int32_t base = in ? row_base(pd, row) : 0;
    ln[r] = len;
    f0[r] = len > 0 ? pd.col[base] : 0;
    const cplx sr = in ? dinv[row] : cx(0.0);
#pragma unroll
    for (int k = 0; k < MJ; ++k) {
      cplx v = cx(0.0), w = cx(0.0);
      if (k < len) {
        const int32_t idx = base + k * kSlice;
        const cplx sc = dinv[pd.col[idx]];
        v = cscaled(pd, idx, a, b, sr, sc);
        if constexpr (UPDATE) w = cscaled(pd, idx, ao, bo, sr, sc);
      }
      vn[k * WR + r] = v;
      if constexpr (UPDATE) vo[k * WR + r] = w;
    }
  }
  __syncthreads();
  // upper band of H: H(i, i + d) = sum over k of conj(Khat(i, k)) Khat(i +
  // d, k) (entries past a row's length are zero, so every product of the
  // overlap is taken).  Rows 0..63 one per lane, the conjugated values of
  // row i kept in registers for its 2 bw + 1 offsets; the last 2 bw rows one
  // (row, offset) pair per lane.
  {
    const int q = lane;
    cplx vi[MJ];
#pragma unroll
    for (int u = 0; u < MJ; ++u) vi[u] = conj(vn[u * WR + q]);
    const int i0 = f0[q];
    for (int d = 0; d < BW2; ++d) {
      const int cr = q + d;
      cplx acc = cx(0.0);
      if (cr < WR) {
        const int dc = f0[cr] - i0;
#pragma unroll
        for (int u = 0; u < MJ; ++u) {
          const int qq = u - dc;
          const bool ok = qq >= 0 && qq < MJ;
          const cplx x = vn[(ok ? qq : 0) * WR + cr];
          cfma(acc, vi[u], ok ? x : cx(0.0));
        }
      }
      hb[q * BW2 + d] = acc;
    }
  }
  for (int e = lane; e < (WR - 64) * BW2; e += 64) {
    const int q = 64 + e / BW2, d = e - (q - 64) * BW2;
    const int cr = q + d;
    cplx acc = cx(0.0);
    if (cr < WR) {
      const int dc = f0[cr] - f0[q];
#pragma unroll
      for (int u = 0; u < MJ; ++u) {
        const int qq = u - dc;
        const bool ok = qq >= 0 && qq < MJ;
        const cplx x = vn[(ok ? qq : 0) * WR + cr];
        cfma(acc, conj(vn[u * WR + q]), ok ? x : cx(0.0));
      }
    }
    hb[q * BW2 + d] = acc;
  }
  __syncthreads();
  const int64_t j = o0 + lane;
  if (j >= n) return;
  const int jr = (int)(j - w0);
  const int nj = ln[jr];
  const int J0 = f0[jr];  // J = J0 .. J0 + nj - 1
  double t2 = 1.0;        // ||t||^2
  if constexpr (UPDATE) {
    // the skip test, as in k_cspai_cols<UPDATE> (column j = row j)
    const cplx al = cplx{alpha_d[0], alpha_d[1]};
    double n_old = 0.0, n_res = 0.0;
#pragma unroll
    for (int t = 0; t < MJ; ++t) {
      if (t < nj) {
        const cplx w = vo[t * WR + jr];
        const cplx d = w - al * vn[t * WR + jr];
        n_old += abs2(w);
        n_res += abs2(d);
      }
    }
    const bool skipped = sqrt(n_res) <= tol * sqrt(n_old);
    skipf[j] = skipped ? 1 : 0;
    const unsigned long long bal = __ballot(skipped);
    if (lane == __ffsll((long long)__ballot(1)) - 1) atomicAdd(skip_count, (int32_t)__popcll(bal));
    if (skipped) {
      obj[j] = sqrt(n_res);
      redo[j] = 0;
      return;
    }
    t2 = n_old;
  }
  cplx p[MJ];
  double res2 = 0.0;
  const bool good = __all(nj == MJ)
                        ? cgram_column<MJ, UPDATE, true>(hb, BW2, w0, J0, nj, vn, vo, WR, jr, f0, ln, t2, p, res2)
                        : cgram_column<MJ, UPDATE, false>(hb, BW2, w0, J0, nj, vn, vo, WR, jr, f0, ln, t2, p, res2);
  redo[j] = good ? 0 : 1;
  if (!good) return;
  const int32_t bj = row_base(pd, j);
#pragma unroll
  for (int t = 0; t < MJ; ++t)
    if (t < nj) hat[bj + t * kSlice] = p[t];
  obj[j] = sqrt(res2);
}

// P = S Phat S, with Phat replaced by (Phat + Phat^T) / 2 when sym; stored
// order, padding 0; v32 the same values rounded to float (interleaved), the
// copy the float32 inner solves of MIXED mode read.  hat holds column c's coefficient for row r at the
// position of (c, r), so Phat(r, c) = hat[mirror of (r, c)].
// The update (skipf given): Q = S Qhat S^{-1}, a skipped column c being
// alpha e_c; nothing is written when every column was skipped (the factor
// is the scalar alpha I, which the solves drop).
__global__ void k_cspai_finalize(PencilDev pd, const cplx* __restrict__ hat,
                                 const cplx* __restrict__ dinv, int sym, cplx* __restrict__ v,
                                 float* __restrict__ v32, const int8_t* __restrict__ skipf,
                                 const double* __restrict__ alpha_d,
                                 const int32_t* __restrict__ skip_count) {
  const int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (r >= (int64_t)pd.n_slices * kSlice) return;
  if (skipf && *skip_count == pd.n) return;
  const int32_t base = row_base(pd, r);
  const int w = (pd.slice_ptr[r / kSlice + 1] - pd.slice_ptr[r / kSlice]) / kSlice;
  const int len = pd.row_len[r];
  const cplx sr = dinv[r];
  for (int k = 0; k < w; ++k) {
    const int32_t idx = base + k * kSlice;
    cplx val = cx(0.0);
    if (k < len) {
      const int32_t c = pd.col[idx];
      if (skipf) {
        const cplx h = skipf[c] ? (c == (int32_t)r ? cplx{alpha_d[0], alpha_d[1]} : cx(0.0))
                                : hat[pd.mirror[idx]];
        val = cdiv(h * sr, dinv[c]);
      } else {
        cplx h = hat[pd.mirror[idx]];
        if (sym) h = 0.5 * (h + hat[idx]);
        val = (h * sr) * dinv[c];
      }
    }
    v[idx] = val;
    v32[2 * (int64_t)idx] = (float)val.re;
    v32[2 * (int64_t)idx + 1] = (float)val.im;
  }
}

// The scalar factor alpha I in CSR order (interleaved complex).
__global__ void k_cexport_scalar(PencilDev pd, cplx alpha, cplx* __restrict__ out) {
  const int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (r >= pd.n) return;
  const int32_t base = row_base(pd, r);
  const int len = pd.row_len[r];
  for (int k = 0; k < len; ++k) {
    const int32_t idx = base + k * kSlice;
    out[pd.csr_pos[idx]] = pd.col[idx] == (int32_t)r ? alpha : cx(0.0);
  }
}

// values (CSR order, interleaved) of a stored-order complex factor
__global__ void k_cexport(PencilDev pd, int64_t stored, const cplx* __restrict__ v,
                          cplx* __restrict__ out) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= stored) return;
  const int32_t e = pd.csr_pos[i];
  if (e >= 0) out[e] = v[i];
}

// ------------------------------------------------------------------ COCG

// CT: the intermediate vector of a preconditioner chain (Q_z ... Q_2 P_1 r
// is applied factor by factor; the last factor writes CZ).
enum CKind { CX = 0, CR0, CR1, CZ, CP0, CP1, CW, CT, CKINDS };
// partial slots: 0, 1 = p^T w;  2 = ||r||^2;  3, 4 = r^T z;  5, 6 = z^T w
constexpr int kCSlots = 7;

struct CSys {
  cplx *rho, *mu, *alpha, *beta;
  double *tol2, *ff, *relres;
  int32_t *active, *istat, *iters, *nact;
  // MIXED mode: refinement state per system (outer active, final status,
  // sweeps, iterations of finished sweeps, ||F||^2) and the count of
  // systems still refined
  int32_t *outer, *ostat, *sweeps, *itot, *nout;
  double* fo;
};

// V: the value type of the vectors and factors (cplx for float64 solves,
// cf for the float32 inner solves of MIXED mode).
template <typename V>
struct CArgsT {
  PencilDev pd;
  int32_t B, m;
  int64_t ld;                // n_pad
  V* ws;
  const cplx* ca;            // per shift a_k
  const cplx* cb;            // per shift b_k
  // per shift its chain of factors (stored order), P_1 first:
  // fac[shift * maxc + q] for q < clen[shift]; clen 0 = identity
  const V* const* fac;
  const int32_t* clen;
  int32_t maxc;
  double* partial;           // [kCSlots][B][GP]
  int32_t GP;                // wavefronts = slices
  CSys sys;
  __device__ __forceinline__ V* vec(int kind, int b) const {
    return ws + ((int64_t)kind * B + b) * ld;
  }
  // where chain position q of a chain of length L writes: the positions
  // alternate between CT and CZ so that the last one writes CZ
  __device__ __forceinline__ int chain_out(int q, int L) const { return ((L - 1 - q) & 1) ? CT : CZ; }
  __device__ __forceinline__ void put(int q, int b, int g, double v) const {
    partial[((int64_t)q * B + b) * GP + g] = v;
  }
};
using CArgs = CArgsT<cplx>;

// The slice of one wavefront: columns and M, K values of its 64 rows (R:
// float64 from the pencil, or its float32 copy).
template <int WMAX, typename R = double>
struct CRows {
  int32_t col[WMAX];
  R mv[WMAX], kv[WMAX];
  int32_t idx0;
  int64_t row;
  __device__ __forceinline__ void load(const PencilDev& pd, int s, int lane) {
    row = (int64_t)s * kSlice + lane;
    idx0 = pd.slice_ptr[s] + lane;
    const int w = (pd.slice_ptr[s + 1] - pd.slice_ptr[s]) / kSlice;
    const R* __restrict__ mp;
    const R* __restrict__ kp;
    if constexpr (sizeof(R) == 8) {
      mp = pd.m64;
      kp = pd.k64;
    } else {
      mp = pd.m32;
      kp = pd.k32;
    }
#pragma unroll
    for (int k = 0; k < WMAX; ++k) {
      const bool in = k < w;
      col[k] = in ? pd.col[idx0 + k * kSlice] : (int32_t)row;
      mv[k] = in ? mp[idx0 + k * kSlice] : R(0);
      kv[k] = in ? kp[idx0 + k * kSlice] : R(0);
    }
  }
  // the factor's values of this row (0 past the slice's width: the stored
  // padding entries hold 0)
  template <typename V>
  __device__ __forceinline__ void factor(const PencilDev& pd, int s, const V* f,
                                         V (&fv)[WMAX]) const {
    const int w = (pd.slice_ptr[s + 1] - pd.slice_ptr[s]) / kSlice;
#pragma unroll
    for (int k = 0; k < WMAX; ++k) fv[k] = k < w ? f[idx0 + k * kSlice] : cvt<V>::real(0.0);
  }
};

template <typename V>
__device__ __forceinline__ void put_total(const CArgsT<V>& A, int q, int b, int g, int lane,
                                          double v) {
  v = wave_total(v);
  if (lane == 0) A.put(q, b, g, v);
}

// z = C r0 for every active system, with r0 = F(:, c) (real; written to
// r) or, rhs_vec = 1 (the inner solves of MIXED mode), the r0 already in r;
// x = 0, p = 0.  Partials ||r0||^2 and r0^T z.  V: value type (float64
// complex, or float complex for the inner solves).
template <int WMAX, typename V>
__global__ void __launch_bounds__(256) k_cinit(CArgsT<V> A, const double* __restrict__ F,
                                               int64_t ldf, int rhs_vec) {
  using R = typename cvt<V>::R;
  const int lane = threadIdx.x & 63;
  const int s = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (s >= A.pd.n_slices) return;
  CRows<WMAX> rows;
  rows.load(A.pd, s, lane);
  const int64_t n = A.pd.n, r = rows.row;
  int loaded = -1;
  V fv[WMAX];
  for (int b = 0; b < A.B; ++b) {
    if (sload(A.sys.active + b) == 0) continue;
    const int sh = b / A.m, c = b % A.m;
    const int L = sload(A.clen + sh);
    const V* fac = L > 0 ? sload(A.fac + (int64_t)sh * A.maxc) : nullptr;
    if (fac && sh != loaded) {
      rows.factor(A.pd, s, fac, fv);
      loaded = sh;
    }
    V z = cvt<V>::real(0.0);
    double rr, rz_re, rz_im;
    if (rhs_vec) {
      const V* __restrict__ r0 = A.vec(CR0, b);
      const V own = r0[r];
      if (fac) {
#pragma unroll
        for (int k = 0; k < WMAX; ++k) cfma(z, fv[k], r0[rows.col[k]]);
      } else {
        z = own;
      }
      const V rzv = own * z;
      rr = (double)abs2(own);
      rz_re = (double)rzv.re;
      rz_im = (double)rzv.im;
    } else {
      const double* f = F + (int64_t)c * ldf;
      const R fr = r < n ? (R)f[r] : R(0);
      if (fac) {
#pragma unroll
        for (int k = 0; k < WMAX; ++k) {
          const int64_t cc = rows.col[k];
          rfma(z, cc < n ? (R)f[cc] : R(0), fv[k]);
        }
      } else {
        z = cvt<V>::real(fr);
      }
      A.vec(CR0, b)[r] = cvt<V>::real(fr);
      rr = (double)(fr * fr);
      rz_re = (double)(fr * z.re);
      rz_im = (double)(fr * z.im);
    }
    A.vec(CX, b)[r] = cvt<V>::real(0.0);
    A.vec(CP1, b)[r] = cvt<V>::real(0.0);
    A.vec(L > 1 ? A.chain_out(0, L) : CZ, b)[r] = z;
    put_total(A, 2, b, s, lane, rr);
    if (L <= 1) {  // otherwise the chain's last factor forms r^T z
      put_total(A, 3, b, s, lane, rz_re);
      put_total(A, 4, b, s, lane, rz_im);
    }
  }
}

// p_new = z + beta p_old;  w = K(s) p_new;  partial p_new^T w.  The
// neighbours' p_new are formed from z and p_old at the column.
template <int WMAX, typename V>
__global__ void __launch_bounds__(256) k_cdir(CArgsT<V> A, int par) {
  using R = typename cvt<V>::R;
  const int lane = threadIdx.x & 63;
  const int s = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (s >= A.pd.n_slices) return;
  CRows<WMAX, R> rows;
  rows.load(A.pd, s, lane);
  const int64_t r = rows.row;
  for (int b = 0; b < A.B; ++b) {
    if (sload(A.sys.active + b) == 0) continue;
    const int sh = b / A.m;
    const V be = cvt<V>::from(sload_c(A.sys.beta + b));
    const V ka = cvt<V>::from(sload_c(A.ca + sh)), kb = cvt<V>::from(sload_c(A.cb + sh));
    const V* __restrict__ z = A.vec(CZ, b);
    const V* __restrict__ po = A.vec(par ? CP0 : CP1, b);
    V am = cvt<V>::real(0.0), ak = cvt<V>::real(0.0);
#pragma unroll
    for (int k = 0; k < WMAX; ++k) {
      const int64_t c = rows.col[k];
      V pc = z[c];
      cfma(pc, be, po[c]);
      rfma(am, rows.mv[k], pc);
      rfma(ak, rows.kv[k], pc);
    }
    V pn = z[r];
    cfma(pn, be, po[r]);
    const V w = ka * am + kb * ak;
    A.vec(par ? CP1 : CP0, b)[r] = pn;
    A.vec(CW, b)[r] = w;
    const V pw = pn * w;
    put_total(A, 0, b, s, lane, (double)pw.re);
    put_total(A, 1, b, s, lane, (double)pw.im);
  }
}

// x += alpha p_new;  r_new = r_old - alpha w;  z = C r_new;  partials
// ||r_new||^2, r_new^T z, z^T w.  The neighbours' r_new are formed from
// r_old and w at the column.
template <int WMAX, typename V>
__global__ void __launch_bounds__(256) k_cupd(CArgsT<V> A, int par) {
  const int lane = threadIdx.x & 63;
  const int s = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (s >= A.pd.n_slices) return;
  CRows<WMAX> rows;
  rows.load(A.pd, s, lane);
  const int64_t r = rows.row;
  int loaded = -1;
  V fv[WMAX];
  for (int b = 0; b < A.B; ++b) {
    if (sload(A.sys.active + b) == 0) continue;
    const int sh = b / A.m;
    const int L = sload(A.clen + sh);
    const V* fac = L > 0 ? sload(A.fac + (int64_t)sh * A.maxc) : nullptr;
    if (fac && sh != loaded) {
      rows.factor(A.pd, s, fac, fv);
      loaded = sh;
    }
    const cplx al64 = sload_c(A.sys.alpha + b);
    const V al = cvt<V>::from(al64);
    const V nal = cvt<V>::from(cx(-al64.re, -al64.im));
    const V* __restrict__ ro = A.vec(par ? CR1 : CR0, b);
    const V* __restrict__ w = A.vec(CW, b);
    V rn = ro[r];
    cfma(rn, nal, w[r]);
    V z = cvt<V>::real(0.0);
    if (fac) {
#pragma unroll
      for (int k = 0; k < WMAX; ++k) {
        const int64_t c = rows.col[k];
        V rc = ro[c];
        cfma(rc, nal, w[c]);
        cfma(z, fv[k], rc);
      }
    } else {
      z = rn;
    }
    V* __restrict__ x = A.vec(CX, b);
    V xv = x[r];
    cfma(xv, al, A.vec(par ? CP1 : CP0, b)[r]);
    x[r] = xv;
    A.vec(par ? CR0 : CR1, b)[r] = rn;
    A.vec(L > 1 ? A.chain_out(0, L) : CZ, b)[r] = z;
    put_total(A, 2, b, s, lane, (double)abs2(rn));
    if (L <= 1) {  // otherwise the chain's last factor forms the products
      const V rz = rn * z, zw = z * w[r];
      put_total(A, 3, b, s, lane, (double)rz.re);
      put_total(A, 4, b, s, lane, (double)rz.im);
      put_total(A, 5, b, s, lane, (double)zw.re);
      put_total(A, 6, b, s, lane, (double)zw.im);
    }
  }
}

// Chain position q >= 1 (the factor Q_{q+1} of Algorithm 5's chain) for
// every active system whose chain is longer than q: z_q = Q z_{q-1}, the
// neighbours' z_{q-1} read from the previous position's vector.  At a
// chain's last position the products of the step: r^T z (init: r = r_0)
// and, in an iteration, z^T w (r = r_new of parity par).
template <int WMAX, typename V>
__global__ void __launch_bounds__(256) k_cchain(CArgsT<V> A, int q, int init, int par) {
  const int lane = threadIdx.x & 63;
  const int s = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (s >= A.pd.n_slices) return;
  CRows<WMAX> rows;
  rows.load(A.pd, s, lane);
  const int64_t r = rows.row;
  int loaded = -1;
  V fv[WMAX];
  for (int b = 0; b < A.B; ++b) {
    if (sload(A.sys.active + b) == 0) continue;
    const int sh = b / A.m;
    const int L = sload(A.clen + sh);
    if (L <= q) continue;
    if (sh != loaded) {
      rows.factor(A.pd, s, sload(A.fac + (int64_t)sh * A.maxc + q), fv);
      loaded = sh;
    }
    const V* __restrict__ zi = A.vec(A.chain_out(q - 1, L), b);
    V z = cvt<V>::real(0.0);
#pragma unroll
    for (int k = 0; k < WMAX; ++k) cfma(z, fv[k], zi[rows.col[k]]);
    A.vec(A.chain_out(q, L), b)[r] = z;
    if (q == L - 1) {
      const V rv = A.vec(init ? CR0 : (par ? CR0 : CR1), b)[r];
      const V rz = rv * z;
      put_total(A, 3, b, s, lane, (double)rz.re);
      put_total(A, 4, b, s, lane, (double)rz.im);
      if (!init) {
        const V zw = z * A.vec(CW, b)[r];
        put_total(A, 5, b, s, lane, (double)zw.re);
        put_total(A, 6, b, s, lane, (double)zw.im);
      }
    }
  }
}

// True residual F - K(s) x (slot 2 = its squared norm) and X out.
template <int WMAX>
__global__ void __launch_bounds__(256) k_cresid(CArgs A, const double* __restrict__ F, int64_t ldf,
                                                double* __restrict__ X, int64_t ldx) {
  const int lane = threadIdx.x & 63;
  const int s = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (s >= A.pd.n_slices) return;
  CRows<WMAX> rows;
  rows.load(A.pd, s, lane);
  const int64_t n = A.pd.n, r = rows.row;
  for (int b = 0; b < A.B; ++b) {
    const int sh = b / A.m, c = b % A.m;
    const cplx ka = sload_c(A.ca + sh), kb = sload_c(A.cb + sh);
    const cplx* __restrict__ x = A.vec(CX, b);
    cplx am = cx(0.0), ak = cx(0.0);
#pragma unroll
    for (int k = 0; k < WMAX; ++k) {
      const cplx xc = x[rows.col[k]];
      rfma(am, rows.mv[k], xc);
      rfma(ak, rows.kv[k], xc);
    }
    const cplx kx = ka * am + kb * ak;
    double res2 = 0.0;
    if (r < n) {
      const cplx rr = cx(F[(int64_t)c * ldf + r]) - kx;
      res2 = abs2(rr);
      const cplx xr = x[r];
      double* xo = X + 2 * ((int64_t)b * ldx + r);
      xo[0] = xr.re;
      xo[1] = xr.im;
    }
    put_total(A, 2, b, s, lane, res2);
  }
}

enum { CM_INIT = 0, CM_PW, CM_ITER, CM_FINAL, CM_OUTER };

struct CRed {
  CSys sys;
  const double* partial;
  int32_t B, GP, max_iter, flexible;
  double tol2_rel;
  // CM_OUTER (MIXED): stop when ||F - K X||^2 <= tol2_abs ||F||^2, after
  // max_sweeps sweeps, or once max_iter_total inner iterations are spent
  double tol2_abs;
  int32_t max_sweeps, max_iter_total;
};

// One block per system: fixed-order sums of the slots the mode needs, then
// the recurrence's scalar logic.
__global__ void __launch_bounds__(256) k_creduce(CRed P, int mode) {
  __shared__ double red[4][kCSlots];
  const int b = blockIdx.x, t = threadIdx.x;
  const CSys& S = P.sys;
  if (mode == CM_OUTER ? S.outer[b] == 0 : (mode != CM_FINAL && S.active[b] == 0)) return;
  double v[kCSlots];
#pragma unroll
  for (int q = 0; q < kCSlots; ++q) v[q] = 0.0;
  const int64_t qs = (int64_t)P.B * P.GP;
  const double* base = P.partial + (int64_t)b * P.GP;
  for (int g = t; g < P.GP; g += 256)
#pragma unroll
    for (int q = 0; q < kCSlots; ++q) v[q] += base[q * qs + g];
#pragma unroll
  for (int q = 0; q < kCSlots; ++q) v[q] = wave_total(v[q]);
  if ((t & 63) == 0)
#pragma unroll
    for (int q = 0; q < kCSlots; ++q) red[t >> 6][q] = v[q];
  __syncthreads();
  if (t != 0) return;
  double s[kCSlots];
#pragma unroll
  for (int q = 0; q < kCSlots; ++q) s[q] = red[0][q] + red[1][q] + red[2][q] + red[3][q];
  const int was = S.active[b];
  int act = was;
  switch (mode) {
    case CM_INIT: {
      S.ff[b] = s[2];
      S.tol2[b] = P.tol2_rel * s[2];
      S.beta[b] = cx(0.0);
      S.rho[b] = cx(s[3], s[4]);
      S.relres[b] = 1.0;
      if (!isfinite(s[2]) || !isfinite(s[3]) || !isfinite(s[4])) { S.istat[b] = AIRGA_SYS_NONFINITE; act = 0; }
      else if (s[2] == 0.0) { S.istat[b] = AIRGA_SYS_CONVERGED; act = 0; }
      break;
    }
    case CM_PW: {
      const cplx mu = cx(s[0], s[1]);
      if (!isfinite(mu.re) || !isfinite(mu.im)) { S.istat[b] = AIRGA_SYS_NONFINITE; act = 0; }
      else if (mu.re == 0.0 && mu.im == 0.0) { S.istat[b] = AIRGA_SYS_BREAKDOWN; act = 0; }
      else { S.mu[b] = mu; S.alpha[b] = cdiv(S.rho[b], mu); }
      break;
    }
    case CM_ITER: {
      const int it = S.iters[b] + 1;
      S.iters[b] = it;
      const cplx rz = cx(s[3], s[4]), zw = cx(s[5], s[6]);
      bool fin = isfinite(s[2]) && isfinite(rz.re) && isfinite(rz.im) && isfinite(zw.re) &&
                 isfinite(zw.im);
      if (!fin) { S.istat[b] = AIRGA_SYS_NONFINITE; act = 0; }
      else if (s[2] <= S.tol2[b]) { S.istat[b] = AIRGA_SYS_CONVERGED; act = 0; }
      else if (it >= P.max_iter) { S.istat[b] = AIRGA_SYS_MAXIT; act = 0; }
      else {
        const cplx bf = cdiv(zw, S.mu[b]);
        S.beta[b] = P.flexible ? cx(-bf.re, -bf.im) : cdiv(rz, S.rho[b]);
        S.rho[b] = rz;
      }
      break;
    }
    case CM_FINAL: {
      S.relres[b] = S.ff[b] > 0 ? sqrt(s[2] / S.ff[b]) : 0.0;
      break;
    }
    case CM_OUTER: {
      // slot 2 = ||F - K X||^2 in float64, slot 3 = ||F||^2 (first time)
      const int sw = S.sweeps[b];
      if (sw == 0) S.fo[b] = s[3];
      const double ff = S.fo[b];
      S.relres[b] = ff > 0 ? sqrt(s[2] / ff) : 0.0;
      S.itot[b] += S.iters[b];
      S.iters[b] = 0;
      int st = -1;
      if (!isfinite(s[2])) st = AIRGA_SYS_NONFINITE;
      else if (s[2] <= P.tol2_abs * ff) st = AIRGA_SYS_CONVERGED;
      else if (sw > 0 && (S.istat[b] == AIRGA_SYS_BREAKDOWN || S.istat[b] == AIRGA_SYS_NONFINITE))
        st = S.istat[b];
      else if (sw >= P.max_sweeps || S.itot[b] >= P.max_iter_total) st = AIRGA_SYS_MAXIT;
      if (st >= 0) {
        S.ostat[b] = st;
        S.outer[b] = 0;
        atomicAdd(S.nout, -1);
      }
      return;
    }
  }
  if (act != was) {
    S.active[b] = act;
    atomicAdd(S.nact, act - was);
  }
}

__global__ void k_cstate(CSys S, int B) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b == 0) *S.nact = B;
  if (b >= B) return;
  S.active[b] = 1;
  S.istat[b] = AIRGA_SYS_MAXIT;
  S.iters[b] = 0;
}

__global__ void k_cfill(cplx* p, int64_t count) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < count) p[i] = cx(0.0);
}

// ------------------------------------------------------------ MIXED mode
//
// Iterative refinement around float32 COCG, as for real points: the
// float64 residual r = F - K(s) X of the float64 solution X, a float32 COCG
// solve K(s) d = r to a relative reduction inner_tol (float32 pencil,
// factors and vectors, float64 scalar recurrence), X += d.

// MIXED state: every system refined, none finished.
__global__ void k_cstate_mixed(CSys S, int B) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b == 0) *S.nout = B;
  if (b >= B) return;
  S.outer[b] = 1;
  S.ostat[b] = AIRGA_SYS_MAXIT;
  S.sweeps[b] = 0;
  S.itot[b] = 0;
  S.iters[b] = 0;
  S.istat[b] = AIRGA_SYS_MAXIT;
}

// The next inner solve: the refined systems are its active ones.
__global__ void k_cstart_inner(CSys S, int B) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b == 0) *S.nact = *S.nout;
  if (b >= B) return;
  S.active[b] = S.outer[b];
  S.istat[b] = AIRGA_SYS_MAXIT;
  S.iters[b] = 0;
}

// float64 residual r = F - K(s) X for the refined systems (xread = 0: X = 0,
// r = F), written in float into the inner solve's r0; partials slot 2 =
// ||r||^2, slot 3 = ||F||^2.  X: complex float64 interleaved, column b at
// X + 2 b ldx (n rows); rows past n give r = 0.
template <int WMAX>
__global__ void __launch_bounds__(256) k_cresid_ir(CArgsT<cf> A, const double* __restrict__ F,
                                                   int64_t ldf, const double* __restrict__ X,
                                                   int64_t ldx, int xread) {
  const int lane = threadIdx.x & 63;
  const int s = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (s >= A.pd.n_slices) return;
  CRows<WMAX> rows;
  rows.load(A.pd, s, lane);
  const int64_t n = A.pd.n, r = rows.row;
  const bool in = r < n;
  for (int b = 0; b < A.B; ++b) {
    if (sload(A.sys.outer + b) == 0) continue;
    const int sh = b / A.m, c = b % A.m;
    const double fr = in ? F[(int64_t)c * ldf + r] : 0.0;
    cplx res = cx(fr);
    if (xread) {
      const cplx ka = sload_c(A.ca + sh), kb = sload_c(A.cb + sh);
      const double* __restrict__ x = X + 2 * (int64_t)b * ldx;
      cplx am = cx(0.0), ak = cx(0.0);
#pragma unroll
      for (int k = 0; k < WMAX; ++k) {
        const int64_t cc = rows.col[k];
        const int64_t ci = cc < n ? cc : 0;  // padding rows: col = row >= n
        const cplx xc = cc < n ? cplx{x[2 * ci], x[2 * ci + 1]} : cx(0.0);
        rfma(am, rows.mv[k], xc);
        rfma(ak, rows.kv[k], xc);
      }
      res = in ? res - (ka * am + kb * ak) : cx(0.0);
    }
    A.vec(CR0, b)[r] = cf{(float)res.re, (float)res.im};
    put_total(A, 2, b, s, lane, abs2(res));
    put_total(A, 3, b, s, lane, fr * fr);
  }
}

// X = 0 (complex float64 interleaved, n rows per column b).
__global__ void k_czero_x(double* __restrict__ X, int64_t ldx, int64_t n) {
  const int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (r >= n) return;
  double* x = X + 2 * ((int64_t)blockIdx.y * ldx + r);
  x[0] = 0.0;
  x[1] = 0.0;
}

// X += d (float32 solution of the inner solve) for the refined systems;
// assign (first sweep): X = d.  Counts the sweep.
__global__ void k_cir_update(CArgsT<cf> A, double* __restrict__ X, int64_t ldx, int assign) {
  const int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int b = blockIdx.y;
  if (A.sys.outer[b] == 0) return;
  if (r < A.pd.n) {
    const cf d = A.vec(CX, b)[r];
    double* x = X + 2 * ((int64_t)b * ldx + r);
    x[0] = (assign ? 0.0 : x[0]) + (double)d.re;
    x[1] = (assign ? 0.0 : x[1]) + (double)d.im;
  }
  if (r == 0) A.sys.sweeps[b] += 1;
}

struct CKernels {
  void (*init)(CArgs, const double*, int64_t, int);
  void (*dir)(CArgs, int);
  void (*upd)(CArgs, int);
  void (*resid)(CArgs, const double*, int64_t, double*, int64_t);
  void (*chain)(CArgs, int, int, int);
};

struct CKernels32 {
  void (*init)(CArgsT<cf>, const double*, int64_t, int);
  void (*dir)(CArgsT<cf>, int);
  void (*upd)(CArgsT<cf>, int);
  void (*chain)(CArgsT<cf>, int, int, int);
};

template <int W>
CKernels32 ckernels32() {
  return CKernels32{k_cinit<W, cf>, k_cdir<W, cf>, k_cupd<W, cf>, k_cchain<W, cf>};
}

template <int W>
CKernels ckernels() {
  return CKernels{k_cinit<W, cplx>, k_cdir<W, cplx>, k_cupd<W, cplx>, k_cresid<W>,
                  k_cchain<W, cplx>};
}

// MIXED mode: float64 refinement around float32 COCG inner solves, every
// system from X = 0.  A: the float64 setup (workspace, shift data, chains
// of float factor copies, state); its vectors are reused as float complex.
// A system ends CONVERGED once its float64 residual meets tol, MAXIT after
// max_sweeps sweeps or max_iter inner iterations in all, BREAKDOWN or
// NONFINITE when an inner solve does.
airga_status cocg_mixed(airga_ctx ctx, const CArgs& A, const double* F, int64_t ldf,
                        double* X, int64_t ldx, const airga_pcg_opts& o,
                        airga_sys_stats* stats) {
  hipStream_t st = ctx->stream;
  const Pencil& pen = ctx->pen;
  const int B = A.B;
  const CSys& S = A.sys;
  CArgsT<cf> A32{};
  A32.pd = A.pd;
  A32.B = B;
  A32.m = A.m;
  A32.ld = A.ld;
  A32.ws = reinterpret_cast<cf*>(A.ws);
  A32.ca = A.ca;
  A32.cb = A.cb;
  A32.fac = reinterpret_cast<const cf* const*>(A.fac);
  A32.clen = A.clen;
  A32.maxc = A.maxc;
  A32.partial = A.partial;
  A32.GP = A.GP;
  A32.sys = S;
  const unsigned grid = blocks_for(pen.n_slices, 4);
  int k = o.poll_every < 2 ? 2 : o.poll_every;
  k += k & 1;
  int64_t cap = o.inner_max > 0 ? o.inner_max : 96;
  cap = (cap + k - 1) / k * k;
  CRed R{S, A.partial, B, A.GP, (int32_t)cap, o.beta_form == AIRGA_BETA_CLASSICAL ? 0 : 1,
         o.inner_tol * o.inner_tol, o.tol * o.tol, o.max_sweeps, o.max_iter};
  // zero float vectors (half as many float64 complex slots), X = 0, state
  const int64_t half = (int64_t)CKINDS * B * A.ld / 2;
  k_cfill<<<blocks_for(half, 256), 256, 0, st>>>(A.ws, half);
  k_czero_x<<<dim3(blocks_for(pen.n, 256), (unsigned)B), 256, 0, st>>>(X, ldx, pen.n);
  k_cstate_mixed<<<blocks_for(B, 256), 256, 0, st>>>(S, B);
  // sweep 0: r = F
  k_cresid_ir<6><<<grid, 256, 0, st>>>(A32, F, ldf, X, ldx, 0);
  k_creduce<<<(unsigned)B, 256, 0, st>>>(R, CM_OUTER);
  AIRGA_HIP(hipGetLastError());
  AIRGA_TRY(ensure_pinned(ctx, 64));
  int32_t* h_cnt = static_cast<int32_t*>(ctx->host_pinned);
  const CKernels32 ks = ckernels32<6>();
  const dim3 ir_grid(blocks_for(pen.n, 256), (unsigned)B);
  const int64_t rounds = cap / k + 2;
  for (int sweep = 0; sweep < o.max_sweeps; ++sweep) {
    AIRGA_HIP(hipMemcpyAsync(h_cnt, S.nout, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    AIRGA_HIP(hipStreamSynchronize(st));
    if (*h_cnt == 0) break;
    // inner COCG on K(s) d = r from d = 0
    k_cstart_inner<<<blocks_for(B, 256), 256, 0, st>>>(S, B);
    ks.init<<<grid, 256, 0, st>>>(A32, F, ldf, 1);
    for (int q = 1; q < A.maxc; ++q) ks.chain<<<grid, 256, 0, st>>>(A32, q, 1, 0);
    k_creduce<<<(unsigned)B, 256, 0, st>>>(R, CM_INIT);
    AIRGA_HIP(hipGetLastError());
    for (int64_t round = 0; round < rounds; ++round) {
      AIRGA_HIP(hipMemcpyAsync(h_cnt, S.nact, sizeof(int32_t), hipMemcpyDeviceToHost, st));
      AIRGA_HIP(hipStreamSynchronize(st));
      if (*h_cnt == 0) break;
      for (int j = 0; j < k; ++j) {
        const int par = j & 1;
        ks.dir<<<grid, 256, 0, st>>>(A32, par);
        k_creduce<<<(unsigned)B, 256, 0, st>>>(R, CM_PW);
        ks.upd<<<grid, 256, 0, st>>>(A32, par);
        for (int q = 1; q < A.maxc; ++q) ks.chain<<<grid, 256, 0, st>>>(A32, q, 0, par);
        k_creduce<<<(unsigned)B, 256, 0, st>>>(R, CM_ITER);
      }
      AIRGA_HIP(hipGetLastError());
    }
    // X += d, then the float64 residual decides
    k_cir_update<<<ir_grid, 256, 0, st>>>(A32, X, ldx, 0);
    k_cresid_ir<6><<<grid, 256, 0, st>>>(A32, F, ldf, X, ldx, 1);
    k_creduce<<<(unsigned)B, 256, 0, st>>>(R, CM_OUTER);
    AIRGA_HIP(hipGetLastError());
  }
  // per-system results: relres, then status, sweeps and iterations
  const size_t rb = sizeof(double) * B, ib = sizeof(int32_t) * B;
  AIRGA_TRY(ensure_pinned(ctx, rb + 3 * ib));
  char* h = static_cast<char*>(ctx->host_pinned);
  AIRGA_HIP(hipMemcpyAsync(h, S.relres, rb, hipMemcpyDeviceToHost, st));
  AIRGA_HIP(hipMemcpyAsync(h + rb, S.ostat, 3 * ib, hipMemcpyDeviceToHost, st));
  AIRGA_HIP(hipStreamSynchronize(st));
  if (stats) {
    const double* rel = reinterpret_cast<const double*>(h);
    const int32_t* ist = reinterpret_cast<const int32_t*>(h + rb);
    for (int b = 0; b < B; ++b) {
      stats[b].status = ist[b];
      stats[b].sweeps = ist[B + b];
      stats[b].iters = ist[2 * B + b];
      stats[b].finished_fp64 = 0;
      stats[b].relres = rel[b];
    }
  }
  return AIRGA_OK;
}

airga_status check_cshift(const Pencil& pen, double re, double im) {
  if (!std::isfinite(re) || !std::isfinite(im))
    return fail(AIRGA_EINVAL, "complex shift must be finite");
  if (pen.max_len > 6)
    return fail(AIRGA_EUNSUPPORTED, "complex shifts take rows of at most 6 entries");
  return AIRGA_OK;
}

// The complex update's launches (everything but the readback of alpha and
// the skip count, which cupdate_finish takes); *out is the new factor, not
// yet chained to old.
airga_status cupdate_launch(airga_ctx ctx, airga_prec old, double s_re, double s_im,
                            const airga_spai_opts* opts, airga_prec* out) {
  *out = nullptr;
  if (!old) return fail(AIRGA_EINVAL, "null preconditioner");
  const Pencil& pen = ctx->pen;
  if (old->ctx != ctx) return fail(AIRGA_EINVAL, "preconditioner belongs to another context");
  if (old->generation != pen.generation)
    return fail(AIRGA_ESTATE, "preconditioner was built for an earlier pencil");
  if (!old->is_complex)
    return fail(AIRGA_EINVAL, "the old factor is real: build it with airga_spai_build_complex");
  AIRGA_TRY(check_cshift(pen, s_re, s_im));
  airga_spai_opts o;
  airga_spai_opts_default(&o);
  if (opts) o = *opts;
  if (o.mr_iters != 0 || o.lfil != 0)
    return fail(AIRGA_EUNSUPPORTED, "the minimal-residual mode is for real shifts only");
  if (!(o.tol >= 0)) return fail(AIRGA_EINVAL, "update tolerance must be >= 0");
  airga_prec p = new (std::nothrow) airga_prec_s();
  if (!p) return fail(AIRGA_ENOMEM, "host allocation failed");
  p->ctx = ctx;
  p->generation = pen.generation;
  p->shift = s_re;
  p->shift_im = s_im;
  p->is_complex = true;
  p->is_update = true;
  const size_t stored = (size_t)pen.nnz_stored;
  const size_t npad = (size_t)pen.n_pad();
  const unsigned nb = blocks_for(pen.n, 256);
  airga_status st;
  // scal: alpha (2 doubles) | skip count (int32 at 16) | skipped flags (from 64)
  if ((st = pool_get(ctx, &p->v64, sizeof(cplx) * stored)) != AIRGA_OK ||
      (st = pool_get(ctx, &p->v32, 2 * sizeof(float) * stored)) != AIRGA_OK ||
      (st = pool_get(ctx, &p->objective, sizeof(double) * pen.n)) != AIRGA_OK ||
      (st = pool_get(ctx, &p->scal, 64 + npad)) != AIRGA_OK ||
      (st = ctx->ws_tmp.reserve(sizeof(cplx) * (stored + npad) + 3 * sizeof(double) * nb)) !=
          AIRGA_OK) {
    pool_put(ctx, &p->v64);
    pool_put(ctx, &p->v32);
    pool_put(ctx, &p->objective);
    pool_put(ctx, &p->scal);
    delete p;
    return st;
  }
  ctx->live_precs++;
  cplx a, b, ao, bo;
  ccoeffs(pen, cx(s_re, s_im), &a, &b);
  ccoeffs(pen, cx(old->shift, old->shift_im), &ao, &bo);
  cplx* dinv = ctx->ws_tmp.as<cplx>();
  cplx* hat = dinv + npad;
  double* part = reinterpret_cast<double*>(hat + stored);
  double* alpha_d = p->scal.as<double>();
  int32_t* skip = reinterpret_cast<int32_t*>(p->scal.as<char>() + 16);
  int8_t* skipf = reinterpret_cast<int8_t*>(p->scal.as<char>() + 64);
  hipStream_t hs = ctx->stream;
  const PencilDev pd = pen.dev();
  // both matrices scaled by the new diagonal: Khat_x = S_new K(s_x) S_new
  k_cdinv<<<blocks_for((int64_t)npad, 256), 256, 0, hs>>>(pd, a, b, o.equilibrate ? 1 : 0, dinv);
  k_calpha_partial<<<nb, 256, 0, hs>>>(pd, a, b, ao, bo, dinv, part);
  k_calpha_final<<<1, 256, 0, hs>>>(part, nb, alpha_d, skip);
  // equilibrated updates on narrow bands of consecutive columns: normal
  // equations first, rotations for the columns they flag
  const bool gram = !o.general_only && o.equilibrate && pen.contiguous && pen.max_len <= 6 &&
                    pen.bandwidth <= kCGramMaxBw;
  int8_t* redo = nullptr;
  if (gram) {
    if ((st = ctx->ws_gather.reserve((size_t)pen.n)) != AIRGA_OK) {
      airga_prec_release(p);
      return st;
    }
    redo = ctx->ws_gather.as<int8_t>();
    k_cspai_gram<6, true><<<blocks_for(pen.n, 64), 64, cspai_gram_lds(pen.bandwidth, 6, true), hs>>>(
        pd, a, b, dinv, pen.bandwidth, hat, p->objective.as<double>(), redo, ao, bo, alpha_d,
        o.tol, skipf, skip);
  }
  k_cspai_cols<6, true><<<blocks_for(pen.n, 64), 64, 0, hs>>>(
      pd, a, b, dinv, hat, p->objective.as<double>(), redo, ao, bo, alpha_d, o.tol, skipf, skip);
  k_cspai_finalize<<<blocks_for((int64_t)npad, 256), 256, 0, hs>>>(
      pd, hat, dinv, 0, p->v64.as<cplx>(), p->v32.as<float>(), skipf, alpha_d, skip);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    airga_prec_release(p);
    return fail(AIRGA_EHIP, "complex SPAI update: %s", hipGetErrorString(e));
  }
  *out = p;
  return AIRGA_OK;
}

// alpha (2 doubles) and the skip count at the head of a complex update's
// scal block
struct CUpdScal {
  double alpha[2];
  int32_t skipped, pad;
};

// The update's scalars once read back; the factor joins old's chain.
void cupdate_finish(airga_prec p, airga_prec old, const CUpdScal& h) {
  p->alpha = h.alpha[0];
  p->alpha_im = h.alpha[1];
  p->alpha_known = true;
  p->skipped = h.skipped;
  p->scalar_only = h.skipped == p->ctx->pen.n;
  p->scalar_known = true;
  p->parent = old;
  old->refs++;
}

}  // namespace
}  // namespace airga

using namespace airga;

extern "C" {

airga_status airga_assemble_shift_complex(airga_ctx ctx, double s_re, double s_im,
                                          double* a_val) {
  AIRGA_TRY(check_pencil(ctx));
  DeviceGuard g(ctx->device);
  if (!a_val) return fail(AIRGA_EINVAL, "null output");
  if (!std::isfinite(s_re) || !std::isfinite(s_im))
    return fail(AIRGA_EINVAL, "complex shift must be finite");
  const Pencil& pen = ctx->pen;
  cplx a, b;
  ccoeffs(pen, cx(s_re, s_im), &a, &b);
  k_cassemble<<<blocks_for(pen.nnz_stored, 256), 256, 0, ctx->stream>>>(pen.dev(), pen.nnz_stored, a,
                                                                        b, a_val);
  AIRGA_HIP(hipGetLastError());
  return AIRGA_OK;
}

airga_status airga_spai_build_complex(airga_ctx ctx, double s_re, double s_im,
                                      const airga_spai_opts* opts, airga_prec* out) {
  AIRGA_TRY(check_pencil(ctx));
  DeviceGuard g(ctx->device);
  if (!out) return fail(AIRGA_EINVAL, "null output handle");
  *out = nullptr;
  const Pencil& pen = ctx->pen;
  AIRGA_TRY(check_cshift(pen, s_re, s_im));
  airga_spai_opts o;
  airga_spai_opts_default(&o);
  if (opts) o = *opts;
  if (o.mr_iters != 0 || o.lfil != 0)
    return fail(AIRGA_EUNSUPPORTED, "the minimal-residual mode is for real shifts only");
  airga_prec p = new (std::nothrow) airga_prec_s();
  if (!p) return fail(AIRGA_ENOMEM, "host allocation failed");
  p->ctx = ctx;
  p->generation = pen.generation;
  p->shift = s_re;
  p->shift_im = s_im;
  p->is_complex = true;
  p->skipped = 0;
  p->scalar_only = false;
  p->scalar_known = true;
  // the Frobenius minimiser of ||I - alpha K(s)||: conj(trace K(s)) / ||K(s)||_F^2
  cplx a, b;
  ccoeffs(pen, cx(s_re, s_im), &a, &b);
  const cplx tr = a * cx(pen.tr_m) + b * cx(pen.tr_k);
  const double fro2 = abs2(a) * pen.gram_mm + 2.0 * (a * conj(b)).re * pen.gram_mk +
                      abs2(b) * pen.gram_kk;
  p->alpha = fro2 > 0 ? tr.re / fro2 : 0.0;
  p->alpha_im = fro2 > 0 ? -tr.im / fro2 : 0.0;
  p->alpha_known = true;
  const size_t stored = (size_t)pen.nnz_stored;
  const size_t npad = (size_t)pen.n_pad();
  airga_status st;
  if ((st = pool_get(ctx, &p->v64, sizeof(cplx) * stored)) != AIRGA_OK ||
      (st = pool_get(ctx, &p->v32, 2 * sizeof(float) * stored)) != AIRGA_OK ||
      (st = pool_get(ctx, &p->objective, sizeof(double) * pen.n)) != AIRGA_OK ||
      (st = ctx->ws_tmp.reserve(sizeof(cplx) * (stored + npad))) != AIRGA_OK) {
    pool_put(ctx, &p->v64);
    pool_put(ctx, &p->v32);
    pool_put(ctx, &p->objective);
    delete p;
    return st;
  }
  ctx->live_precs++;
  cplx* dinv = ctx->ws_tmp.as<cplx>();
  cplx* hat = dinv + npad;
  hipStream_t s = ctx->stream;
  const PencilDev pd = pen.dev();
  k_cdinv<<<blocks_for((int64_t)npad, 256), 256, 0, s>>>(pd, a, b, o.equilibrate ? 1 : 0, dinv);
  // equilibrated builds on narrow bands of consecutive columns: normal
  // equations, with the Givens kernel for the columns they cannot take
  const bool gram = !o.general_only && o.equilibrate && pen.contiguous && pen.max_len <= 6 &&
                    pen.bandwidth <= kCGramMaxBw;
  int8_t* redo = nullptr;
  if (gram) {
    if ((st = ctx->ws_gather.reserve((size_t)pen.n)) != AIRGA_OK) {
      airga_prec_release(p);
      return st;
    }
    redo = ctx->ws_gather.as<int8_t>();
    k_cspai_gram<6, false><<<blocks_for(pen.n, 64), 64, cspai_gram_lds(pen.bandwidth, 6, false), s>>>(
        pd, a, b, dinv, pen.bandwidth, hat, p->objective.as<double>(), redo, cx(0.0), cx(0.0),
        nullptr, 0.0, nullptr, nullptr);
  }
  k_cspai_cols<6, false><<<blocks_for(pen.n, 64), 64, 0, s>>>(
      pd, a, b, dinv, hat, p->objective.as<double>(), redo, cx(0.0), cx(0.0), nullptr, 0.0,
      nullptr, nullptr);
  k_cspai_finalize<<<blocks_for((int64_t)npad, 256), 256, 0, s>>>(
      pd, hat, dinv, o.symmetrize ? 1 : 0, p->v64.as<cplx>(), p->v32.as<float>(), nullptr,
      nullptr, nullptr);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    airga_prec_release(p);
    return fail(AIRGA_EHIP, "complex SPAI launch: %s", hipGetErrorString(e));
  }
  *out = p;
  return AIRGA_OK;
}

airga_status airga_spai_update_complex(airga_ctx ctx, airga_prec old, double s_re, double s_im,
                                       const airga_spai_opts* opts, airga_prec* out) {
  AIRGA_TRY(check_pencil(ctx));
  DeviceGuard g(ctx->device);
  if (!out) return fail(AIRGA_EINVAL, "null output handle");
  *out = nullptr;
  airga_prec p = nullptr;
  AIRGA_TRY(cupdate_launch(ctx, old, s_re, s_im, opts, &p));
  // alpha and the skip count, read once (the solves need to know whether
  // the factor is the scalar alpha I)
  CUpdScal h{};
  hipError_t e = hipMemcpyAsync(&h, p->scal.ptr, sizeof h, hipMemcpyDeviceToHost, ctx->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  if (e != hipSuccess) {
    airga_prec_release(p);
    return fail(AIRGA_EHIP, "complex SPAI update: %s", hipGetErrorString(e));
  }
  cupdate_finish(p, old, h);
  *out = p;
  return AIRGA_OK;
}

airga_status airga_spai_update_complex_many(airga_ctx ctx, int32_t count, const airga_prec* olds,
                                            const double* shifts, const airga_spai_opts* opts,
                                            airga_prec* out) {
  AIRGA_TRY(check_pencil(ctx));
  DeviceGuard g(ctx->device);
  if (count < 0) return fail(AIRGA_EINVAL, "negative count");
  if (count > 0 && (!olds || !shifts || !out)) return fail(AIRGA_EINVAL, "null array");
  for (int i = 0; i < count; ++i) out[i] = nullptr;
  std::vector<airga_prec> ps(count, nullptr);
  auto drop = [&]() {
    for (airga_prec q : ps) airga_prec_release(q);
  };
  for (int i = 0; i < count; ++i) {
    const airga_status st = cupdate_launch(ctx, olds[i], shifts[2 * i], shifts[2 * i + 1], opts, &ps[i]);
    if (st != AIRGA_OK) {
      drop();
      return st;
    }
  }
  if (count == 0) return AIRGA_OK;
  // one readback of every update's scalars
  const airga_status pst = ensure_pinned(ctx, sizeof(CUpdScal) * (size_t)count);
  if (pst != AIRGA_OK) {
    drop();
    return pst;
  }
  CUpdScal* h = static_cast<CUpdScal*>(ctx->host_pinned);
  hipError_t e = hipSuccess;
  for (int i = 0; i < count && e == hipSuccess; ++i)
    e = hipMemcpyAsync(h + i, ps[i]->scal.ptr, sizeof(CUpdScal), hipMemcpyDeviceToHost, ctx->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  if (e != hipSuccess) {
    drop();
    return fail(AIRGA_EHIP, "complex SPAI updates: %s", hipGetErrorString(e));
  }
  for (int i = 0; i < count; ++i) {
    cupdate_finish(ps[i], olds[i], h[i]);
    out[i] = ps[i];
  }
  return AIRGA_OK;
}

airga_status airga_spai_build_complex_many(airga_ctx ctx, int32_t count, const double* shifts,
                                           const airga_spai_opts* opts, airga_prec* out) {
  AIRGA_TRY(check_pencil(ctx));
  if (count < 0) return fail(AIRGA_EINVAL, "negative count");
  if (count > 0 && (!shifts || !out)) return fail(AIRGA_EINVAL, "null array");
  for (int i = 0; i < count; ++i) out[i] = nullptr;
  for (int i = 0; i < count; ++i) {
    const airga_status st = airga_spai_build_complex(ctx, shifts[2 * i], shifts[2 * i + 1], opts, out + i);
    if (st != AIRGA_OK) {
      for (int k = 0; k < i; ++k) {
        airga_prec_release(out[k]);
        out[k] = nullptr;
      }
      return st;
    }
  }
  return AIRGA_OK;
}

airga_status airga_prec_export_complex(airga_prec prec, double* values, double* objective) {
  if (!prec) return fail(AIRGA_EINVAL, "null preconditioner");
  AIRGA_TRY(check_pencil(prec->ctx));
  if (prec->generation != prec->ctx->pen.generation)
    return fail(AIRGA_ESTATE, "preconditioner was built for an earlier pencil");
  if (!prec->is_complex) return fail(AIRGA_EINVAL, "not a complex factor");
  airga_ctx ctx = prec->ctx;
  DeviceGuard g(ctx->device);
  const Pencil& pen = ctx->pen;
  if (values) {
    if (prec->scalar_only)
      k_cexport_scalar<<<blocks_for(pen.n, 256), 256, 0, ctx->stream>>>(
          pen.dev(), cplx{prec->alpha, prec->alpha_im}, reinterpret_cast<cplx*>(values));
    else
      k_cexport<<<blocks_for(pen.nnz_stored, 256), 256, 0, ctx->stream>>>(
          pen.dev(), pen.nnz_stored, prec->v64.as<cplx>(), reinterpret_cast<cplx*>(values));
    AIRGA_HIP(hipGetLastError());
  }
  if (objective)
    AIRGA_HIP(hipMemcpyAsync(objective, prec->objective.ptr, sizeof(double) * pen.n,
                             hipMemcpyDeviceToDevice, ctx->stream));
  return AIRGA_OK;
}

airga_status airga_cocg_solve(airga_ctx ctx, int32_t nshift, const double* shifts,
                              const airga_prec* precs, int32_t m, const double* F, int64_t ldf,
                              double* X, int64_t ldx, const airga_pcg_opts* opts,
                              airga_sys_stats* stats) {
  AIRGA_TRY(check_pencil(ctx));
  DeviceGuard g(ctx->device);
  const Pencil& pen = ctx->pen;
  if (nshift <= 0 || m <= 0) return fail(AIRGA_EINVAL, "nshift and m must be positive");
  if (!shifts || !F || !X) return fail(AIRGA_EINVAL, "null argument");
  if (ldf < pen.n || ldx < pen.n) return fail(AIRGA_EINVAL, "leading dimension < n");
  airga_pcg_opts o;
  airga_pcg_opts_default(&o);
  if (opts) o = *opts;
  if (o.mode != AIRGA_MODE_FP64 && o.mode != AIRGA_MODE_MIXED)
    return fail(AIRGA_EINVAL, "unknown mode");
  const bool mixed = o.mode == AIRGA_MODE_MIXED;
  if (!(o.tol >= 0) || o.max_iter < 0) return fail(AIRGA_EINVAL, "bad tolerance or iteration cap");
  if (mixed && (!(o.inner_tol > 0 && o.inner_tol < 1) || o.max_sweeps < 1 || o.inner_max < 0))
    return fail(AIRGA_EINVAL, "bad refinement options");
  if (o.x0_given) return fail(AIRGA_EUNSUPPORTED, "complex solves start from X = 0");
  const int64_t B64 = (int64_t)nshift * m;
  if (B64 > 4096) return fail(AIRGA_EUNSUPPORTED, "more than 4096 systems");
  const int B = (int)B64;
  std::vector<cplx> ca(nshift), cb(nshift);
  // each shift's chain P_1, Q_2, ..., Q_z of non-scalar factors (a factor
  // that is a scalar alpha I leaves COCG's iterates unchanged and is dropped)
  std::vector<std::vector<const cplx*>> chains(nshift);
  int maxc = 1;
  for (int k = 0; k < nshift; ++k) {
    AIRGA_TRY(check_cshift(pen, shifts[2 * k], shifts[2 * k + 1]));
    ccoeffs(pen, cx(shifts[2 * k], shifts[2 * k + 1]), &ca[k], &cb[k]);
    const airga_prec p = precs ? precs[k] : nullptr;
    if (p) {
      if (p->ctx != ctx) return fail(AIRGA_EINVAL, "preconditioner belongs to another context");
      if (p->generation != pen.generation)
        return fail(AIRGA_ESTATE, "preconditioner was built for an earlier pencil");
      if (!p->is_complex) return fail(AIRGA_EINVAL, "shift %d: a real factor for a complex solve", k);
      if (p->shift != shifts[2 * k] || p->shift_im != shifts[2 * k + 1])
        return fail(AIRGA_EINVAL, "shift %d: the factor was built at another shift", k);
      std::vector<airga_prec> ch;  // newest first
      AIRGA_TRY(prec_chain(p, &ch));
      // MIXED: the float copies of the factors (cf, as the inner solves read them)
      for (auto it = ch.rbegin(); it != ch.rend(); ++it)
        chains[k].push_back(mixed ? reinterpret_cast<const cplx*>((*it)->v32.ptr)
                                  : (*it)->v64.as<cplx>());
      maxc = (int)chains[k].size() > maxc ? (int)chains[k].size() : maxc;
    }
  }
  hipStream_t st = ctx->stream;
  const int64_t ld = pen.n_pad();
  const int GP = pen.n_slices;
  // workspace: vectors | partials | per-shift data | per-system state
  const size_t vec_b = (mixed ? sizeof(cf) : sizeof(cplx)) * (size_t)CKINDS * B * ld;
  const size_t part_b = sizeof(double) * (size_t)kCSlots * B * GP;
  const size_t shift_b = (2 * sizeof(cplx) + sizeof(void*) * maxc + sizeof(int32_t)) * (size_t)nshift;
  const size_t sys_b = (4 * sizeof(cplx) + 4 * sizeof(double) + 7 * sizeof(int32_t)) * (size_t)B + 64;
  auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
  AIRGA_TRY(ctx->ws_vec.reserve(al(vec_b) + al(part_b) + al(shift_b) + al(sys_b)));
  char* base = ctx->ws_vec.as<char>();
  CArgs A{};
  A.pd = pen.dev();
  A.B = B;
  A.m = m;
  A.ld = ld;
  A.ws = reinterpret_cast<cplx*>(base);
  A.partial = reinterpret_cast<double*>(base + al(vec_b));
  A.GP = GP;
  char* shb = base + al(vec_b) + al(part_b);
  A.ca = reinterpret_cast<const cplx*>(shb);
  A.cb = A.ca + nshift;
  A.fac = reinterpret_cast<const cplx* const*>(shb + 2 * sizeof(cplx) * nshift);
  A.clen = reinterpret_cast<const int32_t*>(shb + 2 * sizeof(cplx) * nshift +
                                            sizeof(void*) * maxc * (size_t)nshift);
  A.maxc = maxc;
  char* sb = shb + al(shift_b);
  CSys S;
  cplx* cs = reinterpret_cast<cplx*>(sb);
  S.rho = cs; S.mu = cs + B; S.alpha = cs + 2 * B; S.beta = cs + 3 * B;
  double* ds = reinterpret_cast<double*>(cs + 4 * B);
  S.tol2 = ds; S.ff = ds + B; S.relres = ds + 2 * B; S.fo = ds + 3 * B;
  int32_t* is = reinterpret_cast<int32_t*>(ds + 4 * B);
  S.active = is; S.istat = is + B; S.iters = is + 2 * B; S.outer = is + 3 * B;
  S.ostat = is + 4 * B; S.sweeps = is + 5 * B; S.itot = is + 6 * B;
  S.nact = is + 7 * B; S.nout = is + 7 * B + 1;
  A.sys = S;
  // per-shift data through pinned memory
  AIRGA_TRY(ensure_pinned(ctx, shift_b + 64));
  char* hp = static_cast<char*>(ctx->host_pinned);
  std::memcpy(hp, ca.data(), sizeof(cplx) * nshift);
  std::memcpy(hp + sizeof(cplx) * nshift, cb.data(), sizeof(cplx) * nshift);
  {
    const cplx** hf = reinterpret_cast<const cplx**>(hp + 2 * sizeof(cplx) * nshift);
    int32_t* hl = reinterpret_cast<int32_t*>(hp + 2 * sizeof(cplx) * nshift +
                                             sizeof(void*) * maxc * (size_t)nshift);
    for (int k = 0; k < nshift; ++k) {
      hl[k] = (int32_t)chains[k].size();
      for (int q = 0; q < maxc; ++q)
        hf[(size_t)k * maxc + q] = q < hl[k] ? chains[k][q] : nullptr;
    }
  }
  AIRGA_HIP(hipMemcpyAsync(shb, hp, shift_b, hipMemcpyHostToDevice, st));
  AIRGA_HIP(hipStreamSynchronize(st));
  if (mixed) return cocg_mixed(ctx, A, F, ldf, X, ldx, o, stats);
  // zero vectors (padding rows stay zero), fresh state
  k_cfill<<<blocks_for((int64_t)CKINDS * B * ld, 256), 256, 0, st>>>(A.ws, (int64_t)CKINDS * B * ld);
  k_cstate<<<blocks_for(B, 256), 256, 0, st>>>(S, B);
  AIRGA_HIP(hipGetLastError());
  const CKernels ks = ckernels<6>();
  const unsigned grid = blocks_for(pen.n_slices, 4);
  CRed R{S, A.partial, B, GP, o.max_iter, o.beta_form == AIRGA_BETA_CLASSICAL ? 0 : 1,
         o.tol * o.tol};
  ks.init<<<grid, 256, 0, st>>>(A, F, ldf, 0);
  for (int q = 1; q < maxc; ++q) ks.chain<<<grid, 256, 0, st>>>(A, q, 1, 0);
  k_creduce<<<(unsigned)B, 256, 0, st>>>(R, CM_INIT);
  AIRGA_HIP(hipGetLastError());
  AIRGA_TRY(ensure_pinned(ctx, 64));
  int32_t* h_nact = static_cast<int32_t*>(ctx->host_pinned);
  int k = o.poll_every < 2 ? 2 : o.poll_every;
  k += k & 1;
  const int64_t rounds = (int64_t)o.max_iter / k + 2;
  for (int64_t round = 0; round < rounds; ++round) {
    AIRGA_HIP(hipMemcpyAsync(h_nact, S.nact, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    AIRGA_HIP(hipStreamSynchronize(st));
    if (*h_nact == 0) break;
    for (int j = 0; j < k; ++j) {
      const int par = j & 1;
      ks.dir<<<grid, 256, 0, st>>>(A, par);
      k_creduce<<<(unsigned)B, 256, 0, st>>>(R, CM_PW);
      ks.upd<<<grid, 256, 0, st>>>(A, par);
      for (int q = 1; q < maxc; ++q) ks.chain<<<grid, 256, 0, st>>>(A, q, 0, par);
      k_creduce<<<(unsigned)B, 256, 0, st>>>(R, CM_ITER);
    }
    AIRGA_HIP(hipGetLastError());
  }
  ks.resid<<<grid, 256, 0, st>>>(A, F, ldf, X, ldx);
  k_creduce<<<(unsigned)B, 256, 0, st>>>(R, CM_FINAL);
  AIRGA_HIP(hipGetLastError());
  // per-system results
  const size_t rb = sizeof(double) * B, ib = sizeof(int32_t) * B;
  AIRGA_TRY(ensure_pinned(ctx, rb + 2 * ib));
  char* h = static_cast<char*>(ctx->host_pinned);
  AIRGA_HIP(hipMemcpyAsync(h, S.relres, rb, hipMemcpyDeviceToHost, st));
  AIRGA_HIP(hipMemcpyAsync(h + rb, S.istat, 2 * ib, hipMemcpyDeviceToHost, st));
  AIRGA_HIP(hipStreamSynchronize(st));
  if (stats) {
    const double* rel = reinterpret_cast<const double*>(h);
    const int32_t* ist = reinterpret_cast<const int32_t*>(h + rb);
    for (int b = 0; b < B; ++b) {
      stats[b].status = ist[b];
      stats[b].iters = ist[B + b];
      stats[b].sweeps = 1;
      stats[b].finished_fp64 = 0;
      stats[b].relres = rel[b];
    }
  }
  return AIRGA_OK;
}

}  // extern "C"
