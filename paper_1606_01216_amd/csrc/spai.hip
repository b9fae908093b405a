// SPAI build (Section 3.1, eq. (3.1)) and SPAI update (Section 3.2) on the
// structural pattern of K(s), one GPU lane per column, plus the factor
// handles and the chain application of the update algorithm.
//
// Column j of the build solves  min || e_j - Khat(:, J) p ||_2  and column j
// of the update solves  min || khat_old_j - Khat_new(:, J) q ||_2, with
// J = pattern of column j.  Only the rows I = union of the patterns of the
// columns in J can be nonzero, so each lane streams the rows of Khat(I, J)
// through a Givens QR held in registers (|J| <= kSpaiMaxJ), then solves the
// triangular system.  Khat = S K S with S = diag(K)^{-1/2} when
// equilibrating (S = I otherwise); every entry of K(s) is formed on the fly
// as (s^2 + alpha s) M + (1 + beta s) K from the float64 pencil.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "internal.hpp"

namespace airga {

// Packed upper-triangular index of (k, l), k <= l, in an MJ x MJ factor.
template <int MJ>
__device__ __host__ constexpr int tri(int k, int l) {
  return k * MJ - (k * (k - 1)) / 2 + (l - k);
}

// 1 / sqrt(x) for a normal positive x: the hardware estimate refined by two
// Newton-Raphson steps y <- y + y (1 - x y^2) / 2 (each roughly doubles the
// correct bits), which leaves an error of a few ulp.
__device__ __forceinline__ double rsqrt_newton(double x) {
  double y = __builtin_amdgcn_rsq(x);
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const double e = fma(-x, y * y, 1.0);
    y = fma(0.5 * y, e, y);
  }
  return y;
}

// Fold one row (v, rhs) of the least-squares problem into the triangular
// factor R and Q^T b by Givens rotations; on return rhs holds the component
// of the row left orthogonal to the column space.
template <int MJ>
__device__ __forceinline__ void givens_row(double (&R)[MJ * (MJ + 1) / 2], double (&qtb)[MJ],
                                           double (&v)[MJ], double& rhs, int nj) {
#pragma unroll
  for (int k = 0; k < MJ; ++k) {
    if (k < nj && v[k] != 0.0) {
      const double rkk = R[tri<MJ>(k, k)];
      // h = hypot(rkk, v_k) and 1 / h from the squares through one
      // reciprocal square root; the scaled library routine only where the
      // squares would under- or overflow
      const double h2 = fma(rkk, rkk, v[k] * v[k]);
      double h, ih;
      if (h2 > 1e-290 && h2 < 1e290) {
        ih = rsqrt_newton(h2);
        h = h2 * ih;
      } else {
        h = hypot(rkk, v[k]);
        ih = 1.0 / h;
      }
      const double c = rkk * ih, s = v[k] * ih;
      R[tri<MJ>(k, k)] = h;
#pragma unroll
      for (int l = k + 1; l < MJ; ++l) {
        if (l < nj) {
          const double rl = R[tri<MJ>(k, l)], vl = v[l];
          // explicit fma: every kernel that folds rows rounds the same way
          R[tri<MJ>(k, l)] = fma(c, rl, s * vl);
          v[l] = fma(c, vl, -(s * rl));
        }
      }
      const double qb = qtb[k];
      qtb[k] = fma(c, qb, s * rhs);
      rhs = fma(c, rhs, -(s * qb));
    }
  }
}

// dinv[r] = diag(K(s))_r^{-1/2} (or 1 without equilibration); padding rows 1.
__global__ void k_dinv(PencilDev pd, double a, double b, int equilibrate, double* __restrict__ dinv) {
  const int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (r >= (int64_t)pd.n_slices * kSlice) return;
  double v = 1.0;
  if (r < pd.n && equilibrate) {
    const int32_t q = pd.diag_pos[r];
    v = 1.0 / sqrt(fma(a, pd.m64[q], b * pd.k64[q]));
  }
  dinv[r] = v;
}

// Per-block partial sums of <Khat_old, Khat_new>_F and ||Khat_new||_F^2 (both
// scaled by the new diagonal), the numerator and denominator of the update's
// starting scaling alpha (Section 3.2).
__global__ void k_alpha_partial(PencilDev pd, double a, double b, double a_old, double b_old,
                                const double* __restrict__ dinv, double* __restrict__ part) {
  __shared__ double red[2][4];
  const int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  double num = 0, den = 0;
  if (r < pd.n) {
    const int32_t base = pd.slice_ptr[r / kSlice] + (int32_t)(r % kSlice);
    const int len = pd.row_len[r];
    const double sr = dinv[r];
    for (int k = 0; k < len; ++k) {
      const int32_t idx = base + k * kSlice;
      const double sc = sr * dinv[pd.col[idx]];
      const double m = pd.m64[idx], kk = pd.k64[idx];
      const double an = fma(a, m, b * kk) * sc;
      const double ao = fma(a_old, m, b_old * kk) * sc;
      num = fma(ao, an, num);
      den = fma(an, an, den);
    }
  }
  num = wave_total(num);
  den = wave_total(den);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    red[0][w] = num;
    red[1][w] = den;
  }
  __syncthreads();
  if (threadIdx.x < 2) {
    double t = 0;
    for (int i = 0; i < 4; ++i) t += red[threadIdx.x][i];
    part[(int64_t)blockIdx.x * 2 + threadIdx.x] = t;
  }
}

// alpha = num / den from the per-block partials, summed in a fixed order.
// Per-block partial sums of trace(Khat) and ||Khat||_F^2 for Khat = S K(s) S
// (S = diag(dinv)): the numerator and denominator of the build's starting
// scaling alpha = trace(Khat) / trace(Khat Khat^T) (Algorithm 2, first line).
__global__ void k_alpha_build_partial(PencilDev pd, double a, double b,
                                      const double* __restrict__ dinv, double* __restrict__ part) {
  __shared__ double red[2][4];
  const int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  double num = 0, den = 0;
  if (r < pd.n) {
    const int32_t base = pd.slice_ptr[r / kSlice] + (int32_t)(r % kSlice);
    const int len = pd.row_len[r];
    const double sr = dinv[r];
    for (int k = 0; k < len; ++k) {
      const int32_t idx = base + k * kSlice;
      const int c = pd.col[idx];
      const double v = fma(a, pd.m64[idx], b * pd.k64[idx]) * (sr * dinv[c]);
      if (c == (int)r) num += v;
      den = fma(v, v, den);
    }
  }
  num = wave_sum(num);
  den = wave_sum(den);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    red[0][w] = num;
    red[1][w] = den;
  }
  __syncthreads();
  if (threadIdx.x < 2) {
    double t = 0;
    for (int i = 0; i < 4; ++i) t += red[threadIdx.x][i];
    part[(int64_t)blockIdx.x * 2 + threadIdx.x] = t;
  }
}

__device__ __forceinline__ void alpha_final_block(const double* __restrict__ part, int64_t nb,
                                                  double* __restrict__ out) {
  __shared__ double red[2][256];
  const int t = threadIdx.x;
  double num = 0, den = 0;
  for (int64_t i = t; i < nb; i += blockDim.x) {
    num += part[2 * i];
    den += part[2 * i + 1];
  }
  red[0][t] = num;
  red[1][t] = den;
  __syncthreads();
  for (int h = blockDim.x / 2; h > 0; h >>= 1) {
    if (t < h) {
      red[0][t] += red[0][t + h];
      red[1][t] += red[1][t + h];
    }
    __syncthreads();
  }
  if (t == 0) out[0] = red[0][0] / red[1][0];
}

__global__ void k_alpha_final(const double* __restrict__ part, int64_t nb, double* __restrict__ out) {
  alpha_final_block(part, nb, out);
}

// Entries of Khat = S K(s) S on the stored pattern (0 on padding), with
// K(s) = (s^2 + alpha s) M + (1 + beta s) K formed from the float64 pencil.
__global__ void k_scaled_values(PencilDev pd, double a, double b, const double* __restrict__ dinv,
                                double* __restrict__ out) {
  const int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (r >= (int64_t)pd.n_slices * kSlice) return;
  const int64_t s = r / kSlice;
  const int32_t base = pd.slice_ptr[s] + (int32_t)(r % kSlice);
  const int w = (pd.slice_ptr[s + 1] - pd.slice_ptr[s]) / kSlice;
  const int len = pd.row_len[r];
  const double sr = dinv[r];
  for (int k = 0; k < w; ++k) {
    const int32_t idx = base + k * kSlice;
    out[idx] = k < len ? fma(a, pd.m64[idx], b * pd.k64[idx]) * sr * dinv[pd.col[idx]] : 0.0;
  }
}

// Number of lanes of the block with flag set, stored at part[blockIdx.x]
// (one plain store per block; k_sum_counts adds the blocks in order).
__device__ __forceinline__ void block_count(bool flag, int32_t* __restrict__ part) {
  __shared__ int32_t cnt[4];
  const unsigned long long bal = __ballot(flag);
  if ((threadIdx.x & 63) == 0) cnt[threadIdx.x >> 6] = (int32_t)__popcll(bal);
  __syncthreads();
  if (threadIdx.x == 0) {
    int32_t c = 0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) c += cnt[w];
    part[blockIdx.x] = c;
  }
}

// out[0] = sum of the nb per-block counts, in block order.
__device__ __forceinline__ void sum_counts_block(const int32_t* __restrict__ part, int64_t nb,
                                                 int32_t* __restrict__ out) {
  __shared__ int64_t red[256];
  int64_t c = 0;
  for (int64_t i = threadIdx.x; i < nb; i += blockDim.x) c += part[i];
  red[threadIdx.x] = c;
  __syncthreads();
  for (int h = blockDim.x / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = (int32_t)red[0];
}

__global__ void k_sum_counts(const int32_t* __restrict__ part, int64_t nb, int32_t* __restrict__ out) {
  sum_counts_block(part, nb, out);
}

// One lane per column j, on the scaled entries: ahat = Khat (build) or
// Khat_new (update), aold = Khat_old scaled by the new diagonal (update).
// UPDATE selects the update's right-hand side khat_old_j and its skip test;
// otherwise the right-hand side is e_j.  Column j of the solution is stored
// at the positions of row j's entries (hat[pos(j, J_t)] = p_t; the pattern
// is symmetric), so the stores are coalesced; the finalize kernel reads it
// through the transpose map.
template <int MJ, bool UPDATE>
__global__ void __launch_bounds__(256) k_spai_cols(PencilDev pd, const double* __restrict__ ahat,
                                                   const double* __restrict__ aold,
                                                   const double* __restrict__ alpha_u, double tol,
                                                   double* __restrict__ hat,
                                                   double* __restrict__ obj,
                                                   int32_t* __restrict__ skip_count,
                                                   int8_t* __restrict__ skipf) {
  const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  bool skipped = false;
  if (j < pd.n) {
    const int32_t base_j = pd.slice_ptr[j / kSlice] + (int32_t)(j % kSlice);
    const int nj = pd.row_len[j];
    int J[MJ];
    int32_t jpos[MJ];
#pragma unroll
    for (int t = 0; t < MJ; ++t) {
      J[t] = -1;
      jpos[t] = 0;
      if (t < nj) {
        jpos[t] = base_j + t * kSlice;
        J[t] = pd.col[jpos[t]];
      }
    }
    if constexpr (UPDATE) {
      // skip test on column j (= row j: K(s) and S are symmetric)
      const double al = *alpha_u;
      double n_old = 0, n_res = 0;
#pragma unroll
      for (int t = 0; t < MJ; ++t) {
        if (t < nj) {
          const double vo = aold[jpos[t]];
          const double d = fma(-al, ahat[jpos[t]], vo);
          n_old = fma(vo, vo, n_old);
          n_res = fma(d, d, n_res);
        }
      }
      // a skipped column (alpha e_j) is only flagged; the finalize forms it
      if (sqrt(n_res) <= tol * sqrt(n_old)) {
        skipped = true;
        obj[j] = sqrt(n_res);
      }
      skipf[j] = skipped ? 1 : 0;
    }
    if (!skipped) {
      double R[MJ * (MJ + 1) / 2];
      double qtb[MJ];
#pragma unroll
      for (int q = 0; q < MJ * (MJ + 1) / 2; ++q) R[q] = 0.0;
#pragma unroll
      for (int q = 0; q < MJ; ++q) qtb[q] = 0.0;
      double res2 = 0.0;
#pragma unroll
      for (int t = 0; t < MJ; ++t) {
        if (t < nj) {
          const int k = J[t];
          const int32_t base_k = pd.slice_ptr[k / kSlice] + (k % kSlice);
          const int nk = pd.row_len[k];
          for (int e = 0; e < nk; ++e) {
            const int i = pd.col[base_k + e * kSlice];
            // Row i of Khat restricted to the columns J.  Row i is first met
            // through the earliest column of J whose pattern holds it; later
            // meetings are duplicates and are skipped.
            const int32_t base_i = pd.slice_ptr[i / kSlice] + (i % kSlice);
            const int ni = pd.row_len[i];
            double v[MJ];
#pragma unroll
            for (int u = 0; u < MJ; ++u) v[u] = 0.0;
            int umin = MJ;
            double rhs = 0.0;
            for (int q = 0; q < ni; ++q) {
              const int32_t idx = base_i + q * kSlice;
              const int c = pd.col[idx];
              const double val = ahat[idx];
#pragma unroll
              for (int u = 0; u < MJ; ++u) {
                if (u < nj && J[u] == c) {
                  v[u] += val;
                  umin = u < umin ? u : umin;
                }
              }
              if constexpr (UPDATE) {
                if (c == (int)j) rhs = aold[idx];
              }
            }
            if constexpr (!UPDATE) rhs = (i == (int)j) ? 1.0 : 0.0;
            if (umin < t) continue;
            givens_row<MJ>(R, qtb, v, rhs, nj);
            res2 = fma(rhs, rhs, res2);
          }
        }
      }
      double p[MJ];
#pragma unroll
      for (int t = MJ - 1; t >= 0; --t) {
        p[t] = 0.0;
        if (t < nj) {
          double acc = qtb[t];
#pragma unroll
          for (int u = t + 1; u < MJ; ++u)
            if (u < nj) acc = fma(-R[tri<MJ>(t, u)], p[u], acc);
          const double d = R[tri<MJ>(t, t)];
          p[t] = d != 0.0 ? acc / d : 0.0;
        }
      }
#pragma unroll
      for (int t = 0; t < MJ; ++t)
        if (t < nj) hat[jpos[t]] = p[t];
      obj[j] = sqrt(res2);
    }
  }
  if constexpr (UPDATE) block_count(skipped, skip_count);
}

// Pattern control: relative gap below which two candidate entries count as
// equally large (so that rounding near eps never decides the pattern).
constexpr double kPickTie = 1e-8;

// The paper's minimal-residual column loop (Algorithm 2; Algorithm 4 for the
// update), one lane per column j.  As printed, P (Q) stays alpha I inside the
// loop, so the direction is d = alpha r, dropped to the pattern J of column
// j: p_j stays on J and r on the rows I.  The loop then needs only the
// column's local data, gathered once while the rows of I stream past:
//   G = Khat(I,J)^T Khat(I,J),  g = Khat(I,J)^T t,  |t|^2,  Khat(J,J), t(J),
// with t = e_j (build) or khat_old_j (update).  With w = Khat d:
//   (r, w) = g.d - p^T G d,  (w, w) = d^T G d,  a = (r, w) / (w, w),
//   p += a d,  r(J) -= a Khat(J,J) d,  |r|^2 = |t|^2 - 2 g.p + p^T G p.
// It stops once |r| <= tol |t|, when (w, w) is not positive, or after maxit
// steps.  The update's start test is the exact mode's skip test, so a column
// that takes no step is flagged as alpha e_j.
// Pattern control (lfil > 0): d takes alpha r only on the column's current
// pattern, which starts as {j}; while it holds fewer than lfil entries, each
// step first admits the position of J with the largest |alpha r| outside it
// (ratios to the largest within kPickTie of 1 count as ties: the lowest
// column wins; an exact zero is never admitted).
template <int MJ, bool UPDATE, bool CONTIG>
__global__ void __launch_bounds__(256) k_spai_mr(PencilDev pd, const double* __restrict__ ahat,
                                                 const double* __restrict__ aold,
                                                 const double* __restrict__ alpha_d, double tol,
                                                 int maxit, int lfil, double* __restrict__ hat,
                                                 double* __restrict__ obj,
                                                 int32_t* __restrict__ skip_count,
                                                 int8_t* __restrict__ skipf) {
  constexpr int NT = MJ * (MJ + 1) / 2;
  const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  bool skipped = false;
  if (j < pd.n) {
    const int32_t base_j = pd.slice_ptr[j / kSlice] + (int32_t)(j % kSlice);
    const int nj = pd.row_len[j];
    int J[MJ];
    int32_t jpos[MJ];
#pragma unroll
    for (int t = 0; t < MJ; ++t) {
      J[t] = -1;
      jpos[t] = 0;
      if (t < nj) {
        jpos[t] = base_j + t * kSlice;
        J[t] = pd.col[jpos[t]];
      }
    }
    const double al = *alpha_d;
    if constexpr (UPDATE) {
      double n_old = 0, n_res = 0;
#pragma unroll
      for (int t = 0; t < MJ; ++t) {
        if (t < nj) {
          const double vo = aold[jpos[t]];
          const double d = fma(-al, ahat[jpos[t]], vo);
          n_old = fma(vo, vo, n_old);
          n_res = fma(d, d, n_res);
        }
      }
      if (sqrt(n_res) <= tol * sqrt(n_old)) {
        skipped = true;
        obj[j] = sqrt(n_res);
      }
      skipf[j] = skipped ? 1 : 0;
    }
    if (!skipped) {
      double G[NT], KJ[NT], g[MJ], tJ[MJ];
#pragma unroll
      for (int q = 0; q < NT; ++q) G[q] = KJ[q] = 0.0;
#pragma unroll
      for (int q = 0; q < MJ; ++q) g[q] = tJ[q] = 0.0;
      double t2 = 0.0;
      // folds one row (v, rhs) of Khat(I, J) and t(I) into the local data
      auto fold = [&](int i, const double (&v)[MJ], double rhs) {
#pragma unroll
        for (int u = 0; u < MJ; ++u) {
#pragma unroll
          for (int w = u; w < MJ; ++w) G[tri<MJ>(u, w)] = fma(v[u], v[w], G[tri<MJ>(u, w)]);
          g[u] = fma(v[u], rhs, g[u]);
        }
        t2 = fma(rhs, rhs, t2);
#pragma unroll
        for (int w = 0; w < MJ; ++w) {
          if (w < nj && J[w] == i) {
            tJ[w] = rhs;
#pragma unroll
            for (int u = w; u < MJ; ++u) KJ[tri<MJ>(w, u)] = v[u];
          }
        }
      };
      if constexpr (CONTIG) {
        // every row's columns are consecutive: the rows I are the span of
        // the patterns of J, each met once in ascending order, and column
        // J_0 + u of row i sits in its slot J_0 + u - (row i's first column)
        const int J0 = J[0];
        int lo = (int)j, hi = (int)j;
#pragma unroll
        for (int t = 0; t < MJ; ++t) {
          if (t < nj) {
            const int k = J[t];
            const int32_t base_k = pd.slice_ptr[k / kSlice] + (k % kSlice);
            const int first = pd.col[base_k], last = pd.col[base_k + (pd.row_len[k] - 1) * kSlice];
            lo = first < lo ? first : lo;
            hi = last > hi ? last : hi;
          }
        }
        for (int i = lo; i <= hi; ++i) {
          const int32_t base_i = pd.slice_ptr[i / kSlice] + (i % kSlice);
          const int ni = pd.row_len[i];
          const int i0 = pd.col[base_i];
          double v[MJ];
#pragma unroll
          for (int u = 0; u < MJ; ++u) {
            const int q = J0 + u - i0;
            const bool ok = u < nj && q >= 0 && q < ni;
            const double val = ahat[base_i + (ok ? q : 0) * kSlice];
            v[u] = ok ? val : 0.0;
          }
          double rhs;
          if constexpr (UPDATE) {
            const int qj = (int)j - i0;
            const bool okj = qj >= 0 && qj < ni;
            const double vj = aold[base_i + (okj ? qj : 0) * kSlice];
            rhs = okj ? vj : 0.0;
          } else {
            rhs = i == (int)j ? 1.0 : 0.0;
          }
          fold(i, v, rhs);
        }
      } else {
#pragma unroll
      for (int t = 0; t < MJ; ++t) {
        if (t < nj) {
          const int k = J[t];
          const int32_t base_k = pd.slice_ptr[k / kSlice] + (k % kSlice);
          const int nk = pd.row_len[k];
          for (int e = 0; e < nk; ++e) {
            const int i = pd.col[base_k + e * kSlice];
            // row i of Khat restricted to J, met first through the earliest
            // column of J whose pattern holds it (later meetings skipped)
            const int32_t base_i = pd.slice_ptr[i / kSlice] + (i % kSlice);
            const int ni = pd.row_len[i];
            double v[MJ];
#pragma unroll
            for (int u = 0; u < MJ; ++u) v[u] = 0.0;
            int umin = MJ;
            double rhs = 0.0;
            for (int q = 0; q < ni; ++q) {
              const int32_t idx = base_i + q * kSlice;
              const int c = pd.col[idx];
              const double val = ahat[idx];
#pragma unroll
              for (int u = 0; u < MJ; ++u) {
                if (u < nj && J[u] == c) {
                  v[u] += val;
                  umin = u < umin ? u : umin;
                }
              }
              if constexpr (UPDATE) {
                if (c == (int)j) rhs = aold[idx];
              }
            }
            if constexpr (!UPDATE) rhs = (i == (int)j) ? 1.0 : 0.0;
            if (umin < t) continue;
            fold(i, v, rhs);
          }
        }
      }
      }
      // symmetric packed products
      auto symv = [&](const double (&S)[NT], const double (&x)[MJ], double (&y)[MJ]) {
#pragma unroll
        for (int u = 0; u < MJ; ++u) {
          double acc = 0.0;
#pragma unroll
          for (int w = 0; w < MJ; ++w)
            acc = fma(S[u <= w ? tri<MJ>(u, w) : tri<MJ>(w, u)], x[w], acc);
          y[u] = acc;
        }
      };
      auto resid2 = [&](const double (&x)[MJ]) {
        double gx[MJ];
        symv(G, x, gx);
        double s = t2;
#pragma unroll
        for (int u = 0; u < MJ; ++u) s = fma(x[u], fma(-2.0, g[u], gx[u]), s);
        return s;
      };
      double p[MJ], rJ[MJ], d[MJ], y[MJ];
#pragma unroll
      for (int u = 0; u < MJ; ++u) p[u] = (u < nj && J[u] == (int)j) ? al : 0.0;
      symv(KJ, p, y);
#pragma unroll
      for (int u = 0; u < MJ; ++u) rJ[u] = tJ[u] - y[u];
      double r2 = resid2(p);
      const double thr = tol * tol * t2;
      // the column's current pattern (all of J without pattern control)
      bool in[MJ];
      int cnt = 0;
#pragma unroll
      for (int u = 0; u < MJ; ++u) {
        in[u] = u < nj && (lfil <= 0 || J[u] == (int)j);
        cnt += in[u] ? 1 : 0;
      }
      for (int it = 0; it < maxit && r2 > thr; ++it) {
#pragma unroll
        for (int u = 0; u < MJ; ++u) d[u] = u < nj ? al * rJ[u] : 0.0;
        if (lfil > 0 && cnt < lfil) {
          double top = 0.0;
#pragma unroll
          for (int u = 0; u < MJ; ++u)
            if (u < nj && !in[u]) top = fmax(top, fabs(d[u]));
          if (top > 0.0) {
            int pick = -1;
#pragma unroll
            for (int u = MJ - 1; u >= 0; --u)
              if (u < nj && !in[u] && fabs(d[u]) / top >= 1.0 - kPickTie) pick = u;
#pragma unroll
            for (int u = 0; u < MJ; ++u)
              if (u == pick) in[u] = true;
            cnt += pick >= 0 ? 1 : 0;
          }
        }
#pragma unroll
        for (int u = 0; u < MJ; ++u)
          if (!in[u]) d[u] = 0.0;
        symv(G, d, y);
        double rw = 0.0, ww = 0.0;
#pragma unroll
        for (int u = 0; u < MJ; ++u) {
          rw = fma(g[u], d[u], rw);
          rw = fma(-p[u], y[u], rw);
          ww = fma(d[u], y[u], ww);
        }
        if (!(ww > 0.0)) break;
        const double a = rw / ww;
#pragma unroll
        for (int u = 0; u < MJ; ++u) p[u] = fma(a, d[u], p[u]);
        symv(KJ, d, y);
#pragma unroll
        for (int u = 0; u < MJ; ++u) rJ[u] = fma(-a, y[u], rJ[u]);
        r2 = resid2(p);
      }
#pragma unroll
      for (int t = 0; t < MJ; ++t)
        if (t < nj) hat[jpos[t]] = p[t];
      obj[j] = sqrt(r2 > 0.0 ? r2 : 0.0);
    }
  }
  if constexpr (UPDATE) block_count(skipped, skip_count);
}

// Banded pencils (bandwidth bw <= 64): the same least-squares solves, with
// the rows the block's 256 columns can touch (rows j0 - 2 bw .. j0 + 255 +
// 2 bw) staged in LDS first, their scaled entries formed on the fly from the
// float64 pencil.  Every access of the solve then hits LDS instead of a chain
// of dependent global loads.  RANGE = false folds the rows in the same order
// as k_spai_cols (identical results); RANGE = true (narrow bands) folds the
// span of rows once each in ascending order, with no duplicate search.
//   LDS: vn[MJ][S] (Khat or Khat_new), vo[MJ][S] (Khat_old, update only),
//        cl[MJ][S] (column), ln[S] (row length); S = 256 + 4 bw.
template <int MJ>
__host__ __device__ inline size_t spai_band_lds(int bw, bool update) {
  const size_t S = 256 + 4 * (size_t)bw;
  return S * (MJ * (sizeof(double) * (update ? 2 : 1) + sizeof(int32_t)) + sizeof(int32_t));
}

// One column's least-squares solve on the staged rows (vn = Khat or
// Khat_new, vo = Khat_old, cl = columns, ln = lengths, window rows from
// w0, S per entry slot); update: skip test first (al = the update's alpha).
// Returns whether the column was skipped.
template <int MJ, bool UPDATE, int RANGE>
__device__ __forceinline__ bool spai_band_column(const PencilDev& pd, const double* vn,
                                                 const double* vo, const int32_t* cl,
                                                 const int32_t* ln, int S, int64_t w0,
                                                 int64_t j, double al, double tol,
                                                 double* __restrict__ hat,
                                                 double* __restrict__ obj,
                                                 int8_t* __restrict__ skipf) {
  bool skipped = false;
  {
    const int jr = (int)(j - w0);
    const int32_t base_j = pd.slice_ptr[j / kSlice] + (int32_t)(j % kSlice);
    const int nj = ln[jr];
    int J[MJ];
    // -2 past the row: never equal to a staged column (padding holds -1)
#pragma unroll
    for (int u = 0; u < MJ; ++u) J[u] = u < nj ? cl[u * S + jr] : -2;
    if constexpr (UPDATE) {
      double n_old = 0, n_res = 0;
#pragma unroll
      for (int u = 0; u < MJ; ++u) {
        if (u < nj) {
          const double v_o = vo[u * S + jr];
          const double d = fma(-al, vn[u * S + jr], v_o);
          n_old = fma(v_o, v_o, n_old);
          n_res = fma(d, d, n_res);
        }
      }
      // a skipped column (alpha e_j) is only flagged; the finalize forms it
      if (sqrt(n_res) <= tol * sqrt(n_old)) {
        skipped = true;
        obj[j] = sqrt(n_res);
      }
      skipf[j] = skipped ? 1 : 0;
    }
    if (!skipped) {
      double R[MJ * (MJ + 1) / 2];
      double qtb[MJ];
#pragma unroll
      for (int q = 0; q < MJ * (MJ + 1) / 2; ++q) R[q] = 0.0;
#pragma unroll
      for (int q = 0; q < MJ; ++q) qtb[q] = 0.0;
      double res2 = 0.0;
      if constexpr (RANGE != 0) {
        // Narrow band: the rows I lie in [lo, hi], the span of the patterns
        // of the columns J; each row in it is folded once, in ascending
        // order (rows outside I have v = 0 and rhs = 0 and change nothing).
        int lo = (int)j, hi = (int)j;
#pragma unroll
        for (int u = 0; u < MJ; ++u) {
          if (u < nj) {
            const int kr = (int)(J[u] - w0);
            const int first = cl[kr], last = cl[(ln[kr] - 1) * S + kr];
            lo = first < lo ? first : lo;
            hi = last > hi ? last : hi;
          }
        }
        if constexpr (RANGE == 2) {
          // every row's columns are consecutive, and so are the columns J:
          // column J_0 + u of row i sits in its slot J_0 + u - (row i's first
          // column), so each value is one indexed read instead of a match
          // against every slot (the same values, folded in the same order)
          const int J0 = J[0];
          for (int i = lo; i <= hi; ++i) {
            const int ir = (int)(i - w0);
            const int i0 = cl[ir], li = ln[ir];
            double v[MJ];
#pragma unroll
            for (int u = 0; u < MJ; ++u) {
              const int q = J0 + u - i0;
              const bool ok = u < nj && q >= 0 && q < li;
              const double val = vn[(ok ? q : 0) * S + ir];
              v[u] = ok ? val : 0.0;
            }
            double rhs;
            if constexpr (UPDATE) {
              const int qj = (int)j - i0;
              const bool okj = qj >= 0 && qj < li;
              const double vj = vo[(okj ? qj : 0) * S + ir];
              rhs = okj ? vj : 0.0;
            } else {
              rhs = i == (int)j ? 1.0 : 0.0;
            }
            givens_row<MJ>(R, qtb, v, rhs, nj);
            res2 = fma(rhs, rhs, res2);
          }
        } else {
        for (int i = lo; i <= hi; ++i) {
          const int ir = (int)(i - w0);
          double v[MJ];
#pragma unroll
          for (int u = 0; u < MJ; ++u) v[u] = 0.0;
          double rhs = (!UPDATE && i == (int)j) ? 1.0 : 0.0;
#pragma unroll
          for (int q = 0; q < MJ; ++q) {
            const int c = cl[q * S + ir];
            const double val = vn[q * S + ir];
#pragma unroll
            for (int u = 0; u < MJ; ++u) v[u] = J[u] == c ? val : v[u];
            if constexpr (UPDATE) rhs = c == (int)j ? vo[q * S + ir] : rhs;
          }
          givens_row<MJ>(R, qtb, v, rhs, nj);
          res2 = fma(rhs, rhs, res2);
        }
        }
      } else {
#pragma unroll
      for (int tt = 0; tt < MJ; ++tt) {
        if (tt < nj) {
          const int kr = (int)(J[tt] - w0);
          const int nk = ln[kr];
          for (int e = 0; e < nk; ++e) {
            const int i = cl[e * S + kr];
            const int ir = (int)(i - w0);
            const int ni = ln[ir];
            double v[MJ];
#pragma unroll
            for (int u = 0; u < MJ; ++u) v[u] = 0.0;
            int umin = MJ;
            double rhs = 0.0;
            for (int q = 0; q < ni; ++q) {
              const int c = cl[q * S + ir];
              const double val = vn[q * S + ir];
#pragma unroll
              for (int u = 0; u < MJ; ++u) {
                if (u < nj && J[u] == c) {
                  v[u] += val;
                  umin = u < umin ? u : umin;
                }
              }
              if constexpr (UPDATE) {
                if (c == (int)j) rhs = vo[q * S + ir];
              }
            }
            if constexpr (!UPDATE) rhs = (i == (int)j) ? 1.0 : 0.0;
            if (umin < tt) continue;
            givens_row<MJ>(R, qtb, v, rhs, nj);
            res2 = fma(rhs, rhs, res2);
          }
        }
      }
      }
      double p[MJ];
#pragma unroll
      for (int q = MJ - 1; q >= 0; --q) {
        p[q] = 0.0;
        if (q < nj) {
          double acc = qtb[q];
#pragma unroll
          for (int u = q + 1; u < MJ; ++u)
            if (u < nj) acc = fma(-R[tri<MJ>(q, u)], p[u], acc);
          const double d = R[tri<MJ>(q, q)];
          p[q] = d != 0.0 ? acc / d : 0.0;
        }
      }
#pragma unroll
      for (int u = 0; u < MJ; ++u)
        if (u < nj) hat[base_j + u * kSlice] = p[u];
      obj[j] = sqrt(res2);
    }
  }
  return skipped;
}

template <int MJ, bool UPDATE, int RANGE>
__global__ void __launch_bounds__(256) k_spai_band(PencilDev pd, double a, double b, double ao,
                                                   double bo, const double* __restrict__ dinv,
                                                   int bw, const double* __restrict__ alpha_u,
                                                   double tol, double* __restrict__ hat,
                                                   double* __restrict__ obj,
                                                   int32_t* __restrict__ skip_count,
                                                   int8_t* __restrict__ skipf) {
  extern __shared__ double lds[];
  const int S = 256 + 4 * bw;
  double* vn = lds;
  double* vo = vn + MJ * S;
  int32_t* cl = reinterpret_cast<int32_t*>(UPDATE ? vo + MJ * S : vo);
  int32_t* ln = cl + MJ * S;
  const int64_t j0 = (int64_t)blockIdx.x * 256;
  const int64_t w0 = j0 - 2 * bw > 0 ? j0 - 2 * bw : 0;
  const int64_t w1 = j0 + 256 + 2 * bw < pd.n ? j0 + 256 + 2 * bw : pd.n;
  const int t = threadIdx.x;
  // stage rows [w0, w1); every load is issued unconditionally (entries past
  // the slice width read the last one of the row's slice; padding entries
  // hold the row itself as column) and the values past the row length are
  // dropped by a select
  for (int64_t row = w0 + t; row < w1; row += 256) {
    const int r = (int)(row - w0);
    const int64_t sl = row / kSlice;
    const int32_t sp0 = pd.slice_ptr[sl];
    const int32_t base = sp0 + (int32_t)(row % kSlice);
    const int w = (pd.slice_ptr[sl + 1] - sp0) / kSlice;
    const int len = pd.row_len[row];
    const double sr = dinv[row];
    ln[r] = len;
    int32_t c[MJ];
    double m[MJ], kk[MJ], dc[MJ];
#pragma unroll
    for (int k = 0; k < MJ; ++k) {
      const int32_t idx = base + (k < w ? k : w - 1) * kSlice;
      c[k] = pd.col[idx];
      m[k] = pd.m64[idx];
      kk[k] = pd.k64[idx];
    }
#pragma unroll
    for (int k = 0; k < MJ; ++k) dc[k] = dinv[c[k]];
#pragma unroll
    for (int k = 0; k < MJ; ++k) {
      const bool in = k < len;
      // same association as k_scaled_values
      cl[k * S + r] = in ? c[k] : -1;
      vn[k * S + r] = in ? fma(a, m[k], b * kk[k]) * sr * dc[k] : 0.0;
      if constexpr (UPDATE) vo[k * S + r] = in ? fma(ao, m[k], bo * kk[k]) * sr * dc[k] : 0.0;
    }
  }
  __syncthreads();
  const int64_t j = j0 + t;
  bool skipped = false;
  if (j < pd.n)
    skipped = spai_band_column<MJ, UPDATE, RANGE>(pd, vn, vo, cl, ln, S, w0, j,
                                                  UPDATE ? *alpha_u : 0.0, tol, hat, obj, skipf);
  if constexpr (UPDATE) block_count(skipped, skip_count);
}

// ---- batched update: several shifts, the pencil read once ---------------
//
// The update of each factor is exactly the single-factor one (same
// arithmetic in the same order, so the same results); what is shared is
// the reading of M, K and the pattern, and the launches.
constexpr int kManyMax = 16;  // updates per batched launch

struct UpdMany {
  int32_t count;
  double a[kManyMax], b[kManyMax];    // new shift coefficients
  double ao[kManyMax], bo[kManyMax];  // old shift coefficients
  double* alpha[kManyMax];            // each new factor's alpha (device)
  int32_t* skip[kManyMax];            // each new factor's skipped-column count
  double* obj[kManyMax];              // each new factor's objective
  int8_t* skipf[kManyMax];            // each new factor's skipped-column flags
  double* v64[kManyMax];              // each new factor's values (build from K^2)
  float* v32[kManyMax];
};

// dinv of every shift of the batch: [count][n_pad]; the diagonal is read once.
__global__ void k_dinv_many(PencilDev pd, UpdMany U, int equilibrate, int64_t n_pad,
                            double* __restrict__ dinv) {
  const int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (r >= n_pad) return;
  const bool eq = r < pd.n && equilibrate;
  double m = 0, k = 0;
  if (eq) {
    const int32_t q = pd.diag_pos[r];
    m = pd.m64[q];
    k = pd.k64[q];
  }
  for (int s = 0; s < U.count; ++s)
    dinv[(int64_t)s * n_pad + r] = eq ? 1.0 / sqrt(fma(U.a[s], m, U.b[s] * k)) : 1.0;
}

// diag(K(s))_row^{-1/2} for K(s) = a M + b K, as k_dinv forms it (1 without
// equilibration or past the last row).
__device__ __forceinline__ double row_dinv(const PencilDev& pd, double a, double b, int eq,
                                           int64_t row) {
  if (!eq || row >= pd.n) return 1.0;
  const int32_t q = pd.diag_pos[row];
  return 1.0 / sqrt(fma(a, pd.m64[q], b * pd.k64[q]));
}

// The diagonal scalings of rows [d0, d1) for every shift of the batch, in
// LDS: dl[s * W + (row - d0)] = diag(K(s))_row^{-1/2}, formed as k_dinv_many
// forms them (1 without equilibration); each row's diagonal is read once.
// Every thread of the block calls it (it ends with a barrier).
__device__ __forceinline__ void stage_dinv_many(const PencilDev& pd, const UpdMany& U, int eq,
                                                int64_t d0, int64_t d1, int W, double* dl) {
  for (int64_t row = d0 + threadIdx.x; row < d1; row += blockDim.x) {
    double m = 0, k = 0;
    if (eq) {
      const int32_t q = pd.diag_pos[row];
      m = pd.m64[q];
      k = pd.k64[q];
    }
    for (int s = 0; s < U.count; ++s)
      dl[s * W + (int)(row - d0)] = eq ? 1.0 / sqrt(fma(U.a[s], m, U.b[s] * k)) : 1.0;
  }
  __syncthreads();
}

// LDS of stage_dinv_many for a 256-row block of a pencil of bandwidth bw.
inline size_t dinv_many_lds(int count, int bw) {
  return sizeof(double) * (size_t)count * (256 + 2 * (size_t)bw);
}

// Longest row of a pencil whose updates are batched (longer rows take the
// one-by-one path).
constexpr int kManyJ = 6;

// k_alpha_partial for every shift, each row of the pencil read once:
// part[(s * nb + block) * 2 + {0, 1}].  The block's rows and the bw rows on
// either side (the columns of a banded pattern) have their scalings staged
// for every shift first.
__global__ void k_alpha_partial_many(PencilDev pd, UpdMany U, int bw, int eq,
                                     double* __restrict__ part) {
  extern __shared__ double dl[];
  __shared__ double red[kManyMax][2][4];
  const int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int w = threadIdx.x >> 6;
  const int64_t nb = gridDim.x;
  const int64_t j0 = blockIdx.x * (int64_t)blockDim.x;
  const int64_t d0 = j0 - bw > 0 ? j0 - bw : 0;
  const int64_t d1 = j0 + 256 + bw < pd.n ? j0 + 256 + bw : pd.n;
  const int W = 256 + 2 * bw;
  int len = 0;
  int32_t c[kManyJ];
  double m[kManyJ], kk[kManyJ];
  if (r < pd.n) {
    const int32_t base = pd.slice_ptr[r / kSlice] + (int32_t)(r % kSlice);
    len = pd.row_len[r];
#pragma unroll
    for (int k = 0; k < kManyJ; ++k) {
      const int32_t idx = base + (k < len ? k : 0) * kSlice;
      c[k] = pd.col[idx];
      m[k] = pd.m64[idx];
      kk[k] = pd.k64[idx];
    }
  }
  stage_dinv_many(pd, U, eq, d0, d1, W, dl);
  for (int s = 0; s < U.count; ++s) {
    double num = 0, den = 0;
    if (r < pd.n) {
      const double* __restrict__ ds = dl + s * W;
      const double sr = ds[r - d0];
#pragma unroll
      for (int k = 0; k < kManyJ; ++k) {
        if (k < len) {
          const double sc = sr * ds[c[k] - d0];
          const double an = fma(U.a[s], m[k], U.b[s] * kk[k]) * sc;
          const double ao = fma(U.ao[s], m[k], U.bo[s] * kk[k]) * sc;
          num = fma(ao, an, num);
          den = fma(an, an, den);
        }
      }
    }
    num = wave_total(num);
    den = wave_total(den);
    if ((threadIdx.x & 63) == 0) {
      red[s][0][w] = num;
      red[s][1][w] = den;
    }
  }
  __syncthreads();
  if ((int)threadIdx.x < 2 * U.count) {
    const int s = threadIdx.x >> 1, q = threadIdx.x & 1;
    double t = 0;
    for (int i = 0; i < 4; ++i) t += red[s][q][i];
    part[((int64_t)s * nb + blockIdx.x) * 2 + q] = t;
  }
}

__global__ void k_alpha_final_many(UpdMany U, const double* __restrict__ part, int64_t nb) {
  alpha_final_block(part + (int64_t)blockIdx.x * nb * 2, nb, U.alpha[blockIdx.x]);
}

__global__ void k_sum_counts_many(UpdMany U, const int32_t* __restrict__ part, int64_t nb) {
  sum_counts_block(part + (int64_t)blockIdx.x * nb, nb, U.skip[blockIdx.x]);
}

// LDS of k_spai_update_many: M, K, the scaled new and old values (double)
// and the columns per entry slot, plus the row lengths.
template <int MJ>
__host__ __device__ inline size_t spai_many_lds(int bw) {
  const size_t S = 256 + 4 * (size_t)bw;
  return S * (MJ * (4 * sizeof(double) + sizeof(int32_t)) + sizeof(int32_t)) +
         sizeof(double) * (S + 2 * (size_t)bw);
}

// LDS of k_spai_build_many: M, K and the scaled values (double), the
// window's dinv, columns and lengths.
template <int MJ>
__host__ __device__ inline size_t spai_build_many_lds(int bw) {
  const size_t S = 256 + 4 * (size_t)bw;
  return S * (MJ * (3 * sizeof(double) + sizeof(int32_t)) + sizeof(int32_t)) +
         sizeof(double) * (S + 2 * (size_t)bw);
}

// ---------------------------------------------------------------------------
// Batched build from the normal equations (equilibrated builds on pencils
// whose rows are consecutive runs of columns in a narrow band, like the
// beam's; Section 3.1 for every shift of the batch).
//
// Column j's problem min || e_j - Khat(I, J) p || has the normal equations
//     G p = g,  G = Khat(I, J)^T Khat(I, J) = (Khat^2)(J, J),  g = Khat(J, j),
// because the columns J of Khat vanish outside the rows I, and Khat is
// symmetric.  So the Gram matrix of every column is a block of one banded
// matrix, Khat^2, whose entries are formed once per shift and shared by the
// columns around them; a column then needs a 6 x 6 Cholesky and two
// triangular solves instead of a Givens rotation per row of its problem.
// Its residual norm follows from the objective's exact quadratic form,
// ||e_j - B p||^2 = 1 - 2 g^T p + p^T G p, which is off the minimum only to
// second order in the error of p.  Normal equations square the local
// condition number; after equilibration (which this path requires) it is
// below about 250 on every workload here, and a column whose Cholesky
// loses more than 8 digits (a pivot below 1e-8 of its diagonal) is solved
// by Givens rotations over its rows instead.
//
// Every wavefront works alone (no block barriers): it solves 64 consecutive
// columns and writes the final factor, P = S (Phat + Phat^T) / 2 S (or
// S Phat S), of the 64 - 2 bw rows whose averages those columns cover, in
// float64 and float32, with the coefficients kept in its LDS.
constexpr int kGramWave = 64;

// Per-wavefront LDS of k_spai_gram_wave: window rows [o0 - 3 bw, o0 + 64 +
// 2 bw): their scaled values (MJ each, zero past a row's length), the
// diagonal scaling of those rows +- bw and their diagonal entries of M and
// K, the upper band of Khat^2 (2 bw + 1 entries for rows [o0 - 2 bw, o0 +
// 64)), which then holds the columns' coefficients, and per row its length,
// first column, stored position and slice width.
template <int MJ>
__host__ __device__ inline size_t spai_gram_wave_lds(int bw) {
  const size_t wr = kGramWave + 5 * (size_t)bw;
  const size_t band = (kGramWave + 2 * (size_t)bw) * (2 * (size_t)bw + 1);
  const size_t hatw = (size_t)kGramWave * MJ;
  return sizeof(double) *
             (MJ * wr + 3 * (wr + 2 * (size_t)bw) + (band > hatw ? band : hatw)) +
         4 * sizeof(int32_t) * wr;
}

// Column j's normal equations from the band of Khat^2: G = U^T U (Cholesky,
// G(k, i) = band row jb + k, offset i - k), U^T y = g, U p = y, with g(k) =
// Khat(j, J_k) at vn[k * WR + jr], and the residual norm^2 from the
// quadratic form.  FULL: every lane's column has MJ entries (no per-entry
// tests).  Returns false when a pivot falls below 1e-8 of its diagonal (p is
// then not set).
template <int MJ, bool FULL>
__device__ __forceinline__ bool gram_solve(const double* k2, int BW2, int jb, const double* vn,
                                           int WR, int jr, int nj, double (&p)[MJ],
                                           double& res2) {
  double Uf[MJ * (MJ + 1) / 2], iu[MJ], y[MJ], g[MJ];
  bool good = true;
#pragma unroll
  for (int k = 0; k < MJ; ++k) {
    y[k] = 0.0;
    iu[k] = 0.0;
    g[k] = 0.0;
    if (FULL || k < nj) {
      const double* gk = k2 + (jb + k) * BW2;   // Khat^2(J_k, J_k + d)
      g[k] = vn[k * WR + jr];                   // Khat(j, J_k)
      double dkk = gk[0];
#pragma unroll
      for (int m = 0; m < MJ; ++m)
        if (m < k) dkk = fma(-Uf[tri<MJ>(m, k)], Uf[tri<MJ>(m, k)], dkk);
      good = good && dkk > 1e-8 * gk[0];
      // without a branch: the reciprocal root of a stand-in 1 where dkk <= 0
      const double inv0 = rsqrt_newton(dkk > 0.0 ? dkk : 1.0);
      const double inv = dkk > 0.0 ? inv0 : 0.0;
      iu[k] = inv;
      Uf[tri<MJ>(k, k)] = dkk * inv;
#pragma unroll
      for (int i = 0; i < MJ; ++i) {
        if (i > k && (FULL || i < nj)) {
          double gik = gk[i - k];
#pragma unroll
          for (int m = 0; m < MJ; ++m)
            if (m < k) gik = fma(-Uf[tri<MJ>(m, i)], Uf[tri<MJ>(m, k)], gik);
          Uf[tri<MJ>(k, i)] = gik * inv;
        }
      }
      double yk = g[k];
#pragma unroll
      for (int m = 0; m < MJ; ++m)
        if (m < k) yk = fma(-Uf[tri<MJ>(m, k)], y[m], yk);
      y[k] = yk * inv;
    }
  }
  if (!good) return false;
#pragma unroll
  for (int k = MJ - 1; k >= 0; --k) {
    if (FULL || k < nj) {
      double acc = y[k];
#pragma unroll
      for (int i = 0; i < MJ; ++i)
        if (i > k && (FULL || i < nj)) acc = fma(-Uf[tri<MJ>(k, i)], p[i], acc);
      p[k] = acc * iu[k];
    }
  }
  // ||e_j - B p||^2 = 1 - 2 g^T p + p^T G p, G from the band of Khat^2
  double gp = 0.0, pgp = 0.0;
#pragma unroll
  for (int k = 0; k < MJ; ++k) {
    if (FULL || k < nj) {
      const double* gk = k2 + (jb + k) * BW2;
      gp = fma(g[k], p[k], gp);
      double row = gk[0] * p[k];
#pragma unroll
      for (int i = 0; i < MJ; ++i)
        if (i > k && (FULL || i < nj)) row = fma(2.0 * gk[i - k], p[i], row);
      pgp = fma(p[k], row, pgp);
    }
  }
  res2 = fma(-2.0, gp, 1.0) + pgp;
  res2 = res2 > 0.0 ? res2 : 0.0;
  return true;
}

// BWC > 0: the bandwidth as a compile-time constant (the window sizes and
// the band's index arithmetic then fold); 0: bw_rt at run time.
template <int MJ, int BWC>
__global__ void __launch_bounds__(256, 3) k_spai_gram_wave(PencilDev pd, UpdMany U,
                                                        int64_t n_pad, int bw_rt, int sym,
                                                        size_t wave_lds) {
  const int bw = BWC > 0 ? BWC : bw_rt;
  extern __shared__ double lds_all[];
  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  const int out = kGramWave - 2 * bw;             // rows finished per wavefront
  const int WR = kGramWave + 5 * bw;              // window rows
  const int BW2 = 2 * bw + 1;
  const int R2 = kGramWave + 2 * bw;              // rows of the Khat^2 band
  double* vn = reinterpret_cast<double*>(reinterpret_cast<char*>(lds_all) + wv * wave_lds);
  double* dl = vn + MJ * WR;                      // rows [w0 - bw, w0 + WR + bw)
  double* md = dl + WR + 2 * bw;                  // diag(M), diag(K) of those rows
  double* kd = md + WR + 2 * bw;
  double* k2 = kd + WR + 2 * bw;
  const int K2N = R2 * BW2 > kGramWave * MJ ? R2 * BW2 : kGramWave * MJ;
  int32_t* ln = reinterpret_cast<int32_t*>(k2 + K2N);
  int32_t* cf = ln + WR;                          // first column (rows are consecutive runs)
  int32_t* bs = cf + WR;                          // stored position of the first entry
  int32_t* wd = bs + WR;                          // width of the row's slice
  const int64_t n = pd.n;
  const int64_t o0 = ((int64_t)blockIdx.x * 4 + wv) * out;  // first output row
  if (o0 >= n_pad) return;                                  // whole wavefront
  const int64_t c0 = o0 - bw;                               // first solved column
  const int64_t w0 = o0 - 3 * bw;                           // first window row
  const int64_t k0 = o0 - 2 * bw;                           // first Khat^2 row
  for (int r = lane; r < WR; r += 64) {
    const int64_t row = w0 + r;
    const bool in = row >= 0 && row < n;
    const bool stored = row >= 0 && row < n_pad;  // padding rows hold zeros
    const int len = in ? pd.row_len[row] : 0;
    int32_t base = 0, w = 0;
    if (stored) {
      const int32_t sp0 = pd.slice_ptr[row / kSlice];
      base = sp0 + (int32_t)(row % kSlice);
      w = (pd.slice_ptr[row / kSlice + 1] - sp0) / kSlice;
    }
    ln[r] = len;
    bs[r] = base;
    wd[r] = w;
    cf[r] = len > 0 ? pd.col[base] : 0;
  }
  for (int r = lane; r < WR + 2 * bw; r += 64) {
    const int64_t row = w0 - bw + r;
    double m = 0.0, k = 0.0;
    if (row >= 0 && row < n) {
      const int32_t q = pd.diag_pos[row];
      m = pd.m64[q];
      k = pd.k64[q];
    }
    md[r] = m;
    kd[r] = k;
  }
  const int64_t j = c0 + lane;  // this lane's column
  const bool jin = j >= 0 && j < n;
  const int jr = (int)(j - w0);
  // up to 2 bw + 1 band offsets, unrolled (bw <= 7 at run time)
  constexpr int DMAX = BWC > 0 ? 2 * BWC + 1 : 15;
  for (int s = 0; s < U.count; ++s) {
    const double sa = U.a[s], sb = U.b[s];
    __builtin_amdgcn_wave_barrier();
    // the diagonal scaling diag(K(s))^{-1/2} of the rows (equilibrated
    // builds only), 0 outside the matrix
    for (int r = lane; r < WR + 2 * bw; r += 64) {
      const int64_t row = w0 - bw + r;
      dl[r] = (row >= 0 && row < n) ? 1.0 / sqrt(fma(sa, md[r], sb * kd[r])) : 0.0;
    }
    __builtin_amdgcn_wave_barrier();
    // scaled values Khat(r, c) = S_r K(s)_rc S_c of the window rows: rows
    // 0..63 one per lane (no per-entry tests where every row is full), the
    // last 5 bw rows one (row, entry) pair per lane
    {
      const int r = lane;
      const int len = ln[r];
      const int32_t base = bs[r];
      const int cw = cf[r] - (int)w0 + bw;  // scaling index of the first column
      const double sr = dl[r + bw];
      if (__all(len == MJ)) {
#pragma unroll
        for (int k = 0; k < MJ; ++k) {
          const int32_t idx = base + k * kSlice;
          vn[k * WR + r] = fma(sa, pd.m64[idx], sb * pd.k64[idx]) * sr * dl[cw + k];
        }
      } else {
#pragma unroll
        for (int k = 0; k < MJ; ++k) {
          double v = 0.0;
          if (k < len) {
            const int32_t idx = base + k * kSlice;
            v = fma(sa, pd.m64[idx], sb * pd.k64[idx]) * sr * dl[cw + k];
          }
          vn[k * WR + r] = v;
        }
      }
    }
    for (int e = lane; e < (WR - 64) * MJ; e += 64) {
      const int r = 64 + e / MJ, k = e - (r - 64) * MJ;
      double v = 0.0;
      if (k < ln[r]) {
        const int32_t idx = bs[r] + k * kSlice;
        v = fma(sa, pd.m64[idx], sb * pd.k64[idx]) * dl[r + bw] * dl[cf[r] - (int)w0 + bw + k];
      }
      vn[k * WR + r] = v;
    }
    __builtin_amdgcn_wave_barrier();
    // upper band of Khat^2: Khat^2(i, i + d) = sum over k of Khat(i, k)
    // Khat(i + d, k) (entries past a row's length are zero, so every product
    // of the overlap is taken).  Rows 0..63 of the band one per lane, the
    // values of row i kept in registers for its 2 bw + 1 offsets:
    {
      const int q = lane;
      const int ir = bw + q;  // window index of row k0 + q
      const int ci = cf[ir];
      double vi[MJ];
#pragma unroll
      for (int u = 0; u < MJ; ++u) vi[u] = vn[u * WR + ir];
#pragma unroll
      for (int d = 0; d < DMAX; ++d) {
        if (d < BW2) {
          const int cr = ir + d;
          const int dc = cf[cr] - ci;
          double acc = 0.0;
#pragma unroll
          for (int u = 0; u < MJ; ++u) {
            const int qq = u - dc;
            const bool ok = qq >= 0 && qq < MJ;
            const double xv = vn[(ok ? qq : 0) * WR + cr];
            acc = fma(vi[u], ok ? xv : 0.0, acc);
          }
          k2[q * BW2 + d] = acc;
        }
      }
    }
    __builtin_amdgcn_sched_barrier(0);
    // the last 2 bw rows: one (row, offset) pair per lane
    for (int e = lane; e < (R2 - 64) * BW2; e += 64) {
      const int q = 64 + e / BW2, d = e - (q - 64) * BW2;
      const int ir = bw + q;
      const int cr = ir + d;
      const int dc = cf[cr] - cf[ir];
      double acc = 0.0;
#pragma unroll
      for (int u = 0; u < MJ; ++u) {
        const int qq = u - dc;
        const bool ok = qq >= 0 && qq < MJ;
        const double xv = vn[(ok ? qq : 0) * WR + cr];
        acc = fma(vn[u * WR + ir], ok ? xv : 0.0, acc);
      }
      k2[q * BW2 + d] = acc;
    }
    __builtin_amdgcn_wave_barrier();
    // column j: Cholesky G = U^T U of G = Khat^2(J, J), g = Khat(J, j)
    double p[MJ];
#pragma unroll
    for (int u = 0; u < MJ; ++u) p[u] = 0.0;
    double res2 = 0.0;
    const int nj = jin ? ln[jr] : 0;
    const int J0 = nj > 0 ? cf[jr] : 0;  // J = J0, J0 + 1, ..., J0 + nj - 1
    const int jb = J0 - (int)k0;
    bool good = true;
    if (__all(nj == MJ)) {
      good = gram_solve<MJ, true>(k2, BW2, jb, vn, WR, jr, nj, p, res2);
    } else if (nj > 0) {
      good = gram_solve<MJ, false>(k2, BW2, jb, vn, WR, jr, nj, p, res2);
    }
    if (nj > 0 && !good) {
      // Givens rotations over the rows I (the span of the patterns of J)
      res2 = 0.0;
      int lo = (int)j, hi = (int)j;
#pragma unroll
      for (int u = 0; u < MJ; ++u) {
        if (u < nj) {
          const int kr = J0 + u - (int)w0;
          const int first = cf[kr], last = cf[kr] + ln[kr] - 1;
          lo = first < lo ? first : lo;
          hi = last > hi ? last : hi;
        }
      }
      double R[MJ * (MJ + 1) / 2];
      double qtb[MJ];
#pragma unroll
      for (int q = 0; q < MJ * (MJ + 1) / 2; ++q) R[q] = 0.0;
#pragma unroll
      for (int q = 0; q < MJ; ++q) qtb[q] = 0.0;
      for (int i = lo; i <= hi; ++i) {
        const int ir = (int)(i - w0);
        const int i0 = cf[ir], li = ln[ir];
        double v[MJ];
#pragma unroll
        for (int u = 0; u < MJ; ++u) {
          const int q = J0 + u - i0;
          const bool ok = u < nj && q >= 0 && q < li;
          const double val = vn[(ok ? q : 0) * WR + ir];
          v[u] = ok ? val : 0.0;
        }
        double rhs = i == (int)j ? 1.0 : 0.0;
        givens_row<MJ>(R, qtb, v, rhs, nj);
        res2 = fma(rhs, rhs, res2);
      }
#pragma unroll
      for (int q = MJ - 1; q >= 0; --q) {
        if (q < nj) {
          double acc = qtb[q];
#pragma unroll
          for (int u = q + 1; u < MJ; ++u)
            if (u < nj) acc = fma(-R[tri<MJ>(q, u)], p[u], acc);
          const double d = R[tri<MJ>(q, q)];
          p[q] = d != 0.0 ? acc / d : 0.0;
        }
      }
    }
    // streaming stores for the objective and the factors (written once, read
    // by later kernels), so they do not push the window rows' M and K values,
    // re-read for every shift, out of the cache
    if (nj > 0 && lane >= bw && lane < bw + out) __builtin_nontemporal_store(sqrt(res2), &U.obj[s][j]);
    __builtin_amdgcn_wave_barrier();  // every lane has read the band
    // coefficient u of column c0 + lane (row J0 + u of Phat)
#pragma unroll
    for (int u = 0; u < MJ; ++u) k2[lane * MJ + u] = p[u];
    __builtin_amdgcn_wave_barrier();
    // the final factor for rows [o0, o0 + out): P(r, c) = S_r Pbar(r, c) S_c
    const int64_t r = o0 + (lane - bw);
    const bool wr_row = lane >= bw && lane < bw + out && r < n_pad;
    const int rw = lane + 2 * bw;  // window index of row r
    const bool fullrow = r < n && wd[rw] == MJ && ln[rw] == MJ;
    if (__all(fullrow || !wr_row)) {
      // every written row is full: no per-entry tests
      if (wr_row) {
        const int32_t base = bs[rw];
        const double sr = dl[rw + bw];
        const int r0 = cf[rw];
        double* __restrict__ o64 = U.v64[s];
        float* __restrict__ o32 = U.v32[s];
#pragma unroll
        for (int k = 0; k < MJ; ++k) {
          const int c = r0 + k;
          const int cr = (int)(c - w0);
          const int cfc = cf[cr];
          double h = k2[(int)(c - c0) * MJ + (int)(r - cfc)];  // column c at row r
          if (sym) h = 0.5 * (h + k2[lane * MJ + k]);          // column r at row c
          const double val = h * sr * dl[cr + bw];
          const int32_t idx = base + k * kSlice;
          __builtin_nontemporal_store(val, &o64[idx]);
          __builtin_nontemporal_store((float)val, &o32[idx]);
        }
      }
    } else if (wr_row) {
      const int rr = (int)(r - w0);
      const int32_t base = bs[rr];
      const int w = wd[rr];
      const int len = r < n ? ln[rr] : 0;
      const double sr = r < n ? dl[rr + bw] : 0.0;
      const int r0 = len > 0 ? cf[rr] : 0;
      double* __restrict__ o64 = U.v64[s];
      float* __restrict__ o32 = U.v32[s];
      for (int k = 0; k < w; ++k) {
        double val = 0.0;
        if (k < len) {
          const int c = r0 + k;
          const int cr = (int)(c - w0);
          const int cfc = cf[cr];
          double h = k2[(int)(c - c0) * MJ + (int)(r - cfc)];  // column c at row r
          if (sym) h = 0.5 * (h + k2[lane * MJ + k]);          // column r at row c
          val = h * sr * dl[cr + bw];
        }
        const int32_t idx = base + k * kSlice;
        __builtin_nontemporal_store(val, &o64[idx]);
        __builtin_nontemporal_store((float)val, &o32[idx]);
      }
    }
  }
}

// The banded build column kernel for every shift of the batch (Section 3.1
// for each shift): the block's rows are staged once (M, K, columns), then per
// shift the window's diagonal scaling is staged, the scaled values formed as
// k_spai_band forms them and the columns solved.  hat: [count][stored].
template <int MJ, int RANGE>
__global__ void __launch_bounds__(256) k_spai_build_many(PencilDev pd, UpdMany U,
                                                         const double* __restrict__ dinv,
                                                         int64_t n_pad, int64_t stored, int bw,
                                                         double* __restrict__ hat) {
  extern __shared__ double lds[];
  const int S = 256 + 4 * bw;
  double* mm = lds;
  double* kq = mm + MJ * S;
  double* vn = kq + MJ * S;
  double* dl = vn + MJ * S;  // dinv of rows [d0, d1): the window and bw beyond
  int32_t* cl = reinterpret_cast<int32_t*>(dl + S + 2 * bw);
  int32_t* ln = cl + MJ * S;
  const int64_t j0 = (int64_t)blockIdx.x * 256;
  const int64_t w0 = j0 - 2 * bw > 0 ? j0 - 2 * bw : 0;
  const int64_t w1 = j0 + 256 + 2 * bw < pd.n ? j0 + 256 + 2 * bw : pd.n;
  const int64_t d0 = w0 - bw > 0 ? w0 - bw : 0;
  const int64_t d1 = w1 + bw < pd.n ? w1 + bw : pd.n;
  const int t = threadIdx.x;
  for (int64_t row = w0 + t; row < w1; row += 256) {
    const int r = (int)(row - w0);
    const int64_t sl = row / kSlice;
    const int32_t sp0 = pd.slice_ptr[sl];
    const int32_t base = sp0 + (int32_t)(row % kSlice);
    const int w = (pd.slice_ptr[sl + 1] - sp0) / kSlice;
    const int len = pd.row_len[row];
    ln[r] = len;
#pragma unroll
    for (int k = 0; k < MJ; ++k) {
      const int32_t idx = base + (k < w ? k : w - 1) * kSlice;
      const bool in = k < len;
      const int32_t c = pd.col[idx];
      cl[k * S + r] = in ? c : -1;
      mm[k * S + r] = pd.m64[idx];
      kq[k * S + r] = pd.k64[idx];
    }
  }
  const int64_t j = j0 + t;
  for (int s = 0; s < U.count; ++s) {
    const double* __restrict__ dv = dinv + (int64_t)s * n_pad;
    __syncthreads();  // staged rows ready; the previous shift's columns done
    for (int64_t row = d0 + t; row < d1; row += 256) dl[row - d0] = dv[row];
    __syncthreads();
    for (int64_t row = w0 + t; row < w1; row += 256) {
      const int r = (int)(row - w0);
      const double sr = dl[row - d0];
      const int len = ln[r];
#pragma unroll
      for (int k = 0; k < MJ; ++k) {
        const bool in = k < len;
        const int32_t c = cl[k * S + r];
        const double dc = dl[(in ? c : row) - d0];
        // same association as k_scaled_values
        vn[k * S + r] = in ? fma(U.a[s], mm[k * S + r], U.b[s] * kq[k * S + r]) * sr * dc : 0.0;
      }
    }
    __syncthreads();
    if (j < pd.n)
      spai_band_column<MJ, false, RANGE>(pd, vn, nullptr, cl, ln, S, w0, j, 0.0, 0.0,
                                         hat + (int64_t)s * stored, U.obj[s], nullptr);
  }
}

// The update's skip test for every column and shift of the batch, straight
// from the pencil (one lane per column j, whose pattern is that of row j):
// the same scaled values, in the same association, as the staged test of
// k_spai_update_many below, so the flags agree bit for bit.  Writes the
// flags, the objective of skipped columns, and per (shift, block of 256
// columns) the skipped count and whether any column needs its solve, so the
// staged kernel only visits blocks and shifts with work left.
template <int MJ>
__global__ void __launch_bounds__(256) k_update_test_many(PencilDev pd, UpdMany U, int bw, int eq,
                                                         double tol,
                                                         int32_t* __restrict__ skip_part,
                                                         int32_t* __restrict__ need) {
  extern __shared__ double dl[];
  __shared__ int32_t cnt[kManyMax][4], req[kManyMax][4];
  __shared__ double als[kManyMax];
  const int64_t j0 = (int64_t)blockIdx.x * 256;
  const int64_t j = j0 + threadIdx.x;
  const int wv = threadIdx.x >> 6;
  const bool in = j < pd.n;
  const int64_t d0 = j0 - bw > 0 ? j0 - bw : 0;
  const int64_t d1 = j0 + 256 + bw < pd.n ? j0 + 256 + bw : pd.n;
  const int W = 256 + 2 * bw;
  int len = 0;
  int32_t col[MJ];
  double mm[MJ], kq[MJ];
  if (in) {
    const int32_t base = pd.slice_ptr[j / kSlice] + (int32_t)(j % kSlice);
    len = pd.row_len[j];
#pragma unroll
    for (int u = 0; u < MJ; ++u) {
      col[u] = (int32_t)j;
      mm[u] = kq[u] = 0.0;
      if (u < len) {
        const int32_t idx = base + u * kSlice;
        col[u] = pd.col[idx];
        mm[u] = pd.m64[idx];
        kq[u] = pd.k64[idx];
      }
    }
  }
  // every shift's alpha, loaded once per block (the staging ends with a barrier)
  if ((int)threadIdx.x < U.count) als[threadIdx.x] = *U.alpha[threadIdx.x];
  stage_dinv_many(pd, U, eq, d0, d1, W, dl);
  for (int s = 0; s < U.count; ++s) {
    bool skipped = false, solve = false;
    if (in) {
      const double al = als[s];
      const double* __restrict__ ds = dl + s * W;
      const double sr = ds[j - d0];
      double n_old = 0, n_res = 0;
#pragma unroll
      for (int u = 0; u < MJ; ++u) {
        if (u < len) {
          const double dc = ds[col[u] - d0];
          const double v_n = fma(U.a[s], mm[u], U.b[s] * kq[u]) * sr * dc;
          const double v_o = fma(U.ao[s], mm[u], U.bo[s] * kq[u]) * sr * dc;
          const double d = fma(-al, v_n, v_o);
          n_old = fma(v_o, v_o, n_old);
          n_res = fma(d, d, n_res);
        }
      }
      if (sqrt(n_res) <= tol * sqrt(n_old)) {
        skipped = true;
        U.obj[s][j] = sqrt(n_res);
      } else {
        solve = true;
      }
      U.skipf[s][j] = skipped ? 1 : 0;
    }
    const unsigned long long bs = __ballot(skipped), bn = __ballot(solve);
    if ((threadIdx.x & 63) == 0) {
      cnt[s][wv] = (int32_t)__popcll(bs);
      req[s][wv] = bn != 0ull ? 1 : 0;
    }
  }
  __syncthreads();
  const int64_t nb = gridDim.x;
  if ((int)threadIdx.x < U.count) {
    const int s = threadIdx.x;
    int32_t c = 0, r = 0;
    for (int w = 0; w < 4; ++w) {
      c += cnt[s][w];
      r |= req[s][w];
    }
    skip_part[(int64_t)s * nb + blockIdx.x] = c;
    need[(int64_t)s * nb + blockIdx.x] = r;
  }
}

// The banded update column kernel for every shift of the batch: the block's
// rows are staged once (M, K, columns), then per shift their scaled values
// are formed and the columns solved as in k_spai_band.  hat: [count][stored].
// need (NULL: every block and shift): per (shift, block) whether any column
// failed the skip test of k_update_test_many, which has already written the
// flags, objectives and skipped counts; a block with nothing to solve for
// any shift returns before staging, and a shift with nothing to solve is
// passed over.
template <int MJ, int RANGE>
__global__ void __launch_bounds__(256) k_spai_update_many(PencilDev pd, UpdMany U, int eq,
                                                          int64_t stored, int bw,
                                                          double tol, double* __restrict__ hat,
                                                          int32_t* __restrict__ skip_part,
                                                          const int32_t* __restrict__ need) {
  if (need) {
    // one flag per thread, all loads in flight together
    const int t = threadIdx.x;
    const int mine = t < U.count ? need[(int64_t)t * gridDim.x + blockIdx.x] : 0;
    if (!__syncthreads_or(mine != 0)) return;  // the whole block
  }
  extern __shared__ double lds[];
  const int S = 256 + 4 * bw;
  double* mm = lds;
  double* kq = mm + MJ * S;
  double* vn = kq + MJ * S;
  double* vo = vn + MJ * S;
  double* dl = vo + MJ * S;  // dinv of rows [d0, d1): the window and bw beyond
  int32_t* cl = reinterpret_cast<int32_t*>(dl + S + 2 * bw);
  int32_t* ln = cl + MJ * S;
  const int64_t j0 = (int64_t)blockIdx.x * 256;
  const int64_t w0 = j0 - 2 * bw > 0 ? j0 - 2 * bw : 0;
  const int64_t w1 = j0 + 256 + 2 * bw < pd.n ? j0 + 256 + 2 * bw : pd.n;
  const int64_t d0 = w0 - bw > 0 ? w0 - bw : 0;
  const int64_t d1 = w1 + bw < pd.n ? w1 + bw : pd.n;
  const int t = threadIdx.x;
  for (int64_t row = w0 + t; row < w1; row += 256) {
    const int r = (int)(row - w0);
    const int64_t sl = row / kSlice;
    const int32_t sp0 = pd.slice_ptr[sl];
    const int32_t base = sp0 + (int32_t)(row % kSlice);
    const int w = (pd.slice_ptr[sl + 1] - sp0) / kSlice;
    const int len = pd.row_len[row];
    ln[r] = len;
#pragma unroll
    for (int k = 0; k < MJ; ++k) {
      const int32_t idx = base + (k < w ? k : w - 1) * kSlice;
      const bool in = k < len;
      const int32_t c = pd.col[idx];
      cl[k * S + r] = in ? c : -1;
      mm[k * S + r] = pd.m64[idx];
      kq[k * S + r] = pd.k64[idx];
    }
  }
  const int64_t nb = gridDim.x;
  for (int s = 0; s < U.count; ++s) {
    // the same for every thread of the block
    if (need && need[(int64_t)s * nb + blockIdx.x] == 0) continue;
    double* __restrict__ hs = hat + (int64_t)s * stored;
    __syncthreads();  // staged rows ready; the previous shift's columns done
    for (int64_t row = d0 + t; row < d1; row += 256) dl[row - d0] = row_dinv(pd, U.a[s], U.b[s], eq, row);
    __syncthreads();
    // skip test of column j straight from the staged rows (the scaled
    // values below and in spai_band_column are formed the same way)
    const int64_t j = j0 + t;
    const double al = *U.alpha[s];
    bool skipped = false, solve = false;
    if (j < pd.n) {
      const int jr = (int)(j - w0);
      const int nj = ln[jr];
      const double sr = dl[j - d0];
      double n_old = 0, n_res = 0;
#pragma unroll
      for (int u = 0; u < MJ; ++u) {
        if (u < nj) {
          const int32_t c = cl[u * S + jr];
          const double dc = dl[c - d0];
          const double v_n = fma(U.a[s], mm[u * S + jr], U.b[s] * kq[u * S + jr]) * sr * dc;
          const double v_o = fma(U.ao[s], mm[u * S + jr], U.bo[s] * kq[u * S + jr]) * sr * dc;
          const double d = fma(-al, v_n, v_o);
          n_old = fma(v_o, v_o, n_old);
          n_res = fma(d, d, n_res);
        }
      }
      if (sqrt(n_res) <= tol * sqrt(n_old)) {
        skipped = true;
        U.obj[s][j] = sqrt(n_res);
        U.skipf[s][j] = 1;
      } else {
        solve = true;
      }
    }
    // scaled values of the window only when some column needs its solve
    if (__syncthreads_or(solve)) {
      for (int64_t row = w0 + t; row < w1; row += 256) {
        const int r = (int)(row - w0);
        const double sr = dl[row - d0];
        const int len = ln[r];
#pragma unroll
        for (int k = 0; k < MJ; ++k) {
          const bool in = k < len;
          const int32_t c = cl[k * S + r];
          const double dc = dl[(in ? c : row) - d0];
          // same association as k_scaled_values
          vn[k * S + r] = in ? fma(U.a[s], mm[k * S + r], U.b[s] * kq[k * S + r]) * sr * dc : 0.0;
          vo[k * S + r] = in ? fma(U.ao[s], mm[k * S + r], U.bo[s] * kq[k * S + r]) * sr * dc : 0.0;
        }
      }
      __syncthreads();
      if (solve)
        spai_band_column<MJ, true, RANGE>(pd, vn, vo, cl, ln, S, w0, j, al, tol, hs, U.obj[s],
                                          U.skipf[s]);
    }
    block_count(skipped, skip_part + (int64_t)s * nb);
  }
}

// flags[j] = 1 where the update kept column j at alpha e_j (src NULL: a
// build, no column skipped).
__global__ void k_copy_flags(const int8_t* __restrict__ src, int32_t n, uint8_t* __restrict__ flags) {
  const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (j < n) flags[j] = (src && src[j]) ? 1 : 0;
}

// Map the scaled factor back and store float64 and float32 copies:
//   build:        P = S Phat S          (mode 0)
//   build, sym:   P = S (Phat + Phat^T)/2 S   (mode 1)
//   update:       Q = S Qhat S^{-1}     (mode 2)
// Padding entries are 0.  An update whose every column was skipped
// (skip_total = n) is the scalar alpha I: it is never applied as a factor,
// so nothing is written.
// dinv(i): the diagonal scaling of row i.
template <class Dinv>
__device__ __forceinline__ void finalize_row(const PencilDev& pd, int64_t r,
                                             const double* __restrict__ hat, Dinv dinv, int mode,
                                             const int32_t* __restrict__ skip_total,
                                             const int8_t* __restrict__ skipf,
                                             const double* __restrict__ alpha,
                                             double* __restrict__ v64, float* __restrict__ v32) {
  if (r >= (int64_t)pd.n_slices * kSlice) return;
  if (skip_total && *skip_total == pd.n) return;
  const int64_t s = r / kSlice;
  const int32_t base = pd.slice_ptr[s] + (int32_t)(r % kSlice);
  const int w = (pd.slice_ptr[s + 1] - pd.slice_ptr[s]) / kSlice;
  const int len = pd.row_len[r];
  const double sr = dinv(r);
  for (int k = 0; k < w; ++k) {
    const int32_t idx = base + k * kSlice;
    double val = 0.0;
    if (k < len) {
      const int c = pd.col[idx];
      // hat holds column c's solution at the position of (c, r); a skipped
      // column c (update) is alpha e_c
      double h = (skipf && skipf[c]) ? (c == (int)r ? *alpha : 0.0) : hat[pd.mirror[idx]];
      if (mode == 1) h = 0.5 * (h + hat[idx]);
      val = mode == 2 ? h * sr / dinv(c) : h * sr * dinv(c);
    }
    v64[idx] = val;
    v32[idx] = (float)val;
  }
}

__global__ void k_spai_finalize(PencilDev pd, const double* __restrict__ hat,
                                const double* __restrict__ dinv, int mode,
                                const int32_t* __restrict__ skip_total,
                                const int8_t* __restrict__ skipf, const double* __restrict__ alpha,
                                double* __restrict__ v64, float* __restrict__ v32) {
  finalize_row(pd, blockIdx.x * (int64_t)blockDim.x + threadIdx.x, hat,
               [=](int64_t i) { return dinv[i]; }, mode, skip_total, skipf, alpha, v64, v32);
}

// k_spai_finalize of the updates of a batch, one grid row (blockIdx.y) per
// update: hat [count][stored]; the scalings are formed from the diagonal.
// A grid-stride loop over the rows, so an update whose every column was
// skipped costs few blocks.
__global__ void k_update_finalize_many(PencilDev pd, UpdMany U, const double* __restrict__ hat,
                                       int eq, int64_t stored) {
  const int s = blockIdx.y;
  if (*U.skip[s] == pd.n) return;  // the scalar alpha I: nothing written
  const double a = U.a[s], b = U.b[s];
  const int64_t rows = (int64_t)pd.n_slices * kSlice;
  for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < rows;
       r += (int64_t)gridDim.x * blockDim.x)
    finalize_row(pd, r, hat + (int64_t)s * stored,
                 [&](int64_t i) { return row_dinv(pd, a, b, eq, i); }, 2, U.skip[s], U.skipf[s],
                 U.alpha[s], U.v64[s], U.v32[s]);
}

// out[e] (CSR order) = values[stored idx]
__global__ void k_export(PencilDev pd, int64_t stored, const double* __restrict__ v,
                         double* __restrict__ out) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= stored) return;
  const int32_t e = pd.csr_pos[i];
  if (e >= 0) out[e] = v[i];
}

// The scalar factor alpha I in CSR order: alpha on the diagonal, 0 elsewhere.
__global__ void k_export_scalar(PencilDev pd, double alpha, double* __restrict__ out) {
  const int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (r >= pd.n) return;
  const int64_t s = r / kSlice;
  const int32_t base = pd.slice_ptr[s] + (int32_t)(r % kSlice);
  const int len = pd.row_len[r];
  for (int k = 0; k < len; ++k) {
    const int32_t idx = base + k * kSlice;
    out[pd.csr_pos[idx]] = pd.col[idx] == (int32_t)r ? alpha : 0.0;
  }
}

// y = scale * V x with V on the pattern (stored order), float64; blockIdx.y = vector.
__global__ void k_factor_apply(PencilDev pd, const double* __restrict__ vals, double scale,
                               const double* __restrict__ x, int64_t ldx, double* __restrict__ y,
                               int64_t ldy) {
  const int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (r >= pd.n) return;
  const double* xv = x + (int64_t)blockIdx.y * ldx;
  const int64_t s = r / kSlice;
  const int32_t base = pd.slice_ptr[s] + (int32_t)(r % kSlice);
  const int w = (pd.slice_ptr[s + 1] - pd.slice_ptr[s]) / kSlice;
  double acc = 0;
  if (vals) {
    for (int k = 0; k < w; ++k) {
      const int32_t idx = base + k * kSlice;
      acc = fma(vals[idx], xv[pd.col[idx]], acc);
    }
  } else {
    acc = xv[r];
  }
  y[(int64_t)blockIdx.y * ldy + r] = scale * acc;
}

// ------------------------------------------------------------------- host

airga_status pool_get(airga_ctx ctx, DevBuf* buf, size_t need) {
  // smallest pooled buffer that fits
  size_t best = ctx->pool.size();
  for (size_t i = 0; i < ctx->pool.size(); ++i)
    if (ctx->pool[i].second >= need &&
        (best == ctx->pool.size() || ctx->pool[i].second < ctx->pool[best].second))
      best = i;
  if (best < ctx->pool.size()) {
    buf->adopt(ctx->pool[best].first, ctx->pool[best].second);
    ctx->pool.erase(ctx->pool.begin() + (long)best);
    return AIRGA_OK;
  }
  return buf->reserve(need);
}

void pool_put(airga_ctx ctx, DevBuf* buf) {
  void* p;
  size_t b;
  buf->detach(&p, &b);
  if (p) ctx->pool.emplace_back(p, b);
}

// Device scalars of a factor: alpha (8 bytes), the skip count (4), padding to
// 64, then one byte per column, set when the update kept alpha e_j there.
static int8_t* skip_flags(airga_prec p) { return p->scal.as<int8_t>() + 64; }

static airga_status new_prec(airga_ctx ctx, double s, airga_prec* out) {
  airga_prec p = new (std::nothrow) airga_prec_s();
  if (!p) return fail(AIRGA_ENOMEM, "host allocation failed");
  p->ctx = ctx;
  p->generation = ctx->pen.generation;
  p->shift = s;
  const Pencil& pen = ctx->pen;
  airga_status st;
  if ((st = pool_get(ctx, &p->v64, sizeof(double) * pen.nnz_stored)) != AIRGA_OK ||
      (st = pool_get(ctx, &p->v32, sizeof(float) * pen.nnz_stored)) != AIRGA_OK ||
      (st = pool_get(ctx, &p->objective, sizeof(double) * pen.n)) != AIRGA_OK ||
      (st = pool_get(ctx, &p->scal, 64 + (size_t)pen.n_pad())) != AIRGA_OK) {
    pool_put(ctx, &p->v64);
    pool_put(ctx, &p->v32);
    pool_put(ctx, &p->objective);
    pool_put(ctx, &p->scal);
    delete p;
    return st;
  }
  ctx->live_precs++;
  *out = p;
  return AIRGA_OK;
}

static airga_status check_spai_args(airga_ctx ctx, double s, airga_prec* out) {
  AIRGA_TRY(check_pencil(ctx));
  if (!out) return fail(AIRGA_EINVAL, "null output handle");
  if (!std::isfinite(s) || !(s > 0)) return fail(AIRGA_EINVAL, "shift must be finite and > 0");
  if (!ctx->pen.diag_ok)
    return fail(AIRGA_ENOTSPD, "a diagonal entry of M is <= 0 or of K is < 0: K(s) may not be SPD");
  if (ctx->pen.max_len > kSpaiMaxJ)
    return fail(AIRGA_EUNSUPPORTED, "SPAI needs rows of at most %d entries (longest row: %d)",
                kSpaiMaxJ, ctx->pen.max_len);
  return AIRGA_OK;
}

// Scratch for one SPAI call: [dinv (n_pad) | hat | ahat | aold (stored each) |
// alpha partials (2 nb) | per-block skip counts (nb int32)].
struct SpaiScratch {
  double *dinv, *hat, *ahat, *aold, *part;
  int32_t* skip_part;
};
static airga_status spai_scratch(airga_ctx ctx, SpaiScratch* w, int64_t nb) {
  const Pencil& pen = ctx->pen;
  const size_t need = sizeof(double) * ((size_t)pen.n_pad() + 3 * (size_t)pen.nnz_stored +
                                        2 * nb + (nb + 1) / 2 + 8);
  AIRGA_TRY(ctx->ws_tmp.reserve(need));
  w->dinv = ctx->ws_tmp.as<double>();
  w->hat = w->dinv + pen.n_pad();
  w->ahat = w->hat + pen.nnz_stored;
  w->aold = w->ahat + pen.nnz_stored;
  w->part = w->aold + pen.nnz_stored;
  w->skip_part = reinterpret_cast<int32_t*>(w->part + 2 * nb);
  return AIRGA_OK;
}

// LDS-staged column kernels apply (bandwidth <= 64 and the window fits).
static bool spai_banded(const Pencil& pen, const airga_spai_opts& o, bool update) {
  if (o.general_only || o.mr_iters > 0 || pen.bandwidth > kSlice) return false;
  const size_t lds = pen.max_len <= 6 ? spai_band_lds<6>(pen.bandwidth, update)
                                      : spai_band_lds<kSpaiMaxJ>(pen.bandwidth, update);
  return lds <= 64 * 1024;
}

template <bool UPDATE>
static void launch_band(airga_ctx ctx, double a, double b, double ao, double bo,
                        const double* dinv, const double* alpha_u, double tol, double* hat,
                        double* obj, int32_t* skip, int8_t* skipf) {
  const Pencil& pen = ctx->pen;
  const unsigned nb = blocks_for(pen.n, 256);
  const int bw = pen.bandwidth;
  // fold the row span when it is no longer than the (column, entry) pairs
  const bool range = 4 * bw + 1 <= pen.max_len * pen.max_len;
  hipStream_t st = ctx->stream;
  const PencilDev pd = pen.dev();
  if (pen.max_len <= 6) {
    const size_t lds = spai_band_lds<6>(bw, UPDATE);
    if (range && pen.contiguous)
      k_spai_band<6, UPDATE, 2><<<nb, 256, lds, st>>>(pd, a, b, ao, bo, dinv, bw, alpha_u, tol,
                                                      hat, obj, skip, skipf);
    else if (range)
      k_spai_band<6, UPDATE, 1><<<nb, 256, lds, st>>>(pd, a, b, ao, bo, dinv, bw, alpha_u, tol,
                                                      hat, obj, skip, skipf);
    else
      k_spai_band<6, UPDATE, 0><<<nb, 256, lds, st>>>(pd, a, b, ao, bo, dinv, bw, alpha_u, tol,
                                                      hat, obj, skip, skipf);
  } else {
    const size_t lds = spai_band_lds<kSpaiMaxJ>(bw, UPDATE);
    if (range && pen.contiguous)
      k_spai_band<kSpaiMaxJ, UPDATE, 2><<<nb, 256, lds, st>>>(pd, a, b, ao, bo, dinv, bw,
                                                              alpha_u, tol, hat, obj, skip, skipf);
    else if (range)
      k_spai_band<kSpaiMaxJ, UPDATE, 1><<<nb, 256, lds, st>>>(pd, a, b, ao, bo, dinv, bw,
                                                              alpha_u, tol, hat, obj, skip, skipf);
    else
      k_spai_band<kSpaiMaxJ, UPDATE, 0><<<nb, 256, lds, st>>>(pd, a, b, ao, bo, dinv, bw,
                                                              alpha_u, tol, hat, obj, skip, skipf);
  }
}

// Column kernels sized to the longest row.
template <bool UPDATE>
static void launch_cols(airga_ctx ctx, const SpaiScratch& w, const double* alpha_u, double tol,
                        double* obj, int32_t* skip, int8_t* skipf) {
  const Pencil& pen = ctx->pen;
  const unsigned nb = blocks_for(pen.n, 256);
  if (pen.max_len <= 6)
    k_spai_cols<6, UPDATE><<<nb, 256, 0, ctx->stream>>>(pen.dev(), w.ahat, w.aold, alpha_u, tol,
                                                       w.hat, obj, skip, skipf);
  else
    k_spai_cols<kSpaiMaxJ, UPDATE><<<nb, 256, 0, ctx->stream>>>(pen.dev(), w.ahat, w.aold, alpha_u,
                                                               tol, w.hat, obj, skip, skipf);
}

// Largest step cap of the minimal-residual mode.
constexpr int kMrMaxIters = 100000;

// The minimal-residual column kernels, sized to the longest row.
template <bool UPDATE>
static void launch_mr(airga_ctx ctx, const SpaiScratch& w, const double* alpha, double tol,
                      int maxit, int lfil, double* obj, int32_t* skip, int8_t* skipf) {
  const Pencil& pen = ctx->pen;
  const unsigned nb = blocks_for(pen.n, 256);
  const PencilDev pd = pen.dev();
  if (pen.max_len <= 6 && pen.contiguous)
    k_spai_mr<6, UPDATE, true><<<nb, 256, 0, ctx->stream>>>(pd, w.ahat, w.aold, alpha, tol, maxit,
                                                           lfil, w.hat, obj, skip, skipf);
  else if (pen.max_len <= 6)
    k_spai_mr<6, UPDATE, false><<<nb, 256, 0, ctx->stream>>>(pd, w.ahat, w.aold, alpha, tol, maxit,
                                                            lfil, w.hat, obj, skip, skipf);
  else if (pen.contiguous)
    k_spai_mr<kSpaiMaxJ, UPDATE, true><<<nb, 256, 0, ctx->stream>>>(
        pd, w.ahat, w.aold, alpha, tol, maxit, lfil, w.hat, obj, skip, skipf);
  else
    k_spai_mr<kSpaiMaxJ, UPDATE, false><<<nb, 256, 0, ctx->stream>>>(
        pd, w.ahat, w.aold, alpha, tol, maxit, lfil, w.hat, obj, skip, skipf);
}

// The minimal-residual options: the step cap, and pattern control only with
// it (lfil up to the longest column the kernels hold).
static airga_status check_mr_opts(const airga_spai_opts& o) {
  if (o.mr_iters < 0 || o.mr_iters > kMrMaxIters)
    return fail(AIRGA_EINVAL, "mr_iters must be in [0, %d]", kMrMaxIters);
  if (o.lfil < 0 || o.lfil > kSpaiMaxJ)
    return fail(AIRGA_EINVAL, "lfil must be in [0, %d]", kSpaiMaxJ);
  if (o.lfil > 0 && o.mr_iters == 0)
    return fail(AIRGA_EINVAL, "lfil applies to the minimal-residual mode (mr_iters > 0)");
  return AIRGA_OK;
}

static airga_status run_build(airga_ctx ctx, double s, const airga_spai_opts& o, airga_prec p) {
  const Pencil& pen = ctx->pen;
  hipStream_t st = ctx->stream;
  double a, b;
  shift_coeffs(pen, s, &a, &b);
  const bool mr = o.mr_iters > 0;
  const unsigned nb = blocks_for(pen.n, 256);
  SpaiScratch w;
  AIRGA_TRY(spai_scratch(ctx, &w, mr ? nb : 0));
  const PencilDev pd = pen.dev();
  const unsigned nr = blocks_for(pen.n_pad(), 256);
  k_dinv<<<nr, 256, 0, st>>>(pd, a, b, o.equilibrate, w.dinv);
  AIRGA_HIP(hipGetLastError());
  if (spai_banded(pen, o, false)) {
    launch_band<false>(ctx, a, b, 0.0, 0.0, w.dinv, nullptr, 0.0, w.hat,
                       p->objective.as<double>(), nullptr, nullptr);
  } else {
    k_scaled_values<<<nr, 256, 0, st>>>(pd, a, b, w.dinv, w.ahat);
    AIRGA_HIP(hipGetLastError());
    if (mr) {
      // Algorithm 2: alpha of Khat on the device, no skipped columns
      double* d_alpha = p->scal.as<double>();
      k_alpha_build_partial<<<nb, 256, 0, st>>>(pd, a, b, w.dinv, w.part);
      AIRGA_HIP(hipGetLastError());
      k_alpha_final<<<1, 256, 0, st>>>(w.part, nb, d_alpha);
      AIRGA_HIP(hipGetLastError());
      k_fill_i32<<<1, 64, 0, st>>>(reinterpret_cast<int32_t*>(p->scal.as<char>() + 8), 1, 0);
      AIRGA_HIP(hipGetLastError());
      launch_mr<false>(ctx, w, d_alpha, o.tol, o.mr_iters, o.lfil, p->objective.as<double>(), nullptr,
                       nullptr);
    } else {
      launch_cols<false>(ctx, w, nullptr, 0.0, p->objective.as<double>(), nullptr, nullptr);
    }
  }
  AIRGA_HIP(hipGetLastError());
  k_spai_finalize<<<nr, 256, 0, st>>>(pd, w.hat, w.dinv, o.symmetrize ? 1 : 0, nullptr, nullptr,
                                      nullptr, p->v64.as<double>(), p->v32.as<float>());
  AIRGA_HIP(hipGetLastError());
  // Alg. 2's starting scaling trace(K) / trace(K K^T), from the Gram scalars
  // (minimal-residual mode: that of Khat, read from the device when needed).
  const double nn = a * a * pen.gram_mm + 2 * a * b * pen.gram_mk + b * b * pen.gram_kk;
  p->alpha = (a * pen.tr_m + b * pen.tr_k) / nn;
  p->alpha_known = !mr;
  p->skipped = 0;
  p->scalar_only = false;
  p->scalar_known = true;
  return AIRGA_OK;
}

static airga_status run_update(airga_ctx ctx, airga_prec old, double s_new,
                               const airga_spai_opts& o, airga_prec p) {
  const Pencil& pen = ctx->pen;
  hipStream_t st = ctx->stream;
  double a, b, ao, bo;
  shift_coeffs(pen, s_new, &a, &b);
  shift_coeffs(pen, old->shift, &ao, &bo);
  const unsigned nb = blocks_for(pen.n, 256);
  SpaiScratch w;
  AIRGA_TRY(spai_scratch(ctx, &w, nb));
  const PencilDev pd = pen.dev();
  const unsigned nr = blocks_for(pen.n_pad(), 256);
  double* d_alpha = p->scal.as<double>();
  int32_t* d_skip = reinterpret_cast<int32_t*>(p->scal.as<char>() + 8);
  const bool band = spai_banded(pen, o, true);
  k_dinv<<<nr, 256, 0, st>>>(pd, a, b, o.equilibrate, w.dinv);
  AIRGA_HIP(hipGetLastError());
  if (!band) {
    k_scaled_values<<<nr, 256, 0, st>>>(pd, a, b, w.dinv, w.ahat);
    AIRGA_HIP(hipGetLastError());
    k_scaled_values<<<nr, 256, 0, st>>>(pd, ao, bo, w.dinv, w.aold);
    AIRGA_HIP(hipGetLastError());
  }
  k_alpha_partial<<<nb, 256, 0, st>>>(pd, a, b, ao, bo, w.dinv, w.part);
  AIRGA_HIP(hipGetLastError());
  k_alpha_final<<<1, 256, 0, st>>>(w.part, nb, d_alpha);
  AIRGA_HIP(hipGetLastError());
  if (band)
    launch_band<true>(ctx, a, b, ao, bo, w.dinv, d_alpha, o.tol, w.hat, p->objective.as<double>(),
                      w.skip_part, skip_flags(p));
  else if (o.mr_iters > 0)
    launch_mr<true>(ctx, w, d_alpha, o.tol, o.mr_iters, o.lfil, p->objective.as<double>(), w.skip_part,
                    skip_flags(p));
  else
    launch_cols<true>(ctx, w, d_alpha, o.tol, p->objective.as<double>(), w.skip_part,
                      skip_flags(p));
  AIRGA_HIP(hipGetLastError());
  k_sum_counts<<<1, 256, 0, st>>>(w.skip_part, nb, d_skip);
  AIRGA_HIP(hipGetLastError());
  k_spai_finalize<<<nr, 256, 0, st>>>(pd, w.hat, w.dinv, 2, d_skip, skip_flags(p), d_alpha,
                                      p->v64.as<double>(), p->v32.as<float>());
  AIRGA_HIP(hipGetLastError());
  p->is_update = true;
  p->parent = old;
  old->refs++;
  return AIRGA_OK;
}

// Several updates at once (banded pencils whose staged rows fit in LDS);
// otherwise one after the other.
// Several builds at once (banded pencils whose staged rows fit in LDS);
// otherwise one after the other.  Each factor equals its single build.
// Builds from the Gram matrices of Khat^2 (k_spai_gram_wave): the staged
// batched path on a pencil whose rows are consecutive columns in a narrow
// band (bandwidth at most 8 for rows of 6 entries, like the beam's).
static bool spai_gram_path(const Pencil& pen, const airga_spai_opts& o) {
  const int bw = pen.bandwidth;
  // only the equilibrated problems: without the diagonal scaling the local
  // problems mix rows and columns of very different sizes, and squaring their
  // condition number costs digits the pivot test does not see
  return o.equilibrate && spai_banded(pen, o, false) && pen.max_len <= 6 && pen.contiguous &&
         4 * bw + 1 <= pen.max_len * pen.max_len && 2 * bw < kGramWave / 4 &&
         4 * spai_gram_wave_lds<6>(bw) <= 64 * 1024;
}

static airga_status run_build_many(airga_ctx ctx, int32_t count, const double* shifts,
                                   const airga_spai_opts& o, airga_prec* ps) {
  const Pencil& pen = ctx->pen;
  const bool fits = spai_banded(pen, o, false) && pen.max_len <= 6 &&
                    spai_build_many_lds<6>(pen.bandwidth) <= 64 * 1024;
  if (!fits) {
    for (int i = 0; i < count; ++i) AIRGA_TRY(run_build(ctx, shifts[i], o, ps[i]));
    return AIRGA_OK;
  }
  hipStream_t st = ctx->stream;
  const PencilDev pd = pen.dev();
  const int64_t n_pad = pen.n_pad(), stored = pen.nnz_stored;
  const unsigned nb = blocks_for(pen.n, 256);
  const unsigned nr = blocks_for(n_pad, 256);
  const int bw = pen.bandwidth;
  const bool range = 4 * bw + 1 <= pen.max_len * pen.max_len;
  const size_t lds = spai_build_many_lds<6>(bw);
  // rows of consecutive columns in a narrow band: Gram matrices from Khat^2
  // with the finalize fused in
  const bool gram = spai_gram_path(pen, o);
  // wavefronts of kGramWave - 2 bw output rows, four per block, cover every
  // padded row (padding rows of a factor hold zeros)
  const unsigned ng = blocks_for(n_pad, 4 * (kGramWave - 2 * bw));
  const size_t wave_lds = (spai_gram_wave_lds<6>(bw) + 15) & ~(size_t)15;
  for (int i0 = 0; i0 < count; i0 += kManyMax) {
    const int cnt = count - i0 < kManyMax ? count - i0 : kManyMax;
    // scratch: [dinv (cnt n_pad) | hat (cnt stored)]
    AIRGA_TRY(ctx->ws_tmp.reserve(sizeof(double) * (size_t)cnt * (n_pad + stored)));
    double* dinv = ctx->ws_tmp.as<double>();
    double* hat = dinv + (size_t)cnt * n_pad;
    UpdMany U;
    std::memset(static_cast<void*>(&U), 0, sizeof U);
    U.count = cnt;
    for (int i = 0; i < cnt; ++i) {
      shift_coeffs(pen, shifts[i0 + i], &U.a[i], &U.b[i]);
      U.obj[i] = ps[i0 + i]->objective.as<double>();
    }
    if (gram) {
      // the diagonal scaling is formed inside the kernel from diag(M), diag(K)
      for (int i = 0; i < cnt; ++i) {
        U.v64[i] = ps[i0 + i]->v64.as<double>();
        U.v32[i] = ps[i0 + i]->v32.as<float>();
      }
      if (bw == 3)
        k_spai_gram_wave<6, 3><<<ng, 256, 4 * wave_lds, st>>>(pd, U, n_pad, bw,
                                                             o.symmetrize ? 1 : 0, wave_lds);
      else
        k_spai_gram_wave<6, 0><<<ng, 256, 4 * wave_lds, st>>>(pd, U, n_pad, bw,
                                                             o.symmetrize ? 1 : 0, wave_lds);
    } else {
      k_dinv_many<<<nr, 256, 0, st>>>(pd, U, o.equilibrate, n_pad, dinv);
      if (range && pen.contiguous)
        k_spai_build_many<6, 2><<<nb, 256, lds, st>>>(pd, U, dinv, n_pad, stored, bw, hat);
      else if (range)
        k_spai_build_many<6, 1><<<nb, 256, lds, st>>>(pd, U, dinv, n_pad, stored, bw, hat);
      else
        k_spai_build_many<6, 0><<<nb, 256, lds, st>>>(pd, U, dinv, n_pad, stored, bw, hat);
    }
    AIRGA_HIP(hipGetLastError());
    for (int i = 0; i < cnt; ++i) {
      const airga_prec p = ps[i0 + i];
      if (!gram) {
        k_spai_finalize<<<nr, 256, 0, st>>>(pd, hat + (size_t)i * stored,
                                            dinv + (size_t)i * n_pad, o.symmetrize ? 1 : 0,
                                            nullptr, nullptr, nullptr, p->v64.as<double>(),
                                            p->v32.as<float>());
        AIRGA_HIP(hipGetLastError());
      }
      // Alg. 2's starting scaling trace(K) / trace(K K^T), from the Gram scalars
      const double a = U.a[i], b = U.b[i];
      const double nn = a * a * pen.gram_mm + 2 * a * b * pen.gram_mk + b * b * pen.gram_kk;
      p->alpha = (a * pen.tr_m + b * pen.tr_k) / nn;
      p->alpha_known = true;
      p->skipped = 0;
      p->scalar_only = false;
      p->scalar_known = true;
    }
  }
  return AIRGA_OK;
}

static airga_status run_update_many(airga_ctx ctx, int32_t count, const airga_prec* olds,
                                    const double* s_new, const airga_spai_opts& o,
                                    airga_prec* ps) {
  const Pencil& pen = ctx->pen;
  const bool fits = spai_banded(pen, o, true) && pen.max_len <= kManyJ &&
                    spai_many_lds<6>(pen.bandwidth) <= 64 * 1024 &&
                    dinv_many_lds(kManyMax, pen.bandwidth) + 1024 <= 64 * 1024;
  if (!fits) {
    for (int i = 0; i < count; ++i) AIRGA_TRY(run_update(ctx, olds[i], s_new[i], o, ps[i]));
    return AIRGA_OK;
  }
  hipStream_t st = ctx->stream;
  const PencilDev pd = pen.dev();
  const int64_t n_pad = pen.n_pad(), stored = pen.nnz_stored;
  const unsigned nb = blocks_for(pen.n, 256);
  const int bw = pen.bandwidth;
  const bool range = 4 * bw + 1 <= pen.max_len * pen.max_len;
  for (int i0 = 0; i0 < count; i0 += kManyMax) {
    const int cnt = count - i0 < kManyMax ? count - i0 : kManyMax;
    // scratch: [hat (cnt stored) | alpha partials | skip counts | blocks
    // with columns to solve]
    const size_t bytes = sizeof(double) * ((size_t)cnt * stored + 2 * (size_t)cnt * nb) +
                         2 * sizeof(int32_t) * (size_t)cnt * nb + 64;
    AIRGA_TRY(ctx->ws_tmp.reserve(bytes));
    double* hat = ctx->ws_tmp.as<double>();
    double* part = hat + (size_t)cnt * stored;
    int32_t* skp = reinterpret_cast<int32_t*>(part + 2 * (size_t)cnt * nb);
    int32_t* need = skp + (size_t)cnt * nb;
    UpdMany U;
    std::memset(static_cast<void*>(&U), 0, sizeof U);
    U.count = cnt;
    for (int i = 0; i < cnt; ++i) {
      const airga_prec p = ps[i0 + i];
      shift_coeffs(pen, s_new[i0 + i], &U.a[i], &U.b[i]);
      shift_coeffs(pen, olds[i0 + i]->shift, &U.ao[i], &U.bo[i]);
      U.alpha[i] = p->scal.as<double>();
      U.skip[i] = reinterpret_cast<int32_t*>(p->scal.as<char>() + 8);
      U.obj[i] = p->objective.as<double>();
      U.skipf[i] = skip_flags(p);
    }
    const size_t dl_lds = dinv_many_lds(cnt, bw);
    k_alpha_partial_many<<<nb, 256, dl_lds, st>>>(pd, U, bw, o.equilibrate, part);
    AIRGA_HIP(hipGetLastError());
    k_alpha_final_many<<<(unsigned)cnt, 256, 0, st>>>(U, part, nb);
    AIRGA_HIP(hipGetLastError());
    k_update_test_many<6><<<nb, 256, dl_lds, st>>>(pd, U, bw, o.equilibrate, o.tol, skp, need);
    AIRGA_HIP(hipGetLastError());
    const size_t lds = spai_many_lds<6>(bw);
    if (range && pen.contiguous)
      k_spai_update_many<6, 2><<<nb, 256, lds, st>>>(pd, U, o.equilibrate, stored, bw, o.tol, hat,
                                                     skp, need);
    else if (range)
      k_spai_update_many<6, 1><<<nb, 256, lds, st>>>(pd, U, o.equilibrate, stored, bw, o.tol, hat,
                                                     skp, need);
    else
      k_spai_update_many<6, 0><<<nb, 256, lds, st>>>(pd, U, o.equilibrate, stored, bw, o.tol, hat,
                                                     skp, need);
    AIRGA_HIP(hipGetLastError());
    k_sum_counts_many<<<(unsigned)cnt, 256, 0, st>>>(U, skp, nb);
    AIRGA_HIP(hipGetLastError());
    for (int i = 0; i < cnt; ++i) {
      U.v64[i] = ps[i0 + i]->v64.as<double>();
      U.v32[i] = ps[i0 + i]->v32.as<float>();
    }
    const unsigned fb = blocks_for(n_pad, 256) < 512 ? blocks_for(n_pad, 256) : 512;
    k_update_finalize_many<<<dim3(fb, (unsigned)cnt), 256, 0, st>>>(pd, U, hat, o.equilibrate,
                                                                    stored);
    AIRGA_HIP(hipGetLastError());
    for (int i = 0; i < cnt; ++i) {
      const airga_prec p = ps[i0 + i];
      p->is_update = true;
      p->parent = olds[i0 + i];
      olds[i0 + i]->refs++;
    }
  }
  return AIRGA_OK;
}

// The first 16 bytes of up to kFactsMax factors' device scalars (alpha, the
// skip count), gathered into one block so the host reads them in one copy.
constexpr int kFactsMax = 64;
struct FactsSrc {
  const int4* p[kFactsMax];
};
__global__ void k_gather_facts(FactsSrc src, int count, int4* out) {
  const int i = threadIdx.x;
  if (i < count) out[i] = src.p[i][0];
}

airga_status prec_resolve_many(airga_ctx ctx, const std::vector<airga_prec>& ps) {
  std::vector<airga_prec> todo;
  for (airga_prec p : ps)
    if (!(p->scalar_known && p->alpha_known)) todo.push_back(p);
  if (todo.empty()) return AIRGA_OK;
  struct Facts {
    double alpha;
    int32_t skipped, pad;
  };
  static_assert(sizeof(Facts) == sizeof(int4), "one 16-byte record per factor");
  AIRGA_TRY(ensure_pinned(ctx, sizeof(Facts) * todo.size()));
  AIRGA_TRY(ctx->ws_small.reserve(sizeof(Facts) * kFactsMax));
  Facts* h = static_cast<Facts*>(ctx->host_pinned);
  int4* staged = ctx->ws_small.as<int4>();
  for (size_t i0 = 0; i0 < todo.size(); i0 += kFactsMax) {
    const int cnt = (int)std::min(todo.size() - i0, (size_t)kFactsMax);
    FactsSrc src{};
    for (int i = 0; i < cnt; ++i) src.p[i] = todo[i0 + i]->scal.as<int4>();
    k_gather_facts<<<1, kFactsMax, 0, ctx->stream>>>(src, cnt, staged);
    AIRGA_HIP(hipGetLastError());
    AIRGA_HIP(hipMemcpyAsync(&h[i0], staged, sizeof(Facts) * cnt, hipMemcpyDeviceToHost,
                             ctx->stream));
  }
  AIRGA_HIP(hipStreamSynchronize(ctx->stream));
  for (size_t i = 0; i < todo.size(); ++i) {
    airga_prec p = todo[i];
    p->alpha = h[i].alpha;
    p->alpha_known = true;
    p->skipped = h[i].skipped;
    p->scalar_only = h[i].skipped == ctx->pen.n;
    p->scalar_known = true;
  }
  return AIRGA_OK;
}

airga_status prec_resolve(airga_prec p) {
  return prec_resolve_many(p->ctx, std::vector<airga_prec>{p});
}

airga_status prec_chain(airga_prec p, std::vector<airga_prec>* out) {
  out->clear();
  std::vector<airga_prec> all;
  for (airga_prec q = p; q; q = q->parent) all.push_back(q);
  AIRGA_TRY(prec_resolve_many(p->ctx, all));
  for (airga_prec q : all)
    if (!q->scalar_only) out->push_back(q);
  return AIRGA_OK;
}

static airga_status check_prec(airga_prec p) {
  if (!p) return fail(AIRGA_EINVAL, "null preconditioner");
  AIRGA_TRY(check_pencil(p->ctx));
  if (p->generation != p->ctx->pen.generation)
    return fail(AIRGA_ESTATE, "preconditioner was built for an earlier pencil");
  return AIRGA_OK;
}

}  // namespace airga

using namespace airga;

extern "C" {

void airga_spai_opts_default(airga_spai_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof *o);
  o->tol = 0.01;
  o->equilibrate = 1;
  o->symmetrize = 1;
}

airga_status airga_spai_build(airga_ctx ctx, double s, const airga_spai_opts* opts,
                              airga_prec* out) {
  AIRGA_TRY(check_spai_args(ctx, s, out));
  *out = nullptr;
  airga_spai_opts o;
  airga_spai_opts_default(&o);
  if (opts) o = *opts;
  AIRGA_TRY(check_mr_opts(o));
  if (!(o.tol >= 0)) return fail(AIRGA_EINVAL, "tolerance must be >= 0");
  airga_prec p = nullptr;
  AIRGA_TRY(new_prec(ctx, s, &p));
  // the Gram-matrix kernel of the batched builds serves single builds too,
  // so a factor does not depend on the batch it was built in
  airga_status st = spai_gram_path(ctx->pen, o) ? run_build_many(ctx, 1, &s, o, &p)
                                                : run_build(ctx, s, o, p);
  if (st != AIRGA_OK) {
    airga_prec_release(p);
    return st;
  }
  *out = p;
  return AIRGA_OK;
}

airga_status airga_spai_update(airga_ctx ctx, airga_prec old, double s_new,
                               const airga_spai_opts* opts, airga_prec* out) {
  AIRGA_TRY(check_spai_args(ctx, s_new, out));
  *out = nullptr;
  AIRGA_TRY(check_prec(old));
  if (old->ctx != ctx) return fail(AIRGA_EINVAL, "preconditioner belongs to another context");
  if (old->is_complex)
    return fail(AIRGA_EUNSUPPORTED, "a complex factor: use airga_spai_update_complex");
  airga_spai_opts o;
  airga_spai_opts_default(&o);
  if (opts) o = *opts;
  if (!(o.tol >= 0)) return fail(AIRGA_EINVAL, "update tolerance must be >= 0");
  AIRGA_TRY(check_mr_opts(o));
  airga_prec p = nullptr;
  AIRGA_TRY(new_prec(ctx, s_new, &p));
  airga_status st = run_update(ctx, old, s_new, o, p);
  if (st != AIRGA_OK) {
    airga_prec_release(p);
    return st;
  }
  *out = p;
  return AIRGA_OK;
}

airga_status airga_spai_build_many(airga_ctx ctx, int32_t count, const double* shifts,
                                   const airga_spai_opts* opts, airga_prec* out) {
  AIRGA_TRY(check_pencil(ctx));
  if (count < 0 || (count > 0 && (!shifts || !out))) return fail(AIRGA_EINVAL, "bad build batch");
  for (int32_t i = 0; i < count; ++i) {
    out[i] = nullptr;
    airga_prec dummy;
    AIRGA_TRY(check_spai_args(ctx, shifts[i], &dummy));
  }
  airga_spai_opts o;
  airga_spai_opts_default(&o);
  if (opts) o = *opts;
  AIRGA_TRY(check_mr_opts(o));
  if (!(o.tol >= 0)) return fail(AIRGA_EINVAL, "tolerance must be >= 0");
  std::vector<airga_prec> ps(count, nullptr);
  airga_status st = AIRGA_OK;
  for (int32_t i = 0; i < count && st == AIRGA_OK; ++i) st = new_prec(ctx, shifts[i], &ps[i]);
  if (st == AIRGA_OK) st = run_build_many(ctx, count, shifts, o, ps.data());
  if (st != AIRGA_OK) {
    for (airga_prec p : ps) airga_prec_release(p);
    return st;
  }
  for (int32_t i = 0; i < count; ++i) out[i] = ps[i];
  return AIRGA_OK;
}

airga_status airga_spai_update_many(airga_ctx ctx, int32_t count, const airga_prec* olds,
                                    const double* s_new, const airga_spai_opts* opts,
                                    airga_prec* out) {
  AIRGA_TRY(check_pencil(ctx));
  if (count < 0 || (count > 0 && (!olds || !s_new || !out)))
    return fail(AIRGA_EINVAL, "bad update batch");
  for (int32_t i = 0; i < count; ++i) {
    out[i] = nullptr;
    airga_prec dummy;
    AIRGA_TRY(check_spai_args(ctx, s_new[i], &dummy));
    AIRGA_TRY(check_prec(olds[i]));
    if (olds[i]->ctx != ctx) return fail(AIRGA_EINVAL, "preconditioner belongs to another context");
    if (olds[i]->is_complex)
      return fail(AIRGA_EUNSUPPORTED, "a complex factor: use airga_spai_update_complex");
  }
  airga_spai_opts o;
  airga_spai_opts_default(&o);
  if (opts) o = *opts;
  if (!(o.tol >= 0)) return fail(AIRGA_EINVAL, "update tolerance must be >= 0");
  AIRGA_TRY(check_mr_opts(o));
  std::vector<airga_prec> ps(count, nullptr);
  airga_status st = AIRGA_OK;
  for (int32_t i = 0; i < count && st == AIRGA_OK; ++i) st = new_prec(ctx, s_new[i], &ps[i]);
  if (st == AIRGA_OK) st = run_update_many(ctx, count, olds, s_new, o, ps.data());
  if (st != AIRGA_OK) {
    for (airga_prec p : ps) airga_prec_release(p);
    return st;
  }
  for (int32_t i = 0; i < count; ++i) out[i] = ps[i];
  return AIRGA_OK;
}

airga_status airga_get_prec_info(airga_prec prec, airga_prec_info* out) {
  AIRGA_TRY(check_prec(prec));
  if (!out) return fail(AIRGA_EINVAL, "null output");
  AIRGA_TRY(prec_resolve(prec));
  std::vector<airga_prec> chain;
  AIRGA_TRY(prec_chain(prec, &chain));
  out->shift = prec->shift;
  out->alpha = prec->alpha;
  out->chain_len = (int32_t)chain.size();
  out->scalar_only = prec->scalar_only ? 1 : 0;
  out->skipped_cols = prec->skipped;
  out->shift_im = prec->shift_im;
  out->alpha_im = prec->alpha_im;
  out->is_complex = prec->is_complex ? 1 : 0;
  return AIRGA_OK;
}

airga_status airga_prec_export(airga_prec prec, double* values, double* objective) {
  AIRGA_TRY(check_prec(prec));
  if (prec->is_complex) return fail(AIRGA_EINVAL, "complex factor: use airga_prec_export_complex");
  airga_ctx ctx = prec->ctx;
  if (values) {
    // an update with every column skipped holds no factor values
    AIRGA_TRY(prec_resolve(prec));
    if (prec->is_update && prec->scalar_only)
      k_export_scalar<<<blocks_for(ctx->pen.n, 256), 256, 0, ctx->stream>>>(ctx->pen.dev(),
                                                                            prec->alpha, values);
    else
      k_export<<<blocks_for(ctx->pen.nnz_stored, 256), 256, 0, ctx->stream>>>(
          ctx->pen.dev(), ctx->pen.nnz_stored, prec->v64.as<double>(), values);
    AIRGA_HIP(hipGetLastError());
  }
  if (objective)
    AIRGA_HIP(hipMemcpyAsync(objective, prec->objective.ptr, sizeof(double) * ctx->pen.n,
                             hipMemcpyDeviceToDevice, ctx->stream));
  return AIRGA_OK;
}

airga_status airga_prec_skip_flags(airga_prec prec, uint8_t* flags) {
  AIRGA_TRY(check_prec(prec));
  if (!flags) return fail(AIRGA_EINVAL, "null flags");
  airga_ctx ctx = prec->ctx;
  const int8_t* src = prec->is_update ? skip_flags(prec) : nullptr;
  k_copy_flags<<<blocks_for(ctx->pen.n, 256), 256, 0, ctx->stream>>>(src, ctx->pen.n, flags);
  AIRGA_HIP(hipGetLastError());
  return AIRGA_OK;
}

airga_status airga_prec_apply(airga_prec prec, int32_t count, const double* r, int64_t ldr,
                              double* z, int64_t ldz) {
  AIRGA_TRY(check_prec(prec));
  if (prec->is_complex) return fail(AIRGA_EINVAL, "complex factors apply in airga_cocg_solve only");
  airga_ctx ctx = prec->ctx;
  const Pencil& pen = ctx->pen;
  if (count < 0 || (count > 0 && (!r || !z))) return fail(AIRGA_EINVAL, "bad vectors");
  if (count > 65535) return fail(AIRGA_EUNSUPPORTED, "more than 65535 vectors");
  if (ldr < pen.n || ldz < pen.n) return fail(AIRGA_EINVAL, "leading dimension < n");
  if (count == 0) return AIRGA_OK;
  // factors oldest first: P_1, Q_2, ..., Q_z
  std::vector<airga_prec> all;
  for (airga_prec q = prec; q; q = q->parent) {
    AIRGA_TRY(prec_resolve(q));
    all.push_back(q);
  }
  const size_t per = (size_t)pen.n_pad();
  AIRGA_TRY(ctx->ws_asm.reserve(sizeof(double) * per * 2 * (size_t)count));
  double* tmp[2] = {ctx->ws_asm.as<double>(), ctx->ws_asm.as<double>() + per * count};
  const double* src = r;
  int64_t lds = ldr;
  dim3 grid(blocks_for(pen.n, 256), (unsigned)count);
  for (size_t f = all.size(); f-- > 0;) {
    airga_prec q = all[f];
    const bool last = f == 0;
    double* dst = last ? z : tmp[f & 1];
    const int64_t ldd = last ? ldz : (int64_t)per;
    if (q->scalar_only)
      k_factor_apply<<<grid, 256, 0, ctx->stream>>>(pen.dev(), nullptr, q->alpha, src, lds, dst, ldd);
    else
      k_factor_apply<<<grid, 256, 0, ctx->stream>>>(pen.dev(), q->v64.as<double>(), 1.0, src, lds,
                                                    dst, ldd);
    AIRGA_HIP(hipGetLastError());
    src = dst;
    lds = ldd;
  }
  return AIRGA_OK;
}

void airga_prec_release(airga_prec prec) {
  while (prec) {
    if (--prec->refs > 0) return;
    airga_prec parent = prec->parent;
    airga_ctx ctx = prec->ctx;
    // buffers go back to the context's stream-ordered pool
    pool_put(ctx, &prec->v64);
    pool_put(ctx, &prec->v32);
    pool_put(ctx, &prec->objective);
    pool_put(ctx, &prec->scal);
    ctx->live_precs--;
    delete prec;
    prec = parent;
  }
}

}  // extern "C"
