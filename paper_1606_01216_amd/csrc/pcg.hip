// Batched preconditioned CG for K(s_k) X = F over all (shift, column)
// systems at once, in float64 or in float32 inside float64 iterative
// refinement.  (CG: Section 3 and Section 5; solves of the AIRGA algorithm
// and of its SPAI and SPAI-update variants.)
//
// Data layout.  Matrices are in the pencil's sliced-ELL form (64-row slices,
// one row per lane).  Every per-system vector is contiguous (length n_pad),
// kind-major: vec(kind, b) = ws + (kind * B + b) * n_pad.  A wavefront owns
// R consecutive slices; it loads their column indices and M, K values once
// into registers and then sweeps every active system, so the pencil is read
// once per kernel for the whole batch.  The shifted matrix is never stored:
// K(s_k) p = a_k (M p) + b_k (K p).
//
// One CG iteration is two row-parallel kernels and two tiny reductions:
//   A  p_new = z + beta p_old;  w = K(s) p_new;  partial (p_new, w)
//   reduce -> alpha = (r, z) / (p, w)
//   B  r_new = r - alpha w;  x += alpha p_new;  t = P_1 r_new;  partials of
//      (r_new, r_new), (r_new, z), (z, w)      [z = t for a one-factor chain]
//   [chain: z = Q_c ... Q_2 t, one kernel per further factor]
//   reduce -> convergence; beta = -(z, w) / (p, w)
// Neighbour values (p_new at a column, r_new at a column) are recomputed from
// the previous iterate instead of being exchanged: p and r are double
// buffered, so no kernel reads what another block of the same kernel writes.
// The direction update keeps p_new K-conjugate to p_old, which needs no
// symmetry of the preconditioner (a fixed-pattern right SPAI and every
// update chain are non-symmetric); for a symmetric preconditioner it is the
// classical CG ratio.
//
// Reductions are deterministic: one partial per (system, wavefront) and a
// fixed-order sum per system.
#include <cmath>
#include <cstring>
#include <vector>

#include "internal.hpp"

namespace airga {

enum VecKind { KX = 0, KR0, KR1, KZ, KP0, KP1, KW, KT, KINDS };
constexpr int kSlots = 4;  // partial slots per (system, wave): pw | rr, rz, zw
enum { ST_CONV = AIRGA_SYS_CONVERGED, ST_MAXIT = AIRGA_SYS_MAXIT,
       ST_BREAK = AIRGA_SYS_BREAKDOWN, ST_NONFIN = AIRGA_SYS_NONFINITE };

// Per-system device state.
struct SysDev {
  double *rz, *pw, *alpha, *beta, *tol2, *ff, *relres;
  int32_t *active, *first, *istat, *status, *iters, *sweeps, *outer;
};

template <typename T>
struct SolveArgs {
  PencilDev pd;
  const T* mv;               // M values in T (or the assembled K(s) when kv == nullptr)
  const T* kv;               // K values in T
  int32_t B, m, nshift, G;
  int64_t ld;                // n_pad
  T* ws;                     // vector workspace
  T* x;                      // iteration solution, system b at x + b * ldx
  int64_t ldx;
  const T* ca;               // per shift a_k = s_k^2 + alpha s_k
  const T* cb;               // per shift b_k = 1 + beta s_k
  const T* const* fac;       // per shift [maxc] factor values, fac[sh * maxc + q], oldest first
  const int32_t* clen;       // per shift number of applied factors
  int32_t maxc;
  double* partial;           // [B][G][kSlots]
  SysDev sys;
  int32_t max_iter;
  __device__ __forceinline__ T* vec(int kind, int b) const {
    return ws + ((int64_t)kind * B + b) * ld;
  }
  __device__ __forceinline__ double* slot(int b, int g) const {
    return partial + ((int64_t)b * G + g) * kSlots;
  }
};

// Buffer written by chain position q (0 = the fused first factor) for a chain
// of L factors: the last one lands in KZ, earlier ones alternate with KT.
__device__ __forceinline__ int chain_dst(int q, int L) { return ((L - 1 - q) & 1) ? KT : KZ; }

// Row set of one wavefront: R consecutive slices.
template <int WMAX, int R>
struct Rows {
  int32_t col[R][WMAX];
  int32_t idx0[R];   // stored index of entry 0 of the lane's row in slice i
  int32_t w[R];
  int64_t row[R];
  __device__ __forceinline__ void load(const PencilDev& pd, int wg, int lane) {
#pragma unroll
    for (int i = 0; i < R; ++i) {
      const int64_t s = (int64_t)wg * R + i;
      row[i] = s * kSlice + lane;
      w[i] = 0;
      idx0[i] = 0;
      if (s < pd.n_slices) {
        idx0[i] = pd.slice_ptr[s] + lane;
        w[i] = (pd.slice_ptr[s + 1] - pd.slice_ptr[s]) / kSlice;
#pragma unroll
        for (int k = 0; k < WMAX; ++k) col[i][k] = k < w[i] ? pd.col[idx0[i] + k * kSlice] : 0;
      }
    }
  }
  template <typename T>
  __device__ __forceinline__ void values(const T* __restrict__ v, T (&out)[R][WMAX]) const {
#pragma unroll
    for (int i = 0; i < R; ++i)
#pragma unroll
      for (int k = 0; k < WMAX; ++k) out[i][k] = k < w[i] ? v[idx0[i] + k * kSlice] : T(0);
  }
};

// ---- A: direction update + shifted SpMV + (p, w) -------------------------
template <typename T, int WMAX, int R, bool ASM>
__global__ void __launch_bounds__(256) k_dir_spmv(SolveArgs<T> A, int par) {
  const int lane = threadIdx.x & 63;
  const int wg = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (wg >= A.G) return;
  Rows<WMAX, R> rows;
  rows.load(A.pd, wg, lane);
  T mv[R][WMAX], kv[R][WMAX];
  rows.values(A.mv, mv);
  if constexpr (!ASM) rows.values(A.kv, kv);
  const int64_t n = A.pd.n;
  for (int b = 0; b < A.B; ++b) {
    if (!A.sys.active[b]) continue;
    const int sh = b / A.m;
    const bool first = A.sys.first[b] != 0;
    const T beta = first ? T(0) : (T)A.sys.beta[b];
    const T* __restrict__ z = A.vec(KZ, b);
    const T* __restrict__ pin = A.vec(KP0 + par, b);
    T* __restrict__ pout = A.vec(KP0 + (par ^ 1), b);
    T* __restrict__ wv = A.vec(KW, b);
    T ca = T(1), cb = T(0);
    if constexpr (!ASM) {
      ca = A.ca[sh];
      cb = A.cb[sh];
    }
    T dot = T(0);
#pragma unroll
    for (int i = 0; i < R; ++i) {
      const int64_t r = rows.row[i];
      if (r < n) {
        T am = T(0), ak = T(0);
#pragma unroll
        for (int k = 0; k < WMAX; ++k) {
          if (k < rows.w[i]) {
            const int c = rows.col[i][k];
            const T pc = first ? z[c] : fma(beta, pin[c], z[c]);
            am = fma(mv[i][k], pc, am);
            if constexpr (!ASM) ak = fma(kv[i][k], pc, ak);
          }
        }
        const T pr = first ? z[r] : fma(beta, pin[r], z[r]);
        const T wr = ASM ? am : fma(ca, am, cb * ak);
        pout[r] = pr;
        wv[r] = wr;
        dot = fma(pr, wr, dot);
      }
    }
    dot = wave_sum(dot);
    if (lane == 0) A.slot(b, wg)[0] = (double)dot;
  }
}

// ---- B: x/r update + first preconditioner factor + dots -------------------
// INIT: no update; r is R0 as produced by the residual kernel.
template <typename T, int WMAX, int R, bool INIT>
__global__ void __launch_bounds__(256) k_update_prec(SolveArgs<T> A, int par) {
  const int lane = threadIdx.x & 63;
  const int wg = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (wg >= A.G) return;
  Rows<WMAX, R> rows;
  rows.load(A.pd, wg, lane);
  const int64_t n = A.pd.n;
  for (int sh = 0; sh < A.nshift; ++sh) {
    const int L = A.clen[sh];
    const T* __restrict__ P = L > 0 ? A.fac[(int64_t)sh * A.maxc] : nullptr;
    T pv[R][WMAX];
    bool loaded = false;
    for (int c = 0; c < A.m; ++c) {
      const int b = sh * A.m + c;
      if (!A.sys.active[b]) continue;
      if (P && !loaded) {
        rows.values(P, pv);
        loaded = true;
      }
      const T al = INIT ? T(0) : (T)A.sys.alpha[b];
      const T* __restrict__ rin = A.vec(INIT ? KR0 : KR0 + par, b);
      const T* __restrict__ wv = A.vec(KW, b);
      const T* __restrict__ pcur = A.vec(KP0 + (par ^ 1), b);
      T* __restrict__ rout = A.vec(KR0 + (par ^ 1), b);
      T* __restrict__ zo = A.vec(chain_dst(0, L > 0 ? L : 1), b);
      T* __restrict__ x = A.x + (int64_t)b * A.ldx;
      T rr = T(0), rz = T(0), zw = T(0);
#pragma unroll
      for (int i = 0; i < R; ++i) {
        const int64_t r = rows.row[i];
        if (r < n) {
          T rn, wr = T(0);
          if constexpr (INIT) {
            rn = rin[r];
          } else {
            wr = wv[r];
            rn = fma(-al, wr, rin[r]);
            x[r] = fma(al, pcur[r], x[r]);
            rout[r] = rn;
          }
          T t;
          if (P) {
            t = T(0);
#pragma unroll
            for (int k = 0; k < WMAX; ++k) {
              if (k < rows.w[i]) {
                const int cc = rows.col[i][k];
                const T rc = INIT ? rin[cc] : fma(-al, wv[cc], rin[cc]);
                t = fma(pv[i][k], rc, t);
              }
            }
          } else {
            t = rn;
          }
          zo[r] = t;
          rr = fma(rn, rn, rr);
          rz = fma(rn, t, rz);
          zw = fma(t, wr, zw);
        }
      }
      rr = wave_sum(rr);
      rz = wave_sum(rz);
      zw = wave_sum(zw);
      if (lane == 0) {
        double* s = A.slot(b, wg);
        s[1] = (double)rr;
        s[2] = L > 1 ? 0.0 : (double)rz;
        s[3] = L > 1 ? 0.0 : (double)zw;
      }
    }
  }
}

// ---- chain factor q >= 1 (Q_{q+1} of the update chain) ---------------------
template <typename T, int WMAX, int R>
__global__ void __launch_bounds__(256) k_chain(SolveArgs<T> A, int par, int q, int init) {
  const int lane = threadIdx.x & 63;
  const int wg = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (wg >= A.G) return;
  Rows<WMAX, R> rows;
  rows.load(A.pd, wg, lane);
  const int64_t n = A.pd.n;
  const int rk = init ? KR0 : KR0 + (par ^ 1);
  for (int sh = 0; sh < A.nshift; ++sh) {
    const int L = A.clen[sh];
    if (L <= q) continue;
    const T* __restrict__ F = A.fac[(int64_t)sh * A.maxc + q];
    T fv[R][WMAX];
    bool loaded = false;
    for (int c = 0; c < A.m; ++c) {
      const int b = sh * A.m + c;
      if (!A.sys.active[b]) continue;
      if (!loaded) {
        rows.values(F, fv);
        loaded = true;
      }
      const T* __restrict__ src = A.vec(chain_dst(q - 1, L), b);
      T* __restrict__ dst = A.vec(chain_dst(q, L), b);
      const bool last = q == L - 1;
      const T* __restrict__ rv = A.vec(rk, b);
      const T* __restrict__ wv = A.vec(KW, b);
      T rz = T(0), zw = T(0);
#pragma unroll
      for (int i = 0; i < R; ++i) {
        const int64_t r = rows.row[i];
        if (r < n) {
          T t = T(0);
#pragma unroll
          for (int k = 0; k < WMAX; ++k)
            if (k < rows.w[i]) t = fma(fv[i][k], src[rows.col[i][k]], t);
          dst[r] = t;
          if (last) {
            rz = fma(rv[r], t, rz);
            if (!init) zw = fma(t, wv[r], zw);
          }
        }
      }
      if (last) {
        rz = wave_sum(rz);
        zw = wave_sum(zw);
        if (lane == 0) {
          double* s = A.slot(b, wg);
          s[2] = (double)rz;
          s[3] = (double)zw;
        }
      }
    }
  }
}

// ---- float64 residual r = F - K(s) X (and |F|^2), output in TO -------------
// xmode 0: X is read;  1: X is taken as 0 and zeroed.  Also zeroes the inner
// solution vector (kind KX) when zero_inner is set.
template <typename TO, int WMAX, int R>
__global__ void __launch_bounds__(256) k_residual(SolveArgs<TO> A, const double* __restrict__ F,
                                                  int64_t ldf, double* __restrict__ X,
                                                  int64_t ldX, const double* __restrict__ ca64,
                                                  const double* __restrict__ cb64, int xmode,
                                                  int zero_inner) {
  const int lane = threadIdx.x & 63;
  const int wg = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (wg >= A.G) return;
  Rows<WMAX, R> rows;
  rows.load(A.pd, wg, lane);
  double mv[R][WMAX], kv[R][WMAX];
  rows.values(A.pd.m64, mv);
  rows.values(A.pd.k64, kv);
  const int64_t n = A.pd.n;
  for (int b = 0; b < A.B; ++b) {
    if (!A.sys.outer[b]) continue;
    const int sh = b / A.m, c = b % A.m;
    const double a = ca64[sh], bb = cb64[sh];
    const double* __restrict__ f = F + (int64_t)c * ldf;
    double* __restrict__ x = X + (int64_t)b * ldX;
    TO* __restrict__ r = A.vec(KR0, b);
    TO* __restrict__ xi = A.vec(KX, b);
    double rr = 0, ff = 0;
#pragma unroll
    for (int i = 0; i < R; ++i) {
      const int64_t row = rows.row[i];
      if (row < n) {
        double am = 0, ak = 0;
        if (xmode == 0) {
#pragma unroll
          for (int k = 0; k < WMAX; ++k) {
            if (k < rows.w[i]) {
              const double xc = x[rows.col[i][k]];
              am = fma(mv[i][k], xc, am);
              ak = fma(kv[i][k], xc, ak);
            }
          }
        }
        const double fr = f[row];
        const double res = fr - fma(a, am, bb * ak);
        r[row] = (TO)res;
        if (zero_inner) xi[row] = TO(0);
        rr = fma(res, res, rr);
        ff = fma(fr, fr, ff);
      }
    }
    // X is zeroed after every lane of the grid has read it?  Only when X is
    // not read (xmode 1), so no ordering question arises.
    if (xmode == 1) {
#pragma unroll
      for (int i = 0; i < R; ++i)
        if (rows.row[i] < n) x[rows.row[i]] = 0.0;
    }
    rr = wave_sum(rr);
    ff = wave_sum(ff);
    if (lane == 0) {
      double* s = A.slot(b, wg);
      s[0] = rr;
      s[1] = ff;
    }
  }
}

// X += inner solution (float32 -> float64) for systems refined this sweep.
__global__ void k_ir_update(SolveArgs<float> A, double* __restrict__ X, int64_t ldX) {
  const int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int b = blockIdx.y;
  if (!A.sys.outer[b] || A.sys.istat[b] == ST_NONFIN) return;
  if (r < A.pd.n) X[(int64_t)b * ldX + r] += (double)A.vec(KX, b)[r];
  if (r == 0) A.sys.sweeps[b] += 1;
}

// ---- per-system reductions (one block per system) ------------------------
enum ReduceMode {
  RM_PW = 0,        // after A: alpha = rz / pw
  RM_ITER = 1,      // after B (+chain): convergence, beta
  RM_INIT_ABS = 2,  // after the first preconditioner application, tol2 relative to |F|^2
  RM_INIT_REL = 3,  // same, tol2 relative to the starting residual (inner solves)
  RM_START = 4,     // after the float64 residual: record |F|^2 (FP64 mode)
  RM_OUTER = 5,     // after the float64 residual: refinement control (MIXED)
  RM_FINAL = 6,     // after the final float64 residual: relres only
};

struct ReduceArgs {
  const double* partial;
  int32_t G;
  SysDev sys;
  int32_t max_iter;
  int32_t max_sweeps;
  double tol2_rel;  // tol^2 (outer) or inner_tol^2
  double tol2_abs;  // tol^2 for RM_OUTER
  int32_t mixed;
};

__global__ void __launch_bounds__(256) k_reduce(ReduceArgs P, int mode) {
  __shared__ double red[4][256];
  const int b = blockIdx.x;
  const int t = threadIdx.x;
  const SysDev& S = P.sys;
  const bool use_outer = mode == RM_START || mode == RM_OUTER || mode == RM_FINAL;
  if (use_outer ? !S.outer[b] : !S.active[b]) return;
  double v[4] = {0, 0, 0, 0};
  const double* base = P.partial + (int64_t)b * P.G * kSlots;
  for (int g = t; g < P.G; g += blockDim.x)
#pragma unroll
    for (int q = 0; q < 4; ++q) v[q] += base[(int64_t)g * kSlots + q];
#pragma unroll
  for (int q = 0; q < 4; ++q) red[q][t] = v[q];
  __syncthreads();
  for (int h = blockDim.x / 2; h > 0; h >>= 1) {
    if (t < h)
#pragma unroll
      for (int q = 0; q < 4; ++q) red[q][t] += red[q][t + h];
    __syncthreads();
  }
  if (t != 0) return;
  const double s0 = red[0][0], rr = red[1][0], rz = red[2][0], zw = red[3][0];
  switch (mode) {
    case RM_PW: {
      const double pw = s0;
      if (!isfinite(pw)) { S.istat[b] = ST_NONFIN; S.active[b] = 0; }
      else if (pw <= 0.0) { S.istat[b] = ST_BREAK; S.active[b] = 0; }
      else { S.pw[b] = pw; S.alpha[b] = S.rz[b] / pw; }
      break;
    }
    case RM_ITER: {
      const int it = S.iters[b] + 1;
      S.iters[b] = it;
      if (!isfinite(rr) || !isfinite(rz) || !isfinite(zw)) { S.istat[b] = ST_NONFIN; S.active[b] = 0; }
      else if (rr <= S.tol2[b]) { S.istat[b] = ST_CONV; S.active[b] = 0; }
      else if (it >= P.max_iter) { S.istat[b] = ST_MAXIT; S.active[b] = 0; }
      else { S.beta[b] = -zw / S.pw[b]; S.rz[b] = rz; S.first[b] = 0; }
      break;
    }
    case RM_INIT_ABS:
    case RM_INIT_REL: {
      if (mode == RM_INIT_REL) S.tol2[b] = P.tol2_rel * rr;
      S.first[b] = 1;
      S.beta[b] = 0.0;
      if (!isfinite(rr) || !isfinite(rz)) { S.istat[b] = ST_NONFIN; S.active[b] = 0; }
      else if (rr <= S.tol2[b]) { S.istat[b] = ST_CONV; S.active[b] = 0; }
      else if (S.iters[b] >= P.max_iter) { S.istat[b] = ST_MAXIT; S.active[b] = 0; }
      else { S.rz[b] = rz; S.istat[b] = ST_MAXIT; }
      break;
    }
    case RM_START: {
      // residual kernel slots: 0 = |F - K X|^2, 1 = |F|^2
      S.ff[b] = rr;
      S.tol2[b] = P.tol2_rel * S.ff[b];
      S.relres[b] = S.ff[b] > 0 ? sqrt(s0 / S.ff[b]) : 0.0;
      break;
    }
    case RM_OUTER: {
      // residual kernel slots: 0 = |F - K X|^2, 1 = |F|^2
      if (S.sweeps[b] == 0) S.ff[b] = rr;
      const double ff = S.ff[b];
      S.relres[b] = ff > 0 ? sqrt(s0 / ff) : 0.0;
      if (!isfinite(s0)) { S.status[b] = ST_NONFIN; S.outer[b] = 0; }
      else if (s0 <= P.tol2_abs * ff) { S.status[b] = ST_CONV; S.outer[b] = 0; }
      else if (S.sweeps[b] > 0 && (S.istat[b] == ST_BREAK || S.istat[b] == ST_NONFIN)) {
        S.status[b] = S.istat[b]; S.outer[b] = 0;
      } else if (S.iters[b] >= P.max_iter || S.sweeps[b] >= P.max_sweeps) {
        S.status[b] = ST_MAXIT; S.outer[b] = 0;
      } else {
        S.active[b] = 1;
      }
      break;
    }
    case RM_FINAL: {
      const double ff = S.ff[b];
      S.relres[b] = ff > 0 ? sqrt(s0 / ff) : 0.0;
      break;
    }
  }
}

// ------------------------------------------------------------- dispatch

template <typename T>
struct KernelSet {
  void (*dir)(SolveArgs<T>, int);
  void (*dir_asm)(SolveArgs<T>, int);
  void (*upd)(SolveArgs<T>, int);
  void (*init)(SolveArgs<T>, int);
  void (*chain)(SolveArgs<T>, int, int, int);
  void (*resid)(SolveArgs<T>, const double*, int64_t, double*, int64_t, const double*,
                const double*, int, int);
};

template <typename T, int WMAX, int R>
KernelSet<T> make_set() {
  KernelSet<T> s;
  s.dir = k_dir_spmv<T, WMAX, R, false>;
  s.dir_asm = k_dir_spmv<T, WMAX, R, true>;
  s.upd = k_update_prec<T, WMAX, R, false>;
  s.init = k_update_prec<T, WMAX, R, true>;
  s.chain = k_chain<T, WMAX, R>;
  s.resid = k_residual<T, WMAX, R>;
  return s;
}

template <typename T>
KernelSet<T> kernel_set(int wmax_class, int rows) {
  // wmax_class: 0 -> rows of <= 6 entries, 1 -> <= 8, 2 -> <= 16
  switch (wmax_class * 3 + (rows == 1 ? 0 : rows == 2 ? 1 : 2)) {
    case 0: return make_set<T, 6, 1>();
    case 1: return make_set<T, 6, 2>();
    case 2: return make_set<T, 6, 4>();
    case 3: return make_set<T, 8, 1>();
    case 4: return make_set<T, 8, 2>();
    case 5: return make_set<T, 8, 4>();
    case 6: return make_set<T, 16, 1>();
    case 7: return make_set<T, 16, 2>();
    default: return make_set<T, 16, 4>();
  }
}

inline int wmax_class(int max_len) { return max_len <= 6 ? 0 : max_len <= 8 ? 1 : 2; }

// Launch with optional per-launch event timing.
struct Timer {
  airga_ctx ctx;
  bool on;
  std::vector<hipEvent_t> ev;     // pairs
  std::vector<int> ids;
  airga_status begin(int id, hipEvent_t* e0) {
    if (!on) return AIRGA_OK;
    hipEvent_t a, b;
    AIRGA_HIP(hipEventCreate(&a));
    AIRGA_HIP(hipEventCreate(&b));
    ev.push_back(a);
    ev.push_back(b);
    ids.push_back(id);
    AIRGA_HIP(hipEventRecord(a, ctx->stream));
    *e0 = b;
    return AIRGA_OK;
  }
  airga_status end(hipEvent_t e1) {
    if (!on) return AIRGA_OK;
    AIRGA_HIP(hipEventRecord(e1, ctx->stream));
    return AIRGA_OK;
  }
  airga_status flush() {
    if (!on) return AIRGA_OK;
    AIRGA_HIP(hipStreamSynchronize(ctx->stream));
    for (size_t i = 0; i < ids.size(); ++i) {
      float ms = 0;
      AIRGA_HIP(hipEventElapsedTime(&ms, ev[2 * i], ev[2 * i + 1]));
      ctx->times.launches[ids[i]] += 1;
      ctx->times.ms[ids[i]] += ms;
    }
    for (auto e : ev) (void)hipEventDestroy(e);
    ev.clear();
    ids.clear();
    return AIRGA_OK;
  }
  ~Timer() {
    for (auto e : ev) (void)hipEventDestroy(e);
  }
};

#define TIMED(id, ...)                             \
  do {                                             \
    hipEvent_t e1_ = nullptr;                      \
    AIRGA_TRY(tm.begin((id), &e1_));               \
    __VA_ARGS__;                                   \
    AIRGA_HIP(hipGetLastError());                  \
    AIRGA_TRY(tm.end(e1_));                        \
  } while (0)

// Host-side plan of one solve.
template <typename T>
struct Plan {
  airga_ctx ctx;
  SolveArgs<T> a;
  ReduceArgs red;
  KernelSet<T> ks;
  bool asm_path = false;
  unsigned grid = 0;
  int max_chain_q = 0;   // largest chain length over shifts
  std::vector<int> clen; // host copy
  size_t flags_off = 0;  // offset of the host flag arrays in the pinned buffer
};

// Profiled solves only: count the systems and shifts the next iteration's
// row kernels will sweep (synchronises; kernel durations are unaffected).
template <typename T>
static airga_status count_work(Plan<T>& P, Timer& tm, bool in_iteration) {
  if (!tm.on) return AIRGA_OK;
  const int B = P.a.B, m = P.a.m;
  std::vector<int32_t> act(B);
  AIRGA_HIP(hipMemcpyAsync(act.data(), P.a.sys.active, 4 * B, hipMemcpyDeviceToHost, P.ctx->stream));
  AIRGA_HIP(hipStreamSynchronize(P.ctx->stream));
  int64_t sys = 0, shifts = 0, chain_shifts = 0;
  for (int k = 0; k < P.a.nshift; ++k) {
    int any = 0;
    for (int c = 0; c < m; ++c) any |= act[k * m + c];
    for (int c = 0; c < m; ++c) sys += act[k * m + c] != 0;
    if (any && P.clen[k] > 0) shifts += 1;
    if (any) chain_shifts += P.clen[k] > 1 ? P.clen[k] - 1 : 0;
  }
  KernelTimes& t = P.ctx->times;
  const int id = in_iteration ? K_UPDATE_PREC : K_INIT_PREC;
  if (in_iteration) t.sys_passes[K_DIR_SPMV] += sys;
  t.sys_passes[id] += sys;
  t.shift_passes[id] += shifts;
  t.shift_passes[K_CHAIN] += chain_shifts;
  return AIRGA_OK;
}

template <typename T>
static airga_status iteration(Plan<T>& P, Timer& tm, int par) {
  hipStream_t st = P.ctx->stream;
  const unsigned B = (unsigned)P.a.B;
  AIRGA_TRY(count_work(P, tm, true));
  if (P.asm_path)
    TIMED(K_DIR_SPMV, P.ks.dir_asm<<<P.grid, 256, 0, st>>>(P.a, par));
  else
    TIMED(K_DIR_SPMV, P.ks.dir<<<P.grid, 256, 0, st>>>(P.a, par));
  TIMED(K_REDUCE, k_reduce<<<B, 256, 0, st>>>(P.red, RM_PW));
  TIMED(K_UPDATE_PREC, P.ks.upd<<<P.grid, 256, 0, st>>>(P.a, par));
  for (int q = 1; q < P.max_chain_q; ++q)
    TIMED(K_CHAIN, P.ks.chain<<<P.grid, 256, 0, st>>>(P.a, par, q, 0));
  TIMED(K_REDUCE, k_reduce<<<B, 256, 0, st>>>(P.red, RM_ITER));
  return AIRGA_OK;
}

template <typename T>
static airga_status start_inner(Plan<T>& P, Timer& tm, int rel) {
  hipStream_t st = P.ctx->stream;
  AIRGA_TRY(count_work(P, tm, false));
  TIMED(K_INIT_PREC, P.ks.init<<<P.grid, 256, 0, st>>>(P.a, 0));
  for (int q = 1; q < P.max_chain_q; ++q)
    TIMED(K_CHAIN, P.ks.chain<<<P.grid, 256, 0, st>>>(P.a, 0, q, 1));
  TIMED(K_REDUCE, k_reduce<<<(unsigned)P.a.B, 256, 0, st>>>(P.red, rel ? RM_INIT_REL : RM_INIT_ABS));
  return AIRGA_OK;
}

// Run CG iterations until no system is active (or the host-side cap).
template <typename T>
static airga_status iterate(Plan<T>& P, Timer& tm, const airga_pcg_opts& o, int32_t* h_active,
                            const int32_t* d_active) {
  hipStream_t st = P.ctx->stream;
  const int B = P.a.B;
  int k = o.poll_every < 2 ? 2 : o.poll_every;
  k += k & 1;
  hipGraphExec_t exec = nullptr;
  hipGraph_t graph = nullptr;
  const bool use_graph = o.use_graph && !o.profile;
  if (use_graph) {
    AIRGA_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    airga_status s = AIRGA_OK;
    for (int j = 0; j < k && s == AIRGA_OK; ++j) s = iteration(P, tm, j & 1);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(st, &g);
    if (s != AIRGA_OK) {
      if (g) (void)hipGraphDestroy(g);
      return s;
    }
    if (e != hipSuccess) return fail(AIRGA_EHIP, "graph capture failed: %s", hipGetErrorString(e));
    graph = g;
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
      (void)hipGraphDestroy(graph);
      return fail(AIRGA_EHIP, "graph instantiation failed: %s", hipGetErrorString(e));
    }
  }
  airga_status result = AIRGA_OK;
  // Hard stop: every system is capped by max_iter, so max_iter/k + 2 rounds suffice.
  const int64_t rounds = (int64_t)o.max_iter / k + 2;
  for (int64_t round = 0; round < rounds; ++round) {
    if (use_graph) {
      hipError_t e = hipGraphLaunch(exec, st);
      if (e != hipSuccess) {
        result = fail(AIRGA_EHIP, "hipGraphLaunch: %s", hipGetErrorString(e));
        break;
      }
    } else {
      for (int j = 0; j < k; ++j) {
        result = iteration(P, tm, j & 1);
        if (result != AIRGA_OK) break;
      }
      if (result != AIRGA_OK) break;
    }
    hipError_t e = hipMemcpyAsync(h_active, d_active, sizeof(int32_t) * B, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
      result = fail(AIRGA_EHIP, "polling the active systems: %s", hipGetErrorString(e));
      break;
    }
    result = tm.flush();
    if (result != AIRGA_OK) break;
    int any = 0;
    for (int b = 0; b < B; ++b) any |= h_active[b];
    if (!any) break;
  }
  if (exec) (void)hipGraphExecDestroy(exec);
  if (graph) (void)hipGraphDestroy(graph);
  return result;
}

// Workspace: vectors, partials, per-system state, per-shift data.
struct Layout {
  size_t vec_bytes, part_bytes, sys_bytes, shift_bytes;
};

template <typename T>
static airga_status prepare(airga_ctx ctx, Plan<T>& P, int32_t nshift, const double* shifts,
                            const airga_prec* precs, int32_t m, double* X, int64_t ldx,
                            const airga_pcg_opts& o, int rows) {
  const Pencil& pen = ctx->pen;
  hipStream_t st = ctx->stream;
  const int B = nshift * m;
  const int64_t ld = pen.n_pad();
  const int G = (int)((pen.n_slices + rows - 1) / rows);
  P.ctx = ctx;
  // chains
  std::vector<std::vector<airga_prec>> chains(nshift);
  int maxc = 1;
  for (int k = 0; k < nshift; ++k) {
    if (precs && precs[k]) {
      std::vector<airga_prec> ch;
      AIRGA_TRY(prec_chain(precs[k], &ch));
      chains[k].assign(ch.rbegin(), ch.rend());  // oldest first
      maxc = (int)chains[k].size() > maxc ? (int)chains[k].size() : maxc;
    }
  }
  // memory
  const size_t vec_bytes = sizeof(T) * (size_t)KINDS * B * ld;
  AIRGA_TRY(ctx->ws_vec.reserve(vec_bytes));
  AIRGA_TRY(ctx->ws_partial.reserve(sizeof(double) * (size_t)B * G * kSlots));
  const size_t sys_bytes = (7 * sizeof(double) + 7 * sizeof(int32_t)) * (size_t)B + 256;
  AIRGA_TRY(ctx->ws_sys.reserve(sys_bytes));
  const size_t shift_bytes = 4 * sizeof(double) * nshift + sizeof(void*) * (size_t)nshift * maxc +
                             sizeof(int32_t) * nshift + 256;
  AIRGA_TRY(ctx->ws_shift.reserve(shift_bytes));
  P.flags_off = (shift_bytes + 4095) & ~(size_t)4095;
  AIRGA_TRY(ensure_pinned(ctx, P.flags_off + sizeof(int32_t) * 8 * (size_t)B + 64));
  // per-system state
  char* sb = ctx->ws_sys.as<char>();
  SysDev S;
  double* d = reinterpret_cast<double*>(sb);
  S.rz = d; S.pw = d + B; S.alpha = d + 2 * B; S.beta = d + 3 * B; S.tol2 = d + 4 * B;
  S.ff = d + 5 * B; S.relres = d + 6 * B;
  int32_t* iv = reinterpret_cast<int32_t*>(d + 7 * B);
  S.active = iv; S.first = iv + B; S.istat = iv + 2 * B; S.status = iv + 3 * B;
  S.iters = iv + 4 * B; S.sweeps = iv + 5 * B; S.outer = iv + 6 * B;
  // per-shift block, staged in pinned memory and copied once
  char* hp = static_cast<char*>(ctx->host_pinned);
  double* h_ca64 = reinterpret_cast<double*>(hp);
  double* h_cb64 = h_ca64 + nshift;
  T* h_ca = reinterpret_cast<T*>(h_cb64 + nshift);
  T* h_cb = h_ca + nshift;
  const size_t off_fac = 4 * sizeof(double) * nshift;
  const T** h_fac = reinterpret_cast<const T**>(hp + off_fac);
  int32_t* h_clen = reinterpret_cast<int32_t*>(hp + off_fac + sizeof(void*) * (size_t)nshift * maxc);
  P.clen.assign(nshift, 0);
  P.max_chain_q = 0;
  for (int k = 0; k < nshift; ++k) {
    double a, b;
    shift_coeffs(pen, shifts[k], &a, &b);
    h_ca64[k] = a;
    h_cb64[k] = b;
    h_ca[k] = (T)a;
    h_cb[k] = (T)b;
    const int L = (int)chains[k].size();
    h_clen[k] = L;
    P.clen[k] = L;
    P.max_chain_q = L > P.max_chain_q ? L : P.max_chain_q;
    for (int q = 0; q < maxc; ++q) {
      const T* v = nullptr;
      if (q < L) {
        if constexpr (sizeof(T) == 4) v = chains[k][q]->v32.as<float>();
        else v = chains[k][q]->v64.as<double>();
      }
      h_fac[(size_t)k * maxc + q] = v;
    }
  }
  AIRGA_HIP(hipMemcpyAsync(ctx->ws_shift.ptr, hp, shift_bytes - 256, hipMemcpyHostToDevice, st));
  char* sd = ctx->ws_shift.as<char>();
  // initial per-system state: all zero, then active/outer = 1, istat = MAXIT
  AIRGA_HIP(hipMemsetAsync(ctx->ws_sys.ptr, 0, sys_bytes, st));
  k_fill_i32<<<blocks_for(B, 256), 256, 0, st>>>(S.active, B, 1);
  k_fill_i32<<<blocks_for(B, 256), 256, 0, st>>>(S.outer, B, 1);
  k_fill_i32<<<blocks_for(B, 256), 256, 0, st>>>(S.istat, B, ST_MAXIT);
  k_fill_i32<<<blocks_for(B, 256), 256, 0, st>>>(S.status, B, ST_MAXIT);
  AIRGA_HIP(hipGetLastError());
  // wire the arguments
  SolveArgs<T>& A = P.a;
  A.pd = pen.dev();
  if constexpr (sizeof(T) == 4) {
    A.mv = pen.m32.as<float>();
    A.kv = pen.k32.as<float>();
  } else {
    A.mv = pen.m64.as<double>();
    A.kv = pen.k64.as<double>();
  }
  A.B = B;
  A.m = m;
  A.nshift = nshift;
  A.G = G;
  A.ld = ld;
  A.ws = ctx->ws_vec.as<T>();
  A.ca = reinterpret_cast<const T*>(sd + 2 * sizeof(double) * nshift);
  A.cb = A.ca + nshift;
  A.fac = reinterpret_cast<const T* const*>(sd + off_fac);
  A.clen = reinterpret_cast<const int32_t*>(sd + off_fac + sizeof(void*) * (size_t)nshift * maxc);
  A.maxc = maxc;
  A.partial = ctx->ws_partial.as<double>();
  A.sys = S;
  A.max_iter = o.max_iter;
  if constexpr (sizeof(T) == 8) {
    A.x = X;
    A.ldx = ldx;
  } else {
    A.x = A.ws + (int64_t)KX * B * ld;
    A.ldx = ld;
  }
  P.red.partial = A.partial;
  P.red.G = G;
  P.red.sys = S;
  P.red.max_iter = o.max_iter;
  P.red.max_sweeps = o.max_sweeps;
  P.red.mixed = o.mode == AIRGA_MODE_MIXED;
  P.grid = blocks_for(G, 4);
  P.ks = kernel_set<T>(wmax_class(pen.max_len), rows);
  return AIRGA_OK;
}

static int pick_rows(airga_ctx ctx, int B, int prec) {
  for (const auto& t : ctx->tuned)
    if (t.n_slices == ctx->pen.n_slices && t.batch == B && t.prec == prec) return t.rows;
  // default before tuning: more rows per wave for bigger problems
  return ctx->pen.n_slices >= 4096 ? 2 : 1;
}

// K(s) in stored (sliced-ELL) order, for the single-system float64 path.
__global__ void k_assemble_stored(PencilDev pd, int64_t stored, double a, double b,
                                  double* __restrict__ out) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < stored) out[i] = fma(a, pd.m64[i], b * pd.k64[i]);
}

static airga_status solve_fp64(airga_ctx ctx, int32_t nshift, const double* shifts,
                               const airga_prec* precs, int32_t m, const double* F, int64_t ldf,
                               double* X, int64_t ldx, const airga_pcg_opts& o,
                               airga_sys_stats* stats) {
  const Pencil& pen = ctx->pen;
  hipStream_t st = ctx->stream;
  const int B = nshift * m;
  Plan<double> P;
  const int rows = pick_rows(ctx, B, 8);
  AIRGA_TRY(prepare<double>(ctx, P, nshift, shifts, precs, m, X, ldx, o, rows));
  const double* ca64 = reinterpret_cast<const double*>(ctx->ws_shift.ptr);
  const double* cb64 = ca64 + nshift;
  // One system: store K(s) once (plain float64 CG on the assembled matrix).
  if (nshift == 1) {
    AIRGA_TRY(ctx->ws_asm.reserve(sizeof(double) * pen.nnz_stored));
    double a, b;
    shift_coeffs(pen, shifts[0], &a, &b);
    k_assemble_stored<<<blocks_for(pen.nnz_stored, 256), 256, 0, st>>>(pen.dev(), pen.nnz_stored,
                                                                       a, b, ctx->ws_asm.as<double>());
    AIRGA_HIP(hipGetLastError());
    P.a.mv = ctx->ws_asm.as<double>();
    P.a.kv = nullptr;
    P.asm_path = true;
  }
  P.red.tol2_rel = o.tol * o.tol;
  Timer tm{ctx, o.profile != 0, {}, {}};
  TIMED(K_IR_RESIDUAL, P.ks.resid<<<P.grid, 256, 0, st>>>(P.a, F, ldf, X, ldx, ca64, cb64,
                                                         o.x0_given ? 0 : 1, 0));
  TIMED(K_REDUCE, k_reduce<<<(unsigned)B, 256, 0, st>>>(P.red, RM_START));
  AIRGA_TRY(start_inner(P, tm, 0));
  int32_t* h_active = reinterpret_cast<int32_t*>(static_cast<char*>(ctx->host_pinned) + P.flags_off);
  AIRGA_TRY(iterate(P, tm, o, h_active, P.a.sys.active));
  // true residual of the final iterate
  TIMED(K_IR_RESIDUAL, P.ks.resid<<<P.grid, 256, 0, st>>>(P.a, F, ldf, X, ldx, ca64, cb64, 0, 0));
  TIMED(K_REDUCE, k_reduce<<<(unsigned)B, 256, 0, st>>>(P.red, RM_FINAL));
  AIRGA_TRY(tm.flush());
  if (stats) {
    std::vector<int32_t> ist(B), its(B);
    std::vector<double> rel(B);
    AIRGA_HIP(hipMemcpyAsync(ist.data(), P.a.sys.istat, 4 * B, hipMemcpyDeviceToHost, st));
    AIRGA_HIP(hipMemcpyAsync(its.data(), P.a.sys.iters, 4 * B, hipMemcpyDeviceToHost, st));
    AIRGA_HIP(hipMemcpyAsync(rel.data(), P.a.sys.relres, 8 * B, hipMemcpyDeviceToHost, st));
    AIRGA_HIP(hipStreamSynchronize(st));
    for (int b = 0; b < B; ++b) {
      stats[b].status = ist[b];
      stats[b].iters = its[b];
      stats[b].sweeps = 1;
      stats[b].reserved = 0;
      stats[b].relres = rel[b];
    }
  } else {
    AIRGA_HIP(hipStreamSynchronize(st));
  }
  return AIRGA_OK;
}

static airga_status solve_mixed(airga_ctx ctx, int32_t nshift, const double* shifts,
                                const airga_prec* precs, int32_t m, const double* F, int64_t ldf,
                                double* X, int64_t ldx, const airga_pcg_opts& o,
                                airga_sys_stats* stats) {
  const Pencil& pen = ctx->pen;
  hipStream_t st = ctx->stream;
  const int B = nshift * m;
  Plan<float> P;
  const int rows = pick_rows(ctx, B, 4);
  AIRGA_TRY(prepare<float>(ctx, P, nshift, shifts, precs, m, X, ldx, o, rows));
  const double* ca64 = reinterpret_cast<const double*>(ctx->ws_shift.ptr);
  const double* cb64 = ca64 + nshift;
  P.red.tol2_rel = o.inner_tol * o.inner_tol;
  P.red.tol2_abs = o.tol * o.tol;
  Timer tm{ctx, o.profile != 0, {}, {}};
  int32_t* h_active = reinterpret_cast<int32_t*>(static_cast<char*>(ctx->host_pinned) + P.flags_off);
  int32_t* h_outer = h_active + B;
  // sweep 0 residual
  TIMED(K_IR_RESIDUAL, P.ks.resid<<<P.grid, 256, 0, st>>>(P.a, F, ldf, X, ldx, ca64, cb64,
                                                         o.x0_given ? 0 : 1, 1));
  // inner state starts inactive; RM_OUTER activates the systems to refine
  k_fill_i32<<<blocks_for(B, 256), 256, 0, st>>>(P.a.sys.active, B, 0);
  AIRGA_HIP(hipGetLastError());
  TIMED(K_REDUCE, k_reduce<<<(unsigned)B, 256, 0, st>>>(P.red, RM_OUTER));
  for (int sweep = 0; sweep <= o.max_sweeps; ++sweep) {
    AIRGA_HIP(hipMemcpyAsync(h_outer, P.a.sys.outer, 4 * B, hipMemcpyDeviceToHost, st));
    AIRGA_HIP(hipStreamSynchronize(st));
    int any = 0;
    for (int b = 0; b < B; ++b) any |= h_outer[b];
    if (!any) break;
    AIRGA_TRY(start_inner(P, tm, 1));
    AIRGA_TRY(iterate(P, tm, o, h_active, P.a.sys.active));
    TIMED(K_IR_UPDATE,
          (k_ir_update<<<dim3(blocks_for(pen.n, 256), (unsigned)B), 256, 0, st>>>(P.a, X, ldx)));
    TIMED(K_IR_RESIDUAL, P.ks.resid<<<P.grid, 256, 0, st>>>(P.a, F, ldf, X, ldx, ca64, cb64, 0, 1));
    TIMED(K_REDUCE, k_reduce<<<(unsigned)B, 256, 0, st>>>(P.red, RM_OUTER));
  }
  AIRGA_TRY(tm.flush());
  std::vector<int32_t> sta(B), its(B), swp(B), out(B);
  std::vector<double> rel(B);
  AIRGA_HIP(hipMemcpyAsync(sta.data(), P.a.sys.status, 4 * B, hipMemcpyDeviceToHost, st));
  AIRGA_HIP(hipMemcpyAsync(its.data(), P.a.sys.iters, 4 * B, hipMemcpyDeviceToHost, st));
  AIRGA_HIP(hipMemcpyAsync(swp.data(), P.a.sys.sweeps, 4 * B, hipMemcpyDeviceToHost, st));
  AIRGA_HIP(hipMemcpyAsync(out.data(), P.a.sys.outer, 4 * B, hipMemcpyDeviceToHost, st));
  AIRGA_HIP(hipMemcpyAsync(rel.data(), P.a.sys.relres, 8 * B, hipMemcpyDeviceToHost, st));
  AIRGA_HIP(hipStreamSynchronize(st));
  if (stats) {
    for (int b = 0; b < B; ++b) {
      stats[b].status = out[b] ? ST_MAXIT : sta[b];
      stats[b].iters = its[b];
      stats[b].sweeps = swp[b];
      stats[b].reserved = 0;
      stats[b].relres = rel[b];
    }
  }
  return AIRGA_OK;
}

}  // namespace airga

using namespace airga;

extern "C" {

void airga_pcg_opts_default(airga_pcg_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof *o);
  o->tol = 1e-10;
  o->max_iter = 20000;
  o->mode = AIRGA_MODE_FP64;
  o->inner_tol = 1e-4;
  o->max_sweeps = 12;
  o->poll_every = 8;
  o->x0_given = 0;
  o->use_graph = 1;
  o->profile = 0;
}

airga_status airga_pcg_solve(airga_ctx ctx, int32_t nshift, const double* shifts,
                             const airga_prec* precs, int32_t m, const double* F, int64_t ldf,
                             double* X, int64_t ldx, const airga_pcg_opts* opts,
                             airga_sys_stats* stats) {
  AIRGA_TRY(check_pencil(ctx));
  const Pencil& pen = ctx->pen;
  if (nshift <= 0 || m <= 0) return fail(AIRGA_EINVAL, "nshift and m must be positive");
  if ((int64_t)nshift * m > 65535) return fail(AIRGA_EUNSUPPORTED, "more than 65535 systems");
  if (!shifts || !F || !X) return fail(AIRGA_EINVAL, "null shifts, F or X");
  if (ldf < pen.n || ldx < pen.n) return fail(AIRGA_EINVAL, "leading dimension < n");
  for (int k = 0; k < nshift; ++k) {
    if (!std::isfinite(shifts[k]) || !(shifts[k] > 0))
      return fail(AIRGA_EINVAL, "shift %d must be finite and > 0", k);
    if (precs && precs[k]) {
      if (precs[k]->ctx != ctx) return fail(AIRGA_EINVAL, "preconditioner %d from another context", k);
      if (precs[k]->generation != pen.generation)
        return fail(AIRGA_ESTATE, "preconditioner %d was built for an earlier pencil", k);
    }
  }
  airga_pcg_opts o;
  airga_pcg_opts_default(&o);
  if (opts) o = *opts;
  if (!(o.tol >= 0) || o.max_iter < 0 || (o.mode != AIRGA_MODE_FP64 && o.mode != AIRGA_MODE_MIXED))
    return fail(AIRGA_EINVAL, "bad solver options");
  if (o.mode == AIRGA_MODE_MIXED && (!(o.inner_tol > 0 && o.inner_tol < 1) || o.max_sweeps < 0))
    return fail(AIRGA_EINVAL, "bad refinement options");
  if (o.profile) ctx->times.clear();
  if (o.mode == AIRGA_MODE_FP64)
    return solve_fp64(ctx, nshift, shifts, precs, m, F, ldf, X, ldx, o, stats);
  return solve_mixed(ctx, nshift, shifts, precs, m, F, ldf, X, ldx, o, stats);
}

int32_t airga_kernel_count(void) { return K_COUNT; }

const char* airga_kernel_name(int32_t id) {
  static const char* names[K_COUNT] = {"dir_spmv", "update_prec", "init_prec", "chain",
                                       "reduce", "ir_residual", "ir_update"};
  return id >= 0 && id < K_COUNT ? names[id] : "";
}

airga_status airga_get_kernel_times(airga_ctx ctx, int32_t count, int64_t* launches,
                                    double* total_ms) {
  AIRGA_TRY(check_ctx(ctx));
  if (count < 0 || (count > 0 && (!launches || !total_ms))) return fail(AIRGA_EINVAL, "bad arrays");
  for (int i = 0; i < count && i < K_COUNT; ++i) {
    launches[i] = ctx->times.launches[i];
    total_ms[i] = ctx->times.ms[i];
  }
  return AIRGA_OK;
}

airga_status airga_get_kernel_work(airga_ctx ctx, int32_t count, int64_t* sys_passes,
                                   int64_t* shift_passes) {
  AIRGA_TRY(check_ctx(ctx));
  if (count < 0 || (count > 0 && (!sys_passes || !shift_passes)))
    return fail(AIRGA_EINVAL, "bad arrays");
  for (int i = 0; i < count && i < K_COUNT; ++i) {
    sys_passes[i] = ctx->times.sys_passes[i];
    shift_passes[i] = ctx->times.shift_passes[i];
  }
  return AIRGA_OK;
}

}  // extern "C"
