// Row kernels of the batched PCG (templates; instantiated per precision in
// pcg_sets_f32.hip and pcg_sets_f64.hip).
//
// Data layout.  Matrices are in the pencil's sliced-ELL form (64-row slices,
// one row per lane).  Every per-system vector is contiguous (length n_pad),
// kind-major: vec(kind, b) = ws + (kind * B + b) * n_pad; rows past n are
// padding and hold zeros, so the row kernels need no per-lane bounds test.
// A wavefront owns R consecutive slices; it loads their column indices and
// M, K (or factor) values once into registers and then sweeps the active
// systems in groups of U, issuing every load of a group before its first
// store, so the pencil is read once per kernel for the whole batch and each
// wavefront keeps U systems' traffic in flight.  The shifted matrix is never
// stored: K(s_k) p = a_k (M p) + b_k (K p).
//
// One CG iteration is two row kernels and two tiny reductions:
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
// symmetry of the preconditioner (a fixed-pattern right SPAI and every update
// chain are non-symmetric); for a symmetric preconditioner it is the
// classical CG ratio.
#pragma once

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
  int32_t* nact;    // number of systems with active set (for the host's polling)
  int32_t* handed;  // mixed mode: 1 = left the float32 sweeps for the float64 finish
};

// Storage of preconditioner values: the precision of the solve (float32
// for the inner solves of mixed precision, float64 otherwise).
template <typename T> using fac_t = T;

template <typename T>
struct SolveArgs {
  PencilDev pd;
  const T* mv;               // M values in T (or the assembled K(s) when kv == nullptr)
  const T* kv;               // K values in T
  int32_t B, m, nshift, G;
  int64_t ld;                // n_pad
  T* ws;                     // vector workspace (the iterate x is kind KX)
  const T* ca;               // per shift a_k = s_k^2 + alpha s_k
  const T* cb;               // per shift b_k = 1 + beta s_k
  const fac_t<T>* const* fac;  // per shift [maxc] factor values, fac[sh * maxc + q], oldest first
  const int32_t* clen;       // per shift number of applied factors
  int32_t maxc;
  double* partial;           // [kSlots][B][GP], slot-major
  int32_t GP;                // partial columns per system (blocks if blk, else wavefronts)
  int32_t blk;               // 1: the 4 wavefronts of a block pre-sum their partials in LDS
  int32_t xz;                // 1: each inner solve starts from x = 0, which is never stored:
                             //    its first update writes x = alpha p without reading x
  int32_t bw;                // pencil bandwidth max |c - r| (banded kernels: <= 64)
  int32_t stage_off;         // doubles of dynamic LDS before the banded staging area
  const int32_t* fmap;       // column of F for system b (nullptr: b % m)
  SysDev sys;
  __device__ __forceinline__ T* vec(int kind, int b) const {
    return ws + ((int64_t)kind * B + b) * ld;
  }
  __device__ __forceinline__ double& slot(int q, int b, int g) const {
    return partial[((int64_t)q * B + b) * GP + g];
  }
  // Wave partial of slot q for system b (lane 0 holds the wave total).
  __device__ __forceinline__ void put(double* lds, int q, int b, int wg, int lane, double v) const {
    if (lane != 0) return;
    if (blk) lds[((int)(threadIdx.x >> 6) * B + b) * kSlots + q] = v;
    else slot(q, b, wg) = v;
  }
};

// Bytes of LDS a row kernel needs for the block pre-sum.
inline size_t partial_lds_bytes(int B) { return sizeof(double) * 4 * kSlots * (size_t)B; }

// End of a row kernel in block mode: every (system, slot) the kernel wrote,
// as chosen by sel(b), gets the sum of its 4 wave partials in wave order.
template <typename T, typename Sel>
__device__ __forceinline__ void flush_partials(const SolveArgs<T>& A, const double* lds, int q0,
                                               int q1, Sel sel) {
  if (!A.blk) return;
  __syncthreads();
  const int nq = q1 - q0 + 1;
  for (int idx = threadIdx.x; idx < A.B * nq; idx += blockDim.x) {
    const int b = idx / nq, q = q0 + idx % nq;
    if (!sel(b)) continue;
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < 4; ++w) s += lds[(w * A.B + b) * kSlots + q];
    A.slot(q, b, blockIdx.x) = s;
  }
}

// Buffer written by chain position q (0 = the fused first factor) for a chain
// of L factors: the last one lands in KZ, earlier ones alternate with KT.
__device__ __forceinline__ int chain_dst(int q, int L) { return ((L - 1 - q) & 1) ? KT : KZ; }

// Row set of one wavefront: R consecutive slices.  Slice data are uniform
// across the wavefront (scalar loads).  Entries past a slice's width get the
// row itself as column and value 0, so every loop runs WMAX entries with no
// test; EXACT marks pencils whose slices are all WMAX wide.  OFF8 (banded
// pencils) reads the 1-byte offsets column - row instead of 4-byte columns.
template <int WMAX, int R, bool EXACT>
struct Rows {
  int32_t col[R][WMAX];
  int32_t idx0[R];
  int32_t w[R];
  bool valid[R];
  int64_t row[R];
  template <bool OFF8 = false>
  __device__ __forceinline__ void load(const PencilDev& pd, int wg, int lane) {
#pragma unroll
    for (int i = 0; i < R; ++i) {
      const int s = wg * R + i;
      valid[i] = s < pd.n_slices;
      // a slice past the end aliases row `lane` of slice 0: its loads stay in
      // bounds and its results are never stored
      row[i] = valid[i] ? (int64_t)s * kSlice + lane : lane;
      w[i] = 0;
      idx0[i] = 0;
      if (valid[i]) {
        const int sp0 = pd.slice_ptr[s];
        w[i] = EXACT ? WMAX : (pd.slice_ptr[s + 1] - sp0) / kSlice;
        idx0[i] = sp0 + lane;
      }
#pragma unroll
      for (int k = 0; k < WMAX; ++k) {
        const bool in = valid[i] && (EXACT || k < w[i]);
        if constexpr (OFF8)
          col[i][k] = (int32_t)row[i] + (in ? (int32_t)pd.coff[idx0[i] + k * kSlice] : 0);
        else
          col[i][k] = in ? pd.col[idx0[i] + k * kSlice] : (int32_t)row[i];
      }
    }
  }
  template <typename T>
  __device__ __forceinline__ void values(const T* __restrict__ v, T (&out)[R][WMAX]) const {
#pragma unroll
    for (int i = 0; i < R; ++i)
#pragma unroll
      for (int k = 0; k < WMAX; ++k)
        out[i][k] = (valid[i] && (EXACT || k < w[i])) ? v[idx0[i] + k * kSlice] : T(0);
  }
  // factor values in their storage type, widened to T
  template <typename TS, typename T>
  __device__ __forceinline__ void factor(const TS* __restrict__ v, T (&out)[R][WMAX]) const {
#pragma unroll
    for (int i = 0; i < R; ++i)
#pragma unroll
      for (int k = 0; k < WMAX; ++k)
        out[i][k] = (valid[i] && (EXACT || k < w[i])) ? v[idx0[i] + k * kSlice] : T(0);
  }
};

// Sweep of the systems whose flag is set, in ascending order, U at a time
// (bs[u] = -1 past the last one).  The flags are read 64 at a time into a
// wave-uniform bit mask, so the sweep needs no compacted list.
struct FlagSweep {
  const int32_t* __restrict__ flag;
  int B, c;
  uint64_t mask;
  bool pre;    // f0 holds the first chunk's flag of this lane
  int32_t f0;
  __device__ FlagSweep(const int32_t* f, int nb) : flag(f), B(nb), c(-64), mask(0), pre(false), f0(0) {}
  // Loads the first chunk's flags at once, so their latency overlaps the
  // kernel's set-up loads instead of following them.
  __device__ FlagSweep(const int32_t* f, int nb, int lane)
      : flag(f), B(nb), c(-64), mask(0), pre(true), f0(lane < nb ? f[lane] : 0) {}
  template <int U>
  __device__ __forceinline__ bool next(int (&bs)[U], int lane) {
    while (mask == 0) {
      c += 64;
      if (c >= B) return false;
      if (pre && c == 0) {
        mask = __ballot(f0 != 0);
      } else {
        const int i = c + lane;
        mask = __ballot(i < B && flag[i] != 0);
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (mask) {
        bs[u] = c + __builtin_ctzll(mask);
        mask &= mask - 1;
      } else {
        bs[u] = -1;
      }
    }
    return true;
  }
};

// FlagSweep's systems grouped by column: within each chunk of 64 systems,
// those with b % m == 0 first, then b % m == 1, and so on (ascending within a
// column).  Systems are numbered shift-major (b = shift * m + column), so a
// wavefront meets each right-hand-side column once per chunk and can keep
// its values.  m = 1 gives FlagSweep's order.
struct ColumnSweep {
  const int32_t* __restrict__ flag;
  int B, m, c, col;
  uint64_t chunk, mask;
  __device__ ColumnSweep(const int32_t* f, int nb, int mcols)
      : flag(f), B(nb), m(mcols), c(-64), col(0), chunk(0), mask(0) {}
  template <int U>
  __device__ __forceinline__ bool next(int (&bs)[U], int lane) {
    while (mask == 0) {
      if (chunk != 0 && ++col < m) {
        mask = chunk & __ballot(((c + lane) % m) == col);
        continue;
      }
      c += 64;
      if (c >= B) return false;
      const int i = c + lane;
      chunk = __ballot(i < B && flag[i] != 0);
      col = 0;
      mask = chunk & __ballot((i % m) == 0);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (mask) {
        bs[u] = c + __builtin_ctzll(mask);
        mask &= mask - 1;
      } else {
        bs[u] = -1;
      }
    }
    return true;
  }
};

// Banded staging (pencils of bandwidth <= 64).  A wavefront's R slices and
// the bw rows on each side of them are staged in LDS, one (R + 2) x 64
// window per system of the group, so the column entries of a row are read
// from LDS instead of being gathered from global memory.  Window row j holds
// global row base - 64 + 64 j + lane; with bandwidth <= 64 every column of an
// own row lies in the window.  Loads are issued for every lane (a lane whose
// row is not needed reads an own row instead, already in cache) and the
// value is dropped by a select, so the staging loads have no branches.
template <int WMAX, int R>
struct Window {
  int off[R][WMAX];  // window index of each entry's column
  int64_t base;      // first own row
  int64_t src[R + 2];  // row each lane loads for window row j
  bool keep[R + 2];    // lane's window row j is needed
  template <bool EXACT>
  __device__ __forceinline__ void init(const Rows<WMAX, R, EXACT>& rows, int wg, int n_slices,
                                       int bw, int lane) {
    base = (int64_t)wg * R * kSlice;
    const bool pre = wg > 0 && wg * R <= n_slices;
    const bool post = (int64_t)wg * R + R < n_slices;
#pragma unroll
    for (int i = 0; i < R; ++i)
#pragma unroll
      for (int k = 0; k < WMAX; ++k)
        off[i][k] = rows.valid[i] ? (int)(rows.col[i][k] - base) + kSlice : (i + 1) * kSlice + lane;
#pragma unroll
    for (int j = 0; j < R + 2; ++j) {
      const int64_t row = base - kSlice + (int64_t)j * kSlice + lane;
      if (j == 0) keep[j] = pre && lane >= kSlice - bw;
      else if (j == R + 1) keep[j] = post && lane < bw;
      else keep[j] = rows.valid[j - 1];
      // fallback: an own row of the same lane (its first or last valid
      // slice), or row `lane` for a wavefront past the end
      const int64_t own = j == 0 ? rows.row[0] : j == R + 1 ? rows.row[R - 1] : rows.row[j - 1];
      src[j] = keep[j] ? row : own;
    }
  }
};

template <typename T, int R>
__device__ __forceinline__ T* window_base(double* lds, const SolveArgs<T>& A, int U) {
  return reinterpret_cast<T*>(lds + A.stage_off) + (int)(threadIdx.x >> 6) * U * (R + 2) * kSlice;
}
template <typename TS, int R>
__device__ __forceinline__ TS* window_base_as(double* lds, int stage_off, int U) {
  return reinterpret_cast<TS*>(lds + stage_off) + (int)(threadIdx.x >> 6) * U * (R + 2) * kSlice;
}

// Bytes of LDS for the windows of one block (4 wavefronts, U systems).
inline size_t window_lds_bytes(size_t elem, int R, int U) {
  return elem * 4 * (size_t)U * (R + 2) * kSlice;
}

// ---- A: direction update + shifted SpMV + (p, w) -------------------------
template <typename T, int WMAX, int R, int U, bool ASM, bool EXACT, bool BAND>
__global__ void __launch_bounds__(256) k_dir_spmv(SolveArgs<T> A, int par) {
  // nothing to do once every system has stopped (the rest of a replayed
  // round of iterations): return before the pencil's values are read.  The
  // count and the first 64 activity flags are fetched beside the slice data,
  // not ahead of it.
  const int32_t nact = sload(A.sys.nact);
  const int lane = threadIdx.x & 63;
  FlagSweep sweep(A.sys.active, A.B, lane);
  const int wg = uniform(blockIdx.x * 4 + (threadIdx.x >> 6));
  extern __shared__ double lds_part[];
  Rows<WMAX, R, EXACT> rows;
  rows.template load<BAND>(A.pd, wg, lane);
  if (nact == 0) return;
  T mv[R][WMAX], kv[R][WMAX];
  rows.values(A.mv, mv);
  if constexpr (!ASM) rows.values(A.kv, kv);
  Window<WMAX, R> win;
  T* stg = nullptr;
  if constexpr (BAND) {
    win.init(rows, wg, A.pd.n_slices, A.bw, lane);
    stg = window_base<T, R>(lds_part, A, U);
  }
  int bs[U];
  while (sweep.next(bs, lane)) {
    T pr[U][R], wr[U][R];
    if constexpr (BAND) {
      // p_new over the window of each system, then the SpMV from LDS
      T pw[U][R + 2];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int b = bs[u] >= 0 ? bs[u] : bs[0];
        const bool first = sload(A.sys.first + b) != 0;
        const T beta = first ? T(0) : (T)sload(A.sys.beta + b);
        const T* __restrict__ z = A.vec(KZ, b);
        const T* __restrict__ pin = A.vec(KP0 + par, b);
#pragma unroll
        for (int j = 0; j < R + 2; ++j) {
          const T po = pin[win.src[j]];
          pw[u][j] = fma(beta, first ? T(0) : po, z[win.src[j]]);
        }
      }
      __builtin_amdgcn_wave_barrier();
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int j = 0; j < R + 2; ++j)
          stg[(u * (R + 2) + j) * kSlice + lane] = win.keep[j] ? pw[u][j] : T(0);
      __builtin_amdgcn_wave_barrier();
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int b = bs[u] >= 0 ? bs[u] : bs[0];
        T ca = T(1), cb = T(0);
        if constexpr (!ASM) {
          ca = sload(A.ca + b / A.m);
          cb = sload(A.cb + b / A.m);
        }
        const T* w0 = stg + u * (R + 2) * kSlice;
#pragma unroll
        for (int i = 0; i < R; ++i) {
          T am = T(0), ak = T(0);
#pragma unroll
          for (int k = 0; k < WMAX; ++k) {
            const T pc = w0[win.off[i][k]];
            am = fma(mv[i][k], pc, am);
            if constexpr (!ASM) ak = fma(kv[i][k], pc, ak);
          }
          pr[u][i] = pw[u][i + 1];
          wr[u][i] = ASM ? am : fma(ca, am, cb * ak);
        }
      }
    } else {
      // compute phase: no branches, so every load of the group can be in
      // flight at once (a missing system aliases the group's first one)
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int b = bs[u] >= 0 ? bs[u] : bs[0];
        const bool first = sload(A.sys.first + b) != 0;
        const T beta = first ? T(0) : (T)sload(A.sys.beta + b);
        T ca = T(1), cb = T(0);
        if constexpr (!ASM) {
          ca = sload(A.ca + b / A.m);
          cb = sload(A.cb + b / A.m);
        }
        const T* __restrict__ z = A.vec(KZ, b);
        const T* __restrict__ pin = A.vec(KP0 + par, b);
#pragma unroll
        for (int i = 0; i < R; ++i) {
          T am = T(0), ak = T(0);
#pragma unroll
          for (int k = 0; k < WMAX; ++k) {
            const int c = rows.col[i][k];
            const T po = pin[c];
            const T pc = fma(beta, first ? T(0) : po, z[c]);
            am = fma(mv[i][k], pc, am);
            if constexpr (!ASM) ak = fma(kv[i][k], pc, ak);
          }
          const int64_t r = rows.row[i];
          const T po = pin[r];
          pr[u][i] = fma(beta, first ? T(0) : po, z[r]);
          wr[u][i] = ASM ? am : fma(ca, am, cb * ak);
        }
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int b = bs[u];
      if (b < 0) continue;
      T* __restrict__ pout = A.vec(KP0 + (par ^ 1), b);
      T* __restrict__ wv = A.vec(KW, b);
      T dot = T(0);
      // streaming stores: the vectors of all systems exceed the caches, so
      // each kernel's writes go out to HBM while it runs instead of being
      // left as dirty lines for the next kernel to write back
#pragma unroll
      for (int i = 0; i < R; ++i) {
        if (!rows.valid[i]) continue;
        const int64_t r = rows.row[i];
        __builtin_nontemporal_store(pr[u][i], &pout[r]);
        __builtin_nontemporal_store(wr[u][i], &wv[r]);
        dot = fma(pr[u][i], wr[u][i], dot);
      }
      dot = wave_total(dot);
      A.put(lds_part, 0, b, wg, lane, (double)dot);
    }
  }
  flush_partials(A, lds_part, 0, 0, [&](int b) { return A.sys.active[b] != 0; });
}

// ---- B: x/r update + first preconditioner factor + dots -------------------
// INIT: no update; r is R0 as produced by the residual kernel.
template <typename T, int WMAX, int R, int U, bool INIT, bool EXACT, bool BAND>
__global__ void __launch_bounds__(256) k_update_prec(SolveArgs<T> A, int par) {
  // nothing to do once every system has stopped (the rest of a replayed
  // round of iterations): return before the pencil's values are read.  The
  // count and the first 64 activity flags are fetched beside the slice data,
  // not ahead of it.
  const int32_t nact = sload(A.sys.nact);
  const int lane = threadIdx.x & 63;
  FlagSweep sweep(A.sys.active, A.B, lane);
  const int wg = uniform(blockIdx.x * 4 + (threadIdx.x >> 6));
  extern __shared__ double lds_part[];
  Rows<WMAX, R, EXACT> rows;
  rows.template load<BAND>(A.pd, wg, lane);
  if (nact == 0) return;
  Window<WMAX, R> win;
  T* stg = nullptr;
  if constexpr (BAND) {
    win.init(rows, wg, A.pd.n_slices, A.bw, lane);
    stg = window_base<T, R>(lds_part, A, U);
  }
  int bs[U];
  // First preconditioner factor of each group slot, kept in registers while
  // the systems swept through the slot belong to the same shift (systems
  // are numbered shift-major), so a shift's factor is read once per
  // wavefront, not once per system.  A missing preconditioner is an
  // identity factor supplied by the host.
  T pv[U][R][WMAX];
  int csh[U];
#pragma unroll
  for (int u = 0; u < U; ++u) csh[u] = -1;
  // The restart (INIT, banded, one system per group) moves 8 bytes per row
  // and system, so each system would otherwise wait out a full load latency:
  // the next system's r window is loaded before the current one is used.
  constexpr bool PIPE = INIT && BAND && U == 1;
  T rpre[R + 2];
  bool more = sweep.next(bs, lane);
  if constexpr (PIPE) {
    if (more) {
      const T* __restrict__ rin = A.vec(KR0, bs[0]);
#pragma unroll
      for (int j = 0; j < R + 2; ++j) rpre[j] = rin[win.src[j]];
    }
  }
  while (more) {
    int cb[U];
#pragma unroll
    for (int u = 0; u < U; ++u) cb[u] = bs[u];
    T rcur[R + 2];
    if constexpr (PIPE) {
#pragma unroll
      for (int j = 0; j < R + 2; ++j) rcur[j] = rpre[j];
    }
    more = sweep.next(bs, lane);
    if constexpr (PIPE) {
      if (more) {
        const T* __restrict__ rin = A.vec(KR0, bs[0]);
#pragma unroll
        for (int j = 0; j < R + 2; ++j) rpre[j] = rin[win.src[j]];
      }
    }
    // compute phase: no branches on lane data, so every load of the group
    // can be in flight at once (a missing system aliases the group's first
    // one)
    int Ls[U];
    T rn[U][R], tz[U][R], xn[U][R], wrr[U][R];
    if constexpr (BAND) {
      // r_new over the window of each system, then the factor from LDS
      T rw[U][R + 2], ww[U][R + 2];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int b = cb[u] >= 0 ? cb[u] : cb[0];
        const int sh = b / A.m;
        Ls[u] = sload(A.clen + sh);
        if (sh != csh[u]) {
          rows.factor(sload(A.fac + (int64_t)sh * A.maxc), pv[u]);
          csh[u] = sh;
        }
        const T al = INIT ? T(0) : (T)sload(A.sys.alpha + b);
        const T* __restrict__ rin = A.vec(INIT ? KR0 : KR0 + par, b);
        const T* __restrict__ wv = A.vec(KW, b);
        const T* __restrict__ pcur = A.vec(KP0 + (par ^ 1), b);
        const T* __restrict__ x = A.vec(KX, b);
#pragma unroll
        for (int j = 0; j < R + 2; ++j) {
          T rv;
          if constexpr (PIPE) rv = rcur[j];
          else rv = rin[win.src[j]];
          if constexpr (INIT) {
            ww[u][j] = T(0);
            rw[u][j] = rv;
          } else {
            ww[u][j] = wv[win.src[j]];
            rw[u][j] = fma(-al, ww[u][j], rv);
          }
        }
        if constexpr (!INIT) {
          // a zero start reads p again (in cache) instead of x, and drops it;
          // own-row x and p are read once, with streaming loads
          const bool x0 = A.xz && sload(A.sys.first + b) != 0;
          const T* __restrict__ xs = x0 ? pcur : x;
#pragma unroll
          for (int i = 0; i < R; ++i) {
            const int64_t r = rows.row[i];
            const T xv = __builtin_nontemporal_load(&xs[r]);
            xn[u][i] = fma(al, __builtin_nontemporal_load(&pcur[r]), x0 ? T(0) : xv);
          }
        }
      }
      __builtin_amdgcn_wave_barrier();
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int j = 0; j < R + 2; ++j)
          stg[(u * (R + 2) + j) * kSlice + lane] = win.keep[j] ? rw[u][j] : T(0);
      __builtin_amdgcn_wave_barrier();
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const T* w0 = stg + u * (R + 2) * kSlice;
#pragma unroll
        for (int i = 0; i < R; ++i) {
          T t = T(0);
#pragma unroll
          for (int k = 0; k < WMAX; ++k) t = fma(pv[u][i][k], w0[win.off[i][k]], t);
          rn[u][i] = rw[u][i + 1];
          tz[u][i] = t;
          wrr[u][i] = ww[u][i + 1];
        }
      }
    } else {
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int b = cb[u] >= 0 ? cb[u] : cb[0];
        const int sh = b / A.m;
        Ls[u] = sload(A.clen + sh);
        if (sh != csh[u]) {
          rows.factor(sload(A.fac + (int64_t)sh * A.maxc), pv[u]);
          csh[u] = sh;
        }
        const T al = INIT ? T(0) : (T)sload(A.sys.alpha + b);
        const T* __restrict__ rin = A.vec(INIT ? KR0 : KR0 + par, b);
        const T* __restrict__ wv = A.vec(KW, b);
        const T* __restrict__ pcur = A.vec(KP0 + (par ^ 1), b);
        const T* __restrict__ x = A.vec(KX, b);
        // a zero start reads p again (in cache) instead of x, and drops it
        const bool x0 = !INIT && A.xz && sload(A.sys.first + b) != 0;
        const T* __restrict__ xs = x0 ? pcur : x;
#pragma unroll
        for (int i = 0; i < R; ++i) {
          const int64_t r = rows.row[i];
          T wr = T(0), v;
          if constexpr (INIT) {
            v = rin[r];
          } else {
            wr = wv[r];
            v = fma(-al, wr, rin[r]);
            const T xv = __builtin_nontemporal_load(&xs[r]);
            xn[u][i] = fma(al, __builtin_nontemporal_load(&pcur[r]), x0 ? T(0) : xv);
          }
          T t = T(0);
#pragma unroll
          for (int k = 0; k < WMAX; ++k) {
            const int cc = rows.col[i][k];
            const T rc = INIT ? rin[cc] : fma(-al, wv[cc], rin[cc]);
            t = fma(pv[u][i][k], rc, t);
          }
          rn[u][i] = v;
          tz[u][i] = t;
          wrr[u][i] = wr;
        }
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int b = cb[u];
      if (b < 0) continue;
      const int L = Ls[u];
      T* __restrict__ rout = A.vec(KR0 + (par ^ 1), b);
      T* __restrict__ zo = A.vec(chain_dst(0, L), b);
      T* __restrict__ x = A.vec(KX, b);
      T rr = T(0), rz = T(0), zw = T(0);
#pragma unroll
      for (int i = 0; i < R; ++i) {
        if (!rows.valid[i]) continue;
        const int64_t r = rows.row[i];
        // streaming stores, as in the direction kernel
        if constexpr (!INIT) {
          __builtin_nontemporal_store(xn[u][i], &x[r]);
          __builtin_nontemporal_store(rn[u][i], &rout[r]);
        }
        __builtin_nontemporal_store(tz[u][i], &zo[r]);
        rr = fma(rn[u][i], rn[u][i], rr);
        rz = fma(rn[u][i], tz[u][i], rz);
        zw = fma(tz[u][i], wrr[u][i], zw);
      }
      rr = wave_total(rr);
      rz = wave_total(rz);
      zw = wave_total(zw);
      A.put(lds_part, 1, b, wg, lane, (double)rr);
      A.put(lds_part, 2, b, wg, lane, L > 1 ? 0.0 : (double)rz);
      A.put(lds_part, 3, b, wg, lane, L > 1 ? 0.0 : (double)zw);
    }
  }
  flush_partials(A, lds_part, 1, 3, [&](int b) { return A.sys.active[b] != 0; });
}

// ---- chain factor q >= 1 (Q_{q+1} of the update chain) ---------------------
template <typename T, int WMAX, int R, bool EXACT>
__global__ void __launch_bounds__(256) k_chain(SolveArgs<T> A, int par, int q, int init) {
  // nothing to do once every system has stopped (the rest of a replayed
  // round of iterations): return before touching the pencil
  if (sload(A.sys.nact) == 0) return;
  const int lane = threadIdx.x & 63;
  const int wg = uniform(blockIdx.x * 4 + (threadIdx.x >> 6));
  extern __shared__ double lds_part[];
  Rows<WMAX, R, EXACT> rows;
  rows.load(A.pd, wg, lane);
  const int rk = init ? KR0 : KR0 + (par ^ 1);
  FlagSweep sweep(A.sys.active, A.B);
  int bs[1];
  int loaded_sh = -1;
  T fv[R][WMAX];
  while (sweep.next(bs, lane)) {
    const int b = bs[0];
    const int sh = b / A.m;
    const int L = sload(A.clen + sh);
    if (L <= q) continue;
    if (sh != loaded_sh) {
      rows.factor(sload(A.fac + (int64_t)sh * A.maxc + q), fv);
      loaded_sh = sh;
    }
    const T* __restrict__ src = A.vec(chain_dst(q - 1, L), b);
    T* __restrict__ dst = A.vec(chain_dst(q, L), b);
    const bool last = q == L - 1;
    const T* __restrict__ rv = A.vec(rk, b);
    const T* __restrict__ wv = A.vec(KW, b);
    T rz = T(0), zw = T(0);
#pragma unroll
    for (int i = 0; i < R; ++i) {
      if (!rows.valid[i]) continue;
      const int64_t r = rows.row[i];
      T t = T(0);
#pragma unroll
      for (int k = 0; k < WMAX; ++k) t = fma(fv[i][k], src[rows.col[i][k]], t);
      dst[r] = t;
      if (last) {
        rz = fma(rv[r], t, rz);
        if (!init) zw = fma(t, wv[r], zw);
      }
    }
    if (last) {
      rz = wave_total(rz);
      zw = wave_total(zw);
      A.put(lds_part, 2, b, wg, lane, (double)rz);
      A.put(lds_part, 3, b, wg, lane, (double)zw);
    }
  }
  flush_partials(A, lds_part, 2, 3,
                 [&](int b) { return A.sys.active[b] != 0 && A.clen[b / A.m] == q + 1; });
}

// ---- float64 residual r = F - K(s) X (and |F|^2), output in TO -------------
//   xread: 1 = use X, 0 = take X as 0;   xzero: write zeros into X;
//   kx:    0 = leave the iterate, 1 = zero it, 2 = copy X into it.
// Rows past n write zeros.  Systems: those with outer[b] set.  X and F have
// n rows only, so every index into them is clamped to n - 1 and the value
// dropped by a select where the row is past n.
template <typename TO, int WMAX, int R, int U, bool EXACT, bool BAND>
__global__ void __launch_bounds__(256) k_residual(SolveArgs<TO> A, const double* __restrict__ F,
                                                  int64_t ldf, double* __restrict__ X,
                                                  int64_t ldX, const double* __restrict__ ca64,
                                                  const double* __restrict__ cb64, int xread,
                                                  int xzero, int kx) {
  const int lane = threadIdx.x & 63;
  const int wg = uniform(blockIdx.x * 4 + (threadIdx.x >> 6));
  extern __shared__ double lds_part[];
  Rows<WMAX, R, EXACT> rows;
  rows.template load<BAND>(A.pd, wg, lane);
  // without X (the first residual of a solve from X = 0) r = F: the pencil
  // is not read, and |r|^2 = |F|^2 is summed once
  double mv[R][WMAX] = {}, kv[R][WMAX] = {};
  if (xread) {
    rows.values(A.pd.m64, mv);
    rows.values(A.pd.k64, kv);
  }
  const int64_t n = A.pd.n;
  Window<WMAX, R> win;
  double* stg = nullptr;
  if constexpr (BAND) {
    win.init(rows, wg, A.pd.n_slices, A.bw, lane);
    stg = window_base_as<double, R>(lds_part, A.stage_off, U);
  }
  // systems grouped by column of F, whose own-row values are then loaded
  // once per column and chunk instead of once per system (without a column
  // map; with one, each system loads its own)
  ColumnSweep sweep(A.sys.outer, A.B, A.fmap ? 1 : A.m);
  double fcache[R];
  int fcol = -1;
  int bs[U];
  while (sweep.next(bs, lane)) {
    double res[U][R], fr[U][R], xo[U][R];
    double am[U][R], ak[U][R];
    if (xread) {
      if constexpr (BAND) {
        double xw[U][R + 2];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int b = bs[u] >= 0 ? bs[u] : bs[0];
          const double* __restrict__ x = X + (int64_t)b * ldX;
#pragma unroll
          for (int j = 0; j < R + 2; ++j) {
            const int64_t rs = win.src[j];
            xw[u][j] = x[rs < n ? rs : n - 1];
          }
        }
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
          for (int j = 0; j < R + 2; ++j)
            stg[(u * (R + 2) + j) * kSlice + lane] =
                (win.keep[j] && win.src[j] < n) ? xw[u][j] : 0.0;
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const double* w0 = stg + u * (R + 2) * kSlice;
#pragma unroll
          for (int i = 0; i < R; ++i) {
            double sm = 0, sk = 0;
#pragma unroll
            for (int k = 0; k < WMAX; ++k) {
              const double xc = w0[win.off[i][k]];
              sm = fma(mv[i][k], xc, sm);
              sk = fma(kv[i][k], xc, sk);
            }
            am[u][i] = sm;
            ak[u][i] = sk;
            xo[u][i] = xw[u][i + 1];
          }
        }
      } else {
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int b = bs[u] >= 0 ? bs[u] : bs[0];
          const double* __restrict__ x = X + (int64_t)b * ldX;
#pragma unroll
          for (int i = 0; i < R; ++i) {
            double sm = 0, sk = 0;
#pragma unroll
            for (int k = 0; k < WMAX; ++k) {
              const int64_t c = rows.col[i][k];
              const double xc = x[c < n ? c : n - 1];
              sm = fma(mv[i][k], xc, sm);
              sk = fma(kv[i][k], xc, sk);
            }
            am[u][i] = sm;
            ak[u][i] = sk;
            const int64_t row = rows.row[i];
            xo[u][i] = x[row < n ? row : n - 1];
          }
        }
      }
    } else {
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int i = 0; i < R; ++i) am[u][i] = ak[u][i] = xo[u][i] = 0.0;
    }
    if (!A.fmap && bs[0] % A.m != fcol) {
      // every system of the group has this column
      fcol = bs[0] % A.m;
      const double* __restrict__ f = F + (int64_t)fcol * ldf;
#pragma unroll
      for (int i = 0; i < R; ++i) {
        const int64_t row = rows.row[i];
        fcache[i] = f[row < n ? row : n - 1];
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int b = bs[u] >= 0 ? bs[u] : bs[0];
      const double a = sload(ca64 + b / A.m), cbv = sload(cb64 + b / A.m);
      const double* __restrict__ f = A.fmap ? F + (int64_t)sload(A.fmap + b) * ldf : nullptr;
#pragma unroll
      for (int i = 0; i < R; ++i) {
        const int64_t row = rows.row[i];
        const bool in = row < n;
        const double fv = A.fmap ? f[in ? row : n - 1] : fcache[i];
        fr[u][i] = in ? fv : 0.0;
        res[u][i] = in ? fv - fma(a, am[u][i], cbv * ak[u][i]) : 0.0;
        xo[u][i] = in ? xo[u][i] : 0.0;
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int b = bs[u];
      if (b < 0) continue;
      TO* __restrict__ r = A.vec(KR0, b);
      TO* __restrict__ xi = A.vec(KX, b);
      double* __restrict__ x = X + (int64_t)b * ldX;
      double rr = 0, ff = 0;
#pragma unroll
      for (int i = 0; i < R; ++i) {
        if (!rows.valid[i]) continue;
        const int64_t row = rows.row[i];
        r[row] = (TO)res[u][i];
        if (kx == 1) xi[row] = TO(0);
        if (kx == 2) xi[row] = (TO)xo[u][i];
        if (xzero && row < n) x[row] = 0.0;
        rr = fma(res[u][i], res[u][i], rr);
        ff = fma(fr[u][i], fr[u][i], ff);
      }
      ff = wave_total(ff);
      rr = xread ? wave_total(rr) : ff;  // X = 0: res is F, bit for bit
      A.put(lds_part, 0, b, wg, lane, rr);
      A.put(lds_part, 1, b, wg, lane, ff);
    }
  }
  flush_partials(A, lds_part, 0, 1, [&](int b) { return A.sys.outer[b] != 0; });
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
                const double*, int, int, int);
};

template <typename T, int WMAX, int R, int U, bool EXACT, bool BAND>
KernelSet<T> make_set() {
  KernelSet<T> s;
  s.dir = k_dir_spmv<T, WMAX, R, U, false, EXACT, BAND>;
  s.dir_asm = k_dir_spmv<T, WMAX, R, U, true, EXACT, BAND>;
  s.upd = k_update_prec<T, WMAX, R, U, false, EXACT, BAND>;
  s.init = k_update_prec<T, WMAX, R, U, true, EXACT, BAND>;
  s.chain = k_chain<T, WMAX, R, EXACT>;
  s.resid = k_residual<T, WMAX, R, U, EXACT, BAND>;
  return s;
}

// Tile configurations (rows-of-64 slices per wavefront R, systems per group U)
// the autotuner chooses from.  Rows of up to 16 entries use the small ones only.
struct TileCfg { int rows, sys; };
constexpr TileCfg kCfgs[] = {{1, 1}, {1, 2}, {1, 4}, {2, 1}, {2, 2}, {2, 4}, {4, 1}};
constexpr int kNumCfgs = sizeof(kCfgs) / sizeof(kCfgs[0]);
inline bool cfg_allowed(int wclass, int c) { return wclass < 2 || kCfgs[c].rows * kCfgs[c].sys <= 2; }

// Row-length classes: rows of <= 6, <= 8, <= 16 entries.
inline int wmax_class(int max_len) { return max_len <= 6 ? 0 : max_len <= 8 ? 1 : 2; }
inline int wmax_of(int wclass) { return wclass == 0 ? 6 : wclass == 1 ? 8 : 16; }

// Banded kernels: bandwidth <= 64 (every column within one slice of its row),
// for rows of up to 8 entries.
constexpr int kBandMax = kSlice;

template <typename T, int WMAX, bool EXACT, bool BAND>
KernelSet<T> set_for(int c) {
  switch (c) {
    case 0: return make_set<T, WMAX, 1, 1, EXACT, BAND>();
    case 1: return make_set<T, WMAX, 1, 2, EXACT, BAND>();
    case 2: return make_set<T, WMAX, 1, 4, EXACT, BAND>();
    case 3: return make_set<T, WMAX, 2, 1, EXACT, BAND>();
    case 4: return make_set<T, WMAX, 2, 2, EXACT, BAND>();
    case 5: return make_set<T, WMAX, 2, 4, EXACT, BAND>();
    default: return make_set<T, WMAX, 4, 1, EXACT, BAND>();
  }
}

template <typename T, bool BAND>
KernelSet<T> kernel_set_impl(int wclass, bool exact, int c) {
  if (wclass == 0) return exact ? set_for<T, 6, true, BAND>(c) : set_for<T, 6, false, BAND>(c);
  return exact ? set_for<T, 8, true, BAND>(c) : set_for<T, 8, false, BAND>(c);
}

template <typename T>
KernelSet<T> kernel_set_wide(int c) {
  switch (c) {
    case 1: return make_set<T, 16, 1, 2, false, false>();
    case 3: return make_set<T, 16, 2, 1, false, false>();
    default: return make_set<T, 16, 1, 1, false, false>();
  }
}

// Defined in pcg_sets_f32.hip / pcg_sets_f64.hip (banded and general sets in
// separate files so they compile in parallel).
KernelSet<float> kernel_set_f32(int wclass, bool exact, bool band, int cfg);
KernelSet<double> kernel_set_f64(int wclass, bool exact, bool band, int cfg);

template <typename T>
inline KernelSet<T> kernel_set(int wclass, bool exact, bool band, int cfg) {
  if constexpr (sizeof(T) == 4) return kernel_set_f32(wclass, exact, band, cfg);
  else return kernel_set_f64(wclass, exact, band, cfg);
}

}  // namespace airga
