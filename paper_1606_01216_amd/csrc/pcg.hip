// Batched preconditioned CG for K(s_k) X = F over all (shift, column)
// systems at once, in float64 or in float32 inside float64 iterative
// refinement (CG: Section 3 and Section 5; the solves of the AIRGA algorithm
// and of its SPAI and SPAI-update variants).  Host orchestration, the
// per-system reductions and the tile autotuner; the row kernels are in
// pcg_kernels.hpp.
//
// Reductions are deterministic: one partial per (system, wavefront) and a
// fixed-order sum per system.  The row kernels sweep the systems whose
// active flag is set.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "pcg_kernels.hpp"

namespace airga {

// ---- per-system reductions (one block per system) ------------------------
enum ReduceMode {
  RM_PW = 0,        // after A: alpha = rz / pw
  RM_ITER = 1,      // after B (+chain): convergence, beta
  RM_INIT_ABS = 2,  // after the first preconditioner application, tol2 relative to |F|^2
  RM_INIT_REL = 3,  // same, tol2 relative to the starting residual (inner solves)
  RM_START = 4,     // after the float64 residual: record |F|^2 (FP64 mode)
  RM_OUTER = 5,     // after the float64 residual: refinement control (MIXED)
  RM_FINAL = 6,     // after the final float64 residual: relres only
  RM_NONE = 7,      // sums only, no state change (autotuner timing)
};

constexpr int kReduceThreads = 1024;

struct ReduceArgs {
  const double* partial;  // [kSlots][B][G]
  int32_t G;              // partial columns per system
  int32_t B;
  SysDev sys;
  int32_t max_iter;
  int32_t max_sweeps;
  double tol2_rel;  // tol^2 (outer) or inner_tol^2
  double tol2_abs;  // tol^2 for RM_OUTER
  const int32_t* flex;  // per shift: 1 = flexible beta, 0 = classical ratio
  int32_t m;            // systems per shift
};

// One block of NT threads per system: a fixed-order sum of the system's wave
// partials (per thread, then across the wave, then across the waves), then
// the mode's logic.  Blocks never communicate: the row kernels read the
// active flags themselves, and the host's count of active systems is kept
// by atomic increments of nact.
template <int NT>
__global__ void __launch_bounds__(NT) k_reduce(ReduceArgs P, int mode) {
  __shared__ double red[NT / 64][4];
  const int b = blockIdx.x;
  const int t = threadIdx.x;
  const SysDev& Sy = P.sys;
  const bool use_outer = mode == RM_START || mode == RM_OUTER || mode == RM_FINAL;
  if ((use_outer ? Sy.outer[b] : Sy.active[b]) == 0) return;
  // partial slots this mode uses
  const int q0 = (mode == RM_PW || use_outer || mode == RM_NONE) ? 0 : 1;
  const int q1 = mode == RM_PW ? 0 : use_outer ? 1 : (mode == RM_ITER || mode == RM_NONE) ? 3 : 2;
  // all slots in one pass, so every load of a thread is in flight together
  // (unused slots are read too and ignored: the columns are short)
  const double* __restrict__ base = P.partial + (int64_t)b * P.G;
  const int64_t qs = (int64_t)P.B * P.G;
  double v[4] = {0, 0, 0, 0};
#pragma unroll 2
  for (int g = t; g < P.G; g += NT) {
    double x[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) x[q] = base[q * qs + g];
#pragma unroll
    for (int q = 0; q < 4; ++q) v[q] += x[q];
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) v[q] = (q < q0 || q > q1) ? 0.0 : wave_total(v[q]);
  if ((t & 63) == 0) {
#pragma unroll
    for (int q = 0; q < 4; ++q) red[t >> 6][q] = v[q];
  }
  __syncthreads();
  if (t != 0) return;
  double s4[4] = {0, 0, 0, 0};
  for (int w = 0; w < NT / 64; ++w)
#pragma unroll
    for (int q = 0; q < 4; ++q) s4[q] += red[w][q];
  const double s0 = s4[0], s1 = s4[1], rz = s4[2], zw = s4[3];
  const int was_active = Sy.active[b];
  int act = was_active;
  switch (mode) {
    case RM_PW: {
      if (!isfinite(s0)) { Sy.istat[b] = ST_NONFIN; act = 0; }
      else if (s0 <= 0.0) { Sy.istat[b] = ST_BREAK; act = 0; }
      else { Sy.pw[b] = s0; Sy.alpha[b] = Sy.rz[b] / s0; }
      break;
    }
    case RM_ITER: {
      const int it = Sy.iters[b] + 1;
      Sy.iters[b] = it;
      // the iterate has been written (x = 0 + alpha p, at least)
      Sy.first[b] = 0;
      if (!isfinite(s1) || !isfinite(rz) || !isfinite(zw)) { Sy.istat[b] = ST_NONFIN; act = 0; }
      else if (s1 <= Sy.tol2[b]) { Sy.istat[b] = ST_CONV; act = 0; }
      else if (it >= P.max_iter) { Sy.istat[b] = ST_MAXIT; act = 0; }
      else {
        // flexible: keeps p K-conjugate to the previous direction under any
        // preconditioner; classical: the (r, z) ratio, for a symmetric one
        Sy.beta[b] = P.flex[b / P.m] ? -zw / Sy.pw[b] : rz / Sy.rz[b];
        Sy.rz[b] = rz;
      }
      break;
    }
    case RM_INIT_ABS:
    case RM_INIT_REL: {
      if (mode == RM_INIT_REL) Sy.tol2[b] = P.tol2_rel * s1;
      Sy.first[b] = 1;
      Sy.beta[b] = 0.0;
      if (!isfinite(s1) || !isfinite(rz)) { Sy.istat[b] = ST_NONFIN; act = 0; }
      else if (s1 <= Sy.tol2[b]) { Sy.istat[b] = ST_CONV; act = 0; }
      else if (Sy.iters[b] >= P.max_iter) { Sy.istat[b] = ST_MAXIT; act = 0; }
      else { Sy.rz[b] = rz; Sy.istat[b] = ST_MAXIT; }
      break;
    }
    case RM_START: {
      // residual kernel slots: 0 = |F - K X|^2, 1 = |F|^2
      Sy.ff[b] = s1;
      Sy.tol2[b] = P.tol2_rel * s1;
      Sy.relres[b] = s1 > 0 ? sqrt(s0 / s1) : 0.0;
      break;
    }
    case RM_OUTER: {
      if (Sy.sweeps[b] == 0) Sy.ff[b] = s1;
      const double ff = Sy.ff[b];
      Sy.relres[b] = ff > 0 ? sqrt(s0 / ff) : 0.0;
      if (!isfinite(s0)) { Sy.status[b] = ST_NONFIN; Sy.outer[b] = 0; }
      else if (s0 <= P.tol2_abs * ff) { Sy.status[b] = ST_CONV; Sy.outer[b] = 0; }
      else if (Sy.sweeps[b] > 0 && (Sy.istat[b] == ST_BREAK || Sy.istat[b] == ST_NONFIN)) {
        Sy.status[b] = Sy.istat[b]; Sy.outer[b] = 0;
      } else if (Sy.iters[b] >= P.max_iter || Sy.sweeps[b] >= P.max_sweeps) {
        Sy.status[b] = ST_MAXIT; Sy.outer[b] = 0;
      } else {
        act = 1;
      }
      break;
    }
    case RM_FINAL: {
      const double ff = Sy.ff[b];
      Sy.relres[b] = ff > 0 ? sqrt(s0 / ff) : 0.0;
      break;
    }
  }
  if (act != was_active) {
    Sy.active[b] = act;
    atomicAdd(Sy.nact, act - was_active);
  }
}

// Fresh per-system state: every system active and outer-active.
__global__ void k_init_state(SysDev S, int B) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b < B) {
    S.active[b] = 1;
    S.outer[b] = 1;
    S.istat[b] = ST_MAXIT;
    S.status[b] = ST_MAXIT;
    S.handed[b] = 0;
  }
  if (b == 0) S.nact[0] = B;
}

// Systems still iterating when a sweep reaches its iteration cap leave the
// float32 sweeps (their correction of that sweep is already applied): they
// are marked for the float64 finish and are no longer refined.
__global__ void k_handover(SysDev S, int B) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b < B && S.active[b]) {
    S.handed[b] = 1;
    S.active[b] = 0;
    S.outer[b] = 0;
  }
  if (b == 0) S.nact[0] = 0;
}

// dst column i = src column idx[i] (rows < n), float64.
__global__ void k_gather_cols(const double* __restrict__ src, int64_t lds,
                              const int32_t* __restrict__ idx, int64_t n,
                              double* __restrict__ dst, int64_t ldd) {
  const int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int i = blockIdx.y;
  if (r < n) dst[(int64_t)i * ldd + r] = src[(int64_t)idx[i] * lds + r];
}

// dst column idx[i] = src column i (rows < n), float64.
__global__ void k_scatter_cols(const double* __restrict__ src, int64_t lds,
                               const int32_t* __restrict__ idx, int64_t n,
                               double* __restrict__ dst, int64_t ldd) {
  const int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int i = blockIdx.y;
  if (r < n) dst[(int64_t)idx[i] * ldd + r] = src[(int64_t)i * lds + r];
}

// No system inner-active (before a refinement reduction activates some).
__global__ void k_clear_active(SysDev S, int B) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b < B) S.active[b] = 0;
  if (b == 0) S.nact[0] = 0;
}

// Zero the padding rows [n, n_pad) of every workspace vector.
template <typename T>
__global__ void k_zero_pad(T* ws, int64_t vectors, int64_t n, int64_t ld) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t pad = ld - n;
  if (pad <= 0 || i >= vectors * pad) return;
  ws[(i / pad) * ld + n + (i % pad)] = T(0);
}

// X[:, b] = iterate (rows < n), float64 mode.
__global__ void k_copy_out(const double* __restrict__ ws_x, int64_t ld, int64_t n,
                           double* __restrict__ X, int64_t ldX) {
  const int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int b = blockIdx.y;
  if (r < n) X[(int64_t)b * ldX + r] = ws_x[(int64_t)b * ld + r];
}

// X += inner solution (float32 -> float64) for systems refined this sweep.
__global__ void k_ir_update(SolveArgs<float> A, double* __restrict__ X, int64_t ldX, int assign) {
  const int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int b = blockIdx.y;
  const bool swept = A.sys.outer[b] && A.sys.istat[b] != ST_NONFIN;
  // the float32 iterate holds a correction only if the sweep updated it
  // (first is set at the start of an inner solve and cleared by its first
  // update); assign: X has not been written yet (no starting guess)
  const bool add = swept && A.sys.first[b] == 0;
  if (r < A.pd.n) {
    double* __restrict__ x = X + (int64_t)b * ldX + r;
    if (add) *x = (assign ? 0.0 : *x) + (double)A.vec(KX, b)[r];
    else if (assign) *x = 0.0;
  }
  if (r == 0 && swept) A.sys.sweeps[b] += 1;
}

// K(s) in stored (sliced-ELL) order, for the single-shift float64 path.
__global__ void k_assemble_stored(PencilDev pd, int64_t stored, double a, double b,
                                  double* __restrict__ out) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < stored) out[i] = fma(a, pd.m64[i], b * pd.k64[i]);
}

// ------------------------------------------------------ launch bookkeeping

// Optional per-launch event timing (profiled solves).
struct Timer {
  airga_ctx ctx;
  bool on;
  std::vector<hipEvent_t> ev;  // pairs
  std::vector<int> ids;
  airga_status begin(int id, hipEvent_t* e1) {
    if (!on) return AIRGA_OK;
    hipEvent_t a, b;
    AIRGA_HIP(hipEventCreate(&a));
    AIRGA_HIP(hipEventCreate(&b));
    ev.push_back(a);
    ev.push_back(b);
    ids.push_back(id);
    AIRGA_HIP(hipEventRecord(a, ctx->stream));
    *e1 = b;
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

#define TIMED(id, ...)                 \
  do {                                 \
    hipEvent_t e1_ = nullptr;          \
    AIRGA_TRY(tm.begin((id), &e1_));   \
    __VA_ARGS__;                       \
    AIRGA_HIP(hipGetLastError());      \
    AIRGA_TRY(tm.end(e1_));            \
  } while (0)

// Host-side plan of one solve.
template <typename T>
struct Plan {
  airga_ctx ctx = nullptr;
  SolveArgs<T> a{};
  ReduceArgs red{};
  KernelSet<T> ks{};
  bool asm_path = false;
  unsigned grid = 0;
  size_t lds = 0;          // dynamic LDS of the row kernels (partial pre-sum + windows)
  size_t lds_res = 0;      // same for the float64 residual kernel
  int cfg = 0;            // tile configuration (index into kCfgs)
  int max_chain_q = 0;    // largest chain length over shifts
  std::vector<int> clen;  // host copy
  size_t flags_off = 0;   // offset of the host flag arrays in the pinned buffer
};

// One reduction block per system.
template <typename T>
static void reduce(const Plan<T>& P, int mode) {
  k_reduce<kReduceThreads><<<(unsigned)P.a.B, kReduceThreads, 0, P.ctx->stream>>>(P.red, mode);
}

// Profiled solves only: count the systems and shifts the next row kernels
// sweep (synchronises; kernel durations are unaffected).
template <typename T>
static airga_status count_work(Plan<T>& P, Timer& tm, bool in_iteration) {
  if (!tm.on) return AIRGA_OK;
  const int B = P.a.B, m = P.a.m;
  std::vector<int32_t> act(B);
  AIRGA_HIP(hipMemcpyAsync(act.data(), P.a.sys.active, 4 * B, hipMemcpyDeviceToHost, P.ctx->stream));
  AIRGA_HIP(hipStreamSynchronize(P.ctx->stream));
  int64_t sys = 0, shifts = 0, chain_shifts = 0, chain_sys = 0;
  for (int k = 0; k < P.a.nshift; ++k) {
    int any = 0, nk = 0;
    for (int c = 0; c < m; ++c) any |= act[k * m + c];
    for (int c = 0; c < m; ++c) nk += act[k * m + c] != 0;
    sys += nk;
    if (any && P.clen[k] > 0) shifts += 1;
    if (any) chain_shifts += P.clen[k] > 1 ? P.clen[k] - 1 : 0;
    chain_sys += P.clen[k] > 1 ? (int64_t)nk * (P.clen[k] - 1) : 0;
  }
  KernelTimes& t = P.ctx->times;
  const int id = in_iteration ? K_UPDATE_PREC : K_INIT_PREC;
  if (in_iteration) t.sys_passes[K_DIR_SPMV] += sys;
  t.sys_passes[id] += sys;
  t.shift_passes[id] += shifts;
  t.shift_passes[K_CHAIN] += chain_shifts;
  t.sys_passes[K_CHAIN] += chain_sys;
  return AIRGA_OK;
}

// Profiled solves only: count the systems the float64 residual or the
// solution update sweeps next (those whose refinement flag is set), or all B
// (all_sys).
template <typename T>
static airga_status count_outer(Plan<T>& P, Timer& tm, int id, bool all_sys = false) {
  if (!tm.on) return AIRGA_OK;
  const int B = P.a.B;
  int64_t c = B;
  if (!all_sys) {
    std::vector<int32_t> f(B);
    AIRGA_HIP(hipMemcpyAsync(f.data(), P.a.sys.outer, 4 * B, hipMemcpyDeviceToHost, P.ctx->stream));
    AIRGA_HIP(hipStreamSynchronize(P.ctx->stream));
    c = 0;
    for (int b = 0; b < B; ++b) c += f[b] != 0;
  }
  P.ctx->times.sys_passes[id] += c;
  return AIRGA_OK;
}

template <typename T>
static airga_status iteration(Plan<T>& P, Timer& tm, int par) {
  hipStream_t st = P.ctx->stream;
  const unsigned B = (unsigned)P.a.B;
  AIRGA_TRY(count_work(P, tm, true));
  if (P.asm_path)
    TIMED(K_DIR_SPMV, P.ks.dir_asm<<<P.grid, 256, P.lds, st>>>(P.a, par));
  else
    TIMED(K_DIR_SPMV, P.ks.dir<<<P.grid, 256, P.lds, st>>>(P.a, par));
  TIMED(K_REDUCE, reduce(P, RM_PW));
  TIMED(K_UPDATE_PREC, P.ks.upd<<<P.grid, 256, P.lds, st>>>(P.a, par));
  for (int q = 1; q < P.max_chain_q; ++q)
    TIMED(K_CHAIN, P.ks.chain<<<P.grid, 256, P.lds, st>>>(P.a, par, q, 0));
  TIMED(K_REDUCE, reduce(P, RM_ITER));
  return AIRGA_OK;
}

template <typename T>
static airga_status start_inner(Plan<T>& P, Timer& tm, int rel) {
  hipStream_t st = P.ctx->stream;
  AIRGA_TRY(count_work(P, tm, false));
  TIMED(K_INIT_PREC, P.ks.init<<<P.grid, 256, P.lds, st>>>(P.a, 0));
  for (int q = 1; q < P.max_chain_q; ++q)
    TIMED(K_CHAIN, P.ks.chain<<<P.grid, 256, P.lds, st>>>(P.a, 0, q, 1));
  TIMED(K_REDUCE, reduce(P, rel ? RM_INIT_REL : RM_INIT_ABS));
  return AIRGA_OK;
}

// Run CG iterations until no system is active (bounded by max_iter).
template <typename T>
// Mixed sweeps (cap_iters > 0): the sweep ends for the systems still active
// when cap_iters iterations have run, or earlier once at most a quarter of
// the nact0 systems it started with remain and they have had four times the
// rounds half of the batch needed (plus one): stragglers are then handed to
// the float64 finish instead of holding the batch.  capped reports such an
// end with systems still active.
static airga_status iterate(Plan<T>& P, Timer& tm, const airga_pcg_opts& o, int64_t cap_iters,
                            int nact0, bool* capped) {
  hipStream_t st = P.ctx->stream;
  int32_t* h_nact = reinterpret_cast<int32_t*>(static_cast<char*>(P.ctx->host_pinned) + P.flags_off);
  int k = o.poll_every < 2 ? 2 : o.poll_every;
  k += k & 1;
  airga_ctx ctx = P.ctx;
  const bool use_graph = o.use_graph && !o.profile;
  hipGraphExec_t exec = nullptr;
  if (use_graph) {
    // launch arguments of the k captured iterations, byte for byte
    std::vector<char> key(sizeof(P.a) + sizeof(P.red) + sizeof(P.ks) + 4 * sizeof(int));
    char* kp = key.data();
    std::memcpy(kp, &P.a, sizeof(P.a));
    kp += sizeof(P.a);
    std::memcpy(kp, &P.red, sizeof(P.red));
    kp += sizeof(P.red);
    std::memcpy(kp, &P.ks, sizeof(P.ks));
    kp += sizeof(P.ks);
    const int extra[4] = {k, P.asm_path ? 1 : 0, P.max_chain_q, (int)P.grid};
    std::memcpy(kp, extra, sizeof extra);
    size_t found = ctx->graphs.size();
    for (size_t i = 0; i < ctx->graphs.size(); ++i)
      if (ctx->graphs[i].first == key) found = i;
    if (found < ctx->graphs.size()) {
      // most recently used last
      std::rotate(ctx->graphs.begin() + (long)found, ctx->graphs.begin() + (long)found + 1,
                  ctx->graphs.end());
      exec = ctx->graphs.back().second;
    } else {
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
      e = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      if (e != hipSuccess) return fail(AIRGA_EHIP, "graph instantiation failed: %s", hipGetErrorString(e));
      if (ctx->graphs.size() == airga_ctx_s::kGraphs) {
        (void)hipGraphExecDestroy(ctx->graphs.front().second);
        ctx->graphs.erase(ctx->graphs.begin());
      }
      ctx->graphs.emplace_back(std::move(key), exec);
    }
  }
  airga_status result = AIRGA_OK;
  // every system stops at max_iter, so max_iter / k + 2 rounds always suffice
  int64_t rounds = (int64_t)o.max_iter / k + 2;
  if (cap_iters > 0) rounds = std::min<int64_t>(rounds, (cap_iters + k - 1) / k);
  if (capped) *capped = false;
  int64_t half_rounds = -1;  // rounds until at most half of nact0 was left
  for (int64_t round = 0; round < rounds; ++round) {
    if (use_graph) {
      hipError_t e = hipGraphLaunch(exec, st);
      if (e != hipSuccess) {
        result = fail(AIRGA_EHIP, "hipGraphLaunch: %s", hipGetErrorString(e));
        break;
      }
    } else {
      for (int j = 0; j < k && result == AIRGA_OK; ++j) result = iteration(P, tm, j & 1);
      if (result != AIRGA_OK) break;
    }
    hipError_t e = hipMemcpyAsync(h_nact, P.a.sys.nact, sizeof(int32_t), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
      result = fail(AIRGA_EHIP, "polling the active systems: %s", hipGetErrorString(e));
      break;
    }
    result = tm.flush();
    if (result != AIRGA_OK || *h_nact == 0) break;
    if (cap_iters > 0 && nact0 >= 8) {
      if (half_rounds < 0 && 2 * *h_nact <= nact0) half_rounds = round + 1;
      if (half_rounds > 0 && 4 * *h_nact <= nact0 && round + 1 >= 4 * half_rounds + 1) break;
    }
  }
  if (capped && result == AIRGA_OK && cap_iters > 0 && *h_nact > 0) *capped = true;
  return result;
}

template <typename T>
static airga_status prepare(airga_ctx ctx, Plan<T>& P, int32_t nshift, const double* shifts,
                            const airga_prec* precs, int32_t m, const airga_pcg_opts& o, int cfg) {
  const Pencil& pen = ctx->pen;
  hipStream_t st = ctx->stream;
  const int B = nshift * m;
  const int64_t ld = pen.n_pad();
  const int rows = kCfgs[cfg].rows;
  const int G = (int)((pen.n_slices + rows - 1) / rows);
  P.ctx = ctx;
  // padding bytes too: the launch arguments key the graph cache
  std::memset(static_cast<void*>(&P.a), 0, sizeof(P.a));
  std::memset(static_cast<void*>(&P.red), 0, sizeof(P.red));
  // factor values per shift, oldest first; no preconditioner = the identity
  std::vector<std::vector<const fac_t<T>*>> chains(nshift);
  int maxc = 1;
  {
    std::vector<airga_prec> all;
    for (int k = 0; k < nshift; ++k)
      for (airga_prec q = precs ? precs[k] : nullptr; q; q = q->parent) all.push_back(q);
    AIRGA_TRY(prec_resolve_many(ctx, all));
  }
  for (int k = 0; k < nshift; ++k) {
    if (precs && precs[k]) {
      std::vector<airga_prec> ch;
      AIRGA_TRY(prec_chain(precs[k], &ch));
      for (auto it = ch.rbegin(); it != ch.rend(); ++it) {
        if constexpr (sizeof(T) == 4) chains[k].push_back((*it)->v32.as<float>());
        else chains[k].push_back((*it)->v64.as<double>());
      }
    }
    if (chains[k].empty()) {
      if constexpr (sizeof(T) == 4) chains[k].push_back(pen.id32.as<float>());
      else chains[k].push_back(pen.id64.as<double>());
    }
    maxc = (int)chains[k].size() > maxc ? (int)chains[k].size() : maxc;
  }
  // memory
  const size_t vec_bytes = sizeof(T) * (size_t)KINDS * B * ld;
  AIRGA_TRY(ctx->ws_vec.reserve(vec_bytes));
  // partial columns: one per block when its 4 wavefronts pre-sum in LDS
  const unsigned grid = blocks_for(G, 4);
  const int wc = wmax_class(pen.max_len);
  const bool band = !o.general_only && wc < 2 && pen.bandwidth <= kBandMax;
  const size_t win = band ? window_lds_bytes(sizeof(T), rows, kCfgs[cfg].sys) : 0;
  const size_t win_res = band ? window_lds_bytes(sizeof(double), rows, kCfgs[cfg].sys) : 0;
  const bool blk = partial_lds_bytes(B) + (win > win_res ? win : win_res) <= 64 * 1024;
  const int GP = blk ? (int)grid : 4 * (int)grid;
  AIRGA_TRY(ctx->ws_partial.reserve(sizeof(double) * (size_t)B * GP * kSlots));
  const size_t sys_bytes = (7 * sizeof(double) + 8 * sizeof(int32_t)) * (size_t)B + 256;
  AIRGA_TRY(ctx->ws_sys.reserve(sys_bytes));
  const size_t shift_bytes = 4 * sizeof(double) * nshift + sizeof(void*) * (size_t)nshift * maxc +
                             2 * sizeof(int32_t) * nshift + 256;
  AIRGA_TRY(ctx->ws_shift.reserve(shift_bytes));
  P.flags_off = (shift_bytes + 4095) & ~(size_t)4095;
  AIRGA_TRY(ensure_pinned(ctx, P.flags_off + sizeof(int32_t) * 8 * (size_t)B + 64));
  // per-system state
  double* d = ctx->ws_sys.as<double>();
  SysDev S;
  S.rz = d; S.pw = d + B; S.alpha = d + 2 * B; S.beta = d + 3 * B; S.tol2 = d + 4 * B;
  S.ff = d + 5 * B; S.relres = d + 6 * B;
  int32_t* iv = reinterpret_cast<int32_t*>(d + 7 * B);
  S.active = iv; S.first = iv + B; S.istat = iv + 2 * B; S.status = iv + 3 * B;
  S.iters = iv + 4 * B; S.sweeps = iv + 5 * B; S.outer = iv + 6 * B;
  S.nact = iv + 7 * B;
  S.handed = iv + 7 * B + 64;
  // per-shift block, staged in pinned memory and copied once
  char* hp = static_cast<char*>(ctx->host_pinned);
  double* h_ca64 = reinterpret_cast<double*>(hp);
  double* h_cb64 = h_ca64 + nshift;
  T* h_ca = reinterpret_cast<T*>(h_cb64 + nshift);
  T* h_cb = h_ca + nshift;
  const size_t off_fac = 4 * sizeof(double) * nshift;
  const fac_t<T>** h_fac = reinterpret_cast<const fac_t<T>**>(hp + off_fac);
  int32_t* h_clen = reinterpret_cast<int32_t*>(hp + off_fac + sizeof(void*) * (size_t)nshift * maxc);
  int32_t* h_flex = h_clen + nshift;
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
    for (int q = 0; q < maxc; ++q) h_fac[(size_t)k * maxc + q] = q < L ? chains[k][q] : nullptr;
    h_flex[k] = o.beta_form == AIRGA_BETA_FLEXIBLE;
  }
  AIRGA_HIP(hipMemcpyAsync(ctx->ws_shift.ptr, hp, shift_bytes - 256, hipMemcpyHostToDevice, st));
  char* sd = ctx->ws_shift.as<char>();
  AIRGA_HIP(hipMemsetAsync(ctx->ws_sys.ptr, 0, sys_bytes, st));
  k_init_state<<<blocks_for(B, 256), 256, 0, st>>>(S, B);
  AIRGA_HIP(hipGetLastError());
  // padding rows of every workspace vector hold zeros
  const int64_t vectors = (int64_t)KINDS * B;
  if (ld > pen.n) {
    k_zero_pad<T><<<blocks_for(vectors * (ld - pen.n), 256), 256, 0, st>>>(ctx->ws_vec.as<T>(),
                                                                          vectors, pen.n, ld);
    AIRGA_HIP(hipGetLastError());
  }
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
  A.fac = reinterpret_cast<const fac_t<T>* const*>(sd + off_fac);
  A.clen = reinterpret_cast<const int32_t*>(sd + off_fac + sizeof(void*) * (size_t)nshift * maxc);
  P.red.flex = A.clen + nshift;
  P.red.m = m;
  A.maxc = maxc;
  A.partial = ctx->ws_partial.as<double>();
  A.GP = GP;
  A.blk = blk ? 1 : 0;
  A.xz = 0;
  A.sys = S;
  P.red.partial = A.partial;
  P.red.G = GP;
  P.red.B = B;
  P.red.sys = S;
  P.red.max_iter = o.max_iter;
  P.red.max_sweeps = o.max_sweeps;
  P.grid = grid;
  const size_t part = blk ? partial_lds_bytes(B) : 0;
  P.lds = part + win;
  P.lds_res = part + win_res;
  A.bw = pen.bandwidth;
  A.stage_off = (int32_t)(part / sizeof(double));
  const bool exact = pen.uniform_width && pen.max_len == wmax_of(wmax_class(pen.max_len));
  P.ks = kernel_set<T>(wc, exact, band, cfg);
  P.cfg = cfg;
  ctx->last_cfg = cfg;
  return AIRGA_OK;
}

// ----------------------------------------------------------------- autotuner
//
// The tile configuration (R slices per wavefront, U systems per group) is
// chosen per (pencil size, batch, precision and matrix form, row-length
// class) by timing the two row kernels of an iteration for every allowed
// configuration on the solve's own pencil, preconditioners and batch, with
// zeroed vectors; the solve state is re-initialised afterwards.  The choice
// is cached in the context.
template <typename T>
static airga_status autotune(airga_ctx ctx, int32_t nshift, const double* shifts,
                             const airga_prec* precs, int32_t m, const airga_pcg_opts& o,
                             bool asm_path, const T* asm_vals, int* best) {
  const Pencil& pen = ctx->pen;
  const int wc = wmax_class(pen.max_len);
  const int B = nshift * m;
  const int key_prec = (int)sizeof(T) + (asm_path ? 100 : 0);
  for (const auto& t : ctx->tuned)
    if (t.n_slices == pen.n_slices && t.batch == B && t.prec == key_prec && t.wclass == wc) {
      *best = t.cfg;
      return AIRGA_OK;
    }
  hipStream_t st = ctx->stream;
  hipEvent_t e0, e1;
  AIRGA_HIP(hipEventCreate(&e0));
  AIRGA_HIP(hipEventCreate(&e1));
  float best_ms = 1e30f;
  int best_cfg = 0;
  airga_status result = AIRGA_OK;
  for (int c = 0; c < kNumCfgs && result == AIRGA_OK; ++c) {
    if (!cfg_allowed(wc, c)) continue;
    Plan<T> P;
    result = prepare<T>(ctx, P, nshift, shifts, precs, m, o, c);
    if (result != AIRGA_OK) break;
    if (asm_path) {
      P.a.mv = asm_vals;
      P.a.kv = nullptr;
    }
    hipError_t e = hipMemsetAsync(P.a.ws, 0, sizeof(T) * (size_t)KINDS * P.a.B * P.a.ld, st);
    for (int rep = 0; rep < 4 && e == hipSuccess; ++rep) {
      if (rep == 1) e = hipEventRecord(e0, st);
      if (asm_path) P.ks.dir_asm<<<P.grid, 256, P.lds, st>>>(P.a, 0);
      else P.ks.dir<<<P.grid, 256, P.lds, st>>>(P.a, 0);
      reduce(P, RM_NONE);
      P.ks.upd<<<P.grid, 256, P.lds, st>>>(P.a, 0);
      reduce(P, RM_NONE);
    }
    if (e == hipSuccess) e = hipEventRecord(e1, st);
    if (e == hipSuccess) e = hipGetLastError();
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e != hipSuccess) {
      result = fail(AIRGA_EHIP, "autotuning: %s", hipGetErrorString(e));
      break;
    }
    if (ms < best_ms) {
      best_ms = ms;
      best_cfg = c;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  AIRGA_TRY(result);
  ctx->tuned.push_back({pen.n_slices, B, key_prec, wc, best_cfg, best_ms});
  *best = best_cfg;
  return AIRGA_OK;
}

// ------------------------------------------------------------------ solves

// Per-system results, read back in one copy into pinned memory: relres and
// the int32 arrays after it in the state block (statuses, counts, nact and the
// hand-over flags).  handed (mixed solves): the systems left for the float64
// finish.
static airga_status read_stats(airga_ctx ctx, const SysDev& S, int B, bool mixed,
                               airga_sys_stats* stats, std::vector<int>* handed) {
  hipStream_t st = ctx->stream;
  const char* lo = reinterpret_cast<const char*>(S.relres);
  const size_t bytes = (size_t)(reinterpret_cast<const char*>(S.handed + B) - lo);
  AIRGA_TRY(ensure_pinned(ctx, bytes));
  const char* h = static_cast<const char*>(ctx->host_pinned);
  AIRGA_HIP(hipMemcpyAsync(ctx->host_pinned, lo, bytes, hipMemcpyDeviceToHost, st));
  AIRGA_HIP(hipStreamSynchronize(st));
  auto host = [&](const int32_t* d) {
    return reinterpret_cast<const int32_t*>(h + (reinterpret_cast<const char*>(d) - lo));
  };
  const double* rel = reinterpret_cast<const double*>(h);
  const int32_t *sta = host(S.status), *ist = host(S.istat), *its = host(S.iters);
  const int32_t *swp = host(S.sweeps), *out = host(S.outer), *hnd = host(S.handed);
  if (handed)
    for (int b = 0; b < B; ++b)
      if (hnd[b]) handed->push_back(b);
  if (!stats) return AIRGA_OK;
  for (int b = 0; b < B; ++b) {
    stats[b].status = mixed ? (out[b] ? ST_MAXIT : sta[b]) : ist[b];
    stats[b].iters = its[b];
    stats[b].sweeps = mixed ? swp[b] : 1;
    stats[b].finished_fp64 = 0;
    stats[b].relres = rel[b];
  }
  return AIRGA_OK;
}

// The tile the caller forces (opts.tile_rows/tile_sys), if any.
static airga_status forced_cfg(const Pencil& pen, const airga_pcg_opts& o, int* cfg) {
  *cfg = -1;
  if (o.tile_rows == 0 && o.tile_sys == 0) return AIRGA_OK;
  const int wc = wmax_class(pen.max_len);
  for (int c = 0; c < kNumCfgs; ++c)
    if (kCfgs[c].rows * kSlice == o.tile_rows && kCfgs[c].sys == o.tile_sys && cfg_allowed(wc, c)) {
      *cfg = c;
      return AIRGA_OK;
    }
  return fail(AIRGA_EINVAL, "tile (%d rows, %d systems) is not an allowed configuration",
              o.tile_rows, o.tile_sys);
}

// fmap (device, optional): column of F for each system instead of b % m.
static airga_status solve_fp64(airga_ctx ctx, int32_t nshift, const double* shifts,
                               const airga_prec* precs, int32_t m, const double* F, int64_t ldf,
                               double* X, int64_t ldx, const airga_pcg_opts& o,
                               airga_sys_stats* stats, const int32_t* fmap = nullptr) {
  const Pencil& pen = ctx->pen;
  hipStream_t st = ctx->stream;
  const int B = nshift * m;
  // One shift: store K(s) once (plain float64 CG on the assembled matrix).
  const bool asm_path = nshift == 1;
  if (asm_path) {
    AIRGA_TRY(ctx->ws_asm.reserve(sizeof(double) * pen.nnz_stored));
    double a, b;
    shift_coeffs(pen, shifts[0], &a, &b);
    k_assemble_stored<<<blocks_for(pen.nnz_stored, 256), 256, 0, st>>>(pen.dev(), pen.nnz_stored,
                                                                       a, b, ctx->ws_asm.as<double>());
    AIRGA_HIP(hipGetLastError());
  }
  int cfg = 0;
  AIRGA_TRY(forced_cfg(pen, o, &cfg));
  if (cfg < 0)
    AIRGA_TRY(autotune<double>(ctx, nshift, shifts, precs, m, o, asm_path,
                               ctx->ws_asm.as<double>(), &cfg));
  Plan<double> P;
  AIRGA_TRY(prepare<double>(ctx, P, nshift, shifts, precs, m, o, cfg));
  if (asm_path) {
    P.a.mv = ctx->ws_asm.as<double>();
    P.a.kv = nullptr;
    P.asm_path = true;
  }
  P.a.fmap = fmap;
  const double* ca64 = reinterpret_cast<const double*>(ctx->ws_shift.ptr);
  const double* cb64 = ca64 + nshift;
  P.red.tol2_rel = o.tol * o.tol;
  Timer tm{ctx, o.profile != 0, {}, {}};
  const int x0 = o.x0_given ? 1 : 0;
  AIRGA_TRY(count_outer(P, tm, K_IR_RESIDUAL));
  TIMED(K_IR_RESIDUAL, P.ks.resid<<<P.grid, 256, P.lds_res, st>>>(P.a, F, ldf, X, ldx, ca64, cb64, x0,
                                                         1 - x0, x0 ? 2 : 1));
  TIMED(K_REDUCE, reduce(P, RM_START));
  AIRGA_TRY(start_inner(P, tm, 0));
  AIRGA_TRY(iterate(P, tm, o, 0, 0, nullptr));
  // result out, then its true residual
  AIRGA_TRY(count_outer(P, tm, K_IR_UPDATE, true));
  TIMED(K_IR_UPDATE, (k_copy_out<<<dim3(blocks_for(pen.n, 256), (unsigned)B), 256, 0, st>>>(
                         P.a.ws + (int64_t)KX * B * P.a.ld, P.a.ld, pen.n, X, ldx)));
  AIRGA_TRY(count_outer(P, tm, K_IR_RESIDUAL));
  TIMED(K_IR_RESIDUAL, P.ks.resid<<<P.grid, 256, P.lds_res, st>>>(P.a, F, ldf, X, ldx, ca64, cb64, 1, 0, 0));
  TIMED(K_REDUCE, reduce(P, RM_FINAL));
  AIRGA_TRY(tm.flush());
  return read_stats(ctx, P.a.sys, B, false, stats, nullptr);
}

// Float32 iterations per refinement sweep before a system still iterating
// is handed to the float64 finish.
constexpr int64_t kInnerMax = 96;

// Float64 finish of a mixed solve: the systems `sys` (indices k*m + c) are
// gathered into a contiguous batch, solved by the float64 path from their
// current X, and scattered back; their stats absorb the float64 stage.
static airga_status finish_fp64(airga_ctx ctx, const double* shifts, const airga_prec* precs,
                                int32_t m, const double* F, int64_t ldf, double* X, int64_t ldx,
                                const airga_pcg_opts& o, const std::vector<int>& sys,
                                airga_sys_stats* stats) {
  const Pencil& pen = ctx->pen;
  hipStream_t st = ctx->stream;
  const int Bp = (int)sys.size();
  const int64_t n = pen.n;
  const size_t idx_bytes = (2 * sizeof(int32_t) * (size_t)Bp + 255) & ~(size_t)255;
  AIRGA_TRY(ctx->ws_gather.reserve(idx_bytes + sizeof(double) * (size_t)Bp * n));
  int32_t* d_idx = ctx->ws_gather.as<int32_t>();
  double* Xp = reinterpret_cast<double*>(ctx->ws_gather.as<char>() + idx_bytes);
  AIRGA_TRY(ensure_pinned(ctx, 2 * sizeof(int32_t) * (size_t)Bp));
  int32_t* h_idx = static_cast<int32_t*>(ctx->host_pinned);
  std::vector<double> sh(Bp);
  std::vector<airga_prec> pr(Bp);
  for (int i = 0; i < Bp; ++i) {
    h_idx[i] = sys[i] % m;        // column of F
    h_idx[Bp + i] = sys[i];       // column of X
    sh[i] = shifts[sys[i] / m];
    pr[i] = precs ? precs[sys[i] / m] : nullptr;
  }
  AIRGA_HIP(hipMemcpyAsync(d_idx, h_idx, 2 * sizeof(int32_t) * Bp, hipMemcpyHostToDevice, st));
  // the pinned staging area is rewritten by the solve below
  AIRGA_HIP(hipStreamSynchronize(st));
  const dim3 grid(blocks_for(n, 256), (unsigned)Bp);
  k_gather_cols<<<grid, 256, 0, st>>>(X, ldx, d_idx + Bp, n, Xp, n);
  AIRGA_HIP(hipGetLastError());
  airga_pcg_opts o64 = o;
  o64.mode = AIRGA_MODE_FP64;
  o64.x0_given = 1;
  std::vector<airga_sys_stats> s64(Bp);
  // each system keeps its own column of F through the column map
  AIRGA_TRY(solve_fp64(ctx, Bp, sh.data(), pr.data(), 1, F, ldf, Xp, n, o64, s64.data(), d_idx));
  k_scatter_cols<<<grid, 256, 0, st>>>(Xp, n, d_idx + Bp, n, X, ldx);
  AIRGA_HIP(hipGetLastError());
  for (int i = 0; i < Bp; ++i) {
    airga_sys_stats& e = stats[sys[i]];
    e.status = s64[i].status;
    e.iters += s64[i].iters;
    e.sweeps += 1;
    e.relres = s64[i].relres;
    e.finished_fp64 = 1;
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
  int cfg = 0;
  AIRGA_TRY(forced_cfg(pen, o, &cfg));
  if (cfg < 0) AIRGA_TRY(autotune<float>(ctx, nshift, shifts, precs, m, o, false, nullptr, &cfg));
  Plan<float> P;
  AIRGA_TRY(prepare<float>(ctx, P, nshift, shifts, precs, m, o, cfg));
  const double* ca64 = reinterpret_cast<const double*>(ctx->ws_shift.ptr);
  const double* cb64 = ca64 + nshift;
  P.red.tol2_rel = o.inner_tol * o.inner_tol;
  P.red.tol2_abs = o.tol * o.tol;
  Timer tm{ctx, o.profile != 0, {}, {}};
  int32_t* h_nact = reinterpret_cast<int32_t*>(static_cast<char*>(ctx->host_pinned) + P.flags_off);
  const int x0 = o.x0_given ? 1 : 0;
  // Every inner solve starts from a zero iterate that is never stored (the
  // first update of a sweep writes it), and without a starting guess X is
  // first assigned by the sweep-0 correction instead of zeroed beforehand.
  P.a.xz = 1;
  // sweep 0 residual; RM_OUTER then activates the systems to refine
  AIRGA_TRY(count_outer(P, tm, K_IR_RESIDUAL));
  TIMED(K_IR_RESIDUAL, P.ks.resid<<<P.grid, 256, P.lds_res, st>>>(P.a, F, ldf, X, ldx, ca64, cb64, x0,
                                                         0, 0));
  k_clear_active<<<blocks_for(B, 256), 256, 0, st>>>(P.a.sys, B);
  AIRGA_HIP(hipGetLastError());
  TIMED(K_REDUCE, reduce(P, RM_OUTER));
  const int64_t cap = o.inner_max > 0 ? o.inner_max : kInnerMax;
  bool any_handed = false;
  bool assign = x0 == 0;  // X still unwritten
  const dim3 ir_grid(blocks_for(pen.n, 256), (unsigned)B);
  for (int sweep = 0; sweep <= o.max_sweeps; ++sweep) {
    AIRGA_HIP(hipMemcpyAsync(h_nact, P.a.sys.nact, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    AIRGA_HIP(hipStreamSynchronize(st));
    if (*h_nact == 0) break;
    AIRGA_TRY(start_inner(P, tm, 1));
    bool capped = false;
    AIRGA_TRY(iterate(P, tm, o, cap, *h_nact, &capped));
    AIRGA_TRY(count_outer(P, tm, K_IR_UPDATE));
    TIMED(K_IR_UPDATE, (k_ir_update<<<ir_grid, 256, 0, st>>>(P.a, X, ldx, assign ? 1 : 0)));
    assign = false;
    if (capped) {
      k_handover<<<blocks_for(B, 256), 256, 0, st>>>(P.a.sys, B);
      AIRGA_HIP(hipGetLastError());
      any_handed = true;
    }
    AIRGA_TRY(count_outer(P, tm, K_IR_RESIDUAL));
    TIMED(K_IR_RESIDUAL, P.ks.resid<<<P.grid, 256, P.lds_res, st>>>(P.a, F, ldf, X, ldx, ca64, cb64, 1, 0, 0));
    TIMED(K_REDUCE, reduce(P, RM_OUTER));
  }
  // no sweep ran (every system settled by the first residual): X = 0
  if (assign) {
    k_ir_update<<<ir_grid, 256, 0, st>>>(P.a, X, ldx, 1);
    AIRGA_HIP(hipGetLastError());
  }
  AIRGA_TRY(tm.flush());
  std::vector<airga_sys_stats> mixed(B);
  std::vector<int> handed;
  AIRGA_TRY(read_stats(ctx, P.a.sys, B, true, mixed.data(), any_handed ? &handed : nullptr));
  if (!handed.empty())
    AIRGA_TRY(finish_fp64(ctx, shifts, precs, m, F, ldf, X, ldx, o, handed, mixed.data()));
  if (stats) std::copy(mixed.begin(), mixed.end(), stats);
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
  o->inner_tol = 1e-5;
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
      if (precs[k]->is_complex)
        return fail(AIRGA_EINVAL, "preconditioner %d is complex: use airga_cocg_solve", k);
      if (precs[k]->generation != pen.generation)
        return fail(AIRGA_ESTATE, "preconditioner %d was built for an earlier pencil", k);
    }
  }
  airga_pcg_opts o;
  airga_pcg_opts_default(&o);
  if (opts) o = *opts;
  if (!(o.tol >= 0) || o.max_iter < 0 || (o.mode != AIRGA_MODE_FP64 && o.mode != AIRGA_MODE_MIXED) ||
      o.beta_form < AIRGA_BETA_FLEXIBLE || o.beta_form > AIRGA_BETA_CLASSICAL)
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

airga_status airga_get_tile_config(airga_ctx ctx, int32_t* rows_per_wave,
                                   int32_t* systems_per_group) {
  AIRGA_TRY(check_ctx(ctx));
  if (!rows_per_wave || !systems_per_group) return fail(AIRGA_EINVAL, "null output");
  if (ctx->last_cfg < 0) return fail(AIRGA_ESTATE, "no solve has run on this context");
  *rows_per_wave = kCfgs[ctx->last_cfg].rows * kSlice;
  *systems_per_group = kCfgs[ctx->last_cfg].sys;
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
