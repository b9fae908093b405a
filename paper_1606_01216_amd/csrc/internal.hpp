// Internal declarations of libairga (gfx950).  Not part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

#include "airga.h"

namespace airga {

// Rows per slice of the sliced-ELL layout: one wavefront of 64 lanes, one row
// per lane, so every matrix load of a wavefront is one contiguous 64-entry run.
constexpr int kSlice = 64;
// Longest row the pencil may have.
constexpr int kMaxRow = 16;
// Longest row the SPAI column kernels handle (the Givens factor of a column
// problem lives in registers: kSpaiMaxJ*(kSpaiMaxJ+1)/2 doubles).
constexpr int kSpaiMaxJ = 8;

// ------------------------------------------------------------------ errors

void set_error(const char* fmt, ...);
airga_status fail(airga_status st, const char* fmt, ...);

#define AIRGA_HIP(call)                                                              \
  do {                                                                               \
    hipError_t e_ = (call);                                                          \
    if (e_ != hipSuccess)                                                            \
      return ::airga::fail(AIRGA_EHIP, "%s failed: %s (%s:%d)", #call,               \
                           hipGetErrorString(e_), __FILE__, __LINE__);               \
  } while (0)

#define AIRGA_TRY(expr)                     \
  do {                                      \
    airga_status s_ = (expr);               \
    if (s_ != AIRGA_OK) return s_;          \
  } while (0)

// ------------------------------------------------------------- device memory

// A grow-only device allocation.
struct DevBuf {
  void* ptr = nullptr;
  size_t bytes = 0;
  airga_status reserve(size_t need);
  void release();
  // hand the allocation over (to a pool) / take one over (from a pool)
  void detach(void** p, size_t* b) {
    *p = ptr;
    *b = bytes;
    ptr = nullptr;
    bytes = 0;
  }
  void adopt(void* p, size_t b) {
    release();
    ptr = p;
    bytes = b;
  }
  template <typename T>
  T* as() const { return static_cast<T*>(ptr); }
  ~DevBuf() { release(); }
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
};

// ------------------------------------------------------------------- pencil

// Device view of the pencil in sliced-ELL form.  Slice s holds rows
// [64 s, 64 s + 64); entry k of row r sits at slice_ptr[s] + 64 k + (r % 64)
// for k < width(s) = (slice_ptr[s+1] - slice_ptr[s]) / 64.  Entries past a
// row's length are padding: column = the row itself, value 0.
struct PencilDev {
  int32_t n;
  int32_t n_slices;
  const int32_t* slice_ptr;  // n_slices + 1
  const int32_t* row_len;    // n_slices * 64 (0 for rows >= n)
  const int32_t* col;        // stored entries
  const int32_t* mirror;     // stored index of entry (c, r) for entry (r, c)
  const int32_t* csr_pos;    // CSR position of each stored entry, -1 for padding
  const int32_t* diag_pos;   // stored index of (r, r)
  const int8_t* coff;        // column - row of each stored entry (bandwidth <= 64 only)
  const double* m64;
  const double* k64;
  const float* m32;
  const float* k32;
};

struct Pencil {
  bool valid = false;
  uint64_t generation = 0;
  int32_t n = 0, n_slices = 0, max_len = 0, bandwidth = 0;
  int64_t nnz = 0, nnz_stored = 0;
  double alpha = 0, beta = 0;
  double gram_mm = 0, gram_mk = 0, gram_kk = 0, tr_m = 0, tr_k = 0;
  bool diag_ok = false;  // M_rr > 0 and K_rr >= 0 for every row
  bool uniform_width = false;  // every slice is max_len entries wide
  bool contiguous = false;     // every row's columns are consecutive
  DevBuf slice_ptr, row_len, col, mirror, csr_pos, diag_pos, m64, k64, m32, k32;
  DevBuf coff;        // int8 column offsets (banded pencils)
  DevBuf setup;       // scratch of set_pencil (pattern summary, per-slice data)
  DevBuf gram_ws;     // scratch of set_pencil (Gram partial sums)
  DevBuf id64, id32;  // the identity on the pattern (solves without a preconditioner)
  PencilDev dev() const;
  int64_t n_pad() const { return (int64_t)n_slices * kSlice; }
};

// ------------------------------------------------------------- kernel times

enum KernelId {
  K_DIR_SPMV = 0,   // direction update + shifted SpMV + (p, Kp)
  K_UPDATE_PREC,    // x/r update + first preconditioner factor + dots
  K_INIT_PREC,      // first preconditioner application of a (re)start
  K_CHAIN,          // further chain factors
  K_REDUCE,         // per-system scalar reductions
  K_IR_RESIDUAL,    // float64 residual F - K X
  K_IR_UPDATE,      // X += d
  K_COUNT
};

// Per-kernel launch counts and summed durations (profiled solves), plus the
// work each launch did: systems swept and shifts whose factor was read.
struct KernelTimes {
  int64_t launches[K_COUNT] = {};
  double ms[K_COUNT] = {};
  int64_t sys_passes[K_COUNT] = {};
  int64_t shift_passes[K_COUNT] = {};
  void clear() {
    for (int i = 0; i < K_COUNT; ++i) {
      launches[i] = 0;
      ms[i] = 0;
      sys_passes[i] = 0;
      shift_passes[i] = 0;
    }
  }
};

// ------------------------------------------------------------------ context

}  // namespace airga

struct airga_ctx_s {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  airga::Pencil pen;
  // Solve workspaces (grow-only).
  airga::DevBuf ws_vec, ws_partial, ws_sys, ws_shift, ws_asm, ws_tmp;
  // Block operations of the moment sequence: per-block partial sums, and
  // small results (Gram blocks, coefficients) on their way to the host.
  airga::DevBuf ws_gram, ws_small;
  void* host_pinned = nullptr;
  size_t host_pinned_bytes = 0;
  airga::KernelTimes times;
  std::atomic<int> live_precs{0};
  // Autotuned tile configuration, keyed by (n_slices, batch, precision and
  // matrix form, row-length class); ms = the winning timing.
  struct Tune { int32_t n_slices, batch, prec, wclass, cfg; float ms; };
  std::vector<Tune> tuned;
  int last_cfg = -1;  // tile configuration of the last solve
  // Device buffers of released preconditioners, reused by later ones.  All
  // work of a context is ordered on one stream, so a buffer handed back here
  // can be reused by later work without waiting for earlier kernels.
  std::vector<std::pair<void*, size_t>> pool;
  // Captured iteration graphs, keyed by the launch arguments they were
  // captured with (most recently used last); a graph is replayed whenever a
  // sweep's arguments are identical.  At most kGraphs are kept.
  static constexpr size_t kGraphs = 8;
  std::vector<std::pair<std::vector<char>, hipGraphExec_t>> graphs;
  // Column-gather area of the float64 finish of mixed solves.
  airga::DevBuf ws_gather;
  // Device address of the fixed partial-sum array of airga_gram_noalloc on
  // this context's GPU (looked up when the context is created).
  double* gram_scratch = nullptr;
  ~airga_ctx_s() {
    for (auto& g : graphs) (void)hipGraphExecDestroy(g.second);
    for (auto& b : pool) (void)hipFree(b.first);
  }
};

struct airga_prec_s {
  airga_ctx ctx = nullptr;
  uint64_t generation = 0;
  std::atomic<int> refs{1};
  double shift = 0;
  double shift_im = 0;       // imaginary part of a complex expansion point
  double alpha = 0;          // host copy once known (read lazily)
  double alpha_im = 0;       // complex factors: imaginary part of alpha
  bool is_complex = false;   // complex factor: v64 holds interleaved (re, im) values
  bool alpha_known = false;
  bool is_update = false;
  int64_t skipped = -1;      // host copy once known
  bool scalar_only = false;  // decided on the host after the skip count is read
  bool scalar_known = false;
  airga_prec parent = nullptr;
  // v32: the values rounded to float32, the copy the float32 inner solves read;
  // scal: alpha, the skip count and the skipped-column flags, on device
  airga::DevBuf v64, v32, objective, scal;
};

namespace airga {

airga_status check_ctx(airga_ctx ctx);
airga_status check_pencil(airga_ctx ctx);
airga_status ensure_pinned(airga_ctx ctx, size_t bytes);

// Resolve the lazy host-side facts of update factors (one synchronisation
// for the whole set).
airga_status prec_resolve(airga_prec p);
airga_status prec_resolve_many(airga_ctx ctx, const std::vector<airga_prec>& ps);
// Device buffers from the context's pool (or fresh).
airga_status pool_get(airga_ctx ctx, DevBuf* buf, size_t need);
void pool_put(airga_ctx ctx, DevBuf* buf);
// Non-scalar factors of the chain, newest first.
airga_status prec_chain(airga_prec p, std::vector<airga_prec>* out);

// Shift coefficients a = s^2 + alpha s, b = 1 + beta s.
inline void shift_coeffs(const Pencil& pen, double s, double* a, double* b) {
  *a = s * s + pen.alpha * s;
  *b = 1.0 + pen.beta * s;
}

// ----------------------------------------------------------- device helpers

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

template <typename T>
__device__ __forceinline__ T wave_max(T v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    T o = __shfl_xor(v, off, 64);
    v = o > v ? o : v;
  }
  return v;
}

// Wavefront-wide sum returned in every lane, built from DPP lane moves (no
// LDS round trips): four row shifts make each 16-lane row an inclusive scan,
// two row broadcasts carry the row totals into lane 63, which is then read
// back as a scalar.  All 64 lanes must be active.
template <int CTRL, int ROWMASK>
__device__ __forceinline__ float dpp_add(float v) {
  const int s = __builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROWMASK, 0xf, true);
  return v + __int_as_float(s);
}
template <int CTRL, int ROWMASK>
__device__ __forceinline__ double dpp_add(double v) {
  const long long bits = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)bits, CTRL, ROWMASK, 0xf, true);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(bits >> 32), CTRL, ROWMASK, 0xf, true);
  return v + __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ float lane63(float v) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
}
__device__ __forceinline__ double lane63(double v) {
  const long long bits = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)bits, 63);
  const int hi = __builtin_amdgcn_readlane((int)(bits >> 32), 63);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
template <typename T>
__device__ __forceinline__ T wave_total(T v) {
  v = dpp_add<0x111, 0xf>(v);  // row_shr:1
  v = dpp_add<0x112, 0xf>(v);  // row_shr:2
  v = dpp_add<0x114, 0xf>(v);  // row_shr:4
  v = dpp_add<0x118, 0xf>(v);  // row_shr:8
  v = dpp_add<0x142, 0xa>(v);  // row_bcast:15 into rows 1 and 3
  v = dpp_add<0x143, 0xc>(v);  // row_bcast:31 into rows 2 and 3
  return lane63(v);
}

// Make a wavefront-uniform value scalar (it then lives in an SGPR).
__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

// Load of a wave-uniform address through the constant address space, so it
// becomes a scalar load: it is counted apart from the vector loads in flight
// and does not wait for them.  For data no kernel writes while it runs.
template <typename V>
__device__ __forceinline__ V sload(const V* p) {
  return *(const __attribute__((address_space(4))) V*)p;
}

// Makes `dev` the current device for the scope of a C-ABI call.
struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) (void)hipSetDevice(dev);
  }
  ~DeviceGuard() {
    if (prev >= 0) (void)hipSetDevice(prev);
  }
};

// Launch-size helper.
inline unsigned blocks_for(int64_t work, int per_block) {
  return (unsigned)((work + per_block - 1) / per_block);
}

// Device address of the fixed partial-sum array of airga_gram_noalloc on
// `device` (looked up once per device, with that device current).
airga_status gram_scratch_address(int device, double** out);

// Kernels shared between translation units.
__global__ void k_fill_f64(double* p, int64_t count, double v);
__global__ void k_fill_i32(int32_t* p, int64_t count, int32_t v);

}  // namespace airga
