// Context, errors, and the pencil (M, K): validation, the sliced-ELL copy,
// the transpose map, Gram scalars, shift assembly and the shifted product.
#include <cmath>
#include <cstring>

#include "internal.hpp"

namespace airga {

static thread_local std::string g_err;

void set_error(const char* fmt, ...) {
  char buf[1024];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
}

airga_status fail(airga_status st, const char* fmt, ...) {
  char buf[1024];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return st;
}

airga_status DevBuf::reserve(size_t need) {
  if (ptr && need <= bytes) return AIRGA_OK;
  // growing: queued kernels may still use the old allocation (workspaces are
  // shared between calls on the context stream), so wait for them first
  if (ptr) (void)hipDeviceSynchronize();
  release();
  if (need == 0) return AIRGA_OK;
  hipError_t e = hipMalloc(&ptr, need);
  if (e != hipSuccess) {
    ptr = nullptr;
    bytes = 0;
    (void)hipGetLastError();
    return fail(AIRGA_ENOMEM, "device allocation of %zu bytes failed: %s", need,
                hipGetErrorString(e));
  }
  bytes = need;
  return AIRGA_OK;
}

void DevBuf::release() {
  if (ptr) (void)hipFree(ptr);
  ptr = nullptr;
  bytes = 0;
}

PencilDev Pencil::dev() const {
  PencilDev d;
  d.n = n;
  d.n_slices = n_slices;
  d.slice_ptr = slice_ptr.as<int32_t>();
  d.row_len = row_len.as<int32_t>();
  d.col = col.as<int32_t>();
  d.mirror = mirror.as<int32_t>();
  d.csr_pos = csr_pos.as<int32_t>();
  d.diag_pos = diag_pos.as<int32_t>();
  d.coff = bandwidth <= kSlice ? coff.as<int8_t>() : nullptr;
  d.m64 = m64.as<double>();
  d.k64 = k64.as<double>();
  d.m32 = m32.as<float>();
  d.k32 = k32.as<float>();
  return d;
}

airga_status check_ctx(airga_ctx ctx) {
  if (!ctx) return fail(AIRGA_EINVAL, "null context");
  AIRGA_HIP(hipSetDevice(ctx->device));
  return AIRGA_OK;
}

airga_status check_pencil(airga_ctx ctx) {
  AIRGA_TRY(check_ctx(ctx));
  if (!ctx->pen.valid) return fail(AIRGA_ESTATE, "no pencil set (call airga_set_pencil first)");
  return AIRGA_OK;
}

airga_status ensure_pinned(airga_ctx ctx, size_t bytes) {
  if (ctx->host_pinned && ctx->host_pinned_bytes >= bytes) return AIRGA_OK;
  if (ctx->host_pinned) (void)hipHostFree(ctx->host_pinned);
  ctx->host_pinned = nullptr;
  ctx->host_pinned_bytes = 0;
  AIRGA_HIP(hipHostMalloc(&ctx->host_pinned, bytes, hipHostMallocDefault));
  ctx->host_pinned_bytes = bytes;
  return AIRGA_OK;
}

__global__ void k_fill_f64(double* p, int64_t count, double v) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < count) p[i] = v;
}

__global__ void k_fill_i32(int32_t* p, int64_t count, int32_t v) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < count) p[i] = v;
}

// ------------------------------------------------------------------ kernels

enum PatternFlag : int32_t {
  F_ROWPTR = 1,      // row pointer out of order or out of range
  F_TOO_LONG = 2,    // a row longer than kMaxRow
  F_COL_RANGE = 4,   // column index outside [0, n)
  F_UNSORTED = 8,    // columns not strictly increasing within a row
  F_NO_DIAG = 16,    // diagonal missing
  F_ENDS = 32,       // row_ptr[0] != 0 or row_ptr[n] != nnz
  F_ASYM = 64,       // pattern not structurally symmetric
  F_GAPPED = 128,    // not an error: a row's columns are not consecutive
};

// One thread per (padded) row; a 256-thread block covers four slices, so each
// wavefront is exactly one slice.  Per slice: longest row (slice_w), widest
// band (slice_b) and pattern flags (slice_f), plain stores reduced by
// k_scan_slices (no same-address atomics).
__global__ void k_rows_check(int32_t n, int64_t nnz, int64_t n_pad, const int32_t* __restrict__ rp,
                             const int32_t* __restrict__ ci, int32_t* __restrict__ row_len,
                             int32_t* __restrict__ slice_w, int32_t* __restrict__ slice_b,
                             int32_t* __restrict__ slice_f) {
  const int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  int len = 0, bw = 0, bad = 0;
  if (r < n) {
    const int64_t b = rp[r], e = rp[r + 1];
    if (b < 0 || e < b || e > nnz) {
      bad |= F_ROWPTR;
    } else if (e - b > kMaxRow) {
      bad |= F_TOO_LONG;
      len = kMaxRow + 1;
    } else {
      len = (int)(e - b);
      int prev = -1;
      bool diag = false;
      for (int64_t q = b; q < e; ++q) {
        const int c = ci[q];
        if (c < 0 || c >= n) {
          bad |= F_COL_RANGE;
          continue;
        }
        if (c <= prev) bad |= F_UNSORTED;
        if (prev >= 0 && c != prev + 1) bad |= F_GAPPED;
        prev = c;
        if (c == r) diag = true;
        const int d = c > r ? (int)(c - r) : (int)(r - c);
        bw = d > bw ? d : bw;
      }
      if (!diag) bad |= F_NO_DIAG;
    }
    if (r == 0 && (rp[0] != 0 || rp[n] != nnz)) bad |= F_ENDS;
  }
  if (r < n_pad) row_len[r] = r < n ? len : 0;
  const int lmax = wave_max(len);
  const int bmax = wave_max(bw);
  int bor = bad;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) bor |= __shfl_xor(bor, off, 64);
  if ((threadIdx.x & 63) == 0 && r < n_pad) {
    slice_w[r / kSlice] = lmax;
    slice_b[r / kSlice] = bmax;
    slice_f[r / kSlice] = bor;
  }
}

// Exclusive scan of slice widths * 64 into slice_ptr (one 1024-thread
// block), plus the pattern summary: info = {flags (OR), bandwidth (max),
// longest row (max)} and the stored total.
__global__ void k_scan_slices(int32_t ns, const int32_t* __restrict__ w,
                              const int32_t* __restrict__ b, const int32_t* __restrict__ f,
                              int32_t* __restrict__ sp, int32_t* __restrict__ info,
                              int64_t* total) {
  __shared__ int64_t part[1024];
  __shared__ int32_t red[3][1024];
  const int t = threadIdx.x;
  const int64_t chunk = ((int64_t)ns + 1023) / 1024;
  const int64_t lo = t * chunk;
  const int64_t hi = lo + chunk < ns ? lo + chunk : ns;
  int64_t s = 0;
  int32_t fo = 0, bm = 0, wm = 0;
  for (int64_t i = lo; i < hi; ++i) {
    s += (int64_t)w[i] * kSlice;
    fo |= f[i];
    bm = b[i] > bm ? b[i] : bm;
    wm = w[i] > wm ? w[i] : wm;
  }
  red[0][t] = fo;
  red[1][t] = bm;
  red[2][t] = wm;
  part[t] = s;
  __syncthreads();
  for (int h = 512; h > 0; h >>= 1) {
    if (t < h) {
      red[0][t] |= red[0][t + h];
      red[1][t] = red[1][t + h] > red[1][t] ? red[1][t + h] : red[1][t];
      red[2][t] = red[2][t + h] > red[2][t] ? red[2][t + h] : red[2][t];
    }
    __syncthreads();
  }
  if (t == 0) {
    info[0] = red[0][0];
    info[1] = red[1][0];
    info[2] = red[2][0];
  }
  for (int off = 1; off < 1024; off <<= 1) {
    const int64_t v = t >= off ? part[t - off] : 0;
    __syncthreads();
    part[t] += v;
    __syncthreads();
  }
  int64_t run = part[t] - s;
  const bool fits = part[1023] < (int64_t)INT32_MAX;
  for (int64_t i = lo; i < hi; ++i) {
    if (fits) sp[i] = (int32_t)run;
    run += (int64_t)w[i] * kSlice;
  }
  if (t == 1023) {
    if (fits) sp[ns] = (int32_t)part[1023];
    *total = part[1023];
  }
}

__global__ void k_scatter(int32_t n, int64_t n_pad, const int32_t* __restrict__ rp,
                          const int32_t* __restrict__ ci, const double* __restrict__ mv,
                          const double* __restrict__ kv, const int32_t* __restrict__ sp,
                          const int32_t* __restrict__ row_len, int32_t* __restrict__ col,
                          int32_t* __restrict__ csr_pos, int32_t* __restrict__ diag_pos,
                          double* __restrict__ m64, double* __restrict__ k64,
                          float* __restrict__ m32, float* __restrict__ k32,
                          int8_t* __restrict__ coff) {
  const int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (r >= n_pad) return;
  const int64_t s = r / kSlice;
  const int lane = (int)(r % kSlice);
  const int32_t base = sp[s] + lane;
  const int w = (sp[s + 1] - sp[s]) / kSlice;
  const int len = row_len[r];
  diag_pos[r] = base;
  for (int k = 0; k < w; ++k) {
    const int32_t idx = base + k * kSlice;
    if (k < len) {
      const int64_t e = rp[r] + k;
      const int32_t c = ci[e];
      col[idx] = c;
      if (coff) coff[idx] = (int8_t)(c - r);
      csr_pos[idx] = (int32_t)e;
      const double a = mv[e], b = kv[e];
      m64[idx] = a;
      k64[idx] = b;
      m32[idx] = (float)a;
      k32[idx] = (float)b;
      if (c == r) diag_pos[r] = idx;
    } else {
      col[idx] = (int32_t)r;
      if (coff) coff[idx] = 0;
      csr_pos[idx] = -1;
      m64[idx] = 0.0;
      k64[idx] = 0.0;
      m32[idx] = 0.0f;
      k32[idx] = 0.0f;
    }
  }
}

// mirror[idx(r, c)] = idx(c, r), found by binary search in the sorted CSR row c.
__global__ void k_mirror(int32_t n, int64_t n_pad, const int32_t* __restrict__ rp,
                         const int32_t* __restrict__ ci, const int32_t* __restrict__ sp,
                         const int32_t* __restrict__ row_len, int32_t* __restrict__ mirror,
                         int32_t* flags) {
  const int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (r >= n_pad) return;
  const int64_t s = r / kSlice;
  const int32_t base = sp[s] + (int32_t)(r % kSlice);
  const int w = (sp[s + 1] - sp[s]) / kSlice;
  const int len = row_len[r];
  int bad = 0;
  for (int k = 0; k < w; ++k) {
    const int32_t idx = base + k * kSlice;
    int32_t m = idx;
    if (k < len) {
      const int32_t c = ci[rp[r] + k];
      int64_t lo = rp[c], hi = rp[c + 1] - 1;
      int64_t found = -1;
      while (lo <= hi) {
        const int64_t mid = (lo + hi) >> 1;
        const int32_t v = ci[mid];
        if (v == r) { found = mid; break; }
        if (v < r) lo = mid + 1; else hi = mid - 1;
      }
      if (found < 0) {
        bad = F_ASYM;
      } else {
        const int k2 = (int)(found - rp[c]);
        m = sp[c / kSlice] + k2 * kSlice + (c % kSlice);
      }
    }
    mirror[idx] = m;
  }
  if (bad) atomicOr(flags, bad);
}

// Gram scalars: per-block partial sums [MM, MK, KK, trM, trK, #bad] in
// float64, #bad counting rows with M_rr <= 0 or K_rr < 0 (then K(s) may have a
// non-positive diagonal even for s > 0).
constexpr int kGram = 6;
__global__ void k_gram_partial(PencilDev pd, double* __restrict__ part) {
  __shared__ double red[kGram][256 / 64];
  const int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  double mm = 0, mk = 0, kk = 0, tm = 0, tk = 0, bad = 0;
  if (r < pd.n) {
    const int64_t s = r / kSlice;
    const int32_t base = pd.slice_ptr[s] + (int32_t)(r % kSlice);
    const int len = pd.row_len[r];
    for (int k = 0; k < len; ++k) {
      const int32_t idx = base + k * kSlice;
      const double a = pd.m64[idx], b = pd.k64[idx];
      mm += a * a;
      mk += a * b;
      kk += b * b;
      if (pd.col[idx] == r) {
        tm += a;
        tk += b;
        if (!(a > 0.0) || !(b >= 0.0)) bad += 1.0;
      }
    }
  }
  double v[kGram] = {mm, mk, kk, tm, tk, bad};
  const int wv = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < kGram; ++q) {
    const double t = wave_sum(v[q]);
    if ((threadIdx.x & 63) == 0) red[q][wv] = t;
  }
  __syncthreads();
  if (threadIdx.x < kGram) {
    double t = 0;
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) t += red[threadIdx.x][i];
    part[(int64_t)blockIdx.x * kGram + threadIdx.x] = t;
  }
}

// Fixed-order final sum of per-block partials: out[q] = sum_b part[b*kGram + q].
__global__ void k_sum_gram(const double* __restrict__ part, int64_t nb, double* __restrict__ out) {
  __shared__ double red[kGram][256];
  const int t = threadIdx.x;
  double v[kGram] = {0, 0, 0, 0, 0, 0};
  for (int64_t b = t; b < nb; b += blockDim.x)
    for (int q = 0; q < kGram; ++q) v[q] += part[b * kGram + q];
  for (int q = 0; q < kGram; ++q) red[q][t] = v[q];
  __syncthreads();
  for (int half = blockDim.x / 2; half > 0; half >>= 1) {
    if (t < half)
      for (int q = 0; q < kGram; ++q) red[q][t] += red[q][t + half];
    __syncthreads();
  }
  if (t < kGram) out[t] = red[t][0];
}

// The identity on the stored pattern: 1 at each diagonal entry, 0 elsewhere.
__global__ void k_identity(PencilDev pd, int64_t n_pad, double* __restrict__ v64,
                           float* __restrict__ v32) {
  const int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (r >= n_pad) return;
  const int64_t s = r / kSlice;
  const int32_t base = pd.slice_ptr[s] + (int32_t)(r % kSlice);
  const int w = (pd.slice_ptr[s + 1] - pd.slice_ptr[s]) / kSlice;
  const int len = pd.row_len[r];
  for (int k = 0; k < w; ++k) {
    const int32_t idx = base + k * kSlice;
    const double v = (k < len && pd.col[idx] == r) ? 1.0 : 0.0;
    v64[idx] = v;
    v32[idx] = (float)v;
  }
}

__global__ void k_assemble(PencilDev pd, int64_t stored, double a, double b,
                           double* __restrict__ out) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= stored) return;
  const int32_t e = pd.csr_pos[i];
  if (e >= 0) out[e] = fma(a, pd.m64[i], b * pd.k64[i]);
}

// y = (a M + b K) x, float64, one row per thread, blockIdx.y = vector.
__global__ void k_apply_shift(PencilDev pd, double a, double b, const double* __restrict__ x,
                              int64_t ldx, double* __restrict__ y, int64_t ldy) {
  const int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (r >= pd.n) return;
  const double* xv = x + (int64_t)blockIdx.y * ldx;
  const int64_t s = r / kSlice;
  const int32_t base = pd.slice_ptr[s] + (int32_t)(r % kSlice);
  const int w = (pd.slice_ptr[s + 1] - pd.slice_ptr[s]) / kSlice;
  double am = 0, ak = 0;
  for (int k = 0; k < w; ++k) {
    const int32_t idx = base + k * kSlice;
    const double xc = xv[pd.col[idx]];
    am = fma(pd.m64[idx], xc, am);
    ak = fma(pd.k64[idx], xc, ak);
  }
  y[(int64_t)blockIdx.y * ldy + r] = fma(a, am, b * ak);
}

static airga_status set_pencil_impl(airga_ctx ctx, int32_t n, int64_t nnz, const int32_t* row_ptr,
                                    const int32_t* col_idx, const double* m_val,
                                    const double* k_val, double alpha, double beta) {
  Pencil& pen = ctx->pen;
  pen.valid = false;
  pen.generation++;
  hipStream_t st = ctx->stream;
  const int32_t ns = (int32_t)((n + kSlice - 1) / kSlice);
  const int64_t n_pad = (int64_t)ns * kSlice;
  // setup scratch, kept with the pencil: [info (3) | total | per-slice
  // widths, bands, flags]
  const size_t off_w = 64;
  AIRGA_TRY(pen.setup.reserve(off_w + 3 * sizeof(int32_t) * (size_t)ns));
  int32_t* info = pen.setup.as<int32_t>();
  int64_t* total = reinterpret_cast<int64_t*>(pen.setup.as<char>() + 16);
  int32_t* slice_w = reinterpret_cast<int32_t*>(pen.setup.as<char>() + off_w);
  int32_t* slice_b = slice_w + ns;
  int32_t* slice_f = slice_b + ns;
  AIRGA_TRY(pen.row_len.reserve(sizeof(int32_t) * n_pad));
  AIRGA_TRY(pen.slice_ptr.reserve(sizeof(int32_t) * (ns + 1)));
  k_rows_check<<<blocks_for(n_pad, 256), 256, 0, st>>>(n, nnz, n_pad, row_ptr, col_idx,
                                                       pen.row_len.as<int32_t>(), slice_w, slice_b,
                                                       slice_f);
  AIRGA_HIP(hipGetLastError());
  k_scan_slices<<<1, 1024, 0, st>>>(ns, slice_w, slice_b, slice_f, pen.slice_ptr.as<int32_t>(),
                                    info, total);
  AIRGA_HIP(hipGetLastError());
  struct Summary {
    int32_t flags, bw, maxlen, pad;
    int64_t total;
  };
  // host reads go through the context's pinned buffer (asynchronous copies)
  AIRGA_TRY(ensure_pinned(ctx, 4096));
  AIRGA_HIP(hipMemcpyAsync(ctx->host_pinned, pen.setup.ptr, sizeof(Summary), hipMemcpyDeviceToHost, st));
  AIRGA_HIP(hipStreamSynchronize(st));
  Summary h;
  std::memcpy(&h, ctx->host_pinned, sizeof h);
  if (h.flags & F_TOO_LONG)
    return fail(AIRGA_EUNSUPPORTED, "pattern has a row longer than %d entries", kMaxRow);
  if (h.flags & ~F_GAPPED) {
    std::string why;
    if (h.flags & F_ROWPTR) why += " row_ptr out of order or range;";
    if (h.flags & F_COL_RANGE) why += " column index out of range;";
    if (h.flags & F_UNSORTED) why += " columns not strictly increasing within a row;";
    if (h.flags & F_NO_DIAG) why += " a diagonal entry is missing;";
    if (h.flags & F_ENDS) why += " row_ptr[0] != 0 or row_ptr[n] != nnz;";
    return fail(AIRGA_EINVAL, "invalid pattern:%s", why.c_str());
  }
  if (h.total >= (int64_t)INT32_MAX)
    return fail(AIRGA_EUNSUPPORTED, "sliced-ELL copy needs %lld entries (limit 2^31)",
                (long long)h.total);
  const int64_t stored = h.total;
  AIRGA_TRY(pen.col.reserve(sizeof(int32_t) * stored));
  AIRGA_TRY(pen.mirror.reserve(sizeof(int32_t) * stored));
  AIRGA_TRY(pen.csr_pos.reserve(sizeof(int32_t) * stored));
  AIRGA_TRY(pen.diag_pos.reserve(sizeof(int32_t) * n_pad));
  AIRGA_TRY(pen.m64.reserve(sizeof(double) * stored));
  AIRGA_TRY(pen.k64.reserve(sizeof(double) * stored));
  AIRGA_TRY(pen.m32.reserve(sizeof(float) * stored));
  AIRGA_TRY(pen.k32.reserve(sizeof(float) * stored));
  const bool banded = h.bw <= kSlice;
  if (banded) AIRGA_TRY(pen.coff.reserve(stored));
  k_scatter<<<blocks_for(n_pad, 256), 256, 0, st>>>(
      n, n_pad, row_ptr, col_idx, m_val, k_val, pen.slice_ptr.as<int32_t>(),
      pen.row_len.as<int32_t>(), pen.col.as<int32_t>(), pen.csr_pos.as<int32_t>(),
      pen.diag_pos.as<int32_t>(), pen.m64.as<double>(), pen.k64.as<double>(),
      pen.m32.as<float>(), pen.k32.as<float>(), banded ? pen.coff.as<int8_t>() : nullptr);
  AIRGA_HIP(hipGetLastError());
  k_mirror<<<blocks_for(n_pad, 256), 256, 0, st>>>(n, n_pad, row_ptr, col_idx,
                                                   pen.slice_ptr.as<int32_t>(),
                                                   pen.row_len.as<int32_t>(),
                                                   pen.mirror.as<int32_t>(), info);
  AIRGA_HIP(hipGetLastError());
  pen.n = n;
  pen.n_slices = ns;
  pen.nnz = nnz;
  pen.nnz_stored = stored;
  pen.uniform_width = stored == (int64_t)ns * kSlice * h.maxlen;
  pen.contiguous = (h.flags & F_GAPPED) == 0;
  pen.max_len = h.maxlen;
  pen.bandwidth = h.bw;
  pen.alpha = alpha;
  pen.beta = beta;
  AIRGA_TRY(pen.id64.reserve(sizeof(double) * stored));
  AIRGA_TRY(pen.id32.reserve(sizeof(float) * stored));
  k_identity<<<blocks_for(n_pad, 256), 256, 0, st>>>(pen.dev(), n_pad, pen.id64.as<double>(),
                                                     pen.id32.as<float>());
  AIRGA_HIP(hipGetLastError());
  // Gram scalars
  const unsigned nb = blocks_for(n, 256);
  DevBuf& gp = pen.gram_ws;
  AIRGA_TRY(gp.reserve(sizeof(double) * (kGram * (size_t)nb + kGram)));
  k_gram_partial<<<nb, 256, 0, st>>>(pen.dev(), gp.as<double>());
  AIRGA_HIP(hipGetLastError());
  k_sum_gram<<<1, 256, 0, st>>>(gp.as<double>(), nb, gp.as<double>() + kGram * (size_t)nb);
  AIRGA_HIP(hipGetLastError());
  double g[kGram];
  int32_t flags2 = 0;
  char* hp = static_cast<char*>(ctx->host_pinned);
  AIRGA_HIP(hipMemcpyAsync(hp, gp.as<double>() + kGram * (size_t)nb, sizeof g, hipMemcpyDeviceToHost, st));
  AIRGA_HIP(hipMemcpyAsync(hp + sizeof g, info, 4, hipMemcpyDeviceToHost, st));
  AIRGA_HIP(hipStreamSynchronize(st));
  std::memcpy(g, hp, sizeof g);
  std::memcpy(&flags2, hp + sizeof g, 4);
  if (flags2 & F_ASYM) return fail(AIRGA_EINVAL, "invalid pattern: not structurally symmetric");
  pen.gram_mm = g[0];
  pen.gram_mk = g[1];
  pen.gram_kk = g[2];
  pen.tr_m = g[3];
  pen.tr_k = g[4];
  pen.diag_ok = g[5] == 0.0;
  pen.valid = true;
  return AIRGA_OK;
}

}  // namespace airga

using namespace airga;

extern "C" {

const char* airga_last_error(void) { return g_err.c_str(); }

const char* airga_version(void) { return "0.1.0"; }

airga_status airga_create(airga_ctx* out, int device, void* stream) {
  if (!out) return fail(AIRGA_EINVAL, "null output pointer");
  *out = nullptr;
  int count = 0;
  AIRGA_HIP(hipGetDeviceCount(&count));
  if (device < 0 || device >= count)
    return fail(AIRGA_EINVAL, "device %d out of range (%d devices)", device, count);
  DeviceGuard g(device);
  airga_ctx c = new (std::nothrow) airga_ctx_s();
  if (!c) return fail(AIRGA_ENOMEM, "host allocation failed");
  c->device = device;
  if (stream) {
    c->stream = static_cast<hipStream_t>(stream);
  } else {
    hipError_t e = hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking);
    if (e != hipSuccess) {
      delete c;
      return fail(AIRGA_EHIP, "hipStreamCreateWithFlags: %s", hipGetErrorString(e));
    }
    c->own_stream = true;
  }
  const airga_status st = gram_scratch_address(device, &c->gram_scratch);
  if (st != AIRGA_OK) {
    if (c->own_stream) (void)hipStreamDestroy(c->stream);
    delete c;
    return st;
  }
  *out = c;
  return AIRGA_OK;
}

void airga_destroy(airga_ctx ctx) {
  if (!ctx) return;
  DeviceGuard g(ctx->device);
  (void)hipStreamSynchronize(ctx->stream);
  if (ctx->host_pinned) (void)hipHostFree(ctx->host_pinned);
  if (ctx->own_stream) (void)hipStreamDestroy(ctx->stream);
  delete ctx;
}

airga_status airga_set_pencil(airga_ctx ctx, int32_t n, int64_t nnz, const int32_t* row_ptr,
                              const int32_t* col_idx, const double* m_val, const double* k_val,
                              double alpha, double beta) {
  AIRGA_TRY(check_ctx(ctx));
  DeviceGuard g(ctx->device);
  if (n <= 0 || nnz <= 0) return fail(AIRGA_EINVAL, "n and nnz must be positive");
  if (!row_ptr || !col_idx || !m_val || !k_val) return fail(AIRGA_EINVAL, "null pencil array");
  if (!std::isfinite(alpha) || !std::isfinite(beta) || alpha < 0 || beta < 0)
    return fail(AIRGA_EINVAL, "damping coefficients must be finite and >= 0");
  if (nnz > (int64_t)n * kMaxRow)
    return fail(AIRGA_EUNSUPPORTED, "pattern has a row longer than %d entries", kMaxRow);
  airga_status s = set_pencil_impl(ctx, n, nnz, row_ptr, col_idx, m_val, k_val, alpha, beta);
  if (s != AIRGA_OK) ctx->pen.valid = false;
  return s;
}

airga_status airga_get_pencil_info(airga_ctx ctx, airga_pencil_info* out) {
  AIRGA_TRY(check_pencil(ctx));
  if (!out) return fail(AIRGA_EINVAL, "null output");
  const Pencil& p = ctx->pen;
  out->n = p.n;
  out->max_row_len = p.max_len;
  out->bandwidth = p.bandwidth;
  out->slice_rows = kSlice;
  out->nnz = p.nnz;
  out->nnz_stored = p.nnz_stored;
  out->gram_mm = p.gram_mm;
  out->gram_mk = p.gram_mk;
  out->gram_kk = p.gram_kk;
  out->trace_m = p.tr_m;
  out->trace_k = p.tr_k;
  return AIRGA_OK;
}

airga_status airga_assemble_shift(airga_ctx ctx, double s, double* a_val) {
  AIRGA_TRY(check_pencil(ctx));
  DeviceGuard g(ctx->device);
  if (!a_val) return fail(AIRGA_EINVAL, "null output array");
  if (!std::isfinite(s)) return fail(AIRGA_EINVAL, "shift must be finite");
  double a, b;
  shift_coeffs(ctx->pen, s, &a, &b);
  k_assemble<<<blocks_for(ctx->pen.nnz_stored, 256), 256, 0, ctx->stream>>>(
      ctx->pen.dev(), ctx->pen.nnz_stored, a, b, a_val);
  AIRGA_HIP(hipGetLastError());
  return AIRGA_OK;
}

airga_status airga_apply_shift(airga_ctx ctx, double s, int32_t count, const double* x,
                               int64_t ldx, double* y, int64_t ldy) {
  AIRGA_TRY(check_pencil(ctx));
  DeviceGuard g(ctx->device);
  if (count < 0 || (count > 0 && (!x || !y))) return fail(AIRGA_EINVAL, "bad vectors");
  if (count > 65535) return fail(AIRGA_EUNSUPPORTED, "more than 65535 vectors");
  if (ldx < ctx->pen.n || ldy < ctx->pen.n) return fail(AIRGA_EINVAL, "leading dimension < n");
  if (!std::isfinite(s)) return fail(AIRGA_EINVAL, "shift must be finite");
  if (count == 0) return AIRGA_OK;
  double a, b;
  shift_coeffs(ctx->pen, s, &a, &b);
  dim3 grid(blocks_for(ctx->pen.n, 256), (unsigned)count);
  k_apply_shift<<<grid, 256, 0, ctx->stream>>>(ctx->pen.dev(), a, b, x, ldx, y, ldy);
  AIRGA_HIP(hipGetLastError());
  return AIRGA_OK;
}

airga_status airga_shift_diagnostics(airga_ctx ctx, double s_old, double s_new, double* out) {
  AIRGA_TRY(check_pencil(ctx));
  if (!out) return fail(AIRGA_EINVAL, "null output");
  if (!std::isfinite(s_old) || !std::isfinite(s_new)) return fail(AIRGA_EINVAL, "shift must be finite");
  const Pencil& p = ctx->pen;
  double ao, bo, an, bn;
  shift_coeffs(p, s_old, &ao, &bo);
  shift_coeffs(p, s_new, &an, &bn);
  const double nn = an * an * p.gram_mm + 2 * an * bn * p.gram_mk + bn * bn * p.gram_kk;
  const double tr = an * p.tr_m + bn * p.tr_k;
  const double da = ao - an, db = bo - bn;
  const double dd = da * da * p.gram_mm + 2 * da * db * p.gram_mk + db * db * p.gram_kk;
  const double on = ao * an * p.gram_mm + (ao * bn + an * bo) * p.gram_mk + bo * bn * p.gram_kk;
  const double i_a = (double)p.n - 2 * tr + nn;
  out[0] = std::sqrt(i_a > 0 ? i_a : 0.0);
  out[1] = std::sqrt(dd > 0 ? dd : 0.0);
  out[2] = tr / nn;
  out[3] = on / nn;
  return AIRGA_OK;
}

}  // extern "C"
