// Block operations of the moment sequence of AIRGA (Section 2, Algorithms 1
// and 3): right-hand sides (a M + b K) X, tall-skinny products A^T B over
// the pencil's n rows, orthogonalisation of n x m blocks in the trace inner
// product (global Arnoldi), the thin QR of the collected blocks, and the
// Galerkin projection of eq. (1.4).  Every product over the n rows is a
// fixed-order sum (per-block partials, then one reduction), so results do not
// depend on scheduling.
#include <cmath>
#include <cstring>
#include <mutex>
#include <vector>

#include "internal.hpp"

namespace airga {

// ------------------------------------------------------- pencil products
//
// Y1 = (a1 M + b1 K) X and, when Y2 is given, Y2 = (a2 M + b2 K) X for the
// count columns of X.  One thread per row keeps the row's entries in
// registers and walks the columns, so the pencil is read once for all of
// them (entries past a slice's width act as padding: the row itself, value
// 0).  Each row sums its entries in stored order, as the single-vector
// product does.
template <int WMAX>
__global__ void __launch_bounds__(256) k_spmm_pencil(PencilDev pd, int32_t count,
                                                     const double* __restrict__ X, int64_t ldx,
                                                     double a1, double b1, double* __restrict__ Y1,
                                                     int64_t ldy1, double a2, double b2,
                                                     double* __restrict__ Y2, int64_t ldy2) {
  const int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (r >= pd.n) return;
  const int64_t s = r / kSlice;
  const int32_t base = pd.slice_ptr[s] + (int32_t)(r % kSlice);
  const int w = (pd.slice_ptr[s + 1] - pd.slice_ptr[s]) / kSlice;
  int32_t col[WMAX];
  double mv[WMAX], kv[WMAX];
#pragma unroll
  for (int k = 0; k < WMAX; ++k) {
    const bool in = k < w;
    const int32_t idx = base + k * kSlice;
    col[k] = in ? pd.col[idx] : (int32_t)r;
    mv[k] = in ? pd.m64[idx] : 0.0;
    kv[k] = in ? pd.k64[idx] : 0.0;
  }
#pragma unroll 4
  for (int c = 0; c < count; ++c) {
    const double* __restrict__ x = X + (int64_t)c * ldx;
    double am = 0, ak = 0;
#pragma unroll
    for (int k = 0; k < WMAX; ++k) {
      const double xc = x[col[k]];
      am = fma(mv[k], xc, am);
      ak = fma(kv[k], xc, ak);
    }
    Y1[(int64_t)c * ldy1 + r] = fma(a1, am, b1 * ak);
    if (Y2) Y2[(int64_t)c * ldy2 + r] = fma(a2, am, b2 * ak);
  }
}

static void spmm_pencil(airga_ctx ctx, int32_t count, const double* X, int64_t ldx, double a1,
                        double b1, double* Y1, int64_t ldy1, double a2, double b2, double* Y2,
                        int64_t ldy2) {
  const Pencil& pen = ctx->pen;
  const unsigned grid = blocks_for(pen.n, 256);
  const PencilDev pd = pen.dev();
  if (pen.max_len <= 6)
    k_spmm_pencil<6><<<grid, 256, 0, ctx->stream>>>(pd, count, X, ldx, a1, b1, Y1, ldy1, a2, b2,
                                                    Y2, ldy2);
  else if (pen.max_len <= 8)
    k_spmm_pencil<8><<<grid, 256, 0, ctx->stream>>>(pd, count, X, ldx, a1, b1, Y1, ldy1, a2, b2,
                                                    Y2, ldy2);
  else
    k_spmm_pencil<kMaxRow><<<grid, 256, 0, ctx->stream>>>(pd, count, X, ldx, a1, b1, Y1, ldy1, a2,
                                                          b2, Y2, ldy2);
}

// ------------------------------------------------------------ A^T B kernel
//
// A block sums kGramRowsPerBlock rows for one 64 x 64 tile of the output
// (grid.y, grid.z index the tile), kGramStage rows at a time staged in LDS.
// The products run on the matrix cores: wavefront w owns output rows
// 16 w .. 16 w + 15 and all four 16-column tiles, and each
// v_mfma_f64_16x16x4f64 adds the contribution of 4 staged rows to one
// 16 x 16 tile (operand A = the 16 x 4 slice of A^T, lane i + 16 q holding
// A(row q, column i); operand B = the 4 x 16 slice of B, lane j + 16 q
// holding B(row q, column j); element v of the accumulator holds output
// (lane / 16 + 4 v, lane % 16)).  Block b takes the stages b, b + nblk, ...:
// the blocks running together read consecutive stages.  The next stage's
// loads are issued into registers before the current one is multiplied, so
// they are in flight during the matrix-core work.
constexpr int kGT = 64;
constexpr int kGramStage = 16;
constexpr int64_t kGramRowsPerBlock = 1024;
// Widest operand of a product (the partials take (k/64)(l/64) n/128 KiB).
constexpr int kGramMax = 256;

__global__ void __launch_bounds__(256) k_gram_partial(int64_t n, int32_t k,
                                                      const double* __restrict__ A, int64_t lda,
                                                      int32_t l, const double* __restrict__ B,
                                                      int64_t ldb, double* __restrict__ part) {
  // +1 column: the staging stores of a wavefront (consecutive rows of one
  // column) fall in distinct banks
  __shared__ double As[kGramStage][kGT + 1];
  __shared__ double Bs[kGramStage][kGT + 1];
  typedef double d4 __attribute__((ext_vector_type(4)));
  const int t = threadIdx.x;
  const int wv = t >> 6, lane = t & 63;
  const int li = lane & 15, lq = lane >> 4;
  const int ca0 = blockIdx.y * kGT, cb0 = blockIdx.z * kGT;
  d4 acc[4];
#pragma unroll
  for (int jt = 0; jt < 4; ++jt) acc[jt] = d4{0.0, 0.0, 0.0, 0.0};
  const int64_t stride = (int64_t)gridDim.x * kGramStage;
  // element e = t + 256 q of a stage: row e % kGramStage, column e / kGramStage
  constexpr int Q = kGramStage * kGT / 256;
  double pa[Q], pb[Q];
  auto fetch = [&](int64_t rb) {
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int e = t + 256 * q;
      const int64_t row = rb + (e & (kGramStage - 1));
      const int ca = ca0 + e / kGramStage, cb = cb0 + e / kGramStage;
      pa[q] = (row < n && ca < k) ? A[row + (int64_t)ca * lda] : 0.0;
      pb[q] = (row < n && cb < l) ? B[row + (int64_t)cb * ldb] : 0.0;
    }
  };
  int64_t rb = (int64_t)blockIdx.x * kGramStage;
  if (rb < n) fetch(rb);
  for (; rb < n; rb += stride) {
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int e = t + 256 * q;
      As[e & (kGramStage - 1)][e / kGramStage] = pa[q];
      Bs[e & (kGramStage - 1)][e / kGramStage] = pb[q];
    }
    __syncthreads();
    if (rb + stride < n) fetch(rb + stride);
#pragma unroll
    for (int s4 = 0; s4 < kGramStage; s4 += 4) {
      const double a = As[s4 + lq][16 * wv + li];
#pragma unroll
      for (int jt = 0; jt < 4; ++jt) {
        const double b = Bs[s4 + lq][16 * jt + li];
        acc[jt] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[jt], 0, 0, 0);
      }
    }
    __syncthreads();
  }
  double* out = part + ((int64_t)(blockIdx.y * gridDim.z + blockIdx.z) * gridDim.x + blockIdx.x) *
                           (kGT * kGT);
#pragma unroll
  for (int jt = 0; jt < 4; ++jt)
#pragma unroll
    for (int v = 0; v < 4; ++v) out[(16 * wv + lq + 4 * v) * kGT + 16 * jt + li] = acc[jt][v];
}

// G[i + j ldg] = sum over the row blocks of the tile partials, in a fixed
// order: a block takes 16 outputs (consecutive j, so the partial reads of a
// step are contiguous) and 16 splits of the row blocks; split s sums its
// contiguous range, then the 16 split sums are added in split order.
constexpr int kRedOut = 16, kRedSplit = 16;

__global__ void __launch_bounds__(256) k_gram_reduce(int32_t k, int32_t l, int nblk, int tiles_l,
                                                     const double* __restrict__ part,
                                                     double* __restrict__ G, int64_t ldg) {
  __shared__ double red[kRedSplit][kRedOut];
  const int to = threadIdx.x % kRedOut, sp = threadIdx.x / kRedOut;
  const int64_t idx = (int64_t)blockIdx.x * kRedOut + to;
  const bool in = idx < (int64_t)k * l;
  const int i = in ? (int)(idx / l) : 0, j = in ? (int)(idx % l) : 0;
  const double* p = part + (int64_t)((i / kGT) * tiles_l + j / kGT) * nblk * (kGT * kGT) +
                    (i % kGT) * kGT + j % kGT;
  const int chunk = (nblk + kRedSplit - 1) / kRedSplit;
  const int b0 = sp * chunk, b1 = b0 + chunk < nblk ? b0 + chunk : nblk;
  double s = 0.0;
  if (in) {
#pragma unroll 8
    for (int b = b0; b < b1; ++b) s += p[(int64_t)b * (kGT * kGT)];
  }
  red[sp][to] = s;
  __syncthreads();
  if (sp == 0 && in) {
    double t = 0.0;
    for (int q = 0; q < kRedSplit; ++q) t += red[q][to];
    G[i + (int64_t)j * ldg] = t;
  }
}

// Launch of the two Gram kernels with nblk row blocks per output tile and
// the partials in part (tk * tl * nblk * 64 * 64 doubles, every one written
// by k_gram_partial, so part needs no clearing).  Block b of a tile takes the
// row stages b, b + nblk, ..., so any nblk >= 1 covers all n rows.
static airga_status gram_launch(airga_ctx ctx, int64_t n, int32_t k, const double* A, int64_t lda,
                                int32_t l, const double* B, int64_t ldb, double* G, int64_t ldg,
                                int nblk, double* part) {
  const int tk = (k + kGT - 1) / kGT, tl = (l + kGT - 1) / kGT;
  k_gram_partial<<<dim3((unsigned)nblk, (unsigned)tk, (unsigned)tl), 256, 0, ctx->stream>>>(
      n, k, A, lda, l, B, ldb, part);
  AIRGA_HIP(hipGetLastError());
  k_gram_reduce<<<blocks_for((int64_t)k * l, kRedOut), 256, 0, ctx->stream>>>(k, l, nblk, tl, part,
                                                                             G, ldg);
  AIRGA_HIP(hipGetLastError());
  return AIRGA_OK;
}

// G = 0 for a product over no rows.
static airga_status gram_zero(airga_ctx ctx, int32_t l, double* G, int64_t ldg) {
  k_fill_f64<<<blocks_for((int64_t)ldg * l, 256), 256, 0, ctx->stream>>>(G, ldg * l, 0.0);
  AIRGA_HIP(hipGetLastError());
  return AIRGA_OK;
}

// G (device, k x l, column-major with leading dimension ldg) = A^T B over n
// rows.  Partials go to the context's Gram workspace.
static airga_status gram(airga_ctx ctx, int64_t n, int32_t k, const double* A, int64_t lda,
                         int32_t l, const double* B, int64_t ldb, double* G, int64_t ldg) {
  if (k == 0 || l == 0) return AIRGA_OK;
  if (n == 0) return gram_zero(ctx, l, G, ldg);
  const int nblk = (int)((n + kGramRowsPerBlock - 1) / kGramRowsPerBlock);
  const int tk = (k + kGT - 1) / kGT, tl = (l + kGT - 1) / kGT;
  AIRGA_TRY(ctx->ws_gram.reserve(sizeof(double) * (size_t)tk * tl * nblk * kGT * kGT));
  return gram_launch(ctx, n, k, A, lda, l, B, ldb, G, ldg, nblk, ctx->ws_gram.as<double>());
}

// ------------------------------------------ A^T B without allocation
//
// The partials of airga_gram_noalloc live in a fixed device array, one per
// GPU, held until the process ends.  32 MiB holds 1024 partial tiles of
// 64 x 64: up to 1024 row blocks of 1024 rows for one output tile (so
// products over n <= 1,048,576 rows with k, l <= 64 are summed exactly as
// airga_gram sums them), and 1024 / (tiles of the output) blocks per tile
// for wider products, each block then taking more rows.  Calls that overlap
// on one GPU share the array and race.
constexpr size_t kGramScratchBytes = size_t(32) << 20;
constexpr int64_t kGramScratchTiles = (int64_t)(kGramScratchBytes / (sizeof(double) * kGT * kGT));
static __device__ __align__(256) double scratch[kGramScratchBytes / sizeof(double)];

// Device address of `scratch` per GPU, looked up once per device (host code
// must not pass the array's own name to a kernel: on the host it is only a
// stand-in for the device symbol).
static std::mutex g_scratch_mu;
static std::vector<double*> g_scratch_addr;

airga_status gram_scratch_address(int device, double** out) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (device < 0) return fail(AIRGA_EINVAL, "bad device %d", device);
  if ((size_t)device >= g_scratch_addr.size()) g_scratch_addr.resize(device + 1, nullptr);
  if (!g_scratch_addr[device]) {
    DeviceGuard g(device);
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return fail(AIRGA_EHIP, "hipGetSymbolAddress(scratch) on device %d: %s", device,
                  hipGetErrorString(e));
    g_scratch_addr[device] = static_cast<double*>(ptr);
  }
  *out = g_scratch_addr[device];
  return AIRGA_OK;
}

// Host copy of a device k x l result (synchronises the context stream).
static airga_status to_host(airga_ctx ctx, const double* d, size_t count, double* h) {
  AIRGA_TRY(ensure_pinned(ctx, sizeof(double) * count));
  AIRGA_HIP(hipMemcpyAsync(ctx->host_pinned, d, sizeof(double) * count, hipMemcpyDeviceToHost,
                           ctx->stream));
  AIRGA_HIP(hipStreamSynchronize(ctx->stream));
  std::memcpy(h, ctx->host_pinned, sizeof(double) * count);
  return AIRGA_OK;
}

// Device copy of a host array, through the pinned area (synchronises first,
// since the area may still feed an earlier copy).
static airga_status to_device(airga_ctx ctx, const double* h, size_t count, double* d) {
  AIRGA_HIP(hipStreamSynchronize(ctx->stream));
  AIRGA_TRY(ensure_pinned(ctx, sizeof(double) * count));
  std::memcpy(ctx->host_pinned, h, sizeof(double) * count);
  AIRGA_HIP(hipMemcpyAsync(d, ctx->host_pinned, sizeof(double) * count, hipMemcpyHostToDevice,
                           ctx->stream));
  AIRGA_HIP(hipStreamSynchronize(ctx->stream));
  return AIRGA_OK;
}

// ------------------------------------------------- global orthogonalisation
//
// For the nx blocks X_x (n x m) and the nb blocks V_t:
//   X_x <- X_x - sum_t gamma[x][t] V_t,   squared Frobenius norms of X_x.
// One thread per (row, column c): the nb entries V_t(row, c) stay in
// registers while the thread walks the blocks X_x.
constexpr int kOrthMaxBlocks = 16;

// part[x * (4 gridDim.x) + wave]: one partial per wavefront and block, so the
// walk over the blocks needs no barrier.
__global__ void __launch_bounds__(256) k_orth_update(int64_t n, int32_t m, int32_t nb,
                                                     const double* __restrict__ V, int64_t ldv,
                                                     int32_t nx, double* __restrict__ X,
                                                     int64_t ldx, const double* __restrict__ gam,
                                                     double* __restrict__ part) {
  const int64_t wave = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int64_t nwaves = (int64_t)gridDim.x * 4;
  const int64_t item = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const bool in = item < n * m;
  const int64_t row = in ? item / m : 0;
  const int c = in ? (int)(item % m) : 0;
  double v[kOrthMaxBlocks];
#pragma unroll
  for (int t = 0; t < kOrthMaxBlocks; ++t)
    v[t] = (in && t < nb) ? V[row + (int64_t)(t * m + c) * ldv] : 0.0;
  for (int x = 0; x < nx; ++x) {
    double s = 0.0;
    if (in) {
      double* px = X + row + (int64_t)(x * m + c) * ldx;
      double xv = *px;
      const double* g = gam + (int64_t)x * nb;
#pragma unroll
      for (int t = 0; t < kOrthMaxBlocks; ++t)
        if (t < nb) xv = fma(-sload(g + t), v[t], xv);
      *px = xv;
      s = xv * xv;
    }
    s = wave_total(s);
    if ((threadIdx.x & 63) == 0) part[(int64_t)x * nwaves + wave] = s;
  }
}

// out[x] = sum of part[x][0 .. np): one block per row x; thread t sums the
// entries t, t + 256, ... in order, then thread 0 adds the 256 sums in order.
__global__ void __launch_bounds__(256) k_sum_rows(int64_t np, const double* __restrict__ part,
                                                  double* __restrict__ out) {
  __shared__ double red[256];
  const double* p = part + (int64_t)blockIdx.x * np;
  double s = 0.0;
#pragma unroll 8
  for (int64_t b = threadIdx.x; b < np; b += 256) s += p[b];
  red[threadIdx.x] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int q = 0; q < 256; ++q) t += red[q];
    out[blockIdx.x] = t;
  }
}

// X_x <- X_x * scale[x] for the nx blocks of m columns.
__global__ void k_scale_blocks(int64_t n, int32_t m, double* __restrict__ X, int64_t ldx,
                               const double* __restrict__ scale) {
  const int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int col = blockIdx.y;
  if (r >= n) return;
  X[r + (int64_t)col * ldx] *= sload(scale + col / m);
}

// ------------------------------------------------------------ thin QR
//
// W <- W T for an upper-triangular k x k T (k <= 64): output column j of a
// row is sum_{i <= j} W(row, i) T(i, j).  One thread per row, 32 output
// columns at a time, the upper half first: columns j only read W(:, i <= j),
// so the lower half still finds the entries it needs unchanged.  The row's
// entries are loaded 8 at a time, the next 8 while the current ones are
// multiplied.
constexpr int kQrMax = 64;

__global__ void __launch_bounds__(256) k_right_trmm(int64_t n, int32_t k, double* __restrict__ W,
                                                    int64_t ldw, const double* __restrict__ T) {
  __shared__ double Ts[kQrMax * kQrMax];
  for (int e = threadIdx.x; e < kQrMax * kQrMax; e += blockDim.x) {
    const int i = e / kQrMax, j = e % kQrMax;  // Ts row-major: row i of T
    Ts[e] = (i < k && j < k) ? T[i + (int64_t)j * k] : 0.0;
  }
  __syncthreads();
  const int64_t row = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (row >= n) return;
  double* w = W + row;
  for (int j0 = ((k - 1) / 32) * 32; j0 >= 0; j0 -= 32) {
    double acc[32];
#pragma unroll
    for (int jj = 0; jj < 32; ++jj) acc[jj] = 0.0;
    const int iend = j0 + 32 < k ? j0 + 32 : k;
    double wc[8], wn[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) wc[u] = u < iend ? w[(int64_t)u * ldw] : 0.0;
    for (int i0 = 0; i0 < iend; i0 += 8) {
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int i = i0 + 8 + u;
        wn[u] = i < iend ? w[(int64_t)i * ldw] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        // rows i >= k of Ts are zero, so a chunk past iend adds nothing
        const double* trow = Ts + (i0 + u) * kQrMax + j0;
#pragma unroll
        for (int jj = 0; jj < 32; ++jj) acc[jj] = fma(wc[u], trow[jj], acc[jj]);
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) wc[u] = wn[u];
    }
#pragma unroll
    for (int jj = 0; jj < 32; ++jj)
      if (j0 + jj < k) w[(int64_t)(j0 + jj) * ldw] = acc[jj];
  }
}

// Upper Cholesky factor R (R^T R = G) of a k x k column-major G, in place of
// its upper triangle (the strict lower triangle is zeroed).  False when a
// pivot is not positive.
static bool cholesky_upper(int k, double* G) {
  for (int j = 0; j < k; ++j) {
    double d = G[j + j * k];
    for (int p = 0; p < j; ++p) d -= G[p + j * k] * G[p + j * k];
    if (!(d > 0.0) || !std::isfinite(d)) return false;
    const double rjj = std::sqrt(d);
    G[j + j * k] = rjj;
    for (int i = j + 1; i < k; ++i) {
      double s = G[j + i * k];
      for (int p = 0; p < j; ++p) s -= G[p + j * k] * G[p + i * k];
      G[j + i * k] = s / rjj;
    }
    for (int i = j + 1; i < k; ++i) G[i + j * k] = 0.0;
  }
  return true;
}

// Inverse of an upper-triangular k x k R (column-major) by back
// substitution, column by column.
static void upper_inverse(int k, const double* R, double* T) {
  for (int e = 0; e < k * k; ++e) T[e] = 0.0;
  for (int j = 0; j < k; ++j) {
    T[j + j * k] = 1.0 / R[j + j * k];
    for (int i = j - 1; i >= 0; --i) {
      double s = 0.0;
      for (int p = i + 1; p <= j; ++p) s += R[i + p * k] * T[p + j * k];
      T[i + j * k] = -s / R[i + i * k];
    }
  }
}

}  // namespace airga

using namespace airga;

extern "C" {

airga_status airga_pencil_apply(airga_ctx ctx, double a, double b, int32_t count, const double* x,
                                int64_t ldx, double* y, int64_t ldy) {
  AIRGA_TRY(check_pencil(ctx));
  DeviceGuard g(ctx->device);
  if (count < 0 || (count > 0 && (!x || !y))) return fail(AIRGA_EINVAL, "bad vectors");
  if (count > 65535) return fail(AIRGA_EUNSUPPORTED, "more than 65535 vectors");
  if (ldx < ctx->pen.n || ldy < ctx->pen.n) return fail(AIRGA_EINVAL, "leading dimension < n");
  if (!std::isfinite(a) || !std::isfinite(b)) return fail(AIRGA_EINVAL, "coefficients must be finite");
  if (count == 0) return AIRGA_OK;
  spmm_pencil(ctx, count, x, ldx, a, b, y, ldy, 0.0, 0.0, nullptr, 0);
  AIRGA_HIP(hipGetLastError());
  return AIRGA_OK;
}

airga_status airga_gram(airga_ctx ctx, int32_t k, const double* A, int64_t lda, int32_t l,
                        const double* B, int64_t ldb, double* G) {
  AIRGA_TRY(check_pencil(ctx));
  DeviceGuard g(ctx->device);
  const int64_t n = ctx->pen.n;
  if (k < 0 || l < 0) return fail(AIRGA_EINVAL, "negative column count");
  if ((k > 0 && !A) || (l > 0 && !B) || (k > 0 && l > 0 && !G))
    return fail(AIRGA_EINVAL, "null matrix");
  if ((k > 0 && lda < n) || (l > 0 && ldb < n)) return fail(AIRGA_EINVAL, "leading dimension < n");
  if (k > kGramMax || l > kGramMax) return fail(AIRGA_EUNSUPPORTED, "more than %d columns", kGramMax);
  return gram(ctx, n, k, A, lda, l, B, ldb, G, k);
}

airga_status airga_gram_noalloc(airga_ctx ctx, int32_t k, const double* A, int64_t lda, int32_t l,
                                const double* B, int64_t ldb, double* G) {
  AIRGA_TRY(check_pencil(ctx));
  DeviceGuard g(ctx->device);
  const int64_t n = ctx->pen.n;
  if (k < 0 || l < 0) return fail(AIRGA_EINVAL, "negative column count");
  if ((k > 0 && !A) || (l > 0 && !B) || (k > 0 && l > 0 && !G))
    return fail(AIRGA_EINVAL, "null matrix");
  if ((k > 0 && lda < n) || (l > 0 && ldb < n)) return fail(AIRGA_EINVAL, "leading dimension < n");
  if (k > kGramMax || l > kGramMax) return fail(AIRGA_EUNSUPPORTED, "more than %d columns", kGramMax);
  if (k == 0 || l == 0) return AIRGA_OK;
  if (n == 0) return gram_zero(ctx, l, G, k);
  if (!ctx->gram_scratch) return fail(AIRGA_ESTATE, "no scratch address for device %d", ctx->device);
  const int64_t tiles = (int64_t)((k + kGT - 1) / kGT) * ((l + kGT - 1) / kGT);
  const int64_t full = (n + kGramRowsPerBlock - 1) / kGramRowsPerBlock;
  const int64_t cap = kGramScratchTiles / tiles;
  const int64_t nblk = full < cap ? full : cap;
  if (nblk < 1 || tiles * nblk * kGT * kGT * (int64_t)sizeof(double) > (int64_t)kGramScratchBytes)
    return fail(AIRGA_EUNSUPPORTED, "%lld x %d output tiles exceed the %zu-byte scratch",
                (long long)tiles, (int)nblk, kGramScratchBytes);
  return gram_launch(ctx, n, k, A, lda, l, B, ldb, G, k, (int)nblk, ctx->gram_scratch);
}

airga_status airga_global_orth(airga_ctx ctx, int32_t m, int32_t nb, const double* V, int64_t ldv,
                               int32_t nx, double* X, int64_t ldx, int32_t normalize,
                               double* gamma, double* fro) {
  AIRGA_TRY(check_pencil(ctx));
  DeviceGuard g(ctx->device);
  const int64_t n = ctx->pen.n;
  if (m <= 0 || nb < 0 || nx < 0) return fail(AIRGA_EINVAL, "bad block sizes");
  if (nb > kOrthMaxBlocks) return fail(AIRGA_EUNSUPPORTED, "more than %d basis blocks", kOrthMaxBlocks);
  if ((int64_t)nx * m > kGramMax || (int64_t)nb * m > kGramMax)
    return fail(AIRGA_EUNSUPPORTED, "more than %d columns of blocks", kGramMax);
  if ((nb > 0 && (!V || ldv < n)) || (nx > 0 && (!X || ldx < n)))
    return fail(AIRGA_EINVAL, "null block or leading dimension < n");
  if ((nb > 0 && nx > 0 && !gamma) || (nx > 0 && !fro)) return fail(AIRGA_EINVAL, "null output");
  if (nx == 0) return AIRGA_OK;
  const int kv = nb * m, kx = nx * m;
  // device scratch: G_VX (kv x kx), G_VV (kv x kv), gamma (nx x nb), norms (nx)
  const size_t scratch = (size_t)kv * kx + (size_t)kv * kv + (size_t)nx * nb + nx;
  AIRGA_TRY(ctx->ws_small.reserve(sizeof(double) * scratch));
  double* gvx = ctx->ws_small.as<double>();
  double* gvv = gvx + (size_t)kv * kx;
  double* dgam = gvv + (size_t)kv * kv;
  double* dnrm = dgam + (size_t)nx * nb;
  std::vector<double> gam((size_t)nx * nb, 0.0);
  if (nb > 0) {
    AIRGA_TRY(gram(ctx, n, kv, V, ldv, kx, X, ldx, gvx, kv));
    AIRGA_TRY(gram(ctx, n, kv, V, ldv, kv, V, ldv, gvv, kv));
    std::vector<double> h((size_t)kv * kx + (size_t)kv * kv);
    AIRGA_TRY(to_host(ctx, gvx, h.size(), h.data()));
    const double* hvx = h.data();
    const double* hvv = h.data() + (size_t)kv * kx;
    // trace inner products of the blocks: <V_t, X_x> and <V_t, V_u>
    auto tvx = [&](int t, int x) {
      double s = 0.0;
      for (int c = 0; c < m; ++c) s += hvx[(t * m + c) + (size_t)(x * m + c) * kv];
      return s;
    };
    auto tvv = [&](int t, int u) {
      double s = 0.0;
      for (int c = 0; c < m; ++c) s += hvv[(t * m + c) + (size_t)(u * m + c) * kv];
      return s;
    };
    // Algorithm 1's loop over t subtracts gamma_t V_t from X before the next
    // product, so <V_t, X> there is <V_t, X_0> - sum_{u<t} gamma_u <V_t, V_u>
    for (int x = 0; x < nx; ++x)
      for (int t = 0; t < nb; ++t) {
        double s = tvx(t, x);
        for (int u = 0; u < t; ++u) s -= gam[(size_t)x * nb + u] * tvv(t, u);
        gam[(size_t)x * nb + t] = s;
      }
    AIRGA_TRY(to_device(ctx, gam.data(), gam.size(), dgam));
  }
  const int64_t items = n * m;
  const unsigned nblk = blocks_for(items, 256);
  AIRGA_TRY(ctx->ws_gram.reserve(sizeof(double) * (size_t)nx * nblk * 4));
  double* part = ctx->ws_gram.as<double>();
  k_orth_update<<<nblk, 256, 0, ctx->stream>>>(n, m, nb, V, ldv, nx, X, ldx, dgam, part);
  AIRGA_HIP(hipGetLastError());
  k_sum_rows<<<(unsigned)nx, 256, 0, ctx->stream>>>((int64_t)nblk * 4, part, dnrm);
  AIRGA_HIP(hipGetLastError());
  std::vector<double> nrm(nx);
  AIRGA_TRY(to_host(ctx, dnrm, nx, nrm.data()));
  for (int x = 0; x < nx; ++x) {
    fro[x] = std::sqrt(nrm[x]);
    for (int t = 0; t < nb; ++t) gamma[(size_t)x * nb + t] = gam[(size_t)x * nb + t];
  }
  if (normalize) {
    for (int x = 0; x < nx; ++x) nrm[x] = fro[x] > 0.0 ? 1.0 / fro[x] : 0.0;
    AIRGA_TRY(to_device(ctx, nrm.data(), nx, dnrm));
    k_scale_blocks<<<dim3(blocks_for(n, 256), (unsigned)kx), 256, 0, ctx->stream>>>(n, m, X, ldx,
                                                                                  dnrm);
    AIRGA_HIP(hipGetLastError());
  }
  return AIRGA_OK;
}

airga_status airga_block_qr(airga_ctx ctx, int32_t k, double* W, int64_t ldw, double* R) {
  AIRGA_TRY(check_pencil(ctx));
  DeviceGuard g(ctx->device);
  const int64_t n = ctx->pen.n;
  if (k < 0 || (k > 0 && (!W || !R))) return fail(AIRGA_EINVAL, "bad matrix");
  if (k > kQrMax) return fail(AIRGA_EUNSUPPORTED, "more than %d columns", kQrMax);
  if (k > n) return fail(AIRGA_EINVAL, "more columns than rows");
  if (k > 0 && ldw < n) return fail(AIRGA_EINVAL, "leading dimension < n");
  if (k == 0) return AIRGA_OK;
  const size_t kk = (size_t)k * k;
  AIRGA_TRY(ctx->ws_small.reserve(sizeof(double) * 2 * kk));
  double* dG = ctx->ws_small.as<double>();
  double* dT = dG + kk;
  std::vector<double> G(kk), T(kk), Racc(kk, 0.0), tmp(kk);
  for (int i = 0; i < k; ++i) Racc[i + (size_t)i * k] = 1.0;
  // Shifted Cholesky QR followed by Cholesky QR twice (Fukaya, Kannan,
  // Nakatsukasa, Yamamoto, Yanagisawa, SIAM J. Sci. Comput. 2020): the shift
  // of the first pass keeps its Cholesky factorisation defined for
  // condition numbers up to about 1/eps; the two plain passes then restore
  // orthogonality to working precision.
  for (int pass = 0; pass < 3; ++pass) {
    AIRGA_TRY(gram(ctx, n, k, W, ldw, k, W, ldw, dG, k));
    AIRGA_TRY(to_host(ctx, dG, kk, G.data()));
    if (pass == 0) {
      double tr = 0.0;
      for (int i = 0; i < k; ++i) tr += G[i + (size_t)i * k];
      const double sh = 11.0 * ((double)n * k + (double)k * (k + 1)) * 0x1p-53 * tr;
      for (int i = 0; i < k; ++i) G[i + (size_t)i * k] += sh;
    }
    if (!cholesky_upper(k, G.data()))
      return fail(AIRGA_ENOTSPD, "block QR: the Gram matrix is not positive definite (pass %d): "
                                 "the columns are numerically dependent", pass);
    upper_inverse(k, G.data(), T.data());
    AIRGA_TRY(to_device(ctx, T.data(), kk, dT));
    k_right_trmm<<<blocks_for(n, 256), 256, 0, ctx->stream>>>(n, k, W, ldw, dT);
    AIRGA_HIP(hipGetLastError());
    // R <- R_pass R (both upper triangular)
    for (int j = 0; j < k; ++j)
      for (int i = 0; i <= j; ++i) {
        double s = 0.0;
        for (int p = i; p <= j; ++p) s += G[i + (size_t)p * k] * Racc[p + (size_t)j * k];
        tmp[i + (size_t)j * k] = s;
      }
    for (int j = 0; j < k; ++j)
      for (int i = 0; i < k; ++i) Racc[i + (size_t)j * k] = i <= j ? tmp[i + (size_t)j * k] : 0.0;
  }
  AIRGA_HIP(hipStreamSynchronize(ctx->stream));
  std::memcpy(R, Racc.data(), sizeof(double) * kk);
  return AIRGA_OK;
}

airga_status airga_project(airga_ctx ctx, int32_t k, const double* W, int64_t ldw, double* mhat,
                           double* khat) {
  AIRGA_TRY(check_pencil(ctx));
  DeviceGuard g(ctx->device);
  const int64_t n = ctx->pen.n;
  if (k < 0 || (k > 0 && (!W || !mhat || !khat))) return fail(AIRGA_EINVAL, "bad matrix");
  if (k > kQrMax) return fail(AIRGA_EUNSUPPORTED, "more than %d columns", kQrMax);
  if (k > 0 && ldw < n) return fail(AIRGA_EINVAL, "leading dimension < n");
  if (k == 0) return AIRGA_OK;
  const size_t kk = (size_t)k * k;
  AIRGA_TRY(ctx->ws_tmp.reserve(sizeof(double) * (size_t)n * 2 * k));
  AIRGA_TRY(ctx->ws_small.reserve(sizeof(double) * 2 * kk));
  double* Y = ctx->ws_tmp.as<double>();
  double* dG = ctx->ws_small.as<double>();
  // [M W | K W] in one pass over the pencil, then W^T [M W | K W] =
  // [M_hat | K_hat]   (eq. (1.4))
  spmm_pencil(ctx, k, W, ldw, 1.0, 0.0, Y, n, 0.0, 1.0, Y + (size_t)n * k, n);
  AIRGA_HIP(hipGetLastError());
  AIRGA_TRY(gram(ctx, n, k, W, ldw, 2 * k, Y, n, dG, k));
  std::vector<double> h(2 * kk);
  AIRGA_TRY(to_host(ctx, dG, 2 * kk, h.data()));
  std::memcpy(mhat, h.data(), sizeof(double) * kk);
  std::memcpy(khat, h.data() + kk, sizeof(double) * kk);
  return AIRGA_OK;
}

}  // extern "C"
