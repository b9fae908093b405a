/*
 * airga.h -- C ABI of libairga, the MI355X (gfx950) library for the shifted
 * sparse solves of AIRGA model reduction with SPAI-preconditioned CG, after
 * Singh, Ahuja and Fassbender, "Preconditioned Iterative Solves in Model
 * Reduction of Second Order Linear Dynamical Systems" (arXiv 1606.01216).
 *
 * The problem (Section 1, eq. (1.1); Section 2): a second-order system
 * M x'' + D x' + K x = F u with proportional damping D = alpha M + beta K.
 * Every linear system of the method has the coefficient matrix
 *     K(s) = s^2 M + s D + K = (s^2 + alpha s) M + (1 + beta s) K
 * at a real expansion point s, and right-hand sides F (n x m).  The library
 * builds a sparse approximate inverse of K(s) (Section 3.1, eq. (3.1)),
 * updates it cheaply to a new expansion point (Section 3.2), and solves
 * K(s_k) X_k = F for many shifts at once with preconditioned CG.
 *
 * Conventions shared by every entry point
 *   - Memory: every array argument named as "device" is GPU memory on the
 *     context's device (for example a torch tensor's data pointer), owned by
 *     the caller; the library never frees or keeps it beyond the call except
 *     where stated.  Arguments named "host" are CPU memory.
 *   - Streams: all GPU work of a context is ordered on one HIP stream (the
 *     one given to airga_create, or a stream the context owns).  Calls that
 *     return results to host memory synchronise that stream first.
 *   - Errors: a negative airga_status; airga_last_error() then returns a
 *     message for the calling thread.  On error no output is written unless
 *     stated.  A context is not thread-safe; distinct contexts are.
 *   - Indices are 0-based int32; n * (max row length) must stay below 2^31.
 */
#ifndef AIRGA_H
#define AIRGA_H

#include <stdint.h>

/* Symbols of the C ABI are the only ones the library exports. */
#define AIRGA_API __attribute__((visibility("default")))

#ifdef __cplusplus
extern "C" {
#endif

typedef struct airga_ctx_s* airga_ctx;
typedef struct airga_prec_s* airga_prec;

typedef enum {
  AIRGA_OK = 0,
  AIRGA_EINVAL = -1,      /* bad argument: null pointer, size, pattern, shift    */
  AIRGA_ENOMEM = -2,      /* device or host allocation failed                    */
  AIRGA_EHIP = -3,        /* a HIP runtime call failed                           */
  AIRGA_ENOTSPD = -4,     /* a matrix that must be positive definite is not:     */
                          /* K(s) with a non-positive diagonal entry, a reduced  */
                          /* M, or the Gram matrix of dependent QR columns       */
  AIRGA_ESTATE = -5,      /* call out of order (e.g. no pencil set yet)          */
  AIRGA_EUNSUPPORTED = -6 /* valid input outside the library's supported range   */
} airga_status;

/* Per-system outcome of a solve (airga_sys_stats.status). */
enum {
  AIRGA_SYS_CONVERGED = 0, /* ||F - K(s) X|| <= tol ||F|| (see airga_pcg_opts)    */
  AIRGA_SYS_MAXIT = 1,     /* iteration cap reached                               */
  AIRGA_SYS_BREAKDOWN = 2, /* (p, K(s) p) <= 0: K(s) not positive definite or p=0 */
  AIRGA_SYS_NONFINITE = 3  /* a NaN or infinity appeared                          */
};

enum { AIRGA_MODE_FP64 = 0, AIRGA_MODE_MIXED = 1 };

/* ------------------------------------------------------------------ context */

/* Create a context on HIP device `device`.  `stream` is a hipStream_t to
 * order all work on, or NULL for a context-owned stream (default priority).
 * Errors: EINVAL (null out, bad device), EHIP. */
AIRGA_API airga_status airga_create(airga_ctx* out, int device, void* stream);

/* Release the context, its pencil and workspaces.  Preconditioner handles
 * made by the context must be released before. NULL is ignored. */
AIRGA_API void airga_destroy(airga_ctx ctx);

/* Message for the last non-OK status returned on the calling thread. */
AIRGA_API const char* airga_last_error(void);

/* Library version as "major.minor.patch". */
AIRGA_API const char* airga_version(void);

/* ------------------------------------------------------------------ pencil */

/* Set the pencil (M, K) and the damping coefficients (eq. (1.1):
 * D = alpha M + beta K; D itself is never formed).
 * M and K share ONE structural CSR pattern: row_ptr (device, n+1),
 * col_idx (device, nnz, sorted and unique within each row, symmetric
 * pattern, diagonal present; explicit zeros allowed and kept), values
 * m_val, k_val (device, nnz, float64).  The library copies what it needs
 * (a sliced-ELL copy with 64-row slices, float32 mirrors, the transpose map)
 * and keeps no reference to the inputs.  Replaces any previous pencil;
 * preconditioners built on an earlier pencil become invalid (ESTATE).
 * Errors: EINVAL (n <= 0, nnz <= 0, null pointers, unsorted or out-of-range
 * columns, missing diagonal, asymmetric pattern, alpha or beta < 0),
 * EUNSUPPORTED (a row longer than 16 entries), ENOMEM, EHIP. */
AIRGA_API airga_status airga_set_pencil(airga_ctx ctx, int32_t n, int64_t nnz, const int32_t* row_ptr,
                              const int32_t* col_idx, const double* m_val, const double* k_val,
                              double alpha, double beta);

typedef struct {
  int32_t n;
  int32_t max_row_len;  /* longest row of the pattern                          */
  int32_t bandwidth;    /* max |i - j| over the pattern                         */
  int32_t slice_rows;   /* rows per slice of the sliced-ELL layout (64)         */
  int64_t nnz;          /* entries of the CSR pattern                           */
  int64_t nnz_stored;   /* entries of the sliced-ELL copy (with padding)        */
  double gram_mm, gram_mk, gram_kk; /* <M,M>_F, <M,K>_F, <K,K>_F                */
  double trace_m, trace_k;
} airga_pencil_info;

/* Describe the current pencil (host struct).  Errors: EINVAL, ESTATE. */
AIRGA_API airga_status airga_get_pencil_info(airga_ctx ctx, airga_pencil_info* out);

/* a_val (device, nnz, CSR order of the pattern) = entries of
 * K(s) = (s^2 + alpha s) M + (1 + beta s) K (Section 2; the coefficient
 * matrix of every shifted solve of Algorithms 1, 3 and 5), computed as one fused
 * multiply-add per entry in float64.  Asynchronous.
 * Errors: EINVAL (null a_val, non-finite s), ESTATE (no pencil). */
AIRGA_API airga_status airga_assemble_shift(airga_ctx ctx, double s, double* a_val);

/* y = K(s) x for `count` vectors x (device, n each, leading dimension ldx)
 * into y (device, ldy), float64.  Asynchronous.  Errors: EINVAL, ESTATE. */
AIRGA_API airga_status airga_apply_shift(airga_ctx ctx, double s, int32_t count, const double* x,
                               int64_t ldx, double* y, int64_t ldy);

/* The two quantities the paper tabulates for every expansion point
 * (Tables 6 and 7) and the two scalings of its SPAI algorithms, from the
 * Gram scalars of the pencil (host output out[4]):
 *   out[0] = ||I - K(s_new)||_F
 *   out[1] = ||K(s_old) - K(s_new)||_F
 *   out[2] = trace(K(s_new)) / trace(K(s_new) K(s_new)^T)       (SPAI start)
 *   out[3] = <K(s_old), K(s_new)>_F / ||K(s_new)||_F^2          (update start)
 * Errors: EINVAL, ESTATE. */
AIRGA_API airga_status airga_shift_diagnostics(airga_ctx ctx, double s_old, double s_new, double* out);

/* --------------------------------------------------------- preconditioners */

typedef struct {
  double tol;          /* update: a column keeps q_j = alpha e_j when
                          ||k_old_j - alpha k_new_j|| <= tol ||k_old_j||
                          (the test that opens the inner loop of the update
                          algorithm; the paper uses 0.01).  With mr_iters > 0
                          also the loops' stopping test ||r|| <= tol ||t||,
                          build included.  Default 0.01.                      */
  int32_t equilibrate; /* 1: pose the column problems for S K(s) S with
                          S = diag(K(s))^{-1/2} and map back (default 1)      */
  int32_t symmetrize;  /* build only, 1: replace Phat by (Phat + Phat^T)/2
                          before mapping back (default 1)                      */
  int32_t general_only; /* 1: the general column kernels even for a pencil of
                          bandwidth <= 64 (whose kernels otherwise stage the
                          rows in LDS; same arithmetic, same results)          */
  int32_t mr_iters;    /* 0 (default): each column's least-squares problem on
                          the pattern is solved exactly.  > 0: the paper's
                          minimal-residual column loop (Algorithms 2 and 4):
                          from alpha e_j, steps d = alpha r dropped to the
                          pattern of the column, a = (r, w) / (w, w) with
                          w = K d, until ||r|| <= tol ||t|| (t = e_j or
                          k_old_j), at most mr_iters steps (<= 100000).       */
  int32_t lfil;        /* minimal-residual mode only: 0 (default) steps on the
                          whole pattern of the column from the start; 1..8:
                          pattern control (the sparsity step the paper leaves
                          out of Algorithms 2 and 4): the column's pattern
                          starts as {j} and each step first admits the entry
                          of the pattern of column j of K(s) with the largest
                          |alpha r| outside it, up to lfil entries (ties
                          within a relative 1e-8 go to the lowest row).
                          EINVAL outside [0, 8] or with mr_iters = 0.         */
} airga_spai_opts;

AIRGA_API void airga_spai_opts_default(airga_spai_opts* opts);

/* SPAI of K(s) on the structural pattern of K(s) (eq. (3.1)): for every
 * column j, p_j = argmin || e_j - K(s) p ||_2 over vectors with the
 * pattern of column j, solved exactly per column (Givens QR in float64,
 * one column per GPU lane).  `opts` may be NULL (defaults).  The handle
 * owns the factor (a float64 copy, and a float32 copy for the float32
 * inner solves of MIXED mode) and must be released with
 * airga_prec_release.  Asynchronous.  Pencils of bandwidth <= 64 use
 * kernels that stage each block's rows in LDS (see general_only).
 * Errors: EINVAL (s <= 0 or non-finite, null out), ESTATE (no pencil),
 * ENOTSPD (the pencil has a diagonal entry of M <= 0 or of K < 0, so K(s)
 * need not be SPD), EUNSUPPORTED (a row of more than 8 entries: the column
 * problems are held in registers), ENOMEM, EHIP. */
AIRGA_API airga_status airga_spai_build(airga_ctx ctx, double s, const airga_spai_opts* opts,
                              airga_prec* out);

/* SPAI update (Section 3.2): Q with K(s_new) Q ~ K(s_old) column by column,
 * from Q = alpha I with alpha = <K_old, K_new>_F / ||K_new||_F^2; columns
 * failing the skip test are solved exactly on the pattern.  The result is
 * the chain Q * (old chain): a new handle that references `old` (reference
 * counted; `old` stays valid for the caller).  A factor whose columns all
 * skip is the scalar alpha and is not applied (CG is invariant to a nonzero
 * scaling of the preconditioner); no factor values are written for it and
 * airga_prec_export returns alpha I.  Errors: as airga_spai_build, plus
 * EINVAL for a null or foreign `old`. */
AIRGA_API airga_status airga_spai_update(airga_ctx ctx, airga_prec old, double s_new,
                               const airga_spai_opts* opts, airga_prec* out);

/* Several SPAI builds at once: out[i] = the SPAI of K(shifts[i]), exactly
 * as airga_spai_build(ctx, shifts[i], opts, &out[i]) would give, for
 * i < count (host arrays).  On a banded pencil (bandwidth <= 64, rows of at
 * most 6 entries; exact column solves) each block's rows are staged once per
 * batch of 16 shifts; otherwise the builds run one after the other.  On
 * error no handle is returned (out[i] = NULL).  Errors: as
 * airga_spai_build, plus EINVAL for count < 0 or null arrays. */
AIRGA_API airga_status airga_spai_build_many(airga_ctx ctx, int32_t count, const double* shifts,
                                             const airga_spai_opts* opts, airga_prec* out);

/* Several SPAI updates at once: out[i] = the update of olds[i] to s_new[i],
 * exactly as airga_spai_update(ctx, olds[i], s_new[i], opts, &out[i]) would
 * give, for i < count (host arrays).  On a banded pencil (bandwidth <= 64,
 * rows of at most 6 entries) the pencil is read once per batch of 16 and
 * the launches are shared; otherwise the updates run one after the other.
 * On error no handle is returned (out[i] = NULL).  Errors: as
 * airga_spai_update, plus EINVAL for count < 0 or null arrays. */
AIRGA_API airga_status airga_spai_update_many(airga_ctx ctx, int32_t count, const airga_prec* olds,
                                              const double* s_new, const airga_spai_opts* opts,
                                              airga_prec* out);

typedef struct {
  double shift;         /* expansion point of the newest factor                 */
  double alpha;         /* starting scaling of the newest factor                */
  int32_t chain_len;    /* factors applied per application (scalars excluded)   */
  int32_t scalar_only;  /* 1 when the newest factor collapsed to alpha I        */
  int64_t skipped_cols; /* columns of the newest factor kept at alpha e_j       */
  double shift_im;      /* complex factors: imaginary part of the shift (else 0)*/
  double alpha_im;      /* complex factors: imaginary part of alpha (else 0)    */
  int32_t is_complex;   /* 1 for a complex factor (build or update)             */
} airga_prec_info;

/* Describe a preconditioner (synchronises the context stream). */
AIRGA_API airga_status airga_get_prec_info(airga_prec prec, airga_prec_info* out);

/* Export the newest factor: values (device, nnz, CSR order, float64; the
 * mapped-back factor as applied) and, if objective is not NULL, the per
 * column least-squares residual norm in the scaled problem (device, n).
 * A scalar-only factor exports alpha on the diagonal.  Asynchronous, except
 * that exporting values waits once for an update's skip count. */
AIRGA_API airga_status airga_prec_export(airga_prec prec, double* values, double* objective);

/* Which columns of the newest factor the update kept at alpha e_j
 * (Section 3.2: the test that opens the update's column loop held), so that
 * their least-squares problem was never solved: flags (device, n bytes) = 1
 * for such a column, 0 for a solved one; a build returns all zeros.
 * Asynchronous.  Errors: EINVAL (null flags or handle). */
AIRGA_API airga_status airga_prec_skip_flags(airga_prec prec, uint8_t* flags);

/* z = C r for `count` vectors (device, leading dimensions ldr, ldz),
 * C the whole chain Q_z ... Q_2 P_1 applied factor by factor (float64).
 * Asynchronous.  Errors: EINVAL. */
AIRGA_API airga_status airga_prec_apply(airga_prec prec, int32_t count, const double* r, int64_t ldr,
                              double* z, int64_t ldz);

/* Drop the caller's reference.  NULL is ignored. */
AIRGA_API void airga_prec_release(airga_prec prec);

/* ------------------------------------------------------------------ solves */

enum { AIRGA_BETA_FLEXIBLE = 0, AIRGA_BETA_CLASSICAL = 1 };

typedef struct {
  double tol;          /* stop when ||F - K X|| <= tol ||F|| (float64 residual
                          in MIXED mode, CG recurrence residual in FP64 mode).
                          Default 1e-10.                                        */
  int32_t max_iter;    /* CG iterations per system, summed over sweeps
                          (default 20000)                                       */
  int32_t mode;        /* AIRGA_MODE_FP64 or AIRGA_MODE_MIXED (float32 matrix,
                          arithmetic, vectors and preconditioner values,
                          inside float64 iterative refinement of the residual
                          and the solution)                                     */
  double inner_tol;    /* MIXED: relative residual reduction per sweep (1e-5:
                          two sweeps reach the default tol of 1e-10)          */
  int32_t max_sweeps;  /* MIXED: refinement sweeps (default 12)                 */
  int32_t poll_every;  /* iterations between host checks of the active count
                          (rounded up to even; default 8)                       */
  int32_t x0_given;    /* 1: X holds the starting guess (resume); 0: X0 = 0     */
  int32_t use_graph;   /* 1: replay iterations from a captured HIP graph        */
  int32_t profile;     /* 1: time every launch of the dominant kernels with
                          HIP events (no graph); see airga_get_kernel_times     */
  int32_t tile_rows;   /* 0 (default): the autotuner picks the tile; otherwise
                          matrix rows per wavefront (64, 128 or 256) ...        */
  int32_t tile_sys;    /* ... and systems per group (1, 2 or 4) of an allowed
                          tile (see airga_get_tile_config); EINVAL if not one   */
  int32_t general_only; /* 1: general sliced-ELL kernels even for a pencil of
                          bandwidth <= 64 (whose kernels otherwise stage the
                          neighbour entries in LDS; same arithmetic)             */
  int32_t beta_form;   /* direction update: AIRGA_BETA_FLEXIBLE (default)
                          beta = -(z_new, K p) / (p, K p), valid for any
                          preconditioner and the more robust one in float32;
                          AIRGA_BETA_CLASSICAL the ratio (r,z)_new / (r,z)_old,
                          for symmetric preconditioners only                    */
  int32_t inner_max;   /* MIXED: float32 iterations per sweep (default 96,
                          rounded up to a multiple of poll_every).  A system
                          still iterating at the cap keeps that sweep's
                          correction and is finished by a float64 solve from
                          its current X, batched with the others that hit it:
                          float32 cannot resolve systems whose condition number
                          approaches 1/eps_32, and they would stall the batch  */
} airga_pcg_opts;

AIRGA_API void airga_pcg_opts_default(airga_pcg_opts* opts);

typedef struct {
  int32_t status;      /* AIRGA_SYS_*                                           */
  int32_t iters;       /* CG iterations                                         */
  int32_t sweeps;      /* refinement sweeps (MIXED), 1 for FP64                 */
  int32_t finished_fp64; /* MIXED: 1 if handed to the float64 finish (iters
                          and sweeps include both stages)                      */
  double relres;       /* ||F - K X|| / ||F|| from the float64 residual at exit */
} airga_sys_stats;

/* Solve K(s_k) X[:, c, k] = F[:, c] for every shift k < nshift and column
 * c < m with preconditioned CG (the shifted solves of the AIRGA algorithm,
 * Algorithm 1, and of its SPAI and SPAI-update variants, Algorithms 3 and
 * 5), all nshift*m systems batched in one set of kernels
 * with per-system convergence masking.
 *   shifts: host, nshift real expansion points (each > 0)
 *   precs:  host, nshift handles (NULL entry = no preconditioner)
 *   F:      device, n x m column-major, leading dimension ldf >= n
 *   X:      device, n x m x nshift, column (c, k) at X + (k*m + c)*ldx,
 *           ldx >= n; read as the starting guess when opts->x0_given
 *   stats:  host, nshift*m entries in the same (k, c) order, may be NULL
 * Returns after the stats are on the host.  Non-convergence is not an
 * error: it is reported per system.  Errors: EINVAL, ESTATE, ENOMEM, EHIP. */
AIRGA_API airga_status airga_pcg_solve(airga_ctx ctx, int32_t nshift, const double* shifts,
                             const airga_prec* precs, int32_t m, const double* F, int64_t ldf,
                             double* X, int64_t ldx, const airga_pcg_opts* opts,
                             airga_sys_stats* stats);

/* Kernel timings gathered by the last profiled solve (opts.profile = 1):
 * for kernel id k < count (see airga_kernel_name), the number of launches
 * and their summed duration in milliseconds (HIP events on the context
 * stream).  Host arrays of at least `count` entries. */
AIRGA_API int32_t airga_kernel_count(void);
AIRGA_API const char* airga_kernel_name(int32_t id);
AIRGA_API airga_status airga_get_kernel_times(airga_ctx ctx, int32_t count, int64_t* launches,
                                    double* total_ms);

/* Tile configuration the autotuner chose for the last solve on this
 * context: matrix rows per wavefront (a multiple of 64) and systems swept
 * together per group.  Errors: EINVAL, ESTATE (no solve yet). */
AIRGA_API airga_status airga_get_tile_config(airga_ctx ctx, int32_t* rows_per_wave,
                                             int32_t* systems_per_group);

/* Work done by the row kernels of the last profiled solve, for kernel id
 * k < count: sys_passes[k] = (system, launch) pairs swept (for chain:
 * (system, chain factor) pairs; for ir_residual and ir_update: the systems
 * under refinement when the kernel was launched), shift_passes[k] =
 * (shift, launch) pairs whose first preconditioner factor was read
 * (update_prec) or further chain factors applied (chain).  Together with
 * the pencil size these give the algorithmic bytes each kernel moved. */
AIRGA_API airga_status airga_get_kernel_work(airga_ctx ctx, int32_t count, int64_t* sys_passes,
                                             int64_t* shift_passes);

/* ---------------------------------------------------- complex shifts
 *
 * Complex expansion points s = s_re + i s_im.  The paper keeps its points
 * real by taking the real parts of the reduced poles (Section 5); these
 * calls take complex points as they are.  K(s) = (s^2 + alpha s) M +
 * (1 + beta s) K is then complex symmetric (K(s)^T = K(s)), not Hermitian,
 * so CG becomes conjugate orthogonal CG (COCG: the bilinear form x^T y in
 * place of the inner product; van der Vorst and Melissen, 1990), which needs
 * a complex symmetric preconditioner.  Complex arrays are interleaved
 * (re, im) float64 pairs.  Pencils with rows of at most 6 entries. */

/* a_val (device, 2 nnz: entry e's real part at 2e, imaginary at 2e + 1, CSR
 * order) = K(s) for complex s.  Asynchronous.  Errors: EINVAL (null a_val,
 * non-finite s), ESTATE. */
AIRGA_API airga_status airga_assemble_shift_complex(airga_ctx ctx, double s_re, double s_im,
                                                    double* a_val);

/* SPAI of K(s) for complex s (eq. (3.1) with complex column least squares):
 * for every column j, p_j = argmin || e_j - Khat p ||_2 over complex vectors
 * on the pattern of column j, Khat = S K(s) S with S = diag(K(s))^{-1/2}
 * (principal square root; equilibrate = 0: S = I), solved exactly per column
 * (complex Givens QR in float64, one column per lane); symmetrize = 1
 * replaces Phat by (Phat + Phat^T) / 2 (plain transpose), so that the factor
 * S Phat S is complex symmetric like K(s), as COCG needs.  The handle is an
 * airga_prec for airga_cocg_solve, airga_prec_export_complex,
 * airga_get_prec_info and airga_prec_release; the real calls refuse it.
 * opts may be NULL; tol and mr_iters are not used (mr_iters > 0:
 * EUNSUPPORTED).  Asynchronous.  Errors: EINVAL (non-finite s, null out),
 * ESTATE, EUNSUPPORTED (rows of more than 6 entries), ENOMEM, EHIP. */
AIRGA_API airga_status airga_spai_build_complex(airga_ctx ctx, double s_re, double s_im,
                                                const airga_spai_opts* opts, airga_prec* out);

/* The SPAI update (Section 3.2, Algorithm 4) from a complex factor `old`
 * (built or updated at s_old) to the complex point s_new = s_re + i s_im:
 * Q with K(s_new) Q ~ K(s_old), started from alpha I where alpha minimises
 * ||Khat_old - alpha Khat_new||_F over complex alpha,
 *   alpha = <Khat_new, Khat_old> / <Khat_new, Khat_new>
 * (Hermitian inner product; the paper's formula for real matrices), both
 * matrices scaled by S = diag(K(s_new))^{-1/2} (principal square root).
 * Column j keeps q_j = alpha e_j when ||khat_old_j - alpha khat_new_j|| <=
 * tol ||khat_old_j|| (opts->tol, default 0.01), else it is the complex least
 * squares min ||khat_old_j - Khat_new(I, J) q|| on the pattern (complex
 * Givens QR, one column per lane); Q = S Qhat S^{-1}.  The new handle holds
 * a reference to `old`: airga_cocg_solve applies the chain Q_z ... Q_2 P_1
 * factor by factor (a fully skipped factor, the scalar alpha I, is dropped).
 * Synchronises once (alpha and the skip count).  Errors: EINVAL (null
 * arguments, a real `old`, non-finite s_new, tol < 0, a factor of another
 * context), ESTATE, EUNSUPPORTED (mr_iters or lfil set), ENOMEM, EHIP. */
AIRGA_API airga_status airga_spai_update_complex(airga_ctx ctx, airga_prec old, double s_re,
                                                 double s_im, const airga_spai_opts* opts,
                                                 airga_prec* out);

/* airga_spai_build_complex for `count` complex points at once: shifts (host,
 * 2 count doubles, s_k = shifts[2k] + i shifts[2k+1]), out (host, count
 * handles), each factor equal to its single build.  On an error no handle is
 * returned (every out[k] NULL).  Asynchronous.  Errors: as
 * airga_spai_build_complex, EINVAL (count < 0, null arrays). */
AIRGA_API airga_status airga_spai_build_complex_many(airga_ctx ctx, int32_t count,
                                                     const double* shifts,
                                                     const airga_spai_opts* opts, airga_prec* out);

/* airga_spai_update_complex for `count` (old factor, new point) pairs at
 * once: olds (host, count handles, repeats allowed), shifts (host, 2 count
 * doubles), out (host, count handles), each factor equal to its single
 * update.  All updates are launched before one synchronisation reads every
 * alpha and skip count.  On an error no handle is returned (every out[k]
 * NULL).  Errors: as airga_spai_update_complex, EINVAL (count < 0, null
 * arrays). */
AIRGA_API airga_status airga_spai_update_complex_many(airga_ctx ctx, int32_t count,
                                                      const airga_prec* olds,
                                                      const double* shifts,
                                                      const airga_spai_opts* opts,
                                                      airga_prec* out);

/* Export a complex factor: values (device, 2 nnz, interleaved, CSR order)
 * and, if objective is not NULL, the per-column least-squares residual norm
 * (device, n, real).  Asynchronous.  Errors: EINVAL (not a complex factor),
 * ESTATE. */
AIRGA_API airga_status airga_prec_export_complex(airga_prec prec, double* values,
                                                 double* objective);

/* Solve K(s_k) X[:, c, k] = F[:, c] for complex s_k (k < nshift) and every
 * column c < m of the real F with preconditioned COCG, all nshift*m systems
 * batched in one set of kernels with per-system convergence masking, in
 * complex float64:
 *   shifts: host, 2 nshift doubles (s_k = shifts[2k] + i shifts[2k+1])
 *   precs:  host, nshift complex factors (airga_spai_build_complex or
 *           airga_spai_update_complex) at the same shift, or NULL entries
 *           (no preconditioner); an update applies its whole chain
 *   F:      device, real n x m, leading dimension ldf >= n
 *   X:      device, complex n x m x nshift interleaved, column (c, k) at
 *           X + 2 (k m + c) ldx, ldx >= n (in complex entries)
 *   stats:  host, nshift*m entries in (k, c) order, may be NULL
 * Iteration from X = 0: w = K p, mu = p^T w, alpha = (r^T z) / mu, x += alpha
 * p, r -= alpha w, stop when ||r|| <= tol ||F(:, c)|| (Euclidean norm of
 * the recurrence residual), z = C r (C the chain, factor by factor), beta =
 * -(z^T w) / mu (flexible,
 * default) or (r^T z)_new / (r^T z)_old (beta_form classical), p = z +
 * beta p.  BREAKDOWN when mu = 0; relres in stats is the true residual
 * ||F - K X|| / ||F|| at exit.  Options used: tol, max_iter, poll_every,
 * beta_form, mode; x0_given must be 0 (else EUNSUPPORTED).  mode MIXED:
 * iterative refinement from X = 0, each sweep forming r = F - K X in
 * float64 and solving K d = r by the COCG above in float32 (pencil, factors
 * and vectors; float64 scalars) to a reduction inner_tol or inner_max
 * iterations (default 96, rounded up to a multiple of poll_every), then X +=
 * d; a system stops CONVERGED when its float64 residual meets tol, MAXIT
 * after max_sweeps sweeps or max_iter inner iterations in all, BREAKDOWN or
 * NONFINITE when an inner solve does (no float64 hand-over); stats give the
 * iterations summed over sweeps and the sweep count.  Returns
 * after the stats are on the host.  Errors: EINVAL (sizes, null arrays,
 * non-finite shifts, a real factor or one built at another shift, refinement
 * options out of range), ESTATE,
 * EUNSUPPORTED (more than 4096 systems, rows of more than 6 entries),
 * ENOMEM, EHIP. */
AIRGA_API airga_status airga_cocg_solve(airga_ctx ctx, int32_t nshift, const double* shifts,
                                        const airga_prec* precs, int32_t m, const double* F,
                                        int64_t ldf, double* X, int64_t ldx,
                                        const airga_pcg_opts* opts, airga_sys_stats* stats);

/* ------------------------------------------------ moment sequence blocks
 *
 * The block operations around the shifted solves of AIRGA's moment sequence
 * (Section 2, Algorithm 1; Algorithm 3 keeps them and changes the solves):
 * right-hand sides M V_j, orthogonalisation of the n x m solution blocks in
 * the trace inner product (global Arnoldi), the thin QR of the collected
 * blocks and the Galerkin projection of eq. (1.4).  All matrices are device
 * float64, column-major, with n = the pencil's row count and leading
 * dimensions >= n; the caller owns every array.  Products over the n rows
 * are fixed-order sums: repeated calls give identical bits. */

/* y_c = (a M + b K) x_c for `count` vectors (as airga_apply_shift, with the
 * coefficients given): M V_j is a = 1, b = 0 (Algorithm 1's right-hand side
 * of the moment solves).  Asynchronous.  Errors: EINVAL, ESTATE,
 * EUNSUPPORTED (count > 65535). */
AIRGA_API airga_status airga_pencil_apply(airga_ctx ctx, double a, double b, int32_t count,
                                          const double* x, int64_t ldx, double* y, int64_t ldy);

/* G (device, k x l, column-major, leading dimension k) = A^T B for the
 * n x k matrix A and the n x l matrix B.  Asynchronous.  Errors: EINVAL,
 * ESTATE, EUNSUPPORTED (k or l > 256). */
AIRGA_API airga_status airga_gram(airga_ctx ctx, int32_t k, const double* A, int64_t lda,
                                  int32_t l, const double* B, int64_t ldb, double* G);

/* airga_gram for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc.  Same
 * arguments, result and errors as airga_gram; it calls no hipMalloc or
 * hipFree and allocates nothing, on the device or the host.  Its partial sums
 * live in a fixed 32 MiB device array, one per GPU, held from the first
 * airga_create on that GPU until the process ends.  The array holds 1024
 * partial 64 x 64 tiles: for k, l <= 64 and n <= 1,048,576 the sums are
 * formed exactly as in airga_gram (identical bits); beyond that each block of
 * the product covers more rows, so results agree with airga_gram to rounding.
 * No size within airga_gram's limits is refused for lack of scratch; a
 * product that would need more than the array is refused with
 * EUNSUPPORTED.  Every call on one GPU shares the array, from any context:
 * calls that overlap on one GPU (on different streams, or from several
 * threads) race and must be ordered by the caller.  Nothing in the array
 * needs clearing between calls.  Asynchronous. */
AIRGA_API airga_status airga_gram_noalloc(airga_ctx ctx, int32_t k, const double* A, int64_t lda,
                                          int32_t l, const double* B, int64_t ldb, double* G);

/* Global Arnoldi orthogonalisation (Algorithm 1, the loop over t): each of
 * the nx blocks X_x = X(:, x m : x m + m) is orthogonalised against the nb
 * blocks V_t = V(:, t m : t m + m) in the trace inner product <A, B> =
 * trace(A^T B), in the algorithm's order: for t = 1..nb, gamma_t =
 * <V_t, X_x>, X_x <- X_x - gamma_t V_t.  X is overwritten; gamma (host,
 * nx * nb, gamma[x * nb + t]) and fro (host, nx) = ||X_x||_F after the
 * subtraction are returned; normalize = 1 then divides X_x by fro[x] (a
 * zero block stays zero), which makes the W_i and V_j of Algorithm 1.
 * Synchronous.  Errors: EINVAL, ESTATE, EUNSUPPORTED (nb > 16, or nb m or
 * nx m > 256). */
AIRGA_API airga_status airga_global_orth(airga_ctx ctx, int32_t m, int32_t nb, const double* V,
                                         int64_t ldv, int32_t nx, double* X, int64_t ldx,
                                         int32_t normalize, double* gamma, double* fro);

/* Thin QR of the n x k block W (Algorithm 1's qr of the collected blocks):
 * W is overwritten by Q with orthonormal columns and R (host, k x k,
 * column-major, upper triangular with a positive diagonal) satisfies
 * W_in = Q R.  Computed by a shifted Cholesky QR followed by two Cholesky QR
 * passes.  Synchronous.  Errors: EINVAL (k > n), ESTATE, EUNSUPPORTED
 * (k > 64), ENOTSPD (the columns are numerically dependent: W is left
 * partly transformed). */
AIRGA_API airga_status airga_block_qr(airga_ctx ctx, int32_t k, double* W, int64_t ldw, double* R);

/* Galerkin projection onto the n x k basis W (eq. (1.4)): mhat, khat (host,
 * k x k, column-major) = W^T M W and W^T K W; D_hat = alpha mhat + beta
 * khat for Rayleigh damping.  Synchronous.  Errors: EINVAL, ESTATE,
 * EUNSUPPORTED (k > 64), ENOMEM. */
AIRGA_API airga_status airga_project(airga_ctx ctx, int32_t k, const double* W, int64_t ldw,
                                     double* mhat, double* khat);

/* ------------------------------------------ outer iteration decisions
 *
 * Host computations behind the decisions of AIRGA's outer iteration
 * (Algorithm 1): the poles of the reduced quadratic pencil, whose real parts
 * give the next expansion points (Section 5), and the H2 distance between
 * reduced models, which ends both of the algorithm's loops (Section 5 uses
 * 1e-6 for both).  They run on the calling thread, need no context and no
 * GPU, and are synchronous.  Reduced matrices are host float64,
 * column-major; the caller owns every array. */

typedef struct {
  int32_t r, m, p;     /* order, inputs, outputs                          */
  const double* mhat;  /* r x r, symmetric positive definite              */
  const double* khat;  /* r x r, symmetric                                */
  const double* fhat;  /* r x m                                           */
  const double* cphat; /* p x r: position output                          */
  const double* cvhat; /* p x r: velocity output, or NULL for none        */
} airga_reduced_model;

/* The 2r poles of lambda^2 Mh + lambda (alpha Mh + beta Kh) + Kh, the
 * damping of a projected Rayleigh-damped model (eq. (1.4)): mode by mode in
 * ascending undamped frequency, two entries per mode in re and im (host,
 * 2r each): a complex pair as (+im, -im), two real roots the smaller in
 * magnitude first.  Errors: EINVAL (r <= 0, null arrays, non-finite alpha,
 * beta or matrix entries), ENOTSPD (Mh not positive definite). */
AIRGA_API airga_status airga_qep_poles(int32_t r, const double* mhat, const double* khat,
                                       double alpha, double beta, double* re, double* im);

/* The next l expansion points (shifts, host, l values, ascending) from
 * `count` poles (re, im, host): each conjugate pair gives one candidate
 * -Re(lambda), the real part the paper takes (Section 5); each real pole
 * (|im| <= 1e-12 |lambda|) gives -lambda.  Candidates are ranked by
 * |lambda|, smallest first, and the first l are taken.  Which poles become
 * expansion points the paper leaves to Bonin et al.; this ranking is the
 * library's reading.  Errors: EINVAL (fewer than l candidates, count < 0,
 * l <= 0, null arrays, non-finite poles). */
AIRGA_API airga_status airga_next_shifts(int32_t count, const double* re, const double* im,
                                         int32_t l, double* shifts);

/* out = ||H_a - H_b||_H2 (b NULL: ||H_a||_H2) for reduced models with
 * damping alpha Mh + beta Kh and transfer function
 * H(s) = (C_p + s C_v) (s^2 Mh + s Dh + Kh)^-1 F_h, from their modal forms
 * (a closed-form 2 x 2 cross Gramian for each pair of modes).  The models
 * must share m, p and whether C_v is given.  The distance of nearly equal
 * models is a difference of squared norms: it is resolved to about 1e-8 of
 * ||H_a||.  Errors: EINVAL (sizes, null arrays, non-finite alpha, beta or
 * matrix entries, a mode with alpha + beta w^2 <= 0, whose norm is
 * infinite), ENOTSPD (an Mh not positive definite). */
AIRGA_API airga_status airga_h2_distance(const airga_reduced_model* a,
                                         const airga_reduced_model* b, double alpha, double beta,
                                         double* out);

/* ------------------------------------------------- AIRGA's outer loop
 *
 * The whole model reduction of Algorithm 1 in one call, with SPAI
 * preconditioned CG for every shifted solve (Algorithm 3) and, optionally,
 * the cheap update carried across outer iterations (Algorithm 5).  Each
 * outer iteration: SPAI at the l expansion points (built, or updated from
 * the previous iteration's at the same position, see update_from), the
 * solves X(s_i) = K(s_i)^{-1} F and their thin QR; the moment loop, which
 * takes the point sigma_j with the largest moment error (the fraction of its
 * newest moment block that the basis does not hold yet; sigma_1 = s_1),
 * appends that block normalised in the Frobenius norm as V_j, replaces it
 * by the next moment -K(sigma_j)^{-1} M V_j and orthogonalises every point's
 * block against V_1..V_j in the trace inner product, and stops when the
 * reduced model on the normalised blocks changes by less than tol_inner
 * relative to its H2 norm, or when the basis reaches floor(r_max / m)
 * blocks (the last block is then taken, again by the largest moment
 * error); then the basis V = qr([V_1 .. V_J]), the reduced model of
 * eq. (1.4) and its relative H2 change against the previous iteration's.
 * The outer loop stops when that change is below tol_outer (Section 5 uses
 * 1e-6 for both tests) or after max_outer iterations; otherwise the next
 * points are the real parts of the reduced poles as airga_next_shifts
 * chooses them (Section 5), and the i-th new point is paired with the i-th
 * old one.  Every step runs in the library's kernels and host decisions
 * (the entry points above); only small reduced matrices visit the host. */

typedef struct {
  int32_t r_max;        /* largest reduced order: the basis holds at most
                           floor(r_max / m) blocks of m columns (<= 64
                           columns).  Default 24.                           */
  double tol_inner;     /* moment loop: relative H2 change (default 1e-6)    */
  double tol_outer;     /* outer loop: relative H2 change (default 1e-6)     */
  int32_t max_outer;    /* outer iterations at most (default 10)             */
  int32_t update_from;  /* 0 (default): a new SPAI at every iteration's
                           points; k >= 2: from outer iteration k on (1-based)
                           each point's preconditioner is the SPAI update
                           (Section 3.2) of the previous iteration's factor at
                           the same position, so the chains grow (Alg. 5)    */
  airga_spai_opts spai; /* builds and updates                               */
  airga_pcg_opts pcg;   /* every solve (x0_given is ignored)                 */
} airga_reduce_opts;

AIRGA_API void airga_reduce_opts_default(airga_reduce_opts* opts);

/* Results of airga_reduce.  The caller sets the pointer fields to host
 * arrays (or NULL for outputs it does not want); they are written on
 * success, column-major with leading dimension r (r_max^2, r_max m and
 * p r_max entries suffice). */
typedef struct {
  int32_t iterations;   /* outer iterations run                              */
  int32_t converged;    /* 1 if the last change fell below tol_outer         */
  int32_t r;            /* order of the final model = J m columns of V       */
  double change;        /* the last relative H2 change (NaN after one)       */
  double* mhat;         /* r x r: V^T M V                                     */
  double* khat;         /* r x r: V^T K V (D_hat = alpha mhat + beta khat)    */
  double* fhat;         /* r x m: V^T F                                       */
  double* cphat;        /* p x r: C_p V                                       */
  double* cvhat;        /* p x r: C_v V (only when C_v is given)              */
  double* next_shifts;  /* l: the points a further iteration would use (the
                           last iteration's own points if it converged)      */
} airga_reduce_result;

/* Per outer iteration (optional history). */
typedef struct {
  int32_t blocks;        /* J of this iteration's final basis                */
  int32_t moment_steps;  /* intermediate models formed                        */
  int32_t updated;       /* 1: preconditioners updated, 0: built              */
  int32_t chain_len_max; /* longest preconditioner chain applied             */
  int32_t max_iters;     /* largest CG iteration count of its solves          */
  int32_t all_converged; /* 1 if every solve of the iteration converged       */
  double change;         /* relative H2 change of the final model (NaN first) */
  double last_inner_change; /* the moment loop's last change (NaN if none)   */
} airga_reduce_iter;

/* Reduce the pencil set by airga_set_pencil (with its alpha, beta) for the
 * input F (device, n x m, leading dimension ldf) and the outputs C_p, C_v
 * (device, each stored as its transpose, n x p with leading dimension ldc;
 * Cv may be NULL), from the l initial expansion points shifts0 (host, > 0).
 *   V:          device, n x r_max (ldv >= n): the final orthonormal basis in
 *               its first res->r columns, the rest used as work space
 *   res:        host, see airga_reduce_result
 *   shift_hist: host, max_outer x l (row z = the points of iteration z), or NULL
 *   sigma_hist: host, max_outer x floor(r_max/m) (indices into that row of
 *               shift_hist, -1 past J), or NULL
 *   iter_hist:  host, max_outer entries, or NULL
 * Synchronous.  A solve that does not converge is reported in iter_hist,
 * not as an error.  Errors: EINVAL (sizes, null arrays, shifts, options),
 * EUNSUPPORTED (more than 64 basis columns, l m > 64, m > 16, p > 256, or a
 * new expansion point that is not positive), ENOTSPD (dependent blocks in a
 * thin QR), ESTATE, ENOMEM, EHIP. */
AIRGA_API airga_status airga_reduce(airga_ctx ctx, int32_t m, const double* F, int64_t ldf,
                                    int32_t p, const double* Cp, const double* Cv, int64_t ldc,
                                    int32_t l, const double* shifts0,
                                    const airga_reduce_opts* opts, double* V, int64_t ldv,
                                    airga_reduce_result* res, double* shift_hist,
                                    int32_t* sigma_hist, airga_reduce_iter* iter_hist);

#ifdef __cplusplus
}
#endif

#endif /* AIRGA_H */
