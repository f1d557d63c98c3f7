/*
 * nn.h — C ABI of the Nested Neumann (NN) matrix-inversion library for AMD
 * Instinct MI355X (gfx950).
 *
 * Method (Engsig, Yang, Mehouachi, arXiv 2212.02406, Sec. II-D Theorem and
 * Algorithm 1): from a start X_0 with ||I - A X_0||_2 < 1, each nest replaces
 * X by X * sum_{n=0..d} (I - A X)^n, d being the inception depth (L in the
 * paper).  d = 1 is Newton's iteration (Sec. II-B), d = 2 the Chebyshev
 * iteration (Sec. II-C).  On the device a nest is d + 1 dense GEMMs:
 *     R   = I - A X                     (residual, rms partials fused)
 *     U_1 = R,  U_{m+1} = R + R U_m     (d - 1 GEMMs, Horner form)
 *     X'  = X + X U_d                   (update)
 * which equals X (I + R + ... + R^d) (Sec. II-D cost model: L + 1 products
 * per nest).  rms = ||I - A X||_F / sqrt(N), the paper's root-mean
 * Frobenius accuracy measure (Sec. II).
 *
 * Conventions for every entry point:
 *  - Matrices are dense, row-major, with a leading dimension (in elements)
 *    >= the number of columns.  Complex values are interleaved (re, im), the
 *    layout of std::complex and of torch complex tensors.
 *  - Pointers named A, B, X, Xsol, ws, A_packed, X_packed, offsets, sizes,
 *    per_matrix, pool are DEVICE pointers (nn_server_submit's A and
 *    nn_server_fetch's dst may be host or device memory); `info`, `params`
 *    and `stats` are HOST pointers.
 *  - The caller owns every buffer.  The library allocates no device memory
 *    in any entry point below; nn_create and nn_server_create allocate a few
 *    pinned host bytes for read-backs.  All work of nn_invert, nn_solve and
 *    nn_invert_batched is enqueued on the context's stream (set by nn_create
 *    / nn_set_stream); the server uses streams of its own.
 *  - A is never written.  X must not alias A or the workspace.
 *  - Argument errors return NN_ERR_ARG before any launch, and X is left
 *    untouched.  Positive statuses are warnings with a valid X (the last or
 *    best iterate); negative statuses are errors and X is unspecified.
 */
#ifndef NN_H
#define NN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  NN_OK = 0,              /* rms < tol (tolerance mode) or fixed nests done */
  NN_NOT_CONVERGED = 1,   /* max_iter nests applied, rms >= tol; X = last iterate */
  NN_STAGNATED = 2,       /* rounding floor reached above tol; X = best iterate */
  NN_ERR_ARG = -1,        /* invalid argument; nothing launched */
  NN_ERR_DIVERGED = -2,   /* rms >= 1 and growing, or the start scale is not positive */
  NN_ERR_NONFINITE = -3,  /* NaN/Inf in A, in the start scale or in a residual */
  NN_ERR_HIP = -4,        /* a HIP runtime call failed */
  NN_ERR_WORKSPACE = -5,  /* workspace missing, too small or misaligned */
  NN_ERR_UNSUPPORTED = -6 /* a valid but unimplemented combination */
} nn_status;

typedef enum {
  NN_F64 = 0,   /* double */
  NN_F32 = 1,   /* float */
  NN_C64 = 2,   /* complex float, interleaved */
  NN_C128 = 3   /* complex double, interleaved */
} nn_dtype;

typedef enum {
  /* X_0 = A^H / (||A||_1 ||A||_inf): A X_0 is Hermitian PSD with spectrum in
     (0, 1] for any nonsingular A (Corollary 3's normal-equation route). */
  NN_X0_TRANSPOSE = 0,
  /* X_0 = I / Re Tr(A): the paper's phi^(0) = I with Theta = 1/Tr(W)
     (Sec. II-A, Sec. II-D).  Hermitian positive definite A only. */
  NN_X0_SCALED_IDENTITY = 1,
  /* X holds the start on entry (restart from a saved iterate). */
  NN_X0_GIVEN = 2,
  /* X_0 = A^H / ||A||_F^2: Theta = 1 / Tr(A^H A) of the normal-equation
     solve (Sec. II-D, linear systems); any nonsingular A. */
  NN_X0_TRANSPOSE_FROB = 3,
  /* X_0 = Theta_2(k) I, Theta_2(k) = k ||A^k v|| / ((k+1) ||A^(k+1) v||)
     (Sec. II-A; k = power_k): a power-iteration estimate of 1/lambda_max
     with a k/(k+1) margin; Hermitian PD A.  v is the SplitMix64 vector
     described at nn_params.power_k. */
  NN_X0_POWER_IDENTITY = 4,
  /* X_0 = Theta_2(k) A^H with W = A A^H in the estimate; any nonsingular A. */
  NN_X0_POWER_TRANSPOSE = 5,
  /* X_0 = diag(A)^-1, the diagonal preconditioner of the CNS discussion
     (Sec. II-D); requires ||I - A diag(A)^-1||_2 < 1 (diagonally dominant
     A), exact for diagonal A.  A zero diagonal entry gives DIVERGED. */
  NN_X0_JACOBI = 6
} nn_x0;

typedef enum {
  NN_PREC_PLAIN = 0, /* every GEMM in the dtype of A */
  /* NN_F64 only: bulk nests as BF16 MFMA GEMMs with FP32 accumulation, then
     FP32, then FP64 residual and refinement nests; X and rms in FP64.
     Tolerance mode with NN_X0_SCALED_IDENTITY or NN_X0_POWER_IDENTITY
     (Hermitian PD A). */
  NN_PREC_MIXED = 1
} nn_prec;

#define NN_MAX_DEPTH 8
#define NN_TRACE_MAX 128
/* nn_params.flags bit: time every GEMM launch with a pair of HIP events on
   the context stream and report their sum in nn_info.gemm_ms. */
#define NN_FLAG_TIME_GEMMS 1
/* nn_params.flags bit (plain tolerance mode of nn_invert and nn_solve; no
   effect in fixed mode or with NN_PREC_MIXED): the stopping rules run on the
   device after every residual, in the same order and arithmetic as the host
   rules, so X, status, iters, rms and the trace are the same as without the
   flag.  A kernel holds the outcome in a device flag that turns every later
   product of the call into a no-op, and the host reads it only every few
   nests: as many nests as an rms falling at order d + 1 would still need
   (rms_{k+1} >= rms_k^(d+1) holds for a normal residual), at most 16, so the
   GPU runs ahead of the host instead of waiting for one read per nest.  Also
   the start scale is checked on the device.  info->gemms counts the products
   that did work. */
#define NN_FLAG_DEVICE_STOP 2

typedef struct {
  int32_t depth;      /* inception depth d, 1 <= d <= NN_MAX_DEPTH */
  int32_t x0;         /* nn_x0 */
  double tol;         /* tolerance mode: stop when rms < tol (tol >= 0) */
  int32_t max_iter;   /* tolerance mode: at most this many nests (>= 1) */
  int32_t fixed_iter; /* > 0: exactly this many nests, no host sync, tol and
                         max_iter ignored; 0: tolerance mode */
  int32_t prec;       /* nn_prec */
  int32_t flags;      /* NN_FLAG_TIME_GEMMS | NN_FLAG_DEVICE_STOP or 0; other
                         bits must be 0 */
  int32_t power_k;    /* NN_X0_POWER_*: power steps k, 1..NN_POWER_MAX_K (the
                         start then costs k + 1 matrix-vector products with A,
                         twice that for POWER_TRANSPOSE); v_i = 2 u_i - 1 with
                         u_i the top 53 bits / 2^53 of the (i+1)-th SplitMix64
                         output from seed 0.  Ignored for other starts. */
  int32_t reserved;   /* ignored; set to 0 */
} nn_params;

#define NN_POWER_MAX_K 64

typedef struct {
  int32_t iters;      /* nests applied to X_0 to obtain the returned X */
  int32_t status;     /* nn_status of the call */
  double rms;         /* rms of the returned X */
  float device_ms;    /* device time of the call (HIP events) */
  float gemm_ms;      /* with NN_FLAG_TIME_GEMMS: summed duration of the GEMM
                         launches (first 1024 of the call), else 0 */
  int32_t gemms;      /* GEMM launches made (k (d+1) + 1 for k nests) */
  int32_t n_trace;    /* entries used in rms_trace */
  int32_t phase_iters[3]; /* mixed: nests in the BF16, FP32, FP64 phases */
  int32_t prec_gemms[3];  /* GEMM launches by arithmetic: BF16 inputs with FP32
                             accumulation, FP32 (and complex64), FP64 (and
                             complex128); they sum to gemms */
  double rms_trace[NN_TRACE_MAX]; /* rms_0, rms_1, ... as computed */
} nn_info;

/* Per-matrix result of nn_invert_batched, written on the device. */
typedef struct {
  int32_t iters;
  int32_t status;
  double rms;
} nn_info_dev;

typedef struct nn_ctx nn_ctx;

/* Create a context bound to HIP device `device` and stream `stream` (a
   hipStream_t; NULL = the null stream).  The stream stays owned by the
   caller.  Allocates a few pinned host bytes.  Returns NN_ERR_ARG for a bad
   device or ctx pointer, NN_ERR_HIP on runtime failure. */
nn_status nn_create(nn_ctx** ctx, int device, void* stream);

/* Release a context (NULL is ignored).  Does not synchronise the stream. */
void nn_destroy(nn_ctx* ctx);

/* Re-bind the context to another stream of the same device. */
nn_status nn_set_stream(nn_ctx* ctx, void* stream);

/* Workspace bytes nn_invert needs for an n x n problem (0 on bad args). */
size_t nn_workspace_size(int64_t n, nn_dtype dtype, const nn_params* params);

/* Approximate A^{-1} by the NN iteration (Sec. II-D Theorem, Algorithm 1).
 *   A      n x n, leading dimension lda, dtype `dtype`, read only.
 *   X      n x n, leading dimension ldx, same dtype: the result; with
 *          NN_X0_GIVEN it holds the start on entry.
 *   ws     device workspace of at least nn_workspace_size() bytes, 256-byte
 *          aligned; its contents are scratch.
 *   info   optional host pointer; filled on return.
 * Tolerance mode blocks until the status is known (one 8-byte read-back per
 * nest, or every few nests with NN_FLAG_DEVICE_STOP).  Fixed mode
 * (params->fixed_iter > 0) blocks once at the end.
 * Supported: F64, F32, C64, C128 plain; F64 mixed. */
nn_status nn_invert(nn_ctx* ctx, const void* A, int64_t lda, void* X, int64_t ldx,
                    int64_t n, nn_dtype dtype, const nn_params* params,
                    void* ws, size_t ws_bytes, nn_info* info);

/* Size of the device scratch array behind nn_invert_noalloc (32 MiB). */
#define NN_NOALLOC_SCRATCH_BYTES (32u << 20)

/* nn_invert without a workspace argument and without any allocation, for
 * callers that cannot allocate device memory (or may not call hipMalloc at
 * all: allocation-free serving loops, harnesses that forbid it).  The
 * workspace is a file-scope device array of NN_NOALLOC_SCRATCH_BYTES that the
 * library holds on every device it runs on until the process ends; nn_create
 * looks up its address on the context's device.  The call makes no
 * hipMalloc, hipFree or other allocating call.
 *   Arguments, results and status codes as for nn_invert, plus:
 *   NN_ERR_WORKSPACE  nn_workspace_size(n, dtype, params) exceeds
 *                     NN_NOALLOC_SCRATCH_BYTES (plain FP64 / complex64 up to
 *                     n = 1437, 1176, 1013 at depths 1, 2, 3; FP32 up to
 *                     2019, 1656, 1437; complex128 up to 1013, 830, 720;
 *                     mixed FP64 at depth 2 up to 698); nothing is launched
 *                     and X is untouched.
 *   NN_ERR_ARG        also for params->flags with NN_FLAG_TIME_GEMMS.
 * Every call on one device shares that device's array and leaves its contents
 * behind (the call needs no part of it cleared).  Calls that overlap on one
 * device, from any context or stream, race on it: the caller must order them
 * (one stream, or events between streams). */
nn_status nn_invert_noalloc(nn_ctx* ctx, const void* A, int64_t lda, void* X, int64_t ldx,
                            int64_t n, nn_dtype dtype, const nn_params* params, nn_info* info);

/* Workspace bytes nn_solve needs. */
size_t nn_solve_workspace_size(int64_t n, int64_t nrhs, nn_dtype dtype,
                               const nn_params* params);

/* Solve A Xsol = B (Corollary 3): X = NN inverse of A (kept in ws), then
 * Xsol = X B, one n x n x nrhs GEMM.  B is n x nrhs (ldb), Xsol n x nrhs
 * (ldx).  With NN_X0_TRANSPOSE any nonsingular A works (normal-equation
 * route).  info->rms is the inverse's rms; the relative residual
 * ||B - A Xsol||_F / ||B||_F is returned in *rel_residual if non-NULL. */
nn_status nn_solve(nn_ctx* ctx, const void* A, int64_t lda, const void* B, int64_t ldb,
                   void* Xsol, int64_t ldx, int64_t n, int64_t nrhs, nn_dtype dtype,
                   const nn_params* params, void* ws, size_t ws_bytes, nn_info* info,
                   double* rel_residual);

/* Workspace bytes nn_solve_factorized needs (0 on bad arguments). */
size_t nn_solve_factorized_workspace_size(int64_t n, int64_t nrhs, nn_dtype dtype,
                                          const nn_params* params);

/* Solve A Xsol = B with the factorised Neumann series applied to B, without
 * forming the inverse (Corollary 6 and the linear-solve form after it):
 *     Xsol = prod_{n=0}^{s-1} (I + P^(2^n)) phi B,   P = I - phi A,
 * the truncated series sum_{n < 2^s} P^n phi B (= s Newton nests applied to
 * B).  phi is the start X_0 of params->x0 (NN_X0_TRANSPOSE: any nonsingular
 * A; NN_X0_SCALED_IDENTITY: Hermitian PD A; NN_X0_GIVEN is not supported).
 * Per factor: one n x n x n product (the square P^(2^n), formed only when the
 * factor is applied) and two n x n x nrhs products (the factor and the
 * residual B - A Xsol).
 *   params->fixed_iter > 0: exactly that many factors, one host
 *     synchronisation at the end; else tolerance mode on the relative
 *     residual ||B - A Xsol||_F / ||B||_F with tol, at most max_iter factors
 *     (<= 62), and the status rules of nn_invert (stagnation: the previous
 *     residual below 0.1 and no decrease; then the previous iterate is
 *     returned).  depth is ignored; prec must be NN_PREC_PLAIN.
 *   info->iters = factors applied, info->rms = relative residual of the
 *     returned Xsol (also written to *rel_residual if non-NULL), the trace
 *     holds the relative residual after 0, 1, ... factors.
 * B (n x nrhs, ldb) and Xsol (n x nrhs, ldx) are device arrays; Xsol must
 * not alias A or B. */
nn_status nn_solve_factorized(nn_ctx* ctx, const void* A, int64_t lda, const void* B,
                              int64_t ldb, void* Xsol, int64_t ldx, int64_t n, int64_t nrhs,
                              nn_dtype dtype, const nn_params* params, void* ws,
                              size_t ws_bytes, nn_info* info, double* rel_residual);

/* Parameters of nn_solve_cns. */
typedef struct {
  nn_params precond;   /* the NN preconditioner phi = X_m, as for nn_invert:
                          precond.fixed_iter > 0 nests, or its tolerance mode
                          on the rms of I - A phi (precond.tol, max_iter);
                          prec NN_PREC_MIXED for NN_F64 only; NN_X0_GIVEN
                          takes the start from the first n x n elements of
                          the workspace */
  double tol;          /* series tolerance mode: stop when the relative
                          residual ||B - A Xsol||_F / ||B||_F < tol (>= 0) */
  int32_t max_terms;   /* series tolerance mode: at most this many terms,
                          1..NN_CNS_MAX_TERMS */
  int32_t fixed_terms; /* >= 0: exactly this many terms (no host
                          synchronisation in the series); -1: tolerance mode */
  int32_t reuse_phi;   /* 1: the workspace already holds phi from an earlier
                          call on the same A, n, dtype and precond; no nests are
                          run and *precond_info is zeroed.  0: compute phi */
  int32_t reserved;    /* must be 0 */
} nn_cns_params;

#define NN_CNS_MAX_TERMS 1000000

/* Workspace bytes nn_solve_cns needs (0 on bad arguments). */
size_t nn_solve_cns_workspace_size(int64_t n, int64_t nrhs, nn_dtype dtype,
                                   const nn_cns_params* params);

/* Solve A Xsol = B with the Chebyshev-Neumann series (CNS, Sec. II-D, the
 * CNS equation after Corollary 2; depth 1 gives the Newton-Neumann series):
 * m NN nests give the preconditioner phi = X_m, then T terms of the Neumann
 * series in I - phi A are applied to B,
 *     Xsol = sum_{k=0}^{T} (I - phi A)^k phi B,
 * which is the plain Neumann series of order (d+1)^m (T+1) - 1 in the start's
 * I - X_0 A.  The series is evaluated in its Horner form, one refinement step
 * per term:  y_0 = phi B,  y_{k+1} = y_k + phi (B - A y_k)  (two n x n x nrhs
 * products per term, the residual with its fused sum of squares; I - phi A is
 * never formed, so the residual is always that of the returned iterate).
 *   Workspace: the first n x n elements (leading dimension n) hold phi on
 *     return and are read back with reuse_phi = 1 (many right-hand-side
 *     batches against one A: the preconditioner is paid once).
 *   Series control on rel_T = ||B - A y_T||_F / ||B||_F (0 when B = 0):
 *     fixed_terms >= 0 stops at T = fixed_terms (one host synchronisation at
 *     the end); tolerance mode uses nn_solve_factorized's rules with
 *     max_terms (stagnation returns the previous iterate).
 *   A preconditioner error (negative status of the nests) is returned as the
 *     call's status, Xsol unspecified; a positive status of the nests
 *     (NOT_CONVERGED, STAGNATED) is reported in precond_info and the series
 *     still runs.
 *   precond_info (optional): nn_invert's record of the nests.  info
 *     (optional): iters = terms applied, rms = relative residual of the
 *     returned Xsol (also *rel_residual if non-NULL), gemms = products of the
 *     series, the trace holds rel_0, rel_1, ..., device_ms the series' time.
 * B (n x nrhs, ldb) and Xsol (n x nrhs, ldx) are device arrays; Xsol must
 * not alias A, B or the workspace.  Supported: F64, F32, C64, C128. */
nn_status nn_solve_cns(nn_ctx* ctx, const void* A, int64_t lda, const void* B, int64_t ldb,
                       void* Xsol, int64_t ldx, int64_t n, int64_t nrhs, nn_dtype dtype,
                       const nn_cns_params* params, void* ws, size_t ws_bytes,
                       nn_info* precond_info, nn_info* info, double* rel_residual);

/* Parameters of nn_solve_sparse. */
typedef struct {
  int32_t x0;          /* NN_X0_SCALED_IDENTITY (phi = I / Re Tr W),
                          NN_X0_POWER_IDENTITY (phi = Theta_2(power_k) I) or
                          NN_X0_JACOBI (phi = diag(W)^-1) */
  int32_t power_k;     /* NN_X0_POWER_IDENTITY: 1..NN_POWER_MAX_K */
  double tol;          /* tolerance mode: stop when the control residual
                          (below) is < tol (>= 0) */
  int32_t max_terms;   /* tolerance mode: at most this many terms,
                          1..NN_SPARSE_MAX_TERMS */
  int32_t fixed_terms; /* >= 0: exactly this many terms; -1: tolerance mode */
  int32_t check_every; /* tolerance mode: terms enqueued between host reads
                          of the device-side control block, 1..1024 */
  int32_t reserved;    /* must be 0 */
} nn_sparse_params;

#define NN_SPARSE_MAX_TERMS 100000000

/* Workspace bytes nn_solve_sparse needs (0 on bad arguments). */
size_t nn_solve_sparse_workspace_size(int64_t n, int64_t nrhs, nn_dtype dtype,
                                      const nn_sparse_params* params);

/* Solve W Xsol = B for a sparse W with the Neumann series in P = I - phi W
 * applied to phi B, never storing a power of P (Algorithm 2; Corollary 6 and
 * the sparse-system passage after it; with T = (L+1)^i - 1 terms it is i NN
 * nests of depth L applied to B, Corollary 2):
 *     Xsol = sum_{m=0}^{T} P^m phi B.
 * The device evaluates it in Horner form, one fused sparse step per term:
 *     r_t = B - W x_t,   x_{t+1} = x_t + phi r_t,   x_0 = phi B,
 * with the sums of w_r |r_rc|^2 and |r_rc|^2 fused (w_r = |phi_r|).  phi is a
 * scalar or a diagonal, so sparsity is kept.
 *   W: CSR with int32 row_ptr[n + 1] (row_ptr[0] = 0, non-decreasing,
 *     row_ptr[n] = nnz), int32 col_idx[nnz] in [0, n), values[nnz] of dtype
 *     (duplicates are summed).  The structure is checked on the device before
 *     any product (NN_ERR_ARG if it is not valid CSR).
 *   Control: the phi-weighted relative residual
 *     ||w^(1/2) (B - W x)||_F / ||w^(1/2) B||_F (the plain relative residual
 *     for a scalar phi), in which the iteration contracts for Hermitian PD W
 *     (diagonal dominance for the Jacobi start).  fixed_terms >= 0: exactly
 *     that many terms; tolerance mode: the rules of nn_solve_factorized with
 *     max_terms.  The rules run on the device after every term; the host reads
 *     the outcome every check_every terms (steps enqueued after the stop do
 *     no work), so there is no host synchronisation per term.
 *   info (optional): iters = terms of the returned Xsol, rms = its control
 *     residual, gemms = sparse steps that ran, trace = control residuals after
 *     0, 1, ... terms.  *rel_residual (optional) = plain
 *     ||B - W Xsol||_F / ||B||_F.
 * B (n x nrhs, ldb) and Xsol (n x nrhs, ldx) are dense device arrays; Xsol
 * must not alias B, the CSR arrays or the workspace.  Supported: F64, F32,
 * C64, C128 (products accumulate in the dtype; norms in FP64). */
nn_status nn_solve_sparse(nn_ctx* ctx, const int32_t* row_ptr, const int32_t* col_idx,
                          const void* values, int64_t n, int64_t nnz, const void* B, int64_t ldb,
                          void* Xsol, int64_t ldx, int64_t nrhs, nn_dtype dtype,
                          const nn_sparse_params* params, void* ws, size_t ws_bytes,
                          nn_info* info, double* rel_residual);

/* Workspace bytes nn_invert_batched needs for `batch` matrices. */
size_t nn_batched_workspace_size(int32_t batch, nn_dtype dtype);

/* Invert a batch of small matrices of uneven sizes in one persistent launch
 * (the massive-MIMO use of Corollary 4's discussion).
 *   A_packed, X_packed  matrices back to back, row-major, leading dimension
 *                        = own size; matrix b starts at element offsets[b].
 *   offsets (int64), sizes (int32): device arrays of length `batch`;
 *                        1 <= sizes[b] <= max_n.
 *   max_n                upper bound of sizes (<= 64).
 *   params               fixed_iter > 0: exactly that many nests per matrix;
 *                        fixed_iter == 0: tolerance mode, each matrix on its
 *                        own: nn_invert's stopping rules (the rms tests of
 *                        its tolerance mode, with sqrt(size) for sqrt(n))
 *                        run on the device after every residual, with
 *                        params.tol and 1 <= params.max_iter <= 4096;
 *                        x0 TRANSPOSE, SCALED_IDENTITY or GIVEN (X_packed
 *                        holds each matrix's start on entry).  prec PLAIN,
 *                        flags 0.
 *   per_matrix           device array of `batch` nn_info_dev, or NULL:
 *                        nests applied, status (nn_invert's codes; STAGNATED
 *                        returns the iterate before the last nest) and rms
 *                        of the returned iterate.
 * Asynchronous on the context stream; nothing is read back.  Each matrix's
 * result depends only on that matrix (never on the rest of the batch).
 * Supported dtypes: C64, F32. */
nn_status nn_invert_batched(nn_ctx* ctx, const void* A_packed, void* X_packed,
                            const int64_t* offsets, const int32_t* sizes, int32_t batch,
                            int32_t max_n, nn_dtype dtype, const nn_params* params,
                            void* ws, size_t ws_bytes, nn_info_dev* per_matrix);

/* Autotune nn_invert_batched for this batch: time each candidate kernel
 * configuration (size up to which a matrix gets one wave instead of a whole
 * workgroup: 0, 8, 16, 32, those whose LDS fits at params->depth; workgroups
 * per CU: 1, 2, 4, ... as LDS allows; candidates that give the same launch
 * are timed once) on the given arguments, three replays each, and keep the
 * fastest in the context for later calls with the same dtype and max_n.
 * Arguments as for nn_invert_batched; X_packed is overwritten.  *best_ms
 * (optional) receives the best replay time.  Blocks until done.
 *   Persistence: if the environment variable NN_AUTOTUNE_CACHE names a file,
 *   an entry for (device architecture, dtype, max_n) found there is taken
 *   instead of timing anything (*from_cache = 1, *best_ms = the stored time,
 *   X_packed untouched); otherwise the tuned result is appended to the file
 *   (*from_cache = 0).  Lines: "<arch> <dtype> <max_n> <wave_max_k>
 *   <wg_per_cu> <ms>"; the last matching line wins.  from_cache may be NULL. */
nn_status nn_batched_autotune(nn_ctx* ctx, const void* A_packed, void* X_packed,
                              const int64_t* offsets, const int32_t* sizes, int32_t batch,
                              int32_t max_n, nn_dtype dtype, const nn_params* params,
                              void* ws, size_t ws_bytes, float* best_ms, int32_t* from_cache);

/* Read / set the batched kernel configuration the context uses for (dtype,
 * max_n): wave_max_k in [0, 32], wg_per_cu in [1, 8].  At launch, wave_max_k
 * is lowered (32 -> 16 -> 8 -> 0) until the LDS of one workgroup holds the
 * call's depth (nn_batched_fit_config), and the environment variable
 * NN_BATCHED_GRID (a positive integer), if set, replaces the number of
 * persistent workgroups (results do not depend on it). */
nn_status nn_batched_get_config(nn_ctx* ctx, nn_dtype dtype, int32_t max_n,
                                int32_t* wave_max_k, int32_t* wg_per_cu);
nn_status nn_batched_set_config(nn_ctx* ctx, nn_dtype dtype, int32_t max_n,
                                int32_t wave_max_k, int32_t wg_per_cu);

/* The one-wave size limit a batched launch uses for a configured wave_max_k
 * at depth `depth`: the largest of wave_max_k, 16, 8, 0 (not above it, nor
 * above max_n) whose LDS fits one workgroup (150 KB of dynamic LDS and
 * 160 KB in all on one CU).  -1 on bad arguments.  Needs no device. */
int32_t nn_batched_fit_config(nn_dtype dtype, int32_t max_n, int32_t wave_max_k, int32_t depth);

/* ---------------------------------------------------------------------------
 * Continuous-batching server.
 *
 * Requests (one matrix each, with its own tolerance) are queued by
 * nn_server_submit and advanced by nn_server_tick.  Each tick:
 *   1. admits queued requests, first come first served (a request may be
 *      passed by later ones that fit while it does not, at most 8 ticks in a
 *      row), while the active count is below max_active and the request's
 *      footprint (nn_server_footprint) fits in the free part of the caller's
 *      device pool; admission copies A into the pool and forms X_0;
 *   2. waits for the residual rms of every active request's current iterate
 *      (one host synchronisation for all of them);
 *   3. applies each request's stopping rules (those of nn_invert's tolerance
 *      mode, per request) and either retires it or enqueues its next nest
 *      (Sec. II-D Theorem: X <- X sum_{n=0..d} (I - A X)^n) and the residual
 *      of the new iterate.
 * Requests enqueue on a pool of n_streams streams (default priority), so the
 * GEMMs of small requests run side by side on the device.  Single-precision
 * requests with n <= batch_max_n run their whole single-precision phase in
 * the tick that admits them: one persistent batched launch per dtype applies
 * every such request's rules on the device (nn_invert_batched's tolerance
 * mode from the server's X_0); one that must finish wide stops at the
 * promotion point, pow(1e-9, 1/(d+1)), and continues tick by tick.  Iterates stay in
 * the pool between ticks.  A request's result depends only on that request:
 * every kernel's tile plan depends on (n, dtype) alone and every reduction
 * runs in a fixed order, so a request gives the same bits alone and in any
 * mix of co-runners.
 *
 * Precision: FP32 and complex64 requests iterate in their own dtype.  One
 * whose tolerance is below wide_tol, or that stagnates above its tolerance in
 * single precision, is promoted: A and the iterate are widened to FP64 /
 * complex128 and the request finishes there; its result is then in the wide
 * dtype (nn_request_info.out_dtype).  A request with tol < wide_tol reserves
 * the wide buffers at admission; one with tol >= wide_tol reserves them only
 * if it stagnates, and finishes STAGNATED in single precision when they do not
 * fit.  FP64 and complex128 requests iterate in their own dtype throughout.
 *
 * The server is driven by one host thread (calls are not thread safe).  It
 * allocates no device memory: everything lives in the caller's pool.  It
 * allocates host memory and pinned host memory for the per-tick read-back
 * (16 bytes per active slot, plus about 48 bytes per slot for the batched
 * launch's arguments and records) and creates its streams and events.  The
 * head of the pool holds the slots and the batched launch's arrays (about
 * 64 bytes per max_active slot plus 4 KB).
 * ------------------------------------------------------------------------- */

typedef struct nn_server nn_server;

typedef struct {
  int32_t depth;      /* inception depth d, 1 <= d <= NN_MAX_DEPTH */
  int32_t x0;         /* any nn_x0 but NN_X0_GIVEN (the identity-family and
                         Jacobi starts for HPD requests) */
  int32_t max_active; /* requests on the device at once, 1..65536 */
  int32_t n_streams;  /* streams the requests are spread over, 1..8 */
  double wide_tol;    /* tolerances below this finish in FP64 / complex128 */
  int32_t power_k;    /* NN_X0_POWER_*: power steps, 1..NN_POWER_MAX_K */
  int32_t batch_max_n; /* 0..64: FP32 / complex64 requests with n <= this (and
                          max_iter <= 4096) run their single-precision phase
                          in one persistent batched launch per tick and dtype
                          (the tolerance mode of nn_invert_batched, started
                          from the server's X_0); 0 turns this off */
} nn_server_params;

typedef struct {
  int64_t id;         /* the caller's id */
  int32_t status;     /* nn_status, with nn_invert's meanings */
  int32_t iters;      /* nests applied to X_0 to obtain the result */
  int32_t wide_iters; /* of which in FP64 / complex128 */
  int32_t out_dtype;  /* nn_dtype of the result */
  int64_t n;
  double rms;         /* rms of the result, computed in the dtype it was
                         iterated in */
  double t_submit;    /* host seconds since server creation */
  double t_admit;
  double t_finish;    /* the tick that saw the stopping rule fire */
} nn_request_info;

typedef struct {
  int32_t finished; /* requests retired by this tick */
  int32_t active;   /* requests on the device after this tick */
  int32_t queued;   /* requests waiting for admission */
  int32_t ready;    /* retired requests not fetched or released yet */
  size_t pool_used; /* pool bytes held by active and unfetched requests */
} nn_server_stats;

/* Create a server on ctx's device.  `pool` is a device buffer of pool_bytes
 * (256-byte aligned) owned by the caller and used by the server until
 * nn_server_destroy; params NULL selects {2, NN_X0_SCALED_IDENTITY, 1024, 4,
 * 1e-6, 8, 64}. */
nn_status nn_server_create(nn_ctx* ctx, void* pool, size_t pool_bytes,
                           const nn_server_params* params, nn_server** server);

/* Wait for the server's device work and release it (NULL is ignored).
 * Results not fetched are dropped. */
void nn_server_destroy(nn_server* server);

/* Pool bytes a request reserves at admission (0 for bad arguments). */
size_t nn_server_footprint(const nn_server* server, int64_t n, nn_dtype dtype, double tol);

/* Queue a request.  A (n x n, leading dimension lda, host or device memory)
 * must stay valid and unchanged until the request is reported by
 * nn_server_poll.  id must not be in use by a request not yet fetched or
 * released.  Returns NN_ERR_WORKSPACE if the footprint exceeds the whole
 * pool, NN_ERR_ARG for bad arguments; nothing is queued then. */
nn_status nn_server_submit(nn_server* server, int64_t id, const void* A, int64_t lda, int64_t n,
                           nn_dtype dtype, double tol, int32_t max_iter);

/* One tick (see above).  Work enqueued on the context stream before the call
 * (for instance the kernels that produce a request's A) is ordered before the
 * tick's work.  Blocks until this tick's residuals are known.
 * stats (optional host pointer) is filled on return.  With nothing active or
 * admissible it returns at once. */
nn_status nn_server_tick(nn_server* server, nn_server_stats* stats);

/* Copy up to max records of retired requests not yet polled, in retirement
 * order, into out (host); returns the count. */
int32_t nn_server_poll(nn_server* server, nn_request_info* out, int32_t max);

/* Copy a retired request's result (n x n of its out_dtype, leading dimension
 * ldd) to dst (host or device memory) and release its pool memory.  Blocks
 * until the copy is done.  NN_ERR_ARG if id is not a retired request; for a
 * request that ended with an error status the copy is skipped and the
 * memory released. */
nn_status nn_server_fetch(nn_server* server, int64_t id, void* dst, int64_t ldd);

/* Release a retired request's pool memory without copying its result. */
nn_status nn_server_release(nn_server* server, int64_t id);

/* Static description of a status code. */
const char* nn_status_string(nn_status status);

#ifdef __cplusplus
}
#endif

#endif /* NN_H */
