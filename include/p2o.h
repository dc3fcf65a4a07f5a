/*
 * p2o.h -- C ABI of the FFT-based block-Toeplitz parameter-to-observable
 * library for AMD Instinct MI355X (gfx950).
 *
 * The operator.  A linear time-invariant system stepped with a single-step
 * explicit scheme, w_{k+1} = A w_k + C m_k, d_{k+1} = B w_{k+1} (paper,
 * section 2, "Discrete LTI system"), maps a parameter series m (Nt blocks of
 * Nm values) to observations d (Nt blocks of Nd values) through the block
 * lower-triangular Toeplitz matrix of its time-domain blocks
 *
 *     d_t = sum_{k=0}^{t} F_k m_{t-k},   F_k = B A^k C,   t = 0..Nt-1
 *
 * (equations LTI-time-discrete, ShiftInvariance and p2o; time index 0-based,
 * F_k is the paper's first-column block F_{k+1,1}).  Section 4 ("FFT-based
 * GPU-accelerated p2o and p2q matvecs") applies it by embedding the Toeplitz
 * matrix in a block circulant of length L, transforming the blocks once,
 * and doing one independent Nd x Nm complex matrix-vector product per
 * frequency; the adjoint uses the conjugate-transposed Fourier blocks of the
 * same stored spectrum.
 *
 * Conventions shared by every call.
 *  - Time series are time-major and row-major: m is [nrhs][Nt][Nm], d is
 *    [nrhs][Nt][Nd], contiguous, on the device.  Element type ("I/O type")
 *    is double for P2O_FP64 plans and float for every other precision.
 *  - L = 2 * S(Nt), where S(n) is the smallest 7-smooth integer >= n; the
 *    spectrum keeps the L/2 + 1 non-redundant bins of the real transform.
 *  - The caller owns all device memory (see p2o_required_bytes and
 *    p2o_bind_storage); the plan holds host metadata only.  The apply calls
 *    never allocate and never synchronise; they enqueue on the plan's stream.
 *  - Arguments and plan state are checked before anything is enqueued.  On
 *    error nothing is enqueued, outputs are untouched, a negative status is
 *    returned and p2o_last_error() describes it.  No C++ exception crosses
 *    this interface.
 *  - Calls on one plan are not thread safe; distinct plans are independent.
 */
#ifndef P2O_H
#define P2O_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct p2o_plan p2o_plan;

/* Storage precision of the spectrum.  BF16 and FP16 store one power-of-two
 * scale per (frequency, 4096-column block) and accumulate in FP32. */
typedef enum {
    P2O_FP64 = 0,
    P2O_FP32 = 1,
    P2O_BF16 = 2,
    P2O_FP16 = 3
} p2o_precision;

/* Element type of the time-domain blocks handed to p2o_load_blocks. */
typedef enum {
    P2O_SRC_F64 = 0,
    P2O_SRC_F32 = 1
} p2o_src_dtype;

typedef enum {
    P2O_OK = 0,
    P2O_ERR_ARG = -1,        /* bad shape, pointer, size or enum value      */
    P2O_ERR_STATE = -2,      /* call out of order (e.g. apply before load)  */
    P2O_ERR_DTYPE = -3,      /* precision / element type not supported here */
    P2O_ERR_STORAGE = -4,    /* bound memory smaller than required          */
    P2O_ERR_NONFINITE = -5,  /* NaN or Inf found in the loaded blocks       */
    P2O_ERR_HIP = -6,        /* a HIP runtime call failed                   */
    P2O_ERR_NO_DEVICE = -7   /* no usable GPU                               */
} p2o_status;

/* Describe an operator with Nd sensors, Nm parameters per step and Nt steps
 * (section 2, dimensions of m, d and F after equation p2o), stored in
 * `precision`, applied to at most `max_rhs` right-hand sides per call.
 * Host-only: works without a GPU.  *out receives a new plan. */
p2o_status p2o_create(p2o_plan** out, int64_t Nd, int64_t Nm, int64_t Nt,
                      int32_t precision, int64_t max_rhs);

/* Free the plan's host state (never the caller's device memory). */
p2o_status p2o_destroy(p2o_plan* plan);

/* Derived sizes: circulant length L, number of stored frequencies L/2+1,
 * row pitch of the stored spectrum in complex elements (the smallest value
 * >= Nm that is 32 mod 64, so that rows start an odd number of 128-byte
 * lines apart; columns past Nm hold zeros), and the number of 4096-column
 * scale blocks.  Any pointer may be NULL. */
p2o_status p2o_get_layout(const p2o_plan* plan, int64_t* L, int64_t* nfreq,
                          int64_t* pitch, int64_t* nscale_blocks);

/* Device bytes the caller must provide: the spectrum store (persistent:
 * spectrum, scales, twiddles) and the workspace (scratch for apply calls
 * with up to max_rhs right-hand sides, and for loading). */
p2o_status p2o_required_bytes(const p2o_plan* plan, size_t* fhat_bytes,
                              size_t* workspace_bytes);

/* Attach caller-owned device memory (256-byte aligned).  The plan keeps the
 * pointers; the caller keeps ownership and must keep them alive until
 * p2o_destroy.  Rebinding resets the plan to "not loaded". */
p2o_status p2o_bind_storage(p2o_plan* plan, void* fhat, size_t fhat_bytes,
                            void* workspace, size_t workspace_bytes);

/* Stream (a hipStream_t, NULL = default stream) on which all later calls
 * enqueue their work. */
p2o_status p2o_set_stream(p2o_plan* plan, void* stream);

/* Transform and store columns [col0, col0+ncols) of the time-domain blocks
 * (the blocks' DFT is computed once, offline, and reused by every matvec;
 * section 4, paragraph on FFT-based p2o and p2q matvecs):
 * F_chunk is a device array [Nt][Nd][ncols] of element type src_dtype,
 * holding F_k[:, col0:col0+ncols] for k = 0..Nt-1.  For BF16/FP16 plans col0
 * must be a multiple of 4096 and ncols a multiple of 4096 unless the chunk
 * ends at Nm, so every scale block is loaded whole.  The transform runs in
 * FP64; the result is rounded to nearest-even into the storage precision.
 * Asynchronous; the caller keeps F_chunk alive until the stream reaches it. */
p2o_status p2o_load_blocks(p2o_plan* plan, const void* F_chunk, int64_t col0,
                           int64_t ncols, int32_t src_dtype);

/* Finish loading: synchronises the stream, checks that every column was
 * loaded and that no NaN/Inf was seen (P2O_ERR_NONFINITE), and marks the
 * plan ready for the apply calls. */
p2o_status p2o_load_finalize(p2o_plan* plan);

/* d = F m  (equation p2o) for nrhs right-hand sides.  m: [nrhs][Nt][Nm],
 * d: [nrhs][Nt][Nd].  nt_active (device int32[nrhs], or NULL) restricts
 * right-hand side b to its leading nt_active[b] steps: inputs past it count
 * as zero and outputs past it are written as zero (the leading block
 * principal submatrix of a lower-triangular Toeplitz matrix is the operator
 * of the shorter problem).  1 <= nrhs <= max_rhs. */
p2o_status p2o_apply_F(p2o_plan* plan, const void* m, void* d, int64_t nrhs,
                       const int32_t* nt_active);

/* d = F m exactly as p2o_apply_F, for callers that cannot allocate device
 * memory or must not touch the bound workspace (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the
 * workspace for nrhs right-hand sides is taken from a fixed scratch array in
 * device memory that the library holds on each GPU it runs on (128 MiB per
 * device, kept until the process ends), never from the plan's workspace,
 * and nothing is allocated or freed.  The spectrum must be on the current
 * device.  Every call on one GPU shares that GPU's scratch array: calls that
 * overlap on one GPU (other streams, other threads, other plans) race and
 * must be serialised by the caller.  Returns P2O_ERR_ARG, before anything
 * is enqueued, when nrhs right-hand sides need more than the array holds
 * (the message gives the size), P2O_ERR_HIP if the array's address cannot
 * be obtained; otherwise as p2o_apply_F. */
p2o_status p2o_apply_F_noalloc(p2o_plan* plan, const void* m, void* d, int64_t nrhs,
                               const int32_t* nt_active);

/* m = F^* d, the adjoint (section 2, F^* in equation mmap-problem; section 4,
 * conjugate-transposed Fourier blocks).  d: [nrhs][Nt][Nd] in,
 * m: [nrhs][Nt][Nm] out.  nt_active as for p2o_apply_F. */
p2o_status p2o_apply_Ft(p2o_plan* plan, const void* d, void* m, int64_t nrhs,
                        const int32_t* nt_active);

/* Data-space operator columns h = F F^* e (F Gamma F^* with Gamma = I, the
 * products that assemble K = Gamma_noise + F Gamma_prior F^* column by
 * column, section 4, Phase 2).  e, h: [nrhs][Nt][Nd].  The intermediate
 * parameter series is truncated to Nt steps between the two passes and never
 * leaves the workspace (on an FP16 plan as FP16 pairs with a-priori scales
 * unless P2O_OPT_FP16_OPERANDS is 0).  nt_active as for p2o_apply_F. */
p2o_status p2o_apply_FFt(p2o_plan* plan, const void* e, void* h, int64_t nrhs,
                         const int32_t* nt_active);

/* Data misfit and gradient with diagonal noise covariance (section 2, MAP
 * objective and equation mmap-problem; section 4, diagonal Gamma_noise):
 *   r = F m - d_obs,  misfit[b] = 1/2 r^T Gamma_noise^{-1} r,
 *   grad = F^* Gamma_noise^{-1} r.
 * m, grad: [nrhs][Nt][Nm]; d_obs: [nrhs][Nt][Nd]; noise_var: device double
 * array of length noise_var_len in {1, Nd, Nt*Nd} (one variance, one per
 * sensor, or one per step and sensor); misfit: device double[nrhs], reduced
 * in FP64 in a fixed order (bitwise reproducible).  nt_active as for
 * p2o_apply_F (steps past it carry no data). */
p2o_status p2o_misfit_grad(p2o_plan* plan, const void* m, const void* d_obs,
                           const double* noise_var, int64_t noise_var_len,
                           void* grad, double* misfit, int64_t nrhs,
                           const int32_t* nt_active);

/* ---------------------------------------------------------------------------
 * Offline and online phases on top of the map (section 4, Phases 2-4), with
 * the stand-in prior Gamma_prior = prior_var * I, so that
 * G^* := Gamma_prior F^* = prior_var F^* is the same block Toeplitz map as
 * F^* (the paper precomputes G^* as its own block Toeplitz matrix; with this
 * prior it needs no second spectrum).  The data-space matrix
 * K = Gamma_noise + F G^* (equations woodbury and fast-Hessian-matvec) is
 * dense, N x N with N = Nt * Nd, FP64, column-major with leading dimension
 * ldk >= N (entry (i, j) at K[j * ldk + i]), the data index being
 * j = t * Nd + s (the order of the data series [Nt][Nd]).  noise_var is a
 * device double array of 1, Nd or Nt * Nd variances as for p2o_misfit_grad.
 * ------------------------------------------------------------------------- */

/* Columns [j0, j0 + ncols) of K = Gamma_noise + prior_var F F^* (the
 * column-by-column assembly of section 4, Phase 2): one batched F F^* call on
 * prior_var times the unit vectors e_j (matrix cores for BF16 / FP16 plans),
 * the result widened to FP64 into the columns, the noise variance added on
 * the diagonal.  K is a device pointer; 1 <= ncols <= max_rhs,
 * j0 + ncols <= N.  Uses the workspace; asynchronous on the plan's stream. */
p2o_status p2o_assemble_K(p2o_plan* plan, double prior_var, const double* noise_var,
                          int64_t noise_var_len, double* K, int64_t ldk, int64_t j0,
                          int64_t ncols);

/* K from the blocks themselves (section 4, Phase 2, when the caller holds
 * the blocks F_k rather than only the loaded spectrum): since F is block
 * lower-triangular Toeplitz, block (i, j) of F F^* is
 * sum_{k <= min(i, j)} F_{i-k} F_{j-k}^T, i.e. for i >= j the prefix sum
 * over l <= j of G(i - j + l, l) along a block diagonal of the Gram matrix
 * G = A A^T of the stacked blocks A = [F_0; ...; F_{Nt-1}] (row t Nd + s is
 * sensor s of F_t, the data-space order).  Exact up to FP64 rounding (no
 * stored spectrum involved); FP64 matrix cores.  Two calls:
 *
 * p2o_gram_accumulate: G += A_c A_c^T on the lower triangle (i >= j) for a
 * chunk A_c of A's columns: blocks[(t Nd + s) ldb + c] = F_t[s, c0 + c],
 * c < ncols (device FP64; the layout a loader callback's [Nt][Nd][ncols]
 * chunk has with ldb = ncols).  G: N x N, N = Nt Nd, column-major with
 * leading dimension ldg >= N (device FP64), zeroed by the caller before the
 * first chunk; chunks may come in any order.  Asynchronous on `stream`. */
p2o_status p2o_gram_accumulate(const double* blocks, int64_t Nt, int64_t Nd, int64_t ncols, int64_t ldb, double* G,
                               int64_t ldg, void* stream);

/* p2o_gram_to_K: turns the accumulated G into K = Gamma_noise + prior_var
 * F F^* in place (the block-diagonal prefix sums, the scaling, the noise
 * variance on the diagonal, and the upper triangle mirrored from the lower
 * one: the same matrix p2o_assemble_K assembles column by column).
 * noise_var: device FP64 array of length 1, Nd or Nt Nd (as for
 * p2o_assemble_K).  Asynchronous on `stream`. */
p2o_status p2o_gram_to_K(double* G, int64_t ldg, int64_t Nt, int64_t Nd, double prior_var, const double* noise_var,
                         int64_t noise_var_len, void* stream);

/* In-place Cholesky factorisation A = L L^T of a symmetric positive definite
 * n x n FP64 matrix on the device (column-major, lda >= n; section 4,
 * Phase 2: K is factorised offline): on return the lower triangle (i >= j)
 * holds L and the strict upper triangle holds L^T (entry (i, j), i < j,
 * equals L(j, i)); the input's upper triangle is not read.  *info
 * (device int32) receives 0, or k + 1 when the k-th pivot was not positive
 * (the factor is then not usable).  Blocked right-looking algorithm (blocks
 * of 64; trailing updates on the FP64 matrix cores).  Asynchronous on
 * `stream` (a hipStream_t, NULL = default stream). */
p2o_status p2o_cholesky(double* A, int64_t n, int64_t lda, int32_t* info, void* stream);

/* X <- K^{-1} X with K = L L^T from p2o_cholesky: the two triangular solves
 * of the online phase (section 4, Phase 4), L y = x then L^T x = y, for
 * nrhs right-hand sides, X column-major n x nrhs with leading dimension
 * ldx >= n (device FP64).  L is the matrix as p2o_cholesky leaves it: the
 * forward solve reads its lower triangle, the backward solve its upper
 * triangle (L^T).  Asynchronous on `stream`. */
p2o_status p2o_cholesky_solve(const double* L, int64_t n, int64_t lda, double* X, int64_t nrhs,
                              int64_t ldx, void* stream);

/* MAP point with zero prior mean by equation real-time-parameter (section 4,
 * Phase 4): m_map = (I - G^* K^{-1} F) G^* Gamma_noise^{-1} d_obs with
 * G^* = prior_var F^*, computed as u = G^* Gamma_noise^{-1} d_obs,
 * z = K^{-1} F u (two triangular solves with L, the factor of K from
 * p2o_assemble_K and p2o_cholesky), m_map = G^* (Gamma_noise^{-1} d_obs - z):
 * two adjoint and one forward application of the map.  d_obs: [nrhs][Nt][Nd],
 * m_map: [nrhs][Nt][Nm] (I/O type), L: N x N with leading dimension ldl.
 * Uses the workspace; asynchronous on the plan's stream. */
p2o_status p2o_map_point(p2o_plan* plan, double prior_var, const double* noise_var,
                         int64_t noise_var_len, const double* L, int64_t ldl, const void* d_obs,
                         void* m_map, int64_t nrhs);

/* Posterior covariance action out = Gamma_post v by equation
 * fast-Hessian-matvec (section 4, Phase 2): Gamma_post = (I - G^* K^{-1} F)
 * Gamma_prior, i.e. w = prior_var v, out = w - G^* K^{-1} F w.  v, out:
 * [nrhs][Nt][Nm] (I/O type, distinct buffers); L as for p2o_map_point.
 * Uses the workspace; asynchronous on the plan's stream. */
p2o_status p2o_posterior_cov_apply(p2o_plan* plan, double prior_var, const double* L,
                                   int64_t ldl, const void* v, void* out, int64_t nrhs);

/* h = F G^* e for two plans on the same parameter grid (same Nm, Nt,
 * storage precision and stream, both loaded; nrhs at most both max_rhs):
 * e is a data series of G ([nrhs][Nt / r_G][Nd_G]), h one of F
 * ([nrhs][Nt / r_F][Nd_F]).  With G = F_q (the p2q map, equation p2q) this is
 * the cross product F F_q^* of the QoI phases (section 4, Phase 3); G's
 * adjoint pass and the truncate-and-re-pad run in G's workspace, F's forward
 * pass in F's.  Asynchronous on the plans' stream. */
p2o_status p2o_apply_FGt(p2o_plan* F, p2o_plan* G, const void* e, void* h, int64_t nrhs);

/* Rows [r0, r0 + nrows) of the data-to-QoI map Q = F_q (I - G^* K^{-1} F) G^*
 * Gamma_noise^{-1} (section 4, Phase 3, equation d2q-map; G^* = prior_var F^*)
 * into Q (device FP64, row r at Q + r * ldq, ldq >= N = Nt * Nd): row r is
 * Q^T e_r = prior_var Gamma_noise^{-1} (y - F F^* z) with y = F F_q^* e_r and
 * z = prior_var K^{-1} y, all in data space (no parameter-sized buffer).
 * F: the p2o plan (output stride 1), Fq: the p2q plan (any output stride;
 * Q has Nq (Nt / r) rows, the QoI index being i * Nq + q).  L: K's Cholesky
 * factor.  1 <= nrows <= max_rhs of both plans.  Uses both workspaces. */
p2o_status p2o_d2q_rows(p2o_plan* F, p2o_plan* Fq, double prior_var, const double* noise_var,
                        int64_t noise_var_len, const double* L, int64_t ldl, int64_t r0,
                        int64_t nrows, double* Q, int64_t ldq);

/* Columns [c0, c0 + ncols) of the QoI posterior covariance
 * Gamma_post(q) = F_q (I - G^* K^{-1} F) G_q^* with G_q^* = prior_var F_q^*
 * (section 4, Phase 3, equations qoi-covariance and fast-qoi-covariance),
 * C device FP64, column c at C + c * ldc, ldc >= Nq (Nt / r): column c is
 * prior_var (F_q F_q^* e_c - F_q G^* z) with z = K^{-1} F F_q^* e_c.  Plans
 * and L as for p2o_d2q_rows. */
p2o_status p2o_qoi_posterior_cov(p2o_plan* F, p2o_plan* Fq, double prior_var, const double* L,
                                 int64_t ldl, int64_t c0, int64_t ncols, double* C, int64_t ldc);

/* The online QoI prediction q = Q d (section 4, Phase 4, equation
 * real-time-qoi, zero prior mean): q[b] = Q d[b] for nrhs data vectors of N
 * values (device FP64, d[b] at d + b * N, q[b] at q + b * nq), Q as written
 * by p2o_d2q_rows.  Asynchronous on `stream`. */
p2o_status p2o_d2q_apply(const double* Q, int64_t nq, int64_t N, int64_t ldq, const double* d, double* q,
                         int64_t nrhs, void* stream);

/* Stages of the calls above, for per-stage timing. */
typedef enum {
    P2O_STAGE_R2C = 0,       /* zero-padded real FFT along time              */
    P2O_STAGE_GEMV_FWD = 1,  /* per-frequency products with Fhat_w          */
    P2O_STAGE_GEMV_ADJ = 2,  /* per-frequency products with Fhat_w^H        */
    P2O_STAGE_C2R = 3,       /* inverse FFT and truncation (misfit fused)    */
    P2O_STAGE_PROJECT = 4,   /* truncate and re-pad between F^* and F        */
    P2O_STAGE_REDUCE = 5,    /* fixed-order FP64 misfit reduction            */
    P2O_STAGE_LOAD = 6,      /* spectrum load (FFT along k, rounding)        */
    P2O_STAGE_GEMM_FWD = 7,  /* batched products with Fhat_w on matrix cores */
    P2O_STAGE_GEMM_ADJ = 8,  /* batched products with Fhat_w^H, matrix cores */
    P2O_STAGE_COUNT = 9
} p2o_stage;

/* Plan options (p2o_set_option). */
typedef enum {
    P2O_OPT_BATCHED = 0,     /* value: p2o_batched_mode                      */
    P2O_OPT_GEMM_TILE = 1,   /* value: matrix-core tile variant in [0, p2o_gemm_tile_info's count), or -1
                                (default) for the autotuned or built-in choice; both directions (a
                                variant built for one direction only leaves the other at its
                                built-in choice) */
    P2O_OPT_FFT_FIXED = 2    /* value: 1 (default) runs the time-axis FFTs (section 4's circulant
                                embedding) with kernels compiled for the plan's transform length when
                                the library has them (lengths L = 32, 256, 840, 1000), 0 always with the
                                runtime-length kernels; both compute the same transforms */,
    P2O_OPT_FP16_OPERANDS = 4, /* value: 1 (default) lets p2o_apply_FFt and the calls built on it
                                  (p2o_assemble_K, ...) keep the intermediate parameter-side spectra
                                  of an FP16 plan as FP16 pairs with per-right-hand-side power-of-two
                                  scales bounded a priori (half the bytes of complex FP32; the forward
                                  products round their right-hand sides to FP16 either way), when the
                                  call uses the matrix cores and a compiled-length transform exists;
                                  0 keeps them complex FP32 */
    P2O_OPT_OUTPUT_STRIDE = 3  /* value r >= 1 dividing Nt (default 1): the plan's data series are
                                  observed every r-th step, the multi-rate output of a p2q map whose
                                  QoIs have a coarser time grid than its parameters (section 2, remark
                                  on distinct temporal discretisations; section 5: QoIs at 1 Hz,
                                  parameters at 10 Hz).  Data series then have Nt / r steps, step i
                                  standing for step r (i + 1) - 1 of the parameter grid:
                                  p2o_apply_F returns the outputs at those steps, p2o_apply_Ft and
                                  p2o_apply_FFt take inputs there (zero between them).  Ragged
                                  lengths, the misfit and the data-space calls need r = 1. */
} p2o_option;

/* How calls with several right-hand sides do the per-frequency products.
 * AUTO: matrix cores (one launch for up to 64 right-hand sides per group,
 * FP32 accumulation; a BF16 spectrum takes BF16 products with the BF16
 * hi + lo split of the FP32 right-hand sides, an FP16 spectrum FP16 products
 * with the right-hand sides rounded to FP16 after a per-right-hand-side
 * power-of-two scale) when the spectrum is BF16 or FP16 and nrhs >= 2,
 * otherwise one streaming matrix-vector pass per right-hand side.  GEMV forces the latter; MFMA
 * forces the former (BF16 plans, and FP16 plans whose one-frequency spectrum
 * is under 4 GiB; P2O_ERR_DTYPE otherwise).  FP16 plans use the LDS-ring
 * tile variants only (a forced other variant takes the built-in choice). */
typedef enum {
    P2O_BATCHED_AUTO = 0,
    P2O_BATCHED_GEMV = 1,
    P2O_BATCHED_MFMA = 2
} p2o_batched_mode;

/* Set a plan option; takes effect for later calls. */
p2o_status p2o_set_option(p2o_plan* plan, int32_t option, int64_t value);

/* Matrix-core tile variants of the batched products (section 4's per-frequency
 * products as complex GEMMs, one per frequency).  Variant `tile` assigns
 * 32 * row_groups * blocks output rows (sensors, or parameter columns for the
 * adjoint) and rhs_per_group right-hand sides to a workgroup and stages K in
 * steps of 8 * substeps entries.  Some variants exist for one direction
 * only (the LDS-ring kernels); the autotuner times each variant in the
 * directions it exists for.  Returns P2O_ERR_ARG for an unknown variant;
 * variants are numbered from 0 without gaps, so the first index that fails
 * is the count.  Any output pointer may be NULL. */
p2o_status p2o_gemm_tile_info(int32_t tile, int32_t* row_groups, int32_t* substeps, int32_t* blocks,
                              int32_t* rhs_per_group);

/* Autotuner: times every tile variant of the forward and the adjoint
 * matrix-core products with `nrhs` right-hand sides on this plan's loaded
 * spectrum (one warm-up and `reps` timed launches each, HIP events on the
 * plan's stream), keeps the fastest for later calls with exactly `nrhs`
 * right-hand sides, and returns the choices and their mean launch times in
 * milliseconds (any output pointer may be NULL).  Uses the workspace as
 * operands (its contents are overwritten) and synchronises the stream.
 * Needs a loaded BF16 or FP16 plan whose calls with nrhs right-hand sides
 * use the matrix cores (P2O_ERR_DTYPE otherwise; FP16 plans time the
 * LDS-ring variants only), 1 <= nrhs <= max_rhs and 1 <= reps <= 100. */
p2o_status p2o_autotune(p2o_plan* plan, int64_t nrhs, int32_t reps, int32_t* fwd_tile, int32_t* adj_tile,
                        double* fwd_ms, double* adj_ms);

/* Per-stage timing with HIP events recorded on the plan's stream around
 * every launch (enable = 1) or not (enable = 0).  Either call resets the
 * totals.  Recording adds one event pair per launch and never synchronises. */
p2o_status p2o_profile_enable(p2o_plan* plan, int32_t enable);

/* Total device time in milliseconds and number of launches of `stage` since
 * profiling was enabled.  Waits for the recorded events (synchronising). */
p2o_status p2o_profile_read(p2o_plan* plan, int32_t stage, double* total_ms, int64_t* launches);

/* As p2o_profile_read, restricted to launches made by calls with `nrhs`
 * right-hand sides (nrhs = 0: the spectrum loads). */
p2o_status p2o_profile_read_nrhs(p2o_plan* plan, int32_t stage, int64_t nrhs, double* total_ms,
                                 int64_t* launches);

/* Streaming probe for roofline context (not part of the operator): mode 0
 * reads `bytes` from `src` (non-temporal; each wavefront reads 2 KB chunks,
 * one contiguous kilobyte per load instruction; `dst` receives one 32-bit
 * word per workgroup, at least `blocks` words), mode 1 copies `bytes` from
 * `src` to `dst` (16 bytes per lane).  bytes must be a multiple of 2048 for
 * mode 0 and of 32 for mode 1, blocks in [1, 65536].  Enqueued on `stream`. */
p2o_status p2o_bandwidth_probe(int32_t mode, const void* src, void* dst, size_t bytes,
                               int32_t blocks, void* stream);

/* Human-readable name of a status code (static storage). */
const char* p2o_status_string(int32_t status);

/* Message of the last failed call on this thread ("" if none). */
const char* p2o_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* P2O_H */
