/*
 * elm.h -- C ABI of libelm, an MI355X (gfx950) implementation of the training
 * path of the rank-based pseudoinverse Extreme Learning Machine of Ragala &
 * Kumar, "Rank Based Pseudoinverse Computation in Extreme Learning Machine
 * for large Datasets" (arXiv 2011.02436).
 *
 * Problem (Section 2.1): N samples (x_i, t_i) in R^d x R^m, L hidden nodes with
 * random weights w_j and biases b_j, hidden matrix H[i][j] = g(w_j . x_i + b_j)
 * with g the logistic sigmoid (eqs. 1 and 4; Section 4 names the sigmoid),
 * output weights beta = H^+ T (eqs. 3 and 5), prediction H beta (step 3 of
 * the three-step ELM).  The rank step follows Section 3 (eq. 6, algorithm
 * steps 3-4): a permutation P putting r = rank(H) independent columns first,
 * H P = [H1 H2].  With H2 = H1 K the pseudoinverse is assembled from the
 * full-rank factorisation H = F G, F = H1, G = [I K] P^T:
 *   H^+ = G^T (G G^T)^-1 (F^T F)^-1 F^T,  F^T F = R11^T R11,  G G^T = I + K K^T,
 * where R = [R11 R12] comes from a diagonally pivoted Cholesky of the Gram
 * (eq. 8; H H^T instead of H^T H when N < L, as stated just before eq. 8).
 *
 * Conventions for every entry point:
 *  - Pointers are DEVICE pointers unless the argument says "host".  The caller
 *    owns every buffer passed in; the library owns handles, factors and its
 *    internal workspace (allocated with hipMalloc, released by the matching
 *    destroy call).
 *  - Matrices are row-major with an explicit leading dimension (elements
 *    between consecutive rows).  "Sample-major" H is N x L (row i = sample i,
 *    ld >= L); "node-major" H is its transpose, L x N (row j = node j,
 *    ld >= N).
 *  - Work is enqueued on the handle's HIP stream and is asynchronous unless an
 *    argument says the call synchronises.
 *  - Arguments are validated before any device work; an invalid call returns
 *    an error code and enqueues nothing.  Errors are reported only through the
 *    return value (and elm_last_error for a message); nothing is thrown.
 *  - Calls on one handle must not overlap from several host threads.
 */
#ifndef ELM_H
#define ELM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    ELM_OK = 0,
    ELM_ERR_INVALID_ARG = 1,    /* null pointer, size <= 0, unknown enum, tolerance out of range */
    ELM_ERR_SHAPE = 2,          /* leading dimension too small, or shapes that do not match */
    ELM_ERR_ALLOC = 3,          /* device workspace allocation failed */
    ELM_ERR_HIP = 4,            /* a HIP runtime call (launch, copy, synchronise) failed */
    ELM_ERR_NOT_PSD = 5,        /* the Gram had a NaN/Inf diagonal (non-finite input) */
    ELM_ERR_NO_CONVERGENCE = 6, /* refinement stopped above the requested residual */
    ELM_ERR_UNSUPPORTED = 7     /* valid but not implemented combination of dtypes/layouts */
} elm_status;

typedef enum {
    ELM_F64 = 0,
    ELM_F32 = 1,
    ELM_BF16 = 2,
    ELM_F16 = 3
} elm_dtype;

typedef enum {
    ELM_SAMPLE_MAJOR = 0, /* H is N x L, row = sample */
    ELM_NODE_MAJOR = 1    /* H is L x N, row = hidden node */
} elm_layout;

typedef struct elm_handle elm_handle;
typedef struct elm_factor elm_factor;

/* Per-solve report (host struct, filled by elm_pinv_solve). */
typedef struct {
    int64_t rank;              /* r */
    int32_t transposed;        /* 1 if the rank step used H H^T (N < L) */
    int32_t iterations;        /* refinement corrections applied */
    double ne_residual;        /* final ||H^T (T - H beta)||_F / ||H^T T||_F (FP64), -1 if not computed */
    double ne_history[32];     /* residual before each correction (first `iterations`+1 entries) */
} elm_solve_info;

/* ------------------------------------------------------------------------ */
/* Handle                                                                    */
/* ------------------------------------------------------------------------ */

/* Create a handle bound to `stream` (a hipStream_t; NULL = the default
 * stream) on the current HIP device.  *out receives a library-owned handle.
 * Errors: INVALID_ARG if out is NULL; HIP if the device cannot be queried. */
elm_status elm_create(elm_handle** out, void* stream);

/* Destroy a handle and free its workspace (synchronises its stream).
 * NULL is accepted and ignored. */
elm_status elm_destroy(elm_handle* h);

/* Rebind the handle to another stream (no synchronisation). */
elm_status elm_set_stream(elm_handle* h, void* stream);

/* Static description of a status code. */
const char* elm_status_string(elm_status s);

/* Message describing the last error returned on this handle ("" if none).
 * The string stays valid until the next call on the handle. */
const char* elm_last_error(const elm_handle* h);

/* ------------------------------------------------------------------------ */
/* Step 2 of the RBP-ELM algorithm: the hidden-layer matrix, eqs. (1), (4).   */
/* ------------------------------------------------------------------------ */

/* H[i][j] = 1 / (1 + exp(-(sum_k X[i][k] W[k][j] + b[j]))).
 *
 * X: N x d, ld ldx >= d.  W: d x L, ld ldw >= L.  b: L.  All of dtype `dt`,
 * which is ELM_F64 or ELM_F32; the products are accumulated in `dt` and the
 * sigmoid is evaluated in `dt`.
 * H (optional, may be NULL): sample-major N x L of dtype `dt`, ld ldh >= L.
 * Hlp (optional, may be NULL): node-major L x N copy, ld ldlp >= N, of dtype
 *   lp_dt (ELM_BF16, ELM_F16 or ELM_F32), rounded to nearest even from the
 *   same `dt` value written to H.  It feeds the low-precision Gram.  With
 *   ldlp a multiple of 64 elements and Hlp 16-byte aligned (the layout the
 *   library gives its own copies), every 64-sample stage of a row that the
 *   16-bit Gram loads is whole 128-byte lines; other leading dimensions give
 *   the same Gram, about 5% more slowly.
 * At least one of H and Hlp must be non-NULL.  N, d, L >= 1. */
elm_status elm_hidden(elm_handle* h, int64_t N, int64_t d, int64_t L,
                      const void* X, int64_t ldx, const void* W, int64_t ldw,
                      const void* b, elm_dtype dt,
                      void* H, int64_t ldh,
                      void* Hlp, int64_t ldlp, elm_dtype lp_dt);

/* ------------------------------------------------------------------------ */
/* Steps 3-4: permutation P and rank r (eq. 6), and the full-rank factor.     */
/* ------------------------------------------------------------------------ */

/* Factor the Gram of H: M = H^T H when N >= L, M = H H^T when N < L (n x n
 * with n = min(N, L)).  Accepted inputs (dtype, layout):
 *   (F64, SAMPLE_MAJOR)   FP64 Gram on FP64 MFMA (both orientations);
 *   (F32, NODE_MAJOR)     FP32 Gram on FP32 MFMA, N >= L only;
 *   (BF16|F16, NODE_MAJOR) 16-bit Gram on MFMA with FP32 accumulation, N >= L.
 * The Gram is accumulated in a fixed order per element, so bitwise-equal
 * columns of H give bitwise-equal Gram rows.  It is then widened to FP64 and
 * factored in FP64 by a greedy diagonally pivoted Cholesky: at each step the
 * pivot is the remaining index with the largest Schur-complement diagonal
 * (lowest original index on exact ties); the factorisation stops when that
 * diagonal is <= tau, tau = tau_rel * max_j M_jj, or, when tau_rel <= 0,
 * 16 (n + K) 2^-53 max_j M_jj with K the number of products summed into each
 * Gram entry (N for H^T H, L for H H^T), which keeps the Gram's own rounding
 * from passing for a pivot (tau_rel must be < 1).  Then K = R11^-1 R12 and the
 * Cholesky factor of I + K K^T (or of I + K^T K when n - r < r, used through
 * the Woodbury identity) are formed, all in FP64.
 *
 * *out receives a library-owned factor (free with elm_factor_destroy).
 * rank (host, may be NULL) receives r.  This call synchronises the stream
 * (the rank sizes the later steps; the duplicate check and the certified
 * path below read a few values back each).
 * Errors: INVALID_ARG / SHAPE / UNSUPPORTED as above; NOT_PSD if the Gram has
 * a non-finite diagonal; ALLOC; HIP. */
elm_status elm_rank_factor(elm_handle* h, int64_t N, int64_t L,
                           const void* H, int64_t ldh, elm_dtype h_dt, elm_layout layout,
                           double tau_rel, elm_factor** out, int64_t* rank);

/* The Gram step alone (eq. 8): M = H^T H (N >= L) or H H^T (N < L), n x n
 * FP64 with n = min(N, L), written in full (both triangles, exactly
 * symmetric) to the caller's M (ld ldm >= n).  Same accepted inputs and the
 * same kernels as elm_rank_factor; asynchronous.  A node-major 16-bit H is
 * read fastest with ldh a multiple of 64 elements (see elm_hidden's Hlp). */
elm_status elm_gram(elm_handle* h, int64_t N, int64_t L, const void* H, int64_t ldh,
                    elm_dtype h_dt, elm_layout layout, double* M, int64_t ldm);

/* elm_gram for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc).
 * Same arguments, accepted inputs and result as elm_gram (its FP64 Gram on
 * the 128 x 128 Gram tiles, which take each element's products in the order
 * of elm_gram's FP64 GEMM route); the
 * split-K partial tiles go to a static device array of 64 MiB per GPU
 * (allocated with the library's code on each device it runs on and held
 * until the process ends) instead of the handle's workspace, and this call
 * allocates nothing.  The K splits are those of elm_gram's default rule
 * (autotuned counts are not used), lowered until the partial tiles fit:
 * 128 x 128 FP64 tiles (128 KiB each), FP32 (64 KiB) or 256 x 256 FP32
 * partials of the 16-bit Gram (256 KiB), times the number of upper tiles,
 * times the splits.  With the default rule's count the result is bitwise
 * that of elm_gram; with fewer splits it differs by rounding only.
 * Orders whose tiles do not fit even unsplit (about n > 5600 for the 16-bit
 * and FP32 Grams, n > 3900 for FP64) are rejected with ELM_ERR_SHAPE.
 * All calls on one GPU share the array (it keeps the last call's partials):
 * calls that overlap on one GPU, from several streams or host threads, race.
 * Errors: as elm_gram, plus SHAPE for an order beyond the array and HIP if
 * the array's device address cannot be looked up. */
elm_status elm_gram_noalloc(elm_handle* h, int64_t N, int64_t L, const void* H, int64_t ldh,
                            elm_dtype h_dt, elm_layout layout, double* M, int64_t ldm);

/* Autotuner of the 16-bit Gram's tile schedule.  The Gram of a node-major
 * BF16/FP16 copy Hn (L x N, ld ldn >= N, N >= L; as for elm_gram) is split
 * along the samples into work items of one 256 x 256 output tile each, and
 * the number of splits trades the length of a work item (blocks that share
 * operand panels stay in step, the last round is shorter) against one more
 * FP32 partial tile per split.  This call times the Gram (and its partial
 * sums) of the caller's data with the default rule's split count and with
 * 1/2, 3/4, 3/2 and 2 times it (1 .. 48 splits, at least 2048 samples each),
 * and keeps the fastest (the default's count unless another is at least 2%
 * faster) as the handle's ELM_TUNE_GRAM_SPLITS row for the (dtype, L, N)
 * buckets: later 16-bit Grams of shapes in those buckets on this handle
 * (elm_gram, elm_rank_factor, elm_train, elm_train_batched) use it.  FP32
 * node-major and FP64 sample-major copies tune the FP32/FP64 Gram's K chunks
 * the same way (candidates 1/2, 3/4, 1, 3/2, 2 times the default count,
 * ELM_TUNE_GRAM_CHUNKS rows).
 * splits_out and ms_out (host, may be NULL) receive the choice and its time
 * in milliseconds.  Synchronises the handle's stream; uses a scratch Gram of
 * L x L FP64 in the handle's workspace.
 * Errors: INVALID_ARG; SHAPE; UNSUPPORTED (N < L; FP64 must be sample-major,
 * the others node-major). */
elm_status elm_autotune_gram(elm_handle* h, int64_t N, int64_t L, const void* Hn, int64_t ldn,
                             elm_dtype dt, int32_t* splits_out, double* ms_out);

/* Grow a factor by new hidden nodes: the incremental form of the rank step
 * for a hidden-size sweep (adding nodes to a trained network, as the
 * incremental ELM variants the paper's introduction surveys do), reusing the
 * smaller layer's factorisation.
 *
 * f: a factor of the FP64 column Gram H^T H of an N x L0 hidden matrix H (from
 * elm_rank_factor on FP64 sample-major H with N >= L0, or an earlier
 * elm_factor_grow).  H64: the grown FP64 sample-major hidden matrix H' = [H Hn]
 * (N x L, ld ldh64 >= L, L > L0, N >= L) whose first L0 columns are that H.
 * Only the new Gram blocks H^T Hn and Hn^T Hn are formed (2 N L0 (L - L0) +
 * N (L - L0)^2 flops instead of N L^2); f's accepted pivots stay first, the
 * rows of its R extend over the new columns by a triangular solve, and the
 * greedy diagonal pivoting continues on the Schur complement of the new
 * columns (f's rejected positions cannot become pivots: their Schur
 * diagonals are already below the threshold and only decrease).  The
 * threshold is elm_rank_factor's for the grown shape (tau_rel as there).
 * When f's decision would not stand under it (an accepted pivot at or below
 * the grown threshold, or a rejected one above), H' is factored from scratch
 * instead.  Either way the rank and beta = H'^+ T (through elm_pinv_solve)
 * are those of elm_rank_factor on H'; the pivot order may differ.
 * *out receives a new library-owned factor (f is unchanged); rank (host, may
 * be NULL) its rank; grown (host, may be NULL) 1 when it was grown, 0 when
 * factored from scratch.  Synchronises the stream.
 * Errors: INVALID_ARG; SHAPE (N differs from f's, L <= L0, ldh64);
 * UNSUPPORTED (f not of an FP64 column Gram, N < L); NOT_PSD; ALLOC; HIP. */
elm_status elm_factor_grow(elm_handle* h, const elm_factor* f, int64_t N, int64_t L,
                           const double* H64, int64_t ldh64, double tau_rel,
                           elm_factor** out, int64_t* rank, int32_t* grown);

/* The autotuners' table.  Each row holds a tile-schedule choice of the
 * library for one kind of kernel, one operand dtype and the power-of-two
 * buckets of the Gram's order and reduction length (n_log2 = ceil(log2 n),
 * k_log2 = ceil(log2 K); -1 for "any"):
 *   ELM_TUNE_GRAM_SPLITS  K splits of the 16-bit Gram (work items of one
 *                         256 x 256 tile over N / splits samples);
 *   ELM_TUNE_GRAM_CHUNKS  K chunks of the FP32/FP64 Gram (128 x 128 tiles);
 *   ELM_TUNE_PANEL        panel width of the greedy pivoted Cholesky for
 *                         orders up to 4096 (one value for all: the batched
 *                         form shares panels across problems, and a single
 *                         training must take the same width to give the same
 *                         bits); dtype and buckets -1.
 * A shape without a row takes the default rules.  The choices change speed
 * and rounding order, never the rank decision's rule or the stopping rules. */
typedef enum { ELM_TUNE_GRAM_SPLITS = 1, ELM_TUNE_GRAM_CHUNKS = 2, ELM_TUNE_PANEL = 3 } elm_tune_kind;
typedef struct {
    int32_t kind;     /* elm_tune_kind */
    int32_t dtype;    /* elm_dtype of the Gram's operand, or -1 */
    int32_t n_log2;   /* bucket of the Gram's order, or -1 */
    int32_t k_log2;   /* bucket of the reduction length (samples), or -1 */
    int32_t value;    /* splits, chunks or panel width */
} elm_tune_entry;

/* The handle's table: *count (host) receives the number of rows, and up to
 * `capacity` rows are copied to out (host, may be NULL with capacity 0). */
elm_status elm_tune_table_get(const elm_handle* h, elm_tune_entry* out, int32_t capacity,
                              int32_t* count);
/* Replace the handle's table by `count` rows (host array; count 0 clears it).
 * Errors: INVALID_ARG for an unknown kind or a value out of range (splits and
 * chunks 1..64, panel widths 32, 64, 128 or 256). */
elm_status elm_tune_table_set(elm_handle* h, const elm_tune_entry* rows, int32_t count);
/* Persist the table as text (one row per line: kind dtype n_log2 k_log2
 * value) / read such a file back, replacing the table.  Errors: INVALID_ARG
 * for a null path, a file that cannot be opened or a malformed row. */
elm_status elm_tune_table_save(const elm_handle* h, const char* path);
elm_status elm_tune_table_load(elm_handle* h, const char* path);

/* r of a factor (host read, no synchronisation needed). */
elm_status elm_factor_rank(const elm_factor* f, int64_t* rank);

/* Copy the pivot order (original index at each pivoted position, first r
 * entries independent) into host array piv_host[n]; n = min(N, L).
 * Synchronises the handle's stream. */
elm_status elm_factor_pivots(elm_handle* h, const elm_factor* f, int32_t* piv_host);

/* Diagnostics of the rank decision (host struct, filled by
 * elm_factor_get_info; no synchronisation).  Accepted pivots of the greedy
 * pivoted Cholesky are non-increasing, so the last one is the smallest.
 * noise_floor estimates the rounding noise of the Schur diagonals of the Gram
 * actually factored: a column that is an exact combination of others keeps,
 * after rounding H to unit roundoff u, a Schur diagonal near u^2/3 times the
 * largest diagonal, and FP32 accumulation over kc products adds about
 * sqrt(kc) 2^-24 per Gram entry.  `reliable` is 1 when the decision clears
 * that noise: last_pivot >= 2 noise_floor (r > 0) and first_rejected >=
 * -2 noise_floor (r < n).  A 0 means that the rank found on a low-precision
 * Gram may differ from the FP64 one: the caller should factor a
 * higher-precision Gram (elm_train does so by itself).
 *
 * Certified full rank (Grams of order >= the handle's
 * ELM_OPT_FULL_RANK_MIN_ORDER): the greedy pivots never increase and the
 * last one equals 1 / (M^-1)_jj for the last remaining index j, so all of
 * them are at least lambda = 1 / max_j (M^-1)_jj.  The library first factors
 * M without pivoting (blocked, MFMA updates) and computes lambda from the
 * rows of the inverse factor; when lambda >= max(64 tau, 2 noise_floor) the
 * greedy rule provably keeps every position (r = n), the identity order is
 * used, certified_full_rank is 1 and last_pivot reports lambda (a lower bound
 * on the greedy rule's smallest pivot).  Otherwise the greedy factorisation
 * runs as usual.  Duplicated nodes (Gram rows i != j bitwise equal, which
 * equal columns of H always give; found from the pairs of equal diagonal
 * values with M_ij = M_ii) are set aside first: the greedy rule never pivots
 * a copy after its original (the copy's Schur diagonal is then zero up to
 * rounding), so on the remaining distinct nodes it is the greedy rule on
 * their Gram, which the certificate decides.  On success the order is the
 * distinct nodes ascending, then the copies ascending; r is the number of
 * distinct nodes, certified_full_rank is 2, last_pivot is lambda of their
 * Gram and first_rejected 0 (the copies' R12 columns are their originals'
 * columns of R11). */
typedef struct {
    int64_t rank;          /* r */
    int64_t n;             /* order of the Gram, min(N, L) */
    int32_t transposed;    /* 1: Gram H H^T (N < L) */
    int32_t gram_dtype;    /* elm_dtype of the operand the Gram was formed from */
    double max_diag;       /* largest Gram diagonal (the first pivot) */
    double last_pivot;     /* smallest accepted pivot; +inf if r = 0 */
    double first_rejected; /* largest remaining Schur diagonal at the stop; -inf if r = n */
    double tau;            /* absolute stopping threshold */
    double noise_floor;    /* absolute noise scale of the Schur diagonals */
    int32_t reliable;      /* see above */
    int32_t certified_full_rank; /* 1: rank n certified without the greedy steps; 2: the
                                    distinct nodes certified after setting aside copies */
} elm_factor_info;

elm_status elm_factor_get_info(const elm_factor* f, elm_factor_info* out);

/* Free a factor.  NULL is accepted. */
elm_status elm_factor_destroy(elm_factor* f);

/* ------------------------------------------------------------------------ */
/* Steps 5-9: beta = H^+ T (eqs. 5, 7) from the factor, with optional FP64   */
/* refinement on the normal-equation residual.                               */
/* ------------------------------------------------------------------------ */

/* T: N x m sample-major FP64 targets, ld ldt >= m (one-hot rows for
 * classification).  H64: the FP64 sample-major hidden matrix (N x L, ld
 * ldh64 >= L) that beta is the least-squares solution for; it supplies
 * H^T T and the refinement residuals.  beta: L x m FP64 output, ld ldbeta
 * >= m.  1 <= m <= 64.
 *
 * beta_0 = H^+ T through the factor; then, while the relative normal-equation
 * residual ||H^T (T - H beta)||_F / ||H^T T||_F exceeds ir_tol and fewer
 * than ir_max_iter corrections were made, beta += H^+ (T - H beta) with H^+
 * applied through the (possibly low-precision-derived) factor.  With
 * ir_max_iter >= 1 at least one correction is made whatever the first
 * residual: beta_0's residual can sit at its rounding floor while its forward
 * error is about kappa^2 eps (kappa the condition number of H on its rank),
 * and the first correction removes that.  The loop also
 * stops when a correction did not lower the residual.  A correction that
 * raised it more than fourfold diverged and is taken back (beta is then the
 * previous iterate); a smaller rise is rounding noise at the residual's
 * floor, and that correction is kept (near the floor a correction still
 * removes forward error that the residual does not show).  The reported
 * residual is always that of the returned beta, and `iterations` counts the
 * corrections kept.  ir_max_iter = 0 gives beta_0 and
 * skips the residual.  ir_tol must be in [0, 1).
 * info (host, may be NULL) receives rank, iterations and residuals.
 * Synchronises once per refinement iteration.
 * Errors: NO_CONVERGENCE if ir_max_iter > 0 and the final residual is above
 * ir_tol (beta then holds the last iterate); INVALID_ARG; SHAPE; ALLOC; HIP. */
elm_status elm_pinv_solve(elm_handle* h, const elm_factor* f, int64_t m,
                          const double* T, int64_t ldt,
                          const double* H64, int64_t ldh64,
                          double ir_tol, int32_t ir_max_iter,
                          double* beta, int64_t ldbeta, elm_solve_info* info);

/* The paper's own block form of the solve (Section 3, eqs. 13-23; algorithm
 * steps 5-9) for a hidden matrix of full column rank.  The columns, in the
 * order piv (device int32 array of L original indices; NULL = identity), are
 * split as H P = [H1 H2] with H1 the first `split` of them (1 <= split <= L)
 * and H2 the other L - split, and
 *   A = H2^T H2 (eq. 20),  B = A^-1 H2^T T (eq. 21),
 *   D = H1^T C H1 with C = I - H2 A^-1 H2^T (eqs. 22-23),
 *   beta1 = D^-1 H1^T (T - H2 B),  beta2 = B - A^-1 H2^T H1 beta1 (eq. 19,
 *   read with the transpose on H1 that the printed eq. 19 omits),
 *   beta[piv] = [beta1; beta2] (eq. 7's block order),
 * all in FP64.  Every block product is taken from the Gram M = H^T H and
 * Z = H^T T, so the N x N matrix C is never formed (D = M11 - M12 A^-1 M21).
 * H64: FP64 sample-major N x L (ld ldh64 >= L), N >= L; T: N x m FP64 (ld
 * ldt >= m), 1 <= m <= 64.  M (may be NULL): the FP64 Gram H^T H (L x L, ld
 * ldm >= L, e.g. from elm_gram on H64); when NULL it is formed here in the
 * handle's workspace.  beta: L x m FP64 (ld ldbeta >= m).  For a rank-
 * deficient H the block form has no solution (A or D is singular); use
 * elm_rank_factor and elm_pinv_solve.  Synchronises the stream once.
 * Errors: INVALID_ARG; SHAPE (N < L, leading dimensions); NOT_PSD when a
 * pivot of the Cholesky factorisation of A or D is at or below the rank
 * step's default threshold 16 (L + N) 2^-53 max_j M_jj (H is then not of full
 * column rank to working precision) or the Gram has a non-finite diagonal;
 * ALLOC; HIP. */
elm_status elm_block_solve(elm_handle* h, int64_t N, int64_t L, int64_t m,
                           const double* H64, int64_t ldh64, const double* T, int64_t ldt,
                           const double* M, int64_t ldm, int64_t split, const int32_t* piv,
                           double* beta, int64_t ldbeta);

/* ------------------------------------------------------------------------ */
/* The whole training (steps 2-9) with the precision policy.                 */
/* ------------------------------------------------------------------------ */

typedef struct {
    elm_solve_info solve;    /* of the solve that produced beta */
    elm_factor_info factor;  /* of the factor that produced beta */
    int32_t gram_dtype;      /* elm_dtype of the Gram that produced beta */
    int32_t escalations;     /* precision steps taken after a failed guard (0-2) */
    int32_t guard;           /* last failed guard: 0 none, 1 rank decision within the
                                Gram's noise (elm_factor_info.reliable = 0), 2 the
                                refinement did not reach ir_tol */
} elm_train_info;

/* beta = H^+ T for H = sigma(X W + b) (Section 2.1; algorithm steps 2-9):
 * elm_hidden -> elm_rank_factor -> elm_pinv_solve in one call.
 *
 * X (N x d), W (d x L), b (L), T (N x m): FP64, leading dimensions >= row
 * lengths.  H64: caller buffer N x L FP64 (ld ldh64 >= L), receives H.
 * gram_dt selects the form: ELM_F64 factors the FP64 Gram of H64 (plain form);
 * ELM_F32 / ELM_BF16 / ELM_F16 factor the Gram of a node-major copy of H
 * rounded to that type (precision form), written to Hlp (L x N, ld ldlp >= N,
 * of type gram_dt; a multiple of 64 elements for the fastest Gram, as for
 * elm_hidden) or, when Hlp is NULL, to library workspace.  When N < L the
 * FP64 form is used whatever gram_dt says (the low-precision Gram needs N >= L).
 * Precision policy: if the rank decision on a low-precision Gram is within its
 * rounding noise (elm_factor_info.reliable = 0) or the refinement does not
 * reach ir_tol, the Gram is formed again one step up (16-bit -> FP32 -> FP64)
 * and the factor and solve are redone; info reports the steps taken.
 * tau_rel, ir_tol, ir_max_iter as for elm_rank_factor / elm_pinv_solve.
 * Y (N x m FP64, ld ldy >= m) and labels (N int32), each optional: the
 * training-set outputs H beta and their row arg-max (lowest index on ties) for
 * the returned beta (step 3 of the three-step ELM; Table 2's training
 * accuracy), taken from the last refinement pass, which evaluates H beta for
 * that beta anyway (a separate pass when ir_max_iter = 0).  Need m <= 16.
 * factor_out (may be NULL) receives the final factor (caller frees it).
 * Errors: as the three calls; NO_CONVERGENCE only when the FP64 form does not
 * reach ir_tol (beta then holds the last iterate). */
elm_status elm_train(elm_handle* h, int64_t N, int64_t d, int64_t L, int64_t m,
                     const double* X, int64_t ldx, const double* W, int64_t ldw,
                     const double* b, const double* T, int64_t ldt,
                     elm_dtype gram_dt, double* H64, int64_t ldh64,
                     void* Hlp, int64_t ldlp,
                     double tau_rel, double ir_tol, int32_t ir_max_iter,
                     double* beta, int64_t ldbeta,
                     double* Y, int64_t ldy, int32_t* labels,
                     elm_train_info* info, elm_factor** factor_out);

/* elm_train without storing H: the hidden matrix is formed chunk by chunk
 * (chunk_rows samples at a time) and consumed at once, so device memory is
 * O(L^2 + chunk_rows L + L m) instead of the N x L FP64 H plus its copy: the
 * form for N beyond what HBM holds (the paper's closing remarks name memory
 * as the limit for large data).  Pass 1 over the samples forms each chunk's
 * hidden rows (the node-major gram_dt copy only, or FP64 for the FP64 form)
 * and adds the chunk's Gram to a running FP64 sum, and its H^T T partial to a
 * per-chunk list summed in chunk order; the rank step, factor and beta_0 are
 * those of elm_train on that Gram; every refinement residual is one more
 * pass that forms each chunk's FP64 hidden rows again.  Same precision policy,
 * stopping rules and report as elm_train (its training-set outputs are not
 * produced); the Gram's K splits follow the chunks, so beta agrees with
 * elm_train's to rounding, not bit for bit.  All of X (N x d), W, b, T (N x m)
 * and beta (L x m) are FP64 device arrays as for elm_train; N >= L;
 * 1 <= chunk_rows (clamped to N); 1 <= m <= 64.
 * Errors: as elm_train. */
elm_status elm_train_streamed(elm_handle* h, int64_t N, int64_t d, int64_t L, int64_t m,
                              const double* X, int64_t ldx, const double* W, int64_t ldw,
                              const double* b, const double* T, int64_t ldt,
                              elm_dtype gram_dt, int64_t chunk_rows,
                              double tau_rel, double ir_tol, int32_t ir_max_iter,
                              double* beta, int64_t ldbeta, elm_train_info* info);

/* One independent training of a batch (all pointers device pointers, FP64,
 * with the shapes and leading dimensions of elm_train). */
typedef struct {
    int64_t N, d, L, m;
    const double* X; int64_t ldx;
    const double* W; int64_t ldw;
    const double* b;
    const double* T; int64_t ldt;
    double* H64; int64_t ldh64;   /* caller buffer N x L, receives H */
    double* beta; int64_t ldbeta; /* caller buffer L x m, receives beta */
} elm_problem;

/* elm_train on each of `count` independent problems (e.g. a sweep over
 * hidden-layer sizes or seeds), with one precision form and tolerances for
 * all, and the same results as elm_train gives each problem alone, bit for
 * bit, except that a problem elm_train would certify full rank (see
 * elm_factor_info) takes the greedy rank rule here: its rank is the same and
 * its beta agrees to rounding (the grouped greedy steps serve every order of
 * the group at once; certified factorisations one by one would not).  Each step
 * is one launch for all problems (each block runs the single-problem kernel's
 * arithmetic for its problem), on a batch stream owned by the handle, in
 * three phases: (1) the hidden layer, Z = H^T T and the Gram of every problem
 * with N >= L and m <= 8 (the others on worker streams owned by the handle,
 * created on first use); (2) the pivoted Cholesky rank decisions, one launch
 * per pivot step for the whole group (problems of order <= 512 take one
 * workgroup each), the chain captured once as a HIP graph and replayed by later
 * calls with the same group shape; (3) the factors' dense tails, then beta and
 * the refinement of every problem with N >= L, m <= 8 and rank >= 1, with one
 * host read-back per refinement iteration for all of them (the others on the
 * worker streams).  A
 * problem whose low-precision guard fails is trained again alone from the
 * next precision (as elm_train does).  Problems are grouped so that the
 * Grams, factorisation scratch and phase-1 buffers of a group (about 32 n^2
 * bytes per problem, n = min(N, L), plus its low-precision copy of H) stay
 * within 16 GiB.  The work starts after what is already
 * queued on the handle's stream, and that stream continues only after all of
 * it; the call returns when every training has finished.  infos and statuses
 * (host arrays of `count`, may be NULL) receive each training's report and
 * status; the return value is ELM_OK or the status of the first failed
 * problem (by index), whose message elm_last_error gives.
 * Errors: INVALID_ARG / SHAPE for a malformed problem or argument (nothing
 * runs); those of elm_train per problem. */
elm_status elm_train_batched(elm_handle* h, int32_t count, const elm_problem* probs,
                             elm_dtype gram_dt, double tau_rel, double ir_tol,
                             int32_t ir_max_iter, elm_train_info* infos,
                             elm_status* statuses);

/* Autotuner of a batch's shared tile schedule: runs elm_train_batched on the
 * caller's problems (results are overwritten) with each candidate of a grid
 * -- the greedy pivot panel width (32, 64, 128) times a scale of every
 * grouped problem's Gram split or chunk count (1/2, 1, 2 times what the
 * table or the default rule gives) -- after one untimed call, and keeps the
 * fastest pair if it beats the current choice by at least 2%: the panel row
 * and one split/chunk row per (dtype, order, length) bucket of the batch's
 * Grams go to the handle's table, so later batches and single trainings of
 * those shapes take them.  ms_before / ms_after (host, may be NULL): the
 * batch's time with the table as it was, and with the choice kept.
 * Synchronises.  Errors: those of elm_train_batched. */
elm_status elm_autotune_batch(elm_handle* h, int32_t count, const elm_problem* probs,
                              elm_dtype gram_dt, double tau_rel, double ir_tol, int32_t ir_max_iter,
                              double* ms_before, double* ms_after);

/* How the last elm_train_batched call on a handle ran (host struct, filled by
 * elm_batch_get_report; no synchronisation). */
typedef struct {
    int32_t groups;              /* groups of problems (each within the device budget) */
    int32_t grouped_problems;    /* problems solved in the shared launches */
    int32_t worker_problems;     /* problems run alone on the worker streams (N < L, m > 8,
                                    rank 0, a rank decision within the Gram's noise) */
    int32_t escalations;         /* problems trained again from a higher-precision Gram */
    int32_t batch_stream_syncs;  /* host synchronisations with the batch stream: per group one
                                    read-back of the Grams' largest diagonals (thresholds), one
                                    of the ranks (they size the factors), one of the factors'
                                    definiteness flags and one of the refinement's final state;
                                    plus one per Gram tile table uploaded (first use of a shape) */
    int32_t graph_captures;      /* HIP graphs captured by the call (pivot steps, refinement) */
    int32_t graph_launches;      /* HIP graph launches by the call */
} elm_batch_report;

elm_status elm_batch_get_report(const elm_handle* h, elm_batch_report* out);

/* ------------------------------------------------------------------------ */
/* Step 3 of the three-step ELM: prediction Y = H beta, label = argmax.      */
/* ------------------------------------------------------------------------ */

/* Y = sigma(X W + b) beta without storing H.  X, W, b as for elm_hidden
 * (dtype dt, F64 or F32); beta: L x m FP64, ld ldbeta >= m (converted to dt).
 * Y (optional): N x m of dtype dt, ld ldy >= m.  labels (optional): N int32,
 * index of the largest output of each row (lowest index on ties).  At least
 * one of Y and labels must be non-NULL.  1 <= m <= 64. */
elm_status elm_predict(elm_handle* h, int64_t N, int64_t d, int64_t L, int64_t m,
                       const void* X, int64_t ldx, const void* W, int64_t ldw,
                       const void* b, elm_dtype dt,
                       const double* beta, int64_t ldbeta,
                       void* Y, int64_t ldy, int32_t* labels);

/* Step 3 of the three-step ELM as stated in Section 2.1: multiply the
 * hidden-layer matrix by beta.  H: FP64 sample-major N x L (ld ldh >= L),
 * e.g. the training H from elm_hidden; beta: L x m FP64.  Y (optional): N x m
 * FP64, ld ldy >= m.  labels (optional): N int32 arg-max per row (lowest index
 * on ties).  At least one of Y and labels must be non-NULL.  1 <= m <= 64. */
elm_status elm_predict_hidden(elm_handle* h, int64_t N, int64_t L, int64_t m,
                              const double* H, int64_t ldh,
                              const double* beta, int64_t ldbeta,
                              double* Y, int64_t ldy, int32_t* labels);

/* ------------------------------------------------------------------------ */
/* Stage timers (not part of the method; for measurement).                   */
/* ------------------------------------------------------------------------ */

typedef enum {
    ELM_STAGE_HIDDEN = 0,       /* elm_hidden kernel */
    ELM_STAGE_GRAM = 1,         /* Gram kernel (split-K partial tiles) */
    ELM_STAGE_GRAM_REDUCE = 2,  /* fixed-order FP64 sum of the Gram partials */
    ELM_STAGE_RANK = 3,         /* pivoted Cholesky (all its launches) */
    ELM_STAGE_FACTOR = 4,       /* triangular inverses, K, Cholesky of G G^T */
    ELM_STAGE_SOLVE = 5,        /* applications of H^+ through the factor */
    ELM_STAGE_RHS = 6,          /* H^T T and H^T (T - H beta) passes over H */
    ELM_STAGE_RESIDUAL = 7,     /* T - H beta passes over H */
    ELM_STAGE_PREDICT = 8,      /* elm_predict kernel */
    ELM_STAGE_COUNT = 9
} elm_stage;

typedef struct {
    double ms[ELM_STAGE_COUNT];    /* summed device time between HIP events recorded on the
                                      handle's stream around each stage */
    int64_t count[ELM_STAGE_COUNT]; /* number of timed intervals per stage */
} elm_stage_times;

/* Tuning options of a handle (they change speed, never results beyond
 * rounding).
 *   ELM_OPT_FULL_RANK_MIN_ORDER  Grams of at least this order try the
 *       certified full-rank path before the greedy steps (see
 *       elm_factor_info); <= 0 disables it.  Default 64.
 *   ELM_OPT_BATCH_WORKERS  worker streams of elm_train_batched, 1..16.
 *       Default 8.
 * Errors: INVALID_ARG for an unknown option or a value out of range. */
typedef enum { ELM_OPT_FULL_RANK_MIN_ORDER = 1, ELM_OPT_BATCH_WORKERS = 2 } elm_option;
elm_status elm_set_option(elm_handle* h, elm_option opt, int64_t value);
elm_status elm_get_option(const elm_handle* h, elm_option opt, int64_t* value);

/* enable != 0 starts recording HIP events around every stage on the handle's
 * stream and clears the accumulated times; enable == 0 stops recording.
 * elm_train_batched adds its workers' stage times (concurrent streams, so
 * the sums can exceed the wall time). */
elm_status elm_profile_enable(elm_handle* h, int enable);

/* Accumulated stage times since the last elm_profile_enable(h, 1)
 * (host struct out).  Synchronises the handle's stream. */
elm_status elm_profile_read(elm_handle* h, elm_stage_times* out);

/* ------------------------------------------------------------------------ */
/* Probes of the device's ceilings (not part of the method; for measurement). */
/* ------------------------------------------------------------------------ */

/* Sustained MFMA rate: 2 waves per SIMD on every CU issue independent
 * MFMAs from registers, 8 accumulator chains each: with shape 0, 32x32x16
 * BF16 (dt = ELM_BF16) or 16x16x4 FP64 (ELM_F64); with shape 1 (FP64 only),
 * the four-block 4x4x4 FP64 instruction.  random_operands != 0 fills the
 * operands with random values (the data-dependent power draw lowers the
 * clock), else 1.0.  tflops (host) receives the rate, ms (host, may be NULL)
 * the launch time.  Synchronises.  Errors: UNSUPPORTED dtype or shape. */
elm_status elm_probe_mfma(elm_handle* h, elm_dtype dt, int32_t shape, int32_t random_operands, double* tflops,
                          double* ms);
/* Streaming read of `bytes` of the caller's device buffer (16-byte
 * non-temporal loads, grid-stride): gbs (host) receives GB/s.  buf 16-byte
 * aligned, bytes >= 1 MiB.  Synchronises. */
elm_status elm_probe_stream(elm_handle* h, const void* buf, int64_t bytes, double* gbs, double* ms);
/* Direct global->LDS loads as the 16-bit Gram stages its operands: 1024
 * workgroups of 4 waves each stream 32 KB stages (16-byte loads, one stage
 * in flight) into four LDS buffers, over consecutive parts of the caller's
 * buffer (resident = 0) or re-reading each workgroup's first stage
 * (resident != 0: L2 hits).  gbs (host) receives the aggregate GB/s.  buf
 * 16-byte aligned, bytes >= 128 MiB.  Synchronises. */
elm_status elm_probe_dma(elm_handle* h, const void* buf, int64_t bytes, int32_t resident, double* gbs,
                         double* ms);

#ifdef __cplusplus
}
#endif

#endif /* ELM_H */
