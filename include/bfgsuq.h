/*
 * bfgsuq — BFGS inverse Hessian, randomized SVD and posterior variance on MI355X.
 *
 * C ABI of libbfgsuq.so.  It follows the problem statement of "Preconditioned
 * BFGS-based Uncertainty Quantification in Elastic Full Waveform Inversion"
 * (Liu, Beller, Lei, Peter & Tromp, 2020), section "Preconditioned BFGS-based
 * Uncertainty Quantification": after an optimizer has stored its pairs
 * s_i = m_{i+1} - m_i, y_i = g_{i+1} - g_i and a diagonal initial inverse
 * Hessian B_0, the inverse Hessian B_k of eq. (3) is applied to blocks of
 * vectors, the difference B_k - B_0 is factored by the single-pass randomized
 * SVD of Alg. 3, and the posterior variance diag(V Lambda V^T + B_0) of
 * eqs. (10) and (14) is returned.
 *
 * Conventions for every call
 *   - Pointers marked (device) are HIP device pointers; (host) are host memory.
 *   - Blocks of vectors are column-major n x ncols with leading dimension n:
 *     element (row r, column j) is at offset j * n + r.
 *   - Work is enqueued on the handle's HIP stream; calls return once it is
 *     enqueued unless stated otherwise.  The caller keeps every buffer it
 *     passes alive and unmodified until the stream has reached the call.
 *   - A handle is not thread-safe; distinct handles are independent.
 *   - Return value: BFGS_OK (0) or a negative BFGS_ERR_* code.  Argument
 *     errors are detected before anything is enqueued.  No C++ exception
 *     crosses this boundary.
 *   - Storage type: pairs, h0 and probe blocks are stored in the handle's
 *     storage type (float64, float32 or bfloat16).  Results (apply output,
 *     U, posterior diagonal) are float64 for float64 storage and float32
 *     otherwise.  The k x k and c x c steps always run in float64.
 */
#ifndef BFGSUQ_H
#define BFGSUQ_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct bfgsuq_ctx* bfgs_t;

typedef enum { BFGS_F64 = 0, BFGS_F32 = 1, BFGS_BF16 = 2 } bfgs_dtype;

enum {
    BFGS_OK = 0,
    BFGS_ERR_ARG = -1,        /* bad argument: NULL pointer, size out of range, bad dtype      */
    BFGS_ERR_FULL = -2,       /* push after k_max pairs                                        */
    BFGS_ERR_STATE = -3,      /* call out of order, e.g. posterior_diag before any rsvd        */
    BFGS_ERR_CURVATURE = -4,  /* stored pair has s^T y <= 0: the update of eq. (3) is undefined */
    BFGS_ERR_NONFINITE = -5,  /* NaN or Inf met in inputs or intermediate results              */
    BFGS_ERR_NUMERIC = -6,    /* numerical breakdown: singular Q^T X, eigensolver did not converge */
    BFGS_ERR_ALLOC = -7,      /* device allocation failed                                       */
    BFGS_ERR_HIP = -8         /* other HIP runtime failure                                       */
};

/* Largest probe block (rank + oversampling, and ncols of one apply call). */
#define BFGS_MAX_COLS 256
/* Largest number of stored pairs per handle. */
#define BFGS_MAX_PAIRS 1024

/* bfgs_create — a handle for models of size n holding up to k_max pairs.
 *   n        model size, n >= 1
 *   k_max    capacity in pairs, 1 <= k_max <= BFGS_MAX_PAIRS
 *   H0       (device) n entries of the diagonal initial inverse Hessian B_0
 *            (eq. (4): the inverse of the damped diagonal Hessian guess),
 *            double for BFGS_F64 storage, float otherwise; every entry finite
 *            and > 0 (not checked on the device; a zero or negative entry
 *            gives a matrix that is not positive definite).  Copied.
 *            NULL selects B_0 = gamma I with gamma = s_0^T y_0 / y_0^T y_0
 *            from the first accepted pair (the scaling of Alg. 1), then kept
 *            fixed for the whole history as full-memory BFGS keeps B_0.
 *   storage  type in which pairs, h0 and probes are stored
 *   stream   hipStream_t to enqueue on (NULL = the null stream)
 *   out      (host) receives the handle
 * Allocates about 2 * n * k_max * sizeof(storage) bytes for S and Y (three
 * times that for the bfloat16 form, which also keeps two copies laid out as
 * the matrix-core fragments of the two apply passes read them) plus
 * O(k_max^2) float64 and small workspaces.  Probe, TSQR and basis workspaces
 * (about n * (rank + oversample) * 20 bytes) are allocated on the first
 * rSVD and kept.  Synchronous.                                                */
int bfgs_create(int64_t n, int32_t k_max, const void* H0, bfgs_dtype storage, void* stream,
                bfgs_t* out);

/* bfgs_create_streamed — a handle whose pairs stay in host memory, for histories
 * larger than device memory (the paper keeps its pairs in memory-mapped files
 * on disk and reads them back for every product, section on the 2D elastic
 * Marmousi benchmark).
 *   n, k_max, H0, stream, out   as for bfgs_create
 *   storage      BFGS_F64 or BFGS_F32 (BFGS_ERR_ARG for BFGS_BF16, whose
 *                matrix-core layouts are built in device memory)
 *   slice_rows   rows of S and Y staged to the device at a time, >= 1
 *                (values above n are taken as n)
 * S and Y (2 * n * k_max * sizeof(storage) bytes) live in pinned host memory.
 * The device holds two staging slices of S and Y (4 * slice_rows * k_max *
 * sizeof(storage) bytes), the pair being pushed (2 n) and the same workspaces
 * as a device-resident handle.  Every pass over the pairs (the Gram update of
 * bfgs_push_pair, both passes of bfgs_apply_Hinv / bfgs_apply_Hdiff, the range
 * sample of bfgs_rsvd) copies the slices host -> device on a second stream,
 * the copy of slice i + 1 overlapping the kernels on slice i, so one apply moves
 * 2 * 2 * n * k * sizeof(storage) bytes over the host link.  Results equal
 * those of a device-resident handle up to the order of the float64 partial sums
 * of the first pass (one partial per slice part).  bfgs_apply_Hinv_noalloc
 * returns BFGS_ERR_STATE for such a handle.  Every other call is as for
 * bfgs_create's handles.  Synchronous.                                         */
int bfgs_create_streamed(int64_t n, int32_t k_max, const void* H0, bfgs_dtype storage, int64_t slice_rows,
                         void* stream, bfgs_t* out);

/* bfgs_destroy — frees the handle and all its device memory.  Synchronizes
 * the handle's stream first.  NULL is accepted and ignored.                  */
int bfgs_destroy(bfgs_t h);

/* bfgs_push_pair — appends the pair (s, y) (definitions after eq. (2)).
 *   s, y      (device) n entries each, float64 or float32 per in_dtype
 *   in_dtype  BFGS_F64 or BFGS_F32; the values are rounded to nearest-even
 *             into the storage type
 * The curvature s^T y, r = 1 / (y^T s) of Alg. 1 and the k x k matrices of
 * the compact form are computed from the *stored* (rounded) values.
 * Synchronizes the stream once and then returns BFGS_ERR_CURVATURE if the
 * stored s^T y <= 0, or BFGS_ERR_NONFINITE if it is not finite; the pair is
 * then dropped and the handle stays usable.  BFGS_ERR_FULL after k_max pairs.
 * s and y may be reused once the call has returned.                           */
int bfgs_push_pair(bfgs_t h, const void* s, const void* y, bfgs_dtype in_dtype);

/* bfgs_pop_oldest — forgets the oldest stored pair (s_0, y_0), the step of the
 * limited-memory form (L-BFGS) that the paper compares with full-memory BFGS (the
 * 2-D Marmousi section): the remaining pairs keep their order and B_0 stays as it is
 * (gamma, if it came from the first pair, stays frozen).  The compact form's k x k
 * matrices lose their first row and column; R's inverse is the trailing block of the
 * old one.  Enqueued on the handle's stream; any rSVD result is invalidated.
 * BFGS_ERR_STATE with no pair or for a streamed handle; BFGS_ERR_ARG for bfloat16
 * storage (its matrix-core copies group the pairs by 16).                        */
int bfgs_pop_oldest(bfgs_t h);

/* bfgs_num_pairs — number of accepted pairs k (host). */
int bfgs_num_pairs(bfgs_t h, int32_t* k_out);

/* bfgs_apply_Hinv — out = B_k V, the inverse BFGS matrix of eq. (3) after the k
 * stored pairs (the product Alg. 2 computes one column at a time), for
 * 1 <= ncols <= BFGS_MAX_COLS columns at once.
 *   V    (device) n x ncols, storage type
 *   out  (device) n x ncols, float64 (F64 storage) or float32; must not alias V
 * With k = 0 the result is B_0 V.  Never synchronizes; non-finite results set
 * the deferred status (bfgs_get_status).                                      */
int bfgs_apply_Hinv(bfgs_t h, const void* V, int32_t ncols, void* out);

/* bfgs_apply_Hdiff — out = (B_k - B_0) V: Alg. 2 including its final
 * subtraction of B_0 e_j, the operator that Alg. 3 samples.  Same arguments
 * and behaviour as bfgs_apply_Hinv.                                           */
int bfgs_apply_Hdiff(bfgs_t h, const void* V, int32_t ncols, void* out);

/* bfgs_generate_probes — X, the block of independent random probe vectors of
 * Alg. 3: entry (r, j) is N(0,1) from Philox4x64-10 (key (seed, 0), counter
 * (r / 4, j, 0, 0)) and the Box-Muller transform in float64, rounded to float32
 * and then (bfloat16 storage) to bfloat16, both to nearest-even.
 *   X  (device) n x ncols in the storage type, 1 <= ncols <= BFGS_MAX_COLS   */
int bfgs_generate_probes(bfgs_t h, uint64_t seed, int32_t ncols, void* X);

/* bfgs_rsvd — single-pass randomized SVD of B_k - B_0 (Alg. 3) with
 * c = rank + oversample probe columns drawn as in bfgs_generate_probes:
 *   E = (B_k - B_0) X;  Q R = E (Householder, tall-skinny);  Omega (Q^T X) = Q^T E
 *   (LU with partial pivoting, then symmetrised);  Omega = U_s Lambda U_s^T
 *   (symmetric eigendecomposition, signed eigenvalues ordered by |lambda|
 *   descending, ties by signed value descending then index; each eigenvector's
 *   largest-magnitude entry made positive, lowest index on ties);
 *   U = Q U_s[:, :rank], Sigma = lambda[:rank].
 *   rank        1 <= rank, rank + oversample <= min(n, BFGS_MAX_COLS), oversample >= 0
 *   U           (device) n x rank, float64 (F64 storage) or float32
 *   Sigma       (device) rank doubles (signed eigenvalues of eq. (10)'s Lambda)
 * Also caches the posterior diagonal for bfgs_posterior_diag.  With k = 0,
 * B_k - B_0 = 0: Sigma = 0 and U = 0.  Never synchronizes; a singular Q^T X
 * or an eigensolver failure sets BFGS_ERR_NUMERIC in the deferred status.     */
int bfgs_rsvd(bfgs_t h, int32_t rank, int32_t oversample, uint64_t seed, void* U, double* Sigma);

/* bfgs_rsvd_ex — bfgs_rsvd with variants (flags, OR-ed):
 *   BFGS_RSVD_PRECOND   factor the whitened difference B_0^-1/2 (B_k - B_0) B_0^-1/2,
 *                       whose eigenvalues are those of B_k B_0^-1 - I: the operator the
 *                       paper says "starts from the identity" once B_0 preconditions
 *                       (section "Preconditioned BFGS-based Uncertainty Quantification").
 *                       The probes X are drawn as usual; the whitened sketch is of
 *                       X_w = B_0^1/2 X.  U is then the whitened basis:
 *                       B_k = B_0 + B_0^1/2 U diag(Sigma) U^T B_0^1/2, and the cached
 *                       posterior diagonal is h0 + h0 sum_i Sigma_i U_i^2.
 *   BFGS_RSVD_TWO_PASS  after Q, apply the operator to Q itself and take
 *                       Omega = Q^T (A Q), symmetrised, instead of solving with Q^T X
 *                       (Halko et al.'s two-pass form; one more apply with c columns,
 *                       on the float64 matrix cores whatever the storage).
 * Arguments, results and errors otherwise as bfgs_rsvd; flags = 0 is bfgs_rsvd.  */
#define BFGS_RSVD_PRECOND 1u
#define BFGS_RSVD_TWO_PASS 2u
int bfgs_rsvd_ex(bfgs_t h, int32_t rank, int32_t oversample, uint64_t seed, uint32_t flags, void* U, double* Sigma);

/* bfgs_posterior_diag — out_j = h0_j + sum_i Sigma_i U_ji^2, the diagonal of
 * V Lambda V^T + B_0 (eq. (10)), i.e. the posterior variance of eq. (14) with
 * prior C_m = I, from the last bfgs_rsvd on this handle.
 *   out (device) n entries, float64 (F64 storage) or float32.
 * BFGS_ERR_STATE if no rsvd has run since the last push.                      */
int bfgs_posterior_diag(bfgs_t h, void* out);

/* bfgs_apply_Hinv_noalloc — bfgs_apply_Hinv for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc).  Same arguments, result and errors as bfgs_apply_Hinv,
 * to within the rounding of a different split-K summation; it never calls
 * hipMalloc or hipFree.  Its scratch is a fixed device array of the library
 * (about 90 MiB per GPU, held until the process ends) instead of the handle's
 * workspaces: the split-K depth of the first pass is capped to fit in it, and
 * every size the handle allows (k_max <= BFGS_MAX_PAIRS, ncols <= BFGS_MAX_COLS)
 * fits.  Call it with the handle's device current.  All calls on one GPU share
 * that array, so calls that may overlap on one GPU (other streams, or handles
 * whose streams are not ordered) race; serialise them.                         */
int bfgs_apply_Hinv_noalloc(bfgs_t h, const void* V, int32_t ncols, void* out);

/* bfgs_get_pair — copies stored pair j (0 <= j < k), upcast exactly to
 * float64 (F64 storage) or float32, into s_out / y_out (device, n entries
 * each; either may be NULL).  For checking what the library stored.           */
int bfgs_get_pair(bfgs_t h, int32_t j, void* s_out, void* y_out);

/* bfgs_get_h0 — copies the diagonal B_0 in effect (gamma filled in after the
 * first pair when created with H0 = NULL), float64 or float32, into out
 * (device, n entries).  BFGS_ERR_STATE if gamma is not known yet.            */
int bfgs_get_h0(bfgs_t h, void* out);

/* bfgs_get_status — synchronizes the stream, returns the first deferred error
 * recorded on the device since the last call (or BFGS_OK) and clears it.     */
int bfgs_get_status(bfgs_t h);

/* ---------------------------------------------------------------------------
 * Launch-shape tuning.
 * bfgs_autotune — times the tunable launch shapes for this handle and ncols
 *   probe columns (row slots of the bfloat16 MFMA apply's pass 1, its split-K
 *   depth; number of TSQR chains when rank/U/Sigma are given) with HIP events on the handle's
 *   stream and keeps the fastest in the handle.  V (device, n x ncols, storage
 *   type) and out (device, n x ncols) are scratch inputs/outputs it may
 *   overwrite; U (n x rank) and Sigma (rank) likewise, or NULL to tune the
 *   apply only.  Synchronous; results are unchanged by tuning except for the
 *   summation order of the split-K reduction and of the TSQR tree.
 * bfgs_tuning — reads the current choices (host pointers, either may be NULL).
 * bfgs_set_tuning — sets them: g1_rows in 8 .. 1024 row slots, qr_chains a power
 *   of two in 1 .. 256 (the TSQR uses at most that many chains, fewer when E has
 *   fewer than two 64-row tiles per chain); a value <= 0 keeps the current
 *   choice.  BFGS_ERR_ARG for anything else.  Like bfgs_autotune it changes the
 *   handle's generation, so a captured batch graph refuses to replay.
 * ------------------------------------------------------------------------- */
int bfgs_autotune(bfgs_t h, int32_t ncols, int32_t rank, int32_t oversample, void* V, void* out, void* U,
                  double* Sigma);
int bfgs_tuning(bfgs_t h, int32_t* g1_rows, int32_t* qr_chains);
int bfgs_set_tuning(bfgs_t h, int32_t g1_rows, int32_t qr_chains);

/* ---------------------------------------------------------------------------
 * Batched form: nprob independent inversions of uneven n and k driven as one
 * unit.  Every array argument below is a HOST array of nprob entries (device
 * pointers where the single-problem call takes device pointers).  Problem i
 * has its own handle (bfgs_batch_handle) whose kernels run on one of up to 8
 * side streams forked from `stream` and joined back into it, so the problems
 * overlap on the device.  Semantics per problem are those of the
 * single-problem calls; the rSVD of problem i uses seed + i.
 * ------------------------------------------------------------------------- */
typedef struct bfgsuq_batch* bfgs_batch_t;

/* H0 may be NULL (every problem gamma I) or an array whose NULL entries select gamma I. */
int bfgs_batch_create(int32_t nprob, const int64_t* n, const int32_t* k_max, const void* const* H0, bfgs_dtype storage,
                      void* stream, bfgs_batch_t* out);
/* The handle of problem i (for bfgs_push_pair and inspection; owned by the batch). */
int bfgs_batch_handle(bfgs_batch_t b, int32_t i, bfgs_t* h_out);
/* bfgs_batch_push_pairs — appends kcount[i] pairs to problem i (definitions after
 * eq. (2)): S[i], Y[i] (device) are n_i x kcount[i] column-major blocks (column j
 * = pair j, leading dimension n_i) of in_dtype (BFGS_F64 or BFGS_F32), pushed in
 * column order exactly as bfgs_push_pair would push them.  The problems' pushes
 * run on their own streams and overlap.  A pair that fails the curvature or
 * finiteness check is dropped and the following pairs are still pushed; the
 * return value is the first error met (bfgs_num_pairs tells how many pairs each
 * problem holds).  BFGS_ERR_FULL (nothing pushed) if some problem would exceed
 * its k_max.  Synchronous.                                                      */
int bfgs_batch_push_pairs(bfgs_batch_t b, const void* const* S, const void* const* Y, const int32_t* kcount,
                          bfgs_dtype in_dtype);
int bfgs_batch_apply_Hinv(bfgs_batch_t b, const void* const* V, const int32_t* ncols, void* const* out);
int bfgs_batch_rsvd(bfgs_batch_t b, const int32_t* rank, int32_t oversample, uint64_t seed, void* const* U,
                    double* const* Sigma);
/* bfgs_autotune for every problem (rank/U/Sigma may be NULL). */
int bfgs_batch_autotune(bfgs_batch_t b, const void* const* V, const int32_t* ncols, void* const* out,
                        const int32_t* rank, int32_t oversample, void* const* U, double* const* Sigma);
/* Runs apply + rSVD of every problem once, then captures the same sequence into a
 * hipGraph on `stream` (synchronous).  The buffers passed are baked into the graph,
 * and so are the problems' pair counts, launch shapes and workspaces. */
int bfgs_batch_graph_build(bfgs_batch_t b, const void* const* V, const int32_t* ncols, void* const* out,
                           const int32_t* rank, int32_t oversample, uint64_t seed, void* const* U,
                           double* const* Sigma);
/* Replays the captured graph on `stream`.  BFGS_ERR_STATE if none was built, or
 * if any problem's handle changed since the capture (a pair pushed, a retune, a
 * workspace grown by a call with more columns): the graph is then discarded,
 * nothing is launched, and bfgs_batch_graph_build must be called again.        */
int bfgs_batch_graph_launch(bfgs_batch_t b);
int bfgs_batch_destroy(bfgs_batch_t b);

/* ---------------------------------------------------------------------------
 * GPU-resident full-history BFGS on a quadratic (Alg. 1 with every pair kept and
 * B_0 fixed, search direction p = -B_k g of eq. (1)), for producing histories on the
 * device and for measuring what a B_0 buys in iterations.
 * The misfit is 1/2 m^T A m - b^T m, with A the synthetic stand-in for the
 * wave-equation Hessian on a field-major grid (n = nparam nz nx):
 *   A = diag(D) + P (x) (G_z (x) G_x),  P = I + coupling (1 1^T - I),
 * G_x, G_z the truncated Gaussian smoothers (weights exp(-t^2/(2 sigma^2)), |t| <= half,
 * normalised to sum 1, zero outside the grid).
 * bfgs_gridop_create — D (device, n doubles, copied); sigma > 0; 0 <= half <= 4096.
 *   Synchronous.
 * bfgs_gridop_apply — y = A x for ncols columns (device, n x ncols float64 each,
 *   column-major, y must not alias x), enqueued on the operator's stream.
 * bfgs_minimize_quadratic — runs from m = 0 on an empty handle h (float64 or float32
 *   storage; BFGS_ERR_ARG for bfloat16, BFGS_ERR_STATE if h holds pairs), on the
 *   stream shared by h and op (BFGS_ERR_ARG otherwise): each iteration takes
 *   p = -B_k g (p = -g before the first pair when B_0 = gamma I), the exact line
 *   search alpha = -g^T p / p^T A p, s = alpha p, y = A s, m += s, g += y, and pushes
 *   (s, y) into h.  It stops after max_iter iterations, when |g| <= rel_tol |g_0|, or
 *   when h is full.  m (device, n doubles) receives the iterate; gnorm (host, max_iter
 *   + 1 doubles, or NULL) |g_0|, |g_1|, ...; iters (host) the iterations taken.
 *   Dot products are fixed-order reductions: runs are deterministic.  Synchronizes
 *   once per iteration (the pair's curvature check, the gradient norm).
 * bfgs_minimize_quadratic_ex — the same with two options of the paper's comparison of
 *   L-BFGS with full-memory BFGS (the 2-D Marmousi section): memory > 0 keeps only the
 *   last `memory` pairs (1 <= memory <= k_max; the oldest is dropped by
 *   bfgs_pop_oldest before each push once the window is full, B_0 stays as fixed), 0
 *   keeps them all (bfgs_minimize_quadratic); each step is `damping` times the exact
 *   line minimiser (0 < damping <= 1; 1 = the exact line search).  With exact line
 *   searches on a quadratic both forms take the same steps in exact arithmetic.
 *   BFGS_ERR_ARG for a memory or damping out of range, BFGS_ERR_STATE for a
 *   streamed handle with memory > 0.                                             */
typedef struct bfgsuq_gridop* bfgs_gridop_t;
int bfgs_gridop_create(int64_t nx, int64_t nz, int32_t nparam, const double* D, double sigma, int32_t half,
                       double coupling, void* stream, bfgs_gridop_t* out);
int bfgs_gridop_apply(bfgs_gridop_t op, const double* x, int32_t ncols, double* y);
int bfgs_gridop_destroy(bfgs_gridop_t op);
int bfgs_minimize_quadratic(bfgs_t h, bfgs_gridop_t op, const double* b, int32_t max_iter, double rel_tol, double* m,
                            double* gnorm, int32_t* iters);
int bfgs_minimize_quadratic_ex(bfgs_t h, bfgs_gridop_t op, const double* b, int32_t max_iter, double rel_tol,
                               int32_t memory, double damping, double* m, double* gnorm, int32_t* iters);

/* ---------------------------------------------------------------------------
 * Smoothed, damped diagonal B_0 (eq. (4)): B_0 = (H_0 + lambda I)^-1 from a
 * per-point diagonal Hessian estimate H_0 (the role diag(J^T J) plays in the
 * preconditioners P1-P4), smoothed and stabilised as the paper prescribes for all
 * four ("Numerical examples", the preconditioner comparison): the estimate is
 * smoothed like a gradient and the inverse is damped with the median of the
 * smoothed estimate.
 * bfgs_precond_diag — for a field-major model of nparam fields on an nz x nx grid
 *   (n = nparam nz nx, index (p nz + iz) nx + ix):
 *     hs = each field smoothed by a separable Gaussian, weights exp(-t^2/(2 sigma^2))
 *          for |t| <= half, each 1-D pass divided by the weights inside the grid
 *          (float64 sums, rounded to float32);
 *     lambda = damping * median(hs) (mean of the two middle values for even n);
 *     h0 = 1 / (hs + lambda) (float64, rounded to float32).
 *   hdiag  (device) n floats, finite and > 0
 *   sigma  > 0 (cells); half in [0, 512]; damping >= 0
 *   h0_out (device) n floats; hs_out (device, n floats) or NULL; lambda_out (host) or NULL
 *   stream hipStream_t (NULL = the null stream)
 * The result can be handed to bfgs_create as H0.  Allocates and frees a small
 * workspace; synchronous.                                                       */
int bfgs_precond_diag(int64_t nx, int64_t nz, int32_t nparam, const float* hdiag, double sigma, int32_t half,
                      double damping, float* h0_out, float* hs_out, double* lambda_out, void* stream);

/* ---------------------------------------------------------------------------
 * Learned diagonal B_0: a per-(grid point, parameter) network predicting log h0,
 * the learned counterpart of the diagonal preconditioners of eqs. (4)-(8)
 * (gamma I remains the fallback).  Architecture 8 -> 64 -> 64 -> 1 with GELU
 * (x Phi(x), exact erf); float32 master weights, bfloat16 compute copies,
 * float32 accumulation.  BFGS_MLP_NPARAM parameters flattened as
 * W1 (64 x 8, row-major), b1 (64), W2 (64 x 64, row-major), b2 (64), w3 (64), b3.
 * Features (8 per point, row-major n x 8) of point (param p, iz, ix) of a
 * field-major 3-field model: [logD_p, logD_p+1, logD_p+2, |g0|_p, |g0|_p+1,
 * |g0|_p+2, iz / (nz - 1), sigma_scale] (parameter indices mod 3).
 * All pointers are device pointers; work is enqueued on the stream given at
 * creation.  Gradients and losses are deterministic (fixed-order reductions).
 * ------------------------------------------------------------------------- */
#define BFGS_MLP_NPARAM 4801
typedef struct bfgsuq_mlp* bfgs_mlp_t;

int bfgs_mlp_create(void* stream, bfgs_mlp_t* out);
int bfgs_mlp_destroy(bfgs_mlp_t m);
/* Sets the float32 master weights (and their bfloat16 copy); resets Adam's state. */
int bfgs_mlp_set_params(bfgs_mlp_t m, const float* params);
int bfgs_mlp_get_params(bfgs_mlp_t m, float* params);
/* logD, gabs: n = 3 nx nz floats each; X: n x 8 floats. */
int bfgs_mlp_features(int64_t nx, int64_t nz, const float* logD, const float* gabs, float sigma_scale, float* X,
                      void* stream);
/* out[i] = network(X[i]) (exp_out = 0) or h0_i = exp(network(X[i])) (exp_out = 1). */
int bfgs_mlp_forward(bfgs_mlp_t m, const float* X, int64_t N, float* out, int32_t exp_out);
/* Gradient of mean((network(X) - target)^2) w.r.t. the parameters (grad: NPARAM floats,
 * may be NULL) and the loss (1 float, may be NULL); no update. */
int bfgs_mlp_grad(bfgs_mlp_t m, const float* X, const float* target, int64_t N, float* grad, float* loss);
/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8) on that loss; loss may be NULL. */
int bfgs_mlp_train_step(bfgs_mlp_t m, const float* X, const float* target, int64_t N, float lr, float* loss);

/* Measurement support (not an operation of the method).
 * bfgs_profile — enable (1) or disable (0) per-kernel timing: while enabled,
 *   every kernel group the library enqueues on the handle's stream is
 *   bracketed by HIP events.
 * bfgs_profile_report — synchronizes the stream and writes a JSON object
 *   {"kernel group": [launches, total_ms], ...} of everything recorded since
 *   the last report into buf (host, len bytes, NUL-terminated); clears the
 *   record.  BFGS_ERR_ARG if buf is too small.                               */
int bfgs_profile(bfgs_t h, int32_t enable);
int bfgs_profile_report(bfgs_t h, char* buf, int32_t len);

/* bfgs_tsqr_shape — the configuration the tall-skinny QR of a c-column block
 *   takes (host outputs, either may be NULL): slot_f64 = 1 when the per-chain
 *   c x c triangle is kept in float64 in LDS (0: float32), ring = the number of
 *   LDS entries for 16-reflector groups per chain (even: ring / 2 row tiles of a
 *   chain are folded at once, each in two entries of its own).  BFGS_ERR_ARG
 *   unless 1 <= c <= 256.                                                     */
int bfgs_tsqr_shape(int32_t c, int32_t* slot_f64, int32_t* ring);

/* bfgs_sync — waits until all work enqueued on the handle's stream is done. */
int bfgs_sync(bfgs_t h);

/* bfgs_status_string — static description of a return code. */
const char* bfgs_status_string(int code);

#ifdef __cplusplus
}
#endif

#endif /* BFGSUQ_H */
