/*
 * uhm.h -- uniform H-matrix (UH-matrix) matrix-vector products on AMD Instinct MI355X.
 *
 * A UH-matrix (Definition 2.4 of Bruyninckx, Huybrechs, Meerbergen, "Uniform H-matrix
 * compression with applications to boundary integral equations") stores, for a block
 * partition P = P+ u P- of I x J:
 *   - one orthonormal basis U_tau (|tau| x l_tau) per row cluster tau of an admissible block,
 *   - one orthonormal basis V_sigma (|sigma| x l_sigma) per column cluster,
 *   - one coupling matrix S_b (l_tau x l_sigma) per admissible block b = tau x sigma, so that
 *     A|_b = U_tau S_b V_sigma^*,
 *   - the inadmissible blocks A|_b, b in P-, dense.
 * The product w = A v (section 4.4, Algorithm 6) runs in four stages on the GPU:
 *   forward   u_sigma = V_sigma^* v|_sigma for every column cluster,
 *   coupling  u_tau   = sum_{sigma in row(tau)} S_b u_sigma for every row cluster,
 *   backward  w|_tau += U_tau u_tau,
 *   near field w|_tau += A|_b v|_sigma for b in P-.
 * The H-matrix form (Definition 2.3: A|_b = X_b Y_b^* per admissible block, Algorithm 5)
 * is supported as well, as a comparator for the same operator.
 *
 * Conventions shared by every entry point
 *   - Complex numbers are interleaved (re, im); complex128 = two doubles.
 *   - Every stored matrix is column-major at its element offset (offsets count complex
 *     elements, not bytes).
 *   - Square operators only: rows and columns share one cluster tree over n points.
 *   - "Cluster order": clusters own contiguous ranges [off, off+size) of positions
 *     0..n-1; perm[position] is the user index of that position.  The children of a
 *     cluster partition it.  Vectors passed to the library are in user order.
 *   - Errors are returned as negative ints (no exceptions cross the ABI); uhm_strerror
 *     gives text, uhm_last_error the detail of the last failure in the calling thread.
 *   - Host arrays given to an upload are BORROWED for the duration of the call only.
 *   - An uploaded operator is read-only.  Calls on one operator share its workspace, so
 *     they must be ordered on one stream (or otherwise serialized by the caller).
 */
#ifndef UHM_H
#define UHM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  UHM_OK = 0,
  UHM_EINVAL = -1,   /* null pointer, bad size, inconsistent operator, dtype mismatch */
  UHM_ENOMEM = -2,   /* a device or host allocation failed; the call had no side effects */
  UHM_EHIP = -3,     /* a HIP runtime call failed; see uhm_last_error */
  UHM_ENOCONV = -4,  /* an iterative solve stopped at its iteration limit */
  UHM_ENOTSUP = -5   /* valid request that the library does not support */
};

/* Storage precision of the uploaded operator. */
typedef enum {
  UHM_C128 = 0,      /* complex128 storage and arithmetic; vectors complex128 */
  UHM_C64 = 1,       /* complex64 storage, FP32 accumulation; vectors complex64 */
  UHM_BF16PAIR = 2,  /* (re, im) bfloat16 pairs, FP32 accumulation; vectors complex64 */
  UHM_C128_MULTI = 3, /* complex128 storage and arithmetic laid out for many right-hand sides
                         (FP64 MFMA, up to 64 per pass); vectors complex128 */
  UHM_C128_SYM = 4,   /* complex128, symmetric storage (Remark 4.4): for a complex-symmetric
                         A = A^T on one cluster tree.  The image lists one block of each mirrored
                         pair tau x sigma / sigma x tau (diagonal dense blocks once); the mirror
                         of a stored admissible block is U_sigma S_b^T U_tau^T and that of a
                         stored dense block A|_b^T, with V_c = conj(U_c) implied: V, V_off and
                         rank_col are not read.  Each stored element is read once per product
                         and applied both ways.  uhm_upload only; vectors complex128 */
  UHM_C128_FACTORED = 5, /* complex128 with factored couplings (section 4.2):
                         S_b = S_{X,b} S_{Y,b}^*, applied in two steps (S_{Y,b}^* u_sigma, then
                         S_{X,b} times that) for every block where k_b (l_tau + l_sigma) <
                         l_tau l_sigma, assembled S_b elsewhere.  The image must carry adm_rank,
                         SX and SY.  uhm_upload only; vectors complex128 */
  UHM_C64_FACTORED = 6,     /* UHM_C64 with factored couplings where they store fewer elements
                               (the same rule); the image must carry adm_rank, SX and SY */
  UHM_BF16PAIR_FACTORED = 7, /* UHM_BF16PAIR with factored couplings, likewise */
  UHM_C128_MULTI_FACTORED = 8, /* UHM_C128_MULTI with factored couplings, likewise */
  UHM_C64_STREAM = 9,      /* complex64 storage in the layout of UHM_C128 (one lane per panel
                              column or row, the operator streamed once per right-hand side),
                              FP32 arithmetic; vectors complex64.  For one or a few right-hand
                              sides, where the MFMA forms pad to 16 columns.  uhm_upload only */
  UHM_BF16PAIR_STREAM = 10 /* the same with (re, im) bfloat16-pair storage; vectors complex64 */
} uhm_storage;

typedef struct uhm_op uhm_op; /* opaque; owned by the library until uhm_free */

/*
 * Host image of a UH-matrix (Definition 2.4), produced by the host builder.
 * Cluster tree: nclusters clusters with off/size/parent (parent = -1 at the root).
 * Bases: cluster c has a row basis iff rank_row[c] > 0 (c in L'_I of eq.
 * clusters_in_partition), stored at U + 2*U_off[c] as size[c] x rank_row[c]; likewise V.
 * Admissible block b: rows adm_row[b], columns adm_col[b], S_b at S + 2*S_off[b] as
 * rank_row[adm_row[b]] x rank_col[adm_col[b]].
 * Dense block b: den_row[b] x den_col[b] at D + 2*D_off[b] as size x size.
 * *_len are the lengths of the flat arrays in complex elements (used for bounds checks).
 */
typedef struct {
  int64_t n;
  const int64_t* perm;       /* [n] cluster position -> user index, a permutation */
  int32_t nclusters;
  const int64_t* off;        /* [nclusters] */
  const int64_t* size;       /* [nclusters] */
  const int32_t* parent;     /* [nclusters] */
  const int32_t* rank_row;   /* [nclusters] l_tau, 0 if none */
  const int32_t* rank_col;   /* [nclusters] l_sigma, 0 if none */
  const int64_t* U_off;      /* [nclusters] */
  const int64_t* V_off;      /* [nclusters] */
  const double* U; int64_t U_len;
  const double* V; int64_t V_len;
  int64_t nadm;
  const int32_t* adm_row;    /* [nadm] */
  const int32_t* adm_col;    /* [nadm] */
  const int64_t* S_off;      /* [nadm] */
  const double* S; int64_t S_len;
  int64_t nden;
  const int32_t* den_row;    /* [nden] */
  const int32_t* den_col;    /* [nden] */
  const int64_t* D_off;      /* [nden] */
  const double* D; int64_t D_len;
  /* Factored couplings, read only with UHM_C128_FACTORED (NULL otherwise): block b has
   * k_b = adm_rank[b] >= 1, S_{X,b} (rank_row[adm_row[b]] x k_b) at SX + 2*SX_off[b] and
   * S_{Y,b} (rank_col[adm_col[b]] x k_b) at SY + 2*SY_off[b]. */
  const int32_t* adm_rank;   /* [nadm] */
  const int64_t* SX_off;     /* [nadm] */
  const int64_t* SY_off;     /* [nadm] */
  const double* SX; int64_t SX_len;
  const double* SY; int64_t SY_len;
} uhm_host_operator;

/*
 * Host image of the H-matrix of the same partition (Definition 2.3): admissible block b
 * stores X_b (size[adm_row[b]] x adm_rank[b]) at X + 2*X_off[b] and Y_b
 * (size[adm_col[b]] x adm_rank[b]) at Y + 2*Y_off[b], A|_b = X_b Y_b^*.
 */
typedef struct {
  int64_t n;
  const int64_t* perm;
  int32_t nclusters;
  const int64_t* off;
  const int64_t* size;
  const int32_t* parent;
  int64_t nadm;
  const int32_t* adm_row;
  const int32_t* adm_col;
  const int32_t* adm_rank;
  const int64_t* X_off;
  const int64_t* Y_off;
  const double* X; int64_t X_len;
  const double* Y; int64_t Y_len;
  int64_t nden;
  const int32_t* den_row;
  const int32_t* den_col;
  const int64_t* D_off;
  const double* D; int64_t D_len;
} uhm_host_hmatrix;

/* Sizes and algorithmic traffic of an uploaded operator. */
typedef struct {
  int64_t n;
  int32_t kind;              /* 0 = UH-matrix, 1 = H-matrix */
  int32_t storage;           /* uhm_storage */
  int32_t nleaves;
  int32_t elem_bytes;        /* bytes per stored complex element */
  int64_t nadm, nden;
  int64_t elems_forward;     /* sum n_sigma l_sigma (UH) or sum_b n_sigma k_b (H) */
  int64_t elems_coupling;    /* sum_b l_tau l_sigma (UH), 0 (H) */
  int64_t elems_backward;    /* sum n_tau l_tau (UH) or sum_b n_tau k_b (H) */
  int64_t elems_near;        /* sum_b n_tau n_sigma over P- */
  int64_t rank_space;        /* sum l_sigma (UH) or sum k_b (H): length of the rank-space vectors */
  int64_t device_bytes;      /* device memory held by the operator, workspace excluded */
  int64_t partial_coupling;  /* UHM_C128_SYM: partial sums the transposed coupling products write per
                                right-hand side (complex elements); 0 for the other forms */
  int64_t partial_near;      /* UHM_C128_SYM: the same for the transposed dense blocks */
  int64_t elems_coupling_in; /* UHM_C128_FACTORED: elements of the S_{Y,b} factors, read by the
                                first coupling step (elems_coupling counts the assembled S_b
                                and the S_{X,b} factors); 0 for the other forms */
  int64_t scratch_bytes;     /* complex128 single-RHS forms: device scratch of one product (the
                                workspace uhm_matvec grows, the part of uhm_matvec_noalloc's
                                array a call takes); 0 for the many-RHS forms */
} uhm_op_info;

/*
 * Upload a UH-matrix (Definition 2.4) to the current HIP device, re-laid out for the
 * product (per-leaf panels of the bases, row-chunked couplings).  The host arrays are
 * validated (tree, offsets, bounds) and only read during the call; the copies are
 * enqueued on `hip_stream` (a hipStream_t, or NULL for the default stream) and complete
 * before the call returns.  *out receives an operator to free with uhm_free.
 * Errors: UHM_EINVAL (null pointer, inconsistent operator), UHM_ENOMEM, UHM_EHIP.
 */
int uhm_upload(const uhm_host_operator* h, uhm_storage storage, void* hip_stream, uhm_op** out);

/*
 * Upload the H-matrix form (Definition 2.3) of an operator, for the H-matrix product of
 * Algorithm 5 (section 4.4).  Same semantics and errors as uhm_upload.
 */
int uhm_upload_h(const uhm_host_hmatrix* h, uhm_storage storage, void* hip_stream, uhm_op** out);

/*
 * Y = A X  (w = A v of Algorithms 5 and 6, section 4.4; Y is overwritten).
 * X: device pointer, n x nrhs column-major, leading dimension ldx >= n, user order.
 * Y: device pointer, n x nrhs column-major, leading dimension ldy >= n; must not overlap X.
 * Element type: complex128 for UHM_C128 and UHM_C128_MULTI operators, complex64 otherwise.
 * Asynchronous on `hip_stream`.  nrhs == 0 is a no-op.  Errors: UHM_EINVAL (null
 * pointer, nrhs < 0, ld < n), UHM_ENOMEM (workspace growth failed), UHM_EHIP.
 */
int uhm_matvec(uhm_op* op, const void* X, int64_t ldx, void* Y, int64_t ldy, int32_t nrhs,
               void* hip_stream);

/*
 * uhm_matvec for callers that cannot allocate device memory: code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc.  It computes exactly what
 * uhm_matvec computes (the same kernels in the same order, so the results are bitwise
 * equal) but takes its product scratch (the per-leaf and per-tile partial sums and the
 * rank-space vectors) from one file-scope device array of 512 MiB that the library holds on
 * every GPU it runs on until the process ends, instead of the operator's own workspace.  It
 * calls no hipMalloc or hipFree and allocates nothing else.
 *   - Complex128 single-RHS storage forms only (UHM_C128, UHM_C128_SYM, UHM_C128_FACTORED
 *     and H-matrix uploads); the many-RHS forms return UHM_ENOTSUP.
 *   - An operator whose scratch exceeds 512 MiB is rejected with UHM_EINVAL (the
 *     symmetric N = 262144 sphere operator of leaf 64 needs about 0.3 GiB).
 *   - Every call on one GPU shares that GPU's array: calls that overlap on one GPU (on
 *     different streams, or from different threads) race and give wrong results.  Calls
 *     ordered on one stream are safe.  The array keeps the last call's contents; every
 *     entry a product reads is written earlier in the same product, so nothing needs
 *     clearing.
 * Arguments, layout and the other errors as uhm_matvec.
 */
int uhm_matvec_noalloc(uhm_op* op, const void* X, int64_t ldx, void* Y, int64_t ldy, int32_t nrhs,
                       void* hip_stream);

/* Options of uhm_solve_gmres; a NULL pointer selects the defaults in brackets. */
typedef struct {
  int32_t restart;          /* Krylov dimension m of each GMRES(m) cycle [50] */
  int32_t max_iterations;   /* cap on Krylov iterations per solve, all cycles and refinements [2000] */
  int32_t max_refinements;  /* outer refinement steps when an inner operator is given [30] */
  double inner_tol;         /* residual reduction asked of each inner solve of the refinement [1e-4] */
  int32_t inner_cycles;     /* with an inner operator: an inner solve also ends after this many
                               GMRES(m) cycles, so that with 1 every restart of the inner GMRES is
                               a refinement step (the restart residual is the true FP64 one);
                               0 = end an inner solve at inner_tol only [0] */
} uhm_gmres_opts;

/* What uhm_solve_gmres did. */
typedef struct {
  int32_t iterations;       /* Krylov iterations (products with the Krylov operator); a cycle
                               that stops on its tolerance takes one product more than its
                               Krylov dimension, for the delayed second projection */
  int32_t restarts;         /* GMRES(m) cycles started after the first */
  int32_t refinements;      /* outer refinement steps (0 without an inner operator) */
  int32_t converged;        /* right-hand sides whose final true relative residual <= tol */
  double rel_residual;      /* max over right-hand sides of ||b - A x||_2 / ||b||_2, FP64 operator */
  double seconds_total;     /* wall clock of the solve (synchronized) */
  double seconds_products;  /* of which spent in operator products */
  double seconds_arnoldi;   /* of which spent in the orthogonalisation and updates */
  int64_t second_passes;    /* column-steps whose basis vector got its second projection
                               (every step of every running column) */
} uhm_gmres_info;

/*
 * Solve A X = B by restarted GMRES(m) (textbook GMRES with classical Gram-Schmidt applied
 * twice, the second projection of each basis vector delayed by one step and fused with the
 * first projection of the next (the one-reduction DCGS2 scheme of Swirydowicz et al. and
 * Bielich et al.), FP64 Krylov vectors, Givens least-squares),
 * for nrhs right-hand sides at once, each with its own Krylov space.  X starts at zero
 * and is overwritten.
 *   op:    the operator A in a complex128 storage form (the true-residual operator).
 *   inner: NULL for plain GMRES on op; otherwise an operator of the same matrix in
 *          complex64 or bf16-pair storage, and the solve is mixed-precision iterative
 *          refinement: r = B - A X with op (FP64), an inner GMRES(m) solves
 *          A_inner D = r to inner_tol, or for opts->inner_cycles cycles when that is
 *          positive (products with `inner`, everything else FP64), X += D, until
 *          max_j ||r_j|| / ||b_j|| <= tol.
 * B (ldb >= n), X (ldx >= n): complex128 device arrays, n x nrhs column-major, user order.
 * Synchronous on `hip_stream`; allocates its workspace ((m+1) n nrhs complex128 for the
 * Krylov basis plus a few vectors) for the duration of the call.
 * Returns UHM_OK when every right-hand side reaches tol, UHM_ENOCONV when the iteration
 * or refinement cap is reached first (X holds the last iterate, *info is filled),
 * UHM_EINVAL (bad arguments, n mismatch, op not complex128, inner not low precision),
 * UHM_ENOMEM, UHM_EHIP.  Textbook GMRES (Saad and Schultz); the refinement follows
 * Carson and Higham's GMRES-IR.
 */
int uhm_solve_gmres(uhm_op* op, uhm_op* inner, const void* B, int64_t ldb, void* X, int64_t ldx, int32_t nrhs,
                    double tol, const uhm_gmres_opts* opts, uhm_gmres_info* info, void* hip_stream);

/*
 * Batched products.  A batch binds a fixed set of products Y_k = A_k X_k (k < nops) over
 * operators uploaded in one many-RHS storage form (UHM_C64, UHM_BF16PAIR or
 * UHM_C128_MULTI); X_k, Y_k are device arrays (n_k x nrhs_k, column-major, leading
 * dimensions ldx[k], ldy[k] >= n_k, 1 <= nrhs_k <= 64) that stay bound to the batch.
 * uhm_batch_run executes all of them stage by stage: each stage of the product is one
 * kernel launch over the work of every operator (work lists of (operator, leaf / tile)),
 * so many small operators fill the GPU together.  Each operator's reductions keep their
 * own fixed order, so a product's result does not depend on the rest of the batch.
 * The batch owns its workspace; the operators' own workspace is not used, and the
 * operators must outlive the batch.
 *   uhm_batch_tune    times the candidate schedules (coupling tile width 256/512/1024/2048
 *                     columns x work order: operator-major, largest-first, round-robin
 *                     over cost buckets) on the device and keeps the fastest; the choice is
 *                     cached for batches with the same signature (sizes, ranks, nrhs) in
 *                     this process.  Outputs may be NULL.  Synchronous.
 *   uhm_batch_capture captures the launches of one run into a hipGraph on `hip_stream`
 *                     (not the NULL stream); later runs replay the graph.
 *   uhm_batch_run     asynchronous on `hip_stream`; runs that overlap on different streams
 *                     race on the batch's workspace.
 * Errors: UHM_EINVAL (mixed or single-RHS storage, nrhs out of range, bad pointers),
 * UHM_ENOMEM, UHM_EHIP.  This is not a construct of the paper: it batches the products of
 * Algorithm 6 (section 4.4) of many operators.
 */
typedef struct uhm_batch uhm_batch;
int uhm_batch_create(uhm_op* const* ops, int32_t nops, const void* const* X, const int64_t* ldx, void* const* Y,
                     const int64_t* ldy, const int32_t* nrhs, void* hip_stream, uhm_batch** out);
int uhm_batch_run(uhm_batch* b, void* hip_stream);
int uhm_batch_tune(uhm_batch* b, void* hip_stream, int32_t* tile_width, int32_t* order, double* best_ms);
int uhm_batch_capture(uhm_batch* b, void* hip_stream);
void uhm_batch_free(uhm_batch* b);

/*
 * Resumable (reverse-communication) form of uhm_solve_gmres, for callers that batch the
 * products of many solves (a serving loop).  The solve owns its Krylov workspace and stops
 * whenever it needs a product:
 *   uhm_krylov_next    returns UHM_KRYLOV_PRODUCT_HIGH (the caller writes A*in to out with
 *                      the FP64 operator), UHM_KRYLOV_PRODUCT_LOW (the product with the
 *                      low-precision operator; in/out are still complex128, the caller
 *                      converts), or UHM_KRYLOV_DONE.  in/out: n x nrhs complex128 device
 *                      arrays, leading dimension n, owned by the solve.
 *   uhm_krylov_advance after the product is in out: runs the FP64 Arnoldi / refinement work
 *                      on the solve's stream and prepares the next request.  Synchronous.
 *   uhm_krylov_result  after DONE: X (ldx >= n, may be NULL) receives the solution, *info
 *                      (may be NULL) the counts; returns UHM_OK or UHM_ENOCONV.
 * mixed = 0: plain GMRES(m) with FP64 products; mixed = 1: GMRES-IR as uhm_solve_gmres
 * with an inner operator.  B is copied at creation.  Errors as uhm_solve_gmres.
 */
enum { UHM_KRYLOV_DONE = 0, UHM_KRYLOV_PRODUCT_HIGH = 1, UHM_KRYLOV_PRODUCT_LOW = 2 };
typedef struct uhm_krylov uhm_krylov;
int uhm_krylov_create(int64_t n, int32_t nrhs, const void* B, int64_t ldb, double tol, int32_t mixed,
                      const uhm_gmres_opts* opts, void* hip_stream, uhm_krylov** out);
int uhm_krylov_next(uhm_krylov* k, const void** in, void** out);
int uhm_krylov_advance(uhm_krylov* k);
int uhm_krylov_result(uhm_krylov* k, void* X, int64_t ldx, uhm_gmres_info* info);
void uhm_krylov_free(uhm_krylov* k);

/*
 * One step of many solves at once (continuous batching): every solve with a pending
 * request gets its product, grouped by (operator, precision) into multi-column products of
 * up to 64 columns that read and write the solves' vectors in place through column
 * pointers (with complex64 conversion for the low-precision operators), then every solve
 * advances.  The Arnoldi steps of all solves run as one launch per kernel over all of
 * them, followed by one synchronisation of `hip_stream`.  high[k] / low[k] are solve k's
 * FP64 and low-precision operators (low may be NULL when no solve is mixed).  The
 * operators' staging buffers grow as needed.  Products and Arnoldi kernels run on
 * `hip_stream`; solves created on other streams are synchronised first.  Steps from
 * several host threads are serialised on a process-wide lock around the Arnoldi launches.
 * A solve's columns are products of its own Krylov vectors only, and every reduction is
 * per column in a fixed order, so a solve's iterates are the same alone or in any mix.
 * Returns the number of solves still running, or a negative error code.
 */
int uhm_krylov_step(uhm_krylov* const* ks, uhm_op* const* high, uhm_op* const* low, int32_t count, void* hip_stream);

/* Fill *info for an uploaded operator.  Errors: UHM_EINVAL. */
int uhm_op_info_get(const uhm_op* op, uhm_op_info* info);

/*
 * Kernel timing: while enabled, uhm_matvec records HIP events around each of its kernel
 * launches (on the stream of the call) and accumulates per-kernel milliseconds.
 * uhm_kernel_times writes up to `cap` entries (name pointer, total ms, launch count) and
 * returns the number of kernels; names stay valid until uhm_free.  Reading the times
 * synchronizes with the recorded events.  Enabling resets the totals.
 */
int uhm_set_timing(uhm_op* op, int enabled);
int uhm_kernel_times(uhm_op* op, const char** names, double* total_ms, int64_t* launches, int32_t cap);

/* Release every device allocation of the operator.  NULL is a no-op. */
void uhm_free(uhm_op* op);

/* ---------------------------------------------------------------------------------------
 * Construction on the GPU: blocks of the kernel matrix and their adaptive cross
 * approximation (section 2.3).
 *
 * The matrix is the point-kernel matrix of the Helmholtz single-layer kernel (section 6.1):
 * A_ij = exp(i kappa r_ij) / (4 pi r_ij) with r_ij = |p_i - p_j|, and A_ij = diag where
 * i = j or the two points coincide.  `points` is a DEVICE array of npoints x 3 doubles
 * (row-major, x y z), in cluster order; blocks address rows and columns by position in it.
 * Every pointer below is a device pointer except where stated; nothing is allocated, and
 * the calls are asynchronous on `hip_stream`.  Each block descriptor is checked on the
 * device: a descriptor whose sizes, positions or output ranges do not fit the given
 * lengths is not processed and gets status -1.
 */
typedef struct uhm_block_desc {
  int64_t row_off;  /* first row position, 0 <= row_off, row_off + rows <= npoints */
  int64_t col_off;  /* first column position, likewise */
  int32_t rows;     /* m >= 1 */
  int32_t cols;     /* n >= 1 */
  int32_t cap;      /* ACA: most terms kept, 1 <= cap <= max_cap; uhm_kernel_blocks: unused */
  int32_t reserved; /* 0 */
  int64_t a_off;    /* uhm_kernel_blocks: complex offset of the m x n block in D;
                       uhm_aca: complex offset of u (m x cap) in U */
  int64_t b_off;    /* uhm_aca: complex offset of v (n x cap) in V */
  int64_t p_off;    /* uhm_aca: offset in piv of 2*cap int32 pivots (cap rows, then cap columns) */
} uhm_block_desc;

/*
 * D[a_off + i + j*m] = A[row_off + i, col_off + j] (column-major, complex128) for every
 * block; the dense near-field blocks of the operator (P-, Definition 2.2).  status[b] is 1
 * for a block written, -1 for a rejected descriptor.  D_len counts complex elements.
 * Errors: UHM_EINVAL (negative sizes, null pointers with nblocks > 0), UHM_EHIP.
 */
int uhm_kernel_blocks(const double* points, int64_t npoints, double kappa, double diag,
                      const uhm_block_desc* blocks, int64_t nblocks, double* D, int64_t D_len,
                      int32_t* status, void* hip_stream);

/*
 * ACA with partial pivoting (section 2.3; the variant of Bebendorf the paper cites) of each
 * block A|_b = A[row_off : row_off+m, col_off : col_off+n], one workgroup per block (1 to 16
 * wavefronts, chosen per call from max_rows so that a thread holds about 8 rows):
 *   start from row i_1 = 0; at step k take the residual row r = A[i_k, :] - sum_{l<k}
 *   u_l[i_k] v_l, mark row i_k used, pick j_k maximising |r_j| (if r vanishes, retry with
 *   the unused row of smallest index), set v_k = r / r[j_k] and u_k = A[:, j_k] -
 *   sum_{l<k} v_l[j_k] u_l; stop once |u_k| |v_k| <= eps |sum_{l<=k} u_l v_l^T|_F (the
 *   Frobenius norm updated term by term), else continue from the unused row maximising
 *   |u_k[i]|; at most min(m, n, cap) terms.  Moduli are compared as re^2 + im^2 in FP64 and
 *   the first index wins a tie.
 * Outputs, per block: A|_b ~ sum_{l<k} u_l v_l^T with u_l = U[a_off + l*m : ... + m] and
 * v_l = V[b_off + l*n : ... + n] (complex128, column-major, columns k..cap-1 undefined);
 * piv[p_off + l] = i_l and piv[p_off + cap + l] = j_l (block-relative); rank[b] = k;
 * status[b] = 1 when the stopping test ended the iteration, 2 when the block ran out of
 * rows or reached min(m, n) terms, 0 when `cap` (< min(m, n)) stopped it first (call again
 * with a larger cap), -1 for a rejected descriptor.
 * max_rows (1..65536) and max_cap (1..1024) bound every block's rows and cap and size the
 * local memory of the launch.  U_len, V_len count complex elements, piv_len int32 entries.
 * Errors: UHM_EINVAL (bounds above, eps < 0 or not finite, null pointers), UHM_EHIP.
 */
int uhm_aca(const double* points, int64_t npoints, double kappa, double diag,
            const uhm_block_desc* blocks, int64_t nblocks, int32_t max_rows, int32_t max_cap, double eps,
            double* U, int64_t U_len, double* V, int64_t V_len, int32_t* piv, int64_t piv_len,
            int32_t* rank, int32_t* status, void* hip_stream);

/*
 * The factors of blocks sel[0..cnt) of an earlier uhm_aca call, packed for their algebraic
 * recompression (section 2.3): block b = sel[c] (all of them m x n, rank[b] <= kp terms)
 * gives X[c] = [u_0 .. u_{k-1} 0 ..] and Y[c] = [conj(v_0) .. conj(v_{k-1}) 0 ..], each a
 * row-major m x kp (n x kp) complex128 matrix, so that A|_b ~ X[c] Y[c]^*.  blocks, rank, U,
 * V are that call's device arrays (its descriptors, its outputs); sel, X (cnt m kp complex
 * elements), Y (cnt n kp) and status (cnt) are device arrays.  status[c] = 1 for a packed
 * block, -1 for one whose descriptor does not match (m, n), whose rank exceeds kp or its cap,
 * or whose factors lie outside U_len / V_len (written as zeros).  Nothing is allocated;
 * asynchronous on hip_stream.  Errors: UHM_EINVAL (sizes, null pointers), UHM_EHIP.
 */
int uhm_aca_pack(const uhm_block_desc* blocks, int64_t nblocks, const int32_t* rank, const double* U, int64_t U_len,
                 const double* V, int64_t V_len, const int32_t* sel, int32_t cnt, int32_t m, int32_t n, int32_t kp,
                 double* X, double* Y, int32_t* status, void* hip_stream);

/*
 * Alg. 2's per-cluster factorisation (section 4.2) for a batch of `batch` clusters of one
 * shape: for each X_c (m x n complex128, row-major, X + 2*c*m*n; zero columns allowed)
 * it returns the left singular vectors whose singular values exceed eps * sigma_1 (U_tau,
 * rank l = at least 1) and the rows Sigma V^* = U_tau^* X_c, the same rank rule as a full
 * SVD.  The SVD is taken as: Householder QR with column pivoting of X_c, stopped once the
 * trailing part's Frobenius norm T is at most tol * ||X_c||_F (p steps; the singular values
 * of the resulting p x n factor B satisfy sigma_i(B)^2 <= sigma_i(X_c)^2 <= sigma_i(B)^2 +
 * T^2, because the trailing part is orthogonal to the kept range), an unpivoted QR of B^*,
 * one-sided Jacobi on the columns of that triangle's conjugate transpose (whose rotated
 * columns are the left singular vectors, scaled), and the reflectors applied back.  With tol^2 about
 * 1e-16 eps (1e-11 for eps = 1e-6) a singular value at the threshold eps sigma_1 moves by
 * less than a unit of rounding of sigma_1.
 * X (only read: the library factorises a column-major copy in work), U, SV, sv, rank,
 * psteps, stats, status and work are device arrays:
 *   U[c]:  m x pmax complex (column-major, U + 2*c*m*pmax), columns 0..l-1 written;
 *   SV[c]: pmax x n complex (column-major with leading dimension pmax, SV + 2*c*pmax*n),
 *          rows 0..l-1 written: SV = U^* X;
 *   sv[c*pmax + i]: singular values of B, descending (zeros beyond p);
 *   rank[c] = l, psteps[c] = p;
 *   stats[3c..3c+2] = ||X - U U^* X||_F (the dropped sigma_i(B) and T together), the first
 *          dropped singular value (sqrt(sigma_{l+1}(B)^2 + T^2), an upper bound of sigma_{l+1}(X_c)
 *          within T^2 / (2 sigma_{l+1}); 0 if l = min(m, n)), and T;
 *   status[c] = 0, or bit 0: pmax steps ended before the tolerance (the result is that of
 *          the truncated QR; call again with a larger pmax), bit 1: the Jacobi sweeps did not
 *          converge within 60 sweeps.
 * work: uhm_cluster_basis_work(batch, m, n, pmax) doubles of device memory (work_len counts
 * doubles); nothing is allocated.  Limits: m <= 16384, 1 <= pmax <= min(m, n, 2048), batch
 * <= 65535.  Enqueued on hip_stream; the Jacobi stage reads one counter back per sweep, so
 * the call synchronises that stream about ten times and returns with the rest enqueued.
 * Errors: UHM_EINVAL (sizes, tol or eps negative or not finite, null pointers, work too
 * small), UHM_EHIP.
 */
int uhm_cluster_basis(const double* X, int32_t batch, int32_t m, int32_t n, int32_t pmax, double tol, double eps,
                      double* U, double* SV, double* sv, int32_t* rank, int32_t* psteps, double* stats,
                      int32_t* status, double* work, int64_t work_len, void* hip_stream);

/* Workspace of uhm_cluster_basis in doubles, or -1 for sizes it rejects outright. */
int64_t uhm_cluster_basis_work(int32_t batch, int32_t m, int32_t n, int32_t pmax);

/*
 * The algebraic recompression of ACA factors (section 2.3) for a batch of `batch` blocks of
 * one shape: for each block A|_b ~ X_c Y_c^* (X_c m x kp and Y_c n x kp complex128,
 * row-major at X + 2*c*m*kp and Y + 2*c*n*kp; zero columns allowed) it returns the SVD
 * truncated at eps * sigma_1, U_c Sigma_c V_c^* with k = rank[c] >= 1 terms.  Taken as:
 * unpivoted Householder QR of both factors (X = Q_X R_X, Y = Q_Y R_Y), one-sided Jacobi on
 * M = R_Y R_X^* (M J = W Sigma, so X Y^* = (Q_X J) Sigma (Q_Y W)^*), the kept columns of J
 * and W orthonormalised again and carried back through the reflectors.
 * X, Y (only read: the library works on column-major copies in work), U, V, sv, rank,
 * status and work are device arrays:
 *   U[c]: m x kp complex (column-major, U + 2*c*m*kp), columns 0..k-1 written;
 *   V[c]: n x kp complex (V + 2*c*n*kp), columns 0..k-1 written;
 *   sv[c*kp + i]: the singular values of X_c Y_c^*, descending;
 *   status[c] = 0, or 2 when the Jacobi sweeps did not converge within 60 sweeps.
 * work: uhm_block_recompress_work(batch, m, n, kp) doubles of device memory (work_len counts
 * doubles); nothing is allocated.  Limits: m, n <= 16384, 1 <= kp <= min(m, n, 2048), batch
 * <= 65535.  Enqueued on hip_stream, synchronised once per Jacobi sweep as in
 * uhm_cluster_basis.  Errors: UHM_EINVAL (sizes, eps negative or not finite, null pointers,
 * work too small), UHM_EHIP.
 */
int uhm_block_recompress(const double* X, const double* Y, int32_t batch, int32_t m, int32_t n, int32_t kp, double eps,
                         double* U, double* V, double* sv, int32_t* rank, int32_t* status, double* work,
                         int64_t work_len, void* hip_stream);

/* Workspace of uhm_block_recompress in doubles, or -1 for sizes it rejects outright. */
int64_t uhm_block_recompress_work(int32_t batch, int32_t m, int32_t n, int32_t kp);

/* One admissible block b = (tau, sigma) for uhm_couplings; offsets count complex elements
 * (sig_off: doubles). */
typedef struct uhm_coupling_desc {
  int64_t a_off;   /* L_{tau,b}: L[a_off + q*lt + i] = (U_tau^* X_b)[i][q], i < lt, q < kb */
  int64_t b_off;   /* L_{sigma,b}: L[b_off + q*ls + j], the mirrored block's rows */
  int64_t sig_off; /* sigma_b: sigma[sig_off + q], q < kb (all > 0) */
  int64_t s_off;   /* S_b, lt x ls column-major, at S + s_off */
  int64_t x_off;   /* S_{X,b}, lt x kb column-major, at SX + x_off */
  int64_t y_off;   /* S_{Y,b}, ls x kb column-major, at SY + y_off */
  int32_t lt;      /* l_tau >= 1 */
  int32_t ls;      /* l_sigma >= 1 */
  int32_t kb;      /* the block's rank k_b >= 1 */
  int32_t reserved; /* 0 */
} uhm_coupling_desc;

/*
 * The couplings of the construction (section 4.1; factored form, section 4.2) for every
 * block of `blocks`: with L_{tau,b} = U_tau^* U_b Sigma_b (lt x kb, the rows of Alg. 2's
 * Sigma V^* that belong to block b) and L_{sigma,b} the same for the mirrored block,
 *   S_{X,b} = L_{tau,b} Sigma_b^{-1},  S_{Y,b} = conj(L_{sigma,b}),  S_b = S_{X,b} L_{sigma,b}^T,
 * so that S_b = U_tau^* A|_b V_sigma for the block's factors.  L, sigma, blocks, S, SX, SY and
 * status are device arrays (lengths in complex elements, sigma_len in doubles); status[b] =
 * 1 for a block written, -1 for a descriptor whose sizes or ranges do not fit the lengths
 * (nothing written for it).  One workgroup per block; nothing is allocated; asynchronous
 * on hip_stream.  Errors: UHM_EINVAL (negative lengths, null pointers with nblocks > 0),
 * UHM_EHIP.
 */
int uhm_couplings(const double* L, int64_t L_len, const double* sigma, int64_t sigma_len,
                  const uhm_coupling_desc* blocks, int64_t nblocks, double* S, int64_t S_len, double* SX, int64_t SX_len,
                  double* SY, int64_t SY_len, int32_t* status, void* hip_stream);

const char* uhm_strerror(int code);
const char* uhm_last_error(void);
int uhm_version(void);

#ifdef __cplusplus
}
#endif

#endif /* UHM_H */
