/*
 * bt_si_sq.h - selected inversion (SI) and selected quadratic solve (SQ) of
 * block-tridiagonal (BT) and BT-with-arrowhead (BTA) matrices on MI355X.
 *
 * Problem (Sec. II-A of arXiv 2601.04904): A and B share one BT/BTA pattern
 * with n diagonal blocks of size b and, for BTA, an arrow tip of size a
 * (N = n b + a).  The library returns the blocks of
 *     X^R = A^-1                 (selected inversion, A X = I)
 *     X^< = A^-1 B A^-H          (selected quadratic solve, A X A^H = B)
 * on that same pattern only: X_{i,i}, X_{i,i+1}, X_{i+1,i}, X_{i,t}, X_{t,i},
 * X_{t,t}.  It uses the forward Schur-complement / backward sweeps of RGF
 * (Alg. 1 and Alg. 2), their BTA extension (Sec. III-A) and, for P > 1, the
 * partitioned scheme of Sec. III-B (P partitions eliminated concurrently on
 * one GPU, then the reduced system of 2(P-1) blocks plus the tip, then the
 * partition backward sweeps).  Diagonal blocks are inverted explicitly with
 * partial pivoting inside the block (the inverse-instead-of-trsm formulation
 * of Sec. II-B); there is no pivoting across blocks.
 *
 * Data layout.  Every matrix argument is a bt_blocks of DEVICE pointers to
 * complex128 numbers stored as interleaved (re, im) doubles, each block
 * dense row-major with leading dimension equal to its column count:
 *     diag          n     blocks of b x b     M_{i,i}
 *     upper         n-1   blocks of b x b     M_{i,i+1}
 *     lower         n-1   blocks of b x b     M_{i+1,i}
 *     arrow_right   n     blocks of b x a     M_{i,t}     (NULL when a == 0)
 *     arrow_bottom  n     blocks of a x b     M_{t,i}     (NULL when a == 0)
 *     tip           1     block  of a x a     M_{t,t}     (NULL when a == 0)
 * Blocks of one field are contiguous (block i starts at i * rows * cols
 * complex numbers).  With per-block sizes b_i (bt_desc.block_sizes) block i
 * of diag is b_i x b_i, of upper b_i x b_{i+1}, of lower b_{i+1} x b_i, of
 * arrow_right b_i x a and of arrow_bottom a x b_i, and block i of a field
 * starts after the blocks 0..i-1 of that field (at sum_{j<i} b_j^2,
 * sum_{j<i} b_j b_{j+1} and a sum_{j<i} b_j complex numbers).
 *
 * Ownership.  The caller owns A, B and the output blocks (device memory it
 * allocated).  The library never writes to A or B, and outputs must not
 * alias inputs.  The handle owns its workspace (device memory allocated at
 * create, freed at destroy), which holds the stored factors and the updated
 * (Schur-complemented) blocks.  After bt_si_sq_factor, selected_solve may be
 * called any number of times (different B, e.g. Sigma^< and Sigma^>); it
 * reads the original off-diagonal and arrow blocks of A and the X^R blocks
 * where factor left them, so A and the XR given to factor (if any) must stay
 * allocated and unmodified until the last selected_solve.
 *
 * Streams and errors.  Calls that take a handle enqueue work on the HIP
 * stream given at create and return without waiting, except that they may
 * wait for the previous call's operation list to finish uploading.  Results
 * are valid once that stream is synchronised.  Every function returns a
 * bt_status; nothing is thrown across the ABI.  Argument errors are found
 * on the host and returned at once.  A singular or non-finite pivot found
 * on the device is recorded in the handle and returned by the next
 * bt_si_sq_sync (BT_ERR_SINGULAR, with the block in the message).  A
 * handle must not be used from two threads at once; distinct handles are
 * independent.
 */
#ifndef BT_SI_SQ_H
#define BT_SI_SQ_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct bt_si_sq_plan* bt_si_sq_handle;

typedef enum {
    BT_OK = 0,
    BT_ERR_INVALID = 1,     /* bad descriptor or argument */
    BT_ERR_OOM = 2,         /* device allocation failed */
    BT_ERR_SINGULAR = 3,    /* zero or non-finite pivot in a diagonal-block inverse */
    BT_ERR_HIP = 4,         /* a HIP runtime call failed */
    BT_ERR_STATE = 5,       /* e.g. selected_solve before factor */
    BT_ERR_TOLERANCE = 6    /* mixed path: the error estimate of the FP64 re-run is still
                               above tol; the results and estimates are written */
} bt_status;

typedef enum {
    BT_FP64 = 0,            /* every product in complex128 on FP64 MFMA */
    BT_MIXED = 1            /* Schur-update products in complex64 on FP32 MFMA (FP32
                               accumulation); diagonal-block inverses, the reduced
                               system and the residual check stay FP64 */
} bt_precision;

/* flags */
#define BT_DIAG_ONLY 0x1u   /* outputs are the diagonal blocks X_{i,i} (and X_{t,t}) only, the
                               form Sec. II-B gives after Alg. 2: the off-diagonal blocks of
                               X^R and X^< are computed only where a later backward step
                               reads them again, into the workspace, and the others not at
                               all (for sequential BT two of the 23 block products per step).
                               The off-diagonal and arrow pointers of XR and XL are ignored
                               and may be NULL.  Needs BT_FP64 (BT_ERR_INVALID with
                               BT_MIXED, whose error estimate reads the off-diagonal
                               blocks). */
#define BT_PLAIN 0x2u       /* reference schedule: one launch per single-term block product
                               and per inverse, in program order, on one stream (no
                               grouping, no multi-term fusion, no stream overlap) */
#define BT_GRAPH 0x4u       /* run each compiled launch list as one captured HIP graph
                               (captured at its first run, replayed afterwards; not while
                               profiling).  A batch handle uses graphs when every instance
                               sets the flag. */
#define BT_SIGMA_ANTIHERMITIAN 0x8u
                            /* the caller asserts Sigma^< = -(Sigma^<)^H on the pattern
                               (true of the lesser self-energies of NEGF, Sec. II-A).
                               Every Schur complement of B is then anti-Hermitian, and
                               the forward sweep takes one block of each conjugate pair
                               of B updates as the negated conjugate transpose of the
                               other; the backward sweep takes the k-row products of X^<
                               from the k-column ones the same way: about a sixth fewer
                               flops for BT.  The assertion is not checked; for other B
                               the result is wrong. */
#define BT_FUSED 0x10u      /* small instances: one workgroup runs the instance's whole
                               operation list (every product, diagonal-block inverse and
                               block sum of the sweeps of Alg. 1/2, Sec. III-A and, for
                               P > 1, Sec. III-B) in dependency order, with workgroup
                               barriers only; a batch runs all its BT_FUSED instances in
                               one launch, one workgroup each, beside the grouped launches
                               of the others.  No launch per dependency level, so it pays
                               where those levels are short (small b).  Needs every
                               diagonal block and the tip of size <= 64 and BT_FP64
                               without BT_PLAIN (else BT_ERR_INVALID).  Results agree with
                               the grouped path to rounding (other summation order, and
                               the inverse pivots on the rows of the block). */

typedef struct {
    int32_t n;                  /* number of diagonal blocks, >= 1 */
    int32_t b;                  /* diagonal block size, >= 1 */
    int32_t a;                  /* arrow tip size, >= 0 (0: plain BT) */
    int32_t partitions;         /* P >= 1; 1 = sequential RGF (Alg. 1/2) */
    const int32_t* part_bounds; /* host array of P+1 increasing block indices
                                   0 = s_0 < s_1 < ... < s_P = n, or NULL for
                                   bounds from the cost model.  First and last
                                   partitions need >= 1 block, middle ones >= 2. */
    int32_t precision;          /* bt_precision */
    double tol;                 /* mixed path: re-run in FP64 when the error estimate
                                   exceeds tol (<= 0 selects 1e-4) */
    uint32_t flags;
    const int32_t* block_sizes; /* host array of n diagonal-block sizes (each 1..1024),
                                   or NULL for n blocks of size b.  RGF applies
                                   unchanged to blocks of different sizes (Sec. II-A);
                                   b is then ignored.  Read during the call only. */
    int32_t reduced_parts;      /* P > 1: the reduced system (2(P-1) kept blocks and the
                                   tip) is solved by the same partitioned elimination,
                                   recursively (Sec. III-B), with
                                   q = min(reduced_parts, m/2) parts of an m-block
                                   reduced system while m >= 4, then the sequential
                                   RGF.  0 (default) = 2: first half top-down, second
                                   half bottom-up; 1 = sequential RGF at once.  More
                                   parts shorten the sequential chain but add the middle
                                   parts' fill and flops, and on weakly broadened
                                   inputs (no pivoting across blocks) amplify rounding.
                                   0..1024, else BT_ERR_INVALID. */
} bt_desc;

typedef struct {
    void* diag;
    void* upper;
    void* lower;
    void* arrow_right;
    void* arrow_bottom;
    void* tip;
} bt_blocks;

/* Device bytes the handle for this descriptor allocates (one block: workspace
 * for the stored factors, fill-in, reduced system and intermediates, the
 * inverse scratch, and room for the uploaded operation lists).  Pure host
 * computation, no side effects; 0 for an invalid descriptor.  Used for
 * admission by device-memory footprint. */
size_t bt_si_sq_workspace_bytes(const bt_desc* desc);

/* Partition bounds the library uses for this descriptor (the given ones, or
 * those balancing the per-block cost 8(3b^3 + 11 D b^2 + 10 D^2 b) with D
 * the total size of the block's neighbours).  bounds_out has P+1 entries. */
bt_status bt_si_sq_partition_bounds(const bt_desc* desc, int32_t* bounds_out);

/* Real floating-point operations of one fused SI+SQ solve: `executed` counts
 * the products and inverses the library runs (complex m x n x k product =
 * 8mnk, complex b x b inverse = 8b^3); `useful` counts those of the
 * sequential RGF of the same matrix, without BT_SIGMA_ANTIHERMITIAN.  Pure
 * host computation. */
bt_status bt_si_sq_flops(const bt_desc* desc, double* executed, double* useful);

/* Validate the descriptor, allocate the workspace, bind the HIP stream
 * (hipStream_t passed as void*; NULL = the null stream). */
bt_status bt_si_sq_create(const bt_desc* desc, void* hip_stream, bt_si_sq_handle* out);

/* factor, selected_solve and solve take single-instance handles.
 *
 * Forward Schur-complement sweep of A (the A-chain of Alg. 1, extended to
 * BTA and partitions) and backward selected inversion (Alg. 2, SI part).
 * Writes X^R into XR when XR is non-NULL (the factors and X^R are also kept
 * in the workspace for selected_solve). */
bt_status bt_si_sq_factor(bt_si_sq_handle h, const bt_blocks* A, bt_blocks* XR);

/* Selected quadratic solve for right-hand side B with the factors of the
 * last bt_si_sq_factor (the B-chain of Alg. 1 and the SQ part of Alg. 2).
 * Writes X^< into XL.  err_estimate and used_fp64_fallback (host pointers,
 * may be NULL) are set to 0 for BT_FP64 handles.  For BT_MIXED handles the
 * call waits for the stream: it computes the FP64 selected residuals
 * R^R_i = sum_j A_ij X^R_ji - I and R^<_i = sum_j A_ij X^<_ji - sum_j B_ij
 * (X^R_ij)^H on the GPU, turns them into the estimate
 *     max(rho_R, rho_L) * nA * nG,  rho_R = max_i ||R^R_i||_F / sqrt(d_i),
 *     rho_L = max_i ||R^<_i||_F / (nA max_i ||X^<_ii||_F),
 *     nA = max_i ||A_ii||_F / sqrt(d_i),  nG = max_i ||X^R_ii||_F
 * (a relative residual times a blockwise ||A|| ||A^-1|| estimate), and when
 * it exceeds tol re-runs the whole solve with FP64 products - factor and
 * selected solve of the A and X^R given to the last factor call, so an error
 * that comes from the A-chain is removed too - returning the estimate of the
 * final result and used_fp64_fallback = 1.  If that estimate is still above
 * tol the call returns BT_ERR_TOLERANCE (results and estimate written). */
bt_status bt_si_sq_selected_solve(bt_si_sq_handle h, const bt_blocks* B, bt_blocks* XL,
                                  double* err_estimate, int* used_fp64_fallback);

/* Fused SI+SQ: factor(A) and selected_solve(B) in one schedule, so the
 * B-chain of step k overlaps the A-chain of step k+1 and the SQ backward
 * step k overlaps the SI backward step k-1.  XR may be NULL. */
bt_status bt_si_sq_solve(bt_si_sq_handle h, const bt_blocks* A, const bt_blocks* B,
                         bt_blocks* XR, bt_blocks* XL,
                         double* err_estimate, int* used_fp64_fallback);

/* ---- Batches of uneven instances ----------------------------------------
 * A batch handle holds `count` independent instances (each its own n, b, a,
 * partitions and precision) in one workspace.  One batch_solve builds a single
 * schedule for all of them: at every dependency level the products of all
 * instances share one grouped launch and their diagonal-block inverses one
 * batched inverse, so many small solves fill the GPU together.  Mixed
 * instances get their error estimate and, above their tol, an FP64 re-run
 * of just those instances (the call then waits for the stream);
 * BT_ERR_TOLERANCE when a re-run instance's estimate is still above its tol
 * (every result and estimate written). */
size_t bt_si_sq_batch_workspace_bytes(int32_t count, const bt_desc* descs);

bt_status bt_si_sq_batch_create(int32_t count, const bt_desc* descs, void* hip_stream,
                                bt_si_sq_handle* out);

/* bt_si_sq_batch_create with device memory the caller provides, for callers
 * that keep a pool (a serving loop drawing on a caching allocator): the
 * handle takes its workspace, inverse scratch, status word and the room for
 * its uploaded operation lists from `workspace` (device memory of at least
 * bt_si_sq_batch_workspace_bytes(count, descs) bytes, 256-byte aligned) and
 * allocates no other device memory in normal operation (an operation list
 * larger than that room, which no schedule of the library produces, gets an
 * allocation of its own).  The caller owns `workspace`: it must stay
 * allocated and untouched until bt_si_sq_destroy returns; destroy does not
 * free it.  BT_ERR_INVALID for a null, misaligned or too small workspace. */
bt_status bt_si_sq_batch_create_in(int32_t count, const bt_desc* descs, void* hip_stream,
                                   void* workspace, size_t workspace_bytes, bt_si_sq_handle* out);

/* A, B, XL: arrays of `count` bt_blocks (instance i uses element i); XR may be
 * NULL or have all-NULL elements (X^R then stays in the workspace).
 * err_estimates and used_fp64_fallback: NULL or host arrays of `count`. */
bt_status bt_si_sq_batch_solve(bt_si_sq_handle h, const bt_blocks* A, const bt_blocks* B,
                               bt_blocks* XR, bt_blocks* XL, double* err_estimates,
                               int* used_fp64_fallback);

/* Selected quadratic solve of new right-hand sides on the factors the last
 * batch_solve (or factor) left resident: instance i uses B[i], XL[i]; an
 * instance whose XL[i].diag is NULL is skipped.  Same estimate/fallback rules
 * as batch_solve. */
bt_status bt_si_sq_batch_selected_solve(bt_si_sq_handle h, const bt_blocks* B, bt_blocks* XL,
                                        double* err_estimates, int* used_fp64_fallback);

/* Number of instances of a handle (1 for bt_si_sq_create). */
int32_t bt_si_sq_batch_count(bt_si_sq_handle h);

/* Wait for the handle's stream and return the first device-side error
 * recorded since the last sync (BT_OK if none). */
bt_status bt_si_sq_sync(bt_si_sq_handle h);

/* Free the workspace and the handle.  Waits for the stream first. */
bt_status bt_si_sq_destroy(bt_si_sq_handle h);

/* Message of the last error on this handle ("" if none); with h == NULL the
 * last error of a call that had no handle (create, workspace queries).
 * Valid until the next call on the same handle. */
const char* bt_si_sq_last_error(bt_si_sq_handle h);

/* Number of kernel launches of the last enqueued solve (diagnostics). */
int32_t bt_si_sq_last_launch_count(bt_si_sq_handle h);

/* Per-kernel measurement.  With enable != 0 every launch of the following
 * factor/selected_solve/solve calls is bracketed by HIP events recorded on
 * the handle's stream (all launches then run on that stream, one after
 * another, so each launch's event time is the kernel's own time rather
 * than its share of a GPU that other streams' launches also use), and
 * bt_si_sq_profile_stats returns, per kernel
 * family, the launch count, the summed event time and the summed
 * algorithmic work of those launches.  Enabling (or disabling) clears the
 * totals.  Event bracketing adds host work per launch; time whole solves
 * with profiling off. */
typedef enum {
    BT_KERNEL_PRODUCT_FP64 = 0,   /* grouped complex products, FP64 MFMA */
    BT_KERNEL_PRODUCT_MIXED = 1,  /* grouped complex products, FP32 MFMA */
    BT_KERNEL_INV_PANEL = 2,      /* inverse: panel elimination (the launches also read the
                                     block to invert and write the result) */
    BT_KERNEL_INV_INIT = 3,       /* unused (kept for numbering) */
    BT_KERNEL_INV_FINISH = 4,     /* unused (kept for numbering) */
    BT_KERNEL_SUM = 5,            /* elementwise block sums */
    BT_KERNEL_NORM = 6,           /* block norms of the residual check */
    BT_KERNEL_FUSED = 7,          /* whole BT_FUSED instances, one workgroup each */
    BT_KERNEL_COUNT = 8
} bt_kernel_kind;

typedef struct {
    int32_t kind;        /* bt_kernel_kind */
    int32_t launches;
    double total_ms;     /* summed HIP-event time of the launches */
    double flops;        /* summed algorithmic real flops (complex m x n x k product = 8mnk) */
    double bytes;        /* summed algorithmic HBM bytes (each operand read once, result written once) */
} bt_kernel_stat;

bt_status bt_si_sq_profile(bt_si_sq_handle h, int32_t enable);

/* Waits for the stream, then writes up to max_entries stats (one per kernel
 * family that ran) into out and their number into *count. */
bt_status bt_si_sq_profile_stats(bt_si_sq_handle h, bt_kernel_stat* out, int32_t max_entries,
                                 int32_t* count);

/* ---- Tile-shape tuning of the grouped complex products -------------------
 *
 * Every block update of the sweeps is a dense complex product (Sec. II-B,
 * the products of Alg. 1 and Alg. 2 and their arrowhead and partitioned
 * forms); one launch runs all products of one dependency level.  The
 * product kernel has BT_TILE_SHAPES tile shapes (complex rows x columns):
 * 0 = 32 x 32, 1 = 64 x 32, 2 = 64 x 64.  A launch is classified by
 * precision (0 FP64, 1 mixed), size class (log2 of its largest output
 * dimension, 32..1024 -> 0..5) and work class (log2 of its 64 x 32 tile
 * count, 1..8192 -> 0..13); the shape of a class comes from a process-wide
 * tuning table, or from a default rule for classes never tuned.  Handles
 * compile their launch lists when a pointer set is first used, so a table
 * change reaches launch lists compiled after it. */
#define BT_TILE_SHAPES 3
#define BT_TUNE_SIZE_CLASSES 6
#define BT_TUNE_WORK_CLASSES 14
#define BT_TUNE_ENTRIES (2 * BT_TUNE_SIZE_CLASSES * BT_TUNE_WORK_CLASSES)

/* Times every tile shape on synthetic grouped launches of square products
 * (sizes 64..1024, 1 to 4096 products per launch) in both precisions and
 * stores the fastest shape of each class reached into the tuning table.
 * Allocates and frees its own device scratch (about 300 MB), runs on
 * hip_stream (NULL: the null stream) and returns when done (a few seconds).
 * If report is not NULL, a text line per class ("prec size_class work_class
 * shape us_shape0 us_shape1 us_shape2") is written into it (truncated to cap
 * bytes, NUL-terminated).
 * Errors: BT_ERR_OOM, BT_ERR_HIP (the table is left unchanged). */
bt_status bt_si_sq_autotune(void* hip_stream, char* report, size_t cap);

/* Reads (get != 0) or writes (get == 0) the tuning table: table holds
 * BT_TUNE_ENTRIES int32 values laid out [precision][size class][work class],
 * each a tile shape or -1 (untuned: default rule).  Writing rejects values
 * outside [-1, BT_TILE_SHAPES) with BT_ERR_INVALID and changes nothing. */
bt_status bt_si_sq_tune_table(int32_t* table, int32_t get);

#ifdef __cplusplus
}
#endif

#endif /* BT_SI_SQ_H */
