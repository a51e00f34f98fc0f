/*
 * bt_si_sq_diag.h - diagnostic entry points of the same library: the two
 * kernel families of bt_si_sq.h run on their own, so tests can check each
 * against a reference.  Same conventions as bt_si_sq.h: device pointers to
 * interleaved complex128, row-major, enqueued on the given HIP stream,
 * status codes only.
 */
#ifndef BT_SI_SQ_DIAG_H
#define BT_SI_SQ_DIAG_H

#include "bt_si_sq.h"

#ifdef __cplusplus
extern "C" {
#endif

/* D = beta * C + alpha * op(A) op(B), D and C m x n, op(A) m x k, op(B) k x n.
 * opA/opB: 0 = as stored, 1 = conjugate transpose (then A is stored k x m,
 * B is stored n x k).  alpha, beta: host arrays {re, im}.  C may be NULL
 * (beta ignored) or equal D.  mixed = 1 runs the product in complex64 on
 * FP32 MFMA (the mixed-precision path).  shape: tile shape 0..BT_TILE_SHAPES-1,
 * or -1 for the one the tuning table gives this launch.  Each operand's
 * stored extent must stay below 2 GiB (BT_ERR_INVALID otherwise). */
bt_status bt_si_sq_diag_gemm(int32_t m, int32_t n, int32_t k,
                             const double* alpha, const void* A, int32_t lda, int32_t opA,
                             const void* B, int32_t ldb, int32_t opB,
                             const double* beta, const void* C, int32_t ldc,
                             void* D, int32_t ldd, int32_t mixed, int32_t shape, void* hip_stream);

/* dst[i] = src[i]^-1 for `count` contiguous d x d matrices (Gauss-Jordan with
 * partial pivoting inside each matrix, as used for the diagonal Schur
 * blocks).  Waits for the stream; returns BT_ERR_SINGULAR with *bad_index set
 * to the first matrix found singular or non-finite (bad_index may be NULL). */
bt_status bt_si_sq_diag_inverse(const void* src, void* dst, int32_t d, int32_t count,
                                int32_t* bad_index, void* hip_stream);

/* bt_si_sq_diag_inverse for callers that cannot allocate device memory (code
 * under HIP graph capture, serving loops that forbid hipMalloc): the same
 * result from the same kernels, but every piece of scratch - job descriptors,
 * the device status word, working copies, panel transforms, pivot arrays -
 * lives in one fixed device array of the library (64 MiB on every device the
 * library runs on, held until the process ends; its size is returned by
 * bt_si_sq_diag_inverse_noalloc_max_bytes).  No hipMalloc, hipFree or other
 * allocating call is made.  One call needs 256 + align256(48 count) + count *
 * (align256(16 d^2) + 2 align256(4 d)) bytes; a larger
 * request returns BT_ERR_INVALID before touching the device (message in
 * bt_si_sq_last_error(NULL)).  All calls on one device share the array:
 * calls that overlap on one device (other threads, other streams) race and
 * must be serialised by the caller.  Waits for the stream, like
 * bt_si_sq_diag_inverse. */
bt_status bt_si_sq_diag_inverse_noalloc(const void* src, void* dst, int32_t d, int32_t count,
                                        int32_t* bad_index, void* hip_stream);

/* Size in bytes of the fixed scratch array of bt_si_sq_diag_inverse_noalloc. */
size_t bt_si_sq_diag_inverse_noalloc_max_bytes(void);

/* Schedule of a fused solve for this descriptor, as text: one line per
 * dependency level with its number of products, product tiles (64 x 32
 * complex) and inverses.  Pure host computation.  Writes at most cap bytes
 * (NUL-terminated) and returns the length the full text needs. */
size_t bt_si_sq_diag_schedule(const bt_desc* desc, char* out, size_t cap);

#ifdef __cplusplus
}
#endif

#endif /* BT_SI_SQ_DIAG_H */
