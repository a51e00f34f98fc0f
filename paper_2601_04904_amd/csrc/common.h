// Plain-old-data descriptors shared by the host scheduler and the kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace btsq {

// One term alpha * op(A) * op(B) of a grouped product.  A is m x k after op,
// B is k x n after op; op = H reads the stored matrix conjugate-transposed.
struct GemmTerm {
    const double2* A;
    const double2* B;
    int32_t lda, ldb;     // leading dimensions of the stored matrices (complex elements)
    int32_t k;
    int32_t flags;        // bit0: op(A) = A^H, bit1: op(B) = B^H
    double2 alpha;
};

constexpr int kMaxTerms = 6;
constexpr int kGemmShapes = 3;     // product tile shapes: 32x32, 64x32, 64x64 complex
constexpr int kTermAH = 1;
constexpr int kTermBH = 2;

// D = beta * C + sum_t alpha_t op(A_t) op(B_t), D and C m x n (C may alias D
// or be null, then beta is ignored).  tile_begin: first tile of this product
// in the launch (products of one launch are independent of each other).
struct GemmOp {
    double2* D;
    const double2* C;
    int32_t ldd, ldc;
    int32_t m, n;
    int32_t nterms;
    int32_t tiles_n;      // tiles along n
    int32_t tile_begin;
    int32_t mixed;        // 1: products in complex64 (FP32 MFMA, FP32 accumulation)
    double2 beta;
    GemmTerm t[kMaxTerms];
};

// One diagonal-block inverse dst = src^-1 (d x d) by blocked Gauss-Jordan
// elimination with partial pivoting inside the block.
// Workgroups are dispatched round-robin over the 8 XCDs (each with its own
// L2).  This maps dispatch index b of a grid of g workgroups to a logical
// index so that each XCD receives one contiguous range of logical indices,
// i.e. neighbouring tiles (which share operand rows or columns) meet in the
// same L2.  It is a bijection on [0, g).
constexpr int kNumXcd = 8;
__device__ inline int xcd_remap(int b, int g) {
    const int xcd = b % kNumXcd, idx = b / kNumXcd;
    const int per = g / kNumXcd, rem = g % kNumXcd;
    return xcd < rem ? xcd * (per + 1) + idx : rem * (per + 1) + (xcd - rem) * per + idx;
}

struct InvJob {
    const double2* src;
    double2* dst;
    double2* W;       // d x d working matrix, column-major
    int32_t* perm;    // d pivot rows (perm[j] = pivot row of column j)
    int32_t* used;    // d flags
    int32_t d;
    int32_t tag;      // block id reported on a singular pivot
};

constexpr int kInvNB = 16;          // panel width (panel rows live in registers)
constexpr int kInvMaxDim = 1024;    // 512 threads x 2 rows at most

// Scratch of one inverse job: W (d x d), perm and used (d each), each piece
// starting on a 256-byte boundary.  inv_scratch_bytes is the span of one job's
// pieces from a 256-aligned start, rounded up to 256.
__host__ __device__ inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

__host__ __device__ inline size_t inv_scratch_bytes(int d) {
    return align256((size_t)d * d * sizeof(double2)) + 2 * align256((size_t)d * sizeof(int32_t));
}

// Points the job's scratch at pool + off (off 256-aligned); returns the end offset.
__host__ __device__ inline size_t inv_bind_scratch(InvJob& j, char* pool, size_t off, int d) {
    off = align256(off);
    j.W = reinterpret_cast<double2*>(pool + off);
    off += align256((size_t)d * d * sizeof(double2));
    j.perm = reinterpret_cast<int32_t*>(pool + off);
    off += align256((size_t)d * sizeof(int32_t));
    j.used = reinterpret_cast<int32_t*>(pool + off);
    off += align256((size_t)d * sizeof(int32_t));
    return off;
}

// D = sum_j c_j op_j(X_j), op_j = X or X^H (elementwise, rows x cols, contiguous).
constexpr int kMaxAdd = 17;
struct AddOp {
    double2* D;
    const double2* X[kMaxAdd];
    double2 c[kMaxAdd];
    int32_t nin;
    int32_t rows, cols;
    uint32_t hmask;       // bit j: input j enters as X_j^H (stored cols x rows; must not be D)
};

// *out = ||X||_F of one block.
struct NormJob {
    const double2* X;
    double* out;
    int32_t rows, cols;
};

// Fused small-instance path: one workgroup runs the whole operation list of
// one instance.  A task is the instance's range of step records, in
// dependency order; a record holds the step's kind and its descriptor
// itself (fixed size), so the next step's record can be fetched while the
// current one runs.
constexpr int kFusedMaxDim = 64;    // largest diagonal block / tip the fused path inverts

struct FusedInv {
    const double2* src;   // d x d, row-major
    double2* dst;         // d x d, row-major (may be src)
    int32_t d;
    int32_t tag;          // block id reported on a singular pivot
};

constexpr size_t kFusedBody = sizeof(GemmOp) > sizeof(AddOp) ? sizeof(GemmOp) : sizeof(AddOp);

struct alignas(16) FusedRec {
    int32_t type;         // 0 product, 1 inverse, 2 sum
    int32_t pad[3];
    alignas(16) unsigned char body[(kFusedBody + 15) / 16 * 16];   // a GemmOp, FusedInv or AddOp
};
static_assert(sizeof(FusedInv) <= kFusedBody, "record body too small");
static_assert(sizeof(FusedRec) % 16 == 0, "records are 16-byte multiples");

struct FusedTask {
    int32_t first;        // first record
    int32_t count;
};

// Device-side status: [0] error code (0 = ok, 3 = singular), [1] tag.
struct DevStatus {
    int32_t code;
    int32_t tag;
};

}  // namespace btsq
