// Grouped elementwise block sums D = sum_j c_j op_j(X_j), op_j = identity or
// conjugate transpose.  Used where partitions meet (the arrow tip is the
// original tip plus one Schur contribution per partition, each accumulated
// separately so the partitions never write the same block: the single-GPU
// form of the tip reduction of Sec. III-B), and, for anti-Hermitian Sigma^<,
// to form one block of a conjugate pair from the other.
#include "common.h"

namespace btsq {

constexpr int kTile = 32;

__global__ void add_grouped(const AddOp* __restrict__ ops, int nops) {
    const AddOp& op = ops[blockIdx.y];
    if (op.hmask == 0) {
        const size_t total = (size_t)op.rows * op.cols;
        const size_t stride = (size_t)gridDim.x * blockDim.x;
        for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += stride) {
            double2 acc = make_double2(0.0, 0.0);
            for (int j = 0; j < op.nin; ++j) {
                const double2 x = op.X[j][e];
                const double2 c = op.c[j];
                acc.x += c.x * x.x - c.y * x.y;
                acc.y += c.x * x.y + c.y * x.x;
            }
            op.D[e] = acc;
        }
        return;
    }
    // With transposed inputs: 32 x 32 output tiles; a transposed input is read
    // along its rows (coalesced) into an LDS tile and used along its columns.
    __shared__ double2 tile[kTile][kTile + 1];
    const int rows = op.rows, cols = op.cols;
    const int tr = (rows + kTile - 1) / kTile, tc = (cols + kTile - 1) / kTile;
    constexpr int kPer = kTile * kTile / 256;        // elements per thread (blockDim 256)
    for (int t = blockIdx.x; t < tr * tc; t += gridDim.x) {
        const int r0 = (t / tc) * kTile, c0 = (t % tc) * kTile;
        double2 acc[kPer];
#pragma unroll
        for (int q = 0; q < kPer; ++q) acc[q] = make_double2(0.0, 0.0);
        for (int j = 0; j < op.nin; ++j) {
            const double2 c = op.c[j];
            const double2* X = op.X[j];
            if ((op.hmask >> j) & 1u) {
                __syncthreads();                          // the tile's previous readers are done
#pragma unroll
                for (int q = 0; q < kPer; ++q) {
                    const int e = threadIdx.x + 256 * q;
                    const int xr = c0 + e / kTile, xc = r0 + e % kTile;   // X is cols x rows
                    tile[e / kTile][e % kTile] =
                        (xr < cols && xc < rows) ? X[(size_t)xr * rows + xc] : make_double2(0.0, 0.0);
                }
                __syncthreads();
#pragma unroll
                for (int q = 0; q < kPer; ++q) {
                    const int e = threadIdx.x + 256 * q;
                    const double2 x = tile[e % kTile][e / kTile];    // X(c0 + l, r0 + i), conjugated
                    acc[q].x += c.x * x.x + c.y * x.y;
                    acc[q].y += c.y * x.x - c.x * x.y;
                }
            } else {
#pragma unroll
                for (int q = 0; q < kPer; ++q) {
                    const int e = threadIdx.x + 256 * q;
                    const int i = r0 + e / kTile, l = c0 + e % kTile;
                    if (i < rows && l < cols) {
                        const double2 x = X[(size_t)i * cols + l];
                        acc[q].x += c.x * x.x - c.y * x.y;
                        acc[q].y += c.x * x.y + c.y * x.x;
                    }
                }
            }
        }
#pragma unroll
        for (int q = 0; q < kPer; ++q) {
            const int e = threadIdx.x + 256 * q;
            const int i = r0 + e / kTile, l = c0 + e % kTile;
            if (i < rows && l < cols) op.D[(size_t)i * cols + l] = acc[q];
        }
    }
}

hipError_t launch_add(const AddOp* d_ops, int nops, size_t max_elems, hipStream_t s) {
    if (nops <= 0) return hipSuccess;
    size_t chunks = (max_elems + 255) / 256;
    if (chunks > 256) chunks = 256;
    if (chunks < 1) chunks = 1;
    hipLaunchKernelGGL(add_grouped, dim3((unsigned)chunks, nops), dim3(256), 0, s, d_ops, nops);
    return hipGetLastError();
}

}  // namespace btsq

namespace btsq {

// Frobenius norms of blocks: out[j] = ||X_j||_F, one workgroup per block,
// fixed-order reduction (deterministic).
__global__ void block_norms(const NormJob* __restrict__ jobs) {
    __shared__ double part[256];
    const NormJob J = jobs[blockIdx.x];
    const size_t total = (size_t)J.rows * J.cols;
    double s = 0.0;
    for (size_t e = threadIdx.x; e < total; e += blockDim.x) {
        const double2 v = J.X[e];
        s += v.x * v.x + v.y * v.y;
    }
    part[threadIdx.x] = s;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *J.out = sqrt(part[0]);
}

hipError_t launch_norms(const NormJob* d_jobs, int njobs, hipStream_t s) {
    if (njobs <= 0) return hipSuccess;
    hipLaunchKernelGGL(block_norms, dim3(njobs), dim3(256), 0, s, d_jobs);
    return hipGetLastError();
}

}  // namespace btsq
