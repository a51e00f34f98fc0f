// Batched inverse of the diagonal Schur blocks, S = Atil_kk^-1 (the
// inverse-instead-of-trsm formulation of Sec. II-B), by blocked Gauss-Jordan
// elimination with partial pivoting inside the block.
//
// Pivoting is implicit: no rows are swapped.  For column j the pivot is the
// not-yet-used row of largest |re| + |im| (lowest row index on ties); that row
// is scaled and column j is eliminated from every other row.  In place, the
// slot of column j then holds column p_j of the accumulated transform M
// (M A = Q, Q the permutation with Q e_j = e_{p_j}), so at the end
//     A^-1[j][c] = W[p_j][pinv(c)].
//
// Blocking: a panel of kInvNB columns is eliminated by one workgroup that
// holds the panel rows in registers (one barrier per column: every wave
// publishes its best candidate row, every thread then picks the winner).  The
// effect of the panel on the other columns is M_J = I + Mm Y, where
//     Mm[:, s] = (panel column s) - e_{p_s}   (d x NB)
//     Y[s, :]  = W[p_s, :] outside the panel, 0 inside (NB x d),
// applied by the grouped product kernel as W += Mm Y.
#include "common.h"
#include <climits>

namespace btsq {

__device__ inline double2 cmul_i(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// 1 / v by Smith's algorithm (no overflow for large |v|).
__device__ inline double2 crecip(double2 v) {
    if (fabs(v.x) >= fabs(v.y)) {
        const double r = v.y / v.x, den = v.x + v.y * r;
        return make_double2(1.0 / den, -r / den);
    }
    const double r = v.x / v.y, den = v.x * r + v.y;
    return make_double2(r / den, -1.0 / den);
}

__global__ void inv_init(const InvJob* __restrict__ jobs) {
    const InvJob J = jobs[blockIdx.y];
    const size_t total = (size_t)J.d * J.d;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += stride)
        J.W[e] = J.src[e];
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < (size_t)J.d; e += stride)
        J.used[e] = 0;
}

template <int R>
__global__ __launch_bounds__(kInvThreads)
void inv_panel(const InvJob* __restrict__ jobs, int panel, DevStatus* status) {
    constexpr int NB = kInvNB;
    constexpr int T = kInvThreads;
    constexpr int NW = T / 64;
    __shared__ double cand_v[2][NW];
    __shared__ int cand_r[2][NW];
    __shared__ double2 cand_row[2][NW][NB];
    __shared__ int piv[NB];

    const InvJob J = jobs[blockIdx.x];
    const int d = J.d;
    const int j0 = panel * NB;
    if (j0 >= d) return;
    const int nc = min(NB, d - j0);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;

    double2 P[R][NB];
    int used[R];
    // all panel loads in flight together: indices clamped into the matrix,
    // out-of-range entries zeroed after the loads complete
#pragma unroll
    for (int q = 0; q < R; ++q) {
        const int r = min(tid + q * T, d - 1);
        const double2* row = J.W + (size_t)r * d + j0;
        used[q] = J.used[r];
#pragma unroll
        for (int c = 0; c < NB; ++c) P[q][c] = row[min(c, nc - 1)];
    }
#pragma unroll
    for (int q = 0; q < R; ++q) {
        asm volatile("" : "+v"(used[q]));
#pragma unroll
        for (int c = 0; c < NB; ++c) asm volatile("" : "+v"(P[q][c].x), "+v"(P[q][c].y));
    }
#pragma unroll
    for (int q = 0; q < R; ++q) {
        const bool rin = tid + q * T < d;
        if (!rin) used[q] = 1;
#pragma unroll
        for (int c = 0; c < NB; ++c)
            if (!rin || c >= nc) P[q][c] = make_double2(0.0, 0.0);
    }

#pragma unroll
    for (int s = 0; s < NB; ++s) {
        if (s < nc) {
            const int sb = s & 1;
            // candidate of this thread (rows ascend with q, so ties keep the lower row)
            double bv = -1.0;
            int br = INT_MAX;
#pragma unroll
            for (int q = 0; q < R; ++q) {
                const int r = tid + q * T;
                if (r < d && !used[q]) {
                    double v = fabs(P[q][s].x) + fabs(P[q][s].y);
                    if (!(v >= 0.0)) v = INFINITY;   // NaN: make it win, and be flagged
                    if (v > bv) { bv = v; br = r; }
                }
            }
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) {
                const double ov = __shfl_xor(bv, off);
                const int orr = __shfl_xor(br, off);
                if (ov > bv || (ov == bv && orr < br)) { bv = ov; br = orr; }
            }
            if (br == INT_MAX) {
                if (lane == 0) { cand_v[sb][wave] = -1.0; cand_r[sb][wave] = INT_MAX; }
            } else if (br % T == tid) {
                const int qo = br / T;
                cand_v[sb][wave] = bv;
                cand_r[sb][wave] = br;
#pragma unroll
                for (int q = 0; q < R; ++q)
                    if (q == qo) {
#pragma unroll
                        for (int c = 0; c < NB; ++c) cand_row[sb][wave][c] = P[q][c];
                    }
            }
            __syncthreads();
            double gv = -1.0;
            int gr = INT_MAX, gw = 0;
#pragma unroll
            for (int w = 0; w < NW; ++w) {
                const double v = cand_v[sb][w];
                const int r = cand_r[sb][w];
                if (v > gv || (v == gv && r < gr)) { gv = v; gr = r; gw = w; }
            }
            if (!(gv > 0.0) || gv == INFINITY) {
                if (tid == 0 && atomicCAS(&status->code, 0, 3) == 0) status->tag = J.tag;
            }
            const double2 ip = crecip(cand_row[sb][gw][s]);
            double2 f[R];
#pragma unroll
            for (int q = 0; q < R; ++q) f[q] = P[q][s];
#pragma unroll
            for (int c = 0; c < NB; ++c) {
                const double2 spc = (c == s) ? ip : cmul_i(cand_row[sb][gw][c], ip);
#pragma unroll
                for (int q = 0; q < R; ++q) {
                    const int r = tid + q * T;
                    if (r == gr) {
                        P[q][c] = spc;
                    } else if (c == s) {
                        const double2 t = cmul_i(f[q], ip);
                        P[q][c] = make_double2(-t.x, -t.y);
                    } else {
                        const double2 t = cmul_i(f[q], spc);
                        P[q][c] = make_double2(P[q][c].x - t.x, P[q][c].y - t.y);
                    }
                }
            }
#pragma unroll
            for (int q = 0; q < R; ++q)
                if (tid + q * T == gr) used[q] = 1;
            if (tid == 0) piv[s] = gr;
        }
    }
    __syncthreads();

    // write back: panel columns, Mm, used flags, pivot rows
#pragma unroll
    for (int q = 0; q < R; ++q) {
        const int r = tid + q * T;
        if (r < d) {
            double2* row = J.W + (size_t)r * d + j0;
            double2* mrow = J.Mm + (size_t)r * NB;
#pragma unroll
            for (int c = 0; c < NB; ++c) {
                if (c < nc) {
                    row[c] = P[q][c];
                    double2 v = P[q][c];
                    if (piv[c] == r) v.x -= 1.0;
                    mrow[c] = v;
                } else {
                    mrow[c] = make_double2(0.0, 0.0);
                }
            }
            J.used[r] = used[q];
        }
    }
    if (tid < nc) J.perm[j0 + tid] = piv[tid];
    // Y: gathered pivot rows outside the panel (rows >= nc are zero).  Eight
    // loads per thread are issued before any is used.
    constexpr int U = 8;
    const int total = NB * d;
    for (int base = 0; base < total; base += U * T) {
        double2 v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int e = min(base + u * T + tid, total - 1);
            const int c = e / d, col = e - c * d;
            const int pr = piv[min(c, nc - 1)];
            v[u] = J.W[(size_t)pr * d + col];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) asm volatile("" : "+v"(v[u].x), "+v"(v[u].y));
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int e = base + u * T + tid;
            if (e < total) {
                const int c = e / d, col = e - c * d;
                const bool keep = c < nc && (col < j0 || col >= j0 + nc);
                J.Y[e] = keep ? v[u] : make_double2(0.0, 0.0);
            }
        }
    }
}

__global__ void inv_finish(const InvJob* __restrict__ jobs) {
    __shared__ int perm[kInvMaxDim];
    __shared__ int pinv[kInvMaxDim];
    const InvJob J = jobs[blockIdx.y];
    const int d = J.d;
    for (int e = threadIdx.x; e < d; e += blockDim.x) perm[e] = J.perm[e];
    __syncthreads();
    for (int e = threadIdx.x; e < d; e += blockDim.x) pinv[perm[e]] = e;
    __syncthreads();
    for (int j = blockIdx.x; j < d; j += gridDim.x) {
        const double2* src = J.W + (size_t)perm[j] * d;
        double2* dst = J.dst + (size_t)j * d;
        for (int c = threadIdx.x; c < d; c += blockDim.x) dst[c] = src[pinv[c]];
    }
}

hipError_t launch_inv_init(const InvJob* d_jobs, int njobs, int maxd, hipStream_t s) {
    if (njobs <= 0) return hipSuccess;
    int chunks = (int)(((size_t)maxd * maxd + 255) / 256);
    if (chunks > 64) chunks = 64;
    if (chunks < 1) chunks = 1;
    hipLaunchKernelGGL(inv_init, dim3(chunks, njobs), dim3(256), 0, s, d_jobs);
    return hipGetLastError();
}

hipError_t launch_inv_panel(const InvJob* d_jobs, int njobs, int rows_per_thread, int panel,
                            DevStatus* status, hipStream_t s) {
    if (njobs <= 0) return hipSuccess;
    if (rows_per_thread == 1)
        hipLaunchKernelGGL(inv_panel<1>, dim3(njobs), dim3(kInvThreads), 0, s, d_jobs, panel, status);
    else
        hipLaunchKernelGGL(inv_panel<2>, dim3(njobs), dim3(kInvThreads), 0, s, d_jobs, panel, status);
    return hipGetLastError();
}

hipError_t launch_inv_finish(const InvJob* d_jobs, int njobs, int maxd, hipStream_t s) {
    if (njobs <= 0) return hipSuccess;
    int rows = maxd < 64 ? maxd : 64;
    if (rows < 1) rows = 1;
    hipLaunchKernelGGL(inv_finish, dim3(rows, njobs), dim3(256), 0, s, d_jobs);
    return hipGetLastError();
}

}  // namespace btsq
