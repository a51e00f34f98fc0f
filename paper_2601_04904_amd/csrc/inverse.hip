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

// Maximum over the 64 lanes of a wave, by DPP moves (both halves of the
// double): lanes within rows of 16, then row broadcasts; returned to every lane.
template <int CTRL, int ROW_MASK>
__device__ inline double dpp_double(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = (int)(b & 0xffffffffll), hi = (int)(b >> 32);
    const int olo = __builtin_amdgcn_update_dpp(lo, lo, CTRL, ROW_MASK, 0xf, false);
    const int ohi = __builtin_amdgcn_update_dpp(hi, hi, CTRL, ROW_MASK, 0xf, false);
    return __longlong_as_double(((long long)ohi << 32) | (unsigned int)olo);
}

__device__ inline double wave_max(double x) {
    x = fmax(x, dpp_double<0xB1, 0xf>(x));    // quad_perm [1,0,3,2]
    x = fmax(x, dpp_double<0x4E, 0xf>(x));    // quad_perm [2,3,0,1]
    x = fmax(x, dpp_double<0x124, 0xf>(x));   // row_ror:4
    x = fmax(x, dpp_double<0x128, 0xf>(x));   // row_ror:8  -> every lane holds its row's maximum
    x = fmax(x, dpp_double<0x142, 0xa>(x));   // row_bcast:15 into rows 1 and 3
    x = fmax(x, dpp_double<0x143, 0xc>(x));   // row_bcast:31 into rows 2 and 3 -> lane 63 holds it
    const long long b = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), 63);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), 63);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
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

// One launch per panel p.  Per matrix, workgroup 0 (the panel workgroup)
// applies the transform of panel p-1 to block p (look-ahead) and then
// eliminates block p; workgroups 1.. apply the transform of panel p-1 to the
// other 8-column blocks (all but blocks p-1 and p), each first gathering the
// pivot rows of its own columns, so no workgroup reads what another writes.
// Mm is double-buffered by panel parity (Mm + (p % 2) * d * NB).
constexpr int kUpdCols = 8;

template <int R>
__device__ void step_update(const InvJob& J, int p, int u, int tid) {
    constexpr int NB = kInvNB;
    constexpr int T = kInvThreads;
    constexpr int UC = kUpdCols;
    __shared__ double2 G[NB][UC];
    const int d = J.d;
    const int c0 = u * UC;
    if (c0 >= d || (p - 1) * NB >= d) return;   // no such columns / no panel p-1 for this matrix
    const int blk = c0 / NB;
    if (blk == p - 1 || blk == p) return;
    const int q0 = (p - 1) * NB;                  // first column of panel p-1
    const int nc = min(NB, d - q0);
    const double2* Mm = J.Mm + (size_t)((p - 1) & 1) * d * NB;
    if (tid < NB * UC) {
        const int s = tid / UC, j = tid % UC;
        const int sr = min(s, nc - 1), cc = min(c0 + j, d - 1);
        const double2 v = J.W[(size_t)J.perm[q0 + sr] * d + cc];
        G[s][j] = (s < nc && c0 + j < d) ? v : make_double2(0.0, 0.0);
    }
    __syncthreads();
    const int ncols = min(UC, d - c0);
#pragma unroll
    for (int q = 0; q < R; ++q) {
        const int r = tid + q * T;
        if (r >= d) continue;
        double2 acc[UC];
        const double2* wrow = J.W + (size_t)r * d + c0;
        const double2* mrow = Mm + (size_t)r * NB;
#pragma unroll
        for (int j = 0; j < UC; ++j) acc[j] = wrow[min(j, ncols - 1)];
#pragma unroll 2
        for (int s = 0; s < NB; s += 4) {
            double2 m[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) m[i] = mrow[s + i];
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < UC; ++j) {
                    const double2 g = G[s + i][j];
                    acc[j].x += m[i].x * g.x - m[i].y * g.y;
                    acc[j].y += m[i].x * g.y + m[i].y * g.x;
                }
        }
        double2* wout = J.W + (size_t)r * d + c0;
#pragma unroll
        for (int j = 0; j < UC; ++j)
            if (j < ncols) wout[j] = acc[j];
    }
}

template <int R>
__device__ void step_panel(const InvJob& J, int p, int tid, DevStatus* status) {
    constexpr int NB = kInvNB;
    constexpr int T = kInvThreads;
    constexpr int NW = T / 64;
    __shared__ double cand_v[2][NW];
    __shared__ int cand_r[2][NW];
    __shared__ double2 cand_row[2][NW][NB];
    __shared__ int piv[NB];
    __shared__ double2 G[NB][NB];

    const int d = J.d;
    const int j0 = p * NB;
    if (j0 >= d) return;
    const int nc = min(NB, d - j0);
    const int lane = tid & 63, wave = tid >> 6;

    double2 P[R][NB];
    int used[R];
#pragma unroll
    for (int q = 0; q < R; ++q) {
        const int r = min(tid + q * T, d - 1);
        const double2* row = J.W + (size_t)r * d + j0;
        used[q] = J.used[r];
#pragma unroll
        for (int c = 0; c < NB; ++c) P[q][c] = row[min(c, nc - 1)];
    }
    // look-ahead: apply the transform of panel p-1 to this block
    if (p > 0) {
        const int q0 = (p - 1) * NB;
        const int pnc = min(NB, d - q0);
        if (tid < NB * NB) {
            const int s = tid / NB, c = tid % NB;
            const int sr = min(s, pnc - 1), cc = min(c, nc - 1);
            const double2 v = J.W[(size_t)J.perm[q0 + sr] * d + j0 + cc];
            G[s][c] = (s < pnc && c < nc) ? v : make_double2(0.0, 0.0);
        }
        __syncthreads();
        const double2* Mm = J.Mm + (size_t)((p - 1) & 1) * d * NB;
#pragma unroll
        for (int q = 0; q < R; ++q) {
            const int r = min(tid + q * T, d - 1);
            const double2* mrow = Mm + (size_t)r * NB;
#pragma unroll 2
            for (int s = 0; s < NB; s += 4) {
                double2 m[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) m[i] = mrow[s + i];
#pragma unroll
                for (int i = 0; i < 4; ++i)
#pragma unroll
                    for (int c = 0; c < NB; ++c) {
                        const double2 g = G[s + i][c];
                        P[q][c].x += m[i].x * g.x - m[i].y * g.y;
                        P[q][c].y += m[i].x * g.y + m[i].y * g.x;
                    }
            }
        }
    }
#pragma unroll
    for (int q = 0; q < R; ++q) {
        const bool rin = tid + q * T < d;
        if (!rin) used[q] = 1;
#pragma unroll
        for (int c = 0; c < NB; ++c)
            if (!rin || c >= nc) P[q][c] = make_double2(0.0, 0.0);
    }

    for (int s = 0; s < NB; ++s) {
        if (s < nc) {
            const int sb = s & 1;
            // candidate of this lane: largest |re| + |im| among its unused rows
            // (rows ascend with q, so ties keep the lower row)
            double bv = -1.0;
            int br = INT_MAX;
#pragma unroll
            for (int q = 0; q < R; ++q) {
                const int r = tid + q * T;
                if (r < d && !used[q]) {
                    double v = fabs(P[q][0].x) + fabs(P[q][0].y);
                    if (!(v >= 0.0)) v = INFINITY;   // NaN: make it win, and be flagged
                    if (v > bv) { bv = v; br = r; }
                }
            }
            // wave maximum, then the lowest lane holding it
            const double wmax = wave_max(bv);
            const unsigned long long hit = __ballot(bv == wmax && br != INT_MAX);
            if (hit == 0ull) {
                if (lane == 0) { cand_v[sb][wave] = -1.0; cand_r[sb][wave] = INT_MAX; }
            } else if (lane == (int)__builtin_ctzll(hit)) {
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
            const double2 ip = crecip(cand_row[sb][gw][0]);
            double2 f[R];
#pragma unroll
            for (int q = 0; q < R; ++q) f[q] = P[q][0];
#pragma unroll
            for (int c = 0; c < NB; ++c) {
                const double2 spc = (c == 0) ? ip : cmul_i(cand_row[sb][gw][c], ip);
#pragma unroll
                for (int q = 0; q < R; ++q) {
                    const int r = tid + q * T;
                    const double2 t = cmul_i(f[q], spc);
                    const double ux = (c == 0) ? -t.x : P[q][c].x - t.x;
                    const double uy = (c == 0) ? -t.y : P[q][c].y - t.y;
                    const bool piv_row = r == gr;
                    P[q][c].x = piv_row ? spc.x : ux;
                    P[q][c].y = piv_row ? spc.y : uy;
                }
            }
#pragma unroll
            for (int q = 0; q < R; ++q)
                if (tid + q * T == gr) used[q] = 1;
            if (tid == 0) piv[s] = gr;
        }
#pragma unroll
        for (int q = 0; q < R; ++q) {
            const double2 first = P[q][0];
#pragma unroll
            for (int c = 0; c < NB - 1; ++c) P[q][c] = P[q][c + 1];
            P[q][NB - 1] = first;
        }
    }
    __syncthreads();
    double2* Mm = J.Mm + (size_t)(p & 1) * d * NB;
#pragma unroll
    for (int q = 0; q < R; ++q) {
        const int r = tid + q * T;
        if (r < d) {
            double2* row = J.W + (size_t)r * d + j0;
            double2* mrow = Mm + (size_t)r * NB;
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
}

// grid.x = njobs * wg_per_job; workgroup 0 of a job is the panel workgroup.
template <int R>
__global__ __launch_bounds__(kInvThreads)
void inv_step(const InvJob* __restrict__ jobs, int p, int wg_per_job, DevStatus* status) {
    const int job = blockIdx.x / wg_per_job;
    const int w = blockIdx.x - job * wg_per_job;
    const InvJob J = jobs[job];
    if (w == 0) step_panel<R>(J, p, threadIdx.x, status);
    else if (p > 0) step_update<R>(J, p, w - 1, threadIdx.x);
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

hipError_t launch_inv_step(const InvJob* d_jobs, int njobs, int rows_per_thread, int panel, int maxd,
                           DevStatus* status, hipStream_t s) {
    if (njobs <= 0) return hipSuccess;
    const int wg = 1 + (maxd + kUpdCols - 1) / kUpdCols;
    if (rows_per_thread == 1)
        hipLaunchKernelGGL(inv_step<1>, dim3(njobs * wg), dim3(kInvThreads), 0, s, d_jobs, panel, wg, status);
    else
        hipLaunchKernelGGL(inv_step<2>, dim3(njobs * wg), dim3(kInvThreads), 0, s, d_jobs, panel, wg, status);
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
