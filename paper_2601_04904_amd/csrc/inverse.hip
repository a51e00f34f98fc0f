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
// Layout: the working matrix W (d x d) and the panel transforms Mm (d x NB)
// are stored column-major, element (r, c) at c * d + r.  Every kernel below
// gives each lane its own rows, so a load or store of one column by a wave
// covers 64 consecutive rows (1 KB) instead of 64 scattered pieces.
//
// Blocking: a panel of kInvNB columns is eliminated by one workgroup that
// holds the panel rows in registers (one barrier per column: the best
// candidate of every wave publishes its row and the reciprocal of its pivot
// entry, every thread then picks the winner and updates its rows).  The
// effect of the panel on the other columns is M_J = I + Mm Y, where
//     Mm[:, s] = (panel column s) - e_{p_s}   (d x NB)
//     Y[s, :]  = W[p_s, :] outside the panel, 0 inside (NB x d),
// applied in the next panel's launch as W += Mm Y: by the panel workgroup to
// its own block (look-ahead) and by the other workgroups to the rest.
#include "common.h"
#include <cfloat>
#include <climits>
#include <type_traits>
#include <utility>

namespace btsq {

__device__ inline double2 cmul_i(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// c ? a : b on values (a conditional over two double2 lvalues would select
// an address and keep the register arrays it points into out of registers)
__device__ inline double2 sel2(bool c, double2 a, double2 b) {
    return make_double2(c ? a.x : b.x, c ? a.y : b.y);
}

// acc += a b and acc -= a b, four fused multiply-adds each
__device__ inline void cfma(double2& acc, double2 a, double2 b) {
    acc.x = fma(a.x, b.x, acc.x);
    acc.x = fma(-a.y, b.y, acc.x);
    acc.y = fma(a.x, b.y, acc.y);
    acc.y = fma(a.y, b.x, acc.y);
}

__device__ inline void cfms(double2& acc, double2 a, double2 b) {
    acc.x = fma(-a.x, b.x, acc.x);
    acc.x = fma(a.y, b.y, acc.x);
    acc.y = fma(-a.x, b.y, acc.y);
    acc.y = fma(-a.y, b.x, acc.y);
}

// 1 / v = conj(v) / |v|^2, with v first scaled by a power of two so that
// |v|^2 neither overflows nor underflows (one division).  A zero, infinite
// or NaN v gives a non-finite or zero result, which the caller flags.
__device__ inline double2 crecip(double2 v) {
    int e;
    (void)frexp(fmax(fabs(v.x), fabs(v.y)), &e);
    const double a = ldexp(v.x, -e), b = ldexp(v.y, -e);
    const double inv = 1.0 / (a * a + b * b);
    return make_double2(ldexp(a * inv, -e), ldexp(-b * inv, -e));
}

// Maximum of a 32-bit value over the 64 lanes of a wave: DPP steps within
// rows of 16 lanes, then row broadcasts, after which lane 63 holds the
// maximum; it is returned to every lane.  Lanes that a broadcast does not
// reach take 0, the identity of the maximum, so each step is one max with a
// DPP operand.  The whole wave must be active.
template <int CTRL, int ROW_MASK>
__device__ inline unsigned dpp_umax(unsigned x) {
    return max(x, (unsigned)__builtin_amdgcn_update_dpp(0, (int)x, CTRL, ROW_MASK, 0xf, false));
}

__device__ inline unsigned wave_umax(unsigned x) {
    x = dpp_umax<0xB1, 0xf>(x);    // quad_perm [1,0,3,2]
    x = dpp_umax<0x4E, 0xf>(x);    // quad_perm [2,3,0,1]
    x = dpp_umax<0x124, 0xf>(x);   // row_ror:4
    x = dpp_umax<0x128, 0xf>(x);   // row_ror:8  -> every lane holds its row's maximum
    x = dpp_umax<0x142, 0xa>(x);   // row_bcast:15 into rows 1 and 3
    x = dpp_umax<0x143, 0xc>(x);   // row_bcast:31 into rows 2 and 3 -> lane 63 holds it
    return (unsigned)__builtin_amdgcn_readlane((int)x, 63);
}

// Maximum of a 64-bit key over the wave: the high words first, then the low
// words of the lanes whose high word is that maximum.
__device__ inline unsigned long long wave_max_key(unsigned long long k) {
    const unsigned hi = (unsigned)(k >> 32);
    const unsigned h = wave_umax(hi);
    const unsigned l = wave_umax(hi == h ? (unsigned)k : 0u);
    return ((unsigned long long)h << 32) | l;
}

// Pivot key: the bit pattern of |re| + |im| of the candidate (non-finite
// values clamped to the largest finite double) with the 11 low mantissa bits
// replaced by 2047 - row.  Non-negative doubles order like their bit
// patterns, so the largest key is the largest magnitude (to 41 mantissa bits)
// and, among magnitudes equal to that precision, the lowest row.  Every
// candidate row is below 1024, so a candidate's key is at least 1024 and 0
// means "no candidate".
__device__ inline unsigned long long pivot_key(double2 v, int row) {
    double m = fabs(v.x) + fabs(v.y);
    if (!(m <= DBL_MAX)) m = DBL_MAX;
    return ((unsigned long long)__double_as_longlong(m) & ~2047ull) | (unsigned long long)(2047 - row);
}

__device__ inline int key_row(unsigned long long key) {
    return 2047 - (int)(key & 2047ull);
}

// W = src transposed into the column-major working layout, through 16 x 16
// LDS tiles so that both the row-major reads and the column-major writes are
// contiguous across threads.  256 threads per workgroup.
__global__ void inv_init(const InvJob* __restrict__ jobs) {
    __shared__ double2 tile[16][17];
    const InvJob J = jobs[blockIdx.y];
    const int d = J.d;
    const int nt = (d + 15) / 16;
    const int tid = threadIdx.x;
    const int a = tid >> 4, b = tid & 15;
    for (int t = blockIdx.x; t < nt * nt; t += gridDim.x) {
        const int ti = t / nt, tj = t - ti * nt;
        const int r = ti * 16 + a, c = tj * 16 + b;
        if (r < d && c < d) tile[a][b] = J.src[(size_t)r * d + c];
        __syncthreads();
        const int c2 = tj * 16 + a, r2 = ti * 16 + b;
        if (r2 < d && c2 < d) J.W[(size_t)c2 * d + r2] = tile[b][a];
        __syncthreads();
    }
    for (int e = blockIdx.x * blockDim.x + tid; e < d; e += gridDim.x * blockDim.x) J.used[e] = 0;
}

// One launch per panel p.  Per matrix, workgroup 0 (the panel workgroup)
// applies the transform of panel p-1 to block p (look-ahead) and then
// eliminates block p; workgroups 1.. apply the transform of panel p-1 to the
// other 8-column blocks (all but blocks p-1 and p), each first gathering the
// pivot rows of its own columns, so no workgroup reads what another writes.
// Mm is double-buffered by panel parity (Mm + (p % 2) * d * NB).
constexpr int kUpdCols = 8;

template <int T, int R>
__device__ void step_update(const InvJob& J, int p, int u, int tid) {
    constexpr int NB = kInvNB;
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
        const double2 v = J.W[(size_t)cc * d + J.perm[q0 + sr]];
        G[s][j] = (s < nc && c0 + j < d) ? v : make_double2(0.0, 0.0);
    }
    __syncthreads();
    const int ncols = min(UC, d - c0);
#pragma unroll
    for (int q = 0; q < R; ++q) {
        const int r = tid + q * T;
        if (r >= d) continue;
        double2 acc[UC];
        const double2* wcol = J.W + (size_t)c0 * d + r;
        const double2* mcol = Mm + r;
#pragma unroll
        for (int j = 0; j < UC; ++j) acc[j] = wcol[(size_t)min(j, ncols - 1) * d];
#pragma unroll 2
        for (int s = 0; s < NB; s += 4) {
            double2 m[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) m[i] = mcol[(size_t)(s + i) * d];
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < UC; ++j) {
                    cfma(acc[j], m[i], G[s + i][j]);
                }
        }
        double2* wout = J.W + (size_t)c0 * d + r;
#pragma unroll
        for (int j = 0; j < UC; ++j)
            if (j < ncols) wout[(size_t)j * d] = acc[j];
    }
}

template <int T, int R>
__device__ void step_panel(const InvJob& J, int p, int tid, DevStatus* status) {
    constexpr int NB = kInvNB;
    constexpr int NW = T / 64;
    __shared__ unsigned long long cand_key[2][NW];
    __shared__ double2 cand_ip[2][NW];
    __shared__ double2 cand_row[2][NW][NB];
    __shared__ int piv[NB];
    __shared__ int prev[NB];
    __shared__ double2 G[NB][NB];

    const int d = J.d;
    const int j0 = p * NB;
    if (j0 >= d) return;
    // the panel is the critical path of the launch: its waves win instruction
    // issue over the update workgroups and other kernels' waves on the CU
    __builtin_amdgcn_s_setprio(3);
    const int nc = min(NB, d - j0);
    const int lane = tid & 63, wave = tid >> 6;

    // All global reads are issued here, before any wait: this workgroup's rows
    // of block p, their used flags, their rows of the panel p-1 transform and
    // the pivot rows of panel p-1.
    double2 P[R][NB];
    int used[R];
#pragma unroll
    for (int q = 0; q < R; ++q) {
        const int r = min(tid + q * T, d - 1);
        const double2* col = J.W + (size_t)j0 * d + r;
        used[q] = J.used[r];
#pragma unroll
        for (int c = 0; c < NB; ++c) P[q][c] = col[(size_t)min(c, nc - 1) * d];
    }
    if (p > 0) {
        const int q0 = (p - 1) * NB;
        const int pnc = min(NB, d - q0);
        constexpr int MG = R == 1 ? NB : 4;          // transform entries held at once
        const double2* Mm = J.Mm + (size_t)((p - 1) & 1) * d * NB;
        double2 m[R][MG];
#pragma unroll
        for (int q = 0; q < R; ++q) {
            const double2* mcol = Mm + min(tid + q * T, d - 1);
#pragma unroll
            for (int i = 0; i < MG; ++i) m[q][i] = mcol[(size_t)i * d];
        }
        if (tid < NB) prev[tid] = tid < pnc ? J.perm[q0 + tid] : -1;
        if (tid < NB && tid >= pnc) {
#pragma unroll
            for (int c = 0; c < NB; ++c) G[tid][c] = make_double2(0.0, 0.0);
        }
        __syncthreads();
        // The pivot rows of panel p-1 restricted to block p (not yet
        // transformed) come from the threads that hold them.  Columns past nc
        // of G only reach columns of P that are cleared below.
#pragma unroll
        for (int q = 0; q < R; ++q) {
            const int r = tid + q * T;
            int sm = -1;
#pragma unroll
            for (int s = 0; s < NB; ++s) sm = prev[s] == r ? s : sm;
            if (sm >= 0 && r < d) {
#pragma unroll
                for (int c = 0; c < NB; ++c) G[sm][c] = P[q][c];
            }
        }
        __syncthreads();
        // look-ahead: block p += Mm_{p-1} G
#pragma unroll
        for (int s0 = 0; s0 < NB; s0 += MG) {
            if (s0 > 0) {
#pragma unroll
                for (int q = 0; q < R; ++q) {
                    const double2* mcol = Mm + min(tid + q * T, d - 1);
#pragma unroll
                    for (int i = 0; i < MG; ++i) m[q][i] = mcol[(size_t)(s0 + i) * d];
                }
            }
#pragma unroll
            for (int i = 0; i < MG; ++i)
#pragma unroll
                for (int c = 0; c < NB; ++c) {
                    const double2 g = G[s0 + i][c];
#pragma unroll
                    for (int q = 0; q < R; ++q) cfma(P[q][c], m[q][i], g);
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

    // Candidate of this lane for column s (largest key over its unused rows),
    // the wave maximum, and publication by the lane that holds it: the key,
    // the reciprocal of its pivot entry and its whole row.  Written with
    // selects rather than branches, so that the search of a column and the
    // row updates around it form one block the compiler can interleave.
    unsigned long long bk, wk;
    double2 bip;
    int bq;
    auto search = [&](auto sc) {
        constexpr int s = decltype(sc)::value;
        bk = 0;
        bq = 0;
        double2 pv = P[0][s];
#pragma unroll
        for (int q = 0; q < R; ++q) {
            const unsigned long long kq = pivot_key(P[q][s], tid + q * T);
            const unsigned long long k = used[q] ? 0ull : kq;
            const bool take = k > bk;
            bk = take ? k : bk;
            bq = take ? q : bq;
            pv = sel2(take, P[q][s], pv);
        }
        bip = crecip(pv);
        wk = wave_max_key(bk);
    };
    auto publish = [&](int sb) {
        if (wk == 0) {
            if (lane == 0) cand_key[sb][wave] = 0;
        } else if (bk == wk) {
            cand_key[sb][wave] = wk;
            cand_ip[sb][wave] = bip;
#pragma unroll
            for (int q = 0; q < R; ++q)
                if (q == bq) {
#pragma unroll
                    for (int c = 0; c < NB; ++c) cand_row[sb][wave][c] = P[q][c];
                }
        }
    };
    search(std::integral_constant<int, 0>{});
    publish(0);

    // Column loop, fully unrolled so that every register index is static.
    // Column s + 1 is updated first, so that its pivot search and reciprocal
    // overlap the update of the other columns.  Past the last column of a
    // partial panel every entry is zero, so the update and search of column
    // s + 1 run unconditionally (their result is not used there).
    //
    // Pivot rows are not rescaled when they are chosen: every row is kept as
    // sc * U, with U in registers and sc = 1 until the row becomes a pivot row,
    // sc = 1 / pivot afterwards.  In U the update of any later column is then
    // the same formula for every row (U -= (U[s] / pivot) v), the pivot row of
    // column s only gets U[s] = 1 and skips the update of that column, and the
    // scale is applied once, at write-back.
    double2 sc[R];
#pragma unroll
    for (int q = 0; q < R; ++q) sc[q] = make_double2(1.0, 0.0);
    bool bad = false;
    auto column = [&](auto scst) {
        constexpr int s = decltype(scst)::value;
        constexpr int sb = s & 1;
        if (s >= nc) return;
        __syncthreads();
        unsigned long long gk = cand_key[sb][0];
#pragma unroll
        for (int w = 1; w < NW; ++w) {
            const unsigned long long k = cand_key[sb][w];
            gk = k > gk ? k : gk;
        }
        const int gr = gk == 0 ? -1 : key_row(gk);
        const int gw = gk == 0 ? 0 : min((gr % T) >> 6, NW - 1);
        // the winning row's reciprocal pivot and entries, read together
        const double2 ip = cand_ip[sb][gw];
        double2 v[NB];
#pragma unroll
        for (int c = 0; c < NB; ++c) v[c] = cand_row[sb][gw][c];
        bad = bad || gk == 0 || !(fabs(ip.x) + fabs(ip.y) <= DBL_MAX) || (ip.x == 0.0 && ip.y == 0.0);
        double2 g[R];
        bool pr[R];
#pragma unroll
        for (int q = 0; q < R; ++q) {
            pr[q] = tid + q * T == gr;
            const double2 t = cmul_i(P[q][s], ip);
            g[q] = sel2(pr[q], make_double2(0.0, 0.0), t);
            used[q] = pr[q] ? 1 : used[q];
            sc[q] = sel2(pr[q], ip, sc[q]);
        }
        // every other row: U -= (U[s] / pivot) * pivot row, column s + 1 first
        if constexpr (s + 1 < NB) {
#pragma unroll
            for (int q = 0; q < R; ++q) cfms(P[q][s + 1], g[q], v[s + 1]);
            search(std::integral_constant<int, s + 1>{});
        }
#pragma unroll
        for (int c = 0; c < NB; ++c) {
            if (c == s || c == s + 1) continue;
#pragma unroll
            for (int q = 0; q < R; ++q) cfms(P[q][c], g[q], v[c]);
        }
        // the pivot column slot takes -U[s] / pivot, or 1 in the pivot row
#pragma unroll
        for (int q = 0; q < R; ++q)
            P[q][s] = sel2(pr[q], make_double2(1.0, 0.0), make_double2(-g[q].x, -g[q].y));
        if (tid == 0) piv[s] = gr < 0 ? 0 : gr;
        if (s + 1 < nc) publish(sb ^ 1);
    };
    [&]<int... S>(std::integer_sequence<int, S...>) {
        (column(std::integral_constant<int, S>{}), ...);
    }(std::make_integer_sequence<int, NB>{});
    if (bad && tid == 0 && atomicCAS(&status->code, 0, 3) == 0) status->tag = J.tag;
    __syncthreads();

    // write back block p (rows scaled by sc) and Mm_p = block p minus the
    // pivot unit entries
    double2* Mm = J.Mm + (size_t)(p & 1) * d * NB;
#pragma unroll
    for (int q = 0; q < R; ++q) {
        const int r = tid + q * T;
        if (r < d) {
            double2* col = J.W + (size_t)j0 * d + r;
            double2* mcol = Mm + r;
#pragma unroll
            for (int c = 0; c < NB; ++c) {
                if (c < nc) {
                    double2 v = cmul_i(sc[q], P[q][c]);
                    col[(size_t)c * d] = v;
                    if (piv[c] == r) v.x -= 1.0;
                    mcol[(size_t)c * d] = v;
                } else {
                    mcol[(size_t)c * d] = make_double2(0.0, 0.0);
                }
            }
            J.used[r] = used[q];
        }
    }
    if (tid < nc) J.perm[j0 + tid] = piv[tid];
}

// grid.x = njobs * wg_per_job; workgroup 0 of a job is the panel workgroup.
template <int T, int R>
__global__ __launch_bounds__(T)
void inv_step(const InvJob* __restrict__ jobs, int p, int wg_per_job, DevStatus* status) {
    const int job = blockIdx.x / wg_per_job;
    const int w = blockIdx.x - job * wg_per_job;
    const InvJob J = jobs[job];
    if (w == 0) step_panel<T, R>(J, p, threadIdx.x, status);
    else if (p > 0) step_update<T, R>(J, p, w - 1, threadIdx.x);
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
        const double2* src = J.W + perm[j];           // row perm[j] of the column-major W
        double2* dst = J.dst + (size_t)j * d;
        for (int c = threadIdx.x; c < d; c += blockDim.x) dst[c] = src[(size_t)pinv[c] * d];
    }
}

hipError_t launch_inv_finish(const InvJob* d_jobs, int njobs, int maxd, hipStream_t s);

hipError_t launch_inv_init(const InvJob* d_jobs, int njobs, int maxd, hipStream_t s) {
    if (njobs <= 0) return hipSuccess;
    int chunks = (int)(((size_t)maxd * maxd + 255) / 256);
    if (chunks > 64) chunks = 64;
    if (chunks < 1) chunks = 1;
    hipLaunchKernelGGL(inv_init, dim3(chunks, njobs), dim3(256), 0, s, d_jobs);
    return hipGetLastError();
}

int inv_variant(int d) { return d <= 256 ? 0 : d <= 512 ? 1 : 2; }

hipError_t launch_inv_step(const InvJob* d_jobs, int njobs, int variant, int panel, int maxd,
                           DevStatus* status, hipStream_t s) {
    if (njobs <= 0) return hipSuccess;
    const int wg = 1 + (maxd + kUpdCols - 1) / kUpdCols;
    switch (variant) {
        case 0: hipLaunchKernelGGL((inv_step<256, 1>), dim3(njobs * wg), dim3(256), 0, s, d_jobs, panel, wg, status); break;
        case 1: hipLaunchKernelGGL((inv_step<256, 2>), dim3(njobs * wg), dim3(256), 0, s, d_jobs, panel, wg, status); break;
        default: hipLaunchKernelGGL((inv_step<512, 2>), dim3(njobs * wg), dim3(512), 0, s, d_jobs, panel, wg, status); break;
    }
    return hipGetLastError();
}

// The whole inverse of njobs matrices that all use the panel kernel shape of
// dimension maxd: working copy, every panel launch, unscramble.
hipError_t launch_inverse_sequence(const InvJob* d_jobs, int njobs, int maxd, DevStatus* status,
                                   hipStream_t s) {
    hipError_t e = launch_inv_init(d_jobs, njobs, maxd, s);
    const int npanels = (maxd + kInvNB - 1) / kInvNB;
    for (int p = 0; p <= npanels && e == hipSuccess; ++p)
        e = launch_inv_step(d_jobs, njobs, inv_variant(maxd), p, maxd, status, s);
    if (e == hipSuccess) e = launch_inv_finish(d_jobs, njobs, maxd, s);
    return e;
}

hipError_t launch_inv_finish(const InvJob* d_jobs, int njobs, int maxd, hipStream_t s) {
    if (njobs <= 0) return hipSuccess;
    int rows = maxd < 64 ? maxd : 64;
    if (rows < 1) rows = 1;
    hipLaunchKernelGGL(inv_finish, dim3(rows, njobs), dim3(256), 0, s, d_jobs);
    return hipGetLastError();
}

}  // namespace btsq
