// Batched inverse of the diagonal Schur blocks, S = Atil_kk^-1 (the
// inverse-instead-of-trsm formulation of Sec. II-B), by blocked Gauss-Jordan
// elimination with partial pivoting inside the block.
//
// The elimination runs on M = A^T: a row-major d x d block read as a
// column-major matrix is its transpose, so the caller's block is the working
// matrix's starting value without a copy, and A^-1 = (M^-1)^T.
//
// Pivoting is implicit: no rows are swapped.  For column j the pivot is the
// not-yet-used row of M of largest |re| + |im| (lowest row index among
// magnitudes equal to 11 mantissa bits); that row is scaled and column j is
// eliminated from every other row.  In place, the slot of column j then
// holds column p_j of the accumulated transform T (T M = Q, Q the
// permutation with Q e_j = e_{p_j}), so at the end, with W the working matrix,
//     M^-1[j][c] = W[p_j][pinv(c)],   A^-1[c][j] = W[p_j][pinv(c)].
//
// Layout: W (d x d) is column-major, element (r, c) at c * d + r.  Every
// kernel below gives each lane its own rows, so a load or store of one column
// by a wave covers 64 consecutive rows (1 KB) instead of 64 scattered pieces.
//
// Blocking: panel p (kInvNB columns) is eliminated by one workgroup that
// holds the panel rows in registers.  The effect of the panel on the other
// columns is T_p = I + Tm Y with
//     Tm[:, s] = (panel column s) - e_{p_s}     (d x NB, read from W)
//     Y[s, :]  = W[p_s, :] outside the panel, 0 inside (NB x d),
// applied in the next panel's launch as W += Tm Y: by the panel workgroup to
// its own block (look-ahead) and by the other workgroups to the rest.
//
// One launch per panel p = 0 .. np (np = ceil(d / NB)):
//   p < np : the panel workgroup applies T_{p-1} to block p and eliminates it;
//            every other column block except p - 1 takes T_{p-1}.
//   p = np : every column block except np - 1 takes T_{np-1}, and all of them
//            are written to the result, transposed and unscrambled.
// Column blocks are read from the caller's block until they are first
// written (block 0 and 1 by the panel workgroup, the others in launch 1).
#include "common.h"
#include "cplx.h"
#include <climits>
#include <type_traits>
#include <utility>

namespace btsq {

constexpr int kUpdCols = 8;    // columns per update workgroup (half a panel block)

// Where column block `blk` of the working matrix lives at the start of launch
// p: the caller's block (read as column-major M) until its first write.
__device__ inline const double2* block_source(const InvJob& J, int blk, int p) {
    const bool written = blk <= 1 ? p > blk : p > 1;
    return written ? J.W : J.src;
}

// Update workgroup u of launch p: its kUpdCols columns take T_{p-1}; in the last
// launch they are also written to the result.  It gathers the pivot rows of
// panel p-1 restricted to its own columns first, so no workgroup reads what
// another writes in the same launch.
template <int T, int R>
__device__ void step_update(const InvJob& J, int p, int u, int tid) {
    constexpr int NB = kInvNB;
    constexpr int UC = kUpdCols;
    __shared__ double2 G[NB][UC];
    __shared__ int prow[NB];
    __shared__ int pinv[kInvMaxDim];
    const int d = J.d;
    const int np = (d + NB - 1) / NB;
    const int c0 = u * UC;
    const int blk = c0 / NB;
    if (c0 >= d || p == 0 || p > np) return;          // no such columns / nothing to apply
    const bool last = p == np;
    if (blk == p) return;                              // the panel workgroup's block
    const bool apply = blk != p - 1;                   // block p-1 is final after launch p-1
    if (!apply && !last) return;                       // nothing to do until the write-out
    const int q0 = (p - 1) * NB;                       // first column of panel p-1
    const int nc = min(NB, d - q0);
    const int ncols = min(UC, d - c0);
    const double2* src = block_source(J, blk, p);
    if (tid < NB) prow[tid] = tid < nc ? J.perm[q0 + tid] : -1;
    if (last) {
        // inverse permutation (cleared first: after a singular pivot the
        // pivot rows need not be a permutation, and every index stays in range)
        for (int e = tid; e < d; e += T) pinv[e] = 0;
        __syncthreads();
        for (int e = tid; e < d; e += T) pinv[J.perm[e]] = e;
    }
    __syncthreads();
    if (apply && tid < NB * UC) {
        const int s = tid / UC, j = tid % UC;
        const int sr = min(s, nc - 1), cc = c0 + min(j, ncols - 1);
        const double2 v = src[(size_t)cc * d + prow[sr]];
        G[s][j] = (s < nc && j < ncols) ? v : make_double2(0.0, 0.0);
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < R; ++q) {
        const int r = tid + q * T;
        if (r >= d) continue;
        double2 acc[UC];
        const double2* wcol = src + (size_t)c0 * d + r;
#pragma unroll
        for (int j = 0; j < UC; ++j) acc[j] = wcol[(size_t)min(j, ncols - 1) * d];
        if (apply) {
            const double2* mcol = J.W + (size_t)q0 * d + r;
#pragma unroll 2
            for (int s = 0; s < NB; s += 4) {
                double2 m[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    m[i] = s + i < nc ? mcol[(size_t)(s + i) * d] : make_double2(0.0, 0.0);
                    if (prow[s + i] == r) m[i].x -= 1.0;
                }
#pragma unroll
                for (int i = 0; i < 4; ++i)
#pragma unroll
                    for (int j = 0; j < UC; ++j) cfma(acc[j], m[i], G[s + i][j]);
            }
        }
        if (!last) {
            double2* wout = J.W + (size_t)c0 * d + r;
#pragma unroll
            for (int j = 0; j < UC; ++j)
                if (j < ncols) wout[(size_t)j * d] = acc[j];
        } else {
            // A^-1[perm[col]][pinv(r)] = W[r][col]
            const int jr = pinv[r];
#pragma unroll
            for (int j = 0; j < UC; ++j)
                if (j < ncols) J.dst[(size_t)J.perm[c0 + j] * d + jr] = acc[j];
        }
    }
}

// Panel workgroup of launch p: applies T_{p-1} to block p (look-ahead) and
// eliminates its columns.  The look-ahead is a run-time loop over the
// transform columns (every register index in it is static); the column loop
// is unrolled, since it indexes the panel registers by column.
template <int T, int R>
__device__ void step_panel(const InvJob& J, int p, int tid, DevStatus* status) {
    constexpr int NB = kInvNB;
    constexpr int NW = T / 64;
    __shared__ unsigned cand_key[2][NW];
    __shared__ double2 cand_ip[2][NW];
    __shared__ double2 cand_row[2][NW][NB];
    __shared__ int piv[NB];
    __shared__ int prev[NB];
    __shared__ double2 G[NB][NB];

    const int d = J.d;
    const int j0 = p * NB;
    if (j0 >= d) return;
    // The panel's column chain is the critical path of the whole inverse and
    // is latency-bound; where product workgroups of the other stream share
    // this CU, their waves would otherwise take most of the issue slots.
    __builtin_amdgcn_s_setprio(3);
    const int nc = min(NB, d - j0);
    const int lane = tid & 63, wave = tid >> 6;
    const double2* src = block_source(J, p, p);

    // this workgroup's rows of block p and their used flags
    double2 P[R][NB];
    int used[R];
#pragma unroll
    for (int q = 0; q < R; ++q) {
        const int r = min(tid + q * T, d - 1);
        const double2* col = src + (size_t)j0 * d + r;
        used[q] = p > 0 ? J.used[r] : 0;
#pragma unroll
        for (int c = 0; c < NB; ++c) P[q][c] = col[(size_t)min(c, nc - 1) * d];
    }
    if (p > 0) {
        const int q0 = (p - 1) * NB;
        const int pnc = min(NB, d - q0);
        const double2* Tm = J.W + (size_t)q0 * d;     // panel p-1 columns, final
        // transform entries of columns 0 and 1, loaded two columns ahead below
        double2 ma[R], mb[R];
#pragma unroll
        for (int q = 0; q < R; ++q) {
            const double2* mcol = Tm + min(tid + q * T, d - 1);
            ma[q] = mcol[0];
            mb[q] = mcol[(size_t)min(1, pnc - 1) * d];
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
        // look-ahead: block p += Tm_{p-1} G, Tm = panel columns minus the
        // unit entries at the pivot rows, one transform column per step
        for (int s = 0; s < pnc; ++s) {
            double2 mc[R];
#pragma unroll
            for (int q = 0; q < R; ++q) {
                const double2* mcol = Tm + min(tid + q * T, d - 1);
                mc[q] = mcol[(size_t)min(s + 2, pnc - 1) * d];
            }
            const int pr = prev[s];
#pragma unroll
            for (int q = 0; q < R; ++q)
                if (pr == tid + q * T) ma[q].x -= 1.0;
#pragma unroll
            for (int c = 0; c < NB; ++c) {
                const double2 g = G[s][c];
#pragma unroll
                for (int q = 0; q < R; ++q) cfma(P[q][c], ma[q], g);
            }
#pragma unroll
            for (int q = 0; q < R; ++q) {
                ma[q] = mb[q];
                mb[q] = mc[q];
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
    unsigned bk, wk;
    double2 bip;
    int bq;
    auto search = [&](auto sc) {
        constexpr int s = decltype(sc)::value;
        bk = 0;
        bq = 0;
        double2 pv = P[0][s];
#pragma unroll
        for (int q = 0; q < R; ++q) {
            const unsigned kq = pivot_key(P[q][s], tid + q * T);
            const unsigned k = used[q] ? 0u : kq;
            const bool take = k > bk;
            bk = take ? k : bk;
            bq = take ? q : bq;
            pv = sel2(take, P[q][s], pv);
        }
        bip = crecip(pv);
        wk = wave_umax(bk);
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
        unsigned gk = cand_key[sb][0];
#pragma unroll
        for (int w = 1; w < NW; ++w) gk = max(gk, cand_key[sb][w]);
        const int gr = gk == 0 ? -1 : key_row(gk);
        const int gw = gk == 0 ? 0 : min((gr % T) >> 6, NW - 1);
        // the winning row's reciprocal pivot and entries, read together
        const double2 ip = cand_ip[sb][gw];
        double2 v[NB];
#pragma unroll
        for (int c = 0; c < NB; ++c) v[c] = cand_row[sb][gw][c];
        bad = bad || gk == 0 || !(fabs(ip.x) + fabs(ip.y) <= DBL_MAX);
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

    // write back block p (rows scaled by sc), the used flags and the pivots
#pragma unroll
    for (int q = 0; q < R; ++q) {
        const int r = tid + q * T;
        if (r < d) {
            double2* col = J.W + (size_t)j0 * d + r;
#pragma unroll
            for (int c = 0; c < NB; ++c)
                if (c < nc) col[(size_t)c * d] = cmul_i(sc[q], P[q][c]);
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
    else {
        // The two 8-column slabs of the next panel's block go to the update
        // workgroups 8 and 16 of the job, whose ids are congruent to the panel
        // workgroup's mod 8 (same XCD, same L2), so the next launch's panel
        // workgroup reads them where they were written.  A bijection of the
        // slab indices: two transpositions.
        int u = w - 1;
        const int nslab = wg_per_job - 1;
        const int a = 2 * (p + 1), b = a + 1;
        if (nslab > 15 && b < nslab) {
            u = u == 7 ? a : u == a ? 7 : u;
            u = u == 15 ? b : u == b ? 15 : u;
        }
        step_update<T, R>(J, p, u, threadIdx.x);
    }
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
// dimension maxd: one launch per panel plus the final one.
hipError_t launch_inverse_sequence(const InvJob* d_jobs, int njobs, int maxd, DevStatus* status,
                                   hipStream_t s) {
    hipError_t e = hipSuccess;
    const int npanels = (maxd + kInvNB - 1) / kInvNB;
    for (int p = 0; p <= npanels && e == hipSuccess; ++p)
        e = launch_inv_step(d_jobs, njobs, inv_variant(maxd), p, maxd, status, s);
    return e;
}

}  // namespace btsq
