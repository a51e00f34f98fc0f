// Grouped complex block products on CDNA4 matrix cores.
//
// Every block update of the forward and backward sweeps is a dense complex
// product (or a short sum of them) on b x b, b x a and a x a blocks.  One
// launch executes a list of independent products, each tiled into 64 x 32
// complex output tiles; a workgroup owns one tile of one product.
//
// Complex arithmetic on real MFMA: a complex m x k matrix A stored as
// interleaved (re, im) doubles is read as the real m x 2k matrix A', and
// op(B) (k x n complex) is expanded on the fly into the real 2k x 2n matrix
//     B''[2p+c][2j+d] = Re B[p][j]  (c == d),  Im B[p][j] (c=0,d=1),
//                       -Im B[p][j] (c=1,d=0)
// so that A' B'' is the interleaved complex product.  The real product has
// 4mnk multiply-adds, the same as four planar real products, and both the
// A operand and the output keep the interleaved storage.
//
// FP64 path: v_mfma_f64_16x16x4f64.  Mixed path: operands rounded to FP32
// while staging into LDS, v_mfma_f32_16x16x4f32 with FP32 accumulation, the
// result added to the FP64 output in FP64.
#include "common.h"

namespace btsq {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

constexpr int kBM = 64;          // complex rows per tile
constexpr int kBN = 32;          // complex columns per tile (64 real)
constexpr int kBK = 16;          // complex k per LDS stage
constexpr int kThreads = 256;    // 4 waves, 2 x 2 over the tile

template <bool MIXED> struct Prec;
// Output layout of one 16 x 16 MFMA block: lane l, accumulator register r
// holds row row_of(l, r), real column l % 16.  Measured on gfx950: the FP64
// instruction interleaves rows (l/16 + 4r), the FP32 one blocks them
// (4(l/16) + r).  Inputs: A[l%16][l/16], B[l/16][l%16] for both.
template <> struct Prec<false> {
    typedef double2 C;
    typedef double R;
    typedef v4d Acc;
    static __device__ inline int row_of(int lane, int r) { return (lane >> 4) + 4 * r; }
    static __device__ inline C cvt(double2 v) { return v; }
    static __device__ inline Acc mfma(R a, R b, Acc c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
};
template <> struct Prec<true> {
    typedef float2 C;
    typedef float R;
    typedef v4f Acc;
    static __device__ inline int row_of(int lane, int r) { return 4 * (lane >> 4) + r; }
    static __device__ inline C cvt(double2 v) { return make_float2((float)v.x, (float)v.y); }
    static __device__ inline Acc mfma(R a, R b, Acc c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
};

__device__ inline double2 cmul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

__device__ inline int find_op(const GemmOp* __restrict__ ops, int nops, int bid) {
    int lo = 0, hi = nops - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (ops[mid].tile_begin <= bid) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Global -> registers for one stage of term T at k offset k0.
__device__ inline void load_stage(const GemmTerm& T, int m, int n, int i0, int j0, int k0,
                                  int tid, double2 ra[4], double2 rb[2]) {
    const bool ah = T.flags & kTermAH;
    const bool bh = T.flags & kTermBH;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int e = tid + kThreads * q;
        const int i = ah ? (e & 63) : (e >> 4);
        const int p = ah ? (e >> 6) : (e & 15);
        const int gi = i0 + i, gp = k0 + p;
        double2 v = make_double2(0.0, 0.0);
        if (gi < m && gp < T.k) {
            if (ah) { v = T.A[(size_t)gp * T.lda + gi]; v.y = -v.y; }
            else    { v = T.A[(size_t)gi * T.lda + gp]; }
        }
        ra[q] = v;
    }
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const int e = tid + kThreads * q;
        const int j = bh ? (e >> 4) : (e & 31);
        const int p = bh ? (e & 15) : (e >> 5);
        const int gj = j0 + j, gp = k0 + p;
        double2 v = make_double2(0.0, 0.0);
        if (gj < n && gp < T.k) {
            if (bh) { v = T.B[(size_t)gj * T.ldb + gp]; v.y = -v.y; }
            else    { v = T.B[(size_t)gp * T.ldb + gj]; }
        }
        rb[q] = cmul(T.alpha, v);
    }
}

template <bool MIXED>
__device__ inline void store_stage(bool ah, bool bh, int tid, const double2 ra[4], const double2 rb[2],
                                   typename Prec<MIXED>::C (*As)[kBM + 1],
                                   typename Prec<MIXED>::C (*Bs)[kBN + 1]) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int e = tid + kThreads * q;
        const int i = ah ? (e & 63) : (e >> 4);
        const int p = ah ? (e >> 6) : (e & 15);
        As[p][i] = Prec<MIXED>::cvt(ra[q]);
    }
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const int e = tid + kThreads * q;
        const int j = bh ? (e >> 4) : (e & 31);
        const int p = bh ? (e & 15) : (e >> 5);
        Bs[p][j] = Prec<MIXED>::cvt(rb[q]);
    }
}

template <bool MIXED>
__global__ __launch_bounds__(kThreads)
void zgemm_grouped(const GemmOp* __restrict__ ops, int nops) {
    typedef typename Prec<MIXED>::C CT;
    typedef typename Prec<MIXED>::R RT;
    typedef typename Prec<MIXED>::Acc AccT;
    __shared__ CT As[2][kBK][kBM + 1];
    __shared__ CT Bs[2][kBK][kBN + 1];

    const int bid = blockIdx.x;
    const GemmOp* op = ops + find_op(ops, nops, bid);
    const int m = op->m, n = op->n, nterms = op->nterms;
    const int local = bid - op->tile_begin;
    const int tm = local / op->tiles_n, tn = local - tm * op->tiles_n;
    const int i0 = tm * kBM, j0 = tn * kBN;

    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int wm = wave & 1, wn = wave >> 1;
    const int cA = (lane >> 4) & 1;   // real k within the pair: 0 = re part of A, 1 = im part
    const int pOff = lane >> 5;       // complex k offset within the 4-wide real k step
    const int r16 = lane & 15;
    const int d = lane & 1;           // output component of this lane's B'' column

    AccT acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
            acc[a][b] = AccT{0, 0, 0, 0};

    int t = 0, k0 = 0;
    while (t < nterms && op->t[t].k <= 0) ++t;
    double2 ra[4], rb[2];
    int buf = 0;
    if (t < nterms) {
        load_stage(op->t[t], m, n, i0, j0, k0, tid, ra, rb);
        store_stage<MIXED>(op->t[t].flags & kTermAH, op->t[t].flags & kTermBH, tid, ra, rb, As[0], Bs[0]);
    }
    __syncthreads();
    while (t < nterms) {
        int tn2 = t, kn = k0 + kBK;
        while (tn2 < nterms && kn >= op->t[tn2].k) { ++tn2; kn = 0; }
        const bool has_next = tn2 < nterms;
        if (has_next) load_stage(op->t[tn2], m, n, i0, j0, kn, tid, ra, rb);

#pragma unroll
        for (int kk = 0; kk < kBK / 2; ++kk) {
            const int p = 2 * kk + pOff;
            RT av[2], bv[2];
#pragma unroll
            for (int mi = 0; mi < 2; ++mi) {
                const CT x = As[buf][p][wm * 32 + mi * 16 + r16];
                av[mi] = cA ? x.y : x.x;
            }
#pragma unroll
            for (int ni = 0; ni < 2; ++ni) {
                const int jc = (wn * 32 + ni * 16 + r16) >> 1;
                const CT x = Bs[buf][p][jc];
                RT v = (cA == d) ? x.x : x.y;
                bv[ni] = (cA == 1 && d == 0) ? -v : v;
            }
#pragma unroll
            for (int mi = 0; mi < 2; ++mi)
#pragma unroll
                for (int ni = 0; ni < 2; ++ni)
                    acc[mi][ni] = Prec<MIXED>::mfma(av[mi], bv[ni], acc[mi][ni]);
        }
        if (has_next)
            store_stage<MIXED>(op->t[tn2].flags & kTermAH, op->t[tn2].flags & kTermBH, tid, ra, rb,
                               As[buf ^ 1], Bs[buf ^ 1]);
        __syncthreads();
        buf ^= 1;
        t = tn2;
        k0 = kn;
    }

    // Epilogue: lane holds rows row_of(lane, r) of each 16 x 16 real block, real column lane%16.
    double* D = reinterpret_cast<double*>(op->D);
    const double2* C = op->C;
    const int ldd = op->ldd, ldc = op->ldc;
    const double2 beta = op->beta;
#pragma unroll
    for (int mi = 0; mi < 2; ++mi)
#pragma unroll
        for (int ni = 0; ni < 2; ++ni)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = i0 + wm * 32 + mi * 16 + Prec<MIXED>::row_of(lane, r);
                const int jr = wn * 32 + ni * 16 + r16;
                const int col = j0 + (jr >> 1);
                const int comp = jr & 1;
                if (row < m && col < n) {
                    double v = (double)acc[mi][ni][r];
                    if (C) {
                        const double2 c = C[(size_t)row * ldc + col];
                        v += comp ? (beta.x * c.y + beta.y * c.x) : (beta.x * c.x - beta.y * c.y);
                    }
                    D[2 * ((size_t)row * ldd + col) + comp] = v;
                }
            }
}

int gemm_tiles(int m, int n) {
    return ((m + kBM - 1) / kBM) * ((n + kBN - 1) / kBN);
}
int gemm_tiles_n(int n) { return (n + kBN - 1) / kBN; }

hipError_t launch_gemm(const GemmOp* d_ops, int nops, int total_tiles, bool mixed, hipStream_t s) {
    if (nops <= 0 || total_tiles <= 0) return hipSuccess;
    if (mixed)
        hipLaunchKernelGGL(zgemm_grouped<true>, dim3(total_tiles), dim3(kThreads), 0, s, d_ops, nops);
    else
        hipLaunchKernelGGL(zgemm_grouped<false>, dim3(total_tiles), dim3(kThreads), 0, s, d_ops, nops);
    return hipGetLastError();
}

}  // namespace btsq
