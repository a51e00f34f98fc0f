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
// FP64 path: v_mfma_f64_4x4x4f64 (measured on gfx950 at about 1.6x the
// throughput of the 16x16x4 FP64 shape).  Mixed path: operands rounded to
// FP32 while staging into LDS, v_mfma_f32_16x16x4f32 with FP32 accumulation,
// the result added to the FP64 output in FP64.
#include "common.h"
#include <type_traits>

namespace btsq {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

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
    typedef double Acc;
    static constexpr int NR = 1;   // accumulator values per lane per MFMA
    // row within the 4-row group of lane, accumulator element r
    static __device__ inline int row_of(int lane, int r) { return lane >> 4; }
    static __device__ inline double elem(const Acc& a, int r) { return a; }
    static __device__ inline C cvt(double2 v) { return v; }
    static __device__ inline R flip(R v, bool neg) {
        return __longlong_as_double(__double_as_longlong(v) ^ (neg ? (long long)0x8000000000000000ull : 0ll));
    }
    static __device__ inline Acc mfma(R a, R b, Acc c) {
        return __builtin_amdgcn_mfma_f64_4x4x4f64(a, b, c, 0, 0, 0);
    }
};
template <> struct Prec<true> {
    typedef float2 C;
    typedef float R;
    typedef v4f Acc;
    static constexpr int NR = 4;
    // row within the 16-row block of lane, accumulator element r
    static __device__ inline int row_of(int lane, int r) { return 4 * (lane >> 4) + r; }
    static __device__ inline double elem(const Acc& a, int r) { return (double)a[r]; }
    static __device__ inline C cvt(double2 v) { return make_float2((float)v.x, (float)v.y); }
    static __device__ inline R flip(R v, bool neg) {
        return __int_as_float(__float_as_int(v) ^ (neg ? (int)0x80000000u : 0));
    }
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

// Global pointer in the global address space (the C operand's loads).
#ifdef __HIP_DEVICE_COMPILE__
typedef const __attribute__((address_space(1))) double2* gptr_t;
#else
typedef const double2* gptr_t;
#endif

// Operand loads go through raw buffer resources, one per operand of the
// current term: a lane's load address is base + its own 32-bit byte offset +
// a wave-uniform scalar offset for the stage's k.  A lane whose row, column
// or k lies outside the operand gets the offset kOOB instead; the record
// count of every resource (the operand's extent in bytes, below 2^31) is
// smaller than that, so the hardware returns zeros for it without accessing
// memory.  For every other lane the byte offset plus the scalar offset stays
// inside the operand, so no access leaves it whether or not the hardware's
// range check counts the scalar offset.
constexpr unsigned kOOB = 0x80000000u;
constexpr int kRsrcWord3 = 0x00020000;   // raw buffer, 32-bit data format

__device__ inline __amdgpu_buffer_rsrc_t operand_rsrc(const double2* base, int rows, int cols, int ld) {
    const int extent = ((rows - 1) * ld + cols) * 16;
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<double2*>(base), (short)0, extent, kRsrcWord3);
}

__device__ inline double2 load_b128(__amdgpu_buffer_rsrc_t r, unsigned voff, int soff) {
    return __builtin_bit_cast(double2, __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0));
}

// What a stage's operands need between load and LDS: conjugation of A and
// B, and alpha (folded into B).  Taken from the term, so wave-uniform.
struct StageFlags {
    bool ah, bh;
    int akind;            // alpha: 0 general, 1 exactly +1, 2 exactly -1
    double2 alpha;
};

// Addressing of one thread's loads for one product term, fixed over all k
// stages of the term: the byte offset of each load at k = 0 (kOOB when its
// A row or B column lies outside the matrix) and the bytes per unit of k.
// The term's flags, k and alpha come from the op list in global memory at a
// uniform address, so they are wave-uniform and the choices on them are
// scalar.
template <int BM, int BN>
struct TermAddr {
    static constexpr int NA = BM * kBK / kThreads;
    static constexpr int NB = BN * kBK / kThreads;
    __amdgpu_buffer_rsrc_t ra, rb;
    unsigned va[NA];
    unsigned vb[NB];
    int ska, skb;
    int km1;
    StageFlags f;
};

// Coordinates of load e (= tid + kThreads q) inside the stage tile: A (i, p)
// and B (j, p), chosen so that consecutive threads read consecutive memory.
template <int BM> __device__ inline int a_i(bool ah, int e) { return ah ? (e % BM) : (e / kBK); }
template <int BM> __device__ inline int a_p(bool ah, int e) { return ah ? (e / BM) : (e % kBK); }
template <int BN> __device__ inline int b_j(bool bh, int e) { return bh ? (e / kBK) : (e % BN); }
template <int BN> __device__ inline int b_p(bool bh, int e) { return bh ? (e % kBK) : (e / BN); }

// op(A) is m x k: stored k x m (A^H) or m x k; op(B) is k x n: stored n x k
// (B^H) or k x n.  Element (i, p) of op(A) sits at p lda + i or i lda + p,
// element (p, j) of op(B) at j ldb + p or p ldb + j.
template <int BM, int BN>
__device__ inline void term_setup(const GemmTerm& T, int m, int n, int i0, int j0, int tid,
                                  TermAddr<BM, BN>& ta) {
    const bool ah = T.flags & kTermAH, bh = T.flags & kTermBH;
    ta.f.ah = ah;
    ta.f.bh = bh;
    ta.f.alpha = T.alpha;
    ta.f.akind = T.alpha.y != 0.0 ? 0 : T.alpha.x == 1.0 ? 1 : T.alpha.x == -1.0 ? 2 : 0;
    ta.km1 = T.k - 1;
    ta.ska = (ah ? T.lda : 1) * 16;
    ta.skb = (bh ? 1 : T.ldb) * 16;
    ta.ra = ah ? operand_rsrc(T.A, T.k, m, T.lda) : operand_rsrc(T.A, m, T.k, T.lda);
    ta.rb = bh ? operand_rsrc(T.B, n, T.k, T.ldb) : operand_rsrc(T.B, T.k, n, T.ldb);
#pragma unroll
    for (int q = 0; q < ta.NA; ++q) {
        const int e = tid + kThreads * q;
        const int gi = i0 + a_i<BM>(ah, e);
        const unsigned off = (unsigned)((ah ? gi : gi * T.lda) * 16 + a_p<BM>(ah, e) * ta.ska);
        ta.va[q] = gi < m ? off : kOOB;
    }
#pragma unroll
    for (int q = 0; q < ta.NB; ++q) {
        const int e = tid + kThreads * q;
        const int gj = j0 + b_j<BN>(bh, e);
        const unsigned off = (unsigned)((bh ? gj * T.ldb : gj) * 16 + b_p<BN>(bh, e) * ta.skb);
        ta.vb[q] = gj < n ? off : kOOB;
    }
}

// Raw operands of one stage in flight.
template <int BM, int BN>
struct Stage {
    double2 ra[BM * kBK / kThreads];
    double2 rb[BN * kBK / kThreads];
};

// Issue the global loads of one stage at k offset k0, all before any is
// waited on, so that they overlap the MFMAs of the current stage.  Only the
// last stage of a term whose k is not a multiple of the stage depth has
// lanes past k; they are switched to kOOB.  With live false every lane is
// switched to kOOB: the register set is then defined (all zeros) without
// any memory access, so the caller can issue unconditionally and the
// compiler never has to keep a register set's old and new values at once.
template <int BM, int BN>
__device__ inline void issue_stage(const TermAddr<BM, BN>& ta, int k0, int tid, Stage<BM, BN>& st,
                                   bool live = true) {
    constexpr int NA = BM * kBK / kThreads;
    constexpr int NB = BN * kBK / kThreads;
    const int lim = live ? ta.km1 - k0 : -1;   // largest k offset inside the term
    // wave-uniform by construction; readfirstlane lets the compiler keep them in SGPRs
    const int soa = __builtin_amdgcn_readfirstlane(live ? k0 * ta.ska : 0);
    const int sob = __builtin_amdgcn_readfirstlane(live ? k0 * ta.skb : 0);
    // A lane past k gets the top bit set: lim - p < 0 exactly then, and every
    // in-range offset is below 2^31, so the result is at least kOOB.  Plain
    // arithmetic rather than a choice, so the issue is straight-line code.
#pragma unroll
    for (int q = 0; q < NA; ++q) {
        const unsigned past = (unsigned)(lim - a_p<BM>(ta.f.ah, tid + kThreads * q)) & kOOB;
        st.ra[q] = load_b128(ta.ra, ta.va[q] | past, soa);
    }
#pragma unroll
    for (int q = 0; q < NB; ++q) {
        const unsigned past = (unsigned)(lim - b_p<BN>(ta.f.bh, tid + kThreads * q)) & kOOB;
        st.rb[q] = load_b128(ta.rb, ta.vb[q] | past, sob);
    }
}

// Conjugate and scale by alpha (out-of-range values are already zero).
// Conjugation and alpha = -1 are sign flips with wave-uniform masks, so the
// common case has no branch; only a general alpha takes the complex product.
__device__ inline double flip_sign(double v, unsigned long long mask) {
    return __longlong_as_double(__double_as_longlong(v) ^ (long long)mask);
}

template <int BM, int BN>
__device__ inline void finish_stage(const StageFlags& f, Stage<BM, BN>& st) {
    constexpr int NA = BM * kBK / kThreads;
    constexpr int NB = BN * kBK / kThreads;
    constexpr unsigned long long kSign = 0x8000000000000000ull;
    const bool neg = f.akind == 2;
    const unsigned long long ma = f.ah ? kSign : 0ull;             // Im A
    const unsigned long long mbx = neg ? kSign : 0ull;             // Re B
    const unsigned long long mby = f.bh != neg ? kSign : 0ull;     // Im B
#pragma unroll
    for (int q = 0; q < NA; ++q) st.ra[q].y = flip_sign(st.ra[q].y, ma);
#pragma unroll
    for (int q = 0; q < NB; ++q) {
        st.rb[q].x = flip_sign(st.rb[q].x, mbx);
        st.rb[q].y = flip_sign(st.rb[q].y, mby);
    }
    if (f.akind == 0) {
#pragma unroll
        for (int q = 0; q < NB; ++q) st.rb[q] = cmul(f.alpha, st.rb[q]);
    }
}

template <bool MIXED, int BM, int BN>
__device__ inline void store_stage(const StageFlags& ta, int tid, const Stage<BM, BN>& st,
                                   typename Prec<MIXED>::C (*As)[BM + 1],
                                   typename Prec<MIXED>::C (*Bs)[BN + 1]) {
    constexpr int NA = BM * kBK / kThreads;
    constexpr int NB = BN * kBK / kThreads;
#pragma unroll
    for (int q = 0; q < NA; ++q) {
        const int e = tid + kThreads * q;
        As[a_p<BM>(ta.ah, e)][a_i<BM>(ta.ah, e)] = Prec<MIXED>::cvt(st.ra[q]);
    }
#pragma unroll
    for (int q = 0; q < NB; ++q) {
        const int e = tid + kThreads * q;
        Bs[b_p<BN>(ta.bh, e)][b_j<BN>(ta.bh, e)] = Prec<MIXED>::cvt(st.rb[q]);
    }
}

// One workgroup computes a BM x BN complex tile; its 4 waves split the tile
// 2 x 2 (BM/2 rows x BN real columns each, i.e. row groups x BN/16 MFMA
// column blocks).
template <bool MIXED, int BM, int BN>
__global__ __launch_bounds__(kThreads)
void zgemm_grouped(const GemmOp* __restrict__ ops, int nops) {
    typedef typename Prec<MIXED>::C CT;
    typedef typename Prec<MIXED>::R RT;
    typedef typename Prec<MIXED>::Acc AccT;
    constexpr int MI = BM / 32;
    constexpr int NI = BN / 16;
    __shared__ CT As[2][kBK][BM + 1];
    __shared__ CT Bs[2][kBK][BN + 1];

    const int bid = xcd_remap(blockIdx.x, gridDim.x);
    const GemmOp* op = ops + find_op(ops, nops, bid);
    const int m = op->m, n = op->n, nterms = op->nterms;
    const int local = bid - op->tile_begin;
    const int tm = local / op->tiles_n, tn = local - tm * op->tiles_n;
    const int i0 = tm * BM, j0 = tn * BN;
    const int tid = threadIdx.x;
    const GemmTerm* terms = op->t;     // uniform: read with scalar loads

    const int lane = tid & 63, wave = tid >> 6;
    const int wm = wave & 1, wn = wave >> 1;
    const int cA = (lane >> 4) & 1;   // real k within the pair: 0 = re part of A, 1 = im part
    const int pOff = lane >> 5;       // complex k offset within the 4-wide real k step
    const int r16 = lane & 15;
    const int d = lane & 1;           // output component of this lane's B'' column
    const bool negB = cA == 1 && d == 0;

    // FP64: v_mfma_f64_4x4x4f64 with A replicated over its four blocks acts as
    // a 4-row x 16-column x 4-k product: A[row = lane%4][k = lane/16],
    // B[k = lane/16][col = lane%16], D[row = lane/16][col = lane%16] (layout
    // measured on gfx950).  A wave covers BM/2 rows as RG groups of 4 rows.
    // FP32 (mixed): v_mfma_f32_16x16x4f32, MI blocks of 16 rows.
    constexpr int RG = MIXED ? MI : BM / 8;
    AccT acc[RG][NI];
#pragma unroll
    for (int a = 0; a < RG; ++a)
#pragma unroll
        for (int b = 0; b < NI; ++b)
            acc[a][b] = AccT{};
    if constexpr (!MIXED) {
        // FP64: the accumulators start at beta C (C read before any of D is
        // written, so C may be D), and the epilogue only stores.
        if (op->C) {
            const gptr_t Cp = (gptr_t)op->C;
            const int ldc = op->ldc;
            const double2 beta = op->beta;
            double2 cv[RG][NI];
#pragma unroll
            for (int g = 0; g < RG; ++g)
#pragma unroll
                for (int ni = 0; ni < NI; ++ni) {
                    const int row = min(i0 + wm * (BM / 2) + g * 4 + (lane >> 4), m - 1);
                    const int col = min(j0 + ((wn * BN + ni * 16 + r16) >> 1), n - 1);
                    cv[g][ni] = Cp[(size_t)row * ldc + col];
                }
#pragma unroll
            for (int g = 0; g < RG; ++g)
#pragma unroll
                for (int ni = 0; ni < NI; ++ni) {
                    const double2 c = cv[g][ni];
                    acc[g][ni] = d ? (beta.x * c.y + beta.y * c.x) : (beta.x * c.x - beta.y * c.y);
                }
        }
    }

    // Stages are (term, k offset) pairs in order; next() steps to the
    // following one, skipping empty terms.  Two register sets hold the raw
    // operands of the next two stages: each step first issues the loads of
    // the stage after next (setting up that stage's term when it starts a
    // new one), then runs the MFMAs of the stage in LDS, then converts the
    // next stage's operands (waiting for their loads) into the other LDS
    // buffer.  Each register set carries the flags of the term it was
    // loaded for.
    auto next = [&](int& t, int& k0) {
        k0 += kBK;
        while (t < nterms && k0 >= terms[t].k) { ++t; k0 = 0; }
    };
    int t1 = 0, k1 = 0;
    while (t1 < nterms && terms[t1].k <= 0) ++t1;
    Stage<BM, BN> st[2];
    StageFlags sf[2];
    TermAddr<BM, BN> ta;
    int ta_term = -1;
    bool cur = false, fly = false;
    if (t1 < nterms) {
        term_setup<BM, BN>(terms[t1], m, n, i0, j0, tid, ta);
        ta_term = t1;
        issue_stage<BM, BN>(ta, k1, tid, st[0]);
        finish_stage<BM, BN>(ta.f, st[0]);
        store_stage<MIXED, BM, BN>(ta.f, tid, st[0], As[0], Bs[0]);
        cur = true;
        next(t1, k1);
        fly = t1 < nterms;
        if (fly && t1 != ta_term) { term_setup<BM, BN>(terms[t1], m, n, i0, j0, tid, ta); ta_term = t1; }
        issue_stage<BM, BN>(ta, k1, tid, st[1], fly);
        sf[1] = ta.f;
    }
    __syncthreads();
    int buf = 0;

    // one stage: X = register set in flight (the next stage), Y = free set
    auto step = [&](auto xs) {
        constexpr int X = decltype(xs)::value, Y = 1 - X;
        int t2 = t1, k2 = k1;
        bool fly2 = false;
        if (fly) {
            next(t2, k2);
            fly2 = t2 < nterms;
        }
        if (fly2 && t2 != ta_term) { term_setup<BM, BN>(terms[t2], m, n, i0, j0, tid, ta); ta_term = t2; }
        issue_stage<BM, BN>(ta, k2, tid, st[Y], fly2);
        sf[Y] = ta.f;
        // keep the order issue -> MFMAs -> conversion of the next stage, so
        // that the loads in flight have a whole stage of MFMAs to land
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int kk = 0; kk < kBK / 2; ++kk) {
            const int p = 2 * kk + pOff;
            RT av[RG], bv[NI];
            // one component read per operand: A' takes component cA, B'' takes
            // component cA ^ d, negated for (cA, d) = (1, 0)
#pragma unroll
            for (int g = 0; g < RG; ++g) {
                const int row = MIXED ? (wm * (BM / 2) + g * 16 + r16) : (wm * (BM / 2) + g * 4 + (lane & 3));
                av[g] = reinterpret_cast<const RT*>(&As[buf][p][row])[cA];
            }
#pragma unroll
            for (int ni = 0; ni < NI; ++ni) {
                const int jc = (wn * BN + ni * 16 + r16) >> 1;
                const RT v = reinterpret_cast<const RT*>(&Bs[buf][p][jc])[cA ^ d];
                bv[ni] = Prec<MIXED>::flip(v, negB);
            }
#pragma unroll
            for (int g = 0; g < RG; ++g)
#pragma unroll
                for (int ni = 0; ni < NI; ++ni)
                    acc[g][ni] = Prec<MIXED>::mfma(av[g], bv[ni], acc[g][ni]);
        }
        __builtin_amdgcn_sched_barrier(0);
        // unconditional like the issue: without a next stage st[X] holds
        // zeros from kOOB loads, stored to the buffer no later stage reads
        finish_stage<BM, BN>(sf[X], st[X]);
        store_stage<MIXED, BM, BN>(sf[X], tid, st[X], As[buf ^ 1], Bs[buf ^ 1]);
        __syncthreads();
        cur = fly;
        fly = fly2;
        t1 = t2;
        k1 = k2;
        buf ^= 1;
    };
    // FP64: four steps per iteration.  The compiler's wait counts throttle
    // the load issue only in the first bodies after the loop header, so the
    // longer body keeps the loads two stages ahead in the others.  (The mixed
    // kernels keep two: four would cost them occupancy.)
    while (cur) {
        step(std::integral_constant<int, 1>{});
        if (!cur) break;
        step(std::integral_constant<int, 0>{});
        if constexpr (!MIXED) {
            if (!cur) break;
            step(std::integral_constant<int, 1>{});
            if (!cur) break;
            step(std::integral_constant<int, 0>{});
        }
    }

    // Epilogue: lane holds real column lane%16 (component lane%2 of complex
    // column lane%16 / 2) of rows row_of(lane, r) of each row group.
    constexpr int GR = MIXED ? 16 : 4;             // rows per row group
    constexpr int NR = Prec<MIXED>::NR;
    double* D = reinterpret_cast<double*>(op->D);
    const double2* C = op->C;
    const int ldd = op->ldd, ldc = op->ldc;
    const double2 beta = op->beta;
    if (MIXED && C) {
        // all C loads first (clamped, unconditional), then the stores
        double2 cv[RG][NI][NR];
        const gptr_t Cp = (gptr_t)C;
#pragma unroll
        for (int g = 0; g < RG; ++g)
#pragma unroll
            for (int ni = 0; ni < NI; ++ni)
#pragma unroll
                for (int r = 0; r < NR; ++r) {
                    const int row = min(i0 + wm * (BM / 2) + g * GR + Prec<MIXED>::row_of(lane, r), m - 1);
                    const int col = min(j0 + ((wn * BN + ni * 16 + r16) >> 1), n - 1);
                    cv[g][ni][r] = Cp[(size_t)row * ldc + col];
                }
#pragma unroll
        for (int g = 0; g < RG; ++g)
#pragma unroll
            for (int ni = 0; ni < NI; ++ni)
#pragma unroll
                for (int r = 0; r < NR; ++r)
                    asm volatile("" : "+v"(cv[g][ni][r].x), "+v"(cv[g][ni][r].y));
#pragma unroll
        for (int g = 0; g < RG; ++g)
#pragma unroll
            for (int ni = 0; ni < NI; ++ni)
#pragma unroll
                for (int r = 0; r < NR; ++r) {
                    const int row = i0 + wm * (BM / 2) + g * GR + Prec<MIXED>::row_of(lane, r);
                    const int col = j0 + ((wn * BN + ni * 16 + r16) >> 1);
                    const double2 c = cv[g][ni][r];
                    const double v = Prec<MIXED>::elem(acc[g][ni], r) +
                        (d ? (beta.x * c.y + beta.y * c.x) : (beta.x * c.x - beta.y * c.y));
                    if (row < m && col < n) D[2 * ((size_t)row * ldd + col) + d] = v;
                }
    } else {
#pragma unroll
        for (int g = 0; g < RG; ++g)
#pragma unroll
            for (int ni = 0; ni < NI; ++ni)
#pragma unroll
                for (int r = 0; r < NR; ++r) {
                    const int row = i0 + wm * (BM / 2) + g * GR + Prec<MIXED>::row_of(lane, r);
                    const int col = j0 + ((wn * BN + ni * 16 + r16) >> 1);
                    if (row < m && col < n) D[2 * ((size_t)row * ldd + col) + d] = Prec<MIXED>::elem(acc[g][ni], r);
                }
    }
}

// Tile shapes of the grouped product (complex rows x complex columns).
// Every op of a launch is tiled with the launch's shape: tiles_n and
// tile_begin of the ops must be computed with gemm_tiles_shape().
struct TileShape { int bm, bn; };
constexpr TileShape kShapes[kGemmShapes] = {{32, 32}, {64, 32}, {64, 64}};

int gemm_shape_bm(int shape) { return kShapes[shape].bm; }
int gemm_shape_bn(int shape) { return kShapes[shape].bn; }
int gemm_tiles_shape(int m, int n, int shape) {
    return ((m + kShapes[shape].bm - 1) / kShapes[shape].bm) * ((n + kShapes[shape].bn - 1) / kShapes[shape].bn);
}
int gemm_tiles_n_shape(int n, int shape) { return (n + kShapes[shape].bn - 1) / kShapes[shape].bn; }

template <bool MIXED>
static void launch_mixed(const GemmOp* d_ops, int nops, int total_tiles, int shape, hipStream_t s) {
    switch (shape) {
        case 0: hipLaunchKernelGGL((zgemm_grouped<MIXED, 32, 32>), dim3(total_tiles), dim3(kThreads), 0, s, d_ops, nops); break;
        case 1: hipLaunchKernelGGL((zgemm_grouped<MIXED, 64, 32>), dim3(total_tiles), dim3(kThreads), 0, s, d_ops, nops); break;
        default: hipLaunchKernelGGL((zgemm_grouped<MIXED, 64, 64>), dim3(total_tiles), dim3(kThreads), 0, s, d_ops, nops); break;
    }
}

hipError_t launch_gemm_shape(const GemmOp* d_ops, int nops, int total_tiles, bool mixed, int shape, hipStream_t s) {
    if (nops <= 0 || total_tiles <= 0) return hipSuccess;
    if (shape < 0 || shape >= kGemmShapes) return hipErrorInvalidValue;
    if (mixed) launch_mixed<true>(d_ops, nops, total_tiles, shape, s);
    else launch_mixed<false>(d_ops, nops, total_tiles, shape, s);
    return hipGetLastError();
}

}  // namespace btsq
