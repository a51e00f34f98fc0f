// Whole solves of small instances: one workgroup per instance, one launch
// for a batch.
//
// With diagonal blocks and tip of at most kFusedMaxDim, every operation of
// the sweeps is a product of small blocks, and one grouped launch per
// dependency level leaves the GPU waiting on launches most of the time.
// Here one workgroup executes its instance's whole operation list -- the
// products, diagonal-block inverses and block sums of the forward and
// backward sweeps (Alg. 1 and 2, with the arrowhead terms of Sec. III-A and
// the partition and reduced-system steps of Sec. III-B when asked for) -- in
// dependency order, with a workgroup barrier between consecutive steps.
// Instances are independent, so no workgroup ever waits on another one.
// Each step's descriptor is a fixed-size record; the next record is read
// from memory while the current step runs and handed over through LDS, and
// every field a step branches or addresses on is made wave-uniform.
// The steps are the same operation descriptors the grouped kernels run;
// only the order of the sums inside a product and the inverse's pivoting
// (rows of the block itself instead of its transpose) differ.
#include "common.h"
#include "cplx.h"

namespace btsq {

constexpr int kFT = 256;           // threads per workgroup
constexpr int kFK = 16;            // complex k per product stage
constexpr int kFusedLds = kFusedMaxDim * kFusedMaxDim + 2 * kFusedMaxDim;   // double2 elements
constexpr int kRecWords = sizeof(FusedRec) / 4;
static_assert(kRecWords <= kFT, "one record word per thread");

// Values every lane holds alike (record fields read from LDS), moved to
// scalar registers so that branches and addresses on them stay uniform.
__device__ inline int uni(int x) { return __builtin_amdgcn_readfirstlane(x); }
__device__ inline double uni(double x) {
    const long long b = __double_as_longlong(x);
    const unsigned lo = (unsigned)uni((int)(unsigned)b), hi = (unsigned)uni((int)(unsigned)(b >> 32));
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
__device__ inline double2 uni(double2 x) { return make_double2(uni(x.x), uni(x.y)); }
template <class T> __device__ inline T* uni(T* p) {
    const unsigned long long b = (unsigned long long)p;
    const unsigned lo = (unsigned)uni((int)(unsigned)b), hi = (unsigned)uni((int)(unsigned)(b >> 32));
    return (T*)(((unsigned long long)hi << 32) | lo);
}

// Global-memory pointers as such (not generic), so that their loads and
// stores do not count against the LDS wait counter.
#ifdef __HIP_DEVICE_COMPILE__
typedef const __attribute__((address_space(1))) double2* gcp;
typedef __attribute__((address_space(1))) double2* gp;
typedef __attribute__((address_space(1))) double* gdp;
#else
typedef const double2* gcp;
typedef double2* gp;
typedef double* gdp;
#endif

// One product term with its fields in scalar registers.
struct FTerm {
    gcp A;
    gcp B;
    int lda, ldb, k;
    bool ah, bh;
    double2 alpha;
};
__device__ inline FTerm load_term(const GemmTerm& T) {
    FTerm t;
    t.A = (gcp)uni(T.A);
    t.B = (gcp)uni(T.B);
    t.lda = uni(T.lda);
    t.ldb = uni(T.ldb);
    t.k = uni(T.k);
    const int fl = uni(T.flags);
    t.ah = fl & kTermAH;
    t.bh = fl & kTermBH;
    t.alpha = uni(T.alpha);
    return t;
}

// ---------------------------------------------------------------------------
// Products D = beta C + sum_t alpha_t op(A_t) op(B_t), by the whole
// workgroup: TM x TM output tiles in turn.  Operands pass through LDS kFK
// values of k at a time; the next stage's global loads are issued before the
// current stage's multiply-adds.
template <int TM>
struct FStage {
    static constexpr int NL = TM * kFK / kFT;
    double2 a[NL], b[NL];
    bool oka[NL], okb[NL];     // inside the operand (else the value read is replaced by zero)
};

// Stage element e of op(A) (TM x kFK) and op(B) (kFK x TM), numbered so that
// consecutive threads read consecutive memory.
template <int TM> __device__ inline int fa_i(bool ah, int e) { return ah ? e % TM : e / kFK; }
template <int TM> __device__ inline int fa_k(bool ah, int e) { return ah ? e / TM : e % kFK; }
template <int TM> __device__ inline int fb_j(bool bh, int e) { return bh ? e / kFK : e % TM; }
template <int TM> __device__ inline int fb_k(bool bh, int e) { return bh ? e % kFK : e / TM; }

// Every lane issues all its loads unconditionally (out-of-range entries read
// element 0, always present, and are zeroed when stored to LDS), so the loads
// of a stage are in flight together and nothing waits for them before the
// stage is stored.
template <int TM>
__device__ inline void fgemm_load(const FTerm& T, int m, int n, int i0, int j0, int k0, int tid,
                                  FStage<TM>& st) {
#pragma unroll
    for (int q = 0; q < FStage<TM>::NL; ++q) {
        const int e = tid + kFT * q;
        const int gi = i0 + fa_i<TM>(T.ah, e), ka = k0 + fa_k<TM>(T.ah, e);
        const bool oka = gi < m && ka < T.k;
        const size_t ia = oka ? (T.ah ? (size_t)ka * T.lda + gi : (size_t)gi * T.lda + ka) : 0;
        const int gj = j0 + fb_j<TM>(T.bh, e), kb = k0 + fb_k<TM>(T.bh, e);
        const bool okb = gj < n && kb < T.k;
        const size_t ib = okb ? (T.bh ? (size_t)gj * T.ldb + kb : (size_t)kb * T.ldb + gj) : 0;
        st.a[q] = T.A[ia];
        st.b[q] = T.B[ib];
        st.oka[q] = oka;
        st.okb[q] = okb;
    }
}

// LDS rows of a stage are TM + 1 long, so that the A stores of consecutive
// threads (consecutive k for one row i when A is read as stored) fall into
// different banks.
template <int TM> constexpr int kFLd = TM + 1;

template <int TM>
__device__ inline void fgemm_store(const FTerm& T, int tid, const FStage<TM>& st, double2* As, double2* Bs) {
#pragma unroll
    for (int q = 0; q < FStage<TM>::NL; ++q) {
        const int e = tid + kFT * q;
        double2 a = st.oka[q] ? st.a[q] : make_double2(0.0, 0.0);
        if (T.ah) a.y = -a.y;
        As[fa_k<TM>(T.ah, e) * kFLd<TM> + fa_i<TM>(T.ah, e)] = a;
        double2 b = st.okb[q] ? st.b[q] : make_double2(0.0, 0.0);
        if (T.bh) b.y = -b.y;
        Bs[fb_k<TM>(T.bh, e) * kFLd<TM> + fb_j<TM>(T.bh, e)] = cmul_i(T.alpha, b);
    }
}

// The multiply-adds run on the FP64 matrix cores with the grouped kernel's
// scheme: the complex product as the real product of A' (A read as m x 2k
// real) and B'' (B expanded to 2k x 2n real, [[Re, Im], [-Im, Re]] per
// entry), v_mfma_f64_4x4x4f64 used as a 4-row x 16-column x 4-k product
// with A replicated over its four blocks (A[l%4][l/16], B[l/16][l%16],
// D[l/16][l%16]).  The four waves split the TM x TM tile 2 x 2: each owns
// TM/2 rows (TM/8 groups of 4) and TM/2 complex columns (TM/16 blocks of 16
// real columns).
template <int TM>
__device__ void fused_gemm(const GemmOp& op, double2* lds, int tid) {
    constexpr int RG = TM / 8;                // 4-row groups per wave
    constexpr int NI = TM / 16;               // 16-real-column blocks per wave
    double2* As = lds;
    double2* Bs = lds + kFK * kFLd<TM>;
    const int m = uni(op.m), n = uni(op.n), nt = uni(op.nterms);
    gp D = (gp)uni(op.D);
    gcp C = (gcp)uni(op.C);
    const int ldd = uni(op.ldd), ldc = uni(op.ldc);
    const double2 beta = uni(op.beta);
    const int lane = tid & 63, wave = tid >> 6;
    const int wm = wave & 1, wn = wave >> 1;
    const int cA = (lane >> 4) & 1;           // real k within the pair: 0 = Re of A, 1 = Im
    const int pOff = lane >> 5;               // complex k offset within the 4-wide real k step
    const int r16 = lane & 15;
    const int d = lane & 1;                   // output component of this lane's B'' column
    const unsigned long long negB = (cA == 1 && d == 0) ? 0x8000000000000000ull : 0ull;
    const int tn = (n + TM - 1) / TM;
    const int tiles = ((m + TM - 1) / TM) * tn;
    for (int t = 0; t < tiles; ++t) {
        const int i0 = (t / tn) * TM, j0 = (t % tn) * TM;
        double acc[RG][NI];
#pragma unroll
        for (int g = 0; g < RG; ++g)
#pragma unroll
            for (int ni = 0; ni < NI; ++ni) acc[g][ni] = 0.0;
        // stages are (term, k offset) pairs in order, empty terms skipped
        int s = 0, k0 = 0;
        while (s < nt && uni(op.t[s].k) <= 0) ++s;
        FStage<TM> st;
        FTerm cur{};
        if (s < nt) {
            cur = load_term(op.t[s]);
            fgemm_load<TM>(cur, m, n, i0, j0, 0, tid, st);
        }
        while (s < nt) {
            __syncthreads();                      // the previous stage's readers are done
            fgemm_store<TM>(cur, tid, st, As, Bs);
            __syncthreads();
            int s2 = s, k2 = k0 + kFK;
            while (s2 < nt && k2 >= uni(op.t[s2].k)) { ++s2; k2 = 0; }
            FTerm nxt = cur;
            if (s2 < nt) {
                if (s2 != s) nxt = load_term(op.t[s2]);
                fgemm_load<TM>(nxt, m, n, i0, j0, k2, tid, st);
            }
            // entries past k are zero in both operands: the full depth is exact
#pragma unroll
            for (int kk = 0; kk < kFK / 2; ++kk) {
                const int p = 2 * kk + pOff;
                double av[RG], bv[NI];
#pragma unroll
                for (int g = 0; g < RG; ++g)
                    av[g] = reinterpret_cast<const double*>(&As[p * kFLd<TM> + wm * (TM / 2) + g * 4 + (lane & 3)])[cA];
#pragma unroll
                for (int ni = 0; ni < NI; ++ni) {
                    const double v = reinterpret_cast<const double*>(&Bs[p * kFLd<TM> + ((wn * TM + ni * 16 + r16) >> 1)])[cA ^ d];
                    bv[ni] = __longlong_as_double(__double_as_longlong(v) ^ (long long)negB);
                }
#pragma unroll
                for (int g = 0; g < RG; ++g)
#pragma unroll
                    for (int ni = 0; ni < NI; ++ni)
                        acc[g][ni] = __builtin_amdgcn_mfma_f64_4x4x4f64(av[g], bv[ni], acc[g][ni], 0, 0, 0);
            }
            s = s2;
            k0 = k2;
            cur = nxt;
        }
        // lane: component d of complex column (wn TM + ni 16 + r16) / 2 of row
        // group g's row lane / 16; C may be D: each output element is read
        // and written by the same lane
#pragma unroll
        for (int g = 0; g < RG; ++g)
#pragma unroll
            for (int ni = 0; ni < NI; ++ni) {
                const int gi = i0 + wm * (TM / 2) + g * 4 + (lane >> 4);
                const int gj = j0 + ((wn * TM + ni * 16 + r16) >> 1);
                if (gi < m && gj < n) {
                    double v = acc[g][ni];
                    if (C) {
                        const double2 c = C[(size_t)gi * ldc + gj];
                        v += d ? (beta.x * c.y + beta.y * c.x) : (beta.x * c.x - beta.y * c.y);
                    }
                    reinterpret_cast<gdp>(D + (size_t)gi * ldd + gj)[d] = v;
                }
            }
    }
}

// ---------------------------------------------------------------------------
// Inverse of one d x d block (d <= kFusedMaxDim) in LDS: Gauss-Jordan
// elimination with partial pivoting, in place and without row exchanges.
// Column j takes as pivot row p_j the not-yet-used row of largest
// |re| + |im| in that column (to 11 mantissa bits, lowest row on ties),
// found by wave 0 with one row per lane; row p_j is scaled and column j
// eliminated from every other row, and slot j then holds column p_j of the
// accumulated transform T (T A = Q, Q e_j = e_{p_j}).  Since A^-1 = Q^T T,
//     A^-1[j][c] = W[p_j][pinv(c)],  pinv(p_j) = j,
// with W the working matrix at the end.  W is column-major in LDS, so the
// pivot search, the pivot column and the elimination read consecutive
// addresses.
__device__ void fused_inverse(const FusedInv& J, double2* lds, int* piv, int* pinv, int tid,
                              DevStatus* status) {
    const int d = uni(J.d);
    gcp src = (gcp)uni(J.src);
    gp dst = (gp)uni(J.dst);
    double2* W = lds;                          // W[r][c] at c * d + r
    double2* colj = lds + kFusedMaxDim * kFusedMaxDim;
    double2* rowp = colj + kFusedMaxDim;
    for (int e = tid; e < d * d; e += kFT) {
        const int r = e / d, c = e - r * d;
        W[c * d + r] = src[e];
    }
    bool bad = false;
    bool used = false;                         // wave 0: lane r's row has been a pivot row
    __syncthreads();
    for (int j = 0; j < d; ++j) {
        if (tid < 64) {                        // all of wave 0
            const int r = tid;
            const unsigned key = (r < d && !used) ? pivot_key(W[j * d + r], r) : 0u;
            const unsigned mx = wave_umax(key);
            const int p = mx == 0u ? -1 : key_row(mx);
            used = used || r == p;
            if (tid == 0) piv[j] = p;
        }
        __syncthreads();
        const int p = piv[j];
        bad = bad || p < 0;
        const int pr = p < 0 ? 0 : p;
        const double2 ip = crecip(W[j * d + pr]);
        bad = bad || !(fabs(ip.x) + fabs(ip.y) <= DBL_MAX);
        for (int e = tid; e < d; e += kFT) {
            colj[e] = W[j * d + e];
            rowp[e] = e == j ? ip : cmul_i(W[e * d + pr], ip);
        }
        __syncthreads();
        for (int e = tid; e < d * d; e += kFT) {
            const int c = e / d, r = e - c * d;
            if (r == pr) {
                W[e] = rowp[c];
            } else {
                double2 v = c == j ? make_double2(0.0, 0.0) : W[e];
                cfms(v, colj[r], rowp[c]);
                W[e] = v;
            }
        }
        __syncthreads();
    }
    // after a singular column the pivot rows need not be a permutation:
    // clear first so every index stays in range
    for (int c = tid; c < d; c += kFT) pinv[c] = 0;
    __syncthreads();
    for (int j = tid; j < d; j += kFT) {
        const int p = piv[j];
        if (p >= 0) pinv[p] = j;
    }
    __syncthreads();
    for (int e = tid; e < d * d; e += kFT) {
        const int j = e / d, c = e - j * d;
        const int p = piv[j] < 0 ? 0 : piv[j];
        dst[e] = W[pinv[c] * d + p];
    }
    if (bad && tid == 0 && atomicCAS(&status->code, 0, 3) == 0) status->tag = J.tag;
}

// ---------------------------------------------------------------------------
// Block sum D = sum_j c_j op_j(X_j) (op_j = X_j^H when bit j of hmask is set;
// such an input is stored cols x rows and is not D).
__device__ void fused_add(const AddOp& op, int tid) {
    const int rows = uni(op.rows), cols = uni(op.cols), nin = uni(op.nin);
    const unsigned hmask = (unsigned)uni((int)op.hmask);
    gp D = (gp)uni(op.D);
    for (int e = tid; e < rows * cols; e += kFT) {
        const int r = e / cols, c = e - r * cols;
        double2 acc = make_double2(0.0, 0.0);
        for (int j = 0; j < nin; ++j) {
            gcp X = (gcp)uni(op.X[j]);
            double2 x;
            if ((hmask >> j) & 1u) {
                x = X[(size_t)c * rows + r];
                x.y = -x.y;
            } else {
                x = X[e];
            }
            cfma(acc, uni(op.c[j]), x);
        }
        D[e] = acc;
    }
}

// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kFT)
void fused_solve(const FusedTask* __restrict__ tasks, const FusedRec* __restrict__ recs, DevStatus* status) {
    __shared__ double2 lds[kFusedLds];
    __shared__ int piv[kFusedMaxDim], pinv[kFusedMaxDim];
    __shared__ FusedRec srec[2];
    const FusedTask T = tasks[blockIdx.x];
    const int tid = threadIdx.x;
    const unsigned* words = reinterpret_cast<const unsigned*>(recs + T.first);
    unsigned* sw = reinterpret_cast<unsigned*>(srec);
    if (tid < kRecWords && T.count > 0) sw[tid] = words[tid];
    for (int q = 0; q < T.count; ++q) {
        // the next record is read while this step runs
        unsigned nxt = 0;
        const bool more = q + 1 < T.count;
        if (tid < kRecWords && more) nxt = words[(size_t)(q + 1) * kRecWords + tid];
        // the previous step's global writes and LDS reads are complete
        __syncthreads();
        const FusedRec& R = srec[q & 1];
        const int type = uni(R.type);
        if (type == 0) {
            const GemmOp& g = *reinterpret_cast<const GemmOp*>(R.body);
            if (max(uni(g.m), uni(g.n)) > 32) fused_gemm<64>(g, lds, tid);
            else fused_gemm<32>(g, lds, tid);
        } else if (type == 1) {
            fused_inverse(*reinterpret_cast<const FusedInv*>(R.body), lds, piv, pinv, tid, status);
        } else {
            fused_add(*reinterpret_cast<const AddOp*>(R.body), tid);
        }
        if (tid < kRecWords && more) sw[((q + 1) & 1) * kRecWords + tid] = nxt;
    }
}

hipError_t launch_fused(const FusedTask* d_tasks, int ntasks, const FusedRec* d_recs, DevStatus* status,
                        hipStream_t s) {
    if (ntasks <= 0) return hipSuccess;
    hipLaunchKernelGGL(fused_solve, dim3(ntasks), dim3(kFT), 0, s, d_tasks, d_recs, status);
    return hipGetLastError();
}

}  // namespace btsq
