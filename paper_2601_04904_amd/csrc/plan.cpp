// Host runtime: elimination plan -> DAG of block operations -> grouped launches.
//
// Every step of the method is "eliminate block k against its current
// neighbour set N(k)" (Alg. 1/2 for BT with N(k) = {k+1}; Sec. III-A for BTA
// with N(k) = {k+1, t}; Sec. III-B for partitions, where middle partitions
// eliminate against {s, k+1, t} and create fill-in).  With S = Atil_kk^-1:
//   forward A   S = inv(Atil_kk); T_u = Atil_uk S; Atil_uv -= T_u Atil_kv
//   forward B   S_B = (S Btil_kk) S^H; W_u = T_u Btil_kk;
//               Btil_uv += W_u T_v^H - T_u Btil_kv - Btil_uk T_v^H
//   backward SI tau_v = S Atil_kv; rho_u = sum_w X_uw Atil_wk;
//               X_uk = -rho_u S; X_kv = -sum_w tau_w X_wv;
//               X_kk = S - sum_w tau_w X_wk
//   backward SQ GB_u = sum_w X_uw Btil_wk; BG_v = sum_w Btil_kw X_vw^H;
//               Y21_u = GB_u S^H - rho_u S_B; L_kv = S BG_v - S_B rho_v^H
//               - sum_w tau_w L_wv; L_uk = Y21_u - sum_w L_uw tau_w^H;
//               L_kk = S_B - sum_w L_kw tau_w^H - sum_w tau_w Y21_w
// (u, v, w over N(k); X = X^R, L = X^<).
//
// The builder walks the plan once per call and records each operation with
// the device blocks it reads and writes.  Operations are then put on the
// earliest dependency level (read-after-write, write-after-read and
// write-after-write on whole blocks); all products of one level go into one
// grouped launch and all inverses of one level into one batched inverse.
// Independent chains - the B-chain beside the A-chain, partitions beside each
// other, the two halves of the reduced system, SQ backward beside SI
// backward - therefore share launches.  The A-chain runs on a second stream;
// launch lists are compiled once per pointer set (optionally captured as a
// HIP graph), and product tile shapes come from the tuning table.
#include "../../include/bt_si_sq.h"
#include "common.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <unordered_set>
#include <memory>
#include <string>
#include <atomic>
#include <mutex>
#include <unordered_map>
#include <vector>

namespace btsq {
hipError_t launch_gemm_shape(const GemmOp* d_ops, int nops, int total_tiles, bool mixed, int shape, hipStream_t s);
int gemm_tiles_shape(int m, int n, int shape);
int gemm_tiles_n_shape(int n, int shape);
int gemm_shape_bm(int shape);
int gemm_shape_bn(int shape);
int inv_variant(int d);   // panel kernel shape for dimension d: 0 (256 x 1 rows), 1 (256 x 2), 2 (512 x 2)
hipError_t launch_inv_step(const InvJob* d_jobs, int njobs, int variant, int panel, int maxd,
                           DevStatus* status, hipStream_t s);
hipError_t launch_add(const AddOp* d_ops, int nops, size_t max_elems, hipStream_t s);
hipError_t launch_norms(const NormJob* d_jobs, int njobs, hipStream_t s);
hipError_t launch_fused(const FusedTask* d_tasks, int ntasks, const FusedRec* d_recs, DevStatus* status,
                        hipStream_t s);
}  // namespace btsq

namespace {
thread_local std::string g_last_error;
}  // namespace

namespace btsq {
// error message of a call that has no handle (bt_si_sq_last_error(NULL))
void set_global_error(const std::string& msg) { g_last_error = msg; }
}  // namespace btsq

using namespace btsq;

namespace {

double2 cplx(double re, double im = 0.0) { return make_double2(re, im); }

struct MatRef {
    double2* p = nullptr;
    int r = 0, c = 0;
    bool ok() const { return p != nullptr; }
};

struct TermSpec {
    MatRef A;
    bool ah;
    MatRef B;
    bool bh;
    double2 alpha;
};

enum Kind { K_GEMM = 0, K_INV = 1, K_ADD = 2, K_NORM = 3 };

struct OpRec {
    Kind kind;
    MatRef D, C;
    double2 beta = {0, 0};
    std::vector<TermSpec> terms;
    bool mixed = false;
    int tag = 0;                                   // inverse: block id
    std::vector<std::pair<double2, MatRef>> ins;   // add; norm: (unused, block)
    uint32_t hmask = 0;                            // add: inputs taken as X^H
    int level = 0;
    int cls = 0;          // 1: critical A-chain stream, 0: main stream
    int wait_other = -1;  // highest level of a predecessor on the other stream
    int task = -1;        // >= 0: run by workgroup `task` of the fused launch (BT_FUSED)
};

enum Mode { MODE_FACTOR = 0, MODE_SQ = 1, MODE_BOTH = 2 };

// Block structure of one instance: n diagonal blocks (all of size b, or of
// the sizes in sz when the caller gives them; b is then the largest) and an
// arrow tip of size a.  Blocks of one field are stored one after another, so
// block i of a field starts at the sum of the sizes of blocks 0..i-1.
struct Dims {
    int n = 0, b = 0, a = 0;
    std::vector<int> sz;                  // per-block sizes, empty = uniform b
    std::vector<size_t> od, oul, oar;     // element offsets: diag, upper/lower, arrows
    Dims() = default;
    Dims(int n_, int b_, int a_, const int32_t* sizes = nullptr) : n(n_), b(b_), a(a_) {
        if (sizes) {
            sz.assign(sizes, sizes + n);
            b = *std::max_element(sz.begin(), sz.end());
        }
        od.assign(n + 1, 0);
        oul.assign(n + 1, 0);
        oar.assign(n + 1, 0);
        for (int i = 0; i < n; ++i) {
            const size_t bi = bsz(i), bj = i + 1 < n ? bsz(i + 1) : 0;
            od[i + 1] = od[i] + bi * bi;
            oul[i + 1] = oul[i] + bi * bj;
            oar[i + 1] = oar[i] + bi * (size_t)a;
        }
    }
    int bsz(int i) const { return sz.empty() ? b : sz[i]; }
    int dim(int u) const { return u == n ? a : bsz(u); }
    bool uneven() const {
        for (int v : sz)
            if (v != sz[0]) return true;
        return false;
    }
};

// Elimination plan (host logic only).
struct Elim {
    int k;
    std::vector<int> N;
};

struct PlanShape {
    std::vector<std::vector<Elim>> parts;   // per partition, forward order
    std::vector<int> reduced;               // kept blocks (P > 1)
};

PlanShape make_plan(const Dims& D, const std::vector<int>& bounds) {
    PlanShape ps;
    const int P = (int)bounds.size() - 1;
    const int t = D.n;
    const bool arrow = D.a > 0;
    if (P == 1) {
        std::vector<Elim> seq;
        for (int k = 0; k < D.n; ++k) {
            Elim e{k, {}};
            if (k + 1 < D.n) e.N.push_back(k + 1);
            if (arrow) e.N.push_back(t);
            seq.push_back(e);
        }
        if (arrow) seq.push_back(Elim{t, {}});
        ps.parts.push_back(seq);
        return ps;
    }
    for (int p = 0; p < P; ++p) {
        const int s = bounds[p], e = bounds[p + 1] - 1;
        std::vector<Elim> part;
        if (p == 0) {
            for (int k = s; k < e; ++k) {
                Elim el{k, {k + 1}};
                if (arrow) el.N.push_back(t);
                part.push_back(el);
            }
            ps.reduced.push_back(e);
        } else if (p == P - 1) {
            for (int k = e; k > s; --k) {
                Elim el{k, {k - 1}};
                if (arrow) el.N.push_back(t);
                part.push_back(el);
            }
            ps.reduced.push_back(s);
        } else {
            for (int k = s + 1; k < e; ++k) {
                Elim el{k, {s, k + 1}};
                if (arrow) el.N.push_back(t);
                part.push_back(el);
            }
            ps.reduced.push_back(s);
            ps.reduced.push_back(e);
        }
        ps.parts.push_back(part);
    }
    return ps;
}

bool validate_bounds(const Dims& D, const std::vector<int>& bounds, std::string& msg) {
    const int P = (int)bounds.size() - 1;
    if (P < 1) { msg = "partitions must be >= 1"; return false; }
    if (bounds.front() != 0 || bounds.back() != D.n) { msg = "bounds must run from 0 to n"; return false; }
    for (int p = 0; p < P; ++p) {
        const int sz = bounds[p + 1] - bounds[p];
        const int need = (P == 1 || p == 0 || p == P - 1) ? 1 : 2;
        if (sz < need) {
            char buf[160];
            snprintf(buf, sizeof buf, "partition %d has %d blocks; first/last partitions need >= 1, middle ones >= 2", p, sz);
            msg = buf;
            return false;
        }
    }
    return true;
}

// Bounds for blocks of different sizes: the smallest largest-partition cost
// (sum of F_k over the blocks a partition eliminates) found by bisection, each
// trial assigning partitions left to right as far as the trial cost allows.
std::vector<int> auto_bounds_uneven(const Dims& D, int P) {
    const int n = D.n;
    const double a = D.a;
    auto F = [](double b, double Dn) { return 3 * b * b * b + 11 * Dn * b * b + 10 * Dn * Dn * b; };
    auto bs = [&](int i) { return (double)D.bsz(i); };
    auto last_cost = [&](int s) {
        double c = 0;
        for (int k = s + 1; k < n; ++k) c += F(bs(k), bs(k - 1) + a);
        return c;
    };
    auto trial = [&](double T, std::vector<int>& out) {
        out.assign(1, 0);
        int s = 0;
        for (int p = 0; p < P - 1; ++p) {
            const int need_after = 2 * (P - 2 - p) + 1;   // blocks the later partitions need
            const int minsz = p == 0 ? 1 : 2;
            int e = s + minsz - 1;                        // last block of this partition
            if (e > n - 1 - need_after) return false;
            double c = 0;
            while (e + 1 <= n - 1 - need_after) {
                const double inc = p == 0 ? F(bs(e), bs(e + 1) + a) : F(bs(e), bs(s) + bs(e + 1) + a);
                if (c + inc > T) break;
                c += inc;
                ++e;
            }
            out.push_back(e + 1);
            s = e + 1;
        }
        out.push_back(n);
        return last_cost(s) <= T;
    };
    double hi = 0;
    for (int k = 0; k < n; ++k) hi += F(bs(k), 2 * D.b + a);
    double lo = 0;
    std::vector<int> best, cur;
    if (!trial(hi, best)) return {};
    for (int it = 0; it < 60; ++it) {
        const double mid = 0.5 * (lo + hi);
        if (trial(mid, cur)) { hi = mid; best = cur; }
        else lo = mid;
    }
    return best;
}

// Balance F_k = 8(3b^3 + 11 D b^2 + 10 D^2 b) per partition, D = size of N(k).
std::vector<int> auto_bounds(const Dims& D, int P) {
    std::vector<int> bounds;
    if (P <= 1) return {0, D.n};
    if (D.uneven()) return auto_bounds_uneven(D, P);
    const double b = D.b, a = D.a;
    auto F = [&](double Dn) { return 3 * b * b * b + 11 * Dn * b * b + 10 * Dn * Dn * b; };
    const double fe = F(b + a), fm = F(2 * b + a);
    const double rest = D.n - 2.0 - 2.0 * (P - 2);
    const double C = rest / (2.0 / fe + (P - 2) / fm);
    int mid = (int)std::lround(C / fm + 2.0);
    if (mid < 2) mid = 2;
    int ends = D.n - mid * (P - 2);
    while (ends < 2 && mid > 2) { --mid; ends = D.n - mid * (P - 2); }
    const int first = ends / 2, last = ends - first;
    bounds.push_back(0);
    bounds.push_back(first);
    for (int p = 1; p < P - 1; ++p) bounds.push_back(bounds.back() + mid);
    bounds.push_back(bounds.back() + last);
    (void)last;
    return bounds;
}

uint64_t key3(int u, int v, int tag) {
    return ((uint64_t)(uint32_t)(u + 1) << 42) | ((uint64_t)(uint32_t)(v + 1) << 21) | (uint64_t)(uint32_t)tag;
}

struct StepRec {
    int k;
    std::vector<int> N;
    bool reduced_stage;
    MatRef S, SB, Z;
    std::map<int, MatRef> T, W, Akv, Auk, Bkv, Buk, tau, rho, GB, BG, Y21;
};

struct Builder {
    Dims D;
    std::vector<int> bounds;
    Mode mode;
    bool mixed_bulk;
    // device pointers of the caller's blocks (null members allowed)
    bt_blocks Aext{}, Bext{}, XRext{}, XLext{};
    char* ws = nullptr;   // workspace base (a fake non-null base in dry runs)
    size_t off = 0;
    std::vector<OpRec> ops;
    std::unordered_map<uint64_t, MatRef> curA, curB, wsA, wsB, xR, xL;
    double flops = 0.0;
    int cur_cls = 0;      // stream class of the operations being emitted
    bool check = false;   // emit the FP64 selected-residual check (mixed path)
    bool plain = false;   // reference schedule: single-term products, one stream
    bool antiH = false;   // B anti-Hermitian: derive one block of each conjugate pair
    bool diag_only = false;   // outputs: diagonal blocks only (off-diagonal ones kept
                              // only where the backward sweep reads them again)
    std::unordered_set<uint64_t> needX;   // pairs (u, v) some backward step reads: N(k) x N(k)
    int instance = 0;     // instance id within a batch (reported with singular blocks)
    int reduced_parts = 2;    // partitions of the reduced system's own partitioned solve
    MatRef Ib, Ia;        // identity blocks (filled once at create)
    MatRef norm_out;      // norms written by the check (5 per block row)

    bool emitA() const { return mode == MODE_FACTOR || mode == MODE_BOTH; }
    bool emitB() const { return mode == MODE_SQ || mode == MODE_BOTH; }

    MatRef alloc(int r, int c) {
        off = (off + 255) & ~(size_t)255;
        MatRef m{reinterpret_cast<double2*>(ws + off), r, c};
        off += (size_t)r * c * sizeof(double2);
        return m;
    }

    // Caller block of field f for pair (u, v), or a fake unique address when
    // the caller pointer is null (dry runs only).
    MatRef ext_block(const bt_blocks& blk, int which, int u, int v) {
        const int t = D.n;
        void* base = nullptr;
        size_t offe = 0;
        int r = D.dim(u), c = D.dim(v);
        int field;
        if (u == t && v == t) { field = 5; base = blk.tip; offe = 0; }
        else if (v == t) { field = 3; base = blk.arrow_right; offe = D.oar[u]; }
        else if (u == t) { field = 4; base = blk.arrow_bottom; offe = D.oar[v]; }
        else if (u == v) { field = 0; base = blk.diag; offe = D.od[u]; }
        else if (v == u + 1) { field = 1; base = blk.upper; offe = D.oul[u]; }
        else { field = 2; base = blk.lower; offe = D.oul[v]; }
        double2* p;
        if (base) p = reinterpret_cast<double2*>(base) + offe;
        else p = reinterpret_cast<double2*>((uintptr_t)(((uint64_t)(which * 8 + field + 1)) << 44)) + offe;
        return MatRef{p, r, c};
    }

    void init_stores() {
        const int n = D.n, t = D.n;
        const bool arrow = D.a > 0;
        auto put = [&](int u, int v) {
            curA[key3(u, v, 0)] = ext_block(Aext, 0, u, v);
            curB[key3(u, v, 0)] = ext_block(Bext, 1, u, v);
        };
        for (int i = 0; i < n; ++i) {
            put(i, i);
            if (i + 1 < n) { put(i, i + 1); put(i + 1, i); }
            if (arrow) { put(i, t); put(t, i); }
        }
        if (arrow) put(t, t);
    }

    bool selected(int u, int v) const {
        const int t = D.n;
        if (u == t || v == t) return D.a > 0;
        return std::abs(u - v) <= 1;
    }

    MatRef xloc(bool lesser, int u, int v) {
        auto& store = lesser ? xL : xR;
        const uint64_t kk = key3(u, v, 0);
        auto it = store.find(kk);
        if (it != store.end()) return it->second;
        MatRef m = alloc(D.dim(u), D.dim(v));     // reserved for every pair, used when the caller gives none
        const bt_blocks& out = lesser ? XLext : XRext;
        if (selected(u, v) && !(diag_only && u != v)) {
            MatRef e = ext_block(out, lesser ? 3 : 2, u, v);
            const bool have = (u == D.n && v == D.n) ? out.tip != nullptr
                            : (v == D.n) ? out.arrow_right != nullptr
                            : (u == D.n) ? out.arrow_bottom != nullptr
                            : (u == v) ? out.diag != nullptr
                            : (v == u + 1) ? out.upper != nullptr : out.lower != nullptr;
            if (have) m = e;
        }
        store[kk] = m;
        return m;
    }

    MatRef cur(bool isB, int u, int v, int tag) {
        auto& st = isB ? curB : curA;
        auto it = st.find(key3(u, v, tag));
        return it == st.end() ? MatRef{} : it->second;
    }

    // Workspace slot that a matrix block moves into on its first update.
    MatRef work_slot(bool isB, int u, int v, int tag) {
        auto& st = isB ? wsB : wsA;
        const uint64_t kk = key3(u, v, tag);
        auto it = st.find(kk);
        if (it != st.end()) return it->second;
        MatRef m = alloc(D.dim(u), D.dim(v));
        st[kk] = m;
        return m;
    }

    void gemm(bool emit, MatRef Dst, MatRef Cin, double2 beta, std::vector<TermSpec> terms, bool mixed) {
        std::vector<TermSpec> kept;
        for (auto& t : terms)
            if (t.A.ok() && t.B.ok()) kept.push_back(t);
        if (!emit) return;
        if (plain && kept.size() > 1) {
            // one product per term, accumulating into Dst in program order
            gemm(emit, Dst, Cin, beta, {kept[0]}, mixed);
            for (size_t i = 1; i < kept.size(); ++i) gemm(emit, Dst, Dst, cplx(1), {kept[i]}, mixed);
            return;
        }
        OpRec op;
        op.kind = K_GEMM;
        op.D = Dst;
        op.C = Cin;
        op.beta = beta;
        op.terms = kept;
        op.mixed = mixed;
        op.cls = plain ? 0 : cur_cls;
        for (auto& t : kept) {
            const int k = t.ah ? t.A.r : t.A.c;
            flops += 8.0 * Dst.r * Dst.c * k;
        }
        ops.push_back(op);
    }

    void inv(bool emit, MatRef src, MatRef dst, int tag) {
        if (!emit) return;
        OpRec op;
        op.kind = K_INV;
        op.C = src;
        op.D = dst;
        op.tag = tag;
        op.cls = plain ? 0 : cur_cls;
        flops += 8.0 * (double)dst.r * dst.r * dst.r;
        ops.push_back(op);
    }

    // D = sum_j c_j X_j.  One sum takes at most kMaxAdd inputs; longer sums
    // (the tip of more than kMaxAdd - 1 partitions) are chained: the first
    // part writes D, each later part adds kMaxAdd - 1 more inputs to D.
    void add(bool emit, MatRef Dst, std::vector<std::pair<double2, MatRef>> ins) {
        if (!emit) return;
        std::vector<std::pair<double2, MatRef>> kept;
        for (auto& x : ins)
            if (x.second.ok()) kept.push_back(x);
        size_t i = 0;
        bool first = true;
        do {
            OpRec op;
            op.kind = K_ADD;
            op.D = Dst;
            op.cls = plain ? 0 : cur_cls;
            if (!first) op.ins.push_back({cplx(1), Dst});
            const size_t room = first ? (size_t)kMaxAdd : (size_t)kMaxAdd - 1;
            for (size_t q = 0; q < room && i < kept.size(); ++q, ++i) op.ins.push_back(kept[i]);
            ops.push_back(op);
            first = false;
        } while (i < kept.size());
    }

    // D = sum_j c_j op_j(X_j) with op_j = X_j^H where ins[j].h is set (no
    // transposed input may be D itself).
    struct HIn { double2 c; MatRef X; bool h; };
    void addh(bool emit, MatRef Dst, std::vector<HIn> ins) {
        if (!emit) return;
        OpRec op;
        op.kind = K_ADD;
        op.D = Dst;
        op.cls = plain ? 0 : cur_cls;
        for (size_t j = 0; j < ins.size(); ++j) {
            op.ins.push_back({ins[j].c, ins[j].X});
            if (ins[j].h) op.hmask |= 1u << j;
        }
        ops.push_back(op);
    }

    int tip_tag(int u, int v, int part_tag) const {
        return (u == D.n && v == D.n) ? part_tag : 0;
    }

    StepRec forward(int k, const std::vector<int>& N, int part_tag, bool reduced_stage) {
        StepRec r;
        r.k = k;
        r.N = N;
        r.reduced_stage = reduced_stage;
        const bool mx = mixed_bulk && !reduced_stage;
        const int dk = D.dim(k);
        const double2 one = cplx(1), mone = cplx(-1), zero = cplx(0);
        for (int u : N)
            for (int v : N) needX.insert(key3(u, v, 0));
        r.S = alloc(dk, dk);
        cur_cls = 1;   // the A-chain: inverse, T and Schur updates
        inv(emitA(), cur(false, k, k, tip_tag(k, k, part_tag)), r.S, (instance << 16) | k);
        for (int u : N) {
            r.Auk[u] = cur(false, u, k, 0);
            r.Akv[u] = cur(false, k, u, 0);
            r.T[u] = alloc(D.dim(u), dk);
            gemm(emitA(), r.T[u], MatRef{}, zero, {{r.Auk[u], false, r.S, false, one}}, mx);
        }
        for (int u : N)
            for (int v : N) {
                const int tg = tip_tag(u, v, part_tag);
                MatRef c = cur(false, u, v, tg);
                MatRef dst = work_slot(false, u, v, tg);
                gemm(emitA(), dst, c, one, {{r.T[u], false, r.Akv[v], false, mone}}, mx);
                curA[key3(u, v, tg)] = dst;
            }
        // B-chain
        cur_cls = 0;
        MatRef Bkk = cur(true, k, k, tip_tag(k, k, part_tag));
        r.Z = alloc(dk, dk);
        r.SB = alloc(dk, dk);
        gemm(emitB(), r.Z, MatRef{}, zero, {{r.S, false, Bkk, false, one}}, mx);
        gemm(emitB(), r.SB, MatRef{}, zero, {{r.Z, false, r.S, true, one}}, mx);
        for (int u : N) {
            r.Buk[u] = cur(true, u, k, 0);
            r.Bkv[u] = cur(true, k, u, 0);
            r.W[u] = alloc(D.dim(u), dk);
            gemm(emitB(), r.W[u], MatRef{}, zero, {{r.T[u], false, Bkk, false, one}}, mx);
        }
        for (size_t iu = 0; iu < N.size(); ++iu)
            for (size_t iv = 0; iv < N.size(); ++iv) {
                const int u = N[iu], v = N[iv];
                const int tg = tip_tag(u, v, part_tag);
                MatRef c = cur(true, u, v, tg);
                MatRef dst = work_slot(true, u, v, tg);
                if (!antiH) {
                    gemm(emitB(), dst, c, one,
                         {{r.W[u], false, r.T[v], true, one},
                          {r.T[u], false, r.Bkv[v], false, mone},
                          {r.Buk[u], false, r.T[v], true, mone}}, mx);
                } else if (iu == iv) {
                    // B_uk = -B_ku^H, so B_uk T_u^H = -(T_u B_ku)^H: with M = T_u B_ku,
                    // the update is W_u T_u^H - M + M^H
                    MatRef M = alloc(D.dim(u), D.dim(u));
                    gemm(emitB(), M, MatRef{}, zero, {{r.T[u], false, r.Bkv[u], false, one}}, mx);
                    gemm(emitB(), dst, c, one, {{r.W[u], false, r.T[u], true, one}}, mx);
                    addh(emitB(), dst, {{one, dst, false}, {mone, M, false}, {one, M, true}});
                } else if (iu < iv) {
                    gemm(emitB(), dst, c, one,
                         {{r.W[u], false, r.T[v], true, one},
                          {r.T[u], false, r.Bkv[v], false, mone},
                          {r.Buk[u], false, r.T[v], true, mone}}, mx);
                } else {
                    // the updated block (v, u) is formed above: B_uv = -B_vu^H
                    addh(emitB(), dst, {{mone, curB[key3(v, u, tip_tag(v, u, part_tag))], true}});
                }
                curB[key3(u, v, tg)] = dst;
            }
        return r;
    }

    void backward(StepRec& r) {
        const bool mx = mixed_bulk && !r.reduced_stage;
        const int k = r.k;
        const int dk = D.dim(k);
        const auto& N = r.N;
        const double2 one = cplx(1), mone = cplx(-1), zero = cplx(0);
        // selected inversion, on the critical stream: the A-chain is done by
        // now, so the X^R sweep runs ahead on it while the main stream
        // follows with the X^< products that read each step's X^R
        cur_cls = 1;
        for (int v : N) {
            r.tau[v] = alloc(dk, D.dim(v));
            gemm(emitA(), r.tau[v], MatRef{}, zero, {{r.S, false, r.Akv[v], false, one}}, mx);
        }
        for (int u : N) {
            r.rho[u] = alloc(D.dim(u), dk);
            std::vector<TermSpec> ts;
            for (int w : N) ts.push_back({xloc(false, u, w), false, r.Auk[w], false, one});
            gemm(emitA(), r.rho[u], MatRef{}, zero, ts, mx);
        }
        for (int u : N)
            gemm(emitA(), xloc(false, u, k), MatRef{}, zero, {{r.rho[u], false, r.S, false, mone}}, mx);
        // X_kv: an output, or read again by a later backward step; with
        // diagonal outputs only it is dropped where nothing reads it (the
        // transient-only form after Alg. 2)
        for (int v : N) {
            if (diag_only && !needX.count(key3(k, v, 0))) continue;
            std::vector<TermSpec> ts;
            for (int w : N) ts.push_back({r.tau[w], false, xloc(false, w, v), false, mone});
            gemm(emitA(), xloc(false, k, v), MatRef{}, zero, ts, mx);
        }
        {
            std::vector<TermSpec> ts;
            for (int w : N) ts.push_back({r.tau[w], false, xloc(false, w, k), false, mone});
            gemm(emitA(), xloc(false, k, k), r.S, one, ts, mx);
        }
        // selected quadratic solve
        cur_cls = 0;
        for (int u : N) {
            r.GB[u] = alloc(D.dim(u), dk);
            std::vector<TermSpec> ts;
            for (int w : N) ts.push_back({xloc(false, u, w), false, r.Buk[w], false, one});
            gemm(emitB(), r.GB[u], MatRef{}, zero, ts, mx);
        }
        if (!antiH)
            for (int v : N) {
                r.BG[v] = alloc(dk, D.dim(v));
                std::vector<TermSpec> ts;
                for (int w : N) ts.push_back({r.Bkv[w], false, xloc(false, v, w), true, one});
                gemm(emitB(), r.BG[v], MatRef{}, zero, ts, mx);
            }
        for (int u : N) {
            r.Y21[u] = alloc(D.dim(u), dk);
            gemm(emitB(), r.Y21[u], MatRef{}, zero,
                 {{r.GB[u], false, r.S, true, one}, {r.rho[u], false, r.SB, false, mone}}, mx);
        }
        for (int v : N) {
            MatRef L = xloc(true, k, v);
            if (!antiH)
                gemm(emitB(), L, MatRef{}, zero,
                     {{r.S, false, r.BG[v], false, one}, {r.SB, false, r.rho[v], true, mone}}, mx);
            else   // S BG_v - S_B rho_v^H = -(Y21_v)^H when B is anti-Hermitian
                addh(emitB(), L, {{mone, r.Y21[v], true}});
            std::vector<TermSpec> ts;
            for (int w : N) ts.push_back({r.tau[w], false, xloc(true, w, v), false, mone});
            gemm(emitB(), L, L, one, ts, mx);
        }
        // X^<_{u,k} is computed here even for anti-Hermitian B: taking it as
        // -(X^<_{k,u})^H couples the errors of the two recurrences and was
        // measured to amplify rounding by 10^2 - 10^3 on ill-conditioned inputs.
        for (int u : N) {
            if (diag_only && !needX.count(key3(u, k, 0))) continue;   // as X_kv above
            std::vector<TermSpec> ts;
            for (int w : N) ts.push_back({xloc(true, u, w), false, r.tau[w], true, mone});
            gemm(emitB(), xloc(true, u, k), r.Y21[u], one, ts, mx);
        }
        {
            std::vector<TermSpec> ts;
            for (int w : N) ts.push_back({xloc(true, k, w), false, r.tau[w], true, mone});
            for (int w : N) ts.push_back({r.tau[w], false, r.Y21[w], false, mone});
            gemm(emitB(), xloc(true, k, k), r.SB, one, ts, mx);
        }
    }

    // D = beta Cin + sum of terms, split into several products when there are
    // more terms than one product takes (each later part accumulates into D).
    void gemm_chain(bool emit, MatRef Dst, MatRef Cin, double2 beta, std::vector<TermSpec> terms) {
        std::vector<TermSpec> kept;
        for (auto& t : terms)
            if (t.A.ok() && t.B.ok()) kept.push_back(t);
        size_t i = 0;
        bool first = true;
        do {
            std::vector<TermSpec> part(kept.begin() + i, kept.begin() + std::min(kept.size(), i + (size_t)kMaxTerms));
            if (first) gemm(emit, Dst, Cin, beta, part, false);
            else gemm(emit, Dst, Dst, cplx(1), part, false);
            first = false;
            i += kMaxTerms;
        } while (i < kept.size());
    }

    // FP64 selected residuals of the result (Sec. II-A identities restricted to
    // the pattern): for every block row i,
    //   R^R_i = sum_j A_ij X^R_ji - I,   R^<_i = sum_j A_ij X^<_ji - sum_j B_ij (X^R_ij)^H,
    // then the norms of R^R_i, R^<_i, X^R_ii, X^<_ii and A_ii.
    void residual_check(bool emit) {
        const int n = D.n, t = D.n;
        const bool arrow = D.a > 0;
        const double2 one = cplx(1), mone = cplx(-1);
        std::vector<MatRef> RR, RL;
        for (int i = 0; i <= n; ++i) {
            if (i == n && !arrow) break;
            RR.push_back(alloc(D.dim(i), D.dim(i)));
            RL.push_back(alloc(D.dim(i), D.dim(i)));
        }
        norm_out = alloc(1, (5 * (n + 1) + 1) / 2 + 1);
        if (!emit) return;
        cur_cls = 0;
        for (int i = 0; i <= n; ++i) {
            if (i == n && !arrow) break;
            std::vector<int> cols;
            if (i == t) {
                for (int j = 0; j < n; ++j) cols.push_back(j);
                cols.push_back(t);
            } else {
                if (i > 0) cols.push_back(i - 1);
                cols.push_back(i);
                if (i + 1 < n) cols.push_back(i + 1);
                if (arrow) cols.push_back(t);
            }
            std::vector<TermSpec> tr, tl;
            for (int j : cols) {
                tr.push_back({ext_block(Aext, 0, i, j), false, xloc(false, j, i), false, one});
                tl.push_back({ext_block(Aext, 0, i, j), false, xloc(true, j, i), false, one});
                tl.push_back({ext_block(Bext, 1, i, j), false, xloc(false, i, j), true, mone});
            }
            gemm_chain(true, RR[i], i == t ? Ia : Ib, mone, tr);
            gemm_chain(true, RL[i], MatRef{}, cplx(0), tl);
        }
        OpRec op;
        op.kind = K_NORM;
        op.D = norm_out;
        op.cls = 0;
        for (int i = 0; i <= n; ++i) {
            if (i == n && !arrow) break;
            op.ins.push_back({cplx(5 * i + 0), RR[i]});
            op.ins.push_back({cplx(5 * i + 1), RL[i]});
            op.ins.push_back({cplx(5 * i + 2), xloc(false, i, i)});
            op.ins.push_back({cplx(5 * i + 3), xloc(true, i, i)});
            op.ins.push_back({cplx(5 * i + 4), ext_block(Aext, 0, i, i)});
        }
        ops.push_back(op);
    }

    // tip (t,t) = tip + the accumulators of the given tags, for A and B
    void sum_tip(const std::vector<int>& tags) {
        const int t = D.n;
        for (int isB = 0; isB < 2; ++isB) {
            std::vector<std::pair<double2, MatRef>> ins;
            ins.push_back({cplx(1), cur(isB, t, t, 0)});
            for (int tg : tags) ins.push_back({cplx(1), cur(isB, t, t, tg)});
            MatRef dst = work_slot(isB, t, t, 0);
            cur_cls = isB ? 0 : 1;
            add(isB ? emitB() : emitA(), dst, ins);
            cur_cls = 0;
            (isB ? curB : curA)[key3(t, t, 0)] = dst;
        }
    }

    // The reduced system: the kept blocks R (consecutive entries coupled, by an
    // original or a fill block) plus the tip, itself a BT(A) matrix.  With at
    // least four blocks it is solved by the same partitioned elimination
    // (the recursive call of Sec. III-B) with q = min(reduced_parts, m / 2)
    // contiguous parts of near-equal length: the first top-down, the last
    // bottom-up, the middle ones top-down against their top block with fill,
    // each adding its tip contribution to an accumulator of its own (summed
    // into the tip afterwards); their kept blocks form the next reduced
    // system, solved the same way.  With two parts it is its first half
    // top-down and its second half bottom-up, concurrent, then the two middle
    // blocks and the tip: the sequential chain shrinks from m to m/2 + 1
    // inverses.  Below four blocks: the sequential BTA RGF.
    void solve_reduced(const std::vector<int>& R, int& next_tag) {
        const int t = D.n;
        const bool arrow = D.a > 0;
        const int m = (int)R.size();
        if (m < 4 || reduced_parts < 2) {
            std::vector<StepRec> red;
            for (int j = 0; j < m; ++j) {
                std::vector<int> N;
                if (j + 1 < m) N.push_back(R[j + 1]);
                if (arrow) N.push_back(t);
                red.push_back(forward(R[j], N, 0, true));
            }
            if (arrow) red.push_back(forward(t, {}, 0, true));
            for (auto it = red.rbegin(); it != red.rend(); ++it) backward(*it);
            return;
        }
        const int q = std::max(2, std::min(reduced_parts, m / 2));
        std::vector<std::vector<StepRec>> parts(q);
        std::vector<int> R2, tags;
        for (int p = 0; p < q; ++p) {
            const int s = p * m / q, e = (p + 1) * m / q - 1;
            const int tag = next_tag++;
            tags.push_back(tag);
            auto with_tip = [&](std::vector<int> N) { if (arrow) N.push_back(t); return N; };
            if (p == 0) {
                for (int j = s; j < e; ++j) parts[p].push_back(forward(R[j], with_tip({R[j + 1]}), tag, true));
                R2.push_back(R[e]);
            } else if (p == q - 1) {
                for (int j = e; j > s; --j) parts[p].push_back(forward(R[j], with_tip({R[j - 1]}), tag, true));
                R2.push_back(R[s]);
            } else {
                for (int j = s + 1; j < e; ++j)
                    parts[p].push_back(forward(R[j], with_tip({R[s], R[j + 1]}), tag, true));
                R2.push_back(R[s]);
                R2.push_back(R[e]);
            }
        }
        if (arrow) sum_tip(tags);
        solve_reduced(R2, next_tag);
        for (auto& part : parts)
            for (auto it = part.rbegin(); it != part.rend(); ++it) backward(*it);
    }

    void build() {
        Ib = alloc(D.b, D.b);
        Ia = alloc(std::max(D.a, 1), std::max(D.a, 1));
        init_stores();
        PlanShape ps = make_plan(D, bounds);
        const int P = (int)bounds.size() - 1;
        const bool arrow = D.a > 0;
        std::vector<std::vector<StepRec>> recs(ps.parts.size());
        for (size_t p = 0; p < ps.parts.size(); ++p) {
            const int tag = (P > 1) ? (int)p + 1 : 0;
            for (auto& e : ps.parts[p]) recs[p].push_back(forward(e.k, e.N, tag, false));
        }
        if (P > 1) {
            if (arrow) {
                std::vector<int> tags;
                for (int p = 0; p < P; ++p) tags.push_back(p + 1);
                sum_tip(tags);
            }
            int next_tag = P + 1;
            solve_reduced(ps.reduced, next_tag);
        }
        for (size_t p = 0; p < recs.size(); ++p)
            for (auto it = recs[p].rbegin(); it != recs[p].rend(); ++it) backward(*it);
        residual_check(check && emitB());
    }
};

// Dependency levels on whole blocks (read-after-write, write-after-read,
// write-after-write).  Also records, per operation, the highest level of a
// predecessor that runs on the other stream.
int levelize(std::vector<OpRec>& ops, bool plain = false) {
    if (plain) {
        for (size_t i = 0; i < ops.size(); ++i) { ops[i].level = (int)i; ops[i].wait_other = -1; ops[i].cls = 0; }
        return (int)ops.size();
    }
    struct BufInfo { int wlevel = -1, wcls = 0; int rlevel[2] = {-1, -1}; };
    std::unordered_map<uintptr_t, BufInfo> info;
    int maxl = -1;
    std::vector<MatRef> reads;
    for (auto& op : ops) {
        reads.clear();
        if (op.kind == K_GEMM) {
            if (op.C.ok()) reads.push_back(op.C);
            for (auto& t : op.terms) { reads.push_back(t.A); reads.push_back(t.B); }
        } else if (op.kind == K_INV) {
            reads.push_back(op.C);
        } else {
            for (auto& x : op.ins) reads.push_back(x.second);   // sums and norms
        }
        int lvl = 0, other = -1;
        for (auto& r : reads) {
            auto it = info.find((uintptr_t)r.p);
            if (it == info.end() || it->second.wlevel < 0) continue;
            lvl = std::max(lvl, it->second.wlevel + 1);
            if (it->second.wcls != op.cls) other = std::max(other, it->second.wlevel);
        }
        {
            auto it = info.find((uintptr_t)op.D.p);
            if (it != info.end()) {
                const BufInfo& bi = it->second;
                if (bi.wlevel >= 0) {
                    lvl = std::max(lvl, bi.wlevel + 1);
                    if (bi.wcls != op.cls) other = std::max(other, bi.wlevel);
                }
                for (int c = 0; c < 2; ++c)
                    if (bi.rlevel[c] >= 0) {
                        lvl = std::max(lvl, bi.rlevel[c] + 1);
                        if (c != op.cls) other = std::max(other, bi.rlevel[c]);
                    }
            }
        }
        op.level = lvl;
        op.wait_other = other;
        BufInfo& w = info[(uintptr_t)op.D.p];
        w.wlevel = lvl;
        w.wcls = op.cls;
        for (auto& r : reads) {
            BufInfo& bi = info[(uintptr_t)r.p];
            bi.rlevel[op.cls] = std::max(bi.rlevel[op.cls], lvl);
        }
        maxl = std::max(maxl, lvl);
    }
    return maxl + 1;
}

struct Launch {
    int type;         // 0 gemm, 4 add, 5 norms, 6 inverse panel step, 7 fused instances
    size_t off;       // element offset into the typed array
    int count;
    int tiles;        // gemm: total tiles
    int mixed;        // gemm precision
    int maxd;         // inverse: max dim; panel step: kernel shape (inv_variant)
    int panel;
    size_t maxelems;  // add
    double flops = 0; // algorithmic work of the launch
    double bytes = 0;
    int shape = 1;    // gemm: tile shape (gemm_shape_bm / gemm_shape_bn)
    int cls = 0;      // stream class
    int level = 0;
    int wait_level = -1;  // wait for the other stream up to this level
    int wait_event = -1;  // event slot to wait on before the launch
    int rec_event = -1;   // event slot to record after the launch
};


// Algorithmic flops and HBM bytes of a grouped product launch.
void gemm_work(const GemmOp* ops, int n, double& flops, double& bytes) {
    flops = 0;
    bytes = 0;
    for (int i = 0; i < n; ++i) {
        const GemmOp& g = ops[i];
        double mn = (double)g.m * g.n;
        bytes += 16.0 * mn * (g.C ? 2.0 : 1.0);
        for (int t = 0; t < g.nterms; ++t) {
            flops += 8.0 * mn * g.t[t].k;
            bytes += 16.0 * ((double)g.m * g.t[t].k + (double)g.t[t].k * g.n);
        }
    }
}

struct Program {
    std::vector<GemmOp> gemm;
    std::vector<InvJob> inv;
    std::vector<AddOp> add;
    std::vector<NormJob> norm;
    std::vector<FusedRec> frec;     // fused launch: step records and tasks
    std::vector<FusedTask> ftask;
    std::vector<Launch> launches;
    size_t inv_scratch_bytes = 0;   // scratch the inverses need (max over levels)
    double flops = 0.0;
    int levels = 0;
    int n_events = 0;               // cross-stream events the launches use
    std::string error;              // non-empty: the operation list cannot be launched
};

GemmOp make_gemm_op(const OpRec& o) {
    GemmOp g;
    memset(&g, 0, sizeof g);
    g.D = o.D.p;
    g.C = o.C.p;
    g.ldd = o.D.c;
    g.ldc = o.C.ok() ? o.C.c : 0;
    g.m = o.D.r;
    g.n = o.D.c;
    g.nterms = (int)o.terms.size();
    g.mixed = o.mixed ? 1 : 0;
    g.beta = o.beta;
    for (size_t i = 0; i < o.terms.size(); ++i) {
        const TermSpec& t = o.terms[i];
        GemmTerm& d = g.t[i];
        d.A = t.A.p;
        d.B = t.B.p;
        d.lda = t.A.c;
        d.ldb = t.B.c;
        d.k = t.ah ? t.A.r : t.A.c;
        d.flags = (t.ah ? kTermAH : 0) | (t.bh ? kTermBH : 0);
        d.alpha = t.alpha;
    }
    return g;
}

// Product tile shape per launch.  A launch is classified by precision, the
// size class of its largest output (log2 of max(m, n), 5..10) and the class of
// its work (log2 of its 64 x 32 tile count, 0..13); the shape comes from the
// tuning table (filled by bt_si_sq_autotune or loaded with
// bt_si_sq_tune_table) or, for classes never tuned, from the default rule:
// 32 x 32 tiles below 512 tiles of 64 x 32, 64 x 32 tiles above.
constexpr int kMClasses = 6, kTClasses = 14;
std::atomic<int> g_tune[2][kMClasses][kTClasses];
std::once_flag g_tune_once;

void tune_init() {
    std::call_once(g_tune_once, [] {
        for (auto& a : g_tune) for (auto& b : a) for (auto& c : b) c.store(-1);
    });
}

int log2_class(long v, int lo, int hi) {
    int c = 0;
    while ((1L << (c + 1)) <= v) ++c;
    return std::min(std::max(c, lo), hi) - lo;
}

int default_shape(long tiles64x32) { return tiles64x32 < 512 ? 0 : 1; }

int pick_shape(int mixed, int maxdim, long tiles64x32) {
    tune_init();
    const int mc = log2_class(maxdim, 5, 5 + kMClasses - 1);
    const int tc = log2_class(std::max(1L, tiles64x32), 0, kTClasses - 1);
    const int v = g_tune[mixed ? 1 : 0][mc][tc].load();
    return (v >= 0 && v < kGemmShapes) ? v : default_shape(tiles64x32);
}

void set_shape(Program& pg, Launch& L, int shape) {
    int tiles = 0;
    for (int i = 0; i < L.count; ++i) {
        GemmOp& g = pg.gemm[L.off + i];
        g.tile_begin = tiles;
        g.tiles_n = gemm_tiles_n_shape(g.n, shape);
        tiles += gemm_tiles_shape(g.m, g.n, shape);
    }
    L.tiles = tiles;
    L.shape = shape;
}

void assign_shape(Program& pg, Launch& L) {
    long t1 = 0;
    int maxdim = 1;
    for (int i = 0; i < L.count; ++i) {
        const GemmOp& g = pg.gemm[L.off + i];
        t1 += gemm_tiles_shape(g.m, g.n, 1);
        maxdim = std::max(maxdim, std::max(g.m, g.n));
    }
    set_shape(pg, L, pick_shape(L.mixed, maxdim, t1));
}

AddOp make_add_op(const OpRec& o) {
    AddOp a;
    memset(&a, 0, sizeof a);
    a.D = o.D.p;
    a.nin = (int)o.ins.size();
    a.rows = o.D.r;
    a.cols = o.D.c;
    for (int q = 0; q < a.nin; ++q) {
        a.X[q] = o.ins[q].second.p;
        a.c[q] = o.ins[q].first;
    }
    a.hmask = o.hmask;
    return a;
}

// The operations of BT_FUSED instances (task >= 0): per task, its steps in
// level order (each instance's operations were built in dependency order,
// so a stable sort by level keeps every step after what it reads), and one
// launch with a workgroup per task.  Returns false (pg.error set) for an
// operation the fused kernel does not run.
bool compile_fused(Program& pg, const std::vector<OpRec>& ops) {
    int ntasks = 0;
    for (const auto& o : ops) ntasks = std::max(ntasks, o.task + 1);
    if (ntasks == 0) return true;
    std::vector<std::vector<int>> bytask(ntasks);
    for (int i = 0; i < (int)ops.size(); ++i)
        if (ops[i].task >= 0) bytask[ops[i].task].push_back(i);
    Launch L{};
    L.type = 7;
    L.off = 0;
    L.count = ntasks;
    L.cls = 0;
    L.level = 0;
    for (int t = 0; t < ntasks; ++t) {
        auto& v = bytask[t];
        std::stable_sort(v.begin(), v.end(), [&](int x, int y) { return ops[x].level < ops[y].level; });
        FusedTask task{(int32_t)pg.frec.size(), (int32_t)v.size()};
        for (int i : v) {
            const OpRec& o = ops[i];
            FusedRec rec;
            memset(&rec, 0, sizeof rec);
            if (o.kind == K_GEMM && !o.mixed) {
                GemmOp g = make_gemm_op(o);
                double f = 0, b = 0;
                gemm_work(&g, 1, f, b);
                L.flops += f;
                L.bytes += b;
                rec.type = 0;
                memcpy(rec.body, &g, sizeof g);
            } else if (o.kind == K_INV && o.D.r <= kFusedMaxDim) {
                FusedInv j{o.C.p, o.D.p, o.D.r, o.tag};
                L.flops += 8.0 * (double)j.d * j.d * j.d;
                L.bytes += 32.0 * (double)j.d * j.d;
                rec.type = 1;
                memcpy(rec.body, &j, sizeof j);
            } else if (o.kind == K_ADD && o.ins.size() <= (size_t)kMaxAdd) {
                AddOp a = make_add_op(o);
                L.flops += 8.0 * a.rows * a.cols * a.nin;
                L.bytes += 16.0 * a.rows * a.cols * (a.nin + 1);
                rec.type = 2;
                memcpy(rec.body, &a, sizeof a);
            } else {
                pg.error = "internal: an operation of a BT_FUSED instance has no fused form";
                return false;
            }
            pg.frec.push_back(rec);
        }
        pg.ftask.push_back(task);
    }
    pg.launches.push_back(L);
    return true;
}

// Turn levelled operations into typed device arrays and a launch list.
// Launches are ordered by level and, within a level, critical stream first;
// the fused launch (BT_FUSED instances) comes first, on the main stream.
// inv_pool: base of the inverse scratch pool (may be fake in dry runs).
Program compile(std::vector<OpRec>& ops, int nlevels, char* inv_pool) {
    Program pg;
    pg.levels = nlevels;
    if (!compile_fused(pg, ops)) return pg;
    std::vector<std::vector<int>> bylevel(nlevels);
    for (int i = 0; i < (int)ops.size(); ++i)
        if (ops[i].task < 0) bylevel[ops[i].level].push_back(i);
    auto mk = [&](int type, size_t off, int count, int tiles, int mixed, int maxd, int panel,
                  size_t maxe, int cls, int level, int wait) {
        Launch L{type, off, count, tiles, mixed, maxd, panel, maxe};
        L.cls = cls;
        L.level = level;
        L.wait_level = wait;
        return L;
    };
    for (int L = 0; L < nlevels; ++L) {
        for (int cls = 1; cls >= 0; --cls) {
            // inverses (grouped by the shape of the panel kernel)
            std::vector<int> invs;
            int wait = -1;
            for (int i : bylevel[L])
                if (ops[i].kind == K_INV && ops[i].cls == cls) { invs.push_back(i); wait = std::max(wait, ops[i].wait_other); }
            if (!invs.empty()) {
                std::stable_sort(invs.begin(), invs.end(), [&](int x, int y) {
                    return inv_variant(ops[x].D.r) < inv_variant(ops[y].D.r);
                });
                size_t poff = 0;
                const size_t first = pg.inv.size();
                int maxd = 0;
                for (int i : invs) {
                    const OpRec& o = ops[i];
                    const int d = o.D.r;
                    maxd = std::max(maxd, d);
                    InvJob j;
                    memset(&j, 0, sizeof j);
                    j.src = o.C.p;
                    j.dst = o.D.p;
                    j.d = d;
                    j.tag = o.tag;
                    poff = inv_bind_scratch(j, inv_pool, poff, d);
                    pg.inv.push_back(j);
                }
                pg.inv_scratch_bytes = std::max(pg.inv_scratch_bytes, poff + 256);
                const int nj = (int)invs.size();
                int vcount[3] = {0, 0, 0}, vmaxd[3] = {0, 0, 0};
                for (int i : invs) {
                    const int v = inv_variant(ops[i].D.r);
                    ++vcount[v];
                    vmaxd[v] = std::max(vmaxd[v], ops[i].D.r);
                }
                // one launch per panel and kernel shape, plus the one that applies
                // the last panel and writes the results; the first carries the
                // wait on the other stream
                const int npanels = (maxd + kInvNB - 1) / kInvNB;
                bool first_launch = true;
                for (int p = 0; p <= npanels; ++p) {
                    size_t off = first;
                    for (int v = 0; v < 3; ++v) {
                        if (vcount[v] > 0 && p <= (vmaxd[v] + kInvNB - 1) / kInvNB) {
                            pg.launches.push_back(mk(6, off, vcount[v], vmaxd[v], 0, v, p, 0, cls, L,
                                                     first_launch ? wait : -1));
                            first_launch = false;
                        }
                        off += vcount[v];
                    }
                }
                (void)nj;
            }
            // products, per precision
            for (int mx = 0; mx < 2; ++mx) {
                const size_t g0 = pg.gemm.size();
                int tiles = 0, gw = -1;
                for (int i : bylevel[L]) {
                    const OpRec& o = ops[i];
                    if (o.kind != K_GEMM || (int)o.mixed != mx || o.cls != cls) continue;
                    GemmOp g = make_gemm_op(o);
                    tiles += gemm_tiles_shape(g.m, g.n, 1);
                    pg.gemm.push_back(g);
                    gw = std::max(gw, o.wait_other);
                }
                if (pg.gemm.size() > g0) {
                    Launch gl = mk(0, g0, (int)(pg.gemm.size() - g0), tiles, mx, 0, 0, 0, cls, L, gw);
                    assign_shape(pg, gl);
                    pg.launches.push_back(gl);
                }
            }
            // sums
            {
                const size_t a0 = pg.add.size();
                size_t maxe = 0;
                int aw = -1;
                for (int i : bylevel[L]) {
                    const OpRec& o = ops[i];
                    if (o.kind != K_ADD || o.cls != cls) continue;
                    if (o.ins.size() > (size_t)kMaxAdd) {
                        pg.error = "internal: a block sum has more than 17 inputs";
                        return pg;
                    }
                    AddOp a = make_add_op(o);
                    maxe = std::max(maxe, (size_t)a.rows * a.cols);
                    pg.add.push_back(a);
                    aw = std::max(aw, o.wait_other);
                }
                if (pg.add.size() > a0)
                    pg.launches.push_back(mk(4, a0, (int)(pg.add.size() - a0), 0, 0, 0, 0, maxe, cls, L, aw));
            }
            // block norms
            for (int i : bylevel[L]) {
                const OpRec& o = ops[i];
                if (o.kind != K_NORM || o.cls != cls) continue;
                const size_t n0 = pg.norm.size();
                for (auto& x : o.ins) {
                    NormJob j;
                    memset(&j, 0, sizeof j);
                    j.X = x.second.p;
                    j.rows = x.second.r;
                    j.cols = x.second.c;
                    j.out = reinterpret_cast<double*>(o.D.p) + (int)x.first.x;
                    pg.norm.push_back(j);
                }
                pg.launches.push_back(mk(5, n0, (int)(pg.norm.size() - n0), 0, 0, 0, 0, 0, cls, L, o.wait_other));
            }
        }
    }
    // cross-stream events: a launch that waits for level W of the other stream
    // waits on an event recorded after that stream's last launch at level <= W
    {
        std::vector<int> last_idx[2];
        std::vector<int> last_of_level[2];
        for (int c = 0; c < 2; ++c) last_of_level[c].assign(nlevels, -1);
        for (int i = 0; i < (int)pg.launches.size(); ++i) {
            const Launch& L = pg.launches[i];
            if (L.type == 7) continue;     // independent of every other launch
            last_of_level[L.cls][L.level] = i;
        }
        for (int c = 0; c < 2; ++c)
            for (int l = 1; l < nlevels; ++l)
                if (last_of_level[c][l] < 0) last_of_level[c][l] = last_of_level[c][l - 1];
        for (auto& L : pg.launches) {
            if (L.wait_level < 0) continue;
            const int o = 1 - L.cls;
            const int src = last_of_level[o][std::min(L.wait_level, nlevels - 1)];
            if (src < 0) continue;
            Launch& S = pg.launches[src];
            if (S.rec_event < 0) S.rec_event = pg.n_events++;
            L.wait_event = S.rec_event;
        }
    }
    for (Launch& L : pg.launches) {
        if (L.type == 0) {
            gemm_work(pg.gemm.data() + L.off, L.count, L.flops, L.bytes);
        } else if (L.type == 6) {
            for (int q = 0; q < L.count; ++q) {
                const InvJob& j = pg.inv[L.off + q];
                const int np = (j.d + kInvNB - 1) / kInvNB;
                if (L.panel > np) continue;
                const double pnc = L.panel > 0 ? std::min(kInvNB, j.d - (L.panel - 1) * kInvNB) : 0;
                const double nc = L.panel < np ? std::min(kInvNB, j.d - L.panel * kInvNB) : 0;
                L.flops += 8.0 * ((double)j.d * j.d * pnc + (double)j.d * nc * nc);
                L.bytes += 16.0 * (2.0 * j.d * j.d + (double)j.d * kInvNB);
            }
        } else if (L.type == 4) {
            for (int q = 0; q < L.count; ++q) {
                const AddOp& a = pg.add[L.off + q];
                L.flops += 8.0 * a.rows * a.cols * a.nin;
                L.bytes += 16.0 * a.rows * a.cols * (a.nin + 1);
            }
        }
    }
    return pg;
}

}  // namespace

// ---------------------------------------------------------------------------
// Handle: one or more instances (a batch of uneven BT/BTA solves) that share
// one workspace allocation and one joint schedule.
// ---------------------------------------------------------------------------
struct Instance {
    Dims D{};
    bt_desc desc{};
    std::vector<int> bounds;
    size_t ws_begin = 0, ws_end = 0;   // byte range of this instance in the workspace
    bool factored = false;
    bt_blocks A_used{}, XR_used{};
};

struct bt_si_sq_plan {
    std::vector<Instance> inst;
    hipStream_t stream = nullptr;     // the caller's stream (main stream)
    hipStream_t astream = nullptr;    // internal stream for the critical A-chain
    hipEvent_t ev_start = nullptr, ev_end = nullptr;
    // All device memory of the handle is one block: [workspace | inverse
    // scratch | status word | arena for the uploaded operation lists], either
    // allocated at create (own_block) or given by the caller.
    char* block = nullptr;
    bool own_block = true;
    char* ws = nullptr;
    size_t ws_bytes = 0;
    char* inv_pool = nullptr;
    size_t inv_bytes = 0;
    DevStatus* status = nullptr;
    char* arena = nullptr;
    size_t arena_bytes = 0, arena_used = 0;
    std::string err;
    int32_t last_launches = 0;
    bool use_graph = false;               // BT_GRAPH on every instance
    hipStream_t gstream = nullptr;        // private stream graphs are captured on and replayed from
    hipEvent_t ev_pre = nullptr, ev_post = nullptr;
    struct Cached {
        std::vector<uint64_t> key;
        uint64_t stamp = 0;
        Program prog;
        std::vector<double*> norm_out;    // per selected instance (mixed check), or null
        std::vector<int> sel;             // instances of this program
        char* dev = nullptr;
        size_t dev_bytes = 0;
        bool dev_own = false;             // dev allocated on its own (did not fit the arena)
        std::vector<char> host;           // host copy the upload reads (kept as long as dev)
        size_t off_gemm = 0, off_inv = 0, off_add = 0, off_norm = 0;
        size_t off_frec = 0, off_ftask = 0;
        std::vector<hipEvent_t> events;   // cross-stream events of the launch list
        hipGraphExec_t graph = nullptr;   // the launch list captured as a graph (BT_GRAPH)
    };
    std::vector<Cached> cache;            // small LRU of compiled programs
    uint64_t clock = 0;
    hipEvent_t upload_done = nullptr;
    // profiling
    bool profiling = false;
    std::vector<hipEvent_t> ev_pool;
    struct Pending { int kind; hipEvent_t a, b; double flops, bytes; };
    std::vector<Pending> pending;
    size_t ev_used = 0;
    bt_kernel_stat stats[BT_KERNEL_COUNT];
};

namespace {

constexpr size_t kMaxCached = 8;

bool same_blocks(const bt_blocks& x, const bt_blocks& y) { return memcmp(&x, &y, sizeof x) == 0; }

bt_status set_err(bt_si_sq_plan* h, bt_status st, const std::string& msg) {
    if (h) h->err = msg; else g_last_error = msg;
    return st;
}

bt_status hip_err(bt_si_sq_plan* h, hipError_t e, const char* where) {
    std::string m = std::string(where) + ": " + hipGetErrorString(e);
    return set_err(h, BT_ERR_HIP, m);
}

bool desc_bounds(const bt_desc* d, std::vector<int>& bounds, std::string& msg) {
    if (!d) { msg = "null descriptor"; return false; }
    if (d->n < 1 || d->a < 0) { msg = "need n >= 1, a >= 0"; return false; }
    if (d->n > 65535) { msg = "n above 65535 is not supported"; return false; }
    if (d->block_sizes) {
        for (int i = 0; i < d->n; ++i)
            if (d->block_sizes[i] < 1 || d->block_sizes[i] > kInvMaxDim) {
                msg = "block_sizes[" + std::to_string(i) + "] must lie in 1..1024";
                return false;
            }
    } else if (d->b < 1) {
        msg = "need b >= 1";
        return false;
    }
    if ((!d->block_sizes && d->b > kInvMaxDim) || d->a > kInvMaxDim) {
        msg = "block sizes above 1024 are not supported";
        return false;
    }
    if (d->precision != BT_FP64 && d->precision != BT_MIXED) { msg = "unknown precision"; return false; }
    if ((d->flags & BT_DIAG_ONLY) && d->precision == BT_MIXED) {
        msg = "BT_DIAG_ONLY needs BT_FP64: the mixed path's error estimate reads the off-diagonal blocks";
        return false;
    }
    if (d->flags & BT_FUSED) {
        int mx = d->a;
        if (d->block_sizes) {
            for (int i = 0; i < d->n; ++i) mx = std::max(mx, (int)d->block_sizes[i]);
        } else {
            mx = std::max(mx, (int)d->b);
        }
        if (mx > kFusedMaxDim) {
            msg = "BT_FUSED needs every diagonal block and the arrow tip of size at most 64";
            return false;
        }
        if (d->precision != BT_FP64 || (d->flags & BT_PLAIN)) {
            msg = "BT_FUSED needs BT_FP64 and no BT_PLAIN";
            return false;
        }
    }
    const int P = d->partitions;
    if (P < 1) { msg = "partitions must be >= 1"; return false; }
    if (d->reduced_parts < 0 || d->reduced_parts > 1024) {
        msg = "reduced_parts must lie in 0..1024";
        return false;
    }
    Dims D(d->n, d->b, d->a, d->block_sizes);
    if (d->part_bounds) {
        bounds.assign(d->part_bounds, d->part_bounds + P + 1);
    } else {
        if (P > 1 && d->n < 2 * P - 2) {
            char buf[128];
            snprintf(buf, sizeof buf, "P = %d partitions need n >= 2P - 2 = %d blocks", P, 2 * P - 2);
            msg = buf;
            return false;
        }
        bounds = auto_bounds(D, P);
    }
    return validate_bounds(D, bounds, msg);
}

// Build the operations of the selected instances (sel) into one list.
// With ws == nullptr the workspace is a fake base and offsets are assigned
// (dry run); otherwise each instance builds into its recorded range.
struct Built {
    std::vector<OpRec> ops;
    std::vector<double*> norm_out;
    double flops = 0;
    int fused_tasks = 0;
};

bool build_instances(std::vector<Instance>& inst, const std::vector<int>& sel, Mode mode,
                     char* ws, bool fp64_rerun, const bt_blocks* A, const bt_blocks* B,
                     const bt_blocks* XR, const bt_blocks* XL, Built& out, size_t* dry_total) {
    const bool dry = ws == nullptr;
    char* base = dry ? reinterpret_cast<char*>((uintptr_t)1 << 40) : ws;
    size_t run = 0;
    for (int i : sel) {
        Instance& I = inst[i];
        Builder bd;
        bd.D = I.D;
        bd.bounds = I.bounds;
        bd.reduced_parts = I.desc.reduced_parts > 0 ? I.desc.reduced_parts : 2;
        bd.mode = mode;
        const bool mixed_handle = I.desc.precision == BT_MIXED;
        bd.mixed_bulk = mixed_handle && !fp64_rerun;
        bd.check = mixed_handle;
        bd.plain = (I.desc.flags & BT_PLAIN) != 0;
        bd.antiH = (I.desc.flags & BT_SIGMA_ANTIHERMITIAN) != 0;
        bd.diag_only = (I.desc.flags & BT_DIAG_ONLY) != 0;
        bd.instance = i;
        if (!dry) {
            if (A) bd.Aext = A[i];
            if (B) bd.Bext = B[i];
            if (XR) bd.XRext = XR[i];
            if (XL) bd.XLext = XL[i];
        }
        bd.ws = base;
        bd.off = dry ? run : I.ws_begin;
        const size_t begin = bd.off;
        bd.build();
        if (dry) {
            I.ws_begin = begin;
            I.ws_end = (bd.off + 255) & ~(size_t)255;
            run = I.ws_end;
        } else if (bd.off > I.ws_end) {
            return false;
        }
        out.flops += bd.flops;
        out.norm_out.push_back(bd.check && bd.emitB() ? reinterpret_cast<double*>(bd.norm_out.p) : nullptr);
        const int task = (I.desc.flags & BT_FUSED) ? out.fused_tasks++ : -1;
        for (auto& o : bd.ops) {
            o.task = task;
            out.ops.push_back(std::move(o));
        }
    }
    if (dry_total) *dry_total = run;
    return true;
}

hipEvent_t next_event(bt_si_sq_plan* h) {
    if (h->ev_used == h->ev_pool.size()) {
        hipEvent_t ev;
        if (hipEventCreate(&ev) != hipSuccess) return nullptr;
        h->ev_pool.push_back(ev);
    }
    return h->ev_pool[h->ev_used++];
}

void collect_profile(bt_si_sq_plan* h) {
    for (auto& p : h->pending) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, p.a, p.b) != hipSuccess) continue;
        bt_kernel_stat& s = h->stats[p.kind];
        s.kind = p.kind;
        s.launches += 1;
        s.total_ms += ms;
        s.flops += p.flops;
        s.bytes += p.bytes;
    }
    h->pending.clear();
    h->ev_used = 0;
}

int kernel_kind(const Launch& L) {
    switch (L.type) {
        case 0: return L.mixed ? BT_KERNEL_PRODUCT_MIXED : BT_KERNEL_PRODUCT_FP64;
        case 5: return BT_KERNEL_NORM;
        case 6: return BT_KERNEL_INV_PANEL;
        case 7: return BT_KERNEL_FUSED;
        default: return BT_KERNEL_SUM;
    }
}

hipError_t enqueue_program(bt_si_sq_plan* h, bt_si_sq_plan::Cached& c, hipStream_t main);

// Run a compiled launch list: directly on the handle's stream, or (BT_GRAPH,
// not profiling) as a HIP graph.  The graph is captured at the list's first
// run from the same enqueue sequence on the handle's private graph stream
// (the caller's stream may be the null stream, which cannot be captured); the
// capture spans both streams of the sequence (the critical stream joins
// through ev_start and rejoins through ev_end).  The sequence holds kernel
// launches and event records/waits only: no memsets, no host copies.  A
// replay is ordered after the work already queued on the caller's stream and
// before anything queued there afterwards.
hipError_t run_program(bt_si_sq_plan* h, bt_si_sq_plan::Cached& c) {
    if (!h->use_graph || h->profiling) return enqueue_program(h, c, h->stream);
    hipError_t e = hipSuccess;
    if (!c.graph) {
        e = hipStreamBeginCapture(h->gstream, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return e;
        e = enqueue_program(h, c, h->gstream);
        hipGraph_t g = nullptr;
        hipError_t e2 = hipStreamEndCapture(h->gstream, &g);
        if (e == hipSuccess) e = e2;
        if (e == hipSuccess) e = hipGraphInstantiate(&c.graph, g, nullptr, nullptr, 0);
        if (g) hipGraphDestroy(g);
        if (e != hipSuccess) { c.graph = nullptr; return e; }
    }
    e = hipEventRecord(h->ev_pre, h->stream);
    if (e == hipSuccess) e = hipStreamWaitEvent(h->gstream, h->ev_pre, 0);
    if (e == hipSuccess) e = hipGraphLaunch(c.graph, h->gstream);
    if (e == hipSuccess) e = hipEventRecord(h->ev_post, h->gstream);
    if (e == hipSuccess) e = hipStreamWaitEvent(h->stream, h->ev_post, 0);
    h->last_launches = (int32_t)c.prog.launches.size();
    return e;
}

hipError_t enqueue_program(bt_si_sq_plan* h, bt_si_sq_plan::Cached& c, hipStream_t main) {
    const Program& pg = c.prog;
    GemmOp* dg = reinterpret_cast<GemmOp*>(c.dev + c.off_gemm);
    InvJob* dj = reinterpret_cast<InvJob*>(c.dev + c.off_inv);
    AddOp* da = reinterpret_cast<AddOp*>(c.dev + c.off_add);
    NormJob* dn = reinterpret_cast<NormJob*>(c.dev + c.off_norm);
    hipError_t e = hipSuccess;
    if (h->profiling && h->ev_used + 2 * pg.launches.size() > 200000) {
        // bound the number of outstanding events: fold in what has finished
        hipStreamSynchronize(main);
        hipStreamSynchronize(h->astream);
        collect_profile(h);
    }
    // the critical stream starts after everything already queued on the main stream
    e = hipEventRecord(h->ev_start, main);
    if (e == hipSuccess) e = hipStreamWaitEvent(h->astream, h->ev_start, 0);
    if (e != hipSuccess) return e;
    for (const Launch& L : pg.launches) {
        // profiling runs every launch on the main stream, one after another,
        // so that each launch's events time the kernel alone
        hipStream_t s = (L.cls && !h->profiling) ? h->astream : main;
        if (L.wait_event >= 0) {
            e = hipStreamWaitEvent(s, c.events[L.wait_event], 0);
            if (e != hipSuccess) return e;
        }
        hipEvent_t ea = nullptr, eb = nullptr;
        if (h->profiling) {
            ea = next_event(h);
            eb = next_event(h);
            if (ea) hipEventRecord(ea, s);
        }
        switch (L.type) {
            case 0: e = launch_gemm_shape(dg + L.off, L.count, L.tiles, L.mixed != 0, L.shape, s); break;
            case 4: e = launch_add(da + L.off, L.count, L.maxelems, s); break;
            case 5: e = launch_norms(dn + L.off, L.count, s); break;
            case 6: e = launch_inv_step(dj + L.off, L.count, L.maxd, L.panel, L.tiles, h->status, s); break;
            case 7:
                e = launch_fused(reinterpret_cast<const FusedTask*>(c.dev + c.off_ftask) + L.off, L.count,
                                 reinterpret_cast<const FusedRec*>(c.dev + c.off_frec), h->status, s);
                break;
        }
        if (e != hipSuccess) return e;
        if (h->profiling && ea && eb) {
            hipEventRecord(eb, s);
            h->pending.push_back({kernel_kind(L), ea, eb, L.flops, L.bytes});
        }
        if (L.rec_event >= 0) {
            e = hipEventRecord(c.events[L.rec_event], s);
            if (e != hipSuccess) return e;
        }
    }
    // the solve is complete when the main stream is
    e = hipEventRecord(h->ev_end, h->astream);
    if (e == hipSuccess) e = hipStreamWaitEvent(main, h->ev_end, 0);
    h->last_launches = (int32_t)pg.launches.size();
    return e;
}

std::vector<uint64_t> make_key(Mode mode, bool fp64_rerun, const std::vector<int>& sel,
                               const bt_blocks* A, const bt_blocks* B, const bt_blocks* XR,
                               const bt_blocks* XL) {
    std::vector<uint64_t> k;
    k.push_back((uint64_t)mode | ((uint64_t)fp64_rerun << 8));
    auto put = [&](const bt_blocks* arr, int i) {
        if (!arr) { for (int q = 0; q < 6; ++q) k.push_back(0); return; }
        const bt_blocks& b = arr[i];
        k.push_back((uint64_t)b.diag); k.push_back((uint64_t)b.upper); k.push_back((uint64_t)b.lower);
        k.push_back((uint64_t)b.arrow_right); k.push_back((uint64_t)b.arrow_bottom); k.push_back((uint64_t)b.tip);
    };
    for (int i : sel) {
        k.push_back((uint64_t)i);
        put(A, i); put(B, i); put(XR, i); put(XL, i);
    }
    return k;
}

// Device bytes of a compiled program's operation lists (each array starting
// on a 256-byte boundary, as prepare_and_run lays them out).
struct ProgLayout {
    size_t off_inv, off_add, off_norm, off_frec, off_ftask, total;
};
ProgLayout program_layout(const Program& pg) {
    ProgLayout L;
    L.off_inv = align256(pg.gemm.size() * sizeof(GemmOp));
    L.off_add = align256(L.off_inv + pg.inv.size() * sizeof(InvJob));
    L.off_norm = align256(L.off_add + pg.add.size() * sizeof(AddOp));
    L.off_frec = align256(L.off_norm + pg.norm.size() * sizeof(NormJob));
    L.off_ftask = align256(L.off_frec + pg.frec.size() * sizeof(FusedRec));
    L.total = L.off_ftask + pg.ftask.size() * sizeof(FusedTask) + 256;
    return L;
}

size_t program_bytes(const Program& pg) { return program_layout(pg).total; }

// Layout of a handle's device block (see bt_si_sq_plan): workspace, inverse
// scratch, status word, then room for kArenaPrograms operation lists the size
// of the fused solve's (the largest a handle compiles: selected solves and
// factors take subsets of it, FP64 re-runs the same).
constexpr size_t kArenaPrograms = 4;
struct BlockLayout {
    size_t inv_off, status_off, arena_off, arena_bytes, total;
};
BlockLayout block_layout(size_t ws_bytes, size_t inv_bytes, size_t prog_bytes) {
    BlockLayout L;
    L.inv_off = align256(ws_bytes);
    L.status_off = L.inv_off + align256(std::max<size_t>(inv_bytes, 256));
    L.arena_off = L.status_off + 256;
    L.arena_bytes = kArenaPrograms * align256(prog_bytes);
    L.total = L.arena_off + L.arena_bytes;
    return L;
}

void free_cached(bt_si_sq_plan* h, bt_si_sq_plan::Cached& c) {
    if (c.dev) {
        // the launch list's kernels may still read it on either stream
        hipStreamSynchronize(h->stream);
        hipStreamSynchronize(h->astream);
        if (c.dev_own) hipFree(c.dev);
        c.dev = nullptr;
        c.dev_own = false;
    }
    if (c.graph) {
        hipStreamSynchronize(h->stream);
        if (h->gstream) hipStreamSynchronize(h->gstream);
        hipGraphExecDestroy(c.graph);
        c.graph = nullptr;
    }
    for (auto ev : c.events) hipEventDestroy(ev);
    c.events.clear();
}

// Build (or reuse) and enqueue the program of the selected instances.
bt_status prepare_and_run(bt_si_sq_plan* h, Mode mode, const std::vector<int>& sel,
                          const bt_blocks* A, const bt_blocks* B, const bt_blocks* XR,
                          const bt_blocks* XL, bool fp64_rerun, bt_si_sq_plan::Cached** used) {
    std::vector<uint64_t> key = make_key(mode, fp64_rerun, sel, A, B, XR, XL);
    bt_si_sq_plan::Cached* c = nullptr;
    for (auto& x : h->cache)
        if (x.key == key) { c = &x; break; }
    if (!c) {
        Built bt;
        if (!build_instances(h->inst, sel, mode, h->ws, fp64_rerun, A, B, XR, XL, bt, nullptr))
            return set_err(h, BT_ERR_INVALID, "internal: workspace layout changed");
        bool plain = true;
        for (int i : sel) plain = plain && (h->inst[i].desc.flags & BT_PLAIN);
        int nl = levelize(bt.ops, plain);
        Program pg = compile(bt.ops, nl, h->inv_pool);
        if (!pg.error.empty()) return set_err(h, BT_ERR_INVALID, pg.error);
        if (pg.inv_scratch_bytes > h->inv_bytes)
            return set_err(h, BT_ERR_INVALID, "internal: inverse scratch too small");
        pg.flops = bt.flops;
        const ProgLayout PL = program_layout(pg);
        const size_t total = PL.total;
        // Device room for the lists: the handle's arena, taken in order; when
        // it is full every cached program is dropped (after its streams are
        // idle) and the arena starts over.  A list larger than the whole
        // arena gets an allocation of its own.
        const size_t need = align256(total);
        if (h->arena_used + need > h->arena_bytes && need <= h->arena_bytes) {
            for (auto& x : h->cache) free_cached(h, x);
            h->cache.clear();
            h->arena_used = 0;
        }
        // slot: a free one, else the least recently used
        if (h->cache.size() < kMaxCached) {
            h->cache.emplace_back();
            c = &h->cache.back();
        } else {
            c = &h->cache[0];
            for (auto& x : h->cache)
                if (x.stamp < c->stamp) c = &x;
            free_cached(h, *c);
            c->key.clear();
            c->dev_bytes = 0;
        }
        hipError_t e = hipSuccess;
        if (h->arena_used + need <= h->arena_bytes) {
            c->dev = h->arena + h->arena_used;
            h->arena_used += need;
            c->dev_own = false;
        } else {
            e = hipMalloc(&c->dev, total);
            if (e != hipSuccess) { c->dev = nullptr; return set_err(h, BT_ERR_OOM, "operation list allocation failed"); }
            c->dev_own = true;
        }
        c->dev_bytes = total;
        c->host.assign(total, 0);
        char* stage = c->host.data();
        auto put = [&](size_t off, const void* src, size_t bytes) { if (bytes) memcpy(stage + off, src, bytes); };
        put(0, pg.gemm.data(), pg.gemm.size() * sizeof(GemmOp));
        put(PL.off_inv, pg.inv.data(), pg.inv.size() * sizeof(InvJob));
        put(PL.off_add, pg.add.data(), pg.add.size() * sizeof(AddOp));
        put(PL.off_norm, pg.norm.data(), pg.norm.size() * sizeof(NormJob));
        put(PL.off_frec, pg.frec.data(), pg.frec.size() * sizeof(FusedRec));
        put(PL.off_ftask, pg.ftask.data(), pg.ftask.size() * sizeof(FusedTask));
        e = hipMemcpyAsync(c->dev, stage, total, hipMemcpyHostToDevice, h->stream);
        if (e != hipSuccess) return hip_err(h, e, "hipMemcpyAsync(op list)");
        e = hipEventRecord(h->upload_done, h->stream);
        if (e != hipSuccess) return hip_err(h, e, "hipEventRecord");
        for (int i = 0; i < pg.n_events; ++i) {
            hipEvent_t ev;
            e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
            if (e != hipSuccess) return hip_err(h, e, "hipEventCreate");
            c->events.push_back(ev);
        }
        c->prog = std::move(pg);
        c->norm_out = bt.norm_out;
        c->sel = sel;
        c->off_gemm = 0;
        c->off_inv = PL.off_inv;
        c->off_add = PL.off_add;
        c->off_norm = PL.off_norm;
        c->off_frec = PL.off_frec;
        c->off_ftask = PL.off_ftask;
        c->key = key;
    }
    c->stamp = ++h->clock;
    hipError_t e = run_program(h, *c);
    if (e != hipSuccess) return hip_err(h, e, "kernel launch");
    if (used) *used = c;
    return BT_OK;
}

// Error estimate of a mixed-path result from the FP64 selected residuals:
//   est = max(rho_R, rho_L) * nA * nG
//   rho_R = max_i ||R^R_i||_F / sqrt(d_i)       (relative residual of A X = I)
//   rho_L = max_i ||R^<_i||_F / (nA * max_i ||X^<_ii||_F)
//   nA = max_i ||A_ii||_F / sqrt(d_i),  nG = max_i ||X^R_ii||_F
// i.e. a relative residual times a blockwise estimate of ||A|| ||A^-1||.
bt_status read_estimates(bt_si_sq_plan* h, bt_si_sq_plan::Cached& c, std::vector<double>& est) {
    hipError_t e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return hip_err(h, e, "hipStreamSynchronize");
    est.assign(c.sel.size(), 0.0);
    for (size_t q = 0; q < c.sel.size(); ++q) {
        if (!c.norm_out[q]) continue;
        const Instance& I = h->inst[c.sel[q]];
        const int rows = I.D.n + (I.D.a > 0 ? 1 : 0);
        std::vector<double> v(5 * (I.D.n + 1), 0.0);
        e = hipMemcpyAsync(v.data(), c.norm_out[q], v.size() * sizeof(double), hipMemcpyDeviceToHost, h->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
        if (e != hipSuccess) return hip_err(h, e, "residual readback");
        double nA = 0, nG = 0, nL = 0, rR = 0, rL = 0;
        for (int i = 0; i < rows; ++i) {
            const double sd = std::sqrt((double)I.D.dim(i));
            nA = std::max(nA, v[5 * i + 4] / sd);
            nG = std::max(nG, v[5 * i + 2]);
            nL = std::max(nL, v[5 * i + 3]);
            rR = std::max(rR, v[5 * i + 0] / sd);
            rL = std::max(rL, v[5 * i + 1]);
        }
        rL = (nA * nL > 0) ? rL / (nA * nL) : rL;
        double x = std::max(rR, rL) * nA * nG;
        if (!(x == x)) x = INFINITY;
        est[q] = x;
    }
    return BT_OK;
}

// Run the selected instances; for mixed instances estimate the error and
// re-run in FP64 those above their tolerance.
bt_status run_instances(bt_si_sq_plan* h, Mode mode, const std::vector<int>& sel,
                        const bt_blocks* A, const bt_blocks* B, const bt_blocks* XR,
                        const bt_blocks* XL, double* err, int* fb) {
    bt_si_sq_plan::Cached* c = nullptr;
    bt_status st = prepare_and_run(h, mode, sel, A, B, XR, XL, false, &c);
    if (st != BT_OK) return st;
    for (size_t q = 0; q < sel.size(); ++q) {
        if (err) err[sel[q]] = 0.0;
        if (fb) fb[sel[q]] = 0;
    }
    bool any_mixed = false;
    for (int i : sel) any_mixed |= h->inst[i].desc.precision == BT_MIXED;
    if (!any_mixed || mode == MODE_FACTOR) return BT_OK;
    std::vector<double> est;
    st = read_estimates(h, *c, est);
    if (st != BT_OK) return st;
    std::vector<int> redo;
    for (size_t q = 0; q < sel.size(); ++q) {
        const Instance& I = h->inst[sel[q]];
        if (I.desc.precision == BT_MIXED && est[q] > I.desc.tol) redo.push_back(sel[q]);
        if (err) err[sel[q]] = est[q];
    }
    if (redo.empty()) return BT_OK;
    // The re-run repeats the whole solve with FP64 products: after a mixed
    // factor the stored S, T and X^R carry FP32 rounding, so a selected solve
    // alone (MODE_SQ) on them could not remove an error that comes from the
    // A-chain.  A and X^R are the ones the factor call used.
    st = prepare_and_run(h, MODE_BOTH, redo, A, B, XR, XL, true, &c);
    if (st != BT_OK) return st;
    st = read_estimates(h, *c, est);
    if (st != BT_OK) return st;
    int above = -1;
    for (size_t q = 0; q < redo.size(); ++q) {
        if (err) err[redo[q]] = est[q];
        if (fb) fb[redo[q]] = 1;
        if (above < 0 && est[q] > h->inst[redo[q]].desc.tol) above = redo[q];
    }
    if (above >= 0) {
        char buf[200];
        snprintf(buf, sizeof buf, "instance %d: error estimate %.3e of the FP64 re-run is above tol %.3e "
                 "(results written)", above, est[std::find(redo.begin(), redo.end(), above) - redo.begin()],
                 h->inst[above].desc.tol);
        return set_err(h, BT_ERR_TOLERANCE, buf);
    }
    return BT_OK;
}

bool check_blocks(const Dims& D, const bt_blocks* m, bool need, std::string& msg, const char* name,
                  bool diag_only = false) {
    if (!m) {
        if (need) { msg = std::string(name) + " is null"; return false; }
        return true;
    }
    if (diag_only) {
        if (!m->diag || (D.a > 0 && !m->tip)) {
            msg = std::string(name) + ": diag (and tip for a > 0) pointers missing";
            return false;
        }
        return true;
    }
    if (!m->diag || (D.n > 1 && (!m->upper || !m->lower))) {
        msg = std::string(name) + ": diag/upper/lower pointers missing";
        return false;
    }
    if (D.a > 0 && (!m->arrow_right || !m->arrow_bottom || !m->tip)) {
        msg = std::string(name) + ": arrow/tip pointers missing for a > 0";
        return false;
    }
    return true;
}

bool check_optional_blocks(const Dims& D, const bt_blocks* m, std::string& msg, const char* name,
                           bool diag_only = false) {
    if (!m) return true;
    const bool any = m->diag || m->upper || m->lower || m->arrow_right || m->arrow_bottom || m->tip;
    if (!any) return true;   // all null: X^R stays in the workspace
    return check_blocks(D, m, true, msg, name, diag_only);
}

bool diag_only_of(const Instance& I) { return (I.desc.flags & BT_DIAG_ONLY) != 0; }

// Validate descriptors and size the workspace of a batch (dry run).
bt_status plan_instances(int count, const bt_desc* descs, std::vector<Instance>& inst,
                         size_t& ws_bytes, size_t& inv_bytes, double* flops, size_t* prog_bytes = nullptr) {
    if (count < 1 || !descs) return set_err(nullptr, BT_ERR_INVALID, "need count >= 1 descriptors");
    inst.assign(count, Instance{});
    std::string msg;
    for (int i = 0; i < count; ++i) {
        std::vector<int> bounds;
        if (!desc_bounds(&descs[i], bounds, msg)) {
            if (count > 1) msg = "instance " + std::to_string(i) + ": " + msg;
            return set_err(nullptr, BT_ERR_INVALID, msg);
        }
        inst[i].D = Dims(descs[i].n, descs[i].b, descs[i].a, descs[i].block_sizes);
        inst[i].desc = descs[i];
        inst[i].desc.part_bounds = nullptr;
        inst[i].desc.block_sizes = nullptr;   // the sizes live in inst[i].D
        if (!(inst[i].desc.tol > 0)) inst[i].desc.tol = 1e-4;
        inst[i].bounds = bounds;
    }
    std::vector<int> sel(count);
    for (int i = 0; i < count; ++i) sel[i] = i;
    Built bt;
    size_t total = 0;
    build_instances(inst, sel, MODE_BOTH, nullptr, false, nullptr, nullptr, nullptr, nullptr, bt, &total);
    if (flops) *flops = bt.flops;
    ws_bytes = total + 256;
    bool plain = true;
    for (auto& I : inst) plain = plain && (I.desc.flags & BT_PLAIN);
    int nl = levelize(bt.ops, plain);
    Program pg = compile(bt.ops, nl, reinterpret_cast<char*>((uintptr_t)3 << 40));
    if (!pg.error.empty()) return set_err(nullptr, BT_ERR_INVALID, pg.error);
    inv_bytes = pg.inv_scratch_bytes;
    if (prog_bytes) *prog_bytes = program_bytes(pg);
    return BT_OK;
}

// ext: the caller's device block (ext_bytes at least the layout's total), or
// null to allocate it here.
bt_status create_handle(int count, const bt_desc* descs, void* hip_stream, bt_si_sq_handle* out,
                        void* ext = nullptr, size_t ext_bytes = 0) {
    if (!out) return set_err(nullptr, BT_ERR_INVALID, "out is null");
    *out = nullptr;
    std::unique_ptr<bt_si_sq_plan> h(new bt_si_sq_plan());
    size_t prog = 0;
    bt_status st = plan_instances(count, descs, h->inst, h->ws_bytes, h->inv_bytes, nullptr, &prog);
    if (st != BT_OK) return st;
    const BlockLayout L = block_layout(h->ws_bytes, h->inv_bytes, prog);
    h->stream = reinterpret_cast<hipStream_t>(hip_stream);
    hipError_t e = hipSuccess;
    if (ext) {
        if (ext_bytes < L.total)
            return set_err(nullptr, BT_ERR_INVALID, "workspace of " + std::to_string(ext_bytes) +
                           " bytes is smaller than the " + std::to_string(L.total) + " this handle needs");
        if (reinterpret_cast<uintptr_t>(ext) & 255)
            return set_err(nullptr, BT_ERR_INVALID, "workspace must be 256-byte aligned");
        h->block = static_cast<char*>(ext);
        h->own_block = false;
    } else {
        e = hipMalloc(&h->block, L.total);
        if (e != hipSuccess) { hipGetLastError(); return set_err(nullptr, BT_ERR_OOM, "workspace allocation failed"); }
        h->own_block = true;
    }
    h->ws = h->block;
    h->inv_pool = h->block + L.inv_off;
    h->status = reinterpret_cast<DevStatus*>(h->block + L.status_off);
    h->arena = h->block + L.arena_off;
    h->arena_bytes = L.arena_bytes;
    h->arena_used = 0;
    // status word and the identity blocks of the residual check (each
    // instance's first two slots), ordered on the handle's stream only
    std::vector<double2> host;
    DevStatus z{0, 0};
    e = hipMemcpyAsync(h->status, &z, sizeof z, hipMemcpyHostToDevice, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    for (auto& I : h->inst) {
        if (e != hipSuccess) break;
        const int b = I.D.b, a = std::max(I.D.a, 1);
        host.assign((size_t)b * b, cplx(0));
        for (int i = 0; i < b; ++i) host[(size_t)i * b + i] = cplx(1);
        e = hipMemcpyAsync(h->ws + I.ws_begin, host.data(), host.size() * sizeof(double2), hipMemcpyHostToDevice,
                           h->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
        const size_t offa = I.ws_begin + (((size_t)b * b * sizeof(double2) + 255) & ~(size_t)255);
        host.assign((size_t)a * a, cplx(0));
        for (int i = 0; i < a; ++i) host[(size_t)i * a + i] = cplx(1);
        if (e == hipSuccess)
            e = hipMemcpyAsync(h->ws + offa, host.data(), host.size() * sizeof(double2), hipMemcpyHostToDevice,
                               h->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    }
    if (e == hipSuccess) e = hipEventCreateWithFlags(&h->upload_done, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&h->ev_start, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&h->ev_end, hipEventDisableTiming);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&h->astream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&h->gstream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&h->ev_pre, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&h->ev_post, hipEventDisableTiming);
    h->use_graph = !h->inst.empty();
    for (auto& I : h->inst) h->use_graph = h->use_graph && (I.desc.flags & BT_GRAPH);
    if (e != hipSuccess) {
        if (h->own_block) hipFree(h->block);
        return hip_err(nullptr, e, "create");
    }
    *out = h.release();
    return BT_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

size_t bt_si_sq_workspace_bytes(const bt_desc* desc) {
    return bt_si_sq_batch_workspace_bytes(1, desc);
}

size_t bt_si_sq_batch_workspace_bytes(int32_t count, const bt_desc* descs) {
    std::vector<Instance> inst;
    size_t ws = 0, inv = 0, prog = 0;
    if (plan_instances(count, descs, inst, ws, inv, nullptr, &prog) != BT_OK) return 0;
    return block_layout(ws, inv, prog).total;
}

bt_status bt_si_sq_partition_bounds(const bt_desc* desc, int32_t* bounds_out) {
    std::vector<int> bounds;
    std::string msg;
    if (!bounds_out) return set_err(nullptr, BT_ERR_INVALID, "bounds_out is null");
    if (!desc_bounds(desc, bounds, msg)) return set_err(nullptr, BT_ERR_INVALID, msg);
    for (size_t i = 0; i < bounds.size(); ++i) bounds_out[i] = bounds[i];
    return BT_OK;
}

bt_status bt_si_sq_flops(const bt_desc* desc, double* executed, double* useful) {
    std::vector<Instance> inst;
    size_t ws = 0, inv = 0;
    double fe = 0, fu = 0;
    bt_status st = plan_instances(1, desc, inst, ws, inv, &fe);
    if (st != BT_OK) return st;
    bt_desc seq = *desc;
    seq.partitions = 1;
    seq.part_bounds = nullptr;
    seq.flags &= ~BT_SIGMA_ANTIHERMITIAN;   // the reference count takes no symmetry
    st = plan_instances(1, &seq, inst, ws, inv, &fu);
    if (st != BT_OK) return st;
    if (executed) *executed = fe;
    if (useful) *useful = fu;
    return BT_OK;
}

bt_status bt_si_sq_create(const bt_desc* desc, void* hip_stream, bt_si_sq_handle* out) {
    return create_handle(1, desc, hip_stream, out);
}

bt_status bt_si_sq_batch_create(int32_t count, const bt_desc* descs, void* hip_stream,
                                bt_si_sq_handle* out) {
    return create_handle(count, descs, hip_stream, out);
}

bt_status bt_si_sq_batch_create_in(int32_t count, const bt_desc* descs, void* hip_stream, void* workspace,
                                   size_t workspace_bytes, bt_si_sq_handle* out) {
    if (!workspace) {
        if (out) *out = nullptr;
        return set_err(nullptr, BT_ERR_INVALID, "workspace is null");
    }
    return create_handle(count, descs, hip_stream, out, workspace, workspace_bytes);
}

bt_status bt_si_sq_factor(bt_si_sq_handle h, const bt_blocks* A, bt_blocks* XR) {
    if (!h) return set_err(nullptr, BT_ERR_INVALID, "null handle");
    if (h->inst.size() != 1) return set_err(h, BT_ERR_INVALID, "factor takes a single-instance handle");
    Instance& I = h->inst[0];
    std::string msg;
    if (!check_blocks(I.D, A, true, msg, "A") || !check_optional_blocks(I.D, XR, msg, "XR", diag_only_of(I)))
        return set_err(h, BT_ERR_INVALID, msg);
    bt_status st = run_instances(h, MODE_FACTOR, {0}, A, nullptr, XR, nullptr, nullptr, nullptr);
    if (st == BT_OK) {
        I.factored = true;
        I.A_used = *A;
        I.XR_used = XR ? *XR : bt_blocks{};
    }
    return st;
}

bt_status bt_si_sq_selected_solve(bt_si_sq_handle h, const bt_blocks* B, bt_blocks* XL,
                                  double* err_estimate, int* used_fp64_fallback) {
    if (!h) return set_err(nullptr, BT_ERR_INVALID, "null handle");
    if (err_estimate) *err_estimate = 0.0;
    if (used_fp64_fallback) *used_fp64_fallback = 0;
    if (h->inst.size() != 1) return set_err(h, BT_ERR_INVALID, "selected_solve takes a single-instance handle");
    Instance& I = h->inst[0];
    if (!I.factored) return set_err(h, BT_ERR_STATE, "selected_solve before factor");
    std::string msg;
    if (!check_blocks(I.D, B, true, msg, "B") || !check_blocks(I.D, XL, true, msg, "XL", diag_only_of(I)))
        return set_err(h, BT_ERR_INVALID, msg);
    return run_instances(h, MODE_SQ, {0}, &I.A_used, B, &I.XR_used, XL, err_estimate, used_fp64_fallback);
}

bt_status bt_si_sq_solve(bt_si_sq_handle h, const bt_blocks* A, const bt_blocks* B,
                         bt_blocks* XR, bt_blocks* XL, double* err_estimate, int* used_fp64_fallback) {
    if (!h) return set_err(nullptr, BT_ERR_INVALID, "null handle");
    if (h->inst.size() != 1) return set_err(h, BT_ERR_INVALID, "solve takes a single-instance handle");
    return bt_si_sq_batch_solve(h, A, B, XR, XL, err_estimate, used_fp64_fallback);
}

bt_status bt_si_sq_batch_solve(bt_si_sq_handle h, const bt_blocks* A, const bt_blocks* B,
                               bt_blocks* XR, bt_blocks* XL, double* err_estimates,
                               int* used_fp64_fallback) {
    if (!h) return set_err(nullptr, BT_ERR_INVALID, "null handle");
    const int count = (int)h->inst.size();
    if (err_estimates) for (int i = 0; i < count; ++i) err_estimates[i] = 0.0;
    if (used_fp64_fallback) for (int i = 0; i < count; ++i) used_fp64_fallback[i] = 0;
    if (!A || !B || !XL) return set_err(h, BT_ERR_INVALID, "A, B and XL are required");
    std::string msg;
    for (int i = 0; i < count; ++i) {
        const Dims& D = h->inst[i].D;
        const bool dg = diag_only_of(h->inst[i]);
        if (!check_blocks(D, &A[i], true, msg, "A") || !check_blocks(D, &B[i], true, msg, "B") ||
            !check_optional_blocks(D, XR ? &XR[i] : nullptr, msg, "XR", dg) ||
            !check_blocks(D, &XL[i], true, msg, "XL", dg)) {
            if (count > 1) msg = "instance " + std::to_string(i) + ": " + msg;
            return set_err(h, BT_ERR_INVALID, msg);
        }
    }
    std::vector<int> sel(count);
    for (int i = 0; i < count; ++i) sel[i] = i;
    bt_status st = run_instances(h, MODE_BOTH, sel, A, B, XR, XL, err_estimates, used_fp64_fallback);
    if (st == BT_OK || st == BT_ERR_TOLERANCE)   // results written either way
        for (int i = 0; i < count; ++i) {
            h->inst[i].factored = true;
            h->inst[i].A_used = A[i];
            h->inst[i].XR_used = XR ? XR[i] : bt_blocks{};
        }
    return st;
}

bt_status bt_si_sq_batch_selected_solve(bt_si_sq_handle h, const bt_blocks* B, bt_blocks* XL,
                                        double* err_estimates, int* used_fp64_fallback) {
    if (!h) return set_err(nullptr, BT_ERR_INVALID, "null handle");
    const int count = (int)h->inst.size();
    if (err_estimates) for (int i = 0; i < count; ++i) err_estimates[i] = 0.0;
    if (used_fp64_fallback) for (int i = 0; i < count; ++i) used_fp64_fallback[i] = 0;
    if (!B || !XL) return set_err(h, BT_ERR_INVALID, "B and XL are required");
    std::vector<int> sel;
    std::vector<bt_blocks> Au(count), XRu(count);
    std::string msg;
    for (int i = 0; i < count; ++i) {
        if (!XL[i].diag) continue;              // instance skipped
        const Instance& I = h->inst[i];
        if (!I.factored) {
            return set_err(h, BT_ERR_STATE, "instance " + std::to_string(i) + ": selected_solve before factor");
        }
        if (!check_blocks(I.D, &B[i], true, msg, "B") || !check_blocks(I.D, &XL[i], true, msg, "XL", diag_only_of(I)))
            return set_err(h, BT_ERR_INVALID, "instance " + std::to_string(i) + ": " + msg);
        sel.push_back(i);
    }
    for (int i = 0; i < count; ++i) { Au[i] = h->inst[i].A_used; XRu[i] = h->inst[i].XR_used; }
    if (sel.empty()) return BT_OK;
    return run_instances(h, MODE_SQ, sel, Au.data(), B, XRu.data(), XL, err_estimates, used_fp64_fallback);
}

int32_t bt_si_sq_batch_count(bt_si_sq_handle h) { return h ? (int32_t)h->inst.size() : 0; }

bt_status bt_si_sq_sync(bt_si_sq_handle h) {
    if (!h) return set_err(nullptr, BT_ERR_INVALID, "null handle");
    hipError_t e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return hip_err(h, e, "hipStreamSynchronize");
    DevStatus s{0, 0};
    e = hipMemcpyAsync(&s, h->status, sizeof s, hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return hip_err(h, e, "status readback");
    if (s.code != 0) {
        DevStatus z{0, 0};
        if (hipMemcpyAsync(h->status, &z, sizeof z, hipMemcpyHostToDevice, h->stream) == hipSuccess)
            hipStreamSynchronize(h->stream);
        const int inst = s.tag >> 16, blk = s.tag & 0xffff;
        const bool tip = inst < (int)h->inst.size() && blk == h->inst[inst].D.n;
        char buf[200];
        if (h->inst.size() > 1)
            snprintf(buf, sizeof buf, "singular or non-finite pivot while inverting diagonal block %d%s of instance %d",
                     blk, tip ? " (arrow tip)" : "", inst);
        else
            snprintf(buf, sizeof buf, "singular or non-finite pivot while inverting diagonal block %d%s",
                     blk, tip ? " (arrow tip)" : "");
        return set_err(h, BT_ERR_SINGULAR, buf);
    }
    h->err.clear();
    return BT_OK;
}

bt_status bt_si_sq_destroy(bt_si_sq_handle h) {
    if (!h) return BT_OK;
    hipStreamSynchronize(h->stream);
    hipStreamSynchronize(h->astream);
    if (h->gstream) hipStreamSynchronize(h->gstream);
    for (auto& c : h->cache) free_cached(h, c);
    if (h->upload_done) hipEventDestroy(h->upload_done);
    if (h->ev_start) hipEventDestroy(h->ev_start);
    if (h->ev_end) hipEventDestroy(h->ev_end);
    if (h->ev_pre) hipEventDestroy(h->ev_pre);
    if (h->ev_post) hipEventDestroy(h->ev_post);
    if (h->astream) hipStreamDestroy(h->astream);
    if (h->gstream) hipStreamDestroy(h->gstream);
    for (auto ev : h->ev_pool) hipEventDestroy(ev);
    if (h->own_block) hipFree(h->block);
    delete h;
    return BT_OK;
}

const char* bt_si_sq_last_error(bt_si_sq_handle h) {
    return h ? h->err.c_str() : g_last_error.c_str();
}

int32_t bt_si_sq_last_launch_count(bt_si_sq_handle h) { return h ? h->last_launches : 0; }

bt_status bt_si_sq_profile(bt_si_sq_handle h, int32_t enable) {
    if (!h) return set_err(nullptr, BT_ERR_INVALID, "null handle");
    hipError_t e = hipStreamSynchronize(h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->astream);
    if (e != hipSuccess) return hip_err(h, e, "hipStreamSynchronize");
    h->pending.clear();
    h->ev_used = 0;
    for (int k = 0; k < BT_KERNEL_COUNT; ++k) h->stats[k] = bt_kernel_stat{k, 0, 0.0, 0.0, 0.0};
    h->profiling = enable != 0;
    return BT_OK;
}

bt_status bt_si_sq_profile_stats(bt_si_sq_handle h, bt_kernel_stat* out, int32_t max_entries,
                                 int32_t* count) {
    if (!h || !count || (max_entries > 0 && !out)) return set_err(h, BT_ERR_INVALID, "bad arguments");
    hipError_t e = hipStreamSynchronize(h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->astream);
    if (e != hipSuccess) return hip_err(h, e, "hipStreamSynchronize");
    collect_profile(h);
    int32_t c = 0;
    for (int k = 0; k < BT_KERNEL_COUNT; ++k)
        if (h->stats[k].launches > 0 && c < max_entries) out[c++] = h->stats[k];
    *count = c;
    return BT_OK;
}

bt_status bt_si_sq_tune_table(int32_t* table, int32_t get) {
    if (!table) return set_err(nullptr, BT_ERR_INVALID, "tune_table: null table");
    static_assert(BT_TUNE_ENTRIES == 2 * kMClasses * kTClasses, "tuning table layout");
    static_assert(BT_TILE_SHAPES == kGemmShapes, "tile shape count");
    tune_init();
    if (!get) {
        for (int i = 0; i < BT_TUNE_ENTRIES; ++i)
            if (table[i] < -1 || table[i] >= kGemmShapes)
                return set_err(nullptr, BT_ERR_INVALID, "tune_table: entry out of range");
    }
    int i = 0;
    for (auto& a : g_tune)
        for (auto& b : a)
            for (auto& c : b) {
                if (get) table[i] = c.load();
                else c.store(table[i]);
                ++i;
            }
    return BT_OK;
}

bt_status bt_si_sq_autotune(void* hip_stream, char* report, size_t cap) {
    hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
    tune_init();
    constexpr int kMaxDim = 1024, kMaxOps = 4096;
    const size_t in_bytes = (size_t)kMaxDim * kMaxDim * sizeof(double2);
    const size_t out_bytes = (size_t)256 << 20;
    char* buf = nullptr;
    GemmOp* dops = nullptr;
    hipError_t e = hipMalloc(&buf, 2 * in_bytes + out_bytes);
    if (e != hipSuccess) { hipGetLastError(); return set_err(nullptr, BT_ERR_OOM, "autotune: scratch allocation failed"); }
    e = hipMalloc(&dops, kMaxOps * sizeof(GemmOp));
    if (e != hipSuccess) { hipGetLastError(); hipFree(buf); return set_err(nullptr, BT_ERR_OOM, "autotune: op list allocation failed"); }
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    if (e == hipSuccess) e = hipEventCreate(&ev0);
    if (e == hipSuccess) e = hipEventCreate(&ev1);
    if (e == hipSuccess) e = hipMemsetAsync(buf, 0, 2 * in_bytes + out_bytes, s);
    const double2* A = reinterpret_cast<const double2*>(buf);
    const double2* B = reinterpret_cast<const double2*>(buf + in_bytes);
    double2* out = reinterpret_cast<double2*>(buf + 2 * in_bytes);
    int found[2][kMClasses][kTClasses];
    for (auto& a : found) for (auto& b : a) for (auto& c : b) c = -1;
    std::string rep;
    std::vector<GemmOp> ops;
    for (int prec = 0; prec < 2 && e == hipSuccess; ++prec) {
        for (int mc = 1; mc < kMClasses && e == hipSuccess; ++mc) {
            const int m = 32 << mc;
            const long tpp = gemm_tiles_shape(m, m, 1);
            for (int tc = 0; tc < kTClasses && e == hipSuccess; ++tc) {
                const long target = 1L << tc;
                if (target < tpp) continue;
                const long nops = target / tpp;
                if (nops > kMaxOps || (size_t)nops * m * m * sizeof(double2) > out_bytes) continue;
                ops.assign(nops, GemmOp{});
                for (long q = 0; q < nops; ++q) {
                    GemmOp& g = ops[q];
                    memset(&g, 0, sizeof g);
                    g.D = out + (size_t)q * m * m;
                    g.ldd = m;
                    g.m = g.n = m;
                    g.nterms = 1;
                    g.mixed = prec;
                    g.t[0].A = A;
                    g.t[0].B = B;
                    g.t[0].lda = g.t[0].ldb = m;
                    g.t[0].k = m;
                    g.t[0].alpha = cplx(1.0);
                }
                float best_ms = 0.0f;
                int best = -1;
                float ms[kGemmShapes] = {0, 0, 0};
                for (int sh = 0; sh < kGemmShapes && e == hipSuccess; ++sh) {
                    int tiles = 0;
                    for (auto& g : ops) {
                        g.tile_begin = tiles;
                        g.tiles_n = gemm_tiles_n_shape(m, sh);
                        tiles += gemm_tiles_shape(m, m, sh);
                    }
                    e = hipMemcpyAsync(dops, ops.data(), ops.size() * sizeof(GemmOp), hipMemcpyHostToDevice, s);
                    if (e == hipSuccess) e = launch_gemm_shape(dops, (int)nops, tiles, prec != 0, sh, s);   // warm-up
                    if (e == hipSuccess) e = hipEventRecord(ev0, s);
                    constexpr int kReps = 3;
                    for (int r = 0; r < kReps && e == hipSuccess; ++r)
                        e = launch_gemm_shape(dops, (int)nops, tiles, prec != 0, sh, s);
                    if (e == hipSuccess) e = hipEventRecord(ev1, s);
                    if (e == hipSuccess) e = hipEventSynchronize(ev1);
                    if (e == hipSuccess) e = hipEventElapsedTime(&ms[sh], ev0, ev1);
                    ms[sh] /= kReps;
                    if (e == hipSuccess && (best < 0 || ms[sh] < best_ms)) { best = sh; best_ms = ms[sh]; }
                }
                if (e != hipSuccess || best < 0) break;
                // shapes within 3% of the fastest count as ties, broken toward the
                // larger tile (fewer tiles and launches; keeps repeated tunings stable)
                for (int sh = kGemmShapes - 1; sh >= 0; --sh)
                    if (ms[sh] <= 1.03f * best_ms) { best = sh; break; }
                found[prec][mc][tc] = best;
                char line[160];
                snprintf(line, sizeof line, "%d %d %d %d %.1f %.1f %.1f\n", prec, mc, tc, best,
                         1e3 * ms[0], 1e3 * ms[1], 1e3 * ms[2]);
                rep += line;
            }
        }
    }
    if (ev0) hipEventDestroy(ev0);
    if (ev1) hipEventDestroy(ev1);
    hipError_t e2 = hipStreamSynchronize(s);
    hipFree(dops);
    hipFree(buf);
    if (e == hipSuccess) e = e2;
    if (e != hipSuccess) return hip_err(nullptr, e, "autotune");
    for (int p = 0; p < 2; ++p)
        for (int mc = 0; mc < kMClasses; ++mc)
            for (int tc = 0; tc < kTClasses; ++tc)
                if (found[p][mc][tc] >= 0) g_tune[p][mc][tc].store(found[p][mc][tc]);
    if (report && cap > 0) {
        const size_t nbytes = std::min(cap - 1, rep.size());
        memcpy(report, rep.data(), nbytes);
        report[nbytes] = '\0';
    }
    return BT_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Diagnostic entry points (include/bt_si_sq_diag.h)
// ---------------------------------------------------------------------------
#include "../../include/bt_si_sq_diag.h"

extern "C" {

bt_status bt_si_sq_diag_gemm(int32_t m, int32_t n, int32_t k,
                             const double* alpha, const void* A, int32_t lda, int32_t opA,
                             const void* B, int32_t ldb, int32_t opB,
                             const double* beta, const void* C, int32_t ldc,
                             void* D, int32_t ldd, int32_t mixed, int32_t shape, void* hip_stream) {
    if (m < 0 || n < 0 || k < 0 || !alpha || !beta || !D || (k > 0 && (!A || !B)) ||
        shape < -1 || shape >= kGemmShapes)
        return set_err(nullptr, BT_ERR_INVALID, "diag_gemm: bad arguments");
    if (m == 0 || n == 0) return BT_OK;
    if (k > 0) {
        // the product kernel addresses each operand with 32-bit byte offsets
        const long long extA = opA ? (long long)(k - 1) * lda + m : (long long)(m - 1) * lda + k;
        const long long extB = opB ? (long long)(n - 1) * ldb + k : (long long)(k - 1) * ldb + n;
        if (extA * 16 >= (1ll << 31) || extB * 16 >= (1ll << 31))
            return set_err(nullptr, BT_ERR_INVALID, "diag_gemm: operands of 2 GiB or more are not supported");
    }
    hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
    GemmOp g;
    memset(&g, 0, sizeof g);
    g.D = reinterpret_cast<double2*>(D);
    g.C = reinterpret_cast<const double2*>(C);
    g.ldd = ldd;
    g.ldc = ldc;
    g.m = m;
    g.n = n;
    g.nterms = k > 0 ? 1 : 0;
    if (shape < 0) shape = pick_shape(mixed, std::max(m, n), gemm_tiles_shape(m, n, 1));
    g.tiles_n = gemm_tiles_n_shape(n, shape);
    g.tile_begin = 0;
    g.mixed = mixed;
    g.beta = cplx(beta[0], beta[1]);
    g.t[0].A = reinterpret_cast<const double2*>(A);
    g.t[0].B = reinterpret_cast<const double2*>(B);
    g.t[0].lda = lda;
    g.t[0].ldb = ldb;
    g.t[0].k = k;
    g.t[0].flags = (opA ? kTermAH : 0) | (opB ? kTermBH : 0);
    g.t[0].alpha = cplx(alpha[0], alpha[1]);
    GemmOp* dop = nullptr;
    hipError_t e = hipMalloc(&dop, sizeof g);
    if (e != hipSuccess) return hip_err(nullptr, e, "hipMalloc");
    e = hipMemcpyAsync(dop, &g, sizeof g, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = launch_gemm_shape(dop, 1, gemm_tiles_shape(m, n, shape), mixed != 0, shape, s);
    hipError_t e2 = hipStreamSynchronize(s);
    hipFree(dop);
    if (e != hipSuccess) return hip_err(nullptr, e, "diag_gemm launch");
    if (e2 != hipSuccess) return hip_err(nullptr, e2, "diag_gemm sync");
    return BT_OK;
}

bt_status bt_si_sq_diag_inverse(const void* src, void* dst, int32_t d, int32_t count,
                                int32_t* bad_index, void* hip_stream) {
    if (bad_index) *bad_index = -1;
    if (!src || !dst || d < 1 || d > kInvMaxDim || count < 0)
        return set_err(nullptr, BT_ERR_INVALID, "diag_inverse: bad arguments (1 <= d <= 1024)");
    if (count == 0) return BT_OK;
    hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
    std::vector<OpRec> ops;
    for (int i = 0; i < count; ++i) {
        OpRec o;
        o.kind = K_INV;
        o.C = MatRef{const_cast<double2*>(reinterpret_cast<const double2*>(src)) + (size_t)i * d * d, d, d};
        o.D = MatRef{reinterpret_cast<double2*>(dst) + (size_t)i * d * d, d, d};
        o.tag = i;
        ops.push_back(o);
    }
    int nl = levelize(ops);
    Program dry = compile(ops, nl, reinterpret_cast<char*>((uintptr_t)1 << 40));
    char* pool = nullptr;
    char* dev = nullptr;
    DevStatus* st = nullptr;
    hipError_t e = hipMalloc(&pool, dry.inv_scratch_bytes);
    if (e != hipSuccess) return set_err(nullptr, BT_ERR_OOM, "diag_inverse: scratch");
    Program pg = compile(ops, nl, pool);
    const size_t bg = pg.gemm.size() * sizeof(GemmOp), bi = pg.inv.size() * sizeof(InvJob);
    const size_t off_inv = (bg + 255) & ~(size_t)255;
    e = hipMalloc(&dev, off_inv + bi + 256);
    if (e == hipSuccess) e = hipMalloc(&st, sizeof(DevStatus));
    if (e != hipSuccess) { hipFree(pool); hipFree(dev); return set_err(nullptr, BT_ERR_OOM, "diag_inverse: op list"); }
    std::vector<char> host(off_inv + bi + 256);
    memcpy(host.data(), pg.gemm.data(), bg);
    memcpy(host.data() + off_inv, pg.inv.data(), bi);
    DevStatus z{0, 0};
    e = hipMemcpy(dev, host.data(), host.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(st, &z, sizeof z, hipMemcpyHostToDevice);
    GemmOp* dg = reinterpret_cast<GemmOp*>(dev);
    InvJob* dj = reinterpret_cast<InvJob*>(dev + off_inv);
    for (const Launch& L : pg.launches) {
        if (e != hipSuccess) break;
        switch (L.type) {
            case 0: e = launch_gemm_shape(dg + L.off, L.count, L.tiles, L.mixed != 0, L.shape, s); break;
            case 6: e = launch_inv_step(dj + L.off, L.count, L.maxd, L.panel, L.tiles, st, s); break;
            default: break;
        }
    }
    hipError_t e2 = hipStreamSynchronize(s);
    DevStatus out{0, 0};
    if (e2 == hipSuccess) e2 = hipMemcpy(&out, st, sizeof out, hipMemcpyDeviceToHost);
    hipFree(pool);
    hipFree(dev);
    hipFree(st);
    if (e != hipSuccess) return hip_err(nullptr, e, "diag_inverse launch");
    if (e2 != hipSuccess) return hip_err(nullptr, e2, "diag_inverse sync");
    if (out.code != 0) {
        if (bad_index) *bad_index = out.tag;
        return set_err(nullptr, BT_ERR_SINGULAR, "diag_inverse: singular or non-finite pivot");
    }
    return BT_OK;
}

}  // extern "C"

extern "C" size_t bt_si_sq_diag_schedule(const bt_desc* desc, char* out, size_t cap) {
    std::vector<int> bounds;
    std::string msg;
    if (!desc_bounds(desc, bounds, msg)) { g_last_error = msg; return 0; }
    Builder bd;
    bd.D = Dims(desc->n, desc->b, desc->a, desc->block_sizes);
    bd.bounds = bounds;
    bd.mode = MODE_BOTH;
    bd.mixed_bulk = desc->precision == BT_MIXED;
    bd.antiH = (desc->flags & BT_SIGMA_ANTIHERMITIAN) != 0;
    bd.diag_only = (desc->flags & BT_DIAG_ONLY) != 0;
    bd.ws = reinterpret_cast<char*>((uintptr_t)1 << 40);
    bd.build();
    const int nl = levelize(bd.ops);
    std::vector<int> ng(nl), nt(nl), ni(nl), na(nl), nc1(nl);
    for (auto& o : bd.ops) {
        if (o.kind == K_GEMM) { ng[o.level]++; nt[o.level] += gemm_tiles_shape(o.D.r, o.D.c, 1); }
        else if (o.kind == K_INV) ni[o.level]++;
        else na[o.level]++;
        if (o.cls == 1) nc1[o.level]++;
    }
    std::string txt;
    char line[128];
    for (int L = 0; L < nl; ++L) {
        snprintf(line, sizeof line, "%d %d %d %d %d %d\n", L, ng[L], nt[L], ni[L], na[L], nc1[L]);
        txt += line;
    }
    if (out && cap > 0) {
        size_t c = std::min(cap - 1, txt.size());
        memcpy(out, txt.data(), c);
        out[c] = 0;
    }
    return txt.size() + 1;
}
