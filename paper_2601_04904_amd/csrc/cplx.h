// Complex arithmetic, the pivot key and the wave maximum shared by the
// inverse kernels (the panel-per-launch blocked inverse and the inverse
// inside the fused small-instance kernel).
#pragma once
#include <hip/hip_runtime.h>
#include <cfloat>

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

// 1 / v = conj(v) / |v|^2.  v is first scaled by a power of two so that its
// larger component lies in [0.5, 1), which puts |v|^2 in [0.25, 2); the
// reciprocal of |v|^2 is the hardware estimate refined by two Newton steps
// r <- r (2 - s r) (each at least doubles the number of correct bits).  A
// zero, infinite or NaN v gives a NaN result, which the caller flags.
__device__ inline double2 crecip(double2 v) {
    int e;
    (void)frexp(fmax(fabs(v.x), fabs(v.y)), &e);
    const double a = ldexp(v.x, -e), b = ldexp(v.y, -e);
    const double s = fma(a, a, b * b);
    double r = __builtin_amdgcn_rcp(s);
    r = fma(r, fma(-s, r, 1.0), r);
    r = fma(r, fma(-s, r, 1.0), r);
    return make_double2(ldexp(a * r, -e), ldexp(-b * r, -e));
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

// Pivot key (32 bits): bits 62..41 of the double |re| + |im| (its exponent
// and the top 11 bits of its mantissa; non-finite values clamped to the
// largest finite double) above 1023 - row in the low 10 bits.  Non-negative
// doubles order like their bit patterns, so the largest key is the largest
// magnitude to 11 mantissa bits (any candidate within a relative 2^-11 of the
// largest is as good a pivot) and, among those, the lowest row.  Rows are
// below 1024.  0 means "no candidate" (it is also the key of a zero entry in
// row 1023; either way the column has no usable pivot).
__device__ inline unsigned pivot_key(double2 v, int row) {
    double m = fabs(v.x) + fabs(v.y);
    if (!(m <= DBL_MAX)) m = DBL_MAX;
    const unsigned long long bits = (unsigned long long)__double_as_longlong(m);
    return ((unsigned)(bits >> 41) << 10) | (unsigned)(1023 - row);
}

__device__ inline int key_row(unsigned key) { return 1023 - (int)(key & 1023u); }

}  // namespace btsq
