// x^y rounded to the nearest double, for x > 0 (normal or subnormal) and
// |y log x| < 2^20, on the device.
//
// Evaluated as exp(y log x) in double-double arithmetic (pairs hi + lo of
// doubles, |lo| <= ulp(hi) / 2, each product and sum built from exact
// two-sum / two-product steps):
//   * log: x = 2^e f with f in [1/sqrt 2, sqrt 2); with s = (f - 1)/(f + 1),
//     log f = 2 s sum_j s^(2j) / (2j + 1) (the atanh series; |s| <= 0.1716,
//     so 19 terms leave a truncation below 2^-100); log x = e ln 2 + log f;
//   * exp: E = y log x = n ln 2 + r with n = rint(E / ln 2), |r| <= ln2 / 2;
//     q = expm1(r / 2^8) by its Taylor series to degree 9, then eight
//     squarings (1 + q)^2 = 1 + (2q + q^2); x^y = 2^n (1 + q).
// The double-double value is within about 2^-95 of x^y (relative), so the
// final rounding of hi + lo is the correctly rounded result unless x^y lies
// within that distance of a midpoint between two doubles.  Every operation
// is rounded on its own: no contraction.
#pragma once

#include <hip/hip_runtime.h>

#pragma clang fp contract(off)

namespace rsc {
namespace crp {

struct dd {
    double h, l;
};

__device__ __forceinline__ dd two_sum(double a, double b) {
    const double s = a + b;
    const double bb = s - a;
    return {s, (a - (s - bb)) + (b - bb)};
}

// |a| >= |b| (or a == 0)
__device__ __forceinline__ dd fast_two_sum(double a, double b) {
    const double s = a + b;
    return {s, b - (s - a)};
}

__device__ __forceinline__ dd two_prod(double a, double b) {
    const double p = a * b;
    return {p, __builtin_fma(a, b, -p)};
}

// Sum of two double-doubles, accurate to about 2^-105 (|a| + |b|): every sum
// below either has terms of one sign or one term well below the other, so
// this bound is relative to the result within a small factor.
__device__ __forceinline__ dd add(dd a, dd b) {
    dd s = two_sum(a.h, b.h);
    s.l = s.l + (a.l + b.l);
    return fast_two_sum(s.h, s.l);
}

__device__ __forceinline__ dd add_d(dd a, double b) {
    dd s = two_sum(a.h, b);
    s.l = s.l + a.l;
    return fast_two_sum(s.h, s.l);
}

__device__ __forceinline__ dd mul(dd a, dd b) {
    dd p = two_prod(a.h, b.h);
    p.l = __builtin_fma(a.h, b.l, p.l);
    p.l = __builtin_fma(a.l, b.h, p.l);
    return fast_two_sum(p.h, p.l);
}

__device__ __forceinline__ dd mul_d(dd a, double b) {
    dd p = two_prod(a.h, b);
    p.l = __builtin_fma(a.l, b, p.l);
    return fast_two_sum(p.h, p.l);
}

// 1 / m as a double-double (m a small odd or factorial integer)
__device__ __forceinline__ dd recip(double m) {
    const double h = 1.0 / m;
    return {h, __builtin_fma(-h, m, 1.0) / m};
}

// ln 2 = kLn2Hi + kLn2Lo to about 2^-110
constexpr double kLn2Hi = 0x1.62e42fefa39efp-1;
constexpr double kLn2Lo = 0x1.abc9e3b39803fp-56;

// log x for finite x > 0
__device__ __forceinline__ dd log_dd(double x) {
    int e;
    double f = __builtin_frexp(x, &e);  // x = f 2^e, f in [0.5, 1)
    if (f < 0x1.6a09e667f3bcdp-1) {     // 1/sqrt 2
        f = f * 2.0;
        e = e - 1;
    }
    const double num = f - 1.0;  // exact (f within a factor 2 of 1)
    const dd den = two_sum(f, 1.0);
    const double sh = num / den.h;
    const double rem = __builtin_fma(-sh, den.h, num) - sh * den.l;
    const dd s = fast_two_sum(sh, rem / den.h);
    const dd z = mul(s, s);
    // terms j = 9 .. 18 of sum z^j / (2j + 1), below 2^-45 of the sum: double
    double t = 1.0 / 37.0;
#pragma unroll
    for (int j = 17; j >= 9; --j) t = t * z.h + 1.0 / (double)(2 * j + 1);
    dd p = {t, 0.0};
#pragma unroll
    for (int j = 8; j >= 1; --j) p = add(mul(p, z), recip((double)(2 * j + 1)));
    p = add_d(mul(p, z), 1.0);
    dd lf = mul(s, p);
    lf.h = lf.h * 2.0;
    lf.l = lf.l * 2.0;
    const double ed = (double)e;
    dd el = two_prod(ed, kLn2Hi);
    el = add_d(el, ed * kLn2Lo);
    return add(el, lf);
}

// exp E (E a double-double), result hi + lo before the final rounding,
// scaled by 2^-n (n returned)
__device__ __forceinline__ dd exp_dd(dd E, int *n_out) {
    const double nf = __builtin_rint(E.h * 0x1.71547652b82fep0);  // E / ln 2
    const dd t = two_prod(nf, kLn2Hi);
    const double rh = E.h - t.h;  // exact: E.h within a factor 2 of t.h, or nf = 0
    dd r = two_sum(rh, E.l);
    r = add_d(r, -t.l);
    const dd u = two_prod(nf, kLn2Lo);
    r = add(r, dd{-u.h, -u.l});
    r.h = r.h * 0x1p-8;
    r.l = r.l * 0x1p-8;
    // expm1(r) = r (1 + r (1/2 + r (1/6 + r (1/24 + r w)))), w = 1/120 + ... + r^4/9!
    double w = 1.0 / 362880.0;
    w = w * r.h + 1.0 / 40320.0;
    w = w * r.h + 1.0 / 5040.0;
    w = w * r.h + 1.0 / 720.0;
    w = w * r.h + 1.0 / 120.0;
    dd a = add(mul_d(r, w), recip(24.0));
    a = add(mul(a, r), recip(6.0));
    a = add_d(mul(a, r), 0.5);
    a = add_d(mul(a, r), 1.0);
    dd q = mul(a, r);
#pragma unroll
    for (int k = 0; k < 8; ++k) q = add(dd{2.0 * q.h, 2.0 * q.l}, mul(q, q));
    *n_out = (int)nf;
    return add_d(q, 1.0);
}

// (v.h + v.l) 2^n rounded once to the nearest double (ties to even), for
// v.h in [0.7, 2.1] with |v.l| <= ulp(v.h) / 2.  For n >= -1021 the value is
// normal or overflows, and rounding v.h + v.l then scaling is exact.  Below,
// the result lies on the subnormal grid of 2^-1074 (which also spaces the
// binade [2^-1022, 2^-1021)): z = v 2^(n + 1074) is rounded to an integer,
// with the tail deciding the halfway cases of the head.
__device__ __forceinline__ double scale_round(dd v, int n) {
    if (n >= -1021) return __builtin_ldexp(v.h + v.l, n);
    const int s = n + 1074;
    if (s < -2) return 0.0;  // below 2^-1076: less than half a grid step
    const double zh = __builtin_ldexp(v.h, s), zl = __builtin_ldexp(v.l, s);  // exact scalings
    double r = __builtin_rint(zh);
    const double f = zh - r;  // exact: |f| <= 1/2 on zh's own grid
    if (f == 0.5 && zl > 0.0) r = r + 1.0;
    if (f == -0.5 && zl < 0.0) r = r - 1.0;
    return __builtin_ldexp(r, -1074);  // r < 2^53: exact
}

// x^y rounded to nearest (x > 0 finite, |y log x| < 2^20), by the series
// above alone (no tables).
__device__ __forceinline__ double pow_rn(double x, double y) {
    const dd L = log_dd(x);
    const dd E = mul_d(L, y);
    int n;
    const dd v = exp_dd(E, &n);
    return scale_round(v, n);
}

// ---- table-driven form ------------------------------------------------------
//
// log: x = 2^e f with f in [1, 2) and the cell c = 1 + (2j + 1)/128 of
// f (j = floor(64 (f - 1))); with s = (f - c)/(f + c), |s| <= 2^-8,
// log f = log c + 2 s sum_{i<7} s^(2i) / (2i + 1) (truncation below 2^-110).
// exp: E = (m / 64) ln 2 + r with m = rint(64 E / ln 2), |r| <= ln2 / 128;
// exp E = 2^(m div 64) 2^((m mod 64) / 64) (1 + expm1 r), expm1 by its
// Taylor series to degree 10 (truncation below 2^-107).
// The 64 values log c_j and the 64 values 2^(k/64) (double-doubles) are made
// by the series above (make_pow_tables), accurate to about 2^-97.

constexpr int kPowCells = 64;

struct PowTables {
    dd logc[kPowCells];  // log(1 + (2j + 1)/128)
    dd exp2[kPowCells];  // 2^(k/64)
};

// Entry t of the tables (t < 64: log c_t; else 2^((t - 64)/64)).
__device__ __forceinline__ dd pow_table_entry(int t) {
    if (t < kPowCells) return log_dd(1.0 + (double)(2 * t + 1) * 0x1p-7);
    const double kf = (double)(t - kPowCells) * 0x1p-6;  // exact
    const dd E = mul_d(dd{kLn2Hi, kLn2Lo}, kf);
    int n;
    const dd v = exp_dd(E, &n);
    return {__builtin_ldexp(v.h, n), __builtin_ldexp(v.l, n)};
}

__device__ __forceinline__ dd log_dd_t(double x, const dd *__restrict__ logc) {
    int e;
    double f = __builtin_frexp(x, &e);  // [0.5, 1)
    f = f * 2.0;                        // [1, 2), exact
    e = e - 1;
    const int j = (int)((f - 1.0) * 64.0);  // exact product, 0 .. 63
    const double c = 1.0 + (double)(2 * j + 1) * 0x1p-7;
    const double num = f - c;  // exact (f and c within a factor 2)
    const dd den = two_sum(f, c);
    const double sh = num / den.h;
    const double rem = __builtin_fma(-sh, den.h, num) - sh * den.l;
    const dd s = fast_two_sum(sh, rem / den.h);
    const dd z = mul(s, s);
    double t = 1.0 / 13.0;  // terms 4 .. 6, below 2^-60 of the sum: double
    t = t * z.h + 1.0 / 11.0;
    t = t * z.h + 1.0 / 9.0;
    dd p = {t, 0.0};
#pragma unroll
    for (int i = 3; i >= 1; --i) p = add(mul(p, z), recip((double)(2 * i + 1)));
    p = add_d(mul(p, z), 1.0);
    dd lf = mul(s, p);
    lf.h = lf.h * 2.0;
    lf.l = lf.l * 2.0;
    lf = add(lf, logc[j]);
    const double ed = (double)e;
    dd el = two_prod(ed, kLn2Hi);
    el = add_d(el, ed * kLn2Lo);
    return add(el, lf);
}

// exp E = (hi + lo) 2^n
__device__ __forceinline__ dd exp_dd_t(dd E, const dd *__restrict__ exp2t, int *n_out) {
    const double mf = __builtin_rint(E.h * 0x1.71547652b82fep6);  // 64 E / ln 2
    const dd t = two_prod(mf, kLn2Hi * 0x1p-6);
    const double rh = E.h - t.h;  // exact: E.h within a factor 2 of t.h, or mf = 0
    dd r = two_sum(rh, E.l);
    r = add_d(r, -t.l);
    const dd u = two_prod(mf, kLn2Lo * 0x1p-6);
    r = add(r, dd{-u.h, -u.l});
    double w = 1.0 / 3628800.0;  // degrees 6 .. 10: double
    w = w * r.h + 1.0 / 362880.0;
    w = w * r.h + 1.0 / 40320.0;
    w = w * r.h + 1.0 / 5040.0;
    w = w * r.h + 1.0 / 720.0;
    dd a = add(mul_d(r, w), recip(120.0));
    a = add(mul(a, r), recip(24.0));
    a = add(mul(a, r), recip(6.0));
    a = add_d(mul(a, r), 0.5);
    a = add_d(mul(a, r), 1.0);
    const dd q = mul(a, r);
    const int m = (int)mf;
    const int k = m & (kPowCells - 1);
    *n_out = (m - k) / kPowCells;  // exact division
    const dd T = exp2t[k];
    return add(T, mul(q, T));
}

// x^y rounded to nearest (x > 0 finite, |y log x| < 2^20); results beyond
// the largest double give +inf, results in the subnormal range are rounded
// on its grid
__device__ __forceinline__ double pow_rn_t(double x, double y, const PowTables &tb) {
    const dd L = log_dd_t(x, tb.logc);
    const dd E = mul_d(L, y);
    int n;
    const dd v = exp_dd_t(E, tb.exp2, &n);
    return scale_round(v, n);
}

// x^y1 and x^y2, each rounded to nearest as pow_rn_t, sharing one logarithm
__device__ __forceinline__ void pow2_rn_t(double x, double y1, double y2, const PowTables &tb, double *r1,
                                          double *r2) {
    const dd L = log_dd_t(x, tb.logc);
    int n1, n2;
    const dd v1 = exp_dd_t(mul_d(L, y1), tb.exp2, &n1);
    const dd v2 = exp_dd_t(mul_d(L, y2), tb.exp2, &n2);
    *r1 = scale_round(v1, n1);
    *r2 = scale_round(v2, n2);
}

}  // namespace crp
}  // namespace rsc
