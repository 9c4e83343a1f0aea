// The radius ladder of Sec. 2.1 (power law R_m = R_0 b^-m, b = (R_0/R_M)^(1/M),
// or linear R_m = R_0 - m (R_0 - R_M)/M) evaluated on the device, so that the
// statistic's bins can follow its range without a host round trip.  The host
// forms the same ladder with the C library's pow; the device's powers are
// taken in double-double arithmetic (about 100 bits) and rounded once, which
// gives the correctly rounded power.  The two agree whenever the library's
// pow is correctly rounded for the argument; the caller compares them and
// redoes the bins with the host's ladder where they do not.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>

namespace cil {

// hi + lo, |lo| <= ulp(hi) / 2 (Dekker, Knuth; the error-free sum and the
// fused-multiply-add product).  No function here lets the compiler contract
// a product into a later sum: that would break the error-free steps.
struct DD {
    double hi, lo;
};

__host__ __device__ inline DD dd_two_sum(double a, double b)
{
#pragma clang fp contract(off)
    const double s = a + b, bb = s - a;
    return {s, (a - (s - bb)) + (b - bb)};
}

__host__ __device__ inline DD dd_quick(double a, double b)      // |a| >= |b| or a = 0
{
#pragma clang fp contract(off)
    const double s = a + b;
    return {s, b - (s - a)};
}

__host__ __device__ inline DD dd_add(DD a, DD b)
{
#pragma clang fp contract(off)
    DD s = dd_two_sum(a.hi, b.hi);
    const DD t = dd_two_sum(a.lo, b.lo);
    s.lo += t.hi;
    s = dd_quick(s.hi, s.lo);
    s.lo += t.lo;
    return dd_quick(s.hi, s.lo);
}

__host__ __device__ inline DD dd_mul(DD a, DD b)
{
#pragma clang fp contract(off)
    const double p = a.hi * b.hi;
    double e = fma(a.hi, b.hi, -p);
    e += a.hi * b.lo + a.lo * b.hi;
    return dd_quick(p, e);
}

__host__ __device__ inline DD dd_mul_d(DD a, double b)
{
#pragma clang fp contract(off)
    const double p = a.hi * b;
    double e = fma(a.hi, b, -p);
    e += a.lo * b;
    return dd_quick(p, e);
}

__host__ __device__ inline DD dd_div(DD a, DD b)
{
#pragma clang fp contract(off)
    const double q1 = a.hi / b.hi;
    DD r = dd_add(a, dd_mul_d(b, -q1));
    const double q2 = r.hi / b.hi;
    r = dd_add(r, dd_mul_d(b, -q2));
    const double q3 = r.hi / b.hi;
    return dd_add(dd_quick(q1, q2), DD{q3, 0.0});
}

// ln 2 to double-double precision
constexpr double kLn2Hi = 0x1.62e42fefa39efp-1, kLn2Lo = 0x1.abc9e3b39803fp-56;

// The series' coefficients: 1 / (2k + 1) for the logarithm (k = 0..22) and
// 1 / n for the exponential (n = 1..9), each in double-double.
constexpr int kLogTerms = 23, kExpTerms = 9;
struct DDTables {
    DD inv_odd[kLogTerms];
    DD inv_n[kExpTerms + 1];
};

__host__ __device__ inline DD dd_inv(int n)
{
#pragma clang fp contract(off)
    return dd_div(DD{1.0, 0.0}, DD{(double)n, 0.0});
}

__host__ inline void dd_tables(DDTables &t)
{
    for (int k = 0; k < kLogTerms; ++k) t.inv_odd[k] = dd_inv(2 * k + 1);
    for (int n = 1; n <= kExpTerms; ++n) t.inv_n[n] = dd_inv(n);
}

// log x for finite x > 0: x = m 2^e, m in [1/sqrt 2, sqrt 2), log m = 2 atanh(s)
// with s = (m - 1)/(m + 1), |s| < 0.172, atanh(s)/s = sum_k s^2k / (2k + 1),
// truncated where s^2k < 2^-110.
__host__ __device__ inline DD dd_log(double x, const DDTables &t)
{
#pragma clang fp contract(off)
    int e;
    double m = frexp(x, &e);
    if (m < 0.70710678118654752440) {
        m *= 2.0;
        --e;
    }
    const DD s = dd_div(DD{m - 1.0, 0.0}, dd_two_sum(m, 1.0));   // m - 1 is exact on [1/2, 2]
    const DD s2 = dd_mul(s, s);
    DD sum = t.inv_odd[kLogTerms - 1];
    for (int k = kLogTerms - 2; k >= 0; --k) sum = dd_add(dd_mul(sum, s2), t.inv_odd[k]);
    const DD r = dd_mul_d(dd_mul(sum, s), 2.0);
    return dd_add(r, dd_mul_d(DD{kLn2Hi, kLn2Lo}, (double)e));
}

// exp a for |a| < 700: a = k ln 2 + r, |r| <= ln2 / 2; e^r - 1 of r / 2^10 by
// its series (terms below 2^-107 dropped), then ten doublings of e^t - 1
// (u -> u (2 + u)), which keep its relative precision.
__host__ __device__ inline DD dd_exp(DD a, const DDTables &t)
{
#pragma clang fp contract(off)
    const double k = rint(a.hi / kLn2Hi);
    DD r = dd_add(a, dd_mul_d(DD{kLn2Hi, kLn2Lo}, -k));
    r.hi = ldexp(r.hi, -10);
    r.lo = ldexp(r.lo, -10);
    DD u = dd_mul(r, t.inv_n[kExpTerms]);                      // Horner: r (1 + r/2 (1 + r/3 (...)))
    for (int n = kExpTerms - 1; n >= 1; --n) u = dd_mul(dd_mul(r, dd_add(DD{1.0, 0.0}, u)), t.inv_n[n]);
    for (int i = 0; i < 10; ++i) u = dd_mul(u, dd_add(DD{2.0, 0.0}, u));
    DD v = dd_add(DD{1.0, 0.0}, u);
    const int ki = (int)k;
    return {ldexp(v.hi, ki), ldexp(v.lo, ki)};
}

// sqrt x for finite x >= 0, correctly rounded but for arguments within about
// 2^-100 relative of a rounding boundary: one Newton correction of the
// hardware root, s + (x - s^2) / (2 s) with the residual exact by fma.
__host__ __device__ inline double sqrt_dd(double x)
{
#pragma clang fp contract(off)
    const double s = sqrt(x);
    if (!(s > 0.0) || !isfinite(s)) return s;
    const double r = fma(-s, s, x);
    const DD t = dd_quick(s, r / (2.0 * s));
    return t.hi + t.lo;
}

// The power-law ladder's base b = x^(1/M) (the exponent 1/M as rounded), and
// log b in double-double for the powers b^-m = exp(-m log b):
// log b = (1/M) log x + log(b / x^(1/M)), the last term (b - p)/p from the
// double-double value p of x^(1/M), whose rounding b is (|b - p|/p < 2^-53,
// so the next term of the series is below 2^-107).
__host__ __device__ inline double root_dd(double x, int M, const DDTables &t, DD *logb)
{
#pragma clang fp contract(off)
    if (x == 1.0) {
        *logb = DD{0.0, 0.0};
        return 1.0;
    }
    const DD lx = dd_mul_d(dd_log(x, t), 1.0 / M);
    const DD p = dd_exp(lx, t);
    const double b = p.hi + p.lo;
    *logb = dd_add(lx, dd_div(dd_add(DD{b, 0.0}, DD{-p.hi, -p.lo}), p));
    return b;
}

__host__ __device__ inline double pow_dd_from_log(DD logx, double y, const DDTables &t)
{
#pragma clang fp contract(off)
    const DD p = dd_exp(dd_mul_d(logx, y), t);
    return p.hi + p.lo;
}

// x^y for finite x > 0 and |y log x| < 700, correctly rounded but for
// arguments within about 2^-95 relative of a rounding boundary.
__host__ __device__ inline double pow_dd(double x, double y, const DDTables &t)
{
#pragma clang fp contract(off)
    if (x == 1.0) return 1.0;
    return pow_dd_from_log(dd_log(x, t), y, t);
}

}  // namespace cil
