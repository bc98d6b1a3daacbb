// Double-double arithmetic and E = e^{i zeta} to about 1e-30 relative.
//
// A value is the unevaluated sum hi + lo of two doubles with |lo| <= ulp(hi)/2.
// The error-free transformations are Knuth's two-sum and Dekker's product
// (here with a fused multiply-add); additions and products follow the usual
// double-double formulas.  The elementary functions reduce their argument by
// Cody and Waite's method with the constant split into pieces of 33
// significant bits (so that k times a piece is exact for |k| < 2^20) and
// then sum the Taylor series in nested form, dividing by the integers
// 2, 3, ... instead of storing inverse factorials.
//
// Used once per node and call (k_prep_nodes): with E stored as hi + lo, the
// difference E_q - E_p of two nodes is formed with a relative error of a few
// units of rounding however close the nodes are, which keeps the E quotient
// of the kernel entries as accurate as a cotangent of the exact difference.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>

namespace wwbi {

struct DD {
    double hi, lo;
};

__host__ __device__ inline DD dd_two_sum(double a, double b) {
    const double s = a + b;
    const double bb = s - a;
    const double e = (a - (s - bb)) + (b - bb);
    return {s, e};
}

__host__ __device__ inline DD dd_fast_two_sum(double a, double b) {   // |a| >= |b|
    const double s = a + b;
    return {s, b - (s - a)};
}

__host__ __device__ inline DD dd_two_prod(double a, double b) {
    const double p = a * b;
    return {p, fma(a, b, -p)};
}

__host__ __device__ inline DD dd_add(DD a, DD b) {
    DD s = dd_two_sum(a.hi, b.hi);
    const DD t = dd_two_sum(a.lo, b.lo);
    s.lo += t.hi;
    s = dd_fast_two_sum(s.hi, s.lo);
    s.lo += t.lo;
    return dd_fast_two_sum(s.hi, s.lo);
}

__host__ __device__ inline DD dd_add_d(DD a, double b) {
    DD s = dd_two_sum(a.hi, b);
    s.lo += a.lo;
    return dd_fast_two_sum(s.hi, s.lo);
}

__host__ __device__ inline DD dd_mul(DD a, DD b) {
    DD p = dd_two_prod(a.hi, b.hi);
    p.lo += a.hi * b.lo + a.lo * b.hi;
    return dd_fast_two_sum(p.hi, p.lo);
}

__host__ __device__ inline DD dd_mul_d(DD a, double b) {
    DD p = dd_two_prod(a.hi, b);
    p.lo += a.lo * b;
    return dd_fast_two_sum(p.hi, p.lo);
}

// a / b for a double b (one correction step of the quotient).
__host__ __device__ inline DD dd_div_d(DD a, double b) {
    const double q1 = a.hi / b;
    const DD p = dd_two_prod(q1, b);
    const double r = ((a.hi - p.hi) - p.lo) + a.lo;
    const double q2 = r / b;
    return dd_fast_two_sum(q1, q2);
}

// 1 - a
__host__ __device__ inline DD dd_one_minus(DD a) {
    DD s = dd_two_sum(1.0, -a.hi);
    s.lo -= a.lo;
    return dd_fast_two_sum(s.hi, s.lo);
}

// pi/2 = kPio2[0] + ... + kPio2[3] to about 1e-48: the leading 33 significant
// bits of pi/2, then of each remainder, the last piece a full double.
constexpr double kPio2[4] = {1.5707963267341256, 6.077100506303966e-11, 2.0222662487111665e-21,
                             8.4784276603689e-32};
// ln 2 in the same form.
constexpr double kLn2[4] = {0.6931471806019545, -4.200915072890502e-11, 2.094174429075368e-21,
                            1.94704509238075e-31};

// x - k (c0 + c1 + c2 + c3) as a double-double; each k c_i with |k| < 2^20 is
// exact for the 33-bit pieces.
__host__ __device__ inline DD dd_reduce(double x, double k, const double *c) {
    DD r = dd_two_sum(x, -k * c[0]);
    r = dd_add_d(r, -k * c[1]);
    r = dd_add_d(r, -k * c[2]);
    r = dd_add(r, dd_two_prod(-k, c[3]));
    return r;
}

// sin r and cos r for |r| <= pi/4 + tiny, nested Taylor sums through r^29 and
// r^28 (the next terms are below 1e-33).
__host__ __device__ inline void dd_sincos_reduced(DD r, DD &s, DD &c) {
    const DD r2 = dd_mul(r, r);
    DD ts = {1.0, 0.0}, tc = {1.0, 0.0};
    for (int n = 28; n >= 2; n -= 2) {
        // sin: 1 - r^2 / ((n)(n+1)) (...); cos: 1 - r^2 / ((n-1) n) (...)
        ts = dd_one_minus(dd_div_d(dd_mul(r2, ts), (double)(n * (n + 1))));
        tc = dd_one_minus(dd_div_d(dd_mul(r2, tc), (double)((n - 1) * n)));
    }
    s = dd_mul(r, ts);
    c = tc;
}

// e^r for |r| <= ln(2)/2 + tiny, nested Taylor sum through r^27.
__host__ __device__ inline DD dd_exp_reduced(DD r) {
    DD t = {1.0, 0.0};
    for (int n = 27; n >= 1; --n) t = dd_add_d(dd_div_d(dd_mul(r, t), (double)n), 1.0);
    return t;
}

// E = e^{i (x + i y)} = e^{-y} (cos x + i sin x) as double-doubles, for
// |x| < 1.6e6 and |y| <= 700 (the library limits nodes to |y| <= 30).
__host__ __device__ inline void dd_expi(double x, double y, DD &er, DD &ei) {
    const double kq = rint(x * 0.63661977236758134);    // x / (pi/2)
    const DD r = dd_reduce(x, kq, kPio2);
    DD s, c;
    dd_sincos_reduced(r, s, c);
    const int q = ((int)kq) & 3;
    DD cx, sx;
    if (q == 0) { cx = c; sx = s; }
    else if (q == 1) { cx = {-s.hi, -s.lo}; sx = c; }
    else if (q == 2) { cx = {-c.hi, -c.lo}; sx = {-s.hi, -s.lo}; }
    else { cx = s; sx = {-c.hi, -c.lo}; }
    const double a = -y;
    const double kl = rint(a * 1.4426950408889634);     // a / ln 2
    DD m = dd_exp_reduced(dd_reduce(a, kl, kLn2));
    m.hi = ldexp(m.hi, (int)kl);
    m.lo = ldexp(m.lo, (int)kl);
    er = dd_mul(m, cx);
    ei = dd_mul(m, sx);
}

}  // namespace wwbi
