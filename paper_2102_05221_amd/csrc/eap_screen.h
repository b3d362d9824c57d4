// Certified error bound of the FP32 screening sweep (host and device).
//
// For a warping path of exact cost B (real arithmetic on the float64 inputs)
// with at most N steps over values of magnitude <= A (ERP: A also bounds
// |gap|), eps(B) bounds |V32 - B|, where V32 is the path's cost evaluated in
// FP32 the way the recurrence adds it (u = 2^-24 the unit roundoff).  The
// FP32 sweeps of the squared costs fuse the (weighted) square with the add:
// that removes roundings from the accounting below and keeps the bound.  The FP32 dynamic programme returns the least V32 over all
// paths (min is exact and rounded addition is monotone), so its result D32
// satisfies D32 <= D + eps(D) and D <= screen_bound(D32).
//
// Squared costs (DTW, CDTW, WDTW).  Rounding the inputs moves a difference d
// by e, |e| <= u(|s| + |t|) <= 2uA; the subtraction, the square and (WDTW)
// the rounded weight and its product add at most five relative roundings:
// term32 = W (d+e)^2 (1 + th), |th| <= 5.001u.  With |(d+e)^2 - d^2| <=
// 4uA|d| + 4u^2 A^2, sum W|d| <= sqrt(sum W) sqrt(B) <= sqrt(N B) (weights <= 1,
// Cauchy-Schwarz) and sum W <= N, the terms differ from theirs by at most
// (1 + 5.001u)(4uA sqrt(N B) + 4u^2 A^2 N) + 5.001u B, and the running sum of
// N terms adds gamma_{N-1} = (N-1)u / (1 - (N-1)u) of their total.  For N <=
// 2^13 all of it is below
//     1.01 u ((N + 5) B + 4 A sqrt(N B) + 4 u A^2 N).
// Exact differences (the FP32 sweep reads float64 values and rounds each
// difference once): e = 0 and the difference carries one float64 and one
// FP32 rounding, so the A terms vanish: 1.01 u (N + 5) B.
//
// L1 costs (ERP, MSM, TWE).  A step's term is a sum of at most two absolute
// differences of inputs and non-negative constants (gap distance, c, nu,
// lambda, nu * 2|i-j|), added with at most three roundings: each difference
// is off by at most 2uA (input rounding) plus its own relative rounding, so a
// term is off by 4uA + 4.001u |term| at most, and over N steps with the
// running sum: 1.01 u ((N + 4) B + 4 A N).
//
// Every bound adds N * 4e-38 for FP32 underflow (at most three flushed
// operations per step).  The float64 reference's own rounding (2^-53 per
// operation) sits within the factor 1.01.
#pragma once
#include <math.h>

namespace eap {

// Screen modes: the distance kind, plus kScreenExactDiff when the FP32 sweep
// forms each difference in float64 (no input rounding).
constexpr int kScreenExactDiff = 8;

__host__ __device__ inline bool screen_squared(int kind) {
    const int k = kind & 7;
    return k == 0 || k == 1 || k == 2;   // DTW, CDTW, WDTW
}

__host__ __device__ inline double screen_eps(int kind, double B, double N, double A) {
    const double u = 0x1p-24;
    double e;
    if (kind & kScreenExactDiff) e = u * (N + 5.0) * B;
    else if (screen_squared(kind)) e = u * ((N + 5.0) * B + 4.0 * A * sqrt(N * B) + 4.0 * u * A * A * N);
    else e = u * ((N + 4.0) * B + 4.0 * N * A);
    return 1.01 * e + N * 4e-38;
}

// Largest exact cost C with C <= b + eps(C): a bound on the exact cost of any
// path whose FP32 evaluation is <= b.  For the squared costs eps grows like
// sqrt(C), a quadratic in sqrt(C); at b = 0 the bound is about (4uA)^2 N.
__host__ __device__ inline double screen_bound(int kind, double b, double N, double A) {
    const double u = 1.01 * 0x1p-24;
    double B;
    if (kind & kScreenExactDiff) {
        B = (b + N * 4e-38) / (1.0 - u * (N + 5.0));
    } else if (screen_squared(kind)) {
        const double e0 = b + N * 4e-38 + u * 4.0 * 0x1p-24 * A * A * N;
        const double a = u * (N + 5.0), c = u * 4.0 * A * sqrt(N);
        const double r = (c + sqrt(c * c + 4.0 * (1.0 - a) * e0)) / (2.0 * (1.0 - a));
        B = r * r;
    } else {
        B = (b + N * 4e-38 + u * 4.0 * N * A) / (1.0 - u * (N + 4.0));
    }
    return B * (1.0 + 1e-9);
}

}  // namespace eap
