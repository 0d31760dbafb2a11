// Device-side arithmetic for batched 2x2 / 3x3 symmetric eigendecomposition on
// gfx950.  One lane owns one matrix; nothing here touches memory except through
// the arguments.  Method: Kronenburg, arXiv:1306.6291 (§3 for 2x2, §4-§5 for
// 3x3, §6 for the meaning of the angles).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ksym_poly.hpp"

namespace ksym {

constexpr int FLAG_GENERAL = 0, FLAG_DOUBLE = 1, FLAG_TRIPLE = 2, FLAG_FIXUP = 4,
              FLAG_NONFINITE = 8;

constexpr double kPi = 3.14159265358979323846;
constexpr double kSqrt3 = 1.73205080756887729353;
constexpr double kInvSqrt3 = 0.57735026918962576451;

__device__ __forceinline__ float atan2_fast(float y, float x);
__device__ __forceinline__ double atan2_f64(double y, double x);
__device__ __forceinline__ double sqrt_any64(double x);
__device__ __forceinline__ double rsqrt_any64(double x);

// ---------------------------------------------------------------- math -----
// float uses the hardware approximations (v_sqrt_f32, v_rsq_f32, v_rcp_f32:
// about 1 ulp); double uses the hardware reciprocal square root refined by
// Newton steps (sqrt about 1 ulp) and the correctly rounded division.
template <typename T> struct Mth;

template <> struct Mth<float> {
    // (a constant argument is folded: the target builtin is not)
    static __device__ __forceinline__ float sqrt(float x) {
        return __builtin_constant_p(x) ? __builtin_sqrtf(x) : __builtin_amdgcn_sqrtf(x);
    }
    static __device__ __forceinline__ float rsqrt(float x) { return __builtin_amdgcn_rsqf(x); }
    static __device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
    static __device__ __forceinline__ float div(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }
    static __device__ __forceinline__ float atan2(float y, float x) { return atan2_fast(y, x); }
    static __device__ __forceinline__ float fabs(float x) { return __builtin_fabsf(x); }
};

template <> struct Mth<double> {
    static __device__ __forceinline__ double sqrt(double x) { return sqrt_any64(x); }
    static __device__ __forceinline__ double rsqrt(double x) { return rsqrt_any64(x); }
    static __device__ __forceinline__ double rcp(double x) { return 1.0 / x; }
    static __device__ __forceinline__ double div(double a, double b) { return a / b; }
    static __device__ __forceinline__ double atan2(double y, double x) { return atan2_f64(y, x); }
    static __device__ __forceinline__ double fabs(double x) { return __builtin_fabs(x); }
};

template <typename T> __device__ __forceinline__ T clamp01(T x) {
    return x < T(0) ? T(0) : (x > T(1) ? T(1) : x);
}

template <typename T> __device__ __forceinline__ bool finite(T x) { return __builtin_isfinite(x); }

// Power-of-two scale that brings max|a| into [0.5, 1): exact, so every
// product below stays clear of underflow and overflow; eigenvalues are scaled
// back at the end.  Returns the exponent e with max|a| = m * 2^e.
__device__ __forceinline__ int scale_exponent(double amax) {
    int e = 0;
    if (amax > 0.0 && __builtin_isfinite(amax)) (void)__builtin_frexp(amax, &e);
    return e;
}
__device__ __forceinline__ int scale_exponent_f(float amax) {
    int e = 0;
    if (amax > 0.0f && __builtin_isfinite(amax)) (void)__builtin_frexpf(amax, &e);
    return e;
}

// ------------------------------------------------ polynomial kernels -----
// Coefficients and their derivation: ksym_poly.hpp / gen_poly.py.

// 1/sqrt(x) for normal x > 0: hardware estimate (about 23 bits) refined by
// NEWTON Newton steps; two give full float64 accuracy, one about 2^-44.
template <int NEWTON = 2> __device__ __forceinline__ double rsqrt64(double x) {
    double y = __builtin_amdgcn_rsq(x);
#pragma unroll
    for (int k = 0; k < NEWTON; ++k) {
        const double e = __builtin_fma(-x * y, y, 1.0);
        y = __builtin_fma(0.5 * y, e, y);
    }
    return y;
}

// sqrt(z) for z in [0, 1/4]: sqrt = z / sqrt(z), with one correction step when
// full float64 accuracy is wanted (NEWTON = 2).
template <int NEWTON = 2> __device__ __forceinline__ double sqrt_small64(double z) {
    const double y = rsqrt64<NEWTON>(z);
    double s = z * y;
    if constexpr (NEWTON >= 2) {
        const double d = __builtin_fma(-s, s, z);
        s = __builtin_fma(0.5 * y, d, s);
    }
    return z > 0.0 ? s : 0.0;
}

// 1/sqrt(x) for x > 0 of any magnitude: inputs below 2^-900 are scaled by
// 2^600 first (exact), which keeps the hardware estimate in range.
__device__ __forceinline__ double rsqrt_any64(double x) {
    const bool tiny = x < 0x1p-900;
    const double y = rsqrt64(tiny ? x * 0x1p600 : x);
    return tiny ? y * 0x1p300 : y;
}

// sqrt(x) for x >= 0 of any magnitude (0 for x <= 0, NaN stays NaN):
// x / sqrt(x) and one correction step, about 1 ulp.
__device__ __forceinline__ double sqrt_any64(double x) {
    const bool tiny = x < 0x1p-900;
    const double xs = tiny ? x * 0x1p600 : x;
    const double y = rsqrt64(xs > 0.0 ? xs : 1.0);
    double r = xs * y;
    r = __builtin_fma(0.5 * y, __builtin_fma(-r, r, xs), r);
    r = tiny ? r * 0x1p-300 : r;
    return x > 0.0 ? r : (x == x ? 0.0 : x);
}

// arccos(r) for r in [-1, 1] through asin: |r| <= 1/2 uses
// acos r = pi/2 - asin r; otherwise acos |r| = 2 asin(sqrt((1 - |r|)/2)),
// and acos(-x) = pi - acos(x).
__device__ __forceinline__ double acos64(double r) {
    const double ar = __builtin_fabs(r);
    const bool small = ar <= 0.5;
    const double z = small ? ar * ar : 0.5 * (1.0 - ar);
    const double x = small ? ar : sqrt_small64(z);
    double P = poly::ASIN[11];
#pragma unroll
    for (int k = 10; k >= 0; --k) P = __builtin_fma(P, z, poly::ASIN[k]);
    const double a = __builtin_fma(x * z, P, x);   // asin(x)
    const double big = 2.0 * a;                     // acos(|r|) for |r| > 1/2
    if (small) return 0.5 * kPi - (r < 0.0 ? -a : a);
    return r < 0.0 ? kPi - big : big;
}

// sin and cos of t in [0, pi/3] (Taylor series, no argument reduction).
__device__ __forceinline__ void sincos_third(double t, double &s, double &c) {
    const double t2 = t * t;
    double ps = poly::S[9];
#pragma unroll
    for (int k = 8; k >= 0; --k) ps = __builtin_fma(ps, t2, poly::S[k]);
    double pc = poly::C[10];
#pragma unroll
    for (int k = 9; k >= 0; --k) pc = __builtin_fma(pc, t2, poly::C[k]);
    s = t * ps;
    c = pc;
}

// A float64 constant that needs both halves of a register pair, made opaque
// so that it is set in scalar registers at each use: hoisted out of the tile
// loop it would occupy a vector register pair throughout, or be spilled.
__device__ __forceinline__ double sconst(double c) {
    asm volatile("" : "+s"(c));
    return c;
}

// Float32-tail versions for the cubic stage of the float32 path: the first
// two terms of each series are formed in float64 and only the remainder (at
// most 1.2 % of the value) in float32, with coefficients that are literal
// operands; relative accuracy a few 1e-10.
__device__ __forceinline__ float tail_poly(const float *c, int deg, float t) {
    float p = c[deg];
#pragma unroll
    for (int k = deg - 1; k >= 0; --k) p = __builtin_fmaf(p, t, c[k]);
    return p;
}

// arccos(r) and pi - arccos(r), each formed without cancellation.
__device__ __forceinline__ void acos_pair(double r, double &D, double &Dc) {
    const double ar = __builtin_fabs(r);
    const bool small = ar <= 0.5;
    const double z = small ? ar * ar : 0.5 * (1.0 - ar);
    const double x = small ? ar : sqrt_small64<1>(z);
    const double T = (double)tail_poly(poly::AT, 6, (float)z);
    const double a = __builtin_fma(x * z, __builtin_fma(z, T, sconst(1.0 / 6.0)), x);   // asin(x)
    const double pi = sconst(kPi);
    if (small) {
        const double sa = r < 0.0 ? -a : a;        // asin(r)
        D = 0.5 * pi - sa;
        Dc = 0.5 * pi + sa;
    } else {
        const double b = 2.0 * a;                  // acos(|r|)
        D = r < 0.0 ? pi - b : b;
        Dc = r < 0.0 ? b : pi - b;
    }
}

// sin t for t in [0, pi/3].
__device__ __forceinline__ double sin_third(double t) {
    const double t2 = t * t;
    const double T = (double)tail_poly(poly::ST, 3, (float)t2);
    return __builtin_fma(t * t2, __builtin_fma(t2, T, sconst(-1.0 / 6.0)), t);
}

// atan2(y, x) in float32: reduce to t = min(|x|,|y|)/max(|x|,|y|) in [0, 1],
// atan t = t + t^3 Q(t^2), then fold the octant; y = -0 counts as +0, so the
// result lies in (-pi, pi].
__device__ __forceinline__ float atan2_fast(float y, float x) {
    const float ax = __builtin_fabsf(x), ay = __builtin_fabsf(y);
    const float mn = __builtin_fminf(ax, ay), mx = __builtin_fmaxf(ax, ay);
    const float t = mx > 0.0f ? mn * __builtin_amdgcn_rcpf(mx) : 0.0f;
    const float t2 = t * t;
    float Q = poly::ATAN[8];
#pragma unroll
    for (int k = 7; k >= 0; --k) Q = __builtin_fmaf(Q, t2, poly::ATAN[k]);
    float a = __builtin_fmaf(t * t2, Q, t);
    a = (ay > ax) ? 1.57079632679489662f - a : a;
    a = (x < 0.0f) ? 3.14159265358979324f - a : a;
    return (y < 0.0f) ? -a : a;
}

// The angle in [0, pi/2] whose sine and cosine are s, c >= 0, given also
// their squares s2q and c2q (s2q + c2q = 1): the arcsine of the smaller of
// the two, so the series argument stays in [0, 1/2] and no reciprocal is
// needed; asin x = x + x^3 R(x^2).
__device__ __forceinline__ float angle_from_squares(float s, float s2q, float c, float c2q) {
    const bool lo = s2q <= c2q;
    const float x = lo ? s : c, z = lo ? s2q : c2q;
    float R = poly::ASINF[7];
#pragma unroll
    for (int k = 6; k >= 0; --k) R = __builtin_fmaf(R, z, poly::ASINF[k]);
    const float a = __builtin_fmaf(x * z, R, x);
    return lo ? a : 1.57079632679489662f - a;
}

// ----------------------------------------------------- 3x3 cubic stage -----
// Paper §4, in float64, on the trace-free part B = A - m I with m = b/3.
// The shift is computed so that B's diagonal is exact when A is close to
// isotropic: m0 = A11 + ((A22 - A11) + (A33 - A11)) / 3, d_i = A_ii - m0
// (exact there by Sterbenz' lemma), then the rounding left in the trace is
// removed, d_i -= (d1 + d2 + d3) / 3, and m = m0 + that amount.  Every
// eigenvalue is carried as its deviation mu_k = lam_k - m, so quantities such
// as A11 - lam_k = d1 - mu_k keep their relative accuracy even when the spread
// of the spectrum is far below the last digit of m.
//   b (4.2) enters only through m; p (4.7) as printed (it uses only the
//   differences A_ii - A_jj); q through q = 27 det(B), which equals (4.8) in
//   exact arithmetic and avoids its O(||A||^3) cancellation; Delta (4.9) with
//   its argument clamped to [-1, 1]; (4.10)-(4.12) rewritten with
//   cos(x +- 2pi/3) = -cos(x)/2 -+ (sqrt3/2) sin(x), so one sincos(Delta/3)
//   gives all three, and the gaps in closed form:
//   lam1 - lam2 = sqrt(p) (cos t + sin t / sqrt3)     (max - min)
//   lam1 - lam3 = sqrt(p) (cos t - sin t / sqrt3)     (max - mid)
//   lam3 - lam2 = (2 / sqrt3) sqrt(p) sin t           (mid - min),   t = Delta/3.
struct Cubic {
    double m;                 // centre: lam_k = m + mu_k
    double d1, d2, d3;        // diagonal of B = A - m I (trace 0 up to rounding)
    double mu1, mu2, mu3;     // deviations of max, min, mid
    double g12, g13, g32;     // max-min, max-mid, mid-min (>= 0)
    double sp;                // sqrt(p)
    bool triple;              // p == 0
    bool fin;                 // p finite: every entry of A is finite (p sums
                              // squares of all six, scaled to at most 1)
};

__device__ __forceinline__ void center3(double a11, double a22, double a33, double &m, double &d1,
                                        double &d2, double &d3) {
    const double m0 = a11 + ((a22 - a11) + (a33 - a11)) * (1.0 / 3.0);
    d1 = a11 - m0;
    d2 = a22 - m0;
    d3 = a33 - m0;
    const double t = (d1 + d2 + d3) * (1.0 / 3.0);
    d1 -= t;
    d2 -= t;
    d3 -= t;
    m = m0 + t;
}

__device__ __forceinline__ Cubic cubic_stage(double a11, double a22, double a33, double a12,
                                             double a13, double a23) {
    Cubic c;
    center3(a11, a22, a33, c.m, c.d1, c.d2, c.d3);
    const double d1 = c.d1, d2 = c.d2, d3 = c.d3;
    const double off = a12 * a12 + a13 * a13 + a23 * a23;
    const double x12 = a11 - a22, x13 = a11 - a33, x23 = a22 - a33;
    const double p = 0.5 * (x12 * x12 + x13 * x13 + x23 * x23) + 3.0 * off;
    const double det = d1 * (d2 * d3 - a23 * a23) - a12 * (a12 * d3 - a13 * a23) +
                       a13 * (a12 * a23 - a13 * d2);
    const double q = 27.0 * det;
    // p == 0 is the paper's triple root; below 1e-280 (the matrix is scaled
    // to max |A_ij| in [1/2, 1)) B is so small against m that A is isotropic
    // to working precision, and 1/sqrt(p) would leave the normal range
    c.triple = !(p >= 1e-280);
    c.fin = __builtin_isfinite(p);
    const double ip = rsqrt64(c.triple ? 1.0 : p);   // 1 / sqrt(p)
    const double sp = c.triple ? 0.0 : p * ip;
    double r = 0.5 * q * (ip * ip * ip);              // q / (2 sqrt(p)^3)
    r = r > 1.0 ? 1.0 : (r < -1.0 ? -1.0 : r);
    const double Delta = acos64(r);
    double st, ct;
    sincos_third(Delta * (1.0 / 3.0), st, ct);
    const double spc = sp * ct, sps = sp * st * kInvSqrt3;
    c.mu1 = (2.0 / 3.0) * spc;
    c.mu2 = -(spc + 3.0 * sps) * (1.0 / 3.0);
    c.mu3 = -(spc - 3.0 * sps) * (1.0 / 3.0);
    c.g12 = spc + sps;
    c.g13 = spc - sps;
    c.g32 = 2.0 * sps;
    if (c.g13 < 0.0) c.g13 = 0.0;
    c.sp = sp;
    return c;
}

// The cubic stage of the float32 path: the same quantities as cubic_stage,
// with the three gaps from sines of t = Delta/3 and of pi/3 - t = (pi -
// Delta)/3, so each gap keeps its relative accuracy even when two eigenvalues
// nearly coincide:
//   lam3 - lam2 = (2/sqrt3) sqrt(p) sin t,  lam1 - lam3 = (2/sqrt3) sqrt(p) sin(pi/3 - t),
//   lam1 - lam2 = their sum;  mu1 = (2 g13 + g32) / 3 (the deviations sum to zero),
//   mu2 = mu1 - g12, mu3 = mu1 - g13.
// The arithmetic is float64 with float32 polynomial tails (relative accuracy
// a few 1e-10): the squared direction cosines formed from these deviations
// (u_quotients) can be differences of nearly equal terms, and their square
// roots turn an absolute error e into one of sqrt(e), so eigenvalues good to
// only 1e-8 would leave errors near 1e-4 in D.
__device__ __forceinline__ Cubic cubic_stage_gaps(double a11, double a22, double a33, double a12,
                                                  double a13, double a23) {
    Cubic c;
    center3(a11, a22, a33, c.m, c.d1, c.d2, c.d3);
    const double d1 = c.d1, d2 = c.d2, d3 = c.d3;
    const double off = a12 * a12 + a13 * a13 + a23 * a23;
    const double x12 = a11 - a22, x13 = a11 - a33, x23 = a22 - a33;
    const double p = 0.5 * (x12 * x12 + x13 * x13 + x23 * x23) + 3.0 * off;
    const double det = d1 * (d2 * d3 - a23 * a23) - a12 * (a12 * d3 - a13 * a23) +
                       a13 * (a12 * a23 - a13 * d2);
    c.triple = !(p >= 1e-280);
    c.fin = __builtin_isfinite(p);
    const double ip = rsqrt64<1>(c.triple ? 1.0 : p);
    const double sp = c.triple ? 0.0 : p * ip;
    double r = 13.5 * det * (ip * ip * ip);        // 27 det / (2 sqrt(p)^3)
    r = r > 1.0 ? 1.0 : (r < -1.0 ? -1.0 : r);
    double D, Dc;
    acos_pair(r, D, Dc);
    const double t = D * (1.0 / 3.0), tc = Dc * (1.0 / 3.0);
    const double k = (2.0 * kInvSqrt3) * sp;
    c.g32 = k * sin_third(t);
    c.g13 = k * sin_third(tc);
    c.g12 = c.g13 + c.g32;
    // mu1 + mu2 + mu3 = 0 with mu1 - mu2 = g12, mu1 - mu3 = g13 (a sum of
    // non-negative terms, so no cancellation)
    c.mu1 = (2.0 * c.g13 + c.g32) * (1.0 / 3.0);
    c.mu2 = c.mu1 - c.g12;
    c.mu3 = c.mu1 - c.g13;
    c.sp = sp;
    return c;
}

// ------------------------------------------------ 3x3 angle solve (§5) -----
// 1/x for positive normal x: hardware estimate refined by two Newton steps.
// 1/x for positive normal x: hardware estimate refined by NEWTON Newton steps
// (two: full float64 accuracy; one: about 2^-44).
template <int NEWTON = 2> __device__ __forceinline__ double rcp64(double x) {
    double y = __builtin_amdgcn_rcp(x);
#pragma unroll
    for (int k = 0; k < NEWTON; ++k) {
        const double e = __builtin_fma(-x, y, 1.0);
        y = __builtin_fma(y, e, y);
    }
    return y;
}

// atan2(y, x) in float64: t = min(|x|,|y|) / max(|x|,|y|) in [0, 1]; above
// tan(pi/8) the identity atan t = pi/4 - atan((1 - t)/(1 + t)) brings the
// argument into [0, tan(pi/8)], formed as one quotient (max - min)/(max + min);
// atan t = t + t^3 Q64(t^2) there; then the octant is folded.  Tiny inputs
// are scaled by a power of two first, so the reciprocal stays in range.  y =
// -0 counts as +0, so the result lies in (-pi, pi].
__device__ __forceinline__ double atan2_f64(double y, double x) {
    const double ax = __builtin_fabs(x), ay = __builtin_fabs(y);
    double mn = fmin(ax, ay), mx = fmax(ax, ay);
    const double s = mx < 0x1p-900 ? 0x1p600 : 1.0;
    mn *= s;
    mx *= s;
    const bool big = mn > 0.41421356237309503 * mx;   // tan(pi/8)
    const double num = big ? mx - mn : mn, den = big ? mx + mn : mx;
    const double t = den > 0.0 ? num * rcp64(den) : 0.0;
    const double u = t * t;
    double P = poly::ATAN64[10];
#pragma unroll
    for (int k = 9; k >= 0; --k) P = __builtin_fma(P, u, poly::ATAN64[k]);
    double a = __builtin_fma(t * u, P, t);
    const double pi = sconst(kPi);
    a = big ? 0.25 * pi - a : a;
    a = (ay > ax) ? 0.5 * pi - a : a;
    a = (x < 0.0) ? pi - a : a;
    return (y < 0.0) ? -a : a;
}


// The squared direction cosines of the first row of D, each as its own
// quotient.  With A = D diag(lam) D^T, u_k = D_1k^2 satisfies sum u_k = 1,
// sum u_k lam_k = A11 and sum u_k lam_k^2 = (A^2)_11, whose solution is
//   u_k = n_k / ((lam_k - lam_i)(lam_k - lam_j)),
//   n_k = A12^2 + A13^2 + (A11 - lam_i)(A11 - lam_j).
// Then v = cos^2 phi2 = u1 + u2 (this is (5.1)), 1 - v = u3, w = cos^2 phi3 =
// u1 / (u1 + u2) (this is (5.2)) and 1 - w = u2 / (u1 + u2).  Each pair is
// formed as p / (p + q), q / (p + q) from two non-negative numerators, so both
// members keep their relative accuracy (no 1 - x cancellation when x is close
// to 1) and still sum to 1 to rounding, which keeps D orthogonal; the float64
// numerators keep the quotients accurate when two eigenvalues are close.
// Labels: 1 = max, 2 = min, 3 = mid; e_k = A11 - lam_k; gaps as in Cubic.
//   v : 1 - v = n_v : -n_3 with n_v = (u1 + u2) g13 g32 = A12^2 + A13^2 + e3 (e1 + g32)
//   w : 1 - w = n_1 g32 : n_2 g13
struct URow {
    double v, s2sq, w, cw;   // cos^2 phi2, sin^2 phi2, cos^2 phi3, sin^2 phi3
};


// NEWTON = 1 is enough when the quotients are rounded to float32.
template <int NEWTON = 2>
__device__ __forceinline__ URow u_quotients(double d1, double mu1, double mu2, double mu3, double g13,
                                            double g32, double a12, double a13) {
    const double F = a12 * a12 + a13 * a13;
    const double e1 = d1 - mu1, e2 = d1 - mu2, e3 = d1 - mu3;
    URow u;
    const double pv = fmax(F + e3 * (e1 + g32), 0.0), qv = fmax(-(F + e1 * e2), 0.0);
    const double pw = fmax((F + e2 * e3) * g32, 0.0), qw = fmax((F + e1 * e3) * g13, 0.0);
    // an empty pair gives (1, 0); v = 0 gives w = 1, the paper's convention
    const double tv = pv + qv, tw = pw + qw;
    const bool okv = tv > 0.0, okw = tw > 0.0;
    const double Tv = okv ? tv : 1.0, Tw = okw ? tw : 1.0;
    const double r = rcp64<NEWTON>(Tv * Tw);   // one reciprocal for both pairs
    const double rv = Tw * r, rw = Tv * r;
    u.v = okv ? pv * rv : 1.0;
    u.s2sq = okv ? qv * rv : 0.0;
    u.w = okw ? pw * rw : 1.0;
    u.cw = okw ? qw * rw : 0.0;
    return u;
}

// The float32 path: the same numerators in float64 (they are differences of
// nearly equal terms), each pair's quotients in float32 from them (a few
// float32 ulps).
struct URowF {
    float v, s2sq, w, cw;
};
__device__ __forceinline__ URowF u_quotients_f32(double d1, double mu1, double mu2, double mu3, double g13,
                                                 double g32, double a12, double a13) {
    const double F = a12 * a12 + a13 * a13;
    const double e1 = d1 - mu1, e2 = d1 - mu2, e3 = d1 - mu3;
    const float pv = (float)fmax(F + e3 * (e1 + g32), 0.0), qv = (float)fmax(-(F + e1 * e2), 0.0);
    const float pw = (float)fmax((F + e2 * e3) * g32, 0.0), qw = (float)fmax((F + e1 * e3) * g13, 0.0);
    // an empty pair gives (1, 0); v = 0 gives w = 1, the paper's convention
    const float tv = pv + qv, tw = pw + qw;
    const bool okv = tv > 0.0f, okw = tw > 0.0f;
    const float rv = __builtin_amdgcn_rcpf(okv ? tv : 1.0f), rw = __builtin_amdgcn_rcpf(okw ? tw : 1.0f);
    URowF u;
    u.v = okv ? pv * rv : 1.0f;
    u.s2sq = okv ? qv * rv : 0.0f;
    u.w = okw ? pw * rw : 1.0f;
    u.cw = okw ? qw * rw : 0.0f;
    return u;
}

// Given the labelled eigenvalue differences G12 = lam1 - lam2, G13 = lam1 -
// lam3, G32 = lam3 - lam2 and the squared cosines and sines of phi2, phi3,
// choose the signs of phi2 = +-acos(sqrt v), phi3 = +-acos(sqrt w) (5.3)-(5.4)
// and phi1, and build D = R1 R2 R3 (2.6).
//
// Trig-free form of the selection.  Writing 2-vectors as complex numbers, a
// sign combination only flips signs inside g1 = (s3*alpha, s2*beta) and
// g2 = (gamma, s2*s3*delta) of (5.7)-(5.8).  phi1(1) = arg(conj(f1) g1) and
// 2 phi1(2) = arg(conj(f2) g2) (the angle from f to g, (5.11)-(5.14)), so
// e^{i phi1(2)} is the principal square root of z2 / |z2|, z2 = conj(f2) g2.
// The combination with the smallest circular distance Delta = |phi1(1) -
// phi1(2)| has the largest cos(Delta).  Flipping both signs negates z1 and
// keeps z2, so the two combinations of one product s2*s3 have cos(Delta) of
// opposite signs, and the choice splits in two:
//  - the product is the one with the larger cos^2(Delta), i.e. the larger
//    cos(2 Delta) = Re(z1^2 conj z2) / (|z1|^2 |z2|), where the norms
//    |z1| = |f1||g1|, |z2| = |f2||g2| do not depend on the signs.  Expanding
//    z1 = conj(f1) (alpha +- i beta'), z2 = conj(f2) (gamma +- i delta') and
//    using cos^2 + sin^2 = 1 for both angles, the difference between the two
//    products is exactly
//      Re(z+^2 conj z+) - Re(z-^2 conj z-) = 8 K G12 G13 G32 c2^2 c3 |s2 s3|,
//      K = A12 A13 (A22 - A33) - A23 (A12^2 - A13^2),
//    so the product is +1 when K >= 0 and -1 otherwise (a tie keeps the
//    first, +1).  K depends on the entries of A alone: the caller evaluates
//    it in float64, where its sign stays reliable down to gaps near the
//    float64 rounding level, while the two scores themselves differ only
//    by an amount proportional to the gaps;
//  - the overall sign makes Re(z1 conj h) >= 0, where h is a non-negative
//    multiple of the principal root: h = (|z2| + x, y) for x >= 0 and
//    (|y|, +-(|z2| - x)) for x < 0 (y = +-0 on the negative axis gives +i).
//    The two overall signs give D and D diag(1, -1, -1), so this choice
//    fixes the convention, not the accuracy.
// phi1 is phi1(1) when |f1| >= |f2| and phi1(2) otherwise (5.15); its cosine
// and sine come from normalising +-z1 or h.
// The brackets of (5.7)-(5.8) are rearranged with w + (1 - w) = 1 and
// v + (1 - v) = 1 so that no difference of nearly equal terms is formed:
//   (lam1 - lam2) w + lam2 - lam3 = G13 w - G32 (1 - w),
//   1 + (v - 2) w = (1 - w) - w (1 - v).
__device__ __forceinline__ double product_key(double a12, double a13, double a22, double a33,
                                              double a23) {
    return __builtin_fma(a12 * a13, a22 - a33, -a23 * __builtin_fma(a12, a12, -a13 * a13));
}

template <typename T> struct Rot {
    T c1, s1, c2, s2, c3, s3;   // cos/sin of phi1, phi2, phi3
};

template <typename T>
__device__ __forceinline__ Rot<T> select_angles(T a12, T a13, T a22, T a33, T a23, T G12, T G13, T G32,
                                                T v, T s2sq, T w, T cw, bool plus) {
    using M = Mth<T>;
    Rot<T> R;
    const T c2 = M::sqrt(v), s2 = M::sqrt(s2sq);
    const T c3 = M::sqrt(w), s3 = M::sqrt(cw);
    // g1 = (s3 al, s2 be), g2 = (ga, s2 s3 de), from (5.7)-(5.8) with
    // sin(2 phi) = 2 sin(phi) cos(phi); the product's sign t is folded into
    // al and de, so z1 = conj(f1) (t al + i be), z2 = conj(f2) (ga + i t de)
    const T t = plus ? T(1) : T(-1);
    const T al = t * G12 * c2 * s3 * c3;
    const T be = (G13 * w - G32 * cw) * s2 * c2;
    const T ga = G12 * (cw - w * s2sq) - G32 * v;
    const T de = t * T(2) * G12 * s2 * s3 * c3;
    // conj(f1) = (a12, a13), conj(f2) = (a22 - a33, 2 a23), from (5.5)-(5.6)
    const T e = a22 - a33, f = T(2) * a23;
    const T zx = al * a12 - be * a13, zy = al * a13 + be * a12;
    const T wx = ga * e - de * f, wy = ga * f + de * e;
    const T m2 = M::sqrt(wx * wx + wy * wy);
    const bool right = wx >= T(0);
    const T hx = right ? m2 + wx : M::fabs(wy);
    const T hy = right ? wy : ((wy >= T(0)) ? m2 - wx : wx - m2);
    const T sg = (zx * hx + zy * hy >= T(0)) ? T(1) : T(-1);
    const T f1sq = a12 * a12 + a13 * a13, f2sq = e * e + f * f;
    const bool use1 = f1sq >= f2sq;
    const T ux = use1 ? sg * zx : hx, uy = use1 ? sg * zy : hy;
    const T nn = ux * ux + uy * uy;
    if (nn > T(0)) {
        const T inv = M::rsqrt(nn);
        R.c1 = ux * inv;
        R.s1 = uy * inv;
    } else {
        R.c1 = T(1);
        R.s1 = T(0);
    }
    R.c2 = c2; R.s2 = sg * s2;
    R.c3 = c3; R.s3 = t * sg * s3;
    return R;
}

// D = R1(phi1) R2(phi2) R3(phi3), eq. (2.6), multiplied out (row-major).
template <typename T> __device__ __forceinline__ void build_D(const Rot<T>& R, T D[9]) {
    const T s2c3 = R.s2 * R.c3, s2s3 = R.s2 * R.s3;
    D[0] = R.c2 * R.c3;
    D[1] = -R.c2 * R.s3;
    D[2] = R.s2;
    D[3] = R.c1 * R.s3 + R.s1 * s2c3;
    D[4] = R.c1 * R.c3 - R.s1 * s2s3;
    D[5] = -R.s1 * R.c2;
    D[6] = R.s1 * R.s3 - R.c1 * s2c3;
    D[7] = R.s1 * R.c3 + R.c1 * s2s3;
    D[8] = R.c1 * R.c2;
}

template <typename T> __device__ __forceinline__ void angles_of(const Rot<T>& R, T phi[3]) {
    using M = Mth<T>;
    phi[0] = M::atan2(R.s1, R.c1);
    phi[1] = M::atan2(R.s2, R.c2);
    phi[2] = M::atan2(R.s3, R.c3);
}

// float32: phi2 and phi3 lie in [-pi/2, pi/2] (non-negative cosines c2 =
// sqrt(v), c3 = sqrt(w)), so each is +-asin of the smaller of its sine and
// cosine, from the squared values the angle solve already has; a sine of -0
// gives +0 like the general atan2.  phi1 is folded from the same arcsine of
// its unit vector's smaller component.
__device__ __forceinline__ void angles_of(const Rot<float>& R, float v, float s2sq, float w, float cw,
                                          float phi[3]) {
    // phi1 in (-pi, pi] from the unit vector (c1, s1): the angle of
    // (|c1|, |s1|) in [0, pi/2] from the squares, then folded into its
    // quadrant (a sine of -0 counts as +0, as in atan2_fast)
    const float t1 = angle_from_squares(__builtin_fabsf(R.s1), R.s1 * R.s1, __builtin_fabsf(R.c1), R.c1 * R.c1);
    const float q1 = R.c1 < 0.0f ? 3.14159265358979324f - t1 : t1;
    phi[0] = R.s1 < 0.0f ? -q1 : q1;
    const float t2 = angle_from_squares(__builtin_fabsf(R.s2), s2sq, R.c2, v);
    const float t3 = angle_from_squares(__builtin_fabsf(R.s3), cw, R.c3, w);
    phi[1] = R.s2 < 0.0f ? -t2 : t2;
    phi[2] = R.s3 < 0.0f ? -t3 : t3;
}

// Angles of a rotation D (det +1) with D = R1 R2 R3: phi1 from the third
// column's (D23, D33) = cos(phi2) (-sin phi1, cos phi1); then R1(phi1)^T D =
// R2 R3, whose second row is (sin phi3, cos phi3, 0) and whose (1,3), (3,3)
// entries are (sin phi2, cos phi2).  Computing phi3 and phi2 from R1^T D keeps
// D = R1 R2 R3 accurate also near cos(phi2) = 0.  If |phi3| > pi/2, columns 1
// and 2 of D are negated (still eigenvectors, det unchanged) and phi3 moves by
// pi, so phi2, phi3 land in [-pi/2, pi/2] like the general branch.
template <typename T> __device__ __forceinline__ void extract_angles(T D[9], T phi[3]) {
    using M = Mth<T>;
    T c1 = D[8], s1 = -D[5];
    const T h = c1 * c1 + s1 * s1;
    if (h > T(0)) {
        const T inv = M::rsqrt(h);
        c1 *= inv;
        s1 *= inv;
    } else {
        c1 = T(1);
        s1 = T(0);
    }
    T p3s = c1 * D[3] + s1 * D[6];
    T p3c = c1 * D[4] + s1 * D[7];
    if (p3c < T(0)) {
        for (int r = 0; r < 3; ++r) {
            D[3 * r] = -D[3 * r];
            D[3 * r + 1] = -D[3 * r + 1];
        }
        p3s = -p3s;
        p3c = -p3c;
    }
    phi[0] = M::atan2(s1, c1);
    phi[1] = M::atan2(D[2], c1 * D[8] - s1 * D[5]);
    phi[2] = M::atan2(p3s, p3c);
}

// ------------------------------------------------- a-posteriori check -----
// With B = A - m I (its diagonal d1, d2, d3 and the off-diagonal entries) and
// the deviations mu_k = lam_k - m, the residual of column k is
// r_k = B d_k - mu_k d_k = A d_k - lam_k d_k.  Fails when some ||r_k||^2
// exceeds lim2 = (tau_res ||A||_F)^2; for orthonormal D, ||r_k|| is the norm
// of column k of D^T B D - diag(mu), so this covers both a wrong eigenvector
// (off-diagonal entries) and a wrong pairing with mu_k (diagonal entry).  C is
// the arithmetic type; in float32 its rounding noise is about 1e-7 ||A||_F.
template <typename C>
__device__ __forceinline__ bool check_fails(C d1, C d2, C d3, C a12, C a13, C a23, const C d[9],
                                            C mu1, C mu2, C mu3, C lim2) {
    const C mu[3] = {mu1, mu2, mu3};
    bool bad = false;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const C x = d[k], y = d[3 + k], z = d[6 + k];
        const C r0 = (d1 - mu[k]) * x + a12 * y + a13 * z;
        const C r1 = a12 * x + (d2 - mu[k]) * y + a23 * z;
        const C r2 = a13 * x + a23 * y + (d3 - mu[k]) * z;
        bad |= !(r0 * r0 + r1 * r1 + r2 * r2 <= lim2);
    }
    return bad;
}

// The float32 check on two columns.  For orthonormal columns d0, d1, d2 the
// third residual follows from the first two: its components along d0 and d1
// are r0 . d2 and r1 . d2 (B is symmetric), and along d2 it is
// tr(B) - (mu0 + mu1 + mu2) - r0 . d0 - r1 . d1, where tr(B) and the sum of
// the deviations both vanish (up to rounding).  Hence ||r2||^2 <= ||r0||^2 +
// ||r1||^2 + (r0 . d0)^2 + (r1 . d1)^2 <= 2 (||r0||^2 + ||r1||^2), and the
// test ||r0||^2 + ||r1||^2 <= lim2 bounds every residual: columns 0 and 1 by
// sqrt(lim2), column 2 by sqrt(2 lim2) (float32 rounding of D and B adds
// about 1e-7 ||A||_F).  A wrong eigenvector or a wrong pairing with mu_k in
// any column shows in r0 or r1, since d2 is fixed by d0 and d1.
__device__ __forceinline__ bool check2_fails(float d1, float d2, float d3, float a12, float a13, float a23,
                                             const float d[9], float mu1, float mu2, float lim2) {
    const float mu[2] = {mu1, mu2};
    float n2 = 0.0f;
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const float x = d[k], y = d[3 + k], z = d[6 + k];
        const float r0 = (d1 - mu[k]) * x + a12 * y + a13 * z;
        const float r1 = a12 * x + (d2 - mu[k]) * y + a23 * z;
        const float r2 = a13 * x + a23 * y + (d3 - mu[k]) * z;
        n2 += r0 * r0 + r1 * r1 + r2 * r2;
    }
    return !(n2 <= lim2);
}

// First-order pair correction for differentiated calls (tau_vec > 0), in
// float64 on D as computed (its float type C).  Writing D = V (I + T + S)
// with V the true eigenvectors, T antisymmetric (a rotation) and S symmetric
// (D's departure from orthonormality), the off-diagonal entries of D^T B D
// are, to first order, T_jk (mu_j - mu_k) + (mu_j + mu_k) S_jk, and
// d_j^T d_k = 2 S_jk; so
//   X_jk = d_j^T B d_k - (mu_j + mu_k) / 2 * d_j^T d_k = T_jk (mu_j - mu_k)
// gives the rotation T_jk of each pair (j, k), which the adjoint would
// magnify by 1/(lam_j - lam_k).  D is replaced by D (I - T), which leaves a
// remainder of second order in T, and the angles by phi + dphi, where dphi
// solves M(phi) dphi = w for the body rates w of D^T dD = -T ([w]x = -T;
// M as in angle_body_cotangent), so that D = R1 R2 R3 (phi) still holds to
// first order.  Returns true (refine instead) when a rotation or an angle
// correction exceeds tau (a large one would leave a remainder that matters,
// as near gimbal lock, where dphi1 divides by cos phi2), or when a pair with
// a zero gap is not already exact.  In float32 the X_jk of a small gap would
// drown in rounding noise (about 1e-7 ||A||_F).  Slots 0 = max, 1 = min,
// 2 = mid; gaps g12 = mu1 - mu2 (pair 0, 1), g13 = mu1 - mu3 (0, 2),
// g32 = mu3 - mu2 (1, 2).
template <typename C>
__device__ __forceinline__ bool rotate_pairs64(double d1, double d2, double d3, double a12, double a13,
                                               double a23, double mu1, double mu2, double mu3, double g12,
                                               double g13, double g32, const Rot<C> &R, double tau, C D[9],
                                               C phi[3]) {
    double c[3][3];   // c[k] = column k
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        c[k][0] = (double)D[k];
        c[k][1] = (double)D[3 + k];
        c[k][2] = (double)D[6 + k];
    }
    auto Bcol = [&](int k, double out[3]) {
        out[0] = d1 * c[k][0] + a12 * c[k][1] + a13 * c[k][2];
        out[1] = a12 * c[k][0] + d2 * c[k][1] + a23 * c[k][2];
        out[2] = a13 * c[k][0] + a23 * c[k][1] + d3 * c[k][2];
    };
    auto dot = [&](const double *u, const double *v) { return u[0] * v[0] + u[1] * v[1] + u[2] * v[2]; };
    double b1[3], b2[3];
    Bcol(1, b1);
    Bcol(2, b2);
    const double x01 = dot(c[0], b1) - 0.5 * (mu1 + mu2) * dot(c[0], c[1]);
    const double x02 = dot(c[0], b2) - 0.5 * (mu1 + mu3) * dot(c[0], c[2]);
    const double x12 = dot(c[1], b2) - 0.5 * (mu2 + mu3) * dot(c[1], c[2]);
    // T_jk = X_jk / (lam_j - lam_k): lam0 - lam1 = g12, lam0 - lam2 = g13,
    // lam1 - lam2 = -g32 (a reciprocal good to 2^-44 is ample here)
    const double t01 = g12 > 0.0 ? x01 * rcp64<1>(g12) : 0.0;
    const double t02 = g13 > 0.0 ? x02 * rcp64<1>(g13) : 0.0;
    const double t12 = g32 > 0.0 ? -x12 * rcp64<1>(g32) : 0.0;
    bool big = (g12 == 0.0 && x01 != 0.0) || (g13 == 0.0 && x02 != 0.0) || (g32 == 0.0 && x12 != 0.0);
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        const double n0 = c[0][i] + c[1][i] * t01 + c[2][i] * t02;
        const double n1 = c[1][i] - c[0][i] * t01 + c[2][i] * t12;
        const double n2 = c[2][i] - c[0][i] * t02 - c[1][i] * t12;
        D[3 * i] = (C)n0;
        D[3 * i + 1] = (C)n1;
        D[3 * i + 2] = (C)n2;
    }
    // [w]x = -T: w = (t12, -t02, t01)
    const C w0 = (C)t12, w1 = (C)-t02, w2 = (C)t01;
    const C dp2 = R.s3 * w0 + R.c3 * w1;
    const C dp1 = Mth<C>::div(R.c3 * w0 - R.s3 * w1, R.c2);
    const C dp3 = w2 - R.s2 * dp1;
    const C tc = (C)tau;
    big = big || !(__builtin_fabs(t01) <= tau && __builtin_fabs(t02) <= tau && __builtin_fabs(t12) <= tau &&
                   Mth<C>::fabs(dp1) <= tc && Mth<C>::fabs(dp3) <= tc);
    phi[0] += dp1;
    phi[1] += dp2;
    phi[2] += dp3;
    return big;
}

// The float64 check with Rayleigh-quotient eigenvalues: as check_fails, and
// rq[k] receives d_k^T r_k = d_k^T B d_k - mu_k, the correction that turns
// mu_k into the Rayleigh quotient of column k.  For a unit vector d_k at an
// angle theta from its eigenvector the quotient is off by O(theta^2 ||A||)
// (at most ||r_k||^2 / gap), while the cubic's root can carry an error of
// order eps ||A||^2 / gap near a double root (arccos's slope in (4.9)).
__device__ __forceinline__ bool check_rq64(double d1, double d2, double d3, double a12, double a13, double a23,
                                           const double d[9], double mu1, double mu2, double mu3, double lim2,
                                           double rq[3]) {
    const double mu[3] = {mu1, mu2, mu3};
    double r[9];
    bool bad = false;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const double x = d[k], y = d[3 + k], z = d[6 + k];
        r[k] = (d1 - mu[k]) * x + a12 * y + a13 * z;
        r[3 + k] = a12 * x + (d2 - mu[k]) * y + a23 * z;
        r[6 + k] = a13 * x + a23 * y + (d3 - mu[k]) * z;
        const double n2 = r[k] * r[k] + r[3 + k] * r[3 + k] + r[6 + k] * r[6 + k];
        bad |= !(n2 <= lim2);
        rq[k] = x * r[k] + y * r[3 + k] + z * r[6 + k];
    }
    return bad;
}

// ------------------------------------------------- float64 refinement ------
// For matrices routed off the closed form (not in the paper): take the
// eigenvalue lc farther from the middle one (it is separated from the other
// two by at least half the spread), find its eigenvector u as the largest
// cross product of two rows of A - lc I, complete u to a right-handed
// orthonormal basis (x, y, u), diagonalise the 2x2 block [x y]^T A [x y] with
// one rotation -- the paper's 2x2 method, §3 -- and read the eigenvalues as
// Rayleigh quotients.  Columns are then sorted into the slots (max, min, mid),
// one column negated if that permutation was odd, and the angles re-extracted.
struct Refined {
    double lam[3];
    double D[9];
};

// Input: the shifted diagonal (a11, a22, a33) = diag(A - m I), the
// off-diagonal entries and lc as a deviation from m; outputs are deviations.
__device__ __forceinline__ Refined refine3(double a11, double a22, double a33, double a12,
                                           double a13, double a23, double lc) {
    const double r1x = a11 - lc, r1y = a12, r1z = a13;
    const double r2x = a12, r2y = a22 - lc, r2z = a23;
    const double r3x = a13, r3y = a23, r3z = a33 - lc;
    // cross products of row pairs
    double cx = r1y * r2z - r1z * r2y, cy = r1z * r2x - r1x * r2z, cz = r1x * r2y - r1y * r2x;
    double n = cx * cx + cy * cy + cz * cz;
    {
        const double tx = r1y * r3z - r1z * r3y, ty = r1z * r3x - r1x * r3z, tz = r1x * r3y - r1y * r3x;
        const double tn = tx * tx + ty * ty + tz * tz;
        if (tn > n) { cx = tx; cy = ty; cz = tz; n = tn; }
    }
    {
        const double tx = r2y * r3z - r2z * r3y, ty = r2z * r3x - r2x * r3z, tz = r2x * r3y - r2y * r3x;
        const double tn = tx * tx + ty * ty + tz * tz;
        if (tn > n) { cx = tx; cy = ty; cz = tz; n = tn; }
    }
    double ux, uy, uz;
    if (n > 0.0) {
        const double inv = rsqrt_any64(n);
        ux = cx * inv; uy = cy * inv; uz = cz * inv;
    } else {
        ux = 0.0; uy = 0.0; uz = 1.0;   // A - lc I = 0: any basis diagonalises A
    }
    // x = normalise(u x e_k) with e_k the axis least aligned with u; y = u x x
    const double ax = __builtin_fabs(ux), ay = __builtin_fabs(uy), az = __builtin_fabs(uz);
    double xx, xy, xz;
    if (ax <= ay && ax <= az) {        // u x e1 = (0, uz, -uy)
        xx = 0.0; xy = uz; xz = -uy;
    } else if (ay <= az) {             // u x e2 = (-uz, 0, ux)
        xx = -uz; xy = 0.0; xz = ux;
    } else {                           // u x e3 = (uy, -ux, 0)
        xx = uy; xy = -ux; xz = 0.0;
    }
    {
        const double inv = rsqrt_any64(xx * xx + xy * xy + xz * xz);
        xx *= inv; xy *= inv; xz *= inv;
    }
    const double yx = uy * xz - uz * xy, yy = uz * xx - ux * xz, yz = ux * xy - uy * xx;
    // A x, A y, A u
    const double Axx = a11 * xx + a12 * xy + a13 * xz, Axy = a12 * xx + a22 * xy + a23 * xz,
                 Axz = a13 * xx + a23 * xy + a33 * xz;
    const double Ayx = a11 * yx + a12 * yy + a13 * yz, Ayy = a12 * yx + a22 * yy + a23 * yz,
                 Ayz = a13 * yx + a23 * yy + a33 * yz;
    const double Aux = a11 * ux + a12 * uy + a13 * uz, Auy = a12 * ux + a22 * uy + a23 * uz,
                 Auz = a13 * ux + a23 * uy + a33 * uz;
    const double b11 = xx * Axx + xy * Axy + xz * Axz;
    const double b22 = yx * Ayx + yy * Ayy + yz * Ayz;
    const double b12 = xx * Ayx + xy * Ayy + xz * Ayz;
    const double lu = ux * Aux + uy * Auy + uz * Auz;
    // one rotation of the 2x2 block by the paper's 2x2 closed form (§3)
    const double dd = b11 - b22;
    const double sg = dd >= 0.0 ? 1.0 : -1.0;
    const double q2 = dd * dd + 4.0 * b12 * b12;
    double cphi = 1.0, sphi = 0.0, rr = 0.0;
    if (q2 > 0.0) {
        const double irr = rsqrt_any64(q2);   // 1 / rr
        rr = q2 * irr;
        const double h = 0.5 * (1.0 + __builtin_fabs(dd) * irr);   // in [1/2, 1]
        const double ih = rsqrt64(h);
        cphi = h * ih;                                             // sqrt(h)
        sphi = b12 * sg * irr * ih;                                // (b12 sg / rr) / cphi
    }
    const double mu1 = 0.5 * (b11 + b22 + sg * rr), mu2 = 0.5 * (b11 + b22 - sg * rr);
    // columns: v0 = c x + s y (mu1), v1 = -s x + c y (mu2), v2 = u (lu)
    double val[3] = {mu1, mu2, lu};
    double V[3][3] = {{cphi * xx + sphi * yx, cphi * xy + sphi * yy, cphi * xz + sphi * yz},
                      {-sphi * xx + cphi * yx, -sphi * xy + cphi * yy, -sphi * xz + cphi * yz},
                      {ux, uy, uz}};
    // sort descending with a 3-element network, tracking the parity
    int odd = 0;
    auto cswap = [&](int i, int j) {
        if (val[j] > val[i]) {
            const double t = val[i]; val[i] = val[j]; val[j] = t;
            for (int r = 0; r < 3; ++r) { const double s = V[i][r]; V[i][r] = V[j][r]; V[j][r] = s; }
            odd ^= 1;
        }
    };
    cswap(0, 1);
    cswap(1, 2);
    cswap(0, 1);
    // slots (max, min, mid) = sorted (0, 2, 1): one more transposition
    odd ^= 1;
    const double sgn = odd ? -1.0 : 1.0;
    Refined out;
    out.lam[0] = val[0];
    out.lam[1] = val[2];
    out.lam[2] = val[1];
    for (int r = 0; r < 3; ++r) {
        out.D[3 * r + 0] = V[0][r];
        out.D[3 * r + 1] = V[2][r];
        out.D[3 * r + 2] = sgn * V[1][r];
    }
    return out;
}

// -------------------------------------------------------- 2x2 (§3) ---------
// lam1,2 = (t +- sign(d) r) / 2 with d = A11 - A22, r = sqrt(d^2 + 4 A12^2)
// (3.2)-(3.3), sign(0) = +1.  phi = 1/2 atan2(2 A12 sign(d), |d|) equals
// 1/2 arctan(2 A12 / d) of (3.5) wherever d != 0 and lies in [-pi/4, pi/4];
// D = R(phi) (2.5) is built from the half-angle identities without trig:
// cos(2 phi) = |d| / r, cos(phi) = sqrt((1 + cos 2phi) / 2),
// sin(phi) = sin(2 phi) / (2 cos phi).
template <typename T> struct Eig2 {
    T l1, l2, c, s, phi;
};

template <typename T> __device__ __forceinline__ Eig2<T> eig2_one(T a11, T a22, T a12) {
    using M = Mth<T>;
    Eig2<T> o;
    const T d = a11 - a22;
    const T sg = d >= T(0) ? T(1) : T(-1);
    const T ad = M::fabs(d);
    const T y = T(2) * a12 * sg;
    const T r = M::sqrt(d * d + y * y);
    const T t = a11 + a22;
    o.l1 = T(0.5) * (t + sg * r);
    o.l2 = T(0.5) * (t - sg * r);
    if (r > T(0)) {
        const T ir = M::rcp(r);
        o.c = M::sqrt(T(0.5) + T(0.5) * ad * ir);
        o.s = M::div(T(0.5) * y * ir, o.c);
    } else {
        o.c = T(1);
        o.s = T(0);
    }
    o.phi = T(0.5) * M::atan2(y, ad);
    return o;
}

// ------------------------------------------------------- 3x3 adjoint -------
// Abar = D [diag(glam) + F o (D^T gD)] D^T with F_ij = (lam_j - lam_i) /
// ((lam_j - lam_i)^2 + eps^2).  Only the symmetric part of Abar matters for the
// six planes: with S = M + M^T, S_ii = 2 glam_i and, because F is
// antisymmetric, S_ij = F_ij (E_ij - E_ji) for E = D^T gD; then gA_ij =
// (D S D^T)_ij off the diagonal and gA_ii = (D S D^T)_ii / 2.
// Slots: 0 = max, 1 = min, 2 = mid; gaps g12 = lam0 - lam1, g13 = lam0 - lam2,
// g32 = lam2 - lam1.  wb: the body-rate cotangent of the Euler angles (see
// angle_body_cotangent), added to (E_32, E_13, E_21); zeros without angles.
// The gap-regularised weight d / (d^2 + eps^2) of the adjoint, with the
// value 0 that it takes for every eps > 0 also at d = 0 when eps = 0 (an
// exactly repeated eigenvalue of the zero matrix, whose eps = eps_rel ||lam||
// vanishes), where the formula would read 0/0.
template <typename T> __device__ __forceinline__ T gap_weight(T d, T eps2) {
    return d != T(0) ? Mth<T>::div(d, d * d + eps2) : T(0);
}

template <typename T>
__device__ __forceinline__ void adjoint3(const T D[9], const T gl[3], const T gD[9], T g12, T g13,
                                         T g32, T eps2, const T wb[3], T gA[6]) {
    using M = Mth<T>;
    // K_ij = E_ij - E_ji = sum_r (D_ri gD_rj - D_rj gD_ri)
    T K01 = T(0), K02 = T(0), K12 = T(0);
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        K01 += D[3 * r] * gD[3 * r + 1] - D[3 * r + 1] * gD[3 * r];
        K02 += D[3 * r] * gD[3 * r + 2] - D[3 * r + 2] * gD[3 * r];
        K12 += D[3 * r + 1] * gD[3 * r + 2] - D[3 * r + 2] * gD[3 * r + 1];
    }
    K01 -= wb[2];
    K02 += wb[1];
    K12 -= wb[0];
    // F_01 = (lam1 - lam0)/(..) = -g12/(g12^2+eps2); F_02 = -g13/(..); F_12 = (lam2 - lam1)/(..) = g32/(..)
    const T S01 = -gap_weight(g12, eps2) * K01;
    const T S02 = -gap_weight(g13, eps2) * K02;
    const T S12 = gap_weight(g32, eps2) * K12;
    const T S00 = T(2) * gl[0], S11 = T(2) * gl[1], S22 = T(2) * gl[2];
    // Tm = D S (row-major)
    T Tm[9];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        const T x = D[3 * i], y = D[3 * i + 1], z = D[3 * i + 2];
        Tm[3 * i + 0] = x * S00 + y * S01 + z * S02;
        Tm[3 * i + 1] = x * S01 + y * S11 + z * S12;
        Tm[3 * i + 2] = x * S02 + y * S12 + z * S22;
    }
    auto G = [&](int i, int j) {
        return Tm[3 * i] * D[3 * j] + Tm[3 * i + 1] * D[3 * j + 1] + Tm[3 * i + 2] * D[3 * j + 2];
    };
    gA[0] = T(0.5) * G(0, 0);
    gA[1] = T(0.5) * G(1, 1);
    gA[2] = T(0.5) * G(2, 2);
    gA[3] = G(0, 1);
    gA[4] = G(0, 2);
    gA[5] = G(1, 2);
}

// The Euler angles' cotangent gphi as a cotangent of the body rates w of
// D^T dD = [w]x (D = R1 R2 R3, eq. (2.6), R_k = exp(phi_k [e_k]x)): w = M dphi
// with columns (c2 c3, -c2 s3, s2), (s3, c3, 0), (0, 0, 1), so wb = M^-T gphi.
// M^-T divides by c2 = cos phi2 (gimbal lock at c2 = 0), regularised as
// c2 / (c2^2 + delta2).
template <typename T>
__device__ __forceinline__ void angle_body_cotangent(T c2, T s2, T c3, T s3, const T gphi[3], T delta2,
                                                     T wb[3]) {
    const T u = (gphi[0] - s2 * gphi[2]) * Mth<T>::div(c2, c2 * c2 + delta2);
    const T v = gphi[1];
    wb[0] = c3 * u + s3 * v;
    wb[1] = -s3 * u + c3 * v;
    wb[2] = gphi[2];
}

// ------------------------------------------------------- 2x2 adjoint -------
// The same first-order result for A = D diag(lam1, lam2) D^T with D = R(phi),
// eq. (2.5) (planes D11, D12, D21, D22): E = D^T gD, and the angle cotangent
// enters as E_21 += gphi, since D^T dD = [[0, -dphi], [dphi, 0]] gives
// dphi = d2^T dA d1 / (lam1 - lam2).  M = diag(glam) + F o E with F_12 =
// (lam2 - lam1) / ((lam2 - lam1)^2 + eps^2) = -F_21; Abar = D M D^T and
// gA = (Abar_11, Abar_22, Abar_12 + Abar_21).  d = lam2 - lam1.
template <typename T>
__device__ __forceinline__ void adjoint2(const T D[4], const T gl[2], const T gD[4], T gphi, T d, T eps2,
                                         T gA[3]) {
    const T e12 = D[0] * gD[1] + D[2] * gD[3];
    const T e21 = D[1] * gD[0] + D[3] * gD[2] + gphi;
    const T f = gap_weight(d, eps2);
    const T m00 = gl[0], m01 = f * e12, m10 = -f * e21, m11 = gl[1];
    const T t00 = D[0] * m00 + D[1] * m10, t01 = D[0] * m01 + D[1] * m11;
    const T t10 = D[2] * m00 + D[3] * m10, t11 = D[2] * m01 + D[3] * m11;
    gA[0] = t00 * D[0] + t01 * D[1];
    gA[1] = t10 * D[2] + t11 * D[3];
    gA[2] = (t00 * D[2] + t01 * D[3]) + (t10 * D[0] + t11 * D[1]);
}

}  // namespace ksym
