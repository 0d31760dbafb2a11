// Tile processors and __global__ kernels for the ksym C ABI (gfx950, wave64).
//
// Work decomposition: every wavefront works on its own tiles of 64 * MPL
// matrices (MPL = matrices per lane) and walks them grid-stride; matrix
// k*64 + lane of a tile belongs to `lane`, so every plane load and store is one
// contiguous 64-element run and needs no staging.  The waves of a workgroup
// never wait for each other, except at the float64 kernels' final drain.
//
// Refinement routing (3x3 float32 and float64 check paths): a lane whose
// matrix fails the check stores its provisional result and appends the matrix
// to its wave's queue in LDS (ballot + popcount for the count, mbcnt for the
// lane's rank; the count lives in a scalar register).  When the queue holds 64
// entries the wave refines them together, entry j on lane j, so the float64
// refinement runs on full wavefronts, and overwrites those outputs; what is
// left when the wave has finished its tiles is refined in one partly filled
// round (float32: per wave; float64: pooled over the workgroup, the one
// workgroup barrier of these kernels).
//
// Memory access: every plane is read and written through a raw buffer
// descriptor (base address and size in bytes) with a 32-bit lane offset.  A
// load outside the plane returns 0 and a store outside it is dropped by the
// hardware, so the last, partial tile of a launch needs no bounds tests and an
// absent output plane is simply a plane of size 0.  One launch covers at most
// KSYM_CHUNK matrices (less for array-of-structures input); the host splits
// larger batches.
#pragma once

#include <stddef.h>

#include "ksym_device.hpp"

namespace ksym {


enum { PATH_FP32_FIXUP = 0, PATH_FP64_PLAIN = 1, PATH_FP64_FIXUP = 2 };

// Output planes of the 3x3 forward, in this order: lam (3), D (9, row-major),
// phi (3), gap (3).
constexpr int NOUT3 = 18;
constexpr int O_LAM = 0, O_D = 3, O_PHI = 12, O_GAP = 15;

template <typename T> struct Eig3Ptrs {
    const T *in[6];
    T *out[NOUT3];   // any entry may be null
    uint8_t *flags;
};

// Matrices per launch: plane sizes and offsets inside a launch are 32-bit byte
// counts (structure-of-arrays planes of float64 reach 2^31 bytes; records of
// six float32 / float64 values take 24 / 48 bytes each).
constexpr int64_t KSYM_CHUNK = int64_t(1) << 28;
constexpr int64_t KSYM_CHUNK_AOS_F32 = int64_t(1) << 27;
constexpr int64_t KSYM_CHUNK_AOS_F64 = int64_t(1) << 26;

struct Eig3Params {
    int64_t n;            // at most KSYM_CHUNK
    double tau_gap, tau_res, tau_vec, tau_dbl;
    unsigned *counters;   // [0] refined, [1] non-finite; may be null
    int32_t zero;         // always 0; see put3
    int32_t drain_tiles;  // queue age limit in wave tiles (0 = full waves only)
    // the float32 check's threshold, rounded once on the host so that it
    // stays a scalar operand: (float)tau_res squared in float
    float tau_res2_f, pad_f;
};

// Fills the float32 threshold of a parameter block whose double fields are set.
__host__ inline void finish_params(Eig3Params &prm) {
    const float tr = (float)prm.tau_res;
    prm.tau_res2_f = tr * tr;
    prm.pad_f = 0.0f;
}

template <typename T> struct Eig3Args {
    Eig3Ptrs<T> p;
    Eig3Params prm;
    const T *aos;   // record input for the array-of-structures kernel
};

template <typename T> struct Out3 {
    T v[NOUT3];  // lam, D, phi, gap at O_LAM, O_D, O_PHI, O_GAP
    int flag;
    bool refine;
    double lc;   // isolated eigenvalue (scaled units) handed to the refinement
};

// x * 2^e with one rounding for any e (exact unless the result is subnormal).
// The scale factors themselves would leave the range: a float64 matrix whose
// entries are all subnormal has e < -1022, and float32 entries near the top
// of the range have e = 128.
__device__ __forceinline__ double sc2(double x, int e) { return __builtin_ldexp(x, e); }
__device__ __forceinline__ float sc2(float x, int e) { return __builtin_ldexpf(x, e); }

// One 3x3 matrix through §4-§5 on the plain float64 path: the general branch
// with v, w of (5.1)-(5.2) as printed, or the paper's double-root branch
// (5.20)-(5.25) with the output slots restored, or the triple root; no check.
// (The checked paths stream their outputs: eig3_f32, eig3_f64s.)
template <typename T>
__device__ __forceinline__ void eig3_one(const T ain[6], const Eig3Params &prm, Out3<T> &o) {
    const bool fin = finite(ain[0]) && finite(ain[1]) && finite(ain[2]) && finite(ain[3]) &&
                     finite(ain[4]) && finite(ain[5]);
    double amax = 0.0;
#pragma unroll
    for (int c = 0; c < 6; ++c) amax = fmax(amax, __builtin_fabs((double)ain[c]));
    const int ex = fin ? scale_exponent(amax) : 0;
    double a[6];
#pragma unroll
    for (int c = 0; c < 6; ++c) a[c] = fin ? sc2((double)ain[c], -ex) : 0.0;
    const double a11 = a[0], a22 = a[1], a33 = a[2], a12 = a[3], a13 = a[4], a23 = a[5];
    const Cubic cu = cubic_stage(a11, a22, a33, a12, a13, a23);
    o.refine = false;
    o.lc = 0.0;
    if (cu.triple) {
        // §5, p = 0: A = lam I with lam = A11; D = I, angles 0.
#pragma unroll
        for (int i = 0; i < 9; ++i) o.v[O_D + i] = (i % 4 == 0) ? T(1) : T(0);
        o.v[O_LAM] = o.v[O_LAM + 1] = o.v[O_LAM + 2] = (T)sc2(cu.m, ex);
        o.v[O_PHI] = o.v[O_PHI + 1] = o.v[O_PHI + 2] = T(0);
        o.v[O_GAP] = o.v[O_GAP + 1] = o.v[O_GAP + 2] = T(0);
        o.flag = FLAG_TRIPLE;
    } else {
        const double split = fmin(cu.g13, cu.g32);
        const bool dbl = (cu.g13 * cu.g32 == 0.0) || split < prm.tau_dbl * cu.sp;
        const T A12 = (T)a12, A13 = (T)a13, A22 = (T)a22, A33 = (T)a33, A23 = (T)a23;
        if (dbl) {
            // double root: labels (lam, lam, lam_s), s = cos^2 phi2 (5.21), phi3 = 0;
            // deviations from the centre m keep s accurate when the spread is tiny.
            // The mean lm of the close pair serves (5.21) only: the outputs keep
            // the roots (4.10)-(4.12) and their gaps, which in slot order are
            // (mu1, mu2, mu3) in both cases below
            double lm, ls;
            if (cu.g13 < cu.g32) { lm = 0.5 * (cu.mu1 + cu.mu3); ls = cu.mu2; }
            else { lm = 0.5 * (cu.mu3 + cu.mu2); ls = cu.mu1; }
            const T s = clamp01((T)((cu.d1 - ls) / (lm - ls)));
            // (G12 = 0, phi3 = 0: both products score alike; the first is kept)
            const Rot<T> R = select_angles<T>(A12, A13, A22, A33, A23, T(0), (T)(lm - ls), (T)(ls - lm), s,
                                              T(1) - s, T(1), T(0), true);
            T Di[9];
            build_D(R, Di);
            if (ls > lm) {   // (ls, lm, lm): columns (3, 1, 2), even permutation
                for (int r = 0; r < 3; ++r) {
                    o.v[O_D + 3 * r] = Di[3 * r + 2]; o.v[O_D + 3 * r + 1] = Di[3 * r]; o.v[O_D + 3 * r + 2] = Di[3 * r + 1];
                }
            } else {         // (lm, ls, lm): columns (1, 3, -2), odd permutation + sign
                for (int r = 0; r < 3; ++r) {
                    o.v[O_D + 3 * r] = Di[3 * r]; o.v[O_D + 3 * r + 1] = Di[3 * r + 2]; o.v[O_D + 3 * r + 2] = -Di[3 * r + 1];
                }
            }
            extract_angles<T>(o.v + O_D, o.v + O_PHI);
            o.v[O_LAM] = (T)sc2(cu.m + cu.mu1, ex);
            o.v[O_LAM + 1] = (T)sc2(cu.m + cu.mu2, ex);
            o.v[O_LAM + 2] = (T)sc2(cu.m + cu.mu3, ex);
            o.v[O_GAP] = (T)sc2(cu.g12, ex);
            o.v[O_GAP + 1] = (T)sc2(cu.g13, ex);
            o.v[O_GAP + 2] = (T)sc2(cu.g32, ex);
            o.flag = FLAG_DOUBLE;
        } else {
            // general branch (5.1)-(5.15), with the eigenvalue differences
            // taken from the float64 stage and v, w evaluated as printed
            const T G12 = (T)cu.g12, G13 = (T)cu.g13, G32 = (T)cu.g32;
            const T e1 = (T)(cu.d1 - cu.mu1), e3 = (T)(cu.d1 - cu.mu3);   // A11 - lam1, A11 - lam3
            const T v = clamp01(Mth<T>::div(A12 * A12 + A13 * A13 + e3 * (e1 + G32), G32 * G13));
            const T w = (v == T(0)) ? T(1) : clamp01(Mth<T>::div(e3 + G32 * v, G12 * v));
            const T s2sq = T(1) - v, cw = T(1) - w;
            const bool plus = !(product_key(a12, a13, a22, a33, a23) < 0.0);
            const Rot<T> R = select_angles<T>(A12, A13, A22, A33, A23, G12, G13, G32, v, s2sq, w, cw, plus);
            build_D(R, o.v + O_D);
            angles_of(R, o.v + O_PHI);
            o.v[O_LAM] = (T)sc2(cu.m + cu.mu1, ex);
            o.v[O_LAM + 1] = (T)sc2(cu.m + cu.mu2, ex);
            o.v[O_LAM + 2] = (T)sc2(cu.m + cu.mu3, ex);
            o.v[O_GAP] = (T)sc2(cu.g12, ex);
            o.v[O_GAP + 1] = (T)sc2(cu.g13, ex);
            o.v[O_GAP + 2] = (T)sc2(cu.g32, ex);
            o.flag = FLAG_GENERAL;
        }
    }
    if (!fin) {
        const T nan = T(__builtin_nan(""));
#pragma unroll
        for (int i = 0; i < NOUT3; ++i) o.v[i] = nan;
        o.flag = FLAG_NONFINITE;
        o.refine = false;
    }
}

// The second attempt of the float32 path: the squared cosines v, 1 - v of
// phi2 and w, 1 - w of phi3 (5.1)-(5.2) where the general branch's quotients
// lose them, fed to the general branch's angle selection.
//  - Double root, eqs. (5.20)-(5.25) in the general branch's slot order: the
//    close pair is taken as one eigenvalue lm (their mean) beside the
//    isolated ls.  At a double root A - lm I = (ls - lm) u u^T for the
//    isolated unit eigenvector u, so row i of A - lm I has the squared norm
//    (ls - lm)^2 u_i^2, and any orthonormal basis of the pair's plane
//    completes D.  With u in its slot (max or min) and the pair's basis
//    chosen so that the first-row entry of the other of those two columns
//    vanishes (phi3 = 0 for an isolated max, +-pi/2 for an isolated min),
//    v = u1^2 and w = 1 or 0.  This is (5.21), whose cos^2 phi2 =
//    (A11 - ls)/(lm - ls) is 1 - u1^2 in the paper's column order (u third,
//    phi3 = 0), written for the slot order; v and 1 - v are quotients of the
//    row norms, which keep their relative accuracy where either is near 0
//    (the difference A11 - ls would carry the cubic step's absolute error,
//    and the square root in cos phi2 its square root).  The residuals of
//    this D are bounded by the pair's split, where the general branch's
//    angle formulas lose accuracy as 1 / split.
//  - Diagonal matrix (all off-diagonal entries zero): D is a signed
//    permutation, whose first row is the axis of A11's slot, so v = 1, w = 1
//    (A11 the largest), v = 1, w = 0 (the smallest) or v = 0, w = 1 (the
//    middle one).  The gaps are taken from the sorted diagonal, exact where
//    two entries coincide, and the selection then gives phi1 = 0 or +-pi/2.
//    The general branch reaches these squared cosines, exactly 0 or 1, only
//    up to the cubic step's absolute error, and the square root turned that
//    into about 1e-5 in D.
__device__ __forceinline__ Rot<float> second_attempt_f32(const Cubic &cu, float A12, float A13, float A22,
                                                         float A33, float A23, bool plus, bool diag, float &v,
                                                         float &s2sq, float &w, float &cw) {
    float G12 = (float)cu.g12, G13 = (float)cu.g13, G32 = (float)cu.g32;
    if (diag) {
        const double x0 = cu.d1, x1 = cu.d2, x2 = cu.d3;
        const double hi = fmax(fmax(x0, x1), x2), lo = fmin(fmin(x0, x1), x2);
        const double mid = fmax(fmin(x0, x1), fmin(fmax(x0, x1), x2));
        G12 = (float)(hi - lo);
        G13 = (float)(hi - mid);
        G32 = (float)(mid - lo);
        const bool top = x0 == hi, bottom = !top && x0 == lo;
        v = (top || bottom) ? 1.0f : 0.0f;
        w = bottom ? 0.0f : 1.0f;
    } else {
        const bool iso_max = !(cu.g13 < cu.g32);   // pair (mid, min), isolated max; else pair (max, mid)
        const double lm = iso_max ? 0.5 * (cu.mu3 + cu.mu2) : 0.5 * (cu.mu1 + cu.mu3);
        const double b12 = A12, b13 = A13, b23 = A23;
        const double e1 = cu.d1 - lm, e2 = cu.d2 - lm, e3 = cu.d3 - lm;
        const double r1 = e1 * e1 + b12 * b12 + b13 * b13;                                  // (ls - lm)^2 u1^2
        const double r23 = e2 * e2 + e3 * e3 + b12 * b12 + b13 * b13 + 2.0 * b23 * b23;   // (ls - lm)^2 (u2^2 + u3^2)
        const double inv = 1.0 / (r1 + r23);
        v = (float)(r1 * inv);
        w = iso_max ? 1.0f : 0.0f;
        s2sq = (float)(r23 * inv);
    }
    if (diag) s2sq = 1.0f - v;
    cw = 1.0f - w;
    return select_angles<float>(A12, A13, A22, A33, A23, G12, G13, G32, v, s2sq, w, cw, plus);
}

// The float32 path for one matrix: the cubic stage in float64 (with float32
// polynomial tails), the squared cosines of the angle solve as float64
// quotients, the rest in float32, and the a-posteriori check in float32 on
// B = A - m I.  Outputs leave through sink.put(k, value) as soon as they
// exist (plane k of lam, D, phi, gap), which keeps few of them in registers.
// A result of the general branch that fails the check gets a second attempt,
// checked in the same way, before the matrix goes to the refinement: for a
// diagonal matrix, or where the split of the middle eigenvalue is below
// tau_res sqrt(p), the squared cosines of second_attempt_f32 go through the
// same angle selection; the flag keeps the cubic stage's classification
// (tau_dbl) either way.
// Sets refine (and the isolated eigenvalue lc for the refinement, a float64
// deviation in scaled units) and returns the flag.
template <bool GRAD, typename Sink>
__device__ __forceinline__ int eig3_f32(const float ain[6], const Eig3Params &prm, const Sink &sink,
                                        bool &refine, double &lc) {
    // max|A_ij| ignores a NaN entry and is infinite for an infinite one (then
    // the scale is 1); a non-finite entry makes p non-finite (cu.fin) and the
    // arithmetic below merely carries it along
    float amax = __builtin_fmaxf(__builtin_fmaxf(__builtin_fabsf(ain[0]), __builtin_fabsf(ain[1])),
                                 __builtin_fabsf(ain[2]));
    amax = __builtin_fmaxf(amax, __builtin_fmaxf(__builtin_fmaxf(__builtin_fabsf(ain[3]),
                                                                 __builtin_fabsf(ain[4])),
                                                 __builtin_fabsf(ain[5])));
    const int ex = scale_exponent_f(amax);
    double a[6];
#pragma unroll
    for (int c = 0; c < 6; ++c) a[c] = sc2((double)ain[c], -ex);
    const Cubic cu = cubic_stage_gaps(a[0], a[1], a[2], a[3], a[4], a[5]);
    const bool fin = cu.fin;
    lc = 0.0;
    const double split = cu.g13 < cu.g32 ? cu.g13 : cu.g32;
    const bool dbl = (cu.g13 * cu.g32 == 0.0) || split < prm.tau_dbl * cu.sp;
    // Every matrix runs the general path below, so that every store lies on
    // one straight path: the compiler then counts the memory operations in
    // flight exactly, instead of assuming a path without stores and waiting
    // for the prefetched inputs at every tile.  For p = 0 (A = lam I, §5,
    // which for float32 input means B = 0 exactly) that path yields the
    // special outputs exactly: all gaps and deviations are 0, the squared
    // cosines are the empty pairs' (1, 0), so D = I, the angles are 0 and
    // lam = m.  A non-finite input is queued, and the drain writes NaN.
    const bool special = cu.triple || !fin;
    const int flag = special ? (fin ? FLAG_TRIPLE : FLAG_NONFINITE) : (dbl ? FLAG_DOUBLE : FLAG_GENERAL);
    sink.flag(flag);
    {
        const float lam[3] = {(float)sc2(cu.m + cu.mu1, ex), (float)sc2(cu.m + cu.mu2, ex),
                              (float)sc2(cu.m + cu.mu3, ex)};
        const float gap[3] = {(float)sc2(cu.g12, ex), (float)sc2(cu.g13, ex), (float)sc2(cu.g32, ex)};
        sink.template put_n<3>(O_LAM, lam);
        sink.template put_n<3>(O_GAP, gap);
    }
    // differentiated calls refine every double root (the pair correction
    // needs both columns of a pair); otherwise the check decides
    bool bad = !fin || (GRAD && !cu.triple && dbl);
    if (prm.tau_gap > 0.0) {   // uniform: skipped at the default 0
        asm volatile("");      // (keeps the branch; see check_fails)
        const double l1 = __builtin_fabs(cu.m + cu.mu1), l2 = __builtin_fabs(cu.m + cu.mu2);
        bad = bad || (!cu.triple && split < prm.tau_gap * (l1 > l2 ? l1 : l2));
    }
    lc = (cu.g13 >= cu.g32) ? cu.mu1 : cu.mu2;
    // general branch (5.1)-(5.15): the four squared cosines and sines from
    // float64 numerators (u_quotients_f32), the rest of the angle solve in
    // float32
    const URowF u = u_quotients_f32(cu.d1, cu.mu1, cu.mu2, cu.mu3, cu.g13, cu.g32, a[3], a[4]);
    const float A22 = (float)a[1], A33 = (float)a[2];
    const float A12 = (float)a[3], A13 = (float)a[4], A23 = (float)a[5];
    const float G12 = (float)cu.g12, G13 = (float)cu.g13, G32 = (float)cu.g32;
    const bool plus = !(product_key(a[3], a[4], a[1], a[2], a[5]) < 0.0);
    const float v = u.v, s2sq = u.s2sq, w = u.w, cw = u.cw;
    const Rot<float> R = select_angles<float>(A12, A13, A22, A33, A23, G12, G13, G32, v, s2sq, w, cw, plus);
    float phi[3];
    angles_of(R, v, s2sq, w, cw, phi);
    float D[9];
    if constexpr (GRAD) {
        // differentiated calls (tau_vec > 0): the pairs' first-order rotation
        // removed from D and the angles before they are stored
        build_D(R, D);
        const bool big = rotate_pairs64<float>(cu.d1, cu.d2, cu.d3, a[3], a[4], a[5], cu.mu1, cu.mu2, cu.mu3,
                                               cu.g12, cu.g13, cu.g32, R, prm.tau_vec, D, phi);
        // the adjoint's F_jk = g/(g^2 + eps^2) needs each gap to a few digits;
        // the cubic stage's gaps carry absolute errors of a few 1e-10 sqrt(p)
        // (its float32 tails), so a gap below 1e-5 sqrt(p) takes the
        // refinement, whose Rayleigh quotients give it to float64 rounding
        const bool close = split < 1e-5 * cu.sp;
        bad = bad || big || close;
        sink.template put_n<3>(O_PHI, phi);
        sink.template put_n<9>(O_D, D);
    } else {
        sink.template put_n<3>(O_PHI, phi);
        build_D(R, D);
    }
    // ||A||_F^2 = tr(B^2) + 3 m^2 with tr(B^2) = (2/3) p
    const float fro2 = (float)__builtin_fma((2.0 / 3.0) * cu.sp, cu.sp, 3.0 * cu.m * cu.m);
    const float lim2 = prm.tau_res2_f * fro2;
    bool fails = check2_fails((float)cu.d1, (float)cu.d2, (float)cu.d3, A12, A13, A23, D, (float)cu.mu1,
                              (float)cu.mu2, lim2);
    if constexpr (!GRAD) {
        // second attempt for a diagonal matrix or a (nearly) double root,
        // checked alike.  D is stored after it (it is in registers for the
        // check anyway); the angles, already stored, are overwritten (same
        // lane, same addresses: the stores stay in order)
        const bool cand = fails && fin && !cu.triple;
        if (__ballot(cand)) {
            const bool diag = A12 == 0.0f && A13 == 0.0f && A23 == 0.0f;
            const bool near = dbl || split < prm.tau_res * cu.sp;
            if (cand && (diag || near)) {
                float v2, s2sq2, w2, cw2;
                const Rot<float> R2 = second_attempt_f32(cu, A12, A13, A22, A33, A23, plus, diag, v2, s2sq2, w2,
                                                         cw2);
                angles_of(R2, v2, s2sq2, w2, cw2, phi);
                build_D(R2, D);
                fails = check2_fails((float)cu.d1, (float)cu.d2, (float)cu.d3, A12, A13, A23, D,
                                     (float)cu.mu1, (float)cu.mu2, lim2);
                sink.reloaded().template put_n<3>(O_PHI, phi);
            }
        }
        sink.template put_n<9>(O_D, D);
    }
    refine = bad || fails;
    return flag;
}

// The float64 checked path, streaming its outputs through a sink like
// eig3_f32 (fewer live registers than gathering all eighteen first): the
// float64 cubic stage, the general branch with the squared cosines as float64
// quotients (u_quotients), and the float64 check.  As in eig3_f32, p = 0
// takes the general path's exact result (all deviations and gaps 0: D = I,
// angles 0, lam = m) and a non-finite input is queued for its NaN outputs.
// Sets refine and lc (the isolated eigenvalue handed to the refinement, a
// deviation in scaled units) and returns the flag.
template <bool GRAD, typename Sink>
__device__ __forceinline__ int eig3_f64s(const double ain[6], const Eig3Params &prm, const Sink &sink,
                                         bool &refine, double &lc) {
    // as in eig3_f32, a non-finite entry shows as a non-finite p (cu.fin)
    double amax = 0.0;
#pragma unroll
    for (int c = 0; c < 6; ++c) amax = fmax(amax, __builtin_fabs(ain[c]));
    const int ex = scale_exponent(amax);
    double a[6];
#pragma unroll
    for (int c = 0; c < 6; ++c) a[c] = sc2(ain[c], -ex);
    const Cubic cu = cubic_stage(a[0], a[1], a[2], a[3], a[4], a[5]);
    const bool fin = cu.fin;
    const double split = fmin(cu.g13, cu.g32);
    const bool dbl = (cu.g13 * cu.g32 == 0.0) || split < prm.tau_dbl * cu.sp;
    const int flag = !fin ? FLAG_NONFINITE : (cu.triple ? FLAG_TRIPLE : (dbl ? FLAG_DOUBLE : FLAG_GENERAL));
    sink.flag(flag);
    bool bad = !fin || (!cu.triple && dbl);
    if (prm.tau_gap > 0.0) {   // uniform: skipped at the default 0
        asm volatile("");      // (keeps the branch; see check_fails)
        const double l1 = __builtin_fabs(cu.m + cu.mu1), l2 = __builtin_fabs(cu.m + cu.mu2);
        bad = bad || (!cu.triple && split < prm.tau_gap * fmax(l1, l2));
    }
    lc = (cu.g13 >= cu.g32) ? cu.mu1 : cu.mu2;
    const URow u = u_quotients(cu.d1, cu.mu1, cu.mu2, cu.mu3, cu.g13, cu.g32, a[3], a[4]);
    const bool plus = !(product_key(a[3], a[4], a[1], a[2], a[5]) < 0.0);
    const Rot<double> R = select_angles<double>(a[3], a[4], a[1], a[2], a[5], cu.g12, cu.g13, cu.g32, u.v,
                                                u.s2sq, u.w, u.cw, plus);
    double phi[3];
    angles_of(R, phi);
    double D[9];
    bool big = false;
    if constexpr (GRAD) {   // differentiated calls: as in eig3_f32
        build_D(R, D);
        big = rotate_pairs64<double>(cu.d1, cu.d2, cu.d3, a[3], a[4], a[5], cu.mu1, cu.mu2, cu.mu3, cu.g12, cu.g13,
                                     cu.g32, R, prm.tau_vec, D, phi);
        sink.template put_n<3>(O_PHI, phi);
    } else {
        sink.template put_n<3>(O_PHI, phi);
        build_D(R, D);
    }
    sink.template put_n<9>(O_D, D);
    // ||A||_F^2 = tr(B^2) + 3 m^2 with tr(B^2) = (2/3) p
    const double fro2 = __builtin_fma((2.0 / 3.0) * cu.sp, cu.sp, 3.0 * cu.m * cu.m);
    double rq[3];
    const bool rbad = check_rq64(cu.d1, cu.d2, cu.d3, a[3], a[4], a[5], D, cu.mu1, cu.mu2, cu.mu3,
                                 prm.tau_res * prm.tau_res * fro2, rq);
    const bool cbad = big || rbad;
    // eigenvalues as Rayleigh quotients of the checked columns (their gaps
    // corrected alike); p = 0 keeps the exact lam = m.  A correction that
    // would break the slot order (two eigenvalues within the residual of each
    // other) sends the matrix to the refinement instead.
    const double m1 = cu.triple ? cu.mu1 : cu.mu1 + rq[0], m2 = cu.triple ? cu.mu2 : cu.mu2 + rq[1],
                 m3 = cu.triple ? cu.mu3 : cu.mu3 + rq[2];
    const double g12 = cu.g12 + (m1 - cu.mu1) - (m2 - cu.mu2), g13 = cu.g13 + (m1 - cu.mu1) - (m3 - cu.mu3),
                 g32 = cu.g32 + (m3 - cu.mu3) - (m2 - cu.mu2);
    {
        const double lam[3] = {sc2(cu.m + m1, ex), sc2(cu.m + m2, ex), sc2(cu.m + m3, ex)};
        const double gap[3] = {sc2(fmax(g12, 0.0), ex), sc2(fmax(g13, 0.0), ex), sc2(fmax(g32, 0.0), ex)};
        sink.template put_n<3>(O_LAM, lam);
        sink.template put_n<3>(O_GAP, gap);
    }
    bad = bad || (!cu.triple && (cbad || !(g13 >= 0.0 && g32 >= 0.0)));
    refine = bad;
    return flag;
}

// The refinement of one queued matrix (original entries ain, isolated
// eigenvalue lc as a deviation from the centre, in the scaled units eig3_one
// used; the centre is recomputed here with the same arithmetic).  A matrix
// queued with the p = 0 or the non-finite flag (float32 path) gets the
// special outputs instead: lam = the centre m, D = I, angles and gaps 0, or
// all NaN; the refinement's arithmetic is harmless for those inputs.
__device__ __forceinline__ bool is_special(int flag) { return flag == FLAG_TRIPLE || flag == FLAG_NONFINITE; }
template <typename T>
__device__ __forceinline__ void refine_one(const T ain[6], double lc, int flag, Out3<T> &o) {
    double amax = 0.0;
#pragma unroll
    for (int c = 0; c < 6; ++c) amax = fmax(amax, __builtin_fabs((double)ain[c]));
    const int ex = scale_exponent(amax);
    double m, d1, d2, d3;
    center3(sc2((double)ain[0], -ex), sc2((double)ain[1], -ex), sc2((double)ain[2], -ex), m, d1, d2, d3);
    const Refined rf = refine3(d1, d2, d3, sc2((double)ain[3], -ex), sc2((double)ain[4], -ex),
                               sc2((double)ain[5], -ex), lc);
#pragma unroll
    for (int i = 0; i < 9; ++i) o.v[O_D + i] = (T)rf.D[i];
    extract_angles<T>(o.v + O_D, o.v + O_PHI);
#pragma unroll
    for (int k = 0; k < 3; ++k) o.v[O_LAM + k] = (T)sc2(m + rf.lam[k], ex);
    o.v[O_GAP] = (T)sc2(fmax(rf.lam[0] - rf.lam[1], 0.0), ex);
    o.v[O_GAP + 1] = (T)sc2(fmax(rf.lam[0] - rf.lam[2], 0.0), ex);
    o.v[O_GAP + 2] = (T)sc2(fmax(rf.lam[2] - rf.lam[1], 0.0), ex);
    o.flag = flag | FLAG_FIXUP;
    if (is_special(flag)) {
        const bool fin = flag != FLAG_NONFINITE;
        const T nan = (T)__builtin_nan("");
        const T lam = fin ? (T)sc2(m, ex) : nan, one = fin ? T(1) : nan, zero = fin ? T(0) : nan;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            o.v[O_LAM + k] = lam;
            o.v[O_PHI + k] = zero;
            o.v[O_GAP + k] = zero;
        }
#pragma unroll
        for (int i = 0; i < 9; ++i) o.v[O_D + i] = (i % 4 == 0) ? one : zero;
        o.flag = flag;
    }
}

// ------------------------------------------------------ per-wave tiles -----
constexpr int WAVE = 64;

// The value x, opaque to the optimizer (no instruction is emitted).
__device__ __forceinline__ uint32_t fresh(uint32_t x) {
    asm volatile("" : "+v"(x));
    return x;
}
// The same for a wave-uniform value in a scalar register.
__device__ __forceinline__ int fresh_s(int x) {
    asm volatile("" : "+s"(x));
    return x;
}

// The lane index, recomputed where it is used (two mbcnt) rather than kept in
// a register across the tile loop: under the 96-register budget the compiler
// would otherwise spill it and reload it (with a full memory wait) per tile.
__device__ __forceinline__ int lane_id() {
    return (int)__builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, fresh(0u)));
}
__device__ __forceinline__ int wave_id() {
    return __builtin_amdgcn_readfirstlane((int)(threadIdx.x / WAVE));
}
__device__ __forceinline__ unsigned lane_rank(uint64_t mask) {
    return __builtin_amdgcn_mbcnt_hi((unsigned)(mask >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)mask, 0u));
}
// Orders this wave's LDS accesses around a hand-over between its lanes (the
// hardware executes one wave's LDS instructions in order; this keeps the
// compiler from moving them).
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// ---- raw buffer access -----------------------------------------------------
// A descriptor covers one plane: base address, size in bytes (0 for an absent
// plane), and the fourth word of gfx9-family raw buffers (32-bit data format,
// no swizzle, no stride).  Offsets are byte offsets.
using rsrc_t = __amdgpu_buffer_rsrc_t;
constexpr int kBufWord3 = 0x00020000;
typedef int v2i32 __attribute__((ext_vector_type(2)));
typedef int v4i32 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ rsrc_t plane_rsrc(const void *p, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, (int)(p ? bytes : 0u),
                                             kBufWord3);
}
// Cache policy of the plane loads and stores (the buffer instructions'
// cache-policy operand).  Planes are streams, each element read or written
// once, and the non-temporal policy (the NT bit) keeps them from displacing
// one another in the caches: a copy with the eig3 plane layout (6 planes in,
// 15 out) ran about 5 % faster with it.  Two exceptions, both measured:
//  - stores that the refinement queue overwrites soon after: the drain waits
//    for the wave's stores to complete, which takes longer for non-temporal
//    ones (the float64 checked path drains often; it streams its loads only);
//  - the mixed-batch kernel when its groups' planes start anywhere, so that
//    a cache line is often shared by the tiles of two waves: it then uses
//    the default (see k_mixed's STREAM variant for aligned planes).
constexpr int kCached = 0, kStream = 2;
template <int POL> __device__ __forceinline__ float bload(rsrc_t r, uint32_t off, float) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, (int)off, 0, POL));
}
template <int POL> __device__ __forceinline__ double bload(rsrc_t r, uint32_t off, double) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, (int)off, 0, POL));
}
template <int POL> __device__ __forceinline__ void bstore(rsrc_t r, uint32_t off, float v) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, (int)off, 0, POL);
}
template <int POL> __device__ __forceinline__ void bstore(rsrc_t r, uint32_t off, double v) {
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(v2i32, v), r, (int)off, 0, POL);
}
template <int POL> __device__ __forceinline__ void bstore(rsrc_t r, uint32_t off, uint8_t v) {
    __builtin_amdgcn_raw_buffer_store_b8(v, r, (int)off, 0, POL);
}
// Element `i` of plane p (T values) through a plane descriptor of n elements.
template <typename T, int POL> __device__ __forceinline__ T ld_plane(const T *p, uint32_t n, uint32_t i) {
    return bload<POL>(plane_rsrc(p, n * (uint32_t)sizeof(T)), i * (uint32_t)sizeof(T), T());
}
template <typename T, int POL> __device__ __forceinline__ void st_plane(T *p, uint32_t n, uint32_t i, T v) {
    bstore<POL>(plane_rsrc(p, n * (uint32_t)sizeof(T)), i * (uint32_t)sizeof(T), v);
}

// Per-lane global stores for the refinement's scattered results, whose plane
// pointers may differ from lane to lane (mixed batches).
template <typename T> using gptr = __attribute__((address_space(1))) T *;
template <typename T> __device__ __forceinline__ gptr<T> elem(T *p, uint32_t off) {
    return (gptr<T>)((gptr<char>)p + off * (uint32_t)sizeof(T));
}
// Read-only tables (mixed-batch descriptors and tile entries) in the constant
// address space: they do not change while a kernel runs, so uniform reads
// become scalar loads even though the kernel stores to global memory.
template <typename T> using cptr = const __attribute__((address_space(4))) T *;
template <typename T> __device__ __forceinline__ cptr<T> as_const(const T *p) { return (cptr<T>)p; }

// A plane pointer stored in the kernel-argument segment at byte offset off.
// Read this way, with a plane index offset by a salt (0 at run time, unknown
// to the compiler) where the plane is used, the pointers and the descriptors
// built from them are fetched per tile instead of being hoisted out of the
// tile loop, where dozens of them would exhaust the scalar registers.
template <typename T> __device__ __forceinline__ T *karg_ptr(uint32_t off) {
    typedef __attribute__((address_space(4))) const char *kptr;
    kptr ka = (kptr)__builtin_amdgcn_kernarg_segment_ptr();
    return *(T *const __attribute__((address_space(4))) *)(ka + off);
}

// N consecutive plane pointers, read with one wide scalar load (one wait
// instead of one per pointer).
template <typename T, int N> struct PtrN {
    T *p[N];
};
template <typename T, int N> __device__ __forceinline__ PtrN<T, N> ptrs_at(T *const __attribute__((address_space(4))) *q) {
    PtrN<T, N> r;
#pragma unroll
    for (int i = 0; i < N; ++i) r.p[i] = q[i];
    return r;
}
template <typename T, int N> __device__ __forceinline__ PtrN<T, N> karg_ptrs(uint32_t off) {
    typedef __attribute__((address_space(4))) const char *kptr;
    kptr ka = (kptr)__builtin_amdgcn_kernarg_segment_ptr();
    return ptrs_at<T, N>((T *const __attribute__((address_space(4))) *)(ka + off));
}

// Output plane pointers of a launch in the kernel-argument segment.
// n: matrices in this launch.
template <typename T> struct KernargPlanes {
    uint32_t out_off, flags_off, n;   // byte offsets inside the argument segment
    __device__ __forceinline__ T *out(int k) const { return karg_ptr<T>(out_off + 8 * k); }
    template <int N> __device__ __forceinline__ PtrN<T, N> outs(int k) const {
        return karg_ptrs<T, N>(out_off + 8 * k);
    }
    __device__ __forceinline__ uint8_t *flags(int salt = 0) const { return karg_ptr<uint8_t>(flags_off + 8 * salt); }
};

// Output plane pointers of a group descriptor in device memory.
template <typename T> struct TablePlanes {
    cptr<Eig3Ptrs<T>> p;
    uint32_t n;
    __device__ __forceinline__ T *out(int k) const { return p->out[k]; }
    template <int N> __device__ __forceinline__ PtrN<T, N> outs(int k) const {
        return ptrs_at<T, N>(&p->out[k]);
    }
    __device__ __forceinline__ uint8_t *flags(int salt = 0) const { return (&p->flags)[salt]; }
};

// Store one matrix's outputs (float64 paths).  The plane index is offset by
// salt, which is 0 at run time but not known to the compiler, so the pointer
// loads stay here instead of being hoisted out of the tile loop (where they
// would pin 38 scalar registers for the whole kernel).
template <typename T, int SP, typename Planes>
__device__ __forceinline__ void put3(const Planes &pl, int salt, uint32_t off, const Out3<T> &o) {
#pragma unroll
    for (int k = 0; k < NOUT3; ++k) st_plane<T, SP>(pl.out(k + salt), pl.n, off, o.v[k]);
    st_plane<uint8_t, SP>(pl.flags(salt), pl.n, off, (uint8_t)o.flag);
}

// Stores of one lane's matrix as its outputs are produced (float32 path).
// Lanes past n and absent planes are dropped by the descriptors.  In float32
// an absent plane also skips its store instruction (a branch on the plane
// pointer, uniform over the launch or the mixed batch's group): the
// instruction would still occupy the wave's memory issue, which cost about
// 1 % with the gaps and flags absent and 4 % with D absent too.  The float64
// kernels keep every store (the branches raised their register use from
// about 160 to 180 VGPRs, one wave less per SIMD).
template <typename T, int SP, typename Planes> struct LaneSink {
    const Planes &pl;
    int salt;
    uint32_t off;
    __device__ __forceinline__ void put(int k, T v) const { st_plane<T, SP>(pl.out(k + salt), pl.n, off, v); }
    // planes k0 .. k0 + N - 1
    template <int N> __device__ __forceinline__ void put_n(int k0, const T *v) const {
        const PtrN<T, N> q = pl.template outs<N>(k0 + salt);
#pragma unroll
        for (int i = 0; i < N; ++i)
            if (sizeof(T) == 8 || q.p[i]) st_plane<T, SP>(q.p[i], pl.n, off, v[i]);
    }
    __device__ __forceinline__ void flag(int f) const {
        uint8_t *p = pl.flags(salt);
        if (sizeof(T) == 8 || p) st_plane<uint8_t, SP>(p, pl.n, off, (uint8_t)f);
    }
    // The same sink with plane pointers that are read again where it is
    // used (a rare branch then loads its own descriptors instead of keeping
    // the main path's in scalar registers throughout).
    __device__ __forceinline__ LaneSink reloaded() const { return LaneSink{pl, fresh_s(salt), off}; }
};

// A refined result: scattered per-lane stores (the rare path).
template <typename T, typename Planes>
__device__ __forceinline__ void write_out3(const Planes &pl, int salt, uint32_t off, const Out3<T> &o) {
#pragma unroll
    for (int k = 0; k < NOUT3; ++k) {
        T *dst = pl.out(k + salt);
        if (dst) *elem(dst, fresh(off)) = o.v[k];
    }
    uint8_t *fl = pl.flags(salt);
    if (fl) *elem(fl, fresh(off)) = (uint8_t)o.flag;
}

// One wave's refinement queue: CAP = 64 * (MPL + 1) entries, enough for a
// queue one entry short of a drain plus a whole tile.
template <typename T, int CAP> struct WaveQueue {
    uint32_t off[CAP];   // matrix offset within its launch chunk / group
    int32_t grp[CAP];    // group (mixed batches; 0 otherwise) | flag << 24
    double lc[CAP];
    T a[6][CAP];
};

template <typename T, int MPL, bool QUEUE, bool AOS> struct WaveSmem {
    WaveQueue<T, QUEUE ? WAVE * (MPL + 1) : 1> q;
    __align__(16) T rec[AOS ? WAVE * MPL * 6 : 4];
};

// The inputs of one wave tile held in registers.  SoA: each lane's MPL
// matrices.  AoS: the lane's share of the tile's contiguous records as 16-byte
// vectors, transposed through LDS when the tile is processed.
template <typename T, int MPL, bool AOS> struct WIn {
    static constexpr int VEC = 16 / sizeof(T);
    static constexpr int NV = WAVE * MPL * 6 / VEC;   // 16-byte vectors per tile
    static constexpr int NVL = (NV + WAVE - 1) / WAVE;
    T a[AOS ? 1 : MPL][6];
    T v[AOS ? NVL : 1][AOS ? VEC : 1];
};

// Lanes past n read zeros (the descriptor's bound).  AoS: a 16-byte vector
// that straddles the end of the records is read element by element.
// Input planes (SoA: six pointers; AoS: the record pointer), read where a
// tile is loaded.  Kernel arguments: through the argument segment with a salt;
// mixed batches: from the group descriptor.
template <typename T> struct KernargInputs {
    uint32_t in_off, aos_off;
    int salt;
    __device__ __forceinline__ const T *in(int c) const { return karg_ptr<const T>(in_off + 8 * (c + salt)); }
    __device__ __forceinline__ PtrN<const T, 6> ins() const { return karg_ptrs<const T, 6>(in_off + 8 * salt); }
    __device__ __forceinline__ const T *aos() const { return karg_ptr<const T>(aos_off + 8 * salt); }
};

template <typename T, int MPL, bool AOS, int LP, typename Inputs>
__device__ __forceinline__ void load_wtile3(WIn<T, MPL, AOS> &in, const Inputs &src, uint32_t n,
                                            uint32_t base) {
    const int lane = lane_id();
    if constexpr (AOS) {
        using W = WIn<T, MPL, AOS>;
        constexpr int VEC = W::VEC;
        const uint32_t lim = n * 6;   // elements in the launch
        const rsrc_t r = plane_rsrc(src.aos(), lim * (uint32_t)sizeof(T));
#pragma unroll
        for (int u = 0; u < W::NVL; ++u) {
            const uint32_t j = u * WAVE + lane;
            const uint32_t e0 = base * 6 + j * VEC;
            if (j < (uint32_t)W::NV) {
                if (e0 + VEC <= lim) {
                    const v4i32 x = __builtin_amdgcn_raw_buffer_load_b128(r, (int)(e0 * sizeof(T)), 0, LP);
                    typedef T vec_t __attribute__((ext_vector_type(VEC)));
                    const vec_t y = __builtin_bit_cast(vec_t, x);
#pragma unroll
                    for (int t = 0; t < VEC; ++t) in.v[u][t] = y[t];
                } else {
#pragma unroll
                    for (int t = 0; t < VEC; ++t) in.v[u][t] = bload<LP>(r, (e0 + t) * (uint32_t)sizeof(T), T());
                }
            }
        }
    } else {
        const PtrN<const T, 6> ptrs = src.ins();
#pragma unroll
        for (int k = 0; k < MPL; ++k) {
            const uint32_t off = base + k * WAVE + lane;
#pragma unroll
            for (int c = 0; c < 6; ++c) in.a[k][c] = ld_plane<T, LP>(ptrs.p[c], n, off);
        }
    }
}

// Finish the first `cnt` (<= 64) queue entries, entry j on lane j, and
// overwrite their provisional outputs.  The wave's own provisional stores are
// waited for first, so a final value always lands last.  Returns the number
// of refined (not special) entries.
template <typename T, int CAP, typename PlanesOf>
__device__ __forceinline__ unsigned drain_wave(WaveQueue<T, CAP> *q, int cnt, const PlanesOf &planes_of,
                                               int salt) {
    __builtin_amdgcn_s_waitcnt(0x0f70);   // vmcnt(0): earlier stores of this wave have completed
    const int lane = lane_id();
    const int g = lane < cnt ? q->grp[lane] : 0;
    const bool ref = lane < cnt && !is_special(g >> 24);
    if (lane < cnt) {
        T a[6];
#pragma unroll
        for (int c = 0; c < 6; ++c) a[c] = q->a[c][lane];
        Out3<T> o;
        refine_one<T>(a, q->lc[lane], g >> 24, o);
        write_out3(planes_of(g & 0xffffff), salt, q->off[lane], o);
    }
    return (unsigned)__popcll(__ballot(ref));
}

// Process one wave tile of 64*MPL 3x3 matrices starting at `base` from inputs
// already in registers: compute, store, queue the matrices that need the
// refinement, and drain the queue.  Wave-uniform control flow.
template <typename T, int PATH, int MPL, bool AOS, int SP, bool GRAD, typename Planes, typename PlanesOf>
__device__ __forceinline__ void wtile_eig3(const Planes &pl, const PlanesOf &planes_of, int grp,
                                           const Eig3Params &prm, const WIn<T, MPL, AOS> &in,
                                           uint32_t n, uint32_t base,
                                           WaveSmem<T, MPL, PATH != PATH_FP64_PLAIN, AOS> *sm,
                                           int &qn, int &qage, unsigned &refined, unsigned &nonfinite) {
    constexpr bool QUEUE = PATH != PATH_FP64_PLAIN;
    const int lane = lane_id();
    if constexpr (AOS) {
        using W = WIn<T, MPL, AOS>;
#pragma unroll
        for (int u = 0; u < W::NVL; ++u) {
            const int j = u * WAVE + lane;
            if (j < W::NV) {
#pragma unroll
                for (int t = 0; t < W::VEC; ++t) sm->rec[j * W::VEC + t] = in.v[u][t];
            }
        }
        wave_sync();
    }
#pragma unroll
    for (int k = 0; k < MPL; ++k) {
        const int slot = k * WAVE + lane;
        const uint32_t off = base + slot;
        const bool valid = off < n;
        T A[6];
        if constexpr (AOS) {
#pragma unroll
            for (int c = 0; c < 6; ++c) A[c] = sm->rec[slot * 6 + c];
        } else {
#pragma unroll
            for (int c = 0; c < 6; ++c) A[c] = in.a[k][c];
        }
        const int salt = (int)((base + k) * (uint32_t)prm.zero);
        int flag;
        bool refine;
        double lc;
        if constexpr (PATH == PATH_FP32_FIXUP) {
            flag = eig3_f32<GRAD>(A, prm, LaneSink<T, SP, Planes>{pl, salt, off}, refine, lc);
        } else if constexpr (PATH == PATH_FP64_FIXUP) {
            flag = eig3_f64s<GRAD>(A, prm, LaneSink<T, SP, Planes>{pl, salt, off}, refine, lc);
        } else {
            Out3<T> o;
            eig3_one<T>(A, prm, o);
            put3<T, SP>(pl, salt, off, o);
            flag = o.flag;
            refine = o.refine;
            lc = o.lc;
        }
        nonfinite += (unsigned)__popcll(__ballot(valid && flag == FLAG_NONFINITE));
        if constexpr (QUEUE) {
            const bool r = valid && refine;
            const uint64_t mask = __ballot(r);
            if (mask) {
                if (r) {
                    const int pos = qn + (int)lane_rank(mask);
                    sm->q.off[pos] = off;
                    sm->q.grp[pos] = grp | (flag << 24);
                    sm->q.lc[pos] = lc;
#pragma unroll
                    for (int c = 0; c < 6; ++c) sm->q.a[c][pos] = A[c];
                }
                qn += (int)__popcll(mask);
            }
        }
    }
    if constexpr (AOS) wave_sync();
    if constexpr (QUEUE) {
        // drain rounds of up to 64: when a full round waits, or when the
        // oldest entry has waited drain_tiles tiles (its tile's output lines
        // are then still likely to be in cache when they are overwritten)
        qage = qn > 0 ? qage + 1 : 0;
        while (qn >= WAVE || (qn > 0 && prm.drain_tiles > 0 && qage >= prm.drain_tiles)) {
            const int cnt = qn < WAVE ? qn : WAVE;
            wave_sync();
            refined += drain_wave<T>(&sm->q, cnt, planes_of, (int)(base * (uint32_t)prm.zero));
            const int rest = qn - cnt;
            // move entries [cnt, qn) to the front; a lane reads only entries
            // no lane writes in the same round
            for (int j = lane; j < rest; j += WAVE) {
                const int s = j + cnt;
                const uint32_t o_ = sm->q.off[s];
                const int32_t g_ = sm->q.grp[s];
                const double l_ = sm->q.lc[s];
                T a_[6];
#pragma unroll
                for (int c = 0; c < 6; ++c) a_[c] = sm->q.a[c][s];
                sm->q.off[j] = o_;
                sm->q.grp[j] = g_;
                sm->q.lc[j] = l_;
#pragma unroll
                for (int c = 0; c < 6; ++c) sm->q.a[c][j] = a_[c];
            }
            qn = rest;
            qage = rest > 0 ? 1 : 0;
            wave_sync();
        }
    }
}

// Refine what is left in the queues of all NW waves of the workgroup once
// they have finished their tiles: the leftovers are pooled (entry e of the
// concatenated queues goes to lane e % 64 of wave (e / 64) % NW), so a
// workgroup pays for one partly filled refinement round instead of one per
// wave.  The float64 checked path, which refines a few percent of the
// precision recipe, drains this way (one wave at a time it ran 6 % slower,
// with four times the refinement rounds); the float32 kernels, which refine
// far fewer matrices, let each wave refine its own leftovers with no
// barrier.  A wave with queued entries first waits for its own stores, because
// a refined result may now overwrite a provisional one that this wave wrote
// and another wave refines; a wave with an empty queue (most of them) has no
// store that anything overwrites and goes straight to the barrier.
template <typename T, int MPL, bool AOS, int NW, typename PlanesOf>
__device__ __forceinline__ void final_drain(const PlanesOf &planes_of, WaveSmem<T, MPL, true, AOS> *sm,
                                            int *qcount, int qn, int w, unsigned &refined) {
    const int lane = lane_id();
    if (qn > 0) __builtin_amdgcn_s_waitcnt(0x0f70);   // vmcnt(0): this wave's stores have completed
    if (lane == 0) qcount[w] = qn;
    __syncthreads();
    int pre[NW + 1];
    pre[0] = 0;
#pragma unroll
    for (int v = 0; v < NW; ++v) pre[v + 1] = pre[v] + qcount[v];
    const int total = pre[NW];
    for (int r = w; r * WAVE < total; r += NW) {
        const int e = r * WAVE + lane;
        bool ref = false;
        if (e < total) {
            int src = 0;
#pragma unroll
            for (int v = 1; v < NW; ++v) src += (e >= pre[v]) ? 1 : 0;
            const int i = e - pre[src];
            const WaveQueue<T, WAVE *(MPL + 1)> *q = &sm[src].q;
            T a[6];
#pragma unroll
            for (int c = 0; c < 6; ++c) a[c] = q->a[c][i];
            const int g = q->grp[i];
            ref = !is_special(g >> 24);
            Out3<T> o;
            refine_one<T>(a, q->lc[i], g >> 24, o);
            write_out3(planes_of(g & 0xffffff), 0, q->off[i], o);
        }
        refined += (unsigned)__popcll(__ballot(ref));
    }
}

__device__ __forceinline__ void add_counters(unsigned *counters, unsigned refined, unsigned nonfinite) {
    if (counters && lane_id() == 0) {
        if (refined) atomicAdd(&counters[0], refined);
        if (nonfinite) atomicAdd(&counters[1], nonfinite);
    }
}

// float32: an occupancy target makes the compiler fit the kernel into the
// registers of 6 waves per SIMD (80 VGPRs) with one matrix per lane and of
// 5 waves (96) with two (one wave less for the differentiated variant); two
// matrices per lane at 6 waves would spill, and their queue's LDS allows 5
// waves per SIMD anyway.  The plain float64 path runs faster at 4 waves
// (128 VGPRs, a few spills) than at 3; the checked one does not.  The
// target never exceeds what the workgroup's LDS allows (160 KB per CU).
template <typename T, int PATH, int BS, int MPL, bool AOS, bool GRAD>
constexpr int eig3_waves_target() {
    constexpr int NW = BS / WAVE;
    // (the differentiated float32 variant, with its float64 pair correction,
    // gets one wave less: at the plain variant's budget it would spill)
    constexpr int want = sizeof(T) == 4 ? (MPL == 1 ? 6 - GRAD : MPL == 2 ? 5 - GRAD : 1)
                                        : (PATH == PATH_FP64_PLAIN && MPL == 1 ? 4 : 1);
    constexpr size_t lds = NW * (sizeof(WaveSmem<T, MPL, PATH != PATH_FP64_PLAIN, AOS>) + sizeof(int));
    constexpr int by_lds = (int)(163840 / lds) * NW / 4;
    return want < by_lds ? want : (by_lds > 1 ? by_lds : 1);
}
template <typename T, int PATH, int BS, int MPL, bool AOS, bool GRAD = false>
__global__ __launch_bounds__(BS)
__attribute__((amdgpu_waves_per_eu(eig3_waves_target<T, PATH, BS, MPL, AOS, GRAD>())))
void k_eig3(Eig3Args<T> args) {
    constexpr int NW = BS / WAVE;
    constexpr int WT = WAVE * MPL;
    constexpr bool QUEUE = PATH != PATH_FP64_PLAIN;
    __shared__ WaveSmem<T, MPL, QUEUE, AOS> sm[NW];
    __shared__ int qcount[NW];   // the float64 pooled drain only
    // the wave index, in a scalar register
    const int wid = wave_id();
    WaveSmem<T, MPL, QUEUE, AOS> *my = &sm[wid];
    const uint32_t n = (uint32_t)args.prm.n;
    const uint32_t ntiles = (n + WT - 1) / WT;
    KernargPlanes<T> pl;
    pl.out_off = (uint32_t)(offsetof(Eig3Args<T>, p) + offsetof(Eig3Ptrs<T>, out));
    pl.flags_off = (uint32_t)(offsetof(Eig3Args<T>, p) + offsetof(Eig3Ptrs<T>, flags));
    pl.n = n;
    auto planes_of = [&](int) { return pl; };
    unsigned refined = 0, nonfinite = 0;
    int qn = 0, qage = 0;
    WIn<T, MPL, AOS> cur, nxt;
    const uint32_t stride = gridDim.x * NW;
    uint32_t t = blockIdx.x * NW + wid;
    auto inputs = [&](uint32_t tt) {
        return KernargInputs<T>{(uint32_t)(offsetof(Eig3Args<T>, p) + offsetof(Eig3Ptrs<T>, in)),
                                (uint32_t)offsetof(Eig3Args<T>, aos), (int)(tt * (uint32_t)args.prm.zero)};
    };
    // Software pipeline: the next tile's inputs are loaded while this one is
    // computed.  The first tile is peeled off: inside the loop every input
    // register is then a copy made at the end of the previous tile, so the
    // memory waits the compiler places do not depend on the path into the
    // loop (merged with the entry path they would wait for the prefetch and
    // for the previous tile's stores at every tile).
    // cache policies: see kStream
    constexpr int LP = kStream, SP = PATH == PATH_FP64_FIXUP ? kCached : kStream;
    auto step = [&]() {
        const uint32_t tn = t + stride;
        if (tn < ntiles) load_wtile3<T, MPL, AOS, LP>(nxt, inputs(tn), n, tn * WT);
        wtile_eig3<T, PATH, MPL, AOS, SP, GRAD>(pl, planes_of, 0, args.prm, cur, n, t * WT, my, qn, qage, refined,
                                          nonfinite);
        cur = nxt;
    };
    if (t < ntiles) {
        load_wtile3<T, MPL, AOS, LP>(cur, inputs(t), n, t * WT);
        step();
        for (t += stride; t < ntiles; t += stride) step();
    }
    // what is left (fewer than 64: the tiles drain full rounds): float32 is
    // refined by the wave itself, with no barrier (refinement is rare there,
    // and a workgroup barrier and a pooled round cost more than the
    // occasional partly filled round of one wave); float64 is pooled
    if constexpr (QUEUE) {
        if constexpr (sizeof(T) == 8) {
            final_drain<T, MPL, AOS, NW>(planes_of, sm, qcount, qn, wid, refined);
        } else {
            (void)qcount;
            if (qn > 0) {
                wave_sync();
                refined += drain_wave<T>(&my->q, qn, planes_of, 0);
            }
        }
    }
    add_counters(args.prm.counters, refined, nonfinite);
}

// ------------------------------------------------------ eigenvalues only ---
// Reduced-output mode (float32): with no D and no angle planes requested the
// float64 cubic stage of §4 alone gives the eigenvalues, the gaps and the
// flag, as accurate as the full path's (its refinement exists for the
// eigenvectors), so the angle solve, the check and the refinement queue are
// skipped.  The arithmetic and the stores are those of eig3_f32, so lam, gap
// and flags are bitwise the full kernel's for every matrix it does not
// refine; the FIXUP bit is never set.  A non-finite input gets NaN outputs.
template <typename Sink>
__device__ __forceinline__ int eig3_lam_f32(const float ain[6], const Eig3Params &prm, const Sink &sink) {
    float amax = __builtin_fmaxf(__builtin_fmaxf(__builtin_fabsf(ain[0]), __builtin_fabsf(ain[1])),
                                 __builtin_fabsf(ain[2]));
    amax = __builtin_fmaxf(amax, __builtin_fmaxf(__builtin_fmaxf(__builtin_fabsf(ain[3]),
                                                                 __builtin_fabsf(ain[4])),
                                                 __builtin_fabsf(ain[5])));
    const int ex = scale_exponent_f(amax);
    double a[6];
#pragma unroll
    for (int c = 0; c < 6; ++c) a[c] = sc2((double)ain[c], -ex);
    const Cubic cu = cubic_stage_gaps(a[0], a[1], a[2], a[3], a[4], a[5]);
    const bool fin = cu.fin;
    const double split = cu.g13 < cu.g32 ? cu.g13 : cu.g32;
    const bool dbl = (cu.g13 * cu.g32 == 0.0) || split < prm.tau_dbl * cu.sp;
    const bool special = cu.triple || !fin;
    const int flag = special ? (fin ? FLAG_TRIPLE : FLAG_NONFINITE) : (dbl ? FLAG_DOUBLE : FLAG_GENERAL);
    sink.flag(flag);
    const float nan = __builtin_nanf("");
    const float lam[3] = {fin ? (float)sc2(cu.m + cu.mu1, ex) : nan, fin ? (float)sc2(cu.m + cu.mu2, ex) : nan,
                          fin ? (float)sc2(cu.m + cu.mu3, ex) : nan};
    const float gap[3] = {fin ? (float)sc2(cu.g12, ex) : nan, fin ? (float)sc2(cu.g13, ex) : nan,
                          fin ? (float)sc2(cu.g32, ex) : nan};
    sink.template put_n<3>(O_LAM, lam);
    sink.template put_n<3>(O_GAP, gap);
    return flag;
}

// Wave tiles of 64*MPL matrices, grid-stride, straight from and to HBM (no
// queue and no LDS).
template <int BS, int MPL>
__global__ __launch_bounds__(BS) void k_eig3_lam(Eig3Args<float> args) {
    constexpr int NW = BS / WAVE;
    constexpr int WT = WAVE * MPL;
    const uint32_t n = (uint32_t)args.prm.n;
    const uint32_t ntiles = (n + WT - 1) / WT;
    KernargPlanes<float> pl;
    pl.out_off = (uint32_t)(offsetof(Eig3Args<float>, p) + offsetof(Eig3Ptrs<float>, out));
    pl.flags_off = (uint32_t)(offsetof(Eig3Args<float>, p) + offsetof(Eig3Ptrs<float>, flags));
    pl.n = n;
    const int lane = lane_id();
    unsigned nonfinite = 0;
    for (uint32_t t = blockIdx.x * NW + wave_id(); t < ntiles; t += gridDim.x * NW) {
        const int salt = (int)(t * (uint32_t)args.prm.zero);
        WIn<float, MPL, false> in;
        load_wtile3<float, MPL, false, kStream>(
            in, KernargInputs<float>{(uint32_t)(offsetof(Eig3Args<float>, p) + offsetof(Eig3Ptrs<float>, in)),
                                     (uint32_t)offsetof(Eig3Args<float>, aos), salt},
            n, t * WT);
#pragma unroll
        for (int k = 0; k < MPL; ++k) {
            const uint32_t off = t * WT + k * WAVE + lane;
            const int flag = eig3_lam_f32(in.a[k], args.prm, LaneSink<float, kStream, KernargPlanes<float>>{pl, salt, off});
            nonfinite += (unsigned)__popcll(__ballot(off < n && flag == FLAG_NONFINITE));
        }
    }
    add_counters(args.prm.counters, 0, nonfinite);
}

// ------------------------------------------------------------- 2x2 ---------
template <typename T> struct Eig2Ptrs {
    const T *in[3];
    T *lam[2];
    T *D[4];
    T *phi;
    uint8_t *flags;
};

// One 2x2 matrix (§3) and its stores; out = lam1, lam2, D11, D12, D21, D22,
// phi (absent planes and lanes past n are dropped by the descriptors).
template <typename T, int SP>
__device__ __forceinline__ void eig2_lane(T a11, T a22, T a12, T *const out[7], uint8_t *flags,
                                          uint32_t n, uint32_t off) {
    const bool fin = finite(a11) && finite(a22) && finite(a12);
    // exact power-of-two scaling keeps d^2 + 4 A12^2 in range
    const double amax = fmax(fmax(__builtin_fabs((double)a11), __builtin_fabs((double)a22)),
                             __builtin_fabs((double)a12));
    const int ex = fin ? scale_exponent(amax) : 0;
    Eig2<T> e = eig2_one<T>(sc2(a11, -ex), sc2(a22, -ex), sc2(a12, -ex));
    e.l1 = sc2(e.l1, ex);
    e.l2 = sc2(e.l2, ex);
    if (!fin) {
        const T nan = T(__builtin_nan(""));
        e.l1 = e.l2 = e.c = e.s = e.phi = nan;
    }
    const T v[7] = {e.l1, e.l2, e.c, -e.s, e.s, e.c, e.phi};
#pragma unroll
    for (int k = 0; k < 7; ++k) st_plane<T, SP>(out[k], n, off, v[k]);
    st_plane<uint8_t, SP>(flags, n, off, fin ? (uint8_t)0 : (uint8_t)FLAG_NONFINITE);
}

// One wave tile of 64*MPL 2x2 matrices, straight from and to HBM.
template <typename T, int MPL>
__device__ __forceinline__ void wtile_eig2(const Eig2Ptrs<T> &p, uint32_t n, uint32_t base) {
    const int lane = lane_id();
    T A[MPL][3];
#pragma unroll
    for (int k = 0; k < MPL; ++k) {
        const uint32_t off = base + k * WAVE + lane;
#pragma unroll
        for (int c = 0; c < 3; ++c) A[k][c] = ld_plane<T, kStream>(p.in[c], n, off);
    }
    T *const out[7] = {p.lam[0], p.lam[1], p.D[0], p.D[1], p.D[2], p.D[3], p.phi};
#pragma unroll
    for (int k = 0; k < MPL; ++k)
        eig2_lane<T, kStream>(A[k][0], A[k][1], A[k][2], out, p.flags, n, base + k * WAVE + lane);
}

template <typename T, int BS, int MPL>
__global__ __launch_bounds__(BS) void k_eig2(Eig2Ptrs<T> p, uint32_t n) {
    constexpr int NW = BS / WAVE, WT = WAVE * MPL;
    const uint32_t ntiles = (n + WT - 1) / WT;
    const uint32_t stride = gridDim.x * NW;
    for (uint32_t t = blockIdx.x * NW + wave_id(); t < ntiles; t += stride) wtile_eig2<T, MPL>(p, n, t * WT);
}

// -------------------------------------------------------- adjoint ----------
// sine and cosine in the element type
__device__ __forceinline__ void sincos_t(float x, float &s, float &c) { sincosf(x, &s, &c); }
__device__ __forceinline__ void sincos_t(double x, double &s, double &c) { sincos(x, &s, &c); }

template <typename T> struct BwdPtrs {
    const T *lam[3];
    const T *D[9];
    const T *gap[3];
    const T *glam[3];
    const T *gD[9];
    T *gA[6];
    const T *phi[3];    // the Euler angles and their cotangent (both or none)
    const T *gphi[3];
};

template <typename T> struct BwdArgs {
    BwdPtrs<T> p;
    uint32_t n;
    int32_t zero;     // always 0; see karg_ptr
    double eps_rel;
};

// One lane's adjoint.  Absent cotangents read as zeros; lanes past n read
// zeros and store nothing (the descriptors' bounds).  Plane pointers come
// from the argument segment in groups, one wide scalar load each (salt: see
// karg_ptr), so all 27 plane loads can be issued back to back.
template <typename T>
__device__ __forceinline__ void bwd_lane(bool has_gap, bool has_ang, uint32_t i, uint32_t n, double eps_rel,
                                         int salt) {
    constexpr uint32_t P = (uint32_t)offsetof(BwdArgs<T>, p);
    const PtrN<const T, 12> pin = karg_ptrs<const T, 12>(P + offsetof(BwdPtrs<T>, lam) + 8 * salt);   // lam, D
    const PtrN<const T, 12> pco = karg_ptrs<const T, 12>(P + offsetof(BwdPtrs<T>, glam) + 8 * salt);  // glam, gD
    T L[3], D[9], gl[3], gD[9], gA[6];
#pragma unroll
    for (int c = 0; c < 3; ++c) L[c] = ld_plane<T, kStream>(pin.p[c], n, i);
#pragma unroll
    for (int c = 0; c < 9; ++c) D[c] = ld_plane<T, kStream>(pin.p[3 + c], n, i);
#pragma unroll
    for (int c = 0; c < 3; ++c) gl[c] = ld_plane<T, kStream>(pco.p[c], n, i);
#pragma unroll
    for (int c = 0; c < 9; ++c) gD[c] = ld_plane<T, kStream>(pco.p[3 + c], n, i);
    // the arithmetic is float64 for either storage type: the symmetric part
    // F_jk (E_jk - E_kj) can cancel, and a small gap then magnifies float32
    // rounding of E into the gradient
    double g12, g13, g32;
    if (has_gap) {
        const PtrN<const T, 3> pg = karg_ptrs<const T, 3>(P + offsetof(BwdPtrs<T>, gap) + 8 * salt);
        g12 = (double)ld_plane<T, kStream>(pg.p[0], n, i);
        g13 = (double)ld_plane<T, kStream>(pg.p[1], n, i);
        g32 = (double)ld_plane<T, kStream>(pg.p[2], n, i);
    } else {
        // differences of the stored eigenvalues (exact in float64 for float32)
        g12 = (double)L[0] - (double)L[1];
        g13 = (double)L[0] - (double)L[2];
        g32 = (double)L[2] - (double)L[1];
    }
    double Dd[9], gld[3], gDd[9], gAd[6];
#pragma unroll
    for (int c = 0; c < 9; ++c) Dd[c] = (double)D[c];
#pragma unroll
    for (int c = 0; c < 9; ++c) gDd[c] = (double)gD[c];
#pragma unroll
    for (int c = 0; c < 3; ++c) gld[c] = (double)gl[c];
    const double l0 = L[0], l1 = L[1], l2 = L[2];
    const double eps = eps_rel * sqrt_any64(l0 * l0 + l1 * l1 + l2 * l2);
    double wb[3] = {0.0, 0.0, 0.0};
    if (has_ang) {   // uniform
        const PtrN<const T, 6> pa = karg_ptrs<const T, 6>(P + offsetof(BwdPtrs<T>, phi) + 8 * salt);
        const double f2 = ld_plane<T, kStream>(pa.p[1], n, i), f3 = ld_plane<T, kStream>(pa.p[2], n, i);
        const double gphi[3] = {ld_plane<T, kStream>(pa.p[3], n, i), ld_plane<T, kStream>(pa.p[4], n, i),
                                ld_plane<T, kStream>(pa.p[5], n, i)};
        double s2, c2, s3, c3;
        sincos_t(f2, s2, c2);
        sincos_t(f3, s3, c3);
        angle_body_cotangent<double>(c2, s2, c3, s3, gphi, eps_rel * eps_rel, wb);
    }
    adjoint3<double>(Dd, gld, gDd, g12, g13, g32, eps * eps, wb, gAd);
#pragma unroll
    for (int c = 0; c < 6; ++c) gA[c] = (T)gAd[c];
    const PtrN<T, 6> po = karg_ptrs<T, 6>(P + offsetof(BwdPtrs<T>, gA) + 8 * salt);
#pragma unroll
    for (int c = 0; c < 6; ++c) st_plane<T, kStream>(po.p[c], n, i, gA[c]);
}

template <typename T, int BS, int MPL>
__global__ __launch_bounds__(BS) void k_eig3_bwd(BwdArgs<T> a) {
    constexpr int TILE = BS * MPL;
    const uint32_t n = a.n;
    const uint32_t ntiles = (n + TILE - 1) / TILE;
    const bool has_gap = a.p.gap[0] && a.p.gap[1] && a.p.gap[2];
    const bool has_ang = a.p.phi[0] && a.p.phi[1] && a.p.phi[2] && a.p.gphi[0] && a.p.gphi[1] && a.p.gphi[2];
    for (uint32_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const int salt = (int)(t * (uint32_t)a.zero);
#pragma unroll
        for (int k = 0; k < MPL; ++k)
            bwd_lane<T>(has_gap, has_ang, t * TILE + k * BS + threadIdx.x, n, a.eps_rel, salt);
    }
}

// ---------------------------------------------------- 2x2 adjoint ----------
template <typename T> struct Bwd2Ptrs {
    const T *lam[2];
    const T *D[4];
    const T *glam[2];   // absent cotangents: null planes, read as zeros
    const T *gD[4];
    const T *gphi;
    T *gA[3];
};

template <typename T> struct Bwd2Args {
    Bwd2Ptrs<T> p;
    uint32_t n;
    int32_t pad;
    double eps_rel;
};

// One matrix per lane, grid-stride; the planes are streams.  eps = eps_rel *
// ||lam||; the arithmetic is float64 (the gap lam2 - lam1 exact for float32).
template <typename T, int BS>
__global__ __launch_bounds__(BS) void k_eig2_bwd(Bwd2Args<T> a) {
    const uint32_t n = a.n;
    for (uint32_t i = blockIdx.x * BS + threadIdx.x; i - threadIdx.x < n; i += gridDim.x * BS) {
        T L[2], D[4], gl[2], gD[4], gA[3];
#pragma unroll
        for (int c = 0; c < 2; ++c) L[c] = ld_plane<T, kStream>(a.p.lam[c], n, i);
#pragma unroll
        for (int c = 0; c < 4; ++c) D[c] = ld_plane<T, kStream>(a.p.D[c], n, i);
#pragma unroll
        for (int c = 0; c < 2; ++c) gl[c] = ld_plane<T, kStream>(a.p.glam[c], n, i);
#pragma unroll
        for (int c = 0; c < 4; ++c) gD[c] = ld_plane<T, kStream>(a.p.gD[c], n, i);
        const double gphi = ld_plane<T, kStream>(a.p.gphi, n, i);
        // float64 arithmetic for either storage type (as in the 3x3 adjoint)
        const double l0 = L[0], l1 = L[1];
        const double d = l1 - l0;
        const double eps = a.eps_rel * sqrt_any64(l0 * l0 + l1 * l1);
        double Dd[4], gld[2], gDd[4], gAd[3];
#pragma unroll
        for (int c = 0; c < 4; ++c) Dd[c] = (double)D[c];
#pragma unroll
        for (int c = 0; c < 4; ++c) gDd[c] = (double)gD[c];
        gld[0] = gl[0];
        gld[1] = gl[1];
        adjoint2<double>(Dd, gld, gDd, gphi, d, eps * eps, gAd);
#pragma unroll
        for (int c = 0; c < 3; ++c) gA[c] = (T)gAd[c];
#pragma unroll
        for (int c = 0; c < 3; ++c) st_plane<T, kStream>(a.p.gA[c], n, i, gA[c]);
    }
}

// ----------------------------------------------------- inverse maps -------
// A = D diag(lam) D^T from the angles: D = R1(phi1) R2(phi2) R3(phi3), eq.
// (2.6) (build_D, as the forward), or D = R(phi), eq. (2.5).  Planes as the
// forward reads them; one matrix per lane, grid-stride, streamed.
template <typename T> struct ComposePtrs {
    const T *lam[3];
    const T *phi[3];
    T *A[6];
};
template <typename T> struct ComposeArgs {
    ComposePtrs<T> p;
    uint32_t n;
    int32_t pad;
};


template <typename T, int BS>
__global__ __launch_bounds__(BS) void k_compose3(ComposeArgs<T> a) {
    const uint32_t n = a.n;
    for (uint32_t i = blockIdx.x * BS + threadIdx.x; i - threadIdx.x < n; i += gridDim.x * BS) {
        T L[3], F[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) L[c] = ld_plane<T, kStream>(a.p.lam[c], n, i);
#pragma unroll
        for (int c = 0; c < 3; ++c) F[c] = ld_plane<T, kStream>(a.p.phi[c], n, i);
        Rot<T> R;
        sincos_t(F[0], R.s1, R.c1);
        sincos_t(F[1], R.s2, R.c2);
        sincos_t(F[2], R.s3, R.c3);
        T D[9];
        build_D(R, D);
        // A_ij = sum_k D_ik lam_k D_jk over the unique entries (11, 22, 33, 12, 13, 23)
        constexpr int I[6] = {0, 1, 2, 0, 0, 1}, J[6] = {0, 1, 2, 1, 2, 2};
#pragma unroll
        for (int e = 0; e < 6; ++e) {
            const T *r = D + 3 * I[e], *q = D + 3 * J[e];
            st_plane<T, kStream>(a.p.A[e], n, i, r[0] * L[0] * q[0] + r[1] * L[1] * q[1] + r[2] * L[2] * q[2]);
        }
    }
}

template <typename T, int BS>
__global__ __launch_bounds__(BS) void k_compose2(ComposeArgs<T> a) {
    const uint32_t n = a.n;
    for (uint32_t i = blockIdx.x * BS + threadIdx.x; i - threadIdx.x < n; i += gridDim.x * BS) {
        const T l1 = ld_plane<T, kStream>(a.p.lam[0], n, i), l2 = ld_plane<T, kStream>(a.p.lam[1], n, i);
        T s, c;
        sincos_t(ld_plane<T, kStream>(a.p.phi[0], n, i), s, c);
        st_plane<T, kStream>(a.p.A[0], n, i, c * c * l1 + s * s * l2);
        st_plane<T, kStream>(a.p.A[1], n, i, s * s * l1 + c * c * l2);
        st_plane<T, kStream>(a.p.A[2], n, i, c * s * (l1 - l2));
    }
}

// ------------------------------------------------ mixed persistent batch ---
template <typename T> struct GroupDesc {
    int64_t n;        // at most KSYM_CHUNK (the host splits larger groups)
    int32_t kind;
    int32_t pad;
    Eig3Ptrs<T> p3;   // kind 2 uses in[0..2] and out[O_LAM..+1], out[O_D..+3], out[O_PHI], flags
};

// Where a wave tile of a mixed batch lives: its group descriptor and the
// offset of its first matrix inside the group.
struct TileInfo {
    int32_t group;
    uint32_t base;
};

__device__ __forceinline__ TileInfo tile_at(cptr<TileInfo> tiles, int64_t t) {
    TileInfo r;
    r.group = tiles[t].group;
    r.base = tiles[t].base;
    return r;
}

template <typename T> struct MixedArgs {
    const GroupDesc<T> *groups;
    const TileInfo *tiles;       // one entry per wave tile, in group order
    int32_t ngroups;
    int64_t ntiles;
    Eig3Params prm;              // thresholds and counters (prm.n unused)
};

// Inputs of one mixed-batch wave tile (the 2x2 kind uses planes 0..2; its
// planes 3..5 are absent and read as zeros).
template <typename T> struct TableInputs {
    cptr<GroupDesc<T>> g;
    __device__ __forceinline__ const T *in(int c) const { return g->p3.in[c]; }
    __device__ __forceinline__ PtrN<const T, 6> ins() const { return ptrs_at<const T, 6>(&g->p3.in[0]); }
    __device__ __forceinline__ const T *aos() const { return nullptr; }
};

template <typename T, int MPL, int LP>
__device__ __forceinline__ void load_mixed(WIn<T, MPL, false> &in, cptr<GroupDesc<T>> g, uint32_t base) {
    load_wtile3<T, MPL, false, LP>(in, TableInputs<T>{g}, (uint32_t)g->n, base);
}

// One 2x2 wave tile of a mixed batch from inputs already in registers.
template <typename T, int MPL, int SP>
__device__ __forceinline__ void wtile_eig2_in(const __attribute__((address_space(4))) GroupDesc<T> &g,
                                              const WIn<T, MPL, false> &in, uint32_t base) {
    const uint32_t n = (uint32_t)g.n;
    const int lane = lane_id();
    T *const out[7] = {g.p3.out[O_LAM], g.p3.out[O_LAM + 1], g.p3.out[O_D], g.p3.out[O_D + 1],
                       g.p3.out[O_D + 2], g.p3.out[O_D + 3], g.p3.out[O_PHI]};
#pragma unroll
    for (int k = 0; k < MPL; ++k)
        eig2_lane<T, SP>(in.a[k][0], in.a[k][1], in.a[k][2], out, g.p3.flags, n, base + k * WAVE + lane);
}

// One persistent launch over all groups.  Wave tile t is described by
// tiles[t] (a tile never spans two groups, so a wave runs one kind at a
// time); the wave reads the descriptor of tile t + 2*stride and the inputs of
// tile t + stride while it computes tile t.  3x3 groups share the wave's
// refinement queue.  STREAM: the non-temporal policy for the plane loads and
// (float32) stores, chosen by the host when every plane starts on a 256-byte
// boundary, so that no cache line holds parts of two waves' tiles; otherwise
// the default policy, since two waves writing one line with non-temporal
// stores measured up to 50 % slower.  float32 with one matrix per lane fits
// the 80 VGPRs of 6 waves per SIMD, like k_eig3.
template <typename T, int BS, int MPL, bool STREAM>
__global__ __launch_bounds__(BS) __attribute__((amdgpu_waves_per_eu((sizeof(T) == 4 && MPL == 1) ? 6 : 1)))
void k_mixed(MixedArgs<T> a) {
    constexpr int NW = BS / WAVE;
    constexpr int PATH = (sizeof(T) == 4) ? PATH_FP32_FIXUP : PATH_FP64_FIXUP;
    // (the float64 checked path keeps its stores cached, as in k_eig3)
    constexpr int LP = STREAM ? kStream : kCached;
    constexpr int SP = (STREAM && sizeof(T) == 4) ? kStream : kCached;
    __shared__ WaveSmem<T, MPL, true, false> sm[NW];
    __shared__ int qcount[NW];   // the float64 pooled drain only
    const int wid = wave_id();
    WaveSmem<T, MPL, true, false> *my = &sm[wid];
    const cptr<GroupDesc<T>> groups = as_const(a.groups);
    const cptr<TileInfo> tiles = as_const(a.tiles);
    auto planes_of = [&](int g) { return TablePlanes<T>{&groups[g].p3, (uint32_t)groups[g].n}; };
    unsigned refined = 0, nonfinite = 0;
    int qn = 0, qage = 0;
    const int64_t stride = (int64_t)gridDim.x * NW;
    int64_t t = (int64_t)blockIdx.x * NW + wid;
    TileInfo cur = {0, 0}, nxt = {0, 0};
    WIn<T, MPL, false> in_cur, in_nxt;
    auto step = [&]() {
        const bool has_next = t + stride < a.ntiles;
        TileInfo nxt2 = {0, 0};
        if (t + 2 * stride < a.ntiles) nxt2 = tile_at(tiles, t + 2 * stride);
        if (has_next) load_mixed<T, MPL, LP>(in_nxt, groups + nxt.group, nxt.base);
        const auto &g = groups[cur.group];
        const uint32_t n = (uint32_t)g.n;
        if (g.kind == 3)
            wtile_eig3<T, PATH, MPL, false, SP, false>(planes_of(cur.group), planes_of, cur.group, a.prm,
                                                in_cur, n, cur.base, my, qn, qage, refined, nonfinite);
        else
            wtile_eig2_in<T, MPL, SP>(g, in_cur, cur.base);
        cur = nxt;
        nxt = nxt2;
        in_cur = in_nxt;
    };
    if (t < a.ntiles) {
        // the first tile peeled off, as in k_eig3: inside the loop the inputs
        // are register copies and need no memory wait
        cur = tile_at(tiles, t);
        load_mixed<T, MPL, LP>(in_cur, groups + cur.group, cur.base);
        if (t + stride < a.ntiles) nxt = tile_at(tiles, t + stride);
        step();
        for (t += stride; t < a.ntiles; t += stride) step();
    }
    // the leftovers, as in k_eig3
    if constexpr (sizeof(T) == 8) {
        final_drain<T, MPL, false, NW>(planes_of, sm, qcount, qn, wid, refined);
    } else {
        (void)qcount;
        if (qn > 0) {
            wave_sync();
            refined += drain_wave<T>(&my->q, qn, planes_of, 0);
        }
    }
    add_counters(a.prm.counters, refined, nonfinite);
}

__global__ void k_zero_u32(unsigned *p, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0u;
}

// ------------------------------------------- mixed batch without a plan ----
// The descriptor table and the tile table of a mixed batch written on the
// device from kernel arguments, for the entry point that allocates nothing
// (its tables live in a fixed device array).  DESC_BATCH descriptors travel
// per launch in the argument block (at most 4 KB), with the index of each
// one's first tile; the last batch also carries the total, which closes the
// prefix array.
constexpr int DESC_BATCH = 16;
template <typename T> struct DescBatch {
    GroupDesc<T> d[DESC_BATCH];
    int64_t first_tile[DESC_BATCH];
    int64_t total_tiles;   // written after the last descriptor when last != 0
    int32_t start, count, last, pad;
};
static_assert(sizeof(DescBatch<double>) <= 4096, "descriptor batch exceeds the kernel argument limit");

template <typename T>
__global__ __launch_bounds__(64) void k_put_desc(DescBatch<T> b, GroupDesc<T> *dst, int64_t *first) {
    const int i = threadIdx.x;
    if (i < b.count) {
        dst[b.start + i] = b.d[i];
        first[b.start + i] = b.first_tile[i];
    }
    if (i == 0 && b.last) first[b.start + b.count] = b.total_tiles;
}

// tiles[t] = (descriptor d, offset of the tile's first matrix in d) for the
// descriptor with first[d] <= t < first[d + 1]; empty descriptors (first[d] =
// first[d + 1]) own no tile.  first has ndesc + 1 entries, ndesc >= 1.
__global__ __launch_bounds__(256) void k_fill_tiles(const int64_t *first, int32_t ndesc, TileInfo *tiles,
                                                    int64_t ntiles, int32_t tile) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ntiles) return;
    int32_t lo = 0, hi = ndesc - 1;   // the last d with first[d] <= t
    while (lo < hi) {
        const int32_t mid = lo + (hi - lo + 1) / 2;
        if (first[mid] <= t) lo = mid;
        else hi = mid - 1;
    }
    tiles[t].group = lo;
    tiles[t].base = (uint32_t)((t - first[lo]) * tile);
}

}  // namespace ksym
