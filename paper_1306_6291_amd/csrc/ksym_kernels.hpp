// Tile processors and __global__ kernels for the ksym C ABI (gfx950, wave64).
//
// Work decomposition: every wavefront works on its own tiles of 64 * MPL
// matrices (MPL = matrices per lane) and walks them grid-stride; matrix
// k*64 + lane of a tile belongs to `lane`, so every plane load and store is one
// contiguous 64-element run and needs no staging.  The waves of a workgroup
// never wait for each other: there is no workgroup barrier in the 3x3 kernels.
//
// Refinement routing (3x3 float32 and float64 check paths): a lane whose
// matrix fails the check stores its provisional result and appends the matrix
// to its wave's queue in LDS (ballot + popcount for the count, mbcnt for the
// lane's rank; the count lives in a scalar register).  When the queue holds 64
// entries the wave refines them together, entry j on lane j, so the float64
// refinement always runs on full wavefronts, and overwrites those outputs.
//
// Offsets are 32-bit: one launch covers at most KSYM_CHUNK matrices (the host
// splits larger batches), so every access is a scalar base plus one 32-bit
// lane offset.
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

// Matrices per launch: offsets inside a launch are 32-bit byte offsets.
constexpr int64_t KSYM_CHUNK = int64_t(1) << 28;

struct Eig3Params {
    int64_t n;            // at most KSYM_CHUNK
    double tau_gap, tau_res, tau_vec, tau_dbl;
    unsigned *counters;   // [0] refined, [1] non-finite; may be null
    int32_t zero;         // always 0; see put3
    int32_t drain_tiles;  // queue age limit in wave tiles (0 = full waves only)
};

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

__device__ __forceinline__ double pow2(int e) { return __builtin_ldexp(1.0, e); }

// One 3x3 matrix through §4-§5.  PATH_FP32_FIXUP / PATH_FP64_FIXUP: general
// branch plus the float64 check; matrices failing it, near the double-root
// case or below tau_gap are marked for refinement.  PATH_FP64_PLAIN: general
// branch, or the paper's double-root branch (5.20)-(5.25) with the output slots
// restored, no check.
template <typename T, int PATH>
__device__ __forceinline__ void eig3_one(const T ain[6], const Eig3Params &prm, Out3<T> &o) {
    const bool fin = finite(ain[0]) && finite(ain[1]) && finite(ain[2]) && finite(ain[3]) &&
                     finite(ain[4]) && finite(ain[5]);
    double amax = 0.0;
#pragma unroll
    for (int c = 0; c < 6; ++c) amax = fmax(amax, __builtin_fabs((double)ain[c]));
    const int ex = fin ? scale_exponent(amax) : 0;
    const double sc = pow2(-ex), isc = pow2(ex);
    double a[6];
#pragma unroll
    for (int c = 0; c < 6; ++c) a[c] = fin ? (double)ain[c] * sc : 0.0;
    const double a11 = a[0], a22 = a[1], a33 = a[2], a12 = a[3], a13 = a[4], a23 = a[5];
    const Cubic cu = cubic_stage(a11, a22, a33, a12, a13, a23);
    o.refine = false;
    o.lc = 0.0;
    if (cu.triple) {
        // §5, p = 0: A = lam I with lam = A11; D = I, angles 0.
#pragma unroll
        for (int i = 0; i < 9; ++i) o.v[O_D + i] = (i % 4 == 0) ? T(1) : T(0);
        o.v[O_LAM] = o.v[O_LAM + 1] = o.v[O_LAM + 2] = (T)(cu.m * isc);
        o.v[O_PHI] = o.v[O_PHI + 1] = o.v[O_PHI + 2] = T(0);
        o.v[O_GAP] = o.v[O_GAP + 1] = o.v[O_GAP + 2] = T(0);
        o.flag = FLAG_TRIPLE;
    } else {
        const double split = fmin(cu.g13, cu.g32);
        const bool dbl = (cu.g13 * cu.g32 == 0.0) || split < prm.tau_dbl * cu.sp;
        const T A12 = (T)a12, A13 = (T)a13, A22 = (T)a22, A33 = (T)a33, A23 = (T)a23;
        if (PATH == PATH_FP64_PLAIN && dbl) {
            // double root: labels (lam, lam, lam_s), s = cos^2 phi2 (5.21), phi3 = 0;
            // deviations from the centre m keep s accurate when the spread is tiny
            double lm, ls;
            if (cu.g13 < cu.g32) { lm = 0.5 * (cu.mu1 + cu.mu3); ls = cu.mu2; }
            else { lm = 0.5 * (cu.mu3 + cu.mu2); ls = cu.mu1; }
            const T s = clamp01((T)((cu.d1 - ls) / (lm - ls)));
            const Rot<T> R = select_angles<T>(A12, A13, A22, A33, A23, T(0), (T)(lm - ls), (T)(ls - lm), s,
                                              T(1) - s, T(1), T(0));
            T Di[9];
            build_D(R, Di);
            double L[3];
            if (ls > lm) {   // (ls, lm, lm): columns (3, 1, 2), even permutation
                for (int r = 0; r < 3; ++r) {
                    o.v[O_D + 3 * r] = Di[3 * r + 2]; o.v[O_D + 3 * r + 1] = Di[3 * r]; o.v[O_D + 3 * r + 2] = Di[3 * r + 1];
                }
                L[0] = ls; L[1] = lm; L[2] = lm;
            } else {         // (lm, ls, lm): columns (1, 3, -2), odd permutation + sign
                for (int r = 0; r < 3; ++r) {
                    o.v[O_D + 3 * r] = Di[3 * r]; o.v[O_D + 3 * r + 1] = Di[3 * r + 2]; o.v[O_D + 3 * r + 2] = -Di[3 * r + 1];
                }
                L[0] = lm; L[1] = ls; L[2] = lm;
            }
            extract_angles<T>(o.v + O_D, o.v + O_PHI);
            for (int k = 0; k < 3; ++k) o.v[O_LAM + k] = (T)((cu.m + L[k]) * isc);
            o.v[O_GAP] = (T)((L[0] - L[1]) * isc);
            o.v[O_GAP + 1] = (T)((L[0] - L[2]) * isc);
            o.v[O_GAP + 2] = (T)((L[2] - L[1]) * isc);
            o.flag = FLAG_DOUBLE;
        } else {
            // general branch (5.1)-(5.15), with the eigenvalue differences
            // taken from the float64 stage.  The plain path evaluates v, w as
            // printed; the checked path forms v, 1 - v, w, 1 - w as separate
            // quotients (u_quotients), which stay accurate near coincident
            // eigenvalues.
            const T G12 = (T)cu.g12, G13 = (T)cu.g13, G32 = (T)cu.g32;
            T v, s2sq, w, cw;
            if (PATH == PATH_FP64_PLAIN) {
                const T e1 = (T)(cu.d1 - cu.mu1), e3 = (T)(cu.d1 - cu.mu3);   // A11 - lam1, A11 - lam3
                v = clamp01(Mth<T>::div(A12 * A12 + A13 * A13 + e3 * (e1 + G32), G32 * G13));
                w = (v == T(0)) ? T(1) : clamp01(Mth<T>::div(e3 + G32 * v, G12 * v));
                s2sq = T(1) - v;
                cw = T(1) - w;
            } else {
                const URow u = u_quotients(cu.d1, cu.mu1, cu.mu2, cu.mu3, cu.g13, cu.g32, a12, a13);
                v = (T)u.v; s2sq = (T)u.s2sq; w = (T)u.w; cw = (T)u.cw;
            }
            const Rot<T> R = select_angles<T>(A12, A13, A22, A33, A23, G12, G13, G32, v, s2sq, w, cw);
            build_D(R, o.v + O_D);
            angles_of(R, o.v + O_PHI);
            o.v[O_LAM] = (T)((cu.m + cu.mu1) * isc);
            o.v[O_LAM + 1] = (T)((cu.m + cu.mu2) * isc);
            o.v[O_LAM + 2] = (T)((cu.m + cu.mu3) * isc);
            o.v[O_GAP] = (T)(cu.g12 * isc);
            o.v[O_GAP + 1] = (T)(cu.g13 * isc);
            o.v[O_GAP + 2] = (T)(cu.g32 * isc);
            o.flag = dbl ? FLAG_DOUBLE : FLAG_GENERAL;
            if (PATH != PATH_FP64_PLAIN) {
                const double fro = ::sqrt(a11 * a11 + a22 * a22 + a33 * a33 +
                                          2.0 * (a12 * a12 + a13 * a13 + a23 * a23));
                const double lmax = fmax(__builtin_fabs(cu.m + cu.mu1), __builtin_fabs(cu.m + cu.mu2));
                bool bad = dbl || (split < prm.tau_gap * lmax);
                double dd[9];
#pragma unroll
                for (int i = 0; i < 9; ++i) dd[i] = (double)o.v[O_D + i];
                bad = bad || check_fails<double>(cu.d1, cu.d2, cu.d3, a12, a13, a23, dd, cu.mu1, cu.mu2,
                                                 cu.mu3, cu.g12, cu.g13, cu.g32, prm.tau_res * fro,
                                                 prm.tau_vec);
                o.refine = bad;
                o.lc = (cu.g13 >= cu.g32) ? cu.mu1 : cu.mu2;
            }
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

// The float32 path for one matrix: the cubic stage in float64 (with float32
// polynomial tails), the squared cosines of the angle solve as float64
// quotients, the rest in float32, and the a-posteriori check in float32 on
// B = A - m I.  Outputs leave through sink.put(k, value) as soon as they
// exist (plane k of lam, D, phi, gap), which keeps few of them in registers.
// Sets refine (and the isolated eigenvalue lc for the refinement, a float64
// deviation in scaled units) and returns the flag.
template <typename Sink>
__device__ __forceinline__ int eig3_f32(const float ain[6], const Eig3Params &prm, const Sink &sink,
                                        bool &refine, double &lc) {
    const bool fin = finite(ain[0]) && finite(ain[1]) && finite(ain[2]) && finite(ain[3]) &&
                     finite(ain[4]) && finite(ain[5]);
    float amax = __builtin_fmaxf(__builtin_fmaxf(__builtin_fabsf(ain[0]), __builtin_fabsf(ain[1])),
                                 __builtin_fabsf(ain[2]));
    amax = __builtin_fmaxf(amax, __builtin_fmaxf(__builtin_fmaxf(__builtin_fabsf(ain[3]),
                                                                 __builtin_fabsf(ain[4])),
                                                 __builtin_fabsf(ain[5])));
    const int ex = fin ? scale_exponent((double)amax) : 0;
    const double sc = pow2(-ex), isc = pow2(ex);
    double a[6];
#pragma unroll
    for (int c = 0; c < 6; ++c) a[c] = (double)ain[c] * sc;   // non-finite: handled below
    const Cubic cu = cubic_stage_fast(a[0], a[1], a[2], a[3], a[4], a[5]);
    refine = false;
    lc = 0.0;
    if (cu.triple || !fin) {
        // §5, p = 0: A = lam I, D = I, angles 0 (non-finite input: all NaN)
        const float nan = __builtin_nanf("");
        const float lam = fin ? (float)(cu.m * isc) : nan;
        const float one = fin ? 1.0f : nan, zero = fin ? 0.0f : nan;
#pragma unroll
        for (int k = 0; k < 3; ++k) sink.put(O_LAM + k, lam);
#pragma unroll
        for (int i = 0; i < 9; ++i) sink.put(O_D + i, (i % 4 == 0) ? one : zero);
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            sink.put(O_PHI + k, zero);
            sink.put(O_GAP + k, zero);
        }
        const int flag = fin ? FLAG_TRIPLE : FLAG_NONFINITE;
        sink.flag(flag);
        return flag;
    }
    sink.put(O_LAM, (float)((cu.m + cu.mu1) * isc));
    sink.put(O_LAM + 1, (float)((cu.m + cu.mu2) * isc));
    sink.put(O_LAM + 2, (float)((cu.m + cu.mu3) * isc));
    sink.put(O_GAP, (float)(cu.g12 * isc));
    sink.put(O_GAP + 1, (float)(cu.g13 * isc));
    sink.put(O_GAP + 2, (float)(cu.g32 * isc));
    const double split = cu.g13 < cu.g32 ? cu.g13 : cu.g32;
    const bool dbl = (cu.g13 * cu.g32 == 0.0) || split < prm.tau_dbl * cu.sp;
    const double l1 = __builtin_fabs(cu.m + cu.mu1), l2 = __builtin_fabs(cu.m + cu.mu2);
    bool bad = dbl || (split < prm.tau_gap * (l1 > l2 ? l1 : l2));
    lc = (cu.g13 >= cu.g32) ? cu.mu1 : cu.mu2;
    // general branch (5.1)-(5.15): the four squared cosines and sines as
    // float64 quotients (u_quotients), the rest of the angle solve in float32
    const URow u = u_quotients(cu.d1, cu.mu1, cu.mu2, cu.mu3, cu.g13, cu.g32, a[3], a[4]);
    const float A12 = (float)a[3], A13 = (float)a[4], A23 = (float)a[5];
    const float G12 = (float)cu.g12, G13 = (float)cu.g13, G32 = (float)cu.g32;
    const Rot<float> R = select_angles<float>(A12, A13, (float)a[1], (float)a[2], A23, G12, G13, G32,
                                              (float)u.v, (float)u.s2sq, (float)u.w, (float)u.cw);
    float phi[3];
    angles_of(R, phi);
#pragma unroll
    for (int k = 0; k < 3; ++k) sink.put(O_PHI + k, phi[k]);
    float D[9];
    build_D(R, D);
#pragma unroll
    for (int i = 0; i < 9; ++i) sink.put(O_D + i, D[i]);
    const float fro = __builtin_sqrtf((float)(a[0] * a[0] + a[1] * a[1] + a[2] * a[2] +
                                              2.0 * (a[3] * a[3] + a[4] * a[4] + a[5] * a[5])));
    bad = bad || check_fails<float>((float)cu.d1, (float)cu.d2, (float)cu.d3, A12, A13, A23, D,
                                    (float)cu.mu1, (float)cu.mu2, (float)cu.mu3, G12, G13, G32,
                                    (float)prm.tau_res * fro, (float)prm.tau_vec);
    const int flag = dbl ? FLAG_DOUBLE : FLAG_GENERAL;
    sink.flag(flag);
    refine = bad;
    return flag;
}

// The refinement of one queued matrix (original entries ain, isolated
// eigenvalue lc as a deviation from the centre, in the scaled units eig3_one
// used; the centre is recomputed here with the same arithmetic).
template <typename T>
__device__ __forceinline__ void refine_one(const T ain[6], double lc, int flag, Out3<T> &o) {
    double amax = 0.0;
#pragma unroll
    for (int c = 0; c < 6; ++c) amax = fmax(amax, __builtin_fabs((double)ain[c]));
    const int ex = scale_exponent(amax);
    const double sc = pow2(-ex), isc = pow2(ex);
    double m, d1, d2, d3;
    center3((double)ain[0] * sc, (double)ain[1] * sc, (double)ain[2] * sc, m, d1, d2, d3);
    const Refined rf = refine3(d1, d2, d3, (double)ain[3] * sc, (double)ain[4] * sc,
                               (double)ain[5] * sc, lc);
#pragma unroll
    for (int i = 0; i < 9; ++i) o.v[O_D + i] = (T)rf.D[i];
    extract_angles<T>(o.v + O_D, o.v + O_PHI);
#pragma unroll
    for (int k = 0; k < 3; ++k) o.v[O_LAM + k] = (T)((m + rf.lam[k]) * isc);
    o.v[O_GAP] = (T)(fmax(rf.lam[0] - rf.lam[1], 0.0) * isc);
    o.v[O_GAP + 1] = (T)(fmax(rf.lam[0] - rf.lam[2], 0.0) * isc);
    o.v[O_GAP + 2] = (T)(fmax(rf.lam[2] - rf.lam[1], 0.0) * isc);
    o.flag = flag | FLAG_FIXUP;
}

// ------------------------------------------------------ per-wave tiles -----
constexpr int WAVE = 64;

// The lane index, recomputed where it is used (two mbcnt) rather than kept in
// a register across the tile loop: under the 96-register budget the compiler
// would otherwise spill it and reload it (with a full memory wait) per tile.
__device__ __forceinline__ uint32_t fresh(uint32_t x);
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
// Element `off` of plane p through a 32-bit byte offset (off < KSYM_CHUNK),
// as a global-memory pointer: every plane is device memory, and saying so
// gives global_load / global_store with a scalar base instead of flat
// accesses when the plane pointer itself was read from memory.
template <typename T> using gptr = __attribute__((address_space(1))) T *;
template <typename T> __device__ __forceinline__ gptr<T> elem(T *p, uint32_t off) {
    return (gptr<T>)((gptr<char>)p + off * (uint32_t)sizeof(T));
}
// Read-only tables (mixed-batch descriptors and tile entries) in the constant
// address space: they do not change while a kernel runs, so uniform reads
// become scalar loads even though the kernel stores to global memory.
// The value x, opaque to the optimizer (no instruction is emitted).  Used on
// the 32-bit offset of an access inside a conditional block, so the offset is
// extended to 64 bits in that block and the access can take the scalar-base
// plus 32-bit-offset form instead of a 64-bit per-lane address.
__device__ __forceinline__ uint32_t fresh(uint32_t x) {
    asm volatile("" : "+v"(x));
    return x;
}
template <typename T> using cptr = const __attribute__((address_space(4))) T *;
template <typename T> __device__ __forceinline__ cptr<T> as_const(const T *p) { return (cptr<T>)p; }

// Output plane pointers read from the kernel-argument segment with a
// plane-dependent offset: the pointers are fetched (a few scalar loads) where a
// matrix's outputs are stored instead of being held in scalar registers for
// the whole kernel.
template <typename T> struct KernargPlanes {
    uint32_t out_off, flags_off;   // byte offsets inside the argument segment
    __device__ __forceinline__ T *out(int k) const {
        typedef __attribute__((address_space(4))) const char *kptr;
        kptr ka = (kptr)__builtin_amdgcn_kernarg_segment_ptr();
        return *(T *const __attribute__((address_space(4))) *)(ka + out_off + 8 * k);
    }
    __device__ __forceinline__ uint8_t *flags(int salt = 0) const {
        typedef __attribute__((address_space(4))) const char *kptr;
        kptr ka = (kptr)__builtin_amdgcn_kernarg_segment_ptr();
        return *(uint8_t *const __attribute__((address_space(4))) *)(ka + flags_off + 8 * salt);
    }
};

// Output plane pointers of a group descriptor in device memory.
template <typename T> struct TablePlanes {
    cptr<Eig3Ptrs<T>> p;
    __device__ __forceinline__ T *out(int k) const { return p->out[k]; }
    __device__ __forceinline__ uint8_t *flags(int salt = 0) const { return (&p->flags)[salt]; }
};

// Store one matrix's outputs.  The plane index is offset by salt, which is 0
// at run time but not known to the compiler, so the pointer loads stay here
// instead of being hoisted out of the tile loop (where they would pin 38
// scalar registers for the whole kernel).
template <typename T, typename Planes>
__device__ __forceinline__ void put3(const Planes &pl, int salt, uint32_t off, const Out3<T> &o) {
    T *dst[NOUT3];
#pragma unroll
    for (int k = 0; k < NOUT3; ++k) dst[k] = pl.out(k + salt);
    uint8_t *fl = pl.flags(salt);
#pragma unroll
    for (int k = 0; k < NOUT3; ++k)
        if (dst[k]) *elem(dst[k], fresh(off)) = o.v[k];
    if (fl) *elem(fl, fresh(off)) = (uint8_t)o.flag;
}

// Stores of one lane's matrix as its outputs are produced (float32 path).
// FULL: every lane of the tile holds a matrix (no per-lane bounds test).
template <typename T, typename Planes, bool FULL> struct LaneSink {
    const Planes &pl;
    int salt;
    uint32_t off;
    bool valid;
    __device__ __forceinline__ void put(int k, T v) const {
        T *d = pl.out(k + salt);
        if ((FULL || valid) && d) *elem(d, fresh(off)) = v;
    }
    __device__ __forceinline__ void flag(int f) const {
        uint8_t *fl = pl.flags(salt);
        if ((FULL || valid) && fl) *elem(fl, fresh(off)) = (uint8_t)f;
    }
};

// A refined result: scattered stores (the rare path).
template <typename T, typename Planes>
__device__ __forceinline__ void write_out3(const Planes &pl, uint32_t off, const Out3<T> &o) {
#pragma unroll
    for (int k = 0; k < NOUT3; ++k) {
        T *dst = pl.out(k);
        if (dst) *elem(dst, fresh(off)) = o.v[k];
    }
    uint8_t *fl = pl.flags();
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

// FULL: the whole tile lies below n (unconditional loads).  Otherwise lanes
// past n load the last matrix (a clamped, in-bounds offset) and take zeros.
template <typename T, int MPL, bool AOS, bool FULL>
__device__ __forceinline__ void load_wtile3(WIn<T, MPL, AOS> &in, const T *const *planes,
                                            const T *aos, uint32_t n, uint32_t base) {
    const int lane = lane_id();
    if constexpr (AOS) {
        using W = WIn<T, MPL, AOS>;
        constexpr int VEC = W::VEC;
        const uint32_t lim = (n - base) * 6;   // valid elements from `base` on
        const T *src = aos + (size_t)base * 6;
#pragma unroll
        for (int u = 0; u < W::NVL; ++u) {
            const uint32_t j = u * WAVE + lane;
            const uint32_t e0 = j * VEC;
            if (j < (uint32_t)W::NV && e0 + VEC <= lim) {
                typedef T vec_t __attribute__((ext_vector_type(VEC)));
                const vec_t x = *reinterpret_cast<gptr<const vec_t>>(elem(src, e0));
#pragma unroll
                for (int t = 0; t < VEC; ++t) in.v[u][t] = x[t];
            } else {
#pragma unroll
                for (int t = 0; t < VEC; ++t)
                    in.v[u][t] = (j < (uint32_t)W::NV && e0 + t < lim) ? *elem(src, e0 + t) : T(0);
            }
        }
    } else {
#pragma unroll
        for (int k = 0; k < MPL; ++k) {
            const uint32_t off = base + k * WAVE + lane;
            const bool ok = FULL || off < n;
            const uint32_t offc = ok ? off : n - 1;
#pragma unroll
            for (int c = 0; c < 6; ++c) {
                const T v = *elem(planes[c], offc);
                in.a[k][c] = ok ? v : T(0);
            }
        }
    }
}

// Refine the first `cnt` (<= 64) queue entries, entry j on lane j, and
// overwrite their provisional outputs.  The wave's own provisional stores are
// waited for first, so a refined value always lands last.
template <typename T, int CAP, typename PlanesOf>
__device__ __forceinline__ void drain_wave(WaveQueue<T, CAP> *q, int cnt, const PlanesOf &planes_of) {
    __builtin_amdgcn_s_waitcnt(0x0f70);   // vmcnt(0): earlier stores of this wave have completed
    const int lane = lane_id();
    if (lane < cnt) {
        T a[6];
#pragma unroll
        for (int c = 0; c < 6; ++c) a[c] = q->a[c][lane];
        const int g = q->grp[lane];
        Out3<T> o;
        refine_one<T>(a, q->lc[lane], g >> 24, o);
        write_out3(planes_of(g & 0xffffff), q->off[lane], o);
    }
}

// Process one wave tile of 64*MPL 3x3 matrices starting at `base` from inputs
// already in registers: compute, store, queue the matrices that need the
// refinement, and drain the queue in rounds of 64.  Wave-uniform control flow.
template <typename T, int PATH, int MPL, bool AOS, bool FULL, typename Planes, typename PlanesOf>
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
        const bool valid = FULL || off < n;
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
            flag = eig3_f32(A, prm, LaneSink<T, Planes, FULL>{pl, salt, off, valid}, refine, lc);
        } else {
            Out3<T> o;
            eig3_one<T, PATH>(A, prm, o);
            if (valid) put3(pl, salt, off, o);
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
            drain_wave<T>(&sm->q, cnt, planes_of);
            refined += (unsigned)cnt;
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

// Refine what is left in a wave's queue at the end of its work.
template <typename T, int MPL, bool AOS, typename PlanesOf>
__device__ __forceinline__ void final_drain(const PlanesOf &planes_of, WaveSmem<T, MPL, true, AOS> *sm,
                                            int qn, unsigned &refined) {
    if (qn > 0) {
        wave_sync();
        drain_wave<T>(&sm->q, qn, planes_of);
        refined += (unsigned)qn;
    }
}

__device__ __forceinline__ void add_counters(unsigned *counters, unsigned refined, unsigned nonfinite) {
    if (counters && lane_id() == 0) {
        if (refined) atomicAdd(&counters[0], refined);
        if (nonfinite) atomicAdd(&counters[1], nonfinite);
    }
}

// float32, one matrix per lane, SoA: the refinement path needs a few more
// registers than the main path; asking for 5 waves per SIMD makes the
// compiler fit both into 96 VGPRs (without spills) instead of dropping to 4.
template <typename T, int PATH, int BS, int MPL, bool AOS>
__global__ __launch_bounds__(BS)
__attribute__((amdgpu_waves_per_eu((sizeof(T) == 4 && MPL == 1 && !AOS) ? 5 : 1)))
void k_eig3(Eig3Args<T> args) {
    constexpr int NW = BS / WAVE;
    constexpr int WT = WAVE * MPL;
    constexpr bool QUEUE = PATH != PATH_FP64_PLAIN;
    __shared__ WaveSmem<T, MPL, QUEUE, AOS> sm[NW];
    WaveSmem<T, MPL, QUEUE, AOS> *my = &sm[wave_id()];
    const uint32_t n = (uint32_t)args.prm.n;
    const uint32_t ntiles = (n + WT - 1) / WT;
    KernargPlanes<T> pl;
    pl.out_off = (uint32_t)(offsetof(Eig3Args<T>, p) + offsetof(Eig3Ptrs<T>, out));
    pl.flags_off = (uint32_t)(offsetof(Eig3Args<T>, p) + offsetof(Eig3Ptrs<T>, flags));
    auto planes_of = [&](int) { return pl; };
    unsigned refined = 0, nonfinite = 0;
    int qn = 0, qage = 0;
    WIn<T, MPL, AOS> cur, nxt;
    const uint32_t stride = gridDim.x * NW;
    uint32_t t = blockIdx.x * NW + wave_id();
    const uint32_t nfull = n / WT;   // tiles with no lane past n
    auto load = [&](WIn<T, MPL, AOS> &w, uint32_t tt) {
        if (tt < nfull) load_wtile3<T, MPL, AOS, true>(w, args.p.in, args.aos, n, tt * WT);
        else load_wtile3<T, MPL, AOS, false>(w, args.p.in, args.aos, n, tt * WT);
    };
    if (t < ntiles) load(cur, t);
    for (; t < ntiles; t += stride) {
        const uint32_t tn = t + stride;
        if (tn < ntiles) load(nxt, tn);
        if (t < nfull)
            wtile_eig3<T, PATH, MPL, AOS, true>(pl, planes_of, 0, args.prm, cur, n, t * WT, my, qn, qage,
                                                refined, nonfinite);
        else
            wtile_eig3<T, PATH, MPL, AOS, false>(pl, planes_of, 0, args.prm, cur, n, t * WT, my, qn, qage,
                                                 refined, nonfinite);
        cur = nxt;
    }
    if constexpr (QUEUE) final_drain<T, MPL, AOS>(planes_of, my, qn, refined);
    add_counters(args.prm.counters, refined, nonfinite);
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
// phi (any may be null).
template <typename T>
__device__ __forceinline__ void eig2_lane(T a11, T a22, T a12, T *const out[7], uint8_t *flags,
                                          uint32_t off) {
    const bool fin = finite(a11) && finite(a22) && finite(a12);
    // exact power-of-two scaling keeps d^2 + 4 A12^2 in range
    const double amax = fmax(fmax(__builtin_fabs((double)a11), __builtin_fabs((double)a22)),
                             __builtin_fabs((double)a12));
    const int ex = fin ? scale_exponent(amax) : 0;
    const T sc = (T)pow2(-ex), isc = (T)pow2(ex);
    Eig2<T> e = eig2_one<T>(a11 * sc, a22 * sc, a12 * sc);
    e.l1 *= isc;
    e.l2 *= isc;
    if (!fin) {
        const T nan = T(__builtin_nan(""));
        e.l1 = e.l2 = e.c = e.s = e.phi = nan;
    }
    const T v[7] = {e.l1, e.l2, e.c, -e.s, e.s, e.c, e.phi};
#pragma unroll
    for (int k = 0; k < 7; ++k)
        if (out[k]) *elem(out[k], fresh(off)) = v[k];
    if (flags) *elem(flags, fresh(off)) = fin ? (uint8_t)0 : (uint8_t)FLAG_NONFINITE;
}

// One wave tile of 64*MPL 2x2 matrices, straight from and to HBM.
template <typename T, int MPL, bool FULL>
__device__ __forceinline__ void wtile_eig2(const Eig2Ptrs<T> &p, uint32_t n, uint32_t base) {
    const int lane = lane_id();
    T A[MPL][3];
#pragma unroll
    for (int k = 0; k < MPL; ++k) {
        const uint32_t off = base + k * WAVE + lane;
        const bool ok = FULL || off < n;
        const uint32_t offc = ok ? off : n - 1;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const T v = *elem(p.in[c], offc);
            A[k][c] = ok ? v : T(0);
        }
    }
    T *const out[7] = {p.lam[0], p.lam[1], p.D[0], p.D[1], p.D[2], p.D[3], p.phi};
#pragma unroll
    for (int k = 0; k < MPL; ++k) {
        const uint32_t off = base + k * WAVE + lane;
        if (FULL || off < n) eig2_lane<T>(A[k][0], A[k][1], A[k][2], out, p.flags, off);
    }
}

template <typename T, int BS, int MPL>
__global__ __launch_bounds__(BS) void k_eig2(Eig2Ptrs<T> p, uint32_t n) {
    constexpr int NW = BS / WAVE, WT = WAVE * MPL;
    const uint32_t ntiles = (n + WT - 1) / WT;
    const uint32_t stride = gridDim.x * NW;
    const uint32_t nfull = n / WT;
    for (uint32_t t = blockIdx.x * NW + wave_id(); t < ntiles; t += stride) {
        if (t < nfull) wtile_eig2<T, MPL, true>(p, n, t * WT);
        else wtile_eig2<T, MPL, false>(p, n, t * WT);
    }
}

// -------------------------------------------------------- adjoint ----------
template <typename T> struct BwdPtrs {
    const T *lam[3];
    const T *D[9];
    const T *gap[3];
    const T *glam[3];
    const T *gD[9];
    T *gA[6];
};

// One lane's adjoint.  FULL: i < n is known; otherwise lanes past n read the
// last matrix (in bounds) and store nothing.
template <typename T, bool FULL>
__device__ __forceinline__ void bwd_lane(const BwdPtrs<T> &p, bool has_gap, bool has_gl, bool has_gd,
                                         uint32_t i, uint32_t n, double eps_rel) {
    const bool ok = FULL || i < n;
    const uint32_t ic = ok ? i : n - 1;
    T L[3], D[9], gl[3], gD[9], gA[6];
#pragma unroll
    for (int c = 0; c < 3; ++c) L[c] = *elem(p.lam[c], ic);
#pragma unroll
    for (int c = 0; c < 9; ++c) D[c] = *elem(p.D[c], ic);
#pragma unroll
    for (int c = 0; c < 3; ++c) gl[c] = has_gl ? *elem(p.glam[c], fresh(ic)) : T(0);
#pragma unroll
    for (int c = 0; c < 9; ++c) gD[c] = has_gd ? *elem(p.gD[c], fresh(ic)) : T(0);
    T g12, g13, g32;
    if (has_gap) {
        const uint32_t o = fresh(ic);
        g12 = *elem(p.gap[0], o); g13 = *elem(p.gap[1], o); g32 = *elem(p.gap[2], o);
    } else {
        // differences of the stored eigenvalues, exact in float64
        g12 = (T)((double)L[0] - (double)L[1]);
        g13 = (T)((double)L[0] - (double)L[2]);
        g32 = (T)((double)L[2] - (double)L[1]);
    }
    const T eps = (T)eps_rel * Mth<T>::sqrt(L[0] * L[0] + L[1] * L[1] + L[2] * L[2]);
    adjoint3<T>(D, gl, gD, g12, g13, g32, eps * eps, gA);
    if (ok) {
        const uint32_t o = fresh(i);
#pragma unroll
        for (int c = 0; c < 6; ++c) *elem(p.gA[c], o) = gA[c];
    }
}

template <typename T, int BS, int MPL>
__global__ __launch_bounds__(BS) void k_eig3_bwd(BwdPtrs<T> p, uint32_t n, double eps_rel) {
    constexpr int TILE = BS * MPL;
    const uint32_t ntiles = (n + TILE - 1) / TILE;
    const uint32_t nfull = n / TILE;
    const bool has_gap = p.gap[0] && p.gap[1] && p.gap[2];
    const bool has_gl = p.glam[0] != nullptr;
    const bool has_gd = p.gD[0] != nullptr;
    for (uint32_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
#pragma unroll
        for (int k = 0; k < MPL; ++k) {
            const uint32_t i = t * TILE + k * BS + threadIdx.x;
            if (t < nfull) bwd_lane<T, true>(p, has_gap, has_gl, has_gd, i, n, eps_rel);
            else bwd_lane<T, false>(p, has_gap, has_gl, has_gd, i, n, eps_rel);
        }
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

// Inputs of one mixed-batch wave tile (the 2x2 kind uses planes 0..2; the
// other slots are zero).  One loop for both kinds keeps the tile in registers;
// lanes past n read the group's last matrix (in bounds) and take zeros.
template <typename T, int MPL>
__device__ __forceinline__ void load_mixed(WIn<T, MPL, false> &in, const __attribute__((address_space(4))) GroupDesc<T> &g,
                                           uint32_t base) {
    const uint32_t n = (uint32_t)g.n;
    const int np = g.kind == 3 ? 6 : 3;
    const int lane = lane_id();
#pragma unroll
    for (int c = 0; c < 6; ++c) {
        const T *pc = g.p3.in[c];
#pragma unroll
        for (int k = 0; k < MPL; ++k) {
            const uint32_t off = base + k * WAVE + lane;
            const bool ok = off < n;
            const uint32_t offc = ok ? off : n - 1;
            T v = T(0);
            if (c < np) v = *elem(pc, fresh(offc));
            in.a[k][c] = ok ? v : T(0);
        }
    }
}

// One 2x2 wave tile of a mixed batch from inputs already in registers.
template <typename T, int MPL, bool FULL>
__device__ __forceinline__ void wtile_eig2_in(const __attribute__((address_space(4))) GroupDesc<T> &g,
                                              const WIn<T, MPL, false> &in,
                                              uint32_t base) {
    const uint32_t n = (uint32_t)g.n;
    const int lane = lane_id();
    T *const out[7] = {g.p3.out[O_LAM], g.p3.out[O_LAM + 1], g.p3.out[O_D], g.p3.out[O_D + 1],
                       g.p3.out[O_D + 2], g.p3.out[O_D + 3], g.p3.out[O_PHI]};
#pragma unroll
    for (int k = 0; k < MPL; ++k) {
        const uint32_t off = base + k * WAVE + lane;
        if (FULL || off < n) eig2_lane<T>(in.a[k][0], in.a[k][1], in.a[k][2], out, g.p3.flags, off);
    }
}

// One persistent launch over all groups.  Wave tile t is described by
// tiles[t] (a tile never spans two groups, so a wave runs one kind at a
// time); the wave reads the descriptor of tile t + 2*stride and the inputs of
// tile t + stride while it computes tile t.  3x3 groups share the wave's
// refinement queue.
template <typename T, int BS, int MPL>
__global__ __launch_bounds__(BS) __attribute__((amdgpu_waves_per_eu((sizeof(T) == 4 && MPL == 1) ? 5 : 1)))
void k_mixed(MixedArgs<T> a) {
    constexpr int NW = BS / WAVE;
    constexpr int PATH = (sizeof(T) == 4) ? PATH_FP32_FIXUP : PATH_FP64_FIXUP;
    __shared__ WaveSmem<T, MPL, true, false> sm[NW];
    WaveSmem<T, MPL, true, false> *my = &sm[wave_id()];
    const cptr<GroupDesc<T>> groups = as_const(a.groups);
    const cptr<TileInfo> tiles = as_const(a.tiles);
    auto planes_of = [&](int g) { return TablePlanes<T>{&groups[g].p3}; };
    unsigned refined = 0, nonfinite = 0;
    int qn = 0, qage = 0;
    const int64_t stride = (int64_t)gridDim.x * NW;
    int64_t t = (int64_t)blockIdx.x * NW + wave_id();
    TileInfo cur = {0, 0}, nxt = {0, 0};
    WIn<T, MPL, false> in_cur, in_nxt;
    if (t < a.ntiles) {
        cur = tile_at(tiles, t);
        load_mixed<T, MPL>(in_cur, groups[cur.group], cur.base);
    }
    if (t + stride < a.ntiles) nxt = tile_at(tiles, t + stride);
    for (; t < a.ntiles; t += stride) {
        const bool has_next = t + stride < a.ntiles;
        TileInfo nxt2 = {0, 0};
        if (t + 2 * stride < a.ntiles) nxt2 = tile_at(tiles, t + 2 * stride);
        if (has_next) load_mixed<T, MPL>(in_nxt, groups[nxt.group], nxt.base);
        const auto &g = groups[cur.group];
        const uint32_t n = (uint32_t)g.n;
        const bool full = cur.base + WAVE * MPL <= n;
        if (g.kind == 3) {
            if (full)
                wtile_eig3<T, PATH, MPL, false, true>(planes_of(cur.group), planes_of, cur.group, a.prm,
                                                      in_cur, n, cur.base, my, qn, qage, refined, nonfinite);
            else
                wtile_eig3<T, PATH, MPL, false, false>(planes_of(cur.group), planes_of, cur.group, a.prm,
                                                       in_cur, n, cur.base, my, qn, qage, refined, nonfinite);
        } else {
            if (full) wtile_eig2_in<T, MPL, true>(g, in_cur, cur.base);
            else wtile_eig2_in<T, MPL, false>(g, in_cur, cur.base);
        }
        cur = nxt;
        nxt = nxt2;
        in_cur = in_nxt;
    }
    final_drain<T, MPL, false>(planes_of, my, qn, refined);
    add_counters(a.prm.counters, refined, nonfinite);
}

__global__ void k_zero_u32(unsigned *p, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0u;
}

}  // namespace ksym
