// Tile processors and __global__ kernels for the ksym C ABI (gfx950, wave64).
//
// Work decomposition: a workgroup of BS lanes owns tiles of BS * MPL matrices
// (MPL = matrices per lane) and walks them grid-stride.  Within a tile, matrix
// k*BS + lane belongs to `lane`, so every plane load and store of a wave is one
// contiguous 64-element run.
//
// Refinement routing (3x3 float32 and float64 check paths): a lane whose
// matrix fails the float64 check does not store; it appends the matrix to an
// on-chip queue with one LDS atomic per wavefront (ballot + popcount for the
// wave's total, mbcnt for the lane's rank).  After the tile, the workgroup's
// lanes drain the queue -- entry j to lane j, so the refinement runs on dense
// wavefronts -- and store those matrices' outputs.  Nothing is re-read from
// HBM, and every output element is written exactly once.
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

struct Eig3Params {
    int64_t n;
    double tau_gap, tau_res, tau_vec, tau_dbl;
    unsigned *counters;   // [0] refined, [1] non-finite; may be null
    int32_t zero;         // always 0; see store_tile3
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
            const Rot<T> R = select_angles<T>(A12, A13, A22, A33, A23, T(0), (T)(ls - lm), s, T(1));
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
            // general branch (5.1)-(5.15): v, w with the eigenvalue
            // differences taken from the float64 stage
            const T G12 = (T)cu.g12, G13 = (T)cu.g13, G32 = (T)cu.g32;
            const T e1 = (T)(cu.d1 - cu.mu1), e3 = (T)(cu.d1 - cu.mu3);   // A11 - lam1, A11 - lam3
            const T v = clamp01(Mth<T>::div(A12 * A12 + A13 * A13 + e3 * (e1 + G32), G32 * G13));
            const T w = (v == T(0)) ? T(1) : clamp01(Mth<T>::div(e3 + G32 * v, G12 * v));
            const Rot<T> R = select_angles<T>(A12, A13, A22, A33, A23, G12, G32, v, w);
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

// Per-workgroup staging of a tile's outputs in LDS: the main pass and the
// refinement both write here, then the tile leaves with one coalesced store per
// plane, so every output element is written to HBM exactly once.
template <typename T, int TILE> struct Stage3 {
    T v[NOUT3][TILE];
    uint8_t flag[TILE];
};

template <typename T, int TILE>
__device__ __forceinline__ void stage_put(Stage3<T, TILE> *st, int slot, const Out3<T> &o) {
#pragma unroll
    for (int k = 0; k < NOUT3; ++k) st->v[k][slot] = o.v[k];
    st->flag[slot] = (uint8_t)o.flag;
}

// The float32 path for one matrix, written for a small register footprint:
// everything after the float64 cubic stage is float32, results go to the LDS
// staging slot as soon as they exist (eigenvalues and gaps first, then the
// angles, then D after the check), and the a-posteriori check runs in float32
// on B = A - m I.  Sets `refine` (and the isolated eigenvalue lc for the
// refinement, a float64 deviation in scaled units) and returns the flag.
template <int TILE>
__device__ __forceinline__ int eig3_f32(const float ain[6], const Eig3Params &prm,
                                        Stage3<float, TILE> *st, int slot, bool &refine, double &lc) {
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
    for (int c = 0; c < 6; ++c) a[c] = fin ? (double)ain[c] * sc : 0.0;
    const Cubic cu = cubic_stage_fast(a[0], a[1], a[2], a[3], a[4], a[5]);
    refine = false;
    lc = 0.0;
    int flag;
    if (cu.triple || !fin) {
        // §5, p = 0: A = lam I, D = I, angles 0 (non-finite input: all NaN)
        const float nan = __builtin_nanf("");
        const float lam = fin ? (float)(cu.m * isc) : nan;
        st->v[O_LAM][slot] = lam; st->v[O_LAM + 1][slot] = lam; st->v[O_LAM + 2][slot] = lam;
#pragma unroll
        for (int i = 0; i < 9; ++i) st->v[O_D + i][slot] = fin ? ((i % 4 == 0) ? 1.0f : 0.0f) : nan;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            st->v[O_PHI + k][slot] = fin ? 0.0f : nan;
            st->v[O_GAP + k][slot] = fin ? 0.0f : nan;
        }
        flag = fin ? FLAG_TRIPLE : FLAG_NONFINITE;
        st->flag[slot] = (uint8_t)flag;
        return flag;
    }
    st->v[O_LAM][slot] = (float)((cu.m + cu.mu1) * isc);
    st->v[O_LAM + 1][slot] = (float)((cu.m + cu.mu2) * isc);
    st->v[O_LAM + 2][slot] = (float)((cu.m + cu.mu3) * isc);
    st->v[O_GAP][slot] = (float)(cu.g12 * isc);
    st->v[O_GAP + 1][slot] = (float)(cu.g13 * isc);
    st->v[O_GAP + 2][slot] = (float)(cu.g32 * isc);
    const double split = fmin(cu.g13, cu.g32);
    const bool dbl = (cu.g13 * cu.g32 == 0.0) || split < prm.tau_dbl * cu.sp;
    const double lmax = fmax(__builtin_fabs(cu.m + cu.mu1), __builtin_fabs(cu.m + cu.mu2));
    bool bad = dbl || (split < prm.tau_gap * lmax);
    lc = (cu.g13 >= cu.g32) ? cu.mu1 : cu.mu2;
    // float32 operands of the angle solve and the check (scaled units)
    const float A12 = (float)a[3], A13 = (float)a[4], A23 = (float)a[5];
    const float A22 = (float)a[1], A33 = (float)a[2];
    const float G12 = (float)cu.g12, G13 = (float)cu.g13, G32 = (float)cu.g32;
    const float e1 = (float)(cu.d1 - cu.mu1), e3 = (float)(cu.d1 - cu.mu3);
    const float d1 = (float)cu.d1, d2 = (float)cu.d2, d3 = (float)cu.d3;
    const float m1 = (float)cu.mu1, m2 = (float)cu.mu2, m3 = (float)cu.mu3;
    const float fro = __builtin_sqrtf((float)(a[0] * a[0] + a[1] * a[1] + a[2] * a[2] +
                                              2.0 * (a[3] * a[3] + a[4] * a[4] + a[5] * a[5])));
    // general branch (5.1)-(5.15)
    const float v = clamp01(Mth<float>::div(A12 * A12 + A13 * A13 + e3 * (e1 + G32), G32 * G13));
    const float w = (v == 0.0f) ? 1.0f : clamp01(Mth<float>::div(e3 + G32 * v, G12 * v));
    const Rot<float> R = select_angles<float>(A12, A13, A22, A33, A23, G12, G32, v, w);
    float phi[3];
    angles_of(R, phi);
#pragma unroll
    for (int k = 0; k < 3; ++k) st->v[O_PHI + k][slot] = phi[k];
    float D[9];
    build_D(R, D);
    bad = bad || check_fails<float>(d1, d2, d3, A12, A13, A23, D, m1, m2, m3, G12, G13, G32,
                                    (float)prm.tau_res * fro, (float)prm.tau_vec);
#pragma unroll
    for (int i = 0; i < 9; ++i) st->v[O_D + i][slot] = D[i];
    flag = dbl ? FLAG_DOUBLE : FLAG_GENERAL;
    st->flag[slot] = (uint8_t)flag;
    refine = bad;
    return flag;
}

// Output plane pointers read from the kernel-argument segment with a
// plane-dependent offset: the store loop fetches each pointer with one scalar
// load when it needs it instead of holding all of them in registers.
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
    const Eig3Ptrs<T> *p;
    __device__ __forceinline__ T *out(int k) const { return p->out[k]; }
    __device__ __forceinline__ uint8_t *flags(int salt = 0) const { return (&p->flags)[salt]; }
};

// Store a staged tile.  The plane pointers are fetched here, for this tile: the
// plane index is offset by salt = tile * zero, which is 0 at run time but not
// known to the compiler, so the fully unrolled loop issues all pointer loads
// together without hoisting them out of the tile loop (where they would pin
// 38 scalar registers for the whole kernel).
template <typename T, int BS, int MPL, int TILE, typename Planes>
__device__ __forceinline__ void store_tile3(const Planes &pl, const Stage3<T, TILE> *st, int64_t n,
                                            int64_t base, int salt) {
    const int tid = threadIdx.x;
    T *dst[NOUT3];
#pragma unroll
    for (int k = 0; k < NOUT3; ++k) dst[k] = pl.out(k + salt);
    uint8_t *fl = pl.flags(salt);
#pragma unroll
    for (int m = 0; m < MPL; ++m) {
        const int64_t i = base + m * BS + tid;
        T val[NOUT3];   // all LDS reads first, then the stores
#pragma unroll
        for (int k = 0; k < NOUT3; ++k) val[k] = st->v[k][m * BS + tid];
        if (i < n) {
#pragma unroll
            for (int k = 0; k < NOUT3; ++k)
                if (dst[k]) dst[k][i] = val[k];
        }
    }
    if (fl) {
#pragma unroll
        for (int m = 0; m < MPL; ++m) {
            const int64_t i = base + m * BS + tid;
            if (i < n) fl[i] = st->flag[m * BS + tid];
        }
    }
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

// On-chip refinement queue of one workgroup.  Entries accumulate over tiles;
// the queue is drained when it holds at least one entry per lane, so the
// float64 refinement always runs on full wavefronts.
template <typename T, int CAP> struct Queue {
    int n;
    int64_t idx[CAP];   // matrix index within its group
    int grp[CAP];       // group (mixed batches; 0 otherwise) | flag << 24
    T a[6][CAP];
    double lc[CAP];
};

__device__ __forceinline__ unsigned lane_rank(uint64_t mask) {
    return __builtin_amdgcn_mbcnt_hi((unsigned)(mask >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)mask, 0u));
}

// Inputs of one tile held in registers.  SoA: each lane's MPL matrices.
// AoS: the lane's share of the tile's contiguous records as 16-byte vectors,
// transposed through LDS when the tile is processed.
template <typename T, int BS, int MPL, bool AOS> struct TileIn {
    static constexpr int VEC = 16 / sizeof(T);
    static constexpr int NV = BS * MPL * 6 / VEC;          // 16-byte vectors per tile
    static constexpr int NVL = (NV + BS - 1) / BS;         // per lane
    T a[AOS ? 1 : MPL][6];
    T v[AOS ? NVL : 1][AOS ? VEC : 1];
};

template <typename T, int BS, int MPL, bool AOS>
__device__ __forceinline__ void load_tile3(TileIn<T, BS, MPL, AOS> &in, const T *const *planes,
                                           const T *aos, int64_t n, int64_t base) {
    const int tid = threadIdx.x;
    if constexpr (AOS) {
        using TI = TileIn<T, BS, MPL, AOS>;
        constexpr int VEC = TI::VEC;
        const int64_t lim = (n - base) * 6;   // valid elements in this tile
        const T *src = aos + base * 6;
#pragma unroll
        for (int u = 0; u < TI::NVL; ++u) {
            const int j = u * BS + tid;
            const int64_t e0 = (int64_t)j * VEC;
            if (j < TI::NV && e0 + VEC <= lim) {
                if constexpr (sizeof(T) == 4) {
                    const float4 x = *reinterpret_cast<const float4 *>(src + e0);
                    in.v[u][0] = x.x; in.v[u][1] = x.y; in.v[u][2] = x.z; in.v[u][3] = x.w;
                } else {
                    const double2 x = *reinterpret_cast<const double2 *>(src + e0);
                    in.v[u][0] = x.x; in.v[u][1] = x.y;
                }
            } else {
#pragma unroll
                for (int t = 0; t < VEC; ++t)
                    in.v[u][t] = (j < TI::NV && e0 + t < lim) ? src[e0 + t] : T(0);
            }
        }
    } else {
#pragma unroll
        for (int k = 0; k < MPL; ++k) {
            const int64_t i = base + k * BS + tid;
#pragma unroll
            for (int c = 0; c < 6; ++c) in.a[k][c] = (i < n) ? planes[c][i] : T(0);
        }
    }
}

// Write one matrix's outputs (a refined result) to the output planes.
template <typename T, typename Planes>
__device__ __forceinline__ void write_out3(const Planes &pl, int64_t i, const Out3<T> &o) {
#pragma nounroll
    for (int k = 0; k < NOUT3; ++k) {
        T *dst = pl.out(k);
        if (dst) dst[i] = o.v[k];
    }
    uint8_t *fl = pl.flags();
    if (fl) fl[i] = (uint8_t)o.flag;
}

// Drain the first `cnt` queue entries: entry j goes to lane j (mod BS), each
// result is written straight to its output planes.  The tile store that wrote
// the provisional values happened before the workgroup barrier (with its
// release fence) that precedes every call.
template <typename T, int BS, int CAP, typename PlanesOf>
__device__ __forceinline__ void drain_queue(Queue<T, CAP> *q, int cnt, const PlanesOf &planes_of) {
    for (int j = threadIdx.x; j < cnt; j += BS) {
        T a[6];
#pragma unroll
        for (int c = 0; c < 6; ++c) a[c] = q->a[c][j];
        const int g = q->grp[j];
        Out3<T> o;
        refine_one<T>(a, q->lc[j], g >> 24, o);
        write_out3(planes_of(g & 0xffffff), q->idx[j], o);
    }
}

// Workgroup-shared memory of the 3x3 kernels.
template <typename T, int BS, int TILE, bool QUEUE, bool AOS> struct Smem3 {
    Queue<T, QUEUE ? BS + TILE : 1> q;
    Stage3<T, TILE> st;
    __align__(16) T rec[AOS ? TILE * 6 : 1];
};

// Process one tile of BS*MPL 3x3 matrices starting at `base` from inputs
// already in registers, store it, and drain the refinement queue when it holds
// at least BS entries.  Block-uniform control flow.  The staging slots are
// written and read only by their own lane, so the tile store needs no barrier;
// two barriers per tile make the queue length consistent, two more surround a
// drain.  The AoS record buffer is last read before the first barrier (an
// extra barrier closes the tile when there is no queue).
template <typename T, int PATH, int BS, int MPL, bool AOS, typename Planes, typename PlanesOf>
__device__ __forceinline__ void tile_eig3(const Planes &pl, const PlanesOf &planes_of, int grp,
                                          const Eig3Params &prm, TileIn<T, BS, MPL, AOS> &in,
                                          int64_t n, int64_t base,
                                          Smem3<T, BS, BS * MPL, PATH != PATH_FP64_PLAIN, AOS> *sm,
                                          unsigned &refined, unsigned &nonfinite) {
    constexpr int TILE = BS * MPL;
    const int tid = threadIdx.x;
    if constexpr (AOS) {
        using TI = TileIn<T, BS, MPL, AOS>;
#pragma unroll
        for (int u = 0; u < TI::NVL; ++u) {
            const int j = u * BS + tid;
            if (j < TI::NV) {
#pragma unroll
                for (int t = 0; t < TI::VEC; ++t) sm->rec[j * TI::VEC + t] = in.v[u][t];
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int k = 0; k < MPL; ++k) {
        const int slot = k * BS + tid;
        const bool valid = base + slot < n;
        T A[6];
        if constexpr (AOS) {
#pragma unroll
            for (int c = 0; c < 6; ++c) A[c] = sm->rec[slot * 6 + c];
        } else {
#pragma unroll
            for (int c = 0; c < 6; ++c) A[c] = in.a[k][c];
        }
        bool refine;
        double lc;
        int flag;
        if constexpr (PATH == PATH_FP32_FIXUP) {
            flag = eig3_f32<TILE>(A, prm, &sm->st, slot, refine, lc);
        } else {
            Out3<T> o;
            eig3_one<T, PATH>(A, prm, o);
            stage_put(&sm->st, slot, o);
            refine = o.refine;
            lc = o.lc;
            flag = o.flag;
        }
        if (flag == FLAG_NONFINITE) nonfinite += valid ? 1u : 0u;
        if constexpr (PATH != PATH_FP64_PLAIN) {
            const bool r = valid && refine;
            const uint64_t mask = __ballot(r);
            if (mask) {
                int off = 0;
                if ((tid & 63) == 0) off = atomicAdd(&sm->q.n, (int)__popcll(mask));
                off = __builtin_amdgcn_readfirstlane(off);
                if (r) {
                    const int pos = off + (int)lane_rank(mask);
                    sm->q.idx[pos] = base + slot;
                    sm->q.grp[pos] = grp | (flag << 24);
#pragma unroll
                    for (int c = 0; c < 6; ++c) sm->q.a[c][pos] = A[c];
                    sm->q.lc[pos] = lc;
                }
            }
        }
    }
    store_tile3<T, BS, MPL, TILE>(pl, &sm->st, n, base, (int)(base * prm.zero));
    if constexpr (PATH != PATH_FP64_PLAIN) {
        __syncthreads();
        const int cnt = sm->q.n;
        __syncthreads();
        if (cnt >= BS) {
            // drain whole rounds only, then move the remainder to the front
            const int nfull = cnt - cnt % BS;
            drain_queue<T, BS>(&sm->q, nfull, planes_of);
            refined += (tid == 0) ? (unsigned)nfull : 0u;
            __syncthreads();
            const int rest = cnt - nfull;   // < BS
            if (tid < rest) {
                const int j = nfull + tid;
                const int64_t ix = sm->q.idx[j];
                const int gf = sm->q.grp[j];
                const double l = sm->q.lc[j];
                T a[6];
#pragma unroll
                for (int c = 0; c < 6; ++c) a[c] = sm->q.a[c][j];
                sm->q.idx[tid] = ix;
                sm->q.grp[tid] = gf;
                sm->q.lc[tid] = l;
#pragma unroll
                for (int c = 0; c < 6; ++c) sm->q.a[c][tid] = a[c];
            }
            if (tid == 0) sm->q.n = rest;
            __syncthreads();
        }
    } else if constexpr (AOS) {
        __syncthreads();
    }
}

// Drain what is left in the queue at the end of a workgroup's work.
template <typename T, int PATH, int BS, int TILE, bool AOS, typename PlanesOf>
__device__ __forceinline__ void final_drain(const PlanesOf &planes_of,
                                            Smem3<T, BS, TILE, PATH != PATH_FP64_PLAIN, AOS> *sm,
                                            unsigned &refined) {
    if constexpr (PATH != PATH_FP64_PLAIN) {
        __syncthreads();
        const int cnt = sm->q.n;
        if (cnt > 0) {
            drain_queue<T, BS>(&sm->q, cnt, planes_of);
            refined += (threadIdx.x == 0) ? (unsigned)cnt : 0u;
        }
    }
}

template <typename T, int PATH, int BS, int MPL, bool AOS>
__global__ __launch_bounds__(BS) void k_eig3(Eig3Args<T> args) {
    constexpr int TILE = BS * MPL;
    __shared__ Smem3<T, BS, TILE, PATH != PATH_FP64_PLAIN, AOS> sm;
    if (threadIdx.x == 0) sm.q.n = 0;
    __syncthreads();
    const int64_t n = args.prm.n;
    const int64_t ntiles = (n + TILE - 1) / TILE;
    KernargPlanes<T> pl;
    pl.out_off = (uint32_t)(offsetof(Eig3Args<T>, p) + offsetof(Eig3Ptrs<T>, out));
    pl.flags_off = (uint32_t)(offsetof(Eig3Args<T>, p) + offsetof(Eig3Ptrs<T>, flags));
    auto planes_of = [&](int) { return pl; };
    unsigned refined = 0, nonfinite = 0;
    TileIn<T, BS, MPL, AOS> cur, nxt;
    int64_t t = blockIdx.x;
    if (t < ntiles) load_tile3<T, BS, MPL, AOS>(cur, args.p.in, args.aos, n, t * TILE);
    for (; t < ntiles; t += gridDim.x) {
        const int64_t tn = t + gridDim.x;
        if (tn < ntiles) load_tile3<T, BS, MPL, AOS>(nxt, args.p.in, args.aos, n, tn * TILE);
        tile_eig3<T, PATH, BS, MPL, AOS>(pl, planes_of, 0, args.prm, cur, n, t * TILE, &sm, refined,
                                         nonfinite);
        cur = nxt;
    }
    final_drain<T, PATH, BS, TILE, AOS>(planes_of, &sm, refined);
    if (args.prm.counters) {
        if (threadIdx.x == 0 && refined) atomicAdd(&args.prm.counters[0], refined);
        unsigned s = nonfinite;
        for (int d = 32; d >= 1; d >>= 1) s += __shfl_xor(s, d);
        if ((threadIdx.x & 63) == 0 && s) atomicAdd(&args.prm.counters[1], s);
    }
}

// ------------------------------------------------------------- 2x2 ---------
template <typename T> struct Eig2Ptrs {
    const T *in[3];
    T *lam[2];
    T *D[4];
    T *phi;
    uint8_t *flags;
};

template <typename T, int BS, int MPL>
__device__ __forceinline__ void tile_eig2(const Eig2Ptrs<T> &p, int64_t n, int64_t base) {
    const int tid = threadIdx.x;
    T A[MPL][3];
#pragma unroll
    for (int k = 0; k < MPL; ++k) {
        const int64_t i = base + k * BS + tid;
#pragma unroll
        for (int c = 0; c < 3; ++c) A[k][c] = (i < n) ? p.in[c][i] : T(0);
    }
#pragma unroll
    for (int k = 0; k < MPL; ++k) {
        const int64_t i = base + k * BS + tid;
        if (i >= n) continue;
        const bool fin = finite(A[k][0]) && finite(A[k][1]) && finite(A[k][2]);
        // exact power-of-two scaling keeps d^2 + 4 A12^2 in range
        double amax = fmax(fmax(__builtin_fabs((double)A[k][0]), __builtin_fabs((double)A[k][1])),
                           __builtin_fabs((double)A[k][2]));
        const int ex = fin ? scale_exponent(amax) : 0;
        const T sc = (T)pow2(-ex), isc = (T)pow2(ex);
        Eig2<T> e = eig2_one<T>(A[k][0] * sc, A[k][1] * sc, A[k][2] * sc);
        e.l1 *= isc;
        e.l2 *= isc;
        if (!fin) {
            const T nan = T(__builtin_nan(""));
            e.l1 = e.l2 = e.c = e.s = e.phi = nan;
        }
        if (p.lam[0]) p.lam[0][i] = e.l1;
        if (p.lam[1]) p.lam[1][i] = e.l2;
        if (p.D[0]) p.D[0][i] = e.c;
        if (p.D[1]) p.D[1][i] = -e.s;
        if (p.D[2]) p.D[2][i] = e.s;
        if (p.D[3]) p.D[3][i] = e.c;
        if (p.phi) p.phi[i] = e.phi;
        if (p.flags) p.flags[i] = fin ? (uint8_t)0 : (uint8_t)FLAG_NONFINITE;
    }
}

template <typename T, int BS, int MPL>
__global__ __launch_bounds__(BS) void k_eig2(Eig2Ptrs<T> p, int64_t n) {
    constexpr int TILE = BS * MPL;
    const int64_t ntiles = (n + TILE - 1) / TILE;
    for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) tile_eig2<T, BS, MPL>(p, n, t * TILE);
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

template <typename T, int BS, int MPL>
__global__ __launch_bounds__(BS) void k_eig3_bwd(BwdPtrs<T> p, int64_t n, double eps_rel) {
    constexpr int TILE = BS * MPL;
    const int64_t ntiles = (n + TILE - 1) / TILE;
    const bool has_gap = p.gap[0] && p.gap[1] && p.gap[2];
    const bool has_gl = p.glam[0] != nullptr;
    const bool has_gd = p.gD[0] != nullptr;
    for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
#pragma unroll
        for (int k = 0; k < MPL; ++k) {
            const int64_t i = t * TILE + k * BS + threadIdx.x;
            if (i >= n) continue;
            T L[3], D[9], gl[3], gD[9], gA[6];
#pragma unroll
            for (int c = 0; c < 3; ++c) L[c] = p.lam[c][i];
#pragma unroll
            for (int c = 0; c < 9; ++c) D[c] = p.D[c][i];
#pragma unroll
            for (int c = 0; c < 3; ++c) gl[c] = has_gl ? p.glam[c][i] : T(0);
#pragma unroll
            for (int c = 0; c < 9; ++c) gD[c] = has_gd ? p.gD[c][i] : T(0);
            T g12, g13, g32;
            if (has_gap) {
                g12 = p.gap[0][i]; g13 = p.gap[1][i]; g32 = p.gap[2][i];
            } else {
                // differences of the stored eigenvalues, exact in float64
                g12 = (T)((double)L[0] - (double)L[1]);
                g13 = (T)((double)L[0] - (double)L[2]);
                g32 = (T)((double)L[2] - (double)L[1]);
            }
            const T eps = (T)eps_rel * Mth<T>::sqrt(L[0] * L[0] + L[1] * L[1] + L[2] * L[2]);
            adjoint3<T>(D, gl, gD, g12, g13, g32, eps * eps, gA);
#pragma unroll
            for (int c = 0; c < 6; ++c) p.gA[c][i] = gA[c];
        }
    }
}

// ------------------------------------------------ mixed persistent batch ---
template <typename T> struct GroupDesc {
    int64_t n;
    int32_t kind;
    int32_t pad;
    Eig3Ptrs<T> p3;   // kind 2 uses in[0..2] and out[O_LAM..+1], out[O_D..+3], out[O_PHI], flags
};

template <typename T> struct MixedArgs {
    const GroupDesc<T> *groups;
    const int64_t *tile_begin;   // ngroups + 1 prefix sums of tiles
    int32_t ngroups;
    int64_t ntiles;
    Eig3Params prm;              // thresholds and counters (prm.n unused)
};

template <typename T, int BS, int MPL>
__global__ __launch_bounds__(BS) void k_mixed(MixedArgs<T> a) {
    constexpr int TILE = BS * MPL;
    constexpr int PATH = (sizeof(T) == 4) ? PATH_FP32_FIXUP : PATH_FP64_FIXUP;
    __shared__ Smem3<T, BS, TILE, true, false> sm;
    if (threadIdx.x == 0) sm.q.n = 0;
    __syncthreads();
    auto planes_of = [&](int g) { return TablePlanes<T>{&a.groups[g].p3}; };
    unsigned refined = 0, nonfinite = 0;
    for (int64_t t = blockIdx.x; t < a.ntiles; t += gridDim.x) {
        // binary search: last g with tile_begin[g] <= t (block-uniform)
        int lo = 0, hi = a.ngroups - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (a.tile_begin[mid] <= t) lo = mid; else hi = mid - 1;
        }
        const GroupDesc<T> &g = a.groups[lo];
        const int64_t base = (t - a.tile_begin[lo]) * TILE;
        if (g.kind == 3) {
            TileIn<T, BS, MPL, false> in;
            load_tile3<T, BS, MPL, false>(in, g.p3.in, nullptr, g.n, base);
            tile_eig3<T, PATH, BS, MPL, false>(planes_of(lo), planes_of, lo, a.prm, in, g.n, base, &sm,
                                               refined, nonfinite);
        } else {
            Eig2Ptrs<T> p2;
            for (int c = 0; c < 3; ++c) p2.in[c] = g.p3.in[c];
            p2.lam[0] = g.p3.out[O_LAM]; p2.lam[1] = g.p3.out[O_LAM + 1];
            for (int c = 0; c < 4; ++c) p2.D[c] = g.p3.out[O_D + c];
            p2.phi = g.p3.out[O_PHI];
            p2.flags = g.p3.flags;
            tile_eig2<T, BS, MPL>(p2, g.n, base);
        }
    }
    final_drain<T, PATH, BS, TILE, false>(planes_of, &sm, refined);
    if (a.prm.counters) {
        if (threadIdx.x == 0 && refined) atomicAdd(&a.prm.counters[0], refined);
        unsigned s = nonfinite;
        for (int d = 32; d >= 1; d >>= 1) s += __shfl_xor(s, d);
        if ((threadIdx.x & 63) == 0 && s) atomicAdd(&a.prm.counters[1], s);
    }
}

__global__ void k_zero_u32(unsigned *p, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0u;
}

}  // namespace ksym
