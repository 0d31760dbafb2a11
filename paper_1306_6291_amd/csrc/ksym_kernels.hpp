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

#include "ksym_device.hpp"

namespace ksym {

enum { PATH_FP32_FIXUP = 0, PATH_FP64_PLAIN = 1, PATH_FP64_FIXUP = 2 };

template <typename T> struct Eig3Ptrs {
    const T *in[6];
    T *lam[3];
    T *D[9];
    T *phi[3];
    T *gap[3];
    uint8_t *flags;
};

struct Eig3Params {
    int64_t n;
    double tau_gap, tau_res, tau_vec, tau_dbl;
    unsigned *counters;   // [0] refined, [1] non-finite; may be null
};

template <typename T> struct Eig3Args {
    Eig3Ptrs<T> p;
    Eig3Params prm;
    const T *aos;   // record input for the array-of-structures kernel
};

template <typename T> struct Out3 {
    T lam[3];
    T D[9];
    T phi[3];
    T gap[3];
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
        for (int i = 0; i < 9; ++i) o.D[i] = (i % 4 == 0) ? T(1) : T(0);
        o.lam[0] = o.lam[1] = o.lam[2] = ain[0];
        o.phi[0] = o.phi[1] = o.phi[2] = T(0);
        o.gap[0] = o.gap[1] = o.gap[2] = T(0);
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
                    o.D[3 * r] = Di[3 * r + 2]; o.D[3 * r + 1] = Di[3 * r]; o.D[3 * r + 2] = Di[3 * r + 1];
                }
                L[0] = ls; L[1] = lm; L[2] = lm;
            } else {         // (lm, ls, lm): columns (1, 3, -2), odd permutation + sign
                for (int r = 0; r < 3; ++r) {
                    o.D[3 * r] = Di[3 * r]; o.D[3 * r + 1] = Di[3 * r + 2]; o.D[3 * r + 2] = -Di[3 * r + 1];
                }
                L[0] = lm; L[1] = ls; L[2] = lm;
            }
            extract_angles<T>(o.D, o.phi);
            for (int k = 0; k < 3; ++k) o.lam[k] = (T)((cu.m + L[k]) * isc);
            o.gap[0] = (T)((L[0] - L[1]) * isc);
            o.gap[1] = (T)((L[0] - L[2]) * isc);
            o.gap[2] = (T)((L[2] - L[1]) * isc);
            o.flag = FLAG_DOUBLE;
        } else {
            // general branch (5.1)-(5.15): v, w with the eigenvalue
            // differences taken from the float64 stage
            const T G12 = (T)cu.g12, G13 = (T)cu.g13, G32 = (T)cu.g32;
            const T e1 = (T)(cu.d1 - cu.mu1), e3 = (T)(cu.d1 - cu.mu3);   // A11 - lam1, A11 - lam3
            const T v = clamp01(Mth<T>::div(A12 * A12 + A13 * A13 + e3 * (e1 + G32), G32 * G13));
            const T w = (v == T(0)) ? T(1) : clamp01(Mth<T>::div(e3 + G32 * v, G12 * v));
            const Rot<T> R = select_angles<T>(A12, A13, A22, A33, A23, G12, G32, v, w);
            build_D(R, o.D);
            angles_of(R, o.phi);
            o.lam[0] = (T)((cu.m + cu.mu1) * isc);
            o.lam[1] = (T)((cu.m + cu.mu2) * isc);
            o.lam[2] = (T)((cu.m + cu.mu3) * isc);
            o.gap[0] = (T)(cu.g12 * isc);
            o.gap[1] = (T)(cu.g13 * isc);
            o.gap[2] = (T)(cu.g32 * isc);
            o.flag = dbl ? FLAG_DOUBLE : FLAG_GENERAL;
            if (PATH != PATH_FP64_PLAIN) {
                const double fro = ::sqrt(a11 * a11 + a22 * a22 + a33 * a33 +
                                          2.0 * (a12 * a12 + a13 * a13 + a23 * a23));
                const double lmax = fmax(__builtin_fabs(cu.m + cu.mu1), __builtin_fabs(cu.m + cu.mu2));
                bool bad = dbl || (split < prm.tau_gap * lmax);
                bad = bad || check_fails<T>(cu, a12, a13, a23, o.D, fro, prm.tau_res, prm.tau_vec);
                o.refine = bad;
                o.lc = (cu.g13 >= cu.g32) ? cu.mu1 : cu.mu2;
            }
        }
    }
    if (!fin) {
        const T nan = T(__builtin_nan(""));
#pragma unroll
        for (int i = 0; i < 9; ++i) o.D[i] = nan;
#pragma unroll
        for (int k = 0; k < 3; ++k) { o.lam[k] = nan; o.phi[k] = nan; o.gap[k] = nan; }
        o.flag = FLAG_NONFINITE;
        o.refine = false;
    }
}

template <typename T>
__device__ __forceinline__ void store3(const Eig3Ptrs<T> &p, int64_t i, const Out3<T> &o) {
#pragma unroll
    for (int k = 0; k < 3; ++k)
        if (p.lam[k]) p.lam[k][i] = o.lam[k];
#pragma unroll
    for (int k = 0; k < 9; ++k)
        if (p.D[k]) p.D[k][i] = o.D[k];
#pragma unroll
    for (int k = 0; k < 3; ++k)
        if (p.phi[k]) p.phi[k][i] = o.phi[k];
#pragma unroll
    for (int k = 0; k < 3; ++k)
        if (p.gap[k]) p.gap[k][i] = o.gap[k];
    if (p.flags) p.flags[i] = (uint8_t)o.flag;
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
    for (int i = 0; i < 9; ++i) o.D[i] = (T)rf.D[i];
    extract_angles<T>(o.D, o.phi);
#pragma unroll
    for (int k = 0; k < 3; ++k) o.lam[k] = (T)((m + rf.lam[k]) * isc);
    o.gap[0] = (T)(fmax(rf.lam[0] - rf.lam[1], 0.0) * isc);
    o.gap[1] = (T)(fmax(rf.lam[0] - rf.lam[2], 0.0) * isc);
    o.gap[2] = (T)(fmax(rf.lam[2] - rf.lam[1], 0.0) * isc);
    o.flag = flag | FLAG_FIXUP;
}

// On-chip queue for one workgroup.
template <typename T, int CAP> struct Queue {
    int n;
    int off[CAP];       // in-tile offset | flag << 24
    T a[6][CAP];
    double lc[CAP];
};

__device__ __forceinline__ unsigned lane_rank(uint64_t mask) {
    return __builtin_amdgcn_mbcnt_hi((unsigned)(mask >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)mask, 0u));
}

// Process one tile of BS*MPL 3x3 matrices starting at `base`.  Block-uniform
// control flow; contains workgroup barriers when PATH != PLAIN or AOS.
template <typename T, int PATH, int BS, int MPL, bool AOS, int CAP>
__device__ __forceinline__ void tile_eig3(const Eig3Ptrs<T> &p, const Eig3Params &prm, const T *aos,
                                          int64_t n, int64_t base, Queue<T, CAP> *q, T *stage,
                                          unsigned &refined, unsigned &nonfinite) {
    constexpr int TILE = BS * MPL;
    const int tid = threadIdx.x;
    T A[MPL][6];
    if constexpr (AOS) {
        // stage the tile's records (TILE x 6 contiguous elements) with 16-byte
        // loads, then each lane picks its own records out of LDS
        constexpr int VEC = 16 / sizeof(T);
        constexpr int NV = TILE * 6 / VEC;
        const int64_t lim = (n - base) * 6;   // valid elements in this tile
        const T *src = aos + base * 6;
        for (int j = tid; j < NV; j += BS) {
            const int64_t e0 = (int64_t)j * VEC;
            if (e0 + VEC <= lim) {
                if constexpr (sizeof(T) == 4) {
                    const float4 v = *reinterpret_cast<const float4 *>(src + e0);
                    *reinterpret_cast<float4 *>(stage + e0) = v;
                } else {
                    const double2 v = *reinterpret_cast<const double2 *>(src + e0);
                    *reinterpret_cast<double2 *>(stage + e0) = v;
                }
            } else {
                for (int t = 0; t < VEC; ++t) stage[e0 + t] = (e0 + t < lim) ? src[e0 + t] : T(0);
            }
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < MPL; ++k)
#pragma unroll
            for (int c = 0; c < 6; ++c) A[k][c] = stage[(k * BS + tid) * 6 + c];
        __syncthreads();
    } else {
#pragma unroll
        for (int k = 0; k < MPL; ++k) {
            const int64_t i = base + k * BS + tid;
#pragma unroll
            for (int c = 0; c < 6; ++c) A[k][c] = (i < n) ? p.in[c][i] : T(0);
        }
    }
#pragma unroll
    for (int k = 0; k < MPL; ++k) {
        const int64_t i = base + k * BS + tid;
        const bool valid = i < n;
        Out3<T> o;
        eig3_one<T, PATH>(A[k], prm, o);
        if (o.flag == FLAG_NONFINITE) nonfinite += valid ? 1u : 0u;
        const bool r = valid && o.refine;
        if (valid && !r) store3(p, i, o);
        if constexpr (PATH != PATH_FP64_PLAIN) {
            const uint64_t mask = __ballot(r);
            if (mask) {
                int off = 0;
                if ((tid & 63) == 0) off = atomicAdd(&q->n, (int)__popcll(mask));
                off = __builtin_amdgcn_readfirstlane(off);
                if (r) {
                    const int pos = off + (int)lane_rank(mask);
                    q->off[pos] = (k * BS + tid) | (o.flag << 24);
#pragma unroll
                    for (int c = 0; c < 6; ++c) q->a[c][pos] = A[k][c];
                    q->lc[pos] = o.lc;
                }
            }
        }
    }
    if constexpr (PATH != PATH_FP64_PLAIN) {
        __syncthreads();
        const int cnt = q->n;
        __syncthreads();
        if (cnt > 0) {
            for (int j = tid; j < cnt; j += BS) {
                const int packed = q->off[j];
                T a[6];
#pragma unroll
                for (int c = 0; c < 6; ++c) a[c] = q->a[c][j];
                Out3<T> o;
                refine_one<T>(a, q->lc[j], packed >> 24, o);
                store3(p, base + (packed & 0xffffff), o);
            }
            if (tid == 0) {
                q->n = 0;
                refined += (unsigned)cnt;
            }
            __syncthreads();
        }
    }
}

template <typename T, int PATH, int BS, int MPL, bool AOS>
__global__ __launch_bounds__(BS) void k_eig3(Eig3Args<T> args) {
    constexpr int TILE = BS * MPL;
    constexpr int CAP = (PATH == PATH_FP64_PLAIN) ? 1 : TILE;
    __shared__ Queue<T, CAP> q;
    __shared__ __align__(16) T stage[AOS ? TILE * 6 : 1];
    if (threadIdx.x == 0) q.n = 0;
    __syncthreads();
    const int64_t n = args.prm.n;
    const int64_t ntiles = (n + TILE - 1) / TILE;
    unsigned refined = 0, nonfinite = 0;
    for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x)
        tile_eig3<T, PATH, BS, MPL, AOS, CAP>(args.p, args.prm, args.aos, n, t * TILE, &q, stage,
                                              refined, nonfinite);
    if (args.prm.counters) {
        if (threadIdx.x == 0 && refined) atomicAdd(&args.prm.counters[0], refined);
        const uint64_t m = __ballot(nonfinite != 0);
        if (m) {
            // sum per wave with a shuffle-free scalar loop over the few lanes
            unsigned s = nonfinite;
            for (int d = 32; d >= 1; d >>= 1) s += __shfl_xor(s, d);
            if ((threadIdx.x & 63) == 0) atomicAdd(&args.prm.counters[1], s);
        }
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
    Eig3Ptrs<T> p3;   // for kind 2: in[0..2], lam[0..1], D[0..3], phi[0], flags
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
    __shared__ Queue<T, TILE> q;
    if (threadIdx.x == 0) q.n = 0;
    __syncthreads();
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
            constexpr int PATH = (sizeof(T) == 4) ? PATH_FP32_FIXUP : PATH_FP64_FIXUP;
            tile_eig3<T, PATH, BS, MPL, false, TILE>(g.p3, a.prm, nullptr, g.n, base, &q, nullptr,
                                                     refined, nonfinite);
        } else {
            Eig2Ptrs<T> p2;
            for (int c = 0; c < 3; ++c) p2.in[c] = g.p3.in[c];
            p2.lam[0] = g.p3.lam[0]; p2.lam[1] = g.p3.lam[1];
            for (int c = 0; c < 4; ++c) p2.D[c] = g.p3.D[c];
            p2.phi = g.p3.phi[0];
            p2.flags = g.p3.flags;
            tile_eig2<T, BS, MPL>(p2, g.n, base);
        }
    }
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
