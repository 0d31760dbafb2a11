// C ABI of the ksym library (declared in include/ksym.h): argument checks,
// launch-shape selection, kernel dispatch, plans and graph capture.
#include <hip/hip_runtime.h>

#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/ksym.h"
#include "ksym_kernels.hpp"

using namespace ksym;

namespace {

thread_local std::string g_err;

ksym_status fail(ksym_status s, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return s;
}

ksym_status hip_fail(hipError_t e, const char *what) {
    return fail(KSYM_E_HIP, "%s: %s (%d)", what, hipGetErrorString(e), (int)e);
}

bool aligned(const void *p, size_t a) { return ((uintptr_t)p % a) == 0; }

// per-device compute-unit count, cached after the first query
std::atomic<int> g_cu[64];

ksym_status cu_count(int *out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= 64) return fail(KSYM_E_HIP, "device index %d out of range", dev);
    int c = g_cu[dev].load(std::memory_order_relaxed);
    if (c <= 0) {
        e = hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev);
        if (e != hipSuccess) return hip_fail(e, "hipDeviceGetAttribute");
        if (c <= 0) c = 256;
        g_cu[dev].store(c, std::memory_order_relaxed);
    }
    *out = c;
    return KSYM_OK;
}

template <typename... Args>
hipError_t launch(void (*k)(Args...), dim3 grid, dim3 block, hipStream_t s, Args... args) {
    void *argv[] = {(void *)&args...};
    return hipLaunchKernel((const void *)k, grid, block, argv, 0, s);
}

struct Shape {
    int block, mpl, grid_mult;
};

ksym_status resolve_opts(ksym_dtype dt, const ksym_opts *in, ksym_opts *out) {
    ksym_opts_default(dt, out);
    if (!in) return KSYM_OK;
    ksym_opts o = *in;
    if (o.path == KSYM_PATH_DEFAULT) o.path = out->path;
    if (o.block == 0) o.block = out->block;
    if (o.mats_per_lane == 0) o.mats_per_lane = out->mats_per_lane;
    if (o.grid_mult == 0) o.grid_mult = out->grid_mult;
    if (o.tau_gap < 0) o.tau_gap = out->tau_gap;
    if (o.tau_res < 0) o.tau_res = out->tau_res;
    if (o.tau_vec < 0) o.tau_vec = out->tau_vec;
    if (o.tau_dbl < 0) o.tau_dbl = out->tau_dbl;
    if (o.drain_tiles < 0) o.drain_tiles = out->drain_tiles;
    if (o.block != 64 && o.block != 128 && o.block != 256 && o.block != 512 && o.block != 1024)
        return fail(KSYM_E_ARG, "block must be 64, 128, 256, 512 or 1024 (got %d)", o.block);
    if (o.mats_per_lane != 1 && o.mats_per_lane != 2 && o.mats_per_lane != 4)
        return fail(KSYM_E_ARG, "mats_per_lane must be 1, 2 or 4 (got %d)", o.mats_per_lane);
    if (o.grid_mult < 1 || o.grid_mult > KSYM_GRID_MULT_MAX)
        return fail(KSYM_E_ARG, "grid_mult must be in 1..%d (got %d)", KSYM_GRID_MULT_MAX, o.grid_mult);
    if (o.drain_tiles > (1 << 20)) return fail(KSYM_E_ARG, "drain_tiles must be in 0..2^20");
    if (!(o.tau_res > 0) || !(o.tau_dbl >= 0) || !(o.tau_gap >= 0) || !(o.tau_vec >= 0))
        return fail(KSYM_E_ARG, "thresholds must be finite and non-negative (tau_res > 0)");
    *out = o;
    return KSYM_OK;
}

ksym_status grid_for(int64_t n, int tile, int grid_mult, int *grid) {
    int cus = 0;
    ksym_status s = cu_count(&cus);
    if (s != KSYM_OK) return s;
    const int64_t tiles = (n + tile - 1) / tile;
    int64_t g = (int64_t)grid_mult * cus;
    if (g > tiles) g = tiles;
    if (g < 1) g = 1;
    *grid = (int)g;
    return KSYM_OK;
}

// ------------------------------------------------------ kernel tables -----
template <typename T, int PATH, bool AOS> using Eig3K = void (*)(Eig3Args<T>);

#define KSYM_E3(T, P, A, B, M) \
    if (bs == B && mpl == M) return grad ? &k_eig3<T, P, B, M, A, true> : &k_eig3<T, P, B, M, A, false>;
#define KSYM_E3N(T, P, A, B, M) \
    if (bs == B && mpl == M) return grad ? nullptr : &k_eig3<T, P, B, M, A, false>;

// grad: the variant for differentiated calls (tau_vec > 0), compiled for a
// subset of the shapes (KSYM_E3N: plain variant only)
template <typename T, int PATH, bool AOS> Eig3K<T, PATH, AOS> pick_eig3(int bs, int mpl, bool grad);

// eigenvalues-only kernel (float32 SoA), the same launch shapes as k_eig3<float>
using LamK = void (*)(Eig3Args<float>);
LamK pick_eig3_lam(int bs, int mpl) {
#define KSYM_L(B, M) \
    if (bs == B && mpl == M) return &k_eig3_lam<B, M>;
    KSYM_L(64, 1) KSYM_L(64, 2) KSYM_L(128, 1) KSYM_L(128, 2) KSYM_L(256, 1) KSYM_L(256, 2) KSYM_L(512, 1)
    KSYM_L(512, 2)
#undef KSYM_L
    return nullptr;
}

// true when none of the k planes of an output array is requested
bool none_requested(void *const *planes, int k) {
    if (!planes) return true;
    for (int c = 0; c < k; ++c)
        if (planes[c]) return false;
    return true;
}

template <> Eig3K<float, PATH_FP32_FIXUP, false> pick_eig3<float, PATH_FP32_FIXUP, false>(int bs, int mpl, bool grad) {
    KSYM_E3(float, PATH_FP32_FIXUP, false, 64, 1)
    KSYM_E3N(float, PATH_FP32_FIXUP, false, 64, 2)
    KSYM_E3(float, PATH_FP32_FIXUP, false, 128, 1)
    KSYM_E3N(float, PATH_FP32_FIXUP, false, 128, 2)
    KSYM_E3(float, PATH_FP32_FIXUP, false, 256, 1)
    KSYM_E3(float, PATH_FP32_FIXUP, false, 256, 2)
    KSYM_E3(float, PATH_FP32_FIXUP, false, 512, 1)
    KSYM_E3N(float, PATH_FP32_FIXUP, false, 512, 2)
    return nullptr;
}
template <> Eig3K<float, PATH_FP32_FIXUP, true> pick_eig3<float, PATH_FP32_FIXUP, true>(int bs, int mpl, bool grad) {
    KSYM_E3N(float, PATH_FP32_FIXUP, true, 64, 1)
    KSYM_E3(float, PATH_FP32_FIXUP, true, 128, 1)
    KSYM_E3(float, PATH_FP32_FIXUP, true, 256, 1)
    KSYM_E3(float, PATH_FP32_FIXUP, true, 256, 2)
    KSYM_E3(float, PATH_FP32_FIXUP, true, 512, 1)
    return nullptr;
}
template <> Eig3K<double, PATH_FP64_PLAIN, false> pick_eig3<double, PATH_FP64_PLAIN, false>(int bs, int mpl, bool grad) {
    KSYM_E3N(double, PATH_FP64_PLAIN, false, 64, 1)
    KSYM_E3N(double, PATH_FP64_PLAIN, false, 128, 1)
    KSYM_E3N(double, PATH_FP64_PLAIN, false, 256, 1)
    KSYM_E3N(double, PATH_FP64_PLAIN, false, 256, 2)
    return nullptr;
}
template <> Eig3K<double, PATH_FP64_PLAIN, true> pick_eig3<double, PATH_FP64_PLAIN, true>(int bs, int mpl, bool grad) {
    KSYM_E3N(double, PATH_FP64_PLAIN, true, 256, 1)
    return nullptr;
}
template <> Eig3K<double, PATH_FP64_FIXUP, false> pick_eig3<double, PATH_FP64_FIXUP, false>(int bs, int mpl, bool grad) {
    KSYM_E3N(double, PATH_FP64_FIXUP, false, 64, 1)
    KSYM_E3N(double, PATH_FP64_FIXUP, false, 128, 1)
    KSYM_E3(double, PATH_FP64_FIXUP, false, 256, 1)
    KSYM_E3N(double, PATH_FP64_FIXUP, false, 256, 2)
    return nullptr;
}
template <> Eig3K<double, PATH_FP64_FIXUP, true> pick_eig3<double, PATH_FP64_FIXUP, true>(int bs, int mpl, bool grad) {
    KSYM_E3(double, PATH_FP64_FIXUP, true, 256, 1)
    return nullptr;
}
#undef KSYM_E3
#undef KSYM_E3N

template <typename T> using Eig2K = void (*)(Eig2Ptrs<T>, uint32_t);
template <typename T> Eig2K<T> pick_eig2(int bs, int mpl) {
#define KSYM_E2(B, M) \
    if (bs == B && mpl == M) return &k_eig2<T, B, M>;
    KSYM_E2(64, 1) KSYM_E2(128, 1) KSYM_E2(128, 2) KSYM_E2(256, 1) KSYM_E2(256, 2) KSYM_E2(256, 4)
    KSYM_E2(512, 1) KSYM_E2(512, 2) KSYM_E2(1024, 1)
#undef KSYM_E2
    return nullptr;
}

template <typename T> using BwdK = void (*)(BwdArgs<T>);
template <typename T> BwdK<T> pick_bwd(int bs, int mpl) {
#define KSYM_B(B, M) \
    if (bs == B && mpl == M) return &k_eig3_bwd<T, B, M>;
    KSYM_B(64, 1) KSYM_B(128, 1) KSYM_B(256, 1) KSYM_B(256, 2) KSYM_B(512, 1)
#undef KSYM_B
    return nullptr;
}

template <typename T> using MixK = void (*)(MixedArgs<T>);
template <typename T> MixK<T> pick_mixed(int bs, int mpl, bool stream = false) {
#define KSYM_M(B, M) \
    if (bs == B && mpl == M) return stream ? &k_mixed<T, B, M, true> : &k_mixed<T, B, M, false>;
    KSYM_M(64, 1) KSYM_M(128, 1) KSYM_M(256, 1) KSYM_M(256, 2) KSYM_M(512, 1)
#undef KSYM_M
    return nullptr;
}

// ------------------------------------------------------------- eig3 -------
template <typename T, bool AOS>
ksym_status eig3_impl(int64_t n, const void *const in[6], const void *aos, void *const lam[3],
                      void *const D[9], void *const phi[3], void *const gap[3], uint8_t *flags,
                      void *ws, size_t ws_bytes, const ksym_opts &o, hipStream_t stream) {
    Eig3Args<T> a;
    memset(&a, 0, sizeof a);
    for (int c = 0; c < 6; ++c) a.p.in[c] = AOS ? nullptr : (const T *)in[c];
    for (int c = 0; c < 3; ++c) a.p.out[O_LAM + c] = lam ? (T *)lam[c] : nullptr;
    for (int c = 0; c < 9; ++c) a.p.out[O_D + c] = D ? (T *)D[c] : nullptr;
    for (int c = 0; c < 3; ++c) a.p.out[O_PHI + c] = phi ? (T *)phi[c] : nullptr;
    for (int c = 0; c < 3; ++c) a.p.out[O_GAP + c] = gap ? (T *)gap[c] : nullptr;
    a.p.flags = flags;
    a.aos = (const T *)aos;
    a.prm.n = n;
    a.prm.tau_gap = o.tau_gap;
    a.prm.tau_res = o.tau_res;
    a.prm.tau_vec = o.tau_vec;
    a.prm.tau_dbl = o.tau_dbl;
    a.prm.drain_tiles = o.drain_tiles;
    a.prm.counters = (unsigned *)ws;
    finish_params(a.prm);
    (void)ws_bytes;
    void (*k)(Eig3Args<T>) = nullptr;
    const bool grad = o.tau_vec > 0.0;
    if constexpr (sizeof(T) == 4) {
        // no D and no angles: the eigenvalues-only kernel (reduced-output mode)
        if (!AOS && none_requested(D, 9) && none_requested(phi, 3)) k = pick_eig3_lam(o.block, o.mats_per_lane);
        else k = pick_eig3<float, PATH_FP32_FIXUP, AOS>(o.block, o.mats_per_lane, grad);
    } else {
        // (the plain path has no check, so tau_vec does not apply to it)
        if (o.path == KSYM_PATH_FP64_PLAIN) k = pick_eig3<double, PATH_FP64_PLAIN, AOS>(o.block, o.mats_per_lane, false);
        else k = pick_eig3<double, PATH_FP64_FIXUP, AOS>(o.block, o.mats_per_lane, grad);
    }
    if (!k)
        return fail(KSYM_E_UNSUPPORTED, "no compiled 3x3 kernel for block %d, mats_per_lane %d%s%s",
                    o.block, o.mats_per_lane, AOS ? " (AoS)" : "", grad ? " with tau_vec > 0" : "");
    // one launch per chunk of matrices, every pointer advanced by the chunk start
    const int64_t chunk = !AOS ? KSYM_CHUNK : (sizeof(T) == 4 ? KSYM_CHUNK_AOS_F32 : KSYM_CHUNK_AOS_F64);
    for (int64_t start = 0; start < n; start += chunk) {
        const int64_t len = n - start < chunk ? n - start : chunk;
        Eig3Args<T> c = a;
        c.prm.n = len;
        for (int k = 0; k < 6; ++k) c.p.in[k] = a.p.in[k] ? a.p.in[k] + start : nullptr;
        for (int k = 0; k < NOUT3; ++k) c.p.out[k] = a.p.out[k] ? a.p.out[k] + start : nullptr;
        c.p.flags = a.p.flags ? a.p.flags + start : nullptr;
        c.aos = a.aos ? a.aos + start * 6 : nullptr;
        int grid = 0;
        ksym_status s = grid_for(len, o.block * o.mats_per_lane, o.grid_mult, &grid);
        if (s != KSYM_OK) return s;
        hipError_t e = launch(k, dim3(grid), dim3(o.block), stream, c);
        if (e != hipSuccess) return hip_fail(e, "launch k_eig3");
    }
    return KSYM_OK;
}

ksym_status check_dtype_path(ksym_dtype dt, const ksym_opts &o) {
    if (dt == KSYM_F32 && o.path != KSYM_PATH_FP32_FIXUP)
        return fail(KSYM_E_DTYPE, "float32 input supports only KSYM_PATH_FP32_FIXUP");
    if (dt == KSYM_F64 && o.path != KSYM_PATH_FP64_PLAIN && o.path != KSYM_PATH_FP64_FIXUP)
        return fail(KSYM_E_DTYPE, "float64 input supports KSYM_PATH_FP64_PLAIN or KSYM_PATH_FP64_FIXUP");
    return KSYM_OK;
}

size_t esize(ksym_dtype dt) { return dt == KSYM_F32 ? 4 : 8; }

ksym_status check_outputs3(ksym_dtype dt, void *const lam[3], void *const D[9], void *const phi[3],
                           void *const gap[3]) {
    const size_t es = esize(dt);
    for (int c = 0; c < 3; ++c)
        if (lam && !aligned(lam[c], es)) return fail(KSYM_E_ARG, "lam[%d] misaligned", c);
    for (int c = 0; c < 9; ++c)
        if (D && !aligned(D[c], es)) return fail(KSYM_E_ARG, "D[%d] misaligned", c);
    for (int c = 0; c < 3; ++c)
        if (phi && !aligned(phi[c], es)) return fail(KSYM_E_ARG, "phi[%d] misaligned", c);
    for (int c = 0; c < 3; ++c)
        if (gap && !aligned(gap[c], es)) return fail(KSYM_E_ARG, "gap[%d] misaligned", c);
    return KSYM_OK;
}

// Byte ranges of the planes of one call, for the aliasing test: an output
// may not overlap an input or another output (inputs may share memory; the
// kernels only read them).  Absent planes and empty ranges are skipped.
struct Range {
    uintptr_t lo, hi;
    bool out;
    const char *what;
    int idx;
};

// Sweep in order of start address (sorted in place): a range overlaps an
// earlier-starting one exactly when it starts below the largest end seen so
// far; the largest end over outputs and over all ranges are tracked apart,
// so an input is tested against outputs only.
ksym_status check_ranges(Range *v, size_t n) {
    std::sort(v, v + n, [](const Range &a, const Range &b) { return a.lo < b.lo; });
    uintptr_t end_all = 0, end_out = 0;
    const Range *arg_all = nullptr, *arg_out = nullptr;
    for (size_t i = 0; i < n; ++i) {
        const Range &r = v[i];
        const Range *hit = r.out ? (r.lo < end_all ? arg_all : nullptr) : (r.lo < end_out ? arg_out : nullptr);
        if (hit)
            return fail(KSYM_E_ARG, "%s[%d] overlaps %s[%d] (an output may not alias an input or another output)",
                        r.out ? r.what : hit->what, r.out ? r.idx : hit->idx,
                        r.out ? hit->what : r.what, r.out ? hit->idx : r.idx);
        if (r.hi > end_all) { end_all = r.hi; arg_all = &r; }
        if (r.out && r.hi > end_out) { end_out = r.hi; arg_out = &r; }
    }
    return KSYM_OK;
}

// The ranges of one call, in a heap vector (VecStore) or in a caller-owned
// fixed array (FixedStore, for the entry point that allocates nothing).
struct VecStore {
    std::vector<Range> v;
    void push(const Range &r) { v.push_back(r); }
    Range *data() { return v.data(); }
    size_t size() const { return v.size(); }
};
struct FixedStore {
    Range *v;
    size_t n, cap;
    void push(const Range &r) {
        if (n < cap) v[n++] = r;
    }
    Range *data() { return v; }
    size_t size() const { return n; }
};
template <typename Store> struct RangeSet {
    Store st;
    void add(const void *p, size_t bytes, bool out, const char *what, int idx) {
        if (p && bytes) st.push({(uintptr_t)p, (uintptr_t)p + bytes, out, what, idx});
    }
    void ins(const void *const *p, int k, size_t bytes, const char *what) {
        if (p)
            for (int c = 0; c < k; ++c) add(p[c], bytes, false, what, c);
    }
    void outs(void *const *p, int k, size_t bytes, const char *what) {
        if (p)
            for (int c = 0; c < k; ++c) add(p[c], bytes, true, what, c);
    }
    ksym_status check() { return check_ranges(st.data(), st.size()); }
};
using Ranges = RangeSet<VecStore>;

ksym_status check_ws(void *ws, size_t ws_bytes) {
    if (ws && ws_bytes < 8) return fail(KSYM_E_WORKSPACE, "workspace of %zu bytes is too small (need 8)", ws_bytes);
    if (ws && !aligned(ws, 4)) return fail(KSYM_E_WORKSPACE, "workspace must be 4-byte aligned");
    return KSYM_OK;
}

}  // namespace

struct ksym_plan {
    ksym_dtype dtype;
    ksym_opts opts;
    int32_t ngroups;
    int64_t ntiles;
    int grid;
    void *d_groups;
    TileInfo *d_tiles;
    bool stream;   // every plane line-aligned: the streaming kernel variant
    hipGraph_t graph;
    hipGraphExec_t exec;
};

extern "C" {

int ksym_version(void) { return KSYM_VERSION; }

const char *ksym_last_error(void) { return g_err.c_str(); }

void ksym_opts_default(ksym_dtype dtype, ksym_opts *o) {
    if (!o) return;
    o->path = dtype == KSYM_F64 ? KSYM_PATH_FP64_FIXUP : KSYM_PATH_FP32_FIXUP;
    o->block = 256;
    o->mats_per_lane = 1;
    o->grid_mult = KSYM_GRID_MULT_MAX;   // one tile per wave at every batch size
    o->tau_gap = 0.0;
    o->tau_dbl = dtype == KSYM_F64 ? 1e-6 : 1e-9;
    o->drain_tiles = 8;
    o->reserved = 0;
    if (dtype == KSYM_F64) {
        o->tau_res = 1e-11;
        o->tau_vec = 0.0;
    } else {
        o->tau_res = 2e-6;
        o->tau_vec = 0.0;
    }
}

ksym_status ksym_eig2(ksym_dtype dtype, int64_t n, const void *const in[3], void *const lam[2],
                      void *const D[4], void *phi, uint8_t *flags, const ksym_opts *opts, void *stream) {
    g_err.clear();
    if (dtype != KSYM_F32 && dtype != KSYM_F64) return fail(KSYM_E_DTYPE, "unknown dtype %d", (int)dtype);
    if (n < 0) return fail(KSYM_E_ARG, "n must be >= 0 (got %lld)", (long long)n);
    ksym_opts o;
    ksym_status s = resolve_opts(dtype, opts, &o);
    if (s != KSYM_OK) return s;
    if (n == 0) return KSYM_OK;
    if (!in) return fail(KSYM_E_ARG, "in is NULL");
    const size_t es = esize(dtype);
    for (int c = 0; c < 3; ++c) {
        if (!in[c]) return fail(KSYM_E_ARG, "in[%d] is NULL", c);
        if (!aligned(in[c], es)) return fail(KSYM_E_ARG, "in[%d] misaligned", c);
    }
    for (int c = 0; c < 2; ++c)
        if (lam && !aligned(lam[c], es)) return fail(KSYM_E_ARG, "lam[%d] misaligned", c);
    for (int c = 0; c < 4; ++c)
        if (D && !aligned(D[c], es)) return fail(KSYM_E_ARG, "D[%d] misaligned", c);
    if (!aligned(phi, es)) return fail(KSYM_E_ARG, "phi misaligned");
    {
        Ranges rg;
        const size_t pb = (size_t)n * es;
        rg.ins(in, 3, pb, "in");
        rg.outs(lam, 2, pb, "lam");
        rg.outs(D, 4, pb, "D");
        rg.add(phi, pb, true, "phi", 0);
        rg.add(flags, (size_t)n, true, "flags", 0);
        s = rg.check();
        if (s != KSYM_OK) return s;
    }
    auto go = [&](auto tag) -> ksym_status {
        using T = decltype(tag);
        Eig2K<T> k = pick_eig2<T>(o.block, o.mats_per_lane);
        if (!k)
            return fail(KSYM_E_UNSUPPORTED, "no compiled 2x2 kernel for block %d, mats_per_lane %d",
                        o.block, o.mats_per_lane);
        for (int64_t start = 0; start < n; start += KSYM_CHUNK) {
            const int64_t len = n - start < KSYM_CHUNK ? n - start : KSYM_CHUNK;
            Eig2Ptrs<T> p;
            for (int c = 0; c < 3; ++c) p.in[c] = (const T *)in[c] + start;
            for (int c = 0; c < 2; ++c) p.lam[c] = lam ? (T *)lam[c] + start : nullptr;
            for (int c = 0; c < 4; ++c) p.D[c] = D ? (T *)D[c] + start : nullptr;
            p.phi = phi ? (T *)phi + start : nullptr;
            p.flags = flags ? flags + start : nullptr;
            int grid = 0;
            ksym_status st = grid_for(len, o.block * o.mats_per_lane, o.grid_mult, &grid);
            if (st != KSYM_OK) return st;
            hipError_t e = launch(k, dim3(grid), dim3(o.block), (hipStream_t)stream, p, (uint32_t)len);
            if (e != hipSuccess) return hip_fail(e, "launch k_eig2");
        }
        return KSYM_OK;
    };
    return dtype == KSYM_F32 ? go(float()) : go(double());
}

size_t ksym_eig3_workspace_bytes(ksym_dtype dtype, int64_t n) {
    (void)dtype;
    (void)n;
    return 256;
}

ksym_status ksym_zero_counters(void *ws, size_t ws_bytes, void *stream) {
    g_err.clear();
    if (!ws) return fail(KSYM_E_WORKSPACE, "workspace is NULL");
    ksym_status s = check_ws(ws, ws_bytes);
    if (s != KSYM_OK) return s;
    hipError_t e = launch(&k_zero_u32, dim3(1), dim3(64), (hipStream_t)stream, (unsigned *)ws, 2);
    if (e != hipSuccess) return hip_fail(e, "launch k_zero_u32");
    return KSYM_OK;
}

static ksym_status eig3_common(bool aos_mode, ksym_dtype dtype, int64_t n, const void *const in[6],
                               const void *a_aos, void *const lam[3], void *const D[9],
                               void *const phi[3], void *const gap[3], uint8_t *flags, void *ws,
                               size_t ws_bytes, const ksym_opts *opts, void *stream) {
    g_err.clear();
    if (dtype != KSYM_F32 && dtype != KSYM_F64) return fail(KSYM_E_DTYPE, "unknown dtype %d", (int)dtype);
    if (n < 0) return fail(KSYM_E_ARG, "n must be >= 0 (got %lld)", (long long)n);
    if (n >= ((int64_t)1 << 40)) return fail(KSYM_E_ARG, "n too large");
    ksym_opts o;
    ksym_status s = resolve_opts(dtype, opts, &o);
    if (s != KSYM_OK) return s;
    s = check_dtype_path(dtype, o);
    if (s != KSYM_OK) return s;
    if (n == 0) return KSYM_OK;
    const size_t es = esize(dtype);
    if (aos_mode) {
        if (!a_aos) return fail(KSYM_E_ARG, "a_aos is NULL");
        if (!aligned(a_aos, 16)) return fail(KSYM_E_ARG, "a_aos must be 16-byte aligned");
    } else {
        if (!in) return fail(KSYM_E_ARG, "in is NULL");
        for (int c = 0; c < 6; ++c) {
            if (!in[c]) return fail(KSYM_E_ARG, "in[%d] is NULL", c);
            if (!aligned(in[c], es)) return fail(KSYM_E_ARG, "in[%d] misaligned", c);
        }
    }
    s = check_outputs3(dtype, lam, D, phi, gap);
    if (s != KSYM_OK) return s;
    s = check_ws(ws, ws_bytes);
    if (s != KSYM_OK) return s;
    {
        Ranges rg;
        const size_t pb = (size_t)n * es;
        if (aos_mode) rg.add(a_aos, pb * 6, false, "a_aos", 0);
        else rg.ins(in, 6, pb, "in");
        rg.outs(lam, 3, pb, "lam");
        rg.outs(D, 9, pb, "D");
        rg.outs(phi, 3, pb, "phi");
        rg.outs(gap, 3, pb, "gap");
        rg.add(flags, (size_t)n, true, "flags", 0);
        rg.add(ws, ws_bytes, true, "ws", 0);
        s = rg.check();
        if (s != KSYM_OK) return s;
    }
    hipStream_t st = (hipStream_t)stream;
    if (dtype == KSYM_F32)
        return aos_mode ? eig3_impl<float, true>(n, in, a_aos, lam, D, phi, gap, flags, ws, ws_bytes, o, st)
                        : eig3_impl<float, false>(n, in, a_aos, lam, D, phi, gap, flags, ws, ws_bytes, o, st);
    return aos_mode ? eig3_impl<double, true>(n, in, a_aos, lam, D, phi, gap, flags, ws, ws_bytes, o, st)
                    : eig3_impl<double, false>(n, in, a_aos, lam, D, phi, gap, flags, ws, ws_bytes, o, st);
}

ksym_status ksym_eig3(ksym_dtype dtype, int64_t n, const void *const in[6], void *const lam[3],
                      void *const D[9], void *const phi[3], void *const gap[3], uint8_t *flags,
                      void *ws, size_t ws_bytes, const ksym_opts *opts, void *stream) {
    return eig3_common(false, dtype, n, in, nullptr, lam, D, phi, gap, flags, ws, ws_bytes, opts, stream);
}

ksym_status ksym_eig3_aos(ksym_dtype dtype, int64_t n, const void *a_aos, void *const lam[3],
                          void *const D[9], void *const phi[3], void *const gap[3], uint8_t *flags,
                          void *ws, size_t ws_bytes, const ksym_opts *opts, void *stream) {
    return eig3_common(true, dtype, n, nullptr, a_aos, lam, D, phi, gap, flags, ws, ws_bytes, opts, stream);
}

static ksym_status compose_impl(int k, ksym_dtype dtype, int64_t n, const void *const lam[], const void *const phi[],
                                void *const A[], void *stream) {
    g_err.clear();
    if (dtype != KSYM_F32 && dtype != KSYM_F64) return fail(KSYM_E_DTYPE, "unknown dtype %d", (int)dtype);
    if (n < 0) return fail(KSYM_E_ARG, "n must be >= 0 (got %lld)", (long long)n);
    if (n == 0) return KSYM_OK;
    const size_t es = esize(dtype);
    const int nl = k, nf = k == 3 ? 3 : 1, na = k == 3 ? 6 : 3;
    if (!lam || !phi || !A) return fail(KSYM_E_ARG, "lam, phi and A are required");
    for (int c = 0; c < nl; ++c)
        if (!lam[c] || !aligned(lam[c], es)) return fail(KSYM_E_ARG, "lam[%d] NULL or misaligned", c);
    for (int c = 0; c < nf; ++c)
        if (!phi[c] || !aligned(phi[c], es)) return fail(KSYM_E_ARG, "phi[%d] NULL or misaligned", c);
    for (int c = 0; c < na; ++c)
        if (!A[c] || !aligned(A[c], es)) return fail(KSYM_E_ARG, "A[%d] NULL or misaligned", c);
    {
        Ranges rg;
        const size_t pb = (size_t)n * es;
        rg.ins(lam, nl, pb, "lam");
        rg.ins(phi, nf, pb, "phi");
        rg.outs(A, na, pb, "A");
        ksym_status s = rg.check();
        if (s != KSYM_OK) return s;
    }
    constexpr int BS = 256;
    auto go = [&](auto tag) -> ksym_status {
        using T = decltype(tag);
        for (int64_t start = 0; start < n; start += KSYM_CHUNK) {
            const int64_t len = n - start < KSYM_CHUNK ? n - start : KSYM_CHUNK;
            ComposeArgs<T> ca;
            memset(&ca, 0, sizeof ca);
            for (int c = 0; c < nl; ++c) ca.p.lam[c] = (const T *)lam[c] + start;
            for (int c = 0; c < nf; ++c) ca.p.phi[c] = (const T *)phi[c] + start;
            for (int c = 0; c < na; ++c) ca.p.A[c] = (T *)A[c] + start;
            ca.n = (uint32_t)len;
            int grid = 0;
            ksym_status st = grid_for(len, BS, KSYM_GRID_MULT_MAX, &grid);
            if (st != KSYM_OK) return st;
            hipError_t e = k == 3 ? launch(&k_compose3<T, BS>, dim3(grid), dim3(BS), (hipStream_t)stream, ca)
                                  : launch(&k_compose2<T, BS>, dim3(grid), dim3(BS), (hipStream_t)stream, ca);
            if (e != hipSuccess) return hip_fail(e, "launch k_compose");
        }
        return KSYM_OK;
    };
    return dtype == KSYM_F32 ? go(float()) : go(double());
}

ksym_status ksym_compose3(ksym_dtype dtype, int64_t n, const void *const lam[3], const void *const phi[3],
                          void *const A[6], void *stream) {
    return compose_impl(3, dtype, n, lam, phi, A, stream);
}

ksym_status ksym_compose2(ksym_dtype dtype, int64_t n, const void *const lam[2], const void *phi,
                          void *const A[3], void *stream) {
    const void *const phis[1] = {phi};
    return compose_impl(2, dtype, n, lam, phi ? phis : nullptr, A, stream);
}

ksym_status ksym_eig2_backward(ksym_dtype dtype, int64_t n, const void *const lam[2],
                               const void *const D[4], const void *const glam[2], const void *const gD[4],
                               const void *gphi, void *const gA[3], double eps_rel, void *stream) {
    g_err.clear();
    if (dtype != KSYM_F32 && dtype != KSYM_F64) return fail(KSYM_E_DTYPE, "unknown dtype %d", (int)dtype);
    if (n < 0) return fail(KSYM_E_ARG, "n must be >= 0 (got %lld)", (long long)n);
    if (!(eps_rel >= 0.0) || eps_rel > 1e30) return fail(KSYM_E_ARG, "eps_rel must be finite and >= 0");
    if (n == 0) return KSYM_OK;
    const size_t es = esize(dtype);
    if (!lam || !D || !gA) return fail(KSYM_E_ARG, "lam, D and gA are required");
    for (int c = 0; c < 2; ++c)
        if (!lam[c] || !aligned(lam[c], es)) return fail(KSYM_E_ARG, "lam[%d] NULL or misaligned", c);
    for (int c = 0; c < 4; ++c)
        if (!D[c] || !aligned(D[c], es)) return fail(KSYM_E_ARG, "D[%d] NULL or misaligned", c);
    for (int c = 0; c < 3; ++c)
        if (!gA[c] || !aligned(gA[c], es)) return fail(KSYM_E_ARG, "gA[%d] NULL or misaligned", c);
    if (glam)
        for (int c = 0; c < 2; ++c)
            if (glam[c] && !aligned(glam[c], es)) return fail(KSYM_E_ARG, "glam[%d] misaligned", c);
    if (gD)
        for (int c = 0; c < 4; ++c)
            if (gD[c] && !aligned(gD[c], es)) return fail(KSYM_E_ARG, "gD[%d] misaligned", c);
    if (gphi && !aligned(gphi, es)) return fail(KSYM_E_ARG, "gphi misaligned");
    {
        Ranges rg;
        const size_t pb = (size_t)n * es;
        rg.ins(lam, 2, pb, "lam");
        rg.ins(D, 4, pb, "D");
        rg.ins(glam, 2, pb, "glam");
        rg.ins(gD, 4, pb, "gD");
        rg.add(gphi, pb, false, "gphi", 0);
        rg.outs(gA, 3, pb, "gA");
        ksym_status s = rg.check();
        if (s != KSYM_OK) return s;
    }
    constexpr int BS = 256;
    auto go = [&](auto tag) -> ksym_status {
        using T = decltype(tag);
        for (int64_t start = 0; start < n; start += KSYM_CHUNK) {
            const int64_t len = n - start < KSYM_CHUNK ? n - start : KSYM_CHUNK;
            Bwd2Args<T> ba;
            memset(&ba, 0, sizeof ba);
            for (int c = 0; c < 2; ++c) ba.p.lam[c] = (const T *)lam[c] + start;
            for (int c = 0; c < 4; ++c) ba.p.D[c] = (const T *)D[c] + start;
            for (int c = 0; c < 2; ++c) ba.p.glam[c] = glam && glam[c] ? (const T *)glam[c] + start : nullptr;
            for (int c = 0; c < 4; ++c) ba.p.gD[c] = gD && gD[c] ? (const T *)gD[c] + start : nullptr;
            ba.p.gphi = gphi ? (const T *)gphi + start : nullptr;
            for (int c = 0; c < 3; ++c) ba.p.gA[c] = (T *)gA[c] + start;
            ba.n = (uint32_t)len;
            ba.eps_rel = eps_rel;
            int grid = 0;
            ksym_status st = grid_for(len, BS, KSYM_GRID_MULT_MAX, &grid);
            if (st != KSYM_OK) return st;
            hipError_t e = launch(&k_eig2_bwd<T, BS>, dim3(grid), dim3(BS), (hipStream_t)stream, ba);
            if (e != hipSuccess) return hip_fail(e, "launch k_eig2_bwd");
        }
        return KSYM_OK;
    };
    return dtype == KSYM_F32 ? go(float()) : go(double());
}

static ksym_status eig3_backward_impl(ksym_dtype dtype, int64_t n, const void *const lam[3],
                                      const void *const D[9], const void *const phi[3], const void *const gap[3],
                                      const void *const glam[3], const void *const gD[9],
                                      const void *const gphi[3], void *const gA[6], double eps_rel,
                                      void *stream) {
    if (dtype != KSYM_F32 && dtype != KSYM_F64) return fail(KSYM_E_DTYPE, "unknown dtype %d", (int)dtype);
    if (n < 0) return fail(KSYM_E_ARG, "n must be >= 0 (got %lld)", (long long)n);
    if (!(eps_rel >= 0.0) || eps_rel > 1e30) return fail(KSYM_E_ARG, "eps_rel must be finite and >= 0");
    if (n == 0) return KSYM_OK;
    const size_t es = esize(dtype);
    if (!lam || !D || !gA) return fail(KSYM_E_ARG, "lam, D and gA are required");
    for (int c = 0; c < 3; ++c)
        if (!lam[c] || !aligned(lam[c], es)) return fail(KSYM_E_ARG, "lam[%d] NULL or misaligned", c);
    for (int c = 0; c < 9; ++c)
        if (!D[c] || !aligned(D[c], es)) return fail(KSYM_E_ARG, "D[%d] NULL or misaligned", c);
    for (int c = 0; c < 6; ++c)
        if (!gA[c] || !aligned(gA[c], es)) return fail(KSYM_E_ARG, "gA[%d] NULL or misaligned", c);
    if (gap)
        for (int c = 0; c < 3; ++c)
            if (!gap[c] || !aligned(gap[c], es)) return fail(KSYM_E_ARG, "gap[%d] NULL or misaligned", c);
    if (glam)
        for (int c = 0; c < 3; ++c)
            if (!glam[c] || !aligned(glam[c], es)) return fail(KSYM_E_ARG, "glam[%d] NULL or misaligned", c);
    if (gD)
        for (int c = 0; c < 9; ++c)
            if (!gD[c] || !aligned(gD[c], es)) return fail(KSYM_E_ARG, "gD[%d] NULL or misaligned", c);
    if (phi)
        for (int c = 0; c < 3; ++c)
            if (!phi[c] || !aligned(phi[c], es)) return fail(KSYM_E_ARG, "phi[%d] NULL or misaligned", c);
    if (gphi)
        for (int c = 0; c < 3; ++c)
            if (!gphi[c] || !aligned(gphi[c], es)) return fail(KSYM_E_ARG, "gphi[%d] NULL or misaligned", c);
    {
        Ranges rg;
        const size_t pb = (size_t)n * es;
        rg.ins(lam, 3, pb, "lam");
        rg.ins(D, 9, pb, "D");
        rg.ins(gap, 3, pb, "gap");
        rg.ins(glam, 3, pb, "glam");
        rg.ins(gD, 9, pb, "gD");
        rg.ins(phi, 3, pb, "phi");
        rg.ins(gphi, 3, pb, "gphi");
        rg.outs(gA, 6, pb, "gA");
        ksym_status s = rg.check();
        if (s != KSYM_OK) return s;
    }
    ksym_opts o;
    ksym_opts_default(dtype, &o);
    o.mats_per_lane = 1;
    auto go = [&](auto tag) -> ksym_status {
        using T = decltype(tag);
        BwdK<T> k = pick_bwd<T>(o.block, o.mats_per_lane);
        if (!k) return fail(KSYM_E_UNSUPPORTED, "no compiled backward kernel");
        for (int64_t start = 0; start < n; start += KSYM_CHUNK) {
            const int64_t len = n - start < KSYM_CHUNK ? n - start : KSYM_CHUNK;
            BwdPtrs<T> p;
            for (int c = 0; c < 3; ++c) p.lam[c] = (const T *)lam[c] + start;
            for (int c = 0; c < 9; ++c) p.D[c] = (const T *)D[c] + start;
            for (int c = 0; c < 3; ++c) p.gap[c] = gap ? (const T *)gap[c] + start : nullptr;
            for (int c = 0; c < 3; ++c) p.glam[c] = glam ? (const T *)glam[c] + start : nullptr;
            for (int c = 0; c < 9; ++c) p.gD[c] = gD ? (const T *)gD[c] + start : nullptr;
            for (int c = 0; c < 6; ++c) p.gA[c] = (T *)gA[c] + start;
            for (int c = 0; c < 3; ++c) p.phi[c] = phi ? (const T *)phi[c] + start : nullptr;
            for (int c = 0; c < 3; ++c) p.gphi[c] = gphi ? (const T *)gphi[c] + start : nullptr;
            int grid = 0;
            ksym_status st = grid_for(len, o.block * o.mats_per_lane, o.grid_mult, &grid);
            if (st != KSYM_OK) return st;
            BwdArgs<T> ba;
            memset(&ba, 0, sizeof ba);
            ba.p = p;
            ba.n = (uint32_t)len;
            ba.zero = 0;
            ba.eps_rel = eps_rel;
            hipError_t e = launch(k, dim3(grid), dim3(o.block), (hipStream_t)stream, ba);
            if (e != hipSuccess) return hip_fail(e, "launch k_eig3_bwd");
        }
        return KSYM_OK;
    };
    return dtype == KSYM_F32 ? go(float()) : go(double());
}

ksym_status ksym_eig3_backward(ksym_dtype dtype, int64_t n, const void *const lam[3],
                               const void *const D[9], const void *const gap[3],
                               const void *const glam[3], const void *const gD[9], void *const gA[6],
                               double eps_rel, void *stream) {
    g_err.clear();
    return eig3_backward_impl(dtype, n, lam, D, nullptr, gap, glam, gD, nullptr, gA, eps_rel, stream);
}

ksym_status ksym_eig3_backward_angles(ksym_dtype dtype, int64_t n, const void *const lam[3],
                                      const void *const D[9], const void *const phi[3],
                                      const void *const gap[3], const void *const glam[3],
                                      const void *const gD[9], const void *const gphi[3], void *const gA[6],
                                      double eps_rel, void *stream) {
    g_err.clear();
    if (!phi || !gphi) return fail(KSYM_E_ARG, "phi and gphi are required (ksym_eig3_backward has neither)");
    return eig3_backward_impl(dtype, n, lam, D, phi, gap, glam, gD, gphi, gA, eps_rel, stream);
}

// ------------------------------------------------------------- plans ------
}  // extern "C"

namespace {

// Group checks shared by ksym_plan_create and ksym_mixed_run_noalloc: kinds,
// sizes, alignment, and no output overlapping any input or other output
// across all groups (rg collects the ranges).
template <typename Store>
ksym_status check_groups(ksym_dtype dtype, int32_t ngroups, const ksym_group *groups, RangeSet<Store> &rg) {
    const size_t es = esize(dtype);
    for (int g = 0; g < ngroups; ++g) {
        const ksym_group &G = groups[g];
        if (G.kind != 2 && G.kind != 3) return fail(KSYM_E_ARG, "group %d: kind must be 2 or 3", g);
        if (G.n < 0) return fail(KSYM_E_ARG, "group %d: n < 0", g);
        if (G.n >= ((int64_t)1 << 40)) return fail(KSYM_E_ARG, "group %d: n too large", g);
        const int nin = G.kind == 3 ? 6 : 3;
        if (G.n > 0)
            for (int c = 0; c < nin; ++c)
                if (!G.in[c] || !aligned(G.in[c], es)) return fail(KSYM_E_ARG, "group %d: in[%d] NULL or misaligned", g, c);
        for (int c = 0; c < 3; ++c)
            if (!aligned(G.lam[c], es) || !aligned(G.phi[c], es)) return fail(KSYM_E_ARG, "group %d: output misaligned", g);
        for (int c = 0; c < 9; ++c)
            if (!aligned(G.D[c], es)) return fail(KSYM_E_ARG, "group %d: D[%d] misaligned", g, c);
    }
    for (int g = 0; g < ngroups; ++g) {
        const ksym_group &G = groups[g];
        const size_t pb = (size_t)G.n * es;
        const bool k3 = G.kind == 3;
        rg.ins(G.in, k3 ? 6 : 3, pb, "group in");
        rg.outs(G.lam, k3 ? 3 : 2, pb, "group lam");
        rg.outs(G.D, k3 ? 9 : 4, pb, "group D");
        rg.outs(G.phi, k3 ? 3 : 1, pb, "group phi");
        rg.add(G.flags, (size_t)G.n, true, "group flags", g);
    }
    return rg.check();
}

// Planes a group of kind 2 or 3 uses, for the range count of the checks.
constexpr int kGroupRanges = 6 + 3 + 9 + 3 + 1;

// True when every plane of every group (inputs, outputs and flags present)
// starts on a 256-byte boundary: a wave tile's part of each plane then fills
// whole cache lines, and the mixed kernel can stream.
bool groups_line_aligned(int32_t ngroups, const ksym_group *groups) {
    for (int g = 0; g < ngroups; ++g) {
        const ksym_group &G = groups[g];
        const bool k3 = G.kind == 3;
        auto ok = [](const void *const *p, int k) {
            for (int c = 0; c < k; ++c)
                if (p[c] && !aligned(p[c], 256)) return false;
            return true;
        };
        if (!ok(G.in, k3 ? 6 : 3) || !ok(G.lam, k3 ? 3 : 2) || !ok(G.D, k3 ? 9 : 4) || !ok(G.phi, k3 ? 3 : 1))
            return false;
        if (G.flags && !aligned(G.flags, 256)) return false;
    }
    return true;
}

// The descriptor of matrices [start, start + len) of group G (every plane
// pointer advanced by start; a descriptor covers at most KSYM_CHUNK).
template <typename T> GroupDesc<T> make_desc(const ksym_group &G, int64_t start, int64_t len) {
    GroupDesc<T> d;
    memset(&d, 0, sizeof d);
    d.n = len;
    d.kind = G.kind;
    const int nin = G.kind == 3 ? 6 : 3;
    const int nl = G.kind == 3 ? 3 : 2, nd = G.kind == 3 ? 9 : 4, np = G.kind == 3 ? 3 : 1;
    auto adv = [&](const void *q) { return q ? (T *)q + start : nullptr; };
    for (int c = 0; c < nin; ++c) d.p3.in[c] = adv(G.in[c]);
    for (int c = 0; c < nl; ++c) d.p3.out[O_LAM + c] = adv(G.lam[c]);
    for (int c = 0; c < nd; ++c) d.p3.out[O_D + c] = adv(G.D[c]);
    for (int c = 0; c < np; ++c) d.p3.out[O_PHI + c] = adv(G.phi[c]);
    d.p3.flags = G.flags ? G.flags + start : nullptr;
    return d;
}

// Calls emit(group, start, len, first_tile) for every descriptor of the
// batch in order (one per KSYM_CHUNK matrices of a group, one for an empty
// group) and returns the total number of wave tiles of `tile` matrices.
template <typename F> int64_t for_each_desc(int32_t ngroups, const ksym_group *groups, int tile, F emit) {
    int64_t tiles = 0;
    for (int g = 0; g < ngroups; ++g) {
        const ksym_group &G = groups[g];
        for (int64_t start = 0; start == 0 || start < G.n; start += KSYM_CHUNK) {
            const int64_t len = G.n - start < KSYM_CHUNK ? G.n - start : KSYM_CHUNK;
            emit(g, start, len, tiles);
            tiles += (len + tile - 1) / tile;
        }
    }
    return tiles;
}

// Mixed-batch options: the checked path of the dtype and a compiled shape.
ksym_status mixed_opts(ksym_dtype dtype, const ksym_opts *opts, ksym_opts *o) {
    ksym_status s = resolve_opts(dtype, opts, o);
    if (s != KSYM_OK) return s;
    o->path = dtype == KSYM_F32 ? KSYM_PATH_FP32_FIXUP : KSYM_PATH_FP64_FIXUP;
    if (o->tau_vec > 0.0)
        return fail(KSYM_E_UNSUPPORTED, "tau_vec (differentiated calls) applies to ksym_eig3 and ksym_eig3_aos, "
                                        "not to mixed batches");
    const bool ok = dtype == KSYM_F32 ? pick_mixed<float>(o->block, o->mats_per_lane) != nullptr
                                      : pick_mixed<double>(o->block, o->mats_per_lane) != nullptr;
    if (!ok)
        return fail(KSYM_E_UNSUPPORTED, "no compiled mixed kernel for block %d, mats_per_lane %d", o->block,
                    o->mats_per_lane);
    return KSYM_OK;
}

// Workgroups of the mixed launch: grid_mult per CU, at most one per
// block/64 tiles.
ksym_status mixed_grid(const ksym_opts &o, int64_t ntiles, int *grid) {
    int cus = 0;
    ksym_status s = cu_count(&cus);
    if (s != KSYM_OK) return s;
    int64_t g = (int64_t)o.grid_mult * cus;
    const int64_t need = (ntiles + o.block / 64 - 1) / (o.block / 64);
    if (g > need) g = need;
    if (g < 1) g = 1;
    *grid = (int)g;
    return KSYM_OK;
}

// Counter reset and the persistent mixed kernel over descriptor and tile
// tables already in device memory.
ksym_status launch_mixed(ksym_dtype dtype, const ksym_opts &o, const void *d_groups, const TileInfo *d_tiles,
                         int32_t ndesc, int64_t ntiles, int grid, bool stream, void *ws, hipStream_t st) {
    if (ws) {
        hipError_t e = launch(&k_zero_u32, dim3(1), dim3(64), st, (unsigned *)ws, 2);
        if (e != hipSuccess) return hip_fail(e, "launch k_zero_u32");
    }
    if (ntiles == 0) return KSYM_OK;
    auto go = [&](auto tag) -> ksym_status {
        using T = decltype(tag);
        MixedArgs<T> a;
        memset(&a, 0, sizeof a);
        a.groups = (const GroupDesc<T> *)d_groups;
        a.tiles = d_tiles;
        a.ngroups = ndesc;
        a.ntiles = ntiles;
        a.prm.n = 0;
        a.prm.tau_gap = o.tau_gap;
        a.prm.tau_res = o.tau_res;
        a.prm.tau_vec = o.tau_vec;
        a.prm.tau_dbl = o.tau_dbl;
        a.prm.drain_tiles = o.drain_tiles;
        a.prm.counters = (unsigned *)ws;
        finish_params(a.prm);
        MixK<T> k = pick_mixed<T>(o.block, o.mats_per_lane, stream);
        hipError_t e = launch(k, dim3(grid), dim3(o.block), st, a);
        if (e != hipSuccess) return hip_fail(e, "launch k_mixed");
        return KSYM_OK;
    };
    return dtype == KSYM_F32 ? go(float()) : go(double());
}

}  // namespace

extern "C" {

ksym_status ksym_plan_create(ksym_dtype dtype, int32_t ngroups, const ksym_group *groups,
                             const ksym_opts *opts, ksym_plan **plan, size_t *ws_bytes) {
    g_err.clear();
    if (!plan) return fail(KSYM_E_ARG, "plan is NULL");
    *plan = nullptr;
    if (dtype != KSYM_F32 && dtype != KSYM_F64) return fail(KSYM_E_DTYPE, "unknown dtype %d", (int)dtype);
    if (ngroups <= 0 || !groups) return fail(KSYM_E_ARG, "need ngroups > 0 and a group array");
    ksym_opts o;
    ksym_status s = mixed_opts(dtype, opts, &o);
    if (s != KSYM_OK) return s;
    {
        Ranges rg;
        s = check_groups(dtype, ngroups, groups, rg);
        if (s != KSYM_OK) return s;
    }
    const int tile = 64 * o.mats_per_lane;   // one wave tile
    const bool f32 = dtype == KSYM_F32;
    // one descriptor per KSYM_CHUNK matrices of a group (offsets stay 32-bit)
    std::vector<int64_t> tb;
    std::vector<unsigned char> desc;
    const int64_t ntiles = for_each_desc(ngroups, groups, tile, [&](int g, int64_t start, int64_t len, int64_t first) {
        const size_t at = desc.size();
        if (f32) {
            const GroupDesc<float> d = make_desc<float>(groups[g], start, len);
            desc.resize(at + sizeof d);
            memcpy(desc.data() + at, &d, sizeof d);
        } else {
            const GroupDesc<double> d = make_desc<double>(groups[g], start, len);
            desc.resize(at + sizeof d);
            memcpy(desc.data() + at, &d, sizeof d);
        }
        tb.push_back(first);
    });
    tb.push_back(ntiles);
    const int64_t ndesc = (int64_t)tb.size() - 1;
    if (ndesc >= (1 << 24)) return fail(KSYM_E_ARG, "too many groups (%lld descriptors)", (long long)ndesc);
    ksym_plan *p = new (std::nothrow) ksym_plan();
    if (!p) return fail(KSYM_E_ARG, "out of host memory");
    p->dtype = dtype;
    p->opts = o;
    p->ngroups = (int32_t)ndesc;
    p->ntiles = ntiles;
    p->stream = groups_line_aligned(ngroups, groups);
    s = mixed_grid(o, ntiles, &p->grid);
    if (s != KSYM_OK) { delete p; return s; }
    // one (descriptor, first-matrix offset) entry per wave tile
    std::vector<TileInfo> ti;
    try {
        ti.resize((size_t)p->ntiles);
    } catch (...) {
        delete p;
        return fail(KSYM_E_ARG, "out of host memory for the tile table");
    }
    for (int64_t d = 0; d < ndesc; ++d)
        for (int64_t t = tb[d]; t < tb[d + 1]; ++t) {
            ti[t].group = (int32_t)d;
            ti[t].base = (uint32_t)((t - tb[d]) * tile);
        }
    const size_t tb_bytes = ti.size() * sizeof(TileInfo);
    const size_t total = desc.size() + 256 + tb_bytes;
    hipError_t e = hipMalloc(&p->d_groups, total);
    if (e != hipSuccess) { delete p; return hip_fail(e, "hipMalloc plan descriptors"); }
    p->d_tiles = (TileInfo *)((char *)p->d_groups + ((desc.size() + 255) / 256) * 256);
    e = hipMemcpy(p->d_groups, desc.data(), desc.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess && tb_bytes) e = hipMemcpy(p->d_tiles, ti.data(), tb_bytes, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        (void)hipFree(p->d_groups);
        delete p;
        return hip_fail(e, "hipMemcpy plan descriptors");
    }
    *plan = p;
    if (ws_bytes) *ws_bytes = 256;
    return KSYM_OK;
}

ksym_status ksym_plan_run(ksym_plan *p, void *ws, size_t ws_bytes, void *stream) {
    g_err.clear();
    if (!p) return fail(KSYM_E_ARG, "plan is NULL");
    ksym_status s = check_ws(ws, ws_bytes);
    if (s != KSYM_OK) return s;
    return launch_mixed(p->dtype, p->opts, p->d_groups, p->d_tiles, p->ngroups, p->ntiles, p->grid, p->stream, ws,
                        (hipStream_t)stream);
}

ksym_status ksym_plan_capture(ksym_plan *p, void *ws, size_t ws_bytes, void *stream) {
    g_err.clear();
    if (!p) return fail(KSYM_E_ARG, "plan is NULL");
    hipStream_t st = (hipStream_t)stream;
    if (!st) return fail(KSYM_E_ARG, "capture needs a non-default stream");
    ksym_status s = check_ws(ws, ws_bytes);
    if (s != KSYM_OK) return s;
    if (p->exec) { (void)hipGraphExecDestroy(p->exec); p->exec = nullptr; }
    if (p->graph) { (void)hipGraphDestroy(p->graph); p->graph = nullptr; }
    hipError_t e = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_fail(e, "hipStreamBeginCapture");
    s = ksym_plan_run(p, ws, ws_bytes, stream);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(st, &g);
    if (s != KSYM_OK) { if (g) (void)hipGraphDestroy(g); return s; }
    if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
    hipGraphExec_t x = nullptr;
    e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
    if (e != hipSuccess) { (void)hipGraphDestroy(g); return hip_fail(e, "hipGraphInstantiate"); }
    p->graph = g;
    p->exec = x;
    return KSYM_OK;
}

ksym_status ksym_plan_replay(ksym_plan *p, void *stream) {
    g_err.clear();
    if (!p) return fail(KSYM_E_ARG, "plan is NULL");
    if (!p->exec) return fail(KSYM_E_ARG, "plan has no captured graph (call ksym_plan_capture)");
    hipError_t e = hipGraphLaunch(p->exec, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
    return KSYM_OK;
}

ksym_status ksym_plan_info(const ksym_plan *p, int64_t *tiles, int32_t *grid) {
    g_err.clear();
    if (!p) return fail(KSYM_E_ARG, "plan is NULL");
    if (tiles) *tiles = p->ntiles;
    if (grid) *grid = p->grid;
    return KSYM_OK;
}

void ksym_plan_destroy(ksym_plan *p) {
    if (!p) return;
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    if (p->d_groups) (void)hipFree(p->d_groups);
    delete p;
}

}  // extern "C"

// ------------------------------------------------ mixed batch, no allocation ---
// ksym_mixed_run_noalloc keeps the descriptor table, its first-tile prefix and
// the wave-tile table of one mixed batch in `scratch`, a fixed device array
// (one copy per GPU, held until the process ends).  In host code the array's
// name is only a handle for hipGetSymbolAddress: its device address, which
// differs per GPU, is looked up once per device and kept in g_scratch_addr.
namespace {
constexpr size_t kNaDescBytes = (size_t)KSYM_NOALLOC_MAX_DESCRIPTORS * sizeof(GroupDesc<double>);
constexpr size_t kNaFirstBytes = (((size_t)KSYM_NOALLOC_MAX_DESCRIPTORS + 1) * sizeof(int64_t) + 255) / 256 * 256;
constexpr size_t kNaTileBytes = (size_t)KSYM_NOALLOC_MAX_TILES * sizeof(TileInfo);
constexpr size_t kNaScratchBytes = kNaDescBytes + kNaFirstBytes + kNaTileBytes;
static_assert(sizeof(GroupDesc<float>) == sizeof(GroupDesc<double>), "descriptor layouts differ by dtype");
static_assert(kNaDescBytes % 256 == 0, "descriptor region must keep the next region 256-byte aligned");
}  // namespace

static __device__ __align__(256) unsigned char scratch[kNaScratchBytes];

namespace {
std::atomic<void *> g_scratch_addr[64];
std::mutex g_scratch_mu;

// Device address of `scratch` on the current device (looked up on the
// device's first call).
ksym_status scratch_addr(void **out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= 64) return fail(KSYM_E_HIP, "device index %d out of range", dev);
    void *p = g_scratch_addr[dev].load(std::memory_order_acquire);
    if (!p) {
        std::lock_guard<std::mutex> lk(g_scratch_mu);
        p = g_scratch_addr[dev].load(std::memory_order_relaxed);
        if (!p) {
            e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
            if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
            if (!p) return fail(KSYM_E_HIP, "hipGetSymbolAddress(scratch) gave NULL");
            g_scratch_addr[dev].store(p, std::memory_order_release);
        }
    }
    *out = p;
    return KSYM_OK;
}

// Fixed storage for the aliasing check of ksym_mixed_run_noalloc (plus one
// range for the workspace), guarded by g_na_mu.
Range g_na_ranges[(size_t)KSYM_NOALLOC_MAX_GROUPS * kGroupRanges + 1];
std::mutex g_na_mu;
}  // namespace

extern "C" {

ksym_status ksym_mixed_run_noalloc(ksym_dtype dtype, int32_t ngroups, const ksym_group *groups,
                                   const ksym_opts *opts, void *ws, size_t ws_bytes, void *stream) {
    g_err.clear();
    if (dtype != KSYM_F32 && dtype != KSYM_F64) return fail(KSYM_E_DTYPE, "unknown dtype %d", (int)dtype);
    if (ngroups <= 0 || !groups) return fail(KSYM_E_ARG, "need ngroups > 0 and a group array");
    if (ngroups > KSYM_NOALLOC_MAX_GROUPS)
        return fail(KSYM_E_ARG, "%d groups; ksym_mixed_run_noalloc takes at most %d", (int)ngroups,
                    KSYM_NOALLOC_MAX_GROUPS);
    ksym_opts o;
    ksym_status s = mixed_opts(dtype, opts, &o);
    if (s != KSYM_OK) return s;
    s = check_ws(ws, ws_bytes);
    if (s != KSYM_OK) return s;
    {
        std::lock_guard<std::mutex> lk(g_na_mu);
        RangeSet<FixedStore> rg{FixedStore{g_na_ranges, 0, sizeof g_na_ranges / sizeof g_na_ranges[0]}};
        rg.add(ws, ws_bytes, true, "ws", 0);
        s = check_groups(dtype, ngroups, groups, rg);
        if (s != KSYM_OK) return s;
    }
    const int tile = 64 * o.mats_per_lane;
    int64_t ndesc = 0;
    const int64_t ntiles = for_each_desc(ngroups, groups, tile, [&](int, int64_t, int64_t, int64_t) { ++ndesc; });
    if (ndesc > KSYM_NOALLOC_MAX_DESCRIPTORS)
        return fail(KSYM_E_ARG, "%lld group chunks of at most 2^28 matrices; at most %d", (long long)ndesc,
                    KSYM_NOALLOC_MAX_DESCRIPTORS);
    if (ntiles > KSYM_NOALLOC_MAX_TILES)
        return fail(KSYM_E_ARG, "%lld wave tiles of %d matrices; at most %d", (long long)ntiles, tile,
                    KSYM_NOALLOC_MAX_TILES);
    int grid = 0;
    s = mixed_grid(o, ntiles, &grid);
    if (s != KSYM_OK) return s;
    void *base = nullptr;
    s = scratch_addr(&base);
    if (s != KSYM_OK) return s;
    char *const b = (char *)base;
    void *const d_desc = b;
    int64_t *const d_first = (int64_t *)(b + kNaDescBytes);
    TileInfo *const d_tiles = (TileInfo *)(b + kNaDescBytes + kNaFirstBytes);
    const hipStream_t st = (hipStream_t)stream;
    // descriptors and their first tiles through kernel arguments, DESC_BATCH
    // per launch; then the tile table from the prefix
    auto tables = [&](auto tag) -> ksym_status {
        using T = decltype(tag);
        DescBatch<T> batch;
        memset(&batch, 0, sizeof batch);
        int64_t done = 0;
        hipError_t err = hipSuccess;
        auto flush = [&](bool last) {
            batch.last = last ? 1 : 0;
            batch.total_tiles = ntiles;
            if (err == hipSuccess)
                err = launch(&k_put_desc<T>, dim3(1), dim3(64), st, batch, (GroupDesc<T> *)d_desc, d_first);
            batch.start += batch.count;
            batch.count = 0;
        };
        for_each_desc(ngroups, groups, tile, [&](int g, int64_t start, int64_t len, int64_t first) {
            batch.d[batch.count] = make_desc<T>(groups[g], start, len);
            batch.first_tile[batch.count] = first;
            ++batch.count;
            ++done;
            if (batch.count == DESC_BATCH && done < ndesc) flush(false);
        });
        flush(true);
        if (err != hipSuccess) return hip_fail(err, "launch k_put_desc");
        if (ntiles > 0) {
            err = launch(&k_fill_tiles, dim3((unsigned)((ntiles + 255) / 256)), dim3(256), st,
                         (const int64_t *)d_first, (int32_t)ndesc, d_tiles, ntiles, (int32_t)tile);
            if (err != hipSuccess) return hip_fail(err, "launch k_fill_tiles");
        }
        return KSYM_OK;
    };
    s = dtype == KSYM_F32 ? tables(float()) : tables(double());
    if (s != KSYM_OK) return s;
    return launch_mixed(dtype, o, d_desc, d_tiles, (int32_t)ndesc, ntiles, grid,
                        groups_line_aligned(ngroups, groups), ws, st);
}

}  // extern "C"
