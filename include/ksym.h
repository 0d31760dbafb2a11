/*
 * ksym -- batched closed-form eigendecomposition of 2x2 and 3x3 real symmetric
 * matrices on AMD MI355X (gfx950).
 *
 * Method: M.J. Kronenburg, "A Method for Fast Diagonalization of a 2x2 or 3x3
 * Real Symmetric Matrix", arXiv:1306.6291.  For each matrix A the library finds
 * the eigenvalues from the characteristic polynomial (paper §3 for 2x2, §4 for
 * 3x3), solves the rotation angles from A = D Lambda D^T (§3, §5), forms
 * D = R(phi) (2x2, eq. (2.5)) or D = R1(phi1) R2(phi2) R3(phi3) (3x3, eq. (2.6))
 * and returns the angles, which are the Euler angles of the eigenvectors (§6).
 *
 * ---------------------------------------------------------------- conventions
 * Memory.  Every array argument is a DEVICE pointer owned by the caller.  The
 * library never allocates inside ksym_eig2, ksym_eig3, ksym_eig3_aos,
 * ksym_eig3_backward, ksym_plan_run / ksym_plan_replay or
 * ksym_mixed_run_noalloc.  ksym_plan_create allocates one small descriptor
 * buffer, freed by ksym_plan_destroy.
 *
 * Layout.  Structure of arrays: one contiguous plane of n elements per
 * quantity, element type float (KSYM_F32) or double (KSYM_F64), each plane
 * aligned to its element size.  A 3x3 input is the six planes of its unique
 * entries in the order {A11, A22, A33, A12, A13, A23}; a 2x2 input is
 * {A11, A22, A12}.  D is given as row-major planes {D11, D12, D13, D21, ...};
 * column k of D is the unit eigenvector of lam[k].
 *
 * Output slots.  3x3: lam = {max, min, mid}, the order in which eqs.
 * (4.10)-(4.12) produce lam1 >= lam3 >= lam2; det D = +1 always;
 * phi = {phi1, phi2, phi3} with D = R1(phi1) R2(phi2) R3(phi3),
 * phi1 in (-pi, pi], phi2 and phi3 in [-pi/2, pi/2].  2x2: lam = {lam1, lam2}
 * with lam1 the eigenvalue on A11's side (eqs. (3.2)-(3.3), sign(0) = +1),
 * D = R(phi), phi in [-pi/4, pi/4] (eq. (3.5)).
 *
 * Optional outputs.  Any output pointer (a whole pointer array, or one entry of
 * it) may be NULL: that quantity is not written.
 *
 * Errors.  Calls return ksym_status and never abort or throw.  n == 0 returns
 * KSYM_OK with nothing enqueued.  n < 0, a NULL required input, a pointer not
 * aligned to its element size, an output plane (or workspace) whose bytes
 * overlap those of an input or of another output, or an unknown dtype/path
 * are rejected before any HIP call (KSYM_E_ARG / KSYM_E_DTYPE).  Inputs may
 * share memory with each other.  Asynchronous kernel faults surface as
 * KSYM_E_HIP from a later call or from the caller's stream synchronisation.
 * Non-finite input entries are not an error: that matrix's outputs are NaN and
 * its flag has KSYM_FLAG_NONFINITE.
 * ksym_last_error() returns text for the last non-OK status of the calling
 * thread.
 *
 * Streams.  Work is enqueued on `stream` (a hipStream_t; NULL = the default
 * stream) without host synchronisation.  Calls are re-entrant; the library
 * keeps no mutable global state except a per-device cache of the CU count.
 *
 * Range.  Any finite input is accepted: each matrix is scaled by a power of
 * two (exactly) so that its largest entry lies in [1/2, 1) before any product
 * is formed, and the eigenvalues are scaled back.  Only an output beyond the
 * element type's range overflows (a 3x3 eigenvalue can reach 3 max|A_ij|,
 * a 2x2 one 2 max|A_ij|); outputs below the smallest normal number are
 * subnormal and lose precision gradually.
 */
#ifndef KSYM_H
#define KSYM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define KSYM_VERSION 100   /* 1.0.0 */

/* Element type of the planes.  A plain integer type (not an enum), so that
   any value a caller passes is a valid argument and an unknown one is
   rejected (KSYM_E_DTYPE) rather than undefined. */
typedef int32_t ksym_dtype;
enum { KSYM_F32 = 0, KSYM_F64 = 1 };

typedef enum {
    KSYM_OK = 0,
    KSYM_E_ARG = 1,          /* bad size, NULL required pointer, misalignment, aliasing */
    KSYM_E_DTYPE = 2,        /* unknown dtype, or dtype/path combination not offered */
    KSYM_E_WORKSPACE = 3,    /* workspace pointer NULL or smaller than required */
    KSYM_E_HIP = 4,          /* a HIP runtime call failed; see ksym_last_error() */
    KSYM_E_UNSUPPORTED = 5   /* option outside the compiled variants */
} ksym_status;

/* Per-matrix flag bits, written to the optional uint8 flags plane. */
#define KSYM_FLAG_GENERAL   0u   /* distinct computed eigenvalues: general branch of §5 */
#define KSYM_FLAG_DOUBLE    1u   /* two computed eigenvalues coincide to tau_dbl (special case q^2 = 4p^3 != 0 of §5) */
#define KSYM_FLAG_TRIPLE    2u   /* p = 0: triple eigenvalue, D = I, angles 0 (§5) */
#define KSYM_FLAG_FIXUP     4u   /* result rewritten by the float64 refinement */
#define KSYM_FLAG_NONFINITE 8u   /* an input entry was Inf or NaN; outputs are NaN */

/*
 * Numerical paths for the 3x3 forward.
 *  KSYM_PATH_FP32_FIXUP (dtype F32 only): float32 inputs and outputs; the
 *    cubic step (p, q, arccos, cos/sin, eqs. (4.7)-(4.12)) in float64; the angle
 *    solve of §5 in float32; a float32 a-posteriori check of D.  A result of
 *    the general branch that fails the check is computed again and checked
 *    again: for a diagonal matrix as the signed permutation of its axes, and
 *    where the middle eigenvalue lies within tau_res sqrt(p) of another (or
 *    the eigenvalues coincide) by the double-root branch of §5 (5.20)-(5.25).
 *    Matrices that still fail, or whose relative eigenvalue gap is
 *    below tau_gap, are rewritten by a float64 refinement (isolated
 *    eigenvector by cross products, Rayleigh-Ritz on its complement and one
 *    2x2 Jacobi rotation).  Differentiated calls (tau_vec > 0) refine every
 *    double root instead.
 *  KSYM_PATH_FP64_PLAIN (dtype F64 only): the paper's formulas in float64,
 *    including the double-root branch, with no check and no refinement.
 *  KSYM_PATH_FP64_FIXUP (dtype F64 only): as PLAIN, plus the float64 check and
 *    refinement with float64 thresholds.
 */
typedef enum {
    KSYM_PATH_DEFAULT = -1,     /* FP32_FIXUP for F32, FP64_FIXUP for F64 */
    KSYM_PATH_FP32_FIXUP = 0,
    KSYM_PATH_FP64_PLAIN = 1,
    KSYM_PATH_FP64_FIXUP = 2
} ksym_path;

/* Largest grid_mult (workgroups per compute unit): with 64-thread groups it
 * gives one tile per wave for a launch of up to 2^30 matrices, more than the
 * 2^28 of one launch chunk. */
#define KSYM_GRID_MULT_MAX 65536

/*
 * Launch and threshold options.  Fill with ksym_opts_default() and change
 * fields; a NULL ksym_opts* means the defaults.
 *   block          threads per workgroup: 64, 128, 256, 512 or 1024 (each
 *                  kernel is compiled for a subset; others give
 *                  KSYM_E_UNSUPPORTED).
 *   mats_per_lane  matrices each lane handles per tile: 1, 2 or 4 (3x3
 *                  kernels: 1 or 2).
 *   grid_mult      workgroups per compute unit of the grid-stride launch
 *                  (the grid is min(tiles, grid_mult * CUs));
 *                  1..KSYM_GRID_MULT_MAX.  The default KSYM_GRID_MULT_MAX
 *                  gives every wave one tile at any batch size, which
 *                  measured fastest: a wave that goes on to a further tile
 *                  waits for its previous stores along with the next loads
 *                  (one in-order counter covers both).
 *   tau_gap        relative eigenvalue gap min|lam_i - lam_j| / max|lam|
 *                  below which a matrix always takes the refinement (0 = off).
 *   tau_res        refinement if the residuals r_k = A d_k - lam_k d_k are too
 *                  large: float32 path, ||r_0||^2 + ||r_1||^2 > (tau_res
 *                  ||A||_F)^2 (the third residual then stays within sqrt(2)
 *                  tau_res ||A||_F, as it follows from the first two for
 *                  orthonormal D); float64 paths, some ||r_k|| > tau_res
 *                  ||A||_F.
 *   tau_vec        differentiated calls (0 = off): the first-order rotation
 *                  T_jk of each pair of columns of D against the true
 *                  eigenvectors, T_jk (lam_j - lam_k) = d_j^T A d_k -
 *                  (lam_j + lam_k)/2 d_j^T d_k, is evaluated in float64 and
 *                  removed from D (D (I - T)) and from the angles (which keep
 *                  D = R1 R2 R3 (phi) to first order); a matrix whose |T_jk|
 *                  or angle correction exceeds tau_vec is refined instead.
 *                  The adjoint multiplies eigenvector errors by
 *                  1/(lam_j - lam_k), so a small gap needs D accurate to far
 *                  below the float32 closed form's rounding level.
 *   drain_tiles    refinement queue age limit: each wavefront refines its
 *                  queued matrices once 64 are waiting or once the oldest has
 *                  waited this many of the wave's tiles, whichever comes
 *                  first (0 = only full waves).  Refined outputs overwrite
 *                  provisional ones; a short wait keeps those lines in cache.
 *   tau_dbl        relative split (min distance of the middle eigenvalue to
 *                  the others, divided by sqrt(p)) below which the computed
 *                  eigenvalues are taken as a double root (KSYM_FLAG_DOUBLE):
 *                  the plain path takes the paper's double-root branch; the
 *                  float64 checked path and differentiated calls route the
 *                  matrix to the refinement; the float32 path checks the
 *                  general branch's result and, if it fails, the double-root
 *                  branch's.  Default 1e-6 for F64; 1e-9 for F32, whose angle
 *                  solve takes its squared cosines from float64 quotients
 *                  and is checked anyway.
 * Negative thresholds (and drain_tiles < 0) select the dtype's default.
 */
typedef struct {
    int32_t path;
    int32_t block;
    int32_t mats_per_lane;
    int32_t grid_mult;
    double  tau_gap;
    double  tau_res;
    double  tau_vec;
    double  tau_dbl;
    int32_t drain_tiles;
    int32_t reserved;   /* set to 0 */
} ksym_opts;

/* Library version (KSYM_VERSION of the build). */
int ksym_version(void);

/* Text describing the calling thread's last non-OK status ("" if none).
   The pointer stays valid until that thread's next ksym call. */
const char *ksym_last_error(void);

/* Defaults for dtype (thresholds and launch shape). */
void ksym_opts_default(ksym_dtype dtype, ksym_opts *opts);

/*
 * 2x2 forward, paper §3.  in = {A11, A22, A12} (3 planes, required when n > 0).
 * lam = {lam1, lam2} (eqs. (3.2)-(3.3)), D = {D11, D12, D21, D22} = R(phi)
 * (eq. (2.5)), phi of eq. (3.5) evaluated as 1/2 atan2(2 A12 sign(A11 - A22),
 * |A11 - A22|) (the same value where A11 != A22, 0 when also A12 = 0).
 * flags: KSYM_FLAG_NONFINITE or 0.  Only opts->block and grid_mult are used.
 */
ksym_status ksym_eig2(ksym_dtype dtype, int64_t n, const void *const in[3],
                      void *const lam[2], void *const D[4], void *phi,
                      uint8_t *flags, const ksym_opts *opts, void *stream);

/*
 * Bytes of workspace ksym_eig3 / ksym_eig3_aos need (a few counters; the
 * refinement queue lives in on-chip memory).  Workspace layout: uint32 word 0
 * accumulates the number of refined matrices, word 1 the number of matrices
 * with non-finite input.  The caller zeroes it when it wants fresh counts
 * (ksym_zero_counters); the library only adds.
 */
size_t ksym_eig3_workspace_bytes(ksym_dtype dtype, int64_t n);

/* Zero the counter words of a workspace on `stream` (a kernel, so it may be
   captured in a HIP graph). */
ksym_status ksym_zero_counters(void *ws, size_t ws_bytes, void *stream);

/*
 * 3x3 forward, paper §4-§5 (see the path descriptions above).
 * in  = {A11, A22, A33, A12, A13, A23}: 6 planes, required when n > 0.
 * lam = 3 planes (slots max, min, mid), D = 9 planes (row-major), phi = 3 planes.
 * gap = optional 3 planes {lam1 - lam2, lam1 - lam3, lam3 - lam2} (max - min,
 *       max - mid, mid - min) evaluated in float64 before rounding: saved state
 *       for ksym_eig3_backward (NULL array = not written).
 * flags = optional uint8 plane (KSYM_FLAG_* bits).
 * ws  = workspace of ksym_eig3_workspace_bytes() bytes, or NULL (no counters).
 * Output arrays may be NULL, and so may single planes: those are not written.
 * Performance: planes are read and written in tiles of 64 (float32) or 32
 * (float64) consecutive elements per wavefront; output planes that start on
 * 256-byte boundaries keep every cache line within one tile, and measured
 * 30-40 % faster than output planes offset from that (input alignment
 * matters about 5 %).
 * Eigenvalues-only mode (KSYM_F32): when no plane of D and none of phi is
 * requested, a reduced kernel runs the float64 cubic stage of §4 alone (the
 * angle solve, the check and the refinement serve the eigenvectors) and
 * writes lam, gap and flags: bitwise the full path's for every matrix the
 * full path does not refine, within the float32 tolerance for the others;
 * KSYM_FLAG_FIXUP is never set and the refined counter stays 0.  It moves
 * 36 bytes per matrix instead of 84.
 */
ksym_status ksym_eig3(ksym_dtype dtype, int64_t n, const void *const in[6],
                      void *const lam[3], void *const D[9], void *const phi[3],
                      void *const gap[3], uint8_t *flags, void *ws, size_t ws_bytes,
                      const ksym_opts *opts, void *stream);

/*
 * 3x3 forward on array-of-structures input: a_aos holds n records of six
 * entries {A11, A22, A33, A12, A13, A23} (n x 6 contiguous, record stride 6
 * elements, base aligned to 16 bytes).  Each workgroup stages its records
 * through on-chip memory; outputs and everything else as ksym_eig3.
 */
ksym_status ksym_eig3_aos(ksym_dtype dtype, int64_t n, const void *a_aos,
                          void *const lam[3], void *const D[9], void *const phi[3],
                          void *const gap[3], uint8_t *flags, void *ws, size_t ws_bytes,
                          const ksym_opts *opts, void *stream);

/*
 * ksym_eig3_backward with the cotangent gphi (3 planes) of the Euler angles
 * phi (3 planes, as ksym_eig3 writes them; both required) added to those of
 * lam and D.  With D = R1 R2 R3 (eq. (2.6)) and R_k = exp(phi_k [e_k]x), the
 * body rates w of D^T dD = [w]x are w = M dphi, M's columns (c2 c3, -c2 s3,
 * s2), (s3, c3, 0), (0, 0, 1) (ck, sk: cosine and sine of phi_k); gphi acts
 * as M^-T gphi added to (E_32, E_13, E_21) of E = D^T gD.  M^-T divides by
 * c2 = cos phi2, which vanishes at gimbal lock; it is regularised as
 * c2 / (c2^2 + eps_rel^2).  The angles wrap at the ends of their ranges, where
 * they are not differentiable.  Otherwise as ksym_eig3_backward.
 */
ksym_status ksym_eig3_backward_angles(ksym_dtype dtype, int64_t n, const void *const lam[3],
                                      const void *const D[9], const void *const phi[3],
                                      const void *const gap[3], const void *const glam[3],
                                      const void *const gD[9], const void *const gphi[3], void *const gA[6],
                                      double eps_rel, void *stream);

/*
 * Inverse maps, from the definitions (2.5)-(2.6) (the other side of the
 * forward, not a step of the paper's method): A = D diag(lam) D^T with
 * D = R1(phi1) R2(phi2) R3(phi3) for 3x3, D = R(phi) for 2x2.  lam and phi are
 * laid out as ksym_eig3 / ksym_eig2 write them (any slot order of lam, as
 * long as phi describes the matching D); A receives the unique-entry planes
 * {A11, A22, A33, A12, A13, A23} or {A11, A22, A12}, the forward's input
 * layout.  For on-device generation and round trips.  All planes required.
 * Allocates nothing; asynchronous on `stream`.
 */
ksym_status ksym_compose3(ksym_dtype dtype, int64_t n, const void *const lam[3], const void *const phi[3],
                          void *const A[6], void *stream);
ksym_status ksym_compose2(ksym_dtype dtype, int64_t n, const void *const lam[2], const void *phi,
                          void *const A[3], void *stream);

/*
 * Adjoint of ksym_eig2 (not in the paper: first-order perturbation theory of
 * the symmetric eigenproblem, with D = R(phi) of eq. (2.5)).  From the forward
 * outputs lam (2 planes) and D (4 planes {D11, D12, D21, D22}, as ksym_eig2
 * writes them) and the cotangents glam (2 planes), gD (4 planes) and gphi (one
 * plane) of a scalar loss L, it writes the plane gradients gA = {dL/dA11,
 * dL/dA22, dL/dA12} (3 planes; A12 is one parameter, so the gradient of the
 * symmetric matrix is summed over both off-diagonal entries):
 *   E = D^T gD with E_21 += gphi (D^T dD = [[0, -dphi], [dphi, 0]]),
 *   Abar = D [diag(glam) + F o E] D^T,
 *   F_12 = -F_21 = (lam2 - lam1) / ((lam2 - lam1)^2 + eps^2), eps = eps_rel * ||lam||.
 * A NULL cotangent array or plane counts as zero; lam, D and gA are required.
 * phi is differentiable away from the ends of its range (where it wraps by pi
 * and D changes sign); gphi across such a wrap is the caller's matter.
 * Allocates nothing; asynchronous on `stream`.
 */
ksym_status ksym_eig2_backward(ksym_dtype dtype, int64_t n, const void *const lam[2],
                               const void *const D[4], const void *const glam[2], const void *const gD[4],
                               const void *gphi, void *const gA[3], double eps_rel, void *stream);

/*
 * 3x3 adjoint (not in the paper; first-order perturbation theory of the
 * symmetric eigenproblem).  From the saved forward outputs lam (3 planes) and D
 * (9 planes) and the cotangents glam = dL/dlam (3 planes) and gD = dL/dD
 * (9 planes), writes gA = dL/d(plane) for the six input planes:
 *   Abar = D [diag(glam) + F o (D^T gD)] D^T,
 *   F_ij = (lam_j - lam_i) / ((lam_j - lam_i)^2 + eps^2) (i != j), F_ii = 0,
 *   eps  = eps_rel * sqrt(lam1^2 + lam2^2 + lam3^2)  (= eps_rel * ||A||_F),
 *   gA_ii = Abar_ii, gA_ij = Abar_ij + Abar_ji (each off-diagonal plane feeds
 *   both A_ij and A_ji).
 * gap (optional, from ksym_eig3) supplies the eigenvalue differences in place
 * of differences of the rounded lam.  glam or gD NULL = zero cotangent.
 * gA: 6 planes, required.
 */
ksym_status ksym_eig3_backward(ksym_dtype dtype, int64_t n, const void *const lam[3],
                               const void *const D[9], const void *const gap[3],
                               const void *const glam[3], const void *const gD[9],
                               void *const gA[6], double eps_rel, void *stream);

/*
 * Mixed persistent batch: many groups of 2x2 or 3x3 matrices in one launch.
 * kind = 2 uses in[0..2], lam[0..1], D[0..3], phi[0]; kind = 3 uses the full
 * arrays as in ksym_eig3.  Pointers of unused slots are ignored.  When every
 * plane of every group (and every flags plane) starts on a 256-byte
 * boundary, each wave tile's part of a plane fills whole cache lines and the
 * launch streams its loads and stores (non-temporal policy); otherwise it
 * uses the default policy.  Results are the same either way.
 */
typedef struct {
    int32_t kind;          /* 2 or 3 */
    int64_t n;             /* matrices in this group (>= 0) */
    const void *in[6];
    void *lam[3];
    void *D[9];
    void *phi[3];
    uint8_t *flags;
} ksym_group;

typedef struct ksym_plan ksym_plan;

/*
 * Build a plan for `ngroups` groups (copied; the group array may be freed
 * afterwards, the device planes it points to may not).  Allocates the device
 * descriptor table (the only allocating call).  *ws_bytes receives the
 * workspace size ksym_plan_run needs.  Options with tau_vec > 0 give
 * KSYM_E_UNSUPPORTED (mixed batches are not differentiated).
 */
ksym_status ksym_plan_create(ksym_dtype dtype, int32_t ngroups, const ksym_group *groups,
                             const ksym_opts *opts, ksym_plan **plan, size_t *ws_bytes);

/* Enqueue the whole batch (counter reset kernel + one persistent kernel) on
   `stream`.  ws: NULL, or a 4-byte aligned workspace of ws_bytes >= the
   *ws_bytes that ksym_plan_create reported (its two counter words are
   zeroed, then accumulated as for ksym_eig3); a smaller or misaligned
   workspace gives KSYM_E_WORKSPACE.  No allocation, no synchronisation:
   safe under stream capture. */
ksym_status ksym_plan_run(ksym_plan *plan, void *ws, size_t ws_bytes, void *stream);

/* Capture ksym_plan_run(plan, ws, ws_bytes, stream) into a HIP graph held by
   the plan (replacing any previous one).  Not itself capturable. */
ksym_status ksym_plan_capture(ksym_plan *plan, void *ws, size_t ws_bytes, void *stream);

/* Launch the captured graph on `stream`. */
ksym_status ksym_plan_replay(ksym_plan *plan, void *stream);

/* Number of tiles and the grid size the plan launches (for reporting). */
ksym_status ksym_plan_info(const ksym_plan *plan, int64_t *tiles, int32_t *grid);

/* Free the plan, its descriptor table and its graph.  NULL is a no-op. */
void ksym_plan_destroy(ksym_plan *plan);

/*
 * Mixed batch without a plan, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Runs the same kernels, and gives bitwise the same outputs and
 * counters, as ksym_plan_create + ksym_plan_run on the same groups and
 * options, but allocates nothing: the descriptor and tile tables go into a
 * fixed device array of the library (about 17.8 MiB, one per GPU the library
 * runs on, held until the process ends), written on `stream` by small
 * kernels before the batch kernel.  Limits: at most KSYM_NOALLOC_MAX_GROUPS
 * groups, KSYM_NOALLOC_MAX_DESCRIPTORS chunks of at most 2^28 matrices (a
 * group counts one chunk per started 2^28 matrices, an empty group one), and
 * KSYM_NOALLOC_MAX_TILES wave tiles of 64 * mats_per_lane matrices (a group
 * rounds up to whole tiles; 2^21 tiles hold 2^27 matrices at one matrix per
 * lane).  Beyond them the call returns KSYM_E_ARG before any HIP call.
 * Arguments, checks and ws as for ksym_plan_create and ksym_plan_run.  Every
 * call on one GPU uses that GPU's one array and keeps the last call's tables
 * there: calls that overlap on one GPU (on different streams, or from
 * several threads) race and must be ordered by the caller; calls on one
 * stream are ordered by it.  The first call on a device looks up the array's
 * address there (hipGetSymbolAddress).
 */
#define KSYM_NOALLOC_MAX_GROUPS 4096
#define KSYM_NOALLOC_MAX_DESCRIPTORS 8192
#define KSYM_NOALLOC_MAX_TILES 2097152
ksym_status ksym_mixed_run_noalloc(ksym_dtype dtype, int32_t ngroups, const ksym_group *groups,
                                   const ksym_opts *opts, void *ws, size_t ws_bytes, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* KSYM_H */
