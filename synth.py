"""Seeded synthetic inputs for batched 2x2 / 3x3 real symmetric eigendecomposition.

This module only draws inputs.  It holds none of the method's arithmetic (no
characteristic polynomial, no angle solve): the CPU oracle under ``oracle/`` and
the HIP library both receive exactly the arrays produced here, so the two sides
see the same bits.

Every generator uses numpy's PCG64 (``numpy.random.default_rng``).  Inputs are
built in float64 and rounded once to the stored dtype; the stored, rounded
matrix is the truth every comparison uses.  Layout is structure-of-arrays: one
contiguous plane per unique entry, in the order A11, A22, A33, A12, A13, A23 for
3x3 and A11, A22, A12 for 2x2 (the unique entries of a symmetric A, paper §2).

Workload recipes (sizes are arguments so tests can use small instances of the
same shape and distribution):

* ``plain``      -- i.i.d. U[-1, 1] entries, float64, 3x3 and 2x2 batches.
* ``precision``  -- Q diag(lam) Q^T with Haar-random Q, lam ~ U[-1, 1]^3, with a
  10 % near-degenerate slice (relative gap log-uniform in [1e-7, 1e-3]), a 1 %
  exactly-repeated slice (90 % double, 10 % triple), diagonal matrices (half of
  them with a repeated entry) and zero matrices, positions shuffled; float32.
* ``mixed``      -- groups of 2x2 or 3x3 matrices with log-uniform group sizes
  rescaled to a fixed total, entries N(0, 1), float32.
* ``grad``       -- 3x3 with N(0, 1) entries, redrawn while the relative
  eigenvalue gap is below a bound; cotangents w ~ N(0,1) (3 planes) and
  G ~ N(0,1) (9 planes); float32.
* ``field``      -- a 3-D grid of SPD tensors R(x) diag(lam) R(x)^T with
  lam log-uniform in [1e-4, 1e-2], smoothly varying rotations R = exp([omega]x),
  omega a sum of random low-frequency Fourier modes, and 5 % isotropic voxels
  (lam * I exactly); array-of-structures [nx][ny][nz][6], float32.
"""

from __future__ import annotations

import numpy as np

BASE_SEED = 1306629

PLANES3 = ("a11", "a22", "a33", "a12", "a13", "a23")
PLANES2 = ("a11", "a22", "a12")


def _rng(seed):
    return np.random.default_rng(seed)


def haar_rotations(rng, n):
    """n rotation matrices uniform on SO(3) (unit quaternion from a normalised
    4-D standard normal), shape (n, 3, 3), float64."""
    q = rng.standard_normal((n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    w, x, y, z = q[:, 0], q[:, 1], q[:, 2], q[:, 3]
    R = np.empty((n, 3, 3))
    R[:, 0, 0] = 1 - 2 * (y * y + z * z)
    R[:, 0, 1] = 2 * (x * y - z * w)
    R[:, 0, 2] = 2 * (x * z + y * w)
    R[:, 1, 0] = 2 * (x * y + z * w)
    R[:, 1, 1] = 1 - 2 * (x * x + z * z)
    R[:, 1, 2] = 2 * (y * z - x * w)
    R[:, 2, 0] = 2 * (x * z - y * w)
    R[:, 2, 1] = 2 * (y * z + x * w)
    R[:, 2, 2] = 1 - 2 * (x * x + y * y)
    return R


def _sandwich(Q, lam):
    """Unique entries of Q diag(lam) Q^T, shape (6, n), float64."""
    # A_ij = sum_k Q_ik lam_k Q_jk
    def ent(i, j):
        return np.einsum("nk,nk,nk->n", Q[:, i, :], lam, Q[:, j, :])
    return np.stack([ent(0, 0), ent(1, 1), ent(2, 2), ent(0, 1), ent(0, 2), ent(1, 2)])


def planes3_from_full(A):
    """(n,3,3) symmetric -> (6, n) unique-entry planes."""
    return np.stack([A[:, 0, 0], A[:, 1, 1], A[:, 2, 2], A[:, 0, 1], A[:, 0, 2], A[:, 1, 2]])


def full_from_planes3(P):
    """(6, n) planes -> (n, 3, 3) symmetric, same dtype."""
    a11, a22, a33, a12, a13, a23 = P
    n = P.shape[1]
    A = np.empty((n, 3, 3), dtype=P.dtype)
    A[:, 0, 0], A[:, 1, 1], A[:, 2, 2] = a11, a22, a33
    A[:, 0, 1] = A[:, 1, 0] = a12
    A[:, 0, 2] = A[:, 2, 0] = a13
    A[:, 1, 2] = A[:, 2, 1] = a23
    return A


# ---------------------------------------------------------------------------
# plain: i.i.d. U[-1, 1]
# ---------------------------------------------------------------------------
def make_plain(n3=4096, n2=4096, seed=BASE_SEED + 0, dtype=np.float64):
    rng = _rng(seed)
    p3 = rng.uniform(-1.0, 1.0, size=(6, n3)).astype(dtype)
    p2 = rng.uniform(-1.0, 1.0, size=(3, n2)).astype(dtype)
    return {"planes3": np.ascontiguousarray(p3), "planes2": np.ascontiguousarray(p2)}


# ---------------------------------------------------------------------------
# precision: Haar-rotated spectra with controlled gaps
# ---------------------------------------------------------------------------
def make_precision(n=1 << 24, seed=BASE_SEED + 1, dtype=np.float32,
                   frac_near=0.10, frac_repeat=0.01, n_diag=None, n_zero=None,
                   return_kinds=False):
    """Returns (6, n) planes.  kinds (optional) labels each matrix:
    0 regular, 1 near-degenerate, 2 double, 3 triple, 4 diagonal, 5 zero."""
    rng = _rng(seed)
    if n_diag is None:
        n_diag = min(1 << 14, n // 1024)
    if n_zero is None:
        n_zero = min(1 << 10, n // 16384)
    n_near = int(round(frac_near * n))
    n_rep = int(round(frac_repeat * n))
    n_reg = n - n_near - n_rep - n_diag - n_zero
    assert n_reg >= 0
    lam = rng.uniform(-1.0, 1.0, size=(n, 3))
    kinds = np.zeros(n, dtype=np.int8)
    o = n_reg
    # near-degenerate: (a, a + s*g*M, c), g log-uniform in [1e-7, 1e-3]
    if n_near:
        a = rng.uniform(-1, 1, n_near)
        c = rng.uniform(-1, 1, n_near)
        g = np.exp(rng.uniform(np.log(1e-7), np.log(1e-3), n_near))
        s = rng.choice([-1.0, 1.0], n_near)
        M = np.maximum(np.abs(a), np.abs(c))
        L = np.stack([a, a + s * g * M, c], axis=1)
        L = np.take_along_axis(L, np.argsort(rng.random((n_near, 3)), axis=1), axis=1)
        lam[o:o + n_near] = L
        kinds[o:o + n_near] = 1
        o += n_near
    if n_rep:
        a = rng.uniform(-1, 1, n_rep)
        c = rng.uniform(-1, 1, n_rep)
        trip = rng.random(n_rep) < 0.10
        c = np.where(trip, a, c)
        L = np.stack([a, a, c], axis=1)
        L = np.take_along_axis(L, np.argsort(rng.random((n_rep, 3)), axis=1), axis=1)
        lam[o:o + n_rep] = L
        kinds[o:o + n_rep] = np.where(trip, 3, 2)
        o += n_rep
    Q = haar_rotations(rng, n)
    P = _sandwich(Q, lam)
    if n_diag:
        d = rng.uniform(-1, 1, size=(3, n_diag))
        half = n_diag // 2
        # half of the diagonal matrices repeat one entry
        j = rng.integers(0, 3, half)
        k = (j + 1 + rng.integers(0, 2, half)) % 3
        d[k, np.arange(half)] = d[j, np.arange(half)]
        P[:, o:o + n_diag] = 0.0
        P[0:3, o:o + n_diag] = d
        kinds[o:o + n_diag] = 4
        o += n_diag
    if n_zero:
        P[:, o:o + n_zero] = 0.0
        kinds[o:o + n_zero] = 5
        o += n_zero
    perm = rng.permutation(n)
    P = np.ascontiguousarray(P[:, perm].astype(dtype))
    if return_kinds:
        return P, kinds[perm]
    return P


# ---------------------------------------------------------------------------
# mixed: grouped 2x2 / 3x3 batches
# ---------------------------------------------------------------------------
def mixed_group_sizes(total=1 << 26, ngroups=1024, lo=1e3, hi=1e6, frac2=0.30,
                      seed=BASE_SEED + 2):
    """Group sizes log-uniform in [lo, hi], rescaled multiplicatively so they sum
    to ``total`` exactly; kinds assigned over a shuffled order, 2x2 until at least
    ``frac2`` of all matrices are 2x2, the rest 3x3.  Returns (sizes, kinds)."""
    rng = _rng(seed)
    raw = np.exp(rng.uniform(np.log(lo), np.log(hi), ngroups))
    s = np.maximum(1, np.floor(raw * (total / raw.sum()))).astype(np.int64)
    # distribute the rounding remainder one by one over the largest groups
    rem = total - int(s.sum())
    order = np.argsort(-raw)
    i = 0
    while rem != 0:
        g = order[i % ngroups]
        step = 1 if rem > 0 else -1
        if s[g] + step >= 1:
            s[g] += step
            rem -= step
        i += 1
    kinds = np.full(ngroups, 3, dtype=np.int32)
    acc = 0
    for g in rng.permutation(ngroups):
        if acc >= frac2 * total:
            break
        kinds[g] = 2
        acc += int(s[g])
    return s, kinds


def make_mixed(total=1 << 26, ngroups=1024, seed=BASE_SEED + 2, dtype=np.float32,
               lo=1e3, hi=1e6):
    """List of (kind, planes) with planes (3|6, n_g) N(0, 1)."""
    sizes, kinds = mixed_group_sizes(total, ngroups, lo, hi, seed=seed)
    rng = _rng(seed + 1000)
    out = []
    for s, k in zip(sizes, kinds):
        nplanes = 3 if k == 2 else 6
        out.append((int(k), rng.standard_normal((nplanes, int(s)), dtype=np.float32).astype(dtype)))
    return out


# ---------------------------------------------------------------------------
# grad: N(0,1) entries with a relative-gap floor, plus cotangents
# ---------------------------------------------------------------------------
def relative_gap(P):
    """min_{i<j} |lam_i - lam_j| / max_k |lam_k| of the stored matrices (float64,
    LAPACK eigenvalues).  Zero matrix -> 0."""
    lam = np.linalg.eigvalsh(full_from_planes3(P.astype(np.float64)))
    gaps = np.min(np.diff(lam, axis=1), axis=1)
    scale = np.max(np.abs(lam), axis=1)
    with np.errstate(invalid="ignore", divide="ignore"):
        g = np.where(scale > 0, gaps / scale, 0.0)
    return g


def make_grad(n=1 << 22, seed=BASE_SEED + 3, dtype=np.float32, min_gap=1e-3):
    rng = _rng(seed)
    P = rng.standard_normal((6, n)).astype(dtype)
    bad = relative_gap(P) < min_gap
    while bad.any():
        idx = np.nonzero(bad)[0]
        P[:, idx] = rng.standard_normal((6, idx.size)).astype(dtype)
        bad[idx] = relative_gap(P[:, idx]) < min_gap
    w = rng.standard_normal((3, n)).astype(dtype)
    G = rng.standard_normal((9, n)).astype(dtype)
    return {"planes3": np.ascontiguousarray(P), "w": w, "G": G}


# ---------------------------------------------------------------------------
# field: smooth SPD tensor field, AoS
# ---------------------------------------------------------------------------
def _rodrigues(omega):
    """exp([omega]_x) for omega of shape (n, 3)."""
    th = np.linalg.norm(omega, axis=1)
    with np.errstate(invalid="ignore", divide="ignore"):
        k = np.where(th[:, None] > 0, omega / th[:, None], 0.0)
    c, s = np.cos(th), np.sin(th)
    kx, ky, kz = k[:, 0], k[:, 1], k[:, 2]
    n = omega.shape[0]
    R = np.empty((n, 3, 3))
    C = 1 - c
    R[:, 0, 0] = c + kx * kx * C
    R[:, 0, 1] = kx * ky * C - kz * s
    R[:, 0, 2] = kx * kz * C + ky * s
    R[:, 1, 0] = ky * kx * C + kz * s
    R[:, 1, 1] = c + ky * ky * C
    R[:, 1, 2] = ky * kz * C - kx * s
    R[:, 2, 0] = kz * kx * C - ky * s
    R[:, 2, 1] = kz * ky * C + kx * s
    R[:, 2, 2] = c + kz * kz * C
    return R


def make_field(nx=256, ny=256, nz=256, seed=BASE_SEED + 4, dtype=np.float32,
               frac_iso=0.05, n_modes=8, kmax=4, chunk=1 << 20):
    """Returns dict with 'aos' (n, 6) float32 (n = nx*ny*nz, z fastest),
    'w' (3, n) and 'G' (9, n) cotangents, and 'iso' mask."""
    rng = _rng(seed)
    n = nx * ny * nz
    kvec = rng.integers(-kmax, kmax + 1, size=(3, n_modes, 3))
    amp = rng.normal(0.0, np.pi / 4, size=(3, n_modes))
    phase = rng.uniform(0, 2 * np.pi, size=(3, n_modes))
    lam = 10.0 ** rng.uniform(-4, -2, size=(n, 3))
    iso = rng.random(n) < frac_iso
    lam_iso = 10.0 ** rng.uniform(-4, -2, size=n)
    aos = np.empty((n, 6), dtype=dtype)
    for s0 in range(0, n, chunk):
        idx = np.arange(s0, min(n, s0 + chunk))
        x = (idx // (ny * nz)) / nx
        y = ((idx // nz) % ny) / ny
        z = (idx % nz) / nz
        pos = np.stack([x, y, z], axis=1) * 2 * np.pi
        om = np.zeros((idx.size, 3))
        for c in range(3):
            arg = pos @ kvec[c].T.astype(np.float64) + phase[c]
            om[:, c] = np.cos(arg) @ amp[c]
        R = _rodrigues(om)
        P = _sandwich(R, lam[idx])
        isoc = iso[idx]
        if isoc.any():
            P[:, isoc] = 0.0
            P[0:3, isoc] = lam_iso[idx][isoc]
        aos[idx] = P.T.astype(dtype)
    w = rng.standard_normal((3, n)).astype(dtype)
    G = rng.standard_normal((9, n)).astype(dtype)
    return {"aos": aos, "w": w, "G": G, "iso": iso}
