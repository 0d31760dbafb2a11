"""Shared checks for the tests: residuals, orthogonality, sign-aligned
eigenvector comparison and rotation products.  Nothing here computes an
eigendecomposition; these are the properties any correct result must have."""

from __future__ import annotations

import numpy as np

import synth


def full3(P):
    return synth.full_from_planes3(np.asarray(P, dtype=np.float64))


def fro3(P):
    """||A||_F of each matrix from its six unique-entry planes (float64)."""
    P = np.asarray(P, dtype=np.float64)
    return np.sqrt(P[0] ** 2 + P[1] ** 2 + P[2] ** 2 + 2 * (P[3] ** 2 + P[4] ** 2 + P[5] ** 2))


def as_mats(D9):
    """(9, n) row-major planes -> (n, 3, 3)."""
    return np.asarray(D9, dtype=np.float64).T.reshape(-1, 3, 3)


def _cols(D9):
    """The three columns of row-major D planes (9, n): cols[k][i] = D_ik."""
    D = np.asarray(D9, dtype=np.float64)
    return [(D[k], D[3 + k], D[6 + k]) for k in range(3)]


def residual3(P, lam, D9):
    """max_k ||A d_k - lam_k d_k||_2 / ||A||_F per matrix (0/0 -> 0), plane
    by plane."""
    a11, a22, a33, a12, a13, a23 = np.asarray(P, dtype=np.float64)
    L = np.asarray(lam, dtype=np.float64)
    r = np.zeros(a11.shape)
    for k, (x, y, z) in enumerate(_cols(D9)):
        r1 = a11 * x + a12 * y + a13 * z - L[k] * x
        r2 = a12 * x + a22 * y + a23 * z - L[k] * y
        r3 = a13 * x + a23 * y + a33 * z - L[k] * z
        r = np.maximum(r, np.sqrt(r1 * r1 + r2 * r2 + r3 * r3))
    f = fro3(P)
    with np.errstate(invalid="ignore", divide="ignore"):
        out = np.where(f > 0, r / np.where(f > 0, f, 1), r)
    return out


def orth_err(D9):
    """max_ij |(D^T D - I)_ij| per matrix."""
    c = _cols(D9)
    e = np.zeros(c[0][0].shape)
    for i in range(3):
        for j in range(i, 3):
            dot = c[i][0] * c[j][0] + c[i][1] * c[j][1] + c[i][2] * c[j][2]
            e = np.maximum(e, np.abs(dot - (1.0 if i == j else 0.0)))
    return e


def det3(D9):
    d = np.asarray(D9, dtype=np.float64)
    return (d[0] * (d[4] * d[8] - d[5] * d[7]) - d[1] * (d[3] * d[8] - d[5] * d[6])
            + d[2] * (d[3] * d[7] - d[4] * d[6]))


def rot_planes(phi):
    """R1(phi1) R2(phi2) R3(phi3) with the rotation matrices of paper §2
    (eqs. (2.6)-(2.9)) as row-major planes: phi (3, n) -> (9, n).  The
    product is formed as two 3x3 multiplications, entry by entry."""
    p1, p2, p3 = np.asarray(phi, dtype=np.float64)
    c1, s1, c2, s2, c3, s3 = np.cos(p1), np.sin(p1), np.cos(p2), np.sin(p2), np.cos(p3), np.sin(p3)
    z, o = np.zeros_like(p1), np.ones_like(p1)
    R1 = [[o, z, z], [z, c1, -s1], [z, s1, c1]]
    R2 = [[c2, z, s2], [z, o, z], [-s2, z, c2]]
    R3 = [[c3, -s3, z], [s3, c3, z], [z, z, o]]

    def mul(X, Y):
        return [[X[i][0] * Y[0][j] + X[i][1] * Y[1][j] + X[i][2] * Y[2][j] for j in range(3)] for i in range(3)]

    R = mul(mul(R1, R2), R3)
    return np.stack([R[i][j] for i in range(3) for j in range(3)])


def rot_from_angles(phi):
    """rot_planes as (n, 3, 3) matrices."""
    return as_mats(rot_planes(phi))


def sort3(L):
    """The three rows of L (3, n) sorted ascending per column (a min/max
    network)."""
    a, b, c = np.asarray(L, dtype=np.float64)
    lo1, hi1 = np.minimum(a, b), np.maximum(a, b)
    lo, mid1 = np.minimum(lo1, c), np.maximum(lo1, c)
    mid, hi = np.minimum(mid1, hi1), np.maximum(mid1, hi1)
    return np.stack([lo, mid, hi])


def sorted_lam_err(P, lam, lam_ref):
    """max |sorted(lam) - sorted(lam_ref)| / ||A||_F per matrix."""
    a = sort3(lam)
    b = sort3(lam_ref)
    f = fro3(P)
    e = np.abs(a - b).max(axis=0)
    with np.errstate(invalid="ignore", divide="ignore"):
        return np.where(f > 0, e / np.where(f > 0, f, 1), e)


def rel_gaps(lam_ref):
    """Per matrix and per eigenvalue slot: distance to the nearest other
    eigenvalue divided by max |lam|.  lam_ref (3, n) -> (3, n)."""
    L = np.asarray(lam_ref, dtype=np.float64)
    scale = np.abs(L).max(axis=0)
    g = np.empty_like(L)
    for k in range(3):
        others = [j for j in range(3) if j != k]
        g[k] = np.minimum(np.abs(L[k] - L[others[0]]), np.abs(L[k] - L[others[1]]))
    with np.errstate(invalid="ignore", divide="ignore"):
        return np.where(scale > 0, g / np.where(scale > 0, scale, 1), 0.0)


def nearest_slot(lam_ref, x):
    """Per column: the row j of lam_ref (3, n) closest to x (n,) (the first
    on ties)."""
    R = np.asarray(lam_ref, dtype=np.float64)
    d = np.abs(R - np.asarray(x, dtype=np.float64)[None, :])
    j = np.where(d[1] < d[0], 1, 0)
    best = np.minimum(d[0], d[1])
    return np.where(d[2] < best, 2, j)


def eigvec_err(lam, D9, lam_ref, V9):
    """For every slot k of (lam, D): find the reference column with the closest
    eigenvalue and return min over sign of ||d_k -+ v||_2.  (3, n)."""
    L = np.asarray(lam, dtype=np.float64)
    dc = _cols(D9)
    vc = _cols(V9)
    out = np.empty(L.shape)
    for k in range(3):
        j = nearest_slot(lam_ref, L[k])
        v = [np.choose(j, [vc[0][i], vc[1][i], vc[2][i]]) for i in range(3)]
        m = sum((dc[k][i] - v[i]) ** 2 for i in range(3))
        p = sum((dc[k][i] + v[i]) ** 2 for i in range(3))
        out[k] = np.sqrt(np.minimum(m, p))
    return out


def p_invariant(P):
    """p of the depressed cubic, (4.7), evaluated in float64."""
    P = np.asarray(P, dtype=np.float64)
    return (0.5 * ((P[0] - P[1]) ** 2 + (P[0] - P[2]) ** 2 + (P[1] - P[2]) ** 2)
            + 3 * (P[3] ** 2 + P[4] ** 2 + P[5] ** 2))


def literal_q_lam_tol(P, c=16.0, eps=2.220446049250313e-16):
    """Relative eigenvalue tolerance for the float64 closed form with the
    literal q of (4.8): its O(||A||^3) terms cancel to O(p^(3/2)), so the
    error scales like eps * (1 + ||A||_F^2 / p)."""
    f = fro3(P)
    p = p_invariant(P)
    with np.errstate(invalid="ignore", divide="ignore"):
        return np.where(p > 0, c * eps * (1 + f ** 2 / np.where(p > 0, p, 1)), c * eps)


def closed_form_lam_tol(P, lam_ref, c=16.0, eps=2.220446049250313e-16):
    """literal_q_lam_tol plus the near-double-root term of the trigonometric
    solution: where two eigenvalues are a gap g apart, arccos in (4.9) has slope
    1/sin(Delta) with sin(Delta) ~ g / sqrt(p), which turns an O(eps) error in
    q / (2 sqrt(p^3)) into an eigenvalue error of order eps * p / g."""
    f = fro3(P)
    p = p_invariant(P)
    L = np.sort(np.asarray(lam_ref, dtype=np.float64), axis=0)
    g = np.minimum(L[1] - L[0], L[2] - L[1])
    with np.errstate(invalid="ignore", divide="ignore"):
        extra = np.where(g > 0, p / (np.where(f > 0, f, 1) * np.where(g > 0, g, 1)), np.inf)
    return literal_q_lam_tol(P, c, eps) + c * eps * extra
