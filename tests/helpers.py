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


def residual3(P, lam, D9):
    """max_k ||A d_k - lam_k d_k||_2 / ||A||_F per matrix (0/0 -> 0)."""
    A = full3(P)
    D = as_mats(D9)
    L = np.asarray(lam, dtype=np.float64).T
    r = np.linalg.norm(A @ D - D * L[:, None, :], axis=1).max(axis=1)
    f = fro3(P)
    with np.errstate(invalid="ignore", divide="ignore"):
        out = np.where(f > 0, r / np.where(f > 0, f, 1), r)
    return out


def orth_err(D9):
    D = as_mats(D9)
    return np.abs(np.einsum("nki,nkj->nij", D, D) - np.eye(3)).max(axis=(1, 2))


def det3(D9):
    return np.linalg.det(as_mats(D9))


def rot_from_angles(phi):
    """R1(phi1) R2(phi2) R3(phi3) with the rotation matrices of paper §2
    (eqs. (2.6)-(2.9)); phi (3, n) -> (n, 3, 3)."""
    p1, p2, p3 = np.asarray(phi, dtype=np.float64)
    n = p1.size
    c1, s1, c2, s2, c3, s3 = np.cos(p1), np.sin(p1), np.cos(p2), np.sin(p2), np.cos(p3), np.sin(p3)
    z, o = np.zeros(n), np.ones(n)
    R1 = np.stack([np.stack([o, z, z], 1), np.stack([z, c1, -s1], 1), np.stack([z, s1, c1], 1)], 1)
    R2 = np.stack([np.stack([c2, z, s2], 1), np.stack([z, o, z], 1), np.stack([-s2, z, c2], 1)], 1)
    R3 = np.stack([np.stack([c3, -s3, z], 1), np.stack([s3, c3, z], 1), np.stack([z, z, o], 1)], 1)
    return R1 @ R2 @ R3


def sorted_lam_err(P, lam, lam_ref):
    """max |sorted(lam) - sorted(lam_ref)| / ||A||_F per matrix."""
    a = np.sort(np.asarray(lam, dtype=np.float64), axis=0)
    b = np.sort(np.asarray(lam_ref, dtype=np.float64), axis=0)
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


def eigvec_err(lam, D9, lam_ref, V9):
    """For every slot k of (lam, D): find the reference column with the closest
    eigenvalue and return min over sign of ||d_k -+ v||_2.  (3, n)."""
    L = np.asarray(lam, dtype=np.float64)
    R = np.asarray(lam_ref, dtype=np.float64)
    D = as_mats(D9)
    V = as_mats(V9)
    n = L.shape[1]
    out = np.empty((3, n))
    for k in range(3):
        j = np.argmin(np.abs(R - L[k][None, :]), axis=0)
        v = V[np.arange(n), :, j]
        d = D[:, :, k]
        out[k] = np.minimum(np.linalg.norm(d - v, axis=1), np.linalg.norm(d + v, axis=1))
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
