"""Helpers shared by the GPU tests: device transfer, the certified reference
and the float32-path acceptance checks (tolerances stated here, used by every
float32 parity test)."""

from __future__ import annotations

import numpy as np

import oracle
from tests import helpers as H

# Tolerances of the float32 + refinement path, relative to ||A||_F:
LAM_TOL_F32 = 2e-6          # |delta lam| per sorted eigenvalue
RES_TOL_F32 = 1e-5          # max_k ||A d_k - lam_k d_k||_2
ORTH_TOL_F32 = 1e-5         # max |D^T D - I|
DET_TOL_F32 = 1e-5          # |det D - 1|
VEC_GAP_F32 = 1e-2          # eigenvectors compared up to sign where g_rel >= this
VEC_TOL_F32 = 2.5e-5        # ... with ||d - (+-v)|| <= VEC_TOL_F32 / g_rel (residual-implied)
# float64 paths against the oracle:
LAM_TOL_F64 = 1e-12
RES_TOL_F64 = 1e-10
VEC_TOL_F64 = 1e-8


def to_dev(x, dtype):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).to(device="cuda", dtype=dtype)


def to_np(out):
    return {k: v.cpu().numpy() for k, v in out.items()}


def certified_reference(P64):
    """Eigenpairs of the stored (float64-promoted) matrices in the output slot
    order (max, min, mid): the oracle's result where it is certified -- its
    own float64 residual <= 1e-12 ||A||_F and its eigenvalues within
    1e-14 ||A||_F of the long-double Jacobi solver's -- else the Jacobi
    solver's eigenpairs.  Returns lam (3, n), V (9, n)."""
    o = oracle.eig3(P64)
    j = oracle.jacobi3(P64)
    res = H.residual3(P64, o["lam"], o["D"])
    lam_ok = H.sorted_lam_err(P64, o["lam"], j["lam"]) <= 1e-14
    use_j = ~((res <= 1e-12) & lam_ok)
    # Jacobi returns descending (max, mid, min): reorder to (max, min, mid)
    jl = j["lam"][[0, 2, 1]]
    jV = H.as_mats(j["V"])[:, :, [0, 2, 1]].reshape(-1, 9).T
    lam = np.where(use_j[None, :], jl, o["lam"])
    V = np.where(use_j[None, :], jV, o["D"])
    return lam, V


def check_f32_result(P, out, lam_ref, V_ref, label=""):
    """Acceptance of a float32 3x3 result against the certified reference.
    Returns a dict of error statistics (max values)."""
    P64 = np.asarray(P, dtype=np.float64)
    lam = out["lam"].astype(np.float64)
    D = out["D"].astype(np.float64)
    fro = H.fro3(P64)
    zero = fro == 0
    lam_err = H.sorted_lam_err(P64, lam, lam_ref)
    res = H.residual3(P64, lam, D)
    orth = H.orth_err(D)
    det = np.abs(H.det3(D) - 1)
    g = H.rel_gaps(lam_ref)
    ve = H.eigvec_err(lam, D, lam_ref, V_ref)
    # gap of each output slot: match it to the reference slot with the closest eigenvalue
    idx = np.argmin(np.abs(lam_ref[None, :, :] - lam[:, None, :]), axis=1)
    gk = np.take_along_axis(g, idx, axis=0)
    sel = gk >= VEC_GAP_F32
    vec_ratio = np.where(sel, ve * gk, 0.0)
    stats = {"lam": float(np.max(lam_err, initial=0)), "res": float(np.max(res, initial=0)),
             "orth": float(np.max(orth, initial=0)), "det": float(np.max(det, initial=0)),
             "vec_x_gap": float(np.max(vec_ratio, initial=0))}
    assert np.all(lam_err[~zero] <= LAM_TOL_F32), (label, stats)
    assert np.all(lam[:, zero] == 0), label
    assert np.all(res <= RES_TOL_F32), (label, stats, np.argmax(res))
    assert np.all(orth <= ORTH_TOL_F32), (label, stats)
    assert np.all(det <= DET_TOL_F32), (label, stats)
    assert np.all(vec_ratio <= VEC_TOL_F32), (label, stats)
    # slot order (max, min, mid)
    assert np.all(lam[0] >= lam[2]) and np.all(lam[2] >= lam[1]), label
    # angles reproduce D (eq. (2.6)) to float32 rounding
    R = H.rot_from_angles(out["phi"].astype(np.float64))
    assert np.abs(R - H.as_mats(D)).max() < 2e-5, label
    return stats
