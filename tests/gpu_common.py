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
    gk = np.stack([np.choose(H.nearest_slot(lam_ref, lam[k]), list(g)) for k in range(3)])
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
    if "phi" in out:
        R = H.rot_planes(out["phi"].astype(np.float64))
        assert np.abs(R - D).max() < 2e-5, label
    return stats


def check_f32_whole(P, out, label="", chunk=1 << 22):
    """check_f32_result over a whole batch, chunk by chunk against the
    certified reference of each chunk.  P: (6, n) float32 or float64 planes
    (host); out: host arrays lam (3, n), D (9, n) and optionally phi (3, n).
    Returns the largest statistics over the chunks."""
    n = P.shape[1]
    worst = {}
    for s in range(0, n, chunk):
        e = min(n, s + chunk)
        P64 = np.asarray(P[:, s:e], dtype=np.float64)
        g = {k: v[..., s:e] for k, v in out.items()}
        lam_ref, V_ref = certified_reference(P64)
        st = check_f32_result(P64, g, lam_ref, V_ref, f"{label} [{s}:{e}]")
        for k, v in st.items():
            worst[k] = max(worst.get(k, 0.0), v)
    return worst


def props3_gpu(A, lam, D, chunk=1 << 22):
    """Properties of a 3x3 result that hold at any batch size, evaluated on
    the device in float64 over every matrix: the largest residual
    max_k ||A d_k - lam_k d_k|| / ||A||_F, the largest |D^T D - I| and
    |det D - 1|, and whether every matrix keeps the slot order (max, min,
    mid).  A: (6, n) planes (A11, A22, A33, A12, A13, A23) or a view of
    them; lam (3, n); D (9, n) row-major."""
    import torch
    n = lam.shape[1]
    res_max, orth_max, det_max, order = 0.0, 0.0, 0.0, True
    eye = torch.eye(3, dtype=torch.float64, device=lam.device)
    for s in range(0, n, chunk):
        e = min(n, s + chunk)
        a11, a22, a33, a12, a13, a23 = A[:, s:e].double()
        M = torch.stack([torch.stack([a11, a12, a13], 1), torch.stack([a12, a22, a23], 1),
                         torch.stack([a13, a23, a33], 1)], 1)
        Dm = D[:, s:e].double().T.reshape(-1, 3, 3).contiguous()
        L = lam[:, s:e].double().T
        fro = torch.sqrt((M * M).sum((1, 2))).clamp_min(1e-300)
        r = torch.linalg.vector_norm(torch.bmm(M, Dm) - Dm * L[:, None, :], dim=1).amax(1) / fro
        assert torch.isfinite(r).all()
        res_max = max(res_max, float(r.max()))
        orth = (torch.bmm(Dm.transpose(1, 2).contiguous(), Dm) - eye).abs()
        orth_max = max(orth_max, float(orth.amax()))
        det = (Dm[:, 0, 0] * (Dm[:, 1, 1] * Dm[:, 2, 2] - Dm[:, 1, 2] * Dm[:, 2, 1])
               - Dm[:, 0, 1] * (Dm[:, 1, 0] * Dm[:, 2, 2] - Dm[:, 1, 2] * Dm[:, 2, 0])
               + Dm[:, 0, 2] * (Dm[:, 1, 0] * Dm[:, 2, 1] - Dm[:, 1, 1] * Dm[:, 2, 0]))
        det_max = max(det_max, float((det - 1).abs().max()))
        order = order and bool((L[:, 0] >= L[:, 2]).all()) and bool((L[:, 2] >= L[:, 1]).all())
    return {"res": res_max, "orth": orth_max, "det": det_max, "order": order}


def props2_gpu(A, lam, D, phi):
    """The 2x2 counterpart over every matrix, in float64 on the device: the
    largest residual relative to ||A||_F, the largest deviation of D from
    R(phi) = [[cos, -sin], [sin, cos]] (eq. (2.5)), and the largest |phi|.
    A: (3, n) planes (A11, A22, A12); lam (2, n); D (4, n); phi (n,)."""
    import torch
    if lam.shape[1] == 0:
        return {"res": 0.0, "rot": 0.0, "phi_abs": 0.0}
    a11, a22, a12 = A.double()
    M = torch.stack([torch.stack([a11, a12], 1), torch.stack([a12, a22], 1)], 1)
    Dm = D.double().T.reshape(-1, 2, 2).contiguous()
    L = lam.double().T
    fro = torch.sqrt((M * M).sum((1, 2))).clamp_min(1e-300)
    r = torch.linalg.vector_norm(torch.bmm(M, Dm) - Dm * L[:, None, :], dim=1).amax(1) / fro
    assert torch.isfinite(r).all()
    p = phi.double()
    c, s = torch.cos(p), torch.sin(p)
    rot = (D.double() - torch.stack([c, -s, s, c])).abs().amax()
    return {"res": float(r.max()), "rot": float(rot), "phi_abs": float(p.abs().max())}
