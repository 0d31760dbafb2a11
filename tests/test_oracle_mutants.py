"""Planted mistakes in the oracle must fail the pins.

Each case copies the oracle's C source, plants one plausible slip (a wrong
index, sign, coefficient, operand order or comparison), compiles it with gcc
into a temporary library and runs a compact version of the pin suite against
it.  The unmodified source must pass every check; every mutant must fail at
least one.  CPU only.
"""

import ctypes
import json
import os
import subprocess
import tempfile

import numpy as np
import pytest

import oracle
import synth
from tests import helpers as H

SRC = open(os.path.join(os.path.dirname(oracle.__file__), "ksym_oracle.c")).read()

MUTANTS = [
    ("q wrong index", "27.0 * (a11 * a23 * a23", "27.0 * (a11 * a13 * a23"),
    ("p wrong coefficient", "3.0 * (a12 * a12 + a13 * a13 + a23 * a23);", "2.0 * (a12 * a12 + a13 * a13 + a23 * a23);"),
    ("q dropped term", "+\n               2.0 * (a11 * a11 * a11", "+\n               0.0 * (a11 * a11 * a11"),
    ("lam2 wrong branch", "cos((Delta + 2.0 * KO_PI) / 3.0)", "cos((Delta - 2.0 * KO_PI) / 3.0)"),
    ("v wrong sign", "(a11 + l3 - l1 - l2)) / den", "(a11 - l3 - l1 - l2)) / den"),
    ("w swapped gap", "(a11 - l3 + (l3 - l2) * v)", "(a11 - l3 + (l2 - l3) * v)"),
    ("g1 cos->sin", "0.5 * (l1 - l2) * cos(p2) * sin(2.0 * p3)", "0.5 * (l1 - l2) * sin(p2) * sin(2.0 * p3)"),
    ("g2 v<->w", "(1.0 + (v - 2.0) * w)", "(1.0 + (w - 2.0) * v)"),
    ("f2 sign", "-2.0 * a23 + 0.0", "2.0 * a23 + 0.0"),
    ("f1 index", "{a12 + 0.0, -a13 + 0.0}", "{a12 + 0.0, -a23 + 0.0}"),
    ("selection inverted", "if (delta < best) {\n                best = delta;\n                chosen = c;\n                p1 = (f1n >= f2n) ? e1 : e2;                         /* (5.15) */",
     "if (best == INFINITY || delta > best) {\n                best = delta;\n                chosen = c;\n                p1 = (f1n >= f2n) ? e1 : e2;                         /* (5.15) */"),
    ("selection mod pi", "double delta = fabs(remainder(e1 - e2, 2.0 * KO_PI));   /* R-select */",
     "double delta = fabs(remainder(e1 - e2, KO_PI));   /* R-select */"),
    ("phi1 choice swapped", "p1 = (f1n >= f2n) ? e1 : e2;                         /* (5.15) */",
     "p1 = (f1n >= f2n) ? e2 : e1;                         /* (5.15) */"),
    ("psi rotation sign", "rot2(-psi1, R);", "rot2(psi1, R);"),
    ("R2 transposed", "{{c, 0, s}, {0, 1, 0}, {-s, 0, c}}", "{{c, 0, -s}, {0, 1, 0}, {s, 0, c}}"),
    ("Euler product order", "matmul3(R1, R2, D);\n    matmul3(D, R3, D);", "matmul3(R3, R2, D);\n    matmul3(D, R1, D);"),
    ("double s wrong eigenvalue", "clamp01((a11 - ls) / (lm - ls))", "clamp01((a11 - lm) / (lm - ls))"),
    ("double slot det", "E[i][2] = -D[i][1];", "E[i][2] = D[i][1];"),
    ("double returns the pair's mean", "    lam[0] = l1; lam[1] = l2; lam[2] = l3;\n    D_to_euler(E, phi);",
     "    if (ls > lm) { lam[0] = ls; lam[1] = lm; lam[2] = lm; }\n"
     "    else { lam[0] = lm; lam[1] = ls; lam[2] = lm; }\n    D_to_euler(E, phi);"),
    ("eig2 phi factor", "f = 0.5 * atan(2.0 * a12 / d);", "f = 0.5 * atan(a12 / d);"),
    ("eig2 lam2 sign", "lam[1] = 0.5 * (a11 + a22 - sg * root);", "lam[1] = 0.5 * (a11 + a22 + sg * root);"),
    ("eig2 sign(0)", "double sg = (d >= 0.0) ? 1.0 : -1.0;", "double sg = (d > 0.0) ? 1.0 : -1.0;"),
    ("bwd transposed E", "M[i][j] = (d != 0.0 ? d / (d * d + eps * eps) : 0.0) * E[i][j];",
     "M[i][j] = (d != 0.0 ? d / (d * d + eps * eps) : 0.0) * E[j][i];"),
    ("bwd off-diagonal plane", "gA[4] = Abar[0][2] + Abar[2][0];", "gA[4] = Abar[0][2] + Abar[0][2];"),
    ("bwd gap sign", "double d = lam[j] - lam[i];", "double d = lam[i] - lam[j];"),
    ("eig2 bwd angle slot", "E[1][0] += gphi;", "E[0][1] += gphi;"),
    ("eig2 bwd off-diagonal plane", "gA[2] = Abar[0][1] + Abar[1][0];", "gA[2] = Abar[0][1];"),
    ("eig2 bwd E transposed", "E[i][j] = D[0][i] * G[0][j] + D[1][i] * G[1][j];",
     "E[i][j] = D[i][0] * G[0][j] + D[i][1] * G[1][j];"),
    ("compose3 transposed", "s += D[i][k] * lam[k] * D[j][k];", "s += D[k][i] * lam[k] * D[k][j];"),
    ("compose2 angle sign", "const double D[2][2] = {{c, -s}, {s, c}};", "const double D[2][2] = {{c, s}, {-s, c}};"),
    ("bwd angle column sign", "E[0][2] += -s3 * u + c3 * v;", "E[0][2] += s3 * u + c3 * v;"),
    ("bwd angle gimbal term", "const double u = (gphi[0] - s2 * gphi[2]) * c2",
     "const double u = (gphi[0] + s2 * gphi[2]) * c2"),
    ("compose3 plane order", "A[4] = M[0][2];\n    A[5] = M[1][2];", "A[4] = M[1][2];\n    A[5] = M[0][2];"),
]


def _compile(src, tmp):
    c = os.path.join(tmp, "m.c")
    so = os.path.join(tmp, "m.so")
    open(c, "w").write(src)
    subprocess.run(["gcc", *oracle.CFLAGS, "-o", so, c, "-lm", "-lpthread"], check=True)
    return so


def _pins():
    """Compact pin suite over the oracle module's current library."""
    fails = []
    # 3x3 random: eigenvalues vs LAPACK, residual, orthogonality, det, angles
    P = synth.make_plain(2000, 16, seed=501)["planes3"]
    o = oracle.eig3(P)
    ref = np.linalg.eigvalsh(H.full3(P)).T
    if not np.all(H.sorted_lam_err(P, o["lam"], ref) < H.closed_form_lam_tol(P, ref)):
        fails.append("lam vs lapack")
    if not H.residual3(P, o["lam"], o["D"]).max() < 1e-10:
        fails.append("residual")
    if not H.orth_err(o["D"]).max() < 1e-14 or not np.abs(H.det3(o["D"]) - 1).max() < 1e-14:
        fails.append("orthogonality/det")
    if not np.abs(H.rot_from_angles(o["phi"]) - H.as_mats(o["D"])).max() < 1e-13:
        fails.append("angles")
    # golden 3x3 (double / triple / structured)
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "eig3_exact.json")))
    for c in gold["cases"]:
        A = np.array(c["a"], dtype=np.float64)[:, None]
        g = oracle.eig3(A)
        if not np.allclose(g["lam"][:, 0], c["lam"], atol=1e-12):
            fails.append("golden3 lam")
            break
        if not H.residual3(A, g["lam"], g["D"]).max() < 1e-7 or abs(H.det3(g["D"])[0] - 1) > 1e-12:
            fails.append("golden3 D")
            break
    # rotated doubles
    rng = np.random.default_rng(502)
    a, cc = rng.uniform(-1, 1, 500), rng.uniform(-1, 1, 500)
    keep = np.abs(a - cc) > 0.2
    lam = np.stack([a[keep], a[keep], cc[keep]], 1)
    Pd = synth._sandwich(synth.haar_rotations(rng, lam.shape[0]), lam)
    od = oracle.eig3(Pd)
    if not H.residual3(Pd, od["lam"], od["D"]).max() < 1e-6 or not np.abs(H.det3(od["D"]) - 1).max() < 1e-12:
        fails.append("double")
    # near doubles (split 2e-7 .. 8e-7 of the spread, centred spectra): the
    # double branch keeps the roots, within the trigonometric error bound
    a = rng.uniform(0.5, 1, 500) * rng.choice([-1, 1], 500)
    cc = -a * rng.uniform(0.5, 1, 500)
    sp = np.exp(rng.uniform(np.log(2e-7), np.log(8e-7), 500)) * np.abs(a - cc)
    Pn = synth._sandwich(synth.haar_rotations(rng, 500), np.stack([a, a + sp, cc], 1))
    on = oracle.eig3(Pn)
    Ln = np.sort(np.linalg.eigvalsh(H.full3(Pn)).T, axis=0)
    fn, pn = H.fro3(Pn), H.p_invariant(Pn)
    gn = np.minimum(Ln[1] - Ln[0], Ln[2] - Ln[1])
    tol = 2 * 2.220446049250313e-16 * (1 + fn ** 2 / pn) * (1 + pn / (fn * gn))
    if not np.all(H.sorted_lam_err(Pn, on["lam"], Ln) <= tol):
        fails.append("near double")
    # 2x2 golden and residual
    g2 = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "eig2_exact.json")))["cases"]
    P2 = np.array([c["a"] for c in g2], dtype=np.float64).T
    o2 = oracle.eig2(P2)
    for i, c in enumerate(g2):
        phi = float(eval(c["phi"], {"pi": np.pi, "atan": np.arctan}))
        if not (np.allclose(o2["lam"][:, i], c["lam"], atol=1e-14) and abs(o2["phi"][i] - phi) < 1e-14):
            fails.append("golden2")
            break
    # adjoint vs central differences of the long-double Jacobi forward
    d = synth.make_grad(60, seed=503, dtype=np.float64, min_gap=5e-2)
    Pg, w, G = d["planes3"], d["w"].astype(np.float64), d["G"].astype(np.float64)
    j0 = oracle.jacobi3(Pg)
    gA = oracle.eig3_bwd(j0["lam"], j0["V"], w, G, 0.0)
    V0 = H.as_mats(j0["V"])

    def loss(Pp):
        j = oracle.jacobi3(Pp)
        V = H.as_mats(j["V"])
        V = V * np.sign(np.einsum("nik,nik->nk", V, V0))[:, None, :]
        return (w * j["lam"]).sum(0) + (G * V.reshape(-1, 9).T).sum(0)

    h = 1e-6
    fd = np.empty_like(gA)
    for k in range(6):
        Pp, Pm = Pg.copy(), Pg.copy()
        Pp[k] += h
        Pm[k] -= h
        fd[k] = (loss(Pp) - loss(Pm)) / (2 * h)
    if not (np.linalg.norm(fd - gA, axis=0) / np.linalg.norm(gA, axis=0)).max() < 1e-6:
        fails.append("adjoint")
    # 2x2 adjoint (lam, D and phi cotangents) vs central differences of the 2x2 forward
    rng2 = np.random.default_rng(504)
    P2r = rng2.uniform(-1, 1, (3, 200))
    f2 = oracle.eig2(P2r)
    w2, G2, g2c = rng2.standard_normal((2, 200)), rng2.standard_normal((4, 200)), rng2.standard_normal(200)
    gA2 = oracle.eig2_bwd(f2["lam"], f2["D"], w2, G2, g2c, eps=0.0)

    def loss2(Pp):
        f = oracle.eig2(Pp)
        return (w2 * f["lam"]).sum(0) + (G2 * f["D"]).sum(0) + g2c * f["phi"]

    fd2 = np.empty_like(gA2)
    for k in range(3):
        Pp, Pm = P2r.copy(), P2r.copy()
        Pp[k] += h
        Pm[k] -= h
        fd2[k] = (loss2(Pp) - loss2(Pm)) / (2 * h)
    sm = np.all(np.abs(fd2) < 1e3, axis=0) & (np.abs(f2["lam"][0] - f2["lam"][1]) > 0.05)
    if sm.sum() < 150:
        fails.append("adjoint2 (forward too rough)")
    elif not (np.linalg.norm(fd2 - gA2, axis=0)[sm] / np.linalg.norm(gA2, axis=0)[sm]).max() < 1e-6:
        fails.append("adjoint2")
    # angle cotangents of the 3x3 adjoint vs central differences of the forward's angles
    da = synth.make_grad(120, seed=506, dtype=np.float64, min_gap=5e-2)
    Pa = da["planes3"]
    oa = oracle.eig3(Pa)
    gpa = np.random.default_rng(507).standard_normal((3, Pa.shape[1]))
    gAa = oracle.eig3_bwd(oa["lam"], oa["D"], None, None, eps=0.0, phi=oa["phi"], gphi=gpa)
    fda = np.empty_like(gAa)
    for k in range(6):
        Pp, Pm = Pa.copy(), Pa.copy()
        Pp[k] += h
        Pm[k] -= h
        fda[k] = ((gpa * oracle.eig3(Pp)["phi"]).sum(0) - (gpa * oracle.eig3(Pm)["phi"]).sum(0)) / (2 * h)
    pa = oa["phi"]
    oka = ((np.cos(pa[1]) > 0.2) & (np.abs(np.abs(pa[0]) - np.pi) > 0.1)
           & (np.abs(np.abs(pa[2]) - np.pi / 2) > 0.1) & np.all(np.abs(fda) < 1e3, axis=0))
    if oka.sum() < 40:
        fails.append("adjoint angles (too few smooth cases)")
    elif not (np.linalg.norm(fda - gAa, axis=0)[oka] / np.linalg.norm(gAa, axis=0)[oka]).max() < 1e-5:
        fails.append("adjoint angles")
    # inverse maps: round trips through the forward
    Pc = synth.make_plain(300, 16, seed=505)["planes3"]
    oc = oracle.eig3(Pc)
    err = np.abs(oracle.compose3(oc["lam"], oc["phi"]) - Pc).max(0) / H.fro3(Pc)
    if not np.all(err <= 4 * H.residual3(Pc, oc["lam"], oc["D"]) + 1e-13):
        fails.append("compose3")
    o2c = oracle.eig2(P2r)
    if not np.abs(oracle.compose2(o2c["lam"], o2c["phi"]) - P2r).max() < 1e-14:
        fails.append("compose2")
    return fails


def _with_lib(path):
    saved = oracle._lib
    oracle._lib = None
    lib = ctypes.CDLL(path)
    # reuse the module's signatures by loading through the same setter
    oracle._lib = lib
    P = ctypes.c_void_p
    i64, dbl, cint = ctypes.c_int64, ctypes.c_double, ctypes.c_int
    lib.ko_eig3_batch.argtypes = [i64, P, P, P, P, P, dbl, cint]
    lib.ko_eig2_batch.argtypes = [i64, P, P, P, P, cint]
    lib.ko_jacobi3_batch.argtypes = [i64, P, P, P, P, cint]
    lib.ko_eig3_bwd_batch.argtypes = [i64, P, P, P, P, P, P, P, dbl, dbl, cint]
    lib.ko_eig2_bwd_batch.argtypes = [i64, P, P, P, P, P, P, dbl, cint]
    lib.ko_compose3_batch.argtypes = [i64, P, P, P, cint]
    lib.ko_compose2_batch.argtypes = [i64, P, P, P, cint]
    lib.ko_eig3_dbg.argtypes = [P, dbl, P, P, P, P]
    lib.ko_eig3_dbg.restype = cint
    try:
        return _pins()
    finally:
        oracle._lib = saved


def test_unmodified_oracle_passes_compact_pins():
    with tempfile.TemporaryDirectory() as tmp:
        assert _with_lib(_compile(SRC, tmp)) == []


@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_planted_mistake_is_caught(name, old, new):
    assert SRC.count(old) >= 1, f"mutation anchor not found: {name}"
    src = SRC.replace(old, new, 1)
    with tempfile.TemporaryDirectory() as tmp:
        fails = _with_lib(_compile(src, tmp))
    assert fails, f"planted mistake '{name}' passed every pin"
