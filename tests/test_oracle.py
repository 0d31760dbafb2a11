"""Pins for the CPU oracle (paper §3-§5 in float64).

The oracle is checked against things other than itself: worked cases with
exact answers (tests/golden), an independent long-double cyclic Jacobi solver,
LAPACK, algebraic invariants, matrices built from known angles and spectra, and
the paper's own special cases and symmetries.  A planted-mistake test at the
end shows that plausible slips in the oracle's arithmetic fail these pins.
"""

import json
import math
import os

import numpy as np
import pytest

import oracle
import synth
from tests import helpers as H

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _eval_phi(expr):
    return float(eval(expr, {"pi": math.pi, "atan": math.atan}))


# ---------------------------------------------------------------- 2x2, §3 ---
def test_eig2_golden():
    cases = json.load(open(os.path.join(GOLD, "eig2_exact.json")))["cases"]
    P = np.array([c["a"] for c in cases], dtype=np.float64).T
    o = oracle.eig2(P)
    for i, c in enumerate(cases):
        assert np.allclose(o["lam"][:, i], c["lam"], atol=1e-14), (c, o["lam"][:, i])
        phi = _eval_phi(c["phi"])
        assert abs(o["phi"][i] - phi) < 1e-15, (c, o["phi"][i])
        cp, sp = math.cos(phi), math.sin(phi)
        assert np.allclose(o["D"][:, i], [cp, -sp, sp, cp], atol=1e-15)


def _mats2(P):
    a11, a22, a12 = P
    return np.stack([np.stack([a11, a12], 1), np.stack([a12, a22], 1)], 1)


def test_eig2_random_vs_lapack_and_residual():
    P = synth.make_plain(16, 20000, seed=11)["planes2"]
    o = oracle.eig2(P)
    A = _mats2(P)
    D = o["D"].T.reshape(-1, 2, 2)
    f = np.linalg.norm(A.reshape(-1, 4), axis=1)
    ref = np.linalg.eigvalsh(A)
    err = np.abs(np.sort(o["lam"], axis=0).T - ref).max(axis=1) / f
    assert err.max() < 4e-16 * 8
    res = np.linalg.norm(A @ D - D * o["lam"].T[:, None, :], axis=1).max(axis=1) / f
    assert res.max() < 2e-15
    # D = R(phi), eq. (2.5); phi in [-pi/4, pi/4]
    c, s = np.cos(o["phi"]), np.sin(o["phi"])
    assert np.abs(o["D"] - np.stack([c, -s, s, c])).max() < 1e-15
    assert np.all(np.abs(o["phi"]) <= math.pi / 4 + 1e-15)
    # lam1 belongs to A11's side: first column leans on e1
    assert np.all(np.abs(D[:, 0, 0]) >= np.abs(D[:, 1, 0]) - 1e-15)


def test_eig2_swap_symmetry():
    """§3: interchanging A11 and A22 interchanges lam1, lam2 and flips phi
    (off the tie line A11 = A22, where sign(0) breaks the symmetry)."""
    P = synth.make_plain(16, 5000, seed=12)["planes2"]
    Q = P[[1, 0, 2]]
    a, b = oracle.eig2(P), oracle.eig2(Q)
    assert np.allclose(a["lam"][0], b["lam"][1], atol=1e-15, rtol=0)
    assert np.allclose(a["lam"][1], b["lam"][0], atol=1e-15, rtol=0)
    assert np.allclose(a["phi"], -b["phi"], atol=1e-16, rtol=0)


def test_eig2_special_case():
    """§3: A11 = A22 and A12 = 0 gives lam1 = lam2 and phi = 0."""
    x = np.linspace(-3, 3, 13)
    o = oracle.eig2(np.stack([x, x, 0 * x]))
    assert np.all(o["phi"] == 0.0)
    assert np.all(o["lam"][0] == x) and np.all(o["lam"][1] == x)


# ---------------------------------------------------------------- 3x3 -------
def test_eig3_golden():
    cases = json.load(open(os.path.join(GOLD, "eig3_exact.json")))["cases"]
    branch = {"general": oracle.GENERAL, "double": oracle.DOUBLE, "triple": oracle.TRIPLE}
    for c in cases:
        o = oracle.eig3(np.array(c["a"], dtype=np.float64)[:, None])
        lam = o["lam"][:, 0]
        assert np.allclose(lam, c["lam"], atol=1e-14), (c, lam)
        assert o["branch"][0] == branch[c["branch"]], c
        D = o["D"][:, 0].reshape(3, 3)
        assert abs(np.linalg.det(D) - 1) < 1e-14
        for k, v in enumerate(c["vec"]):
            if v is None:
                continue
            v = np.array(v, float) / np.linalg.norm(v)
            assert min(np.linalg.norm(D[:, k] - v), np.linalg.norm(D[:, k] + v)) < 1e-7, (c, k, D)
        if c.get("exact_D"):
            assert np.array_equal(D, np.eye(3))
            assert np.all(o["phi"][:, 0] == 0)


def _jacobi_checks(P, lam_tol, vec_tol_over_gap, res_tol):
    o = oracle.eig3(P)
    j = oracle.jacobi3(P)
    lam_err = H.sorted_lam_err(P, o["lam"], j["lam"])
    assert np.all(lam_err < lam_tol), lam_err.max()
    g = H.rel_gaps(j["lam"])
    ve = H.eigvec_err(o["lam"], o["D"], j["lam"], j["V"])
    gk = np.take_along_axis(g, np.argsort(np.argsort(-o["lam"], axis=0), axis=0), axis=0)
    ok = gk > 1e-3
    assert (ve[ok] * gk[ok]).max() < vec_tol_over_gap
    res = H.residual3(P, o["lam"], o["D"])
    assert res.max() < res_tol, res.max()
    return o


def test_eig3_uniform_vs_long_double_jacobi():
    """U[-1,1] entries: paper formulas in float64 agree with an independent
    long-double solver to ~1e-15 ||A||_F in eigenvalues and to ~sqrt(eps) at
    worst in eigenvectors (the angle solve's conditioning)."""
    P = synth.make_plain(20000, 16, seed=21)["planes3"]
    o = _jacobi_checks(P, lam_tol=1e-14, vec_tol_over_gap=1e-9, res_tol=1e-10)
    assert np.all(o["branch"] == oracle.GENERAL)


def test_eig3_haar_spectra_vs_jacobi():
    """Q diag(lam) Q^T with Haar Q and a well-separated spectrum.  The literal
    q of (4.8) is a sum of O(||A||^3) terms that cancel down to O(p^(3/2)) when
    the spectrum sits far from zero relative to its spread, so the float64
    eigenvalue error scales like eps * (1 + ||A||_F^2 / p) * ||A||_F."""
    rng = np.random.default_rng(22)
    n = 20000
    lam = rng.uniform(-1, 1, (n, 3))
    keep = np.min(np.abs(np.diff(np.sort(lam, axis=1), axis=1)), axis=1) > 0.02
    lam = lam[keep]
    Q = synth.haar_rotations(rng, lam.shape[0])
    P = synth._sandwich(Q, lam)
    _jacobi_checks(P, lam_tol=H.literal_q_lam_tol(P), vec_tol_over_gap=1e-9, res_tol=1e-10)


def test_eig3_vs_lapack():
    P = synth.make_plain(10000, 16, seed=23)["planes3"]
    o = oracle.eig3(P)
    ref = np.linalg.eigvalsh(H.full3(P)).T
    assert H.sorted_lam_err(P, o["lam"], ref).max() < 1e-14


def test_eig3_invariants_and_order():
    """trace, determinant, Frobenius norm (eq. (2.1)); D orthogonal with
    det +1 (§2); slot order lam1 >= lam3 >= lam2 of (4.10)-(4.12)."""
    P = synth.make_plain(10000, 16, seed=24)["planes3"]
    o = oracle.eig3(P)
    A = H.full3(P)
    f = H.fro3(P)
    L = o["lam"]
    assert np.abs(L.sum(0) - np.trace(A, axis1=1, axis2=2)).max() < 1e-14 * f.max() * 4
    assert (np.abs(L.prod(0) - np.linalg.det(A)) / f ** 3).max() < 1e-14
    assert (np.abs((L ** 2).sum(0) - f ** 2) / f ** 2).max() < 1e-14
    assert H.orth_err(o["D"]).max() < 1e-15 * 4
    assert np.abs(H.det3(o["D"]) - 1).max() < 1e-15 * 4
    assert np.all(L[0] >= L[2]) and np.all(L[2] >= L[1])


def test_eig3_angles_reproduce_D():
    """D = R1(phi1) R2(phi2) R3(phi3) (eq. (2.6)); general-branch ranges."""
    P = synth.make_plain(5000, 16, seed=25)["planes3"]
    o = oracle.eig3(P)
    R = H.rot_from_angles(o["phi"])
    assert np.abs(R - H.as_mats(o["D"])).max() < 1e-14
    assert np.all(np.abs(o["phi"][1:]) <= math.pi / 2 + 1e-15)
    assert np.all(np.abs(o["phi"][0]) <= math.pi + 1e-15)


def test_eig3_round_trip_from_known_angles():
    """Build A = D Lambda D^T from chosen angles and spectrum (§2, (2.1) and
    (2.6)); the oracle recovers the spectrum and D up to the sign of each column."""
    rng = np.random.default_rng(26)
    n = 5000
    phi = np.stack([rng.uniform(-math.pi, math.pi, n), rng.uniform(-1.4, 1.4, n),
                    rng.uniform(-1.4, 1.4, n)])
    lam = np.sort(rng.uniform(-1, 1, (n, 3)), axis=1)[:, ::-1]
    keep = np.min(-np.diff(lam, axis=1), axis=1) > 0.05
    phi, lam = phi[:, keep], lam[keep]
    R = H.rot_from_angles(phi)
    A = np.einsum("nik,nk,njk->nij", R, lam, R)
    P = synth.planes3_from_full(A)
    o = oracle.eig3(P)
    L = o["lam"]
    err = np.abs(np.sort(L, axis=0)[::-1] - lam.T).max(axis=0) / H.fro3(P)
    assert np.all(err < H.literal_q_lam_tol(P))
    D = H.as_mats(o["D"])
    for k in range(3):
        j = np.argmin(np.abs(lam[:, :, None] - L.T[:, None, :]), axis=1)[:, k]
        d = D[:, :, k]
        v = R[np.arange(len(j)), :, j]
        err = np.minimum(np.linalg.norm(d - v, axis=1), np.linalg.norm(d + v, axis=1))
        assert err.max() < 1e-8


def test_eig3_triple():
    """§5: p = 0 gives the triple eigenvalue b/3, all angles 0, D = I."""
    x = np.array([0.0, 1.0, -2.5, 1e-30, 3e30])
    P = np.stack([x, x, x, 0 * x, 0 * x, 0 * x])
    o = oracle.eig3(P)
    assert np.all(o["branch"] == oracle.TRIPLE)
    assert np.array_equal(o["lam"], np.stack([x, x, x]))
    assert np.all(o["phi"] == 0)
    assert np.array_equal(H.as_mats(o["D"]), np.broadcast_to(np.eye(3), (5, 3, 3)))


def test_eig3_double_root_cases():
    """§5 special case q^2 = 4 p^3 != 0: exact double spectra, diagonal and
    rotated; output slots (max, min, mid), det D = +1, small residual."""
    rng = np.random.default_rng(27)
    n = 3000
    a = rng.uniform(-1, 1, n)
    c = rng.uniform(-1, 1, n)
    # keep the spread well above the literal-q cancellation level, so that the
    # computed split of the double pair stays below the tau_dbl reading
    keep = np.abs(a - c) > 0.1 * np.maximum(np.abs(a), np.abs(c))
    a, c = a[keep], c[keep]
    n = a.size
    lam = np.stack([a, a, c], 1)
    # permutations of diag(a, a, c)
    for perm in ([0, 1, 2], [0, 2, 1], [2, 0, 1]):
        P = np.zeros((6, n))
        P[0:3] = lam[:, perm].T
        o = oracle.eig3(P)
        assert np.all(o["branch"] == oracle.DOUBLE)
        # acos(sqrt(s)) of (5.22) turns an O(eps) error in s near 0 or 1 into
        # an O(sqrt(eps)) angle, hence a residual of order 1e-8
        assert H.residual3(P, o["lam"], o["D"]).max() < 1e-7
        assert np.abs(H.det3(o["D"]) - 1).max() < 1e-15
        L = o["lam"]
        assert np.all(L[0] >= L[2]) and np.all(L[2] >= L[1])
        assert np.abs(H.rot_from_angles(o["phi"]) - H.as_mats(o["D"])).max() < 1e-14
    # rotated doubles with integer-exact structure are rare in floating point;
    # rotated ones still land in the double branch via the split reading
    Q = synth.haar_rotations(rng, n)
    P = synth._sandwich(Q, lam)
    o = oracle.eig3(P)
    assert np.mean(o["branch"] == oracle.DOUBLE) > 0.99
    assert H.residual3(P, o["lam"], o["D"]).max() < 1e-7
    assert H.sorted_lam_err(P, o["lam"], np.sort(lam, axis=1).T).max() < 1e-7


def test_eig3_near_double_keeps_the_roots():
    """R-double: spectra whose two close eigenvalues differ by 2e-7 .. 8e-7
    of their spread take the double branch (split below tau_dbl = 1e-6 of
    sqrt(p)), which builds D from (5.20)-(5.25) but returns the roots
    (4.10)-(4.12) as computed.  Against the long-double Jacobi solver they stay
    within the trigonometric solution's error bound, eps (1 + ||A||^2/p)
    (1 + p / (||A|| gap)) relative to ||A||_F: the literal q's cancellation
    times arccos's slope near a double root.  The spectra are centred (p of
    the order of ||A||_F^2), where that bound is tight, and replacing the
    close pair by its mean -- off by half the split -- would miss it by far."""
    rng = np.random.default_rng(29)
    n = 4000
    a = rng.uniform(0.5, 1, n) * rng.choice([-1, 1], n)
    c = -a * rng.uniform(0.5, 1, n)
    split = np.exp(rng.uniform(np.log(2e-7), np.log(8e-7), n)) * np.abs(a - c)
    lam = np.stack([a, a + split, c], 1)
    P = synth._sandwich(synth.haar_rotations(rng, n), lam)
    o = oracle.eig3(P)
    j = oracle.jacobi3(P)
    assert np.all(o["branch"] == oracle.DOUBLE)
    f = H.fro3(P)
    p = H.p_invariant(P)
    L = np.sort(j["lam"], axis=0)
    g = np.minimum(L[1] - L[0], L[2] - L[1])
    eps = np.finfo(np.float64).eps
    tol = 2 * eps * (1 + f ** 2 / p) * (1 + p / (f * g))
    err = H.sorted_lam_err(P, o["lam"], j["lam"])
    assert np.all(err <= tol), (err / tol).max()
    # the mean of the close pair would miss by half the split
    assert np.all(0.5 * split / f > 10 * tol)
    L = o["lam"]
    assert np.all(L[0] >= L[2]) and np.all(L[2] >= L[1])


def test_eig3_f1_or_f2_zero():
    """§5 conjecture (2) structures: |f1| = 0 (A12 = A13 = 0) or |f2| = 0
    (A22 = A33, A23 = 0) still give a correct decomposition."""
    rng = np.random.default_rng(28)
    n = 4000
    P = rng.uniform(-1, 1, (6, n))
    P1 = P.copy(); P1[3] = 0; P1[4] = 0
    P2 = P.copy(); P2[2] = P2[1]; P2[5] = 0
    for Q in (P1, P2):
        o = oracle.eig3(Q)
        assert H.residual3(Q, o["lam"], o["D"]).max() < 1e-7
        ref = np.linalg.eigvalsh(H.full3(Q)).T
        assert np.all(H.sorted_lam_err(Q, o["lam"], ref) < H.closed_form_lam_tol(Q, ref))


def test_conjecture_unique_combination():
    """§5 conjecture (1): with |f1|, |f2| != 0 exactly one sign combination of
    (phi2, phi3) makes phi1(1) = phi1(2); the selection finds it."""
    P = synth.make_plain(3000, 16, seed=29)["planes3"]
    best, second = [], []
    for i in range(P.shape[1]):
        d = oracle.eig3_debug(P[:, i])
        s = sorted(d["delta"])
        best.append(s[0]); second.append(s[1])
        assert d["delta"][d["chosen"]] == s[0]
    assert max(best) < 1e-9
    assert min(second) > 1e-6


def test_f_and_g_have_equal_norms():
    """Identities (5.9)-(5.10) imply |f1| = |g1| and |f2| = |g2| for the chosen
    combination."""
    P = synth.make_plain(2000, 16, seed=30)["planes3"]
    for i in range(P.shape[1]):
        d = oracle.eig3_debug(P[:, i])
        scale = math.sqrt(d["p"])
        assert abs(d["f1n"] - d["g1n"]) < 1e-9 * scale
        assert abs(d["f2n"] - d["g2n"]) < 1e-9 * scale


def test_p_q_against_characteristic_polynomial():
    """(4.2)-(4.8): b = trace, and the depressed-cubic invariants p and q agree
    with the LAPACK eigenvalues: p = sum_{i<j} (lam_i - lam_j)^2 / 2 and
    q = prod_k (3 lam_k - b)."""
    P = synth.make_plain(500, 16, seed=31)["planes3"]
    ev = np.linalg.eigvalsh(H.full3(P))
    for i in range(P.shape[1]):
        d = oracle.eig3_debug(P[:, i])
        l = ev[i]
        b = l.sum()
        p = 0.5 * ((l[0] - l[1]) ** 2 + (l[0] - l[2]) ** 2 + (l[1] - l[2]) ** 2)
        q = np.prod(3 * l - b)
        assert abs(d["b"] - b) < 1e-14
        assert abs(d["p"] - p) < 1e-13 * max(1, p)
        assert abs(d["q"] - q) < 1e-12 * max(1, abs(p) ** 1.5)


def test_sign_of_q_symmetry():
    """§4 remark after (4.12): negating A (so q -> -q) negates the spectrum."""
    P = synth.make_plain(5000, 16, seed=32)["planes3"]
    a, b = oracle.eig3(P), oracle.eig3(-P)
    assert np.abs(np.sort(a["lam"], axis=0) + np.sort(b["lam"], axis=0)[::-1]).max() < 1e-14


def test_euler_identity_fixed_vs_rotating_axes():
    """§6 (6.2)-(6.5): R3''(phi3) R2'(phi2) R1(phi1) = R1 R2 R3 with the same
    angles; the angles the oracle returns are therefore the Euler angles."""
    P = synth.make_plain(500, 16, seed=33)["planes3"]
    o = oracle.eig3(P)
    for i in range(P.shape[1]):
        p1, p2, p3 = o["phi"][:, i]
        z = np.zeros(1)
        R1 = H.rot_from_angles(np.array([[p1], [0.0], [0.0]]))[0]
        R2 = H.rot_from_angles(np.array([[0.0], [p2], [0.0]]))[0]
        R3 = H.rot_from_angles(np.array([[0.0], [0.0], [p3]]))[0]
        R2p = R1 @ R2 @ R1.T
        S = R2p @ R1
        R3pp = S @ R3 @ S.T
        assert np.abs(R3pp @ R2p @ R1 - o["D"][:, i].reshape(3, 3)).max() < 1e-14
        del z


# --------------------------------------------------------------- adjoint ----
def _fd_forward(P):
    """Accurate forward for finite differences: the long-double Jacobi."""
    j = oracle.jacobi3(P)
    return j["lam"], j["V"]


def test_adjoint_against_central_differences():
    """dL/dA of L = sum w*lam + sum G*D, with the oracle adjoint, against
    central differences of an independent accurate forward (sign-aligned)."""
    d = synth.make_grad(400, seed=34, dtype=np.float64, min_gap=5e-2)
    P, w, G = d["planes3"], d["w"].astype(np.float64), d["G"].astype(np.float64)
    lam0, V0 = _fd_forward(P)
    gA = oracle.eig3_bwd(lam0, V0, w, G, eps=0.0)
    h = 1e-6
    V0m = H.as_mats(V0)

    def loss(Pp):
        lam, V = _fd_forward(Pp)
        Vm = H.as_mats(V)
        # align each column's sign to the base point
        s = np.sign(np.einsum("nik,nik->nk", Vm, V0m))
        Vm = Vm * s[:, None, :]
        return (w * lam).sum(0) + (G * Vm.reshape(-1, 9).T).sum(0)

    fd = np.empty_like(gA)
    for k in range(6):
        Pp = P.copy(); Pp[k] += h
        Pm = P.copy(); Pm[k] -= h
        fd[k] = (loss(Pp) - loss(Pm)) / (2 * h)
    rel = np.linalg.norm(fd - gA, axis=0) / np.linalg.norm(gA, axis=0)
    assert rel.max() < 1e-6, rel.max()


def test_adjoint_eigenvalue_part():
    """With Dbar = 0 the adjoint is sum_k lam_bar_k d_k d_k^T (textbook first
    order perturbation): check gA = diag + 2 x off-diagonal of that matrix."""
    P = synth.make_plain(200, 16, seed=35)["planes3"]
    o = oracle.eig3(P)
    rng = np.random.default_rng(36)
    wl = rng.standard_normal((3, P.shape[1]))
    gA = oracle.eig3_bwd(o["lam"], o["D"], wl, None, 0.0)
    D = H.as_mats(o["D"])
    M = np.einsum("nik,nk,njk->nij", D, wl.T, D)
    ref = np.stack([M[:, 0, 0], M[:, 1, 1], M[:, 2, 2], 2 * M[:, 0, 1], 2 * M[:, 0, 2], 2 * M[:, 1, 2]])
    assert np.abs(gA - ref).max() < 1e-14


def test_adjoint_regulariser_limit():
    """eps -> 0 recovers the unregularised adjoint; large eps damps the
    eigenvector part towards zero."""
    d = synth.make_grad(200, seed=37, dtype=np.float64, min_gap=1e-2)
    o = oracle.eig3(d["planes3"])
    a = oracle.eig3_bwd(o["lam"], o["D"], None, d["G"], 0.0)
    b = oracle.eig3_bwd(o["lam"], o["D"], None, d["G"], 1e-12)
    c = oracle.eig3_bwd(o["lam"], o["D"], None, d["G"], 1e12)
    assert np.abs(a - b).max() < 1e-9 * np.abs(a).max()
    assert np.abs(c).max() < 1e-10


def test_adjoint_at_exactly_repeated_eigenvalues():
    """With eps = 0 an exactly repeated pair takes the weight the regularised
    adjoint gives it for every eps > 0 (zero), instead of 0/0: on the zero
    matrix, diag(a, a, c) and a 2x2 multiple of I the eps = 0 adjoint is finite
    and equals the adjoint at eps = 1e-150 (a regulariser that changes no
    weight of a separated pair), and for the zero matrix it is the eigenvalue
    part alone."""
    rng = np.random.default_rng(43)
    P = np.zeros((6, 3))
    P[0, 1], P[1, 1], P[2, 1] = 0.5, 0.5, -0.25        # diag(a, a, c)
    P[0, 2], P[1, 2], P[2, 2] = 0.0, 1.0, 1.0          # diag(0, 1, 1)
    o = oracle.eig3(P)
    w, G = rng.standard_normal((3, 3)), rng.standard_normal((9, 3))
    a = oracle.eig3_bwd(o["lam"], o["D"], w, G, 0.0)
    b = oracle.eig3_bwd(o["lam"], o["D"], w, G, 1e-150)
    assert np.all(np.isfinite(a)) and np.abs(a - b).max() < 1e-14
    D = H.as_mats(o["D"])[0]
    M = D @ np.diag(w[:, 0]) @ D.T
    ref0 = [M[0, 0], M[1, 1], M[2, 2], 2 * M[0, 1], 2 * M[0, 2], 2 * M[1, 2]]
    assert np.abs(a[:, 0] - ref0).max() < 1e-15
    Q = np.array([[2.0, 0.0], [2.0, 0.0], [0.0, 0.0]])  # 2I and the zero 2x2
    o2 = oracle.eig2(Q)
    g2 = oracle.eig2_bwd(o2["lam"], o2["D"], rng.standard_normal((2, 2)), rng.standard_normal((4, 2)),
                         rng.standard_normal(2), eps=0.0)
    assert np.all(np.isfinite(g2))


def test_eig2_adjoint_against_central_differences():
    """2x2 adjoint of L = sum w*lam + sum G*D + g*phi (oracle) against central
    differences of the oracle's 2x2 forward (§3, pinned above), on matrices
    with well-separated eigenvalues and angles away from the ends of their
    range (where phi and D jump)."""
    rng = np.random.default_rng(41)
    n = 600
    P = rng.uniform(-1, 1, (3, n))
    f0 = oracle.eig2(P)
    lam, D, phi = f0["lam"], f0["D"], f0["phi"]
    w = rng.standard_normal((2, n))
    G = rng.standard_normal((4, n))
    g = rng.standard_normal(n)
    gA = oracle.eig2_bwd(lam, D, w, G, g, eps=0.0)
    h = 1e-6

    def loss(Pp):
        f = oracle.eig2(Pp)
        return (w * f["lam"]).sum(0) + (G * f["D"]).sum(0) + g * f["phi"]

    fd = np.empty_like(gA)
    for k in range(3):
        Pp = P.copy(); Pp[k] += h
        Pm = P.copy(); Pm[k] -= h
        fd[k] = (loss(Pp) - loss(Pm)) / (2 * h)
    # no jump of phi inside the stencil, eigenvalues apart
    smooth = np.all(np.abs(fd) < 1e3, axis=0) & (np.abs(lam[0] - lam[1]) > 0.05)
    assert smooth.sum() > 500
    rel = np.linalg.norm(fd - gA, axis=0)[smooth] / np.linalg.norm(gA, axis=0)[smooth]
    assert rel.max() < 1e-6, rel.max()
    # each cotangent on its own (the angle term separately pins its sign and scale)
    for cot in ((w, None, None), (None, G, None), (None, None, g)):
        gA1 = oracle.eig2_bwd(lam, D, *cot, eps=0.0)

        def loss1(Pp, cot=cot):
            f = oracle.eig2(Pp)
            out = np.zeros(n)
            if cot[0] is not None:
                out += (cot[0] * f["lam"]).sum(0)
            if cot[1] is not None:
                out += (cot[1] * f["D"]).sum(0)
            if cot[2] is not None:
                out += cot[2] * f["phi"]
            return out

        for k in range(3):
            Pp = P.copy(); Pp[k] += h
            Pm = P.copy(); Pm[k] -= h
            fdk = (loss1(Pp) - loss1(Pm)) / (2 * h)
            err = np.abs(fdk - gA1[k])[smooth]
            assert err.max() < 1e-6 * (1 + np.abs(gA1[k][smooth]).max()), (k, err.max())


def test_eig2_adjoint_regulariser_limit():
    """eps -> 0 recovers the unregularised 2x2 adjoint; a large eps leaves only
    the eigenvalue part."""
    rng = np.random.default_rng(42)
    P = rng.uniform(-1, 1, (3, 300))
    o = oracle.eig2(P)
    w = rng.standard_normal((2, 300))
    G = rng.standard_normal((4, 300))
    g = rng.standard_normal(300)
    a = oracle.eig2_bwd(o["lam"], o["D"], w, G, g, eps=0.0)
    b = oracle.eig2_bwd(o["lam"], o["D"], w, G, g, eps=1e-12)
    c = oracle.eig2_bwd(o["lam"], o["D"], w, G, g, eps=1e12)
    lam_only = oracle.eig2_bwd(o["lam"], o["D"], w, None, None, eps=0.0)
    assert np.abs(a - b).max() < 1e-9 * np.abs(a).max()
    assert np.abs(c - lam_only).max() < 1e-10


def test_compose_round_trips_and_closed_forms():
    """The inverse map (eqs. (2.5)-(2.6)): composing the forward's own outputs
    gives back the input (3x3 and 2x2, random and Haar spectra); zero angles
    give diag(lam); a quarter turn of the third angle swaps the first two
    axes; trace and Frobenius norm are those of diag(lam)."""
    # the round trip is as good as the forward's own residual (the closed form
    # loses accuracy near coincident eigenvalues); mostly at rounding level
    for P in (synth.make_plain(3000, 16, seed=51)["planes3"],
              synth.make_precision(3000, seed=52).astype(np.float64)):
        o = oracle.eig3(P)
        A = oracle.compose3(o["lam"], o["phi"])
        res = H.residual3(P, o["lam"], o["D"])
        err = np.abs(A - P).max(0) / H.fro3(P)
        assert np.all(err <= 4 * res + 1e-13), (err - 4 * res).max()
        assert np.median(err) < 1e-15
    rng = np.random.default_rng(53)
    lam = rng.uniform(-1, 1, (3, 500))
    A0 = oracle.compose3(lam, np.zeros((3, 500)))
    assert np.array_equal(A0[:3], lam) and np.all(A0[3:] == 0)
    Aq = oracle.compose3(lam, np.stack([np.zeros(500), np.zeros(500), np.full(500, np.pi / 2)]))
    assert np.abs(Aq[:3] - lam[[1, 0, 2]]).max() < 1e-15 and np.abs(Aq[3:]).max() < 1e-15
    phi = np.stack([rng.uniform(-np.pi, np.pi, 500), rng.uniform(-np.pi / 2, np.pi / 2, 500),
                    rng.uniform(-np.pi / 2, np.pi / 2, 500)])
    Ar = oracle.compose3(lam, phi)
    assert np.abs(Ar[:3].sum(0) - lam.sum(0)).max() < 1e-14
    fro2 = (Ar[:3] ** 2).sum(0) + 2 * (Ar[3:] ** 2).sum(0)
    assert np.abs(fro2 - (lam ** 2).sum(0)).max() < 1e-14
    P2 = rng.uniform(-1, 1, (3, 2000))
    o2 = oracle.eig2(P2)
    A2 = oracle.compose2(o2["lam"], o2["phi"])
    assert np.abs(A2 - P2).max() < 1e-14
    A20 = oracle.compose2(lam[:2], np.zeros(500))
    assert np.array_equal(A20[:2], lam[:2]) and np.all(A20[2] == 0)


def test_adjoint_with_angle_cotangents_against_central_differences():
    """3x3 adjoint with cotangents of the Euler angles (eq. (2.6)), alone and
    with lam and D, against central differences of the oracle's forward, on
    matrices with separated eigenvalues, away from gimbal lock (cos phi2 = 0)
    and from the ends of the angle ranges; the gimbal regulariser's limits."""
    d = synth.make_grad(800, seed=43, dtype=np.float64, min_gap=5e-2)
    P = d["planes3"]
    o = oracle.eig3(P)
    lam, D, phi = o["lam"], o["D"], o["phi"]
    rng = np.random.default_rng(44)
    n = P.shape[1]
    w, G, gp = rng.standard_normal((3, n)), rng.standard_normal((9, n)), rng.standard_normal((3, n))
    h = 1e-6

    def fd_of(loss):
        fd = np.empty((6, n))
        for k in range(6):
            Pp = P.copy(); Pp[k] += h
            Pm = P.copy(); Pm[k] -= h
            fd[k] = (loss(Pp) - loss(Pm)) / (2 * h)
        return fd

    away = (np.cos(phi[1]) > 0.2) & (np.abs(np.abs(phi[0]) - np.pi) > 0.1) & (np.abs(np.abs(phi[2]) - np.pi / 2) > 0.1)
    for use_rest in (False, True):
        gA = oracle.eig3_bwd(lam, D, w if use_rest else None, G if use_rest else None, eps=0.0,
                             phi=phi, gphi=gp)

        def loss(Pp, use_rest=use_rest):
            f = oracle.eig3(Pp)
            out = (gp * f["phi"]).sum(0)
            if use_rest:
                out = out + (w * f["lam"]).sum(0) + (G * f["D"]).sum(0)
            return out

        fd = fd_of(loss)
        ok = away & np.all(np.abs(fd) < 1e3, axis=0)
        assert ok.sum() > 300
        rel = np.linalg.norm(fd - gA, axis=0)[ok] / np.linalg.norm(gA, axis=0)[ok]
        assert rel.max() < 1e-5, (use_rest, rel.max())
    a = oracle.eig3_bwd(lam, D, None, None, eps=0.0, phi=phi, gphi=gp, delta=0.0)
    b = oracle.eig3_bwd(lam, D, None, None, eps=0.0, phi=phi, gphi=gp, delta=1e-12)
    assert np.abs(a - b)[:, away].max() < 1e-9 * np.abs(a[:, away]).max()
    # a huge delta leaves only the parts of gphi that do not divide by cos(phi2)
    c = oracle.eig3_bwd(lam, D, None, None, eps=0.0, phi=phi, gphi=np.stack([gp[0], 0 * gp[1], 0 * gp[2]]),
                        delta=1e12)
    assert np.abs(c).max() < 1e-9
