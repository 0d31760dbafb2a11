"""GPU parity of the 3x3 forward (paper §4-§5) against the CPU oracle, through
the C ABI.  Every input is seeded and synthetic (synth.py)."""

import numpy as np
import pytest

import oracle
import synth
from tests import helpers as H
from tests.gpu_common import (LAM_TOL_F32, LAM_TOL_F64, RES_TOL_F64, VEC_TOL_F64, certified_reference,
                              check_f32_result, to_dev, to_np)

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ksym():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1306_6291_amd as k
    return k


def _run(ksym, P, dtype, path=None, outputs=("lam", "D", "phi", "gap", "flags"), **opt):
    t = to_dev(P, dtype)
    o = ksym.Opts.defaults(ksym.F32 if dtype == torch.float32 else ksym.F64, **opt)
    if path is not None:
        o.path = path
    ws = ksym.workspace()
    out = ksym.eig3(t, opts=o, outputs=outputs, ws=ws)
    torch.cuda.synchronize()
    r = to_np(out)
    r["ws"] = ws.cpu().numpy()
    return r


def _f64_parity(P, g, ref):
    lam_err = H.sorted_lam_err(P, g["lam"], ref["lam"])
    assert np.all(lam_err <= LAM_TOL_F64), lam_err.max()
    res = H.residual3(P, g["lam"], g["D"])
    assert res.max() <= RES_TOL_F64, res.max()
    # same slots as the oracle: column-wise agreement up to sign
    Dg, Do = H.as_mats(g["D"]), H.as_mats(ref["D"])
    dcol = np.minimum(np.abs(Dg - Do).max(axis=1), np.abs(Dg + Do).max(axis=1))
    assert dcol.max() <= VEC_TOL_F64, dcol.max()
    assert np.abs(H.rot_from_angles(g["phi"]) - Dg).max() < 1e-13
    assert np.abs(H.det3(g["D"]) - 1).max() < 1e-14


@pytest.mark.parametrize("path_name", ["PATH_FP64_PLAIN", "PATH_FP64_FIXUP"])
def test_plain_uniform_f64_matches_oracle(ksym, path_name):
    """4096 matrices with U[-1,1] entries, float64: |dlam| <= 1e-12 ||A||_F,
    residual <= 1e-10 ||A||_F, D equal to the oracle's column by column up to
    sign (1e-8), angles reproduce D."""
    P = synth.make_plain(4096, 16)["planes3"]
    ref = oracle.eig3(P)
    g = _run(ksym, P, torch.float64, path=getattr(ksym, path_name))
    _f64_parity(P, g, ref)
    # the general branch everywhere, like the oracle
    assert np.all((g["flags"] & 3) == 0)
    # angles agree with the oracle's up to the symmetry of D's columns
    if path_name == "PATH_FP64_PLAIN":
        assert np.all(g["flags"] == 0)


def test_plain_f64_ragged_sizes_and_launch_shapes(ksym):
    """Sizes that leave ragged tails, several launch shapes: bitwise identical
    outputs, all matching the oracle."""
    P = synth.make_plain(5000, 16, seed=77)["planes3"]
    ref = None
    for n in (1, 63, 64, 65, 1000, 4999):
        Pn = np.ascontiguousarray(P[:, :n])
        ref = oracle.eig3(Pn)
        g = _run(ksym, Pn, torch.float64, path=ksym.PATH_FP64_PLAIN)
        _f64_parity(Pn, g, ref)
    base = _run(ksym, P, torch.float64, path=ksym.PATH_FP64_FIXUP)
    for block, mpl, gm in ((64, 1, 1), (128, 1, 3), (256, 2, 1), (256, 1, 64)):
        g = _run(ksym, P, torch.float64, path=ksym.PATH_FP64_FIXUP, block=block,
                 mats_per_lane=mpl, grid_mult=gm)
        for k in ("lam", "D", "phi", "gap", "flags"):
            assert np.array_equal(g[k], base[k]), (block, mpl, gm, k)


def test_f64_double_and_triple_branches(ksym):
    """Exact double and triple spectra: the plain path takes the paper's
    special cases (5.20)-(5.25) and p = 0; slots, det and residual hold.
    Eigenvalues: the plain path returns the roots (4.10)-(4.12) in the double
    branch (reading R-double), which at an exact double root carry the
    arccos step's sqrt(eps) error (q^2 = 4 p^3 holds only up to rounding), as
    the oracle's do with their own rounding; the pair still sums exactly to
    the trace.  The checked path's Rayleigh-quotient eigenvalues meet the exact
    spectrum to 1e-14."""
    rng = np.random.default_rng(91)
    n = 2000
    a, c = rng.uniform(-1, 1, n), rng.uniform(-1, 1, n)
    keep = np.abs(a - c) > 0.1
    a, c = a[keep], c[keep]
    P = np.zeros((6, a.size))
    P[0], P[1], P[2] = a, a, c
    P2 = np.zeros((6, a.size))
    P2[0], P2[1], P2[2] = c, a, a
    Pt = np.zeros((6, 64))
    Pt[0:3] = np.linspace(-2, 2, 64)
    for Q in (P, P2):
        ref = oracle.eig3(Q)
        exact = Q[0:3]
        for path in (ksym.PATH_FP64_PLAIN, ksym.PATH_FP64_FIXUP):
            g = _run(ksym, Q, torch.float64, path=path)
            assert np.all(g["flags"] & 1), path
            if path == ksym.PATH_FP64_PLAIN:
                assert H.sorted_lam_err(Q, g["lam"], exact).max() < 1e-7
                assert H.sorted_lam_err(Q, g["lam"], ref["lam"]).max() < 1e-7
                assert np.abs(g["lam"].sum(0) - exact.sum(0)).max() < 1e-14
            else:
                assert H.sorted_lam_err(Q, g["lam"], exact).max() < 1e-14
            assert H.residual3(Q, g["lam"], g["D"]).max() < (1e-7 if path == ksym.PATH_FP64_PLAIN else 1e-14)
            assert np.abs(H.det3(g["D"]) - 1).max() < 1e-14
            L = g["lam"]
            assert np.all(L[0] >= L[2]) and np.all(L[2] >= L[1])
            assert np.abs(H.rot_from_angles(g["phi"]) - H.as_mats(g["D"])).max() < 1e-13
    g = _run(ksym, Pt, torch.float64, path=ksym.PATH_FP64_PLAIN)
    assert np.all(g["flags"] == 2)
    assert np.array_equal(g["lam"], np.stack([Pt[0]] * 3))
    assert np.array_equal(H.as_mats(g["D"]), np.broadcast_to(np.eye(3), (64, 3, 3)))
    assert np.all(g["phi"] == 0)


def test_precision_workload_f32_small(ksym):
    """The precision workload's recipe at 2^17 + 77 matrices (ragged tail):
    float32 in and out, float64 cubic step, refinement of flagged matrices."""
    n = (1 << 17) + 77
    P32 = synth.make_precision(n, seed=1306630)
    P64 = P32.astype(np.float64)
    lam_ref, V_ref = certified_reference(P64)
    g = _run(ksym, P32, torch.float32)
    stats = check_f32_result(P64, g, lam_ref, V_ref, "precision-f32")
    flags = g["flags"]
    nfix = int(np.sum((flags & 4) != 0))
    assert int(g["ws"][0]) == nfix
    assert int(g["ws"][1]) == 0
    print("precision f32:", stats, "refined fraction", nfix / n)


def test_plain_uniform_f32(ksym):
    """U[-1,1] float32 matrices through the float32 path."""
    P32 = synth.make_plain(1 << 16, 16, seed=55, dtype=np.float32)["planes3"]
    P64 = P32.astype(np.float64)
    lam_ref, V_ref = certified_reference(P64)
    g = _run(ksym, P32, torch.float32)
    check_f32_result(P64, g, lam_ref, V_ref, "uniform-f32")


def test_f32_launch_shapes_bitwise(ksym):
    """Every compiled launch shape gives bitwise-identical float32 results, and
    two runs of the same shape agree bitwise (the refinement queue order does
    not leak into the results)."""
    P32 = synth.make_precision(50000, seed=4242)
    base = _run(ksym, P32, torch.float32)
    again = _run(ksym, P32, torch.float32)
    for k in ("lam", "D", "phi", "gap", "flags"):
        assert np.array_equal(base[k], again[k], equal_nan=True), k
    for block, mpl in ((64, 1), (64, 2), (128, 1), (128, 2), (256, 1), (256, 2), (512, 1), (512, 2)):
        for gm in (1, 16, 1024):
            g = _run(ksym, P32, torch.float32, block=block, mats_per_lane=mpl, grid_mult=gm)
            for k in ("lam", "D", "phi", "gap", "flags"):
                assert np.array_equal(g[k], base[k], equal_nan=True), (block, mpl, gm, k)


def test_special_inputs_f32(ksym):
    """Zero, isotropic, diagonal, exact doubles, tiny and huge scales, and
    non-finite entries."""
    rng = np.random.default_rng(5)
    cols = []
    cols.append(np.zeros(6))
    cols.append(np.array([2.5, 2.5, 2.5, 0, 0, 0]))
    cols.append(np.array([1, 1, 3, 0, 0, 0.0]))
    cols.append(np.array([3, 1, 2, 0, 0, 0.0]))
    cols.append(np.array([2, 2, 2, 1, 1, 1.0]))
    for s in (1e-30, 1e-12, 1e12, 1e30):
        cols.append(rng.uniform(-1, 1, 6) * s)
    P = np.stack(cols, 1).astype(np.float32)
    P64 = P.astype(np.float64)
    lam_ref, V_ref = certified_reference(P64)
    g = _run(ksym, P, torch.float32)
    check_f32_result(P64, g, lam_ref, V_ref, "special")
    assert np.all(g["flags"][:2] == 2)
    bad = np.array([[np.nan, 0, 0, 0, 0, 0], [0, np.inf, 0, 0, 0, 0], [1, 1, 1, 0, -np.inf, 0]],
                   dtype=np.float32).T
    g = _run(ksym, np.ascontiguousarray(bad), torch.float32)
    assert np.all(g["flags"] == 8)
    assert np.all(np.isnan(g["lam"])) and np.all(np.isnan(g["D"]))
    assert int(g["ws"][1]) == 3


def test_special_inputs_f64(ksym):
    """Non-finite entries scattered through a ragged float64 batch: NaN outputs
    and flag 8 for exactly those matrices on both float64 paths, the checked
    path counts them, and the finite neighbours are unchanged bitwise."""
    P = synth.make_plain(3001, 16, seed=808)["planes3"]
    rng = np.random.default_rng(809)
    idx = rng.choice(P.shape[1], 40, replace=False)
    Pb = P.copy()
    for j, i in enumerate(idx):
        Pb[j % 6, i] = (np.nan, np.inf, -np.inf)[j % 3]
    mask = np.zeros(P.shape[1], bool)
    mask[idx] = True
    for path in (ksym.PATH_FP64_PLAIN, ksym.PATH_FP64_FIXUP):
        base = _run(ksym, P, torch.float64, path=path)
        g = _run(ksym, Pb, torch.float64, path=path)
        assert np.all(g["flags"][mask] == 8) and np.all(g["flags"][~mask] != 8), path
        for k in ("lam", "D", "phi", "gap"):
            assert np.all(np.isnan(g[k][:, mask])), (path, k)
            assert np.array_equal(g[k][:, ~mask], base[k][:, ~mask]), (path, k)
        if path == ksym.PATH_FP64_FIXUP:
            assert int(g["ws"][1]) == mask.sum()


def test_default_launch_shape_f64_bitwise(ksym):
    """The default float64 launch shape and a large non-persistent grid agree
    bitwise with a persistent one-workgroup-per-CU-multiple launch."""
    P = synth.make_precision(30001, seed=4343).astype(np.float64)
    base = _run(ksym, P, torch.float64, path=ksym.PATH_FP64_FIXUP, grid_mult=1)
    for opt in ({}, {"grid_mult": 1024}, {"block": 64, "grid_mult": 1024},
                {"block": 256, "mats_per_lane": 2, "grid_mult": 1024}):
        g = _run(ksym, P, torch.float64, path=ksym.PATH_FP64_FIXUP, **opt)
        for k in ("lam", "D", "phi", "gap", "flags"):
            assert np.array_equal(g[k], base[k]), (opt, k)


@pytest.mark.parametrize("dtype,k", [("float64", -1040), ("float64", -1000), ("float64", 1021),
                                     ("float32", -135), ("float32", 120), ("float32", 126)])
def test_power_of_two_scaling_extremes(ksym, dtype, k):
    """Every path first scales a matrix by a power of two, so A and B = A 2^-k
    (exact) give the same D, angles and flags bit for bit, and eigenvalues
    and gaps that differ by the factor 2^k (one rounding each; a float32
    result in the subnormal range may differ by one unit there, as it is
    rounded twice on the host side).  The k reach float64 matrices with
    subnormal entries only and float32 ones near the top of the range, where
    the scale factors themselves are not representable."""
    f64 = dtype == "float64"
    np_dt = np.float64 if f64 else np.float32
    P = synth.make_plain(1500, 16, seed=1234)["planes3"].astype(np_dt)
    P = np.concatenate([P, synth.make_precision(1500, seed=1235).astype(np_dt)], axis=1)
    A = np.ldexp(P, k).astype(np_dt)
    B = np.ldexp(A, -k).astype(np_dt)
    assert np.all(np.isfinite(A)) and np.array_equal(np.ldexp(B, k).astype(np_dt), A)
    tdt = torch.float64 if f64 else torch.float32
    for path in ((ksym.PATH_FP64_PLAIN, ksym.PATH_FP64_FIXUP) if f64 else (None,)):
        gA = _run(ksym, A, tdt, path=path)
        gB = _run(ksym, B, tdt, path=path)
        for key in ("D", "phi", "flags"):
            assert np.array_equal(gA[key], gB[key]), (path, key)
        for key in ("lam", "gap"):
            want = np.ldexp(gB[key], k).astype(np_dt)
            if f64:
                assert np.array_equal(gA[key], want), (path, key)
            else:
                diff = np.abs(gA[key].astype(np.float64) - want.astype(np.float64))
                assert diff.max() <= 2.0 ** -149, (key, diff.max())


def test_eigenvalues_only_mode_f32(ksym):
    """Reduced-output mode: float32 with no D and no angle planes runs the
    eigenvalues-only kernel.  Flags are the full path's without the FIXUP
    bit; lam and gap are bitwise the full path's wherever that path did not
    refine, and within the float32 tolerance of the certified reference
    everywhere; ragged sizes and launch shapes give the same bits; a
    non-finite input gives NaN and flag 8, and is counted."""
    n = (1 << 17) + 77
    P32 = synth.make_precision(n, seed=1306631)
    P64 = P32.astype(np.float64)
    lam_ref, _ = certified_reference(P64)
    full = _run(ksym, P32, torch.float32)
    lam_only = _run(ksym, P32, torch.float32, outputs=("lam", "gap", "flags"))
    assert "D" not in lam_only and "phi" not in lam_only
    assert np.array_equal(lam_only["flags"], full["flags"] & ~np.uint8(4))
    kept = (full["flags"] & 4) == 0
    assert kept.mean() > 0.99
    for k in ("lam", "gap"):
        assert np.array_equal(lam_only[k][:, kept], full[k][:, kept]), k
    err = H.sorted_lam_err(P64, lam_only["lam"].astype(np.float64), lam_ref)
    assert err.max() <= LAM_TOL_F32, err.max()
    assert int(lam_only["ws"][0]) == 0
    for m in (1, 63, 65, 4999):
        Pm = np.ascontiguousarray(P32[:, :m])
        g = _run(ksym, Pm, torch.float32, outputs=("lam", "gap", "flags"))
        for k in ("lam", "gap", "flags"):
            assert np.array_equal(g[k], lam_only[k][..., :m]), (m, k)
    for block, mpl, gm in ((64, 2, 1), (256, 1, 1024), (512, 2, 16)):
        g = _run(ksym, P32, torch.float32, outputs=("lam", "flags"), block=block, mats_per_lane=mpl,
                 grid_mult=gm)
        for k in ("lam", "flags"):
            assert np.array_equal(g[k], lam_only[k]), (block, mpl, gm, k)
    bad = np.array([[np.nan, 0, 0, 0, 0, 0], [0, np.inf, 0, 0, 0, 0], [1, 1, 1, 0, -np.inf, 0],
                    [2, 1, 0, 0.5, 0, 0]], dtype=np.float32).T
    g = _run(ksym, np.ascontiguousarray(bad), torch.float32, outputs=("lam", "gap", "flags"))
    assert np.array_equal(g["flags"], np.array([8, 8, 8, 0], np.uint8))
    assert np.all(np.isnan(g["lam"][:, :3])) and np.all(np.isnan(g["gap"][:, :3]))
    assert np.all(np.isfinite(g["lam"][:, 3]))
    assert int(g["ws"][1]) == 3


def test_all_matrices_refined_f32(ksym):
    """A batch where every matrix takes the refinement (exact doubles):
    the on-chip queue fills completely at every launch shape."""
    rng = np.random.default_rng(6)
    n = 20000
    a, c = rng.uniform(-1, 1, n), rng.uniform(-1, 1, n)
    Q = synth.haar_rotations(rng, n)
    P32 = synth._sandwich(Q, np.stack([a, a, c], 1)).astype(np.float32)
    P64 = P32.astype(np.float64)
    lam_ref, V_ref = certified_reference(P64)
    for block, mpl in ((64, 1), (256, 2), (512, 2)):
        g = _run(ksym, P32, torch.float32, block=block, mats_per_lane=mpl, tau_gap=1.0)
        assert np.all(g["flags"] & 4)
        check_f32_result(P64, g, lam_ref, V_ref, f"all-refined {block}x{mpl}")


def test_second_attempt_doubles_and_diagonals_f32(ksym):
    """Matrices on which the general branch's angle formulas lose accuracy:
    Haar-rotated diag(a, a, c) rounded to float32 (the pair's split is then
    at the rounding level), diagonal matrices with one entry repeated (an
    exact zero split) and diagonal matrices with distinct entries (each
    squared cosine exactly 0 or 1).  Where the general branch's result fails
    the check, the double-root branch of §5 (5.20)-(5.25), or for a diagonal
    matrix the signed permutation of its axes, is tried before the
    refinement; nearly none of these matrices then need the refinement,
    every result meets the float32 tolerances, and the flags keep the cubic
    step's classification (the same branch bits as when tau_gap forces
    every matrix into the refinement)."""
    rng = np.random.default_rng(16)
    n_rot, n_diag = 16384, 4096
    a, c = rng.uniform(-1, 1, n_rot), rng.uniform(-1, 1, n_rot)
    Q = synth.haar_rotations(rng, n_rot)
    P_rot = synth._sandwich(Q, np.stack([a, a, c], 1))
    d = rng.uniform(-1, 1, (3, n_diag))
    j = rng.integers(0, 3, n_diag)
    k = (j + 1 + rng.integers(0, 2, n_diag)) % 3
    d[k, np.arange(n_diag)] = d[j, np.arange(n_diag)]
    P_rep = np.concatenate([d, np.zeros((3, n_diag))])
    P_dist = np.concatenate([rng.uniform(-1, 1, (3, n_diag)), np.zeros((3, n_diag))])
    P32 = np.ascontiguousarray(np.concatenate([P_rot, P_rep, P_dist], axis=1).astype(np.float32))
    P64 = P32.astype(np.float64)
    lam_ref, V_ref = certified_reference(P64)
    g = _run(ksym, P32, torch.float32)
    stats = check_f32_result(P64, g, lam_ref, V_ref, "doubles and diagonals")
    fixed = (g["flags"] & 4) != 0
    parts = {"rotated doubles": fixed[:n_rot], "diagonal, repeated": fixed[n_rot:n_rot + n_diag],
             "diagonal, distinct": fixed[n_rot + n_diag:]}
    print("second attempt:", stats, {key: float(v.mean()) for key, v in parts.items()})
    for key, v in parts.items():
        assert v.mean() < 0.005, (key, v.mean())
    assert int(g["ws"][0]) == int(fixed.sum())
    forced = _run(ksym, P32, torch.float32, tau_gap=1.0)
    assert np.all(forced["flags"] & 4)
    check_f32_result(P64, forced, lam_ref, V_ref, "doubles and diagonals, all refined")
    assert np.array_equal(forced["flags"] & 3, g["flags"] & 3)


def test_eigenvalues_and_angles_mode_f32(ksym):
    """Reduced-output mode lam + phi (no D planes, 48 B per matrix): the
    angles alone determine D (eq. (2.6)), so a caller can drop D's 36 B.  The
    kernel still forms D in registers for the check and the refinement, so
    lam, phi, gap and flags are bitwise the full path's for every matrix
    (refined ones included), and R1 R2 R3 (phi) meets the float32 tolerances
    against the certified reference: eigenvalues, residual, orthogonality and
    eigenvectors up to sign where the relative gap is at least 1e-2."""
    n = (1 << 17) + 77
    P32 = synth.make_precision(n, seed=1306632)
    P64 = P32.astype(np.float64)
    full = _run(ksym, P32, torch.float32)
    lp = _run(ksym, P32, torch.float32, outputs=("lam", "phi", "gap", "flags"))
    assert "D" not in lp
    for k in ("lam", "phi", "gap", "flags"):
        assert np.array_equal(lp[k], full[k]), k
    assert int(lp["ws"][0]) == int(full["ws"][0]) > 0
    lam_ref, V_ref = certified_reference(P64)
    g = {"lam": lp["lam"], "D": H.rot_planes(lp["phi"].astype(np.float64)).astype(np.float32)}
    check_f32_result(P64, g, lam_ref, V_ref, "lam + phi mode, D from the angles")


def test_optional_outputs(ksym):
    P32 = synth.make_plain(3000, 16, seed=8, dtype=np.float32)["planes3"]
    full = _run(ksym, P32, torch.float32)
    part = _run(ksym, P32, torch.float32, outputs=("lam",))
    assert set(part) == {"lam", "ws"}
    assert np.array_equal(part["lam"], full["lam"])


def test_absent_planes_leave_the_others_bitwise(ksym):
    """The float32 kernels skip the stores of absent output planes, and the
    arithmetic that only fed them: every subset of planes that keeps the full
    kernel (D or the angles present) gives bitwise the full run's values on
    the planes it has, on the precision recipe (second attempts and
    refinement included) and in differentiated calls (tau_vec > 0)."""
    P32 = synth.make_precision(40000 + 17, seed=77)
    subsets = (("lam", "D"), ("D", "gap"), ("phi", "flags"), ("D", "phi", "flags"), ("lam", "phi", "gap"))
    for extra in ({}, {"tau_vec": 1e-4}):
        full = _run(ksym, P32, torch.float32, **extra)
        assert int(full["ws"][0]) > 0
        for outs in subsets:
            part = _run(ksym, P32, torch.float32, outputs=outs, **extra)
            for k in outs:
                assert np.array_equal(part[k], full[k], equal_nan=True), (extra, outs, k)
            assert int(part["ws"][0]) == int(full["ws"][0]), (extra, outs)


def test_aos_matches_soa(ksym):
    """Array-of-structures input (records of six) gives bitwise the SoA result."""
    P32 = synth.make_precision(70001, seed=99)
    soa = _run(ksym, P32, torch.float32)
    rec = to_dev(np.ascontiguousarray(P32.T), torch.float32)
    for block, mpl in ((64, 1), (128, 1), (256, 1), (256, 2), (512, 1)):
        o = ksym.Opts.defaults(ksym.F32, block=block, mats_per_lane=mpl)
        out = ksym.eig3_aos(rec, opts=o, outputs=("lam", "D", "phi", "gap", "flags"))
        torch.cuda.synchronize()
        out = to_np(out)
        for k in ("lam", "D", "phi", "gap", "flags"):
            assert np.array_equal(out[k], soa[k]), (block, mpl, k)
    P64 = synth.make_plain(3001, 16, seed=3)["planes3"]
    soa = _run(ksym, P64, torch.float64, path=ksym.PATH_FP64_FIXUP)
    o64 = ksym.Opts.defaults(ksym.F64)
    o64.path = ksym.PATH_FP64_FIXUP
    out = to_np(ksym.eig3_aos(to_dev(np.ascontiguousarray(P64.T), torch.float64), opts=o64,
                              outputs=("lam", "D", "phi", "gap", "flags")))
    for k in ("lam", "D", "phi", "gap", "flags"):
        assert np.array_equal(out[k], soa[k]), k


def test_f64_paths_on_precision_recipe(ksym):
    """Both float64 paths on the precision recipe (float32-rounded matrices
    promoted): no NaN; orthonormal D with det +1; the checked path meets
    residual <= 2e-11 ||A||_F (sqrt(3) tau_res) and |delta lam| <= 1e-12
    ||A||_F against the certified reference on every matrix (its eigenvalues
    are the Rayleigh quotients of the checked columns); the plain path meets
    the float32 tolerances away from its known weak spot (relative gaps below
    1e-3, where the closed-form angle solve loses accuracy even in
    float64)."""
    n = (1 << 16) + 5
    P32, kinds = synth.make_precision(n, seed=1306631, return_kinds=True)
    P64 = P32.astype(np.float64)
    lam_ref, _ = certified_reference(P64)
    for path in (ksym.PATH_FP64_PLAIN, ksym.PATH_FP64_FIXUP):
        g = _run(ksym, P64, torch.float64, path=path)
        bad = ~np.isfinite(g["D"]).all(0) | ~np.isfinite(g["lam"]).all(0) | ~np.isfinite(g["phi"]).all(0)
        assert not bad.any(), (path, int(bad.sum()), np.bincount(kinds[bad], minlength=6),
                               P64[:, np.nonzero(bad)[0][:3]].T.tolist())
        assert H.orth_err(g["D"]).max() < 1e-14
        assert np.abs(H.det3(g["D"]) - 1).max() < 1e-14
        res = H.residual3(P64, g["lam"], g["D"])
        if path == ksym.PATH_FP64_FIXUP:
            assert res.max() < 2e-11, res.max()   # each |B_jk| <= 1e-11 ||A||_F: sqrt(3) x
            lam_err = H.sorted_lam_err(P64, g["lam"], lam_ref)
            assert lam_err.max() <= LAM_TOL_F64, (lam_err.max(), np.bincount(kinds[lam_err > LAM_TOL_F64],
                                                                             minlength=6))
        else:
            g_rel = H.rel_gaps(lam_ref).min(0)
            ok = g_rel >= 1e-3
            assert res[ok].max() < 1e-5, res[ok].max()


@pytest.mark.parametrize("spread", [0.0, 1e-12, 1e-9, 1e-6])
def test_near_isotropic_all_paths(ksym, spread):
    """a I rotated by Haar matrices (rounding leaves off-diagonals around 1e-17)
    plus perturbations of relative size `spread`: every path returns finite,
    orthonormal D with det +1 and residual at the level of float rounding."""
    rng = np.random.default_rng(int(spread * 1e15) + 17)
    n = 20000
    a = rng.uniform(-1, 1, n)
    Q = synth.haar_rotations(rng, n)
    lam = a[:, None] + spread * rng.standard_normal((n, 3))
    P32 = synth._sandwich(Q, lam).astype(np.float32)
    P64 = P32.astype(np.float64)
    lam_ref, V_ref = certified_reference(P64)
    g = _run(ksym, P32, torch.float32)
    check_f32_result(P64, g, lam_ref, V_ref, f"near-iso f32 {spread}")
    for path in (ksym.PATH_FP64_PLAIN, ksym.PATH_FP64_FIXUP):
        g = _run(ksym, P64, torch.float64, path=path)
        assert np.isfinite(g["D"]).all() and np.isfinite(g["lam"]).all() and np.isfinite(g["phi"]).all()
        assert H.orth_err(g["D"]).max() < 1e-14
        assert np.abs(H.det3(g["D"]) - 1).max() < 1e-14
        jac = oracle.jacobi3(P64)["lam"]
        assert H.sorted_lam_err(P64, g["lam"], jac).max() < 1e-14
        assert H.residual3(P64, g["lam"], g["D"]).max() < 1e-13


def test_library_outputs_start_on_256_byte_boundaries(ksym):
    """At a batch size that is not a multiple of 64, the planes the binding
    allocates (forward, backward, inverse map, 2x2) each start on a 256-byte
    boundary (a row-strided view), and every result equals, bitwise, the same
    call with contiguous caller-provided outputs."""
    n = (1 << 16) - 24
    P = synth.make_precision(n, seed=synth.BASE_SEED + 81)
    A = to_dev(P, torch.float32)
    print(f"line-aligned outputs: n={n}", flush=True)
    out = ksym.eig3(A, outputs=("lam", "D", "phi", "gap", "flags"))
    for key in ("lam", "D", "phi", "gap"):
        rows = ksym._rows(out[key], out[key].shape[0])[0]
        assert all(p % 256 == 0 for p in rows), key
    mine = {"lam": torch.empty((3, n), device="cuda"), "D": torch.empty((9, n), device="cuda"),
            "phi": torch.empty((3, n), device="cuda"), "gap": torch.empty((3, n), device="cuda"),
            "flags": torch.empty((n,), dtype=torch.uint8, device="cuda")}
    ksym.eig3(A, out=mine)
    torch.cuda.synchronize()
    for key in mine:
        assert torch.equal(out[key], mine[key]), key
    g = torch.Generator(device="cuda").manual_seed(5)
    w = torch.randn((3, n), device="cuda", generator=g)
    G = torch.randn((9, n), device="cuda", generator=g)
    gA = ksym.eig3_backward(out["lam"], out["D"], w, G, gap=out["gap"])
    gA2 = ksym.eig3_backward(mine["lam"], mine["D"], w, G, gap=mine["gap"], out=torch.empty((6, n), device="cuda"))
    assert all(p % 256 == 0 for p in ksym._rows(gA, 6)[0]) and torch.equal(gA, gA2)
    C = ksym.compose3(out["lam"], out["phi"])
    assert torch.equal(C, ksym.compose3(mine["lam"], mine["phi"], out=torch.empty((6, n), device="cuda")))
    B = to_dev(np.random.default_rng(6).uniform(-1, 1, (3, n)), torch.float32)
    o2 = ksym.eig2(B)
    m2 = {"lam": torch.empty((2, n), device="cuda"), "D": torch.empty((4, n), device="cuda"),
          "phi": torch.empty((n,), device="cuda"), "flags": torch.empty((n,), dtype=torch.uint8, device="cuda")}
    ksym.eig2(B, out=m2)
    torch.cuda.synchronize()
    for key in m2:
        assert torch.equal(o2[key], m2[key]), key
