"""Batches larger than one launch chunk, through the C ABI.  The library splits
a batch into launches of at most 2^28 matrices (2^27 float32 and 2^26 float64
array-of-structures records), each with its pointers advanced by the chunk
start, so every in-kernel offset stays 32-bit.  Each test runs a batch a
little past a chunk boundary and checks a window across the boundary, the
ragged tail and the head: bitwise against separate calls on those matrices
alone (whose parity with the oracle the other tests establish), and for the
float32 3x3 forward also against the certified reference.  Inputs are drawn
on the device from seeded generators."""

import numpy as np
import pytest

from tests.gpu_common import certified_reference, check_f32_result

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

CHUNK = 1 << 28
CHUNK_AOS_F32 = 1 << 27
CHUNK_AOS_F64 = 1 << 26


@pytest.fixture(scope="module")
def ksym():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1306_6291_amd as k
    return k


@pytest.fixture(autouse=True)
def _release():
    yield
    torch.cuda.synchronize()
    torch.cuda.empty_cache()


def _randn(shape, seed, dtype=torch.float32):
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    return torch.randn(shape, generator=g, device="cuda", dtype=dtype)


def _windows(chunk, n, w=256):
    """Index ranges checked: the head, a window across the first chunk
    boundary, and the ragged tail of the last chunk."""
    return [(0, w), (chunk - w, min(n, chunk + w)), (max(0, n - w), n)]


def _cols(t, a, b):
    """Columns a:b as a fresh allocation (aligned like any other)."""
    return t[..., a:b].clone() if t.dim() == 2 else t[a:b].clone()


def test_eig3_f32_soa_across_chunks(ksym):
    n = CHUNK + 777
    A = _randn((6, n), 301)
    opts = ksym.tuned_opts("eig3", ksym.F32)
    out = ksym.eig3(A, opts=opts, outputs=("lam", "D", "phi", "flags"))
    torch.cuda.synchronize()
    for a, b in _windows(CHUNK, n):
        ref = ksym.eig3(_cols(A, a, b), opts=opts, outputs=("lam", "D", "phi", "flags"))
        for k in ref:
            assert torch.equal(_cols(out[k], a, b), ref[k]), (k, a, b)
        P64 = A[:, a:b].double().cpu().numpy()
        g = {k: _cols(out[k], a, b).cpu().numpy() for k in ("lam", "D", "phi")}
        lam_ref, V_ref = certified_reference(P64)
        check_f32_result(P64, g, lam_ref, V_ref, f"chunk window {a}:{b}")
    del out
    # eigenvalues-only mode on the same batch
    lam = ksym.eig3(A, opts=ksym.tuned_opts("eig3_lam", ksym.F32), outputs=("lam", "flags"))
    torch.cuda.synchronize()
    for a, b in _windows(CHUNK, n):
        ref = ksym.eig3(_cols(A, a, b), opts=ksym.tuned_opts("eig3_lam", ksym.F32), outputs=("lam", "flags"))
        for k in ref:
            assert torch.equal(_cols(lam[k], a, b), ref[k]), (k, a, b)


@pytest.mark.parametrize("path_name", ["PATH_FP64_PLAIN", "PATH_FP64_FIXUP"])
def test_eig3_f64_soa_across_chunks(ksym, path_name):
    """float64 structure-of-arrays input just past one launch chunk: each
    plane of the first chunk spans 2^31 bytes, the most a 32-bit buffer
    offset reaches.  Both float64 paths; windows bitwise equal to separate
    calls and within the float64 tolerances of the oracle."""
    import oracle
    from tests import helpers as H
    from tests.gpu_common import LAM_TOL_F64, RES_TOL_F64
    n = CHUNK + 333
    A = _randn((6, n), 308, torch.float64)
    opts = ksym.Opts.defaults(ksym.F64)
    opts.path = getattr(ksym, path_name)
    out = ksym.eig3(A, opts=opts, outputs=("lam", "D", "phi", "flags"))
    torch.cuda.synchronize()
    for a, b in _windows(CHUNK, n):
        ref = ksym.eig3(_cols(A, a, b), opts=opts, outputs=("lam", "D", "phi", "flags"))
        for k in ref:
            assert torch.equal(_cols(out[k], a, b), ref[k]), (path_name, k, a, b)
        P64 = A[:, a:b].cpu().numpy()
        lam = _cols(out["lam"], a, b).cpu().numpy()
        D = _cols(out["D"], a, b).cpu().numpy()
        o = oracle.eig3(P64)
        assert H.sorted_lam_err(P64, lam, o["lam"]).max() <= LAM_TOL_F64, (path_name, a, b)
        assert H.residual3(P64, lam, D).max() <= RES_TOL_F64, (path_name, a, b)


@pytest.mark.parametrize("dtype,chunk", [(torch.float32, CHUNK_AOS_F32), (torch.float64, CHUNK_AOS_F64)])
def test_eig3_aos_across_chunks(ksym, dtype, chunk):
    n = chunk + 513
    rec = _randn((n, 6), 302, dtype)
    dt = ksym.F32 if dtype == torch.float32 else ksym.F64
    opts = ksym.Opts.defaults(dt)
    out = ksym.eig3_aos(rec, opts=opts, outputs=("lam", "D", "phi", "flags"))
    torch.cuda.synchronize()
    for a, b in _windows(chunk, n):
        ref = ksym.eig3_aos(rec[a:b].clone(), opts=opts, outputs=("lam", "D", "phi", "flags"))
        for k in ref:
            assert torch.equal(_cols(out[k], a, b), ref[k]), (k, a, b)


def test_eig2_across_chunks(ksym):
    n = CHUNK + 99
    A = _randn((3, n), 303)
    out = ksym.eig2(A)
    torch.cuda.synchronize()
    for a, b in _windows(CHUNK, n):
        ref = ksym.eig2(_cols(A, a, b))
        for k in ref:
            assert torch.equal(_cols(out[k], a, b), ref[k]), (k, a, b)


def test_backward_across_chunks(ksym):
    n = CHUNK + 33
    lam, D = _randn((3, n), 304), _randn((9, n), 305)
    w, G = _randn((3, n), 306), _randn((9, n), 307)
    gA = ksym.eig3_backward(lam, D, w, G)
    torch.cuda.synchronize()
    for a, b in _windows(CHUNK, n):
        ref = ksym.eig3_backward(_cols(lam, a, b), _cols(D, a, b), _cols(w, a, b), _cols(G, a, b))
        assert torch.equal(_cols(gA, a, b), ref), (a, b)


def test_backward_angles_and_2x2_backward_across_chunks(ksym):
    """The 3x3 adjoint with the Euler angles' cotangent, and the 2x2 adjoint
    with the angle's cotangent."""
    n = CHUNK + 65
    lam, D = _randn((3, n), 310), _randn((9, n), 311)
    phi, gphi = _randn((3, n), 312), _randn((3, n), 313)
    gA = ksym.eig3_backward(lam, D, None, None, phi=phi, gphi=gphi)
    torch.cuda.synchronize()
    for a, b in _windows(CHUNK, n):
        ref = ksym.eig3_backward(_cols(lam, a, b), _cols(D, a, b), None, None,
                                 phi=_cols(phi, a, b), gphi=_cols(gphi, a, b))
        assert torch.equal(_cols(gA, a, b), ref), (a, b)
    del lam, D, phi, gphi, gA
    torch.cuda.empty_cache()
    n2 = CHUNK + 17
    lam2, D2, w2 = _randn((2, n2), 314), _randn((4, n2), 315), _randn((2, n2), 316)
    G2, gp2 = _randn((4, n2), 317), _randn((n2,), 318)
    gA2 = ksym.eig2_backward(lam2, D2, w2, G2, gp2)
    torch.cuda.synchronize()
    for a, b in _windows(CHUNK, n2):
        ref = ksym.eig2_backward(_cols(lam2, a, b), _cols(D2, a, b), _cols(w2, a, b), _cols(G2, a, b),
                                 _cols(gp2, a, b))
        assert torch.equal(_cols(gA2, a, b), ref), (a, b)


def test_compose_across_chunks(ksym):
    """The inverse maps (lam, phi) -> A, 3x3 and 2x2."""
    n = CHUNK + 129
    lam, phi = _randn((3, n), 319), _randn((3, n), 320)
    A = ksym.compose3(lam, phi)
    torch.cuda.synchronize()
    for a, b in _windows(CHUNK, n):
        assert torch.equal(_cols(A, a, b), ksym.compose3(_cols(lam, a, b), _cols(phi, a, b))), (a, b)
    del lam, phi, A
    torch.cuda.empty_cache()
    lam2, phi2 = _randn((2, n), 321), _randn((n,), 322)
    A2 = ksym.compose2(lam2, phi2)
    torch.cuda.synchronize()
    for a, b in _windows(CHUNK, n):
        assert torch.equal(_cols(A2, a, b), ksym.compose2(_cols(lam2, a, b), _cols(phi2, a, b))), (a, b)


def test_plan_group_across_chunks(ksym):
    """A mixed plan whose 2x2 group is larger than one chunk (the plan splits
    it into several table entries) beside a small 3x3 group."""
    n2, n3 = CHUNK + 5, 1000
    A2, A3 = _randn((3, n2), 308), _randn((6, n3), 309)
    o2 = {"lam": torch.empty((2, n2), device="cuda"), "D": torch.empty((4, n2), device="cuda"),
          "phi": torch.empty((n2,), device="cuda")}
    o3 = {"lam": torch.empty((3, n3), device="cuda"), "D": torch.empty((9, n3), device="cuda"),
          "phi": torch.empty((3, n3), device="cuda")}
    plan = ksym.Plan([(2, A2, o2), (3, A3, o3)])
    plan.run()
    torch.cuda.synchronize()
    for a, b in _windows(CHUNK, n2):
        ref = ksym.eig2(_cols(A2, a, b), opts=plan.opts)
        for k in o2:
            assert torch.equal(_cols(o2[k], a, b), ref[k]), (k, a, b)
    ref3 = ksym.eig3(A3, opts=plan.opts, outputs=("lam", "D", "phi"))
    for k in o3:
        assert torch.equal(o3[k], ref3[k]), k
    plan.close()
    assert np.isfinite(o2["lam"][:, -10:].cpu().numpy()).all()
