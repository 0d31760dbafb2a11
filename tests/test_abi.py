"""C-ABI checks that need no GPU: libksym.so loads, exports every function
include/ksym.h declares, and rejects bad arguments before touching HIP."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ksym.h")
# KSYM_ABI_LIB: another build of the library to check (the sanitizer run)
LIB = os.environ.get("KSYM_ABI_LIB") or os.path.join(ROOT, "paper_1306_6291_amd", "libksym.so")


def _declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\**\s*(ksym_[a-z0-9_]+)\s*\(", src, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        # build.py by path: the package's __init__ refuses to import without the library
        import importlib.util
        spec = importlib.util.spec_from_file_location(
            "_ksym_build", os.path.join(ROOT, "paper_1306_6291_amd", "build.py"))
        b = importlib.util.module_from_spec(spec)
        spec.loader.exec_module(b)
        b.build_library()
    return ctypes.CDLL(LIB)


def test_header_declares_the_boundary():
    names = _declared_functions()
    for required in ("ksym_eig2", "ksym_eig3", "ksym_eig3_aos", "ksym_eig3_backward",
                     "ksym_eig3_workspace_bytes", "ksym_plan_create", "ksym_plan_run",
                     "ksym_plan_capture", "ksym_plan_replay", "ksym_plan_destroy",
                     "ksym_last_error", "ksym_version", "ksym_opts_default"):
        assert required in names


def test_library_exports_every_declared_symbol(lib):
    for name in _declared_functions():
        assert hasattr(lib, name), f"{name} declared in ksym.h but not exported"


def test_package_binding_has_the_same_names():
    import paper_1306_6291_amd as ksym
    for name in ("eig2", "eig3", "eig3_aos", "eig3_backward", "Plan", "Eig3Function"):
        assert hasattr(ksym, name)
    assert ksym.version() == 100


class Opts(ctypes.Structure):
    _fields_ = [("path", ctypes.c_int32), ("block", ctypes.c_int32),
                ("mats_per_lane", ctypes.c_int32), ("grid_mult", ctypes.c_int32),
                ("tau_gap", ctypes.c_double), ("tau_res", ctypes.c_double),
                ("tau_vec", ctypes.c_double), ("tau_dbl", ctypes.c_double),
                ("drain_tiles", ctypes.c_int32), ("reserved", ctypes.c_int32)]


def _err(lib):
    lib.ksym_last_error.restype = ctypes.c_char_p
    return lib.ksym_last_error().decode()


def test_defaults(lib):
    o = Opts()
    lib.ksym_opts_default(0, ctypes.byref(o))
    assert o.path == 0 and o.block == 256 and o.mats_per_lane in (1, 2, 4)
    assert 0 < o.tau_res < 1e-5
    assert o.drain_tiles >= 0 and o.reserved == 0
    assert 1 <= o.grid_mult <= 65536
    lib.ksym_opts_default(1, ctypes.byref(o))
    assert o.path == 2 and 0 < o.tau_res < 1e-9


def _planes(k, dtype_size=4, misalign=False):
    # fake, never dereferenced: every call below fails validation first
    base = 0x10000 + (1 if misalign else 0)
    return (ctypes.c_void_p * k)(*[base + i * 4096 for i in range(k)])


def test_eig3_argument_errors(lib):
    P = ctypes.c_void_p
    f = lib.ksym_eig3
    f.argtypes = [ctypes.c_int, ctypes.c_int64, P, P, P, P, P, P, P, ctypes.c_size_t, P, P]
    f.restype = ctypes.c_int
    ok = _planes(6)
    assert f(0, -1, ok, None, None, None, None, None, None, 0, None, None) == 1
    assert "n must be" in _err(lib)
    assert f(7, 10, ok, None, None, None, None, None, None, 0, None, None) == 2
    assert f(0, 0, None, None, None, None, None, None, None, 0, None, None) == 0   # nothing to do
    assert f(0, 10, None, None, None, None, None, None, None, 0, None, None) == 1
    nul = (ctypes.c_void_p * 6)(0x10000, 0x20000, None, 0x30000, 0x40000, 0x50000)
    assert f(0, 10, nul, None, None, None, None, None, None, 0, None, None) == 1
    assert "in[2]" in _err(lib)
    assert f(0, 10, _planes(6, misalign=True), None, None, None, None, None, None, 0, None, None) == 1
    assert "misaligned" in _err(lib)
    # float64 pointers must be 8-byte aligned
    odd = (ctypes.c_void_p * 6)(*[0x10004 + i * 4096 for i in range(6)])
    assert f(1, 10, odd, None, None, None, None, None, None, 0, None, None) == 1
    # workspace too small
    assert f(0, 10, ok, None, None, None, None, None, ctypes.c_void_p(0x90000), 4, None, None) == 3
    # dtype / path combinations
    o = Opts()
    lib.ksym_opts_default(0, ctypes.byref(o))
    o.path = 1
    assert f(0, 10, ok, None, None, None, None, None, None, 0, ctypes.byref(o), None) == 2
    lib.ksym_opts_default(1, ctypes.byref(o))
    o.path = 0
    assert f(1, 10, ok, None, None, None, None, None, None, 0, ctypes.byref(o), None) == 2
    # launch-shape options
    for field, bad in (("block", 96), ("mats_per_lane", 3), ("grid_mult", -1), ("grid_mult", 65537),
                       ("drain_tiles", (1 << 20) + 1)):
        lib.ksym_opts_default(0, ctypes.byref(o))
        setattr(o, field, bad)
        assert f(0, 10, ok, None, None, None, None, None, None, 0, ctypes.byref(o), None) == 1, field
    lib.ksym_opts_default(0, ctypes.byref(o))
    o.tau_res = 0.0
    assert f(0, 10, ok, None, None, None, None, None, None, 0, ctypes.byref(o), None) == 1
    # an output plane misaligned
    outs = (ctypes.c_void_p * 3)(0x70000, 0x70003, 0x71000)
    assert f(0, 10, ok, outs, None, None, None, None, None, 0, None, None) == 1


def test_eig3_aos_argument_errors(lib):
    P = ctypes.c_void_p
    f = lib.ksym_eig3_aos
    f.argtypes = [ctypes.c_int, ctypes.c_int64, P, P, P, P, P, P, P, ctypes.c_size_t, P, P]
    f.restype = ctypes.c_int
    assert f(0, 5, None, None, None, None, None, None, None, 0, None, None) == 1
    assert f(0, 5, ctypes.c_void_p(0x10008), None, None, None, None, None, None, 0, None, None) == 1
    assert "16-byte" in _err(lib)
    assert f(0, -3, ctypes.c_void_p(0x10000), None, None, None, None, None, None, 0, None, None) == 1


def test_eig2_argument_errors(lib):
    P = ctypes.c_void_p
    f = lib.ksym_eig2
    f.argtypes = [ctypes.c_int, ctypes.c_int64, P, P, P, P, P, P, P]
    f.restype = ctypes.c_int
    assert f(0, -2, _planes(3), None, None, None, None, None, None) == 1
    assert f(3, 2, _planes(3), None, None, None, None, None, None) == 2
    assert f(0, 2, None, None, None, None, None, None, None) == 1
    assert f(0, 2, _planes(3, misalign=True), None, None, None, None, None, None) == 1
    assert f(0, 0, None, None, None, None, None, None, None) == 0
    assert f(0, 2, _planes(3), None, None, ctypes.c_void_p(0x50001), None, None, None) == 1


def test_backward_argument_errors(lib):
    P = ctypes.c_void_p
    f = lib.ksym_eig3_backward
    f.argtypes = [ctypes.c_int, ctypes.c_int64, P, P, P, P, P, P, ctypes.c_double, P]
    f.restype = ctypes.c_int
    L, D, gA = _planes(3), _planes(9), _planes(6)
    assert f(0, -1, L, D, None, None, None, gA, 1e-6, None) == 1
    assert f(0, 4, None, D, None, None, None, gA, 1e-6, None) == 1
    assert f(0, 4, L, D, None, None, None, None, 1e-6, None) == 1
    assert f(0, 4, L, D, None, None, None, gA, -1.0, None) == 1
    assert f(0, 4, L, D, None, None, None, gA, float("nan"), None) == 1
    assert f(0, 0, None, None, None, None, None, None, 1e-6, None) == 0
    bad = (ctypes.c_void_p * 3)(0x1000, None, 0x3000)
    assert f(0, 4, L, D, bad, None, None, gA, 1e-6, None) == 1
    assert f(5, 4, L, D, None, None, None, gA, 1e-6, None) == 2


def test_eig2_backward_argument_errors(lib):
    P = ctypes.c_void_p
    f = lib.ksym_eig2_backward
    f.argtypes = [ctypes.c_int, ctypes.c_int64, P, P, P, P, P, P, ctypes.c_double, P]
    f.restype = ctypes.c_int
    L, D, gA = _planes(2), _planes(4), _planes(3)
    assert f(0, -1, L, D, None, None, None, gA, 1e-6, None) == 1
    assert f(0, 4, None, D, None, None, None, gA, 1e-6, None) == 1
    assert f(0, 4, L, None, None, None, None, gA, 1e-6, None) == 1
    assert f(0, 4, L, D, None, None, None, None, 1e-6, None) == 1
    assert f(0, 4, L, D, None, None, None, gA, -1.0, None) == 1
    assert f(0, 4, L, D, None, None, None, gA, float("nan"), None) == 1
    assert f(0, 0, None, None, None, None, None, None, 1e-6, None) == 0
    misaligned = (ctypes.c_void_p * 2)(0x1000, 0x1002)
    assert f(0, 4, L, D, misaligned, None, None, gA, 1e-6, None) == 1
    assert f(0, 4, L, D, None, None, ctypes.c_void_p(0x1001), gA, 1e-6, None) == 1
    assert f(5, 4, L, D, None, None, None, gA, 1e-6, None) == 2


def test_backward_angles_argument_errors(lib):
    P = ctypes.c_void_p
    f = lib.ksym_eig3_backward_angles
    f.argtypes = [ctypes.c_int, ctypes.c_int64, P, P, P, P, P, P, P, P, ctypes.c_double, P]
    f.restype = ctypes.c_int
    L, D, F, GP, gA = _planes(3), _planes(9), _planes(3), _planes(3), _planes(6)
    assert f(0, 4, L, D, None, None, None, None, GP, gA, 1e-6, None) == 1     # phi required
    assert f(0, 4, L, D, F, None, None, None, None, gA, 1e-6, None) == 1      # gphi required
    assert f(0, 4, L, D, _planes(3, misalign=True), None, None, None, GP, gA, 1e-6, None) == 1
    assert f(0, -1, L, D, F, None, None, None, GP, gA, 1e-6, None) == 1
    assert f(0, 4, L, D, F, None, None, None, GP, gA, -1.0, None) == 1
    assert f(3, 4, L, D, F, None, None, None, GP, gA, 1e-6, None) == 2


def test_compose_argument_errors(lib):
    P = ctypes.c_void_p
    f3, f2 = lib.ksym_compose3, lib.ksym_compose2
    for f in (f3, f2):
        f.argtypes = [ctypes.c_int, ctypes.c_int64, P, P, P, P]
        f.restype = ctypes.c_int
    L3, F3, A6 = _planes(3), _planes(3), _planes(6)
    assert f3(0, -1, L3, F3, A6, None) == 1
    assert f3(0, 4, None, F3, A6, None) == 1
    assert f3(0, 4, L3, None, A6, None) == 1
    assert f3(0, 4, L3, F3, None, None) == 1
    assert f3(0, 4, L3, _planes(3, misalign=True), A6, None) == 1
    assert f3(0, 0, None, None, None, None) == 0
    assert f3(7, 4, L3, F3, A6, None) == 2
    L2, A3 = _planes(2), _planes(3)
    assert f2(0, 4, L2, None, A3, None) == 1
    assert f2(0, 4, L2, ctypes.c_void_p(0x10001), A3, None) == 1
    assert f2(0, 4, None, ctypes.c_void_p(0x10000), A3, None) == 1


def test_plan_argument_errors(lib):
    P = ctypes.c_void_p
    f = lib.ksym_plan_create
    f.argtypes = [ctypes.c_int, ctypes.c_int32, P, P, P, P]
    f.restype = ctypes.c_int
    h = ctypes.c_void_p()
    assert f(0, 0, None, None, ctypes.byref(h), None) == 1
    assert f(0, 1, None, None, None, None) == 1
    assert f(9, 1, ctypes.c_void_p(0x1000), None, ctypes.byref(h), None) == 2
    import paper_1306_6291_amd as ksym
    arr = (ksym.Group * 2)()
    arr[0].kind = 4
    arr[0].n = 3
    assert f(0, 2, ctypes.cast(arr, ctypes.c_void_p), None, ctypes.byref(h), None) == 1
    assert "kind" in _err(lib)
    arr[0].kind = 3
    arr[0].n = -5
    assert f(0, 2, ctypes.cast(arr, ctypes.c_void_p), None, ctypes.byref(h), None) == 1
    arr[0].n = 10   # in pointers NULL
    assert f(0, 2, ctypes.cast(arr, ctypes.c_void_p), None, ctypes.byref(h), None) == 1
    lib.ksym_plan_destroy.argtypes = [P]
    lib.ksym_plan_destroy(None)   # no-op
    lib.ksym_plan_run.argtypes = [P, P, ctypes.c_size_t, P]
    assert lib.ksym_plan_run(None, None, 0, None) == 1
    lib.ksym_plan_capture.argtypes = [P, P, ctypes.c_size_t, P]
    assert lib.ksym_plan_capture(None, None, 0, None) == 1
    lib.ksym_plan_replay.argtypes = [P, P]
    assert lib.ksym_plan_replay(None, None) == 1


def test_zero_counters_rejects_null(lib):
    lib.ksym_zero_counters.argtypes = [ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]
    assert lib.ksym_zero_counters(None, 0, None) == 3


def test_product_path_does_not_reference_the_oracle():
    """The binding and the HIP sources never import, load or include the oracle."""
    pkg = os.path.join(ROOT, "paper_1306_6291_amd")
    for dirpath, _, files in os.walk(pkg):
        for fn in files:
            if fn.endswith((".py", ".hip", ".hpp", ".h", ".cpp")):
                txt = open(os.path.join(dirpath, fn)).read()
                assert "import oracle" not in txt and "liboracle" not in txt and "ksym_oracle" not in txt, fn


def _fake(base, k, stride=1 << 16):
    # fake device addresses, never dereferenced: each call below is rejected
    # (or, for the control calls, would launch only after every check passes;
    # those controls use n = 0 or an invalid dtype/option to stop first)
    return (ctypes.c_void_p * k)(*[base + i * stride for i in range(k)])


def test_outputs_aliasing_inputs_are_rejected(lib):
    """An output plane whose bytes overlap an input plane or another output
    plane is rejected with KSYM_E_ARG before any HIP call; the message names
    both planes."""
    P = ctypes.c_void_p
    f = lib.ksym_eig3
    f.argtypes = [ctypes.c_int, ctypes.c_int64, P, P, P, P, P, P, P, ctypes.c_size_t, P, P]
    f.restype = ctypes.c_int
    n = 1000                                   # 4000 bytes per float32 plane
    ins = _fake(0x100000, 6)
    lam = _fake(0x900000, 3)
    # lam[1] starts inside in[4] (0x140000 .. 0x140fa0)
    bad = (ctypes.c_void_p * 3)(0x900000, 0x140f00, 0x920000)
    assert f(0, n, ins, bad, None, None, None, None, None, 0, None, None) == 1
    msg = _err(lib)
    assert "lam[1]" in msg and "in[4]" in msg
    # an output overlapping another output (D[5] over lam[2])
    D = _fake(0xa00000, 9)
    D[5] = 0x920010
    assert f(0, n, ins, lam, D, None, None, None, None, 0, None, None) == 1
    assert "overlaps" in _err(lib)
    # the flags plane (n bytes) over an input, and the workspace over an output
    assert f(0, n, ins, lam, None, None, None, ctypes.c_void_p(0x100100), None, 0, None, None) == 1
    assert "flags" in _err(lib)
    assert f(0, n, ins, lam, None, None, None, None, ctypes.c_void_p(0x910000), 256, None, None) == 1
    assert "ws" in _err(lib)
    # control calls: block 1024 passes the option checks, but no 3x3 kernel is
    # compiled for it, so a call that clears every argument check stops with
    # KSYM_E_UNSUPPORTED just before its first HIP call
    o = Opts()
    lib.ksym_opts_default(0, ctypes.byref(o))
    o.block = 1024
    assert f(0, n, ins, lam, None, None, None, None, None, 0, ctypes.byref(o), None) == 5
    # float64 planes are twice as long: lam[0] starts 4096 bytes into in[5],
    # past a float32 plane of n elements (4000 bytes) but inside a float64 one
    near = (ctypes.c_void_p * 3)(0x100000 + 5 * (1 << 16) + 4096, 0x980000, 0x990000)
    assert f(0, n, ins, near, None, None, None, None, None, 0, ctypes.byref(o), None) == 5
    lib.ksym_opts_default(1, ctypes.byref(o))
    o.block = 1024
    assert f(1, n, ins, near, None, None, None, None, None, 0, ctypes.byref(o), None) == 1
    assert "lam[0]" in _err(lib) and "in[5]" in _err(lib)
    # inputs may share memory with each other (the same plane six times)
    same = (ctypes.c_void_p * 6)(*([0x100000] * 6))
    lib.ksym_opts_default(0, ctypes.byref(o))
    o.block = 1024
    assert f(0, n, same, lam, None, None, None, None, None, 0, ctypes.byref(o), None) == 5


def test_aliasing_rejected_in_every_entry_point(lib):
    P = ctypes.c_void_p
    n = 64
    # AoS records: the n x 6 block covers 0x100000 .. +1536 bytes
    f = lib.ksym_eig3_aos
    f.argtypes = [ctypes.c_int, ctypes.c_int64, P, P, P, P, P, P, P, ctypes.c_size_t, P, P]
    f.restype = ctypes.c_int
    lam = (ctypes.c_void_p * 3)(0x900000, 0x100400, 0x920000)
    assert f(0, n, ctypes.c_void_p(0x100000), lam, None, None, None, None, None, 0, None, None) == 1
    assert "a_aos" in _err(lib)
    # 2x2 forward: phi over A12
    g = lib.ksym_eig2
    g.argtypes = [ctypes.c_int, ctypes.c_int64, P, P, P, P, P, P, P]
    g.restype = ctypes.c_int
    ins = _fake(0x100000, 3)
    assert g(0, n, ins, None, None, ctypes.c_void_p(0x120000 + 8), None, None, None) == 1
    assert "phi" in _err(lib) and "in[2]" in _err(lib)
    # 3x3 adjoint: gA[3] over gD[8]
    b = lib.ksym_eig3_backward
    b.argtypes = [ctypes.c_int, ctypes.c_int64, P, P, P, P, P, P, ctypes.c_double, P]
    b.restype = ctypes.c_int
    L, D, gl, gD = _fake(0x100000, 3), _fake(0x200000, 9), _fake(0x300000, 3), _fake(0x400000, 9)
    gA = _fake(0x500000, 6)
    gA[3] = 0x400000 + 8 * (1 << 16)
    assert b(0, n, L, D, None, gl, gD, gA, 1e-6, None) == 1
    assert "gA[3]" in _err(lib) and "gD[8]" in _err(lib)
    # angle adjoint: gA over phi
    ba = lib.ksym_eig3_backward_angles
    ba.argtypes = [ctypes.c_int, ctypes.c_int64, P, P, P, P, P, P, P, P, ctypes.c_double, P]
    ba.restype = ctypes.c_int
    F, GP = _fake(0x600000, 3), _fake(0x700000, 3)
    gA2 = _fake(0x600000 + 2 * (1 << 16), 6)
    assert ba(0, n, L, D, F, None, gl, gD, GP, gA2, 1e-6, None) == 1
    assert "phi" in _err(lib)
    # 2x2 adjoint: gA[0] over gphi
    b2 = lib.ksym_eig2_backward
    b2.argtypes = [ctypes.c_int, ctypes.c_int64, P, P, P, P, P, P, ctypes.c_double, P]
    b2.restype = ctypes.c_int
    gA3 = (ctypes.c_void_p * 3)(0x800000, 0x810000, 0x820000)
    assert b2(0, n, _fake(0x100000, 2), _fake(0x200000, 4), None, None, ctypes.c_void_p(0x800000), gA3,
              1e-6, None) == 1
    assert "gphi" in _err(lib)
    # inverse maps: A[5] over lam[0]
    c3 = lib.ksym_compose3
    c3.argtypes = [ctypes.c_int, ctypes.c_int64, P, P, P, P]
    c3.restype = ctypes.c_int
    A6 = _fake(0x900000, 6)
    A6[5] = 0x100000
    assert c3(0, n, _fake(0x100000, 3), _fake(0x200000, 3), A6, None) == 1
    assert "A[5]" in _err(lib) and "lam[0]" in _err(lib)
    c2 = lib.ksym_compose2
    c2.argtypes = [ctypes.c_int, ctypes.c_int64, P, P, P, P]
    c2.restype = ctypes.c_int
    assert c2(0, n, _fake(0x100000, 2), ctypes.c_void_p(0x300000), _fake(0x300000, 3), None) == 1
    assert "A[0]" in _err(lib)


def test_plan_rejects_aliasing_across_groups(lib):
    """A plan whose group 1 writes over group 0's input is rejected before
    anything is allocated."""
    import paper_1306_6291_amd as ksym
    P = ctypes.c_void_p
    f = lib.ksym_plan_create
    f.argtypes = [ctypes.c_int, ctypes.c_int32, P, P, P, P]
    f.restype = ctypes.c_int
    arr = (ksym.Group * 2)()
    for g, base in enumerate((0x1000000, 0x2000000)):
        arr[g].kind = 3
        arr[g].n = 100
        for c in range(6):
            arr[g].in_[c] = base + c * 0x10000
        for c in range(3):
            arr[g].lam[c] = base + 0x100000 + c * 0x10000
    arr[1].lam[2] = 0x1000000 + 3 * 0x10000 + 64      # inside group 0's in[3]
    h = ctypes.c_void_p()
    assert f(0, 2, ctypes.cast(arr, ctypes.c_void_p), None, ctypes.byref(h), None) == 1
    assert "overlaps" in _err(lib)
    assert not h.value


def _noalloc(lib):
    f = lib.ksym_mixed_run_noalloc
    P = ctypes.c_void_p
    f.argtypes = [ctypes.c_int, ctypes.c_int32, P, P, P, ctypes.c_size_t, P]
    f.restype = ctypes.c_int
    return f


def _disjoint_groups(ksym, ng, n, kind=3, stride=0x100000):
    """ng groups of n matrices at made-up, non-overlapping addresses (never
    dereferenced: every case below is rejected before any HIP call)."""
    arr = (ksym.Group * ng)()
    base = 0x10000000
    for g in range(ng):
        arr[g].kind = kind
        arr[g].n = n
        for c in range(6 if kind == 3 else 3):
            arr[g].in_[c] = base
            base += stride
        for c in range(3 if kind == 3 else 2):
            arr[g].lam[c] = base
            base += stride
    return arr


def test_noalloc_rejects_bad_batches_before_any_hip_call(lib):
    """ksym_mixed_run_noalloc: group count, chunk count and tile count beyond
    the fixed tables, bad groups, aliasing across groups and a short
    workspace are KSYM_E_ARG / KSYM_E_WORKSPACE, reported before any HIP call
    (this host has no GPU)."""
    import paper_1306_6291_amd as ksym
    f = _noalloc(lib)
    arr = _disjoint_groups(ksym, 2, 1000)
    g = ctypes.cast(arr, ctypes.c_void_p)
    assert f(0, 0, g, None, None, 0, None) == 1
    assert f(0, 2, None, None, None, 0, None) == 1
    assert f(7, 2, g, None, None, 0, None) == 2
    big = _disjoint_groups(ksym, 4097, 1, stride=0x1000)
    assert f(0, 4097, ctypes.cast(big, ctypes.c_void_p), None, None, 0, None) == 1
    assert "at most 4096" in _err(lib)
    # 2^21 tiles of 64 matrices: one group of 2^27 + 1 matrices needs one more
    one = _disjoint_groups(ksym, 1, (1 << 27) + 1, stride=1 << 30)
    assert f(0, 1, ctypes.cast(one, ctypes.c_void_p), None, None, 0, None) == 1
    assert "wave tiles" in _err(lib)
    # 8192 chunks of 2^28: 33 groups of 2^33 matrices give 33 * 32 = 1056 chunks
    # (allowed), 257 such groups 8224 (too many)
    many = _disjoint_groups(ksym, 257, 1 << 33, stride=1 << 36)
    assert f(1, 257, ctypes.cast(many, ctypes.c_void_p), None, None, 0, None) == 1
    assert "chunks" in _err(lib)
    arr[1].kind = 5
    assert f(0, 2, g, None, None, 0, None) == 1
    arr[1].kind = 3
    arr[1].lam[2] = arr[0].in_[4] + 64          # an output inside another group's input
    assert f(0, 2, g, None, None, 0, None) == 1
    assert "overlaps" in _err(lib)
    arr = _disjoint_groups(ksym, 2, 1000)
    g = ctypes.cast(arr, ctypes.c_void_p)
    ws = 0x7000000000
    assert f(0, 2, g, None, ctypes.c_void_p(ws), 4, None) == 3     # too small
    assert f(0, 2, g, None, ctypes.c_void_p(ws + 2), 256, None) == 3  # misaligned
    assert f(0, 2, g, None, ctypes.c_void_p(arr[0].lam[1]), 256, None) == 1  # ws inside an output
    assert "overlaps" in _err(lib)


def test_binding_row_pointers_and_line_aligned_planes():
    """Host logic of the binding (CPU tensors, no GPU call): row pointers of a
    contiguous (k, n) tensor, of a row-strided view and of a plane list; a
    transposed view is refused; _planes and line_aligned_planes round the
    row stride up to 256 bytes only when n needs it."""
    torch = pytest.importorskip("torch")
    import paper_1306_6291_amd as ksym
    t = torch.zeros((6, 1000))
    ptrs, n, _ = ksym._rows(t, 6)
    assert n == 1000 and [p - ptrs[0] for p in ptrs] == [c * 4000 for c in range(6)]
    wide = torch.zeros((3, 1024))[:, :1000]
    ptrs, n, _ = ksym._rows(wide, 3)
    assert n == 1000 and [p - ptrs[0] for p in ptrs] == [0, 4096, 8192]
    with pytest.raises(ValueError):
        ksym._rows(torch.zeros((1000, 3)).T, 3)
    with pytest.raises(ValueError):
        ksym._rows(torch.zeros((4, 1000)), 3)
    planes = [torch.zeros(7) for _ in range(3)]
    assert ksym._rows(planes, 3)[0] == [p.data_ptr() for p in planes]
    for dtype, es in ((torch.float32, 4), (torch.float64, 8)):
        for n in (0, 1, 63, 64, 65, 1000, 1 << 14):
            p = ksym._planes(5, n, dtype, "cpu")
            assert p.shape == (5, n)
            if n > 0:
                row = n if p.is_contiguous() else p.stride(0)
                assert (row * es) % 256 == 0 and n <= row < n + 256 // es, (dtype, n, row)
            lst = ksym.line_aligned_planes(3, n, dtype=dtype, device="cpu")
            assert len(lst) == 3 and all(x.numel() == n and x.is_contiguous() for x in lst)
            assert all((x.data_ptr() - lst[0].data_ptr()) % 256 == 0 for x in lst)
    # contiguous when n already fills whole 256-byte blocks
    assert ksym._planes(3, 1 << 14, torch.float32, "cpu").is_contiguous()
    assert not ksym._planes(3, 1000, torch.float32, "cpu").is_contiguous()
