"""C-ABI checks that need no GPU: libksym.so loads, exports every function
include/ksym.h declares, and rejects bad arguments before touching HIP."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ksym.h")
LIB = os.path.join(ROOT, "paper_1306_6291_amd", "libksym.so")


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
    assert 1 <= o.grid_mult <= 1024
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
    for field, bad in (("block", 96), ("mats_per_lane", 3), ("grid_mult", -1), ("grid_mult", 1025),
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
    lib.ksym_plan_run.argtypes = [P, P, P]
    assert lib.ksym_plan_run(None, None, None) == 1
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
