"""ksym: batched closed-form eigendecomposition of 2x2 / 3x3 real symmetric
matrices on AMD MI355X (gfx950), after Kronenburg, arXiv:1306.6291.

This module is argument marshalling only: torch supplies device memory and the
current HIP stream, every computation runs in the HIP kernels of libksym.so
behind the C ABI of include/ksym.h.  If libksym.so is missing, importing this
package raises -- there is no fallback path.

Tensors are structure-of-arrays: a 3x3 batch is a (6, n) tensor whose rows are
the planes A11, A22, A33, A12, A13, A23; a 2x2 batch is (3, n) with rows A11,
A22, A12.  Outputs: lam (3, n) in the slots (max, min, mid), D (9, n) row-major
with column k the eigenvector of lam[k], phi (3, n) with D = R1 R2 R3 (paper
eq. (2.6)), gap (3, n) = (max-min, max-mid, mid-min), flags (n,) uint8.
"""

from __future__ import annotations

import ctypes
import json
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libksym.so")
TUNED_PATH = os.path.join(_HERE, "tuned.json")

if not os.path.exists(LIB_PATH):
    raise ImportError(
        f"{LIB_PATH} is missing: build it with `python paper_1306_6291_amd/build.py` "
        "(hipcc, gfx950).  There is no fallback implementation.")

_lib = ctypes.CDLL(LIB_PATH)

F32, F64 = 0, 1
PATH_DEFAULT, PATH_FP32_FIXUP, PATH_FP64_PLAIN, PATH_FP64_FIXUP = -1, 0, 1, 2
FLAG_GENERAL, FLAG_DOUBLE, FLAG_TRIPLE, FLAG_FIXUP, FLAG_NONFINITE = 0, 1, 2, 4, 8
STATUS = {0: "KSYM_OK", 1: "KSYM_E_ARG", 2: "KSYM_E_DTYPE", 3: "KSYM_E_WORKSPACE",
          4: "KSYM_E_HIP", 5: "KSYM_E_UNSUPPORTED"}


class KsymError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class Opts(ctypes.Structure):
    _fields_ = [("path", ctypes.c_int32), ("block", ctypes.c_int32),
                ("mats_per_lane", ctypes.c_int32), ("grid_mult", ctypes.c_int32),
                ("tau_gap", ctypes.c_double), ("tau_res", ctypes.c_double),
                ("tau_vec", ctypes.c_double), ("tau_dbl", ctypes.c_double),
                ("drain_tiles", ctypes.c_int32), ("reserved", ctypes.c_int32)]

    @classmethod
    def defaults(cls, dtype=F32, **kw):
        o = cls()
        _lib.ksym_opts_default(dtype, ctypes.byref(o))
        for k, v in kw.items():
            setattr(o, k, v)
        return o

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class Group(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("n", ctypes.c_int64),
                ("in_", ctypes.c_void_p * 6), ("lam", ctypes.c_void_p * 3),
                ("D", ctypes.c_void_p * 9), ("phi", ctypes.c_void_p * 3),
                ("flags", ctypes.c_void_p)]


_P = ctypes.c_void_p
_lib.ksym_version.restype = ctypes.c_int
_lib.ksym_last_error.restype = ctypes.c_char_p
_lib.ksym_opts_default.argtypes = [ctypes.c_int, ctypes.POINTER(Opts)]
_lib.ksym_opts_default.restype = None
_lib.ksym_eig2.argtypes = [ctypes.c_int, ctypes.c_int64, _P, _P, _P, _P, _P, ctypes.POINTER(Opts), _P]
_lib.ksym_eig3_workspace_bytes.argtypes = [ctypes.c_int, ctypes.c_int64]
_lib.ksym_eig3_workspace_bytes.restype = ctypes.c_size_t
_lib.ksym_zero_counters.argtypes = [_P, ctypes.c_size_t, _P]
_lib.ksym_eig3.argtypes = [ctypes.c_int, ctypes.c_int64, _P, _P, _P, _P, _P, _P, _P, ctypes.c_size_t,
                           ctypes.POINTER(Opts), _P]
_lib.ksym_eig3_aos.argtypes = [ctypes.c_int, ctypes.c_int64, _P, _P, _P, _P, _P, _P, _P,
                               ctypes.c_size_t, ctypes.POINTER(Opts), _P]
_lib.ksym_eig3_backward.argtypes = [ctypes.c_int, ctypes.c_int64, _P, _P, _P, _P, _P, _P,
                                    ctypes.c_double, _P]
_lib.ksym_eig2_backward.argtypes = [ctypes.c_int, ctypes.c_int64, _P, _P, _P, _P, _P, _P,
                                    ctypes.c_double, _P]
_lib.ksym_eig3_backward_angles.argtypes = [ctypes.c_int, ctypes.c_int64, _P, _P, _P, _P, _P, _P, _P, _P,
                                           ctypes.c_double, _P]
_lib.ksym_compose3.argtypes = [ctypes.c_int, ctypes.c_int64, _P, _P, _P, _P]
_lib.ksym_compose2.argtypes = [ctypes.c_int, ctypes.c_int64, _P, _P, _P, _P]
_lib.ksym_plan_create.argtypes = [ctypes.c_int, ctypes.c_int32, ctypes.POINTER(Group),
                                  ctypes.POINTER(Opts), ctypes.POINTER(ctypes.c_void_p),
                                  ctypes.POINTER(ctypes.c_size_t)]
_lib.ksym_plan_run.argtypes = [_P, _P, ctypes.c_size_t, _P]
_lib.ksym_plan_capture.argtypes = [_P, _P, ctypes.c_size_t, _P]
_lib.ksym_mixed_run_noalloc.argtypes = [ctypes.c_int, ctypes.c_int32, ctypes.POINTER(Group),
                                        ctypes.POINTER(Opts), _P, ctypes.c_size_t, _P]
_lib.ksym_plan_replay.argtypes = [_P, _P]
_lib.ksym_plan_info.argtypes = [_P, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int32)]
_lib.ksym_plan_destroy.argtypes = [_P]
_lib.ksym_plan_destroy.restype = None
for _f in ("ksym_eig2", "ksym_zero_counters", "ksym_eig3", "ksym_eig3_aos", "ksym_eig3_backward",
           "ksym_eig2_backward", "ksym_compose3", "ksym_compose2", "ksym_eig3_backward_angles",
           "ksym_plan_create", "ksym_plan_run", "ksym_plan_capture", "ksym_plan_replay",
           "ksym_plan_info", "ksym_mixed_run_noalloc"):
    getattr(_lib, _f).restype = ctypes.c_int


def version():
    return _lib.ksym_version()


def _check(status):
    if status != 0:
        raise KsymError(status, _lib.ksym_last_error().decode(errors="replace"))


def _dt(t):
    if t.dtype == torch.float32:
        return F32
    if t.dtype == torch.float64:
        return F64
    raise TypeError(f"ksym supports float32 and float64 tensors, got {t.dtype}")


def _first_plane(planes):
    """A tensor of a group's inputs: the (k, n) tensor, or the first of its k planes."""
    return planes[0] if isinstance(planes, (list, tuple)) else planes


def _ptr_array(ptrs):
    return (ctypes.c_void_p * len(ptrs))(*[p if p else None for p in ptrs])


def _rows(t, k):
    """Pointers of the k rows of a (k, n) tensor whose rows are each contiguous
    (a contiguous tensor, or a view of a wider one as _planes makes), or of a
    list of k 1-D tensors."""
    if isinstance(t, (list, tuple)):
        assert len(t) == k
        n = t[0].numel()
        for x in t:
            if not x.is_contiguous() or x.numel() != n or x.dtype != t[0].dtype or x.device != t[0].device:
                raise ValueError("planes must be contiguous, same length, dtype and device")
        return [x.data_ptr() for x in t], n, t[0]
    if t.dim() != 2 or t.shape[0] != k:
        raise ValueError(f"expected a ({k}, n) tensor, got shape {tuple(t.shape)}")
    n = t.shape[1]
    if t.is_contiguous():
        row = n
    elif t.stride(1) == 1 and t.stride(0) >= n:
        row = t.stride(0)
    else:
        raise ValueError(f"the rows of the ({k}, n) tensor must each be contiguous (stride {tuple(t.stride())})")
    es = t.element_size()
    base = t.data_ptr()
    return [base + c * row * es for c in range(k)], n, t


def _planes(k, n, dtype, device):
    """A (k, n) tensor of output planes that each start on a 256-byte
    boundary: contiguous when n elements fill whole 256-byte blocks, else a
    view of a (k, stride) allocation with the row stride rounded up.  Output
    planes that share cache lines between the tiles of two waves measured
    30-40 % slower."""
    es = torch.empty((), dtype=dtype).element_size()
    stride = -(-max(int(n), 1) * es // 256) * 256 // es
    if stride == n:
        return torch.empty((k, n), dtype=dtype, device=device)
    return torch.empty((k, stride), dtype=dtype, device=device)[:, :n]


def _stream(t):
    if not t.is_cuda:
        raise ValueError("ksym works on device tensors (torch.device('cuda'))")
    return ctypes.c_void_p(torch.cuda.current_stream(t.device).cuda_stream)


def _opts(dtype, opts, **kw):
    if opts is None:
        opts = tuned_opts(kw.pop("_kind", "eig3"), dtype)
    else:
        kw.pop("_kind", None)
    if isinstance(opts, dict):
        opts = Opts.defaults(dtype, **opts)
    for k, v in kw.items():
        if v is not None:
            setattr(opts, k, v)
    return opts


_TUNED = None


def tuned_opts(kind="eig3", dtype=F32):
    """Options the autotuner recorded for (kind, dtype), else the library defaults."""
    global _TUNED
    if _TUNED is None:
        _TUNED = {}
        if os.path.exists(TUNED_PATH):
            with open(TUNED_PATH) as f:
                _TUNED = json.load(f)
    key = f"{kind}/{'f32' if dtype == F32 else 'f64'}"
    rec = _TUNED.get(key)
    if rec:
        return Opts.defaults(dtype, **rec["opts"])
    return Opts.defaults(dtype)


def line_aligned_planes(k, n, dtype=torch.float32, device="cuda", fill=None):
    """k planes of n elements that each start on a 256-byte boundary: one
    (k, stride) allocation with the row stride rounded up to 64 elements (the
    caching allocator's blocks are 512-byte aligned), returned as a list of
    1-D views.  Mixed-batch groups laid out this way let the launch stream its
    loads and stores (include/ksym.h, ksym_group).  fill: optional (k, n)
    tensor or array copied in."""
    t = _planes(k, n, dtype, device)
    if fill is not None:
        t.copy_(torch.as_tensor(fill))
    return [t[c] for c in range(k)]


def workspace(device=None):
    """A small device workspace (counters) for eig3: uint32[64]."""
    nbytes = _lib.ksym_eig3_workspace_bytes(F32, 0)
    return torch.zeros(nbytes // 4, dtype=torch.int32, device=device or "cuda")


# ---------------------------------------------------------------- 2x2 -------
def eig2(planes, opts=None, out=None):
    """2x2 forward (paper §3).  planes: (3, n) tensor (A11, A22, A12).
    Returns dict lam (2, n), D (4, n) = (D11, D12, D21, D22), phi (n,), flags (n,);
    lam and D rows each start on a 256-byte boundary (see eig3)."""
    ptrs, n, ref = _rows(planes, 3)
    dt = _dt(ref)
    o = _opts(dt, opts, _kind="eig2")
    if out is None:
        out = {"lam": _planes(2, n, ref.dtype, ref.device),
               "D": _planes(4, n, ref.dtype, ref.device),
               "phi": torch.empty((n,), dtype=ref.dtype, device=ref.device),
               "flags": torch.empty((n,), dtype=torch.uint8, device=ref.device)}
    lam = _ptr_array(_rows(out["lam"], 2)[0]) if out.get("lam") is not None else None
    D = _ptr_array(_rows(out["D"], 4)[0]) if out.get("D") is not None else None
    phi = out["phi"].data_ptr() if out.get("phi") is not None else None
    fl = out["flags"].data_ptr() if out.get("flags") is not None else None
    _check(_lib.ksym_eig2(dt, n, _ptr_array(ptrs), lam, D, phi, fl, ctypes.byref(o), _stream(ref)))
    return out


# ---------------------------------------------------------------- 3x3 -------
def _alloc3(n, ref, outputs):
    rows = {"lam": 3, "D": 9, "phi": 3, "gap": 3}
    out = {k: _planes(rows[k], n, ref.dtype, ref.device) for k in rows if k in outputs}
    if "flags" in outputs:
        out["flags"] = torch.empty((n,), dtype=torch.uint8, device=ref.device)
    return out


def _out_ptrs3(out):
    def arr(key, k):
        t = out.get(key)
        return _ptr_array(_rows(t, k)[0]) if t is not None else None
    fl = out.get("flags")
    return arr("lam", 3), arr("D", 9), arr("phi", 3), arr("gap", 3), (fl.data_ptr() if fl is not None else None)


def eig3(planes, opts=None, path=None, outputs=("lam", "D", "phi", "flags"), out=None, ws=None):
    """3x3 forward (paper §4-§5).  planes: (6, n) tensor or 6 plane tensors.
    path: PATH_FP32_FIXUP (float32), PATH_FP64_PLAIN or PATH_FP64_FIXUP (float64).
    Outputs the binding allocates are (k, n) tensors whose rows each start on
    a 256-byte boundary: row-strided views when n needs it (use reshape, not
    view, on them).
    ws: optional workspace() tensor; its words 0 and 1 accumulate the counts of
    refined and non-finite matrices."""
    ptrs, n, ref = _rows(planes, 6)
    dt = _dt(ref)
    # no D and no angles (float32): the eigenvalues-only kernel, tuned apart
    wanted = (lambda k: out.get(k) is not None) if out is not None else (lambda k: k in outputs)
    lam_only = dt == F32 and not wanted("D") and not wanted("phi")
    o = _opts(dt, opts, path=path, _kind="eig3_lam" if lam_only else "eig3")
    if out is None:
        out = _alloc3(n, ref, outputs)
    lam, D, phi, gap, fl = _out_ptrs3(out)
    wsp, wsb = (ws.data_ptr(), ws.numel() * ws.element_size()) if ws is not None else (None, 0)
    _check(_lib.ksym_eig3(dt, n, _ptr_array(ptrs), lam, D, phi, gap, fl, wsp, wsb, ctypes.byref(o),
                          _stream(ref)))
    return out


def eig3_aos(records, opts=None, path=None, outputs=("lam", "D", "phi", "flags"), out=None, ws=None):
    """3x3 forward on array-of-structures input: records (n, 6) contiguous with
    columns A11, A22, A33, A12, A13, A23 (16-byte aligned base)."""
    if records.dim() != 2 or records.shape[1] != 6 or not records.is_contiguous():
        raise ValueError("records must be a contiguous (n, 6) tensor")
    n = records.shape[0]
    dt = _dt(records)
    o = _opts(dt, opts, path=path, _kind="eig3_aos")
    if out is None:
        out = _alloc3(n, records, outputs)
    lam, D, phi, gap, fl = _out_ptrs3(out)
    wsp, wsb = (ws.data_ptr(), ws.numel() * ws.element_size()) if ws is not None else (None, 0)
    _check(_lib.ksym_eig3_aos(dt, n, records.data_ptr(), lam, D, phi, gap, fl, wsp, wsb,
                              ctypes.byref(o), _stream(records)))
    return out


def eig3_backward(lam, D, glam=None, gD=None, gap=None, eps_rel=None, out=None, phi=None, gphi=None):
    """Adjoint of eig3 for the plane gradients gA (6, n); see include/ksym.h.
    With gphi (the cotangent of the Euler angles) the angles phi are needed
    too, and ksym_eig3_backward_angles runs."""
    lp, n, ref = _rows(lam, 3)
    dt = _dt(ref)
    if eps_rel is None:
        eps_rel = 1e-6 if dt == F32 else 1e-12
    Dp = _rows(D, 9)[0]
    gl = _ptr_array(_rows(glam, 3)[0]) if glam is not None else None
    gd = _ptr_array(_rows(gD, 9)[0]) if gD is not None else None
    gp = _ptr_array(_rows(gap, 3)[0]) if gap is not None else None
    if out is None:
        out = _planes(6, n, ref.dtype, ref.device)
    if gphi is not None:
        if phi is None:
            raise ValueError("gphi needs the angles phi")
        _check(_lib.ksym_eig3_backward_angles(dt, n, _ptr_array(lp), _ptr_array(Dp), _ptr_array(_rows(phi, 3)[0]),
                                              gp, gl, gd, _ptr_array(_rows(gphi, 3)[0]),
                                              _ptr_array(_rows(out, 6)[0]), float(eps_rel), _stream(ref)))
        return out
    _check(_lib.ksym_eig3_backward(dt, n, _ptr_array(lp), _ptr_array(Dp), gp, gl, gd,
                                   _ptr_array(_rows(out, 6)[0]), float(eps_rel), _stream(ref)))
    return out


def eig2_backward(lam, D, glam=None, gD=None, gphi=None, eps_rel=None, out=None):
    """Adjoint of eig2 for the plane gradients gA (3, n) = (A11, A22, A12) from
    the forward outputs lam (2, n), D (4, n) and the cotangents of lam, D and
    phi (None = zero); see include/ksym.h."""
    lp, n, ref = _rows(lam, 2)
    dt = _dt(ref)
    if eps_rel is None:
        eps_rel = 1e-6 if dt == F32 else 1e-12
    Dp = _rows(D, 4)[0]
    gl = _ptr_array(_rows(glam, 2)[0]) if glam is not None else None
    gd = _ptr_array(_rows(gD, 4)[0]) if gD is not None else None
    gp = None
    if gphi is not None:
        if gphi.dtype != ref.dtype or not gphi.is_contiguous() or gphi.numel() != n:
            raise ValueError("gphi must be a contiguous (n,) tensor of the planes' dtype")
        gp = gphi.data_ptr()
    if out is None:
        out = _planes(3, n, ref.dtype, ref.device)
    _check(_lib.ksym_eig2_backward(dt, n, _ptr_array(lp), _ptr_array(Dp), gl, gd, gp,
                                   _ptr_array(_rows(out, 3)[0]), float(eps_rel), _stream(ref)))
    return out


def compose3(lam, phi, out=None):
    """Inverse map, eq. (2.6): the planes (6, n) of A = D diag(lam) D^T with
    D = R1(phi1) R2(phi2) R3(phi3), from lam (3, n) and phi (3, n)."""
    lp, n, ref = _rows(lam, 3)
    fp = _rows(phi, 3)[0]
    if out is None:
        out = _planes(6, n, ref.dtype, ref.device)
    _check(_lib.ksym_compose3(_dt(ref), n, _ptr_array(lp), _ptr_array(fp), _ptr_array(_rows(out, 6)[0]),
                              _stream(ref)))
    return out


def compose2(lam, phi, out=None):
    """Inverse map, eq. (2.5): the planes (3, n) = (A11, A22, A12) of
    R(phi) diag(lam) R(phi)^T, from lam (2, n) and phi (n,)."""
    lp, n, ref = _rows(lam, 2)
    if phi.dtype != ref.dtype or not phi.is_contiguous() or phi.numel() != n:
        raise ValueError("phi must be a contiguous (n,) tensor of lam's dtype")
    if out is None:
        out = _planes(3, n, ref.dtype, ref.device)
    _check(_lib.ksym_compose2(_dt(ref), n, _ptr_array(lp), phi.data_ptr(), _ptr_array(_rows(out, 3)[0]),
                              _stream(ref)))
    return out


def zero_counters(ws):
    _check(_lib.ksym_zero_counters(ws.data_ptr(), ws.numel() * ws.element_size(), _stream(ws)))


# ------------------------------------------------------------ autograd ------
def _grad_opts(planes, opts):
    """Forward options for a differentiated call: the caller's, else the tuned
    gradient setting, whose tau_vec > 0 has the forward remove each
    eigenvector pair's first-order rotation in float64 (the adjoint's
    1/(lam_i - lam_j) terms would magnify it)."""
    return opts if opts is not None else tuned_opts("eig3_grad", _dt(planes))


class Eig3Function(torch.autograd.Function):
    """lam, D = Eig3Function.apply(planes, eps_rel, opts): differentiable in lam
    and D through the hand-written adjoint kernel.  planes is a (6, n) tensor;
    opts None takes the tuned gradient setting (tau_vec > 0)."""

    @staticmethod
    def forward(ctx, planes, eps_rel=None, opts=None):
        out = eig3(planes.contiguous(), opts=_grad_opts(planes, opts), outputs=("lam", "D", "gap"))
        ctx.save_for_backward(out["lam"], out["D"], out["gap"])
        ctx.eps_rel = eps_rel
        return out["lam"], out["D"]

    @staticmethod
    def backward(ctx, glam, gD):
        lam, D, gap = ctx.saved_tensors
        gA = eig3_backward(lam, D, glam.contiguous() if glam is not None else None,
                           gD.contiguous() if gD is not None else None, gap=gap,
                           eps_rel=ctx.eps_rel)
        return gA, None, None


def eig3_autograd(planes, eps_rel=None, opts=None):
    return Eig3Function.apply(planes, eps_rel, opts)


class Eig3AnglesFunction(torch.autograd.Function):
    """lam, D, phi = Eig3AnglesFunction.apply(planes, eps_rel, opts):
    differentiable in lam, D and the Euler angles (regularised at gimbal lock;
    the angles are not differentiable where they wrap); opts as for
    Eig3Function."""

    @staticmethod
    def forward(ctx, planes, eps_rel=None, opts=None):
        out = eig3(planes.contiguous(), opts=_grad_opts(planes, opts), outputs=("lam", "D", "phi", "gap"))
        ctx.save_for_backward(out["lam"], out["D"], out["phi"], out["gap"])
        ctx.eps_rel = eps_rel
        return out["lam"], out["D"], out["phi"]

    @staticmethod
    def backward(ctx, glam, gD, gphi):
        lam, D, phi, gap = ctx.saved_tensors
        gA = eig3_backward(lam, D, glam.contiguous() if glam is not None else None,
                           gD.contiguous() if gD is not None else None, gap=gap, eps_rel=ctx.eps_rel,
                           phi=phi, gphi=gphi.contiguous() if gphi is not None else None)
        return gA, None, None


def eig3_autograd_angles(planes, eps_rel=None, opts=None):
    return Eig3AnglesFunction.apply(planes, eps_rel, opts)


class Eig2Function(torch.autograd.Function):
    """lam, D, phi = Eig2Function.apply(planes, eps_rel): differentiable in lam,
    D and phi through the 2x2 adjoint kernel.  planes is a (3, n) tensor."""

    @staticmethod
    def forward(ctx, planes, eps_rel=None, opts=None):
        out = eig2(planes.contiguous(), opts=opts)
        ctx.save_for_backward(out["lam"], out["D"])
        ctx.eps_rel = eps_rel
        return out["lam"], out["D"], out["phi"]

    @staticmethod
    def backward(ctx, glam, gD, gphi):
        lam, D = ctx.saved_tensors
        gA = eig2_backward(lam, D, glam.contiguous() if glam is not None else None,
                           gD.contiguous() if gD is not None else None,
                           gphi.contiguous() if gphi is not None else None, eps_rel=ctx.eps_rel)
        return gA, None, None


def eig2_autograd(planes, eps_rel=None, opts=None):
    return Eig2Function.apply(planes, eps_rel, opts)


# ------------------------------------------------------- mixed plans --------
def _group_array(groups):
    """ctypes array of ksym_group for [(kind, planes, out), ...] (see Plan)."""
    arr = (Group * len(groups))()
    for g, (kind, planes, out) in enumerate(groups):
        k = 3 if kind == 3 else 2
        ptrs, n, t = _rows(planes, 6 if k == 3 else 3)
        G = arr[g]
        G.kind = k
        G.n = n
        for c, p in enumerate(ptrs):
            G.in_[c] = p
        nl, nd = (3, 9) if k == 3 else (2, 4)
        if out.get("lam") is not None:
            for c, p in enumerate(_rows(out["lam"], nl)[0]):
                G.lam[c] = p
        if out.get("D") is not None:
            for c, p in enumerate(_rows(out["D"], nd)[0]):
                G.D[c] = p
        if out.get("phi") is not None:
            ph = out["phi"]
            if k == 3:
                for c, p in enumerate(_rows(ph, 3)[0]):
                    G.phi[c] = p
            else:
                G.phi[0] = ph.data_ptr()
        if out.get("flags") is not None:
            G.flags = out["flags"].data_ptr()
    return arr


class Plan:
    """Mixed persistent batch of 2x2 and 3x3 groups (one kernel launch).
    groups: list of (kind, planes, out) with planes a (3|6, n) tensor and out a
    dict of preallocated outputs (lam, D, phi, flags; any may be missing)."""

    def __init__(self, groups, opts=None):
        ref = _first_plane(groups[0][1])
        dt = _dt(ref)
        self.dtype = dt
        self.device = ref.device
        self._keep = [(planes, out) for _, planes, out in groups]
        arr = _group_array(groups)
        o = _opts(dt, opts, _kind="mixed")
        self.opts = o
        h = ctypes.c_void_p()
        wsb = ctypes.c_size_t()
        _check(_lib.ksym_plan_create(dt, len(groups), arr, ctypes.byref(o), ctypes.byref(h),
                                     ctypes.byref(wsb)))
        self._h = h
        self.ws = torch.zeros(max(1, wsb.value // 4), dtype=torch.int32, device=self.device)

    def info(self):
        t = ctypes.c_int64()
        g = ctypes.c_int32()
        _check(_lib.ksym_plan_info(self._h, ctypes.byref(t), ctypes.byref(g)))
        return {"tiles": t.value, "grid": g.value}

    def _ws_bytes(self):
        return self.ws.numel() * self.ws.element_size()

    def _st(self, stream):
        if stream is None:
            return ctypes.c_void_p(torch.cuda.current_stream(self.device).cuda_stream)
        return ctypes.c_void_p(stream.cuda_stream)

    def run(self, stream=None):
        _check(_lib.ksym_plan_run(self._h, self.ws.data_ptr(), self._ws_bytes(), self._st(stream)))

    def capture(self, stream):
        _check(_lib.ksym_plan_capture(self._h, self.ws.data_ptr(), self._ws_bytes(), self._st(stream)))

    def replay(self, stream=None):
        _check(_lib.ksym_plan_replay(self._h, self._st(stream)))

    def close(self):
        if getattr(self, "_h", None):
            _lib.ksym_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def mixed_run_noalloc(groups, opts=None, ws=None, stream=None):
    """The mixed batch of Plan(groups, opts).run(), in one call that allocates
    no device memory (the library's fixed tables; see include/ksym.h for the
    limits).  groups as for Plan; ws: None or a workspace() tensor, whose
    counters are zeroed and accumulated.  Calls that overlap on one GPU race."""
    ref = _first_plane(groups[0][1])
    dt = _dt(ref)
    arr = _group_array(groups)
    o = _opts(dt, opts, _kind="mixed")
    st = _stream(ref) if stream is None else ctypes.c_void_p(stream.cuda_stream)
    wp, wb = (ws.data_ptr(), ws.numel() * ws.element_size()) if ws is not None else (None, 0)
    _check(_lib.ksym_mixed_run_noalloc(dt, len(groups), arr, ctypes.byref(o), wp, wb, st))
