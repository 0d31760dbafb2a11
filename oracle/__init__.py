"""CPU oracle for batched 2x2 / 3x3 real symmetric eigendecomposition.

TEST INFRASTRUCTURE ONLY.  A plain, slow, float64 C implementation of the
paper's closed forms (Kronenburg, arXiv:1306.6291, §3-§5) plus an independent
long-double cyclic Jacobi solver and the first-order adjoint.  Only the tests,
``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py`` may import
this package; the GPU library never does and shares no code with it.

Arrays are numpy float64 structure-of-arrays planes: 3x3 input (6, n) in the
order (A11, A22, A33, A12, A13, A23); 2x2 input (3, n) as (A11, A22, A12).
"""

from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ksym_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
CFLAGS = ["-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared", "-Wall"]
# the checking build (AddressSanitizer and UndefinedBehaviorSanitizer, every
# report fatal), loaded instead of the plain one when KSYM_ORACLE_SANITIZE=1;
# the process then needs gcc's libasan and libubsan preloaded
_LIB_SAN = os.path.join(_HERE, "liboracle_san.so")
SAN_FLAGS = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g"]

GENERAL, DOUBLE, TRIPLE = 0, 1, 2
TAU_DBL = 1e-6          # relative split below which the double-root case is taken

_lib = None


def build(force=True, sanitize=False):
    """Compile the oracle with gcc into oracle/liboracle.so (sanitize: the
    checking build oracle/liboracle_san.so)."""
    lib = _LIB_SAN if sanitize else _LIB
    cmd = ["gcc", *CFLAGS, *(SAN_FLAGS if sanitize else []), "-o", lib + ".tmp", _SRC, "-lm", "-lpthread"]
    subprocess.run(cmd, check=True)
    os.replace(lib + ".tmp", lib)


def _load():
    global _lib
    if _lib is None:
        san = os.environ.get("KSYM_ORACLE_SANITIZE") == "1"
        lib = _LIB_SAN if san else _LIB
        if not os.path.exists(lib) or os.path.getmtime(lib) < os.path.getmtime(_SRC):
            build(sanitize=san)
        _lib = ctypes.CDLL(lib)
        P = ctypes.c_void_p
        i64, dbl, cint = ctypes.c_int64, ctypes.c_double, ctypes.c_int
        _lib.ko_eig3_batch.argtypes = [i64, P, P, P, P, P, dbl, cint]
        _lib.ko_eig2_batch.argtypes = [i64, P, P, P, P, cint]
        _lib.ko_jacobi3_batch.argtypes = [i64, P, P, P, P, cint]
        _lib.ko_eig3_bwd_batch.argtypes = [i64, P, P, P, P, P, P, P, dbl, dbl, cint]
        _lib.ko_eig2_bwd_batch.argtypes = [i64, P, P, P, P, P, P, dbl, cint]
        _lib.ko_compose3_batch.argtypes = [i64, P, P, P, cint]
        _lib.ko_compose2_batch.argtypes = [i64, P, P, P, cint]
        _lib.ko_eig3_dbg.argtypes = [P, dbl, P, P, P, P]
        _lib.ko_eig3_dbg.restype = cint
    return _lib


def default_threads():
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        n = os.cpu_count() or 1
    return max(1, min(n, 16))


def _ptrs(arrs):
    """Array of plane pointers for a list of contiguous float64 1-D arrays."""
    a = (ctypes.c_void_p * len(arrs))(*[x.ctypes.data for x in arrs])
    return a


def _planes(x, k):
    x = np.ascontiguousarray(np.asarray(x, dtype=np.float64))
    assert x.ndim == 2 and x.shape[0] == k, x.shape
    return [np.ascontiguousarray(x[i]) for i in range(k)]


def eig3(planes, tau_dbl=TAU_DBL, threads=None):
    """Paper §4-§5 on each matrix.  Returns dict lam (3,n), D (9,n), phi (3,n),
    branch (n,) int8 (0 general, 1 double, 2 triple)."""
    lib = _load()
    ins = _planes(planes, 6)
    n = ins[0].size
    lam = np.empty((3, n)); D = np.empty((9, n)); phi = np.empty((3, n))
    br = np.empty(n, dtype=np.int8)
    keep = (ins, lam, D, phi)
    lib.ko_eig3_batch(n, ctypes.cast(_ptrs(ins), ctypes.c_void_p),
                      ctypes.cast(_ptrs(list(lam)), ctypes.c_void_p),
                      ctypes.cast(_ptrs(list(D)), ctypes.c_void_p),
                      ctypes.cast(_ptrs(list(phi)), ctypes.c_void_p),
                      br.ctypes.data, tau_dbl, threads or default_threads())
    del keep
    return {"lam": lam, "D": D, "phi": phi, "branch": br}


def eig2(planes, threads=None):
    """Paper §3 on each matrix.  Returns dict lam (2,n), D (4,n), phi (n,)."""
    lib = _load()
    ins = _planes(planes, 3)
    n = ins[0].size
    lam = np.empty((2, n)); D = np.empty((4, n)); phi = np.empty(n)
    lib.ko_eig2_batch(n, ctypes.cast(_ptrs(ins), ctypes.c_void_p),
                      ctypes.cast(_ptrs(list(lam)), ctypes.c_void_p),
                      ctypes.cast(_ptrs(list(D)), ctypes.c_void_p),
                      phi.ctypes.data, threads or default_threads())
    return {"lam": lam, "D": D, "phi": phi}


def jacobi3(planes, threads=None):
    """Long-double cyclic Jacobi: lam (3,n) descending (rounded to float64),
    V (9,n) row-major with columns the eigenvectors, det V = +1, and lam_lo, the
    long-double remainder lam_ld - float64(lam_ld)."""
    lib = _load()
    ins = _planes(planes, 6)
    n = ins[0].size
    lam = np.empty((3, n)); V = np.empty((9, n)); lo = np.empty((3, n))
    lib.ko_jacobi3_batch(n, ctypes.cast(_ptrs(ins), ctypes.c_void_p),
                         ctypes.cast(_ptrs(list(lam)), ctypes.c_void_p),
                         ctypes.cast(_ptrs(list(V)), ctypes.c_void_p),
                         ctypes.cast(_ptrs(list(lo)), ctypes.c_void_p),
                         threads or default_threads())
    return {"lam": lam, "V": V, "lam_lo": lo}


def eig3_bwd(lam, D, glam=None, gD=None, eps=0.0, threads=None, phi=None, gphi=None, delta=0.0):
    """Adjoint: plane gradients gA (6, n) from the forward outputs and the
    cotangents (None = zero).  eps is the absolute gap regulariser; with phi
    and gphi (the angles and their cotangents) the angle term is included,
    delta regularising 1/cos(phi2)."""
    lib = _load()
    L = _planes(lam, 3); Dp = _planes(D, 9)
    n = L[0].size
    gl = _planes(glam, 3) if glam is not None else None
    gd = _planes(gD, 9) if gD is not None else None
    ang = phi is not None and gphi is not None
    ph = _planes(phi, 3) if ang else None
    gp = _planes(gphi, 3) if ang else None
    gA = np.empty((6, n))
    lib.ko_eig3_bwd_batch(
        n, ctypes.cast(_ptrs(L), ctypes.c_void_p), ctypes.cast(_ptrs(Dp), ctypes.c_void_p),
        ctypes.cast(_ptrs(gl), ctypes.c_void_p) if gl else None,
        ctypes.cast(_ptrs(gd), ctypes.c_void_p) if gd else None,
        ctypes.cast(_ptrs(ph), ctypes.c_void_p) if ph else None,
        ctypes.cast(_ptrs(gp), ctypes.c_void_p) if gp else None,
        ctypes.cast(_ptrs(list(gA)), ctypes.c_void_p), float(eps), float(delta), threads or default_threads())
    return gA


def eig2_bwd(lam, D, glam=None, gD=None, gphi=None, eps=0.0, threads=None):
    """2x2 adjoint: plane gradients gA (3, n) = (A11, A22, A12) from the
    forward outputs and the cotangents of lam, D and phi (None = zero)."""
    lib = _load()
    L = _planes(lam, 2); Dp = _planes(D, 4)
    n = L[0].size
    gl = _planes(glam, 2) if glam is not None else None
    gd = _planes(gD, 4) if gD is not None else None
    gp = np.ascontiguousarray(np.asarray(gphi, dtype=np.float64).reshape(-1)) if gphi is not None else None
    gA = np.empty((3, n))
    lib.ko_eig2_bwd_batch(
        n, ctypes.cast(_ptrs(L), ctypes.c_void_p), ctypes.cast(_ptrs(Dp), ctypes.c_void_p),
        ctypes.cast(_ptrs(gl), ctypes.c_void_p) if gl else None,
        ctypes.cast(_ptrs(gd), ctypes.c_void_p) if gd else None,
        gp.ctypes.data if gp is not None else None,
        ctypes.cast(_ptrs(list(gA)), ctypes.c_void_p), float(eps), threads or default_threads())
    return gA


def compose3(lam, phi, threads=None):
    """Inverse map, eq. (2.6): planes A (6, n) = D diag(lam) D^T with
    D = R1(phi1) R2(phi2) R3(phi3), from lam (3, n) and phi (3, n)."""
    lib = _load()
    L = _planes(lam, 3); F = _planes(phi, 3)
    n = L[0].size
    A = np.empty((6, n))
    lib.ko_compose3_batch(n, ctypes.cast(_ptrs(L), ctypes.c_void_p), ctypes.cast(_ptrs(F), ctypes.c_void_p),
                          ctypes.cast(_ptrs(list(A)), ctypes.c_void_p), threads or default_threads())
    return A


def compose2(lam, phi, threads=None):
    """Inverse map, eq. (2.5): planes A (3, n) = (A11, A22, A12) of
    R(phi) diag(lam) R(phi)^T, from lam (2, n) and phi (n,)."""
    lib = _load()
    L = _planes(lam, 2)
    n = L[0].size
    f = np.ascontiguousarray(np.asarray(phi, dtype=np.float64).reshape(-1))
    A = np.empty((3, n))
    lib.ko_compose2_batch(n, ctypes.cast(_ptrs(L), ctypes.c_void_p), f.ctypes.data,
                          ctypes.cast(_ptrs(list(A)), ctypes.c_void_p), threads or default_threads())
    return A


class Debug3(ctypes.Structure):
    _fields_ = [("b", ctypes.c_double), ("p", ctypes.c_double), ("q", ctypes.c_double),
                ("Delta", ctypes.c_double), ("v", ctypes.c_double), ("w", ctypes.c_double),
                ("delta", ctypes.c_double * 4), ("f1n", ctypes.c_double),
                ("f2n", ctypes.c_double), ("g1n", ctypes.c_double), ("g2n", ctypes.c_double),
                ("chosen", ctypes.c_int), ("branch", ctypes.c_int)]


def eig3_debug(A6, tau_dbl=TAU_DBL):
    """One matrix with the intermediate quantities of §4-§5 (b, p, q, Delta, v,
    w, the four selection distances, |f1|, |f2|, |g1|, |g2|, chosen, branch)."""
    lib = _load()
    A = np.ascontiguousarray(np.asarray(A6, dtype=np.float64))
    lam = np.empty(3); D = np.empty(9); phi = np.empty(3)
    dbg = Debug3()
    lib.ko_eig3_dbg(A.ctypes.data, tau_dbl, lam.ctypes.data, D.ctypes.data,
                    phi.ctypes.data, ctypes.addressof(dbg))
    out = {k: getattr(dbg, k) for k, _ in Debug3._fields_}
    out["delta"] = list(dbg.delta)
    out.update(lam=lam, D=D.reshape(3, 3), phi=phi)
    return out
