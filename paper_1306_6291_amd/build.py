"""Build the ksym HIP library (libksym.so) for gfx950 with hipcc.

Usage: python paper_1306_6291_amd/build.py  (or call build_library()).  Run it by
path: importing the package itself needs the built library.
"""

from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "csrc", "ksym_api.hip")
LIB = os.path.join(HERE, "libksym.so")
ARCH = os.environ.get("KSYM_ARCH", "gfx950")

HIPCC_FLAGS = [
    f"--offload-arch={ARCH}",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
    # no packed float32 instructions anywhere in the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found (set HIPCC or install ROCm)")


def sources():
    d = os.path.join(HERE, "csrc")
    return [os.path.join(d, f) for f in sorted(os.listdir(d))] + [
        os.path.join(os.path.dirname(HERE), "include", "ksym.h")]


# The checking build of the host code (argument checks, plans, dispatch):
# AddressSanitizer and UndefinedBehaviorSanitizer on the host side only (each
# -fsanitize= directly after -Xarch_host; the device code is built as usual).
# Loaded by the ABI tests when KSYM_ABI_LIB names it, with clang's ASan runtime
# preloaded.
LIB_SAN = os.path.join(HERE, "libksym_san.so")
SAN_FLAGS = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer"]


def build_library(verbose: bool = False, sanitize: bool = False) -> str:
    """Compile csrc/ksym_api.hip into libksym.so (always recompiles);
    sanitize: the host-checking build libksym_san.so instead."""
    lib = LIB_SAN if sanitize else LIB
    tmp = lib + ".tmp"
    cmd = [hipcc(), *HIPCC_FLAGS, *(SAN_FLAGS if sanitize else []), "-o", tmp, SRC]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    noise = "is not a recognized feature for this target"
    msg = "\n".join(l for l in (r.stdout + r.stderr).splitlines() if noise not in l)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed ({r.returncode}):\n{msg}")
    if msg.strip() and verbose:
        print(msg)
    os.replace(tmp, lib)
    return lib


def is_stale() -> bool:
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    return any(os.path.getmtime(s) > t for s in sources())


if __name__ == "__main__":
    print(build_library(verbose=True))
    sys.exit(0)
