"""The host-side code under AddressSanitizer and UndefinedBehaviorSanitizer,
every report fatal: the oracle (gcc build) under its pins, and the library's
host code -- argument checks, aliasing sweep, plans, dispatch (hipcc, with the
sanitizers on the host side only) -- under the ABI tests.  Each runs in a
child process with the sanitizer runtime preloaded (the interpreter itself is
not instrumented)."""

import glob
import importlib.util
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _child(env_extra, args):
    env = dict(os.environ)
    env.update({"ASAN_OPTIONS": "detect_leaks=0", "UBSAN_OPTIONS": "print_stacktrace=1"})
    env.update(env_extra)
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", *args],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    assert r.returncode == 0, (r.stdout[-4000:], r.stderr[-4000:])
    assert " passed" in r.stdout, r.stdout[-2000:]


def _gcc_runtime(name):
    p = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True).stdout.strip()
    return p if os.path.isabs(p) and os.path.exists(p) else None


def test_oracle_under_sanitizers():
    import oracle
    libs = [_gcc_runtime("libasan.so"), _gcc_runtime("libubsan.so")]
    if None in libs:
        pytest.skip("gcc's sanitizer runtimes are not installed")
    oracle.build(sanitize=True)
    _child({"LD_PRELOAD": ":".join(libs), "KSYM_ORACLE_SANITIZE": "1"},
           ["tests/test_oracle.py", "tests/test_selection_rule.py"])


def test_host_code_under_sanitizers():
    rt = sorted(glob.glob("/opt/rocm/lib/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    if not rt:
        pytest.skip("clang's AddressSanitizer runtime is not installed")
    spec = importlib.util.spec_from_file_location("_ksym_build", os.path.join(ROOT, "paper_1306_6291_amd",
                                                                             "build.py"))
    b = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(b)
    lib = b.LIB_SAN
    if not os.path.exists(lib) or any(os.path.getmtime(s) > os.path.getmtime(lib) for s in b.sources()):
        b.build_library(sanitize=True)
    _child({"LD_PRELOAD": rt[-1], "KSYM_ABI_LIB": lib}, ["tests/test_abi.py"])
